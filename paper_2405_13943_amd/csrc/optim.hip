// Streaming kernels of the ADMM layer:
//   - Adam with the scaled ADMM penalty (Eq. 8a; per-attribute rho of the
//     supplementary Sec. C): g' = g + rho_a (x - w), w = z - u;
//   - the consensus step (Eq. 8b-c, Alg. 2): z = mean of the holders' local
//     copies, u += x - z, w = z - u, with optional over-relaxation (Sec. 3.3).
// Both are pure HBM streams over the SoA planes: 16-byte vector accesses,
// one pass, no re-reads.
#include "adam.hpp"
#include "gs_device.hpp"
#include "gs_internal.hpp"

#include <cmath>

namespace gs {

// grid: y = plane, x covers the plane in 4-wide vectors (tail handled by the last vector)
template <bool PEN, bool MASK, bool VEC>
__global__ __launch_bounds__(256) void k_adam_admm(float* __restrict__ x, const float* __restrict__ g,
                                                    float* __restrict__ m, float* __restrict__ v,
                                                    const float* __restrict__ w, const float* __restrict__ mask,
                                                    int64_t n, int64_t sx, int64_t sg, int64_t sm, int64_t sv,
                                                    int64_t sw, AdamConsts c) {
    const int a = blockIdx.y;
    const int grp = plane_group(a);
    const float lr = c.lr[grp], rho = c.rho[grp];
    const int64_t i4 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
    if (i4 >= n) return;
    float* X = x + a * sx;
    const float* G = g + a * sg;
    float* M = m + a * sm;
    float* Vv = v + a * sv;
    const float* Wp = PEN ? w + a * sw : nullptr;
    if (VEC && i4 + 4 <= n) {
        float4 xv = *reinterpret_cast<const float4*>(X + i4);
        const float4 gv = *reinterpret_cast<const float4*>(G + i4);
        float4 mv = *reinterpret_cast<const float4*>(M + i4);
        float4 vv = *reinterpret_cast<const float4*>(Vv + i4);
        float4 wv = make_float4(0.f, 0.f, 0.f, 0.f), kv = make_float4(1.f, 1.f, 1.f, 1.f);
        if (PEN) wv = *reinterpret_cast<const float4*>(Wp + i4);
        if (MASK) kv = *reinterpret_cast<const float4*>(mask + i4);
        adam_one(xv.x, gv.x, mv.x, vv.x, wv.x, PEN ? rho * kv.x : 0.f, lr, c);
        adam_one(xv.y, gv.y, mv.y, vv.y, wv.y, PEN ? rho * kv.y : 0.f, lr, c);
        adam_one(xv.z, gv.z, mv.z, vv.z, wv.z, PEN ? rho * kv.z : 0.f, lr, c);
        adam_one(xv.w, gv.w, mv.w, vv.w, wv.w, PEN ? rho * kv.w : 0.f, lr, c);
        *reinterpret_cast<float4*>(X + i4) = xv;
        *reinterpret_cast<float4*>(M + i4) = mv;
        *reinterpret_cast<float4*>(Vv + i4) = vv;
    } else {
        for (int64_t i = i4; i < n && i < i4 + 4; i++) {
            float xs = X[i], ms = M[i], vs = Vv[i];
            const float ws = PEN ? Wp[i] : 0.f;
            const float r = PEN ? rho * (MASK ? mask[i] : 1.f) : 0.f;
            adam_one(xs, G[i], ms, vs, ws, r, lr, c);
            X[i] = xs; M[i] = ms; Vv[i] = vs;
        }
    }
}

template <bool PEN, bool MASK>
static void adam_launch(bool vec, dim3 grid, hipStream_t s, float* x, const float* g, float* m, float* v,
                        const float* w, const float* mask, int64_t n, int64_t sx, int64_t sg, int64_t sm, int64_t sv,
                        int64_t sw, const AdamConsts& c) {
    if (vec)
        GS_LAUNCH("k_adam_admm", (k_adam_admm<PEN, MASK, true>), grid, dim3(256), 0, s, x, g, m, v, w, mask, n, sx, sg, sm, sv, sw, c);
    else
        GS_LAUNCH("k_adam_admm", (k_adam_admm<PEN, MASK, false>), grid, dim3(256), 0, s, x, g, m, v, w, mask, n, sx, sg, sm, sv, sw, c);
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

hipError_t launch_adam_admm(gs_params& x, const gs_params& g, gs_params& m, gs_params& v, const gs_params* w,
                            const float* mask, const gs_adam_cfg& cfg, hipStream_t s) {
    const int64_t n = x.n;
    if (n == 0) return hipSuccess;
    const int A = 11 + 3 * (x.sh_degree + 1) * (x.sh_degree + 1);
    const AdamConsts c = adam_consts(cfg);
    bool vec = aligned16(x.data) && aligned16(g.data) && aligned16(m.data) && aligned16(v.data) &&
               x.stride % 4 == 0 && g.stride % 4 == 0 && m.stride % 4 == 0 && v.stride % 4 == 0;
    if (w) vec = vec && aligned16(w->data) && w->stride % 4 == 0;
    if (mask) vec = vec && aligned16(mask);
    dim3 grid(unsigned((n + 1023) / 1024), unsigned(A));
    float* X = static_cast<float*>(x.data);
    const float* G = static_cast<const float*>(g.data);
    float* M = static_cast<float*>(m.data);
    float* V = static_cast<float*>(v.data);
    const float* Wd = w ? static_cast<const float*>(w->data) : nullptr;
    const int64_t sw = w ? w->stride : 0;
    if (w && mask) adam_launch<true, true>(vec, grid, s, X, G, M, V, Wd, mask, n, x.stride, g.stride, m.stride, v.stride, sw, c);
    else if (w) adam_launch<true, false>(vec, grid, s, X, G, M, V, Wd, mask, n, x.stride, g.stride, m.stride, v.stride, sw, c);
    else adam_launch<false, false>(vec, grid, s, X, G, M, V, Wd, mask, n, x.stride, g.stride, m.stride, v.stride, sw, c);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// consensus: one thread per global id, all planes

__global__ __launch_bounds__(256) void k_consensus(const float* __restrict__ x, float* __restrict__ u,
                                                   float* __restrict__ w, float* __restrict__ z,
                                                   const int64_t* __restrict__ hptr, const int64_t* __restrict__ hidx,
                                                   int64_t n_global, int A, int64_t sx, int64_t su, int64_t sw,
                                                   int64_t sz, float relax, float* __restrict__ resid) {
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    float rp[5] = {0, 0, 0, 0, 0}, rd[5] = {0, 0, 0, 0, 0};
    if (gid < n_global) {
        const int64_t h0 = hptr[gid], h1 = hptr[gid + 1];
        if (h1 > h0) {
            const float cnt = float(h1 - h0);
            for (int a = 0; a < A; a++) {
                const float zp = z[a * sz + gid];
                float acc = 0.f;
                for (int64_t h = h0; h < h1; h++) {
                    const float xv = x[a * sx + hidx[h]];
                    acc += relax == 1.0f ? xv : relax * xv + (1.0f - relax) * zp;
                }
                const float zn = acc / cnt;
                z[a * sz + gid] = zn;
                const int grp = plane_group(a);
                for (int64_t h = h0; h < h1; h++) {
                    const int64_t l = hidx[h];
                    const float xv = x[a * sx + l];
                    const float xh = relax == 1.0f ? xv : relax * xv + (1.0f - relax) * zp;
                    const float un = u[a * su + l] + xh - zn;
                    u[a * su + l] = un;
                    w[a * sw + l] = zn - un;
                    rp[grp] += (xv - zn) * (xv - zn);
                }
                rd[grp] += (zn - zp) * (zn - zp);
            }
        }
    }
    if (resid) {
#pragma unroll
        for (int k = 0; k < 5; k++) {
            const float a = wave_sum(rp[k]), b = wave_sum(rd[k]);
            if (lane_id() == 0) {
                atomicAdd(resid + k, a);
                atomicAdd(resid + 5 + k, b);
            }
        }
    }
}

hipError_t launch_consensus(const gs_params& x, gs_params& u, gs_params& w, gs_params& z, const int64_t* hptr,
                            const int64_t* hidx, float relax, float* resid, hipStream_t s) {
    const int64_t G = z.n;
    if (G == 0) return hipSuccess;
    const int A = 11 + 3 * (x.sh_degree + 1) * (x.sh_degree + 1);
    GS_LAUNCH("k_consensus", k_consensus, dim3(unsigned((G + 255) / 256)), dim3(256), 0, s, static_cast<const float*>(x.data),
                       static_cast<float*>(u.data), static_cast<float*>(w.data), static_cast<float*>(z.data), hptr, hidx,
                       G, A, x.stride, u.stride, w.stride, z.stride, relax, resid);
    return hipGetLastError();
}

}  // namespace gs
