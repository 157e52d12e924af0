// Streaming kernels of the ADMM layer:
//   - Adam with the scaled ADMM penalty (Eq. 8a; per-attribute rho of the
//     supplementary Sec. C): g' = g + rho_a (x - w), w = z - u;
//   - the consensus step (Eq. 8b-c, Alg. 2): z = mean of the holders' local
//     copies, u += x - z, w = z - u, with optional over-relaxation and the
//     primal/dual residual sums of Sec. 3.3;
//   - the rescale of the scaled duals when the penalty changes (Sec. 3.3).
// All are pure HBM streams over the SoA planes, one pass, no re-reads.
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
                                                    int64_t sw, AdamConsts c, uint32_t* __restrict__ status) {
    if (adam_skipped(status)) return;
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
        // g, m, v and w are touched once per step: streamed past the caches
        const float4 gv = load_stream4(G + i4);
        float4 mv = load_stream4(M + i4);
        float4 vv = load_stream4(Vv + i4);
        float4 wv = make_float4(0.f, 0.f, 0.f, 0.f), kv = make_float4(1.f, 1.f, 1.f, 1.f);
        if (PEN) wv = load_stream4(Wp + i4);
        if (MASK) kv = *reinterpret_cast<const float4*>(mask + i4);
        adam_one(xv.x, gv.x, mv.x, vv.x, wv.x, PEN ? rho * kv.x : 0.f, lr, c);
        adam_one(xv.y, gv.y, mv.y, vv.y, wv.y, PEN ? rho * kv.y : 0.f, lr, c);
        adam_one(xv.z, gv.z, mv.z, vv.z, wv.z, PEN ? rho * kv.z : 0.f, lr, c);
        adam_one(xv.w, gv.w, mv.w, vv.w, wv.w, PEN ? rho * kv.w : 0.f, lr, c);
        *reinterpret_cast<float4*>(X + i4) = xv;
        store_stream4(M + i4, mv);
        store_stream4(Vv + i4, vv);
        float fin = 0.f;
        adam_finite(fin, xv.x, vv.x);
        adam_finite(fin, xv.y, vv.y);
        adam_finite(fin, xv.z, vv.z);
        adam_finite(fin, xv.w, vv.w);
        adam_flag(status, fin);
    } else {
        float fin = 0.f;
        for (int64_t i = i4; i < n && i < i4 + 4; i++) {
            float xs = X[i], ms = M[i], vs = Vv[i];
            const float ws = PEN ? Wp[i] : 0.f;
            const float r = PEN ? rho * (MASK ? mask[i] : 1.f) : 0.f;
            adam_one(xs, G[i], ms, vs, ws, r, lr, c);
            X[i] = xs; M[i] = ms; Vv[i] = vs;
            adam_finite(fin, xs, vs);
        }
        adam_flag(status, fin);
    }
}

template <bool PEN, bool MASK>
static void adam_launch(bool vec, dim3 grid, hipStream_t s, float* x, const float* g, float* m, float* v,
                        const float* w, const float* mask, int64_t n, int64_t sx, int64_t sg, int64_t sm, int64_t sv,
                        int64_t sw, const AdamConsts& c, uint32_t* status) {
    if (vec)
        GS_LAUNCH("k_adam_admm", (k_adam_admm<PEN, MASK, true>), grid, dim3(256), 0, s, x, g, m, v, w, mask, n, sx, sg,
                  sm, sv, sw, c, status);
    else
        GS_LAUNCH("k_adam_admm", (k_adam_admm<PEN, MASK, false>), grid, dim3(256), 0, s, x, g, m, v, w, mask, n, sx, sg,
                  sm, sv, sw, c, status);
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

hipError_t launch_adam_admm(gs_params& x, const gs_params& g, gs_params& m, gs_params& v, const gs_params* w,
                            const float* mask, const gs_adam_cfg& cfg, uint32_t* status, hipStream_t s) {
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
    if (w && mask)
        adam_launch<true, true>(vec, grid, s, X, G, M, V, Wd, mask, n, x.stride, g.stride, m.stride, v.stride, sw, c,
                                status);
    else if (w)
        adam_launch<true, false>(vec, grid, s, X, G, M, V, Wd, mask, n, x.stride, g.stride, m.stride, v.stride, sw, c,
                                 status);
    else
        adam_launch<false, false>(vec, grid, s, X, G, M, V, Wd, mask, n, x.stride, g.stride, m.stride, v.stride, sw, c,
                                  status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// consensus.  The stream is latency bound unless many loads are in flight, so
// a workgroup takes 64 consecutive global ids at a time (grid-stride) and
// each of its wavefronts one chunk of 8 planes of them: a lane holds one
// global id, issues every load of its chunk before using any, then stores.
// The kernel is specialised on the SH degree, so the plane count and every
// plane's attribute group are compile-time constants.  Global ids with one or
// two holders (every id of a slab partition) share one branch-free path: a
// missing second holder reads the first holder's column again and its stores
// are predicated off, so a wavefront mixing the two does not diverge.  Three
// or four holders take two half chunks; more take a plain loop.

constexpr int kChunk = 8;                 // planes per wavefront

__host__ __device__ constexpr int sh_planes(int deg) { return 11 + 3 * (deg + 1) * (deg + 1); }

// element at byte offset off (32-bit, per lane) from a plane base (uniform)
__device__ __forceinline__ float& at(float* base, uint32_t off) {
    return *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + off);
}
__device__ __forceinline__ float at(const float* base, uint32_t off) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + off);
}
// store with the non-temporal hint: z, u and w are written once per round and
// not read again by it, so they need not take cache lines from the loads
__device__ __forceinline__ void store_stream(float* base, uint32_t off, float v) {
    __builtin_nontemporal_store(v, reinterpret_cast<float*>(reinterpret_cast<char*>(base) + off));
}

// Planes [A0, A0 + NP) (clipped to A) of one global id (byte offset og in the
// z planes) whose nh <= NH holders sit at byte offsets ol[0..NH) in the local
// planes (offsets past nh repeat ol[0]).  A single holder gets z = xh
// exactly, so its u cannot change and is not stored.
template <int A, int A0, int NP, int NH, bool RELAX, bool ZP>
__device__ __forceinline__ void consensus_chunk(const float* __restrict__ x, float* __restrict__ u,
                                                float* __restrict__ w, float* __restrict__ z, int64_t sx, int64_t su,
                                                int64_t sw, int64_t sz, uint32_t og, const uint32_t (&ol)[NH], int nh,
                                                float relax, float (&rp)[5], float (&rd)[5]) {
    constexpr int N = (A - A0) < NP ? (A - A0) : NP;
    float xv[N][NH], uv[N][NH], zp[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int a = A0 + i;
        zp[i] = ZP ? at(z + a * sz, og) : 0.f;
#pragma unroll
        for (int j = 0; j < NH; j++) {
            xv[i][j] = at(x + a * sx, ol[j]);
            uv[i][j] = at(u + a * su, ol[j]);
        }
    }
    const float cnt = float(nh);
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int a = A0 + i;
        const int grp = plane_group(a);
        float xh[NH];
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < NH; j++) {
            xh[j] = RELAX ? relax * xv[i][j] + (1.0f - relax) * zp[i] : xv[i][j];
            if (j == 0 || j < nh) acc += xh[j];
        }
        const float zn = acc / cnt;
        store_stream(z + a * sz, og, zn);
#pragma unroll
        for (int j = 0; j < NH; j++) {
            if (j == 0 || j < nh) {
                const float un = uv[i][j] + xh[j] - zn;
                if (nh > 1) store_stream(u + a * su, ol[j], un);
                store_stream(w + a * sw, ol[j], zn - un);
                rp[grp] += (xv[i][j] - zn) * (xv[i][j] - zn);
            }
        }
        if (ZP) rd[grp] += cnt * (zn - zp[i]) * (zn - zp[i]);
    }
}

// planes [A0, A1) for any number of holders (holder indices re-read per plane)
template <int A0, int A1, bool RELAX, bool ZP>
__device__ __forceinline__ void consensus_any(const float* __restrict__ x, float* __restrict__ u,
                                              float* __restrict__ w, float* __restrict__ z, int64_t sx, int64_t su,
                                              int64_t sw, int64_t sz, int64_t gid, const int64_t* __restrict__ hidx,
                                              int64_t h0, int64_t h1, float relax, float (&rp)[5], float (&rd)[5]) {
    const float cnt = float(h1 - h0);
#pragma unroll 1
    for (int a = A0; a < A1; a++) {
        const int grp = plane_group(a);
        float sp = 0.f;
        const float zp = ZP ? z[a * sz + gid] : 0.f;
        float acc = 0.f;
        for (int64_t h = h0; h < h1; h++) {
            const float xv = x[a * sx + hidx[h]];
            acc += RELAX ? relax * xv + (1.0f - relax) * zp : xv;
        }
        const float zn = acc / cnt;
        z[a * sz + gid] = zn;
        for (int64_t h = h0; h < h1; h++) {
            const int64_t c = hidx[h];
            const float xv = x[a * sx + c];
            const float xh = RELAX ? relax * xv + (1.0f - relax) * zp : xv;
            const float un = u[a * su + c] + xh - zn;
            u[a * su + c] = un;
            w[a * sw + c] = zn - un;
            sp += (xv - zn) * (xv - zn);
        }
        const float sd = ZP ? cnt * (zn - zp) * (zn - zp) : 0.f;
#pragma unroll
        for (int k = 0; k < 5; k++) {       // constant indices keep rp, rd in registers
            rp[k] += grp == k ? sp : 0.f;
            rd[k] += grp == k ? sd : 0.f;
        }
    }
}

// the chunk of planes [A0, A0 + kChunk) of one global id, by holder count
template <int A, int A0, bool RELAX, bool ZP>
__device__ __forceinline__ void consensus_planes(const float* __restrict__ x, float* __restrict__ u,
                                                 float* __restrict__ w, float* __restrict__ z,
                                                 const int64_t* __restrict__ hidx, int64_t sx, int64_t su, int64_t sw,
                                                 int64_t sz, int64_t gid, int64_t h0, int64_t nh, float relax,
                                                 float (&rp)[5], float (&rd)[5]) {
    if constexpr (A0 < A) {
        // byte offsets fit 32 bits: the host caps local and global columns at 2^30
        const uint32_t og = uint32_t(gid) * 4u;
        if (nh <= 2) {
            const uint32_t c0 = uint32_t(hidx[h0]) * 4u;
            const uint32_t ol[2] = {c0, nh > 1 ? uint32_t(hidx[h0 + 1]) * 4u : c0};
            consensus_chunk<A, A0, kChunk, 2, RELAX, ZP>(x, u, w, z, sx, su, sw, sz, og, ol, int(nh), relax, rp, rd);
        } else if (nh <= 4) {
            const uint32_t c0 = uint32_t(hidx[h0]) * 4u;
            const uint32_t ol[4] = {c0, uint32_t(hidx[h0 + 1]) * 4u, uint32_t(hidx[h0 + 2]) * 4u,
                                    nh > 3 ? uint32_t(hidx[h0 + 3]) * 4u : c0};
            consensus_chunk<A, A0, kChunk / 2, 4, RELAX, ZP>(x, u, w, z, sx, su, sw, sz, og, ol, int(nh), relax, rp, rd);
            if constexpr (A0 + kChunk / 2 < A)
                consensus_chunk<A, A0 + kChunk / 2, kChunk / 2, 4, RELAX, ZP>(x, u, w, z, sx, su, sw, sz, og, ol,
                                                                               int(nh), relax, rp, rd);
        } else {
            constexpr int A1 = A0 + kChunk < A ? A0 + kChunk : A;
            consensus_any<A0, A1, RELAX, ZP>(x, u, w, z, sx, su, sw, sz, gid, hidx, h0, h0 + nh, relax, rp, rd);
        }
    }
}

// block-wide sums of the 10 residual accumulators, one atomic per value and block
template <int NW>
__device__ __forceinline__ void residual_flush(const float (&rp)[5], const float (&rd)[5], float* __restrict__ resid) {
    __shared__ float part[NW][10];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; k++) {
        const float a = wave_sum(rp[k]), b = wave_sum(rd[k]);
        if (lane_id() == 0) { part[wv][k] = a; part[wv][5 + k] = b; }
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        float t = 0.f;
        for (int i = 0; i < NW; i++) t += part[i][threadIdx.x];
        atomicAdd(resid + threadIdx.x, t);
    }
}

__host__ __device__ constexpr int consensus_waves(int deg) { return (sh_planes(deg) + kChunk - 1) / kChunk; }

template <int DEG, bool RELAX, bool RESID>
__global__ __launch_bounds__(64 * consensus_waves(DEG)) void k_consensus(
    const float* __restrict__ x, float* __restrict__ u, float* __restrict__ w, float* __restrict__ z,
    const int64_t* __restrict__ hptr, const int64_t* __restrict__ hidx, int64_t n_global, int64_t sx, int64_t su,
    int64_t sw, int64_t sz, float relax, float* __restrict__ resid) {
    constexpr int A = sh_planes(DEG);
    constexpr int NW = consensus_waves(DEG);
    constexpr bool ZP = RELAX || RESID;
    const int chunk = threadIdx.x >> 6;     // uniform per wavefront
    float rp[5] = {0, 0, 0, 0, 0}, rd[5] = {0, 0, 0, 0, 0};
    const int64_t groups = (n_global + 63) >> 6;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t gid = (g << 6) + lane_id();
        if (gid >= n_global) continue;
        const int64_t h0 = hptr[gid], nh = hptr[gid + 1] - h0;
        if (nh <= 0) continue;
#define GS_CHUNK(C)                                                                                               \
    case C:                                                                                                       \
        consensus_planes<A, C * kChunk, RELAX, ZP>(x, u, w, z, hidx, sx, su, sw, sz, gid, h0, nh, relax, rp, rd); \
        break
        switch (chunk) {
            GS_CHUNK(0); GS_CHUNK(1); GS_CHUNK(2); GS_CHUNK(3);
            GS_CHUNK(4); GS_CHUNK(5); GS_CHUNK(6); GS_CHUNK(7);
            default: break;
        }
#undef GS_CHUNK
    }
    if (RESID) residual_flush<NW>(rp, rd, resid);
}


template <int DEG>
static void consensus_launch(int64_t G, hipStream_t s, bool rel, float* resid, const float* X, float* U, float* W,
                             float* Z, const int64_t* hptr, const int64_t* hidx, int64_t sx, int64_t su, int64_t sw,
                             int64_t sz, float relax) {
    static_assert(consensus_waves(DEG) <= 8, "one wavefront per chunk of planes");
    const int64_t groups = (G + 63) / 64;
    const dim3 grid(unsigned(groups < 2048 ? groups : 2048)), block(64 * consensus_waves(DEG));
#define GS_CONSENSUS(R, Q)                                                                                     \
    GS_LAUNCH("k_consensus", (k_consensus<DEG, R, Q>), grid, block, 0, s, X, U, W, Z, hptr, hidx, G, sx, su, sw, \
              sz, relax, resid)
    if (rel && resid) GS_CONSENSUS(true, true);
    else if (rel) GS_CONSENSUS(true, false);
    else if (resid) GS_CONSENSUS(false, true);
    else GS_CONSENSUS(false, false);
#undef GS_CONSENSUS
}

hipError_t launch_consensus(const gs_params& x, gs_params& u, gs_params& w, gs_params& z, const int64_t* hptr,
                            const int64_t* hidx, float relax, float* resid, hipStream_t s) {
    const int64_t G = z.n;
    if (G == 0) return hipSuccess;
    const float* X = static_cast<const float*>(x.data);
    float* U = static_cast<float*>(u.data);
    float* W = static_cast<float*>(w.data);
    float* Z = static_cast<float*>(z.data);
    const bool rel = relax != 1.0f;
    switch (x.sh_degree) {
    case 0: consensus_launch<0>(G, s, rel, resid, X, U, W, Z, hptr, hidx, x.stride, u.stride, w.stride, z.stride, relax); break;
    case 1: consensus_launch<1>(G, s, rel, resid, X, U, W, Z, hptr, hidx, x.stride, u.stride, w.stride, z.stride, relax); break;
    case 2: consensus_launch<2>(G, s, rel, resid, X, U, W, Z, hptr, hidx, x.stride, u.stride, w.stride, z.stride, relax); break;
    default: consensus_launch<3>(G, s, rel, resid, X, U, W, Z, hptr, hidx, x.stride, u.stride, w.stride, z.stride, relax); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dual rescale after a penalty change: u_k *= scale[group], w_k = z - u_k.
// Only entries whose u actually changes are written (u = 0, the state of
// every copy without a second holder, or scale = 1 leave u and w as they are).

struct GroupScale {
    float s[5];
};

// Planes [A0, A0 + NP) (clipped to A) of the NH local copies at byte offsets
// ol (offsets past n repeat ol[0]) of one global id (byte offset og in z).
// Planes of a group at scale 1 are not read.
template <int A, int A0, int NP, int NH>
__device__ __forceinline__ void rescale_chunk(float* __restrict__ u, float* __restrict__ w,
                                              const float* __restrict__ z, int64_t su, int64_t sw, int64_t sz,
                                              uint32_t og, const uint32_t (&ol)[NH], int n, const GroupScale& sc) {
    constexpr int N = (A - A0) < NP ? (A - A0) : NP;
    float uv[N][NH];
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int a = A0 + i;
        if (sc.s[plane_group(a)] == 1.0f) continue;
#pragma unroll
        for (int j = 0; j < NH; j++) uv[i][j] = at(u + a * su, ol[j]);
    }
    // z only where some u of this lane's chunk changes, all planes in one batch
    bool chg = false;
#pragma unroll
    for (int i = 0; i < N; i++) {
        const float f = sc.s[plane_group(A0 + i)];
        if (f == 1.0f) continue;
#pragma unroll
        for (int j = 0; j < NH; j++) chg = chg || ((j == 0 || j < n) && uv[i][j] * f != uv[i][j]);
    }
    if (!chg) return;
    float zv[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int a = A0 + i;
        if (sc.s[plane_group(a)] != 1.0f) zv[i] = at(z + a * sz, og);
    }
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int a = A0 + i;
        const float f = sc.s[plane_group(a)];
        if (f == 1.0f) continue;
#pragma unroll
        for (int j = 0; j < NH; j++) {
            const float us = uv[i][j] * f;
            if ((j == 0 || j < n) && us != uv[i][j]) {
                store_stream(u + a * su, ol[j], us);
                store_stream(w + a * sw, ol[j], zv[i] - us);
            }
        }
    }
}

// one lane per global id, one wavefront per chunk of planes (as the
// consensus); the copies of a global id two at a time (each copy is rescaled
// on its own, so any holder count takes the same unrolled path)
template <int DEG>
__global__ __launch_bounds__(64 * consensus_waves(DEG)) void k_dual_rescale(
    float* __restrict__ u, float* __restrict__ w, const float* __restrict__ z, const int64_t* __restrict__ hptr,
    const int64_t* __restrict__ hidx, int64_t n_global, int64_t su, int64_t sw, int64_t sz, GroupScale sc) {
    constexpr int A = sh_planes(DEG);
    const int chunk = threadIdx.x >> 6;
    const int64_t groups = (n_global + 63) >> 6;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t gid = (g << 6) + lane_id();
        if (gid >= n_global) continue;
        const int64_t h0 = hptr[gid], h1 = hptr[gid + 1];
        const uint32_t og = uint32_t(gid) * 4u;
        for (int64_t h = h0; h < h1; h += 2) {
            const uint32_t c0 = uint32_t(hidx[h]) * 4u;
            const uint32_t ol[2] = {c0, h + 1 < h1 ? uint32_t(hidx[h + 1]) * 4u : c0};
            const int n = int(h1 - h);
#define GS_CHUNK(C)                                                                                   \
    case C:                                                                                           \
        if constexpr (C * kChunk < A) rescale_chunk<A, C * kChunk, kChunk, 2>(u, w, z, su, sw, sz, og, ol, n, sc); \
        break
            switch (chunk) {
                GS_CHUNK(0); GS_CHUNK(1); GS_CHUNK(2); GS_CHUNK(3);
                GS_CHUNK(4); GS_CHUNK(5); GS_CHUNK(6); GS_CHUNK(7);
                default: break;
            }
#undef GS_CHUNK
        }
    }
}

hipError_t launch_dual_rescale(gs_params& u, gs_params& w, const gs_params& z, const int64_t* hptr,
                               const int64_t* hidx, const float* scale, hipStream_t s) {
    const int64_t G = z.n;
    if (G == 0) return hipSuccess;
    GroupScale sc;
    bool any = false;
    for (int k = 0; k < 5; k++) { sc.s[k] = scale[k]; any = any || scale[k] != 1.0f; }
    if (!any) return hipSuccess;
    float* U = static_cast<float*>(u.data);
    float* W = static_cast<float*>(w.data);
    const float* Z = static_cast<const float*>(z.data);
    const int64_t groups = (G + 63) / 64;
    const dim3 grid(unsigned(groups < 2048 ? groups : 2048));
#define GS_RESCALE(D)                                                                                           \
    GS_LAUNCH("k_dual_rescale", k_dual_rescale<D>, grid, dim3(64 * consensus_waves(D)), 0, s, U, W, Z, hptr, hidx, G, \
              u.stride, w.stride, z.stride, sc)
    switch (u.sh_degree) {
    case 0: GS_RESCALE(0); break;
    case 1: GS_RESCALE(1); break;
    case 2: GS_RESCALE(2); break;
    default: GS_RESCALE(3); break;
    }
#undef GS_RESCALE
    return hipGetLastError();
}

}  // namespace gs
