// The photometric loss of Eq. 3 with its structural term:
//   L_j = w_j (mean |C - target| + lambda (1 - mean SSIM)),
// SSIM of Wang et al. under an 11 x 11 Gaussian window (sigma 1.5, zero
// outside the image), per colour channel, mean over pixels and channels.
//
// Each job's image is cut into 32 x 32 pixel tiles, numbered jobs first, then
// row-major (the count follows from the job's binning-tile grid).  The two
// passes run a persistent grid over those tiles: a workgroup walks (tile,
// channel) items, staging the tile plus a 5-pixel halo in LDS and blurring
// separably (rows, then columns, four outputs per thread), while the next
// item's loads are in flight.
//   k_ssim_fwd  blurs x, y, x^2, y^2, xy; forms SSIM and its derivatives with
//               respect to the window sums (mu_x, E[x^2], E[xy]); writes the
//               three derivative maps (pre-scaled by -w lambda / N) and adds
//               the tile's share of the job's loss;
//   k_ssim_bwd  blurs the three maps and combines them with x and y into
//               dL/dC (plus the L1 term), the external gradient of the
//               compositing backward.
// (A grid over every binning tile, with three of four workgroups exiting at
// once, spent 40% of its time dispatching workgroups that did nothing.)
#include "gs_device.hpp"
#include "gs_internal.hpp"

#include <cmath>

namespace gs {

namespace {

constexpr int kTile = 32;                    // output pixels per side
constexpr int kRad = 5;                      // window radius
constexpr int kTaps = 2 * kRad + 1;
constexpr int kIn = kTile + 2 * kRad;        // staged rows / columns
constexpr int kPitch = kIn + 1;              // LDS row pitch (bank spread)
constexpr int kHPitch = kTile + 1;
constexpr int kThreads = 256;
constexpr int kBlk = 4;                      // outputs per thread and pass (register blocking)
static_assert(kTile * kTile / kBlk == kThreads, "column pass: one item per thread");
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Taps {
    float g[kTaps];
};

struct SsimTile {
    int job, x0, y0, W, H;
    int64_t px;       // first element of the job's channel-0 plane
    int64_t plane;    // elements per channel plane
};

// 32 x 32 tiles of job j: ceil(width / 32) x ceil(height / 32), counted from
// the job's binning tiles (32 is a multiple of every binning tile side)
__device__ inline uint32_t job_tiles(const gs_job& job, int tw, int th, int& nax) {
    nax = (job.tiles_x * tw + kTile - 1) / kTile;
    const int nay = (job.tiles_y * th + kTile - 1) / kTile;
    return uint32_t(nax) * uint32_t(nay);
}

__device__ inline uint32_t frame_tiles(const gs_frame& f, int tw, int th) {
    uint32_t n = 0;
    for (int j = 0; j < f.n_jobs; j++) {
        int nax;
        n += job_tiles(f.jobs[j], tw, th, nax);
    }
    return n;
}

// the i-th 32 x 32 tile of the frame (jobs in order, row-major inside a job)
__device__ inline SsimTile tile_at(const gs_frame& f, int tw, int th, uint32_t i) {
    SsimTile t;
    int j = 0, nax = 1;
    uint32_t k = i;
    for (; j < f.n_jobs; j++) {
        const uint32_t n = job_tiles(f.jobs[j], tw, th, nax);
        if (k < n) break;
        k -= n;
    }
    const gs_job job = f.jobs[j];
    const gs_camera cam = f.cams[job.cam];
    t.job = j;
    t.x0 = int(k % uint32_t(nax)) * kTile;
    t.y0 = int(k / uint32_t(nax)) * kTile;
    t.W = cam.width;
    t.H = cam.height;
    t.plane = int64_t(t.W) * t.H;
    t.px = 3 * job.px0;
    return t;
}

// Staged element i (row-major over the kIn x kIn halo tile) of a plane: the
// address is clamped into the image so every load is issued unconditionally
// (all of a thread's loads in flight at once); `in` says whether it was
// inside.
constexpr int kStage = (kIn * kIn + kThreads - 1) / kThreads;

struct StageIdx {
    int32_t off[kStage];      // element offset inside the plane (clamped)
    uint32_t in;              // bit it: element inside the image
};

__device__ inline StageIdx stage_index(const SsimTile& t) {
    StageIdx s;
    s.in = 0;
#pragma unroll
    for (int it = 0; it < kStage; it++) {
        const int i = min(int(threadIdx.x) + it * kThreads, kIn * kIn - 1);
        const int r = i / kIn, c = i % kIn;
        const int gy = t.y0 - kRad + r, gx = t.x0 - kRad + c;
        const int cy = min(max(gy, 0), t.H - 1), cx = min(max(gx, 0), t.W - 1);
        s.off[it] = cy * t.W + cx;
        if (gy == cy && gx == cx) s.in |= 1u << it;
    }
    return s;
}

__device__ inline float block_sum(float v, float* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; i++) s += red[i];
    __syncthreads();
    return s;
}

// horizontal pass of M staged planes: dst[m][r][c] = sum_k g[k] src[m][r][c + k]
// (kBlk consecutive outputs per item, each staged value read once)
template <int M>
__device__ inline void blur_rows(const float (*src)[kIn][kPitch], float (*dst)[kIn][kHPitch], const Taps& taps) {
    for (int i = threadIdx.x; i < kIn * (kTile / kBlk); i += kThreads) {
        const int r = i / (kTile / kBlk), c0 = (i % (kTile / kBlk)) * kBlk;
        float acc[M][kBlk];
#pragma unroll
        for (int q = 0; q < kBlk; q++)
#pragma unroll
            for (int m = 0; m < M; m++) acc[m][q] = 0.f;
#pragma unroll
        for (int k = 0; k < kBlk + kTaps - 1; k++) {
            float h[M];
#pragma unroll
            for (int m = 0; m < M; m++) h[m] = src[m][r][c0 + k];
#pragma unroll
            for (int q = 0; q < kBlk; q++) {
                const int tap = k - q;
                if (tap < 0 || tap >= kTaps) continue;
                const float g = taps.g[tap];
#pragma unroll
                for (int m = 0; m < M; m++) acc[m][q] += g * h[m];
            }
        }
#pragma unroll
        for (int m = 0; m < M; m++)
#pragma unroll
            for (int q = 0; q < kBlk; q++) dst[m][r][c0 + q] = acc[m][q];
    }
}

// horizontal pass of the forward: from staged x and y, the five window sums
// of x, y, x^2, y^2, xy (products formed once per staged value and item)
__device__ inline void blur_rows_moments(const float (*src)[kIn][kPitch], float (*dst)[kIn][kHPitch],
                                         const Taps& taps) {
    for (int i = threadIdx.x; i < kIn * (kTile / kBlk); i += kThreads) {
        const int r = i / (kTile / kBlk), c0 = (i % (kTile / kBlk)) * kBlk;
        float acc[5][kBlk];
#pragma unroll
        for (int q = 0; q < kBlk; q++)
#pragma unroll
            for (int m = 0; m < 5; m++) acc[m][q] = 0.f;
#pragma unroll
        for (int k = 0; k < kBlk + kTaps - 1; k++) {
            const float a = src[0][r][c0 + k], b = src[1][r][c0 + k];
            const float h[5] = {a, b, a * a, b * b, a * b};
#pragma unroll
            for (int q = 0; q < kBlk; q++) {
                const int tap = k - q;
                if (tap < 0 || tap >= kTaps) continue;
                const float g = taps.g[tap];
#pragma unroll
                for (int m = 0; m < 5; m++) acc[m][q] += g * h[m];
            }
        }
#pragma unroll
        for (int m = 0; m < 5; m++)
#pragma unroll
            for (int q = 0; q < kBlk; q++) dst[m][r][c0 + q] = acc[m][q];
    }
}

// vertical pass for this thread's column c and rows r0 .. r0 + kBlk - 1
template <int M>
__device__ inline void blur_cols(const float (*src)[kIn][kHPitch], int c, int r0, const Taps& taps,
                                 float (&acc)[M][kBlk]) {
#pragma unroll
    for (int q = 0; q < kBlk; q++)
#pragma unroll
        for (int m = 0; m < M; m++) acc[m][q] = 0.f;
#pragma unroll
    for (int k = 0; k < kBlk + kTaps - 1; k++) {
        float h[M];
#pragma unroll
        for (int m = 0; m < M; m++) h[m] = src[m][r0 + k][c];
#pragma unroll
        for (int q = 0; q < kBlk; q++) {
            const int tap = k - q;
            if (tap < 0 || tap >= kTaps) continue;
            const float g = taps.g[tap];
#pragma unroll
            for (int m = 0; m < M; m++) acc[m][q] += g * h[m];
        }
    }
}

__global__ __launch_bounds__(kThreads, 3) void k_ssim_fwd(gs_frame f, int tw, int th, const float* __restrict__ rgb,
                                                       const float* __restrict__ tgt,
                                                       float lambda, Taps taps, float* __restrict__ dmaps,
                                                       int64_t map_stride, float* __restrict__ loss_out) {
    __shared__ float st[2][kIn][kPitch];       // staged x, y
    __shared__ float hs[5][kIn][kHPitch];
    __shared__ float red[kThreads / 64];
    const uint32_t cnt = frame_tiles(f, tw, th);
    uint32_t i = blockIdx.x;
    if (i >= cnt) return;
    SsimTile t = tile_at(f, tw, th, i);
    StageIdx si = stage_index(t);
    float va[kStage], vb[kStage];
#pragma unroll
    for (int it = 0; it < kStage; it++) {
        va[it] = rgb[t.px + si.off[it]];
        vb[it] = tgt[t.px + si.off[it]];
    }
    const int c = int(threadIdx.x) % kTile, r0 = (int(threadIdx.x) / kTile) * kBlk;
    // loss sums of the workgroup's tiles of one job, added to loss_out when
    // the job changes or the workgroup is done (one atomic per job and
    // workgroup: per-tile atomics on one word would serialise)
    float s_sum = 0.f, l1_sum = 0.f;
    int firsts = 0;
    while (true) {
        const gs_job job = f.jobs[t.job];
        const float n = 3.f * float(t.W) * float(t.H);
        const float coef = -job.loss_weight * lambda / n;
        const uint32_t inext = i + gridDim.x;
        SsimTile tn = t;
        StageIdx sn = si;
        for (int ch = 0; ch < 3; ch++) {
            const int64_t base = t.px + ch * t.plane;
#pragma unroll
            for (int it = 0; it < kStage; it++) {
                const int e = int(threadIdx.x) + it * kThreads;
                if (e < kIn * kIn) {
                    const bool in = (si.in >> it) & 1u;
                    st[0][e / kIn][e % kIn] = in ? va[it] : 0.f;
                    st[1][e / kIn][e % kIn] = in ? vb[it] : 0.f;
                }
            }
            __syncthreads();
            // the next item's tile, in flight during this one
            if (ch < 2) {
#pragma unroll
                for (int it = 0; it < kStage; it++) {
                    va[it] = rgb[base + t.plane + si.off[it]];
                    vb[it] = tgt[base + t.plane + si.off[it]];
                }
            } else if (inext < cnt) {
                tn = tile_at(f, tw, th, inext);
                sn = stage_index(tn);
#pragma unroll
                for (int it = 0; it < kStage; it++) {
                    va[it] = rgb[tn.px + sn.off[it]];
                    vb[it] = tgt[tn.px + sn.off[it]];
                }
            }
            blur_rows_moments(st, hs, taps);
            __syncthreads();
            float acc[5][kBlk];
            blur_cols<5>(hs, c, r0, taps, acc);
#pragma unroll
            for (int q = 0; q < kBlk; q++) {
                const int r = r0 + q;
                const int gy = t.y0 + r, gx = t.x0 + c;
                if (gy >= t.H || gx >= t.W) continue;
                const float mx = acc[0][q], my = acc[1][q];
                const float vx = acc[2][q] - mx * mx, vy = acc[3][q] - my * my, cxy = acc[4][q] - mx * my;
                const float a1 = 2.f * mx * my + kC1, a2 = 2.f * cxy + kC2;
                const float b1 = mx * mx + my * my + kC1, b2 = vx + vy + kC2;
                const float inv = 1.f / (b1 * b2);
                const float s = a1 * a2 * inv;
                const float d_xx = -s * (b1 * inv);          // -S / B2
                const float d_xy = 2.f * a1 * inv;
                const float d_mu = 2.f * my * a2 * inv - 2.f * mx * s * (b2 * inv) - 2.f * mx * d_xx - my * d_xy;
                const int64_t o = base + int64_t(gy) * t.W + gx;
                dmaps[o] = coef * d_mu;
                dmaps[map_stride + o] = coef * d_xx;
                dmaps[2 * map_stride + o] = coef * d_xy;
                s_sum += s;
                const float d = st[0][r + kRad][c + kRad] - st[1][r + kRad][c + kRad];
                l1_sum += d < 0.f ? -d : d;
            }
            __syncthreads();                   // st and hs are rewritten by the next item
        }
        if (t.x0 == 0 && t.y0 == 0) firsts++;
        // uniform: the loss is optional, and the next tile is the same for the workgroup
        if (loss_out != nullptr && (inext >= cnt || tn.job != t.job)) {
            const float ss = block_sum(s_sum, red);
            const float ls = block_sum(l1_sum, red);
            if (threadIdx.x == 0) {
                // w (mean |d| - lambda mean S), plus w lambda once per job for the 1 of 1 - mean S
                const float add = job.loss_weight * (ls - lambda * ss) / n + float(firsts) * job.loss_weight * lambda;
                atomicAdd(loss_out + t.job, add);
            }
            s_sum = l1_sum = 0.f;
            firsts = 0;
        }
        if (inext >= cnt) break;
        i = inext;
        t = tn;
        si = sn;
    }
}

__device__ inline void out_index(const SsimTile& t, int c, int r0, int32_t (&oo)[kBlk], uint32_t& oin) {
    oin = 0;
#pragma unroll
    for (int q = 0; q < kBlk; q++) {
        const int gy = t.y0 + r0 + q, gx = t.x0 + c;
        oo[q] = min(gy, t.H - 1) * t.W + min(gx, t.W - 1);
        if (gy < t.H && gx < t.W) oin |= 1u << q;
    }
}

__global__ __launch_bounds__(kThreads) void k_ssim_bwd(gs_frame f, int tw, int th, const float* __restrict__ rgb,
                                                       const float* __restrict__ tgt,
                                                       Taps taps, const float* __restrict__ dmaps, int64_t map_stride,
                                                       float* __restrict__ grad) {
    __shared__ float sd[3][kIn][kPitch];
    __shared__ float hd[3][kIn][kHPitch];
    const uint32_t cnt = frame_tiles(f, tw, th);
    uint32_t i = blockIdx.x;
    if (i >= cnt) return;
    const int c = int(threadIdx.x) % kTile, r0 = (int(threadIdx.x) / kTile) * kBlk;
    SsimTile t = tile_at(f, tw, th, i);
    StageIdx si = stage_index(t);
    int32_t oo[kBlk];
    uint32_t oin;
    out_index(t, c, r0, oo, oin);
    float v0[kStage], v1[kStage], v2[kStage], xo[kBlk], yo[kBlk];
#pragma unroll
    for (int it = 0; it < kStage; it++) {
        v0[it] = dmaps[t.px + si.off[it]];
        v1[it] = dmaps[map_stride + t.px + si.off[it]];
        v2[it] = dmaps[2 * map_stride + t.px + si.off[it]];
    }
#pragma unroll
    for (int q = 0; q < kBlk; q++) {
        xo[q] = rgb[t.px + oo[q]];
        yo[q] = tgt[t.px + oo[q]];
    }
    while (true) {
        const gs_job job = f.jobs[t.job];
        const float l1 = job.loss_weight / (3.f * float(t.W) * float(t.H));
        const uint32_t inext = i + gridDim.x;
        SsimTile tn = t;
        StageIdx sn = si;
        int32_t on[kBlk];
        uint32_t onin = oin;
#pragma unroll
        for (int q = 0; q < kBlk; q++) on[q] = oo[q];
        for (int ch = 0; ch < 3; ch++) {
            const int64_t base = t.px + ch * t.plane;
#pragma unroll
            for (int it = 0; it < kStage; it++) {
                const int e = int(threadIdx.x) + it * kThreads;
                if (e < kIn * kIn) {
                    const bool in = (si.in >> it) & 1u;
                    sd[0][e / kIn][e % kIn] = in ? v0[it] : 0.f;
                    sd[1][e / kIn][e % kIn] = in ? v1[it] : 0.f;
                    sd[2][e / kIn][e % kIn] = in ? v2[it] : 0.f;
                }
            }
            float xc[kBlk], yc[kBlk];
#pragma unroll
            for (int q = 0; q < kBlk; q++) { xc[q] = xo[q]; yc[q] = yo[q]; }
            __syncthreads();
            // the next item's tile, in flight during this one
            if (ch < 2) {
                const int64_t nb = base + t.plane;
#pragma unroll
                for (int it = 0; it < kStage; it++) {
                    v0[it] = dmaps[nb + si.off[it]];
                    v1[it] = dmaps[map_stride + nb + si.off[it]];
                    v2[it] = dmaps[2 * map_stride + nb + si.off[it]];
                }
#pragma unroll
                for (int q = 0; q < kBlk; q++) {
                    xo[q] = rgb[nb + oo[q]];
                    yo[q] = tgt[nb + oo[q]];
                }
            } else if (inext < cnt) {
                tn = tile_at(f, tw, th, inext);
                sn = stage_index(tn);
                out_index(tn, c, r0, on, onin);
#pragma unroll
                for (int it = 0; it < kStage; it++) {
                    v0[it] = dmaps[tn.px + sn.off[it]];
                    v1[it] = dmaps[map_stride + tn.px + sn.off[it]];
                    v2[it] = dmaps[2 * map_stride + tn.px + sn.off[it]];
                }
#pragma unroll
                for (int q = 0; q < kBlk; q++) {
                    xo[q] = rgb[tn.px + on[q]];
                    yo[q] = tgt[tn.px + on[q]];
                }
            }
            blur_rows<3>(sd, hd, taps);
            __syncthreads();
            float acc[3][kBlk];
            blur_cols<3>(hd, c, r0, taps, acc);
#pragma unroll
            for (int q = 0; q < kBlk; q++) {
                const float x = xc[q], y = yc[q];
                const float d = x - y;
                const float s1 = d > 0.f ? l1 : (d < 0.f ? -l1 : 0.f);
                if ((oin >> q) & 1u) grad[base + oo[q]] = s1 + acc[0][q] + 2.f * x * acc[1][q] + y * acc[2][q];
            }
            __syncthreads();
        }
        if (inext >= cnt) break;
        i = inext;
        t = tn;
        si = sn;
        oin = onin;
#pragma unroll
        for (int q = 0; q < kBlk; q++) oo[q] = on[q];
    }
}

Taps window_taps() {
    Taps t;
    double g[kTaps], sum = 0.0;
    for (int k = 0; k < kTaps; k++) {
        const double r = double(k - kRad);
        g[k] = std::exp(-r * r / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k < kTaps; k++) t.g[k] = float(g[k] / sum);
    return t;
}

}  // namespace

size_t ssim_workspace_size(int64_t n_pixels) { return size_t(n_pixels) * 3 * 3 * sizeof(float); }

hipError_t launch_ssim_loss_grad(const gs_frame& f, const gs_raster_cfg& cfg, const float* rgb, const float* tgt,
                                 float lambda, float* grad, float* loss, void* ws, hipStream_t s) {
    if (f.n_tiles == 0) return hipSuccess;
    const Taps taps = window_taps();
    const int64_t stride = 3 * f.n_pixels;
    float* maps = static_cast<float*>(ws);
    // persistent grids: as many workgroups as the device holds at once (never
    // more than the frame's 32 x 32 tiles, which are at most its binning tiles)
    static int resident[2] = {0, 0};
    static int resident_dev = -1;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (resident_dev != dev) {
        int cus = 0, nf = 0, nb = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nf, k_ssim_fwd, kThreads, 0)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ssim_bwd, kThreads, 0)) != hipSuccess) return e;
        resident[0] = cus * (nf > 0 ? nf : 1);
        resident[1] = cus * (nb > 0 ? nb : 1);
        resident_dev = dev;
    }
    const int gf = f.n_tiles < resident[0] ? f.n_tiles : resident[0];
    const int gb = f.n_tiles < resident[1] ? f.n_tiles : resident[1];
    GS_LAUNCH("k_ssim_fwd", k_ssim_fwd, dim3(unsigned(gf)), dim3(kThreads), 0, s, f, cfg.tile_w, cfg.tile_h, rgb, tgt,
              lambda, taps, maps, stride, loss);
    GS_LAUNCH("k_ssim_bwd", k_ssim_bwd, dim3(unsigned(gb)), dim3(kThreads), 0, s, f, cfg.tile_w, cfg.tile_h, rgb, tgt,
              taps, maps, stride, grad);
    return hipGetLastError();
}

}  // namespace gs
