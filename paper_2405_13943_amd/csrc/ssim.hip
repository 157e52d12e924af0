// The photometric loss of Eq. 3 with its structural term:
//   L_j = w_j (mean |C - target| + lambda (1 - mean SSIM)),
// SSIM of Wang et al. under an 11 x 11 Gaussian window (sigma 1.5, zero
// outside the image), per colour channel, mean over pixels and channels.
//
// Two passes over 32 x 32 pixel tiles, each staging its tile plus a 5-pixel
// halo in LDS and blurring separably (rows, then columns):
//   k_ssim_fwd  blurs x, y, x^2, y^2, xy; forms SSIM and its derivatives with
//               respect to the window sums (mu_x, E[x^2], E[xy]); writes the
//               three derivative maps (pre-scaled by -w lambda / N) and adds
//               the job's loss;
//   k_ssim_bwd  blurs the three maps and combines them with x and y into
//               dL/dC (plus the L1 term), the external gradient of the
//               compositing backward.
// Both passes stream their inputs once from HBM (the halo re-reads hit L2).
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
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Taps {
    float g[kTaps];
};

struct SsimTile {
    int job, x0, y0, W, H;
    int64_t base;     // first element of this channel's plane
    bool active;
};

// The tile of this workgroup: binning tiles at multiples of 32 pixels own a
// 32 x 32 block; the others have nothing to do.
__device__ inline SsimTile ssim_tile(const gs_frame& f, int tw, int th) {
    SsimTile t;
    const int tile = int(blockIdx.x);
    t.job = job_of_tile(f.jobs, f.n_jobs, tile);
    const gs_job job = f.jobs[t.job];
    const gs_camera cam = f.cams[job.cam];
    const int lt = tile - job.tile0;
    const int tx = lt % job.tiles_x, ty = lt / job.tiles_x;
    t.x0 = tx * tw;
    t.y0 = ty * th;
    t.W = cam.width;
    t.H = cam.height;
    t.active = (t.x0 % kTile) == 0 && (t.y0 % kTile) == 0;
    const int64_t plane = int64_t(t.W) * t.H;
    t.base = 3 * job.px0 + int64_t(blockIdx.y) * plane;
    return t;
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

__global__ __launch_bounds__(kThreads) void k_ssim_fwd(gs_frame f, int tw, int th, const float* __restrict__ rgb,
                                                       const float* __restrict__ tgt, float lambda, Taps taps,
                                                       float* __restrict__ dmaps, int64_t map_stride,
                                                       float* __restrict__ loss_out) {
    __shared__ float sx[kIn][kPitch], sy[kIn][kPitch];
    __shared__ float hs[5][kIn][kHPitch];
    __shared__ float red[kThreads / 64];
    const SsimTile t = ssim_tile(f, tw, th);
    if (!t.active) return;                    // uniform per workgroup
    const gs_job job = f.jobs[t.job];
    for (int i = threadIdx.x; i < kIn * kIn; i += kThreads) {
        const int r = i / kIn, c = i % kIn;
        const int gy = t.y0 - kRad + r, gx = t.x0 - kRad + c;
        const bool in = gy >= 0 && gy < t.H && gx >= 0 && gx < t.W;
        const int64_t o = t.base + int64_t(gy) * t.W + gx;
        sx[r][c] = in ? rgb[o] : 0.f;
        sy[r][c] = in ? tgt[o] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kIn * kTile; i += kThreads) {
        const int r = i / kTile, c = i % kTile;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
        for (int k = 0; k < kTaps; k++) {
            const float g = taps.g[k], a = sx[r][c + k], b = sy[r][c + k];
            a0 += g * a;
            a1 += g * b;
            a2 += g * (a * a);
            a3 += g * (b * b);
            a4 += g * (a * b);
        }
        hs[0][r][c] = a0;
        hs[1][r][c] = a1;
        hs[2][r][c] = a2;
        hs[3][r][c] = a3;
        hs[4][r][c] = a4;
    }
    __syncthreads();
    const float n = 3.f * float(t.W) * float(t.H);
    const float coef = -job.loss_weight * lambda / n;
    float s_sum = 0.f, l1_sum = 0.f;
    for (int i = threadIdx.x; i < kTile * kTile; i += kThreads) {
        const int r = i / kTile, c = i % kTile;
        const int gy = t.y0 + r, gx = t.x0 + c;
        if (gy >= t.H || gx >= t.W) continue;
        float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
        for (int k = 0; k < kTaps; k++) {
            const float g = taps.g[k];
            mx += g * hs[0][r + k][c];
            my += g * hs[1][r + k][c];
            exx += g * hs[2][r + k][c];
            eyy += g * hs[3][r + k][c];
            exy += g * hs[4][r + k][c];
        }
        const float vx = exx - mx * mx, vy = eyy - my * my, cxy = exy - mx * my;
        const float a1 = 2.f * mx * my + kC1, a2 = 2.f * cxy + kC2;
        const float b1 = mx * mx + my * my + kC1, b2 = vx + vy + kC2;
        const float inv = 1.f / (b1 * b2);
        const float s = a1 * a2 * inv;
        const float d_xx = -s / b2;
        const float d_xy = 2.f * a1 * inv;
        const float d_mu = 2.f * my * a2 * inv - 2.f * mx * s / b1 - 2.f * mx * d_xx - my * d_xy;
        const int64_t o = t.base + int64_t(gy) * t.W + gx;
        dmaps[o] = coef * d_mu;
        dmaps[map_stride + o] = coef * d_xx;
        dmaps[2 * map_stride + o] = coef * d_xy;
        s_sum += s;
        const float d = sx[r + kRad][c + kRad] - sy[r + kRad][c + kRad];
        l1_sum += d < 0.f ? -d : d;
    }
    if (loss_out == nullptr) return;          // uniform: the loss is optional
    const float ss = block_sum(s_sum, red);
    const float ls = block_sum(l1_sum, red);
    if (threadIdx.x == 0) {
        // w (mean |d| - lambda mean S), plus w lambda once per job for the 1 of 1 - mean S
        float add = job.loss_weight * (ls - lambda * ss) / n;
        if (t.x0 == 0 && t.y0 == 0 && blockIdx.y == 0) add += job.loss_weight * lambda;
        atomicAdd(loss_out + t.job, add);
    }
}

__global__ __launch_bounds__(kThreads) void k_ssim_bwd(gs_frame f, int tw, int th, const float* __restrict__ rgb,
                                                       const float* __restrict__ tgt, Taps taps,
                                                       const float* __restrict__ dmaps, int64_t map_stride,
                                                       float* __restrict__ grad) {
    __shared__ float sd[3][kIn][kPitch];
    __shared__ float hd[3][kIn][kHPitch];
    const SsimTile t = ssim_tile(f, tw, th);
    if (!t.active) return;
    const gs_job job = f.jobs[t.job];
    for (int i = threadIdx.x; i < kIn * kIn; i += kThreads) {
        const int r = i / kIn, c = i % kIn;
        const int gy = t.y0 - kRad + r, gx = t.x0 - kRad + c;
        const bool in = gy >= 0 && gy < t.H && gx >= 0 && gx < t.W;
        const int64_t o = t.base + int64_t(gy) * t.W + gx;
        sd[0][r][c] = in ? dmaps[o] : 0.f;
        sd[1][r][c] = in ? dmaps[map_stride + o] : 0.f;
        sd[2][r][c] = in ? dmaps[2 * map_stride + o] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kIn * kTile; i += kThreads) {
        const int r = i / kTile, c = i % kTile;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int k = 0; k < kTaps; k++) {
            const float g = taps.g[k];
            a0 += g * sd[0][r][c + k];
            a1 += g * sd[1][r][c + k];
            a2 += g * sd[2][r][c + k];
        }
        hd[0][r][c] = a0;
        hd[1][r][c] = a1;
        hd[2][r][c] = a2;
    }
    __syncthreads();
    const float l1 = job.loss_weight / (3.f * float(t.W) * float(t.H));
    for (int i = threadIdx.x; i < kTile * kTile; i += kThreads) {
        const int r = i / kTile, c = i % kTile;
        const int gy = t.y0 + r, gx = t.x0 + c;
        if (gy >= t.H || gx >= t.W) continue;
        float b_mu = 0.f, b_xx = 0.f, b_xy = 0.f;
#pragma unroll
        for (int k = 0; k < kTaps; k++) {
            const float g = taps.g[k];
            b_mu += g * hd[0][r + k][c];
            b_xx += g * hd[1][r + k][c];
            b_xy += g * hd[2][r + k][c];
        }
        const int64_t o = t.base + int64_t(gy) * t.W + gx;
        const float x = rgb[o], y = tgt[o];
        const float d = x - y;
        const float s1 = d > 0.f ? l1 : (d < 0.f ? -l1 : 0.f);
        grad[o] = s1 + b_mu + 2.f * x * b_xx + y * b_xy;
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
                                 float lambda, float* grad, float* loss, float* ws, hipStream_t s) {
    if (f.n_tiles == 0) return hipSuccess;
    const Taps taps = window_taps();
    const int64_t stride = 3 * f.n_pixels;
    const dim3 grid(unsigned(f.n_tiles), 3), block(kThreads);
    GS_LAUNCH("k_ssim_fwd", k_ssim_fwd, grid, block, 0, s, f, cfg.tile_w, cfg.tile_h, rgb, tgt, lambda, taps, ws, stride,
              loss);
    GS_LAUNCH("k_ssim_bwd", k_ssim_bwd, grid, block, 0, s, f, cfg.tile_w, cfg.tile_h, rgb, tgt, taps, ws, stride,
              grad);
    return hipGetLastError();
}

}  // namespace gs
