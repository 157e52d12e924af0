// Device-side helpers shared by the libgs kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gs {

constexpr int kWave = 64;

// 16-byte accesses with the non-temporal hint, for state that one step
// touches once (the optimiser's moments and the consensus target): they
// keep it from evicting the lines that the same kernel reads again
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ inline float4 load_stream4(const float* p) {
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline void store_stream4(float* p, float4 v) {
    const f32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(p));
}

// ---------------------------------------------------------------------------
// scalar-type traits: FP32 product path, FP64 instantiation for adjoint checks

template <typename T> struct Num;
template <> struct Num<float> {
    __device__ static inline float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
    __device__ static inline float log2(float x) { return __log2f(x); }
    __device__ static inline float exp(float x) { return __expf(x); }
    __device__ static inline float log(float x) { return __logf(x); }
    __device__ static inline float sqrt(float x) { return __builtin_sqrtf(x); }
    __device__ static inline float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }   // hardware, ~1 ulp
    __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }    // hardware, ~1 ulp
    __device__ static inline float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    __device__ static inline float max(float a, float b) { return __builtin_fmaxf(a, b); }
    __device__ static inline float min(float a, float b) { return __builtin_fminf(a, b); }
};
template <> struct Num<double> {
    __device__ static inline double exp2(double x) { return ::exp2(x); }
    __device__ static inline double log2(double x) { return ::log2(x); }
    __device__ static inline double exp(double x) { return ::exp(x); }
    __device__ static inline double log(double x) { return ::log(x); }
    __device__ static inline double sqrt(double x) { return ::sqrt(x); }
    __device__ static inline double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    __device__ static inline double rcp(double x) { return 1.0 / x; }
    __device__ static inline double fma(double a, double b, double c) { return ::fma(a, b, c); }
    __device__ static inline double max(double a, double b) { return ::fmax(a, b); }
    __device__ static inline double min(double a, double b) { return ::fmin(a, b); }
};

// ln 2 and log2 e as the scalar type
template <typename T> __device__ constexpr T kLn2() { return T(0.69314718055994530942); }
template <typename T> __device__ constexpr T kLog2e() { return T(1.44269504088896340736); }

// ---------------------------------------------------------------------------
// Frame of the compositing backward's second moments.  A footprint much
// longer than it is wide puts almost all of sum ge (p - m)(p - m)^T along its
// long axis, while the gradient of the screen covariance is dominated by the
// part across it; taken from pixel-frame sums, that part would come out of a
// near-cancellation.  So the backward accumulates the moments in the
// footprint's axes: e1 along the axis of the conic's largest eigenvalue (the
// narrow one) and e2 across it.  The projection stores that axis as one word,
// t = tan(theta / 2) of its direction (cos theta, sin theta) with
// cos theta >= 0, and every user decodes the same word with the same
// operations, so all of them rotate by the same matrix.

// code of the narrow axis of the conic [[a, b], [b, c]] (any axis when a = c
// and b = 0)
template <typename T>
__device__ inline T narrow_axis_code(T a, T b, T c) {
    const T h = T(0.5) * (a - c);
    const T r = Num<T>::sqrt(Num<T>::fma(h, h, b * b));
    // eigenvector of the eigenvalue (a + c) / 2 + r, from the better-conditioned row
    T vx = h >= T(0) ? h + r : b;
    T vy = h >= T(0) ? b : r - h;
    const T n2 = Num<T>::fma(vx, vx, vy * vy);
    if (!(n2 > T(0))) return T(0);
    const T inv = Num<T>::rsqrt(n2);
    vx *= inv;
    vy *= inv;
    if (vx < T(0)) {
        vx = -vx;
        vy = -vy;
    }
    return vy / (T(1) + vx);
}

// (cos theta, sin theta) of a narrow-axis code
template <typename T>
__device__ inline void narrow_axis(T t, T& c, T& s) {
    const T w = T(1) / Num<T>::fma(t, t, T(1));
    c = Num<T>::fma(-t, t, T(1)) * w;
    s = (t + t) * w;
}

// ---------------------------------------------------------------------------
// per-record metadata word 1: covered tiles in the low 24 bits, the colour
// clamp of each channel (SH sum + 0.5 <= 0) in bits 24..26

// compositing wavefronts per tile of the forward and the backward (0 reads
// as 1; GS_WAVES_ADAPTIVE in the backward: per tile, see adaptive_waves)
__host__ __device__ inline int fwd_waves(const gs_raster_cfg& c) {
    return c.fwd_waves == GS_WAVES_ADAPTIVE ? 0 : (c.fwd_waves <= 1 ? 1 : c.fwd_waves);
}
__host__ __device__ inline bool bwd_adaptive(const gs_raster_cfg& c) { return c.bwd_waves == GS_WAVES_ADAPTIVE; }
__host__ __device__ inline int bwd_waves(const gs_raster_cfg& c) {
    return bwd_adaptive(c) ? 0 : (c.bwd_waves <= 1 ? 1 : c.bwd_waves);
}
// backward partial slots per tile pair the projection backward reads: one
// per wavefront; adaptive: one (split tiles fold theirs into the first)
__host__ __device__ inline int bwd_slots(const gs_raster_cfg& c) { return bwd_adaptive(c) ? 1 : bwd_waves(c); }

// Wavefronts of one tile in an adaptive compositing pass, from its list
// length against the frame's mean list length: 4 above 4 x the mean, 2 above
// 1.25 x, else 1; never more than the tile's quadrants.  Exact integer
// arithmetic, so every kernel that needs it agrees.
__device__ inline int adaptive_waves(uint32_t count, uint32_t pairs, int n_tiles, int quads) {
    const uint64_t a = 4ull * count * uint64_t(n_tiles);
    const int s = a > 16ull * pairs ? 4 : (a > 5ull * pairs ? 2 : 1);
    return s < quads ? s : quads;
}

// Wavefront gw of an adaptive compositing launch -> (tile, sub, waves) from
// the plan of k_tile_plan; false when the wavefront has no work (past the
// plan, or a plan that does not describe n_tiles tiles).
__device__ inline bool plan_wave(const uint32_t* __restrict__ order, int n_tiles, uint32_t gw, int& tile, int& sub,
                                 int& waves) {
    const uint32_t nt = uint32_t(n_tiles), n4 = order[0], n2 = order[1], n1 = order[2];
    if (n4 > nt || n2 > nt || n1 > nt || n4 + n2 + n1 != nt) return false;
    const uint32_t* list = order + 4;
    uint32_t g = gw, t;
    if (g < 4u * n4) {
        t = list[g / 4u];
        sub = int(g % 4u);
        waves = 4;
    } else if ((g -= 4u * n4) < 2u * n2) {
        t = list[n4 + g / 2u];
        sub = int(g % 2u);
        waves = 2;
    } else if ((g -= 2u * n2) < n1) {
        t = list[n4 + n2 + g];
        sub = 0;
        waves = 1;
    } else {
        return false;
    }
    tile = int(t);
    return t < nt;
}

// Partials of wavefront `sub` for pair e in the adaptive layout: slot 0 of
// every pair dense at e, the slots of the further wavefronts of split tiles
// after all of them (3 per pair), so a one-wavefront tile's pairs stay
// contiguous.  Capacity counts pairs; 9 values per slot.
__host__ __device__ inline int64_t adaptive_slot(uint64_t capacity, uint64_t e, int sub) {
    return sub == 0 ? int64_t(e) * 9 : (int64_t(capacity) + int64_t(e) * 3 + (sub - 1)) * 9;
}

// quadrants (bit k = quadrant k of the tile) owned by wavefront `sub` of `waves`
__device__ inline uint32_t owned_quadrants(int quads, int waves, int sub) {
    const int per = quads / waves;
    return ((1u << per) - 1u) << (sub * per);
}

constexpr uint32_t kTilesMask = 0xffffffu;
__host__ __device__ inline uint32_t meta_tiles(uint32_t y) { return y & kTilesMask; }
__host__ __device__ inline uint32_t meta_clamp(uint32_t y) { return (y >> 24) & 7u; }

// ---------------------------------------------------------------------------
// job lookup: jobs are laid out in ascending rec0 / tile0 / px0 order

__device__ inline int job_of_record(const gs_job* __restrict__ jobs, int n_jobs, int64_t r) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].rec0 <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int job_of_tile(const gs_job* __restrict__ jobs, int n_jobs, int tile) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// wave64 primitives

__device__ inline int lane_id() { return __lane_id(); }

__device__ inline uint64_t lanemask_lt() { return (uint64_t(1) << lane_id()) - 1; }

// lanes where b holds, as a wave-uniform 64-bit mask (every lane active)
__device__ inline uint64_t lane_mask(bool b) { return __builtin_amdgcn_ballot_w64(b); }
// this lane's bit of a wave-uniform lane mask, read as a per-lane condition
// without moving the mask into vector registers
__device__ inline bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Sum over the 64 lanes of a wave, returned to every lane.  FP32 uses DPP
// (quad permutes, row rotations, then row broadcasts into lane 63); FP64
// uses a butterfly of cross-lane shuffles.
template <int CTRL, int ROW_MASK>
__device__ inline float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// DPP move over all rows and banks in which a lane without a source reads 0
template <int CTRL>
__device__ inline float dpp_move_bc(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

__device__ inline float wave_sum(float v) {
    v += dpp_move<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x124, 0xf>(v);  // row_ror:4
    v += dpp_move<0x128, 0xf>(v);  // row_ror:8
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum over each row of 16 lanes, complete in the row's last lane (15):
// quad sums, then shifts right by 4 and 8 lanes within the row (lanes with
// no source add zero), so every step is one fused DPP add.
__device__ inline float row_sum_last(float v) {
    v += dpp_move_bc<0xb1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move_bc<0x4e>(v);    // quad_perm [2,3,0,1]
    v += dpp_move_bc<0x114>(v);   // row_shr:4
    v += dpp_move_bc<0x118>(v);   // row_shr:8
    return v;
}

__device__ inline double row_sum_last(double v) {
    for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over each row of 16 lanes, returned to every lane of the row.
__device__ inline float row_sum(float v) {
    v += dpp_move<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x124, 0xf>(v);  // row_ror:4
    v += dpp_move<0x128, 0xf>(v);  // row_ror:8
    return v;
}

__device__ inline double row_sum(double v) {
    for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// inclusive prefix sum over the lanes of a wave
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = lane_id();
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    return v;
}

// ---------------------------------------------------------------------------
// XCD-aware block order: the dispatcher hands consecutive workgroups to the
// 8 XCDs round robin.  Remapping so that each XCD receives one contiguous run
// of work items keeps neighbouring tiles (which share Gaussians) in the same
// L2.
__device__ inline int xcd_block(int b, int nb) {
    const int xcd = b & 7, idx = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    const int base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return base + idx;
}

}  // namespace gs
