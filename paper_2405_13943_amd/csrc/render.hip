// Per-tile front-to-back alpha compositing (Eq. 2) and its hand-written
// backward.
//
// One wavefront owns one screen tile made of QX x QY quadrants of 8x8 pixels
// (or, split per tile from the frame's plan, a run of its quadrants); lane l
// holds pixel (l % 8, l / 8) of every quadrant, so PPL = QX * QY pixels per
// lane.  The wave walks the tile's record list in (depth, record) order,
// staging a batch of records at a time in a wave-private LDS slice (one record
// per lane, read back as broadcasts): no workgroup barrier in the walk, and
// each wave stops as soon as all its pixels have terminated.  While staging,
// each lane also computes which quadrants its record can reach (pixel box and
// an exact, conservative bound of alpha over the quadrant); only records that
// reach one are staged (compacted with a ballot prefix), and the compositing
// loop skips (uniformly, per quadrant) every Gaussian that cannot reach
// alpha_min there.  The forward hands these quadrant masks to the backward,
// one byte per list entry.  Past that test the per-pixel work is predicated
// (selects, not branches): a pixel that does not keep a Gaussian adds an
// exact zero and keeps its transmittance, and the forward keeps its per-pixel
// stop flags as wave-wide lane masks, so their bookkeeping runs on the scalar
// unit.  Workgroups are remapped so that each XCD renders one contiguous run
// of tiles (neighbouring tiles share records in that XCD's L2).
//
// The backward runs front to back as well: it recomputes alpha, T and the
// accumulated colour with the forward's operations, keeps a Gaussian at a
// pixel exactly when alpha >= alpha_min and its list position is below the
// forward's contributor count there, and gets the colour behind a Gaussian
// as C_final - C_accumulated, so no per-pair transmittance is ever stored.
// Per (tile, record) pair it forms nine partials per lane and reduces those
// of two records at once with the gfx950 lane-swap instructions and a row
// sum; a row's last lane stores them at the pair's emission index, where the
// projection backward adds each record's pairs in a fixed order
// (deterministic, no float atomics).  The nine values are, with
// ge = dL/dalpha * alpha summed over the pair's pixels and (e1, e2) the
// offset pixel - mean in the footprint's axes (e1 along the conic's narrow
// axis (c, s) that the record carries, e2 = (-s, c) across):
//   sum ge, sum ge e1, sum ge e2, sum ge e1^2, sum ge e1 e2, sum ge e2^2,
//   and dL/dcolour (r, g, b).
// The geometric gradients follow from these moments in closed form.
#include "gs_device.hpp"
#include "gs_internal.hpp"

namespace gs {

constexpr int kRenderWaves = 4;
constexpr int kBwdBatch = 48;   // records staged per backward batch (of the 64 lanes)

// record words as produced by the projection
enum { R_MX = 0, R_MY, R_QA, R_QB, R_QC, R_LO, R_CR, R_CG, R_CB, R_AXIS, R_HX, R_HY };
// LDS slots of a staged backward record past the first nine: the moment frame
enum { S_AXC = 9, S_AXS = 10 };

template <typename T>
struct Rec {
    T mx, my, qa, qb, qc, lo, c[3];
};

// log2 of the Gaussian's alpha at offset (dx, dy) from its mean:
// log2 o - (a dx^2 + 2 b dx dy + c dy^2) log2(e) / 2 with the scale folded
// into qa, qb, qc
template <typename T>
__device__ inline T log2_alpha(const Rec<T>& g, T dx, T dy) {
    using N = Num<T>;
    const T t = N::fma(g.qa, dx, g.qb * dy);
    return N::fma(t, dx, N::fma(g.qc * dy, dy, g.lo));
}

// min(alpha, alpha_max) for alpha >= +0 or NaN: non-negative floats order
// like their bit patterns, and a NaN's pattern lies above every finite one,
// so the unsigned minimum equals fminf (NaN gives alpha_max) in one integer
// instruction, without the NaN quieting fminf costs
template <typename T> __device__ inline T clamp_alpha(T al, T amax);
template <> __device__ inline float clamp_alpha<float>(float al, float amax) {
    return __uint_as_float(min(__float_as_uint(al), __float_as_uint(amax)));
}
template <> __device__ inline double clamp_alpha<double>(double al, double amax) { return Num<double>::min(al, amax); }

template <typename T> __device__ inline T recip(T x);
template <> __device__ inline float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double recip<double>(double x) { return 1.0 / x; }

template <typename T>
__device__ inline Rec<T> lds_rec(const T* s) {
    Rec<T> g;
    g.mx = s[R_MX]; g.my = s[R_MY]; g.qa = s[R_QA]; g.qb = s[R_QB]; g.qc = s[R_QC]; g.lo = s[R_LO];
    g.c[0] = s[R_CR]; g.c[1] = s[R_CG]; g.c[2] = s[R_CB];
    return g;
}

// Load record r into registers (one record per lane while staging).
template <typename T>
__device__ inline void load_rec(const T* __restrict__ rec, uint32_t r, T (&w)[GS_REC_WORDS]) {
    const T* src = rec + int64_t(r) * GS_REC_WORDS;
#pragma unroll
    for (int i = 0; i < GS_REC_WORDS; i++) w[i] = src[i];
}

template <typename T>
__device__ inline T clamp_to(T v, T lo, T hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Quadrant mask of a record for the tile whose top-left pixel is (px0, py0):
// bit k is set unless no pixel centre of quadrant k can reach alpha_min.
// Two conservative tests must both pass.  (1) The record's pixel box
// [mean -+ half-extent] meets the quadrant.  (2) The largest log2 alpha over
// the quadrant's rectangle of pixel centres is at least log2 alpha_min, less a
// margin that covers the rounding of this bound and of the per-pixel
// evaluation.  The exponent is a concave quadratic in (dx, dy): over a
// rectangle that holds the mean its maximum is at the mean, otherwise on an
// edge, at the edge's stationary point clamped to the edge.  Test (2) drops
// what the box keeps only because it is axis-aligned (elongated, rotated
// Gaussians); a skipped pixel would have had alpha < alpha_min, so images and
// gradients are unchanged.
template <typename T>
__device__ inline uint32_t quad_mask_n(const T (&w)[GS_REC_WORDS], int px0, int py0, int nqx, int nq, T lmin) {
    using N = Num<T>;
    const T mx = w[R_MX], my = w[R_MY], qa = w[R_QA], qb = w[R_QB], qc = w[R_QC], lo = w[R_LO];
    const T x0 = mx - w[R_HX], x1 = mx + w[R_HX];
    const T y0 = my - w[R_HY], y1 = my + w[R_HY];
    // on an edge dx = e the maximum over dy sits at dy = sx e; on dy = e, at dx = sy e
    const T sx = -qb * recip(T(2) * qc), sy = -qb * recip(T(2) * qa);
    const T aqb = qb < T(0) ? -qb : qb;
    const T alo = lo < T(0) ? -lo : lo;
    auto expo = [&](T dx, T dy) { return N::fma(N::fma(qa, dx, qb * dy), dx, qc * dy * dy); };
    uint32_t mask = 0;
#pragma unroll 1
    for (int k = 0; k < nq; k++) {
        const T qx = T(px0 + 8 * (k % nqx)), qy = T(py0 + 8 * (k / nqx));
        const bool box = x1 >= qx + T(0.5) && x0 <= qx + T(7.5) && y1 >= qy + T(0.5) && y0 <= qy + T(7.5);
        const T ax = qx + T(0.5) - mx, bx = qx + T(7.5) - mx;
        const T ay = qy + T(0.5) - my, by = qy + T(7.5) - my;
        const bool inside = ax <= T(0) && bx >= T(0) && ay <= T(0) && by >= T(0);
        T best = expo(ax, clamp_to(sx * ax, ay, by));
        best = N::max(best, expo(bx, clamp_to(sx * bx, ay, by)));
        best = N::max(best, expo(clamp_to(sy * ay, ax, bx), ay));
        best = N::max(best, expo(clamp_to(sy * by, ax, bx), by));
        // magnitude of the exponent's terms over the rectangle: scale of the rounding
        const T X = N::max(-ax, bx), Y = N::max(-ay, by);
        const T mag = N::fma(-qa * X, X, N::fma(aqb * X, Y, -qc * Y * Y)) + alo;
        const bool ell = inside || best + lo >= lmin - (T(1e-3) + mag * T(4e-6));
        mask |= box && ell ? (1u << k) : 0u;
    }
    return mask;
}

// the same over the QX x QY quadrants from pixel (px0, py0)
template <typename T, int QX, int QY>
__device__ inline uint32_t quad_mask(const T (&w)[GS_REC_WORDS], int px0, int py0, T lmin) {
    return quad_mask_n(w, px0, py0, QX, QX * QY, lmin);
}

__device__ inline uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// centre coordinate of a lane's pixel in quadrant column/row q: the lane's
// quadrant-0 centre plus 8 q (exact in floating point), so that every tile
// shape computes the same pixel - mean offsets bit for bit
template <typename T>
__device__ inline T quad_centre(T base, int q) {
    return q == 0 ? base : base + T(8 * q);
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stores the nine partials of two records' pairs (a at da, b at db; db may
// be null), each summed over the wave's 64 lanes.  FP32: the two records are
// reduced together; a swap of wave halves (v_permlane32_swap) and an add
// leave record a's sums in lanes 0-31 and b's in lanes 32-63; a swap of
// odd and even rows (v_permlane16_swap) between neighbouring partials and an
// add leave in each row of 16 lanes five partials of one record (the even or
// the odd ones); a row sum finishes them in the row's last lane, which
// stores them.  A fixed sequence of operations: the sums are deterministic.
__device__ inline float swap_add32(float a, float b) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ inline float swap_add16(float a, float b) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

__device__ inline void store_pair_partials(const float (&va)[9], const float (&vb)[9], float* da, float* db) {
    const int lane = lane_id();
    float x[9], y[5];
#pragma unroll
    for (int q = 0; q < 9; q++) x[q] = swap_add32(va[q], vb[q]);
#pragma unroll
    for (int j = 0; j < 4; j++) y[j] = swap_add16(x[2 * j], x[2 * j + 1]);
    y[4] = swap_add16(x[8], 0.f);
#pragma unroll
    for (int j = 0; j < 5; j++) y[j] = row_sum_last(y[j]);
    if ((lane & 15) == 15) {
        const int r = lane >> 4;
        float* dst = r < 2 ? da : db;
        const int par = r & 1;
        if (dst)
#pragma unroll
            for (int j = 0; j < 5; j++)
                if (2 * j + par < 9) dst[2 * j + par] = y[j];
    }
}

__device__ inline void store_pair_partials(const double (&va)[9], const double (&vb)[9], double* da, double* db) {
    double sa[9], sb[9];
#pragma unroll
    for (int q = 0; q < 9; q++) {
        sa[q] = wave_sum(va[q]);
        sb[q] = wave_sum(vb[q]);
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int q = 0; q < 9; q++) {
            da[q] = sa[q];
            if (db) db[q] = sb[q];
        }
    }
}

// ---------------------------------------------------------------------------
// forward

// STATS: also add the number of (pixel, Gaussian) contributions of the
// launch to *kept (one 64-bit atomic per wave).  At least kFwdWavesPerSimd
// wavefronts per SIMD: the FP32 forward then fits in 72 registers without
// spilling, against 80 (6 per SIMD) left to itself.
constexpr int kFwdWavesPerSimd = 7;
template <typename T, int QX, int QY, int NS, bool STATS>
__global__ __launch_bounds__(kWave * kRenderWaves, kFwdWavesPerSimd) void k_render_fwd(
    gs_frame frame, gs_raster_cfg cfg, const T* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, T* __restrict__ rgb, T* __restrict__ Tout, uint32_t* __restrict__ ncontrib,
    unsigned long long* __restrict__ kept, const uint32_t* __restrict__ order, uint8_t* __restrict__ qmask) {
    constexpr int PPL = QX * QY;
    // NS wavefronts per tile, wave `sub` owning the tile's sub-tile of QX x QY
    // quadrants; NS = 0: the plan's wavefronts, heavy tiles first, each owning
    // a run of the tile's quadrants (QX x QY is then the tile)
    constexpr bool ADAPT = NS == 0;
    constexpr int NSD = ADAPT ? 1 : NS;
    __shared__ T s_rec[kRenderWaves][kWave][GS_REC_WORDS];
    __shared__ uint32_t s_mask[kRenderWaves][kWave];
    const int wave = threadIdx.x / kWave, lane = lane_id();
    int tile, sub;
    uint32_t owned = (1u << PPL) - 1u;
    if (ADAPT) {
        int waves;
        if (!plan_wave(order, frame.n_tiles, blockIdx.x * kRenderWaves + wave, tile, sub, waves)) return;
        owned = owned_quadrants(PPL, waves, sub);
    } else {
        const int gw = xcd_block(blockIdx.x, gridDim.x) * kRenderWaves + wave;
        tile = gw / NSD;
        sub = gw % NSD;
        if (tile >= frame.n_tiles) return;
    }
    const int j = job_of_tile(frame.jobs, frame.n_jobs, tile);
    const gs_job job = frame.jobs[j];
    const gs_camera& cam = frame.cams[job.cam];
    const int W = cam.width, H = cam.height;
    const int lt = tile - job.tile0;
    const int sxn = cfg.tile_w / (8 * QX);   // sub-tiles per tile row
    const int tpx = (lt % job.tiles_x) * cfg.tile_w + (ADAPT ? 0 : (sub % sxn) * 8 * QX);
    const int tpy = (lt / job.tiles_x) * cfg.tile_h + (ADAPT ? 0 : (sub / sxn) * 8 * QY);
    const int lx = lane & 7, ly = lane >> 3;
    // pixel centre of quadrant k: (bx + 8 (k % QX), by + 8 (k / QX))
    const T bx = T(tpx + lx) + T(0.5), by = T(tpy + ly) + T(0.5);

    // per quadrant, the lanes whose pixel has stopped (or lies outside the
    // image or the wavefront's quadrants): a wave-uniform lane mask, so the
    // stop bookkeeping runs on the scalar unit
    T Tr[PPL], C[PPL][3];
    uint64_t stopm[PPL];
    uint32_t last[PPL];
    uint32_t n_kept = 0;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        const int x = tpx + 8 * (k % QX) + lx, y = tpy + 8 * (k / QX) + ly;
        stopm[k] = lane_mask(!(x < W && y < H && (owned & (1u << k))));
        Tr[k] = T(1);
        C[k][0] = C[k][1] = C[k][2] = T(0);
        last[k] = 0;
    }
    const uint2 range = ranges[tile];
    const T amin = T(cfg.alpha_min), amax = T(cfg.alpha_max), tmin = T(cfg.T_min);
    const T lmin = Num<T>::log2(amin);
    for (uint32_t base = range.x; base < range.y; base += kWave) {
        uint64_t all_stopped = ~uint64_t(0);
#pragma unroll
        for (int k = 0; k < PPL; k++) all_stopped &= stopm[k];
        if (all_stopped == ~uint64_t(0)) break;
        const uint32_t cnt = min(uint32_t(kWave), range.y - base);
        // stage the batch's records that reach some quadrant, compacted, each
        // with its quadrant mask and its position in the tile list
        T w[GS_REC_WORDS];
        uint32_t m = 0, r = 0;
        if (uint32_t(lane) < cnt) {
            r = vals[base + lane];
            load_rec(rec, r, w);
            if (ADAPT || NSD == 1) {
                // this wavefront's quadrants are the tile's: its mask is the tile mask
                const uint32_t mt = quad_mask<T, QX, QY>(w, tpx, tpy, lmin);
                if (qmask) qmask[base + lane] = uint8_t(mt);
                m = mt & owned;
            } else {
                m = quad_mask<T, QX, QY>(w, tpx, tpy, lmin) & owned;
                if (qmask) {
                    const int tx0 = (lt % job.tiles_x) * cfg.tile_w, ty0 = (lt / job.tiles_x) * cfg.tile_h;
                    const int nqx = cfg.tile_w / 8;
                    qmask[base + lane] = uint8_t(quad_mask_n(w, tx0, ty0, nqx, nqx * (cfg.tile_h / 8), lmin));
                }
            }
        }
        const uint64_t staged = __ballot(m != 0);
        if (m != 0) {
            const uint32_t slot = __builtin_popcountll(staged & lanemask_lt());
            const T* src = rec + int64_t(r) * GS_REC_WORDS;
            T* dst = s_rec[wave][slot];
#pragma unroll
            for (int q = 0; q < 6; q++) dst[q] = w[q];
#pragma unroll
            for (int q = 6; q < 9; q++) dst[q] = src[q];
            s_mask[wave][slot] = m | (uint32_t(lane) << 8);
        }
        wave_lds_sync();
        const uint32_t n = __builtin_popcountll(staged);
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t word = uniform(s_mask[wave][i]);
            const uint32_t qmask = word & 0xffu, pos = word >> 8;
            const Rec<T> g = lds_rec(s_rec[wave][i]);
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (!(qmask & (1u << k))) continue;   // uniform: box misses quadrant k
                const T dx = quad_centre(bx, k % QX) - g.mx, dy = quad_centre(by, k / QX) - g.my;
                const T al = Num<T>::exp2(log2_alpha(g, dx, dy));
                const uint64_t livem = lane_mask(al >= amin) & ~stopm[k];
                if (livem == 0) continue;     // uniform: no pixel of the wave reached
                const T a = clamp_alpha(al, amax);
                const T aT = a * Tr[k];
                const T tn = Tr[k] - aT;
                const uint64_t stopb = lane_mask(tn < tmin) & livem;
                stopm[k] |= stopb;
                const uint64_t keepm = livem & ~stopb;
                const bool keep = lane_in(keepm);
                const T wgt = keep ? aT : T(0);
                C[k][0] = Num<T>::fma(wgt, g.c[0], C[k][0]);
                C[k][1] = Num<T>::fma(wgt, g.c[1], C[k][1]);
                C[k][2] = Num<T>::fma(wgt, g.c[2], C[k][2]);
                Tr[k] = keep ? tn : Tr[k];
                last[k] = keep ? base - range.x + pos + 1 : last[k];
                if (STATS) n_kept += uint32_t(__builtin_popcountll(keepm));   // uniform: the wave's count
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (STATS && lane == 0) atomicAdd(kept, static_cast<unsigned long long>(n_kept));
    const int64_t plane = int64_t(W) * H;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        const int x = tpx + 8 * (k % QX) + lx, y = tpy + 8 * (k / QX) + ly;
        if (x < W && y < H && (owned & (1u << k))) {
            const int64_t p = job.px0 + int64_t(y) * W + x;
            T* out = rgb + 3 * job.px0 + int64_t(y) * W + x;
            out[0] = C[k][0] + Tr[k] * T(cfg.bg[0]);
            out[plane] = C[k][1] + Tr[k] * T(cfg.bg[1]);
            out[2 * plane] = C[k][2] + Tr[k] * T(cfg.bg[2]);
            Tout[p] = Tr[k];
            ncontrib[p] = last[k];
        }
    }
}

// ---------------------------------------------------------------------------
// backward

template <typename T, int QX, int QY, int NS>
__global__ __launch_bounds__(kWave * kRenderWaves) void k_render_bwd(
    gs_frame frame, gs_raster_cfg cfg, const T* __restrict__ rec, const uint4* __restrict__ meta,
    const uint32_t* __restrict__ pair_off, const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ order, uint64_t capacity, const T* __restrict__ rgb,
    const uint32_t* __restrict__ ncontrib, int mode, const T* __restrict__ gin, T* __restrict__ loss_out,
    T* __restrict__ pg, const uint8_t* __restrict__ qmask) {
    constexpr int PPL = QX * QY;
    // NS wavefronts per tile, wave `sub` owning the tile's sub-tile of QX x QY
    // quadrants and storing its own nine partials per pair (slot e NS + sub);
    // NS = 0: the plan's wavefronts, heavy tiles first, each owning a run of
    // the tile's quadrants (QX x QY is then the tile), partials in the
    // adaptive layout
    constexpr bool ADAPT = NS == 0;
    constexpr int NSD = ADAPT ? 1 : NS;
    __shared__ T s_rec[kRenderWaves][kBwdBatch][GS_REC_WORDS];
    __shared__ uint32_t s_mask[kRenderWaves][kBwdBatch];
    __shared__ uint32_t s_eown[kRenderWaves][kBwdBatch];   // emission index of each staged pair
    const int wave = threadIdx.x / kWave, lane = lane_id();
    int tile = 0, sub = 0, nwaves = NSD;
    uint32_t owned = (1u << PPL) - 1u;
    bool valid = true;   // adaptive: no early return, the workgroup may meet at a barrier below
    // L1 loss, adaptive: the workgroup's wavefronts leave their sums in LDS
    // and the last to arrive adds them per job, one global atomic per job
    // and workgroup instead of one per wavefront (same-address atomics from
    // every wavefront of the launch cost it about a sixth of its time)
    __shared__ T s_loss[kRenderWaves];
    __shared__ int s_ljob[kRenderWaves];
    __shared__ uint32_t s_larrived;
    const bool wg_loss = ADAPT && mode == GS_LOSS_L1 && loss_out != nullptr;
    auto arrive = [&](T l, int jl) {
        if (lane != 0) return;
        s_loss[wave] = l;
        s_ljob[wave] = jl;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (atomicAdd(&s_larrived, 1u) != uint32_t(kRenderWaves - 1)) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int a = 0; a < kRenderWaves; a++) {
            const int ja = s_ljob[a];
            bool first = ja >= 0;
            for (int b = 0; b < a; b++) first = first && s_ljob[b] != ja;
            if (!first) continue;
            T sum = T(0);
            for (int b = a; b < kRenderWaves; b++) sum += s_ljob[b] == ja ? s_loss[b] : T(0);
            atomicAdd(loss_out + ja, sum);
        }
    };
    if (wg_loss) {
        if (threadIdx.x == 0) s_larrived = 0u;
        __syncthreads();
    }
    if (ADAPT) {
        valid = plan_wave(order, frame.n_tiles, blockIdx.x * kRenderWaves + wave, tile, sub, nwaves);
        owned = valid ? owned_quadrants(PPL, nwaves, sub) : 0u;
        if (wg_loss && !valid) arrive(T(0), -1);
    } else {
        const int gw = xcd_block(blockIdx.x, gridDim.x) * kRenderWaves + wave;
        tile = gw / NSD;
        sub = gw % NSD;
        if (tile >= frame.n_tiles) return;
    }
    auto pslot = [&](uint32_t e) {
        return ADAPT ? adaptive_slot(capacity, e, sub) : (int64_t(e) * NSD + sub) * 9;
    };
    do {
    if (!valid) break;
    const int j = job_of_tile(frame.jobs, frame.n_jobs, tile);
    const gs_job job = frame.jobs[j];
    const gs_camera& cam = frame.cams[job.cam];
    const int W = cam.width, H = cam.height;
    const int lt = tile - job.tile0;
    const int tx = lt % job.tiles_x, ty = lt / job.tiles_x;
    const int sxn = cfg.tile_w / (8 * QX);
    const int tpx = tx * cfg.tile_w + (ADAPT ? 0 : (sub % sxn) * 8 * QX);
    const int tpy = ty * cfg.tile_h + (ADAPT ? 0 : (sub / sxn) * 8 * QY);
    const int lx = lane & 7, ly = lane >> 3;
    const T bx = T(tpx + lx) + T(0.5), by = T(tpy + ly) + T(0.5);
    const int64_t plane = int64_t(W) * H;
    const T inv = T(job.loss_weight) / T(3 * plane);

    // per pixel: transmittance, dL/dC, D = sum_c dL/dC_c * C_final_c, the
    // running S = sum_c dL/dC_c * C_accumulated_c, and the forward's count
    // of list entries up to its last contributor (nc): a Gaussian is kept
    // at a pixel exactly when alpha >= alpha_min and its list position is
    // below nc, so the forward's stop rule needs no re-evaluation
    T Tr[PPL], gc[PPL][3], D[PPL], S[PPL];
    uint32_t nc[PPL];
    T loss = T(0);
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        const int x = tpx + 8 * (k % QX) + lx, y = tpy + 8 * (k / QX) + ly;
        const bool in = x < W && y < H && (owned & (1u << k));
        Tr[k] = T(1);
        D[k] = S[k] = T(0);
        gc[k][0] = gc[k][1] = gc[k][2] = T(0);
        nc[k] = 0u;
        if (in) {
            nc[k] = ncontrib[job.px0 + int64_t(y) * W + x];
            const int64_t o = 3 * job.px0 + int64_t(y) * W + x;
#pragma unroll
            for (int ch = 0; ch < 3; ch++) {
                const T c = rgb[o + ch * plane];
                T g;
                if (mode == GS_LOSS_L1) {
                    const T d = c - gin[o + ch * plane];
                    g = d > T(0) ? inv : (d < T(0) ? -inv : T(0));
                    loss += (d < T(0) ? -d : d) * inv;
                } else {
                    g = gin[o + ch * plane];
                }
                gc[k][ch] = g;
                D[k] = Num<T>::fma(g, c, D[k]);
            }
        }
    }
    if (mode == GS_LOSS_L1 && loss_out) {
        const T l = wave_sum(loss);
        if (wg_loss) arrive(l, j);
        else if (lane == 0) atomicAdd(loss_out + j, l);
    }

    const uint2 range = ranges[tile];
    const T amin = T(cfg.alpha_min), amax = T(cfg.alpha_max);
    const T lmin = Num<T>::log2(amin);
    // per quadrant, the list entries any of its pixels still needs
    uint32_t qend[PPL];
    uint32_t wend = 0u;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        qend[k] = uniform(wave_max_u32(nc[k]));
        wend = qend[k] > wend ? qend[k] : wend;
    }
    for (uint32_t base = range.x; base < range.y; base += kBwdBatch) {
        const uint32_t cnt = min(uint32_t(kBwdBatch), range.y - base);
        const uint32_t pos0 = base - range.x;   // list position of the batch's first entry
        uint32_t e_own = 0;   // pair this lane stores at the end of the batch
        T w[GS_REC_WORDS];
        uint32_t m = 0, r = 0;
        if (uint32_t(lane) < cnt) {
            r = vals[base + lane];
            const uint32_t pos = pos0 + uint32_t(lane);
            if (pos < wend) {
                load_rec(rec, r, w);
                if (qmask == nullptr) {
                    m = quad_mask<T, QX, QY>(w, tpx, tpy, lmin);
                } else if (ADAPT || NSD == 1) {
                    m = qmask[base + lane];   // the forward's tile mask: this wavefront's quadrants are the tile's
                } else {
                    // the forward's tile mask, bits of this wavefront's sub-tile
                    const uint32_t mt = qmask[base + lane];
                    const int nqx = cfg.tile_w / 8, qx0 = (sub % sxn) * QX, qy0 = (sub / sxn) * QY;
                    m = 0;
#pragma unroll
                    for (int k = 0; k < PPL; k++)
                        m |= ((mt >> ((qy0 + k / QX) * nqx + qx0 + k % QX)) & 1u) << k;
                }
                m &= owned;
#pragma unroll
                for (int k = 0; k < PPL; k++) m &= pos < qend[k] ? ~0u : ~(1u << k);
            }
            // emission index of pair (this tile, r): the record's pairs run
            // row by row over its tile rectangle
            const uint4 mt = meta[r];
            const uint32_t x0 = mt.z & 0xffffu, y0 = mt.z >> 16, x1 = mt.w & 0xffffu;
            e_own = pair_off[r] + (uint32_t(ty) - y0) * (x1 - x0 + 1) + (uint32_t(tx) - x0);
        }
        if (pos0 >= wend) {
            // past every pixel's last contributor: the rest of the tile's
            // pairs carry zero gradient
            if (uint32_t(lane) < cnt)
#pragma unroll
                for (int q = 0; q < 9; q++) pg[pslot(e_own) + q] = T(0);
            continue;
        }
        // records that reach some quadrant are staged compacted, with their
        // list position; the others store zero partials below
        const uint64_t staged = __ballot(m != 0);
        const uint32_t slot = __builtin_popcountll(staged & lanemask_lt());
        if (m != 0) {
            const T* src = rec + int64_t(r) * GS_REC_WORDS;
            T* dst = s_rec[wave][slot];
#pragma unroll
            for (int q = 0; q < 6; q++) dst[q] = w[q];
#pragma unroll
            for (int q = 6; q < 9; q++) dst[q] = src[q];
            narrow_axis(w[R_AXIS], dst[S_AXC], dst[S_AXS]);
            s_mask[wave][slot] = m | (uint32_t(lane) << 8);
            s_eown[wave][slot] = e_own;
        } else if (uint32_t(lane) < cnt) {
            // reaches no quadrant this wave owns: zero partials
#pragma unroll
            for (int q = 0; q < 9; q++) pg[pslot(e_own) + q] = T(0);
        }
        wave_lds_sync();
        const uint32_t n = __builtin_popcountll(staged);
        // composites staged record i over the wave's quadrants, leaves its nine
        // partials (per lane) in v; false when no pixel kept it
        auto composite = [&](uint32_t i, T (&v)[9]) -> bool {
            const uint32_t word = uniform(s_mask[wave][i]);
            const uint32_t qmask = word & 0xffu, pos = pos0 + (word >> 8);
            const Rec<T> g = lds_rec(s_rec[wave][i]);
            const T axc = s_rec[wave][i][S_AXC], axs = s_rec[wave][i][S_AXS];
#pragma unroll
            for (int q = 0; q < 9; q++) v[q] = -T(0);   // -0: the first x + v folds to x
            T* mo = v;
            T* dcol = v + 6;
            bool hit = false;   // uniform: some lane kept the record
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (!(qmask & (1u << k))) continue;   // uniform: box misses quadrant k
                const T dx = quad_centre(bx, k % QX) - g.mx, dy = quad_centre(by, k / QX) - g.my;
                const T al = Num<T>::exp2(log2_alpha(g, dx, dy));
                const bool keep = al >= amin && pos < nc[k];
                if (__ballot(keep) == 0) continue;     // uniform: no pixel of the wave keeps it
                hit = true;
                // the forward's operations on the kept pixels; zeros elsewhere
                const T a = clamp_alpha(al, amax);
                const T ak = keep ? a : T(0);
                const T wgt = ak * Tr[k];
                const T gcc = Num<T>::fma(gc[k][2], g.c[2], Num<T>::fma(gc[k][1], g.c[1], gc[k][0] * g.c[0]));
                S[k] = Num<T>::fma(wgt, gcc, S[k]);
                // dL/dalpha = sum_c gc_c (c_c T - (C_final_c - C_acc_c) / (1 - alpha))
                const T ga = Num<T>::fma(Tr[k], gcc, -(D[k] - S[k]) * recip(T(1) - a));
#pragma unroll
                for (int ch = 0; ch < 3; ch++) dcol[ch] = Num<T>::fma(gc[k][ch], wgt, dcol[ch]);
                Tr[k] -= wgt;
                // alpha clamped at alpha_max: no gradient to the Gaussian's shape
                const T ge = (al < amax ? ak : T(0)) * ga;
                const T e1 = Num<T>::fma(axc, dx, axs * dy), e2 = Num<T>::fma(axc, dy, -(axs * dx));
                const T t1 = ge * e1, t2 = ge * e2;
                mo[0] += ge;
                mo[1] += t1;
                mo[2] += t2;
                mo[3] = Num<T>::fma(t1, e1, mo[3]);
                mo[4] = Num<T>::fma(t1, e2, mo[4]);
                mo[5] = Num<T>::fma(t2, e2, mo[5]);
            }
            return hit;
        };
        // records in pairs: composited in list order, their partials summed
        // over the wave together and stored
        for (uint32_t i = 0; i < n; i += 2) {
            T va[9], vb[9];
            const bool ha = composite(i, va);
            bool hb = false;
            if (i + 1 < n) {
                hb = composite(i + 1, vb);
            } else {
#pragma unroll
                for (int q = 0; q < 9; q++) vb[q] = T(0);
            }
            T* da = pg + pslot(uniform(s_eown[wave][i]));
            T* db = i + 1 < n ? pg + pslot(uniform(s_eown[wave][i + 1])) : nullptr;
            if (ha || hb) {
                store_pair_partials(va, vb, da, db);
            } else if (lane < 9) {
                da[lane] = T(0);
                if (db) db[lane] = T(0);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    } while (0);

    // Adaptive: a split tile's wavefronts share this workgroup.  Once all of
    // them have stored their partials, fold each pair's further slots into
    // slot 0 (slot 0 + 1 + 2 + 3, in that order), so the projection backward
    // reads one dense slot per pair.  Whether a workgroup holds a split tile
    // is the same for all its wavefronts (the plan puts split tiles first),
    // and none of them has left the kernel.
    if (ADAPT) {
        const uint64_t split_waves = 4ull * order[0] + 2ull * order[1];
        if (4ull * blockIdx.x < split_waves) {
            __syncthreads();
            if (valid && nwaves > 1) {
                const int jf = job_of_tile(frame.jobs, frame.n_jobs, tile);
                const gs_job jb = frame.jobs[jf];
                const int ltf = tile - jb.tile0;
                const uint32_t ftx = uint32_t(ltf % jb.tiles_x), fty = uint32_t(ltf / jb.tiles_x);
                const uint2 rg = ranges[tile];
                for (uint32_t i = rg.x + uint32_t(sub * kWave + lane); i < rg.y; i += uint32_t(nwaves * kWave)) {
                    const uint32_t r = vals[i];
                    const uint4 mt = meta[r];
                    const uint32_t x0 = mt.z & 0xffffu, y0 = mt.z >> 16, x1 = mt.w & 0xffffu;
                    const uint32_t e = pair_off[r] + (fty - y0) * (x1 - x0 + 1) + (ftx - x0);
                    T* d0 = pg + adaptive_slot(capacity, e, 0);
                    T acc[9];
#pragma unroll
                    for (int q = 0; q < 9; q++) acc[q] = d0[q];
                    for (int sl = 1; sl < nwaves; sl++) {
                        const T* src = pg + adaptive_slot(capacity, e, sl);
#pragma unroll
                        for (int q = 0; q < 9; q++) acc[q] += src[q];
                    }
#pragma unroll
                    for (int q = 0; q < 9; q++) d0[q] = acc[q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------

// grid of a compositing launch: NS (or 4, adaptive) wavefronts per tile, in
// workgroups of kRenderWaves wavefronts (1, adaptive)
template <int NS>
static void compositing_grid(const gs_frame& f, dim3& grid, dim3& block) {
    const int wpt = NS == 0 ? 4 : NS;   // adaptive: at most 4 per tile, the plan's count
    grid = dim3(unsigned((int64_t(f.n_tiles) * wpt + kRenderWaves - 1) / kRenderWaves));
    block = dim3(unsigned(kWave * kRenderWaves));
}

template <typename T, int QX, int QY, int NS>
static void fwd_launch(const gs_frame& f, const gs_raster_cfg& cfg, const T* rec, const gs_bins& b, T* rgb,
                       T* Tfin, uint32_t* nc, unsigned long long* kept, hipStream_t s) {
    dim3 grid, block;
    compositing_grid<NS>(f, grid, block);
    if (kept)
        GS_LAUNCH("k_render_fwd", (k_render_fwd<T, QX, QY, NS, true>), grid, block, 0, s, f, cfg, rec, b.vals,
                  reinterpret_cast<const uint2*>(b.ranges), rgb, Tfin, nc, kept, b.tile_order, b.qmask);
    else
        GS_LAUNCH("k_render_fwd", (k_render_fwd<T, QX, QY, NS, false>), grid, block, 0, s, f, cfg, rec, b.vals,
                  reinterpret_cast<const uint2*>(b.ranges), rgb, Tfin, nc, kept, b.tile_order, b.qmask);
}

template <typename T, int QX, int QY, int NS>
static void bwd_launch(const gs_frame& f, const gs_raster_cfg& cfg, const T* rec, const uint32_t* meta,
                       const gs_bins& b, const T* rgb, const uint32_t* nc, int mode, const T* gin, T* loss, T* pg,
                       hipStream_t s) {
    dim3 grid, block;
    compositing_grid<NS>(f, grid, block);
    GS_LAUNCH("k_render_bwd", (k_render_bwd<T, QX, QY, NS>), grid, block, 0, s, f, cfg, rec,
              reinterpret_cast<const uint4*>(meta), b.pair_off, b.vals, reinterpret_cast<const uint2*>(b.ranges),
              b.tile_order, b.capacity, rgb, nc, mode, gin, loss, pg, b.qmask);
}

// (binning tile, wavefronts per tile) -> quadrants per wavefront QX x QY:
// 8x8/1 = 1x1; 16x8/1 = 2x1, /2 = 1x1; 16x16/1 = 2x2, /2 = 2x1 (halves stacked),
// /4 = 1x1; 32x8/1 = 4x1, /2 = 2x1 (halves side by side), /4 = 1x1.  Adaptive
// (WAVES = 0): the whole tile's quadrants, split per tile at run time.
#define GS_TILE_DISPATCH(WAVES, FN, ...)                                                  \
    do {                                                                                  \
        const int S_ = WAVES;                                                             \
        if (cfg.tile_w == 8 && cfg.tile_h == 8) {                                         \
            if (S_ == 0) FN<T, 1, 1, 0>(__VA_ARGS__);                                     \
            else FN<T, 1, 1, 1>(__VA_ARGS__);                                             \
        } else if (cfg.tile_w == 16 && cfg.tile_h == 8) {                                 \
            if (S_ == 0) FN<T, 2, 1, 0>(__VA_ARGS__);                                     \
            else if (S_ == 2) FN<T, 1, 1, 2>(__VA_ARGS__);                                \
            else FN<T, 2, 1, 1>(__VA_ARGS__);                                             \
        } else if (cfg.tile_w == 32 && cfg.tile_h == 8) {                                 \
            if (S_ == 0) FN<T, 4, 1, 0>(__VA_ARGS__);                                     \
            else if (S_ == 4) FN<T, 1, 1, 4>(__VA_ARGS__);                                \
            else if (S_ == 2) FN<T, 2, 1, 2>(__VA_ARGS__);                                \
            else FN<T, 4, 1, 1>(__VA_ARGS__);                                             \
        } else {                                                                          \
            if (S_ == 0) FN<T, 2, 2, 0>(__VA_ARGS__);                                     \
            else if (S_ == 4) FN<T, 1, 1, 4>(__VA_ARGS__);                                \
            else if (S_ == 2) FN<T, 2, 1, 2>(__VA_ARGS__);                                \
            else FN<T, 2, 2, 1>(__VA_ARGS__);                                             \
        }                                                                                 \
    } while (0)

template <typename T>
hipError_t launch_render_fwd(const gs_frame& f, const gs_raster_cfg& cfg, const T* rec, const gs_bins& bins,
                             T* rgb, T* Tfin, uint32_t* ncontrib, unsigned long long* kept, hipStream_t s) {
    if (f.n_tiles == 0) return hipSuccess;
    GS_TILE_DISPATCH(fwd_waves(cfg), fwd_launch, f, cfg, rec, bins, rgb, Tfin, ncontrib, kept, s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_render_bwd(const gs_frame& f, const gs_raster_cfg& cfg, const T* rec, const uint32_t* meta,
                             const gs_bins& bins, const T* rgb, const uint32_t* nc, gs_loss_mode mode, const T* gin,
                             T* loss, T* pg, hipStream_t s) {
    if (f.n_tiles == 0) return hipSuccess;
    GS_TILE_DISPATCH(bwd_waves(cfg), bwd_launch, f, cfg, rec, meta, bins, rgb, nc, int(mode), gin, loss, pg, s);
    return hipGetLastError();
}

template hipError_t launch_render_fwd<float>(const gs_frame&, const gs_raster_cfg&, const float*, const gs_bins&, float*, float*, uint32_t*, unsigned long long*, hipStream_t);
template hipError_t launch_render_fwd<double>(const gs_frame&, const gs_raster_cfg&, const double*, const gs_bins&, double*, double*, uint32_t*, unsigned long long*, hipStream_t);
template hipError_t launch_render_bwd<float>(const gs_frame&, const gs_raster_cfg&, const float*, const uint32_t*, const gs_bins&, const float*, const uint32_t*, gs_loss_mode, const float*, float*, float*, hipStream_t);
template hipError_t launch_render_bwd<double>(const gs_frame&, const gs_raster_cfg&, const double*, const uint32_t*, const gs_bins&, const double*, const uint32_t*, gs_loss_mode, const double*, double*, double*, hipStream_t);

}  // namespace gs
