// Projection of 3D Gaussians into each job's view (forward) and the chain
// rule from per-record screen-space gradients back to the raw parameter
// planes (backward).  One thread per (job, Gaussian) record forward and one
// thread per Gaussian backward; both stream the SoA planes coalesced.
//
// Paper: Sec. 3.1 (Eq. 1: Gaussian with Sigma = R S S^T R^T; Eq. 2 and
// alpha = o X^proj(p); attributes x = {u, q, s, f, o}).  X^proj is read as the
// EWA local-affine projection (Sigma' = J W Sigma W^T J^T + dilation I).
#include "adam.hpp"
#include "gs_device.hpp"
#include "gs_internal.hpp"

namespace gs {

template <typename T>
struct Cam {
    T R[9], t[3], fx, fy, cx, cy;
    int W, H;
};

template <typename T>
__device__ inline void load_cam(const gs_camera& c, Cam<T>& o) {
#pragma unroll
    for (int k = 0; k < 9; k++) o.R[k] = T(c.R[k]);
#pragma unroll
    for (int k = 0; k < 3; k++) o.t[k] = T(c.t[k]);
    o.fx = T(c.fx); o.fy = T(c.fy); o.cx = T(c.cx); o.cy = T(c.cy);
    o.W = c.width; o.H = c.height;
}

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 as polynomials in the unit
// direction (x, y, z): orthonormal, Condon-Shortley phase, index
// k = l*l + l + m with m = -l..l.  The constants are
//   c1 = sqrt(3/(4pi)), c2a = sqrt(15/(4pi)), c2b = sqrt(5/(16pi)),
//   c2c = sqrt(15/(16pi)), c3a = sqrt(35/(32pi)), c3b = sqrt(105/(4pi)),
//   c3c = sqrt(21/(32pi)), c3d = sqrt(7/(16pi)), c3e = sqrt(105/(16pi)).
template <typename T>
struct SH {
    static constexpr double c0 = 0.28209479177387814, c1 = 0.48860251190291992;
    static constexpr double c2a = 1.0925484305920792, c2b = 0.31539156525252005, c2c = 0.54627421529603959;
    static constexpr double c3a = 0.59004358992664352, c3b = 2.8906114426405538, c3c = 0.45704579946446572;
    static constexpr double c3d = 0.37317633259011540, c3e = 1.4453057213202769;

    template <int D>
    __device__ static inline void basis(T x, T y, T z, T* Y) {
        Y[0] = T(c0);
        if (D >= 1) { Y[1] = -T(c1) * y; Y[2] = T(c1) * z; Y[3] = -T(c1) * x; }
        if (D >= 2) {
            const T xx = x * x, yy = y * y, zz = z * z;
            Y[4] = T(c2a) * x * y;
            Y[5] = -T(c2a) * y * z;
            Y[6] = T(c2b) * (T(2) * zz - xx - yy);
            Y[7] = -T(c2a) * x * z;
            Y[8] = T(c2c) * (xx - yy);
            if (D >= 3) {
                Y[9] = -T(c3a) * y * (T(3) * xx - yy);
                Y[10] = T(c3b) * x * y * z;
                Y[11] = -T(c3c) * y * (T(4) * zz - xx - yy);
                Y[12] = T(c3d) * z * (T(2) * zz - T(3) * xx - T(3) * yy);
                Y[13] = -T(c3c) * x * (T(4) * zz - xx - yy);
                Y[14] = T(c3e) * z * (xx - yy);
                Y[15] = -T(c3a) * x * (xx - T(3) * yy);
            }
        }
    }

    // d = sum_k w[k] grad Y_k(x, y, z)
    template <int D>
    __device__ static inline void grad_dot(T x, T y, T z, const T* w, T* d) {
        T gx = 0, gy = 0, gz = 0;
        if (D >= 1) { gy -= T(c1) * w[1]; gz += T(c1) * w[2]; gx -= T(c1) * w[3]; }
        if (D >= 2) {
            gx += T(c2a) * y * w[4];            gy += T(c2a) * x * w[4];
            gy -= T(c2a) * z * w[5];            gz -= T(c2a) * y * w[5];
            gx -= T(2 * c2b) * x * w[6];        gy -= T(2 * c2b) * y * w[6];   gz += T(4 * c2b) * z * w[6];
            gx -= T(c2a) * z * w[7];            gz -= T(c2a) * x * w[7];
            gx += T(2 * c2c) * x * w[8];        gy -= T(2 * c2c) * y * w[8];
            if (D >= 3) {
                const T xx = x * x, yy = y * y, zz = z * z;
                gx -= T(6 * c3a) * x * y * w[9];
                gy -= T(3 * c3a) * (xx - yy) * w[9];
                gx += T(c3b) * y * z * w[10]; gy += T(c3b) * x * z * w[10]; gz += T(c3b) * x * y * w[10];
                gx += T(2 * c3c) * x * y * w[11];
                gy -= T(c3c) * (T(4) * zz - xx - T(3) * yy) * w[11];
                gz -= T(8 * c3c) * y * z * w[11];
                gx -= T(6 * c3d) * x * z * w[12];
                gy -= T(6 * c3d) * y * z * w[12];
                gz += T(3 * c3d) * (T(2) * zz - xx - yy) * w[12];
                gx -= T(c3c) * (T(4) * zz - T(3) * xx - yy) * w[13];
                gy += T(2 * c3c) * x * y * w[13];
                gz -= T(8 * c3c) * x * z * w[13];
                gx += T(2 * c3e) * x * z * w[14]; gy -= T(2 * c3e) * y * z * w[14]; gz += T(c3e) * (xx - yy) * w[14];
                gx -= T(3 * c3a) * (xx - yy) * w[15];
                gy += T(6 * c3a) * x * y * w[15];
            }
        }
        d[0] = gx; d[1] = gy; d[2] = gz;
    }
};

// ---------------------------------------------------------------------------
// Geometry of one Gaussian in one view.

template <typename T>
struct Geo {
    T u[3];          // mean
    T t[3];          // camera-space mean
    T rz;            // 1 / t_z
    T rx, ry;        // clamped x/z, y/z
    bool clx, cly;   // clamp active
    T qn[4], qinv;   // normalised quaternion, 1/|q|
    T R[9];          // rotation of the Gaussian
    T s[3];          // scales
    T Sig[6];        // xx xy xz yy yz zz
    T t0[3], t1[3];  // rows of J W
    T sxx, sxy, syy; // screen covariance (incl. dilation)
    T a, b, c;       // conic
    T mx, my;
    T o;             // opacity
};

template <typename T>
__device__ inline T plane(const T* __restrict__ P, int64_t stride, int a, int64_t g) {
    return P[int64_t(a) * stride + g];
}

// v * 0 is 0 for finite v and NaN for NaN or +-Inf: a sum of such products
// stays 0 exactly while every value added is finite
template <typename T>
__device__ inline void finite_acc(T& acc, T v) { acc += v * T(0); }

// Returns false when culled by the near plane or the opacity threshold.
// fin (may be null): every parameter value read is added as v * 0.
template <typename T>
__device__ inline bool geometry(const T* __restrict__ P, int64_t stride, int64_t g, const Cam<T>& cam,
                                const gs_raster_cfg& cfg, Geo<T>& G, T* fin = nullptr) {
    using N = Num<T>;
#pragma unroll
    for (int k = 0; k < 3; k++) G.u[k] = plane(P, stride, k, g);
    if (fin)
#pragma unroll
        for (int k = 0; k < 3; k++) finite_acc(*fin, G.u[k]);
#pragma unroll
    for (int r = 0; r < 3; r++)
        G.t[r] = cam.R[3 * r] * G.u[0] + cam.R[3 * r + 1] * G.u[1] + cam.R[3 * r + 2] * G.u[2] + cam.t[r];
    if (!(G.t[2] > T(cfg.near_z))) return false;
    const T logit = plane(P, stride, 10, g);
    if (fin) finite_acc(*fin, logit);
    G.o = N::rcp(T(1) + N::exp(-logit));
    if (G.o < T(cfg.alpha_min)) return false;

    T q[4];
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = plane(P, stride, 3 + k, g);
    if (fin)
#pragma unroll
        for (int k = 0; k < 4; k++) finite_acc(*fin, q[k]);
    G.qinv = N::rsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
    for (int k = 0; k < 4; k++) G.qn[k] = q[k] * G.qinv;
    const T w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
    G.R[0] = T(1) - T(2) * (y * y + z * z); G.R[1] = T(2) * (x * y - w * z); G.R[2] = T(2) * (x * z + w * y);
    G.R[3] = T(2) * (x * y + w * z); G.R[4] = T(1) - T(2) * (x * x + z * z); G.R[5] = T(2) * (y * z - w * x);
    G.R[6] = T(2) * (x * z - w * y); G.R[7] = T(2) * (y * z + w * x); G.R[8] = T(1) - T(2) * (x * x + y * y);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const T ls = plane(P, stride, 7 + k, g);
        if (fin) finite_acc(*fin, ls);
        G.s[k] = N::exp(ls);
    }
    // Sigma = R diag(s^2) R^T
    T M[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) M[3 * r + c] = G.R[3 * r + c] * G.s[c];
    G.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    G.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    G.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    G.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    G.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    G.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];

    // Jacobian of the perspective map at the (clamped) mean
    G.rz = N::rcp(G.t[2]);
    const T limx = T(cfg.jac_clip) * T(0.5) * T(cam.W) * N::rcp(cam.fx);
    const T limy = T(cfg.jac_clip) * T(0.5) * T(cam.H) * N::rcp(cam.fy);
    const T ux = G.t[0] * G.rz, uy = G.t[1] * G.rz;
    G.clx = (ux < -limx) || (ux > limx);
    G.cly = (uy < -limy) || (uy > limy);
    G.rx = ux < -limx ? -limx : (ux > limx ? limx : ux);
    G.ry = uy < -limy ? -limy : (uy > limy ? limy : uy);
    const T J00 = cam.fx * G.rz, J02 = -cam.fx * G.rx * G.rz;
    const T J11 = cam.fy * G.rz, J12 = -cam.fy * G.ry * G.rz;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        G.t0[k] = J00 * cam.R[k] + J02 * cam.R[6 + k];
        G.t1[k] = J11 * cam.R[3 + k] + J12 * cam.R[6 + k];
    }
    // screen covariance t_i^T Sigma t_j
    T St0[3], St1[3];
    St0[0] = G.Sig[0] * G.t0[0] + G.Sig[1] * G.t0[1] + G.Sig[2] * G.t0[2];
    St0[1] = G.Sig[1] * G.t0[0] + G.Sig[3] * G.t0[1] + G.Sig[4] * G.t0[2];
    St0[2] = G.Sig[2] * G.t0[0] + G.Sig[4] * G.t0[1] + G.Sig[5] * G.t0[2];
    St1[0] = G.Sig[0] * G.t1[0] + G.Sig[1] * G.t1[1] + G.Sig[2] * G.t1[2];
    St1[1] = G.Sig[1] * G.t1[0] + G.Sig[3] * G.t1[1] + G.Sig[4] * G.t1[2];
    St1[2] = G.Sig[2] * G.t1[0] + G.Sig[4] * G.t1[1] + G.Sig[5] * G.t1[2];
    G.sxx = G.t0[0] * St0[0] + G.t0[1] * St0[1] + G.t0[2] * St0[2] + T(cfg.dilation);
    G.sxy = G.t0[0] * St1[0] + G.t0[1] * St1[1] + G.t0[2] * St1[2];
    G.syy = G.t1[0] * St1[0] + G.t1[1] * St1[1] + G.t1[2] * St1[2] + T(cfg.dilation);
    const T rdet = N::rcp(G.sxx * G.syy - G.sxy * G.sxy);
    G.a = G.syy * rdet;
    G.b = -G.sxy * rdet;
    G.c = G.sxx * rdet;
    G.mx = cam.fx * G.t[0] * G.rz + cam.cx;
    G.my = cam.fy * G.t[1] * G.rz + cam.cy;
    return true;
}

// view direction from the camera centre c = -R^T t to the mean
template <typename T>
__device__ inline T view_dir(const Geo<T>& G, const Cam<T>& cam, T* dir) {
    T v[3];
#pragma unroll
    for (int k = 0; k < 3; k++)
        v[k] = G.u[k] + (cam.R[k] * cam.t[0] + cam.R[3 + k] * cam.t[1] + cam.R[6 + k] * cam.t[2]);
    const T vinv = Num<T>::rsqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
    for (int k = 0; k < 3; k++) dir[k] = v[k] * vinv;
    return vinv;
}

// ---------------------------------------------------------------------------
// forward

// status (may be null): GS_STATUS_NONFINITE is OR-ed in when a parameter value
// the projection reads is NaN or Inf (the mean of every Gaussian; the rest
// of those that pass the near plane; the SH planes of those on screen)
template <typename T>
__device__ inline void flag_nonfinite(uint32_t* status, T fin) {
    if (status && !(fin == T(0))) atomicOr(status, GS_STATUS_NONFINITE);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_project(const T* __restrict__ P, int64_t stride, gs_frame frame,
                                                  gs_raster_cfg cfg, T* __restrict__ rec,
                                                  uint4* __restrict__ meta, uint32_t* __restrict__ status) {
    constexpr int NK = (D + 1) * (D + 1);
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= frame.n_records) return;
    const int j = job_of_record(frame.jobs, frame.n_jobs, r);
    const gs_job job = frame.jobs[j];
    const int64_t g = job.g0 + (r - job.rec0);
    Cam<T> cam;
    load_cam(frame.cams[job.cam], cam);
    Geo<T> G;
    uint4 m = make_uint4(0xffffffffu, 0u, 0u, 0u);
    T fin = T(0);
    if (!geometry(P, stride, g, cam, cfg, G, &fin)) {
        meta[r] = m;
        flag_nonfinite(status, fin);
        return;
    }

    // conservative pixel rectangle of {alpha >= alpha_min}: the ellipse
    // d^T A d <= 2 ln(o / alpha_min) has half-extents sqrt(thr * Sigma'_xx), ...
    using N = Num<T>;
    const T thr = T(2) * N::log(G.o / T(cfg.alpha_min));
    const T hx = N::sqrt(thr * G.sxx) * T(1.0001) + T(0.01);
    const T hy = N::sqrt(thr * G.syy) * T(1.0001) + T(0.01);
    T x0 = ceil(G.mx - hx - T(0.5)), x1 = floor(G.mx + hx - T(0.5));
    T y0 = ceil(G.my - hy - T(0.5)), y1 = floor(G.my + hy - T(0.5));
    x0 = x0 < T(0) ? T(0) : x0;
    y0 = y0 < T(0) ? T(0) : y0;
    x1 = x1 > T(cam.W - 1) ? T(cam.W - 1) : x1;
    y1 = y1 > T(cam.H - 1) ? T(cam.H - 1) : y1;
    if (!(x0 <= x1 && y0 <= y1)) {
        meta[r] = m;
        flag_nonfinite(status, fin);
        return;
    }
    const int tx0 = int(x0) / cfg.tile_w, tx1 = int(x1) / cfg.tile_w;
    const int ty0 = int(y0) / cfg.tile_h, ty1 = int(y1) / cfg.tile_h;

    // colour from the SH coefficients at the view direction (read with the
    // non-temporal hint: 48 of the 59 planes, not needed again until the
    // optimiser, so they leave the cache to the geometry planes and records)
    T dir[3];
    view_dir(G, cam, dir);
    T Y[16];
    SH<T>::template basis<D>(dir[0], dir[1], dir[2], Y);
    T col[3];
    uint32_t clamp = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < NK; k++) {
            const T f = __builtin_nontemporal_load(P + int64_t(11 + 3 * k + ch) * stride + g);
            finite_acc(fin, f);
            s += Y[k] * f;
        }
        s += T(0.5);
        col[ch] = s > T(0) ? s : T(0);
        clamp |= s > T(0) ? 0u : (1u << ch);
    }

    T* o = rec + r * GS_REC_WORDS;
    o[0] = G.mx;
    o[1] = G.my;
    o[2] = T(-0.5) * kLog2e<T>() * G.a;
    o[3] = -kLog2e<T>() * G.b;
    o[4] = T(-0.5) * kLog2e<T>() * G.c;
    o[5] = N::log2(G.o);
    o[6] = col[0];
    o[7] = col[1];
    o[8] = col[2];
    o[9] = narrow_axis_code(G.a, G.b, G.c);   // frame of the backward's moments
    o[10] = hx;   // conservative half-extents of {alpha >= alpha_min} in pixels
    o[11] = hy;
    m.x = __float_as_uint(float(G.t[2]));
    m.y = uint32_t((tx1 - tx0 + 1) * (ty1 - ty0 + 1)) | (clamp << 24);
    m.z = uint32_t(tx0) | (uint32_t(ty0) << 16);
    m.w = uint32_t(tx1) | (uint32_t(ty1) << 16);
    meta[r] = m;
    flag_nonfinite(status, fin);
}

// ---------------------------------------------------------------------------
// backward: sum each record's per-pair partials, then apply the chain rule
// through the projection to every raw parameter plane.

// Per lane: the 9 partials of its record, the sum of its np pairs starting at
// p0.  A lane sums a small record itself; the wave sums a large one together
// (strided partial sums, then a fixed reduction tree), so a Gaussian spanning
// thousands of tiles does not serialise one lane.  Every lane of the wave
// must call this (cross-lane reductions).
template <typename T>
__device__ inline void record_pair_sum(const T* __restrict__ pg, uint64_t p0, uint64_t np, T* d) {
    constexpr uint64_t kCoop = 24;
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < 9; i++) d[i] = T(0);
    const bool big = np > kCoop;
    if (!big) {
        // four pairs per round trip: their loads are issued before any is
        // added; past the last pair a lane reloads its last pair (in bounds)
        // and adds -0 instead, which leaves every sum unchanged, so the sums
        // are the one-pair-at-a-time sums bit for bit
        const T* src = pg + int64_t(p0) * 9;
        for (uint64_t k = 0; k < np; k += 4) {
            T t[4][9];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const bool in = k + j < np;
                const T* sj = src + (in ? k + j : np - 1) * 9;
#pragma unroll
                for (int i = 0; i < 9; i++) t[j][i] = sj[i];
#pragma unroll
                for (int i = 0; i < 9; i++) t[j][i] = in ? t[j][i] : -T(0);
            }
#pragma unroll
            for (int j = 0; j < 4; j++)
#pragma unroll
                for (int i = 0; i < 9; i++) d[i] += t[j][i];
        }
    }
    uint64_t bigmask = __ballot(big);
    while (bigmask) {
        const int src_lane = __ffsll((long long)bigmask) - 1;
        bigmask &= bigmask - 1;
        const uint64_t bp0 = __shfl(p0, src_lane, kWave), bnp = __shfl(np, src_lane, kWave);
        T part[9];
#pragma unroll
        for (int i = 0; i < 9; i++) part[i] = T(0);
        // four strided pairs per lane and round trip, added in the order of
        // the one-at-a-time loop (past the end: the lane's first pair
        // reloaded, -0 added)
        const T* src = pg + int64_t(bp0) * 9;
        for (uint64_t k0 = lane; k0 < bnp; k0 += 4 * kWave) {
            T t[4][9];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint64_t k = k0 + uint64_t(j) * kWave;
                const bool in = k < bnp;
                const T* sj = src + (in ? k : k0) * 9;
#pragma unroll
                for (int i = 0; i < 9; i++) t[j][i] = sj[i];
#pragma unroll
                for (int i = 0; i < 9; i++) t[j][i] = in ? t[j][i] : -T(0);
            }
#pragma unroll
            for (int j = 0; j < 4; j++)
#pragma unroll
                for (int i = 0; i < 9; i++) part[i] += t[j][i];
        }
#pragma unroll
        for (int i = 0; i < 9; i++) {
            const T t = wave_sum(part[i]);
            if (lane == src_lane) d[i] = t;
        }
    }
}

// emitted pairs of a record (pairs past the capacity never were: the
// overflow status is set and the step must be redone)
__device__ inline void record_pairs(uint32_t ntiles, uint32_t off, uint64_t capacity, uint64_t& p0,
                                    uint64_t& np) {
    p0 = off;
    np = ntiles == 0 || p0 >= capacity ? 0 : (p0 + ntiles > capacity ? capacity - p0 : ntiles);
}

// Where the compositing backward left a pair's partials: `slots` consecutive
// slots per pair, one per wavefront of its tile (one when the wavefronts were
// adaptive: split tiles fold theirs into the first).
struct PartialLayout {
    int slots;
};

// Per lane: the 9 partials of its record summed over its pairs' slots (pair,
// then slot, ascending; large records cooperatively).  Every lane of the wave
// must call this.
template <typename T>
__device__ inline void record_partials(const T* __restrict__ pg, const PartialLayout& L, const uint4& m,
                                       uint32_t off, uint64_t capacity, T* d) {
    uint64_t p0, np;
    record_pairs(meta_tiles(m.y), off, capacity, p0, np);
    record_pair_sum(pg, p0 * uint64_t(L.slots), np * uint64_t(L.slots), d);
}

// Chain rule of one visible record of Gaussian g seen by `camera`; emit(a, v)
// receives the gradient v of parameter plane a.  Plane a of Gaussian g is
// read (if at all) before emit(a, .) is called and never after, so emit may
// update the parameter in place.
// With sh_basis_out / sh_dc_out, also hands out the SH basis values Y[k] and
// the clamped colour gradient dc[ch], whose products are the SH-plane
// gradients.
template <typename T, int D, typename Emit>
__device__ inline void record_chain(const T* P, int64_t stride, int64_t g, const gs_camera& camera,
                                    const gs_raster_cfg& cfg, uint32_t meta_y, const T* d, T axis, Emit emit,
                                    T* sh_basis_out = nullptr, T* sh_dc_out = nullptr) {
    constexpr int NK = (D + 1) * (D + 1);
    const uint4 m = make_uint4(0u, meta_y, 0u, 0u);
    Cam<T> cam;
    load_cam(camera, cam);
    Geo<T> G;
    geometry(P, stride, g, cam, cfg, G);

    // The compositing backward hands over, per record, the moments of
    // ge = dL/dalpha * alpha over the covered pixels, with the offset
    // delta = pixel - mean in the axes R = [v w] of the record's moment frame
    // (v = (cs, sn) the conic's narrow axis, w = (-sn, cs); e = R^T delta):
    // d[0] = sum ge, d[1..2] = sum ge e, d[3..5] = sum ge (e1^2, e1 e2, e2^2);
    // and dL/dcolour in d[6..8].  With alpha = o exp(-delta^T A delta / 2):
    //   dL/dlogit = sum ge (1 - o);
    //   dL/dmean2d = A sum ge delta = R Dg (d1, d2)  with Dg = R^T A R;
    //   dL/dA = -(1/2) sum ge delta delta^T, so the screen covariance
    //   Sigma' = A^-1 gets dL/dSigma' = -A dL/dA A = (1/2) R Dg Se Dg R^T,
    //   Se = [[d3, d4], [d4, d5]].
    // Dg is diagonal up to rounding; R is exactly the rotation the moments
    // were taken in, so nothing here subtracts the large along-axis moments
    // from the small across-axis ones.
    emit(10, d[0] * (T(1) - G.o));
    // in the moment frame; what the later steps need (the mean gradient, the
    // rotation and P = Dg Se Dg / 2) replaces the conic and the moments
    // before the SH planes are read, which keeps the values live across
    // those loads few
    T cs, sn;
    narrow_axis(axis, cs, sn);
    T dmx, dmy, P11, P12, P22;
    {
        const T cs2 = cs * cs, sn2 = sn * sn, csn = cs * sn;
        const T D11 = G.a * cs2 + T(2) * G.b * csn + G.c * sn2;
        const T D22 = G.a * sn2 - T(2) * G.b * csn + G.c * cs2;
        const T D12 = (G.c - G.a) * csn + G.b * (cs2 - sn2);
        const T q1 = D11 * d[1] + D12 * d[2], q2 = D12 * d[1] + D22 * d[2];
        dmx = cs * q1 - sn * q2;
        dmy = sn * q1 + cs * q2;
        const T E11 = D11 * d[3] + D12 * d[4], E12 = D11 * d[4] + D12 * d[5];
        const T E21 = D12 * d[3] + D22 * d[4], E22 = D12 * d[4] + D22 * d[5];
        P11 = T(0.5) * (E11 * D11 + E12 * D12);
        P12 = T(0.5) * (E11 * D12 + E12 * D22);
        P22 = T(0.5) * (E21 * D12 + E22 * D22);
    }

    // colour: c = max(0, sum_k Y_k f_k + 0.5)
    T dir[3];
    const T vinv = view_dir(G, cam, dir);
    T Y[16];
    SH<T>::template basis<D>(dir[0], dir[1], dir[2], Y);
    // the projection recorded which channels the clamp at zero cut off
    const uint32_t clamp = meta_clamp(m.y);
    T dc[3];
#pragma unroll
    for (int ch = 0; ch < 3; ch++) dc[ch] = (clamp >> ch) & 1u ? T(0) : d[6 + ch];
    if (sh_basis_out) {
#pragma unroll
        for (int k = 0; k < NK; k++) sh_basis_out[k] = Y[k];
#pragma unroll
        for (int ch = 0; ch < 3; ch++) sh_dc_out[ch] = dc[ch];
    }
    T wk[16];
#pragma unroll
    for (int k = 0; k < NK; k++) {
        T s = 0;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            s += plane(P, stride, 11 + 3 * k + ch, g) * dc[ch];
            emit(11 + 3 * k + ch, Y[k] * dc[ch]);
        }
        wk[k] = s;
    }
    T ddir[3];
    SH<T>::template grad_dot<D>(dir[0], dir[1], dir[2], wk, ddir);
    const T dd = ddir[0] * dir[0] + ddir[1] * dir[1] + ddir[2] * dir[2];
    T du[3];
#pragma unroll
    for (int k = 0; k < 3; k++) du[k] = (ddir[k] - dir[k] * dd) * vinv;

    // moments -> screen covariance: dSigma' = R P R^T
    const T cs2 = cs * cs, sn2 = sn * sn, csn = cs * sn;
    const T S00 = cs2 * P11 - T(2) * csn * P12 + sn2 * P22;
    const T S01 = csn * (P11 - P22) + (cs2 - sn2) * P12;
    const T S11 = sn2 * P11 + T(2) * csn * P12 + cs2 * P22;

    // screen covariance -> Sigma and the rows t0, t1 of J W
    T St0[3], St1[3];
    St0[0] = G.Sig[0] * G.t0[0] + G.Sig[1] * G.t0[1] + G.Sig[2] * G.t0[2];
    St0[1] = G.Sig[1] * G.t0[0] + G.Sig[3] * G.t0[1] + G.Sig[4] * G.t0[2];
    St0[2] = G.Sig[2] * G.t0[0] + G.Sig[4] * G.t0[1] + G.Sig[5] * G.t0[2];
    St1[0] = G.Sig[0] * G.t1[0] + G.Sig[1] * G.t1[1] + G.Sig[2] * G.t1[2];
    St1[1] = G.Sig[1] * G.t1[0] + G.Sig[3] * G.t1[1] + G.Sig[4] * G.t1[2];
    St1[2] = G.Sig[2] * G.t1[0] + G.Sig[4] * G.t1[1] + G.Sig[5] * G.t1[2];
    T dt0[3], dt1[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        dt0[k] = T(2) * (S00 * St0[k] + S01 * St1[k]);
        dt1[k] = T(2) * (S11 * St1[k] + S01 * St0[k]);
    }
    // dSigma (symmetric, full-matrix gradient)
    T dS[6];
    dS[0] = S00 * G.t0[0] * G.t0[0] + S11 * G.t1[0] * G.t1[0] + T(2) * S01 * G.t0[0] * G.t1[0];
    dS[3] = S00 * G.t0[1] * G.t0[1] + S11 * G.t1[1] * G.t1[1] + T(2) * S01 * G.t0[1] * G.t1[1];
    dS[5] = S00 * G.t0[2] * G.t0[2] + S11 * G.t1[2] * G.t1[2] + T(2) * S01 * G.t0[2] * G.t1[2];
    dS[1] = S00 * G.t0[0] * G.t0[1] + S11 * G.t1[0] * G.t1[1] + S01 * (G.t0[0] * G.t1[1] + G.t1[0] * G.t0[1]);
    dS[2] = S00 * G.t0[0] * G.t0[2] + S11 * G.t1[0] * G.t1[2] + S01 * (G.t0[0] * G.t1[2] + G.t1[0] * G.t0[2]);
    dS[4] = S00 * G.t0[1] * G.t0[2] + S11 * G.t1[1] * G.t1[2] + S01 * (G.t0[1] * G.t1[2] + G.t1[1] * G.t0[2]);

    // t0 = J00 W0 + J02 W2, t1 = J11 W1 + J12 W2
    const T dJ00 = dt0[0] * cam.R[0] + dt0[1] * cam.R[1] + dt0[2] * cam.R[2];
    const T dJ02 = dt0[0] * cam.R[6] + dt0[1] * cam.R[7] + dt0[2] * cam.R[8];
    const T dJ11 = dt1[0] * cam.R[3] + dt1[1] * cam.R[4] + dt1[2] * cam.R[5];
    const T dJ12 = dt1[0] * cam.R[6] + dt1[1] * cam.R[7] + dt1[2] * cam.R[8];
    const T rz = G.rz, rz2 = G.rz * G.rz;
    const T tx = G.t[0], ty = G.t[1];
    T dtc[3];
    dtc[0] = dmx * cam.fx * rz;
    dtc[1] = dmy * cam.fy * rz;
    dtc[2] = -(dmx * cam.fx * tx + dmy * cam.fy * ty) * rz2;
    dtc[2] += -(dJ00 * cam.fx + dJ11 * cam.fy) * rz2;
    dtc[2] += (dJ02 * cam.fx * G.rx + dJ12 * cam.fy * G.ry) * rz2;
    const T drx = -dJ02 * cam.fx * rz, dry = -dJ12 * cam.fy * rz;
    if (!G.clx) { dtc[0] += drx * rz; dtc[2] -= drx * tx * rz2; }
    if (!G.cly) { dtc[1] += dry * rz; dtc[2] -= dry * ty * rz2; }
    // t = W u + t_cw
#pragma unroll
    for (int k = 0; k < 3; k++)
        emit(k, du[k] + cam.R[k] * dtc[0] + cam.R[3 + k] * dtc[1] + cam.R[6 + k] * dtc[2]);

    // Sigma = M M^T with M = R diag(s): dM = 2 dSigma M
    const T dSf[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
    T dR[9];
#pragma unroll
    for (int cidx = 0; cidx < 3; cidx++) {
        T ds = 0;
#pragma unroll
        for (int ridx = 0; ridx < 3; ridx++) {
            T dM = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) dM += dSf[3 * ridx + k] * G.R[3 * k + cidx];
            dM *= T(2) * G.s[cidx];
            ds += dM * G.R[3 * ridx + cidx];
            dR[3 * ridx + cidx] = dM * G.s[cidx];
        }
        emit(7 + cidx, ds * G.s[cidx]);   // s = exp(log-scale)
    }
    // R(qn)
    const T w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
    T dq[4];
    dq[0] = T(2) * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = T(2) * (y * dR[1] + z * dR[2] + y * dR[3] - T(2) * x * dR[4] - w * dR[5] + z * dR[6] +
                    w * dR[7] - T(2) * x * dR[8]);
    dq[2] = T(2) * (-T(2) * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                    z * dR[7] - T(2) * y * dR[8]);
    dq[3] = T(2) * (-T(2) * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - T(2) * z * dR[4] + y * dR[5] +
                    x * dR[6] + y * dR[7]);
    const T qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
#pragma unroll
    for (int k = 0; k < 4; k++) emit(3 + k, (dq[k] - G.qn[k] * qd) * G.qinv);
}

// Jobs over disjoint Gaussian ranges: one thread per record, each gradient
// plane stored once, as soon as it is known.  Culled records get zeros.
template <typename T, int D>
__global__ __launch_bounds__(128) void k_project_bwd_rec(const T* __restrict__ P, int64_t stride, gs_frame frame,
                                                          gs_raster_cfg cfg, const T* __restrict__ rec,
                                                          const uint4* __restrict__ meta,
                                                          const uint32_t* __restrict__ pair_off, uint64_t capacity,
                                                          PartialLayout L, const T* __restrict__ pg, T* __restrict__ grad,
                                                          int64_t gstride) {
    constexpr int A = 11 + 3 * (D + 1) * (D + 1);
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool active = r < frame.n_records;   // no early return before the wave-wide sums
    const int j = job_of_record(frame.jobs, frame.n_jobs, active ? r : 0);
    const gs_job job = frame.jobs[j];
    const int64_t g = job.g0 + (r - job.rec0);
    const uint4 m = active ? meta[r] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t ntiles = meta_tiles(m.y);
    const T axis = ntiles ? rec[r * GS_REC_WORDS + 9] : T(0);   // moment frame, loaded early
    T d[9];
    record_partials(pg, L, m, ntiles ? pair_off[r] : 0u, capacity, d);
    if (!active) return;
    T* gout = grad + g;
    if (ntiles == 0) {
#pragma unroll
        for (int a = 0; a < A; a++) gout[int64_t(a) * gstride] = T(0);
        return;
    }
    record_chain<T, D>(P, stride, g, frame.cams[job.cam], cfg, m.y, d, axis,
                       [&](int a, T v) { gout[int64_t(a) * gstride] = v; });
}

// Gaussians held by several jobs (several views of one block in one step):
// one thread per Gaussian adds its records' contributions in job order.
template <typename T, int D>
__global__ __launch_bounds__(128) void k_project_bwd_acc(const T* __restrict__ P, int64_t stride, int64_t n,
                                                          gs_frame frame, gs_raster_cfg cfg,
                                                          const T* __restrict__ rec, const uint4* __restrict__ meta,
                                                          const uint32_t* __restrict__ pair_off, uint64_t capacity,
                                                          PartialLayout L, const T* __restrict__ pg, T* __restrict__ grad,
                                                          int64_t gstride) {
    constexpr int A = 11 + 3 * (D + 1) * (D + 1);
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool active = g < n;
    T* gout = grad + (active ? g : 0);
    if (active)
        for (int a = 0; a < A; a++) gout[int64_t(a) * gstride] = T(0);
    for (int j = 0; j < frame.n_jobs; j++) {
        const gs_job job = frame.jobs[j];
        const bool in_job = active && g >= job.g0 && g < job.g1;
        const int64_t r = in_job ? job.rec0 + (g - job.g0) : 0;
        const uint4 m = in_job ? meta[r] : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t ntiles = meta_tiles(m.y);
        const T axis = ntiles ? rec[r * GS_REC_WORDS + 9] : T(0);
        T d[9];
        record_partials(pg, L, m, ntiles ? pair_off[r] : 0u, capacity, d);
        if (ntiles == 0) continue;
        record_chain<T, D>(P, stride, g, frame.cams[job.cam], cfg, m.y, d, axis,
                           [&](int a, T v) { gout[int64_t(a) * gstride] += v; });
    }
}

// Fused projection backward + Adam/ADMM for jobs over disjoint Gaussian
// ranges (one record per Gaussian).  A block of kFusedBlock records works in
// two phases.  (1) Each thread runs the chain rule of its record and leaves in
// LDS the 11 geometry gradients, the SH basis values Y[k] and the clamped
// colour gradient dc[ch] (the SH-plane gradient is the product Y[k] dc[ch],
// formed exactly as the chain rule emits it); a culled record leaves zeros.
// (2) The block streams the optimiser over all planes of its Gaussians: when
// they are contiguous and 16-byte aligned, as items of (plane, 4 Gaussians)
// with 16-byte accesses, else one Gaussian per thread.  The gradient never
// reaches HBM and the parameters read by the chain are still in cache for the
// update.  Same arithmetic as k_project_bwd_rec followed by k_adam_admm.
constexpr int kFusedBlock = 256;

// gradient of plane a of the block's Gaussian i from the phase-1 LDS arrays
// (geo [11][kFusedBlock], Y [NK][kFusedBlock], dc [3][kFusedBlock])
__device__ inline float staged_grad(const float* geo, const float* Y, const float* dc, int a, int i) {
    return a < 11 ? geo[a * kFusedBlock + i]
                  : Y[((a - 11) / 3) * kFusedBlock + i] * dc[((a - 11) % 3) * kFusedBlock + i];
}

// phase 2 over contiguous, 16-byte aligned Gaussians g0 .. g0 + kFusedBlock - 1:
// each wavefront takes every fourth plane, its lanes 4 Gaussians each with
// 16-byte accesses; the loads of kUnroll planes are issued before any of
// them is used, so several lines per lane are in flight.  m, v and w stream
// past the caches (x stays cached: the chain rule has just read part of it)
constexpr int kUnroll = 3;
template <int A, bool PEN, bool MASK>
__device__ inline void adam_block_vec(float* __restrict__ X, int64_t sx, float* __restrict__ M, int64_t sm,
                                      float* __restrict__ V, int64_t sv, const float* __restrict__ Wp, int64_t sw,
                                      const float* __restrict__ mask, int64_t g0, const float* geo, const float* Y,
                                      const float* dc, const AdamConsts& c, float& fin) {
    constexpr int kCols = kFusedBlock / 4;
    static_assert(kCols == kWave, "one plane per wavefront and step");
    constexpr int kStep = kFusedBlock / kCols;
    const int t = threadIdx.x;
    const int col = t % kCols;
    const int i = 4 * col;
    const int64_t gv = g0 + i;
    const int a_first = __builtin_amdgcn_readfirstlane(t / kCols);   // the wavefront's first plane
    float4 kv = make_float4(1.f, 1.f, 1.f, 1.f);
    if (MASK) kv = *reinterpret_cast<const float4*>(mask + gv);
    for (int a0 = a_first; a0 < A; a0 += kUnroll * kStep) {
        float4 xv[kUnroll], mv[kUnroll], vv[kUnroll], wv[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const int a = a0 + u * kStep;   // uniform
            if (a >= A) break;
            xv[u] = *reinterpret_cast<const float4*>(X + a * sx + gv);
            mv[u] = load_stream4(M + a * sm + gv);
            vv[u] = load_stream4(V + a * sv + gv);
            wv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (PEN) wv[u] = load_stream4(Wp + a * sw + gv);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const int a = a0 + u * kStep;
            if (a >= A) break;
            const int grp = plane_group(a);
            const float lr = c.lr[grp], rho = c.rho[grp];
            // the four Gaussians' gradients of plane a: one 16-byte LDS read per array
            float4 gq;
            if (a < 11) {
                gq = *reinterpret_cast<const float4*>(geo + a * kFusedBlock + i);
            } else {
                const float4 yq = *reinterpret_cast<const float4*>(Y + ((a - 11) / 3) * kFusedBlock + i);
                const float4 dq = *reinterpret_cast<const float4*>(dc + ((a - 11) % 3) * kFusedBlock + i);
                gq = make_float4(yq.x * dq.x, yq.y * dq.y, yq.z * dq.z, yq.w * dq.w);
            }
            adam_one(xv[u].x, gq.x, mv[u].x, vv[u].x, wv[u].x, PEN ? rho * kv.x : 0.f, lr, c);
            adam_one(xv[u].y, gq.y, mv[u].y, vv[u].y, wv[u].y, PEN ? rho * kv.y : 0.f, lr, c);
            adam_one(xv[u].z, gq.z, mv[u].z, vv[u].z, wv[u].z, PEN ? rho * kv.z : 0.f, lr, c);
            adam_one(xv[u].w, gq.w, mv[u].w, vv[u].w, wv[u].w, PEN ? rho * kv.w : 0.f, lr, c);
            *reinterpret_cast<float4*>(X + a * sx + gv) = xv[u];
            store_stream4(M + a * sm + gv, mv[u]);
            store_stream4(V + a * sv + gv, vv[u]);
            adam_finite(fin, xv[u].x, vv[u].x);
            adam_finite(fin, xv[u].y, vv[u].y);
            adam_finite(fin, xv[u].z, vv[u].z);
            adam_finite(fin, xv[u].w, vv[u].w);
        }
    }
}

// phase 2 for one Gaussian g (the block's i-th record), all planes
template <int A, bool PEN, bool MASK>
__device__ inline void adam_block_one(float* __restrict__ X, int64_t sx, float* __restrict__ M, int64_t sm,
                                      float* __restrict__ V, int64_t sv, const float* __restrict__ Wp, int64_t sw,
                                      const float* __restrict__ mask, int64_t g, int i, const float* geo,
                                      const float* Y, const float* dc, const AdamConsts& c, float& fin) {
    const float k = MASK ? mask[g] : 1.f;
    for (int a = 0; a < A; a++) {
        const int grp = plane_group(a);
        float xv = X[a * sx + g], mv = M[a * sm + g], vv = V[a * sv + g];
        const float wv = PEN ? Wp[a * sw + g] : 0.f;
        adam_one(xv, staged_grad(geo, Y, dc, a, i), mv, vv, wv, PEN ? c.rho[grp] * k : 0.f, c.lr[grp], c);
        X[a * sx + g] = xv;
        M[a * sm + g] = mv;
        V[a * sv + g] = vv;
        adam_finite(fin, xv, vv);
    }
}

template <int D, bool PEN, bool MASK, bool VEC>
__global__ __launch_bounds__(kFusedBlock) void k_project_bwd_adam(
    float* X, int64_t sx, gs_frame frame, gs_raster_cfg cfg, const float* __restrict__ rec,
    const uint4* __restrict__ meta, const uint32_t* __restrict__ pair_off, uint64_t capacity, PartialLayout L,
    const float* __restrict__ pg,
    float* __restrict__ M,
    int64_t sm, float* __restrict__ V, int64_t sv, const float* __restrict__ Wp, int64_t sw,
    const float* __restrict__ mask, AdamConsts c, uint32_t* __restrict__ status) {
    constexpr int NK = (D + 1) * (D + 1);
    constexpr int A = 11 + 3 * NK;
    if (adam_skipped(status)) return;   // uniform over the grid: no wavefront reaches the barrier
    __shared__ __align__(16) float s_geo[11][kFusedBlock];
    __shared__ __align__(16) float s_Y[NK][kFusedBlock];
    __shared__ __align__(16) float s_dc[3][kFusedBlock];
    const int t = threadIdx.x;
    const int64_t r0 = int64_t(blockIdx.x) * kFusedBlock;
    const int64_t r = r0 + t;
    const bool active = r < frame.n_records;   // no early return before the wave-wide sums and the barrier
    const int j = job_of_record(frame.jobs, frame.n_jobs, active ? r : 0);
    const gs_job job = frame.jobs[j];
    const int64_t g = job.g0 + (r - job.rec0);
    const uint4 m = active ? meta[r] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t ntiles = meta_tiles(m.y);
    const float axis = ntiles ? rec[r * GS_REC_WORDS + 9] : 0.f;   // moment frame, loaded early
    float d[9];
    record_partials(pg, L, m, ntiles ? pair_off[r] : 0u, capacity, d);

    // phase 1: chain rule into LDS
    float Y[NK], dc[3];
#pragma unroll
    for (int a = 0; a < 11; a++) s_geo[a][t] = 0.f;
#pragma unroll
    for (int q = 0; q < NK; q++) Y[q] = 0.f;
    dc[0] = dc[1] = dc[2] = 0.f;
    if (active && ntiles != 0)
        record_chain<float, D>(X, sx, g, frame.cams[job.cam], cfg, m.y, d, axis,
                               [&](int a, float v) {
                                   if (a < 11) s_geo[a][t] = v;
                               },
                               Y, dc);
#pragma unroll
    for (int q = 0; q < NK; q++) s_Y[q][t] = Y[q];
#pragma unroll
    for (int ch = 0; ch < 3; ch++) s_dc[ch][t] = dc[ch];
    // the block's Gaussians are contiguous when its records all lie in one job
    const int j0 = job_of_record(frame.jobs, frame.n_jobs, r0);
    const int64_t g0 = frame.jobs[j0].g0 + (r0 - frame.jobs[j0].rec0);
    const bool contiguous = __syncthreads_and(active && j == j0) != 0;

    // phase 2: optimiser over the planes
    float fin = 0.f;
    if (VEC && contiguous && (g0 & 3) == 0)
        adam_block_vec<A, PEN, MASK>(X, sx, M, sm, V, sv, Wp, sw, mask, g0, &s_geo[0][0], &s_Y[0][0], &s_dc[0][0], c,
                                     fin);
    else if (active)
        adam_block_one<A, PEN, MASK>(X, sx, M, sm, V, sv, Wp, sw, mask, g, t, &s_geo[0][0], &s_Y[0][0], &s_dc[0][0],
                                     c, fin);
    adam_flag(status, fin);
}

// Adam/ADMM with a zero gradient for Gaussians outside every job (disjoint
// jobs that do not cover [0, n)); the fused kernel updates all the others.
template <bool PEN, bool MASK>
__global__ __launch_bounds__(256) void k_adam_uncovered(int64_t n, gs_frame frame, int A, float* __restrict__ X,
                                                        int64_t sx, float* __restrict__ M, int64_t sm,
                                                        float* __restrict__ V, int64_t sv,
                                                        const float* __restrict__ Wp, int64_t sw,
                                                        const float* __restrict__ mask, AdamConsts c,
                                                        uint32_t* __restrict__ status) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n || adam_skipped(status)) return;
    for (int j = 0; j < frame.n_jobs; j++)
        if (g >= frame.jobs[j].g0 && g < frame.jobs[j].g1) return;
    const float k = MASK ? mask[g] : 1.f;
    float fin = 0.f;
    for (int a = 0; a < A; a++) {
        const int grp = plane_group(a);
        float xv = X[a * sx + g], mv = M[a * sm + g], vv = V[a * sv + g];
        const float wv = PEN ? Wp[a * sw + g] : 0.f;
        adam_one(xv, 0.f, mv, vv, wv, PEN ? c.rho[grp] * k : 0.f, c.lr[grp], c);
        X[a * sx + g] = xv;
        M[a * sm + g] = mv;
        V[a * sv + g] = vv;
        adam_finite(fin, xv, vv);
    }
    adam_flag(status, fin);
}

// zeros for Gaussians outside every job (disjoint jobs that do not cover [0, n))
template <typename T>
__global__ __launch_bounds__(256) void k_zero_uncovered(int64_t n, gs_frame frame, int A, T* __restrict__ grad,
                                                        int64_t gstride) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    for (int j = 0; j < frame.n_jobs; j++)
        if (g >= frame.jobs[j].g0 && g < frame.jobs[j].g1) return;
    for (int a = 0; a < A; a++) grad[int64_t(a) * gstride + g] = T(0);
}

// ---------------------------------------------------------------------------

template <typename T>
hipError_t launch_project(const gs_params& p, const gs_frame& f, const gs_raster_cfg& cfg, T* rec,
                          uint32_t* meta, uint32_t* status, hipStream_t s) {
    const int64_t n = f.n_records;
    if (n == 0) return hipSuccess;
    dim3 grid(unsigned((n + 255) / 256)), block(256);
    const T* P = static_cast<const T*>(p.data);
    uint4* M = reinterpret_cast<uint4*>(meta);
    switch (p.sh_degree) {
        case 0: GS_LAUNCH("k_project", (k_project<T, 0>), grid, block, 0, s, P, p.stride, f, cfg, rec, M, status); break;
        case 1: GS_LAUNCH("k_project", (k_project<T, 1>), grid, block, 0, s, P, p.stride, f, cfg, rec, M, status); break;
        case 2: GS_LAUNCH("k_project", (k_project<T, 2>), grid, block, 0, s, P, p.stride, f, cfg, rec, M, status); break;
        default: GS_LAUNCH("k_project", (k_project<T, 3>), grid, block, 0, s, P, p.stride, f, cfg, rec, M, status); break;
    }
    return hipGetLastError();
}

template <typename T>
static PartialLayout partial_layout(const gs_raster_cfg& cfg, const gs_bins&, const T*) {
    PartialLayout L;
    L.slots = bwd_slots(cfg);
    return L;
}

template <typename T, int D>
static void project_bwd_dispatch(const gs_params& p, const gs_frame& f, const gs_raster_cfg& cfg, const T* rec,
                                 const uint4* M,
                                 const uint32_t* pair_off, uint64_t capacity, const PartialLayout& L, const T* pg,
                                 gs_params& grad, hipStream_t s) {
    const T* P = static_cast<const T*>(p.data);
    T* Gd = static_cast<T*>(grad.data);
    if (f.jobs_disjoint) {
        const bool covers = f.n_records == p.n && f.g_max == p.n;
        if (!covers)
            GS_LAUNCH("k_zero_uncovered", (k_zero_uncovered<T>), dim3(unsigned((p.n + 255) / 256)), dim3(256), 0, s, p.n, f,
                               11 + 3 * (D + 1) * (D + 1), Gd, grad.stride);
        if (f.n_records > 0)
            GS_LAUNCH("k_project_bwd_rec", (k_project_bwd_rec<T, D>), dim3(unsigned((f.n_records + 127) / 128)), dim3(128), 0, s,
                               P, p.stride, f, cfg, rec, M, pair_off, capacity, L, pg, Gd, grad.stride);
    } else {
        GS_LAUNCH("k_project_bwd_acc", (k_project_bwd_acc<T, D>), dim3(unsigned((p.n + 127) / 128)), dim3(128), 0, s, P,
                           p.stride, p.n, f, cfg, rec, M, pair_off, capacity, L, pg, Gd, grad.stride);
    }
}

template <typename T>
hipError_t launch_project_bwd(const gs_params& p, const gs_frame& f, const gs_raster_cfg& cfg, const T* rec,
                              const uint32_t* meta, const gs_bins& bins, const T* pg, gs_params& grad, hipStream_t s) {
    if (p.n == 0) return hipSuccess;
    const uint4* M = reinterpret_cast<const uint4*>(meta);
    const PartialLayout L = partial_layout(cfg, bins, pg);
    const uint32_t* po = bins.pair_off;
    const uint64_t cap = bins.capacity;
    switch (p.sh_degree) {
        case 0: project_bwd_dispatch<T, 0>(p, f, cfg, rec, M, po, cap, L, pg, grad, s); break;
        case 1: project_bwd_dispatch<T, 1>(p, f, cfg, rec, M, po, cap, L, pg, grad, s); break;
        case 2: project_bwd_dispatch<T, 2>(p, f, cfg, rec, M, po, cap, L, pg, grad, s); break;
        default: project_bwd_dispatch<T, 3>(p, f, cfg, rec, M, po, cap, L, pg, grad, s); break;
    }
    return hipGetLastError();
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <int D, bool PEN, bool MASK>
static void project_bwd_adam_launch(gs_params& x, const gs_frame& f, const gs_raster_cfg& cfg, const float* rec,
                                    const uint4* M,
                                    const uint32_t* pair_off, uint64_t capacity, const PartialLayout& L,
                                    const float* pg, gs_params& m, gs_params& v, const gs_params* w,
                                    const float* mask, const AdamConsts& c, uint32_t* status, hipStream_t s) {
    float* X = static_cast<float*>(x.data);
    float* Mo = static_cast<float*>(m.data);
    float* Vo = static_cast<float*>(v.data);
    const float* Wd = w ? static_cast<const float*>(w->data) : nullptr;
    const int64_t sw = w ? w->stride : 0;
    const bool covers = f.n_records == x.n && f.g_max == x.n;
    if (!covers)
        GS_LAUNCH("k_adam_uncovered", (k_adam_uncovered<PEN, MASK>), dim3(unsigned((x.n + 255) / 256)), dim3(256), 0, s, x.n, f,
                           11 + 3 * (D + 1) * (D + 1), X, x.stride, Mo, m.stride, Vo, v.stride, Wd, sw, mask, c,
                           status);
    const bool vec = aligned16(X) && aligned16(Mo) && aligned16(Vo) && (!Wd || aligned16(Wd)) &&
                     (!mask || aligned16(mask)) && x.stride % 4 == 0 && m.stride % 4 == 0 && v.stride % 4 == 0 &&
                     sw % 4 == 0;
    const dim3 grid(unsigned((f.n_records + kFusedBlock - 1) / kFusedBlock)), block(kFusedBlock);
    if (f.n_records > 0 && vec)
        GS_LAUNCH("k_project_bwd_adam", (k_project_bwd_adam<D, PEN, MASK, true>), grid, block, 0, s, X, x.stride, f,
                  cfg, rec, M, pair_off, capacity, L, pg, Mo, m.stride, Vo, v.stride, Wd, sw, mask, c, status);
    else if (f.n_records > 0)
        GS_LAUNCH("k_project_bwd_adam", (k_project_bwd_adam<D, PEN, MASK, false>), grid, block, 0, s, X, x.stride,
                  f, cfg, rec, M, pair_off, capacity, L, pg, Mo, m.stride, Vo, v.stride, Wd, sw, mask, c, status);
}

template <int D>
static void project_bwd_adam_pen(gs_params& x, const gs_frame& f, const gs_raster_cfg& cfg, const float* rec,
                                 const uint4* M,
                                 const uint32_t* po, uint64_t cap, const PartialLayout& L, const float* pg,
                                 gs_params& m, gs_params& v, const gs_params* w, const float* mask,
                                 const AdamConsts& c, uint32_t* st, hipStream_t s) {
    if (w && mask) project_bwd_adam_launch<D, true, true>(x, f, cfg, rec, M, po, cap, L, pg, m, v, w, mask, c, st, s);
    else if (w) project_bwd_adam_launch<D, true, false>(x, f, cfg, rec, M, po, cap, L, pg, m, v, w, mask, c, st, s);
    else project_bwd_adam_launch<D, false, false>(x, f, cfg, rec, M, po, cap, L, pg, m, v, w, mask, c, st, s);
}

hipError_t launch_project_bwd_adam(gs_params& x, const gs_frame& f, const gs_raster_cfg& cfg, const float* rec,
                                   const uint32_t* meta,
                                   const gs_bins& bins, const float* pg, gs_params& m, gs_params& v,
                                   const gs_params* w, const float* mask, const gs_adam_cfg& acfg, hipStream_t s) {
    if (x.n == 0) return hipSuccess;
    const uint4* M = reinterpret_cast<const uint4*>(meta);
    const AdamConsts c = adam_consts(acfg);
    const PartialLayout L = partial_layout(cfg, bins, pg);
    const uint32_t* po = bins.pair_off;
    const uint64_t cap = bins.capacity;
    uint32_t* st = bins.counters + GS_CTR_STATUS;
    switch (x.sh_degree) {
        case 0: project_bwd_adam_pen<0>(x, f, cfg, rec, M, po, cap, L, pg, m, v, w, mask, c, st, s); break;
        case 1: project_bwd_adam_pen<1>(x, f, cfg, rec, M, po, cap, L, pg, m, v, w, mask, c, st, s); break;
        case 2: project_bwd_adam_pen<2>(x, f, cfg, rec, M, po, cap, L, pg, m, v, w, mask, c, st, s); break;
        default: project_bwd_adam_pen<3>(x, f, cfg, rec, M, po, cap, L, pg, m, v, w, mask, c, st, s); break;
    }
    return hipGetLastError();
}

template hipError_t launch_project<float>(const gs_params&, const gs_frame&, const gs_raster_cfg&, float*, uint32_t*, uint32_t*, hipStream_t);
template hipError_t launch_project<double>(const gs_params&, const gs_frame&, const gs_raster_cfg&, double*, uint32_t*, uint32_t*, hipStream_t);
template hipError_t launch_project_bwd<float>(const gs_params&, const gs_frame&, const gs_raster_cfg&, const float*, const uint32_t*, const gs_bins&, const float*, gs_params&, hipStream_t);
template hipError_t launch_project_bwd<double>(const gs_params&, const gs_frame&, const gs_raster_cfg&, const double*, const uint32_t*, const gs_bins&, const double*, gs_params&, hipStream_t);

}  // namespace gs
