/*
 * gs.h -- C ABI of libgs: the per-block training step of ADMM-consensus
 * Gaussian splatting on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow the paper's statement of the problem (DOGS,
 * "Distributed-Oriented Gaussian Splatting ... via Gaussian Consensus"):
 *   - Gaussians x = {u, q, s, f, o} (Sec. 3.1, Eq. 1-3 and the attribute list
 *     that follows Eq. 3);
 *   - rendering by projection and front-to-back alpha compositing (Eq. 2);
 *   - the block x-update with the scaled ADMM penalty, per-attribute rho
 *     (Eq. 8a; supplementary Sec. C);
 *   - the consensus z = mean of the local copies and the dual update
 *     u += x - z (Eq. 8b-c; Alg. 2), duals initialised to zero.
 * Where the paper is silent (projection, tiling, thresholds) the readings are
 * the constants of gs_raster_cfg, documented field by field below.
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev or stored in gs_params / gs_bins are DEVICE
 *     pointers; the structs themselves (gs_params, gs_frame, gs_raster_cfg,
 *     gs_adam_cfg, gs_bins) are read on the host and passed by value to the
 *     kernels.  gs_frame.cams and gs_frame.jobs point to device copies.
 *   - The caller owns every buffer, including workspaces; libgs allocates no
 *     device memory and keeps no per-call state.
 *   - Calls are asynchronous on the given HIP stream (NULL = default stream)
 *     and re-entrant.
 *   - A call returns GS_OK or an error code; on error nothing was launched
 *     (GS_E_INVALID, GS_E_UNSUPPORTED) or a launch failed (GS_E_DEVICE).
 *     gs_last_error() returns a thread-local description.  No C++ exception
 *     crosses this interface.
 *   - Conditions only known on the device (pair-capacity overflow) are
 *     reported through gs_bins.counters; check them after the stream work is
 *     done, grow the buffers and run again.
 *   - FP32 entry points take float planes; the *_f64 variants are the same
 *     kernels instantiated for double (for adjoint checks).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 5

typedef enum {
    GS_OK = 0,
    GS_E_INVALID = 1,      /* null pointer, negative size, SH degree > 3, bad tile shape */
    GS_E_CAPACITY = 2,     /* a host-visible size exceeds a buffer */
    GS_E_DEVICE = 3,       /* a HIP call or kernel launch failed */
    GS_E_UNSUPPORTED = 4   /* valid request this build does not implement */
} gs_status;

/* status bits OR-ed into a device status word (gs_bins.counters[GS_CTR_STATUS],
 * or the status_dev argument of gs_project and gs_adam_admm); sticky: no call
 * clears them, so one check after many steps covers all of them */
#define GS_STATUS_PAIR_OVERFLOW 1u   /* gs_bin_sort: more pairs than bins.capacity */
#define GS_STATUS_NONFINITE 2u       /* gs_project / the optimiser met a NaN or Inf */

/* indices into gs_bins.counters (device, uint32[GS_N_COUNTERS]) */
#define GS_CTR_VISIBLE 0   /* records with at least one covered tile */
#define GS_CTR_PAIRS 1     /* (tile, record) pairs required (may exceed capacity) */
#define GS_CTR_STATUS 2
#define GS_CTR_OVERFLOWED 3  /* gs_bin_sort calls that ended with GS_STATUS_PAIR_OVERFLOW
                                set (counted until the caller clears it): the steps whose
                                optimiser updates were skipped */
#define GS_N_COUNTERS 4

typedef void *gs_stream;   /* hipStream_t */

/* Parameter planes (Sec. 3.1): one plane per scalar attribute, plane a at
 * data + a * stride elements:
 *   0..2  mean u;  3..6 quaternion q (w, x, y, z), unnormalised;
 *   7..9  log scale;  10 opacity logit;
 *   11 + 3k + c  SH coefficient k = l*l + l + m of colour channel c.
 * A = 11 + 3 (sh_degree + 1)^2 planes.  The same layout holds Adam moments,
 * duals u, consensus targets w = z - u, gradients and the global model z. */
typedef struct {
    void *data;          /* device, float (or double for *_f64) */
    int64_t n;           /* number of Gaussians */
    int64_t stride;      /* elements between planes, >= n */
    int32_t sh_degree;   /* 0..3 */
    int32_t reserved;
} gs_params;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  A world point X
 * maps to camera point R X + t and to pixel (fx x/z + cx, fy y/z + cy);
 * pixel (i, j) samples the point (i + 1/2, j + 1/2). */
typedef struct {
    float R[9];          /* world -> camera rotation, row major */
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} gs_camera;

/* One render job: the Gaussians [g0, g1) seen through camera `cam`.  The
 * fields marked (plan) are filled by gs_frame_plan. */
typedef struct {
    int32_t cam;
    int32_t tiles_x;     /* (plan) */
    int32_t tiles_y;     /* (plan) */
    int32_t tile0;       /* (plan) first global tile id */
    int64_t g0, g1;
    int64_t rec0;        /* (plan) first projected-record slot */
    int64_t px0;         /* (plan) first pixel; the job's image is [3][H][W] at 3*px0 */
    float loss_weight;   /* weight of this job's L1 loss term */
    int32_t reserved;
} gs_job;

typedef struct {
    const gs_camera *cams;   /* device */
    const gs_job *jobs;      /* device, planned */
    int32_t n_jobs;
    int32_t n_tiles;         /* total tiles over all jobs */
    int64_t n_records;       /* sum of (g1 - g0) */
    int64_t n_pixels;        /* sum of W * H */
    int64_t g_max;           /* max g1 over jobs; must not exceed the parameter count */
    int32_t jobs_disjoint;   /* 1 when no two jobs share a Gaussian */
    int32_t reserved;
} gs_frame;

/* Rasterizer constants.  The paper writes alpha = o X^proj(p) (Eq. 2) without
 * defining X^proj; the readings: EWA local-affine projection with `dilation`
 * px^2 added to the screen covariance, x/z and y/z clamped to `jac_clip`
 * times the half field of view inside the Jacobian, cull at depth <=
 * `near_z`, alpha = min(alpha_max, o G), keep when alpha >= alpha_min, stop
 * before the Gaussian that takes T below T_min, background bg. */
typedef struct {
    int32_t tile_w, tile_h;  /* binning tile: 8x8, 16x8, 16x16 or 32x8 */
    float near_z;            /* 0.2 */
    float alpha_min;         /* 1/255 */
    float alpha_max;         /* 0.99 */
    float T_min;             /* 1e-4 */
    float dilation;          /* 0.3 */
    float jac_clip;          /* 1.3 */
    float bg[3];             /* 0, 0, 0 */
    int16_t fwd_waves;       /* wavefronts per tile in the forward and in the backward */
    int16_t bwd_waves;       /* compositing, each owning an equal part of the tile and walking
                                the whole list: 1 (0 = 1), 2 (16x8, 16x16, 32x8) or 4 (16x16,
                                32x8); GS_WAVES_ADAPTIVE picks 1, 2 or 4 per tile from its
                                list length against the frame mean (4 above 4x, 2 above
                                1.25x; needs gs_bins.tile_order).  Images do not depend on them; gradients only
                                through the order of their sums. */
} gs_raster_cfg;

#define GS_WAVES_ADAPTIVE (-1)

/* Tile bins produced by gs_bin_sort. */
typedef struct {
    uint32_t *vals;          /* device [capacity]: record ids in (tile, depth, record) order */
    uint32_t *ranges;        /* device [n_tiles][2]: [start, end) into vals; (0, 0) when empty */
    uint32_t *pair_off;      /* device [n_records]: first pair of each visible record */
    uint32_t *counters;      /* device [GS_N_COUNTERS] */
    uint64_t capacity;       /* pairs vals can hold */
    uint32_t *tile_order;    /* device [n_tiles + 4] or NULL: the compositing plan written by
                                gs_bin_sort, needed when fwd_waves or bwd_waves is
                                GS_WAVES_ADAPTIVE: [0..2] = tiles taking 4, 2 and 1 wavefronts,
                                then the tile ids, those groups in that order */
    uint8_t *qmask;          /* device [capacity] or NULL: per list entry (vals order), bit q set
                                unless no pixel centre of 8x8 quadrant q of its tile (row-major
                                over the tile's quadrants, at most 4) can reach alpha_min for
                                its record.  Written by gs_render_fwd for the entries it walks,
                                read by gs_render_bwd of the same frame and bins, which then
                                need not recompute these conservative tests; with NULL the
                                backward computes them itself (same results bit for bit). */
} gs_bins;

/* Adam with the ADMM penalty (Eq. 8a, supplementary Sec. C).  Groups in the
 * paper's order: 0 p (mean), 1 q (rotation), 2 s (scale), 3 f (SH), 4 o. */
typedef struct {
    float lr[5];
    float rho[5];
    float beta1, beta2, eps;
    int32_t reserved;
    int64_t step;            /* 1-based, for bias correction */
} gs_adam_cfg;

typedef enum { GS_LOSS_L1 = 0, GS_LOSS_EXTERNAL = 1 } gs_loss_mode;

/* Records written by gs_project, per (job, Gaussian) slot: */
#define GS_REC_WORDS 12      /* T-typed words per record */
#define GS_META_WORDS 4      /* uint32 words per record: depth bits, n_tiles, rect lo, rect hi */

/* ------------------------------------------------------------------ */

int32_t gs_abi_version(void);
const char *gs_last_error(void);

/* Defaults of gs_raster_cfg (16x16 tiles and the constants listed above). */
void gs_raster_cfg_default(gs_raster_cfg *cfg);

/* Host-side planning of a frame: fills tiles_x/tiles_y/tile0/rec0/px0 of each
 * job from the host copy of the cameras, and the totals of gs_frame (n_tiles,
 * n_records, n_pixels, g_max, jobs_disjoint).  No device work.  The device job table handed
 * to the other calls must be a copy of the planned jobs. */
gs_status gs_frame_plan(const gs_camera *cams_host, int32_t n_cams, gs_job *jobs_host, int32_t n_jobs,
                        const gs_raster_cfg *cfg, int64_t *n_records, int64_t *n_pixels, int32_t *n_tiles,
                        int64_t *g_max, int32_t *jobs_disjoint);

/* Projection (Sec. 3.1: Eq. 1, Sigma = R S S^T R^T, alpha = o X^proj(p), SH
 * colour).  For every (job, Gaussian) slot r = rec0 + g - g0 writes
 *   rec [r][12]: mean2d x, y; the conic scaled for exp2 (-a/2, -b, -c/2
 *                times log2 e); log2 opacity; colour r, g, b; the axis of
 *                the conic's largest eigenvalue as tan(theta / 2) of its
 *                direction (cos theta, sin theta), cos theta >= 0 (the frame
 *                in which the backward sums its second moments); the
 *                conservative half-extents (x, y) in pixels of the region
 *                where alpha >= alpha_min
 *   meta[r][4]:  FP32 bits of the depth, number of covered tiles (0 = culled) in
 *                bits 0..23 with the colour-clamp flags of r, g, b in bits 24..26,
 *                tile rectangle lo (x | y << 16) and hi (inclusive).
 * The rectangle is conservative: every pixel where alpha >= alpha_min lies
 * inside it.  status_dev (device uint32, may be NULL; e.g. the bins'
 * counters + GS_CTR_STATUS): GS_STATUS_NONFINITE is OR-ed in when a
 * parameter value the projection reads is NaN or Inf (the mean of every
 * Gaussian of a job; its other geometry planes when it passes the near
 * plane; its SH planes when its rectangle meets the image). */
gs_status gs_project(const gs_params *params, const gs_frame *frame, const gs_raster_cfg *cfg,
                     void *rec_dev, uint32_t *meta_dev, uint32_t *status_dev, gs_stream stream);
gs_status gs_project_f64(const gs_params *params, const gs_frame *frame, const gs_raster_cfg *cfg,
                         void *rec_dev, uint32_t *meta_dev, uint32_t *status_dev, gs_stream stream);

/* Tile binning (no counterpart in the paper; an exact acceleration of the
 * per-pixel definition).  Emits one pair per (covered tile, record), sorts
 * the pairs by global tile id (LSD radix) and then each tile's list by the
 * unique key (depth bits, record), so every list is ordered by
 * (depth, record).  Writes vals, ranges, pair_off (the first pair of each
 * visible record in record order: the layout of the backward's per-pair
 * partials) and counters.  When the pairs exceed bins->capacity, sets
 * GS_STATUS_PAIR_OVERFLOW, stores the needed count in counters[GS_CTR_PAIRS]
 * (saturating at 2^32 - 1) and leaves vals/ranges truncated to the first
 * `capacity` pairs (in bounds, but not the frame's lists).  Every call that
 * ends with the overflow bit set (this call's or an earlier, uncleared one)
 * adds 1 to counters[GS_CTR_OVERFLOWED]: with the sticky bit, the optimiser
 * updates of that many steps were skipped and are to be redone.  The workspace
 * (device, caller-owned, at least gs_bin_sort_workspace_size bytes for the
 * frame's records, the bins' capacity and the frame's tiles) holds 8 bytes
 * per record, 16 per pair of capacity and 4 per tile, plus about 1 MiB. */
size_t gs_bin_sort_workspace_size(int64_t n_records, uint64_t capacity, int32_t n_tiles);
gs_status gs_bin_sort(const gs_frame *frame, const gs_raster_cfg *cfg, const uint32_t *meta_dev,
                      const gs_bins *bins, void *ws_dev, size_t ws_bytes, gs_stream stream);

/* gs_bin_sort for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): the same
 * kernels and results, with the workspace taken from a static device array
 * of the library (gs_bin_sort_noalloc_max_bytes() = 64 MiB per GPU, held
 * from the library's load to the end of the process) instead of a caller
 * buffer.  The caller still passes meta and the bins.  A frame whose
 * workspace (gs_bin_sort_workspace_size) exceeds that size gets
 * GS_E_CAPACITY and nothing is launched.  The call allocates nothing; its
 * first call on a device (the current one) looks up that device's copy of
 * the array.  Every call on one GPU shares the array, so calls that overlap
 * on one GPU (concurrent streams, or threads on one stream without ordering)
 * race and give undefined bins; calls ordered on one stream are safe.  No
 * content of the array carries from one call to the next. */
size_t gs_bin_sort_noalloc_max_bytes(void);
gs_status gs_bin_sort_noalloc(const gs_frame *frame, const gs_raster_cfg *cfg, const uint32_t *meta_dev,
                              const gs_bins *bins, gs_stream stream);

/* Forward compositing (Eq. 2) per pixel over its tile's list.  Writes
 * rgb [3][H][W] per job at 3*px0 (C + T bg), T_final [H][W] at px0 and
 * n_contrib (list position after the last contributor) at px0. */
gs_status gs_render_fwd(const gs_frame *frame, const gs_raster_cfg *cfg, const void *rec_dev,
                        const gs_bins *bins, void *rgb_dev, void *T_dev, uint32_t *n_contrib_dev,
                        gs_stream stream);
gs_status gs_render_fwd_f64(const gs_frame *frame, const gs_raster_cfg *cfg, const void *rec_dev,
                            const gs_bins *bins, void *rgb_dev, void *T_dev, uint32_t *n_contrib_dev,
                            gs_stream stream);
/* gs_render_fwd (FP32) that also adds the number of (pixel, Gaussian)
 * contributions of the frame (kept pairs of Eq. 2, each pixel up to its
 * termination) to *kept_dev (device uint64; the caller zeroes it).  Same
 * image; a measurement of the work the compositing passes do. */
gs_status gs_render_fwd_stats(const gs_frame *frame, const gs_raster_cfg *cfg, const void *rec_dev,
                              const gs_bins *bins, void *rgb_dev, void *T_dev, uint32_t *n_contrib_dev,
                              uint64_t *kept_dev, gs_stream stream);

/* Backward of the loss through compositing and projection to the raw
 * parameter planes.  GS_LOSS_L1: L = sum_jobs loss_weight * mean |C - target|
 * over 3HW (the L1 part of Eq. 3), target laid out like rgb; the per-job
 * loss is added to loss_out[job] (may be NULL).  GS_LOSS_EXTERNAL: grad_in is
 * dL/dC laid out like rgb.  rgb_dev and n_contrib_dev are the outputs of
 * gs_render_fwd for the same frame, records and bins (the contributor counts
 * carry the forward's stop decisions).  The transmittance is recomputed
 * front to back (never stored per pair).  grad->data receives dense gradient
 * planes (zero for Gaussians in no job or culled); grad must cover
 * params->n.  Workspace: gs_render_bwd_workspace_size bytes (nine partials
 * per tile pair and compositing wavefront, sized for up to 4 wavefronts per
 * tile). */
size_t gs_render_bwd_workspace_size(uint64_t capacity, int32_t f64);
gs_status gs_render_bwd(const gs_params *params, const gs_frame *frame, const gs_raster_cfg *cfg,
                        const void *rec_dev, const uint32_t *meta_dev, const gs_bins *bins,
                        const void *rgb_dev, const uint32_t *n_contrib_dev, gs_loss_mode mode,
                        const void *grad_in_dev, float *loss_out_dev, gs_params *grad, void *ws_dev,
                        size_t ws_bytes, gs_stream stream);
gs_status gs_render_bwd_f64(const gs_params *params, const gs_frame *frame, const gs_raster_cfg *cfg,
                            const void *rec_dev, const uint32_t *meta_dev, const gs_bins *bins,
                            const void *rgb_dev, const uint32_t *n_contrib_dev, gs_loss_mode mode,
                            const void *grad_in_dev, double *loss_out_dev, gs_params *grad, void *ws_dev,
                            size_t ws_bytes, gs_stream stream);

/* Photometric loss of Eq. 3 with its structural term, per job j:
 *   L_j = w_j (mean |C - target| + lambda (1 - mean SSIM)),
 * w_j = jobs[j].loss_weight, means over the job's 3 H W colour values.  SSIM
 * is that of Wang et al. (cited by the paper for its SSIM metric) under an
 * 11 x 11 Gaussian window of sigma 1.5 normalised to 1, zero outside the
 * image (a "same" correlation), per colour channel, C1 = 0.01^2,
 * C2 = 0.03^2; L_ssim = 1 - SSIM is the D-SSIM of the splatting recipe the
 * paper trains with.  rgb_dev / target_dev: planar [3][H][W] images at
 * 3 * px0 (as gs_render_fwd writes them).  grad_out_dev (same layout)
 * receives dL/dC (sign(0) = 0 for the L1 part): pass it to gs_render_bwd /
 * gs_render_bwd_adam with GS_LOSS_EXTERNAL.  loss_out_dev (float[n_jobs],
 * may be NULL) accumulates L_j; the caller zeroes it; its float additions
 * run in no fixed order.  cfg gives the binning tiles the frame was planned
 * with (its wavefront fields are not used).  Workspace (device, 4-byte
 * aligned): gs_ssim_workspace_size(frame->n_pixels) bytes (three FP32
 * derivative maps per colour value).  lambda >= 0 and finite; lambda = 0
 * gives the L1 loss alone. */
size_t gs_ssim_workspace_size(int64_t n_pixels);
gs_status gs_ssim_loss_grad(const gs_frame *frame, const gs_raster_cfg *cfg, const float *rgb_dev,
                            const float *target_dev, float lambda, float *grad_out_dev, float *loss_out_dev,
                            void *ws_dev, size_t ws_bytes, gs_stream stream);

/* x-update step of Eq. 8a: Adam (bias-corrected) on g + rho_a (x - w), where
 * w = z - u is the consensus target and rho_a the per-attribute penalty
 * (supplementary Sec. C).  w == NULL: no penalty.  mask (device float [n],
 * may be NULL): per-Gaussian penalty weight.  Updates x, m, v in place over
 * all x->n Gaussians; all five gs_params must share n and sh_degree.
 * status_dev (device uint32, may be NULL; e.g. the bins' counters +
 * GS_CTR_STATUS): while GS_STATUS_PAIR_OVERFLOW is set in it the update is
 * skipped (x, m, v untouched: a gradient from truncated tile lists must not
 * move the parameters); GS_STATUS_NONFINITE is OR-ed in when an updated
 * parameter or second moment is NaN or Inf, which any NaN or Inf among x, g,
 * m, v, w and mask leads to. */
gs_status gs_adam_admm(gs_params *x, const gs_params *g, gs_params *m, gs_params *v, const gs_params *w,
                       const float *mask_dev, const gs_adam_cfg *cfg, uint32_t *status_dev, gs_stream stream);

/* Backward and x-update of one local step in one call: gs_render_bwd in
 * FP32 followed by gs_adam_admm, with the gradient of each parameter plane
 * handed from the projection backward to the optimiser in registers (it is
 * never written to memory).  Same results, bit for bit, as gs_render_bwd
 * into a gradient buffer followed by gs_adam_admm on it.  Requires jobs over
 * disjoint Gaussian ranges (frame->jobs_disjoint; otherwise GS_E_UNSUPPORTED:
 * use the two calls); Gaussians in no job take the update with a zero
 * gradient.  x is read by the backward and updated in place; m, v, w, mask
 * and acfg as in gs_adam_admm, with bins->counters[GS_CTR_STATUS] as the
 * status word (the update is skipped after a pair overflow; non-finite
 * updates are flagged); the other arguments and the workspace as in
 * gs_render_bwd. */
gs_status gs_render_bwd_adam(gs_params *x, const gs_frame *frame, const gs_raster_cfg *cfg,
                             const void *rec_dev, const uint32_t *meta_dev, const gs_bins *bins,
                             const void *rgb_dev, const uint32_t *n_contrib_dev, gs_loss_mode mode,
                             const void *grad_in_dev, float *loss_out_dev, gs_params *m, gs_params *v,
                             const gs_params *w, const float *mask_dev, const gs_adam_cfg *acfg, void *ws_dev,
                             size_t ws_bytes, gs_stream stream);

/* Per-kernel timing with HIP events (measurement tooling; off by default).
 * gs_profile_set(names): comma-separated kernel names to time, "*" for all,
 * NULL or "" for none; resets every total.  While a kernel is selected, each
 * of its launches records a pair of events on its stream (a few microseconds
 * of device time).  gs_profile_get(name, &total_ms, &launches): waits for the
 * recorded launches of that kernel and returns their summed durations (0 and
 * 0 for a kernel never launched). */
gs_status gs_profile_set(const char *names);
gs_status gs_profile_get(const char *name, double *total_ms, int64_t *launches);
/* gs_profile_enable(on): on = 0 stops the selected kernels from recording
 * events, keeping their totals and the selection; on != 0 resumes
 * recording.  A caller can so time a sample of the launches of a long run
 * without paying the event pairs on every launch.  gs_profile_set resumes
 * recording as well.  Host-side only; never fails. */
gs_status gs_profile_enable(int32_t on);

/* Tile-shape autotuner (no counterpart in the paper: a choice of launch
 * shapes for the batched K-block step of Alg. 2, S1).  A candidate is a
 * binning tile and the wavefronts per tile of the forward and the backward
 * compositing passes (the fields of gs_raster_cfg they set; each must be a
 * combination gs_raster_cfg accepts).  The workgroup is always 4
 * wavefronts: the adaptive split puts a tile's wavefronts in one workgroup. */
typedef struct {
    int32_t tile_w, tile_h;
    int32_t fwd_waves, bwd_waves;
} gs_tune_choice;

/* One step of the caller's workload with the given launch shapes, enqueued on
 * the stream handed to gs_autotune (or synchronous); returns 0 on success. */
typedef int32_t (*gs_tune_step_fn)(const gs_tune_choice *choice, void *user);

/* Cache of tuned choices: path of a JSON file ({"<key>": {"tile": [w, h,
 * fwd, bwd], "ms": {...}}}) read now and rewritten after each new tuning, or
 * NULL for an in-memory cache only.  Clears the in-memory cache first.
 * GS_E_INVALID for a file that is not such JSON (the cache is then empty).
 * Without a call, the cache is in memory only. */
gs_status gs_set_tune_cache(const char *path);

/* Fastest of n_candidates launch shapes for the workload named shape_key:
 * when the key is cached, *best (and *best_ms, the cached time or -1) come
 * from the cache and step is never called.  Otherwise, per candidate, step is
 * called once untimed, then reps times between two HIP events on `stream`;
 * the candidate with the least time per step wins (ties: the first), is
 * cached under shape_key and returned.  best_ms (may be NULL) receives its
 * milliseconds per step.  Errors: GS_E_INVALID for null or empty arguments,
 * n_candidates or reps below 1, an invalid candidate or a step that returns
 * non-zero; GS_E_DEVICE when the events fail. */
gs_status gs_autotune(const char *shape_key, const gs_tune_choice *candidates, int32_t n_candidates, int32_t reps,
                      gs_tune_step_fn step, void *user, gs_stream stream, gs_tune_choice *best, double *best_ms);

/* Consensus step (Eq. 8b-c, Alg. 2) over K blocks held in one parameter
 * store.  For each global id gid with local holders
 * holder_idx[holder_ptr[gid] .. holder_ptr[gid+1]) (ascending block order):
 *   xh_k = relax * x_k + (1 - relax) * z_gid   (over-relaxation; relax = 1: none)
 *   z_gid = mean_k xh_k;  u_k += xh_k - z_gid;  w_k = z_gid - u_k.
 * z_global is read (previous z) and overwritten.  resid_out (device float[10],
 * may be NULL) accumulates, per attribute group (p, q, s, f, o), the squared
 * residual sums of Sec. 3.3 over every local copy of every held Gaussian:
 * [0..4] primal sum_k (x_k - z)^2 with the unrelaxed x_k; [5..9] dual
 * sum_k (z - z_prev)^2, i.e. |H| (z - z_prev)^2 per global id (the penalty
 * factor of s = rho (z - z_prev) is left to gs_penalty_update).  The caller
 * zeroes it; the order of the float additions varies from call to call.
 * A copy whose Gaussian has a single holder gets z = x exactly, so its u is
 * not rewritten. */
gs_status gs_consensus(const gs_params *x_local, gs_params *u_local, gs_params *w_local, gs_params *z_global,
                       const int64_t *holder_ptr_dev, const int64_t *holder_idx_dev, float relax,
                       float *resid_out_dev, gs_stream stream);

/* Residual-balancing penalty update of Sec. 3.3 (host only, no device work).
 * resid_host: the 10 sums gs_consensus accumulated (copied to the host).
 * Per group k, with ||r|| = sqrt(resid[k]) and ||s|| = rho[k] sqrt(resid[5+k]):
 *   rho[k] *= tau_inc when ||r|| > mu ||s||;  rho[k] /= tau_dec when
 *   ||s|| > mu ||r||;  unchanged otherwise (decisions taken in double).
 * rho (host float[5]) is updated in place; scale_out (host float[5], may be
 * NULL) receives old rho / new rho, the factor gs_dual_rescale applies to the
 * scaled duals.  Requires mu > 1, tau_inc >= 1, tau_dec >= 1 and finite,
 * non-negative sums; on error nothing is written. */
gs_status gs_penalty_update(const float *resid_host, float *rho_host, float mu, float tau_inc, float tau_dec,
                            float *scale_out_host);

/* Scaled duals after a penalty change (Sec. 3.3 with the scaled form of
 * Eq. 7: u = y / rho, so keeping y while rho becomes rho' multiplies u by
 * rho / rho').  For every local copy k of every held global id and every
 * plane of group g: u_k *= scale_host[g]; w_k = z_gid - u_k.  Entries whose u
 * does not change (u = 0, or scale 1) are left untouched, so w must already
 * equal z - u there, as gs_consensus leaves it.  Groups with scale 1 are not
 * read.  u_local/w_local as in gs_consensus; z_global is read only. */
gs_status gs_dual_rescale(gs_params *u_local, gs_params *w_local, const gs_params *z_global,
                          const int64_t *holder_ptr_dev, const int64_t *holder_idx_dev, const float *scale_host,
                          gs_stream stream);

/* Scene splitting into K blocks (Alg. 1; host only, no device work).
 * points (host double [n][3]): the initial point cloud.  Starting from the
 * tight box of all points, rounds cut every current cell (first in, first
 * out) in two along its longer ground axis and append the two re-tightened
 * halves, until there are K cells (the last round stops at K).  The cut
 * puts the floor(m/2) points of a cell with the smallest (coordinate, point
 * id) in the first half (a median cut: blocks of similar point counts).
 * ground_axes: bit mask of the axes that may be cut (the paper assumes one
 * axis is aligned with the ground; 5 = x and z with y up).  Ties between
 * axis extents go to the lower axis.  boxes (host double [K][6], lo xyz then
 * hi xyz) receives the cells' tight boxes in the algorithm's order;
 * cell_of (host int64 [n], may be NULL) each point's cell.  Requires
 * 1 <= K <= n and finite coordinates. */
gs_status gs_split_scene(const double *points_host, int64_t n, int32_t K, int32_t ground_axes,
                         double *boxes_host, int64_t *cell_of_host);

/* Overlap grouping (Sec. 3.2, scene splitting): block k holds every point
 * (or camera centre) covered by its cell box scaled by `scale` (>= 1; the
 * paper uses 1.4) about the box centre, computed as each side moved out by
 * (scale - 1) / 2 of the box extent, bounds inclusive, on the axes of the
 * test_axes bit mask (7 for points; the ground axes for camera centres,
 * which lie above the point cloud, so that views follow their ground-plane
 * cell as the paper assigns them).  counts (host int64
 * [K]) and *total receive the block sizes; members (host int64, may be
 * NULL), when capacity >= *total, receives block 0's point ids ascending,
 * then block 1's, ...; a smaller non-NULL buffer gives GS_E_CAPACITY after
 * the counts are written. */
gs_status gs_split_group(const double *boxes_host, int32_t K, double scale, int32_t test_axes,
                         const double *points_host, int64_t n, int64_t *counts_host, int64_t *members_host,
                         int64_t capacity, int64_t *total_host);

/* Storage order for a Gaussian store (no counterpart in the paper; a memory
 * layout).  perm_host (int64 [n]) receives the Gaussians in Z-order
 * (Morton order) of their means: mean_host holds the three mean planes
 * (host FP32, plane a at mean_host + a * stride, stride >= n); each
 * coordinate is quantised to `bits` (1..21) bits over the bounding box of
 * the means, the bits are interleaved (x lowest, then y, then z, from the
 * least significant level up) and ties keep index order.  With strands > 1
 * the Z-ordered sequence is cut into chunks of `chunk` Gaussians (the tail
 * of n mod chunk stays last) and strand s (0 .. strands-1) takes chunks
 * s, s + strands, s + 2 strands, ..., the strands one after another.
 * Storing a model as params[:, perm] puts Gaussians that are close in space
 * close in memory: what one view sees then forms long runs (or, with
 * strands, whole chunks), which the projection and the compositing read in
 * whole cache lines; the strands spread each region over the store, so that
 * a workgroup's consecutive Gaussians mix seen and unseen ones.  Renders of
 * the permuted model equal those of the original except where two Gaussians
 * have the same depth bits (their order follows the index). */
gs_status gs_spatial_order(const float *mean_host, int64_t n, int64_t stride, int32_t bits, int32_t chunk,
                           int32_t strands, int64_t *perm_host);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
