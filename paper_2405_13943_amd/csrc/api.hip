// C ABI of libgs (declared in include/gs.h): argument validation, workspace
// sizing and kernel launches.  No device memory is allocated here.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "gs_internal.hpp"

namespace {

thread_local char g_err[512] = "";

gs_status fail(gs_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

gs_status check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(GS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    g_err[0] = 0;
    return GS_OK;
}

gs_status check_params(const gs_params* p, const char* name, bool allow_null_data = false) {
    if (!p) return fail(GS_E_INVALID, "%s: null gs_params", name);
    if (p->n < 0) return fail(GS_E_INVALID, "%s: negative n", name);
    if (p->stride < p->n) return fail(GS_E_INVALID, "%s: stride %lld < n %lld", name, (long long)p->stride, (long long)p->n);
    if (p->sh_degree < 0 || p->sh_degree > 3) return fail(GS_E_INVALID, "%s: sh_degree %d outside 0..3", name, p->sh_degree);
    if (!p->data && !(allow_null_data || p->n == 0)) return fail(GS_E_INVALID, "%s: null data", name);
    return GS_OK;
}

bool waves_ok(const gs_raster_cfg* c, int waves) {
    const int S = waves == 0 ? 1 : waves;
    if (c->tile_w == 8 && c->tile_h == 8) return S == 1;
    if (c->tile_w == 16 && c->tile_h == 8) return S == 1 || S == 2;
    if ((c->tile_w == 16 && c->tile_h == 16) || (c->tile_w == 32 && c->tile_h == 8)) return S == 1 || S == 2 || S == 4;
    return false;
}

bool tile_ok(const gs_raster_cfg* c) {
    auto ok = [&](int w) { return w == GS_WAVES_ADAPTIVE ? waves_ok(c, 1) : waves_ok(c, w); };
    return ok(c->fwd_waves) && ok(c->bwd_waves);
}

gs_status check_frame(const gs_frame* f, const gs_raster_cfg* cfg) {
    if (!f || !cfg) return fail(GS_E_INVALID, "null frame or raster config");
    if (f->n_jobs < 0 || f->n_tiles < 0 || f->n_records < 0 || f->n_pixels < 0 || f->g_max < 0)
        return fail(GS_E_INVALID, "negative frame totals");
    if (f->n_jobs > 0 && (!f->cams || !f->jobs)) return fail(GS_E_INVALID, "null cams/jobs");
    if (f->n_records >= (int64_t(1) << 32)) return fail(GS_E_UNSUPPORTED, "more than 2^32 - 1 records");
    if (!tile_ok(cfg))
        return fail(GS_E_INVALID, "tile %dx%d with %d/%d wavefronts per tile (fwd/bwd): not one of 8x8/1, 16x8/1-2, "
                    "16x16/1-2-4, 32x8/1-2-4", cfg->tile_w, cfg->tile_h, cfg->fwd_waves, cfg->bwd_waves);
    if (!(cfg->alpha_min > 0.f) || !(cfg->alpha_max > cfg->alpha_min) || !(cfg->alpha_max < 1.f) ||
        !(cfg->T_min > 0.f) || !(cfg->near_z > 0.f) || !(cfg->dilation >= 0.f) || !(cfg->jac_clip > 0.f))
        return fail(GS_E_INVALID, "raster constants out of range");
    return GS_OK;
}

gs_status check_bins(const gs_bins* b, const gs_frame* f, const gs_raster_cfg* cfg = nullptr) {
    if (!b) return fail(GS_E_INVALID, "null gs_bins");
    if (cfg && !b->tile_order && (cfg->fwd_waves == GS_WAVES_ADAPTIVE || cfg->bwd_waves == GS_WAVES_ADAPTIVE))
        return fail(GS_E_INVALID, "adaptive wavefronts need gs_bins.tile_order");
    if (!b->counters || !b->ranges || (!b->pair_off && f->n_records > 0) || (!b->vals && b->capacity > 0))
        return fail(GS_E_INVALID, "null gs_bins buffer");
    if (b->capacity >= (uint64_t(1) << 32)) return fail(GS_E_UNSUPPORTED, "pair capacity must be below 2^32");
    return GS_OK;
}

template <typename T>
gs_status project_impl(const gs_params* params, const gs_frame* frame, const gs_raster_cfg* cfg, void* rec,
                       uint32_t* meta, uint32_t* status, gs_stream stream) {
    gs_status st;
    if ((st = check_params(params, "params")) != GS_OK) return st;
    if ((st = check_frame(frame, cfg)) != GS_OK) return st;
    if (frame->g_max > params->n) return fail(GS_E_INVALID, "jobs reach Gaussian %lld, params hold %lld",
                                              (long long)frame->g_max, (long long)params->n);
    if (frame->n_records > 0 && (!rec || !meta)) return fail(GS_E_INVALID, "null record buffers");
    return check_hip(gs::launch_project<T>(*params, *frame, *cfg, static_cast<T*>(rec), meta, status,
                                           (hipStream_t)stream),
                     "gs_project");
}

template <typename T>
gs_status render_fwd_impl(const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec, const gs_bins* bins,
                          void* rgb, void* Tf, uint32_t* nc, gs_stream stream, uint64_t* kept = nullptr) {
    gs_status st;
    if ((st = check_frame(frame, cfg)) != GS_OK) return st;
    if ((st = check_bins(bins, frame, cfg)) != GS_OK) return st;
    if (frame->n_pixels > 0 && (!rgb || !Tf || !nc)) return fail(GS_E_INVALID, "null image buffers");
    if (frame->n_records > 0 && !rec) return fail(GS_E_INVALID, "null record buffer");
    return check_hip(gs::launch_render_fwd<T>(*frame, *cfg, static_cast<const T*>(rec), *bins, static_cast<T*>(rgb),
                                              static_cast<T*>(Tf), nc, reinterpret_cast<unsigned long long*>(kept),
                                              (hipStream_t)stream),
                     "gs_render_fwd");
}

// nine partials per tile pair and compositing wavefront, up to 4 wavefronts per tile
size_t bwd_ws(uint64_t capacity, int f64) {
    const size_t e = f64 ? sizeof(double) : sizeof(float);
    return size_t(capacity > 0 ? capacity : 1) * 9 * 4 * e;
}

template <typename T>
gs_status render_bwd_impl(const gs_params* params, const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec,
                          const uint32_t* meta, const gs_bins* bins, const void* rgb, const uint32_t* nc,
                          gs_loss_mode mode, const void* gin, T* loss, gs_params* grad, void* ws, size_t ws_bytes,
                          gs_stream stream) {
    gs_status st;
    if ((st = check_params(params, "params")) != GS_OK) return st;
    if ((st = check_params(grad, "grad")) != GS_OK) return st;
    if ((st = check_frame(frame, cfg)) != GS_OK) return st;
    if ((st = check_bins(bins, frame, cfg)) != GS_OK) return st;
    if (grad->n != params->n || grad->sh_degree != params->sh_degree)
        return fail(GS_E_INVALID, "grad planes do not match params");
    if (frame->g_max > params->n) return fail(GS_E_INVALID, "jobs reach Gaussian %lld, params hold %lld",
                                              (long long)frame->g_max, (long long)params->n);
    if (mode != GS_LOSS_L1 && mode != GS_LOSS_EXTERNAL) return fail(GS_E_INVALID, "unknown loss mode");
    if (frame->n_pixels > 0 && (!rgb || !nc || !gin))
        return fail(GS_E_INVALID, "null image, contributor count or gradient input");
    if (frame->n_records > 0 && (!rec || !meta)) return fail(GS_E_INVALID, "null record buffers");
    if (!ws || ws_bytes < bwd_ws(bins->capacity, sizeof(T) == 8))
        return fail(GS_E_CAPACITY, "backward workspace too small (%zu < %zu)", ws_bytes,
                    bwd_ws(bins->capacity, sizeof(T) == 8));
    T* pg = static_cast<T*>(ws);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gs::launch_render_bwd<T>(*frame, *cfg, static_cast<const T*>(rec), meta, *bins,
                                            static_cast<const T*>(rgb), nc, mode, static_cast<const T*>(gin), loss,
                                            pg, s);
    if (e != hipSuccess) return check_hip(e, "gs_render_bwd (composite)");
    return check_hip(gs::launch_project_bwd<T>(*params, *frame, *cfg, static_cast<const T*>(rec), meta, *bins, pg,
                                               *grad, s),
                     "gs_render_bwd (projection)");
}

}  // namespace

extern "C" {

int32_t gs_abi_version(void) { return GS_ABI_VERSION; }

const char* gs_last_error(void) { return g_err; }

void gs_raster_cfg_default(gs_raster_cfg* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->tile_w = 16;
    cfg->tile_h = 16;
    cfg->near_z = 0.2f;
    cfg->alpha_min = 1.0f / 255.0f;
    cfg->alpha_max = 0.99f;
    cfg->T_min = 1e-4f;
    cfg->dilation = 0.3f;
    cfg->jac_clip = 1.3f;
    cfg->fwd_waves = 1;
    cfg->bwd_waves = 1;
}

gs_status gs_frame_plan(const gs_camera* cams, int32_t n_cams, gs_job* jobs, int32_t n_jobs, const gs_raster_cfg* cfg,
                        int64_t* n_records, int64_t* n_pixels, int32_t* n_tiles, int64_t* g_max,
                        int32_t* jobs_disjoint) {
    if (!cfg || !tile_ok(cfg)) return fail(GS_E_INVALID, "bad raster config / tile shape");
    if (n_jobs < 0 || n_cams < 0 || (n_jobs > 0 && (!jobs || !cams))) return fail(GS_E_INVALID, "bad job list");
    int64_t rec = 0, px = 0, tiles = 0, gmax = 0;
    for (int32_t j = 0; j < n_jobs; j++) {
        gs_job& J = jobs[j];
        if (J.cam < 0 || J.cam >= n_cams) return fail(GS_E_INVALID, "job %d: camera %d out of range", j, J.cam);
        if (J.g0 < 0 || J.g1 < J.g0) return fail(GS_E_INVALID, "job %d: bad Gaussian range", j);
        const gs_camera& c = cams[J.cam];
        if (c.width <= 0 || c.height <= 0 || c.width > 65535 * 8 || c.height > 65535 * 8)
            return fail(GS_E_INVALID, "job %d: bad image size", j);
        if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(GS_E_INVALID, "job %d: bad focal length", j);
        J.tiles_x = (c.width + cfg->tile_w - 1) / cfg->tile_w;
        J.tiles_y = (c.height + cfg->tile_h - 1) / cfg->tile_h;
        J.tile0 = int32_t(tiles);
        J.rec0 = rec;
        J.px0 = px;
        tiles += int64_t(J.tiles_x) * J.tiles_y;
        rec += J.g1 - J.g0;
        if (J.g1 > gmax) gmax = J.g1;
        px += int64_t(c.width) * c.height;
        if (tiles >= (int64_t(1) << 31)) return fail(GS_E_UNSUPPORTED, "too many tiles");
        if (int64_t(J.tiles_x) * J.tiles_y >= (int64_t(1) << 24))
            return fail(GS_E_UNSUPPORTED, "job %d: more than 2^24 tiles in one view", j);
    }
    int32_t disjoint = 1;
    for (int32_t a = 0; a < n_jobs && disjoint; a++)
        for (int32_t b = a + 1; b < n_jobs; b++)
            if (jobs[a].g0 < jobs[b].g1 && jobs[b].g0 < jobs[a].g1 && jobs[a].g1 > jobs[a].g0 &&
                jobs[b].g1 > jobs[b].g0) {
                disjoint = 0;
                break;
            }
    if (n_records) *n_records = rec;
    if (n_pixels) *n_pixels = px;
    if (n_tiles) *n_tiles = int32_t(tiles);
    if (g_max) *g_max = gmax;
    if (jobs_disjoint) *jobs_disjoint = disjoint;
    g_err[0] = 0;
    return GS_OK;
}

gs_status gs_project(const gs_params* params, const gs_frame* frame, const gs_raster_cfg* cfg, void* rec,
                     uint32_t* meta, uint32_t* status, gs_stream stream) {
    return project_impl<float>(params, frame, cfg, rec, meta, status, stream);
}

gs_status gs_project_f64(const gs_params* params, const gs_frame* frame, const gs_raster_cfg* cfg, void* rec,
                         uint32_t* meta, uint32_t* status, gs_stream stream) {
    return project_impl<double>(params, frame, cfg, rec, meta, status, stream);
}

size_t gs_bin_sort_workspace_size(int64_t n_records, uint64_t capacity, int32_t n_tiles) {
    return gs::bin_workspace_size(n_records, capacity, n_tiles);
}

gs_status gs_bin_sort(const gs_frame* frame, const gs_raster_cfg* cfg, const uint32_t* meta, const gs_bins* bins,
                      void* ws, size_t ws_bytes, gs_stream stream) {
    gs_status st;
    if ((st = check_frame(frame, cfg)) != GS_OK) return st;
    if ((st = check_bins(bins, frame, cfg)) != GS_OK) return st;
    if (frame->n_records > 0 && !meta) return fail(GS_E_INVALID, "null meta");
    const size_t need = gs::bin_workspace_size(frame->n_records, bins->capacity, frame->n_tiles);
    if (!ws || ws_bytes < need) return fail(GS_E_CAPACITY, "binning workspace too small (%zu < %zu)", ws_bytes, need);
    return check_hip(gs::launch_bin_sort(*frame, *cfg, meta, *bins, ws, ws_bytes, (hipStream_t)stream), "gs_bin_sort");
}

// ---------------------------------------------------------------------------
// Binning without a caller workspace: the workspace lives in `scratch`, a
// device array of this file that each GPU holds from the library's load to
// the end of the process.  Host code never passes `scratch` itself (on the
// host the name stands for a host-side shadow, not a device address): the
// device address is looked up once per device, with that device current, and
// kept in g_scratch_dev.

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// device address of the current device's scratch (looked up on first use)
gs_status scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GS_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(GS_E_UNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GS_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return GS_OK;
}

}  // namespace

gs_status gs_set_tune_cache(const char* path) {
    std::string err;
    const gs_status st = gs::tune_set_cache(path, err);
    return st == GS_OK ? GS_OK : fail(st, "%s", err.c_str());
}

gs_status gs_autotune(const char* key, const gs_tune_choice* cand, int32_t n, int32_t reps, gs_tune_step_fn step,
                      void* user, gs_stream stream, gs_tune_choice* best, double* best_ms) {
    if (!key || !*key || !cand || !step || !best) return fail(GS_E_INVALID, "null or empty autotune argument");
    if (n < 1 || reps < 1) return fail(GS_E_INVALID, "autotune needs at least one candidate and one repetition");
    for (int32_t i = 0; i < n; i++) {
        gs_raster_cfg c;
        gs_raster_cfg_default(&c);
        c.tile_w = cand[i].tile_w;
        c.tile_h = cand[i].tile_h;
        c.fwd_waves = int16_t(cand[i].fwd_waves);
        c.bwd_waves = int16_t(cand[i].bwd_waves);
        if (cand[i].fwd_waves != c.fwd_waves || cand[i].bwd_waves != c.bwd_waves || !tile_ok(&c))
            return fail(GS_E_INVALID, "candidate %d: tile %dx%d with %d/%d wavefronts is not a valid launch shape", i,
                        cand[i].tile_w, cand[i].tile_h, cand[i].fwd_waves, cand[i].bwd_waves);
    }
    std::string err;
    bool found = false;
    gs_status st = gs::tune_lookup(key, best, best_ms, &found, err);
    if (st != GS_OK) return fail(st, "%s", err.c_str());
    if (found) return GS_OK;
    st = gs::tune_run(key, cand, n, reps, step, user, (hipStream_t)stream, best, best_ms, err);
    return st == GS_OK ? GS_OK : fail(st, "%s", err.c_str());
}

size_t gs_bin_sort_noalloc_max_bytes(void) { return kScratchBytes; }

gs_status gs_bin_sort_noalloc(const gs_frame* frame, const gs_raster_cfg* cfg, const uint32_t* meta,
                              const gs_bins* bins, gs_stream stream) {
    gs_status st;
    if ((st = check_frame(frame, cfg)) != GS_OK) return st;
    if ((st = check_bins(bins, frame, cfg)) != GS_OK) return st;
    if (frame->n_records > 0 && !meta) return fail(GS_E_INVALID, "null meta");
    const size_t need = gs::bin_workspace_size(frame->n_records, bins->capacity, frame->n_tiles);
    if (need > kScratchBytes)
        return fail(GS_E_CAPACITY, "binning needs %zu workspace bytes for %lld records, %llu pairs and %d tiles; "
                    "the static scratch holds %zu: use gs_bin_sort with a caller workspace", need,
                    (long long)frame->n_records, (unsigned long long)bins->capacity, frame->n_tiles, kScratchBytes);
    void* ws = nullptr;
    if ((st = scratch_address(&ws)) != GS_OK) return st;
    return check_hip(gs::launch_bin_sort(*frame, *cfg, meta, *bins, ws, kScratchBytes, (hipStream_t)stream),
                     "gs_bin_sort_noalloc");
}

gs_status gs_render_fwd(const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec, const gs_bins* bins, void* rgb,
                        void* T, uint32_t* nc, gs_stream stream) {
    return render_fwd_impl<float>(frame, cfg, rec, bins, rgb, T, nc, stream);
}

gs_status gs_render_fwd_stats(const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec, const gs_bins* bins,
                              void* rgb, void* Tf, uint32_t* nc, uint64_t* kept, gs_stream stream) {
    if (!kept) return fail(GS_E_INVALID, "null contribution counter");
    return render_fwd_impl<float>(frame, cfg, rec, bins, rgb, Tf, nc, stream, kept);
}

gs_status gs_render_fwd_f64(const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec, const gs_bins* bins,
                            void* rgb, void* T, uint32_t* nc, gs_stream stream) {
    return render_fwd_impl<double>(frame, cfg, rec, bins, rgb, T, nc, stream);
}

size_t gs_render_bwd_workspace_size(uint64_t capacity, int32_t f64) { return bwd_ws(capacity, f64); }

size_t gs_ssim_workspace_size(int64_t n_pixels) { return n_pixels > 0 ? gs::ssim_workspace_size(n_pixels) : 0; }

gs_status gs_ssim_loss_grad(const gs_frame* frame, const gs_raster_cfg* cfg, const float* rgb, const float* tgt,
                            float lambda, float* grad, float* loss, void* ws, size_t ws_bytes, gs_stream stream) {
    gs_status st;
    if ((st = check_frame(frame, cfg)) != GS_OK) return st;
    if (!(lambda >= 0.f) || !std::isfinite(lambda)) return fail(GS_E_INVALID, "lambda %g not finite and >= 0", double(lambda));
    if (frame->n_pixels == 0) return GS_OK;
    if (!rgb || !tgt || !grad) return fail(GS_E_INVALID, "null image, target or gradient");
    if (frame->n_tiles == 0) return GS_OK;
    const size_t need = gs::ssim_workspace_size(frame->n_pixels);
    if (!ws || ws_bytes < need) return fail(GS_E_CAPACITY, "ssim workspace %zu bytes < %zu", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(ws) & 3) != 0) return fail(GS_E_INVALID, "ssim workspace not 4-byte aligned");
    return check_hip(gs::launch_ssim_loss_grad(*frame, *cfg, rgb, tgt, lambda, grad, loss, ws, (hipStream_t)stream),
                     "gs_ssim_loss_grad");
}

gs_status gs_render_bwd(const gs_params* params, const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec,
                        const uint32_t* meta, const gs_bins* bins, const void* rgb, const uint32_t* n_contrib,
                        gs_loss_mode mode, const void* gin, float* loss, gs_params* grad, void* ws, size_t ws_bytes,
                        gs_stream stream) {
    return render_bwd_impl<float>(params, frame, cfg, rec, meta, bins, rgb, n_contrib, mode, gin, loss, grad, ws,
                                  ws_bytes, stream);
}

gs_status gs_render_bwd_f64(const gs_params* params, const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec,
                            const uint32_t* meta, const gs_bins* bins, const void* rgb, const uint32_t* n_contrib,
                            gs_loss_mode mode, const void* gin, double* loss, gs_params* grad, void* ws,
                            size_t ws_bytes, gs_stream stream) {
    return render_bwd_impl<double>(params, frame, cfg, rec, meta, bins, rgb, n_contrib, mode, gin, loss, grad, ws,
                                   ws_bytes, stream);
}

namespace {

// x, m, v (and w when given) are planes of one shape; g too when given
gs_status check_adam(const gs_params* x, const gs_params* g, const gs_params* m, const gs_params* v,
                     const gs_params* w, const float* mask, const gs_adam_cfg* cfg) {
    gs_status st;
    if ((st = check_params(x, "x")) != GS_OK) return st;
    if (g && (st = check_params(g, "g")) != GS_OK) return st;
    if ((st = check_params(m, "m")) != GS_OK) return st;
    if ((st = check_params(v, "v")) != GS_OK) return st;
    if (w && (st = check_params(w, "w")) != GS_OK) return st;
    if (!cfg) return fail(GS_E_INVALID, "null adam config");
    const gs_params* all[4] = {g, m, v, w};
    for (const gs_params* p : all)
        if (p && (p->n != x->n || p->sh_degree != x->sh_degree))
            return fail(GS_E_INVALID, "adam planes disagree in n or sh_degree");
    if (cfg->step < 1) return fail(GS_E_INVALID, "adam step must be >= 1");
    if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps >= 0.f))
        return fail(GS_E_INVALID, "adam betas/eps out of range");
    if (mask && !w) return fail(GS_E_INVALID, "mask given without a consensus target");
    return GS_OK;
}

}  // namespace

gs_status gs_adam_admm(gs_params* x, const gs_params* g, gs_params* m, gs_params* v, const gs_params* w,
                       const float* mask, const gs_adam_cfg* cfg, uint32_t* status, gs_stream stream) {
    gs_status st;
    if (!g) return fail(GS_E_INVALID, "g: null gs_params");
    if ((st = check_adam(x, g, m, v, w, mask, cfg)) != GS_OK) return st;
    return check_hip(gs::launch_adam_admm(*x, *g, *m, *v, w, mask, *cfg, status, (hipStream_t)stream),
                     "gs_adam_admm");
}

gs_status gs_render_bwd_adam(gs_params* x, const gs_frame* frame, const gs_raster_cfg* cfg, const void* rec,
                             const uint32_t* meta, const gs_bins* bins, const void* rgb, const uint32_t* n_contrib,
                             gs_loss_mode mode, const void* gin, float* loss, gs_params* m, gs_params* v,
                             const gs_params* w,
                             const float* mask, const gs_adam_cfg* acfg, void* ws, size_t ws_bytes,
                             gs_stream stream) {
    gs_status st;
    if ((st = check_adam(x, nullptr, m, v, w, mask, acfg)) != GS_OK) return st;
    if ((st = check_frame(frame, cfg)) != GS_OK) return st;
    if ((st = check_bins(bins, frame, cfg)) != GS_OK) return st;
    if (!frame->jobs_disjoint)
        return fail(GS_E_UNSUPPORTED, "jobs share Gaussians: call gs_render_bwd, then gs_adam_admm");
    if (frame->g_max > x->n) return fail(GS_E_INVALID, "jobs reach Gaussian %lld, params hold %lld",
                                         (long long)frame->g_max, (long long)x->n);
    if (mode != GS_LOSS_L1 && mode != GS_LOSS_EXTERNAL) return fail(GS_E_INVALID, "unknown loss mode");
    if (frame->n_pixels > 0 && (!rgb || !n_contrib || !gin))
        return fail(GS_E_INVALID, "null image, contributor count or gradient input");
    if (frame->n_records > 0 && (!rec || !meta)) return fail(GS_E_INVALID, "null record buffers");
    if (!ws || ws_bytes < bwd_ws(bins->capacity, 0))
        return fail(GS_E_CAPACITY, "backward workspace too small (%zu < %zu)", ws_bytes, bwd_ws(bins->capacity, 0));
    float* pg = static_cast<float*>(ws);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gs::launch_render_bwd<float>(*frame, *cfg, static_cast<const float*>(rec), meta, *bins,
                                                static_cast<const float*>(rgb), n_contrib, mode,
                                                static_cast<const float*>(gin), loss, pg, s);
    if (e != hipSuccess) return check_hip(e, "gs_render_bwd_adam (composite)");
    return check_hip(gs::launch_project_bwd_adam(*x, *frame, *cfg, static_cast<const float*>(rec), meta, *bins, pg,
                                                 *m, *v, w, mask, *acfg, s),
                     "gs_render_bwd_adam (projection + optimiser)");
}

gs_status gs_consensus(const gs_params* x, gs_params* u, gs_params* w, gs_params* z, const int64_t* hptr,
                       const int64_t* hidx, float relax, float* resid, gs_stream stream) {
    gs_status st;
    if ((st = check_params(x, "x_local")) != GS_OK) return st;
    if ((st = check_params(u, "u_local")) != GS_OK) return st;
    if ((st = check_params(w, "w_local")) != GS_OK) return st;
    if ((st = check_params(z, "z_global")) != GS_OK) return st;
    if (u->n != x->n || w->n != x->n) return fail(GS_E_INVALID, "local planes disagree in n");
    if (u->sh_degree != x->sh_degree || w->sh_degree != x->sh_degree || z->sh_degree != x->sh_degree)
        return fail(GS_E_INVALID, "planes disagree in sh_degree");
    if (z->n > 0 && (!hptr || !hidx)) return fail(GS_E_INVALID, "null holder CSR");
    if (!(relax > 0.f && relax < 2.f)) return fail(GS_E_INVALID, "relaxation %g outside (0, 2)", double(relax));
    if (x->n >= (int64_t(1) << 30) || z->n >= (int64_t(1) << 30))
        return fail(GS_E_INVALID, "consensus supports fewer than 2^30 local and global columns");
    return check_hip(gs::launch_consensus(*x, *u, *w, *z, hptr, hidx, relax, resid, (hipStream_t)stream),
                     "gs_consensus");
}

gs_status gs_penalty_update(const float* resid, float* rho, float mu, float tau_inc, float tau_dec, float* scale) {
    if (!resid || !rho) return fail(GS_E_INVALID, "null resid or rho");
    if (!(mu > 1.f) || !(tau_inc >= 1.f) || !(tau_dec >= 1.f) || !std::isfinite(mu) || !std::isfinite(tau_inc) ||
        !std::isfinite(tau_dec))
        return fail(GS_E_INVALID, "penalty update needs mu > 1 and tau >= 1 (got %g, %g, %g)", double(mu),
                    double(tau_inc), double(tau_dec));
    float out[5];
    for (int k = 0; k < 5; k++) {
        const double rp = resid[k], rd = resid[5 + k], r0 = rho[k];
        if (!(rp >= 0) || !(rd >= 0) || !std::isfinite(rp) || !std::isfinite(rd))
            return fail(GS_E_INVALID, "residual sums of group %d not finite and >= 0", k);
        if (!(r0 > 0) || !std::isfinite(r0)) return fail(GS_E_INVALID, "rho[%d] = %g not positive", k, r0);
        const double r = std::sqrt(rp), sn = r0 * std::sqrt(rd);
        double nr = r0;
        if (r > double(mu) * sn) nr = r0 * double(tau_inc);
        else if (sn > double(mu) * r) nr = r0 / double(tau_dec);
        out[k] = float(nr);
    }
    for (int k = 0; k < 5; k++) {
        if (scale) scale[k] = rho[k] / out[k];
        rho[k] = out[k];
    }
    return GS_OK;
}

gs_status gs_spatial_order(const float* mean, int64_t n, int64_t stride, int32_t bits, int32_t chunk, int32_t strands,
                           int64_t* perm) {
    if (n < 0) return fail(GS_E_INVALID, "negative n");
    if (n == 0) return GS_OK;
    if (!mean || !perm) return fail(GS_E_INVALID, "null means or permutation");
    if (stride < n) return fail(GS_E_INVALID, "stride %lld below n %lld", (long long)stride, (long long)n);
    if (bits < 1 || bits > 21) return fail(GS_E_INVALID, "bits %d not in 1..21", bits);
    if (chunk < 1 || strands < 1) return fail(GS_E_INVALID, "chunk %d and strands %d must be >= 1", chunk, strands);
    for (int a = 0; a < 3; a++)
        for (int64_t i = 0; i < n; i++)
            if (!std::isfinite(mean[a * stride + i]))
                return fail(GS_E_INVALID, "mean %d of Gaussian %lld not finite", a, (long long)i);
    gs::spatial_order(mean, n, stride, bits, chunk, strands, perm);
    return GS_OK;
}

gs_status gs_split_scene(const double* points, int64_t n, int32_t K, int32_t ground_axes, double* boxes,
                         int64_t* cell_of) {
    if (!points || !boxes) return fail(GS_E_INVALID, "null points or boxes");
    if (n < 1 || K < 1 || int64_t(K) > n) return fail(GS_E_INVALID, "need 1 <= K (%d) <= points (%lld)", K, (long long)n);
    if (ground_axes <= 0 || ground_axes > 7) return fail(GS_E_INVALID, "ground axis mask %d not in 1..7", ground_axes);
    for (int64_t i = 0; i < 3 * n; i++)
        if (!std::isfinite(points[i])) return fail(GS_E_INVALID, "point coordinate %lld not finite", (long long)i);
    return gs::split_scene(points, n, K, ground_axes, boxes, cell_of);
}

gs_status gs_split_group(const double* boxes, int32_t K, double scale, int32_t test_axes, const double* points,
                         int64_t n, int64_t* counts, int64_t* members, int64_t capacity, int64_t* total) {
    if (!boxes || !counts || !total || (n > 0 && !points)) return fail(GS_E_INVALID, "null boxes, points, counts or total");
    if (K < 1 || n < 0) return fail(GS_E_INVALID, "need K >= 1 and n >= 0");
    if (!(scale >= 1.0) || !std::isfinite(scale)) return fail(GS_E_INVALID, "scale %g not finite and >= 1", scale);
    if (test_axes <= 0 || test_axes > 7) return fail(GS_E_INVALID, "test axis mask %d not in 1..7", test_axes);
    gs::split_group(boxes, K, scale, test_axes, points, n, counts, members, capacity, total);
    if (members && capacity < *total)
        return fail(GS_E_CAPACITY, "members capacity %lld < %lld", (long long)capacity, (long long)*total);
    return GS_OK;
}

gs_status gs_dual_rescale(gs_params* u, gs_params* w, const gs_params* z, const int64_t* hptr, const int64_t* hidx,
                          const float* scale, gs_stream stream) {
    gs_status st;
    if ((st = check_params(u, "u_local")) != GS_OK) return st;
    if ((st = check_params(w, "w_local")) != GS_OK) return st;
    if ((st = check_params(z, "z_global")) != GS_OK) return st;
    if (w->n != u->n) return fail(GS_E_INVALID, "local planes disagree in n");
    if (w->sh_degree != u->sh_degree || z->sh_degree != u->sh_degree)
        return fail(GS_E_INVALID, "planes disagree in sh_degree");
    if (!scale) return fail(GS_E_INVALID, "null scale");
    for (int k = 0; k < 5; k++)
        if (!(scale[k] > 0.f) || !std::isfinite(scale[k]))
            return fail(GS_E_INVALID, "scale[%d] = %g not positive and finite", k, double(scale[k]));
    if (z->n > 0 && (!hptr || !hidx)) return fail(GS_E_INVALID, "null holder CSR");
    if (u->n >= (int64_t(1) << 30) || z->n >= (int64_t(1) << 30))
        return fail(GS_E_INVALID, "dual rescale supports fewer than 2^30 local and global columns");
    return check_hip(gs::launch_dual_rescale(*u, *w, *z, hptr, hidx, scale, (hipStream_t)stream), "gs_dual_rescale");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// per-kernel timing

namespace {

struct ProfState {
    std::mutex mu;
    std::atomic<bool> on{false};
    bool paused = false;
    bool all = false;
    std::set<std::string> names;
    struct Entry {
        std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
        double ms = 0;
        int64_t launches = 0;
    };
    std::map<std::string, Entry> entries;
    std::vector<hipEvent_t> pool;
};

ProfState& prof() {
    static ProfState* p = new ProfState();   // lives until the process ends
    return *p;
}

// waits for a recorded pair and adds its duration; returns the events to the pool
void resolve(ProfState& P, ProfState::Entry& e) {
    for (auto& ev : e.pending) {
        float t = 0.f;
        if (ev.second && hipEventSynchronize(ev.second) == hipSuccess &&
            hipEventElapsedTime(&t, ev.first, ev.second) == hipSuccess)
            e.ms += t;
        e.launches += 1;
        P.pool.push_back(ev.first);
        if (ev.second) P.pool.push_back(ev.second);
    }
    e.pending.clear();
}

}  // namespace

namespace gs {

bool profile_wanted(const char* name) {
    ProfState& P = prof();
    if (!P.on.load(std::memory_order_relaxed)) return false;
    std::lock_guard<std::mutex> lk(P.mu);
    return P.all || P.names.count(name) != 0;
}

hipEvent_t profile_event() {
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    if (!P.pool.empty()) {
        hipEvent_t e = P.pool.back();
        P.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void profile_record(const char* name, hipEvent_t begin, hipEvent_t end) {
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.entries[name].pending.emplace_back(begin, end);
}

}  // namespace gs

gs_status gs_profile_set(const char* names) {
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto& kv : P.entries) resolve(P, kv.second);
    P.entries.clear();
    P.names.clear();
    P.all = false;
    std::string s = names ? names : "";
    size_t a = 0;
    while (a <= s.size() && !s.empty()) {
        size_t b = s.find(',', a);
        if (b == std::string::npos) b = s.size();
        std::string n = s.substr(a, b - a);
        if (n == "*") P.all = true;
        else if (!n.empty()) P.names.insert(n);
        a = b + 1;
    }
    P.paused = false;
    P.on.store(P.all || !P.names.empty(), std::memory_order_relaxed);
    g_err[0] = 0;
    return GS_OK;
}

gs_status gs_profile_enable(int32_t on) {
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.paused = on == 0;
    P.on.store(!P.paused && (P.all || !P.names.empty()), std::memory_order_relaxed);
    g_err[0] = 0;
    return GS_OK;
}

gs_status gs_profile_get(const char* name, double* total_ms, int64_t* launches) {
    if (!name || !total_ms || !launches) return fail(GS_E_INVALID, "gs_profile_get: null argument");
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.entries.find(name);
    if (it == P.entries.end()) {
        *total_ms = 0;
        *launches = 0;
        return GS_OK;
    }
    resolve(P, it->second);
    *total_ms = it->second.ms;
    *launches = it->second.launches;
    return GS_OK;
}
