// Host-side launchers of the libgs kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "gs.h"

namespace gs {

// Optional per-kernel timing (gs_profile_set): when a kernel's name is
// selected, HIP events are recorded on its stream around each launch and
// resolved by gs_profile_get.  One relaxed flag test per launch otherwise.
bool profile_wanted(const char* name);
hipEvent_t profile_event();
void profile_record(const char* name, hipEvent_t begin, hipEvent_t end);

struct KernelTimer {
    const char* name;
    hipStream_t stream;
    hipEvent_t begin = nullptr;
    KernelTimer(const char* n, hipStream_t s) : name(n), stream(s) {
        if (profile_wanted(n) && (begin = profile_event()) != nullptr) (void)hipEventRecord(begin, s);
    }
    ~KernelTimer() {
        if (!begin) return;
        hipEvent_t end = profile_event();
        if (end) (void)hipEventRecord(end, stream);
        profile_record(name, begin, end);
    }
};

#define GS_LAUNCH(NAME, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)             \
    do {                                                                     \
        ::gs::KernelTimer gs_kernel_timer_(NAME, STREAM);                    \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__); \
    } while (0)

// project.hip
template <typename T>
hipError_t launch_project(const gs_params& p, const gs_frame& f, const gs_raster_cfg& cfg, T* rec,
                          uint32_t* meta, uint32_t* status, hipStream_t s);
template <typename T>
hipError_t launch_project_bwd(const gs_params& p, const gs_frame& f, const gs_raster_cfg& cfg, const T* rec,
                              const uint32_t* meta, const gs_bins& bins, const T* pg, gs_params& grad, hipStream_t s);

// fused projection backward + Adam/ADMM (FP32, jobs over disjoint ranges)
hipError_t launch_project_bwd_adam(gs_params& x, const gs_frame& f, const gs_raster_cfg& cfg, const float* rec,
                                   const uint32_t* meta,
                                   const gs_bins& bins, const float* pg, gs_params& m, gs_params& v,
                                   const gs_params* w, const float* mask, const gs_adam_cfg& acfg, hipStream_t s);

// binning.hip
size_t bin_workspace_size(int64_t n_records, uint64_t capacity, int32_t n_tiles);
hipError_t launch_bin_sort(const gs_frame& f, const gs_raster_cfg& cfg, const uint32_t* meta, const gs_bins& bins,
                           void* ws, size_t ws_bytes, hipStream_t s);

// render.hip
template <typename T>
hipError_t launch_render_fwd(const gs_frame& f, const gs_raster_cfg& cfg, const T* rec, const gs_bins& bins,
                             T* rgb, T* Tfin, uint32_t* ncontrib, unsigned long long* kept, hipStream_t s);
template <typename T>
hipError_t launch_render_bwd(const gs_frame& f, const gs_raster_cfg& cfg, const T* rec, const uint32_t* meta,
                             const gs_bins& bins, const T* rgb, const uint32_t* ncontrib, gs_loss_mode mode,
                             const T* grad_in, T* loss_out, T* pg, hipStream_t s);

// ssim.hip
size_t ssim_workspace_size(int64_t n_pixels);
hipError_t launch_ssim_loss_grad(const gs_frame& f, const gs_raster_cfg& cfg, const float* rgb, const float* tgt,
                                 float lambda, float* grad, float* loss, void* ws, hipStream_t s);

// split.hip (host)
gs_status split_scene(const double* points, int64_t n, int32_t K, int32_t axes, double* boxes, int64_t* cell_of);
// layout.hip
void spatial_order(const float* mean, int64_t n, int64_t stride, int32_t bits, int32_t chunk, int32_t strands,
                   int64_t* perm);
void split_group(const double* boxes, int32_t K, double s, int32_t axes, const double* points, int64_t n,
                 int64_t* counts, int64_t* members, int64_t capacity, int64_t* total);

// tune.hip (host)
gs_status tune_set_cache(const char* path, std::string& err);
gs_status tune_lookup(const char* key, gs_tune_choice* best, double* best_ms, bool* found, std::string& err);
gs_status tune_run(const char* key, const gs_tune_choice* cand, int32_t n, int32_t reps, gs_tune_step_fn step,
                   void* user, hipStream_t stream, gs_tune_choice* best, double* best_ms, std::string& err);

// optim.hip
hipError_t launch_adam_admm(gs_params& x, const gs_params& g, gs_params& m, gs_params& v, const gs_params* w,
                            const float* mask, const gs_adam_cfg& cfg, uint32_t* status, hipStream_t s);
hipError_t launch_consensus(const gs_params& x, gs_params& u, gs_params& w, gs_params& z, const int64_t* hptr,
                            const int64_t* hidx, float relax, float* resid, hipStream_t s);
hipError_t launch_dual_rescale(gs_params& u, gs_params& w, const gs_params& z, const int64_t* hptr,
                               const int64_t* hidx, const float* scale, hipStream_t s);

}  // namespace gs
