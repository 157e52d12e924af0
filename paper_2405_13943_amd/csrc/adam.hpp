// Per-element Adam update with the scaled ADMM penalty (Eq. 8a, per-attribute
// rho and learning rate of the supplementary Sec. C), shared by the streaming
// optimiser kernel and the fused projection-backward + optimiser kernel so
// that both produce the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "gs.h"

namespace gs {

// attribute group of plane a: 0 p (mean), 1 q (rotation), 2 s (scale), 3 f (SH), 4 o (opacity)
__host__ __device__ constexpr int plane_group(int a) {
    return a < 3 ? 0 : (a < 7 ? 1 : (a < 10 ? 2 : (a == 10 ? 4 : 3)));
}

struct AdamConsts {
    float lr[5], rho[5];
    float b1, b2, eps, rbc1, rbc2;
};

// reciprocals of the bias corrections 1 - beta^t, evaluated in double on the
// host, then rounded
inline AdamConsts adam_consts(const gs_adam_cfg& cfg) {
    AdamConsts c;
    for (int k = 0; k < 5; k++) { c.lr[k] = cfg.lr[k]; c.rho[k] = cfg.rho[k]; }
    c.b1 = cfg.beta1; c.b2 = cfg.beta2; c.eps = cfg.eps;
    c.rbc1 = float(1.0 / (1.0 - std::pow(double(cfg.beta1), double(cfg.step))));
    c.rbc2 = float(1.0 / (1.0 - std::pow(double(cfg.beta2), double(cfg.step))));
    return c;
}

// g' = g + rho (x - w); m, v moments; x -= lr m^ / (sqrt(v^) + eps).
// The bias corrections are applied as products with their reciprocals and
// the step's quotient as a product with the hardware reciprocal of the
// hardware square root plus eps (each within an ulp or two): a few
// instructions where the correctly rounded divisions and square root take
// about forty, in a pass that streams every parameter
__device__ inline float adam_one(float& x, float g, float& m, float& v, float w, float rho, float lr,
                                 const AdamConsts& c) {
    const float gp = g + rho * (x - w);
    m = c.b1 * m + (1.0f - c.b1) * gp;
    v = c.b2 * v + (1.0f - c.b2) * gp * gp;
    const float mh = m * c.rbc1;
    const float vh = v * c.rbc2;
    x = x - lr * mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + c.eps);
    return x;
}

// Non-finite detection for the optimiser: fin += x * 0 + v * 0 stays 0
// while the updated parameter and second moment are finite, and turns NaN
// otherwise.  A NaN or Inf in any of x, g, m, v, w (or the mask) reaches the
// updated x or v through the update above, so checking the two outputs
// covers every input.
__device__ inline void adam_finite(float& fin, float x, float v) { fin += x * 0.0f + v * 0.0f; }

// Device status word handed to the optimiser kernels (may be null): the
// update is skipped while GS_STATUS_PAIR_OVERFLOW is set (a gradient from
// truncated tile lists must not move the parameters), and
// GS_STATUS_NONFINITE is OR-ed in when an update meets a NaN or Inf.
__device__ inline bool adam_skipped(const uint32_t* status) {
    return status != nullptr && (*status & GS_STATUS_PAIR_OVERFLOW) != 0u;
}
__device__ inline void adam_flag(uint32_t* status, float fin) {
    if (status != nullptr && !(fin == 0.0f)) atomicOr(status, GS_STATUS_NONFINITE);
}

}  // namespace gs
