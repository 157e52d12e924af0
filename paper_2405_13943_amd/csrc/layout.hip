// Storage order of a Gaussian store (host code; a layout, not a step of the
// method).  Z-order (Morton order) of the means: each coordinate quantised to
// `bits` bits over the cloud's bounding box, the bits interleaved (x lowest,
// then y, then z, from the least significant level up), ties by index.
// Gaussians close in space become close in memory, so the set one view sees
// forms long runs: the projection's loads of culled Gaussians then skip
// whole cache lines, and a tile's records share lines.
//
// Optionally the Z-ordered sequence is cut into chunks of `chunk` Gaussians
// (one cache line of a plane at 16) that are dealt over `strands` strands:
// strand s takes chunks s, s + strands, ..., and the strands follow one
// another.  Lines stay coherent in space, while a run of consecutive chunks
// (one optimiser workgroup's Gaussians) comes from regions far apart, so
// every such run mixes Gaussians the view sees and Gaussians it does not.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "gs_internal.hpp"

namespace gs {

void spatial_order(const float* mean, int64_t n, int64_t stride, int32_t bits, int32_t chunk, int32_t strands,
                   int64_t* perm) {
    double lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = hi[a] = double(mean[a * stride]);
        for (int64_t i = 1; i < n; i++) {
            const double v = double(mean[a * stride + i]);
            lo[a] = std::min(lo[a], v);
            hi[a] = std::max(hi[a], v);
        }
    }
    const int64_t cells = int64_t(1) << bits;
    std::vector<std::pair<uint64_t, int64_t>> key(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; i++) {
        uint64_t q[3];
        for (int a = 0; a < 3; a++) {
            const double ext = std::max(hi[a] - lo[a], 1e-30);
            const double c = std::floor((double(mean[a * stride + i]) - lo[a]) / ext * double(cells));
            q[a] = uint64_t(std::min<double>(std::max(c, 0.0), double(cells - 1)));
        }
        uint64_t code = 0;
        for (int b = 0; b < bits; b++)
            for (int a = 0; a < 3; a++) code |= ((q[a] >> b) & 1u) << (3 * b + a);
        key[size_t(i)] = {code, i};
    }
    std::sort(key.begin(), key.end());
    const int64_t nch = n / chunk;
    if (strands <= 1 || nch == 0) {
        for (int64_t i = 0; i < n; i++) perm[i] = key[size_t(i)].second;
        return;
    }
    int64_t o = 0;
    for (int64_t s = 0; s < strands; s++)
        for (int64_t c = s; c < nch; c += strands)
            for (int64_t j = 0; j < chunk; j++) perm[o++] = key[size_t(c * chunk + j)].second;
    for (int64_t i = nch * chunk; i < n; i++) perm[o++] = key[size_t(i)].second;
}

}  // namespace gs
