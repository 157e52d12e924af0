// Tile binning: turns per-record tile rectangles into per-tile lists of
// record ids ordered by (depth, record).  The paper does not describe tiling
// (its rasterizer is cited, not specified); this is an exact acceleration of
// the per-pixel compositing order (depth, index).
//
//   1. compact the visible records (scan of n_tiles > 0), in record order;
//   2. scan their tile counts: each record's pairs are contiguous from its
//      first pair (pair_off), the layout the backward's per-pair partials use;
//   3. emit one (tile id, record) pair per covered tile and sort the pairs by
//      tile id (LSD radix, ceil(log2 tiles) bits);
//   4. sort each tile's list by the unique key (depth bits, record) on chip
//      (k_tile_sort: positive floats order like their bits).
// Sorting every tile's short list in LDS replaces four global radix passes
// over all visible records by their depth.
//
// Every count that depends on the data (visible records V, pairs P) stays on
// the device: kernels read it from the counters and size their loops from
// it, so the whole chain runs without a host round trip.
#include "gs_device.hpp"
#include "gs_internal.hpp"

#include <algorithm>

namespace gs {

constexpr int kScanBlock = 256;
constexpr int kRsBlock = 256;
constexpr int kRsItems = 4;
constexpr int kRsTile = kRsBlock * kRsItems;
constexpr int kMaxGrid = 1024;

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct BinWs {
    uint32_t* dval[1];    // visible record ids, [n_records]
    uint32_t* tkey[2];    // tile keys, [capacity] each
    uint32_t* tval;       // alternate record-id buffer, [capacity]
    uint32_t* part;       // scan partials, [kMaxGrid + 1]
    uint32_t* hist;       // radix histograms, [256 * kMaxGrid]
    uint32_t* coltot;     // per-digit totals of one radix pass, [256]
    uint32_t* poff;       // first pair of each visible record in compacted order, [n_records]
    uint64_t* key[2];     // sort keys of long tile lists, [capacity] each
    size_t bytes;
};

static BinWs carve(void* base, int64_t n_records, uint64_t capacity) {
    BinWs w;
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) { char* q = p ? p + off : nullptr; off += align256(bytes); return reinterpret_cast<uint32_t*>(q); };
    const size_t nr = size_t(n_records > 0 ? n_records : 1) * 4, nc = size_t(capacity > 0 ? capacity : 1) * 4;
    w.dval[0] = take(nr);
    w.tkey[0] = take(nc); w.tkey[1] = take(nc);
    w.tval = take(nc);
    w.part = take(size_t(kMaxGrid + 1) * 4);
    w.hist = take(size_t(256) * kMaxGrid * 4);
    w.coltot = take(256 * 4);
    w.poff = take(nr);
    w.key[0] = reinterpret_cast<uint64_t*>(take(nc * 2));
    w.key[1] = reinterpret_cast<uint64_t*>(take(nc * 2));
    w.bytes = off;
    return w;
}

size_t bin_workspace_size(int64_t n_records, uint64_t capacity, int32_t) {
    return carve(nullptr, n_records, capacity).bytes;
}

// ---------------------------------------------------------------------------
// small helpers

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// exclusive scan of one value per thread over a 256-thread block
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t& total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) s_wave[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / kWave; w++) {
        const uint32_t s = s_wave[w];
        if (w < wave) before += s;
        total += s;
    }
    __syncthreads();
    return before + inc - v;
}

// chunk of items [lo, hi) that block b of G handles when n items are split
__device__ inline void block_range(uint32_t n, int G, int b, uint32_t granule, uint32_t& lo, uint32_t& hi) {
    uint32_t chunk = (n + G - 1) / G;
    chunk = (chunk + granule - 1) / granule * granule;
    lo = min(n, uint32_t(b) * chunk);
    hi = min(n, lo + chunk);
}

// ---------------------------------------------------------------------------
// reduce-then-scan over a device-sized sequence; two flavours of input/output

struct VisibleFlag {      // item i: record i is visible; output: the compacted record ids
    const uint4* meta;
    uint32_t* val_out;
    __device__ uint32_t value(uint32_t i) const { return meta_tiles(meta[i].y) > 0 ? 1u : 0u; }
    __device__ void emit(uint32_t i, uint32_t pre) const {
        if (meta_tiles(meta[i].y) > 0) val_out[pre] = i;
    }
};

struct PairCount {        // item s: visible record s; output: its first pair
    const uint4* meta;
    const uint32_t* sorted_rec;
    uint32_t* pair_off;       // by record
    uint32_t* poff;           // by depth rank
    __device__ uint32_t value(uint32_t s) const { return meta_tiles(meta[sorted_rec[s]].y); }
    __device__ void emit(uint32_t s, uint32_t pre) const {
        pair_off[sorted_rec[s]] = pre;
        poff[s] = pre;
    }
};

template <typename F>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(F f, const uint32_t* __restrict__ n_dev, uint32_t n_host,
                                                            uint32_t* __restrict__ part, int G) {
    __shared__ uint32_t s_wave[kScanBlock / kWave];
    const uint32_t n = n_dev ? min(*n_dev, n_host) : n_host;
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, kScanBlock, lo, hi);
    uint32_t acc = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kScanBlock) acc += f.value(i);
    uint32_t tot;
    block_excl_scan(acc, s_wave, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single block: exclusive scan of the G partials in place; total to counters
__global__ __launch_bounds__(kScanBlock) void k_scan_spine(uint32_t* __restrict__ part, int G,
                                                           uint32_t* __restrict__ counters, int total_idx,
                                                           uint64_t capacity) {
    __shared__ uint32_t s_wave[kScanBlock / kWave];
    uint32_t carry = 0;
    for (int base = 0; base < G; base += kScanBlock) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < G ? part[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, s_wave, tot);
        if (i < G) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        counters[total_idx] = carry;
        if (capacity && uint64_t(carry) > capacity) counters[GS_CTR_STATUS] |= GS_STATUS_PAIR_OVERFLOW;
    }
}

template <typename F>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(F f, const uint32_t* __restrict__ n_dev, uint32_t n_host,
                                                           const uint32_t* __restrict__ part, int G) {
    __shared__ uint32_t s_wave[kScanBlock / kWave];
    const uint32_t n = n_dev ? min(*n_dev, n_host) : n_host;
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, kScanBlock, lo, hi);
    uint32_t carry = part[blockIdx.x];
    for (uint32_t base = lo; base < hi; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < hi ? f.value(i) : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, s_wave, tot);
        if (i < hi) f.emit(i, carry + ex);
        carry += tot;
    }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (uint32 key, uint32 value), 8-bit digits,
// reduce-then-scan with a fixed grid of G blocks over device-sized n

__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
                                                      uint32_t n_host, int shift, uint32_t* __restrict__ hist, int G) {
    __shared__ uint32_t h[kRsBlock / kWave][256];
    const int wave = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < 256 * (kRsBlock / kWave); i += kRsBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = min(*n_dev, n_host);
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, kRsTile, lo, hi);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kRsBlock) atomicAdd(&h[wave][(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kRsBlock / kWave; w++) s += h[w][d];
    hist[d * G + blockIdx.x] = s;
}

// one block per digit: exclusive scan of that digit's counts over the G
// blocks (in place) and the digit's total; the digits' base offsets are
// then an exclusive scan of 256 totals, done by every scatter block
__global__ __launch_bounds__(kRsBlock) void k_rs_colscan(uint32_t* __restrict__ hist, int G,
                                                         uint32_t* __restrict__ coltot) {
    __shared__ uint32_t s_wave[kRsBlock / kWave];
    uint32_t* col = hist + size_t(blockIdx.x) * G;
    constexpr int PER = kMaxGrid / kRsBlock;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int i = threadIdx.x * PER + k;
        v[k] = i < G ? col[i] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(sum, s_wave, tot);
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int i = threadIdx.x * PER + k;
        if (i < G) col[i] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) coltot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                         uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                         const uint32_t* __restrict__ n_dev, uint32_t n_host, int shift,
                                                         const uint32_t* __restrict__ hist, int G,
                                                         const uint32_t* __restrict__ coltot) {
    constexpr int NW = kRsBlock / kWave;
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t wpre[NW][256];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t n = min(*n_dev, n_host);
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, kRsTile, lo, hi);
    {
        __shared__ uint32_t s_wave[NW];
        uint32_t tot;
        const uint32_t base = block_excl_scan(coltot[tid], s_wave, tot);
        run[tid] = base + hist[tid * G + blockIdx.x];
    }
    for (uint32_t base = lo; base < hi; base += kRsTile) {
        for (int d = lane; d < 256; d += kWave) wcnt[wave][d] = 0;
        __builtin_amdgcn_wave_barrier();
        uint32_t key[kRsItems], val[kRsItems], rank[kRsItems];
#pragma unroll
        for (int k = 0; k < kRsItems; k++) {
            const uint32_t i = base + wave * (kWave * kRsItems) + k * kWave + lane;
            key[k] = 0; val[k] = 0; rank[k] = 0;
            if (i < hi) {
                key[k] = kin[i];
                val[k] = vin[i];
                const uint32_t dg = (key[k] >> shift) & 255u;
                uint64_t peers = __ballot(1);
#pragma unroll
                for (int bit = 0; bit < 8; bit++) {
                    const uint64_t m = __ballot((dg >> bit) & 1u);
                    peers &= ((dg >> bit) & 1u) ? m : ~m;
                }
                const uint32_t before = wcnt[wave][dg];
                rank[k] = before + uint32_t(__popcll(peers & lanemask_lt()));
                const int leader = 63 - __clzll(peers);
                if (lane == leader) wcnt[wave][dg] = before + uint32_t(__popcll(peers));
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        uint32_t tot = 0;
        {
            const int d = tid;
#pragma unroll
            for (int w = 0; w < NW; w++) {
                wpre[w][d] = tot;
                tot += wcnt[w][d];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRsItems; k++) {
            const uint32_t i = base + wave * (kWave * kRsItems) + k * kWave + lane;
            if (i < hi) {
                const uint32_t dg = (key[k] >> shift) & 255u;
                const uint32_t pos = run[dg] + wpre[wave][dg] + rank[k];
                kout[pos] = key[k];
                vout[pos] = val[k];
            }
        }
        __syncthreads();
        run[tid] += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// pair emission and tile ranges

// Pair-parallel emission: block-sized chunks of the P pairs; each chunk finds
// the depth-ordered records it spans by binary search over their first-pair
// offsets (staged in LDS), so a Gaussian covering thousands of tiles is
// spread over many threads instead of serialising one.
constexpr int kEmitChunk = 2048;

__global__ __launch_bounds__(256) void k_emit(const uint4* __restrict__ meta, const uint32_t* __restrict__ sorted_rec,
                                              const uint32_t* __restrict__ poff, const uint32_t* __restrict__ counters,
                                              gs_frame frame, uint64_t capacity, uint32_t* __restrict__ tkey,
                                              uint32_t* __restrict__ tval) {
    __shared__ uint32_t s_off[kEmitChunk];
    __shared__ uint32_t s_rec[kEmitChunk];
    __shared__ uint32_t s_lo, s_hi;
    const uint32_t V = counters[GS_CTR_VISIBLE];
    const uint32_t P = uint32_t(min(uint64_t(counters[GS_CTR_PAIRS]), capacity));
    for (uint32_t e0 = blockIdx.x * kEmitChunk; e0 < P; e0 += gridDim.x * kEmitChunk) {
        const uint32_t e1 = min(P, e0 + kEmitChunk);
        if (threadIdx.x < 2) {
            // last visible rank whose first pair is <= target (ranks with zero
            // pairs do not exist: every visible record covers a tile)
            const uint32_t target = threadIdx.x == 0 ? e0 : e1 - 1;
            uint32_t lo = 0, hi = V - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (poff[mid] <= target) lo = mid; else hi = mid - 1;
            }
            if (threadIdx.x == 0) s_lo = lo; else s_hi = lo;
        }
        __syncthreads();
        const uint32_t lo = s_lo, n = s_hi - s_lo + 1;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            s_off[i] = poff[lo + i];
            s_rec[i] = sorted_rec[lo + i];
        }
        __syncthreads();
        for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            uint32_t a = 0, b = n - 1;
            while (a < b) {
                const uint32_t mid = (a + b + 1) >> 1;
                if (s_off[mid] <= e) a = mid; else b = mid - 1;
            }
            const uint32_t r = s_rec[a], k = e - s_off[a];
            const uint4 m = meta[r];
            const int j = job_of_record(frame.jobs, frame.n_jobs, r);
            const uint32_t x0 = m.z & 0xffffu, y0 = m.z >> 16, x1 = m.w & 0xffffu;
            const uint32_t w = x1 - x0 + 1;
            tkey[e] = uint32_t(frame.jobs[j].tile0) + (y0 + k / w) * uint32_t(frame.jobs[j].tiles_x) + x0 + k % w;
            tval[e] = r;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// per-tile depth order: each tile's list (record ids, any order) sorted by the
// unique key (depth bits, record id).  k_tile_sort (persistent grid) takes
// lists of up to kSortChunk entries: up to one workgroup's width a rank sort
// in LDS (each thread counts the keys smaller than its own), longer ones a
// bitonic sort in LDS.  k_tile_sort_long takes the longer lists (dense
// views), one large workgroup each.

constexpr int kSortBlock = 256;
constexpr int kSortChunk = 2048;

__device__ __forceinline__ uint64_t depth_key(const uint4* __restrict__ meta, uint32_t r) {
    return (uint64_t(meta[r].x) << 32) | r;
}

// number of keys in run[0, n) smaller than k (the run is sorted)
__device__ __forceinline__ uint32_t count_less(const uint64_t* run, uint32_t n, uint64_t k) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (run[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ascending bitonic sort of sk[0, p), p a power of two, by a workgroup of B
template <int B>
__device__ __forceinline__ void bitonic_lds(uint64_t* sk, uint32_t p) {
    for (uint32_t k = 2; k <= p; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < p; i += B) {
                const uint32_t ij = i ^ j;
                if (ij > i) {
                    const uint64_t a = sk[i], b = sk[ij];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) { sk[i] = b; sk[ij] = a; }
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kSortBlock) void k_tile_sort(const uint4* __restrict__ meta,
                                                          const uint2* __restrict__ ranges, int n_tiles,
                                                          uint32_t* __restrict__ vals) {
    __shared__ uint64_t sk[kSortChunk];
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint2 rg = ranges[tile];
        const uint32_t n = rg.y - rg.x;
        if (n < 2) continue;                                   // uniform per workgroup
        uint32_t* v = vals + rg.x;
        if (n <= kSortBlock) {
            const uint32_t i = threadIdx.x;
            const uint64_t k = i < n ? depth_key(meta, v[i]) : 0;
            if (i < n) sk[i] = k;
            __syncthreads();
            if (i < n) {
                uint32_t rank = 0;
                for (uint32_t j = 0; j < n; j++) rank += sk[j] < k ? 1u : 0u;
                v[rank] = uint32_t(k);
            }
            __syncthreads();
            continue;
        }
        if (n > uint32_t(kSortChunk)) continue;                 // k_tile_sort_long takes it
        // bitonic sort in LDS (padded with the largest key)
        uint32_t p = 1;
        while (p < n) p <<= 1;
        for (uint32_t i = threadIdx.x; i < p; i += kSortBlock) sk[i] = i < n ? depth_key(meta, v[i]) : ~0ull;
        __syncthreads();
        bitonic_lds<kSortBlock>(sk, p);
        for (uint32_t i = threadIdx.x; i < n; i += kSortBlock) v[i] = uint32_t(sk[i]);
        __syncthreads();
    }
}

// Lists longer than kSortChunk: one workgroup of kLongBlock threads per list,
// chunks of kLongChunk keys bitonic-sorted in LDS, then (lists longer than a
// chunk) pairwise merges of sorted key runs through two scratch ranges (each
// key's place is its index in its run plus the number of smaller keys in the
// other run, by binary search).
constexpr int kLongBlock = 1024;
constexpr int kLongChunk = 8192;

__global__ __launch_bounds__(kLongBlock) void k_tile_sort_long(const uint4* __restrict__ meta,
                                                               const uint2* __restrict__ ranges, int n_tiles,
                                                               uint32_t* __restrict__ vals, uint64_t* __restrict__ ka,
                                                               uint64_t* __restrict__ kb) {
    __shared__ uint64_t sk[kLongChunk];
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint2 rg = ranges[tile];
        const uint32_t n = rg.y - rg.x;
        if (n <= uint32_t(kSortChunk)) continue;                // uniform per workgroup
        uint32_t* v = vals + rg.x;
        uint64_t* src = ka + rg.x;
        uint64_t* dst = kb + rg.x;
        for (uint32_t c0 = 0; c0 < n; c0 += kLongChunk) {
            const uint32_t m = min(uint32_t(kLongChunk), n - c0);
            uint32_t p = 1;
            while (p < m) p <<= 1;
            for (uint32_t i = threadIdx.x; i < p; i += kLongBlock) sk[i] = i < m ? depth_key(meta, v[c0 + i]) : ~0ull;
            __syncthreads();
            bitonic_lds<kLongBlock>(sk, p);
            if (n <= uint32_t(kLongChunk)) {
                for (uint32_t i = threadIdx.x; i < m; i += kLongBlock) v[i] = uint32_t(sk[i]);
            } else {
                for (uint32_t i = threadIdx.x; i < m; i += kLongBlock) src[c0 + i] = sk[i];
            }
            __syncthreads();
        }
        if (n <= uint32_t(kLongChunk)) continue;
        for (uint32_t run = kLongChunk; run < n; run <<= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += kLongBlock) {
                const uint32_t a0 = (i / (2 * run)) * (2 * run), b0 = a0 + run, b1 = min(a0 + 2 * run, n);
                const uint64_t k = src[i];
                if (b0 >= n) { dst[i] = k; continue; }
                if (i < b0) dst[i + count_less(src + b0, b1 - b0, k)] = k;
                else dst[a0 + (i - b0) + count_less(src + a0, run, k)] = k;
            }
            __syncthreads();
            uint64_t* t = src;
            src = dst;
            dst = t;
        }
        for (uint32_t i = threadIdx.x; i < n; i += kLongBlock) v[i] = uint32_t(src[i]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tkey, const uint32_t* __restrict__ counters,
                                                uint64_t capacity, uint2* __restrict__ ranges) {
    const uint32_t P = uint32_t(min(uint64_t(counters[GS_CTR_PAIRS]), capacity));
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < P; e += gridDim.x * blockDim.x) {
        const uint32_t t = tkey[e];
        if (e == 0 || tkey[e - 1] != t) ranges[t].x = e;
        if (e + 1 == P || tkey[e + 1] != t) ranges[t].y = e + 1;
    }
}

// Compositing plan for adaptive wavefronts: every tile's wavefront count
// (adaptive_waves of its list length) and the tiles grouped by it, 4-wave
// tiles first (one workgroup each, and the longest lists start first), then
// 2-wave, then 1-wave tiles.  One workgroup; the order inside a group is
// whatever the LDS atomics give, which changes no result (each tile is
// composited on its own).
__global__ __launch_bounds__(1024) void k_tile_plan(const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ counters, int n_tiles, int quads,
                                                    uint32_t* __restrict__ order) {
    __shared__ uint32_t cnt[3], cur[3];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t pairs = counters[GS_CTR_PAIRS];
    const int lane = lane_id();
    auto group = [&](int t) {
        if (t >= n_tiles) return -1;
        const uint2 rg = ranges[t];
        const int w = adaptive_waves(rg.y - rg.x, pairs, n_tiles, quads);
        return w == 4 ? 0 : (w == 2 ? 1 : 2);
    };
    // counts: one LDS atomic per group and wavefront
    const int n_round = (n_tiles + int(blockDim.x) - 1) / int(blockDim.x) * int(blockDim.x);
    for (int t = threadIdx.x; t < n_round; t += blockDim.x) {
        const int gr = group(t);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint64_t b = __ballot(gr == k);
            if (lane == 0 && b) atomicAdd(&cnt[k], uint32_t(__builtin_popcountll(b)));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cur[0] = 0u;
        cur[1] = cnt[0];
        cur[2] = cnt[0] + cnt[1];
    }
    if (threadIdx.x < 3) order[threadIdx.x] = cnt[threadIdx.x];
    __syncthreads();
    // scatter: a wavefront reserves a run per group, lanes rank inside it
    for (int t = threadIdx.x; t < n_round; t += blockDim.x) {
        const int gr = group(t);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint64_t b = __ballot(gr == k);
            uint32_t base = 0u;
            if (lane == 0 && b) base = atomicAdd(&cur[k], uint32_t(__builtin_popcountll(b)));
            base = __shfl(base, 0, kWave);
            if (gr == k) order[4 + base + __builtin_popcountll(b & lanemask_lt())] = uint32_t(t);
        }
    }
}

// ---------------------------------------------------------------------------

static int grid_for(uint64_t n_max, int per_block) {
    uint64_t g = (n_max + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    return int(g);
}

static hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
                             uint32_t n_max, int bits, uint32_t** k_final, hipStream_t s, BinWs& w) {
    const int G = grid_for(n_max, kRsTile * 4);
    uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
    for (int shift = 0; shift < bits; shift += 8) {
        GS_LAUNCH("k_rs_hist", k_rs_hist, dim3(G), dim3(kRsBlock), 0, s, ki, n_dev, n_max, shift, w.hist, G);
        GS_LAUNCH("k_rs_colscan", k_rs_colscan, dim3(256), dim3(kRsBlock), 0, s, w.hist, G, w.coltot);
        GS_LAUNCH("k_rs_scatter", k_rs_scatter, dim3(G), dim3(kRsBlock), 0, s, ki, vi, ko, vo, n_dev, n_max, shift, w.hist, G,
                           w.coltot);
        uint32_t* t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    *k_final = ki;
    return hipGetLastError();
}

hipError_t launch_bin_sort(const gs_frame& f, const gs_raster_cfg& cfg, const uint32_t* meta_u32, const gs_bins& bins,
                           void* ws, size_t ws_bytes, hipStream_t s) {
    (void)cfg;
    (void)ws_bytes;
    BinWs w = carve(ws, f.n_records, bins.capacity);
    const uint4* meta = reinterpret_cast<const uint4*>(meta_u32);
    const uint32_t nrec = uint32_t(f.n_records);
    // counts restart every call; the status bits are sticky until the caller clears them
    GS_LAUNCH("k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, bins.counters, 0u, int64_t(GS_CTR_STATUS));
    const int64_t nr2 = int64_t(f.n_tiles) * 2;
    GS_LAUNCH("k_fill_u32", k_fill_u32, dim3(unsigned(std::min<int64_t>((nr2 + 255) / 256, 2048))), dim3(256), 0, s,
                       bins.ranges, 0u, nr2);
    auto plan = [&]() {
        if (bins.tile_order && (fwd_waves(cfg) == 0 || bwd_waves(cfg) == 0))
            GS_LAUNCH("k_tile_plan", k_tile_plan, dim3(1), dim3(1024), 0, s,
                      reinterpret_cast<const uint2*>(bins.ranges), bins.counters, f.n_tiles,
                      (cfg.tile_w / 8) * (cfg.tile_h / 8), bins.tile_order);
    };
    if (nrec == 0) {
        plan();
        return hipGetLastError();
    }

    // 1. compact the visible records (record order)
    const int Gs = grid_for(nrec, kScanBlock * 8);
    VisibleFlag vf{meta, w.dval[0]};
    GS_LAUNCH("k_scan_reduce", k_scan_reduce<VisibleFlag>, dim3(Gs), dim3(kScanBlock), 0, s, vf, nullptr, nrec, w.part, Gs);
    GS_LAUNCH("k_scan_spine", k_scan_spine, dim3(1), dim3(kScanBlock), 0, s, w.part, Gs, bins.counters, GS_CTR_VISIBLE,
                       uint64_t(0));
    GS_LAUNCH("k_scan_apply", k_scan_apply<VisibleFlag>, dim3(Gs), dim3(kScanBlock), 0, s, vf, nullptr, nrec, w.part, Gs);
    const uint32_t* n_vis = bins.counters + GS_CTR_VISIBLE;
    const uint32_t* sorted_rec = w.dval[0];
    hipError_t e;

    // 2. first pair of each visible record; total pairs
    PairCount pc{meta, sorted_rec, bins.pair_off, w.poff};
    GS_LAUNCH("k_scan_reduce", k_scan_reduce<PairCount>, dim3(Gs), dim3(kScanBlock), 0, s, pc, n_vis, nrec, w.part, Gs);
    GS_LAUNCH("k_scan_spine", k_scan_spine, dim3(1), dim3(kScanBlock), 0, s, w.part, Gs, bins.counters, GS_CTR_PAIRS,
                       bins.capacity);
    GS_LAUNCH("k_scan_apply", k_scan_apply<PairCount>, dim3(Gs), dim3(kScanBlock), 0, s, pc, n_vis, nrec, w.part, Gs);

    // 3. emit (tile, record) pairs, then sort them by tile id
    int bits = 0;
    while ((1ll << bits) < int64_t(f.n_tiles)) bits++;
    const int passes = (bits + 7) / 8;
    uint32_t* emit_val = (passes & 1) ? w.tval : bins.vals;
    uint32_t* other_val = (passes & 1) ? bins.vals : w.tval;
    GS_LAUNCH("k_emit", k_emit, dim3(unsigned(grid_for(bins.capacity, kEmitChunk))), dim3(256), 0, s, meta, sorted_rec,
                       w.poff, bins.counters, f, bins.capacity, w.tkey[0], emit_val);
    const uint32_t pmax = uint32_t(std::min<uint64_t>(bins.capacity, 0xffffffffull));
    uint32_t* tk_final = w.tkey[0];
    if (passes > 0) {
        e = radix_sort(w.tkey[0], emit_val, w.tkey[1], other_val, bins.counters + GS_CTR_PAIRS, pmax, passes * 8,
                       &tk_final, s, w);
        if (e != hipSuccess) return e;
    }

    // 4. per-tile [start, end)
    GS_LAUNCH("k_ranges", k_ranges, dim3(2048), dim3(256), 0, s, tk_final, bins.counters, bins.capacity,
                       reinterpret_cast<uint2*>(bins.ranges));
    // 5. each tile's list in (depth bits, record) order
    if (f.n_tiles > 0) {
        GS_LAUNCH("k_tile_sort", k_tile_sort, dim3(unsigned(std::min(f.n_tiles, 4096))), dim3(kSortBlock), 0, s, meta,
                  reinterpret_cast<const uint2*>(bins.ranges), f.n_tiles, bins.vals);
        GS_LAUNCH("k_tile_sort_long", k_tile_sort_long, dim3(unsigned(std::min(f.n_tiles, 256))), dim3(kLongBlock), 0,
                  s, meta, reinterpret_cast<const uint2*>(bins.ranges), f.n_tiles, bins.vals, w.key[0], w.key[1]);
    }
    // 6. compositing plan, when a pass splits tiles adaptively
    plan();
    return hipGetLastError();
}

}  // namespace gs
