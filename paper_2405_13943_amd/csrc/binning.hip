// Tile binning: turns per-record tile rectangles into per-tile lists of
// record ids ordered by (depth, record).  The paper does not describe tiling
// (its rasterizer is cited, not specified); this is an exact acceleration of
// the per-pixel compositing order (depth, index).
//
//   1. one scan over the records: the visible ones (at least one covered
//      tile) compacted in record order, and each one's first pair
//      (pair_off), the layout the backward's per-pair partials use;
//   2. emit one (tile id, record) pair per covered tile and sort the pairs by
//      tile id (LSD radix, ceil(log2 tiles) bits in one or more passes of at
//      most 8, each staged through LDS so that writes leave in runs);
//   3. per-tile [start, end);
//   4. sort each tile's list by the unique key (depth bits, record) on chip
//      (positive floats order like their bits).
//
// Every count that depends on the data (visible records V, pairs P) stays on
// the device: kernels read it from the counters and size their loops from
// it, so the whole chain runs without a host round trip.
#include "gs_device.hpp"
#include "gs_internal.hpp"

#include <algorithm>

namespace gs {

constexpr int kScanBlock = 256;
constexpr int kEmitChunk = 1024;                 // pairs per emission chunk
constexpr int kRsBlock = 256;
constexpr int kRsItemsLarge = 16;                // keys per thread and iteration of a radix pass: large
constexpr int kRsItemsSmall = 4;                 // and small sorts (more workgroups)
constexpr uint32_t kRsSmallMax = 1u << 22;       // pair capacity up to which the small form is used
constexpr int kMaxGrid = 1024;

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct BinWs {
    uint32_t* vis;        // visible record ids in record order, [n_records]
    uint32_t* poff;       // first pair of each visible record in that order, [n_records]
    uint32_t* cfirst;     // visible rank holding pair c * kEmitChunk, [capacity / kEmitChunk + 1]
    uint32_t* tkey[2];    // tile keys, [capacity] each
    uint32_t* tval;       // alternate record-id buffer, [capacity]
    uint64_t* key[2];     // sort keys of tile lists longer than one LDS chunk, [capacity] each
    uint32_t* hist;       // radix histograms, [256 * kMaxGrid]
    uint32_t* coltot;     // per-digit totals of one radix pass, [256]
    uint32_t* longq;      // lists longer than one LDS chunk: count, then tile ids, [1 + n_tiles]
    void* part;           // scan partials, [kMaxGrid + 1] x 8 bytes
    size_t bytes;
};

// key[0] overlays the two tile-key buffers and key[1] the alternate values:
// the long-list sort runs after the tile sort and the ranges are done
static BinWs carve(void* base, int64_t n_records, uint64_t capacity, int32_t n_tiles) {
    BinWs w;
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) { char* q = p ? p + off : nullptr; off += align256(bytes); return q; };
    const size_t nr = size_t(n_records > 0 ? n_records : 1) * 4, nc = size_t(capacity > 0 ? capacity : 1);
    w.vis = reinterpret_cast<uint32_t*>(take(nr));
    w.poff = reinterpret_cast<uint32_t*>(take(nr));
    w.cfirst = reinterpret_cast<uint32_t*>(take((nc / kEmitChunk + 1) * 4));
    char* a = take(nc * 8);
    char* b = take(nc * 8);
    w.key[0] = reinterpret_cast<uint64_t*>(a);
    w.key[1] = reinterpret_cast<uint64_t*>(b);
    w.tkey[0] = reinterpret_cast<uint32_t*>(a);
    w.tkey[1] = a ? reinterpret_cast<uint32_t*>(a + nc * 4) : nullptr;
    w.tval = reinterpret_cast<uint32_t*>(b);
    w.hist = reinterpret_cast<uint32_t*>(take(size_t(256) * kMaxGrid * 4));
    w.coltot = reinterpret_cast<uint32_t*>(take(256 * 4));
    w.longq = reinterpret_cast<uint32_t*>(take((size_t(n_tiles > 0 ? n_tiles : 0) + 1) * 4));
    w.part = take(size_t(kMaxGrid + 1) * 8);
    w.bytes = off;
    return w;
}

size_t bin_workspace_size(int64_t n_records, uint64_t capacity, int32_t n_tiles) {
    return carve(nullptr, n_records, capacity, n_tiles).bytes;
}

// ---------------------------------------------------------------------------
// small helpers

// counters of a frame without records: no visible record, no pair; an
// uncleared overflow still counts the call (its step's update is skipped)
__global__ void k_counters_empty(uint32_t* __restrict__ counters) {
    if (threadIdx.x == 0) {
        counters[GS_CTR_VISIBLE] = 0u;
        counters[GS_CTR_PAIRS] = 0u;
        if (counters[GS_CTR_STATUS] & GS_STATUS_PAIR_OVERFLOW) counters[GS_CTR_OVERFLOWED] += 1u;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// (visible records, pairs): the pair sum saturates at 2^32 - 1, which is
// above every capacity, so an oversized frame is reported, never wrapped
struct VisPairs {
    uint32_t v, p;
};

__device__ inline uint32_t scan_add(uint32_t a, uint32_t b) { return a + b; }
__device__ inline VisPairs scan_add(VisPairs a, VisPairs b) {
    const uint32_t p = a.p + b.p;
    return {a.v + b.v, p < a.p ? 0xffffffffu : p};
}
__device__ inline uint32_t shfl_up_v(uint32_t x, int off) { return __shfl_up(x, off, kWave); }
__device__ inline VisPairs shfl_up_v(VisPairs x, int off) {
    return {__shfl_up(x.v, off, kWave), __shfl_up(x.p, off, kWave)};
}

// exclusive scan of one value per thread over a B-thread block (s_wave
// holds B / kWave values); total = the block's sum.  Only the
// (associative) scan_add is used.
template <int B = kScanBlock, typename T>
__device__ inline T block_excl_scan(T v, T* s_wave, T& total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    T inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const T t = shfl_up_v(inc, off);
        if (lane >= off) inc = scan_add(t, inc);
    }
    T ex = shfl_up_v(inc, 1);
    if (lane == 0) ex = T{};
    if (lane == kWave - 1) s_wave[wave] = inc;
    __syncthreads();
    T before{};
    total = T{};
#pragma unroll
    for (int w = 0; w < B / kWave; w++) {
        const T s = s_wave[w];
        if (w < wave) before = scan_add(before, s);
        total = scan_add(total, s);
    }
    __syncthreads();
    return scan_add(before, ex);
}

// chunk of items [lo, hi) that block b of G handles when n items are split
__device__ inline void block_range(uint32_t n, int G, int b, uint32_t granule, uint32_t& lo, uint32_t& hi) {
    uint32_t chunk = (n + G - 1) / G;
    chunk = (chunk + granule - 1) / granule * granule;
    lo = min(n, uint32_t(b) * chunk);
    hi = min(n, lo + chunk);
}

// ---------------------------------------------------------------------------
// reduce-then-scan over a sequence of n items (two launches: per-block
// sums, then each block's exclusive prefixes)

struct RecordScan {       // item i: record i; output: compacted ids and first pairs
    using T = VisPairs;
    const uint4* meta;
    uint32_t* vis;
    uint32_t* pair_off;       // by record
    uint32_t* poff;           // by visible rank
    uint32_t* cfirst;         // by emission chunk: the visible rank holding its first pair
    uint64_t capacity;
    __device__ T value(uint32_t i) const {
        const uint32_t n = meta_tiles(meta[i].y);
        return {n > 0 ? 1u : 0u, n};
    }
    __device__ void emit(uint32_t i, T pre, T v) const {
        if (v.v) {
            vis[pre.v] = i;
            poff[pre.v] = pre.p;
            pair_off[i] = pre.p;
            // the emission chunks whose first pair is one of this record's
            const uint64_t p0 = pre.p, p1 = min(p0 + v.p, capacity);
            for (uint64_t c = (p0 + kEmitChunk - 1) / kEmitChunk; c * kEmitChunk < p1; c++) cfirst[c] = pre.v;
        }
    }
    __device__ static void finish(T total, uint32_t* counters, uint64_t capacity) {
        counters[GS_CTR_VISIBLE] = total.v;
        counters[GS_CTR_PAIRS] = total.p;
        if (uint64_t(total.p) > capacity) counters[GS_CTR_STATUS] |= GS_STATUS_PAIR_OVERFLOW;
        if (counters[GS_CTR_STATUS] & GS_STATUS_PAIR_OVERFLOW) counters[GS_CTR_OVERFLOWED] += 1u;
    }
};

// The reduce also zeroes `clear[0, n_clear)` (grid-stride) and the word
// `*clear1` (when not null), for buffers the later steps fill in part or
// count into: it saves launches.  kReduceBlock threads per workgroup over
// the ranges of kScanBlock granules.
constexpr int kReduceBlock = 1024;
template <typename F>
__global__ __launch_bounds__(kReduceBlock) void k_scan_reduce(F f, uint32_t n, typename F::T* __restrict__ part,
                                                              int G, uint32_t* __restrict__ clear, int64_t n_clear,
                                                              uint32_t* __restrict__ clear1) {
    using T = typename F::T;
    __shared__ T s_wave[kReduceBlock / kWave];
    for (int64_t i = int64_t(blockIdx.x) * kReduceBlock + threadIdx.x; i < n_clear; i += int64_t(G) * kReduceBlock)
        clear[i] = 0u;
    if (clear1 != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *clear1 = 0u;
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, kScanBlock, lo, hi);
    T acc{};
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kReduceBlock) acc = scan_add(acc, f.value(i));
    T tot;
    block_excl_scan<kReduceBlock>(acc, s_wave, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Each workgroup's exclusive prefix is the sum of the partials before it (at
// most kMaxGrid, read by the whole workgroup), then its items' prefixes in
// chunks of kApplyBlock (the reduce's ranges, kApplyBlock threads: fewer
// rounds of the block scan); the last workgroup also hands the total to
// F::finish.
constexpr int kApplyBlock = 1024;
template <typename F>
__global__ __launch_bounds__(kApplyBlock) void k_scan_apply(F f, uint32_t n, const typename F::T* __restrict__ part,
                                                            int G, uint32_t* __restrict__ counters,
                                                            uint64_t capacity) {
    using T = typename F::T;
    __shared__ T s_wave[kApplyBlock / kWave];
    T before{};
    for (int i = threadIdx.x; i < int(blockIdx.x); i += kApplyBlock) before = scan_add(before, part[i]);
    T carry;
    block_excl_scan<kApplyBlock>(before, s_wave, carry);
    if (blockIdx.x == unsigned(G - 1) && threadIdx.x == 0) F::finish(scan_add(carry, part[G - 1]), counters, capacity);
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, kScanBlock, lo, hi);
    for (uint32_t base = lo; base < hi; base += kApplyBlock) {
        const uint32_t i = base + threadIdx.x;
        const T v = i < hi ? f.value(i) : T{};
        T tot;
        const T ex = block_excl_scan<kApplyBlock>(v, s_wave, tot);
        if (i < hi) f.emit(i, scan_add(carry, ex), v);
        carry = scan_add(carry, tot);
    }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (uint32 key, uint32 value) by digits of `bits`
// bits (at most 8), reduce-then-scan with a fixed grid of G workgroups over a
// device-sized n; each workgroup takes a contiguous range of the keys

__device__ __forceinline__ uint32_t digit_of(uint32_t k, int shift, int bits) {
    return (k >> shift) & ((1u << bits) - 1u);
}

__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
                                                      uint32_t n_host, int shift, int bits, uint32_t* __restrict__ hist,
                                                      int G, uint32_t granule) {
    __shared__ uint32_t h[kRsBlock / kWave][256];
    const int wave = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < 256 * (kRsBlock / kWave); i += kRsBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = min(*n_dev, n_host);
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, granule, lo, hi);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kRsBlock) atomicAdd(&h[wave][digit_of(keys[i], shift, bits)], 1u);
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kRsBlock / kWave; w++) s += h[w][d];
    hist[d * G + blockIdx.x] = s;
}

// one workgroup per digit: exclusive scan of that digit's counts over the G
// workgroups (in place) and the digit's total; the digits' base offsets are
// then an exclusive scan of 256 totals, done by every scatter workgroup
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

// Scatter: per iteration kRsBlock * ITEMS keys are ranked by digit (wave ballots for
// the rank among equal digits, LDS counts across waves), staged in LDS in
// digit order, then written out by consecutive threads to consecutive
// addresses of each digit's output run.
template <int ITEMS>
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                         uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                         const uint32_t* __restrict__ n_dev, uint32_t n_host, int shift,
                                                         int bits, const uint32_t* __restrict__ hist, int G,
                                                         const uint32_t* __restrict__ coltot) {
    constexpr int NW = kRsBlock / kWave;
    constexpr int PER_WAVE = kWave * ITEMS;
    constexpr int kRsTile = kRsBlock * ITEMS;
    __shared__ uint32_t run[256];          // next output index of each digit
    __shared__ uint32_t loc[256];          // first staging slot of each digit
    __shared__ uint32_t wcnt[NW][256];     // per wave: count, then first rank, of each digit
    __shared__ uint32_t s_wave[NW];
    __shared__ uint32_t sk[kRsTile], sv[kRsTile];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t n = min(*n_dev, n_host);
    uint32_t lo, hi;
    block_range(n, G, blockIdx.x, kRsTile, lo, hi);
    {
        uint32_t tot;
        const uint32_t base = block_excl_scan(coltot[tid], s_wave, tot);
        run[tid] = base + hist[tid * G + blockIdx.x];
    }
    for (uint32_t base = lo; base < hi; base += kRsTile) {
        for (int d = lane; d < 256; d += kWave) wcnt[wave][d] = 0;
        __builtin_amdgcn_wave_barrier();
        uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; k++) {
            const uint32_t i = base + wave * PER_WAVE + k * kWave + lane;
            key[k] = 0; val[k] = 0; rank[k] = 0;
            if (i < hi) {
                key[k] = kin[i];
                val[k] = vin[i];
                const uint32_t dg = digit_of(key[k], shift, bits);
                uint64_t peers = __ballot(1);
                for (int bit = 0; bit < bits; bit++) {
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
        // thread d: the waves' first ranks of digit d, then the digit's first slot
        uint32_t tot = 0;
        {
            const int d = tid;
#pragma unroll
            for (int w = 0; w < NW; w++) {
                const uint32_t c = wcnt[w][d];
                wcnt[w][d] = tot;
                tot += c;
            }
            uint32_t all;
            loc[d] = block_excl_scan(tot, s_wave, all);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; k++) {
            const uint32_t i = base + wave * PER_WAVE + k * kWave + lane;
            if (i < hi) {
                const uint32_t dg = digit_of(key[k], shift, bits);
                const uint32_t pos = loc[dg] + wcnt[wave][dg] + rank[k];
                sk[pos] = key[k];
                sv[pos] = val[k];
            }
        }
        __syncthreads();
        const uint32_t m = min(uint32_t(kRsTile), hi - base);
        for (uint32_t j = tid; j < m; j += kRsBlock) {
            const uint32_t k = sk[j], dg = digit_of(k, shift, bits);
            const uint32_t o = run[dg] + (j - loc[dg]);
            kout[o] = k;
            vout[o] = sv[j];
        }
        __syncthreads();
        run[tid] += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// pair emission and tile ranges

// Pair-parallel emission: workgroup b of G takes the pairs that block b of
// the first radix pass takes (block_range with the same G and granule), in
// chunks of kEmitChunk; each chunk finds the visible records it spans by
// binary search over their first-pair offsets (staged in LDS), so a
// Gaussian covering thousands of tiles is spread over many threads instead
// of serialising one.  With hist set, the workgroup also counts the first
// radix digit (the low bits0 bits of the tile id) of its pairs and stores
// the counts as that pass's histogram column, which saves the pass its
// counting launch.  A chunk's first and last records come from cfirst
// (written by the record scan) instead of binary searches over all visible
// records.
constexpr int kEmitBlock = 256;

__global__ __launch_bounds__(kEmitBlock) void k_emit(const uint4* __restrict__ meta, const uint32_t* __restrict__ vis,
                                                     const uint32_t* __restrict__ poff,
                                                     const uint32_t* __restrict__ cfirst,
                                                     const uint32_t* __restrict__ counters, gs_frame frame,
                                                     uint64_t capacity, uint32_t* __restrict__ tkey,
                                                     uint32_t* __restrict__ tval, int G, uint32_t granule, int bits0,
                                                     uint32_t* __restrict__ hist) {
    static_assert(kEmitBlock == 256, "one histogram bin per thread");
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_rec[kEmitChunk + 1];
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    const uint32_t mask0 = (1u << bits0) - 1u;
    const uint32_t V = counters[GS_CTR_VISIBLE];
    const uint32_t P = uint32_t(min(uint64_t(counters[GS_CTR_PAIRS]), capacity));
    uint32_t lo_e, hi_e;
    block_range(P, G, blockIdx.x, granule, lo_e, hi_e);
    for (uint32_t e0 = lo_e; e0 < hi_e; e0 += kEmitChunk) {
        const uint32_t e1 = min(hi_e, e0 + kEmitChunk);
        // the ranks holding pairs e0 and e1 (both multiples of kEmitChunk
        // unless e1 = P), at most kEmitChunk + 1 of them: the searches below
        // never pick the last one when its first pair is e1
        const uint32_t lo = cfirst[e0 / kEmitChunk];
        const uint32_t hi = e1 < P ? cfirst[e1 / kEmitChunk] : V - 1;
        const uint32_t n = min(uint32_t(kEmitChunk + 1), hi - lo + 1);
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            s_off[i] = poff[lo + i];
            s_rec[i] = vis[lo + i];
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
            const uint32_t t = uint32_t(frame.jobs[j].tile0) + (y0 + k / w) * uint32_t(frame.jobs[j].tiles_x) + x0 + k % w;
            tkey[e] = t;
            tval[e] = r;
            if (hist != nullptr) atomicAdd(&h[t & mask0], 1u);
        }
        __syncthreads();
    }
    if (hist != nullptr) {
        __syncthreads();
        hist[threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
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

// ---------------------------------------------------------------------------
// per-tile depth order: each tile's list (record ids, any order) sorted by the
// unique key (depth bits, record id).  k_tile_sort<ITEMS> (persistent grid,
// one list per workgroup at a time) takes lists of up to kSortBlock * ITEMS
// entries: up to one workgroup's width a rank sort in LDS (each thread
// counts the keys below its own), longer ones a merge sort in LDS (4 keys
// per thread up to 1024 entries, ITEMS beyond).  ITEMS is 8 (16 KB of LDS
// per workgroup, twice as many workgroups resident) unless the frame's
// lists are long on average (ITEMS 16, lists up to 4096 on chip).
// k_tile_sort_long takes the longer lists, one large workgroup each.
//
// The merge sort: every thread sorts E consecutive keys in registers (a
// sorting network), then rounds of pairwise merges double the sorted runs;
// in a round each thread produces E consecutive outputs of its pair of runs,
// finding where they start in the two inputs by binary search along the
// merge path and then merging sequentially (ties go to the first run).  The
// work is O(n log n) with one LDS read and write per key and round.

constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;                           // lists up to 2048 on chip
constexpr int kSortItemsDense = 16;                     // lists up to 4096 on chip
constexpr uint64_t kDenseList = 1024;                   // mean list length (capacity / tiles) above which: dense
constexpr int kSortItemsShort = 4;                      // lists up to 1024: more threads, shorter merges
constexpr int kLongBlock = 1024;
constexpr int kLongItems = 8;
constexpr int kLongChunk = kLongBlock * kLongItems;     // 8192

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

// ascending bitonic network over E keys in registers
template <int E>
__device__ __forceinline__ void sort_registers(uint64_t (&r)[E]) {
#pragma unroll
    for (int k = 2; k <= E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < E; i++) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t a = r[i], b = r[l];
                    const bool swap = (a > b) == ((i & k) == 0);
                    r[i] = swap ? b : a;
                    r[l] = swap ? a : b;
                }
            }
        }
    }
}

// Sorts sk[0, n) ascending in LDS, n <= B * E, by a workgroup of B threads;
// the keys must be visible to the workgroup (a barrier after they were
// written).  sk must hold ceil(n / E) * E keys (the tail is padded with the
// largest key).  Ends with a barrier.
template <int B, int E>
__device__ void block_merge_sort(uint64_t* sk, uint32_t n) {
    const uint32_t np = (n + E - 1) / E * E;
    const uint32_t base = threadIdx.x * E;
    const bool active = base < np;
    for (uint32_t i = n + threadIdx.x; i < np; i += B) sk[i] = ~0ull;
    __syncthreads();
    uint64_t r[E];
    if (active) {
#pragma unroll
        for (int j = 0; j < E; j++) r[j] = sk[base + j];
        sort_registers<E>(r);
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int j = 0; j < E; j++) sk[base + j] = r[j];
    }
    __syncthreads();
    for (uint32_t run = E; run < np; run <<= 1) {
        if (active) {
            const uint32_t a0 = base / (2 * run) * (2 * run);
            const uint32_t a1 = min(a0 + run, np), b1 = min(a0 + 2 * run, np);
            const uint32_t la = a1 - a0, lb = b1 - a1, d = base - a0;
            // outputs [d, d + E) of this pair: how many come from the first run
            uint32_t lo = d > lb ? d - lb : 0u, hi = min(d, la);
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (sk[a0 + mid] <= sk[a1 + d - mid - 1]) lo = mid + 1; else hi = mid;
            }
            uint32_t ia = lo, ib = d - lo;
            uint64_t ka = sk[a0 + min(ia, la - 1)];
            uint64_t kb = lb ? sk[a1 + min(ib, lb - 1)] : 0ull;
#pragma unroll
            for (int j = 0; j < E; j++) {
                const bool from_a = ia < la && (ib >= lb || ka <= kb);
                r[j] = from_a ? ka : kb;
                if (from_a) ia++; else ib++;
                const uint32_t next = from_a ? a0 + min(ia, la - 1) : a1 + min(ib, lb - 1);
                const uint64_t nk = sk[next];
                if (from_a) ka = nk; else kb = nk;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int j = 0; j < E; j++) sk[base + j] = r[j];
        }
        __syncthreads();
    }
}

// Compositing plan for adaptive wavefronts: every tile's wavefront count
// (adaptive_waves of its list length) and the tiles grouped by it, 4-wave
// tiles first (one workgroup each), then 2-wave, then 1-wave tiles; inside
// a group the longer lists first, by buckets of half the frame's mean list
// length (the last bucket open-ended), so that the heaviest tiles of each
// group do not start last.  One workgroup (of any multiple of the
// wavefront); the order inside a bucket is whatever the LDS atomics give,
// which changes no result (each tile is composited on its own).  The first
// pass counts the buckets and keeps each tile's bucket in `cache` (LDS, when
// n_tiles <= cache_cap) for the second, which places the tiles.
constexpr int kPlanBuckets = 16;

__device__ void tile_plan(const uint2* __restrict__ ranges, const uint32_t* __restrict__ counters, int n_tiles,
                          int quads, uint32_t* __restrict__ order, uint8_t* cache, int cache_cap) {
    constexpr int NB = 3 * kPlanBuckets;
    static_assert(NB <= 256, "a tile's bin fits a byte");
    __shared__ uint32_t cnt[NB];
    const bool cached = cache != nullptr && n_tiles <= cache_cap;
    const uint64_t pairs = counters[GS_CTR_PAIRS];
    for (int k = threadIdx.x; k < NB; k += blockDim.x) cnt[k] = 0u;
    __syncthreads();
    // bin: group (4, 2, 1 wavefronts) major, then the length bucket, longest first
    auto bin = [&](int t) {
        const uint32_t n = ranges[t].y - ranges[t].x;
        const int w = adaptive_waves(n, uint32_t(pairs), n_tiles, quads);
        const int grp = w == 4 ? 0 : (w == 2 ? 1 : 2);
        const uint64_t q = pairs ? (2ull * n * uint64_t(n_tiles)) / pairs : 0ull;   // n / (mean / 2)
        const int bucket = q < uint64_t(kPlanBuckets - 1) ? int(q) : kPlanBuckets - 1;
        return grp * kPlanBuckets + (kPlanBuckets - 1 - bucket);
    };
    for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) {
        const int b = bin(t);
        if (cached) cache[t] = uint8_t(b);
        atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0u, tot[3] = {0u, 0u, 0u};
        for (int k = 0; k < NB; k++) {
            const uint32_t c = cnt[k];
            cnt[k] = run;                  // first place of the bin
            run += c;
            tot[k / kPlanBuckets] += c;
        }
        order[0] = tot[0];
        order[1] = tot[1];
        order[2] = tot[2];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) {
        const int b = cached ? int(cache[t]) : bin(t);
        order[4 + atomicAdd(&cnt[b], 1u)] = uint32_t(t);
    }
}

__global__ __launch_bounds__(1024) void k_tile_plan(const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ counters, int n_tiles, int quads,
                                                    uint32_t* __restrict__ order) {
    tile_plan(ranges, counters, n_tiles, quads, order, nullptr, 0);
}

// With order set, workgroup 0 makes the compositing plan (tile_plan) and the
// others sort; the plan only reads the ranges, so it runs beside the sorts.
template <int ITEMS>
__global__ __launch_bounds__(kSortBlock) void k_tile_sort(const uint4* __restrict__ meta,
                                                          const uint2* __restrict__ ranges, int n_tiles,
                                                          uint32_t* __restrict__ vals, uint32_t* __restrict__ longq,
                                                          const uint32_t* __restrict__ counters, int quads,
                                                          uint32_t* __restrict__ order) {
    constexpr int kSortChunk = kSortBlock * ITEMS;
    __shared__ uint64_t sk[kSortChunk];
    const int first = order != nullptr ? 1 : 0;
    if (int(blockIdx.x) < first) {
        tile_plan(ranges, counters, n_tiles, quads, order, reinterpret_cast<uint8_t*>(sk), int(sizeof(sk)));
        return;
    }
    const int nsort = int(gridDim.x) - first;
    for (int tile = int(blockIdx.x) - first; tile < n_tiles; tile += nsort) {
        const uint2 rg = ranges[tile];
        const uint32_t n = rg.y - rg.x;
        if (n < 2) continue;                                   // uniform per workgroup
        if (n > uint32_t(kSortChunk)) {                         // for k_tile_sort_long
            if (threadIdx.x == 0) longq[1 + atomicAdd(&longq[0], 1u)] = uint32_t(tile);
            continue;
        }
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
        for (uint32_t i = threadIdx.x; i < n; i += kSortBlock) sk[i] = depth_key(meta, v[i]);
        __syncthreads();
        if (n <= kSortBlock * kSortItemsShort) block_merge_sort<kSortBlock, kSortItemsShort>(sk, n);
        else block_merge_sort<kSortBlock, ITEMS>(sk, n);
        for (uint32_t i = threadIdx.x; i < n; i += kSortBlock) v[i] = uint32_t(sk[i]);
        __syncthreads();
    }
}

// Lists longer than k_tile_sort takes (queued by it, in any order): one
// workgroup of kLongBlock threads per list,
// chunks of kLongChunk keys merge-sorted in LDS, then (lists longer than a
// chunk) pairwise merges of sorted runs through two scratch ranges (each
// key's place is its index in its run plus the number of smaller keys in the
// other run, by binary search).
__global__ __launch_bounds__(kLongBlock) void k_tile_sort_long(const uint4* __restrict__ meta,
                                                               const uint2* __restrict__ ranges,
                                                               const uint32_t* __restrict__ longq,
                                                               uint32_t* __restrict__ vals, uint64_t* __restrict__ ka,
                                                               uint64_t* __restrict__ kb) {
    __shared__ uint64_t sk[kLongChunk];
    const uint32_t nq = longq[0];
    for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const uint2 rg = ranges[longq[1 + q]];
        const uint32_t n = rg.y - rg.x;
        uint32_t* v = vals + rg.x;
        uint64_t* src = ka + rg.x;
        uint64_t* dst = kb + rg.x;
        for (uint32_t c0 = 0; c0 < n; c0 += kLongChunk) {
            const uint32_t m = min(uint32_t(kLongChunk), n - c0);
            for (uint32_t i = threadIdx.x; i < m; i += kLongBlock) sk[i] = depth_key(meta, v[c0 + i]);
            __syncthreads();
            block_merge_sort<kLongBlock, kLongItems>(sk, m);
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

// ---------------------------------------------------------------------------

static int grid_for(uint64_t n_max, int per_block) {
    uint64_t g = (n_max + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    return int(g);
}

// Grid and keys per workgroup of the radix passes over at most n_max keys.
struct RadixShape {
    bool small;
    uint32_t tile;
    int G;
};
static RadixShape radix_shape(uint32_t n_max) {
    const bool small = n_max <= kRsSmallMax;
    const uint32_t tile = kRsBlock * (small ? kRsItemsSmall : kRsItemsLarge);
    return {small, tile, grid_for(n_max, int(tile))};
}
static int radix_passes(int bits) { return (bits + 7) / 8; }
// width of pass p's digit: near-equal widths over the passes
static int radix_digit(int bits, int p) {
    const int passes = radix_passes(bits);
    int shift = 0;
    for (int q = 0; q < p; q++) shift += (bits - shift) / (passes - q);
    return (bits - shift) / (passes - p);
}

// sorts by the low `bits` bits of the keys in passes of at most 8 bits;
// returns (in k_final) the buffer that holds the sorted keys.  With
// first_hist_done the first pass's histogram is already in w.hist (k_emit
// counted it).
static hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
                             uint32_t n_max, int bits, bool first_hist_done, uint32_t** k_final, hipStream_t s,
                             BinWs& w) {
    const RadixShape rs = radix_shape(n_max);
    const bool small = rs.small;
    const uint32_t tile = rs.tile;
    const int G = rs.G;
    const int passes = radix_passes(bits);
    uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
    for (int p = 0, shift = 0; p < passes; p++) {
        const int b = radix_digit(bits, p);
        if (p > 0 || !first_hist_done)
            GS_LAUNCH("k_rs_hist", k_rs_hist, dim3(G), dim3(kRsBlock), 0, s, ki, n_dev, n_max, shift, b, w.hist, G,
                      tile);
        GS_LAUNCH("k_rs_colscan", k_rs_colscan, dim3(256), dim3(kRsBlock), 0, s, w.hist, G, w.coltot);
        if (small)
            GS_LAUNCH("k_rs_scatter", k_rs_scatter<kRsItemsSmall>, dim3(G), dim3(kRsBlock), 0, s, ki, vi, ko, vo, n_dev,
                      n_max, shift, b, w.hist, G, w.coltot);
        else
            GS_LAUNCH("k_rs_scatter", k_rs_scatter<kRsItemsLarge>, dim3(G), dim3(kRsBlock), 0, s, ki, vi, ko, vo, n_dev,
                      n_max, shift, b, w.hist, G, w.coltot);
        shift += b;
        uint32_t* t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    *k_final = ki;
    return hipGetLastError();
}

hipError_t launch_bin_sort(const gs_frame& f, const gs_raster_cfg& cfg, const uint32_t* meta_u32, const gs_bins& bins,
                           void* ws, size_t ws_bytes, hipStream_t s) {
    (void)ws_bytes;
    BinWs w = carve(ws, f.n_records, bins.capacity, f.n_tiles);
    const uint4* meta = reinterpret_cast<const uint4*>(meta_u32);
    const uint32_t nrec = uint32_t(f.n_records);
    uint2* ranges = reinterpret_cast<uint2*>(bins.ranges);
    // counts restart every call (the record scan writes them); the status
    // bits are sticky until the caller clears them
    const int64_t nt = f.n_tiles;
    const bool want_plan = bins.tile_order && (fwd_waves(cfg) == 0 || bwd_waves(cfg) == 0);
    const int quads = (cfg.tile_w / 8) * (cfg.tile_h / 8);
    auto plan = [&]() {
        if (want_plan)
            GS_LAUNCH("k_tile_plan", k_tile_plan, dim3(1), dim3(1024), 0, s, ranges, bins.counters, f.n_tiles, quads,
                      bins.tile_order);
    };
    if (nrec == 0) {
        GS_LAUNCH("k_counters_empty", k_counters_empty, dim3(1), dim3(64), 0, s, bins.counters);
        GS_LAUNCH("k_fill_u32", k_fill_u32, dim3(unsigned(std::min<int64_t>((2 * nt + 255) / 256, 2048))), dim3(256), 0,
                  s, bins.ranges, 0u, 2 * nt);
        plan();
        return hipGetLastError();
    }

    // 1. visible records in record order, their first pairs; V and P (the
    //    reduce clears the tile ranges, which step 3 fills for tiles with
    //    pairs; and the long-list queue count, which follows the ranges)
    static_assert(sizeof(uint2) == 8, "ranges are pairs of 32-bit words");
    {
        const int G = grid_for(nrec, kScanBlock * 8);
        RecordScan rs{meta, w.vis, bins.pair_off, w.poff, w.cfirst, bins.capacity};
        VisPairs* part = static_cast<VisPairs*>(w.part);
        GS_LAUNCH("k_scan_reduce", k_scan_reduce<RecordScan>, dim3(G), dim3(kReduceBlock), 0, s, rs, nrec, part, G,
                  bins.ranges, 2 * nt, w.longq);
        GS_LAUNCH("k_scan_apply", k_scan_apply<RecordScan>, dim3(G), dim3(kApplyBlock), 0, s, rs, nrec, part, G,
                  bins.counters, bins.capacity);
    }
    // 2. emit (tile, record) pairs in record order, then sort them by tile id
    //    (the emission counts the first radix digit)
    int bits = 0;
    while ((1ll << bits) < nt) bits++;
    const int passes = radix_passes(bits);
    uint32_t* emit_val = (passes & 1) ? w.tval : bins.vals;
    uint32_t* other_val = (passes & 1) ? bins.vals : w.tval;
    const uint32_t pmax = uint32_t(std::min<uint64_t>(bins.capacity, 0xffffffffull));
    if (passes > 0) {
        const RadixShape rs = radix_shape(pmax);
        GS_LAUNCH("k_emit", k_emit, dim3(rs.G), dim3(kEmitBlock), 0, s, meta, w.vis, w.poff, w.cfirst, bins.counters, f,
                  bins.capacity, w.tkey[0], emit_val, rs.G, rs.tile, radix_digit(bits, 0), w.hist);
    } else {
        const int G = grid_for(pmax, kEmitChunk);
        GS_LAUNCH("k_emit", k_emit, dim3(G), dim3(kEmitBlock), 0, s, meta, w.vis, w.poff, w.cfirst, bins.counters, f,
                  bins.capacity, w.tkey[0], emit_val, G, uint32_t(kEmitChunk), 0, static_cast<uint32_t*>(nullptr));
    }
    uint32_t* tk_final = w.tkey[0];
    if (passes > 0) {
        const hipError_t e = radix_sort(w.tkey[0], emit_val, w.tkey[1], other_val, bins.counters + GS_CTR_PAIRS, pmax,
                                        bits, true, &tk_final, s, w);
        if (e != hipSuccess) return e;
    }
    // 3. per-tile [start, end)
    GS_LAUNCH("k_ranges", k_ranges, dim3(2048), dim3(256), 0, s, tk_final, bins.counters, bins.capacity, ranges);
    // 4. each tile's list in (depth bits, record) order, and (5.) beside it
    //    the compositing plan, when a pass splits tiles adaptively
    if (nt > 0) {
        uint32_t* order = want_plan ? bins.tile_order : nullptr;
        const dim3 grid(unsigned(std::min<int64_t>(nt, 4096) + (want_plan ? 1 : 0)));
        if (bins.capacity > uint64_t(nt) * kDenseList)
            GS_LAUNCH("k_tile_sort", k_tile_sort<kSortItemsDense>, grid, dim3(kSortBlock), 0, s, meta, ranges,
                      f.n_tiles, bins.vals, w.longq, bins.counters, quads, order);
        else
            GS_LAUNCH("k_tile_sort", k_tile_sort<kSortItems>, grid, dim3(kSortBlock), 0, s, meta, ranges, f.n_tiles,
                      bins.vals, w.longq, bins.counters, quads, order);
        GS_LAUNCH("k_tile_sort_long", k_tile_sort_long, dim3(unsigned(std::min<int64_t>(nt, 256))), dim3(kLongBlock), 0,
                  s, meta, ranges, w.longq, bins.vals, w.key[0], w.key[1]);
    } else {
        plan();
    }
    return hipGetLastError();
}

}  // namespace gs
