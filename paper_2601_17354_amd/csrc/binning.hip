// Tile binning and the (tile, depth) key sort that yields the permutation pi
// of PocketGS's index-mapping subsection.
//
// The pairs are ordered by (tile, depth bits, canonical id).  Instead of
// sorting all 46 significant key bits of every pair, the Gaussians are
// sorted once by depth and the pairs emitted in that order, so that a stable
// sort on the tile bits alone finishes the order:
//   depth    stable LSD sort of the (depth bits, item) of every Gaussian of
//            every view (4 passes over n items instead of 4 over the pairs)
//   scan     exclusive prefix sum of tiles_touched in depth order -> pair
//            offsets + count
//   emit     one (key, canonical id) pair per Gaussian x rectangle tile,
//            key = tile << 32 | bits(float32 depth), each workgroup filling
//            an equal range of pairs (binary search over the offsets), so
//            large Gaussians do not serialise
//   sort     stable LSD radix sort on the tile bits only, 8-bit digits;
//            every pass is histogram -> device scan of the digit-major
//            histogram -> stable scatter
//   ranges   per-tile [start, end)
//
// Every kernel reads the item and pair counts from device memory and is
// launched on a grid sized for the capacity, so nothing travels to the host
// and the whole sequence can be captured in a HIP graph.
#include <mutex>

#include "common.hpp"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanIpt = 8;
constexpr int kScanItems = kScanThreads * kScanIpt;  // 2048 per block

constexpr int kSortThreads = 256;  // 256 keys per round
// Rounds per workgroup: 8 (2048 keys) for large sorts; 4 (1024 keys) for
// sorts of at most kSmallSort keys, which would otherwise run on too few
// workgroups to fill the chip.
constexpr int kSortRoundsLarge = 8;
constexpr int kSortRoundsSmall = 4;
constexpr uint32_t kSmallSort = 1u << 20;
constexpr int kRadix = 256;

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }
inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Block-wide exclusive scan of one value per thread (Hillis-Steele in LDS).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s, uint32_t& total) {
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint32_t add = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    total = s[kScanThreads - 1];
    const uint32_t incl = s[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                              uint32_t n, uint32_t* __restrict__ partial) {
    __shared__ uint32_t s[kScanThreads];
    const uint32_t base = blockIdx.x * kScanItems + threadIdx.x * kScanIpt;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k)
        if (base + k < n) sum += in[base + k];
    uint32_t total;
    block_exclusive_scan(sum, s, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Per-block exclusive scan of `in` offset by the sum of the preceding
// blocks' partial sums (each block adds those up itself, so the partials
// need no scan launch of their own); the last block writes the grand total
// to *total_out (if not null).  `out` may alias `in`.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint32_t* in, uint32_t n,
                                                             const uint32_t* __restrict__ partial,
                                                             uint32_t* out,
                                                             uint32_t* __restrict__ total_out) {
    __shared__ uint32_t s[kScanThreads];
    uint32_t before = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) before += partial[i];
    uint32_t offset;
    block_exclusive_scan(before, s, offset);
    const uint32_t base = blockIdx.x * kScanItems + threadIdx.x * kScanIpt;
    uint32_t loc[kScanIpt];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
        loc[k] = (base + k < n) ? in[base + k] : 0u;
        sum += loc[k];
    }
    uint32_t total;
    uint32_t run = offset + block_exclusive_scan(sum, s, total);
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
        if (base + k < n) out[base + k] = run;
        run += loc[k];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = offset + total;
}

size_t scan_workspace(uint32_t n) { return align_up((size_t)div_up(n, kScanItems) * 4); }

// Exclusive scan in -> out (may alias), total to total_out (device, may be null).
pgs_status scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total_out,
                    uint32_t* partial, hipStream_t s) {
    const uint32_t nb = div_up(n, kScanItems);
    if (nb == 0) return PGS_OK;
    k_scan_reduce<<<nb, kScanThreads, 0, s>>>(in, n, partial);
    k_scan_apply<<<nb, kScanThreads, 0, s>>>(in, n, partial, out, total_out);
    PGS_CHECK_LAUNCH("scan");
    return PGS_OK;
}

// Items of a bin/sort: item i = v * n + g is Gaussian g in view v (one view:
// v = 0), keyed with view v's global tile numbers; values hold the id g.
struct EmitViews {
    int n_views;
    int TX[PGS_MAX_VIEWS];
    int tile_off[PGS_MAX_VIEWS];
};

__device__ __forceinline__ void view_tiles(const EmitViews& ev, int v, int& TX, int& off) {
    TX = ev.TX[0];
    off = ev.tile_off[0];
    for (int u = 1; u < ev.n_views; ++u)
        if (u == v) {
            TX = ev.TX[u];
            off = ev.tile_off[u];
        }
}

__global__ void k_clear_u32(uint32_t* __restrict__ p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Depth keys of every item (float32 depth bits; culled items sort last),
// values = item index, the item count for the depth sort, and the first
// radix pass's digit histogram: workgroup b takes the same 256 R items as
// the sort's workgroup b, so it writes its column of the digit-major
// histogram itself.  Also clears the tile ranges and the pair count.
template <int R>
__global__ __launch_bounds__(kSortThreads) void k_depth_keys(uint32_t items, int n,
                                                             const float* __restrict__ proj_all,
                                                             const uint32_t* __restrict__ touched_all,
                                                             uint32_t* __restrict__ dkeys,
                                                             uint32_t* __restrict__ dvals,
                                                             uint32_t* __restrict__ count, uint32_t nb,
                                                             uint32_t* __restrict__ hist,
                                                             uint32_t* __restrict__ ranges, uint32_t n_ranges,
                                                             uint32_t* __restrict__ num_pairs) {
    __shared__ uint32_t h[kRadix];
    const int t = threadIdx.x;
    if (blockIdx.x == 0 && t == 0) {
        *count = items;
        *num_pairs = 0u;
    }
    for (uint32_t i = blockIdx.x * kSortThreads + t; i < n_ranges; i += gridDim.x * kSortThreads) ranges[i] = 0u;
    h[t] = 0u;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortThreads * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = base + r * kSortThreads + t;
        if (i < items) {
            // the record's depth is read only for items with pairs (one
            // 4-byte read per 64-byte record, so culled items cost a line)
            uint32_t key = 0xffffffffu;
            if (touched_all[i]) key = __float_as_uint(proj_all[(size_t)i * PGS_PROJ_STRIDE + PGS_PROJ_DEPTH]);
            dkeys[i] = key;
            dvals[i] = i;
            atomicAdd(&h[key & 0xffu], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)t * nb + blockIdx.x] = h[t];
}

// Pairs of the items in depth order.  Workgroup b fills pairs
// [256 R b, 256 R (b + 1)), the range of the pair sort's workgroup b: one
// binary search over the scanned counts finds the item of its first pair;
// every item of the range has at least one pair (empty items share their
// successor's offset), so the range spans at most 256 R items, whose offsets
// go to LDS; each thread then finds its pairs' items there.  The work per
// workgroup is even however unevenly the rectangles are sized.  Each
// workgroup also writes its column of the pair sort's first digit-major
// histogram (the tile's low 8 bits), zeros past the pair count.

__device__ __forceinline__ uint32_t last_le(const uint32_t* off, uint32_t n, uint32_t p) {
    uint32_t lo = 0, hi = n - 1;  // last j with off[j] <= p (off[0] <= p)
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int R>
__global__ __launch_bounds__(kSortThreads) void k_emit_sorted(uint32_t items, int n, EmitViews ev,
                                                              const uint32_t* __restrict__ dkeys,
                                                              const uint32_t* __restrict__ rect_all,
                                                              const uint32_t* __restrict__ dvals,
                                                              const uint32_t* __restrict__ off,
                                                              const uint32_t* __restrict__ num_pairs,
                                                              uint32_t capacity, uint64_t* __restrict__ keys,
                                                              uint32_t* __restrict__ values,
                                                              uint32_t* __restrict__ flags, uint32_t nb,
                                                              uint32_t* __restrict__ hist) {
    constexpr uint32_t kPairs = kSortThreads * R;
    __shared__ uint32_t s_off[kPairs + 1];
    __shared__ uint32_t s_first;
    __shared__ uint32_t h[kRadix];
    const int t = threadIdx.x;
    const uint32_t total = *num_pairs;
    if (blockIdx.x == 0 && t == 0 && total > capacity) atomicOr(flags, PGS_FLAG_PAIR_OVERFLOW);
    const uint32_t count = min(total, capacity);
    const uint32_t p0 = blockIdx.x * kPairs;
    h[t] = 0u;
    if (p0 < count) {  // uniform for the block
        const uint32_t p1 = min(p0 + kPairs, count);
        if (t == 0) s_first = last_le(off, items, p0);
        __syncthreads();
        const uint32_t i0 = s_first;
        const uint32_t span = min(kPairs + 1, items - i0);
        for (uint32_t q = t; q < span; q += kSortThreads) s_off[q] = off[i0 + q];
        __syncthreads();
        for (uint32_t p = p0 + t; p < p1; p += kSortThreads) {
            const uint32_t j = last_le(s_off, span, p);
            const uint32_t item = dvals[i0 + j], local = p - s_off[j];
            const uint32_t v = item / (uint32_t)n, g = item - v * (uint32_t)n;
            int TX, toff;
            view_tiles(ev, (int)v, TX, toff);
            const uint32_t r0 = rect_all[(size_t)v * 2 * n + g], r1 = rect_all[(size_t)v * 2 * n + n + g];
            const uint32_t x0 = r0 & 0xffff, y0 = r0 >> 16, x1 = r1 & 0xffff;
            const uint32_t w = x1 - x0 + 1;
            const uint32_t ty = y0 + local / w, tx = x0 + local % w;
            const uint64_t tile = (uint64_t)((uint32_t)toff + ty * (uint32_t)TX + tx);
            // the depth bits are the sorted key itself (no read of the record)
            const uint32_t dbits = dkeys[i0 + j];
            keys[p] = (tile << 32) | (uint64_t)dbits;
            values[p] = g;
            atomicAdd(&h[(uint32_t)tile & 0xffu], 1u);
        }
    }
    __syncthreads();
    if (blockIdx.x < nb) hist[(size_t)t * nb + blockIdx.x] = h[t];
}

__device__ __forceinline__ uint32_t clamp_count(const uint32_t* num, uint32_t capacity) {
    const uint32_t c = *num;
    return c < capacity ? c : capacity;
}

// Digit histogram of each block's chunk of 256 R keys, stored digit-major
// hist[d * nb + block] so that one exclusive scan yields every block's
// output offset for every digit.
template <int R, class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K* __restrict__ keys,
                                                             const uint32_t* __restrict__ num,
                                                             uint32_t capacity, int shift, uint32_t nb,
                                                             uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kRadix];
    const uint32_t count = clamp_count(num, capacity);
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortThreads * R;
    if (base < count) {
        uint32_t d[R];  // every load in flight before the first atomic
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t idx = base + r * kSortThreads + threadIdx.x;
            d[r] = idx < count ? (uint32_t)(keys[idx] >> shift) & 0xffu : kRadix;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (d[r] < kRadix) atomicAdd(&h[d[r]], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter through LDS.  The block's digit counts are the differences
// of consecutive entries of the scanned digit-major histogram (the last
// entry's successor is the key count).  Each round handles 256 consecutive
// keys; a key's position inside the block is (the digit's start in the
// block) + (keys of its digit already placed) + (same digit in lower waves
// of this round) + (same digit in lower lanes of its wave), the last found
// by matching the 8 digit bits with wave ballots.  The keys go to LDS in
// that order and leave as one contiguous run per digit, so the global
// writes coalesce.  With gdst, the pass also writes gdst[pos] = gsrc[value]
// (a gather in the output order).
template <int R, class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin,
    K* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ num,
    uint32_t capacity, int shift, uint32_t nb, const uint32_t* __restrict__ offs,
    const uint32_t* __restrict__ gsrc, uint32_t* __restrict__ gdst) {
    constexpr int NW = kSortThreads / 64;
    __shared__ K s_key[kSortThreads * R];
    __shared__ uint32_t s_val[kSortThreads * R];
    __shared__ uint32_t s_run[kRadix];     // next local position per digit
    __shared__ uint32_t s_lbase[kRadix];   // digit start inside the block
    __shared__ uint32_t s_gbase[kRadix];   // digit start in the output
    __shared__ uint32_t s_wcnt[2][NW][kRadix];  // per-wave digit counts, two rounds in flight
    __shared__ uint32_t s_scan[kSortThreads];
    const uint32_t count = clamp_count(num, capacity);
    const uint32_t base = blockIdx.x * kSortThreads * R;
    if (base >= count) return;  // uniform for the block
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const size_t e = (size_t)t * nb + blockIdx.x;
    const uint32_t g0 = offs[e];
    const uint32_t g1 = (e + 1 < (size_t)kRadix * nb) ? offs[e + 1] : count;
    s_gbase[t] = g0;
    for (int w = 0; w < NW; ++w) s_wcnt[0][w][t] = s_wcnt[1][w][t] = 0;
    uint32_t total;
    const uint32_t lb = block_exclusive_scan(g1 - g0, s_scan, total);
    s_lbase[t] = lb;
    s_run[t] = lb;
    // All of the block's loads are issued before the first round, so the
    // rounds wait on LDS only.
    K kreg[R];
    uint32_t vreg[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = base + r * kSortThreads + t;
        kreg[r] = idx < count ? kin[idx] : (K)0;
        vreg[r] = idx < count ? vin[idx] : 0u;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        uint32_t (*cnt)[kRadix] = s_wcnt[r & 1];
        const bool valid = base + r * kSortThreads + t < count;
        const uint32_t digit = (uint32_t)(kreg[r] >> shift) & 0xffu;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) cnt[wv][digit] = __popcll(peers);
        __syncthreads();
        // The other buffer was last read before this barrier; clear it for
        // the next round, whose writes come after the next barrier.
        for (int w = 0; w < NW; ++w) s_wcnt[(r + 1) & 1][w][t] = 0;
        if (valid) {
            uint32_t pos = s_run[digit] + rank;
            for (int w = 0; w < wv; ++w) pos += cnt[w][digit];
            s_key[pos] = kreg[r];
            s_val[pos] = vreg[r];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < NW; ++w) add += cnt[w][t];
        s_run[t] += add;
    }
    const uint32_t here = min((uint32_t)kSortThreads * R, count - base);
    for (uint32_t i = t; i < here; i += kSortThreads) {
        const K key = s_key[i];
        const uint32_t d = (uint32_t)(key >> shift) & 0xffu;
        const uint32_t pos = s_gbase[d] + (i - s_lbase[d]);
        kout[pos] = key;
        vout[pos] = s_val[i];
        if (gdst) gdst[pos] = gsrc[s_val[i]];
    }
}

template <class K>
__global__ void k_copy_pairs(const K* __restrict__ ks, const uint32_t* __restrict__ vs,
                             K* __restrict__ kd, uint32_t* __restrict__ vd,
                             const uint32_t* __restrict__ num, uint32_t capacity) {
    const uint32_t count = clamp_count(num, capacity);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

__global__ void k_ranges(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ num,
                         uint32_t capacity, uint32_t n_tiles, uint32_t* __restrict__ ranges) {
    const uint32_t count = clamp_count(num, capacity);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint32_t tile = (uint32_t)(keys[i] >> 32);
        if (tile >= n_tiles) continue;
        if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[tile] = i;
        if (i + 1 == count || (uint32_t)(keys[i + 1] >> 32) != tile) ranges[n_tiles + tile] = i + 1;
    }
}

// Heavy-first tile order: a one-workgroup counting sort of the view's tiles
// by list length in 8-pair buckets, longest first, so the longest tiles start
// first and the launch has no long tail.  Order inside a bucket is arbitrary;
// it only changes scheduling, never a result.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 256;

__device__ __forceinline__ uint32_t order_bucket(const uint32_t* ranges, uint32_t n_tiles_total, uint32_t gt) {
    const uint32_t len = ranges[n_tiles_total + gt] - ranges[gt];
    const uint32_t b = len >> 3;
    return (kOrderBuckets - 1) - (b < (uint32_t)(kOrderBuckets - 1) ? b : (uint32_t)(kOrderBuckets - 1));
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint32_t* __restrict__ ranges,
                                                              uint32_t n_view, uint32_t offset,
                                                              uint32_t n_tiles_total,
                                                              uint32_t* __restrict__ order) {
    __shared__ uint32_t hist[kOrderBuckets];
    for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderThreads) hist[b] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_view; i += kOrderThreads)
        atomicAdd(&hist[order_bucket(ranges, n_tiles_total, offset + i)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int b = 0; b < kOrderBuckets; ++b) {
            const uint32_t c = hist[b];
            hist[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_view; i += kOrderThreads) {
        const uint32_t pos = atomicAdd(&hist[order_bucket(ranges, n_tiles_total, offset + i)], 1u);
        order[pos] = i;
    }
}

struct SortWs {
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* hist;
    uint32_t* partial;
    uint32_t nb;
    int rounds;
    size_t bytes;
};

SortWs sort_layout(void* base, uint32_t capacity) {
    SortWs w{};
    const int rounds = capacity <= kSmallSort ? kSortRoundsSmall : kSortRoundsLarge;
    const uint32_t nb = div_up(capacity, (uint64_t)kSortThreads * rounds);
    size_t off = 0;
    char* p = static_cast<char*>(base);
    w.keys_alt = reinterpret_cast<uint64_t*>(p + off); off += align_up((size_t)capacity * 8);
    w.vals_alt = reinterpret_cast<uint32_t*>(p + off); off += align_up((size_t)capacity * 4);
    w.hist = reinterpret_cast<uint32_t*>(p + off); off += align_up((size_t)nb * kRadix * 4);
    w.partial = reinterpret_cast<uint32_t*>(p + off); off += scan_workspace(nb * kRadix);
    w.nb = nb;
    w.rounds = rounds;
    w.bytes = off;
    return w;
}

// Sorts key bits [start_bit, start_bit + key_bits) (stable).  first_hist:
// the caller already wrote the first pass's digit histogram into w.hist.
// With gdst, the last pass also writes gdst[i] = gsrc[value at i].
// Keys of type K (uint64_t, or uint32_t for the depth sort, whose keys are
// 32 bits: a third less traffic per pass); the ping-pong key buffer is sized
// for 64-bit keys and holds either.
template <class K>
pgs_status radix_sort(K* keys, uint32_t* vals, const uint32_t* num, uint32_t capacity,
                      int key_bits, const SortWs& w, hipStream_t s, int start_bit = 0, bool first_hist = false,
                      const uint32_t* gsrc = nullptr, uint32_t* gdst = nullptr) {
    if (capacity == 0) return PGS_OK;
    const int passes = (key_bits + 7) / 8;
    K* kin = keys; uint32_t* vin = vals;
    K* kout = reinterpret_cast<K*>(w.keys_alt); uint32_t* vout = w.vals_alt;
    for (int p = 0; p < passes; ++p) {
        const int shift = start_bit + 8 * p;
        const bool last = p + 1 == passes;
        const uint32_t* gs = last ? gsrc : nullptr;
        uint32_t* gd = last ? gdst : nullptr;
        if (p > 0 || !first_hist) {
            if (w.rounds == kSortRoundsSmall)
                k_radix_hist<kSortRoundsSmall, K><<<w.nb, kSortThreads, 0, s>>>(kin, num, capacity, shift, w.nb,
                                                                                w.hist);
            else
                k_radix_hist<kSortRoundsLarge, K><<<w.nb, kSortThreads, 0, s>>>(kin, num, capacity, shift, w.nb,
                                                                                w.hist);
        }
        pgs_status st = scan_u32(w.hist, w.hist, w.nb * kRadix, nullptr, w.partial, s);
        if (st != PGS_OK) return st;
        if (w.rounds == kSortRoundsSmall)
            k_radix_scatter<kSortRoundsSmall, K><<<w.nb, kSortThreads, 0, s>>>(kin, vin, kout, vout, num, capacity,
                                                                               shift, w.nb, w.hist, gs, gd);
        else
            k_radix_scatter<kSortRoundsLarge, K><<<w.nb, kSortThreads, 0, s>>>(kin, vin, kout, vout, num, capacity,
                                                                               shift, w.nb, w.hist, gs, gd);
        PGS_CHECK_LAUNCH("radix pass");
        K* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
    }
    if (kin != keys) {
        k_copy_pairs<K><<<1024, 256, 0, s>>>(kin, vin, keys, vals, num, capacity);
        PGS_CHECK_LAUNCH("radix copy");
    }
    return PGS_OK;
}

int bits_for(uint32_t v) {  // number of bits needed for values < v
    int b = 0;
    while (b < 32 && ((uint64_t)1 << b) < v) ++b;
    return b;
}

}  // namespace

extern "C" size_t pgs_sort_workspace(uint32_t capacity) { return sort_layout(nullptr, capacity).bytes; }

extern "C" pgs_status pgs_tile_order(const uint32_t* ranges_dev, int32_t tiles_in_view,
                                     int32_t view_tile_offset, int32_t n_tiles, uint32_t* order_dev,
                                     void* stream) {
    PGS_REQUIRE(tiles_in_view > 0 && view_tile_offset >= 0 && view_tile_offset + tiles_in_view <= n_tiles,
                "pgs_tile_order: bad tile counts");
    PGS_REQUIRE(ranges_dev && order_dev, "pgs_tile_order: null pointer");
    k_tile_order<<<1, kOrderThreads, 0, pgs::as_stream(stream)>>>(ranges_dev, (uint32_t)tiles_in_view,
                                                                 (uint32_t)view_tile_offset, (uint32_t)n_tiles,
                                                                 order_dev);
    PGS_CHECK_LAUNCH("pgs_tile_order");
    return PGS_OK;
}

extern "C" pgs_status pgs_sort_pairs(uint64_t* keys_dev, uint32_t* values_dev, const uint32_t* count_dev,
                                     uint32_t capacity, int32_t key_bits, void* workspace_dev,
                                     size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(key_bits >= 1 && key_bits <= 64, "pgs_sort_pairs: key_bits %d", key_bits);
    if (capacity == 0) return PGS_OK;
    PGS_REQUIRE(keys_dev && values_dev && count_dev && workspace_dev, "pgs_sort_pairs: null pointer");
    SortWs w = sort_layout(workspace_dev, capacity);
    PGS_REQUIRE(workspace_bytes >= w.bytes, "pgs_sort_pairs: workspace %zu < %zu", workspace_bytes, w.bytes);
    return radix_sort(keys_dev, values_dev, count_dev, capacity, key_bits, w, pgs::as_stream(stream));
}

// Workspace of pgs_sort_pairs_noalloc: one array per GPU, in the code
// object, alive until the process ends.  Host code must not pass the name
// `scratch` to a kernel (on the host it is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress gave for the device.
static __device__ __align__(256) unsigned char scratch[PGS_SORT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
pgs_status scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        pgs::set_error("pgs_sort_pairs_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return PGS_ERR_HIP;
    }
    PGS_REQUIRE(dev >= 0 && dev < kMaxDevices, "pgs_sort_pairs_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            pgs::set_error("pgs_sort_pairs_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return PGS_ERR_HIP;
        }
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return PGS_OK;
}

}  // namespace

extern "C" pgs_status pgs_sort_pairs_noalloc(uint64_t* keys_dev, uint32_t* values_dev, const uint32_t* count_dev,
                                             uint32_t capacity, int32_t key_bits, void* stream) {
    PGS_REQUIRE(key_bits >= 1 && key_bits <= 64, "pgs_sort_pairs_noalloc: key_bits %d", key_bits);
    PGS_REQUIRE(capacity <= PGS_SORT_NOALLOC_MAX_PAIRS,
                "pgs_sort_pairs_noalloc: capacity %u exceeds the %u pairs its fixed scratch holds "
                "(use pgs_sort_pairs with a workspace)", capacity, (unsigned)PGS_SORT_NOALLOC_MAX_PAIRS);
    if (capacity == 0) return PGS_OK;
    PGS_REQUIRE(keys_dev && values_dev && count_dev, "pgs_sort_pairs_noalloc: null pointer");
    const size_t need = sort_layout(nullptr, capacity).bytes;
    PGS_REQUIRE(need <= sizeof(scratch), "pgs_sort_pairs_noalloc: workspace %zu exceeds the scratch (%zu)", need,
                sizeof(scratch));
    void* ws = nullptr;
    const pgs_status st = scratch_address(&ws);
    if (st != PGS_OK) return st;
    return radix_sort(keys_dev, values_dev, count_dev, capacity, key_bits, sort_layout(ws, capacity),
                      pgs::as_stream(stream));
}

namespace {

// Workspace of a bin/sort over `items` Gaussians (all views) and `capacity`
// pairs: depth keys and item ids, pair offsets, scan partials, the item
// count word, and the two sorts' ping-pong buffers.
struct BinWs {
    uint32_t* dkeys;
    uint32_t* dvals;
    uint32_t* off;
    uint32_t* partial;
    uint32_t* count;
    SortWs items_ws;
    SortWs pairs_ws;
    size_t bytes;
};

BinWs bin_layout(void* base, uint32_t items, uint32_t capacity) {
    BinWs w{};
    char* p = static_cast<char*>(base);
    size_t off = 0;
    w.dkeys = reinterpret_cast<uint32_t*>(p + off); off += align_up((size_t)items * 4);
    w.dvals = reinterpret_cast<uint32_t*>(p + off); off += align_up((size_t)items * 4);
    w.off = reinterpret_cast<uint32_t*>(p + off); off += align_up((size_t)items * 4);
    w.partial = reinterpret_cast<uint32_t*>(p + off); off += scan_workspace(items);
    w.count = reinterpret_cast<uint32_t*>(p + off); off += align_up(4);
    w.items_ws = sort_layout(p ? p + off : nullptr, items); off += w.items_ws.bytes;
    w.pairs_ws = sort_layout(p ? p + off : nullptr, capacity); off += w.pairs_ws.bytes;
    w.bytes = off;
    return w;
}

pgs_status bin_sort_items(uint32_t items, int n, const EmitViews& ev, int n_tiles, const float* proj_all,
                          const uint32_t* rect_all, const uint32_t* touched_all, uint32_t capacity,
                          uint64_t* keys, uint32_t* values, uint32_t* ranges, uint32_t* num_pairs,
                          uint32_t* flags, const BinWs& w, hipStream_t s, const char* who) {
    if (items == 0) {
        k_clear_u32<<<256, 256, 0, s>>>(ranges, 2u * (uint32_t)n_tiles);
        k_clear_u32<<<1, 64, 0, s>>>(num_pairs, 1u);
        PGS_CHECK_LAUNCH(who);
        return PGS_OK;
    }
    // depth keys with the first depth pass's histogram (and the clears of
    // ranges and pair count); the depth sort's last pass gathers
    // tiles_touched into depth order; the emit writes the pair sort's first
    // histogram
    const SortWs& iw = w.items_ws;
    if (iw.rounds == kSortRoundsSmall)
        k_depth_keys<kSortRoundsSmall><<<iw.nb, kSortThreads, 0, s>>>(items, n, proj_all, touched_all, w.dkeys,
                                                                      w.dvals, w.count, iw.nb, iw.hist, ranges,
                                                                      2u * (uint32_t)n_tiles, num_pairs);
    else
        k_depth_keys<kSortRoundsLarge><<<iw.nb, kSortThreads, 0, s>>>(items, n, proj_all, touched_all, w.dkeys,
                                                                      w.dvals, w.count, iw.nb, iw.hist, ranges,
                                                                      2u * (uint32_t)n_tiles, num_pairs);
    PGS_CHECK_LAUNCH(who);
    pgs_status st = radix_sort(w.dkeys, w.dvals, w.count, items, 32, iw, s, 0, true, touched_all, w.off);
    if (st != PGS_OK) return st;
    st = scan_u32(w.off, w.off, items, num_pairs, w.partial, s);
    if (st != PGS_OK) return st;
    const SortWs& pw = w.pairs_ws;
    const uint32_t ge = pw.nb > 0 ? pw.nb : 1u;
    if (pw.rounds == kSortRoundsSmall)
        k_emit_sorted<kSortRoundsSmall><<<ge, kSortThreads, 0, s>>>(items, n, ev, w.dkeys, rect_all, w.dvals,
                                                                    w.off, num_pairs, capacity, keys, values,
                                                                    flags, pw.nb, pw.hist);
    else
        k_emit_sorted<kSortRoundsLarge><<<ge, kSortThreads, 0, s>>>(items, n, ev, w.dkeys, rect_all, w.dvals,
                                                                    w.off, num_pairs, capacity, keys, values,
                                                                    flags, pw.nb, pw.hist);
    PGS_CHECK_LAUNCH(who);
    if (capacity == 0) return PGS_OK;
    st = radix_sort(keys, values, num_pairs, capacity, bits_for((uint32_t)n_tiles), pw, s, 32, true);
    if (st != PGS_OK) return st;
    const uint32_t grid = div_up(capacity, 256) < 4096 ? div_up(capacity, 256) : 4096;
    k_ranges<<<grid, 256, 0, s>>>(keys, num_pairs, capacity, (uint32_t)n_tiles, ranges);
    PGS_CHECK_LAUNCH(who);
    return PGS_OK;
}

}  // namespace

extern "C" size_t pgs_bin_sort_workspace(int32_t n, uint32_t capacity) {
    return bin_layout(nullptr, n > 0 ? (uint32_t)n : 0u, capacity).bytes;
}

extern "C" pgs_status pgs_bin_sort(int32_t n, const float* proj_dev, const uint32_t* rect_dev,
                                   const uint32_t* touched_dev, int32_t tiles_x, int32_t n_tiles,
                                   int32_t view_tile_offset, uint32_t capacity, uint64_t* keys_dev,
                                   uint32_t* values_dev, uint32_t* ranges_dev, uint32_t* num_pairs_dev,
                                   uint32_t* flags_dev, void* workspace_dev, size_t workspace_bytes,
                                   void* stream) {
    PGS_REQUIRE(n >= 0 && tiles_x > 0 && n_tiles > 0 && view_tile_offset >= 0 &&
                    view_tile_offset < n_tiles, "pgs_bin_sort: bad sizes");
    PGS_REQUIRE(ranges_dev && num_pairs_dev && flags_dev, "pgs_bin_sort: null pointer");
    PGS_REQUIRE(n == 0 || (proj_dev && rect_dev && touched_dev), "pgs_bin_sort: null pointer");
    PGS_REQUIRE(capacity == 0 || (keys_dev && values_dev), "pgs_bin_sort: null pointer");
    const size_t need = pgs_bin_sort_workspace(n, capacity);
    PGS_REQUIRE(workspace_dev && workspace_bytes >= need, "pgs_bin_sort: workspace %zu < %zu",
                workspace_bytes, need);
    EmitViews ev{};
    ev.n_views = 1;
    ev.TX[0] = tiles_x;
    ev.tile_off[0] = view_tile_offset;
    const BinWs w = bin_layout(workspace_dev, (uint32_t)n, capacity);
    return bin_sort_items((uint32_t)n, n > 0 ? n : 1, ev, n_tiles, proj_dev, rect_dev, touched_dev, capacity,
                          keys_dev, values_dev, ranges_dev, num_pairs_dev, flags_dev, w, pgs::as_stream(stream),
                          "pgs_bin_sort");
}

extern "C" pgs_status pgs_bin_sort_views(const pgs_view_batch* views, int32_t n, const float* proj_all_dev,
                                         const uint32_t* rect_all_dev, const uint32_t* touched_all_dev,
                                         uint32_t capacity, uint64_t* keys_dev, uint32_t* values_dev,
                                         uint32_t* ranges_dev, uint32_t* num_pairs_dev, uint32_t* flags_dev,
                                         void* workspace_dev, size_t workspace_bytes, void* stream) {
    pgs_status st = pgs::check_views(views, "pgs_bin_sort_views");
    if (st != PGS_OK) return st;
    PGS_REQUIRE(n >= 0 && (int64_t)n * views->n_views < (1ll << 31), "pgs_bin_sort_views: bad n");
    PGS_REQUIRE(ranges_dev && num_pairs_dev && flags_dev, "pgs_bin_sort_views: null pointer");
    PGS_REQUIRE(n == 0 || (proj_all_dev && rect_all_dev && touched_all_dev), "pgs_bin_sort_views: null pointer");
    PGS_REQUIRE(capacity == 0 || (keys_dev && values_dev), "pgs_bin_sort_views: null pointer");
    const int32_t items = n * views->n_views;
    const size_t need = pgs_bin_sort_workspace(items, capacity);
    PGS_REQUIRE(workspace_dev && workspace_bytes >= need, "pgs_bin_sort_views: workspace %zu < %zu",
                workspace_bytes, need);
    const pgs::ViewsLayout lay = pgs::views_layout(*views);
    EmitViews ev{};
    ev.n_views = views->n_views;
    for (int v = 0; v < views->n_views; ++v) {
        ev.TX[v] = lay.TX[v];
        ev.tile_off[v] = lay.tile_off[v];
    }
    const BinWs w = bin_layout(workspace_dev, (uint32_t)items, capacity);
    return bin_sort_items((uint32_t)items, n > 0 ? n : 1, ev, lay.tile_off[views->n_views], proj_all_dev,
                          rect_all_dev, touched_all_dev, capacity, keys_dev, values_dev, ranges_dev, num_pairs_dev,
                          flags_dev, w, pgs::as_stream(stream), "pgs_bin_sort_views");
}
