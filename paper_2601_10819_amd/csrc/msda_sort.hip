// Stable LSD radix sort of (key, value) u32 pairs and segment boundaries,
// the grouping step of the deterministic grad_feat reduction.
//
// The backward gather writes one record per sample, at the sample's index:
// key = the bilinear cell the sample falls in (or the number of cells, a
// sentinel that sorts last, for a sample outside its level). A stable sort
// by key leaves each cell's records contiguous and in sample order, so the
// tiled reduction that follows sums them in a fixed order: grad_feat is
// bitwise reproducible, and no float atomics are needed.
//
// The key bits are split into as few passes as digits of at most 8 bits
// allow (a 20-bit key space, about a million cells, takes three of 7 bits:
// wider digits leave runs too short for whole-line writes and cost more
// ballots). Each pass: a per-tile digit histogram (one row per tile), the
// tiles' global offsets per digit (band sums, then a walk down each band),
// then a stable scatter where a tile ranks equal digits by wave ballots,
// sorts itself by digit in LDS and writes each digit's run to consecutive
// addresses.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // elements per tile
constexpr int kMaxDigitBits = 8;
constexpr int kMaxDigits = 1 << kMaxDigitBits;         // one thread per digit below
constexpr int kBand = 32;                              // tiles per band of the offset scan
constexpr int kScanTile = 4096;                          // scan: 256 threads x 16

__global__ void __launch_bounds__(kSortThreads)
radix_hist_kernel(const u32* __restrict__ keys, u32 n, const u32* n_dev, int shift, int bits,
                  u32* __restrict__ table, u32 ntiles) {
    __shared__ u32 h[kMaxDigits];
    if (n_dev) n = min(n, *n_dev);
    const int digits = 1 << bits;
    for (int d = threadIdx.x; d < digits; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const u32 mask = (u32)digits - 1u;
    const u32 base = blockIdx.x * (u32)kSortTile;
    u32 k[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {          // every load in flight at once
        const u32 idx = base + i * kSortThreads + threadIdx.x;
        k[i] = idx < n ? keys[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
        if (base + i * kSortThreads + threadIdx.x < n) atomicAdd(&h[(k[i] >> shift) & mask], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < digits; d += kSortThreads)
        table[(size_t)blockIdx.x * digits + d] = h[d];      // tile-major: one coalesced row
}

// Tile offsets from the tile-major count table, in two launches: the column
// sums of each band of kBand tiles, then per band: the digit's start over the
// whole input (an exclusive scan over digits of the digit totals) + the
// counts of earlier bands, walked down the band's tiles in order, each count
// replaced by its tile's global start for the digit. One thread per digit.
__global__ void __launch_bounds__(kMaxDigits) digit_band_kernel(const u32* __restrict__ table,
                                                                u32 ntiles, int digits,
                                                                u32* __restrict__ band_sum) {
    const int d = threadIdx.x;
    if (d >= digits) return;
    const u32 t0 = blockIdx.x * (u32)kBand;
    u32 c[kBand];
#pragma unroll
    for (int k = 0; k < kBand; ++k)            // every load in flight at once
        c[k] = t0 + k < ntiles ? table[(size_t)(t0 + k) * digits + d] : 0u;
    u32 s = 0;
#pragma unroll
    for (int k = 0; k < kBand; ++k) s += c[k];
    band_sum[(size_t)blockIdx.x * digits + d] = s;
}

__global__ void __launch_bounds__(kMaxDigits) digit_offsets_kernel(u32* __restrict__ table,
                                                                   u32 ntiles, int digits,
                                                                   const u32* __restrict__ band_sum,
                                                                   u32 nbands) {
    __shared__ u32 lds4[4];
    const int d = threadIdx.x;
    const u32 t0 = blockIdx.x * (u32)kBand;
    u32 c[kBand];
    u32 total = 0, before = 0;
    if (d < digits) {
#pragma unroll
        for (int k = 0; k < kBand; ++k)
            c[k] = t0 + k < ntiles ? table[(size_t)(t0 + k) * digits + d] : 0u;
        constexpr int kStep = 8;               // band sums read 8 at a time
        for (u32 b = 0; b < nbands; b += kStep) {
            u32 v[kStep];
#pragma unroll
            for (int k = 0; k < kStep; ++k)
                v[k] = b + k < nbands ? band_sum[(size_t)(b + k) * digits + d] : 0u;
#pragma unroll
            for (int k = 0; k < kStep; ++k) {
                total += v[k];
                if (b + k < blockIdx.x) before += v[k];
            }
        }
    }
    u32 all;
    u32 off = block_inclusive_scan(total, lds4, &all) - total + before;
    if (d >= digits) return;
#pragma unroll
    for (int k = 0; k < kBand; ++k) {
        if (t0 + k < ntiles) {
            table[(size_t)(t0 + k) * digits + d] = off;
            off += c[k];
        }
    }
}

// Scan, phase 1: per-tile sums.
__global__ void __launch_bounds__(256) scan_reduce_kernel(const u32* __restrict__ x, u32 n,
                                                          u32* __restrict__ partial) {
    __shared__ u32 lds4[4];
    const u32 base = blockIdx.x * (u32)kScanTile + threadIdx.x * 16u;
    u32 s = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < n) s += x[base + i];
    u32 total;
    block_inclusive_scan(s, lds4, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Scan, phase 2: exclusive scan of the tile sums in one block.
__global__ void __launch_bounds__(256) scan_partials_kernel(u32* partial, u32 np) {
    __shared__ u32 lds4[4];
    const u32 per = (np + 255) / 256;
    const u32 b0 = threadIdx.x * per;
    u32 s = 0;
    for (u32 i = 0; i < per; ++i)
        if (b0 + i < np) s += partial[b0 + i];
    u32 total;
    const u32 incl = block_inclusive_scan(s, lds4, &total);
    u32 run = incl - s;
    for (u32 i = 0; i < per; ++i) {
        if (b0 + i < np) {
            const u32 v = partial[b0 + i];
            partial[b0 + i] = run;
            run += v;
        }
    }
}

// Scan, phase 3: exclusive scan within each tile, offset by its tile sum.
__global__ void __launch_bounds__(256) scan_apply_kernel(u32* x, u32 n,
                                                         const u32* __restrict__ partial) {
    __shared__ u32 lds4[4];
    const u32 base = blockIdx.x * (u32)kScanTile + threadIdx.x * 16u;
    u32 v[16];
    u32 s = 0;
    for (int i = 0; i < 16; ++i) {
        v[i] = base + i < n ? x[base + i] : 0u;
        s += v[i];
    }
    u32 total;
    const u32 incl = block_inclusive_scan(s, lds4, &total);
    u32 run = incl - s + partial[blockIdx.x];
    for (int i = 0; i < 16; ++i) {
        if (base + i < n) x[base + i] = run;
        run += v[i];
    }
}

// Stable scatter of one tile by the `bits`-bit digit at `shift`. vals_in ==
// nullptr means the value is the element's index (first pass).
//
// Wave w owns the tile's elements [w*kWaveItems, (w+1)*kWaveItems) and loads
// all of them at once (lane-consecutive, kSortItems per lane). Ranking needs
// no block barrier: per round of 64, lanes with equal digits are found with
// one ballot per digit bit and ranked by lane, and the wave's running count
// of the digit (in LDS, one row per wave) is read by every peer and advanced
// by the group size. After the rounds, per digit, the waves' counts become
// exclusive prefixes in wave order, offset by the digit's start in the tile
// (an exclusive scan of the tile's digit counts), so an element's place in
// the tile, sorted by digit, is that start + its running rank: wave order,
// then round order, then lane order, i.e. index order (stable). The tile is
// sorted in LDS, then written out by consecutive lanes, so each digit's run
// leaves as consecutive addresses.
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kWaveItems = 64 * kSortItems;

template <int BITS>
__global__ void __launch_bounds__(kSortThreads)
radix_scatter_kernel(const u32* __restrict__ keys_in, const u32* __restrict__ vals_in,
                     u32* __restrict__ keys_out, u32* __restrict__ vals_out, u32 n,
                     const u32* n_dev, int shift, const u32* __restrict__ table) {
    constexpr int bits = BITS;
    __shared__ u32 s_keys[kSortTile];
    __shared__ u32 s_vals[kSortTile];
    __shared__ u32 wcount[kSortWaves][kMaxDigits];
    __shared__ u32 dest_base[kMaxDigits];      // global start - start in the tile (mod 2^32)
    __shared__ u32 lds4[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int digits = 1 << bits;
    const u32 mask = (u32)digits - 1u;
    if (n_dev) n = min(n, *n_dev);
    const u32 tile0 = blockIdx.x * (u32)kSortTile;
    if (tile0 >= n) return;                    // block-uniform: a tile past a device count
    const u32 tile_n = min((u32)kSortTile, n - tile0);
    for (int i = tid; i < kSortWaves * digits; i += kSortThreads)
        wcount[i / digits][i % digits] = 0;

    u32 key[kSortItems], val[kSortItems], rank[kSortItems];
    const u32 w0 = tile0 + (u32)(wave * kWaveItems) + (u32)lane;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const u32 idx = w0 + (u32)(r * 64);
        const bool valid = idx < n;
        key[r] = valid ? keys_in[idx] : 0u;
        val[r] = valid ? (vals_in ? vals_in[idx] : idx) : 0u;
    }
    __syncthreads();                           // wcount cleared

    const unsigned long long lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    u32* const run = wcount[wave];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const bool valid = w0 + (u32)(r * 64) < n;
        const u32 d = (key[r] >> shift) & mask;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < bits; ++bit) {
            const unsigned long long b = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? b : ~b;
        }
        if (valid) {
            // every peer reads the running count, then writes the same new
            // value; the next round's reads come after this write in the
            // wave's program order
            const u32 before = run[d];
            rank[r] = before + (u32)__popcll(peers & lt_mask);
            run[d] = before + (u32)__popcll(peers);
        }
    }
    __syncthreads();

    // per digit: waves' counts -> exclusive prefixes; the tile's digit
    // counts -> exclusive scan (each thread owns dpt consecutive digits)
    const int dpt = digits > kSortThreads ? digits / kSortThreads : 1;
    const int d0 = tid * dpt;
    u32 cnt_own = 0;
    for (int k = 0; k < dpt; ++k) {
        const int d = d0 + k;
        if (d < digits) {
            u32 pre = 0;
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const u32 c = wcount[w][d];
                wcount[w][d] = pre;
                pre += c;
            }
            cnt_own += pre;
            dest_base[d] = pre;                // the digit's count, for now
        }
    }
    u32 total;
    u32 start = block_inclusive_scan(cnt_own, lds4, &total) - cnt_own;
    for (int k = 0; k < dpt; ++k) {
        const int d = d0 + k;
        if (d < digits) {
            const u32 c = dest_base[d];
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) wcount[w][d] += start;
            dest_base[d] = table[(size_t)blockIdx.x * digits + d] - start;
            start += c;
        }
    }
    __syncthreads();

#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (w0 + (u32)(r * 64) < n) {
            const u32 pos = run[(key[r] >> shift) & mask] + rank[r];
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();

    for (u32 j = (u32)tid; j < tile_n; j += kSortThreads) {
        const u32 k = s_keys[j];
        const u32 dest = dest_base[(k >> shift) & mask] + j;
        if (dest < n) {                        // always true for a consistent histogram
            keys_out[dest] = k;
            vals_out[dest] = s_vals[j];
        }
    }
}

// ---------------------------------------------------------------- bucket sort
//
// The dense single call's records arrive bucketed (see RecordSink): bucket k
// = (batch item b, region r) holds the A*P samples of region r in (anchor,
// keypoint) order -- which is their sample order -- keyed by local cell
// (the batched form: bucket k = the batch's region k, A_s*P samples).
// Every sample of a cell lies in one bucket, so sorting each bucket by key,
// stably, gives exactly the order of the global sort (each cell's records in
// sample order), in one launch and without leaving LDS.
//
// One workgroup of 1024 threads per bucket. Each element is the composite
// key << 15 | pos (pos = its place in the bucket), held in registers: wave w
// owns elements [w*64E, (w+1)*64E), E per lane. LSD passes over the key bits
// with digits of at most 8 bits; a pass ranks equal digits by wave ballots
// with per-wave running counts (as radix_scatter_kernel), turns the counts
// into places, writes each element to its place in an LDS buffer and reloads
// the registers from it in the new order. Then the sorted composites give
// vals (sample index from b, r and pos) and, by a binary search per cell,
// the cells' first positions.
constexpr int kBucketThreads = 1024;
constexpr int kBucketWaves = kBucketThreads / 64;
constexpr int kBucketPosBits = 15;

struct BucketSortArgs {
    const u32* keys;
    const int32_t* shapes;
    // the visible-view form: the exclusive scan of the visible flags over
    // the view-major items (b*N + n)*A + a, and the compacted item list
    const u32* place;
    const u32* items;
    u32* vals;
    u32* off;
    // the tiled reduction's tables, written by block 0 (as region_tables_kernel)
    u32* cell_start;
    u32* tile_start;
    u32* tile_region;
    int B, N, L, A, P;
    u32 ap;                     // A*P records per bucket (the visible-view form: at most)
    u32 cells_per_item;
};

// n / d for n < 2^15 and 1 <= d <= 2^15 as (n * m) >> k, with k = 15 +
// ceil(log2 d) and m = ceil(2^k / d): m < 2^16 + 1, so n * m fits 32 bits,
// and the error term stays below 1/d, so the quotient is exact.
struct Div15 {
    u32 m;
    int k;
    __device__ explicit Div15(u32 d) {
        int l = 0;
        while ((1u << l) < d) ++l;
        k = 15 + l;
        m = (u32)(((1ull << k) + d - 1) / d);
    }
    __device__ u32 operator()(u32 n) const { return (n * m) >> k; }
};

size_t bucket_sort_lds_bytes(u32 ap) {
    return ((size_t)ap + (size_t)kBucketWaves * kMaxDigits + kMaxDigits + 32) * 4;
}

// Exclusive scan of v over the 1024 threads of a bucket-sort block (wave
// sums in lds[0..15]); returns the thread's exclusive prefix and the total.
__device__ __forceinline__ u32 bucket_block_scan(u32 v, u32* lds, u32* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    u32 x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const u32 t = __shfl_up(x, d, 64);
        if (lane >= d) x += t;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    u32 before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBucketWaves; ++w) {
        const u32 t = lds[w];
        if (w < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// LDS of a bucket-sort block: [ap] composites, per-wave digit counts,
// digit starts, wave totals, block-scan scratch.
struct BucketLds {
    u32 *buf, *wcount, *dstart, *lds16, *lds_scan;
    __device__ BucketLds(u32* bsm, u32 ap_max) {
        buf = bsm;
        wcount = bsm + ap_max;
        dstart = wcount + kBucketWaves * kMaxDigits;
        lds16 = dstart + kMaxDigits;
        lds_scan = lds16 + 16;
    }
};

// Sorts one bucket of ap <= 64*E*16 records by key (keys[j] < nkeys, larger
// keys clamped to nkeys - 1), stably: leaves the composites key << 15 | j in
// key order in m.buf[0, ap).
template <int E>
__device__ __forceinline__ void bucket_sort_core(const u32* __restrict__ keys, u32 ap, u32 nkeys,
                                                 const BucketLds& m) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int kb = 1;
    while (kb < 32 && ((nkeys - 1) >> kb) != 0) ++kb;
    const int passes = (kb + kMaxDigitBits - 1) / kMaxDigitBits;
    const int bits = (kb + passes - 1) / passes;
    const int digits = 1 << bits;
    const u32 mask = (u32)digits - 1u;

    u32 v[E], rank[E];
    const u32 j0 = (u32)(wave * 64 * E + lane);
#pragma unroll
    for (int e = 0; e < E; ++e) {                          // every load in flight at once
        const u32 j = j0 + (u32)(e * 64);
        v[e] = j < ap ? (min(keys[j], nkeys - 1u) << kBucketPosBits) | j : 0u;
    }
    const unsigned long long lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    u32* const run = m.wcount + wave * kMaxDigits;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = kBucketPosBits + pass * bits;
        for (int i = tid; i < kBucketWaves * digits; i += kBucketThreads)
            m.wcount[(i >> bits) * kMaxDigits + (i & (digits - 1))] = 0u;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool valid = j0 + (u32)(e * 64) < ap;
            const u32 d = (v[e] >> shift) & mask;
            unsigned long long peers = __ballot(valid);
            for (int bit = 0; bit < bits; ++bit) {
                const unsigned long long bb = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? bb : ~bb;
            }
            if (valid) {
                // every peer reads the running count, then writes the same
                // new value; the next element's reads follow in program order
                const u32 before = run[d];
                rank[e] = before + (u32)__popcll(peers & lt_mask);
                run[d] = before + (u32)__popcll(peers);
            }
        }
        __syncthreads();
        // per digit: the waves' counts -> exclusive prefixes in wave order,
        // plus the digit's start (exclusive scan of the digit totals)
        u32 cnt = 0;
        if (tid < digits) {
#pragma unroll
            for (int w = 0; w < kBucketWaves; ++w) {
                const u32 c = m.wcount[w * kMaxDigits + tid];
                m.wcount[w * kMaxDigits + tid] = cnt;
                cnt += c;
            }
        }
        // scan of cnt over the first `digits` threads (at most 4 waves)
        u32 x = cnt;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const u32 t = __shfl_up(x, dd, 64);
            if (lane >= dd) x += t;
        }
        if (lane == 63 && wave < 4) m.lds16[wave] = x;
        __syncthreads();
        if (tid < digits) {
            u32 before = 0;
            for (int w = 0; w < wave; ++w) before += m.lds16[w];
            m.dstart[tid] = before + x - cnt;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (j0 + (u32)(e * 64) < ap) {
                const u32 d = (v[e] >> shift) & mask;
                m.buf[m.dstart[d] + m.wcount[wave * kMaxDigits + d] + rank[e]] = v[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const u32 j = j0 + (u32)(e * 64);
            if (j < ap) v[e] = m.buf[j];
        }
        // the next pass clears wcount only after this barrier: every wave
        // has read its places
        __syncthreads();
    }
}

// The first position of each of a bucket's nkeys local cells from its
// sorted composites: off[c] = base + the first position whose key is >= c
// (ap after the last key). off: the bucket's first cell; base: its first
// record. Two ways to the same table:
//  - by record (the dense forms, whose buckets hold every anchor's samples
//    of a region): element i writes the cells in (key[i-1], key[i]] (from
//    0 for the first, up to the last cell for i = ap);
//  - by cell (the visible-view form, whose buckets are sparse and clustered
//    where the walk above would leave a few threads long runs of empty
//    cells: its sort took 123 instead of 43 us): each thread takes a
//    contiguous run of cells, binary-searches the first, then advances a
//    pointer over the records, switching to a binary search over the rest
//    when a cell lies more than 16 records further on.
// (Measured on the 64-camera scene: by record 42 us, by cell 49 us.)
__device__ __forceinline__ u32 first_key_at_least(const u32* buf, u32 lo, u32 hi, u32 c) {
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if ((buf[mid] >> kBucketPosBits) < c) lo = mid + 1u; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void bucket_cell_starts(const u32* buf, u32 ap, u32 nkeys, u32 base,
                                                   u32* __restrict__ off, bool by_cell) {
    if (!by_cell) {
        for (u32 i = (u32)threadIdx.x; i <= ap; i += kBucketThreads) {
            const u32 c1 = i < ap ? buf[i] >> kBucketPosBits : nkeys - 1u;
            const u32 c0 = i == 0 ? 0u : (buf[i - 1] >> kBucketPosBits) + 1u;
            for (u32 c = c0; c <= c1; ++c) off[c] = base + i;
        }
        return;
    }
    const u32 per = (nkeys + kBucketThreads - 1) / kBucketThreads;
    const u32 c_lo = (u32)threadIdx.x * per;
    const u32 c_hi = min(c_lo + per, nkeys);
    if (c_lo >= c_hi) return;
    u32 ptr = first_key_at_least(buf, 0u, ap, c_lo);
    off[c_lo] = base + ptr;
    for (u32 c = c_lo + 1; c < c_hi; ++c) {
        int steps = 0;
        while (ptr < ap && (buf[ptr] >> kBucketPosBits) < c && steps < 16) {
            ++ptr;
            ++steps;
        }
        if (ptr < ap && (buf[ptr] >> kBucketPosBits) < c)
            ptr = first_key_at_least(buf, ptr, ap, c);
        off[c] = base + ptr;
    }
}

template <int E>
__global__ void __launch_bounds__(kBucketThreads) bucket_sort_kernel(BucketSortArgs p) {
    extern __shared__ __align__(16) u32 bsm[];
    const BucketLds m(bsm, p.ap);
    const int tid = threadIdx.x;
    const u32 k = blockIdx.x;
    const int NL = p.N * p.L;
    const int b = (int)(k / (u32)NL), r = (int)(k % (u32)NL);

    // The region tables (NL <= 1024: one region per thread): the first cell
    // of every region ((H+1)(W+1) bilinear cells and the outside cell each)
    // -- this block's own, and block 0 writes them all -- and, over the
    // processing slots (coarse levels first: slot o -> region
    // (o % N) * L + (L - 1 - o / N)), the first tile and region of each slot.
    {
        u32 cells = 0, tiles = 0;
        int rs = 0;
        if (tid < NL) {
            cells = (u32)(p.shapes[2 * tid] + 1) * (u32)(p.shapes[2 * tid + 1] + 1) + 1u;
            rs = (tid % p.N) * p.L + (p.L - 1 - tid / p.N);
            tiles = ((u32)(p.shapes[2 * rs] + kTileH - 1) / kTileH) *
                    ((u32)(p.shapes[2 * rs + 1] + kTileW - 1) / kTileW);
        }
        u32 tc, tt;
        const u32 cs = bucket_block_scan(cells, m.lds_scan, &tc);
        const u32 ts = bucket_block_scan(tiles, m.lds_scan, &tt);
        if (tid == r) m.dstart[0] = cs;                    // this bucket's region
        if (k == 0 && tid < NL) {
            p.cell_start[tid] = cs;
            p.tile_start[tid] = ts;
            p.tile_region[tid] = (u32)rs;
            if (tid == NL - 1) p.tile_start[NL] = tt;
        }
        __syncthreads();
    }
    const u32 cstart = m.dstart[0];
    __syncthreads();                                       // dstart is reused below
    const u32 H = (u32)p.shapes[2 * r], W = (u32)p.shapes[2 * r + 1];
    const u32 nkeys = (H + 1) * (W + 1) + 1;               // local keys, the outside cell last
    const u32 n_ = (u32)p.N, L_ = (u32)p.L, A_ = (u32)p.A, P_ = (u32)p.P;
    const u32 nr = (u32)r / L_, lr = (u32)r % L_;
    const u32 bn = (u32)b * n_ + nr;
    // the bucket: dense, A*P records at k*A*P; visible-view, the cnt visible
    // anchors of (b, camera nr) from item s0 on, their P*L records per item
    // level-major from s0*P*L, so this level's cnt*P at s0*P*L + lr*cnt*P
    u32 ap = p.ap, base = k * p.ap, s0 = 0u;
    if (p.place) {
        s0 = p.place[(size_t)bn * A_];
        ap = (p.place[(size_t)(bn + 1) * A_] - s0) * P_;
        base = s0 * P_ * L_ + lr * ap;
    }
    if (ap > 0) bucket_sort_core<E>(p.keys + base, ap, nkeys, m);

    // outputs: m.buf holds the bucket's composites in key order
    u32* vals = p.vals + base;
    const Div15 by_p(P_);
    for (u32 i = (u32)tid; i < ap; i += kBucketThreads) {
        const u32 pos = m.buf[i] & ((1u << kBucketPosBits) - 1u);
        const u32 q = by_p(pos), pp = pos - q * P_;
        // the anchor: the q-th of the bucket (dense) or of the item list
        const u32 a = p.place ? p.items[s0 + q] - bn * A_ : q;
        // sample index of (b, a, pp, nr, lr)
        vals[i] = ((((u32)b * A_ + a) * P_ + pp) * n_ + nr) * L_ + lr;
    }
    bucket_cell_starts(m.buf, ap, nkeys, base, p.off + (size_t)b * p.cells_per_item + cstart,
                       p.place != nullptr);
    if (k + 1 == gridDim.x && tid == 0)
        p.off[(size_t)p.B * p.cells_per_item] =
            p.place ? p.place[(size_t)p.B * n_ * A_] * P_ * L_ : (u32)gridDim.x * p.ap;
}

// The batched form: bucket k = the batch's region k, scene s (the last with
// region_start[s] <= k), region r = k - region_start[s] = n*L + l of it,
// holding the scene's A_s*P samples of that region in (anchor, keypoint)
// order at sample_start[s] + r*A_s*P. Buckets, and the cells of the batch
// tables, follow the regions in order, so the per-bucket results form the
// global sorted order and off[] of the whole batch.
template <int E>
__global__ void __launch_bounds__(kBucketThreads) bucket_sort_batched_kernel(BatchArgs b,
                                                                             u32 ap_max,
                                                                             u32* __restrict__ vals,
                                                                             u32* __restrict__ off) {
    extern __shared__ __align__(16) u32 bsm[];
    const BucketLds m(bsm, ap_max);
    const u32 k = blockIdx.x;
    const int s = scene_of(b.t.region_start, b.S, k);
    const msda_scene& sc = b.scenes[s];
    const u32 r = k - b.t.region_start[s];
    const u32 N = (u32)sc.num_cams, L = (u32)b.L, P = (u32)b.P;
    const u32 ap = (u32)sc.num_anchors * P;
    const u32 base = b.t.sample_start[s] + r * ap;
    const u32 H = (u32)sc.spatial_shapes[2 * r], W = (u32)sc.spatial_shapes[2 * r + 1];
    const u32 nkeys = (H + 1) * (W + 1) + 1;               // local keys, the outside cell last
    if (ap > 0) bucket_sort_core<E>(b.rec_key + base, ap, nkeys, m);

    const u32 nr = r / L, lr = r % L;
    const Div15 by_p(P);
    for (u32 i = (u32)threadIdx.x; i < ap; i += kBucketThreads) {
        const u32 pos = m.buf[i] & ((1u << kBucketPosBits) - 1u);
        const u32 a = by_p(pos), pp = pos - a * P;
        vals[base + i] = b.t.sample_start[s] + ((a * P + pp) * N + nr) * L + lr;
    }
    bucket_cell_starts(m.buf, ap, nkeys, base, off + b.t.cell_start[k], false);
    if (k + 1 == gridDim.x && threadIdx.x == 0) off[b.total_cells] = b.total_samples;
}

hipError_t launch_bucket_sort(const u32* keys, const int32_t* shapes, int32_t B, int32_t N,
                              int32_t L, int32_t A, int32_t P, u32 cells_per_item, u32* vals,
                              u32* off, u32* cell_start, u32* tile_start, u32* tile_region,
                              const u32* place, const u32* items, hipStream_t s) {
    BucketSortArgs p;
    p.keys = keys;
    p.shapes = shapes;
    p.place = place;
    p.items = items;
    p.cell_start = cell_start;
    p.tile_start = tile_start;
    p.tile_region = tile_region;
    p.vals = vals;
    p.off = off;
    p.B = B;
    p.N = N;
    p.L = L;
    p.A = A;
    p.P = P;
    p.ap = (u32)A * (u32)P;
    p.cells_per_item = cells_per_item;
    const unsigned grid = (unsigned)(B * N * L);
    if (grid == 0 || p.ap == 0) return hipSuccess;
    const size_t lds = bucket_sort_lds_bytes(p.ap);
    const u32 per_lane = (p.ap + kBucketThreads - 1) / kBucketThreads;
    mark_begin("bucket_sort", s);
    if (per_lane <= 4)
        hipLaunchKernelGGL(bucket_sort_kernel<4>, dim3(grid), dim3(kBucketThreads), lds, s, p);
    else if (per_lane <= 8)
        hipLaunchKernelGGL(bucket_sort_kernel<8>, dim3(grid), dim3(kBucketThreads), lds, s, p);
    else if (per_lane <= 16)
        hipLaunchKernelGGL(bucket_sort_kernel<16>, dim3(grid), dim3(kBucketThreads), lds, s, p);
    else if (per_lane <= 32)
        hipLaunchKernelGGL(bucket_sort_kernel<32>, dim3(grid), dim3(kBucketThreads), lds, s, p);
    else {
        mark_end(s);
        return hipErrorInvalidValue;               // ap > kBucketMaxRecords: the caller's check
    }
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_bucket_sort_batched(const BatchArgs& b, u32 max_ap, u32* vals, u32* off,
                                      hipStream_t s) {
    const unsigned grid = b.total_regions;
    if (grid == 0) return hipSuccess;
    const size_t lds = bucket_sort_lds_bytes(max_ap);
    const u32 per_lane = (max_ap + kBucketThreads - 1) / kBucketThreads;
    mark_begin("bucket_sort_batched", s);
    if (per_lane <= 4)
        hipLaunchKernelGGL(bucket_sort_batched_kernel<4>, dim3(grid), dim3(kBucketThreads), lds,
                           s, b, max_ap, vals, off);
    else if (per_lane <= 8)
        hipLaunchKernelGGL(bucket_sort_batched_kernel<8>, dim3(grid), dim3(kBucketThreads), lds,
                           s, b, max_ap, vals, off);
    else if (per_lane <= 16)
        hipLaunchKernelGGL(bucket_sort_batched_kernel<16>, dim3(grid), dim3(kBucketThreads), lds,
                           s, b, max_ap, vals, off);
    else if (per_lane <= 32)
        hipLaunchKernelGGL(bucket_sort_batched_kernel<32>, dim3(grid), dim3(kBucketThreads), lds,
                           s, b, max_ap, vals, off);
    else {
        mark_end(s);
        return hipErrorInvalidValue;               // max_ap > kBucketMaxRecords: the caller's check
    }
    mark_end(s);
    return hipGetLastError();
}

// off[r] = first position whose key is >= r, for r in [0, nrows]; keys are
// sorted and every key is <= nrows.
__global__ void segment_bounds_kernel(const u32* __restrict__ keys, u32 n, const u32* n_dev,
                                      u32 nrows, u32* __restrict__ off) {
    if (n_dev) n = min(n, *n_dev);
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const u32 lo = i == 0 ? 0u : min(keys[i - 1], nrows) + 1u;
    const u32 hi = i == n ? nrows : min(keys[i], nrows);
    for (u32 r = lo; r <= hi; ++r) off[r] = i;
}

// The same bounds by a binary search per cell: used when n is a device
// count (the visible-view form), where the records cover few cells and the
// per-record form would leave a thread to fill a long run of empty cells.
__global__ void segment_bounds_search_kernel(const u32* __restrict__ keys, u32 n,
                                             const u32* n_dev, u32 nrows,
                                             u32* __restrict__ off) {
    const u32 r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > nrows) return;
    if (n_dev) n = min(n, *n_dev);
    u32 lo = 0, hi = n;                       // first position with key >= r
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (keys[mid] < r) lo = mid + 1; else hi = mid;
    }
    off[r] = lo;
}

hipError_t launch_exclusive_scan(u32* x, u32 n, u32* partial, hipStream_t s) {
    const u32 tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 0) return hipSuccess;
    mark_begin("scan_reduce", s);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(tiles), dim3(256), 0, s, x, n, partial);
    mark_end(s);
    mark_begin("scan_partials", s);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(256), 0, s, partial, tiles);
    mark_end(s);
    mark_begin("scan_apply", s);
    hipLaunchKernelGGL(scan_apply_kernel, dim3(tiles), dim3(256), 0, s, x, n, partial);
    mark_end(s);
    return hipGetLastError();
}

size_t scan_scratch_words(u32 n) { return (n + kScanTile - 1) / kScanTile + 1; }

static u32 bands_of(u32 ntiles) { return (ntiles + kBand - 1) / kBand; }

size_t sort_scratch_words(u32 n) {
    const u32 ntiles = (n + kSortTile - 1) / kSortTile;
    return (size_t)kMaxDigits * ntiles + (size_t)kMaxDigits * bands_of(ntiles);
}

// Passes and digit width for keys in [0, max_key]: the fewest passes of at
// most kMaxDigitBits bits, the bits shared evenly.
static void sort_plan(u32 max_key, int* passes, int* bits) {
    int kb = 0;
    while (kb < 32 && (max_key >> kb) != 0) ++kb;
    if (kb == 0) kb = 1;
    *passes = (kb + kMaxDigitBits - 1) / kMaxDigitBits;
    *bits = (kb + *passes - 1) / *passes;
}

int sort_passes(u32 max_key) {
    int passes, bits;
    sort_plan(max_key, &passes, &bits);
    return passes;
}

hipError_t launch_sort_records(u32* keys_a, u32* keys_b, u32* vals_a, u32* vals_b, u32 n,
                               u32 nrows, u32* scratch, u32* off, u32** sorted_vals,
                               hipStream_t s, const u32* n_dev, bool vals_given) {
    hipError_t e = hipSuccess;
    const u32 ntiles = (n + kSortTile - 1) / kSortTile;
    const u32 nbands = bands_of(ntiles);
    u32* table = scratch;
    u32* band_sum = scratch + (size_t)kMaxDigits * ntiles;
    u32* kin = keys_a;
    u32* kout = keys_b;
    // first pass: values are the indices, or the caller's (in vals_a)
    u32* vin = vals_given ? vals_a : nullptr;
    u32* vout = vals_given ? vals_b : vals_a;
    int passes, bits;
    sort_plan(nrows, &passes, &bits);
    for (int p = 0; p < passes && n > 0; ++p) {
        const int shift = bits * p;
        mark_begin("radix_hist", s);
        hipLaunchKernelGGL(radix_hist_kernel, dim3(ntiles), dim3(kSortThreads), 0, s, kin, n,
                           n_dev, shift, bits, table, ntiles);
        mark_end(s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        mark_begin("digit_band", s);
        hipLaunchKernelGGL(digit_band_kernel, dim3(nbands), dim3(kMaxDigits), 0, s, table, ntiles,
                           1 << bits, band_sum);
        mark_end(s);
        mark_begin("digit_offsets", s);
        hipLaunchKernelGGL(digit_offsets_kernel, dim3(nbands), dim3(kMaxDigits), 0, s, table,
                           ntiles, 1 << bits, band_sum, nbands);
        mark_end(s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        mark_begin("radix_scatter", s);
        switch (bits) {
#define MSDA_SCATTER_BITS(B)                                                                   \
    case B:                                                                                    \
        hipLaunchKernelGGL(radix_scatter_kernel<B>, dim3(ntiles), dim3(kSortThreads), 0, s, kin, \
                           vin, kout, vout, n, n_dev, shift, table);                           \
        break;
            MSDA_SCATTER_BITS(1) MSDA_SCATTER_BITS(2) MSDA_SCATTER_BITS(3) MSDA_SCATTER_BITS(4)
            MSDA_SCATTER_BITS(5) MSDA_SCATTER_BITS(6) MSDA_SCATTER_BITS(7) MSDA_SCATTER_BITS(8)
#undef MSDA_SCATTER_BITS
            default: return hipErrorInvalidValue;    // sort_plan keeps bits in [1, 8]
        }
        mark_end(s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // next pass reads what this one wrote
        u32* t = kin; kin = kout; kout = t;
        vin = vout;
        vout = (vin == vals_a) ? vals_b : vals_a;
    }
    *sorted_vals = vin;      // nullptr when n == 0 and no values were given
    mark_begin("segment_bounds", s);
    if (n_dev)
        hipLaunchKernelGGL(segment_bounds_search_kernel, dim3((nrows + 1 + 255) / 256), dim3(256),
                           0, s, kin, n, n_dev, nrows, off);
    else
        hipLaunchKernelGGL(segment_bounds_kernel, dim3((n + 1 + 255) / 256), dim3(256), 0, s, kin,
                           n, n_dev, nrows, off);
    mark_end(s);
    return hipGetLastError();
}

}  // namespace msda
