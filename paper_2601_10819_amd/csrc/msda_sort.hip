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
// The key bits are split into as few passes as digits of at most 10 bits
// allow (a 20-bit key space, about a million cells, takes two). Each pass:
// a per-tile digit histogram, an exclusive scan of the histograms in
// digit-major order, then a stable scatter where a tile ranks equal digits
// by wave ballots (lanes in order), then waves in order, then rounds in
// order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // elements per tile
constexpr int kMaxDigitBits = 10;
constexpr int kMaxDigits = 1 << kMaxDigitBits;
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
#pragma unroll 4
    for (int i = 0; i < kSortItems; ++i) {
        const u32 idx = base + i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < digits; d += kSortThreads)
        table[(size_t)d * ntiles + blockIdx.x] = h[d];      // digit-major
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
// nullptr means the value is the element's index (first pass). Per round of
// 256 elements: lanes of a wave with equal digits are found with one ballot
// per digit bit and ranked by lane; the first lane of each such group
// publishes the group size for its wave, so a lane's place is the tile's
// offset for the digit + the digit's count in earlier rounds + the groups
// of earlier waves + its rank. Only the entries a round sets are cleared.
__global__ void __launch_bounds__(kSortThreads)
radix_scatter_kernel(const u32* __restrict__ keys_in, const u32* __restrict__ vals_in,
                     u32* __restrict__ keys_out, u32* __restrict__ vals_out, u32 n,
                     const u32* n_dev, int shift, int bits, const u32* __restrict__ table,
                     u32 ntiles) {
    __shared__ u32 base_off[kMaxDigits];
    __shared__ u32 running[kMaxDigits];
    __shared__ u32 wcount[kSortThreads / 64][kMaxDigits];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int digits = 1 << bits;
    const u32 mask = (u32)digits - 1u;
    if (n_dev) n = min(n, *n_dev);
    for (int d = tid; d < digits; d += kSortThreads) {
        base_off[d] = table[(size_t)d * ntiles + blockIdx.x];
        running[d] = 0;
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; ++w) wcount[w][d] = 0;
    }
    __syncthreads();
    const u64 lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortItems; ++r) {
        const u32 idx = blockIdx.x * (u32)kSortTile + r * kSortThreads + tid;
        const bool valid = idx < n;
        const u32 key = valid ? keys_in[idx] : 0u;
        const u32 val = valid ? (vals_in ? vals_in[idx] : idx) : 0u;
        const u32 d = (key >> shift) & mask;
        // lanes of this wave holding the same digit
        u64 peers = __ballot(valid);
        for (int bit = 0; bit < bits; ++bit) {
            const u64 b = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? b : ~b;
        }
        const u32 rank = __popcll(peers & lt_mask);
        const u32 count = __popcll(peers);
        const bool leader = valid && rank == 0;
        if (leader) wcount[wave][d] = count;
        __syncthreads();
        if (valid) {
            u32 before = 0;
            for (int w = 0; w < wave; ++w) before += wcount[w][d];
            const u32 dest = base_off[d] + running[d] + before + rank;
            if (dest < n) {            // always true for a consistent histogram
                keys_out[dest] = key;
                vals_out[dest] = val;
            }
        }
        __syncthreads();
        if (leader) {
            atomicAdd(&running[d], count);   // integer: the order of the adds does not matter
            wcount[wave][d] = 0;
        }
        __syncthreads();
    }
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

size_t sort_scratch_words(u32 n) {
    const u32 ntiles = (n + kSortTile - 1) / kSortTile;
    const size_t table = (size_t)kMaxDigits * ntiles;
    const size_t partial = (table + kScanTile - 1) / kScanTile + 1;
    return table + partial;
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
    u32* table = scratch;
    u32* partial = scratch + (size_t)kMaxDigits * ntiles;
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
        if ((e = launch_exclusive_scan(table, (u32)(ntiles << bits), partial, s)) != hipSuccess)
            return e;
        mark_begin("radix_scatter", s);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(ntiles), dim3(kSortThreads), 0, s, kin, vin,
                           kout, vout, n, n_dev, shift, bits, table, ntiles);
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
