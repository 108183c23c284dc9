// Stable LSD radix sort of (key, value) u32 pairs and segment boundaries,
// the grouping step of the deterministic grad_feat reduction.
//
// The backward kernel writes one record per (sample, corner) at position
// 4*sample + corner: key = the feature row the corner touches (or the number
// of rows, a sentinel that sorts last, for a corner outside its level). A
// stable sort by key leaves each row's records contiguous and in sample
// order, so the per-row reduction that follows sums them in a fixed order:
// grad_feat is bitwise reproducible, and no float atomics are needed.
//
// Each pass sorts by 8 key bits: a per-tile digit histogram, an exclusive
// scan of the histograms in digit-major order, then a stable scatter where a
// tile ranks equal digits by wave ballots (lanes in order), then waves in
// order, then rounds in order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // elements per tile
constexpr int kDigits = 256;
constexpr int kScanTile = 4096;                          // scan: 256 threads x 16

__global__ void __launch_bounds__(kSortThreads)
radix_hist_kernel(const u32* __restrict__ keys, u32 n, int shift, u32* __restrict__ table,
                  u32 ntiles) {
    __shared__ u32 h[kDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const u32 base = blockIdx.x * (u32)kSortTile;
#pragma unroll 4
    for (int i = 0; i < kSortItems; ++i) {
        const u32 idx = base + i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (kDigits - 1)], 1u);
    }
    __syncthreads();
    table[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];   // digit-major
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

// Stable scatter of one tile by the digit at `shift`. vals_in == nullptr
// means the value is the element's index (first pass).
__global__ void __launch_bounds__(kSortThreads)
radix_scatter_kernel(const u32* __restrict__ keys_in, const u32* __restrict__ vals_in,
                     u32* __restrict__ keys_out, u32* __restrict__ vals_out, u32 n, int shift,
                     const u32* __restrict__ table, u32 ntiles) {
    __shared__ u32 base_off[kDigits];
    __shared__ u32 running[kDigits];
    __shared__ u32 wcount[4][kDigits];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base_off[tid] = table[(size_t)tid * ntiles + blockIdx.x];
    running[tid] = 0;
    const u64 lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortItems; ++r) {
        const u32 idx = blockIdx.x * (u32)kSortTile + r * kSortThreads + tid;
        const bool valid = idx < n;
        const u32 key = valid ? keys_in[idx] : 0u;
        const u32 val = valid ? (vals_in ? vals_in[idx] : idx) : 0u;
        const u32 d = (key >> shift) & (kDigits - 1);
        // lanes of this wave holding the same digit
        u64 peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const u64 b = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? b : ~b;
        }
        const u32 rank = __popcll(peers & lt_mask);
        for (int k = tid; k < 4 * kDigits; k += kSortThreads) (&wcount[0][0])[k] = 0;
        __syncthreads();
        if (valid && rank == 0) wcount[wave][d] = __popcll(peers);
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
        running[tid] += wcount[0][tid] + wcount[1][tid] + wcount[2][tid] + wcount[3][tid];
        __syncthreads();
    }
}

// off[r] = first position whose key is >= r, for r in [0, nrows]; keys are
// sorted and every key is <= nrows.
__global__ void segment_bounds_kernel(const u32* __restrict__ keys, u32 n, u32 nrows,
                                      u32* __restrict__ off) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const u32 lo = i == 0 ? 0u : min(keys[i - 1], nrows) + 1u;
    const u32 hi = i == n ? nrows : min(keys[i], nrows);
    for (u32 r = lo; r <= hi; ++r) off[r] = i;
}

static hipError_t launch_scan(u32* x, u32 n, u32* partial, hipStream_t s) {
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

size_t sort_scratch_words(u32 n) {
    const u32 ntiles = (n + kSortTile - 1) / kSortTile;
    const size_t table = (size_t)kDigits * ntiles;
    const size_t partial = (table + kScanTile - 1) / kScanTile + 1;
    return table + partial;
}

int sort_passes(u32 max_key) {
    int bits = 0;
    while (bits < 32 && (max_key >> bits) != 0) ++bits;
    return bits == 0 ? 1 : (bits + 7) / 8;
}

hipError_t launch_sort_records(u32* keys_a, u32* keys_b, u32* vals_a, u32* vals_b, u32 n,
                               u32 nrows, u32* scratch, u32* off, u32** sorted_vals,
                               hipStream_t s) {
    hipError_t e = hipSuccess;
    const u32 ntiles = (n + kSortTile - 1) / kSortTile;
    u32* table = scratch;
    u32* partial = scratch + (size_t)kDigits * ntiles;
    u32* kin = keys_a;
    u32* kout = keys_b;
    u32* vin = nullptr;       // first pass: values are the indices
    u32* vout = vals_a;
    const int passes = sort_passes(nrows);
    for (int p = 0; p < passes && n > 0; ++p) {
        const int shift = 8 * p;
        mark_begin("radix_hist", s);
        hipLaunchKernelGGL(radix_hist_kernel, dim3(ntiles), dim3(kSortThreads), 0, s, kin, n,
                           shift, table, ntiles);
        mark_end(s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_scan(table, kDigits * ntiles, partial, s)) != hipSuccess) return e;
        mark_begin("radix_scatter", s);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(ntiles), dim3(kSortThreads), 0, s, kin, vin,
                           kout, vout, n, shift, table, ntiles);
        mark_end(s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // next pass reads what this one wrote
        u32* t = kin; kin = kout; kout = t;
        vin = vout;
        vout = (vout == vals_a) ? vals_b : vals_a;
    }
    *sorted_vals = vin;      // nullptr when n == 0
    mark_begin("segment_bounds", s);
    hipLaunchKernelGGL(segment_bounds_kernel, dim3((n + 1 + 255) / 256), dim3(256), 0, s, kin, n,
                       nrows, off);
    mark_end(s);
    return hipGetLastError();
}

}  // namespace msda
