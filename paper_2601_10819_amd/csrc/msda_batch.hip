// Tables of the batched form, built on the device from the scene table so
// that a batched call needs no host-to-device copy (and can be captured in
// a HIP graph): per scene the first anchor, sample (record) and region; per
// region its first bilinear cell; and the processing slots of the tiled
// grad_feat reduction -- heavy (coarse) levels first, then coarsest level
// first, then scene, then camera -- with the first tile of each slot.
//
// A (scene, level) is heavy when the level's area (camera 0) is at most
// 1/16 of the scene's largest level area: there a pixel collects 16x or
// more the samples of the finest level. The host computes the same split
// from its mirrors to size the two tile launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

// Heavy flag of (scene s, level l) from the LDS copy of the shapes.
__device__ __forceinline__ bool level_is_heavy(const uint16_t* sh_h, const uint16_t* sh_w,
                                               const u32* rstart, int s, int l, int L) {
    const u32 r0 = rstart[s];                      // camera 0's regions: r0 + l
    u32 max_area = 0;
    for (int k = 0; k < L; ++k) max_area = max(max_area, (u32)sh_h[r0 + k] * (u32)sh_w[r0 + k]);
    return (u32)sh_h[r0 + l] * (u32)sh_w[r0 + l] * 16u <= max_area;
}

__global__ void __launch_bounds__(256) batch_tables_kernel(BatchArgs b, int backward) {
    __shared__ u32 s_anchors[kMaxBatchScenes];
    __shared__ u32 s_cams[kMaxBatchScenes];
    __shared__ u32 rstart[kMaxBatchScenes + 1];
    __shared__ uint16_t sh_h[kMaxBatchRegions];
    __shared__ uint16_t sh_w[kMaxBatchRegions];
    __shared__ u32 grp[2 * 8 * kMaxBatchScenes];    // first slot of (class, level, scene)
    __shared__ u32 tiles[kMaxBatchRegions];         // tiles of each slot, then their scan
    __shared__ u32 lds4[4];
    const int S = b.S, L = b.L, tid = threadIdx.x;

    for (int s = tid; s < S; s += blockDim.x) {
        s_anchors[s] = (u32)b.scenes[s].num_anchors;
        s_cams[s] = (u32)b.scenes[s].num_cams;
    }
    __syncthreads();
    if (tid == 0) {
        u32 a = 0, smp = 0, reg = 0;
        for (int s = 0; s < S; ++s) {
            b.t.anchor_start[s] = a;
            b.t.sample_start[s] = smp;
            b.t.region_start[s] = reg;
            rstart[s] = reg;
            a += s_anchors[s];
            const u32 per_anchor = (u32)b.P * s_cams[s] * (u32)L;
            smp += s_anchors[s] * per_anchor;
            reg += s_cams[s] * (u32)L;
            // s / per_anchor for s < 2^30 as (s * m) >> k, m = ceil(2^k / d)
            int lg = 0;
            while ((1u << lg) < per_anchor) ++lg;
            const int k = 32 + lg;
            b.t.magic[s] = ((1ull << k) + per_anchor - 1) / per_anchor;
            b.t.magic_shift[s] = (u32)k;
        }
        b.t.anchor_start[S] = a;
        b.t.sample_start[S] = smp;
        b.t.region_start[S] = reg;
        rstart[S] = reg;
    }
    __syncthreads();
    if (!backward) return;

    const u32 R = rstart[S];
    // (H, W) of every region
    for (u32 g = tid; g < R; g += blockDim.x) {
        int lo = 0, hi = S - 1;                    // last scene with rstart <= g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rstart[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const u32 i = g - rstart[lo];
        sh_h[g] = (uint16_t)b.scenes[lo].spatial_shapes[2 * i];
        sh_w[g] = (uint16_t)b.scenes[lo].spatial_shapes[2 * i + 1];
    }
    __syncthreads();

    // first cell of every region: exclusive scan of (H+1)(W+1) + 1 (the
    // bilinear cells and the region's outside cell), regions in order
    {
        const u32 per = (R + blockDim.x - 1) / blockDim.x;
        const u32 g0 = tid * per;
        u32 sum = 0;
        for (u32 k = 0; k < per; ++k)
            if (g0 + k < R) sum += ((u32)sh_h[g0 + k] + 1u) * ((u32)sh_w[g0 + k] + 1u) + 1u;
        u32 total;
        u32 run = block_inclusive_scan(sum, lds4, &total) - sum;
        for (u32 k = 0; k < per; ++k) {
            if (g0 + k < R) {
                b.t.cell_start[g0 + k] = run;
                run += ((u32)sh_h[g0 + k] + 1u) * ((u32)sh_w[g0 + k] + 1u) + 1u;
            }
        }
    }

    // slot groups: (class, level descending, scene), each holding the scene's cameras
    if (tid == 0) {
        u32 run = 0;
        for (int cls = 0; cls < 2; ++cls)
            for (int ld = 0; ld < L; ++ld)
                for (int s = 0; s < S; ++s) {
                    const int l = L - 1 - ld;
                    const bool heavy = level_is_heavy(sh_h, sh_w, rstart, s, l, L);
                    grp[(cls * L + ld) * S + s] = run;
                    if (heavy == (cls == 0)) run += s_cams[s];
                }
    }
    __syncthreads();
    for (u32 g = tid; g < R; g += blockDim.x) {
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rstart[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const int s = lo;
        const u32 i = g - rstart[s];
        const int n = (int)(i / (u32)L), l = (int)(i % (u32)L);
        const int cls = level_is_heavy(sh_h, sh_w, rstart, s, l, L) ? 0 : 1;
        const u32 slot = grp[(cls * L + (L - 1 - l)) * S + s] + (u32)n;
        b.t.slot_scene[slot] = (u32)s;
        b.t.slot_region[slot] = i;
        tiles[slot] = (((u32)sh_h[g] + kTileH - 1) / kTileH) * (((u32)sh_w[g] + kTileW - 1) / kTileW);
    }
    __syncthreads();
    // first tile of every slot
    {
        const u32 per = (R + blockDim.x - 1) / blockDim.x;
        const u32 g0 = tid * per;
        u32 sum = 0;
        for (u32 k = 0; k < per; ++k)
            if (g0 + k < R) sum += tiles[g0 + k];
        u32 total;
        u32 run = block_inclusive_scan(sum, lds4, &total) - sum;
        for (u32 k = 0; k < per; ++k) {
            if (g0 + k < R) {
                b.t.tile_start[g0 + k] = run;
                run += tiles[g0 + k];
            }
        }
        if (tid == 0) b.t.tile_start[R] = total;
    }
}

hipError_t launch_batch_tables(const BatchArgs& b, bool backward, hipStream_t s) {
    mark_begin("batch_tables", s);
    hipLaunchKernelGGL(batch_tables_kernel, dim3(1), dim3(256), 0, s, b, backward ? 1 : 0);
    mark_end(s);
    return hipGetLastError();
}

}  // namespace msda
