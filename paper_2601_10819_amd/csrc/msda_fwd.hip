// Forward kernel of multi-scale deformable aggregation (paper Sec. 3.1 /
// Sec. 3.2): out[b,a,:] = sum over (keypoint, camera, level) of weight *
// bilinear sample. One workgroup per (batch item, anchor); its waves split
// the anchor's (keypoint, camera) pairs, each wave staging a chunk of
// locations and weights in LDS, and the waves' partial sums are added in a
// fixed order at the end (the forward is deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

int max_pairs_per_chunk(int L, int G) {
    int j = (kStageWords * 64) / (L * G);
    if (j > 32) j = 32;          // 2*J locations fit one 64-lane load
    return j < 1 ? 1 : j;
}

size_t lds_bytes_for(const OpArgs& a, int waves) {
    const size_t geo = (size_t)a.N * a.L * sizeof(Geo);
    const size_t stage = (size_t)waves * a.pairs_per_chunk * (a.L * a.G + 2) * sizeof(float);
    const size_t red = (size_t)waves * a.C * sizeof(float);
    return geo + (stage > red ? stage : red);
}

// The forward of one anchor (index ba = b*A + a of `a`) by the whole
// workgroup; the geometry of `a` is already staged in geo. Called by every
// thread of the block (it ends with block-wide barriers).
template <class FT, int CPL>
__device__ __forceinline__ void fwd_anchor(const OpArgs& a, const int ba, const Geo* geo,
                                           float* work) {
    using RowT = Row<FT, CPL>;
    const int LG = a.L * a.G;
    const int J = a.pairs_per_chunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    float* sw = work + wave * J * (LG + 2);
    float* sl = sw + J * LG;

    const int b = ba / a.A;
    const int npairs = a.P * a.N;
    const float* gl = a.loc + (size_t)ba * npairs * 2;
    const float* gw = a.w + (size_t)ba * npairs * LG;

    const int lps = 1 << a.lps_shift;
    const int spw = 64 >> a.lps_shift;
    const int sub = lane >> a.lps_shift;
    const int c0 = (lane & (lps - 1)) * CPL;
    const int g = c0 / (a.C / a.G);
    const u32 row_bytes = (u32)a.C * FT::kBytes;
    const u32 lane_off = (u32)c0 * FT::kBytes;
    const rsrc_t feat = make_rsrc(static_cast<const char*>(a.feat) + (size_t)b * a.batch_bytes,
                                  a.batch_bytes);

    float acc[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[i] = 0.f;

    const int nchunks = (npairs + J - 1) / J;
    for (int k = wave; k < nchunks; k += nwaves) {
        const int j0 = k * J;
        const int nj = min(J, npairs - j0);
        stage_chunk(sw, sl, gw + (size_t)j0 * LG, gl + (size_t)j0 * 2, nj, LG, lane);
        for (int jj = sub; jj < nj; jj += spw) {
            const int n = (j0 + jj) % a.N;
            const float u = sl[2 * jj], v = sl[2 * jj + 1];
            const float* wj = sw + jj * LG + g;
            for (int l0 = 0; l0 < a.L; l0 += 4) {
                u32 raw[4][4][RowT::kWords];
                float cw[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int l = l0 + q;
                    if (l < a.L) {
                        const Geo gm = geo[n * a.L + l];
                        const Corners cr = corners_of(u, v, gm, row_bytes, lane_off);
                        float wl = wj[l * a.G];
                        if constexpr (FT::kBytes == 1) wl *= gm.scale;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            cw[q][c] = cr.cw[c] * wl;
                            load_words<RowT::kWords>(feat, cr.off[c], raw[q][c]);
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            cw[q][c] = 0.f;
#pragma unroll
                            for (int t = 0; t < RowT::kWords; ++t) raw[q][c][t] = 0u;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        float f[CPL];
                        widen<FT, CPL>(raw[q][c], f);
#pragma unroll
                        for (int i = 0; i < CPL; ++i) acc[i] = fmaf(cw[q][c], f[i], acc[i]);
                    }
                }
            }
        }
        end_chunk();
    }

    // Samples of a wave that share channels: butterfly over the sub-wave index.
    for (int s = lps; s < 64; s <<= 1) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[i] += xor_shuffle(acc[i], s);
    }
    float* out = a.out + (size_t)ba * a.C;
    if (nwaves == 1) {
        if (sub == 0) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) out[c0 + i] = acc[i];
        }
        return;
    }
    __syncthreads();                       // every wave is done with its staging slot
    if (sub == 0) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) work[wave * a.C + c0 + i] = acc[i];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < a.C; c += blockDim.x) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += work[w * a.C + c];   // fixed order
        out[c] = s;
    }
    __syncthreads();                       // work is free again
}

template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_kernel(OpArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    float* work = reinterpret_cast<float*>(smem + (size_t)a.N * a.L * sizeof(Geo));
    stage_geometry(geo, a);
    __syncthreads();
    fwd_anchor<FT, CPL>(a, (int)blockIdx.x, geo, work);
}

// Batched forward: persistent workgroups stride over the anchors of all
// scenes; each restages its scene's geometry before the anchor.
template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_batched_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    float* work = reinterpret_cast<float*>(smem + (size_t)b.max_regions_per_scene * sizeof(Geo));
    for (u32 item = blockIdx.x; item < b.total_anchors; item += gridDim.x) {
        const int s = scene_of(b.t.anchor_start, b.S, item);
        const OpArgs a = scene_view(b, s, FT::kBytes);
        __syncthreads();                    // the previous anchor is done with geo and work
        stage_geometry(geo, a);
        __syncthreads();
        fwd_anchor<FT, CPL>(a, (int)(item - b.t.anchor_start[s]), geo, work);
    }
}

template <class FT, int CPL>
static hipError_t fwd_batched_launch(const BatchArgs& b, int waves, int blocks, size_t lds,
                                     hipStream_t s) {
    mark_begin("msda_fwd_batched_kernel", s);
    hipLaunchKernelGGL((msda_fwd_batched_kernel<FT, CPL>), dim3(blocks), dim3(64 * waves), lds, s,
                       b);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_forward_batched(const BatchArgs& b, int dtype, int cpl, int waves, int blocks,
                                  size_t lds, hipStream_t s) {
    switch (dtype * 100 + cpl) {
        case kF32 * 100 + 1: return fwd_batched_launch<TF32, 1>(b, waves, blocks, lds, s);
        case kF32 * 100 + 2: return fwd_batched_launch<TF32, 2>(b, waves, blocks, lds, s);
        case kF32 * 100 + 4: return fwd_batched_launch<TF32, 4>(b, waves, blocks, lds, s);
        case kBF16 * 100 + 2: return fwd_batched_launch<TBF16, 2>(b, waves, blocks, lds, s);
        case kBF16 * 100 + 4: return fwd_batched_launch<TBF16, 4>(b, waves, blocks, lds, s);
        case kBF16 * 100 + 8: return fwd_batched_launch<TBF16, 8>(b, waves, blocks, lds, s);
        case kFP8 * 100 + 4: return fwd_batched_launch<TFP8, 4>(b, waves, blocks, lds, s);
        case kFP8 * 100 + 8: return fwd_batched_launch<TFP8, 8>(b, waves, blocks, lds, s);
        case kFP8 * 100 + 16: return fwd_batched_launch<TFP8, 16>(b, waves, blocks, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <class FT, int CPL>
static hipError_t fwd_launch(const OpArgs& a, int waves, size_t lds, hipStream_t s) {
    mark_begin("msda_fwd_kernel", s);
    hipLaunchKernelGGL((msda_fwd_kernel<FT, CPL>), dim3((unsigned)(a.B * a.A)),
                       dim3(64 * waves), lds, s, a);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_forward(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                          hipStream_t s) {
    switch (dtype * 100 + cpl) {
        case kF32 * 100 + 1: return fwd_launch<TF32, 1>(a, waves, lds, s);
        case kF32 * 100 + 2: return fwd_launch<TF32, 2>(a, waves, lds, s);
        case kF32 * 100 + 4: return fwd_launch<TF32, 4>(a, waves, lds, s);
        case kBF16 * 100 + 2: return fwd_launch<TBF16, 2>(a, waves, lds, s);
        case kBF16 * 100 + 4: return fwd_launch<TBF16, 4>(a, waves, lds, s);
        case kBF16 * 100 + 8: return fwd_launch<TBF16, 8>(a, waves, lds, s);
        case kFP8 * 100 + 4: return fwd_launch<TFP8, 4>(a, waves, lds, s);
        case kFP8 * 100 + 8: return fwd_launch<TFP8, 8>(a, waves, lds, s);
        case kFP8 * 100 + 16: return fwd_launch<TFP8, 16>(a, waves, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace msda
