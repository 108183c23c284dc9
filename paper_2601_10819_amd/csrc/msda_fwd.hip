// Forward kernels of multi-scale deformable aggregation (paper Sec. 3.1 /
// Sec. 3.2): out[b,a,:] = sum over (keypoint, camera, level) of weight *
// bilinear sample.
//
// Anchor order (msda_fwd_kernel): one workgroup per (batch item, anchor);
// its waves split the anchor's (keypoint, camera) pairs in chunks and the
// waves' partial sums are added in a fixed order at the end.
//
// View order (msda_fwd_view_kernel): the (view, anchor) items are cut into
// one contiguous range per XCD (see slot_span); each wave sums one anchor
// over its views in the slot and writes a per-slot partial row, and
// fwd_view_reduce adds the slots' partials in slot order. Both orders are
// deterministic.
//
// In both, a wave stages a chunk of pairs -- the pairs' weights and the
// corner taps of their samples, one sample per lane, so the coordinate
// arithmetic is done once per sample rather than once per lane of a sample
// -- then each group of C/CPL lanes takes a pair and issues the corner
// loads of all its levels before using them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_gather.h"

namespace msda {

int max_pairs_per_chunk(int L, int G) {
    int j = (kStageWords * 64) / (L * G);
    if (j > 32) j = 32;
    return j < 1 ? 1 : j;
}

size_t lds_bytes_for(const OpArgs& a, int waves) {
    const size_t geo = (size_t)a.N * a.L * sizeof(Geo);
    const size_t stage = (size_t)waves * wave_stage_bytes(a.pairs_per_chunk, a.L, a.G);
    const size_t red = (size_t)waves * a.C * sizeof(float);
    return geo + (stage > red ? stage : red);
}

size_t batch_view_lds(int view_cams, int L, int J, int G, int waves) {
    return (size_t)waves * batch_view_wave_bytes(view_cams, L, J, G);
}

size_t lds_bytes_view(const OpArgs& a, int waves) {
    return (size_t)a.N * a.L * sizeof(Geo) +
           (size_t)waves * wave_stage_bytes(a.pairs_per_chunk, a.L, a.G);
}

// The forward of one anchor (index ba = b*A + a of `a`) by the whole
// workgroup in anchor order; the geometry of `a` is already staged in geo.
// Called by every thread of the block (it ends with block-wide barriers).
template <class FT, int CPL>
__device__ __forceinline__ void fwd_anchor(const OpArgs& a, const int ba, const Geo* geo,
                                           unsigned char* work) {
    const int LG = a.L * a.G;
    const int J = a.pairs_per_chunk;
    const int wave = wave_index(), nwaves = blockDim.x >> 6;
    const Lanes q = lanes_of<FT, CPL>(a);
    const StageSlot st = stage_slot(work, wave, J, a.L, a.G);
    const int b = ba / a.A;
    const int npairs = a.P * a.N;
    const float* gl = a.loc + (size_t)ba * npairs * 2;
    const WSrc gw = anchor_weights(a, (size_t)ba, (size_t)npairs * LG);
    const u32 row_bytes = (u32)a.C * FT::kBytes;
    const rsrc_t feat = make_rsrc(static_cast<const char*>(a.feat) + (size_t)b * a.batch_bytes,
                                  a.batch_bytes);
    const AnchorOrder order{a.N};
    const RecordSink none{};

    float acc[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[i] = 0.f;
    const int nchunks = (npairs + J - 1) / J;
    for (int k = wave; k < nchunks; k += nwaves) {
        const int k0 = k * J;
        const int nj = min(J, npairs - k0);
        stage_chunk<FT::kBytes == 1, false>(st, order, k0, nj, gw, gl, geo, a.L, LG, row_bytes,
                                            q.lane, none);
        fwd_chunk<FT, CPL>(st, nj, a.L, a.G, q, feat, acc);
        end_chunk();
    }
    reduce_subwaves<CPL>(q, acc);

    float* out = a.out + (size_t)ba * a.C;
    if (nwaves == 1) {
        if (q.sub == 0) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) out[q.c0 + i] = acc[i];
        }
        return;
    }
    float* red = reinterpret_cast<float*>(work);
    __syncthreads();                       // every wave is done with its staging slot
    if (q.sub == 0) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) red[wave * a.C + q.c0 + i] = acc[i];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < a.C; c += blockDim.x) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += red[w * a.C + c];   // fixed order
        out[c] = s;
    }
    __syncthreads();                       // work is free again
}

template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_kernel(OpArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)a.N * a.L * sizeof(Geo);
    stage_geometry(geo, a);
    __syncthreads();
    fwd_anchor<FT, CPL>(a, (int)blockIdx.x, geo, work);
}

// View order: workgroup w serves slot w % kSlots; its waves take
// consecutive rows of the slot. Each wave writes its row's partial sum
// (zeros for an empty row) to part[slot][b*A + a].
template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_view_kernel(OpArgs a, float* part) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)a.N * a.L * sizeof(Geo);
    stage_geometry(geo, a);
    __syncthreads();                       // the only block-wide barrier

    const int x = (int)(blockIdx.x % kSlots);
    const int wave = wave_index(), nwaves = blockDim.x >> 6;
    const int64_t r = (int64_t)(blockIdx.x / kSlots) * nwaves + wave;
    const SlotSpan span = slot_span(x, a.B, a.N, a.A);
    if (r >= slot_rows(span, a.A)) return;
    ViewRow row = view_row(span, r, a.N, a.A);
    // every field is the same across the wave (r is per wave)
    row.b = uniform(row.b);
    row.a = uniform(row.a);
    row.n_lo = uniform(row.n_lo);
    row.nv = uniform(row.nv);

    const int LG = a.L * a.G;
    const int J = a.pairs_per_chunk;
    const Lanes q = lanes_of<FT, CPL>(a);
    const StageSlot st = stage_slot(work, wave, J, a.L, a.G);
    const int ba = row.b * a.A + row.a;
    const int npairs = a.P * a.N;
    const float* gl = a.loc + (size_t)ba * npairs * 2;
    const WSrc gw = anchor_weights(a, (size_t)ba, (size_t)npairs * LG);
    const u32 row_bytes = (u32)a.C * FT::kBytes;
    const rsrc_t feat = make_rsrc(
        static_cast<const char*>(a.feat) + (size_t)row.b * a.batch_bytes, a.batch_bytes);
    const ViewOrder order{a.N, a.P, row.n_lo};
    const RecordSink none{};

    float acc[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[i] = 0.f;
    const int nk = row.nv * a.P;
    for (int k0 = 0; k0 < nk; k0 += J) {
        const int nj = min(J, nk - k0);
        stage_chunk<FT::kBytes == 1, false>(st, order, k0, nj, gw, gl, geo, a.L, LG, row_bytes,
                                            q.lane, none);
        fwd_chunk<FT, CPL>(st, nj, a.L, a.G, q, feat, acc);
        end_chunk();
    }
    reduce_subwaves<CPL>(q, acc);
    if (q.sub == 0) {
        float* dst = part + ((size_t)x * a.B * a.A + ba) * a.C + q.c0;
#pragma unroll
        for (int i = 0; i < CPL; ++i) dst[i] = acc[i];
    }
}

// out[i] = sum over the slots that touch i's batch item of part[slot][i],
// in slot order; four floats per thread (C % 4 == 0) or one.
template <int V>
__global__ void __launch_bounds__(256) fwd_view_reduce(const float* part, float* out, int B,
                                                       int N, int A, int C) {
    const size_t total = (size_t)B * A * C;
    const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * V;
    if (i >= total) return;
    const int b = (int)(i / ((size_t)A * C));
    float s[V];
#pragma unroll
    for (int v = 0; v < V; ++v) s[v] = 0.f;
    for (int x = 0; x < kSlots; ++x) {
        const SlotSpan span = slot_span(x, B, N, A);
        if (b < span.b_first || b > span.b_last) continue;
        const float* p = part + (size_t)x * total + i;
        if constexpr (V == 4) {
            const float4 t = *reinterpret_cast<const float4*>(p);
            s[0] += t.x; s[1] += t.y; s[2] += t.z; s[3] += t.w;
        } else {
            s[0] += p[0];
        }
    }
    if constexpr (V == 4) {
        *reinterpret_cast<float4*>(out + i) = make_float4(s[0], s[1], s[2], s[3]);
    } else {
        out[i] = s[0];
    }
}

// Batched forward: persistent workgroups stride over the anchors of all
// scenes; each restages its scene's geometry before the anchor.
template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_batched_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)b.max_regions_per_scene * sizeof(Geo);
    for (u32 item = blockIdx.x; item < b.total_anchors; item += gridDim.x) {
        const int s = scene_of(b.t.anchor_start, b.S, item);
        const OpArgs a = scene_view(b, s, FT::kBytes);
        __syncthreads();                    // the previous anchor is done with geo and work
        stage_geometry(geo, a);
        __syncthreads();
        fwd_anchor<FT, CPL>(a, (int)(item - b.t.anchor_start[s]), geo, work);
    }
}

// Batched forward in view order: workgroup w serves XCD slot w % kSlots;
// each wave takes one global anchor g over its scene's cameras in that slot
// (the single call's slot split of the scene), stages just those cameras'
// geometry in its own LDS slice and writes the row's partial sum (zeros for
// an anchor with no cameras in the slot) to part[slot][g]. Per anchor the
// arithmetic is the single call's view order.
template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_batched_view_kernel(BatchArgs b, float* part) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int x = (int)(blockIdx.x % kSlots);
    const int wave = wave_index(), nwaves = blockDim.x >> 6;
    const u32 g = (blockIdx.x / kSlots) * (u32)nwaves + (u32)wave;
    if (g >= b.total_anchors) return;
    unsigned char* mine =
        smem + (size_t)wave * batch_view_wave_bytes(b.view_cams, b.L, b.pairs_per_chunk, b.G);
    Geo* geo = reinterpret_cast<Geo*>(mine);
    unsigned char* work =
        mine + (((size_t)b.view_cams * b.L * sizeof(Geo) + 15) & ~(size_t)15);
    const BatchRow row = batch_row(b, x, g);
    const OpArgs a = scene_view(b, row.s, FT::kBytes);
    const Lanes q = lanes_of<FT, CPL>(a);
    stage_geometry_range(geo, a, row.n_lo, row.nv, q.lane);

    const int LG = a.L * a.G;
    const int J = a.pairs_per_chunk;
    const StageSlot st = stage_slot(work, 0, J, a.L, a.G);
    const int npairs = a.P * a.N;
    const float* gl = a.loc + (size_t)row.a * npairs * 2;
    const WSrc gw = anchor_weights(a, (size_t)row.a, (size_t)npairs * LG);
    const u32 row_bytes = (u32)a.C * FT::kBytes;
    const rsrc_t feat = make_rsrc(a.feat, a.batch_bytes);
    const ViewOrder order{a.N, a.P, row.n_lo, row.n_lo};
    const RecordSink none{};

    float acc[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[i] = 0.f;
    const int nk = row.nv * a.P;
    for (int k0 = 0; k0 < nk; k0 += J) {
        const int nj = min(J, nk - k0);
        stage_chunk<FT::kBytes == 1, false>(st, order, k0, nj, gw, gl, geo, a.L, LG, row_bytes,
                                            q.lane, none);
        fwd_chunk<FT, CPL>(st, nj, a.L, a.G, q, feat, acc);
        end_chunk();
    }
    reduce_subwaves<CPL>(q, acc);
    if (q.sub == 0) {
        float* dst = part + ((size_t)x * b.total_anchors + g) * b.C + q.c0;
#pragma unroll
        for (int i = 0; i < CPL; ++i) dst[i] = acc[i];
    }
}

// out of global anchor g = sum over the slots of part[slot][g], in slot
// order, written to its scene's output; V floats per thread.
template <int V>
__global__ void __launch_bounds__(256) fwd_batched_view_reduce(BatchArgs b, const float* part) {
    const size_t total = (size_t)b.total_anchors * b.C;
    const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * V;
    if (i >= total) return;
    const u32 g = (u32)(i / (size_t)b.C);
    const int c = (int)(i - (size_t)g * b.C);
    const int sc = scene_of(b.t.anchor_start, b.S, g);
    float s[V];
#pragma unroll
    for (int v = 0; v < V; ++v) s[v] = 0.f;
    for (int x = 0; x < kSlots; ++x) {
        const float* p = part + (size_t)x * total + i;
        if constexpr (V == 4) {
            const float4 t = *reinterpret_cast<const float4*>(p);
            s[0] += t.x; s[1] += t.y; s[2] += t.z; s[3] += t.w;
        } else {
            s[0] += p[0];
        }
    }
    float* out = b.scenes[sc].out + (size_t)(g - b.t.anchor_start[sc]) * b.C + c;
    if constexpr (V == 4) {
        *reinterpret_cast<float4*>(out) = make_float4(s[0], s[1], s[2], s[3]);
    } else {
        out[0] = s[0];
    }
}

template <class FT, int CPL>
static hipError_t fwd_batched_view_launch(const BatchArgs& b, int waves, size_t lds, float* part,
                                          hipStream_t s) {
    const unsigned blocks =
        (unsigned)(kSlots * (((size_t)b.total_anchors + waves - 1) / (size_t)waves));
    mark_begin("msda_fwd_batched_view_kernel", s);
    hipLaunchKernelGGL((msda_fwd_batched_view_kernel<FT, CPL>), dim3(blocks), dim3(64 * waves),
                       lds, s, b, part);
    mark_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)b.total_anchors * b.C;
    mark_begin("fwd_batched_view_reduce", s);
    if (b.C % 4 == 0) {
        hipLaunchKernelGGL(fwd_batched_view_reduce<4>, dim3((unsigned)((total / 4 + 255) / 256)),
                           dim3(256), 0, s, b, part);
    } else {
        hipLaunchKernelGGL(fwd_batched_view_reduce<1>, dim3((unsigned)((total + 255) / 256)),
                           dim3(256), 0, s, b, part);
    }
    mark_end(s);
    return hipGetLastError();
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

template <class FT, int CPL>
static hipError_t fwd_launch(const OpArgs& a, int waves, size_t lds, hipStream_t s) {
    mark_begin("msda_fwd_kernel", s);
    hipLaunchKernelGGL((msda_fwd_kernel<FT, CPL>), dim3((unsigned)(a.B * a.A)),
                       dim3(64 * waves), lds, s, a);
    mark_end(s);
    return hipGetLastError();
}

template <class FT, int CPL>
static hipError_t fwd_view_launch(const OpArgs& a, int waves, size_t lds, float* part,
                                  hipStream_t s) {
    const int64_t rows = max_slot_rows(a.B, a.N, a.A);
    const unsigned blocks = (unsigned)(kSlots * ((rows + waves - 1) / waves));
    mark_begin("msda_fwd_view_kernel", s);
    hipLaunchKernelGGL((msda_fwd_view_kernel<FT, CPL>), dim3(blocks), dim3(64 * waves), lds, s,
                       a, part);
    mark_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)a.B * a.A * a.C;
    mark_begin("fwd_view_reduce", s);
    if (a.C % 4 == 0) {
        hipLaunchKernelGGL(fwd_view_reduce<4>, dim3((unsigned)((total / 4 + 255) / 256)),
                           dim3(256), 0, s, part, a.out, a.B, a.N, a.A, a.C);
    } else {
        hipLaunchKernelGGL(fwd_view_reduce<1>, dim3((unsigned)((total + 255) / 256)), dim3(256),
                           0, s, part, a.out, a.B, a.N, a.A, a.C);
    }
    mark_end(s);
    return hipGetLastError();
}

// Instantiations by (dtype, channels per lane).
#define MSDA_FOR_EACH_LAYOUT(F, ...)                                    \
    switch (dtype * 100 + cpl) {                                        \
        case kF32 * 100 + 1: return F<TF32, 1>(__VA_ARGS__);            \
        case kF32 * 100 + 2: return F<TF32, 2>(__VA_ARGS__);            \
        case kF32 * 100 + 4: return F<TF32, 4>(__VA_ARGS__);            \
        case kBF16 * 100 + 2: return F<TBF16, 2>(__VA_ARGS__);          \
        case kBF16 * 100 + 4: return F<TBF16, 4>(__VA_ARGS__);          \
        case kBF16 * 100 + 8: return F<TBF16, 8>(__VA_ARGS__);          \
        case kF16 * 100 + 2: return F<TF16, 2>(__VA_ARGS__);            \
        case kF16 * 100 + 4: return F<TF16, 4>(__VA_ARGS__);            \
        case kF16 * 100 + 8: return F<TF16, 8>(__VA_ARGS__);            \
        case kFP8 * 100 + 4: return F<TFP8, 4>(__VA_ARGS__);            \
        case kFP8 * 100 + 8: return F<TFP8, 8>(__VA_ARGS__);            \
        case kFP8 * 100 + 16: return F<TFP8, 16>(__VA_ARGS__);          \
        default: return hipErrorInvalidValue;                           \
    }

hipError_t launch_forward_batched(const BatchArgs& b, int dtype, int cpl, int waves, int blocks,
                                  size_t lds, hipStream_t s) {
    MSDA_FOR_EACH_LAYOUT(fwd_batched_launch, b, waves, blocks, lds, s)
}

hipError_t launch_forward_batched_view(const BatchArgs& b, int dtype, int cpl, int waves,
                                       size_t lds, float* part, hipStream_t s) {
    MSDA_FOR_EACH_LAYOUT(fwd_batched_view_launch, b, waves, lds, part, s)
}

hipError_t launch_forward(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                          hipStream_t s) {
    MSDA_FOR_EACH_LAYOUT(fwd_launch, a, waves, lds, s)
}

hipError_t launch_forward_view(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                               float* part, hipStream_t s) {
    MSDA_FOR_EACH_LAYOUT(fwd_view_launch, a, waves, lds, part, s)
}

}  // namespace msda
