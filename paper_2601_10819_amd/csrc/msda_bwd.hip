// Backward gathers of multi-scale deformable aggregation: gradients of
// <grad_out, out> with respect to the sampling locations and the weights,
// and the grad_feat records.
//
// msda_bwd_kernel (one workgroup per (batch item, anchor), the forward's lane
// layout) and msda_bwd_view_kernel (view order) re-gather the 4 corner rows
// of each sample and form, per lane, d[c] = <grad_out, corner c> over its
// channels. Then
//   grad_w[g]  = sum over the group's lanes of sum_c cw[c] * d[c]
//                (a shuffle reduction within the group's lanes),
//   grad_loc   = sum over levels of W (H) * w * (d/dx (d/dy) of the bilinear
//                blend of d), reduced over the sample's lanes once per
//                (keypoint, camera) pair.
// For grad_feat they either emit one record per sample -- the bilinear cell
// the sample falls in (its top-left neighbour, (y0+1, x0+1) in an
// (H+1) x (W+1) grid per region) and its fractions (lx, ly) -- for the
// sorted, tiled reduction (msda_sort.hip, msda_tiles.hip; deterministic, no
// float atomics), or add w * cw * grad_out to an FP32 accumulator with float
// atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_gather.h"

namespace msda {

// The backward gather of one anchor (index ba = b*A + a of `a`) by the
// whole workgroup in anchor order; the geometry of `a` is already staged in
// geo. The lane that stages a sample also writes its grad_feat record.
template <class FT, int CPL>
__device__ __forceinline__ void bwd_anchor(const OpArgs& a, const int ba, const Geo* geo,
                                           unsigned char* work) {
    const int J = a.pairs_per_chunk;
    const int wave = wave_index(), nwaves = blockDim.x >> 6;
    const Lanes q = lanes_of<FT, CPL>(a);
    const StageSlot st = stage_slot(work, wave, J, a.L, a.G);
    float go[CPL];
    const BwdAnchor x = bwd_anchor_ctx<FT, CPL>(a, ba, q, go);
    const AnchorOrder order{a.N};
    const int npairs = a.P * a.N;
    const int nchunks = (npairs + J - 1) / J;
    for (int k = wave; k < nchunks; k += nwaves) {
        const int k0 = k * J;
        const int nj = min(J, npairs - k0);
        stage_chunk<false, true>(st, order, k0, nj, x.gw, x.gl, geo, a.L, a.L * a.G,
                                 (u32)a.C * FT::kBytes, q.lane, x.rec);
        bwd_chunk<FT, CPL>(a, st, nj, geo, q, x, go);
        end_chunk();
    }
}

template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_bwd_kernel(OpArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)a.N * a.L * sizeof(Geo);
    stage_geometry(geo, a);
    __syncthreads();
    bwd_anchor<FT, CPL>(a, (int)blockIdx.x, geo, work);
}

// View order (see slot_span): workgroup w serves slot w % kSlots, each wave
// one anchor over a small group of cameras (a.view_cams; groups aligned
// within the batch item) in the slot's view-major order, so an XCD's L2
// holds the pyramids of about a group of cameras at a time (the forward's
// rows span all of a slot's cameras, whose partial sums it must add; here
// every output is per sample or per pair, so the rows need no combining).
template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_bwd_view_kernel(OpArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)a.N * a.L * sizeof(Geo);
    stage_geometry(geo, a);
    __syncthreads();                       // the only block-wide barrier

    const int xs = (int)(blockIdx.x % kSlots);
    const int wave = wave_index(), nwaves = blockDim.x >> 6;
    const int64_t r = (int64_t)(blockIdx.x / kSlots) * nwaves + wave;
    const SlotSpan span = slot_span(xs, a.B, a.N, a.A);
    // one anchor over a group of a.view_cams cameras per wave (groups
    // aligned within each batch item), rows in the slot's view-major order:
    // the waves in flight on an XCD work through a few cameras at a time
    if (span.hi <= span.lo) return;
    const int M = max(1, a.view_cams);
    const int gpb = (a.N + M - 1) / M;                     // camera groups per batch item
    const int64_t vf = span.lo / a.A, vl = (span.hi - 1) / a.A;
    const int64_t gf = (vf / a.N) * gpb + (vf % a.N) / M;
    const int64_t g = gf + r / a.A;
    const int64_t gl = (vl / a.N) * gpb + (vl % a.N) / M;
    if (g > gl) return;
    ViewRow row;
    {
        row.a = (int32_t)(r % a.A);
        row.b = (int32_t)(g / gpb);
        const int j = (int)(g - (int64_t)row.b * gpb);
        const int64_t base = (int64_t)row.b * a.N;
        int64_t v0 = base + (int64_t)j * M, v1 = base + min((j + 1) * M, a.N);
        // the views whose item (view, a) lies in the slot
        const int64_t lo_v = (span.lo - row.a + a.A - 1) / a.A;
        const int64_t hi_v = (span.hi - row.a + a.A - 1) / a.A;
        if (v0 < lo_v) v0 = lo_v;
        if (v1 > hi_v) v1 = hi_v;
        row.n_lo = (int32_t)(v0 - base);
        row.nv = v1 > v0 ? (int32_t)(v1 - v0) : 0;
    }
    // every field is the same across the wave (r is per wave)
    row.b = uniform(row.b);
    row.a = uniform(row.a);
    row.n_lo = uniform(row.n_lo);
    row.nv = uniform(row.nv);
    if (row.nv == 0) return;

    const int J = a.pairs_per_chunk;
    const Lanes q = lanes_of<FT, CPL>(a);
    const StageSlot st = stage_slot(work, wave, J, a.L, a.G);
    float go[CPL];
    const BwdAnchor x = bwd_anchor_ctx<FT, CPL>(a, row.b * a.A + row.a, q, go);
    const ViewOrder order{a.N, a.P, row.n_lo};
    const int nk = row.nv * a.P;
    for (int k0 = 0; k0 < nk; k0 += J) {
        const int nj = min(J, nk - k0);
        stage_chunk<false, true>(st, order, k0, nj, x.gw, x.gl, geo, a.L, a.L * a.G,
                                 (u32)a.C * FT::kBytes, q.lane, x.rec);
        bwd_chunk<FT, CPL>(a, st, nj, geo, q, x, go);
        end_chunk();
    }
}

// Batched backward gather: persistent workgroups stride over the anchors of
// all scenes; records go to the batch's sample space, per (scene, region)
// bucket with local cells or at the sample index with batch-global cells.
template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_bwd_batched_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)b.max_regions_per_scene * sizeof(Geo);
    for (u32 item = blockIdx.x; item < b.total_anchors; item += gridDim.x) {
        const int s = scene_of(b.t.anchor_start, b.S, item);
        const OpArgs a = scene_view(b, s, FT::kBytes);
        __syncthreads();                    // the previous anchor is done with geo
        stage_geometry(geo, a);
        __syncthreads();
        bwd_anchor<FT, CPL>(a, (int)(item - b.t.anchor_start[s]), geo, work);
    }
}

// Batched backward gather in view order (see msda_fwd_batched_view_kernel):
// one wave per (XCD slot, global anchor) row over the anchor's cameras in
// the slot; every output is per sample or per pair.
template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_bwd_batched_view_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int x = (int)(blockIdx.x % kSlots);
    const int wave = wave_index(), nwaves = blockDim.x >> 6;
    const u32 g = (blockIdx.x / kSlots) * (u32)nwaves + (u32)wave;
    if (g >= b.total_anchors) return;
    const BatchRow row = batch_row(b, x, g);
    if (row.nv == 0) return;
    unsigned char* mine =
        smem + (size_t)wave * batch_view_wave_bytes(b.view_cams, b.L, b.pairs_per_chunk, b.G);
    Geo* geo = reinterpret_cast<Geo*>(mine);
    unsigned char* work =
        mine + (((size_t)b.view_cams * b.L * sizeof(Geo) + 15) & ~(size_t)15);
    const OpArgs a = scene_view(b, row.s, FT::kBytes);
    const Lanes q = lanes_of<FT, CPL>(a);
    stage_geometry_range(geo, a, row.n_lo, row.nv, q.lane);

    const int J = a.pairs_per_chunk;
    const StageSlot st = stage_slot(work, 0, J, a.L, a.G);
    float go[CPL];
    const BwdAnchor xa = bwd_anchor_ctx<FT, CPL>(a, row.a, q, go);
    const ViewOrder order{a.N, a.P, row.n_lo, row.n_lo};
    const int nk = row.nv * a.P;
    for (int k0 = 0; k0 < nk; k0 += J) {
        const int nj = min(J, nk - k0);
        stage_chunk<false, true>(st, order, k0, nj, xa.gw, xa.gl, geo, a.L, a.L * a.G,
                                 (u32)a.C * FT::kBytes, q.lane, xa.rec);
        bwd_chunk<FT, CPL>(a, st, nj, geo, q, xa, go);
        end_chunk();
    }
}

// ---------------------------------------------------------------- launchers

template <class FT, int CPL>
static hipError_t bwd_launch(const OpArgs& a, int waves, size_t lds, hipStream_t s) {
    mark_begin("msda_bwd_kernel", s);
    hipLaunchKernelGGL((msda_bwd_kernel<FT, CPL>), dim3((unsigned)(a.B * a.A)),
                       dim3(64 * waves), lds, s, a);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_backward(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                           hipStream_t s) {
    switch (dtype * 100 + cpl) {
        case kF32 * 100 + 1: return bwd_launch<TF32, 1>(a, waves, lds, s);
        case kF32 * 100 + 2: return bwd_launch<TF32, 2>(a, waves, lds, s);
        case kF32 * 100 + 4: return bwd_launch<TF32, 4>(a, waves, lds, s);
        case kBF16 * 100 + 2: return bwd_launch<TBF16, 2>(a, waves, lds, s);
        case kF16 * 100 + 2: return bwd_launch<TF16, 2>(a, waves, lds, s);
        case kBF16 * 100 + 4: return bwd_launch<TBF16, 4>(a, waves, lds, s);
        case kF16 * 100 + 4: return bwd_launch<TF16, 4>(a, waves, lds, s);
        case kBF16 * 100 + 8: return bwd_launch<TBF16, 8>(a, waves, lds, s);
        case kF16 * 100 + 8: return bwd_launch<TF16, 8>(a, waves, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <class FT, int CPL>
static hipError_t bwd_view_launch(const OpArgs& a, int waves, size_t lds, hipStream_t s) {
    // rows per slot at most: the camera groups a slot touches, times A
    int64_t rows = 0;
    const int M = max(1, a.view_cams), gpb = (a.N + M - 1) / M;
    for (int x = 0; x < kSlots; ++x) {
        const SlotSpan sp = slot_span(x, a.B, a.N, a.A);
        if (sp.hi <= sp.lo) continue;
        const int64_t vf = sp.lo / a.A, vl = (sp.hi - 1) / a.A;
        const int64_t gf = (vf / a.N) * gpb + (vf % a.N) / M;
        const int64_t gl = (vl / a.N) * gpb + (vl % a.N) / M;
        rows = max(rows, (gl - gf + 1) * (int64_t)a.A);
    }
    const unsigned blocks = (unsigned)(kSlots * ((rows + waves - 1) / waves));
    mark_begin("msda_bwd_view_kernel", s);
    hipLaunchKernelGGL((msda_bwd_view_kernel<FT, CPL>), dim3(blocks), dim3(64 * waves), lds, s,
                       a);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_backward_view(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                                hipStream_t s) {
    switch (dtype * 100 + cpl) {
        case kF32 * 100 + 1: return bwd_view_launch<TF32, 1>(a, waves, lds, s);
        case kF32 * 100 + 2: return bwd_view_launch<TF32, 2>(a, waves, lds, s);
        case kF32 * 100 + 4: return bwd_view_launch<TF32, 4>(a, waves, lds, s);
        case kBF16 * 100 + 2: return bwd_view_launch<TBF16, 2>(a, waves, lds, s);
        case kF16 * 100 + 2: return bwd_view_launch<TF16, 2>(a, waves, lds, s);
        case kBF16 * 100 + 4: return bwd_view_launch<TBF16, 4>(a, waves, lds, s);
        case kF16 * 100 + 4: return bwd_view_launch<TF16, 4>(a, waves, lds, s);
        case kBF16 * 100 + 8: return bwd_view_launch<TBF16, 8>(a, waves, lds, s);
        case kF16 * 100 + 8: return bwd_view_launch<TF16, 8>(a, waves, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <class FT, int CPL>
static hipError_t bwd_batched_launch(const BatchArgs& b, int waves, int blocks, size_t lds,
                                     hipStream_t s) {
    mark_begin("msda_bwd_batched_kernel", s);
    hipLaunchKernelGGL((msda_bwd_batched_kernel<FT, CPL>), dim3(blocks), dim3(64 * waves), lds, s,
                       b);
    mark_end(s);
    return hipGetLastError();
}

template <class FT, int CPL>
static hipError_t bwd_batched_view_launch(const BatchArgs& b, int waves, size_t lds,
                                          hipStream_t s) {
    const unsigned blocks =
        (unsigned)(kSlots * (((size_t)b.total_anchors + waves - 1) / (size_t)waves));
    mark_begin("msda_bwd_batched_view_kernel", s);
    hipLaunchKernelGGL((msda_bwd_batched_view_kernel<FT, CPL>), dim3(blocks), dim3(64 * waves),
                       lds, s, b);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_backward_batched_view(const BatchArgs& b, int dtype, int cpl, int waves,
                                        size_t lds, hipStream_t s) {
    switch (dtype * 100 + cpl) {
        case kF32 * 100 + 1: return bwd_batched_view_launch<TF32, 1>(b, waves, lds, s);
        case kF32 * 100 + 2: return bwd_batched_view_launch<TF32, 2>(b, waves, lds, s);
        case kF32 * 100 + 4: return bwd_batched_view_launch<TF32, 4>(b, waves, lds, s);
        case kBF16 * 100 + 2: return bwd_batched_view_launch<TBF16, 2>(b, waves, lds, s);
        case kF16 * 100 + 2: return bwd_batched_view_launch<TF16, 2>(b, waves, lds, s);
        case kBF16 * 100 + 4: return bwd_batched_view_launch<TBF16, 4>(b, waves, lds, s);
        case kF16 * 100 + 4: return bwd_batched_view_launch<TF16, 4>(b, waves, lds, s);
        case kBF16 * 100 + 8: return bwd_batched_view_launch<TBF16, 8>(b, waves, lds, s);
        case kF16 * 100 + 8: return bwd_batched_view_launch<TF16, 8>(b, waves, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward_batched(const BatchArgs& b, int dtype, int cpl, int waves, int blocks,
                                   size_t lds, hipStream_t s) {
    switch (dtype * 100 + cpl) {
        case kF32 * 100 + 1: return bwd_batched_launch<TF32, 1>(b, waves, blocks, lds, s);
        case kF32 * 100 + 2: return bwd_batched_launch<TF32, 2>(b, waves, blocks, lds, s);
        case kF32 * 100 + 4: return bwd_batched_launch<TF32, 4>(b, waves, blocks, lds, s);
        case kBF16 * 100 + 2: return bwd_batched_launch<TBF16, 2>(b, waves, blocks, lds, s);
        case kF16 * 100 + 2: return bwd_batched_launch<TF16, 2>(b, waves, blocks, lds, s);
        case kBF16 * 100 + 4: return bwd_batched_launch<TBF16, 4>(b, waves, blocks, lds, s);
        case kF16 * 100 + 4: return bwd_batched_launch<TF16, 4>(b, waves, blocks, lds, s);
        case kBF16 * 100 + 8: return bwd_batched_launch<TBF16, 8>(b, waves, blocks, lds, s);
        case kF16 * 100 + 8: return bwd_batched_launch<TF16, 8>(b, waves, blocks, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace msda
