// The per-chunk work of the MSDA gathers, shared by every work order
// (anchor order, view order, visible views): the forward's accumulation of
// a staged chunk of (keypoint, camera) pairs, and the backward's gradients
// of one. The staging itself (weights, corner taps, records) is in
// msda_common.h.
#pragma once

#include "msda_common.h"

namespace msda {

// Adds the staged chunk's nj pairs into acc: each group of lanes takes a
// pair and loads the 4 corners of 4 levels at a time (padded levels read
// zeros without touching memory) before using them.
template <class FT, int CPL>
__device__ __forceinline__ void fwd_chunk(const StageSlot& st, int nj, int L, int G,
                                          const Lanes& q, rsrc_t feat, float* acc) {
    using RowT = Row<FT, CPL>;
    const int LG = L * G, Lp = padded_levels(L);
    for (int jj = q.sub; jj < nj; jj += q.spw) {
        const float* wj = st.w + jj * LG + q.g;
        const Taps* tj = st.taps + jj * Lp;
        for (int l0 = 0; l0 < Lp; l0 += 4) {
            u32 raw[4][4][RowT::kWords];
            float cw[4][4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const Taps t = tj[l0 + k];
                // a padded level has zero taps; any real weight keeps them zero
                const float wl = wj[min(l0 + k, L - 1) * G];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    cw[k][c] = t.cw[c] * wl;
                    load_words<RowT::kWords>(feat, t.off[c] + q.lane_off, raw[k][c]);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float f[CPL];
                    widen<FT, CPL>(raw[k][c], f);
#pragma unroll
                    for (int i = 0; i < CPL; ++i) acc[i] = fmaf(cw[k][c], f[i], acc[i]);
                }
            }
        }
    }
}

// Sums the per-sample partials of a wave's sub-waves (samples that share
// channels): a butterfly over the sub-wave index.
template <int CPL>
__device__ __forceinline__ void reduce_subwaves(const Lanes& q, float* acc) {
    for (int s = q.lps; s < 64; s <<= 1) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[i] = xor_sum(acc[i], s);
    }
}

// Per-anchor context of the backward gather: grad_out row in registers and
// the anchor's output and record bases.
struct BwdAnchor {
    const float* gw;       // weights of the anchor [P*N][L*G]
    const float* gl;       // locations [P*N][2]
    float* gwout;          // grad_weights of the anchor (or nullptr)
    float* glout;          // grad_sampling_loc of the anchor (or nullptr)
    float* gacc;           // atomic grad_feat: FP32 accumulator row base + c0 (or nullptr)
    RecordSink rec;        // sorted grad_feat records
    rsrc_t feat;
};

template <class FT, int CPL>
__device__ __forceinline__ BwdAnchor bwd_anchor_ctx(const OpArgs& a, int ba, const Lanes& q,
                                                    float* go) {
    const int b = ba / a.A;
    const int npairs = a.P * a.N;
    const int LG = a.L * a.G;
    BwdAnchor x;
    x.gw = a.w + (size_t)ba * npairs * LG;
    x.gl = a.loc + (size_t)ba * npairs * 2;
    x.gwout = a.grad_w ? a.grad_w + (size_t)ba * npairs * LG : nullptr;
    x.glout = a.grad_loc ? a.grad_loc + (size_t)ba * npairs * 2 : nullptr;
    x.gacc = a.gfeat_acc ? a.gfeat_acc + (size_t)b * a.R * a.C + q.c0 : nullptr;
    x.rec.key = a.rec_key;
    x.rec.frac = a.rec_frac;
    x.rec.base = a.sample_offset + (u32)ba * (u32)npairs * (u32)a.L;
    x.rec.cell_base = a.cell_offset + (u32)b * a.cells_per_item;
    x.rec.no_cell = a.no_cell;
    x.rec.val = nullptr;
    x.rec.cbase = 0u;
    x.rec.bucket_ap = a.rec_bucket_ap;
    x.rec.bucket_base = a.sample_offset + (u32)b * (u32)(a.N * a.L) * a.rec_bucket_ap +
                        (u32)(ba - b * a.A) * (u32)a.P;
    x.rec.N = (u32)a.N;
    x.feat = make_rsrc(static_cast<const char*>(a.feat) + (size_t)b * a.batch_bytes,
                       a.batch_bytes);
#pragma unroll
    for (int i = 0; i < CPL; ++i) go[i] = a.grad_out[(size_t)ba * a.C + q.c0 + i];
    return x;
}

// The gradients of one staged chunk of nj pairs. Per sample it re-gathers
// the 4 corners and forms d[c] = <grad_out, corner c> over the lane's
// channels; grad_w is a shuffle reduction over the group's lanes, grad_loc
// one over the sample's lanes per pair; the atomic grad_feat form adds
// w * cw * grad_out into the FP32 accumulator.
//
// out_scale multiplies the grad_w and grad_loc written (the fused form's
// per-view weight; 1 otherwise). dot (or nullptr) accumulates, on each
// group's first lane, sum of w * (sum over the group's channels of grad_out
// * value) -- <grad_out, the anchor's feature in this view> -- for the
// fused form's score gradient.
// FULL: grad_weights and grad_sampling_loc wanted, no float-atomic grad_feat
// and no fusion dot product -- the common case, with those tests folded away.
template <class FT, int CPL, int LPG, int LPS, bool FULL = false>
__device__ __forceinline__ void bwd_chunk_w(const OpArgs& a, const StageSlot& st, int nj,
                                            const Geo* geo, const Lanes& q, const BwdAnchor& x0,
                                            const float* go, float out_scale, float* dot) {
    using RowT = Row<FT, CPL>;
    const int L = a.L, G = a.G, LG = L * G;
    const int lpg = (a.C / a.G) / CPL;             // lanes of one group (a power of two)
    BwdAnchor x = x0;
    if constexpr (FULL) {
        x.gacc = nullptr;
        dot = nullptr;
    }
    const bool need_vals = FULL || x.gwout || x.glout || dot;
    // byte offset of a row -> float offset in the FP32 accumulator
    constexpr int kOffToAcc = FT::kBytes == 4 ? 2 : FT::kBytes == 2 ? 1 : 0;
    for (int jj = q.sub; jj < nj; jj += q.spw) {
        const u32 src = st.src[jj];
        const float* wj = st.w + jj * LG + q.g;
        const Taps* tj = st.taps + jj * padded_levels(L);
        const float4* kj = st.dk + jj * padded_levels(L);
        float gx = 0.f, gy = 0.f;
        for (int l = 0; l < L; ++l) {
            const Taps t = tj[l];
            const float wl = wj[l * G];
            if (x.gacc) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (t.off[c] != kOOB) {
                        float* dst = x.gacc + (t.off[c] >> kOffToAcc);
                        const float cwl = t.cw[c] * wl;
#pragma unroll
                        for (int i = 0; i < CPL; ++i) unsafeAtomicAdd(dst + i, cwl * go[i]);
                    }
                }
            }
            if (!need_vals) continue;
            u32 raw[4][RowT::kWords];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                load_words<RowT::kWords>(x.feat, t.off[c] + q.lane_off, raw[c]);
            float d[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float f[CPL];
                widen<FT, CPL>(raw[c], f);
                float sum = 0.f;
#pragma unroll
                for (int i = 0; i < CPL; ++i) sum = fmaf(go[i], f[i], sum);
                d[c] = sum;
            }
            if (FULL || x.gwout || dot) {
                float tw = t.cw[0] * d[0] + t.cw[1] * d[1] + t.cw[2] * d[2] + t.cw[3] * d[3];
                tw = group_sum_w<LPG>(tw, lpg);
                if ((q.lane & (lpg - 1)) == 0) {
                    if (FULL || x.gwout) x.gwout[(size_t)src * LG + l * G + q.g] = tw * out_scale;
                    if (!FULL && dot) *dot = fmaf(wl, tw, *dot);
                }
            }
            // d val / dx = W ((1-ly)(F01 - F00) + ly (F11 - F10)) (x = u W - 0.5),
            // and d val / dy alike, the factors staged per sample
            const float4 k = kj[l];
            gx = fmaf(wl, k.x * (d[1] - d[0]) + k.y * (d[3] - d[2]), gx);
            gy = fmaf(wl, k.z * (d[2] - d[0]) + k.w * (d[3] - d[1]), gy);
        }
        if (FULL || x.glout) {
            gx = group_sum_w<LPS>(gx, q.lps);
            gy = group_sum_w<LPS>(gy, q.lps);
            if ((q.lane & (q.lps - 1)) == 0) {
                x.glout[(size_t)src * 2] = gx * out_scale;
                x.glout[(size_t)src * 2 + 1] = gy * out_scale;
            }
        }
    }
}

// The lane widths of the common layouts (C = 256 in G = 8 groups: 32 lanes
// per sample in groups of 4 with 8 channels per lane, 64 in groups of 8
// with 4) are compile-time in their copies of the loop; others take the
// run-time widths.
template <class FT, int CPL>
__device__ __forceinline__ void bwd_chunk(const OpArgs& a, const StageSlot& st, int nj,
                                          const Geo* geo, const Lanes& q, const BwdAnchor& x,
                                          const float* go, float out_scale = 1.f,
                                          float* dot = nullptr) {
    const int lpg = (a.C / a.G) / CPL;
    if (lpg == 4 && q.lps == 32 && x.gwout && x.glout && !x.gacc && !dot)
        bwd_chunk_w<FT, CPL, 4, 32, true>(a, st, nj, geo, q, x, go, out_scale, nullptr);
    else if (lpg == 4 && q.lps == 32)
        bwd_chunk_w<FT, CPL, 4, 32>(a, st, nj, geo, q, x, go, out_scale, dot);
    else if (lpg == 8 && q.lps == 64)
        bwd_chunk_w<FT, CPL, 8, 64>(a, st, nj, geo, q, x, go, out_scale, dot);
    else
        bwd_chunk_w<FT, CPL, 0, 0>(a, st, nj, geo, q, x, go, out_scale, dot);
}

}  // namespace msda
