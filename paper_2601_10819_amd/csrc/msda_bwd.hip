// Backward of multi-scale deformable aggregation: gradients of <grad_out, out>
// with respect to the sampling locations, the weights and the features.
//
// msda_bwd_kernel (one workgroup per (batch item, anchor), the forward's lane
// layout) re-gathers the 4 corner rows of each sample and forms, per lane,
// d[c] = <grad_out, corner c> over its channels. Then
//   grad_w[g]  = sum over the group's lanes of sum_c cw[c] * d[c]
//                (a shuffle reduction within the group's lanes),
//   grad_loc   = sum over levels of W (H) * w * (d/dx (d/dy) of the bilinear
//                blend of d), reduced over the sample's lanes once per
//                (keypoint, camera) pair.
// For grad_feat it either emits one record per (sample, corner) -- the row
// touched and the corner weight, at a fixed position 4*sample + corner --
// for the sorted per-row reduction below (deterministic, no float atomics),
// or adds w * cw * grad_out to an FP32 accumulator with float atomics.
//
// gfeat_reduce_kernel: after the records are sorted by row (msda_sort.hip),
// one group of lanes per feature row sums cw * w[g] * grad_out[anchor] over
// the row's records in sample order and writes the row once, in FP32 or
// BF16 (rounded to nearest even), zeros for rows no sample touches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_bwd_kernel(OpArgs a) {
    using RowT = Row<FT, CPL>;
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    float* work = reinterpret_cast<float*>(smem + (size_t)a.N * a.L * sizeof(Geo));
    stage_geometry(geo, a);
    __syncthreads();

    const int LG = a.L * a.G;
    const int J = a.pairs_per_chunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    float* sw = work + wave * J * (LG + 2);
    float* sl = sw + J * LG;

    const int ba = blockIdx.x;
    const int b = ba / a.A;
    const int npairs = a.P * a.N;
    const float* gl = a.loc + (size_t)ba * npairs * 2;
    const float* gw = a.w + (size_t)ba * npairs * LG;

    const int lps = 1 << a.lps_shift;
    const int spw = 64 >> a.lps_shift;
    const int sub = lane >> a.lps_shift;
    const int sl_lane = lane & (lps - 1);          // lane within the sample
    const int c0 = sl_lane * CPL;
    const int cpg = a.C / a.G;
    const int g = c0 / cpg;
    const int lpg = cpg / CPL;                     // lanes of one group (a power of two)
    const u32 row_bytes = (u32)a.C * FT::kBytes;
    const u32 lane_off = (u32)c0 * FT::kBytes;
    const rsrc_t feat = make_rsrc(static_cast<const char*>(a.feat) + (size_t)b * a.batch_bytes,
                                  a.batch_bytes);

    float go[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) go[i] = a.grad_out[(size_t)ba * a.C + c0 + i];
    float* gacc = a.gfeat_acc ? a.gfeat_acc + (size_t)b * a.R * a.C + c0 : nullptr;
    float* gwout = a.grad_w ? a.grad_w + (size_t)ba * npairs * LG : nullptr;
    float* glout = a.grad_loc ? a.grad_loc + (size_t)ba * npairs * 2 : nullptr;
    const bool need_vals = gwout || glout;
    const u32 row_base = (u32)b * (u32)a.R;        // first global row of this batch item
    const u32 no_row = (u32)a.B * (u32)a.R;        // key of a corner outside its level

    const int nchunks = (npairs + J - 1) / J;
    for (int k = wave; k < nchunks; k += nwaves) {
        const int j0 = k * J;
        const int nj = min(J, npairs - j0);
        stage_chunk(sw, sl, gw + (size_t)j0 * LG, gl + (size_t)j0 * 2, nj, LG, lane);
        for (int jj = sub; jj < nj; jj += spw) {
            const int j = j0 + jj;
            const int n = j % a.N;
            const float u = sl[2 * jj], v = sl[2 * jj + 1];
            const float* wj = sw + jj * LG + g;
            float gx = 0.f, gy = 0.f;
            for (int l = 0; l < a.L; ++l) {
                const Geo gm = geo[n * a.L + l];
                const Corners cr = corners_of(u, v, gm, row_bytes, lane_off);
                const float wl = wj[l * a.G];
                if (a.rec_key) {
                    // records of this sample's 4 corners, written by its first lanes
                    const u32 s4 = ((u32)(ba * npairs + j) * (u32)a.L + (u32)l) * 4u;
                    for (int q = sl_lane; q < 4; q += lps) {
                        const int row = q == 0 ? cr.row[0] : q == 1 ? cr.row[1]
                                      : q == 2 ? cr.row[2] : cr.row[3];
                        const float cw = q == 0 ? cr.cw[0] : q == 1 ? cr.cw[1]
                                       : q == 2 ? cr.cw[2] : cr.cw[3];
                        a.rec_key[s4 + q] = row >= 0 ? row_base + (u32)row : no_row;
                        a.rec_cw[s4 + q] = cw;
                    }
                }
                if (gacc) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (cr.row[c] >= 0) {
                            float* dst = gacc + (size_t)cr.row[c] * a.C;
                            const float cwl = cr.cw[c] * wl;
#pragma unroll
                            for (int i = 0; i < CPL; ++i) unsafeAtomicAdd(dst + i, cwl * go[i]);
                        }
                    }
                }
                if (!need_vals) continue;
                u32 raw[4][RowT::kWords];
#pragma unroll
                for (int c = 0; c < 4; ++c) load_words<RowT::kWords>(feat, cr.off[c], raw[c]);
                // d[c] = <grad_out, corner c> over this lane's channels
                float d[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float f[CPL];
                    widen<FT, CPL>(raw[c], f);
                    float s = 0.f;
#pragma unroll
                    for (int i = 0; i < CPL; ++i) s = fmaf(go[i], f[i], s);
                    d[c] = s;
                }
                if (gwout) {
                    float t = cr.cw[0] * d[0] + cr.cw[1] * d[1] + cr.cw[2] * d[2] +
                              cr.cw[3] * d[3];
                    for (int s = 1; s < lpg; s <<= 1) t += xor_shuffle(t, s);
                    if ((lane & (lpg - 1)) == 0) gwout[(size_t)j * LG + l * a.G + g] = t;
                }
                // d val / dx = hy (F01 - F00) + ly (F11 - F10); x = u W - 0.5
                const float hx = 1.f - cr.lx, hy = 1.f - cr.ly;
                gx += (float)gm.W * wl * (hy * (d[1] - d[0]) + cr.ly * (d[3] - d[2]));
                gy += (float)gm.H * wl * (hx * (d[2] - d[0]) + cr.lx * (d[3] - d[1]));
            }
            if (glout) {
                for (int s = 1; s < lps; s <<= 1) {
                    gx += xor_shuffle(gx, s);
                    gy += xor_shuffle(gy, s);
                }
                if (sl_lane == 0) {
                    glout[(size_t)j * 2] = gx;
                    glout[(size_t)j * 2 + 1] = gy;
                }
            }
        }
        end_chunk();
    }
}

template <class OT, int CPL>
__device__ __forceinline__ void store_row(void* base, size_t elem, const float* acc) {
    if constexpr (OT::kBytes == 4) {
        float* p = static_cast<float*>(base) + elem;
        if constexpr (CPL == 4) {
            *reinterpret_cast<float4*>(p) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        } else {
#pragma unroll
            for (int i = 0; i < CPL; ++i) p[i] = acc[i];
        }
    } else {
        uint16_t* p = static_cast<uint16_t*>(base) + elem;
        if constexpr (CPL == 4) {
            const u32 lo = (u32)bf16_rne(acc[0]) | ((u32)bf16_rne(acc[1]) << 16);
            const u32 hi = (u32)bf16_rne(acc[2]) | ((u32)bf16_rne(acc[3]) << 16);
            *reinterpret_cast<u32x2*>(p) = u32x2{lo, hi};
        } else {
#pragma unroll
            for (int i = 0; i < CPL; ++i) p[i] = bf16_rne(acc[i]);
        }
    }
}

template <int CPL>
__device__ __forceinline__ void load_go(const float* p, float* v) {
    if constexpr (CPL == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
#pragma unroll
        for (int i = 0; i < CPL; ++i) v[i] = p[i];
    }
}

template <class OT, int CPL>
__global__ void __launch_bounds__(256) gfeat_reduce_kernel(ReduceArgs r) {
    const int lane = threadIdx.x & 63;
    const int lps = 1 << r.lps_shift;
    const u32 row = blockIdx.x * (blockDim.x >> r.lps_shift) + (threadIdx.x >> r.lps_shift);
    if (row >= r.nrows) return;
    const int c0 = (lane & (lps - 1)) * CPL;
    const int g = c0 / (r.C / r.G);
    // offsets and indices are checked so that an inconsistent sort could only
    // give wrong sums, never an access outside the workspace
    const u32 e1 = min(r.off[row + 1], r.nrec);
    const u32 e0 = min(r.off[row], e1);
    float acc[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[i] = 0.f;
    u32 e = e0;
    // four records at a time: their loads are issued before the sums
    for (; e + 4 <= e1; e += 4) {
        u32 idx[4];
        float coef[4], gv[4][CPL];
#pragma unroll
        for (int q = 0; q < 4; ++q) idx[q] = min(r.vals[e + q], r.nrec - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32 s = idx[q] >> 2;
            coef[q] = r.rec_cw[idx[q]] * r.w[(size_t)s * r.G + g];
            const u32 anchor = fast_div(s, r.magic, r.magic_shift);
            load_go<CPL>(r.grad_out + (size_t)anchor * r.C + c0, gv[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[i] = fmaf(coef[q], gv[q][i], acc[i]);
        }
    }
    for (; e < e1; ++e) {
        const u32 idx = min(r.vals[e], r.nrec - 1);
        const u32 s = idx >> 2;
        const float coef = r.rec_cw[idx] * r.w[(size_t)s * r.G + g];
        const u32 anchor = fast_div(s, r.magic, r.magic_shift);
        float gv[CPL];
        load_go<CPL>(r.grad_out + (size_t)anchor * r.C + c0, gv);
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[i] = fmaf(coef, gv[i], acc[i]);
    }
    store_row<OT, CPL>(r.grad_feat, (size_t)row * r.C + c0, acc);
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
        case kBF16 * 100 + 4: return bwd_launch<TBF16, 4>(a, waves, lds, s);
        case kBF16 * 100 + 8: return bwd_launch<TBF16, 8>(a, waves, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <class OT, int CPL>
static hipError_t reduce_launch(const ReduceArgs& r, hipStream_t s) {
    const u32 rows_per_block = 256u >> r.lps_shift;
    const u32 blocks = (r.nrows + rows_per_block - 1) / rows_per_block;
    if (blocks == 0) return hipSuccess;
    mark_begin("gfeat_reduce_kernel", s);
    hipLaunchKernelGGL((gfeat_reduce_kernel<OT, CPL>), dim3(blocks), dim3(256), 0, s, r);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_gfeat_reduce(const ReduceArgs& r, int out_dtype, int cpl, hipStream_t s) {
    switch (out_dtype * 100 + cpl) {
        case kF32 * 100 + 1: return reduce_launch<TF32, 1>(r, s);
        case kF32 * 100 + 2: return reduce_launch<TF32, 2>(r, s);
        case kF32 * 100 + 4: return reduce_launch<TF32, 4>(r, s);
        case kBF16 * 100 + 1: return reduce_launch<TBF16, 1>(r, s);
        case kBF16 * 100 + 2: return reduce_launch<TBF16, 2>(r, s);
        case kBF16 * 100 + 4: return reduce_launch<TBF16, 4>(r, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace msda
