// Keypoint projection and the visible-view form of MSDA (paper Sec. 3.1,
// Sec. 3.2).
//
// project_keypoints_kernel: one thread per (batch item, anchor, camera)
// places the anchor's keypoints in the world -- box centre + yaw rotation
// of the box-frame offset scaled by (w, l, h) + velocity * dt (the motion
// compensation) -- projects them with the camera's 3x4 matrix, writes the
// normalised sampling locations (a point at or behind the camera gets a
// location outside every level) and whether any keypoint lands in the
// image: the anchor's visibility in that camera.
//
// Visible-view MSDA: only the (batch item, camera, anchor) items flagged
// visible are computed. The flags are compacted in view-major order (a scan
// of the flags gives each visible item its place), so consecutive items
// share a camera; the persistent gathers cut the item list into one range
// per XCD (as the view order does) and each wave takes one item at a time:
// the anchor's keypoints in that camera, all levels. The forward writes one
// partial row per item and fwd_visible_reduce adds an anchor's items in
// camera order; the backward writes grad_w / grad_loc of the visible pairs
// and one compacted grad_feat record per sample, which the sort and the
// tile reduction of the dense backward then consume.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_gather.h"

namespace msda {

constexpr float kDepthEps = 1e-5f;
constexpr float kBehind = -2.0f;   // a location outside every level

__global__ void __launch_bounds__(256) project_keypoints_kernel(ProjArgs p) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)p.B * p.A * p.N;
    if (t >= total) return;
    const int n = (int)(t % (size_t)p.N);
    const size_t ba = t / (size_t)p.N;                 // b * A + a
    const int b = (int)(ba / (size_t)p.A);
    const float* an = p.anchors + ba * 10;
    const float x = an[0], y = an[1], z = an[2], w = an[3], l = an[4], h = an[5];
    const float yaw = an[6];
    const float mx = p.dt * an[7], my = p.dt * an[8], mz = p.dt * an[9];
    float sy, cy;
    sincosf(yaw, &sy, &cy);
    const float* M = p.projection + ((size_t)b * p.N + n) * 12;
    const float W = (float)p.image_hw[2 * n + 1], H = (float)p.image_hw[2 * n];
    bool seen = false;
    for (int k = 0; k < p.P; ++k) {
        const float* kp = p.keypoints + (ba * p.P + k) * 3;
        const float ox = kp[0] * w, oy = kp[1] * l, oz = kp[2] * h;
        const float X = x + (cy * ox - sy * oy) + mx;
        const float Y = y + (sy * ox + cy * oy) + my;
        const float Z = z + oz + mz;
        const float u = M[0] * X + M[1] * Y + M[2] * Z + M[3];
        const float v = M[4] * X + M[5] * Y + M[6] * Z + M[7];
        const float d = M[8] * X + M[9] * Y + M[10] * Z + M[11];
        float lu = kBehind, lv = kBehind;
        if (d > kDepthEps) {
            const float px = u / d, py = v / d;
            lu = px / W;
            lv = py / H;
            seen |= px >= 0.f && px < W && py >= 0.f && py < H;
        }
        float* dst = p.loc + ((ba * p.P + k) * p.N + n) * 2;
        dst[0] = lu;
        dst[1] = lv;
    }
    p.visible[t] = seen ? 1 : 0;
}

hipError_t launch_project_keypoints(const ProjArgs& p, hipStream_t s) {
    const size_t total = (size_t)p.B * p.A * p.N;
    if (total == 0) return hipSuccess;
    mark_begin("project_keypoints", s);
    hipLaunchKernelGGL(project_keypoints_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, s, p);
    mark_end(s);
    return hipGetLastError();
}

// flags[v] = visible[b][a][n] for the view-major item v = (b*N + n)*A + a,
// and flags[V] = 0 (so that an exclusive scan leaves the count there).
__global__ void __launch_bounds__(256) visible_flags_kernel(const uint8_t* __restrict__ visible,
                                                            int B, int N, int A,
                                                            u32* __restrict__ flags) {
    const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t V = (size_t)B * N * A;
    if (v > V) return;
    if (v == V) {
        flags[V] = 0u;
        return;
    }
    const int a = (int)(v % (size_t)A);
    const size_t bn = v / (size_t)A;
    const int n = (int)(bn % (size_t)N), b = (int)(bn / (size_t)N);
    flags[v] = visible[((size_t)b * A + a) * N + n] ? 1u : 0u;
}

// items[place[v]] = v for every visible v (place = exclusive scan of flags);
// the thread past the end writes the record count, items * per_item.
__global__ void __launch_bounds__(256) visible_items_kernel(const uint8_t* __restrict__ visible,
                                                            const u32* __restrict__ place,
                                                            int B, int N, int A, u32 per_item,
                                                            u32* __restrict__ items,
                                                            u32* __restrict__ rec_count) {
    const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t V = (size_t)B * N * A;
    if (v > V) return;
    if (v == V) {
        if (rec_count) rec_count[0] = place[V] * per_item;
        return;
    }
    const int a = (int)(v % (size_t)A);
    const size_t bn = v / (size_t)A;
    const int n = (int)(bn % (size_t)N), b = (int)(bn / (size_t)N);
    if (visible[((size_t)b * A + a) * N + n]) items[place[v]] = (u32)v;
}

// Visibility-weighted fusion (Sec. 3.2, Eq. 2). One wave per (batch item,
// anchor); V = the sum of the scores of the anchor's visible cameras, added
// lane-strided then by a fixed butterfly (the same order in every pass).
__device__ __forceinline__ float wave_score_sum(const uint8_t* visible, const float* score,
                                                size_t o, int N, int lane) {
    float V = 0.f;
    for (int n = lane; n < N; n += 64)
        if (visible[o + n]) V += score[o + n];
    return group_sum(V, 64);
}

// vt[b][a][n] = score / V for visible cameras; 0 for the others, and for
// every camera when V <= 0.
__global__ void __launch_bounds__(256) view_scale_kernel(const uint8_t* __restrict__ visible,
                                                         const float* __restrict__ score,
                                                         int BA, int N, float* __restrict__ vt) {
    const int ba = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (ba >= BA) return;                     // whole waves
    const size_t o = (size_t)ba * N;
    const float V = wave_score_sum(visible, score, o, N, lane);
    for (int n = lane; n < N; n += 64)
        vt[o + n] = visible[o + n] && V > 0.f ? score[o + n] / V : 0.f;
}

// grad_score[b][a][n] = (<grad_out, g_n> - <grad_out, f>) / V for visible
// cameras (0 otherwise, and when V <= 0): g_n's product with grad_out comes
// from the backward gather (item_dot), f is the fused forward output.
__global__ void __launch_bounds__(256) grad_score_kernel(const float* __restrict__ grad_out,
                                                         const float* __restrict__ out,
                                                         const uint8_t* __restrict__ visible,
                                                         const float* __restrict__ score,
                                                         const u32* __restrict__ place,
                                                         const float* __restrict__ item_dot,
                                                         int B, int A, int N, int C,
                                                         float* __restrict__ grad_score) {
    const int ba = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (ba >= B * A) return;                  // whole waves
    const int b = ba / A, an = ba - b * A;
    const size_t o = (size_t)ba * N;
    const float V = wave_score_sum(visible, score, o, N, lane);
    float fdot = 0.f;
    for (int c = lane; c < C; c += 64)
        fdot = fmaf(grad_out[(size_t)ba * C + c], out[(size_t)ba * C + c], fdot);
    fdot = group_sum(fdot, 64);
    for (int n = lane; n < N; n += 64) {
        float gs = 0.f;
        if (visible[o + n] && V > 0.f) {
            const u32 i = place[((size_t)b * N + n) * A + an];
            gs = (item_dot[i] - fdot) / V;
        }
        grad_score[o + n] = gs;
    }
}

// The persistent walk over the visible items: workgroup w serves range
// w % kSlots of the item list; its waves take consecutive items, then move
// on by the slot's wave count. Calls f(item index, b, a, n) per item.
template <class F>
__device__ __forceinline__ void for_each_visible_item(const OpArgs& a, const u32* items,
                                                      const u32* count, F&& f) {
    const u32 nnz = uniform((int)*count);
    const int x = (int)(blockIdx.x % kSlots);
    const int wave = wave_index(), nwaves = blockDim.x >> 6;
    const u32 lo = (u32)(((u64)nnz * x) / kSlots), hi = (u32)(((u64)nnz * (x + 1)) / kSlots);
    const u32 per_slot = (gridDim.x / kSlots + (x < (int)(gridDim.x % kSlots) ? 1u : 0u));
    const u32 stride = per_slot * (u32)nwaves;
    for (u32 r = (blockIdx.x / kSlots) * (u32)nwaves + (u32)wave; lo + r < hi; r += stride) {
        const u32 i = lo + r;
        const u32 v = uniform((int)items[i]);
        const int an = (int)(v % (u32)a.A);
        const u32 bn = v / (u32)a.A;
        f(i, (int)(bn / (u32)a.N), an, (int)(bn % (u32)a.N));
    }
}

template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_visible_kernel(OpArgs a, const u32* items,
                                                               const u32* count, float* part) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)a.N * a.L * sizeof(Geo);
    stage_geometry(geo, a);
    __syncthreads();                       // the only block-wide barrier

    const int LG = a.L * a.G;
    const int J = a.pairs_per_chunk;
    const Lanes q = lanes_of<FT, CPL>(a);
    const StageSlot st = stage_slot(work, wave_index(), J, a.L, a.G);
    const u32 row_bytes = (u32)a.C * FT::kBytes;
    const int npairs = a.P * a.N;
    const RecordSink none{};
    for_each_visible_item(a, items, count, [&](u32 i, int b, int an, int n) {
        const int ba = b * a.A + an;
        const float* gl = a.loc + (size_t)ba * npairs * 2;
        const WSrc gw = anchor_weights(a, (size_t)ba, (size_t)npairs * LG);
        const rsrc_t feat = make_rsrc(static_cast<const char*>(a.feat) + (size_t)b * a.batch_bytes,
                                      a.batch_bytes);
        const ViewOrder order{a.N, a.P, n};
        float acc[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = 0.f;
        for (int k0 = 0; k0 < a.P; k0 += J) {
            const int nj = min(J, a.P - k0);
            stage_chunk<FT::kBytes == 1, false>(st, order, k0, nj, gw, gl, geo, a.L, LG,
                                                row_bytes, q.lane, none);
            fwd_chunk<FT, CPL>(st, nj, a.L, a.G, q, feat, acc);
            end_chunk();
        }
        reduce_subwaves<CPL>(q, acc);
        if (q.sub == 0) {
            float* dst = part + (size_t)i * a.C + q.c0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) dst[c] = acc[c];
        }
    });
}

// out[b, a, :] = sum over the anchor's visible cameras, in camera order, of
// the items' partial rows, each times vt (the fused form's per-view weight)
// when vt is given; zero when no camera sees the anchor. One wave per
// anchor, 4 channels per lane per pass: a ballot of the visibility flags
// of 64 cameras, then the items' rows 4 at a time (loads in flight
// together, added in camera order).
__global__ void __launch_bounds__(256) fwd_visible_reduce(const float* __restrict__ part,
                                                          const uint8_t* __restrict__ visible,
                                                          const u32* __restrict__ place,
                                                          const float* __restrict__ vt, int B,
                                                          int N, int A, int C,
                                                          float* __restrict__ out) {
    const int ba = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (ba >= B * A) return;                  // whole waves
    const int b = ba / A, an = ba - b * A;
    const size_t o = (size_t)ba * N;
    for (int c0 = 0; c0 < C; c0 += 256) {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int n0 = 0; n0 < N; n0 += 64) {
            const int n = n0 + lane;
            const bool f = n < N && visible[o + n];
            const u32 pl = f ? place[((size_t)b * N + n) * A + an] : 0u;
            const float sc = f && vt ? vt[o + n] : 1.f;
            uint64_t mask = __ballot(f);
            while (mask) {
                int k[4];
                int m = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    k[q] = mask ? __builtin_ctzll(mask) : 0;
                    if (mask) { mask &= mask - 1; ++m; }
                }
                float g[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const u32 i = (u32)__shfl((int)pl, k[q], 64);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int c = c0 + lane + 64 * j;
                        g[q][j] = q < m && c < C ? part[(size_t)i * C + c] : 0.f;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q >= m) break;
                    const float w = __shfl(sc, k[q], 64);
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[j] = vt ? fmaf(w, g[q][j], acc[j]) : acc[j] + g[q][j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = c0 + lane + 64 * j;
            if (c < C) out[(size_t)ba * C + c] = acc[j];
        }
    }
}

template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_bwd_visible_kernel(OpArgs a, const u32* items,
                                                               const u32* place,
                                                               const u32* count,
                                                               u32* rec_val, const float* vt,
                                                               float* item_dot) {
    extern __shared__ __align__(16) unsigned char smem[];
    Geo* geo = reinterpret_cast<Geo*>(smem);
    unsigned char* work = smem + (size_t)a.N * a.L * sizeof(Geo);
    stage_geometry(geo, a);
    __syncthreads();                       // the only block-wide barrier

    const int J = a.pairs_per_chunk;
    const Lanes q = lanes_of<FT, CPL>(a);
    const StageSlot st = stage_slot(work, wave_index(), J, a.L, a.G);
    for_each_visible_item(a, items, count, [&](u32 i, int b, int an, int n) {
        float go[CPL];
        BwdAnchor x = bwd_anchor_ctx<FT, CPL>(a, b * a.A + an, q, go);
        if (a.rec_bucket_ap) {
            // records per (b, n, l) bucket (launch_bucket_sort's visible-view
            // layout): the cnt visible anchors of (b, n) from item s0 on,
            // level-major; stage_chunk adds (n*L + l)*bucket_ap + p, so the
            // base drops n*L*bucket_ap (modulo 2^32)
            const u32 bn = (u32)(b * a.N + n), P = (u32)a.P, L = (u32)a.L;
            const u32 s0 = place[(size_t)bn * a.A];
            x.rec.bucket_ap = (place[(size_t)(bn + 1) * a.A] - s0) * P;
            x.rec.bucket_base = s0 * P * L + (i - s0) * P - (u32)n * L * x.rec.bucket_ap;
            x.rec.val = nullptr;
        } else {
            x.rec.val = rec_val;
            x.rec.cbase = i * (u32)(a.P * a.L);
        }
        const ViewOrder order{a.N, a.P, n};
        const float scale = vt ? vt[((size_t)b * a.A + an) * a.N + n] : 1.f;
        float dot = 0.f;
        for (int k0 = 0; k0 < a.P; k0 += J) {
            const int nj = min(J, a.P - k0);
            stage_chunk<false, true>(st, order, k0, nj, x.gw, x.gl, geo, a.L, a.L * a.G,
                                     (u32)a.C * FT::kBytes, q.lane, x.rec);
            bwd_chunk<FT, CPL>(a, st, nj, geo, q, x, go, scale, item_dot ? &dot : nullptr);
            end_chunk();
        }
        if (item_dot) {
            dot = group_sum(dot, 64);
            if (q.lane == 0) item_dot[i] = dot;
        }
    });
}

// Persistent grids: 16 workgroups of `waves` waves per CU's worth of slots,
// rounded to whole slots.
static unsigned visible_blocks(int waves) {
    const unsigned per_cu = 16u / (unsigned)waves > 0 ? 16u / (unsigned)waves : 1u;
    return 256u * per_cu / kSlots * kSlots;
}

template <class FT, int CPL>
static hipError_t fwd_visible_launch(const OpArgs& a, int waves, size_t lds, const u32* items,
                                     const u32* count, const u32* place, const uint8_t* visible,
                                     const float* vt, float* part, hipStream_t s) {
    mark_begin("msda_fwd_visible_kernel", s);
    hipLaunchKernelGGL((msda_fwd_visible_kernel<FT, CPL>), dim3(visible_blocks(waves)),
                       dim3(64 * waves), lds, s, a, items, count, part);
    mark_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t anchors = (size_t)a.B * a.A;
    mark_begin("fwd_visible_reduce", s);
    hipLaunchKernelGGL(fwd_visible_reduce, dim3((unsigned)((anchors + 3) / 4)), dim3(256), 0, s,
                       part, visible, place, vt, a.B, a.N, a.A, a.C, a.out);
    mark_end(s);
    return hipGetLastError();
}

template <class FT, int CPL>
static hipError_t bwd_visible_launch(const OpArgs& a, int waves, size_t lds, const u32* items,
                                     const u32* place, const u32* count, u32* rec_val,
                                     const float* vt, float* item_dot, hipStream_t s) {
    mark_begin("msda_bwd_visible_kernel", s);
    hipLaunchKernelGGL((msda_bwd_visible_kernel<FT, CPL>), dim3(visible_blocks(waves)),
                       dim3(64 * waves), lds, s, a, items, place, count, rec_val, vt, item_dot);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_visible_items(const uint8_t* visible, int B, int N, int A, u32 per_item,
                                u32* place, u32* items, u32* rec_count, u32* scan_partial,
                                hipStream_t s) {
    const size_t V = (size_t)B * N * A;
    mark_begin("visible_flags", s);
    hipLaunchKernelGGL(visible_flags_kernel, dim3((unsigned)((V + 1 + 255) / 256)), dim3(256), 0,
                       s, visible, B, N, A, place);
    mark_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_exclusive_scan(place, (u32)(V + 1), scan_partial, s)) != hipSuccess) return e;
    mark_begin("visible_items", s);
    hipLaunchKernelGGL(visible_items_kernel, dim3((unsigned)((V + 1 + 255) / 256)), dim3(256), 0,
                       s, visible, place, B, N, A, per_item, items, rec_count);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_forward_visible(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                                  const u32* items, const u32* count, const u32* place,
                                  const uint8_t* visible, const float* vt, float* part,
                                  hipStream_t s) {
    switch (dtype * 100 + cpl) {
#define MSDA_CASE(D, T, K) \
        case D * 100 + K: \
            return fwd_visible_launch<T, K>(a, waves, lds, items, count, place, visible, vt, \
                                            part, s);
        MSDA_CASE(kF32, TF32, 1) MSDA_CASE(kF32, TF32, 2) MSDA_CASE(kF32, TF32, 4)
        MSDA_CASE(kBF16, TBF16, 2) MSDA_CASE(kBF16, TBF16, 4) MSDA_CASE(kBF16, TBF16, 8)
        MSDA_CASE(kF16, TF16, 2) MSDA_CASE(kF16, TF16, 4) MSDA_CASE(kF16, TF16, 8)
        MSDA_CASE(kFP8, TFP8, 4) MSDA_CASE(kFP8, TFP8, 8) MSDA_CASE(kFP8, TFP8, 16)
#undef MSDA_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward_visible(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                                   const u32* items, const u32* place, const u32* count,
                                   u32* rec_val, const float* vt, float* item_dot, hipStream_t s) {
    switch (dtype * 100 + cpl) {
#define MSDA_CASE(D, T, K) \
        case D * 100 + K: \
            return bwd_visible_launch<T, K>(a, waves, lds, items, place, count, rec_val, vt, \
                                            item_dot, s);
        MSDA_CASE(kF32, TF32, 1) MSDA_CASE(kF32, TF32, 2) MSDA_CASE(kF32, TF32, 4)
        MSDA_CASE(kBF16, TBF16, 2) MSDA_CASE(kBF16, TBF16, 4) MSDA_CASE(kBF16, TBF16, 8)
        MSDA_CASE(kF16, TF16, 2) MSDA_CASE(kF16, TF16, 4) MSDA_CASE(kF16, TF16, 8)
#undef MSDA_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_view_scale(const uint8_t* visible, const float* score, int BA, int N,
                             float* vt, hipStream_t s) {
    if (BA <= 0) return hipSuccess;
    mark_begin("view_scale", s);
    hipLaunchKernelGGL(view_scale_kernel, dim3((unsigned)((BA + 3) / 4)), dim3(256), 0, s,
                       visible, score, BA, N, vt);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_grad_score(const float* grad_out, const float* out, const uint8_t* visible,
                             const float* score, const u32* place, const float* item_dot, int B,
                             int A, int N, int C, float* grad_score, hipStream_t s) {
    if (B * A <= 0) return hipSuccess;
    mark_begin("grad_score", s);
    hipLaunchKernelGGL(grad_score_kernel, dim3((unsigned)((B * A + 3) / 4)), dim3(256), 0, s,
                       grad_out, out, visible, score, place, item_dot, B, A, N, C, grad_score);
    mark_end(s);
    return hipGetLastError();
}

}  // namespace msda
