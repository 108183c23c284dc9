// Fused weight generation: the per-group softmax that turns the weight
// logits into MSDA's weights (over the P*N*L (keypoint, camera, level)
// entries of each (batch item, anchor, group)), and its gradient.
//
// The forward never writes the weights: softmax_stats_kernel reduces each
// group's logits to (max, 1/sum of exp) and the gathers apply
// exp(logit - max) / sum while they stage the weights. The backward writes
// the FP32 weights once (weights_f32_kernel), runs the plain backward on
// them, and softmax_grad_kernel maps grad_weights to the logits' gradient
// in place: d logit = w * (d w - sum over the group of w * d w).
//
// Blocks of 256 threads over chunks of 4096 entries of one anchor. G is a
// power of two <= 64, so entry e of an anchor (groups fastest) belongs to
// group e % G and thread t sees only group t % G; partials are combined with
// the other threads of that group, then over the chunks, in a fixed order
// (bitwise reproducible).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float load_weight(const void* p, bool bf16, size_t i) {
    return bf16 ? __uint_as_float((uint32_t) static_cast<const uint16_t*>(p)[i] << 16)
                : static_cast<const float*>(p)[i];
}

// (max, sum of exp(x - max)) of two disjoint sets.
__device__ __forceinline__ float2 merge(float2 a, float2 b) {
    if (b.y == 0.f) return a;
    if (a.y == 0.f) return b;
    const float m = fmaxf(a.x, b.x);
    return make_float2(m, a.y * expf(a.x - m) + b.y * expf(b.x - m));
}

// Combines the values of the threads that share a group (t % G): within the
// wave by xor steps over the lane bits above log2(G), then the 4 waves in
// order through LDS. Returns the group's total in threads t < G.
template <class T, class F>
__device__ __forceinline__ T group_total(T v, int G, T* lds, F combine) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int m = G; m < 64; m <<= 1) {
        T o;
        if constexpr (sizeof(T) == 8) {
            o.x = __shfl_xor(v.x, m, 64);
            o.y = __shfl_xor(v.y, m, 64);
        } else {
            o = __shfl_xor(v, m, 64);
        }
        // the lower lane keeps its own value first: both lanes then agree
        v = (lane & m) ? combine(o, v) : combine(v, o);
    }
    if (lane < G) lds[wave * 64 + lane] = v;
    __syncthreads();
    T r = v;
    if (t < G) {
        r = lds[t];
        for (int w = 1; w < kThreads / 64; ++w) r = combine(r, lds[w * 64 + t]);
    }
    __syncthreads();
    return r;
}

// Work split: each anchor's n = P*N*L*G entries are cut into chunks of
// kChunk; block (chunk, anchor) handles one chunk, each thread kChunk/256
// entries of its group (independent loads, all in flight together).
constexpr int kChunk = 4096;

__host__ __device__ __forceinline__ int chunks_of(size_t n) { return (int)((n + kChunk - 1) / kChunk); }

// Per (anchor, chunk, group): (max, sum of exp(x - max)) of the chunk's logits.
__global__ void __launch_bounds__(kThreads) softmax_partial_kernel(const void* logits, int bf16,
                                                                   int PNL, int G,
                                                                   float2* part) {
    __shared__ float2 lds[kThreads];
    const size_t ba = blockIdx.y;
    const size_t n = (size_t)PNL * G;
    const int nch = chunks_of(n);
    const size_t e0 = (size_t)blockIdx.x * kChunk + threadIdx.x;
    float x[kChunk / kThreads];
#pragma unroll
    for (int k = 0; k < kChunk / kThreads; ++k) {
        const size_t e = e0 + (size_t)k * kThreads;
        x[k] = e < n ? load_weight(logits, bf16 != 0, ba * n + e) : -INFINITY;
    }
    float m = -INFINITY;
#pragma unroll
    for (int k = 0; k < kChunk / kThreads; ++k) m = fmaxf(m, x[k]);
    float sum = 0.f;
    if (m != -INFINITY) {
#pragma unroll
        for (int k = 0; k < kChunk / kThreads; ++k) sum += expf(x[k] - m);   // exp(-inf) = 0
    }
    const float2 tot = group_total(make_float2(m, sum), G, lds, merge);
    if ((int)threadIdx.x < G) part[(ba * nch + blockIdx.x) * G + threadIdx.x] = tot;
}

// stats[anchor][g] = (max, 1/sum) from the chunks' partials, in chunk order.
__global__ void __launch_bounds__(kThreads) softmax_merge_kernel(const float2* part, int BA,
                                                                 int nch, int G,
                                                                 float2* stats) {
    const size_t t = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (size_t)BA * G) return;
    const size_t ba = t / G, g = t % G;
    float2 acc = make_float2(-INFINITY, 0.f);
    for (int c = 0; c < nch; ++c) acc = merge(acc, part[(ba * nch + c) * G + g]);
    stats[t] = make_float2(acc.x, 1.f / acc.y);
}

// w = softmax weight (stats given) or the widened weight (stats nullptr).
__global__ void __launch_bounds__(kThreads) weights_f32_kernel(const void* src, int bf16,
                                                               const float2* stats, int PNL,
                                                               int G, float* w) {
    const size_t ba = blockIdx.y;
    const size_t n = (size_t)PNL * G;
    const size_t e0 = (size_t)blockIdx.x * kChunk + threadIdx.x;
    const float2 st = stats ? stats[ba * G + (threadIdx.x & (G - 1))] : make_float2(0.f, 1.f);
#pragma unroll
    for (int k = 0; k < kChunk / kThreads; ++k) {
        const size_t e = e0 + (size_t)k * kThreads;
        if (e < n) {
            float x = load_weight(src, bf16 != 0, ba * n + e);
            if (stats) x = expf(x - st.x) * st.y;
            w[ba * n + e] = x;
        }
    }
}

// Per (anchor, chunk, group): sum of w * grad over the chunk.
__global__ void __launch_bounds__(kThreads) softmax_dot_kernel(const float* w, const float* grad,
                                                               int PNL, int G, float* part) {
    __shared__ float lds[kThreads];
    const size_t ba = blockIdx.y;
    const size_t n = (size_t)PNL * G;
    const int nch = chunks_of(n);
    const size_t e0 = (size_t)blockIdx.x * kChunk + threadIdx.x;
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kChunk / kThreads; ++k) {
        const size_t e = e0 + (size_t)k * kThreads;
        if (e < n) acc = fmaf(w[ba * n + e], grad[ba * n + e], acc);
    }
    const float tot = group_total(acc, G, lds, [](float a, float b) { return a + b; });
    if ((int)threadIdx.x < G) part[(ba * nch + blockIdx.x) * G + threadIdx.x] = tot;
}

// dot[anchor][g] = the chunk partials' sum, in chunk order.
__global__ void __launch_bounds__(kThreads) softmax_dot_merge_kernel(const float* part, int BA,
                                                                     int nch, int G,
                                                                     float* dot) {
    const size_t t = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (size_t)BA * G) return;
    const size_t ba = t / G, g = t % G;
    float d = 0.f;
    for (int c = 0; c < nch; ++c) d += part[(ba * nch + c) * G + g];
    dot[t] = d;
}

// grad = w * (grad - D), D the group's sum of w * grad.
__global__ void __launch_bounds__(kThreads) softmax_apply_kernel(const float* w, float* grad,
                                                                 const float* dot, int PNL,
                                                                 int G) {
    const size_t ba = blockIdx.y;
    const size_t n = (size_t)PNL * G;
    const float d = dot[ba * G + (threadIdx.x & (G - 1))];
    const size_t e0 = (size_t)blockIdx.x * kChunk + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kChunk / kThreads; ++k) {
        const size_t e = e0 + (size_t)k * kThreads;
        if (e < n) grad[ba * n + e] = w[ba * n + e] * (grad[ba * n + e] - d);
    }
}

dim3 chunk_grid(int BA, int PNL, int G) {
    return dim3((unsigned)chunks_of((size_t)PNL * G), (unsigned)BA);
}

}  // namespace

size_t softmax_scratch_bytes(int BA, int PNL, int G) {
    // per-chunk partials, then (backward) the merged group sums
    return (size_t)BA * chunks_of((size_t)PNL * G) * G * sizeof(float2) +
           (size_t)BA * G * sizeof(float);
}

hipError_t launch_softmax_stats(const void* logits, bool bf16, int BA, int PNL, int G,
                                float2* part, float2* stats, hipStream_t s) {
    if (BA <= 0) return hipSuccess;
    mark_begin("softmax_partial", s);
    hipLaunchKernelGGL(softmax_partial_kernel, chunk_grid(BA, PNL, G), dim3(kThreads), 0, s,
                       logits, (int)bf16, PNL, G, part);
    mark_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nch = chunks_of((size_t)PNL * G);
    mark_begin("softmax_merge", s);
    hipLaunchKernelGGL(softmax_merge_kernel, dim3((unsigned)(((size_t)BA * G + kThreads - 1) /
                                                             kThreads)),
                       dim3(kThreads), 0, s, part, BA, nch, G, stats);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_weights_f32(const void* src, bool bf16, const float2* stats, int BA, int PNL,
                              int G, float* w, hipStream_t s) {
    if (BA <= 0) return hipSuccess;
    mark_begin("weights_f32", s);
    hipLaunchKernelGGL(weights_f32_kernel, chunk_grid(BA, PNL, G), dim3(kThreads), 0, s, src,
                       (int)bf16, stats, PNL, G, w);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_softmax_grad(const float* w, float* grad, int BA, int PNL, int G, float* part,
                               hipStream_t s) {
    if (BA <= 0) return hipSuccess;
    mark_begin("softmax_dot", s);
    hipLaunchKernelGGL(softmax_dot_kernel, chunk_grid(BA, PNL, G), dim3(kThreads), 0, s, w, grad,
                       PNL, G, part);
    mark_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nch = chunks_of((size_t)PNL * G);
    float* dot = part + (size_t)BA * nch * G * 2;      // after the float2-sized partials
    mark_begin("softmax_dot_merge", s);
    hipLaunchKernelGGL(softmax_dot_merge_kernel,
                       dim3((unsigned)(((size_t)BA * G + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, part, BA, nch, G, dot);
    mark_end(s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    mark_begin("softmax_apply", s);
    hipLaunchKernelGGL(softmax_apply_kernel, chunk_grid(BA, PNL, G), dim3(kThreads), 0, s, w,
                       grad, dot, PNL, G);
    mark_end(s);
    return hipGetLastError();
}

}  // namespace msda
