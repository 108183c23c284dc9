// Helper kernels: zero fill, FP32 -> BF16 rounding, the per-level FP8
// quantiser (amax, scale, encode) and the streaming-copy reference kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_common.h"

namespace msda {

// Zero `bytes` bytes at a 4-byte aligned p (16-byte stores, then the tail).
__global__ void fill_zero_kernel(unsigned char* p, size_t bytes) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t head = (16 - ((uintptr_t)p & 15)) & 15;   // bytes before 16-byte alignment
    const size_t pre = head < bytes ? head : bytes;
    const size_t n16 = (bytes - pre) / 16;
    u32x4* p4 = reinterpret_cast<u32x4*>(p + pre);
    for (size_t k = i; k < n16; k += stride) p4[k] = u32x4{0u, 0u, 0u, 0u};
    for (size_t k = i; k < pre; k += stride) p[k] = 0;
    for (size_t k = pre + n16 * 16 + i; k < bytes; k += stride) p[k] = 0;
}

__global__ void f32_to_bf16_kernel(const float* src, uint16_t* dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = bf16_rne(src[k]);
}

__global__ void f32_to_f16_kernel(const float* src, uint16_t* dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = f16_rne(src[k]);
}

// --- FP8 per-level quantisation: amax, scale, encode.

// Grid (Y, N*L, B): block (y, region, b) streams the y-th contiguous chunk
// of kQuantChunk float4 of its region (the host sizes Y for the largest
// region; blocks past a smaller region's end do nothing). Consecutive blocks
// take consecutive chunks, so the blocks in flight read a few contiguous
// spans, as a streaming copy does. VEC:
// C % 4 == 0 and x 16-byte aligned, so every region starts on a float4 and
// holds a whole number of them.
constexpr int kQuantThreads = 256;
constexpr int kQuantUnroll = 16;                          // float4 loads in flight per thread
constexpr int kQuantChunk = kQuantThreads * kQuantUnroll; // float4 per block (64 KiB)

// The largest |x| of each (batch item, region): per thread over float4
// loads, then the block's maximum (wave butterfly, then across the 4 waves in
// LDS) and one atomicMax of its bits per block into the region's own slot
// (non-negative floats order like their bit patterns), so that no more than
// Y blocks meet at one address.
template <bool VEC>
__global__ void __launch_bounds__(kQuantThreads) amax_kernel(const float* x, const int32_t* shapes,
                                                             const int32_t* starts, int N, int L,
                                                             int64_t R, int C, u32* amax) {
    __shared__ float wmax[kQuantThreads / 64];
    const int region = blockIdx.y;
    const int b = blockIdx.z;
    const int64_t rows = (int64_t)shapes[2 * region] * shapes[2 * region + 1];
    const size_t base = ((size_t)b * R + starts[region]) * C;
    const size_t n = (size_t)rows * C;
    float m = 0.f;
    if constexpr (VEC) {
        const float4* p = reinterpret_cast<const float4*>(x + base);
        const size_t lo = (size_t)blockIdx.x * kQuantChunk;
        const size_t hi = min(lo + (size_t)kQuantChunk, n / 4);
        size_t k = lo + threadIdx.x;
        for (; k + (kQuantUnroll - 1) * kQuantThreads < hi; k += kQuantUnroll * kQuantThreads) {
            float4 t[kQuantUnroll];
#pragma unroll
            for (int u = 0; u < kQuantUnroll; ++u) t[u] = p[k + u * kQuantThreads];
#pragma unroll
            for (int u = 0; u < kQuantUnroll; ++u)
                m = fmaxf(m, fmaxf(fmaxf(fabsf(t[u].x), fabsf(t[u].y)),
                                   fmaxf(fabsf(t[u].z), fabsf(t[u].w))));
        }
        for (; k < hi; k += kQuantThreads) {
            const float4 t = p[k];
            m = fmaxf(m, fmaxf(fmaxf(fabsf(t.x), fabsf(t.y)), fmaxf(fabsf(t.z), fabsf(t.w))));
        }
    } else {
        const size_t lo = (size_t)blockIdx.x * kQuantChunk * 4;
        const size_t hi = min(lo + (size_t)kQuantChunk * 4, n);
        for (size_t k = lo + threadIdx.x; k < hi; k += kQuantThreads)
            m = fmaxf(m, fabsf(x[base + k]));
    }
    for (int s = 32; s > 0; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float bm = wmax[0];
        for (int w = 1; w < kQuantThreads / 64; ++w) bm = fmaxf(bm, wmax[w]);
        if (bm > 0.f) atomicMax(&amax[(size_t)b * N * L + region], __float_as_uint(bm));
    }
}

// scale[l] = (max over the (batch item, camera) slots of level l) / 448,
// 1 for an all-zero level. One block; wave l % 4 serves level l.
__global__ void __launch_bounds__(256) scale_kernel(const u32* amax, float* scale, int BN, int L) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int l = wave; l < L; l += 4) {
        u32 m = 0u;
        for (int i = lane; i < BN; i += 64) m = max(m, amax[(size_t)i * L + l]);
        for (int s = 32; s > 0; s >>= 1) m = max(m, (u32)__shfl_xor((int)m, s, 64));
        if (lane == 0) {
            const float f = __uint_as_float(m);
            scale[l] = f > 0.f ? f / 448.f : 1.f;
        }
    }
}

// The codes of two values: IEEE division by the level's scale, clamp to
// the format's range (+-448), then gfx950's converter to OCP e4m3 (round to
// nearest even), written to byte pair HI of `old`.
template <bool HI>
__device__ __forceinline__ u32 quant_two(float x0, float x1, float s, u32 old) {
    const float q0 = fminf(fmaxf(x0 / s, -448.f), 448.f);
    const float q1 = fminf(fmaxf(x1 / s, -448.f), 448.f);
    return (u32)__builtin_amdgcn_cvt_pk_fp8_f32(q0, q1, (int)old, HI);
}

__device__ __forceinline__ u32 quant_four(float4 t, float s) {
    return quant_two<true>(t.z, t.w, s, quant_two<false>(t.x, t.y, s, 0u));
}

// Same grid as amax_kernel. VEC: each float4 becomes 4 codes stored as one
// 32-bit word (the region's codes start on a multiple of 4 bytes).
template <bool VEC>
__global__ void __launch_bounds__(kQuantThreads) quantize_kernel(
    const float* x, const int32_t* shapes, const int32_t* starts, int N, int L, int64_t R, int C,
    const float* scale, uint8_t* codes) {
    const int region = blockIdx.y;
    const int b = blockIdx.z;
    const int l = region % L;
    const int64_t rows = (int64_t)shapes[2 * region] * shapes[2 * region + 1];
    const size_t off = ((size_t)b * R + starts[region]) * C;
    const size_t n = (size_t)rows * C;
    const float s = scale[l];
    if constexpr (VEC) {
        const float4* p = reinterpret_cast<const float4*>(x + off);
        u32* q = reinterpret_cast<u32*>(codes + off);
        const size_t lo = (size_t)blockIdx.x * kQuantChunk;
        const size_t hi = min(lo + (size_t)kQuantChunk, n / 4);
        size_t k = lo + threadIdx.x;
        for (; k + (kQuantUnroll - 1) * kQuantThreads < hi; k += kQuantUnroll * kQuantThreads) {
            float4 t[kQuantUnroll];
#pragma unroll
            for (int u = 0; u < kQuantUnroll; ++u) t[u] = p[k + u * kQuantThreads];
#pragma unroll
            for (int u = 0; u < kQuantUnroll; ++u) q[k + u * kQuantThreads] = quant_four(t[u], s);
        }
        for (; k < hi; k += kQuantThreads) q[k] = quant_four(p[k], s);
    } else {
        const size_t lo = (size_t)blockIdx.x * kQuantChunk * 4;
        const size_t hi = min(lo + (size_t)kQuantChunk * 4, n);
        for (size_t k = lo + threadIdx.x; k < hi; k += kQuantThreads)
            codes[off + k] = (uint8_t)(quant_two<false>(x[off + k], 0.f, s, 0u) & 0xffu);
    }
}

__global__ void stream_copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                   size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = src[k];
}

static unsigned grid_for(size_t n, unsigned block, unsigned cap) {
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    mark_begin("fill_zero", s);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(bytes / 16 + 1, 256, 8192)), dim3(256), 0,
                       s, static_cast<unsigned char*>(p), bytes);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    mark_begin("f32_to_bf16", s);
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, src,
                       dst, n);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_f32_to_f16(const float* src, uint16_t* dst, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    mark_begin("f32_to_f16", s);
    hipLaunchKernelGGL(f32_to_f16_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, src,
                       dst, n);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_quantize_fp8(const float* x, const int32_t* shapes, const int32_t* starts,
                               int32_t B, int32_t N, int32_t L, int64_t R, int32_t C,
                               int64_t max_region_rows, uint8_t* codes, float* level_scale,
                               uint32_t* amax_ws, hipStream_t s) {
    hipError_t e = launch_fill_zero(amax_ws, (size_t)B * N * L * 4, s);
    if (e != hipSuccess) return e;
    const bool vec = C % 4 == 0 && ((uintptr_t)x & 15) == 0;
    // blocks per region: chunks of kQuantChunk float4 (or 4 * kQuantChunk
    // floats) of the largest region
    const size_t most = (size_t)max_region_rows * (size_t)C;
    const size_t per = (size_t)kQuantChunk * 4;
    const size_t y = (most + per - 1) / per;   // < 2^16: a batch item is under 4 GiB
    const dim3 grid((unsigned)(y < 1 ? 1 : y), (unsigned)(N * L), (unsigned)B);
    mark_begin("fp8_amax", s);
    if (vec)
        hipLaunchKernelGGL(amax_kernel<true>, grid, dim3(kQuantThreads), 0, s, x, shapes, starts, N,
                           L, R, C, amax_ws);
    else
        hipLaunchKernelGGL(amax_kernel<false>, grid, dim3(kQuantThreads), 0, s, x, shapes, starts,
                           N, L, R, C, amax_ws);
    mark_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark_begin("fp8_scale", s);
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(256), 0, s, amax_ws, level_scale, B * N, L);
    mark_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark_begin("fp8_quantize", s);
    if (vec)
        hipLaunchKernelGGL(quantize_kernel<true>, grid, dim3(kQuantThreads), 0, s, x, shapes,
                           starts, N, L, R, C, level_scale, codes);
    else
        hipLaunchKernelGGL(quantize_kernel<false>, grid, dim3(kQuantThreads), 0, s, x, shapes,
                           starts, N, L, R, C, level_scale, codes);
    mark_end(s);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    mark_begin("stream_copy", s);
    hipLaunchKernelGGL(stream_copy_kernel, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, s,
                       static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    mark_end(s);
    return hipGetLastError();
}

}  // namespace msda
