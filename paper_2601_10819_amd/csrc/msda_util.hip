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

// One block per (batch item, camera, level) region; atomicMax of |x| as bits
// (non-negative floats order like their bit patterns).
__global__ void amax_kernel(const float* x, const int32_t* shapes, const int32_t* starts,
                            int N, int L, int64_t R, int C, u32* amax) {
    const int region = blockIdx.x % (N * L);
    const int b = blockIdx.x / (N * L);
    const int l = region % L;
    const int64_t rows = (int64_t)shapes[2 * region] * shapes[2 * region + 1];
    const float* base = x + ((size_t)b * R + starts[region]) * C;
    const size_t n = (size_t)rows * C;
    float m = 0.f;
    for (size_t k = threadIdx.x + (size_t)blockIdx.y * blockDim.x; k < n;
         k += (size_t)blockDim.x * gridDim.y)
        m = fmaxf(m, fabsf(base[k]));
    for (int s = 32; s > 0; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&amax[l], __float_as_uint(m));
}

__global__ void scale_kernel(const u32* amax, float* scale, int L) {
    const int l = threadIdx.x;
    if (l < L) {
        const float m = __uint_as_float(amax[l]);
        scale[l] = m > 0.f ? m / 448.f : 1.f;
    }
}

// OCP e4m3, round to nearest even, |q| <= 448 on entry.
__device__ __forceinline__ u32 e4m3_rne(float q) {
    const u32 bits = __float_as_uint(q);
    const u32 sign = (bits >> 24) & 0x80u;
    const float a = fabsf(q);
    u32 code;
    if (a < 0.015625f) {                       // below 2^-6: spacing 2^-9
        code = (u32)rintf(a * 512.f);          // exact scaling; rint ties to even; 8 -> 2^-6
    } else {
        const u32 ab = bits & 0x7fffffffu;
        const u32 e = (ab >> 23) - 127u + 7u;  // biased e4m3 exponent, 1..15
        const u32 m = ab & 0x7fffffu;
        code = (e << 3) | (m >> 20);
        const u32 rem = m & 0xfffffu;
        if (rem > 0x80000u || (rem == 0x80000u && (code & 1u))) code += 1u;  // may carry into e
    }
    return sign | code;
}

__global__ void quantize_kernel(const float* x, const int32_t* shapes, const int32_t* starts,
                                int N, int L, int64_t R, int C, const float* scale,
                                uint8_t* codes) {
    const int region = blockIdx.x % (N * L);
    const int b = blockIdx.x / (N * L);
    const int l = region % L;
    const int64_t rows = (int64_t)shapes[2 * region] * shapes[2 * region + 1];
    const size_t off = ((size_t)b * R + starts[region]) * C;
    const size_t n = (size_t)rows * C;
    const float s = scale[l];
    for (size_t k = threadIdx.x + (size_t)blockIdx.y * blockDim.x; k < n;
         k += (size_t)blockDim.x * gridDim.y) {
        float q = x[off + k] / s;                   // IEEE division, as the reference
        q = fminf(fmaxf(q, -448.f), 448.f);
        codes[off + k] = (uint8_t)e4m3_rne(q);
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
                               uint8_t* codes, float* level_scale, uint32_t* amax_ws,
                               hipStream_t s) {
    hipError_t e = launch_fill_zero(amax_ws, (size_t)L * 4, s);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)(B * N * L), 8);
    mark_begin("fp8_amax", s);
    hipLaunchKernelGGL(amax_kernel, grid, dim3(256), 0, s, x, shapes, starts, N, L, R, C, amax_ws);
    mark_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark_begin("fp8_scale", s);
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(64), 0, s, amax_ws, level_scale, L);
    mark_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark_begin("fp8_quantize", s);
    hipLaunchKernelGGL(quantize_kernel, grid, dim3(256), 0, s, x, shapes, starts, N, L, R, C,
                       level_scale, codes);
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
