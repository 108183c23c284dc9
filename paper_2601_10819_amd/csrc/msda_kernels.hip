// HIP kernels for multi-scale deformable aggregation (MSDA) on gfx950.
//
// Operator: paper Sec. 3.1 / Sec. 3.2 (keypoints of each 3D anchor projected
// into every camera, the camera's multi-scale feature maps sampled
// bilinearly there and aggregated with learned weights); Sec. 5.3 names it
// and notes that it is memory-bound, with low arithmetic intensity and
// scattered accesses. So this is a gather, not a contraction: no MFMA. The
// design choices for CDNA4:
//
//  * One workgroup per (batch item, anchor); its waves split the anchor's
//    (keypoint, camera) pairs. A pair's L levels share one location.
//  * Each lane owns `CPL` consecutive channels, so a sample is C/CPL lanes
//    ("lanes per sample"), and a 64-lane wave works on 64/(C/CPL) samples at
//    once. Corner rows are read with 4/8/16-byte buffer loads: the 4 corner
//    gathers of a sample are channel-contiguous and coalesced.
//  * Feature reads go through a buffer resource that spans one batch item.
//    A corner outside its level gets an offset past the end of the resource,
//    so the hardware returns 0 without touching memory: zero padding costs no
//    branch, and no computed index can read outside the tensor.
//  * Each wave stages its chunk of locations and weights in LDS with
//    coalesced loads; lanes then read their sample's values as LDS broadcasts.
//  * The coordinate x = u*W - 0.5 is formed from the exact product u*W
//    (Dekker/TwoProduct split via fma), so floor() and the fraction are exact
//    to a few 1e-8 px instead of ~4e-6 px at W = 176.
//  * Per-group (grad_weights) and per-sample (grad_sampling_loc) reductions
//    use cross-lane shuffles within the lanes of one sample.
//  * All interpolation and accumulation is FP32; BF16 and FP8 are storage
//    formats widened in registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_internal.h"

namespace msda {

typedef uint32_t u32;
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

// Offset used for a corner outside its level: beyond every resource (whose
// size is < 2^31), so a buffer load returns zeros.
constexpr u32 kOOB = 0x80000000u;
// Per-lane registers' worth of weights staged per wave step (see max_pairs_per_chunk).
constexpr int kStageWords = 8;

// Word 3 of a raw (untyped, stride 0) buffer resource on gfx9-family GPUs.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, u32 bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

// ---------------------------------------------------------------- feature types

struct TF32 { static constexpr int kBytes = 4; };
struct TBF16 { static constexpr int kBytes = 2; };
struct TFP8 { static constexpr int kBytes = 1; };

template <class FT, int CPL>
struct Row {
    static constexpr int kBytes = FT::kBytes * CPL;   // 4, 8 or 16
    static constexpr int kWords = kBytes / 4;
    static_assert(kBytes == 4 || kBytes == 8 || kBytes == 16, "unsupported lane width");
};

template <int WORDS>
__device__ __forceinline__ void load_words(rsrc_t r, u32 off, u32* d) {
    if constexpr (WORDS == 4) {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
    } else if constexpr (WORDS == 2) {
        u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        d[0] = v.x; d[1] = v.y;
    } else {
        d[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    }
}

// Widen CPL stored channels (in `w`) to FP32.
template <class FT, int CPL>
__device__ __forceinline__ void widen(const u32* w, float* f) {
    if constexpr (FT::kBytes == 4) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) f[i] = __uint_as_float(w[i]);
    } else if constexpr (FT::kBytes == 2) {
        // bfloat16 is the top half of an FP32: widening is a shift.
#pragma unroll
        for (int i = 0; i < CPL / 2; ++i) {
            f[2 * i] = __uint_as_float(w[i] << 16);
            f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    } else {
        // OCP e4m3 to FP32 with the hardware converter, two codes at a time.
#pragma unroll
        for (int i = 0; i < CPL / 4; ++i) {
            f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
            f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
            f[4 * i] = lo.x; f[4 * i + 1] = lo.y; f[4 * i + 2] = hi.x; f[4 * i + 3] = hi.y;
        }
    }
}

// ---------------------------------------------------------------- geometry

struct Geo { int H, W, start; float scale; };

__device__ __forceinline__ void stage_geometry(Geo* geo, const OpArgs& a) {
    const int NL = a.N * a.L;
    for (int i = threadIdx.x; i < NL; i += blockDim.x) {
        Geo g;
        g.H = a.shapes[2 * i];
        g.W = a.shapes[2 * i + 1];
        g.start = a.starts[i];
        g.scale = a.level_scale ? a.level_scale[i % a.L] : 1.f;
        geo[i] = g;
    }
}

// Integer part and fraction of t = u*n - 0.5 along one axis of a level with n
// pixels, and whether -1 < t < n. u*n is split exactly into p + e (fma), the
// floor is taken of p, and the fraction is assembled from exact pieces, so
// only the final add rounds.
struct Axis { int i0; float l; bool ok; };

__device__ __forceinline__ Axis axis_of(float u, int n) {
    const float fn = (float)n;
    const float p = u * fn;
    const float e = fmaf(u, fn, -p);            // u*n == p + e exactly
    const float fp = floorf(p);
    const float f = ((p - fp) - 0.5f) + e;      // t - fp, in about [-0.5, 0.5)
    const float flo = f < 0.f ? -1.f : 0.f;
    float l = f - flo;
    float i0f = fp + flo;
    if (l >= 1.f) { l = 0.f; i0f += 1.f; }      // f a hair below 0: t is an integer
    i0f = fminf(fmaxf(i0f, -4.f), fn + 4.f);    // keeps the int conversion defined; NaN -> -4
    Axis a;
    a.i0 = (int)i0f;
    a.ok = (a.i0 >= 0 || (a.i0 == -1 && l > 0.f)) && a.i0 < n;
    a.l = a.ok ? l : 0.f;
    return a;
}

// The 4 corners of one sample: byte offsets (kOOB when outside) and bilinear
// weights (0 when outside), in the order (y0,x0), (y0,x0+1), (y0+1,x0), (y0+1,x0+1).
struct Corners {
    u32 off[4];
    float cw[4];
    float lx, ly;
    int row[4];     // -1 when outside
    bool valid;
};

__device__ __forceinline__ Corners corners_of(float u, float v, const Geo& g, u32 row_bytes,
                                              u32 lane_off) {
    const Axis ax = axis_of(u, g.W);
    const Axis ay = axis_of(v, g.H);
    Corners c;
    c.valid = ax.ok && ay.ok;
    c.lx = c.valid ? ax.l : 0.f;
    c.ly = c.valid ? ay.l : 0.f;
    const float hx = 1.f - c.lx, hy = 1.f - c.ly;
    const bool in_x0 = ax.i0 >= 0, in_x1 = ax.i0 + 1 < g.W;
    const bool in_y0 = ay.i0 >= 0, in_y1 = ay.i0 + 1 < g.H;
    const bool in[4] = {c.valid && in_y0 && in_x0, c.valid && in_y0 && in_x1,
                        c.valid && in_y1 && in_x0, c.valid && in_y1 && in_x1};
    const float wt[4] = {hy * hx, hy * c.lx, c.ly * hx, c.ly * c.lx};
    const int base = g.start + ay.i0 * g.W + ax.i0;
    const int rows[4] = {base, base + 1, base + g.W, base + g.W + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c.row[k] = in[k] ? rows[k] : -1;
        c.off[k] = in[k] ? (u32)rows[k] * row_bytes + lane_off : kOOB;
        c.cw[k] = in[k] ? wt[k] : 0.f;
    }
    return c;
}

// ---------------------------------------------------------------- shared pieces

template <class T>
__device__ __forceinline__ T xor_shuffle(T v, int mask) {
    return __shfl_xor(v, mask, 64);
}


// Copy one chunk of nj pairs' weights (nj*LG floats) and locations (nj*2)
// into this wave's LDS slot. Both are contiguous in global memory.
__device__ __forceinline__ void stage_chunk(float* sw, float* sl, const float* gw,
                                            const float* gl, int nj, int LG, int lane) {
    const int nw = nj * LG;
#pragma unroll
    for (int t = 0; t < kStageWords; ++t) {
        const int i = t * 64 + lane;
        if (i < nw) sw[i] = gw[i];
    }
    if (lane < 2 * nj) sl[lane] = gl[lane];
    // LDS accesses of one wave are performed in program order; this keeps the
    // compiler from moving the reads that follow above the writes.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void end_chunk() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// ---------------------------------------------------------------- forward

template <class FT, int CPL>
__global__ void __launch_bounds__(512) msda_fwd_kernel(OpArgs a) {
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
}

// ---------------------------------------------------------------- backward

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
    const int c0 = (lane & (lps - 1)) * CPL;
    const int cpg = a.C / a.G;
    const int g = c0 / cpg;
    const int lpg = cpg / CPL;             // lanes of one group (a power of two)
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
                    // grad_w[g] = sum over the group's channels of grad_out * val
                    float t = cr.cw[0] * d[0] + cr.cw[1] * d[1] + cr.cw[2] * d[2] +
                              cr.cw[3] * d[3];
                    for (int s = 1; s < lpg; s <<= 1) t += xor_shuffle(t, s);
                    if ((lane & (lpg - 1)) == 0) gwout[(size_t)j * LG + l * a.G + g] = t;
                }
                // d val / dx = hy (F01 - F00) + ly (F11 - F10); x = u W - 0.5
                const float hx = 1.f - cr.lx, hy = 1.f - cr.ly;
                gx += (float)gm.W * wl * (hy * (d[1] - d[0]) + cr.ly * (d[3] - d[2]));
                gy += (float)gm.H * wl * (hx * (d[2] - d[0]) + cr.lx * (d[3] - d[1]));
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
            }
            if (glout) {
                for (int s = 1; s < lps; s <<= 1) {
                    gx += xor_shuffle(gx, s);
                    gy += xor_shuffle(gy, s);
                }
                if ((lane & (lps - 1)) == 0) {
                    glout[(size_t)j * 2] = gx;
                    glout[(size_t)j * 2 + 1] = gy;
                }
            }
        }
        end_chunk();
    }
}

// ---------------------------------------------------------------- small kernels

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

// FP32 -> bfloat16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    const u32 b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__global__ void f32_to_bf16_kernel(const float* src, uint16_t* dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = bf16_rne(src[k]);
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

// ---------------------------------------------------------------- launchers

template <class FT, int CPL>
static hipError_t fwd_launch(const OpArgs& a, int waves, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((msda_fwd_kernel<FT, CPL>), dim3((unsigned)(a.B * a.A)),
                       dim3(64 * waves), lds, s, a);
    return hipGetLastError();
}

template <class FT, int CPL>
static hipError_t bwd_launch(const OpArgs& a, int waves, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((msda_bwd_kernel<FT, CPL>), dim3((unsigned)(a.B * a.A)),
                       dim3(64 * waves), lds, s, a);
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

static unsigned grid_for(size_t n, unsigned block, unsigned cap) {
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(bytes / 16 + 1, 256, 8192)), dim3(256), 0,
                       s, static_cast<unsigned char*>(p), bytes);
    return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, src,
                       dst, n);
    return hipGetLastError();
}

hipError_t launch_quantize_fp8(const float* x, const int32_t* shapes, const int32_t* starts,
                               int32_t B, int32_t N, int32_t L, int64_t R, int32_t C,
                               uint8_t* codes, float* level_scale, uint32_t* amax_ws,
                               hipStream_t s) {
    hipError_t e = launch_fill_zero(amax_ws, (size_t)L * 4, s);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)(B * N * L), 8);
    hipLaunchKernelGGL(amax_kernel, grid, dim3(256), 0, s, x, shapes, starts, N, L, R, C, amax_ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(64), 0, s, amax_ws, level_scale, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(quantize_kernel, grid, dim3(256), 0, s, x, shapes, starts, N, L, R, C,
                       level_scale, codes);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, s,
                       static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    return hipGetLastError();
}

}  // namespace msda
