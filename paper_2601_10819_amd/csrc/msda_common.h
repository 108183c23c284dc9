// Device-side building blocks shared by the MSDA kernels for gfx950:
// buffer resources and lane-width loads, storage widening, sample geometry,
// and the per-wave LDS staging of locations and weights.
//
// The operator (paper Sec. 3.1 / Sec. 3.2; named in Sec. 5.3) samples every
// camera's feature pyramid bilinearly at each projected keypoint and sums the
// samples with per-(keypoint, camera, level, group) weights. It is a gather
// with low arithmetic intensity (Sec. 5.3), so the kernels are organised
// around memory access, not matrix cores:
//
//  * Each lane owns CPL consecutive channels; a sample occupies C/CPL lanes
//    ("lanes per sample", a power of two <= 64) and a 64-lane wave works on
//    64/(C/CPL) samples at once. Corner rows are read with 4/8/16-byte buffer
//    loads, so the 4 corner gathers of a sample are channel-contiguous.
//  * Feature reads go through a buffer resource spanning one batch item. A
//    corner outside its level gets an offset past the end of the resource and
//    the hardware returns 0 without touching memory: zero padding costs no
//    branch, and no computed index can read outside the tensor.
//  * The coordinate t = u*W - 0.5 is assembled from the exact product u*W
//    (an fma recovers the rounding error of the multiply), so floor(t) and the
//    bilinear fraction are exact to ~1e-7 px instead of half an FP32 ulp of t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msda_internal.h"

namespace msda {

typedef uint32_t u32;
typedef uint64_t u64;
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;


// Word 3 of a raw (untyped, stride 0) buffer resource on gfx9-family GPUs.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, u32 bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

// ---------------------------------------------------------------- storage types

// kKind matches the FeatType code of the storage type.
struct TF32 { static constexpr int kBytes = 4, kKind = 0; };
struct TBF16 { static constexpr int kBytes = 2, kKind = 1; };
struct TFP8 { static constexpr int kBytes = 1, kKind = 2; };
struct TF16 { static constexpr int kBytes = 2, kKind = 3; };

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

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

// Widen CPL stored channels (packed in `w`) to FP32.
template <class FT, int CPL>
__device__ __forceinline__ void widen(const u32* w, float* f) {
    if constexpr (FT::kBytes == 4) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) f[i] = __uint_as_float(w[i]);
    } else if constexpr (FT::kKind == 1) {
        // bfloat16 is the top half of an FP32: widening is a shift.
#pragma unroll
        for (int i = 0; i < CPL / 2; ++i) {
            f[2 * i] = __uint_as_float(w[i] << 16);
            f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    } else if constexpr (FT::kKind == 3) {
        // IEEE half to FP32 is exact; feeding it straight into an FMA lets the
        // compiler use v_fma_mix_f32, which widens either half of a word
        // inside the FP32 FMA itself.
#pragma unroll
        for (int i = 0; i < CPL / 2; ++i) {
            const half2_t h = __builtin_bit_cast(half2_t, w[i]);
            f[2 * i] = (float)h.x;
            f[2 * i + 1] = (float)h.y;
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

// FP32 -> IEEE half with the hardware conversion: round to nearest even
// (the default rounding mode), overflow to infinity, NaN stays NaN.
__device__ __forceinline__ uint16_t f16_rne(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
}

// FP32 -> bfloat16 with gfx950's converter (v_cvt_pk_bf16_f32): round to
// nearest even, overflow to infinity, NaN stays NaN.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    return __builtin_bit_cast(uint16_t, (__bf16)x);
}

// Two values at once, lo in the low half: one instruction.
__device__ __forceinline__ u32 bf16x2_rne(float lo, float hi) {
    const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(u32, v);
}

// ---------------------------------------------------------------- geometry

// One (camera, level) region: its size, first row, first bilinear cell (for
// the sorted grad_feat records; 0 when unused) and the FP8 level scale (1
// for other storage types).
struct Geo { int H, W, start; float scale; u32 cstart, pad0, pad1, pad2; };

__device__ __forceinline__ void stage_geometry(Geo* geo, const OpArgs& a) {
    const int NL = a.N * a.L;
    for (int i = threadIdx.x; i < NL; i += blockDim.x) {
        Geo g;
        g.H = a.shapes[2 * i];
        g.W = a.shapes[2 * i + 1];
        g.start = a.starts[i];
        g.scale = a.level_scale ? a.level_scale[i % a.L] : 1.f;
        g.cstart = a.cell_start ? a.cell_start[i] : 0u;
        g.pad0 = g.pad1 = g.pad2 = 0u;
        geo[i] = g;
    }
}

// Integer part and fraction of t = u*n - 0.5 along one axis of a level with n
// pixels, and whether -1 < t < n. u*n is split exactly into p + e, the floor
// is taken of p, and the fraction is assembled from exact pieces, so only the
// final add rounds.
struct Axis { int i0; float l; bool ok; };

__device__ __forceinline__ Axis axis_of(float u, int n) {
    // The split only works if each operation is rounded as written: a fused
    // u*n - fp would already contain e, which is then added a second time.
#pragma clang fp contract(off)
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

// The 4 corners of one sample, in the order (y0,x0), (y0,x0+1), (y0+1,x0),
// (y0+1,x0+1): byte offsets (kOOB when outside), bilinear weights (0 when
// outside) and rows within the batch item (-1 when outside).
struct Corners {
    u32 off[4];
    float cw[4];
    float lx, ly;
    int row[4];
    int x0, y0;     // top-left neighbour (meaningful when valid)
    bool valid;
};

__device__ __forceinline__ Corners corners_of(float u, float v, const Geo& g, u32 row_bytes,
                                              u32 lane_off) {
    const Axis ax = axis_of(u, g.W);
    const Axis ay = axis_of(v, g.H);
    Corners c;
    c.valid = ax.ok && ay.ok;
    c.x0 = ax.i0;
    c.y0 = ay.i0;
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

// ---------------------------------------------------------------- lanes and LDS

// Index of the calling wave in its workgroup, as a wave-uniform (scalar)
// value: the compiler cannot see that threadIdx.x / 64 is the same for the
// whole wave, and values derived from it (a batch item's buffer resource, a
// loop bound) would otherwise live in vector registers -- a buffer load
// with a per-lane resource becomes a loop over the distinct resources.
__device__ __forceinline__ int wave_index() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// A value the caller knows to be the same in every lane, marked as such for
// the compiler (it is then kept in scalar registers).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ const void* uniform(const void* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return reinterpret_cast<const void*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float xor_shuffle(float v, int mask) {
    return __shfl_xor(v, mask, 64);
}

// Cross-lane steps that stay in the VALU (no LDS round trip): DPP row
// permutations and the gfx950 row / half-wave swaps. Callers keep every
// lane of a group active together, so no step reads a disabled lane.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// v + v of the lane 16 (resp. 32) away: the swap pairs rows 0-1 and 2-3
// (resp. the two halves); each lane ends with both values of its pair.
__device__ __forceinline__ float swap16_sum(float v) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                    false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

__device__ __forceinline__ float swap32_sum(float v) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                    false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

// Sum over aligned groups of `width` lanes (a power of two <= 64, the same in
// every lane): quad butterflies, then row half-mirror and mirror (pairing
// the halves of 8 and of 16 lanes), then the swaps. Every lane of a group
// ends with its group's sum, the same bits in each.
__device__ __forceinline__ float group_sum(float v, int width) {
    if (width > 1) v += dpp<0xB1>(v);     // quad_perm [1,0,3,2]
    if (width > 2) v += dpp<0x4E>(v);     // quad_perm [2,3,0,1]
    if (width > 4) v += dpp<0x141>(v);    // row_half_mirror
    if (width > 8) v += dpp<0x140>(v);    // row_mirror
    if (width > 16) v = swap16_sum(v);
    if (width > 32) v = swap32_sum(v);
    return v;
}

// group_sum with the width known at compile time (no branches); W = 0:
// the width given at run time.
template <int W>
__device__ __forceinline__ float group_sum_w(float v, int width) {
    if constexpr (W == 0) {
        return group_sum(v, width);
    } else {
        if constexpr (W > 1) v += dpp<0xB1>(v);
        if constexpr (W > 2) v += dpp<0x4E>(v);
        if constexpr (W > 4) v += dpp<0x141>(v);
        if constexpr (W > 8) v += dpp<0x140>(v);
        if constexpr (W > 16) v = swap16_sum(v);
        if constexpr (W > 32) v = swap32_sum(v);
        return v;
    }
}

// v + v[lane ^ mask] for a power-of-two mask (the same in every lane).
__device__ __forceinline__ float xor_sum(float v, int mask) {
    if (mask == 32) return swap32_sum(v);
    if (mask == 16) return swap16_sum(v);
    if (mask == 8) return v + dpp<0x128>(v);   // row_ror:8
    return v + xor_shuffle(v, mask);
}

// Per-lane registers' worth of weights staged per wave step.
constexpr int kStageWords = 8;

// The 4 corner taps of one sample as staged in LDS: byte offsets of the
// corner rows within the batch item (kOOB outside; each lane adds its own
// channel offset) and the bilinear weights (times the FP8 level scale).
struct alignas(16) Taps { u32 off[4]; float cw[4]; };

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// One wave's LDS staging slot for a chunk of up to J (keypoint, camera)
// pairs of one anchor: per pair its index p*N + n among the anchor's pairs
// and its camera, its L*G weights, and the taps of its L samples; for the
// backward also each sample's location-derivative factors
// (W(1-ly), W ly, H(1-lx), H lx): d(blend)/dx = W((1-ly)(F01-F00) +
// ly(F11-F10)) and d(blend)/dy = H((1-lx)(F10-F00) + lx(F11-F01)).
struct StageSlot {
    u32* src;
    u32* cam;
    float* w;
    Taps* taps;
    float4* dk;
};

// Levels per pair in the staged taps: L rounded up to a multiple of 4, so the
// forward issues the loads of 4 levels at a time without a branch (a padded
// level's taps point outside the feature and weigh 0).
__host__ __device__ constexpr int padded_levels(int L) { return (L + 3) & ~3; }

// Every part starts 16-byte aligned (taps are read as 16-byte words), and so
// does every wave's slot.
__host__ __device__ constexpr size_t wave_stage_bytes(int J, int L, int G) {
    return align16((size_t)J * 8) + align16((size_t)J * L * G * 4) +
           (size_t)J * padded_levels(L) * sizeof(Taps) +
           (size_t)J * padded_levels(L) * sizeof(float4);
}

__device__ __forceinline__ StageSlot stage_slot(unsigned char* work, int wave, int J, int L,
                                                int G) {
    unsigned char* p = work + (size_t)wave * wave_stage_bytes(J, L, G);
    StageSlot s;
    s.src = reinterpret_cast<u32*>(p);
    s.cam = s.src + J;
    p += align16((size_t)J * 8);
    s.w = reinterpret_cast<float*>(p);
    p += align16((size_t)J * L * G * 4);
    s.taps = reinterpret_cast<Taps*>(p);
    s.dk = reinterpret_cast<float4*>(s.taps + (size_t)J * padded_levels(L));
    return s;
}

// Makes this wave's LDS writes visible to its later reads: LDS accesses of
// one wave are performed in program order; the fences keep the compiler
// from moving the reads that follow above the writes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pair orders: the k-th pair a wave processes -> (index p*N + n, camera n).
// Anchor order walks the anchor's pairs as stored (keypoint-major); view
// order walks cameras [n_lo, n_lo + nv) one after the other, every
// keypoint of a camera before the next camera.
struct AnchorOrder {
    int N;
    __device__ __forceinline__ void operator()(int k, u32* src, u32* cam) const {
        *src = (u32)k;
        *cam = (u32)(k % N);
    }
};

struct ViewOrder {
    int N, P, n_lo;
    int geo_lo = 0;     // first camera of the staged geometry (a wave's own slice)
    __device__ __forceinline__ void operator()(int k, u32* src, u32* cam) const {
        const int q = k / P, p = k - q * P;
        *cam = (u32)(n_lo + q - geo_lo);
        *src = (u32)(p * N + n_lo + q);
    }
};

// Where the backward writes its grad_feat records (key = bilinear cell,
// frac = (lx, ly)) while staging. The sample (pair src, level l) has the
// index s = base + src*L + l; its fractions go to frac[s]. Dense records
// (val == nullptr): the record is key[s] and its value is s. Compacted
// records (the visible-view form): the k-th pair the wave processes writes
// record r = cbase + k*L + l, key[r] and val[r] = s. key == nullptr: none.
//
// Bucketed records (bucket_ap != 0, the dense single call): the record of
// pair src = p*N + n, level l goes to bucket (b, n, l) at slot a*P + p,
// i.e. key[bucket_base + (n*L + l)*bucket_ap + p] with bucket_base =
// b*N*L*bucket_ap + a*P, and its key is the local cell of the region
// ((H+1)(W+1) outside the level); frac is still written at s.
struct RecordSink {
    u32* key;
    float2* frac;
    u32 base;            // first sample of the anchor
    u32 cell_base;       // first cell of the batch item
    u32 no_cell;         // key of a sample outside its level
    u32* val;            // compacted records' values, or nullptr
    u32 cbase;           // compacted: first record of the wave's item
    u32 bucket_ap;       // bucketed: A*P records per bucket (0: not bucketed)
    u32 bucket_base;     // bucketed: b*N*L*A*P + a*P
    u32 N;               // bucketed: cameras
};

// One anchor's weights as the gathers stage them: FP32 or bfloat16 storage,
// and optionally logits turned into the per-group softmax on the fly
// (w = exp(logit - max_g) / sum_g, the group's statistics precomputed).
struct WSrc {
    const void* p;          // the anchor's [P*N][L*G] weights or logits
    const float2* stats;    // per group (max, 1/sum), or nullptr (plain weights)
    int G;
    bool bf16;
    __device__ WSrc(const float* w) : p(w), stats(nullptr), G(1), bf16(false) {}
    __device__ WSrc(const void* w, const float2* st, int g, bool b)
        : p(w), stats(st), G(g), bf16(b) {}
    // entry i as stored (FP32, or bfloat16 widened exactly)
    __device__ __forceinline__ float raw(size_t i) const {
        return bf16 ? __uint_as_float((u32)static_cast<const uint16_t*>(p)[i] << 16)
                    : static_cast<const float*>(p)[i];
    }
    // the softmax weight of a logit x of group g (G is a power of two, and
    // entry i of a chunk belongs to group i & (G - 1))
    __device__ __forceinline__ float softmax(float x, int g) const {
        const float2 st = stats[g];
        return expf(x - st.x) * st.y;
    }
};

// The weights of anchor ba (npw = P*N*L*G entries per anchor) as staged.
__device__ __forceinline__ WSrc anchor_weights(const OpArgs& a, size_t ba, size_t npw) {
    const void* p = a.w_bf16 ? static_cast<const void*>(
                                   reinterpret_cast<const uint16_t*>(a.w) + ba * npw)
                             : static_cast<const void*>(a.w + ba * npw);
    return WSrc(p, a.wstats ? a.wstats + ba * (size_t)a.G : nullptr, a.G, a.w_bf16 != 0);
}

// Stages pairs [k0, k0 + nj) (in the wave's pair order) of the anchor whose
// weights / locations start at gw / gl: pair table, weights (coalesced
// within each pair's L*G run), and one sample's taps per lane. Ends with
// the slot readable by the whole wave.
template <bool SCALE_TAPS, bool FRACS, class Order>
__device__ __forceinline__ void stage_chunk(const StageSlot& s, const Order& order, int k0, int nj,
                                            const WSrc& gw, const float* gl, const Geo* geo,
                                            int L, int LG, u32 row_bytes, int lane,
                                            const RecordSink& rec) {
    if (lane < nj) {
        u32 src, cam;
        order(k0 + lane, &src, &cam);
        s.src[lane] = src;
        s.cam[lane] = cam;
    }
    wave_lds_sync();
    const int nw = nj * LG;
#pragma unroll
    for (int t = 0; t < kStageWords; ++t) {
        const int i = t * 64 + lane;
        if (i < nw) {
            const int jj = i / LG;
            s.w[i] = gw.raw((size_t)s.src[jj] * LG + (i - jj * LG));
        }
    }
    if (gw.stats) {
        // logits -> softmax weights: each lane rewrites the entries it staged
        for (int i = lane; i < nw; i += 64) s.w[i] = gw.softmax(s.w[i], i & (gw.G - 1));
    }
    const int Lp = padded_levels(L);
    for (int i = lane; i < nj * Lp; i += 64) {
        const int jj = i / Lp, l = i - jj * Lp;
        Taps t;
        if (l >= L) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                t.off[c] = kOOB;
                t.cw[c] = 0.f;
            }
            s.taps[i] = t;
            if constexpr (FRACS) s.dk[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        const u32 src = s.src[jj];
        const Geo gm = geo[s.cam[jj] * L + l];
        const Corners cr = corners_of(gl[2 * src], gl[2 * src + 1], gm, row_bytes, 0u);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            t.off[c] = cr.off[c];
            t.cw[c] = SCALE_TAPS ? cr.cw[c] * gm.scale : cr.cw[c];
        }
        s.taps[i] = t;
        if constexpr (FRACS) {
            const float fw = (float)gm.W, fh = (float)gm.H;
            s.dk[i] = make_float4(fw * (1.f - cr.ly), fw * cr.ly, fh * (1.f - cr.lx), fh * cr.lx);
            if (rec.key) {
                const u32 smp = rec.base + src * (u32)L + (u32)l;
                const u32 local = cr.valid ? (u32)(cr.y0 + 1) * (u32)(gm.W + 1) + (u32)(cr.x0 + 1)
                                           : (u32)(gm.H + 1) * (u32)(gm.W + 1);
                const u32 key = cr.valid ? rec.cell_base + gm.cstart + local : rec.no_cell;
                if (rec.bucket_ap) {
                    const u32 p = src / rec.N, n = src - p * rec.N;
                    rec.key[rec.bucket_base + (n * (u32)L + (u32)l) * rec.bucket_ap + p] = local;
                } else if (rec.val) {
                    const u32 r = rec.cbase + (u32)(k0 + jj) * (u32)L + (u32)l;
                    rec.key[r] = key;
                    rec.val[r] = smp;
                } else {
                    rec.key[smp] = key;
                }
                rec.frac[smp] = make_float2(cr.lx, cr.ly);
            }
        }
    }
    wave_lds_sync();
}

// Lane layout of one wave: CPL channels per lane, C/CPL lanes per sample.
struct Lanes {
    int lane, lps, spw, sub, c0, g;
    u32 lane_off;
};

template <class FT, int CPL>
__device__ __forceinline__ Lanes lanes_of(const OpArgs& a) {
    Lanes q;
    q.lane = threadIdx.x & 63;
    q.lps = 1 << a.lps_shift;
    q.spw = 64 >> a.lps_shift;
    q.sub = q.lane >> a.lps_shift;
    q.c0 = (q.lane & (q.lps - 1)) * CPL;
    q.g = q.c0 / (a.C / a.G);
    q.lane_off = (u32)q.c0 * FT::kBytes;
    return q;
}

// Ends a chunk: the next staging may overwrite the slot.
__device__ __forceinline__ void end_chunk() { wave_lds_sync(); }

// Inclusive scan across the 256 threads of a block (4 waves); returns the
// thread's inclusive sum and the block total in *total.
__device__ __forceinline__ u32 block_inclusive_scan(u32 v, u32* lds4, u32* total) {
    const int lane = threadIdx.x & 63, wave = wave_index();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const u32 t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    if (lane == 63) lds4[wave] = v;
    __syncthreads();
    u32 before = 0;
    for (int w = 0; w < wave; ++w) before += lds4[w];
    *total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
    __syncthreads();
    return v + before;
}

// ---------------------------------------------------------------- batched form

// The scene of a batch item index: the last s with start[s] <= item (start
// is a non-decreasing prefix table of S+1 entries).
__device__ __forceinline__ int scene_of(const u32* start, int S, u32 item) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Scene s of a batch as a single-call argument set with B = 1.
__device__ __forceinline__ OpArgs scene_view(const BatchArgs& b, int s, int feat_bytes) {
    const msda_scene& sc = b.scenes[s];
    OpArgs a = {};
    a.feat = sc.feat;
    a.shapes = sc.spatial_shapes;
    a.starts = sc.level_start_index;
    a.loc = sc.sampling_loc;
    // under a weight flag: the FP32 weights (backward), or the scene's
    // logits / BF16 weights with its anchors' softmax statistics (forward)
    a.w = b.w32 ? b.w32 + (size_t)b.t.sample_start[s] * (size_t)b.G : sc.weights;
    a.w_bf16 = b.w32 ? 0 : b.w_bf16;
    a.wstats = (b.w32 || !b.wstats) ? nullptr : b.wstats + (size_t)b.t.anchor_start[s] * (size_t)b.G;
    a.level_scale = b.level_scale;
    a.grad_out = sc.grad_out;
    a.out = sc.out;
    a.grad_loc = sc.grad_sampling_loc;
    a.grad_w = sc.grad_weights;
    a.rec_key = b.rec_key;
    a.rec_frac = b.rec_frac;
    a.cell_start = b.rec_key ? b.t.cell_start + b.t.region_start[s] : nullptr;
    a.cells_per_item = 0;
    a.cell_offset = 0;
    a.no_cell = b.total_cells;
    a.sample_offset = b.rec_key ? b.t.sample_start[s] : 0u;
    a.rec_bucket_ap = b.rec_key && b.rec_bucketed ? (u32)sc.num_anchors * (u32)b.P : 0u;
    a.B = 1;
    a.N = sc.num_cams;
    a.L = b.L;
    a.A = sc.num_anchors;
    a.P = b.P;
    a.C = b.C;
    a.G = b.G;
    a.R = sc.rows;
    a.batch_bytes = (u32)(sc.rows * (int64_t)b.C * feat_bytes);
    a.lps_shift = b.lps_shift;
    a.pairs_per_chunk = b.pairs_per_chunk;
    return a;
}

// A row of the batched view order: one anchor of one scene over that
// scene's cameras in XCD slot x, the single call's slot split of the scene
// with B = 1. nv = 0: the anchor has no cameras in the slot.
struct BatchRow {
    int s, a, n_lo, nv;
};

__device__ __forceinline__ BatchRow batch_row(const BatchArgs& b, int x, u32 g) {
    BatchRow r;
    r.s = scene_of(b.t.anchor_start, b.S, g);
    r.a = (int)(g - b.t.anchor_start[r.s]);
    const int N = b.scenes[r.s].num_cams, A = b.scenes[r.s].num_anchors;
    const SlotSpan span = slot_span(x, 1, N, A);
    r.n_lo = 0;
    r.nv = 0;
    if (slot_rows(span, A) > 0) {
        const ViewRow v = view_row(span, r.a, N, A);
        r.n_lo = v.n_lo;
        r.nv = v.nv;
    }
    // every field is the same across the wave (g is per wave)
    r.s = uniform(r.s);
    r.a = uniform(r.a);
    r.n_lo = uniform(r.n_lo);
    r.nv = uniform(r.nv);
    return r;
}

// Bytes of one wave's LDS in the batched view order: the geometry of its
// row's cameras (at most view_cams) and its staging slot.
__host__ __device__ inline size_t batch_view_wave_bytes(int view_cams, int L, int J, int G) {
    return (((size_t)view_cams * L * sizeof(Geo) + 15) & ~(size_t)15) +
           wave_stage_bytes(J, L, G);
}

// The geometry of cameras [n_lo, n_lo + nv) of `a` into one wave's slice
// (entry (n - n_lo) * L + l), then readable by the whole wave.
__device__ __forceinline__ void stage_geometry_range(Geo* geo, const OpArgs& a, int n_lo, int nv,
                                                     int lane) {
    for (int i = lane; i < nv * a.L; i += 64) {
        const int l = i % a.L, r = (n_lo + i / a.L) * a.L + l;
        Geo g;
        g.H = a.shapes[2 * r];
        g.W = a.shapes[2 * r + 1];
        g.start = a.starts[r];
        g.scale = a.level_scale ? a.level_scale[l] : 1.f;
        g.cstart = a.cell_start ? a.cell_start[r] : 0u;
        g.pad0 = g.pad1 = g.pad2 = 0u;
        geo[i] = g;
    }
    wave_lds_sync();
}

// Quotient of n < 2^30 by the divisor whose magic is (m, shift): exact
// (Granlund-Montgomery with a round-up multiplier, see divmagic()).
__device__ __forceinline__ u32 fast_div(u32 n, u64 m, int shift) {
    return (u32)(((u64)n * m) >> shift);
}

}  // namespace msda
