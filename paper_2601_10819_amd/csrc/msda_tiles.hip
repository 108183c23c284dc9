// The deterministic grad_feat reduction of the backward, after the
// samples' records are sorted by bilinear cell (msda_sort.hip): each 4x4 tile
// of pixels of a region visits the 5x5 cells whose samples touch it, in a
// fixed order, and adds w * cw * grad_out[anchor] of each sample's corners
// that fall in the tile to register accumulators; each sample's grad_out row
// is read once per tile it touches (about 1.6 times on average) instead of
// once per corner. The tile's records are split between its waves and the
// partial sums added in a fixed order, so grad_feat is bitwise reproducible;
// every pixel is written once, in FP32, BF16 or FP16 (rounded to nearest
// even), zeros where no sample lands.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "msda_common.h"

namespace msda {

template <int I>
using int_c = std::integral_constant<int, I>;

// f(int_c<0>{}), ..., f(int_c<N-1>{}): a loop whose index is a compile-time constant.
template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(int_c<I>{});
        static_for<N, I + 1>(f);
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
        // one rounding of the FP32 sum to the storage type
        auto rnd = [](float x) -> u32 {
            if constexpr (OT::kKind == 3) return f16_rne(x);
            else return bf16_rne(x);
        };
        uint16_t* p = static_cast<uint16_t*>(base) + elem;
        if constexpr (CPL == 4) {
            u32 lo, hi;
            if constexpr (OT::kKind == 3) {
                lo = rnd(acc[0]) | (rnd(acc[1]) << 16);
                hi = rnd(acc[2]) | (rnd(acc[3]) << 16);
            } else {
                lo = bf16x2_rne(acc[0], acc[1]);
                hi = bf16x2_rne(acc[2], acc[3]);
            }
            *reinterpret_cast<u32x2*>(p) = u32x2{lo, hi};
        } else {
#pragma unroll
            for (int i = 0; i < CPL; ++i) p[i] = (uint16_t)rnd(acc[i]);
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

// Tables of the tiled reduction for one batch item, from the shapes: the
// first cell of each region (regions in order, (H+1)(W+1) bilinear cells
// each and one for the region's samples outside the level) and,
// over processing slots (coarse levels first: slot o = (L-1-l)*N + n), the
// first tile and the region of each slot. One block of 256 threads; N*L <=
// 1024 regions, 4 per thread.
__global__ void __launch_bounds__(256) region_tables_kernel(const int32_t* shapes, int N, int L,
                                                            u32* cell_start, u32* tile_start,
                                                            u32* tile_region) {
    __shared__ u32 lds4[4];
    const int NL = N * L;
    u32 cells[4], tiles[4], sum_c = 0, sum_t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = 4 * threadIdx.x + k;
        cells[k] = tiles[k] = 0u;
        if (i < NL) {
            const u32 H = (u32)shapes[2 * i], W = (u32)shapes[2 * i + 1];
            cells[k] = (H + 1) * (W + 1) + 1;    // + the region's outside cell
            const int o = i;                     // slot o -> region r
            const int r = (o % N) * L + (L - 1 - o / N);
            const u32 Hr = (u32)shapes[2 * r], Wr = (u32)shapes[2 * r + 1];
            tiles[k] = ((Hr + kTileH - 1) / kTileH) * ((Wr + kTileW - 1) / kTileW);
        }
        sum_c += cells[k];
        sum_t += tiles[k];
    }
    u32 total_c, total_t;
    u32 run_c = block_inclusive_scan(sum_c, lds4, &total_c) - sum_c;
    u32 run_t = block_inclusive_scan(sum_t, lds4, &total_t) - sum_t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = 4 * threadIdx.x + k;
        if (i < NL) {
            cell_start[i] = run_c;
            tile_start[i] = run_t;
            tile_region[i] = (u32)((i % N) * L + (L - 1 - i / N));
        }
        run_c += cells[k];
        run_t += tiles[k];
    }
    if (threadIdx.x == 0) tile_start[NL] = total_t;
}

// One sample's corners that fall in the tile, added to the accumulators.
// The sample's cell sits at tile offset (DY, DX), so the corner -> pixel map
// is static: corners land on (DY-1, DX-1), (DY-1, DX), (DY, DX-1), (DY, DX).
// f holds the bilinear factors ((1-ly)(1-lx), (1-ly)lx, ly(1-lx), ly lx),
// computed once per record; each corner's weight is its factor times wv.
template <int DY, int DX, int TH, int TW, int CPL>
__device__ __forceinline__ void add_sample(float (&acc)[TH][TW][CPL], float4 f, float wv,
                                           const float* gv) {
    const float k00 = f.x * wv, k01 = f.y * wv;
    const float k10 = f.z * wv, k11 = f.w * wv;
    if constexpr (DY >= 1 && DX >= 1) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[DY - 1][DX - 1][i] = fmaf(k00, gv[i], acc[DY - 1][DX - 1][i]);
    }
    if constexpr (DY >= 1 && DX < TW) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[DY - 1][DX][i] = fmaf(k01, gv[i], acc[DY - 1][DX][i]);
    }
    if constexpr (DY < TH && DX >= 1) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[DY][DX - 1][i] = fmaf(k10, gv[i], acc[DY][DX - 1][i]);
    }
    if constexpr (DY < TH && DX < TW) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[DY][DX][i] = fmaf(k11, gv[i], acc[DY][DX][i]);
    }
}

// Dispatch on the cell position pos = DY * 5 + DX of a 4x4 tile's 5x5 cells
// (uniform within the lane group) to the static accumulation: a switch, which
// the compiler lowers to a jump table.
template <int CPL>
__device__ __forceinline__ void add_sample_at(int pos, float (&acc)[4][4][CPL], float4 f,
                                              float wv, const float* gv) {
#define MSDA_CELL_CASE(P) \
    case P: add_sample<(P) / 5, (P) % 5, 4, 4, CPL>(acc, f, wv, gv); break;
    switch (pos) {
        MSDA_CELL_CASE(0) MSDA_CELL_CASE(1) MSDA_CELL_CASE(2) MSDA_CELL_CASE(3) MSDA_CELL_CASE(4)
        MSDA_CELL_CASE(5) MSDA_CELL_CASE(6) MSDA_CELL_CASE(7) MSDA_CELL_CASE(8) MSDA_CELL_CASE(9)
        MSDA_CELL_CASE(10) MSDA_CELL_CASE(11) MSDA_CELL_CASE(12) MSDA_CELL_CASE(13)
        MSDA_CELL_CASE(14) MSDA_CELL_CASE(15) MSDA_CELL_CASE(16) MSDA_CELL_CASE(17)
        MSDA_CELL_CASE(18) MSDA_CELL_CASE(19) MSDA_CELL_CASE(20) MSDA_CELL_CASE(21)
        MSDA_CELL_CASE(22) MSDA_CELL_CASE(23) MSDA_CELL_CASE(24)
        default: break;
    }
#undef MSDA_CELL_CASE
}

// One sample of a statically known cell (DY, DX): the arithmetic of the
// switch's case (DY * 5 + DX).
template <int DY, int DX, int CPL>
__device__ __forceinline__ void cell_sample(float (&acc)[4][4][CPL], float4 f, float wv,
                                            const float* gv) {
    add_sample<DY, DX, 4, 4, CPL>(acc, f, wv, gv);
}

// Floats per record-table entry: the 4 bilinear factors, the anchor, the
// cell position, 2 spare, then the G weights (16-byte multiple, so the
// factors load as one vector).
__host__ __device__ inline int tile_entry_floats(int G) { return 8 + ((G + 3) & ~3); }

// Cell boundaries of a tile's TH+1 cell rows, (TW+2) per row.
constexpr int kBndPerGroup = (kTileH + 1) * (kTileW + 2);

// LDS bytes of the boundary slots: one per lane group of every wave.
__host__ __device__ inline size_t bnd_lds_bytes(int waves, int lps_shift) {
    const size_t groups = (size_t)waves * (size_t)(64 >> lps_shift);
    return (groups * kBndPerGroup * 4 + 15) & ~(size_t)15;
}

// Records handled per group of grad_out loads in flight.
constexpr int kGoBatch = 8;

// Everything one tile's reduction needs (from the single-call or the
// batched tables).
struct TileView {
    const u32* vals;            // sorted record indices (global sample indices)
    const u32* off;             // first record of each cell
    const float2* frac;         // per record (global index): (lx, ly)
    const float* w;             // the scene's weights [S][G]
    const float* grad_out;      // the scene's grad_out [A][C]
    void* grad_feat;            // the scene's grad_feat
    size_t row_base;            // first grad_feat row of the tile's batch item
    u32 nrec;                   // records in the sort (all scenes)
    u32 sample_offset;          // first record index of the scene
    u32 sample_count;           // records of the scene
    u32 cbase;                  // first cell of the tile's region
    int H, W, start;            // the region
    int ty, tx;                 // the tile's first pixel
    int C, G;
    u64 magic;                  // scene-local sample -> anchor
    int magic_shift;
    const float* vscale;        // [anchor][N] per-view weight factor, or nullptr
    int N, L;
    bool active;
    bool w16;                   // G % 4 == 0 and w 16-byte aligned
};

// grad_out row of a whole-wave record: the anchor (a table entry every lane
// reads at the same address) taken as uniform, so the row address is scalar
// arithmetic and each lane adds only its channel offset.
__device__ __forceinline__ const float* go_row(const TileView& v, float anchor_bits) {
    const u32 an = (u32)uniform((int)__float_as_uint(anchor_bits));
    return v.grad_out + (size_t)an * (u32)v.C;
}

// The reduction of one tile by a group of lps lanes (grp-th group of its
// wave, lane sl within it); `waves` waves of the block share its records,
// this wave being the wt-th of them (waves == 1: wt == 0, and the other
// waves of the block reduce tiles of their own).
// CELLS (whole-wave groups only): walk each chunk's records cell by cell in
// a static loop over the tile's 5x5 cells, so every record's corner ->
// pixel map is a compile-time constant (no per-record dispatch); records of
// a cell are consecutive in the sorted order, so the visiting order, and
// the sums, are those of the flat walk.
template <class OT, int CPL, bool WHOLE_WAVE, bool CELLS, int QB = 4>
__device__ __forceinline__ void tile_reduce(const TileView& v, const int lps, const int spw,
                                            const int grp, const int sl, const int waves,
                                            const int wt,
                                            u32* bnd_lds, float* work) {
    constexpr int TH = kTileH, TW = kTileW;
    // the wave index is uniform: chunk bounds and cell runs below stay scalar
    const int lane = threadIdx.x & 63, wave = uniform((int)(threadIdx.x >> 6));
    const int stride = tile_entry_floats(v.G);      // floats per record-table entry
    float* tab = work + (size_t)wave * 64 * stride + (size_t)(lane - sl) * stride;
    const bool active = v.active;
    const int H = v.H, W = v.W, ty = v.ty, tx = v.tx;
    const u32 cbase = v.cbase;
    const int c0 = sl * CPL;
    const int g = c0 / (v.C / v.G);

    // The tile's cells are TH+1 rows of TW+1 consecutive cells; each row's
    // records are one contiguous range of the sorted order. The group stores
    // the (TH+1) x (TW+2) cell boundaries of those rows in its LDS slot.
    constexpr int NB = kBndPerGroup;
    u32* bslot = bnd_lds + ((size_t)wave * spw + (size_t)grp) * NB;
    for (int k = sl; k < NB; k += lps) {
        const int dy = k / (TW + 2), dx = k % (TW + 2);
        u32 bv = 0u;
        if (active && ty + dy <= H) {
            // cells past W+1 clamp to the row's end
            const u32 cell = cbase + (u32)(ty + dy) * (u32)(W + 1) + (u32)min(tx + dx, W + 1);
            bv = min(v.off[cell], v.nrec);
        }
        bslot[k] = bv;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    u32 rs[TH + 1], rn[TH + 1];                     // row range start and length
    u32 total = 0;
#pragma unroll
    for (int dy = 0; dy <= TH; ++dy) {
        const u32 a0 = bslot[dy * (TW + 2)];
        const u32 a1 = bslot[dy * (TW + 2) + TW + 1];
        rs[dy] = a0;
        rn[dy] = active && ty + dy <= H && a1 > a0 ? a1 - a0 : 0u;
        total += rn[dy];
    }

    float acc[TH][TW][CPL];
#pragma unroll
    for (int py = 0; py < TH; ++py)
#pragma unroll
        for (int px = 0; px < TW; ++px)
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[py][px][i] = 0.f;

    // The tile's records as one flat list, in chunks of lps; chunk k goes to
    // wave k % waves. Each lane of the group fills one table entry (all the
    // chunk's loads in flight together), then the group walks the chunk.
    for (u32 base = (u32)(wt * lps); base < total; base += (u32)(waves * lps)) {
        const int n = (int)min((u32)lps, total - base);
        if (sl < n) {
            // flat index -> (row dy, sorted position e) -> cell position dx
            u32 f = base + (u32)sl;
            int dy = 0;
#pragma unroll
            for (int k = 0; k < TH; ++k)
                if (dy == k && f >= rn[k]) { f -= rn[k]; dy = k + 1; }
            u32 e = rs[0] + f;
#pragma unroll
            for (int k = 1; k <= TH; ++k)
                if (dy == k) e = rs[k] + f;
            int dx = 0;
#pragma unroll
            for (int k = 1; k <= TW; ++k)
                if (e >= bslot[dy * (TW + 2) + k]) dx = k;
            const u32 s = min(v.vals[e], v.nrec - 1u);
            const float2 fr = v.frac[s];
            float* ent = tab + sl * stride;
            // the scene-local sample (clamped into the scene: an inconsistent
            // sort could only give wrong sums, never a read outside it)
            const u32 ls = s - v.sample_offset < v.sample_count ? s - v.sample_offset : 0u;
            const float* ws = v.w + (size_t)ls * v.G;
            const u32 an = fast_div(ls, v.magic, v.magic_shift);
            if (v.vscale) {
                // the fused form: the sample's weights times its view's factor
                const u32 n = (ls / (u32)v.L) % (u32)v.N;
                const float sc = v.vscale[(size_t)an * v.N + n];
                for (int k = 0; k < v.G; ++k) ent[8 + k] = ws[k] * sc;
            } else if (v.w16) {
                // rows of G % 4 == 0 floats from a 16-byte aligned base: 16-byte
                // loads and LDS stores
                const float4* ws4 = reinterpret_cast<const float4*>(ws);
                float4* e4 = reinterpret_cast<float4*>(ent + 8);
                for (int k = 0; k < (v.G >> 2); ++k) e4[k] = ws4[k];
            } else {
                for (int k = 0; k < v.G; ++k) ent[8 + k] = ws[k];
            }
            const float hx = 1.f - fr.x, hy = 1.f - fr.y;
            *reinterpret_cast<float4*>(ent) =
                make_float4(hy * hx, hy * fr.x, fr.y * hx, fr.y * fr.x);
            ent[4] = __uint_as_float(an);
            ent[5] = __int_as_float(dy * (TW + 1) + dx);
        }
        // LDS accesses of one wave are performed in order; keep the compiler
        // from hoisting the reads above the writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if constexpr (CELLS && WHOLE_WAVE) {
            // flat index of each row's first record, then each cell's run
            // clipped to this chunk [base, base + n)
            u32 f0 = 0;
            static_for<TH + 1>([&](auto dyc) {
                constexpr int DY = decltype(dyc)::value;
                const u32 rlen = (u32)uniform((int)rn[DY]);
                if (rlen) {
                    const u32 rstart = (u32)uniform((int)rs[DY]);
                    static_for<TW + 1>([&](auto dxc) {
                        constexpr int DX = decltype(dxc)::value;
                        const u32 e0 = (u32)uniform((int)bslot[DY * (TW + 2) + DX]);
                        const u32 e1 = (u32)uniform((int)bslot[DY * (TW + 2) + DX + 1]);
                        const u32 lo = max(f0 + (e0 - rstart), base);
                        const u32 hi = min(f0 + (e1 - rstart), base + (u32)n);
                        int qq = (int)lo - (int)base;
                        const int qe = (int)hi - (int)base;
                        for (; qq + QB <= qe; qq += QB) {
                            float gv[QB][CPL];
#pragma unroll
                            for (int k = 0; k < QB; ++k) {
                                const float* ent = tab + (qq + k) * stride;
                                load_go<CPL>(go_row(v, ent[4]) + (u32)c0, gv[k]);
                            }
#pragma unroll
                            for (int k = 0; k < QB; ++k) {
                                const float* ent = tab + (qq + k) * stride;
                                cell_sample<DY, DX, CPL>(
                                    acc, *reinterpret_cast<const float4*>(ent), ent[8 + g], gv[k]);
                            }
                        }
                        for (; qq < qe; ++qq) {
                            const float* ent = tab + qq * stride;
                            float gv[CPL];
                            load_go<CPL>(go_row(v, ent[4]) + (u32)c0, gv);
                            cell_sample<DY, DX, CPL>(acc, *reinterpret_cast<const float4*>(ent),
                                                     ent[8 + g], gv);
                        }
                    });
                }
                f0 += rlen;
            });
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            continue;
        }
        int q = 0;
        for (; q + kGoBatch <= n; q += kGoBatch) {
            float gv[kGoBatch][CPL];
#pragma unroll
            for (int k = 0; k < kGoBatch; ++k) {
                const float* ent = tab + (q + k) * stride;
                load_go<CPL>(v.grad_out + (size_t)__float_as_uint(ent[4]) * v.C + c0, gv[k]);
            }
#pragma unroll
            for (int k = 0; k < kGoBatch; ++k) {
                const float* ent = tab + (q + k) * stride;
                add_sample_at<CPL>(__float_as_int(ent[5]), acc,
                                   *reinterpret_cast<const float4*>(ent), ent[8 + g], gv[k]);
            }
        }
        for (; q < n; ++q) {
            const float* ent = tab + q * stride;
            float gv[CPL];
            load_go<CPL>(v.grad_out + (size_t)__float_as_uint(ent[4]) * v.C + c0, gv);
            add_sample_at<CPL>(__float_as_int(ent[5]), acc, *reinterpret_cast<const float4*>(ent),
                               ent[8 + g], gv);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // partial sums of the waves, added pairwise in a fixed tree order:
    // wave w += wave w + h for h = waves/2, waves/4, ..., 1
    if (waves > 1) {
        constexpr int E = TH * TW * CPL;
        float* part = work;
        __syncthreads();                             // record tables are dead from here on
        for (int h = waves >> 1; h >= 1; h >>= 1) {
            if (wt >= h && wt < 2 * h) {
#pragma unroll
                for (int py = 0; py < TH; ++py)
#pragma unroll
                    for (int px = 0; px < TW; ++px)
#pragma unroll
                        for (int i = 0; i < CPL; ++i)
                            part[((wt - h) * E + (py * TW + px) * CPL + i) * 64 + lane] =
                                acc[py][px][i];
            }
            __syncthreads();
            if (wt < h) {
#pragma unroll
                for (int py = 0; py < TH; ++py)
#pragma unroll
                    for (int px = 0; px < TW; ++px)
#pragma unroll
                        for (int i = 0; i < CPL; ++i)
                            acc[py][px][i] += part[(wt * E + (py * TW + px) * CPL + i) * 64 + lane];
            }
            __syncthreads();
        }
    }
    if (wt != 0 || !active) return;
    const int start = v.start;
#pragma unroll
    for (int py = 0; py < TH; ++py) {
#pragma unroll
        for (int px = 0; px < TW; ++px) {
            const int y = ty + py, x = tx + px;
            if (y < H && x < W) {
                const size_t row = v.row_base + (size_t)(start + y * W + x);
                store_row<OT, CPL>(v.grad_feat, row * (size_t)v.C + (size_t)c0, acc[py][px]);
            }
        }
    }
}

// The tile of id gt (ids run over batch items first, then processing slots
// within [tile_begin, tile_end)) by `waves` waves of the block, this wave the
// wt-th of them.
template <class OT, int CPL, bool WHOLE_WAVE, bool CELLS, int QB = 4>
__device__ __forceinline__ void gfeat_tile_body(const TileArgs& t, const u32 gt, const int waves,
                                                const int wt) {
    static_assert(kTileH == 4 && kTileW == 4, "the cell dispatch is written for 4x4 tiles");
    // LDS: per lane group its tile's cell boundaries; per wave a record table
    // (64 entries of bilinear factors, anchor, cell position and G weights);
    // after the records, the waves' partial sums reuse the record tables'
    // space.
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TH = kTileH, TW = kTileW;
    const int lane = threadIdx.x & 63;
    const int lps = WHOLE_WAVE ? 64 : 1 << t.lps_shift;
    const int spw = WHOLE_WAVE ? 1 : 64 >> t.lps_shift;
    const int grp = WHOLE_WAVE ? 0 : lane >> t.lps_shift;
    const int sl = WHOLE_WAVE ? lane : lane & (lps - 1);   // lane within its tile's group
    u32* bnd_lds = reinterpret_cast<u32*>(smem_raw);
    float* work = reinterpret_cast<float*>(smem_raw +
                                           bnd_lds_bytes((int)(blockDim.x >> 6), t.lps_shift));

    const u32 span = t.tile_end - t.tile_begin;
    TileView v;
    v.active = gt < span * (u32)t.B;
    const u32 tt = t.tile_begin + (v.active ? gt / (u32)t.B : 0u);
    const int b = v.active ? (int)(gt % (u32)t.B) : 0;
    int lo = 0, hi = t.NL - 1;                      // last slot with tile_start <= tt
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.tile_start[mid] <= tt) lo = mid; else hi = mid - 1;
    }
    const int r = (int)t.tile_region[lo];
    v.H = t.shapes[2 * r];
    v.W = t.shapes[2 * r + 1];
    v.start = t.starts[r];
    const u32 lt = tt - t.tile_start[lo];
    const u32 tpr = (u32)(v.W + TW - 1) / TW;
    v.ty = (int)(lt / tpr) * TH;
    v.tx = (int)(lt % tpr) * TW;
    v.cbase = (u32)b * t.cells_per_item + t.cell_start[r];
    v.row_base = (size_t)b * (size_t)t.R;
    v.vals = t.vals;
    v.off = t.off;
    v.frac = t.frac;
    v.w = t.w;
    v.w16 = (t.G & 3) == 0 && ((uintptr_t)t.w & 15) == 0;
    v.grad_out = t.grad_out;
    v.grad_feat = t.grad_feat;
    v.nrec = t.nrec;
    v.sample_offset = 0;
    v.sample_count = t.nrec;
    v.C = t.C;
    v.G = t.G;
    v.magic = t.magic;
    v.magic_shift = t.magic_shift;
    v.vscale = t.view_scale;
    v.N = t.N;
    v.L = t.L;
    tile_reduce<OT, CPL, WHOLE_WAVE, CELLS, QB>(v, lps, spw, grp, sl, waves, wt, bnd_lds, work);
}

// Whole-wave lane groups (C = 64 * CPL): at most 128 VGPRs, i.e. 4 waves per
// SIMD. The reduction waits on record and grad_out loads, and a fourth wave
// hides more of that than the few registers it spills cost (measured on the
// 64-camera scene: light tiles 0.28 -> 0.24 ms, coarse 0.19 -> 0.18 ms).
// Narrower groups keep the compiler's choice (they would spill heavily).
// QB: records whose grad_out rows are loaded together in the cell walk; 2
// for the one-wave light tiles (fewer registers: no spills at 128), 4 for
// the coarse tiles (measured: light 0.248 -> 0.234 ms with 2, coarse 0.180
// -> 0.191 ms).
//
// One launch for both kinds of tiles: the coarse tiles (ids below
// (tile_split - tile_begin) * B) first, a block of 4 waves each, then the
// light ones, 4 per block, one wave each; the light blocks fill the CUs
// around the long coarse ones instead of waiting for them to drain.
constexpr int kTileBlockWaves = 4;

template <class OT, int CPL>
__global__ void __launch_bounds__(64 * kTileBlockWaves) __attribute__((amdgpu_waves_per_eu(4, 8)))
gfeat_tile_kernel(TileArgs t) {
    constexpr int BW = kTileBlockWaves;
    const u32 heavy = (t.tile_split - t.tile_begin) * (u32)t.B;
    const int wave = uniform((int)(threadIdx.x >> 6));
    if (blockIdx.x < heavy)
        gfeat_tile_body<OT, CPL, true, true, 4>(t, blockIdx.x, BW, wave);
    else
        gfeat_tile_body<OT, CPL, true, true, 2>(
            t, heavy + (blockIdx.x - heavy) * (u32)BW + (u32)wave, 1, 0);
}

// Narrower lane groups: spw tiles per wave, t.waves waves sharing them.
template <class OT, int CPL>
__global__ void __launch_bounds__(256) gfeat_tile_group_kernel(TileArgs t) {
    const int spw = 64 >> t.lps_shift;
    const u32 gt = blockIdx.x * (u32)spw + (u32)((threadIdx.x & 63) >> t.lps_shift);
    gfeat_tile_body<OT, CPL, false, false>(t, gt, t.waves, (int)(threadIdx.x >> 6));
}

// Batched tiled reduction: tiles of all scenes' regions in slot order; the
// tile of id gt (from tile_begin) by `waves` waves, this wave the wt-th.
template <class OT, int CPL, bool WHOLE_WAVE, int QB = 4>
__device__ __forceinline__ void gfeat_tile_batched_body(const BatchArgs& b, const u32 gt,
                                                        const int waves, const int wt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TH = kTileH, TW = kTileW;
    const int lane = threadIdx.x & 63;
    const int lps = WHOLE_WAVE ? 64 : 1 << b.lps_shift;
    const int spw = WHOLE_WAVE ? 1 : 64 >> b.lps_shift;
    const int grp = WHOLE_WAVE ? 0 : lane >> b.lps_shift;
    const int sl = WHOLE_WAVE ? lane : lane & (lps - 1);
    u32* bnd_lds = reinterpret_cast<u32*>(smem_raw);
    float* work = reinterpret_cast<float*>(smem_raw +
                                           bnd_lds_bytes((int)(blockDim.x >> 6), b.lps_shift));

    TileView v;
    v.active = gt < b.tile_end - b.tile_begin;
    const u32 tt = b.tile_begin + (v.active ? gt : 0u);
    const int slot = scene_of(b.t.tile_start, (int)b.total_regions, tt);
    const int s = (int)b.t.slot_scene[slot];
    const int r = (int)b.t.slot_region[slot];
    const msda_scene& sc = b.scenes[s];
    v.H = sc.spatial_shapes[2 * r];
    v.W = sc.spatial_shapes[2 * r + 1];
    v.start = sc.level_start_index[r];
    const u32 lt = tt - b.t.tile_start[slot];
    const u32 tpr = (u32)(v.W + TW - 1) / TW;
    v.ty = (int)(lt / tpr) * TH;
    v.tx = (int)(lt % tpr) * TW;
    v.cbase = b.t.cell_start[b.t.region_start[s] + (u32)r];
    v.row_base = 0;
    v.vals = b.vals;
    v.off = b.off;
    v.frac = b.rec_frac;
    v.w = b.w32 ? b.w32 + (size_t)b.t.sample_start[s] * (size_t)b.G : sc.weights;
    v.w16 = (b.G & 3) == 0 && ((uintptr_t)v.w & 15) == 0;
    v.grad_out = sc.grad_out;
    v.grad_feat = sc.grad_feat;
    v.nrec = b.total_samples;
    v.sample_offset = b.t.sample_start[s];
    v.sample_count = b.t.sample_start[s + 1] - b.t.sample_start[s];
    v.C = b.C;
    v.G = b.G;
    v.magic = b.t.magic[s];
    v.magic_shift = (int)b.t.magic_shift[s];
    v.vscale = nullptr;
    v.N = 1;
    v.L = 1;
    tile_reduce<OT, CPL, WHOLE_WAVE, WHOLE_WAVE, QB>(v, lps, spw, grp, sl, waves, wt, bnd_lds,
                                                     work);
}

// As gfeat_tile_kernel: the heavy tiles ([tile_begin, tile_split)) 4 waves
// each, then the light ones 4 per block, one wave each. Both walk with 2
// grad_out rows in flight: with the batch's scene lookups, 4 for the heavy
// tiles spilled 64 bytes under the 128-VGPR cap (the 12-scene batch's step:
// 9.37 ms with 4, 9.22 ms with 2).
template <class OT, int CPL>
__global__ void __launch_bounds__(64 * kTileBlockWaves) __attribute__((amdgpu_waves_per_eu(4, 8)))
gfeat_tile_batched_kernel(BatchArgs b) {
    constexpr int BW = kTileBlockWaves;
    const u32 heavy = b.tile_split - b.tile_begin;
    const int wave = uniform((int)(threadIdx.x >> 6));
    if (blockIdx.x < heavy)
        gfeat_tile_batched_body<OT, CPL, true, 2>(b, blockIdx.x, BW, wave);
    else
        gfeat_tile_batched_body<OT, CPL, true, 2>(
            b, heavy + (blockIdx.x - heavy) * (u32)BW + (u32)wave, 1, 0);
}

template <class OT, int CPL>
__global__ void __launch_bounds__(256) gfeat_tile_batched_group_kernel(BatchArgs b) {
    const int spw = 64 >> b.lps_shift;
    const u32 gt = blockIdx.x * (u32)spw + (u32)((threadIdx.x & 63) >> b.lps_shift);
    gfeat_tile_batched_body<OT, CPL, false>(b, gt, b.waves, (int)(threadIdx.x >> 6));
}

// ---------------------------------------------------------------- launchers

// LDS of a tile block of `waves` waves: the cell boundaries, then the larger
// of the record tables and the partial sums (coarse tiles: waves/2 halves of
// a tile's accumulators).
template <int CPL>
static size_t tile_lds_bytes(int waves, int lps_shift, int G, bool coarse) {
    const size_t part = coarse ? (size_t)(waves / 2) * kTileH * kTileW * CPL * 64 * 4 : 0;
    const size_t tables = (size_t)waves * 64 * tile_entry_floats(G) * sizeof(float);
    return bnd_lds_bytes(waves, lps_shift) + (part > tables ? part : tables);
}

// Whole-wave groups: one launch of gfeat_tile_kernel over [tile_begin,
// tile_end) (coarse up to tile_split). Narrower groups: two launches of the
// group kernel, 4 waves per coarse tile group, 1 per light one.
template <class OT, int CPL>
static hipError_t tile_launch(const TileArgs& t0, hipStream_t s) {
    const u32 B = (u32)t0.B;
    if (t0.lps_shift == 6) {
        const u32 heavy = (t0.tile_split - t0.tile_begin) * B;
        const u32 light = (t0.tile_end - t0.tile_split) * B;
        constexpr int BW = kTileBlockWaves;
        const u32 blocks = heavy + (light + BW - 1) / BW;
        if (blocks == 0) return hipSuccess;
        const size_t lds = tile_lds_bytes<CPL>(BW, 6, t0.G, heavy > 0);
        mark_begin("gfeat_tile_kernel", s);
        hipLaunchKernelGGL((gfeat_tile_kernel<OT, CPL>), dim3(blocks), dim3(64 * BW), lds, s,
                           t0);
        mark_end(s);
        return hipGetLastError();
    }
    const u32 split[3] = {t0.tile_begin, t0.tile_split, t0.tile_end};
    for (int part = 0; part < 2; ++part) {
        TileArgs t = t0;
        t.tile_begin = split[part];
        t.tile_end = split[part + 1];
        t.waves = part == 0 ? 4 : 1;
        const u32 spw = 64u >> t.lps_shift;
        const u32 blocks = ((t.tile_end - t.tile_begin) * B + spw - 1) / spw;
        if (blocks == 0) continue;
        const size_t lds = tile_lds_bytes<CPL>(t.waves, t.lps_shift, t.G, t.waves > 1);
        mark_begin(t.waves > 1 ? "gfeat_tile_kernel_coarse" : "gfeat_tile_kernel", s);
        hipLaunchKernelGGL((gfeat_tile_group_kernel<OT, CPL>), dim3(blocks),
                           dim3(64 * t.waves), lds, s, t);
        mark_end(s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class OT, int CPL>
static hipError_t tile_batched_launch(const BatchArgs& b0, hipStream_t s) {
    if (b0.lps_shift == 6) {
        const u32 heavy = b0.tile_split - b0.tile_begin;
        const u32 light = b0.tile_end - b0.tile_split;
        constexpr int BW = kTileBlockWaves;
        const u32 blocks = heavy + (light + BW - 1) / BW;
        if (blocks == 0) return hipSuccess;
        const size_t lds = tile_lds_bytes<CPL>(BW, 6, b0.G, heavy > 0);
        mark_begin("gfeat_tile_batched", s);
        hipLaunchKernelGGL((gfeat_tile_batched_kernel<OT, CPL>), dim3(blocks), dim3(64 * BW), lds,
                           s, b0);
        mark_end(s);
        return hipGetLastError();
    }
    const u32 split[3] = {b0.tile_begin, b0.tile_split, b0.tile_end};
    for (int part = 0; part < 2; ++part) {
        BatchArgs b = b0;
        b.tile_begin = split[part];
        b.tile_end = split[part + 1];
        b.waves = part == 0 ? 4 : 1;
        const u32 spw = 64u >> b.lps_shift;
        const u32 blocks = (b.tile_end - b.tile_begin + spw - 1) / spw;
        if (blocks == 0) continue;
        const size_t lds = tile_lds_bytes<CPL>(b.waves, b.lps_shift, b.G, b.waves > 1);
        mark_begin(b.waves > 1 ? "gfeat_tile_batched_coarse" : "gfeat_tile_batched", s);
        hipLaunchKernelGGL((gfeat_tile_batched_group_kernel<OT, CPL>), dim3(blocks),
                           dim3(64 * b.waves), lds, s, b);
        mark_end(s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_gfeat_tiles_batched(const BatchArgs& b, int out_dtype, int cpl, hipStream_t s) {
    switch (out_dtype * 100 + cpl) {
        case kF32 * 100 + 1: return tile_batched_launch<TF32, 1>(b, s);
        case kF32 * 100 + 2: return tile_batched_launch<TF32, 2>(b, s);
        case kF32 * 100 + 4: return tile_batched_launch<TF32, 4>(b, s);
        case kBF16 * 100 + 1: return tile_batched_launch<TBF16, 1>(b, s);
        case kF16 * 100 + 1: return tile_batched_launch<TF16, 1>(b, s);
        case kBF16 * 100 + 2: return tile_batched_launch<TBF16, 2>(b, s);
        case kF16 * 100 + 2: return tile_batched_launch<TF16, 2>(b, s);
        case kBF16 * 100 + 4: return tile_batched_launch<TBF16, 4>(b, s);
        case kF16 * 100 + 4: return tile_batched_launch<TF16, 4>(b, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gfeat_tiles(const TileArgs& t, int out_dtype, int cpl, hipStream_t s) {
    switch (out_dtype * 100 + cpl) {
        case kF32 * 100 + 1: return tile_launch<TF32, 1>(t, s);
        case kF32 * 100 + 2: return tile_launch<TF32, 2>(t, s);
        case kF32 * 100 + 4: return tile_launch<TF32, 4>(t, s);
        case kBF16 * 100 + 1: return tile_launch<TBF16, 1>(t, s);
        case kF16 * 100 + 1: return tile_launch<TF16, 1>(t, s);
        case kBF16 * 100 + 2: return tile_launch<TBF16, 2>(t, s);
        case kF16 * 100 + 2: return tile_launch<TF16, 2>(t, s);
        case kBF16 * 100 + 4: return tile_launch<TBF16, 4>(t, s);
        case kF16 * 100 + 4: return tile_launch<TF16, 4>(t, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_region_tables(const int32_t* shapes, int32_t N, int32_t L, u32* cell_start,
                                u32* tile_start, u32* tile_region, hipStream_t s) {
    mark_begin("region_tables", s);
    hipLaunchKernelGGL(region_tables_kernel, dim3(1), dim3(256), 0, s, shapes, N, L, cell_start,
                       tile_start, tile_region);
    mark_end(s);
    return hipGetLastError();
}

}  // namespace msda
