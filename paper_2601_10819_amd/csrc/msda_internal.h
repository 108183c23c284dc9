// Internal interface between the C-ABI layer (msda_api.cpp) and the HIP
// kernels (msda_fwd.hip, msda_bwd.hip, msda_sort.hip, msda_util.hip). Not
// installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/msda.h"

namespace msda {

// Byte offset used for a corner outside its level: at or beyond the end of
// every feature resource (a batch item is at most kOOB bytes, one buffer
// resource with 32-bit offsets), so a buffer load returns zeros; a lane adds
// at most one row (<= kMaxRowBytes) to it, which cannot wrap past 2^32.
constexpr uint32_t kMaxRowBytes = 4096u;
constexpr uint32_t kOOB = 0xFFFFE000u;

// Everything one forward/backward launch needs. Pointers are device memory.
struct OpArgs {
    const void* feat;             // [B][R][C], dtype below
    const int32_t* shapes;        // [N][L][2] (H, W)
    const int32_t* starts;        // [N][L]
    const float* loc;             // [B][A][P][N][2]
    const float* w;               // [B][A][P][N][L][G]
    const float* level_scale;     // [L] (FP8) or nullptr
    const float* grad_out;        // [B][A][C] (backward)
    float* out;                   // [B][A][C] (forward)
    float* gfeat_acc;             // atomic grad_feat: FP32 [B][R][C] accumulator, or nullptr
    uint32_t* rec_key;            // sorted grad_feat: [S] bilinear-cell keys, or nullptr
    float2* rec_frac;             // sorted grad_feat: [S] (lx, ly) bilinear fractions
    const uint32_t* cell_start;   // [N*L] first cell of each region (sorted grad_feat)
    uint32_t cells_per_item;      // cells of one batch item: sum of (H+1)(W+1)
    uint32_t cell_offset;         // added to every cell key (a scene's place in a batch)
    uint32_t no_cell;             // key of a sample outside its level (sorts last)
    uint32_t sample_offset;       // added to every record index
    float* grad_loc;              // or nullptr
    float* grad_w;                // or nullptr
    const float2* wstats;         // forward: w holds logits; per (b, a, g) (max, 1/sum of exp)
    int32_t w_bf16;               // forward: w holds bfloat16 bit patterns
    int32_t B, N, L, A, P, C, G;
    int64_t R;
    uint32_t batch_bytes;         // R * C * sizeof(feat element) (<= kOOB, under 4 GiB)
    int32_t lps_shift;            // log2(lanes per sample) = log2(C / chans_per_lane)
    int32_t pairs_per_chunk;      // (keypoint, camera) pairs staged per wave step
    // Bucketed records (dense single call): 0, or A*P -- the record of
    // sample (b, a, p, n, l) then goes to bucket (b, n, l) at a*P + p, its
    // key the local cell of region (n, l) (see launch_bucket_sort).
    uint32_t rec_bucket_ap;
    // Backward view order: cameras of one anchor per wave (>= 1).
    int32_t view_cams;
};

// The tiled grad_feat reduction over records sorted by bilinear cell.
// Tiles are kTileH x kTileW pixels of one region; processing slot o covers
// region tile_region[o], regions ordered coarse levels first.
constexpr int kTileH = 4, kTileW = 4;

struct TileArgs {
    const uint32_t* vals;         // sample indices, sorted by cell (stable)
    const uint32_t* off;          // [B * cells_per_item + 1] first record of each cell
    const float2* frac;           // [S] (lx, ly)
    const float* w;               // weights, [S][G]
    const float* grad_out;        // [B*A][C]
    void* grad_feat;              // [B][R][C], FP32 or BF16
    const int32_t* shapes;        // [N*L][2]
    const int32_t* starts;        // [N*L]
    const uint32_t* cell_start;   // [N*L]
    const uint32_t* tile_start;   // [N*L + 1], by processing slot
    const uint32_t* tile_region;  // [N*L], region of each processing slot
    const float* view_scale;      // [B*A][N] per-view weight factor (fused form), or nullptr
    int32_t N, L;                 // cameras and levels (to find a sample's view)
    uint32_t tiles_per_item;
    // the tiles of each batch item (slot order) to reduce: [tile_begin,
    // tile_split) coarse (4 waves each), [tile_split, tile_end) light
    uint32_t tile_begin, tile_split, tile_end;
    uint32_t cells_per_item;
    uint32_t nrec;                // S (records, one per sample)
    int32_t NL, B, C, G;
    int64_t R;
    int32_t lps_shift;            // log2(C / chans_per_lane)
    int32_t waves;                // narrower lane groups: waves sharing each tile's records (set by the launcher)
    uint64_t magic;               // sample -> anchor: s / (P*N*L) == (s * magic) >> magic_shift
    int32_t magic_shift;
};

// Batched form: tables over all scenes, built on the device from the scene
// table by batch_tables_kernel. Regions are numbered scene by scene (scene
// s owns regions [region_start[s], region_start[s+1]), camera-major); slots
// order the regions for the tiled reduction: heavy (coarse) levels first,
// then by level (coarsest first), scene and camera.
constexpr int kMaxBatchScenes = 256;
constexpr int kMaxBatchRegions = 4096;

struct BatchTables {
    uint32_t* anchor_start;       // [S+1] first anchor (over all scenes) of each scene
    uint32_t* sample_start;       // [S+1] first sample / record of each scene
    uint32_t* region_start;       // [S+1] first region of each scene
    uint32_t* cell_start;         // [regions] first cell of each region (global)
    uint32_t* slot_scene;         // [regions] scene of each slot
    uint32_t* slot_region;        // [regions] region (within its scene) of each slot
    uint32_t* tile_start;         // [regions + 1] first tile of each slot
    uint64_t* magic;              // [S] sample -> anchor division by P*Ncam*L
    uint32_t* magic_shift;        // [S]
};

struct BatchArgs {
    const msda_scene* scenes;     // device scene table
    int32_t S, L, P, C, G;
    const float* level_scale;
    BatchTables t;
    uint32_t total_anchors;
    uint32_t total_samples;
    uint32_t total_cells;
    uint32_t total_regions;
    int32_t lps_shift;            // log2(C / chans_per_lane)
    int32_t pairs_per_chunk;
    int32_t max_regions_per_scene;   // LDS sizing of the geometry table
    int32_t view_cams;            // view order: cameras of a row at most (geometry slice)
    uint32_t* rec_key;            // backward, grad_feat records (or nullptr)
    float2* rec_frac;
    int32_t rec_bucketed;         // records written per (scene, region) bucket (launch_bucket_sort_batched)
    // weight flags: forward, softmax statistics of every anchor (scenes in
    // order; w holds logits) and BF16 weights; backward, FP32 weights of
    // every sample (scenes in order), read in place of each scene's weights
    const float2* wstats;
    int32_t w_bf16;
    const float* w32;
    // tiled reduction
    const uint32_t* vals;
    const uint32_t* off;
    int32_t waves;                // narrower lane groups: as TileArgs::waves
    uint32_t tile_begin, tile_split, tile_end;  // as TileArgs
};

enum FeatType { kF32 = 0, kBF16 = 1, kFP8 = 2, kF16 = 3 };

// Keypoint projection (device pointers).
struct ProjArgs {
    const float* anchors;         // [B][A][10] x, y, z, w, l, h, yaw, vx, vy, vz
    const float* keypoints;       // [B][A][P][3] box-frame offsets in units of (w, l, h)
    const float* projection;      // [B][N][3][4]
    const int32_t* image_hw;      // [N][2] (H, W) pixels
    float* loc;                   // [B][A][P][N][2]
    uint8_t* visible;             // [B][A][N]
    int32_t B, A, P, N;
    float dt;
};

// ---------------------------------------------------------------- view order
//
// In view order the work of a call -- every (view, anchor) item, a view
// being one (batch item, camera), P*L samples each -- is cut, view-major,
// into kSlots contiguous ranges of equal size. Slot x runs on the workgroups
// whose index is x modulo kSlots: the hardware hands workgroups to the
// chip's kSlots XCDs round-robin, so slot x stays on one XCD and its L2
// holds the pyramids of the few cameras the slot is working through instead
// of every camera's. A wave takes one "row" of its slot: one anchor of a
// batch item the slot touches, over the anchor's views inside the slot
// (possibly none at the slot's edges).
constexpr int kSlots = 8;

struct SlotSpan {
    int64_t lo, hi;               // items [lo, hi), item = (b*N + n)*A + a
    int32_t b_first, b_last;      // batch items touched (b_last < b_first: none)
};

__host__ __device__ inline SlotSpan slot_span(int x, int B, int N, int A) {
    const int64_t T = (int64_t)B * N * A;
    SlotSpan s;
    s.lo = T * x / kSlots;
    s.hi = T * (x + 1) / kSlots;
    if (s.hi <= s.lo) {
        s.b_first = 1;
        s.b_last = 0;
    } else {
        s.b_first = (int32_t)(s.lo / A / N);
        s.b_last = (int32_t)((s.hi - 1) / A / N);
    }
    return s;
}

// Rows of slot x: (batch items touched) * A.
__host__ __device__ inline int64_t slot_rows(const SlotSpan& s, int A) {
    return s.b_last < s.b_first ? 0 : (int64_t)(s.b_last - s.b_first + 1) * A;
}

struct ViewRow {
    int32_t b, a;                 // batch item and anchor
    int32_t n_lo, nv;             // cameras [n_lo, n_lo + nv) of this row (nv may be 0)
};

// Row r (< slot_rows) of slot span s.
__host__ __device__ inline ViewRow view_row(const SlotSpan& s, int64_t r, int N, int A) {
    ViewRow v;
    v.b = s.b_first + (int32_t)(r / A);
    v.a = (int32_t)(r % A);
    // items of anchor a lie at views v with v*A + a in [lo, hi)
    int64_t v0 = (s.lo - v.a + A - 1) / A, v1 = (s.hi - v.a + A - 1) / A;
    const int64_t first = (int64_t)v.b * N, last = first + N;
    if (v0 < first) v0 = first;
    if (v1 > last) v1 = last;
    v.n_lo = (int32_t)(v0 - first);
    v.nv = v1 > v0 ? (int32_t)(v1 - v0) : 0;
    return v;
}

// The largest slot_rows over the slots (sizes the grid of a view launch).
inline int64_t max_slot_rows(int B, int N, int A) {
    int64_t m = 0;
    for (int x = 0; x < kSlots; ++x) {
        const int64_t r = slot_rows(slot_span(x, B, N, A), A);
        if (r > m) m = r;
    }
    return m;
}

// Launchers return hipSuccess or the launch error. They enqueue only.
hipError_t launch_forward(const OpArgs& a, int dtype, int cpl, int waves, size_t lds_bytes,
                          hipStream_t s);
hipError_t launch_backward(const OpArgs& a, int dtype, int cpl, int waves, size_t lds_bytes,
                           hipStream_t s);
// View order: `waves` waves per workgroup, each its own row. The forward
// writes per-slot partial sums to part ([kSlots][B*A][C] FP32) and adds
// them into out in slot order.
hipError_t launch_forward_view(const OpArgs& a, int dtype, int cpl, int waves, size_t lds_bytes,
                               float* part, hipStream_t s);
hipError_t launch_backward_view(const OpArgs& a, int dtype, int cpl, int waves, size_t lds_bytes,
                                hipStream_t s);
hipError_t launch_gfeat_tiles(const TileArgs& t, int out_dtype, int cpl, hipStream_t s);
// cell_start[N*L], tile_start[N*L + 1] and tile_region[N*L] from the shapes.
hipError_t launch_region_tables(const int32_t* shapes, int32_t N, int32_t L, uint32_t* cell_start,
                                uint32_t* tile_start, uint32_t* tile_region, hipStream_t s);
// Stable sort of the n record keys (keys_a; values = the indices, or the
// caller's in vals_a when vals_given) by key in [0, nrows]; *sorted_vals
// receives the sorted values (in vals_a or vals_b) and off[0..nrows] the
// segment starts. n_dev (or nullptr): a device count that caps n at run
// time. scratch: sort_scratch_words(n) words.
hipError_t launch_sort_records(uint32_t* keys_a, uint32_t* keys_b, uint32_t* vals_a,
                               uint32_t* vals_b, uint32_t n, uint32_t nrows, uint32_t* scratch,
                               uint32_t* off, uint32_t** sorted_vals, hipStream_t s,
                               const uint32_t* n_dev = nullptr, bool vals_given = false);
size_t sort_scratch_words(uint32_t n);
// The dense single call's record sort, one workgroup per bucket (b, region):
// bucket k = b*N*L + r holds the A*P records of region r of batch item b in
// (anchor, keypoint) order at [k*ap, (k+1)*ap) of keys, key = the local cell
// in [0, (H+1)(W+1)] ((H+1)(W+1): outside the level). Sorts each bucket by
// key, stably, in LDS; writes vals[k*ap + i] = the sample index of the
// bucket's i-th record in key order and off[] of the bucket's cells (global
// cell b*cells_per_item + cell_start[r] + local), and off[B*cells_per_item]
// = B*N*L*ap. Also writes the region tables of launch_region_tables
// (cell_start, tile_start, tile_region). Requires ap <= kBucketMaxRecords,
// (H+1)(W+1) + 1 <= kBucketMaxKeys for every region, N*L <= 1024, and
// bucket_sort_lds_bytes(ap) of LDS. The visible-view form (place, items
// non-null: the exclusive scan of the visible flags over the view-major items
// (b*N + n)*A + a and the compacted item list): bucket (b, n, l) holds the
// cnt*P records of the cnt visible anchors of (b, n), at s0*P*L + l*cnt*P
// with s0 = place[(b*N + n)*A], in (anchor, keypoint) order, ap = A*P
// bounding cnt*P; vals and off as above, off[B*cells_per_item] = the number
// of visible records.
constexpr uint32_t kBucketMaxRecords = 1u << 15;
constexpr uint32_t kBucketMaxKeys = 1u << 17;
size_t bucket_sort_lds_bytes(uint32_t ap);
hipError_t launch_bucket_sort(const uint32_t* keys, const int32_t* shapes, int32_t B, int32_t N,
                              int32_t L, int32_t A, int32_t P, uint32_t cells_per_item,
                              uint32_t* vals, uint32_t* off, uint32_t* cell_start,
                              uint32_t* tile_start, uint32_t* tile_region, const uint32_t* place,
                              const uint32_t* items, hipStream_t s);
// The batched form's record sort: bucket k = the batch's region k (scene s,
// region r of it), A_s*P records at sample_start[s] + r*A_s*P, keyed by
// local cell; writes the sorted global sample indices to vals (bucket k's
// part at the same place) and off[] of the batch's cells (cell_start of the
// batch tables, (H+1)(W+1) + 1 per region), off[total_cells] = total
// samples. max_ap: the largest A_s*P (<= kBucketMaxRecords; LDS
// bucket_sort_lds_bytes(max_ap)).
hipError_t launch_bucket_sort_batched(const BatchArgs& b, uint32_t max_ap, uint32_t* vals,
                                      uint32_t* off, hipStream_t s);
// In-place exclusive scan of n words; partial: scan_scratch_words(n) words.
hipError_t launch_exclusive_scan(uint32_t* x, uint32_t n, uint32_t* partial, hipStream_t s);
size_t scan_scratch_words(uint32_t n);

// Keypoint projection and the visible-view form (msda_vis.hip).
hipError_t launch_project_keypoints(const ProjArgs& p, hipStream_t s);
// place[0..V] = exclusive scan of the view-major visibility flags (place[V]
// = the number of visible items), items[place[v]] = v, and *rec_count =
// place[V] * per_item (or nothing when rec_count is nullptr).
hipError_t launch_visible_items(const uint8_t* visible, int B, int N, int A, uint32_t per_item,
                                uint32_t* place, uint32_t* items, uint32_t* rec_count,
                                uint32_t* scan_partial, hipStream_t s);
// vt (or nullptr): the fused form's per-view weights [B][A][N].
hipError_t launch_forward_visible(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                                  const uint32_t* items, const uint32_t* count,
                                  const uint32_t* place, const uint8_t* visible, const float* vt,
                                  float* part, hipStream_t s);
// item_dot (or nullptr): per item, <grad_out, the anchor's feature in the view>.
hipError_t launch_backward_visible(const OpArgs& a, int dtype, int cpl, int waves, size_t lds,
                                   const uint32_t* items, const uint32_t* place,
                                   const uint32_t* count, uint32_t* rec_val, const float* vt,
                                   float* item_dot, hipStream_t s);
// Fused weight generation (per-group softmax of logits, BF16 weights).
// stats[(b*A + a)*G + g] = (max, 1 / sum of exp(logit - max)) over the
// anchor's P*N*L logits of group g; logits FP32 or bfloat16 bit patterns.
// part: scratch of softmax_scratch_bytes (per-chunk partials).
size_t softmax_scratch_bytes(int BA, int PNL, int G);
hipError_t launch_softmax_stats(const void* logits, bool bf16, int BA, int PNL, int G,
                                float2* part, float2* stats, hipStream_t s);
// w[i] = softmax weight (stats given) or the widened weight (stats nullptr),
// FP32, for all BA*PNL*G entries.
hipError_t launch_weights_f32(const void* src, bool bf16, const float2* stats, int BA, int PNL,
                              int G, float* w, hipStream_t s);
// In place: grad[i] = w[i] * (grad[i] - sum over the anchor's group of w * grad),
// the gradient through the per-group softmax; part: softmax_scratch_bytes.
hipError_t launch_softmax_grad(const float* w, float* grad, int BA, int PNL, int G, float* part,
                               hipStream_t s);
hipError_t launch_view_scale(const uint8_t* visible, const float* score, int BA, int N,
                             float* vt, hipStream_t s);
hipError_t launch_grad_score(const float* grad_out, const float* out, const uint8_t* visible,
                             const float* score, const uint32_t* place, const float* item_dot,
                             int B, int A, int N, int C, float* grad_score, hipStream_t s);
int sort_passes(uint32_t max_key);

hipError_t launch_batch_tables(const BatchArgs& b, bool backward, hipStream_t s);
hipError_t launch_forward_batched(const BatchArgs& b, int dtype, int cpl, int waves, int blocks,
                                  size_t lds_bytes, hipStream_t s);
hipError_t launch_backward_batched(const BatchArgs& b, int dtype, int cpl, int waves, int blocks,
                                   size_t lds_bytes, hipStream_t s);
// Batched gathers in view order: one wave per (XCD slot, global anchor)
// row; grid kSlots * ceil(total_anchors / waves); LDS waves *
// batch_view_wave_bytes. The forward's per-slot partials go to part
// ([kSlots][total_anchors][C] FP32) and are added into each scene's out.
size_t batch_view_lds(int view_cams, int L, int J, int G, int waves);
hipError_t launch_forward_batched_view(const BatchArgs& b, int dtype, int cpl, int waves,
                                       size_t lds, float* part, hipStream_t s);
hipError_t launch_backward_batched_view(const BatchArgs& b, int dtype, int cpl, int waves,
                                        size_t lds, hipStream_t s);
hipError_t launch_gfeat_tiles_batched(const BatchArgs& b, int out_dtype, int cpl, hipStream_t s);

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, size_t n, hipStream_t s);
hipError_t launch_f32_to_f16(const float* src, uint16_t* dst, size_t n, hipStream_t s);
// max_region_rows: the largest H*W over the regions (sizes the grid).
hipError_t launch_quantize_fp8(const float* x, const int32_t* shapes, const int32_t* starts,
                               int32_t B, int32_t N, int32_t L, int64_t R, int32_t C,
                               int64_t max_region_rows, uint8_t* codes, float* level_scale,
                               uint32_t* amax_ws, hipStream_t s);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// LDS bytes of a forward/backward launch: geometry table + per-wave staging
// (or the cross-wave reduction area, whichever is larger).
size_t lds_bytes_for(const OpArgs& a, int waves);
// The same for a view-order launch (staging only).
size_t lds_bytes_view(const OpArgs& a, int waves);
int max_pairs_per_chunk(int L, int G);

// Benchmark instrumentation (msda_set_kernel_events): called around every
// kernel launch; records the caller's events when enabled, else does nothing.
// Sets the thread's last-error message (msda_last_error) and returns st.
msda_status set_error(msda_status st, const char* message);

void mark_begin(const char* kernel, hipStream_t s);
void mark_end(hipStream_t s);

}  // namespace msda
