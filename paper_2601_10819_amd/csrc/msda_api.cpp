// C-ABI layer of libmsda.so: host-side validation, launch-shape choice and
// dispatch to the HIP kernels. Nothing here allocates, frees or synchronises.
// The operator and the argument conventions are documented in include/msda.h.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/msda.h"
#include "msda_internal.h"

namespace {

thread_local std::string g_error;
// Benchmark hook state (msda_set_kernel_events).
thread_local void* const* g_events = nullptr;
thread_local int32_t g_event_cap = 0;
thread_local int32_t g_event_used = 0;
thread_local const char* g_event_names[256];
thread_local std::string g_event_filter;     // record only this kernel name ("" = all)
thread_local bool g_event_open = false;      // the last mark_begin recorded an event

msda_status fail(msda_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

msda_status ok() {
    g_error.clear();
    return MSDA_OK;
}

constexpr uint32_t kWeightFlags = MSDA_WEIGHT_LOGITS | MSDA_WEIGHTS_BF16;

int elem_bytes(int32_t dtype) {
    switch (dtype) {
        case MSDA_F32: return 4;
        case MSDA_BF16: return 2;
        case MSDA_F16: return 2;
        case MSDA_FP8_E4M3: return 1;
        default: return 0;
    }
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int log2i(int64_t v) {
    int s = 0;
    while ((int64_t(1) << s) < v) ++s;
    return s;
}

// Channels per lane the kernels are built for, widest first (16-byte loads).
const int* cpl_candidates(int32_t dtype) {
    static const int f32[] = {4, 2, 1, 0};
    static const int bf16[] = {8, 4, 2, 0};
    static const int fp8[] = {16, 8, 4, 0};
    switch (dtype) {
        case MSDA_F32: return f32;
        case MSDA_BF16:
        case MSDA_F16: return bf16;
        default: return fp8;
    }
}

bool cpl_fits(int cpl, int32_t C, int32_t G) {
    if (cpl <= 0 || C % cpl) return false;
    const int64_t lps = C / cpl;
    if (!is_pow2(lps) || lps > 64) return false;
    const int32_t cpg = C / G;
    return cpg % cpl == 0 && is_pow2(cpg / cpl);
}

bool cpl_is_candidate(int cpl, int32_t dtype) {
    for (const int* c = cpl_candidates(dtype); *c; ++c)
        if (*c == cpl) return true;
    return false;
}

// Sizes, dtype and the (camera, level) regions, checked against the host
// mirrors. Shared by the operator and the quantiser.
msda_status check_regions(const msda_desc* d, int64_t* batch_bytes_out) {
    if (!d) return fail(MSDA_ERR_INVALID_ARGUMENT, "desc is NULL");
    if (d->batch < 1 || d->num_cams < 1 || d->num_levels < 1 || d->num_anchors < 0 ||
        d->num_points < 1 || d->channels < 1 || d->groups < 1 || d->rows < 1)
        return fail(MSDA_ERR_INVALID_ARGUMENT,
                    "sizes must be positive (B=%d Ncam=%d L=%d A=%d P=%d C=%d G=%d R=%lld)",
                    d->batch, d->num_cams, d->num_levels, d->num_anchors, d->num_points,
                    d->channels, d->groups, (long long)d->rows);
    if (d->num_levels > 8) return fail(MSDA_ERR_UNSUPPORTED, "at most 8 levels (L=%d)", d->num_levels);
    if (d->channels % d->groups)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "channels (%d) not divisible by groups (%d)",
                    d->channels, d->groups);
    const int eb = elem_bytes(d->feat_dtype);
    if (!eb) return fail(MSDA_ERR_INVALID_ARGUMENT, "unknown feat_dtype %d", d->feat_dtype);
    if (d->feat_dtype == MSDA_FP8_E4M3 && !d->level_scale)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "FP8 features need level_scale");
    if (!d->host_spatial_shapes || !d->host_level_start_index)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "host mirrors of spatial_shapes/level_start_index are NULL");
    const int64_t NL = (int64_t)d->num_cams * d->num_levels;
    if (NL > 1024)
        return fail(MSDA_ERR_UNSUPPORTED, "too many (camera, level) regions (%lld > 1024)",
                    (long long)NL);
    for (int64_t i = 0; i < NL; ++i) {
        const int64_t H = d->host_spatial_shapes[2 * i], W = d->host_spatial_shapes[2 * i + 1];
        const int64_t s0 = d->host_level_start_index[i];
        if (H < 1 || W < 1 || H > 32768 || W > 32768)
            return fail(MSDA_ERR_INVALID_ARGUMENT, "region %lld: H=%lld W=%lld out of [1, 32768]",
                        (long long)i, (long long)H, (long long)W);
        if (s0 < 0 || s0 + H * W > d->rows)
            return fail(MSDA_ERR_INVALID_ARGUMENT,
                        "region %lld: rows [%lld, %lld) outside [0, R=%lld)", (long long)i,
                        (long long)s0, (long long)(s0 + H * W), (long long)d->rows);
    }
    // one batch item is one buffer resource with 32-bit byte offsets, and
    // the out-of-level marker offset msda::kOOB lies at or past its end
    if ((int64_t)d->channels * eb > (int64_t)msda::kMaxRowBytes)
        return fail(MSDA_ERR_UNSUPPORTED, "a feature row is %lld bytes (limit %u)",
                    (long long)d->channels * eb, msda::kMaxRowBytes);
    const int64_t batch_bytes = d->rows * d->channels * (int64_t)eb;
    if (batch_bytes > (int64_t)msda::kOOB)
        return fail(MSDA_ERR_UNSUPPORTED,
                    "one batch item of feat is %lld bytes (limit %lld, 4 GiB - 8 KiB)",
                    (long long)batch_bytes, (long long)msda::kOOB);
    if ((int64_t)d->batch * d->num_anchors > 0x7fffffffLL)
        return fail(MSDA_ERR_UNSUPPORTED, "batch * anchors exceeds 2^31 - 1");
    *batch_bytes_out = batch_bytes;
    return MSDA_OK;
}

// The gathers' work order: explicit, else view order once there are at
// least kSlots (batch item, camera) views to spread over the XCDs. A
// forward without a workspace always runs in anchor order.
int resolve_order(const msda_desc* d, bool can_view) {
    const int o = d->tile ? d->tile->order : MSDA_ORDER_AUTO;
    if (o != MSDA_ORDER_AUTO) return o;
    const int64_t views = (int64_t)d->batch * d->num_cams;
    return can_view && views >= msda::kSlots ? MSDA_ORDER_VIEW : MSDA_ORDER_ANCHOR;
}

// LDS one workgroup may use on the current device (160 KB on gfx950), the
// attribute read once per device; 0 if it cannot be read.
size_t device_lds_limit() {
    static int max_lds[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (max_lds[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess || v <= 0)
            v = -1;
        max_lds[dev] = v;
    }
    return max_lds[dev] > 0 ? (size_t)max_lds[dev] : 0;
}

// Validates everything and chooses the launch shape for the given order;
// fills `a` except pointers.
msda_status prepare(const msda_desc* d, int order, msda::OpArgs* a, int* cpl_out,
                    int* waves_out) {
    int64_t batch_bytes = 0;
    msda_status st = check_regions(d, &batch_bytes);
    if (st != MSDA_OK) return st;
    int cpl = 0;
    if (d->tile && d->tile->chans_per_lane) {
        cpl = d->tile->chans_per_lane;
        if (!cpl_is_candidate(cpl, d->feat_dtype) || !cpl_fits(cpl, d->channels, d->groups))
            return fail(MSDA_ERR_UNSUPPORTED, "chans_per_lane=%d does not fit C=%d G=%d dtype=%d",
                        cpl, d->channels, d->groups, d->feat_dtype);
    } else {
        for (const int* c = cpl_candidates(d->feat_dtype); *c; ++c)
            if (cpl_fits(*c, d->channels, d->groups)) { cpl = *c; break; }
        if (!cpl)
            return fail(MSDA_ERR_UNSUPPORTED,
                        "no lane layout for C=%d G=%d: need C/k a power of two <= 64 and "
                        "C/G/k a power of two for k in the dtype's lane widths",
                        d->channels, d->groups);
    }
    if (order != MSDA_ORDER_ANCHOR && order != MSDA_ORDER_VIEW)
        return fail(MSDA_ERR_UNSUPPORTED, "unknown order %d", order);
    if (d->flags & ~(MSDA_DETERMINISTIC | kWeightFlags))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", (unsigned)d->flags);

    a->B = d->batch;
    a->N = d->num_cams;
    a->L = d->num_levels;
    a->A = d->num_anchors;
    a->P = d->num_points;
    a->C = d->channels;
    a->G = d->groups;
    a->R = d->rows;
    a->batch_bytes = (uint32_t)batch_bytes;
    a->lps_shift = log2i(d->channels / cpl);
    a->pairs_per_chunk = msda::max_pairs_per_chunk(d->num_levels, d->groups);

    const int64_t npairs = (int64_t)d->num_points * d->num_cams;
    const int64_t nchunks = (npairs + a->pairs_per_chunk - 1) / a->pairs_per_chunk;
    int waves = 0;
    if (d->tile && d->tile->waves_per_anchor) {
        waves = d->tile->waves_per_anchor;
        if (!is_pow2(waves) || waves > 8)
            return fail(MSDA_ERR_UNSUPPORTED, "waves_per_anchor=%d not in {1,2,4,8}", waves);
    } else if (order == MSDA_ORDER_VIEW) {
        waves = 4;
    } else {
        // Aim for about 8 waves per SIMD across the chip (256 CUs x 4 SIMDs),
        // but no more waves than the anchor has staging chunks.
        const int64_t blocks = (int64_t)d->batch * d->num_anchors;
        waves = 1;
        while (waves < 8 && blocks * waves * 2 <= 8192 && waves * 2 <= nchunks) waves *= 2;
    }
    auto lds_of = [&](int w) {
        return order == MSDA_ORDER_VIEW ? msda::lds_bytes_view(*a, w) : msda::lds_bytes_for(*a, w);
    };
    // a chosen (not requested) wave count shrinks until the staging fits
    // 64 KiB (a quarter of the CU's LDS or less: 4 workgroups per CU); a
    // requested one may use what the device allows a workgroup
    if (!(d->tile && d->tile->waves_per_anchor))
        while (waves > 1 && lds_of(waves) > 65536) waves /= 2;
    // (64 KiB, every gfx9 device's minimum, if the device cannot be asked)
    const size_t lds = lds_of(waves), limit = device_lds_limit() ? device_lds_limit() : 65536;
    if (lds > limit)
        return fail(MSDA_ERR_UNSUPPORTED, "launch needs %zu bytes of LDS (limit %zu)", lds, limit);
    *cpl_out = cpl;
    *waves_out = waves;
    return MSDA_OK;
}

msda_status hip_fail(hipError_t e, const char* what) {
    return fail(MSDA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t n) { return ((uintptr_t)p % n) == 0; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Fused weight generation: the softmax statistics (forward and backward)
// and the FP32 weights the backward works on.
// The statistics [B*A][G] float2, then the per-chunk partials they are
// merged from (reused for the backward's per-chunk group sums).
size_t stats_only_bytes(const msda_desc* d) {
    return align256((size_t)d->batch * (size_t)(d->num_anchors > 0 ? d->num_anchors : 0) *
                    (size_t)d->groups * sizeof(float2));
}

size_t stats_bytes(const msda_desc* d) {
    if (!(d->flags & MSDA_WEIGHT_LOGITS)) return 0;
    const int BA = d->batch * (d->num_anchors > 0 ? d->num_anchors : 0);
    return stats_only_bytes(d) +
           align256(msda::softmax_scratch_bytes(
               BA, d->num_points * d->num_cams * d->num_levels, d->groups));
}

// Workspace of the sorted grad_feat form: record keys (x2 for the sort),
// values (x2), fractions, per-cell offsets, region tables and the sort's
// histogram scratch.
struct SortedWs {
    size_t keys_a, keys_b, vals_a, vals_b, frac, off, cell_start, tile_start, tile_region,
        scratch, total;
};

SortedWs sorted_layout(uint64_t nrec, uint64_t ncells, uint64_t nregions) {
    SortedWs w;
    const size_t rec = align256(nrec * 4);
    w.keys_a = 0;
    w.keys_b = w.keys_a + rec;
    w.vals_a = w.keys_b + rec;
    w.vals_b = w.vals_a + rec;
    w.frac = w.vals_b + rec;
    w.off = w.frac + align256(nrec * 8);
    w.cell_start = w.off + align256((ncells + 1) * 4);
    w.tile_start = w.cell_start + align256(nregions * 4);
    w.tile_region = w.tile_start + align256((nregions + 1) * 4);
    w.scratch = w.tile_region + align256(nregions * 4);
    w.total = w.scratch + align256(msda::sort_scratch_words((uint32_t)nrec) * 4);
    return w;
}

// Cells and 4x4 tiles of one batch item (from the host mirror of the shapes):
// each region's cells are its (H+1)(W+1) bilinear cells and one more for its
// samples outside the level (region_tables_kernel, batch_tables_kernel).
void cells_and_tiles(const msda_desc* d, uint64_t* cells, uint64_t* tiles) {
    *cells = *tiles = 0;
    const int64_t NL = (int64_t)d->num_cams * d->num_levels;
    for (int64_t i = 0; i < NL; ++i) {
        const uint64_t H = d->host_spatial_shapes[2 * i], W = d->host_spatial_shapes[2 * i + 1];
        *cells += (H + 1) * (W + 1) + 1;
        *tiles += ((H + msda::kTileH - 1) / msda::kTileH) * ((W + msda::kTileW - 1) / msda::kTileW);
    }
}

// Tiles (of one batch item, in slot order: coarse levels first) of the levels
// whose regions are at most 1/16 of the largest region's area -- the levels
// where a pixel collects 16x or more the samples of the finest one.
uint32_t heavy_tiles(const msda_desc* d) {
    const int N = d->num_cams, L = d->num_levels;
    int64_t max_area = 0;
    for (int i = 0; i < N * L; ++i)
        max_area = std::max<int64_t>(max_area, (int64_t)d->host_spatial_shapes[2 * i] *
                                                   d->host_spatial_shapes[2 * i + 1]);
    uint32_t tiles = 0;
    for (int o = 0; o < N * L; ++o) {            // slot o -> level L-1-o/N, camera o%N
        const int l = L - 1 - o / N, n = o % N, r = n * L + l;
        const int64_t H = d->host_spatial_shapes[2 * r], W = d->host_spatial_shapes[2 * r + 1];
        if (H * W * 16 > max_area) break;
        tiles += (uint32_t)(((H + msda::kTileH - 1) / msda::kTileH) *
                            ((W + msda::kTileW - 1) / msda::kTileW));
    }
    return tiles;
}

// 1 if the regions are pairwise disjoint; *cover = they tile [0, R) exactly.
bool regions_disjoint(const msda_desc* d, bool* cover) {
    const int64_t NL = (int64_t)d->num_cams * d->num_levels;
    std::vector<std::pair<int64_t, int64_t>> iv;
    iv.reserve(NL);
    for (int64_t i = 0; i < NL; ++i)
        iv.emplace_back(d->host_level_start_index[i],
                        d->host_level_start_index[i] + (int64_t)d->host_spatial_shapes[2 * i] *
                                                           d->host_spatial_shapes[2 * i + 1]);
    std::sort(iv.begin(), iv.end());
    int64_t end = 0, covered = 0;
    for (const auto& p : iv) {
        if (p.first < end) return false;
        covered += p.second - p.first;
        end = p.second;
    }
    *cover = covered == d->rows;
    return true;
}

int scatter_mode(const msda_desc* d) {
    const int m = d->tile ? d->tile->scatter : MSDA_SCATTER_AUTO;
    return m == MSDA_SCATTER_AUTO ? MSDA_SCATTER_SORTED : m;
}

uint64_t num_samples(const msda_desc* d) {
    return (uint64_t)d->batch * (uint64_t)d->num_anchors * (uint64_t)d->num_points *
           (uint64_t)d->num_cams * (uint64_t)d->num_levels;
}

// s / d for s < 2^30 as (s * m) >> shift (round-up multiplier).
void divmagic(uint32_t d, uint64_t* m, int* shift) {
    int l = 0;
    while ((1ull << l) < d) ++l;
    const int k = 32 + l;
    *m = ((1ull << k) + d - 1) / d;
    *shift = k;
}

}  // namespace

namespace msda {

msda_status set_error(msda_status st, const char* message) {
    g_error = message ? message : "";
    return st;
}

void mark_begin(const char* kernel, hipStream_t s) {
    g_event_open = false;
    if (!g_events || g_event_used >= g_event_cap) return;
    if (!g_event_filter.empty() && g_event_filter != kernel) return;
    g_event_open = true;
    g_event_names[g_event_used] = kernel;
    // instrumentation only: a failed record shows as a missing duration
    (void)hipEventRecord(static_cast<hipEvent_t>(g_events[2 * g_event_used]), s);
}

void mark_end(hipStream_t s) {
    if (!g_event_open) return;
    g_event_open = false;
    (void)hipEventRecord(static_cast<hipEvent_t>(g_events[2 * g_event_used + 1]), s);
    ++g_event_used;
}

}  // namespace msda

extern "C" {

int32_t msda_abi_version(void) { return MSDA_ABI_VERSION; }

msda_status msda_set_kernel_events(void* const* events, int32_t max_kernels) {
    if (events && (max_kernels < 1 || max_kernels > 256))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "max_kernels must be in [1, 256]");
    g_events = events;
    g_event_cap = events ? max_kernels : 0;
    g_event_used = 0;
    return ok();
}

msda_status msda_set_kernel_event_filter(const char* kernel) {
    if (kernel && std::strlen(kernel) > 255)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "kernel name longer than 255 characters");
    g_event_filter = kernel ? kernel : "";
    return ok();
}

int32_t msda_recorded_kernels(void) { return g_event_used; }

const char* msda_recorded_kernel_name(int32_t i) {
    return (i >= 0 && i < g_event_used) ? g_event_names[i] : "";
}

const char* msda_last_error(void) { return g_error.c_str(); }

// Shared body of msda_forward / msda_forward_ws.
static msda_status forward_impl(const void* feat, const int32_t* spatial_shapes,
                                const int32_t* level_start_index, const float* sampling_loc,
                                const float* weights, float* out, void* workspace,
                                size_t workspace_bytes, bool has_ws, const msda_desc* desc,
                                void* stream) {
    if (!desc) return fail(MSDA_ERR_INVALID_ARGUMENT, "desc is NULL");
    const int order = resolve_order(desc, has_ws);
    if (order == MSDA_ORDER_VIEW && !has_ws)
        return fail(MSDA_ERR_WORKSPACE, "the view-order forward needs a workspace "
                                        "(msda_forward_ws)");
    msda::OpArgs a = {};
    int cpl = 0, waves = 0;
    msda_status st = prepare(desc, order, &a, &cpl, &waves);
    if (st != MSDA_OK) return st;
    // the view-order forward runs fastest with one wave (one anchor row) per
    // workgroup (measured on the 64-camera workload in FP32 and BF16)
    if (order == MSDA_ORDER_VIEW && !(desc->tile && desc->tile->waves_per_anchor)) waves = 1;
    // sampling_loc, weights and out hold zero elements when A == 0 and may be NULL then
    if (!feat || !spatial_shapes || !level_start_index ||
        (a.A > 0 && (!sampling_loc || !weights || !out)))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "a required device pointer is NULL");
    if (!aligned(feat, 16)) return fail(MSDA_ERR_UNSUPPORTED, "feat must be 16-byte aligned");
    const size_t part_bytes = order == MSDA_ORDER_VIEW
                                  ? (size_t)msda::kSlots * a.B * a.A * a.C * sizeof(float) : 0;
    const size_t stats_off = align256(part_bytes);
    const size_t need = stats_off + stats_bytes(desc);
    if (need && !has_ws)
        return fail(MSDA_ERR_WORKSPACE, "weight logits need a workspace (msda_forward_ws)");
    if (need && (!workspace || workspace_bytes < need || !aligned(workspace, 256)))
        return fail(MSDA_ERR_WORKSPACE, "forward workspace: need %zu bytes, 256-byte aligned "
                                        "(got %zu at %p)", need, workspace_bytes, workspace);
    if (a.A == 0) return ok();
    const bool wbf16 = desc->flags & MSDA_WEIGHTS_BF16;
    a.w_bf16 = wbf16;
    if (desc->flags & MSDA_WEIGHT_LOGITS) {
        char* base = static_cast<char*>(workspace) + stats_off;
        float2* stats = reinterpret_cast<float2*>(base);
        float2* part = reinterpret_cast<float2*>(base + stats_only_bytes(desc));
        const hipError_t e = msda::launch_softmax_stats(weights, wbf16, a.B * a.A,
                                                        a.P * a.N * a.L, a.G, part, stats,
                                                        (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "softmax statistics");
        a.wstats = stats;
    }
    a.feat = feat;
    a.shapes = spatial_shapes;
    a.starts = level_start_index;
    a.loc = sampling_loc;
    a.w = weights;
    a.level_scale = desc->feat_dtype == MSDA_FP8_E4M3 ? desc->level_scale : nullptr;
    a.out = out;
    const hipError_t e =
        order == MSDA_ORDER_VIEW
            ? msda::launch_forward_view(a, desc->feat_dtype, cpl, waves,
                                        msda::lds_bytes_view(a, waves),
                                        static_cast<float*>(workspace), (hipStream_t)stream)
            : msda::launch_forward(a, desc->feat_dtype, cpl, waves, msda::lds_bytes_for(a, waves),
                                   (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "msda_forward launch");
    return ok();
}

msda_status msda_forward(const void* feat, const int32_t* spatial_shapes,
                         const int32_t* level_start_index, const float* sampling_loc,
                         const float* weights, float* out, const msda_desc* desc, void* stream) {
    return forward_impl(feat, spatial_shapes, level_start_index, sampling_loc, weights, out,
                        nullptr, 0, false, desc, stream);
}

msda_status msda_forward_ws(const void* feat, const int32_t* spatial_shapes,
                            const int32_t* level_start_index, const float* sampling_loc,
                            const float* weights, float* out, void* workspace,
                            size_t workspace_bytes, const msda_desc* desc, void* stream) {
    return forward_impl(feat, spatial_shapes, level_start_index, sampling_loc, weights, out,
                        workspace, workspace_bytes, true, desc, stream);
}

size_t msda_forward_workspace_size(const msda_desc* d) {
    if (!d || d->batch < 1 || d->num_cams < 1 || d->channels < 1 || d->num_anchors < 0) return 0;
    const size_t part = resolve_order(d, true) == MSDA_ORDER_VIEW
                            ? (size_t)msda::kSlots * (size_t)d->batch * (size_t)d->num_anchors *
                                  (size_t)d->channels * sizeof(float)
                            : 0;
    return align256(part) + stats_bytes(d);
}

// The backward gather in the chosen order. In view order each wave takes
// one anchor over a group of cameras: 2 for 1- and 2-byte features, 1 for
// FP32 (measured at 64 cameras: BF16 0.457 ms with 2 against 0.478 with 1
// and 0.470 with 4; FP32 0.709 ms with 1 against 0.754 with 2).
static hipError_t launch_gather(const msda::OpArgs& a0, int order, int dtype, int cpl, int waves,
                                hipStream_t s) {
    msda::OpArgs a = a0;
    a.view_cams = dtype == MSDA_F32 ? 1 : 2;
    if (order == MSDA_ORDER_VIEW)
        return msda::launch_backward_view(a, dtype, cpl, waves, msda::lds_bytes_view(a, waves), s);
    return msda::launch_backward(a, dtype, cpl, waves, msda::lds_bytes_for(a, waves), s);
}

// Extra workspace of the visible-view form: the scanned flags (V + 1 words),
// the scan's scratch, the item list (V words) and the record count.
struct VisibleWs {
    size_t place, partial, items, rec_count, vt, dot, total;
};

VisibleWs visible_layout(const msda_desc* d, size_t at) {
    const uint64_t V = (uint64_t)d->batch * d->num_cams * (uint64_t)(d->num_anchors > 0 ? d->num_anchors : 0);
    VisibleWs w;
    w.place = at;
    w.partial = w.place + align256((V + 1) * 4);
    w.items = w.partial + align256(msda::scan_scratch_words((uint32_t)(V + 1)) * 4);
    w.rec_count = w.items + align256(V * 4 + 4);
    w.vt = w.rec_count + 256;                 // the fused form's per-view weights
    w.dot = w.vt + align256(V * 4);           // and its per-item score products
    w.total = w.dot + align256(V * 4);
    return w;
}

// Whether the dense backward's records fit the per-bucket LDS sort: A*P
// records per (batch item, region) bucket, every region's local keys within
// the composite key, and the bucket's LDS within the device's per-block
// limit (looked up once per device; no bucket sort if that fails).
// Whether a bucket-sort block of ap records fits the current device's LDS.
static bool bucket_lds_fits(uint64_t ap) {
    return msda::bucket_sort_lds_bytes((uint32_t)ap) <= device_lds_limit();
}

// Whether the region tables' cells of every region (bilinear cells and the
// outside cell) fit the bucket sort's composite keys.
static bool bucket_keys_fit(const int32_t* shapes, int64_t regions) {
    for (int64_t i = 0; i < regions; ++i) {
        const uint64_t H = shapes[2 * i], W = shapes[2 * i + 1];
        if ((H + 1) * (W + 1) + 1 > msda::kBucketMaxKeys) return false;
    }
    return true;
}

static bool bucket_sort_fits(const msda_desc* d) {
    const uint64_t ap = (uint64_t)d->num_anchors * (uint64_t)d->num_points;
    if (ap == 0 || ap > msda::kBucketMaxRecords) return false;
    return bucket_keys_fit(d->host_spatial_shapes, (int64_t)d->num_cams * d->num_levels) &&
           bucket_lds_fits(ap);
}

// The backward's workspace without the weight flags' part.
static size_t base_backward_bytes(const msda_desc* d) {
    if (!d || d->batch < 1 || d->rows < 1 || d->channels < 1 || d->num_anchors < 0) return 0;
    if (scatter_mode(d) == MSDA_SCATTER_ATOMIC) {
        if (d->feat_dtype == MSDA_BF16 || d->feat_dtype == MSDA_F16)   // FP32 accumulator
            return (size_t)d->batch * (size_t)d->rows * (size_t)d->channels * sizeof(float);
        return 0;
    }
    if (!d->host_spatial_shapes || d->num_cams < 1 || d->num_levels < 1) return 0;
    uint64_t cells, tiles;
    cells_and_tiles(d, &cells, &tiles);
    return sorted_layout(num_samples(d), cells * (uint64_t)d->batch,
                         (uint64_t)d->num_cams * d->num_levels).total;
}

// The FP32 weights the backward works on under a weight flag.
static size_t weights_f32_bytes(const msda_desc* d) {
    return (d->flags & kWeightFlags) ? align256(num_samples(d) * (size_t)d->groups * 4) : 0;
}

size_t msda_backward_workspace_size(const msda_desc* d) {
    if (!d || d->batch < 1 || d->rows < 1 || d->channels < 1 || d->num_anchors < 0) return 0;
    return align256(base_backward_bytes(d)) + stats_bytes(d) + weights_f32_bytes(d);
}

// The backward, dense (visible == nullptr) or over the visible views only.
// The fused form's extra operands (visibility-weighted fusion, Eq. 2).
struct Fusion {
    const float* score;     // [B][A][N]
    const float* out;       // the fused forward output [B][A][C] (for grad_score)
    float* grad_score;      // [B][A][N], or nullptr
};

static msda_status backward_impl(const void* feat, const int32_t* spatial_shapes,
                                 const int32_t* level_start_index, const float* sampling_loc,
                                 const float* weights, const uint8_t* visible,
                                 const Fusion* fuse, const float* grad_out, void* grad_feat,
                                 float* grad_sampling_loc, float* grad_weights, void* workspace,
                                 size_t workspace_bytes, const msda_desc* desc, void* stream) {
    if (!desc) return fail(MSDA_ERR_INVALID_ARGUMENT, "desc is NULL");
    // the visible-view gathers walk a compacted item list in ranges per XCD,
    // with the view order's launch shape
    const int order = visible ? MSDA_ORDER_VIEW : resolve_order(desc, true);
    msda::OpArgs a = {};
    int cpl = 0, waves = 0;
    msda_status st = prepare(desc, order, &a, &cpl, &waves);
    if (st != MSDA_OK) return st;
    // sampling_loc, weights and grad_out hold zero elements when A == 0 and may be NULL then
    if (!feat || !spatial_shapes || !level_start_index ||
        (a.A > 0 && (!sampling_loc || !weights || !grad_out)))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "a required device pointer is NULL");
    if (fuse && a.A > 0 && (!fuse->score || (fuse->grad_score && !fuse->out)))
        return fail(MSDA_ERR_INVALID_ARGUMENT,
                    "view_score, and out when grad_score is requested, must not be NULL");
    if (!aligned(feat, 16)) return fail(MSDA_ERR_UNSUPPORTED, "feat must be 16-byte aligned");
    if (desc->feat_dtype == MSDA_FP8_E4M3)
        return fail(MSDA_ERR_UNSUPPORTED, "the backward takes FP32 or BF16 features (not FP8)");
    const int mode = scatter_mode(desc);
    if (mode != MSDA_SCATTER_SORTED && mode != MSDA_SCATTER_SORTED_GLOBAL &&
        mode != MSDA_SCATTER_ATOMIC)
        return fail(MSDA_ERR_UNSUPPORTED, "unknown scatter mode %d", mode);
    if (visible && mode == MSDA_SCATTER_ATOMIC)
        return fail(MSDA_ERR_UNSUPPORTED, "the visible-view backward has the sorted form only");
    if (visible && desc->tile && desc->tile->order == MSDA_ORDER_ANCHOR)
        return fail(MSDA_ERR_UNSUPPORTED, "the visible-view form runs in view order only");
    if ((desc->flags & MSDA_DETERMINISTIC) && mode == MSDA_SCATTER_ATOMIC)
        return fail(MSDA_ERR_UNSUPPORTED, "MSDA_DETERMINISTIC excludes MSDA_SCATTER_ATOMIC");
    const uint64_t nrec = num_samples(desc);
    uint64_t cells = 0, tiles = 0;
    cells_and_tiles(desc, &cells, &tiles);
    const uint64_t ncells = cells * (uint64_t)a.B;
    // the reduction's lane layout: FP32 accumulators, 4/2/1 channels per lane
    int rcpl = 0;
    for (int c : {4, 2, 1})
        if (cpl_fits(c, a.C, a.G)) { rcpl = c; break; }
    bool cover = true;
    if (grad_feat && mode != MSDA_SCATTER_ATOMIC) {
        if (!regions_disjoint(desc, &cover))
            return fail(MSDA_ERR_UNSUPPORTED,
                        "sorted grad_feat needs disjoint regions (use MSDA_SCATTER_ATOMIC)");
        if (ncells >= 0x7fffffffull)
            return fail(MSDA_ERR_UNSUPPORTED, "B * cells = %llu exceeds 2^31 - 1",
                        (unsigned long long)ncells);
        if (nrec >= (1ull << 30))
            return fail(MSDA_ERR_UNSUPPORTED, "B*A*P*Ncam*L = %llu samples exceeds 2^30",
                        (unsigned long long)nrec);
        if (!rcpl) return fail(MSDA_ERR_UNSUPPORTED, "no reduction lane layout for C=%d G=%d", a.C, a.G);
        if (a.G > 64)
            return fail(MSDA_ERR_UNSUPPORTED, "sorted grad_feat supports G <= 64 (G=%d)", a.G);
        if (rcpl == 4 && !aligned(grad_out, 16))
            return fail(MSDA_ERR_UNSUPPORTED, "grad_out must be 16-byte aligned");
    }
    const size_t sorted_need = grad_feat ? base_backward_bytes(desc) : 0;
    const VisibleWs VW = visible_layout(desc, align256(sorted_need));
    // weight flags: softmax statistics and FP32 weights after the rest
    const size_t base_need = visible && a.A > 0 ? VW.total : sorted_need;
    const size_t wx_off = align256(base_need);
    const size_t wx_bytes = a.A > 0 ? stats_bytes(desc) + weights_f32_bytes(desc) : 0;
    const size_t need = wx_bytes ? wx_off + wx_bytes : base_need;
    if (need) {
        if (!workspace || workspace_bytes < need)
            return fail(MSDA_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                        workspace ? workspace_bytes : (size_t)0);
        if (!aligned(workspace, 256))
            return fail(MSDA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    }
    if (grad_feat && !aligned(grad_feat, 16))
        return fail(MSDA_ERR_UNSUPPORTED, "grad_feat must be 16-byte aligned");

    const hipStream_t s = (hipStream_t)stream;
    const size_t gf_elems = (size_t)a.B * (size_t)a.R * (size_t)a.C;
    const size_t gf_bytes = gf_elems * (desc->feat_dtype == MSDA_F32 ? 4 : 2);
    char* ws = static_cast<char*>(workspace);
    hipError_t e = hipSuccess;
    // Under a weight flag the backward works on FP32 weights written once
    // (the softmax of the logits, or the widened BF16 weights); with logits,
    // grad_weights is mapped to the logits' gradient at the end.
    const bool logits = (desc->flags & MSDA_WEIGHT_LOGITS) && a.A > 0;
    const float* weff = weights;
    float* w32 = nullptr;
    float2* part = nullptr;
    if (wx_bytes) {
        float2* stats = logits ? reinterpret_cast<float2*>(ws + wx_off) : nullptr;
        part = reinterpret_cast<float2*>(ws + wx_off + stats_only_bytes(desc));
        w32 = reinterpret_cast<float*>(ws + wx_off + stats_bytes(desc));
        const bool wbf16 = desc->flags & MSDA_WEIGHTS_BF16;
        const int PNL = a.P * a.N * a.L;
        if ((logits && (e = msda::launch_softmax_stats(weights, wbf16, a.B * a.A, PNL, a.G, part,
                                                       stats, s)) != hipSuccess) ||
            (e = msda::launch_weights_f32(weights, wbf16, stats, a.B * a.A, PNL, a.G, w32, s)) !=
                hipSuccess)
            return hip_fail(e, "weights from logits");
        weff = w32;
    }
    auto finish = [&]() -> msda_status {
        if (logits && grad_weights) {
            const hipError_t ee = msda::launch_softmax_grad(w32, grad_weights, a.B * a.A,
                                                            a.P * a.N * a.L, a.G,
                                                            reinterpret_cast<float*>(part), s);
            if (ee != hipSuccess) return hip_fail(ee, "gradient through the softmax");
        }
        return ok();
    };
    a.feat = feat;
    a.shapes = spatial_shapes;
    a.starts = level_start_index;
    a.loc = sampling_loc;
    a.w = weff;
    a.grad_out = grad_out;
    a.grad_loc = grad_sampling_loc;
    a.grad_w = grad_weights;

    if (grad_feat && mode == MSDA_SCATTER_ATOMIC) {
        float* acc = desc->feat_dtype == MSDA_F32 ? static_cast<float*>(grad_feat)
                                                  : reinterpret_cast<float*>(ws);
        if ((e = msda::launch_fill_zero(acc, gf_elems * sizeof(float), s)) != hipSuccess)
            return hip_fail(e, "zero grad_feat accumulator");
        a.gfeat_acc = acc;
        if (a.A > 0 && (e = launch_gather(a, order, desc->feat_dtype, cpl, waves, s)) !=
                           hipSuccess)
            return hip_fail(e, "msda_backward launch");
        if (desc->feat_dtype == MSDA_BF16 &&
            (e = msda::launch_f32_to_bf16(acc, static_cast<uint16_t*>(grad_feat), gf_elems, s)) !=
                hipSuccess)
            return hip_fail(e, "round grad_feat to bf16");
        if (desc->feat_dtype == MSDA_F16 &&
            (e = msda::launch_f32_to_f16(acc, static_cast<uint16_t*>(grad_feat), gf_elems, s)) !=
                hipSuccess)
            return hip_fail(e, "round grad_feat to f16");
        return finish();
    }

    SortedWs W = {};
    uint32_t *cell_start = nullptr, *tile_start = nullptr, *tile_region = nullptr;
    if (grad_feat) {
        W = sorted_layout(nrec, ncells, (uint64_t)a.N * a.L);
        cell_start = reinterpret_cast<uint32_t*>(ws + W.cell_start);
        tile_start = reinterpret_cast<uint32_t*>(ws + W.tile_start);
        tile_region = reinterpret_cast<uint32_t*>(ws + W.tile_region);
        // records sorted per (batch item, region) bucket in LDS when the
        // buckets fit (that launch also writes the region tables), else, or
        // when asked, by the global radix sort
        if (mode != MSDA_SCATTER_SORTED_GLOBAL && bucket_sort_fits(desc))
            a.rec_bucket_ap = (uint32_t)(a.A * a.P);
        if (!a.rec_bucket_ap &&
            (e = msda::launch_region_tables(spatial_shapes, a.N, a.L, cell_start, tile_start,
                                            tile_region, s)) != hipSuccess)
            return hip_fail(e, "region tables");
        a.rec_key = reinterpret_cast<uint32_t*>(ws + W.keys_a);
        a.rec_frac = reinterpret_cast<float2*>(ws + W.frac);
        // bucketed records carry local cells: the gather needs no cell table
        a.cell_start = a.rec_bucket_ap ? nullptr : cell_start;
        a.cells_per_item = (uint32_t)cells;
        a.cell_offset = 0;
        a.no_cell = (uint32_t)ncells;
        a.sample_offset = 0;
        // rows outside every region are not visited by a tile
        if (!cover && (e = msda::launch_fill_zero(grad_feat, gf_bytes, s)) != hipSuccess)
            return hip_fail(e, "zero grad_feat");
    }
    uint32_t* rec_count = nullptr;
    float* vt = nullptr;
    uint32_t* vis_place = nullptr;
    uint32_t* vis_items = nullptr;
    if (visible) {
        // invisible pairs take no part: their gradients are zero
        if (a.A > 0 && grad_weights &&
            (e = msda::launch_fill_zero(grad_weights, num_samples(desc) * a.G * sizeof(float),
                                        s)) != hipSuccess)
            return hip_fail(e, "zero grad_weights");
        if (a.A > 0 && grad_sampling_loc &&
            (e = msda::launch_fill_zero(grad_sampling_loc,
                                        num_samples(desc) / a.L * 2 * sizeof(float), s)) !=
                hipSuccess)
            return hip_fail(e, "zero grad_sampling_loc");
        float* grad_score = fuse ? fuse->grad_score : nullptr;   // written whole below
        if (a.A > 0 && (grad_feat || grad_sampling_loc || grad_weights || grad_score)) {
            uint32_t* place = vis_place = reinterpret_cast<uint32_t*>(ws + VW.place);
            uint32_t* items = vis_items = reinterpret_cast<uint32_t*>(ws + VW.items);
            rec_count = reinterpret_cast<uint32_t*>(ws + VW.rec_count);
            const size_t V = (size_t)a.B * a.N * a.A;
            if (fuse) {
                vt = reinterpret_cast<float*>(ws + VW.vt);
                if ((e = msda::launch_view_scale(visible, fuse->score, a.B * a.A, a.N, vt, s)) !=
                    hipSuccess)
                    return hip_fail(e, "fused view weights");
            }
            float* item_dot = grad_score ? reinterpret_cast<float*>(ws + VW.dot) : nullptr;
            if ((e = msda::launch_visible_items(visible, a.B, a.N, a.A, (uint32_t)(a.P * a.L),
                                                place, items, rec_count,
                                                reinterpret_cast<uint32_t*>(ws + VW.partial),
                                                s)) != hipSuccess ||
                (e = msda::launch_backward_visible(
                     a, desc->feat_dtype, cpl, waves, msda::lds_bytes_view(a, waves), items,
                     place, place + V,
                     grad_feat ? reinterpret_cast<uint32_t*>(ws + W.vals_a) : nullptr, vt,
                     item_dot, s)) != hipSuccess)
                return hip_fail(e, "msda_backward_visible launch");
            if (grad_score &&
                (e = msda::launch_grad_score(grad_out, fuse->out, visible, fuse->score, place,
                                             item_dot, a.B, a.A, a.N, a.C, grad_score, s)) !=
                    hipSuccess)
                return hip_fail(e, "grad_score");
        }
    } else if (a.A > 0 && (grad_feat || grad_sampling_loc || grad_weights) &&
               (e = launch_gather(a, order, desc->feat_dtype, cpl, waves, s)) != hipSuccess) {
        return hip_fail(e, "msda_backward launch");
    }
    if (!grad_feat) return finish();

    uint32_t* sorted = nullptr;
    uint32_t* off = reinterpret_cast<uint32_t*>(ws + W.off);
    if (a.rec_bucket_ap) {
        sorted = reinterpret_cast<uint32_t*>(ws + W.vals_a);
        e = msda::launch_bucket_sort(reinterpret_cast<uint32_t*>(ws + W.keys_a), spatial_shapes,
                                     a.B, a.N, a.L, a.A, a.P, (uint32_t)cells, sorted, off,
                                     cell_start, tile_start, tile_region, vis_place, vis_items,
                                     s);
    } else {
        e = msda::launch_sort_records(reinterpret_cast<uint32_t*>(ws + W.keys_a),
                                      reinterpret_cast<uint32_t*>(ws + W.keys_b),
                                      reinterpret_cast<uint32_t*>(ws + W.vals_a),
                                      reinterpret_cast<uint32_t*>(ws + W.vals_b), (uint32_t)nrec,
                                      (uint32_t)ncells, reinterpret_cast<uint32_t*>(ws + W.scratch),
                                      off, &sorted, s, rec_count, rec_count != nullptr);
    }
    if (e != hipSuccess) return hip_fail(e, "sort grad_feat records");
    msda::TileArgs t = {};
    t.vals = sorted ? sorted : reinterpret_cast<uint32_t*>(ws + W.vals_a);
    t.off = off;
    t.frac = a.rec_frac;
    t.w = weff;
    t.grad_out = grad_out;
    t.grad_feat = grad_feat;
    t.shapes = spatial_shapes;
    t.starts = level_start_index;
    t.cell_start = cell_start;
    t.tile_start = tile_start;
    t.tile_region = tile_region;
    t.tiles_per_item = (uint32_t)tiles;
    t.cells_per_item = (uint32_t)cells;
    t.nrec = (uint32_t)(nrec > 0 ? nrec : 1);
    t.NL = a.N * a.L;
    t.B = a.B;
    t.C = a.C;
    t.G = a.G;
    t.R = a.R;
    t.view_scale = vt;
    t.N = a.N;
    t.L = a.L;
    t.lps_shift = log2i(a.C / rcpl);
    divmagic((uint32_t)a.P * (uint32_t)a.N * (uint32_t)a.L, &t.magic, &t.magic_shift);
    // Tiles of coarse levels collect many more samples per pixel: they come
    // first in slot order and get 4 waves each (partial sums added as a
    // tree); the rest get one wave each.
    t.tile_begin = 0;
    t.tile_split = heavy_tiles(desc);
    t.tile_end = (uint32_t)tiles;
    if ((e = msda::launch_gfeat_tiles(t, desc->feat_dtype, rcpl, s)) != hipSuccess)
        return hip_fail(e, "grad_feat tile reduction");
    return finish();
}

msda_status msda_backward(const void* feat, const int32_t* spatial_shapes,
                          const int32_t* level_start_index, const float* sampling_loc,
                          const float* weights, const float* grad_out, void* grad_feat,
                          float* grad_sampling_loc, float* grad_weights, void* workspace,
                          size_t workspace_bytes, const msda_desc* desc, void* stream) {
    return backward_impl(feat, spatial_shapes, level_start_index, sampling_loc, weights, nullptr,
                         nullptr, grad_out, grad_feat, grad_sampling_loc, grad_weights, workspace,
                         workspace_bytes, desc, stream);
}

msda_status msda_backward_visible(const void* feat, const int32_t* spatial_shapes,
                                  const int32_t* level_start_index, const float* sampling_loc,
                                  const float* weights, const uint8_t* visible,
                                  const float* grad_out, void* grad_feat,
                                  float* grad_sampling_loc, float* grad_weights, void* workspace,
                                  size_t workspace_bytes, const msda_desc* desc, void* stream) {
    if (!visible && desc && desc->num_anchors > 0)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "visible is NULL");
    static const uint8_t none = 0;
    return backward_impl(feat, spatial_shapes, level_start_index, sampling_loc, weights,
                         visible ? visible : &none, nullptr, grad_out, grad_feat,
                         grad_sampling_loc, grad_weights, workspace, workspace_bytes, desc,
                         stream);
}

msda_status msda_backward_fused(const void* feat, const int32_t* spatial_shapes,
                                const int32_t* level_start_index, const float* sampling_loc,
                                const float* weights, const uint8_t* visible,
                                const float* view_score, const float* out,
                                const float* grad_out, void* grad_feat,
                                float* grad_sampling_loc, float* grad_weights,
                                float* grad_score, void* workspace, size_t workspace_bytes,
                                const msda_desc* desc, void* stream) {
    if (!visible && desc && desc->num_anchors > 0)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "visible is NULL");
    static const uint8_t none = 0;
    const Fusion fuse{view_score, out, grad_score};
    return backward_impl(feat, spatial_shapes, level_start_index, sampling_loc, weights,
                         visible ? visible : &none, &fuse, grad_out, grad_feat,
                         grad_sampling_loc, grad_weights, workspace, workspace_bytes, desc,
                         stream);
}

size_t msda_backward_fused_workspace_size(const msda_desc* d) {
    return msda_backward_visible_workspace_size(d);
}

size_t msda_backward_visible_workspace_size(const msda_desc* d) {
    if (!d || d->batch < 1 || d->rows < 1 || d->channels < 1 || d->num_anchors < 0) return 0;
    const size_t base = visible_layout(d, align256(base_backward_bytes(d))).total;
    const size_t extra = stats_bytes(d) + weights_f32_bytes(d);
    return extra ? align256(base) + extra : base;
}

// The visible-view forward's workspace: the compaction, then one partial
// row per (batch item, camera, anchor) item.
static size_t forward_visible_part(const msda_desc* d, size_t* part_off) {
    const VisibleWs vw = visible_layout(d, 0);
    *part_off = vw.total;
    const uint64_t V = (uint64_t)d->batch * d->num_cams * (uint64_t)d->num_anchors;
    return vw.total + align256(V * (uint64_t)d->channels * sizeof(float));
}

size_t msda_forward_visible_workspace_size(const msda_desc* d) {
    if (!d || d->batch < 1 || d->num_cams < 1 || d->channels < 1 || d->num_anchors < 0) return 0;
    size_t part_off;
    return align256(forward_visible_part(d, &part_off)) + stats_bytes(d);
}

static msda_status forward_visible_impl(const void* feat, const int32_t* spatial_shapes,
                                        const int32_t* level_start_index,
                                        const float* sampling_loc, const float* weights,
                                        const uint8_t* visible, bool fused, const float* score,
                                        float* out, void* workspace, size_t workspace_bytes,
                                        const msda_desc* desc, void* stream) {
    if (!desc) return fail(MSDA_ERR_INVALID_ARGUMENT, "desc is NULL");
    if (desc->tile && desc->tile->order == MSDA_ORDER_ANCHOR)
        return fail(MSDA_ERR_UNSUPPORTED, "the visible-view form runs in view order only");
    msda::OpArgs a = {};
    int cpl = 0, waves = 0;
    msda_status st = prepare(desc, MSDA_ORDER_VIEW, &a, &cpl, &waves);
    if (st != MSDA_OK) return st;
    if (!feat || !spatial_shapes || !level_start_index ||
        (a.A > 0 && (!sampling_loc || !weights || !out || !visible || (fused && !score))))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "a required device pointer is NULL");
    if (!aligned(feat, 16)) return fail(MSDA_ERR_UNSUPPORTED, "feat must be 16-byte aligned");
    if ((uint64_t)a.B * a.N * (uint64_t)a.A >= (1ull << 31))
        return fail(MSDA_ERR_UNSUPPORTED, "B * Ncam * A must be < 2^31");
    size_t part_off = 0;
    const size_t stats_off = align256(forward_visible_part(desc, &part_off));
    const size_t need = stats_off + stats_bytes(desc);
    if (a.A == 0) return ok();
    if (!workspace || workspace_bytes < need || !aligned(workspace, 256))
        return fail(MSDA_ERR_WORKSPACE, "forward workspace: need %zu bytes, 256-byte aligned "
                                        "(got %zu at %p)", need, workspace_bytes, workspace);
    a.feat = feat;
    a.shapes = spatial_shapes;
    a.starts = level_start_index;
    a.loc = sampling_loc;
    a.w = weights;
    a.level_scale = desc->feat_dtype == MSDA_FP8_E4M3 ? desc->level_scale : nullptr;
    a.out = out;
    char* ws = static_cast<char*>(workspace);
    const VisibleWs vw = visible_layout(desc, 0);
    uint32_t* place = reinterpret_cast<uint32_t*>(ws + vw.place);
    uint32_t* items = reinterpret_cast<uint32_t*>(ws + vw.items);
    const size_t V = (size_t)a.B * a.N * a.A;
    const hipStream_t s = (hipStream_t)stream;
    float* vt = fused ? reinterpret_cast<float*>(ws + vw.vt) : nullptr;
    const bool wbf16 = desc->flags & MSDA_WEIGHTS_BF16;
    a.w_bf16 = wbf16;
    if (desc->flags & MSDA_WEIGHT_LOGITS) {
        float2* stats = reinterpret_cast<float2*>(ws + stats_off);
        float2* spart = reinterpret_cast<float2*>(ws + stats_off + stats_only_bytes(desc));
        const hipError_t es = msda::launch_softmax_stats(weights, wbf16, a.B * a.A,
                                                         a.P * a.N * a.L, a.G, spart, stats, s);
        if (es != hipSuccess) return hip_fail(es, "softmax statistics");
        a.wstats = stats;
    }
    hipError_t e = msda::launch_visible_items(visible, a.B, a.N, a.A, 0u, place, items, nullptr,
                                              reinterpret_cast<uint32_t*>(ws + vw.partial), s);
    if (e == hipSuccess && fused) e = msda::launch_view_scale(visible, score, a.B * a.A, a.N, vt, s);
    if (e == hipSuccess)
        e = msda::launch_forward_visible(a, desc->feat_dtype, cpl, waves,
                                         msda::lds_bytes_view(a, waves), items, place + V, place,
                                         visible, vt, reinterpret_cast<float*>(ws + part_off), s);
    if (e != hipSuccess) return hip_fail(e, "msda_forward_visible launch");
    return ok();
}

msda_status msda_forward_visible(const void* feat, const int32_t* spatial_shapes,
                                 const int32_t* level_start_index, const float* sampling_loc,
                                 const float* weights, const uint8_t* visible, float* out,
                                 void* workspace, size_t workspace_bytes, const msda_desc* desc,
                                 void* stream) {
    return forward_visible_impl(feat, spatial_shapes, level_start_index, sampling_loc, weights,
                                visible, false, nullptr, out, workspace, workspace_bytes, desc,
                                stream);
}

msda_status msda_forward_fused(const void* feat, const int32_t* spatial_shapes,
                               const int32_t* level_start_index, const float* sampling_loc,
                               const float* weights, const uint8_t* visible,
                               const float* view_score, float* out, void* workspace,
                               size_t workspace_bytes, const msda_desc* desc, void* stream) {
    return forward_visible_impl(feat, spatial_shapes, level_start_index, sampling_loc, weights,
                                visible, true, view_score, out, workspace, workspace_bytes, desc,
                                stream);
}

size_t msda_forward_fused_workspace_size(const msda_desc* d) {
    return msda_forward_visible_workspace_size(d);
}

msda_status msda_project_keypoints(const float* anchors, const float* keypoints,
                                   const float* projection, const int32_t* image_hw,
                                   float* sampling_loc, uint8_t* visible,
                                   const msda_projection_desc* d, void* stream) {
    if (!d) return fail(MSDA_ERR_INVALID_ARGUMENT, "desc is NULL");
    if (d->batch < 1 || d->num_anchors < 0 || d->num_points < 1 || d->num_cams < 1)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "sizes must be positive (B=%d A=%d P=%d Ncam=%d)",
                    d->batch, d->num_anchors, d->num_points, d->num_cams);
    if ((uint64_t)d->batch * d->num_anchors * (uint64_t)d->num_points * d->num_cams >=
        (1ull << 31))
        return fail(MSDA_ERR_UNSUPPORTED, "B * A * P * Ncam must be < 2^31");
    if (!(d->dt == d->dt)) return fail(MSDA_ERR_INVALID_ARGUMENT, "dt is NaN");
    if (d->num_anchors == 0) return ok();
    if (!anchors || !keypoints || !projection || !image_hw || !sampling_loc || !visible)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "a required device pointer is NULL");
    msda::ProjArgs p = {};
    p.anchors = anchors;
    p.keypoints = keypoints;
    p.projection = projection;
    p.image_hw = image_hw;
    p.loc = sampling_loc;
    p.visible = visible;
    p.B = d->batch;
    p.A = d->num_anchors;
    p.P = d->num_points;
    p.N = d->num_cams;
    p.dt = d->dt;
    const hipError_t e = msda::launch_project_keypoints(p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "msda_project_keypoints launch");
    return ok();
}

size_t msda_quantize_workspace_size(const msda_desc* d) {
    if (!d || d->batch < 1 || d->num_cams < 1 || d->num_levels < 1) return 0;
    return (size_t)d->batch * (size_t)d->num_cams * (size_t)d->num_levels * sizeof(uint32_t);
}

msda_status msda_quantize_fp8(const float* feat_f32, const int32_t* spatial_shapes,
                              const int32_t* level_start_index, uint8_t* codes,
                              float* level_scale, void* workspace, size_t workspace_bytes,
                              const msda_desc* desc, void* stream) {
    if (!desc) return fail(MSDA_ERR_INVALID_ARGUMENT, "desc is NULL");
    msda_desc d = *desc;
    d.feat_dtype = MSDA_F32;            // the input is FP32
    d.level_scale = nullptr;
    int64_t batch_bytes = 0;
    msda_status st = check_regions(&d, &batch_bytes);
    if (st != MSDA_OK) return st;
    if (!feat_f32 || !spatial_shapes || !level_start_index || !codes || !level_scale)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "a required device pointer is NULL");
    if (!workspace || workspace_bytes < msda_quantize_workspace_size(desc))
        return fail(MSDA_ERR_WORKSPACE, "quantize workspace too small");
    if (!aligned(workspace, 4)) return fail(MSDA_ERR_WORKSPACE, "workspace must be 4-byte aligned");
    if (!aligned(codes, 4)) return fail(MSDA_ERR_INVALID_ARGUMENT, "codes must be 4-byte aligned");
    const hipStream_t s = (hipStream_t)stream;
    // Rows in no region read as code 0: zero the codes first unless the
    // regions tile [0, R) exactly (disjoint, no gaps).
    const int64_t NL = (int64_t)d.num_cams * d.num_levels;
    std::vector<std::pair<int64_t, int64_t>> spans((size_t)NL);
    int64_t max_rows = 0;
    for (int64_t i = 0; i < NL; ++i) {
        const int64_t n = (int64_t)d.host_spatial_shapes[2 * i] * d.host_spatial_shapes[2 * i + 1];
        spans[(size_t)i] = {d.host_level_start_index[i], n};
        max_rows = std::max(max_rows, n);
    }
    std::sort(spans.begin(), spans.end());
    int64_t end = 0;
    bool tiled = true;
    for (const auto& sp : spans) {
        if (sp.first != end) { tiled = false; break; }
        end = sp.first + sp.second;
    }
    tiled = tiled && end == d.rows;
    hipError_t e = hipSuccess;
    if (!tiled) {
        e = msda::launch_fill_zero(codes, (size_t)d.batch * d.rows * d.channels, s);
        if (e != hipSuccess) return hip_fail(e, "zero codes");
    }
    e = msda::launch_quantize_fp8(feat_f32, spatial_shapes, level_start_index, d.batch,
                                  d.num_cams, d.num_levels, d.rows, d.channels, max_rows, codes,
                                  level_scale, static_cast<uint32_t*>(workspace), s);
    if (e != hipSuccess) return hip_fail(e, "msda_quantize_fp8 launch");
    return ok();
}

// ---------------------------------------------------------------- batched form

}  // extern "C"

namespace {

struct BatchWs {
    size_t anchor_start, sample_start, region_start, cell_start, slot_scene, slot_region,
        tile_start, magic, magic_shift, keys_a, keys_b, vals_a, vals_b, frac, off, scratch, part,
        wstats, wscratch, w32, total;
};

// Weight-flag buffers of a batch: softmax statistics per anchor of every
// scene, one softmax scratch (the per-scene launches run in stream order and
// share it), and for the backward the FP32 weights of every sample.
struct BatchWeights {
    uint64_t stats_bytes, scratch_bytes, w32_bytes;
};

// part_bytes: the view-order forward's per-slot partial sums (always part of
// the forward's workspace, so that the order can change without resizing).
BatchWs batch_layout(uint64_t S, uint64_t regions, uint64_t nsamp, uint64_t ncells, bool records,
                     uint64_t part_bytes = 0, const BatchWeights& wb = BatchWeights{}) {
    BatchWs w = {};
    size_t at = 0;
    auto take = [&](size_t bytes) { const size_t here = at; at += align256(bytes); return here; };
    w.anchor_start = take((S + 1) * 4);
    w.sample_start = take((S + 1) * 4);
    w.region_start = take((S + 1) * 4);
    w.cell_start = take(regions * 4);
    w.slot_scene = take(regions * 4);
    w.slot_region = take(regions * 4);
    w.tile_start = take((regions + 1) * 4);
    w.magic = take(S * 8);
    w.magic_shift = take(S * 4);
    if (records) {
        w.keys_a = take(nsamp * 4);
        w.keys_b = take(nsamp * 4);
        w.vals_a = take(nsamp * 4);
        w.vals_b = take(nsamp * 4);
        w.frac = take(nsamp * 8);
        w.off = take((ncells + 1) * 4);
        w.scratch = take(msda::sort_scratch_words((uint32_t)nsamp) * 4);
    }
    if (part_bytes) w.part = take(part_bytes);
    if (wb.stats_bytes) w.wstats = take(wb.stats_bytes);
    if (wb.scratch_bytes) w.wscratch = take(wb.scratch_bytes);
    if (wb.w32_bytes) w.w32 = take(wb.w32_bytes);
    w.total = at;
    return w;
}

// Sizes of a validated batch.
struct BatchPlan {
    uint64_t anchors, samples, regions, cells, tiles, heavy_tiles;
    int max_regions_per_scene, max_cams;
    int cpl, waves;
    int64_t max_batch_bytes;
    int order;                    // MSDA_ORDER_ANCHOR or MSDA_ORDER_VIEW
    int view_cams;                // view order: cameras of a row at most
    int view_waves_fwd, view_waves_bwd;
    uint64_t part_bytes;          // view-order forward partials
    uint64_t max_ap;              // the largest A_s * P
    bool keys_fit;                // every region's cells fit the bucket sort's keys
};

// Validates the batch (every scene against its host mirrors) and sizes it.
msda_status plan_batch(const msda_batch* b, bool backward, BatchPlan* p) {
    if (!b) return fail(MSDA_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (b->num_scenes < 1 || b->num_scenes > msda::kMaxBatchScenes)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "num_scenes=%d not in [1, %d]", b->num_scenes,
                    msda::kMaxBatchScenes);
    if (!b->scenes || !b->host_scenes || !b->host_spatial_shapes || !b->host_level_start_index)
        return fail(MSDA_ERR_INVALID_ARGUMENT, "scene table or host mirrors are NULL");
    if (b->flags & ~(MSDA_DETERMINISTIC | kWeightFlags))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", (unsigned)b->flags);
    *p = BatchPlan{};
    p->keys_fit = true;
    const int eb = elem_bytes(b->feat_dtype);
    for (int s = 0; s < b->num_scenes; ++s) {
        const msda_scene& sc = b->host_scenes[s];
        msda_desc d = {};
        d.batch = 1;
        d.num_cams = sc.num_cams;
        d.num_levels = b->num_levels;
        d.num_anchors = sc.num_anchors;
        d.num_points = b->num_points;
        d.channels = b->channels;
        d.groups = b->groups;
        d.feat_dtype = b->feat_dtype;
        d.rows = sc.rows;
        d.host_spatial_shapes = b->host_spatial_shapes[s];
        d.host_level_start_index = b->host_level_start_index[s];
        d.level_scale = b->level_scale;
        d.flags = b->flags;
        d.tile = b->tile;
        int64_t bb = 0;
        msda_status st = check_regions(&d, &bb);
        if (st != MSDA_OK) {
            const std::string msg = g_error;
            return fail(st, "scene %d: %s", s, msg.c_str());
        }
        if (!sc.feat || !sc.spatial_shapes || !sc.level_start_index)
            return fail(MSDA_ERR_INVALID_ARGUMENT, "scene %d: a required device pointer is NULL", s);
        if (sc.num_anchors > 0 && (!sc.sampling_loc || !sc.weights ||
                                   (backward ? !sc.grad_out : !sc.out)))
            return fail(MSDA_ERR_INVALID_ARGUMENT, "scene %d: a required device pointer is NULL", s);
        if (!aligned(sc.feat, 16))
            return fail(MSDA_ERR_UNSUPPORTED, "scene %d: feat must be 16-byte aligned", s);
        p->anchors += (uint64_t)sc.num_anchors;
        p->samples += (uint64_t)sc.num_anchors * b->num_points * sc.num_cams * b->num_levels;
        p->regions += (uint64_t)sc.num_cams * b->num_levels;
        p->max_regions_per_scene = std::max(p->max_regions_per_scene, sc.num_cams * b->num_levels);
        p->max_cams = std::max(p->max_cams, sc.num_cams);
        p->max_batch_bytes = std::max<int64_t>(p->max_batch_bytes, bb);
        uint64_t cells = 0, tiles = 0;
        cells_and_tiles(&d, &cells, &tiles);
        p->cells += cells;
        p->tiles += tiles;
        p->max_ap = std::max<uint64_t>(p->max_ap, (uint64_t)sc.num_anchors * b->num_points);
        if (!bucket_keys_fit(d.host_spatial_shapes, (int64_t)sc.num_cams * b->num_levels))
            p->keys_fit = false;
        // heavy (scene, level): camera 0's area at most 1/16 of its largest level
        int64_t max_area = 0;
        for (int l = 0; l < b->num_levels; ++l)
            max_area = std::max<int64_t>(max_area, (int64_t)d.host_spatial_shapes[2 * l] *
                                                       d.host_spatial_shapes[2 * l + 1]);
        for (int l = 0; l < b->num_levels; ++l) {
            if ((int64_t)d.host_spatial_shapes[2 * l] * d.host_spatial_shapes[2 * l + 1] * 16 >
                max_area)
                continue;
            for (int n = 0; n < sc.num_cams; ++n) {
                const int r = n * b->num_levels + l;
                const uint64_t H = d.host_spatial_shapes[2 * r], W = d.host_spatial_shapes[2 * r + 1];
                p->heavy_tiles += ((H + msda::kTileH - 1) / msda::kTileH) *
                                  ((W + msda::kTileW - 1) / msda::kTileW);
            }
        }
    }
    (void)eb;
    if (p->regions > (uint64_t)msda::kMaxBatchRegions)
        return fail(MSDA_ERR_UNSUPPORTED, "%llu (camera, level) regions in the batch (limit %d)",
                    (unsigned long long)p->regions, msda::kMaxBatchRegions);
    if (p->anchors > 0x7fffffffull)
        return fail(MSDA_ERR_UNSUPPORTED, "too many anchors in the batch");
    // launch shape, from a single-call descriptor of the largest scene
    msda_desc d = {};
    d.batch = 1;
    d.num_cams = p->max_cams;
    d.num_levels = b->num_levels;
    d.num_anchors = (int32_t)std::min<uint64_t>(p->anchors, 0x7fffffff);
    d.num_points = b->num_points;
    d.channels = b->channels;
    d.groups = b->groups;
    d.feat_dtype = b->feat_dtype;
    d.rows = 1;
    d.tile = b->tile;
    msda::OpArgs a = {};
    // prepare() needs valid host mirrors: one 1x1 region per camera and level
    std::vector<int32_t> shp((size_t)p->max_cams * b->num_levels * 2, 1), st((size_t)p->max_cams * b->num_levels);
    for (size_t i = 0; i < st.size(); ++i) st[i] = (int32_t)i;
    d.rows = (int64_t)st.size();
    d.host_spatial_shapes = shp.data();
    d.host_level_start_index = st.data();
    d.level_scale = b->level_scale;
    msda_status stt = prepare(&d, MSDA_ORDER_ANCHOR, &a, &p->cpl, &p->waves);
    if (stt != MSDA_OK) return stt;
    // work order: view order (one camera range per XCD) unless anchor order
    // is asked for; each scene is split over the XCD slots as a single call
    // with B = 1 would be, and a row covers at most max_cams / 8 + 2 cameras
    const int req = b->tile ? b->tile->order : MSDA_ORDER_AUTO;
    if (req != MSDA_ORDER_AUTO && req != MSDA_ORDER_ANCHOR && req != MSDA_ORDER_VIEW)
        return fail(MSDA_ERR_UNSUPPORTED, "unknown order %d", req);
    p->order = req == MSDA_ORDER_ANCHOR ? MSDA_ORDER_ANCHOR : MSDA_ORDER_VIEW;
    p->view_cams = p->max_cams / msda::kSlots + 2;
    const int tw = b->tile ? b->tile->waves_per_anchor : 0;
    p->view_waves_fwd = tw ? tw : 1;
    p->view_waves_bwd = tw ? tw : 4;
    p->part_bytes = (uint64_t)msda::kSlots * p->anchors * (uint64_t)b->channels * sizeof(float);
    if (p->order == MSDA_ORDER_VIEW) {
        const int J = msda::max_pairs_per_chunk(b->num_levels, b->groups);
        const int wmax = std::max(p->view_waves_fwd, p->view_waves_bwd);
        const size_t need = msda::batch_view_lds(p->view_cams, b->num_levels, J, b->groups, wmax);
        if (need > 65536)
            return fail(MSDA_ERR_UNSUPPORTED, "view-order batched launch needs %zu bytes of LDS",
                        need);
    }
    return MSDA_OK;
}

void fill_batch_args(const msda_batch* b, const BatchPlan& p, char* ws, const BatchWs& w,
                     msda::BatchArgs* a) {
    *a = msda::BatchArgs{};
    a->scenes = b->scenes;
    a->S = b->num_scenes;
    a->L = b->num_levels;
    a->P = b->num_points;
    a->C = b->channels;
    a->G = b->groups;
    a->level_scale = b->feat_dtype == MSDA_FP8_E4M3 ? b->level_scale : nullptr;
    a->t.anchor_start = reinterpret_cast<uint32_t*>(ws + w.anchor_start);
    a->t.sample_start = reinterpret_cast<uint32_t*>(ws + w.sample_start);
    a->t.region_start = reinterpret_cast<uint32_t*>(ws + w.region_start);
    a->t.cell_start = reinterpret_cast<uint32_t*>(ws + w.cell_start);
    a->t.slot_scene = reinterpret_cast<uint32_t*>(ws + w.slot_scene);
    a->t.slot_region = reinterpret_cast<uint32_t*>(ws + w.slot_region);
    a->t.tile_start = reinterpret_cast<uint32_t*>(ws + w.tile_start);
    a->t.magic = reinterpret_cast<uint64_t*>(ws + w.magic);
    a->t.magic_shift = reinterpret_cast<uint32_t*>(ws + w.magic_shift);
    a->total_anchors = (uint32_t)p.anchors;
    a->total_samples = (uint32_t)p.samples;
    a->total_cells = (uint32_t)p.cells;
    a->total_regions = (uint32_t)p.regions;
    a->lps_shift = log2i(b->channels / p.cpl);
    a->pairs_per_chunk = msda::max_pairs_per_chunk(b->num_levels, b->groups);
    a->max_regions_per_scene = p.max_regions_per_scene;
    a->view_cams = p.view_cams;
}

// The weight-flag buffers of a batch (all zero without a weight flag).
BatchWeights batch_weights(const msda_batch* b, const BatchPlan& p, bool backward) {
    BatchWeights w{};
    if (b->flags & MSDA_WEIGHT_LOGITS) {
        w.stats_bytes = p.anchors * (uint64_t)b->groups * sizeof(float2);
        for (int sc = 0; sc < b->num_scenes; ++sc) {
            const msda_scene& h = b->host_scenes[sc];
            if (h.num_anchors > 0)
                w.scratch_bytes = std::max<uint64_t>(
                    w.scratch_bytes,
                    msda::softmax_scratch_bytes(h.num_anchors,
                                                b->num_points * h.num_cams * b->num_levels,
                                                b->groups));
        }
    }
    if (backward && (b->flags & kWeightFlags)) w.w32_bytes = p.samples * (uint64_t)b->groups * 4;
    return w;
}

// Under a weight flag, per scene with anchors (in stream order): the softmax
// statistics of its logits, and for the backward its FP32 weights (softmax
// weights, or BF16 weights widened) at its samples' place, which the
// batched kernels then read in place of the scene's weights.
msda_status batch_weight_prep(const msda_batch* b, char* ws, const BatchWs& w, bool backward,
                              msda::BatchArgs* a, hipStream_t s) {
    const bool logits = b->flags & MSDA_WEIGHT_LOGITS, wbf16 = b->flags & MSDA_WEIGHTS_BF16;
    if (!logits && !wbf16) return MSDA_OK;
    float2* stats = logits ? reinterpret_cast<float2*>(ws + w.wstats) : nullptr;
    float2* part = logits ? reinterpret_cast<float2*>(ws + w.wscratch) : nullptr;
    float* w32 = backward ? reinterpret_cast<float*>(ws + w.w32) : nullptr;
    const int G = b->groups;
    uint64_t a0 = 0, s0 = 0;
    for (int sc = 0; sc < b->num_scenes; ++sc) {
        const msda_scene& h = b->host_scenes[sc];
        const int A = h.num_anchors, PNL = b->num_points * h.num_cams * b->num_levels;
        if (A > 0) {
            float2* st = logits ? stats + a0 * G : nullptr;
            hipError_t e = hipSuccess;
            if (logits && (e = msda::launch_softmax_stats(h.weights, wbf16, A, PNL, G, part, st,
                                                          s)) != hipSuccess)
                return hip_fail(e, "batched softmax statistics");
            if (w32 && (e = msda::launch_weights_f32(h.weights, wbf16, st, A, PNL, G,
                                                     w32 + s0 * G, s)) != hipSuccess)
                return hip_fail(e, "batched FP32 weights");
        }
        a0 += (uint64_t)(A > 0 ? A : 0);
        s0 += (uint64_t)(A > 0 ? A : 0) * (uint64_t)PNL;
    }
    if (backward) {
        a->w32 = w32;
    } else {
        a->wstats = stats;
        a->w_bf16 = wbf16 ? 1 : 0;
    }
    return MSDA_OK;
}

// With logits, grad_weights as the gather leaves it (with respect to the
// softmax weights) mapped in place to the logits' gradient, per scene.
msda_status batch_softmax_grad(const msda_batch* b, char* ws, const BatchWs& w, hipStream_t s) {
    if (!(b->flags & MSDA_WEIGHT_LOGITS)) return MSDA_OK;
    const float* w32 = reinterpret_cast<const float*>(ws + w.w32);
    float* part = reinterpret_cast<float*>(ws + w.wscratch);
    const int G = b->groups;
    uint64_t s0 = 0;
    for (int sc = 0; sc < b->num_scenes; ++sc) {
        const msda_scene& h = b->host_scenes[sc];
        const int A = h.num_anchors, PNL = b->num_points * h.num_cams * b->num_levels;
        if (A > 0 && h.grad_weights) {
            const hipError_t e = msda::launch_softmax_grad(w32 + s0 * G, h.grad_weights, A, PNL, G,
                                                           part, s);
            if (e != hipSuccess) return hip_fail(e, "batched gradient through the softmax");
        }
        s0 += (uint64_t)(A > 0 ? A : 0) * (uint64_t)PNL;
    }
    return MSDA_OK;
}

size_t batch_lds(const msda_batch* b, const BatchPlan& p) {
    msda::OpArgs o = {};
    o.N = p.max_cams;
    o.L = b->num_levels;
    o.G = b->groups;
    o.C = b->channels;
    o.pairs_per_chunk = msda::max_pairs_per_chunk(b->num_levels, b->groups);
    return msda::lds_bytes_for(o, p.waves);
}

int persistent_blocks(uint64_t items, int waves) {
    const uint64_t cap = 256ull * (uint64_t)(16 / waves);     // 256 CUs, ~16 waves each
    return (int)std::max<uint64_t>(1, std::min(items, cap));
}

// Which gradients the batch asks for; they must agree over the scenes.
// grad_sampling_loc and grad_weights of a scene without anchors hold no
// elements and may be NULL either way.
msda_status batch_grads(const msda_batch* b, bool* gf, bool* gl, bool* gw) {
    const msda_scene& s0 = b->host_scenes[0];
    *gf = s0.grad_feat != nullptr;
    int ref = -1;                                   // first scene with anchors
    for (int s = 0; s < b->num_scenes && ref < 0; ++s)
        if (b->host_scenes[s].num_anchors > 0) ref = s;
    *gl = ref >= 0 && b->host_scenes[ref].grad_sampling_loc != nullptr;
    *gw = ref >= 0 && b->host_scenes[ref].grad_weights != nullptr;
    for (int s = 0; s < b->num_scenes; ++s) {
        const msda_scene& sc = b->host_scenes[s];
        const bool empty = sc.num_anchors == 0;
        if ((sc.grad_feat != nullptr) != *gf ||
            (!empty && ((sc.grad_sampling_loc != nullptr) != *gl ||
                        (sc.grad_weights != nullptr) != *gw)))
            return fail(MSDA_ERR_INVALID_ARGUMENT,
                        "scene %d requests other gradients than scene %d (NULL in all or none)", s,
                        ref < 0 ? 0 : ref);
    }
    return MSDA_OK;
}

}  // namespace

extern "C" {

size_t msda_batched_workspace_size(const msda_batch* b, int32_t backward) {
    BatchPlan p;
    if (plan_batch(b, backward != 0, &p) != MSDA_OK) return 0;
    bool gf = false, gl = false, gw = false;
    if (backward && batch_grads(b, &gf, &gl, &gw) != MSDA_OK) return 0;
    return batch_layout(b->num_scenes, p.regions, p.samples, p.cells, backward && gf,
                        backward ? 0 : p.part_bytes, batch_weights(b, p, backward != 0))
        .total;
}

msda_status msda_forward_batched(const msda_batch* b, void* workspace, size_t workspace_bytes,
                                 void* stream) {
    BatchPlan p;
    msda_status st = plan_batch(b, false, &p);
    if (st != MSDA_OK) return st;
    const BatchWs w = batch_layout(b->num_scenes, p.regions, p.samples, p.cells, false,
                                   p.part_bytes, batch_weights(b, p, false));
    if (!workspace || workspace_bytes < w.total)
        return fail(MSDA_ERR_WORKSPACE, "workspace of %zu bytes needed", w.total);
    if (!aligned(workspace, 256)) return fail(MSDA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t lds = batch_lds(b, p);
    if (lds > 65536) return fail(MSDA_ERR_UNSUPPORTED, "batched launch needs %zu bytes of LDS", lds);
    msda::BatchArgs a;
    fill_batch_args(b, p, static_cast<char*>(workspace), w, &a);
    const hipStream_t s = (hipStream_t)stream;
    hipError_t e = msda::launch_batch_tables(a, false, s);
    if (e != hipSuccess) return hip_fail(e, "batch tables");
    if (p.anchors == 0) return ok();
    if ((st = batch_weight_prep(b, static_cast<char*>(workspace), w, false, &a, s)) != MSDA_OK)
        return st;
    if (p.order == MSDA_ORDER_VIEW) {
        const size_t vlds = msda::batch_view_lds(p.view_cams, b->num_levels, a.pairs_per_chunk,
                                                 b->groups, p.view_waves_fwd);
        e = msda::launch_forward_batched_view(
            a, b->feat_dtype, p.cpl, p.view_waves_fwd, vlds,
            reinterpret_cast<float*>(static_cast<char*>(workspace) + w.part), s);
    } else {
        e = msda::launch_forward_batched(a, b->feat_dtype, p.cpl, p.waves,
                                         persistent_blocks(p.anchors, p.waves), lds, s);
    }
    if (e != hipSuccess) return hip_fail(e, "msda_forward_batched launch");
    return ok();
}

msda_status msda_backward_batched(const msda_batch* b, void* workspace, size_t workspace_bytes,
                                  void* stream) {
    BatchPlan p;
    msda_status st = plan_batch(b, true, &p);
    if (st != MSDA_OK) return st;
    if (b->feat_dtype == MSDA_FP8_E4M3)
        return fail(MSDA_ERR_UNSUPPORTED, "the backward takes FP32 or BF16 features (not FP8)");
    if (b->tile && b->tile->scatter == MSDA_SCATTER_ATOMIC)
        return fail(MSDA_ERR_UNSUPPORTED, "the batched backward has only the sorted grad_feat form");
    bool gf, gl, gw;
    if ((st = batch_grads(b, &gf, &gl, &gw)) != MSDA_OK) return st;
    int rcpl = 0;
    for (int c : {4, 2, 1})
        if (cpl_fits(c, b->channels, b->groups)) { rcpl = c; break; }
    if (gf) {
        if (p.samples >= (1ull << 30))
            return fail(MSDA_ERR_UNSUPPORTED, "%llu samples in the batch exceeds 2^30",
                        (unsigned long long)p.samples);
        if (p.cells >= 0x7fffffffull)
            return fail(MSDA_ERR_UNSUPPORTED, "too many bilinear cells in the batch");
        if (!rcpl) return fail(MSDA_ERR_UNSUPPORTED, "no reduction lane layout for C=%d G=%d",
                               b->channels, b->groups);
        if (b->groups > 64) return fail(MSDA_ERR_UNSUPPORTED, "sorted grad_feat supports G <= 64");
    }
    for (int s = 0; s < b->num_scenes; ++s) {
        const msda_scene& sc = b->host_scenes[s];
        if (gf && !aligned(sc.grad_feat, 16))
            return fail(MSDA_ERR_UNSUPPORTED, "scene %d: grad_feat must be 16-byte aligned", s);
        if (gf && rcpl == 4 && sc.grad_out && !aligned(sc.grad_out, 16))
            return fail(MSDA_ERR_UNSUPPORTED, "scene %d: grad_out must be 16-byte aligned", s);
        if (gf) {
            msda_desc d = {};
            d.num_cams = sc.num_cams;
            d.num_levels = b->num_levels;
            d.rows = sc.rows;
            d.host_spatial_shapes = b->host_spatial_shapes[s];
            d.host_level_start_index = b->host_level_start_index[s];
            bool cover = true;
            if (!regions_disjoint(&d, &cover))
                return fail(MSDA_ERR_UNSUPPORTED, "scene %d: grad_feat needs disjoint regions", s);
        }
    }
    const BatchWs w = batch_layout(b->num_scenes, p.regions, p.samples, p.cells, gf, 0,
                                   batch_weights(b, p, true));
    if (!workspace || workspace_bytes < w.total)
        return fail(MSDA_ERR_WORKSPACE, "workspace of %zu bytes needed", w.total);
    if (!aligned(workspace, 256)) return fail(MSDA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t lds = batch_lds(b, p);
    if (lds > 65536) return fail(MSDA_ERR_UNSUPPORTED, "batched launch needs %zu bytes of LDS", lds);

    char* ws = static_cast<char*>(workspace);
    msda::BatchArgs a;
    fill_batch_args(b, p, ws, w, &a);
    const hipStream_t s = (hipStream_t)stream;
    hipError_t e = msda::launch_batch_tables(a, true, s);
    if (e != hipSuccess) return hip_fail(e, "batch tables");
    if (p.anchors > 0 && (st = batch_weight_prep(b, ws, w, true, &a, s)) != MSDA_OK) return st;
    // grad_feat records bucketed per (scene, region) when every bucket fits
    // one bucket-sort block (sorted by launch_bucket_sort_batched), else in
    // sample order with batch-global cells (the global radix sort)
    const bool bucketed = gf && p.keys_fit && p.max_ap <= msda::kBucketMaxRecords &&
                          bucket_lds_fits(p.max_ap) &&
                          !(b->tile && b->tile->scatter == MSDA_SCATTER_SORTED_GLOBAL);
    if (gf) {
        a.rec_key = reinterpret_cast<uint32_t*>(ws + w.keys_a);
        a.rec_frac = reinterpret_cast<float2*>(ws + w.frac);
        a.rec_bucketed = bucketed ? 1 : 0;
        // rows outside every region are not visited by a tile
        for (int sc = 0; sc < b->num_scenes; ++sc) {
            msda_desc d = {};
            d.num_cams = b->host_scenes[sc].num_cams;
            d.num_levels = b->num_levels;
            d.rows = b->host_scenes[sc].rows;
            d.host_spatial_shapes = b->host_spatial_shapes[sc];
            d.host_level_start_index = b->host_level_start_index[sc];
            bool cover = true;
            regions_disjoint(&d, &cover);
            if (!cover) {
                const size_t bytes = (size_t)d.rows * b->channels * (b->feat_dtype == MSDA_F32 ? 4 : 2);
                if ((e = msda::launch_fill_zero(b->host_scenes[sc].grad_feat, bytes, s)) != hipSuccess)
                    return hip_fail(e, "zero grad_feat");
            }
        }
    }
    if (p.anchors > 0 && (gf || gl || gw)) {
        if (p.order == MSDA_ORDER_VIEW) {
            const size_t vlds = msda::batch_view_lds(p.view_cams, b->num_levels,
                                                     a.pairs_per_chunk, b->groups,
                                                     p.view_waves_bwd);
            e = msda::launch_backward_batched_view(a, b->feat_dtype, p.cpl, p.view_waves_bwd,
                                                   vlds, s);
        } else {
            e = msda::launch_backward_batched(a, b->feat_dtype, p.cpl, p.waves,
                                              persistent_blocks(p.anchors, p.waves), lds, s);
        }
        if (e != hipSuccess) return hip_fail(e, "msda_backward_batched launch");
    }
    if (!gf) return p.anchors > 0 ? batch_softmax_grad(b, ws, w, s) : ok();
    uint32_t* sorted = nullptr;
    uint32_t* off = reinterpret_cast<uint32_t*>(ws + w.off);
    if (bucketed)
        e = msda::launch_bucket_sort_batched(a, (uint32_t)p.max_ap,
                                             reinterpret_cast<uint32_t*>(ws + w.vals_a), off, s);
    else
        e = msda::launch_sort_records(reinterpret_cast<uint32_t*>(ws + w.keys_a),
                                      reinterpret_cast<uint32_t*>(ws + w.keys_b),
                                      reinterpret_cast<uint32_t*>(ws + w.vals_a),
                                      reinterpret_cast<uint32_t*>(ws + w.vals_b),
                                      (uint32_t)p.samples, (uint32_t)p.cells,
                                      reinterpret_cast<uint32_t*>(ws + w.scratch), off, &sorted, s);
    if (e != hipSuccess) return hip_fail(e, "sort grad_feat records");
    a.vals = sorted ? sorted : reinterpret_cast<uint32_t*>(ws + w.vals_a);
    a.off = off;
    a.total_samples = (uint32_t)std::max<uint64_t>(p.samples, 1);
    a.lps_shift = log2i(b->channels / rcpl);
    a.tile_begin = 0;
    a.tile_split = (uint32_t)p.heavy_tiles;
    a.tile_end = (uint32_t)p.tiles;
    if ((e = msda::launch_gfeat_tiles_batched(a, b->feat_dtype, rcpl, s)) != hipSuccess)
        return hip_fail(e, "batched grad_feat tile reduction");
    return p.anchors > 0 ? batch_softmax_grad(b, ws, w, s) : ok();
}

namespace {
struct SortWs { size_t keys_a, keys_b, vals_a, vals_b, scratch, total; };
SortWs sort_layout(uint32_t n) {
    SortWs w = {};
    size_t at = 0;
    auto take = [&](size_t bytes) { const size_t here = at; at += align256(bytes); return here; };
    w.keys_a = take((size_t)n * 4);
    w.keys_b = take((size_t)n * 4);
    w.vals_a = take((size_t)n * 4);
    w.vals_b = take((size_t)n * 4);
    w.scratch = take(msda::sort_scratch_words(n) * 4);
    w.total = at;
    return w;
}
}  // namespace

size_t msda_sort_workspace_size(uint32_t n, uint32_t max_key) {
    (void)max_key;
    return sort_layout(n).total;
}

msda_status msda_sort_keys(const uint32_t* keys, uint32_t n, uint32_t max_key, uint32_t* order,
                           uint32_t* seg, void* workspace, size_t workspace_bytes, void* stream) {
    if (!seg || (n > 0 && (!keys || !order)))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "a required device pointer is NULL");
    if (max_key == UINT32_MAX) return fail(MSDA_ERR_INVALID_ARGUMENT, "max_key must be < 2^32 - 1");
    if (n > (1u << 31)) return fail(MSDA_ERR_INVALID_ARGUMENT, "n must be <= 2^31");
    const SortWs w = sort_layout(n);
    if (!workspace || workspace_bytes < w.total)
        return fail(MSDA_ERR_WORKSPACE, "sort workspace too small");
    if (!aligned(workspace, 256)) return fail(MSDA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const hipStream_t s = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    hipError_t e = hipSuccess;
    if (n > 0 && (e = hipMemcpyAsync(ws + w.keys_a, keys, (size_t)n * 4,
                                     hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return hip_fail(e, "copy keys");
    uint32_t* sorted = nullptr;
    e = msda::launch_sort_records(reinterpret_cast<uint32_t*>(ws + w.keys_a),
                                  reinterpret_cast<uint32_t*>(ws + w.keys_b),
                                  reinterpret_cast<uint32_t*>(ws + w.vals_a),
                                  reinterpret_cast<uint32_t*>(ws + w.vals_b), n, max_key,
                                  reinterpret_cast<uint32_t*>(ws + w.scratch), seg, &sorted, s);
    if (e != hipSuccess) return hip_fail(e, "msda_sort_keys launch");
    if (n > 0 && (e = hipMemcpyAsync(order, sorted, (size_t)n * 4, hipMemcpyDeviceToDevice, s)) !=
                     hipSuccess)
        return hip_fail(e, "copy order");
    return ok();
}

msda_status msda_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src) return fail(MSDA_ERR_INVALID_ARGUMENT, "NULL pointer");
    if (bytes % 16 || !aligned(dst, 16) || !aligned(src, 16))
        return fail(MSDA_ERR_INVALID_ARGUMENT, "copy needs 16-byte aligned pointers and size");
    const hipError_t e = msda::launch_stream_copy(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "msda_stream_copy launch");
    return ok();
}

}  // extern "C"
