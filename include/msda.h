/*
 * msda.h -- C ABI of the MI355X (gfx950) multi-scale deformable aggregation
 * (MSDA) library, libmsda.so.
 *
 * The operator (paper Sec. 3.1 and Sec. 3.2; named and accelerated in
 * Sec. 5.3): the keypoints of every 3D anchor are projected into every camera;
 * at each projected point the camera's multi-level feature pyramid is sampled
 * bilinearly, and the samples are summed with one weight per (keypoint,
 * camera, level, channel group) into a single C-channel feature per anchor:
 *
 *   out[b,a,c] = sum_{p,n,l} weights[b,a,p,n,l,c/(C/G)] *
 *                bilinear(feat[b, region(n,l)], u*W_nl - 0.5, v*H_nl - 0.5)[c]
 *
 * with (u, v) = sampling_loc[b,a,p,n], pixel centres at integer + 0.5, a
 * neighbour outside the level contributing zero, and a sample skipped unless
 * -1 < x < W and -1 < y < H.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layouts (row-major, contiguous, element strides implied):
 *   feat               [B][R][C]          R rows per batch item, channels fastest;
 *                                          FP32, BF16, FP16 or FP8-e4m3 (OCP e4m3fn)
 *   spatial_shapes     [Ncam][L][2] int32 (H, W) of level l of camera n
 *   level_start_index  [Ncam][L]   int32  first row of region (n, l) in a batch item
 *   sampling_loc       [B][A][P][Ncam][2] FP32, (x, y) normalised so 0..1 spans the image
 *   weights            [B][A][P][Ncam][L][G] FP32; channel c uses group c / (C/G)
 *   out, grad_out      [B][A][C] FP32
 *   grad_sampling_loc  like sampling_loc, grad_weights like weights (FP32)
 *   grad_feat          like feat, in the feat dtype (FP32, BF16 or FP16)
 * Pointers named "device" are HIP device memory; "host" pointers are read
 * during the call only. The caller owns every buffer, including workspaces;
 * the library never allocates, frees or synchronises on these calls, so they
 * may be captured into a HIP graph. Outputs are overwritten, never
 * accumulated into, and must not alias inputs. Out-of-range samples give exact
 * zeros in every output. Work is enqueued on `stream` (a hipStream_t; NULL =
 * the null stream) and the call returns before it completes.
 *
 * Errors: every argument is validated on the host before anything is
 * enqueued; on failure nothing is launched, no output is touched, and the
 * status says why (msda_last_error() has the message, thread-local, valid
 * until the next call on the thread). A HIP launch error returns
 * MSDA_ERR_HIP. Nothing aborts, nothing throws across the ABI. Device faults
 * are reported by HIP asynchronously, at the caller's next synchronisation.
 */
#ifndef MSDA_H
#define MSDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSDA_ABI_VERSION 8

typedef enum msda_status {
    MSDA_OK = 0,
    MSDA_ERR_INVALID_ARGUMENT = 1, /* sizes, pointers or regions inconsistent      */
    MSDA_ERR_UNSUPPORTED = 2,      /* valid request this build does not implement  */
    MSDA_ERR_HIP = 3,              /* the HIP runtime reported an error            */
    MSDA_ERR_WORKSPACE = 4         /* workspace missing, too small or misaligned   */
} msda_status;

typedef enum msda_dtype {
    MSDA_F32 = 0,
    MSDA_BF16 = 1,
    MSDA_FP8_E4M3 = 2, /* OCP e4m3fn codes; value = decode(code) * level_scale[l] */
    MSDA_F16 = 3       /* IEEE binary16; grad_feat also binary16 (FP32 sums, one RNE rounding) */
} msda_dtype;

/* msda_desc.flags */
#define MSDA_DETERMINISTIC 1u /* backward: grad_feat must be summed in a fixed order
                                 (bitwise reproducible run to run); rejects
                                 MSDA_SCATTER_ATOMIC */
/* Fused weight generation (the weights' upstream step, paper Sec. 3.1 / 3.2):
 * `weights` holds logits, and the operator uses their softmax over the P*Ncam*L
 * (keypoint, camera, level) entries of each (batch item, anchor, group):
 *   w[b][a][p][n][l][g] = exp(x - max) / sum over (p', n', l') of exp(x' - max)
 * (a logit of -inf is a masked entry with weight 0). The forward applies it
 * while staging the weights (they are never written); grad_weights is then
 * the gradient with respect to the logits, w * (dw - sum over the group of
 * w * dw). Forward and backward need a workspace (msda_forward_ws). */
#define MSDA_WEIGHT_LOGITS 2u
/* `weights` (or the logits) are stored as bfloat16: the pointer holds
 * uint16 bit patterns in the same layout; grad_weights stays FP32. */
#define MSDA_WEIGHTS_BF16 4u
/* The visible-view and fused forms take both flags (their workspaces grow
 * accordingly; with logits, the softmax runs over every camera's entries,
 * visible or not, and the logits' gradient reaches invisible entries through
 * its normalisation). The batched form takes both too (msda_batch.flags,
 * the same for every scene): its workspace then also holds the softmax
 * statistics of every anchor and, for the backward, FP32 weights of every
 * sample; each scene's grad_weights is FP32. */

/* msda_tile.scatter: how the backward forms grad_feat */
#define MSDA_SCATTER_AUTO 0   /* the library's choice (currently SORTED)                */
#define MSDA_SCATTER_SORTED 1 /* records sorted by feature row, then one pass per row
                                 summing in sample order: deterministic, no atomics   */
#define MSDA_SCATTER_ATOMIC 2 /* FP32 float atomics into an accumulator: run-to-run
                                 differences in the last bits                        */
#define MSDA_SCATTER_SORTED_GLOBAL 3 /* SORTED, with the records always grouped by one
                                 global radix sort instead of per-region buckets in
                                 LDS: the same grad_feat bit for bit (a reference for
                                 tests and a fallback)                               */

/* msda_tile.order: how the gathers split the work */
#define MSDA_ORDER_AUTO 0   /* the library's choice                                    */
#define MSDA_ORDER_ANCHOR 1 /* one workgroup per (batch item, anchor); its waves split
                               the anchor's (keypoint, camera) pairs                   */
#define MSDA_ORDER_VIEW 2   /* the (batch item, camera) x anchor work is cut, camera-
                               major, into 8 equal ranges, one per XCD, so each XCD's
                               L2 holds the pyramids of a few cameras at a time; each
                               wave takes one anchor over its cameras in a range. The
                               forward then adds 8 partial sums per anchor in a fixed
                               order and needs a workspace (msda_forward_ws)           */

/* Launch shape. A zero field means "choose". */
typedef struct msda_tile {
    int32_t waves_per_anchor; /* anchor order: wavefronts (64 lanes) sharing one
                                 anchor; view order: wavefronts per workgroup, one
                                 anchor each. 1, 2, 4 or 8                            */
    int32_t chans_per_lane;   /* channels each lane owns: 1, 2, 4 (FP32), 2, 4, 8
                                 (BF16, FP16), 4, 8, 16 (FP8)                        */
    int32_t order;            /* MSDA_ORDER_*                                          */
    int32_t scatter;          /* MSDA_SCATTER_* (backward only)                        */
} msda_tile;

/* Sizes and options of one call. */
typedef struct msda_desc {
    int32_t batch;       /* B  >= 1                                              */
    int32_t num_cams;    /* Ncam >= 1                                            */
    int32_t num_levels;  /* L in 1..8                                            */
    int32_t num_anchors; /* A >= 0 (0: arrays sized by A are empty and may be NULL) */
    int32_t num_points;  /* P >= 1 keypoints per anchor                          */
    int32_t channels;    /* C >= 1, C % groups == 0                              */
    int32_t groups;      /* G >= 1                                               */
    int32_t feat_dtype;  /* msda_dtype                                           */
    int64_t rows;        /* R: rows of one batch item of feat                    */
    /* host mirrors of spatial_shapes [Ncam][L][2] and level_start_index
       [Ncam][L], used only to validate regions without reading the device */
    const int32_t* host_spatial_shapes;
    const int32_t* host_level_start_index;
    const float* level_scale; /* device [L] FP32; FP8 only, else NULL        */
    uint32_t flags;           /* MSDA_DETERMINISTIC | MSDA_WEIGHT_LOGITS |
                                 MSDA_WEIGHTS_BF16; other bits are invalid    */
    const msda_tile* tile;    /* NULL = built-in choice                       */
} msda_desc;

/*
 * Forward (paper Sec. 3.1/3.2): out = sum over keypoints, cameras and levels
 * of weight * bilinear sample. All pointers device.
 * Requirements: every region [start, start + H*W) lies in [0, R); H, W >= 1;
 * R*C*sizeof(feat element) <= 4 GiB - 8 KiB (one batch item is addressed
 * with 32-bit byte offsets; larger inputs are split by the caller) and
 * C*sizeof(feat element) <= 4096 (UNSUPPORTED otherwise); feat 16-byte
 * aligned.
 * Returns INVALID_ARGUMENT / UNSUPPORTED as listed above, else OK.
 */
msda_status msda_forward(const void* feat, const int32_t* spatial_shapes,
                         const int32_t* level_start_index, const float* sampling_loc,
                         const float* weights, float* out, const msda_desc* desc,
                         void* stream);

/*
 * msda_forward (the same operator, Sec. 3.1/3.2) with a workspace, which lets
 * the library use view order
 * (MSDA_ORDER_VIEW) for the forward: the library's choice for inputs with at
 * least 8 (batch item, camera) views. Same results contract as
 * msda_forward; the two orders add the samples in different orders, each
 * fixed (deterministic).
 * workspace: device, 256-byte aligned, at least
 * msda_forward_workspace_size(desc) bytes (may be NULL when that is 0).
 * Returns MSDA_ERR_WORKSPACE if it is missing or too small.
 */
msda_status msda_forward_ws(const void* feat, const int32_t* spatial_shapes,
                            const int32_t* level_start_index, const float* sampling_loc,
                            const float* weights, float* out, void* workspace,
                            size_t workspace_bytes, const msda_desc* desc, void* stream);

/* Bytes of device workspace msda_forward_ws needs for desc: 8*B*A*C*4 when
 * the forward runs in view order (chosen or requested), plus B*A*G*8 (the
 * softmax statistics) with MSDA_WEIGHT_LOGITS, each part rounded up to 256. */
size_t msda_forward_workspace_size(const msda_desc* desc);

/*
 * msda_forward_ws without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc. Same operator, arguments, results and
 * errors as msda_forward_ws (bitwise the same output for the same desc); it
 * calls no allocating routine. The workspace lives in a fixed device array
 * of MSDA_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on until the process ends (looked up on the first call on that device).
 * Every call on one GPU shares that array and leaves its contents behind:
 * calls that overlap on one GPU (on two streams, or from two threads without
 * ordering) race and may return wrong results; order them on one stream.
 * Returns MSDA_ERR_UNSUPPORTED, before any HIP call, when
 * msda_forward_workspace_size(desc) exceeds MSDA_NOALLOC_SCRATCH_BYTES (for
 * the view order: B*A*C > 1,048,576 less the statistics' share; the anchor
 * order, msda_tile.order = MSDA_ORDER_ANCHOR, needs none), MSDA_ERR_HIP if
 * the device or the array cannot be looked up.
 */
#define MSDA_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
msda_status msda_forward_noalloc(const void* feat, const int32_t* spatial_shapes,
                                 const int32_t* level_start_index, const float* sampling_loc,
                                 const float* weights, float* out, const msda_desc* desc,
                                 void* stream);

/*
 * Backward: gradients of <grad_out, out> with respect to feat, sampling_loc
 * and weights (the analytic derivative of the forward; at an integer
 * coordinate the right-hand derivative). The paper describes and accelerates
 * the forward only (Sec. 5.3); the model it belongs to is trained end to end
 * with the losses of Sec. 3.3 (Eq. 3), which is why the operator needs a
 * backward at all. Its form here -- the derivative of the sum defined above,
 * with a deterministic grad_feat reduction -- is this library's design, not
 * a procedure from the paper. Any of grad_feat,
 * grad_sampling_loc, grad_weights may be NULL to skip it. grad_feat has the
 * feat dtype; FP8 grad_feat is UNSUPPORTED. Accumulation is FP32; a BF16 or
 * FP16 grad_feat is rounded once (to nearest even) from the FP32 sum.
 * grad_feat is formed as msda_tile.scatter says: by default every (sample,
 * corner) contribution is recorded, the records are sorted by feature row
 * (a stable radix sort) and each row is summed in sample order and written
 * once -- bitwise reproducible; MSDA_SCATTER_ATOMIC instead adds them with
 * FP32 atomics (correct to rounding, last bits vary run to run).
 * workspace: device, 256-byte aligned, at least
 * msda_backward_workspace_size(desc) bytes (may be NULL when that is 0).
 * Limits of the sorted form: B*R < 2^31 and 4*B*A*P*Ncam*L < 2^32.
 */
msda_status msda_backward(const void* feat, const int32_t* spatial_shapes,
                          const int32_t* level_start_index, const float* sampling_loc,
                          const float* weights, const float* grad_out, void* grad_feat,
                          float* grad_sampling_loc, float* grad_weights, void* workspace,
                          size_t workspace_bytes, const msda_desc* desc, void* stream);

/* Bytes of device workspace msda_backward needs for desc (0 if none): about
 * 24 bytes per sample plus 4 per bilinear cell for the sorted form; B*R*C*4
 * for the atomic form with BF16 or FP16 features; with MSDA_WEIGHT_LOGITS or
 * MSDA_WEIGHTS_BF16 also the FP32 weights (4*G per sample) and the softmax
 * statistics (B*A*G*8). */
size_t msda_backward_workspace_size(const msda_desc* desc);

/*
 * Keypoint projection with motion compensation (paper Sec. 3.1, Sec. 3.2):
 * the step that produces MSDA's sampling locations. For each batch item b,
 * anchor a, keypoint p and camera n:
 *   world = (x, y, z) + Rz(yaw) (k_x w, k_y l, k_z h) + dt (vx, vy, vz)
 *   (u', v', d) = M[b][n] (world, 1);  pixel = (u'/d, v'/d) when d > 1e-5
 *   sampling_loc[b][a][p][n] = (pixel_x / W_img[n], pixel_y / H_img[n]),
 *                              (-2, -2) when d <= 1e-5 (skipped by MSDA)
 *   visible[b][a][n] = 1 if some keypoint has d > 1e-5 and a pixel inside
 *                      [0, W_img) x [0, H_img), else 0
 * anchors [B][A][10] (x, y, z, w, l, h, yaw, vx, vy, vz), FP32; keypoints
 * [B][A][P][3] box-frame offsets in units of (w, l, h); projection
 * [B][Ncam][3][4] (intrinsics times world-to-camera extrinsics, pixels);
 * image_hw [Ncam][2] int32 (H, W). All device; outputs overwritten.
 */
typedef struct msda_projection_desc {
    int32_t batch;       /* B >= 1    */
    int32_t num_anchors; /* A >= 0    */
    int32_t num_points;  /* P >= 1    */
    int32_t num_cams;    /* Ncam >= 1 */
    float dt;            /* seconds, the motion-compensation time offset */
} msda_projection_desc;

msda_status msda_project_keypoints(const float* anchors, const float* keypoints,
                                   const float* projection, const int32_t* image_hw,
                                   float* sampling_loc, uint8_t* visible,
                                   const msda_projection_desc* desc, void* stream);

/*
 * Visible-view MSDA: the forward and backward restricted to the (batch item,
 * anchor, camera) pairs with visible[b][a][n] != 0 (the cameras an anchor is
 * seen from; the paper scores visibility per object and camera, Sec. 3.2 /
 * Eq. 1, with a network -- here any flag, e.g. the geometric one of
 * msda_project_keypoints) (uint8 [B][A][Ncam],
 * device; e.g. from msda_project_keypoints). Samples of other pairs are not
 * read or computed: out sums over the visible pairs only, and their
 * grad_sampling_loc and grad_weights are written as zero. The visible items
 * are compacted camera-major on the device and processed in view order, so
 * the work and the traffic scale with the number of visible pairs. The
 * forward adds an anchor's cameras in camera order (deterministic); the
 * backward has the sorted grad_feat form only. Same layouts, dtypes and
 * limits as msda_forward / msda_backward; workspaces (device, 256-byte
 * aligned) of at least the sizes below.
 */
msda_status msda_forward_visible(const void* feat, const int32_t* spatial_shapes,
                                 const int32_t* level_start_index, const float* sampling_loc,
                                 const float* weights, const uint8_t* visible, float* out,
                                 void* workspace, size_t workspace_bytes, const msda_desc* desc,
                                 void* stream);
size_t msda_forward_visible_workspace_size(const msda_desc* desc);
msda_status msda_backward_visible(const void* feat, const int32_t* spatial_shapes,
                                  const int32_t* level_start_index, const float* sampling_loc,
                                  const float* weights, const uint8_t* visible,
                                  const float* grad_out, void* grad_feat,
                                  float* grad_sampling_loc, float* grad_weights, void* workspace,
                                  size_t workspace_bytes, const msda_desc* desc, void* stream);
size_t msda_backward_visible_workspace_size(const msda_desc* desc);

/*
 * Visibility-weighted fusion over the visible views (paper Sec. 3.2, Eq. 2):
 * the anchor's feature in camera n alone, g_n = the visible-view sum over
 * camera n's samples, is weighted by the camera's visibility score,
 *   V[b][a] = sum over visible n of view_score[b][a][n]
 *   out[b][a] = sum over visible n of view_score[b][a][n] / V * g_n
 * (out = 0 when V <= 0). view_score: FP32 [B][A][Ncam], device (scores of
 * invisible cameras are ignored). The backward returns the visible-view
 * gradients with grad_out scaled per camera by view_score / V, and
 *   grad_score[b][a][n] = (<grad_out, g_n> - <grad_out, out>) / V
 * for visible cameras (0 otherwise and when V <= 0); it needs the forward's
 * out [B][A][C] (FP32, device) when grad_score is requested; any of
 * grad_feat, grad_sampling_loc, grad_weights, grad_score may be NULL. Cameras
 * are added in camera order in both passes (deterministic). Layouts, dtypes,
 * limits and errors as msda_forward_visible / msda_backward_visible;
 * workspaces (device, 256-byte aligned) of at least the sizes below.
 */
msda_status msda_forward_fused(const void* feat, const int32_t* spatial_shapes,
                               const int32_t* level_start_index, const float* sampling_loc,
                               const float* weights, const uint8_t* visible,
                               const float* view_score, float* out, void* workspace,
                               size_t workspace_bytes, const msda_desc* desc, void* stream);
size_t msda_forward_fused_workspace_size(const msda_desc* desc);
msda_status msda_backward_fused(const void* feat, const int32_t* spatial_shapes,
                                const int32_t* level_start_index, const float* sampling_loc,
                                const float* weights, const uint8_t* visible,
                                const float* view_score, const float* out,
                                const float* grad_out, void* grad_feat,
                                float* grad_sampling_loc, float* grad_weights,
                                float* grad_score, void* workspace, size_t workspace_bytes,
                                const msda_desc* desc, void* stream);
size_t msda_backward_fused_workspace_size(const msda_desc* desc);

/*
 * Per-level FP8 quantisation of an FP32 feat (the precision form's storage;
 * the paper stores MSDA's features in FP16, Sec. 5.3, and e4m3 with a scale
 * per level is this library's lower-precision option):
 * scale_l = amax_l / 448 over every batch item, camera and channel of level l
 * (1 when the level is all zero), code = round-to-nearest-even(clamp(x /
 * scale_l, -448, 448)) in OCP e4m3fn. Rows in no region are written as 0.
 * feat_f32 [B][R][C] device; codes [B][R][C] uint8 device; level_scale [L]
 * FP32 device (written). workspace: device, 4-byte aligned, >=
 * msda_quantize_workspace_size (4 bytes per (batch item, camera, level):
 * each region's running maximum), contents not kept.
 */
msda_status msda_quantize_fp8(const float* feat_f32, const int32_t* spatial_shapes,
                              const int32_t* level_start_index, uint8_t* codes,
                              float* level_scale, void* workspace, size_t workspace_bytes,
                              const msda_desc* desc, void* stream);
size_t msda_quantize_workspace_size(const msda_desc* desc);

/*
 * Batched form: several scenes of uneven size in one persistent launch per
 * pass (the scenes of a multi-camera deployment processed together). The
 * paper measures how many camera streams one GPU serves (Sec. 5.3, App. B,
 * App. C) but gives no batched kernel; this form is this library's design
 * for that workload. Each
 * scene is one batch item with its own cameras, feature geometry and
 * anchors; levels, keypoints, channels, groups and the feature dtype are
 * shared. The results are those of msda_forward / msda_backward called on
 * each scene with B = 1 (bitwise for the forward with the same launch shape,
 * and for the default sorted grad_feat).
 */
typedef struct msda_scene {
    const void* feat;                 /* [R][C] in the batch's feat dtype               */
    const int32_t* spatial_shapes;    /* [Ncam][L][2] (H, W)                             */
    const int32_t* level_start_index; /* [Ncam][L]                                       */
    const float* sampling_loc;        /* [A][P][Ncam][2]                                 */
    const float* weights;             /* [A][P][Ncam][L][G]                              */
    float* out;                       /* [A][C]  forward output                          */
    const float* grad_out;            /* [A][C]  backward input                          */
    void* grad_feat;                  /* [R][C]  backward output (feat dtype), or NULL   */
    float* grad_sampling_loc;         /* backward output, or NULL                        */
    float* grad_weights;              /* backward output, or NULL                        */
    int64_t rows;                     /* R                                               */
    int32_t num_cams;                 /* Ncam >= 1                                       */
    int32_t num_anchors;              /* A >= 0                                          */
} msda_scene;

typedef struct msda_batch {
    int32_t num_scenes;               /* 1 .. 256                                        */
    int32_t num_levels;               /* L, shared                                       */
    int32_t num_points;               /* P, shared                                       */
    int32_t channels;                 /* C, shared                                       */
    int32_t groups;                   /* G, shared                                       */
    int32_t feat_dtype;               /* msda_dtype, shared                              */
    const msda_scene* scenes;         /* device copy of the scene table                  */
    const msda_scene* host_scenes;    /* host copy of the same table (validation)        */
    const int32_t* const* host_spatial_shapes;     /* per scene, host mirror            */
    const int32_t* const* host_level_start_index;  /* per scene, host mirror            */
    const float* level_scale;         /* device [L], FP8 only                            */
    uint32_t flags;                   /* MSDA_DETERMINISTIC, MSDA_WEIGHT_LOGITS,
                                         MSDA_WEIGHTS_BF16 (all scenes alike)            */
    const msda_tile* tile;            /* NULL = built-in choice                          */
} msda_batch;

/* Workspace bytes of msda_forward_batched (backward == 0) or
 * msda_backward_batched (backward != 0); 0 on invalid input. */
size_t msda_batched_workspace_size(const msda_batch* batch, int32_t backward);

/*
 * Forward of every scene of the batch in one launch per pass. Work order
 * (msda_batch.tile->order): view order by default -- each scene's (camera,
 * anchor) items are split over the 8 XCD slots exactly as a single call with
 * B = 1 splits them, one wave per (slot, anchor) row, then one kernel adds
 * the slots' partial sums in slot order, so every scene's result is bitwise
 * the single call's in view order; MSDA_ORDER_ANCHOR: persistent workgroups
 * stride over all anchors of all scenes (bitwise the single call's in
 * anchor order). workspace: device, 256-byte aligned, >=
 * msda_batched_workspace_size(batch, 0) (it includes the view order's
 * 8 * anchors * C FP32 partial sums in either order). Validation as for
 * msda_forward, per scene; in addition at most 4096 (camera, level)
 * regions over all scenes.
 */
msda_status msda_forward_batched(const msda_batch* batch, void* workspace,
                                 size_t workspace_bytes, void* stream);

/*
 * Backward of every scene: one gather launch for all anchors of all scenes
 * (in the forward's work order), one sort of all scenes' grad_feat records,
 * one tiled reduction over all scenes' pixels (two launches: coarse, fine). A
 * gradient pointer must be NULL in every scene or in none. Only the sorted
 * grad_feat form is available here. workspace: >=
 * msda_batched_workspace_size(batch, 1).
 */
msda_status msda_backward_batched(const msda_batch* batch, void* workspace,
                                  size_t workspace_bytes, void* stream);

/*
 * The grouping step of the backward's deterministic grad_feat reduction on
 * its own (the scatter of the samples' contributions to the features, done
 * by sorting the samples' records by bilinear cell; part of this library's
 * backward, which the paper does not describe -- see msda_backward): a stable sort of n uint32 keys in [0, max_key].
 * keys [n] device, read only; order [n] device, written: order[i] is the
 * index of the i-th smallest key, equal keys in index order; seg
 * [max_key + 1] device, written: seg[r] is the first position of the sorted
 * keys whose key is >= r (n if none). A key above max_key is not detected:
 * only its low bits are used, so its place is unspecified (no access leaves
 * the buffers). workspace: device, 256-byte aligned, >=
 * msda_sort_workspace_size(n, max_key) bytes, contents not kept. n == 0
 * writes seg only. Asynchronous on `stream`.
 */
msda_status msda_sort_keys(const uint32_t* keys, uint32_t n, uint32_t max_key, uint32_t* order,
                           uint32_t* seg, void* workspace, size_t workspace_bytes, void* stream);
size_t msda_sort_workspace_size(uint32_t n, uint32_t max_key);

/*
 * Streaming copy of `bytes` (multiple of 16) from src to dst, both device and
 * 16-byte aligned: the achievable-bandwidth reference kernel used when
 * reporting the fraction of HBM bandwidth the MSDA kernels reach.
 */
msda_status msda_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/*
 * Benchmark instrumentation. `events` is an array of 2 * max_kernels
 * hipEvent_t owned by the caller. While it is set on the calling thread, the
 * i-th kernel the library launches (counting from this call, i <
 * max_kernels) is bracketed by events[2i] and events[2i+1], recorded on its
 * stream, so each kernel's own duration can be read with
 * hipEventElapsedTime. msda_recorded_kernels() returns how many were
 * recorded so far and msda_recorded_kernel_name(i) the name of the i-th.
 * events == NULL turns the hook off. Not for use during graph capture.
 * msda_set_kernel_event_filter(name) restricts the hook to kernels of that
 * instrumentation name (as msda_recorded_kernel_name reports it; other
 * launches record nothing and use no slot), so that one kernel can be timed
 * without an event pair around every other launch; NULL or "" records all.
 * The filter is per calling thread and stays until changed.
 */
msda_status msda_set_kernel_events(void* const* events, int32_t max_kernels);
msda_status msda_set_kernel_event_filter(const char* kernel);
int32_t msda_recorded_kernels(void);
const char* msda_recorded_kernel_name(int32_t i);

const char* msda_last_error(void);
int32_t msda_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MSDA_H */
