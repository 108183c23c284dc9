// Internal interface between the C-ABI layer (msda_api.cpp) and the HIP
// kernels (msda_kernels.hip). Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace msda {

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
    float* gfeat_acc;             // FP32 [B][R][C] accumulator for grad_feat, or nullptr
    float* grad_loc;              // or nullptr
    float* grad_w;                // or nullptr
    int32_t B, N, L, A, P, C, G;
    int64_t R;
    uint32_t batch_bytes;         // R * C * sizeof(feat element) (< 2^31)
    int32_t lps_shift;            // log2(lanes per sample) = log2(C / chans_per_lane)
    int32_t pairs_per_chunk;      // (keypoint, camera) pairs staged per wave step
};

enum FeatType { kF32 = 0, kBF16 = 1, kFP8 = 2 };

// Launchers return hipSuccess or the launch error. They enqueue only.
hipError_t launch_forward(const OpArgs& a, int dtype, int cpl, int waves, size_t lds_bytes,
                          hipStream_t s);
hipError_t launch_backward(const OpArgs& a, int dtype, int cpl, int waves, size_t lds_bytes,
                           hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, size_t n, hipStream_t s);
hipError_t launch_quantize_fp8(const float* x, const int32_t* shapes, const int32_t* starts,
                               int32_t B, int32_t N, int32_t L, int64_t R, int32_t C,
                               uint8_t* codes, float* level_scale, uint32_t* amax_ws,
                               hipStream_t s);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Per-sample LDS bytes: geometry table + per-wave staging / reduction area.
size_t lds_bytes_for(const OpArgs& a, int waves);
int max_pairs_per_chunk(int L, int G);

}  // namespace msda
