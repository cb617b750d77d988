// Internal declarations of surrogate inference (map form) with plain fallback.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "seb_internal.hpp"
#include "seb_net_internal.hpp"

namespace seb {
namespace sur {

struct SurArgs {
    const float* height;         // map [H][ld], NaN = unknown
    int64_t ld;
    int W, H;
    float inv_res;
    int K, U, mirror;            // yaw bins, units evaluated (K/2 if mirrored), mirror offset
    int pitch;                   // LDS pitch of the fallback kernel's table offsets
    // network
    const float* theta;          // float32 parameters (biases and Wy are read from here)
    net::PackedWeights pw;       // bf16 GEMM weights
    // workspace
    const float2* yaw_sc;        // [U]                 (sin, cos) of yaw unit u's angle
    net::bf16* o2map;            // [(H+16)(W+16)][32]  conv2 at positions -12 .. H+3
    net::f16* ymap;              // [U][128]            fc1's yaw term Wy . (sin, cos) per unit
    float* known;                // [H*W]               known fraction of the 24 x 24 window
    uint8_t* need;               // [U][H*W]            1 = state falls back to the plain method
    int32_t* n_fallback;         // optional device counter of fallen-back states
    uint16_t* work_cells;        // fallback workspace (see AssessArgs)
    int32_t* block_count;
    int32_t* item_box;
    // fallback rule
    float risk_max, band, min_known;
};

// Network part: fills `a`'s outputs for the states it answers and s.need for
// the others.  The caller then re-assesses the flagged states with the plain
// method (launch_assess_flagged).
hipError_t launch_surrogate(const SurArgs& s, const AssessArgs& a, hipStream_t stream);

}  // namespace sur
}  // namespace seb
