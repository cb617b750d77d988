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
    int32_t* n_fallback;         // optional device counter of fallen-back states
    // flagged states, per (unit, block of tf x tf cells) and block row: the
    // row's count and its block-local columns (see AssessArgs)
    uint8_t* row_count;          // [U * blocks][tf]
    uint8_t* work_cols;          // [U * blocks][tf][tf]
    int tf, blocks_x, blocks;
    // fallback rule
    float risk_max, band, min_known;
};

// Network part: fills `a`'s outputs for the states it answers and lists the
// others in s.row_count / s.work_cols.  The caller then re-assesses the listed
// states with the plain method (launch_assess_flagged).
hipError_t launch_surrogate(const SurArgs& s, const AssessArgs& a, hipStream_t stream);

}  // namespace sur
}  // namespace seb
