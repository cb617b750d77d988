// Internal declarations of the learned surrogate (kernels + host glue).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace seb {
namespace net {

typedef __bf16 bf16;
typedef _Float16 f16;

// Network shape: 24 x 24 patch, three input channels (x-slope, y-slope,
// known), conv 3->16 (4x4, stride 2) -> 11x11, conv 16->32 (3x3, stride 2) ->
// 5x5, fc 800 (+ sin/cos yaw) -> 128 -> 64 -> 4.  Map form: the same network
// evaluated at every cell, convolutions dilated 1, 2 and 4.
constexpr int PATCH = 24, HALF = 12;
constexpr int C0 = 3, C1 = 16, C2 = 32;
constexpr int P1 = 11, P2 = 5;                 // conv output sizes (patch form)
constexpr int K1 = C0 * 16, K1P = 64;          // conv1 im2col width (padded)
constexpr int K2 = C1 * 9, K2P = 160;          // conv2 im2col width (padded)
constexpr int F = C2 * P2 * P2;                // 800
constexpr int H1 = 128, H2 = 64, NOUT = 4;
constexpr float S_Z = 0.05f, S_A = 0.5f;       // output scales (m, rad)

// Offsets of the parameter tensors in the flat float32 parameter vector.
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + C1 * K1;
constexpr int64_t OFF_W2 = OFF_B1 + C1;
constexpr int64_t OFF_B2 = OFF_W2 + C2 * K2;
constexpr int64_t OFF_W3 = OFF_B2 + C2;
constexpr int64_t OFF_WY = OFF_W3 + (int64_t)H1 * F;
constexpr int64_t OFF_B3 = OFF_WY + H1 * 2;
constexpr int64_t OFF_W4 = OFF_B3 + H1;
constexpr int64_t OFF_B4 = OFF_W4 + H2 * H1;
constexpr int64_t OFF_W5 = OFF_B4 + H2;
constexpr int64_t OFF_B5 = OFF_W5 + NOUT * H2;
constexpr int64_t N_PARAMS = OFF_B5 + NOUT;

// bf16 copies of the weights in the layouts the GEMMs read ([out][in], and
// transposed [in][out] for the backward pass).  Column order of conv2's
// im2col is (tap, channel); the parameter vector keeps (channel, tap).
struct PackedWeights {
    bf16* w1;    // [16][64]        (c, i, j) columns, 48..63 zero
    bf16* w2;    // [32][160]       (tap, c) columns, 144..159 zero
    bf16* w3;    // [128][800]
    bf16* w4;    // [64][128]
    bf16* w5;    // [16][64]        rows 4..15 zero
    bf16* w2t;   // [160][32]
    bf16* w3t;   // [800][128]
    bf16* w4t;   // [128][64]
    bf16* w5t;   // [64][32]        columns 4..31 zero
    bf16* w3f;   // [50][4][64][8]  w3 as 32x32x16 MFMA A fragments: K step kk, neuron tile t,
                 //                 lane l -> W3[32t + l % 32][16kk + 8 (l / 32) + e]
    f16* w4h;    // [64][128]       w4 in fp16 (the bf16 values, exactly): inference head
    f16* w5h;    // [16][64]        w5 in fp16, rows 4..15 zero
};

struct GemmArgs {
    const bf16* A;               // [M][K] row-major, lda % 8 == 0
    int64_t lda;
    const bf16* B;               // [N][K] row-major, ldb % 8 == 0
    int64_t ldb;
    int M, N, K;                 // K % 32 == 0
    int kchunk;                  // split-K chunk (multiple of 32); partial z at C + z * split
    int64_t split;               // 0 = no split
    float* C;                    // fp32 output [M][ldc] (or partials)
    int64_t ldc;
    bf16* Cb;                    // optional bf16 output [M][ldcb]
    int64_t ldcb;
    const float* bias;           // optional [N]
    const float* rowv;           // optional yaw term: v += rowv[m][0] colv[n][0] + rowv[m][1] colv[n][1]
    const float* colv;
    int relu;
    const bf16* gate;            // optional: v *= (gate[m][n] > 0)
    int64_t ldg;
};

}  // namespace net
}  // namespace seb

struct seb_net;
namespace seb {
namespace net {
// Read access to a network's device parameters for the inference kernels.
const float* net_theta(const seb_net* n);
PackedWeights net_packed(const seb_net* n);
}  // namespace net
}  // namespace seb
