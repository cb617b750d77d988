// Surrogate inference on a whole map (map form of the network) with the plain
// method as fallback, for gfx950.
//
// The patch network (24 x 24 window, stride-2 convolutions) equals, cell for
// cell, a fully convolutional network with dilations 1, 2 and 4: conv1 and
// conv2 are evaluated once per map position and shared by every cell whose
// window covers that position; fc1 gathers 25 conv2 positions (4 cells apart)
// per cell.  The head (fc1's yaw term, fc2, fc3) runs per state on MFMA.
// Yaw bins k and k + K/2 are mirror images (roll and pitch change sign), as in
// the plain kernel, so the network is evaluated for the first K/2 bins only.
//
// z is predicted relative to a reference height: the own cell's, else the
// mean of its known 8-neighbours.  Flagged states -- no reference, too few
// known cells in the window (out of the training distribution), or predicted
// risk within `band` of risk_max -- are marked in a per-state mask; the plain
// method then re-assesses exactly those, compacted block by block
// (launch_assess_flagged: compact_kernel, then flagged_kernel).
#include <cmath>

#include "seb.h"
#include "seb_internal.hpp"
#include "seb_net_internal.hpp"
#include "seb_state_device.hpp"
#include "seb_surrogate_internal.hpp"

namespace seb {
namespace sur {
namespace {

using namespace dev;
using net::bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16 to_bf16(float f) {
    return (bf16)f;   // round to nearest even (v_cvt_pk_bf16_f32)
}
__device__ __forceinline__ float from_bf16(bf16 h) {
    return __uint_as_float((uint32_t)__builtin_bit_cast(uint16_t, h) << 16);
}

__device__ __forceinline__ float height_at(const SurArgs& s, int y, int x, float* known) {
    if (y < 0 || x < 0 || y >= s.H || x >= s.W) {
        *known = 0.f;
        return 0.f;
    }
    const float h = s.height[(int64_t)y * s.ld + x];
    const bool ok = fabsf(h) < HEIGHT_LIMIT;
    *known = ok ? 1.f : 0.f;
    return ok ? h : 0.f;
}

// Height the z output is relative to: the cell's own height when known, else
// the mean of its known 8-neighbours, summed in row-major order (false when
// none is known).  The nine loads are issued together from clamped positions
// and masked afterwards.
__device__ __forceinline__ bool ref_height(const SurArgs& s, int cy, int cx, float* h) {
    float v[9];
    uint32_t known = 0u;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int y = cy + k / 3 - 1, x = cx + k % 3 - 1;
        known |= (uint32_t)(y >= 0 && x >= 0 && y < s.H && x < s.W) << k;
        v[k] = s.height[(int64_t)min(max(y, 0), s.H - 1) * s.ld + min(max(x, 0), s.W - 1)];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k)
        if (!(fabsf(v[k]) < HEIGHT_LIMIT)) known &= ~(1u << k);
    if (known & (1u << 4)) {
        *h = v[4];
        return true;
    }
    float sum = 0.f, n = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (k == 4 || !((known >> k) & 1u)) continue;
        sum += v[k];
        n += 1.f;
    }
    *h = n > 0.f ? sum / n : 0.f;
    return n > 0.f;
}

// Trunk of the map form, one launch with two kinds of workgroups.
//
// Convolution tiles (the first tiles_y2 * tiles_x2 workgroups): conv1 and
// conv2 for a 16 x 16 tile of conv2 positions (y2, x2) in [-12, H+4) x
// [-12, W+4).  conv2 at (y2, x2) reads conv1 at (y2 + 2i, x2 + 2j), i, j < 3
// (dilation 2), so the tile needs conv1 on 20 x 20 positions, whose 4 x 4
// windows and slopes cover 25 x 25 cells.  Both layers run on MFMA with the
// weights as A and the positions as B, so a lane receives four consecutive
// output channels of one position:
//   conv1: D (16 ch x 16 positions) = W1 (16 x 64) . im2col^T, K = (channel,
//          row, column) of the 4 x 4 window (48 used);
//   conv2: D (32 ch x 16 positions) = W2 (32 x 160) . im2col^T, K = (tap,
//          channel) (144 used).
// Inputs (x-slope, y-slope, known) and conv1's outputs are bf16 as in
// training; conv1's output tile stays in LDS, conv2's goes to o2map.
//
// Known-fraction tiles (the remaining workgroups): the fraction of known
// cells in each cell's 24 x 24 window [c - 12, c + 12), for 16 x 16 cells,
// from an LDS tile of known flags (row sums, then column sums).  The first of
// them also clears the fallback counter.
constexpr int TT = 16;                       // conv2 positions per tile side
constexpr int T1 = TT + 4;                   // conv1 positions per tile side
constexpr int TC = T1 + 4;                   // input cells per side (window 4, slope +1 -> 25 heights)

__global__ __launch_bounds__(256) void trunk_kernel(const SurArgs s) {
    __shared__ float hs[TC + 1][TC + 1];     // heights (0 where unknown)
    __shared__ float ks[TC + 1][TC + 1];     // known flags
    __shared__ float cin[3][TC][TC + 1];     // bf16-rounded inputs: x-slope, y-slope, known
    __shared__ bf16x8 o1s[T1 * T1][2];       // conv1 outputs [position][channels 0-7, 8-15]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    const int tx2 = (s.W + 16 + TT - 1) / TT, ty2 = (s.H + 16 + TT - 1) / TT;
    const int nconv = tx2 * ty2;
    if ((int)blockIdx.x >= nconv) {
        // ---- known fraction of 16 x 16 cells ----
        constexpr int T = 16, SPAN = T + net::PATCH - 1;     // 39 rows / columns of flags
        float (*kf)[SPAN + 1] = reinterpret_cast<float (*)[SPAN + 1]>(&cin[0][0][0]);
        float (*rs)[T + 1] = reinterpret_cast<float (*)[T + 1]>(&o1s[0][0]);
        static_assert(sizeof(cin) >= sizeof(float) * SPAN * (SPAN + 1), "flag tile fits");
        static_assert(sizeof(o1s) >= sizeof(float) * SPAN * (T + 1), "row sums fit");
        const int b = blockIdx.x - nconv;
        const int kx = (s.W + T - 1) / T;
        const int x0 = (b % kx) * T, y0 = (b / kx) * T;
        if (b == 0 && tid == 0 && s.n_fallback) *s.n_fallback = 0;
        // six loads per thread in flight, from clamped positions, masked afterwards
        constexpr int NB = (SPAN * SPAN + 255) / 256;
        float hv[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = min(tid + 256 * j, SPAN * SPAN - 1);
            const int y = y0 - net::HALF + i / SPAN, x = x0 - net::HALF + i % SPAN;
            hv[j] = s.height[(int64_t)min(max(y, 0), s.H - 1) * s.ld + min(max(x, 0), s.W - 1)];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = tid + 256 * j;
            if (i >= SPAN * SPAN) continue;
            const int rr = i / SPAN, cc = i % SPAN;
            const int y = y0 - net::HALF + rr, x = x0 - net::HALF + cc;
            const bool in = y >= 0 && x >= 0 && y < s.H && x < s.W;
            kf[rr][cc] = (in && fabsf(hv[j]) < HEIGHT_LIMIT) ? 1.f : 0.f;
        }
        __syncthreads();
        for (int i = tid; i < SPAN * T; i += 256) {
            const int rr = i / T, cc = i % T;
            float n = 0.f;
            for (int d = 0; d < net::PATCH; ++d) n += kf[rr][cc + d];
            rs[rr][cc] = n;
        }
        __syncthreads();
        const int cc = tid % T, rr = tid / T;
        const int x = x0 + cc, y = y0 + rr;
        if (x < s.W && y < s.H) {
            float n = 0.f;
            for (int d = 0; d < net::PATCH; ++d) n += rs[rr + d][cc];
            s.known[(int64_t)y * s.W + x] = n * (1.f / (net::PATCH * net::PATCH));
        }
        return;
    }
    // ---- conv1 + conv2 of a 16 x 16 tile of conv2 positions ----
    const int Y2 = (blockIdx.x / tx2) * TT - 12, X2 = (blockIdx.x % tx2) * TT - 12;
    // Weights and biases first, with the cell loads, before any wait.
    bf16x8 w1f[2];                           // W1[4g' .. ][..]: A fragments, rows r, K 32ks + 8g
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) w1f[k2] = *(const bf16x8*)(s.pw.w1 + r * net::K1P + 32 * k2 + 8 * g);
    const float4 b1 = *(const float4*)(s.theta + net::OFF_B1 + 4 * g);
    float4 b2[2];
    bf16x8 w2f[2][5];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        b2[t] = *(const float4*)(s.theta + net::OFF_B2 + 16 * t + 4 * g);
#pragma unroll
        for (int k2 = 0; k2 < 5; ++k2)
            w2f[t][k2] = *(const bf16x8*)(s.pw.w2 + (16 * t + r) * net::K2P + 32 * k2 + 8 * g);
    }
    static_assert(net::OFF_B1 % 4 == 0 && net::OFF_B2 % 4 == 0, "biases read as float4");
    constexpr int NH = ((TC + 1) * (TC + 1) + 255) / 256;      // 3 cells per thread
    float hv[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int i = min(tid + 256 * j, (TC + 1) * (TC + 1) - 1);
        const int y = Y2 + i / (TC + 1), x = X2 + i % (TC + 1);
        hv[j] = s.height[(int64_t)min(max(y, 0), s.H - 1) * s.ld + min(max(x, 0), s.W - 1)];
    }
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int i = tid + 256 * j;
        if (i >= (TC + 1) * (TC + 1)) continue;
        const int rr = i / (TC + 1), cc = i % (TC + 1);
        const int y = Y2 + rr, x = X2 + cc;
        const bool ok = y >= 0 && x >= 0 && y < s.H && x < s.W && fabsf(hv[j]) < HEIGHT_LIMIT;
        hs[rr][cc] = ok ? hv[j] : 0.f;
        ks[rr][cc] = ok ? 1.f : 0.f;
    }
    __syncthreads();
    // Input channels of the 24 x 24 cells, rounded to bf16 as in training.
    for (int i = tid; i < TC * TC; i += 256) {
        const int rr = i / TC, cc = i % TC;
        const float v0 = ks[rr][cc], vx = ks[rr][cc + 1], vy = ks[rr + 1][cc];
        const float h0 = hs[rr][cc];
        cin[0][rr][cc] = (float)(bf16)(v0 * vx * (hs[rr][cc + 1] - h0) * s.inv_res);
        cin[1][rr][cc] = (float)(bf16)(v0 * vy * (hs[rr + 1][cc] - h0) * s.inv_res);
        cin[2][rr][cc] = v0;
    }
    __syncthreads();
    // conv1: 25 groups of 16 positions, spread over the waves.  Lane (r, g)
    // supplies position 16 m + r at K = 32 ks + 8 g .. + 7: channel 2 ks + g / 2,
    // window rows 2 (g % 2) and 2 (g % 2) + 1, columns 0..3 (channel 3: zero).
    for (int m = wave; m < (T1 * T1) / 16; m += 4) {
        const int pp = 16 * m + r, py = pp / T1, px = pp % T1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k2 = 0; k2 < 2; ++k2) {
            const int ch = 2 * k2 + (g >> 1), i0 = 2 * (g & 1);
            bf16x8 bop = {};
            if (ch < 3) {
#pragma unroll
                for (int e = 0; e < 8; ++e) bop[e] = (bf16)cin[ch][py + i0 + e / 4][px + e % 4];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f[k2], bop, acc, 0, 0, 0);
        }
        // rows 4g .. 4g+3 = channels of position pp
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        const bf16x4 o = {(bf16)fmaxf(acc[0] + b1.x, 0.f), (bf16)fmaxf(acc[1] + b1.y, 0.f),
                          (bf16)fmaxf(acc[2] + b1.z, 0.f), (bf16)fmaxf(acc[3] + b1.w, 0.f)};
        *reinterpret_cast<bf16x4*>(reinterpret_cast<bf16*>(&o1s[pp][0]) + 4 * g) = o;
    }
    __syncthreads();
    // conv2: 16 groups of 16 positions (one tile row each), 4 per wave.  Lane
    // (r, g) supplies position (row, r) at K = 32 ks + 8 g .. + 7: tap
    // 2 ks + g / 2, channels 8 (g % 2) .. + 7.
    const int W2m = s.W + 16, H2m = s.H + 16;
    for (int q = wave; q < TT; q += 4) {
        const int y2 = Y2 + q, x2 = X2 + r;
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int k2 = 0; k2 < 5; ++k2) {
            const int tap = 2 * k2 + (g >> 1);
            bf16x8 bop = {};
            if (tap < 9) bop = o1s[(q + 2 * (tap / 3)) * T1 + r + 2 * (tap % 3)][g & 1];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2f[t][k2], bop, acc[t], 0, 0, 0);
        }
        if (y2 + 12 < H2m && x2 + 12 < W2m) {
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            bf16* dst = s.o2map + ((int64_t)(y2 + 12) * W2m + (x2 + 12)) * net::C2;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const float4 bb = b2[t];
                const bf16x4 o = {(bf16)fmaxf(acc[t][0] + bb.x, 0.f), (bf16)fmaxf(acc[t][1] + bb.y, 0.f),
                                  (bf16)fmaxf(acc[t][2] + bb.z, 0.f), (bf16)fmaxf(acc[t][3] + bb.w, 0.f)};
                *reinterpret_cast<bf16x4*>(dst + 16 * t + 4 * g) = o;
            }
        }
    }
}

// fc1 without the yaw term, per cell: T[cell][n] = b3[n] + W3[n] . (conv2 at
// the 5 x 5 positions cell - 12 + 4 (a, b)), stored as fp16 for the head in
// chunks of eight neurons, [n / 8][cell][n % 8], so that both this kernel's
// stores and the head's loads are contiguous across lanes.
// Implicit GEMM on the 32x32x16 MFMA (measured about 1.5 times the throughput
// of 16x16x32 on this device), D (128 neurons x cells) = W3 (128 x 800) .
// gather^T.  A workgroup owns a tile of 2 x 32 cells.  Their gathered conv2
// vectors come from 10 rows x 48 columns of conv2 positions (rows
// cy + 4 a + {0, 1}, columns cx + 4 b + 0..31), staged in LDS at once (every
// load in flight together: conv2's map was just written, so these reads miss
// in L2).  The two waves split K: wave 0 takes gathered positions 0..12, wave
// 1 positions 13..24, each for both cell rows and all 128 neurons (8
// accumulator tiles), streaming its half of W3 from the fragment-ordered copy
// (1 KB contiguous per fragment) with the next step's fragments in flight;
// wave 1's partial sums are added through LDS at the end.  In the 32x32x16
// MFMA lane l supplies A's row and B's column l % 32 at K 8 (l / 32) .. + 7 and
// receives D's column l % 32, rows 8 q + 4 (l / 32) + (0..3), q = 0..3.
constexpr int F1_TY = 2, F1_TX = 32;                  // cells per tile
constexpr int F1_ROWS = F1_TY * net::P2;              // 10 staged position rows
constexpr int F1_COLS = F1_TX + 4 * (net::P2 - 1);    // 48 staged position columns
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) void fc1_kernel(const SurArgs s) {
    // staged conv2 vectors [row][piece of 8 channels][column] (consecutive
    // lanes read consecutive 16-byte entries); the first 32 KB are reused for
    // wave 1's partial sums [tile][quarter][lane]
    constexpr int NFP = F1_ROWS * F1_COLS * 4, NPART = 8 * 16 * 64 / 4;   // 16-byte entries
    __shared__ bf16x8 fp[NFP > NPART ? NFP : NPART];
    f32x4* part = reinterpret_cast<f32x4*>(fp);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lc = lane & 31, lh = lane >> 5;
    const int W2m = s.W + 16, H2m = s.H + 16, cells = s.H * s.W;
    const int tx = (s.W + F1_TX - 1) / F1_TX;
    const int cy0 = (blockIdx.x / tx) * F1_TY, cx0 = (blockIdx.x % tx) * F1_TX;
    constexpr int KS = net::P2 * net::P2;     // 25 gathered positions
    constexpr int KH = (KS + 1) / 2;
    const int k0 = wave == 0 ? 0 : KH, k1 = wave == 0 ? KH : KS;
    const bf16x8* w3f = reinterpret_cast<const bf16x8*>(s.pw.w3f) + lane;
    // Staging: 10 x 48 positions x 4 pieces, 15 per thread, all in flight.
    constexpr int NP = NFP / 128;
    static_assert(NFP % 128 == 0, "whole staging passes");
    bf16x8 v[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int i = tid + 128 * j, piece = i & 3, pos = i >> 2;
        const int rr = pos / F1_COLS, cc = pos - rr * F1_COLS;
        // staged row rr = 2 a + dy is position row cy0 + 4 a + dy (o2map row)
        const int y = min(cy0 + 4 * (rr >> 1) + (rr & 1), H2m - 1);
        const int x = min(cx0 + cc, W2m - 1);
        v[j] = *(const bf16x8*)(s.o2map + ((int64_t)y * W2m + x) * net::C2 + 8 * piece);
    }
    // A fragments of gathered position k: K16 steps 2k, 2k + 1, tiles 0..3
    auto load_a = [&](int k, bf16x8 (&av)[2][4]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int t = 0; t < 4; ++t) av[h][t] = w3f[((2 * k + h) * 4 + t) * 64];
    };
    bf16x8 a_cur[2][4], a_nxt[2][4];
    load_a(k0, a_cur);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int i = tid + 128 * j, piece = i & 3, pos = i >> 2;
        const int rr = pos / F1_COLS, cc = pos - rr * F1_COLS;
        fp[(rr * 4 + piece) * F1_COLS + cc] = v[j];
    }
    __syncthreads();
    f32x16 acc[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[m][t][j] = 0.f;
    auto step = [&](int k, const bf16x8 (&av)[2][4]) {
        const int a5 = k / net::P2, b5 = k - a5 * net::P2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 bv[2];
#pragma unroll
            for (int m = 0; m < 2; ++m)       // cell (dy, dx) = (m, lc): channels 16 h + 8 lh ..
                bv[m] = fp[((2 * a5 + m) * 4 + 2 * h + lh) * F1_COLS + lc + 4 * b5];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[h][t], bv[m], acc[m][t], 0, 0, 0);
        }
    };
    // Two steps per iteration over two fragment buffers (no register copies).
    int k = k0;
    for (; k + 1 < k1; k += 2) {
        load_a(k + 1, a_nxt);
        step(k, a_cur);
        if (k + 2 < k1) load_a(k + 2, a_cur);
        step(k + 1, a_nxt);
    }
    if (k < k1) step(k, a_cur);
    __syncthreads();                          // every wave is done with the staged vectors
    if (wave == 1) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    part[((m * 4 + t) * 4 + q) * 64 + lane] =
                        f32x4{acc[m][t][4 * q], acc[m][t][4 * q + 1], acc[m][t][4 * q + 2],
                              acc[m][t][4 * q + 3]};
    }
    __syncthreads();
    if (wave == 1) return;
    static_assert(net::OFF_B3 % 4 == 0, "fc1 biases are read as float4");
    typedef _Float16 f16x4v __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // neurons 32 t + 8 q + 4 lh + (0..3)
            const int n = 32 * t + 8 * q + 4 * lh;
            const float4 bb = *(const float4*)(s.theta + net::OFF_B3 + n);
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int cy = cy0 + m, cx = cx0 + lc;
                const f32x4 pv = part[((m * 4 + t) * 4 + q) * 64 + lane];
                const f16x4v o = {(_Float16)(acc[m][t][4 * q] + pv[0] + bb.x),
                                  (_Float16)(acc[m][t][4 * q + 1] + pv[1] + bb.y),
                                  (_Float16)(acc[m][t][4 * q + 2] + pv[2] + bb.z),
                                  (_Float16)(acc[m][t][4 * q + 3] + pv[3] + bb.w)};
                // T is [neuron chunk of 8][cell][8]: chunk 4 t + q, half lh
                if (cy < s.H && cx < s.W)
                    *reinterpret_cast<f16x4v*>(s.T + ((int64_t)(4 * t + q) * cells + cy * s.W + cx) * 8 +
                                               4 * lh) = o;
            }
        }
}

// Head of every state (cell, yaw unit): a wave owns 32 cells and loops over
// a range of yaw units, keeping fc2's weights, its biases and the cells' fc1
// values (without the yaw term) in registers.  Activations are fp16 (the
// weights are the network's bf16 values, held exactly in fp16), so fc1's yaw
// term and ReLU run as packed fp16 adds and maxima, two neurons per
// instruction, and fc2's ReLU converts two neurons per instruction.  Both
// layers run on the 32x32x16 MFMA (measured 1.8 times the throughput of
// 16x16x32 on this device), transposed, neurons x states:
//   fc2: D2 (64 x 32) = W4 (64 x 128) . h1^T + b4,   h1 = ReLU(T + Y[u])
//   fc3: D3 (32 x 32, rows 0..3 used) = W5' (32 x 64) . h2^T,  h2 = ReLU(D2)
// Lane l = (c, h) = (l % 32, l / 32) supplies A's row and B's column c at
// reduction indices 8h .. 8h+7 of each 16-wide K step, and receives D's
// column c, rows 8q + 4h + j (q, j = 0..3).  So lane (c, h) holds, for
// state c, fc2's neurons 32t + 8q + 4h + j; fc3's K step kk takes the eight
// of them with t = kk / 2 and q = 2 (kk % 2) + {0, 1} as its indices 8h .. 8h+7,
// and W5' is gathered in the same order, which leaves the sum unchanged and
// needs no trip through LDS.  fc2's bias enters as the accumulator of its
// first product.  Stores go to 32 consecutive cells of one yaw plane.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f16x2 pack_rtz(float x, float y) {
    return __builtin_bit_cast(f16x2, __builtin_amdgcn_cvt_pkrtz(x, y));
}

__device__ __forceinline__ f16x8 cat(f16x2 a, f16x2 b, f16x2 c, f16x2 d) {
    const f16x4 lo = __builtin_shufflevector(a, b, 0, 1, 2, 3);
    const f16x4 hi = __builtin_shufflevector(c, d, 0, 1, 2, 3);
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

constexpr int HEAD_CELLS = 32;               // cells per wave

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void head_kernel(const SurArgs s, const AssessArgs a) {
    // LDS: fc2's weights as fp16 MFMA fragments ([t][kk][lane]), shared by
    // the four waves, then the yaw term [U][16] (eight fp16 neurons each).
    extern __shared__ f16x8 lds[];
    f16x8* w4s = lds;
    f16x8* ys = lds + 16 * 64;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int cl = lane & 31, lh = lane >> 5;
    const int cells = s.H * s.W;
    const int c0 = (blockIdx.x * 4 + wave) * HEAD_CELLS;
    const int u0 = blockIdx.y * s.upw, u1 = min(s.U, u0 + s.upw);
    const bool real = c0 + cl < cells;
    const int cell = real ? c0 + cl : cells - 1;
    // Every global load of the workgroup is issued here, before the first
    // wait: fc2's weights and the yaw term for LDS, then the wave's own
    // operands (its cells' fc1 values, fc2's biases, fc3's weights and
    // biases, the nine heights of each cell's reference and its known
    // fraction).
    f16x8 wst[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int f = tid + 256 * j;                   // fragment (t, kk, lane')
        const int t = f >> 9, kk = (f >> 6) & 7, ln = f & 63;
        wst[j] = *(const f16x8*)(s.pw.w4h + (32 * t + (ln & 31)) * net::H1 + 16 * kk +
                                 8 * (ln >> 5));
    }
    // fc1's yaw term Y[u][n] = Wy[n] . (sin, cos)(theta_u), eight neurons per
    // entry, entries tid and tid + 256 (more than 32 yaw units: see below).
    const int ny = s.U * (net::H1 / 8);
    float2 ysc[2];
    float4 wy[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = min(tid + 256 * j, ny - 1);
        ysc[j] = s.yaw_sc[i >> 4];
        const float4* wp = (const float4*)(s.theta + net::OFF_WY + 16 * (i & 15));
#pragma unroll
        for (int q = 0; q < 4; ++q) wy[j][q] = wp[q];
    }
    static_assert(net::OFF_WY % 4 == 0, "yaw weights read as float4");
    f16x8 tv[8];                             // [kk]: T[cell][16kk + 8lh + e] (chunk 2kk + lh)
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
        tv[kk] = *(const f16x8*)(s.T + ((int64_t)(2 * kk + lh) * cells + cell) * 8);
    f32x16 b4v[2];                           // [t]: b4[32t + 8q + 4lh + j] at 4q + j
    static_assert(net::OFF_B4 % 4 == 0, "fc2 biases are read as float4");
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 b = *(const float4*)(s.theta + net::OFF_B4 + 32 * t + 8 * q + 4 * lh);
            b4v[t][4 * q] = b.x;
            b4v[t][4 * q + 1] = b.y;
            b4v[t][4 * q + 2] = b.z;
            b4v[t][4 * q + 3] = b.w;
        }
    f16x8 w5[4];                             // [kk]: W5[cl][neuron(kk, lh, e)], rows >= 4 zero
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        // neurons 32 (kk / 2) + 8 (2 (kk % 2) + e / 4) + 4 lh + e % 4
        const int nb = 32 * (kk >> 1) + 16 * (kk & 1) + 4 * lh;
        const int row = min(cl, 3);
        const f16x4 lo = *(const f16x4*)(s.pw.w5h + row * net::H2 + nb);
        const f16x4 hi = *(const f16x4*)(s.pw.w5h + row * net::H2 + nb + 8);
        const f16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        w5[kk] = cl < 4 ? v : f16x8{};
    }
    float b5[4];
    for (int j = 0; j < 4; ++j) b5[j] = s.theta[net::OFF_B5 + j];
    // Per-cell part of the fallback rule and the plane height offset.
    const int cy = cell / s.W, cx = cell - cy * s.W;
    float hc;
    const bool has_ref = ref_height(s, cy, cx, &hc);
    const bool out_of_dist = !has_ref || s.known[cell] < s.min_known;
#pragma unroll
    for (int j = 0; j < 4; ++j) w4s[tid + 256 * j] = wst[j];
    // (Wy is [n][2]: float4 q holds neurons 2q and 2q + 1 of the entry.)
    auto yaw_entry = [](float2 sc, const float4 (&w)[4]) {
        f16x8 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[2 * q] = (_Float16)(sc.x * w[q].x + sc.y * w[q].y);
            v[2 * q + 1] = (_Float16)(sc.x * w[q].z + sc.y * w[q].w);
        }
        return v;
    };
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = tid + 256 * j;
        if (i < ny) ys[i] = yaw_entry(ysc[j], wy[j]);
    }
    for (int i = tid + 512; i < ny; i += 256) {          // more than 32 yaw units
        const float4* wp = (const float4*)(s.theta + net::OFF_WY + 16 * (i & 15));
        const float4 w[4] = {wp[0], wp[1], wp[2], wp[3]};
        ys[i] = yaw_entry(s.yaw_sc[i >> 4], w);
    }
    __syncthreads();
    if (c0 >= cells) return;
    f16x8 w4[2][8];                          // [t][kk]: W4[32t + cl][16kk + 8lh + e]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) w4[t][kk] = w4s[(t * 8 + kk) * 64 + lane];
    // Every load above is complete before the loop: a wait inside it would
    // also wait for the previous unit's stores.
    __builtin_amdgcn_s_waitcnt(0);

    const f16x8 zero8 = {};
    const int64_t plane = (int64_t)cells;
    for (int u = u0; u < u1; ++u) {
        f32x16 acc[2];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const f16x8 h = __builtin_elementwise_max(tv[kk] + ys[u * 16 + 2 * kk + lh], zero8);
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w4[t][kk], h,
                                                                 kk == 0 ? b4v[t] : acc[t], 0, 0, 0);
        }
        f32x16 y3 = {};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const f32x16& p = acc[kk >> 1];
            const int q0 = 4 * 2 * (kk & 1);             // first of the two q's, times 4
            const f16x8 h2 = __builtin_elementwise_max(
                cat(pack_rtz(p[q0], p[q0 + 1]), pack_rtz(p[q0 + 2], p[q0 + 3]),
                    pack_rtz(p[q0 + 4], p[q0 + 5]), pack_rtz(p[q0 + 6], p[q0 + 7])),
                zero8);
            y3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(w5[kk], h2, y3, 0, 0, 0);
        }
        // Lanes with lh = 0 hold rows 0..3, the four outputs of state (cell, u).
        if (lh == 0 && real) {
            const float o0 = y3[0] + b5[0];
            const float o1 = y3[1] + b5[1];
            const float o2 = y3[2] + b5[2];
            const float o3 = y3[3] + b5[3];
            const float risk = fminf(fmaxf(o3, 0.f), 1.f);
            const bool fb = out_of_dist || fabsf(risk - s.risk_max) < s.band;
            s.need[u * plane + cell] = fb ? 1 : 0;
            if (!fb) {
                Result res;
                res.z = hc + net::S_Z * o0;
                res.roll = net::S_A * o1;
                res.pitch = net::S_A * o2;
                res.risk = risk;
                res.st = SEB_ST_VALID | SEB_ST_SURROGATE | (risk <= s.risk_max ? SEB_ST_TRAV : 0);
                store(a, u, cell, res, false);
                if (a.mirror) store(a, u + a.mirror, cell, res, true);
            }
        }
    }
}

}  // namespace

hipError_t launch_surrogate(const SurArgs& s, const AssessArgs& a, hipStream_t stream) {
    const int64_t cells = (int64_t)s.H * s.W;
    auto blocks = [](int64_t n, int b) { return (unsigned)((n + b - 1) / b); };
    const int conv_tiles = ((s.H + 16 + TT - 1) / TT) * ((s.W + 16 + TT - 1) / TT);
    const int known_tiles = ((s.H + 15) / 16) * ((s.W + 15) / 16);
    hipLaunchKernelGGL(trunk_kernel, dim3(conv_tiles + known_tiles), dim3(256), 0, stream, s);
    hipLaunchKernelGGL(fc1_kernel, dim3(((s.H + F1_TY - 1) / F1_TY) * ((s.W + F1_TX - 1) / F1_TX)),
                       dim3(128), 0, stream, s);
    hipLaunchKernelGGL(head_kernel, dim3(blocks(cells, 4 * HEAD_CELLS), (s.U + s.upw - 1) / s.upw),
                       dim3(256),
                       (size_t)(net::H2 * net::H1 + s.U * net::H1) * sizeof(net::f16), stream, s, a);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace seb
