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
// method then re-assesses exactly those, from the per-block row lists the
// network's kernel writes (launch_assess_flagged: flagged_kernel).
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

// Trunk of the map form, one launch with three kinds of workgroups.
//
// Convolution tiles (the first tiles_y2 * tiles_x2 workgroups, rounded up to
// a multiple of 8; see the XCD bands below): conv1 and
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
// Workgroups have eight waves: with one or two workgroups per CU the launch
// is bound by each wave's chain of dependent LDS reads and products, which
// twice the waves per tile halves.
//
// Known-fraction tiles (the remaining workgroups): the fraction of known
// cells in each cell's 24 x 24 window [c - 12, c + 12), for 16 x 16 cells,
// from an LDS tile of known flags (row sums, then column sums).
//
// One more workgroup clears the fallback counter and computes fc1's yaw term
// for every yaw unit.
constexpr int TT = 16;                       // conv2 positions per tile side
constexpr int T1 = TT + 4;                   // conv1 positions per tile side
constexpr int TC = T1 + 4;                   // input cells per side (window 4, slope +1 -> 25 heights)
constexpr int TB = 512, TW = TB / 64;        // threads and waves of a workgroup

__global__ __launch_bounds__(TB) void trunk_kernel(const SurArgs s) {
    __shared__ float hs[TC + 1][TC + 1];     // heights (0 where unknown)
    __shared__ float ks[TC + 1][TC + 1];     // known flags
    __shared__ float cin[3][TC][TC + 1];     // bf16-rounded inputs: x-slope, y-slope, known
    __shared__ bf16x8 o1s[T1 * T1][2];       // conv1 outputs [position][channels 0-7, 8-15]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    const int tx2 = (s.W + 16 + TT - 1) / TT, ty2 = (s.H + 16 + TT - 1) / TT;
    const int nconv = 8 * ((tx2 * ty2 + 7) / 8);   // convolution workgroups, a multiple of 8
    if (blockIdx.x == gridDim.x - 1) {
        // ---- the last workgroup: clears the fallback counter and computes
        // fc1's yaw term Y[u][n] = Wy[n] . (sin, cos)(theta_u), eight fp16
        // neurons per entry (Wy is [n][2]: float4 q of an entry holds neurons
        // 2q and 2q + 1) ----
        if (tid == 0 && s.n_fallback) *s.n_fallback = 0;
        static_assert(net::OFF_WY % 4 == 0, "yaw weights read as float4");
        for (int i = tid; i < s.U * (net::H1 / 8); i += TB) {
            const float2 sc = s.yaw_sc[i >> 4];
            const float4* wp = (const float4*)(s.theta + net::OFF_WY + 16 * (i & 15));
            typedef _Float16 h8 __attribute__((ext_vector_type(8)));
            h8 v;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 w = wp[q];
                v[2 * q] = (_Float16)(sc.x * w.x + sc.y * w.y);
                v[2 * q + 1] = (_Float16)(sc.x * w.z + sc.y * w.w);
            }
            reinterpret_cast<h8*>(s.ymap)[i] = v;
        }
        return;
    }
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
        // three loads per thread in flight, from clamped positions, masked afterwards
        constexpr int NB = (SPAN * SPAN + TB - 1) / TB;
        float hv[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = min(tid + TB * j, SPAN * SPAN - 1);
            const int y = y0 - net::HALF + i / SPAN, x = x0 - net::HALF + i % SPAN;
            hv[j] = s.height[(int64_t)min(max(y, 0), s.H - 1) * s.ld + min(max(x, 0), s.W - 1)];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = tid + TB * j;
            if (i >= SPAN * SPAN) continue;
            const int rr = i / SPAN, cc = i % SPAN;
            const int y = y0 - net::HALF + rr, x = x0 - net::HALF + cc;
            const bool in = y >= 0 && x >= 0 && y < s.H && x < s.W;
            kf[rr][cc] = (in && fabsf(hv[j]) < HEIGHT_LIMIT) ? 1.f : 0.f;
        }
        __syncthreads();
        for (int i = tid; i < SPAN * T; i += TB) {
            const int rr = i / T, cc = i % T;
            float n = 0.f;
            for (int d = 0; d < net::PATCH; ++d) n += kf[rr][cc + d];
            rs[rr][cc] = n;
        }
        __syncthreads();
        const int cc = tid % T, rr = tid / T;
        const int x = x0 + cc, y = y0 + rr;
        if (rr < T && x < s.W && y < s.H) {
            float n = 0.f;
            for (int d = 0; d < net::PATCH; ++d) n += rs[rr + d][cc];
            s.known[(int64_t)y * s.W + x] = n * (1.f / (net::PATCH * net::PATCH));
        }
        return;
    }
    // ---- conv1 + conv2 of a 16 x 16 tile of conv2 positions ----
    // Tiles in XCD bands, as in net_kernel: workgroup i (on XCD i % 8) takes
    // tile (i % 8) * per + i / 8, so each XCD writes one band of the conv2 map.
    const int per = nconv / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= tx2 * ty2) return;
    const int Y2 = (tile / tx2) * TT - 12, X2 = (tile % tx2) * TT - 12;
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
    constexpr int NH = ((TC + 1) * (TC + 1) + TB - 1) / TB;      // 2 cells per thread
    float hv[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int i = min(tid + TB * j, (TC + 1) * (TC + 1) - 1);
        const int y = Y2 + i / (TC + 1), x = X2 + i % (TC + 1);
        hv[j] = s.height[(int64_t)min(max(y, 0), s.H - 1) * s.ld + min(max(x, 0), s.W - 1)];
    }
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int i = tid + TB * j;
        if (i >= (TC + 1) * (TC + 1)) continue;
        const int rr = i / (TC + 1), cc = i % (TC + 1);
        const int y = Y2 + rr, x = X2 + cc;
        const bool ok = y >= 0 && x >= 0 && y < s.H && x < s.W && fabsf(hv[j]) < HEIGHT_LIMIT;
        hs[rr][cc] = ok ? hv[j] : 0.f;
        ks[rr][cc] = ok ? 1.f : 0.f;
    }
    __syncthreads();
    // Input channels of the 24 x 24 cells, rounded to bf16 as in training.
    for (int i = tid; i < TC * TC; i += TB) {
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
    for (int m = wave; m < (T1 * T1) / 16; m += TW) {
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
    // conv2: 16 groups of 16 positions (one tile row each), 2 per wave.  Lane
    // (r, g) supplies position (row, r) at K = 32 ks + 8 g .. + 7: tap
    // 2 ks + g / 2, channels 8 (g % 2) .. + 7.
    const int W2m = s.W + 16, H2m = s.H + 16;
    for (int q = wave; q < TT; q += TW) {
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

// fc1, fc2 and fc3 of every state in one kernel: fc1's output stays in LDS.
// fc1's yaw term comes precomputed per yaw unit (trunk_kernel).
// A workgroup (four waves) owns a tile of 2 x 32 cells.
//
// fc1 without the yaw term, per cell: T[n] = b3[n] + W3[n] . (conv2 at the
// 5 x 5 positions cell - 12 + 4 (a, b)).  Implicit GEMM on the 32x32x16 MFMA
// (measured about 1.5 times the throughput of 16x16x32 on this device),
// D (128 neurons x cells) = W3 (128 x 800) . gather^T.  The tile's gathered
// conv2 vectors come from 10 rows x 48 columns of conv2 positions (rows
// cy + 4 a + {0, 1}, columns cx + 4 b + 0..31), staged in LDS at once (every
// load in flight together: conv2's map was just written, so these reads miss
// in L2).  Wave w computes neurons 32 w .. 32 w + 31 of both cell rows over
// the whole reduction, streaming its rows of W3 from the fragment-ordered copy
// (1 KB contiguous per fragment, A_DEPTH fragments in flight), so no partial
// sums have to be added across waves.  T goes to LDS as fp16,
// [cell row][neuron / 8][column][neuron % 8].
//
// Head of every state (cell, yaw unit): wave w takes cell row w % 2 and half
// of the yaw units, keeping fc2's weights, its biases and its cells' fc1
// values in registers.  Activations are fp16 (the weights are the network's
// bf16 values, held exactly in fp16), so fc1's yaw term and ReLU run as packed
// fp16 adds and maxima, two neurons per instruction, and fc2's ReLU converts
// two neurons per instruction.  Both layers run on the 32x32x16 MFMA
// (measured 1.8 times the throughput of 16x16x32 on this device), transposed,
// neurons x states:
//   fc2: D2 (64 x 32) = W4 (64 x 128) . h1^T + b4,   h1 = ReLU(T + Y[u])
//   fc3: D3 (32 x 32, rows 0..3 used) = W5' (32 x 64) . h2^T,  h2 = ReLU(D2)
// In the 32x32x16 MFMA lane l = (c, h) = (l % 32, l / 32) supplies A's row
// and B's column c at reduction indices 8h .. 8h+7 of each 16-wide K step,
// and receives D's column c, rows 8q + 4h + j (q, j = 0..3).  So lane (c, h)
// holds, for state c, fc2's neurons 32t + 8q + 4h + j; fc3's K step kk takes
// the eight of them with t = kk / 2 and q = 2 (kk % 2) + {0, 1} as its indices
// 8h .. 8h+7, and W5' is gathered in the same order, which leaves the sum
// unchanged and needs no trip through LDS.  fc2's bias enters as the
// accumulator of its first product.  Stores go to 32 consecutive cells of one
// yaw plane.
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

constexpr int NT_Y = 2, NT_X = 32;                    // cells per tile
constexpr int G_ROWS = NT_Y * net::P2;                // 10 staged position rows
constexpr int G_COLS = NT_X + 4 * (net::P2 - 1);      // 48 staged position columns
constexpr int G_ENTRIES = G_ROWS * G_COLS * 4;        // 16-byte entries, 8 channels each
constexpr int T_ENTRIES = NT_Y * (net::H1 / 8) * NT_X;
constexpr int W4_ENTRIES = (net::H2 / 32) * (net::H1 / 16) * 64;
constexpr int W5_ENTRIES = (net::H2 / 16) * 64;
constexpr int HEAD_ENTRIES = T_ENTRIES + W4_ENTRIES + W5_ENTRIES;
constexpr int REGION_A = G_ENTRIES > HEAD_ENTRIES ? G_ENTRIES : HEAD_ENTRIES;
constexpr int KSTEPS = net::F / 16;                   // fc1's 16-wide reduction steps
constexpr int A_DEPTH = 8;
static_assert(net::H1 == 4 * 32 && net::H2 == 2 * 32, "one neuron tile of fc1 per wave, two of fc2");

inline size_t net_lds_bytes(int U) { return (size_t)(REGION_A + U * (net::H1 / 8)) * 16; }

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void net_kernel(const SurArgs s, const AssessArgs a) {
    // LDS (16-byte entries): region A holds the staged conv2 vectors
    // [row][piece of 8 channels][column] during fc1, then T [cell row][neuron
    // chunk][column] and fc2's weights as fp16 MFMA fragments [t][kk][lane];
    // after it, the yaw term [U][16] (eight fp16 neurons each).
    extern __shared__ f16x8 lds[];
    bf16x8* gs = reinterpret_cast<bf16x8*>(lds);
    f16x8* ts = lds;
    f16x8* w4s = lds + T_ENTRIES;
    f16x8* w5s = w4s + W4_ENTRIES;
    f16x8* ys = lds + REGION_A;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int cl = lane & 31, lh = lane >> 5;
    const int W2m = s.W + 16, H2m = s.H + 16;
    const int tx = (s.W + NT_X - 1) / NT_X;
    // Tiles in XCD bands: the hardware hands workgroup i to XCD i % 8, so
    // workgroup i takes tile (i % 8) * per + i / 8, and each XCD works through
    // one contiguous band of tile rows, whose conv2 vectors its L2 then holds
    // (row-major tiles would send every XCD over the whole conv2 map).
    const int nt = ((s.H + NT_Y - 1) / NT_Y) * tx;
    const int per = (nt + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= nt) return;
    const int cy0 = (tile / tx) * NT_Y, cx0 = (tile % tx) * NT_X;

    // Every global load of the workgroup is issued before the first wait:
    // the gathered conv2 vectors, the first A_DEPTH fragments of W3, fc1's
    // biases, fc2's weights, the yaw term and the head's per-cell operands.
    constexpr int NG = (G_ENTRIES + 255) / 256;
    bf16x8 g[NG];
#pragma unroll
    for (int j = 0; j < NG; ++j) {
        const int i = min(tid + 256 * j, G_ENTRIES - 1), piece = i & 3, pos = i >> 2;
        const int rr = pos / G_COLS, cc = pos - rr * G_COLS;
        // staged row rr = 2 a + dy is position row cy0 + 4 a + dy (o2map row)
        const int y = min(cy0 + 4 * (rr >> 1) + (rr & 1), H2m - 1);
        const int x = min(cx0 + cc, W2m - 1);
        g[j] = *(const bf16x8*)(s.o2map + ((int64_t)y * W2m + x) * net::C2 + 8 * piece);
    }
    // fragment (K step st, neuron tile t) of W3 is w3f[(st * 4 + t) * 64 + lane]
    const bf16x8* w3f = reinterpret_cast<const bf16x8*>(s.pw.w3f) + wave * 64 + lane;
    bf16x8 ar[A_DEPTH];
#pragma unroll
    for (int st = 0; st < A_DEPTH; ++st) ar[st] = w3f[st * 256];
    static_assert(net::OFF_B3 % 4 == 0, "fc1 biases are read as float4");
    float4 b3[4];                            // [q]: b3[32 wave + 8q + 4lh + (0..3)]
#pragma unroll
    for (int q = 0; q < 4; ++q) b3[q] = *(const float4*)(s.theta + net::OFF_B3 + 32 * wave + 8 * q + 4 * lh);
    f16x8 wst[4];
    // fc1's yaw term [U][16] (eight fp16 neurons per entry), entries tid and
    // tid + 256 (more than 32 yaw units: see below)
    const int ny = s.U * (net::H1 / 8);
    const f16x8* ymap = reinterpret_cast<const f16x8*>(s.ymap);
    f16x8 yv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) yv[j] = ymap[min(tid + 256 * j, ny - 1)];
    // The head's cell: row cy0 + wave % 2, column cx0 + cl.
    const int hy = cy0 + (wave & 1), hx = cx0 + cl;
    const bool real = hy < s.H && hx < s.W;
    const int cy = min(hy, s.H - 1), cx = min(hx, s.W - 1);
    const int cell = cy * s.W + cx;
    float hc;
    const bool has_ref = ref_height(s, cy, cx, &hc);
    const float kf = s.known[cell];

#pragma unroll
    for (int j = 0; j < NG; ++j) {
        const int i = tid + 256 * j, piece = i & 3, pos = i >> 2;
        const int rr = pos / G_COLS, cc = pos - rr * G_COLS;
        if (i < G_ENTRIES) gs[(rr * 4 + piece) * G_COLS + cc] = g[j];
    }
    __syncthreads();

    f32x16 acc1[2];                          // [cell row m]: neurons 32 wave + 8q + 4lh + j at 4q + j
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc1[m][j] = 0.f;
#pragma unroll
    for (int st = 0; st < KSTEPS; ++st) {
        const bf16x8 av = ar[st % A_DEPTH];
        if (st + A_DEPTH < KSTEPS) ar[st % A_DEPTH] = w3f[(st + A_DEPTH) * 256];
        if (st == KSTEPS - A_DEPTH - 4) {
            // fc2's weights for LDS, issued late in the loop so they do not
            // add to the workgroup's first wave of loads
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int f = tid + 256 * j;                   // fragment (t, kk, lane')
                const int t = f >> 9, kk = (f >> 6) & 7, ln = f & 63;
                wst[j] = *(const f16x8*)(s.pw.w4h + (32 * t + (ln & 31)) * net::H1 + 16 * kk + 8 * (ln >> 5));
            }
        }
        // K step st covers channels 16 h .. 16 h + 15 of gathered position k
        const int k = st >> 1, h = st & 1, a5 = k / net::P2, b5 = k - a5 * net::P2;
#pragma unroll
        for (int m = 0; m < 2; ++m) {         // cell (m, cl): channels 16 h + 8 lh ..
            const bf16x8 bv = gs[((2 * a5 + m) * 4 + 2 * h + lh) * G_COLS + cl + 4 * b5];
            acc1[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc1[m], 0, 0, 0);
        }
    }
    // fc2's biases and fc3's weights and biases, for the head
    // fc2's bias enters as one more product, D2 += B4 . ONES, with K index 0
    // and 1 of lane row c carrying b4's fp16 high and low parts (their sum is
    // b4 to 2^-22) and the other indices zero: b4's 32 per-lane values would
    // otherwise take 32 registers.
    f16x8 w4b[2];                            // [t]: A fragment, row 32t + cl
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const float b = s.theta[net::OFF_B4 + 32 * t + cl];
        const _Float16 hi = (_Float16)b, lo = (_Float16)(b - (float)hi);
        w4b[t] = lh == 0 ? f16x8{hi, lo, 0, 0, 0, 0, 0, 0} : f16x8{};
    }
    const f16x8 ones = lh == 0 ? f16x8{1, 1, 0, 0, 0, 0, 0, 0} : f16x8{};
    // fc3's A fragment (kk, lane') = W5[c'][neuron(kk, h', e)] for lane'
    // (c', h'), rows c' >= 4 zero; this thread's fragment is (tid / 64, tid % 64)
    f16x8 w5f;
    {
        const int kk = tid >> 6, c5 = tid & 31, h5 = (tid >> 5) & 1;
        // neurons 32 (kk / 2) + 8 (2 (kk % 2) + e / 4) + 4 h' + e % 4
        const int nb = 32 * (kk >> 1) + 16 * (kk & 1) + 4 * h5;
        const int row = min(c5, 3);
        const f16x4 lo = *(const f16x4*)(s.pw.w5h + row * net::H2 + nb);
        const f16x4 hi = *(const f16x4*)(s.pw.w5h + row * net::H2 + nb + 8);
        const f16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        w5f = c5 < 4 ? v : f16x8{};
    }
    static_assert(W5_ENTRIES == 256, "one fc3 fragment per thread");
    float b5[4];
    for (int j = 0; j < 4; ++j) b5[j] = s.theta[net::OFF_B5 + j];
    __syncthreads();                          // every wave is done with the staged vectors
    // T: neurons 32 wave + 8q + 4lh + (0..3) of cell (m, cl) are chunk
    // 4 wave + q, half lh
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const f16x4 o = {(_Float16)(acc1[m][4 * q] + b3[q].x), (_Float16)(acc1[m][4 * q + 1] + b3[q].y),
                             (_Float16)(acc1[m][4 * q + 2] + b3[q].z), (_Float16)(acc1[m][4 * q + 3] + b3[q].w)};
            *reinterpret_cast<f16x4*>(reinterpret_cast<_Float16*>(ts + (m * 16 + 4 * wave + q) * NT_X + cl) +
                                      4 * lh) = o;
        }
#pragma unroll
    for (int j = 0; j < 4; ++j) w4s[tid + 256 * j] = wst[j];
    w5s[tid] = w5f;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = tid + 256 * j;
        if (i < ny) ys[i] = yv[j];
    }
    for (int i = tid + 512; i < ny; i += 256) ys[i] = ymap[i];     // more than 32 yaw units
    __syncthreads();
    if (hy >= s.H) return;                    // a tile's second row past the map's edge
    const int mh = wave & 1;
    // T[cell][16kk + 8lh + e] (chunk 2kk + lh) is tc[(2kk + lh) * NT_X]
    const f16x8* tc = ts + mh * 16 * NT_X + cl;
    f16x8 w4[2][8];                          // [t][kk]: W4[32t + cl][16kk + 8lh + e]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) w4[t][kk] = w4s[(t * 8 + kk) * 64 + lane];
    const bool out_of_dist = !has_ref || kf < s.min_known;
    const int uh = (s.U + 1) >> 1;
    const int u0 = wave < 2 ? 0 : uh, u1 = wave < 2 ? uh : s.U;
    // Every load above is complete before the loop: a wait inside it would
    // also wait for the previous unit's stores.
    __builtin_amdgcn_s_waitcnt(0);

    // Fallback lists: the cell's block (tf x tf cells), row and column in it;
    // unit u's lists start at u * blocks * tf * tf.
    const int bcol = hx % s.tf;
    const int blk = (hy / s.tf) * s.blocks_x + hx / s.tf;
    const int crow = blk * s.tf + hy % s.tf;               // row-count index
    const int lrow = crow * s.tf;                           // row list start
    const uint32_t bmask = s.tf == 32 ? 0xffffffffu : (cl < 16 ? 0xffffu : 0xffff0000u);
    const bool first = lh == 0 && real && bcol == 0;
    const f16x8 zero8 = {};
    for (int u = u0; u < u1; ++u) {
        // zero (u < 2^30), but not known to be: it keeps the per-unit LDS
        // reads of T and W5 inside the loop instead of in registers
        const int zo = u & (1 << 30);
        f32x16 acc[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w4b[t], ones, f32x16{}, 0, 0, 0);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const f16x8 h = __builtin_elementwise_max(tc[(2 * kk + lh) * NT_X + zo] + ys[u * 16 + 2 * kk + lh], zero8);
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w4[t][kk], h, acc[t], 0, 0, 0);
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
            y3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(w5s[kk * 64 + lane + zo], h2, y3, 0, 0, 0);
        }
        // Lanes with lh = 0 hold rows 0..3, the four outputs of state (cell, u).
        bool fb = false;
        if (lh == 0 && real) {
            const float o0 = y3[0] + b5[0];
            const float o1 = y3[1] + b5[1];
            const float o2 = y3[2] + b5[2];
            const float o3 = y3[3] + b5[3];
            const float risk = fminf(fmaxf(o3, 0.f), 1.f);
            fb = out_of_dist || fabsf(risk - s.risk_max) < s.band;
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
        // The row segment's flagged states go to its blocks' row lists (one
        // block of 32 columns, or two of 16): a flagged lane writes its column
        // at its rank among the block's flagged lanes, each block's first lane
        // the row's count.
        const uint32_t mine = (uint32_t)__ballot(fb) & bmask;
        const int64_t lists = (int64_t)u * s.blocks * s.tf * s.tf;
        if (fb) s.work_cols[lists + lrow + __popc(mine & ((1u << cl) - 1u))] = (uint8_t)bcol;
        if (first) s.row_count[lists / s.tf + crow] = (uint8_t)__popc(mine);
    }
}

}  // namespace

hipError_t launch_surrogate(const SurArgs& s, const AssessArgs& a, hipStream_t stream) {
    const int conv_tiles = 8 * ((((s.H + 16 + TT - 1) / TT) * ((s.W + 16 + TT - 1) / TT) + 7) / 8);
    const int known_tiles = ((s.H + 15) / 16) * ((s.W + 15) / 16);
    hipLaunchKernelGGL(trunk_kernel, dim3(conv_tiles + known_tiles + 1), dim3(TB), 0, stream, s);
    const int net_tiles = ((s.H + NT_Y - 1) / NT_Y) * ((s.W + NT_X - 1) / NT_X);
    hipLaunchKernelGGL(net_kernel, dim3(8 * ((net_tiles + 7) / 8)), dim3(256),
                       net_lds_bytes(s.U), stream, s, a);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace seb
