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

// conv1 at every position (y1, x1) in [-12, H+8) x [-12, W+8): ReLU(b1 + W1 . input
// window [y1, y1+4) x [x1, x1+4)); inputs and outputs rounded to bf16 as in training.
__global__ __launch_bounds__(256) void conv1_map_kernel(const SurArgs s) {
    __shared__ float4 w[net::K1][net::C1 / 4];      // [input][output], transposed
    const int W1 = s.W + 20;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = p < (int64_t)(s.H + 20) * W1;
    const int64_t pc = live ? p : 0;
    const int y1 = (int)(pc / W1) - 12, x1 = (int)(pc % W1) - 12;
    // Every load of the thread is issued before the first wait: the 5 x 5
    // heights the window's slopes use (clamped positions, masked afterwards:
    // unknown and out-of-map cells read as 0 with weight 0), its three
    // weights for the LDS table and the biases.
    float hv[25], kv[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int y = y1 + k / 5, x = x1 + k % 5;
        hv[k] = s.height[(int64_t)min(max(y, 0), s.H - 1) * s.ld + min(max(x, 0), s.W - 1)];
        kv[k] = (y >= 0 && x >= 0 && y < s.H && x < s.W) ? 1.f : 0.f;
    }
    constexpr int NW1 = net::C1 * net::K1 / 256;
    static_assert(net::C1 * net::K1 % 256 == 0, "conv1 weight staging assumes whole passes");
    bf16 wv[NW1];
#pragma unroll
    for (int j = 0; j < NW1; ++j) {
        const int i = threadIdx.x + 256 * j;
        wv[j] = s.pw.w1[(i / net::K1) * net::K1P + i % net::K1];
    }
    float b1[net::C1];
#pragma unroll
    for (int o = 0; o < net::C1; ++o) b1[o] = s.theta[net::OFF_B1 + o];
#pragma unroll
    for (int j = 0; j < NW1; ++j) {
        const int i = threadIdx.x + 256 * j;
        reinterpret_cast<float*>(&w[i % net::K1][0])[i / net::K1] = from_bf16(wv[j]);
    }
    __syncthreads();
    if (!live) return;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const bool ok = kv[k] > 0.f && fabsf(hv[k]) < HEIGHT_LIMIT;
        kv[k] = ok ? 1.f : 0.f;
        hv[k] = ok ? hv[k] : 0.f;
    }
    float in[net::K1];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = i * 5 + j;
            const float v0 = kv[k], vx = kv[k + 1], vy = kv[k + 5];
            const float h0 = hv[k], hx = hv[k + 1], hy = hv[k + 5];
            in[0 * 16 + i * 4 + j] = from_bf16(to_bf16(v0 * vx * (hx - h0) * s.inv_res));
            in[1 * 16 + i * 4 + j] = from_bf16(to_bf16(v0 * vy * (hy - h0) * s.inv_res));
            in[2 * 16 + i * 4 + j] = v0;
        }
    // The 16 outputs accumulate side by side (16 independent chains), each
    // input's 16 weights arriving in four vector LDS reads; every output still
    // sums its 48 products in input order.
    float acc[net::C1];
#pragma unroll
    for (int o = 0; o < net::C1; ++o) acc[o] = 0.f;
#pragma unroll
    for (int c = 0; c < net::K1; ++c) {
#pragma unroll
        for (int q = 0; q < net::C1 / 4; ++q) {
            const float4 wq = w[c][q];
            acc[4 * q + 0] = fmaf(wq.x, in[c], acc[4 * q + 0]);
            acc[4 * q + 1] = fmaf(wq.y, in[c], acc[4 * q + 1]);
            acc[4 * q + 2] = fmaf(wq.z, in[c], acc[4 * q + 2]);
            acc[4 * q + 3] = fmaf(wq.w, in[c], acc[4 * q + 3]);
        }
    }
    bf16* out = s.o1map + p * net::C1;
#pragma unroll
    for (int o = 0; o < net::C1; ++o) out[o] = to_bf16(fmaxf(acc[o] + b1[o], 0.f));
}

// conv2 at every position (y2, x2) in [-12, H+4) x [-12, W+4), dilation 2 on
// conv1's map: implicit GEMM, M = positions, N = 32, K = 9 taps x 16 channels.
__global__ __launch_bounds__(256) void conv2_map_kernel(const SurArgs s) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int W1 = s.W + 20, W2 = s.W + 16;
    const int64_t M = (int64_t)(s.H + 16) * W2;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (row0 >= M) return;
    const int r = lane & 15, kq = lane >> 4;
    const int64_t pr = min(row0 + r, M - 1);
    const int y2 = (int)(pr / W2) - 12, x2 = (int)(pr % W2) - 12;
    // Biases first: a load issued after the stores below would wait for them.
    const float bias[2] = {s.theta[net::OFF_B2 + r], s.theta[net::OFF_B2 + 16 + r]};
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    const bf16x8 zero8 = {};
    for (int ks = 0; ks < net::K2P / 32; ++ks) {
        const int k = 32 * ks + 8 * kq;
        const int tap = k / 16, coff = k % 16;
        bf16x8 a = zero8;
        if (tap < 9) {
            const int y1 = y2 + 2 * (tap / 3), x1 = x2 + 2 * (tap % 3);
            a = *(const bf16x8*)(s.o1map + ((int64_t)(y1 + 12) * W1 + (x1 + 12)) * net::C1 + coff);
        }
        for (int t = 0; t < 2; ++t) {
            const bf16x8 b = *(const bf16x8*)(s.pw.w2 + (16 * t + r) * net::K2P + k);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
    for (int t = 0; t < 2; ++t)
        for (int e = 0; e < 4; ++e) {
            const int64_t row = row0 + 4 * kq + e;
            const int n = 16 * t + r;
            if (row >= M) continue;
            const float v = fmaxf(acc[t][e] + bias[t], 0.f);
            s.o2map[row * net::C2 + n] = to_bf16(v);
        }
}

// fc1 without the yaw term, per cell: T[cell][n] = b3[n] + W3[n] . (conv2 at
// the 5 x 5 positions cell - 12 + 4 (a, b)).  Implicit GEMM: a workgroup owns
// FC1_CELLS cells.  For each row a of the 5 x 5 gather it stages the cells'
// five conv2 vectors (FC1_CELLS x 5 x 32 bf16) in LDS once, so the four waves
// share them instead of each fetching them from L2; wave w then multiplies
// them with W3's rows [32 w, 32 w + 32).  Each output still accumulates its 25
// k-steps in order.
constexpr int FC1_CELLS = 128;
constexpr int FC1_STRIDE = net::P2 * net::C2 + 8;     // bf16 per cell in LDS (16 B pad)
constexpr int FC1_ITEMS = FC1_CELLS * net::P2 * 4;    // 16-byte pieces staged per gather row
static_assert(FC1_ITEMS % 256 == 0, "fc1 staging assumes whole passes");

__global__ __launch_bounds__(256) void fc1_map_kernel(const SurArgs s) {
    __shared__ bf16x8 As[FC1_CELLS * FC1_STRIDE / 8];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int W2 = s.W + 16;
    const int64_t cells = (int64_t)s.H * s.W;
    const int64_t c0 = (int64_t)blockIdx.x * FC1_CELLS;
    const int r = lane & 15, kq = lane >> 4;
    // Biases first: a load issued after the stores below would wait for them.
    const float bias[2] = {s.theta[net::OFF_B3 + 32 * wave + r],
                           s.theta[net::OFF_B3 + 32 * wave + 16 + r]};
    // Staging pieces of this thread: piece = tid + 256 j -> (cell, b, quarter).
    constexpr int NJ = FC1_ITEMS / 256;
    int64_t src[NJ];
    int dst[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int piece = tid + 256 * j;
        const int cell = piece / (net::P2 * 4), rem = piece % (net::P2 * 4);
        const int b5 = rem / 4, q = rem % 4;
        const int64_t c = min(c0 + cell, cells - 1);
        const int cy = (int)(c / s.W), cx = (int)(c % s.W);
        // conv2 position (cy - 12 + 4 a, cx - 12 + 4 b) sits at row cy + 4 a, column cx + 4 b
        src[j] = ((int64_t)cy * W2 + (cx + 4 * b5)) * net::C2 + 8 * q;
        dst[j] = (cell * FC1_STRIDE + b5 * net::C2 + 8 * q) / 8;
    }
    f32x4 acc[FC1_CELLS / 16][2];
#pragma unroll
    for (int i = 0; i < FC1_CELLS / 16; ++i)
        for (int t = 0; t < 2; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int a5 = 0; a5 < net::P2; ++a5) {
        bf16x8 v[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            v[j] = *(const bf16x8*)(s.o2map + src[j] + (int64_t)a5 * 4 * W2 * net::C2);
        bf16x8 bfr[net::P2][2];
#pragma unroll
        for (int b5 = 0; b5 < net::P2; ++b5)
            for (int t = 0; t < 2; ++t)
                bfr[b5][t] = *(const bf16x8*)(s.pw.w3 + (int64_t)(32 * wave + 16 * t + r) * net::F +
                                              32 * (a5 * net::P2 + b5) + 8 * kq);
        if (a5 > 0) __syncthreads();        // the previous row's products are done with As
#pragma unroll
        for (int j = 0; j < NJ; ++j) As[dst[j]] = v[j];
        __syncthreads();
#pragma unroll
        for (int b5 = 0; b5 < net::P2; ++b5)
#pragma unroll
            for (int i = 0; i < FC1_CELLS / 16; ++i) {
                const bf16x8 a = As[((16 * i + r) * FC1_STRIDE + b5 * net::C2 + 8 * kq) / 8];
                for (int t = 0; t < 2; ++t)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[b5][t], acc[i][t], 0, 0, 0);
            }
    }
#pragma unroll
    for (int i = 0; i < FC1_CELLS / 16; ++i)
        for (int t = 0; t < 2; ++t)
            for (int e = 0; e < 4; ++e) {
                const int64_t c = c0 + 16 * i + 4 * kq + e;
                const int n = 32 * wave + 16 * t + r;
                if (c < cells) s.T[c * net::H1 + n] = acc[i][t][e] + bias[t];
            }
}

// Per-map preparation in one launch.  Workgroup (bx, by) computes, for its
// 16 x 16 cells, the known fraction of each cell's 24 x 24 window
// [c - 12, c + 12) from an LDS tile of known flags (row sums, then column
// sums).  Workgroup (0, 0) also writes fc1's yaw term for the first U yaw
// bins, Y[u][n] = Wy[n] . (sin, cos)(2 pi u / K), and clears the fallback
// counters.
__global__ __launch_bounds__(256) void prep_kernel(const SurArgs s) {
    constexpr int T = 16, SPAN = T + net::PATCH - 1;     // 39 rows / columns of flags
    __shared__ float kf[SPAN][SPAN + 1];
    __shared__ float rs[SPAN][T + 1];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * T, y0 = blockIdx.y * T;
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        if (tid == 0 && s.n_fallback) *s.n_fallback = 0;
        for (int i = tid; i < s.U * net::H1; i += 256) {
            const int u = i / net::H1, n = i % net::H1;
            const double th = 2.0 * 3.14159265358979323846 * (double)u / (double)s.K;
            const float sn = (float)sin(th), cs = (float)cos(th);
            s.Y[i] = sn * s.theta[net::OFF_WY + 2 * n] + cs * s.theta[net::OFF_WY + 2 * n + 1];
        }
    }
    {
        // Known flags of the (16 + 23)^2 span: six loads per thread in flight,
        // from clamped positions, masked afterwards.
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
            const int r = i / SPAN, c = i % SPAN;
            const int y = y0 - net::HALF + r, x = x0 - net::HALF + c;
            const bool in = y >= 0 && x >= 0 && y < s.H && x < s.W;
            kf[r][c] = (in && fabsf(hv[j]) < HEIGHT_LIMIT) ? 1.f : 0.f;
        }
    }
    __syncthreads();
    for (int i = tid; i < SPAN * T; i += 256) {
        const int r = i / T, c = i % T;
        float n = 0.f;
        for (int d = 0; d < net::PATCH; ++d) n += kf[r][c + d];
        rs[r][c] = n;
    }
    __syncthreads();
    const int c = tid % T, r = tid / T;
    const int x = x0 + c, y = y0 + r;
    if (x < s.W && y < s.H) {
        float n = 0.f;
        for (int d = 0; d < net::PATCH; ++d) n += rs[r + d][c];
        s.known[(int64_t)y * s.W + x] = n * (1.f / (net::PATCH * net::PATCH));
    }
}

// Head of every state (cell, yaw unit): a wave owns 16 cells and loops over
// the yaw units, keeping fc2's weights, its biases and the cells' fc1 values
// (without the yaw term) in registers.  Both layers are computed transposed,
// neurons x states:
//   fc2: D2 (64 x 16) = W4 (64 x 128) . h1^T,   h1 = ReLU(T + Y[u]) in bf16
//   fc3: D3 (16 x 16, rows 0..3 used) = W5' (16 x 64) . h2^T,  h2 = ReLU(D2 + b4)
// In the 16x16x32 MFMA, lane (r, g) = (lane % 16, lane / 16) supplies A's row r
// and B's column r at reduction indices 8g .. 8g+7 and receives D rows
// 4g .. 4g+3 of column r.  The lane holding D2's rows 16t + 4g + e (t = 0..3)
// is therefore the lane that supplies fc3's B column r: fc3 takes them as
// reduction index 32ks + 8g + e' with neuron 32ks + 4g + e' for e' < 4 and
// 32ks + 16 + 4g + (e' - 4) for e' >= 4, and W5' is gathered in the same
// order, which leaves the sum unchanged and needs no trip through LDS.  Stores
// go to 16 consecutive cells of one yaw plane.
__global__ __launch_bounds__(256) void head_kernel(const SurArgs s, const AssessArgs a) {
    extern __shared__ float ys[];            // [U][128] yaw term, shared by the workgroup
    {
        // Eight loads per thread in flight before the LDS writes.
        const int n = s.U * net::H1;
        for (int i0 = threadIdx.x; i0 < n; i0 += 256 * 8) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = s.Y[min(i0 + 256 * j, n - 1)];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (i0 + 256 * j < n) ys[i0 + 256 * j] = v[j];
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int64_t cells = (int64_t)s.H * s.W;
    const int64_t c0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (c0 >= cells) return;
    const bool real = c0 + r < cells;
    const int64_t cell = real ? c0 + r : cells - 1;

    bf16x8 w4[4][4];                         // [t][ks]: W4[16t + r][32ks + 8g + e]
    float b4v[4][4];                         // [t][e]:  b4[16t + 4g + e]
    float tv[4][8];                          // [ks][e]: T[cell][32ks + 8g + e]
    bf16x8 w5[2];                            // [ks][e']: W5[r][neuron(ks, g, e')]
    static_assert(net::OFF_B4 % 4 == 0, "fc2 biases are read as float4");
    for (int t = 0; t < 4; ++t) {
        for (int ks = 0; ks < 4; ++ks)
            w4[t][ks] = *(const bf16x8*)(s.pw.w4 + (16 * t + r) * net::H1 + 32 * ks + 8 * g);
        const float4 b = *(const float4*)(s.theta + net::OFF_B4 + 16 * t + 4 * g);
        b4v[t][0] = b.x;
        b4v[t][1] = b.y;
        b4v[t][2] = b.z;
        b4v[t][3] = b.w;
    }
    for (int ks = 0; ks < 4; ++ks) {
        const float4* tp = (const float4*)(s.T + cell * net::H1 + 32 * ks + 8 * g);
        const float4 t0 = tp[0], t1 = tp[1];
        tv[ks][0] = t0.x; tv[ks][1] = t0.y; tv[ks][2] = t0.z; tv[ks][3] = t0.w;
        tv[ks][4] = t1.x; tv[ks][5] = t1.y; tv[ks][6] = t1.z; tv[ks][7] = t1.w;
    }
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    for (int ks = 0; ks < 2; ++ks) {
        // neurons 32 ks + 4 g .. + 3, then 32 ks + 16 + 4 g .. + 3 (rows 4..15 of
        // the packed W5 are zero)
        const bf16x4 lo = *(const bf16x4*)(s.pw.w5 + r * net::H2 + 32 * ks + 4 * g);
        const bf16x4 hi = *(const bf16x4*)(s.pw.w5 + r * net::H2 + 32 * ks + 16 + 4 * g);
        for (int e = 0; e < 4; ++e) {
            w5[ks][e] = lo[e];
            w5[ks][4 + e] = hi[e];
        }
    }

    float b5[4];
    for (int j = 0; j < 4; ++j) b5[j] = s.theta[net::OFF_B5 + j];

    // Per-cell part of the fallback rule and the plane height offset.
    const int cy = (int)(cell / s.W), cx = (int)(cell % s.W);
    float hc;
    const bool has_ref = ref_height(s, cy, cx, &hc);
    const bool out_of_dist = !has_ref || s.known[cell] < s.min_known;
    // Every load above is complete before the loop: a wait inside it would
    // also wait for the previous unit's stores.
    __builtin_amdgcn_s_waitcnt(0);

    for (int u = 0; u < s.U; ++u) {
        f32x4 acc[4];
        for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 4; ++ks) {
            const float4* yp = (const float4*)(ys + u * net::H1 + 32 * ks + 8 * g);
            const float4 y0 = yp[0], y1 = yp[1];
            bf16x8 h;
            h[0] = to_bf16(fmaxf(tv[ks][0] + y0.x, 0.f));
            h[1] = to_bf16(fmaxf(tv[ks][1] + y0.y, 0.f));
            h[2] = to_bf16(fmaxf(tv[ks][2] + y0.z, 0.f));
            h[3] = to_bf16(fmaxf(tv[ks][3] + y0.w, 0.f));
            h[4] = to_bf16(fmaxf(tv[ks][4] + y1.x, 0.f));
            h[5] = to_bf16(fmaxf(tv[ks][5] + y1.y, 0.f));
            h[6] = to_bf16(fmaxf(tv[ks][6] + y1.z, 0.f));
            h[7] = to_bf16(fmaxf(tv[ks][7] + y1.w, 0.f));
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w4[t][ks], h, acc[t], 0, 0, 0);
        }
        f32x4 y3 = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 h2;
            for (int e = 0; e < 4; ++e) {
                h2[e] = to_bf16(fmaxf(acc[2 * ks][e] + b4v[2 * ks][e], 0.f));
                h2[4 + e] = to_bf16(fmaxf(acc[2 * ks + 1][e] + b4v[2 * ks + 1][e], 0.f));
            }
            y3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w5[ks], h2, y3, 0, 0, 0);
        }
        // Lanes of group 0 hold the four outputs of state (cell, u).
        if (g == 0 && real) {
            const float o0 = y3[0] + b5[0];
            const float o1 = y3[1] + b5[1];
            const float o2 = y3[2] + b5[2];
            const float o3 = y3[3] + b5[3];
            const float risk = fminf(fmaxf(o3, 0.f), 1.f);
            const bool fb = out_of_dist || fabsf(risk - s.risk_max) < s.band;
            s.need[(int64_t)u * cells + cell] = fb ? 1 : 0;
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
    hipLaunchKernelGGL(prep_kernel, dim3((s.W + 15) / 16, (s.H + 15) / 16), dim3(256), 0, stream, s);
    hipLaunchKernelGGL(conv1_map_kernel, dim3(blocks((int64_t)(s.H + 20) * (s.W + 20), 256)),
                       dim3(256), 0, stream, s);
    hipLaunchKernelGGL(conv2_map_kernel, dim3(blocks((int64_t)(s.H + 16) * (s.W + 16), 64)),
                       dim3(256), 0, stream, s);
    hipLaunchKernelGGL(fc1_map_kernel, dim3(blocks(cells, FC1_CELLS)), dim3(256), 0, stream, s);
    hipLaunchKernelGGL(head_kernel, dim3(blocks(cells, 64)), dim3(256),
                       (size_t)s.U * net::H1 * sizeof(float), stream, s, a);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace seb
