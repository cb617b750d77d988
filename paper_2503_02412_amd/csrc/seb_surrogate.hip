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
// Flagged states -- unknown own cell, too few known cells in the window (out
// of the training distribution), or predicted risk within `band` of risk_max
// -- are appended to per-yaw lists and re-assessed by the plain method.
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
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(bf16, (uint16_t)(u >> 16));
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

// conv1 at every position (y1, x1) in [-12, H+8) x [-12, W+8): ReLU(b1 + W1 . input
// window [y1, y1+4) x [x1, x1+4)); inputs and outputs rounded to bf16 as in training.
__global__ __launch_bounds__(256) void conv1_map_kernel(const SurArgs s) {
    __shared__ float w[net::C1 * net::K1];
    for (int i = threadIdx.x; i < net::C1 * net::K1; i += 256) {
        const int o = i / net::K1, c = i % net::K1;
        w[i] = from_bf16(s.pw.w1[o * net::K1P + c]);
    }
    __syncthreads();
    const int W1 = s.W + 20;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)(s.H + 20) * W1) return;
    const int y1 = (int)(p / W1) - 12, x1 = (int)(p % W1) - 12;
    float in[net::K1];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            float v0, vx, vy;
            const float h0 = height_at(s, y1 + i, x1 + j, &v0);
            const float hx = height_at(s, y1 + i, x1 + j + 1, &vx);
            const float hy = height_at(s, y1 + i + 1, x1 + j, &vy);
            in[0 * 16 + i * 4 + j] = from_bf16(to_bf16(v0 * vx * (hx - h0) * s.inv_res));
            in[1 * 16 + i * 4 + j] = from_bf16(to_bf16(v0 * vy * (hy - h0) * s.inv_res));
            in[2 * 16 + i * 4 + j] = v0;
        }
    bf16* out = s.o1map + p * net::C1;
    for (int o = 0; o < net::C1; ++o) {
        float acc = 0.f;
        for (int c = 0; c < net::K1; ++c) acc = fmaf(w[o * net::K1 + c], in[c], acc);
        out[o] = to_bf16(fmaxf(acc + s.theta[net::OFF_B1 + o], 0.f));
    }
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
            const float v = fmaxf(acc[t][e] + s.theta[net::OFF_B2 + n], 0.f);
            s.o2map[row * net::C2 + n] = to_bf16(v);
        }
}

// fc1 without the yaw term, per cell: T[cell][n] = b3[n] + W3[n] . (conv2 at
// the 5 x 5 positions cell - 12 + 4 (a, b)).  Implicit GEMM: a workgroup owns 64
// cells; wave w computes outputs [32 w, 32 w + 32).
__global__ __launch_bounds__(256) void fc1_map_kernel(const SurArgs s) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int W2 = s.W + 16;
    const int64_t cells = (int64_t)s.H * s.W;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const int r = lane & 15, kq = lane >> 4;
    int cy[4], cx[4];
    for (int i = 0; i < 4; ++i) {
        const int64_t c = min(c0 + 16 * i + r, cells - 1);
        cy[i] = (int)(c / s.W);
        cx[i] = (int)(c % s.W);
    }
    f32x4 acc[4][2];
    for (int i = 0; i < 4; ++i)
        for (int t = 0; t < 2; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < net::F / 32; ++ks) {
        const int a5 = ks / 5, b5 = ks % 5;
        bf16x8 bfr[2];
        for (int t = 0; t < 2; ++t)
            bfr[t] = *(const bf16x8*)(s.pw.w3 + (int64_t)(32 * wave + 16 * t + r) * net::F + 32 * ks +
                                      8 * kq);
        for (int i = 0; i < 4; ++i) {
            const int y2 = cy[i] - 12 + 4 * a5, x2 = cx[i] - 12 + 4 * b5;
            const bf16x8 a =
                *(const bf16x8*)(s.o2map + ((int64_t)(y2 + 12) * W2 + (x2 + 12)) * net::C2 + 8 * kq);
            for (int t = 0; t < 2; ++t)
                acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[t], acc[i][t], 0, 0, 0);
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int t = 0; t < 2; ++t)
            for (int e = 0; e < 4; ++e) {
                const int64_t c = c0 + 16 * i + 4 * kq + e;
                const int n = 32 * wave + 16 * t + r;
                if (c < cells) s.T[c * net::H1 + n] = acc[i][t][e] + s.theta[net::OFF_B3 + n];
            }
}

// Yaw term of fc1 for the first U yaw bins: Y[u][n] = Wy[n] . (sin, cos)(2 pi u / K).
__global__ void yaw_kernel(const SurArgs s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.U * net::H1) {
        if (i < s.K) s.counts[i] = 0;
        return;
    }
    const int u = i / net::H1, n = i % net::H1;
    const double th = 2.0 * 3.14159265358979323846 * (double)u / (double)s.K;
    const float sn = (float)sin(th), cs = (float)cos(th);
    s.Y[i] = sn * s.theta[net::OFF_WY + 2 * n] + cs * s.theta[net::OFF_WY + 2 * n + 1];
    if (i < s.K) s.counts[i] = 0;
}

// Known cells in each cell's 24 x 24 window: row sums, then column sums.
__global__ void known_rows_kernel(const SurArgs s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)s.H * s.W) return;
    const int y = (int)(p / s.W), x = (int)(p % s.W);
    float n = 0.f, v;
    for (int dx = -net::HALF; dx < net::HALF; ++dx) {
        height_at(s, y, x + dx, &v);
        n += v;
    }
    s.rows[p] = n;
}

__global__ void known_cols_kernel(const SurArgs s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)s.H * s.W) return;
    const int y = (int)(p / s.W), x = (int)(p % s.W);
    float n = 0.f;
    for (int dy = -net::HALF; dy < net::HALF; ++dy) {
        const int yy = y + dy;
        if (yy >= 0 && yy < s.H) n += s.rows[(int64_t)yy * s.W + x];
    }
    s.known[p] = n * (1.f / (net::PATCH * net::PATCH));
}

// Head per state (cell, yaw unit), 16 states per wave tile:
// h1 = ReLU(T + Y) -> fc2 (MFMA) -> ReLU -> fc3 (MFMA) -> outputs and flags.
__global__ __launch_bounds__(256) void head_kernel(const SurArgs s, const AssessArgs a) {
    __shared__ bf16 h2s[4][16][net::H2 + 8];
    __shared__ float ys[4][16][4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t cells = (int64_t)s.H * s.W;
    const int64_t states = cells * s.U;
    const int64_t s0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (s0 >= states) return;
    const int r = lane & 15, kq = lane >> 4;
    const int64_t st = min(s0 + r, states - 1);
    const int64_t cell = st / s.U;
    const int u = (int)(st % s.U);
    f32x4 acc[4];
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < net::H1 / 32; ++ks) {
        const int k = 32 * ks + 8 * kq;
        const float4* tp = (const float4*)(s.T + cell * net::H1 + k);
        const float4* yp = (const float4*)(s.Y + u * net::H1 + k);
        const float4 t0 = tp[0], t1 = tp[1], y0 = yp[0], y1 = yp[1];
        bf16x8 a;
        a[0] = to_bf16(fmaxf(t0.x + y0.x, 0.f));
        a[1] = to_bf16(fmaxf(t0.y + y0.y, 0.f));
        a[2] = to_bf16(fmaxf(t0.z + y0.z, 0.f));
        a[3] = to_bf16(fmaxf(t0.w + y0.w, 0.f));
        a[4] = to_bf16(fmaxf(t1.x + y1.x, 0.f));
        a[5] = to_bf16(fmaxf(t1.y + y1.y, 0.f));
        a[6] = to_bf16(fmaxf(t1.z + y1.z, 0.f));
        a[7] = to_bf16(fmaxf(t1.w + y1.w, 0.f));
        for (int t = 0; t < 4; ++t) {
            const bf16x8 b = *(const bf16x8*)(s.pw.w4 + (16 * t + r) * net::H1 + k);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
    for (int t = 0; t < 4; ++t)
        for (int e = 0; e < 4; ++e) {
            const int n = 16 * t + r;
            h2s[wave][4 * kq + e][n] = to_bf16(fmaxf(acc[t][e] + s.theta[net::OFF_B4 + n], 0.f));
        }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): LDS writes of this wave done
    __builtin_amdgcn_wave_barrier();
    f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < net::H2 / 32; ++ks) {
        const int k = 32 * ks + 8 * kq;
        const bf16x8 av = *(const bf16x8*)(&h2s[wave][r][k]);
        const bf16x8 b = *(const bf16x8*)(s.pw.w5 + r * net::H2 + k);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, y, 0, 0, 0);
    }
    if (r < net::NOUT)
        for (int e = 0; e < 4; ++e) ys[wave][4 * kq + e][r] = y[e] + s.theta[net::OFF_B5 + r];
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    if (lane >= 16 || s0 + lane >= states) return;
    const float* o = ys[wave][lane];
    const int cy = (int)(cell / s.W), cx = (int)(cell % s.W);
    float kn;
    const float hc = height_at(s, cy, cx, &kn);
    const float risk = fminf(fmaxf(o[3], 0.f), 1.f);
    const bool fallback = !(kn > 0.f) || s.known[cell] < s.min_known ||
                          fabsf(risk - s.risk_max) < s.band;
    if (fallback) {
        const int idx = atomicAdd(&s.counts[u], 1);
        s.lists[(int64_t)u * cells + idx] = (int)cell;
        return;
    }
    Result res;
    res.z = hc + net::S_Z * o[0];
    res.roll = net::S_A * o[1];
    res.pitch = net::S_A * o[2];
    res.risk = risk;
    res.st = SEB_ST_VALID | SEB_ST_SURROGATE | (risk <= s.risk_max ? SEB_ST_TRAV : 0);
    store(a, u, cell, res, false);
    if (a.mirror) store(a, u + a.mirror, cell, res, true);
}

// The map with SENTINEL for unknown cells and an R-cell border, so the
// fallback kernel reads footprint corners without bounds checks.
__global__ void pad_kernel(const SurArgs s) {
    const int Wp = s.W + 2 * s.R;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)(s.H + 2 * s.R) * Wp) return;
    const int y = (int)(i / Wp) - s.R, x = (int)(i % Wp) - s.R;
    float v = SENTINEL;
    if (y >= 0 && x >= 0 && y < s.H && x < s.W) {
        const float h = s.height[(int64_t)y * s.ld + x];
        if (fabsf(h) < HEIGHT_LIMIT) v = h;
    }
    s.pad[i] = v;
}

// Plain-method re-assessment of the listed states of yaw unit blockIdx.y:
// the same arithmetic as the tiled kernel, heights from the padded map.
template <int NW, int FIT>
__global__ __launch_bounds__(64) void fallback_kernel(const SurArgs s, const AssessArgs a) {
    const int u = blockIdx.y;
    const int count = s.counts[u];
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (blockIdx.x * 64 >= count) return;
    const bool active = i < count;
    const int64_t cells = (int64_t)s.H * s.W;
    const int cell = active ? s.lists[(int64_t)u * cells + i] : 0;
    const int ix = cell % s.W, iy = cell / s.W;
    const int ldp = s.W + 2 * s.R;
    PaddedSource src;
    src.base = s.pad + (int64_t)(iy + s.R) * ldp + (ix + s.R);
    src.ldp = ldp;
    src.P = s.pitch;
    const float hc = src.base[0];
    const Result r = assess_state<NW, FIT>(a, src, u, hc, active);
    if (active) {
        store(a, u, cell, r, false);
        if (a.mirror) store(a, u + a.mirror, cell, r, true);
    }
}

__global__ void total_kernel(const SurArgs s, int32_t* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int n = 0;
    for (int u = 0; u < s.U; ++u) n += s.counts[u];
    *out = n * (s.mirror ? 2 : 1);
}

template <int FIT>
void launch_fallback(const SurArgs& s, const AssessArgs& a, dim3 fg, hipStream_t stream) {
    switch (a.row_len) {
        case 4: hipLaunchKernelGGL((fallback_kernel<4, FIT>), fg, dim3(64), 0, stream, s, a); break;
        case 12: hipLaunchKernelGGL((fallback_kernel<12, FIT>), fg, dim3(64), 0, stream, s, a); break;
        case 24: hipLaunchKernelGGL((fallback_kernel<24, FIT>), fg, dim3(64), 0, stream, s, a); break;
        default: hipLaunchKernelGGL((fallback_kernel<0, FIT>), fg, dim3(64), 0, stream, s, a); break;
    }
}

}  // namespace

hipError_t launch_surrogate(const SurArgs& s, const AssessArgs& a, int32_t* n_fallback,
                            hipStream_t stream) {
    const int64_t cells = (int64_t)s.H * s.W;
    auto blocks = [](int64_t n, int b) { return (unsigned)((n + b - 1) / b); };
    hipLaunchKernelGGL(yaw_kernel, dim3(blocks(std::max<int64_t>(s.U * net::H1, s.K), 256)),
                       dim3(256), 0, stream, s);
    hipLaunchKernelGGL(pad_kernel, dim3(blocks((int64_t)(s.H + 2 * s.R) * (s.W + 2 * s.R), 256)),
                       dim3(256), 0, stream, s);
    hipLaunchKernelGGL(known_rows_kernel, dim3(blocks(cells, 256)), dim3(256), 0, stream, s);
    hipLaunchKernelGGL(known_cols_kernel, dim3(blocks(cells, 256)), dim3(256), 0, stream, s);
    hipLaunchKernelGGL(conv1_map_kernel, dim3(blocks((int64_t)(s.H + 20) * (s.W + 20), 256)),
                       dim3(256), 0, stream, s);
    hipLaunchKernelGGL(conv2_map_kernel, dim3(blocks((int64_t)(s.H + 16) * (s.W + 16), 64)),
                       dim3(256), 0, stream, s);
    hipLaunchKernelGGL(fc1_map_kernel, dim3(blocks(cells, 64)), dim3(256), 0, stream, s);
    hipLaunchKernelGGL(head_kernel, dim3(blocks(cells * s.U, 64)), dim3(256), 0, stream, s, a);
    const dim3 fg(blocks(cells, 64), s.U);
    if (a.fit == 1)
        launch_fallback<1>(s, a, fg, stream);
    else
        launch_fallback<0>(s, a, fg, stream);
    if (n_fallback) hipLaunchKernelGGL(total_kernel, dim3(1), dim3(64), 0, stream, s, n_fallback);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace seb
