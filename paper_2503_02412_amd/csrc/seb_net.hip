// Learned surrogate of the SE(2) assessment: training kernels (patch form) on
// bf16 MFMA for gfx950, Adam, and the C ABI of the network handle.
//
// Every layer of the patch-form network is one "NT" GEMM, C[m][n] =
// sum_k A[m][k] B[n][k], both operands K-contiguous bf16, fp32 accumulation on
// v_mfma_f32_16x16x32_bf16.  Backward data products use transposed weight
// copies; weight gradients are NT GEMMs of transposed deltas and activations
// with split-K partials reduced deterministically into the parameter layout.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include "seb_trace.hpp"
#include <string>
#include <vector>

#include "seb.h"
#include "seb_net_internal.hpp"

namespace seb {
namespace net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16 to_bf16(float f) {
    return (bf16)f;   // round to nearest even (v_cvt_pk_bf16_f32)
}
__device__ __forceinline__ float from_bf16(bf16 h) {
    return __uint_as_float((uint32_t)__builtin_bit_cast(uint16_t, h) << 16);
}

// ------------------------------------------------------------------ GEMM
// Block tile 64 x 64, four waves of 32 x 32 (2 x 2 MFMA tiles of 16 x 16).
// Operand fragments are loaded straight from global memory: lane l holds
// row (l % 16) and k-block 8 (l / 16) of its 16 x 32 A and B slices; the
// accumulator of lane l holds rows 4 (l / 16) + e, column l % 16.
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int bx, int by, int bz) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = bx * 64 + (wave >> 1) * 32;
    const int n0 = by * 64 + (wave & 1) * 32;
    const int kb = bz * g.kchunk;
    const int ke = min(g.K, kb + g.kchunk);
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (m0 < g.M && n0 < g.N) {
        // Fragments of the next GD K steps in flight.  Rows past M and columns
        // past N read the last row or column: they only feed accumulator
        // entries that are never stored.
        const bf16* arow[2];
        const bf16* brow[2];
        for (int t = 0; t < 2; ++t) {
            arow[t] = g.A + (int64_t)min(m0 + 16 * t + r, g.M - 1) * g.lda + kq;
            brow[t] = g.B + (int64_t)min(n0 + 16 * t + r, g.N - 1) * g.ldb + kq;
        }
        constexpr int GD = 4;
        bf16x8 a[GD][2], b[GD][2];
        const int steps = (ke - kb) / 32;
#pragma unroll
        for (int p = 0; p < GD; ++p) {
            const int k = kb + 32 * min(p, steps - 1);
            for (int t = 0; t < 2; ++t) {
                a[p][t] = *(const bf16x8*)(arow[t] + k);
                b[p][t] = *(const bf16x8*)(brow[t] + k);
            }
        }
        for (int s0 = 0; s0 < steps; s0 += GD) {
#pragma unroll
            for (int p = 0; p < GD; ++p) {
                if (s0 + p < steps) {
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[p][i], b[p][j], acc[i][j], 0, 0, 0);
                    // the next loads of this slot (the last GD steps re-load a valid step)
                    const int k = kb + 32 * min(s0 + p + GD, steps - 1);
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        a[p][t] = *(const bf16x8*)(arow[t] + k);
                        b[p][t] = *(const bf16x8*)(brow[t] + k);
                    }
                }
            }
        }
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][e];
                if (g.split) {
                    g.C[bz * g.split + (int64_t)m * g.ldc + n] = v;
                    continue;
                }
                if (g.bias) v += g.bias[n];
                if (g.rowv)
                    v += g.rowv[2 * m] * g.colv[2 * n] + g.rowv[2 * m + 1] * g.colv[2 * n + 1];
                if (g.relu) v = fmaxf(v, 0.f);
                if (g.gate && !(from_bf16(g.gate[(int64_t)m * g.ldg + n]) > 0.f)) v = 0.f;
                if (g.C) g.C[(int64_t)m * g.ldc + n] = v;
                if (g.Cb) g.Cb[(int64_t)m * g.ldcb + n] = to_bf16(v);
            }
}

__global__ __launch_bounds__(256) void gemm_nt_kernel(const GemmArgs g) {
    gemm_tile(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Several independent products in one launch (the weight gradients of a
// backward pass): product k covers workgroups [block0_k, block0_k + gx_k gy_k
// gz_k) of a one-dimensional grid, in gemm_nt_kernel's (x, y, z) order.
constexpr int kGemmGroup = 5;
struct GemmGroup {
    GemmArgs a[kGemmGroup];
    int block0[kGemmGroup], gx[kGemmGroup], gy[kGemmGroup];
    int n;
};

__global__ __launch_bounds__(256) void gemm_group_kernel(const GemmGroup G) {
    int k = 0;
    for (int q = 1; q < G.n; ++q)
        if ((int)blockIdx.x >= G.block0[q]) k = q;
    const int local = (int)blockIdx.x - G.block0[k];
    const int gx = G.gx[k], gy = G.gy[k];
    gemm_tile(G.a[k], local % gx, (local / gx) % gy, local / (gx * gy));
}

// ------------------------------------------------------ patch-form inputs
struct BatchArgs {
    const float* maps;            // [n_maps][mh][mw]
    int n_maps, mh, mw;
    float inv_res;
    int K;
    const float* lz;              // labels [n_maps][K][mh][mw] (may be null: no targets)
    const float* lroll;
    const float* lpitch;
    const float* lrisk;
    const int32_t* samples;       // [B][4] (map, cy, cx, k)
    int B;
};

__device__ __forceinline__ float map_at(const BatchArgs& a, int mi, int y, int x, float* known) {
    if (y < 0 || x < 0 || y >= a.mh || x >= a.mw) {
        *known = 0.f;
        return 0.f;
    }
    const float h = a.maps[((int64_t)mi * a.mh + y) * a.mw + x];
    const bool ok = fabsf(h) < 0x1p60f;
    *known = ok ? 1.f : 0.f;
    return ok ? h : 0.f;
}

// Height the z output is relative to: the cell's own height when known, else
// the mean of its known 8-neighbours (false when none is known).
__device__ __forceinline__ bool ref_height(const BatchArgs& a, int mi, int cy, int cx, float* h) {
    float v;
    const float h0 = map_at(a, mi, cy, cx, &v);
    if (v > 0.f) {
        *h = h0;
        return true;
    }
    float sum = 0.f, n = 0.f;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dy == 0 && dx == 0) continue;
            sum += map_at(a, mi, cy + dy, cx + dx, &v);      // 0 when unknown
            n += v;
        }
    *h = n > 0.f ? sum / n : 0.f;
    return n > 0.f;
}

// conv1 on its im2col rows, row (b*121 + a*11 + bb) column c*16 + i*4 + j;
// yaw features and targets.  One thread per row (sample b, conv1 position
// (a, bb)): the 5 x 5 cells under its 4 x 4 window and the next row and
// column (for the slopes) are read once, the row's 48 inputs are rounded to
// bf16, and the 16 outputs ReLU(b1 + W1 . row) go out as two 16-byte stores
// of bf16 (with FP32 products and sums, as the MFMA products of the other
// layers); in training the row is also written as a column of the transposed
// im2col A1t (a wave's lanes write 64 consecutive entries of each of its
// rows), for conv1's weight gradient.  Input channels at cell (y, x), with k
// the known flag and h the height (0 where unknown): x-slope k(y,x) k(y,x+1)
// (h(y,x+1) - h(y,x)) / res, y-slope the same with (y+1, x), and k(y,x).
__global__ __launch_bounds__(256) void im2col1_kernel(const BatchArgs a, const bf16* w1, const float* b1,
                                                      bf16* o1, bf16* A1t, float* sc, float* tgt) {
    __shared__ float ws[C1][K1];             // conv1's weights (their bf16 values)
    for (int i = threadIdx.x; i < C1 * K1; i += 256) ws[i / K1][i % K1] = from_bf16(w1[(i / K1) * K1P + i % K1]);
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    static_assert(K1 == 48 && K1P % 8 == 0 && C1 == 16, "three channels of 4 x 4; 16 outputs");
    if (idx < (int64_t)a.B * P1 * P1) {
        const int pos = (int)(idx % (P1 * P1));
        const int b = (int)(idx / (P1 * P1));
        const int mi = a.samples[4 * b], cy = a.samples[4 * b + 1], cx = a.samples[4 * b + 2];
        const int y0 = cy - HALF + 2 * (pos / P1), x0 = cx - HALF + 2 * (pos % P1);
        float h[5][5], v[5][5];
#pragma unroll
        for (int i = 0; i < 5; ++i)
#pragma unroll
            for (int j = 0; j < 5; ++j) h[i][j] = map_at(a, mi, y0 + i, x0 + j, &v[i][j]);
        float in[K1];                          // the row's inputs, rounded to bf16
#pragma unroll
        for (int col = 0; col < K1; ++col) {
            const int c = col / 16, i = (col / 4) % 4, j = col % 4;
            float val;
            if (c == 0)
                val = v[i][j] * v[i][j + 1] * (h[i][j + 1] - h[i][j]) * a.inv_res;
            else if (c == 1)
                val = v[i][j] * v[i + 1][j] * (h[i + 1][j] - h[i][j]) * a.inv_res;
            else
                val = v[i][j];
            in[col] = from_bf16(to_bf16(val));
        }
        if (A1t) {                             // training: the transposed im2col, A1t[col][row]
            const int64_t rows = (int64_t)a.B * P1 * P1;
#pragma unroll
            for (int col = 0; col < K1P; ++col)
                A1t[(int64_t)col * rows + idx] = to_bf16(col < K1 ? in[col] : 0.f);
        }
        // conv1: o1[row][o] = bf16(ReLU(b1[o] + sum_col W1[o][col] in[col]))
        bf16x8 out[2];
#pragma unroll
        for (int o = 0; o < C1; ++o) {
            float acc = 0.f;
#pragma unroll
            for (int col = 0; col < K1; ++col) acc = fmaf(ws[o][col], in[col], acc);
            out[o / 8][o % 8] = to_bf16(fmaxf(acc + b1[o], 0.f));
        }
        bf16x8* dst = reinterpret_cast<bf16x8*>(o1 + idx * C1);
        dst[0] = out[0];
        dst[1] = out[1];
    }
    if (idx < a.B) {
        const int b = (int)idx;
        const int mi = a.samples[4 * b], cy = a.samples[4 * b + 1], cx = a.samples[4 * b + 2];
        const int k = a.samples[4 * b + 3];
        const double th = 2.0 * 3.14159265358979323846 * (double)k / (double)a.K;
        sc[2 * b] = (float)sin(th);
        sc[2 * b + 1] = (float)cos(th);
        if (a.lz) {
            const int64_t o = (((int64_t)mi * a.K + k) * a.mh + cy) * a.mw + cx;
            float hc;
            ref_height(a, mi, cy, cx, &hc);     // samples are drawn where one exists
            tgt[4 * b] = (a.lz[o] - hc) / S_Z;
            tgt[4 * b + 1] = a.lroll[o] / S_A;
            tgt[4 * b + 2] = a.lpitch[o] / S_A;
            tgt[4 * b + 3] = a.lrisk[o];
        }
    }
}

// conv2 im2col: A2[(b*25 + a2*5 + b2)][(i*3 + j)*16 + c] = o1[b*121 + (2a2+i)*11 + 2b2+j][c].
// One thread per (row, group of 16 columns): group t < 9 is tap t, whose 16
// channels are 32 contiguous bytes of o1 and of A2; group 9 is the padding.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void im2col2_kernel(const bf16* o1, bf16* A2, int B) {
    static_assert(C1 == 16 && K2 == 9 * 16 && K2P % 16 == 0, "a tap is 32 bytes of channels");
    constexpr int G = K2P / 16;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)B * P2 * P2 * G) return;
    const int tap = (int)(idx % G);
    const int64_t row = idx / G;
    const int pos = (int)(row % (P2 * P2));
    const int b = (int)(row / (P2 * P2));
    u32x4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
    if (tap < 9) {
        const int y = 2 * (pos / P2) + tap / 3, x = 2 * (pos % P2) + tap % 3;
        const u32x4* src = reinterpret_cast<const u32x4*>(o1 + ((int64_t)b * P1 * P1 + y * P1 + x) * C1);
        v0 = src[0];
        v1 = src[1];
    }
    u32x4* dst = reinterpret_cast<u32x4*>(A2 + row * K2P + tap * 16);
    dst[0] = v0;
    dst[1] = v1;
}

// Backward of im2col2, gated by conv1's ReLU: da1[b*121 + p][c], four
// channels per thread (in each channel the same sum, in the same order, as
// one channel at a time).
__global__ __launch_bounds__(256) void col2im2_kernel(const float* dA2, const bf16* o1, bf16* da1,
                                                      int B) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)B * P1 * P1 * (C1 / 4)) return;
    const int c = 4 * (int)(idx % (C1 / 4));
    const int64_t row = idx / (C1 / 4);
    const int p = (int)(row % (P1 * P1));
    const int b = (int)(row / (P1 * P1));
    const int y = p / P1, x = p % P1;
    float4 s = {0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < 3; ++i) {
        const int ty = y - i;
        if (ty < 0 || (ty & 1) || ty / 2 >= P2) continue;
        for (int j = 0; j < 3; ++j) {
            const int tx = x - j;
            if (tx < 0 || (tx & 1) || tx / 2 >= P2) continue;
            const int pos = (ty / 2) * P2 + tx / 2;
            const float4 d =
                *reinterpret_cast<const float4*>(dA2 + ((int64_t)b * P2 * P2 + pos) * K2P + (i * 3 + j) * 16 + c);
            s.x += d.x;
            s.y += d.y;
            s.z += d.z;
            s.w += d.w;
        }
    }
    const int64_t o = row * C1 + c;
    da1[o] = to_bf16(from_bf16(o1[o]) > 0.f ? s.x : 0.f);
    da1[o + 1] = to_bf16(from_bf16(o1[o + 1]) > 0.f ? s.y : 0.f);
    da1[o + 2] = to_bf16(from_bf16(o1[o + 2]) > 0.f ? s.z : 0.f);
    da1[o + 3] = to_bf16(from_bf16(o1[o + 3]) > 0.f ? s.w : 0.f);
}

// Tiled transposes of bf16 matrices, dst[c][r] = src[r][c], all of a
// backward pass's in prep_kernel's launch: job j covers workgroups [block0_j, block0_j
// + tiles_x_j * tiles_y_j).  A workgroup moves a 64 x 64 tile through LDS;
// each thread reads two 16-byte runs of a source row and writes two 16-byte
// runs of a destination row (element by element where a run is cut by the
// matrix edge or is not 16-byte aligned).
struct TrJob {
    const bf16* src;
    int R, C;
    int64_t lds;
    bf16* dst;
    int64_t ldd;
    int tiles_x, block0;
};
constexpr int kTrJobs = 9;
struct TrJobs {
    TrJob j[kTrJobs];
    int n;
};

__device__ __forceinline__ void transpose_body(const TrJobs& J, int bid) {
    typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
    __shared__ uint16_t tile[64][66];
    int jk = 0;
    for (int q = 1; q < J.n; ++q)
        if (bid >= J.j[q].block0) jk = q;
    const TrJob& jb = J.j[jk];
    const int R = jb.R, Ccols = jb.C;
    const int64_t lds = jb.lds, ldd = jb.ldd;
    const int tb = bid - jb.block0;
    const int t = threadIdx.x;
    const int r0 = (tb / jb.tiles_x) * 64, c0 = (tb % jb.tiles_x) * 64;
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(jb.src);
    uint16_t* d16 = reinterpret_cast<uint16_t*>(jb.dst);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int rr = (t >> 3) + 32 * k, cc = (t & 7) * 8;
        const int r = r0 + rr, c = c0 + cc;
        if (r >= R) continue;
        const uint16_t* p = s16 + (int64_t)r * lds + c;
        if (c + 8 <= Ccols && ((uintptr_t)p & 15) == 0) {
            const u16x8 v = *reinterpret_cast<const u16x8*>(p);
#pragma unroll
            for (int e = 0; e < 8; ++e) tile[rr][cc + e] = v[e];
        } else {
            for (int e = 0; e < 8 && c + e < Ccols; ++e) tile[rr][cc + e] = p[e];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int cc = (t >> 3) + 32 * k, rr = (t & 7) * 8;
        const int c = c0 + cc, r = r0 + rr;
        if (c >= Ccols) continue;
        uint16_t* p = d16 + (int64_t)c * ldd + r;
        if (r + 8 <= R && ((uintptr_t)p & 15) == 0) {
            u16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = tile[rr + e][cc];
            *reinterpret_cast<u16x8*>(p) = v;
        } else {
            for (int e = 0; e < 8 && r + e < R; ++e) p[e] = tile[rr + e][cc];
        }
    }
}

// Loss: mean over the batch of sum_o w_o (y_o - t_o)^2; dy = dL/dy in bf16
// ([B][32], columns >= 4 stay zero); per-block partial loss sums.
__global__ __launch_bounds__(256) void loss_kernel(const float* y, int64_t ldy, const float* t,
                                                   int B, bf16* dy, float* partial) {
    __shared__ float red[256];
    const int b = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (b < B) {
        for (int o = 0; o < NOUT; ++o) {
            const float r = y[(int64_t)b * ldy + o] - t[4 * b + o];
            l += r * r;
            dy[(int64_t)b * 32 + o] = to_bf16(2.f * r / (float)B);
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// The loss: the mean over the batch of the loss kernel's per-block sums.
struct LossJob {
    const float* partial;
    int n, B;
    float* out;                  // null: no loss asked for
};

__device__ __forceinline__ void finish_loss_body(const LossJob& L) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < L.n; ++i) s += L.partial[i];
    *L.out = (float)(s / L.B);
}

// Sums of the split-K partial products part[z][M][N] over z, written to the
// gradients in the parameter layout (kind 0: [M][N]; 1: conv1's first K1 of
// K1P columns; 2: conv2's (tap, channel) columns to (channel, tap)), for every
// weight gradient, in finish_kernel's launch.  Job j
// covers workgroups [block0_j, block0_j + blocks_j); a workgroup adds `per`
// outputs (64, 16 or 8): thread (o, q) sums z = q, q + L, ... with
// L = 256 / per lanes (coalesced over o), and the lanes are added in a fixed
// order.
struct RedJob {
    const float* part;
    int Z, M, N, kind, per, blocks, block0;
    float* dst;
};
constexpr int kRedJobs = 5;
struct RedJobs {
    RedJob j[kRedJobs];
    int n;
};

__device__ __forceinline__ void reduce_split_body(const RedJobs& J, int bid) {
    __shared__ float red[256];
    int k = 0;
    for (int q = 1; q < J.n; ++q)
        if (bid >= J.j[q].block0) k = q;
    const RedJob& jb = J.j[k];
    const int per = jb.per, L = 256 / per, N = jb.N;
    const int o = threadIdx.x % per, q = threadIdx.x / per;
    const int idx = (bid - jb.block0) * per + o;
    const int64_t mn = (int64_t)jb.M * N;
    float s = 0.f;
    if (idx < mn)
        for (int z = q; z < jb.Z; z += L) s += jb.part[(int64_t)z * mn + idx];
    red[threadIdx.x] = s;
    __syncthreads();
    if (q != 0 || idx >= mn) return;
    s = red[o];
    for (int j = 1; j < L; ++j) s += red[o + per * j];
    const int m = idx / N, n = idx % N;
    if (jb.kind == 0) {
        jb.dst[idx] = s;
    } else if (jb.kind == 1) {
        if (n < K1) jb.dst[m * K1 + n] = s;
    } else {
        if (n < K2) jb.dst[m * K2 + (n % 16) * 9 + n / 16] = s;
    }
}

// Column sums of the first N columns of bf16 matrices D [M][ld] (N a power
// of two <= 256), optionally weighted by w[m][0/1]: the bias gradients of
// every layer, in prep_kernel's and finish_kernel's launches.  Job
// j covers blocks [block0_j, block0_j + blocks_j) of the first pass, and
// block b of a job sums rows [b * rows, (b + 1) * rows): thread t takes
// column t % N and every (256 / N)-th row from row t / N on, so 256 / N rows
// are read per step; the row lanes are then added in order through LDS into
// the job's partial[b][N][nw].  The second pass adds the blocks' partials of
// one output per workgroup (a fixed-order tree), so the sums are
// deterministic.  Products and sums are rounded one at a time.
struct ColJob {
    const bf16* D;
    int64_t ld;
    int M, N, rows, blocks, block0, out0;
    const float* w;     // [M][2] row weights, or null
    float* part;        // the job's partial sums
    float* dst;         // N (or 2N, interleaved) outputs
};
constexpr int kColJobs = 6;
static_assert(NOUT + H2 + 2 * H1 + H1 + C2 + C1 <= 512, "partials of every job fit kColBlocks x 512");
struct ColJobs {
    ColJob j[kColJobs];
    int n;
};

__device__ __forceinline__ void colsum_body(const ColJobs& J, int bid) {
#pragma clang fp contract(off)
    __shared__ float red[2][256];
    int k = 0;
    for (int q = 1; q < J.n; ++q)
        if (bid >= J.j[q].block0) k = q;
    const ColJob& jb = J.j[k];
    const int N = jb.N, M = jb.M;
    const int blk = bid - jb.block0;
    const int t = threadIdx.x, c = t & (N - 1), lanes = 256 / N;
    const int r0 = blk * jb.rows, r1 = min(M, r0 + jb.rows);
    float s0 = 0.f, s1 = 0.f;
    for (int m = r0 + t / N; m < r1; m += lanes) {
        const float v = from_bf16(jb.D[(int64_t)m * jb.ld + c]);
        if (jb.w) {
            s0 += v * jb.w[2 * m];
            s1 += v * jb.w[2 * m + 1];
        } else {
            s0 += v;
        }
    }
    red[0][t] = s0;
    red[1][t] = s1;
    __syncthreads();
    if (t < N) {
        float a0 = 0.f, a1 = 0.f;
        for (int j = 0; j < lanes; ++j) {
            a0 += red[0][t + N * j];
            a1 += red[1][t + N * j];
        }
        if (jb.w) {
            jb.part[((int64_t)blk * N + t) * 2] = a0;
            jb.part[((int64_t)blk * N + t) * 2 + 1] = a1;
        } else {
            jb.part[(int64_t)blk * N + t] = a0;
        }
    }
}

__device__ __forceinline__ void colsum_finish_body(const ColJobs& J, int bid) {
    __shared__ float red[256];
    int k = 0;
    for (int q = 1; q < J.n; ++q)
        if (bid >= J.j[q].out0) k = q;
    const ColJob& jb = J.j[k];
    const int cnt = jb.N * (jb.w ? 2 : 1);
    const int i = bid - jb.out0, t = threadIdx.x;       // output i of the job
    float s = 0.f;
    for (int b = t; b < jb.blocks; b += 256) s += jb.part[(int64_t)b * cnt + i];
    red[t] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0) jb.dst[i] = red[0];
}

// The backward pass's two launches after its input gradients and products:
// prep_kernel runs every transpose (workgroups [0, tr_blocks)) and the first
// pass of every column sum (the rest); finish_kernel adds every column sum's
// block partials (workgroups [0, col_outputs)), every weight gradient's
// split-K partials (the next red_blocks) and, when asked for, the loss.
__global__ __launch_bounds__(256) void prep_kernel(const TrJobs T, int tr_blocks, const ColJobs C) {
    if ((int)blockIdx.x < tr_blocks)
        transpose_body(T, blockIdx.x);
    else
        colsum_body(C, (int)blockIdx.x - tr_blocks);
}

__global__ __launch_bounds__(256) void finish_kernel(const ColJobs C, int col_outputs, const RedJobs R,
                                                     int red_blocks, const LossJob L) {
    if ((int)blockIdx.x < col_outputs)
        colsum_finish_body(C, blockIdx.x);
    else if ((int)blockIdx.x < col_outputs + red_blocks)
        reduce_split_body(R, (int)blockIdx.x - col_outputs);
    else
        finish_loss_body(L);     // one more workgroup when the loss is asked for
}

// bf16 weight copies in GEMM layouts (see PackedWeights).
__global__ __launch_bounds__(256) void pack_kernel(const float* th, PackedWeights w) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < C1 * K1P) {                               // w1 [16][64]
        const int o = i / K1P, c = i % K1P;
        w.w1[i] = to_bf16(c < K1 ? th[OFF_W1 + o * K1 + c] : 0.f);
    }
    if (i < C2 * K2P) {                               // w2 [32][160], w2t [160][32]
        const int o = i / K2P, c = i % K2P;
        const float v = c < K2 ? th[OFF_W2 + o * K2 + (c % 16) * 9 + c / 16] : 0.f;
        w.w2[i] = to_bf16(v);
        w.w2t[c * C2 + o] = to_bf16(v);
    }
    if (i < H1 * F) {                                 // w3 [128][800], w3t [800][128]
        const int o = i / F, c = i % F;
        const float v = th[OFF_W3 + i];
        w.w3[i] = to_bf16(v);
        w.w3t[c * H1 + o] = to_bf16(v);
        const int kk = c / 16, h = (c % 16) / 8, e = c % 8, t = o / 32, l = o % 32 + 32 * h;
        w.w3f[(((int64_t)kk * 4 + t) * 64 + l) * 8 + e] = to_bf16(v);
    }
    if (i < H2 * H1) {                                // w4 [64][128], w4t [128][64]
        const int o = i / H1, c = i % H1;
        const float v = th[OFF_W4 + i];
        w.w4[i] = to_bf16(v);
        w.w4t[c * H2 + o] = to_bf16(v);
        w.w4h[i] = (f16)(float)to_bf16(v);
    }
    if (i < 16 * H2) {                                // w5 [16][64], w5t [64][32]
        const int o = i / H2, c = i % H2;
        const bf16 b = to_bf16(o < NOUT ? th[OFF_W5 + o * H2 + c] : 0.f);
        w.w5[i] = b;
        w.w5h[i] = (f16)(float)b;
    }
    if (i < H2 * 32) {
        const int c = i / 32, o = i % 32;
        w.w5t[i] = to_bf16(o < NOUT ? th[OFF_W5 + o * H2 + c] : 0.f);
    }
}

// Adam step fused with the bf16 refresh: parameter i's new value also goes
// to its places in the packed GEMM copies, the inverse of pack_kernel's
// mapping (the copies' padding, written by pack_kernel, never changes).
__global__ __launch_bounds__(256) void adam_pack_kernel(float* theta, float* m, float* v, const float* g,
                                                        int64_t n, float lr, float c1, float c2,
                                                        PackedWeights w) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    theta[i] = th;
    const bf16 b = to_bf16(th);
    if (i >= OFF_W1 && i < OFF_W1 + C1 * K1) {
        const int j = (int)(i - OFF_W1), o = j / K1, c = j % K1;
        w.w1[o * K1P + c] = b;
    } else if (i >= OFF_W2 && i < OFF_W2 + C2 * K2) {
        const int j = (int)(i - OFF_W2), o = j / K2, t = j % K2;
        const int c = (t % 9) * 16 + t / 9;          // column (tap, channel) of parameter (channel, tap)
        w.w2[o * K2P + c] = b;
        w.w2t[c * C2 + o] = b;
    } else if (i >= OFF_W3 && i < OFF_W3 + (int64_t)H1 * F) {
        const int j = (int)(i - OFF_W3), o = j / F, c = j % F;
        w.w3[j] = b;
        w.w3t[c * H1 + o] = b;
        const int kk = c / 16, h = (c % 16) / 8, e = c % 8, t = o / 32, l = o % 32 + 32 * h;
        w.w3f[(((int64_t)kk * 4 + t) * 64 + l) * 8 + e] = b;
    } else if (i >= OFF_W4 && i < OFF_W4 + H2 * H1) {
        const int j = (int)(i - OFF_W4), o = j / H1, c = j % H1;
        w.w4[j] = b;
        w.w4t[c * H2 + o] = b;
        w.w4h[j] = (f16)(float)b;
    } else if (i >= OFF_W5 && i < OFF_W5 + NOUT * H2) {
        const int j = (int)(i - OFF_W5), o = j / H2, c = j % H2;
        w.w5[o * H2 + c] = b;
        w.w5h[o * H2 + c] = (f16)(float)b;
        w.w5t[c * 32 + o] = b;
    }
}

// Counter-based init: splitmix64 of (seed, index) -> uniform in [-1, 1).
__global__ __launch_bounds__(256) void init_kernel(float* th, int64_t n, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float u = (float)((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f;
    // He-uniform bound sqrt(6 / fan_in) per weight tensor; biases start at zero.
    float bound = 0.f;
    if (i < OFF_B1) bound = sqrtf(6.f / K1);
    else if (i >= OFF_W2 && i < OFF_B2) bound = sqrtf(6.f / K2);
    else if (i >= OFF_W3 && i < OFF_B3) bound = sqrtf(6.f / (F + 2));
    else if (i >= OFF_W4 && i < OFF_B4) bound = sqrtf(6.f / H1);
    else if (i >= OFF_W5 && i < OFF_B5) bound = sqrtf(6.f / H2);
    th[i] = u * bound;
}

}  // namespace net
}  // namespace seb

// ========================================================================
// Host side: the network handle and its C ABI.
// ========================================================================

using seb::net::bf16;
namespace N = seb::net;

namespace {

thread_local std::string g_net_error;

int net_fail(int code, const std::string& msg) {
    g_net_error = msg;
    return code;
}

}  // namespace

struct seb_net {
    int max_batch = 0;
    int64_t step = 0;
    int device = 0;
    float* theta = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    N::PackedWeights pw{};
    // workspace (max_batch rows)
    bf16 *A1t = nullptr, *o1 = nullptr, *da1 = nullptr, *da1t = nullptr;
    bf16 *A2 = nullptr, *A2t = nullptr, *f = nullptr, *ft = nullptr, *da2 = nullptr, *da2t = nullptr;
    bf16 *h1 = nullptr, *h1t = nullptr, *da3 = nullptr, *da3t = nullptr;
    bf16 *h2 = nullptr, *h2t = nullptr, *da4 = nullptr, *da4t = nullptr;
    bf16 *dy = nullptr, *dyt = nullptr;
    float *dA2 = nullptr, *y = nullptr, *tgt = nullptr, *sc = nullptr;
    float *part = nullptr, *lpart = nullptr, *cpart = nullptr;
    std::vector<void*> allocs;
};

namespace {

constexpr int kColBlocks = 1024;     // most blocks of a column-sum pass
constexpr int kColSteps = 32;        // row steps per block when blocks allow

// Split-K partial buffer: the largest Z * M * N of the weight-gradient GEMMs.
// Split-K chunks of the weight gradients (multiples of 32): a few hundred
// workgroups per product.  The conv layers reduce over 0.1 M and 0.5 M rows.
constexpr int kFcChunk = 256, kConvChunk = 1024;

int64_t part_floats(int64_t Bm) {
    auto z = [](int64_t K, int64_t chunk) { return (K + chunk - 1) / chunk; };
    // every layer's partial products side by side (one reduction launch)
    int64_t m = z(Bm, kFcChunk) * N::H1 * N::F;
    m += z(Bm, kFcChunk) * N::H2 * N::H1;
    m += z(Bm, kFcChunk) * N::NOUT * N::H2;
    m += z(Bm * N::P2 * N::P2, kConvChunk) * N::C2 * N::K2P;
    m += z(Bm * N::P1 * N::P1, kConvChunk) * N::C1 * N::K1P;
    return m;
}

template <typename T>
bool dalloc(seb_net* n, T** p, int64_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)count * sizeof(T)) != hipSuccess) return false;
    n->allocs.push_back(q);
    *p = (T*)q;
    return true;
}

int64_t blocks_for(int64_t n) { return (n + 255) / 256; }

hipError_t gemm(const N::GemmArgs& g, hipStream_t s) {
    const int zc = g.split ? (g.K + g.kchunk - 1) / g.kchunk : 1;
    dim3 grid((g.M + 63) / 64, (g.N + 63) / 64, zc);
    hipLaunchKernelGGL(N::gemm_nt_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

int gemm_zcount(const N::GemmArgs& g) { return g.split ? (g.K + g.kchunk - 1) / g.kchunk : 1; }

// Adds the product g to G; run_group launches them together.
void add_gemm(N::GemmGroup& G, const N::GemmArgs& g) {
    const int k = G.n;
    G.a[k] = g;
    G.gx[k] = (g.M + 63) / 64;
    G.gy[k] = (g.N + 63) / 64;
    G.block0[k] = k == 0 ? 0 : G.block0[k - 1] + G.gx[k - 1] * G.gy[k - 1] * gemm_zcount(G.a[k - 1]);
    G.n += 1;
}

void run_group(const N::GemmGroup& G, hipStream_t s) {
    const int k = G.n - 1;
    const int blocks = G.block0[k] + G.gx[k] * G.gy[k] * gemm_zcount(G.a[k]);
    hipLaunchKernelGGL(N::gemm_group_kernel, dim3(blocks), dim3(256), 0, s, G);
}

N::GemmArgs gemm_args(const bf16* A, int64_t lda, const bf16* B, int64_t ldb, int M, int Nn, int K) {
    N::GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.M = M;
    g.N = Nn;
    g.K = K;
    g.kchunk = K;
    return g;
}

// Adds the transpose dst = src^T (src [R][C], row strides lds and ldd) to T
// (run by prep_kernel).
void add_transpose(N::TrJobs& T, const bf16* src, int R, int C, int64_t lds, bf16* dst, int64_t ldd) {
    N::TrJob& jb = T.j[T.n];
    int block0 = 0;
    if (T.n > 0) {
        const N::TrJob& pj = T.j[T.n - 1];
        block0 = pj.block0 + pj.tiles_x * ((pj.R + 63) / 64);
    }
    jb.src = src;
    jb.R = R;
    jb.C = C;
    jb.lds = lds;
    jb.dst = dst;
    jb.ldd = ldd;
    jb.tiles_x = (C + 63) / 64;
    jb.block0 = block0;
    T.n += 1;
}

int tr_blocks(const N::TrJobs& T) {
    const N::TrJob& last = T.j[T.n - 1];
    return last.block0 + last.tiles_x * ((last.R + 63) / 64);
}

// Weight gradient dst = A^T-style NT GEMM of [M][K] and [Nn][K] with split-K
// into the layer's own region of n->part: the product is added to G (one
// launch for every layer, run_group) and its reduction to R (finish_kernel).
void weight_grad(seb_net* n, N::GemmGroup& G, N::RedJobs& R, const bf16* A, const bf16* B, int M, int Nn,
                 int K, int kchunk, int kind, float* dst) {
    float* part = n->part;
    int block0 = 0;
    if (R.n > 0) {
        const N::RedJob& pj = R.j[R.n - 1];
        part = const_cast<float*>(pj.part) + (int64_t)pj.Z * pj.M * pj.N;
        block0 = pj.block0 + pj.blocks;
    }
    N::GemmArgs g = gemm_args(A, K, B, K, M, Nn, K);
    g.kchunk = kchunk;
    g.split = (int64_t)M * Nn;
    g.C = part;
    g.ldc = Nn;
    add_gemm(G, g);
    const int Z = (K + kchunk - 1) / kchunk;
    const int per = Z >= 64 ? 8 : Z >= 16 ? 16 : 64;      // outputs per workgroup
    N::RedJob& jb = R.j[R.n];
    jb.part = part;
    jb.Z = Z;
    jb.M = M;
    jb.N = Nn;
    jb.kind = kind;
    jb.per = per;
    jb.blocks = (int)(((int64_t)M * Nn + per - 1) / per);
    jb.block0 = block0;
    jb.dst = dst;
    R.n += 1;
}

int red_blocks(const N::RedJobs& R) {
    const N::RedJob& last = R.j[R.n - 1];
    return last.block0 + last.blocks;
}

// Adds a column-sum job (see colsum_body) to J (run by prep_kernel and
// finish_kernel).
void add_colsum(N::ColJobs& J, seb_net* n, const bf16* D, int64_t ld, int M, int Nn, const float* w,
                float* dst) {
    // rows per block: kColSteps steps of 256 / Nn rows, more when that would
    // need more than kColBlocks blocks
    const int lanes = 256 / Nn;
    const int64_t per = std::max<int64_t>((int64_t)lanes * kColSteps, ((int64_t)M + kColBlocks - 1) / kColBlocks);
    const int rows = (int)((per + lanes - 1) / lanes * lanes);
    const int blocks = std::max(1, (int)(((int64_t)M + rows - 1) / rows));
    N::ColJob& jb = J.j[J.n];
    float* part = n->cpart;
    int block0 = 0, out0 = 0;
    if (J.n > 0) {
        const N::ColJob& pj = J.j[J.n - 1];
        const int pnw = pj.w ? 2 : 1;
        part = pj.part + (int64_t)pj.blocks * pj.N * pnw;
        block0 = pj.block0 + pj.blocks;
        out0 = pj.out0 + pj.N * pnw;
    }
    jb.D = D;
    jb.ld = ld;
    jb.M = M;
    jb.N = Nn;
    jb.rows = rows;
    jb.blocks = blocks;
    jb.block0 = block0;
    jb.out0 = out0;
    jb.w = w;
    jb.part = part;
    jb.dst = dst;
    J.n += 1;
}

int col_blocks(const N::ColJobs& J) {
    const N::ColJob& last = J.j[J.n - 1];
    return last.block0 + last.blocks;
}

int col_outputs(const N::ColJobs& J) {
    const N::ColJob& last = J.j[J.n - 1];
    return last.out0 + last.N * (last.w ? 2 : 1);
}

int check_batch(const seb_net* n, const seb_train_batch* b, bool need_labels) {
    if (!n || !b) return net_fail(SEB_ERR_INVALID, "net and batch must be non-NULL");
    if (!b->maps || !b->samples) return net_fail(SEB_ERR_INVALID, "maps and samples must be set");
    if (b->batch <= 0 || b->batch % 32 != 0 || b->batch > n->max_batch)
        return net_fail(SEB_ERR_INVALID, "batch must be a positive multiple of 32 <= max_batch");
    if (b->n_maps <= 0 || b->map_h <= 0 || b->map_w <= 0 || b->n_yaw <= 0 ||
        !(b->resolution > 0.0))
        return net_fail(SEB_ERR_INVALID, "bad map geometry");
    if (need_labels && (!b->label_z || !b->label_roll || !b->label_pitch || !b->label_risk))
        return net_fail(SEB_ERR_INVALID, "training needs all four label arrays");
    return SEB_OK;
}

N::BatchArgs batch_args(const seb_train_batch* b) {
    N::BatchArgs a;
    a.maps = b->maps;
    a.n_maps = b->n_maps;
    a.mh = b->map_h;
    a.mw = b->map_w;
    a.inv_res = (float)(1.0 / b->resolution);
    a.K = b->n_yaw;
    a.lz = b->label_z;
    a.lroll = b->label_roll;
    a.lpitch = b->label_pitch;
    a.lrisk = b->label_risk;
    a.samples = b->samples;
    a.B = b->batch;
    return a;
}

// Forward pass of the patch-form network for a batch; outputs y [B][4] into out.
// train: also lay out conv1's im2col transposed (A1t), for its weight gradient.
hipError_t forward_pass(seb_net* n, const seb_train_batch* bt, float* out, bool train, hipStream_t s) {
    const int B = bt->batch;
    const N::BatchArgs ba = batch_args(bt);
    const int64_t r1 = (int64_t)B * N::P1 * N::P1, r2 = (int64_t)B * N::P2 * N::P2;
    hipLaunchKernelGGL(N::im2col1_kernel, dim3(blocks_for(r1)), dim3(256), 0, s, ba, n->pw.w1,
                       n->theta + N::OFF_B1, n->o1, train ? n->A1t : nullptr, n->sc, n->tgt);
    hipLaunchKernelGGL(N::im2col2_kernel, dim3(blocks_for(r2 * (N::K2P / 16))), dim3(256), 0, s, n->o1,
                       n->A2, B);
    N::GemmArgs g = gemm_args(n->A2, N::K2P, n->pw.w2, N::K2P, (int)r2, N::C2, N::K2P);
    g.bias = n->theta + N::OFF_B2;
    g.relu = 1;
    g.Cb = n->f;
    g.ldcb = N::C2;
    gemm(g, s);
    g = gemm_args(n->f, N::F, n->pw.w3, N::F, B, N::H1, N::F);
    g.bias = n->theta + N::OFF_B3;
    g.rowv = n->sc;
    g.colv = n->theta + N::OFF_WY;
    g.relu = 1;
    g.Cb = n->h1;
    g.ldcb = N::H1;
    gemm(g, s);
    g = gemm_args(n->h1, N::H1, n->pw.w4, N::H1, B, N::H2, N::H1);
    g.bias = n->theta + N::OFF_B4;
    g.relu = 1;
    g.Cb = n->h2;
    g.ldcb = N::H2;
    gemm(g, s);
    g = gemm_args(n->h2, N::H2, n->pw.w5, N::H2, B, N::NOUT, N::H2);
    g.bias = n->theta + N::OFF_B5;
    g.C = out;
    g.ldc = N::NOUT;
    return gemm(g, s);
}

hipError_t pack(seb_net* n, hipStream_t s) {
    hipLaunchKernelGGL(N::pack_kernel, dim3(blocks_for((int64_t)N::H1 * N::F)), dim3(256), 0, s,
                       n->theta, n->pw);
    return hipGetLastError();
}

}  // namespace

namespace seb {
namespace net {
const float* net_theta(const seb_net* n) { return n->theta; }
PackedWeights net_packed(const seb_net* n) { return n->pw; }
}  // namespace net
}  // namespace seb

extern "C" {

int64_t seb_net_param_count(void) { return N::N_PARAMS; }

const char* seb_net_last_error(void) { return g_net_error.c_str(); }

void seb_net_destroy(seb_net* n) {
    if (!n) return;
    for (void* p : n->allocs) (void)hipFree(p);
    delete n;
}

int seb_net_create(uint64_t seed, int32_t max_batch, seb_net** out) {
    SEB_TRACE_RANGE();
    if (!out) return net_fail(SEB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (max_batch < 32 || max_batch % 32 != 0 || max_batch > (1 << 16))
        return net_fail(SEB_ERR_INVALID, "max_batch must be a multiple of 32 in [32, 65536]");
    seb_net* n = new (std::nothrow) seb_net();
    if (!n) return net_fail(SEB_ERR_ALLOC, "host allocation failed");
    n->max_batch = max_batch;
    (void)hipGetDevice(&n->device);
    const int64_t Bm = max_batch;
    const int64_t r1 = Bm * N::P1 * N::P1, r2 = Bm * N::P2 * N::P2;
    bool ok = dalloc(n, &n->theta, N::N_PARAMS) && dalloc(n, &n->m, N::N_PARAMS) &&
              dalloc(n, &n->v, N::N_PARAMS) && dalloc(n, &n->grad, N::N_PARAMS) &&
              dalloc(n, &n->pw.w1, N::C1 * N::K1P) && dalloc(n, &n->pw.w2, N::C2 * N::K2P) &&
              dalloc(n, &n->pw.w3, N::H1 * N::F) && dalloc(n, &n->pw.w4, N::H2 * N::H1) &&
              dalloc(n, &n->pw.w5, 16 * N::H2) && dalloc(n, &n->pw.w2t, N::K2P * N::C2) &&
              dalloc(n, &n->pw.w3t, N::F * N::H1) && dalloc(n, &n->pw.w4t, N::H1 * N::H2) &&
              dalloc(n, &n->pw.w5t, N::H2 * 32) && dalloc(n, &n->pw.w4h, N::H2 * N::H1) &&
              dalloc(n, &n->pw.w3f, N::H1 * N::F) &&
              dalloc(n, &n->pw.w5h, 16 * N::H2) && dalloc(n, &n->A1t, r1 * N::K1P) && dalloc(n, &n->o1, r1 * N::C1) &&
              dalloc(n, &n->da1, r1 * N::C1) && dalloc(n, &n->da1t, r1 * N::C1) &&
              dalloc(n, &n->A2, r2 * N::K2P) && dalloc(n, &n->A2t, r2 * N::K2P) &&
              dalloc(n, &n->dA2, r2 * N::K2P) && dalloc(n, &n->f, Bm * N::F) &&
              dalloc(n, &n->ft, Bm * N::F) && dalloc(n, &n->da2, Bm * N::F) &&
              dalloc(n, &n->da2t, Bm * N::F) && dalloc(n, &n->h1, Bm * N::H1) &&
              dalloc(n, &n->h1t, Bm * N::H1) && dalloc(n, &n->da3, Bm * N::H1) &&
              dalloc(n, &n->da3t, Bm * N::H1) && dalloc(n, &n->h2, Bm * N::H2) &&
              dalloc(n, &n->h2t, Bm * N::H2) && dalloc(n, &n->da4, Bm * N::H2) &&
              dalloc(n, &n->da4t, Bm * N::H2) && dalloc(n, &n->dy, Bm * 32) &&
              dalloc(n, &n->dyt, Bm * 32) && dalloc(n, &n->y, Bm * N::NOUT) &&
              dalloc(n, &n->tgt, Bm * N::NOUT) && dalloc(n, &n->sc, Bm * 2) &&
              dalloc(n, &n->part, part_floats(Bm)) && dalloc(n, &n->lpart, Bm / 256 + 1) &&
              dalloc(n, &n->cpart, kColBlocks * 512);   // >= kColBlocks x (sum of N x nw of the jobs)
    if (!ok) {
        seb_net_destroy(n);
        return net_fail(SEB_ERR_ALLOC, "device allocation failed");
    }
    hipError_t e;
    if ((e = hipMemset(n->dy, 0, Bm * 32 * sizeof(bf16))) != hipSuccess ||
        (e = hipMemset(n->m, 0, N::N_PARAMS * sizeof(float))) != hipSuccess ||
        (e = hipMemset(n->v, 0, N::N_PARAMS * sizeof(float))) != hipSuccess) {
        seb_net_destroy(n);
        return net_fail(SEB_ERR_HIP, std::string("hipMemset: ") + hipGetErrorString(e));
    }
    hipLaunchKernelGGL(N::init_kernel, dim3(blocks_for(N::N_PARAMS)), dim3(256), 0, 0, n->theta,
                       N::N_PARAMS, seed);
    pack(n, 0);
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        seb_net_destroy(n);
        return net_fail(SEB_ERR_HIP, std::string("init: ") + hipGetErrorString(e));
    }
    *out = n;
    return SEB_OK;
}

int seb_net_get_params(const seb_net* n, float* host) {
    if (!n || !host) return net_fail(SEB_ERR_INVALID, "net and host must be non-NULL");
    hipError_t e = hipMemcpy(host, n->theta, N::N_PARAMS * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    return SEB_OK;
}

int seb_net_set_params(seb_net* n, const float* host) {
    if (!n || !host) return net_fail(SEB_ERR_INVALID, "net and host must be non-NULL");
    hipError_t e;
    if ((e = hipMemcpy(n->theta, host, N::N_PARAMS * sizeof(float), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemset(n->m, 0, N::N_PARAMS * sizeof(float))) != hipSuccess ||
        (e = hipMemset(n->v, 0, N::N_PARAMS * sizeof(float))) != hipSuccess)
        return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    n->step = 0;
    pack(n, 0);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    return SEB_OK;
}

// File: "SEBNET01", int64 parameter count, int64 Adam step, then theta, m, v (float32).
int seb_net_save(const seb_net* n, const char* path) {
    if (!n || !path) return net_fail(SEB_ERR_INVALID, "net and path must be non-NULL");
    std::vector<float> buf(3 * N::N_PARAMS);
    hipError_t e;
    if ((e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(buf.data(), n->theta, N::N_PARAMS * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(buf.data() + N::N_PARAMS, n->m, N::N_PARAMS * 4, hipMemcpyDeviceToHost)) !=
            hipSuccess ||
        (e = hipMemcpy(buf.data() + 2 * N::N_PARAMS, n->v, N::N_PARAMS * 4,
                       hipMemcpyDeviceToHost)) != hipSuccess)
        return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return net_fail(SEB_ERR_IO, std::string("cannot open ") + path);
    const int64_t hdr[2] = {N::N_PARAMS, n->step};
    bool ok = std::fwrite("SEBNET01", 1, 8, fp) == 8 && std::fwrite(hdr, 8, 2, fp) == 2 &&
              std::fwrite(buf.data(), 4, buf.size(), fp) == buf.size();
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? SEB_OK : net_fail(SEB_ERR_IO, std::string("write failed: ") + path);
}

int seb_net_load(seb_net* n, const char* path) {
    if (!n || !path) return net_fail(SEB_ERR_INVALID, "net and path must be non-NULL");
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return net_fail(SEB_ERR_IO, std::string("cannot open ") + path);
    char magic[8];
    int64_t hdr[2];
    std::vector<float> buf(3 * N::N_PARAMS);
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "SEBNET01", 8) == 0 &&
              std::fread(hdr, 8, 2, fp) == 2 && hdr[0] == N::N_PARAMS && hdr[1] >= 0 &&
              std::fread(buf.data(), 4, buf.size(), fp) == buf.size();
    std::fclose(fp);
    if (!ok) return net_fail(SEB_ERR_IO, std::string("not a valid network file: ") + path);
    hipError_t e;
    if ((e = hipMemcpy(n->theta, buf.data(), N::N_PARAMS * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(n->m, buf.data() + N::N_PARAMS, N::N_PARAMS * 4, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(n->v, buf.data() + 2 * N::N_PARAMS, N::N_PARAMS * 4,
                       hipMemcpyHostToDevice)) != hipSuccess)
        return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    n->step = hdr[1];
    pack(n, 0);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    return SEB_OK;
}

int seb_net_forward(seb_net* n, const seb_train_batch* b, float* y_dev, void* stream) {
    SEB_TRACE_RANGE();
    int rc = check_batch(n, b, false);
    if (rc != SEB_OK) return rc;
    if (!y_dev) return net_fail(SEB_ERR_INVALID, "y_dev is NULL");
    hipError_t e = forward_pass(n, b, y_dev, false, (hipStream_t)stream);
    if (e != hipSuccess) return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    return SEB_OK;
}

int seb_net_train_step(seb_net* n, const seb_train_batch* bt, float lr, float* loss_dev,
                       float* grad_dev, void* stream) {
    SEB_TRACE_RANGE();
    int rc = check_batch(n, bt, true);
    if (rc != SEB_OK) return rc;
    if (!(lr >= 0.f) || !std::isfinite(lr)) return net_fail(SEB_ERR_INVALID, "bad learning rate");
    hipStream_t s = (hipStream_t)stream;
    const int B = bt->batch;
    const int r1 = B * N::P1 * N::P1, r2 = B * N::P2 * N::P2;
    hipError_t e = forward_pass(n, bt, n->y, true, s);
    if (e != hipSuccess) return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    float* g = n->grad;

    // loss and dy
    const int lb = (B + 255) / 256;
    hipLaunchKernelGGL(N::loss_kernel, dim3(lb), dim3(256), 0, s, n->y, (int64_t)N::NOUT, n->tgt, B,
                       n->dy, n->lpart);
    N::LossJob lj;             // finished in the backward pass's last launch
    lj.partial = n->lpart;
    lj.n = lb;
    lj.B = B;
    lj.out = loss_dev;
    // Input gradients, layer by layer, gated by the forward pass's ReLUs.
    // fc3
    N::GemmArgs ga = gemm_args(n->dy, 32, n->pw.w5t, 32, B, N::H2, 32);
    ga.gate = n->h2;
    ga.ldg = N::H2;
    ga.Cb = n->da4;
    ga.ldcb = N::H2;
    gemm(ga, s);
    // fc2
    ga = gemm_args(n->da4, N::H2, n->pw.w4t, N::H2, B, N::H1, N::H2);
    ga.gate = n->h1;
    ga.ldg = N::H1;
    ga.Cb = n->da3;
    ga.ldcb = N::H1;
    gemm(ga, s);
    // fc1
    ga = gemm_args(n->da3, N::H1, n->pw.w3t, N::H1, B, N::F, N::H1);
    ga.gate = n->f;
    ga.ldg = N::F;
    ga.Cb = n->da2;
    ga.ldcb = N::F;
    gemm(ga, s);
    // conv2 (da2 viewed as [B*25][32]), then conv1's through col2im
    ga = gemm_args(n->da2, N::C2, n->pw.w2t, N::C2, r2, N::K2P, N::C2);
    ga.C = n->dA2;
    ga.ldc = N::K2P;
    gemm(ga, s);
    hipLaunchKernelGGL(N::col2im2_kernel, dim3(blocks_for((int64_t)r1 * (N::C1 / 4))), dim3(256), 0, s,
                       n->dA2, n->o1, n->da1, B);
    // The weight gradients' operands, transposed in one launch (conv1's
    // im2col was laid out transposed by the forward pass).
    N::TrJobs tj;
    tj.n = 0;
    add_transpose(tj, n->dy, B, 32, 32, n->dyt, B);
    add_transpose(tj, n->h2, B, N::H2, N::H2, n->h2t, B);
    add_transpose(tj, n->da4, B, N::H2, N::H2, n->da4t, B);
    add_transpose(tj, n->h1, B, N::H1, N::H1, n->h1t, B);
    add_transpose(tj, n->da3, B, N::H1, N::H1, n->da3t, B);
    add_transpose(tj, n->f, B, N::F, N::F, n->ft, B);
    add_transpose(tj, n->da2, r2, N::C2, N::C2, n->da2t, r2);
    add_transpose(tj, n->A2, r2, N::K2P, N::K2P, n->A2t, r2);
    add_transpose(tj, n->da1, r1, N::C1, N::C1, n->da1t, r1);
    N::ColJobs cj;
    cj.n = 0;
    add_colsum(cj, n, n->dy, 32, B, N::NOUT, nullptr, g + N::OFF_B5);
    add_colsum(cj, n, n->da4, N::H2, B, N::H2, nullptr, g + N::OFF_B4);
    add_colsum(cj, n, n->da3, N::H1, B, N::H1, n->sc, g + N::OFF_WY);
    add_colsum(cj, n, n->da3, N::H1, B, N::H1, nullptr, g + N::OFF_B3);
    add_colsum(cj, n, n->da2, N::C2, r2, N::C2, nullptr, g + N::OFF_B2);
    add_colsum(cj, n, n->da1, N::C1, r1, N::C1, nullptr, g + N::OFF_B1);
    // every transpose and the bias gradients' first pass, in one launch
    const int trb = tr_blocks(tj);
    hipLaunchKernelGGL(N::prep_kernel, dim3(trb + col_blocks(cj)), dim3(256), 0, s, tj, trb, cj);
    // weight gradients: split-K products, one grouped launch
    N::GemmGroup gg;
    gg.n = 0;
    N::RedJobs rj;
    rj.n = 0;
    weight_grad(n, gg, rj, n->dyt, n->h2t, N::NOUT, N::H2, B, kFcChunk, 0, g + N::OFF_W5);
    weight_grad(n, gg, rj, n->da4t, n->h1t, N::H2, N::H1, B, kFcChunk, 0, g + N::OFF_W4);
    weight_grad(n, gg, rj, n->da3t, n->ft, N::H1, N::F, B, kFcChunk, 0, g + N::OFF_W3);
    weight_grad(n, gg, rj, n->da2t, n->A2t, N::C2, N::K2P, r2, kConvChunk, 2, g + N::OFF_W2);
    weight_grad(n, gg, rj, n->da1t, n->A1t, N::C1, N::K1P, r1, kConvChunk, 1, g + N::OFF_W1);
    run_group(gg, s);
    // the bias gradients' block sums and the weight gradients' split sums, in one launch
    const int co = col_outputs(cj);
    const int rb = red_blocks(rj);
    hipLaunchKernelGGL(N::finish_kernel, dim3(co + rb + (loss_dev ? 1 : 0)), dim3(256), 0, s, cj, co, rj, rb,
                       lj);

    if (grad_dev) {
        e = hipMemcpyAsync(grad_dev, g, N::N_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, s);
    } else {
        n->step += 1;
        const double c1 = 1.0 / (1.0 - std::pow(0.9, (double)n->step));
        const double c2 = 1.0 / (1.0 - std::pow(0.999, (double)n->step));
        hipLaunchKernelGGL(N::adam_pack_kernel, dim3(blocks_for(N::N_PARAMS)), dim3(256), 0, s, n->theta,
                           n->m, n->v, g, N::N_PARAMS, lr, (float)c1, (float)c2, n->pw);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return net_fail(SEB_ERR_HIP, hipGetErrorString(e));
    return SEB_OK;
}

}  // extern "C"
