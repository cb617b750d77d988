// SE(2) signed distance field of the obstacle states and the trilinear
// Risk / SDF query, for gfx950.
//
// The planner side of the method (Sec. VI-B, VI-C) needs, at every state, the
// distance to the edge of the nearest obstacle region (negative inside), and
// reads that field and the risk at arbitrary poses by trilinear interpolation
// with the yaw on SO(2).
//
// sdf_kernel: a workgroup owns a strip of R rows of one yaw plane and 256 - 2C
// of its columns; its 256 threads stand for those columns plus C more on each
// side.  With distances capped at C cells every target that matters lies
// within C cells in x and in y, so the exact two-pass transform runs on that
// window alone:
//   column pass -- each thread sweeps its column from C rows below the strip
//     up, then from C rows above it down, and keeps, for each strip row, the
//     distance in rows to the nearest obstacle and the nearest free cell of
//     the column (none beyond C), one byte each;
//   row pass -- for each cell, the minimum over |dx| <= C of dx^2 plus the
//     squared column value at x + dx for the opposite class.  A 64-bit ballot per word
//     of each row marks the columns holding any target; the nearest marked
//     column starts the scan, and a cell with none within C takes the cap at
//     once.  The scan ends once dx^2 alone reaches the best so far.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "seb.h"
#include "seb_sdf_internal.hpp"

namespace seb {
namespace {

constexpr int NT = 256;                   // threads = window columns
constexpr int NWORD = NT / 64;            // 64-bit column masks per row
constexpr uint8_t FAR = 0xFF;             // no target within C rows
constexpr int BIG = 1 << 20;
constexpr int DU = 4;                     // row-scan unroll; also the LDS row padding

struct SdfArgs {
    const uint8_t* status;                // [K][H][W], ring layout
    float* sdf;                           // [K][H][W], ring layout
    int W, H, K, rx, ry;
    int cap;                              // C, cells
    int tiles_x;                          // column blocks of NT - 2C
    float res;
    int unknown_is_obstacle;
};

__device__ __forceinline__ int wrap(int v, int n) { return v >= n ? v - n : v; }

// Distance from column t to the nearest set bit of the row mask m (NT bits),
// looking at most one word to either side (enough for C <= 64); > 64 if none.
__device__ __forceinline__ int nearest_marked(const uint64_t* m, int t) {
    const int w = t >> 6, b = t & 63;
    int left = -BIG, right = BIG;
    const uint64_t lo = m[w] & ((2ull << b) - 1ull);          // bits 0..b
    if (lo) left = (w << 6) + 63 - __clzll(lo);
    else if (w > 0 && m[w - 1]) left = ((w - 1) << 6) + 63 - __clzll(m[w - 1]);
    const uint64_t hi = m[w] & (~0ull << b);                  // bits b..63
    if (hi) right = (w << 6) + __ffsll((unsigned long long)hi) - 1;
    else if (w < NWORD - 1 && m[w + 1])
        right = ((w + 1) << 6) + __ffsll((unsigned long long)m[w + 1]) - 1;
    return min(t - left, right - t);
}

template <int R>
__global__ __launch_bounds__(NT) void sdf_kernel(const SdfArgs a) {
    // Column values (vertical distance in rows, <= C, or FAR), DU padding
    // entries (never a target) at both ends of a row.
    __shared__ uint8_t g_obs_p[R][NT + 2 * DU], g_free_p[R][NT + 2 * DU];
    __shared__ uint64_t m_obs[R][NWORD], m_free[R][NWORD];
    const int C = a.cap, TX = NT - 2 * C;
    const int t = threadIdx.x;
    // Workgroups are handed to the 8 XCDs in turn (linear id mod 8).  Give each
    // XCD a contiguous run of (plane, strip, column block), so that strips
    // sharing halo rows meet in the same L2.
    int bx, by, k;
    {
        const int64_t n = (int64_t)gridDim.x * gridDim.y;
        const int64_t lin = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        const int64_t q = n / 8, r = n % 8, xcd = lin % 8, pos = lin / 8;
        const int64_t lg = xcd < r ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
        const int64_t per_plane = (int64_t)gridDim.x;        // tiles_x * strips
        k = (int)(lg / per_plane);
        const int rest = (int)(lg - (int64_t)k * per_plane);
        bx = rest % a.tiles_x;
        by = rest / a.tiles_x;
    }
    const int xs = bx * TX - C + t;                          // this thread's column
    const int y0 = by * R, ny = min(R, a.H - y0);
    auto g_obs = [&](int j) { return &g_obs_p[j][DU]; };
    auto g_free = [&](int j) { return &g_free_p[j][DU]; };
    if (t < 2 * DU) {
        const int pc = t < DU ? t : NT + t;
        for (int j = 0; j < ny; ++j) g_obs_p[j][pc] = g_free_p[j][pc] = FAR;
    }

    if (xs >= 0 && xs < a.W) {
        const uint8_t* plane = a.status + (int64_t)k * a.W * a.H;
        const int cx = wrap(xs + a.rx, a.W);
        const int unk = a.unknown_is_obstacle;
        // Loads are unconditional, from rows clamped into the map, into plain
        // integers (one plane holds fewer than 2^31 cells); the guards and the
        // obstacle test come afterwards, so each batch of loads is in flight
        // at once.
        auto load = [&](int y) -> int { return plane[wrap(y + a.ry, a.H) * a.W + cx]; };
        // 1: CURV or TILT, a surrogate answer that is not traversable, or
        // UNKNOWN if counted
        auto obstacle = [&](int st) {
            return ((st >> 1) | (st >> 2) | ((st >> 5) & ~(st >> 4)) | (unk & ~st)) & 1;
        };
        // The halos only contribute the nearest obstacle / free row beyond the
        // strip: a min (below) and a max (above), HB rows at a time.
        constexpr int HB = 16;
        int no = BIG, nf = BIG;
        for (int yb = y0 + ny, ye = min(a.H, y0 + ny + C); yb < ye; yb += HB) {
            int sv[HB];
#pragma unroll
            for (int u = 0; u < HB; ++u) sv[u] = load(min(yb + u, ye - 1));
#pragma unroll
            for (int u = 0; u < HB; ++u) {
                const int y = yb + u < ye ? yb + u : BIG;
                if (obstacle(sv[u])) no = min(no, y); else nf = min(nf, y);
            }
        }
        int sv[R];
#pragma unroll
        for (int j = 0; j < R; ++j) sv[j] = load(min(y0 + j, a.H - 1));
        uint32_t ob = 0;                         // bit j: strip row j is an obstacle
#pragma unroll
        for (int j = 0; j < R; ++j) ob |= (uint32_t)obstacle(sv[j]) << j;
#pragma unroll
        for (int j = R - 1; j >= 0; --j) {
            if (j < ny) {
                if ((ob >> j) & 1) no = y0 + j; else nf = y0 + j;
                g_obs(j)[t] = (uint8_t)min(no - (y0 + j), C + 1);
                g_free(j)[t] = (uint8_t)min(nf - (y0 + j), C + 1);
            }
        }
        int ao = -BIG, af = -BIG;
        for (int yb = max(0, y0 - C); yb < y0; yb += HB) {
            int hv[HB];
#pragma unroll
            for (int u = 0; u < HB; ++u) hv[u] = load(min(yb + u, y0 - 1));
#pragma unroll
            for (int u = 0; u < HB; ++u) {
                const int y = yb + u < y0 ? yb + u : -BIG;
                if (obstacle(hv[u])) ao = max(ao, y); else af = max(af, y);
            }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (j < ny) {
                if ((ob >> j) & 1) ao = y0 + j; else af = y0 + j;
                const int d_o = min((int)g_obs(j)[t], y0 + j - ao);
                const int d_f = min((int)g_free(j)[t], y0 + j - af);
                g_obs(j)[t] = d_o <= C ? (uint8_t)d_o : FAR;
                g_free(j)[t] = d_f <= C ? (uint8_t)d_f : FAR;
            }
        }
    } else {
        for (int j = 0; j < ny; ++j) g_obs(j)[t] = g_free(j)[t] = FAR;   // outside the map
    }
    __syncthreads();
    // Column masks: wave w holds columns 64w .. 64w + 63.
    for (int j = 0; j < ny; ++j) {
        const uint64_t bo = __ballot(g_obs(j)[t] != FAR);
        const uint64_t bf = __ballot(g_free(j)[t] != FAR);
        if ((t & 63) == 0) {
            m_obs[j][t >> 6] = bo;
            m_free[j][t >> 6] = bf;
        }
    }
    __syncthreads();

    const int x_lo = bx * TX;                                 // first output column
    const int n_cols = min(TX, a.W - x_lo);
    const float res = a.res;
    for (int i = t; i < ny * n_cols; i += NT) {
        const int j = i / n_cols, c = i - j * n_cols;
        const int tc = C + c;                                 // window column of the cell
        const bool obst = g_obs(j)[tc] == 0;
        const uint8_t* g = obst ? g_free(j) : g_obs(j);
        const int dmin = nearest_marked(obst ? m_free[j] : m_obs[j], tc);
        int best = C * C;
        if (dmin <= C) {
            int dx = dmin;
            best = BIG;
            if (dx == 0) {
                best = g[tc] * g[tc];
                dx = 1;
            }
            // DU steps at a time: the 2 DU reads stay inside the padded row
            // (|dx| <= C + DU - 1) and are issued together; steps past C are
            // ignored.
            for (; dx <= C && dx * dx < best; dx += DU) {
                int gl[DU], gr[DU];
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    gl[u] = g[tc - dx - u];
                    gr[u] = g[tc + dx + u];
                }
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    const int e = dx + u, e2 = e <= C ? e * e : BIG;
                    if (gl[u] != FAR) best = min(best, e2 + gl[u] * gl[u]);
                    if (gr[u] != FAR) best = min(best, e2 + gr[u] * gr[u]);
                }
            }
            best = min(best, C * C);
        }
        const float v = (sqrtf((float)best) - 0.5f) * res;
        const int x = x_lo + c, y = y0 + j;
        a.sdf[(int64_t)k * a.W * a.H + (int64_t)wrap(y + a.ry, a.H) * a.W + wrap(x + a.rx, a.W)] =
            obst ? -v : v;
    }
}

struct QueryArgs {
    const float* fa;                      // [K][H][W], ring layout
    const float* fb;                      // [K][H][W] or nullptr
    const float* poses;                   // [n][3]
    float* out;                           // [n][8]
    int64_t n;
    int W, H, K, rx, ry;
    double res;
};

// Trilinear value and gradient of one field at one pose (corners c[w][v][u]).
__device__ __forceinline__ void trilinear(const float (&c)[2][2][2], float fu, float fv, float fw,
                                          float* o) {
    float cu[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) cu[a][b] = c[a][b][0] + fu * (c[a][b][1] - c[a][b][0]);
    float cuv[2], du_v[2];
    for (int a = 0; a < 2; ++a) {
        cuv[a] = cu[a][0] + fv * (cu[a][1] - cu[a][0]);
        const float d0 = c[a][0][1] - c[a][0][0], d1 = c[a][1][1] - c[a][1][0];
        du_v[a] = d0 + fv * (d1 - d0);
    }
    o[0] = cuv[0] + fw * (cuv[1] - cuv[0]);
    o[1] = du_v[0] + fw * (du_v[1] - du_v[0]);                            // d/du
    const float dv0 = cu[0][1] - cu[0][0], dv1 = cu[1][1] - cu[1][0];
    o[2] = dv0 + fw * (dv1 - dv0);                                         // d/dv
    o[3] = cuv[1] - cuv[0];                                                // d/dw
}

__device__ __forceinline__ void query_pose(const QueryArgs& q, int64_t n);

__global__ __launch_bounds__(256) void query_kernel(const QueryArgs q) {
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < q.n;
         n += (int64_t)gridDim.x * 256)
        query_pose(q, n);
}

__device__ __forceinline__ void query_pose(const QueryArgs& q, int64_t n) {
    const double x = q.poses[3 * n], y = q.poses[3 * n + 1], th = q.poses[3 * n + 2];
    const double ur = x / q.res - 0.5, vr = y / q.res - 0.5;
    const double u = fmin(fmax(ur, 0.0), q.W - 1.0), v = fmin(fmax(vr, 0.0), q.H - 1.0);
    const bool in_u = ur >= 0.0 && ur <= q.W - 1.0, in_v = vr >= 0.0 && vr <= q.H - 1.0;
    const double dth = 2.0 * 3.14159265358979323846 / q.K;
    double w = fmod(th / dth, (double)q.K);
    if (w < 0.0) w += q.K;
    if (w >= q.K) w -= q.K;
    if (!(w >= 0.0 && w < q.K)) w = 0.0;   // NaN / Inf yaw
    const int i0 = q.W > 1 ? min((int)floor(u), q.W - 2) : 0;
    const int j0 = q.H > 1 ? min((int)floor(v), q.H - 2) : 0;
    const int k0 = min((int)floor(w), q.K - 1);
    const float fu = (float)(u - i0), fv = (float)(v - j0), fw = (float)(w - floor(w));
    const int i1 = min(i0 + 1, q.W - 1), j1 = min(j0 + 1, q.H - 1), k1 = k0 + 1 == q.K ? 0 : k0 + 1;
    const int64_t plane = (int64_t)q.W * q.H;
    int64_t idx[2][2][2];
    const int ks[2] = {k0, k1}, js[2] = {j0, j1}, is[2] = {i0, i1};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e)
                idx[a][b][e] = ks[a] * plane + (int64_t)wrap(js[b] + q.ry, q.H) * q.W +
                               wrap(is[e] + q.rx, q.W);
    const float sx = in_u ? (float)(1.0 / q.res) : 0.f, sy = in_v ? (float)(1.0 / q.res) : 0.f;
    const float sw = (float)(1.0 / dth);
    float4 res[2];
    for (int f = 0; f < 2; ++f) {
        const float* g = f == 0 ? q.fa : q.fb;
        float o[4] = {0.f, 0.f, 0.f, 0.f};
        if (g) {
            float c[2][2][2];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int e = 0; e < 2; ++e) c[a][b][e] = g[idx[a][b][e]];
            trilinear(c, fu, fv, fw, o);
        }
        res[f] = make_float4(o[0], o[1] * sx, o[2] * sy, o[3] * sw);
    }
    // 32 bytes per pose, as two 16-byte stores (out is 16-byte aligned)
    float4* dst = reinterpret_cast<float4*>(q.out + 8 * n);
    dst[0] = res[0];
    dst[1] = res[1];
}

}  // namespace

hipError_t launch_sdf(const uint8_t* status, float* sdf, int W, int H, int K, int rx, int ry,
                      int cap, float res, int unknown_is_obstacle, hipStream_t stream) {
    SdfArgs a;
    a.status = status;
    a.sdf = sdf;
    a.W = W;
    a.H = H;
    a.K = K;
    a.rx = rx;
    a.ry = ry;
    a.cap = cap;
    a.res = res;
    a.unknown_is_obstacle = unknown_is_obstacle;
    const int TX = NT - 2 * cap;
    a.tiles_x = (W + TX - 1) / TX;
    // Taller strips share the column halo among more rows; shorter ones give
    // small maps enough workgroups.
    auto blocks = [&](int R) { return (int64_t)a.tiles_x * ((H + R - 1) / R); };
    const int R = blocks(32) * K >= 2048 ? 32 : blocks(16) * K >= 1024 ? 16 : 8;
    const dim3 grid((unsigned)blocks(R), K);
    if (R == 32) hipLaunchKernelGGL(sdf_kernel<32>, grid, dim3(NT), 0, stream, a);
    else if (R == 16) hipLaunchKernelGGL(sdf_kernel<16>, grid, dim3(NT), 0, stream, a);
    else hipLaunchKernelGGL(sdf_kernel<8>, grid, dim3(NT), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_query(const float* fa, const float* fb, const float* poses, float* out, int64_t n,
                        int W, int H, int K, int rx, int ry, double res, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    QueryArgs q;
    q.fa = fa;
    q.fb = fb;
    q.poses = poses;
    q.out = out;
    q.n = n;
    q.W = W;
    q.H = H;
    q.K = K;
    q.rx = rx;
    q.ry = ry;
    q.res = res;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, int64_t(1) << 20);
    hipLaunchKernelGGL(query_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, q);
    return hipGetLastError();
}

}  // namespace seb
