// SE(2) signed distance field of the obstacle states and the trilinear
// Risk / SDF query, for gfx950.
//
// The planner side of the method (Sec. VI-B, VI-C) needs, at every state, the
// distance to the edge of the nearest obstacle region (negative inside), and
// reads that field and the risk at arbitrary poses by trilinear interpolation
// with the yaw on SO(2).
//
// sdf_kernel: a workgroup owns a 32 x 32 block of cells of one yaw plane.  With
// distances capped at C cells, every target that matters lies within C cells
// in x and in y, so the block's flags with a C-cell halo are staged in LDS and
// the exact two-pass transform runs there: per column, the squared distance to
// the nearest obstacle (and nearest free) cell in that column within C rows;
// then per cell, the minimum over |dx| <= C of dx^2 plus the column value at
// x + dx.  Distances beyond C come out as C, as the cap asks.
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "seb.h"
#include "seb_sdf_internal.hpp"

namespace seb {
namespace {

constexpr int ST = 32;                    // block side (cells)
constexpr uint16_t FAR = 0xFFFF;          // no target within C rows
enum : uint8_t { FREE = 0, OBST = 1, OUTSIDE = 2 };

struct SdfArgs {
    const uint8_t* status;                // [K][H][W], ring layout
    float* sdf;                           // [K][H][W], ring layout
    int W, H, K, rx, ry;
    int cap;                              // C, cells
    float res;
    int unknown_is_obstacle;
};

__device__ __forceinline__ int wrap(int v, int n) { return v >= n ? v - n : v; }

__global__ __launch_bounds__(256) void sdf_kernel(const SdfArgs a) {
    extern __shared__ uint8_t lds[];
    const int C = a.cap;
    const int span = ST + 2 * C;
    uint8_t* flag = lds;                                          // [span][span]
    uint16_t* g_obs = (uint16_t*)(lds + ((span * span + 3) & ~3));  // [ST][span]
    uint16_t* g_free = g_obs + ST * span;                         // [ST][span]
    const int tid = threadIdx.x;
    const int bx = blockIdx.x, k = blockIdx.y;
    const int tiles_x = (a.W + ST - 1) / ST;
    const int x0 = (bx % tiles_x) * ST, y0 = (bx / tiles_x) * ST;
    const uint8_t* plane = a.status + (int64_t)k * a.W * a.H;

    for (int i = tid; i < span * span; i += 256) {
        const int r = i / span, c = i - r * span;
        const int y = y0 - C + r, x = x0 - C + c;
        uint8_t f = OUTSIDE;
        if (x >= 0 && x < a.W && y >= 0 && y < a.H) {
            const uint8_t st = plane[(int64_t)wrap(y + a.ry, a.H) * a.W + wrap(x + a.rx, a.W)];
            const bool obst = (st & (SEB_ST_CURV | SEB_ST_TILT)) != 0 ||
                              (a.unknown_is_obstacle && (st & SEB_ST_VALID) == 0);
            f = obst ? OBST : FREE;
        }
        flag[i] = f;
    }
    __syncthreads();

    // Column pass over the block's rows: nearest obstacle / free cell in the
    // same column within C rows, searched outwards.
    for (int i = tid; i < ST * span; i += 256) {
        const int r = i / span, c = i - r * span;
        const int rr = r + C;
        int dob = -1, dfr = -1;
        for (int d = 0; d <= C && (dob < 0 || dfr < 0); ++d) {
            const uint8_t up = flag[(rr - d) * span + c];
            const uint8_t dn = flag[(rr + d) * span + c];
            if (dob < 0 && (up == OBST || dn == OBST)) dob = d;
            if (dfr < 0 && (up == FREE || dn == FREE)) dfr = d;
        }
        g_obs[r * span + c] = dob < 0 ? FAR : (uint16_t)(dob * dob);
        g_free[r * span + c] = dfr < 0 ? FAR : (uint16_t)(dfr * dfr);
    }
    __syncthreads();

    // Row pass: per cell of the block, the nearest target among columns
    // x + dx, |dx| <= C, stopping once dx^2 alone reaches the best so far.
    for (int i = tid; i < ST * ST; i += 256) {
        const int r = i / ST, c = i - r * ST;
        const int x = x0 + c, y = y0 + r;
        if (x >= a.W || y >= a.H) continue;
        const uint8_t f = flag[(r + C) * span + (c + C)];
        const uint16_t* g = (f == OBST ? g_free : g_obs) + r * span + (c + C);
        int best = g[0] == FAR ? 0x7FFFFFFF : (int)g[0];
        for (int dx = 1; dx <= C && dx * dx < best; ++dx) {
            const int gl = g[-dx], gr = g[dx];
            if (gl != FAR) best = min(best, dx * dx + gl);
            if (gr != FAR) best = min(best, dx * dx + gr);
        }
        const float d = fminf(sqrtf((float)min(best, C * C)), (float)C);
        const float v = (d - 0.5f) * a.res;
        a.sdf[(int64_t)k * a.W * a.H + (int64_t)wrap(y + a.ry, a.H) * a.W + wrap(x + a.rx, a.W)] =
            f == OBST ? -v : v;
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

__global__ __launch_bounds__(256) void query_kernel(const QueryArgs q) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= q.n) return;
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
        float* dst = q.out + 8 * n + 4 * f;
        dst[0] = o[0];
        dst[1] = o[1] * sx;
        dst[2] = o[2] * sy;
        dst[3] = o[3] * sw;
    }
}

}  // namespace

int sdf_max_cap() { return 64; }

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
    const int span = ST + 2 * cap;
    const size_t lds = (size_t)((span * span + 3) & ~3) + (size_t)2 * ST * span * sizeof(uint16_t);
    const dim3 grid(((W + ST - 1) / ST) * ((H + ST - 1) / ST), K);
    hipLaunchKernelGGL(sdf_kernel, grid, dim3(256), lds, stream, a);
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
    hipLaunchKernelGGL(query_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, q);
    return hipGetLastError();
}

}  // namespace seb
