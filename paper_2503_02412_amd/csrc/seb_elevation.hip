// Elevation-map update before the assessment, for gfx950 (Sec. V-A).
//
// A scan's points are taken to the map frame, filtered (map range, body-frame
// height band) and given the variance of their height (Eq. 5-9).  The points
// of each map cell then update the cell's height and variance with a
// one-dimensional Kalman filter; several heights in one cell are handled by
// the classical elevation map's Mahalanobis test (a higher outlier replaces
// the cell, a lower one is dropped).  The fold over a cell's points is
// sequential by nature, so points are grouped by cell and each cell folds its
// own points in point order: a count per cell (atomics), an exclusive prefix
// sum, a scatter into per-cell buckets, then the fold: a cell with at most 8
// points is sorted and folded by one thread in registers; a larger one by a
// workgroup that places its points in LDS by rank (point index) and lets one
// thread fold them.  Every decision (the cell's floor, the
// height band, the gate) is taken in FP64 from the same operations, in the
// same order and without contraction, as the FP64 reference writes them.
//
// Before fusion, each point's ray from the sensor resets to unknown the known
// cells it crosses (its xy projection entering their interior), other than the
// point's own cell, that stand higher than the ray over the crossing.  A ray
// walks its cells with a DDA clipped to the window, also trying both
// neighbours where it passes within 1e-9 (in ray parameter) of a corner, and
// decides every candidate with the same slab clipping as the reference.  A
// reset writes NaN -- as a compare-and-swap when resets are counted, so each
// cell counts once -- and the result is a union that no ray order changes.
//
// Unknown cells can then be filled from the nearest known cell within a
// radius (nearest-neighbour inpainting, the method of the experiments), from
// an LDS tile with a halo of that radius and a list of offsets sorted by
// distance.
#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "seb_elevation_internal.hpp"

namespace seb {
namespace elev {
namespace {

constexpr int SMALL = 8;                  // points a thread folds alone, in registers
constexpr int CAP = 2048;                 // points a workgroup ranks in LDS

__global__ __launch_bounds__(256) void clear_kernel(int32_t* count, int32_t* fill, int64_t n,
                                                    int32_t* n_fused, int32_t* n_large) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        count[i] = 0;
        fill[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *n_fused = 0;
        *n_large = 0;
    }
}

// One point of the fold: the one-dimensional Kalman update with the
// several-heights rule.  Returns whether the point changed the cell.
__device__ __forceinline__ bool fold_point(double& h, double& v, double zi, double si, double tau2) {
#pragma clang fp contract(off)
    if (!isfinite(h)) {
        h = zi;
        v = si;
        return true;
    }
    const double dz = zi - h;
    if (dz * dz > tau2 * v) {
        if (zi > h) {
            h = zi;
            v = si;
            return true;
        }
        return false;
    }
    h = (v * zi + si * h) / (v + si);
    v = (v * si) / (v + si);
    return true;
}

__global__ __launch_bounds__(256) void points_kernel(const ScanArgs s, FuseWork w) {
#pragma clang fp contract(off)
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < s.n; i += stride) {
        const double px = s.pts[3 * i], py = s.pts[3 * i + 1], pz = s.pts[3 * i + 2];
        // body frame q = R_BS p + p_BS, map frame l = R_B q + p_B
        const double q0 = s.A[0] * px + s.A[1] * py + s.A[2] * pz + s.a[0];
        const double q1 = s.A[3] * px + s.A[4] * py + s.A[5] * pz + s.a[1];
        const double q2 = s.A[6] * px + s.A[7] * py + s.A[8] * pz + s.a[2];
        const double lx = s.R[0] * q0 + s.R[1] * q1 + s.R[2] * q2 + s.b[0];
        const double ly = s.R[3] * q0 + s.R[4] * q1 + s.R[5] * q2 + s.b[1];
        const double lz = s.R[6] * q0 + s.R[7] * q1 + s.R[8] * q2 + s.b[2];
        // Eq. 9 with the sensor model written without square roots
        const double jp = s.js[0] * px + s.js[1] * py + s.js[2] * pz;
        const double r2 = px * px + py * py + pz * pz;
        const double sensor = r2 > 0.0 ? s.sr2 * (jp * jp) / r2 + s.sa2 * (r2 - jp * jp) : s.sr2;
        const double k0 = q1 * s.g[2] - q2 * s.g[1];
        const double k1 = q2 * s.g[0] - q0 * s.g[2];
        const double k2 = q0 * s.g[1] - q1 * s.g[0];
        const double rot = k0 * (s.SR[0] * k0 + s.SR[1] * k1 + s.SR[2] * k2) +
                           k1 * (s.SR[3] * k0 + s.SR[4] * k1 + s.SR[5] * k2) +
                           k2 * (s.SR[6] * k0 + s.SR[7] * k1 + s.SR[8] * k2);
        const double var = sensor + rot + s.sb22;
        const double cx = floor(lx / s.res) - (double)s.ox;
        const double cy = floor(ly / s.res) - (double)s.oy;
        const bool keep = q2 >= s.zmin && q2 <= s.zmax && cx >= 0.0 && cx < (double)s.W &&
                          cy >= 0.0 && cy < (double)s.H && isfinite(lz);
        int32_t c = -1;
        if (keep) {
            c = (int32_t)cy * s.W + (int32_t)cx;
            atomicAdd(&w.count[c], 1);
        }
        w.cell[i] = c;
        w.z[i] = lz;
        w.var[i] = var;
    }
}

// Exclusive prefix sum of count[0, n) into offs, in three passes: block sums,
// a scan of the block sums, and a local scan of each block with its offset.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* lds, int32_t* total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int32_t add = t >= d ? lds[t - d] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const int32_t incl = lds[t];
    *total = lds[255];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void block_sums_kernel(const int32_t* count, int64_t n,
                                                         int32_t* partial) {
    __shared__ int32_t lds[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 16;
    int32_t s = 0;
    for (int u = 0; u < 16; ++u)
        if (base + u < n) s += count[base + u];
    int32_t total;
    block_exclusive_scan(s, lds, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void scan_partials_kernel(int32_t* partial, int64_t nb) {
    __shared__ int32_t lds[256];
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int32_t v = i < nb ? partial[i] : 0;
        int32_t total;
        const int32_t ex = block_exclusive_scan(v, lds, &total);
        if (i < nb) partial[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(256) void local_scan_kernel(const int32_t* count, int64_t n,
                                                         const int32_t* partial, int32_t* offs) {
    __shared__ int32_t lds[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 16;
    int32_t v[16], s = 0;
    for (int u = 0; u < 16; ++u) {
        v[u] = base + u < n ? count[base + u] : 0;
        s += v[u];
    }
    int32_t total;
    int32_t run = partial[blockIdx.x] + block_exclusive_scan(s, lds, &total);
    for (int u = 0; u < 16; ++u) {
        if (base + u < n) offs[base + u] = run;
        run += v[u];
    }
}

__global__ __launch_bounds__(256) void scatter_kernel(int64_t n, FuseWork w) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const int32_t c = w.cell[i];
        if (c >= 0) w.bucket[w.offs[c] + atomicAdd(&w.fill[c], 1)] = (int32_t)i;
    }
}

// In-place ascending sort of a cell's point indices: insertion sort for short
// buckets, heapsort (no extra memory, n log n) for long ones.
__device__ void sort_bucket(int32_t* b, int n) {
    if (n <= 32) {
        for (int i = 1; i < n; ++i) {
            const int32_t v = b[i];
            int j = i - 1;
            while (j >= 0 && b[j] > v) {
                b[j + 1] = b[j];
                --j;
            }
            b[j + 1] = v;
        }
        return;
    }
    auto sift = [&](int root, int end) {
        while (2 * root + 1 < end) {
            int child = 2 * root + 1;
            if (child + 1 < end && b[child] < b[child + 1]) ++child;
            if (b[root] >= b[child]) return;
            const int32_t t = b[root];
            b[root] = b[child];
            b[child] = t;
            root = child;
        }
    };
    for (int i = n / 2 - 1; i >= 0; --i) sift(i, n);
    for (int end = n - 1; end > 0; --end) {
        const int32_t t = b[0];
        b[0] = b[end];
        b[end] = t;
        sift(0, end);
    }
}

__global__ __launch_bounds__(256) void fuse_small_kernel(const FuseArgs f, FuseWork w) {
    __shared__ int32_t used_lds[256];
    const int64_t n_cells = (int64_t)f.W * f.H;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int32_t used = 0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n_cells; c += stride) {
        const int n = w.count[c];
        if (n == 0) continue;
        if (n > SMALL) {
            w.large[atomicAdd(w.n_large, 1)] = (int32_t)c;
            continue;
        }
        // indices (clamped loads, then padding), sorted by an odd-even
        // transposition network, then every (z, var) load at once
        const int32_t* b = w.bucket + w.offs[c];
        int32_t idx[SMALL];
#pragma unroll
        for (int k = 0; k < SMALL; ++k) {
            const int32_t v = b[min(k, n - 1)];
            idx[k] = k < n ? v : INT32_MAX;
        }
#pragma unroll
        for (int r = 0; r < SMALL; ++r) {
#pragma unroll
            for (int k = r & 1; k + 1 < SMALL; k += 2) {
                const int32_t lo = min(idx[k], idx[k + 1]), hi = max(idx[k], idx[k + 1]);
                idx[k] = lo;
                idx[k + 1] = hi;
            }
        }
        double zs[SMALL], ss[SMALL];
#pragma unroll
        for (int k = 0; k < SMALL; ++k) {
            const int32_t i = idx[k < n ? k : 0];
            zs[k] = w.z[i];
            ss[k] = w.var[i];
        }
        const int lx = (int)(c % f.W), ly = (int)(c / f.W);
        const int64_t at = (int64_t)((ly + f.ry) % f.H) * f.ld + (lx + f.rx) % f.W;
        double h = (double)f.height[at], v = (double)f.variance[at];
#pragma unroll
        for (int k = 0; k < SMALL; ++k)
            if (k < n) used += fold_point(h, v, zs[k], ss[k], f.tau2);
        f.height[at] = (float)h;
        f.variance[at] = (float)v;
    }
    int32_t total;
    block_exclusive_scan(used, used_lds, &total);
    if (threadIdx.x == 0 && total) atomicAdd(f.n_fused, total);
}

// A workgroup per listed cell.  Point indices are distinct, so a point's rank
// among its cell's indices is its place in the fold.
__global__ __launch_bounds__(256) void fuse_large_kernel(const FuseArgs f, FuseWork w) {
    __shared__ int32_t keys[CAP];
    __shared__ double zs[CAP], ss[CAP];
    const int n_large = *w.n_large;
    for (int li = blockIdx.x; li < n_large; li += gridDim.x) {
        const int32_t c = w.large[li];
        const int n = w.count[c];
        int32_t* b = w.bucket + w.offs[c];
        if (n <= CAP) {
            for (int e = threadIdx.x; e < n; e += 256) keys[e] = b[e];
            __syncthreads();
            for (int e = threadIdx.x; e < n; e += 256) {
                const int32_t k = keys[e];
                int rank = 0;
                for (int j = 0; j < n; ++j) rank += keys[j] < k;
                zs[rank] = w.z[k];
                ss[rank] = w.var[k];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (n > CAP) sort_bucket(b, n);            // rare: in place in HBM
            const int lx = c % f.W, ly = c / f.W;
            const int64_t at = (int64_t)((ly + f.ry) % f.H) * f.ld + (lx + f.rx) % f.W;
            double h = (double)f.height[at], v = (double)f.variance[at];
            int32_t used = 0;
            if (n <= CAP) {
                // the next point's (z, var) is read from LDS while this one
                // folds, so its latency hides behind the divisions
                double zn = n > 0 ? zs[0] : 0.0, sn = n > 0 ? ss[0] : 0.0;
                for (int k = 0; k < n; ++k) {
                    const double zi = zn, si = sn;
                    if (k + 1 < n) {
                        zn = zs[k + 1];
                        sn = ss[k + 1];
                    }
                    used += fold_point(h, v, zi, si, f.tau2);
                }
            } else {
                for (int k = 0; k < n; ++k) used += fold_point(h, v, w.z[b[k]], w.var[b[k]], f.tau2);
            }
            f.height[at] = (float)h;
            f.variance[at] = (float)v;
            if (used) atomicAdd(f.n_fused, used);
        }
        __syncthreads();
    }
}

// Parameter interval of s + t d inside cell c along one axis.
__device__ __forceinline__ void slab(int64_t c, double res, double s, double d, double& lo,
                                     double& hi) {
#pragma clang fp contract(off)
    const double e0 = (double)c * res, e1 = ((double)c + 1.0) * res;
    if (d != 0.0) {
        const double t1 = (e0 - s) / d, t2 = (e1 - s) / d;
        lo = fmin(t1, t2);
        hi = fmax(t1, t2);
    } else {
        const bool in = e0 <= s && s < e1;
        lo = in ? -INFINITY : INFINITY;
        hi = in ? INFINITY : -INFINITY;
    }
}

struct Ray {
    double dx, dy, dz;
    int64_t ei, ej;          // the point's own cell
    int64_t i0, i1, j0, j1;  // cells between the sensor's and the point's
};

__device__ __forceinline__ int ray_cell(const RayArgs& r, const Ray& q, int64_t i, int64_t j) {
#pragma clang fp contract(off)
    if (i < r.ox || i >= r.ox + r.W || j < r.oy || j >= r.oy + r.H) return 0;
    if (i < q.i0 || i > q.i1 || j < q.j0 || j > q.j1) return 0;
    if (i == q.ei && j == q.ej) return 0;
    double xlo, xhi, ylo, yhi;
    slab(i, r.res, r.sx, q.dx, xlo, xhi);
    slab(j, r.res, r.sy, q.dy, ylo, yhi);
    const double t0 = fmax(fmax(xlo, ylo), 0.0);
    const double t1 = fmin(fmin(xhi, yhi), 1.0);
    if (!(t1 > t0)) return 0;
    const double zmax = fmax(r.sz + t0 * q.dz, r.sz + t1 * q.dz);
    const int lx = (int)(i - r.ox), ly = (int)(j - r.oy);
    float* p = r.height + (int64_t)((ly + r.ry) % r.H) * r.ld + (lx + r.rx) % r.W;
    const float h = *p;
    if (!((double)h > zmax + r.margin)) return 0;
    if (!r.n_reset) {                        // no count wanted: the store is idempotent
        *p = __builtin_nanf("");
        return 0;
    }
    const unsigned int old = __float_as_uint(h);
    return atomicCAS(reinterpret_cast<unsigned int*>(p), old, 0x7FC00000u) == old;
}

__global__ __launch_bounds__(256) void zero_kernel(int32_t* v) { *v = 0; }

constexpr int RAY_PARTS = 8;

__global__ __launch_bounds__(256) void raycast_kernel(const RayArgs r) {
#pragma clang fp contract(off)
    __shared__ int32_t cnt_lds[256];
    const int64_t stride = (int64_t)gridDim.x * 256;
    const double X0 = (double)r.ox * r.res, X1 = (double)(r.ox + r.W) * r.res;
    const double Y0 = (double)r.oy * r.res, Y1 = (double)(r.oy + r.H) * r.res;
    int32_t count = 0;
    // Work item w walks part w % RAY_PARTS of ray w / RAY_PARTS (adjacent lanes
    // share a ray), so that a wave waits on the longest part of a ray, not on
    // the longest ray (2, 4 and 8 parts measured 0.29, 0.26 and 0.245 ms
    // against 0.36 ms for whole rays on a 190k-ray scan).
    for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < r.n * RAY_PARTS; w += stride) {
        const int64_t n = w / RAY_PARTS;
        const int part = (int)(w - n * RAY_PARTS);
        const double px = r.pts[3 * n], py = r.pts[3 * n + 1], pz = r.pts[3 * n + 2];
        const double q0 = r.A[0] * px + r.A[1] * py + r.A[2] * pz + r.a[0];
        const double q1 = r.A[3] * px + r.A[4] * py + r.A[5] * pz + r.a[1];
        const double q2 = r.A[6] * px + r.A[7] * py + r.A[8] * pz + r.a[2];
        const double lx = r.R[0] * q0 + r.R[1] * q1 + r.R[2] * q2 + r.b[0];
        const double ly = r.R[3] * q0 + r.R[4] * q1 + r.R[5] * q2 + r.b[1];
        const double lz = r.R[6] * q0 + r.R[7] * q1 + r.R[8] * q2 + r.b[2];
        if (!isfinite(lx) || !isfinite(ly) || !isfinite(lz)) continue;
        Ray q;
        q.dx = lx - r.sx;
        q.dy = ly - r.sy;
        q.dz = lz - r.sz;
        const double big = 1e15;
        q.ei = (int64_t)fmin(fmax(floor(lx / r.res), -big), big);
        q.ej = (int64_t)fmin(fmax(floor(ly / r.res), -big), big);
        const int64_t si = (int64_t)floor(r.sx / r.res), sj = (int64_t)floor(r.sy / r.res);
        q.i0 = min(si, q.ei);
        q.i1 = max(si, q.ei);
        q.j0 = min(sj, q.ej);
        q.j1 = max(sj, q.ej);
        // the part of the segment inside the window, [ta, tb]
        double ta = 0.0, tb = 1.0;
        if (q.dx != 0.0) {
            const double t1 = (X0 - r.sx) / q.dx, t2 = (X1 - r.sx) / q.dx;
            ta = fmax(ta, fmin(t1, t2));
            tb = fmin(tb, fmax(t1, t2));
        } else if (!(X0 <= r.sx && r.sx < X1)) {
            continue;
        }
        if (q.dy != 0.0) {
            const double t1 = (Y0 - r.sy) / q.dy, t2 = (Y1 - r.sy) / q.dy;
            ta = fmax(ta, fmin(t1, t2));
            tb = fmin(tb, fmax(t1, t2));
        } else if (!(Y0 <= r.sy && r.sy < Y1)) {
            continue;
        }
        if (!(tb >= ta)) continue;
        // This part's share [tl, th] of [ta, tb].  It starts from the cell that
        // holds the point at tl and, like the whole walk, stops once both next
        // crossings lie past its end: the parts overlap at their ends, so every
        // cell the whole walk would try is tried by some part (a cell tried
        // twice gets the same decision).
        const double tl = ta + (tb - ta) * ((double)part / RAY_PARTS);
        const double th = part + 1 == RAY_PARTS ? tb : ta + (tb - ta) * ((double)(part + 1) / RAY_PARTS);
        const double xa = r.sx + tl * q.dx, ya = r.sy + tl * q.dy;
        int64_t i = (int64_t)floor(xa / r.res), j = (int64_t)floor(ya / r.res);
        i = i < r.ox ? r.ox : (i >= r.ox + r.W ? r.ox + r.W - 1 : i);
        j = j < r.oy ? r.oy : (j >= r.oy + r.H ? r.oy + r.H - 1 : j);
        const int step_x = q.dx > 0.0 ? 1 : (q.dx < 0.0 ? -1 : 0);
        const int step_y = q.dy > 0.0 ? 1 : (q.dy < 0.0 ? -1 : 0);
        double tmx = q.dx != 0.0 ? ((double)(i + (step_x > 0)) * r.res - r.sx) / q.dx : INFINITY;
        double tmy = q.dy != 0.0 ? ((double)(j + (step_y > 0)) * r.res - r.sy) / q.dy : INFINITY;
        const double tdx = q.dx != 0.0 ? r.res / fabs(q.dx) : INFINITY;
        const double tdy = q.dy != 0.0 ? r.res / fabs(q.dy) : INFINITY;
        for (int s = 0; s < r.W + r.H + 4; ++s) {
            count += ray_cell(r, q, i, j);
            if (fabs(tmx - tmy) <= 1e-9) {       // near a corner: both neighbours
                count += ray_cell(r, q, i + step_x, j);
                count += ray_cell(r, q, i, j + step_y);
            }
            if (fmin(tmx, tmy) > th + 1e-9) break;
            if (tmx < tmy) {
                i += step_x;
                tmx += tdx;
            } else {
                j += step_y;
                tmy += tdy;
            }
            if (i < r.ox || i >= r.ox + r.W || j < r.oy || j >= r.oy + r.H) break;
        }
    }
    if (r.n_reset) {
        int32_t total;
        block_exclusive_scan(count, cnt_lds, &total);
        if (threadIdx.x == 0 && total) atomicAdd(r.n_reset, total);
    }
}

constexpr int IT = 32;                                  // inpaint tile side
constexpr int ISPAN = IT + 2 * INPAINT_MAX_RADIUS;      // 64

__global__ __launch_bounds__(256) void inpaint_kernel(const InpaintArgs a) {
    __shared__ float tile[ISPAN * ISPAN];
    __shared__ int lin[INPAINT_MAX_OFFS];                 // offsets as tile index steps
    const int r = a.radius, span = IT + 2 * r;
    for (int k = threadIdx.x; k < a.n_offs; k += 256) lin[k] = a.offs[k].y * span + a.offs[k].x;
    const int tiles_x = (a.W + IT - 1) / IT;
    const int x0 = (blockIdx.x % tiles_x) * IT, y0 = (blockIdx.x / tiles_x) * IT;
    // Loads from coordinates clamped into the map, the out-of-map test after.
    for (int i = threadIdx.x; i < span * span; i += 256) {
        const int rr = i / span, cc = i - rr * span;
        const int y = y0 - r + rr, x = x0 - r + cc;
        const int yc = min(max(y, 0), a.H - 1), xc = min(max(x, 0), a.W - 1);
        const float v = a.src[(int64_t)((yc + a.ry) % a.H) * a.ld + (xc + a.rx) % a.W];
        const bool in = x >= 0 && x < a.W && y >= 0 && y < a.H;
        tile[i] = in && isfinite(v) ? v : __builtin_nanf("");
    }
    __syncthreads();
    for (int i = threadIdx.x; i < IT * IT; i += 256) {
        const int ly = i / IT, lx = i - ly * IT;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= a.W || y >= a.H) continue;
        const int at = (ly + r) * span + lx + r;
        float v = tile[at];
        if (v != v) {
            for (int k = 0; k < a.n_offs; ++k) {
                const float t = tile[at + lin[k]];
                if (t == t) {
                    v = t;
                    break;
                }
            }
        }
        a.dst[(int64_t)((y + a.ry) % a.H) * a.dst_ld + (x + a.rx) % a.W] = v;
    }
}

}  // namespace

hipError_t launch_fuse_scan(const ScanArgs& s, const FuseArgs& f, const FuseWork& w,
                            hipStream_t stream) {
    const int64_t n_cells = (int64_t)f.W * f.H;
    const int64_t nb = partial_blocks(n_cells);
    auto grid = [](int64_t items) {
        return dim3((unsigned)std::min<int64_t>(std::max<int64_t>((items + 255) / 256, 1), 8192));
    };
    hipLaunchKernelGGL(clear_kernel, grid(n_cells), dim3(256), 0, stream, w.count, w.fill, n_cells,
                       f.n_fused, w.n_large);
    if (s.n > 0) hipLaunchKernelGGL(points_kernel, grid(s.n), dim3(256), 0, stream, s, w);
    hipLaunchKernelGGL(block_sums_kernel, dim3((unsigned)nb), dim3(256), 0, stream, w.count,
                       n_cells, w.partial);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(256), 0, stream, w.partial, nb);
    hipLaunchKernelGGL(local_scan_kernel, dim3((unsigned)nb), dim3(256), 0, stream, w.count,
                       n_cells, w.partial, w.offs);
    if (s.n > 0) hipLaunchKernelGGL(scatter_kernel, grid(s.n), dim3(256), 0, stream, s.n, w);
    hipLaunchKernelGGL(fuse_small_kernel, grid(n_cells), dim3(256), 0, stream, f, w);
    hipLaunchKernelGGL(fuse_large_kernel, dim3(8192), dim3(256), 0, stream, f, w);
    return hipGetLastError();
}

// Workspace of seb_fuse_scan_static: one file-scope array per device (each
// GPU the library runs on holds its own copy until the process ends), carved
// into the FuseWork buffers for up to STATIC_MAX_POINTS points and
// STATIC_MAX_CELLS map cells.  Host code never passes the array's name to a
// kernel (there it is a host-side stand-in); it uses the device address that
// static_fuse_work looks up once per device.
namespace {
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t STATIC_PARTIALS = (STATIC_MAX_CELLS + SCAN_CHUNK - 1) / SCAN_CHUNK;
constexpr size_t STATIC_BYTES =
    2 * align256((size_t)STATIC_MAX_POINTS * 4) + 2 * align256((size_t)STATIC_MAX_POINTS * 8) +
    4 * align256((size_t)STATIC_MAX_CELLS * 4) + align256(STATIC_PARTIALS * 4) + 2 * 256;
static_assert(STATIC_BYTES <= (size_t)16 << 20, "static fusion workspace above 16 MiB");
__device__ __align__(256) unsigned char scratch[STATIC_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};     // device address of scratch, per device ordinal
}  // namespace

hipError_t static_fuse_work(FuseWork* w) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    unsigned char* base;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!ptr) return hipErrorInvalidSymbol;
            g_scratch_ptr[dev] = ptr;
        }
        base = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    }
    size_t o = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base + o;
        o += align256(bytes);
        return p;
    };
    w->cell = (int32_t*)take((size_t)STATIC_MAX_POINTS * 4);
    w->bucket = (int32_t*)take((size_t)STATIC_MAX_POINTS * 4);
    w->z = (double*)take((size_t)STATIC_MAX_POINTS * 8);
    w->var = (double*)take((size_t)STATIC_MAX_POINTS * 8);
    w->count = (int32_t*)take((size_t)STATIC_MAX_CELLS * 4);
    w->fill = (int32_t*)take((size_t)STATIC_MAX_CELLS * 4);
    w->offs = (int32_t*)take((size_t)STATIC_MAX_CELLS * 4);
    w->large = (int32_t*)take((size_t)STATIC_MAX_CELLS * 4);
    w->partial = (int32_t*)take(STATIC_PARTIALS * 4);
    w->n_large = (int32_t*)take(4);
    w->n_fused = (int32_t*)take(4);
    return o <= STATIC_BYTES ? hipSuccess : hipErrorInvalidValue;
}

hipError_t launch_raycast(const RayArgs& r, hipStream_t stream) {
    if (r.n_reset) hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(1), 0, stream, r.n_reset);
    if (r.n > 0) {
        const unsigned blocks = (unsigned)std::min<int64_t>((r.n * RAY_PARTS + 255) / 256, 16384);
        hipLaunchKernelGGL(raycast_kernel, dim3(blocks), dim3(256), 0, stream, r);
    }
    return hipGetLastError();
}

hipError_t launch_inpaint(const InpaintArgs& a, hipStream_t stream) {
    const int tiles = ((a.W + IT - 1) / IT) * ((a.H + IT - 1) / IT);
    hipLaunchKernelGGL(inpaint_kernel, dim3((unsigned)tiles), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace elev
}  // namespace seb
