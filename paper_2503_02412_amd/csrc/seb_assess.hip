// HIP kernels for gfx950: SE(2)-grid traversability assessment (Sec. V-B,
// Algorithm 1, with the pose of Sec. III, Eq. 1-3) and rolling-window cell
// insertion (Sec. V-A).
//
// Work decomposition.  A workgroup stages the heights of a 16 x 16 block of
// states plus an R-cell halo into LDS once, then loops over yaw bins; each
// lane owns one state (cell) and walks the footprint samples of the current
// yaw bin in table order.  The table entry of a sample (LDS offset, bilinear
// weights, body coordinates) is the same for every lane, so the whole wave
// reads it with scalar loads and the FMAs take it as a scalar operand.  Lanes
// map to 16 consecutive x-cells of 4 rows, which with a row pitch of 16 mod 32
// floats keeps every LDS read conflict-free.
//
// Yaw bins k and k + K/2 sample exactly the same map points with body
// coordinates negated, so one pass yields both: height, curvature, tilt and
// risk are shared, roll and pitch change sign.
//
// Per-state arithmetic.  Heights are centred on a per-state reference (the
// state's own cell, else the first valid sample in table order) before the
// moments are summed in FP32.  The exact integer moments of the valid sample
// positions (N, sum p, sum q, sum p^2, sum pq, sum q^2) give an exact gate
// (enough samples, not collinear) and exact centred second moments; the
// least-squares plane is then a closed-form 2 x 2 solve.
#include <cmath>

#include "../../include/seb.h"
#include "seb_internal.hpp"

namespace seb {
namespace {

template <typename T>
struct Moments {
    T Sz, Spz, Sqz, Szz;          // sums over valid samples of z, p z, q z, z^2 (z centred)
    int32_t N, Sp, Sq, Spp, Spq, Sqq;
};

struct Result {
    float z, roll, pitch, risk;
    uint8_t st;
};

__device__ __forceinline__ int wrap(int v, int n) { return v >= n ? v - n : v; }

// The footprint table is read-only for the lifetime of a launch.  Reading it
// through the constant address space lets the compiler fetch wave-uniform
// entries with scalar loads even though the kernel also stores to global memory.
// (The host compilation pass of this file only parses the kernels, so there
// the qualifier is dropped.)
#if defined(__HIP_DEVICE_COMPILE__)
#define SEB_CONSTANT_AS __attribute__((address_space(4)))
#else
#define SEB_CONSTANT_AS
#endif
template <typename T>
using cptr = const SEB_CONSTANT_AS T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)(p);
}

// Least-squares plane z = a + b u + c v from the moments, then Eq. 1-3 and
// Algorithm 1.  u = hu p, v = hv q are the body-frame sample coordinates.
template <typename T>
__device__ Result finish(const AssessArgs& a, const Moments<T>& m, T ref) {
    Result r;
    const int64_t N = m.N;
    const int64_t D = N * (int64_t)m.Spp - (int64_t)m.Sp * m.Sp;
    const int64_t E = N * (int64_t)m.Sqq - (int64_t)m.Sq * m.Sq;
    const int64_t F = N * (int64_t)m.Spq - (int64_t)m.Sp * m.Sq;
    const int64_t det = D * E - F * F;
    if (N < a.min_valid || det <= 0) {
        r.z = r.roll = r.pitch = __builtin_nanf("");
        r.risk = 1.f;
        r.st = 0;
        return r;
    }
    uint8_t st = SEB_ST_VALID;
    const double de = (double)(D + E);
    if (2 * N < a.n_total || (4.0 * (double)det) / (de * de) < a.rho16) st |= SEB_ST_DEGEN;

    const T invN = T(1) / T(N);
    const T zb = m.Sz * invN;
    const T pz = m.Spz - T(m.Sp) * zb;      // sum (p - pbar)(z - zbar)
    const T qz = m.Sqz - T(m.Sq) * zb;
    const T zz = m.Szz - m.Sz * zb;         // sum (z - zbar)^2
    const T tdet = T(det);
    const T bp = T(N) * (T(E) * pz - T(F) * qz) / tdet;   // dz/dp
    const T bq = T(N) * (T(D) * qz - T(F) * pz) / tdet;   // dz/dq
    const T b = bp / T(a.hu), c = bq / T(a.hv);           // dz/du, dz/dv
    const T zc = ref + zb - bp * (T(m.Sp) * invN) - bq * (T(m.Sq) * invN);
    T sse = zz - bp * pz - bq * qz;
    if (sse < T(0)) sse = T(0);
    const T s2 = T(1) + b * b + c * c;
    const T tr = T(a.hu) * T(a.hu) * T(D) * invN + T(a.hv) * T(a.hv) * T(E) * invN + zz;
    const float kappa = (tr > T(0)) ? (float)(sse / (s2 * tr)) : 0.f;

    const float bf = (float)b, cf = (float)c;
    const float c1 = 1.f + cf * cf;
    r.z = (float)zc;
    r.roll = atanf(cf);                              // asin(b3 . y_b)
    r.pitch = -atan2f(bf, sqrtf(c1));               // atan2(-b3 . x_b, b3 . z_b)
    const float phx = atan2f(fabsf(bf), sqrtf(c1 * c1 + bf * bf * cf * cf));   // |asin(b3 . x_b)|
    const float phy = fabsf(r.roll);                                             // |asin(b3 . y_b)|
    float risk;
    if (kappa > a.kappa_max) {
        risk = 1.f;
        st |= SEB_ST_CURV;
    } else if (phx > a.phi_x_max || phy > a.phi_y_max) {
        risk = 1.f;
        st |= SEB_ST_TILT;
    } else {
        risk = a.w_kappa * kappa / a.kappa_max + a.w_phi_x * phx / a.phi_x_max +
               a.w_phi_y * phy / a.phi_y_max;
    }
    if (risk <= a.risk_max) st |= SEB_ST_TRAV;
    r.risk = risk;
    r.st = st;
    return r;
}

// Bilinear sample of the lane's state, centred on ref.  Corner weights are
// wave-uniform scalars; the four heights come from two paired LDS reads.
template <int P>
__device__ __forceinline__ float sample(const float* tp0, int off, float4 w, float ref) {
    const float* tp = tp0 + off;
    float z = fmaf(w.x, tp[0], -ref);
    z = fmaf(w.y, tp[1], z);
    z = fmaf(w.z, tp[P], z);
    return fmaf(w.w, tp[P + 1], z);
}

// Per-segment integer moments: (count, sum q, sum q^2) unpacked from pk and
// combined with the segment's body-x index p.
__device__ __forceinline__ void add_segment(Moments<float>& m, int p, uint32_t pk, int qoff,
                                            uint32_t mask1, int sh2, float rz) {
    const int c = (int)(pk & 63u);
    const int Q = (int)((pk >> 6) & mask1) - qoff * c;
    const int QQ = (int)(pk >> sh2);
    m.N += c;
    m.Sp += p * c;
    m.Spp += p * p * c;
    m.Sq += Q;
    m.Spq += p * Q;
    m.Sqq += QQ;
    m.Sz += rz;
    m.Spz = fmaf((float)p, rz, m.Spz);
}

constexpr int bits_for(int v) {
    int b = 0;
    while ((1 << b) <= v) ++b;
    return b;
}

// FP32 moments of one yaw bin when every segment is a full row of NW samples:
// the row loop is unrolled, so q and the packed integer constants of each
// sample are literals and only the weights and offsets are loaded.
template <int P, int NW>
__device__ __forceinline__ void accumulate_rows(const AssessArgs& a, const float* tp0,
                                                cptr<float4> W, cptr<int32_t> O, float ref,
                                                Moments<float>& m) {
    constexpr int kQoff = NW - 1;
    constexpr int kSh2 = 6 + bits_for(NW * 2 * kQoff);
    constexpr uint32_t kMask1 = (1u << (kSh2 - 6)) - 1u;
    static_assert(kSh2 + bits_for(NW * kQoff * kQoff) <= 32, "packed moments overflow");
    m.Sz = m.Spz = m.Sqz = m.Szz = 0.f;
    m.N = m.Sp = m.Sq = m.Spp = m.Spq = m.Sqq = 0;
    const int nrows = a.n_segs;
    int p = 1 - nrows;
    for (int i = 0; i < nrows; ++i, p += 2) {
        float rz = 0.f;
        uint32_t pk = 0u;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const float z = sample<P>(tp0, O[i * NW + j], W[i * NW + j], ref);
            if (fabsf(z) < VALID_LIMIT) {
                const int q = 2 * j - kQoff;
                rz += z;
                m.Sqz = fmaf((float)q, z, m.Sqz);
                m.Szz = fmaf(z, z, m.Szz);
                pk += 1u | ((uint32_t)(2 * j) << 6) | ((uint32_t)(q * q) << kSh2);
            }
        }
        add_segment(m, p, pk, kQoff, kMask1, kSh2, rz);
    }
}

// FP32 moments of one yaw bin, any footprint (segments of any length).
template <int P>
__device__ __forceinline__ void accumulate_segments(const AssessArgs& a, const float* tp0,
                                                    cptr<float4> W, cptr<int32_t> O, float ref,
                                                    Moments<float>& m) {
    m.Sz = m.Spz = m.Sqz = m.Szz = 0.f;
    m.N = m.Sp = m.Sq = m.Spp = m.Spq = m.Sqq = 0;
    const cptr<Segment> segs = as_const(a.segs);
    const cptr<float> qs = as_const(a.qs);
    const cptr<uint32_t> pks = as_const(a.pks);
    for (int g = 0; g < a.n_segs; ++g) {
        const Segment sg = segs[g];
        float rz = 0.f;
        uint32_t pk = 0u;
        for (int s = sg.first; s < sg.first + sg.count; ++s) {
            const float z = sample<P>(tp0, O[s], W[s], ref);
            if (fabsf(z) < VALID_LIMIT) {
                rz += z;
                m.Sqz = fmaf(qs[s], z, m.Sqz);
                m.Szz = fmaf(z, z, m.Szz);
                pk += pks[s];
            }
        }
        add_segment(m, sg.p, pk, a.qoff, a.mask1, a.sh2, rz);
    }
}

// FP64 moments of one yaw bin, with FP64 bilinear weights (near-degenerate path).
template <int P>
__device__ void accumulate64(const AssessArgs& a, const float* tp0, cptr<int32_t> O,
                             cptr<double2> FR, double ref, Moments<double>& m) {
    m.Sz = m.Spz = m.Sqz = m.Szz = 0.0;
    m.N = m.Sp = m.Sq = m.Spp = m.Spq = m.Sqq = 0;
    const cptr<Segment> segs = as_const(a.segs);
    const cptr<float> qs = as_const(a.qs);
    for (int g = 0; g < a.n_segs; ++g) {
        const Segment sg = segs[g];
        double rz = 0.0;
        for (int s = sg.first; s < sg.first + sg.count; ++s) {
            const double2 f = FR[s];
            const float* tp = tp0 + O[s];
            const double gx = 1.0 - f.x, gy = 1.0 - f.y;
            const double z = gx * gy * (double)tp[0] + f.x * gy * (double)tp[1] +
                             gx * f.y * (double)tp[P] + f.x * f.y * (double)tp[P + 1] - ref;
            if (fabs(z) < (double)VALID_LIMIT) {
                const int q = (int)qs[s];
                rz += z;
                m.Sqz += (double)q * z;
                m.Szz += z * z;
                m.N += 1;
                m.Sq += q;
                m.Sqq += q * q;
                m.Sp += sg.p;
                m.Spp += sg.p * sg.p;
                m.Spq += sg.p * q;
            }
        }
        m.Sz += rz;
        m.Spz += (double)sg.p * rz;
    }
}

__device__ __forceinline__ void store(const AssessArgs& a, int k, int64_t cell, const Result& r,
                                      bool negate) {
    const int64_t o = (int64_t)k * a.H * a.W + cell;
    a.z[o] = r.z;
    a.roll[o] = negate ? -r.roll : r.roll;
    a.pitch[o] = negate ? -r.pitch : r.pitch;
    a.risk[o] = r.risk;
    a.status[o] = r.st;
}

template <int P, int NW>
__global__ __launch_bounds__(BLOCK) void assess_kernel(const AssessArgs a) {
    extern __shared__ float tile[];
    const int tid = threadIdx.x;

    // Which rectangle and which tile of it.
    const int b = blockIdx.x;
    int ri = 0;
    while (ri + 1 < a.n_rects && b >= a.tile_start[ri + 1]) ++ri;
    const int lb = b - a.tile_start[ri];
    const int tyi = lb / a.tiles_x[ri];
    const int txi = lb - tyi * a.tiles_x[ri];
    const int sx0 = a.rect[ri][0] + txi * TILE;
    const int sy0 = a.rect[ri][1] + tyi * TILE;
    const int sx1 = a.rect[ri][0] + a.rect[ri][2];
    const int sy1 = a.rect[ri][1] + a.rect[ri][3];
    const int R = a.R;
    const int tw = TILE + 2 * R;

    // Stage heights of logical cells [sx0-R, sx0+16+R) x [sy0-R, sy0+16+R).
    for (int i = tid; i < tw * tw; i += BLOCK) {
        const int ly = i / tw;
        const int lx = i - ly * tw;
        const int gx = sx0 - R + lx, gy = sy0 - R + ly;
        float v = SENTINEL;
        if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H) {
            const int px = wrap(gx + a.rx, a.W), py = wrap(gy + a.ry, a.H);
            const float h = a.height[(int64_t)py * a.ld + px];
            if (fabsf(h) < HEIGHT_LIMIT) v = h;      // false for NaN and +-Inf
        }
        tile[ly * P + lx] = v;
    }
    __syncthreads();

    const int lane = tid & 63;
    const int lx = lane & 15;
    const int ly = (tid >> 6) * 4 + (lane >> 4);
    const int ix = sx0 + lx, iy = sy0 + ly;
    const bool active = ix < sx1 && iy < sy1;
    const float* tp0 = tile + (ly + R) * P + (lx + R);
    const float hc = tp0[0];
    const int64_t cell = (int64_t)wrap(iy + a.ry, a.H) * a.W + wrap(ix + a.rx, a.W);

    const int u0 = blockIdx.y * a.units_per_group;
    const int u1 = min(a.n_units, u0 + a.units_per_group);
    for (int u = u0; u < u1; ++u) {
        const int64_t ub = (int64_t)u * a.n_samples;
        const cptr<float4> W = as_const(a.wts) + ub;
        const cptr<int32_t> O = as_const(a.offs) + ub;

        // Reference height: own cell, else the first valid sample in table order.
        // A state with no valid sample keeps ref = 0, so every sample stays invalid.
        float ref = (fabsf(hc) < HEIGHT_LIMIT) ? hc : 0.f;
        bool need = active && !(fabsf(hc) < HEIGHT_LIMIT);
        if (__ballot(need)) {
            for (int s = 0; s < a.n_samples; ++s) {
                if (!__ballot(need)) break;
                const float4 w = W[s];
                const int off = O[s];
                if (need) {
                    const float h = sample<P>(tp0, off, w, 0.f);
                    if (fabsf(h) < VALID_LIMIT) {
                        ref = h;
                        need = false;
                    }
                }
            }
        }

        Moments<float> m;
        if constexpr (NW > 0)
            accumulate_rows<P, NW>(a, tp0, W, O, ref, m);
        else
            accumulate_segments<P>(a, tp0, W, O, ref, m);
        Result r = finish<float>(a, m, ref);

        if (a.precision == 1) {
            const bool redo = (r.st & SEB_ST_DEGEN) != 0;
            if (__ballot(redo) && redo) {
                Moments<double> md;
                accumulate64<P>(a, tp0, O, as_const(a.frac) + ub, (double)ref, md);
                r = finish<double>(a, md, (double)ref);
            }
        }

        if (active) {
            store(a, u, cell, r, false);
            if (a.mirror) store(a, u + a.mirror, cell, r, true);
        }
    }
}

// Write newly exposed cells (or unknown) into the ring.
__global__ __launch_bounds__(BLOCK) void insert_kernel(const InsertArgs a) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int lx, ly;
    float v;
    if (a.full) {
        if (i >= (int64_t)a.W * a.H) return;
        ly = (int)(i / a.W);
        lx = (int)(i - (int64_t)ly * a.W);
        v = a.src ? a.src[(int64_t)ly * a.src_ld + lx] : __builtin_nanf("");
    } else {
        const int64_t nrow = (int64_t)a.rows_n * a.W;
        const int rem = a.H - a.rows_n;
        if (i < nrow) {
            ly = a.rows_lo + (int)(i / a.W);
            lx = (int)(i % a.W);
        } else {
            const int64_t j = i - nrow;
            if (a.cols_n == 0 || j >= (int64_t)a.cols_n * rem) return;
            const int r = (int)(j / a.cols_n);
            ly = (a.rows_lo == 0 ? a.rows_n : 0) + r;
            lx = a.cols_lo + (int)(j - (int64_t)r * a.cols_n);
        }
        v = a.src ? a.src[i] : __builtin_nanf("");
    }
    const int px = wrap(lx + a.rx, a.W), py = wrap(ly + a.ry, a.H);
    a.ring[(int64_t)py * a.ld + px] = v;
}

}  // namespace

int pick_pitch(int R) {
    const int need = TILE + 2 * R;
    static const int pitches[] = {48, 80, 112, 144};
    for (int p : pitches)
        if (p >= need) return p;
    return 0;
}

bool has_row_kernel(int row_len) { return row_len == 4 || row_len == 12 || row_len == 24; }

template <int P>
static hipError_t launch_p(const AssessArgs& a, dim3 grid, size_t lds, hipStream_t stream) {
    switch (a.row_len) {
        case 4: hipLaunchKernelGGL((assess_kernel<P, 4>), grid, dim3(BLOCK), lds, stream, a); break;
        case 12: hipLaunchKernelGGL((assess_kernel<P, 12>), grid, dim3(BLOCK), lds, stream, a); break;
        case 24: hipLaunchKernelGGL((assess_kernel<P, 24>), grid, dim3(BLOCK), lds, stream, a); break;
        default: hipLaunchKernelGGL((assess_kernel<P, 0>), grid, dim3(BLOCK), lds, stream, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_assess(const AssessArgs& a, int pitch, hipStream_t stream) {
    const int tiles = a.tile_start[a.n_rects];
    if (tiles == 0) return hipSuccess;
    const int groups = (a.n_units + a.units_per_group - 1) / a.units_per_group;
    const dim3 grid(tiles, groups);
    const size_t lds = (size_t)(TILE + 2 * a.R) * pitch * sizeof(float);
    switch (pitch) {
        case 48: return launch_p<48>(a, grid, lds, stream);
        case 80: return launch_p<80>(a, grid, lds, stream);
        case 112: return launch_p<112>(a, grid, lds, stream);
        case 144: return launch_p<144>(a, grid, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_insert(const InsertArgs& a, hipStream_t stream) {
    int64_t n = a.full ? (int64_t)a.W * a.H
                       : (int64_t)a.rows_n * a.W + (int64_t)a.cols_n * (a.H - a.rows_n);
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(insert_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

}  // namespace seb
