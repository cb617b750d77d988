// Device code of the per-state assessment (Sec. V-B, Algorithm 1, with the
// pose of Sec. III, Eq. 1-3) for the tiled kernel, which serves full maps,
// rolling-window bands and the surrogate's fallback states alike.  Heights
// are read through a source type (the LDS tile).
#pragma once

#include <cmath>

#include "seb.h"
#include "seb_internal.hpp"

namespace seb {
namespace dev {

__device__ __forceinline__ int wrap(int v, int n) { return v >= n ? v - n : v; }

// The footprint table is read-only for the lifetime of a launch.  Reading it
// through the constant address space lets the compiler fetch wave-uniform
// entries with scalar loads even though the kernel also stores to global memory.
// (The host compilation pass of the .hip files only parses the kernels, so
// there the qualifier is dropped.)
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

template <typename T>
struct Moments {
    T Sz, Spz, Sqz, Szz;          // sums over valid samples of z, p z, q z, z^2 (z centred)
    int32_t N, Sp, Sq, Spp, Spq, Sqq;
};

struct Result {
    float z, roll, pitch, risk;
    uint8_t st;
};

// Algorithm 1's two early-outs and the weighted risk, from the curvature and
// the two tilt magnitudes; sets the obstacle and traversable bits.
__device__ __forceinline__ float weigh_risk(const AssessArgs& a, float kappa, float phx, float phy,
                                            uint8_t& st) {
    float risk;
    if (kappa > a.kappa_max) {
        risk = 1.f;
        st |= SEB_ST_CURV;
    } else if (phx > a.phi_x_max || phy > a.phi_y_max) {
        risk = 1.f;
        st |= SEB_ST_TILT;
    } else {
        risk = a.c_kappa * kappa + a.c_phi_x * phx + a.c_phi_y * phy;
    }
    if (risk <= a.risk_max) st |= SEB_ST_TRAV;
    return risk;
}

// Principal-component plane of Algorithm 1: the eigenvector of the footprint
// scatter S (N times the covariance) with the smallest eigenvalue, turned to
// point up, and kappa = lambda_min / tr S.  Always solved in FP64.
// lambda_min is the smallest root of the characteristic polynomial
// f(l) = l^3 - c2 l^2 + c1 l - c0 (c2 = tr S, c1 = sum of the principal 2 x 2
// minors, c0 = det S), found by Newton's method from l = 0.  S is positive
// semi-definite, so every root is real and >= 0, and lambda_min <= tr S / 3;
// on [0, lambda_min] f is therefore increasing and concave (f'' = 6 l - 2 c2),
// and the iterates rise monotonically to lambda_min without overshooting it:
// quadratically for a simple root, halving the distance for a double one.
// The iteration stops when a step no longer increases l.  The eigenvector is
// the longest of the three cross products of two rows of S - lambda_min I
// (each is orthogonal to the row space).  A scatter whose smallest eigenvalue
// is repeated has no unique normal; it gets (0, 0, 1).
struct PcaPlane {
    double nu, nv, nz;   // unit normal in the yaw frame, nz >= 0
    double kappa;
};

__device__ inline PcaPlane pca_plane(double suu, double svv, double szz, double suv, double suz,
                                     double svz) {
    const double c2 = suu + svv + szz;
    const double c1 = (suu * svv - suv * suv) + (suu * szz - suz * suz) + (svv * szz - svz * svz);
    const double c0 = suu * (svv * szz - svz * svz) - suv * (suv * szz - svz * suz) +
                      suz * (suv * svz - svv * suz);
    double lam = 0.0;
    for (int it = 0; it < 128; ++it) {
        const double f = ((lam - c2) * lam + c1) * lam - c0;
        const double df = (3.0 * lam - 2.0 * c2) * lam + c1;
        if (!(f < 0.0) || !(df > 0.0)) break;
        const double next = lam - f / df;
        if (!(next > lam)) break;
        lam = next;
    }
    const double a0 = suu - lam, a1 = svv - lam, a2 = szz - lam;
    // rows (a0, suv, suz), (suv, a1, svz), (suz, svz, a2)
    const double x01 = suv * svz - suz * a1, y01 = suz * suv - a0 * svz, z01 = a0 * a1 - suv * suv;
    const double x02 = suv * a2 - suz * svz, y02 = suz * suz - a0 * a2, z02 = a0 * svz - suv * suz;
    const double x12 = a1 * a2 - svz * svz, y12 = svz * suz - suv * a2, z12 = suv * svz - a1 * suz;
    const double d01 = x01 * x01 + y01 * y01 + z01 * z01;
    const double d02 = x02 * x02 + y02 * y02 + z02 * z02;
    const double d12 = x12 * x12 + y12 * y12 + z12 * z12;
    double x = 0.0, y = 0.0, z = 1.0, d = 1.0;
    if (d01 >= d02 && d01 >= d12 && d01 > 0.0) {
        x = x01; y = y01; z = z01; d = d01;
    } else if (d02 >= d12 && d02 > 0.0) {
        x = x02; y = y02; z = z02; d = d02;
    } else if (d12 > 0.0) {
        x = x12; y = y12; z = z12; d = d12;
    }
    const double s = (z < 0.0 ? -1.0 : 1.0) / sqrt(d);
    PcaPlane pl;
    pl.nu = x * s;
    pl.nv = y * s;
    pl.nz = z * s;
    pl.kappa = (c2 > 0.0) ? lam / c2 : 0.0;
    return pl;
}

// 1 / x: the hardware reciprocal (within 1 ulp) in FP32, exact division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Plane from the moments, then Eq. 1-3 and Algorithm 1.  u = hu p, v = hv q
// are the body-frame sample coordinates.  fit 0: least-squares plane
// z = a + b u + c v; fit 1: principal-component plane.
template <int FIT, typename T>
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

    const T invN = recip(T(N));
    const T zb = m.Sz * invN;
    const T pz = m.Spz - T(m.Sp) * zb;      // sum (p - pbar)(z - zbar)
    const T qz = m.Sqz - T(m.Sq) * zb;
    const T zz = m.Szz - m.Sz * zb;         // sum (z - zbar)^2
    if constexpr (FIT == 1) {
        // Scatter in metres: S_uu = hu^2 D / N, S_vv = hv^2 E / N, S_uv = hu hv F / N.
        const double hu = a.hu, hv = a.hv, dN = (double)N;
        const PcaPlane pl = pca_plane(hu * hu * (double)D / dN, hv * hv * (double)E / dN,
                                      (double)zz, hu * hv * (double)F / dN, hu * (double)pz,
                                      hv * (double)qz);
        // The plane through the centroid, evaluated at the state's cell centre.
        const double ubar = hu * (double)m.Sp / dN, vbar = hv * (double)m.Sq / dN;
        r.z = (float)((double)ref + (double)zb + (pl.nu * ubar + pl.nv * vbar) / pl.nz);
        const float nu = (float)pl.nu, nv = (float)pl.nv, nz = (float)pl.nz;
        const float l2 = nv * nv + nz * nz;
        r.roll = atan2f(-nv, nz);                                        // asin(b3 . y_b)
        r.pitch = atan2f(nu, sqrtf(l2));                                 // atan2(-b3 . x_b, b3 . z_b)
        const float phx = atan2f(nz * fabsf(nu), sqrtf(nu * nu * nv * nv + l2 * l2));
        r.risk = weigh_risk(a, (float)pl.kappa, phx, fabsf(r.roll), st);
        r.st = st;
        return r;
    }
    const T ndet = T(N) * recip(T(det));
    const T bp = (T(E) * pz - T(F) * qz) * ndet;          // dz/dp
    const T bq = (T(D) * qz - T(F) * pz) * ndet;          // dz/dq
    T b, c;                                               // dz/du, dz/dv
    if constexpr (sizeof(T) == 4) {
        b = bp * a.inv_hu;
        c = bq * a.inv_hv;
    } else {
        b = bp / T(a.hu);
        c = bq / T(a.hv);
    }
    const T zc = ref + zb - bp * (T(m.Sp) * invN) - bq * (T(m.Sq) * invN);
    T sse = zz - bp * pz - bq * qz;
    if (sse < T(0)) sse = T(0);
    const T s2 = T(1) + b * b + c * c;
    const T tr = T(a.hu) * T(a.hu) * T(D) * invN + T(a.hv) * T(a.hv) * T(E) * invN + zz;
    const float kappa = (tr > T(0)) ? (float)(sse * recip(s2 * tr)) : 0.f;

    const float bf = (float)b, cf = (float)c;
    const float c1 = 1.f + cf * cf;
    r.z = (float)zc;
    r.roll = atanf(cf);                              // asin(b3 . y_b)
    r.pitch = -atan2f(bf, sqrtf(c1));               // atan2(-b3 . x_b, b3 . z_b)
    const float phx = atan2f(fabsf(bf), sqrtf(c1 * c1 + bf * bf * cf * cf));   // |asin(b3 . x_b)|
    const float phy = fabsf(r.roll);                                             // |asin(b3 . y_b)|
    r.risk = weigh_risk(a, kappa, phx, phy, st);
    r.st = st;
    return r;
}

// Height source of a state's footprint samples.  quad() returns the four
// corners (0,0) (1,0) (0,1) (1,1) of the sample whose corner (0,0) sits at
// table offset `off` (dy * P + dx) from the state's cell; unknown and
// out-of-map cells read as SENTINEL.
template <int P>
struct LdsSource {
    const float* tp0;   // the state's own cell in the LDS tile
    __device__ __forceinline__ void quad(int off, float& h00, float& h01, float& h10,
                                         float& h11) const {
        const float* tp = tp0 + off;
        h00 = tp[0];
        h01 = tp[1];
        h10 = tp[P];
        h11 = tp[P + 1];
    }
};

// Bilinear sample of the state, centred on ref.  Corner weights are
// wave-uniform scalars.
template <class Src>
__device__ __forceinline__ float sample(const Src& src, int off, float4 w, float ref) {
    float h00, h01, h10, h11;
    src.quad(off, h00, h01, h10, h11);
    float z = fmaf(w.x, h00, -ref);
    z = fmaf(w.y, h01, z);
    z = fmaf(w.z, h10, z);
    return fmaf(w.w, h11, z);
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

// One footprint row of NW samples (see accumulate_rows).  SEARCH: some lanes
// have no reference height yet (need); such a lane takes the raw value of
// its first valid sample in table order as its reference (that sample then
// counts as z = 0), which is exactly the value a separate search in table
// order would find, since no earlier sample contributes.  REUSE: a sample
// whose corner cell equals the previous sample's (a wave-uniform test on the
// table) takes that sample's four heights instead of reading the tile again;
// samples are half a cell apart, so about two in five repeat their quad.
// (Reusing the two shared corners of a quad one cell over as well measured
// slower: the extra branches cost more than the reads they save.)
// (prev_o, hp) carry the previous sample's offset and heights.
template <int NW, bool SEARCH, bool REUSE, class Src>
__device__ __forceinline__ void accumulate_row(const Src& src, cptr<float4> W, cptr<int32_t> O,
                                               int i, int row1, float4 (&wn)[4], int (&on)[4],
                                               float& ref, bool& need, float& rz, uint32_t& pk,
                                               Moments<float>& m, int& prev_o, float (&hp)[4]) {
    constexpr int kQoff = NW - 1;
    constexpr int kSh2 = 6 + bits_for(NW * 2 * kQoff);
    constexpr int CH = 4;
#pragma unroll
    for (int c = 0; c < NW; c += CH) {
        float4 w[CH];
        int o[CH];
#pragma unroll
        for (int s = 0; s < CH; ++s) { w[s] = wn[s]; o[s] = on[s]; }
        float h[CH][4];
        if constexpr (REUSE) {
            // A wave-uniform branch per sample.  Each repeat waits for the
            // previous sample's reads; measured, this still beats reading
            // every quad and selecting afterwards.
#pragma unroll
            for (int s = 0; s < CH; ++s) {
                const int po = s == 0 ? prev_o : o[s - 1];
                if (o[s] == po) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) h[s][t] = s == 0 ? hp[t] : h[s - 1][t];
                    continue;
                }
                src.quad(o[s], h[s][0], h[s][1], h[s][2], h[s][3]);
            }
        } else {
#pragma unroll
            for (int s = 0; s < CH; ++s) src.quad(o[s], h[s][0], h[s][1], h[s][2], h[s][3]);
        }
        if constexpr (REUSE) {
            prev_o = o[CH - 1];
#pragma unroll
            for (int t = 0; t < 4; ++t) hp[t] = h[CH - 1][t];
        }
        // prefetch the next chunk's table entries (the last chunk of the
        // range re-loads itself, so no read leaves the unit's table)
        const int nx = min(i * NW + c + CH, row1 * NW - CH);
#pragma unroll
        for (int s = 0; s < CH; ++s) { wn[s] = W[nx + s]; on[s] = O[nx + s]; }
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int j = c + s;
            float z = fmaf(w[s].x, h[s][0], -ref);
            z = fmaf(w[s].y, h[s][1], z);
            z = fmaf(w[s].z, h[s][2], z);
            z = fmaf(w[s].w, h[s][3], z);
            if (fabsf(z) < VALID_LIMIT) {
                if constexpr (SEARCH) {
                    if (need) {
                        ref = z;
                        z = 0.f;
                        need = false;
                    }
                }
                const int q = 2 * j - kQoff;
                rz += z;
                m.Sqz = fmaf((float)q, z, m.Sqz);
                m.Szz = fmaf(z, z, m.Szz);
                pk += 1u | ((uint32_t)(2 * j) << 6) | ((uint32_t)(q * q) << kSh2);
            }
        }
    }
}

// FP32 moments of rows [row0, row1) of one yaw bin when every segment is a
// full row of NW samples: the row loop is unrolled, so q and the packed
// integer constants of each sample are compile-time values.  A row runs the
// reference-adopting body only while some lane of the wave still lacks a
// reference height (normally the first row or two).
template <int NW, bool REUSE, class Src>
__device__ __forceinline__ void accumulate_rows(const AssessArgs& a, const Src& src,
                                                cptr<float4> W, cptr<int32_t> O, float& ref,
                                                bool& need, Moments<float>& m, int row0,
                                                int row1) {
    constexpr int kQoff = NW - 1;
    constexpr int kSh2 = 6 + bits_for(NW * 2 * kQoff);
    constexpr uint32_t kMask1 = (1u << (kSh2 - 6)) - 1u;
    static_assert(kSh2 + bits_for(NW * kQoff * kQoff) <= 32, "packed moments overflow");
    m.Sz = m.Spz = m.Sqz = m.Szz = 0.f;
    m.N = m.Sp = m.Sq = m.Spp = m.Spq = m.Sqq = 0;
    const int nrows = a.n_segs;
    int p = 1 - nrows + 2 * row0;
    // Samples go in chunks of four.  A chunk's table entries arrive in two
    // wide scalar loads, issued together with its eight LDS reads and the
    // next chunk's table prefetch, so a wave waits once per chunk instead of
    // once per sample (scalar and LDS loads share one wait counter).
    constexpr int CH = 4;
    static_assert(NW % CH == 0, "row length must be a multiple of the chunk");
    float4 wn[CH];
    int on[CH];
#pragma unroll
    for (int s = 0; s < CH; ++s) { wn[s] = W[row0 * NW + s]; on[s] = O[row0 * NW + s]; }
    int prev_o = INT32_MIN;                  // no previous sample: never equal to an offset
    float hp[4] = {0.f, 0.f, 0.f, 0.f};
    int i = row0;
    for (; i < row1 && __ballot(need); ++i, p += 2) {
        float rz = 0.f;
        uint32_t pk = 0u;
        accumulate_row<NW, true, REUSE>(src, W, O, i, row1, wn, on, ref, need, rz, pk, m, prev_o, hp);
        add_segment(m, p, pk, kQoff, kMask1, kSh2, rz);
    }
    for (; i < row1; ++i, p += 2) {
        float rz = 0.f;
        uint32_t pk = 0u;
        accumulate_row<NW, false, REUSE>(src, W, O, i, row1, wn, on, ref, need, rz, pk, m, prev_o,
                                         hp);
        add_segment(m, p, pk, kQoff, kMask1, kSh2, rz);
    }
}

// FP32 moments of one yaw bin, any footprint (segments of any length).
template <bool SEARCH, class Src>
__device__ __forceinline__ void accumulate_segments(const AssessArgs& a, const Src& src,
                                                    cptr<float4> W, cptr<int32_t> O, float& ref,
                                                    bool& need, Moments<float>& m, int seg0,
                                                    int seg1) {
    m.Sz = m.Spz = m.Sqz = m.Szz = 0.f;
    m.N = m.Sp = m.Sq = m.Spp = m.Spq = m.Sqq = 0;
    const cptr<Segment> segs = as_const(a.segs);
    const cptr<float> qs = as_const(a.qs);
    const cptr<uint32_t> pks = as_const(a.pks);
    for (int g = seg0; g < seg1; ++g) {
        const Segment sg = segs[g];
        float rz = 0.f;
        uint32_t pk = 0u;
        for (int s = sg.first; s < sg.first + sg.count; ++s) {
            float z = sample(src, O[s], W[s], ref);
            if (fabsf(z) < VALID_LIMIT) {
                if constexpr (SEARCH) {
                    if (need) {
                        ref = z;
                        z = 0.f;
                        need = false;
                    }
                }
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
template <class Src>
__device__ void accumulate64(const AssessArgs& a, const Src& src, cptr<int32_t> O,
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
            float h00, h01, h10, h11;
            src.quad(O[s], h00, h01, h10, h11);
            const double gx = 1.0 - f.x, gy = 1.0 - f.y;
            const double z = gx * gy * (double)h00 + f.x * gy * (double)h01 +
                             gx * f.y * (double)h10 + f.x * f.y * (double)h11 - ref;
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

// Outputs are written once and not read again by the kernel: non-temporal
// stores keep them from evicting the footprint table (read by every wave
// through the scalar cache) and the height map from L2.
__device__ __forceinline__ void store(const AssessArgs& a, int k, int64_t cell, const Result& r,
                                      bool negate) {
    const int64_t o = (int64_t)k * a.H * a.W + cell;
    __builtin_nontemporal_store(r.z, a.z + o);
    __builtin_nontemporal_store(negate ? -r.roll : r.roll, a.roll + o);
    __builtin_nontemporal_store(negate ? -r.pitch : r.pitch, a.pitch + o);
    __builtin_nontemporal_store(r.risk, a.risk + o);
    __builtin_nontemporal_store(r.st, a.status + o);
}

// Result of a state from its FP32 moments; with precision 1, near-degenerate
// states are recomputed from FP64 moments about the same reference.
template <int FIT, class Src>
__device__ __forceinline__ Result finish_state(const AssessArgs& a, const Src& src, int u,
                                               const Moments<float>& m, float ref) {
    Result r = finish<FIT>(a, m, ref);
    if (a.precision == 1) {
        const bool redo = (r.st & SEB_ST_DEGEN) != 0;
        if (__ballot(redo) && redo) {
            const int64_t ub = (int64_t)u * a.n_samples;
            Moments<double> md;
            accumulate64(a, src, as_const(a.offs) + ub, as_const(a.frac) + ub, (double)ref, md);
            r = finish<FIT>(a, md, (double)ref);
        }
    }
    return r;
}

// FP32 moments of rows (segments) [g0, g1) of yaw unit u.  On entry ref is
// the own cell's height, or 0 with need set when that cell is unknown; a lane
// with need adopts its first valid sample in table order (see accumulate_rows).
// REUSE: skip the tile reads of samples that repeat the previous sample's
// corner cell (see accumulate_row).
template <int NW, class Src, bool REUSE = false>
__device__ __forceinline__ void partial_moments(const AssessArgs& a, const Src& src, int u, int g0,
                                                int g1, float& ref, bool& need,
                                                Moments<float>& m) {
    const int64_t ub = (int64_t)u * a.n_samples;
    const cptr<float4> W = as_const(a.wts) + ub;
    const cptr<int32_t> O = as_const(a.offs) + ub;
    if constexpr (NW > 0) {
        accumulate_rows<NW, REUSE>(a, src, W, O, ref, need, m, g0, g1);
    } else {
        if (__ballot(need))
            accumulate_segments<true>(a, src, W, O, ref, need, m, g0, g1);
        else
            accumulate_segments<false>(a, src, W, O, ref, need, m, g0, g1);
    }
}

// Partial moments of the waves that share a state's footprint rows, kept in
// LDS per wave and lane.
struct Parts {
    float f[BLOCK / 64][5][64];   // reference, Sz, Spz, Sqz, Szz
    int i[BLOCK / 64][7][64];     // reference found, N, Sp, Sq, Spp, Spq, Sqq
};

__device__ __forceinline__ void put_part(Parts& pt, int wave, int lane, const Moments<float>& m,
                                         float ref, bool need) {
    pt.f[wave][0][lane] = ref;
    pt.f[wave][1][lane] = m.Sz;
    pt.f[wave][2][lane] = m.Spz;
    pt.f[wave][3][lane] = m.Sqz;
    pt.f[wave][4][lane] = m.Szz;
    pt.i[wave][0][lane] = need ? 0 : 1;
    pt.i[wave][1][lane] = m.N;
    pt.i[wave][2][lane] = m.Sp;
    pt.i[wave][3][lane] = m.Sq;
    pt.i[wave][4][lane] = m.Spp;
    pt.i[wave][5][lane] = m.Spq;
    pt.i[wave][6][lane] = m.Sqq;
}

// Adds the partial moments of waves w0 .. w0 + n - 1 (the rows that follow
// in table order) to m.  A state whose own cell is unknown has, per wave, the
// first valid sample of that wave's rows as reference; the sums are shifted
// exactly onto the first reference found in table order:
//   S(z - r) = S(z - r_w) + N_w d,  S q(z - r) = S q(z - r_w) + d S q,
//   S (z - r)^2 = S (z - r_w)^2 + 2 d S(z - r_w) + N_w d^2,  d = r_w - r.
// d is 0 whenever the own cell is known (every wave then uses its height).
__device__ __forceinline__ void merge_parts(const Parts& pt, int w0, int n, int lane,
                                            Moments<float>& m, float& ref, bool& need) {
    for (int k = 0; k < n; ++k) {
        const int w = w0 + k;
        const float rw = pt.f[w][0][lane];
        const int nw = pt.i[w][1][lane];
        if (need && pt.i[w][0][lane]) {
            ref = rw;                    // no valid sample so far: take this wave's reference
            need = false;
        }
        const float d = rw - ref;
        const float sz = pt.f[w][1][lane];
        m.Sz += sz + (float)nw * d;
        m.Spz += pt.f[w][2][lane] + d * (float)pt.i[w][2][lane];
        m.Sqz += pt.f[w][3][lane] + d * (float)pt.i[w][3][lane];
        m.Szz += pt.f[w][4][lane] + 2.f * d * sz + (float)nw * d * d;
        m.N += nw;
        m.Sp += pt.i[w][2][lane];
        m.Sq += pt.i[w][3][lane];
        m.Spp += pt.i[w][4][lane];
        m.Spq += pt.i[w][5][lane];
        m.Sqq += pt.i[w][6][lane];
    }
}

// Reference height, moments, optional FP64 redo and result of one state for
// yaw unit u.  hc = the state's own cell (SENTINEL if unknown); `active`
// lanes take part in the reference search.
template <int NW, int FIT, class Src>
__device__ __forceinline__ Result assess_state(const AssessArgs& a, const Src& src, int u, float hc,
                                               bool active) {
    // Reference height: own cell, else the first valid sample in table order
    // (adopted inside the sample loop).  A state with no valid sample keeps
    // ref = 0, and every sample stays invalid.
    float ref = (fabsf(hc) < HEIGHT_LIMIT) ? hc : 0.f;
    bool need = active && !(fabsf(hc) < HEIGHT_LIMIT);

    Moments<float> m;
    partial_moments<NW>(a, src, u, 0, a.n_segs, ref, need, m);
    return finish_state<FIT>(a, src, u, m, ref);
}

}  // namespace dev
}  // namespace seb
