/*
 * FP64 CPU oracle for SE(2)-grid traversability assessment.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition the HIP library is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the HIP library.
 *
 * What it computes, per SE(2) state (ix, iy, k) of a height map, following the
 * paper (SEB-Naver, arXiv 2503.02412):
 *   Sec. III, Eq. 1-3 : terrain pose mapping F: SE(2) -> R x S^2_+, the body
 *                       axes y_b = z_b x x_yaw / |.|, x_b = y_b x z_b, and the
 *                       Z-X-Y Euler angles of the attitude.
 *   Sec. V-B, Alg. 1  : gather the footprint points, their mean and covariance,
 *                       the terrain normal z_b and curvature kappa, the two
 *                       early-outs (kappa > kappa_max; tilt above phi_max) and
 *                       the weighted risk.
 *
 * Readings taken where the paper is silent (all are stated again in the
 * design notes of the repository):
 *   - footprint = body-frame midpoint grid of fp_nl x fp_nw samples over a
 *     fp_length x fp_width rectangle (optionally clipped to the inscribed
 *     ellipse, decided in exact integers), centred on the state's cell centre;
 *   - yaw bins theta_k = 2 pi k / K;
 *   - a sample reads the bilinear interpolation of the four surrounding cell
 *     centres; grid offsets within 1e-6 of an integer are snapped to it; a
 *     corner with zero weight is not required; the sample is dropped unless
 *     every required corner is inside the map and finite;
 *   - fit 0 (default): least-squares plane z = a + b u + c v over the valid
 *     points in the yaw frame; its unit normal is z_b; kappa = n^T C n / tr C
 *     (surface variation).  fit 1: the paper-literal minimum eigenvector of
 *     C, kappa = lambda_min / tr C;
 *   - fewer than min_valid valid samples, or collinear valid samples (exact
 *     integer test), leave the state UNKNOWN: z = roll = pitch = NaN, risk 1;
 *   - z = height of the fitted plane at the state's cell centre;
 *   - thresholds: strict '>' for the early-outs, 'risk <= r_max' for the
 *     traversable bit.
 *
 * Status bits: 1 fit valid, 2 curvature obstacle, 4 tilt obstacle,
 *              8 near-degenerate footprint, 16 traversable.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t width, height;
    double res;
    int32_t n_yaw;
    double fp_length, fp_width;
    int32_t fp_nl, fp_nw;
    int32_t fp_shape;           /* 0 rectangle, 1 inscribed ellipse */
    double kappa_max, phi_x_max, phi_y_max;
    double w_kappa, w_phi_x, w_phi_y, risk_max;
    int32_t min_valid;
    int32_t fit;                /* 0 least squares, 1 principal component */
} orc_params;

/* Per-state result, all FP64. */
typedef struct {
    double z, roll, pitch, risk, kappa, phi_x, phi_y;
    int32_t n_valid;
    uint8_t status;
} orc_state;

enum { ST_VALID = 1, ST_CURV = 2, ST_TILT = 4, ST_DEGEN = 8, ST_TRAV = 16 };

static const double ORC_PI = 3.14159265358979323846;
static const double SNAP_EPS = 1e-6;

/* Footprint sample (i, j) in the body frame: x forward (length), y left. */
static int in_footprint(const orc_params* P, int i, int j, double* u, double* v,
                        int* p, int* q) {
    *p = 2 * i - (P->fp_nl - 1);
    *q = 2 * j - (P->fp_nw - 1);
    *u = (i + 0.5) * P->fp_length / P->fp_nl - 0.5 * P->fp_length;
    *v = (j + 0.5) * P->fp_width / P->fp_nw - 0.5 * P->fp_width;
    if (P->fp_shape == 1) {
        /* (u / e_x)^2 + (v / e_y)^2 <= 1 with semi-axes L/2, W/2  <=>
           (p / nl)^2 + (q / nw)^2 <= 1, decided in exact integers. */
        int64_t nl = P->fp_nl, nw = P->fp_nw;
        int64_t lhs = (int64_t)(*p) * (*p) * nw * nw + (int64_t)(*q) * (*q) * nl * nl;
        if (lhs > nl * nl * nw * nw) return 0;
    }
    return 1;
}

static double snap(double o) {
    double r = nearbyint(o);
    return fabs(o - r) < SNAP_EPS ? r : o;
}

static int cell_ok(const orc_params* P, const float* H, int64_t ld, int64_t x, int64_t y,
                   double* h) {
    if (x < 0 || y < 0 || x >= P->width || y >= P->height) return 0;
    double v = (double)H[y * ld + x];
    if (!isfinite(v)) return 0;
    *h = v;
    return 1;
}

/* One bilinear footprint sample; returns 0 when the sample is dropped. */
static int sample_height(const orc_params* P, const float* H, int64_t ld, int ix, int iy,
                         double cth, double sth, double u, double v, double* h) {
    double ox = snap((u * cth - v * sth) / P->res);
    double oy = snap((u * sth + v * cth) / P->res);
    double fxd = floor(ox), fyd = floor(oy);
    double fx = ox - fxd, fy = oy - fyd;
    int64_t x0 = ix + (int64_t)fxd, y0 = iy + (int64_t)fyd;
    double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy};
    double acc = 0.0;
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
            double w = wx[a] * wy[b];
            if (w > 0.0) {
                double c;
                if (!cell_ok(P, H, ld, x0 + a, y0 + b, &c)) return 0;
                acc += w * c;
            }
        }
    *h = acc;
    return 1;
}

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix.
   On return d[] holds eigenvalues, column m of V the eigenvector of d[m]. */
static void jacobi3(const double A_in[3][3], double d[3], double V[3][3]) {
    double A[3][3];
    memcpy(A, A_in, sizeof(A));
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off == 0.0 || off <= 1e-300 || off < 1e-18 * scale) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {          /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {          /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {          /* V <- V J */
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int m = 0; m < 3; ++m) d[m] = A[m][m];
}

static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* rho_full = 4 det / (D + E)^2 of the complete footprint: the threshold scale
   of the near-degenerate flag. */
static double rho_full(const orc_params* P, int* n_total) {
    int64_t N = 0, Sp = 0, Sq = 0, Spp = 0, Spq = 0, Sqq = 0;
    for (int i = 0; i < P->fp_nl; ++i)
        for (int j = 0; j < P->fp_nw; ++j) {
            double u, v; int p, q;
            if (!in_footprint(P, i, j, &u, &v, &p, &q)) continue;
            N += 1; Sp += p; Sq += q; Spp += (int64_t)p * p; Spq += (int64_t)p * q; Sqq += (int64_t)q * q;
        }
    *n_total = (int)N;
    int64_t D = N * Spp - Sp * Sp, E = N * Sqq - Sq * Sq, F = N * Spq - Sp * Sq;
    int64_t det = D * E - F * F;
    double de = (double)(D + E);
    return (de > 0) ? (4.0 * (double)det) / (de * de) : 0.0;
}

/* The exact gate of the fit on the integer sample coordinates (p, q) of the
   valid samples (N, sums and sums of products): -1 = no fit (fewer than
   min_valid samples, or all of them on one line: det = 0), 0 = fit,
   1 = fit on a near-degenerate footprint, i.e. fewer than half of the n_total
   samples, or rho = 4 det / (D + E)^2 below rho_f / 16. */
static int gate(int64_t N, int64_t Sp, int64_t Sq, int64_t Spp, int64_t Spq, int64_t Sqq,
                int min_valid, int n_total, double rho_f) {
    int64_t D = N * Spp - Sp * Sp, E = N * Sqq - Sq * Sq, F = N * Spq - Sp * Sq;
    int64_t det = D * E - F * F;
    if (N < min_valid || det <= 0) return -1;
    double de = (double)(D + E);
    double rho = (4.0 * (double)det) / (de * de);
    return (2 * N < n_total || rho < rho_f / 16.0) ? 1 : 0;
}

static void assess_state(const orc_params* P, const float* H, int64_t ld, int ix, int iy,
                         int k, double rho_f, int n_total, orc_state* out) {
    const double theta = 2.0 * ORC_PI * (double)k / (double)P->n_yaw;
    const double cth = cos(theta), sth = sin(theta);

    /* FindEllipticalPoints: the valid footprint points, in the yaw frame. */
    int cap = P->fp_nl * P->fp_nw;
    double* pts = (double*)malloc(sizeof(double) * 3 * (size_t)cap);
    int n = 0;
    int64_t N = 0, Sp = 0, Sq = 0, Spp = 0, Spq = 0, Sqq = 0;
    for (int i = 0; i < P->fp_nl; ++i)
        for (int j = 0; j < P->fp_nw; ++j) {
            double u, v, h; int p, q;
            if (!in_footprint(P, i, j, &u, &v, &p, &q)) continue;
            if (!sample_height(P, H, ld, ix, iy, cth, sth, u, v, &h)) continue;
            pts[3 * n + 0] = u; pts[3 * n + 1] = v; pts[3 * n + 2] = h; ++n;
            N += 1; Sp += p; Sq += q;
            Spp += (int64_t)p * p; Spq += (int64_t)p * q; Sqq += (int64_t)q * q;
        }

    memset(out, 0, sizeof(*out));
    out->n_valid = n;
    /* Exact gate: enough points and not all on one line (integer scatter). */
    const int g = gate(N, Sp, Sq, Spp, Spq, Sqq, P->min_valid, n_total, rho_f);
    if (g < 0) {
        out->z = out->roll = out->pitch = NAN;
        out->kappa = out->phi_x = out->phi_y = NAN;
        out->risk = 1.0;
        out->status = 0;
        free(pts);
        return;
    }
    uint8_t status = ST_VALID;
    if (g > 0) status |= ST_DEGEN;

    /* GetMeanPosition and the covariance accumulation of Algorithm 1. */
    double mean[3] = {0, 0, 0};
    for (int m = 0; m < n; ++m)
        for (int a = 0; a < 3; ++a) mean[a] += pts[3 * m + a];
    for (int a = 0; a < 3; ++a) mean[a] /= (double)n;
    double C[3][3] = {{0}};
    for (int m = 0; m < n; ++m) {
        double e[3] = {pts[3 * m] - mean[0], pts[3 * m + 1] - mean[1], pts[3 * m + 2] - mean[2]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) C[a][b] += e[a] * e[b];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) C[a][b] /= (double)n;
    free(pts);
    double trC = C[0][0] + C[1][1] + C[2][2];

    /* Terrain normal n (yaw frame, n_z > 0), curvature, plane height. */
    double nrm[3], kappa, zc;
    if (P->fit == 1) {
        double d[3], V[3][3];
        jacobi3(C, d, V);
        int mi = 0;
        for (int m = 1; m < 3; ++m)
            if (d[m] < d[mi]) mi = m;
        double s = (V[2][mi] >= 0.0) ? 1.0 : -1.0;
        double len = sqrt(V[0][mi] * V[0][mi] + V[1][mi] * V[1][mi] + V[2][mi] * V[2][mi]);
        for (int a = 0; a < 3; ++a) nrm[a] = s * V[a][mi] / len;
        kappa = (trC > 0.0) ? d[mi] / trC : 0.0;
        if (kappa < 0.0) kappa = 0.0;
        zc = mean[2] + (nrm[0] * mean[0] + nrm[1] * mean[1]) / nrm[2];
    } else {
        /* Least squares z = a + b u + c v: centred normal equations. */
        double det2 = C[0][0] * C[1][1] - C[0][1] * C[0][1];
        double b = (C[1][1] * C[0][2] - C[0][1] * C[1][2]) / det2;
        double c = (C[0][0] * C[1][2] - C[0][1] * C[0][2]) / det2;
        double s = sqrt(1.0 + b * b + c * c);
        nrm[0] = -b / s; nrm[1] = -c / s; nrm[2] = 1.0 / s;
        double nCn = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) nCn += nrm[a] * C[a][bb] * nrm[bb];
        kappa = (trC > 0.0) ? nCn / trC : 0.0;
        if (kappa < 0.0) kappa = 0.0;
        zc = mean[2] - b * mean[0] - c * mean[1];
    }

    /* Eq. 1-3: z_b in the world frame, then y_b and x_b. */
    double zb[3] = {cth * nrm[0] - sth * nrm[1], sth * nrm[0] + cth * nrm[1], nrm[2]};
    double xyaw[3] = {cth, sth, 0.0};
    double yb[3], xb[3];
    cross3(zb, xyaw, yb);
    double ly = sqrt(yb[0] * yb[0] + yb[1] * yb[1] + yb[2] * yb[2]);
    for (int a = 0; a < 3; ++a) yb[a] /= ly;
    cross3(yb, zb, xb);

    /* Z-X-Y Euler angles of [x_b y_b z_b] = R_z(yaw) R_x(roll) R_y(pitch). */
    double sx = xb[2], sy = yb[2], sz = zb[2];
    if (sy > 1.0) sy = 1.0;
    if (sy < -1.0) sy = -1.0;
    if (sx > 1.0) sx = 1.0;
    if (sx < -1.0) sx = -1.0;
    out->z = zc;
    out->roll = asin(sy);
    out->pitch = atan2(-sx, sz);
    out->kappa = kappa;
    out->phi_x = fabs(asin(sx));
    out->phi_y = fabs(asin(sy));

    /* Algorithm 1: early-outs, then the weighted risk. */
    double risk;
    if (kappa > P->kappa_max) {
        risk = 1.0;
        status |= ST_CURV;
    } else if (out->phi_x > P->phi_x_max || out->phi_y > P->phi_y_max) {
        risk = 1.0;
        status |= ST_TILT;
    } else {
        risk = P->w_kappa * kappa / P->kappa_max + P->w_phi_x * out->phi_x / P->phi_x_max +
               P->w_phi_y * out->phi_y / P->phi_y_max;
    }
    if (risk <= P->risk_max) status |= ST_TRAV;
    out->risk = risk;
    out->status = status;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (called from oracle/oracle.py through ctypes).     */
/* ------------------------------------------------------------------------ */

/* Assess every state in the rectangle [x0, x0+nx) x [y0, y0+ny), yaw bins
   [k0, k0+nk).  Output arrays are laid out [k - k0][iy - y0][ix - x0].
   Any output pointer may be NULL.  Returns 0, or -1 on a bad argument. */
int orc_assess_rect(const orc_params* P, const float* H, int64_t ld, int x0, int y0, int nx,
                    int ny, int k0, int nk, double* z, double* roll, double* pitch,
                    double* risk, double* kappa, double* phi_x, double* phi_y,
                    uint8_t* status, int32_t* n_valid, int n_threads) {
    if (!P || !H || nx < 0 || ny < 0 || nk < 0 || P->n_yaw <= 0 || P->fp_nl <= 0 ||
        P->fp_nw <= 0 || P->res <= 0.0)
        return -1;
    int n_total;
    double rho_f = rho_full(P, &n_total);
    int64_t plane = (int64_t)nx * ny;
    int64_t total = plane * nk;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t row = 0; row < (int64_t)nk * ny; ++row) {
        int kk = (int)(row / ny), yy = (int)(row % ny);
        for (int xx = 0; xx < nx; ++xx) {
            orc_state st;
            assess_state(P, H, ld, x0 + xx, y0 + yy, k0 + kk, rho_f, n_total, &st);
            int64_t o = (int64_t)kk * plane + (int64_t)yy * nx + xx;
            if (z) z[o] = st.z;
            if (roll) roll[o] = st.roll;
            if (pitch) pitch[o] = st.pitch;
            if (risk) risk[o] = st.risk;
            if (kappa) kappa[o] = st.kappa;
            if (phi_x) phi_x[o] = st.phi_x;
            if (phi_y) phi_y[o] = st.phi_y;
            if (status) status[o] = st.status;
            if (n_valid) n_valid[o] = st.n_valid;
        }
    }
    (void)total;
    return 0;
}

/* Assess an explicit list of states (ix[m], iy[m], k[m]); outputs indexed by m. */
int orc_assess_list(const orc_params* P, const float* H, int64_t ld, int64_t n,
                    const int32_t* ix, const int32_t* iy, const int32_t* k, double* z,
                    double* roll, double* pitch, double* risk, double* kappa, double* phi_x,
                    double* phi_y, uint8_t* status, int32_t* n_valid, int n_threads) {
    if (!P || !H || n < 0 || !ix || !iy || !k) return -1;
    int n_total;
    double rho_f = rho_full(P, &n_total);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t m = 0; m < n; ++m) {
        orc_state st;
        assess_state(P, H, ld, ix[m], iy[m], k[m], rho_f, n_total, &st);
        if (z) z[m] = st.z;
        if (roll) roll[m] = st.roll;
        if (pitch) pitch[m] = st.pitch;
        if (risk) risk[m] = st.risk;
        if (kappa) kappa[m] = st.kappa;
        if (phi_x) phi_x[m] = st.phi_x;
        if (phi_y) phi_y[m] = st.phi_y;
        if (status) status[m] = st.status;
        if (n_valid) n_valid[m] = st.n_valid;
    }
    return 0;
}

/* Cells a state's footprint can read: the extent of every required corner
   offset over all yaw bins and samples (the reach of the assessment). */
int orc_reach(const orc_params* P, int32_t* dx_min, int32_t* dx_max, int32_t* dy_min,
              int32_t* dy_max) {
    int lo_x = 0, hi_x = 0, lo_y = 0, hi_y = 0;
    for (int k = 0; k < P->n_yaw; ++k) {
        double theta = 2.0 * ORC_PI * (double)k / (double)P->n_yaw;
        double cth = cos(theta), sth = sin(theta);
        for (int i = 0; i < P->fp_nl; ++i)
            for (int j = 0; j < P->fp_nw; ++j) {
                double u, v; int p, q;
                if (!in_footprint(P, i, j, &u, &v, &p, &q)) continue;
                double ox = snap((u * cth - v * sth) / P->res);
                double oy = snap((u * sth + v * cth) / P->res);
                double fxd = floor(ox), fyd = floor(oy);
                int ax = (int)fxd, ay = (int)fyd;
                int bx = ax + (ox - fxd > 0.0 ? 1 : 0), by = ay + (oy - fyd > 0.0 ? 1 : 0);
                if (ax < lo_x) lo_x = ax;
                if (bx > hi_x) hi_x = bx;
                if (ay < lo_y) lo_y = ay;
                if (by > hi_y) hi_y = by;
            }
    }
    *dx_min = lo_x; *dx_max = hi_x; *dy_min = lo_y; *dy_max = hi_y;
    return 0;
}

/* rho_full of the configuration's footprint (the scale of the near-degenerate
   threshold, Sec. V-B gate reading) and its sample count n_total. */
double orc_rho_full(const orc_params* P, int32_t* n_total) {
    int n;
    double r = rho_full(P, &n);
    if (n_total) *n_total = n;
    return r;
}

/* The gate of a set of n valid samples given by their integer body-grid
   coordinates (p[m], q[m]) (the sample at body (u, v) = (p du/2, q dv/2)),
   for a footprint of n_total samples whose complete set has rho_full rho_f:
   -1 no fit, 0 fit, 1 near-degenerate fit. */
int orc_gate_points(const int32_t* p, const int32_t* q, int n, int min_valid, int n_total,
                    double rho_f) {
    int64_t N = 0, Sp = 0, Sq = 0, Spp = 0, Spq = 0, Sqq = 0;
    for (int m = 0; m < n; ++m) {
        N += 1; Sp += p[m]; Sq += q[m];
        Spp += (int64_t)p[m] * p[m]; Spq += (int64_t)p[m] * q[m]; Sqq += (int64_t)q[m] * q[m];
    }
    return gate(N, Sp, Sq, Spp, Spq, Sqq, min_valid, n_total, rho_f);
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
