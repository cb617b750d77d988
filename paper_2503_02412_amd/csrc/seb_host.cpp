// Host side of the SE(2) traversability library: configuration checks, the
// FP64 footprint/yaw table, rolling-window geometry and the C ABI (seb.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "seb.h"
#include "seb_internal.hpp"
#include "seb_net_internal.hpp"
#include "seb_sdf_internal.hpp"
#include "seb_elevation_internal.hpp"
#include "seb_surrogate_internal.hpp"
#include "seb_trace.hpp"

using namespace seb;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return SEB_ERR_HIP;
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kSnap = 1e-6;

int bits_for(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) <= v) ++b;
    return b;
}

// Footprint sample geometry of one body-frame sample (i, j).
struct BodySample {
    int i, j, p, q;
    double u, v;
};

bool footprint_sample(const seb_config& c, int i, int j, BodySample* s) {
    s->i = i;
    s->j = j;
    s->p = 2 * i - (c.fp_nl - 1);
    s->q = 2 * j - (c.fp_nw - 1);
    s->u = (i + 0.5) * c.fp_length / c.fp_nl - 0.5 * c.fp_length;
    s->v = (j + 0.5) * c.fp_width / c.fp_nw - 0.5 * c.fp_width;
    if (c.fp_shape == 1) {
        // inside the inscribed ellipse, decided in exact integers
        const int64_t nl = c.fp_nl, nw = c.fp_nw;
        const int64_t lhs = (int64_t)s->p * s->p * nw * nw + (int64_t)s->q * s->q * nl * nl;
        if (lhs > nl * nl * nw * nw) return false;
    }
    return true;
}

double snap_int(double o) {
    const double r = std::nearbyint(o);
    return std::fabs(o - r) < kSnap ? r : o;
}

// Grid offset of a body sample at yaw theta: o = R(theta) (u, v) / res.
void grid_offset(const seb_config& c, double cth, double sth, const BodySample& s, double* ox,
                 double* oy) {
    *ox = snap_int((s.u * cth - s.v * sth) / c.resolution);
    *oy = snap_int((s.u * sth + s.v * cth) / c.resolution);
}

struct Geometry {
    std::vector<BodySample> samples;      // footprint samples in table order
    std::vector<Segment> segs;
    int n_units = 0, mirror = 0;
    int R = 0;                            // LDS halo (covers the unconditional +1 corner reads)
    int dx_min = 0, dx_max = 0, dy_min = 0, dy_max = 0;   // required-corner reach
    int qoff = 0, w1 = 0, sh2 = 0;
    double rho_full = 0.0;
};

int build_geometry(const seb_config& c, Geometry* g, std::string* why) {
    // Table order: rows of constant body-x index i, samples of increasing j.
    std::vector<std::vector<BodySample>> rows(c.fp_nl);
    for (int i = 0; i < c.fp_nl; ++i)
        for (int j = 0; j < c.fp_nw; ++j) {
            BodySample s;
            if (footprint_sample(c, i, j, &s)) rows[i].push_back(s);
        }
    // Packed integer moments: choose the longest segment whose fields fit 32 bits.
    g->qoff = c.fp_nw - 1;
    const int64_t qmax = g->qoff;
    int seg_len = 0;
    for (int m = std::min(63, c.fp_nw); m >= 1; --m) {
        const int w1 = bits_for((int64_t)m * 2 * qmax);
        const int w2 = bits_for((int64_t)m * qmax * qmax);
        if (6 + w1 + w2 <= 32) {
            seg_len = m;
            g->w1 = w1;
            g->sh2 = 6 + w1;
            break;
        }
    }
    if (seg_len == 0) {
        *why = "footprint sample grid too wide for the packed moments";
        return SEB_ERR_UNSUPPORTED;
    }
    g->samples.clear();
    g->segs.clear();
    for (int i = 0; i < c.fp_nl; ++i) {
        const auto& r = rows[i];
        for (size_t s0 = 0; s0 < r.size(); s0 += seg_len) {
            Segment sg;
            sg.p = 2 * i - (c.fp_nl - 1);
            sg.first = (int)g->samples.size();
            sg.count = (int)std::min<size_t>(seg_len, r.size() - s0);
            sg.pad = 0;
            for (int t = 0; t < sg.count; ++t) g->samples.push_back(r[s0 + t]);
            g->segs.push_back(sg);
        }
    }
    if (g->samples.empty()) {
        *why = "footprint has no samples";
        return SEB_ERR_INVALID;
    }
    // Yaw bins k and k + K/2 share sample positions: compute half, mirror the rest.
    g->mirror = (c.n_yaw % 2 == 0) ? c.n_yaw / 2 : 0;
    g->n_units = g->mirror ? c.n_yaw / 2 : c.n_yaw;

    // Reach over all yaw bins (both halves, to be safe).
    int R = 0, dx0 = 0, dx1 = 0, dy0 = 0, dy1 = 0;
    for (int k = 0; k < c.n_yaw; ++k) {
        const double th = 2.0 * kPi * (double)k / (double)c.n_yaw;
        const double cth = std::cos(th), sth = std::sin(th);
        for (const auto& s : g->samples) {
            double ox, oy;
            grid_offset(c, cth, sth, s, &ox, &oy);
            const double fx = std::floor(ox), fy = std::floor(oy);
            const int ax = (int)fx, ay = (int)fy;
            const int bx = ax + (ox - fx > 0.0 ? 1 : 0), by = ay + (oy - fy > 0.0 ? 1 : 0);
            dx0 = std::min(dx0, ax);
            dx1 = std::max(dx1, bx);
            dy0 = std::min(dy0, ay);
            dy1 = std::max(dy1, by);
            R = std::max({R, -ax, ax + 1, -ay, ay + 1});
        }
    }
    g->R = R;
    g->dx_min = dx0;
    g->dx_max = dx1;
    g->dy_min = dy0;
    g->dy_max = dy1;

    // Scale of the near-degenerate test: 4 det / (D + E)^2 of the full footprint.
    int64_t N = 0, Sp = 0, Sq = 0, Spp = 0, Spq = 0, Sqq = 0;
    for (const auto& s : g->samples) {
        N += 1;
        Sp += s.p;
        Sq += s.q;
        Spp += (int64_t)s.p * s.p;
        Spq += (int64_t)s.p * s.q;
        Sqq += (int64_t)s.q * s.q;
    }
    const int64_t D = N * Spp - Sp * Sp, E = N * Sqq - Sq * Sq, F = N * Spq - Sp * Sq;
    const int64_t det = D * E - F * F;
    const double de = (double)(D + E);
    g->rho_full = (de > 0) ? (4.0 * (double)det) / (de * de) : 0.0;
    return SEB_OK;
}

int validate(const seb_config* c, std::string* why) {
    if (!c) {
        *why = "config is NULL";
        return SEB_ERR_INVALID;
    }
    if (c->width < 1 || c->height < 1 || c->width > (1 << 20) || c->height > (1 << 20)) {
        *why = "width/height must be in [1, 2^20]";
        return SEB_ERR_INVALID;
    }
    if ((int64_t)c->width * c->height * std::max(c->n_yaw, 1) > (int64_t(1) << 40)) {
        *why = "too many states";
        return SEB_ERR_INVALID;
    }
    if (!(c->resolution > 0.0) || !std::isfinite(c->resolution)) {
        *why = "resolution must be positive";
        return SEB_ERR_INVALID;
    }
    if (c->n_yaw < 1 || c->n_yaw > 4096) {
        *why = "n_yaw must be in [1, 4096]";
        return SEB_ERR_INVALID;
    }
    if (!(c->fp_length > 0.0) || !(c->fp_width > 0.0) || !std::isfinite(c->fp_length) ||
        !std::isfinite(c->fp_width)) {
        *why = "footprint extents must be positive";
        return SEB_ERR_INVALID;
    }
    if (c->fp_nl < 1 || c->fp_nw < 1 || c->fp_nl > 4096 || c->fp_nw > 4096) {
        *why = "footprint sample grid must be in [1, 4096]^2";
        return SEB_ERR_INVALID;
    }
    if (c->fp_shape != 0 && c->fp_shape != 1) {
        *why = "fp_shape must be 0 (rectangle) or 1 (ellipse)";
        return SEB_ERR_INVALID;
    }
    if (!(c->kappa_max > 0.0) || !(c->phi_x_max > 0.0) || !(c->phi_y_max > 0.0)) {
        *why = "kappa_max, phi_x_max and phi_y_max must be positive";
        return SEB_ERR_INVALID;
    }
    if (!std::isfinite(c->w_kappa) || !std::isfinite(c->w_phi_x) || !std::isfinite(c->w_phi_y) ||
        !std::isfinite(c->risk_max)) {
        *why = "risk weights and risk_max must be finite";
        return SEB_ERR_INVALID;
    }
    if (c->min_valid < 3) {
        *why = "min_valid must be >= 3";
        return SEB_ERR_INVALID;
    }
    if (c->precision != 0 && c->precision != 1) {
        *why = "precision must be 0 or 1";
        return SEB_ERR_INVALID;
    }
    if (c->fit != 0 && c->fit != 1) {
        *why = "fit must be 0 or 1";
        return SEB_ERR_INVALID;
    }
    if ((int64_t)c->fp_nl * c->fp_nw > 65536) {
        *why = "at most 65536 footprint samples are supported";
        return SEB_ERR_UNSUPPORTED;
    }
    return SEB_OK;
}

int64_t floor_div_cell(double x, double res) { return (int64_t)std::floor(x / res); }

int64_t pos_mod(int64_t a, int64_t n) {
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

}  // namespace

struct seb_ctx {
    seb_config cfg;
    Geometry geo;
    int pitch = 0;
    int fpitch = 0;                       // pitch of the surrogate's fallback kernel
    int row_len = 0;
    float4* d_wts = nullptr;
    int32_t* d_offs = nullptr;
    int32_t* d_offs_f = nullptr;          // offsets at fpitch (d_offs when equal)
    double2* d_frac = nullptr;
    float* d_qs = nullptr;
    uint32_t* d_pks = nullptr;
    Segment* d_segs = nullptr;
    int2* d_inpaint = nullptr;            // (dx, dy) by (dx^2 + dy^2, dy, dx), radius <= 16
    std::vector<int> inpaint_count;       // offsets within radius r, r = 0 .. 16
    int device = 0;
};

struct seb_fuser {
    seb_ctx* ctx;
    int64_t max_points;
    std::vector<void*> allocs;
    elev::FuseWork w;
};

struct seb_surrogate {
    seb_ctx* ctx;
    std::vector<void*> allocs;
    seb::sur::SurArgs ws;   // workspace pointers and map geometry
};

struct seb_window {
    seb_ctx* ctx;
    float* ring;
    int64_t ld;
    seb_out out;
    int64_t ox, oy;    // world cell of logical (0, 0)
};

namespace {

// Fill the per-call part of the kernel arguments.
void base_args(const seb_ctx* c, AssessArgs* a) {
    std::memset(a, 0, sizeof(*a));
    const seb_config& g = c->cfg;
    a->W = g.width;
    a->H = g.height;
    a->wts = c->d_wts;
    a->offs = c->d_offs;
    a->frac = c->d_frac;
    a->qs = c->d_qs;
    a->pks = c->d_pks;
    a->segs = c->d_segs;
    a->row_len = c->row_len;
    a->n_units = c->geo.n_units;
    a->mirror = c->geo.mirror;
    a->n_samples = (int)c->geo.samples.size();
    a->n_segs = (int)c->geo.segs.size();
    a->K = g.n_yaw;
    a->R = c->geo.R;
    a->qoff = c->geo.qoff;
    a->mask1 = (uint32_t)((1u << c->geo.w1) - 1u);
    a->sh2 = c->geo.sh2;
    a->hu = (float)(0.5 * g.fp_length / g.fp_nl);
    a->hv = (float)(0.5 * g.fp_width / g.fp_nw);
    a->inv_hu = (float)(2.0 * g.fp_nl / g.fp_length);
    a->inv_hv = (float)(2.0 * g.fp_nw / g.fp_width);
    a->c_kappa = (float)(g.w_kappa / g.kappa_max);
    a->c_phi_x = (float)(g.w_phi_x / g.phi_x_max);
    a->c_phi_y = (float)(g.w_phi_y / g.phi_y_max);
    a->rho16 = c->geo.rho_full / 16.0;
    a->n_total = (int)c->geo.samples.size();
    a->kappa_max = (float)g.kappa_max;
    a->phi_x_max = (float)g.phi_x_max;
    a->phi_y_max = (float)g.phi_y_max;
    a->w_kappa = (float)g.w_kappa;
    a->w_phi_x = (float)g.w_phi_x;
    a->w_phi_y = (float)g.w_phi_y;
    a->risk_max = (float)g.risk_max;
    a->min_valid = g.min_valid;
    a->precision = g.precision;
    a->fit = g.fit;
}

// Tile decomposition of the state rectangles; chooses the yaw bins per workgroup.
void set_rects(AssessArgs* a, int n, const int32_t (*rects)[4], int pitch) {
    a->n_rects = 0;
    int start = 0;
    // Pairing edge tiles doubles the LDS block; only where 8 workgroups (32
    // waves) still fit in a CU's 160 KB.
    const bool pair_ok = edge_pair_lds(a->R, pitch) <= 20 * 1024;
    for (int r = 0; r < n; ++r) {
        if (rects[r][2] <= 0 || rects[r][3] <= 0) continue;
        const int i = a->n_rects++;
        for (int t = 0; t < 4; ++t) a->rect[i][t] = rects[r][t];
        a->tiles_x[i] = (rects[r][2] + TILE - 1) / TILE;
        a->tiles_y[i] = (rects[r][3] + TILE - 1) / TILE;
        const int rem = rects[r][2] % TILE;
        a->edge_pair[i] = pair_ok && rem >= 1 && rem <= TILE / 2;
        a->tile_start[i] = start;
        start += a->edge_pair[i] ? (a->tiles_x[i] - 1) * a->tiles_y[i] + (a->tiles_y[i] + 1) / 2
                                 : a->tiles_x[i] * a->tiles_y[i];
    }
    a->tile_start[a->n_rects] = start;
    // One yaw unit per workgroup: the most workgroups and the best balance
    // over 256 CUs (measured faster than grouping units on every workload).
    a->units_per_group = 1;
}

int check_out(const seb_out* o) {
    if (!o || !o->z || !o->roll || !o->pitch || !o->risk || !o->status)
        return fail(SEB_ERR_INVALID, "output arrays must all be non-NULL");
    return SEB_OK;
}

int run_assess(seb_ctx* c, const float* height, int64_t ld, int rx, int ry, const seb_out* out,
               int n_rects, const int32_t (*rects)[4], hipStream_t stream,
               const InsertArgs* ins = nullptr) {
    AssessArgs a;
    base_args(c, &a);
    a.height = height;
    a.ld = ld;
    a.rx = rx;
    a.ry = ry;
    a.z = out->z;
    a.roll = out->roll;
    a.pitch = out->pitch;
    a.risk = out->risk;
    a.status = out->status;
    set_rects(&a, n_rects, rects, c->pitch);
    if (ins) {
        // the move's ring insert rides on the assessment: its cells in chunks of
        // BLOCK, spread over the launch's unit groups
        a.ins = *ins;
        a.ins_on = 1;
        const int64_t n = (int64_t)ins->rows_n * ins->W + (int64_t)ins->cols_n * (ins->H - ins->rows_n);
        const int64_t groups = (a.n_units + a.units_per_group - 1) / a.units_per_group;
        const int64_t chunks = (n + BLOCK - 1) / BLOCK;
        a.ins_blocks = (int32_t)((chunks + groups - 1) / groups);
    }
    const hipError_t e = launch_assess(a, c->pitch, stream);
    if (e != hipSuccess) return hip_fail(e, "assessment kernel launch");
    return SEB_OK;
}

// Band of states whose footprint reaches a changed cell, as disjoint rects.
void plan_geometry(const seb_config& cfg, const Geometry& g, int64_t ox, int64_t oy,
                   int64_t nox, int64_t noy, seb_window_plan* p) {
    const int W = cfg.width, H = cfg.height;
    std::memset(p, 0, sizeof(*p));
    p->old_origin_x = ox;
    p->old_origin_y = oy;
    p->new_origin_x = nox;
    p->new_origin_y = noy;
    const int64_t dx = nox - ox, dy = noy - oy;
    if (std::llabs(dx) >= W || std::llabs(dy) >= H) {
        p->full_reset = 1;
        p->exposed_rows = H;
        p->exposed_cols = 0;
        p->n_cells_exposed = (int64_t)W * H;
        p->n_rects = 1;
        p->rects[0][0] = 0;
        p->rects[0][1] = 0;
        p->rects[0][2] = W;
        p->rects[0][3] = H;
        p->n_states = (int64_t)W * H * cfg.n_yaw;
        return;
    }
    const int ady = (int)std::llabs(dy), adx = (int)std::llabs(dx);
    p->exposed_rows = ady;
    p->exposed_cols = adx;
    p->n_cells_exposed = (int64_t)ady * W + (int64_t)adx * (H - ady);

    // State intervals along one axis affected by a shift d of that axis.
    auto intervals = [](int d, int n, int lo_reach, int hi_reach, std::vector<std::pair<int, int>>* iv) {
        // lo_reach = -min offset (>= 0), hi_reach = max offset (>= 0)
        if (d > 0) {
            iv->push_back({n - d - hi_reach, n});      // reach the new cells [n-d, n)
            iv->push_back({0, lo_reach});              // reach the cells that left (< 0)
        } else if (d < 0) {
            iv->push_back({0, -d + lo_reach});         // reach the new cells [0, -d)
            iv->push_back({n - hi_reach, n});          // reach the cells that left (>= n)
        }
    };
    auto merge = [](std::vector<std::pair<int, int>> iv, int n) {
        std::vector<std::pair<int, int>> out;
        for (auto& x : iv) {
            x.first = std::max(0, x.first);
            x.second = std::min(n, x.second);
        }
        std::sort(iv.begin(), iv.end());
        for (auto& x : iv) {
            if (x.first >= x.second) continue;
            if (!out.empty() && x.first <= out.back().second)
                out.back().second = std::max(out.back().second, x.second);
            else
                out.push_back(x);
        }
        return out;
    };
    std::vector<std::pair<int, int>> rv, cv;
    intervals((int)dy, H, -g.dy_min, g.dy_max, &rv);
    intervals((int)dx, W, -g.dx_min, g.dx_max, &cv);
    rv = merge(rv, H);
    cv = merge(cv, W);
    int n = 0;
    int64_t states = 0;
    for (auto& r : rv) {
        p->rects[n][0] = 0;
        p->rects[n][1] = r.first;
        p->rects[n][2] = W;
        p->rects[n][3] = r.second - r.first;
        states += (int64_t)W * (r.second - r.first);
        ++n;
    }
    // Rows not covered by row bands, crossed with the column bands.
    std::vector<std::pair<int, int>> rem;
    int y = 0;
    for (auto& r : rv) {
        if (r.first > y) rem.push_back({y, r.first});
        y = r.second;
    }
    if (y < H) rem.push_back({y, H});
    for (auto& rr : rem)
        for (auto& cc : cv) {
            p->rects[n][0] = cc.first;
            p->rects[n][1] = rr.first;
            p->rects[n][2] = cc.second - cc.first;
            p->rects[n][3] = rr.second - rr.first;
            states += (int64_t)(cc.second - cc.first) * (rr.second - rr.first);
            ++n;
        }
    p->n_rects = n;
    p->n_states = states * cfg.n_yaw;
}

void origin_for(const seb_config& cfg, double x, double y, int64_t* ox, int64_t* oy) {
    // Eq. 4: the map frame sits at the robot's cell; the window is centred on it.
    *ox = floor_div_cell(x, cfg.resolution) - cfg.width / 2;
    *oy = floor_div_cell(y, cfg.resolution) - cfg.height / 2;
}

}  // namespace

extern "C" {

int seb_validate_config(const seb_config* cfg) {
    std::string why;
    int rc = validate(cfg, &why);
    if (rc != SEB_OK) return fail(rc, why);
    Geometry g;
    rc = build_geometry(*cfg, &g, &why);
    if (rc != SEB_OK) return fail(rc, why);
    if (pick_pitch(g.R) == 0) return fail(SEB_ERR_UNSUPPORTED, "footprint reach exceeds the widest LDS tile (64 cells)");
    return SEB_OK;
}

int seb_create(const seb_config* cfg, seb_ctx** out) {
    SEB_TRACE_RANGE();
    if (!out) return fail(SEB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int rc = seb_validate_config(cfg);
    if (rc != SEB_OK) return rc;
    seb_ctx* c = new (std::nothrow) seb_ctx();
    if (!c) return fail(SEB_ERR_ALLOC, "host allocation failed");
    c->cfg = *cfg;
    std::string why;
    build_geometry(*cfg, &c->geo, &why);
    c->pitch = pick_pitch(c->geo.R);
    // The fallback kernel takes 32 x 32 blocks when their halo fits a pitch:
    // four times as many flagged cells per block fill its 64-lane items.
    c->fpitch = c->pitch;
    for (int p : {48, 80, 112, 144})
        if (p >= 32 + 2 * c->geo.R) {
            c->fpitch = std::max(p, c->pitch);
            break;
        }
    (void)hipGetDevice(&c->device);

    // FP64 table: per yaw bin, per sample, the snapped grid offset split into
    // an integer corner and bilinear fractions.
    const Geometry& g = c->geo;
    const int ns = (int)g.samples.size();
    std::vector<float4> wts((size_t)g.n_units * ns);
    std::vector<int32_t> offs((size_t)g.n_units * ns), offs_f((size_t)g.n_units * ns);
    std::vector<double2> frac((size_t)g.n_units * ns);
    std::vector<float> qs(ns);
    std::vector<uint32_t> pks(ns);
    for (int s = 0; s < ns; ++s) {
        const BodySample& b = g.samples[s];
        qs[s] = (float)b.q;
        pks[s] = 1u | ((uint32_t)(b.q + g.qoff) << 6) | ((uint32_t)(b.q * b.q) << g.sh2);
    }
    for (int u = 0; u < g.n_units; ++u) {
        const double th = 2.0 * kPi * (double)u / (double)cfg->n_yaw;
        const double cth = std::cos(th), sth = std::sin(th);
        for (int s = 0; s < ns; ++s) {
            double ox, oy;
            grid_offset(*cfg, cth, sth, g.samples[s], &ox, &oy);
            const double flx = std::floor(ox), fly = std::floor(oy);
            const double fx = ox - flx, fy = oy - fly;
            const size_t e = (size_t)u * ns + s;
            offs[e] = (int)fly * c->pitch + (int)flx;
            offs_f[e] = (int)fly * c->fpitch + (int)flx;
            wts[e] = make_float4((float)((1.0 - fx) * (1.0 - fy)), (float)(fx * (1.0 - fy)),
                                 (float)((1.0 - fx) * fy), (float)(fx * fy));
            frac[e] = make_double2(fx, fy);
        }
    }
    // The unrolled row kernels need every segment to be one full row.
    c->row_len = 0;
    if (has_row_kernel(cfg->fp_nw) && (int)g.segs.size() == cfg->fp_nl) {
        bool rows = true;
        for (size_t i = 0; i < g.segs.size(); ++i)
            rows = rows && g.segs[i].count == cfg->fp_nw && g.segs[i].first == (int)i * cfg->fp_nw;
        if (rows) c->row_len = cfg->fp_nw;
    }
    // Inpainting offsets, nearest first (ties: smaller dy, then smaller dx).
    std::vector<int2> ioffs;
    const int rmax = elev::INPAINT_MAX_RADIUS;
    for (int dy = -rmax; dy <= rmax; ++dy)
        for (int dx = -rmax; dx <= rmax; ++dx) {
            const int d2 = dx * dx + dy * dy;
            if (d2 > 0 && d2 <= rmax * rmax) ioffs.push_back(make_int2(dx, dy));
        }
    std::sort(ioffs.begin(), ioffs.end(), [](const int2& p, const int2& q) {
        const int dp = p.x * p.x + p.y * p.y, dq = q.x * q.x + q.y * q.y;
        if (dp != dq) return dp < dq;
        if (p.y != q.y) return p.y < q.y;
        return p.x < q.x;
    });
    c->inpaint_count.assign(rmax + 1, 0);
    for (int r = 0; r <= rmax; ++r)
        for (const int2& o : ioffs) c->inpaint_count[r] += o.x * o.x + o.y * o.y <= r * r;
    hipError_t e;
    auto upload = [&](void** dst, const void* src, size_t bytes) {
        if ((e = hipMalloc(dst, bytes)) != hipSuccess) return false;
        return (e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice)) == hipSuccess;
    };
    if (!upload((void**)&c->d_wts, wts.data(), wts.size() * sizeof(float4)) ||
        !upload((void**)&c->d_offs, offs.data(), offs.size() * sizeof(int32_t)) ||
        (c->fpitch != c->pitch &&
         !upload((void**)&c->d_offs_f, offs_f.data(), offs_f.size() * sizeof(int32_t))) ||
        !upload((void**)&c->d_frac, frac.data(), frac.size() * sizeof(double2)) ||
        !upload((void**)&c->d_qs, qs.data(), qs.size() * sizeof(float)) ||
        !upload((void**)&c->d_pks, pks.data(), pks.size() * sizeof(uint32_t)) ||
        !upload((void**)&c->d_segs, g.segs.data(), g.segs.size() * sizeof(Segment)) ||
        !upload((void**)&c->d_inpaint, ioffs.data(), ioffs.size() * sizeof(int2))) {
        const int code = (e == hipErrorOutOfMemory) ? SEB_ERR_ALLOC : SEB_ERR_HIP;
        g_last_error = std::string("table upload: ") + hipGetErrorString(e);
        seb_destroy(c);
        return code;
    }
    if (c->fpitch == c->pitch) c->d_offs_f = c->d_offs;
    *out = c;
    return SEB_OK;
}

void seb_destroy(seb_ctx* c) {
    if (!c) return;
    if (c->d_offs_f && c->d_offs_f != c->d_offs) (void)hipFree(c->d_offs_f);
    for (void* p : {(void*)c->d_wts, (void*)c->d_offs, (void*)c->d_frac, (void*)c->d_qs,
                    (void*)c->d_pks, (void*)c->d_segs, (void*)c->d_inpaint})
        if (p) (void)hipFree(p);
    delete c;
}

int seb_assess_se2(seb_ctx* c, const float* height, int64_t ld, int32_t x0, int32_t y0,
                   int32_t nx, int32_t ny, const seb_out* out, void* stream) {
    SEB_TRACE_RANGE();
    if (!c) return fail(SEB_ERR_INVALID, "ctx is NULL");
    if (nx < 0 || ny < 0) return fail(SEB_ERR_INVALID, "nx and ny must be >= 0");
    if (nx == 0 || ny == 0) return SEB_OK;
    if (!height) return fail(SEB_ERR_INVALID, "height is NULL");
    int rc = check_out(out);
    if (rc != SEB_OK) return rc;
    if (ld < c->cfg.width) return fail(SEB_ERR_INVALID, "ld must be >= width");
    if (x0 < 0 || y0 < 0 || (int64_t)x0 + nx > c->cfg.width || (int64_t)y0 + ny > c->cfg.height)
        return fail(SEB_ERR_INVALID, "state rectangle outside the map");
    const int32_t rect[1][4] = {{x0, y0, nx, ny}};
    return run_assess(c, height, ld, 0, 0, out, 1, rect, (hipStream_t)stream);
}

int seb_window_create(seb_ctx* c, float* height_ring, int64_t ld, const seb_out* out_ring,
                      double x, double y, seb_window** out) {
    SEB_TRACE_RANGE();
    if (!out) return fail(SEB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!c || !height_ring) return fail(SEB_ERR_INVALID, "ctx and height_ring must be non-NULL");
    int rc = check_out(out_ring);
    if (rc != SEB_OK) return rc;
    if (ld < c->cfg.width) return fail(SEB_ERR_INVALID, "ld must be >= width");
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(SEB_ERR_INVALID, "position not finite");
    seb_window* w = new (std::nothrow) seb_window();
    if (!w) return fail(SEB_ERR_ALLOC, "host allocation failed");
    w->ctx = c;
    w->ring = height_ring;
    w->ld = ld;
    w->out = *out_ring;
    origin_for(c->cfg, x, y, &w->ox, &w->oy);
    *out = w;
    return SEB_OK;
}

void seb_window_destroy(seb_window* w) { delete w; }

int seb_window_origin(const seb_window* w, int64_t* origin_x, int64_t* origin_y, int32_t* ring_x,
                      int32_t* ring_y) {
    if (!w) return fail(SEB_ERR_INVALID, "window is NULL");
    if (origin_x) *origin_x = w->ox;
    if (origin_y) *origin_y = w->oy;
    if (ring_x) *ring_x = (int32_t)pos_mod(w->ox, w->ctx->cfg.width);
    if (ring_y) *ring_y = (int32_t)pos_mod(w->oy, w->ctx->cfg.height);
    return SEB_OK;
}

int seb_window_reset(seb_window* w, double x, double y, const float* heights, int64_t ld,
                     void* stream) {
    SEB_TRACE_RANGE();
    if (!w) return fail(SEB_ERR_INVALID, "window is NULL");
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(SEB_ERR_INVALID, "position not finite");
    seb_ctx* c = w->ctx;
    if (heights && ld < c->cfg.width) return fail(SEB_ERR_INVALID, "ld must be >= width");
    origin_for(c->cfg, x, y, &w->ox, &w->oy);
    InsertArgs ia;
    std::memset(&ia, 0, sizeof(ia));
    ia.ring = w->ring;
    ia.ld = w->ld;
    ia.W = c->cfg.width;
    ia.H = c->cfg.height;
    ia.rx = (int)pos_mod(w->ox, ia.W);
    ia.ry = (int)pos_mod(w->oy, ia.H);
    ia.src = heights;
    ia.src_ld = ld;
    ia.full = 1;
    hipError_t e = launch_insert(ia, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ring insert launch");
    const int32_t rect[1][4] = {{0, 0, c->cfg.width, c->cfg.height}};
    return run_assess(c, w->ring, w->ld, ia.rx, ia.ry, &w->out, 1, rect, (hipStream_t)stream);
}

int seb_window_plan_move(const seb_window* w, double x, double y, seb_window_plan* plan) {
    if (!w || !plan) return fail(SEB_ERR_INVALID, "window and plan must be non-NULL");
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(SEB_ERR_INVALID, "position not finite");
    int64_t nox, noy;
    origin_for(w->ctx->cfg, x, y, &nox, &noy);
    plan_geometry(w->ctx->cfg, w->ctx->geo, w->ox, w->oy, nox, noy, plan);
    return SEB_OK;
}

int seb_plan_window_move(const seb_config* cfg, int64_t origin_x, int64_t origin_y, double x,
                         double y, seb_window_plan* plan) {
    if (!plan) return fail(SEB_ERR_INVALID, "plan is NULL");
    int rc = seb_validate_config(cfg);
    if (rc != SEB_OK) return rc;
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(SEB_ERR_INVALID, "position not finite");
    Geometry g;
    std::string why;
    build_geometry(*cfg, &g, &why);
    int64_t nox, noy;
    origin_for(*cfg, x, y, &nox, &noy);
    plan_geometry(*cfg, g, origin_x, origin_y, nox, noy, plan);
    return SEB_OK;
}

int seb_update_window(seb_window* w, double x, double y, const float* new_cells, void* stream,
                      int64_t* n_states_recomputed) {
    SEB_TRACE_RANGE();
    seb_window_plan p;
    int rc = seb_window_plan_move(w, x, y, &p);
    if (rc != SEB_OK) return rc;
    seb_ctx* c = w->ctx;
    const int W = c->cfg.width, H = c->cfg.height;
    InsertArgs ia;
    std::memset(&ia, 0, sizeof(ia));
    ia.ring = w->ring;
    ia.ld = w->ld;
    ia.W = W;
    ia.H = H;
    ia.rx = (int)pos_mod(p.new_origin_x, W);
    ia.ry = (int)pos_mod(p.new_origin_y, H);
    ia.src = new_cells;
    const int64_t dx = p.new_origin_x - p.old_origin_x, dy = p.new_origin_y - p.old_origin_y;
    if (p.full_reset) {
        ia.full = 1;
        ia.src_ld = W;
    } else {
        ia.rows_n = p.exposed_rows;
        ia.rows_lo = dy > 0 ? H - (int)dy : 0;
        ia.cols_n = p.exposed_cols;
        ia.cols_lo = dx > 0 ? W - (int)dx : 0;
    }
    w->ox = p.new_origin_x;
    w->oy = p.new_origin_y;
    if (n_states_recomputed) *n_states_recomputed = p.n_states;
    if (p.full_reset || p.n_rects == 0) {
        hipError_t e = launch_insert(ia, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "ring insert launch");
        if (p.n_rects == 0) return SEB_OK;
        return run_assess(c, w->ring, w->ld, ia.rx, ia.ry, &w->out, p.n_rects, p.rects,
                          (hipStream_t)stream);
    }
    // A partial move: one launch assesses the band, staging the exposed cells
    // from new_cells, and writes them into the ring.
    return run_assess(c, w->ring, w->ld, ia.rx, ia.ry, &w->out, p.n_rects, p.rects,
                      (hipStream_t)stream, &ia);
}

int seb_surrogate_create(seb_ctx* c, seb_surrogate** out) {
    SEB_TRACE_RANGE();
    if (!out) return fail(SEB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!c) return fail(SEB_ERR_INVALID, "ctx is NULL");
    if (c->geo.n_units > 128)
        return fail(SEB_ERR_UNSUPPORTED, "the surrogate supports at most 128 yaw units (256 bins)");
    seb_surrogate* s = new (std::nothrow) seb_surrogate();
    if (!s) return fail(SEB_ERR_ALLOC, "host allocation failed");
    s->ctx = c;
    const int64_t W = c->cfg.width, H = c->cfg.height, cells = W * H;
    const int U = c->geo.n_units;
    auto al = [&](void** p, size_t bytes) {
        if (hipMalloc(p, bytes) != hipSuccess) return false;
        s->allocs.push_back(*p);
        return true;
    };
    seb::sur::SurArgs& w = s->ws;
    std::memset(&w, 0, sizeof(w));
    // fallback lists: per (unit, block of tf x tf cells) a count per block row
    // and the row's columns
    const int tf = flagged_tile(c->geo.R, c->fpitch);
    const int64_t n_slots = flagged_blocks((int)W, (int)H, U, c->geo.R, c->fpitch);
    const bool ok =
        al((void**)&w.yaw_sc, (size_t)U * sizeof(float2)) &&
        al((void**)&w.o2map, (size_t)(H + 16) * (W + 16) * seb::net::C2 * 2) &&
        al((void**)&w.ymap, (size_t)U * seb::net::H1 * 2) &&
        al((void**)&w.known, (size_t)cells * 4) &&
        al((void**)&w.row_count, (size_t)n_slots * tf) &&
        al((void**)&w.work_cols, (size_t)n_slots * tf * tf);
    if (!ok) {
        seb_surrogate_destroy(s);
        return fail(SEB_ERR_ALLOC, "device allocation failed");
    }
    // Counts of block rows past the map's edge are never written: zero once.
    const std::vector<uint8_t> zeros((size_t)n_slots * tf, 0);
    if (hipMemcpy(w.row_count, zeros.data(), zeros.size(), hipMemcpyHostToDevice) != hipSuccess) {
        seb_surrogate_destroy(s);
        return fail(SEB_ERR_HIP, "fallback list initialisation failed");
    }
    w.tf = tf;
    w.blocks_x = (int)((W + tf - 1) / tf);
    w.blocks = w.blocks_x * (int)((H + tf - 1) / tf);
    {
        // (sin, cos) of each evaluated yaw unit's angle 2 pi u / K, in FP64
        std::vector<float2> sc(U);
        for (int u = 0; u < U; ++u) {
            const double th = 2.0 * M_PI * (double)u / (double)c->cfg.n_yaw;
            sc[u] = make_float2((float)std::sin(th), (float)std::cos(th));
        }
        if (hipMemcpy((void*)w.yaw_sc, sc.data(), sc.size() * sizeof(float2),
                      hipMemcpyHostToDevice) != hipSuccess) {
            seb_surrogate_destroy(s);
            return fail(SEB_ERR_HIP, "yaw table upload failed");
        }
    }
    w.W = (int)W;
    w.H = (int)H;
    w.inv_res = (float)(1.0 / c->cfg.resolution);
    w.K = c->cfg.n_yaw;
    w.U = U;
    w.mirror = c->geo.mirror;
    w.pitch = c->fpitch;
    w.risk_max = (float)c->cfg.risk_max;
    *out = s;
    return SEB_OK;
}

void seb_surrogate_destroy(seb_surrogate* s) {
    if (!s) return;
    for (void* p : s->allocs) (void)hipFree(p);
    delete s;
}

int seb_surrogate_infer(seb_surrogate* s, const seb_net* net, const float* height, int64_t ld,
                        const seb_out* out, float band, float min_known, int32_t* n_fallback_dev,
                        void* stream) {
    SEB_TRACE_RANGE();
    if (!s || !net || !height) return fail(SEB_ERR_INVALID, "surrogate, net and height must be set");
    int rc = check_out(out);
    if (rc != SEB_OK) return rc;
    if (ld < s->ws.W) return fail(SEB_ERR_INVALID, "ld must be >= width");
    if (!(band >= 0.f) || !(min_known >= 0.f) || !(min_known <= 1.f))
        return fail(SEB_ERR_INVALID, "band must be >= 0 and min_known in [0, 1]");
    seb::sur::SurArgs w = s->ws;
    w.height = height;
    w.ld = ld;
    w.theta = seb::net::net_theta(net);
    w.pw = seb::net::net_packed(net);
    w.band = band;
    w.min_known = min_known;
    w.n_fallback = n_fallback_dev;
    AssessArgs a;
    base_args(s->ctx, &a);
    a.height = height;
    a.ld = ld;
    a.z = out->z;
    a.roll = out->roll;
    a.pitch = out->pitch;
    a.risk = out->risk;
    a.status = out->status;
    hipError_t e = seb::sur::launch_surrogate(w, a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "surrogate launch");
    // The plain method for the listed states.
    a.count = n_fallback_dev;
    a.row_count = w.row_count;
    a.work_cols = w.work_cols;
    a.offs = s->ctx->d_offs_f;
    e = launch_assess_flagged(a, s->ctx->fpitch, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fallback assessment launch");
    return SEB_OK;
}

int seb_fuser_create(seb_ctx* c, int64_t max_points, seb_fuser** out) {
    SEB_TRACE_RANGE();
    if (!out) return fail(SEB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!c) return fail(SEB_ERR_INVALID, "ctx is NULL");
    if (max_points < 1 || max_points >= (int64_t(1) << 31))
        return fail(SEB_ERR_INVALID, "max_points must be in [1, 2^31)");
    const int64_t n_cells = (int64_t)c->cfg.width * c->cfg.height;
    if (n_cells >= (int64_t(1) << 31))
        return fail(SEB_ERR_UNSUPPORTED, "elevation fusion needs W * H < 2^31");
    seb_fuser* f = new (std::nothrow) seb_fuser();
    if (!f) return fail(SEB_ERR_ALLOC, "host allocation");
    f->ctx = c;
    f->max_points = max_points;
    auto alloc = [&](void** p, size_t bytes) {
        if (hipMalloc(p, std::max<size_t>(bytes, 4)) != hipSuccess) return false;
        f->allocs.push_back(*p);
        return true;
    };
    elev::FuseWork& w = f->w;
    const size_t np = (size_t)max_points, nc = (size_t)n_cells;
    if (!alloc((void**)&w.cell, np * 4) || !alloc((void**)&w.z, np * 8) ||
        !alloc((void**)&w.var, np * 8) || !alloc((void**)&w.bucket, np * 4) ||
        !alloc((void**)&w.count, nc * 4) || !alloc((void**)&w.fill, nc * 4) ||
        !alloc((void**)&w.offs, nc * 4) ||
        !alloc((void**)&w.partial, (size_t)elev::partial_blocks(n_cells) * 4) ||
        !alloc((void**)&w.large, nc * 4) || !alloc((void**)&w.n_large, 4) ||
        !alloc((void**)&w.n_fused, 4)) {
        seb_fuser_destroy(f);
        return fail(SEB_ERR_ALLOC, "fuser workspace allocation");
    }
    *out = f;
    return SEB_OK;
}

void seb_fuser_destroy(seb_fuser* f) {
    if (!f) return;
    for (void* p : f->allocs) (void)hipFree(p);
    delete f;
}

namespace {

// Checks of a fusion call and its kernel arguments (shared by seb_fuse_scan
// and seb_fuse_scan_static); returns SEB_OK or the error, nothing launched.
int fuse_args(const seb_ctx* c, float* height, float* variance, int64_t ld, int64_t origin_x,
              int64_t origin_y, const seb_scan* sc, int64_t max_points, elev::ScanArgs* out_s,
              elev::FuseArgs* out_a) {
    const seb_config& g = c->cfg;
    if (ld < g.width) return fail(SEB_ERR_INVALID, "ld must be >= width");
    {
        const char* h0 = (const char*)height;
        const char* h1 = (const char*)(height + (int64_t)(g.height - 1) * ld + g.width);
        const char* v0 = (const char*)variance;
        const char* v1 = (const char*)(variance + (int64_t)(g.height - 1) * ld + g.width);
        if (h0 < v1 && v0 < h1) return fail(SEB_ERR_INVALID, "height and variance overlap");
    }
    if (sc->n_points < 0 || sc->n_points > max_points)
        return fail(SEB_ERR_INVALID, "n_points outside [0, max_points]");
    if (sc->n_points > 0 && !sc->points) return fail(SEB_ERR_INVALID, "points is NULL");
    const double* all[] = {sc->R_B, sc->p_B, sc->R_BS, sc->p_BS, sc->Sigma_R, sc->Sigma_B};
    const int len[] = {9, 3, 9, 3, 9, 9};
    for (int k = 0; k < 6; ++k)
        for (int i = 0; i < len[k]; ++i)
            if (!std::isfinite(all[k][i])) return fail(SEB_ERR_INVALID, "pose or covariance not finite");
    if (!(sc->sigma_range > 0.0) || !(sc->sigma_angle >= 0.0) || !(sc->Sigma_B[8] >= 0.0) ||
        !std::isfinite(sc->sigma_range) || !std::isfinite(sc->sigma_angle))
        return fail(SEB_ERR_INVALID, "need sigma_range > 0, sigma_angle >= 0, Sigma_B[2][2] >= 0");
    if (!(sc->z_min <= sc->z_max) || !(sc->mahalanobis > 0.0) || !std::isfinite(sc->mahalanobis))
        return fail(SEB_ERR_INVALID, "need z_min <= z_max and mahalanobis > 0");
    if (std::fabs((double)origin_x) > 1e15 || std::fabs((double)origin_y) > 1e15)
        return fail(SEB_ERR_INVALID, "origin out of range");
    elev::ScanArgs& s = *out_s;
    s.pts = sc->points;
    s.n = sc->n_points;
    for (int i = 0; i < 9; ++i) {
        s.A[i] = sc->R_BS[i];
        s.R[i] = sc->R_B[i];
        s.SR[i] = sc->Sigma_R[i];
    }
    for (int i = 0; i < 3; ++i) {
        s.a[i] = sc->p_BS[i];
        s.b[i] = sc->p_B[i];
        // J_S = (R_B R_BS)^T b3: row 2 of R_B R_BS; g = R_B^T b3: row 2 of R_B
        s.js[i] = s.R[6] * s.A[i] + s.R[7] * s.A[3 + i] + s.R[8] * s.A[6 + i];
        s.g[i] = s.R[6 + i];
    }
    s.sb22 = sc->Sigma_B[8];
    s.sr2 = sc->sigma_range * sc->sigma_range;
    s.sa2 = sc->sigma_angle * sc->sigma_angle;
    s.zmin = sc->z_min;
    s.zmax = sc->z_max;
    s.res = g.resolution;
    s.W = g.width;
    s.H = g.height;
    s.ox = origin_x;
    s.oy = origin_y;
    elev::FuseArgs& a = *out_a;
    a.height = height;
    a.variance = variance;
    a.ld = ld;
    a.W = g.width;
    a.H = g.height;
    a.rx = (int32_t)pos_mod(origin_x, g.width);
    a.ry = (int32_t)pos_mod(origin_y, g.height);
    a.tau2 = sc->mahalanobis * sc->mahalanobis;
    return SEB_OK;
}

}  // namespace

int seb_fuse_scan(seb_fuser* f, float* height, float* variance, int64_t ld, int64_t origin_x,
                  int64_t origin_y, const seb_scan* sc, int32_t* n_fused_dev, void* stream) {
    SEB_TRACE_RANGE();
    if (!f || !height || !variance || !sc)
        return fail(SEB_ERR_INVALID, "fuser, height, variance and scan must be non-NULL");
    elev::ScanArgs s;
    elev::FuseArgs a;
    const int rc = fuse_args(f->ctx, height, variance, ld, origin_x, origin_y, sc, f->max_points,
                             &s, &a);
    if (rc != SEB_OK) return rc;
    a.n_fused = n_fused_dev ? n_fused_dev : f->w.n_fused;
    hipError_t e = elev::launch_fuse_scan(s, a, f->w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fusion launch");
    return SEB_OK;
}

int seb_fuse_scan_static(seb_ctx* c, float* height, float* variance, int64_t ld,
                         int64_t origin_x, int64_t origin_y, const seb_scan* sc,
                         int32_t* n_fused_dev, void* stream) {
    SEB_TRACE_RANGE();
    if (!c || !height || !variance || !sc)
        return fail(SEB_ERR_INVALID, "ctx, height, variance and scan must be non-NULL");
    if ((int64_t)c->cfg.width * c->cfg.height > elev::STATIC_MAX_CELLS)
        return fail(SEB_ERR_INVALID, "map larger than the static fusion workspace (2^18 cells)");
    if (sc->n_points > elev::STATIC_MAX_POINTS)
        return fail(SEB_ERR_INVALID, "more points than the static fusion workspace (2^18)");
    elev::ScanArgs s;
    elev::FuseArgs a;
    const int rc = fuse_args(c, height, variance, ld, origin_x, origin_y, sc,
                             elev::STATIC_MAX_POINTS, &s, &a);
    if (rc != SEB_OK) return rc;
    elev::FuseWork w;
    hipError_t e = elev::static_fuse_work(&w);
    if (e != hipSuccess) return hip_fail(e, "static fusion workspace lookup");
    a.n_fused = n_fused_dev ? n_fused_dev : w.n_fused;
    e = elev::launch_fuse_scan(s, a, w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fusion launch");
    return SEB_OK;
}

int seb_raycast_reset(seb_ctx* c, float* height, int64_t ld, int64_t origin_x, int64_t origin_y,
                      const seb_scan* sc, double margin, int32_t* n_reset_dev, void* stream) {
    SEB_TRACE_RANGE();
    if (!c || !height || !sc) return fail(SEB_ERR_INVALID, "ctx, height and scan must be non-NULL");
    const seb_config& g = c->cfg;
    if (ld < g.width) return fail(SEB_ERR_INVALID, "ld must be >= width");
    if (sc->n_points < 0 || sc->n_points >= (int64_t(1) << 40))
        return fail(SEB_ERR_INVALID, "n_points out of range");
    if (sc->n_points > 0 && !sc->points) return fail(SEB_ERR_INVALID, "points is NULL");
    const double* all[] = {sc->R_B, sc->p_B, sc->R_BS, sc->p_BS};
    const int len[] = {9, 3, 9, 3};
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < len[k]; ++i)
            if (!std::isfinite(all[k][i])) return fail(SEB_ERR_INVALID, "pose not finite");
    if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(SEB_ERR_INVALID, "margin must be >= 0");
    if (std::fabs((double)origin_x) > 1e12 || std::fabs((double)origin_y) > 1e12)
        return fail(SEB_ERR_INVALID, "origin out of range");
    elev::RayArgs r;
    r.pts = sc->points;
    r.n = sc->n_points;
    for (int i = 0; i < 9; ++i) {
        r.A[i] = sc->R_BS[i];
        r.R[i] = sc->R_B[i];
    }
    for (int i = 0; i < 3; ++i) {
        r.a[i] = sc->p_BS[i];
        r.b[i] = sc->p_B[i];
    }
    // sensor origin R_B p_BS + p_B, in the reference's order of operations
    r.sx = r.R[0] * r.a[0] + r.R[1] * r.a[1] + r.R[2] * r.a[2] + r.b[0];
    r.sy = r.R[3] * r.a[0] + r.R[4] * r.a[1] + r.R[5] * r.a[2] + r.b[1];
    r.sz = r.R[6] * r.a[0] + r.R[7] * r.a[1] + r.R[8] * r.a[2] + r.b[2];
    r.res = g.resolution;
    r.margin = margin;
    r.W = g.width;
    r.H = g.height;
    r.rx = (int32_t)pos_mod(origin_x, g.width);
    r.ry = (int32_t)pos_mod(origin_y, g.height);
    r.ox = origin_x;
    r.oy = origin_y;
    r.height = height;
    r.ld = ld;
    r.n_reset = n_reset_dev;
    hipError_t e = elev::launch_raycast(r, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ray-casting launch");
    return SEB_OK;
}

int seb_inpaint_nearest(seb_ctx* c, const float* height, int64_t ld, int32_t ring_x,
                        int32_t ring_y, int32_t radius, float* out, int64_t out_ld, void* stream) {
    SEB_TRACE_RANGE();
    if (!c || !height || !out) return fail(SEB_ERR_INVALID, "ctx, height and out must be non-NULL");
    const seb_config& g = c->cfg;
    if (ld < g.width || out_ld < g.width) return fail(SEB_ERR_INVALID, "row strides must be >= width");
    if (ring_x < 0 || ring_x >= g.width || ring_y < 0 || ring_y >= g.height)
        return fail(SEB_ERR_INVALID, "ring offset outside the map");
    if (radius < 0 || radius > elev::INPAINT_MAX_RADIUS)
        return fail(SEB_ERR_INVALID, "radius must be in [0, 16]");
    const char* h0 = (const char*)height;
    const char* h1 = (const char*)(height + (int64_t)(g.height - 1) * ld + g.width);
    const char* o0 = (const char*)out;
    const char* o1 = (const char*)(out + (int64_t)(g.height - 1) * out_ld + g.width);
    if (h0 < o1 && o0 < h1) return fail(SEB_ERR_INVALID, "out overlaps height");
    elev::InpaintArgs a;
    a.src = height;
    a.ld = ld;
    a.dst = out;
    a.dst_ld = out_ld;
    a.W = g.width;
    a.H = g.height;
    a.rx = ring_x;
    a.ry = ring_y;
    a.radius = radius;
    a.offs = c->d_inpaint;
    a.n_offs = c->inpaint_count[radius];
    hipError_t e = elev::launch_inpaint(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "inpaint launch");
    return SEB_OK;
}

int seb_sdf_se2(seb_ctx* c, const uint8_t* status, int32_t ring_x, int32_t ring_y,
                int32_t cap_cells, int32_t unknown_is_obstacle, float* sdf, void* stream) {
    SEB_TRACE_RANGE();
    if (!c || !status || !sdf) return fail(SEB_ERR_INVALID, "ctx, status and sdf must be non-NULL");
    const seb_config& g = c->cfg;
    if (ring_x < 0 || ring_x >= g.width || ring_y < 0 || ring_y >= g.height)
        return fail(SEB_ERR_INVALID, "ring offset outside the map");
    if (cap_cells < 1) return fail(SEB_ERR_INVALID, "cap_cells must be >= 1");
    if (cap_cells > sdf_max_cap())
        return fail(SEB_ERR_UNSUPPORTED, "cap_cells above " + std::to_string(sdf_max_cap()));
    if ((int64_t)g.width * g.height >= (int64_t(1) << 31))
        return fail(SEB_ERR_UNSUPPORTED, "sdf planes of 2^31 cells or more");
    hipError_t e = launch_sdf(status, sdf, g.width, g.height, g.n_yaw, ring_x, ring_y, cap_cells,
                              (float)g.resolution, unknown_is_obstacle != 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sdf launch");
    return SEB_OK;
}

int seb_query_se2(seb_ctx* c, const float* sdf, const float* risk, int32_t ring_x, int32_t ring_y,
                  const float* poses, int64_t n, float* out, void* stream) {
    SEB_TRACE_RANGE();
    if (!c) return fail(SEB_ERR_INVALID, "ctx is NULL");
    if (n < 0) return fail(SEB_ERR_INVALID, "n must be >= 0");
    if (!sdf && !risk) return fail(SEB_ERR_INVALID, "sdf and risk are both NULL");
    const seb_config& g = c->cfg;
    if (ring_x < 0 || ring_x >= g.width || ring_y < 0 || ring_y >= g.height)
        return fail(SEB_ERR_INVALID, "ring offset outside the map");
    if (n == 0) return SEB_OK;
    if (!poses || !out) return fail(SEB_ERR_INVALID, "poses and out must be non-NULL");
    if (((uintptr_t)out & 15) != 0) return fail(SEB_ERR_INVALID, "out must be 16-byte aligned");
    if (n > (int64_t(1) << 40)) return fail(SEB_ERR_INVALID, "n too large");
    hipError_t e = launch_query(sdf, risk, poses, out, n, g.width, g.height, g.n_yaw, ring_x,
                                ring_y, g.resolution, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "query launch");
    return SEB_OK;
}

const char* seb_strerror(int status) {
    switch (status) {
        case SEB_OK: return "success";
        case SEB_ERR_INVALID: return "invalid argument";
        case SEB_ERR_HIP: return "HIP runtime error";
        case SEB_ERR_ALLOC: return "allocation failed";
        case SEB_ERR_UNSUPPORTED: return "unsupported configuration";
        case SEB_ERR_IO: return "I/O error";
        default: return "unknown status";
    }
}

const char* seb_last_error(void) { return g_last_error.c_str(); }

const char* seb_version(void) { return "seb-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"
