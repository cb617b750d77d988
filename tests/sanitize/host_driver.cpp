// Drives libseb's host code (configuration checks, FP64 footprint tables,
// window geometry, argument validation of every entry point) with the kernel
// launchers and HIP runtime calls replaced by host stand-ins
// (host_stubs.cpp), for the address / undefined-behaviour sanitizer test.
// Test infrastructure only.
#include <cmath>
#include <cstdio>
#include <vector>

#include "seb.h"

static int fails = 0;
#define EXPECT(c) do { if (!(c)) { std::printf("failed: %s (line %d)\n", #c, __LINE__); ++fails; } } while (0)

static seb_config cfg(int W, int H, double res, int K, double L, double Wf, int nl, int nw,
                      int shape = 0, int precision = 0, int fit = 0) {
    seb_config c{};
    c.width = W; c.height = H; c.resolution = res; c.n_yaw = K;
    c.fp_length = L; c.fp_width = Wf; c.fp_nl = nl; c.fp_nw = nw; c.fp_shape = shape;
    c.kappa_max = 0.03; c.phi_x_max = 0.52; c.phi_y_max = 0.52;
    c.w_kappa = c.w_phi_x = c.w_phi_y = 1.0 / 3; c.risk_max = 0.5;
    c.min_valid = 3; c.precision = precision; c.fit = fit;
    return c;
}

int main() {
    const seb_config good[] = {
        cfg(64, 64, 0.1, 16, 0.6, 0.4, 6, 4), cfg(200, 200, 0.1, 36, 1.0, 0.6, 20, 12),
        cfg(400, 400, 0.05, 72, 1.0, 0.6, 20, 12), cfg(800, 800, 0.05, 72, 2.0, 1.2, 40, 24),
        cfg(50, 40, 0.1, 9, 0.6, 0.4, 6, 4, 1, 1, 1), cfg(33, 17, 0.07, 5, 0.5, 0.3, 5, 3, 0, 1, 0)};
    for (const seb_config& c : good) {
        EXPECT(seb_validate_config(&c) == SEB_OK);
        seb_ctx* ctx = nullptr;
        EXPECT(seb_create(&c, &ctx) == SEB_OK);
        if (!ctx) continue;
        const size_t cells = (size_t)c.width * c.height, states = cells * c.n_yaw;
        std::vector<float> h(cells, 0.f), z(states), ro(states), pi(states), ri(states), sdf(states);
        std::vector<uint8_t> st(states);
        seb_out out{z.data(), ro.data(), pi.data(), ri.data(), st.data()};
        EXPECT(seb_assess_se2(ctx, h.data(), c.width, 0, 0, c.width, c.height, &out, nullptr) ==
               SEB_ERR_HIP);                                   // launch: no device here
        EXPECT(seb_assess_se2(ctx, nullptr, c.width, 0, 0, 1, 1, &out, nullptr) == SEB_ERR_INVALID);
        EXPECT(seb_assess_se2(ctx, h.data(), c.width, -1, 0, 1, 1, &out, nullptr) == SEB_ERR_INVALID);
        EXPECT(seb_assess_se2(ctx, h.data(), c.width - 1, 0, 0, 1, 1, &out, nullptr) == SEB_ERR_INVALID);
        seb_window* w = nullptr;
        EXPECT(seb_window_create(ctx, h.data(), c.width, &out, 1.0, -2.0, &w) == SEB_OK);
        if (w) {
            int64_t ox, oy;
            int32_t rx, ry;
            EXPECT(seb_window_origin(w, &ox, &oy, &rx, &ry) == SEB_OK);
            seb_window_plan plan;
            double x = 1.0, y = -2.0;
            for (int s = 0; s < 40; ++s) {
                x += 0.37 * std::cos(0.7 * s) * (s % 9 == 0 ? 40.0 : 1.0);
                y += 0.41 * std::sin(1.3 * s);
                EXPECT(seb_window_plan_move(w, x, y, &plan) == SEB_OK);
                int64_t n = -1;
                const int rc = seb_update_window(w, x, y, nullptr, nullptr, &n);
                EXPECT(rc == SEB_OK || rc == SEB_ERR_HIP);
            }
            seb_window_destroy(w);
        }
        EXPECT(seb_sdf_se2(ctx, st.data(), 0, 0, 8, 1, sdf.data(), nullptr) == SEB_ERR_HIP);
        EXPECT(seb_sdf_se2(ctx, st.data(), 0, 0, 100000, 1, sdf.data(), nullptr) == SEB_ERR_UNSUPPORTED);
        EXPECT(seb_sdf_se2(ctx, st.data(), 0, 0, 0, 1, sdf.data(), nullptr) == SEB_ERR_INVALID);
        std::vector<float> poses(30, 0.1f), q(80);
        EXPECT(seb_query_se2(ctx, sdf.data(), ri.data(), 0, 0, poses.data(), 10, q.data(), nullptr) ==
               SEB_ERR_HIP);
        EXPECT(seb_inpaint_nearest(ctx, h.data(), c.width, 0, 0, 4, z.data(), c.width, nullptr) == SEB_ERR_HIP);
        seb_surrogate* sur = nullptr;
        if (seb_surrogate_create(ctx, &sur) == SEB_OK) {
            EXPECT(seb_surrogate_infer(sur, nullptr, h.data(), c.width, &out, 0.1f, 0.5f, nullptr,
                                       nullptr) == SEB_ERR_INVALID);
            seb_surrogate_destroy(sur);
        }
        seb_fuser* fu = nullptr;
        EXPECT(seb_fuser_create(ctx, 1000, &fu) == SEB_OK);
        seb_scan sc{};
        std::vector<float> pts(3000, 0.5f);
        sc.points = pts.data();
        sc.n_points = 1000;
        sc.R_B[0] = sc.R_B[4] = sc.R_B[8] = 1.0;
        sc.R_BS[0] = sc.R_BS[4] = sc.R_BS[8] = 1.0;
        sc.sigma_range = 0.02;
        sc.z_min = -2.0;
        sc.z_max = 2.0;
        sc.mahalanobis = 3.0;
        if (fu) {
            EXPECT(seb_fuse_scan(fu, h.data(), z.data(), c.width, 0, 0, &sc, nullptr, nullptr) == SEB_ERR_HIP);
            sc.n_points = 1001;
            EXPECT(seb_fuse_scan(fu, h.data(), z.data(), c.width, 0, 0, &sc, nullptr, nullptr) == SEB_ERR_INVALID);
            sc.n_points = 1000;
            seb_fuser_destroy(fu);
        }
        const int rs = seb_fuse_scan_static(ctx, h.data(), z.data(), c.width, 0, 0, &sc, nullptr, nullptr);
        EXPECT(rs == SEB_ERR_HIP || rs == SEB_ERR_INVALID);
        EXPECT(seb_raycast_reset(ctx, h.data(), c.width, 0, 0, &sc, 0.0, nullptr, nullptr) == SEB_ERR_HIP);
        seb_destroy(ctx);
    }
    seb_config bad = cfg(64, 64, 0.1, 16, 0.6, 0.4, 6, 4);
    bad.resolution = NAN;
    EXPECT(seb_validate_config(&bad) == SEB_ERR_INVALID);
    seb_ctx* none = nullptr;
    EXPECT(seb_create(&bad, &none) == SEB_ERR_INVALID && none == nullptr);
    bad = cfg(64, 64, 0.1, 16, 12.0, 12.0, 6, 4);
    EXPECT(seb_validate_config(&bad) == SEB_ERR_UNSUPPORTED);
    seb_window_plan plan;
    const seb_config c5 = good[3];
    for (int s = 0; s < 200; ++s)
        EXPECT(seb_plan_window_move(&c5, 17 * s - 1000, -13 * s, 0.93 * s - 40.0, std::sin(s) * 90.0,
                                    &plan) == SEB_OK);
    for (int code = 1; code >= -6; --code) EXPECT(seb_strerror(code) != nullptr);
    EXPECT(seb_last_error() != nullptr && seb_version() != nullptr);
    std::printf(fails ? "host driver: %d failures\n" : "host driver ok\n", fails);
    return fails != 0;
}
