/* Runs the FP64 oracle's entry points on small seeded maps with unknown
 * cells, map edges, both fits and both footprint shapes, for the address /
 * undefined-behaviour sanitizer test.  Test infrastructure only. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "seb_oracle.c"

static unsigned long long rng = 88172645463325252ull;
static double uni(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0;
}

int main(void) {
    const int W = 24, H = 20;
    float* h = malloc(sizeof(float) * W * H);
    for (int i = 0; i < W * H; ++i) h[i] = uni() < 0.15 ? NAN : (float)(0.3 * sin(0.4 * i) + 0.05 * uni());
    h[5] = INFINITY;
    h[7] = -INFINITY;
    int fails = 0;
    for (int shape = 0; shape < 2; ++shape)
        for (int fit = 0; fit < 2; ++fit) {
            orc_params P = {W, H, 0.1, 8, 0.6, 0.4, 6, 4, shape, 0.03, 0.52, 0.52,
                            1.0 / 3, 1.0 / 3, 1.0 / 3, 0.5, 3, fit};
            const int n = W * H * P.n_yaw;
            double *z = malloc(8 * n), *ro = malloc(8 * n), *pi = malloc(8 * n), *ri = malloc(8 * n),
                   *ka = malloc(8 * n), *px = malloc(8 * n), *py = malloc(8 * n);
            uint8_t* st = malloc(n);
            int32_t* nv = malloc(4 * n);
            fails += orc_assess_rect(&P, h, W, 0, 0, W, H, 0, P.n_yaw, z, ro, pi, ri, ka, px, py, st,
                                     nv, 2) != 0;
            int32_t ix[5] = {0, W - 1, 3, 10, 0}, iy[5] = {0, H - 1, 4, 9, H - 1}, kk[5] = {0, 7, 3, 4, 5};
            fails += orc_assess_list(&P, h, W, 5, ix, iy, kk, z, ro, pi, ri, ka, px, py, st, nv, 1) != 0;
            int32_t a, b, c, d, nt;
            fails += orc_reach(&P, &a, &b, &c, &d) != 0;
            const double rf = orc_rho_full(&P, &nt);
            int32_t p[3] = {-5, 1, 5}, q[3] = {-3, 3, -1};
            (void)orc_gate_points(p, q, 3, 3, nt, rf);
            free(z); free(ro); free(pi); free(ri); free(ka); free(px); free(py); free(st); free(nv);
        }
    /* rejected arguments */
    orc_params bad = {W, H, 0.1, 8, 0.6, 0.4, 6, 4, 0, 0.03, 0.52, 0.52, 1.0 / 3, 1.0 / 3,
                      1.0 / 3, 0.5, 3, 0};
    double dz[1];
    uint8_t ds[1];
    int32_t dn[1];
    fails += orc_assess_rect(&bad, h, W, 0, 0, -1, 1, 0, 1, dz, dz, dz, dz, dz, dz, dz, ds, dn, 1) == 0;
    bad.res = 0.0;
    fails += orc_assess_rect(&bad, h, W, 0, 0, 1, 1, 0, 1, dz, dz, dz, dz, dz, dz, dz, ds, dn, 1) == 0;
    /* states outside the map are valid queries (every sample out of map: unknown) */
    bad.res = 0.1;
    fails += orc_assess_rect(&bad, h, W, W, H, 1, 1, 0, 1, dz, dz, dz, dz, dz, dz, dz, ds, dn, 1) != 0;
    fails += (ds[0] & 1) != 0;
    free(h);
    printf(fails ? "oracle driver: %d failures\n" : "oracle driver ok\n", fails);
    return fails != 0;
}
