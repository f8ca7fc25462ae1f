/*
 * Memory-safety driver of the FP64 oracle, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host (tests/test_asan.py).  It calls
 * every oracle function on small inputs of many shapes (ragged grids, Haar
 * levels 0..3, non-square frames, both low-pass modes, the illumination
 * term) and checks a few identities on the way, so that an out-of-bounds
 * access or undefined operation in any loop is reported by the sanitizers.
 * Prints "oracle asan ok" and returns 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "hb_oracle.h"

#define NW 7

static int fail(const char *what) {
    fprintf(stderr, "oracle asan: %s\n", what);
    return 1;
}

int main(void) {
    double ehb[NW], eox[NW], resp[3 * NW];
    for (int j = 0; j < NW; ++j) {
        ehb[j] = 0.02 + 0.01 * j;
        eox[j] = 0.05 - 0.005 * j;
        for (int k = 0; k < 3; ++k) resp[k * NW + j] = exp(-0.5 * (j - 2.0 * k - 1.0) * (j - 2.0 * k - 1.0));
    }
    orc_model m = {NW, ehb, eox, resp, 0.1};

    double mu[3], E[6], M[6], g;
    orc_mu(&m, 40.0, 60.0, mu);
    orc_jacobian(&m, 40.0, 60.0, E);
    if (orc_tikhonov(3, E, 1e-3, M, &g) != 0) return fail("tikhonov");
    if (orc_tikhonov(2, E, 0.0, M, &g) != 0) return fail("tikhonov 2x2");

    /* Haar round trips on ragged, non-square frames. */
    const int hw[][3] = {{4, 4, 1}, {8, 12, 2}, {16, 8, 3}, {6, 10, 1}, {5, 7, 0}, {32, 24, 3}};
    for (size_t t = 0; t < sizeof(hw) / sizeof(hw[0]); ++t) {
        const int h = hw[t][0], w = hw[t][1], lv = hw[t][2];
        double *x = malloc(sizeof(double) * h * w), *c = malloc(sizeof(double) * h * w),
               *y = malloc(sizeof(double) * h * w);
        for (int i = 0; i < h * w; ++i) x[i] = sin(0.37 * i) + 0.1 * i;
        orc_haar_forward(x, h, w, lv, c);
        orc_haar_inverse(c, h, w, lv, y);
        for (int i = 0; i < h * w; ++i)
            if (fabs(x[i] - y[i]) > 1e-12 * (1.0 + fabs(x[i]))) return fail("haar round trip");
        free(x);
        free(c);
        free(y);
    }

    /* Whole path over grids, levels, modes and the illumination term. */
    const int cases[][6] = {
        /* h, w, levels, grid_thb, grid_so2, n */
        {8, 8, 1, 1, 1, 1}, {8, 12, 2, 3, 5, 2}, {16, 16, 3, 7, 4, 1}, {12, 20, 0, 4, 4, 2}, {16, 8, 2, 16, 9, 3},
    };
    for (size_t t = 0; t < sizeof(cases) / sizeof(cases[0]); ++t)
        for (int lowpass = 0; lowpass < 2; ++lowpass)
            for (int illum = 0; illum < 2; ++illum) {
                const int h = cases[t][0], w = cases[t][1], n = cases[t][5];
                orc_params p = {w, h, cases[t][2], cases[t][3], cases[t][4], 20.0, 200.0, 0.3, 1.0, 1e-3, 0.01,
                                1e-4, 1e-3, 44.0, 66.0, lowpass, illum};
                const long G = (long)p.grid_thb * p.grid_so2;
                double *c = malloc(sizeof(double) * 2 * G), *gm = malloc(sizeof(double) * 3 * G);
                orc_grid(&p, &m, c, gm);
                double yb[3] = {gm[0] + 0.01, gm[1] - 0.02, gm[2]}, post[2];
                orc_posterior_mean(c, gm, G, yb, p.sigma, illum, post);
                if (!isfinite(post[0]) || !isfinite(post[1])) return fail("posterior");
                double *fr = malloc(sizeof(double) * n * h * w * 3), *maps = malloc(sizeof(double) * n * 4 * h * w);
                for (int i = 0; i < n * h * w * 3; ++i) fr[i] = 0.3 + 0.5 * (0.5 + 0.5 * sin(0.11 * i));
                fr[0] = -1.0;  /* clamped */
                fr[3] = NAN;   /* pixel (0, 1): propagates through its block */
                if (orc_estimate(&p, &m, fr, n, maps) != 0) return fail("estimate");
                if (!isnan(maps[1])) return fail("NaN pixel did not propagate");
                free(c);
                free(gm);
                free(fr);
                free(maps);
            }
    orc_params bad = {7, 8, 1, 4, 4, 20.0, 200.0, 0.3, 1.0, 1e-3, 0.01, 1e-4, 1e-3, 44.0, 66.0, 0, 0};
    double dummy[1];
    if (orc_estimate(&bad, &m, dummy, 1, dummy) >= 0) return fail("odd width accepted");
    printf("oracle asan ok (%d threads)\n", orc_threads());
    return 0;
}
