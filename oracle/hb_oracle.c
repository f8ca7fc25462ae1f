/*
 * FP64 CPU oracle for the haemoglobin-estimation path of Jones et al.,
 * "Fast Estimation of Haemoglobin Concentration in Tissue Via Wavelet
 * Decomposition" (arXiv 1706.07263).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code with the GPU path.
 *
 * It follows the method's steps in the paper's order, in plain loops:
 *   log-attenuation -> n-level 2D Haar (Method, Eq. 1-2) -> Tikhonov on the
 *   directional coefficients (Method, Eq. 5) -> posterior mean over a
 *   (THb, SO2) grid on the low-pass coefficients (Method, the low-pass
 *   paragraph; the grid posterior replaces the cited Bayesian method, whose
 *   text is not part of the paper) -> inverse Haar (Eq. 4, "since H = H*")
 *   -> THb and SO2 maps (Fig. 1).
 *
 * Readings where the paper is silent (the test suite pins each one):
 *   - the log is taken before the Haar transform;
 *   - Tikhonov maps log-attenuation coefficients directly to (Hb, HbO2)
 *     through E, the Jacobian of the RGB forward model at a reference point;
 *     gamma is relative: gamma = lambda * tr(E'E) / 2;
 *   - the likelihood is Gaussian on the natural-log attenuation of the block
 *     mean, exp(-|ybar - mu_g|^2 / (2 sigma^2)), with a uniform prior over the
 *     nodes of an inclusive THb x SO2 grid;
 *   - intensities below `floor` are clamped (NaN propagates);
 *   - SO2 is NaN where THb <= thb_eps.
 *
 * Parity: every function here is pinned by the not-gpu tests (golden Haar
 * matrix of Eq. 2, perfect reconstruction, Parseval, Kronecker brute force,
 * normal equations, augmented least squares, lambda -> 0 inverse, complex-step
 * Jacobian, single-wavelength Beer-Lambert, 1- and 2-node posterior closed
 * forms, truncated-normal posterior, sigma -> infinity grid mean, grid-aligned
 * convergence, commutation invariant, dense brute force on 4x4 and 8x8 frames).
 */
#include "hb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* The 2D Haar matrix of Method, Eq. 2. */
static const double HAAR[4][4] = {
    {0.5, 0.5, 0.5, 0.5},
    {0.5, 0.5, -0.5, -0.5},
    {0.5, -0.5, -0.5, 0.5},
    {0.5, -0.5, 0.5, -0.5},
};

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Forward model.  Each camera channel k integrates Beer-Lambert attenuation
 * over its sensitivity, normalised to unit sum:
 *   mu_k(c) = -ln sum_j s~_k(l_j) exp(-L (eps_hb(l_j) c_hb + eps_hbo2(l_j) c_hbo2))
 * ------------------------------------------------------------------------- */
static double resp_sum(const orc_model *m, int k) {
    double s = 0.0;
    for (int j = 0; j < m->n_wl; ++j) s += m->response[k * m->n_wl + j];
    return s;
}

void orc_mu(const orc_model *m, double hb, double hbo2, double out[3]) {
    for (int k = 0; k < 3; ++k) {
        double norm = resp_sum(m, k);
        double acc = 0.0;
        for (int j = 0; j < m->n_wl; ++j) {
            double s = m->response[k * m->n_wl + j] / norm;
            acc += s * exp(-m->path_cm * (m->eps_hb[j] * hb + m->eps_hbo2[j] * hbo2));
        }
        out[k] = -log(acc);
    }
}

/* d mu_k / d c_i = L * sum_j w_kj eps_i(l_j),  w_kj = s~_kj a_j / sum_j s~_kj a_j. */
void orc_jacobian(const orc_model *m, double hb, double hbo2, double E[6]) {
    for (int k = 0; k < 3; ++k) {
        double norm = resp_sum(m, k);
        double den = 0.0, n_hb = 0.0, n_hbo2 = 0.0;
        for (int j = 0; j < m->n_wl; ++j) {
            double s = m->response[k * m->n_wl + j] / norm;
            double a = exp(-m->path_cm * (m->eps_hb[j] * hb + m->eps_hbo2[j] * hbo2));
            den += s * a;
            n_hb += s * a * m->eps_hb[j];
            n_hbo2 += s * a * m->eps_hbo2[j];
        }
        E[k * 2 + 0] = m->path_cm * n_hb / den;
        E[k * 2 + 1] = m->path_cm * n_hbo2 / den;
    }
}

/* Tikhonov operator of Method, Eq. 5 with C -> E:  M = (E'E + gamma I)^-1 E'. */
int orc_tikhonov(int rows, const double *E, double lambda_rel, double *M, double *gamma_abs) {
    double A[2][2] = {{0, 0}, {0, 0}};
    for (int r = 0; r < rows; ++r)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) A[i][j] += E[r * 2 + i] * E[r * 2 + j];
    double gamma = lambda_rel * (A[0][0] + A[1][1]) / 2.0;
    if (gamma_abs) *gamma_abs = gamma;
    double B00 = A[0][0] + gamma, B01 = A[0][1], B10 = A[1][0], B11 = A[1][1] + gamma;
    double det = B00 * B11 - B01 * B10;
    double scale = fabs(B00 * B11) + fabs(B01 * B10);
    if (!(fabs(det) > 1e-14 * scale)) return -1;
    double I00 = B11 / det, I01 = -B01 / det, I10 = -B10 / det, I11 = B00 / det;
    for (int r = 0; r < rows; ++r) {
        M[0 * rows + r] = I00 * E[r * 2 + 0] + I01 * E[r * 2 + 1];
        M[1 * rows + r] = I10 * E[r * 2 + 0] + I11 * E[r * 2 + 1];
    }
    return 0;
}

static double lin(double lo, double hi, int n, int i) {
    return n == 1 ? lo : lo + (hi - lo) * (double)i / (double)(n - 1);
}

void orc_grid(const orc_params *p, const orc_model *m, double *c, double *mu) {
    for (int a = 0; a < p->grid_thb; ++a) {
        double thb = lin(p->thb_min, p->thb_max, p->grid_thb, a);
        for (int b = 0; b < p->grid_so2; ++b) {
            double so2 = lin(p->so2_min, p->so2_max, p->grid_so2, b);
            long g = (long)a * p->grid_so2 + b;
            c[g * 2 + 0] = thb * (1.0 - so2);
            c[g * 2 + 1] = thb * so2;
            orc_mu(m, c[g * 2 + 0], c[g * 2 + 1], &mu[g * 3]);
        }
    }
}

/* ---------------------------------------------------------------------------
 * 2D Haar (Method, Eq. 1-2).  The window of a 2x2 block at rows (2i, 2i+1),
 * columns (2j, 2j+1) is v = {x(2i,2j), x(2i,2j+1), x(2i+1,2j), x(2i+1,2j+1)}
 * (the paper's {I(x,y), I(x,y+1), I(x+1,y), I(x+1,y+1)} with x the row), and
 * its coefficients are the row vector v * H:
 *   [LL, D1, D2, D3] = [low-pass, row difference, diagonal, column difference].
 * Mallat layout of an hh x ww (sub-)image after one level:
 *   LL at (i, j), D1 at (hh/2 + i, j), D2 at (hh/2 + i, ww/2 + j),
 *   D3 at (i, ww/2 + j);  level l + 1 recurses on the LL quadrant.
 * ------------------------------------------------------------------------- */
void orc_haar_forward(const double *x, int h, int w, int levels, double *coef) {
    memcpy(coef, x, sizeof(double) * (size_t)h * w);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)h * w);
    for (int l = 0; l < levels; ++l) {
        int hh = h >> l, ww = w >> l;
        for (int i = 0; i < hh / 2; ++i)
            for (int j = 0; j < ww / 2; ++j) {
                double v[4] = {coef[(size_t)(2 * i) * w + 2 * j], coef[(size_t)(2 * i) * w + 2 * j + 1],
                               coef[(size_t)(2 * i + 1) * w + 2 * j], coef[(size_t)(2 * i + 1) * w + 2 * j + 1]};
                double o[4];
                for (int col = 0; col < 4; ++col) {
                    o[col] = 0.0;
                    for (int r = 0; r < 4; ++r) o[col] += v[r] * HAAR[r][col];
                }
                tmp[(size_t)i * w + j] = o[0];
                tmp[(size_t)(hh / 2 + i) * w + j] = o[1];
                tmp[(size_t)(hh / 2 + i) * w + ww / 2 + j] = o[2];
                tmp[(size_t)i * w + ww / 2 + j] = o[3];
            }
        for (int i = 0; i < hh; ++i)
            memcpy(&coef[(size_t)i * w], &tmp[(size_t)i * w], sizeof(double) * ww);
    }
    free(tmp);
}

/* Inverse: since H = H^-1 (Eq. 4, "H = H*"), each window is restored as coef * H. */
void orc_haar_inverse(const double *coef, int h, int w, int levels, double *x) {
    memcpy(x, coef, sizeof(double) * (size_t)h * w);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)h * w);
    for (int l = levels - 1; l >= 0; --l) {
        int hh = h >> l, ww = w >> l;
        for (int i = 0; i < hh / 2; ++i)
            for (int j = 0; j < ww / 2; ++j) {
                double cf[4] = {x[(size_t)i * w + j], x[(size_t)(hh / 2 + i) * w + j],
                                x[(size_t)(hh / 2 + i) * w + ww / 2 + j], x[(size_t)i * w + ww / 2 + j]};
                double v[4];
                for (int col = 0; col < 4; ++col) {
                    v[col] = 0.0;
                    for (int r = 0; r < 4; ++r) v[col] += cf[r] * HAAR[r][col];
                }
                tmp[(size_t)(2 * i) * w + 2 * j] = v[0];
                tmp[(size_t)(2 * i) * w + 2 * j + 1] = v[1];
                tmp[(size_t)(2 * i + 1) * w + 2 * j] = v[2];
                tmp[(size_t)(2 * i + 1) * w + 2 * j + 1] = v[3];
            }
        for (int i = 0; i < hh; ++i)
            memcpy(&x[(size_t)i * w], &tmp[(size_t)i * w], sizeof(double) * ww);
    }
    free(tmp);
}

/* ---------------------------------------------------------------------------
 * Posterior mean on the low-pass band: uniform prior over the grid nodes,
 * Gaussian likelihood l_g = -|ybar - mu_g|^2 / (2 sigma^2), weights
 * exp(l_g - max l), mean of (Hb, HbO2) under those weights.
 *
 * Illumination term (the constant column of the attenuation coefficients,
 * Method, before Eq. 9: a change that is the same at every wavelength).  In
 * log space it adds b (1, 1, 1) to the observation; with a flat prior on b
 * the Gaussian integral over b leaves the likelihood of the residual with its
 * channel mean removed: l_g = -|d - mean(d)|^2 / (2 sigma^2), d = ybar - mu_g.
 * ------------------------------------------------------------------------- */
void orc_posterior_mean(const double *c, const double *mu, long G, const double ybar[3],
                        double sigma, int illumination, double out[2]) {
    double *l = (double *)malloc(sizeof(double) * (size_t)G);
    double mx = -INFINITY;
    for (long g = 0; g < G; ++g) {
        double d0 = ybar[0] - mu[g * 3 + 0], d1 = ybar[1] - mu[g * 3 + 1], d2 = ybar[2] - mu[g * 3 + 2];
        if (illumination) {
            const double dm = (d0 + d1 + d2) / 3.0;
            d0 -= dm;
            d1 -= dm;
            d2 -= dm;
        }
        l[g] = -(d0 * d0 + d1 * d1 + d2 * d2) / (2.0 * sigma * sigma);
        if (l[g] > mx) mx = l[g];
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long g = 0; g < G; ++g) {
        double wgt = exp(l[g] - mx);
        s0 += wgt;
        s1 += wgt * c[g * 2 + 0];
        s2 += wgt * c[g * 2 + 1];
    }
    free(l);
    out[0] = s1 / s0;
    out[1] = s2 / s0;
}

/* ---------------------------------------------------------------------------
 * The whole path for n frames.
 * ------------------------------------------------------------------------- */
int orc_estimate(const orc_params *p, const orc_model *m, const double *frames, int n,
                 double *maps) {
    const int h = p->height, w = p->width, L = p->levels;
    if (h <= 0 || w <= 0 || L < 0 || L > 16 || n < 0) return -1;
    if ((h % (1 << L)) != 0 || (w % (1 << L)) != 0) return -2;
    if (p->grid_thb < 1 || p->grid_so2 < 1 || !(p->sigma > 0.0)) return -1;
    const size_t HW = (size_t)h * w;
    const long G = (long)p->grid_thb * p->grid_so2;

    /* Plan: forward model linearised at the reference point, Tikhonov operator, grid. */
    double E[6], M[6], gamma, mu_ref[3];
    orc_jacobian(m, p->ref_hb, p->ref_hbo2, E);
    if (orc_tikhonov(3, E, p->lambda_rel, M, &gamma) != 0) return -6;
    orc_mu(m, p->ref_hb, p->ref_hbo2, mu_ref);
    double *gc = (double *)malloc(sizeof(double) * (size_t)G * 2);
    double *gmu = (double *)malloc(sizeof(double) * (size_t)G * 3);
    orc_grid(p, m, gc, gmu);

    double *y = (double *)malloc(sizeof(double) * HW * 3);
    double *cy = (double *)malloc(sizeof(double) * HW * 3);
    double *cc = (double *)malloc(sizeof(double) * HW * 2);
    double *xc = (double *)malloc(sizeof(double) * HW * 2);
    const int hl = h >> L, wl = w >> L;
    const double scale = ldexp(1.0, L);  /* LL_n = 2^n * block mean */

    for (int f = 0; f < n; ++f) {
        const double *fr = frames + (size_t)f * HW * 3;
        /* 1. Log-attenuation per channel (plane k). */
        for (size_t px = 0; px < HW; ++px)
            for (int k = 0; k < 3; ++k) {
                double v = fr[px * 3 + k];
                if (v < p->floor) v = p->floor;   /* NaN stays NaN */
                y[k * HW + px] = -log(v);
            }
        /* 2. n-level Haar of each channel. */
        for (int k = 0; k < 3; ++k) orc_haar_forward(&y[k * HW], h, w, L, &cy[k * HW]);
        /* 3. Tikhonov on every directional coefficient. */
        for (int r = 0; r < h; ++r)
            for (int col = 0; col < w; ++col) {
                size_t px = (size_t)r * w + col;
                if (r < hl && col < wl) continue;
                for (int i = 0; i < 2; ++i)
                    cc[i * HW + px] = M[i * 3 + 0] * cy[px] + M[i * 3 + 1] * cy[HW + px] +
                                      M[i * 3 + 2] * cy[2 * HW + px];
            }
        /* 4. Low-pass band: posterior mean (or Tikhonov) of the block mean. */
#pragma omp parallel for schedule(dynamic, 4)
        for (long q = 0; q < (long)hl * wl; ++q) {
            size_t px = (size_t)(q / wl) * w + (size_t)(q % wl);
            double ybar[3] = {cy[px] / scale, cy[HW + px] / scale, cy[2 * HW + px] / scale};
            double est[2];
            if (p->lowpass == 1) {
                for (int i = 0; i < 2; ++i)
                    est[i] = (i == 0 ? p->ref_hb : p->ref_hbo2) +
                             M[i * 3 + 0] * (ybar[0] - mu_ref[0]) + M[i * 3 + 1] * (ybar[1] - mu_ref[1]) +
                             M[i * 3 + 2] * (ybar[2] - mu_ref[2]);
            } else {
                orc_posterior_mean(gc, gmu, G, ybar, p->sigma, p->illumination, est);
            }
            cc[px] = scale * est[0];
            cc[HW + px] = scale * est[1];
        }
        /* 5. Inverse Haar of both concentration planes. */
        orc_haar_inverse(&cc[0], h, w, L, &xc[0]);
        orc_haar_inverse(&cc[HW], h, w, L, &xc[HW]);
        /* 6. Maps. */
        double *out = maps + (size_t)f * 4 * HW;
        for (size_t px = 0; px < HW; ++px) {
            double hb = xc[px], hbo2 = xc[HW + px], thb = hb + hbo2;
            out[px] = hb;
            out[HW + px] = hbo2;
            out[2 * HW + px] = thb;
            out[3 * HW + px] = (thb > p->thb_eps) ? hbo2 / thb : NAN;
        }
    }
    free(y); free(cy); free(cc); free(xc); free(gc); free(gmu);
    return 0;
}
