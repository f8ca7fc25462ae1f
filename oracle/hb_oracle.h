/*
 * FP64 CPU oracle for the per-frame haemoglobin-estimation path of
 * "Fast Estimation of Haemoglobin Concentration in Tissue Via Wavelet
 * Decomposition" (Jones et al., arXiv 1706.07263).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct
 * reference the GPU path is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Everything is double precision.  Frames are passed as doubles: the caller
 * widens the stored FP32/FP16/BF16 values exactly before the call.
 *
 * Parity status of each function is stated at its definition in hb_oracle.c.
 */
#ifndef HB_ORACLE_H
#define HB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Known camera spectral sensitivity and attenuation spectra (Method: the camera
 * matrix C and the attenuation coefficients xi). */
typedef struct {
    int n_wl;
    const double *eps_hb;     /* [n_wl] cm^-1 uM^-1, natural-log units          */
    const double *eps_hbo2;   /* [n_wl]                                          */
    const double *response;   /* [3][n_wl] R, G, B camera sensitivities          */
    double path_cm;           /* optical path length                              */
} orc_model;

typedef struct {
    int width, height, levels;            /* Haar levels n                        */
    int grid_thb, grid_so2;               /* posterior grid size                  */
    double thb_min, thb_max;              /* uM, inclusive                        */
    double so2_min, so2_max;              /* fraction, inclusive                  */
    double lambda_rel;                    /* Tikhonov gamma relative to tr(E'E)/2 */
    double sigma;                         /* likelihood s.d., natural-log units   */
    double floor;                         /* intensity clamp before the log       */
    double thb_eps;                       /* SO2 = NaN where THb <= thb_eps       */
    double ref_hb, ref_hbo2;              /* linearisation point of E (uM)        */
    int lowpass;                          /* 0 = Bayesian, 1 = Tikhonov           */
    int illumination;                     /* 1: marginalise a per-pixel additive  */
                                          /* log offset (same in every channel)   */
} orc_params;

/* mu(c): RGB log-attenuation of concentration c = (Hb, HbO2). */
void orc_mu(const orc_model *m, double hb, double hbo2, double out[3]);
/* E = d mu / d c at c (3x2, row-major). */
void orc_jacobian(const orc_model *m, double hb, double hbo2, double E[6]);
/* M = (E'E + gamma I)^-1 E' for an rows x 2 matrix E; gamma = lambda_rel*tr(E'E)/2.
 * Returns 0, or -1 if the 2x2 system is singular. */
int orc_tikhonov(int rows, const double *E, double lambda_rel, double *M, double *gamma_abs);
/* Grid nodes: c [G][2] = (Hb, HbO2) and mu [G][3]; node index a*grid_so2 + b. */
void orc_grid(const orc_params *p, const orc_model *m, double *c, double *mu);
/* n-level 2D Haar of an h x w plane into the Mallat layout (see hb_oracle.c). */
void orc_haar_forward(const double *x, int h, int w, int levels, double *coef);
void orc_haar_inverse(const double *coef, int h, int w, int levels, double *x);
/* Posterior mean of (Hb, HbO2) over G grid nodes for one observation ybar[3];
 * with `illumination` the likelihood integrates out an offset b*(1,1,1). */
void orc_posterior_mean(const double *c, const double *mu, long G, const double ybar[3],
                        double sigma, int illumination, double out[2]);
/* Whole path.  frames [n][h][w][3]; maps [n][4][h][w] = Hb, HbO2, THb, SO2.
 * Returns 0, or a negative value for invalid arguments. */
int orc_estimate(const orc_params *p, const orc_model *m, const double *frames, int n,
                 double *maps);
/* Number of OpenMP threads the estimate uses. */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
