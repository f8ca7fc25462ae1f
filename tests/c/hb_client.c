/*
 * A C client of the C ABI in include/hb.h, with no Python or PyTorch: it
 * builds a plan, sets the forward model, copies frames to the device with the
 * HIP runtime, estimates on the default stream and copies the maps back.
 *
 *   hb_client check
 *       host-side checks only (no device): defaults, status strings and
 *       argument validation before any device work.
 *   hb_client run IN OUT WIDTH HEIGHT LEVELS GRID
 *       IN:  float32 frames [n][HEIGHT][WIDTH][3] followed by nothing else;
 *            n is taken from the file size.
 *            The forward model is read from IN.model: int32 n_wl, then
 *            float64 eps_hb[n_wl], eps_hbo2[n_wl], response[3][n_wl], path_cm.
 *       OUT: float32 maps [n][4][HEIGHT][WIDTH] (Hb, HbO2, THb, SO2).
 * Exit status 0 on success; a failing call prints its status string.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hb.h"

#define CHECK_HB(call)                                                                  \
    do {                                                                                \
        hb_status_t st_ = (call);                                                       \
        if (st_ != HB_OK) {                                                             \
            fprintf(stderr, "%s:%d %s -> %s\n", __FILE__, __LINE__, #call, hb_status_string(st_)); \
            return 1;                                                                   \
        }                                                                               \
    } while (0)
#define CHECK_HIP(call)                                                                 \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            fprintf(stderr, "%s:%d %s -> %s\n", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
            return 1;                                                                   \
        }                                                                               \
    } while (0)
#define EXPECT(cond)                                                                    \
    do {                                                                                \
        if (!(cond)) {                                                                  \
            fprintf(stderr, "%s:%d expected %s\n", __FILE__, __LINE__, #cond);         \
            return 1;                                                                   \
        }                                                                               \
    } while (0)

static int host_checks(void) {
    hb_plan_desc_t d;
    EXPECT(hb_plan_desc_default(&d) == HB_OK);
    EXPECT(d.width == 64 && d.height == 64 && d.levels == 1 && d.max_batch == 1);
    EXPECT(d.illumination == 0 && d.posterior_tolerance == 1e-6);
    EXPECT(strcmp(hb_status_string(HB_ERR_SHAPE), "unknown status") != 0);
    hb_plan_t p = NULL;
    d.width = 66; /* not a multiple of 2^levels = 2: fine; 2^3 below is not */
    d.levels = 3;
    EXPECT(hb_plan_create(&d, 0, &p) == HB_ERR_SHAPE && p == NULL);
    hb_plan_desc_default(&d);
    d.sigma = -1.0;
    EXPECT(hb_plan_create(&d, 0, &p) == HB_ERR_INVALID_ARG && p == NULL);
    EXPECT(hb_plan_create(NULL, 0, &p) == HB_ERR_INVALID_ARG);
    EXPECT(hb_estimate_frames(NULL, NULL, 1, NULL, NULL) == HB_ERR_INVALID_ARG);
    EXPECT(hb_destroy(NULL) == HB_OK); /* destroying nothing is a no-op */
    printf("host checks passed\n");
    return 0;
}

static void *read_file(const char *path, size_t *bytes) {
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    void *buf = malloc((size_t)n);
    if (buf && fread(buf, 1, (size_t)n, f) != (size_t)n) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    *bytes = (size_t)n;
    return buf;
}

static int run(const char *in, const char *out, int width, int height, int levels, int grid) {
    size_t fbytes = 0, mbytes = 0;
    float *frames = (float *)read_file(in, &fbytes);
    char model_path[4096];
    snprintf(model_path, sizeof model_path, "%s.model", in);
    char *model = (char *)read_file(model_path, &mbytes);
    EXPECT(frames && model);
    const size_t px = (size_t)width * height;
    const int n = (int)(fbytes / (px * 3 * sizeof(float)));
    EXPECT(n >= 1 && fbytes == (size_t)n * px * 3 * sizeof(float));
    int n_wl;
    memcpy(&n_wl, model, sizeof n_wl);
    const double *md = (const double *)(model + 8);
    EXPECT(mbytes == 8 + sizeof(double) * (5 * (size_t)n_wl + 1));

    hb_plan_desc_t d;
    CHECK_HB(hb_plan_desc_default(&d));
    d.width = width;
    d.height = height;
    d.levels = levels;
    d.frame_dtype = HB_F32;
    d.max_batch = n;
    d.grid_thb = d.grid_so2 = grid;
    hb_plan_t plan = NULL;
    CHECK_HB(hb_plan_create(&d, 0, &plan));
    hb_forward_model_t fm;
    fm.n_wavelengths = n_wl;
    fm.wavelength_nm = NULL;
    fm.eps_hb = md;
    fm.eps_hbo2 = md + n_wl;
    fm.response = md + 2 * n_wl;
    fm.path_length_cm = md[5 * n_wl];
    CHECK_HB(hb_set_forward_model(plan, &fm));

    void *d_frames = NULL;
    float *d_maps = NULL;
    CHECK_HIP(hipMalloc(&d_frames, fbytes));
    CHECK_HIP(hipMalloc((void **)&d_maps, sizeof(float) * 4 * n * px));
    CHECK_HIP(hipMemcpy(d_frames, frames, fbytes, hipMemcpyHostToDevice));
    hb_maps_t maps;
    maps.hb = d_maps;
    maps.hbo2 = d_maps + (size_t)n * px;
    maps.thb = d_maps + 2 * (size_t)n * px;
    maps.so2 = d_maps + 3 * (size_t)n * px;
    CHECK_HB(hb_estimate_frames(plan, d_frames, n, &maps, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    /* planar per map: [4][n][H][W] on the device -> [n][4][H][W] in the file */
    float *host = (float *)malloc(sizeof(float) * 4 * n * px);
    EXPECT(host != NULL);
    for (int k = 0; k < 4; ++k)
        for (int f = 0; f < n; ++f)
            CHECK_HIP(hipMemcpy(host + ((size_t)f * 4 + k) * px, d_maps + ((size_t)k * n + f) * px,
                                sizeof(float) * px, hipMemcpyDeviceToHost));
    FILE *fo = fopen(out, "wb");
    EXPECT(fo && fwrite(host, sizeof(float), 4 * n * px, fo) == 4 * n * px);
    fclose(fo);
    CHECK_HB(hb_destroy(plan));
    CHECK_HIP(hipFree(d_frames));
    CHECK_HIP(hipFree(d_maps));
    free(host);
    free(frames);
    free(model);
    printf("estimated %d frame(s) of %dx%d\n", n, width, height);
    return 0;
}

int main(int argc, char **argv) {
    if (argc >= 2 && strcmp(argv[1], "check") == 0) return host_checks();
    if (argc == 8 && strcmp(argv[1], "run") == 0)
        return run(argv[2], argv[3], atoi(argv[4]), atoi(argv[5]), atoi(argv[6]), atoi(argv[7]));
    fprintf(stderr, "usage: %s check | run IN OUT WIDTH HEIGHT LEVELS GRID\n", argv[0]);
    return 2;
}
