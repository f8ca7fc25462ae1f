// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "hb.h"

namespace hb {

// Posterior grid tiles: 8 x 8 nodes of the THb x SO2 grid.  One tile is
//   [0]  Hb of the tile centre        [1]  HbO2 of the tile centre
//   [2..4] lower corner of the tile's box, relative to the tile centre
//   [5..7] upper corner                [8]  probe slot (int bits)
//   [9..11] tile centre in scaled, centred log-attenuation space (high part)
//   [12..14] its low part (double-float)                          [15] pad
//   [16 + 0*64 + i]  scaled log-attenuation of node i minus the centre, channel R
//   [16 + 1*64 + i]  ... channel G
//   [16 + 2*64 + i]  ... channel B
//   [16 + 3*64 + i]  Hb of node i minus the tile centre
//   [16 + 4*64 + i]  HbO2 of node i minus the tile centre
// Unused slots of edge tiles sit far away (weight exactly 0) with zero offsets.
constexpr int kTileSide = 8;
constexpr int kTileNodes = kTileSide * kTileSide;
constexpr int kTileHdr = 16;
constexpr int kTileFloats = kTileHdr + 5 * kTileNodes;
constexpr float kPadCoord = 1.0e18f;

// Strip of pixels one workgroup of the Haar kernels stages in LDS.
constexpr int kStripPixels = 2048;
constexpr int kBlockThreads = 256;

// LL pixels per thread in the posterior kernel.
constexpr int kPosteriorPix = 4;

// Partial moments per LL pixel and grid split:
//   [0] logit reference, [1] S0, [2] S1 about the anchor, [3] S2 about the anchor,
//   [4] anchor Hb, [5] anchor HbO2.
constexpr int kPartFields = 6;

struct Dims {
    int H, W, levels;
    int hl, wl;        // low-pass band size
    long long LL;      // hl * wl
    int bps;           // blocks per strip
    int strips_per_row;
};

struct HaarArgs {
    Dims d;
    int dtype;
    float floor;
    float iref[3];           // float32 reference intensities exp(-mu_ref)
    const float *M;          // device, 6 floats (FP32 Tikhonov operator)
    float *z;                // [n][6][LL]: high parts R,G,B then low parts
    float2 *det;             // [n][H][W]
};

struct PosteriorArgs {
    long long LL;
    int n_frames;
    const float *z;          // [n][6][LL]
    const float *tiles;      // [n_tiles][kTileFloats]
    int n_tiles;
    int split;
    float scale;             // sqrt(log2(e) / (2 sigma^2))
    float *part;             // [n][split][kPartFields][LL]
};

struct RecomposeArgs {
    Dims d;
    int lowpass;
    int split;
    const float *part;       // posterior partials
    const float *z;          // low-pass observation (Tikhonov low-pass)
    const float *M;          // device FP32 M (6) followed by the low-pass offset (2)
    const float2 *det;
    float2 *est;             // [n][LL] low-pass estimate (side output)
    float thb_eps;
    float *hb, *hbo2, *thb, *so2;
};

// Launchers (hb_kernels.hip).  They only enqueue work.
hipError_t launch_tikhonov_fp64(const double *d_in, double *d_out, float *d_mf, hipStream_t s);
hipError_t launch_log_haar(const void *frames, int n_frames, const HaarArgs &a, hipStream_t s);
hipError_t launch_posterior(const PosteriorArgs &a, hipStream_t s);
hipError_t launch_recompose(int n_frames, const RecomposeArgs &a, hipStream_t s);

}  // namespace hb
