// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "hb.h"

namespace hb {

// Posterior grid super-tiles: SUP x SUP nodes of the THb x SO2 grid (SUP is
// 8, 16 or 32), cut into 4 x 4-node chunks of 16 nodes.  Coordinates are
// scaled log-attenuations centred on mu_ref; inside a super-tile they are
// stored relative to the super-tile centre.  One super-tile is
//   header (kSupHdr floats)
//     [0..2]  centre, high parts        [3..5] centre, low parts (double-float)
//     [6] Hb of the centre node set     [7] HbO2 of it (moments are relative to these)
//     [8..10] box lower corner          [11..13] box upper corner (relative)
//     [14] number of probes (int bits)
//   probes (kMaxProbes x kProbeFloats): relative coordinates (3), Hb, HbO2
//   chunks (kChunkFloats each), node j = 4 * (THb offset) + (SO2 offset):
//     [0 + 16k + j], k = 0..2: relative coordinate k of node j
//     [48 + j]: minus the squared norm of the relative coordinates of node j
//     Slots outside the grid hold kPadCoord coordinates and kPadLogit here.
//     [64 + j]: Hb of node j minus header[6]     [80 + j]: HbO2 minus header[7]
//     [96..98] chunk box lower corner, [99..101] upper corner (absolute:
//       centre plus the stored coordinates, rounded outward)
//     [104 + 4 a + (0..3)], a = 0..3: for the chunk row of THb offset a,
//       Hb = A_h + B_h s at SO2 offset s = 0..3 relative to header[6] (exact
//       on a product grid: THb is constant along the row and SO2 is linear
//       in s), and the row's THb minus header[6] + header[7], as
//       (A_h, B_h, A_t, 0); HbO2 = THb - Hb.
// The first 64 floats of a chunk hold the node coordinates and squared
// norms (lane l: node row i = l % 16, column k = l / 16).
//
// Split operand table (the A operand of the posterior's 16x16x32 bf16 MFMA),
// kSplitLaneBytes per lane and kSplitChunkBytes per chunk, chunks in the
// order of the super-tile table: lane l = 16 g + i holds 8 bf16 values for
// node i of the chunk.  Every FP32 value x used below is split exactly into
// three bf16 parts x = x1 + x2 + x3 (each the nearest bf16 to what remains).
// For g = 0..2 and coordinate v = node coordinate g the 8 values are
//   (v1, v2, v1, v3, v2, v1, v3, v2)
// and the pixel (B) operand carries the parts of u = twice the pixel's
// coordinate g as (u1, u1, u2, u1, u2, u3, u2, u3), so the eight products
// are every u_a v_b except u3 v3 (below 2^-34 |u v|).  For g = 3 the node
// holds the parts of its squared-norm entry and three ones,
// (n1, n2, n3, 1, 1, 1, 0, 0), and the pixel (1, 1, 1, c1, c2, c3, 0, 0)
// with its constant c = -(|r|^2 + m).  The MFMA then forms the same
// expanded logit as FP32 products of the FP32 values, up to its accumulation
// rounding, and lane l of the result holds pixel l % 16 and the four nodes
// of chunk row l / 16.
constexpr int kSplitLaneBytes = 16;
constexpr int kSplitChunkBytes = 64 * kSplitLaneBytes;
// Precision rule for the MFMA kernel.  Its expanded logit rounds at the scale
// of the squared super-tile radius R^2 (scaled units), and a coarse grid
// (node spacing h in uM of Hb/HbO2) turns a logit error into an estimate error
// of about R^2 h u with little averaging.  The MFMA kernel is used when
// R^2 h <= kMfmaPrecisionBudget, the direct kernel otherwise.  Measured
// against the oracle (64 x 64 frame, grids 32..256, sigma 0.002..0.01): up
// to R^2 h = 700 the MFMA kernel's largest error was 4.6e-5 uM; between 800
// and 1000 it reached 8.0e-5 uM (sigma 0.004 on a 256 x 256 grid), too
// close to the 1e-4 uM tolerance.
constexpr double kMfmaPrecisionBudget = 700.0;
// The rule above holds for observations near the grid's surface in scaled
// units (within kFarRhoMin of a node: the calibration's noisy frames).  An
// observation at scaled distance rho from the nodes makes the expanded
// logit's terms about (R + rho) R instead of R^2.  Measured on seeded random
// frames, the error per unit of (R + rho) R h reached 1.6e-7 uM (a 50 x 101
// grid at sigma 0.002, whose posterior sits on few coarse nodes: 1.04e-4 uM
// at rho = 9.0, R = 8.5, h = 4.4 uM), so the MFMA kernel forms the sums of
// pixels with rho > max(kFarRhoMin, kMfmaFarBudget / (R h) - R) again with
// double-float logits (rho: the soft minimum over the nodes); at the budget
// that constant gives 5.6e-5 uM.
constexpr double kMfmaFarBudget = 350.0;
constexpr double kFarRhoMin = 3.0;
// Plans with R^2 h above kMfmaDfcIndex also sum the pixel operand's constant
// |r|^2 + m as a double-float (about 0.5 more vector instructions per
// chunk-block).  Measured on seeded random frames at sigma 0.002 on grids
// whose nodes lie about 4 scaled units apart (the posterior on very few
// nodes): 9.7e-5 uM with the float32 constant at R^2 h = 608, 8.6e-5 with
// the double-float one.
constexpr double kMfmaDfcIndex = 350.0;
// Precision rule for the direct kernel.  Its float32 difference-form logit
// of a node at scaled distance d from the observation carries an absolute
// error of a few d^2 u; for a pixel between two neighbouring nodes at scaled
// distance D apart, whose Hb/HbO2 differ by dc uM, the posterior mean then
// moves by up to about 8e-9 D^2 dc uM (measured 1.4e-4 uM on a grid with
// four THb nodes 68 uM apart).  Plans whose direct index max(D^2 dc) exceeds
// kDirectPrecisionBudget (8e-9 x 3800 = 3e-5 uM) form the logits from
// double-float coordinate differences instead.
constexpr double kDirectPrecisionBudget = 3800.0;
// The float32 direct kernel's differences also round at the scale of an
// observation's distance rho from the nodes: measured on seeded random
// frames at sigma 0.002 (noisy half-precision frames), 6e-5 to 8.3e-5 uM at
// rho^2 h = 3600-5400 (h: node spacing in uM), i.e. up to 2e-8 uM per unit.
// Pixels with rho^2 h > kDirectFarBudget take the double-float pass as in
// the MFMA kernel (2e-5 uM at the budget).
constexpr double kDirectFarBudget = 1000.0;
// Precision rule for K1.  With float32 log-ratios u = ln(R/I), their rounding
// reaches the maps through the Tikhonov operator M: measured on seeded random
// frames, up to 7.3e-5 uM at |M|inf = 1.13e3 uM per unit log-attenuation and
// 1.1-1.2e-4 uM at 1.4e3-3.1e3 (two levels).  Plans whose |M|inf exceeds
// kK1PrecisionBudget, and every plan with three or more levels, run K1 with
// double-float log-ratios, Haar cascade and Tikhonov apply (4x the ALU work:
// kept off the default camera, |M|inf = 1.05e3).
constexpr double kK1PrecisionBudget = 1100.0;
// Low parts of a chunk's node coordinates (3 coordinates x 16 nodes).
constexpr int kLoFloats = 48;

// Posterior chunk skipping.  exp2 of anything below -kExactSkipLog2 is exactly
// 0 in float32 (the smallest subnormal is 2^-149; the margin covers rounding
// of bounds and logits), so skipping at this threshold changes no bit.  A
// tolerance-derived threshold T skips more: every skipped weight is below
// 2^-T of the pixel's reference weight, while the kept weights sum to at least
// about 1 (the reference node itself, within rounding; counted as 1/2), so
// the posterior mean moves by at most 2 G 2^-T max|c_g - c_hat| <= 2 G 2^-T
// thb_max for G grid nodes.
constexpr float kExactSkipLog2 = 160.0f;
constexpr float kMinSkipLog2 = 16.0f;
// Budgeted skipping below a tolerance-derived threshold.  The hard threshold
// is T + 1, which spends at most half of the tolerance on G 2^-(T+1); a wave
// may also leave out chunks bounded between kBandLog2 and T + 1 below its
// reference, each of whose weights sum to at most 16 2^-(T+1-kBandLog2), as
// long as its count of such chunks stays within the budget the rest of the
// tolerance buys (every pixel of the wave then loses at most that mass).
constexpr float kBandLog2 = 6.0f;
struct SkipRule {
    float skip_log2 = kExactSkipLog2, band_log2 = kExactSkipLog2;
    int band_chunks = 0;
    double bound = 0.0;   // uM, stated bound on the posterior-mean change
};
constexpr int kChunkNodes = 16;
constexpr int kSupHdr = 32;
constexpr int kMaxProbes = 16;
constexpr int kProbeFloats = 8;
constexpr int kChunkFloats = 120;
constexpr float kPadLogit = -1.0e30f;
// Coordinates of slots outside the grid: far from every observation (weight
// exactly 0 in the difference form) yet small enough for the MFMA operands.
constexpr float kPadCoord = 1.0e4f;

// Side of a super-tile: about 1/8 of the grid (multiple of 4, 4..32).  The
// expanded logit loses precision with the squared extent of the super-tile in
// log-attenuation space, so coarse grids get small super-tiles.
inline int super_side(int grid_thb, int grid_so2) {
    const int g = grid_thb < grid_so2 ? grid_thb : grid_so2;
    const int side = 4 * (g / 32);
    return side < 4 ? 4 : (side > 32 ? 32 : side);
}
inline int super_floats(int side) {
    return kSupHdr + kMaxProbes * kProbeFloats + (side / 4) * (side / 4) * kChunkFloats;
}

// Strip of pixels one workgroup of the Haar kernels stages in LDS.
constexpr int kStripPixels = 2048;
constexpr int kBlockThreads = 256;

// Pixel blocks of 16 per wave in the posterior kernel (an 8 x 4 tile of LL
// pixels for two).  Each chunk's 1 KB split operand is loaded once per wave
// and used for every block, so more blocks cut the vector-memory traffic per
// pair; fewer blocks give tighter skip boxes (fewer pairs evaluated).  Two
// measured fastest (one was 10% slower, bound by operand loads).
constexpr int kPixelBlocks = 2;

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
    int n_frames;
    int vec4;                // frames pointer aligned to 4 stored values (vector loads allowed)
    int dtype;
    float floor;
    float iref[3];           // float32 reference intensities exp(-mu_ref)
    const float *M;          // device, 6 floats (FP32 Tikhonov operator)
    float *z;                // [n][6][LL]: high parts R,G,B then low parts
    float2 *det;             // [n][H][W] spatial detail part (inverse Haar of the details)
    int project;             // project z onto the plane orthogonal to (1,1,1)
    int df;                  // double-float log-ratios, Haar and Tikhonov (always from three levels on)
};

struct PosteriorArgs {
    long long LL;
    int hl, wl;              // low-pass band size (LL = hl * wl)
    int n_frames;
    const float *z;          // [n][6][LL]
    const float *supers;     // [n_supers][super_floats(side)]
    const void *split_ops;   // [n_supers][chunks_per_super][kSplitChunkBytes] bf16 A operands
    int n_supers;
    int super_stride;        // floats
    int chunks_per_super;
    int split;
    float scale;             // sqrt(log2(e) / (2 sigma^2))
    float skip_log2;         // chunks bounded more than this below the reference are skipped
    float band_log2;         // chunks bounded more than this below it are skipped while the budget lasts
    int band_chunks;         // budget: chunks a wave may skip between band_log2 and skip_log2
    float *gref;             // [n][LL] best probe logit over the whole grid, or null (one split)
    float *part;             // [n][split][kPartFields][LL]
    const float *lo;         // [chunk][kLoFloats] coordinate low parts (double-float logits)
    int precise;             // direct kernel: every logit from double-float differences
    unsigned long long *work;  // optional: [0] pairs evaluated (pixel x node), added per wave,
                               // [1] (pixel, split) sums formed again with double-float logits
    float far_rho2;          // pixels whose squared soft-minimum distance to the nodes exceeds
                             // this take double-float logits (INFINITY: none)
    int dfc;                 // MFMA kernel: form the pixel operand's constant |r|^2 + m as a
                             // double-float (plans with R^2 h > kMfmaDfcIndex)
    // Fused recomposition (one split, MFMA kernel, levels <= 2): the kernel
    // writes the low-pass estimate and the maps itself instead of partials.
    int fuse;
    int levels, H, W;
    int vec;                 // pixels per map store: 1, 2 or 4 (pointer alignment)
    const float2 *det;       // [n][H][W] spatial detail part
    float2 *est;             // [n][LL] low-pass estimate
    float thb_eps;
    float *hb, *hbo2, *thb, *so2;
};

struct RecomposeArgs {
    Dims d;
    int n_frames;
    int lowpass;
    int split;
    const float *part;       // posterior partials
    const float *z;          // low-pass observation (Tikhonov low-pass)
    const float *M;          // device FP32 M (6) followed by the low-pass offset (2)
    const float2 *det;       // [n][H][W] spatial detail part (inverse Haar of the details)
    float2 *est;             // [n][LL] low-pass estimate (side output)
    float thb_eps;
    float *hb, *hbo2, *thb, *so2;
};

// Static scratch of hb_estimate_frames_noalloc (hb_kernels.hip): one device
// array of kStaticScratchBytes per device.  static_scratch() must be called
// with `device` current; it looks the array's device address up once per
// device (at plan creation, so that the allocation-free call never loads
// modules or looks up symbols) and returns it.
constexpr size_t kStaticScratchBytes = HB_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxScratchDevices = 64;
hipError_t static_scratch(int device, void **ptr);

// Launchers (hb_kernels.hip).  They only enqueue work.
hipError_t launch_tikhonov_fp64(const double *d_in, double *d_out, float *d_mf, hipStream_t s);
hipError_t launch_log_haar(const void *frames, int n_frames, const HaarArgs &a, hipStream_t s);
hipError_t launch_reference(const PosteriorArgs &a, hipStream_t s);
hipError_t launch_posterior(const PosteriorArgs &a, bool mfma, hipStream_t s);
hipError_t launch_recompose(int n_frames, const RecomposeArgs &a, hipStream_t s);

}  // namespace hb
