// Host side of the C ABI: plan validation, device buffers, the FP64 posterior
// grid table and the launch sequence of hb_estimate_frames.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "hb.h"
#include "hb_internal.h"

using namespace hb;

namespace {

constexpr int kMaxLevels = 5;
constexpr int kMaxGrid = 4096;
constexpr int kMaxTimedCalls = 4096;

}  // namespace

struct hb_plan_s {
    hb_plan_desc_t desc{};
    int device = 0;
    Dims dims{};
    int split = 1;
    int side = 8;
    float far_rho2 = INFINITY;  // MFMA kernel: squared room for far observations (scaled units)
    double radius = 0;        // largest super-tile radius, scaled units
    double node_h = 0;        // node spacing, uM of Hb/HbO2 (the larger of the two grid directions)
    bool use_mfma = true;
    bool precise = false;       // direct kernel with double-float logits
    int k1_df = 0;              // K1 in double-float (large |M|)
    int n_tiles = 0;      // super-tiles
    long long n_nodes = 0;
    bool has_model = false;

    // Device memory.
    double *d_k0 = nullptr;   // K0 inputs followed by outputs
    size_t k0_in = 0;         // doubles of K0 input
    float *d_mf = nullptr;    // M (6) and the low-pass Tikhonov offset (2) as float32, then their low parts
    float *d_tiles = nullptr;   // super-tile table
    float *d_lo = nullptr;      // low parts of the node coordinates (double-float direct logits)
    void *d_split = nullptr;    // split bf16 A operands of the chunks
    float *d_z = nullptr;
    float2 *d_det = nullptr;
    float *d_part = nullptr;
    float *d_gref = nullptr;  // global posterior reference per LL pixel (split grids)
    float2 *d_est = nullptr;
    unsigned long long *d_work = nullptr;  // posterior pairs evaluated while timing
    void *scratch = nullptr;  // device address of the static scratch array (hb_estimate_frames_noalloc)
    size_t bytes = 0;
    long long full_pairs = 0;              // algorithmic pairs of the timed calls

    hb_plan_info_t info{};
    float iref[3] = {1, 1, 1};
    float scale = 1.0f;
    float skip_log2 = kExactSkipLog2;
    float band_log2 = kExactSkipLog2;   // = skip_log2 when no budget is in use
    int band_chunks = 0;

    hipEvent_t done = nullptr;       // recorded after each uncaptured hb_estimate_frames
    bool timing = false;
    std::vector<hipEvent_t> events;  // 4 per recorded call
    int timed_calls = 0;
    int last_frames = 0;
};

namespace {

bool is_finite(double x) { return std::isfinite(x); }

hb_status_t check_desc(const hb_plan_desc_t *d) {
    if (!d) return HB_ERR_INVALID_ARG;
    if (d->levels < 0 || d->levels > kMaxLevels) return HB_ERR_INVALID_ARG;
    if (d->width <= 0 || d->height <= 0) return HB_ERR_SHAPE;
    if ((d->width % (1 << d->levels)) != 0 || (d->height % (1 << d->levels)) != 0) return HB_ERR_SHAPE;
    if ((long long)d->width * d->height > (1LL << 28)) return HB_ERR_SHAPE;
    if (d->frame_dtype != HB_F32 && d->frame_dtype != HB_F16 && d->frame_dtype != HB_BF16)
        return HB_ERR_INVALID_ARG;
    if (d->max_batch < 1 || d->max_batch > 4096) return HB_ERR_INVALID_ARG;
    if (d->grid_thb < 1 || d->grid_so2 < 1 || d->grid_thb > kMaxGrid || d->grid_so2 > kMaxGrid)
        return HB_ERR_INVALID_ARG;
    if (!is_finite(d->thb_min) || !is_finite(d->thb_max) || d->thb_min < 0 || d->thb_max < d->thb_min)
        return HB_ERR_INVALID_ARG;
    if (!is_finite(d->so2_min) || !is_finite(d->so2_max) || d->so2_min < 0 || d->so2_max > 1 ||
        d->so2_max < d->so2_min)
        return HB_ERR_INVALID_ARG;
    if (!is_finite(d->lambda) || d->lambda < 0) return HB_ERR_INVALID_ARG;
    if (!is_finite(d->sigma) || !(d->sigma > 0)) return HB_ERR_INVALID_ARG;
    if (!is_finite(d->intensity_floor) || !(d->intensity_floor > 0)) return HB_ERR_INVALID_ARG;
    if (!is_finite(d->thb_eps)) return HB_ERR_INVALID_ARG;
    const bool ref_default = std::isnan(d->ref_thb) && std::isnan(d->ref_so2);
    if (!ref_default && (!is_finite(d->ref_thb) || !is_finite(d->ref_so2) || d->ref_thb < 0 ||
                         d->ref_so2 < 0 || d->ref_so2 > 1))
        return HB_ERR_INVALID_ARG;
    if (d->lowpass != HB_LOWPASS_BAYES && d->lowpass != HB_LOWPASS_TIKHONOV) return HB_ERR_INVALID_ARG;
    if (d->grid_split < 0 || d->grid_split > 256) return HB_ERR_INVALID_ARG;
    if (d->illumination != 0 && d->illumination != 1) return HB_ERR_INVALID_ARG;
    if (!is_finite(d->posterior_tolerance)) return HB_ERR_INVALID_ARG;
    return HB_OK;
}

Dims make_dims(const hb_plan_desc_t &d) {
    Dims m{};
    m.H = d.height;
    m.W = d.width;
    m.levels = d.levels;
    m.hl = d.height >> d.levels;
    m.wl = d.width >> d.levels;
    m.LL = (long long)m.hl * m.wl;
    m.bps = std::max(1, kStripPixels >> (2 * d.levels));
    m.strips_per_row = (m.wl + m.bps - 1) / m.bps;
    return m;
}

// Skip thresholds and band budget for a posterior tolerance tol (uM) on a
// grid of G nodes with THb up to thb_max, seen by `split` grid splits.
// tol > 0: T = the smallest threshold with 2 G 2^-T thb_max <= tol; skip hard
// at T + 1 (at most half of tol) and spend the rest on a per-wave budget of
// chunks bounded between T + 1 and T + 1 - kBandLog2 (each at most 16 nodes
// of weight 2^-(T + 1 - kBandLog2)), shared out between the splits.  At the
// exact threshold (T reaching kExactSkipLog2) there is no band and no error.
// tol == 0: exact skipping.  tol < 0: no skipping.
SkipRule skip_rule(double G, double thb_max, double tol, int split) {
    SkipRule r;
    if (tol > 0) {
        const double t = std::ceil(std::log2(2.0 * G * thb_max / tol));
        r.skip_log2 = (float)std::min<double>(kExactSkipLog2, std::max<double>(kMinSkipLog2, t));
        r.band_log2 = r.skip_log2;
        if (r.skip_log2 + 1.0f < kExactSkipLog2) {
            r.skip_log2 += 1.0f;
            r.band_log2 = r.skip_log2 - kBandLog2;
            const double hard = 2.0 * G * std::exp2(-(double)r.skip_log2) * thb_max;
            const double per_chunk = 2.0 * kChunkNodes * std::exp2(-(double)r.band_log2) * thb_max;
            const double n = std::floor((tol - hard) / per_chunk / split);
            r.band_chunks = (int)std::max(0.0, std::min(n, 1.0e6));
        }
        if (r.skip_log2 < kExactSkipLog2)
            r.bound = 2.0 * G * std::exp2(-(double)r.skip_log2) * thb_max +
                      2.0 * kChunkNodes * std::exp2(-(double)r.band_log2) * thb_max * (double)r.band_chunks * split;
    } else if (tol < 0) {
        r.skip_log2 = r.band_log2 = INFINITY;   // every chunk holding a grid node is evaluated
    }
    return r;
}

int auto_split(const Dims &dm, int n_tiles, int max_batch) {
    // One split unless a full batch gives fewer than kMinWaves waves.  With
    // skipping, a split adds a reference pass, a global-reference kernel and
    // the merge kernel, and far splits still pay their per-wave set-up:
    // measured per frame at batch 1, one split was fastest from 640x480
    // (600 waves) to 3840x2160.  The split is fixed per plan, so a frame gives
    // the same bits in any batch.
    constexpr long long kMinWaves = 256;
    const long long per_wave = 16LL * kPixelBlocks;
    const long long waves = std::max(1LL, ((long long)max_batch * dm.LL + per_wave - 1) / per_wave);
    int s = 1;
    while (s < 64 && waves * s < kMinWaves) s *= 2;
    return std::max(1, std::min(s, n_tiles));
}

hb_status_t dev_alloc(hb_plan_s *p, void **ptr, size_t bytes) {
    if (hipMalloc(ptr, bytes) != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return HB_ERR_OUT_OF_MEMORY;
    }
    p->bytes += bytes;
    return HB_OK;
}

void free_plan(hb_plan_s *p) {
    (void)hipFree(p->d_k0);
    (void)hipFree(p->d_mf);
    (void)hipFree(p->d_tiles);
    (void)hipFree(p->d_lo);
    (void)hipFree(p->d_split);
    (void)hipFree(p->d_z);
    (void)hipFree(p->d_det);
    (void)hipFree(p->d_part);
    (void)hipFree(p->d_gref);
    (void)hipFree(p->d_est);
    (void)hipFree(p->d_work);
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    if (p->done) (void)hipEventDestroy(p->done);
    delete p;
}

hb_status_t set_device(int dev) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return HB_ERR_DEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return HB_ERR_DEVICE;
    return HB_OK;
}

double lin(double lo, double hi, int n, int i) { return n == 1 ? lo : lo + (hi - lo) * (double)i / (double)(n - 1); }

// RGB log-attenuation of concentration (hb, hbo2): channel k integrates
// Beer-Lambert attenuation over its normalised sensitivity.
struct ForwardModel {
    int n = 0;
    std::vector<double> ehb, eox, resp;  // resp rows normalised
    double L = 0;
    void mu(double hb, double hbo2, double out[3]) const {
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += resp[k * n + j] * std::exp(-L * (ehb[j] * hb + eox[j] * hbo2));
            out[k] = -std::log(acc);
        }
    }
};

// Largest float <= x and smallest float >= x (infinities stay).
float float_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, -INFINITY);
    return f;
}
float float_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

// Build the super-tile table (FP64 arithmetic, FP32 storage): scaled
// log-attenuation of every grid node centred on mu_ref, stored relative to its
// super-tile centre in the MFMA operand layout, plus moments, boxes and probes.
// With the illumination term the node vectors are projected onto the plane
// orthogonal to (1,1,1), as the observations are.
//
// `lo` receives, per chunk, the low parts of the stored node coordinates
// ([chunk][coordinate k][node j], 48 floats: the FP64 relative coordinate
// minus its float32 value), for the direct kernel's double-float logits.
// `direct_index` receives max over neighbouring nodes of the squared scaled
// distance between them times their largest Hb/HbO2 difference (uM): with
// float32 logits the posterior mean of a pixel between two such nodes can
// move by about 8e-9 times this.
double build_supers(const hb_plan_desc_t &d, const ForwardModel &fm, const double mu_ref[3], double scale,
                    int side, std::vector<float> &table, std::vector<float> &lo, double &direct_index) {
    const bool project = d.illumination && d.lowpass == HB_LOWPASS_BAYES;
    const int GT = d.grid_thb, GS = d.grid_so2;
    const int nsa = (GT + side - 1) / side, nss = (GS + side - 1) / side;
    const int n_sup = nsa * nss;
    const int stride = super_floats(side);
    const int cps = side / 4;  // chunks per super-tile side
    table.assign((size_t)n_sup * stride, 0.0f);
    lo.assign((size_t)n_sup * cps * cps * kLoFloats, 0.0f);
    std::vector<double> radius(n_sup, 0.0), index(n_sup, 0.0);
    auto work = [&](int s_begin, int s_end) {
        std::vector<double> mu((size_t)side * side * 3), chb((size_t)side * side), cox((size_t)side * side);
        std::vector<char> real((size_t)side * side);
        for (int sidx = s_begin; sidx < s_end; ++sidx) {
            const int sa = sidx / nss, ss = sidx % nss;
            const int a0 = sa * side, b0 = ss * side;
            float *T = &table[(size_t)sidx * stride];
            // nodes of this super-tile
            double cen[3] = {0, 0, 0}, mhb = 0, mox = 0;
            int nreal = 0;
            for (int i = 0; i < side; ++i)
                for (int j = 0; j < side; ++j) {
                    const int n = i * side + j;
                    real[n] = (a0 + i < GT) && (b0 + j < GS);
                    if (!real[n]) continue;
                    const double thb = lin(d.thb_min, d.thb_max, GT, a0 + i);
                    const double so2 = lin(d.so2_min, d.so2_max, GS, b0 + j);
                    chb[n] = thb * (1.0 - so2);
                    cox[n] = thb * so2;
                    double m[3];
                    fm.mu(chb[n], cox[n], m);
                    double v[3];
                    for (int k = 0; k < 3; ++k) v[k] = m[k] - mu_ref[k];
                    if (project) {
                        const double mean = (v[0] + v[1] + v[2]) / 3.0;
                        for (int k = 0; k < 3; ++k) v[k] -= mean;
                    }
                    for (int k = 0; k < 3; ++k) {
                        mu[3 * n + k] = scale * v[k];
                        cen[k] += mu[3 * n + k];
                    }
                    mhb += chb[n];
                    mox += cox[n];
                    ++nreal;
                }
            float cen_hi[3], cen_lo[3];
            double cen_d[3];
            for (int k = 0; k < 3; ++k) {
                const double c = cen[k] / nreal;
                cen_hi[k] = (float)c;
                cen_lo[k] = (float)(c - (double)cen_hi[k]);
                cen_d[k] = (double)cen_hi[k] + (double)cen_lo[k];
            }
            const float chb_c = (float)(mhb / nreal), cox_c = (float)(mox / nreal);
            auto rel = [&](int n, int k) { return mu[3 * n + k] - cen_d[k]; };
            // neighbouring nodes inside the super-tile (both grid directions)
            for (int i = 0; i < side; ++i)
                for (int j = 0; j < side; ++j) {
                    const int n = i * side + j;
                    if (!real[n]) continue;
                    for (int dir = 0; dir < 2; ++dir) {
                        const int ii = i + (dir == 0), jj = j + (dir == 1);
                        if (ii >= side || jj >= side || !real[ii * side + jj]) continue;
                        const int q = ii * side + jj;
                        double d2 = 0;
                        for (int k = 0; k < 3; ++k) d2 += (mu[3 * n + k] - mu[3 * q + k]) * (mu[3 * n + k] - mu[3 * q + k]);
                        const double dc = std::max(std::fabs(chb[n] - chb[q]), std::fabs(cox[n] - cox[q]));
                        index[sidx] = std::max(index[sidx], d2 * dc);
                    }
                }
            float blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
            // chunks
            for (int ca = 0; ca < cps; ++ca)
                for (int cs = 0; cs < cps; ++cs) {
                    float *C = T + kSupHdr + kMaxProbes * kProbeFloats + (size_t)(ca * cps + cs) * kChunkFloats;
                    float *LO = &lo[((size_t)sidx * cps * cps + (size_t)(ca * cps + cs)) * kLoFloats];
                    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
                    double alo[3] = {INFINITY, INFINITY, INFINITY}, ahi[3] = {-INFINITY, -INFINITY, -INFINITY};
                    for (int j = 0; j < kChunkNodes; ++j) {
                        const int n = (4 * ca + j / 4) * side + 4 * cs + j % 4;
                        if (!real[n]) {
                            C[j] = C[16 + j] = C[32 + j] = kPadCoord;
                            C[48 + j] = kPadLogit;
                            C[64 + j] = C[80 + j] = 0.0f;
                            continue;
                        }
                        double sq = 0;
                        for (int k = 0; k < 3; ++k) {
                            const float v = (float)rel(n, k);
                            C[16 * k + j] = v;
                            LO[16 * k + j] = (float)(rel(n, k) - (double)v);
                            sq += (double)v * (double)v;
                            clo[k] = std::min(clo[k], v);
                            chi[k] = std::max(chi[k], v);
                            alo[k] = std::min(alo[k], cen_d[k] + (double)v);
                            ahi[k] = std::max(ahi[k], cen_d[k] + (double)v);
                        }
                        C[48 + j] = (float)(-sq);
                        radius[sidx] = std::max(radius[sidx], std::sqrt(sq));
                        C[64 + j] = (float)(chb[n] - (double)chb_c);
                        C[80 + j] = (float)(cox[n] - (double)cox_c);
                    }
                    for (int k = 0; k < 3; ++k) {
                        // absolute box of the stored nodes, rounded outward
                        C[96 + k] = float_down(alo[k]);
                        C[99 + k] = float_up(ahi[k]);
                        blo[k] = std::min(blo[k], clo[k]);
                        bhi[k] = std::max(bhi[k], chi[k]);
                    }
                    // row moments: Hb and HbO2 along each THb row are affine in
                    // the SO2 offset (THb fixed, SO2 a linspace)
                    const double dso2 = GS > 1 ? (d.so2_max - d.so2_min) / (GS - 1) : 0.0;
                    for (int ra = 0; ra < 4; ++ra) {
                        float *Q = C + 104 + 4 * ra;
                        const int ga = a0 + 4 * ca + ra;
                        if (ga >= GT) {
                            Q[0] = Q[1] = Q[2] = Q[3] = 0.0f;
                            continue;
                        }
                        const double thb = lin(d.thb_min, d.thb_max, GT, ga);
                        const double so2 = lin(d.so2_min, d.so2_max, GS, b0 + 4 * cs);
                        Q[0] = (float)(thb * (1.0 - so2) - (double)chb_c);
                        Q[1] = (float)(-thb * dso2);
                        // THb is constant along the row: the HbO2 moment is the
                        // THb moment minus the Hb moment
                        Q[2] = (float)(thb - (double)chb_c - (double)cox_c);
                        Q[3] = 0.0f;
                    }
                    for (int k = 102; k < 104; ++k) C[k] = 0.0f;
                }
            // probes: the middle real node of each 8 x 8 patch
            int np = 0;
            for (int pa = 0; pa < side; pa += 8)
                for (int pb = 0; pb < side; pb += 8) {
                    const int na = std::min(std::min(8, side), GT - a0 - pa);
                    const int nb = std::min(std::min(8, side), GS - b0 - pb);
                    if (na <= 0 || nb <= 0) continue;
                    const int n = (pa + (na - 1) / 2) * side + pb + (nb - 1) / 2;
                    float *P = T + kSupHdr + np * kProbeFloats;
                    for (int k = 0; k < 3; ++k) {
                        // the probe must carry the same float coordinates as its node
                        P[k] = (float)rel(n, k);
                    }
                    P[3] = (float)chb[n];
                    P[4] = (float)cox[n];
                    ++np;
                }
            for (int k = 0; k < 3; ++k) {
                T[k] = cen_hi[k];
                T[3 + k] = cen_lo[k];
                T[8 + k] = blo[k];
                T[11 + k] = bhi[k];
            }
            T[6] = chb_c;
            T[7] = cox_c;
            std::memcpy(&T[14], &np, sizeof(int));
        }
    };
    unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 32u));
    nt = std::min<unsigned>(nt, (unsigned)n_sup);
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nt; ++i)
        th.emplace_back(work, (int)((long long)n_sup * i / nt), (int)((long long)n_sup * (i + 1) / nt));
    for (auto &x : th) x.join();
    direct_index = *std::max_element(index.begin(), index.end());
    return *std::max_element(radius.begin(), radius.end());
}

// Nearest bf16 (ties to even) of a finite float, and its float value.
uint16_t bf16_nearest(float x) {
    uint32_t u;
    std::memcpy(&u, &x, sizeof(u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float x;
    std::memcpy(&x, &u, sizeof(x));
    return x;
}
// x = x1 + x2 + x3 exactly: each remainder is exact in float and the last one
// has at most 8 significant bits.
void split3(float x, uint16_t p[3]) {
    p[0] = bf16_nearest(x);
    const float r1 = x - bf16_value(p[0]);
    p[1] = bf16_nearest(r1);
    const float r2 = r1 - bf16_value(p[1]);
    p[2] = bf16_nearest(r2);
}

// Split bf16 A operands of every chunk from the FP32 coordinates and
// squared-norm entries of the super-tile table (layout in hb_internal.h).
void build_split_ops(const std::vector<float> &table, int n_sup, int side, std::vector<uint16_t> &ops) {
    const int stride = super_floats(side);
    const int n_chunks = (side / 4) * (side / 4);
    constexpr int kLaneHalves = kSplitLaneBytes / 2;
    ops.assign((size_t)n_sup * n_chunks * 64 * kLaneHalves, 0);
    for (int si = 0; si < n_sup; ++si)
        for (int c = 0; c < n_chunks; ++c) {
            const float *C = &table[(size_t)si * stride + kSupHdr + kMaxProbes * kProbeFloats + (size_t)c * kChunkFloats];
            uint16_t *O = &ops[((size_t)si * n_chunks + c) * 64 * kLaneHalves];
            for (int g = 0; g < 4; ++g)
                for (int i = 0; i < 16; ++i) {
                    uint16_t *L = O + (size_t)(16 * g + i) * kLaneHalves;
                    uint16_t v[3];
                    split3(C[16 * g + i], v);   // g = 3: the squared-norm entry
                    if (g < 3) {
                        const int order[8] = {0, 1, 0, 2, 1, 0, 2, 1};
                        for (int e = 0; e < 8; ++e) L[e] = v[order[e]];
                    } else {
                        const uint16_t one = bf16_nearest(1.0f);
                        for (int e = 0; e < 3; ++e) {
                            L[e] = v[e];
                            L[3 + e] = one;   // picks up the pixel's constant
                        }
                    }
                }
        }
}

// Per-call device buffers of hb_estimate_frames: the plan's own, or carved
// from the static scratch array by hb_estimate_frames_noalloc.
struct CallBuffers {
    float *z;       // [n][6][LL] low-pass observation
    float2 *det;    // [n][H][W] detail part
    float *part;    // [n][split][kPartFields][LL] posterior partials (Bayesian low-pass)
    float *gref;    // [n][LL] global posterior reference (split grids), else null
    float2 *est;    // [n][LL] low-pass estimate
};

// Argument and state checks shared by both estimate calls (nothing launched).
hb_status_t check_call(hb_plan_t p, const void *d_frames, int32_t n_frames, const hb_maps_t *d_out) {
    if (!p || !d_out) return HB_ERR_INVALID_ARG;
    if (n_frames < 0) return HB_ERR_INVALID_ARG;
    if (n_frames > p->desc.max_batch) return HB_ERR_BATCH;
    if (!p->has_model) return HB_ERR_NO_FORWARD_MODEL;
    if (n_frames == 0) return HB_OK;
    if (!d_frames) return HB_ERR_INVALID_ARG;
    return HB_OK;
}

// Lay the buffers of an n-frame call out in the static scratch (each rounded
// up to 256 bytes); false if they do not fit.
bool carve_scratch(const hb_plan_s *p, int n, unsigned char *base, CallBuffers &cb) {
    const size_t LL = (size_t)p->dims.LL, HW = (size_t)p->desc.width * p->desc.height, nb = (size_t)n;
    const bool bayes = p->desc.lowpass == HB_LOWPASS_BAYES;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *q = base + off;
        off += (bytes + 255) / 256 * 256;
        return q;
    };
    cb.z = (float *)take(sizeof(float) * nb * 6 * LL);
    cb.det = (float2 *)take(sizeof(float2) * nb * HW);
    cb.part = bayes ? (float *)take(sizeof(float) * nb * p->split * kPartFields * LL) : nullptr;
    cb.gref = (bayes && p->split > 1) ? (float *)take(sizeof(float) * nb * LL) : nullptr;
    cb.est = (float2 *)take(sizeof(float2) * nb * LL);
    return off <= kStaticScratchBytes;
}

// The launch sequence of one estimate call into the buffers cb (arguments
// already checked).  `timed`: record the plan's timing events and work
// counter when timing is enabled (hb_estimate_frames_noalloc passes false:
// creating events could allocate).
hb_status_t estimate(hb_plan_s *p, const void *d_frames, int32_t n_frames, const hb_maps_t *d_out, hipStream_t s,
                     const CallBuffers &cb, bool timed) {
    if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
    hipEvent_t *ev = nullptr;
    if (timed && p->timing && p->timed_calls < kMaxTimedCalls) {
        const size_t need = 4 * (size_t)(p->timed_calls + 1);
        while (p->events.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return HB_ERR_DEVICE;
            p->events.push_back(e);
        }
        ev = &p->events[4 * (size_t)p->timed_calls];
        p->timed_calls++;
    }
    auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };

    HaarArgs ha{};
    ha.d = p->dims;
    ha.dtype = p->desc.frame_dtype;
    ha.floor = (float)p->desc.intensity_floor;
    for (int k = 0; k < 3; ++k) ha.iref[k] = p->iref[k];
    ha.M = p->d_mf;
    ha.z = cb.z;
    ha.det = cb.det;
    ha.project = p->desc.illumination && p->desc.lowpass == HB_LOWPASS_BAYES;
    ha.df = p->k1_df;

    if (mark(0) != hipSuccess) return HB_ERR_DEVICE;
    if (launch_log_haar(d_frames, n_frames, ha, s) != hipSuccess) return HB_ERR_DEVICE;
    if (mark(1) != hipSuccess) return HB_ERR_DEVICE;
    bool fused = false;
    if (p->desc.lowpass == HB_LOWPASS_BAYES) {
        PosteriorArgs pa{};
        pa.LL = p->dims.LL;
        pa.hl = p->dims.hl;
        pa.wl = p->dims.wl;
        pa.n_frames = n_frames;
        pa.z = cb.z;
        pa.supers = p->d_tiles;
        pa.split_ops = p->d_split;
        pa.n_supers = p->n_tiles;
        pa.super_stride = super_floats(p->side);
        pa.chunks_per_super = (p->side / 4) * (p->side / 4);
        pa.split = p->split;
        pa.scale = p->scale;
        pa.skip_log2 = p->skip_log2;
        pa.band_log2 = p->band_log2;
        pa.band_chunks = p->band_chunks;
        pa.part = cb.part;
        pa.lo = p->d_lo;
        pa.precise = p->precise ? 1 : 0;
        pa.far_rho2 = p->far_rho2;
        pa.dfc = p->info.mfma_df_constant;
        pa.work = ev ? p->d_work : nullptr;
        if (ev) p->full_pairs += (long long)n_frames * p->dims.LL * p->n_nodes;
        if (cb.gref) {
            pa.gref = cb.gref;
            if (launch_reference(pa, s) != hipSuccess) return HB_ERR_DEVICE;
        }
        // One split, MFMA kernel, n <= 2: the posterior writes the maps.
        fused = p->use_mfma && p->split == 1 && p->dims.levels <= 2;
        if (fused) {
            const int B = 1 << p->dims.levels;
            auto fits = [&](int v) {
                if (B % v) return false;
                for (const float *m : {d_out->hb, d_out->hbo2, d_out->thb, d_out->so2})
                    if (m && ((uintptr_t)m % (sizeof(float) * v)) != 0) return false;
                return true;
            };
            pa.fuse = 1;
            pa.vec = fits(4) ? 4 : (fits(2) ? 2 : 1);
            pa.levels = p->dims.levels;
            pa.H = p->dims.H;
            pa.W = p->dims.W;
            pa.det = cb.det;
            pa.est = cb.est;
            pa.thb_eps = (float)p->desc.thb_eps;
            pa.hb = d_out->hb;
            pa.hbo2 = d_out->hbo2;
            pa.thb = d_out->thb;
            pa.so2 = d_out->so2;
        }
        if (launch_posterior(pa, p->use_mfma, s) != hipSuccess) return HB_ERR_DEVICE;
    }
    if (mark(2) != hipSuccess) return HB_ERR_DEVICE;
    RecomposeArgs ra{};
    ra.d = p->dims;
    ra.lowpass = p->desc.lowpass;
    ra.split = p->split;
    ra.part = cb.part;
    ra.z = cb.z;
    ra.M = p->d_mf;
    ra.det = cb.det;
    ra.est = cb.est;
    ra.thb_eps = (float)p->desc.thb_eps;
    ra.hb = d_out->hb;
    ra.hbo2 = d_out->hbo2;
    ra.thb = d_out->thb;
    ra.so2 = d_out->so2;
    if (!fused && launch_recompose(n_frames, ra, s) != hipSuccess) return HB_ERR_DEVICE;
    if (mark(3) != hipSuccess) return HB_ERR_DEVICE;
    // Completion marker for hb_destroy (not recorded into a graph under capture).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return HB_ERR_DEVICE;
    if (cap == hipStreamCaptureStatusNone && hipEventRecord(p->done, s) != hipSuccess) return HB_ERR_DEVICE;
    p->last_frames = n_frames;
    return HB_OK;
}

}  // namespace

extern "C" {

hb_status_t hb_plan_desc_default(hb_plan_desc_t *d) {
    if (!d) return HB_ERR_INVALID_ARG;
    std::memset(d, 0, sizeof(*d));
    d->width = 64;
    d->height = 64;
    d->levels = 1;
    d->frame_dtype = HB_F32;
    d->max_batch = 1;
    d->grid_thb = 128;
    d->grid_so2 = 128;
    d->thb_min = 20.0;
    d->thb_max = 200.0;
    d->so2_min = 0.3;
    d->so2_max = 1.0;
    d->lambda = 1e-3;
    d->sigma = 0.01;
    d->intensity_floor = 1e-4;
    d->ref_thb = NAN;
    d->ref_so2 = NAN;
    d->thb_eps = 1e-3;
    d->lowpass = HB_LOWPASS_BAYES;
    d->grid_split = 0;
    d->illumination = 0;
    d->posterior_tolerance = 1e-6;
    return HB_OK;
}

const char *hb_status_string(hb_status_t s) {
    // C callers may pass any int; read it as one (an out-of-range value of the
    // enum type is not a valid C++ value).
    int v;
    std::memcpy(&v, &s, sizeof(v));
    switch (v) {
        case HB_OK: return "ok";
        case HB_ERR_INVALID_ARG: return "invalid argument";
        case HB_ERR_SHAPE: return "invalid frame shape (width and height must be positive multiples of 2^levels)";
        case HB_ERR_NO_FORWARD_MODEL: return "forward model not set";
        case HB_ERR_OUT_OF_MEMORY: return "device allocation failed";
        case HB_ERR_DEVICE: return "HIP device error";
        case HB_ERR_ILL_POSED: return "Tikhonov system is singular";
        case HB_ERR_BATCH: return "n_frames exceeds the plan's max_batch";
        case HB_ERR_SCRATCH: return "the call's buffers exceed the static scratch of hb_estimate_frames_noalloc";
    }
    return "unknown status";
}

hb_status_t hb_plan_create(const hb_plan_desc_t *desc, int device, hb_plan_t *out) {
    if (!out) return HB_ERR_INVALID_ARG;
    *out = nullptr;
    hb_status_t st = check_desc(desc);
    if (st != HB_OK) return st;
    if (device < 0) return HB_ERR_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        (void)hipGetLastError();
        return HB_ERR_DEVICE;
    }
    if (set_device(device) != HB_OK) return HB_ERR_DEVICE;

    hb_plan_s *p = new (std::nothrow) hb_plan_s();
    if (!p) return HB_ERR_OUT_OF_MEMORY;
    p->desc = *desc;
    p->device = device;
    p->dims = make_dims(*desc);
    p->side = super_side(desc->grid_thb, desc->grid_so2);
    const int nsa = (desc->grid_thb + p->side - 1) / p->side, nss = (desc->grid_so2 + p->side - 1) / p->side;
    p->n_tiles = nsa * nss;
    p->n_nodes = (long long)desc->grid_thb * desc->grid_so2;
    p->split = desc->grid_split > 0 ? std::min(desc->grid_split, p->n_tiles) : auto_split(p->dims, p->n_tiles, desc->max_batch);

    const size_t nb = (size_t)desc->max_batch;
    const size_t LL = (size_t)p->dims.LL;
    const size_t HW = (size_t)desc->height * desc->width;
    st = HB_OK;
    if (st == HB_OK) st = dev_alloc(p, (void **)&p->d_mf, sizeof(float) * 16);
    if (st == HB_OK) st = dev_alloc(p, (void **)&p->d_tiles, sizeof(float) * (size_t)p->n_tiles * super_floats(p->side));
    if (st == HB_OK)
        st = dev_alloc(p, &p->d_split, (size_t)kSplitChunkBytes * p->n_tiles * (p->side / 4) * (p->side / 4));
    if (st == HB_OK)
        st = dev_alloc(p, (void **)&p->d_lo, sizeof(float) * kLoFloats * p->n_tiles * (p->side / 4) * (p->side / 4));
    if (st == HB_OK) st = dev_alloc(p, (void **)&p->d_z, sizeof(float) * nb * 6 * LL);
    if (st == HB_OK) st = dev_alloc(p, (void **)&p->d_det, sizeof(float2) * nb * HW);
    if (st == HB_OK && desc->lowpass == HB_LOWPASS_BAYES)
        st = dev_alloc(p, (void **)&p->d_part, sizeof(float) * nb * p->split * kPartFields * LL);
    if (st == HB_OK && desc->lowpass == HB_LOWPASS_BAYES && p->split > 1)
        st = dev_alloc(p, (void **)&p->d_gref, sizeof(float) * nb * LL);
    if (st == HB_OK) st = dev_alloc(p, (void **)&p->d_est, sizeof(float2) * nb * LL);
    if (st == HB_OK) st = dev_alloc(p, (void **)&p->d_work, 2 * sizeof(unsigned long long));
    if (st == HB_OK && hipMemset(p->d_work, 0, 2 * sizeof(unsigned long long)) != hipSuccess) st = HB_ERR_DEVICE;
    if (st == HB_OK && hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
        p->done = nullptr;
        st = HB_ERR_DEVICE;
    }
    if (st != HB_OK) {
        free_plan(p);
        return st;
    }
    // Device address of the static scratch, looked up here with the plan's
    // device current so that hb_estimate_frames_noalloc never has to.  A
    // failed lookup only disables that call (it then returns HB_ERR_DEVICE).
    if (static_scratch(device, &p->scratch) != hipSuccess) {
        (void)hipGetLastError();
        p->scratch = nullptr;
    }
    p->info.grid_split = p->split;
    p->info.n_tiles = p->n_tiles;
    p->info.n_nodes = p->n_nodes;
    const SkipRule rule = skip_rule((double)p->n_nodes, desc->thb_max, desc->posterior_tolerance, p->split);
    p->skip_log2 = rule.skip_log2;
    p->band_log2 = rule.band_log2;
    p->band_chunks = rule.band_chunks;
    p->info.skip_bound = rule.bound;
    p->info.skip_log2 = p->skip_log2;
    p->info.band_log2 = p->band_log2;
    p->info.band_chunks = p->band_chunks;
    *out = p;
    return HB_OK;
}

hb_status_t hb_set_forward_model(hb_plan_t p, const hb_forward_model_t *fm) {
    if (!p || !fm) return HB_ERR_INVALID_ARG;
    const int n = fm->n_wavelengths;
    if (n < 1 || n > 100000 || !fm->eps_hb || !fm->eps_hbo2 || !fm->response) return HB_ERR_INVALID_ARG;
    if (!is_finite(fm->path_length_cm) || !(fm->path_length_cm > 0)) return HB_ERR_INVALID_ARG;
    ForwardModel model;
    model.n = n;
    model.L = fm->path_length_cm;
    model.ehb.assign(fm->eps_hb, fm->eps_hb + n);
    model.eox.assign(fm->eps_hbo2, fm->eps_hbo2 + n);
    model.resp.assign(fm->response, fm->response + 3 * (size_t)n);
    for (int j = 0; j < n; ++j)
        if (!is_finite(model.ehb[j]) || !is_finite(model.eox[j])) return HB_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k) {
        double sum = 0;
        for (int j = 0; j < n; ++j) {
            const double v = model.resp[k * n + j];
            if (!is_finite(v) || v < 0) return HB_ERR_INVALID_ARG;
            sum += v;
        }
        if (!(sum > 0)) return HB_ERR_INVALID_ARG;
        for (int j = 0; j < n; ++j) model.resp[k * n + j] /= sum;
    }
    if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
    // From here on the plan's model state is being replaced: until every step
    // below has succeeded the plan has no model, so a failed replacement can
    // never leave new device values next to old tables.
    p->has_model = false;

    const hb_plan_desc_t &d = p->desc;
    double ref_thb = d.ref_thb, ref_so2 = d.ref_so2;
    if (std::isnan(ref_thb) && std::isnan(ref_so2)) {
        ref_thb = 0.5 * (d.thb_min + d.thb_max);
        ref_so2 = 0.5 * (d.so2_min + d.so2_max);
    }
    const double ref_hb = ref_thb * (1.0 - ref_so2), ref_hbo2 = ref_thb * ref_so2;

    // K0 (device, FP64): E and M.
    std::vector<double> in(5 + 5 * (size_t)n);
    in[0] = n;
    in[1] = model.L;
    in[2] = ref_hb;
    in[3] = ref_hbo2;
    in[4] = d.lambda;
    std::copy(model.ehb.begin(), model.ehb.end(), in.begin() + 5);
    std::copy(model.eox.begin(), model.eox.end(), in.begin() + 5 + n);
    std::copy(model.resp.begin(), model.resp.end(), in.begin() + 5 + 2 * n);
    if (p->d_k0 && p->k0_in < in.size()) {
        (void)hipFree(p->d_k0);
        p->d_k0 = nullptr;
    }
    if (!p->d_k0) {
        if (dev_alloc(p, (void **)&p->d_k0, sizeof(double) * (in.size() + 16)) != HB_OK) return HB_ERR_OUT_OF_MEMORY;
        p->k0_in = in.size();
    }
    double k0_out[14];
    if (hipMemcpy(p->d_k0, in.data(), sizeof(double) * in.size(), hipMemcpyHostToDevice) != hipSuccess)
        return HB_ERR_DEVICE;
    if (launch_tikhonov_fp64(p->d_k0, p->d_k0 + p->k0_in, p->d_mf, nullptr) != hipSuccess) return HB_ERR_DEVICE;
    if (hipMemcpy(k0_out, p->d_k0 + p->k0_in, sizeof(k0_out), hipMemcpyDeviceToHost) != hipSuccess)
        return HB_ERR_DEVICE;
    if (k0_out[13] != 1.0) return HB_ERR_ILL_POSED;

    // Centring: float32 reference intensities and the exact offsets they imply.
    double mu_ref[3];
    model.mu(ref_hb, ref_hbo2, mu_ref);
    double r[3];
    for (int k = 0; k < 3; ++k) {
        p->iref[k] = (float)std::exp(-mu_ref[k]);
        r[k] = -std::log((double)p->iref[k]);
    }
    p->scale = (float)std::sqrt(1.4426950408889634 / (2.0 * d.sigma * d.sigma));

    // Low-pass Tikhonov offset: c_ref + M (r - mu_ref), so that the low-pass
    // estimate is that offset + M z with z = ybar - r.
    // Float32 value and low part of each (the device's M parts come from K0).
    float mf_extra[2], mf_extra_lo[2];
    for (int i = 0; i < 2; ++i) {
        double v = (i == 0 ? ref_hb : ref_hbo2);
        for (int k = 0; k < 3; ++k) v += k0_out[6 + 3 * i + k] * (r[k] - mu_ref[k]);
        mf_extra[i] = (float)v;
        mf_extra_lo[i] = (float)(v - (double)mf_extra[i]);
    }
    if (hipMemcpy(p->d_mf + 6, mf_extra, sizeof(mf_extra), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_mf + 14, mf_extra_lo, sizeof(mf_extra_lo), hipMemcpyHostToDevice) != hipSuccess)
        return HB_ERR_DEVICE;

    std::vector<float> tiles, lo;
    double direct_index = 0.0;
    p->radius = build_supers(d, model, r, (double)p->scale, p->side, tiles, lo, direct_index);
    const double h_thb = d.grid_thb > 1 ? (d.thb_max - d.thb_min) / (d.grid_thb - 1) : 0.0;
    const double h_so2 = d.grid_so2 > 1 ? d.thb_max * (d.so2_max - d.so2_min) / (d.grid_so2 - 1) : 0.0;
    p->node_h = std::max(h_thb, h_so2);
    p->info.mfma_index = p->radius * p->radius * p->node_h;
    p->use_mfma = p->info.mfma_index <= kMfmaPrecisionBudget;
    p->info.mfma_df_constant = p->use_mfma && p->info.mfma_index > kMfmaDfcIndex ? 1 : 0;
    p->info.direct_index = direct_index;
    p->precise = !p->use_mfma && direct_index > kDirectPrecisionBudget;
    // Distance from the nodes beyond which a pixel's sums take double-float
    // logits: the MFMA kernel's room under its precision budget, the float32
    // direct kernel's, none for double-float logits everywhere.
    const double rh = p->radius * p->node_h;
    if (p->use_mfma)
        p->info.far_room = rh > 0.0 ? std::max(kFarRhoMin, kMfmaFarBudget / rh - p->radius) : INFINITY;
    else if (!p->precise)
        p->info.far_room = p->node_h > 0.0 ? std::sqrt(kDirectFarBudget / p->node_h) : INFINITY;
    else
        p->info.far_room = INFINITY;
    p->far_rho2 = std::isfinite(p->info.far_room) ? (float)(p->info.far_room * p->info.far_room) : INFINITY;
    p->info.posterior_kernel = p->use_mfma ? 0 : (p->precise ? 2 : 1);
    if (hipMemcpy(p->d_tiles, tiles.data(), sizeof(float) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess)
        return HB_ERR_DEVICE;
    if (hipMemcpy(p->d_lo, lo.data(), sizeof(float) * lo.size(), hipMemcpyHostToDevice) != hipSuccess)
        return HB_ERR_DEVICE;
    std::vector<uint16_t> split_ops;
    build_split_ops(tiles, p->n_tiles, p->side, split_ops);
    if (hipMemcpy(p->d_split, split_ops.data(), sizeof(uint16_t) * split_ops.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return HB_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return HB_ERR_DEVICE;

    for (int i = 0; i < 6; ++i) {
        p->info.E[i] = k0_out[i];
        p->info.M[i] = k0_out[6 + i];
    }
    double m_norm = 0.0;
    for (int i = 0; i < 2; ++i)
        m_norm = std::max(m_norm, std::fabs(k0_out[6 + 3 * i]) + std::fabs(k0_out[7 + 3 * i]) +
                                      std::fabs(k0_out[8 + 3 * i]));
    p->info.m_norm = m_norm;
    p->k1_df = (m_norm > kK1PrecisionBudget || p->dims.levels >= 3) ? 1 : 0;
    p->info.k1_double_float = p->k1_df;
    p->info.gamma = k0_out[12];
    p->info.ref_hb = ref_hb;
    p->info.ref_hbo2 = ref_hbo2;
    for (int k = 0; k < 3; ++k) p->info.mu_ref[k] = r[k];
    p->has_model = true;
    return HB_OK;
}

hb_status_t hb_estimate_frames(hb_plan_t p, const void *d_frames, int32_t n_frames, const hb_maps_t *d_out,
                               void *stream) {
    const hb_status_t st = check_call(p, d_frames, n_frames, d_out);
    if (st != HB_OK || n_frames == 0) return st;
    const CallBuffers cb{p->d_z, p->d_det, p->d_part, p->d_gref, p->d_est};
    return estimate(p, d_frames, n_frames, d_out, (hipStream_t)stream, cb, true);
}

hb_status_t hb_estimate_frames_noalloc(hb_plan_t p, const void *d_frames, int32_t n_frames,
                                       const hb_maps_t *d_out, void *stream) {
    const hb_status_t st = check_call(p, d_frames, n_frames, d_out);
    if (st != HB_OK || n_frames == 0) return st;
    if (!p->scratch) return HB_ERR_DEVICE;
    CallBuffers cb{};
    if (!carve_scratch(p, n_frames, (unsigned char *)p->scratch, cb)) return HB_ERR_SCRATCH;
    return estimate(p, d_frames, n_frames, d_out, (hipStream_t)stream, cb, false);
}

hb_status_t hb_destroy(hb_plan_t p) {
    if (!p) return HB_OK;
    hb_status_t st = HB_OK;
    // Wait for the plan's last uncaptured call only (other streams keep running).
    if (set_device(p->device) != HB_OK || hipEventSynchronize(p->done) != hipSuccess) st = HB_ERR_DEVICE;
    free_plan(p);
    return st;
}

size_t hb_plan_device_bytes(hb_plan_t p) { return p ? p->bytes : 0; }

hb_status_t hb_plan_get_info(hb_plan_t p, hb_plan_info_t *info) {
    if (!p || !info) return HB_ERR_INVALID_ARG;
    if (!p->has_model) return HB_ERR_NO_FORWARD_MODEL;
    *info = p->info;
    return HB_OK;
}

hb_status_t hb_plan_set_timing(hb_plan_t p, int32_t enable) {
    if (!p) return HB_ERR_INVALID_ARG;
    if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return HB_ERR_DEVICE;
    if (hipMemset(p->d_work, 0, 2 * sizeof(unsigned long long)) != hipSuccess) return HB_ERR_DEVICE;
    p->full_pairs = 0;
    p->timing = enable != 0;
    p->timed_calls = 0;
    return HB_OK;
}

hb_status_t hb_plan_get_work(hb_plan_t p, int64_t *evaluated, int64_t *full) {
    if (!p || !evaluated || !full) return HB_ERR_INVALID_ARG;
    if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
    unsigned long long v = 0;
    if (hipDeviceSynchronize() != hipSuccess) return HB_ERR_DEVICE;
    if (hipMemcpy(&v, p->d_work, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return HB_ERR_DEVICE;
    *evaluated = (int64_t)v;
    *full = p->full_pairs;
    return HB_OK;
}

hb_status_t hb_plan_get_far_pixels(hb_plan_t p, int64_t *pixels) {
    if (!p || !pixels) return HB_ERR_INVALID_ARG;
    if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
    unsigned long long v = 0;
    if (hipDeviceSynchronize() != hipSuccess) return HB_ERR_DEVICE;
    if (hipMemcpy(&v, p->d_work + 1, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return HB_ERR_DEVICE;
    *pixels = (int64_t)v;
    return HB_OK;
}

hb_status_t hb_plan_get_timing(hb_plan_t p, double ms[4], int64_t launches[4]) {
    if (!p || !ms || !launches) return HB_ERR_INVALID_ARG;
    for (int i = 0; i < 4; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
    for (int c = 0; c < p->timed_calls; ++c) {
        hipEvent_t *e = &p->events[4 * (size_t)c];
        if (hipEventSynchronize(e[3]) != hipSuccess) return HB_ERR_DEVICE;
        const int from[4] = {0, 1, 2, 0}, to[4] = {1, 2, 3, 3};
        for (int i = 0; i < 4; ++i) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, e[from[i]], e[to[i]]) != hipSuccess) return HB_ERR_DEVICE;
            ms[i] += t;
        }
        launches[0]++;
        if (p->desc.lowpass == HB_LOWPASS_BAYES) launches[1]++;
        launches[2]++;
        launches[3]++;
    }
    p->timed_calls = 0;
    return HB_OK;
}

hb_status_t hb_debug_copy(hb_plan_t p, int32_t which, int32_t frame, void *host_dst, size_t bytes) {
    if (!p || !host_dst) return HB_ERR_INVALID_ARG;
    if (frame < 0 || frame >= p->desc.max_batch) return HB_ERR_INVALID_ARG;
    const size_t LL = (size_t)p->dims.LL, HW = (size_t)p->desc.width * p->desc.height;
    const void *src = nullptr;
    size_t avail = 0;
    switch (which) {
        case HB_DEBUG_LOWPASS_OBS:
            src = p->d_z + (size_t)frame * 6 * LL;
            avail = sizeof(float) * 6 * LL;
            break;
        case HB_DEBUG_DETAILS:
            src = p->d_det + (size_t)frame * HW;
            avail = sizeof(float2) * HW;
            break;
        case HB_DEBUG_LOWPASS_EST:
            src = p->d_est + (size_t)frame * LL;
            avail = sizeof(float2) * LL;
            break;
        case HB_DEBUG_NODE_OPERANDS:
        case HB_DEBUG_SPLIT_OPERANDS: {
            if (!p->has_model) return HB_ERR_NO_FORWARD_MODEL;
            const int cps = (p->side / 4) * (p->side / 4);
            const size_t n_chunks = (size_t)p->n_tiles * cps;
            if (which == HB_DEBUG_SPLIT_OPERANDS) {
                src = p->d_split;
                avail = n_chunks * kSplitChunkBytes;
                break;
            }
            // gather the first 64 floats of every chunk from a host copy of the table
            if (bytes > n_chunks * 64 * sizeof(float)) return HB_ERR_INVALID_ARG;
            if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
            if (hipDeviceSynchronize() != hipSuccess) return HB_ERR_DEVICE;
            const int stride = super_floats(p->side);
            std::vector<float> table((size_t)p->n_tiles * stride);
            if (hipMemcpy(table.data(), p->d_tiles, sizeof(float) * table.size(), hipMemcpyDeviceToHost) !=
                hipSuccess)
                return HB_ERR_DEVICE;
            std::vector<float> ops(n_chunks * 64);
            for (size_t c = 0; c < n_chunks; ++c) {
                const size_t si = c / cps, ci = c % cps;
                const float *C = &table[si * stride + kSupHdr + kMaxProbes * kProbeFloats + ci * kChunkFloats];
                std::memcpy(&ops[c * 64], C, 64 * sizeof(float));
            }
            std::memcpy(host_dst, ops.data(), bytes);
            return HB_OK;
        }
        default:
            return HB_ERR_INVALID_ARG;
    }
    if (bytes > avail) return HB_ERR_INVALID_ARG;
    if (set_device(p->device) != HB_OK) return HB_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return HB_ERR_DEVICE;
    if (hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost) != hipSuccess) return HB_ERR_DEVICE;
    return HB_OK;
}

}  // extern "C"
