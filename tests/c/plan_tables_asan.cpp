// Memory-safety driver of the library's host table code, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host only
// (tests/test_asan.py).  It compiles the plan source into this translation
// unit and calls the FP64 super-tile table builder and the bf16 split-operand
// builder directly, for ragged and square grids of every super-tile side,
// with and without the illumination projection, and checks the layout's
// invariants on the way: probe counts, padded slots, absolute chunk boxes
// that hold their nodes, and that every split operand's three parts add up
// to its float value exactly.  It also checks
// the skip rule's stated bound against the tolerance over a range of grids
// and tolerances, and runs the plan's host-side validation (no device is
// needed for any of this).  The
// kernel launchers and the static scratch lookup are stubs: nothing here
// touches a GPU.  Prints "plan tables asan ok" and returns 0 on success.
#include "hb_plan.cpp"

#include <cstdio>

namespace hb {
hipError_t launch_tikhonov_fp64(const double *, double *, float *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_log_haar(const void *, int, const HaarArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_reference(const PosteriorArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_posterior(const PosteriorArgs &, bool, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_recompose(int, const RecomposeArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t static_scratch(int, void **ptr) {
    *ptr = nullptr;
    return hipErrorInvalidValue;
}
}  // namespace hb

static int fail(const char *what, int a, int b) {
    std::fprintf(stderr, "plan tables asan: %s (%d, %d)\n", what, a, b);
    return 1;
}

int main() {
    ForwardModel fm;
    fm.n = 9;
    fm.L = 0.1;
    for (int j = 0; j < fm.n; ++j) {
        fm.ehb.push_back(0.02 + 0.01 * j);
        fm.eox.push_back(0.05 - 0.004 * j);
    }
    for (int k = 0; k < 3; ++k) {
        double s = 0;
        std::vector<double> row;
        for (int j = 0; j < fm.n; ++j) row.push_back(std::exp(-0.5 * (j - 3.0 * k - 1.0) * (j - 3.0 * k - 1.0)));
        for (double v : row) s += v;
        for (double v : row) fm.resp.push_back(v / s);
    }
    const int grids[][2] = {{1, 1}, {3, 5}, {16, 16}, {33, 7}, {40, 40}, {100, 37}, {128, 128}, {256, 256}, {300, 17}};
    for (const auto &g : grids)
        for (int illum = 0; illum < 2; ++illum) {
            hb_plan_desc_t d;
            hb_plan_desc_default(&d);
            d.grid_thb = g[0];
            d.grid_so2 = g[1];
            d.illumination = illum;
            if (check_desc(&d) != HB_OK) return fail("descriptor rejected", g[0], g[1]);
            const int side = super_side(d.grid_thb, d.grid_so2);
            const int nsa = (d.grid_thb + side - 1) / side, nss = (d.grid_so2 + side - 1) / side;
            const int n_sup = nsa * nss;
            double mu_ref[3];
            fm.mu(50.0, 70.0, mu_ref);
            std::vector<float> table, lo;
            double direct_index = -1.0;
            const double radius = build_supers(d, fm, mu_ref, 40.0, side, table, lo, direct_index);
            if (!(radius >= 0.0) || table.size() != (size_t)n_sup * super_floats(side))
                return fail("table size or radius", g[0], g[1]);
            if (lo.size() != (size_t)n_sup * (side / 4) * (side / 4) * kLoFloats || !(direct_index >= 0.0))
                return fail("low parts or direct index", g[0], g[1]);
            std::vector<uint16_t> ops;
            build_split_ops(table, n_sup, side, ops);
            const int cps = (side / 4) * (side / 4);
            if (ops.size() != (size_t)n_sup * cps * 64 * (kSplitLaneBytes / 2)) return fail("ops size", g[0], g[1]);
            long real = 0;
            for (int si = 0; si < n_sup; ++si) {
                const float *T = &table[(size_t)si * super_floats(side)];
                int np;
                std::memcpy(&np, &T[14], sizeof(int));
                if (np < 1 || np > kMaxProbes) return fail("probe count", si, np);
                for (int c = 0; c < cps; ++c) {
                    const float *C = T + kSupHdr + kMaxProbes * kProbeFloats + (size_t)c * kChunkFloats;
                    const uint16_t *O = &ops[((size_t)si * cps + c) * 64 * (kSplitLaneBytes / 2)];
                    for (int j = 0; j < kChunkNodes; ++j) {
                        real += C[48 + j] != kPadLogit;
                        // the absolute chunk box holds the node: centre (double-float) plus
                        // its stored coordinates, in exact arithmetic
                        for (int k = 0; k < 3 && C[48 + j] != kPadLogit; ++k) {
                            const double at = ((double)T[k] + (double)T[3 + k]) + (double)C[16 * k + j];
                            if (!((double)C[96 + k] <= at && at <= (double)C[99 + k]))
                                return fail("absolute chunk box misses a node", si, c);
                        }
                        const float *LO = &lo[((size_t)si * cps + c) * kLoFloats];
                        for (int k = 0; k < 3; ++k)
                            if (C[48 + j] != kPadLogit && !(std::fabs(LO[16 * k + j]) <=
                                                             std::fabs(C[16 * k + j]) * 6.0e-8f + 1e-30f))
                                return fail("low part larger than half an ulp", si, c);
                        for (int gi = 0; gi < 4; ++gi) {
                            const uint16_t *L = O + (size_t)(16 * gi + j) * (kSplitLaneBytes / 2);
                            // parts 1, 2, 3 sit in slots 0, 1, 3 for coordinates and 0, 1, 2 for the norm
                            const int s3 = gi < 3 ? 3 : 2;
                            const float sum = (bf16_value(L[0]) + bf16_value(L[1])) + bf16_value(L[s3]);
                            if (sum != C[16 * gi + j]) return fail("split parts do not add up", si, c);
                        }
                    }
                }
            }
            if (real != (long)d.grid_thb * d.grid_so2) return fail("real node count", g[0], g[1]);
        }
    // Skip rule: the stated bound never exceeds the tolerance, the hard
    // threshold spends at most half of it, and the band sits kBandLog2 above.
    for (double G : {1.0, 16.0, 1024.0, 65536.0, 1048576.0})
        for (double thb_max : {100.0, 200.0})
            for (double tol : {1e-12, 1e-9, 1e-6, 1e-4, 1e-2, 1.0, 1e3})
                for (int split : {1, 3, 16}) {
                    const SkipRule r = skip_rule(G, thb_max, tol, split);
                    const double hard = 2.0 * G * std::exp2(-(double)r.skip_log2) * thb_max;
                    if (!(r.bound <= tol) || r.band_chunks < 0 || r.skip_log2 < kMinSkipLog2 ||
                        r.skip_log2 > kExactSkipLog2)
                        return fail("skip bound above tolerance", (int)G, split);
                    if (r.skip_log2 < kExactSkipLog2 && !(r.bound >= hard && hard <= 0.5 * tol + 1e-300))
                        return fail("hard threshold spends more than half", (int)G, split);
                    if (r.band_chunks > 0 && r.band_log2 != r.skip_log2 - kBandLog2)
                        return fail("band threshold", (int)G, split);
                    if (r.band_chunks == 0 && r.skip_log2 < kExactSkipLog2 && r.band_log2 != r.skip_log2 &&
                        r.band_log2 != r.skip_log2 - kBandLog2)
                        return fail("band threshold without budget", (int)G, split);
                }
    {
        const SkipRule e = skip_rule(65536.0, 200.0, 0.0, 1), n = skip_rule(65536.0, 200.0, -1.0, 1);
        const SkipRule d = skip_rule(65536.0, 200.0, 1e-6, 1);
        if (e.skip_log2 != kExactSkipLog2 || e.band_log2 != kExactSkipLog2 || e.band_chunks || e.bound != 0.0)
            return fail("exact skipping rule", 0, 0);
        if (!std::isinf(n.skip_log2) || !std::isinf(n.band_log2) || n.band_chunks || n.bound != 0.0)
            return fail("no-skipping rule", 0, 0);
        // 256 x 256 grid, thb_max 200, 1e-6 uM: T = 45, hard at 46, band to 40, 107 chunks
        if (d.skip_log2 != 46.0f || d.band_log2 != 40.0f || d.band_chunks != 107)
            return fail("default rule", (int)d.skip_log2, d.band_chunks);
    }
    // Host-side validation and the no-device path of plan creation.
    hb_plan_desc_t d;
    hb_plan_desc_default(&d);
    d.width = 30;
    d.levels = 2;
    hb_plan_t p = nullptr;
    if (hb_plan_create(&d, 0, &p) != HB_ERR_SHAPE || p) return fail("odd width accepted", 0, 0);
    if (hb_estimate_frames_noalloc(nullptr, nullptr, 1, nullptr, nullptr) != HB_ERR_INVALID_ARG)
        return fail("null plan accepted", 0, 0);
    for (int s = 0; s >= -9; --s)
        if (!hb_status_string((hb_status_t)s)) return fail("status string", s, 0);
    std::printf("plan tables asan ok\n");
    return 0;
}
