// Double-float (unevaluated sum of two float32) helpers for the few places
// where the path needs more than float32 precision without using FP64:
// the natural log of a ratio of two float32 intensities, sums, and products
// with a double-float operator.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace hb {

#define HB_HD __host__ __device__ __forceinline__

// The error-free transformations below are exact only if every addition and
// product in them is rounded on its own: HIP compiles device code with FMA
// contraction on, which after inlining could fuse a caller's product into
// the leading addition of a two-sum and lose the product's rounding error
// from the compensation term.  Each body therefore turns contraction off.

// s + e == a + b exactly (Knuth).
HB_HD void two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Requires |a| >= |b| (Dekker).
HB_HD void fast_two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
    s = a + b;
    e = b - (s - a);
}

// (hi, lo) += x
HB_HD void df_add(float &hi, float &lo, float x) {
#pragma clang fp contract(off)
    float s, e;
    two_sum(hi, x, s, e);
    e += lo;
    fast_two_sum(s, e, hi, lo);
}

// (hi, lo) += (xh, xl)
HB_HD void df_add2(float &hi, float &lo, float xh, float xl) {
#pragma clang fp contract(off)
    float s, e;
    two_sum(hi, xh, s, e);
    e += lo + xl;
    fast_two_sum(s, e, hi, lo);
}

// (hi, lo) += (mh + ml) (xh + xl), the leading product split exactly by FMA
// and the cross terms (below the leading one's rounding) added in float32.
HB_HD void df_mul_add(float &hi, float &lo, float mh, float ml, float xh, float xl) {
#pragma clang fp contract(off)
    const float p = mh * xh;
    const float pe = fmaf(mh, xh, -p);
    float s, e;
    two_sum(hi, p, s, e);
    e += lo + (pe + fmaf(mh, xl, ml * xh));
    fast_two_sum(s, e, hi, lo);
}

// ln(R / I) as a double-float for positive, finite float32 R and I, with an
// absolute error of a few 1e-10 over the ratios that occur here.
//   1. q = R/I as q_hi + q_lo (the residual of the division is exact by FMA);
//   2. q_hi = 2^e m with m in [sqrt(1/2), sqrt(2)), f = m - 1 exact;
//   3. ln(1 + f) = 2 atanh(s), s = f / (2 + f): 2s in double-float plus the
//      odd series s^3 (2/3 + 2/5 s^2 + ... + 2/15 s^12) in float32
//      (|s| <= 0.1716, truncation below 2e-14);
//   4. ln q = e ln2 + ln(1 + f) + q_lo / q_hi.
HB_HD void ln_ratio_df(float R, float I, float &hi, float &lo) {
#pragma clang fp contract(off)
    const float q = R / I;
    const float r = fmaf(-q, I, R);
    const float qlo_rel = (r / I) / q;
    int e;
    float m = frexpf(q, &e);  // q = m 2^e, m in [0.5, 1)
    if (m < 0.70710678f) {
        m *= 2.0f;
        e -= 1;
    }
    const float f = m - 1.0f;  // exact
    float dh, dl;
    fast_two_sum(2.0f, f, dh, dl);
    const float sh = f / dh;
    const float sl = (fmaf(-sh, dh, f) - sh * dl) / dh;
    const float s2 = sh * sh;
    float p = 2.0f / 15.0f;
    p = fmaf(p, s2, 2.0f / 13.0f);
    p = fmaf(p, s2, 2.0f / 11.0f);
    p = fmaf(p, s2, 2.0f / 9.0f);
    p = fmaf(p, s2, 2.0f / 7.0f);
    p = fmaf(p, s2, 2.0f / 5.0f);
    p = fmaf(p, s2, 2.0f / 3.0f);
    const float tail = fmaf(s2 * sh, p, 2.0f * s2 * sl);
    // ln2 split so that e * LN2_HI is exact for |e| < 2^9.
    const float LN2_HI = 0.693145751953125f;
    const float LN2_LO = 1.4286068203094172e-06f;
    const float ef = (float)e;
    hi = ef * LN2_HI;
    lo = 0.0f;
    df_add(hi, lo, 2.0f * sh);
    df_add(hi, lo, fmaf(ef, LN2_LO, 2.0f * sl + tail + qlo_rel));
}

#undef HB_HD

}  // namespace hb
