// HIP kernels of the haemoglobin-estimation path for gfx950 (MI355X).
//
//   K0  k_tikhonov_fp64     plan time, FP64: E, (E'E + gamma I)^-1 E'   (Method, Eq. 5)
//   K1  k_log_haar_reg<n>   log-attenuation, n-level 2D Haar, Tikhonov on the
//                           directional coefficients and the inverse Haar of
//                           that detail part, one block per thread (n <= 2)
//       k_log_haar          the same in LDS-staged strips (any n)  (Eq. 1-2, 4, 5)
//   K2a k_reference         best probe over the whole grid (split grids only)
//   K2  k_posterior         posterior mean over the THb x SO2 grid on the
//                           low-pass band (MFMA logits); with one split it
//                           also writes the maps                   (Fig. 1)
//       k_posterior_direct  the same with VALU logits (coarse grids, small sigma;
//                           double-float logits for the coarsest)
//   K3  k_recompose         split merge plus detail part to the THb/SO2 maps
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "hb_df.h"
#include "hb_internal.h"

namespace hb {

namespace {

// ---------------------------------------------------------------------------
// K0: Jacobian of the forward model at the reference point and the Tikhonov
// operator, in double precision.  in = [n, L, ref_hb, ref_hbo2, lambda,
// eps_hb[n], eps_hbo2[n], response[3][n] (rows normalised to unit sum)];
// out = [E(6), M(6), gamma, ok]; mf[0..5] = M rounded to float32 and
// mf[8..13] the low parts (M - mf[0..5], rounded), so that mf[i] + mf[8 + i]
// carries M to double-float precision (mf[6, 7] and mf[14, 15] are the
// host's low-pass offset).
// ---------------------------------------------------------------------------
__global__ void k_tikhonov_fp64(const double *__restrict__ in, double *__restrict__ out,
                                float *__restrict__ mf) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int n = (int)in[0];
    const double L = in[1], chb = in[2], chbo2 = in[3], lam = in[4];
    const double *ehb = in + 5, *eox = in + 5 + n, *resp = in + 5 + 2 * n;
    double E[6];
    for (int k = 0; k < 3; ++k) {
        double den = 0.0, nh = 0.0, no = 0.0;
        for (int j = 0; j < n; ++j) {
            double w = resp[k * n + j] * exp(-L * (ehb[j] * chb + eox[j] * chbo2));
            den += w;
            nh += w * ehb[j];
            no += w * eox[j];
        }
        E[2 * k] = L * nh / den;
        E[2 * k + 1] = L * no / den;
    }
    double a00 = 0, a01 = 0, a11 = 0;
    for (int k = 0; k < 3; ++k) {
        a00 += E[2 * k] * E[2 * k];
        a01 += E[2 * k] * E[2 * k + 1];
        a11 += E[2 * k + 1] * E[2 * k + 1];
    }
    const double gamma = lam * 0.5 * (a00 + a11);
    const double b00 = a00 + gamma, b11 = a11 + gamma;
    const double det = b00 * b11 - a01 * a01;
    const bool ok = fabs(det) > 1e-14 * (fabs(b00 * b11) + a01 * a01);
    const double i00 = b11 / det, i01 = -a01 / det, i11 = b00 / det;
    for (int k = 0; k < 3; ++k) {
        double m0 = i00 * E[2 * k] + i01 * E[2 * k + 1];
        double m1 = i01 * E[2 * k] + i11 * E[2 * k + 1];
        out[6 + k] = m0;
        out[9 + k] = m1;
        mf[k] = (float)m0;
        mf[3 + k] = (float)m1;
        mf[8 + k] = (float)(m0 - (double)(float)m0);   // low parts
        mf[11 + k] = (float)(m1 - (double)(float)m1);
    }
    for (int i = 0; i < 6; ++i) out[i] = E[i];
    out[12] = gamma;
    out[13] = ok ? 1.0 : 0.0;
}

// Clang vector types (the non-temporal builtins and the MFMA builtins take these).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x3 __attribute__((ext_vector_type(3)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
// Word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;

// ---------------------------------------------------------------------------
// Storage-type loads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float load_px(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float load_px(const __half *p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ float load_px(const uint16_t *p, size_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);  // bfloat16 -> float32 is exact
}

__device__ __forceinline__ void load4(const float *p, float v[4]) {
    const float4 x = *reinterpret_cast<const float4 *>(p);
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
}
__device__ __forceinline__ void load4(const __half *p, float v[4]) {
    const uint2 x = *reinterpret_cast<const uint2 *>(p);
    v[0] = __half2float(__ushort_as_half((unsigned short)(x.x & 0xffffu)));
    v[1] = __half2float(__ushort_as_half((unsigned short)(x.x >> 16)));
    v[2] = __half2float(__ushort_as_half((unsigned short)(x.y & 0xffffu)));
    v[3] = __half2float(__ushort_as_half((unsigned short)(x.y >> 16)));
}
__device__ __forceinline__ void load4(const uint16_t *p, float v[4]) {
    const uint2 x = *reinterpret_cast<const uint2 *>(p);
    v[0] = __uint_as_float(x.x << 16);
    v[1] = __uint_as_float(x.x & 0xffff0000u);
    v[2] = __uint_as_float(x.y << 16);
    v[3] = __uint_as_float(x.y & 0xffff0000u);
}

struct StripPos {
    int f, br, blk0, nb, ncols, Wt, row0, col0, B;
};

__device__ __forceinline__ StripPos strip_pos(const Dims &d) {
    StripPos s;
    int idx = blockIdx.x;
    const int sc = idx % d.strips_per_row;
    idx /= d.strips_per_row;
    s.br = idx % d.hl;
    s.f = idx / d.hl;
    s.blk0 = sc * d.bps;
    s.nb = min(d.bps, d.wl - s.blk0);
    s.B = 1 << d.levels;
    s.ncols = s.nb << d.levels;
    s.Wt = d.bps << d.levels;
    s.row0 = s.br << d.levels;
    s.col0 = s.blk0 << d.levels;
    return s;
}

// -ln(I / R) for a pixel relative to its block mean R, rinv = 1 / R: with
// x = (I - R) rinv (one rounded product), ln(1 + x) for |x| <= 1/16 is the
// series x + x^2 (-1/2 + x/3 - x^2/4 + x^3/5 - x^4/6 + x^5/7) (truncation
// below 2^-28 relative; 0.55 ulp worst measured against a double log1p over
// 5e7 samples), and log1pf beyond.  Both K1 variants use this, so they agree
// bit for bit.
__device__ __forceinline__ float neg_log_ratio(float I, float R, float rinv) {
    const float x = (I - R) * rinv;
    if (fabsf(x) <= 0.0625f) {
        float q = fmaf(x, 1.0f / 7.0f, -1.0f / 6.0f);
        q = fmaf(q, x, 0.2f);
        q = fmaf(q, x, -0.25f);
        q = fmaf(q, x, 1.0f / 3.0f);
        q = fmaf(q, x, -0.5f);
        return -fmaf(x * x, q, x);
    }
    return -log1pf(x);
}

// ---------------------------------------------------------------------------
// K1: one workgroup per strip of 2^n pixel rows x (bps * 2^n) columns.
//
// Numerics: each block's log-attenuation is carried relative to the block's
// mean intensity R, u(q) = -ln(I(q)/R) = -log1p((I(q) - R)/R), so directional
// coefficients are computed from small, accurately rounded numbers.  Details of
// u equal those of y = -ln I (they differ by a per-block constant); the block
// mean of y is recovered as -ln(R/I_ref) + mean(u) relative to the plan's
// reference intensity I_ref.
//
// DF (three levels or more): u and the Haar cascade are double-floats (the
// low parts in s_i once the intensities are used) and the Tikhonov operator
// is applied with M as a double-float.  With float32 u, the rounding of u,
// which grows with the block, reaches the maps through |M| (1e3 to 2e3 uM
// per unit) at up to 1.3e-4 uM for three levels; the double-float form
// leaves the rounding of the Tikhonov results and of the inverse Haar.
// ---------------------------------------------------------------------------
template <typename T, bool DF>
__global__ __launch_bounds__(kBlockThreads) void k_log_haar(const T *__restrict__ frames, HaarArgs a) {
    __shared__ float s_i[3][kStripPixels];
    __shared__ float s_u[3][kStripPixels];
    __shared__ float s_r[3][kStripPixels / 4];
    const Dims &d = a.d;
    const StripPos s = strip_pos(d);
    const int n = d.levels, B = s.B, Wt = s.Wt, ncols = s.ncols;
    const int tid = threadIdx.x;

    // 1. Coalesced load of the strip, clamp.  Each row of the strip is one
    //    contiguous HWC run of ncols * 3 values; with 4-value alignment the
    //    loads are 16-byte (FP32) or 8-byte (FP16/BF16) vectors, all issued
    //    before any is used.
    const size_t frame_off = (size_t)s.f * d.H * d.W * 3;
    const int run = ncols * 3;
    const T *__restrict__ base = frames + frame_off + ((size_t)s.row0 * d.W + s.col0) * 3;
    const size_t row_stride = (size_t)d.W * 3;
    auto put = [&](int r, int p, float v) {
        const int c = p / 3, k = p - 3 * c;
        v = (v < a.floor) ? a.floor : v;  // NaN stays NaN
        s_i[k][r * Wt + c] = v;
        s_u[k][r * Wt + c] = v;
    };
    if (a.vec4 && (d.W & 3) == 0 && (run & 3) == 0) {
        const int r4 = run >> 2, total = B * r4;
        constexpr int kMaxVec = kStripPixels * 3 / 4 / kBlockThreads;   // 6
        float v[kMaxVec][4];
        int rr[kMaxVec], jj[kMaxVec];
#pragma unroll
        for (int t = 0; t < kMaxVec; ++t) {
            const int idx = tid + t * kBlockThreads;
            rr[t] = idx < total ? idx / r4 : 0;
            jj[t] = idx < total ? idx - rr[t] * r4 : -1;
            if (jj[t] >= 0) load4(base + rr[t] * row_stride + 4 * jj[t], v[t]);
        }
#pragma unroll
        for (int t = 0; t < kMaxVec; ++t)
            if (jj[t] >= 0)
#pragma unroll
                for (int e = 0; e < 4; ++e) put(rr[t], 4 * jj[t] + e, v[t][e]);
    } else {
        for (int r = 0; r < B; ++r)
            for (int p = tid; p < run; p += kBlockThreads) put(r, p, load_px(base, r * row_stride + p));
    }
    __syncthreads();

    // 2. Block sums of intensity by a 2x2 cascade, then the block mean R.
    for (int l = 1; l <= n; ++l) {
        const int h = 1 << (l - 1), g2 = 2 * h, gc = ncols >> l;
        for (int r = 0; r < B; r += g2)
            for (int q = tid; q < gc * 3; q += kBlockThreads) {
                const int cg = q / 3, k = q - 3 * cg, c = cg * g2;
                float *u = s_u[k];
                u[r * Wt + c] = (u[r * Wt + c] + u[r * Wt + c + h]) + (u[(r + h) * Wt + c] + u[(r + h) * Wt + c + h]);
            }
        __syncthreads();
    }
    if (n > 0) {
        const float inv = 1.0f / (float)(1 << (2 * n));
        for (int q = tid; q < s.nb * 3; q += kBlockThreads) {
            const int j = q / 3, k = q - 3 * j;
            s_r[k][j] = s_u[k][j << n] * inv;
        }
    }
    __syncthreads();

    // 3. Log-ratio to the block reference.
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            for (int c = tid; c < ncols; c += kBlockThreads) {
                const float I = s_i[k][r * Wt + c];
                const float R = (n > 0) ? s_r[k][c >> n] : I;
                if constexpr (DF) {
                    // with no level u = 0 exactly, and s_i keeps the intensity
                    // that step 5 then reads as the block reference
                    float uh = 0.0f, ul = 0.0f;
                    if (n > 0) {
                        ln_ratio_df(R, I, uh, ul);   // ln(R / I) = -ln(I / R)
                        s_i[k][r * Wt + c] = ul;
                    }
                    s_u[k][r * Wt + c] = uh;
                } else {
                    s_u[k][r * Wt + c] = neg_log_ratio(I, R, 1.0f / R);
                }
            }
    __syncthreads();

    // 4. n-level Haar in place.  Window (a, b, c, d) = (r,c), (r,c+h), (r+h,c),
    //    (r+h,c+h); coefficients = window * H (Eq. 1-2): LL -> (r,c),
    //    row difference -> (r+h,c), diagonal -> (r+h,c+h), column difference -> (r,c+h).
    for (int l = 1; l <= n; ++l) {
        const int h = 1 << (l - 1), g2 = 2 * h, gc = ncols >> l;
        for (int r = 0; r < B; r += g2)
            for (int q = tid; q < gc * 3; q += kBlockThreads) {
                const int cg = q / 3, k = q - 3 * cg, c = cg * g2;
                float *u = s_u[k];
                const int i0 = r * Wt + c, i1 = i0 + h, i2 = (r + h) * Wt + c, i3 = i2 + h;
                if constexpr (DF) {
                    const float *ul = s_i[k];
                    float ah = u[i0], al = ul[i0], bh = u[i2], bl = ul[i2];
                    float ch = ah, cl = al, dh = bh, dl = bl;
                    df_add2(ah, al, u[i1], ul[i1]);     // w0 + w1
                    df_add2(bh, bl, u[i3], ul[i3]);     // w2 + w3
                    df_add2(ch, cl, -u[i1], -ul[i1]);   // w0 - w1
                    df_add2(dh, dl, -u[i3], -ul[i3]);   // w2 - w3
                    float llh = ah, lll = al, d1h = ah, d1l = al, d2h = ch, d2l = cl, d3h = ch, d3l = cl;
                    df_add2(llh, lll, bh, bl);
                    df_add2(d1h, d1l, -bh, -bl);
                    df_add2(d2h, d2l, -dh, -dl);
                    df_add2(d3h, d3l, dh, dl);
                    float *vl = s_i[k];
                    u[i0] = 0.5f * llh;
                    vl[i0] = 0.5f * lll;
                    u[i2] = 0.5f * d1h;
                    vl[i2] = 0.5f * d1l;
                    u[i3] = 0.5f * d2h;
                    vl[i3] = 0.5f * d2l;
                    u[i1] = 0.5f * d3h;
                    vl[i1] = 0.5f * d3l;
                } else {
                    const float w0 = u[i0], w1 = u[i1];
                    const float w2 = u[i2], w3 = u[i3];
                    u[i0] = 0.5f * ((w0 + w1) + (w2 + w3));
                    u[i2] = 0.5f * ((w0 + w1) - (w2 + w3));
                    u[i3] = 0.5f * ((w0 - w1) - (w2 - w3));
                    u[i1] = 0.5f * ((w0 - w1) + (w2 - w3));
                }
            }
        __syncthreads();
    }

    // 5. Centred low-pass observation z = ybar - mu_ref per block, as a
    //    double-float: ybar - mu_ref = ln(I_ref / R) + mean(u).  With the
    //    illumination term z loses its mean over the channels (the component
    //    along (1,1,1) that a common log offset can absorb).
    const float invB = 1.0f / (float)B;
    if (!a.project) {
        for (int q = tid; q < s.nb * 3; q += kBlockThreads) {
            const int j = q / 3, k = q - 3 * j;
            const float R = (n > 0) ? s_r[k][j] : s_i[k][j];
            float zh, zl;
            ln_ratio_df(a.iref[k], R, zh, zl);
            if constexpr (DF)
                df_add2(zh, zl, s_u[k][j << n] * invB, n > 0 ? s_i[k][j << n] * invB : 0.0f);
            else
                df_add(zh, zl, s_u[k][j << n] * invB);
            const size_t o = (size_t)s.br * d.wl + s.blk0 + j;
            a.z[((size_t)s.f * 6 + k) * d.LL + o] = zh;
            a.z[((size_t)s.f * 6 + 3 + k) * d.LL + o] = zl;
        }
    } else {
        for (int j = tid; j < s.nb; j += kBlockThreads) {
            float zh[3], zl[3];
            for (int k = 0; k < 3; ++k) {
                const float R = (n > 0) ? s_r[k][j] : s_i[k][j];
                ln_ratio_df(a.iref[k], R, zh[k], zl[k]);
                if constexpr (DF)
                    df_add2(zh[k], zl[k], s_u[k][j << n] * invB, n > 0 ? s_i[k][j << n] * invB : 0.0f);
                else
                    df_add(zh[k], zl[k], s_u[k][j << n] * invB);
            }
            float sh = zh[0], sl = zl[0];
            df_add2(sh, sl, zh[1], zl[1]);
            df_add2(sh, sl, zh[2], zl[2]);
            // (sh + sl) / 3: the remainder of the leading quotient is exact by FMA
            const float mh = sh * (1.0f / 3.0f);
            const float ml = (fmaf(-3.0f, mh, sh) + sl) * (1.0f / 3.0f);
            const size_t o = (size_t)s.br * d.wl + s.blk0 + j;
            for (int k = 0; k < 3; ++k) {
                df_add2(zh[k], zl[k], -mh, -ml);
                a.z[((size_t)s.f * 6 + k) * d.LL + o] = zh[k];
                a.z[((size_t)s.f * 6 + 3 + k) * d.LL + o] = zl[k];
            }
        }
    }

    // 6. Tikhonov on every directional coefficient: (Hb, HbO2) = M * (R, G, B),
    //    the low-pass slot set to 0 (s_i, read by step 5 when n = 0, then
    //    holds the result).
    __syncthreads();
    const float m0 = a.M[0], m1 = a.M[1], m2 = a.M[2], m3 = a.M[3], m4 = a.M[4], m5 = a.M[5];
    for (int r = 0; r < B; ++r)
        for (int c = tid; c < ncols; c += kBlockThreads) {
            float ox = 0.0f, oy = 0.0f;
            if (((r | c) & (B - 1)) != 0) {
                const float d0 = s_u[0][r * Wt + c], d1 = s_u[1][r * Wt + c], d2 = s_u[2][r * Wt + c];
                if constexpr (DF) {
                    // every low part is read before this thread overwrites its element
                    const float e0 = s_i[0][r * Wt + c], e1 = s_i[1][r * Wt + c], e2 = s_i[2][r * Wt + c];
                    float xh = 0.0f, xl = 0.0f, yh = 0.0f, yl = 0.0f;
                    df_mul_add(xh, xl, m0, a.M[8], d0, e0);
                    df_mul_add(xh, xl, m1, a.M[9], d1, e1);
                    df_mul_add(xh, xl, m2, a.M[10], d2, e2);
                    df_mul_add(yh, yl, m3, a.M[11], d0, e0);
                    df_mul_add(yh, yl, m4, a.M[12], d1, e1);
                    df_mul_add(yh, yl, m5, a.M[13], d2, e2);
                    ox = xh + xl;
                    oy = yh + yl;
                } else {
                    ox = fmaf(m0, d0, fmaf(m1, d1, m2 * d2));
                    oy = fmaf(m3, d0, fmaf(m4, d1, m5 * d2));
                }
            }
            s_i[0][r * Wt + c] = ox;
            s_i[1][r * Wt + c] = oy;
        }
    __syncthreads();

    // 7. Inverse Haar of the detail part (Eq. 4: window = coefficients * H,
    //    levels n..1): the maps are this plus the block's low-pass estimate.
    for (int l = n; l >= 1; --l) {
        const int h = 1 << (l - 1), g2 = 2 * h, gc = ncols >> l;
        for (int r = 0; r < B; r += g2)
            for (int q = tid; q < gc * 2; q += kBlockThreads) {
                const int k = q & 1, c = (q >> 1) * g2;
                float *u = s_i[k];
                const float ll = u[r * Wt + c], d1 = u[(r + h) * Wt + c];
                const float d2 = u[(r + h) * Wt + c + h], d3 = u[r * Wt + c + h];
                u[r * Wt + c] = 0.5f * ((ll + d1) + (d2 + d3));
                u[r * Wt + c + h] = 0.5f * ((ll + d1) - (d2 + d3));
                u[(r + h) * Wt + c] = 0.5f * ((ll - d1) - (d2 - d3));
                u[(r + h) * Wt + c + h] = 0.5f * ((ll - d1) + (d2 - d3));
            }
        __syncthreads();
    }
    for (int r = 0; r < B; ++r)
        for (int c = tid; c < ncols; c += kBlockThreads)
            a.det[((size_t)s.f * d.H + s.row0 + r) * d.W + s.col0 + c] =
                make_float2(s_i[0][r * Wt + c], s_i[1][r * Wt + c]);
}

// ---------------------------------------------------------------------------
// K1, register variant for n <= 2: one thread per 2^n x 2^n block, the block
// held in registers (no LDS, no barriers), the strip kernel's arithmetic in
// the same order (so both give the same bits).  Each block row is a run of
// 3 * 2^n stored values starting at a multiple of 2^n values: three vector
// loads of 2^n values when the frames pointer is aligned to 2^n values.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ float half_bits(unsigned b);
template <>
__device__ __forceinline__ float half_bits<__half>(unsigned b) {
    return __half2float(__ushort_as_half((unsigned short)b));
}
template <>
__device__ __forceinline__ float half_bits<uint16_t>(unsigned b) {
    return __uint_as_float(b << 16);  // bfloat16 -> float32 is exact
}

template <typename T, int BW>
__device__ __forceinline__ void load_run(const T *p, float *v) {
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (BW == 4) {
            const float4 x = *reinterpret_cast<const float4 *>(p);
            v[0] = x.x;
            v[1] = x.y;
            v[2] = x.z;
            v[3] = x.w;
        } else if constexpr (BW == 2) {
            const float2 x = *reinterpret_cast<const float2 *>(p);
            v[0] = x.x;
            v[1] = x.y;
        } else {
            v[0] = p[0];
        }
    } else {
        if constexpr (BW == 4) {
            const uint2 x = *reinterpret_cast<const uint2 *>(p);
            v[0] = half_bits<T>(x.x & 0xffffu);
            v[1] = half_bits<T>(x.x >> 16);
            v[2] = half_bits<T>(x.y & 0xffffu);
            v[3] = half_bits<T>(x.y >> 16);
        } else if constexpr (BW == 2) {
            const unsigned x = *reinterpret_cast<const unsigned *>(p);
            v[0] = half_bits<T>(x & 0xffffu);
            v[1] = half_bits<T>(x >> 16);
        } else {
            v[0] = half_bits<T>(*reinterpret_cast<const unsigned short *>(p));
        }
    }
}

// Detail-part rows are streamed out (non-temporal): they are read again
// only by the posterior's epilogue or the recomposition kernel.
template <int BW>
__device__ __forceinline__ void store_row(float2 *p, const float2 *o) {
    if constexpr (BW == 4) {
        __builtin_nontemporal_store(f32x4{o[0].x, o[0].y, o[1].x, o[1].y}, reinterpret_cast<f32x4 *>(p));
        __builtin_nontemporal_store(f32x4{o[2].x, o[2].y, o[3].x, o[3].y}, reinterpret_cast<f32x4 *>(p) + 1);
    } else if constexpr (BW == 2) {
        __builtin_nontemporal_store(f32x4{o[0].x, o[0].y, o[1].x, o[1].y}, reinterpret_cast<f32x4 *>(p));
    } else {
        __builtin_nontemporal_store(f32x2{o[0].x, o[0].y}, reinterpret_cast<f32x2 *>(p));
    }
}

template <typename T, int N, bool DF>
__global__ __launch_bounds__(kBlockThreads) void k_log_haar_reg(const T *__restrict__ frames, HaarArgs a) {
    constexpr int BW = 1 << N, NP = BW * BW;
    const Dims &d = a.d;
    const long long idx = (long long)blockIdx.x * kBlockThreads + threadIdx.x;
    if (idx >= (long long)a.n_frames * d.LL) return;
    const int f = (int)(idx / d.LL);
    const long long q = idx - (long long)f * d.LL;
    const int br = (int)(q / d.wl), bc = (int)(q - (long long)br * d.wl);
    const int row0 = br << N, col0 = bc << N;
    const T *__restrict__ base = frames + ((size_t)f * d.H * d.W + (size_t)row0 * d.W + col0) * 3;

    // 1. Loads (all issued first), clamp.  I[k][r * BW + c].
    float v[BW][3 * BW];
#pragma unroll
    for (int r = 0; r < BW; ++r)
#pragma unroll
        for (int t = 0; t < 3; ++t) load_run<T, BW>(base + (size_t)r * d.W * 3 + t * BW, &v[r][t * BW]);
    float I[3][NP], u[3][NP];
#pragma unroll
    for (int r = 0; r < BW; ++r)
#pragma unroll
        for (int e = 0; e < 3 * BW; ++e) {
            const float x = v[r][e];
            I[e % 3][r * BW + e / 3] = (x < a.floor) ? a.floor : x;  // NaN stays NaN
        }

    // 2. Block sum by the 2x2 cascade, block mean R.
    float R[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int i = 0; i < NP; ++i) u[k][i] = I[k][i];
#pragma unroll
        for (int l = 1; l <= N; ++l) {
            const int h = 1 << (l - 1), g2 = 2 * h;
#pragma unroll
            for (int r = 0; r < BW; r += g2)
#pragma unroll
                for (int c = 0; c < BW; c += g2)
                    u[k][r * BW + c] = (u[k][r * BW + c] + u[k][r * BW + c + h]) +
                                       (u[k][(r + h) * BW + c] + u[k][(r + h) * BW + c + h]);
        }
        R[k] = (N > 0) ? u[k][0] * (1.0f / (float)(1 << (2 * N))) : I[k][0];
    }

    // 3. Log-ratio to the block mean; 4. Haar in place (window * H, Eq. 1-2).
    //    DF: u, the cascade and (step 6) the Tikhonov apply as double-floats
    //    (low parts in ul), as in the strip kernel.
    float ul[3][NP];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float rinv = 1.0f / R[k];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if constexpr (DF)
                ln_ratio_df(R[k], I[k][i], u[k][i], ul[k][i]);   // ln(R / I) = -ln(I / R)
            else
                u[k][i] = neg_log_ratio(I[k][i], R[k], rinv);
        }
#pragma unroll
        for (int l = 1; l <= N; ++l) {
            const int h = 1 << (l - 1), g2 = 2 * h;
#pragma unroll
            for (int r = 0; r < BW; r += g2)
#pragma unroll
                for (int c = 0; c < BW; c += g2) {
                    const int i0 = r * BW + c, i1 = i0 + h, i2 = (r + h) * BW + c, i3 = i2 + h;
                    if constexpr (DF) {
                        float ah = u[k][i0], al = ul[k][i0], bh = u[k][i2], bl = ul[k][i2];
                        float ch = ah, cl = al, dh = bh, dl = bl;
                        df_add2(ah, al, u[k][i1], ul[k][i1]);     // w0 + w1
                        df_add2(bh, bl, u[k][i3], ul[k][i3]);     // w2 + w3
                        df_add2(ch, cl, -u[k][i1], -ul[k][i1]);   // w0 - w1
                        df_add2(dh, dl, -u[k][i3], -ul[k][i3]);   // w2 - w3
                        float llh = ah, lll = al, d1h = ah, d1l = al, d2h = ch, d2l = cl, d3h = ch, d3l = cl;
                        df_add2(llh, lll, bh, bl);
                        df_add2(d1h, d1l, -bh, -bl);
                        df_add2(d2h, d2l, -dh, -dl);
                        df_add2(d3h, d3l, dh, dl);
                        u[k][i0] = 0.5f * llh;
                        ul[k][i0] = 0.5f * lll;
                        u[k][i2] = 0.5f * d1h;
                        ul[k][i2] = 0.5f * d1l;
                        u[k][i3] = 0.5f * d2h;
                        ul[k][i3] = 0.5f * d2l;
                        u[k][i1] = 0.5f * d3h;
                        ul[k][i1] = 0.5f * d3l;
                    } else {
                        const float w0 = u[k][i0], w1 = u[k][i1];
                        const float w2 = u[k][i2], w3 = u[k][i3];
                        u[k][i0] = 0.5f * ((w0 + w1) + (w2 + w3));
                        u[k][i2] = 0.5f * ((w0 + w1) - (w2 + w3));
                        u[k][i3] = 0.5f * ((w0 - w1) - (w2 - w3));
                        u[k][i1] = 0.5f * ((w0 - w1) + (w2 - w3));
                    }
                }
        }
    }

    // 5. Centred low-pass observation (double-float), optionally projected.
    const float invB = 1.0f / (float)BW;
    float zh[3], zl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ln_ratio_df(a.iref[k], R[k], zh[k], zl[k]);
        if constexpr (DF)
            df_add2(zh[k], zl[k], u[k][0] * invB, ul[k][0] * invB);
        else
            df_add(zh[k], zl[k], u[k][0] * invB);
    }
    if (a.project) {
        float sh = zh[0], sl = zl[0];
        df_add2(sh, sl, zh[1], zl[1]);
        df_add2(sh, sl, zh[2], zl[2]);
        const float mh = sh * (1.0f / 3.0f);
        const float ml = (fmaf(-3.0f, mh, sh) + sl) * (1.0f / 3.0f);
#pragma unroll
        for (int k = 0; k < 3; ++k) df_add2(zh[k], zl[k], -mh, -ml);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a.z[((size_t)f * 6 + k) * d.LL + q] = zh[k];
        a.z[((size_t)f * 6 + 3 + k) * d.LL + q] = zl[k];
    }

    // 6. Tikhonov on the directional coefficients (low-pass slot 0); 7. the
    //    inverse Haar of this detail part; block rows as vector stores.
    const float m0 = a.M[0], m1 = a.M[1], m2 = a.M[2], m3 = a.M[3], m4 = a.M[4], m5 = a.M[5];
    float o[2][NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        o[0][i] = o[1][i] = 0.0f;
        if (i != 0) {
            const float d0 = u[0][i], d1 = u[1][i], d2 = u[2][i];
            if constexpr (DF) {
                float xh = 0.0f, xl = 0.0f, yh = 0.0f, yl = 0.0f;
                df_mul_add(xh, xl, m0, a.M[8], d0, ul[0][i]);
                df_mul_add(xh, xl, m1, a.M[9], d1, ul[1][i]);
                df_mul_add(xh, xl, m2, a.M[10], d2, ul[2][i]);
                df_mul_add(yh, yl, m3, a.M[11], d0, ul[0][i]);
                df_mul_add(yh, yl, m4, a.M[12], d1, ul[1][i]);
                df_mul_add(yh, yl, m5, a.M[13], d2, ul[2][i]);
                o[0][i] = xh + xl;
                o[1][i] = yh + yl;
            } else {
                o[0][i] = fmaf(m0, d0, fmaf(m1, d1, m2 * d2));
                o[1][i] = fmaf(m3, d0, fmaf(m4, d1, m5 * d2));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int l = N; l >= 1; --l) {
            const int h = 1 << (l - 1), g2 = 2 * h;
#pragma unroll
            for (int r = 0; r < BW; r += g2)
#pragma unroll
                for (int c = 0; c < BW; c += g2) {
                    const float ll = o[k][r * BW + c], d1 = o[k][(r + h) * BW + c];
                    const float d2 = o[k][(r + h) * BW + c + h], d3 = o[k][r * BW + c + h];
                    o[k][r * BW + c] = 0.5f * ((ll + d1) + (d2 + d3));
                    o[k][r * BW + c + h] = 0.5f * ((ll + d1) - (d2 + d3));
                    o[k][(r + h) * BW + c] = 0.5f * ((ll - d1) - (d2 - d3));
                    o[k][(r + h) * BW + c + h] = 0.5f * ((ll - d1) + (d2 - d3));
                }
        }
#pragma unroll
    for (int r = 0; r < BW; ++r) {
        float2 row[BW];
#pragma unroll
        for (int c = 0; c < BW; ++c) row[c] = make_float2(o[0][r * BW + c], o[1][r * BW + c]);
        store_row<BW>(a.det + ((size_t)f * d.H + row0 + r) * d.W + col0, row);
    }
}

// Maps of V consecutive pixels (offset o) from their detail part and the
// block's low-pass estimate e; vector stores when V > 1 (the host checks the
// alignment of the map pointers).  Null maps are skipped.
template <int V>
__device__ __forceinline__ void write_maps(float *mhb, float *mox, float *mth, float *mso, float thb_eps, size_t o,
                                           float2 e, const float2 *dp) {
    float hb[V], ox[V], th[V], so[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        hb[i] = e.x + dp[i].x;
        ox[i] = e.y + dp[i].y;
        th[i] = hb[i] + ox[i];
        so[i] = (th[i] > thb_eps) ? ox[i] / th[i] : __builtin_nanf("");
    }
    // streaming stores (non-temporal): the maps are not read again here
    auto put = [&](float *m, const float *v) {
        if (!m) return;
        if constexpr (V == 4) {
            __builtin_nontemporal_store(f32x4{v[0], v[1], v[2], v[3]}, reinterpret_cast<f32x4 *>(m + o));
        } else if constexpr (V == 2) {
            __builtin_nontemporal_store(f32x2{v[0], v[1]}, reinterpret_cast<f32x2 *>(m + o));
        } else {
            __builtin_nontemporal_store(v[0], m + o);
        }
    };
    put(mhb, hb);
    put(mox, ox);
    put(mth, th);
    put(mso, so);
}

// V consecutive detail-part values from offset o (streaming loads).
template <int V>
__device__ __forceinline__ void load_detail(const float2 *det, size_t o, float2 *dp) {
    if constexpr (V == 4) {
        const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(det + o));
        const f32x4 y = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(det + o + 2));
        dp[0] = make_float2(x.x, x.y);
        dp[1] = make_float2(x.z, x.w);
        dp[2] = make_float2(y.x, y.y);
        dp[3] = make_float2(y.z, y.w);
    } else if constexpr (V == 2) {
        const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(det + o));
        dp[0] = make_float2(x.x, x.y);
        dp[1] = make_float2(x.z, x.w);
    } else {
        const f32x2 x = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(det + o));
        dp[0] = make_float2(x.x, x.y);
    }
}

// ---------------------------------------------------------------------------
// K2: posterior mean over the grid on the low-pass band.
//
// Likelihood in base 2 with scaled coordinates: t_g = -|s z - s mu'_g|^2 with
// s = sqrt(log2(e) / (2 sigma^2)) and mu' centred on mu_ref.  Inside a
// super-tile both the observation r = s z - centre (formed from the
// double-float observation) and the node coordinates v_g are small.
//
// The weights are taken relative to a per-pixel reference m fixed before the
// main loop: m_lo = best logit of one probe node per 8 x 8 patch (a true
// logit, so the top weight is >= 1 and the sum cannot underflow), m_up = best
// upper bound over the super-tiles' boxes.  If m_up - m_lo <= kFarGap for the
// whole wave, m = m_lo and every weight lies in [0, 2^kFarGap]; otherwise the
// wave first takes the exact maximum over its nodes.  Moments are accumulated
// relative to the super-tile's centre inside a super-tile and merged relative
// to the pixel's anchor (its best probe node); the partial sums of the lanes
// are combined with compensated pairwise steps and the grid splits with Kahan
// compensation (recomposition kernel).
//
// Two kernels share this: k_posterior (MFMA logits, used when every
// super-tile is compact in scaled units) and k_posterior_direct (VALU
// difference form, for grids too coarse for the expanded logit's precision).
// ---------------------------------------------------------------------------
constexpr float kFarGap = 64.0f;

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Sum over the four lanes l, l ^ 16, l ^ 32, l ^ 48, each pairwise step exact
// up to a carried error term (two-sum), the error added at the end.
__device__ __forceinline__ float lane_sum_rows(float x) {
    float e = 0.0f;
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
        const float y = __shfl_xor(x, o), ye = __shfl_xor(e, o);
        float s, err;
        two_sum(x, y, s, err);
        x = s;
        e = (e + ye) + err;
    }
    return x + e;
}

__device__ __forceinline__ f32x4 mfma_16x16x32_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Nearest bf16 (ties to even) of lo and hi, packed (lo in the low half).
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// Pixel (B) operand of the split bf16 MFMA.  Lane groups 0..2 carry the
// exact three-part split of u (twice the pixel's coordinate) in the order
// that pairs with the node parts of the split operand table; group 3 carries
// ones that pick up the node's squared-norm parts and the three parts of the
// pixel's constant c = -(|r|^2 + m), paired with node ones.  The parts are
// x1 = bf16(x), x2 = bf16(x - x1), x3 = bf16(x - x1 - x2), each difference
// exact in float32.
__device__ __forceinline__ bf16x8 split_pixel_operand(float u, float c, bool coord) {
    const float x = coord ? u : c;
    const unsigned p11 = pack_bf16(x, x);                        // (x1, x1)
    const float r1 = x - __uint_as_float(p11 << 16);             // x - x1, exact
    const float r2 = r1 - __uint_as_float(pack_bf16(r1, r1) << 16);   // r1 - x2, exact
    const unsigned p23 = pack_bf16(r1, r2);                      // (x2, x3)
    u32x4 b;
    b[0] = coord ? p11 : 0x3f803f80u;                            // (x1, x1) or (1, 1)
    b[1] = pack_bf16(coord ? r1 : 1.0f, x);                      // (x2, x1) or (1, x1)
    b[2] = p23;                                                  // (x2, x3)
    b[3] = coord ? p23 : 0u;                                     // (x2, x3) or (0, 0)
    return __builtin_bit_cast(bf16x8, b);
}


constexpr int kXcds = 8;   // accelerator complex dies of an MI355X, each with its own L2
// Workgroups of four waves resident at once: 256 CUs x 4 SIMDs x 6 waves / 4.
constexpr int kResidentGroups = 256 * 4 * 6 / 4;
constexpr int kOrderSquare = 8;

// A wave takes a compact 8-wide tile of LL pixels (PW / 8 rows), four waves
// of a workgroup stack vertically; compact tiles keep the wave's observations
// close together, which is what the skipping test below relies on.
constexpr int kWaveTileW = 8;

struct WaveWork {
    int f, split, s0, s1;
    int r0, c0;  // wave tile origin in LL pixels
};

// (p, pe) = r^2 exactly (product and its FMA residual) if sq, else (m, 0).
__device__ __forceinline__ void square_or(float r, float m, bool sq, float &p, float &pe) {
#pragma clang fp contract(off)
    const float rr = r * r;
    p = sq ? rr : m;
    pe = sq ? fmaf(r, r, -rr) : 0.0f;
}

template <int PW>
__device__ __forceinline__ WaveWork wave_work(const PosteriorArgs &a) {
    constexpr int TH = PW / kWaveTileW;
    WaveWork w;
    const int wave = threadIdx.x >> 6;
    const int S = a.split;
    // Workgroups are dealt to the 8 XCDs in turn; renumber them so that each
    // XCD takes a contiguous run of tiles (neighbouring pixels keep
    // overlapping chunks, which then stay in that XCD's L2).  The last
    // gridDim.x % 8 workgroups keep their numbers.  A launch whose
    // workgroups are all resident at once keeps the plain numbering: its
    // time is that of the slowest XCD, and interleaved tiles spread the
    // frame's costly regions over all eight (measured 1.5% faster for one
    // 1080p frame, slower from two frames on).
    int bid = blockIdx.x;
    const int per_xcd = gridDim.x / kXcds;
    if (gridDim.x > kResidentGroups && bid < per_xcd * kXcds) bid = (bid % kXcds) * per_xcd + bid / kXcds;
    w.split = bid % S;
    const int chunk = bid / S;
    const int bcols = (a.wl + kWaveTileW - 1) / kWaveTileW;
    const int brows = (a.hl + 4 * TH - 1) / (4 * TH);
    const int per_frame = bcols * brows;
    w.f = chunk / per_frame;
    const int t = chunk % per_frame;
    // Blocks in squares of kOrderSquare x kOrderSquare (bands of that many
    // block rows, squares left to right, row-major inside a square): the
    // workgroups an XCD runs at once then cover a compact part of the frame.
    const int band = t / (kOrderSquare * bcols), in_band = t % (kOrderSquare * bcols);
    const int R = min(kOrderSquare, brows - band * kOrderSquare);
    const int full = bcols / kOrderSquare;          // full-width squares in the band
    int br, bc;
    if (in_band < full * R * kOrderSquare) {
        const int sq = in_band / (R * kOrderSquare), o = in_band % (R * kOrderSquare);
        br = o / kOrderSquare;
        bc = sq * kOrderSquare + o % kOrderSquare;
    } else {
        const int wl = bcols - full * kOrderSquare, o = in_band - full * R * kOrderSquare;
        br = o / wl;
        bc = full * kOrderSquare + o % wl;
    }
    w.r0 = (band * kOrderSquare + br) * 4 * TH + wave * TH;
    w.c0 = bc * kWaveTileW;
    w.s0 = (int)((long long)a.n_supers * w.split / S);
    w.s1 = (int)((long long)a.n_supers * (w.split + 1) / S);
    return w;
}

// LL index of the wave's i-th pixel (clamped into the image) and whether it exists.
__device__ __forceinline__ bool wave_pixel(const PosteriorArgs &a, const WaveWork &w, int i, long long &p) {
    const int r = w.r0 + i / kWaveTileW, c = w.c0 + i % kWaveTileW;
    const bool valid = r < a.hl && c < a.wl;
    p = (long long)min(r, a.hl - 1) * a.wl + min(c, a.wl - 1);
    return valid;
}

// Scaled double-float observation of LL pixel p, channel k.
__device__ __forceinline__ void load_obs(const float *zf, long long LL, long long p, int k, float sc,
                                         float &h, float &l) {
    const float zh = zf[k * LL + p], zl = zf[(3 + k) * LL + p];
    h = sc * zh;
    l = fmaf(sc, zh, -h) + sc * zl;
}

__device__ __forceinline__ void recentre(const float *T, const float ph[3], const float pl[3], float r[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = (ph[k] - T[k]) + (pl[k] - T[3 + k]);
}

// Upper bound of the logit over an axis-aligned box [lo, hi] (6 floats).
__device__ __forceinline__ float box_bound(const float *box, const float r[3]) {
    const float e0 = fmaxf(fmaxf(box[0] - r[0], r[0] - box[3]), 0.0f);
    const float e1 = fmaxf(fmaxf(box[1] - r[1], r[1] - box[4]), 0.0f);
    const float e2 = fmaxf(fmaxf(box[2] - r[2], r[2] - box[5]), 0.0f);
    return -fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
}

// Upper bound of the logit between two boxes (6 floats each: lo[3], hi[3]).
__device__ __forceinline__ float box_box_bound(const float *box, const float r[6]) {
    const float e0 = fmaxf(fmaxf(box[0] - r[3], r[0] - box[3]), 0.0f);
    const float e1 = fmaxf(fmaxf(box[1] - r[4], r[1] - box[4]), 0.0f);
    const float e2 = fmaxf(fmaxf(box[2] - r[5], r[2] - box[5]), 0.0f);
    return -fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
}

// Chunks a wave evaluates, from v = its logit bound minus the wave's
// reference (one chunk per lane, the lanes of real chunks set in
// lane_mask): every chunk with v > nband, and those with nskip < v <= nband
// unless the wave's remaining budget band_left (wave-uniform) covers all of
// them, which it then shrinks by their count.  With nband == nskip no budget
// is in use.
__device__ __forceinline__ unsigned long long kept_chunks(unsigned long long lane_mask, float v, float nskip,
                                                          float nband, int &band_left) {
    const unsigned long long keep = __builtin_amdgcn_ballot_w64(v > nband) & lane_mask;
    const unsigned long long any = __builtin_amdgcn_ballot_w64(v > nskip) & lane_mask;
    const int nb = __popcll(any & ~keep);
    if (nb <= band_left) {
        band_left -= nb;
        return keep;
    }
    return any;
}

// Widening of the wave's observation box for rounding (scaled units).
constexpr float kBoxSlack = 1.0e-3f;

struct PixelRef {
    float m, ahb, aox;
    float mup;  // wave-level upper bound of every logit of the split
};

// Best probe of super-tile T for observation r (recentred on T): updates the
// running best logit and its anchor node.
__device__ __forceinline__ void probe_supertile(const float *__restrict__ T, const float r[3], float &mlo,
                                                float &ahb, float &aox) {
    const int np = __float_as_int(T[14]);
    for (int i = 0; i < np; ++i) {
        const float *P = T + kSupHdr + i * kProbeFloats;
        const float d0 = r[0] - P[0], d1 = r[1] - P[1], d2 = r[2] - P[2];
        const float tp = -fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        if (tp > mlo) {
            mlo = tp;
            ahb = P[3];
            aox = P[4];
        }
    }
}

// Observation box of the wave (every lane's pixel), for bounds that hold for
// all of its pixels at once; widened by kBoxSlack once here, which covers the
// rounding of high + low parts, of the super-tile centre and of the
// recentring subtractions below.
__device__ __forceinline__ void wave_obs_box(const float ph[3], const float pl[3], float zlo[3], float zhi[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) zlo[k] = zhi[k] = ph[k] + pl[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            zlo[k] = fminf(zlo[k], __shfl_xor(zlo[k], o));
            zhi[k] = fmaxf(zhi[k], __shfl_xor(zhi[k], o));
        }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        zlo[k] -= kBoxSlack;
        zhi[k] += kBoxSlack;
    }
}

// Upper bound of the logit between the wave's (widened) observation box and
// the node box of super-tile si; rbox is the observation box relative to the
// super-tile's centre.
__device__ __forceinline__ float wave_super_bound(const PosteriorArgs &a, int si, const float zlo[3],
                                                  const float zhi[3], float rbox[6]) {
    const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float c = T[k] + T[3 + k];
        rbox[k] = zlo[k] - c;
        rbox[3 + k] = zhi[k] - c;
    }
    return box_box_bound(T + 8, rbox);
}

// Probes i = part, part + LPP, ... of super-tile T for observation r.
template <int LPP>
__device__ __forceinline__ void probe_part(const float *__restrict__ T, const float r[3], int part, float &mlo,
                                           float &ahb, float &aox) {
    const int np = __float_as_int(T[14]);
    for (int i = part; i < np; i += LPP) {
        const float *P = T + kSupHdr + i * kProbeFloats;
        const float d0 = r[0] - P[0], d1 = r[1] - P[1], d2 = r[2] - P[2];
        const float tp = -fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        if (tp > mlo) {
            mlo = tp;
            ahb = P[3];
            aox = P[4];
        }
    }
}

// Per-pixel reference logit and anchor: the best probe over the split's
// super-tiles.  Each pixel is handled by LPP lanes (lane / PW selects the
// part), which split every super-tile's probes between them.  The wave first
// bounds all super-tiles at once (one per lane, against its observation box),
// probes the one with the highest bound, then only super-tiles whose bound
// exceeds the lowest best probe of the wave: the result equals a full probe
// scan (a super-tile bounded below a pixel's best probe cannot improve it).
// The caller refines the reference with far_gap_max when some weight could
// exceed 2^kFarGap relative to it.
template <int PW, int LPP>
__device__ PixelRef pixel_reference(const PosteriorArgs &a, const WaveWork &w, const float ph[3],
                                    const float pl[3], int part, const float zlo[3], const float zhi[3]) {
    const int lane = threadIdx.x & 63;
    float mup = -INFINITY;
    int best = w.s0;
    for (int g = w.s0; g < w.s1; g += 64) {
        const int si = g + lane;
        float rbox[6];
        float bm = si < w.s1 ? wave_super_bound(a, si, zlo, zhi, rbox) : -INFINITY;
        int bi = si;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {  // wave arg-max, lowest index on ties
            const float ob = __shfl_xor(bm, o);
            const int oi = __shfl_xor(bi, o);
            if (ob > bm || (ob == bm && oi < bi)) {
                bm = ob;
                bi = oi;
            }
        }
        if (bm > mup) {
            mup = bm;
            best = bi;
        }
    }
    best = __builtin_amdgcn_readfirstlane(best);
    float mlo = -INFINITY, ahb = 0.0f, aox = 0.0f;
    auto combine = [&]() {  // the LPP lanes of a pixel agree (the lower part wins ties)
#pragma unroll
        for (int o = PW; o < 64; o <<= 1) {
            const float om = __shfl_xor(mlo, o), oh = __shfl_xor(ahb, o), oo = __shfl_xor(aox, o);
            const bool take = (lane & o) == 0 ? (om > mlo) : !(mlo > om);
            if (take) {
                mlo = om;
                ahb = oh;
                aox = oo;
            }
        }
    };
    {
        const float *__restrict__ T = a.supers + (size_t)best * a.super_stride;
        float r[3];
        recentre(T, ph, pl, r);
        probe_part<LPP>(T, r, part, mlo, ahb, aox);
        combine();
    }
    float mwave = mlo;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mwave = fminf(mwave, __shfl_xor(mwave, o));
    for (int g = w.s0; g < w.s1; g += 64) {
        const int sl = g + lane;
        float rbox[6];
        const bool cand = sl < w.s1 && sl != best && !(wave_super_bound(a, sl, zlo, zhi, rbox) <= mwave);
        unsigned long long mask = __ballot(cand);
        while (mask) {
            const int si = g + __builtin_ctzll(mask);
            mask &= mask - 1;
            const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
            float r[3];
            recentre(T, ph, pl, r);
            if (!__any(box_bound(T + 8, r) > mlo)) continue;
            probe_part<LPP>(T, r, part, mlo, ahb, aox);
        }
    }
    combine();
    PixelRef ref{mlo, ahb, aox, mup};
    return ref;
}

// Global reference for split grids: one lane per LL pixel, the best probe
// logit over all super-tiles (the same search as above without the split).
// Each split then skips against max(own reference, global reference), so a
// split far from the pixel's posterior skips against the posterior's peak.
__global__ __launch_bounds__(kBlockThreads) void k_reference(PosteriorArgs a) {
    const long long i = (long long)blockIdx.x * kBlockThreads + threadIdx.x;
    if (i >= (long long)a.n_frames * a.LL) return;
    const long long f = i / a.LL, p = i - f * a.LL;
    const float *zf = a.z + (size_t)f * 6 * a.LL;
    float ph[3], pl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) load_obs(zf, a.LL, p, k, a.scale, ph[k], pl[k]);
    float mlo = -INFINITY, mup = -INFINITY, ahb = 0.0f, aox = 0.0f;
    int best = 0;
    for (int si = 0; si < a.n_supers; ++si) {
        const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
        float r[3];
        recentre(T, ph, pl, r);
        const float ub = box_bound(T + 8, r);
        if (ub > mup) {
            mup = ub;
            best = si;
        }
    }
    {
        const float *__restrict__ T = a.supers + (size_t)best * a.super_stride;
        float r[3];
        recentre(T, ph, pl, r);
        probe_supertile(T, r, mlo, ahb, aox);
    }
    for (int si = 0; si < a.n_supers; ++si) {
        const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
        float r[3];
        recentre(T, ph, pl, r);
        if (si != best && box_bound(T + 8, r) > mlo) probe_supertile(T, r, mlo, ahb, aox);
    }
    a.gref[i] = mlo;
}

// Exact maximum logit over the nodes of the chunks a wave keeps (the same
// super-tile and chunk tests as the main loop), difference form; each pixel's
// LPP lanes split every chunk's nodes.  Returns max(current, that maximum).
template <int PW, int LPP>
__device__ float far_gap_max(const PosteriorArgs &a, const WaveWork &w, const float ph[3], const float pl[3],
                             int part, const float zlo[3], const float zhi[3], float mmin, float cur) {
    const int lane = threadIdx.x & 63;
    const float nskip = -a.skip_log2;
    const float zbox[6] = {zlo[0], zlo[1], zlo[2], zhi[0], zhi[1], zhi[2]};
    float mx = cur;
    for (int g = w.s0; g < w.s1; g += 64) {
        float rbox[6];
        const int sl = g + lane;
        unsigned long long smask = __ballot(sl < w.s1 && wave_super_bound(a, sl, zlo, zhi, rbox) - mmin > nskip);
        while (smask) {
            const int si = g + __builtin_ctzll(smask);
            smask &= smask - 1;
            const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
            float r[3];
            recentre(T, ph, pl, r);
            const float *__restrict__ C0 = T + kSupHdr + kMaxProbes * kProbeFloats;
            for (int cg = 0; cg < a.chunks_per_super; cg += 64) {
                const int ct = min(cg + lane, a.chunks_per_super - 1);
                unsigned long long mask = __ballot(cg + lane < a.chunks_per_super &&
                                                   box_box_bound(C0 + (size_t)ct * kChunkFloats + 96, zbox) - mmin > nskip);
                while (mask) {
                    const float *__restrict__ C = C0 + (size_t)(cg + __builtin_ctzll(mask)) * kChunkFloats;
                    mask &= mask - 1;
                    for (int j = part; j < kChunkNodes; j += LPP) {
                        const float d0 = r[0] - C[j], d1 = r[1] - C[16 + j], d2 = r[2] - C[32 + j];
                        mx = fmaxf(mx, -fmaf(d0, d0, fmaf(d1, d1, d2 * d2)));
                    }
                }
            }
        }
    }
#pragma unroll
    for (int o = PW; o < 64; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    return mx;
}

// Fused recomposition for one split and n <= 2: every lane of pixel row lp
// holds the pixel's complete sums after the lane reduction, so the estimate
// is anchor + S1 / S0 (what the split merge gives for one split, bit for
// bit).  The wave then writes the maps of its tile, (4 x 2^n) x (8 x 2^n)
// pixels in units of V along a row: the unit's estimate is fetched from its
// pixel's lanes (uniform trip count) before any lane branches.
template <int PB, int V>
__device__ __forceinline__ void fused_maps(const PosteriorArgs &a, const WaveWork &w, const float *anc_hb,
                                           const float *anc_ox, const float *R0, const float *R1,
                                           const float *R2, int lane) {
    const int lp = lane & 15, lk = lane >> 4;
    const int n = a.levels, B = 1 << n;
    float ex[PB], ey[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        ex[b] = anc_hb[b] + R1[b] / R0[b];
        ey[b] = anc_ox[b] + R2[b] / R0[b];
        long long p;
        if (lk == 0 && wave_pixel(a, w, b * 16 + lp, p)) a.est[(size_t)w.f * a.LL + p] = make_float2(ex[b], ey[b]);
    }
    const int per_row = (kWaveTileW * B) / V;             // units per tile row
    const int n_units = (16 * PB / kWaveTileW) * B * per_row;
    const int T = (n_units + 63) / 64;                     // same for every lane
    for (int t = 0; t < T; ++t) {
        const int u = lane + 64 * t;
        const bool live = u < n_units;
        const int y = live ? u / per_row : 0, x = live ? (u - y * per_row) * V : 0;
        const int ty = y >> n, tx = x >> n;
        const int i = ty * kWaveTileW + tx;                 // LL pixel of the tile
        float2 e = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const float sx = __shfl(ex[b], i & 15), sy = __shfl(ey[b], i & 15);
            if ((i >> 4) == b) e = make_float2(sx, sy);
        }
        const int gr = w.r0 + ty, gc = w.c0 + tx;
        if (!live || gr >= a.hl || gc >= a.wl) continue;
        const size_t o = ((size_t)w.f * a.H + ((size_t)gr << n) + (y & (B - 1))) * a.W + ((size_t)gc << n) +
                         (x & (B - 1));
        float2 dp[V];
        load_detail<V>(a.det, o, dp);
        write_maps<V>(a.hb, a.hbo2, a.thb, a.so2, a.thb_eps, o, e, dp);
    }
}

// Logit minus the reference, nm - |r - v_j|^2 (nm = -m), with r and node j's
// coordinates v_j = C + LO held as double-floats: the differences, their
// squares and the sum carry their rounding errors, and the result is
// returned as a double-float (high part returned, low part in tl), so the
// weight exp2(t) (1 + tl ln 2) is free of the logit's float32 rounding too
// (a float32 difference form rounds at the scale of |r| and |v_j| instead,
// which coarse grids make large; on grids with very few nodes even the
// rounding of the logit itself, at a scale of tens of units, moves a
// posterior mean between two distant nodes by up to 1e-4 uM).
__device__ __forceinline__ float df_logit_v(const float rh[3], const float rl[3], const float vh[3],
                                            const float vl[3], float nm, float &tl) {
#pragma clang fp contract(off)
    float sh = 0.0f, sl = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float dh, e;
        two_sum(rh[k], -vh[k], dh, e);
        const float dl = e + (rl[k] - vl[k]);
        const float q = dh * dh;
        const float qe = fmaf(2.0f * dh, dl, fmaf(dh, dh, -q));
        float s, es;
        two_sum(sh, q, s, es);
        sh = s;
        sl += es + qe;
    }
    float th, e;
    two_sum(nm, -sh, th, e);
    tl = e - sl;
    return th;
}

__device__ __forceinline__ float df_logit(const float rh[3], const float rl[3], const float *__restrict__ C,
                                          const float *__restrict__ LO, int j, float nm, float &tl) {
    const float vh[3] = {C[j], C[16 + j], C[32 + j]}, vl[3] = {LO[j], LO[16 + j], LO[32 + j]};
    return df_logit_v(rh, rl, vh, vl, nm, tl);
}

// The same pointer, hidden from the optimiser: loads through it are issued
// where they are written instead of being merged with earlier ones.
template <typename P>
__device__ __forceinline__ P *opaque(P *p) {
    asm volatile("" : "+s"(p));
    return p;
}

// The kernel's argument as it lies in the argument segment (address space 4).
using KernArgs = const __attribute__((address_space(4))) PosteriorArgs;

// The fields the far-pixel pass reads, loaded from the argument segment.
__device__ __forceinline__ PosteriorArgs far_args(KernArgs *k) {
    PosteriorArgs f{};
    f.LL = k->LL;
    f.hl = k->hl;
    f.wl = k->wl;
    f.z = k->z;
    f.scale = k->scale;
    f.gref = k->gref;
    f.far_rho2 = k->far_rho2;
    f.skip_log2 = k->skip_log2;
    f.supers = k->supers;
    f.super_stride = k->super_stride;
    f.chunks_per_super = k->chunks_per_super;
    f.lo = k->lo;
    return f;
}

// A lane value the optimiser cannot trace back (it is formed again where used).
__device__ __forceinline__ int opaque_v(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Posterior sums of one pixel over the wave's split with double-float logits
// (as the precise direct kernel forms them), for observations too far from the
// grid's surface for the MFMA kernel's expanded logit.  The whole wave works
// on the pixel: super-tiles one after another, lane l on node l % 16 of
// chunks l / 16, l / 16 + 4, ...  Skipping is the hard rule against the
// pixel's own reference m_skip (no budget band); nm = -m is the logit
// reference of the sums.  Returns the sums S0, S1, S2 about the anchors on
// every lane.
__device__ __forceinline__ void far_pixel_sums(const PosteriorArgs &a, const WaveWork &w, const float qh[3],
                                               const float ql[3], float m_skip, float nm, float anc_hb,
                                               float anc_ox, float S[3]) {
    const int lane = threadIdx.x & 63;
    const int j = lane & 15;
    const float nskip = -a.skip_log2;
    float zbox[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        zbox[k] = (qh[k] + ql[k]) - kBoxSlack;
        zbox[3 + k] = (qh[k] + ql[k]) + kBoxSlack;
    }
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    for (int si = w.s0; si < w.s1; ++si) {
        float rbox[6];
        if (!(wave_super_bound(a, si, zbox, zbox + 3, rbox) - m_skip > nskip)) continue;
        const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
        float rh[3], rl[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float sk, e;
            two_sum(qh[k], -T[k], sk, e);
            fast_two_sum(sk, e + (ql[k] - T[3 + k]), rh[k], rl[k]);
        }
        const float *__restrict__ C0 = T + kSupHdr + kMaxProbes * kProbeFloats;
        const float *__restrict__ LO0 = a.lo + (size_t)si * a.chunks_per_super * kLoFloats;
        float L0 = 0.f, L1 = 0.f, L2 = 0.f;
        for (int ci = lane >> 4; ci < a.chunks_per_super; ci += 4) {
            const float *__restrict__ C = C0 + (size_t)ci * kChunkFloats;
            if (box_box_bound(C + 96, zbox) - m_skip > nskip) {
                float tl;
                const float th = df_logit(rh, rl, C, LO0 + (size_t)ci * kLoFloats, j, nm, tl);
                const float e = __builtin_amdgcn_exp2f(th);
                const float wt = fmaf(e, tl * 0.6931471805599453f, e);
                L0 += wt;
                L1 = fmaf(wt, C[64 + j], L1);
                L2 = fmaf(wt, C[80 + j], L2);
            }
        }
        kahan_add(s0, c0, L0);
        kahan_add(s1, c1, fmaf(T[6] - anc_hb, L0, L1));
        kahan_add(s2, c2, fmaf(T[7] - anc_ox, L0, L2));
    }
    // Sum over the 64 lanes, each pairwise step carrying its rounding error.
    float x[3] = {s0 - c0, s1 - c1, s2 - c2}, e[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int o = 1; o <= 32; o <<= 1)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float y = __shfl_xor(x[k], o), ye = __shfl_xor(e[k], o);
            float t, err;
            two_sum(x[k], y, t, err);
            x[k] = t;
            e[k] = (e[k] + ye) + err;
        }
#pragma unroll
    for (int k = 0; k < 3; ++k) S[k] = x[k] + e[k];
}

// MFMA kernel: a wave takes PB blocks of 16 LL pixels.  Per super-tile,
// 16-node chunk and pixel block one v_mfma_f32_16x16x32_bf16 forms the
// 16 x 16 logits
//   t - m = [v_g, -|v_g|^2, 1] . [2 r, 1, -(|r|^2 + m)]
// (nodes as rows, pixels as columns) from exact three-part bf16 splits of the
// FP32 operands: every product except the smallest (u3 v3), in half the
// cycles of the FP32 16x16x4 MFMA.  The node operand (1 KB per chunk) is
// loaded once for all PB blocks.  Each lane then holds 1 pixel x the 4
// nodes of one chunk row (lane l: pixel l % 16, THb row l / 16, SO2 offsets
// 0..3) and runs the exponentials and the moments on the VALU.
// Two pixel blocks per wave (an 8 x 4 tile) at six waves per SIMD (80 VGPRs;
// spills only inside the far-observation pass) measured fastest on the 1080p
// workload; WAVES = 4 (88 VGPRs, three operand buffers, wave priority by
// predicted work) serves launches small enough to be resident at once.  Both
// evaluate the same chunks in the same order.  DFC: the pixel operand's
// constant |r|^2 + m summed as a double-float (plans near the precision
// budget).
template <int PB, int WAVES, bool DFC>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_posterior(PosteriorArgs a) {
    constexpr int PW = 16 * PB;
    constexpr int LPP = 64 / PW;
    const int lane = threadIdx.x & 63;
    const int lp = lane & 15, lk = lane >> 4;
    const WaveWork w = wave_work<PW>(a);
    // Tiles below the last row of the frame (the workgroup grid rounds the
    // rows up) hold no pixel: nothing to do.
    if (w.r0 >= a.hl) return;
    const float *zf = a.z + (size_t)w.f * 6 * a.LL;
    const float sc = a.scale;

    // Per-pixel pass: lane -> pixel lane % PW of the wave tile.
    const int part = lane / PW;
    float ph[3], pl[3];
    {
        long long p;
        wave_pixel(a, w, lane % PW, p);
#pragma unroll
        for (int k = 0; k < 3; ++k) load_obs(zf, a.LL, p, k, sc, ph[k], pl[k]);
    }
    float zlo[3], zhi[3];
    wave_obs_box(ph, pl, zlo, zhi);
    PixelRef ref = pixel_reference<PW, LPP>(a, w, ph, pl, part, zlo, zhi);

    // Skipping.  A chunk (or super-tile) whose logit upper bound lies more
    // than skip_log2 below every pixel's reference has every weight below
    // 2^-skip_log2 (exactly 0 in float32 at kExactSkipLog2, so then leaving
    // it out changes no bit); chunks between band_log2 and skip_log2 below it
    // are left out while the wave's budget lasts.  The bound is taken between
    // the chunk's box and the box of the wave's observations (min reference
    // over the wave), one chunk per lane.
    const float nskip = -a.skip_log2, nband = -a.band_log2;
    int band_left = a.band_chunks;
    float mmin = ref.m;
    if (a.gref) {
        long long p;
        wave_pixel(a, w, lane % PW, p);
        mmin = fmaxf(mmin, a.gref[(size_t)w.f * a.LL + p]);
    }
    // A pixel without a finite logit (a NaN observation) gets NaN maps
    // whatever is kept; it must not switch skipping off for its wave.
    if (!(mmin > -INFINITY)) mmin = INFINITY;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mmin = fminf(mmin, __shfl_xor(mmin, o));
    // If some weight could exceed 2^kFarGap relative to the best probe, take
    // the exact maximum over the nodes of the chunks that will be kept (the
    // only weights evaluated); a split far from the posterior usually keeps
    // none, and then the reference needs no refinement.
    if (__any(!(ref.mup - ref.m <= kFarGap))) ref.m = far_gap_max<PW, LPP>(a, w, ph, pl, part, zlo, zhi, mmin, ref.m);

    // Pixel operand (the MFMA B operand) of block b: lane (lp, lk) holds
    // coordinate lk of pixel b*16 + lp (lk == 3: the homogeneous 1, and m for
    // the constant term).
    float ah[PB], al[PB], am[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        long long p;
        wave_pixel(a, w, b * 16 + lp, p);
        load_obs(zf, a.LL, p, lk < 3 ? lk : 0, sc, ah[b], al[b]);
        am[b] = __shfl(ref.m, b * 16 + lp);
    }
    // Result layout: lane (lp, lk) holds pixel b*16 + lp and the four nodes
    // of chunk row lk; its sums run over those nodes of every kept chunk.
    // Sums across super-tiles carry Kahan compensation terms K0..K2.
    float anc_hb[PB], anc_ox[PB], R0[PB], R1[PB], R2[PB], K0[PB], K1[PB], K2[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        anc_hb[b] = __shfl(ref.ahb, b * 16 + lp);
        anc_ox[b] = __shfl(ref.aox, b * 16 + lp);
        R0[b] = R1[b] = R2[b] = 0.0f;
        K0[b] = K1[b] = K2[b] = 0.0f;
    }

    const f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
    unsigned executed = 0;   // chunks evaluated by this wave
    // Split operands through a buffer resource: the lane offset stays in a
    // register and the chunk offset is scalar; loads past the table return 0.
    const __amdgpu_buffer_rsrc_t split_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(a.split_ops), (short)0, a.n_supers * a.chunks_per_super * kSplitChunkBytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t super_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(a.supers), (short)0, a.n_supers * a.super_stride * 4, kBufferWord3);
    // A super-tile holds at most 64 chunks (side <= 32): one chunk per lane.
    const int ct = min(lane, a.chunks_per_super - 1);
    const unsigned long long chunk_lanes =
        a.chunks_per_super >= 64 ? ~0ull : (1ull << a.chunks_per_super) - 1;
    const float zbox[6] = {zlo[0], zlo[1], zlo[2], zhi[0], zhi[1], zhi[2]};
    // Super-tiles are tested one per lane; the kept ones are walked in order.
    for (int g = w.s0; g < w.s1; g += 64) {
      float rbox[6];
      const int sl = g + lane;
      unsigned long long smask = __ballot(sl < w.s1 && wave_super_bound(a, sl, zlo, zhi, rbox) - mmin > nskip);
      if constexpr (WAVES < 6) {
        // All waves of such a launch start together and the launch lasts as
        // long as its busiest wave, whose work the count of super-tiles it
        // keeps predicts: busier waves get the SIMD first (scheduling only).
        // Thresholds at 1/3, 3/8 and 5/12 of the split's super-tiles; on
        // 1080p frames with a 256^2 grid waves keeping 5/12 or more average
        // twice the chunks of the median wave.
        if (g == w.s0) {
          const int kept = 24 * __popcll(smask), n = w.s1 - w.s0;
          if (kept >= 10 * n) __builtin_amdgcn_s_setprio(3);
          else if (kept >= 9 * n) __builtin_amdgcn_s_setprio(2);
          else if (kept >= 8 * n) __builtin_amdgcn_s_setprio(1);
        }
      }
      while (smask) {
        const int si = g + __builtin_ctzll(smask);
        smask &= smask - 1;
        const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
        const float *__restrict__ C0 = T + kSupHdr + kMaxProbes * kProbeFloats;
        // chunk tests, one chunk per lane (absolute boxes)
        const unsigned long long mask = kept_chunks(
            chunk_lanes, box_box_bound(C0 + (size_t)ct * kChunkFloats + 96, zbox) - mmin, nskip, nband, band_left);
        if (mask == 0) continue;
        const int kk = lk < 3 ? lk : 0;
        const float ch = T[kk], cl = T[3 + kk];
        bf16x8 av[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const float r = (ah[b] - ch) + (al[b] - cl);
            // |r|^2 + m over the pixel's four lanes (same value on each)
            if constexpr (DFC) {
                // as a double-float (plans near the precision budget)
                float p, pe;
                square_or(r, am[b], lk < 3, p, pe);
#pragma unroll
                for (int o = 16; o <= 32; o <<= 1) {
                    const float q = __shfl_xor(p, o), qe = __shfl_xor(pe, o);
                    float s, e;
                    two_sum(p, q, s, e);
                    p = s;
                    pe = (pe + qe) + e;
                }
                av[b] = split_pixel_operand(2.0f * r, -(p + pe), lk < 3);
            } else {
                float a2 = lk < 3 ? r * r : am[b];
                a2 += __shfl_xor(a2, 16);
                a2 += __shfl_xor(a2, 32);
                av[b] = split_pixel_operand(2.0f * r, -a2, lk < 3);
            }
        }
        float L0[PB], L1[PB], L2[PB];
        const int s_first = si * a.chunks_per_super;   // first chunk of the super-tile in the split table
        // byte offset of the first chunk's row coefficients in the super-tile table
        const int c_first = (si * a.super_stride + kSupHdr + kMaxProbes * kProbeFloats + 104) * 4;
        // Walk the kept chunks with two operand buffers: the next chunk's
        // operands are in flight while the current one is evaluated.  The
        // loads are issued unconditionally (the last chunk is simply loaded
        // again), so the wait counts match on every path and a wait for the
        // current chunk never waits for the next one.
        unsigned long long walk = mask;
        int last = 0;
        auto take = [&](bf16x8 &bv, f32x3 &qm) -> bool {
            const bool got = walk != 0;
            last = got ? __builtin_ctzll(walk | (1ull << 63)) : last;
            walk &= walk - 1;
            bv = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(
                                                split_rsrc, lane * kSplitLaneBytes,
                                                (s_first + last) * kSplitChunkBytes, 0));
            qm = __builtin_bit_cast(f32x3, __builtin_amdgcn_raw_buffer_load_b96(
                                               super_rsrc, lk * 16, c_first + last * (kChunkFloats * 4), 0));
            // keep these loads ahead of the evaluation that follows
            __builtin_amdgcn_sched_barrier(0);
            return got;
        };
        // Weights of the row's four nodes (SO2 offsets s = 0..3): their sum
        // W0 and first moment W1 = sum s w_s give the row's Hb moment
        // through the affine row coefficients, and W0 its THb moment (THb
        // is constant along the row); HbO2 = THb - Hb after the super-tile.
        // The first chunk of the super-tile starts the sums.
        auto eval = [&](const bf16x8 &bv, const f32x3 &qm, auto first) {
            ++executed;
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const f32x4 d = mfma_16x16x32_bf16(bv, av[b], zero4);
                const float w0 = __builtin_amdgcn_exp2f(d[0]), w1 = __builtin_amdgcn_exp2f(d[1]);
                const float w2 = __builtin_amdgcn_exp2f(d[2]), w3 = __builtin_amdgcn_exp2f(d[3]);
                const float W0 = (w0 + w1) + (w2 + w3);
                const float W1 = fmaf(3.0f, w3, fmaf(2.0f, w2, w1));
                if constexpr (decltype(first)::value) {
                    L0[b] = W0;
                    L1[b] = fmaf(qm.x, W0, qm.y * W1);
                    L2[b] = qm.z * W0;
                } else {
                    L0[b] += W0;
                    L1[b] = fmaf(qm.x, W0, fmaf(qm.y, W1, L1[b]));
                    L2[b] = fmaf(qm.z, W0, L2[b]);
                }
            }
        };
        using First = std::true_type;
        using Next = std::false_type;
        // The mask holds at least one chunk: the first take gets it.
        if constexpr (WAVES >= 6) {
            bf16x8 bA, bB;
            f32x3 qA, qB;
            take(bA, qA);
            bool more = take(bB, qB);
            eval(bA, qA, First{});
            while (more) {
                const bool gotA = take(bA, qA);
                eval(bB, qB, Next{});
                if (!gotA) break;
                more = take(bB, qB);
                eval(bA, qA, Next{});
            }
        } else {
            // Fewer resident waves hide less latency: three buffers, two
            // chunks' operands in flight.
            bf16x8 bA, bB, bC;
            f32x3 qA, qB, qC;
            take(bA, qA);
            bool gotB = take(bB, qB);
            bool gotC = take(bC, qC);
            eval(bA, qA, First{});
            while (gotB) {
                const bool gotA = take(bA, qA);
                eval(bB, qB, Next{});
                if (!gotC) break;
                gotB = take(bB, qB);
                eval(bC, qC, Next{});
                if (!gotA) break;
                gotC = take(bC, qC);
                eval(bA, qA, Next{});
            }
        }
        const float chb = T[6], cox = T[7];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            kahan_add(R0[b], K0[b], L0[b]);
            kahan_add(R1[b], K1[b], fmaf(chb - anc_hb[b], L0[b], L1[b]));
            kahan_add(R2[b], K2[b], fmaf(cox - anc_ox[b], L0[b], L2[b] - L1[b]));   // HbO2 = THb - Hb
        }
      }
    }

    // Reduce over the four chunk-row lanes of each pixel with compensated
    // (two-sum) pairwise steps, then lanes with lk == 0 write.
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        R0[b] = lane_sum_rows(R0[b]);
        R1[b] = lane_sum_rows(R1[b]);
        R2[b] = lane_sum_rows(R2[b]);
    }

    // Pixels whose observation lies farther than sqrt(far_rho2) (scaled
    // units) from the grid's nodes: the expanded logit's terms grow with that
    // distance, so their sums are formed again with double-float logits (the
    // plan sets far_rho2 from the precision budget).  The distance is the
    // soft minimum over the split's nodes, rho^2 = -log2 sum_j 2^-|r - v_j|^2
    // = -(m + log2 S0), at most the nearest node's; with a split grid, also
    // that of the best probe of the whole grid (-gref): a split whose nodes
    // all lie far from an observation that lies close to others carries a
    // negligible part of the posterior.
    unsigned far_pixels = 0;
    static_assert(PW <= 64, "one mask bit per pixel of the wave");
    unsigned long long far = 0;
    // Lane indices for what follows, formed here again rather than kept
    // across the main loop.
    const int lane_e = opaque_v((int)threadIdx.x) & 63;
    const int lp_e = lane_e & 15, lk_e = lane_e >> 4;
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        long long p;
        const bool valid = wave_pixel(a, w, b * 16 + lp_e, p);
        const float m = __shfl(ref.m, b * 16 + lp_e);
        far |= (__ballot(lk_e == 0 && valid && m + __log2f(R0[b]) < -a.far_rho2) & 0xffffull) << (16 * b);
    }
    // The pass reads the kernel's arguments again from the argument segment
    // (PosteriorArgs is the kernel's only argument): keeping the values it
    // needs live across the main loop would cost that loop registers.
    KernArgs *ka = (KernArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    while (__builtin_expect(far != 0, 0)) {
        const PosteriorArgs fa = far_args(opaque(ka));
        const int q = __builtin_ctzll(far);   // pixel q of the wave: block q / 16, row lane q % 16
        far &= far - 1;
        const int qb = q >> 4, ql16 = q & 15;
        float xa = anc_hb[0], xo = anc_ox[0];
#pragma unroll
        for (int b = 1; b < PB; ++b)
            if (qb == b) {
                xa = anc_hb[b];
                xo = anc_ox[b];
            }
        long long pq;
        wave_pixel(fa, w, q, pq);
        const float *zq = fa.z + (size_t)w.f * 6 * fa.LL;
        float qh[3], qlo[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) load_obs(zq, fa.LL, pq, k, fa.scale, qh[k], qlo[k]);
        const float mq = __shfl(ref.m, q);
        float m_skip = mq;
        if (fa.gref) {
            const float g = fa.gref[(size_t)w.f * fa.LL + pq];
            if (!(g < -fa.far_rho2)) continue;
            m_skip = fmaxf(m_skip, g);
        }
        ++far_pixels;
        float S[3];
        far_pixel_sums(fa, w, qh, qlo, m_skip, -mq, __shfl(xa, ql16), __shfl(xo, ql16), S);
#pragma unroll
        for (int b = 0; b < PB; ++b)
            if (qb == b && lp_e == ql16) {
                R0[b] = S[0];
                R1[b] = S[1];
                R2[b] = S[2];
            }
    }
    if (a.work && lane == 0) {
        atomicAdd(a.work, (unsigned long long)executed * PW * kChunkNodes);
        if (far_pixels) atomicAdd(a.work + 1, (unsigned long long)far_pixels);
    }
    if (a.fuse) {
        switch (a.vec) {
            case 4: fused_maps<PB, 4>(a, w, anc_hb, anc_ox, R0, R1, R2, lane_e); break;
            case 2: fused_maps<PB, 2>(a, w, anc_hb, anc_ox, R0, R1, R2, lane_e); break;
            default: fused_maps<PB, 1>(a, w, anc_hb, anc_ox, R0, R1, R2, lane_e); break;
        }
        return;
    }
    float *out = a.part + ((size_t)w.f * a.split + w.split) * kPartFields * a.LL;
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        const int src = b * 16 + lp_e;
        const float m = __shfl(ref.m, src);
        long long p;
        const bool valid = wave_pixel(a, w, src, p);
        if (lk_e == 0 && valid) {
            out[p] = m;
            out[a.LL + p] = R0[b];
            out[2 * a.LL + p] = R1[b];
            out[3 * a.LL + p] = R2[b];
            out[4 * a.LL + p] = anc_hb[b];
            out[5 * a.LL + p] = anc_ox[b];
        }
    }
}


// Direct kernel: one LL pixel per lane, logits in the difference form
// t - m = -(r - v_g)^2 - m on the VALU with wave-uniform (scalar) node loads;
// PRECISE: from double-float differences (df_logit), for grids whose nodes
// are too far apart for float32 logits.  Skipping, the global reference, the
// exact maximum over kept chunks and (float32 logits) the double-float pass
// for far observations are as in the MFMA kernel.
template <bool PRECISE>
__global__ __launch_bounds__(kBlockThreads) void k_posterior_direct(PosteriorArgs a) {
    constexpr int PW = 64;
    const int lane = threadIdx.x & 63;
    const WaveWork w = wave_work<PW>(a);
    if (w.r0 >= a.hl) return;   // a tile below the frame's last row holds no pixel
    const float *zf = a.z + (size_t)w.f * 6 * a.LL;
    long long p;
    const bool valid = wave_pixel(a, w, lane, p);
    float ph[3], pl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) load_obs(zf, a.LL, p, k, a.scale, ph[k], pl[k]);
    float zlo[3], zhi[3];
    wave_obs_box(ph, pl, zlo, zhi);
    PixelRef ref = pixel_reference<PW, 1>(a, w, ph, pl, 0, zlo, zhi);
    const float nskip = -a.skip_log2, nband = -a.band_log2;
    int band_left = a.band_chunks;
    float mmin = ref.m;
    if (a.gref) mmin = fmaxf(mmin, a.gref[(size_t)w.f * a.LL + p]);
    if (!(mmin > -INFINITY)) mmin = INFINITY;  // NaN observation: see the MFMA kernel
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mmin = fminf(mmin, __shfl_xor(mmin, o));
    if (__any(!(ref.mup - ref.m <= kFarGap))) ref.m = far_gap_max<PW, 1>(a, w, ph, pl, 0, zlo, zhi, mmin, ref.m);
    const float nm = -ref.m;
    const float zbox[6] = {zlo[0], zlo[1], zlo[2], zhi[0], zhi[1], zhi[2]};
    float R0 = 0.f, R1 = 0.f, R2 = 0.f, K0 = 0.f, K1 = 0.f, K2 = 0.f;
    unsigned executed = 0;
    for (int g = w.s0; g < w.s1; g += 64) {
        float rbox[6];
        const int sl = g + lane;
        unsigned long long smask = __ballot(sl < w.s1 && wave_super_bound(a, sl, zlo, zhi, rbox) - mmin > nskip);
        while (smask) {
            const int si = g + __builtin_ctzll(smask);
            smask &= smask - 1;
            const float *__restrict__ T = a.supers + (size_t)si * a.super_stride;
            float r[3], rh[3], rl[3];
            if (PRECISE) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float sk, e;
                    two_sum(ph[k], -T[k], sk, e);
                    fast_two_sum(sk, e + (pl[k] - T[3 + k]), rh[k], rl[k]);
                }
            } else {
                recentre(T, ph, pl, r);
            }
            float L0 = 0.f, L1 = 0.f, L2 = 0.f;
            const float *__restrict__ C0 = T + kSupHdr + kMaxProbes * kProbeFloats;
            for (int cg = 0; cg < a.chunks_per_super; cg += 64) {
                const int ct = min(cg + lane, a.chunks_per_super - 1);
                const int nc = a.chunks_per_super - cg;
                unsigned long long mask =
                    kept_chunks(nc >= 64 ? ~0ull : (1ull << nc) - 1,
                                box_box_bound(C0 + (size_t)ct * kChunkFloats + 96, zbox) - mmin, nskip, nband, band_left);
                while (mask) {
                    const int ci = cg + __builtin_ctzll(mask);
                    const float *__restrict__ C = C0 + (size_t)ci * kChunkFloats;
                    const float *__restrict__ LO = PRECISE ? a.lo + ((size_t)si * a.chunks_per_super + ci) * kLoFloats
                                                           : nullptr;
                    mask &= mask - 1;
                    ++executed;
#pragma unroll
                    for (int j = 0; j < kChunkNodes; ++j) {
                        float wt;
                        if (PRECISE) {
                            float tl;
                            const float th = df_logit(rh, rl, C, LO, j, nm, tl);
                            const float w = __builtin_amdgcn_exp2f(th);
                            wt = fmaf(w, tl * 0.6931471805599453f, w);
                        } else {
                            const float d0 = r[0] - C[j], d1 = r[1] - C[16 + j], d2 = r[2] - C[32 + j];
                            float t = fmaf(-d0, d0, nm);
                            t = fmaf(-d1, d1, t);
                            t = fmaf(-d2, d2, t);
                            wt = __builtin_amdgcn_exp2f(t);
                        }
                        L0 += wt;
                        L1 = fmaf(wt, C[64 + j], L1);
                        L2 = fmaf(wt, C[80 + j], L2);
                    }
                }
            }
            kahan_add(R0, K0, L0);
            kahan_add(R1, K1, fmaf(T[6] - ref.ahb, L0, L1));
            kahan_add(R2, K2, fmaf(T[7] - ref.aox, L0, L2));
        }
    }
    if (a.work && lane == 0) atomicAdd(a.work, (unsigned long long)executed * PW * kChunkNodes);
    if constexpr (!PRECISE) {
        // Pixels whose observation lies far from the grid's nodes: the float32
        // differences round at the scale of that distance, so their sums are
        // formed again with double-float logits, as in the MFMA kernel (the
        // plan sets far_rho2 from this kernel's precision budget).
        unsigned long long far = __ballot(valid && ref.m + __log2f(R0) < -a.far_rho2);
        unsigned far_pixels = 0;
        while (__builtin_expect(far != 0, 0)) {
            const int q = __builtin_ctzll(far);   // the pixel of lane q
            far &= far - 1;
            float qh[3], ql[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                qh[k] = __shfl(ph[k], q);
                ql[k] = __shfl(pl[k], q);
            }
            const float mq = __shfl(ref.m, q);
            float m_skip = mq;
            if (a.gref) {
                long long pq;
                wave_pixel(a, w, q, pq);
                const float g = a.gref[(size_t)w.f * a.LL + pq];
                if (!(g < -a.far_rho2)) continue;
                m_skip = fmaxf(m_skip, g);
            }
            ++far_pixels;
            float S[3];
            far_pixel_sums(a, w, qh, ql, m_skip, -mq, __shfl(ref.ahb, q), __shfl(ref.aox, q), S);
            if (lane == q) {
                R0 = S[0];
                R1 = S[1];
                R2 = S[2];
            }
        }
        if (a.work && lane == 0 && far_pixels) atomicAdd(a.work + 1, (unsigned long long)far_pixels);
    }
    if (valid) {
        float *out = a.part + ((size_t)w.f * a.split + w.split) * kPartFields * a.LL;
        out[p] = ref.m;
        out[a.LL + p] = R0;
        out[2 * a.LL + p] = R1;
        out[3 * a.LL + p] = R2;
        out[4 * a.LL + p] = ref.ahb;
        out[5 * a.LL + p] = ref.aox;
    }
}

// ---------------------------------------------------------------------------
// K3: merge the grid splits per LL pixel, inverse Haar of the Tikhonov
// details with the low-pass estimate added once at the end (the inverse of a
// low-pass-only block is that constant on every pixel), and the output maps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 lowpass_estimate(const RecomposeArgs &a, int f, long long q) {
    if (a.lowpass == HB_LOWPASS_TIKHONOV) {
        // offset + M z with M, the offset and z as double-floats: the terms
        // are about |M| |z| (~1e3 uM) while the estimate is tens of uM.
        const long long LL = a.d.LL;
        const float *zf = a.z + (size_t)f * 6 * LL;
        const float *M = a.M;
        float hh = M[6], hl = M[14], oh = M[7], ol = M[15];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float zh = zf[k * LL + q], zl = zf[(3 + k) * LL + q];
            df_mul_add(hh, hl, M[k], M[8 + k], zh, zl);
            df_mul_add(oh, ol, M[3 + k], M[11 + k], zh, zl);
        }
        return make_float2(hh + hl, oh + ol);
    }
    const long long LL = a.d.LL;
    const float *P = a.part + (size_t)f * a.split * kPartFields * LL + q;
    float m = -INFINITY;
    for (int i = 0; i < a.split; ++i) m = fmaxf(m, P[(size_t)i * kPartFields * LL]);
    const float a_hb = P[4 * LL], a_ox = P[5 * LL];
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    for (int i = 0; i < a.split; ++i) {
        const float *Pi = P + (size_t)i * kPartFields * LL;
        const float fct = exp2f(Pi[0] - m);
        const float S0 = Pi[LL];
        kahan_add(s0, c0, S0 * fct);
        kahan_add(s1, c1, fmaf(Pi[4 * LL] - a_hb, S0, Pi[2 * LL]) * fct);
        kahan_add(s2, c2, fmaf(Pi[5 * LL] - a_ox, S0, Pi[3 * LL]) * fct);
    }
    return make_float2(a_hb + s1 / s0, a_ox + s2 / s0);
}

// K3: one thread per (frame, block, block row): the block's low-pass
// estimate (split merge, or the Tikhonov low-pass), plus the row's detail
// part, to the four maps, V pixels per vector access.
template <int V>
__global__ __launch_bounds__(kBlockThreads) void k_recompose(RecomposeArgs a) {
    const Dims &d = a.d;
    const int n = d.levels, B = 1 << n;
    const long long idx = (long long)blockIdx.x * kBlockThreads + threadIdx.x;
    if (idx >= (long long)a.n_frames * d.LL * B) return;
    const long long blk = idx >> n;
    const int r = (int)(idx & (B - 1));
    const int f = (int)(blk / d.LL);
    const long long q = blk - (long long)f * d.LL;
    const int br = (int)(q / d.wl), bc = (int)(q - (long long)br * d.wl);
    const float2 e = lowpass_estimate(a, f, q);
    if (r == 0) a.est[(size_t)f * d.LL + q] = e;
    const size_t row = ((size_t)f * d.H + ((size_t)br << n) + r) * d.W + ((size_t)bc << n);
    for (int c = 0; c < B; c += V) {
        float2 dp[V];
        load_detail<V>(a.det, row + c, dp);
        write_maps<V>(a.hb, a.hbo2, a.thb, a.so2, a.thb_eps, row + c, e, dp);
    }
}

}  // namespace

hipError_t launch_tikhonov_fp64(const double *d_in, double *d_out, float *d_mf, hipStream_t s) {
    hipLaunchKernelGGL(k_tikhonov_fp64, dim3(1), dim3(64), 0, s, d_in, d_out, d_mf);
    return hipGetLastError();
}

namespace {

template <typename T, int N>
void launch_reg(const void *frames, const HaarArgs &b, long long blocks, hipStream_t s) {
    if (b.df)
        hipLaunchKernelGGL((k_log_haar_reg<T, N, true>), dim3((unsigned)blocks), dim3(kBlockThreads), 0, s,
                           (const T *)frames, b);
    else
        hipLaunchKernelGGL((k_log_haar_reg<T, N, false>), dim3((unsigned)blocks), dim3(kBlockThreads), 0, s,
                           (const T *)frames, b);
}

template <typename T>
void launch_k1(const void *frames, const HaarArgs &b, hipStream_t s) {
    const int n = b.d.levels;
    const bool aligned = ((uintptr_t)frames % ((size_t)(1 << n) * sizeof(T))) == 0;
    HaarArgs c = b;
    c.vec4 = ((uintptr_t)frames % (4 * sizeof(T))) == 0;
    if (n <= 2 && aligned) {
        const long long blocks = ((long long)b.n_frames * b.d.LL + kBlockThreads - 1) / kBlockThreads;
        if (n == 0) launch_reg<T, 0>(frames, b, blocks, s);
        else if (n == 1) launch_reg<T, 1>(frames, b, blocks, s);
        else launch_reg<T, 2>(frames, b, blocks, s);
    } else {
        const long long grid = (long long)b.n_frames * b.d.hl * b.d.strips_per_row;
        // Up to two levels the strip kernel keeps the register kernel's bits.
        if (n >= 3 || b.df)
            hipLaunchKernelGGL((k_log_haar<T, true>), dim3((unsigned)grid), dim3(kBlockThreads), 0, s,
                               (const T *)frames, c);
        else
            hipLaunchKernelGGL((k_log_haar<T, false>), dim3((unsigned)grid), dim3(kBlockThreads), 0, s,
                               (const T *)frames, c);
    }
}

}  // namespace

hipError_t launch_log_haar(const void *frames, int n_frames, const HaarArgs &a, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    HaarArgs b = a;
    b.n_frames = n_frames;
    switch (a.dtype) {
        case HB_F32: launch_k1<float>(frames, b, s); break;
        case HB_F16: launch_k1<__half>(frames, b, s); break;
        default: launch_k1<uint16_t>(frames, b, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_reference(const PosteriorArgs &a, hipStream_t s) {
    const long long n = (long long)a.n_frames * a.LL;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reference, dim3((unsigned)((n + kBlockThreads - 1) / kBlockThreads)), dim3(kBlockThreads),
                       0, s, a);
    return hipGetLastError();
}

hipError_t launch_posterior(const PosteriorArgs &a, bool mfma, hipStream_t s) {
    const int th = (mfma ? 16 * kPixelBlocks : 64) / kWaveTileW;
    const long long per_frame = (long long)((a.wl + kWaveTileW - 1) / kWaveTileW) * ((a.hl + 4 * th - 1) / (4 * th));
    const long long grid = per_frame * a.n_frames * a.split;
    if (grid <= 0) return hipSuccess;
    // A launch whose workgroups are all resident at once runs about four
    // waves per SIMD: the variant built for four keeps more loads in flight
    // (same arithmetic, same bits).
    const dim3 g((unsigned)grid), blk(kBlockThreads);
    if (mfma && grid <= kResidentGroups && a.dfc)
        hipLaunchKernelGGL((k_posterior<kPixelBlocks, 4, true>), g, blk, 0, s, a);
    else if (mfma && grid <= kResidentGroups)
        hipLaunchKernelGGL((k_posterior<kPixelBlocks, 4, false>), g, blk, 0, s, a);
    else if (mfma && a.dfc)
        hipLaunchKernelGGL((k_posterior<kPixelBlocks, 6, true>), g, blk, 0, s, a);
    else if (mfma)
        hipLaunchKernelGGL((k_posterior<kPixelBlocks, 6, false>), g, blk, 0, s, a);
    else if (a.precise)
        hipLaunchKernelGGL(k_posterior_direct<true>, dim3((unsigned)grid), dim3(kBlockThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_posterior_direct<false>, dim3((unsigned)grid), dim3(kBlockThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_recompose(int n_frames, const RecomposeArgs &a, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    RecomposeArgs b = a;
    b.n_frames = n_frames;
    const int B = 1 << a.d.levels;
    const long long blocks = ((long long)n_frames * a.d.LL * B + kBlockThreads - 1) / kBlockThreads;
    // widest vector the block width and every map pointer allow
    auto fits = [&](int v) {
        if (B % v) return false;
        for (const float *m : {a.hb, a.hbo2, a.thb, a.so2})
            if (m && ((uintptr_t)m % (sizeof(float) * v)) != 0) return false;
        return true;
    };
    if (fits(4))
        hipLaunchKernelGGL(k_recompose<4>, dim3((unsigned)blocks), dim3(kBlockThreads), 0, s, b);
    else if (fits(2))
        hipLaunchKernelGGL(k_recompose<2>, dim3((unsigned)blocks), dim3(kBlockThreads), 0, s, b);
    else
        hipLaunchKernelGGL(k_recompose<1>, dim3((unsigned)blocks), dim3(kBlockThreads), 0, s, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static scratch of hb_estimate_frames_noalloc: the per-call buffers
// (low-pass observation, detail part, posterior partials, global reference,
// low-pass estimate) are carved out of this array instead of the plan's own
// allocations.  Each device holds its own copy for the life of the process.
// Host code never passes the array's name to a kernel (on the host it is only
// a registration handle): static_scratch() looks up the device address once
// per device, with that device current, and every launch uses that address.
// ---------------------------------------------------------------------------
namespace {
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t static_scratch(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace hb
