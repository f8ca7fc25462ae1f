// HIP kernels of the haemoglobin-estimation path for gfx950 (MI355X).
//
//   K0  k_tikhonov_fp64  plan time, FP64: E, (E'E + gamma I)^-1 E'      (Method, Eq. 5)
//   K1  k_log_haar       log-attenuation, n-level 2D Haar, Tikhonov on the
//                        directional coefficients; LDS-staged strips (Eq. 1-2, 5)
//   K2  k_posterior      posterior mean over the THb x SO2 grid on the low-pass band
//   K3  k_recompose      split merge, inverse Haar, THb/SO2 maps           (Eq. 4, Fig. 1)
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hb_df.h"
#include "hb_internal.h"

namespace hb {

namespace {

// ---------------------------------------------------------------------------
// K0: Jacobian of the forward model at the reference point and the Tikhonov
// operator, in double precision.  in = [n, L, ref_hb, ref_hbo2, lambda,
// eps_hb[n], eps_hbo2[n], response[3][n] (rows normalised to unit sum)];
// out = [E(6), M(6), gamma, ok].
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
    }
    for (int i = 0; i < 6; ++i) out[i] = E[i];
    out[12] = gamma;
    out[13] = ok ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Storage-type loads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float load_px(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float load_px(const __half *p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ float load_px(const uint16_t *p, size_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);  // bfloat16 -> float32 is exact
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

// ---------------------------------------------------------------------------
// K1: one workgroup per strip of 2^n pixel rows x (bps * 2^n) columns.
//
// Numerics: each block's log-attenuation is carried relative to the block's
// mean intensity R, u(q) = -ln(I(q)/R) = -log1p((I(q) - R)/R), so directional
// coefficients are computed from small, accurately rounded numbers.  Details of
// u equal those of y = -ln I (they differ by a per-block constant); the block
// mean of y is recovered as -ln(R/I_ref) + mean(u) relative to the plan's
// reference intensity I_ref.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlockThreads) void k_log_haar(const T *__restrict__ frames, HaarArgs a) {
    __shared__ float s_i[3][kStripPixels];
    __shared__ float s_u[3][kStripPixels];
    __shared__ float s_r[3][kStripPixels / 4];
    const Dims &d = a.d;
    const StripPos s = strip_pos(d);
    const int n = d.levels, B = s.B, Wt = s.Wt, ncols = s.ncols;
    const int tid = threadIdx.x;

    // 1. Coalesced load of the strip (rows are contiguous HWC runs), clamp.
    const size_t frame_off = (size_t)s.f * d.H * d.W * 3;
    const int run = ncols * 3;
    for (int i = tid; i < B * run; i += kBlockThreads) {
        const int r = i / run, rem = i - r * run, c = rem / 3, k = rem - 3 * c;
        float v = load_px(frames, frame_off + ((size_t)(s.row0 + r) * d.W + s.col0) * 3 + rem);
        v = (v < a.floor) ? a.floor : v;  // NaN stays NaN
        s_i[k][r * Wt + c] = v;
        s_u[k][r * Wt + c] = v;
    }
    __syncthreads();

    // 2. Block sums of intensity by a 2x2 cascade, then the block mean R.
    for (int l = 1; l <= n; ++l) {
        const int h = 1 << (l - 1), g2 = 2 * h, gr = B / g2, gc = ncols / g2;
        for (int i = tid; i < gr * gc * 3; i += kBlockThreads) {
            const int k = i % 3, q = i / 3, r = (q / gc) * g2, c = (q % gc) * g2;
            float *u = s_u[k];
            u[r * Wt + c] = (u[r * Wt + c] + u[r * Wt + c + h]) + (u[(r + h) * Wt + c] + u[(r + h) * Wt + c + h]);
        }
        __syncthreads();
    }
    if (n > 0) {
        const float inv = 1.0f / (float)(1 << (2 * n));
        for (int i = tid; i < s.nb * 3; i += kBlockThreads) {
            const int k = i % 3, j = i / 3;
            s_r[k][j] = s_u[k][j << n] * inv;
        }
    }
    __syncthreads();

    // 3. Log-ratio to the block reference.
    for (int i = tid; i < B * ncols * 3; i += kBlockThreads) {
        const int k = i % 3, q = i / 3, r = q / ncols, c = q - r * ncols;
        const float I = s_i[k][r * Wt + c];
        const float R = (n > 0) ? s_r[k][c >> n] : I;
        s_u[k][r * Wt + c] = -log1pf((I - R) / R);
    }
    __syncthreads();

    // 4. n-level Haar in place.  Window (a, b, c, d) = (r,c), (r,c+h), (r+h,c),
    //    (r+h,c+h); coefficients = window * H (Eq. 1-2): LL -> (r,c),
    //    row difference -> (r+h,c), diagonal -> (r+h,c+h), column difference -> (r,c+h).
    for (int l = 1; l <= n; ++l) {
        const int h = 1 << (l - 1), g2 = 2 * h, gr = B / g2, gc = ncols / g2;
        for (int i = tid; i < gr * gc * 3; i += kBlockThreads) {
            const int k = i % 3, q = i / 3, r = (q / gc) * g2, c = (q % gc) * g2;
            float *u = s_u[k];
            const float w0 = u[r * Wt + c], w1 = u[r * Wt + c + h];
            const float w2 = u[(r + h) * Wt + c], w3 = u[(r + h) * Wt + c + h];
            u[r * Wt + c] = 0.5f * ((w0 + w1) + (w2 + w3));
            u[(r + h) * Wt + c] = 0.5f * ((w0 + w1) - (w2 + w3));
            u[(r + h) * Wt + c + h] = 0.5f * ((w0 - w1) - (w2 - w3));
            u[r * Wt + c + h] = 0.5f * ((w0 - w1) + (w2 - w3));
        }
        __syncthreads();
    }

    // 5. Centred low-pass observation z = ybar - mu_ref per block, as a
    //    double-float: ybar - mu_ref = ln(I_ref / R) + mean(u).
    const float invB = 1.0f / (float)B;
    for (int i = tid; i < s.nb * 3; i += kBlockThreads) {
        const int k = i % 3, j = i / 3;
        const float R = (n > 0) ? s_r[k][j] : s_i[k][j];
        float zh, zl;
        ln_ratio_df(a.iref[k], R, zh, zl);
        df_add(zh, zl, s_u[k][j << n] * invB);
        const size_t q = (size_t)s.br * d.wl + s.blk0 + j;
        a.z[((size_t)s.f * 6 + k) * d.LL + q] = zh;
        a.z[((size_t)s.f * 6 + 3 + k) * d.LL + q] = zl;
    }

    // 6. Tikhonov on every directional coefficient: (Hb, HbO2) = M * (R, G, B).
    const float m0 = a.M[0], m1 = a.M[1], m2 = a.M[2], m3 = a.M[3], m4 = a.M[4], m5 = a.M[5];
    for (int i = tid; i < B * ncols; i += kBlockThreads) {
        const int r = i / ncols, c = i - r * ncols;
        float2 o = make_float2(0.0f, 0.0f);
        if (((r | c) & (B - 1)) != 0) {
            const float d0 = s_u[0][r * Wt + c], d1 = s_u[1][r * Wt + c], d2 = s_u[2][r * Wt + c];
            o.x = fmaf(m0, d0, fmaf(m1, d1, m2 * d2));
            o.y = fmaf(m3, d0, fmaf(m4, d1, m5 * d2));
        }
        a.det[((size_t)s.f * d.H + s.row0 + r) * d.W + s.col0 + c] = o;
    }
}

// ---------------------------------------------------------------------------
// K2: posterior mean over the grid for PIX LL pixels per lane.
//
// Likelihood in base 2 with scaled coordinates: t_g = -|s z - s mu'_g|^2,
// s = sqrt(log2(e) / (2 sigma^2)), mu' centred on mu_ref.  The observation
// arrives as a double-float; per tile it is re-centred on the tile's centre
// (double-float subtraction), so the per-node differences are formed from
// small numbers and keep their precision.  Node data are wave-uniform and come
// through scalar loads.  The weights are taken relative to a per-pixel
// reference m_ref that never changes inside the loop:
//   m_lo = best logit over one probe node per tile (a true logit, so the top
//          weight is >= 1: no underflow of the whole sum);
//   m_up = best upper bound over the tiles' boxes (>= every logit).
// If m_up - m_lo <= kFarGap for every lane of the wave, m_ref = m_lo and all
// weights lie in [0, 2^kFarGap]; otherwise the wave first takes the exact
// maximum over its nodes.  Moments are centred on the tile centre inside a
// tile and on the best probe node (the anchor) across tiles; tile sums are
// merged with Kahan compensation.
// ---------------------------------------------------------------------------
constexpr float kFarGap = 64.0f;

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

template <int PIX>
__global__ __launch_bounds__(kBlockThreads) void k_posterior(PosteriorArgs a) {
    const int S = a.split;
    const int split = blockIdx.x % S;
    const int chunk = blockIdx.x / S;
    const long long per_block = (long long)kBlockThreads * PIX;
    const int chunks_per_frame = (int)((a.LL + per_block - 1) / per_block);
    const int f = chunk / chunks_per_frame;
    const long long base = (long long)(chunk % chunks_per_frame) * per_block + threadIdx.x;
    const int t0 = (int)((long long)a.n_tiles * split / S);
    const int t1 = (int)((long long)a.n_tiles * (split + 1) / S);

    // Scaled observation s * z as a double-float per channel.
    float zh[3][PIX], zl[3][PIX];
    const float *zf = a.z + (size_t)f * 6 * a.LL;
#pragma unroll
    for (int j = 0; j < PIX; ++j) {
        long long p = base + (long long)j * kBlockThreads;
        p = p < a.LL ? p : a.LL - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float h = zf[k * a.LL + p], l = zf[(3 + k) * a.LL + p];
            const float ph = a.scale * h;
            zh[k][j] = ph;
            zl[k][j] = fmaf(a.scale, h, -ph) + a.scale * l;
        }
    }

    // Probe pass: m_lo, anchor, m_up.
    float mlo[PIX], mup[PIX], ahb[PIX], aox[PIX];
#pragma unroll
    for (int j = 0; j < PIX; ++j) {
        mlo[j] = -INFINITY;
        mup[j] = -INFINITY;
        ahb[j] = 0.0f;
        aox[j] = 0.0f;
    }
    for (int t = t0; t < t1; ++t) {
        const float *__restrict__ T = a.tiles + (size_t)t * kTileFloats;
        const float *__restrict__ N = T + kTileHdr;
        const int ps = __float_as_int(T[8]);
        const float p0 = N[ps], p1 = N[kTileNodes + ps], p2 = N[2 * kTileNodes + ps];
        const float phb = T[0] + N[3 * kTileNodes + ps];
        const float pox = T[1] + N[4 * kTileNodes + ps];
#pragma unroll
        for (int j = 0; j < PIX; ++j) {
            const float r0 = (zh[0][j] - T[9]) + (zl[0][j] - T[12]);
            const float r1 = (zh[1][j] - T[10]) + (zl[1][j] - T[13]);
            const float r2 = (zh[2][j] - T[11]) + (zl[2][j] - T[14]);
            const float d0 = r0 - p0, d1 = r1 - p1, d2 = r2 - p2;
            const float tp = -fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
            if (tp > mlo[j]) {
                mlo[j] = tp;
                ahb[j] = phb;
                aox[j] = pox;
            }
            const float e0 = fmaxf(fmaxf(T[2] - r0, r0 - T[5]), 0.0f);
            const float e1 = fmaxf(fmaxf(T[3] - r1, r1 - T[6]), 0.0f);
            const float e2 = fmaxf(fmaxf(T[4] - r2, r2 - T[7]), 0.0f);
            mup[j] = fmaxf(mup[j], -fmaf(e0, e0, fmaf(e1, e1, e2 * e2)));
        }
    }
    bool far = false;
#pragma unroll
    for (int j = 0; j < PIX; ++j) far |= !(mup[j] - mlo[j] <= kFarGap);
    float nref[PIX];
#pragma unroll
    for (int j = 0; j < PIX; ++j) nref[j] = -mlo[j];
    if (__any(far)) {
        // Exact maximum over this split's nodes.
        float mx[PIX];
#pragma unroll
        for (int j = 0; j < PIX; ++j) mx[j] = mlo[j];
        for (int t = t0; t < t1; ++t) {
            const float *__restrict__ T = a.tiles + (size_t)t * kTileFloats;
            const float *__restrict__ N = T + kTileHdr;
            float r0[PIX], r1[PIX], r2[PIX];
#pragma unroll
            for (int j = 0; j < PIX; ++j) {
                r0[j] = (zh[0][j] - T[9]) + (zl[0][j] - T[12]);
                r1[j] = (zh[1][j] - T[10]) + (zl[1][j] - T[13]);
                r2[j] = (zh[2][j] - T[11]) + (zl[2][j] - T[14]);
            }
            for (int i = 0; i < kTileNodes; ++i) {
                const float n0 = N[i], n1 = N[kTileNodes + i], n2 = N[2 * kTileNodes + i];
#pragma unroll
                for (int j = 0; j < PIX; ++j) {
                    const float d0 = r0[j] - n0, d1 = r1[j] - n1, d2 = r2[j] - n2;
                    mx[j] = fmaxf(mx[j], -fmaf(d0, d0, fmaf(d1, d1, d2 * d2)));
                }
            }
        }
#pragma unroll
        for (int j = 0; j < PIX; ++j) nref[j] = -mx[j];
    }

    // Main pass.
    float s0[PIX], s1[PIX], s2[PIX], c0[PIX], c1[PIX], c2[PIX];
#pragma unroll
    for (int j = 0; j < PIX; ++j) s0[j] = s1[j] = s2[j] = c0[j] = c1[j] = c2[j] = 0.0f;
    for (int t = t0; t < t1; ++t) {
        const float *__restrict__ T = a.tiles + (size_t)t * kTileFloats;
        const float *__restrict__ N = T + kTileHdr;
        float r0[PIX], r1[PIX], r2[PIX];
        float t0s[PIX], t1s[PIX], t2s[PIX];
#pragma unroll
        for (int j = 0; j < PIX; ++j) {
            r0[j] = (zh[0][j] - T[9]) + (zl[0][j] - T[12]);
            r1[j] = (zh[1][j] - T[10]) + (zl[1][j] - T[13]);
            r2[j] = (zh[2][j] - T[11]) + (zl[2][j] - T[14]);
            t0s[j] = t1s[j] = t2s[j] = 0.0f;
        }
#pragma unroll 16
        for (int i = 0; i < kTileNodes; ++i) {
            const float n0 = N[i], n1 = N[kTileNodes + i], n2 = N[2 * kTileNodes + i];
            const float dh = N[3 * kTileNodes + i], dx = N[4 * kTileNodes + i];
#pragma unroll
            for (int j = 0; j < PIX; ++j) {
                const float d0 = r0[j] - n0, d1 = r1[j] - n1, d2 = r2[j] - n2;
                float tt = fmaf(-d0, d0, nref[j]);
                tt = fmaf(-d1, d1, tt);
                tt = fmaf(-d2, d2, tt);
                const float w = __builtin_amdgcn_exp2f(tt);
                t0s[j] += w;
                t1s[j] = fmaf(w, dh, t1s[j]);
                t2s[j] = fmaf(w, dx, t2s[j]);
            }
        }
        const float chb = T[0], cox = T[1];
#pragma unroll
        for (int j = 0; j < PIX; ++j) {
            kahan_add(s0[j], c0[j], t0s[j]);
            kahan_add(s1[j], c1[j], fmaf(chb - ahb[j], t0s[j], t1s[j]));
            kahan_add(s2[j], c2[j], fmaf(cox - aox[j], t0s[j], t2s[j]));
        }
    }

    float *out = a.part + ((size_t)f * S + split) * kPartFields * a.LL;
#pragma unroll
    for (int j = 0; j < PIX; ++j) {
        const long long p = base + (long long)j * kBlockThreads;
        if (p < a.LL) {
            out[p] = -nref[j];
            out[a.LL + p] = s0[j];
            out[2 * a.LL + p] = s1[j];
            out[3 * a.LL + p] = s2[j];
            out[4 * a.LL + p] = ahb[j];
            out[5 * a.LL + p] = aox[j];
        }
    }
}

// ---------------------------------------------------------------------------
// K3: merge the grid splits per LL pixel, inverse Haar of the Tikhonov
// details with the low-pass estimate added once at the end (the inverse of a
// low-pass-only block is that constant on every pixel), and the output maps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 lowpass_estimate(const RecomposeArgs &a, int f, long long q) {
    if (a.lowpass == HB_LOWPASS_TIKHONOV) {
        const long long LL = a.d.LL;
        const float *zf = a.z + (size_t)f * 6 * LL;
        const float z0 = zf[q] + zf[3 * LL + q], z1 = zf[LL + q] + zf[4 * LL + q];
        const float z2 = zf[2 * LL + q] + zf[5 * LL + q];
        const float *M = a.M;
        return make_float2(M[6] + fmaf(M[0], z0, fmaf(M[1], z1, M[2] * z2)),
                           M[7] + fmaf(M[3], z0, fmaf(M[4], z1, M[5] * z2)));
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

__global__ __launch_bounds__(kBlockThreads) void k_recompose(RecomposeArgs a) {
    __shared__ float s_c[2][kStripPixels];
    __shared__ float s_e[2][kStripPixels];
    const Dims &d = a.d;
    const StripPos s = strip_pos(d);
    const int n = d.levels, B = s.B, Wt = s.Wt, ncols = s.ncols;
    const int tid = threadIdx.x;

    for (int j = tid; j < s.nb; j += kBlockThreads) {
        const long long q = (long long)s.br * d.wl + s.blk0 + j;
        const float2 e = lowpass_estimate(a, s.f, q);
        s_e[0][j] = e.x;
        s_e[1][j] = e.y;
        a.est[(size_t)s.f * d.LL + q] = e;
    }
    for (int i = tid; i < B * ncols; i += kBlockThreads) {
        const int r = i / ncols, c = i - r * ncols;
        const float2 v = a.det[((size_t)s.f * d.H + s.row0 + r) * d.W + s.col0 + c];
        s_c[0][r * Wt + c] = v.x;
        s_c[1][r * Wt + c] = v.y;
    }
    __syncthreads();

    // Inverse Haar (Eq. 4): window = coefficients * H, levels n..1.
    for (int l = n; l >= 1; --l) {
        const int h = 1 << (l - 1), g2 = 2 * h, gr = B / g2, gc = ncols / g2;
        for (int i = tid; i < gr * gc * 2; i += kBlockThreads) {
            const int k = i & 1, q = i >> 1, r = (q / gc) * g2, c = (q % gc) * g2;
            float *u = s_c[k];
            const float ll = u[r * Wt + c], d1 = u[(r + h) * Wt + c];
            const float d2 = u[(r + h) * Wt + c + h], d3 = u[r * Wt + c + h];
            u[r * Wt + c] = 0.5f * ((ll + d1) + (d2 + d3));
            u[r * Wt + c + h] = 0.5f * ((ll + d1) - (d2 + d3));
            u[(r + h) * Wt + c] = 0.5f * ((ll - d1) - (d2 - d3));
            u[(r + h) * Wt + c + h] = 0.5f * ((ll - d1) + (d2 - d3));
        }
        __syncthreads();
    }

    for (int i = tid; i < B * ncols; i += kBlockThreads) {
        const int r = i / ncols, c = i - r * ncols, j = c >> n;
        const float hb = s_e[0][j] + s_c[0][r * Wt + c];
        const float hbo2 = s_e[1][j] + s_c[1][r * Wt + c];
        const float thb = hb + hbo2;
        const size_t o = ((size_t)s.f * d.H + s.row0 + r) * d.W + s.col0 + c;
        if (a.hb) a.hb[o] = hb;
        if (a.hbo2) a.hbo2[o] = hbo2;
        if (a.thb) a.thb[o] = thb;
        if (a.so2) a.so2[o] = (thb > a.thb_eps) ? hbo2 / thb : __builtin_nanf("");
    }
}

}  // namespace

hipError_t launch_tikhonov_fp64(const double *d_in, double *d_out, float *d_mf, hipStream_t s) {
    hipLaunchKernelGGL(k_tikhonov_fp64, dim3(1), dim3(64), 0, s, d_in, d_out, d_mf);
    return hipGetLastError();
}

hipError_t launch_log_haar(const void *frames, int n_frames, const HaarArgs &a, hipStream_t s) {
    const long long grid = (long long)n_frames * a.d.hl * a.d.strips_per_row;
    if (grid <= 0) return hipSuccess;
    switch (a.dtype) {
        case HB_F32:
            hipLaunchKernelGGL(k_log_haar<float>, dim3((unsigned)grid), dim3(kBlockThreads), 0, s,
                               (const float *)frames, a);
            break;
        case HB_F16:
            hipLaunchKernelGGL(k_log_haar<__half>, dim3((unsigned)grid), dim3(kBlockThreads), 0, s,
                               (const __half *)frames, a);
            break;
        default:
            hipLaunchKernelGGL(k_log_haar<uint16_t>, dim3((unsigned)grid), dim3(kBlockThreads), 0, s,
                               (const uint16_t *)frames, a);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_posterior(const PosteriorArgs &a, hipStream_t s) {
    const long long per_block = (long long)kBlockThreads * kPosteriorPix;
    const long long chunks = (a.LL + per_block - 1) / per_block;
    const long long grid = chunks * a.n_frames * a.split;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_posterior<kPosteriorPix>, dim3((unsigned)grid), dim3(kBlockThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_recompose(int n_frames, const RecomposeArgs &a, hipStream_t s) {
    const long long grid = (long long)n_frames * a.d.hl * a.d.strips_per_row;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_recompose, dim3((unsigned)grid), dim3(kBlockThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace hb
