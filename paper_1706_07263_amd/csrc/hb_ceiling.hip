// Instruction-mix microbenchmarks for gfx950 (MI355X): the issue ceilings
// that bound the posterior kernel, measured with register-only loops (no
// memory traffic inside the timed loop).  Measurement code, not part of the
// estimation path; built into its own library (libhbceiling.so).
//
// Each kernel runs `iters` iterations per wave on every lane.  Loop-carried
// chains keep the work in the loop; in MIX an empty asm statement that claims
// to modify the node operand stops the compiler from hoisting the
// (otherwise loop-invariant) MFMAs, at no instruction cost.  Results are
// written once at the end so that nothing is dead.
//
// Kinds (per wave and iteration):
//   0 MIX    the posterior's chunk evaluation for two 16-pixel blocks: per
//            block one v_mfma_f32_16x16x32_bf16, four v_exp_f32 and nine VALU
//            (three adds folding the weights, two FMAs for the first moment,
//            one add and three FMAs into the moment sums); 512 (pixel, node)
//            pairs per iteration
//   1 FMA    16 independent v_fmac_f32 chains; 16 x 64 lane-FMAs
//   2 EXP    16 v_exp_f32; 16 x 64 lane-exps
//   3 MFMA   4 independent v_mfma_f32_16x16x32_bf16; 4 MFMAs
//   4 MFMA_FMA  one v_mfma_f32_16x16x32_bf16 and 16 independent FMAs that do
//            not use its result (does the matrix pipe overlap the VALU?); 1 MFMA
//   5 EXP_FMA   8 v_exp_f32 and 8 independent FMAs; 8 x 64 lane-exps
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;

template <typename T>
__device__ __forceinline__ void opaque(T &x) {
    asm volatile("" : "+v"(x));
}

__device__ __forceinline__ bf16x8 operand(float seed) {
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (__bf16)(seed * (float)(i + 1) * 1.0e-3f);
    return v;
}

__global__ __launch_bounds__(kThreads) void k_mix(int iters, float *out) {
    const int lane = threadIdx.x & 63;
    bf16x8 node = operand(-(float)lane);
    bf16x8 px0 = operand(0.5f + lane), px1 = operand(0.25f + lane);
    float qx = 0.1f, qy = 0.2f, qz = 0.3f;
    float L0a = 0, L1a = 0, L2a = 0, L0b = 0, L1b = 0, L2b = 0;
    const f32x4 zero = {0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
        opaque(node);
        opaque(qx);
        opaque(qy);
        opaque(qz);
        const f32x4 da = __builtin_amdgcn_mfma_f32_16x16x32_bf16(node, px0, zero, 0, 0, 0);
        const f32x4 db = __builtin_amdgcn_mfma_f32_16x16x32_bf16(node, px1, zero, 0, 0, 0);
        {
            const float w0 = __builtin_amdgcn_exp2f(da[0]), w1 = __builtin_amdgcn_exp2f(da[1]);
            const float w2 = __builtin_amdgcn_exp2f(da[2]), w3 = __builtin_amdgcn_exp2f(da[3]);
            const float W0 = (w0 + w1) + (w2 + w3);
            const float W1 = fmaf(3.0f, w3, fmaf(2.0f, w2, w1));
            L0a += W0;
            L1a = fmaf(qx, W0, fmaf(qy, W1, L1a));
            L2a = fmaf(qz, W0, L2a);
        }
        {
            const float w0 = __builtin_amdgcn_exp2f(db[0]), w1 = __builtin_amdgcn_exp2f(db[1]);
            const float w2 = __builtin_amdgcn_exp2f(db[2]), w3 = __builtin_amdgcn_exp2f(db[3]);
            const float W0 = (w0 + w1) + (w2 + w3);
            const float W1 = fmaf(3.0f, w3, fmaf(2.0f, w2, w1));
            L0b += W0;
            L1b = fmaf(qx, W0, fmaf(qy, W1, L1b));
            L2b = fmaf(qz, W0, L2b);
        }
    }
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = L0a + L1a + L2a + L0b + L1b + L2b;
}

__global__ __launch_bounds__(kThreads) void k_fma(int iters, float *out) {
    float x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = (float)(threadIdx.x + i);
    const float a = 0.999f, b = 1.0e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += x[i];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_exp(int iters, float *out) {
    float x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = -(float)(threadIdx.x + i) * 1.0e-3f;
    float s = 0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = __builtin_amdgcn_exp2f(x[i]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) s += x[i];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_mfma(int iters, float *out) {
    const int lane = threadIdx.x & 63;
    bf16x8 a = operand((float)lane), b = operand(1.0f - lane);
    f32x4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
    for (int it = 0; it < iters; ++it) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
    }
    const f32x4 s = c0 + c1 + c2 + c3;
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(kThreads) void k_mfma_fma(int iters, float *out) {
    const int lane = threadIdx.x & 63;
    bf16x8 a = operand((float)lane), b = operand(1.0f - lane);
    f32x4 c0 = {0, 0, 0, 0};
    float x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = (float)(threadIdx.x + i);
    const float p = 0.999f, q = 1.0e-3f;
    for (int it = 0; it < iters; ++it) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = fmaf(x[i], p, q);
    }
    float s = c0[0] + c0[1] + c0[2] + c0[3];
#pragma unroll
    for (int i = 0; i < 16; ++i) s += x[i];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_exp_fma(int iters, float *out) {
    float x[8], y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        x[i] = -(float)(threadIdx.x + i) * 1.0e-3f;
        y[i] = (float)(threadIdx.x + i);
    }
    const float p = 0.999f, q = 1.0e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            x[i] = __builtin_amdgcn_exp2f(x[i]);
            y[i] = fmaf(y[i], p, q);
        }
    }
    float s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += x[i] + y[i];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// Work units per wave and iteration of each kind (see the table above).
double units_per_wave_iter(int kind) {
    switch (kind) {
        case 0: return 512.0;
        case 1: return 16.0 * 64.0;
        case 2: return 16.0 * 64.0;
        case 3: return 4.0;
        case 4: return 1.0;
        case 5: return 8.0 * 64.0;
    }
    return 0.0;
}

}  // namespace

extern "C" {

// Runs microbenchmark `kind` (0..5) with `blocks` workgroups of 256 threads
// (4 waves each) and `iters` loop iterations per wave on the current device,
// `reps` timed launches after one untimed launch.  *ms = fastest launch in
// milliseconds (HIP events on a stream of its own), *units = work units of
// one launch (pairs for MIX, lane-operations for FMA/EXP/EXP_FMA, MFMA
// instructions for MFMA/MFMA_FMA).  Returns 0, or -1 on a bad argument,
// -2 on a HIP error.  Allocates its output buffer and frees it before
// returning.
int hb_ceiling_measure(int kind, int blocks, int iters, int reps, double *ms, double *units) {
    if (!ms || !units || kind < 0 || kind > 5 || blocks < 1 || blocks > (1 << 20) || iters < 1 || reps < 1)
        return -1;
    float *out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * kThreads) != hipSuccess) return -2;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = -2;
    auto launch = [&]() {
        switch (kind) {
            case 0: hipLaunchKernelGGL(k_mix, dim3(blocks), dim3(kThreads), 0, s, iters, out); break;
            case 1: hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(kThreads), 0, s, iters, out); break;
            case 2: hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(kThreads), 0, s, iters, out); break;
            case 3: hipLaunchKernelGGL(k_mfma, dim3(blocks), dim3(kThreads), 0, s, iters, out); break;
            case 4: hipLaunchKernelGGL(k_mfma_fma, dim3(blocks), dim3(kThreads), 0, s, iters, out); break;
            default: hipLaunchKernelGGL(k_exp_fma, dim3(blocks), dim3(kThreads), 0, s, iters, out); break;
        }
        return hipGetLastError();
    };
    double best = 1e30;
    if (rc == 0 && (launch() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)) rc = -2;
    for (int r = 0; rc == 0 && r < reps; ++r) {
        float t = 0;
        if (hipEventRecord(e0, s) != hipSuccess || launch() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            rc = -2;
            break;
        }
        if (t < best) best = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(out);
    if (rc != 0) return rc;
    *ms = best;
    *units = units_per_wave_iter(kind) * (double)iters * (double)blocks * (kThreads / 64);
    return 0;
}

}  // extern "C"
