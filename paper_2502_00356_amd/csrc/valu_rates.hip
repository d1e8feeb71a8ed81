// valu_rates.hip - issue rates of single VALU instructions on gfx950, the table
// behind the per-node issue-clock weights of the roofline (build.py issue_cost).
//
// Each probe kernel runs eight independent dependency chains of one operation per
// lane (so that the chain latency is hidden and only issue throughput counts) in a
// loop of `iters` trips, over `blocks` workgroups of 256 lanes. The host times one
// launch with a pair of HIP events and returns milliseconds; the caller turns that
// into wave64 instructions per CU-clock. The results are written to `sink` so that
// no chain is dead code. This is a measurement aid, not part of the
// K_nu path, and is built into its own library (libvalurates.so).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

template <typename T, typename Op>
__device__ __forceinline__ void run_chains(T (&a)[kChains], int iters, Op op)
{
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = op(a[k]);
    }
}

template <int OP>
__global__ __launch_bounds__(256) void k_rate(int iters, double p, double q, double* __restrict__ sink)
{
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const double seed = p + 1e-9 * (double)threadIdx.x;
    double outv = 0.0;
    if constexpr (OP == 0 || OP == 1 || OP == 2 || OP == 9 || OP == 13 || OP == 14) {
        double a[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = seed + k;
        if constexpr (OP == 0) run_chains(a, iters, [&](double v) { return fma(v, p, q); });
        if constexpr (OP == 1) run_chains(a, iters, [&](double v) { return v + q; });
        if constexpr (OP == 2) run_chains(a, iters, [&](double v) { return v * p; });
        if constexpr (OP == 9) run_chains(a, iters, [&](double v) { return __builtin_amdgcn_rcp(v); });
        if constexpr (OP == 13) run_chains(a, iters, [&](double v) { return __builtin_amdgcn_ldexp(v, 1); });
        if constexpr (OP == 14) run_chains(a, iters, [&](double v) { return __builtin_amdgcn_rsq(v); });
#pragma unroll
        for (int k = 0; k < kChains; ++k) outv += a[k];
    } else if constexpr (OP == 11) {
        // FP64 -> FP32 -> FP64 pairs: two conversions per step
        double a[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = seed + k;
        // the compiler folds a plain round trip, so each conversion is written out
        run_chains(a, iters, [&](double v) {
            float f;
            double r;
            asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(f) : "v"(v));
            asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(r) : "v"(f));
            return r;
        });
#pragma unroll
        for (int k = 0; k < kChains; ++k) outv += a[k];
    } else if constexpr (OP == 15) {
        unsigned int a[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = (unsigned int)tid + k;
        const unsigned int b = (unsigned int)q;
        run_chains(a, iters, [&](unsigned int v) {      // written out: a loop of adds folds
            unsigned int r;
            asm volatile("v_add_u32 %0, %1, %2" : "=v"(r) : "v"(v), "v"(b));
            return r;
        });
#pragma unroll
        for (int k = 0; k < kChains; ++k) outv += (double)a[k];
    } else {
        float a[kChains];
        const float pf = (float)p, qf = (float)q;
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = (float)seed + (float)k;
        if constexpr (OP == 3) run_chains(a, iters, [&](float v) { return fmaf(v, pf, qf); });
        if constexpr (OP == 4) run_chains(a, iters, [&](float v) { return v + qf; });
        if constexpr (OP == 5) run_chains(a, iters, [&](float v) { return v * pf; });
        if constexpr (OP == 6) run_chains(a, iters, [&](float v) { return __builtin_amdgcn_exp2f(v); });
        if constexpr (OP == 7) run_chains(a, iters, [&](float v) { return __builtin_amdgcn_logf(v); });
        if constexpr (OP == 8) run_chains(a, iters, [&](float v) { return __builtin_amdgcn_rcpf(v); });
        if constexpr (OP == 10) run_chains(a, iters, [&](float v) { return __builtin_amdgcn_sqrtf(v); });
        if constexpr (OP == 12) run_chains(a, iters, [&](float v) {   // written out: max is idempotent
            float r;
            asm volatile("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(v), "v"(qf));
            return r;
        });
#pragma unroll
        for (int k = 0; k < kChains; ++k) outv += (double)a[k];
    }
    sink[tid] = outv;
}

template <int OP>
int time_op(int iters, int blocks, double* sink, float* ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 2;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return 2; }
    int st = 0;
    // one untimed launch, then the timed one
    for (int rep = 0; rep < 2 && st == 0; ++rep) {
        if (rep == 1 && hipEventRecord(e0, nullptr) != hipSuccess) st = 2;
        hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(256), 0, nullptr, iters, 0.999999, 1e-7, sink);
        if (hipGetLastError() != hipSuccess) st = 2;
        if (rep == 1 && hipEventRecord(e1, nullptr) != hipSuccess) st = 2;
    }
    if (st == 0 && hipEventSynchronize(e1) != hipSuccess) st = 2;
    if (st == 0 && hipEventElapsedTime(ms, e0, e1) != hipSuccess) st = 2;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

// Operation codes: 0 fma_f64, 1 add_f64, 2 mul_f64, 3 fma_f32, 4 add_f32, 5 mul_f32,
// 6 exp_f32, 7 log_f32, 8 rcp_f32, 9 rcp_f64, 10 sqrt_f32, 11 cvt f64->f32->f64
// (two instructions a step), 12 max_f32, 13 ldexp_f64, 14 rsq_f64, 15 add_u32.
// sink: device buffer of blocks * 256 doubles. Returns 0, 1 (bad op) or 2 (HIP error).
extern "C" int valu_rate_ms(int op, int iters, int blocks, double* sink, float* ms)
{
    switch (op) {
    case 0: return time_op<0>(iters, blocks, sink, ms);
    case 1: return time_op<1>(iters, blocks, sink, ms);
    case 2: return time_op<2>(iters, blocks, sink, ms);
    case 3: return time_op<3>(iters, blocks, sink, ms);
    case 4: return time_op<4>(iters, blocks, sink, ms);
    case 5: return time_op<5>(iters, blocks, sink, ms);
    case 6: return time_op<6>(iters, blocks, sink, ms);
    case 7: return time_op<7>(iters, blocks, sink, ms);
    case 8: return time_op<8>(iters, blocks, sink, ms);
    case 9: return time_op<9>(iters, blocks, sink, ms);
    case 10: return time_op<10>(iters, blocks, sink, ms);
    case 11: return time_op<11>(iters, blocks, sink, ms);
    case 12: return time_op<12>(iters, blocks, sink, ms);
    case 13: return time_op<13>(iters, blocks, sink, ms);
    case 14: return time_op<14>(iters, blocks, sink, ms);
    case 15: return time_op<15>(iters, blocks, sink, ms);
    default: return 1;
    }
}
