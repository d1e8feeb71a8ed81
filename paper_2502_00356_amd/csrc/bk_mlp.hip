// bk_mlp.hip - the window-predicting MLP (2 -> 64 -> 64 -> 3, ReLU): model handle,
// FP32 training kernels (forward/backward, weight-gradient reduction, Adam), FP16
// matrix-core inference, and the learned evaluation form of K_nu and of the
// Matern tiles.
//
// The learned form replaces the per-entry peak/window solve of Sec. IV-B with a
// prediction of [t_lo, t_hi] and the node count N from (log10 x, nu). The network
// has two inputs, so its predictions are tabulated once per model: the training
// box is cut into cells, and each cell holds the window that contains the
// network's predictions at its four corners (smallest t_lo, largest t_hi and N);
// an entry reads its cell (one 16-byte load) instead of evaluating the network.
// The Matern kernels tabulate it along log10 x at the launch's nu instead. The node
// sum is taken relative to t_lo (the first node) with the direct-exponent walk of
// bk_math.hpp (WalkF). Node exponents can then be large and positive; the FP32
// exponential is split as 2^k 2^f with k integer and f in [-1/2, 1/2] formed in
// FP64, so FP32 rounding only touches f. The node count is the predicted one,
// raised if needed to what the strip bound asks for the predicted window (one
// half-width, in FP32), so the step is always admissible. An entry is accepted
// only if (a) it lies inside the model's training box and (b) the integral beyond
// each end of the window, bounded from the two end nodes (g is concave right of an
// inflection point that lies left of the peak; the convex piece near t = 0 is
// bounded separately), is below a tolerance; otherwise it is recomputed with the
// plain FP64 solver and FP32-compensated node terms.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <random>
#include <vector>

#include "../../include/besselk.h"
#include "bk_internal.hpp"

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));

namespace bk {

constexpr int kH = 64;                 // hidden width
constexpr int kOffW1 = 0;              // offsets into the flat parameter vector
constexpr int kOffB1 = kOffW1 + kH * 2;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + 3 * kH;
constexpr int kNParam = kOffB3 + 3;
static_assert(kNParam == BK_MLP_NPARAM, "parameter count");

// Acceptance tolerance of the learned form: bound on the integral beyond an end
// node, relative to the whole. With the L = 15 window (quadrature error <= ~2.5e-7)
// and FP32 node rounding (~2e-7) this keeps the total well inside 2e-6.
constexpr float kTailTol = 3e-7f;
constexpr int kTableSize = 1024;       // Matern: MLP tabulated over log10 x at fixed nu
// Standalone K_nu: prediction cells over the training box, log10 x by nu.
constexpr int kCellsLx = 512, kCellsNu = 64, kCells = kCellsLx * kCellsNu;
// Learned Matern workspace: the window table and the interval plans of the call's
// nu (kMaternTabBytes), then the wave bitmap (one bit per wave of the call).
constexpr size_t kMaternTableOff = 0;                                   // kTableSize float4
constexpr size_t kMaternRecBytes = 96;                                  // one interval's plan record
constexpr int kRecQ = (int)(kMaternRecBytes / 16);                        // its float4 slots
// Learned Matern launch shape: a wave covers 64 rows and kMlCols columns of a tile,
// a workgroup four waves side by side.
constexpr int kMlCols = 32, kMlGroupCols = 4 * kMlCols;
constexpr size_t kMaternRecOff = kMaternTableOff + 16 * kTableSize;       // (kTableSize - 1) records
constexpr size_t kMaternTabBytes = 128 * kTableSize;                      // 128 KiB (16 KiB unused)

// Device-side constants of a model for inference.
struct MlpDev {
    const half4_t* a1;   // [4 mt][64 lanes]      layer-1 A operand (W1 | b1 | 0), K = 16
    const half8_t* a2;   // [4 mt][2 c][64]       layer-2 A operand (W2), K = 32 chunks
    const half8_t* a3;   // [2 c][64]             layer-3 A operand (W3, rows >= 3 zero)
    const float* b2;     // [64]
    const float* b3;     // [3]
    float cx, sx, cnu, snu, st, sn;     // normalisation
    float isx, isnu;                    // 1 / sx, 1 / snu
    float lx_lo, lx_hi, nu_lo, nu_hi;   // training box
    float d_lo, d_hi, eta, n_add;       // margins
    const float4_t* cells;              // [kCellsLx][kCellsNu] cell windows (normalised y0, y1, y2, 0)
    const float4_t* plan_a;             // [cell] quadrature plan: t_lo, dc, N (int bits), flags | m_pk << 1 (int bits)
    const double4_t* plan_b;            // [cell] quadrature plan: h, cosh t_lo, cosh(t_lo + h), 2 cosh h
    float cl_scale, cn_scale;           // cells per unit of log10 x and of nu
};

}  // namespace bk

struct bk_model {
    float* params = nullptr;      // device FP32 master parameters [kNParam]
    half4_t* pack = nullptr;      // device FP16 operand pack (a1, a2, a3)
    float* bias = nullptr;        // device b2 (64) and b3 (3)
    float* cells = nullptr;       // device prediction cells [kCellsLx][kCellsNu][4]
    float* plan_a = nullptr;      // device per-cell quadrature plans (float4 part)
    double* plan_b = nullptr;     // device per-cell quadrature plans (double4 part)
    double plan_Lq = -1.0;        // node target the plans were built for (< 0: none)
    double norm[8] = {-0.5, 3.5, 5.005, 4.995, 8.0, 32.0, 0.0, 0.0};
    double box[4] = {-4.0, 3.0, 0.01, 10.0};
    double margins[4] = {0.05, 0.05, 0.05, 1.0};
    double train_L[2] = {15.0, 14.5};
    int table_source = BK_TABLE_NETWORK;   // what fills the cells and the Matern table
    bool trained = false;
    int device = 0;
};

namespace bk {

static int hip_ok(hipError_t e) { return e == hipSuccess ? BK_OK : BK_EHIP; }

static MlpDev make_dev(const bk_model* m)
{
    MlpDev d;
    d.a1 = m->pack;
    d.a2 = reinterpret_cast<const half8_t*>(m->pack + 4 * 64);
    d.a3 = reinterpret_cast<const half8_t*>(m->pack + 20 * 64);
    d.b2 = m->bias;
    d.b3 = m->bias + 64;
    d.cx = (float)m->norm[0]; d.sx = (float)m->norm[1];
    d.cnu = (float)m->norm[2]; d.snu = (float)m->norm[3];
    d.isx = (float)(1.0 / m->norm[1]); d.isnu = (float)(1.0 / m->norm[3]);
    d.st = (float)m->norm[4]; d.sn = (float)m->norm[5];
    d.lx_lo = (float)m->box[0]; d.lx_hi = (float)m->box[1];
    d.nu_lo = (float)m->box[2]; d.nu_hi = (float)m->box[3];
    d.d_lo = (float)m->margins[0]; d.d_hi = (float)m->margins[1];
    d.eta = (float)m->margins[2]; d.n_add = (float)m->margins[3];
    d.cells = reinterpret_cast<const float4_t*>(m->cells);
    d.plan_a = reinterpret_cast<const float4_t*>(m->plan_a);
    d.plan_b = reinterpret_cast<const double4_t*>(m->plan_b);
    d.cl_scale = (float)((double)kCellsLx / (m->box[1] - m->box[0]));
    d.cn_scale = (float)((double)kCellsNu / (m->box[3] - m->box[2]));
    return d;
}

// ---------------------------------------------------------------------------
// Inference on matrix cores. Layers are computed transposed, H^T = W H_in^T, so
// that the accumulator layout of one layer (v_mfma_f32_16x16x*: lane holds rows
// 4q..4q+3 of column r, q = lane/16, r = lane%16) is the B operand of the next.
// Layer 1 (K = 3 inputs + bias, padded to 16) uses v_mfma_f32_16x16x16f16, where a
// lane's B operand is k = 4q..4q+3. Layers 2 and 3 (K = 64) use the gfx950
// v_mfma_f32_16x16x32f16 in two K = 32 chunks, where a lane's B operand is
// k = 8q..8q+7; chunk c takes the lane's accumulator rows of the two 16-unit
// tiles 2c and 2c+1 as they stand, i.e. its k order is
//   k = 8q + j  <->  hidden unit 16 (2c + (j >= 4)) + 4q + (j & 3),
// and the A operands (W2, W3) are packed on the host in that same order. A wave
// evaluates its 64 entries as four column tiles of 16; all 64 lanes must be active.
// ---------------------------------------------------------------------------
// ReLU after rounding to FP16: packed conversion (two v_cvt_pk_f16_f32) and a
// packed maximum with zero (two v_pk_max on half pairs). Rounding commutes with
// max(., 0), so this equals rounding the FP32 ReLU.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ half4_t relu_h4(float4_t v)
{
    half2_t lo, hi;
    lo[0] = (_Float16)v[0];
    lo[1] = (_Float16)v[1];
    hi[0] = (_Float16)v[2];
    hi[1] = (_Float16)v[3];
    const half2_t z = {(_Float16)0.0f, (_Float16)0.0f};
    lo = __builtin_elementwise_max(lo, z);
    hi = __builtin_elementwise_max(hi, z);
    half4_t h;
    h[0] = lo[0];
    h[1] = lo[1];
    h[2] = hi[0];
    h[3] = hi[1];
    return h;
}

// Cross-lane read of v from the lane whose byte address (4 x lane) is addr.
__device__ __forceinline__ float bperm(int addr, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

__device__ __forceinline__ half8_t cat8(half4_t lo, half4_t hi)
{
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ inline void mlp_wave(const MlpDev& M, float u0, float u1, float& y0, float& y1, float& y2)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const float4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
    // Layer 1 for the wave's four 16-entry column tiles (bias folded in through the
    // constant-1 input row).
    half4_t h1[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int src = (16 * nt + r) << 2;
        const float e0 = bperm(src, u0);
        const float e1 = bperm(src, u1);
        half4_t b0;
        b0[0] = (_Float16)(q == 0 ? e0 : 0.0f);
        b0[1] = (_Float16)(q == 0 ? e1 : 0.0f);
        b0[2] = (_Float16)(q == 0 ? 1.0f : 0.0f);
        b0[3] = (_Float16)0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            h1[nt][mt] = relu_h4(__builtin_amdgcn_mfma_f32_16x16x16f16(M.a1[mt * 64 + lane], b0, zero, 0, 0, 0));
    }
    // Layers 2 and 3, one 16-unit row block of layer 2 at a time: each weight
    // fragment is read once per wave and applied to the four column tiles (four
    // independent accumulation chains); layer 3 consumes a K chunk as soon as both
    // of its layer-2 tiles are done.
    float4_t o[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int it = 0; it < 4; ++it) o[nt][it] = (q == 0 && it < 3) ? M.b3[it] : 0.0f;
    half4_t h2[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const float4_t bias = *reinterpret_cast<const float4_t*>(M.b2 + 16 * mt + 4 * q);
        float4_t acc[4] = {bias, bias, bias, bias};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const half8_t a = M.a2[(mt * 2 + c) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, cat8(h1[nt][2 * c], h1[nt][2 * c + 1]), acc[nt],
                                                                 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) h2[nt][mt & 1] = relu_h4(acc[nt]);
        if (mt & 1) {
            const half8_t a3 = M.a3[(mt >> 1) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a3, cat8(h2[nt][0], h2[nt][1]), o[nt], 0, 0, 0);
        }
    }
    // outputs of entry 16 nt + r sit in lane r (q == 0) of tile nt, items 0..2
    y0 = y1 = y2 = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float s0 = bperm(r << 2, o[nt][0]), s1 = bperm(r << 2, o[nt][1]), s2 = bperm(r << 2, o[nt][2]);
        if (q == nt) { y0 = s0; y1 = s1; y2 = s2; }
    }
}

__global__ __launch_bounds__(256) void k_mlp_infer(MlpDev M, const float* __restrict__ u, float* __restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float u0 = 0.0f, u1 = 0.0f;
    if (i < n) { u0 = u[2 * i]; u1 = u[2 * i + 1]; }
    float y0, y1, y2;
    mlp_wave(M, u0, u1, y0, y1, y2);
    if (i < n) { y[3 * i] = y0; y[3 * i + 1] = y1; y[3 * i + 2] = y2; }
}

// Prediction cells: one lane per cell (i along log10 x, j along nu) evaluates the
// network at the cell's four corners and keeps the window that contains all four
// predictions. Corner (i, j) lies at (lx_lo + i dl, nu_lo + j dn); the corner
// inputs are rounded operation by operation (contraction into FMA is off here),
// so that they can be reproduced exactly elsewhere.
__global__ __launch_bounds__(256) void k_cell_table(MlpDev M, float4_t* __restrict__ cells)
{
#pragma clang fp contract(off)
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int cc = min(c, kCells - 1);
    const int i = cc / kCellsNu, j = cc % kCellsNu;
    const float dl = (M.lx_hi - M.lx_lo) / (float)kCellsLx;
    const float dn = (M.nu_hi - M.nu_lo) / (float)kCellsNu;
    float4_t w = {__builtin_inff(), -__builtin_inff(), -__builtin_inff(), 0.0f};
    for (int k = 0; k < 4; ++k) {          // uniform trip count: the whole wave runs the network
        const float lx = M.lx_lo + (float)(i + (k & 1)) * dl;
        const float nu = M.nu_lo + (float)(j + (k >> 1)) * dn;
        float y0, y1, y2;
        mlp_wave(M, (lx - M.cx) * M.isx, (nu - M.cnu) * M.isnu, y0, y1, y2);
        w[0] = fminf(w[0], y0);
        w[1] = fmaxf(w[1], y1);
        w[2] = fmaxf(w[2], y2);
    }
    if (c < kCells) cells[c] = w;
}

// The plain solver's window (Sec. IV-B: peak, window ends at g* - L, strip-bound
// node count for exp(-Lq)) at (nu, 10^lx), in the network's normalised output
// units (t_lo / st, t_hi / st, N / sn). N / sn is exact in FP32 (sn is a power of
// two), so the decode gives back N.
__device__ inline void solver_prediction(const MlpDev& M, float lx, float nu, double L, double Lq, float& y0,
                                         float& y1, float& y2)
{
    const Solved s = plain_solve((double)nu, exp10((double)lx), L, Lq, rule_tab(), rule_tab().tab);
    y0 = (float)(s.p.t0 / (double)M.st);
    y1 = (float)(s.t1 / (double)M.st);
    y2 = (float)((double)s.p.N / (double)M.sn);
}

// Prediction cells filled by the plain solver instead of the network, at the same
// four corners (the union of the solver's windows there): the learned form without
// the network, for measuring what the network itself contributes.
__global__ __launch_bounds__(256) void k_cell_table_solver(MlpDev M, double L, double Lq,
                                                           float4_t* __restrict__ cells)
{
#pragma clang fp contract(off)
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= kCells) return;
    const int i = c / kCellsNu, j = c % kCellsNu;
    const float dl = (M.lx_hi - M.lx_lo) / (float)kCellsLx;
    const float dn = (M.nu_hi - M.nu_lo) / (float)kCellsNu;
    float4_t w = {__builtin_inff(), -__builtin_inff(), -__builtin_inff(), 0.0f};
    for (int k = 0; k < 4; ++k) {
        const float lx = M.lx_lo + (float)(i + (k & 1)) * dl;
        const float nu = M.nu_lo + (float)(j + (k >> 1)) * dn;
        float y0, y1, y2;
        solver_prediction(M, lx, nu, L, Lq, y0, y1, y2);
        w[0] = fminf(w[0], y0);
        w[1] = fmaxf(w[1], y1);
        w[2] = fmaxf(w[2], y2);
    }
    cells[c] = w;
}

// The cell of an entry inside the training box (the last cell of each axis also
// takes the box's upper edge).
__device__ __forceinline__ int cell_index(const MlpDev& M, float lx, float v)
{
    const int i = min(max((int)((lx - M.lx_lo) * M.cl_scale), 0), kCellsLx - 1);
    const int j = min(max((int)((v - M.nu_lo) * M.cn_scale), 0), kCellsNu - 1);
    return i * kCellsNu + j;
}

// ---------------------------------------------------------------------------
// Learned node sum. Reference t_ref = t_lo (node 0), outward walk only.
// ---------------------------------------------------------------------------
struct LearnedOut {
    double hs;      // h * S (trapezoid value of the scaled integral)
    double delta;   // log prefactor Delta at t_ref
    int reason;     // 0 accepted, else a BK_STAT_FB_* index
};

// Quadrature plan of a learned window: nodes t_lo + m h, m = 0..N, the start of the
// cosh recurrence, c0 = cosh t_lo, c1 = cosh(t_lo + h), kappa = 2 cosh h, and the
// parts that depend on nu as well: rho = e^(-2 nu h), Q0 = 1 + e^(-2 nu t_lo),
// b2 = nu h log2 e, dnu = nu t_lo - ln 2.
struct LearnedPlan {
    double tlo, h, c0, c1, kappa;
    double rho, Q0, b2, dnu;
    int N;
};

// The nu-dependent part of a plan (T: the table 2^(j/64) of exp_tab). Q only needs
// FP32 accuracy: e^(-2 nu t_lo) in FP32 moves it by < 6e-8 relative.
__device__ __forceinline__ void plan_for_nu(LearnedPlan& P, double nu, const double* T)
{
    P.rho = exp_tab(-2.0 * nu * P.h, T);
    P.Q0 = 1.0 + (double)__expf((float)(-2.0 * nu * P.tlo));
    P.b2 = nu * P.h * kLog2e;
    P.dnu = nu * P.tlo - kLn2;
}

// The plan of the window [t_lo, t_hi] with N intervals. Any step works as long as
// the walk uses it consistently: an FP32 reciprocal of N puts the last node within
// ~1e-7 of t_hi. T: the table 2^(j/64) of exp_tab.
__device__ inline LearnedPlan learned_plan(double tlo, double thi, int N, const double* T)
{
    LearnedPlan P;
    P.tlo = tlo;
    P.N = N;
    P.h = (thi - tlo) * (double)__builtin_amdgcn_rcpf((float)N);
    const double e = exp_tab(tlo, T), ei = recip(e);
    const double q2 = exp_tab(P.h, T), qi2 = recip(q2);
    P.c0 = 0.5 * (e + ei);
    P.c1 = 0.5 * (e * q2 + ei * qi2);
    P.kappa = q2 + qi2;
    return P;
}

// Node sum of the standalone learned form: terms relative to node 0, or with kBias
// to 2^eb (eb in log2 units, an estimate of the largest node's exponent from the
// cell), so that every FP32 exponential sees an argument of moderate size and the
// 2^k 2^f split is not needed (the prefactor carries 2^eb); else the split is made
// at every node. The factor Q = 1 + e^(-2 nu t) follows Q' = rho Q + (1 - rho) in
// FP64 and is rounded to FP32 once per node. An argument d converts to FP32 with an
// absolute error of |d| 2^-24; the terms that carry the sum lie within a few units
// of eb, the others are smaller by 2^-|d|, so this adds a few 1e-8 to the sum. The
// FP32 terms are summed in FP64, whose rounding is negligible next to theirs.
template <bool kBias>
__device__ inline void learned_sum(WalkF& w, int N, float& e0, float& e1, float& eprev, float& elast, double& Sd)
{
    auto node = [&]() {
        const double d = walkf_exponent2(w);
        float t;
        if (kBias) {
            t = __builtin_amdgcn_exp2f((float)d) * (float)w.Q;
        } else {
            const double kf = rint(d);
            t = ldexpf(__builtin_amdgcn_exp2f((float)(d - kf)) * (float)w.Q, (int)kf);
        }
        walkf_step(w);
        return t;
    };
    // groups of four are added pairwise in FP32 (two roundings, <= 1.2e-7 of the
    // group, all terms positive) and the groups sum in FP64
    e0 = node();
    e1 = node();                               // N >= kNodeMin: at least five nodes
    Sd = (double)(e0 + e1);
    eprev = e0;
    elast = e1;
    int m = 2;
    for (; m + 3 <= N; m += 4) {
        const float ta = node(), tb = node(), tc = node(), td = node();
        Sd += (double)((ta + tb) + (tc + td));
        eprev = tc;
        elast = td;
    }
    if (m + 1 <= N) {
        const float ta = node(), tb = node();
        Sd += (double)(ta + tb);
        eprev = ta;
        elast = tb;
        m += 2;
    }
    if (m == N) {                               // one node left
        const float t = node();
        Sd += (double)t;
        eprev = elast;
        elast = t;
    }
}

// Right tail beyond the last node t_N, in units of the trapezoid sum S (integral /
// h). g = log cosh(nu t) - x cosh t has g'' = nu^2 sech^2(nu t) - x cosh t,
// decreasing in t: g is convex on [0, t_c) and concave on [t_c, inf) (t_c = 0 if
// nu^2 <= x), and g' > 0 on (0, t_c], so the peak t* lies right of t_c. If e_N <
// e_{N-1}, the mean value theorem puts a point xi > t* in (t_{N-1}, t_N) where g'(xi)
// is the secant slope; g' decreases right of t_c, so |g'| >= |secant| on [t_N, inf)
// and the tail is at most e_N / |log(e_N / e_{N-1})|. First without the logarithm:
// |log r| >= 1 - r for r = e_N / e_{N-1} < 1, so e_N e_{N-1} <= tol S (e_{N-1} -
// e_N) already implies the bound.
__device__ __forceinline__ bool right_tail_ok(float eprev, float elast, float S)
{
    if (!(elast < eprev)) return false;
    bool ok = elast * eprev <= kTailTol * S * (eprev - elast);
    if (__builtin_expect(!ok, 0)) {             // rare: a branch, not computed for every entry
        const float lr = __builtin_amdgcn_logf(elast * __builtin_amdgcn_rcpf(eprev)) * 0.69314718f;
        ok = elast <= -lr * kTailTol * S;
    }
    return ok;
}

// Left tail below the first node t_lo > 0 (e_0 < e_1 needed, so t_lo < t*), in
// units of S, for the same g. t_c is the fixed point of the decreasing map F(t) =
// acosh(nu / sqrt(x cosh t)) / nu (0 where the argument is <= 1), so F(0) >= t_c,
// and alternate iterates from there bound t_c from below and above: lo <= t_c <= up
// (each FP32 value moved outward by 2^-10 relative, far above its rounding). F(0)
// alone settles most windows (t_lo >= F(0)); the others take two more pairs of
// iterates. D = g(t_lo) - g(0) >= Delta = nu t_lo - ln 2 - x (cosh t_lo - 1) (the
// log(1 + e^(-2 nu t_lo)) part dropped; the caller passes Delta), and ll = log(e_1 /
// e_0) = s h, s the secant slope of the first two nodes.
//  - t_lo >= up: as on the right, g'(t) >= s on [t_c, t_lo], so g lies below the
//    line through t_lo of slope s there; on [0, up] g is below the chord from (0,
//    g(0)) to (up, line(up)) (convex up to t_c, and the line bounds the rest), so
//    the tail is at most e_0 (1 / ll + (up / h) (e^a - e^b) / (a - b)), a = -ll (t_lo
//    - up) / h, b = -D.
//  - t_lo <= lo: g is convex on [0, t_lo], below its chord, and the tail is at most
//    e_0 (t_lo / h) (1 - e^-D) / D.
//  - otherwise the window is rejected.
__device__ inline bool left_tail_ok(double x, double nu, float tlof, float hf, float e0, float e1, float delta,
                                    float S)
{
    if (!(e0 < e1)) return false;
    const float ll = __builtin_amdgcn_logf(e1 * __builtin_amdgcn_rcpf(e0)) * 0.69314718f;
    const float nuf = (float)nu, xf = (float)x, inu = __builtin_amdgcn_rcpf(nuf);
    auto F = [&](float ch) {                    // ch = cosh t
        const float y = nuf * __builtin_amdgcn_rsqf(xf * ch);
        if (!(y > 1.0f)) return 0.0f;
        return __builtin_amdgcn_logf(y + __builtin_amdgcn_sqrtf(fmaf(y, y, -1.0f))) * 0.69314718f * inu;
    };
    auto coshf_ = [](float t) {
        const float e = __builtin_amdgcn_exp2f(t * 1.44269504f);
        return 0.5f * (e + __builtin_amdgcn_rcpf(e));
    };
    const float ih = __builtin_amdgcn_rcpf(hf);
    float up = F(1.0f) * 1.0009765625f, lo = 0.0f;
    if (!(tlof >= up)) {                        // t_lo near t_c: narrow the bounds
        lo = F(coshf_(up)) * 0.9990234375f;
        up = fminf(up, F(coshf_(lo)) * 1.0009765625f);
        lo = fmaxf(lo, F(coshf_(up)) * 0.9990234375f);
        up = fminf(up, F(coshf_(lo)) * 1.0009765625f);
    }
    const float D = fmaxf(delta, 0.0f);
    float bound;
    if (tlof >= up) {
        const float a = -ll * (tlof - up) * ih, b = -D, dab = a - b;
        const float ea = __builtin_amdgcn_exp2f(a * 1.44269504f), eb2 = __builtin_amdgcn_exp2f(b * 1.44269504f);
        // mean of e^t between b and a (at most the larger end value)
        const float chord = fabsf(dab) > 1e-3f ? (ea - eb2) * __builtin_amdgcn_rcpf(dab) : fmaxf(ea, eb2);
        bound = e0 * (__builtin_amdgcn_rcpf(ll) + up * ih * chord);
    } else if (tlof <= lo) {
        const float r = D > 1e-3f ? (1.0f - __builtin_amdgcn_exp2f(-D * 1.44269504f)) * __builtin_amdgcn_rcpf(D)
                                  : 1.0f;       // (1 - e^-D) / D <= 1
        bound = e0 * tlof * ih * r;
    } else {
        return false;
    }
    return bound <= kTailTol * S;
}

// The node sum of a plan (for its nu) at one x, its prefactor and the acceptance
// tests. Reference t_ref = t_lo (node 0), outward walk only; kBias as learned_sum.
template <bool kBias>
__device__ inline LearnedOut learned_walk(double x, double nu, const LearnedPlan& P, double eb = 0.0)
{
    LearnedOut o;
    o.reason = 0;
    const double tlo = P.tlo, h = P.h;
    const int N = P.N;
    // sinh^2(t/2) = (cosh t - 1) / 2 loses ~1e-16 absolute, i.e. at most ~2e-13
    // relative in the scale for x <= 1e3, far inside this form's budget
    o.delta = P.dnu - x * (P.c0 - 1.0);
    WalkF w;
    w.kappa = P.kappa;
    w.c = P.c0;
    w.cn = P.c1;
    w.a2 = -x * kLog2e;
    w.b2 = P.b2;
    w.e = x * P.c0 * kLog2e;
    if (kBias) {
        w.e -= eb;
        o.delta = fma(eb, kLn2, o.delta);
    }
    w.rho = P.rho;
    w.omr = 1.0 - P.rho;
    w.Q = P.Q0;
    float e0, e1, eprev, elast;
    double Sd;
    learned_sum<kBias>(w, N, e0, e1, eprev, elast, Sd);
    Sd -= (double)(0.5f * (e0 + elast));       // one FP32 rounding of a term-sized value
    o.hs = h * Sd;
    if (!(Sd > 0.0) || !isfinite(Sd)) { o.reason = BK_STAT_FB_NONFINITE; return o; }
    const float S = (float)Sd;
    if (!right_tail_ok(eprev, elast, S)) { o.reason = BK_STAT_FB_TAIL; return o; }
    if (tlo > 0.0) {
        const float D = (float)(kBias ? fma(-eb, kLn2, o.delta) : o.delta);
        if (!left_tail_ok(x, nu, (float)tlo, (float)h, e0, e1, D, S)) { o.reason = BK_STAT_FB_TAIL; return o; }
    }
    return o;
}

// Step floor for the learned forms: the strip bound of node_step at a single
// half-width, a = min(sqrt(2 (Lq + ln 2) / (x + nu + 1)), 1.3) (the maximiser of
// the bound's small-a expansion, capped), in FP32 with 1 - cos a = 2 sin^2(a/2),
// shrunk by 0.1% so that rounding can only add nodes. Any a in (0, pi/2) gives an
// admissible step; over the grid law this one is within 6% of the best of the 15
// candidates the plain solver tries (median 0.5%), for a fraction of the work.
__device__ __forceinline__ float node_step_learned(float nu, float x, float Lq)
{
    const float c = Lq + 0.693147181f, nu1 = nu + 1.0f;
    const float a = fminf(__builtin_amdgcn_sqrtf(2.0f * c * __builtin_amdgcn_rcpf(x + nu1)), 1.3f);
    const float s = __sinf(0.5f * a);
    // cos a >= cos 1.3 > 0.26: the hardware logarithm needs no range handling
    const float den = c + 2.0f * x * s * s - nu1 * 0.69314718f * __builtin_amdgcn_logf(__cosf(a));
    return 6.28318531f * 0.999f * a * __builtin_amdgcn_rcpf(den);
}

// Window from a prediction (normalised outputs y), with the model's margins; the
// node count is the prediction or the step floor's count for this window,
// whichever is larger (raised says which). N = -1 if the floor asks for more than
// kNodeMax intervals (no admissible step within the cap).
__device__ __forceinline__ void decode_window(const MlpDev& M, float y0, float y1, float y2, double nu, double x,
                                              double Lq, double& tlo, double& thi, int& N, bool& raised)
{
    tlo = fmax(0.0, (double)(y0 * M.st - M.d_lo));
    thi = (double)(y1 * M.st + M.d_hi);
    float nf = ceilf(y2 * M.sn * (1.0f + M.eta) + M.n_add);
    if (!(nf >= (float)kNodeMin)) nf = (float)kNodeMin;
    if (nf > (float)kNodeMax) nf = (float)kNodeMax;
    float nr = ceilf((float)(thi - tlo) * __builtin_amdgcn_rcpf(node_step_learned((float)nu, (float)x, (float)Lq)));
    if (nr > (float)kNodeMax) { raised = true; N = -1; return; }
    if (!(nr >= (float)kNodeMin)) nr = (float)kNodeMin;
    raised = nr > nf;
    N = (int)(raised ? nr : nf);
}

__device__ __forceinline__ bool in_box(const MlpDev& M, float lx, float v)
{
    return lx >= M.lx_lo && lx <= M.lx_hi && v >= M.nu_lo && v <= M.nu_hi;
}

// Quadrature plans of the prediction cells for the node target Lq, one lane per
// cell: the window decoded from the cell's union with the model's margins; the node
// count from the prediction, raised to the strip-bound floor taken at the cell's
// corner of largest x and nu (at any point of the cell the half-width of that
// corner gives a larger admissible step, so this floor holds over the whole cell);
// and the start of the walk in FP64. plan_a: t_lo; dc = cosh t_pk - cosh t_lo for
// the node t_pk = t_lo + m_pk h of the largest term at the cell's centre (without
// the bounded log(1 + e^(-2 nu t)) part); N (-1 if the window is empty or not
// finite); flags (bit 0: N raised; bits 1 up: m_pk); the last two as int bits.
// The walk scales its FP32 terms by the term at t_pk, so that no node needs the
// 2^k 2^f split of an unbounded exponent.
__global__ __launch_bounds__(256) void k_cell_plans(MlpDev M, double Lq, float4_t* __restrict__ pa,
                                                    double4_t* __restrict__ pb)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= kCells) return;
    const int i = c / kCellsNu, j = c % kCellsNu;
    const float4_t y = M.cells[c];
    const double lxm = (double)M.lx_lo + (double)(i + 1) * (((double)M.lx_hi - (double)M.lx_lo) / kCellsLx);
    const double xm = exp10(lxm);
    const double num = (double)M.nu_lo + (double)(j + 1) * (((double)M.nu_hi - (double)M.nu_lo) / kCellsNu);
    double tlo, thi;
    int N;
    bool raised;
    decode_window(M, y[0], y[1], y[2], num, xm, Lq, tlo, thi, N, raised);
    const bool valid = thi > tlo && isfinite(thi) && N >= 0;
    float4_t a;
    a[0] = (float)tlo;                    // exact: the window ends are FP32 values
    a[1] = 0.0f;
    a[2] = __int_as_float(valid ? N : -1);
    int flags = raised ? 1 : 0;
    double4_t b = {0.0, 1.0, 1.0, 2.0};
    if (valid) {
        const double h = (thi - tlo) * (double)__builtin_amdgcn_rcpf((float)N);
        b[0] = h;
        b[1] = cosh(tlo);
        b[2] = cosh(tlo + h);
        b[3] = 2.0 * cosh(h);
        const double xc = exp10(lxm - 0.5 * (((double)M.lx_hi - (double)M.lx_lo) / kCellsLx));
        const double nuc = num - 0.5 * (((double)M.nu_hi - (double)M.nu_lo) / kCellsNu);
        int mpk = 0;
        double best = 0.0;
        for (int m = 1; m <= N; ++m) {
            const double d = nuc * (double)m * h - xc * (cosh(tlo + (double)m * h) - b[1]);
            if (d > best) { best = d; mpk = m; }
        }
        a[1] = (float)(cosh(tlo + (double)mpk * h) - b[1]);
        flags |= mpk << 1;
    }
    a[3] = __int_as_float(flags);
    pa[c] = a;
    pb[c] = b;
}

// c e^r for the FP32-term forms: r log2 e = k + f is split in FP64 (|f| <= 1/2),
// 2^f is the FP32 exponential (about an ulp, 1.2e-7 relative) and 2^k is applied
// last, so that only the final result rounds (into the subnormal range, if it
// lies there). The split's rounding, |r| 2^-53 <= 1e-13 for the arguments here,
// and the conversion of f to FP32 (< 2e-8) add less than 2e-7 in all, inside the
// 2e-6 budget of these forms.
__device__ __forceinline__ double scaled_exp(double r, double c)
{
    const double y = r * kLog2e;
    const double k = rint(y);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(y - k)) * c, (int)k);
}

// c 2^k rounded to the output type (exact scaling; for FP32 output one rounding of
// c to FP32 first where c lies well inside its range).
template <typename OutT>
__device__ __forceinline__ OutT scale2_out(double c, int k)
{
    if constexpr (sizeof(OutT) == sizeof(float)) {
        if (!(c > 1e-30 && c < 1e30)) return (float)ldexp(c, k);
        return ldexpf((float)c, k);
    } else {
        return ldexp(c, k);
    }
}

// Final value for the FP32-term forms: c = h S times e^(Delta - z) (or e^Delta).
__device__ __forceinline__ double assemble_k(double z, double delta, double hs, int result)
{
    if (result == BK_RESULT_SCALED) return scaled_exp(delta, hs);
    if (result == BK_RESULT_LOG) return (delta - z) + log(hs);
    return scaled_exp(delta - z, hs);
}

__device__ __forceinline__ bool special_k(double v, double z, int result, double& r)
{
    if (isnan(v) || isnan(z) || z < 0.0) { r = __builtin_nan(""); return true; }
    if (z == 0.0 || isinf(v)) { r = __builtin_inf(); return true; }
    if (isinf(z)) { r = (result == BK_RESULT_LOG) ? -__builtin_inf() : 0.0; return true; }
    return false;
}

__device__ void block_stats(unsigned long long* stats, const unsigned long long* v, int nv)
{
    __shared__ unsigned long long red[4][8];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < nv; ++k) {
        unsigned long long a = v[k];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (lane == 0) red[wid][k] = a;
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        unsigned long long t = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        if (t) atomicAdd(stats + threadIdx.x, t);
    }
}

// Workspace: [0] fallback count (uint32), queue of uint32 indices from byte 256.
__global__ void k_zero_u32(unsigned int* p) { if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0u; }

// Per-block statistics reduction for blocks of nw wave64s (nw <= 16).
__device__ void block_stats_w(unsigned long long* stats, const unsigned long long* v, int nv, int nw)
{
    __shared__ unsigned long long red[16][8];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < nv; ++k) {
        unsigned long long a = v[k];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (lane == 0) red[wid][k] = a;
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        unsigned long long t = 0;
        for (int w = 0; w < nw; ++w) t += red[w][threadIdx.x];
        if (t) atomicAdd(stats + threadIdx.x, t);
    }
}

// Learned K_nu. Phase 1 (entry order): range check, the entry's prediction cell
// and, with kPlan (the call's node target is the one the cells' plans were built
// for), the cell's quadrature plan, else the window decoded for this entry.
// Phase 2: the block's entries are counting-sorted by node count
// through LDS, so each wave walks entries of similar N (the wave runs as many
// node steps as its largest N). Phase 3 (sorted order): node sums, tail checks,
// stores to the entry's own index or the fallback queue.
constexpr int kLearnedBlock = 256;
constexpr int kSortBins = 64;

template <bool kPlan>
__global__ __launch_bounds__(kLearnedBlock, 5) void k_besselk_learned(MlpDev M, const double* __restrict__ nu,
                                                                   const double* __restrict__ x,
                                                                   double* __restrict__ out, int64_t n, int result,
                                                                   double Lq, 
                                                                   unsigned int* __restrict__ qcount,
                                                                   unsigned int* __restrict__ queue,
                                                                   unsigned long long* __restrict__ stats)
{
    __shared__ unsigned int hist[kSortBins];
    __shared__ double s_exp2[64];
    __shared__ double s_v[kLearnedBlock], s_z[kLearnedBlock], s_tlo[kLearnedBlock], s_thi[kLearnedBlock];
    __shared__ int s_N[kLearnedBlock];
    __shared__ unsigned int s_idx[kLearnedBlock];
    __shared__ int s_cell[kLearnedBlock];        // plan path only
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kLearnedBlock + tid;
    int cell = 0;
    const bool live = i < n;
    double v = 0.0, z = 1.0;
    if (live) { v = fabs(nu[i]); z = x[i]; }
    if (tid < kSortBins) hist[tid] = 0u;
    if (tid < 64) s_exp2[tid] = rule_tab().tab[tid];         // 2^(j/64); read after the sort's barriers
    const float lx = __log2f((float)(z > 0.0 ? z : 1.0)) * 0.30102999566f;   // log10 x in FP32
    // per-lane statistics as scalars (a dynamically indexed array would live in scratch)
    unsigned int c_range = 0, c_tail = 0, c_raised = 0, c_nonfin = 0, c_nodes = 0, c_ent = 0;
    double tlo = 0.0, thi = 0.0;             // plan path: thi holds the cell's dc
    int N = -1, mpk = 0;
    // the ordinary case (finite nu, 0 < x < inf) in three compares; special_k covers
    // every other input
    const bool ordinary = z > 0.0 && z < __builtin_inf() && v < __builtin_inf();
    if (live) {
        double r;
        if (!ordinary) {
            special_k(v, z, result, r);
            out[i] = r;
        } else {
            bool reject = false;
            if (!in_box(M, lx, (float)v)) {
                reject = true;
                c_range = 1;
            } else {
                if constexpr (kPlan) {
                    cell = cell_index(M, lx, (float)v);
                    const float4_t a = M.plan_a[cell];
                    tlo = (double)a[0];
                    thi = (double)a[1];
                    const int Nd = __float_as_int(a[2]), fl = __float_as_int(a[3]);
                    c_raised = (unsigned int)(fl & 1);
                    if (Nd < 0) { reject = true; c_nonfin = 1; }
                    else { N = Nd; mpk = fl >> 1; }
                } else {
                    bool raised;
                    int Nd;
                    const float4_t y = M.cells[cell_index(M, lx, (float)v)];
                    decode_window(M, y[0], y[1], y[2], v, z, Lq, tlo, thi, Nd, raised);
                    c_raised = raised ? 1u : 0u;
                    if (!(thi > tlo) || !isfinite(thi) || Nd < 0) { reject = true; c_nonfin = 1; }
                    else N = Nd;
                }
            }
            if (reject) {
                const unsigned int slot = atomicAdd(qcount, 1u);
                queue[slot] = (unsigned int)i;
            }
        }
    }
    // counting sort of the block by N (bins 0..63; N >= 63 share the last bin)
    __syncthreads();
    const int key = N < 0 ? 0 : (N < kSortBins - 1 ? N : kSortBins - 1);
    const unsigned int rank = atomicAdd(&hist[key], 1u);
    __syncthreads();
    if (tid < 64) {
        const unsigned int h = hist[tid];
        hist[tid] = wave_incl_scan(h) - h;    // exclusive prefix: first slot of the bin
    }
    __syncthreads();
    const unsigned int dst = hist[key] + rank;
    s_v[dst] = v;
    s_z[dst] = z;
    s_tlo[dst] = tlo;
    s_thi[dst] = thi;
    if constexpr (kPlan) s_cell[dst] = cell;
    s_N[dst] = N < 0 ? -1 : (N | (mpk << 16));   // N <= kNodeMax < 2^16
    s_idx[dst] = (unsigned int)i;
    __syncthreads();
    const int Np = s_N[tid];
    if (Np >= 0) {
        const int Ns = Np & 0xffff;
        const double vs = s_v[tid], zs = s_z[tid];
        const unsigned int idx = s_idx[tid];
        LearnedPlan P;
        if constexpr (kPlan) {
            const double4_t b = M.plan_b[s_cell[tid]];
            P.tlo = s_tlo[tid];
            P.h = b[0];
            P.c0 = b[1];
            P.c1 = b[2];
            P.kappa = b[3];
            P.N = Ns;
        } else {
            P = learned_plan(s_tlo[tid], s_thi[tid], Ns, s_exp2);
        }
        plan_for_nu(P, vs, s_exp2);
        LearnedOut lo;
        if constexpr (kPlan) {
            // log2 of the term at the cell's peak node t_pk relative to node 0, at this entry
            const double eb = (vs * ((double)(Np >> 16) * P.h) - zs * s_thi[tid]) * kLog2e;
            lo = learned_walk<true>(zs, vs, P, eb);
        } else {
            lo = learned_walk<false>(zs, vs, P);
        }
        c_nodes = (unsigned int)(Ns + 1);
        c_ent = 1;
        if (lo.reason == 0) {
            out[idx] = assemble_k(zs, lo.delta, lo.hs, result);
        } else {
            if (lo.reason == BK_STAT_FB_TAIL) c_tail += 1; else c_nonfin += 1;
            const unsigned int slot = atomicAdd(qcount, 1u);
            queue[slot] = idx;
        }
    }
    if (stats) {
        unsigned long long cnt[8];
        cnt[BK_STAT_ENTRIES] = c_ent;
        cnt[BK_STAT_NODES] = c_nodes;
        cnt[BK_STAT_FB_RANGE] = c_range;
        cnt[BK_STAT_FB_TAIL] = c_tail;
        cnt[BK_STAT_NODE_RAISED] = c_raised;
        cnt[BK_STAT_FB_NONFINITE] = c_nonfin;
        cnt[BK_STAT_FB_NODES] = 0;
        unsigned int wmax = c_nodes;
        for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, (unsigned int)__shfl_xor((int)wmax, o, 64));
        cnt[BK_STAT_LANE_SLOTS] = (threadIdx.x & 63) == 0 ? 64ull * wmax : 0ull;
        block_stats_w(stats, cnt, 8, kLearnedBlock / 64);
    }
}

// Fallback: plain FP64 solve with FP32-compensated node terms, over the queue.
__global__ __launch_bounds__(256) void k_besselk_fallback(const double* __restrict__ nu, const double* __restrict__ x,
                                                          double* __restrict__ out, int result,
                                                          const unsigned int* __restrict__ qcount,
                                                          const unsigned int* __restrict__ queue, double L, double Lq,
                                                          
                                                          unsigned long long* __restrict__ stats)
{
    __shared__ double s_tab[kTabLen];
    const unsigned int cnt = *qcount;
    if (blockIdx.x * 256u >= cnt) return;      // the whole block has no entry (uniform)
    stage_tab(s_tab);
    unsigned long long nodes = 0, ents = 0;
    for (unsigned int j = blockIdx.x * 256 + threadIdx.x; j < cnt; j += gridDim.x * 256) {
        const unsigned int i = queue[j];
        const double v = fabs(nu[i]), z = x[i];
        Solved s = plain_solve(v, z, L, Lq, rule_tab(), s_tab);
        const double S = sum_mixed(v, z, s.p, s.A, s_tab);
        out[i] = assemble_k(z, s.delta, s.p.h * S, result);
        nodes += (unsigned long long)(s.p.N + 1);
        ents += 1;
    }
    if (stats) {
        unsigned long long c[2] = {ents, nodes};
        block_stats(stats, c, 2);
    }
}

// ---------------------------------------------------------------------------
// Matern, learned form: the MLP is tabulated once per launch over log10 x on
// kTableSize points of the training box at the launch's nu, and each interval
// between two points gets the quadrature plan of the union of their predictions
// (k_matern_plans). An entry takes its interval's plan; entries that fail the
// acceptance checks are marked and recomputed by k_matern_fallback.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_matern_table(MlpDev M, float nu, float* __restrict__ table)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const float lx = M.lx_lo + (M.lx_hi - M.lx_lo) * (float)min(i, kTableSize - 1) / (float)(kTableSize - 1);
    float y0, y1, y2;
    mlp_wave(M, (lx - M.cx) * M.isx, (nu - M.cnu) * M.isnu, y0, y1, y2);
    if (i < kTableSize) {
        table[4 * i] = y0;
        table[4 * i + 1] = y1;
        table[4 * i + 2] = y2;
        table[4 * i + 3] = 0.0f;
    }
}

// The Matern window table filled by the plain solver at the same points.
__global__ __launch_bounds__(256) void k_matern_table_solver(MlpDev M, float nu, double L, double Lq,
                                                             float* __restrict__ table)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kTableSize) return;
    const float lx = M.lx_lo + (M.lx_hi - M.lx_lo) * (float)i / (float)(kTableSize - 1);
    float y0, y1, y2;
    solver_prediction(M, lx, nu, L, Lq, y0, y1, y2);
    table[4 * i] = y0;
    table[4 * i + 1] = y1;
    table[4 * i + 2] = y2;
    table[4 * i + 3] = 0.0f;
}

// Quadrature plans of the Matern table's cells (between rows k and k + 1) at the
// launch's nu and node target, one lane per cell: the union of the two rows'
// windows with the model's margins, the node count raised to the strip-bound floor
// at the cell's larger x (the floor falls with x, so it holds over the cell) and then
// to N + 1 a multiple of four, and the whole walk set-up, nu and sigma^2 included.
// The walk is biased by 2^eb, eb = B0 - z B1 (log2 of the term at the node m_pk of
// the largest term at the interval's middle, relative to node 0: B0 = nu m_pk h
// log2 e, B1 = (cosh t_pk - cosh t_lo) log2 e). With zl = z log2 e, the log2 of the
// prefactor times sigma^2 h, divided by that bias, is
//   y = A2 + nu log2(z / z_k) - zl cosh t_pk,
//   A2 = (pref + ln(sigma^2 h) + nu ln z_k + nu t_lo - ln 2) log2 e + B0,
// and with y = kq + f (kq an integer) node 0's exponent is f - eb = A2 + nu log2(z /
// z_k) - B0 - kq - zl cosh t_lo. One 96-byte record per interval (kMaternRecBytes):
//   [0] float4  t_lo, P_0 = e^(-2 nu t_lo), rho = e^(-2 nu h) (FP32), N (int; -1: no plan)
//   [1] double2 cosh t_lo, cosh(t_lo + h)
//   [2] double2 2 cosh h, b2 = nu h log2 e
//   [3] double2 A2, ln 2 / z_k
//   [4] double2 cosh t_pk, B0
//   [5]         rho (FP64), h (FP32), raised (int): read off the main path only
// t_lo is rounded to FP32 first, so that every field describes the same window.
// ln sigma^2 is folded in where sigma^2 is finite and positive; the caller applies
// sigma^2 = 0 or +inf itself.
__global__ __launch_bounds__(256) void k_matern_plans(MlpDev M, double nu, double Lq, double pref, double lsig,
                                                      const float* __restrict__ table, float4_t* __restrict__ rec)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= kTableSize - 1) return;
    const float* t0 = table + 4 * k;
    const float* t1 = t0 + 4;
    const double dlx = ((double)M.lx_hi - (double)M.lx_lo) / (kTableSize - 1);
    const double lxm = (double)M.lx_lo + (double)(k + 1) * dlx;
    double tlo, thi;
    int N;
    bool raised;
    decode_window(M, fminf(t0[0], t1[0]), fmaxf(t0[1], t1[1]), fmaxf(t0[2], t1[2]), nu, exp10(lxm), Lq, tlo, thi,
                  N, raised);
    tlo = (double)(float)tlo;
    // N + 1 raised to a multiple of four (a finer step on the same window), so that
    // the kernel's walk runs whole groups of four nodes; N >= kNodeMin gives N >= 7
    if (N >= 0) N = ((N + 4) & ~3) - 1;
    const bool valid = thi > tlo && isfinite(thi) && N >= 7 && N <= kNodeMax;
    double h = 0.0, c0 = 0.0, c1 = 0.0, kappa = 0.0, rho = 0.0, b2 = 0.0, A2 = 0.0, izk = 0.0, chpk = 0.0, B0 = 0.0;
    float P0 = 0.0f;
    if (valid) {
        const double* T = rule_tab().tab;
        h = (thi - tlo) * (double)__builtin_amdgcn_rcpf((float)N);
        c0 = cosh(tlo);
        c1 = cosh(tlo + h);
        kappa = 2.0 * cosh(h);
        rho = exp_tab(-2.0 * nu * h, T);
        P0 = __expf((float)(-2.0 * nu * tlo));
        b2 = nu * h * kLog2e;
        const double zk = exp10((double)M.lx_lo + (double)k * dlx);
        const double zc = exp10((double)M.lx_lo + ((double)k + 0.5) * dlx);
        int mpk = 0;
        double best = 0.0;
        for (int m = 1; m <= N; ++m) {
            const double d = nu * (double)m * h - zc * (cosh(tlo + (double)m * h) - c0);
            if (d > best) { best = d; mpk = m; }
        }
        B0 = nu * (double)mpk * h * kLog2e;
        chpk = cosh(tlo + (double)mpk * h);
        A2 = (pref + lsig + log(h) + nu * log(zk) + nu * tlo - kLn2) * kLog2e + B0;
        izk = kLn2 / zk;
    }
    float4_t* r = rec + kRecQ * k;
    float4_t q0;
    q0[0] = (float)tlo;
    q0[1] = P0;
    q0[2] = (float)rho;
    q0[3] = __int_as_float(valid ? N : -1);
    r[0] = q0;
    const double2_t q1 = {c0, c1}, q2 = {kappa, b2}, q3 = {A2, izk}, q4 = {chpk, B0};
    *(double2_t*)(r + 1) = q1;
    *(double2_t*)(r + 2) = q2;
    *(double2_t*)(r + 3) = q3;
    *(double2_t*)(r + 4) = q4;
    double2_t q5;
    q5[0] = rho;
    q5[1] = 0.0;
    float4_t q5f = __builtin_bit_cast(float4_t, q5);
    q5f[2] = (float)h;
    q5f[3] = __int_as_float(raised ? 1 : 0);
    r[5] = q5f;
}

// log(1 + u) for |u| <= 0.02 in FP32, by its Taylor series through u^4: the
// truncation is below u^5 / 5 < 7e-10 and the FP32 rounding of u and of the
// series about 2^-24 |u| < 1.2e-9, absolute. The learned Matern kernel multiplies
// it by nu, so an order nu moves C by about nu 2e-9 relative (2e-8 at nu = 10).
__device__ __forceinline__ float log1p_small_f(float u)
{
    float p = fmaf(u, -0.25f, 0.333333333f);
    p = fmaf(p, u, -0.5f);
    p = fmaf(p, u, 1.0f);
    return p * u;
}

struct TileGeomL {
    int64_t n;
    int32_t ts, T, lower;
    int32_t rb_per_tile, cb_per_tile;
};

__host__ __device__ inline int64_t tile_offset_l(int64_t n, int64_t ts, int64_t T, int lower, int64_t I, int64_t J)
{
    int64_t nJ = (J == T - 1) ? n - J * ts : ts;
    if (lower) return ts * (J * n - ts * (J * (J - 1) / 2)) + nJ * (I - J) * ts;
    return J * ts * n + nJ * I * ts;
}

// Tile (I, J) of packed tile p (tiles column by column). Lower: column J starts at
// s(J) = J T - J (J - 1) / 2; the FP32 root of s(J) = p lands within a step or two of
// J (values below 2^34 at ~6e-8 relative; the cancellation in b^2 - 8 p adds a few
// steps only for T in the tens of thousands), and the loops settle it exactly. The
// work is uniform across the wave: scalar integer loops after a handful of FP32
// vector instructions.
__device__ inline void tile_of_l(int64_t p, const TileGeomL& g, int64_t& I, int64_t& J)
{
    int64_t T = g.T;
    if (!g.lower) { J = p / T; I = p - J * T; return; }
    const float b = 2.0f * (float)T + 1.0f;
    int64_t j = (int64_t)((b - __builtin_amdgcn_sqrtf(fmaxf(fmaf(b, b, -8.0f * (float)p), 0.0f))) * 0.5f);
    if (j < 0) j = 0;
    if (j > T - 1) j = T - 1;
    while (j > 0 && j * T - j * (j - 1) / 2 > p) --j;
    while (j + 1 <= T - 1 && (j + 1) * T - (j + 1) * j / 2 <= p) ++j;
    J = j;
    I = J + (p - (J * T - J * (J - 1) / 2));
}

// Sum of a per-lane count over a wave (every lane active), added once to a global
// counter by lane 0.
__device__ inline void wave_count_l(unsigned long long* dst, unsigned int v)
{
    unsigned long long a = v;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0 && a) atomicAdd(dst, a);
}

// Node sum of the learned Matern walk over N + 1 = 4q nodes (q >= 2). Node m's
// term is 2^(d_m) (1 + P_m): d_m = -zl c_m + e_m in log2 units, c_m = cosh t_m by
// the recurrence c_(m+1) = kappa c_m - c_(m-1), e_m advanced by b2 = nu h log2 e,
// and P_m = e^(-2 nu t_m).
// kQf: P is carried in FP32 (P' = rho P) and the term formed as e + e P with one
// rounding. Each step rounds P by 2^-24 relative and rho in FP32 is off by up to
// 2^-24, so P_m is off by m 2^-23 relative, and the term by m 2^-23 P_m / (1 + P_m)
// <= 2^-23 m rho^m <= 2^-23 / (e ln(1 / rho)); with 2 nu h >= 1/2 (rho <= e^-1/2)
// that is below 9e-8. Otherwise Q = 1 + P follows Q' = rho Q + (1 - rho) in FP64
// and is rounded to FP32 once per node.
// Nodes go in groups of four, added pairwise in FP32 (two roundings, <= 1.2e-7 of
// the group, all terms positive); the groups sum in FP64. The trapezoid's end
// weights 1/2 are taken inside the first and last groups (an exact halving and the
// group's own rounding). Returns the sum, with the first two and last two terms.
template <bool kQf>
__device__ inline double matern_node_sum(double zl, double c, double cn, double kappa, double e, double b2, float P,
                                         float rhof, double Q, double rho, double omr, int N, float& e0, float& e1,
                                         float& eprev, float& elast)
{
    auto node = [&]() {
        const double d = fma(-zl, c, e);
        const double c2 = fma(kappa, cn, -c);
        c = cn;
        cn = c2;
        e += b2;
        const float ex = __builtin_amdgcn_exp2f((float)d);
        float t;
        if constexpr (kQf) {
            t = fmaf(ex, P, ex);
            P *= rhof;
        } else {
            t = ex * (float)Q;
            Q = fma(Q, rho, omr);
        }
        return t;
    };
    const float ta = node(), tb = node(), tc = node(), td = node();
    e0 = ta;
    e1 = tb;
    double Sd = (double)(fmaf(ta, 0.5f, tb) + (tc + td));
    // middle groups start at nodes 4, 8, ..., N - 7 (a counter common to the wave)
    const int mlast = N - 7;
    for (int m = 4; m <= mlast; m += 4) {
        const float ua = node(), ub = node(), uc = node(), ud = node();
        Sd += (double)((ua + ub) + (uc + ud));
    }
    const float ua = node(), ub = node(), uc = node(), ud = node();
    eprev = uc;
    elast = ud;
    return Sd + (double)((ua + ub) + fmaf(ud, 0.5f, uc));
}

// Learned Matern. Wave w of the call (the workgroup's index (tile x column blocks +
// column block) x row blocks + row block, times 4, plus the wave in the group)
// covers 64 rows of a tile column block and kMlCols of its columns. An
// entry the learned form rejects is written as NaN and bit w of the call's wave
// bitmap is set; k_matern_fallback then recomputes the NaN entries of the marked
// waves with the mixed form. Keeping the fallback out of this kernel keeps its
// registers (and so its occupancy) those of the learned pass. kStats: the
// statistics variant (lanes past a ragged tile's last row stay in the wave, idle,
// so that the wave can sum its counts).
// kb = log2(e) / beta; an entry's interval is fpos = fa log2(zl) + fb in
// [0, kTableSize - 1] (zl = z log2 e); sig_mul: sigma^2 where it is 0 or +inf (the
// records then carry no ln sigma^2), else 1 and unused.
template <typename OutT, bool kStats>
__global__ __launch_bounds__(256, 8) void k_matern_learned(const float4_t* __restrict__ rec,
                                                        const double* __restrict__ lx_, const double* __restrict__ ly_,
                                                        TileGeomL g, int64_t tile_base, double sigma2, double kb,
                                                        float fa, float fb, int nu_ok, double nu, double sig_mul,
                                                        unsigned int* __restrict__ bitmap, OutT* __restrict__ out,
                                                        unsigned long long* __restrict__ stats)
{
    constexpr int kColsPerWave = kMlCols, kColsPerGroup = kMlGroupCols;
    // grid: (row block, column block, tile of the launch)
    const unsigned wg_per_tile = (unsigned)g.rb_per_tile * (unsigned)g.cb_per_tile;
    const int64_t p = tile_base + (int64_t)blockIdx.z;
    const int rb = (int)blockIdx.x, cb = (int)blockIdx.y;
    int64_t I, J;
    tile_of_l(p, g, I, J);
    const int64_t mI = min((int64_t)g.ts, g.n - I * g.ts);
    const int64_t nJ = min((int64_t)g.ts, g.n - J * g.ts);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t il = (int64_t)rb * 64 + lane;
    const int64_t jl0 = (int64_t)cb * kColsPerGroup + (int64_t)wave * kColsPerWave;
    const bool row_ok = il < mI;
    // the statistics variant keeps every wave to the end for its block-wide sums
    if (!kStats && (jl0 >= nJ || !row_ok)) return;
    const int64_t base = tile_offset_l(g.n, g.ts, g.T, g.lower, I, J);
    const int64_t ilr = row_ok ? il : 0;
    const double xi = lx_[I * g.ts + ilr], yi = ly_[I * g.ts + ilr];
    // the row point is waited for here, once: a wait for it inside the column loop
    // would also wait for the previous column's store
    asm volatile("" ::"v"(xi), "v"(yi));
    const int cend = (kStats && (!row_ok || jl0 >= nJ)) ? 0 : (int)min((int64_t)kColsPerWave, nJ - jl0);
    const double* __restrict__ xc = lx_ + J * g.ts + jl0;      // this wave's columns
    const double* __restrict__ yc = ly_ + J * g.ts + jl0;
    const double nul2e = nu * kLog2e;
    bool rejected = false;
    unsigned int c_ent = 0, c_nodes = 0, c_range = 0, c_tail = 0, c_nonfin = 0, c_raised = 0;
    unsigned int col_nodes[kColsPerWave] = {};      // statistics: nodes per column walked
    double xj = 0.0, yj = 0.0;
    if (cend > 0) {
        xj = xc[0];
        yj = yc[0];
    }
    for (int c = 0; c < cend; ++c) {
        // the next column's point is read one column ahead
        const int cnext = c + 1 < cend ? c + 1 : c;
        const double xjn = xc[cnext], yjn = yc[cnext];
        const double dx = xj - xi, dy = yj - yi;
        xj = xjn;
        yj = yjn;
        const double r2 = dx * dx + dy * dy;
        OutT val = (OutT)sigma2;
        if (r2 != 0.0) {
            // r from the hardware reciprocal square root (about 5e-8 relative) and one
            // Goldschmidt step, which squares that error (measured: <= 4.1e-15 relative
            // over r^2 in [1e-40, 1e4]). An r^2 below the normal range can give no
            // finite zl (a flushed reciprocal square root), which fails the range test:
            // the fallback recomputes that entry.
            const double yr = __builtin_amdgcn_rsq(r2);
            const double s0 = r2 * yr, h0 = 0.5 * yr;
            const double zl = fma(s0, fma(-s0, h0, 0.5), s0) * kb;
            const float fpos = fmaf(__builtin_amdgcn_logf((float)zl), fa, fb);
            bool ok = nu_ok && fpos >= 0.0f && fpos <= (float)(kTableSize - 1);
            if (kStats && !ok) c_range += 1;
            double Sd = 0.0, kq = 0.0;
            float S = 0.0f;
            if (ok) {
                // the whole record is read at once (an interval without a plan, N < 0,
                // holds zeros and is walked harmlessly, then rejected)
                const unsigned k0 = min((unsigned)fpos, (unsigned)(kTableSize - 2));
                const float4_t* R = rec + __umul24(k0, (unsigned)kRecQ);
                const float4_t q0 = R[0];
                const double2_t q1 = *(const double2_t*)(R + 1), q2 = *(const double2_t*)(R + 2);
                const double2_t q3 = *(const double2_t*)(R + 3), q4 = *(const double2_t*)(R + 4);
                const int N = __float_as_int(q0[3]);
                if (kStats) c_raised += (unsigned int)(__float_as_int(R[5][3]) & 1);
                // y = A2 + nu log2(z / z_k) - zl cosh t_pk, y = kq + f; node 0's exponent
                // A2 + nu log2(z / z_k) - B0 - kq - zl cosh t_lo (k_matern_plans).
                // log(z / z_k) = log1p(u), |u| < 0.016.
                const double w = fma(nul2e, (double)log1p_small_f((float)fma(zl, q3[1], -1.0)), q3[0]);
                kq = rint(fma(-zl, q4[0], w));
                const double e_init = (w - q4[1]) - kq;
                float e0, e1, eprev, elast;
                if (q2[1] >= 0.25 * kLog2e) {       // b2 = nu h log2 e: 2 nu h >= 1/2
                    Sd = matern_node_sum<true>(zl, q1[0], q1[1], q2[0], e_init, q2[1], q0[1], q0[2], 0.0, 0.0, 0.0,
                                               N, e0, e1, eprev, elast);
                } else {
                    const double rho = *(const double*)(R + 5);
                    Sd = matern_node_sum<false>(zl, q1[0], q1[1], q2[0], e_init, q2[1], 0.0f, 0.0f,
                                                1.0 + (double)q0[1], rho, 1.0 - rho, N, e0, e1, eprev, elast);
                }
                S = (float)Sd;
                int reason = 0;
                if (N < 0 || !(Sd > 0.0) || !isfinite(Sd)) {
                    reason = BK_STAT_FB_NONFINITE;
                } else if (!right_tail_ok(eprev, elast, S)) {
                    reason = BK_STAT_FB_TAIL;
                } else if (q0[0] > 0.0f) {
                    // Delta = nu t_lo - ln 2 - z (cosh t_lo - 1), without the bias
                    const double z = zl * kLn2, tlo = (double)q0[0];
                    const float D = (float)(fma(nu, tlo, -kLn2) - z * (q1[0] - 1.0));
                    if (!left_tail_ok(z, nu, q0[0], R[5][2], e0, e1, D, S)) reason = BK_STAT_FB_TAIL;
                }
                ok = reason == 0;
                if (kStats) {
                    if (N >= 0) {
                        c_ent += 1;
                        c_nodes += (unsigned int)(N + 1);
                        col_nodes[c] = (unsigned int)(N + 1);
                        c_tail += reason == BK_STAT_FB_TAIL ? 1u : 0u;
                    }
                    c_nonfin += reason == BK_STAT_FB_NONFINITE ? 1u : 0u;
                }
            }
            if (ok) {
                // Sd lies within a few powers of two of 1 (the terms are taken relative
                // to the largest), so the FP32 scaling is exact unless the value itself
                // leaves the FP32 range
                if constexpr (sizeof(OutT) == sizeof(float))
                    val = ldexpf(S, (int)kq);
                else
                    val = ldexp(Sd, (int)kq);
                if (sig_mul != 1.0) val *= (OutT)sig_mul;
            } else {
                val = (OutT)__builtin_nan("");
                rejected = true;
            }
        }
        out[base + il + (jl0 + c) * mI] = val;
    }
    // lane 0 is active whenever any lane of the wave is (rows grow with the lane)
    if (__ballot(rejected) != 0ull && lane == 0) {
        const int64_t blk = p * (int64_t)wg_per_tile + (int64_t)cb * g.rb_per_tile + rb;
        const int64_t w = (blk << 2) + wave;
        atomicOr(bitmap + (w >> 5), 1u << (unsigned)(w & 31));
    }
    if (kStats) {
        // one atomic per counter per workgroup (per-wave atomics on the same eight
        // addresses serialise in L2 over millions of waves)
        unsigned int slots = 0;
#pragma unroll
        for (int c = 0; c < kColsPerWave; ++c) {
            unsigned int v = col_nodes[c];
            for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned int)__shfl_xor((int)v, o, 64));
            slots += 64u * v;
        }
        unsigned long long cnt[8];
        cnt[BK_STAT_ENTRIES] = c_ent;
        cnt[BK_STAT_NODES] = c_nodes;
        cnt[BK_STAT_FB_RANGE] = c_range;
        cnt[BK_STAT_FB_TAIL] = c_tail;
        cnt[BK_STAT_NODE_RAISED] = c_raised;
        cnt[BK_STAT_FB_NONFINITE] = c_nonfin;
        cnt[BK_STAT_FB_NODES] = 0;
        cnt[BK_STAT_LANE_SLOTS] = lane == 0 ? slots : 0u;
        block_stats_w(stats, cnt, 8, 4);
    }
}

// Fallback of the learned Matern kernel. Each wave scans 64 words of the wave
// bitmap at a time (grid-stride), and for every marked wave re-derives its rows and
// columns and recomputes the NaN entries with the mixed form (FP64 solve, FP32
// node terms). The marked waves are few, so the scan is the bulk of the work.
template <typename OutT>
__global__ __launch_bounds__(256) void k_matern_fallback(const double* __restrict__ lx_, const double* __restrict__ ly_,
                                                         TileGeomL g, double sigma2, double inv_beta, double nu,
                                                         double pref, double L, double Lq,
                                                         const unsigned int* __restrict__ bitmap, int64_t nwords,
                                                         OutT* __restrict__ out, unsigned long long* __restrict__ stats)
{
    constexpr int kColsPerWave = kMlCols, kColsPerGroup = kMlGroupCols;
    __shared__ double s_tab[kTabLen];
    stage_tab(s_tab);
    const int lane = threadIdx.x & 63;
    const int64_t wg_per_tile = (int64_t)g.rb_per_tile * g.cb_per_tile;
    unsigned int ents = 0, nodes = 0;
    const int64_t stride = (int64_t)gridDim.x * 4 * 64;
    for (int64_t w0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64; w0 < nwords; w0 += stride) {
        const unsigned int word = (w0 + lane < nwords) ? bitmap[w0 + lane] : 0u;
        unsigned long long live = __ballot(word != 0u);
        while (live) {                                   // wave-uniform loops
            const int l = __builtin_ctzll(live);
            live &= live - 1;
            unsigned int bits = (unsigned int)__shfl((int)word, l, 64);
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1;
                const int64_t id = (w0 + l) * 32 + b;    // the marked wave
                const int64_t blk = id >> 2;
                const int wave = (int)(id & 3);
                const int64_t p = blk / wg_per_tile;
                const int64_t local = blk - p * wg_per_tile;
                const int rb = (int)(local % g.rb_per_tile), cb = (int)(local / g.rb_per_tile);
                int64_t I, J;
                tile_of_l(p, g, I, J);
                const int64_t mI = min((int64_t)g.ts, g.n - I * g.ts);
                const int64_t nJ = min((int64_t)g.ts, g.n - J * g.ts);
                const int64_t il = (int64_t)rb * 64 + lane;
                const int64_t jl0 = (int64_t)cb * kColsPerGroup + (int64_t)wave * kColsPerWave;
                if (il >= mI || jl0 >= nJ) continue;
                const int64_t base = tile_offset_l(g.n, g.ts, g.T, g.lower, I, J);
                const double xi = lx_[I * g.ts + il], yi = ly_[I * g.ts + il];
                const int cend = (int)min((int64_t)kColsPerWave, nJ - jl0);
                for (int c = 0; c < cend; ++c) {
                    const int64_t o = base + il + (jl0 + c) * mI;
                    if (!isnan((double)out[o])) continue;
                    const int64_t jl = jl0 + c;
                    const double dx = lx_[J * g.ts + jl] - xi, dy = ly_[J * g.ts + jl] - yi;
                    const double z = sqrt(dx * dx + dy * dy) * inv_beta;
                    const Solved s = plain_solve(nu, z, L, Lq, rule_tab(), s_tab);
                    const double hs = s.p.h * sum_mixed(nu, z, s.p, s.A, s_tab);
                    out[o] = (OutT)(sigma2 * exp(pref + nu * log(z) + (s.delta - z)) * hs);
                    ents += 1;
                    nodes += (unsigned int)(s.p.N + 1);
                }
            }
        }
    }
    if (stats) {
        wave_count_l(stats + BK_STAT_ENTRIES, ents);
        wave_count_l(stats + BK_STAT_NODES, nodes);
        wave_count_l(stats + BK_STAT_FB_NODES, nodes);
    }
}

// Clears n 32-bit words (a fill kernel rather than a memset node, so that a
// captured graph replays it correctly).
__global__ __launch_bounds__(256) void k_fill_u32(unsigned int* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Training kernels (FP32, one lane per sample)
// ---------------------------------------------------------------------------
// Targets and inputs from the plain-solver window: u = normalised (log10 x, nu),
// target = (t_lo / st, t_hi / st, N / sn).
__global__ __launch_bounds__(256) void k_make_targets(const double* __restrict__ nu, const double* __restrict__ x,
                                                      const double* __restrict__ tlo, const double* __restrict__ thi,
                                                      const int32_t* __restrict__ nodes, int64_t n, float cx, float sx,
                                                      float cnu, float snu, float st, float sn,
                                                      float* __restrict__ u, float* __restrict__ tgt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    u[2 * i] = ((float)log10(x[i]) - cx) / sx;
    u[2 * i + 1] = ((float)fabs(nu[i]) - cnu) / snu;
    tgt[3 * i] = (float)tlo[i] / st;
    tgt[3 * i + 1] = (float)thi[i] / st;
    tgt[3 * i + 2] = (float)nodes[i] / sn;
}

// Training gradient of one tile of kTrainTile = 64 samples per 256-lane workgroup
// (FP32 on the vector ALU: on gfx950 the FP32 matrix cores have the vector units'
// peak, and these 64 x 64 x 64 products are too small to gain from them). The
// tile's activations and back-propagated gradients live in LDS, one row per
// sample; every 64 x 64 product is split over the 256 lanes, 16 outputs each
// (lane t: sample or unit t / 4, units or columns 16 (t % 4) ... + 15), so each
// lane runs a quarter of one sample's work instead of a whole sample:
//   h1 = relu(W1 u + b1), z2 = W2 h1 + b2, h2 = relu(z2), y = W3 h2 + b3,
//   gy = dL/dy, g2 = [z2 > 0] W3^T gy, g1 = [h1 > 0] W2^T g2,
//   dW2 = sum_s g2 h1^T, dW1 = sum_s g1 u^T, dW3 = sum_s gy h2^T, biases likewise.
// The tile's gradient (kNParam floats) goes to its row of `partial`; k_grad_reduce
// sums the rows in a fixed order. Sample b of the batch is row perm(b) =
// (pa * (start + b) + pb) mod n of the data (n = 0: row b); samples past B add
// nothing (their gy is zero).
constexpr int kTrainTile = 64;
constexpr int kTrainThreads = 256;
constexpr int kTrainLd = kH + 1;          // padded LDS rows

__device__ __forceinline__ uint64_t train_row(int64_t start, int64_t b, int64_t n, uint64_t pa, uint64_t pb)
{
    uint64_t row = (uint64_t)(start + b);
    if (n > 0) row = (pa * row + pb) % (uint64_t)n;      // pa, row < n < 2^31: no overflow
    return row;
}

__global__ __launch_bounds__(kTrainThreads) void k_train_tile(const float* __restrict__ P, const float* __restrict__ U,
                                                              const float* __restrict__ T, const float* __restrict__ tau,
                                                              int64_t B, int64_t n, uint64_t pa, uint64_t pb,
                                                              int64_t start, float* __restrict__ partial,
                                                              float* __restrict__ loss)
{
    __shared__ float sP[kNParam];
    __shared__ float sW2T[kH * kH];           // W2 transposed (rows of W2^T for g1)
    __shared__ float sH1[kTrainTile * kTrainLd], sH2[kTrainTile * kTrainLd];
    __shared__ float sG1[kTrainTile * kTrainLd], sG2[kTrainTile * kTrainLd];
    __shared__ float sU[kTrainTile * 2], sGy[kTrainTile * 4];
    const int t = threadIdx.x;
    for (int k = t; k < kNParam; k += kTrainThreads) sP[k] = P[k];
    for (int k = t; k < kH * kH; k += kTrainThreads) sW2T[(k % kH) * kH + k / kH] = P[kOffW2 + k];
    const int64_t tile0 = (int64_t)blockIdx.x * kTrainTile;
    const int r = t >> 2, q0 = 16 * (t & 3);  // lane's sample (or unit) r and its 16 columns
    const bool live_r = tile0 + r < B;
    float u0 = 0.0f, u1 = 0.0f;
    if (live_r) {
        const uint64_t row = train_row(start, tile0 + r, n, pa, pb);
        u0 = U[2 * row];
        u1 = U[2 * row + 1];
    }
    if ((t & 3) == 0) {
        sU[2 * r] = u0;
        sU[2 * r + 1] = u1;
    }
    __syncthreads();
    // h1 (sample r, units q0..q0+15)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int j = q0 + k;
        sH1[r * kTrainLd + j] = fmaxf(fmaf(sP[kOffW1 + 2 * j], u0, fmaf(sP[kOffW1 + 2 * j + 1], u1, sP[kOffB1 + j])), 0.0f);
    }
    __syncthreads();
    {   // h2 = relu(W2 h1 + b2)
        float h[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j) h[j] = sH1[r * kTrainLd + j];
        for (int k = 0; k < 16; ++k) {
            const int i = q0 + k;
            float z = sP[kOffB2 + i];
#pragma unroll
            for (int j = 0; j < kH; ++j) z = fmaf(sP[kOffW2 + i * kH + j], h[j], z);
            sH2[r * kTrainLd + i] = fmaxf(z, 0.0f);   // h2 > 0 iff z2 > 0
        }
    }
    __syncthreads();
    // output, loss and gy: lanes 0..191, sample t / 3, output t % 3
    float l = 0.0f;
    if (t < 3 * kTrainTile) {
        const int s = t / 3, o = t - 3 * (t / 3);
        float gy = 0.0f;
        if (tile0 + s < B) {
            float y = sP[kOffB3 + o];
#pragma unroll 16
            for (int i = 0; i < kH; ++i) y = fmaf(sP[kOffW3 + o * kH + i], sH2[s * kTrainLd + i], y);
            const uint64_t row = train_row(start, tile0 + s, n, pa, pb);
            const float e = T[3 * row + o] - y;
            const float w = e < 0.0f ? 1.0f - tau[o] : tau[o];
            l = w * e * e;
            gy = -2.0f * w * e / (float)B;
        }
        sGy[4 * s + o] = gy;
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((t & 63) == 0 && t < 3 * kTrainTile) atomicAdd(loss, l / (float)B);
    __syncthreads();
    // g2 = [h2 > 0] W3^T gy (sample r, units q0..q0+15)
    {
        const float gy0 = sGy[4 * r], gy1 = sGy[4 * r + 1], gy2 = sGy[4 * r + 2];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int i = q0 + k;
            const float g = sP[kOffW3 + i] * gy0 + sP[kOffW3 + kH + i] * gy1 + sP[kOffW3 + 2 * kH + i] * gy2;
            sG2[r * kTrainLd + i] = sH2[r * kTrainLd + i] > 0.0f ? g : 0.0f;
        }
    }
    __syncthreads();
    {   // g1 = [h1 > 0] W2^T g2 (sample r, units q0..q0+15)
        float g2[kH];
#pragma unroll
        for (int i = 0; i < kH; ++i) g2[i] = sG2[r * kTrainLd + i];
        for (int k = 0; k < 16; ++k) {
            const int j = q0 + k;
            float g = 0.0f;
#pragma unroll
            for (int i = 0; i < kH; ++i) g = fmaf(sW2T[j * kH + i], g2[i], g);
            sG1[r * kTrainLd + j] = sH1[r * kTrainLd + j] > 0.0f ? g : 0.0f;
        }
    }
    __syncthreads();
    float* out = partial + (int64_t)blockIdx.x * kNParam;
    {   // dW2 row r, columns q0..q0+15, and db2[r]
        float acc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0f;
        float db = 0.0f;
        for (int s = 0; s < kTrainTile; ++s) {
            const float g = sG2[s * kTrainLd + r];
            db += g;
#pragma unroll
            for (int k = 0; k < 16; ++k) acc[k] = fmaf(g, sH1[s * kTrainLd + q0 + k], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) out[kOffW2 + r * kH + q0 + k] = acc[k];
        if ((t & 3) == 0) out[kOffB2 + r] = db;
    }
    // dW1 and db1: lanes 0..191 (unit t / 3; column 0, 1 or the bias)
    if (t < 3 * kH) {
        const int j = t / 3, c = t - 3 * (t / 3);
        float acc = 0.0f;
        for (int s = 0; s < kTrainTile; ++s) acc = fmaf(sG1[s * kTrainLd + j], c < 2 ? sU[2 * s + (c & 1)] : 1.0f, acc);
        if (c < 2) out[kOffW1 + 2 * j + c] = acc;
        else out[kOffB1 + j] = acc;
    } else {
        // dW3 and db3: lanes 192..255 (unit t - 192, all three outputs)
        const int i = t - 3 * kH;
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        for (int s = 0; s < kTrainTile; ++s) {
            const float h = sH2[s * kTrainLd + i];
            a0 = fmaf(sGy[4 * s], h, a0);
            a1 = fmaf(sGy[4 * s + 1], h, a1);
            a2 = fmaf(sGy[4 * s + 2], h, a2);
        }
        out[kOffW3 + i] = a0;
        out[kOffW3 + kH + i] = a1;
        out[kOffW3 + 2 * kH + i] = a2;
        if (i < 3) {
            float d = 0.0f;
            for (int s = 0; s < kTrainTile; ++s) d += sGy[4 * s + i];
            out[kOffB3 + i] = d;
        }
    }
}

// Training step after k_train_tile: the batch gradient (the tiles' rows summed in
// tile order, as k_grad_reduce) and the Adam update of k_adam, in one launch.
__global__ __launch_bounds__(256) void k_grad_adam(const float* __restrict__ partial, int tiles, float* __restrict__ p,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= kNParam) return;
    float gi = 0.0f;
    for (int t = 0; t < tiles; ++t) gi += partial[(int64_t)t * kNParam + k];
    const float mi = b1 * m[k] + (1.0f - b1) * gi;
    const float vi = b2 * v[k] + (1.0f - b2) * gi * gi;
    m[k] = mi;
    v[k] = vi;
    p[k] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Batch gradient: the sum of the tiles' rows of `partial`, in tile order.
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ partial, int tiles,
                                                     float* __restrict__ grad)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= kNParam) return;
    float s = 0.0f;
    for (int t = 0; t < tiles; ++t) s += partial[(int64_t)t * kNParam + k];
    grad[k] = s;
}

__global__ void k_zero_f32(float* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Residuals of the inference-path predictions against the targets (for margins):
// r[0] = pred t_lo - t_lo, r[1] = t_hi - pred t_hi, r[2] = N / pred N - 1 (all in absolute units).
__global__ __launch_bounds__(256) void k_residuals(MlpDev M, const float* __restrict__ U, const float* __restrict__ T,
                                                   int64_t n, float* __restrict__ res)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float u0 = 0.0f, u1 = 0.0f;
    if (i < n) { u0 = U[2 * i]; u1 = U[2 * i + 1]; }
    float y0, y1, y2;
    mlp_wave(M, u0, u1, y0, y1, y2);
    if (i < n) {
        res[3 * i] = (y0 - T[3 * i]) * M.st;
        res[3 * i + 1] = (T[3 * i + 1] - y1) * M.st;
        res[3 * i + 2] = T[3 * i + 2] / fmaxf(y2, 1e-3f) - 1.0f;
    }
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
// FP16 operand pack from the FP32 master parameters (host arrays).
// Hidden unit at position k = 8q + j of K chunk c of the 16x16x32 operands (see the
// inference comment above).
static int chunk_unit(int c, int q, int j) { return 16 * (2 * c + (j >= 4 ? 1 : 0)) + 4 * q + (j & 3); }

static void pack_weights(const float* P, std::vector<_Float16>& pack, std::vector<float>& bias)
{
    pack.assign((size_t)24 * 64 * 4, (_Float16)0.0f);
    _Float16* A1 = pack.data();                 // [4 mt][64][4]
    _Float16* A2 = pack.data() + 4 * 64 * 4;    // [4 mt][2 c][64][8]
    _Float16* A3 = pack.data() + 20 * 64 * 4;   // [2 c][64][8]
    for (int mt = 0; mt < 4; ++mt)
        for (int lane = 0; lane < 64; ++lane) {
            const int r = lane & 15, q = lane >> 4, j = 16 * mt + r;
            _Float16* a1 = A1 + ((size_t)mt * 64 + lane) * 4;
            if (q == 0) {
                a1[0] = (_Float16)P[kOffW1 + 2 * j];
                a1[1] = (_Float16)P[kOffW1 + 2 * j + 1];
                a1[2] = (_Float16)P[kOffB1 + j];
            }
            for (int c = 0; c < 2; ++c) {
                _Float16* a2 = A2 + ((size_t)(mt * 2 + c) * 64 + lane) * 8;
                for (int jj = 0; jj < 8; ++jj) a2[jj] = (_Float16)P[kOffW2 + j * kH + chunk_unit(c, q, jj)];
            }
        }
    for (int c = 0; c < 2; ++c)
        for (int lane = 0; lane < 64; ++lane) {
            const int r = lane & 15, q = lane >> 4;
            _Float16* a3 = A3 + ((size_t)c * 64 + lane) * 8;
            if (r < 3)
                for (int jj = 0; jj < 8; ++jj) a3[jj] = (_Float16)P[kOffW3 + r * kH + chunk_unit(c, q, jj)];
        }
    bias.assign(68, 0.0f);
    for (int j = 0; j < kH; ++j) bias[j] = P[kOffB2 + j];
    for (int o = 0; o < 3; ++o) bias[64 + o] = P[kOffB3 + o];
}

static void model_free(bk_model* m)
{
    void* bufs[] = {m->params, m->pack, m->bias, m->cells, m->plan_a, m->plan_b};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    m->params = nullptr;
    m->pack = nullptr;
    m->bias = nullptr;
    m->cells = nullptr;
    m->plan_a = nullptr;
    m->plan_b = nullptr;
}

// Device buffers of a model; on any failure everything is released again, so a
// model is either fully allocated or holds nothing.
static int model_alloc(bk_model* m)
{
    if (m->params) return BK_OK;
    if (hipGetDevice(&m->device) != hipSuccess) return BK_EHIP;
    const bool ok = hipMalloc((void**)&m->params, sizeof(float) * kNParam) == hipSuccess &&
                    hipMalloc((void**)&m->pack, sizeof(_Float16) * 24 * 64 * 4) == hipSuccess &&
                    hipMalloc((void**)&m->bias, sizeof(float) * 68) == hipSuccess &&
                    hipMalloc((void**)&m->cells, sizeof(float) * 4 * kCells) == hipSuccess &&
                    hipMalloc((void**)&m->plan_a, sizeof(float) * 4 * kCells) == hipSuccess &&
                    hipMalloc((void**)&m->plan_b, sizeof(double) * 4 * kCells) == hipSuccess;
    if (!ok) {
        model_free(m);
        return BK_ENOMEM;
    }
    return BK_OK;
}

// Prediction cells and their quadrature plans (at the default node target) for the
// current parameters, normalisation, box and margins (synchronous, on the null
// stream; nothing to do before the parameters exist).
static int model_cells(bk_model* m)
{
    if (!m->params) return BK_OK;
    m->plan_Lq = -1.0;
    int st = m->table_source == BK_TABLE_SOLVER
                 ? launch(k_cell_table_solver, dim3((kCells + 255) / 256), dim3(256), nullptr, make_dev(m),
                          m->train_L[0], m->train_L[1], reinterpret_cast<float4_t*>(m->cells))
                 : launch(k_cell_table, dim3((kCells + 255) / 256), dim3(256), nullptr, make_dev(m),
                          reinterpret_cast<float4_t*>(m->cells));
    if (st == BK_OK)
        st = launch(k_cell_plans, dim3((kCells + 255) / 256), dim3(256), nullptr, make_dev(m), kDefaultLqMixed,
                    reinterpret_cast<float4_t*>(m->plan_a), reinterpret_cast<double4_t*>(m->plan_b));
    if (st != BK_OK) return st;
    st = hip_ok(hipStreamSynchronize(nullptr));
    if (st == BK_OK) m->plan_Lq = kDefaultLqMixed;
    return st;
}

// Upload host parameters: master copy and inference pack, then the prediction
// cells (synchronous).
static int model_upload(bk_model* m, const float* hostP)
{
    int st = model_alloc(m);
    if (st) return st;
    std::vector<_Float16> pack;
    std::vector<float> bias;
    pack_weights(hostP, pack, bias);
    if (hipMemcpy(m->params, hostP, sizeof(float) * kNParam, hipMemcpyHostToDevice) != hipSuccess) return BK_EHIP;
    if (hipMemcpy(m->pack, pack.data(), sizeof(_Float16) * pack.size(), hipMemcpyHostToDevice) != hipSuccess) return BK_EHIP;
    if (hipMemcpy(m->bias, bias.data(), sizeof(float) * bias.size(), hipMemcpyHostToDevice) != hipSuccess) return BK_EHIP;
    return model_cells(m);
}

// Per-tile gradient rows of one batch.
static size_t grad_scratch_floats(int64_t B) { return (size_t)((B + kTrainTile - 1) / kTrainTile) * kNParam; }

static int launch_grad(const float* params, const float* u, const float* tgt, const float* tau, int64_t B,
                       int64_t n, uint64_t pa, uint64_t pb, int64_t start, float* grad, float* loss, float* scr,
                       hipStream_t s)
{
    const unsigned tiles = (unsigned)((B + kTrainTile - 1) / kTrainTile);
    const int st = launch(k_train_tile, dim3(tiles), dim3(kTrainThreads), s, params, u, tgt, tau, B, n, pa, pb, start,
                          scr, loss);
    if (st != BK_OK) return st;
    return launch(k_grad_reduce, dim3((kNParam + 255) / 256), dim3(256), s, (const float*)scr, (int)tiles, grad);
}

}  // namespace bk

using namespace bk;

// ---------------------------------------------------------------------------
// Learned evaluation entry points (called from bk_kernels.hip)
// ---------------------------------------------------------------------------
namespace bk {

int bk_besselk_learned(const double* nu, const double* x, double* out, int64_t n, const bk_params* prm, double L,
                       double Lq, hipStream_t stream)
{
    const bk_model* m = prm->model;
    if (!m || !m->params || !m->trained) return BK_ENOMODEL;
    if (!prm->workspace || prm->workspace_bytes < bk_workspace_bytes(n)) return BK_ENOMEM;
    if (n >= (int64_t)0xffffffffLL) return BK_EINVAL;
    unsigned int* qcount = (unsigned int*)prm->workspace;
    unsigned int* queue = (unsigned int*)((char*)prm->workspace + 256);
    const MlpDev M = make_dev(m);
    int st = launch(k_zero_u32, dim3(1), dim3(64), stream, qcount);
    if (st != BK_OK) return st;
    const unsigned blocks = (unsigned)((n + kLearnedBlock - 1) / kLearnedBlock);
    if (mark_kernel_event(prm, 0, stream) != hipSuccess) return BK_EHIP;
    st = (m->plan_Lq == Lq)
        ? launch(k_besselk_learned<true>, dim3(blocks), dim3(kLearnedBlock), stream, M, nu, x, out, n, prm->result,
                 Lq, qcount, queue, prm->stats)
        : launch(k_besselk_learned<false>, dim3(blocks), dim3(kLearnedBlock), stream, M, nu, x, out, n, prm->result,
                 Lq, qcount, queue, prm->stats);
    if (st != BK_OK) return st;
    if (mark_kernel_event(prm, 1, stream) != hipSuccess) return BK_EHIP;
    return launch(k_besselk_fallback, dim3(1024), dim3(256), stream, nu, x, out, prm->result, qcount, queue, L, Lq,
                  prm->stats);
}

size_t matern_learned_workspace_bytes(int64_t n, int32_t tile_size, int32_t lower_only)
{
    if (n <= 0 || tile_size <= 0) return 0;
    const int64_t T = (n + tile_size - 1) / tile_size;
    const int64_t ntiles = lower_only ? T * (T + 1) / 2 : T * T;
    const int64_t wg_per_tile = (int64_t)((tile_size + 63) / 64) * ((tile_size + kMlGroupCols - 1) / kMlGroupCols);
    const int64_t words = (ntiles * wg_per_tile * 4 + 31) / 32;
    return kMaternTabBytes + (((size_t)words * 4 + 255) & ~(size_t)255);
}

int bk_matern_learned(const bk_locs* locs, const bk_params* prm, int32_t tile_size, int32_t lower_only, void* out,
                      double L, double Lq, void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    const bk_model* m = prm->model;
    if (!m || !m->params || !m->trained) return BK_ENOMODEL;
    const size_t need = matern_learned_workspace_bytes(locs->n, tile_size, lower_only);
    if (!workspace || workspace_bytes < need) return BK_ENOMEM;
    char* ws = (char*)workspace;
    float* table = (float*)(ws + kMaternTableOff);
    float4_t* rec = (float4_t*)(ws + kMaternRecOff);
    unsigned int* bitmap = (unsigned int*)(ws + kMaternTabBytes);
    const int64_t nwords = (int64_t)((need - kMaternTabBytes) / 4);
    const MlpDev M = make_dev(m);
    const double nu = prm->nu;
    const double pref = (1.0 - nu) * kLn2 - lgamma(nu);
    TileGeomL g;
    g.n = locs->n;
    g.ts = tile_size;
    g.T = (int32_t)((locs->n + tile_size - 1) / tile_size);
    g.lower = lower_only ? 1 : 0;
    g.rb_per_tile = (tile_size + 63) / 64;
    g.cb_per_tile = (tile_size + kMlGroupCols - 1) / kMlGroupCols;
    const int64_t T = g.T;
    const int64_t ntiles = g.lower ? T * (T + 1) / 2 : T * T;
    const int64_t wg_per_tile = (int64_t)g.rb_per_tile * g.cb_per_tile;
    // tiles per launch: below 2^31 work-items and within the grid's third dimension
    const int64_t max_wg = 1LL << 23;
    const int64_t tiles_per_launch = std::min<int64_t>(max_wg / wg_per_tile > 0 ? max_wg / wg_per_tile : 1, 65535);
    // ln sigma^2 goes into the plans where it is finite; sigma^2 = 0 or +inf is
    // applied to each entry instead
    const double sigma2 = prm->sigma2;
    const bool sig_fold = sigma2 > 0.0 && isfinite(sigma2);
    const double lsig = sig_fold ? log(sigma2) : 0.0;
    const double sig_mul = sig_fold ? 1.0 : sigma2;
    const double ib = 1.0 / prm->beta, kb = kLog2e / prm->beta;
    // interval position from log2(zl), zl = z log2 e: (log10 z - lx_lo) (kTableSize - 1) / (lx_hi - lx_lo)
    const double tsc = (double)(kTableSize - 1) / ((double)M.lx_hi - (double)M.lx_lo);
    const float fa = (float)(std::log10(2.0) * tsc);
    const float fb = (float)((-std::log2(kLog2e) * std::log10(2.0) - (double)M.lx_lo) * tsc);
    const int nu_ok = (float)nu >= M.nu_lo && (float)nu <= M.nu_hi ? 1 : 0;
    int st = m->table_source == BK_TABLE_SOLVER
                 ? launch(k_matern_table_solver, dim3((kTableSize + 255) / 256), dim3(256), stream, M, (float)nu,
                          m->train_L[0], m->train_L[1], table)
                 : launch(k_matern_table, dim3((kTableSize + 255) / 256), dim3(256), stream, M, (float)nu, table);
    if (st == BK_OK)
        st = launch(k_matern_plans, dim3((kTableSize + 254) / 256), dim3(256), stream, M, nu, Lq, pref, lsig,
                    (const float*)table, rec);
    if (st == BK_OK)
        st = launch(k_fill_u32, dim3((unsigned)std::min<int64_t>((nwords + 255) / 256, 4096)), dim3(256), stream,
                    bitmap, nwords);
    if (st != BK_OK) return st;
    if (mark_kernel_event(prm, 0, stream) != hipSuccess) return BK_EHIP;
    const bool f32 = prm->out_dtype == BK_OUT_F32;
    for (int64_t t0 = 0; t0 < ntiles; t0 += tiles_per_launch) {
        const int64_t nt = ntiles - t0 < tiles_per_launch ? ntiles - t0 : tiles_per_launch;
        const dim3 grid((unsigned)g.rb_per_tile, (unsigned)g.cb_per_tile, (unsigned)nt);
        const float4_t* rc = rec;
        if (f32)
            st = prm->stats ? launch(k_matern_learned<float, true>, grid, dim3(256), stream, rc, locs->x, locs->y, g,
                                     t0, sigma2, kb, fa, fb, nu_ok, nu, sig_mul, bitmap, (float*)out, prm->stats)
                            : launch(k_matern_learned<float, false>, grid, dim3(256), stream, rc, locs->x, locs->y, g,
                                     t0, sigma2, kb, fa, fb, nu_ok, nu, sig_mul, bitmap, (float*)out, prm->stats);
        else
            st = prm->stats ? launch(k_matern_learned<double, true>, grid, dim3(256), stream, rc, locs->x, locs->y, g,
                                     t0, sigma2, kb, fa, fb, nu_ok, nu, sig_mul, bitmap, (double*)out, prm->stats)
                            : launch(k_matern_learned<double, false>, grid, dim3(256), stream, rc, locs->x, locs->y,
                                     g, t0, sigma2, kb, fa, fb, nu_ok, nu, sig_mul, bitmap, (double*)out,
                                     prm->stats);
        if (st != BK_OK) return st;
    }
    if (mark_kernel_event(prm, 1, stream) != hipSuccess) return BK_EHIP;
    const dim3 fgrid((unsigned)std::min<int64_t>((nwords + 255) / 256, 1024));
    return f32 ? launch(k_matern_fallback<float>, fgrid, dim3(256), stream, locs->x, locs->y, g, prm->sigma2, ib, nu,
                        pref, L, Lq, (const unsigned int*)bitmap, nwords, (float*)out, prm->stats)
               : launch(k_matern_fallback<double>, fgrid, dim3(256), stream, locs->x, locs->y, g, prm->sigma2, ib,
                        nu, pref, L, Lq, (const unsigned int*)bitmap, nwords, (double*)out, prm->stats);
}

}  // namespace bk

// ---------------------------------------------------------------------------
// C ABI: model, training and MLP primitives
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// No-allocation learned Matern: the workspace of bk_matern_tiles' learned form
// (window table, interval plans, wave bitmap) lives in a static device array, one
// copy per GPU, held until the process ends. Host code never passes the array's
// name to a kernel: its address on each device comes from hipGetSymbolAddress,
// taken once per device with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[BK_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of this device's scratch (set up on the first call on the device).
int scratch_for_current_device(void** ptr)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return BK_EHIP;
    if (dev < 0 || dev >= kMaxScratchDevices) return BK_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BK_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return BK_OK;
}
}  // namespace

extern "C" int bk_matern_tiles_noalloc(const bk_locs* locs, const bk_params* prm, int32_t tile_size,
                                       int32_t lower_only, void* out, hipStream_t stream)
{
    if (!locs || !prm || tile_size <= 0 || locs->n < 0) return BK_EINVAL;
    if (prm->mode != BK_LEARNED || locs->n == 0)     // the other forms use no workspace
        return matern_tiles_dispatch(locs, prm, tile_size, lower_only, out, nullptr, 0, stream);
    const size_t need = matern_learned_workspace_bytes(locs->n, tile_size, lower_only);
    if (need == 0 || need > (size_t)BK_NOALLOC_SCRATCH_BYTES) return BK_ENOMEM;
    if (stream) {                // the scratch address is per device: the stream must be the current device's
        int dev = -1, sdev = -1;
        if (hipGetDevice(&dev) != hipSuccess || hipStreamGetDevice(stream, &sdev) != hipSuccess) return BK_EHIP;
        if (dev != sdev) return BK_EINVAL;
    }
    void* ws = nullptr;
    const int st = scratch_for_current_device(&ws);
    if (st != BK_OK) return st;
    return matern_tiles_dispatch(locs, prm, tile_size, lower_only, out, ws, (size_t)BK_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" size_t bk_workspace_bytes(int64_t n)
{
    return 256 + (size_t)(n > 0 ? n : 0) * sizeof(unsigned int);
}

extern "C" size_t bk_matern_workspace_bytes(int64_t n, int32_t tile_size, int32_t lower_only)
{
    return matern_learned_workspace_bytes(n, tile_size, lower_only);
}

extern "C" int bk_model_create(bk_model** m)
{
    if (!m) return BK_EINVAL;
    *m = new (std::nothrow) bk_model();
    return *m ? BK_OK : BK_ENOMEM;
}

extern "C" void bk_model_destroy(bk_model* m)
{
    if (!m) return;
    model_free(m);
    delete m;
}

static const char kMagic[8] = {'B', 'K', 'M', 'L', 'P', '0', '0', '1'};

extern "C" int bk_model_save(const bk_model* m, const char* path)
{
    if (!m || !path || !m->params) return BK_EINVAL;
    std::vector<float> P(kNParam);
    if (hipMemcpy(P.data(), m->params, sizeof(float) * kNParam, hipMemcpyDeviceToHost) != hipSuccess) return BK_EHIP;
    FILE* f = fopen(path, "wb");
    if (!f) return BK_EIO;
    double hdr[20] = {0};
    for (int i = 0; i < 8; ++i) hdr[i] = m->norm[i];
    for (int i = 0; i < 4; ++i) hdr[8 + i] = m->box[i];
    for (int i = 0; i < 4; ++i) hdr[12 + i] = m->margins[i];
    hdr[16] = m->train_L[0];
    hdr[17] = m->train_L[1];
    hdr[18] = (double)kNParam;
    hdr[19] = m->trained ? 1.0 : 0.0;
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(hdr, sizeof(double), 20, f) == 20 &&
              fwrite(P.data(), sizeof(float), kNParam, f) == (size_t)kNParam;
    ok = (fclose(f) == 0) && ok;
    return ok ? BK_OK : BK_EIO;
}

extern "C" int bk_model_load(bk_model* m, const char* path)
{
    if (!m || !path) return BK_EINVAL;
    FILE* f = fopen(path, "rb");
    if (!f) return BK_EIO;
    char mg[8];
    double hdr[20];
    std::vector<float> P(kNParam);
    bool ok = fread(mg, 1, 8, f) == 8 && memcmp(mg, kMagic, 8) == 0 && fread(hdr, sizeof(double), 20, f) == 20 &&
              hdr[18] == (double)kNParam && fread(P.data(), sizeof(float), kNParam, f) == (size_t)kNParam;
    fclose(f);
    if (!ok) return BK_EIO;
    for (int i = 0; i < kNParam; ++i)
        if (!std::isfinite(P[i])) return BK_EIO;
    for (int i = 0; i < 8; ++i) m->norm[i] = hdr[i];
    for (int i = 0; i < 4; ++i) m->box[i] = hdr[8 + i];
    for (int i = 0; i < 4; ++i) m->margins[i] = hdr[12 + i];
    m->train_L[0] = hdr[16];
    m->train_L[1] = hdr[17];
    int st = model_upload(m, P.data());
    if (st) return st;
    m->trained = hdr[19] != 0.0;
    return BK_OK;
}

extern "C" int bk_model_set_margins(bk_model* m, double d_lo, double d_hi, double eta, double n_add)
{
    if (!m || !(d_lo >= 0) || !(d_hi >= 0) || !(eta >= 0) || !(n_add >= 0)) return BK_EINVAL;
    m->margins[0] = d_lo;
    m->margins[1] = d_hi;
    m->margins[2] = eta;
    m->margins[3] = n_add;
    return model_cells(m);
}

extern "C" int bk_model_get_margins(const bk_model* m, double* m4)
{
    if (!m || !m4) return BK_EINVAL;
    for (int i = 0; i < 4; ++i) m4[i] = m->margins[i];
    return BK_OK;
}

extern "C" int bk_model_set_table_source(bk_model* m, int32_t source)
{
    if (!m || (source != BK_TABLE_NETWORK && source != BK_TABLE_SOLVER)) return BK_EINVAL;
    if (!m->params) return BK_ENOMODEL;
    m->table_source = source;
    return model_cells(m);
}

extern "C" int bk_model_get_params(const bk_model* m, float* host)
{
    if (!m || !host || !m->params) return BK_EINVAL;
    return hip_ok(hipMemcpy(host, m->params, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
}

extern "C" int bk_model_set_params(bk_model* m, const float* host)
{
    if (!m || !host) return BK_EINVAL;
    for (int i = 0; i < kNParam; ++i)
        if (!std::isfinite(host[i])) return BK_EINVAL;
    int st = model_upload(m, host);
    if (st == BK_OK) m->trained = true;
    return st;
}

extern "C" int bk_model_get_norm(const bk_model* m, double* n8)
{
    if (!m || !n8) return BK_EINVAL;
    memcpy(n8, m->norm, sizeof(m->norm));
    return BK_OK;
}

extern "C" int bk_model_set_norm(bk_model* m, const double* n8)
{
    if (!m || !n8 || !(n8[1] > 0) || !(n8[3] > 0) || !(n8[4] > 0) || !(n8[5] > 0)) return BK_EINVAL;
    memcpy(m->norm, n8, sizeof(m->norm));
    return model_cells(m);
}

extern "C" int bk_model_get_box(const bk_model* m, double* b4)
{
    if (!m || !b4) return BK_EINVAL;
    memcpy(b4, m->box, sizeof(m->box));
    return BK_OK;
}

extern "C" int bk_model_set_box(bk_model* m, const double* b4)
{
    if (!m || !b4 || !(b4[1] > b4[0]) || !(b4[3] > b4[2])) return BK_EINVAL;
    memcpy(m->box, b4, sizeof(m->box));
    return model_cells(m);
}

extern "C" int bk_model_get_cells(const bk_model* m, float* host, int64_t cap, int32_t* dims)
{
    if (!m || !dims) return BK_EINVAL;
    dims[0] = kCellsLx;
    dims[1] = kCellsNu;
    if (!host) return BK_OK;
    if (cap < (int64_t)4 * kCells) return BK_EINVAL;
    if (!m->params) return BK_ENOMODEL;
    return hip_ok(hipMemcpy(host, m->cells, sizeof(float) * 4 * kCells, hipMemcpyDeviceToHost));
}

extern "C" int bk_mlp_infer(const bk_model* m, const float* u, float* y, int64_t n, hipStream_t s)
{
    if (!m || n < 0) return BK_EINVAL;
    if (n == 0) return BK_OK;
    if (!u || !y) return BK_EINVAL;
    if (!m->params) return BK_ENOMODEL;
    return launch(k_mlp_infer, dim3((unsigned)((n + 255) / 256)), dim3(256), s, make_dev(m), u, y, n);
}

extern "C" size_t bk_mlp_grad_scratch_bytes(int64_t B)
{
    return B > 0 ? sizeof(float) * grad_scratch_floats(B) : 0;
}

extern "C" int bk_mlp_grad(const float* params, const float* u, const float* tgt, const float* tau, int64_t B,
                           float* grad, float* loss, void* scratch, size_t scratch_bytes, hipStream_t s)
{
    if (!params || !u || !tgt || !tau || !grad || !loss || !scratch || B <= 0 || B > (1 << 20)) return BK_EINVAL;
    if (scratch_bytes < bk_mlp_grad_scratch_bytes(B)) return BK_ENOMEM;
    const int st = launch(k_zero_f32, dim3(1), dim3(256), s, loss, (int64_t)1);
    if (st != BK_OK) return st;
    return launch_grad(params, u, tgt, tau, B, 0, 1, 0, 0, grad, loss, (float*)scratch, s);
}

extern "C" int bk_adam_step(float* p, const float* g, float* m, float* v, int64_t n, int32_t step, float lr,
                            float beta1, float beta2, float eps, hipStream_t s)
{
    if (!p || !g || !m || !v || n < 0 || step < 1 || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
        return BK_EINVAL;
    if (n == 0) return BK_OK;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    return launch(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), s, p, g, m, v, n, lr, beta1, beta2, eps, c1,
                  c2);
}

static uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

extern "C" int bk_model_train(bk_model* m, const double* nu, const double* x, int64_t n, const bk_train_cfg* cfg,
                              float* final_loss, hipStream_t s)
{
    if (!m || !nu || !x || !cfg || n < 1024 || cfg->epochs < 1 || cfg->batch < 1 || cfg->batch > 65536 ||
        n >= ((int64_t)1 << 31) || !(cfg->lr > 0))
        return BK_EINVAL;
    int st = model_alloc(m);
    if (st) return st;
    double L, Lq;
    resolve_thresholds(BK_MIXED_F32C, cfg->L_window, cfg->L_quad, &L, &Lq);
    m->train_L[0] = L;
    m->train_L[1] = Lq;
    const int64_t B = cfg->batch;
    // device buffers
    double *tlo = nullptr, *thi = nullptr;
    int32_t* nodes = nullptr;
    float *U = nullptr, *T = nullptr, *scr = nullptr, *grad = nullptr, *mom = nullptr, *vel = nullptr, *loss = nullptr,
          *tau = nullptr, *res = nullptr;
    auto cleanup = [&]() {
        void* bufs[] = {tlo, thi, nodes, U, T, scr, grad, mom, vel, loss, tau, res};
        for (void* b : bufs)
            if (b) (void)hipFree(b);
    };
    if (hipMalloc((void**)&tlo, 8 * n) || hipMalloc((void**)&thi, 8 * n) || hipMalloc((void**)&nodes, 4 * n) ||
        hipMalloc((void**)&U, 8 * n) || hipMalloc((void**)&T, 12 * n) ||
        hipMalloc((void**)&scr, sizeof(float) * grad_scratch_floats(B)) || hipMalloc((void**)&grad, 4 * kNParam) ||
        hipMalloc((void**)&mom, 4 * kNParam) || hipMalloc((void**)&vel, 4 * kNParam) || hipMalloc((void**)&loss, 4) ||
        hipMalloc((void**)&tau, 16) || hipMalloc((void**)&res, 12 * n)) {
        cleanup();
        return BK_ENOMEM;
    }
    // targets from the plain solver
    st = bk_window(nu, x, tlo, thi, nodes, n, L, Lq, s);
    const unsigned nb = (unsigned)((n + 255) / 256);
    const float cx = (float)m->norm[0], sx = (float)m->norm[1], cnu = (float)m->norm[2], snu = (float)m->norm[3];
    const float stn = (float)m->norm[4], snn = (float)m->norm[5];
    if (st == BK_OK)
        st = launch(k_make_targets, dim3(nb), dim3(256), s, (const double*)nu, (const double*)x, (const double*)tlo,
                    (const double*)thi, (const int32_t*)nodes, n, cx, sx, cnu, snu, stn, snn, U, T);
    // training box = range of the data
    {
        std::vector<double> hx(n), hn(n);
        if (st == BK_OK && (hipMemcpyAsync(hx.data(), x, 8 * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
                            hipMemcpyAsync(hn.data(), nu, 8 * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
                            hipStreamSynchronize(s) != hipSuccess))
            st = BK_EHIP;
        if (st == BK_OK) {
            double lo = 1e300, hi = -1e300, nlo = 1e300, nhi = -1e300;
            for (int64_t i = 0; i < n; ++i) {
                double lx = log10(hx[i]);
                lo = std::min(lo, lx); hi = std::max(hi, lx);
                nlo = std::min(nlo, fabs(hn[i])); nhi = std::max(nhi, fabs(hn[i]));
            }
            // rounded outward to 1e-3, so that inputs from the same law just past the
            // sample's extremes still use the model (a sliver of extrapolation that the
            // acceptance tests guard)
            m->box[0] = floor(lo * 1e3) / 1e3;
            m->box[1] = ceil(hi * 1e3) / 1e3;
            m->box[2] = std::max(0.0, floor(nlo * 1e3) / 1e3);
            m->box[3] = ceil(nhi * 1e3) / 1e3;
        }
    }
    // He initialisation from a seeded host generator
    std::vector<float> P(kNParam, 0.0f);
    {
        std::mt19937_64 rng(cfg->seed);
        std::normal_distribution<float> nd(0.0f, 1.0f);
        for (int i = 0; i < kH * 2; ++i) P[kOffW1 + i] = nd(rng) * sqrtf(2.0f / 2.0f);
        for (int i = 0; i < kH; ++i) P[kOffB1 + i] = 0.1f * nd(rng);
        for (int i = 0; i < kH * kH; ++i) P[kOffW2 + i] = nd(rng) * sqrtf(2.0f / (float)kH);
        for (int i = 0; i < 3 * kH; ++i) P[kOffW3 + i] = nd(rng) * sqrtf(1.0f / (float)kH);
        P[kOffB3 + 0] = 0.2f; P[kOffB3 + 1] = 0.8f; P[kOffB3 + 2] = 0.5f;
    }
    const float htau[4] = {cfg->tau_lo, cfg->tau_hi, cfg->tau_n, 0.0f};
    if (st == BK_OK && (hipMemcpyAsync(m->params, P.data(), 4 * kNParam, hipMemcpyHostToDevice, s) != hipSuccess ||
                        hipMemcpyAsync(tau, htau, 16, hipMemcpyHostToDevice, s) != hipSuccess ||
                        hipMemsetAsync(mom, 0, 4 * kNParam, s) != hipSuccess ||
                        hipMemsetAsync(vel, 0, 4 * kNParam, s) != hipSuccess))
        st = BK_EHIP;
    std::mt19937_64 prng(cfg->seed ^ 0x9e3779b97f4a7c15ULL);
    const int64_t steps_per_epoch = (n + B - 1) / B;
    const int64_t total = steps_per_epoch * cfg->epochs;
    int64_t step = 0;
    float last = 0.0f;
    for (int ep = 0; ep < cfg->epochs && st == BK_OK; ++ep) {
        // a fresh affine permutation of the rows each epoch
        uint64_t pa = prng() % (uint64_t)n;
        while (pa == 0 || gcd_u64(pa, (uint64_t)n) != 1) pa = prng() % (uint64_t)n;
        const uint64_t pb = prng() % (uint64_t)n;
        st = launch(k_zero_f32, dim3(1), dim3(256), s, loss, (int64_t)1);
        for (int64_t b0 = 0; b0 < n && st == BK_OK; b0 += B) {
            const int64_t bs = std::min(B, n - b0);
            ++step;
            // cosine decay of the step size to 5% of its initial value
            const double frac = (double)step / (double)total;
            const float lr = (float)(cfg->lr * (0.05 + 0.95 * 0.5 * (1.0 + cos(M_PI * frac))));
            // tile gradients, then their sum and the Adam update in one launch (the same
            // arithmetic as bk_mlp_grad followed by bk_adam_step)
            const unsigned tiles = (unsigned)((bs + kTrainTile - 1) / kTrainTile);
            st = launch(k_train_tile, dim3(tiles), dim3(kTrainThreads), s, (const float*)m->params, (const float*)U,
                        (const float*)T, (const float*)tau, bs, n, pa, pb, b0, scr, loss);
            if (st == BK_OK) {
                const int32_t t = (int32_t)std::min<int64_t>(step, 1 << 30);
                const float c1 = 1.0f - powf(cfg->beta1, (float)t), c2 = 1.0f - powf(cfg->beta2, (float)t);
                st = launch(k_grad_adam, dim3((kNParam + 255) / 256), dim3(256), s, (const float*)scr, (int)tiles,
                            m->params, mom, vel, lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2);
            }
        }
        float hl = 0.0f;
        if (st == BK_OK && (hipMemcpyAsync(&hl, loss, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                            hipStreamSynchronize(s) != hipSuccess))
            st = BK_EHIP;
        last = hl / (float)steps_per_epoch;
    }
    // inference pack, then margins from the inference-path residuals on the training set
    if (st == BK_OK) {
        if (hipMemcpyAsync(P.data(), m->params, 4 * kNParam, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = BK_EHIP;
        for (int i = 0; st == BK_OK && i < kNParam; ++i)
            if (!std::isfinite(P[i])) st = BK_EINVAL;
        if (st == BK_OK) st = model_upload(m, P.data());
    }
    if (st == BK_OK) {
        st = launch(k_residuals, dim3(nb), dim3(256), s, make_dev(m), (const float*)U, (const float*)T, n, res);
        std::vector<float> hr(3 * n);
        if (st == BK_OK && (hipMemcpyAsync(hr.data(), res, 12 * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
                            hipStreamSynchronize(s) != hipSuccess))
            st = BK_EHIP;
        if (st == BK_OK) {
            // Window margins: the 99.8% quantile of the inference-path residuals
            // (+0.01). No node-count margin: the kernel raises N to the strip-bound
            // rule's count for the widened window, which is always sufficient.
            double mg[2];
            std::vector<float> col(n);
            for (int k = 0; k < 2; ++k) {
                for (int64_t i = 0; i < n; ++i) col[i] = hr[3 * i + k];
                const int64_t q = (int64_t)(0.998 * (double)(n - 1));
                std::nth_element(col.begin(), col.begin() + q, col.end());
                mg[k] = std::max(0.0, (double)col[q]);
            }
            m->margins[0] = mg[0] + 0.01;
            m->margins[1] = mg[1] + 0.01;
            m->margins[2] = 0.0;
            m->margins[3] = 0.0;
        }
    }
    if (st == BK_OK) st = model_cells(m);     // the plans depend on the margins just set
    cleanup();
    if (st == BK_OK) m->trained = true;
    if (final_loss) *final_loss = last;
    return st;
}
