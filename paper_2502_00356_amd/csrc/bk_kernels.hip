// bk_kernels.hip - HIP kernels and C ABI for standalone K_nu(x), the window
// export, tiled Matern covariance generation (arXiv 2502.00356, Sec. IV-B,
// Sec. III-A, Alg. 3), the paper's refined algorithm (Sec. IV-A, IV-C, Alg. 2),
// and the derivatives of K_nu and of the Matern covariance, for gfx950.
//
// Mapping: one lane per output entry. Standalone K_nu: 512-entry workgroups whose
// entries are re-sorted through LDS between phases (coalesced FP64 loads, stores
// to each entry's own index); the other kernels: 256-lane workgroups.
// Matern: each wave covers 64 consecutive rows of a tile column (one 512-byte
// FP64 or 256-byte FP32 store per column); the row location lives in VGPRs and
// the column location is wave-uniform, so it is read through scalar loads
// instead of being staged in LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/besselk.h"
#include "bk_math.hpp"
#include "bk_internal.hpp"

namespace bk {

void resolve_thresholds(int mode, double L_in, double Lq_in, double* L, double* Lq)
{
    bool plain = (mode == BK_PLAIN_F64);
    *L = L_in > 0.0 ? L_in : (plain ? kDefaultLPlain : kDefaultLMixed);
    *Lq = Lq_in > 0.0 ? Lq_in : (plain ? kDefaultLqPlain : kDefaultLqMixed);
}

// Sum of a per-lane value over a workgroup of nw wave64s (nw <= 16), added once to
// a global counter.
__device__ void block_count_w(unsigned long long* dst, unsigned long long v, int nw)
{
    __shared__ unsigned long long red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < nw; ++w) t += red[w];
        atomicAdd(dst, t);
    }
}

// Sum of a per-lane count over a wave (every lane active), added once to a global
// counter by lane 0.
__device__ inline void wave_count(unsigned long long* dst, unsigned int v)
{
    unsigned long long a = v;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0 && a) atomicAdd(dst, a);
}

// Largest per-lane value over a wave (every lane active).
__device__ inline unsigned int wave_max_u32(unsigned int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned int)__shfl_xor((int)v, o, 64));
    return v;
}

// Special values shared by every form; returns true if handled.
__device__ __forceinline__ bool special_value(double v, double z, int result, double& r)
{
    if (isnan(v) || isnan(z) || z < 0.0) { r = __builtin_nan(""); return true; }
    if (z == 0.0 || isinf(v)) { r = __builtin_inf(); return true; }
    if (isinf(z)) { r = (result == BK_RESULT_LOG) ? -__builtin_inf() : 0.0; return true; }
    return false;
}

// Final assembly from exp(-x) exp(Delta) h S (see bk_math.hpp).
__device__ __forceinline__ double assemble(double z, double delta, double hs, int result)
{
    if (result == BK_RESULT_SCALED) return exp(delta) * hs;
    if (result == BK_RESULT_LOG) return (delta - z) + log(hs);
    if (z < 708.0) return exp(-z) * exp(delta) * hs;   // exp(-z) still a normal number
    // subnormal range: e^(-z) formed 2^64 larger, product scaled back (one rounding)
    return ldexp(exp(64.0 * kLn2 - z) * exp(delta) * hs, -64);
}

// The plain and mixed forms take Temme's series with the forward recurrence (Sec. IV-A; the
// paper's branch for x < 0.1 in Alg. 2) where x < 0.1 and K_nu(x) stays far inside
// the double range: log K_nu(x) <= log Gamma(nu) + nu log(2/x) for x < 0.1, bounded
// here by nu (log(2/x) + log(nu + 1)) + log(1/nu + 1) < 600. On 2^24 pairs with
// x in [1e-4, 0.1) it is 3.7 times faster than the windowed FP64 quadrature and as
// accurate (max relative error 3.0e-15 against 6.4e-15); it also takes 10% off the
// FP32-term form on the 2^24 grid, at FP64 accuracy for those entries.
__device__ __forceinline__ bool temme_applies(double v, double z)
{
    if (!(z < kPaperTemmeX) || !(v > 0.0)) return false;
    const float vf = (float)v;
    const float lb = vf * (__logf(2.0f / (float)z) + __logf(vf + 1.0f)) + __logf(1.0f / vf + 1.0f);
    return lb < 600.0f;
}

// K_nu(z) by Temme's series, as the requested result (K, e^z K or log K).
__device__ __forceinline__ double temme_result(double v, double z, int result)
{
    const double k = temme_k(v, z, temme_tab());
    if (result == BK_RESULT_SCALED) return k * exp(z);
    if (result == BK_RESULT_LOG) return log(k);
    return k;
}

// Counting sort of a block's lanes by a small key (0..63): returns the lane's slot
// in key order. Equal keys keep no particular order; results do not depend on it,
// since every entry is computed by one lane from its own inputs.
template <int NB>
__device__ unsigned int block_sort_slot(int key, unsigned int* hist)
{
    const int tid = threadIdx.x;
    if (tid < 64) hist[tid] = 0u;
    __syncthreads();
    const unsigned int rank = atomicAdd(&hist[key], 1u);
    __syncthreads();
    if (tid < 64) {
        const unsigned int h = hist[tid];
        hist[tid] = wave_incl_scan(h) - h;
    }
    __syncthreads();
    const unsigned int slot = hist[key] + rank;
    __syncthreads();   // hist may be reused by the caller after this
    return slot;
}

// Plain and mixed K_nu. A block of kSolveBlock entries is processed in three
// phases, with the lanes re-sorted between them through LDS so that each wave
// holds entries that take the same branches and loop counts:
//  1. entry order: special values; key = peak regime (0: nu^2 <= x, t* = 0;
//     1: interior peak, window from t = 0; 2: interior peak with a left root
//     likely, estimated by nu asinh(nu/x) > L; 4: x < 0.1, Temme's series);
//  2. regime order: Temme's series (and its store), or the FP64 peak / window
//     solve and node count;
//  3. node-count order: the node walk, the prefactor and the store to the
//     entry's own index.
constexpr int kSolveBlock = 512;

// Six waves per SIMD is what the block's LDS allows (three 512-lane blocks per CU);
// without the hint the plain form takes 81 VGPRs and gets five (7% slower).
template <int MODE>
__global__ __launch_bounds__(kSolveBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_besselk(const double* __restrict__ nu,
                                                         const double* __restrict__ x,
                                                         double* __restrict__ out, int64_t n, int result,
                                                         double L, double Lq, 
                                                         unsigned long long* __restrict__ stats)
{
    __shared__ unsigned int hist[64];
    __shared__ double s_tab[kTabLen];
    // staged per entry between phases: v, z, t_ref, h, Delta, then for the plain
    // form dlo, e^t_ref, e^-t_ref, expm1(t_ref) (paired walk), for the mixed form
    // t0 and x cosh(t_ref) / 2
    constexpr int kRows = MODE == BK_PLAIN_F64 ? 9 : 7;
    __shared__ double s_d[kRows][kSolveBlock];
    __shared__ int s_i[3][kSolveBlock];
    const int tid = threadIdx.x;
    if (tid < kTabLen) s_tab[tid] = rule_tab().tab[tid];   // read after the sorts' barriers
    const int64_t i = (int64_t)blockIdx.x * kSolveBlock + tid;
    double v = 0.0, z = 1.0;
    bool work = false;
    if (i < n) {
        v = fabs(nu[i]);
        z = x[i];
        double r;
        if (special_value(v, z, result, r)) out[i] = r;
        else work = true;
    }
    int key = 0;
    if (work && v * v > z) key = ((float)v * asinhf((float)(v / z)) > (float)L) ? 2 : 1;
    if (work && temme_applies(v, z)) key = 4;
    // phase 1 -> 2: sort by regime (Temme's series in waves of their own)
    unsigned int slot = block_sort_slot<kSolveBlock>(work ? key : 3, hist);
    s_d[0][slot] = v;
    s_d[1][slot] = z;
    s_i[0][slot] = work ? (int)(i - (int64_t)blockIdx.x * kSolveBlock) : -1;
    s_i[1][slot] = key;
    __syncthreads();
    int li = s_i[0][tid];
    const double v2 = s_d[0][tid], z2 = s_d[1][tid];
    const bool temme = li >= 0 && s_i[1][tid] == 4;
    __syncthreads();
    Solved sv;
    sv.p.N = -1;
    if (temme) {
        out[(int64_t)blockIdx.x * kSolveBlock + li] = temme_result(v2, z2, result);
        li = -1;
    } else if (li >= 0) {
        sv = plain_solve(v2, z2, L, Lq, rule_tab(), s_tab);
    }
    // phase 2 -> 3: sort by node count
    const int nkey = li < 0 ? 0 : (sv.p.N < 63 ? sv.p.N : 63);
    slot = block_sort_slot<kSolveBlock>(nkey, hist);
    s_d[0][slot] = v2;
    s_d[1][slot] = z2;
    s_d[2][slot] = sv.p.tref;
    s_d[3][slot] = sv.p.h;
    s_d[4][slot] = sv.delta;
    if constexpr (MODE == BK_PLAIN_F64) {
        s_d[5][slot] = sv.dlo;
        s_d[6][slot] = sv.E;
        s_d[7][slot] = sv.Ei;
        s_d[8][slot] = sv.Sr;
    } else {
        s_d[5][slot] = sv.p.t0;
        s_d[6][slot] = sv.A;
    }
    s_i[0][slot] = li;
    s_i[1][slot] = sv.p.N;
    s_i[2][slot] = sv.p.mc;
    __syncthreads();
    const int l3 = s_i[0][tid];
    unsigned long long nodes = 0, ents = 0;
    if (l3 >= 0) {
        const double v3 = s_d[0][tid], z3 = s_d[1][tid];
        Plan p;
        p.tref = s_d[2][tid];
        p.h = s_d[3][tid];
        p.N = s_i[1][tid];
        p.mc = s_i[2][tid];
        double hs;
        if constexpr (MODE == BK_PLAIN_F64) {
            p.t0 = 0.0;                       // not used by the paired walk
            hs = p.h * sum_f64(v3, z3, p, s_d[6][tid], s_d[7][tid], s_d[8][tid], s_tab);
            hs = fma(hs, s_d[5][tid], hs);    // the low part of Delta
        } else {
            p.t0 = s_d[5][tid];
            hs = p.h * sum_mixed(v3, z3, p, s_d[6][tid], s_tab);
        }
        out[(int64_t)blockIdx.x * kSolveBlock + l3] = assemble(z3, s_d[4][tid], hs, result);
        nodes = (unsigned long long)(p.N + 1);
        ents = 1;
    }
    if (stats) {
        block_count_w(stats + BK_STAT_NODES, nodes, kSolveBlock / 64);
        block_count_w(stats + BK_STAT_ENTRIES, ents, kSolveBlock / 64);
        const unsigned int wmax = wave_max_u32((unsigned int)nodes);
        block_count_w(stats + BK_STAT_LANE_SLOTS, (threadIdx.x & 63) == 0 ? 64ull * wmax : 0ull, kSolveBlock / 64);
    }
}

// The paper's refined algorithm (Alg. 2), one lane per entry, FP64: Temme's
// series with the forward recurrence for x < 0.1, the fixed-window sum otherwise.
__global__ __launch_bounds__(256) void k_besselk_paper(const double* __restrict__ nu, const double* __restrict__ x,
                                                       double* __restrict__ out, int64_t n, int result, int bins,
                                                       double T, 
                                                       
                                                       unsigned long long* __restrict__ stats)
{
    __shared__ double s_tab[kTabLen];
    stage_tab(s_tab);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long nodes = 0, ents = 0;
    if (i < n) {
        const double v = fabs(nu[i]), z = x[i];
        double r;
        if (!special_value(v, z, result, r)) {
            if (z < kPaperTemmeX) {
                // K directly; written as exp(-z) exp(0) (e^z K) for the shared assembly
                r = assemble(z, 0.0, temme_k(v, z, temme_tab()) * exp(z), result);
            } else {
                const FixedOut f = paper_fixed(v, z, bins, T, s_tab);
                // K = exp(lscale) h S, written through Delta = lscale + z so that the
                // shared assembly (exp(-z) exp(Delta) h S) applies
                r = assemble(z, f.lscale + z, f.hs, result);
                nodes = (unsigned long long)(bins + 1);
                ents = 1;
            }
        }
        out[i] = r;
    }
    if (stats) {
        block_count_w(stats + BK_STAT_NODES, nodes, 4);
        block_count_w(stats + BK_STAT_ENTRIES, ents, 4);
    }
}

__global__ __launch_bounds__(256) void k_window(const double* __restrict__ nu,
                                                const double* __restrict__ x,
                                                double* __restrict__ tlo, double* __restrict__ thi,
                                                int32_t* __restrict__ nodes, int64_t n, double L,
                                                double Lq)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double v = fabs(nu[i]), z = x[i];
    if (!(z > 0.0) || isinf(z) || isnan(v) || isinf(v)) {
        tlo[i] = __builtin_nan(""); thi[i] = __builtin_nan(""); nodes[i] = 0;
        return;
    }
    Solved s = plain_solve(v, z, L, Lq, rule_tab(), rule_tab().tab);
    tlo[i] = s.p.t0;
    thi[i] = s.t1;
    nodes[i] = s.p.N;
}

// e^x-scaled value s to the requested result (K or e^x K).
__device__ __forceinline__ double unscale(double z, double s, int result)
{
    if (result == BK_RESULT_SCALED) return s;
    if (z < 708.0) return exp(-z) * s;
    return ldexp(exp(64.0 * kLn2 - z) * s, -64);
}

// K_nu(x), dK/dx and dK/dnu, one lane per entry, FP64: the K integral at orders
// nu and |nu - 1| and the dK/dnu integral, each with its own plain solve. NULL
// outputs are skipped (dK/dx still evaluates K_nu). dK/dnu carries the sign of nu.
__global__ __launch_bounds__(256, 3) void k_besselk_deriv(const double* __restrict__ nu, const double* __restrict__ x,
                                                       double* __restrict__ k, double* __restrict__ dkdx,
                                                       double* __restrict__ dkdnu, int64_t n, int result, double L,
                                                       double Lq, 
                                                       unsigned long long* __restrict__ stats)
{
    __shared__ double s_tab[kTabLen];
    stage_tab(s_tab);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long nodes = 0, ents = 0;
    if (i < n) {
        const double nr = nu[i], z = x[i], v = fabs(nr);
        double rk, rx, rn;
        if (isnan(nr) || isnan(z) || z < 0.0) {
            rk = rx = rn = __builtin_nan("");
        } else if (z == 0.0 || isinf(v)) {
            rk = __builtin_inf();
            rx = -__builtin_inf();
            rn = v == 0.0 ? 0.0 : copysign(__builtin_inf(), nr);
        } else if (isinf(z)) {
            rk = 0.0;
            rx = -0.0;
            rn = copysign(0.0, nr);
        } else {
            const RuleTable& R = rule_tab();
            const Solved s0 = plain_solve(v, z, L, Lq, R, s_tab);
            double hs0 = s0.p.h * sum_f64(v, z, s0.p, s0.E, s0.Ei, s0.Sr, s_tab);
            hs0 = fma(hs0, s0.dlo, hs0);
            rk = assemble(z, s0.delta, hs0, result);
            nodes += (unsigned long long)(s0.p.N + 1);
            rx = 0.0;
            if (dkdx) {
                const double v1 = fabs(v - 1.0);
                const Solved s1 = plain_solve(v1, z, L, Lq, R, s_tab);
                double hs1 = s1.p.h * sum_f64(v1, z, s1.p, s1.E, s1.Ei, s1.Sr, s_tab);
                hs1 = fma(hs1, s1.dlo, hs1);
                nodes += (unsigned long long)(s1.p.N + 1);
                rx = -unscale(z, exp(s1.delta) * hs1 + (v / z) * (exp(s0.delta) * hs0), result);
            }
            rn = 0.0;
            if (dkdnu && v > 0.0) {
                const Solved sd = dnu_solve(v, z, s0.p.t0, L, Lq, R, s_tab);
                const double hsd = sd.p.h * sum_dnu_f64(v, sd.p, sd.A, sd.B, s_tab);
                nodes += (unsigned long long)(sd.p.N + 1);
                rn = copysign(assemble(z, sd.delta, hsd, result), nr);
            } else if (dkdnu) {
                rn = copysign(0.0, nr);
            }
            ents = 1;
        }
        if (k) k[i] = rk;
        if (dkdx) dkdx[i] = rx;
        if (dkdnu) dkdnu[i] = rn;
    }
    if (stats) {
        block_count_w(stats + BK_STAT_NODES, nodes, 4);
        block_count_w(stats + BK_STAT_ENTRIES, ents, 4);
    }
}

// ---------------------------------------------------------------------------
// Matern tiles
// ---------------------------------------------------------------------------
constexpr int kRowsPerWave = 64;
constexpr int kColsPerWave = 8;
constexpr int kColsPerGroup = 4 * kColsPerWave;

struct TileGeom {
    int64_t n;
    int32_t ts, T, lower;
    int32_t rb_per_tile, cb_per_tile;
};

__host__ __device__ inline int64_t tile_offset(int64_t n, int64_t ts, int64_t T, int lower, int64_t I, int64_t J)
{
    int64_t nJ = (J == T - 1) ? n - J * ts : ts;
    if (lower) return ts * (J * n - ts * (J * (J - 1) / 2)) + nJ * (I - J) * ts;
    return J * ts * n + nJ * I * ts;
}

__device__ inline void tile_of(int64_t p, const TileGeom& g, int64_t& I, int64_t& J)
{
    int64_t T = g.T;
    if (!g.lower) { J = p / T; I = p - J * T; return; }
    // largest J with off(J) = J T - J (J - 1) / 2 <= p
    double b = 2.0 * (double)T + 1.0;
    int64_t j = (int64_t)floor((b - sqrt(fmax(b * b - 8.0 * (double)p, 0.0))) * 0.5);
    if (j < 0) j = 0;
    if (j > T - 1) j = T - 1;
    while (j > 0 && j * T - j * (j - 1) / 2 > p) --j;
    while (j + 1 <= T - 1 && (j + 1) * T - (j + 1) * j / 2 <= p) ++j;
    J = j;
    I = J + (p - (J * T - J * (J - 1) / 2));
}

// kStats: the statistics variant, which also counts the entries evaluated by
// quadrature and their nodes (lanes past a ragged tile's last row stay in the
// wave, idle, so that the wave can sum its counts).
template <int MODE, typename OutT, bool kStats>
__global__ __launch_bounds__(256, 4) void k_matern(const double* __restrict__ lx,
                                                const double* __restrict__ ly, TileGeom g,
                                                int64_t tile_base, double sigma2, double inv_beta,
                                                double nu, double pref, double L, double Lq,
                                                int bins, double T, OutT* __restrict__ out,
                                                unsigned long long* __restrict__ stats)
{
    __shared__ double s_tab[kTabLen];
    stage_tab(s_tab);                   // before any wave leaves
    // block -> (tile, row block, column block) in 32-bit arithmetic (a 64-bit
    // division is a long instruction sequence)
    const unsigned wg_per_tile = (unsigned)g.rb_per_tile * (unsigned)g.cb_per_tile;
    const unsigned tq = blockIdx.x / wg_per_tile, local = blockIdx.x - tq * wg_per_tile;
    const int64_t p = tile_base + (int64_t)tq;
    const int rb = (int)(local % (unsigned)g.rb_per_tile), cb = (int)(local / (unsigned)g.rb_per_tile);
    int64_t I, J;
    tile_of(p, g, I, J);
    const int64_t mI = min((int64_t)g.ts, g.n - I * g.ts);
    const int64_t nJ = min((int64_t)g.ts, g.n - J * g.ts);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t il = (int64_t)rb * kRowsPerWave + lane;
    const int64_t jl0 = (int64_t)cb * kColsPerGroup + (int64_t)wave * kColsPerWave;
    const bool row_ok = il < mI;
    // the statistics variant keeps every wave to the end for its block-wide sums
    if (!kStats && (jl0 >= nJ || !row_ok)) return;
    const int64_t base = tile_offset(g.n, g.ts, g.T, g.lower, I, J);
    const int64_t ilr = row_ok ? il : 0;
    const double xi = lx[I * g.ts + ilr], yi = ly[I * g.ts + ilr];
    const int cend = (kStats && (!row_ok || jl0 >= nJ)) ? 0 : (int)min((int64_t)kColsPerWave, nJ - jl0);
    unsigned int c_ent = 0, c_nodes = 0;
    unsigned int col_nodes[kColsPerWave] = {};      // statistics: nodes per column walked
    for (int c = 0; c < cend; ++c) {
        const int64_t jl = jl0 + c;
        const double xj = lx[J * g.ts + jl], yj = ly[J * g.ts + jl];
        const double dx = xj - xi, dy = yj - yi;
        const double r = sqrt(dx * dx + dy * dy);
        double val;
        if (r == 0.0) {
            val = sigma2;
        } else {
            const double z = r * inv_beta;
            if (MODE == BK_PAPER_REFINED) {
                if (z < kPaperTemmeX) {
                    val = sigma2 * exp(pref + nu * log(z)) * temme_k(nu, z, temme_tab());
                } else {
                    const FixedOut f = paper_fixed(nu, z, bins, T, s_tab);
                    val = sigma2 * exp(pref + nu * log(z) + f.lscale) * f.hs;
                    c_nodes += (unsigned int)(bins + 1);
                    c_ent += 1;
                    if (kStats) col_nodes[c] = (unsigned int)(bins + 1);
                }
            } else {
                Solved s = plain_solve(nu, z, L, Lq, rule_tab(), s_tab);
                double hs;
                if constexpr (MODE == BK_PLAIN_F64) {
                    hs = s.p.h * sum_f64(nu, z, s.p, s.E, s.Ei, s.Sr, s_tab);
                    hs = fma(hs, s.dlo, hs);
                } else {
                    hs = s.p.h * sum_mixed(nu, z, s.p, s.A, s_tab);
                }
                val = sigma2 * exp(pref + nu * log(z) + (s.delta - z)) * hs;
                c_nodes += (unsigned int)(s.p.N + 1);
                c_ent += 1;
                if (kStats) col_nodes[c] = (unsigned int)(s.p.N + 1);
            }
        }
        out[base + il + jl * mI] = (OutT)val;
    }
    if (kStats) {      // one atomic per counter per workgroup
        unsigned int slots = 0;
#pragma unroll
        for (int c = 0; c < kColsPerWave; ++c) slots += 64u * wave_max_u32(col_nodes[c]);
        block_count_w(stats + BK_STAT_ENTRIES, c_ent, 4);
        block_count_w(stats + BK_STAT_NODES, c_nodes, 4);
        block_count_w(stats + BK_STAT_LANE_SLOTS, (threadIdx.x & 63) == 0 ? slots : 0u, 4);
    }
}

// Matern covariance and its partial derivatives in beta and nu (Sec. III-A
// formula, differentiated), FP64, same tiling and lane mapping as k_matern. With
// z = r / beta and c(nu) = 2^(1-nu) / Gamma(nu):
//   M       = sigma2 c z^nu K_nu(z)
//   dM/dbeta = sigma2 c z^(nu+1) K_{nu-1}(z) / beta     (d/dz z^nu K_nu = -z^nu K_{nu-1})
//   dM/dnu   = M (ln z - ln 2 - psi(nu)) + sigma2 c z^nu dK_nu/dnu(z)
// pref = ln c and psi = psi(nu) come from the host. A NULL output is skipped.
template <typename OutT>
__global__ __launch_bounds__(256) void k_matern_grad(const double* __restrict__ lx, const double* __restrict__ ly,
                                                     TileGeom g, int64_t tile_base, double sigma2, double inv_beta,
                                                     double nu, double pref, double psi, double L, double Lq,
                                                      OutT* __restrict__ oc,
                                                     OutT* __restrict__ ob, OutT* __restrict__ on)
{
    __shared__ double s_tab[kTabLen];
    stage_tab(s_tab);                   // before any wave leaves
    // block -> (tile, row block, column block) in 32-bit arithmetic (a 64-bit
    // division is a long instruction sequence)
    const unsigned wg_per_tile = (unsigned)g.rb_per_tile * (unsigned)g.cb_per_tile;
    const unsigned tq = blockIdx.x / wg_per_tile, local = blockIdx.x - tq * wg_per_tile;
    const int64_t p = tile_base + (int64_t)tq;
    const int rb = (int)(local % (unsigned)g.rb_per_tile), cb = (int)(local / (unsigned)g.rb_per_tile);
    int64_t I, J;
    tile_of(p, g, I, J);
    const int64_t mI = min((int64_t)g.ts, g.n - I * g.ts);
    const int64_t nJ = min((int64_t)g.ts, g.n - J * g.ts);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t il = (int64_t)rb * kRowsPerWave + lane;
    const int64_t jl0 = (int64_t)cb * kColsPerGroup + (int64_t)wave * kColsPerWave;
    if (il >= mI || jl0 >= nJ) return;
    const int64_t base = tile_offset(g.n, g.ts, g.T, g.lower, I, J);
    const double xi = lx[I * g.ts + il], yi = ly[I * g.ts + il];
    const int cend = (int)min((int64_t)kColsPerWave, nJ - jl0);
    const double nu1 = fabs(nu - 1.0);
    for (int c = 0; c < cend; ++c) {
        const int64_t jl = jl0 + c;
        const double xj = lx[J * g.ts + jl], yj = ly[J * g.ts + jl];
        const double dx = xj - xi, dy = yj - yi;
        const double r = sqrt(dx * dx + dy * dy);
        double vc = sigma2, vb = 0.0, vn = 0.0;
        if (r != 0.0) {
            const RuleTable& R = rule_tab();
            const double z = r * inv_beta, lz = log(z);
            const Solved s0 = plain_solve(nu, z, L, Lq, R, s_tab);
            // the same expression as k_matern, so that C is bit-identical with or without the derivatives
            double hs0 = s0.p.h * sum_f64(nu, z, s0.p, s0.E, s0.Ei, s0.Sr, s_tab);
            hs0 = fma(hs0, s0.dlo, hs0);
            vc = sigma2 * exp(pref + nu * lz + (s0.delta - z)) * hs0;
            if (ob) {
                const Solved s1 = plain_solve(nu1, z, L, Lq, R, s_tab);
                const double hs1 = s1.p.h * sum_f64(nu1, z, s1.p, s1.E, s1.Ei, s1.Sr, s_tab);
                vb = sigma2 * inv_beta * exp(pref + (nu + 1.0) * lz + (s1.delta - z)) * fma(hs1, s1.dlo, hs1);
            }
            if (on) {
                const Solved sd = dnu_solve(nu, z, s0.p.t0, L, Lq, R, s_tab);
                vn = vc * (lz - kLn2 - psi) +
                     sigma2 * exp(pref + nu * lz + (sd.delta - z)) * (sd.p.h * sum_dnu_f64(nu, sd.p, sd.A, sd.B, s_tab));
            }
        }
        const int64_t o = base + il + jl * mI;
        if (oc) oc[o] = (OutT)vc;
        if (ob) ob[o] = (OutT)vb;
        if (on) on[o] = (OutT)vn;
    }
}

}  // namespace bk

using namespace bk;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" const char* bk_status_str(int status)
{
    switch (status) {
    case BK_OK: return "BK_OK";
    case BK_EINVAL: return "BK_EINVAL: invalid argument";
    case BK_EHIP: return "BK_EHIP: HIP runtime error";
    case BK_ENOMEM: return "BK_ENOMEM: workspace too small or allocation failed";
    case BK_ENOMODEL: return "BK_ENOMODEL: learned form requested without a trained model";
    case BK_EIO: return "BK_EIO: model file error";
    case BK_ENOTPD: return "BK_ENOTPD: covariance matrix not positive definite";
    default: return "unknown bk_status";
    }
}

extern "C" int bk_version(void) { return 10000; }

extern "C" int bk_besselk(const double* nu, const double* x, double* out, int64_t n, hipStream_t stream)
{
    bk_params p;
    memset(&p, 0, sizeof(p));
    p.mode = BK_PLAIN_F64;
    return bk_besselk_ex(nu, x, out, n, &p, stream);
}

// One kernel between the caller's optional event pair.
template <typename K, typename... A>
static int launch_timed(const bk_params* prm, K k, dim3 grid, dim3 block, hipStream_t stream, A&&... a)
{
    if (mark_kernel_event(prm, 0, stream) != hipSuccess) return BK_EHIP;
    const int st = launch(k, grid, block, stream, std::forward<A>(a)...);
    if (st != BK_OK) return st;
    return mark_kernel_event(prm, 1, stream) == hipSuccess ? BK_OK : BK_EHIP;
}

extern "C" int bk_besselk_ex(const double* nu, const double* x, double* out, int64_t n,
                             const bk_params* prm, hipStream_t stream)
{
    if (!prm || n < 0) return BK_EINVAL;
    if (n == 0) return BK_OK;
    if (!nu || !x || !out) return BK_EINVAL;
    if (prm->result < BK_RESULT_K || prm->result > BK_RESULT_LOG) return BK_EINVAL;
    if (prm->L_window < 0.0 || prm->L_quad < 0.0) return BK_EINVAL;
    double L, Lq;
    resolve_thresholds(prm->mode, prm->L_window, prm->L_quad, &L, &Lq);
    const int64_t blocks = (n + kSolveBlock - 1) / kSolveBlock;
    if (blocks > 0x7fffffffLL) return BK_EINVAL;
    switch (prm->mode) {
    case BK_PLAIN_F64:
        return launch_timed(prm, k_besselk<BK_PLAIN_F64>, dim3((unsigned)blocks), dim3(kSolveBlock), stream, nu, x,
                            out, n, prm->result, L, Lq, prm->stats);
    case BK_MIXED_F32C:
        return launch_timed(prm, k_besselk<BK_MIXED_F32C>, dim3((unsigned)blocks), dim3(kSolveBlock), stream, nu, x,
                            out, n, prm->result, L, Lq, prm->stats);
    case BK_LEARNED:
        return bk_besselk_learned(nu, x, out, n, prm, L, Lq, stream);
    case BK_PAPER_REFINED: {
        if (prm->bins < 0 || prm->bins > 100000 || prm->t_upper < 0.0) return BK_EINVAL;
        const int64_t b256 = (n + 255) / 256;
        return launch_timed(prm, k_besselk_paper, dim3((unsigned)b256), dim3(256), stream, nu, x, out, n,
                            prm->result, prm->bins > 0 ? prm->bins : kPaperBins,
                            prm->t_upper > 0.0 ? prm->t_upper : kPaperT, prm->stats);
    }
    default:
        return BK_EINVAL;
    }
}

extern "C" int bk_window(const double* nu, const double* x, double* t_lo, double* t_hi, int32_t* nodes,
                         int64_t n, double L_window, double L_quad, hipStream_t stream)
{
    if (n < 0 || L_window < 0.0 || L_quad < 0.0) return BK_EINVAL;
    if (n == 0) return BK_OK;
    if (!nu || !x || !t_lo || !t_hi || !nodes) return BK_EINVAL;
    double L, Lq;
    resolve_thresholds(BK_MIXED_F32C, L_window, L_quad, &L, &Lq);
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL) return BK_EINVAL;
    return launch(k_window, dim3((unsigned)blocks), dim3(256), stream, nu, x, t_lo, t_hi, nodes, n, L, Lq);
}

extern "C" int64_t bk_matern_out_elems(int64_t n, int32_t tile_size, int32_t lower_only)
{
    if (n < 0 || tile_size <= 0) return -1;
    if (n == 0) return 0;
    int64_t ts = tile_size, T = (n + ts - 1) / ts;
    if (!lower_only) return n * n;
    return tile_offset(n, ts, T, 1, T - 1, T - 1) + (n - (T - 1) * ts) * (n - (T - 1) * ts);
}

extern "C" int64_t bk_matern_tile_offset(int64_t n, int32_t tile_size, int32_t lower_only, int32_t I, int32_t J)
{
    if (n <= 0 || tile_size <= 0) return -1;
    int64_t ts = tile_size, T = (n + ts - 1) / ts;
    if (I < 0 || J < 0 || I >= T || J >= T) return -1;
    if (lower_only && J > I) return -1;
    return tile_offset(n, ts, T, lower_only ? 1 : 0, I, J);
}

// Matern tiles of the plain, mixed and paper forms: launches of at most 2^23
// workgroups (below 2^31 work-items each); the caller's event pair, if any,
// brackets them all.
template <int MODE, typename OutT>
static int launch_matern(const bk_locs* locs, const bk_params* prm, const TileGeom& g, int64_t ntiles,
                         double L, double Lq, void* out, hipStream_t stream)
{
    const double nu = prm->nu;
    const double pref = (1.0 - nu) * kLn2 - lgamma(nu);
    const int64_t wg_per_tile = (int64_t)g.rb_per_tile * g.cb_per_tile;
    const int64_t max_wg = 1LL << 23;
    const int64_t tiles_per_launch = max_wg / wg_per_tile > 0 ? max_wg / wg_per_tile : 1;
    const int bins = prm->bins > 0 ? prm->bins : kPaperBins;
    const double T = prm->t_upper > 0.0 ? prm->t_upper : kPaperT;
    if (mark_kernel_event(prm, 0, stream) != hipSuccess) return BK_EHIP;
    for (int64_t t0 = 0; t0 < ntiles; t0 += tiles_per_launch) {
        const int64_t nt = ntiles - t0 < tiles_per_launch ? ntiles - t0 : tiles_per_launch;
        const dim3 grid((unsigned)(nt * wg_per_tile));
        const int st = prm->stats
            ? launch(k_matern<MODE, OutT, true>, grid, dim3(256), stream, locs->x, locs->y, g, t0, prm->sigma2,
                     1.0 / prm->beta, nu, pref, L, Lq, bins, T, (OutT*)out, prm->stats)
            : launch(k_matern<MODE, OutT, false>, grid, dim3(256), stream, locs->x, locs->y, g, t0, prm->sigma2,
                     1.0 / prm->beta, nu, pref, L, Lq, bins, T, (OutT*)out, prm->stats);
        if (st != BK_OK) return st;
    }
    return mark_kernel_event(prm, 1, stream) == hipSuccess ? BK_OK : BK_EHIP;
}

namespace bk {

int matern_tiles_dispatch(const bk_locs* locs, const bk_params* prm, int32_t tile_size, int32_t lower_only,
                          void* out, void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (!locs || !prm || tile_size <= 0 || locs->n < 0) return BK_EINVAL;
    if (!(prm->beta > 0.0) || !(prm->nu > 0.0) || !(prm->sigma2 >= 0.0) || isinf(prm->nu) || isinf(prm->beta))
        return BK_EINVAL;
    if (prm->out_dtype != BK_OUT_F64 && prm->out_dtype != BK_OUT_F32) return BK_EINVAL;
    if (prm->L_window < 0.0 || prm->L_quad < 0.0) return BK_EINVAL;
    if (locs->n == 0) return BK_OK;
    if (!locs->x || !locs->y || !out) return BK_EINVAL;
    TileGeom g;
    g.n = locs->n;
    g.ts = tile_size;
    g.T = (int32_t)((locs->n + tile_size - 1) / tile_size);
    g.lower = lower_only ? 1 : 0;
    g.rb_per_tile = (tile_size + kRowsPerWave - 1) / kRowsPerWave;
    g.cb_per_tile = (tile_size + kColsPerGroup - 1) / kColsPerGroup;
    const int64_t T = g.T;
    const int64_t ntiles = g.lower ? T * (T + 1) / 2 : T * T;
    double L, Lq;
    resolve_thresholds(prm->mode, prm->L_window, prm->L_quad, &L, &Lq);
    const bool f32 = prm->out_dtype == BK_OUT_F32;
    switch (prm->mode) {
    case BK_PLAIN_F64:
        return f32 ? launch_matern<BK_PLAIN_F64, float>(locs, prm, g, ntiles, L, Lq, out, stream)
                   : launch_matern<BK_PLAIN_F64, double>(locs, prm, g, ntiles, L, Lq, out, stream);
    case BK_MIXED_F32C:
        return f32 ? launch_matern<BK_MIXED_F32C, float>(locs, prm, g, ntiles, L, Lq, out, stream)
                   : launch_matern<BK_MIXED_F32C, double>(locs, prm, g, ntiles, L, Lq, out, stream);
    case BK_LEARNED:
        return bk_matern_learned(locs, prm, tile_size, lower_only, out, L, Lq, workspace, workspace_bytes, stream);
    case BK_PAPER_REFINED:
        if (prm->bins < 0 || prm->bins > 100000 || prm->t_upper < 0.0) return BK_EINVAL;
        return f32 ? launch_matern<BK_PAPER_REFINED, float>(locs, prm, g, ntiles, L, Lq, out, stream)
                   : launch_matern<BK_PAPER_REFINED, double>(locs, prm, g, ntiles, L, Lq, out, stream);
    default:
        return BK_EINVAL;
    }
}

}  // namespace bk

extern "C" int bk_matern_tiles(const bk_locs* locs, const bk_params* prm, int32_t tile_size,
                               int32_t lower_only, void* out, hipStream_t stream)
{
    if (!prm) return BK_EINVAL;
    return matern_tiles_dispatch(locs, prm, tile_size, lower_only, out, prm->workspace, prm->workspace_bytes,
                                 stream);
}

// Digamma psi(v), v > 0, on the host in long double: shift up with
// psi(v) = psi(v + 1) - 1/v until v >= 12, then the asymptotic expansion
// ln v - 1/(2v) - 1/(12 v^2) + 1/(120 v^4) - 1/(252 v^6) + 1/(240 v^8) - 1/(132 v^10)
// + 691/(32760 v^12) (Abramowitz & Stegun 6.3.18); the first omitted term,
// 1/(12 v^14), is below 3e-17 of psi(12).
static double digamma_host(double v)
{
    long double t = v, acc = 0.0L;
    for (; t < 12.0L; t += 1.0L) acc -= 1.0L / t;
    const long double w = 1.0L / (t * t);
    const long double tail =
        w * (1.0L / 12 - w * (1.0L / 120 - w * (1.0L / 252 - w * (1.0L / 240 - w * (1.0L / 132 - w * (691.0L / 32760))))));
    return (double)(acc + logl(t) - 0.5L / t - tail);
}

static int check_deriv_params(const bk_params* prm, bk_params* use)
{
    if (prm) *use = *prm;
    else memset(use, 0, sizeof(*use));
    if (use->mode != BK_PLAIN_F64) return BK_EINVAL;
    if (use->result != BK_RESULT_K && use->result != BK_RESULT_SCALED) return BK_EINVAL;
    if (use->L_window < 0.0 || use->L_quad < 0.0) return BK_EINVAL;
    return BK_OK;
}

extern "C" int bk_besselk_deriv(const double* nu, const double* x, double* k, double* dk_dx, double* dk_dnu,
                                int64_t n, const bk_params* prm, hipStream_t stream)
{
    bk_params p;
    if (n < 0) return BK_EINVAL;
    int st = check_deriv_params(prm, &p);
    if (st != BK_OK) return st;
    if (n == 0) return BK_OK;
    if (!nu || !x || (!k && !dk_dx && !dk_dnu)) return BK_EINVAL;
    double L, Lq;
    resolve_thresholds(BK_PLAIN_F64, p.L_window, p.L_quad, &L, &Lq);
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL) return BK_EINVAL;
    return launch(k_besselk_deriv, dim3((unsigned)blocks), dim3(256), stream, nu, x, k, dk_dx, dk_dnu, n, p.result,
                  L, Lq, p.stats);
}

template <typename OutT>
static int launch_matern_grad(const bk_locs* locs, const bk_params* prm, const TileGeom& g, int64_t ntiles,
                              double L, double Lq, void* c, void* db, void* dn, hipStream_t stream)
{
    const double nu = prm->nu;
    const double pref = (1.0 - nu) * kLn2 - lgamma(nu);
    const double psi = digamma_host(nu);
    const int64_t wg_per_tile = (int64_t)g.rb_per_tile * g.cb_per_tile;
    const int64_t max_wg = 1LL << 23;
    const int64_t tiles_per_launch = max_wg / wg_per_tile > 0 ? max_wg / wg_per_tile : 1;
    for (int64_t t0 = 0; t0 < ntiles; t0 += tiles_per_launch) {
        const int64_t nt = ntiles - t0 < tiles_per_launch ? ntiles - t0 : tiles_per_launch;
        const int st = launch(k_matern_grad<OutT>, dim3((unsigned)(nt * wg_per_tile)), dim3(256), stream, locs->x,
                              locs->y, g, t0, prm->sigma2, 1.0 / prm->beta, nu, pref, psi, L, Lq, (OutT*)c,
                              (OutT*)db, (OutT*)dn);
        if (st != BK_OK) return st;
    }
    return BK_OK;
}

extern "C" int bk_matern_grad_tiles(const bk_locs* locs, const bk_params* prm, int32_t tile_size, int32_t lower_only,
                                    void* c, void* dc_dbeta, void* dc_dnu, hipStream_t stream)
{
    if (!locs || !prm || tile_size <= 0 || locs->n < 0) return BK_EINVAL;
    if (prm->mode != BK_PLAIN_F64) return BK_EINVAL;
    if (!(prm->beta > 0.0) || !(prm->nu > 0.0) || !(prm->sigma2 >= 0.0) || isinf(prm->nu) || isinf(prm->beta))
        return BK_EINVAL;
    if (prm->out_dtype != BK_OUT_F64 && prm->out_dtype != BK_OUT_F32) return BK_EINVAL;
    if (prm->L_window < 0.0 || prm->L_quad < 0.0) return BK_EINVAL;
    if (locs->n == 0) return BK_OK;
    if (!locs->x || !locs->y || (!c && !dc_dbeta && !dc_dnu)) return BK_EINVAL;
    TileGeom g;
    g.n = locs->n;
    g.ts = tile_size;
    g.T = (int32_t)((locs->n + tile_size - 1) / tile_size);
    g.lower = lower_only ? 1 : 0;
    g.rb_per_tile = (tile_size + kRowsPerWave - 1) / kRowsPerWave;
    g.cb_per_tile = (tile_size + kColsPerGroup - 1) / kColsPerGroup;
    const int64_t T = g.T;
    const int64_t ntiles = g.lower ? T * (T + 1) / 2 : T * T;
    double L, Lq;
    resolve_thresholds(BK_PLAIN_F64, prm->L_window, prm->L_quad, &L, &Lq);
    if (prm->out_dtype == BK_OUT_F32)
        return launch_matern_grad<float>(locs, prm, g, ntiles, L, Lq, c, dc_dbeta, dc_dnu, stream);
    return launch_matern_grad<double>(locs, prm, g, ntiles, L, Lq, c, dc_dbeta, dc_dnu, stream);
}
