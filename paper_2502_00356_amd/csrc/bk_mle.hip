// bk_mle.hip - Gaussian log-likelihood of observations under the Matern
// covariance, and its gradient in (sigma2, beta, nu): the consumer of the
// generated matrix (Sec. III-A; the paper generates Matern matrices for
// likelihood maximisation).
//
//   l = -1/2 z^T Sigma^-1 z - 1/2 log det Sigma - n/2 log(2 pi)
//   dl/dtheta = 1/2 a^T dSigma a - 1/2 tr(Sigma^-1 dSigma),  a = Sigma^-1 z
//
// Sigma (and for the gradient dSigma/dbeta, dSigma/dnu) comes from this library's
// Matern kernels as one full column-major tile; the Cholesky factorisation, the
// triangular solves and the inverse are rocSOLVER's (potrf, potrs, potri); the
// log-determinant, the dot product and the fused trace / quadratic-form pass over
// the lower triangles are this file's kernels (deterministic two-stage sums).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "../../include/besselk.h"
#include "bk_internal.hpp"

namespace bk {

constexpr int kRedBlock = 256;
constexpr int64_t kMleMaxN = 46340;     // n * n stays below 2^31 (rocSOLVER's 32-bit sizes)

// Sum of one double per thread over a block of kRedBlock threads; result in thread 0.
__device__ double block_sum(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedBlock / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Stage 1 of log det: partial sums of log L_ii over a grid-stride range.
__global__ __launch_bounds__(kRedBlock) void k_logdiag(const double* __restrict__ A, int64_t n,
                                                      double* __restrict__ part)
{
    __shared__ double red[kRedBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedBlock)
        s += log(A[i + i * n]);
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Stage 1 of a dot product u^T v.
__global__ __launch_bounds__(kRedBlock) void k_dot(const double* __restrict__ u, const double* __restrict__ v,
                                                  int64_t n, double* __restrict__ part)
{
    __shared__ double red[kRedBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedBlock)
        s += u[i] * v[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Stage 1 of the gradient terms, one block per column j, over the lower
// triangle i >= j of the symmetric matrices (weight 2 off the diagonal):
//   part[4 j + 0] = sum_i w a_i a_j dB_ij        part[4 j + 1] = sum_i w Sinv_ij dB_ij
//   part[4 j + 2] = sum_i w a_i a_j dN_ij        part[4 j + 3] = sum_i w Sinv_ij dN_ij
// Sinv holds the inverse in its lower triangle (potri); columns are coalesced.
__global__ __launch_bounds__(kRedBlock) void k_grad_terms(const double* __restrict__ Sinv,
                                                         const double* __restrict__ dB,
                                                         const double* __restrict__ dN,
                                                         const double* __restrict__ a, int64_t n,
                                                         double* __restrict__ part)
{
    __shared__ double red[kRedBlock / 64];
    const int64_t j = blockIdx.x;
    const double aj = a[j];
    double qb = 0.0, tb = 0.0, qn = 0.0, tn = 0.0;
    for (int64_t i = j + threadIdx.x; i < n; i += kRedBlock) {
        const int64_t o = i + j * n;
        const double w = (i == j) ? 1.0 : 2.0;
        const double wa = w * a[i] * aj, ws = w * Sinv[o];
        qb += wa * dB[o];
        tb += ws * dB[o];
        qn += wa * dN[o];
        tn += ws * dN[o];
    }
    double r;
    r = block_sum(qb, red); if (threadIdx.x == 0) part[4 * j + 0] = r;
    r = block_sum(tb, red); if (threadIdx.x == 0) part[4 * j + 1] = r;
    r = block_sum(qn, red); if (threadIdx.x == 0) part[4 * j + 2] = r;
    r = block_sum(tn, red); if (threadIdx.x == 0) part[4 * j + 3] = r;
}

// Stage 2: res[k] = sum_p part[p * stride + k] for k < stride, one block, fixed order.
__global__ __launch_bounds__(kRedBlock) void k_finish(const double* __restrict__ part, int64_t np, int stride,
                                                     double* __restrict__ res)
{
    __shared__ double red[kRedBlock / 64];
    for (int k = 0; k < stride; ++k) {
        double s = 0.0;
        for (int64_t p = threadIdx.x; p < np; p += kRedBlock) s += part[p * stride + k];
        const double t = block_sum(s, red);
        if (threadIdx.x == 0) res[k] = t;
    }
}

// One rocBLAS handle per device, created on first use and kept for the life of
// the process; calls on one device are serialised by its mutex (the handle's
// stream is per call).
struct HandleSlot {
    std::mutex mu;
    rocblas_handle h = nullptr;
};

static HandleSlot* handle_slot(int dev)
{
    static HandleSlot slots[64];
    if (dev < 0 || dev >= 64) return nullptr;
    return &slots[dev];
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct MleLayout {
    size_t S, dB, dN, a, part, res, info, mws, total;
};

static MleLayout mle_layout(int64_t n, int with_grad)
{
    MleLayout L;
    const size_t mat = align256(sizeof(double) * (size_t)n * (size_t)n);
    const int64_t np = n > 1024 ? n : 1024;
    size_t o = 0;
    L.S = o; o += mat;
    L.dB = o; o += with_grad ? mat : 0;
    L.dN = o; o += with_grad ? mat : 0;
    L.a = o; o += align256(sizeof(double) * (size_t)n);
    L.part = o; o += align256(sizeof(double) * 4 * (size_t)np);
    L.res = o; o += 256;
    L.info = o; o += 256;
    L.mws = o; o += matern_learned_workspace_bytes(n, (int32_t)n, 0);   // for a learned-form Sigma
    L.total = o;
    return L;
}

}  // namespace bk

using namespace bk;

extern "C" size_t bk_matern_loglik_workspace_bytes(int64_t n, int32_t with_grad)
{
    if (n <= 0 || n > kMleMaxN) return 0;
    return mle_layout(n, with_grad ? 1 : 0).total;
}

extern "C" int bk_matern_loglik(const bk_locs* locs, const double* z, const bk_params* prm, int32_t with_grad,
                                double* result, void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (!locs || !prm || !z || !result || !workspace) return BK_EINVAL;
    const int64_t n = locs->n;
    if (n <= 0 || n > kMleMaxN || !locs->x || !locs->y) return BK_EINVAL;
    if (with_grad && prm->mode != BK_PLAIN_F64) return BK_EINVAL;
    if (!(prm->beta > 0.0) || !(prm->nu > 0.0) || !(prm->sigma2 > 0.0)) return BK_EINVAL;
    const MleLayout L = mle_layout(n, with_grad ? 1 : 0);
    if (workspace_bytes < L.total) return BK_ENOMEM;
    char* ws = (char*)workspace;
    double* S = (double*)(ws + L.S);
    double* dB = (double*)(ws + L.dB);
    double* dN = (double*)(ws + L.dN);
    double* a = (double*)(ws + L.a);
    double* part = (double*)(ws + L.part);
    double* res = (double*)(ws + L.res);
    rocblas_int* info = (rocblas_int*)(ws + L.info);

    // Sigma (and its derivatives) as one full column-major n x n tile, FP64
    bk_params p = *prm;
    p.out_dtype = BK_OUT_F64;
    p.workspace = ws + L.mws;
    p.workspace_bytes = L.total - L.mws;
    int st = with_grad ? bk_matern_grad_tiles(locs, &p, (int32_t)n, 0, S, dB, dN, stream)
                       : bk_matern_tiles(locs, &p, (int32_t)n, 0, S, stream);
    if (st != BK_OK) return st;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BK_EHIP;
    HandleSlot* hs = handle_slot(dev);
    if (!hs) return BK_EHIP;
    std::lock_guard<std::mutex> lk(hs->mu);
    if (!hs->h && rocblas_create_handle(&hs->h) != rocblas_status_success) {
        hs->h = nullptr;
        return BK_EHIP;
    }
    rocblas_handle h = hs->h;
    if (rocblas_set_stream(h, stream) != rocblas_status_success) return BK_EHIP;
    const rocblas_int ni = (rocblas_int)n;

    if (rocsolver_dpotrf(h, rocblas_fill_lower, ni, S, ni, info) != rocblas_status_success) return BK_EHIP;
    if (hipMemcpyAsync(a, z, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess) return BK_EHIP;
    if (rocsolver_dpotrs(h, rocblas_fill_lower, ni, 1, S, ni, a, ni) != rocblas_status_success) return BK_EHIP;

    const int nb = (int)((n + kRedBlock - 1) / kRedBlock < 1024 ? (n + kRedBlock - 1) / kRedBlock : 1024);
    st = launch(k_logdiag, dim3(nb), dim3(kRedBlock), stream, (const double*)S, n, part);
    if (st == BK_OK) st = launch(k_finish, dim3(1), dim3(kRedBlock), stream, (const double*)part, (int64_t)nb, 1, res + 0);
    if (st == BK_OK) st = launch(k_dot, dim3(nb), dim3(kRedBlock), stream, z, (const double*)a, n, part);
    if (st == BK_OK) st = launch(k_finish, dim3(1), dim3(kRedBlock), stream, (const double*)part, (int64_t)nb, 1, res + 1);
    if (st != BK_OK) return st;
    if (with_grad) {
        if (rocsolver_dpotri(h, rocblas_fill_lower, ni, S, ni, info + 1) != rocblas_status_success) return BK_EHIP;
        st = launch(k_grad_terms, dim3((unsigned)n), dim3(kRedBlock), stream, (const double*)S, (const double*)dB,
                    (const double*)dN, (const double*)a, n, part);
        if (st == BK_OK) st = launch(k_finish, dim3(1), dim3(kRedBlock), stream, (const double*)part, n, 4, res + 2);
        if (st != BK_OK) return st;
    }
    double hres[6] = {0, 0, 0, 0, 0, 0};
    rocblas_int hinfo[2] = {0, 0};
    if (hipMemcpyAsync(hres, res, sizeof(hres), hipMemcpyDeviceToHost, stream) != hipSuccess) return BK_EHIP;
    if (hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, stream) != hipSuccess) return BK_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return BK_EHIP;
    if (hinfo[0] != 0 || (with_grad && hinfo[1] != 0)) return BK_ENOTPD;
    const double logdet = 2.0 * hres[0], quad = hres[1];
    result[0] = -0.5 * quad - 0.5 * logdet - 0.5 * (double)n * 1.8378770664093454836;   // log(2 pi)
    if (with_grad) {
        result[1] = 0.5 * (quad - (double)n) / prm->sigma2;
        result[2] = 0.5 * hres[2] - 0.5 * hres[3];
        result[3] = 0.5 * hres[4] - 0.5 * hres[5];
    }
    return BK_OK;
}
