/*
 * besselk.h - C ABI of libbesselk.so: the modified Bessel function of the second
 * kind K_nu(x), evaluated on MI355X (gfx950) by finite-window trapezoid
 * quadrature of its integral form, standalone and fused into tiled Matern
 * covariance generation (arXiv 2502.00356, "GPU-Accelerated Modified Bessel
 * Function of the Second Kind for Gaussian Processes").
 *
 * Conventions shared by every entry point
 *  - Array arguments are DEVICE pointers owned by the caller, unless a comment
 *    says "host". The library never frees or retains them.
 *  - Calls only enqueue work on the given HIP stream (NULL = the default stream)
 *    and return without synchronising, unless documented otherwise.
 *  - The return value is a bk_status; arguments are checked before anything is
 *    enqueued, and no call aborts or throws. n == 0 is valid and enqueues nothing.
 *  - Element-level domain (as scipy.special.kv): x < 0 or NaN -> NaN, x == 0 ->
 *    +inf, NaN order -> NaN; a negative order is replaced by its absolute value
 *    because K_{-nu} = K_nu (the integrand of Sec. IV-B is even in nu).
 */
#ifndef BESSELK_H
#define BESSELK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BK_OK = 0,
    BK_EINVAL = 1,   /* bad argument: null pointer, negative size, bad parameter */
    BK_EHIP = 2,     /* a HIP runtime call or kernel launch failed */
    BK_ENOMEM = 3,   /* workspace too small or allocation failed */
    BK_ENOMODEL = 4, /* BK_LEARNED without a trained model */
    BK_EIO = 5,      /* model file could not be read or written, or is malformed */
    BK_ENOTPD = 6    /* covariance matrix not positive definite (Cholesky failed) */
} bk_status;

/* Evaluation form.
 *  BK_PLAIN_F64  : per-entry peak and window solve in FP64 (the bracket/Newton
 *                  search of Sec. IV-B), node count from the trapezoid strip
 *                  bound, FP64 node terms and FP64 accumulation. bk_besselk and
 *                  bk_besselk_ex take Temme's series with the forward recurrence
 *                  instead (Sec. IV-A, the paper's branch for x < 0.1) where
 *                  x < 0.1 and K_nu(x) lies far inside the double range.
 *  BK_MIXED_F32C : the same FP64 solve; node exponents formed in FP64 without
 *                  cancellation, exponentials in FP32, Kahan-compensated FP32 sum,
 *                  FP64 prefactor. Looser window (relative error ~1e-7 class).
 *                  Like BK_PLAIN_F64, Temme's series (FP64) where x < 0.1.
 *  BK_LEARNED    : a 2-64-64-3 MLP on (log10 x, nu) predicts the window and node
 *                  count in place of the solve (the count is raised to the
 *                  strip-bound rule's if lower); the standalone form reads the
 *                  prediction from the model's cells (bk_model_get_cells), the
 *                  Matern form from a table along log10 x at its nu; terms as in
 *                  BK_MIXED_F32C; entries
 *                  outside the model's training box, or whose window fails the
 *                  tail check, are recomputed with BK_MIXED_F32C.
 *  BK_PAPER_REFINED: the paper's refined algorithm (Sec. IV-C, Alg. 2), FP64:
 *                  for x < 0.1 Temme's series with the forward recurrence
 *                  (Sec. IV-A); otherwise the fixed window [0, t_upper] (default
 *                  9) with b bins (default 40), scaled by the largest node value.
 *                  Its accuracy for x >= 0.1 is the paper's trade-off of b against
 *                  x (large x needs many bins). */
typedef enum { BK_PLAIN_F64 = 0, BK_MIXED_F32C = 1, BK_LEARNED = 2, BK_PAPER_REFINED = 3 } bk_mode;

/* Matern output element type. */
typedef enum { BK_OUT_F64 = 0, BK_OUT_F32 = 1 } bk_dtype;

/* What bk_besselk_ex writes per entry. */
typedef enum { BK_RESULT_K = 0, BK_RESULT_SCALED = 1, BK_RESULT_LOG = 2 } bk_result;

/* Indices into the optional statistics array (device, unsigned 64-bit counters,
 * accumulated, never cleared by the library). bk_besselk_ex and bk_matern_tiles
 * fill them for every form (the paper form counts its integral branch only).
 * Counting costs time (the Matern kernels have counting variants), so time
 * calls without it. */
enum {
    BK_STAT_ENTRIES = 0,      /* entries evaluated by quadrature               */
    BK_STAT_NODES = 1,        /* sum over entries of (N + 1) trapezoid nodes    */
    BK_STAT_FB_RANGE = 2,     /* learned: (nu, x) outside the training box      */
    BK_STAT_FB_TAIL = 3,      /* learned: an end node carried too much weight   */
    BK_STAT_NODE_RAISED = 4,  /* learned: predicted N below the strip-bound rule
                                 for the predicted window, raised (not a fallback) */
    BK_STAT_FB_NONFINITE = 5, /* learned: non-finite prediction or sum          */
    BK_STAT_FB_NODES = 6,     /* learned: nodes of the entries the fallback launch
                                 recomputed (already counted in BK_STAT_NODES,
                                 as are those entries in BK_STAT_ENTRIES)     */
    BK_STAT_LANE_SLOTS = 7,   /* main kernel (plain, mixed, learned forms): sum over
                                 its waves, per group of entries a wave walks side
                                 by side, of 64 x the largest N + 1 among them: the
                                 lane-node slots the node walk occupies. Nodes of the
                                 main kernel / LANE_SLOTS is the share that did work */
    BK_STATS_LEN = 8
};

typedef struct bk_model bk_model;

/* Per-call options. Zero-initialise and set what you need.
 *  L_window : window threshold L of Sec. IV-B, [t0,t1] = {t : g(t) >= g(t_max) - L}.
 *             0 selects the form's default (36 for BK_PLAIN_F64, 15 otherwise).
 *  L_quad   : node-count target: the step keeps the strip-bound discretisation
 *             error near exp(-L_quad). 0 selects 35 (plain) or 14.5 (others).
 *  result   : bk_result, for bk_besselk_ex only.
 *  sigma2, beta, nu : Matern parameters theta = (sigma^2, beta, nu) of Sec. III-A
 *             (sigma2 >= 0, beta > 0, nu > 0), for bk_matern_tiles only.
 *  out_dtype: bk_dtype of the Matern output, for bk_matern_tiles only.
 *  model    : trained model, required for BK_LEARNED.
 *  stats    : device array of BK_STATS_LEN counters, or NULL.
 *  workspace, workspace_bytes : device scratch owned by the caller, for BK_LEARNED
 *             only: bk_besselk_ex needs bk_workspace_bytes(n) bytes (the fallback
 *             queue), bk_matern_tiles bk_matern_workspace_bytes(n, tile_size,
 *             lower_only) bytes (window table, interval plans, fallback bitmap).
 *             Its contents need not be initialised and are undefined afterwards;
 *             calls that share a workspace must not overlap.
 *  kernel_events : optional pair of hipEvent_t handles (cast to void*), owned by
 *             the caller. When both are set, bk_besselk_ex and bk_matern_tiles
 *             record [0] just before and [1] just after the form's main kernel
 *             launches on the call's stream, so that they can be timed alone
 *             (BK_LEARNED's table, plan, reset and fallback launches fall outside
 *             the pair). A failed record returns BK_EHIP. */
typedef struct {
    int32_t mode;
    int32_t result;
    int32_t out_dtype;
    int32_t bins;        /* BK_PAPER_REFINED: number of bins b (0 selects 40) */
    double L_window;
    double L_quad;
    double sigma2;
    double beta;
    double nu;
    const bk_model* model;
    unsigned long long* stats;
    void* workspace;
    size_t workspace_bytes;
    double t_upper;      /* BK_PAPER_REFINED: upper end of the window (0 selects 9) */
    void* kernel_events[2];
} bk_params;

/* Human-readable name of a status code (static string). */
const char* bk_status_str(int status);

/* Library version as major*10000 + minor*100 + patch. */
int bk_version(void);

/* K_nu(x) for n pairs in plain FP64 (BK_PLAIN_F64, default window).
 * Defines: the integral K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt of
 * Sec. IV-B, evaluated as g(t_max) + log of the trapezoid sum of
 * exp(g(t_m) - g(t_max)) over the window (Sec. IV-B, Eq. "refined").
 * nu, x : n doubles each (device). out : n doubles (device), K_nu(x).
 * Past x ~ 708 K underflows double; use bk_besselk_ex with BK_RESULT_SCALED. */
int bk_besselk(const double* nu, const double* x, double* out, int64_t n, hipStream_t stream);

/* K_nu(x) with options: any bk_mode, and result K, e^x K or log K.
 * Same layout and ownership as bk_besselk. Returns BK_ENOMODEL for BK_LEARNED
 * without params->model, BK_ENOMEM if the workspace is too small. */
int bk_besselk_ex(const double* nu, const double* x, double* out, int64_t n,
                  const bk_params* params, hipStream_t stream);

/* Device workspace that BK_LEARNED needs for n entries (bytes). */
size_t bk_workspace_bytes(int64_t n);

/* Location set for Matern generation: n points as FP64 structure-of-arrays,
 * x[i], y[i] (device). Sec. IV-C, Alg. 3 passes locations as coordinate vectors. */
typedef struct {
    const double* x;
    const double* y;
    int64_t n;
} bk_locs;

/* Tiled Matern covariance matrix (Sec. III-A formula; Alg. 3 per tile):
 *   C(r) = sigma2 / (2^(nu-1) Gamma(nu)) (r/beta)^nu K_nu(r/beta),  C(0) = sigma2,
 * with r the FP64 Euclidean distance between locations i and j and an exactly
 * zero distance giving sigma2 (Alg. 3).
 * Tiling: T = ceil(n / tile_size) tile rows and columns; tile (I, J) covers rows
 * [I*ts, min(n,(I+1)*ts)) and columns [J*ts, ...). With lower_only != 0 the tiles
 * with J <= I are stored, else all tiles. Tiles are stored one after another in
 * J-major order (J = 0, 1, ...; within a column I ascending), each m_I x n_J
 * column-major with leading dimension m_I: entry (i, j) of tile (I, J) is at
 * bk_matern_tile_offset(I, J) + i + j * m_I. Diagonal tiles are written in full
 * (both triangles). With tile_size >= n and lower_only == 0 the output is the
 * whole n x n column-major matrix.
 * out : device buffer of bk_matern_out_elems(n, tile_size, lower_only) elements
 *       of params->out_dtype. params->mode selects the form; BK_LEARNED needs a
 *       model and a workspace of bk_matern_workspace_bytes(...) bytes, and only
 *       reads the model, so calls on different streams may share one model. */
int bk_matern_tiles(const bk_locs* locs, const bk_params* params, int32_t tile_size,
                    int32_t lower_only, void* out, hipStream_t stream);

/* Device workspace bk_matern_tiles needs for BK_LEARNED (bytes; the other forms
 * need none): a 128 KiB window table and interval plans for the call's nu, then
 * one bit per wave of 2048 entries (about 1/65536 of an FP32 output). 0 if the
 * sizes are invalid. */
size_t bk_matern_workspace_bytes(int64_t n, int32_t tile_size, int32_t lower_only);

/* bk_matern_tiles for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation, output and arguments, but the learned form's workspace comes from a
 * static device array inside the library, BK_NOALLOC_SCRATCH_BYTES per GPU, set up
 * on the first call on each device and held until the process ends.
 * params->workspace and params->workspace_bytes are ignored. The forms other than
 * BK_LEARNED use no workspace and behave exactly as bk_matern_tiles.
 * Limits and errors: BK_ENOMEM if bk_matern_workspace_bytes(n, tile_size,
 * lower_only) exceeds BK_NOALLOC_SCRATCH_BYTES (about 6.7e10 stored entries with
 * 1,024-tiles; the 316 x 316-point lower-tile build needs 0.42 MiB); BK_EINVAL if a
 * non-NULL stream belongs to another device than the current one; otherwise the
 * statuses of bk_matern_tiles.
 * No call allocates or frees memory. Every call on one GPU uses that GPU's one
 * array (each call clears what it needs), so calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller. */
#define BK_NOALLOC_SCRATCH_BYTES (4u << 20)
int bk_matern_tiles_noalloc(const bk_locs* locs, const bk_params* params, int32_t tile_size,
                            int32_t lower_only, void* out, hipStream_t stream);

/* Number of output elements bk_matern_tiles writes (host computation). */
int64_t bk_matern_out_elems(int64_t n, int32_t tile_size, int32_t lower_only);

/* Element offset of tile (I, J) in the bk_matern_tiles output, or -1 if the tile
 * is not stored or out of range (host computation). */
int64_t bk_matern_tile_offset(int64_t n, int32_t tile_size, int32_t lower_only, int32_t I, int32_t J);

/* Integration window of the plain solver (Sec. IV-B): t_lo, t_hi bound
 * {t : g(t) >= g(t_max) - L_window} (t_lo = 0 when g(0) is above the threshold)
 * and nodes = N, the trapezoid interval count for target exp(-L_quad).
 * These are the training targets of the window-predicting MLP.
 * nu, x : n doubles (device). t_lo, t_hi : n doubles, nodes : n int32 (device).
 * L_window, L_quad >= 0 (0 selects 15 and 14.5). */
int bk_window(const double* nu, const double* x, double* t_lo, double* t_hi, int32_t* nodes,
              int64_t n, double L_window, double L_quad, hipStream_t stream);

/* K_nu(x) and its partial derivatives in x and nu, FP64 (plain solve), for n pairs.
 * Defines (derivatives are the paper's future work, Sec. VI; both come from
 * differentiating the integral of Sec. IV-B under the integral sign):
 *   dK/dx  = -int_0^inf cosh t cosh(nu t) exp(-x cosh t) dt = -(K_{nu-1} + (nu/x) K_nu)
 *   dK/dnu =  int_0^inf t sinh(nu t) exp(-x cosh t) dt  (sign of nu for nu < 0)
 * nu, x : n doubles (device). k, dk_dx, dk_dnu : n doubles each (device) or NULL
 * to skip that output (at least one must be given).
 * params may be NULL (defaults); otherwise mode must be BK_PLAIN_F64, result
 * BK_RESULT_K or BK_RESULT_SCALED (all three outputs multiplied by e^x), and
 * L_window, L_quad, stats are honoured. Special values: x == 0 gives +inf, -inf
 * and +-inf (0 for nu == 0); x == +inf gives 0, -0, 0; NaN or x < 0 gives NaN. */
int bk_besselk_deriv(const double* nu, const double* x, double* k, double* dk_dx, double* dk_dnu,
                     int64_t n, const bk_params* params, hipStream_t stream);

/* Matern covariance tiles and their partial derivatives in beta and nu (the
 * Sec. III-A formula differentiated; inputs of gradient-based likelihood
 * maximisation). With z = r / beta and c = 2^(1-nu) / Gamma(nu):
 *   C        = sigma2 c z^nu K_nu(z)
 *   dC/dbeta = sigma2 c z^(nu+1) K_{nu-1}(z) / beta
 *   dC/dnu   = C (ln z - ln 2 - psi(nu)) + sigma2 c z^nu dK_nu/dnu(z)
 * and C = sigma2, dC/dbeta = dC/dnu = 0 at r == 0 (dC/dsigma2 is C / sigma2).
 * Same tiling, layout and element type (params->out_dtype) as bk_matern_tiles;
 * params->mode must be BK_PLAIN_F64. c, dc_dbeta, dc_dnu : device buffers of
 * bk_matern_out_elems(...) elements each, or NULL to skip (at least one given). */
int bk_matern_grad_tiles(const bk_locs* locs, const bk_params* params, int32_t tile_size, int32_t lower_only,
                         void* c, void* dc_dbeta, void* dc_dnu, hipStream_t stream);

/* Gaussian log-likelihood of observations z (n doubles, device) at the locations
 * under the Matern covariance Sigma of bk_matern_tiles (Sec. III-A; the matrix the
 * paper generates is the covariance of this likelihood):
 *   l = -1/2 z^T Sigma^-1 z - 1/2 log det Sigma - n/2 log(2 pi),
 * by Sigma = L L^T (rocSOLVER potrf) and a = Sigma^-1 z (potrs). With with_grad != 0
 * also the gradient, from bk_matern_grad_tiles and Sigma^-1 (potri):
 *   dl/dtheta = 1/2 a^T (dSigma/dtheta) a - 1/2 tr(Sigma^-1 dSigma/dtheta),
 * theta = (sigma2, beta, nu); dSigma/dsigma2 = Sigma / sigma2.
 * result : HOST array, result[0] = l and, with the gradient, result[1..3] =
 *          dl/dsigma2, dl/dbeta, dl/dnu.
 * params : sigma2 > 0, beta > 0, nu > 0; mode selects the form that builds Sigma
 *          (BK_LEARNED needs a model); the gradient needs BK_PLAIN_F64.
 * workspace : device scratch of bk_matern_loglik_workspace_bytes(n, with_grad)
 *          bytes (the n x n matrices: 8 n^2 bytes each, three with the gradient).
 * 1 <= n <= 46340. Synchronises the stream (the results are host values).
 * Returns BK_ENOTPD if the Cholesky factorisation fails. Calls on one device are
 * serialised (one rocBLAS handle per device, kept for the life of the process). */
int bk_matern_loglik(const bk_locs* locs, const double* z, const bk_params* params, int32_t with_grad,
                     double* result, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Workspace bytes bk_matern_loglik needs (0 if n is out of range). */
size_t bk_matern_loglik_workspace_bytes(int64_t n, int32_t with_grad);

/* ---------------------------------------------------------------------------
 * Window-predicting MLP (2 -> 64 -> 64 -> 3, ReLU).
 * Inputs u = ((log10 x - cx)/sx, (nu - cnu)/snu); outputs (t_lo/st, t_hi/st, N/sn).
 * Flat FP32 parameter vector of BK_MLP_NPARAM floats, in this order:
 *   W1[64][2], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]   (row-major, W[out][in])
 * ------------------------------------------------------------------------- */
#define BK_MLP_NPARAM 4547

/* Training configuration. */
typedef struct {
    int32_t epochs;        /* passes over the training set                     */
    int32_t batch;         /* minibatch size, 1..65536                         */
    float lr;              /* Adam step size                                   */
    float beta1, beta2;    /* Adam moment decay rates                          */
    float eps;             /* Adam denominator offset                          */
    float tau_lo, tau_hi, tau_n; /* expectile levels of the three outputs      */
    uint64_t seed;         /* initialisation and shuffling seed                */
    double L_window, L_quad; /* window targets (0 selects 15 and 14.5)         */
} bk_train_cfg;

/* Create an empty model (host handle; device memory owned by the model). */
int bk_model_create(bk_model** model);
/* Release a model and its device memory. NULL is accepted. */
void bk_model_destroy(bk_model* model);
/* Load / save a model file (host path). Format: little-endian, magic "BKMLP001",
 * header of doubles (normalisation, training box, margins), then the parameters.
 * bk_model_load synchronises the device. */
int bk_model_load(bk_model* model, const char* path);
int bk_model_save(const bk_model* model, const char* path);

/* Train the model on n (nu, x) pairs (device arrays): targets come from
 * bk_window at cfg's thresholds, then minibatch Adam on the expectile loss.
 * Synchronises the stream; *final_loss (host, may be NULL) receives the mean
 * loss of the last epoch. Sets the training box from the data range, rounded
 * outward to multiples of 1e-3. */
int bk_model_train(bk_model* model, const double* nu, const double* x, int64_t n,
                   const bk_train_cfg* cfg, float* final_loss, hipStream_t stream);

/* Set the safety margins used at inference: t_lo -= d_lo, t_hi += d_hi,
 * N = ceil(N_pred * (1 + eta) + n_add) (host values). */
int bk_model_set_margins(bk_model* model, double d_lo, double d_hi, double eta, double n_add);

/* The four margins (d_lo, d_hi, eta, n_add) into m4 (host). */
int bk_model_get_margins(const bk_model* model, double* m4);

/* What fills the learned form's prediction tables (the standalone cells, their
 * plans, and the Matern window table of each call).
 *  BK_TABLE_NETWORK : the network's predictions (default).
 *  BK_TABLE_SOLVER  : the plain window solver of Sec. IV-B (bk_window at the
 *                     model's training thresholds) at the same points: the same
 *                     kernels without the network, for measuring what the
 *                     network contributes. The margins still apply; set them to
 *                     zero for the solver's windows as they are. */
typedef enum { BK_TABLE_NETWORK = 0, BK_TABLE_SOLVER = 1 } bk_table_source;

/* Select the table source (bk_table_source) and rebuild the prediction cells
 * (synchronous). BK_ENOMODEL if the model has no parameters yet. */
int bk_model_set_table_source(bk_model* model, int32_t source);

/* Copy the flat FP32 parameter vector to host (BK_MLP_NPARAM floats) or set it
 * (setting it, the normalisation or the box rebuilds the prediction cells below
 * and synchronises the device). */
int bk_model_get_params(const bk_model* model, float* host_params);
int bk_model_set_params(bk_model* model, const float* host_params);

/* Normalisation constants: norm[0..7] = cx, sx, cnu, snu, st, sn, (unused) (host). */
int bk_model_get_norm(const bk_model* model, double* norm8);
int bk_model_set_norm(bk_model* model, const double* norm8);

/* Training box: box[0..3] = log10 x min, log10 x max, nu min, nu max (host). */
int bk_model_get_box(const bk_model* model, double* box4);
int bk_model_set_box(bk_model* model, const double* box4);

/* Prediction cells of the learned K_nu form (an implementation choice, not from
 * the paper: the network's two inputs allow tabulating it). The training box is
 * cut into dims[0] cells along log10 x by dims[1] along nu; cell (i, j) has its
 * corners at (box[0] + (i + a) (box[1] - box[0]) / dims[0],
 * box[2] + (j + b) (box[3] - box[2]) / dims[1]), a, b in {0, 1}, and holds the
 * smallest normalised t_lo and the largest t_hi and N that the network predicts
 * at those four corners, then 0: four floats at host[4 (i dims[1] + j)].
 * The cells are rebuilt (synchronously) whenever the parameters, normalisation
 * or box change. dims (host, 2 ints) is always filled; host (cap floats) may be
 * NULL to query dims only; BK_EINVAL if cap < 4 dims[0] dims[1], BK_ENOMODEL
 * before parameters exist. Synchronous copy. */
int bk_model_get_cells(const bk_model* model, float* host, int64_t cap, int32_t* dims);

/* MLP forward pass as used at inference (FP16 matrix-core products with FP32
 * accumulation) on n normalised inputs u (n x 2 floats, device), writing y
 * (n x 3 floats, device): y = W3 relu(W2 relu(W1 u + b1) + b2) + b3. */
int bk_mlp_infer(const bk_model* model, const float* u, float* y, int64_t n, hipStream_t stream);

/* Loss and gradient for one batch in FP32, the kernels training uses:
 * params (BK_MLP_NPARAM floats), u (B x 2), target (B x 3), tau (3) device;
 * grad (BK_MLP_NPARAM floats) and loss (1 float) device outputs, overwritten.
 * Loss = sum_k mean_b |tau_k - [e_bk < 0]| e_bk^2 with e = target - y.
 * scratch: device buffer of at least bk_mlp_grad_scratch_bytes(B) bytes. */
int bk_mlp_grad(const float* params, const float* u, const float* target, const float* tau,
                int64_t B, float* grad, float* loss, void* scratch, size_t scratch_bytes,
                hipStream_t stream);
size_t bk_mlp_grad_scratch_bytes(int64_t B);

/* One Adam update in place on device arrays of length n (Kingma & Ba 2015):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr mhat / (sqrt(vhat) + eps),
 * with mhat = m / (1 - b1^step), vhat = v / (1 - b2^step); step >= 1. */
int bk_adam_step(float* p, const float* g, float* m, float* v, int64_t n, int32_t step,
                 float lr, float beta1, float beta2, float eps, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* BESSELK_H */
