/*
 * klr.h - C ABI of the MI355X rational-program library.
 *
 * The library implements the data-parallel core of the rational-program method for choosing
 * kernel launch parameters (arXiv 1911.02373):
 *   - klr_fit_batched   : step 2 of the paper's six-step algorithm ("Rational function
 *                         estimation") and section "Building a Driver Program: Rational
 *                         function estimation" - least-squares fits of rational functions
 *                         p(D,P)/q(D,P) to sampled low-level metrics;
 *   - klr_eval_argmin   : steps 4 and 5 ("Rational program evaluation", "Selection of optimal
 *                         values of program parameters") - evaluation of the MWP-CWP-style
 *                         cycle estimate built from the fitted metrics over every launch
 *                         configuration, and an exhaustive per-query argmin;
 *   - klr_surrogate_*   : a learned MLP surrogate of the log-cycle estimate with the exact
 *                         rational program as fallback (not in the paper).
 *
 * Conventions
 *   - Array arguments are DEVICE pointers (caller-owned, e.g. torch tensors) unless marked
 *     [host].  The library never frees caller memory.  Every call is asynchronous on `stream`
 *     (a hipStream_t; NULL = the null stream); results are visible after the stream syncs.
 *   - Descriptors live in device memory.  Host-detectable errors (NULL pointers, bad sizes,
 *     invalid hardware constants, too small a workspace) return KLR_E_INVALID or
 *     KLR_E_WORKSPACE immediately and launch nothing.  Descriptor contents are validated on the
 *     device against the array lengths passed in; an invalid descriptor is reported per item
 *     (fit status bit KLR_FIT_BAD_INPUT, program status) and never read out of bounds.
 *   - HIP errors map to KLR_E_HIP with text from klr_last_error.
 *   - Identical inputs give bitwise-identical outputs (no atomics in value reductions).
 *   - One handle per host thread; calls that share a workspace on one stream are ordered by it.
 */
#ifndef KLR_H
#define KLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t klr_status;
#define KLR_OK 0
#define KLR_E_INVALID (-1)      /* bad argument detected on the host; nothing launched */
#define KLR_E_WORKSPACE (-2)    /* workspace too small; nothing launched */
#define KLR_E_HIP (-3)          /* a HIP runtime call failed; see klr_last_error */
#define KLR_E_UNSUPPORTED (-4)  /* valid request outside what the library implements */

#define KLR_MAX_VARS 8          /* variables per fit (data parameters first, then launch) */
#define KLR_N_METRICS 8         /* fitted metrics per rational program */
#define KLR_MAX_NDEG 3          /* highest power of the data size N in an evaluated metric */
#define KLR_MAX_UNKNOWNS 128    /* n_num + n_den - 1 per fit */
#define KLR_MAX_LAUNCH 4        /* launch parameters per configuration */
#define KLR_MAX_SAMPLES 4096    /* samples per fit */

typedef struct klr_handle_s* klr_handle;

/* Create a handle bound to HIP device `device` (makes it current on the calling thread).
 * Owns the last-error text and the tuned launch shapes; allocates no device memory. */
klr_status klr_create(klr_handle* out, int device);
void klr_destroy(klr_handle h);
/* [host] text of the last failure on this handle ("" if none); valid until the next call. */
const char* klr_last_error(klr_handle h);

/* ------------------------------------------------------------------------------------------
 * Fits.  One fit = one low-level metric g_i of one kernel, modelled as the rational function
 * p(x~)/q(x~) of the section "Building a Driver Program: Rational function estimation",
 * with monomial sets given explicitly (this covers the paper's per-variable degree bounds and
 * total-degree sets alike).  Variables are scaled by powers of two, x~_k = x_k * 2^-s_k
 * (exact).  The fit solves the linearised least-squares problem
 *     min_y || A y - f ||_2,   A = [ x~^a (a in numerator set) | -f * x~^b (b in denominator
 *                                   set without its constant row) ]
 * i.e. f*q - p = 0 with q's constant coefficient fixed to 1.
 */
typedef struct {
  int64_t x0;             /* element offset of the fit's samples in X: m rows of v int32      */
  int64_t f0;             /* element offset of its m targets in f (float64)                   */
  int64_t coef0;          /* element offset of its n_num + n_den - 1 output coefficients:     */
                          /*   numerator in set order, then denominator without the constant  */
  int32_t m;              /* samples, 0 <= m <= KLR_MAX_SAMPLES                                */
  int32_t v;              /* variables, 1..KLR_MAX_VARS                                        */
  int32_t num0, n_num;    /* numerator exponent rows [num0, num0+n_num) of exps                */
  int32_t den0, n_den;    /* denominator rows; row den0 must be all-zero (its coefficient = 1) */
  int8_t scale_exp[KLR_MAX_VARS]; /* s_k; entries beyond v ignored                            */
} klr_fit_desc;           /* 56 bytes */

/* status bits of klr_fit_info.status */
#define KLR_FIT_RANK_DEFICIENT 1u   /* numerical rank < n (min-norm-type solution returned)  */
#define KLR_FIT_UNDERDETERMINED 2u  /* m < n                                                   */
#define KLR_FIT_NOT_CONVERGED 4u    /* refinement stopped at max_iter above tol                */
#define KLR_FIT_FELL_BACK_FP64 8u   /* reduced-precision Gram replaced by the FP64 path        */
#define KLR_FIT_BAD_INPUT 16u       /* bad descriptor, m == 0, or a NaN/Inf sample             */
#define KLR_FIT_Q_NONPOS 32u        /* fitted q(x~_i) <= 0 at some sample (possible pole)      */
#define KLR_FIT_UNSUPPORTED 128u    /* KLR_FP64_SVD: n > 48, m > 1024, or m > 512 with n > 16 */
#define KLR_FIT_NO_SCRATCH 64u      /* the workspace holds fewer scratch rows than the batch's  */
                                    /*   workgroup-class fits need (size it by sum of m); no    */
                                    /*   coefficients computed (zeros written)                   */

typedef struct {
  uint32_t status;
  int32_t rank;           /* numerical rank of the equilibrated Gram factor at the Gram's own  */
                          /*   precision (pivots above 4 mu): for FP32/BF16 Grams it counts the */
                          /*   directions the preconditioner resolves, not the FP64 rank        */
  int32_t iters;          /* refinement iterations used                                        */
  int32_t q_nonpos;       /* samples with fitted q(x~_i) <= 0                                  */
  double resid_norm;      /* || A y - f ||_2 in FP64                                            */
  double err_est;         /* estimated ||A (y - y*)|| / ||f||: error of the fitted linearised   */
                          /*   values vs the exact least-squares solution y*                  */
} klr_fit_info;           /* 32 bytes */

typedef enum { KLR_FP64 = 0, KLR_FP32_REFINED = 1, KLR_BF16_REFINED = 2, KLR_FP64_SVD = 3 } klr_precision;

/* Workspace bytes klr_fit_batched needs for n_fits fits with total_rows = sum of their sample
 * counts m (an upper bound is enough): the schedule (a small plan record, two int32 per fit for
 * the longest-first order and the fits' buckets, one int64 per fit for its scratch offset), then
 * two FP64 values per sample row of private refinement scratch (residual and A t).  Each fit
 * that takes the workgroup kernel owns its own scratch rows (an exclusive prefix of m formed on
 * the device), so fits may share or overlap target ranges in f.  The call needs at least
 * klr_fit_workspace(n_fits, 0, precision) bytes (else KLR_E_WORKSPACE); a fit whose scratch rows
 * do not fit in the rest gets status KLR_FIT_NO_SCRATCH. */
size_t klr_fit_workspace(int32_t n_fits, int64_t total_rows, int32_t precision);

/* Fit n_fits independent rational functions (uneven m and monomial sets in one launch).
 *   desc[n_fits], exps[n_exp_rows][8] (uint8 exponent tuples), X[x_len] int32,
 *   f[f_len] float64, coef[coef_len] float64 (out), info[n_fits] (out).
 * Method (one wavefront per fit when n <= 48, v <= 4, m <= 1024 and every exponent <= 3, else
 * one workgroup per fit): the design matrix is built from X and f (in registers or LDS-staged
 * row chunks, never stored in device memory); the Gram matrix A^T A is formed on the matrix
 * cores and A^T f in FP64; columns are equilibrated by powers of two;
 * the equilibrated Gram matrix, shifted by mu = 8 u tr/n (u = unit roundoff of the Gram
 * precision), is factored by diagonally pivoted Cholesky in FP64 (the numerical rank is the
 * count of pivots above 4 mu); the normal-equations solution is then refined by conjugate
 * gradients on the least-squares problem, right-preconditioned by that factor, with residuals
 * f - A y recomputed from the samples in FP64, until the estimated error of the fitted values,
 * ||A (y - y*)|| / ||f|| (sum of the last three conjugate-gradient step energies), is <= tol or
 * max_iter iterations have run.
 *   precision: KLR_FP64 forms the Gram matrix in FP64; KLR_FP32_REFINED / KLR_BF16_REFINED
 *   round the design matrix to FP32 / BF16 for the Gram product and accumulate in FP32; a fit
 *   that does not converge is redone with the FP64 Gram (status KLR_FIT_FELL_BACK_FP64).
 *   The factorisation and the residuals are FP64 on every path.
 *   KLR_FP64_SVD solves each fit by the singular value decomposition the paper uses (section
 *   "Building a Driver Program: Rational function estimation"): one-sided Jacobi rotations of
 *   the column-equilibrated design matrix in FP64, one workgroup per fit with the rows in
 *   registers; numerical rank = singular values above 10 max(m, n) 2^-52 sigma_max; the
 *   minimum-norm least-squares solution of the equilibrated problem; iters = Jacobi sweeps;
 *   err_est = 2^-53 times the condition number of the kept part.  Limits: n <= 48 and m <= 1024
 *   (m <= 512 when n > 16); other fits get KLR_FIT_UNSUPPORTED and zero coefficients; max_iter
 *   and tol are not used (at most 30 sweeps).
 * Coefficients are in the scaled-variable basis x~ (x~_k = x_k 2^-scale_exp[k]; the raw-basis
 * coefficient of a monomial with exponents e is this one times 2^-(sum_k scale_exp[k] e_k), an
 * exact scaling the caller can apply, but one whose range overflows FP32 consumers at degree 3,
 * so the library keeps the scaled basis throughout).  On the Cholesky + CGLS paths a
 * rank-deficient fit gets a least-squares solution that is not necessarily the minimum-norm
 * one: its values on the samples are the unique least-squares values; KLR_FP64_SVD returns the
 * minimum-norm solution. */
klr_status klr_fit_batched(klr_handle h, const klr_fit_desc* desc, int32_t n_fits,
                           const uint8_t* exps, int32_t n_exp_rows,
                           const int32_t* X, int64_t x_len, const double* f, int64_t f_len,
                           int32_t precision, int32_t max_iter, double tol,
                           double* coef, int64_t coef_len, klr_fit_info* info,
                           void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------
 * Evaluation and argmin (steps 4 and 5).  A rational program is one kernel: 8 fits in the
 * metric order I_comp (compute instructions per thread), I_mc (coalesced memory instructions
 * per thread), I_mu (uncoalesced memory instructions per thread), U (transactions per
 * uncoalesced wave access), I_sync (synchronisations per thread), R (registers per thread),
 * Z (LDS bytes per block), B_w (bytes per wave memory transaction).  Each fit has v = 1 +
 * v_launch variables: the data size N, then the launch parameters.  The cost of configuration
 * L at data size N is the MWP-CWP-style cycle estimate whose FP32 operation sequence is
 * fixed by this library's documentation; occupancy follows the paper's flowchart (Example
 * "Hardware occupancy", eq. occupancy) with the wavefront for the warp.
 */
typedef struct {          /* hardware parameters H, fixed per call [host]                     */
  int32_t n_cu;           /* compute units                                                      */
  int32_t wave;           /* wavefront width (the paper's warp)                                 */
  int32_t w_max;          /* resident waves per CU                                              */
  int32_t b_max;          /* resident workgroups per CU                                         */
  int32_t r_max;          /* register-lanes per CU                                              */
  int32_t z_max;          /* LDS bytes per CU                                                   */
  int32_t t_max;          /* threads per workgroup                                              */
  int32_t reserved;       /* must be 0                                                          */
  float mem_lat;          /* memory latency, cycles (> 0)                                       */
  float dep_delay;        /* departure delay, cycles (> 0)                                      */
  float issue_cycles;     /* cycles per issued instruction (> 0)                                */
  float bw;               /* bytes per cycle per CU (> 0)                                       */
} klr_hw;                 /* 48 bytes */

#define KLR_GRID_1D 0     /* blocks = ceil(N / prod L)                                          */
#define KLR_GRID_2D 1     /* blocks = ceil(N / L0) * ceil(N / L1) (needs v_launch >= 2)         */

/* What a program's cost is. */
#define KLR_COST_CYCLES 0 /* the MWP-CWP-style cycle estimate from KLR_N_METRICS fitted metrics */
#define KLR_COST_METRIC 1 /* the program's one fitted function itself (fit0 only): the target   */
                          /*   metric was the quantity to minimise (e.g. the measured time), so  */
                          /*   the fitted rational function is the rational program; cost =     */
                          /*   p/q, inadmissible where q <= 0 or not finite, and the launch     */
                          /*   constraints (every L >= 1 and <= N, T <= t_max, T % wave == 0)   */
                          /*   apply; occupancy terms and the grid do not enter                 */
#define KLR_COST_PIECEWISE 2 /* a piecewise rational program with a fitted decision node (fits    */
                          /*   fit0, fit0 + 1, fit0 + 2 = d, g_a, g_b): cost = g_a where d >= 0,  */
                          /*   else g_b; inadmissible where d or the branch taken has q <= 0 or  */
                          /*   is not finite, and under the launch constraints of KLR_COST_METRIC */

typedef struct {
  int64_t cfg0;           /* element offset of its n_cfg configurations in cfgs (rows of       */
                          /*   v_launch int32)                                                  */
  int64_t q0;             /* offset of its n_q queries in queries, argmin and best_cost        */
  int64_t cost0;          /* offset of its n_cfg x n_q cost matrix (config-major) in all_costs */
  int32_t fit0;           /* first of its KLR_N_METRICS consecutive fit descriptors             */
  int32_t v_launch;       /* launch parameters per configuration, 1..KLR_MAX_LAUNCH             */
  int32_t n_cfg;          /* configurations, 0..max_cfg                                         */
  int32_t n_q;            /* queries, 0..max_q                                                  */
  int32_t grid_kind;      /* KLR_GRID_1D or KLR_GRID_2D                                         */
  int32_t cost_kind;      /* KLR_COST_CYCLES (fits fit0 .. fit0 + 7), KLR_COST_METRIC (fit0),   */
                          /*   KLR_COST_PIECEWISE (fit0 .. fit0 + 2)                            */
} klr_program;            /* 48 bytes */

/* program status bits (prog_status) */
#define KLR_PROG_BAD_DESC 1      /* program descriptor out of range: no output written          */
#define KLR_PROG_BAD_FIT 2       /* a metric's fit descriptor or exponents invalid: every query */
                                 /*   of the program reports -1 / +inf                          */

/* Workspace bytes klr_eval_argmin needs. */
size_t klr_eval_workspace(int32_t n_progs, int32_t max_cfg);

/* Evaluate every program at each of its queries over each of its configurations and take the
 * argmin: strict "<" in configuration order, so ties keep the lowest index; inadmissible or
 * non-finite costs never win; a query with no admissible configuration gets -1 and +inf.
 *   progs[n_progs]; desc[n_fits], exps[n_exp_rows][8], coef[coef_len] (the fitted
 *   coefficients); cfgs[cfgs_len] int32; queries[q_len] int32 data sizes;
 *   argmin[q_len] int32 and best_cost[q_len] float (out, at each program's q0 .. q0+n_q);
 *   all_costs[costs_len] float (optional, may be NULL): the full cost matrix, +inf where
 *   inadmissible; prog_status[n_progs] int32 (optional, may be NULL).
 *   max_cfg / max_q bound every program's n_cfg / n_q (launch sizing). */
klr_status klr_eval_argmin(klr_handle h, const klr_program* progs, int32_t n_progs,
                           int32_t max_cfg, int32_t max_q, const klr_hw* hw,
                           const klr_fit_desc* desc, int32_t n_fits,
                           const uint8_t* exps, int32_t n_exp_rows,
                           const double* coef, int64_t coef_len,
                           const int32_t* cfgs, int64_t cfgs_len,
                           const int32_t* queries, int64_t q_len,
                           int32_t* argmin, float* best_cost,
                           float* all_costs, int64_t costs_len, int32_t* prog_status,
                           void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): klr_eval_argmin with the same arguments and results,
 * minus the workspace.  The workspace is a fixed array of KLR_NOALLOC_SCRATCH_BYTES in device
 * memory, one per GPU, held from the library's load until the process ends; its address on a
 * device is looked up by klr_create, so the handle's device must be current.  A batch whose
 * klr_eval_workspace(n_progs, max_cfg) exceeds the array returns KLR_E_WORKSPACE and launches
 * nothing.  The call allocates nothing, creates no events, does not autotune (it uses the
 * launch shape already tuned for this batch shape on the handle, else the default) and records
 * no kernel timing.  Every call on one GPU shares that GPU's array (it keeps the last call's
 * contents; nothing in it needs clearing, since the collapse rewrites every slot the sweep
 * reads): calls that overlap in time on one GPU - other streams, other handles or threads -
 * race and must be serialised by the caller. */
#define KLR_NOALLOC_SCRATCH_BYTES (64u << 20)
klr_status klr_eval_argmin_noalloc(klr_handle h, const klr_program* progs, int32_t n_progs,
                                   int32_t max_cfg, int32_t max_q, const klr_hw* hw,
                                   const klr_fit_desc* desc, int32_t n_fits,
                                   const uint8_t* exps, int32_t n_exp_rows,
                                   const double* coef, int64_t coef_len,
                                   const int32_t* cfgs, int64_t cfgs_len,
                                   const int32_t* queries, int64_t q_len,
                                   int32_t* argmin, float* best_cost,
                                   float* all_costs, int64_t costs_len, int32_t* prog_status,
                                   void* stream);

/* ------------------------------------------------------------------------------------------
 * Learned surrogate (not in the paper): one network shared by all kernels (programs),
 * conditioned on a learned scalar embedding e_k per kernel, predicting standardised log-cycles:
 *   x = (log2 N / 26, log2 bx / 10, log2 by / 10, e_k); h1 = relu(W1 x + b1) [256];
 *   h2 = relu(W2 h1 + b2) [256]; y = w3 . h2 + b3;  ln C ~ mu + sigma y.
 * The 256 x 256 layer runs on BF16 MFMA (BF16 weights and activations, FP32 accumulation);
 * layers 1 and 3 run in FP32.  FP32 master weights, Adam moments in FP32.
 *
 * Parameter blob (caller-owned device memory of klr_surrogate_param_bytes(n_kernels) bytes):
 *   float hdr[16]      : hdr[0] = mu, hdr[1] = sigma (set by klr_surrogate_train)
 *   float P[NP], M[NP], V[NP]: parameters, Adam first and second moments, each laid out as
 *                        W2[256][256] | W1[256][4] | b1[256] | b2[256] | w3[256] | b3 | pad(15)
 *                        | emb[n_kernels] | pad to a multiple of 64 floats (NP)
 *   bf16 W2b[256][256], W2Tb[256][256]: working copies of W2 and its transpose
 * klr_surrogate_layout returns these offsets for bindings. */
#define KLR_MLP_HIDDEN 256
#define KLR_MLP_IN 4

typedef struct {
  float lr;               /* peak learning rate (cosine decay to 0 over all steps)             */
  float beta1, beta2, eps;
  int32_t batch;          /* samples per step, multiple of 128, 128..65536                      */
  int32_t epochs;         /* full passes; each pass visits floor(n / batch) batches             */
  uint64_t seed;          /* seeds the per-epoch sample permutation                             */
} klr_train_cfg;

size_t klr_surrogate_param_bytes(int32_t n_kernels);
/* Write the BF16 working copies (W2b, W2Tb) from P; call after filling P from the host. */
klr_status klr_surrogate_init(klr_handle h, void* params, int32_t n_kernels, void* stream);
/* [host] writes up to n of {NP, P offset, M offset, V offset (floats), W2b offset, W2Tb offset,
 * total (bytes), offsets of W2, W1, b1, b2, w3, b3, emb inside P (floats)}; returns the count. */
int32_t klr_surrogate_layout(int32_t n_kernels, int64_t* out, int32_t n);
/* Workspace bytes of klr_surrogate_train for this batch size and kernel count. */
size_t klr_surrogate_train_workspace(int32_t n_kernels, int32_t batch);
/* Train on n samples (sample i: kernel kernel_id[i] in [0, n_kernels), data size N[i] >= 1,
 * launch (launch[2i], launch[2i+1]) >= 1, exact cost cost[i] > 0; samples whose cost is not
 * finite and positive get zero weight).  mu, sigma of ln cost are computed first and stored in
 * the blob; params must hold initial P with zero M and V.  loss_per_epoch[epochs] (device, out):
 * mean training loss of each epoch on the standardised scale. */
klr_status klr_surrogate_train(klr_handle h, void* params, int32_t n_kernels,
                               const int32_t* kernel_id, const int32_t* N, const int32_t* launch,
                               const float* cost, int64_t n, const klr_train_cfg* cfg /*[host]*/,
                               float* loss_per_epoch, void* ws, size_t ws_bytes, void* stream);
/* Forward pass only: pred[i] = mu + sigma y(sample i) for n samples (ln C predictions). */
klr_status klr_surrogate_predict(klr_handle h, const void* params, int32_t n_kernels,
                                 const int32_t* kernel_id, const int32_t* N, const int32_t* launch,
                                 int64_t n, float* pred, void* stream);
/* One training step on one batch without the permutation (samples [0, batch) in order), for
 * gradient checks: writes the mean loss and, when grads != NULL, the gradient of every
 * parameter in the P layout (float[NP]) before applying Adam with (lr, step). */
klr_status klr_surrogate_step(klr_handle h, void* params, int32_t n_kernels,
                              const int32_t* kernel_id, const int32_t* N, const int32_t* launch,
                              const float* target_std, int32_t batch, float lr, int32_t step,
                              float beta1, float beta2, float eps, float* grads, float* loss,
                              void* ws, size_t ws_bytes, void* stream);
/* Surrogate selection over the same programs, configurations and queries as klr_eval_argmin:
 * program p uses embedding p (p < n_kernels).  For each query the network predicts ln C of
 * every configuration the exact program admits at that N (T <= t_max, T % wave == 0, every
 * L <= N, every fitted metric defined - q > 0 and a finite value - and at least one block
 * resident: the exact sweep's own FP32 steps, so a configuration left out has exact cost
 * +inf); the pick is the lowest prediction (lowest index on ties).  If the predicted margin to
 * the second best is below ln(1 + margin), or the exact cost of the pick is +inf (possible only
 * where the cycle estimate overflows FP32), the query falls back to the exact rational program
 * (klr_eval_argmin semantics) and fell_back[q] = 1.
 * Queries that do not fall back take a shortlist (KLR_OPT_SURR_SHORTLIST, K = 4 by default): the
 * network's K best-predicted admissible configurations are evaluated exactly (the FP32 cost of
 * klr_eval_argmin) and the pick is the lowest exact cost among them, lowest index on ties; a
 * shortlist whose exact costs are all +inf falls back.  With K = 1 the pick is the network's.
 * pred_cost[q] = exp(predicted ln C) of the pick, or the exact cost on fallback.
 * pred_margin[q] (optional, may be NULL): second-best minus best prediction in ln units (+inf
 * with a single candidate; NaN when the network makes no pick: no admissible configuration, or
 * a program it cannot represent - v_launch != 2 or more than 1024 configurations - which the
 * exact path answers).  prog_status[n_progs] (optional): as in
 * klr_eval_argmin; a program with KLR_PROG_BAD_DESC gets no output, one with KLR_PROG_BAD_FIT
 * falls back to the exact path and reports -1 / +inf.  Queries are counted per program over its
 * own range, so programs may share query ranges (their outputs then overwrite each other, as in
 * klr_eval_argmin) without overflowing the workspace.  Needs klr_surrogate_eval_workspace bytes
 * (linear in n_progs * max_q, which must stay below 2^31). */
size_t klr_surrogate_eval_workspace(int32_t n_progs, int32_t max_cfg, int32_t max_q);
klr_status klr_surrogate_eval(klr_handle h, const void* params, int32_t n_kernels,
                              const klr_program* progs, int32_t n_progs, int32_t max_cfg,
                              int32_t max_q, const klr_hw* hw, const klr_fit_desc* desc,
                              int32_t n_fits, const uint8_t* exps, int32_t n_exp_rows,
                              const double* coef, int64_t coef_len, const int32_t* cfgs,
                              int64_t cfgs_len, const int32_t* queries, int64_t q_len,
                              float margin, int32_t* argmin, float* pred_cost, uint8_t* fell_back,
                              float* pred_margin, int32_t* prog_status,
                              void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------
 * Launch-time decision service: the driver program's run-time role (paper: section "KLARAPTOR: A
 * Dynamic Optimization tool for CUDA" - at a kernel's launch its data parameters are known, the
 * rational program is evaluated for the admissible configurations and the best is used, and the
 * decision is kept in a history for later launches with the same data; section "Input/Output
 * Builder" - the result is the launch's grid and block dimensions; section "Annotating the source
 * code" - constraints on the launch parameters are Python-syntax expressions).
 *
 * A service holds host copies of the programs and configurations, per-program constraints and the
 * decision history (a hash map from (program, data size) to the decision; cleared when it would
 * exceed its limit, default 2^20 entries, and whenever a constraint is added).  A decision call
 * answers data sizes found in the history at once and evaluates the others with klr_eval_argmin
 * (one program, up to max_batch sizes per evaluation) in the caller's device workspace; with
 * constraints the cost rows come back to the host and the argmin is taken over the configurations
 * every constraint admits (strict "<" in configuration order).  Calls are synchronous on
 * `stream`; one thread at a time per service. */
typedef struct {
  int32_t gx, gy, gz;     /* grid: 1-D ceil(N / prod L), 1, 1; 2-D ceil(N / L0), ceil(N / L1), 1 */
  int32_t bx, by, bz;     /* block: the first three launch parameters (1 where absent)           */
  int32_t config;         /* configuration index in the program's list; -1: none admissible       */
  float cost;             /* the rational program's value there (+inf when none)                 */
} klr_launch;             /* 32 bytes */
typedef struct klr_service_s* klr_service;

/* Device workspace bytes of a service whose programs have at most max_cfg configurations and that
 * evaluates at most max_batch data sizes at once. */
size_t klr_service_workspace(int32_t max_cfg, int32_t max_batch);
/* progs [host] (n_progs; q0, n_q, cost0 ignored), hw [host], desc / exps / coef device arrays as
 * for klr_eval_argmin (they must stay valid while the service lives), configurations both as a
 * host copy (cfgs_host) and on the device (cfgs_dev), cfgs_len entries each; ws: device
 * workspace of klr_service_workspace(max over programs of n_cfg, max_batch) bytes, 256-byte
 * aligned, owned by the caller for the service's life. */
klr_status klr_service_create(klr_handle h, klr_service* out, const klr_program* progs, int32_t n_progs,
                              const klr_hw* hw, const klr_fit_desc* desc, int32_t n_fits, const uint8_t* exps,
                              int32_t n_exp_rows, const double* coef, int64_t coef_len, const int32_t* cfgs_host,
                              const int32_t* cfgs_dev, int64_t cfgs_len, int32_t max_batch, void* ws,
                              size_t ws_bytes);
void klr_service_destroy(klr_service s);
/* Add a constraint (a Python boolean expression over N, bx, by, bz (also L0..L3) and T = their
 * product, with or / and / not, chained comparisons, + - * / // % **, min / max / abs) to program
 * `prog`, or to every program when prog = -1.  KLR_E_INVALID with the parse error in
 * klr_last_error. */
klr_status klr_service_add_constraint(klr_service s, int32_t prog, const char* expr);
/* Decisions for program `prog` at n data sizes N [host]; out [host] receives n records. */
klr_status klr_service_decide(klr_service s, int32_t prog, const int32_t* N, int32_t n, klr_launch* out,
                              void* stream);
/* [host] counters: answers from the history, sizes evaluated, klr_eval_argmin calls, history size. */
klr_status klr_service_stats(klr_service s, int64_t* hits, int64_t* misses, int64_t* evaluations,
                             int64_t* entries);
klr_status klr_service_set_history_limit(klr_service s, int64_t max_entries);
/* [host] Compile `expr` and evaluate it at (N, L[0 .. v_launch)): 1 true, 0 false (a division by
 * zero is false), -1 on a parse error (message in err[err_len]). */
int32_t klr_constraint_check(const char* expr, int32_t N, const int32_t* L, int32_t v_launch, char* err,
                             int32_t err_len);

/* ------------------------------------------------------------------------------------------
 * Data collection (paper: step 1 of the section "An Algorithm to Build and Deploy a
 * Performance-Predicting Rational Program" and section "Building a Driver Program: Data
 * collection": the program is run at sample points and a metric is measured at each).  The
 * library carries target kernels with a two-dimensional launch configuration (bx, by) over
 * N x N single-precision grids; klr_collect_times measures each sample's kernel time (HIP events
 * around `reps` launches after one warm-up launch, on `stream`), the metric that a
 * KLR_COST_METRIC program fits and minimises; klr_target_attributes reports the compiled
 * kernel's registers per thread and LDS bytes per block (the R and Z metrics). */
#define KLR_TARGET_TRANSPOSE 0  /* out[x][y] = in[y][x]                                          */
#define KLR_TARGET_STENCIL 1    /* five-point Jacobi step, fixed boundary                        */
#define KLR_COLLECT_MAX_N 16384
/* Device buffer bytes for samples up to data size max_n (two N x N float grids). */
size_t klr_collect_buffer(int32_t target, int32_t max_n);
klr_status klr_target_attributes(klr_handle h, int32_t target, int32_t* regs, int32_t* lds_bytes);
/* samples [host]: n_samples rows (N, bx, by), 1 <= N <= KLR_COLLECT_MAX_N, bx, by >= 1,
 * bx * by <= 1024 (checked before any launch); time_us [host, out]: mean microseconds per launch;
 * buf: device buffer of klr_collect_buffer(target, max N) bytes (its contents are overwritten). */
klr_status klr_collect_times(klr_handle h, int32_t target, const int32_t* samples, int32_t n_samples,
                             int32_t reps, double* time_us, void* buf, size_t buf_bytes, void* stream);

/* ------------------------------------------------------------------------------------------
 * Options of a handle. */
#define KLR_OPT_FIT_PERSISTENT 0  /* 1 (default): fits are ordered longest first (m n^2) on the */
                                  /*   device; small fits (one wavefront each) are started in   */
                                  /*   that order and larger ones run in persistent workgroups  */
                                  /*   popping a device queue; 0: fits in descriptor order, one */
                                  /*   wavefront or workgroup each.  Results are identical.     */
#define KLR_OPT_EVAL_VARIANT 1    /* -1 (default): launch shape of the evaluation sweep chosen by */
                                  /*   the autotuner; >= 0: a fixed variant index                 */
#define KLR_OPT_FIT_VARIANT 2     /* -1 (default): fits per workgroup of the one-wavefront fit  */
                                  /*   kernel (4, 2 or 1) chosen by the autotuner (HIP-event     */
                                  /*   timing of each on the first batch of a shape, cached in   */
                                  /*   the handle and KLR_TUNE_CACHE); >= 0: variant 0, 1, 2.    */
                                  /*   Every variant gives bit-identical results                 */
#define KLR_OPT_SURR_SHORTLIST 3  /* 4 (default): klr_surrogate_eval re-ranks the network's K   */
                                  /*   best-predicted configurations of a query that does not   */
                                  /*   fall back by their exact costs and picks the lowest      */
                                  /*   (lowest index on ties); 1: the network's pick as it is;  */
                                  /*   values are clamped to [1, 4]                             */
#define KLR_OPT_COUNT 8
klr_status klr_set_option(klr_handle h, int32_t option, int64_t value);

/* ------------------------------------------------------------------------------------------
 * Graph capture of a sequence of calls (e.g. klr_fit_batched then klr_eval_argmin) issued on a
 * non-null stream between klr_capture_begin and klr_capture_end; klr_graph_launch replays it
 * with the same arguments (the same device buffers; their contents may change between
 * replays).  None of the captured calls allocates, synchronises or records memset nodes; the
 * evaluation's launch shape inside a capture is the one tuned earlier (or the default), and
 * kernel timing is off while capturing.  klr_surrogate_train is not capturable. */
typedef struct klr_graph_s* klr_graph;
klr_status klr_capture_begin(klr_handle h, void* stream);
klr_status klr_capture_end(klr_handle h, void* stream, klr_graph* out);
klr_status klr_graph_launch(klr_handle h, klr_graph g, void* stream);
void klr_graph_destroy(klr_graph g);

/* ------------------------------------------------------------------------------------------
 * Kernel timing.  When enabled on a handle, every kernel the handle launches is bracketed by a
 * pair of HIP events recorded on the caller's stream (so the elapsed time is the kernel's own,
 * on the stream it runs on).  klr_profile_read synchronises the recorded events, returns the
 * summed milliseconds and launch count of one kernel kind since the last reset, and never
 * launches work.  Kinds: */
#define KLR_K_COLLAPSE 0       /* per-(program, configuration) coefficient collapse            */
#define KLR_K_EVAL 1           /* evaluation + argmin sweep                                    */
#define KLR_K_FIT_GRAM 2       /* fit: design matrix + Gram                                    */
#define KLR_K_FIT_SOLVE 3      /* fit: factorisation + refinement + epilogue                   */
#define KLR_K_MLP 4            /* surrogate network training kernels                           */
#define KLR_K_SURR 5           /* surrogate selection (forward over the query x config grid)   */
#define KLR_K_FALLBACK 6       /* pick check, compaction, exact re-evaluation of flagged queries */
#define KLR_K_COUNT 7
klr_status klr_profile_enable(klr_handle h, int32_t on);   /* on != 0: enable; 0: disable+reset */
klr_status klr_profile_read(klr_handle h, int32_t kind, double* total_ms, int64_t* launches);

/* [host] Self-test of the invariant-divisor multiplication the evaluation uses for the grid
 * (floor(n / d) = mulhi(n, m) >> s for 0 <= n < 2^31): checks every divisor 1..d_max on
 * dividends around its multiples and at the ends of the range; returns the mismatch count. */
int64_t klr_selftest_divisors(uint32_t d_max);

/* [host] The same check for n_ds listed divisors of up to 64 bits (the evaluation divides by
 * T * n_cu, up to 2^32; divisors >= 2^31 give the quotient 0); ds is a host array; a zero
 * divisor counts as one mismatch.  Returns the mismatch count. */
int64_t klr_selftest_divisor_list(const uint64_t* ds, int32_t n_ds);

/* [device, synchronous] Self-test of the short quotient the evaluation takes where the collapse
 * encloses a metric's (or the cycle estimate's) numerator and denominator in [2^-40, 2^40]
 * (paper: step 4, "Rational program evaluation"; the FP32 sequence is this library's): for each
 * b mantissa in [b_first, b_first + b_count) of the 2^23 in [1, 2) and every a mantissa, the short
 * quotient against the correctly rounded FP32 division, plus the reciprocal estimate's exact
 * scaling with b's exponent (2^-60 .. 2^60) and sign.  Runs on the current device in slices of
 * 2^16 b mantissas (the whole range, 2^46 pairs, takes about half a minute) and waits for them.
 * Returns the mismatch count (0: the short quotient is the IEEE quotient for those b), or -1 if
 * b_first < 0, b_count < 0, b_first + b_count > 2^23 or a HIP call failed. */
int64_t klr_selftest_short_division(int32_t b_first, int32_t b_count);

/* [host] ABI self-description for binding checks: writes up to n entries of
 * {sizeof(klr_fit_desc), sizeof(klr_fit_info), sizeof(klr_hw), sizeof(klr_program), ...}
 * and returns the number of entries available. */
int32_t klr_abi_layout(int64_t* out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* KLR_H */
