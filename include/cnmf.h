/*
 * cnmf.h -- C ABI of the MI355X (gfx950) compressed-NeNMF library.
 *
 * Method: F. Yahaya, M. Puigt, G. Delmaire, G. Roussel, "Faster-than-fast NMF
 * using random projections and Nesterov iterations" (arXiv 1812.04315).
 *
 *   NMF model X ~ G F with X (n x m) >= 0, G (n x p) >= 0, F (p x m) >= 0:
 *     Sec. 1, Eq. (1); alternating subproblems Eqs. (2) and (3).
 *   NeNMF inner loop (Nesterov optimal gradient): Sec. 2.
 *   Compressed NMF strategy: Sec. 3, Algorithm 1.
 *   Randomized subspace iteration: Sec. 3, Algorithm 2.
 *   Relative reconstruction error: Sec. 4, Eq. (4).
 *
 * Conventions for every entry point:
 *   - Matrices are row-major.  "ld" is the row pitch in elements (>= columns).
 *   - Every array pointer is a caller-owned DEVICE pointer on the context's
 *     device, unless the comment says "host".  The library never frees,
 *     retains or reallocates caller memory.  Scratch lives in the context.
 *   - Calls are asynchronous: they validate arguments on the host, enqueue
 *     kernels on the context's HIP stream and return.  Argument errors are
 *     returned synchronously; errors found by the kernels (non-finite or
 *     negative data, a basis that cannot be completed, a stalled grid
 *     barrier) are OR-ed into a device status word read by cnmf_status().
 *   - Return value: CNMF_OK (0) or a negative CNMF_E* code.
 *   - One context per stream; a context is not thread-safe.
 */
#ifndef CNMF_H
#define CNMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes --------------------------------------------------- */
#define CNMF_OK          0
#define CNMF_EINVAL     -1   /* bad argument: shape, limit, NULL, alignment   */
#define CNMF_ENOMEM     -2   /* workspace allocation failed                    */
#define CNMF_EHIP       -3   /* a HIP runtime call failed                      */
#define CNMF_EDEVICE    -4   /* cnmf_status(): the device status word is set   */
#define CNMF_ENODERIV   -5   /* cnmf_adj_backward(): the rank rule replaced a
                                basis column, where the bases of Algorithm 2
                                have no derivative                            */
#define CNMF_ETOOBIG    -6   /* cnmf_solve_noalloc(): the problem needs more
                                scratch than CNMF_NOALLOC_SCRATCH_BYTES       */

/* ---- device status word bits (cnmf_status) ----------------------------- */
#define CNMF_ST_NONFINITE   0x01  /* NaN/Inf met in data, a Gram or a norm     */
#define CNMF_ST_NEGATIVE    0x02  /* X has a negative entry (validation pass)  */
#define CNMF_ST_BREAKDOWN   0x04  /* replacement basis column also deficient   */
#define CNMF_ST_ZERO_LIPS   0x08  /* warning: W = 0, factor left unchanged     */
#define CNMF_ST_TIMEOUT     0x10  /* a grid barrier stalled; results invalid   */

/* ---- limits ---------------------------------------------------------- */
#define CNMF_MAX_RANK    32   /* p and l = p + nu are at most 32              */
#define CNMF_MAX_ROWS    65536 /* n and m of a solve (and of cnmf_nnls's rows):
                                  every subproblem runs in one launch whose
                                  workgroups (64 to 256 rows each, at most 256)
                                  must all be resident on the GPU at once;
                                  larger n or m is rejected with CNMF_EINVAL.
                                  The RSI and the sweeps have no such limit. */

/* ---- parameters ------------------------------------------------------ */
#define CNMF_STOP_GLOBAL      0  /* tol = ratio * ||(P grad_G, P grad_F)|| at (G0,F0); /10 rule */
#define CNMF_STOP_SUBPROBLEM  1  /* tol = ratio * ||P grad(Z_0)|| per inner loop              */

#define CNMF_PREC_FP32  0
#define CNMF_PREC_BF16  1

#define CNMF_FLAG_VALIDATE_INPUT  0x1  /* check X finite and >= 0 before the sketch */

#define CNMF_METHOD_PLAIN       0  /* NeNMF on X (Sec. 2)                   */
#define CNMF_METHOD_COMPRESSED  1  /* NeNMF on X_L, X_R (Algorithm 1)       */

#define CNMF_SOLVER_NESTEROV  0  /* NeNMF inner loop (Sec. 2)                             */
#define CNMF_SOLVER_HALS      1  /* HALS column sweeps (Sec. 1, Cichocki 2007), inner_max
                                    sweeps per subproblem                                */
#define CNMF_SOLVER_MU        2  /* multiplicative updates in the semi-NMF form of Ding
                                    et al. 2010 (Sec. 3), inner_max per subproblem       */

#define CNMF_RESTART_NONE      0
#define CNMF_RESTART_GRADIENT  1  /* O'Donoghue and Candes 2015 (Sec. 4 footnote): the
                                     momentum of a row restarts when its gradient at the
                                     extrapolated point opposes the last step            */

typedef struct cnmf_params {
    int32_t p;            /* factorisation rank, 1 <= p <= 32 (Eq. (1))                */
    int32_t nu;           /* oversampling: sketch width l = p + nu, l <= min(n,m), <= 32;
                             the paper's target rank (Sec. 3) is l                      */
    int32_t q;            /* power iterations of Algorithm 2, q >= 1                    */
    int32_t outer_iters;  /* outer (alternating) iterations T >= 0                      */
    int32_t inner_max;    /* Max_iter of the inner loop (Sec. 2), 1..100000             */
    int32_t inner_min;    /* earliest step at which the gradient bound is tested, >= 1  */
    double  inner_ratio;  /* gradient-bound ratio (e.g. 1e-3)                           */
    double  tau2;         /* numerical-rank threshold of the orthonormalisation (1e-9)  */
    int32_t stop_rule;    /* CNMF_STOP_*                                                */
    int32_t sweep_prec;   /* CNMF_PREC_*: arithmetic of the X-sized sweeps              */
    int32_t flags;        /* CNMF_FLAG_*                                                */
    int32_t solver;       /* CNMF_SOLVER_*: update rule of every subproblem             */
    int32_t restart;      /* CNMF_RESTART_*: adaptive restart of the Nesterov momentum  */
    int32_t reserved;     /* must be 0                                                  */
    double  time_budget;  /* > 0: device seconds after which the outer loop stops
                             (Sec. 3 admits a time limit as the outer stopping
                             criterion); 0: run all outer_iters                        */
} cnmf_params;

/* Fills p = 0 ... with the library defaults (q = 4, inner_max = 500,
 * inner_min = 1, inner_ratio = 1e-3, tau2 = 1e-9, global stop, FP32,
 * Nesterov inner loop without restart, no time budget). */
void cnmf_params_default(cnmf_params* out);

/* Optional per-outer-iteration trace of cnmf_solve.  Every pointer is a
 * device pointer or NULL.  T = outer_iters. */
typedef struct cnmf_trace {
    int32_t*  steps;   /* T x 2: inner steps taken (G update, F update)            */
    double*   lips;    /* T x 2: Lipschitz constants used                           */
    double*   tols;    /* T x 2: gradient bound in force                            */
    uint64_t* ticks;   /* T + 1: device wall clock (cnmf_clock_hz) at the start and
                          at the end of every outer iteration                        */
    float*    G_hist;  /* T x n x p: G after every outer iteration                  */
    float*    F_hist;  /* T x p x m: F after every outer iteration                  */
    float*    W_hist;  /* T x 2 x p x p: the Gram W each subproblem used (FP32, as
                          in its gradient; L is computed from (W + W^T) / 2)        */
    int32_t*  outer_done; /* 1: outer iterations completed (< T when the time
                          budget ran out; later entries of the trace unset)        */
} cnmf_trace;

typedef struct cnmf_ctx cnmf_ctx;

/* ---- context --------------------------------------------------------- */

/* Creates a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the null stream).  *out receives the handle. */
int cnmf_create(cnmf_ctx** out, int device, void* stream);
int cnmf_destroy(cnmf_ctx* ctx);
int cnmf_set_stream(cnmf_ctx* ctx, void* stream);
/* Frequency in Hz of the device clock written to cnmf_trace.ticks. */
int cnmf_clock_hz(cnmf_ctx* ctx, double* hz_out /* host */);
/* Waits for the stream, returns the status word in *status (host) and
 * clears it.  Returns CNMF_EDEVICE when any error bit (not the zero-
 * Lipschitz warning) was set. */
int cnmf_status(cnmf_ctx* ctx, int32_t* status /* host */);
const char* cnmf_strerror(int code);

/* ---- the hot path ---------------------------------------------------- */

/* Randomized subspace iteration, Sec. 3, Algorithm 2, l = p + nu.
 *   X        n x m (ldx), >= 0.
 *   omega_L  m x l Gaussian (Algorithm 2's Omega_L), row-major, ld = l.
 *   omega_R  l x n Gaussian (Algorithm 2's Omega_R), row-major, ld = n.
 *   Q_L      out, n x l, orthonormal columns, basis of (X X^T)^q Omega_R^T.
 *   Q_R      out, m x l, orthonormal columns, basis of (X^T X)^q Omega_L.
 *   X_L      out, l x m = Q_L^T X   (Algorithm 1's L X).
 *   X_R      out, n x l = X Q_R     (Algorithm 1's X R).
 * Two independent chains, re-orthonormalised at every half-step by
 * CholeskyQR with FP64 Gram and Cholesky (a second pass, CholeskyQR2, when
 * some pivot falls below 1e-7 of its diagonal entry, where one FP64 pass
 * could leave an orthogonality loss above FP32 rounding, and after column
 * replacements).  Both products of a half-step come from one read of X
 * (cnmf_sweep_dual).  A column whose Cholesky pivot
 * is <= tau2 * max_j ||y_j||^2 is replaced by the same column of the other
 * Gaussian draw (Omega_R^T for n-space panels, Omega_L for m-space panels).
 * Sweeps run in FP32 (sweep_prec must be CNMF_PREC_FP32 here). */
int cnmf_rsi(cnmf_ctx* ctx, int64_t n, int64_t m, const float* X, int64_t ldx,
             const cnmf_params* prm, const float* omega_L, const float* omega_R,
             float* Q_L, float* Q_R, float* X_L, float* X_R);

/* Same, with the X-sized sweeps in BF16 on MFMA (FP32 accumulation):
 *   Xb  n x m (ldxb >= m, any alignment) bfloat16 bit patterns of X (see
 *       cnmf_to_bf16).
 * Every X product takes its skinny operand (Omega, then the current basis)
 * rounded to bfloat16; the orthonormalisation (FP64 Gram and Cholesky, FP32
 * apply) and the outputs are as in cnmf_rsi; X_L, X_R are products with Xb.
 * sweep_prec is ignored. */
int cnmf_rsi_bf16(cnmf_ctx* ctx, int64_t n, int64_t m, const uint16_t* Xb,
                  int64_t ldxb, const cnmf_params* prm, const float* omega_L,
                  const float* omega_R, float* Q_L, float* Q_R, float* X_L,
                  float* X_R);

/* Compression matrices of Sec. 3 (Algorithm 1 takes L, R as inputs), in the
 * layout of cnmf_rsi's outputs (Q_L n x l with X_L = Q_L^T X, Q_R m x l with
 * X_R = X Q_R; l = p + nu), for the compressed solve:
 *   CNMF_COMPRESS_RSI       randomized subspace iteration, Algorithm 2
 *                           (identical to cnmf_rsi);
 *   CNMF_COMPRESS_GAUSSIAN  the plain random projection of Sec. 3: Gaussian
 *                           matrices scaled by 1/sqrt(l), Q_L = Omega_R^T /
 *                           sqrt(l), Q_R = Omega_L / sqrt(l) (not orthonormal;
 *                           q and tau2 unused); one pass over X;
 *   CNMF_COMPRESS_POWER     randomized power iteration without
 *                           re-orthonormalisation (the structured random
 *                           projection Sec. 3 cites): Q_R = orth((X^T X)^q
 *                           Omega_L), Q_L = orth((X X^T)^q Omega_R^T), each
 *                           intermediate product scaled to unit Frobenius norm
 *                           (ranges unchanged), one CholeskyQR(2) with the rank
 *                           rule of cnmf_rsi at the end; the same 2q + 1
 *                           passes over X per chain as Algorithm 2, in exact
 *                           arithmetic the same subspaces, but the weak
 *                           directions drown in FP32 rounding after the powers.
 * Arguments as cnmf_rsi (FP32 sweeps). */
#define CNMF_COMPRESS_RSI       0
#define CNMF_COMPRESS_GAUSSIAN  1
#define CNMF_COMPRESS_POWER     2
int cnmf_compress(cnmf_ctx* ctx, int32_t kind, int64_t n, int64_t m, const float* X,
                  int64_t ldx, const cnmf_params* prm, const float* omega_L,
                  const float* omega_R, float* Q_L, float* Q_R, float* X_L, float* X_R);

/* Round X (n x m, ldx) to bfloat16 (round to nearest even) into Xb (ldxb). */
int cnmf_to_bf16(cnmf_ctx* ctx, int64_t n, int64_t m, const float* X,
                 int64_t ldx, uint16_t* Xb, int64_t ldxb);

/* NeNMF outer loop: plain (Sec. 2, needs X) or compressed (Algorithm 1,
 * needs Q_L, Q_R, X_L, X_R from cnmf_rsi; X may then be NULL).
 *   n, m <= CNMF_MAX_ROWS.  Results are bitwise repeatable: every reduction
 *   (split sums, workgroup exchanges, norms) runs in a fixed order.
 *   G  in/out n x p (ld = p), F in/out p x m (ld = m); G0, F0 >= 0.
 *   trace  optional (host struct of device pointers), may be NULL.
 *   replay optional device int32 T x 2: run exactly these inner step counts
 *          instead of testing the gradient bound (parity runs).
 * Per outer iteration: G update on Eq. (2) (or its compressed form), then F
 * update on Eq. (3), each by one Nesterov inner loop with step 1/L, where L
 * is an upper bound of lambda_max(W) within 1e-12 relative (FP64), and the
 * projected gradient norms are summed in FP64. */
int cnmf_solve(cnmf_ctx* ctx, int method, int64_t n, int64_t m,
               const float* X, int64_t ldx,
               const float* Q_L, const float* Q_R, const float* X_L,
               const float* X_R, const cnmf_params* prm, float* G, float* F,
               const cnmf_trace* trace, const int32_t* replay);

/* cnmf_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results as cnmf_solve, but the call
 * allocates nothing.  Its scratch (partial products of the phases, the
 * warm-start vectors of lambda_max and, for the plain method, B = X F^T,
 * G^T X and their split partial sums) lives in a static device array of
 * CNMF_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs
 * on until the process ends; its device address is looked up once per
 * device by cnmf_create.  Limit: the compressed method always fits
 * (n, m <= 65536 need at most 2 MiB); the plain method needs about
 * 4 (n + m) p bytes plus the split sums of its two X sweeps (at most about
 * 16 MiB on 256 compute units; 10000 x 10000 at p = 15 needs 17 MiB in
 * all) and returns CNMF_ETOOBIG, enqueuing nothing, when that exceeds the
 * array.  Every call on one GPU
 * shares that GPU's array (whatever the context), and the array keeps the
 * last call's contents (nothing in it needs clearing: every word is
 * written before it is read within a call).  Calls that overlap on one GPU
 * -- on different streams or from different threads -- race on it and must
 * be serialised by the caller. */
#define CNMF_NOALLOC_SCRATCH_BYTES (32u << 20)
int cnmf_solve_noalloc(cnmf_ctx* ctx, int method, int64_t n, int64_t m,
                       const float* X, int64_t ldx,
                       const float* Q_L, const float* Q_R, const float* X_L,
                       const float* X_R, const cnmf_params* prm, float* G, float* F,
                       const cnmf_trace* trace, const int32_t* replay);

/* Relative reconstruction error, Sec. 4, Eq. (4), for `count` factor pairs
 * G_i = G + i*strideG, F_i = F + i*strideF (element strides):
 *   out[i] = ||X - G_i F_i||_F / ||X||_F   (device double[count]).
 * Direct residual with FP64 accumulation. */
int cnmf_rre(cnmf_ctx* ctx, int64_t n, int64_t m, const float* X, int64_t ldx,
             int32_t p, const float* G, int64_t strideG, const float* F,
             int64_t strideF, int32_t count, double* out);

/* ---- kernel-level entry points (the steps above, one at a time) ------ */

/* Y (R x k, ldy) = X (R x C, ldx) * A, where A is C x k (a_trans = 0,
 * row pitch lda) or is given as its transpose k x C (a_trans = 1).
 * FP32 MFMA, FP32 accumulation.  k <= 32. */
int cnmf_sweep_right(cnmf_ctx* ctx, int64_t R, int64_t C, const float* X,
                     int64_t ldx, int32_t k, const float* A, int64_t lda,
                     int32_t a_trans, float* Y, int64_t ldy);

/* Z = X^T (C x R) * B (R x k, ldb): written C x k (z_trans = 0) or as its
 * transpose k x C (z_trans = 1), row pitch ldz.  FP32 MFMA.  k <= 32. */
int cnmf_sweep_left(cnmf_ctx* ctx, int64_t R, int64_t C, const float* X,
                    int64_t ldx, int32_t k, const float* B, int64_t ldb,
                    float* Z, int64_t ldz, int32_t z_trans);

/* Both sweeps from one read of X, as every half-step of Algorithm 2 needs
 * them (one product per chain): Y (R x k, ldy) = X * A with A given as its
 * transpose AT (k x C, row pitch ldat), and Z = X^T * B (B R x k, ldb)
 * written C x k (z_trans = 0) or k x C (z_trans = 1), row pitch ldz.
 * FP32 accuracy on the BF16 matrix cores: X, A and B are each split
 * exactly into three BF16 parts (x = h + m + l) and the six largest cross
 * products are accumulated in FP32 (the terms left out are below 2^-23 of
 * |x a|).  Results bitwise reproducible.  R, C >= 1, 1 <= k <= 32; Y and Z
 * must not overlap the inputs. */
int cnmf_sweep_dual(cnmf_ctx* ctx, int64_t R, int64_t C, const float* X,
                    int64_t ldx, int32_t k, const float* AT, int64_t ldat,
                    const float* B, int64_t ldb, float* Y, int64_t ldy,
                    float* Z, int64_t ldz, int32_t z_trans);

/* BF16 form of the two sweeps (the precision form of the X-sized products
 * of Algorithm 2): Xb holds X as bfloat16 bit patterns (R x C, row pitch
 * ldxb >= C, any alignment); the skinny operand is rounded to bfloat16
 * (nearest even) inside the call; products on the matrix cores with FP32
 * accumulation.  Arguments and outputs otherwise as cnmf_sweep_right /
 * cnmf_sweep_left; R, C >= 1, 1 <= k <= 32. */
int cnmf_sweep_right_bf16(cnmf_ctx* ctx, int64_t R, int64_t C, const uint16_t* Xb,
                          int64_t ldxb, int32_t k, const float* A, int64_t lda,
                          int32_t a_trans, float* Y, int64_t ldy);
int cnmf_sweep_left_bf16(cnmf_ctx* ctx, int64_t R, int64_t C, const uint16_t* Xb,
                         int64_t ldxb, int32_t k, const float* B, int64_t ldb,
                         float* Z, int64_t ldz, int32_t z_trans);

/* Both BF16 sweeps from one read of Xb (bfloat16 bit patterns, R x C, row
 * pitch ldxb), as every half-step of Algorithm 2 in the precision form
 * needs them: Y (R x k, ldy) = Xb * bf16(A) with A given as its transpose
 * AT (k x C, ldat), and Z = Xb^T * bf16(B) (B R x k, ldb) written C x k
 * (z_trans = 0) or k x C (z_trans = 1), row pitch ldz.  The skinny operands
 * are rounded to bfloat16 (nearest even), products accumulate in FP32 on
 * the matrix cores: the values of cnmf_sweep_right_bf16 and
 * cnmf_sweep_left_bf16 up to FP32 summation order.  Results bitwise
 * reproducible.  R, C >= 1, 1 <= k <= 32; Y and Z must not overlap the
 * inputs. */
int cnmf_sweep_dual_bf16(cnmf_ctx* ctx, int64_t R, int64_t C, const uint16_t* Xb,
                         int64_t ldxb, int32_t k, const float* AT, int64_t ldat,
                         const float* B, int64_t ldb, float* Y, int64_t ldy,
                         float* Z, int64_t ldz, int32_t z_trans);

/* Orthonormal basis of Y (N x l, ld = l) by CholeskyQR(2) with the rank rule
 * of cnmf_rsi; pool is N x l (pool_trans = 0, ld = l) or l x N
 * (pool_trans = 1, ld = N).  Q out N x l.  replaced out: l int32 flags. */
int cnmf_orth(cnmf_ctx* ctx, int64_t N, int32_t l, const float* Y,
              const float* pool, int32_t pool_trans, double tau2, float* Q,
              int32_t* replaced);

/* L = lambda_max(W) of the symmetric p x p FP32 matrix W, FP64
 * Householder tridiagonalisation and bisection.  out: device double. */
int cnmf_lipschitz(cnmf_ctx* ctx, int32_t p, const float* W, double* out);

/* One Nesterov inner loop (Sec. 2) on min_{Z>=0} 0.5 tr(Z W Z^T) - tr(B^T Z)
 * over `rows` independent rows of p unknowns: gradient Z W - B.
 *   Z  in/out, element (r, c) at Z[r*z_rs + c*z_cs] (G: z_rs = p, z_cs = 1;
 *      F viewed by columns: z_rs = 1, z_cs = m).
 *   W  p x p FP32; B rows x p FP32 (ld = p).
 *   tol      gradient bound (used when forced < 0).
 *   forced   >= 0: run exactly this many steps.
 *   steps_out, L_out, pg2_out: device int32 / double / double (may be NULL);
 *   pg2_out receives ||P grad(Z_0)||^2. */
int cnmf_nnls(cnmf_ctx* ctx, int64_t rows, int32_t p, float* Z, int64_t z_rs,
              int64_t z_cs, const float* W, const float* B, double tol,
              int32_t inner_max, int32_t inner_min, int32_t forced,
              int32_t* steps_out, double* L_out, double* pg2_out);

/* ---- batched form: many independent instances ------------------------
 * Randomized subspace iteration (Algorithm 2) and compressed NeNMF
 * (Algorithm 1) for `count` independent instances of uneven n, m, p.  Each
 * subproblem phase of all instances runs in one persistent launch: a
 * schedule packs every instance's workgroups into rounds of resident
 * workgroups (row tiles of 64 x tiles rows, tiles in {1, 2, 4} per side,
 * chosen by cnmf_batch_tune), and the outer loop of cnmf_batch_solve is
 * captured once in a HIP graph and replayed.  Per-instance arguments as in
 * cnmf_rsi and cnmf_solve; all pointers are caller-owned device memory that
 * must stay valid for the life of the batch. */
typedef struct cnmf_instance {
    int64_t n, m;
    int32_t p, nu;            /* 1 <= p, p + nu <= min(n, m), p + nu <= 32     */
    const float* X;           /* n x m, row pitch ldx (multiple of 4, 16-byte  */
    int64_t ldx;              /* aligned rows)                                */
    const float* omega_L;     /* m x l                                        */
    const float* omega_R;     /* l x n                                        */
    float* Q_L;               /* n x l   (written by cnmf_batch_rsi)          */
    float* Q_R;               /* m x l                                        */
    float* X_L;               /* l x m                                        */
    float* X_R;               /* n x l                                        */
    float* G;                 /* n x p, in/out                                */
    float* F;                 /* p x m, in/out                                */
    int32_t* steps;           /* optional T x 2 inner step counts (out)       */
    const int32_t* replay;    /* optional T x 2 forced inner step counts      */
} cnmf_instance;

typedef struct cnmf_batch cnmf_batch;

/* Plan a batch: copies the descriptors (host array), allocates the batch's
 * device state, builds the schedules with tiles_g / tiles_f (1, 2 or 4; 0
 * picks the smallest that fits).  prm: q, outer_iters, inner_*, stop_rule,
 * tau2 apply to every instance (its p and nu come from the descriptor). */
int cnmf_batch_create(cnmf_ctx* ctx, const cnmf_instance* inst, int32_t count,
                      const cnmf_params* prm, int32_t tiles_g, int32_t tiles_f,
                      cnmf_batch** out);
int cnmf_batch_destroy(cnmf_batch* b);
/* Algorithm 2 for every instance (Q_L, Q_R, X_L, X_R). */
int cnmf_batch_rsi(cnmf_batch* b);
/* Autotune: times a few outer iterations of the batched solve for every
 * (tiles_g, tiles_f) that fits, on scratch copies of G and F, keeps the
 * fastest schedule and writes it to tiles_out[2] (host). */
int cnmf_batch_tune(cnmf_batch* b, int32_t tune_iters, int32_t* tiles_out);
/* Compressed NeNMF outer loop for every instance; use_graph != 0 captures
 * the whole loop in a HIP graph on first use and replays it afterwards. */
int cnmf_batch_solve(cnmf_batch* b, int32_t use_graph);

/* ---- differentiation form -------------------------------------------
 * Reverse mode of compressed NeNMF (Algorithms 1 and 2, Sec. 2 inner loop)
 * unrolled over T = prm->outer_iters outer iterations with exactly
 * K = prm->inner_max (1..8) inner steps per subproblem.
 * cnmf_adj_forward: randomized subspace iteration (prm->q, tau2) keeping
 *   every panel, then the outer loop from (G0, F0), keeping (G, F) every
 *   ckpt outer iterations; writes G_T, F_T and returns the tape.  X,
 *   omega_L and omega_R must stay valid until the tape is destroyed.
 * cnmf_adj_backward: given dL/dG_T (n x p) and dL/dF_T (p x m), writes
 *   dL/dX (n x m, row pitch lddx) and, if non-NULL, dL/dG0, dL/dF0.  Each
 *   checkpoint segment is recomputed; the subproblems are reversed through
 *   their projections and momentum, L = lambda_max(W) through its top
 *   eigenvector, the bases through the thin-QR adjoint.  Returns
 *   CNMF_ENODERIV, computing nothing, when the rank rule replaced a basis
 *   column during the forward pass (the bases have no derivative there).
 *   The tape can be reused. */
typedef struct cnmf_tape cnmf_tape;
int cnmf_adj_forward(cnmf_ctx* ctx, int64_t n, int64_t m, const float* X, int64_t ldx,
                     const cnmf_params* prm, int32_t ckpt, const float* omega_L,
                     const float* omega_R, const float* G0, const float* F0,
                     float* G_out, float* F_out, cnmf_tape** tape);
int cnmf_adj_backward(cnmf_tape* tape, const float* dG, const float* dF, float* dX,
                      int64_t lddx, float* dG0, float* dF0);
int cnmf_tape_bytes(const cnmf_tape* tape, uint64_t* bytes /* host */);
int cnmf_tape_destroy(cnmf_tape* tape);

#ifdef __cplusplus
}
#endif
#endif /* CNMF_H */
