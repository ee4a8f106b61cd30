/*
 * tk.h -- C ABI of the packed tensor-kernel library for MI355X (gfx950).
 *
 * The library implements the hot path of tensor-kernel l_p-regularised
 * regression (p = m/(m-1), m even): the order-m symmetric tensor kernel stored
 * in the packed layout of Section 5 (one value per sorted index tuple
 * t_0 <= ... <= t_{m-1} < n, nested-loop order, C(n+m-1, m) values), its
 * contraction g = K . alpha^{m-1}, the dual solve of eq. dual_tensor_kernel,
 * primal recovery, prediction and model-selection derivatives.
 *
 * Conventions (all entry points):
 *  - Return value: TK_OK (0) or a negative tk_status.  On error a message is
 *    available from tk_last_error() (thread-local) and outputs are untouched
 *    unless stated.  No exceptions cross the ABI.
 *  - Pointers named d_* are DEVICE pointers owned by the caller; pointers named
 *    h_* are host pointers owned by the caller.  The library never frees caller
 *    memory and never keeps a pointer after the call returns.
 *  - Matrices are row-major and dense.  Batched vectors (B right-hand sides)
 *    are stored as B consecutive rows of length n: d_alpha[b*n + i].
 *  - `stream` is a hipStream_t (0 = the null stream).  Every entry point only
 *    enqueues work on `stream` and returns, except where "synchronises" is
 *    stated.
 *  - Regularisation: lambda = 1/gamma of the text (which weights the loss by
 *    gamma); the dual solved is
 *        D(alpha) = (1/m) <K, alpha^{(x)m}> + (lambda/2)||alpha||^2 - <y, alpha>.
 *  - Calls that share a workspace must not overlap in time; distinct
 *    workspaces may be used concurrently on different streams.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TK_OK = 0,
    TK_EINVAL = -1,      /* invalid argument (odd or unsupported m, n < 1, lambda <= 0, ...) */
    TK_EOVERFLOW = -2,   /* C(n+m-1, m) or a byte count does not fit int64 */
    TK_ENOMEM = -3,      /* workspace too small or device allocation failed */
    TK_EHIP = -4,        /* a HIP runtime call failed */
    TK_ENOCONV = -5,     /* iteration limit reached before the tolerance */
    TK_ENAN = -6,        /* NaN or Inf met in an input or an iterate */
    TK_EUNSUPPORTED = -7 /* combination not built (e.g. n above the compiled maximum) */
} tk_status;

typedef enum { TK_F64 = 0, TK_F32 = 1, TK_BF16 = 2 } tk_dtype;

typedef enum {
    TK_LINEAR = 0, /* k(x_1..x_m) = sum_j x_{1j} .. x_{mj}              (Section 4) */
    TK_POLY = 1,   /* (linear)^s, s = kparam, integer >= 1               (eq. poly_tensor) */
    TK_EXP = 2     /* exp(linear)                                        (Section 4) */
} tk_kernel;

/* Accumulation used by the contraction. */
typedef enum {
    TK_ACC_AUTO = 0,  /* COMPENSATED for TK_F64 storage, F32 otherwise */
    TK_ACC_COMPENSATED = 1, /* FP64 with error-free products and compensated sums (TK_F64 only) */
    TK_ACC_F64 = 2,   /* plain FP64 (TK_F64 only) */
    TK_ACC_F32 = 3    /* plain FP32 (TK_F32 / TK_BF16 storage) */
} tk_acc;

/* Message of the last failed call on this thread ("" if none). */
const char *tk_last_error(void);

/* Largest n accepted by the contraction kernels (compile-time tile limit). */
int64_t tk_max_points(void);

/*
 * Number of packed entries C(n+m-1, m) (Section 5, eq. b_tensor4 for m = 4)
 * and the size in bytes of a buffer holding them as `dtype` (BF16 buffers are
 * rounded up to a multiple of 4 bytes, since they are read a dword at a
 * time).  Pure host arithmetic, no device work.
 * Errors: TK_EINVAL (n < 1, m < 1), TK_EOVERFLOW.
 */
int tk_packed_count(int64_t n, int m, int64_t *h_count);
int tk_packed_bytes(int64_t n, int m, int dtype, int64_t *h_bytes);

/*
 * Build the packed tensor kernel of the n points d_X[n*d] (Section 4:
 * K_t = k(x_{t_0}, .., x_{t_{m-1}}) for every sorted tuple t, stored in the
 * nested-loop order of Section 5).  The kernel value is computed in FP64 and
 * rounded to `dtype` (round-to-nearest-even) when stored into d_K, which must
 * hold tk_packed_bytes(n, m, dtype) bytes.  BF16 with an odd number of
 * entries: the 2 bytes after the last entry are read together with it and
 * this call sets them to zero (a BF16 array filled by other means must hold a
 * finite value there).
 * Errors: TK_EINVAL (m < 2 or odd, n/d < 1, kernel/kparam invalid),
 * TK_EOVERFLOW, TK_EUNSUPPORTED (n > tk_max_points()), TK_EHIP.
 */
int tk_build_packed_tensor(const double *d_X, int64_t n, int64_t d, int m, int kernel,
                           double kparam, int dtype, void *d_K, void *stream);

/*
 * Workspace bytes needed by tk_contract / tk_hvp for these sizes.
 */
int tk_contract_workspace(int64_t n, int m, int64_t B, int dtype, size_t *h_bytes);

/*
 * g = K . alpha^{m-1} for B vectors:  g_b[a] = sum_{i_2..i_m} K[a,i_2..i_m] alpha_b[i_2]..alpha_b[i_m]
 * (the gradient of the first term of eq. dual_tensor_kernel).  The packed
 * array d_K (dtype) is streamed once per pass; alpha and g are FP64 [B*n].
 * `acc` selects the accumulation (tk_acc).  The reduction order is fixed, so
 * results are bitwise reproducible for a given (n, m, B, dtype, acc).
 * Errors: TK_EINVAL, TK_ENOMEM (work_bytes too small), TK_EUNSUPPORTED, TK_EHIP.
 */
int tk_contract(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha,
                int64_t B, double *d_g, int acc, void *d_work, size_t work_bytes, void *stream);

/*
 * Directional derivative of the contraction (the adjoint of Section 4's
 * gradient map; its Jacobian is symmetric so the VJP equals the JVP):
 *   h_b = (m-1) K x_2 v_b x_3 alpha_b .. x_m alpha_b.
 * If d_g is not NULL it also receives g_b = K . alpha_b^{m-1} from the same
 * pass.  `acc`: TK_ACC_AUTO and TK_ACC_F64 = plain FP64 for TK_F64 storage
 * (FP32 for FP32/BF16 storage); TK_ACC_COMPENSATED = compensated FP64
 * (TK_F64 storage only).
 * Errors: as tk_contract.
 */
int tk_hvp(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha,
           const double *d_v, int64_t B, double *d_h, double *d_g, int acc, void *d_work,
           size_t work_bytes, void *stream);

/*
 * Workspace bytes needed by tk_hessian for (n, m).
 */
int tk_hessian_workspace(int64_t n, int m, size_t *h_bytes);

/*
 * Hessian of the first dual term, i.e. the Jacobian of the contraction
 * (Section 4): J = (m-1) K . alpha^{m-2}, the n x n matrix with
 *   J[i][j] = (m-1) sum_{i_3..i_m} K[i,j,i_3..i_m] alpha[i_3]..alpha[i_m],
 * so that J v equals tk_hvp's h for every direction v.  One alpha vector
 * (device, FP64 [n]); d_J receives FP64 [n*n], row-major and symmetric.  The
 * packed array (any dtype) is read twice (once for m = 2) and the arithmetic
 * is plain FP64 with a fixed reduction order (bitwise reproducible).  The
 * dual solve uses it for its preconditioner.  d_work sized by
 * tk_hessian_workspace.
 * Errors: TK_EINVAL, TK_ENOMEM (work_bytes too small), TK_EUNSUPPORTED, TK_EHIP.
 */
int tk_hessian(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha, double *d_J,
               void *d_work, size_t work_bytes, void *stream);

/*
 * Autotuner of the vector tile: the number of alpha vectors (and directions)
 * that share one read of the packed tensor inside a workgroup, for
 * tk_contract (d_v == NULL) or tk_hvp with B vectors and accumulation `acc`.
 * Times tiles 1, 2 and 4 (those the accumulation mode has: FP32 1/2/4, plain
 * FP64 1/2/4 for contractions and 1/2 for directional derivatives,
 * compensated 1) on this tensor and these inputs, keeps the fastest for the
 * current device and shape (later tk_contract / tk_hvp / tk_solve_dual calls
 * of that shape use it) and returns it in *h_tile.  h_ms (optional, host, 3
 * entries) receives milliseconds per call for tiles 1, 2, 4 (-1 where not
 * timed).  d_alpha, d_v: [B*n] device inputs; d_out [B*n] device scratch for
 * the results; d_work sized by tk_contract_workspace.  Synchronises.
 * Errors: as tk_contract.
 */
int tk_autotune(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha,
                const double *d_v, int64_t B, int acc, double *d_out, void *d_work,
                size_t work_bytes, void *stream, int *h_tile, double *h_ms);

/* Options of the dual solve (host struct). */
typedef struct {
    int max_newton;      /* Newton iterations per lambda (default 100) */
    int max_cg;          /* CG iterations per Newton step (default 2000) */
    double tol;          /* stop when ||grad D||_2 <= tol * lambda * ||alpha||_2 (default 1e-11):
                            by lambda-strong convexity the relative error of alpha is then <= tol */
    int fixed_iters;     /* > 0: run exactly this many Newton iterations, ignore tol */
    int warm_start;      /* nonzero: d_alpha holds the starting point on entry */
    const void *polish_K;/* optional FP64 packed tensor of the same points: after
                            the reduced-precision solve, Newton steps on it with
                            compensated gradients until tol is met (may be NULL) */
    int polish_dtype;    /* dtype of polish_K (must be TK_F64 when set) */
    int verbose;         /* print one line per Newton iteration to stderr */
    int precond;         /* 1 (default): at every Newton step J, the Hessian of the
                            contraction, is assembled by tk_hessian (FP64, on the FP64
                            tensor or the polish tensor) and CG runs on the dense system
                            (J + lambda I) p = -grad, preconditioned with an inverse
                            (J' + lambda' I)^{-1} factored on the host from an earlier
                            Hessian; 0: unpreconditioned CG whose products are tk_hvp
                            passes over the tensor */
    int precond_refresh; /* refactor the inverse after a Newton step that needed more than
                            this many CG steps (default 25) */
    int continuation;    /* B > 1: 1 (default) solves the lambdas one after another from the
                            largest down, each started from the previous solution and keeping
                            its preconditioner; 0: all lambdas in lock step, sharing every
                            pass */
} tk_solve_opts;

typedef struct {
    int newton_iters;
    int cg_iters;
    int passes;          /* passes over the packed tensor outside Hessian assembly
                            (contractions, and HVPs when precond = 0) */
    double grad_norm;    /* final ||grad D||_2 (compensated FP64 when polished or FP64 storage) */
    double objective;    /* final D(alpha) */
    double alpha_norm;
    int status;          /* TK_OK or TK_ENOCONV / TK_ENAN for this lambda */
    int hess_passes;     /* passes over the packed tensor spent on Hessian assembly (two per
                            Hessian, one for m = 2) */
    int precond_updates; /* preconditioner factorisations for this lambda */
} tk_solve_info;

void tk_solve_opts_default(tk_solve_opts *h_opts);

int tk_solve_workspace(int64_t n, int m, int64_t B, int dtype, size_t *h_bytes);

/*
 * Minimise the dual D(alpha) of eq. dual_tensor_kernel for B regularisation
 * values (a lambda path), by truncated Newton: each Newton step solves
 * (J(alpha) + lambda I) p = -grad D with preconditioned conjugate gradients
 * on the assembled Hessian (tk_hessian; tk_hvp passes when opts->precond is
 * 0), followed by an Armijo backtracking line search on D.  With opts->continuation the lambdas are solved in decreasing
 * order from each other's solutions; otherwise all B share every pass.  d_y is the FP64 response [n]; h_lambdas
 * holds B values (host); d_alpha [B*n] receives the solutions (and holds the
 * warm start when opts->warm_start).  h_info receives B records.
 * Synchronises: returns when every lambda has converged or hit its limits.
 * Returns TK_OK when all converged, TK_ENOCONV if any did not (check h_info).
 */
int tk_solve_dual(const void *d_K, int dtype, int64_t n, int m, const double *d_y,
                  const double *h_lambdas, int64_t B, const tk_solve_opts *h_opts,
                  double *d_alpha, tk_solve_info *h_info, void *d_work, size_t work_bytes,
                  void *stream);

/*
 * Primal weights of the linear tensor kernel (eq. tensor_representer with q = m
 * even): W_b = (X^T alpha_b)^{m-1}, d_X [n*d], d_alpha [B*n] -> d_W [B*d].
 * The product X^T alpha runs on FP64 MFMA tiles.
 */
int tk_primal_weights(const double *d_X, int64_t n, int64_t d, int m, const double *d_alpha,
                      int64_t B, double *d_W, void *stream);

/*
 * Prediction <w_b, x> for N query points (eq. tensor_1): d_W [B*d] (from
 * tk_primal_weights), d_Xq [N*d] -> d_f [B*N].  FP64 MFMA.
 */
int tk_predict(const double *d_W, int64_t d, int64_t B, const double *d_Xq, int64_t N,
               double *d_f, void *stream);

/*
 * Dense shortcut of a finite feature map (linear kernel): g_b = X (X^T alpha_b)^{m-1},
 * equal to tk_contract in exact arithmetic (eq. tensor_1).  FP64 MFMA.
 * d_work must hold B*d doubles.
 */
int tk_contract_dense(const double *d_X, int64_t n, int64_t d, int m, const double *d_alpha,
                      int64_t B, double *d_g, double *d_work, void *stream);

/*
 * Adaptive threshold of Section 6.3: tau_b = 2 * std(W_b) (population standard
 * deviation over the d weights) and mask_b[j] = |W_b[j]| > tau_b.
 * d_W [B*d] -> d_mask [B*d] (uint8), d_tau [B].
 */
int tk_support(const double *d_W, int64_t d, int64_t B, uint8_t *d_mask, double *d_tau,
               void *stream);

/*
 * Nystrom-type subsampling (Section 6.1): gather the rows d_idx[0..l) of
 * d_X [N*d] into d_out [l*d].  Indices are drawn by the caller.
 * Errors: TK_EINVAL when an index is outside [0, N) (checked on the device;
 * synchronises to report it).
 */
int tk_gather_rows(const double *d_X, int64_t N, int64_t d, const int64_t *d_idx, int64_t l,
                   double *d_out, void *stream);

/*
 * Derivative of the validation error with respect to lambda at a dual optimum
 * alpha* (implicit differentiation of grad D(alpha*(lambda)) = 0):
 *   MSE_val = mean((X_val w - y_val)^2), w = (X^T alpha*)^{m-1},
 *   (J(alpha*) + lambda I) z = d MSE_val / d alpha,   dMSE/dlambda = -z^T alpha*.
 * CG on tk_hvp passes (rel. residual cg_tol).  Outputs on the host: h_mse,
 * h_dmse; d_z [n] (may be NULL) receives z.  Synchronises.
 */
int tk_dmse_dlambda(const void *d_K, int dtype, int64_t n, int m, const double *d_X, int64_t d,
                    const double *d_alpha, double lambda, const double *d_Xval,
                    const double *d_yval, int64_t nval, double cg_tol, int max_cg,
                    double *h_mse, double *h_dmse, double *d_z, void *d_work, size_t work_bytes,
                    void *stream);

int tk_dmse_workspace(int64_t n, int m, int64_t d, int64_t nval, int dtype, size_t *h_bytes);

/*
 * Instrumentation (not part of the method): while enabled, every kernel that
 * streams the packed tensor (the first pass of tk_contract / tk_hvp and the two
 * streaming kernels of tk_hessian, also inside tk_solve_dual or
 * tk_dmse_dlambda) is bracketed by HIP events on its own stream.
 * tk_timing_stop synchronises those events and returns, per kind (0 =
 * contraction with compensated accumulation, 1 = directional derivative, 2 =
 * contraction with plain accumulation, 3 = Hessian tile sums, 4 = Hessian unit
 * vectors), the number of launches, their summed duration in milliseconds and
 * the bytes of the packed tensor they read (entries x storage size per read).
 * Arrays are host arrays of length TK_TIMING_KINDS.
 */
#define TK_TIMING_KINDS 5
int tk_timing_start(void);
int tk_timing_stop(int64_t *h_launches, double *h_ms, double *h_bytes);

#ifdef __cplusplus
}
#endif

#endif /* TK_H */
