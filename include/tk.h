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
 *  - Non-finite values: the asynchronous entry points do not inspect the
 *    values they are given (that would need a synchronisation); a NaN or Inf
 *    input propagates into the outputs by IEEE arithmetic.  The synchronous
 *    entry points (tk_solve_dual, tk_dmse_dlambda) check their vector and
 *    matrix inputs first and return TK_ENAN before any pass.
 *  - Reproducibility: reductions run in a fixed order for a given launch
 *    shape, and launch shapes follow the device's compute-unit count and the
 *    kernels' occupancy, so results are bitwise reproducible per (device
 *    model, n, m, B, dtype, acc, vector tile), not across device models.
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
 * array d_K (dtype) is streamed once per tile of vectors: a workgroup applies
 * each entry it loads to a tile of 1, 2 or 4 vectors (tk_autotune picks the
 * tile), so a batch of B vectors reads K ceil(B / tile) times.  Plain FP64
 * accumulation of an FP64 tensor with m >= 4 and n <= 256 runs the first
 * pass, from 16 vectors on (or where tk_autotune chose it), as dense products
 * on the FP64 matrix cores, 16 vectors per tile, two tiles per workgroup:
 * each entry is staged once for its row tile and once for its column tile
 * per workgroup, and the workgroups of one range of K share an XCD's L2, so
 * HBM traffic is about three reads of K per launch of 64 vectors (measured
 * at n = 256), growing with the number of workgroup tiles.  alpha and g
 * are FP64 [B*n].  `acc` selects the accumulation (tk_acc).  The reduction
 * order is fixed for a launch shape (see the reproducibility convention).
 * Errors: TK_EINVAL, TK_ENOMEM (work_bytes too small), TK_EUNSUPPORTED, TK_EHIP.
 */
int tk_contract(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha,
                int64_t B, double *d_g, int acc, void *d_work, size_t work_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * contraction as tk_contract, with the same kernels, launch shapes and results,
 * but no caller workspace.  Its workspace and the work plans of its passes live
 * in a fixed device array of the library (64 MiB per device, held from the
 * first call on that device until the process ends); the plans are copied
 * there from host memory on every call.  The call performs no device
 * allocation or free and records no timing events.  Calls whose workspace
 * exceeds tk_contract_noalloc_max_bytes() (compare tk_contract_workspace for
 * the shape) fail with TK_ENOMEM and a message, before any device work.  Every call on one device shares that device's array: calls that
 * overlap in time on one device (different streams, or host threads) race and
 * must be serialised by the caller; consecutive calls on one stream are safe.
 * The array keeps the last call's contents; no kernel of the contraction
 * reads workspace it has not written in the same call.
 * Errors: as tk_contract, TK_ENOMEM (above the maximum).
 */
int tk_contract_noalloc(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha,
                        int64_t B, double *d_g, int acc, void *stream);
size_t tk_contract_noalloc_max_bytes(void);

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
 * compensated 1) and, for plain FP64 contractions of an FP64 tensor with
 * m >= 4, the FP64-MFMA batch pass (tile 16, see tk_contract) on this tensor
 * and these inputs, keeps the fastest for the current device and shape
 * (later tk_contract / tk_hvp / tk_solve_dual calls of that shape use it) and
 * returns it in *h_tile.  h_ms (optional, host, 4 entries) receives
 * milliseconds per call for tiles 1, 2, 4, 16 (-1 where not timed).  d_alpha, d_v: [B*n] device inputs; d_out [B*n] device scratch for
 * the results; d_work sized by tk_contract_workspace.  Synchronises.
 * Errors: as tk_contract.
 */
int tk_autotune(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha,
                const double *d_v, int64_t B, int acc, double *d_out, void *d_work,
                size_t work_bytes, void *stream, int *h_tile, double *h_ms);

/* Loss of the primal problem (eq. tensor_infinite_2); the dual replaces it by
 * its Fenchel conjugate (Section 4). */
typedef enum {
    TK_LOSS_SQUARE = 0,   /* L(y, t) = (y - t)^2 / 2: the dual of eq. dual_tensor_kernel */
    TK_LOSS_LOGISTIC = 1  /* L(y, t) = log(1 + exp(-y t)), y in {-1, +1}: the dual term
                             (1/lambda) sum_i [p_i log p_i + (1 - p_i) log(1 - p_i)],
                             p_i = lambda y_i alpha_i in (0, 1) */
} tk_loss;

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
                            (J' + lambda' I)^{-1} of an earlier Hessian (Newton-Schulz on
                            the device, a host Cholesky when that does not settle); 0:
                            unpreconditioned CG whose products are tk_hvp passes over the
                            tensor */
    int precond_refresh; /* remake the inverse after a Newton step that needed more than
                            this many CG steps (default 25; more than one step while the
                            last remake was a warm Newton-Schulz update that held), and,
                            for a Hessian from an FP64 tensor inverted on the device,
                            whenever lambda has fallen below half the lambda' it was made
                            at */
    int continuation;    /* B > 1: 1 (default) solves the lambdas one after another from the
                            largest down, each started from the previous solution and keeping
                            its preconditioner; 0: all lambdas in lock step, sharing every
                            pass */
    int loss;            /* tk_loss (default TK_LOSS_SQUARE).  The logistic loss starts cold
                            solves at the centre of the dual's domain (p_i = 1/2), keeps every
                            step inside it (at most 0.99 of the way to its boundary) and
                            backtracks on D; the Newton operator is J + diag(lambda / (p (1-p))) */
    int support_stop;    /* > 0 (linear tensor kernel only): also stop a lambda once the
                            2-std support of w = (X^T alpha)^{m-1} (Section 6.3 threshold, as
                            tk_support) has stayed the same for this many consecutive Newton
                            steps; info.stop_reason records it.  0 (default): off */
    const double *support_X; /* device [n*support_d]: the points the tensor was built from */
    int64_t support_d;
} tk_solve_opts;

/* Why a solve that returned TK_OK stopped. */
typedef enum {
    TK_STOP_TOL = 0,     /* ||grad D|| <= tol * lambda * ||alpha|| (or an exactly zero gradient) */
    TK_STOP_SUPPORT = 1, /* the stable-support rule (opts.support_stop) */
    TK_STOP_FLOOR = 2    /* reduced-precision storage without a polish tensor: the gradient
                            stopped falling at the noise floor of the storage rounding (no
                            halving in 3 Newton steps, growth 1000x past its best, or a
                            line search whose predicted decrease is below the FP32 noise
                            of the objective, 1e-6 |D|); the
                            iterate of smallest gradient is returned and grad_norm is its
                            reduced-precision gradient.  By lambda-strong convexity the
                            error of alpha is at most ||grad D(alpha)|| / lambda with the
                            gradient of the FP64 problem, which a caller holding the FP64
                            tensor can evaluate with tk_contract */
} tk_stop_reason;

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
    int stop_reason;     /* with status TK_OK: what ended this lambda (tk_stop_reason) */
} tk_solve_info;

void tk_solve_opts_default(tk_solve_opts *h_opts);

int tk_solve_workspace(int64_t n, int m, int64_t B, int dtype, size_t *h_bytes);
/* Workspace of tk_solve_dual with opts->support_stop > 0 (points of dimension support_d). */
int tk_solve_workspace_ex(int64_t n, int m, int64_t B, int dtype, int64_t support_d, size_t *h_bytes);

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
 * Returns TK_OK when all converged, TK_ENOCONV if any did not (check h_info),
 * TK_ENAN when d_y (or the warm start) holds a NaN or Inf (checked before any
 * pass; outputs untouched) or an iterate became non-finite.
 */
int tk_solve_dual(const void *d_K, int dtype, int64_t n, int m, const double *d_y,
                  const double *h_lambdas, int64_t B, const tk_solve_opts *h_opts,
                  double *d_alpha, tk_solve_info *h_info, void *d_work, size_t work_bytes,
                  void *stream);

/*
 * Several packed tensors of the same (n, m, dtype) side by side: tensor t
 * starts k_stride entries after tensor t-1.  tk_packed_stride gives the
 * smallest stride that keeps every tensor 256-byte aligned (C(n+m-1, m)
 * rounded up); any larger stride with 16-byte alignment is accepted.  This is
 * the layout of the subsample grid of Section 6.1: T random draws of n
 * landmarks each, one tensor per draw.
 */
int tk_packed_stride(int64_t n, int m, int dtype, int64_t *h_stride);

/* Build T tensors: d_X [T*n*d] (draw t's points from row t*n), d_K [T*k_stride]. */
int tk_build_packed_multi(const double *d_X, int64_t T, int64_t n, int64_t d, int m, int kernel,
                          double kparam, int dtype, void *d_K, int64_t k_stride, void *stream);

/*
 * g_t = K_t . alpha_t^{m-1} for T tensors in one launch per pass (vector t
 * contracts tensor t; each tensor is read once).  d_alpha, d_g [T*n];
 * workspace tk_contract_workspace(n, m, T, dtype).  Errors: as tk_contract.
 */
int tk_contract_multi(const void *d_K, int dtype, int64_t n, int m, int64_t T, int64_t k_stride,
                      const double *d_alpha, double *d_g, int acc, void *d_work, size_t work_bytes,
                      void *stream);

/*
 * The (subsample, lambda) grid of Section 6.1: the dual of each of T tensors
 * (draws) for each of L regularisation values.  The draws of one lambda are
 * solved in lock step (up to 64 per batch: every pass over the tensors is one
 * launch for the batch), the lambdas by continuation from the largest down,
 * each draw keeping its own Hessian and preconditioner from lambda to lambda.
 * d_y [T*n] (draw t's responses from t*n); d_alpha [L*T*n] receives the
 * solutions, lambda-major: d_alpha[(l*T + t)*n + i]; h_info [L*T] the same
 * order.  opts as tk_solve_dual (no polish tensor, no support_stop; loss
 * allowed).  Workspace: tk_solve_workspace(n, m, min(T, 64), dtype).
 * Synchronises.  Returns TK_OK when every problem converged, else TK_ENOCONV /
 * TK_ENAN (check h_info).
 */
int tk_solve_dual_multi(const void *d_K, int dtype, int64_t n, int m, int64_t T, int64_t k_stride,
                        const double *d_y, const double *h_lambdas, int64_t L,
                        const tk_solve_opts *h_opts, double *d_alpha, tk_solve_info *h_info,
                        void *d_work, size_t work_bytes, void *stream);

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
 * Prediction with a general tensor kernel (Section 4: the model written
 * through the kernel, for feature maps with no finite form):
 *   f_b(x) = sum_{sorted (m-1)-tuples T of training points} c(T) alpha_b^T
 *            k(x_{T_1}, .., x_{T_{m-1}}, x),   c(T) = (m-1)! / prod_v mult_v(T)!
 * i.e. the sum over all ordered (m-1)-tuples grouped by their sorted form.
 * kernel/kparam as in tk_build_packed_tensor (linear, eq. poly_tensor, exp).
 * d_X [n*d] training points (or landmarks), d_alpha [B*n] dual vectors,
 * d_Xq [N*d] query points -> d_f [B*N].  FP64 throughout: the inner products
 * sum_j prod_{t in T} x_{t,j} xq_j run on FP64 MFMA tiles (64 tuples x 64
 * points), the weighted sums over tuples in a fixed order.  Work grows as
 * C(n+m-2, m-1) * N * d.  For the linear kernel tk_predict on the primal
 * weights is the cheap route (same value in exact arithmetic).
 * d_work: tk_predict_kernel_workspace bytes.
 * Errors: TK_EINVAL (sizes, m odd or > 8, N > 65535*64, kernel/kparam),
 * TK_EOVERFLOW, TK_ENOMEM (workspace too small), TK_EHIP.
 */
int tk_predict_kernel_workspace(int64_t n, int m, int64_t B, int64_t N, size_t *h_bytes);
int tk_predict_kernel(const double *d_X, int64_t n, int64_t d, int m, int kernel, double kparam,
                      const double *d_alpha, int64_t B, const double *d_Xq, int64_t N, double *d_f,
                      void *d_work, size_t work_bytes, void *stream);

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
 * Errors: TK_EINVAL, TK_ENOMEM, TK_EHIP; TK_ENAN when an input holds a NaN or
 * Inf (checked before any pass) or the result is not finite; TK_ENOCONV when
 * CG ends above cg_tol (max_cg reached or positive curvature lost) -- the
 * outputs then hold the last CG iterate's values.
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

/*
 * Instrumentation (not part of the method): a plain streaming read of `bytes`
 * bytes (a positive multiple of 16, d_src 16-byte aligned) by `groups`
 * workgroups of 256 threads, each thread keeping eight non-temporal 16-byte
 * loads in flight.  d_sink [groups] receives one word per workgroup (a checksum that
 * keeps the loads live).  Timed beside the kernels that stream the packed
 * tensor, it gives the achievable HBM read rate of the device.
 * Errors: TK_EINVAL, TK_EHIP.
 */
int tk_probe_stream_read(const void *d_src, int64_t bytes, uint64_t *d_sink, int groups, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TK_H */
