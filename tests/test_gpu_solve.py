"""GPU parity of the dual solve, primal recovery, prediction, support, landmark
gather and the implicit lambda derivative, against the CPU oracle."""
import numpy as np
import pytest
import torch

import paper_2003_10482_amd as tk
from gpu_util import device, to_dev, to_np
from oracle import dual as D
from oracle import tensor as T
from synth import make_workload, planted_regression, random_alpha

pytestmark = pytest.mark.gpu


def _solve(wl, lambdas, dtype="f64", **kw):
    Xd = to_dev(wl.X)
    K = tk.build_packed_tensor(Xd, wl.m, dtype=dtype)
    alpha, infos = tk.solve_dual(K, to_dev(wl.y), lambdas, **kw)
    return K, alpha, infos


def _dyadic_problem(n=64, d=20, seed=21):
    """Points with entries k/16: the packed FP64 tensor is then exact, so the
    GPU solves exactly the oracle's problem and alpha itself can be compared."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-40, 41, size=(n, d)) / 16.0
    w = np.zeros(d)
    w[rng.choice(d, 4, replace=False)] = rng.uniform(-1, 1, 4)
    y = X @ w + 0.01 * rng.standard_normal(n)
    return X, y, w


def test_solve_exact_tensor_alpha_parity():
    """North-star accuracy of the FP64 path: alpha within 1e-10 relative of the
    oracle's closed-form solution when the stored tensor is exact."""
    X, y, _ = _dyadic_problem()
    K = tk.build_packed_tensor(to_dev(X), 4)
    lams = [1.0, 1e-1, 1e-2, 3e-3]
    alpha, infos = tk.solve_dual(K, to_dev(y), lams, tol=1e-12)
    for b, lam in enumerate(lams):
        assert infos[b]["status"] == 0, infos[b]
        # the oracle's FP64 solve is itself limited by the cancellation in its
        # gradient; refine it with exactly computed gradients
        ref, _ = D.solve_linear(X, y, lam, 4)
        ref = D.refine_linear_exact(X, y, lam, 4, ref)
        assert np.linalg.norm(to_np(alpha[b]) - ref) <= 1e-10 * np.linalg.norm(ref), (lam, infos[b])


def test_solve_config1_matches_oracle():
    wl = make_workload("c1_n64_m4")
    K, alpha, infos = _solve(wl, [wl.lam])
    assert infos[0]["status"] == 0, infos
    a = to_np(alpha[0])
    ref, rinfo = D.solve_linear(wl.X, wl.y, wl.lam, wl.m)
    # Gaussian points: each stored FP64 entry carries one rounding, which the
    # cancellation at the optimum passes on to alpha's null(X^T) component
    assert np.linalg.norm(a - ref) <= 1e-8 * np.linalg.norm(ref)
    w = to_np(tk.primal_weights(to_dev(wl.X), alpha[0], wl.m))
    w_ref = D.primal_from_dual(wl.X, ref, wl.m)
    np.testing.assert_allclose(w, w_ref, rtol=1e-9, atol=1e-12 * np.abs(w_ref).max())
    mask, tau = tk.support(to_dev(w))
    mref, tref = D.support_threshold(w_ref)
    assert np.array_equal(to_np(mask), mref)


@pytest.mark.parametrize("m", [4, 6])
def test_solve_without_assembled_hessian(m):
    """precond=False: truncated Newton with unpreconditioned CG whose products
    are directional-derivative passes over the tensor (no Hessian kernel),
    backtracking line search; same optimum as the default solver."""
    wl = make_workload("c1_n64_m4")
    X, y = to_dev(wl.X), to_dev(wl.y)
    K = tk.build_packed_tensor(X, m)
    a1, i1 = tk.solve_dual(K, y, [wl.lam], tol=1e-11, precond=False)
    a2, i2 = tk.solve_dual(K, y, [wl.lam], tol=1e-11)
    assert i1[0]["status"] == 0 and i2[0]["status"] == 0, (i1, i2)
    assert i1[0]["hess_passes"] == 0 and i2[0]["hess_passes"] > 0
    ref, _ = D.solve_linear(wl.X, wl.y, wl.lam, m)
    w_ref = D.primal_from_dual(wl.X, ref, m)
    for a in (a1, a2):
        w = to_np(tk.primal_weights(X, a[0], m))
        assert np.linalg.norm(w - w_ref) <= 1e-8 * np.linalg.norm(w_ref)


@pytest.mark.parametrize("lam", [1.0, 1e-1])
def test_solve_order2_is_krr(lam):
    rng = np.random.default_rng(5)
    X, y, _, _ = planted_regression(rng, 40, 12, 3, 0.05)
    K = tk.build_packed_tensor(to_dev(X), 2)
    alpha, infos = tk.solve_dual(K, to_dev(y), [lam])
    ref = D.krr_closed_form(X, y, lam)
    np.testing.assert_allclose(to_np(alpha[0]), ref, rtol=1e-10, atol=1e-12)


def test_solve_lambda_batch_matches_oracle():
    wl = make_workload("c1_n64_m4")
    lams = [1.0, 1e-1, 1e-2, 3e-3]
    K, alpha, infos = _solve(wl, lams)
    for b, lam in enumerate(lams):
        ref, _ = D.solve_linear(wl.X, wl.y, lam, wl.m)
        w = D.primal_from_dual(wl.X, to_np(alpha[b]), wl.m)
        w_ref = D.primal_from_dual(wl.X, ref, wl.m)
        assert np.linalg.norm(w - w_ref) <= 1e-9 * np.linalg.norm(w_ref), (lam, infos[b])
        assert np.linalg.norm(to_np(alpha[b]) - ref) <= 1e-7 * np.linalg.norm(ref), (lam, infos[b])


def test_predict_and_dense_ops():
    wl = make_workload("c5_n128_m6")
    A = random_alpha(128, seed=4, batch=2) * 0.1
    W = tk.primal_weights(to_dev(wl.X), to_dev(A), 6)
    f = tk.predict(W, to_dev(wl.X_val))
    for b in range(2):
        w_ref = D.primal_from_dual(wl.X, A[b], 6)
        np.testing.assert_allclose(to_np(W[b]), w_ref, rtol=1e-10, atol=1e-14 * np.abs(w_ref).max())
        f_ref = D.predict_linear(w_ref, wl.X_val)
        np.testing.assert_allclose(to_np(f[b]), f_ref, rtol=1e-9, atol=1e-12 * np.abs(f_ref).max())


def test_gather_rows_landmarks():
    wl = make_workload("c3_nystrom")
    Xd = to_dev(wl.X)
    idx = torch.as_tensor(wl.landmarks, device=device())
    Xl = tk.gather_rows(Xd, idx)
    np.testing.assert_array_equal(to_np(Xl), wl.X[wl.landmarks])
    with pytest.raises(RuntimeError):
        tk.gather_rows(Xd, torch.as_tensor([0, wl.X.shape[0]], dtype=torch.int64, device=device()))


def test_dmse_dlambda_matches_oracle():
    rng = np.random.default_rng(8)
    X, y, w, _ = planted_regression(rng, 40, 10, 3, 0.05, n_extra=200)
    Xt, yt, Xv, yv = X[:40], y[:40], X[40:], y[40:]
    m, lam = 4, 0.05
    a, _ = D.solve_linear(Xt, yt, lam, m)
    K = tk.build_packed_tensor(to_dev(Xt), m)
    mse, dmse, z = tk.dmse_dlambda(K, to_dev(Xt), to_dev(a), lam, to_dev(Xv), to_dev(yv))
    assert mse == pytest.approx(D.val_mse_linear(Xt, a, m, Xv, yv), rel=1e-11)
    assert dmse == pytest.approx(D.dmse_dlambda_linear(Xt, a, lam, m, Xv, yv), rel=1e-7)
    h = to_np(tk.hvp(K, to_dev(a), to_dev(random_alpha(40, 3)), acc=tk.ACC_COMPENSATED))
    np.testing.assert_allclose(h, T.hvp_closed(Xt, a, random_alpha(40, 3), m), rtol=1e-9,
                               atol=1e-12 * np.abs(h).max())


def test_autograd_backward_is_hvp():
    n, m = 20, 4
    X = np.random.default_rng(1).standard_normal((n, 6))
    K = tk.build_packed_tensor(to_dev(X), m)
    a = to_dev(random_alpha(n, 3)).requires_grad_(True)
    gvec = to_dev(random_alpha(n, 4))
    out = tk.contract_autograd(K, a)
    (out * gvec).sum().backward()
    ref = T.hvp_closed(X, to_np(a.detach()), to_np(gvec), m)
    np.testing.assert_allclose(to_np(a.grad), ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("m", [2, 4, 6])
def test_solve_zero_targets(m):
    """y = 0: the dual objective (strictly convex for lambda > 0) has its
    minimum at alpha = 0, where the gradient is exactly zero, so the solve
    stops there at once, for every lambda and storage type."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((40, 8))
    y = np.zeros(40)
    lams = [1.0, 1e-2, 1e-4]
    for dtype in ("f64", "f32"):
        K = tk.build_packed_tensor(to_dev(X), m, dtype=dtype)
        alpha, infos = tk.solve_dual(K, to_dev(y), lams)
        assert not to_np(alpha).any()
        for inf in infos:
            assert inf["status"] == 0 and inf["newton_iters"] == 0, inf


def _abs_terms_predict(X, a, Xq, m, kernel, kparam):
    """Sum of the absolute values of the terms of f (every term made
    nonnegative): |k| <= linear(|X|, |Xq|)^s for the linear and polynomial
    kernels, and exp is positive."""
    if kernel == "exp":
        return D.predict_kernel(X, np.abs(a), Xq, m, "exp")
    return D.predict_kernel(np.abs(X), np.abs(a), np.abs(Xq), m, kernel, kparam)


@pytest.mark.parametrize("kernel,kparam", [("linear", 0.0), ("poly", 2), ("poly", 3), ("exp", 0.0)])
@pytest.mark.parametrize("n,m,N", [(12, 4, 70), (30, 2, 65), (7, 6, 9), (1, 4, 3)])
def test_predict_general_kernel_matches_oracle(kernel, kparam, n, m, N):
    """General-kernel prediction through the C ABI against the oracle's
    expansion over sorted (m-1)-tuples: several tuple tiles and a ragged query
    tile; held to 1e-12 of the sum of the absolute values of the terms."""
    rng = np.random.default_rng(100 + n + m)
    d = 5
    X = 0.5 * rng.standard_normal((n, d))
    Xq = 0.5 * rng.standard_normal((N, d))
    A = random_alpha(n, seed=7 + m, batch=3)
    f = to_np(tk.predict_kernel(to_dev(X), to_dev(A), to_dev(Xq), m, kernel, kparam))
    assert f.shape == (3, N)
    for b in range(3):
        ref = D.predict_kernel(X, A[b], Xq, m, kernel, kparam)
        E = _abs_terms_predict(X, A[b], Xq, m, kernel, kparam)
        assert np.all(np.abs(f[b] - ref) <= 1e-12 * E + 1e-300), (b, np.max(np.abs(f[b] - ref) / E))


@pytest.mark.parametrize("kernel,kparam", [("poly", 2), ("exp", 0.0)])
def test_predict_at_training_points_is_the_contraction(kernel, kparam):
    """At a training point x_a the prediction is (K . alpha^{m-1})_a: the
    general prediction and the packed contraction agree."""
    rng = np.random.default_rng(5)
    n, d, m = 70, 6, 4
    X = 0.4 * rng.standard_normal((n, d))
    a = random_alpha(n, seed=6)
    Xd = to_dev(X)
    K = tk.build_packed_tensor(Xd, m, kernel=kernel, kparam=kparam)
    g = to_np(tk.contract(K, to_dev(a), acc=tk.ACC_COMPENSATED))
    f = to_np(tk.predict_kernel(Xd, to_dev(a), Xd, m, kernel, kparam))
    # both kernels are nonnegative here (even degree, exp), so the oracle's
    # contraction of the tensor with |alpha| is the sum of |terms|
    E = T.contract_packed(T.build_packed(X, m, kernel, kparam), n, m, np.abs(a))
    assert np.all(np.abs(f - g) <= 1e-12 * E)


def test_predict_general_batch_above_chunk():
    """More vectors than one launch carries (16): chunked over the batch; the
    linear kernel equals <w_b, x> with w_b = (X^T alpha_b)^{m-1}."""
    rng = np.random.default_rng(12)
    n, d, m, N = 40, 7, 4, 33
    X = rng.standard_normal((n, d))
    Xq = rng.standard_normal((N, d))
    A = random_alpha(n, seed=13, batch=21)
    f = to_np(tk.predict_kernel(to_dev(X), to_dev(A), to_dev(Xq), m))
    for b in range(21):
        ref = D.predict_linear(D.primal_from_dual(X, A[b], m), Xq)
        E = np.abs(Xq) @ ((np.abs(X).T @ np.abs(A[b])) ** (m - 1))
        assert np.all(np.abs(f[b] - ref) <= 1e-12 * E)


@pytest.mark.parametrize("kernel,kparam,lam", [("poly", 2, 0.1), ("exp", 0.0, 0.1), ("poly", 2, 1e-2)])
def test_solve_general_kernel_matches_oracle(kernel, kparam, lam):
    """Dual solve on a polynomial (degree 2, as used in Section 6.2) and on an
    exponential tensor kernel against the oracle's damped Newton on the packed
    tensor, then prediction on held-out points with each side's alpha."""
    rng = np.random.default_rng(31)
    n, d, m = 24, 6, 4
    X = 0.5 * rng.standard_normal((n + 30, d))
    w = np.zeros(d)
    w[[1, 4]] = [1.0, -0.7]
    y = X @ w + 0.05 * rng.standard_normal(n + 30)
    Xt, yt, Xq = X[:n], y[:n], X[n:]
    K_or = T.build_packed(Xt, m, kernel, kparam)
    c, j = D.packed_callbacks(K_or, n, m)
    ref, info = D.solve_dual_newton(c, j, yt, lam, m)
    K = tk.build_packed_tensor(to_dev(Xt), m, kernel=kernel, kparam=kparam)
    alpha, infos = tk.solve_dual(K, to_dev(yt), [lam], tol=1e-11)
    assert infos[0]["status"] == 0, infos
    a = to_np(alpha[0])
    assert np.linalg.norm(a - ref) <= 1e-8 * np.linalg.norm(ref), np.linalg.norm(a - ref) / np.linalg.norm(ref)
    f = to_np(tk.predict_kernel(to_dev(Xt), alpha[0], to_dev(Xq), m, kernel, kparam))
    f_ref = D.predict_kernel(Xt, ref, Xq, m, kernel, kparam)
    E = _abs_terms_predict(Xt, ref, Xq, m, kernel, kparam)
    assert np.all(np.abs(f - f_ref) <= 1e-7 * E)


def test_nonfinite_inputs_are_rejected():
    """tk_solve_dual and tk_dmse_dlambda check their inputs and return TK_ENAN
    (-6) before any pass."""
    rng = np.random.default_rng(2)
    n, d, m = 20, 5, 4
    X = rng.standard_normal((n, d))
    y = rng.standard_normal(n)
    K = tk.build_packed_tensor(to_dev(X), m)
    for bad in (np.nan, np.inf):
        yb = y.copy()
        yb[7] = bad
        with pytest.raises(tk.api._lib.TkError) as ei:
            tk.solve_dual(K, to_dev(yb), [0.1], raise_on_noconv=True)
        assert ei.value.code == -6
        a0 = np.zeros(n)
        a0[3] = bad
        with pytest.raises(tk.api._lib.TkError) as ei:
            tk.solve_dual(K, to_dev(y), [0.1], alpha0=to_dev(a0[None, :]), raise_on_noconv=True)
        assert ei.value.code == -6
        Xv = rng.standard_normal((30, d))
        yv = rng.standard_normal(30)
        yv[0] = bad
        with pytest.raises(tk.api._lib.TkError) as ei:
            tk.dmse_dlambda(K, to_dev(X), to_dev(np.ones(n)), 0.1, to_dev(Xv), to_dev(yv))
        assert ei.value.code == -6


def test_dmse_dlambda_reports_unconverged_cg():
    """A CG limit below what the system needs is reported as TK_ENOCONV (-5)."""
    rng = np.random.default_rng(8)
    X, y, w, _ = planted_regression(rng, 40, 10, 3, 0.05, n_extra=200)
    Xt, yt, Xv, yv = X[:40], y[:40], X[40:], y[40:]
    a, _ = D.solve_linear(Xt, yt, 0.05, 4)
    K = tk.build_packed_tensor(to_dev(Xt), 4)
    with pytest.raises(tk.api._lib.TkError) as ei:
        tk.dmse_dlambda(K, to_dev(Xt), to_dev(a), 0.05, to_dev(Xv), to_dev(yv), cg_tol=1e-14, max_cg=2)
    assert ei.value.code == -5
