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
