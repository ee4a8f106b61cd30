"""Pins of the oracle's general-loss dual (Section 4: the dual of
eq. tensor_infinite_2 through the Fenchel conjugate of the loss) for the
logistic loss, against what the mathematics fixes independently: the
conjugate as a numerical supremum, strong duality, an independent primal
solve, the p = 2 case as L2-regularised logistic regression (scikit-learn),
and finite differences of the dual gradient."""
import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from oracle import dual as D
from oracle import tensor as T


def _cls_data(seed, n=30, d=6):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    w = np.zeros(d)
    w[[0, 3]] = [1.5, -1.0]
    y = np.sign(X @ w + 0.3 * rng.standard_normal(n))
    y[y == 0] = 1.0
    return X, y


def test_conjugate_is_the_supremum():
    """L*(y, s) = sup_t (s t - L(y, t)), computed by a scalar maximisation."""
    rng = np.random.default_rng(0)
    for _ in range(40):
        y = rng.choice([-1.0, 1.0])
        u = rng.uniform(0.02, 0.98)
        s = -u * y
        res = minimize_scalar(lambda t: -(s * t - float(D.logistic_loss(y, t))), bounds=(-60, 60),
                              method="bounded", options={"xatol": 1e-12})
        assert float(D.logistic_conjugate(np.array([y]), np.array([s]))[0]) == pytest.approx(-res.fun, abs=1e-9)
    # outside u in [0, 1] the supremum is unbounded; at the ends it is 0
    assert np.isinf(D.logistic_conjugate(np.array([1.0]), np.array([0.5]))[0])
    assert D.logistic_conjugate(np.array([1.0, -1.0]), np.array([0.0, 1.0])).tolist() == [0.0, 0.0]


@pytest.mark.parametrize("m,lam", [(4, 0.1), (4, 1.0), (2, 0.5), (6, 0.3)])
def test_strong_duality_and_primal_solve(m, lam):
    """min F = -min Lambda at w* = (X^T alpha*)^{m-1} (eq. tensor_representer),
    and an independent L-BFGS solve of the primal reaches the same w."""
    X, y = _cls_data(1 + m)
    a, info = D.solve_logistic_linear(X, y, lam, m)
    assert info.converged
    w = D.primal_from_dual(X, a, m)
    Fp = D.logistic_primal_objective(X, y, w, lam, m)
    Ld = D.logistic_dual_objective(T.contract_closed(X, a, m), a, y, lam, m)
    assert Fp + Ld == pytest.approx(0.0, abs=1e-9 * (abs(Fp) + 1))
    p = m / (m - 1.0)

    def F(v):
        z = y * (X @ v)
        sig = 0.5 * (1 - np.tanh(0.5 * z))          # 1 / (1 + e^z)
        val = float(np.sum(np.logaddexp(0.0, -z))) / lam + float(np.sum(np.abs(v) ** p)) / p
        grad = -(X.T @ (y * sig)) / lam + np.sign(v) * np.abs(v) ** (p - 1)
        return val, grad

    res = minimize(F, np.zeros(X.shape[1]), jac=True, method="L-BFGS-B",
                   options={"maxiter": 20000, "ftol": 1e-16, "gtol": 1e-12})
    assert res.fun == pytest.approx(Fp, rel=1e-8)
    np.testing.assert_allclose(res.x, w, rtol=1e-4, atol=1e-4 * np.abs(w).max())


def test_order2_is_l2_logistic_regression():
    """m = 2 (p = 2): the primal is L2-regularised logistic regression with
    C = 1/lambda and no intercept; scikit-learn's solver gives the same w."""
    from sklearn.linear_model import LogisticRegression
    X, y = _cls_data(7, n=50, d=5)
    lam = 0.2
    a, _ = D.solve_logistic_linear(X, y, lam, 2)
    w = X.T @ a
    clf = LogisticRegression(C=1.0 / lam, fit_intercept=False, tol=1e-12, max_iter=10000).fit(X, y)
    np.testing.assert_allclose(w, clf.coef_[0], rtol=1e-6, atol=1e-8)


def test_dual_gradient_finite_differences():
    X, y = _cls_data(3)
    lam, m = 0.2, 4
    rng = np.random.default_rng(4)
    a = y * rng.uniform(0.1, 0.9, y.size) / lam       # p in (0.1, 0.9)
    g = T.contract_closed(X, a, m)
    gr = D.logistic_dual_grad(g, a, y, lam)
    h = 1e-6
    for i in range(0, y.size, 3):
        e = np.zeros_like(a)
        e[i] = h
        fp = D.logistic_dual_objective(T.contract_closed(X, a + e, m), a + e, y, lam, m)
        fm = D.logistic_dual_objective(T.contract_closed(X, a - e, m), a - e, y, lam, m)
        assert gr[i] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-7)
    # the separable Hessian diagonal against differences of the gradient
    hd = D.logistic_dual_hess_diag(a, y, lam)
    for i in range(0, y.size, 5):
        e = np.zeros_like(a)
        e[i] = h
        dg = (D.logistic_dual_grad(0.0, a + e, y, lam) - D.logistic_dual_grad(0.0, a - e, y, lam)) / (2 * h)
        assert hd[i] == pytest.approx(dg[i], rel=1e-6)


def test_square_loss_is_the_special_case():
    """The square loss L(y, t) = (y - t)^2 / 2 has L*(y, s) = s y + s^2 / 2, so
    gamma L*(y, -alpha/gamma) = -alpha y + lambda alpha^2 / 2: the dual solved
    for regression.  Checked as a numerical supremum."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        yv, s = rng.standard_normal(2)
        res = minimize_scalar(lambda t: -(s * t - 0.5 * (yv - t) ** 2))
        assert -res.fun == pytest.approx(s * yv + 0.5 * s * s, abs=1e-9)
