"""Dual problem, its solution and what is read off it (Sections 4 and 6).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Notation: m is the (even) tensor order, p = m/(m-1) the primal exponent and
lambda = 1/gamma the regularisation (the text weights the loss by gamma).

  primal (eq. tensor_primal, divided by gamma):
      P(w) = 1/(2 lambda) ||X w - y||^2 + (1/p) ||w||_p^p
  dual (eq. dual_tensor_kernel with 1/(2 gamma) = lambda/2):
      D(alpha) = (1/m) <K, alpha^{(x)m}> + (lambda/2) ||alpha||^2 - <y, alpha>
  gradient      grad D = g + lambda alpha - y,   g = K . alpha^{m-1}
  Hessian       J(alpha) + lambda I,   J = dg/dalpha = (m-1) K x_3 alpha .. x_m alpha
  representer   w = J_q(X^T alpha) = (X^T alpha)^{m-1}   (eq. tensor_representer, q = m even)

The solver is damped Newton with Armijo backtracking and a Cholesky solve of
the n x n Newton system.  Because D is lambda-strongly convex its minimiser is
unique, so any correct solver must reach the same alpha*.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla

from . import tensor as T


@dataclass
class SolveInfo:
    iterations: int
    grad_norm: float
    converged: bool
    objective: float


def dual_objective(g, alpha, y, lam: float, m: int) -> float:
    """D(alpha) from g = K.alpha^{m-1}; uses <K, alpha^{(x)m}> = alpha^T g."""
    return float(alpha @ g) / m + 0.5 * lam * float(alpha @ alpha) - float(y @ alpha)


def dual_grad(g, alpha, y, lam: float) -> np.ndarray:
    return g + lam * alpha - y


def solve_dual_newton(contract: Callable, jacobian: Callable, y, lam: float, m: int,
                      alpha0: Optional[np.ndarray] = None, rtol: float = 1e-14,
                      max_iter: int = 500) -> tuple:
    """Damped Newton on D.  Stops when ||grad D|| <= rtol * (||y|| + ||g|| + lam ||alpha||)
    or when the gradient norm stops decreasing (the rounding floor)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    a = np.zeros(n) if alpha0 is None else np.array(alpha0, dtype=np.float64)
    g = contract(a)
    f = dual_objective(g, a, y, lam, m)
    gr = dual_grad(g, a, y, lam)
    best = (np.linalg.norm(gr), a.copy())
    stall = 0
    it = 0
    converged = False
    for it in range(1, max_iter + 1):
        gn = np.linalg.norm(gr)
        scale = np.linalg.norm(y) + np.linalg.norm(g) + lam * np.linalg.norm(a)
        if gn <= rtol * scale:
            converged = True
            it -= 1
            break
        H = jacobian(a) + lam * np.eye(n)
        step = -sla.cho_solve(sla.cho_factor(H, lower=True), gr)
        slope = float(gr @ step)
        t = 1.0
        while True:
            a_new = a + t * step
            g_new = contract(a_new)
            f_new = dual_objective(g_new, a_new, y, lam, m)
            if f_new <= f + 1e-4 * t * slope or t < 1e-12:
                break
            t *= 0.5
        a, g, f = a_new, g_new, f_new
        gr = dual_grad(g, a, y, lam)
        gn_new = np.linalg.norm(gr)
        if gn_new < best[0]:
            best = (gn_new, a.copy())
        # rounding floor: near the solution, Newton steps that no longer halve
        # the gradient norm
        if gn_new > 0.5 * gn and gn < 1e-8 * scale:
            stall += 1
            if stall >= 3:
                converged = True
                break
        else:
            stall = 0
    gn, a = best
    g = contract(a)
    return a, SolveInfo(it, float(np.linalg.norm(dual_grad(g, a, y, lam))), converged,
                        dual_objective(g, a, y, lam, m))


def linear_callbacks(X, m: int):
    """Contraction and Jacobian of the linear tensor kernel in closed form."""
    return (lambda a: T.contract_closed(X, a, m)), (lambda a: T.jacobian_closed(X, a, m))


def packed_callbacks(K, n: int, m: int):
    """Contraction and Jacobian read from the packed array (any tensor kernel)."""
    return (lambda a: T.contract_packed(K, n, m, a)), (lambda a: T.jacobian_packed(K, n, m, a))


def solve_linear(X, y, lam: float, m: int, **kw):
    c, j = linear_callbacks(X, m)
    return solve_dual_newton(c, j, y, lam, m, **kw)


def dual_grad_exact_linear(X, y, lam: float, m: int, alpha) -> np.ndarray:
    """Gradient X (X^T alpha)^{m-1} + lam alpha - y of the dual objective of the
    linear tensor kernel (Section 3.2, closed form of K . alpha^{m-1}), evaluated
    in exact rational arithmetic on the given FP64 values and rounded once.

    Near the optimum the terms cancel by many orders of magnitude, so a plain
    FP64 evaluation loses most of its digits; this one does not.  Small
    problems only (cost grows with n d and the operand bit lengths)."""
    from fractions import Fraction
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    Xf = [[Fraction(float(v)) for v in row] for row in X]
    af = [Fraction(float(v)) for v in np.asarray(alpha, dtype=np.float64)]
    u = [sum((Xf[i][j] * af[i] for i in range(n)), Fraction(0)) for j in range(d)]
    w = [uj ** (m - 1) for uj in u]
    lf = Fraction(float(lam))
    yf = [Fraction(float(v)) for v in np.asarray(y, dtype=np.float64)]
    g = [sum((Xf[i][j] * w[j] for j in range(d)), Fraction(0)) + lf * af[i] - yf[i] for i in range(n)]
    return np.array([float(gi) for gi in g])


def refine_linear_exact(X, y, lam: float, m: int, alpha, steps: int = 2) -> np.ndarray:
    """Newton corrections alpha <- alpha - H^{-1} g with the gradient g taken
    exactly (dual_grad_exact_linear) and H = (m-1) X diag(u^{m-2}) X^T + lam I
    in FP64: the correction is tiny, so its own rounding does not matter, and
    the result is the FP64 point nearest (to within a few units in the last
    place times the condition number) to the exact optimum."""
    X = np.asarray(X, dtype=np.float64)
    a = np.array(alpha, dtype=np.float64)
    for _ in range(steps):
        g = dual_grad_exact_linear(X, y, lam, m, a)
        u = X.T @ a
        H = (m - 1) * (X * (u ** (m - 2))) @ X.T + lam * np.eye(a.size)
        a = a - sla.solve(H, g, assume_a="pos")
    return a


def refine_linear(X, y, lam: float, m: int, alpha, steps: int = 3) -> np.ndarray:
    """Newton corrections alpha <- alpha - H^{-1} g without line search, with
    the gradient of the linear tensor kernel's dual (Section 3.2 closed form)
    evaluated in extended precision (x87 80-bit long double: 11 more bits
    than FP64).  Near the optimum at small lambda, FP64 Newton iterates
    stagnate where the FP64 gradient's rounding meets the Hessian's
    conditioning; the extended gradient moves that floor down by ~2000x.
    H = (m-1) X diag(u^{m-2}) X^T + lam I in FP64."""
    X = np.asarray(X, dtype=np.float64)
    Xl = X.astype(np.longdouble)
    yl = np.asarray(y, dtype=np.float64).astype(np.longdouble)
    a = np.array(alpha, dtype=np.float64)
    for _ in range(steps):
        al = a.astype(np.longdouble)
        ul = Xl.T @ al
        g = np.asarray(Xl @ ul ** (m - 1) + np.longdouble(lam) * al - yl, dtype=np.float64)
        u = X.T @ a
        H = (m - 1) * (X * (u ** (m - 2))) @ X.T + lam * np.eye(a.size)
        a = a - sla.solve(H, g, assume_a="pos")
    return a


def solve_path(X, y, lambdas, m: int, **kw):
    """Independent solves along a lambda path, warm-started in increasing
    lambda order (the minimiser of each is unique, so warm starts only change
    the iteration count)."""
    lambdas = np.asarray(lambdas, dtype=np.float64)
    order = np.argsort(lambdas)
    out = np.zeros((lambdas.size, np.asarray(y).size))
    infos = [None] * lambdas.size
    a0 = None
    for k in order:
        a, info = solve_linear(X, y, float(lambdas[k]), m, alpha0=a0, **kw)
        out[k] = a
        infos[k] = info
        a0 = a
    return out, infos


def primal_from_dual(X, alpha, m: int) -> np.ndarray:
    """w = J_q(X^T alpha) = (X^T alpha)^{m-1} (eq. tensor_representer, q = m even)."""
    return (np.asarray(X, dtype=np.float64).T @ np.asarray(alpha, dtype=np.float64)) ** (m - 1)


def primal_objective(X, y, w, lam: float, m: int) -> float:
    p = m / (m - 1.0)
    r = np.asarray(X) @ w - y
    return float(r @ r) / (2.0 * lam) + float(np.sum(np.abs(w) ** p)) / p


def duality_gap(X, y, alpha, lam: float, m: int) -> float:
    """P(w(alpha)) + D(alpha) with w(alpha) from the representer."""
    w = primal_from_dual(X, alpha, m)
    g = T.contract_closed(X, alpha, m)
    return primal_objective(X, y, w, lam, m) + dual_objective(g, alpha, y, lam, m)


def support_threshold(w) -> tuple:
    """Section 6.3: features whose weight magnitude exceeds twice the standard
    deviation of the weights (population std, strict inequality)."""
    w = np.asarray(w, dtype=np.float64)
    tau = 2.0 * float(np.std(w))
    return np.abs(w) > tau, tau


def f1_score(mask, true_support) -> float:
    pred = set(np.flatnonzero(mask).tolist())
    true = set(np.asarray(true_support).tolist())
    tp = len(pred & true)
    if tp == 0:
        return 0.0
    prec = tp / len(pred)
    rec = tp / len(true)
    return 2 * prec * rec / (prec + rec)


def predict_linear(w, Xq) -> np.ndarray:
    """<w, x> for every query row (eq. tensor_1 left-hand side)."""
    return np.asarray(Xq, dtype=np.float64) @ w


def predict_kernel(X, alpha, Xq, m: int, kernel: str = "linear", kparam: float = 0.0) -> np.ndarray:
    """General tensor kernel prediction (Section 4, general feature map):
    f(x) = sum_{i_1..i_{m-1}} k(x_{i_1}, .., x_{i_{m-1}}, x) alpha_{i_1} .. alpha_{i_{m-1}},
    summed over sorted (m-1)-tuples times their number of orderings.  Python
    loops: small n only."""
    from itertools import combinations_with_replacement
    from math import factorial
    from collections import Counter
    X = np.asarray(X, dtype=np.float64)
    Xq = np.asarray(Xq, dtype=np.float64)
    n = X.shape[0]
    out = np.zeros(Xq.shape[0])
    Z = np.vstack([X, Xq])
    for t in combinations_with_replacement(range(n), m - 1):
        cnt = Counter(t)
        mult = factorial(m - 1)
        for c in cnt.values():
            mult //= factorial(c)
        coef = mult * float(np.prod(np.asarray(alpha)[list(t)]))
        for q in range(Xq.shape[0]):
            out[q] += coef * T.kernel_entry(Z, list(t) + [n + q], kernel, kparam)
    return out


def mse(f, y) -> float:
    """MSE of Section 6.1: mean of squared residuals."""
    r = np.asarray(f) - np.asarray(y)
    return float(r @ r) / r.size


def krr_closed_form(X, y, lam: float) -> np.ndarray:
    """Kernel ridge regression (m = 2): the dual eq. classic_dual with
    1/gamma = lambda is minimised by alpha = (X X^T + lambda I)^{-1} y."""
    X = np.asarray(X, dtype=np.float64)
    return np.linalg.solve(X @ X.T + lam * np.eye(X.shape[0]), y)


def dalpha_dlambda(jac, alpha, lam: float) -> np.ndarray:
    """Differentiating grad D(alpha*(lambda)) = 0 in lambda: (J + lambda I) dalpha/dlambda = -alpha*."""
    H = jac + lam * np.eye(alpha.size)
    return -np.linalg.solve(H, alpha)


def val_mse_linear(X, alpha, m: int, X_val, y_val) -> float:
    return mse(predict_linear(primal_from_dual(X, alpha, m), X_val), y_val)


def grad_alpha_val_mse(X, alpha, m: int, X_val, y_val) -> np.ndarray:
    """d MSE_val / d alpha = (2/N) (m-1) X diag(u^{m-2}) X_val^T r, u = X^T alpha."""
    X = np.asarray(X, dtype=np.float64)
    u = X.T @ alpha
    r = X_val @ (u ** (m - 1)) - y_val
    return (2.0 / y_val.size) * (m - 1) * (X @ ((u ** (m - 2)) * (X_val.T @ r)))


def dmse_dlambda_linear(X, alpha, lam: float, m: int, X_val, y_val) -> float:
    """dMSE_val/dlambda = grad_alpha MSE . dalpha*/dlambda = -z^T alpha* with
    (J + lambda I) z = grad_alpha MSE (J symmetric)."""
    H = T.jacobian_closed(X, alpha, m) + lam * np.eye(alpha.size)
    z = np.linalg.solve(H, grad_alpha_val_mse(X, alpha, m, X_val, y_val))
    return -float(z @ alpha)


# ---------------------------------------------------------------------------
# General convex loss through the Fenchel conjugate (Section 4, the dual of
# eq. tensor_infinite_2):
#     Lambda(alpha) = (1/q) ||Phi_n^* alpha||_q^q + gamma sum_i L*(y_i, -alpha_i / gamma),
# with (1/q) ||Phi_n^* alpha||_q^q = (1/m) <K, alpha^{(x)m}> (q = m) and
# gamma = 1/lambda.  For the square loss L(y, t) = (y - t)^2 / 2 this is the
# dual above.  The classification loss used here is the logistic loss
# L(y, t) = log(1 + exp(-y t)), y in {-1, +1} (the text prints 1 + e^{-yf};
# read as the logistic loss it names).  Its conjugate, with u = -s y:
#     L*(y, s) = u log u + (1 - u) log(1 - u)   for u in [0, 1], +inf otherwise,
# so the separable dual term is, with p_i = lambda y_i alpha_i in [0, 1],
#     gamma L*(y_i, -alpha_i / gamma) = (1/lambda) [p_i log p_i + (1 - p_i) log(1 - p_i)].
# ---------------------------------------------------------------------------

def logistic_loss(y, t) -> np.ndarray:
    """L(y, t) = log(1 + exp(-y t)), evaluated without overflow."""
    return np.logaddexp(0.0, -np.asarray(y, dtype=np.float64) * np.asarray(t, dtype=np.float64))


def logistic_conjugate(y, s) -> np.ndarray:
    """L*(y, s) = sup_t (s t - L(y, t)) = u log u + (1 - u) log(1 - u), u = -s y,
    +inf outside u in [0, 1] (0 log 0 = 0)."""
    u = -np.asarray(s, dtype=np.float64) * np.asarray(y, dtype=np.float64)
    out = np.full(u.shape, np.inf)
    ok = (u >= 0) & (u <= 1)
    uu = u[ok]
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(uu > 0, uu * np.log(np.where(uu > 0, uu, 1.0)), 0.0)
        b = np.where(uu < 1, (1 - uu) * np.log(np.where(uu < 1, 1 - uu, 1.0)), 0.0)
    out[ok] = a + b
    return out


def logistic_dual_objective(g, alpha, y, lam: float, m: int) -> float:
    """Lambda(alpha) from g = K . alpha^{m-1} (<K, alpha^{(x)m}> = alpha^T g)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    sep = logistic_conjugate(y, -lam * alpha)          # L*(y_i, -alpha_i / gamma), gamma = 1/lam
    return float(alpha @ g) / m + float(np.sum(sep)) / lam


def logistic_dual_grad(g, alpha, y, lam: float) -> np.ndarray:
    """d Lambda / d alpha = g + y log(p / (1 - p)), p = lam y alpha (inside the domain)."""
    p = lam * np.asarray(y) * np.asarray(alpha)
    return g + np.asarray(y) * (np.log(p) - np.log1p(-p))


def logistic_dual_hess_diag(alpha, y, lam: float) -> np.ndarray:
    """Second derivative of the separable term: lam / (p (1 - p))."""
    p = lam * np.asarray(y) * np.asarray(alpha)
    return lam / (p * (1.0 - p))


def solve_dual_logistic(contract: Callable, jacobian: Callable, y, lam: float, m: int,
                        alpha0: Optional[np.ndarray] = None, rtol: float = 1e-14,
                        max_iter: int = 500) -> tuple:
    """Damped Newton on the logistic dual, from the centre of the domain
    (p_i = 1/2) unless alpha0 is given.  Each step solves (J + diag(h)) s = -grad
    by Cholesky, is shortened to stay inside the domain (at most 0.99 of the way
    to its boundary), then backtracked (Armijo).  Stops when ||grad|| <= rtol *
    (||g|| + ||sep. gradient|| + 1) or when the gradient stops decreasing."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    a = y / (2.0 * lam) if alpha0 is None else np.array(alpha0, dtype=np.float64)
    g = contract(a)
    f = logistic_dual_objective(g, a, y, lam, m)
    gr = logistic_dual_grad(g, a, y, lam)
    best = (np.linalg.norm(gr), a.copy())
    stall = 0
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        gn = np.linalg.norm(gr)
        scale = np.linalg.norm(g) + np.linalg.norm(gr - g) + 1.0
        if gn <= rtol * scale:
            converged = True
            it -= 1
            break
        H = jacobian(a) + np.diag(logistic_dual_hess_diag(a, y, lam))
        step = -sla.cho_solve(sla.cho_factor(H, lower=True), gr)
        # largest t keeping p + t dp inside (0, 1), dp = lam y step
        p = lam * y * a
        dp = lam * y * step
        tmax = np.inf
        neg, pos = dp < 0, dp > 0
        if neg.any():
            tmax = min(tmax, float(np.min(-p[neg] / dp[neg])))
        if pos.any():
            tmax = min(tmax, float(np.min((1 - p[pos]) / dp[pos])))
        t = min(1.0, 0.99 * tmax)
        slope = float(gr @ step)
        while True:
            a_new = a + t * step
            g_new = contract(a_new)
            f_new = logistic_dual_objective(g_new, a_new, y, lam, m)
            if f_new <= f + 1e-4 * t * slope or t < 1e-14:
                break
            t *= 0.5
        a, g, f = a_new, g_new, f_new
        gr = logistic_dual_grad(g, a, y, lam)
        gn_new = np.linalg.norm(gr)
        if gn_new < best[0]:
            best = (gn_new, a.copy())
        if gn_new > 0.5 * gn and gn < 1e-8 * scale:
            stall += 1
            if stall >= 3:
                converged = True
                break
        else:
            stall = 0
    gn, a = best
    g = contract(a)
    return a, SolveInfo(it, float(np.linalg.norm(logistic_dual_grad(g, a, y, lam))), converged,
                        logistic_dual_objective(g, a, y, lam, m))


def solve_logistic_linear(X, y, lam: float, m: int, **kw):
    c, j = linear_callbacks(X, m)
    return solve_dual_logistic(c, j, y, lam, m, **kw)


def logistic_primal_objective(X, y, w, lam: float, m: int) -> float:
    """F(w) = gamma sum_i L(y_i, <x_i, w>) + (1/p) ||w||_p^p (eq. tensor_infinite_2, gamma = 1/lam)."""
    p = m / (m - 1.0)
    return float(np.sum(logistic_loss(y, np.asarray(X) @ w))) / lam + float(np.sum(np.abs(w) ** p)) / p
