"""Pins for the oracle's dual solve, primal recovery, prediction, support
selection and model-selection derivatives (Sections 3, 4, 6)."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import dual as D
from oracle import precision as P
from oracle import tensor as T
from synth import make_workload, random_alpha


def _small(seed=0, n=24, d=10, s=3, sigma=0.05):
    from synth import planted_regression
    rng = np.random.default_rng(seed)
    X, y, w, sup = planted_regression(rng, n, d, s, sigma)
    return X, y, w, sup


def test_duality_maps_inverse_and_conjugate_identity():
    """J_p o J_q = Id (Section 4) and eq. tensor_sub_jq:
    u^T J_q(u) - (1/p)||J_q(u)||_p^p = (1/q)||u||_q^q."""
    rng = np.random.default_rng(0)
    for q in (2, 4, 6, 8):
        p = q / (q - 1.0)
        u = rng.standard_normal(50)
        Jq = np.sign(u) * np.abs(u) ** (q - 1)
        Jp = np.sign(Jq) * np.abs(Jq) ** (p - 1)
        np.testing.assert_allclose(Jp, u, rtol=1e-12)
        # q even: J_q(u) = u^{q-1}
        np.testing.assert_allclose(Jq, u ** (q - 1), rtol=1e-14)
        lhs = u @ Jq - np.sum(np.abs(Jq) ** p) / p
        assert lhs == pytest.approx(np.sum(np.abs(u) ** q) / q, rel=1e-12)


def test_order2_is_kernel_ridge_regression():
    """m = 2: the dual is the kernel ridge dual (eq. classic_dual), whose
    minimiser is (X X^T + lambda I)^{-1} y (LAPACK solve)."""
    X, y, _, _ = _small(1)
    for lam in (1e-3, 1e-1, 1.0):
        ref = D.krr_closed_form(X, y, lam)
        H = X @ X.T + lam * np.eye(X.shape[0])
        tol = 100 * np.linalg.cond(H) * 2.0 ** -53      # both solves are backward stable
        a, info = D.solve_linear(X, y, lam, 2)
        assert np.linalg.norm(a - ref) <= tol * np.linalg.norm(ref)
        K = T.build_packed(X, 2)
        c, j = D.packed_callbacks(K, X.shape[0], 2)
        a2, _ = D.solve_dual_newton(c, j, y, lam, 2)
        assert np.linalg.norm(a2 - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("m", [4, 6])
def test_gap_identity_at_arbitrary_alpha(m):
    """P(w(alpha)) + D(alpha) = ||grad D(alpha)||^2 / (2 lambda) for the linear kernel."""
    X, y, _, _ = _small(2)
    for s in range(5):
        a = 0.3 * random_alpha(X.shape[0], 40 + s)
        lam = 10.0 ** (-s)
        gap = D.duality_gap(X, y, a, lam, m)
        gr = D.dual_grad(T.contract_closed(X, a, m), a, y, lam)
        assert gap == pytest.approx(gr @ gr / (2 * lam), rel=1e-9)
        assert gap >= 0


@pytest.mark.parametrize("m,lam", [(4, 1e-2), (4, 1.0), (6, 1e-2), (4, 1e-4)])
def test_optimality_conditions_and_strong_duality(m, lam):
    X, y, _, _ = _small(3)
    a, info = D.solve_linear(X, y, lam, m)
    assert info.converged
    w = D.primal_from_dual(X, a, m)
    p = m / (m - 1.0)
    # eq. jp_4 (gamma^{-1} = lambda): X^T (X w - y) + lambda J_p(w) = 0
    # both residuals equal -X^T grad D and -grad D in exact arithmetic, so they
    # are bounded by the dual gradient norm the solve reached (plus rounding)
    floor = info.grad_norm + 1e-13 * (np.linalg.norm(y) + lam * np.linalg.norm(a))
    assert info.grad_norm <= 1e-6 * np.linalg.norm(y)
    r = X.T @ (X @ w - y) + lam * np.sign(w) * np.abs(w) ** (p - 1)
    assert np.linalg.norm(r) <= 4 * np.linalg.norm(X, 2) * floor
    # eq. tensor_sub_r: X w = y - lambda alpha
    assert np.linalg.norm(X @ w - (y - lam * a)) <= 4 * floor
    # strong duality (Section 4): min P = -min D
    Pw = D.primal_objective(X, y, w, lam, m)
    assert Pw == pytest.approx(-info.objective, rel=1e-9, abs=1e-10)


def test_independent_primal_solve_matches():
    """Minimising the d-dimensional primal directly (L-BFGS, SciPy) reaches
    the w recovered from the dual through the representer."""
    X, y, _, _ = _small(4, n=30, d=6)
    m, lam = 4, 0.05
    p = m / (m - 1.0)
    a, _ = D.solve_linear(X, y, lam, m)
    w_dual = D.primal_from_dual(X, a, m)

    def f(w):
        r = X @ w - y
        val = r @ r / (2 * lam) + np.sum(np.abs(w) ** p) / p
        grad = X.T @ r / lam + np.sign(w) * np.abs(w) ** (p - 1)
        return val, grad
    res = minimize(f, np.zeros(X.shape[1]), jac=True, method="L-BFGS-B",
                   options={"maxiter": 20000, "gtol": 1e-12, "ftol": 1e-15})
    np.testing.assert_allclose(res.x, w_dual, rtol=2e-4, atol=2e-5)


def test_packed_solve_matches_closed_form_solve():
    X, y, _, _ = _small(5, n=12, d=5)
    for m in (4, 6):
        K = T.build_packed(X, m)
        c, j = D.packed_callbacks(K, X.shape[0], m)
        a_p, ip = D.solve_dual_newton(c, j, y, 1e-2, m)
        a_c, ic = D.solve_linear(X, y, 1e-2, m)
        # strong convexity: |a_p - a*| <= |grad D(a_p)|/lambda, where the packed
        # gradient carries its own rounding (bounded by u * sum|terms| * count)
        E = T.abs_bound_closed(X, a_p, m)
        slack = np.linalg.norm(E) * 2.0 ** -53 * T.packed_count(X.shape[0], m)
        assert np.linalg.norm(a_p - a_c) <= (ip.grad_norm + ic.grad_norm + slack) / 1e-2
        w_p, w_c = D.primal_from_dual(X, a_p, m), D.primal_from_dual(X, a_c, m)
        np.testing.assert_allclose(w_p, w_c, rtol=1e-6, atol=1e-8 * np.abs(w_c).max())


def test_planted_support_recovery():
    """Section 6.3 thresholding recovers the planted support of the synthetic
    data model (Section 5.4) on the order-4 workloads."""
    wl = make_workload("c2_n256_m4")
    a, _ = D.solve_linear(wl.X, wl.y, wl.lam, wl.m)
    mask, tau = D.support_threshold(D.primal_from_dual(wl.X, a, wl.m))
    assert D.f1_score(mask, wl.support) == 1.0
    wl = make_workload("c1_n64_m4")
    a, _ = D.solve_linear(wl.X, wl.y, wl.lam, wl.m)
    mask, _ = D.support_threshold(D.primal_from_dual(wl.X, a, wl.m))
    assert D.f1_score(mask, wl.support) >= 0.8


def test_support_threshold_rule():
    w = np.array([0.0, 1.0, -3.0, 0.5, 0.0, 0.0, 0.0, 0.0])
    mask, tau = D.support_threshold(w)
    assert tau == pytest.approx(2 * np.sqrt(np.mean((w - w.mean()) ** 2)))
    assert np.flatnonzero(mask).tolist() == [2]
    assert D.f1_score(mask, [2]) == 1.0
    assert D.f1_score(mask, [1, 2]) == pytest.approx(2 * 1 * 0.5 / 1.5)


def test_prediction_general_equals_primal_linear():
    """eq. tensor_1: sum_j (sum_i alpha_i x_ij)^{m-1} x_j equals the multilinear
    kernel expansion over (m-1)-tuples of training points."""
    X, y, _, _ = _small(6, n=6, d=4)
    Xq = np.random.default_rng(9).standard_normal((3, 4))
    for m in (2, 4):
        a = random_alpha(6, 11 + m)
        f_k = D.predict_kernel(X, a, Xq, m)
        f_w = D.predict_linear(D.primal_from_dual(X, a, m), Xq)
        np.testing.assert_allclose(f_k, f_w, rtol=1e-12)


@pytest.mark.parametrize("kernel,kparam", [("poly", 2), ("poly", 3), ("exp", 0.0), ("linear", 0.0)])
@pytest.mark.parametrize("m", [2, 4])
def test_prediction_general_kernel_bruteforce(kernel, kparam, m):
    """General-feature-map prediction (Section 4, after eq. tensor_1):
    f(x) = sum over ordered (m-1)-tuples of k(x_{i_1}, .., x_{i_{m-1}}, x)
    alpha_{i_1} .. alpha_{i_{m-1}}.  Pinned against the full tensor of the
    training and query points together (einsum of the linear kernel, then the
    polynomial power or the exponential), and at training points against the
    contraction (f(x_a) = (K alpha^{m-1})_a)."""
    rng = np.random.default_rng(40 + m)
    n, d, N = 5, 3, 4
    X = 0.6 * rng.standard_normal((n, d))
    Xq = 0.6 * rng.standard_normal((N, d))
    a = random_alpha(n, 41 + m)
    Z = np.vstack([X, Xq])
    lin = T.full_tensor_linear(Z, m)
    F = lin ** int(kparam) if kernel == "poly" else (np.exp(lin) if kernel == "exp" else lin)
    ref = np.empty(N)
    for q in range(N):
        sl = F[(slice(0, n),) * (m - 1) + (n + q,)]
        ref[q] = float(T.contract_full(sl, a) @ a) if m > 2 else float(sl @ a)
    got = D.predict_kernel(X, a, Xq, m, kernel, kparam)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    # at the training points the prediction is the gradient map K . alpha^{m-1}
    g_full = T.contract_full(F[(slice(0, n),) * m], a)
    np.testing.assert_allclose(D.predict_kernel(X, a, X, m, kernel, kparam), g_full, rtol=1e-12,
                               atol=1e-14 * np.abs(g_full).max())
    # a plausible mistake (every sorted tuple counted once, no multiplicity)
    # must be caught by the brute-force pin
    if m > 2:
        from itertools import combinations_with_replacement
        wrong = np.zeros(N)
        for t in combinations_with_replacement(range(n), m - 1):
            c = float(np.prod(a[list(t)]))
            for q in range(N):
                wrong[q] += c * F[tuple(t) + (n + q,)]
        assert not np.allclose(wrong, ref, rtol=1e-6)


def test_mse_definition():
    assert D.mse([1.0, 2.0, 4.0], [1.0, 1.0, 1.0]) == pytest.approx((0 + 1 + 9) / 3)


@pytest.mark.parametrize("m", [4, 6])
def test_dalpha_dlambda_and_dmse_against_finite_differences(m):
    X, y, _, _ = _small(7, n=20, d=8)
    Xv, yv, _, _ = _small(8, n=50, d=8)
    lam, h = 0.05, 1e-6
    a, _ = D.solve_linear(X, y, lam, m)
    ap, _ = D.solve_linear(X, y, lam + h, m, alpha0=a)
    am, _ = D.solve_linear(X, y, lam - h, m, alpha0=a)
    da = D.dalpha_dlambda(T.jacobian_closed(X, a, m), a, lam)
    np.testing.assert_allclose(da, (ap - am) / (2 * h), rtol=1e-5, atol=1e-6 * np.abs(da).max())
    dm = D.dmse_dlambda_linear(X, a, lam, m, Xv, yv)
    fd = (D.val_mse_linear(X, ap, m, Xv, yv) - D.val_mse_linear(X, am, m, Xv, yv)) / (2 * h)
    assert dm == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_lambda_path_warm_starts_do_not_change_answers():
    X, y, _, _ = _small(9, n=16, d=6)
    lams = np.array([1.0, 1e-2, 1e-1])
    path, infos = D.solve_path(X, y, lams, 4)
    for k, lam in enumerate(lams):
        a, _ = D.solve_linear(X, y, lam, 4)
        np.testing.assert_allclose(path[k], a, rtol=1e-9, atol=1e-12)


def test_bf16_rounding_pins():
    """Round-to-nearest-even to 8 significant bits, checked on exact cases."""
    r = P.round_bf16_scalar
    assert r(1.0) == 1.0
    assert r(1.0 + 2 ** -8) == 1.0                 # tie -> even (1.0000000)
    assert r(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie -> even (1.0000010)
    assert r(1.0 + 2 ** -8 + 2 ** -30) == 1.0 + 2 ** -7
    assert r(-(1.0 + 2 ** -7)) == -(1.0 + 2 ** -7)
    assert r(3.0 * 2 ** 100) == 3.0 * 2 ** 100
    assert r(2.0 ** 128) == np.inf
    assert r((2 - 2 ** -8) * 2.0 ** 127) == np.inf          # rounds up past the largest
    assert r((2 - 2 ** -7) * 2.0 ** 127) == (2 - 2 ** -7) * 2.0 ** 127
    assert r(2.0 ** -133) == 2.0 ** -133                  # smallest subnormal
    assert r(2.0 ** -134) == 0.0                          # tie to even zero
    rng = np.random.default_rng(0)
    x = rng.standard_normal(2000) * 10.0 ** rng.integers(-5, 5, 2000)
    y = P.round_bf16(x)
    # result has 8 significant bits and is within half a unit in the last place
    f, e = np.frexp(y)
    assert np.all(f * 256 == np.round(f * 256))
    assert np.all(np.abs(y - x) <= 2.0 ** (e - 9) + 0.0)
    # the vectorised form follows the scalar definition exactly, including ties,
    # subnormals and overflow
    z = np.concatenate([x, [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 2.0 ** -134, 2.0 ** -133, 3 * 2.0 ** -135,
                            (2 - 2 ** -8) * 2.0 ** 127, -0.0, 0.0, np.inf, -np.inf]])
    np.testing.assert_array_equal(P.round_bf16(z), np.array([P.round_bf16_scalar(v) for v in z]))


def test_fp32_rounding_pins():
    """Round-to-nearest-even to FP32 (24 significant bits, exponent range
    [-126, 127], subnormal quantum 2^-149), checked on cases whose answer
    follows from that definition alone: exact ties, values just off a tie,
    the subnormal range and the overflow threshold."""
    r = lambda v: float(P.round_fp32(np.array([v]))[0])
    assert r(1.0) == 1.0
    assert r(1.0 + 2 ** -24) == 1.0                          # tie -> even significand
    assert r(1.0 + 3 * 2 ** -24) == 1.0 + 2 ** -22           # tie -> even (...10)
    assert r(1.0 + 2 ** -24 + 2 ** -40) == 1.0 + 2 ** -23    # just above the tie
    assert r(-(1.0 + 2 ** -23)) == -(1.0 + 2 ** -23)         # representable, sign kept
    assert r(3.0 * 2 ** 100) == 3.0 * 2 ** 100
    assert r(2.0 ** -149) == 2.0 ** -149                     # smallest subnormal
    assert r(2.0 ** -150) == 0.0                             # tie between 0 and 2^-149 -> 0
    assert r(3 * 2.0 ** -150) == 2.0 ** -148                 # tie between 1 and 2 quanta -> 2
    assert r(2.0 ** -150 + 2.0 ** -160) == 2.0 ** -149       # just above the tie
    assert r(5 * 2.0 ** -151) == 2.0 ** -149                 # 1.25 quanta -> 1
    assert r(2.0 ** -126) == 2.0 ** -126                     # smallest normal
    big = (2 - 2 ** -23) * 2.0 ** 127                        # largest finite FP32
    assert r(big) == big
    assert r((2 - 2 ** -24) * 2.0 ** 127) == np.inf          # tie above the largest -> 2^128
    assert r((2 - 2 ** -23 + 2 ** -30) * 2.0 ** 127) == big  # below that tie
    assert r(-0.0) == 0.0 and np.signbit(P.round_fp32(np.array([-0.0]))[0])
    rng = np.random.default_rng(1)
    x = rng.standard_normal(2000) * 10.0 ** rng.integers(-30, 30, 2000)
    y = P.round_fp32(x)
    f, e = np.frexp(y)
    assert np.all(f * 2 ** 24 == np.round(f * 2 ** 24))      # 24 significant bits
    assert np.all(np.abs(y - x) <= 2.0 ** (e - 25))          # within half a unit in the last place


def test_exact_gradient_and_refinement():
    """The exact-arithmetic gradient agrees with the FP64 closed form where no
    cancellation occurs (alpha far from the optimum), and after refinement the
    exact gradient at the dual optimum is at rounding level of its terms."""
    rng = np.random.default_rng(31)
    n, d, m, lam = 24, 8, 4, 0.1
    X = rng.integers(-40, 41, size=(n, d)) / 16.0
    y = rng.standard_normal(n)
    a_far = rng.standard_normal(n)
    g_plain = X @ ((X.T @ a_far) ** (m - 1)) + lam * a_far - y
    g_exact = D.dual_grad_exact_linear(X, y, lam, m, a_far)
    np.testing.assert_allclose(g_exact, g_plain, rtol=1e-12, atol=1e-12 * np.abs(g_plain).max())
    a0, _ = D.solve_linear(X, y, lam, m)
    a1 = D.refine_linear_exact(X, y, lam, m, a0)
    u = X.T @ a1
    terms = np.abs(X) @ (np.abs(u) ** (m - 1)) + lam * np.abs(a1) + np.abs(y)
    g1 = D.dual_grad_exact_linear(X, y, lam, m, a1)
    assert np.abs(g1).max() <= 64 * np.finfo(float).eps * terms.max()
    # the refinement moves the FP64 solution by no more than the FP64 solver's accuracy
    assert np.linalg.norm(a1 - a0) <= 1e-8 * np.linalg.norm(a0)


def test_extended_refinement_matches_exact():
    """The extended-precision refinement reaches the exact-arithmetic
    refinement's optimum on an exactly representable problem, and cuts the
    exact gradient of a small-lambda FP64 solve."""
    assert np.finfo(np.longdouble).nmant >= 63
    rng = np.random.default_rng(32)
    n, d, m = 24, 8, 4
    X = rng.integers(-40, 41, size=(n, d)) / 16.0
    y = rng.standard_normal(n)
    for lam in (0.1, 1e-3):
        a0, _ = D.solve_linear(X, y, lam, m)
        a_ext = D.refine_linear(X, y, lam, m, a0)
        a_ex = D.refine_linear_exact(X, y, lam, m, a0)
        assert np.linalg.norm(a_ext - a_ex) <= 1e-11 * np.linalg.norm(a_ex)
        g0 = np.abs(D.dual_grad_exact_linear(X, y, lam, m, a0)).max()
        g1 = np.abs(D.dual_grad_exact_linear(X, y, lam, m, a_ext)).max()
        assert g1 <= max(g0, 1e-300)
