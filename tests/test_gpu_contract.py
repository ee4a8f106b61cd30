"""GPU parity of the packed build, contraction and directional derivative
against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2003_10482_amd as tk
from gpu_util import U32, U64, UBF16, abs_terms, device, to_dev, to_np
from oracle import dual as D
from oracle import layout as L
from oracle import precision as P
from oracle import tensor as T
from synth import make_workload, random_alpha, random_symmetric_packed_values

pytestmark = pytest.mark.gpu

SHAPES = [(1, 4), (3, 2), (9, 2), (7, 4), (20, 4), (70, 4), (130, 4), (5, 6), (12, 6), (40, 6), (66, 6)]


def _packed_dev(Kh, n, m, dtype="f64"):
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    if dtype == "bf16":
        bits = P.round_bf16(Kh)
        t = tk.empty_packed(n, m, "bf16", device())
        t.copy_(torch.tensor(bits, dtype=torch.float64).to(torch.float32).to(torch.bfloat16))
        return tk.PackedTensor(t, n, m, tk.BF16), bits
    if dtype == "f32":
        r = P.round_fp32(Kh)
        return tk.PackedTensor(torch.tensor(r, dtype=torch.float32, device=device()), n, m, tk.F32), r
    return tk.PackedTensor(to_dev(Kh), n, m, tk.F64), Kh


def _dyadic_X(n, d, seed):
    # entries k/16: products and sums of up to 64 terms are exact in FP64, but
    # need more significant bits than FP32 or BF16 hold
    rng = np.random.default_rng(seed)
    return rng.integers(-40, 41, size=(n, d)) / 16.0


@pytest.mark.parametrize("n,m", [(12, 4), (70, 4), (9, 6), (66, 6), (30, 2), (150, 4)])
def test_build_exact_and_rounded(n, m):
    d = 16
    X = _dyadic_X(n, d, seed=n + m)
    Kref = T.build_packed(X, m)          # exact in FP64 for these inputs
    Xd = to_dev(X)
    K64 = tk.build_packed_tensor(Xd, m, dtype="f64")
    np.testing.assert_array_equal(to_np(K64.data), Kref)
    K32 = tk.build_packed_tensor(Xd, m, dtype="f32")
    np.testing.assert_array_equal(to_np(K32.data).astype(np.float64), P.round_fp32(Kref))
    Kb = tk.build_packed_tensor(Xd, m, dtype="bf16")
    np.testing.assert_array_equal(to_np(Kb.data.to(torch.float32)).astype(np.float64), P.round_bf16(Kref))


@pytest.mark.parametrize("n,m,d", [(250, 2, 37), (256, 2, 5), (70, 4, 37), (17, 6, 19)])
def test_build_column_tail_and_ragged_features(n, m, d):
    """Rows up to the full 256 columns with a ragged last 16-column block, and
    feature counts that end inside a staged chunk: exact on dyadic points."""
    X = _dyadic_X(n, d, seed=3 * n + m)
    Kref = T.build_packed(X, m)
    K64 = tk.build_packed_tensor(to_dev(X), m, dtype="f64")
    np.testing.assert_array_equal(to_np(K64.data), Kref)


@pytest.mark.parametrize("kernel,kparam", [("poly", 2), ("exp", 0.0)])
def test_build_poly_exp(kernel, kparam):
    n, d, m = 11, 6, 4
    X = 0.4 * np.random.default_rng(3).standard_normal((n, d))
    Kref = T.build_packed(X, m, kernel, kparam)
    K = tk.build_packed_tensor(to_dev(X), m, kernel=kernel, kparam=kparam)
    np.testing.assert_allclose(to_np(K.data), Kref, rtol=1e-13, atol=1e-15)


def test_build_sampled_entries_config2():
    """Full-size build (n=256, d=200, m=4): sampled entries, each recomputed
    alone by the oracle, and the entry count."""
    wl = make_workload("c2_n256_m4")
    K = tk.build_packed_tensor(to_dev(wl.X), 4)
    assert K.data.numel() == L.packed_count(256, 4) == 183181376
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.integers(0, K.data.numel(), 300), [0, K.data.numel() - 1]])
    got = to_np(K.data[torch.as_tensor(idx, device=device())])
    for e, v in zip(idx.tolist(), got.tolist()):
        t = L.unrank(e, 256, 4)
        ref = T.kernel_entry(wl.X, t)
        bound = 4 * 200 * U64 * T.kernel_entry(np.abs(wl.X), t)
        assert abs(v - ref) <= bound + 1e-300


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("acc", [tk.ACC_COMPENSATED, tk.ACC_F64])
def test_contract_f64_random_tensor(n, m, acc):
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=10 * n + m)
    B = 3 if L.packed_count(n, m) < 10 ** 6 else 1
    A = random_alpha(n, seed=n + 100 * m, batch=B)
    Kd, _ = _packed_dev(K, n, m)
    g = to_np(tk.contract(Kd, to_dev(A), acc=acc))
    for b in range(B):
        ref = T.contract_packed(K, n, m, A[b])
        E = abs_terms(K, n, m, A[b])
        # both sides are sums of the same terms; each errs by at most its depth x u x E
        depth = L.packed_count(n, m - 1) + 4 * n + 64
        assert np.all(np.abs(g[b] - ref) <= 2 * depth * U64 * E + 1e-300), (n, m, b)
        np.testing.assert_allclose(g[b], ref, rtol=1e-10, atol=1e-12 * E.max())


@pytest.mark.parametrize("n,m", [(20, 4), (70, 4), (200, 4), (12, 6), (40, 6)])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_contract_reduced_precision(n, m, storage):
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=7 * n + m)
    B = 5 if L.packed_count(n, m) < 10 ** 7 else 2
    A = random_alpha(n, seed=3 * n + m, batch=B)
    Kd, Kr = _packed_dev(K, n, m, storage)
    g = to_np(tk.contract(Kd, to_dev(A)))
    us = U32 if storage == "f32" else UBF16
    for b in range(B):
        ref = T.contract_packed(K, n, m, A[b])
        E = abs_terms(K, n, m, A[b])
        # a-priori bound: storage rounding of K, FP32 rounding of alpha and of each
        # product (m+1 factors), and FP32 accumulation along chains of at most
        # (rows of the order m array + 4n + 64) additions
        depth = L.packed_count(n, m - 1) + 4 * n + 64
        bound = (us + (m + 2) * U32 + depth * U32) * E
        assert np.all(np.abs(g[b] - ref) <= bound), (n, m, storage, b)
        # typical error: the same result computed from the rounded tensor in FP64
        ref_r = T.contract_packed(Kr, n, m, A[b])
        assert np.max(np.abs(g[b] - ref_r) / E) <= 64 * U32 * np.sqrt(depth)


@pytest.mark.parametrize("n,m", [(129, 4), (200, 4), (256, 2), (150, 2)])
@pytest.mark.parametrize("storage", ["f32", "bf16", "f64-f32"])
def test_reduced_precision_relative(n, m, storage):
    """FP32 accumulation against the FP64 contraction of the same stored values,
    relative to max |g| (the absolute-term bound of the test above is loose
    enough to hide lost entries).  Sizes cover 3 and 4 column blocks, tails and
    the first rows of many waves; one-hot directions probe single entries."""
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=11 * n + m)
    kind = "f64" if storage == "f64-f32" else storage
    Kd, Kr = _packed_dev(K, n, m, kind)
    acc = tk.ACC_F32 if storage == "f64-f32" else tk.ACC_AUTO
    nb = 5 if m == 2 else 2
    A = random_alpha(n, seed=5 * n + m, batch=nb)
    g = to_np(tk.contract(Kd, to_dev(A), acc=acc))
    for b in range(nb):
        ref = T.contract_packed(Kr, n, m, A[b])
        assert np.max(np.abs(g[b] - ref)) <= 1e-4 * np.max(np.abs(ref)), (n, m, storage, b)
    # one-hot directions: h = J e_c, column c of the Jacobian
    cols = [0, 3, 64, 67, 70, 127, n // 2 + 1, n - 2, n - 1] if m == 2 else [67, n - 1]
    V = np.zeros((len(cols), n))
    for i, c in enumerate(cols):
        V[i, c] = 1.0
    Ab = np.repeat(A[:1], len(cols), axis=0)
    h = to_np(tk.hvp(Kd, to_dev(Ab), to_dev(V), acc=acc))
    for i in range(len(cols)):
        ref = T.hvp_packed(Kr, n, m, Ab[i], V[i])
        assert np.max(np.abs(h[i] - ref)) <= 1e-4 * np.max(np.abs(ref)), (n, m, storage, cols[i])


@pytest.mark.parametrize("acc", ["f64", "f32"])
@pytest.mark.parametrize("hv", [False, True])
def test_autotuned_tiles(acc, hv):
    """The autotuner times the vector tiles (and, for plain FP64 contractions,
    the MFMA batch pass) and keeps one; the last candidate's results (left in
    the output by the tuner) and the tuned call both match the oracle (plain
    FP64 / FP32 accumulation bounds)."""
    n, m, B = 70, 4, 6
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=91 + int(hv))
    A = random_alpha(n, seed=92, batch=B)
    V = random_alpha(n, seed=93, batch=B)
    if acc == "f64":
        Kd, Kr = _packed_dev(K, n, m, "f64")
        a = tk.ACC_F64
    else:
        Kd, Kr = _packed_dev(K, n, m, "f32")
        a = tk.ACC_AUTO
    tile, ms, out = tk.autotune(Kd, to_dev(A), to_dev(V) if hv else None, acc=a)
    # the FP64-MFMA batch pass (tile 16) is a candidate for plain FP64 contractions only
    assert tile in ms and set(ms) == ({1, 2, 4, 16} if (acc == "f64" and not hv) else {1, 2} if hv and acc == "f64"
                                      else {1, 2, 4})
    got = to_np(tk.hvp(Kd, to_dev(A), to_dev(V), acc=a) if hv else tk.contract(Kd, to_dev(A), acc=a))
    for res in (to_np(out), got):
        for b in range(B):
            ref = (T.hvp_packed(Kr, n, m, A[b], V[b]) if hv else T.contract_packed(Kr, n, m, A[b]))
            tol = 1e-12 if acc == "f64" else 1e-4
            assert np.max(np.abs(res[b] - ref)) <= tol * np.max(np.abs(ref)), (acc, hv, tile, b)


@pytest.mark.parametrize("n", [200, 256])
def test_full_size_fp64_passes_element_by_element(n):
    """The FP64 passes of the benchmark shape (m = 4, n in (192, 256]: the
    fourth 64-column block present) against the oracle, element by element, on
    a random symmetric tensor: the plain and compensated contraction (one
    vector, and a tile of 4 through the autotuner, whose returned results come
    from the largest tile it times), and the plain directional derivative in
    the solver's line-search form (alpha := the Newton direction x, v := the
    iterate, with g), one vector and a tile of 2."""
    m = 4
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=n + 5)
    X4 = random_alpha(n, seed=n + 6, batch=4)
    Kd, _ = _packed_dev(K, n, m)
    x, a = X4[0], X4[1]
    ref = [T.contract_packed(K, n, m, X4[b]) for b in range(4)]
    E = [abs_terms(K, n, m, X4[b]) for b in range(4)]
    depth = L.packed_count(n, m - 1) + 4 * n + 64
    for acc in (tk.ACC_F64, tk.ACC_COMPENSATED):
        g = to_np(tk.contract(Kd, to_dev(x), acc=acc))
        assert np.all(np.abs(g - ref[0]) <= 2 * depth * U64 * E[0]), acc
        np.testing.assert_allclose(g, ref[0], rtol=1e-10, atol=1e-12 * E[0].max())
    tile, _, out = tk.autotune(Kd, to_dev(X4), acc=tk.ACC_F64)
    out = to_np(out)
    for b in range(4):
        assert np.all(np.abs(out[b] - ref[b]) <= 2 * depth * U64 * E[b]), b
    # line-search form: h = 3 K x^2 a, g = K x^3
    h, g = tk.hvp(Kd, to_dev(x), to_dev(a), with_g=True, acc=tk.ACC_F64)
    h, g = to_np(h), to_np(g)
    ref_h = T.hvp_packed(K, n, m, x, a)
    Eh = T.hvp_packed(np.abs(K), n, m, np.abs(x), np.abs(a))
    assert np.all(np.abs(h - ref_h) <= 2 * depth * U64 * Eh)
    assert np.all(np.abs(g - ref[0]) <= 2 * depth * U64 * E[0])
    np.testing.assert_allclose(h, ref_h, rtol=1e-9, atol=1e-11 * Eh.max())
    V2 = np.stack([a, X4[2]])
    _, _, out = tk.autotune(Kd, to_dev(X4[:2]), to_dev(V2), acc=tk.ACC_F64)
    out = to_np(out)
    ref_h1 = T.hvp_packed(K, n, m, X4[1], X4[2])
    Eh1 = T.hvp_packed(np.abs(K), n, m, np.abs(X4[1]), np.abs(X4[2]))
    assert np.all(np.abs(out[0] - ref_h) <= 2 * depth * U64 * Eh)
    assert np.all(np.abs(out[1] - ref_h1) <= 2 * depth * U64 * Eh1)


@pytest.mark.parametrize("n,m", [(7, 4), (70, 4), (130, 4), (5, 6), (40, 6), (66, 6), (9, 2)])
def test_hvp_f64_random_tensor(n, m):
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=n * m + 1)
    B = 2
    A = random_alpha(n, seed=n + 1, batch=B)
    V = random_alpha(n, seed=n + 2, batch=B)
    Kd, _ = _packed_dev(K, n, m)
    h, g = tk.hvp(Kd, to_dev(A), to_dev(V), with_g=True)
    h, g = to_np(h), to_np(g)
    for b in range(B):
        ref_h = T.hvp_packed(K, n, m, A[b], V[b])
        ref_g = T.contract_packed(K, n, m, A[b])
        Eh = T.hvp_packed(np.abs(K), n, m, np.abs(A[b]), np.abs(V[b]))
        np.testing.assert_allclose(h[b], ref_h, rtol=1e-9, atol=1e-11 * Eh.max())
        np.testing.assert_allclose(g[b], ref_g, rtol=1e-9, atol=1e-11 * abs_terms(K, n, m, A[b]).max())


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_hvp_reduced_precision(storage):
    n, m = 70, 4
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=5)
    A = random_alpha(n, seed=6, batch=5)
    V = random_alpha(n, seed=7, batch=5)
    Kd, Kr = _packed_dev(K, n, m, storage)
    h = to_np(tk.hvp(Kd, to_dev(A), to_dev(V)))
    for b in range(5):
        ref = T.hvp_packed(Kr, n, m, A[b], V[b])
        Eh = T.hvp_packed(np.abs(K), n, m, np.abs(A[b]), np.abs(V[b]))
        assert np.max(np.abs(h[b] - ref) / Eh.max()) <= 1e-4


def _exact_closed_form(X, a, m):
    """g = X (X^T a)^{m-1} in exact rational arithmetic (eq. tensor_1)."""
    from fractions import Fraction
    Xf = [[Fraction(v) for v in row] for row in X.tolist()]
    af = [Fraction(v) for v in a.tolist()]
    n, d = len(Xf), len(Xf[0])
    u = [sum(Xf[i][j] * af[i] for i in range(n)) for j in range(d)]
    w = [uj ** (m - 1) for uj in u]
    return np.array([float(sum(Xf[i][j] * w[j] for j in range(d))) for i in range(n)])


def test_contract_compensated_at_dual_optimum():
    """Near the dual optimum the packed sum cancels by ~9 orders of magnitude.
    With dyadic points the packed FP64 tensor is exact, so the compensated FP64
    contraction must match the exact value of X (X^T alpha)^{m-1} (rational
    arithmetic) to about one rounding of g, while a plain FP64 sum of the same
    terms does not."""
    from synth import planted_regression
    n, d, m = 64, 20, 4
    X = _dyadic_X(n, d, seed=11)
    rng = np.random.default_rng(12)
    _, y, _, _ = planted_regression(rng, n, d, 4, 0.01)
    y = X @ np.where(np.arange(d) < 4, 1.0, 0.0) + 0.01 * y
    a, _ = D.solve_linear(X, y, 1e-2, m)
    exact = _exact_closed_form(X, a, m)
    K = tk.build_packed_tensor(to_dev(X), m)
    assert np.array_equal(to_np(K.data), T.build_packed(X, m))     # the stored tensor is exact
    g = to_np(tk.contract(K, to_dev(a)))
    E = abs_terms(T.build_packed(X, m), n, m, a)
    assert E.max() / np.abs(exact).max() > 1e5                        # heavy cancellation indeed
    assert np.max(np.abs(g - exact)) <= 4 * U64 * np.max(np.abs(exact)) + 64 * U64 ** 2 * E.max()
    g_plain = to_np(tk.contract(K, to_dev(a), acc=tk.ACC_F64))
    assert np.max(np.abs(g_plain - exact)) > 1e3 * np.max(np.abs(g - exact))


def test_contract_deterministic():
    n, m = 130, 4
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=1)
    Kd, _ = _packed_dev(K, n, m)
    a = to_dev(random_alpha(n, seed=2, batch=2))
    g1 = tk.contract(Kd, a)
    g2 = tk.contract(Kd, a)
    assert torch.equal(g1, g2)


def test_dense_shortcut_matches_closed_form():
    wl = make_workload("c2_n256_m4")
    A = random_alpha(256, seed=9, batch=3)
    g = to_np(tk.contract_dense(to_dev(wl.X), to_dev(A), 4))
    for b in range(3):
        ref = T.contract_closed(wl.X, A[b], 4)
        np.testing.assert_allclose(g[b], ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("storage,acc,B", [("f32", tk.ACC_AUTO, 2), ("f32", tk.ACC_AUTO, 1), ("bf16", tk.ACC_AUTO, 2),
                                           ("f64", tk.ACC_COMPENSATED, 1), ("f64", tk.ACC_F64, 2),
                                           ("f64", tk.ACC_F32, 2)])
@pytest.mark.parametrize("n,m", [(129, 4), (200, 4), (40, 6)])
def test_workspace_contents_do_not_matter(n, m, storage, acc, B):
    """Every workspace entry a pass reads is written first: a NaN-filled
    workspace gives the same (finite) result as a zero-filled one."""
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=3 * n + m)
    Kd, _ = _packed_dev(K, n, m, storage)
    A = to_dev(random_alpha(n, seed=n + B, batch=B))
    nbytes = tk.contract_workspace(n, m, B, Kd.dtype)
    outs = []
    for fill in (0.0, float("nan")):
        work = torch.full(((nbytes + 7) // 8,), fill, dtype=torch.float64, device=device()).view(torch.uint8)
        outs.append(to_np(tk.contract(Kd, A, acc=acc, work=work)))
    assert np.all(np.isfinite(outs[1])), np.flatnonzero(~np.isfinite(outs[1]).all(axis=0))
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,m", [(129, 4), (150, 4), (192, 4), (70, 4), (256, 2), (140, 2)])
def test_memory_past_the_tensor_is_not_read(n, m, storage):
    """NaN in the memory that follows the packed array (beyond the half dword
    a BF16 array shares with its last entry) changes no result: columns past
    n, in whichever column block they fall, never reach past the array
    (n in (128, 192] runs the four-block kernels with a partial third block)."""
    count = L.packed_count(n, m)
    K = random_symmetric_packed_values(count, seed=7 * n + m)
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[storage]
    code = {"f64": tk.F64, "f32": tk.F32, "bf16": tk.BF16}[storage]
    vals = torch.as_tensor(K, device=device()).to(dt)
    A = to_dev(random_alpha(n, seed=n, batch=2))
    V = to_dev(random_alpha(n, seed=n + 1, batch=2))
    res = []
    for fill in (0.0, float("nan")):
        buf = torch.full((count + 4096,), fill, dtype=dt, device=device())
        buf[:count + (count & 1)] = 0
        buf[:count] = vals
        Kd = tk.PackedTensor(buf[:count], n, m, code)
        res.append([to_np(tk.contract(Kd, A)), to_np(tk.hvp(Kd, A, V))])
    for a, b in zip(res[0], res[1]):
        assert np.all(np.isfinite(b))
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("n,m", [(70, 4), (13, 6), (30, 2)])
def test_empty_batch_and_zero_vector(n, m):
    """Degenerate inputs: an empty batch of vectors gives an empty result (no
    launch); alpha = 0 gives g = 0 and h = 0 exactly (every term of the sum
    has a factor alpha_i), for every accumulation mode."""
    Kh = random_symmetric_packed_values(tk.packed_count(n, m), seed=n + m)
    K, _ = _packed_dev(Kh, n, m)
    empty = torch.zeros(0, n, dtype=torch.float64, device=device())
    assert tuple(tk.contract(K, empty).shape) == (0, n)
    h, g = tk.hvp(K, empty, empty, with_g=True)
    assert tuple(h.shape) == (0, n) and tuple(g.shape) == (0, n)
    zero = torch.zeros(2, n, dtype=torch.float64, device=device())
    for acc in (tk.ACC_F64, tk.ACC_COMPENSATED):
        assert not to_np(tk.contract(K, zero, acc=acc)).any()
    v = to_dev(random_alpha(n, seed=4, batch=2))
    h = to_np(tk.hvp(K, zero, v, acc=tk.ACC_COMPENSATED))
    if m == 2:   # h = K v, independent of alpha
        assert np.all(np.isfinite(h))
    else:
        assert not h.any()


MFMA_SHAPES = [(1, 4), (7, 4), (15, 4), (16, 4), (17, 4), (63, 4), (64, 4), (65, 4), (70, 4), (129, 4),
               (5, 6), (12, 6), (40, 6), (6, 8), (14, 8)]


@pytest.mark.parametrize("n,m", MFMA_SHAPES)
@pytest.mark.parametrize("B", [16, 17, 40])
def test_mfma_batch_pass(n, m, B):
    """Plain FP64 contraction of a batch of 16 or more vectors (the first pass
    on the FP64 matrix cores, 16 vectors per tile, ragged last tile at 17 and
    40; n across the 16-row tiles and their ragged tails) against the oracle,
    element by element, within the same summation bound as the vector passes."""
    count = L.packed_count(n, m)
    K = random_symmetric_packed_values(count, seed=17 * n + m + B)
    A = random_alpha(n, seed=n + 1000 * m + B, batch=B)
    Kd, _ = _packed_dev(K, n, m)
    g = to_np(tk.contract(Kd, to_dev(A), acc=tk.ACC_F64))
    depth = L.packed_count(n, m - 1) + 4 * n + 64
    check = range(B) if count * B < 4 * 10 ** 7 else sorted({0, 15, min(16, B - 1), B - 1})
    for b in check:
        ref = T.contract_packed(K, n, m, A[b])
        E = abs_terms(K, n, m, A[b])
        assert np.all(np.abs(g[b] - ref) <= 2 * depth * U64 * E + 1e-300), (n, m, B, b)


def test_mfma_batch_full_size():
    """The benchmark shape (n = 256, m = 4, C(259,4) FP64 entries) with 64
    vectors through the MFMA batch pass: four sampled vectors (first and last
    of the first tile, first of the second, the last) against the oracle
    element by element; every vector against the same vector contracted alone
    (the vector pass)."""
    n, m, B = 256, 4, 64
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=611)
    A = random_alpha(n, seed=612, batch=B)
    Kd, _ = _packed_dev(K, n, m)
    g = to_np(tk.contract(Kd, to_dev(A), acc=tk.ACC_F64))
    depth = L.packed_count(n, m - 1) + 4 * n + 64
    for b in (0, 15, 16, 63):
        ref = T.contract_packed(K, n, m, A[b])
        E = abs_terms(K, n, m, A[b])
        assert np.all(np.abs(g[b] - ref) <= 2 * depth * U64 * E), b
    for b in range(B):
        one = to_np(tk.contract(Kd, to_dev(A[b]), acc=tk.ACC_F64))
        np.testing.assert_allclose(g[b], one, rtol=1e-9, atol=1e-11 * np.abs(one).max())


@pytest.mark.parametrize("n,m", [(129, 4), (150, 4), (192, 4), (193, 4), (70, 4), (40, 6)])
def test_mfma_batch_reads_nothing_past_the_tensor_or_unwritten_workspace(n, m):
    """NaN after the packed array, and NaN in the whole workspace, change no
    result of the MFMA batch pass (B = 17: a full and a one-vector tile)."""
    count = L.packed_count(n, m)
    K = random_symmetric_packed_values(count, seed=5 * n + m)
    A = to_dev(random_alpha(n, seed=n + 7, batch=17))
    nbytes = tk.contract_workspace(n, m, 17, tk.F64)
    res = []
    for fill in (0.0, float("nan")):
        buf = torch.full((count + 4096,), fill, dtype=torch.float64, device=device())
        buf[:count] = torch.as_tensor(K, device=device())
        Kd = tk.PackedTensor(buf[:count], n, m, tk.F64)
        work = torch.full(((nbytes + 7) // 8,), fill, dtype=torch.float64, device=device()).view(torch.uint8)
        res.append(to_np(tk.contract(Kd, A, acc=tk.ACC_F64, work=work)))
    assert np.all(np.isfinite(res[1]))
    np.testing.assert_array_equal(res[0], res[1])


def test_batch_reads_the_tensor_once_per_launch_by_the_library_count():
    """A plain FP64 contraction of 64 vectors runs its pass over K once (the
    FP64-MFMA batch pass): the library's own count of the pass's tensor bytes
    is C x 8 for the whole batch, and results match 64 separate calls."""
    n, m, B = 70, 4, 64
    count = L.packed_count(n, m)
    K = random_symmetric_packed_values(count, seed=4242)
    Kd, _ = _packed_dev(K, n, m)
    A = to_dev(random_alpha(n, seed=4243, batch=B))
    tk.contract(Kd, A, acc=tk.ACC_F64)   # plans and workspace
    torch.cuda.synchronize()
    tk.timing_start()
    g = tk.contract(Kd, A, acc=tk.ACC_F64)
    torch.cuda.synchronize()
    launches, _, nbytes = tk.timing_stop()["contract_plain"]
    assert launches == 1 and nbytes == count * 8
    g = to_np(g)
    for b in (0, 31, 32, 63):
        one = to_np(tk.contract(Kd, A[b], acc=tk.ACC_F64))
        np.testing.assert_allclose(g[b], one, rtol=1e-10, atol=1e-12 * np.abs(one).max())
