"""CPU emulation of the GPU kernels' index arithmetic, with bounds checks.

Each function below restates, in Python, the offset expressions of one HIP
kernel (the same recurrences and clamps, not the definition), and the tests
check every offset against the packed layout of Section 5: live positions map
to the entry the kernel means to read, and every other position stays inside
the range the kernel's buffer descriptor (or row) allows.  Sizes cover one
64-column block, its edges and the maximum n of the FP64-MFMA batch pass:
n in {1, 63, 64, 65, 128, 129, 192, 193, 256}.  No GPU is used.
"""
from math import comb

import numpy as np
import pytest

from oracle import layout as L

NS = [1, 63, 64, 65, 128, 129, 192, 193, 256]
KFAR = 1 << 27


def unit_rel(n, k0):
    """rel[r, l]: offset of entry (r, l) of a unit from its entry (k0, k0),
    k0 <= r <= l < n, from the row lengths n - k (Section 5: within a unit the
    last two indices run as a triangle); -1 elsewhere."""
    rel = -np.ones((n, n), dtype=np.int64)
    start = 0
    for r in range(k0, n):
        rel[r, r:] = start + np.arange(n - r)
        start += n - r
    return rel


def unit_prefixes(n, qp):
    """Sorted prefixes P' of length qp in nested-loop order, with k0 = P'_last."""
    return list(L.nested_loop_tuples(n, qp))


# ---------------------------------------------------------------------------
# FP64-MFMA batch pass (tk_batch.hip): staging offsets of one (unit, row tile,
# chunk), from the table fl[l] = F(l) - l and the per-segment Rq/Dq/Tq/Cq.

def batch_stage_offsets(n, k0, t, c):
    """Offsets (entries from (k0, k0)) and the (row, column) of M each of the
    16 slots x 64 lanes reads, as the kernel computes them.  Returns
    (off, r, l, live) arrays of shape [16, 64]; off may be past the unit
    (then the load reads 0)."""
    F = lambda x: x * n - (x * (x - 1)) // 2   # noqa: E731
    fl = np.array([F(x) - x for x in range(256)], dtype=np.int64)
    Fk0 = F(k0)
    lane = np.arange(64)
    li, lk = lane & 15, lane >> 4
    ulo, ntile = k0 >> 4, (n + 15) >> 4
    off = np.full((16, 64), -(1 << 40), dtype=np.int64)
    rr = np.zeros((16, 64), dtype=np.int64)
    ll = np.zeros((16, 64), dtype=np.int64)
    used = np.zeros((16, 64), dtype=bool)
    for j in range(4):
        u = 4 * c + j
        if u < ulo or u >= ntile:
            continue
        for q in range(4):
            i = 4 * j + q
            if u >= t:
                a, b = 4 * q + lk, 16 * j + li
            else:
                a, b = li, 16 * j + 4 * q + lk
            r, l = 16 * t + a, 64 * c + b
            rr[i], ll[i], used[i] = r, l, True
            if u > t:
                rq_r = 16 * t + 4 * q + lk
                Rq = np.where((rq_r >= k0) & (rq_r < n), fl[rq_r] - Fk0, KFAR)
                cj = 16 * u + li + np.where(16 * u + li < n, 0, KFAR)
                off[i] = Rq + cj
            elif u == t:
                lr = 16 * t + li
                lo = np.minimum(rq := 16 * t + 4 * q + lk, lr)
                ok = (lo >= k0) & (rq < n) & (lr < n)
                flr, fll = fl[rq] - Fk0, fl[lr] - Fk0
                off[i] = np.where(ok, np.where(lr >= rq, flr + lr, fll + rq), KFAR)
            else:
                r_m = 16 * t + li
                Cq = np.where(r_m < n, r_m - Fk0, KFAR)
                lm = 16 * u + 4 * q + lk
                Tq = np.where(16 * ulo + 4 * q + lk < k0, KFAR, 0) if u == ulo else 0
                off[i] = fl[lm] + Cq + Tq
    lo = np.minimum(rr, ll)
    hi = np.maximum(rr, ll)
    live = used & (lo >= k0) & (hi < n)
    return off, lo, hi, live, used


@pytest.mark.parametrize("n", NS)
def test_batch_mfma_staging_offsets(n):
    """Every slot of every (unit start k0, row tile t >= k0/16, chunk) either
    reads entry (min, max) of the unit (live: inside the unit's triangle) or an
    offset past the unit's range (so its load reads 0); byte offsets stay
    below 2^32."""
    ntile = (n + 15) >> 4
    for k0 in range(n):
        rel = unit_rel(n, k0)
        nent = (n - k0) * (n - k0 + 1) // 2
        for t in range(k0 >> 4, ntile):
            for c in range((k0 >> 4) >> 2, ((ntile - 1) >> 2) + 1):
                off, lo, hi, live, used = batch_stage_offsets(n, k0, t, c)
                assert np.all(off[used] * 8 < 2 ** 32), (n, k0, t, c)
                if live.any():
                    want = rel[lo[live], hi[live]]
                    assert np.all(want >= 0)
                    np.testing.assert_array_equal(off[live], want, err_msg=f"n={n} k0={k0} t={t} c={c}")
                dead = used & ~live
                # dead slots must land outside [0, nent): past the end (or wrapped negative)
                od = off[dead]
                assert np.all((od >= nent) | (od < 0)), (n, k0, t, c, od[(od >= 0) & (od < nent)][:5])


def walk_units(n, qp, u_lo, u_hi):
    """The batch kernel's successor of a prefix (fixed indexing: the last
    index below n-1 goes up by one and the later ones take its value) and
    its offset update uoff += (n-k0)(n-k0+1)/2, from the rank of u_lo."""
    P = list(L.unrank(u_lo, n, qp))
    k0 = P[-1]
    uoff = L.rank_closed_form(P + [k0, k0], n)
    out = [(tuple(P), uoff)]
    for _ in range(u_lo + 1, u_hi):
        uoff += (n - k0) * (n - k0 + 1) // 2
        pos = 0
        for i in range(1, qp):
            if P[i] != n - 1:
                pos = i
        v = P[pos] + 1
        for i in range(qp):
            if i >= pos:
                P[i] = v
        k0 = P[-1]
        out.append((tuple(P), uoff))
    return out


@pytest.mark.parametrize("n,qp", [(1, 2), (63, 2), (64, 2), (65, 2), (129, 2), (256, 2), (9, 4), (17, 4), (7, 6)])
def test_batch_walk_matches_nested_loop_order(n, qp):
    """The unit walk (successor and offsets) visits the prefixes in nested-loop
    order with the packed offset of their (k0, k0) entry, from any start."""
    units = unit_prefixes(n, qp)
    U = len(units)
    starts = sorted({0, U // 3, U // 2, U - 1})
    for u_lo in starts:
        u_hi = min(U, u_lo + 400)
        got = walk_units(n, qp, u_lo, u_hi)
        for k, (P, uoff) in enumerate(got):
            assert P == units[u_lo + k]
            assert uoff == L.rank_closed_form(list(P) + [P[-1], P[-1]], n)


# ---------------------------------------------------------------------------
# Vector pass (tk_pass.hpp, batch_fast): buffer offsets of the rows of a unit.

def batch_rows_kb(nb, kb, long_units):
    """Rows loaded per batch (FP64/FP32 storage): about 16 loads; 16 rows in
    the last column block for order-4 units (long_units)."""
    segs = nb - kb
    r0 = 16 // segs
    return 16 if (long_units and segs == 1 and r0 >= 16) else 8 if r0 >= 8 else 4 if r0 >= 4 else 2


def pass_row_offsets(n, k0, rr, e_base_rel, long_units):
    """Byte offsets (entries, ES = 1) the fast row batches of one unit load, as
    batch_fast computes them: so = off - k - e_base + 64 KB per batch, plus
    lane and segment, minus the tail shift of lanes past n, and
    so += n - k - 1 - r from row to row (rows past the batch continue the
    recurrence).  Offsets are relative to the unit's (k0, k0) entry shifted by
    e_base_rel.  Yields (row, l, offset, live) arrays per batch."""
    nb = (n + 63) // 64
    lane = np.arange(64)
    # compensated mode: the first row of a run (rr > 1) goes through the
    # general path; the plain modes start the fast batches at k0 (as rr = 1)
    k = k0 + 1 if rr > 1 else k0
    off = 0 if k == k0 else n - k0   # packed offset of row k from (k0, k0)
    while k < n:
        kb = k >> 6
        rb = batch_rows_kb(nb, kb, long_units)
        blk_end = (kb + 1) * 64
        lim = min(blk_end, n)
        nrows = min(lim - k, rb)
        so = off - k - e_base_rel + kb * 64
        for r in range(rb):
            for j in range(nb - kb):
                l = (kb + j) * 64 + lane
                vtail = np.where(l < n, 0, n - 1 - l)
                o = so + lane + j * 64 + vtail
                yield k + r, l, o, r < nrows
            so += n - k - 1 - r
        off += nrows * (n - k) - nrows * (nrows - 1) // 2
        k += nrows


@pytest.mark.parametrize("long_units", [True, False])
@pytest.mark.parametrize("n", NS)
def test_vector_pass_row_offsets(n, long_units):
    """Live lanes (l >= row, l < n, rows of the batch) read entry (row, l);
    every lane of a row of the batch stays at or above the descriptor base,
    which lies 64 entries before the wave's first entry (here: this unit's).
    Rows past the batch (zero coefficients) may step below the base near the
    end of a unit: their offsets then wrap past the descriptor's range and
    read 0, in loads of their own, so they never zero a live row's quad."""
    rel_cache = {}
    for k0 in range(n):
        for rr in (1, 2):
            if rr == 2 and k0 == 0 and n == 1:
                continue
            rel = rel_cache.setdefault(k0, unit_rel(n, k0))
            for row, l, o, live_row in pass_row_offsets(n, k0, rr, -64, long_units):
                if live_row:
                    assert row < n and np.all(o >= 0), (n, k0, rr, row)
                    m = (l >= row) & (l < n)
                    if m.any():
                        np.testing.assert_array_equal(o[m] - 64, rel[row, l[m]], err_msg=f"n={n} k0={k0} row={row}")
                    # lanes past n re-read column n-1 of the same row
                    mt = l >= n
                    if mt.any():
                        assert np.all(o[mt] - 64 == rel[row, n - 1])


# ---------------------------------------------------------------------------
# Hessian unit vectors (tk_hess.hip, hess_unit_kernel): row offsets ro[r] of a
# batch of 8 rows and the clamped in-row index.

@pytest.mark.parametrize("n", NS)
def test_hessian_unit_row_offsets(n):
    """Each load K[ro[r] + ix] stays inside row kk[r] of the unit (ix in
    [0, n-1-kk]) and, for valid positions, is entry (k, l)."""
    lane = np.arange(64)
    for d in range(n):
        rel = unit_rel(n, d)
        nent = (n - d) * (n - d + 1) // 2
        roff = 0
        for kb in range(d, n, 8):
            ro, kk = [], []
            o = roff
            for r in range(8):
                k = kb + r
                kk.append(k if k < n else n - 1)
                ro.append(o)
                if k < n - 1:
                    o += n - k
            roff = o
            for b in range((kb >> 6), (n + 63) // 64):
                l = 64 * b + lane
                for r in range(8):
                    pos = l - kk[r]
                    ix = np.where(pos < 0, 0, np.where(l < n, pos, n - 1 - kk[r]))
                    idx = ro[r] + ix
                    assert np.all((idx >= 0) & (idx < nent)), (n, d, kb, r)
                    assert np.all(ix <= n - 1 - kk[r])
                    k = kb + r
                    valid = (k < n) & (pos >= 0) & (l < n)
                    if valid.any():
                        np.testing.assert_array_equal(idx[valid], rel[k, l[valid]])


def test_unit_rel_matches_layout_rank():
    """The per-unit offsets used above agree with the packed layout's rank
    (closed form and by counting) for a few prefixes."""
    n = 9
    for P in [(0, 0), (2, 5), (8, 8)]:
        k0 = P[-1]
        rel = unit_rel(n, k0)
        base = L.rank_closed_form(list(P) + [k0, k0], n)
        for r in range(k0, n):
            for l in range(r, n):
                assert rel[r, l] == L.rank_closed_form(list(P) + [r, l], n) - base
                assert rel[r, l] == L.rank_by_counting(list(P) + [r, l], n) - base
    assert comb(n + 3, 4) == L.packed_count(n, 4)
