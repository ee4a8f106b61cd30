"""Pins for the oracle's packed layout (Section 5) against numbers the paper
prints and against independent enumerations."""
from math import comb

import numpy as np
import pytest

from conftest import read_golden
from oracle import layout as L
from oracle import tensor as T


def test_table_t_size_counts_and_percentages():
    rows = read_golden("t_size.txt")
    assert len(rows) == 6
    for r in rows:
        n = int(r[0])
        vals = [int(x) if "." not in x else float(x) for x in r[1:]]
        full2, b2, pct2, full3, b3, pct3, full4, b4, pct4 = vals
        assert (n ** 2, n ** 3, n ** 4) == (full2, full3, full4)
        assert L.packed_count(n, 2) == b2
        assert L.packed_count(n, 3) == b3
        assert L.packed_count(n, 4) == b4
        for full, b, pct in ((full2, b2, pct2), (full3, b3, pct3), (full4, b4, pct4)):
            assert round(100.0 * (full - b) / full, 2) == pytest.approx(pct, abs=1e-9)


def test_memory_gain_section_5_1():
    gib = 2.0 ** 30
    rows = read_golden("memory_gain.txt")
    for r in rows:
        if r[0] == "fit8":
            full_n, packed_n = int(r[1]), int(r[2])
            cap = 8 * gib
            assert full_n ** 4 * 8 <= cap < (full_n + 1) ** 4 * 8
            assert L.packed_count(packed_n, 4) * 8 <= cap < L.packed_count(packed_n + 1, 4) * 8
        elif r[0] == "n10":
            assert 10 ** 4 == int(r[1]) and L.packed_count(10, 4) == int(r[2])
        elif r[0] == "n60":
            assert L.packed_count(60, 4) == int(r[1]) and 60 ** 4 == int(r[2])
        elif r[0] == "n200":
            assert 200 ** 4 == int(r[1])
            assert L.packed_count(200, 4) // 10 ** 6 == int(r[2])
            assert round(200 ** 4 * 8 / gib, 2) == float(r[3])
        else:
            n, full_gb, packed_gb, dec = int(r[0]), float(r[1]), float(r[2]), int(r[3])
            assert round(n ** 4 * 8 / gib, dec) == round(full_gb, dec)
            assert round(L.packed_count(n, 4) * 8 / gib, dec) == round(packed_gb, dec)


def test_worked_example_v2d():
    (n, r, c, full, skip, v), = [list(map(int, x)) for x in read_golden("index_2d_example.txt")]
    assert r * n + c == full
    assert L.skip2d(r) == skip
    assert L.v2d(r, c, n) == v
    # the printed map is the position in nested-loop order
    assert L.rank_closed_form((r, c), n) == v


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_nested_loop_order_equals_rank(n, m):
    tuples = list(L.nested_loop_tuples(n, m))
    assert len(tuples) == L.packed_count(n, m) == comb(n + m - 1, m)
    assert tuples == list(L.all_sorted_tuples(n, m))
    for e, t in enumerate(tuples):
        assert L.rank_by_counting(t, n) == e
        assert L.rank_closed_form(t, n) == e
        assert L.unrank(e, n, m) == t


@pytest.mark.parametrize("n,m", [(7, 4), (5, 6), (9, 2), (4, 3)])
def test_c_oracle_enumeration_matches(n, m):
    Tc = T.enumerate_tuples(n, m)
    assert [tuple(x) for x in Tc.tolist()] == list(L.nested_loop_tuples(n, m))


def test_rank_spot_checks_large():
    rng = np.random.default_rng(7)
    for n, m in ((256, 4), (128, 6), (200, 4)):
        cnt = L.packed_count(n, m)
        for e in rng.integers(0, cnt, size=200).tolist() + [0, cnt - 1]:
            t = L.unrank(e, n, m)
            assert list(t) == sorted(t)
            assert L.rank_closed_form(t, n) == e
    assert L.packed_count(128, 6) == 6856577728 > 2 ** 32


@pytest.mark.parametrize("n", [3, 4, 5, 9])
def test_paper_v3d_v4d_readings(n):
    """eq. v3d / skip_3d and eq. v4d / skip_4d / skip_3d_inv as printed are
    the nested-loop positions up to one constant offset, once v4d's t*n^4 is
    read as t*n^3 (the layer index is the smallest of the tuple)."""
    t3 = L.skip3d_table(n)
    off3 = L.v3d_paper(0, 0, 0, n, t3)
    assert off3 == -L.skip2d(n - 1)
    for (d, r, c) in L.nested_loop_tuples(n, 3):
        assert L.v3d_paper(r, c, d, n, t3) - off3 == L.rank_closed_form((d, r, c), n)
    t4 = L.skip4d_table(n)
    off4 = L.v4d_read(0, 0, 0, 0, n, t3, t4)
    for (t, d, r, c) in L.nested_loop_tuples(n, 4):
        assert L.v4d_read(r, c, d, t, n, t3, t4) - off4 == L.rank_closed_form((t, d, r, c), n)
