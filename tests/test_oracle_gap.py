"""Pins of the GAP oracle (section "PACO GAP", equation (gap)): linear gap
costs reduce it to the textbook edit-distance recurrence (Wagner-Fischer),
affine gap costs to Gotoh's three-table recurrence, and on tiny grids it is
the cheapest of every path of diagonal steps and row/column jumps."""
import functools

import numpy as np
import pytest

import oracle

INF = oracle.INF


def symbols(s, m, n):
    return [oracle.gap_s(s, i, j) for i in range(m + 1) for j in range(n + 1)]


def s_table(s, m, n):
    t = np.zeros((m + 1, n + 1), np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            t[i, j] = oracle.gap_s(s, i, j)
    return t


def test_substitution_symbols():
    # s takes only the two costs, and equal symbols recur at the alphabet's rate
    s = (0, 5, 2, 11, 22)
    t = s_table(s, 60, 60)[1:, 1:]
    assert set(np.unique(t).tolist()) <= {0, 5}
    assert 0.15 < (t == 0).mean() < 0.35   # 4 symbols: about 1/4 equal


def wagner_fischer(m, n, g_row, g_col, S, d0):
    """Textbook edit distance with indel costs g_row (along a row) and
    g_col (along a column) and substitution table S."""
    E = np.zeros((m + 1, n + 1), np.int64)
    E[0, 0] = d0
    for j in range(1, n + 1):
        E[0, j] = E[0, j - 1] + g_row
    for i in range(1, m + 1):
        E[i, 0] = E[i - 1, 0] + g_col
        for j in range(1, n + 1):
            E[i, j] = min(E[i - 1, j - 1] + S[i, j], E[i, j - 1] + g_row, E[i - 1, j] + g_col)
    return E


def gotoh(m, n, ar, br, ac, bc, S, d0):
    """Gotoh's recurrence for affine gaps a + b k: Q ends in a row gap, P in
    a column gap."""
    D = np.full((m + 1, n + 1), 1 << 40, np.int64)
    P = np.full((m + 1, n + 1), 1 << 40, np.int64)
    Q = np.full((m + 1, n + 1), 1 << 40, np.int64)
    for i in range(m + 1):
        for j in range(n + 1):
            if i == 0 and j == 0:
                D[0, 0] = d0
                continue
            if j >= 1:
                Q[i, j] = min(D[i, j - 1] + ar + br, Q[i, j - 1] + br)
            if i >= 1:
                P[i, j] = min(D[i - 1, j] + ac + bc, P[i - 1, j] + bc)
            best = min(P[i, j], Q[i, j])
            if i >= 1 and j >= 1:
                best = min(best, D[i - 1, j - 1] + S[i, j])
            D[i, j] = best
    return np.minimum(D, INF)


@pytest.mark.parametrize("m,n,g_row,g_col,s", [(40, 57, 1, 1, (0, 1, 2, 3, 4)), (33, 20, 3, 2, (1, 4, 1, 9, 8)),
                                               (1, 30, 2, 5, (0, 1, 2, 0, 0)), (25, 1, 2, 5, (0, 7, 3, 5, 6))])
def test_linear_gaps_are_edit_distance(m, n, g_row, g_col, s):
    D = oracle.gap(m, n, ("affine", 0, g_row, 0), ("affine", 0, g_col, 0), s, d0=3)
    assert np.array_equal(D.astype(np.int64), wagner_fischer(m, n, g_row, g_col, s_table(s, m, n), 3))


@pytest.mark.parametrize("m,n,ar,br,ac,bc,s", [(30, 41, 5, 1, 3, 2, (0, 4, 2, 1, 2)), (17, 9, 0, 3, 7, 1, (2, 9, 1, 4, 4)),
                                                (24, 24, 11, 0, 11, 0, (0, 6, 3, 7, 8))])
def test_affine_gaps_are_gotoh(m, n, ar, br, ac, bc, s):
    D = oracle.gap(m, n, ("affine", ar, br, 0), ("affine", ac, bc, 0), s, d0=0)
    assert np.array_equal(D.astype(np.int64), gotoh(m, n, ar, br, ac, bc, s_table(s, m, n), 0))


def brute(m, n, wr, wc, S, d0):
    """Cheapest path to every cell over all step sequences, by plain
    enumeration of predecessors (no table reuse)."""
    @functools.lru_cache(maxsize=None)
    def paths_cost(i, j):
        # enumerate every path ending at (i, j) explicitly: returns the list
        # of all path costs
        if i == 0 and j == 0:
            return (d0,)
        out = []
        if i >= 1 and j >= 1:
            out += [c + S[i, j] for c in paths_cost(i - 1, j - 1)]
        for q in range(j):
            out += [c + wr(q, j) for c in paths_cost(i, q)]
        for p in range(i):
            out += [c + wc(p, i) for c in paths_cost(p, j)]
        return tuple(out)
    E = np.zeros((m + 1, n + 1), np.int64)
    for i in range(m + 1):
        for j in range(n + 1):
            E[i, j] = min(min(paths_cost(i, j)), INF)
    return E


@pytest.mark.parametrize("wrow,wcol,s", [(("hash", 0, 8, 1), ("hash", 3, 6, 2), (0, 50, 2, 3, 4)),
                                         (("affine", 4, 2, 0), ("hash", 0, 9, 7), (5, 1, 1, 8, 9))])
def test_brute_force_every_path(wrow, wcol, s):
    m, n = 3, 4
    wr = lambda q, j: oracle.dp1d_w(wrow[0], wrow[1], wrow[2], wrow[3], q, j)
    wc = lambda p, i: oracle.dp1d_w(wcol[0], wcol[1], wcol[2], wcol[3], p, i)
    D = oracle.gap(m, n, wrow, wcol, s, d0=2)
    assert np.array_equal(D.astype(np.int64), brute(m, n, wr, wc, s_table(s, m, n), 2))


def test_first_row_and_column_are_1d_problems():
    # row 0 has no column or diagonal terms: it is the 1D problem with w
    m, n = 30, 200
    D = oracle.gap(m, n, ("hash", 1, 12, 4), ("hash", 0, 12, 6), (0, 3, 2, 1, 1), d0=5)
    assert np.array_equal(D[0], oracle.dp1d(n, "hash", 1, 12, 4, 5))
    assert np.array_equal(D[:, 0], oracle.dp1d(m, "hash", 0, 12, 6, 5))


def test_infinite_start_and_check():
    D = oracle.gap(20, 20, ("hash", 0, 8, 1), ("hash", 0, 8, 2), (0, 1, 2, 1, 2), d0=INF)
    assert (D == INF).all()
    wrow, wcol, s = ("hash", 0, 14, 3), ("affine", 2, 1, 0), (0, 4, 2, 5, 6)
    D = oracle.gap(60, 70, wrow, wcol, s)
    cells = [(i, j) for i in range(61) for j in range(71)]
    assert oracle.gap_check(D, cells, wrow, wcol, s) == 0
    bad = D.copy()
    bad[30, 40] += 1
    assert oracle.gap_check(bad, [(30, 40)], wrow, wcol, s) == 1
