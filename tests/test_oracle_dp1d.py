"""Pins of the 1D-problem oracle (section "PACO 1D", equation (1D)):
published hash vectors, brute force over every chain on small n, closed
forms of the affine weights, saturation, and the sampled recurrence check."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

INF = oracle.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fmix32_published_vectors():
    with open(os.path.join(GOLDEN, "murmur3_fmix32.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        assert oracle.fmix32(c["seed"]) == int(c["hash"], 16)


def test_fmix32_is_a_bijection_on_a_block():
    # an invertible mix: 2^16 consecutive keys give 2^16 distinct values
    vals = {oracle.fmix32(x) for x in range(0x12340000, 0x12350000)}
    assert len(vals) == 1 << 16


def test_hash_weights_range_and_spread():
    a, b = 100, 12
    w = np.array([oracle.dp1d_w("hash", a, b, 5, i, j) for i in range(64) for j in range(i + 1, 64)])
    assert w.min() >= a and w.max() < a + (1 << b)
    # uniform on 2^12 values: mean near the middle, many distinct values
    assert abs(w.mean() - (a + (1 << b) / 2)) < 0.1 * (1 << b)
    assert len(set(w.tolist())) > 1500


def brute(n, wfun, d0):
    """min over all chains 0 = i0 < i1 < ... < it = j of d0 + sum w, by
    enumerating every subset of intermediate points."""
    out = [d0]
    for j in range(1, n + 1):
        best = INF
        for r in range(0, j):
            for mid in itertools.combinations(range(1, j), r):
                pts = (0,) + mid + (j,)
                s = d0 + sum(wfun(pts[t], pts[t + 1]) for t in range(len(pts) - 1))
                best = min(best, s)
        out.append(min(best, INF))
    return np.array(out, np.int64)


@pytest.mark.parametrize("kind,a,b,seed,d0", [
    ("hash", 0, 10, 3, 0), ("hash", 50, 8, 11, 7), ("hash", 0, 20, 0, 1000),
    ("affine", 4, 3, 0, 2), ("affine", 0, 5, 0, 0)])
def test_brute_force_every_chain(kind, a, b, seed, d0):
    n = 9
    wfun = lambda i, j: oracle.dp1d_w(kind, a, b, seed, i, j)
    D = oracle.dp1d(n, kind, a, b, seed, d0)
    assert np.array_equal(D.astype(np.int64), brute(n, wfun, d0))


def test_affine_closed_forms():
    # a > 0: one jump is cheapest, D[j] = d0 + a + b j; a = 0: every chain
    # costs d0 + b j
    n = 3000
    j = np.arange(n + 1, dtype=np.int64)
    D = oracle.dp1d(n, "affine", 17, 3, 0, 9)
    exp = np.minimum(9 + 17 + 3 * j, INF)
    exp[0] = 9
    assert np.array_equal(D.astype(np.int64), exp)
    D = oracle.dp1d(n, "affine", 0, 5, 0, 4)
    assert np.array_equal(D.astype(np.int64), 4 + 5 * j)


def test_affine_saturates_at_inf():
    # w reaches INF beyond j = 2^20 / 1024: every later D is INF
    n = 3000
    D = oracle.dp1d(n, "affine", 0, 1 << 20, 0, 0)
    j = np.arange(n + 1, dtype=np.int64)
    assert np.array_equal(D.astype(np.int64), np.minimum(j << 20, INF))


def test_infinite_start_stays_infinite():
    D = oracle.dp1d(500, "hash", 0, 16, 1, INF)
    assert (D == INF).all()


def test_constant_weights():
    # b = 0 bits: w = a everywhere, D[j] = d0 + a
    D = oracle.dp1d(200, "hash", 42, 0, 9, 1)
    assert D[0] == 1 and (D[1:] == 43).all()


def test_recurrence_check_accepts_and_rejects():
    n = 4000
    D = oracle.dp1d(n, "hash", 0, 18, 2, 0)
    js = np.arange(1, n + 1)
    assert oracle.dp1d_check(D, js, "hash", 0, 18, 2) == 0
    bad = D.copy()
    bad[1234] += 1
    assert oracle.dp1d_check(bad, [1234], "hash", 0, 18, 2) == 1
    bad = D.copy()
    bad[3999] -= 1   # below the minimum: no predecessor gives it
    assert oracle.dp1d_check(bad, [3999], "hash", 0, 18, 2) == 1
