"""Pins for the CPU oracle: each check compares it with something other than
its own formula -- hand-worked fixtures, closed forms, identities, absorption,
reductions to integer matrix products done by numpy, associativity, and
Strassen against the classic product.  Non-square shapes throughout, so a
transposed operand or swapped index fails."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF, NEG_INF = oracle.INF, oracle.NEG_INF
SHAPES = [(1, 1, 1), (3, 5, 7), (7, 4, 2), (2, 9, 13), (17, 6, 33)]


def _rng(seed=0):
    return np.random.default_rng(seed)


def _ilog_floor(v, base):
    """Largest e with base**e <= v, v >= 1 (exact on Python ints)."""
    e = 0
    p = base
    while p <= v:
        p *= base
        e += 1
    return e


def _maxplus_by_powers(A, B):
    """max_l (a+b) for small non-negative ints via one integer matrix product:
    with X = k+1, sum_l X^(a+b) lies in [X^max, k X^max] < X^(max+1)."""
    n, k = A.shape
    X = k + 1
    P = np.vectorize(lambda v: X ** int(v), otypes=[object])(A)
    Q = np.vectorize(lambda v: X ** int(v), otypes=[object])(B)
    S = P.dot(Q)
    return np.vectorize(lambda v: _ilog_floor(v, X), otypes=[np.int64])(S)


# ----------------------------------------------------------------- (min,+)

def test_minplus_hand_worked_graph():
    g = json.load(open(os.path.join(GOLD, "tropical_graph.json")))
    W = np.array(g["W"], np.int32)
    D2 = oracle.minplus(W, W)
    np.testing.assert_array_equal(D2, np.array(g["D2"]))
    np.testing.assert_array_equal(oracle.minplus(D2, D2), np.array(g["D4"]))


@pytest.mark.parametrize("n,m,k", SHAPES)
def test_minplus_identity(n, m, k):
    A, B = workloads.minplus_operands(n, m, k, seed=3)
    In = np.full((k, k), INF, np.int32)
    np.fill_diagonal(In, 0)
    Im = np.full((n, n), INF, np.int32)
    np.fill_diagonal(Im, 0)
    np.testing.assert_array_equal(oracle.minplus(A, In), A)
    np.testing.assert_array_equal(oracle.minplus(Im, A), A)


def test_minplus_absorption():
    A, B = workloads.minplus_operands(9, 11, 13, seed=4)
    A[2, :] = INF
    B[:, 5] = INF
    C = oracle.minplus(A, B)
    assert (C[2, :] == INF).all() and (C[:, 5] == INF).all()


@pytest.mark.parametrize("n,m,k", SHAPES)
def test_minplus_zero_matrix_gives_row_minima(n, m, k):
    A, _ = workloads.minplus_operands(n, m, k, seed=5)
    C = oracle.minplus(A, np.zeros((k, m), np.int32))
    np.testing.assert_array_equal(C, np.repeat(A.min(axis=1, keepdims=True), m, axis=1))


def test_minplus_k1_is_saturated_outer_sum():
    a = np.array([[0], [5], [INF], [(1 << 30) - 1]], np.int32)
    b = np.array([[3, INF, (1 << 30) - 2, 0]], np.int32)
    C = oracle.minplus(a, b)
    expect = np.minimum(a.astype(np.int64) + b.astype(np.int64), INF)
    np.testing.assert_array_equal(C, expect)


def test_minplus_k0_is_empty_fold():
    C = oracle.minplus(np.zeros((3, 0), np.int32), np.zeros((0, 4), np.int32))
    assert (C == INF).all()


@pytest.mark.parametrize("n,m,k", SHAPES)
def test_minplus_zero_inf_matches_boolean_integer_product(n, m, k):
    r = _rng(n * 100 + k)
    A = np.where(r.random((n, k)) < 0.3, 0, INF).astype(np.int32)
    B = np.where(r.random((k, m)) < 0.3, 0, INF).astype(np.int32)
    hit = (A == 0).astype(np.int64) @ (B == 0).astype(np.int64) > 0
    np.testing.assert_array_equal(oracle.minplus(A, B), np.where(hit, 0, INF))


@pytest.mark.parametrize("n,m,k", SHAPES)
def test_minplus_matches_power_sum_reduction(n, m, k):
    r = _rng(7 + n + m + k)
    A = r.integers(0, 9, (n, k)).astype(np.int32)
    B = r.integers(0, 9, (k, m)).astype(np.int32)
    # min(a+b) = 16 - max((8-a)+(8-b))
    expect = 16 - _maxplus_by_powers(8 - A.astype(np.int64), 8 - B.astype(np.int64))
    np.testing.assert_array_equal(oracle.minplus(A, B), expect)


def test_minplus_associative_with_inf():
    A, B = workloads.minplus_operands(6, 7, 5, seed=8)
    _, D = workloads.minplus_operands(7, 4, 7, seed=9)
    lhs = oracle.minplus(oracle.minplus(A, B), D)
    rhs = oracle.minplus(A, oracle.minplus(B, D))
    np.testing.assert_array_equal(lhs, rhs)


def test_minplus_path_graph_powers():
    # unit-weight undirected path on 12 vertices: after s products of the
    # adjacency (0 diagonal), distance |i-j| is reached iff |i-j| <= s+1
    N = 12
    W = np.full((N, N), INF, np.int32)
    for i in range(N):
        W[i, i] = 0
        if i + 1 < N:
            W[i, i + 1] = W[i + 1, i] = 1
    D = W.copy()
    for s in range(1, 5):
        D = oracle.minplus(D, W)
        d = np.abs(np.subtract.outer(np.arange(N), np.arange(N)))
        np.testing.assert_array_equal(D, np.where(d <= s + 1, d, INF))


def test_minplus_accumulate():
    A, B = workloads.minplus_operands(5, 6, 7, seed=10)
    C0 = workloads.minplus_matrix(11, 0, (5, 6))
    np.testing.assert_array_equal(oracle.minplus(A, B, C0),
                                  np.minimum(C0, oracle.minplus(A, B)))


def test_minplus_saturation_at_domain_edge():
    A = np.full((2, 3), (1 << 30) - 1, np.int32)
    B = np.full((3, 2), (1 << 30) - 1, np.int32)
    assert (oracle.minplus(A, B) == INF).all()
    A[0, 1] = 0
    B[1, 0] = 5
    C = oracle.minplus(A, B)
    # C[0,1] = A[0,1] + B[1,1] = 0 + (2^30 - 1) stays finite
    assert C[0, 0] == 5 and C[0, 1] == (1 << 30) - 1 and (C[1] == INF).all()


# ----------------------------------------------------------------- (max,+)

@pytest.mark.parametrize("n,m,k", SHAPES)
def test_maxplus_identity(n, m, k):
    A, _ = workloads.maxplus_operands(n, m, k, seed=12)
    I = np.full((k, k), NEG_INF, np.int32)
    np.fill_diagonal(I, 0)
    np.testing.assert_array_equal(oracle.maxplus(A, I), A)


@pytest.mark.parametrize("n,m,k", SHAPES)
def test_maxplus_zero_matrix_gives_row_maxima(n, m, k):
    A, _ = workloads.maxplus_operands(n, m, k, seed=13)
    C = oracle.maxplus(A, np.zeros((k, m), np.int32))
    np.testing.assert_array_equal(C, np.repeat(A.max(axis=1, keepdims=True), m, axis=1))


@pytest.mark.parametrize("n,m,k", SHAPES)
def test_maxplus_matches_power_sum_reduction(n, m, k):
    r = _rng(99 + n * m)
    A = r.integers(0, 9, (n, k)).astype(np.int32)
    B = r.integers(0, 9, (k, m)).astype(np.int32)
    np.testing.assert_array_equal(oracle.maxplus(A, B), _maxplus_by_powers(A, B))
    # shifting the domain shifts the result: pins signed arithmetic
    np.testing.assert_array_equal(oracle.maxplus(A - 20000, B - 300),
                                  _maxplus_by_powers(A, B) - 20300)


def test_maxplus_neg_inf_absorbs():
    M = oracle.MAXPLUS_FINITE_MAX
    A = np.array([[NEG_INF, M], [3, NEG_INF]], np.int32)
    B = np.array([[M, 0], [NEG_INF, NEG_INF]], np.int32)
    # every product has a NEG_INF factor except A[1,0]*B[0,*]
    C = oracle.maxplus(A, B)
    np.testing.assert_array_equal(C, [[NEG_INF, NEG_INF], [3 + M, 3]])


def test_maxplus_associative():
    A, B = workloads.maxplus_operands(5, 6, 4, seed=14)
    _, D = workloads.maxplus_operands(6, 3, 6, seed=15)
    A[1, :] = NEG_INF
    lhs = oracle.maxplus(oracle.maxplus(A, B), D)
    rhs = oracle.maxplus(A, oracle.maxplus(B, D))
    np.testing.assert_array_equal(lhs, rhs)


def test_maxplus_k0_is_empty_fold():
    assert (oracle.maxplus(np.zeros((2, 0), np.int32), np.zeros((0, 3), np.int32)) == NEG_INF).all()


# ----------------------------------------------------------------- boolean

@pytest.mark.parametrize("n,m,k", SHAPES + [(40, 70, 100), (33, 64, 31)])
def test_bool_bits_is_integer_product_positive(n, m, k):
    a, b, _, _ = workloads.bool_operands(n, m, k, density=0.2, seed=n + k)
    expect = (a.astype(np.int64) @ b.astype(np.int64)) > 0
    np.testing.assert_array_equal(oracle.bool_bits(a, b), expect.astype(np.uint8))


def test_bool_exhaustive_2x2():
    for code in range(256):
        bits = [(code >> s) & 1 for s in range(8)]
        a = np.array(bits[:4], np.uint8).reshape(2, 2)
        b = np.array(bits[4:], np.uint8).reshape(2, 2)
        expect = (a.astype(int) @ b.astype(int)) > 0
        np.testing.assert_array_equal(oracle.bool_bits(a, b), expect.astype(np.uint8))


@pytest.mark.parametrize("n,m,k", [(5, 40, 70), (64, 64, 64), (33, 100, 31), (3, 1, 1)])
def test_bool_packed_agrees_with_bits(n, m, k):
    a, b, ap, bp = workloads.bool_operands(n, m, k, density=0.1, seed=m)
    Cw = oracle.bool_packed(ap, bp, n, m, k)
    np.testing.assert_array_equal(oracle.unpack_bits(Cw, m), oracle.bool_bits(a, b))
    if m % 32:
        assert (Cw[:, -1] >> np.uint32(m % 32) == 0).all()   # padding bits stay 0


def test_bool_ones_gives_row_any():
    a, _, ap, _ = workloads.bool_operands(20, 45, 37, density=0.03, seed=2)
    ones = np.ones((37, 45), np.uint8)
    C = oracle.bool_bits(a, ones)
    np.testing.assert_array_equal(C, np.repeat(a.any(axis=1, keepdims=True), 45, axis=1))


def test_bool_accumulate_keeps_old_bits():
    a, b, _, _ = workloads.bool_operands(6, 7, 8, density=0.1, seed=3)
    C0 = np.eye(6, 7, dtype=np.uint8)
    np.testing.assert_array_equal(oracle.bool_bits(a, b, C0), C0 | oracle.bool_bits(a, b))


# ----------------------------------------------------------------- ring

@pytest.mark.parametrize("n,m,k", SHAPES + [(31, 45, 257)])
def test_ring_small_integers_exact(n, m, k):
    A, B = workloads.small_int_operands(n, m, k, seed=k)
    expect = A.astype(np.int64) @ B.astype(np.int64)
    np.testing.assert_array_equal(oracle.ring_f64(A, B), expect.astype(np.float64))


def test_ring_normal_within_rounding_bound_of_library_product():
    A, B = workloads.ring_operands(37, 29, 1500, seed=1)
    C, absC = oracle.ring_f64(A, B, with_abs=True)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    bound = 2 * 1500 * 2.0 ** -53 * absC
    assert (np.abs(C - ref) <= bound).all()
    ref_abs = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    assert (np.abs(absC - ref_abs) <= bound).all()


def test_ring_rows_subset_and_identity():
    A, B = workloads.ring_operands(20, 9, 11, seed=2)
    rows = np.array([19, 0, 7, 7])
    full = oracle.ring_f64(A, B)
    np.testing.assert_array_equal(oracle.ring_f64(A, B, rows=rows), full[rows])
    I = np.eye(11, dtype=np.float32)
    np.testing.assert_array_equal(oracle.ring_f64(A, I), A.astype(np.float64))


# ----------------------------------------------------------------- Strassen

def test_strassen_hand_worked_2x2():
    g = json.load(open(os.path.join(GOLD, "strassen_2x2.json")))
    A, B = np.array(g["A"]), np.array(g["B"])
    np.testing.assert_array_equal(oracle.strassen_i64(A, B, 1), np.array(g["C"]))
    np.testing.assert_array_equal(oracle.strassen_f64(A, B, 1), np.array(g["C"]))


@pytest.mark.parametrize("n,levels", [(2, 1), (4, 2), (12, 2), (16, 3), (40, 3)])
def test_strassen_int64_equals_classic(n, levels):
    r = _rng(n + levels)
    A = r.integers(-50, 50, (n, n))
    B = r.integers(-50, 50, (n, n))
    np.testing.assert_array_equal(oracle.strassen_i64(A, B, levels), A @ B)
    np.testing.assert_array_equal(oracle.ring_i64(A, B), A @ B)


def test_strassen_f64_close_to_classic():
    A, B = workloads.strassen_operands(64, seed=3)
    C = oracle.strassen_f64(A, B, 2)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    assert np.abs(C - ref).max() <= 1e-12 * np.abs(ref).max() * 64


def test_strassen_levels0_is_classic():
    A, B = workloads.strassen_operands(10, seed=4)
    np.testing.assert_array_equal(oracle.strassen_f64(A, B, 0),
                                  oracle.ring_f64(A, B))
