"""CPU oracle for semiring matrix multiplication and Strassen's algorithm.

TEST INFRASTRUCTURE ONLY: importable from the test suite, the smoke check and
the benchmark's CPU-baseline leg.  The GPU library never imports it, and it
imports nothing from the GPU library.

Every function is a thin numpy/ctypes wrapper over `oracle.c`, which holds
the plain definitions (section "PACO MM" problem statement, section "PACO
Strassen" formulas, section "PACO 1D", equation (1D), and section "PACO
GAP", equation (gap)); see that file's header for the semiring readings.
"""
import ctypes
import os

import numpy as np

from . import build as _build

INF = 1 << 30          # (min,+) zero element
NEG_INF = -(1 << 30)   # (max,+) zero element
MAXPLUS_FINITE_MAX = 1 << 28   # finite (max,+) domain is [-2^28, 2^28]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        for name in ("oracle_minplus", "oracle_maxplus"):
            getattr(L, name).argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, ci]
        for name in ("oracle_bool_bits", "oracle_bool_packed"):
            getattr(L, name).argtypes = [i64, i64, i64, vp, vp, vp, ci]
        L.oracle_ring_f64.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, vp]
        L.oracle_ring_f64_dd.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
        L.oracle_ring_i64.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
        L.oracle_strassen_f64.argtypes = [i64, vp, vp, vp, ci]
        L.oracle_strassen_i64.argtypes = [i64, vp, vp, vp, ci]
        L.oracle_set_threads.argtypes = [ci]
        L.oracle_fmix32.argtypes = [ctypes.c_uint32]
        L.oracle_fmix32.restype = ctypes.c_uint32
        L.oracle_dp1d_w.argtypes = [ci, i64, i64, ctypes.c_uint32, i64, i64]
        L.oracle_dp1d_w.restype = i64
        L.oracle_dp1d.argtypes = [i64, ci, i64, i64, ctypes.c_uint32, vp]
        L.oracle_dp1d_check.argtypes = [ci, i64, i64, ctypes.c_uint32, vp, vp, i64]
        L.oracle_dp1d_check.restype = i64
        L.oracle_gap_s.argtypes = [i64, i64, ci, ctypes.c_uint32, ctypes.c_uint32, i64, i64]
        L.oracle_gap_s.restype = i64
        L.oracle_gap.argtypes = [i64, i64, vp, vp, vp, vp, i64]
        L.oracle_gap_check.argtypes = [i64, i64, vp, vp, vp, vp, i64, vp, i64]
        L.oracle_gap_check.restype = i64
        L.oracle_num_threads.restype = ci
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _shape(A, B):
    n, k = A.shape
    k2, m = B.shape
    assert k == k2, (A.shape, B.shape)
    return n, m, k


def minplus(A, B, C=None):
    """(min,+) product of int32 matrices; C given means C <- C (+) A (x) B."""
    A = np.ascontiguousarray(A, np.int32)
    B = np.ascontiguousarray(B, np.int32)
    n, m, k = _shape(A, B)
    acc = C is not None
    out = np.ascontiguousarray(C, np.int32).copy() if acc else np.empty((n, m), np.int32)
    lib().oracle_minplus(n, m, k, _p(A), k, _p(B), m, _p(out), m, int(acc))
    return out


def maxplus(A, B, C=None):
    """(max,+) product of int32 matrices; C given means C <- C (+) A (x) B."""
    A = np.ascontiguousarray(A, np.int32)
    B = np.ascontiguousarray(B, np.int32)
    n, m, k = _shape(A, B)
    acc = C is not None
    out = np.ascontiguousarray(C, np.int32).copy() if acc else np.empty((n, m), np.int32)
    lib().oracle_maxplus(n, m, k, _p(A), k, _p(B), m, _p(out), m, int(acc))
    return out


def bool_bits(A, B, C=None):
    """Boolean OR-AND product of unpacked 0/1 uint8 matrices."""
    A = np.ascontiguousarray(A, np.uint8)
    B = np.ascontiguousarray(B, np.uint8)
    n, m, k = _shape(A, B)
    acc = C is not None
    out = np.ascontiguousarray(C, np.uint8).copy() if acc else np.empty((n, m), np.uint8)
    lib().oracle_bool_bits(n, m, k, _p(A), _p(B), _p(out), int(acc))
    return out


def bool_packed(Aw, Bw, n, m, k, Cw=None):
    """Boolean product of bit-packed rows (uint32 words, LSB first)."""
    kw, mw = (k + 31) // 32, (m + 31) // 32
    Aw = np.ascontiguousarray(Aw, np.uint32)
    Bw = np.ascontiguousarray(Bw, np.uint32)
    assert Aw.shape == (n, kw) and Bw.shape == (k, mw), (Aw.shape, Bw.shape)
    acc = Cw is not None
    out = np.ascontiguousarray(Cw, np.uint32).copy() if acc else np.empty((n, mw), np.uint32)
    lib().oracle_bool_packed(n, m, k, _p(Aw), _p(Bw), _p(out), int(acc))
    return out


def ring_f64(A, B, rows=None, with_abs=False):
    """Binary64 (+,x) product of float32 matrices, ascending-l sums.

    rows: optional 1-D array of row indices; only those rows are computed.
    with_abs: also return sum_l |A||B| per entry (the error scale).
    """
    A = np.ascontiguousarray(A, np.float32)
    B = np.ascontiguousarray(B, np.float32)
    n, m, k = _shape(A, B)
    if rows is None:
        nr, rp = n, None
    else:
        rows = np.ascontiguousarray(rows, np.int64)
        assert rows.size == 0 or (rows.min() >= 0 and rows.max() < n)
        nr, rp = rows.size, _p(rows)
    C = np.empty((nr, m), np.float64)
    Ab = np.empty((nr, m), np.float64) if with_abs else None
    lib().oracle_ring_f64(n, m, k, _p(A), k, _p(B), m, rp, nr, _p(C),
                          _p(Ab) if with_abs else None)
    return (C, Ab) if with_abs else C


def ring_i64(A, B):
    A = np.ascontiguousarray(A, np.int64)
    B = np.ascontiguousarray(B, np.int64)
    n, m, k = _shape(A, B)
    C = np.empty((n, m), np.int64)
    lib().oracle_ring_i64(n, m, k, _p(A), k, _p(B), m, _p(C), m)
    return C


def strassen_f64(A, B, levels):
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    n = A.shape[0]
    assert A.shape == (n, n) and B.shape == (n, n)
    C = np.empty((n, n), np.float64)
    lib().oracle_strassen_f64(n, _p(A), _p(B), _p(C), int(levels))
    return C


def strassen_i64(A, B, levels):
    A = np.ascontiguousarray(A, np.int64)
    B = np.ascontiguousarray(B, np.int64)
    n = A.shape[0]
    assert A.shape == (n, n) and B.shape == (n, n)
    C = np.empty((n, n), np.int64)
    lib().oracle_strassen_i64(n, _p(A), _p(B), _p(C), int(levels))
    return C


W_KIND = {"affine": 0, "hash": 1}


def fmix32(h):
    return lib().oracle_fmix32(int(h) & 0xFFFFFFFF)


def dp1d_w(kind, a, b, seed, i, j):
    """The weight w(i, j) of the 1D problem (see oracle.c)."""
    return lib().oracle_dp1d_w(W_KIND[kind], a, b, int(seed) & 0xFFFFFFFF, i, j)


def dp1d(n, kind, a, b, seed=0, d0=0):
    """D[0..n] of the 1D problem, D[0] = d0 (section "PACO 1D")."""
    D = np.empty(n + 1, np.int32)
    D[0] = d0
    lib().oracle_dp1d(n, W_KIND[kind], a, b, int(seed) & 0xFFFFFFFF, _p(D))
    return D


def dp1d_check(D, js, kind, a, b, seed=0):
    """How many of the listed j do not satisfy the recurrence over the given
    D[0..j-1]."""
    D = np.ascontiguousarray(D, np.int32)
    js = np.ascontiguousarray(js, np.int64)
    assert js.size == 0 or (js.min() >= 0 and js.max() < D.size)
    return lib().oracle_dp1d_check(W_KIND[kind], a, b, int(seed) & 0xFFFFFFFF, _p(D), _p(js), js.size)


def _gap_params(wrow, wcol, s):
    """wrow, wcol: (kind, a, b, seed); s: (s_match, s_mismatch, bits, seed_x, seed_y)."""
    wr = np.array([W_KIND[wrow[0]], wrow[1], wrow[2], wrow[3] & 0xFFFFFFFF], np.int64)
    wc = np.array([W_KIND[wcol[0]], wcol[1], wcol[2], wcol[3] & 0xFFFFFFFF], np.int64)
    sp = np.array([s[0], s[1], s[2], s[3] & 0xFFFFFFFF, s[4] & 0xFFFFFFFF], np.int64)
    return wr, wc, sp


def gap_s(s, i, j):
    return lib().oracle_gap_s(s[0], s[1], s[2], s[3] & 0xFFFFFFFF, s[4] & 0xFFFFFFFF, i, j)


def gap(m, n, wrow, wcol, s, d0=0):
    """The (m+1) x (n+1) grid of the GAP problem (section "PACO GAP")."""
    wr, wc, sp = _gap_params(wrow, wcol, s)
    D = np.empty((m + 1, n + 1), np.int32)
    D[0, 0] = d0
    lib().oracle_gap(m, n, _p(wr), _p(wc), _p(sp), _p(D), n + 1)
    return D


def gap_check(D, cells, wrow, wcol, s):
    """How many listed (i, j) cells do not satisfy the recurrence over the given D."""
    D = np.ascontiguousarray(D, np.int32)
    m, n = D.shape[0] - 1, D.shape[1] - 1
    cells = np.ascontiguousarray(cells, np.int64).reshape(-1, 2)
    assert cells.size == 0 or (cells[:, 0].max() <= m and cells[:, 1].max() <= n and cells.min() >= 0)
    wr, wc, sp = _gap_params(wrow, wcol, s)
    return lib().oracle_gap_check(m, n, _p(wr), _p(wc), _p(sp), _p(D), n + 1, _p(cells), cells.shape[0])


def unpack_bits(W, cols):
    """Oracle-side unpacking of packed rows into 0/1 uint8 (LSB first)."""
    W = np.ascontiguousarray(W, np.uint32)
    rows = W.shape[0]
    out = np.zeros((rows, cols), np.uint8)
    for c in range(cols):
        out[:, c] = (W[:, c // 32] >> np.uint32(c % 32)) & np.uint32(1)
    return out


def num_threads():
    return lib().oracle_num_threads()


def set_threads(n):
    """Threads for the oracle's OpenMP loops from now on."""
    lib().oracle_set_threads(int(n))
