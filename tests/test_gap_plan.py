"""Host-side checks of the GAP plan (section "PACO GAP"): base blocks tile
the grid exactly, every cube is split into pieces that tile it, cubes only
read blocks finished before them and write blocks finished after them, and
a numpy replay of the launch order reproduces the oracle."""
import numpy as np
import pytest

import oracle
import paper_2011_01441_amd as P

INF = oracle.INF


def fmix_np(h):
    h = np.asarray(h, np.uint32).copy()
    h ^= h >> np.uint32(16)
    h *= np.uint32(0x85EBCA6B)
    h ^= h >> np.uint32(13)
    h *= np.uint32(0xC2B2AE35)
    h ^= h >> np.uint32(16)
    return h


def wmat(w, frm, to):
    """gap weight w(from, to) on a grid (test side, int64)."""
    kind, a, b, seed = w
    f = np.asarray(frm, np.int64)[:, None]
    t = np.asarray(to, np.int64)[None, :]
    if kind == "affine":
        return np.minimum(a + b * (t - f), INF)
    key = ((f.astype(np.uint64) * 0x9E3779B9 + t.astype(np.uint64)) & 0xFFFFFFFF).astype(np.uint32) ^ np.uint32(seed)
    return np.minimum(a + (fmix_np(key).astype(np.int64) & ((1 << b) - 1)), INF)


def replay(m, n, wr, wc, s, d0, la, bl, pc):
    D = np.full((m + 1, n + 1), INF, np.int64)
    D[0, 0] = d0
    S = np.zeros((m + 1, n + 1), np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            S[i, j] = oracle.gap_s(s, i, j)
    for base, off, cnt in la:
        if base:
            for r0, r1, c0, c1 in bl[off:off + cnt]:
                for i in range(r0, r1):
                    for j in range(c0, c1):
                        v = D[i, j]
                        if i >= 1 and j >= 1:
                            v = min(v, D[i - 1, j - 1] + S[i, j])
                        if j > c0:
                            v = min(v, int((D[i, c0:j] + wmat(wr, range(c0, j), [j])[:, 0]).min()))
                        if i > r0:
                            v = min(v, int((D[r0:i, j] + wmat(wc, range(r0, i), [i])[:, 0]).min()))
                        D[i, j] = min(v, INF)
        else:
            for col, t0, t1, x0, x1, o0, o1 in pc[off:off + cnt]:
                if col:
                    # D[o][t] = min over x of D[x][t] + w'(x, o)
                    c = D[x0:x1, t0:t1][:, None, :] + wmat(wc, range(x0, x1), range(o0, o1))[:, :, None]
                    D[o0:o1, t0:t1] = np.minimum(D[o0:o1, t0:t1], np.minimum(c.min(axis=0), INF))
                else:
                    c = D[t0:t1, x0:x1][:, :, None] + wmat(wr, range(x0, x1), range(o0, o1))[None, :, :]
                    D[t0:t1, o0:o1] = np.minimum(D[t0:t1, o0:o1], np.minimum(c.min(axis=1), INF))
    return D


CASES = [(0, 0, "paco", 8, 1), (0, 300, "paco", 16, 64), (250, 0, "paco", 16, 64), (63, 64, "paco", 4, 1),
         (64, 65, "paco", 64, 4096), (200, 130, "paco", 33, 1000), (300, 300, "grid", 64, 2000),
         (129, 257, "paco", 1024, 65536)]


@pytest.mark.parametrize("m,n,part,p,minp", CASES)
def test_plan_structure(m, n, part, p, minp):
    la, bl, pc, cubes = P.gap_plan(m, n, part, p, minp)
    done = np.zeros((m + 1, n + 1), bool)
    for base, off, cnt in la:
        if base:
            assert cnt >= 1
            for r0, r1, c0, c1 in bl[off:off + cnt]:
                assert 0 <= r0 < r1 <= m + 1 and 0 <= c0 < c1 <= n + 1
                assert r1 - r0 <= 64 and c1 - c0 <= 64
                assert not done[r0:r1, c0:c1].any()
                # every cell above, left and above-left is final already
                if r0 > 0:
                    assert done[r0 - 1, c0:c1].all()
                if c0 > 0:
                    assert done[r0:r1, c0 - 1].all()
                done[r0:r1, c0:c1] = True
        else:
            for col, t0, t1, x0, x1, o0, o1 in pc[off:off + cnt]:
                assert t0 < t1 and x0 < x1 and o0 < o1 and x1 <= o0
                if col:
                    assert t1 <= n + 1 and o1 <= m + 1
                    assert done[x0:x1, t0:t1].all() and not done[o0:o1, t0:t1].any()
                else:
                    assert t1 <= m + 1 and o1 <= n + 1
                    assert done[t0:t1, x0:x1].all() and not done[t0:t1, o0:o1].any()
    assert done.all() and len(bl) == sum(c for b, _, c in la if b)


def test_cube_pieces_tile_each_cube():
    # pieces of one launch, grouped by cube (same flag, batch, input and
    # output spans after merging), cover every (t, x, o) once
    m = n = 300
    la, bl, pc, cubes = P.gap_plan(m, n, "paco", 96, 64)
    total = 0
    for base, off, cnt in la:
        if base:
            continue
        cover = {}
        for col, t0, t1, x0, x1, o0, o1 in pc[off:off + cnt]:
            for t in range(t0, t1):
                key = (col, t)
                arr = cover.setdefault(key, {})
                arr[(x0, x1, o0, o1)] = arr.get((x0, x1, o0, o1), 0) + 1
                total += (x1 - x0) * (o1 - o0)
        for key, spans in cover.items():
            assert all(v == 1 for v in spans.values())
    # every pair (q < j) of every row and (p < i) of every column is one
    # cube term or one in-block term
    inblock = sum((r1 - r0) * (c1 - c0) * ((c1 - c0 - 1) + (r1 - r0 - 1)) // 2 for r0, r1, c0, c1 in bl)
    assert total + inblock == (m + 1) * (n + 1) * n // 2 + (n + 1) * (m + 1) * m // 2


@pytest.mark.parametrize("m,n,part,p,minp", [(90, 140, "paco", 37, 500), (150, 70, "grid", 16, 300),
                                             (130, 130, "paco", 64, 1)])
@pytest.mark.parametrize("wr,wc,s", [(("hash", 0, 12, 3), ("hash", 2, 10, 4), (0, 5, 2, 7, 8)),
                                     (("affine", 4, 1, 0), ("affine", 0, 2, 0), (1, 3, 1, 9, 9))])
def test_replay_of_plan_matches_oracle(m, n, part, p, minp, wr, wc, s):
    la, bl, pc, _ = P.gap_plan(m, n, part, p, minp)
    got = replay(m, n, wr, wc, s, 3, la, bl, pc)
    assert np.array_equal(got, oracle.gap(m, n, wr, wc, s, d0=3).astype(np.int64))


def test_plan_export_rejects_bad_arguments():
    with pytest.raises(P.PacoError):
        P.gap_plan(10, 10, "paco", 0, 1)
    with pytest.raises(P.PacoError):
        P.gap_plan(-1, 10, "paco", 4, 1)
