"""Host-side checks of the 1D-problem plan (section "PACO 1D"): base
triangles tile [0, n] in order, every square's pieces tile it exactly and
stay inside D, input-cut pieces are flagged, the PACO cut rule gives equal
pieces, and a numpy replay of the plan's launch order reproduces the oracle."""
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


def wmat(kind, a, b, seed, i, j):
    """w on the grid i x j (test-side, int64)."""
    i = np.asarray(i, np.int64)[:, None]
    j = np.asarray(j, np.int64)[None, :]
    if kind == "affine":
        return np.minimum(a + b * (j - i), INF)
    key = ((i.astype(np.uint64) * 0x9E3779B9 + j.astype(np.uint64)) & 0xFFFFFFFF).astype(np.uint32) ^ np.uint32(seed)
    return np.minimum(a + (fmix_np(key).astype(np.int64) & ((1 << b) - 1)), INF)


def test_test_side_weights_match_oracle():
    rng = np.random.default_rng(0)
    for kind, a, b, seed in (("affine", 3, 7, 0), ("hash", 11, 20, 0xDEADBEEF)):
        for _ in range(50):
            i, j = sorted(rng.integers(0, 1 << 20, 2))
            assert wmat(kind, a, b, seed, [i], [j])[0, 0] == oracle.dp1d_w(kind, a, b, seed, int(i), int(j))


def replay(n, kind, a, b, seed, d0, first, squares, pieces):
    D = np.full(n + 1, INF, np.int64)
    D[0] = d0

    def tri(lo, ln):
        for j in range(lo, lo + ln):
            if j > lo:
                c = D[lo:j] + wmat(kind, a, b, seed, np.arange(lo, j), [j])[:, 0]
                D[j] = min(D[j], int(c.min()))
            D[j] = min(D[j], INF)

    tri(0, first)
    for lo, mid, hi, off, cnt, tlo, tln, _ in squares:
        for i0, i1, j0, j1, _ in pieces[off:off + cnt]:
            c = D[i0:i1, None] + wmat(kind, a, b, seed, np.arange(i0, i1), np.arange(j0, j1))
            D[j0:j1] = np.minimum(D[j0:j1], np.minimum(c.min(axis=0), INF))
        tri(tlo, tln)
    return D


CASES = [(1, "paco", 64, 64, 1), (63, "paco", 16, 64, 16), (64, "paco", 16, 64, 16),
         (1000, "paco", 64, 128, 256), (1000, "grid", 64, 128, 256), (3000, "paco", 97, 256, 1024),
         (3000, "paco", 1024, 512, 65536), (5000, "grid", 300, 64, 100)]


@pytest.mark.parametrize("n,part,p,base,minp", CASES)
def test_plan_structure(n, part, p, base, minp):
    first, ntri, sq, pc = P.dp1d_plan(n, part, p, base, minp)
    assert 1 <= first <= base and ntri == len(sq) + 1
    # base triangles tile [0, n] in launch order
    pos = first
    for lo, mid, hi, off, cnt, tlo, tln, ntri in sq:
        assert 0 <= lo < mid < hi <= n + 1
        # the pieces the triangle waits for come first, and are exactly
        # those whose outputs reach into it
        assert 1 <= ntri <= cnt
        reach = pc[off:off + cnt, 2] < tlo + tln
        assert reach[:ntri].all() and not reach[ntri:].any()
        # the square's inputs are all finished when it launches
        assert mid <= pos and tlo == pos and 1 <= tln <= base
        pos += tln
        # its pieces tile [lo, mid) x [mid, hi) exactly
        pcs = pc[off:off + cnt]
        assert 1 <= cnt <= max(1, p) and len(pcs) == cnt
        cover = np.zeros((mid - lo, hi - mid), np.int32)
        for i0, i1, j0, j1, at in pcs:
            assert lo <= i0 < i1 <= mid and mid <= j0 < j1 <= hi
            assert at == (1 if (i1 - i0) < (mid - lo) else 0)
            if part == "grid":
                assert at == 0
            cover[i0 - lo:i1 - lo, j0 - mid:j1 - mid] += 1
        assert (cover == 1).all()
    assert pos == n + 1


def test_paco_cut_rule_balances_pieces():
    # large squares go to all p processors with near-equal areas (cut
    # quanta 64 x 8 bound the spread)
    first, ntri, sq, pc = P.dp1d_plan(1 << 16, "paco", 256, 512, 65536)
    lo, mid, hi, off, cnt, _, _, _ = sq[np.argmax(sq[:, 2] - sq[:, 1])]
    assert cnt == 256
    areas = (pc[off:off + cnt, 1] - pc[off:off + cnt, 0]) * (pc[off:off + cnt, 3] - pc[off:off + cnt, 2])
    assert areas.sum() == (mid - lo) * (hi - mid)
    assert areas.max() / areas.mean() < 1.02


def test_grid_baseline_cuts_outputs_only():
    first, ntri, sq, pc = P.dp1d_plan(1 << 14, "grid", 1024, 512, 65536)
    assert (pc[:, 4] == 0).all()
    for lo, mid, hi, off, cnt, _, _, _ in sq:
        assert (pc[off:off + cnt, 0] == lo).all() and (pc[off:off + cnt, 1] == mid).all()


@pytest.mark.parametrize("kind,a,b,seed,d0", [("hash", 0, 16, 5, 0), ("affine", 9, 2, 0, 3), ("hash", 100, 20, 1, 7)])
@pytest.mark.parametrize("n,part,p,base,minp", [(700, "paco", 64, 64, 64), (1500, "paco", 37, 128, 500),
                                                (1500, "grid", 64, 128, 500)])
def test_replay_of_plan_matches_oracle(kind, a, b, seed, d0, n, part, p, base, minp):
    first, ntri, sq, pc = P.dp1d_plan(n, part, p, base, minp)
    got = replay(n, kind, a, b, seed, d0, first, sq, pc)
    assert np.array_equal(got, oracle.dp1d(n, kind, a, b, seed, d0).astype(np.int64))


def test_plan_export_rejects_bad_arguments():
    with pytest.raises(P.PacoError):
        P.dp1d_plan(100, "paco", 0, 512, 65536)
    with pytest.raises(P.PacoError):
        P.dp1d_plan(100, "paco", 64, 2048, 65536)
    with pytest.raises(P.PacoError):
        P.dp1d_plan(100, "multi", 64, 512, 65536)
