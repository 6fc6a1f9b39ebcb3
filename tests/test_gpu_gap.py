"""The GAP problem on the GPU (paco_gap) against the oracle, bit-exact:
degenerate and ragged grids, single base blocks of many shapes, one to many
base blocks, both partitions,
p not a power of two, both weight families, repeated calls on one plan, a
padded leading dimension, and a full-size grid checked at sampled cells."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

import paper_2011_01441_amd as P  # noqa: E402

DEV = torch.device("cuda:0")
INF = oracle.INF
WH = (("hash", 0, 12, 3), ("hash", 2, 10, 4), (0, 5, 2, 7, 8))
WA = (("affine", 4, 1, 0), ("affine", 0, 2, 0), (1, 3, 1, 9, 9))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.close()


def run(ctx, m, n, wr, wc, s, d0=0, ld=None, **kw):
    ld = ld or n + 1
    buf = torch.full((m + 1, ld), -5, dtype=torch.int32, device=DEV)
    D = buf[:, :n + 1]
    D[0, 0] = d0
    _, r = ctx.gap(D, wr, wc, s, return_result=True, **kw)
    torch.cuda.synchronize()
    return D.cpu().numpy(), r


@pytest.mark.parametrize("m,n", [(0, 0), (0, 200), (150, 0), (1, 1), (63, 64), (64, 65), (200, 300), (513, 257)])
@pytest.mark.parametrize("w", [WH, WA])
def test_sizes(ctx, m, n, w):
    print(f"gap m={m} n={n} {w[0][0]}", flush=True)
    got, _ = run(ctx, m, n, *w, d0=3)
    assert np.array_equal(got, oracle.gap(m, n, *w, d0=3))


# grids of one base block (R x C cells, R, C <= 64): the block's
# anti-diagonals run in loops of one slot count per side, which changes where
# max(R, C) - 1 crosses 16, 32 and 48; square, flat and tall blocks on both
# sides of each change
@pytest.mark.parametrize("R,C", [(16, 16), (17, 17), (18, 5), (5, 18), (33, 2), (2, 33), (34, 50), (50, 34),
                                 (49, 49), (64, 17), (17, 64), (64, 1), (1, 64), (64, 64)])
@pytest.mark.parametrize("w", [WH, WA])
def test_single_block_shapes(ctx, R, C, w):
    print(f"gap one block {R}x{C} {w[0][0]}", flush=True)
    got, r = run(ctx, R - 1, C - 1, *w, d0=1)
    assert r["base_blocks"] == 1
    assert np.array_equal(got, oracle.gap(R - 1, C - 1, *w, d0=1))


@pytest.mark.parametrize("part,p,minp", [("paco", 0, 0), ("paco", 37, 500), ("paco", 1, 1), ("grid", 0, 0),
                                         ("grid", 100, 4096), ("paco", 2000, 64)])
def test_partitions(ctx, part, p, minp):
    m, n = 700, 900
    print(f"gap {m}x{n} part={part} p={p} min_piece={minp}", flush=True)
    got, r = run(ctx, m, n, *WH, part=part, p=p, min_piece=minp)
    assert np.array_equal(got, oracle.gap(m, n, *WH))
    assert r["launches"] >= 2 and r["base_blocks"] >= 1


def test_repeated_calls_and_padded_rows(ctx):
    m, n = 333, 444
    for d0, w in ((0, WH), (7, WA), (INF, WH)):
        got, _ = run(ctx, m, n, *w, d0=d0, ld=512, p=97, min_piece=2048)
        assert np.array_equal(got, oracle.gap(m, n, *w, d0=d0))


# one weight family per direction: the base and cube kernels have one
# instantiation per (row, column) pair of families
@pytest.mark.parametrize("wr,wc", [(("hash", 1, 11, 5), ("affine", 3, 2, 0)), (("affine", 2, 1, 0), ("hash", 0, 9, 6))])
@pytest.mark.parametrize("part", ["paco", "grid"])
def test_mixed_weight_kinds(ctx, wr, wc, part):
    m, n = 300, 517
    s = (1, 4, 2, 3, 4)
    print(f"gap {m}x{n} rows {wr[0]} columns {wc[0]} part={part}", flush=True)
    got, _ = run(ctx, m, n, wr, wc, s, d0=2, part=part)
    assert np.array_equal(got, oracle.gap(m, n, wr, wc, s, d0=2))


def test_edit_distance_instance(ctx):
    # linear gaps, unit costs over 4 symbols: the Levenshtein distance of two
    # hashed DNA-like strings (the oracle's Wagner-Fischer pin)
    m, n = 400, 350
    w = (("affine", 0, 1, 0), ("affine", 0, 1, 0), (0, 1, 2, 11, 22))
    got, _ = run(ctx, m, n, *w)
    assert np.array_equal(got, oracle.gap(m, n, *w))
    assert 0 < got[m, n] <= max(m, n)


def test_errors(ctx):
    D = torch.zeros((11, 11), dtype=torch.int32, device=DEV)
    with pytest.raises(P.PacoError):
        ctx.gap(D, ("affine", 1 << 29, 1 << 26, 0), WH[1], WH[2])   # a + b side > 2^30
    with pytest.raises(P.PacoError):
        ctx.gap(D, ("hash", 0, 30, 0), WH[1], WH[2])                # bits > 29
    with pytest.raises(ValueError):
        ctx.gap(D.float(), *WH)


def test_full_size_sampled(ctx):
    m = n = 4096
    print(f"gap full size {m}x{n}", flush=True)
    got, r = run(ctx, m, n, *WH)
    rng = np.random.default_rng(0)
    cells = np.concatenate([rng.integers(0, m + 1, (600, 2)),
                            [[0, n], [m, 0], [m, n], [1, 1], [64, 64], [2048, 2049]]])
    assert oracle.gap_check(got, cells, *WH) == 0
