"""The 1D problem on the GPU (paco_dp1d) against the oracle, bit-exact:
sizes spanning several base triangles, single triangles of many lengths,
ragged ends, p not a power of two,
both partitions, both weight families, repeated calls on one plan, the
degenerate sizes, and a full-size run checked on sampled outputs."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

import paper_2011_01441_amd as P  # noqa: E402

DEV = torch.device("cuda:0")
INF = oracle.INF


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.close()


def run(ctx, n, kind, a, b, seed=0, d0=0, **kw):
    D = torch.full((n + 1,), -7, dtype=torch.int32, device=DEV)
    D[0] = d0
    _, r = ctx.dp1d(D, kind, a, b, seed, return_result=True, **kw)
    torch.cuda.synchronize()
    return D.cpu().numpy(), r


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 511, 512, 513, 1000, 4097])
@pytest.mark.parametrize("kind,a,b", [("hash", 0, 20), ("affine", 5, 3)])
def test_small_sizes(ctx, n, kind, a, b):
    print(f"dp1d n={n} {kind}", flush=True)
    got, _ = run(ctx, n, kind, a, b, seed=3, d0=11)
    assert np.array_equal(got, oracle.dp1d(n, kind, a, b, 3, 11))


# one base triangle of n + 1 positions (base 1024): the next block's update
# runs from two 64-position blocks on, the far update beside the chain from
# three; lengths on both sides of those counts, ragged last blocks, the
# largest triangle
@pytest.mark.parametrize("n", [127, 128, 129, 191, 192, 193, 320, 447, 448, 1023])
@pytest.mark.parametrize("kind,a,b", [("hash", 1, 19), ("affine", 2, 7)])
def test_one_triangle_lengths(ctx, n, kind, a, b):
    print(f"dp1d one triangle n={n} {kind}", flush=True)
    got, _ = run(ctx, n, kind, a, b, seed=5, d0=2, base=1024)
    assert np.array_equal(got, oracle.dp1d(n, kind, a, b, 5, 2))


@pytest.mark.parametrize("part,p,base,minp", [("paco", 0, 0, 0), ("paco", 97, 64, 64), ("paco", 1000, 1024, 4096),
                                              ("grid", 0, 0, 0), ("grid", 33, 128, 1024), ("paco", 1, 256, 1)])
def test_partitions_and_bases(ctx, part, p, base, minp):
    n = 20000
    print(f"dp1d n={n} part={part} p={p} base={base} min_piece={minp}", flush=True)
    got, r = run(ctx, n, "hash", 7, 18, seed=0xABCDEF, d0=0, part=part, p=p, base=base, min_piece=minp)
    assert np.array_equal(got, oracle.dp1d(n, "hash", 7, 18, 0xABCDEF, 0))
    assert r["launches"] == r["squares"] + 1 and r["triangles"] == r["squares"] + 1
    if part == "grid":
        assert r["atomic_pieces"] == 0


def test_input_cuts_are_exercised(ctx):
    # a plan whose squares cut their inputs: pieces flagged atomic
    n = 30000
    got, r = run(ctx, n, "hash", 0, 22, seed=9, part="paco", p=512, base=256, min_piece=4096)
    assert r["atomic_pieces"] > 0 and r["max_pieces"] == 512
    assert np.array_equal(got, oracle.dp1d(n, "hash", 0, 22, 9, 0))


def test_repeated_calls_reuse_plan(ctx):
    # the launch counters are left at zero: a second and third call on the
    # cached plan, with other inputs, are exact too
    n = 12345
    for seed, d0 in ((1, 0), (2, 100), (3, INF)):
        got, _ = run(ctx, n, "hash", 3, 16, seed=seed, d0=d0, p=200, base=128, min_piece=2048)
        assert np.array_equal(got, oracle.dp1d(n, "hash", 3, 16, seed, d0))


def test_saturation_and_constant_weights(ctx):
    n = 3000
    got, _ = run(ctx, n, "affine", 0, 1 << 18, d0=0)
    j = np.arange(n + 1, dtype=np.int64)
    assert np.array_equal(got.astype(np.int64), np.minimum(j << 18, INF))
    got, _ = run(ctx, n, "hash", 42, 0, seed=5, d0=1)
    assert got[0] == 1 and (got[1:] == 43).all()


def test_degenerate_sizes_and_errors(ctx):
    D = torch.tensor([5], dtype=torch.int32, device=DEV)
    ctx.dp1d(D, "hash", 0, 10)
    assert int(D.item()) == 5                       # n = 0: nothing to do
    D = torch.zeros(101, dtype=torch.int32, device=DEV)
    with pytest.raises(P.PacoError):
        ctx.dp1d(D, "affine", 1 << 29, 1 << 24)     # a + b n > 2^30
    with pytest.raises(P.PacoError):
        ctx.dp1d(D, "hash", 0, 30)                  # bits > 29
    with pytest.raises(P.PacoError):
        ctx.dp1d(D, "hash", 0, 10, base=32)         # base below 64
    with pytest.raises(ValueError):
        ctx.dp1d(D.float(), "hash", 0, 10)


def test_full_size_sampled(ctx):
    # the benchmark's shape: every sampled output satisfies the recurrence
    # over the GPU's own earlier outputs, and the affine run matches its
    # closed form everywhere
    n = 1 << 18
    print(f"dp1d full size n={n}", flush=True)
    got, r = run(ctx, n, "hash", 0, 20, seed=0, d0=0)
    rng = np.random.default_rng(0)
    js = np.concatenate([np.arange(1, 300), rng.integers(1, n + 1, 700), np.arange(n - 300, n + 1)])
    assert oracle.dp1d_check(got, js, "hash", 0, 20, 0) == 0
    got, _ = run(ctx, n, "affine", 1, 3, d0=2)
    j = np.arange(n + 1, dtype=np.int64)
    exp = 2 + 1 + 3 * j
    exp[0] = 2
    assert np.array_equal(got.astype(np.int64), exp)
