"""GPU parity: libpaco's HIP path against the CPU oracle on the same seeded
inputs.  Integer and boolean results must be bit-exact; ring results within
the componentwise bound max |C - C64| / (|A||B|) <= 2^-20."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

import paper_2011_01441_amd as P  # noqa: E402
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def comp_err(C, A, B):
    C64, S = oracle.ring_f64(A, B, with_abs=True)
    d = np.abs(C.astype(np.float64) - C64)
    return float(np.max(np.where(S > 0, d / np.where(S > 0, S, 1), d)))


# ---------------------------------------------------------------- (min,+)

def test_minplus_config0_bit_exact(ctx):
    print("case: minplus 384x320x256 seed 0", flush=True)
    A, B = workloads.minplus_operands(384, 256, 320, seed=0)
    C, res = ctx.semiring_mm(dev(A), dev(B), "minplus", return_result=True)
    assert np.array_equal(host(C), oracle.minplus(A, B))
    # default p: one processor per resident workgroup slot (a multiple of the CUs)
    cus = P.lib().paco_num_cus(ctx._h)
    assert res["p"] % cus == 0 and res["n_pieces"] == res["p"] and res["n_kcuts"] > 0


@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (5, 3, 2), (97, 130, 75), (300, 77, 129), (64, 64, 1000)])
def test_minplus_ragged(ctx, n, m, k):
    print(f"case: minplus {n}x{m}x{k}", flush=True)
    A, B = workloads.minplus_operands(n, m, k, seed=n + m + k)
    assert np.array_equal(host(ctx.semiring_mm(dev(A), dev(B), "minplus")), oracle.minplus(A, B))


@pytest.mark.parametrize("p,part", [(1, "paco"), (3, "paco"), (257, "paco"), (256, "grid")])
def test_minplus_partition_invariance(ctx, p, part):
    print(f"case: minplus invariance p={p} {part}", flush=True)
    A, B = workloads.minplus_operands(384, 256, 320, seed=0)
    C = ctx.semiring_mm(dev(A), dev(B), "minplus", p=p, part=part)
    assert np.array_equal(host(C), oracle.minplus(A, B))


# ---------------------------------------------------------------- (max,+)

@pytest.mark.parametrize("n,m,k", [(4096, 64, 512), (300, 77, 129), (33, 250, 64)])
def test_maxplus_bit_exact(ctx, n, m, k):
    print(f"case: maxplus {n}x{m}x{k}", flush=True)
    A, B = workloads.maxplus_operands(n, m, k, seed=7)
    A[3, :] = oracle.NEG_INF
    assert np.array_equal(host(ctx.semiring_mm(dev(A), dev(B), "maxplus")), oracle.maxplus(A, B))


# ---------------------------------------------------------------- boolean

@pytest.mark.parametrize("n,m,k,dens", [(50, 100, 70, 0.05), (512, 1024, 2048, 0.0092),
                                        (300, 33, 1000, 0.01), (1, 1, 1, 1.0)])
def test_bool_bit_exact(ctx, n, m, k, dens):
    print(f"case: bool {n}x{m}x{k} d={dens}", flush=True)
    _, _, ap, bp = workloads.bool_operands(n, m, k, density=dens, seed=5)
    Cw = ctx.semiring_mm(dev(ap.view(np.int32)), dev(bp.view(np.int32)), "bool", n=n, m=m, k=k)
    assert np.array_equal(host(Cw).view(np.uint32), oracle.bool_packed(ap, bp, n, m, k))


# ---------------------------------------------------------------- ring

@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("n,m,k", [(70, 90, 300), (256, 512, 1024), (33, 17, 65)])
def test_ring_small_integers_exact(ctx, prec, n, m, k):
    print(f"case: ring small-int {prec} {n}x{m}x{k}", flush=True)
    A, B = workloads.small_int_operands(n, m, k, seed=k)
    C = host(ctx.semiring_mm(dev(A), dev(B), "ring", precision=prec))
    assert np.array_equal(C.astype(np.float64), oracle.ring_f64(A, B))


@pytest.mark.parametrize("prec,k", [("fp32", 512), ("bf16x3", 4096), ("bf16x6", 256)])
def test_ring_normal_within_bound(ctx, prec, k):
    print(f"case: ring normal {prec} k={k}", flush=True)
    A, B = workloads.ring_operands(200, 300, k, seed=3)
    C = host(ctx.semiring_mm(dev(A), dev(B), "ring", precision=prec))
    assert comp_err(C, A, B) <= 2.0 ** -20


def test_ring_verify_rows_matches_oracle(ctx):
    print("case: ring verify", flush=True)
    A, B = workloads.ring_operands(64, 96, 700, seed=4)
    Ad, Bd = dev(A), dev(B)
    C, res = ctx.semiring_mm(Ad, Bd, "ring", precision="bf16x3", verify_rows=64,
                             return_result=True)
    Ch = host(C)
    C64, S = oracle.ring_f64(A, B, with_abs=True)
    rel = np.max(np.abs(Ch - C64) / S)
    assert res["verify_max_rel"] == pytest.approx(rel, rel=1e-9)


# ---------------------------------------------------------------- Strassen

@pytest.mark.parametrize("levels", [1, 2])
def test_strassen_small_integers_exact(ctx, levels):
    print(f"case: strassen small-int L={levels}", flush=True)
    A, B = workloads.small_int_operands(256, 256, 256, seed=9)
    C = host(ctx.strassen_mm(dev(A), dev(B), levels=levels, leaf="bf16x3"))
    expect = oracle.strassen_i64(A.astype(np.int64), B.astype(np.int64), levels)
    assert np.array_equal(C.astype(np.int64), expect)


# ------------------------------------------------- pruned-BFS PACO Strassen

@pytest.mark.parametrize("n,p,gamma,base", [(512, 8, 0, 64), (512, 256, 0, 32), (384, 3, 0, 16),
                                            (500, 5, 0, 8), (256, 1, 0, 64), (512, 7, 1, 32),
                                            (448, 64, 2, 16)])
def test_strassen_pbfs_small_integers_exact(ctx, n, p, gamma, base):
    # Strassen is exact over the integers; with entries in {-2..2} every
    # S, T, M and C value is an integer below 2^24, so any depth of the
    # pruned-BFS schedule must reproduce the classic product bit for bit
    print(f"case: strassen pbfs small-int n={n} p={p} gamma={gamma} base={base}", flush=True)
    A, B = workloads.small_int_operands(n, n, n, seed=11)
    C, res = ctx.strassen_pbfs(dev(A), dev(B), p=p, gamma=gamma, base=base, leaf="bf16x3",
                               return_result=True)
    expect = oracle.ring_i64(A.astype(np.int64), B.astype(np.int64))
    assert np.array_equal(host(C).astype(np.int64), expect)
    levels, wc, _ = P.strassen_schedule(n, p, gamma, base)
    assert res["nodes"] == sum(lv["assigned"] for lv in levels) and res["p"] == p
    assert res["max_work"] == pytest.approx(wc.max()) and res["min_work"] == pytest.approx(wc.min())


@pytest.mark.parametrize("p", [8, 256])
def test_strassen_pbfs_float_normwise(ctx, p):
    # float32 inputs U[-1,1], bf16x3 nodes: normwise error against the
    # float64 classic product within the 2^-16 bound
    print(f"case: strassen pbfs float n=1024 p={p}", flush=True)
    A, B = workloads.strassen_operands(1024, seed=2)
    C = host(ctx.strassen_pbfs(dev(A), dev(B), p=p, base=64, leaf="bf16x3"))
    C64 = oracle.ring_f64(A, B)
    err = np.linalg.norm(C.astype(np.float64) - C64) / (np.linalg.norm(A.astype(np.float64)) *
                                                        np.linalg.norm(B.astype(np.float64)))
    assert err <= 2.0 ** -16, err


def test_strassen_pbfs_rejects_bad_arguments(ctx):
    A = torch.zeros((64, 64), device=DEV)
    with pytest.raises(Exception):
        ctx.strassen_pbfs(A, A, p=100000)
    with pytest.raises(Exception):
        ctx.strassen_pbfs(A, A, gamma=-1)


# --------------------------------------------- multi-piece pruned BFS (GPU)

@pytest.mark.parametrize("p", [0, 3, 251, 256])
def test_minplus_multi_piece_bit_exact(ctx, p):
    print(f"case: minplus multi-piece p={p}", flush=True)
    A, B = workloads.minplus_operands(384, 256, 320, seed=12)
    C, res = ctx.semiring_mm(dev(A), dev(B), "minplus", part="multi", p=p, return_result=True)
    assert np.array_equal(host(C), oracle.minplus(A, B))
    assert res["n_pieces"] >= res["p"]


def test_ring_multi_piece_small_integers_exact(ctx):
    print("case: ring multi-piece small ints p=97", flush=True)
    A, B = workloads.small_int_operands(700, 530, 1500, seed=13)
    C = host(ctx.semiring_mm(dev(A), dev(B), "ring", part="multi", p=97, precision="bf16x3"))
    assert np.array_equal(C.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64))


def test_bool_and_maxplus_multi_piece(ctx):
    print("case: bool and maxplus multi-piece", flush=True)
    n, m, k = 300, 333, 1000
    _, _, ap, bp = workloads.bool_operands(n, m, k, density=0.01, seed=14)
    C = host(ctx.semiring_mm(dev(ap.view(np.int32)), dev(bp.view(np.int32)), "bool", n=n, m=m, k=k,
                             part="multi", p=200))
    assert np.array_equal(C.view(np.uint32), oracle.bool_packed(ap, bp, n, m, k))
    A, B = workloads.maxplus_operands(257, 129, 513, seed=15)
    C = host(ctx.semiring_mm(dev(A), dev(B), "maxplus", part="multi", p=3))
    assert np.array_equal(C, oracle.maxplus(A, B))


# --------------------------------------- heterogeneous split (measured rates)

def test_calibrate_rates(ctx):
    print("case: calibrate 256 processors", flush=True)
    r = ctx.calibrate(256, iters=20000)
    assert r.shape == (256,) and np.all(np.isfinite(r)) and np.all(r > 0)
    # one rate per XCD; together at most the dense bf16 peak
    assert all(len(set(r[32 * x:32 * x + 32])) == 1 for x in range(8))
    assert 0.2 * 2500 < r.sum() < 1.02 * 2500, r.sum()


def test_weighted_split_exact(ctx):
    print("case: weighted split minplus and ring", flush=True)
    A, B = workloads.minplus_operands(384, 256, 320, seed=16)
    w = 1.0 + (np.arange(256) % 4)            # four processor speeds
    C, res = ctx.semiring_mm(dev(A), dev(B), "minplus", p=256, weights=w, return_result=True)
    assert np.array_equal(host(C), oracle.minplus(A, B))
    assert res["max_piece_volume"] > 2 * res["min_piece_volume"]   # faster processors got more
    A, B = workloads.small_int_operands(1000, 700, 2048, seed=17)
    C = host(ctx.semiring_mm(dev(A), dev(B), "ring", p=256, weights=w, precision="bf16x3"))
    assert np.array_equal(C.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64))
    with pytest.raises(Exception):
        ctx.semiring_mm(dev(A), dev(B), "ring", p=256, weights=-w)
    with pytest.raises(Exception):
        ctx.semiring_mm(dev(A), dev(B), "ring", weights=w)     # needs an explicit p
    # weights held by the context serve default-p ring calls
    ctx.set_processor_weights(w)
    try:
        C, res = ctx.semiring_mm(dev(A), dev(B), "ring", precision="bf16x3", return_result=True)
        assert np.array_equal(host(C).astype(np.int64), A.astype(np.int64) @ B.astype(np.int64))
        assert res["p"] == 256 and res["max_piece_volume"] > 2 * res["min_piece_volume"]
    finally:
        ctx.set_processor_weights(None)


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("sr,n,m,k", [("minplus", 300, 77, 129), ("maxplus", 517, 64, 700), ("minplus", 129, 260, 96)])
def test_int_tiles_bit_exact(ctx, tile, sr, n, m, k, monkeypatch):
    """Every (min,+)/(max,+) tile shape (forced through PACO_INT_TILE),
    ragged sizes, k-cuts from the default plan: bit-exact."""
    monkeypatch.setenv("PACO_INT_TILE", str(tile))
    print(f"case: int tile {tile} {sr} {n}x{m}x{k}", flush=True)
    gen = workloads.minplus_operands if sr == "minplus" else workloads.maxplus_operands
    A, B = gen(n, m, k, seed=tile + n)
    ref = (oracle.minplus if sr == "minplus" else oracle.maxplus)(A, B)
    for part in ("paco", "grid"):
        assert np.array_equal(host(ctx.semiring_mm(dev(A), dev(B), sr, part=part)), ref), part


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_ring_forced_tiles_exact(ctx, tile, prec, monkeypatch):
    """Every ring tile shape forced through PACO_RING_TILE (the four-wave
    128 x 128 one included), small integers: exact; the 256 x 256 tile
    with three bf16 parts falls back to a tile that fits."""
    monkeypatch.setenv("PACO_RING_TILE", str(tile))
    n, m, k = 300, 260, 2000
    print(f"case: ring forced tile {tile} {prec}", flush=True)
    A, B = workloads.small_int_operands(n, m, k, seed=tile + 3)
    C = host(ctx.semiring_mm(dev(A), dev(B), "ring", precision=prec, p=64))
    assert np.array_equal(C.astype(np.float64), oracle.ring_f64(A, B))


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("sr", ["minplus", "maxplus"])
def test_int_ragged_k_steps(ctx, tile, sr, monkeypatch):
    """Pieces whose k-range ends anywhere inside a 32-deep step (the kernel
    stops a piece's last step after the 8-deep chunk holding k1 - 1): every
    tile, k from 1 to 257, split-k grids of 1, 3 and 7 parts and the PACO
    plan at p = 5; bit-exact."""
    monkeypatch.setenv("PACO_INT_TILE", str(tile))
    gen = workloads.minplus_operands if sr == "minplus" else workloads.maxplus_operands
    ref_fn = oracle.minplus if sr == "minplus" else oracle.maxplus
    n, m = 70, 90
    for k in (1, 7, 8, 9, 33, 40, 257):
        A, B = gen(n, m, k, seed=tile * 7 + k)
        ref = ref_fn(A, B)
        for sk in (1, 3, 7):
            if sk > k:
                continue
            print(f"case: int ragged k tile {tile} {sr} k={k} split_k={sk}", flush=True)
            got = host(ctx.semiring_mm(dev(A), dev(B), sr, part="grid", split_k=sk))
            assert np.array_equal(got, ref), (k, sk)
        print(f"case: int ragged k tile {tile} {sr} k={k} paco p=5", flush=True)
        assert np.array_equal(host(ctx.semiring_mm(dev(A), dev(B), sr, p=5, kcut_cost=1.0)), ref), k


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("sr", ["minplus", "maxplus"])
def test_int_vector_and_scalar_loads(ctx, tile, sr, monkeypatch):
    """The integer kernel loads four elements at a time where rows and work
    items are 16-byte aligned, one at a time otherwise.  The same operands
    through the aligned path, through A one element off alignment, and
    through a leading dimension that is not a multiple of four (B as well)
    all give the oracle's result bit for bit, on every tile shape."""
    monkeypatch.setenv("PACO_INT_TILE", str(tile))
    n, m, k = 300, 260, 516
    print(f"case: {sr} {n}x{m}x{k} tile {tile} aligned/offset/padded", flush=True)
    gen = workloads.minplus_operands if sr == "minplus" else workloads.maxplus_operands
    A, B = gen(n, m, k, seed=40 + tile)
    ref = (oracle.minplus if sr == "minplus" else oracle.maxplus)(A, B)
    dA, dB = dev(A), dev(B)
    assert np.array_equal(host(ctx.semiring_mm(dA, dB, sr)), ref)
    flat = torch.empty(n * k + 1, dtype=dA.dtype, device=DEV)
    Aoff = flat[1:].view(n, k)
    Aoff.copy_(dA)
    assert Aoff.data_ptr() % 16 != 0
    assert np.array_equal(host(ctx.semiring_mm(Aoff, dB, sr)), ref)
    Apad = torch.empty(n, k + 1, dtype=dA.dtype, device=DEV)[:, :k]
    Bpad = torch.empty(k, m + 3, dtype=dB.dtype, device=DEV)[:, :m]
    Apad.copy_(dA)
    Bpad.copy_(dB)
    assert np.array_equal(host(ctx.semiring_mm(Apad, Bpad, sr)), ref)


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
def test_bool_tiles_bit_exact(ctx, tile, monkeypatch):
    """Every boolean tile shape (4 x 16 register tiles on the three wide
    ones, 4 x 4 on 64 x 64 words) forced through PACO_BOOL_TILE, ragged
    sizes, PACO and split-k grids: bit-exact."""
    monkeypatch.setenv("PACO_BOOL_TILE", str(tile))
    for (n, m, k, dens) in [(300, 1000, 777, 0.02), (513, 2080, 160, 0.05), (64, 31, 4100, 0.005)]:
        _, _, ap, bp = workloads.bool_operands(n, m, k, density=dens, seed=tile + n)
        ref = oracle.bool_packed(ap, bp, n, m, k)
        Ad, Bd = dev(ap.view(np.int32)), dev(bp.view(np.int32))
        for kw in ({}, {"part": "grid", "split_k": 1}, {"part": "grid", "split_k": 3}, {"p": 7, "kcut_cost": 1.0}):
            print(f"case: bool tile {tile} {n}x{m}x{k} {kw}", flush=True)
            got = host(ctx.semiring_mm(Ad, Bd, "bool", n=n, m=m, k=k, **kw)).view(np.uint32)
            assert np.array_equal(got, ref), kw


@pytest.mark.parametrize("sr", ["ring", "minplus", "maxplus", "bool"])
def test_degenerate_shapes(ctx, sr):
    """Section "PACO MM" on empty cuboids: k = 0 is the empty fold, so C is
    the semiring's zero (0, INF, NEG_INF, no bits set) as the oracle gives
    it; with accumulate it leaves C unchanged; n = 0 or m = 0 writes
    nothing.  Also rows of A and columns of B that are all zero elements
    ((min,+): INF, (max,+): NEG_INF) give zero rows and columns of C."""
    print(f"case: {sr} degenerate shapes", flush=True)
    n, m = 37, 70
    dt = torch.float32 if sr == "ring" else torch.int32
    kw = dict(n=n, m=m, k=0) if sr == "bool" else {}
    mw = (m + 31) // 32 if sr == "bool" else m
    A0 = torch.empty((n, 0), dtype=dt, device=DEV)
    B0 = torch.empty((0, mw), dtype=dt, device=DEV)
    C = torch.full((n, mw), 5, dtype=dt, device=DEV)
    ctx.semiring_mm(A0, B0, sr, C=C, **kw)
    want = {"ring": 0, "minplus": oracle.INF, "maxplus": oracle.NEG_INF, "bool": 0}[sr]
    assert (host(C) == want).all()
    if sr == "minplus":
        assert np.array_equal(host(C), oracle.minplus(np.zeros((n, 0), np.int32), np.zeros((0, m), np.int32)))
    if sr == "maxplus":
        assert np.array_equal(host(C), oracle.maxplus(np.zeros((n, 0), np.int32), np.zeros((0, m), np.int32)))
    C.fill_(5)
    ctx.semiring_mm(A0, B0, sr, C=C, accumulate=True, **kw)
    assert (host(C) == 5).all()
    # n = 0 and m = 0: valid calls that write nothing
    k = 33
    kw = dict(n=0, m=m, k=k) if sr == "bool" else {}
    ctx.semiring_mm(torch.empty((0, (k + 31) // 32 if sr == "bool" else k), dtype=dt, device=DEV),
                    torch.empty(((k if sr == "bool" else k), mw), dtype=dt, device=DEV), sr,
                    C=torch.empty((0, mw), dtype=dt, device=DEV), **kw)
    if sr in ("minplus", "maxplus"):
        gen = workloads.minplus_operands if sr == "minplus" else workloads.maxplus_operands
        A, B = gen(n, m, 300, seed=77)
        zero = oracle.INF if sr == "minplus" else oracle.NEG_INF
        A[3, :] = zero
        A[:, 7] = zero
        B[:, 11] = zero
        got = host(ctx.semiring_mm(dev(A), dev(B), sr))
        ref = (oracle.minplus if sr == "minplus" else oracle.maxplus)(A, B)
        assert np.array_equal(got, ref)
        assert (got[3, :] == zero).all() and (got[:, 11] == zero).all()


def _wide_range(shape, seed, stream):
    """float32 sign x 2^e x [1, 2) with e uniform in [-40, 40]: entries
    spanning 24 decades, from seeded counter-based words."""
    w = workloads.words(seed, stream, 3 * int(np.prod(shape))).reshape(3, -1)
    u = workloads.uniform01(w)
    e = np.floor(u[0] * 81.0) - 40.0
    sign = np.where(u[1] < 0.5, -1.0, 1.0)
    return (sign * np.exp2(e) * (1.0 + u[2])).astype(np.float32).reshape(shape)


@pytest.mark.parametrize("prec,bound", [("fp32", 2.0 ** -20), ("bf16x6", 2.0 ** -20), ("bf16x3", 2.0 ** -15)])
def test_ring_wide_exponent_range(ctx, prec, bound):
    """The split products on entries over 24 decades (no overflow, no
    subnormal parts): bf16x6 and float32 stay within the 2^-20 componentwise
    bound relative to |A||B|.  bf16x3 drops up to about 3 * 2^-18 |a||b| per
    product (the lo*lo' term and the rounding of both low parts); its 2^-20
    at long k relies on many terms of similar size averaging out, which a
    wide range of exponents defeats, so here the bound is 2^-15 (emulated
    with exact sums on these operands: 2^-15.9)."""
    n, m, k = 200, 130, 777
    print(f"case: ring wide range {prec}", flush=True)
    A, B = _wide_range((n, k), 3, 90), _wide_range((k, m), 3, 91)
    C = host(ctx.semiring_mm(dev(A), dev(B), "ring", precision=prec))
    assert np.isfinite(C).all()
    assert comp_err(C, A.astype(np.float64), B.astype(np.float64)) <= bound


@pytest.mark.parametrize("sr", ["minplus", "maxplus"])
def test_int_domain_edges(ctx, sr):
    """Entries at the ends of the integer domains: (min,+) values up to
    INF = 2^30, whose sums reach 2^31 and saturate to INF; (max,+) values
    at -2^28 and 2^28 beside NEG_INF, so finite sums sit right at the
    threshold that tells them from absorbed ones.  Bit-exact against the
    oracle."""
    n, m, k = 130, 97, 211
    print(f"case: {sr} domain edges", flush=True)
    w = workloads.words(9, 95 if sr == "minplus" else 96, 2 * (n * k + k * m)).reshape(2, -1)
    u = workloads.uniform01(w)
    if sr == "minplus":
        # half the entries within 2^10 of INF, a tenth exactly INF, the rest small
        def mk(a, b):
            v = np.where(u[0, a:b] < 0.5, (1 << 30) - np.floor(u[1, a:b] * 1024.0),
                         np.floor(u[1, a:b] * 1000.0))
            return np.where(u[0, a:b] > 0.9, float(oracle.INF), v).astype(np.int64).astype(np.int32)
        fn = oracle.minplus
    else:
        lim = oracle.MAXPLUS_FINITE_MAX
        def mk(a, b):
            v = np.where(u[0, a:b] < 0.45, -lim, np.where(u[0, a:b] < 0.9, lim, oracle.NEG_INF))
            v = np.where(u[1, a:b] < 0.2, np.floor(u[1, a:b] * 2000.0) - 1000.0, v)
            return v.astype(np.int64).astype(np.int32)
        fn = oracle.maxplus
    A = mk(0, n * k).reshape(n, k)
    B = mk(n * k, n * k + k * m).reshape(k, m)
    # rows of A and columns of B that put the outputs on the edges
    if sr == "minplus":
        A[0::3, :] = np.maximum(A[0::3, :], (1 << 30) - 1024)   # with the columns below: INF
        A[1::3, :] = np.maximum(A[1::3, :], (1 << 29) - 7)
        B[:, 1::3] = np.maximum(B[:, 1::3], (1 << 29) + 3)      # (1::3, 1::3): sums just below INF
    else:
        A[0::3, :] = -lim
        B[:, 0::3] = -lim                                       # (0::3, 0::3): exactly -2^29
        A[1::3, 1:] = oracle.NEG_INF                            # one finite column left
        B[0, 2::3] = oracle.NEG_INF
    ref = fn(A, B)
    if sr == "minplus":
        assert (ref[0::3, 1::3] == oracle.INF).all() and (ref[1::3, 1::3] < oracle.INF).any()
    else:
        assert (ref[0::3, 0::3] == -2 * lim).all() and (ref == oracle.NEG_INF).any()
    assert np.array_equal(host(ctx.semiring_mm(dev(A), dev(B), sr)), ref)
    assert np.array_equal(host(ctx.semiring_mm(dev(A), dev(B), sr, part="grid", split_k=3)), ref)
