"""GPU parity against the oracle at the workloads' full sizes, element by
element wherever the oracle computes the whole result in seconds:

* (max,+) C2a 131072x512x64 and boolean C2b 8192^3 bits: every output,
  bit-exact;
* the 1D problem at n = 2^18, both weight families: every output, bit-exact
  (equation (1D));
* the GAP problem on the 4097^2 grid: cell (i, j) depends only on cells
  (p, q) with p <= i, q <= j, so the top-left 1025^2 block of the full run
  equals the oracle's 1024 x 1024 instance with the same weights and
  symbols, bit for bit (equation (gap));
* Strassen with 2 fixed levels over the MM-1-Piece batch of its 49 leaves
  (section "PACO Strassen") at n = 16384: sampled rows against the float64
  classic product, normwise error <= 2^-16, componentwise error reported;
* accumulation C <- C (+) A (x) B for every semiring on shapes whose
  partition cuts k (temporary faces folded onto the caller's C).
"""
import math

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


# ------------------------------------------------------------ C2a and C2b

def test_c2a_maxplus_every_output(ctx):
    print("case: C2a (max,+) 131072x512x64 seed 0, every output", flush=True)
    A, B = workloads.maxplus_operands(131072, 64, 512, seed=0)
    C, res = ctx.semiring_mm(dev(A), dev(B), "maxplus", return_result=True)
    assert np.array_equal(host(C), oracle.maxplus(A, B))
    assert res["n_pieces"] >= 256


@pytest.mark.parametrize("density", [0.05, 0.0092])
def test_c2b_bool_every_output(ctx, density):
    # 0.05 is the workload (C is almost all ones); 0.0092 gives about half
    # ones, so a wrong bit anywhere is seen
    print(f"case: C2b boolean 8192^3 bits density {density} seed 0, every output", flush=True)
    n = m = k = 8192
    ap, bp = workloads.bool_operands_packed(n, m, k, density=density, seed=0)
    Cw = ctx.semiring_mm(dev(ap.view(np.int32)), dev(bp.view(np.int32)), "bool", n=n, m=m, k=k)
    expect = oracle.bool_packed(ap, bp, n, m, k)
    assert np.array_equal(host(Cw).view(np.uint32), expect)
    if density < 0.01:
        ones = np.unpackbits(expect.view(np.uint8)).mean()
        assert 0.2 < ones < 0.8


# ------------------------------------------------------------- 1D and GAP

@pytest.mark.parametrize("kind,a,b,seed,d0", [("hash", 0, 20, 0, 0), ("affine", 1, 3, 0, 2)])
def test_dp1d_2pow18_every_output(ctx, kind, a, b, seed, d0):
    n = 1 << 18
    print(f"case: dp1d n=2^18 {kind} every output", flush=True)
    D = torch.full((n + 1,), -7, dtype=torch.int32, device=DEV)
    D[0] = d0
    ctx.dp1d(D, kind, a, b, seed)
    assert np.array_equal(host(D), oracle.dp1d(n, kind, a, b, seed, d0))


@pytest.mark.parametrize("w", [
    (("hash", 0, 12, 3), ("hash", 2, 10, 4), (0, 5, 2, 7, 8)),       # the gap_hash workload
    (("affine", 4, 1, 0), ("affine", 4, 1, 0), (0, 3, 2, 7, 8)),     # the gap_affine workload
])
def test_gap_4097_top_left_block(ctx, w):
    m = n = 4096
    print(f"case: gap {m + 1}^2 {w[0][0]}, top-left 1025^2 block", flush=True)
    D = torch.full((m + 1, n + 1), -5, dtype=torch.int32, device=DEV)
    D[0, 0] = 0
    ctx.gap(D, *w)
    got = D[:1025, :1025].cpu().numpy()
    assert np.array_equal(got, oracle.gap(1024, 1024, *w))


# ------------------------------------------------- C3: 2 fixed levels

def test_c3_strassen_levels2_sampled(ctx):
    n = 16384
    print("case: C3 Strassen n=16384, 2 levels, 49 leaves over MM-1-Piece, bf16x3, sampled rows", flush=True)
    A, B = workloads.strassen_operands(n, seed=0)
    Ad, Bd = dev(A), dev(B)
    C = ctx.strassen_mm(Ad, Bd, levels=2, leaf="bf16x3")
    rng = np.random.default_rng(6)
    rows = np.unique(np.concatenate([[0, n // 4 - 1, n // 4, n // 2, n - 1], rng.integers(0, n, 11)]))
    C64, S = oracle.ring_f64(A, B, rows=rows, with_abs=True)
    Cr = C[torch.from_numpy(rows).to(DEV)].cpu().numpy().astype(np.float64)
    num = math.sqrt(np.sum((Cr - C64) ** 2) * n / len(rows))
    den = float(np.linalg.norm(A.astype(np.float64))) * float(np.linalg.norm(B.astype(np.float64)))
    comp = float(np.max(np.abs(Cr - C64) / S))
    print(f"  normwise 2^{math.log2(num / den):.1f}, componentwise 2^{math.log2(comp):.1f}", flush=True)
    assert num / den <= 2.0 ** -16
    assert np.all(np.isfinite(Cr))


# ------------------------------------------------------------ accumulate

@pytest.mark.parametrize("sr,n,m,k", [("minplus", 384, 256, 320), ("minplus", 64, 96, 5000),
                                      ("maxplus", 300, 77, 4000), ("maxplus", 256, 64, 512)])
def test_accumulate_integer_semirings(ctx, sr, n, m, k):
    print(f"case: accumulate {sr} {n}x{m}x{k}", flush=True)
    gen = workloads.minplus_operands if sr == "minplus" else workloads.maxplus_operands
    A, B = gen(n, m, k, seed=21)
    C0 = gen(n, 1, m, seed=22)[0]          # an initial n x m C of the same distribution
    fn = oracle.minplus if sr == "minplus" else oracle.maxplus
    Cd = dev(C0)
    C, res = ctx.semiring_mm(dev(A), dev(B), sr, C=Cd, accumulate=True, p=256, return_result=True)
    assert res["n_kcuts"] > 0
    assert np.array_equal(host(C), fn(A, B, C=C0))


def test_accumulate_boolean(ctx):
    n, m, k = 96, 200, 9000
    print(f"case: accumulate bool {n}x{m}x{k}", flush=True)
    _, _, ap, bp = workloads.bool_operands(n, m, k, density=0.0005, seed=23)
    c0 = workloads.bool_operands(n, 1, m, density=0.3, seed=24)[2]   # n x m bits, packed
    Cd = dev(c0.view(np.int32))
    C, res = ctx.semiring_mm(dev(ap.view(np.int32)), dev(bp.view(np.int32)), "bool", n=n, m=m, k=k, C=Cd,
                             accumulate=True, p=256, return_result=True)
    assert res["n_kcuts"] > 0
    assert np.array_equal(host(C).view(np.uint32), oracle.bool_packed(ap, bp, n, m, k, Cw=c0))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_accumulate_ring_small_integers(ctx, prec):
    # entries in {-2..2} and an integer C: every partial sum is an integer
    # below 2^24, so the accumulated result is exact
    n, m, k = 300, 260, 6000
    print(f"case: accumulate ring {prec} {n}x{m}x{k}", flush=True)
    A, B = workloads.small_int_operands(n, m, k, seed=25)
    C0 = workloads.small_int_operands(n, 1, m, seed=26, lo=-1000, hi=1000)[0]
    Cd = dev(C0.astype(np.float32))
    C, res = ctx.semiring_mm(dev(A), dev(B), "ring", C=Cd, accumulate=True, precision=prec, p=256,
                             kcut_cost=1.0, return_result=True)
    assert res["n_kcuts"] > 0
    expect = C0.astype(np.int64) + oracle.ring_i64(A.astype(np.int64), B.astype(np.int64))
    assert np.array_equal(host(C).astype(np.int64), expect)


# ------------------------------------------------ streams and the checker

def test_calls_on_two_streams_share_the_workspace_safely(ctx):
    # both products cut k (temporary faces at the start of the context's
    # workspace); the second call, made on another stream with no host
    # synchronisation, must wait for the first one's faces to be folded
    print("case: k-cut calls on two streams", flush=True)
    A1, B1 = workloads.minplus_operands(384, 256, 6000, seed=31)
    A2, B2 = workloads.minplus_operands(256, 384, 6000, seed=32)
    d = [dev(x) for x in (A1, B1, A2, B2)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        with torch.cuda.stream(s1):
            C1, r1 = ctx.semiring_mm(d[0], d[1], "minplus", p=256, return_result=True)
        with torch.cuda.stream(s2):
            C2, r2 = ctx.semiring_mm(d[2], d[3], "minplus", p=256, return_result=True)
        assert r1["n_kcuts"] > 0 and r2["n_kcuts"] > 0
        outs.append((C1, C2))
    torch.cuda.synchronize()
    e1, e2 = oracle.minplus(A1, B1), oracle.minplus(A2, B2)
    for C1, C2 in outs:
        assert np.array_equal(C1.cpu().numpy(), e1)
        assert np.array_equal(C2.cpu().numpy(), e2)


def test_verify_reports_nan_as_infinite_error(ctx):
    print("case: float64 checker with a NaN in C", flush=True)
    A, B = workloads.ring_operands(64, 96, 300, seed=33)
    Ad, Bd = dev(A), dev(B)
    C = ctx.semiring_mm(Ad, Bd, "ring", precision="bf16x3")
    rows = torch.tensor([0, 5, 63], dtype=torch.int64)
    mrel, mabs, sd, sr = ctx.verify_rows(Ad, Bd, C, rows)
    assert 0 < mrel <= 2.0 ** -15 and math.isfinite(mabs)
    C[5, 17] = float("nan")
    mrel, mabs, sd, sr = ctx.verify_rows(Ad, Bd, C, rows)
    assert mrel == math.inf and mabs == math.inf
    C[5, 17] = float("inf")
    mrel, mabs, _, _ = ctx.verify_rows(Ad, Bd, C, rows)
    assert mrel == math.inf and mabs == math.inf
    # a NaN outside the sampled rows is not seen
    C[5, 17] = 0.0
    C[6, 3] = float("nan")
    mrel, _, _, _ = ctx.verify_rows(Ad, Bd, C, rows)
    assert math.isfinite(mrel)
