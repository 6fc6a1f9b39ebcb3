"""GPU parity at the workloads' full sizes, in the launch configuration
bench.py times (default PACO call), checked on sampled output rows that the
oracle computes one by one: bit-exact for the integer and boolean semirings,
max |C - C64| / (|A||B|) <= 2^-20 for the ring, normwise <= 2^-16 for
Strassen."""
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


def sample_rows(n, count, seed):
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, count)]))
    return rows


def test_c1_ring_longk_sampled(ctx):
    print("case: C1 2048x65536x1024 bf16x3 and fp32, sampled rows", flush=True)
    A, B = workloads.ring_operands(2048, 1024, 65536, seed=0)
    Ad, Bd = dev(A), dev(B)
    rows = sample_rows(2048, 14, 1)
    C64, S = oracle.ring_f64(A, B, rows=rows, with_abs=True)
    for prec in ("bf16x3", "fp32"):
        C = ctx.semiring_mm(Ad, Bd, "ring", precision=prec)
        Cr = C[torch.from_numpy(rows).to(DEV)].cpu().numpy().astype(np.float64)
        err = np.max(np.abs(Cr - C64) / S)
        print(f"  {prec}: max rel 2^{math.log2(err):.1f}", flush=True)
        assert err <= 2.0 ** -20, (prec, err)


def test_c2a_maxplus_full_sampled(ctx):
    print("case: C2a (max,+) 131072x512x64, sampled rows", flush=True)
    A, B = workloads.maxplus_operands(131072, 64, 512, seed=0)
    C = ctx.semiring_mm(dev(A), dev(B), "maxplus")
    rows = sample_rows(131072, 200, 2)
    got = C[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert np.array_equal(got, oracle.maxplus(A[rows], B))


@pytest.mark.parametrize("density", [0.05, 0.0092])
def test_c2b_bool_full_sampled(ctx, density):
    # 0.05 is the workload (C is almost all ones); 0.0092 gives about half
    # ones, so the check is not vacuous
    print(f"case: C2b boolean 8192^3 bits density {density}, sampled rows", flush=True)
    n = m = k = 8192
    ap, bp = workloads.bool_operands_packed(n, m, k, density=density)
    Cw = ctx.semiring_mm(dev(ap.view(np.int32)), dev(bp.view(np.int32)), "bool", n=n, m=m, k=k)
    rows = sample_rows(n, 100, 3)
    got = Cw[torch.from_numpy(rows).to(DEV)].cpu().numpy().view(np.uint32)
    expect = oracle.bool_packed(ap[rows], bp, len(rows), m, k)
    assert np.array_equal(got, expect)
    if density < 0.01:
        ones = np.unpackbits(expect.view(np.uint8)).mean()
        assert 0.2 < ones < 0.8


def test_minplus_8192_sampled(ctx):
    print("case: (min,+) 8192^3, sampled rows", flush=True)
    A, B = workloads.minplus_operands(8192, 8192, 8192, seed=0)
    C, res = ctx.semiring_mm(dev(A), dev(B), "minplus", return_result=True)
    rows = sample_rows(8192, 30, 4)
    got = C[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert np.array_equal(got, oracle.minplus(A[rows], B))
    assert res["p"] % 256 == 0


def test_c3_strassen_pbfs_sampled(ctx):
    print("case: C3 PACO Strassen 16384^2 p=8 bf16x3, sampled rows", flush=True)
    n = 16384
    A, B = workloads.strassen_operands(n, seed=0)
    Ad, Bd = dev(A), dev(B)
    C = ctx.strassen_pbfs(Ad, Bd, p=8, leaf="bf16x3")
    rows = sample_rows(n, 10, 5)
    C64 = oracle.ring_f64(A, B, rows=rows)
    Cr = C[torch.from_numpy(rows).to(DEV)].cpu().numpy().astype(np.float64)
    # normwise ||C - C64||_F / (||A||_F ||B||_F), numerator extrapolated from the rows
    num = math.sqrt(np.sum((Cr - C64) ** 2) * n / len(rows))
    den = float(np.linalg.norm(A.astype(np.float64))) * float(np.linalg.norm(B.astype(np.float64)))
    print(f"  normwise 2^{math.log2(num / den):.1f}", flush=True)
    assert num / den <= 2.0 ** -16


@pytest.mark.parametrize("p", [97, 200, 251])
def test_c1_arbitrary_p_sampled(ctx, p):
    """C1 over a prime and other non-power-of-two processor counts: the
    tile-grid MM-1-Piece plan (its k-cuts and faces differ from p = 256)
    stays within the bound on rows the oracle computes one by one."""
    print(f"case: C1 bf16x3 p={p}, sampled rows", flush=True)
    A, B = workloads.ring_operands(2048, 1024, 65536, seed=0)
    Ad, Bd = dev(A), dev(B)
    rows = sample_rows(2048, 6, p)
    C64, S = oracle.ring_f64(A, B, rows=rows, with_abs=True)
    C, res = ctx.semiring_mm(Ad, Bd, "ring", precision="bf16x3", p=p, return_result=True)
    assert res["p"] == p and res["n_pieces"] <= p
    Cr = C[torch.from_numpy(rows).to(DEV)].cpu().numpy().astype(np.float64)
    err = np.max(np.abs(Cr - C64) / S)
    print(f"  max rel 2^{math.log2(err):.1f}, faces {res['n_kcuts']}", flush=True)
    assert err <= 2.0 ** -20


@pytest.mark.parametrize("p", [7, 97, 200, 251])
def test_ring_arbitrary_p_small_integers_exact(ctx, p):
    """Small integers make every partial sum exact: at any p the tile-grid
    plan (ragged sizes, k-cuts, faces folded in ascending k) gives the
    oracle's result bit for bit."""
    n, m, k = 700, 530, 3000
    print(f"case: ring small integers {n}x{m}x{k} p={p}", flush=True)
    A, B = workloads.small_int_operands(n, m, k, seed=p)
    for prec in ("bf16x3", "fp32"):
        C = ctx.semiring_mm(dev(A), dev(B), "ring", precision=prec, p=p)
        assert np.array_equal(C.cpu().numpy().astype(np.float64), oracle.ring_f64(A, B)), prec
