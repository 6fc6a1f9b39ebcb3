"""Fused folding of temporary faces (the product kernel's last piece to
finish a reduction cell folds it) against the oracle and against the
separate fold launch.  Both fold each cell in the same order, so even float
results are bit-identical; counters reset themselves, so repeated calls and
graph replays stay exact."""
import os

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


@pytest.fixture
def fuse():
    old = os.environ.get("PACO_FUSE_FOLD")

    def set_(v):
        os.environ["PACO_FUSE_FOLD"] = v
    yield set_
    if old is None:
        os.environ.pop("PACO_FUSE_FOLD", None)
    else:
        os.environ["PACO_FUSE_FOLD"] = old


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [("minplus", 384, 256, 320, 0), ("minplus", 97, 130, 75, 0), ("maxplus", 257, 65, 900, 64),
         ("minplus", 70, 50, 3000, 37), ("bool", 96, 200, 9000, 256), ("ring", 300, 260, 6000, 256),
         ("ring", 130, 70, 1000, 97)]


def operands(sr, n, m, k, seed):
    if sr == "minplus":
        A, B = workloads.minplus_operands(n, m, k, seed=seed)
        return A, B, oracle.minplus(A, B), {}
    if sr == "maxplus":
        A, B = workloads.maxplus_operands(n, m, k, seed=seed)
        return A, B, oracle.maxplus(A, B), {}
    if sr == "bool":
        _, _, ap, bp = workloads.bool_operands(n, m, k, density=0.0005, seed=seed)
        return (ap.view(np.int32), bp.view(np.int32), oracle.bool_packed(ap, bp, n, m, k).view(np.int32),
                dict(n=n, m=m, k=k))
    A, B = workloads.small_int_operands(n, m, k, seed=seed)
    return A, B, oracle.ring_f64(A, B).astype(np.float32), dict(precision="bf16x3")


@pytest.mark.parametrize("sr,n,m,k,p", CASES)
def test_fused_matches_oracle_and_separate_fold(ctx, fuse, sr, n, m, k, p):
    print(f"case: fused fold {sr} {n}x{m}x{k} p={p}", flush=True)
    A, B, ref, kw = operands(sr, n, m, k, seed=n + m + k)
    Ad, Bd = dev(A), dev(B)
    fuse("0")
    C0, r0 = ctx.semiring_mm(Ad, Bd, sr, p=p, return_result=True, **kw)
    base = host(C0)
    fuse("1")
    outs = []
    for _ in range(3):   # counters left at zero by each call
        C1, r1 = ctx.semiring_mm(Ad, Bd, sr, p=p, return_result=True, **kw)
        outs.append(host(C1))
    assert r1["n_kcuts"] > 0 and r1["n_kcuts"] == r0["n_kcuts"]
    assert np.array_equal(base, ref)
    for o in outs:
        assert np.array_equal(o.view(np.uint32), base.view(np.uint32))


def test_fused_accumulate_and_graph(ctx, fuse):
    n, m, k = 384, 256, 320
    print("case: fused fold accumulate + graph replays", flush=True)
    fuse("1")
    A, B = workloads.minplus_operands(n, m, k, seed=41)
    C0 = workloads.minplus_operands(n, 1, m, seed=42)[0]
    Cd = dev(C0)
    C, r = ctx.semiring_mm(dev(A), dev(B), "minplus", C=Cd, accumulate=True, return_result=True)
    assert r["n_kcuts"] > 0
    assert np.array_equal(host(C), oracle.minplus(A, B, C=C0))
    Cg = torch.empty((n, m), dtype=torch.int32, device=DEV)
    Ad, Bd = dev(A), dev(B)
    g = ctx.graph(Ad, Bd, "minplus", C=Cg, repeat=2)
    expect = oracle.minplus(A, B)
    for rep in range(4):
        Cg.fill_(0)
        ctx.semiring_mm(Ad, Bd, "minplus")   # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        assert np.array_equal(host(Cg), expect), rep
    g.close()


def test_fused_noalloc(ctx, fuse):
    """The allocation-free entry point carries the fold counters in its
    scratch, zeroed with the plan tables at every call."""
    fuse("1")
    for (n, m, k) in ((384, 256, 320), (97, 130, 75)):
        print(f"case: fused fold noalloc minplus {n}x{m}x{k}", flush=True)
        A, B = workloads.minplus_operands(n, m, k, seed=n)
        C = torch.full((n, m), 5, dtype=torch.int32, device=DEV)
        ctx.semiring_mm_noalloc(dev(A), dev(B), "minplus", C=C)
        assert np.array_equal(host(C), oracle.minplus(A, B))
