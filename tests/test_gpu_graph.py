"""Captured calls (paco_graph_*): every replay checked against the eager /
oracle result, with eager work and synchronisations between the replays."""
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


def test_minplus_graph_replays(ctx):
    print("case: graph minplus 384x320x256 (k-cut reduction in the graph)", flush=True)
    A, B = workloads.minplus_operands(384, 256, 320, seed=21)
    expect = oracle.minplus(A, B)
    Ad, Bd = dev(A), dev(B)
    Cg = torch.empty((384, 256), dtype=torch.int32, device=DEV)
    g = ctx.graph(Ad, Bd, "minplus", C=Cg)
    assert np.array_equal(host(Cg), expect)          # the eager warm-up call
    X, Y = dev(workloads.minplus_operands(100, 90, 80, seed=3)[0]), None
    for rep in range(4):
        Cg.fill_(-1)                                  # eager work between replays
        Y = ctx.semiring_mm(X, X[:80, :].contiguous(), "minplus")
        torch.cuda.synchronize()
        g.launch()
        assert np.array_equal(host(Cg), expect), rep
    g.close()


def test_ring_graph_replays_bitwise_and_reads_inputs_at_replay(ctx):
    print("case: graph ring 256x256x8192 bf16x3 (k-cuts)", flush=True)
    A, B = workloads.ring_operands(256, 256, 8192, seed=22)
    Ad, Bd = dev(A), dev(B)
    Ce = ctx.semiring_mm(Ad, Bd, "ring", precision="bf16x3")
    eager = host(Ce).copy()
    Cg = torch.empty_like(Ce)
    g = ctx.graph(Ad, Bd, "ring", C=Cg, precision="bf16x3")
    for rep in range(4):
        Cg.zero_()
        torch.cuda.synchronize()
        g.launch()
        assert np.array_equal(host(Cg), eager), rep   # same plan, same order: same bits
    # the replay reads the buffers as they are now
    A2, _ = workloads.ring_operands(256, 256, 8192, seed=23)
    Ad.copy_(dev(A2))
    torch.cuda.synchronize()
    g.launch()
    C2 = host(Cg).astype(np.float64)
    C64, S = oracle.ring_f64(A2, B, with_abs=True)
    assert np.max(np.abs(C2 - C64) / S) <= 2.0 ** -20
    g.close()


def test_strassen_graph_replays(ctx):
    print("case: graph strassen pbfs n=512", flush=True)
    A, B = workloads.small_int_operands(512, 512, 512, seed=24)
    expect = oracle.ring_i64(A.astype(np.int64), B.astype(np.int64))
    Ad, Bd = dev(A), dev(B)
    Cg = torch.empty((512, 512), device=DEV)
    g = ctx.graph_strassen(Ad, Bd, Cg, p=8, base=64)
    for rep in range(3):
        Cg.fill_(7.0)
        ctx.semiring_mm(Ad, Bd, "ring", precision="fp32")   # eager work on the same context
        torch.cuda.synchronize()
        g.launch()
        assert np.array_equal(host(Cg).astype(np.int64), expect), rep
    g.close()


def test_stale_graph_is_refused():
    print("case: graph stale after workspace growth", flush=True)
    c = P.Context(0)
    try:
        A, B = workloads.minplus_operands(384, 256, 320, seed=25)
        Cg = torch.empty((384, 256), dtype=torch.int32, device=DEV)
        g = c.graph(dev(A), dev(B), "minplus", C=Cg)
        # a call with far larger temporary faces (1024 processors on a long k:
        # 16 output tiles, each cut 64-way in k) grows and so reallocates the
        # workspace
        X = torch.randn(1024, 65536, device=DEV)
        Y = torch.randn(65536, 1024, device=DEV)
        _, r = c.semiring_mm(X, Y, "ring", precision="bf16x3", p=1024, return_result=True)
        assert r["temp_elems"] * 4 > 64 << 20
        torch.cuda.synchronize()
        with pytest.raises(Exception):
            g.launch()
        g.close()
    finally:
        c.close()


def test_plan_cache_is_bounded():
    # 520 call shapes overflow the 512-plan cache: every result stays exact,
    # and a graph captured before the cache was dropped refuses to replay
    print("case: plan cache bound", flush=True)
    c = P.Context(0)
    try:
        A, B = workloads.minplus_operands(40, 24, 16, seed=26)
        Cg = torch.empty((40, 24), dtype=torch.int32, device=DEV)
        g = c.graph(dev(A), dev(B), "minplus", C=Cg)
        g.launch()
        assert np.array_equal(host(Cg), oracle.minplus(A, B))
        Bd = dev(B)
        for n in range(1, 521):
            An = dev(A[:n % 40 + 1]) if n <= 40 else dev(np.resize(A, (n, 16)).astype(np.int32))
            C = c.semiring_mm(An, Bd, "minplus")
            if n % 97 == 0 or n == 520:
                assert np.array_equal(host(C), oracle.minplus(host(An), B))
        with pytest.raises(Exception):
            g.launch()
        g.close()
        C = c.semiring_mm(dev(A), Bd, "minplus")
        assert np.array_equal(host(C), oracle.minplus(A, B))
    finally:
        c.close()


# ------------------------------------------------------------ autotuner

@pytest.mark.parametrize("sr", ["minplus", "ring"])
def test_tune_then_default_calls_stay_exact(ctx, sr):
    print(f"case: tune {sr}", flush=True)
    if sr == "minplus":
        A, B = workloads.minplus_operands(384, 256, 320, seed=26)
        expect = oracle.minplus(A, B)
        C = torch.empty((384, 256), dtype=torch.int32, device=DEV)
        kw = {}
    else:
        A, B = workloads.small_int_operands(700, 600, 3000, seed=27)
        expect = A.astype(np.int64) @ B.astype(np.int64)
        C = torch.empty((700, 600), device=DEV)
        kw = {"precision": "bf16x3"}
    Ad, Bd = dev(A), dev(B)
    r = ctx.tune(Ad, Bd, sr, C=C, **kw)
    assert r["candidates"] > 4 and r["best_ms"] <= r["default_ms"] + 1e-9
    C2, res = ctx.semiring_mm(Ad, Bd, sr, return_result=True, **kw)
    got = host(C2)
    assert np.array_equal(got.astype(np.int64) if sr == "ring" else got, expect)
    if r["tuned"]:
        assert res["p"] == r["p"] and res["kcut_cost"] == r["kcut_cost"]
    ctx.tune_clear()


def test_graph_repeat_runs_every_call(ctx):
    # accumulate mode makes every captured run visible: C = C0 + r * A B
    print("case: graph repeat=5 ring accumulate", flush=True)
    A, B = workloads.small_int_operands(300, 200, 700, seed=28)
    AB = A.astype(np.int64) @ B.astype(np.int64)
    Ad, Bd = dev(A), dev(B)
    C = torch.zeros((300, 200), device=DEV)
    g = ctx.graph(Ad, Bd, "ring", C=C, precision="bf16x3", accumulate=True, repeat=5)
    # the eager warm-up call accumulated once
    assert np.array_equal(host(C).astype(np.int64), AB)
    for rep in range(2):
        C.zero_()
        torch.cuda.synchronize()
        g.launch()
        assert np.array_equal(host(C).astype(np.int64), 5 * AB), rep
    g.close()
