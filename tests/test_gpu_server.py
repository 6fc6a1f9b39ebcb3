"""GPU: the batching request server against the CPU oracle.

Requests are views into resident operand pools (as a serving system keeps
operands in HBM); every result is compared with the oracle: (min,+)
bit-exact, ring within the componentwise bound."""
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


@pytest.fixture(scope="module")
def pools():
    ra, rb = workloads.ring_operands(700, 700, 700, seed=5)
    ma, mb = workloads.minplus_operands(700, 700, 700, seed=6)
    return dict(ring=(ra, rb, torch.from_numpy(ra).to(DEV), torch.from_numpy(rb).to(DEV)),
                minplus=(ma, mb, torch.from_numpy(ma).to(DEV), torch.from_numpy(mb).to(DEV)))


def _run(srv, pools, shapes):
    out = []
    for i, (kind, n, m, k) in enumerate(shapes):
        a, b, ad, bd = pools[kind]
        C = torch.empty((n, m), dtype=ad.dtype, device=DEV)
        t = srv.submit(ad[:n, :k], bd[:k, :m], C, kind)
        out.append((t, kind, n, m, k, C))
    srv.drain()
    return out


def _check(pools, srv, runs):
    torch.cuda.synchronize()
    for t, kind, n, m, k, C in runs:
        done, res = srv.poll(t)
        assert done and res["status"] == 0, res
        a, b = pools[kind][0][:n, :k], pools[kind][1][:k, :m]
        got = C.cpu().numpy()
        if kind == "minplus":
            assert np.array_equal(got, oracle.minplus(a, b)), (n, m, k)
        else:
            C64, S = oracle.ring_f64(a, b, with_abs=True)
            err = np.max(np.abs(got - C64) / S)
            assert err <= 2.0 ** -20, (n, m, k, res["precision"], np.log2(err))


SHAPES = [("ring", 33, 47, 65), ("minplus", 100, 300, 50), ("ring", 640, 512, 700),
          ("minplus", 1, 1, 1), ("ring", 129, 3, 333), ("minplus", 512, 640, 256),
          ("ring", 64, 64, 64), ("minplus", 77, 91, 700)] * 3


@pytest.mark.parametrize("per_request,spin_s", [(False, 0.0), (True, 0.0), (False, 0.002)])
def test_server_mixed_batch_matches_oracle(ctx, pools, per_request, spin_s):
    print(f"case: server per_request={per_request} spin_s={spin_s}", flush=True)
    srv = P.Server(ctx, per_request=per_request, spin_s=spin_s)
    runs = _run(srv, pools, SHAPES)
    _check(pools, srv, runs)
    st = srv.stats()
    assert st["completed"] == len(SHAPES) and st["failed"] == 0
    if per_request:
        assert st["batches"] == len(SHAPES)
    srv.close()


def test_server_small_budget_queues_and_rejects(ctx, pools):
    print("case: server admission budget", flush=True)
    budget = 3 * 4 * 640 * 700    # about one large request at a time
    srv = P.Server(ctx, hbm_budget=budget)
    runs = _run(srv, pools, SHAPES[:8])
    _check(pools, srv, runs)
    a, b, ad, bd = pools["ring"]
    C = torch.empty((700, 700), device=DEV)
    with pytest.raises(P.PacoError) as ei:
        srv.submit(ad, bd, C, "ring")
    assert ei.value.status == 4     # PACO_ERR_BUDGET
    srv.close()


def test_server_failed_batch_releases_budget(ctx, pools):
    # the failure path: a batch that fails before launch fails only its own
    # requests, returns their bytes to the admission budget, and the
    # requests after it complete and match the oracle
    print("case: server failed batch", flush=True)
    srv = P.Server(ctx)
    srv.fail_batches(1)
    first = _run(srv, pools, SHAPES[:6])
    st = srv.stats()
    assert st["bytes_in_flight"] == 0
    failed = []
    for t, kind, n, m, k, C in first:
        done, res = srv.poll(t)
        assert done
        if res["status"] != 0:
            assert res["status"] == 6          # PACO_ERR_INTERNAL
            failed.append(res["batch_id"])
    assert failed and len(set(failed)) == 1    # exactly one batch failed, all of its requests
    assert st["failed"] == len(failed) and st["completed"] == 6 - len(failed)
    later = _run(srv, pools, SHAPES[6:14])
    _check(pools, srv, later)
    st = srv.stats()
    assert st["failed"] == len(failed) and st["completed"] == 14 - len(failed)
    assert st["bytes_in_flight"] == 0 and st["retained"] == 0
    srv.close()


def test_server_forgets_polled_requests(ctx, pools):
    # memory stays bounded: a request is dropped once it is reported done,
    # and the latency statistics live in a fixed-size histogram
    print("case: server retention", flush=True)
    srv = P.Server(ctx)
    a, b, ad, bd = pools["minplus"]
    C = torch.empty((8, 8), dtype=ad.dtype, device=DEV)
    lat = []
    for rnd in range(4):
        ts = [srv.submit(ad[:8, :8], bd[:8, :8], C, "minplus") for _ in range(500)]
        srv.drain()
        assert srv.stats()["retained"] == 500
        for t in ts:
            done, res = srv.poll(t)
            assert done and res["status"] == 0
            lat.append(res["done_s"] - res["arrival_s"])
        st = srv.stats()
        assert st["retained"] == 0
        with pytest.raises(P.PacoError) as ei:
            srv.poll(ts[0])
        assert ei.value.status == 7            # PACO_ERR_NOT_FOUND
    st = srv.stats()
    assert st["completed"] == 2000
    lat = np.sort(np.array(lat))
    for q, key in ((0.5, "p50_s"), (0.99, "p99_s")):
        exact = lat[min(len(lat) - 1, int(q * (len(lat) - 1) + 0.5))]
        assert abs(st[key] - exact) <= 0.003 * exact + 1e-7, (key, st[key], exact)
    assert st["max_s"] == pytest.approx(lat[-1])
    assert np.array_equal(C.cpu().numpy(), oracle.minplus(a[:8, :8], b[:8, :8]))
    srv.close()


def test_server_dispatch_paths(ctx, pools):
    """The ways a batch reaches the GPU, each checked against the oracle:
    a lone small request (one kernel group: the main stream, descriptors
    read from pinned host memory), a lone (min,+) request whose descriptors
    exceed 64 KiB (copied to device memory first), and one batch of both
    kinds (a stream per kernel group, joined by events)."""
    for shapes in ([("ring", 100, 100, 100)], [("minplus", 700, 700, 700)]):
        print(f"case: server lone request {shapes[0]}", flush=True)
        srv = P.Server(ctx)
        runs = _run(srv, pools, shapes)
        _check(pools, srv, runs)
        srv.close()
    print("case: server one mixed batch", flush=True)
    srv = P.Server(ctx, window_s=0.2)
    runs = _run(srv, pools, [("ring", 100, 100, 100), ("minplus", 700, 700, 700),
                             ("ring", 640, 512, 700), ("minplus", 33, 47, 65)])
    _check(pools, srv, runs)
    st = srv.stats()
    assert st["batches"] == 1 and st["completed"] == 4, st
    srv.close()


def test_server_rejects_negative_spin(ctx):
    with pytest.raises(P.PacoError):
        P.Server(ctx, spin_s=-1.0)
