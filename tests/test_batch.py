"""Host logic of the request server: the processor split over a batch.

Every request's cuboid must be covered exactly once by its pieces, pieces
of one request must sit on processors of one contiguous range, and the
work per processor must be balanced to within the largest single request
share (requests smaller than one processor's share run whole)."""
import collections

import numpy as np
import pytest

import paper_2011_01441_amd as P  # noqa: E402


def _reqs(count, seed, lo=32, hi=4096):
    r = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n, m, k = np.exp(r.uniform(np.log(lo), np.log(hi), 3)).astype(int)
        out.append(dict(n=int(n), m=int(m), k=int(k),
                        semiring="ring" if r.random() < 0.7 else "minplus"))
    return out


def _cover_check(reqs, pieces):
    vol = collections.Counter()
    for pc in pieces:
        assert pc["n1"] > pc["n0"] and pc["m1"] > pc["m0"] and pc["k1"] > pc["k0"]
        vol[pc["req"]] += (pc["n1"] - pc["n0"]) * (pc["m1"] - pc["m0"]) * (pc["k1"] - pc["k0"])
    for i, r in enumerate(reqs):
        assert vol[i] == r["n"] * r["m"] * r["k"], f"request {i} not covered exactly"


@pytest.mark.parametrize("count,p", [(1, 256), (7, 256), (64, 256), (500, 256), (300, 17)])
def test_batch_cover_and_processor_ranges(count, p):
    reqs = _reqs(count, seed=count)
    pieces = P.batch_partition(reqs, p)
    _cover_check(reqs, pieces)
    procs = collections.defaultdict(set)
    for pc in pieces:
        procs[pc["req"]].add(pc["proc"])
    for i, s in procs.items():
        assert max(s) - min(s) + 1 == len(s) or len(s) == 1, "a request's processors must be contiguous"


def test_batch_pieces_do_not_overlap_within_a_request():
    reqs = [dict(n=300, m=200, k=1000, semiring="ring"), dict(n=64, m=64, k=64, semiring="minplus")]
    pieces = P.batch_partition(reqs, 64)
    for i, r in enumerate(reqs):
        cube = np.zeros((r["n"], r["m"], r["k"]), np.int8)
        for pc in pieces:
            if pc["req"] == i:
                cube[pc["n0"]:pc["n1"], pc["m0"]:pc["m1"], pc["k0"]:pc["k1"]] += 1
        assert (cube == 1).all()


def test_single_large_request_gets_all_processors_like_mm1piece():
    # a ring request alone gets every processor and the library call's plan:
    # MM-1-Piece on the 256 x 256 tile grid, one output tile 8192 deep each
    pieces = P.batch_partition([dict(n=2048, m=1024, k=65536, semiring="ring",
                                     precision="bf16x3")], 256)
    assert len(pieces) == 256 and len({pc["proc"] for pc in pieces}) == 256
    ext = {(pc["n1"] - pc["n0"], pc["m1"] - pc["m0"], pc["k1"] - pc["k0"]) for pc in pieces}
    assert ext == {(256, 256, 8192)}
    items, *_ = P.plan_export(2048, 1024, 65536, "ring", p=256, precision="bf16x3")
    assert ext == {tuple(e) for e in (items[:, [2, 4, 6]] - items[:, [1, 3, 5]]).tolist()}


def test_single_integer_request_keeps_the_paper_rule(monkeypatch):
    monkeypatch.setenv("PACO_KCUT_COST", "1")   # the paper's longest-dimension rule
    pieces = P.batch_partition([dict(n=2048, m=1024, k=65536, semiring="minplus")], 256)
    ext = {(pc["n1"] - pc["n0"], pc["m1"] - pc["m0"], pc["k1"] - pc["k0"]) for pc in pieces}
    assert ext == {(512, 1024, 1024)}


def test_batch_balance_of_equal_requests():
    reqs = [dict(n=512, m=512, k=512, semiring="ring", precision="bf16x3")] * 64
    pieces = P.batch_partition(reqs, 256)
    load = collections.Counter()
    for pc in pieces:
        load[pc["proc"]] += (pc["n1"] - pc["n0"]) * (pc["m1"] - pc["m0"]) * (pc["k1"] - pc["k0"])
    v = np.array(list(load.values()))
    assert len(v) == 256 and v.max() <= 1.05 * v.mean()
