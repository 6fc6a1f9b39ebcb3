"""PACO partitioner (host C++ through the C ABI) against the paper's pins:
the pruned-BFS figure, exactly-p assignment per round, disjoint cover,
balance for arbitrary (prime) p, the largest-piece volume of theorem mm, the
MM-1-Piece dimension bound of its corollary, the heterogeneous ratio split,
quanta and the k-cut cost option."""
import json
import math
import os

import numpy as np
import pytest

import paper_2011_01441_amd as P  # noqa: E402
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _vol(pc):
    return (pc["n1"] - pc["n0"]) * (pc["m1"] - pc["m0"]) * (pc["k1"] - pc["k0"])


def _cover(pcs, n, m, k):
    cube = np.zeros((n, m, k), np.int16)
    for pc in pcs:
        cube[pc["n0"]:pc["n1"], pc["m0"]:pc["m1"], pc["k0"]:pc["k1"]] += 1
    return cube


def _path(pc, size):
    # cube with ties n, m, k: depth i cuts dimension i % 3
    lo = [pc["n0"], pc["m0"], pc["k0"]]
    out = ""
    cnt = [0, 0, 0]
    for i in range(pc["depth"]):
        d = i % 3
        half = size >> (cnt[d] + 1)
        out += "R" if (lo[d] // half) % 2 else "L"
        cnt[d] += 1
    return out


def test_pruned_bfs_figure_p3():
    g = json.load(open(os.path.join(GOLD, "pruned_bfs_p3.json")))
    pcs = P.partition(64, 64, 64, g["p"], multi_piece=True)
    got = {}
    for pc in pcs:
        if pc["round"] < 2:
            got[_path(pc, 64)] = pc["round"] + 1
    assert got == g["assigned"]
    # processors get the first p nodes of a round in BFS (left-to-right) order
    r0 = sorted((pc for pc in pcs if pc["round"] == 0), key=lambda pc: pc["proc"])
    assert [_path(pc, 64) for pc in r0] == ["LL", "LR", "RL"]
    later = {_path(pc, 64)[:4] for pc in pcs if pc["round"] >= 2}
    assert set(g["continues_after_round_2"]) <= later


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 31, 64, 127])
def test_multi_piece_rounds_and_cover(p):
    n, m, k = 48, 40, 36
    pcs = P.partition(n, m, k, p, multi_piece=True)
    assert (_cover(pcs, n, m, k) == 1).all()
    rounds = {}
    for pc in pcs:
        rounds.setdefault(pc["round"], []).append(pc)
    last = max(rounds)
    for r, lst in rounds.items():
        if r < last:
            assert sorted(pc["proc"] for pc in lst) == list(range(p)), "exactly p per round"
        else:
            assert len(lst) <= 2 * p   # base cases dealt round-robin
    # no processor holds two cuboids of the same depth (theorem mm)
    for q in range(p):
        depths = [pc["depth"] for pc in pcs if pc["proc"] == q and pc["round"] < last]
        assert len(depths) == len(set(depths))


@pytest.mark.parametrize("p", [2, 4, 8, 16, 32, 64, 128, 256])
def test_multi_piece_largest_volume_is_V_over_2_ceil_log2_p(p):
    n = m = k = 256
    pcs = P.partition(n, m, k, p, multi_piece=True)
    V = n * m * k
    for q in range(p):
        vmax = max(_vol(pc) for pc in pcs if pc["proc"] == q)
        assert vmax == V // 2 ** math.ceil(math.log2(p))


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 31, 127, 251, 255, 256, 257])
def test_mm1_piece_exactly_one_cuboid_per_processor(p):
    n, m, k = 300, 200, 500
    pcs = P.partition(n, m, k, p)
    assert len(pcs) == p and sorted(pc["proc"] for pc in pcs) == list(range(p))
    assert (_cover(pcs, n, m, k) == 1).all()
    vols = np.array([_vol(pc) for pc in pcs])
    # balance: floor(p/2):ceil(p/2) ratio cuts keep every volume near V/p
    assert vols.max() <= 1.25 * n * m * k / p + (n * m + m * k + n * k)


@pytest.mark.parametrize("p", [3, 5, 7, 11, 13, 127, 251])
def test_mm1_piece_dimensions_within_constant_of_virtual(p):
    # corollary mm-1-piece: every dimension stays within a constant factor of
    # the even (virtual) split's; the worst right-branch shrink is
    # prod (2^i + 1) / (2^(i+1) + 1) = Theta(1/p)
    n, m, k = 4096, 2048, 1024
    pcs = P.partition(n, m, k, p)
    L = math.ceil(math.log2(p))
    vol_even = n * m * k / 2 ** L
    for pc in pcs:
        assert _vol(pc) <= 2.0 * vol_even * (2 ** L / p) * 2
        assert _vol(pc) >= 0.25 * n * m * k / p


def test_mm1_piece_power_of_two_is_even():
    pcs = P.partition(1024, 512, 256, 256)
    assert {_vol(pc) for pc in pcs} == {1024 * 512 * 256 // 256}


def test_heterogeneous_weights_give_proportional_volumes():
    w = [1.0] * 6 + [3.0] * 2          # two processors three times faster
    pcs = P.partition(960, 960, 960, 8, weights=w)
    assert (_cover(pcs, 960, 960, 960) == 1).all()
    V = 960 ** 3
    for pc in pcs:
        share = w[pc["proc"]] / sum(w)
        assert abs(_vol(pc) / V - share) < 0.02


def test_quanta_put_cuts_on_multiples():
    pcs = P.partition(1000, 999, 777, 37, q=(16, 32, 8))
    for pc in pcs:
        assert pc["n0"] % 16 == 0 and (pc["n1"] % 16 == 0 or pc["n1"] == 1000)
        assert pc["m0"] % 32 == 0 and (pc["m1"] % 32 == 0 or pc["m1"] == 999)
        assert pc["k0"] % 8 == 0 and (pc["k1"] % 8 == 0 or pc["k1"] == 777)


def test_kcut_cost_option():
    base = P.partition(2048, 1024, 65536, 256)
    assert {pc["k1"] - pc["k0"] for pc in base} == {1024}          # the paper's rule
    heavy = P.partition(2048, 1024, 65536, 256, kcut_cost=1e9)
    assert {pc["k1"] - pc["k0"] for pc in heavy} == {65536}         # n, m cuts only
    assert all(pc["temp"] == 0 for pc in heavy)


def test_temp_flags_follow_k0():
    for pc in P.partition(64, 64, 4096, 64):
        assert pc["temp"] == (1 if pc["k0"] > 0 else 0)


@pytest.mark.parametrize("p,rounds", [(3, 1), (3, 2), (200, 2), (251, 4), (256, 1)])
def test_multi_piece_round_cap(p, rounds):
    """max_rounds: rounds of exactly p pieces, then every remaining cuboid
    round-robin; the pieces still tile the cuboid."""
    n, m, k = 512, 384, 640
    pcs = P.partition(n, m, k, p, multi_piece=True, max_rounds=rounds)
    vol = sum((q["n1"] - q["n0"]) * (q["m1"] - q["m0"]) * (q["k1"] - q["k0"]) for q in pcs)
    assert vol == n * m * k
    by_round = {}
    for q in pcs:
        by_round.setdefault(q["round"], []).append(q)
    full = sorted(r for r in by_round if r < rounds)
    for r in full:
        assert len(by_round[r]) == p and sorted(q["proc"] for q in by_round[r]) == list(range(p))
    assert max(by_round) <= rounds
