"""Host logic: the pruned-BFS schedule of PACO Strassen (section "PACO
Strassen" and corollary Strassen-Const-Pieces), pinned to the statements the
paper makes about it rather than to the rule that generates it."""
import math

import pytest

import paper_2011_01441_amd as P  # noqa: E402

OMEGA = math.log2(7)
BIG = 1 << 30          # deep enough that node size never stops the schedule


def ceil_log7(x):
    d, v = 0, 1
    while v < x:
        v *= 7
        d += 1
    return d


@pytest.mark.parametrize("p", list(range(1, 60)) + [100, 255, 256, 343, 344, 1000, 2400, 2401, 2402])
def test_first_assignment_depth_and_at_most_six_cubes(p):
    # after the first ceil(log7 p) rounds of 7-way branching every processor
    # gets the same number of same-sized cubes, at most 6
    levels, _, _ = P.strassen_schedule(BIG, p, 0, 1)
    first = next(lv for lv in levels if lv["assigned"] > 0)
    assert first["depth"] == ceil_log7(p)
    assert first["assigned"] % p == 0 or first is levels[-1]
    assert 1 <= first["assigned"] // p <= 6


@pytest.mark.parametrize("p", [p for p in range(2, 2402) if 7 ** ceil_log7(p) < 2 * p and 7 ** ceil_log7(p) != p][::7])
def test_second_super_round_depth(p):
    # with 7^i1 < 2p exactly p cubes go out first, and the next assignment
    # comes ceil(log7(p / (7^i1 - p))) rounds later
    levels, _, _ = P.strassen_schedule(BIG, p, 0, 1)
    supers = [lv["depth"] for lv in levels if lv["super_round"]]
    i1 = ceil_log7(p)
    assert supers[0] == i1
    # ceil(log7 x) for real x is the least d with 7^d >= ceil(x)
    assert supers[1] - i1 == ceil_log7(math.ceil(p / (7 ** i1 - p)))


@pytest.mark.parametrize("gamma", [1, 2, 3, 4, 6, 8])
def test_const_pieces_imbalance_bound(gamma):
    # f_comp <= 1 - 2^(gamma-1) / (2^(gamma-1) + 1), in Strassen work h^omega
    bound = 1 - 2 ** (gamma - 1) / (2 ** (gamma - 1) + 1)
    for p in list(range(2, 70)) + [100, 200, 255, 256, 257, 500, 1000]:
        _, _, ws = P.strassen_schedule(BIG, p, gamma, 1)
        f = (ws.max() - ws.min()) / ws.max()
        assert f <= bound + 1e-12, (p, gamma, f, bound)
    if gamma == 8:
        assert bound < 0.01   # "less than 1%"


@pytest.mark.parametrize("n,p,gamma,base", [(16384, 256, 0, 256), (16384, 8, 0, 256), (4096, 3, 2, 64),
                                            (1 << 20, 5, 0, 1), (1000, 8, 0, 1), (2048, 1, 0, 64)])
def test_strassen_work_is_conserved(n, p, gamma, base):
    # a divided node passes its whole h^omega to its 7 children, so the
    # processors' Strassen work sums to n^omega however deep the tree goes
    levels, wc, ws = P.strassen_schedule(n, p, gamma, base)
    assert math.isclose(ws.sum(), n ** OMEGA, rel_tol=1e-9)
    assert levels[-1]["assigned"] == levels[-1]["nodes"]
    for a, b in zip(levels, levels[1:]):
        assert b["nodes"] == 7 * (a["nodes"] - a["assigned"]) and b["h"] * 2 == a["h"]


def test_c3_schedules():
    # the 16384^2 workload: one processor per compute unit and one per XCD
    levels, wc, _ = P.strassen_schedule(16384, 256, 0, 256)
    assert [(lv["nodes"], lv["assigned"]) for lv in levels[3:]] == [(343, 256), (609, 512), (679, 512),
                                                                   (1169, 1169)]
    assert wc.max() / wc.min() < 1.002
    levels, wc, _ = P.strassen_schedule(16384, 8, 0, 256)
    assert [(lv["nodes"], lv["assigned"]) for lv in levels[2:]] == [(49, 48), (7, 0), (49, 48), (7, 0),
                                                                   (49, 49)]


def test_base_and_odd_sizes_stop_division():
    levels, _, _ = P.strassen_schedule(1000, 8, 0, 1)        # 1000 -> 500 -> 250 -> 125 (odd)
    assert levels[-1]["h"] == 125 and levels[-1]["assigned"] == levels[-1]["nodes"]
    levels, _, _ = P.strassen_schedule(4096, 256, 0, 2048)   # nothing may go below 2048
    assert [lv["h"] for lv in levels] == [4096, 2048]
    levels, _, _ = P.strassen_schedule(4096, 1, 0, 1)         # one processor runs the root
    assert len(levels) == 1 and levels[0]["assigned"] == 1
