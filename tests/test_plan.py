"""Host logic: the work plan libpaco launches, replayed on the CPU.

paco_plan_export returns the exact work items and reduction tiles a call
launches.  Replaying them with numpy -- each item folds its k-range into C
or into its temporary face, then every reduction tile folds its faces in
order -- must give the oracle's result, and the plan must cover every
(i, j, l) exactly once with disjoint writes (the paper's no-data-race
model)."""
import numpy as np
import pytest

import oracle
import workloads

import paper_2011_01441_amd as P  # noqa: E402
INF, NEG_INF = oracle.INF, oracle.NEG_INF


def _partial(sr, A, B, it):
    _, n0, n1, m0, m1, k0, k1, _ = it
    a = A[n0:n1, k0:k1].astype(np.int64)
    b = B[k0:k1, m0:m1].astype(np.int64)
    if sr == "minplus":
        return np.minimum(np.min(a[:, :, None] + b[None, :, :], axis=1), INF)
    if sr == "maxplus":
        s = a[:, :, None] + b[None, :, :]
        s = np.where((a[:, :, None] == NEG_INF) | (b[None, :, :] == NEG_INF), NEG_INF, s)
        return np.max(s, axis=1)
    return a @ b    # ring on small integers


def _fold(sr, x, y):
    return {"minplus": np.minimum, "maxplus": np.maximum}.get(sr, np.add)(x, y)


def replay(sr, A, B, n, m, k, **kw):
    items, wg, tiles, srcs, info = P.plan_export(n, m, k, sr, **kw)
    C = np.full((n, m), 12345678, np.int64)
    ws = np.full(max(info["temp_elems"], 1), -7777, np.int64)
    written = np.zeros((n, m), np.int64)
    kcover = np.zeros((n, m), np.int64)
    face_owner = np.full(ws.shape, -1, np.int64)
    for q in range(info["n_wg"]):
        for idx in range(wg[q], wg[q + 1]):
            it = items[idx]
            _, n0, n1, m0, m1, k0, k1, off = it
            part = _partial(sr, A, B, it)
            kcover[n0:n1, m0:m1] += k1 - k0
            if off < 0:
                C[n0:n1, m0:m1] = part
                written[n0:n1, m0:m1] += 1
            else:
                sz = (n1 - n0) * (m1 - m0)
                assert (face_owner[off:off + sz] < 0).all(), "temporary faces overlap"
                face_owner[off:off + sz] = idx
                ws[off:off + sz] = part.reshape(-1)
    assert (written == 1).all(), "each C element must be written by exactly one piece"
    assert (kcover == k).all(), "each (i, j) must see every l exactly once"
    for t in tiles:
        _, i0, i1, j0, j1, s0, s1 = t
        for s in range(s0, s1):
            off, ld, r0, c0 = srcs[s]
            rr = np.arange(i0, i1)[:, None] - r0
            cc = np.arange(j0, j1)[None, :] - c0
            C[i0:i1, j0:j1] = _fold(sr, C[i0:i1, j0:j1], ws[off + rr * ld + cc])
    return C, info


@pytest.mark.parametrize("p,part,sk", [(256, "paco", 0), (1, "paco", 0), (3, "paco", 0),
                                       (257, "paco", 0), (7, "grid", 3), (256, "grid", 0)])
def test_minplus_config0_plan_replay(p, part, sk):
    A, B = workloads.minplus_operands(384, 256, 320, seed=0)
    C, info = replay("minplus", A, B, 384, 256, 320, part=part, p=p, split_k=sk)
    np.testing.assert_array_equal(C, oracle.minplus(A, B))


@pytest.mark.parametrize("n,m,k", [(97, 130, 75), (33, 250, 64), (5, 3, 200)])
def test_maxplus_plan_replay(n, m, k):
    A, B = workloads.maxplus_operands(n, m, k, seed=3)
    A[2, :] = NEG_INF
    C, _ = replay("maxplus", A, B, n, m, k, p=64)
    np.testing.assert_array_equal(C, oracle.maxplus(A, B))


@pytest.mark.parametrize("n,m,k,p", [(64, 48, 2048, 64), (70, 90, 300, 256), (256, 256, 256, 7)])
def test_ring_plan_replay_small_integers(n, m, k, p):
    A, B = workloads.small_int_operands(n, m, k, seed=1)
    C, info = replay("ring", A.astype(np.int64), B.astype(np.int64), n, m, k, p=p)
    np.testing.assert_array_equal(C, oracle.ring_i64(A.astype(np.int64), B.astype(np.int64)))


def test_plan_sizes_match_paper_shapes():
    # long k: (2048, 1024, 65536) on 256 processors -> 512 x 1024 x 1024 pieces,
    # k cut 64-way: 252 temporary faces (4 n-blocks x 63) under the paper's
    # longest-dimension rule (k-cut cost 1)
    pcs = P.partition(2048, 1024, 65536, 256, q=(16, 16, 32), kcut_cost=1.0)
    ext = np.array([[p["n1"] - p["n0"], p["m1"] - p["m0"], p["k1"] - p["k0"]] for p in pcs])
    assert (ext == [512, 1024, 1024]).all()
    assert sum(p["temp"] for p in pcs) == 252


def test_ring_plan_long_k_pieces():
    # the ring plan on the 256 x 256 tile grid: every processor gets one
    # output tile 8192 deep (k cut 8-way: 224 faces); the first three cuts
    # go to the eight dies in groups of 32 consecutive processors
    items, wg, tiles, srcs, info = P.plan_export(2048, 1024, 65536, "ring", p=256, precision="bf16x3")
    ext = items[:, [2, 4, 6]] - items[:, [1, 3, 5]]
    assert (ext == [256, 256, 8192]).all()
    assert (items[:, 7] >= 0).sum() == 224
    assert info["xcd_remap"] == 1 and info["n_wg"] == 256 and info["tile"] == 4


RING_TILE = {0: (256, 128), 1: (128, 128), 2: (128, 64), 3: (128, 128), 4: (256, 256)}


def padded_critical(items, wg, info, k_ovh=64):
    """Busiest workgroup's padded work (whole tiles x k-range on the 32-deep
    step, plus two steps of overhead per tile) over the even share."""
    tm, tn = RING_TILE[info["tile"]]
    worst = 0
    for q in range(info["n_wg"]):
        w = 0
        for i in range(wg[q], wg[q + 1]):
            _, n0, n1, m0, m1, k0, k1, _ = items[i]
            w += -(-(n1 - n0) // tm) * tm * -(-(m1 - m0) // tn) * tn * (-(-(k1 - k0) // 32) * 32 + k_ovh)
        worst = max(worst, w)
    return worst


@pytest.mark.parametrize("n,m,k,p,bound", [(2048, 1024, 65536, 251, 1.06), (2048, 1024, 65536, 200, 1.06),
                                           (2048, 1024, 65536, 97, 1.03), (200704, 4096, 4096, 256, 1.02),
                                           (8192, 8192, 8192, 200, 1.06)])
def test_ring_plan_tile_balance(n, m, k, p, bound):
    """Arbitrary (also prime) p on the tile grid: the busiest processor's
    padded work stays within a few percent of n m k / p, where cuts of n and
    m rounded to whole tiles alone would pad whole tile rows (the batched
    Strassen leaves (49 x 4096, 4096, 4096) over 256 processors leave
    3.06 row tiles per processor)."""
    items, wg, _, _, info = P.plan_export(n, m, k, "ring", p=p, precision="bf16x3")
    assert info["n_wg"] == p
    assert padded_critical(items, wg, info) <= bound * n * m * k / p


@pytest.mark.parametrize("n,m,k", [(2048, 1024, 65536), (8192, 8192, 8192), (3000, 2000, 5000), (700, 900, 33000)])
@pytest.mark.parametrize("p", [7, 97, 128, 200, 251, 256])
def test_tile_search_never_worse_than_paper_rule(n, m, k, p):
    """The tile-grid search picks each cut's dimension among all of them,
    the paper's choice included, so its busiest processor (same quanta, same
    cost: whole 256 x 256 tiles, k on the 32-step, two steps per tile, four
    more for a piece that writes a face) is never worse than under the
    paper's longest-dimension rule."""
    def cost(pcs):
        w = {}
        for pc in pcs:
            t = -(-(pc["n1"] - pc["n0"]) // 256) * -(-(pc["m1"] - pc["m0"]) // 256)
            kk = -(-(pc["k1"] - pc["k0"]) // 32) * 32
            if pc["n1"] > pc["n0"] and pc["m1"] > pc["m0"] and kk > 0:
                w[pc["proc"]] = w.get(pc["proc"], 0) + t * (kk + 64 + (128 if pc["k0"] > 0 else 0))
        return max(w.values())
    q = (256 if n >= 512 else 16, 256 if m >= 512 else 16, 32)
    paper = P.partition(n, m, k, p, q=q, kcut_cost=16.0)
    tiled = P.partition(n, m, k, p, q=q, kcut_cost=16.0, tile_balance=True)
    assert sorted(pc["proc"] for pc in tiled) == list(range(p))
    vol = sum((pc["n1"] - pc["n0"]) * (pc["m1"] - pc["m0"]) * (pc["k1"] - pc["k0"]) for pc in tiled)
    assert vol == n * m * k
    assert cost(tiled) <= cost(paper) * (1 + 1e-9)


@pytest.mark.parametrize("sr,n,m,k", [("minplus", 384, 256, 320), ("minplus", 700, 300, 2048),
                                      ("maxplus", 4096, 64, 512), ("maxplus", 257, 513, 129)])
def test_default_choice_plan_replay(sr, n, m, k):
    """p = 0: the call's default choice of processor count, tile and k-cut
    cost still yields a plan that covers every (i, j, l) once."""
    if sr == "minplus":
        A, B = workloads.minplus_operands(n, m, k, seed=5)
        ref = oracle.minplus(A, B)
    else:
        A, B = workloads.maxplus_operands(n, m, k, seed=5)
        ref = oracle.maxplus(A, B)
    C, info = replay(sr, A, B, n, m, k, part="paco", p=0)
    np.testing.assert_array_equal(C, ref)
    assert info["n_wg"] % 256 == 0   # slots (or 4x slots) of 256 compute units


@pytest.mark.parametrize("p", [3, 200, 251, 256])
def test_multi_piece_plan_replay(p):
    """Multi-piece pruned BFS (part="multi"): several pieces per processor,
    each (i, j, l) still covered once and the result the oracle's."""
    A, B = workloads.minplus_operands(384, 256, 320, seed=7)
    C, info = replay("minplus", A, B, 384, 256, 320, part="multi", p=p)
    np.testing.assert_array_equal(C, oracle.minplus(A, B))
    items, wg, _, _, _ = P.plan_export(384, 256, 320, "minplus", part="multi", p=p)
    assert info["n_wg"] == p and len(items) >= p


def test_multi_piece_ring_plan_replay():
    A, B = workloads.small_int_operands(300, 200, 700, seed=4)
    C, _ = replay("ring", A.astype(np.int64), B.astype(np.int64), 300, 200, 700, part="multi", p=97)
    np.testing.assert_array_equal(C, A.astype(np.int64) @ B.astype(np.int64))


def replay_fused(sr, A, B, n, m, k, seed, **kw):
    """The fused-fold plan replayed with the pieces finishing in a random
    order: each finished item counts itself in every cell it covers; the
    item completing a cell's count folds it (C then its faces, in list
    order) and resets the counter."""
    items, wg, tiles, srcs, info = P.plan_export(n, m, k, sr, **kw)
    pads, itf, fl, info2 = P.plan_export_fold(n, m, k, sr, **kw)
    assert info["fused"] == 1 and info2["n_fold_list"] == len(fl)
    # each cell's count is the number of items whose rectangle meets it,
    # and each item lists exactly the cells its rectangle meets
    for idx, it in enumerate(items):
        _, n0, n1, m0, m1, k0, k1, off = it
        meet = [c for c, t in enumerate(tiles) if t[1] < n1 and t[2] > n0 and t[3] < m1 and t[4] > m0]
        b, cnt = itf[idx]
        assert sorted(fl[b:b + cnt].tolist()) == meet
    for c in range(len(tiles)):
        assert pads[c] == sum(c in fl[b:b + cnt].tolist() for b, cnt in itf)
    C = np.full((n, m), 12345678, np.int64)
    ws = np.full(max(info["temp_elems"], 1), -7777, np.int64)
    counter = np.zeros(len(tiles), np.int64)
    folded = np.zeros(len(tiles), np.int64)
    order = np.random.default_rng(seed).permutation(len(items))
    for idx in order:
        it = items[idx]
        _, n0, n1, m0, m1, k0, k1, off = it
        part = _partial(sr, A, B, it)
        if off < 0:
            C[n0:n1, m0:m1] = part
        else:
            ws[off:off + part.size] = part.reshape(-1)
        b, cnt = itf[idx]
        for c in fl[b:b + cnt]:
            counter[c] += 1
            if counter[c] == pads[c]:
                counter[c] = 0
                folded[c] += 1
                _, i0, i1, j0, j1, s0, s1 = tiles[c]
                for s in range(s0, s1):
                    o, ld, r0, c0 = srcs[s]
                    rr = np.arange(i0, i1)[:, None] - r0
                    cc = np.arange(j0, j1)[None, :] - c0
                    C[i0:i1, j0:j1] = _fold(sr, C[i0:i1, j0:j1], ws[o + rr * ld + cc])
    assert (folded == 1).all() and (counter == 0).all()
    return C


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("sr,n,m,k,p", [("minplus", 384, 256, 320, 0), ("minplus", 97, 130, 75, 0),
                                        ("maxplus", 257, 65, 900, 64), ("minplus", 70, 50, 3000, 37)])
def test_fused_fold_plan_replay(sr, n, m, k, p, seed, monkeypatch):
    """Plans whose cells are small fold inside the product kernel: whatever
    order the pieces finish in, every cell is folded exactly once, by the
    last piece to reach it, after every piece covering it has written, and
    the counters end at zero.  (PACO_FUSE_FOLD=1 fuses plans whose cells
    are larger too.)"""
    monkeypatch.setenv("PACO_FUSE_FOLD", "1")
    gen = workloads.minplus_operands if sr == "minplus" else workloads.maxplus_operands
    A, B = gen(n, m, k, seed=seed + 11)
    C = replay_fused(sr, A, B, n, m, k, seed, p=p)
    np.testing.assert_array_equal(C, (oracle.minplus if sr == "minplus" else oracle.maxplus)(A, B))


def test_fold_policy(monkeypatch):
    # default: a separate fold launch
    _, _, _, _, info = P.plan_export(384, 256, 320, "minplus", p=0)
    assert info["fused"] == 0
    # PACO_FUSE_FOLD=2 fuses plans whose cells are small: not the long-k
    # ring product, where every cell is a 256 x 256 tile with seven faces
    # (1.75 MiB read by one fold)
    monkeypatch.setenv("PACO_FUSE_FOLD", "2")
    _, _, _, _, info = P.plan_export(2048, 1024, 65536, "ring", p=256, precision="bf16x3")
    assert info["fused"] == 0
    _, _, _, _, info = P.plan_export(384, 256, 320, "minplus", p=0)
    assert info["fused"] == 1


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
def test_forced_ring_tile_plan(tile, prec, monkeypatch):
    """PACO_RING_TILE forces any of the ring kernel's tile shapes (also the
    four-wave 128 x 128 one outside the default candidates); the 256 x 256
    tile cannot hold three bf16 parts and is then ignored.  The plan still
    covers every (i, j, l) once."""
    monkeypatch.setenv("PACO_RING_TILE", str(tile))
    n, m, k = 300, 260, 2000
    _, _, _, _, info = P.plan_export(n, m, k, "ring", p=64, precision=prec)
    assert info["tile"] == (tile if not (tile == 4 and prec == "bf16x6") else info["tile"])
    assert info["tile"] != 4 or prec != "bf16x6"
    A, B = workloads.small_int_operands(n, m, k, seed=tile)
    C, _ = replay("ring", A.astype(np.int64), B.astype(np.int64), n, m, k, p=64, precision=prec)
    np.testing.assert_array_equal(C, oracle.ring_i64(A.astype(np.int64), B.astype(np.int64)))


@pytest.mark.parametrize("sr,n,m,k,kw", [
    ("minplus", 384, 256, 320, dict(p=0)),
    ("minplus", 384, 256, 320, dict(part="multi", p=200)),
    ("ring", 2048, 1024, 65536, dict(p=256, precision="bf16x3")),
    ("ring", 837, 837, 837, dict(p=256, precision="bf16x6")),
    ("ring", 300, 200, 700, dict(part="multi", p=97)),
    ("maxplus", 257, 513, 129, dict(p=251)),
    ("minplus", 70, 50, 3000, dict(part="grid", p=37, split_k=5)),
])
def test_fold_sources_complete_and_in_k_order(sr, n, m, k, kw):
    """Section "PACO MM" combines the temporary faces of height cuts by the
    semiring's addition; for the float ring the order of that fold decides
    the bits, and the plan fixes it as ascending k.  Every reduction tile
    lists exactly the faces that cover it, each covering the whole tile,
    in strictly ascending k0; every element covered by a face lies in
    exactly one tile, and no tile lies outside the faces."""
    items, _, tiles, srcs, info = P.plan_export(n, m, k, sr, **kw)
    faces = {int(it[7]): it for it in items if it[7] >= 0}
    assert len(faces) == sum(1 for it in items if it[7] >= 0) > 0   # distinct offsets
    covered = np.zeros((n, m), np.int64)
    for it in faces.values():
        covered[it[1]:it[2], it[3]:it[4]] = 1
    tiled = np.zeros((n, m), np.int64)
    for t in tiles:
        _, i0, i1, j0, j1, s0, s1 = (int(x) for x in t)
        tiled[i0:i1, j0:j1] += 1
        want = sorted((int(it[5]), off) for off, it in faces.items()
                      if it[1] < i1 and it[2] > i0 and it[3] < j1 and it[4] > j0)
        got = []
        for s in range(s0, s1):
            off, ld, r0, c0 = (int(x) for x in srcs[s])
            it = faces[off]
            assert (r0, c0, ld) == (it[1], it[3], it[4] - it[3])
            assert it[1] <= i0 and i1 <= it[2] and it[3] <= j0 and j1 <= it[4], "face must cover its tile"
            got.append((int(it[5]), off))
        assert got == want, "sources must be every covering face, in ascending k"
        assert all(a[0] < b[0] for a, b in zip(got, got[1:]))
    np.testing.assert_array_equal(tiled, covered)


@pytest.mark.parametrize("sr", ["minplus", "maxplus"])
@pytest.mark.parametrize("n,m,k,kw", [(384, 256, 320, dict(p=0)), (8192, 8192, 8192, dict(p=0)),
                                      (3000, 3000, 3000, dict(p=0)), (300, 77, 129, dict(p=0)),
                                      (1000, 999, 997, dict(p=251)), (97, 130, 75, dict(p=3)),
                                      (384, 256, 320, dict(part="multi", p=200)),
                                      (517, 260, 700, dict(part="grid", p=64, split_k=7))])
def test_integer_items_start_four_aligned(sr, n, m, k, kw):
    """The integer kernel's 128-bit loads need every work item to start on a
    multiple of four in k and m (the call checks the operands' alignment);
    integer plans cut m and k on multiples of four so that they all do."""
    items, _, _, _, _ = P.plan_export(n, m, k, sr, **kw)
    assert len(items) > 0
    assert all(it[3] % 4 == 0 and it[5] % 4 == 0 for it in items)
