"""The allocation-free semiring MM entry point (paco_semiring_mm_noalloc),
called through the C ABI, against the allocating one (paco_semiring_mm_ex)
on the same operands: the two share the plan and the kernels, so their
results must be bit-identical for every semiring, including the float32
ring.  Each case makes two calls in a row, the second on a smaller input,
so the fixed scratch memory is reused with the first call's contents still
in it."""
import ctypes

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

import paper_2011_01441_amd as P  # noqa: E402

DEV = torch.device("cuda:0")
OK, ERR_UNSUPPORTED, ERR_BUDGET = 0, 2, 4


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def desc(sr, n, m, k, A, B, C, **kw):
    d = P.MMDesc()
    d.n, d.m, d.k, d.sr = n, m, k, P.SEMIRING[sr]
    d.A, d.lda = A.data_ptr(), A.stride(0)
    d.B, d.ldb = B.data_ptr(), B.stride(0)
    d.C, d.ldc = C.data_ptr(), C.stride(0)
    d.precision = P.PRECISION[kw.get("precision", "auto")]
    d.part = P.PART[kw.get("part", "paco")]
    d.p = kw.get("p", 0)
    d.accumulate = 1 if kw.get("accumulate") else 0
    d.kcut_cost = kw.get("kcut_cost", 0.0)
    d.verify_rows = kw.get("verify_rows", 0)
    return d


def operands(sr, n, m, k, seed):
    """(A, B, C-shape, dtype) on the device for one case."""
    if sr == "minplus":
        A, B = workloads.minplus_operands(n, m, k, seed=seed)
    elif sr == "maxplus":
        A, B = workloads.maxplus_operands(n, m, k, seed=seed)
    elif sr == "bool":
        _, _, ap, bp = workloads.bool_operands(n, m, k, density=0.05, seed=seed)
        A, B = ap.view(np.int32), bp.view(np.int32)
        return dev(A), dev(B), (n, (m + 31) // 32), torch.int32
    else:
        A, B = workloads.ring_operands(n, m, k, seed=seed)
    return dev(A), dev(B), (n, m), dev(A).dtype


def both(ctx, sr, n, m, k, seed, **kw):
    """C from paco_semiring_mm_ex and from paco_semiring_mm_noalloc (C of the
    latter prefilled with a sentinel), plus the allocating call's result."""
    L = P.lib()
    ctx._stream()
    A, B, cshape, dt = operands(sr, n, m, k, seed)
    C_ref = torch.zeros(cshape, dtype=dt, device=DEV)
    C_na = torch.full(cshape, 7, dtype=dt, device=DEV)
    if kw.get("accumulate"):
        base = torch.randint(0, 1 << 20, cshape, dtype=torch.int32, device=DEV)
        C_ref.copy_(base.to(dt))
        C_na.copy_(base.to(dt))
    r_ref, r_na = P.MMResult(), P.MMResult()
    d = desc(sr, n, m, k, A, B, C_ref, **kw)
    assert L.paco_semiring_mm_ex(ctx._h, ctypes.byref(d), ctypes.byref(r_ref)) == OK
    d = desc(sr, n, m, k, A, B, C_na, **kw)
    st = L.paco_semiring_mm_noalloc(ctx._h, ctypes.byref(d), ctypes.byref(r_na))
    assert st == OK, L.paco_last_error(ctx._h).decode()
    torch.cuda.synchronize()
    assert r_na.n_kcuts == r_ref.n_kcuts and r_na.temp_elems == r_ref.temp_elems and r_na.p == r_ref.p
    return C_ref.cpu().numpy(), C_na.cpu().numpy(), r_ref


CASES = [
    # (semiring, first shape, second (smaller) shape, options)
    ("minplus", (384, 256, 320), (97, 130, 75), {}),
    ("maxplus", (1024, 64, 512), (300, 77, 129), {"kcut_cost": 1.0}),
    ("bool", (512, 700, 4096), (50, 100, 70), {}),
    ("ring", (512, 512, 8192), (130, 70, 1000), {"precision": "bf16x3"}),
    ("ring", (256, 384, 4096), (64, 96, 333), {"precision": "fp32"}),
    ("ring", (300, 260, 2048), (33, 65, 129), {"precision": "bf16x6"}),
    ("minplus", (256, 256, 2048), (100, 90, 700), {"accumulate": True}),
    ("ring", (256, 256, 4096), (40, 50, 600), {"precision": "bf16x3", "accumulate": True}),
]


@pytest.mark.parametrize("sr,first,second,kw", CASES)
def test_noalloc_matches_allocating_call(ctx, sr, first, second, kw):
    kcuts = []
    for i, (n, m, k) in enumerate((first, second)):
        print(f"case: noalloc {sr} {n}x{m}x{k} {kw} call {i + 1}", flush=True)
        ref, got, r = both(ctx, sr, n, m, k, seed=n + 3 * m + 7 * k, **kw)
        assert ref.shape == got.shape
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32)), f"call {i + 1} differs"
        kcuts.append(r.n_kcuts)
    # the first call of each case reads temporary faces from the scratch
    assert kcuts[0] > 0


def test_noalloc_rejects_oversized_plan(ctx):
    """A plan whose temporary faces exceed the fixed array is refused before
    anything is launched: C keeps its contents."""
    L = P.lib()
    ctx._stream()
    cap = L.paco_noalloc_scratch_bytes()
    assert cap == 64 << 20
    n, m, k = 1024, 1024, 65536   # 1024 processors: 16 tiles cut 64-way in k, 252 MiB of faces
    print(f"case: noalloc oversized ring {n}x{m}x{k}", flush=True)
    A = torch.zeros((n, k), dtype=torch.float32, device=DEV)
    B = torch.zeros((k, m), dtype=torch.float32, device=DEV)
    C = torch.full((n, m), 3.0, dtype=torch.float32, device=DEV)
    d = desc("ring", n, m, k, A, B, C, precision="bf16x3", p=1024)
    r = P.MMResult()
    st = L.paco_semiring_mm_noalloc(ctx._h, ctypes.byref(d), ctypes.byref(r))
    assert st == ERR_BUDGET
    assert b"scratch" in L.paco_last_error(ctx._h)
    torch.cuda.synchronize()
    assert bool((C == 3.0).all())
    # verify_rows needs device buffers: refused
    d = desc("ring", 64, 64, 64, A, B, C, precision="bf16x3", verify_rows=4)
    assert L.paco_semiring_mm_noalloc(ctx._h, ctypes.byref(d), ctypes.byref(r)) == ERR_UNSUPPORTED
    # a call that fits still works after the refusals
    ref, got, _ = both(ctx, "minplus", 130, 140, 600, seed=5)
    assert np.array_equal(ref, got)
