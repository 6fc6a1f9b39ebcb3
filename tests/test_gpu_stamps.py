"""Device-side per-processor timestamps (paco_set_piece_stamps): every
processor of a call records a start no later than its end, on one of the
device's compute units, and the results are unchanged by recording."""
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


@pytest.mark.parametrize("sr,shape,part", [("minplus", (384, 256, 320), "paco"), ("ring", (512, 512, 4096), "paco"),
                                           ("ring", (512, 512, 4096), "grid"), ("bool", (256, 512, 2048), "paco")])
def test_stamps_recorded(ctx, sr, shape, part):
    n, m, k = shape
    print(f"case: stamps {sr} {shape} {part}", flush=True)
    if sr == "bool":
        _, _, ap, bp = workloads.bool_operands(n, m, k, seed=1)
        A, B = torch.from_numpy(ap.view(np.int32)).to(DEV), torch.from_numpy(bp.view(np.int32)).to(DEV)
        kw = dict(n=n, m=m, k=k)
        ref = oracle.bool_packed(ap, bp, n, m, k).view(np.int32)
    elif sr == "minplus":
        a, b = workloads.minplus_operands(n, m, k, seed=1)
        A, B, kw, ref = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV), {}, oracle.minplus(a, b)
    else:
        a, b = workloads.small_int_operands(n, m, k, seed=1)
        A, B = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
        kw, ref = dict(precision="bf16x3"), oracle.ring_f64(a, b).astype(np.float32)
    st = torch.full((4096, 4), -1, dtype=torch.int64, device=DEV)
    ctx.set_piece_stamps(st)
    try:
        C, r = ctx.semiring_mm(A, B, sr, part=part, return_result=True, **kw)
        torch.cuda.synchronize()
    finally:
        ctx.set_piece_stamps(None)
    assert np.array_equal(C.cpu().numpy(), ref)
    s = st.cpu().numpy()
    p = r["p"]
    assert p <= 4096
    rec = s[:p]
    assert (rec[:, 0] > 0).all() and (rec[:, 1] >= rec[:, 0]).all()
    assert (s[p:, 0] == -1).all()                       # no slot beyond the call's processors
    assert set(np.unique(rec[:, 2] & 0xF)) <= set(range(8))
    span = (rec[:, 1].max() - rec[:, 0].min()) / 100.0  # microseconds
    assert 0 < span < 1e6
    # the call after turning it off writes nothing
    st.fill_(-1)
    ctx.semiring_mm(A, B, sr, part=part, **kw)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == -1).all()
