"""Device peak probes (paco_peak): each returns a finite rate inside what
the part can physically do (published peaks as upper bounds, with margin for
clock boost), and an unknown probe is rejected."""
import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu

import paper_2011_01441_amd as P  # noqa: E402

# (probe, lower, upper): lower bounds are far below any working part;
# upper bounds are the published peaks plus 10 %
BOUNDS = [("mfma_bf16", 200.0, 2750.0), ("valu_i32", 4.0, 43.3),
          ("valu_f32", 8.0, 86.5), ("hbm_copy", 500.0, 8800.0)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind,lo,hi", BOUNDS)
def test_peak_in_range(ctx, kind, lo, hi):
    r = ctx.peak(kind)
    print(kind, r)
    assert lo < r < hi


def test_peak_unknown_kind(ctx):
    r = ctypes.c_double(0.0)
    st = ctx._L.paco_peak(ctx._h, 17, ctypes.byref(r))
    assert st == 1   # PACO_ERR_INVALID_ARG
