"""lb_totals_noalloc, the entry point for callers that cannot allocate, against
lb_totals on the same states: two calls in a row on one GPU (sharing the
library's fixed scratch array), the second with a smaller lattice, so a stale
partial record from the first would show."""
import numpy as np
import pytest

from lbcases import Case, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a gfx950 GPU")]


def _noalloc_totals(s):
    import torch

    from paper_1806_10247_amd import capi as C
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    C.lb_totals_noalloc(s.ctx, out.data_ptr())
    C.lb_synchronize(s.ctx)
    return out.cpu().numpy()


def _state(case, storage, steps):
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    s = case.gpu(storage)
    s.write_populations(f0, g0)
    s.step(steps)
    return s


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_noalloc_totals_match_lb_totals_on_two_calls(storage):
    big = Case("D3Q27", (96, 80, 72), walls=(False, True, True), nu=0.05, force=(1e-5, 0, 0), seed=31)
    small = Case("D2Q9_D2Q5", (37, 29, 1), nu=0.04, D=0.03, force=(1e-5, -1e-5, 0), source=1e-5, seed=32)
    for case, steps in ((big, 5), (small, 3)):
        with _state(case, storage, steps) as s:
            ref = s.totals()
            got = _noalloc_totals(s)
            again = _noalloc_totals(s)
        assert np.isfinite(got).all()
        # float64 sums of the same stored values in another order: the running sums
        # stay below N in magnitude, so the orders differ by a few of their ulps; a
        # lost or stale partial record (256 nodes) would move them by far more
        tol = 1e-13 * (np.abs(ref) + case.N)
        assert np.all(np.abs(got - ref) <= tol), (case, got, ref)
        assert np.array_equal(got, again)


def test_noalloc_totals_rejects_null_and_uninitialised():
    from paper_1806_10247_amd import capi as C
    from paper_1806_10247_amd.solver import Solver
    with Solver("D2Q9", (8, 8, 1)) as s:
        with pytest.raises(C.LbError) as e:
            C.lb_totals_noalloc(s.ctx, 0)
        assert e.value.code == C.LB_EINVAL
        with pytest.raises(C.LbError) as e:
            C.lb_totals_noalloc(s.ctx, 1 << 20)
        assert e.value.code == C.LB_ESTATE
