"""Debug poison (LB_FLAG_DEBUG_POISON): before every step the buffer the step
writes is filled with NaN bit patterns, so a node the step kernel leaves
unwritten would surface as NaN.  Over every lattice, storage and launch shape
(block widths, one or two rows per thread, x-adjacent node pairs, XCD-ordered
blocks, walls on every axis, moving walls and heating, residual steps) the
poisoned runs must equal the plain runs bit for bit and stay finite."""
import sys

import numpy as np
import pytest

from lbcases import Case, gpu_available
from test_gpu_parity import parity_cases
from test_gpu_walls import _gpu as _wall_gpu
from test_gpu_walls import _oracle as _wall_oracle
from test_gpu_walls import wall_cases

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a gfx950 GPU")]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _shapes(case, storage):
    from paper_1806_10247_amd import capi as C
    shapes = [(64, 1, 0, 1), (128, 2, 0, 1), (192, 1, C.LB_FLAG_XCD_REMAP, 1), (256, 2, C.LB_FLAG_XCD_REMAP, 1)]
    if storage == "f16" and case.shape[0] % 2 == 0 and not case.walls[0]:
        shapes += [(64, 1, 0, 2), (128, 1, C.LB_FLAG_XCD_REMAP, 2)]
    return shapes


def _run(case, storage, f0, g0, bx, rows, flags, xp, steps=15):
    with case.gpu(storage, block_x=bx, rows_per_thread=rows, flags=flags, residual_interval=7, x_pairs=xp) as s:
        s.write_populations(f0, g0)
        s.step(steps)
        f, g = s.populations()
        r, at, tot = s.residual()
    return f, g, r, tot


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("idx", range(10))
def test_poisoned_steps_write_every_node(idx, storage):
    from paper_1806_10247_amd import capi as C
    case = parity_cases()[idx]
    _say("case", case, storage)
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    for bx, rows, flags, xp in _shapes(case, storage):
        ref = _run(case, storage, f0, g0, bx, rows, flags, xp)
        got = _run(case, storage, f0, g0, bx, rows, flags | C.LB_FLAG_DEBUG_POISON, xp)
        assert np.isfinite(got[0]).all(), (bx, rows, flags, xp, int((~np.isfinite(got[0])).sum()))
        assert np.array_equal(got[0], ref[0]), (bx, rows, flags, xp)
        if got[1] is not None:
            assert np.isfinite(got[1]).all() and np.array_equal(got[1], ref[1])
        assert got[2] == ref[2] and np.array_equal(got[3], ref[3])


@pytest.mark.parametrize("idx", range(3))
def test_poisoned_wall_and_heating_steps(idx):
    from paper_1806_10247_amd import capi as C
    case, wu, pw, heat = wall_cases()[idx]
    dom = _wall_oracle(case, wu, pw, heat)
    f0, g0 = case.perturbed_state(dom)
    out = []
    for flags in (0, C.LB_FLAG_DEBUG_POISON):
        with _wall_gpu(case, wu, pw, heat, storage="f32", flags=flags, residual_interval=5) as s:
            s.write_populations(f0, g0)
            s.step(12)
            out.append(s.populations())
    assert np.isfinite(out[1][0]).all() and np.array_equal(out[0][0], out[1][0])
    if out[0][1] is not None:
        assert np.isfinite(out[1][1]).all() and np.array_equal(out[0][1], out[1][1])


def test_poison_reaches_the_plane_padding():
    """The fill covers the whole destination buffer: the padding after each
    population plane (never written by a step) holds the NaN pattern after a
    poisoned step, and the nodes hold the step's values."""
    import torch

    from paper_1806_10247_amd import capi as C
    case = Case("D2Q9", (40, 6, 1), nu=0.05, force=(1e-5, 0, 0))
    cfg = C.lb_config_default(lattice=C.LB_D2Q9, storage=C.LB_STORE_F32_DEV, nx=40, ny=6, nz=1, nu=0.05,
                              plane_pad=8, residual_interval=0,
                              flags=C.LB_FLAG_EXTERNAL_BUFFERS | C.LB_FLAG_DEBUG_POISON)
    nbytes = C.lb_required_bytes(cfg)
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    ctx = C.lb_create(cfg)
    try:
        C.lb_bind_buffers(ctx, a.data_ptr(), b.data_ptr(), nbytes)
        C.lb_init_equilibrium(ctx)
        C.lb_step(ctx, 1)
        C.lb_synchronize(ctx)
        cur = C.lb_get_info(ctx).buf_current
        buf = (b if cur == b.data_ptr() else a).view(torch.float32).cpu().numpy().reshape(9, 240 + 8)
        assert np.isfinite(buf[:, :240]).all()
        assert np.isnan(buf[:, 240:]).all()
    finally:
        C.lb_destroy(ctx)
    del case
