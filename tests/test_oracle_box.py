"""The sampled full-size parity tests compare GPU nodes with the oracle run on a
small box around them.  This checks that sampling scheme on the CPU: the
oracle on a box (walls where the lattice has walls, wrapped elsewhere) agrees
exactly with the oracle on the whole lattice at every node it marks valid."""
import numpy as np

import oracle as O
from casclb_inputs import coords, fourier_modes, smooth_fields_at
from lbcases import Case, oracle_box


def _full_run(case, steps, seed):
    dom = case.oracle()
    rho, u, phi = smooth_fields_at(case.shape, coords(case.shape), case.dims, seed=seed)
    dom.init_equilibrium(rho, u, phi)
    dom.run(steps)
    return dom


def _box_f(dom, case, lo, ext):
    pts = coords(tuple(ext))
    pts = (pts + np.array(lo)[:, None]) % np.array(case.shape)[:, None]
    idx = pts[0] + case.shape[0] * (pts[1] + case.shape[1] * pts[2])
    return dom.f[:, idx], (None if dom.g is None else dom.g[:, idx])


def test_box_sampling_matches_full_lattice():
    steps, seed = 3, 4
    modes = fourier_modes((14, 12, 10), nmodes=3, amp=1e-4, kmax=2, seed=1)
    cases = [
        Case("D3Q27", (14, 12, 10), walls=(False, True, True), nu=0.08, force=(1e-4, 2e-5, 0)),
        Case("D3Q27", (14, 12, 10), nu=0.05, force_field=lambda p: modes.evaluate(p)),
        Case("D2Q9_D2Q5", (16, 13, 1), walls=(False, True, False), nu=0.04, D=0.03, force=(1e-4, 0, 0),
             source_field=lambda p: 1e-4 * np.sin(2 * np.pi * p[0] / 16)),
    ]
    for case in cases:
        full = _full_run(case, steps, seed)
        init = lambda pts, c=case: smooth_fields_at(c.shape, pts, c.dims, seed=seed)
        for lo in [(0, 0, 0), (10, 7, 3), (5, 4, 0)]:
            ext = (9, 9, 9 if case.dims == 3 else 1)
            ext = tuple(min(e, n) for e, n in zip(ext, case.shape))
            # boxes stay inside walls; on periodic axes they may wrap
            lo = tuple(min(a, n - e) if w else a for a, e, n, w in zip(lo, ext, case.shape, case.walls))
            box, valid = oracle_box(case, lo, ext, steps, init_fields=init)
            assert valid.sum() > 0
            f, g = _box_f(full, case, lo, ext)
            assert np.abs(box.f[:, valid] - f[:, valid]).max() < 1e-15, (case, lo)
            if g is not None:
                assert np.abs(box.g[:, valid] - g[:, valid]).max() < 1e-15
