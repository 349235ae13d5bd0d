"""Parity at the full workload sizes, in the launch configuration the benchmark
times (library defaults).  The oracle cannot run these lattices, so it checks
sampled outputs one box at a time: the GPU runs s steps of the whole lattice
from a seeded smooth initial state, and the oracle runs the same s steps on a
small box around each sample (walls where the lattice has walls, wrapped
elsewhere), which fixes every node at least s nodes inside the box.  After
long runs, properties that hold at any size are checked against closed forms.
"""
import sys

import numpy as np
import pytest

import oracle as O
from casclb_inputs import (coords, duct_3d, fourier_modes, product_source_2d, smooth_fields_at, vortex_force_2d,
                           coupled_2d)
from lbcases import Case, gpu_available, oracle_box, reduced_precision_bound

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a gfx950 GPU")]

STEPS = 3
TOL_F64 = 1e-12


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bound(steps, storage, scale):
    return reduced_precision_bound(steps, storage, scale)


def _rest(lattice):
    lat = {"D3Q27": O.D3Q27, "D3Q15": O.D3Q15}.get(lattice, O.D2Q9)
    return O.flow_equilibrium(lat, 1.0, [0, 0, 0])


def _sampled_parity(case, storage, boxes, steps=STEPS, init_seed=5, **launch):
    """Run `steps` steps of the full lattice on the GPU from smooth_fields_at, then
    check the given boxes against the oracle."""
    shape = case.shape
    d = case.dims
    _say(f"[fullsize] {case} {storage}: generating initial fields")
    rho, u, phi = smooth_fields_at(shape, coords(shape), d, seed=init_seed)
    init = lambda pts: smooth_fields_at(shape, pts, d, seed=init_seed)
    with case.gpu(storage, **launch) as s:
        s.init_equilibrium(rho, u, phi if case.lattice == "D2Q9_D2Q5" else None)
        del rho, u, phi
        s.step(steps)
        s.synchronize()
        rest = _rest(case.lattice)
        for lo, ext in boxes:
            dom, valid = oracle_box(case, lo, ext, steps, init_fields=init)
            f, g = s.populations_box(lo, ext)
            dev = dom.f[:, valid] - rest[:, None]
            err = np.abs(f[:, valid] - dom.f[:, valid]).max()
            scale = np.abs(dev).max()
            _say(f"[fullsize]   box lo={lo} ext={ext}: {valid.sum()} nodes, max err {err:.3e}, "
                 f"deviation scale {scale:.3e}")
            if storage == "f64":
                assert err <= TOL_F64
                assert err <= 1e-6 * scale      # meaningful relative to the deviations themselves
            else:
                assert err <= _bound(steps, storage, scale)
            if g is not None:
                errg = np.abs(g[:, valid] - dom.g[:, valid]).max()
                scale_g = np.abs(dom.g[:, valid]).max()
                assert errg <= (TOL_F64 if storage == "f64" else _bound(steps, storage, scale_g))


def _duct_case():
    w = duct_3d(256)
    return Case("D3Q27", w.shape, walls=w.walls, nu=w.nu, force=w.force)


DUCT_BOXES = [((100, 0, 0), (9, 8, 8)),       # corner of two walls
              ((250, 0, 120), (9, 8, 9)),     # wall y = 0, wraps in x
              ((30, 248, 248), (9, 8, 8)),    # opposite corner
              ((120, 124, 124), (9, 9, 9))]   # centre


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_duct_256_sampled(storage):
    """In the launch configuration the benchmark times for each storage (float64 with
    the XCD-ordered block mapping)."""
    import bench
    from paper_1806_10247_amd import capi as C
    st = {"f64": C.LB_STORE_F64, "f32": C.LB_STORE_F32_DEV, "f16": C.LB_STORE_F16_DEV}[storage]
    _sampled_parity(_duct_case(), storage, DUCT_BOXES, flags=bench.launch_flags(C, st))


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_duct_256_d3q15_sampled(storage):
    """The D3Q15 duct the benchmark times (Appendix A lattice), same boxes."""
    w = duct_3d(256)
    _sampled_parity(Case("D3Q15", w.shape, walls=w.walls, nu=w.nu, force=w.force), storage, DUCT_BOXES)


def test_periodic_512_fourier_force_sampled():
    modes = fourier_modes((512, 512, 512), seed=0)
    force = lambda pts: modes.evaluate(pts)
    case = Case("D3Q27", (512, 512, 512), nu=(0.76 - 0.5) / 3, force_field=force)
    _sampled_parity(case, "f64", [((0, 0, 0), (9, 9, 9)), ((507, 250, 3), (9, 9, 9)),
                                  ((300, 511, 100), (9, 9, 9))])


def test_poiseuille_4x64_20000_steps():
    """The Poiseuille channel at its full run: 4 x 64 (x periodic, halfway bounce-back
    walls), Fx = 1e-6, nu = 1/6, float64, 20000 steps from rest.  Every population
    against the oracle's 20000 steps (<= 1e-12); the GPU profile against the
    start-up Fourier series (a constant wall slip apart); mass kept to round-off."""
    nu, F, ny = 1.0 / 6.0, 1e-6, 64
    dom = O.Domain(O.D2Q9, 4, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force=(F, 0))
    dom.init_equilibrium()
    dom.run(20000)
    case = Case("D2Q9", (4, ny, 1), walls=(False, True, False), nu=nu, force=(F, 0.0, 0.0))
    with case.gpu("f64") as s:
        s.init_equilibrium()
        s.step(20000)
        f, _ = s.populations()
        _, u, _ = s.moments(1)
        tot = s.totals()
    err = np.abs(f - dom.f).max()
    _say(f"[fullsize] Poiseuille 4x64 20000 steps: max |f_gpu - f_oracle| = {err:.3e}")
    assert err <= TOL_F64
    ux = u[0].reshape(ny, 4)[:, 0]
    y = np.arange(ny) + 0.5
    L = ny / 2
    eta = (y - L) / L
    series = 1 - eta**2
    for n in range(400):
        k = 2 * n + 1
        series -= 32 * (-1) ** n / (k**3 * np.pi**3) * np.cos(k * np.pi * eta / 2) * np.exp(
            -k * k * np.pi**2 * nu * 20000 / (4 * L * L))
    ua = F * L * L / (2 * nu) * series
    assert np.ptp(ux - ua) < 6e-9
    assert abs((ux - ua).mean()) < 1e-3 * ua.max()
    assert abs(tot[0] - 4 * ny) < 1e-11


def _coupled_case():
    w = coupled_2d(4096)
    A, B = w.extra["A"], w.extra["B"]
    return Case("D2Q9_D2Q5", w.shape, nu=w.nu, D=w.D,
                force_field=lambda pts: vortex_force_2d(w.shape, A, pts), force_time=(O.TIME_COS, w.force_omega),
                source_field=lambda pts: product_source_2d(w.shape, B, pts)), w


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_coupled_4096_sampled(storage):
    """In the launch configuration the benchmark times for each storage (XCD-ordered
    blocks for float64, x-adjacent node pairs for float16)."""
    import bench
    from paper_1806_10247_amd import capi as C
    case, _ = _coupled_case()
    st = {"f64": C.LB_STORE_F64, "f32": C.LB_STORE_F32_DEV, "f16": C.LB_STORE_F16_DEV}[storage]
    flags = bench.launch_flags(C, st)
    _sampled_parity(case, storage, [((0, 0, 0), (13, 13, 1)), ((4090, 2000, 0), (13, 13, 1)),
                                    ((1000, 4091, 0), (13, 13, 1))], steps=4, flags=flags)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_coupled_4096_1000_steps_closed_form(storage):
    """1000 steps of the 4096^2 coupled workload from rest.  The force is a single
    Taylor-Green mode A (sin kx cos ky, -cos kx sin ky) cos(w t), whose nonlinear term
    is a pressure gradient, so u = a(t) (sin kx cos ky, -cos kx sin ky) with
    a' = -2 nu k^2 a + A cos(w t); the scalar, advected at |u| <~ 0.01 over a 4096
    wavelength, grows as phi = B sin kx sin ky times the integral of the source.  Both
    amplitudes are compared after projecting the fields on their modes.  Float16
    storage rounds stochastically: with rounding to nearest the scalar's per-step
    source share S/5 ~ 2e-7 falls below half a float16 unit once phi ~ 1e-3."""
    case, w = _coupled_case()
    A, B = w.extra["A"], w.extra["B"]
    n = 4096
    k = 2 * np.pi / n
    N = w.steps
    with case.gpu(storage) as s:
        s.init_equilibrium()
        s.step(N)
        rho, u, phi = s.moments(1)
        tot = s.totals()
    pts = coords(case.shape)
    mode = vortex_force_2d(case.shape, 1.0, pts)
    a_num = (u * mode).sum() / (mode * mode).sum()
    # a' = -lam a + A cos(w t), a(0) = 0, lam = 2 nu k^2: closed form
    lam, om = 2 * case.nu * k * k, w.force_omega
    a_exact = A * (lam * np.cos(om * N) + om * np.sin(om * N) - lam * np.exp(-lam * N)) / (lam**2 + om**2)
    _say(f"[fullsize] coupled {storage}: a = {a_num:.6e}, closed form {a_exact:.6e}")
    assert abs(a_num / a_exact - 1) < 2e-3
    smode = product_source_2d(case.shape, 1.0, pts)
    b_num = (phi * smode).sum() / (smode * smode).sum()
    lamp = 2 * case.D * k * k
    b_exact = B * (1 - np.exp(-lamp * N)) / lamp
    _say(f"[fullsize] coupled {storage}: phi amplitude = {b_num:.6e}, closed form {b_exact:.6e}")
    assert abs(b_num / b_exact - 1) < 2e-3
    # mass is conserved; the mode forces and sources sum to zero over the lattice.
    # Float16 stores rounded stochastically make the mass a random walk of
    # ~sqrt(9 N steps) = 4e5 rounding errors of ~1e-7 (measured: 0.03)
    assert abs(tot[0] - n * n) < {"f64": 1e-9, "f32": 1e-2, "f16": 0.2}[storage]
    assert np.abs(rho - 1).max() < 1e-3


def test_duct_256_benchmark_runs_against_the_startup_profile_and_float64():
    """The benchmark's own 256^3 duct runs (its launch configuration, graph runs
    and step count: 5 warm-up, 195 priming, 20 timed and 50 single steps from
    rest) against the duct's start-up profile (heat equation with a uniform
    source between two pairs of walls, Duhamel's integral of error functions)
    at t = steps + 1/2, and the float32 / float16 runs against the float64 run
    of the same steps.  Bounds: the measured errors with a margin of about 1.5;
    at this time the wall layers are about 5 nodes thick, so the error against
    the continuum profile is the layers' second-order discretisation error in
    every storage, float16 adding its stochastic-rounding noise."""
    import torch

    import bench
    from paper_1806_10247_amd import capi as C
    w = duct_3d(256)
    runs = {}
    for name, st in (("f64", C.LB_STORE_F64), ("f32", C.LB_STORE_F32_DEV), ("f16", C.LB_STORE_F16_DEV)):
        _say(f"[fullsize] 256^3 duct, {name}, benchmark configuration")
        runs[name] = bench.run_storage(torch, C, st, 20, 5)
    assert {r["steps_total"] for r in runs.values()} == {270}
    t = 270.5
    centre = float(runs["f64"]["u"][0].view(256, 256, 256)[128, 128, 0])
    assert abs(centre / (w.force[0] * t) - 1) < 1e-8      # the interior has not felt the walls
    vs_a = bench.duct_vs_analytic(torch, runs, 256, w.force[0], w.nu)
    vs_64 = bench.errors_vs_f64(runs)
    _say(f"[fullsize]   vs the start-up profile {vs_a}; vs float64 {vs_64}")
    for name, (l2, mx) in {"f64": (2.5e-3, 1e-2), "f32": (2.5e-3, 1e-2), "f16": (8e-3, 4.5e-2)}.items():
        assert vs_a[name]["rel_l2"] <= l2 and vs_a[name]["max_rel"] <= mx, (name, vs_a[name])
    assert vs_64["f32"]["rel_l2"] <= 1e-5 and vs_64["f32"]["max_rel"] <= 1e-5
    assert vs_64["f16"]["rel_l2"] <= 1.5e-2 and vs_64["f16"]["max_rel"] <= 5e-2
    # the layers are resolved: float32 and float64 agree with the profile equally well
    assert abs(vs_a["f32"]["rel_l2"] / vs_a["f64"]["rel_l2"] - 1) < 0.01
