"""Float16 deviation storage with stochastic rounding against float64 runs of
the same problems, and the rounding-to-nearest alternative.

At the square duct's force (Fx = 1e-7, Sec. 6) the per-step kick of a D3Q27
population, F/18 = 5.6e-9, is below half the smallest float16 subnormal
(2^-25 = 3.0e-8): rounded to nearest it is lost at every store and the duct
never leaves rest.  Rounded stochastically the expected stored value is the
float32 value, so the flow develops and follows the float64 run within the
storage's noise, and the momentum budget of eq. 27 (each step adds F per
node) holds on average."""
import sys

import numpy as np
import pytest

from lbcases import Case, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a gfx950 GPU")]

TAU = 0.76
NU = (TAU - 0.5) / 3.0


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _duct(storage, n, steps, **extra):
    from paper_1806_10247_amd.solver import Solver
    with Solver("D3Q27", (n, n, n), storage=storage, walls=(False, True, True), nu=NU, **extra) as s:
        s.init_equilibrium()
        s.set_force(1e-7, 0.0, 0.0)
        s.step(steps)
        _, u, _ = s.moments(1)
        tot = s.totals()
    return u, tot


@pytest.mark.parametrize("steps", [200, 2000])
def test_f16_duct_from_rest_develops_like_f64(steps):
    """64^3 duct from rest at Fx = 1e-7: the float16 run moves (the mean velocity
    and the momentum follow the float64 run within 0.1%) and its velocity field is
    within 3% (200 steps: u ~ 2e-5, a few float16 units of the deviations) and
    0.5% (2000 steps) of the float64 field in relative l2 norm."""
    n = 64
    u64, t64 = _duct("f64", n, steps)
    u16, t16 = _duct("f16", n, steps)
    rel = np.linalg.norm(u16 - u64) / np.linalg.norm(u64)
    _say(f"duct 64^3 f16 after {steps} steps: mean u {u16[0].mean():.5e} (f64 {u64[0].mean():.5e}), "
         f"momentum {t16[1]:.6e} (f64 {t64[1]:.6e}), rel l2 {rel:.3e}")
    assert abs(u16[0].mean() / u64[0].mean() - 1) < 1e-3
    assert abs(t16[1] / t64[1] - 1) < 1e-3
    assert rel < (3e-2 if steps == 200 else 5e-3)


@pytest.mark.parametrize("steps", [200, 2000])
def test_f32_duct_from_rest_follows_f64(steps):
    """The float32-deviation duct from rest at Fx = 1e-7 (the kicks, 5.6e-9, are far
    above float32's unit at these deviations): mean velocity and momentum within
    1e-5 of the float64 run, the velocity field within 1e-5 in relative l2 norm,
    bounds that do not grow with the step count."""
    n = 64
    u64, t64 = _duct("f64", n, steps)
    u32, t32 = _duct("f32", n, steps)
    rel = np.linalg.norm(u32 - u64) / np.linalg.norm(u64)
    _say(f"duct 64^3 f32 after {steps} steps: momentum {t32[1]:.9e} (f64 {t64[1]:.9e}), rel l2 {rel:.3e}")
    assert abs(u32[0].mean() / u64[0].mean() - 1) < 1e-5
    assert abs(t32[1] / t64[1] - 1) < 1e-5
    assert rel < 1e-5


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_momentum_budget_from_rest(storage):
    """Periodic 64^3 lattice from rest driven by a force field F(x) = 1e-7 (1 + 0.5
    sin(2 pi x / 64)) for 100 steps: the momentum gained must be k sum_x F (eq. 27).
    From rest the momenta stay below k max F = 1.5e-5, so float32 rounding
    (unit 6e-8 of them) allows a relative error of about 1e-6 (bound 1e-4); float16
    with stochastic rounding is unbiased, its random walk ~1% (bound 5%).  A kernel
    that rounded the kicks away would gain nothing."""
    from paper_1806_10247_amd.solver import Solver
    n = 64
    x = np.arange(n ** 3) % n
    fx = 1e-7 * (1.0 + 0.5 * np.sin(2 * np.pi * x / n))
    field = np.stack([fx, np.zeros_like(fx), np.zeros_like(fx)])
    with Solver("D3Q27", (n, n, n), storage=storage, nu=0.05) as s:
        s.init_equilibrium()
        s.set_force_field(field)
        t0 = s.totals()
        s.step(100)
        t1 = s.totals()
    gained, want = t1[1] - t0[1], 100 * fx.sum()
    _say(f"{storage} momentum gained from rest {gained:.9e}, k sum F = {want:.9e}")
    assert abs(gained / want - 1) < (1e-4 if storage == "f32" else 5e-2)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_steady_duct_45_against_the_series(storage):
    """The paper's square duct grid (3 x 45 x 45, tau = 0.76, Fx = 1e-7, Sec. 6)
    from rest for 40,000 steps (the slowest mode has decayed by e^-34): u_x against
    the steady Fourier series within the lattice's own discretisation error
    (relative l2 1.8e-3 in float64; bound 2.5e-3, float16 4e-3), and against the
    float64 run of the same steps (float32 2e-5, float16 5e-3)."""
    import bench
    from paper_1806_10247_amd.solver import Solver
    n, F = 45, 1e-7
    out = {}
    for st in dict.fromkeys(("f64", storage)):
        with Solver("D3Q27", (3, n, n), storage=st, walls=(False, True, True), nu=NU) as s:
            s.init_equilibrium()
            s.set_force(F, 0.0, 0.0)
            s.step(40000)
            _, u, _ = s.moments(1)
        out[st] = u[0].reshape(n, n, 3)[:, :, 0]
    ua = bench.duct_steady_series(n, F, NU)
    ux = out[storage]
    rel = np.linalg.norm(ux - ua) / np.linalg.norm(ua)
    vs64 = np.linalg.norm(ux - out["f64"]) / np.linalg.norm(out["f64"])
    _say(f"steady duct 45 {storage}: rel l2 vs series {rel:.3e}, vs f64 {vs64:.3e}")
    assert rel < (4e-3 if storage == "f16" else 2.5e-3)
    assert vs64 <= {"f64": 0.0, "f32": 2e-5, "f16": 5e-3}[storage]


def test_f16_momentum_budget_is_unbiased():
    """Periodic 64^3 lattice from a perturbed state (deviations ~ 3e-3, float16
    units ~ 1.5e-6), uniform Fx = 1e-7 for 100 steps: the momentum gained must be
    N k F (eq. 27) up to the random walk of the rounding errors (~0.6% here); a
    kernel that rounds the kicks away gains nothing."""
    from paper_1806_10247_amd.solver import Solver
    case = Case("D3Q27", (64, 64, 64), nu=0.05, seed=41)
    rho, u, _ = case.initial_fields()
    with Solver("D3Q27", case.shape, storage="f16", nu=0.05) as s:
        s.init_equilibrium(rho, u)
        s.set_force(1e-7, 0.0, 0.0)
        t0 = s.totals()
        s.step(100)
        t1 = s.totals()
    gained, want = t1[1] - t0[1], case.N * 100 * 1e-7
    _say(f"f16 momentum gained {gained:.6e}, N k F = {want:.6e}")
    assert abs(gained / want - 1) < 0.03


def test_f16_rounding_to_nearest_refuses_underflowing_forces():
    """LB_FLAG_F16_NEAREST: a force or source whose largest per-population change
    is below 2^-25 is refused (LB_EINVAL); larger ones are accepted; the default
    (stochastic rounding) accepts both."""
    from paper_1806_10247_amd import capi as C
    from paper_1806_10247_amd.solver import Solver
    with Solver("D3Q27", (8, 8, 8), storage="f16", nu=NU, flags=C.LB_FLAG_F16_NEAREST) as s:
        with pytest.raises(C.LbError) as e:
            s.set_force(1e-7, 0.0, 0.0)          # 1e-7 / 18 = 5.6e-9
        assert e.value.code == C.LB_EINVAL and "float16" in str(e.value)
        s.set_force(1e-6, 0.0, 0.0)              # 5.6e-8 > 3.0e-8
        with pytest.raises(C.LbError):
            s.set_force_field(np.full((3, 512), 1e-7))
        s.set_force(0.0, 0.0, 0.0)
    with Solver("D2Q9_D2Q5", (8, 8, 1), storage="f16", nu=0.1, D_phi=0.1, flags=C.LB_FLAG_F16_NEAREST) as s:
        with pytest.raises(C.LbError):
            s.set_source(1e-7)                   # S/5 = 2e-8
        s.set_source(1e-6)
    with Solver("D3Q27", (8, 8, 8), storage="f16", nu=NU) as s:
        s.set_force(1e-7, 0.0, 0.0)
        s.set_force_field(np.full((3, 512), 1e-9))


def test_f16_stochastic_rounding_repeats_and_varies_with_the_step():
    """The random bits depend on node, population and step only: the same start
    gives bit-identical runs, and restarting the step counter elsewhere changes
    the rounding (different bits, same statistics)."""
    case = Case("D3Q27", (24, 20, 18), walls=(False, True, True), nu=0.07, force=(2e-6, 0, 0), seed=43)
    dom = case.oracle()
    f0, _ = case.perturbed_state(dom)
    out = []
    for start in (0, 0, 1000):
        with case.gpu("f16") as s:
            s.write_populations(f0)
            s.step_count = start
            s.step(30)
            out.append(s.populations()[0])
    assert np.array_equal(out[0], out[1])
    assert not np.array_equal(out[0], out[2])
    assert np.abs(out[0] - out[2]).max() < 1e-4
