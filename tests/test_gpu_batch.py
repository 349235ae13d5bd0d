"""Batched independent Hartmann channels on the GPU (one persistent launch),
against the oracle domain by domain, against the analytic Hartmann profile
with the velocity-dependent Lorentz force, and for graph replay and the
autotuner leaving the state unchanged."""
import sys

import numpy as np
import pytest

import oracle as O
from casclb_inputs import hartmann_batch
from lbcases import gpu_available, reduced_precision_bound

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a gfx950 GPU")]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle(d, steps):
    nx, ny, nu, fb, s = d[:5]
    dom = O.Domain(O.D2Q9, nx, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force=(fb, 0.0), lorentz=s)
    dom.init_equilibrium()
    dom.run(steps)
    return dom


def _batch(domains, storage, **cfg):
    from paper_1806_10247_amd import capi as C
    st = {"f64": C.LB_STORE_F64, "f32": C.LB_STORE_F32_DEV}[storage]
    c = C.lb_batch_config_default(storage=st, check_interval=cfg.pop("check_interval", 50), **cfg)
    b = C.lb_batch_create(c, [d[:5] for d in domains])
    C.lb_batch_init(b)
    return b


# sizes both below and above the LDS budget (f64: about 1100 nodes, f32: about 2200)
SMALL = [(4, 16, 0.05, 3e-5, 0.0), (7, 33, 0.12, 1e-5, 2e-3), (64, 16, 0.03, 2e-5, 5e-4),
         (40, 40, 0.08, 1e-5, 1e-3), (13, 97, 0.02, 5e-6, 0.0), (64, 70, 0.15, 1e-5, 3e-3),
         (1, 20, 0.1, 1e-5, 1e-3)]


@pytest.mark.parametrize("storage,lds_policy", [("f64", 0), ("f64", 1), ("f32", 0)])
def test_batch_matches_oracle(storage, lds_policy):
    from paper_1806_10247_amd import capi as C
    steps = 300
    b = _batch(SMALL, storage, lds_policy=lds_policy, block=256)
    try:
        C.lb_batch_run(b, steps, 0.0)
        st, res, status = C.lb_batch_results(b, len(SMALL))
        assert np.all(st == steps), st
        assert np.all(status == C.LB_BATCH_MAX_STEPS), status
        for i, d in enumerate(SMALL):
            dom = _oracle(d, steps)
            f = np.empty((9, d[0] * d[1]))
            C.lb_batch_read_populations(b, i, f)
            err = np.abs(f - dom.f).max()
            scale = np.abs(dom.f - O.flow_equilibrium(O.D2Q9, 1.0, [0, 0])[:, None]).max()
            _say(f"  batch {storage} lds={lds_policy} domain {d[:2]}: max err {err:.3e} (deviation scale {scale:.2e})")
            if storage == "f64":
                assert err <= 1e-12
            else:
                assert err <= reduced_precision_bound(steps, "f32", scale)
            rho = np.empty(d[0] * d[1])
            u = np.empty((2, d[0] * d[1]))
            C.lb_batch_read_moments(b, i, rho, u)
            rho_o, u_o, _ = dom.moments(1)
            if storage == "f64":
                assert np.abs(u - u_o).max() <= 1e-12
            else:
                # u_x sums six populations (|e_x| = 1) of the state checked above, then
                # the float32 moment kernel rounds a nine-term sum and one division
                umax = np.abs(u_o).max()
                assert np.abs(u - u_o).max() <= 6 * err + 2.0**-24 * (16 * scale + 8 * umax)
    finally:
        C.lb_batch_destroy(b)


def test_batch_graph_replay_continues_the_run():
    """Two replays of the captured graph (N steps each) equal 2N oracle steps."""
    from paper_1806_10247_amd import capi as C
    doms = SMALL[:4]
    b = _batch(doms, "f64")
    try:
        C.lb_batch_run(b, 150, 0.0)
        C.lb_batch_results(b, len(doms))
        C.lb_batch_run(b, 150, 0.0)
        C.lb_batch_results(b, len(doms))
        for i, d in enumerate(doms):
            f = np.empty((9, d[0] * d[1]))
            C.lb_batch_read_populations(b, i, f)
            assert np.abs(f - _oracle(d, 300).f).max() <= 1e-12
    finally:
        C.lb_batch_destroy(b)


def test_batch_hartmann_steady_profiles():
    """Run a seeded batch of Hartmann channels to r < 1e-8 (float64 storage) and compare each
    steady profile with u = F_b/s (1 - cosh(Ha y/L)/cosh Ha) (Poiseuille when Ha = 0)."""
    from paper_1806_10247_amd import capi as C
    # Hartmann layers resolved by >= 4 nodes (the oracle's own error is below 1.5% there)
    doms = hartmann_batch(24, seed=3, nx_range=(2, 8), ny_range=(32, 48), ha_range=(0.0, 4.0),
                          nu_range=(0.1, 0.2))
    b = _batch(doms, "f64", check_interval=100)
    try:
        C.lb_batch_run(b, 400000, 1e-8)
        st, res, status = C.lb_batch_results(b, len(doms))
        assert np.all(status == C.LB_BATCH_CONVERGED), (status, res)
        worst = 0.0
        for i, d in enumerate(doms):
            nx, ny, nu, fb, s, ha = d
            L = ny / 2
            y = np.arange(ny) + 0.5 - L
            if ha < 1e-9:
                ua = fb * L * L / (2 * nu) * (1 - (y / L) ** 2)
            else:
                ua = fb / s * (1 - np.cosh(ha * y / L) / np.cosh(ha))
            rho = np.empty(nx * ny)
            u = np.empty((2, nx * ny))
            C.lb_batch_read_moments(b, i, rho, u)
            uc = u[0].reshape(ny, nx)[:, 0]
            err = np.sqrt(((uc - ua) ** 2).sum() / (ua**2).sum())
            worst = max(worst, err)
            assert err < 2.5e-2, (d, err)
            if i < 3:
                # the steady state the oracle reaches from the analytic profile
                dom = O.Domain(O.D2Q9, nx, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force=(fb, 0.0), lorentz=s)
                u0 = np.zeros((2, nx * ny))
                u0[0] = np.tile(ua[:, None], (1, nx)).ravel()
                dom.init_equilibrium(u=u0)
                dom.run(int(12 * L * L / nu))
                _, uo, _ = dom.moments(1)
                assert np.abs(u[0] - uo[0]).max() < 1e-5 * np.abs(uo[0]).max(), d
        _say(f"  hartmann batch: steps {st.min()}..{st.max()}, worst relative l2 error {worst:.3e}")
    finally:
        C.lb_batch_destroy(b)


def test_batch_autotune_keeps_state():
    from paper_1806_10247_amd import capi as C
    doms = SMALL
    b = _batch(doms, "f32")
    try:
        C.lb_batch_run(b, 100, 0.0)
        C.lb_batch_results(b, len(doms))
        before = []
        for i, d in enumerate(doms):
            f = np.empty((9, d[0] * d[1]))
            C.lb_batch_read_populations(b, i, f)
            before.append(f)
        blk, pol, ms = C.lb_batch_autotune(b, 50)
        assert blk in (256, 512, 1024) and pol in (0, 1) and ms > 0
        for i, d in enumerate(doms):
            f = np.empty((9, d[0] * d[1]))
            C.lb_batch_read_populations(b, i, f)
            assert np.array_equal(f, before[i])
    finally:
        C.lb_batch_destroy(b)


def test_batch_rejects_bad_input():
    from paper_1806_10247_amd import capi as C
    c = C.lb_batch_config_default()
    for bad in [[(0, 10, 0.1, 0, 0)], [(4, 10, -0.1, 0, 0)], [(4, 10, 0.1, 0, -1.0)], [(2048, 1024, 0.1, 0, 0)]]:
        with pytest.raises(C.LbError) as e:
            C.lb_batch_create(c, bad)
        assert e.value.code == C.LB_EINVAL
    c.check_interval = 0
    with pytest.raises(C.LbError):
        C.lb_batch_create(c, [(4, 10, 0.1, 0, 0)])
    # compute units for routed domains: not negative, and some must stay with the persistent launch
    for routed, routed_cus in ((1, -1), (1, 100000)):
        c = C.lb_batch_config_default(routed=routed, routed_cus=routed_cus)
        with pytest.raises(C.LbError) as e:
            C.lb_batch_create(c, [(4, 10, 0.1, 0, 0), (4, 12, 0.1, 0, 0)])
        assert e.value.code == C.LB_EINVAL


@pytest.mark.parametrize("lattice", ["D2Q9", "D2Q9_D2Q5"])
def test_lattice_lorentz_force_matches_oracle(lattice):
    """lb_set_lorentz on an ordinary context (the implicit-midpoint Lorentz force of
    the batched solver on the multi-workgroup step kernel): 1000 float64 steps of a
    walled channel from a perturbed state against the oracle, populations and the
    half-forced velocity (whose x part is (j_x + F/2)/(rho + s/2)) <= 1e-12."""
    from lbcases import Case
    s_l = 3e-3
    case = Case(lattice, (12, 37, 1), walls=(False, True, False), nu=0.07, D=0.05, force=(2e-5, 0.0, 0.0),
                source=1e-5, seed=61)
    dom = O.Domain(O.D2Q9_D2Q5 if lattice == "D2Q9_D2Q5" else O.D2Q9, 12, 37, bc=(O.PERIODIC, O.BOUNCE_BACK),
                   nu=0.07, D=0.05 if lattice == "D2Q9_D2Q5" else None, force=(2e-5, 0.0),
                   source=1e-5 if lattice == "D2Q9_D2Q5" else 0.0, lorentz=s_l)
    f0, g0 = case.perturbed_state(dom)
    dom.f[:] = f0
    if g0 is not None:
        dom.g[:] = g0
    with case.gpu("f64") as s:
        s.set_lorentz(s_l)
        s.write_populations(f0, g0)
        s.step(1000)
        f, g = s.populations()
        _, u, _ = s.moments(1)
    dom.run(1000)
    _, u_o, _ = dom.moments(1)
    assert np.abs(f - dom.f).max() <= 1e-12
    if g is not None:
        assert np.abs(g - dom.g).max() <= 1e-12
    assert np.abs(u - u_o).max() <= 1e-12


def test_routed_domains_match_the_persistent_run():
    """routed = 3: the three domains of longest expected time are stepped by
    ordinary launches (one per step, 256-node workgroups) beside the persistent
    launch, which covers all compute units or leaves 96 of them to the routed
    launches.  Float64, to a 1e-8 residual: every domain stops at the same step
    with the same status as in the all-persistent run, its populations agree to
    1e-12, and a routed domain's 300 fixed steps equal the oracle's."""
    from paper_1806_10247_amd import capi as C
    doms = hartmann_batch(12, seed=5, nx_range=(2, 8), ny_range=(24, 40), ha_range=(0.0, 4.0),
                          nu_range=(0.1, 0.2))
    out = []
    for routed, routed_cus in ((0, 0), (3, 0), (3, 96)):
        b = _batch(doms, "f64", check_interval=100, routed=routed, routed_cus=routed_cus)
        try:
            C.lb_batch_run(b, 400000, 1e-8)
            st, res, status = C.lb_batch_results(b, len(doms))
            pops = []
            for i, d in enumerate(doms):
                f = np.empty((9, d[0] * d[1]))
                C.lb_batch_read_populations(b, i, f)
                pops.append(f)
            out.append((st, status, pops))
        finally:
            C.lb_batch_destroy(b)
    st0, s0, p0 = out[0]
    assert np.all(s0 == C.LB_BATCH_CONVERGED)
    for st1, s1, p1 in out[1:]:
        assert np.array_equal(s0, s1)
        assert np.array_equal(st0, st1), (st0, st1)
        assert max(np.abs(a - c).max() for a, c in zip(p0, p1)) <= 1e-12
    # fixed steps on the routed path against the oracle
    d = SMALL[5]
    b = _batch([d], "f64", routed=1)
    try:
        C.lb_batch_run(b, 300, 0.0)
        st, _, status = C.lb_batch_results(b, 1)
        assert st[0] == 300 and status[0] == C.LB_BATCH_MAX_STEPS
        f = np.empty((9, d[0] * d[1]))
        C.lb_batch_read_populations(b, 0, f)
        assert np.abs(f - _oracle(d, 300).f).max() <= 1e-12
    finally:
        C.lb_batch_destroy(b)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_all_routed_fixed_steps_are_bit_identical(storage):
    """Every domain routed (the persistent launch has none), an odd check
    interval (7: check intervals alternate the buffer parity) and a step limit
    that is not a multiple of it (the steps after the last check, then the
    limit's status): the populations are bit-identical to the all-persistent
    run (the same node update), steps and statuses equal, residuals equal to
    rounding (another summation order)."""
    from paper_1806_10247_amd import capi as C
    doms = hartmann_batch(9, seed=8, nx_range=(2, 40), ny_range=(16, 80), ha_range=(0.0, 6.0), nu_range=(0.05, 0.2))
    out = []
    for routed in (0, len(doms)):
        b = _batch(doms, storage, check_interval=7, routed=routed)
        try:
            C.lb_batch_run(b, 299, 0.0)
            st, res, status = C.lb_batch_results(b, len(doms))
            pops = []
            for i, d in enumerate(doms):
                f = np.empty((9, d[0] * d[1]))
                C.lb_batch_read_populations(b, i, f)
                pops.append(f)
            out.append((st, res, status, pops))
        finally:
            C.lb_batch_destroy(b)
    (st0, r0, s0, p0), (st1, r1, s1, p1) = out
    assert np.all(st0 == 299) and np.array_equal(st0, st1)
    assert np.all(s0 == C.LB_BATCH_MAX_STEPS) and np.array_equal(s0, s1)
    assert np.allclose(r0, r1, rtol=1e-9, atol=0)
    for a, c in zip(p0, p1):
        assert np.array_equal(a, c)
