"""GPU parity: the HIP library, driven through the C ABI, against the FP64 oracle.

FP64 storage must match the oracle to max-abs <= 1e-12 on the post-collision
populations after 1000 steps, for every lattice, periodic and walled, with
uniform and spatially varying forces/sources, constant and cos(w t) in time,
at sizes that span several blocks and end in ragged tails."""
import sys

import numpy as np
import pytest

import oracle as O
from casclb_inputs import coords, noise, product_source_2d, rng, vortex_force_2d
from lbcases import LAT_O as LAT_O_, Case, gpu_available, reduced_precision_bound

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a gfx950 GPU")]

TOL_F64 = 1e-12


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _field2d(shape, seed, amp=1e-4, comps=2):
    return noise((comps, int(np.prod(shape))), amp, seed=seed)


def parity_cases():
    g = rng(100)
    cases = [
        Case("D2Q9", (64, 48, 1), nu=0.04, omega_bulk=1.2, omega_third=0.8, omega_fourth=1.3,
             force_field=_field2d((64, 48, 1), 1), force_time=(O.TIME_COS, 0.01), seed=1),
        Case("D2Q9", (300, 45, 1), walls=(False, True, False), nu=0.1, force=(2e-5, -1e-5, 0.0), seed=2),
        Case("D2Q9", (5, 7, 1), walls=(True, True, False), nu=0.02, force=(1e-4, 3e-5, 0.0), seed=3),
        Case("D2Q9_D2Q5", (64, 40, 1), nu=0.06, D=0.02, omega_bulk=1.1, omega_phi_high=1.2,
             force_field=_field2d((64, 40, 1), 4), force_time=(O.TIME_COS, 0.02),
             source_field=noise(64 * 40, 1e-4, seed=5), source_time=(O.TIME_COS, 0.03), seed=4),
        Case("D2Q9_D2Q5", (37, 29, 1), walls=(False, True, False), nu=0.03, D=0.05, force=(1e-5, 0.0, 0.0),
             source=2e-5, seed=6),
        Case("D3Q27", (16, 16, 16), nu=0.05, omega_bulk=1.3, omega_third=0.9, omega_fourth=1.1,
             force_field=_field2d((16, 16, 16), 7, comps=3), seed=7),
        Case("D3Q27", (19, 13, 11), walls=(False, True, True), nu=(0.76 - 0.5) / 3, force=(1e-5, 0.0, 0.0), seed=8),
        Case("D3Q27", (7, 9, 5), walls=(True, True, True), nu=0.08, force=(1e-5, -2e-5, 3e-5),
             force_time=(O.TIME_COS, 0.05), seed=9),
        Case("D3Q15", (12, 10, 8), nu=0.05, omega_bulk=1.2, omega_third=0.9, omega_fourth=1.1,
             force_field=_field2d((12, 10, 8), 10, comps=3), force_time=(O.TIME_COS, 0.02), seed=10),
        Case("D3Q15", (9, 11, 7), walls=(True, True, True), nu=0.07, force=(2e-5, -1e-5, 1.5e-5), seed=11),
    ]
    return cases


@pytest.mark.parametrize("case", parity_cases(), ids=repr)
def test_f64_parity_1000_steps(case):
    _say("case", case)
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    dom.f[:] = f0
    if g0 is not None:
        dom.g[:] = g0
    with case.gpu("f64") as s:
        s.write_populations(f0, g0)
        f_back, g_back = s.populations()
        assert np.abs(f_back - f0).max() < 1e-15
        s.step(1000)
        dom.run(1000)
        f, g = s.populations()
        err = np.abs(f - dom.f).max()
        _say("  max|f - oracle| =", err)
        assert err <= TOL_F64, err
        if g is not None:
            errg = np.abs(g - dom.g).max()
            _say("  max|g - oracle| =", errg)
            assert errg <= TOL_F64, errg
        # macroscopic readout of the same state
        for kind in (0, 1):
            rho, u, phi = s.moments(kind)
            rho_o, u_o, phi_o = dom.moments(kind)
            assert np.abs(rho - rho_o).max() <= TOL_F64
            assert np.abs(u - u_o).max() <= TOL_F64
            if phi is not None:
                assert np.abs(phi - phi_o).max() <= TOL_F64
        tot = s.totals()
        tot_o = dom.totals()
        assert np.allclose(tot, tot_o, rtol=0, atol=1e-10 * max(1.0, np.abs(tot_o).max()))


@pytest.mark.parametrize("lattice,shape,walls", [("D2Q9", (70, 33, 1), (False, True, False)),
                                                 ("D2Q9_D2Q5", (33, 70, 1), (False, False, False)),
                                                 ("D3Q27", (12, 10, 9), (False, True, True)),
                                                 ("D3Q15", (11, 9, 10), (False, True, False))])
def test_init_equilibrium_matches_oracle(lattice, shape, walls):
    case = Case(lattice, shape, walls=walls)
    rho, u, phi = case.initial_fields()
    dom = case.oracle()
    dom.init_equilibrium(rho, u, phi)
    with case.gpu("f64") as s:
        s.init_equilibrium(rho, u, phi if lattice == "D2Q9_D2Q5" else None)
        f, g = s.populations()
        assert np.abs(f - dom.f).max() < 1e-15
        if g is not None:
            assert np.abs(g - dom.g).max() < 1e-15
        s.step(50)
        dom.run(50)
        f, g = s.populations()
        assert np.abs(f - dom.f).max() < TOL_F64


def _reduced_precision_bound(steps, storage, scale):
    return reduced_precision_bound(steps, storage, scale)


@pytest.mark.parametrize("storage,steps", [("f32", 1000), ("f16", 100), ("f16", 1000)])
@pytest.mark.parametrize("idx", [0, 3, 5, 6, 8])
def test_reduced_precision_error(storage, steps, idx):
    case = parity_cases()[idx]
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    dom.f[:] = f0
    if g0 is not None:
        dom.g[:] = g0
    with case.gpu(storage) as s:
        s.write_populations(f0, g0)
        s.step(steps)
        dom.run(steps)
        f, g = s.populations()
    # scale of the stored deviations |f - w rho0|
    feq_rest = O.flow_equilibrium({"D3Q27": O.D3Q27, "D3Q15": O.D3Q15}.get(case.lattice, O.D2Q9), 1.0, [0, 0, 0])
    scale = np.abs(dom.f - feq_rest[:, None]).max()
    err = np.abs(f - dom.f).max()
    bound = _reduced_precision_bound(steps, storage, scale)
    eps = 2.0**-11 if storage == "f16" else 2.0**-24
    _say(f"  {case} {storage} {steps} steps: max err {err:.3e} = {err / (eps * scale):.2f} eps scale "
         f"(bound {bound:.3e}, scale {scale:.3e})")
    assert err <= bound
    if g is not None:
        scale_g = np.abs(dom.g).max()
        assert np.abs(g - dom.g).max() <= _reduced_precision_bound(steps, storage, scale_g)


def test_edge_cases_small_and_degenerate():
    """nx = 1 periodic axis, a single node (D2Q9 1x1 periodic is a closed system),
    zero steps, and a lattice one node thick between walls."""
    for case in [Case("D2Q9", (1, 6, 1), walls=(False, True, False), force=(1e-4, 0, 0)),
                 Case("D2Q9", (1, 1, 1), force=(1e-4, 2e-4, 0)),
                 Case("D3Q27", (1, 1, 3), walls=(False, False, True), force=(1e-4, 0, 0)),
                 Case("D3Q27", (2, 1, 1), walls=(True, True, True), force=(0, 1e-4, 0)),
                 Case("D3Q15", (1, 1, 3), walls=(False, False, True), force=(1e-4, 0, 0)),
                 Case("D3Q15", (2, 1, 1), walls=(True, True, True), force=(0, 1e-4, 0))]:
        dom = case.oracle()
        f0, _ = case.perturbed_state(dom)
        dom.f[:] = f0
        with case.gpu("f64") as s:
            s.write_populations(f0)
            s.step(0)
            assert np.array_equal(s.populations()[0], s.populations()[0])
            s.step(200)
            dom.run(200)
            assert np.abs(s.populations()[0] - dom.f).max() <= TOL_F64, case


@pytest.mark.parametrize("idx", [1, 3, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_launch_shapes_agree(idx, storage):
    """Every legal block width, rows per thread, x-adjacent nodes per thread (16-bit storage,
    even nx, periodic x) and block order gives bit-identical results (the launch shape must
    not matter); odd row counts exercise the inactive last row."""
    from paper_1806_10247_amd import capi as C
    case = parity_cases()[idx]
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    pairs = storage == "f16" and case.shape[0] % 2 == 0 and not case.walls[0]
    ref = None
    shapes = [(64, 1, 0, 1), (128, 2, 0, 1), (192, 1, 0, 1), (256, 2, 0, 1), (256, 1, C.LB_FLAG_XCD_REMAP, 1),
              (64, 2, C.LB_FLAG_XCD_REMAP, 1)]
    if pairs:
        shapes += [(64, 1, 0, 2), (128, 1, C.LB_FLAG_XCD_REMAP, 2), (256, 1, 0, 2)]
    for bx, rows, flags, xp in shapes:
        with case.gpu(storage, block_x=bx, rows_per_thread=rows, flags=flags, residual_interval=7,
                      x_pairs=xp) as s:
            s.write_populations(f0, g0)
            s.step(20)
            f, g = s.populations()
            tot = s.residual()[2]
        if ref is None:
            ref = (f, g, tot)
        assert np.array_equal(f, ref[0]), (bx, rows, flags, xp, int((f != ref[0]).sum()),
                                           float(np.abs(f - ref[0]).max()))
        if g is not None:
            assert np.array_equal(g, ref[1])
        assert np.allclose(tot, ref[2], rtol=0, atol=1e-9)


@pytest.mark.parametrize("shape,walls", [((200, 9, 7), (False, True, True)), ((16, 6, 5), (False, False, True)),
                                         ((64, 5, 4), (False, False, False)), ((2, 3, 2), (False, True, True)),
                                         ((2, 1, 1), (False, False, False))])
def test_f16_d3q27_launch_shapes_agree(shape, walls):
    """Float16 D3Q27: block widths that split a row (a last block of 8 nodes or 36
    node pairs), one or two rows per thread, one or two x-adjacent nodes per thread,
    wall rows on y and z: bit-identical states, within the storage bound of the oracle."""
    from paper_1806_10247_amd import capi as C
    case = Case("D3Q27", shape, walls=walls, nu=0.07, force=(2e-5, -1e-5, 1e-5), seed=21)
    dom = case.oracle()
    f0, _ = case.perturbed_state(dom)
    ref = None
    for bx, rows, xp in [(64, 2, 1), (64, 1, 1), (128, 1, 1), (192, 1, 1), (256, 1, 1), (256, 2, 1), (64, 1, 2),
                         (128, 1, 2), (192, 1, 2), (256, 1, 2)]:
        with case.gpu("f16", block_x=bx, rows_per_thread=rows, x_pairs=xp) as s:
            s.write_populations(f0)
            s.step(20)
            f, _ = s.populations()
        if ref is None:
            ref = f
        assert np.array_equal(f, ref), (bx, rows, xp)
    dom.f[:] = f0
    dom.run(20)
    scale = np.abs(dom.f - O.flow_equilibrium(O.D3Q27, 1.0, [0, 0, 0])[:, None]).max()
    assert np.abs(ref - dom.f).max() <= _reduced_precision_bound(20, "f16", scale)


def test_checkpoint_resume_bit_identical():
    case = parity_cases()[3]
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    with case.gpu("f32") as a:
        a.write_populations(f0, g0)
        a.step(30)
        fa, ga = a.populations()
    with case.gpu("f32") as b:
        b.write_populations(f0, g0)
        b.step(17)
        fb, gb = b.populations()
    with case.gpu("f32") as c:
        c.write_populations(fb, gb)
        c.step_count = 17
        c.step(13)
        fc, gc = c.populations()
    assert np.array_equal(fa, fc) and np.array_equal(ga, gc)


def test_residual_and_totals_record():
    """The fused residual check: r = ||u^n - u^{n-K}|| / (K ||u^n||) of the half-forced
    velocity, and the mass/momentum/scalar of the state the checked step wrote."""
    from paper_1806_10247_amd import capi as C
    case = parity_cases()[4]
    K = 10
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    dom.f[:] = f0
    dom.g[:] = g0
    with case.gpu("f64", residual_interval=K) as s:
        s.write_populations(f0, g0)
        s.step(K)
        r, at, tot = s.residual()
        assert at == K and r == np.inf
        dom.run(K - 1)
        _, u_prev, _ = dom.moments(1)
        dom.run(1)
        assert np.allclose(tot, dom.totals(), rtol=0, atol=1e-10)
        dom.run(K - 1)
        _, u_now, _ = dom.moments(1)
        s.step(K)
        r, at, tot = s.residual()
        assert at == 2 * K
        want = np.sqrt(((u_now - u_prev) ** 2).sum()) / (K * np.sqrt((u_now**2).sum()))
        assert abs(r - want) <= 1e-9 * want
        dom.run(1)
        assert np.allclose(tot, dom.totals(), rtol=0, atol=1e-10)


def test_nonfinite_state_is_reported():
    """A NaN written from the host is caught by the next residual check and lb_step
    then refuses to continue (forced from the host; every kernel exits normally)."""
    from paper_1806_10247_amd import capi as C
    case = Case("D2Q9", (64, 8, 1), force=(1e-5, 0, 0))
    with case.gpu("f32", residual_interval=5) as s:
        s.init_equilibrium()
        f, _ = s.populations()
        f[3, 17] = np.nan
        s.write_populations(f)
        s.step(5)
        with pytest.raises(C.LbError) as e:
            s.residual()
        assert e.value.code == C.LB_ENONFINITE
        with pytest.raises(C.LbError) as e:
            s.step(1)
        assert e.value.code == C.LB_ENONFINITE


def test_error_paths():
    from paper_1806_10247_amd import capi as C
    case = Case("D2Q9", (8, 8, 1))
    with case.gpu("f64") as s:
        with pytest.raises(C.LbError) as e:
            s.step(1)   # not initialised
        assert e.value.code == C.LB_ESTATE
        with pytest.raises(C.LbError):
            s.set_source(1.0)   # no scalar lattice
        with pytest.raises(C.LbError):
            C.lb_set_force_time(s.ctx, 7, 0.0)
        s.init_equilibrium()
        with pytest.raises(C.LbError):
            C.lb_step(s.ctx, -1)
        with pytest.raises(C.LbError):
            C.lb_read_populations_box(s.ctx, (0, 0, 0), (0, 1, 1), np.empty((9, 1)))
        bad = np.zeros((2, 64))
        bad[0, 3] = np.inf
        with pytest.raises(C.LbError):
            s.set_force_field(bad)


def test_stacked_2d_slices_match_independent_oracles():
    """A 2D lattice with nz > 1 is a stack of independent lattices: every slice equals
    its own oracle lattice (own force and source fields, own initial state) after
    1000 float64 steps."""
    nx, ny, nz = 23, 17, 3
    n2 = nx * ny
    slices = []
    for z in range(nz):
        case = Case("D2Q9_D2Q5", (nx, ny, 1), walls=(False, True, False), nu=0.05, D=0.03, omega_bulk=1.1,
                    force_field=_field2d((nx, ny, 1), 20 + z), source_field=noise(n2, 1e-4, seed=30 + z), seed=40 + z)
        dom = case.oracle()
        f0, g0 = case.perturbed_state(dom)
        dom.f[:] = f0
        dom.g[:] = g0
        slices.append((case, dom, f0, g0))
    stack = Case("D2Q9_D2Q5", (nx, ny, nz), walls=(False, True, False), nu=0.05, D=0.03, omega_bulk=1.1,
                 force_field=np.concatenate([c._field(c.force_field) for c, *_ in slices], axis=1),
                 source_field=np.concatenate([c.source_field for c, *_ in slices]))
    with stack.gpu("f64") as s:
        s.write_populations(np.concatenate([f for *_, f, _ in slices], axis=1),
                            np.concatenate([g for *_, g in slices], axis=1))
        s.step(1000)
        f, g = s.populations()
    for z, (case, dom, _, _) in enumerate(slices):
        dom.run(1000)
        ef = np.abs(f[:, z * n2:(z + 1) * n2] - dom.f).max()
        eg = np.abs(g[:, z * n2:(z + 1) * n2] - dom.g).max()
        _say(f"  slice {z}: max |df| {ef:.2e}, |dg| {eg:.2e}")
        assert ef <= 1e-12 and eg <= 1e-12


def test_scalar_residual_record():
    """r_phi = ||phi^n - phi^{n-K}|| / (K ||phi^n||) of the half-sourced scalar, from
    the same fused check as the velocity residual."""
    case = parity_cases()[3]
    K = 10
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    dom.f[:] = f0
    dom.g[:] = g0
    with case.gpu("f64", residual_interval=K) as s:
        s.write_populations(f0, g0)
        s.step(K)
        assert s.residual_scalar() == np.inf
        dom.run(K - 1)
        _, _, phi_prev = dom.moments(1)
        dom.run(1)
        dom.run(K - 1)
        _, _, phi_now = dom.moments(1)
        s.step(K)
        r = s.residual_scalar()
        want = np.sqrt(((phi_now - phi_prev) ** 2).sum()) / (K * np.sqrt((phi_now**2).sum()))
        _say(f"  r_phi {r:.6e} want {want:.6e}")
        assert abs(r - want) <= 1e-9 * want


@pytest.mark.parametrize("idx", [1, 4, 9])   # constant force (and source)
def test_step_graphs_are_bit_identical(idx):
    """Runs of plain steps replayed from captured graphs (constant force and source)
    give the same bits as the same steps launched one by one (a cos(0 t) time
    factor: identical arithmetic, but arguments that may change every step)."""
    case = parity_cases()[idx]
    import copy
    slow = copy.copy(case)
    slow.force_time = (O.TIME_COS, 0.0)
    slow.source_time = (O.TIME_COS, 0.0)
    dom = case.oracle()
    f0, g0 = case.perturbed_state(dom)
    out = []
    for c in (case, slow):
        with c.gpu("f64", residual_interval=70) as s:
            s.write_populations(f0, g0)
            # full 64-step graphs, graphs of the rest of a run between checks (odd
            # and even lengths), and runs too short for a graph
            for n in (333, 400, 29, 97, 5, 140):
                s.step(n)
            out.append(s.populations())
            r = s.residual()
    assert np.array_equal(out[0][0], out[1][0])
    if out[0][1] is not None:
        assert np.array_equal(out[0][1], out[1][1])


def periodic_2d_cases():
    """Periodic 2D lattices with force and source fields constant in time (the
    warm start's kind), one of them a stack of three slices."""
    return [
        Case("D2Q9", (64, 48, 1), nu=0.04, omega_bulk=1.2, omega_third=0.8, omega_fourth=1.3,
             force_field=_field2d((64, 48, 1), 1), seed=21),
        Case("D2Q9_D2Q5", (64, 40, 1), nu=0.06, D=0.02, omega_bulk=1.1, omega_phi_high=1.2,
             force_field=_field2d((64, 40, 1), 4), source_field=noise(64 * 40, 1e-4, seed=5), seed=22),
        Case("D2Q9_D2Q5", (32, 8, 3), nu=0.1, D=0.05, force=(1e-5, -2e-5, 0.0), source=1e-5, seed=23),
    ]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("idx", range(3))
def test_periodic_2d_graph_runs_are_bit_identical(idx, storage):
    """Runs of plain steps replayed from the step graphs give the same bits as
    single steps launched one by one (a cos(0 t) time factor: identical
    arithmetic, but no graphs), over runs of both parities and lengths; float64
    single-slice lattices also match the oracle to 1e-12."""
    import copy
    case = periodic_2d_cases()[idx]
    slow = copy.copy(case)
    slow.force_time = (O.TIME_COS, 0.0)
    slow.source_time = (O.TIME_COS, 0.0)
    dom = case.oracle() if case.shape[2] == 1 else None
    flat = Case(case.lattice, (case.shape[0], case.shape[1] * case.shape[2], 1), seed=case.seed)
    f0, g0 = (case if dom is not None else flat).perturbed_state(dom if dom is not None else flat.oracle())
    out = []
    for c in (case, slow):
        with c.gpu(storage, residual_interval=70) as s:
            s.write_populations(f0, g0)
            for n in (333, 97, 29, 140):
                s.step(n)
            out.append(s.populations())
    assert np.array_equal(out[0][0], out[1][0])
    if out[0][1] is not None:
        assert np.array_equal(out[0][1], out[1][1])
    if dom is not None and storage == "f64":
        dom.f[:] = f0
        if g0 is not None:
            dom.g[:] = g0
        dom.run(599)
        assert np.abs(out[0][0] - dom.f).max() <= 1e-12
        if g0 is not None:
            assert np.abs(out[0][1] - dom.g).max() <= 1e-12


@pytest.mark.parametrize("lattice,shape", [("D2Q9_D2Q5", (12, 10, 1)), ("D2Q9", (9, 7, 1)), ("D3Q27", (6, 5, 4)),
                                           ("D3Q15", (6, 5, 4)), ("D2Q9_D2Q5", (8, 6, 3))])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_moment_reset_matches_host(lattice, shape, storage):
    """lb_reset_moments_device: every node's populations are shifted by the
    oracle's equilibrium of the target minus that of their own moments, so
    f - f_eq is kept and the stored moments become the target's."""
    import torch
    from paper_1806_10247_amd import capi as C
    case = Case(lattice, shape, seed=31)
    # a stack of 2D slices has the node order of one (nx, ny * nz) lattice, and the
    # reset is per node: its state comes from the oracle's lattice of that shape
    flat = Case(lattice, (shape[0], shape[1] * shape[2], 1), seed=31) if case.dims == 2 else case
    f0, g0 = flat.perturbed_state(flat.oracle())
    N, d = case.N, case.dims
    scalar = lattice == "D2Q9_D2Q5"
    g = np.random.default_rng(5)
    rho_t = 1.0 + 0.01 * g.standard_normal(N)
    u_t = 0.02 * g.standard_normal((d, N))
    phi_t = g.standard_normal(N) if scalar else None
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    R, U = dev(rho_t), dev(u_t)
    P = dev(phi_t) if scalar else None
    with case.gpu(storage) as s:
        s.write_populations(f0, g0)
        C.lb_reset_moments_device(s.ctx, R.data_ptr(), U.data_ptr(), P.data_ptr() if scalar else None)
        s.synchronize()
        f, gs = s.populations()
    lat = LAT_O_[lattice]
    E = O.velocities(lat).astype(np.float64)
    # float16 deviation storage: the written deviations round to 2^-11 of their size (<~ 0.05)
    tol = {"f64": 1e-14, "f32": 2e-6, "f16": 5e-5}[storage]
    for n in range(N):
        rho_s = f0[:, n].sum()
        u_s = E.T @ f0[:, n] / rho_s
        ut = np.zeros(3)
        ut[:d] = u_t[:, n]
        want = f0[:, n] - O.flow_equilibrium(lat, rho_s, u_s) + O.flow_equilibrium(lat, rho_t[n], ut)
        assert np.abs(f[:, n] - want).max() <= tol, n
        assert abs(f[:, n].sum() - rho_t[n]) <= 10 * tol
        assert np.abs(E.T @ f[:, n] - rho_t[n] * ut).max() <= 10 * tol
        if scalar:
            wg = g0[:, n] - O.scalar_equilibrium(g0[:, n].sum(), u_s[:2]) + O.scalar_equilibrium(phi_t[n], ut[:2])
            # the scalar populations are stored whole, not as deviations: in float16 both
            # the written input and the result round to 2^-11 of their own size
            tg = tol if storage != "f16" else 2.0**-10 * (np.abs(g0[:, n]).max() + np.abs(wg).max())
            assert np.abs(gs[:, n] - wg).max() <= tg, n
            assert abs(gs[:, n].sum() - phi_t[n]) <= 10 * tg


def test_moment_reset_rejects_bad_calls():
    from paper_1806_10247_amd import capi as C
    case = Case("D2Q9_D2Q5", (8, 6, 1))
    import torch
    d = torch.zeros(2 * case.N, dtype=torch.float64, device="cuda")
    with case.gpu("f64") as s:
        s.init_equilibrium()
        for args in ((None, d.data_ptr(), d.data_ptr()), (d.data_ptr(), None, d.data_ptr()),
                     (d.data_ptr(), d.data_ptr(), None)):
            with pytest.raises(C.LbError):
                C.lb_reset_moments_device(s.ctx, *args)
