"""Pins of the oracle's D2Q5 scalar update (Sec. 5) against the basis of eq. (35),
the central-moment definitions and equilibria of eqs. (37)-(39), the source
budget of eqs. (44)/(46), and closed-form convection-diffusion solutions with
a source."""
import numpy as np

import oracle as O
from casclb_inputs import rng

# eq. (34)
EX = np.array([0, 1, 0, -1, 0], dtype=float)
EY = np.array([0, 0, 1, 0, -1], dtype=float)


def l_matrix():
    """Columns L0..L4 of eq. (35)/(36)."""
    one = np.ones(5)
    return np.stack([one, EX, EY, 5 * (EX**2 + EY**2) - 4 * one, EX**2 - EY**2], axis=1)


def central(g, ux, uy):
    cx, cy = EX - ux, EY - uy
    return np.array([(g * cx).sum(), (g * cy).sum(), (g * cx * cx).sum(), (g * cy * cy).sum()])


def test_l_basis_orthogonal():
    """Eq. (35) is orthogonal with norms (5,2,2,20,4) and <L_b|1> = 5 delta_b0 (used in eq. 46)."""
    L = l_matrix()
    assert np.allclose(L.T @ L, np.diag([5, 2, 2, 20, 4]))
    assert np.allclose(L.T @ np.ones(5), [5, 0, 0, 0, 0])


def test_eq48_rows_equal_L_times_h():
    g = rng(11)
    L = l_matrix()
    for _ in range(20):
        gg, h = g.standard_normal(5), g.standard_normal(5)
        assert np.allclose(O.d2q5_apply_l(gg, h) - gg, L @ h, atol=1e-14)


def test_equilibrium_central_moments_eq39():
    g = rng(12)
    for _ in range(10):
        phi, u = g.uniform(-2, 2), 0.1 * g.standard_normal(2)
        geq = O.scalar_equilibrium(phi, u)
        assert abs(geq.sum() - phi) < 1e-14
        k = central(geq, *u)
        assert np.allclose(k, [0, 0, phi / 3, phi / 3], atol=1e-14)


def test_source_budget_eq46():
    """The zeroth moment grows by exactly the step's source (eqs. 44, 46, 47); collision alone
    conserves it."""
    g = rng(13)
    for _ in range(20):
        gg = O.scalar_equilibrium(g.uniform(0.1, 2), 0.05 * g.standard_normal(2)) + 0.01 * g.standard_normal(5)
        spre, stot = 1e-3 * g.standard_normal(2)
        gp = O.d2q5_collide(gg, 0.05 * g.standard_normal(2), spre, stot, g.uniform(0.3, 1.9, 4))
        assert abs(gp.sum() - gg.sum() - stot) < 1e-15


def test_collision_relaxes_central_moments_with_corrected_sign():
    """With the u^2 phi terms of eq. (41) taken with a minus sign, the post-collision central
    moments (eq. 37, about the flow u, zeroth moment the source-kicked phi of eq. 43) are
    exactly (1 - w1) k_x, (1 - w2) k_y, trace -> trace + w3 (2 c^2 phi - trace),
    deviator -> (1 - w4) deviator, i.e. relaxed towards eq. (39).  With the printed plus sign
    the second-order ones are not: this is why the oracle uses the minus sign."""
    g = rng(14)
    for printed in (False, True):
        worst = 0.0
        for _ in range(20):
            ux, uy = 0.1 * g.standard_normal(2)
            phi0 = g.uniform(0.2, 2.0)
            gg = O.scalar_equilibrium(phi0, [0.03, -0.02]) + 0.02 * g.standard_normal(5)
            spre = 1e-2 * g.standard_normal()
            w = g.uniform(0.3, 1.9, 4)
            gp = O.d2q5_collide(gg, [ux, uy], spre, 0.0, w, printed_sign=printed)
            phi = gg.sum() + spre / 2
            # moments of the pre-collision state with the zeroth moment replaced by phi
            a = central(gg, ux, uy) + np.array([-ux, -uy, ux * ux, uy * uy]) * (phi - gg.sum())
            b = central(gp, ux, uy)   # collision conserves the zeroth moment of gp (stot = 0) ...
            b = b + np.array([-ux, -uy, ux * ux, uy * uy]) * (phi - gp.sum())   # ... which is replaced by phi too
            want = np.array([(1 - w[0]) * a[0], (1 - w[1]) * a[1], 0, 0])
            tr = a[2] + a[3] + w[2] * (2 * phi / 3 - a[2] - a[3])
            dv = (1 - w[3]) * (a[2] - a[3])
            want[2], want[3] = (tr + dv) / 2, (tr - dv) / 2
            worst = max(worst, np.abs(b - want).max())
        if printed:
            assert worst > 1e-4
        else:
            assert worst < 1e-14


def test_equilibrium_fixed_point():
    g = rng(15)
    for _ in range(5):
        u = 0.05 * g.standard_normal(2)
        geq = O.scalar_equilibrium(g.uniform(0.1, 2), u)
        gp = O.d2q5_collide(geq, u, 0.0, 0.0, g.uniform(0.3, 1.9, 4))
        assert np.abs(gp - geq).max() < 1e-15


def _advected_source_run(printed, U=(0.05, 0.03), D=0.02, N=64, B=1e-4, steps=(500, 1000)):
    i = np.arange(N)
    X, Y = np.meshgrid(i, i, indexing="xy")
    kx = ky = 2 * np.pi / N
    S = B * np.sin(kx * X + ky * Y)
    d = O.Domain(O.D2Q9_D2Q5, N, N, nu=0.05, D=D, source_field=S.ravel(), d2q5_printed_sign=printed)
    u = np.zeros((2, N * N))
    u[0], u[1] = U
    d.init_equilibrium(u=u)
    lam = D * (kx * kx + ky * ky) + 1j * (kx * U[0] + ky * U[1])
    errs = []
    done = 0
    for t in steps:
        d.run(t - done)
        done = t
        ph = (-1j * B) / lam * (1 - np.exp(-lam * t))
        phia = np.real(ph * np.exp(1j * (kx * X + ky * Y))).ravel()
        _, uu, phi = d.moments(1)
        assert np.abs(uu[0] - U[0]).max() < 1e-15   # uniform flow stays exactly uniform
        errs.append(np.sqrt(((phi - phia) ** 2).sum() / (phia**2).sum()))
    return errs


def test_uniform_advection_with_source_closed_form():
    """Uniform velocity U (flow at rest in its frame, no force) and source B sin(k.x): each
    Fourier mode obeys dphi/dt = -(D k^2 + i k.U) phi + S, D = (tau_phi - 1/2)/3 (Sec. 6), so
    phi(t) = Re{ S^/lambda (1 - e^{-lambda t}) e^{i k.x} } with S^ = -i B."""
    errs = _advected_source_run(False)
    assert max(errs) < 3e-3, errs


def test_printed_sign_gives_velocity_dependent_diffusivity():
    """A pure-diffusion mode (no source) advected by a strong uniform U = (0.2, 0) along its
    wave vector decays at D k^2 with the corrected sign; the printed sign changes the decay by
    a U^2-dependent amount (anisotropic diffusivity error)."""
    N, D = 32, 0.05
    kx = 2 * np.pi / N
    rates = {}
    for printed in (False, True):
        i = np.arange(N)
        X, Y = np.meshgrid(i, i, indexing="xy")
        d = O.Domain(O.D2Q9_D2Q5, N, N, nu=0.05, D=D, d2q5_printed_sign=printed)
        u = np.zeros((2, N * N))
        u[0] = 0.2
        d.init_equilibrium(u=u, phi=(np.cos(kx * X)).ravel())
        amps = []
        for _ in range(2):
            d.run(200)
            _, _, phi = d.moments(0)
            c = np.fft.fft2(phi.reshape(N, N))[0, 1] / (N * N) * 2
            amps.append(abs(c))
        rates[printed] = np.log(amps[0] / amps[1]) / 200
    exact = D * kx * kx
    assert abs(rates[False] / exact - 1) < 2e-2, rates
    assert abs(rates[True] / exact - 1) > 5 * abs(rates[False] / exact - 1), rates


def test_scalar_budget_on_domain():
    """Periodic domain: the scalar total grows by exactly sum_x S_tot(x) per step."""
    g = rng(16)
    nx, ny = 9, 8
    S = 1e-3 * g.standard_normal(nx * ny)
    w = 0.3
    d = O.Domain(O.D2Q9_D2Q5, nx, ny, nu=0.05, D=0.03, source_field=S, source_time=(O.TIME_COS, w),
                 force=(1e-4, -2e-4))
    d.init_equilibrium(1 + 0.01 * g.standard_normal(nx * ny), 0.03 * g.standard_normal((2, nx * ny)),
                       g.uniform(0.5, 1.5, nx * ny))
    for n in range(4):
        t0 = d.totals()[4]
        cp, cq = O.time_factors(O.TIME_COS, w, n)
        d.run(1)
        assert abs(d.totals()[4] - t0 - 0.5 * (cp + cq) * S.sum()) < 1e-13
