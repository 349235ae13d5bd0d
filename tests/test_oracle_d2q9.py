"""Pins of the oracle's D2Q9 flow update (Sec. 4) against what the paper and
the mathematics fix: the basis of eq. (17), the central-moment definitions and
equilibria of eqs. (19)-(21), the momentum budget of eq. (27), fixed points,
an all-rates-equal closed form, and the Poiseuille, four-rolls-mill and
Hartmann benchmarks of Sec. 6."""
import numpy as np
import pytest

import oracle as O
from casclb_inputs import rng

# eq. (15), written out independently of the oracle
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def k_matrix():
    """Columns K0..K8 of eq. (17)/(18)."""
    one = np.ones(9)
    cols = [one, EX, EY, 3 * (EX**2 + EY**2) - 4 * one, EX**2 - EY**2, EX * EY,
            -3 * EX**2 * EY + 2 * EY, -3 * EX * EY**2 + 2 * EX, 9 * EX**2 * EY**2 - 6 * (EX**2 + EY**2) + 4 * one]
    return np.stack(cols, axis=1)


def near_eq(g, rho_s=0.05, u_s=0.05, noise=0.01):
    rho = 1 + rho_s * g.standard_normal()
    u = u_s * g.standard_normal(2)
    return O.flow_equilibrium(O.D2Q9, rho, u) + noise * g.standard_normal(9)


def pseudo_central(f, ux, uy, rho):
    """Central moments about u of eq. (19) with the first raw moments replaced by rho*u."""
    cx, cy = EX - ux, EY - uy
    out = {}
    # sum f (e-u)^m: expand and replace first raw moments by rho u
    jx, jy = (f * EX).sum(), (f * EY).sum()
    for (m, n) in [(2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]:
        v = (f * cx**m * cy**n).sum()
        # correction for the replaced first raw moments: d/dj of the expansion
        # of sum f (e_x-u_x)^m (e_y-u_y)^n is the coefficient of e_x (resp. e_y)
        coef_x = m * (-ux) ** (m - 1) * (-uy) ** n if m >= 1 else 0.0
        coef_y = n * (-uy) ** (n - 1) * (-ux) ** m if n >= 1 else 0.0
        v += coef_x * (rho * ux - jx) + coef_y * (rho * uy - jy)
        out[(m, n)] = v
    return out


def test_k_basis_orthogonal():
    """Eq. (17) is orthogonal with norms (9,6,6,36,4,4,12,12,36); <K_b|e_x> = 6 delta_b1 (eq. 29)."""
    K = k_matrix()
    G = K.T @ K
    assert np.allclose(G, np.diag([9, 6, 6, 36, 4, 4, 12, 12, 36]))
    assert np.allclose(K.T @ EX, [0, 6, 0, 0, 0, 0, 0, 0, 0])
    assert np.allclose(K.T @ EY, [0, 0, 6, 0, 0, 0, 0, 0, 0])


def test_eq32_rows_equal_K_times_g():
    """The printed post-collision rows (eq. 32) are f + K g with K of eq. (17)."""
    g = rng(1)
    K = k_matrix()
    for _ in range(20):
        f = g.standard_normal(9)
        gh = g.standard_normal(9)
        assert np.allclose(O.d2q9_apply_k(f, gh) - f, K @ gh, atol=1e-13)


def test_equilibrium_central_moments_eq20():
    """The product-form initial equilibrium has exactly the central moments of eq. (20)."""
    g = rng(2)
    for _ in range(10):
        rho, u = 1 + 0.1 * g.standard_normal(), 0.1 * g.standard_normal(2)
        f = O.flow_equilibrium(O.D2Q9, rho, u)
        cx, cy = EX - u[0], EY - u[1]
        want = {(0, 0): rho, (1, 0): 0, (0, 1): 0, (2, 0): rho / 3, (0, 2): rho / 3, (1, 1): 0,
                (2, 1): 0, (1, 2): 0, (2, 2): rho / 9}
        for (m, n), v in want.items():
            assert abs((f * cx**m * cy**n).sum() - v) < 1e-14


def test_collision_relaxes_pseudo_central_moments():
    """Eq. (23), evaluated at the half-forced u of eq. (25), relaxes the central moments
    (eq. 19, first raw moments taken as rho*u) towards eq. (20) with omega_3..omega_8:
    trace with w3, xx-yy with w4, xy with w5, xxy w6, xyy w7, xxyy w8."""
    g = rng(3)
    for _ in range(30):
        f = near_eq(g)
        fpre = 1e-3 * g.standard_normal(2)
        ftot = 1e-3 * g.standard_normal(2)
        w = g.uniform(0.3, 1.9, size=6)
        fp, u = O.d2q9_collide(f, fpre, ftot, w)
        rho = f.sum()
        assert np.allclose(u, ((f * EX).sum() + fpre[0] / 2) / rho * np.array([1, 0]) +
                           ((f * EY).sum() + fpre[1] / 2) / rho * np.array([0, 1]), atol=1e-15)
        fc = fp - (ftot[0] * EX + ftot[1] * EY) / 6.0       # remove the post-collision kick (eq. 31)
        a = pseudo_central(f, u[0], u[1], rho)
        b = pseudo_central(fc, u[0], u[1], rho)
        tr_a, tr_b = a[(2, 0)] + a[(0, 2)], b[(2, 0)] + b[(0, 2)]
        assert abs(tr_b - (tr_a + w[0] * (2 * rho / 3 - tr_a))) < 1e-14
        dv_a, dv_b = a[(2, 0)] - a[(0, 2)], b[(2, 0)] - b[(0, 2)]
        assert abs(dv_b - (1 - w[1]) * dv_a) < 1e-14
        assert abs(b[(1, 1)] - (1 - w[2]) * a[(1, 1)]) < 1e-14
        assert abs(b[(2, 1)] - (1 - w[3]) * a[(2, 1)]) < 1e-14
        assert abs(b[(1, 2)] - (1 - w[4]) * a[(1, 2)]) < 1e-14
        assert abs(b[(2, 2)] - (a[(2, 2)] + w[5] * (rho / 9 - a[(2, 2)]))) < 1e-14


def test_node_mass_and_momentum_budget_eq27():
    """Mass is unchanged and the momentum changes by exactly the step's force (eq. 27)."""
    g = rng(4)
    for _ in range(30):
        f = near_eq(g)
        fpre, ftot = 1e-3 * g.standard_normal(2), 1e-3 * g.standard_normal(2)
        fp, _ = O.d2q9_collide(f, fpre, ftot, g.uniform(0.3, 1.9, size=6))
        assert abs(fp.sum() - f.sum()) < 1e-15
        assert abs((fp * EX).sum() - (f * EX).sum() - ftot[0]) < 1e-16
        assert abs((fp * EY).sum() - (f * EY).sum() - ftot[1]) < 1e-16


def test_fixed_points():
    """With no force, the rest state and any uniform-flow equilibrium are unchanged."""
    g = rng(5)
    w = g.uniform(0.3, 1.9, size=6)
    for rho, u in [(1.0, (0.0, 0.0)), (1.03, (0.04, -0.02)), (0.97, (-0.08, 0.05))]:
        f = O.flow_equilibrium(O.D2Q9, rho, u)
        fp, _ = O.d2q9_collide(f, [0, 0], [0, 0], w)
        assert np.abs(fp - f).max() < 1e-15   # a few ulps of f ~ 0.5


def test_all_rates_equal_closed_form():
    """With all rates equal to W the update equals f - W (f~ - f_eq(rho, u)) + F.e/6, where
    f~ adds F.e/4 on the four axis links (a closed form independent of eq. 23's cascade)."""
    g = rng(6)
    for _ in range(20):
        W = g.uniform(0.3, 1.9)
        f = near_eq(g)
        F = 1e-3 * g.standard_normal(2)
        fp, u = O.d2q9_collide(f, F, F, [W] * 6)
        axis = (np.abs(EX) + np.abs(EY)) == 1
        ft = f + np.where(axis, (F[0] * EX + F[1] * EY) / 4, 0.0)
        want = f - W * (ft - O.flow_equilibrium(O.D2Q9, f.sum(), u)) + (F[0] * EX + F[1] * EY) / 6
        assert np.abs(fp - want).max() < 1e-15


def test_time_factors_trapezoid():
    """Half-step trapezoidal averages of cos(w t): their running sum approximates the integral
    of cos over [0, N] to second order; the constant mode gives exactly 1."""
    assert O.time_factors(O.TIME_CONSTANT, 0.3, 17) == (1.0, 1.0)
    w = 2 * np.pi / 1000
    N = 700
    s = sum(0.5 * sum(O.time_factors(O.TIME_COS, w, n)) for n in range(N))
    # composite trapezoid with h = 1/2: |error| <= (b - a) h^2 max|f''| / 12 = N w^2 / 48
    assert abs(s - np.sin(w * N) / w) <= N * w**2 / 48
    a, b = O.time_factors(O.TIME_COS, w, 0)
    assert a > b > 0 and a <= 1.0


def _poiseuille_startup(y, L, nu, F, t):
    eta = (y - L) / L
    s = 1 - eta**2
    for n in range(400):
        k = 2 * n + 1
        s -= 32 * (-1) ** n / (k**3 * np.pi**3) * np.cos(k * np.pi * eta / 2) * np.exp(-k * k * np.pi**2 * nu * t / (4 * L * L))
    return F * L * L / (2 * nu) * s


def test_poiseuille_channel_4x64():
    """Body-force Poiseuille flow (Sec. 6) on 4 x 64, periodic x, halfway bounce-back walls,
    Fx = 1e-6, nu = 1/6, 20000 steps: the interior profile has exact second difference
    -F/(rho nu) (a parabola), follows the start-up Fourier series up to a constant wall slip,
    and the mass is conserved while momentum grows by N F minus the wall exchange."""
    nu, F, ny = 1.0 / 6.0, 1e-6, 64
    d = O.Domain(O.D2Q9, 4, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force=(F, 0))
    d.init_equilibrium()
    m0 = d.totals()
    d.run(20000)
    _, u, _ = d.moments(1)
    ux = d.grid(u[0])[0, :, 0]
    assert np.allclose(d.grid(u[0])[0], ux[:, None], atol=1e-18)   # x-invariant
    y = np.arange(ny) + 0.5
    ua = _poiseuille_startup(y, ny / 2, nu, F, 20000)
    err = ux - ua
    # constant slip offset, well below 1e-3 of the centre-line velocity
    assert np.ptp(err) < 2e-9 * 3  # the start-up series itself is time-accurate to O(dt)
    assert abs(err.mean()) < 1e-3 * ua.max()
    # a parabola in the steady limit: continue to steady state
    d.run(80000)
    _, u, _ = d.moments(1)
    ux = d.grid(u[0])[0, :, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    assert np.allclose(d2, -F / nu, rtol=1e-9)
    m1 = d.totals()
    assert abs(m1[0] - m0[0]) < 1e-11


def test_poiseuille_diffusive_convergence():
    """Grid convergence under diffusive scaling (Sec. 6, tau = 0.55, Re = 100): the relative
    l2 error of eq. (sca) falls with slope 2 (the paper reports 2.00)."""
    tau = 0.55
    nu = (tau - 0.5) / 3
    Hs = (15, 31, 61)
    errs = []
    for H in Hs:
        L = H / 2
        Umax = 100 * nu / H
        F = 2 * nu * Umax / L**2
        d = O.Domain(O.D2Q9, 3, H, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force=(F, 0))
        y = np.arange(H) + 0.5
        ua = Umax * (1 - ((y - L) / L) ** 2)
        u0 = np.zeros((2, 3 * H))
        u0[0] = np.repeat(ua, 3)
        d.init_equilibrium(u=u0)
        d.run(int(12 * H * H / (np.pi**2 * nu)))
        _, u, _ = d.moments(1)
        uc = d.grid(u[0])[0, :, 1]
        errs.append(np.sqrt(((uc - ua) ** 2).sum() / (ua**2).sum()))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(Hs))
    assert np.all(np.abs(slopes + 2.0) < 0.05), slopes


def _four_rolls(N, u0=0.01, nu_phys=0.0011):
    dx = 2 * np.pi / N
    nu = nu_phys / dx
    x = np.arange(N) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    Fx = 2 * nu * u0 * dx * dx * np.sin(X) * np.sin(Y)
    Fy = 2 * nu * u0 * dx * dx * np.cos(X) * np.cos(Y)
    ua = np.stack([(u0 * np.sin(X) * np.sin(Y)).ravel(), (u0 * np.cos(X) * np.cos(Y)).ravel()])
    d = O.Domain(O.D2Q9, N, N, nu=nu, force_field=np.stack([Fx.ravel(), Fy.ravel()]))
    d.init_equilibrium(u=ua)
    d.run(int(6 / (2 * nu * dx * dx)))
    _, u, _ = d.moments(1)
    return np.sqrt(((u[0] - ua[0]) ** 2).sum() / (ua[0] ** 2).sum())


def test_four_rolls_convective_convergence():
    """Four-rolls mill (Sec. 6), u0 = 0.01, nu = 0.0011, convective scaling
    tau_j = 1/2 + (tau_i - 1/2) N_j / N_i: error slope about -2 (the paper reports -2.0)."""
    e24, e48 = _four_rolls(24), _four_rolls(48)
    slope = np.log(e48 / e24) / np.log(2.0)
    assert -2.2 < slope < -1.8, slope
    assert e48 < 3e-3


def test_hartmann_prescribed_force():
    """Hartmann flow (Sec. 6) with the Lorentz force imposed from the analytic induced field:
    F_x(y) = F_b + B0 dB_x/dy = F_b Ha cosh(Ha y/L) / sinh(Ha) (from the printed B_x(y)),
    steady u = F_b L^2 coth(Ha)/(Ha nu) (1 - cosh(Ha y/L)/cosh(Ha))."""
    ny, nu, Fb = 100, 0.1, 1e-6   # the paper's 3 x 100 channel
    L = ny / 2
    y = np.arange(ny) + 0.5 - L
    for Ha in (3.0, 10.0):
        Fx = Fb + Fb * (Ha * np.cosh(Ha * y / L) / np.sinh(Ha) - 1.0)
        ff = np.zeros((2, 3 * ny))
        ff[0] = np.repeat(Fx, 3)
        d = O.Domain(O.D2Q9, 3, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force_field=ff)
        ua = Fb * L * L / np.tanh(Ha) / (Ha * nu) * (1 - np.cosh(Ha * y / L) / np.cosh(Ha))
        u0 = np.zeros((2, 3 * ny))
        u0[0] = np.repeat(ua, 3)
        d.init_equilibrium(u=u0)
        d.run(int(4 * L * L / nu))   # slowest viscous mode decays as exp(-nu pi^2 t / (4 L^2))
        _, u, _ = d.moments(1)
        uc = d.grid(u[0])[0, :, 0]
        err = np.sqrt(((uc - ua) ** 2).sum() / (ua**2).sum())
        assert err < 5e-3, (Ha, err)


def test_womersley_oscillating_force():
    """Womersley flow (Sec. 6, eq. wo): F = Fm cos(w t), T = 10000 on 3 x 100, Wo = 4,
    trapezoidal half-step force.  Compared over the fourth period with the analytic
    Re{ i Fm/w [1 - cos(gamma y/L)/cos(gamma)] e^{-i w t} }, gamma = sqrt(i Wo^2).
    With gamma = sqrt(i) Wo the printed form needs e^{-i w t} to solve
    du/dt = nu u'' + Fm cos(w t) (with e^{+i w t} it is the time-reversed solution);
    the core then moves as (Fm/w) sin(w t), as the force dictates."""
    ny, T, Fm, Wo = 100, 10000, 1e-5, 4.0
    w = 2 * np.pi / T
    L = ny / 2
    nu = w * L * L / Wo**2
    d = O.Domain(O.D2Q9, 3, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force=(Fm, 0),
                 force_time=(O.TIME_COS, w))
    d.init_equilibrium()
    y = np.arange(ny) + 0.5 - L
    gam = np.sqrt(1j * Wo**2)
    prof = 1j * Fm / w * (1 - np.cos(gam * y / L) / np.cos(gam))
    d.run(3 * T)
    worst = 0.0
    for k in range(4):
        _, u, _ = d.moments(1)
        t = d.step_count
        ua = np.real(prof * np.exp(-1j * w * t))
        uc = d.grid(u[0])[0, :, 0]
        worst = max(worst, np.abs(uc - ua).max() / np.abs(prof).max())
        d.run(T // 4)
    assert worst < 1e-2, worst


def test_budget_periodic_time_dependent():
    """Periodic lattice: mass is conserved and the total momentum changes by exactly
    sum_x F_tot(x) each step (eq. 27), including a cos(w t) force."""
    g = rng(7)
    nx, ny = 11, 7
    ff = 1e-4 * g.standard_normal((2, nx * ny))
    w = 0.37
    d = O.Domain(O.D2Q9, nx, ny, nu=0.05, force_field=ff, force_time=(O.TIME_COS, w))
    rho = 1 + 0.01 * g.standard_normal(nx * ny)
    u = 0.02 * g.standard_normal((2, nx * ny))
    d.init_equilibrium(rho, u)
    for n in range(5):
        m0 = d.totals()
        cp, cq = O.time_factors(O.TIME_COS, w, n)
        d.run(1)
        m1 = d.totals()
        assert abs(m1[0] - m0[0]) < 1e-13
        # round-off of summing 9 N values of size ~0.1: a few 1e-16 per sum
        assert np.allclose(m1[1:3] - m0[1:3], 0.5 * (cp + cq) * ff.sum(axis=1), rtol=0, atol=1e-14)


def test_budget_bounce_back():
    """Halfway bounce-back: M(n+1) - M(n) = N F_tot - 2 sum f^p_a(x) e_a over links that
    point from a fluid node into a wall."""
    g = rng(8)
    nx, ny = 6, 9
    F = np.array([3e-5, -2e-5])
    d = O.Domain(O.D2Q9, nx, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=0.1, force=F)
    d.init_equilibrium(1 + 0.01 * g.standard_normal(nx * ny), 0.03 * g.standard_normal((2, nx * ny)))
    e = np.stack([EX, EY], axis=1)
    for _ in range(3):
        fp = d.f.reshape(9, ny, nx)
        exch = np.zeros(2)
        for a in range(9):
            for yy in range(ny):
                if 0 <= yy + e[a, 1] < ny:
                    continue
                exch += 2 * fp[a, yy, :].sum() * e[a]
        m0 = d.totals()
        d.run(1)
        m1 = d.totals()
        assert np.allclose(m1[1:3] - m0[1:3], nx * ny * F - exch, rtol=0, atol=1e-14)
        assert abs(m1[0] - m0[0]) < 1e-13


def test_checkpoint_resume_bit_identical():
    """Running 7 + 5 steps from a saved state equals 12 uninterrupted steps bit for bit."""
    g = rng(9)
    nx, ny = 8, 6
    kw = dict(nu=0.07, force=(1e-4, 2e-5), force_time=(O.TIME_COS, 0.2), bc=(O.PERIODIC, O.BOUNCE_BACK))
    a = O.Domain(O.D2Q9, nx, ny, **kw)
    a.init_equilibrium(1 + 0.01 * g.standard_normal(nx * ny), 0.02 * g.standard_normal((2, nx * ny)))
    b = O.Domain(O.D2Q9, nx, ny, **kw)
    b.f[:] = a.f
    a.run(12)
    b.run(7)
    c = O.Domain(O.D2Q9, nx, ny, **kw)
    c.f[:] = b.f
    c.step_count = b.step_count
    c.run(5)
    assert np.array_equal(a.f, c.f)


def test_generic_route_equals_eq23_on_domain():
    """The lattice-independent pseudo-central construction (used for D3Q27) run on D2Q9
    reproduces the printed update over many steps of a forced, walled domain."""
    g = rng(10)
    nx, ny = 9, 7
    ff = 1e-4 * g.standard_normal((2, nx * ny))
    kw = dict(nu=0.04, omega_bulk=1.3, omega_third=0.9, omega_fourth=1.1, force_field=ff,
              bc=(O.PERIODIC, O.BOUNCE_BACK))
    a = O.Domain(O.D2Q9, nx, ny, **kw)
    b = O.Domain(O.D2Q9, nx, ny, d2q9_generic=True, **kw)
    rho, u = 1 + 0.01 * g.standard_normal(nx * ny), 0.03 * g.standard_normal((2, nx * ny))
    a.init_equilibrium(rho, u)
    b.init_equilibrium(rho, u)
    a.run(200)
    b.run(200)
    assert np.abs(a.f - b.f).max() < 1e-14


def test_lorentz_force_implicit_midpoint_recurrence():
    """Velocity-dependent force F_x = F_b - s u_x (s = sigma B0^2) on a uniform periodic lattice:
    with the half steps taken implicitly (the paper: such a force turns eq. 13 into an implicit
    equation for u) the momentum follows the implicit-midpoint recurrence
    j_{n+1} = j_n (1 - s/2)/(1 + s/2) + F_b/(1 + s/2), i.e. j_n = (F_b/s)(1 - r^n)."""
    Fb, s = 2e-5, 0.03
    d = O.Domain(O.D2Q9, 4, 3, nu=0.07, force=(Fb, 0), lorentz=s)
    d.init_equilibrium()
    r = (1 - s / 2) / (1 + s / 2)
    for n in (1, 5, 40, 300):
        d.run(n - d.step_count)
        jx = d.totals()[1] / 12
        assert abs(jx - Fb / s * (1 - r**n)) < 1e-15, n
    # the half-forced velocity returned for kind 1 is the implicit one
    _, u, _ = d.moments(1)
    assert np.allclose(u[0], (jx + Fb / 2) / (1 + s / 2), rtol=0, atol=1e-15)


def test_hartmann_lorentz_force():
    """Hartmann flow driven by F_b and retarded by the velocity-dependent Lorentz force
    -sigma B0^2 u_x, sigma B0^2 = Ha^2 rho nu / L^2: steady
    u = F_b/(sigma B0^2) (1 - cosh(Ha y/L)/cosh Ha) on the paper's 3 x 100 channel."""
    ny, nu = 100, 0.1
    L = ny / 2
    y = np.arange(ny) + 0.5 - L
    for Ha in (3.0, 10.0):
        s = Ha**2 * nu / L**2
        Fb = 0.01 * s / (1 - 1 / np.cosh(Ha))      # centre-line velocity 0.01
        ua = Fb / s * (1 - np.cosh(Ha * y / L) / np.cosh(Ha))
        d = O.Domain(O.D2Q9, 3, ny, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=nu, force=(Fb, 0), lorentz=s)
        u0 = np.zeros((2, 3 * ny))
        u0[0] = np.repeat(ua, 3)
        d.init_equilibrium(u=u0)
        d.run(int(4 * L * L / nu))
        _, u, _ = d.moments(1)
        uc = d.grid(u[0])[0, :, 0]
        err = np.sqrt(((uc - ua) ** 2).sum() / (ua**2).sum())
        assert err < 5e-3, (Ha, err)
