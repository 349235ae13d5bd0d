"""Pins of the oracle's strain-rate magnitude S:S, the viscous-heating source per
unit coefficient (Sec. 6, thermal Couette flow: S_r = 2 nu / C_v S:S).

The paper prints only the off-diagonal relation S_xy = -3 w_5 / (2 rho0) Pi_xy;
the oracle takes the same first-order relation for each second-order moment
with its own relaxation rate: S_xx - S_yy from Pi_xx - Pi_yy with w_shear,
S_xx + S_yy from the trace with w_bulk.  Thermal Couette flow has
S_xx = S_yy = 0, so these pins use flows whose diagonal strain is not zero and
compare with the strain rate of the velocity field itself, never with the
formula:

* four-rolls mill (Sec. 6): u = u0 (sin x sin y, cos x cos y) has S_xy = 0 and
  S_xx = -S_yy = u0 k cos x sin y, so S:S = 2 u0^2 k^2 cos^2 x sin^2 y
  (deviator only; second-order convergence from N = 24 to 48);
* a standing plane sound wave along x: div u != 0, S_xx = d u_x / dx,
  S_yy = S_xy = 0 (trace and deviator both carry it);
* the same wave along the diagonal: S_xx = S_yy = S_xy, all three parts.

The wave cases compare with the spectral derivative of the oracle's own
half-forced velocity, run with w_bulk = 0.8 != w_shear = 1.79 so that a swapped
rate shows.  `test_planted_mistakes_fail_the_pins` evaluates plausible wrong
formulas on the same streamed populations and checks that each misses a pin.
"""
import numpy as np
import pytest

import oracle as O


def _four_rolls(N, u0=0.01, nu_phys=0.0011, omega_bulk=1.4):
    dx = 2 * np.pi / N
    nu = nu_phys / dx
    x = np.arange(N) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    Fx = 2 * nu * u0 * dx * dx * np.sin(X) * np.sin(Y)
    Fy = 2 * nu * u0 * dx * dx * np.cos(X) * np.cos(Y)
    ua = np.stack([(u0 * np.sin(X) * np.sin(Y)).ravel(), (u0 * np.cos(X) * np.cos(Y)).ravel()])
    d = O.Domain(O.D2Q9, N, N, nu=nu, omega_bulk=omega_bulk, force_field=np.stack([Fx.ravel(), Fy.ravel()]))
    d.init_equilibrium(u=ua)
    d.run(int(6 / (2 * nu * dx * dx)))
    exact = (2 * u0 * u0 * dx * dx * np.cos(X) ** 2 * np.sin(Y) ** 2).ravel()
    return d, exact


def _spectral_derivative(a, axis):
    n = a.shape[axis]
    k = 2 * np.pi * np.fft.fftfreq(n)
    shape = [1, 1]
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(a, axis=axis), axis=axis))


def _sound_wave(N, diag, omega_bulk=0.8, nu=0.02, eps=1e-3):
    """Standing wave from rho = 1 + eps cos(k.x) at rest, a quarter period on
    (velocity near its largest).  Returns the domain and S:S of its velocity."""
    ny = N if diag else 1
    X, Y = np.meshgrid(np.arange(N), np.arange(ny), indexing="xy")
    k = 2 * np.pi / N
    phase = k * (X + Y) if diag else k * X
    d = O.Domain(O.D2Q9, N, ny, nu=nu, omega_bulk=omega_bulk)
    d.init_equilibrium(rho=(1 + eps * np.cos(phase)).ravel())
    kmag = k * (np.sqrt(2) if diag else 1.0)
    d.run(int(round(0.25 * 2 * np.pi / (kmag / np.sqrt(3)))))
    _, u, _ = d.moments(1)
    ux, uy = u[0].reshape(ny, N), u[1].reshape(ny, N)
    sxx = _spectral_derivative(ux, 1)
    syy = _spectral_derivative(uy, 0) if diag else np.zeros_like(ux)
    sxy = 0.5 * (_spectral_derivative(ux, 0) + _spectral_derivative(uy, 1)) if diag else 0.5 * _spectral_derivative(uy, 1)
    return d, (sxx**2 + syy**2 + 2 * sxy**2).ravel()


def _rel_err(ss, exact):
    return float(np.abs(ss - exact).max() / exact.max())


def test_four_rolls_strain_rate_second_order():
    """Deviatoric part (w_shear): S:S against 2 u0^2 k^2 cos^2 x sin^2 y."""
    errs = []
    for N in (24, 48):
        d, exact = _four_rolls(N)
        errs.append(_rel_err(d.strain_rate_squared(), exact))
    assert errs[0] < 0.015 and errs[1] < 0.004, errs
    assert 3.5 < errs[0] / errs[1] < 4.7, errs   # second order


@pytest.mark.parametrize("N,diag,tol", [(128, False, 2e-3), (64, True, 0.015)])
def test_sound_wave_strain_rate(N, diag, tol):
    """Trace part (w_bulk) and, along the diagonal, S_xy too: S:S against the
    spectral strain rate of the oracle's own velocity field."""
    d, exact = _sound_wave(N, diag)
    assert _rel_err(d.strain_rate_squared(), exact) < tol


def test_sound_wave_strain_rate_converges():
    e = [_rel_err(d.strain_rate_squared(), ex) for d, ex in (_sound_wave(N, True) for N in (32, 64))]
    assert e[1] < e[0] / 3, e


def _streamed(d):
    """Streamed populations of a periodic D2Q9 domain: f_a(x) = f^p_a(x - e_a)."""
    nx, ny, _ = d.shape
    e = O.velocities(O.D2Q9)
    f = d.f.reshape(9, ny, nx)
    return np.stack([np.roll(f[a], (e[a, 1], e[a, 0]), axis=(0, 1)) for a in range(9)]).reshape(9, -1)


def _variant(d, kind):
    """Wrong strain-rate formulas a slip could produce, on the same streamed populations."""
    f = _streamed(d)
    e = O.velocities(O.D2Q9)
    rho = f.sum(0)
    ux, uy = (f * e[:, 0:1]).sum(0) / rho, (f * e[:, 1:2]).sum(0) / rho
    pxx = (f * e[:, 0:1] ** 2).sum(0) - rho * ux * ux - rho / 3
    pyy = (f * e[:, 1:2] ** 2).sum(0) - rho * uy * uy - rho / 3
    pxy = (f * (e[:, 0] * e[:, 1])[:, None]).sum(0) - rho * ux * uy
    ws, wb = d.params.omega_shear, d.params.omega_bulk
    if kind == "rates_swapped":
        ws, wb = wb, ws
    dif, tr, sxy = -1.5 * ws * (pxx - pyy), -1.5 * wb * (pxx + pyy), -1.5 * ws * pxy
    if kind == "trace_with_shear_rate":
        tr = -1.5 * ws * (pxx + pyy)
    sxx, syy = 0.5 * (tr + dif), 0.5 * (tr - dif)
    if kind == "no_half":
        sxx, syy = tr + dif, tr - dif
    w_xy = 1.0 if kind == "single_xy" else 2.0
    return sxx**2 + syy**2 + w_xy * sxy**2


@pytest.mark.parametrize("kind", ["rates_swapped", "trace_with_shear_rate", "no_half", "single_xy"])
def test_planted_mistakes_fail_the_pins(kind):
    """Each plausible mistake in the diagonal terms misses at least one pin by a
    wide margin (the oracle's own formula passes them all above)."""
    worst = 0.0
    d, ex = _four_rolls(48)
    worst = max(worst, _rel_err(_variant(d, kind), ex) / 0.004)
    for N, diag, tol in [(128, False, 2e-3), (64, True, 0.015)]:
        d, ex = _sound_wave(N, diag)
        worst = max(worst, _rel_err(_variant(d, kind), ex) / tol)
    assert worst > 10.0, (kind, worst)
