"""Pins of the D3Q15 oracle (Appendix A): basis, printed post-collision rows,
central-moment relaxation of every moment the cascaded collision sets, the
mass/momentum budget, the rest state, and the plane Poiseuille parabola."""
from math import comb

import numpy as np
import pytest

import oracle as O

E = None


def _E():
    global E
    if E is None:
        E = O.velocities(O.D3Q15).astype(np.float64)
    return E


def test_velocity_set_and_basis():
    """Eq. (A1) velocities with their opposites; eq. (2A) basis orthogonal with the
    squared norms 15, 10 x3, 8 x3, 4, 12, 18, 160 x3, 8, 1440; <K|e_x> = 10 delta_1 (eq. 12A)."""
    e = _E()
    assert e.shape == (15, 3)
    for a in range(15):
        assert sum(np.array_equal(e[b], -e[a]) for b in range(15)) == 1
    K = O.d3q15_basis()
    G = K @ K.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert list(np.diag(G)) == [15, 10, 10, 10, 8, 8, 8, 4, 12, 18, 160, 160, 160, 8, 1440]
    for ax in range(3):
        want = np.zeros(15)
        want[1 + ax] = 10
        assert np.array_equal(K @ e[:, ax], want)


# Coefficients of g_0..g_14 in the post-collision rows as printed after eq. (13A),
# row by row (alpha = 0..14).
PRINTED_ROWS = [
    [1, 0, 0, 0, 0, 0, 0, 0, 0, -2, 0, 0, 0, 0, 32],
    [1, 1, 0, 0, 0, 0, 0, 1, 1, -1, -8, 0, 0, 0, -8],
    [1, -1, 0, 0, 0, 0, 0, 1, 1, -1, 8, 0, 0, 0, -8],
    [1, 0, 1, 0, 0, 0, 0, -1, 1, -1, 0, -8, 0, 0, -8],
    [1, 0, -1, 0, 0, 0, 0, -1, 1, -1, 0, 8, 0, 0, -8],
    [1, 0, 0, 1, 0, 0, 0, 0, -2, -1, 0, 0, -8, 0, -8],
    [1, 0, 0, -1, 0, 0, 0, 0, -2, -1, 0, 0, 8, 0, -8],
    [1, 1, 1, 1, 1, 1, 1, 0, 0, 1, 2, 2, 2, 1, 2],
    [1, -1, 1, 1, -1, -1, 1, 0, 0, 1, -2, 2, 2, -1, 2],
    [1, 1, -1, 1, -1, 1, -1, 0, 0, 1, 2, -2, 2, -1, 2],
    [1, -1, -1, 1, 1, -1, -1, 0, 0, 1, -2, -2, 2, 1, 2],
    [1, 1, 1, -1, 1, -1, -1, 0, 0, 1, 2, 2, -2, -1, 2],
    [1, -1, 1, -1, -1, 1, -1, 0, 0, 1, -2, 2, -2, -1, 2],
    [1, 1, -1, -1, -1, -1, 1, 0, 0, 1, 2, -2, -2, 1, 2],
    [1, -1, -1, -1, 1, 1, 1, 0, 0, 1, -2, -2, -2, -1, 2],
]


def test_printed_rows_are_K_transposed_except_one_sign():
    """The printed rows equal K^T of eq. (2A) except the g_13 coefficient of row
    12, printed -1: e_x e_y e_z = (-1)(1)(-1) = +1 for alpha = 12 (the oracle uses K)."""
    K = O.d3q15_basis()
    P = np.array(PRINTED_ROWS, dtype=np.float64)
    diff = np.argwhere(P != K.T)
    assert diff.tolist() == [[12, 13]]
    assert P[12, 13] == -1 and K[13, 12] == 1


def _eq(rho, u):
    f = np.zeros(15)
    O.lib().orc_flow_equilibrium(O.D3Q15, rho, O._p(np.array(u, dtype=np.float64)), O._p(f))
    return f


def _central(f, u, m, n, p, rho_u=True):
    """Central moment about u, first raw moments taken as rho u (pseudo-central)."""
    e = _E()
    R = f.sum()
    s = 0.0
    for a in range(m + 1):
        for b in range(n + 1):
            for c in range(p + 1):
                if a + b + c == 1 and rho_u:
                    r = R * u[[a, b, c].index(1)]
                else:
                    r = float((f * e[:, 0] ** a * e[:, 1] ** b * e[:, 2] ** c).sum())
                s += comb(m, a) * comb(n, b) * comb(p, c) * (-u[0]) ** (m - a) * (-u[1]) ** (n - b) * \
                    (-u[2]) ** (p - c) * r
    return s


RELAXED = {   # moment: (combination of (m, n, p), rate index, equilibrium / rho)
    "xy": ([(1, (1, 1, 0))], 0, 0.0), "xz": ([(1, (1, 0, 1))], 0, 0.0), "yz": ([(1, (0, 1, 1))], 0, 0.0),
    "xx-yy": ([(1, (2, 0, 0)), (-1, (0, 2, 0))], 0, 0.0),
    "xx+yy-2zz": ([(1, (2, 0, 0)), (1, (0, 2, 0)), (-2, (0, 0, 2))], 0, 0.0),
    "trace": ([(1, (2, 0, 0)), (1, (0, 2, 0)), (1, (0, 0, 2))], 1, 1.0),
    "xyy": ([(1, (1, 2, 0))], 2, 0.0), "xxy": ([(1, (2, 1, 0))], 2, 0.0), "xxz": ([(1, (2, 0, 1))], 2, 0.0),
    "xyz": ([(1, (1, 1, 1))], 2, 0.0), "xxyy": ([(1, (2, 2, 0))], 3, 1.0 / 9.0),
}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_collision_relaxes_each_central_moment(seed):
    """Without force, every moment the collision sets ends at (1 - w) k + w k_eq
    about the node's velocity: second order to 0 (trace to rho), the four third
    order ones to 0, k_xxyy to rho/9 (the reading of the undefined term of g_14)."""
    g = np.random.default_rng(seed)
    u0 = g.uniform(-0.05, 0.05, 3)
    f = _eq(1.0 + g.uniform(-0.02, 0.02), u0) + 2e-3 * g.standard_normal(15)
    w = g.uniform(0.6, 1.8, 4)
    fp, u = O.d3q15_collide(f, np.zeros(3), np.zeros(3), w)
    rho = f.sum()
    for name, (terms, wi, eq) in RELAXED.items():
        pre = sum(c * _central(f, u, *mnp) for c, mnp in terms)
        post = sum(c * _central(fp, u, *mnp) for c, mnp in terms)
        want = (1 - w[wi]) * pre + w[wi] * eq * rho
        assert abs(post - want) <= 1e-14 * max(1.0, abs(want)), (name, post, want)


def test_budget_and_rest_state():
    """Budgets of the half force steps, and the rest state as a fixed point.  The
    latter pins the fourth-order equilibrium of g_14 (a term eq. 6A leaves
    undefined): the isotropy-fixed weights give the rest state k_xxyy = 8/72 =
    1/9, so with a fourth-order rate of 0.7 the rest state stays put only if
    g_14 relaxes k_xxyy towards rho/9."""
    g = np.random.default_rng(5)
    f = _eq(1.01, [0.02, -0.01, 0.03]) + 1e-3 * g.standard_normal(15)
    F = np.array([1e-4, -3e-4, 2e-4])
    fp, u = O.d3q15_collide(f, F, F, [1.1, 1.0, 0.9, 1.2])
    assert abs(fp.sum() - f.sum()) < 1e-15
    ulp = 16 * np.finfo(float).eps * np.abs(f).sum()   # rounding of 15-term sums
    assert np.abs((fp - f) @ _E() - F).max() < ulp
    assert np.allclose(u * f.sum(), f @ _E() + F / 2, rtol=0, atol=ulp)
    w0 = _eq(1.0, [0, 0, 0])
    assert np.allclose(w0, [2 / 9] + [1 / 9] * 6 + [1 / 72] * 8, rtol=0, atol=1e-17)
    e = _E()
    assert abs(w0 @ (e[:, 0] ** 2 * e[:, 1] ** 2) - 1 / 9) < 1e-16
    fr, _ = O.d3q15_collide(w0, np.zeros(3), np.zeros(3), [1.3, 0.8, 1.1, 0.7])
    assert np.abs(fr - w0).max() < 1e-15   # rounding of O(1) moment differences


def test_plane_poiseuille_is_an_exact_parabola():
    """Periodic x and z, halfway walls on y: the steady profile has the constant
    second difference -F/(rho nu) of the exact solution (plus a constant slip)."""
    nu, F, ny = 1.0 / 6.0, 1e-6, 24
    d = O.Domain(O.D3Q15, 2, ny, 2, bc=(O.PERIODIC, O.BOUNCE_BACK, O.PERIODIC), nu=nu, force=(F, 0.0, 0.0))
    d.init_equilibrium()
    d.run(12000)
    _, u, _ = d.moments(1)
    ux = u[0].reshape(2, ny, 2)[0, :, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    assert np.abs(d2 + F / nu).max() < 1e-6 * F / nu
    y = np.arange(ny) + 0.5
    ua = F / (2 * nu) * y * (ny - y)
    slip = ux - ua
    assert np.ptp(slip) < 1e-6 * ua.max()          # a constant offset ...
    assert np.abs(slip).max() < 1e-2 * ua.max()    # ... and a small one
