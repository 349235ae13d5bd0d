"""Oracle pins of the wall conditions and the viscous-heating source of the
thermal Couette problem (Sec. 6): moving-wall bounce-back reproduces the
linear Couette profile, the fixed-value scalar walls reproduce linear
conduction, and with the heating source the temperature follows the analytical
profile with errors of the size Table 1 reports (tests/golden)."""
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thermal_couette_table1.txt")
NX, NY = 3, 64
U0 = 0.05
NU, D = (0.70 - 0.5) / 3.0, (0.782 - 0.5) / 3.0
Y = np.arange(NY) + 0.5   # halfway walls at 0 and NY


def table1():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {int(a): float(b) for a, b in rows}


def couette(ec, wall_u=U0, t_low=0.0, t_high=1.0):
    ch = 2.0 * NU * ec * (t_high - t_low) / U0**2 if ec else 0.0   # c_h = 2 nu / C_v, Ec = U0^2 / (C_v dT)
    d = O.Domain(O.D2Q9_D2Q5, NX, NY, bc=(O.PERIODIC, O.BOUNCE_BACK), nu=NU, D=D,
                 wall_velocity={(1, 1): (wall_u, 0.0, 0.0)}, phi_walls={(1, 0): t_low, (1, 1): t_high},
                 viscous_heating=ch)
    d.init_equilibrium()
    prev = None
    for _ in range(80):
        d.run(5000)
        _, u, phi = d.moments(1)
        T = phi.reshape(NY, NX)[:, 0]
        if prev is not None and np.abs(T - prev).max() < 1e-13:
            break
        prev = T.copy()
    return u[0].reshape(NY, NX)[:, 0], T


def test_moving_wall_gives_the_linear_couette_profile_and_conduction_is_linear():
    ux, T = couette(0)
    assert np.abs(ux - U0 * Y / NY).max() < 1e-10
    assert np.abs(T - Y / NY).max() < 1e-11


def test_fixed_value_walls_hold_any_two_temperatures():
    _, T = couette(0, wall_u=0.0, t_low=0.3, t_high=-0.4)
    assert np.abs(T - (0.3 - 0.7 * Y / NY)).max() < 1e-11


@pytest.mark.parametrize("ec", [10, 40, 100])
def test_thermal_couette_matches_the_analytic_profile_at_the_size_of_table_1(ec):
    """T/dT = y/H + (Pr Ec/2)(y/H)(1 - y/H): the heating must carry the factor
    2 nu/C_v and the strain rate of the non-equilibrium moments (a dropped
    factor gives errors of order 1e-1)."""
    _, T = couette(ec)
    Ta = Y / NY + (NU / D) * ec / 2.0 * (Y / NY) * (1.0 - Y / NY)
    err = np.sqrt(((T - Ta) ** 2).sum() / (Ta**2).sum())
    assert err <= 1.5 * table1()[ec], (ec, err)
