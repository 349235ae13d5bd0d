"""Helpers shared by the GPU parity tests: build the same case on the HIP
library (through the C ABI) and on the oracle, from the same seeded inputs."""
import numpy as np

import oracle as O
from casclb_inputs import coords, noise, smooth_fields

LAT_O = {"D2Q9": O.D2Q9, "D2Q9_D2Q5": O.D2Q9_D2Q5, "D3Q27": O.D3Q27, "D3Q15": O.D3Q15}


def reduced_precision_bound(steps, storage, scale, k_store=4.0, k_arith=8.0):
    """Bound on max |f_gpu - f_oracle| after `steps` steps with float32 or float16
    deviation storage and float32 arithmetic, for deviations of size `scale`:
    (k_store eps + k_arith eps32) scale (1 + sqrt(steps)), eps the unit round-off
    of the storage, eps32 that of float32.  The rounding errors of successive
    steps are independent and the collision damps the non-hydrodynamic part, so
    they add up like a random walk, not linearly.  Largest measured values of
    err / (eps scale): float32 12.9 (D3Q15 duct from deviations ~1e-2, 3 steps),
    66.8 (batch channel, 300 steps), 22 (parity cases, 1000 steps); float16 with
    stochastic rounding 3.7 (100 steps) and 3.0 (1000 steps); the bound gives
    32.8, 220 and 391 (float32) and 44 and 130 (float16).  A float16 lattice that
    drops the force kicks (100 steps at F ~ 1e-5) is off by ~100 eps scale."""
    eps = {"f16": 2.0**-11, "f32": 2.0**-24}[storage]
    return (k_store * eps + k_arith * 2.0**-24) * scale * (1.0 + np.sqrt(steps))


def gpu_available():
    try:
        from paper_1806_10247_amd import capi as C
        C.lib()
    except Exception:
        return False
    try:
        cfg = C.lb_config_default(lattice=C.LB_D2Q9, nx=1, ny=1, nz=1, residual_interval=0)
        ctx = C.lb_create(cfg)
        C.lb_destroy(ctx)
        return True
    except Exception:
        return False


class Case:
    """A parity case: lattice, shape, walls, rates and forcing."""

    def __init__(self, lattice, shape, walls=(False, False, False), nu=0.05, omega_bulk=1.0, omega_third=1.0,
                 omega_fourth=1.0, D=0.03, omega_phi_high=1.0, force=(0.0, 0.0, 0.0), force_field=None,
                 force_time=(0, 0.0), source=0.0, source_field=None, source_time=(0, 0.0), seed=0):
        self.lattice = lattice
        self.shape = tuple(shape)
        self.walls = tuple(walls)
        self.nu, self.D = nu, D
        self.omega_bulk, self.omega_third, self.omega_fourth = omega_bulk, omega_third, omega_fourth
        self.omega_phi_high = omega_phi_high
        self.force, self.force_field, self.force_time = force, force_field, force_time
        self.source, self.source_field, self.source_time = source, source_field, source_time
        self.seed = seed
        self.dims = 3 if lattice in ("D3Q27", "D3Q15") else 2
        self.N = int(np.prod(self.shape))

    def __repr__(self):
        return f"{self.lattice}{self.shape} walls={self.walls}"

    def _field(self, fld):
        return fld(coords(self.shape)) if callable(fld) else fld

    # -- oracle side ---------------------------------------------------------
    def oracle(self):
        bc = tuple(O.BOUNCE_BACK if w else O.PERIODIC for w in self.walls)
        return O.Domain(LAT_O[self.lattice], *self.shape, bc=bc, nu=self.nu, omega_bulk=self.omega_bulk,
                        omega_third=self.omega_third, omega_fourth=self.omega_fourth, D=self.D,
                        omega_phi_high=self.omega_phi_high, force=self.force,
                        force_field=self._field(self.force_field), force_time=self.force_time, source=self.source,
                        source_field=self._field(self.source_field), source_time=self.source_time)

    # -- GPU side ------------------------------------------------------------
    def gpu(self, storage="f64", **extra):
        from paper_1806_10247_amd.solver import Solver
        s = Solver(self.lattice, self.shape, storage=storage, walls=self.walls, nu=self.nu,
                   omega_bulk=self.omega_bulk, omega_third=self.omega_third, omega_fourth=self.omega_fourth,
                   D_phi=self.D if self.lattice == "D2Q9_D2Q5" else 1.0 / 6.0, omega_phi_high=self.omega_phi_high,
                   **extra)
        if self.force_field is not None:
            s.set_force_field(self._field(self.force_field))
        else:
            s.set_force(*self.force)
        s.set_force_time(*self.force_time)
        if self.lattice == "D2Q9_D2Q5":
            if self.source_field is not None:
                s.set_source_field(self._field(self.source_field))
            else:
                s.set_source(self.source)
            s.set_source_time(*self.source_time)
        return s

    # -- common initial state -------------------------------------------------
    def initial_fields(self):
        return smooth_fields(self.shape, self.dims, seed=self.seed)

    def perturbed_state(self, dom, scale=2e-3):
        """Oracle equilibrium of the seeded fields plus seeded non-equilibrium noise."""
        rho, u, phi = self.initial_fields()
        dom.init_equilibrium(rho, u, phi)
        f = dom.f + noise(dom.f.shape, scale, seed=self.seed + 1)
        g = None if dom.g is None else dom.g + noise(dom.g.shape, scale, seed=self.seed + 2)
        return f, g


def oracle_box(case, lo, ext, steps, init_fields=None):
    """Run the oracle on the sub-box [lo, lo+ext) of `case` for `steps` steps.

    Sides of the box that coincide with a wall of the case get halfway
    bounce-back; other sides are open (the box wraps onto itself there), so
    only nodes at least `steps` away from an open side are valid.  The force
    and source fields and the initial fields are sliced from full-lattice
    callables evaluated at the box coordinates.
    Returns (domain, valid_mask[N_box])."""
    shape = case.shape
    bc = []
    valid = np.ones(tuple(ext[::-1]), dtype=bool)  # [z][y][x]
    for ax in range(3):
        n, a, e = shape[ax], lo[ax], ext[ax]
        if case.walls[ax]:
            assert 0 <= a and a + e <= n, "a box may not cross a wall"
        lo_bb = case.walls[ax] and a == 0
        hi_bb = case.walls[ax] and a + e == n
        if e == n and not case.walls[ax]:
            bc.append((O.PERIODIC, O.PERIODIC))
            continue
        bc.append((O.BOUNCE_BACK if lo_bb else O.PERIODIC, O.BOUNCE_BACK if hi_bb else O.PERIODIC))
        idx = np.arange(e)
        ok = np.ones(e, dtype=bool)
        if not lo_bb:
            ok &= idx >= steps
        if not hi_bb:
            ok &= idx <= e - 1 - steps
        sl = [slice(None)] * 3
        sl[2 - ax] = ~ok
        valid[tuple(sl)] = False
    pts = coords(tuple(ext))
    pts = (pts + np.array(lo)[:, None]) % np.array(shape)[:, None]
    sub = Case(case.lattice, tuple(ext), walls=case.walls, nu=case.nu, omega_bulk=case.omega_bulk,
               omega_third=case.omega_third, omega_fourth=case.omega_fourth, D=case.D,
               omega_phi_high=case.omega_phi_high, force=case.force, force_time=case.force_time,
               source=case.source, source_time=case.source_time)
    if callable(case.force_field):
        sub.force_field = case.force_field(pts)
    if callable(case.source_field):
        sub.source_field = case.source_field(pts)
    dom = sub.oracle()
    for ax in range(3):
        dom.params.bc_lo[ax], dom.params.bc_hi[ax] = bc[ax]
    if init_fields is None:
        dom.init_equilibrium()
    else:
        rho, u, phi = init_fields(pts)
        dom.init_equilibrium(rho, u, phi)
    dom.run(steps)
    return dom, valid.ravel()
