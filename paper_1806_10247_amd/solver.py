"""Thin object wrapper around one casclb context (argument marshalling only)."""
import numpy as np

from . import capi as C

_LATTICES = {"D2Q9": C.LB_D2Q9, "D2Q9_D2Q5": C.LB_D2Q9_D2Q5, "D3Q27": C.LB_D3Q27, "D3Q15": C.LB_D3Q15}
_STORAGE = {"f64": C.LB_STORE_F64, "f32": C.LB_STORE_F32_DEV, "f16": C.LB_STORE_F16_DEV}


class Solver:
    """One lattice on one GPU.

    lattice: "D2Q9" | "D2Q9_D2Q5" | "D3Q27" | "D3Q15"; storage: "f64" | "f32" | "f16";
    walls: per-axis halfway bounce-back flags; other keywords are lb_config
    fields (nu, omega_bulk, omega_third, omega_fourth, D_phi, omega_phi_high,
    rho0, residual_interval, device, stream, plane_pad, block_x).
    """

    def __init__(self, lattice, shape, storage="f64", walls=(False, False, False), **cfg):
        nx, ny, nz = (tuple(shape) + (1, 1))[:3]
        self.lattice = lattice
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.dims = 3 if lattice in ("D3Q27", "D3Q15") else 2
        self.q = {"D3Q27": 27, "D3Q15": 15}.get(lattice, 9)
        self.qs = 5 if lattice == "D2Q9_D2Q5" else 0
        bc = [C.LB_HALFWAY_BB if w else C.LB_PERIODIC for w in (tuple(walls) + (False,) * 3)[:3]]
        self.cfg = C.lb_config_default(lattice=_LATTICES[lattice], storage=_STORAGE[storage], nx=nx, ny=ny, nz=nz,
                                       bc=bc, **cfg)
        self.ctx = C.lb_create(self.cfg)

    # context management
    def close(self):
        if self.ctx:
            C.lb_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state
    def init_equilibrium(self, rho=None, u=None, phi=None):
        f = lambda a, n: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(n)
        C.lb_init_equilibrium(self.ctx, f(rho, self.N), f(u, self.dims * self.N), f(phi, self.N))

    def set_force(self, fx=0.0, fy=0.0, fz=0.0):
        C.lb_set_force_uniform(self.ctx, fx, fy, fz)

    def set_force_field(self, F, dtype=np.float64):
        if F is None:
            C.lb_set_force_field(self.ctx, None)
            return
        F = np.ascontiguousarray(F, dtype=dtype).reshape(self.dims, self.N)
        C.lb_set_force_field(self.ctx, F, C.LB_DTYPE_F64 if dtype == np.float64 else C.LB_DTYPE_F32)

    def set_force_time(self, mode, omega=0.0):
        C.lb_set_force_time(self.ctx, mode, omega)

    def set_source(self, s):
        C.lb_set_source_uniform(self.ctx, s)

    def set_source_field(self, S, dtype=np.float64):
        if S is None:
            C.lb_set_source_field(self.ctx, None)
            return
        S = np.ascontiguousarray(S, dtype=dtype).reshape(self.N)
        C.lb_set_source_field(self.ctx, S, C.LB_DTYPE_F64 if dtype == np.float64 else C.LB_DTYPE_F32)

    def set_source_time(self, mode, omega=0.0):
        C.lb_set_source_time(self.ctx, mode, omega)

    def step(self, n=1):
        C.lb_step(self.ctx, n)

    def synchronize(self):
        C.lb_synchronize(self.ctx)

    @property
    def step_count(self):
        return C.lb_get_step(self.ctx)

    @step_count.setter
    def step_count(self, n):
        C.lb_set_step(self.ctx, n)

    def moments(self, kind=C.LB_MOMENTS_HALF_FORCED):
        rho = np.empty(self.N)
        u = np.empty((self.dims, self.N))
        phi = np.empty(self.N) if self.qs else None
        C.lb_read_moments(self.ctx, kind, rho, u, phi)
        return rho, u, phi

    def populations(self):
        f = np.empty((self.q, self.N))
        g = np.empty((5, self.N)) if self.qs else None
        C.lb_read_populations(self.ctx, f, g)
        return f, g

    def write_populations(self, f, g=None):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q, self.N)
        if g is not None:
            g = np.ascontiguousarray(g, dtype=np.float64).reshape(5, self.N)
        C.lb_write_populations(self.ctx, f, g)

    def populations_box(self, lo, ext):
        bn = int(np.prod(ext))
        f = np.empty((self.q, bn))
        g = np.empty((5, bn)) if self.qs else None
        C.lb_read_populations_box(self.ctx, lo, ext, f, g)
        return f, g

    def totals(self):
        return C.lb_totals(self.ctx)

    def residual(self):
        return C.lb_residual(self.ctx)

    def set_wall_velocity(self, axis, side, ux, uy=0.0):
        C.lb_set_wall_velocity(self.ctx, axis, side, ux, uy)

    def set_scalar_wall(self, axis, side, value=None):
        """value None: no-flux wall; a number: scalar held at that value."""
        C.lb_set_scalar_wall(self.ctx, axis, side, value is not None, 0.0 if value is None else value)

    def set_lorentz(self, s):
        C.lb_set_lorentz(self.ctx, s)

    def set_viscous_heating(self, coefficient):
        C.lb_set_viscous_heating(self.ctx, coefficient)

    def residual_scalar(self):
        return C.lb_residual_scalar(self.ctx)

    def info(self):
        return C.lb_get_info(self.ctx)
