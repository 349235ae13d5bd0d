"""FP64 CPU oracle for the cascaded LB update with Strang-split force/source steps.

TEST INFRASTRUCTURE ONLY: the slow, plain reference the GPU library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU library; the C source
``casclb_oracle.c`` cites the equation each step follows.

Array conventions (same for every function here):
  * a population array is ``[Q][N]`` (float64), N = nx*ny*nz, x fastest;
  * the D2Q9 order is that of eq. (15), the D2Q5 order that of eq. (34),
    D3Q27 uses alpha = d(ex) + 3 d(ey) + 9 d(ez), d(0)=0, d(+1)=1, d(-1)=2;
  * the stored state is the post-collision population f^p; a step pulls it,
    applies half force step, collision, half force step, and stores f^p again.

Parity status: every function is pinned by the ``-m "not gpu"`` tests.  The
fourth-order equilibrium rho/9 that the D3Q15 collision (eq. 6A, g_14) relaxes
k_xxyy towards, a term the paper leaves undefined, is pinned at rest: with the
isotropy-fixed D3Q15 weights the rest state has k_xxyy = 8/72 = 1/9, and it is a
fixed point of the collision at a fourth-order rate != 1 only for that value
(``test_budget_and_rest_state``).  The diagonal strain terms of the
viscous-heating source are pinned by four-rolls-mill and sound-wave strain
rates (``tests/test_oracle_strain.py``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")

D2Q9, D2Q9_D2Q5, D3Q27, D3Q15 = 0, 1, 2, 3
PERIODIC, BOUNCE_BACK = 0, 1
TIME_CONSTANT, TIME_COS = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("d2q9_generic", ctypes.c_int32),
        ("d2q5_printed_sign", ctypes.c_int32),
        ("nthreads", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("omega_bulk", ctypes.c_double),
        ("omega_shear", ctypes.c_double),
        ("omega_third", ctypes.c_double),
        ("omega_fourth", ctypes.c_double),
        ("omega_phi_diff", ctypes.c_double),
        ("omega_phi_high", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("force_field", ctypes.c_void_p),
        ("force_time_mode", ctypes.c_int32),
        ("force_omega", ctypes.c_double),
        ("source", ctypes.c_double),
        ("source_field", ctypes.c_void_p),
        ("source_time_mode", ctypes.c_int32),
        ("source_omega", ctypes.c_double),
        ("lorentz", ctypes.c_double),
        ("wall_u", ctypes.c_double * 18),          # [axis][side][component]
        ("phi_wall", ctypes.c_int32 * 6),          # [axis][side]
        ("phi_wall_value", ctypes.c_double * 6),   # [axis][side]
        ("viscous_heating", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load liborc.so, building it with gcc first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_d2q9_collide.argtypes = [dp, dp, dp, dp, dp, dp]
        L.orc_d2q9_apply_k.argtypes = [dp, dp, dp]
        L.orc_d2q5_collide.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int, dp]
        L.orc_d2q5_apply_l.argtypes = [dp, dp, dp]
        L.orc_generic_collide.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_d3q15_collide.argtypes = [dp, dp, dp, dp, dp, dp]
        L.orc_d3q15_basis.argtypes = [dp]
        L.orc_generic_matrix.argtypes = [ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_int)]
        L.orc_flow_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_scalar_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_time_factors.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp]
        L.orc_run.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.c_int64, ctypes.c_int64]
        L.orc_run.restype = ctypes.c_int
        L.orc_moments.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.c_int64, ctypes.c_int, dp, dp, dp]
        L.orc_strain_rate_field.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_int64, dp]
        L.orc_strain_rate_field.restype = ctypes.c_int
        L.orc_velocity.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_d2q5_velocity.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x, n):
    a = np.zeros(n, dtype=np.float64)
    if x is not None:
        x = np.asarray(x, dtype=np.float64).ravel()
        a[: len(x)] = x
    return a


def max_threads():
    return int(lib().orc_max_threads())


def num_dirs(lattice):
    return {D3Q27: 27, D3Q15: 15}.get(lattice, 9)


def num_dims(lattice):
    return 3 if lattice in (D3Q27, D3Q15) else 2


def velocities(lattice):
    """Velocity set [Q][3] of the flow lattice (ints)."""
    L = lib()
    q = num_dirs(lattice)
    return np.array([[L.orc_velocity(lattice, a, i) for i in range(3)] for a in range(q)], dtype=np.int64)


def scalar_velocities():
    L = lib()
    return np.array([[L.orc_d2q5_velocity(a, i) for i in range(2)] for a in range(5)], dtype=np.int64)


# ---------------------------------------------------------------------------
# per-node routines (vectorised here only by looping over nodes)
# ---------------------------------------------------------------------------

def d2q9_collide(f, fpre, ftot, omega):
    """Eqs. (24), (25), (23), (31), (32) on one node.  Returns (f^p, u)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    fp = np.zeros(9)
    u = np.zeros(2)
    lib().orc_d2q9_collide(_p(f), _p(_vec(fpre, 2)), _p(_vec(ftot, 2)), _p(_vec(omega, 6)), _p(fp), _p(u))
    return fp, u


def d2q9_apply_k(f, g):
    """Eq. (32) rows: f + K g."""
    fp = np.zeros(9)
    lib().orc_d2q9_apply_k(_p(_vec(f, 9)), _p(_vec(g, 9)), _p(fp))
    return fp


def d2q5_collide(g, u, spre, stot, omega, printed_sign=False):
    """Eqs. (42), (43), (41), (47), (48) on one node.  Returns g^p."""
    gp = np.zeros(5)
    lib().orc_d2q5_collide(_p(_vec(g, 5)), _p(_vec(u, 2)), float(spre), float(stot), _p(_vec(omega, 4)),
                           int(bool(printed_sign)), _p(gp))
    return gp


def d2q5_apply_l(g, h):
    """Eq. (48) rows: g + L h."""
    gp = np.zeros(5)
    lib().orc_d2q5_apply_l(_p(_vec(g, 5)), _p(_vec(h, 5)), _p(gp))
    return gp


def generic_collide(lattice, f, fpre, ftot, rates):
    """Lattice-independent pseudo-central collision + kicks on one node.

    rates = (omega_bulk, omega_shear, omega_third, omega_fourth_and_higher).
    Returns (f^p, u)."""
    q, d = num_dirs(lattice), num_dims(lattice)
    fp = np.zeros(q)
    u = np.zeros(3)
    lib().orc_generic_collide(lattice, _p(_vec(f, q)), _p(_vec(fpre, 3)), _p(_vec(ftot, 3)), _p(_vec(rates, 4)),
                              _p(fp), _p(u))
    return fp, u[:d]


def d3q15_collide(f, fpre, ftot, rates):
    """Appendix A update on one D3Q15 node (eqs. 8A, 6A, 13A, f^p = f + K g).
    rates = (shear omega_4..8, bulk omega_9, third omega_10..13, fourth omega_14).
    Returns (f^p, u)."""
    fp = np.zeros(15)
    u = np.zeros(3)
    lib().orc_d3q15_collide(_p(_vec(f, 15)), _p(_vec(fpre, 3)), _p(_vec(ftot, 3)), _p(_vec(rates, 4)), _p(fp), _p(u))
    return fp, u


def d3q15_basis():
    """K[beta][alpha] of eq. (2A)."""
    K = np.zeros((15, 15))
    lib().orc_d3q15_basis(_p(K))
    return K


def generic_matrix(lattice):
    q = num_dirs(lattice)
    m = np.zeros((q, q))
    mi = np.zeros((q, q))
    ex = np.zeros((q, 3), dtype=np.int32)
    lib().orc_generic_matrix(lattice, _p(m), _p(mi), ex.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return m, mi, ex


def flow_equilibrium(lattice, rho, u):
    q = num_dirs(lattice)
    feq = np.zeros(q)
    lib().orc_flow_equilibrium(lattice, float(rho), _p(_vec(u, 3)), _p(feq))
    return feq


def scalar_equilibrium(phi, u):
    geq = np.zeros(5)
    lib().orc_scalar_equilibrium(float(phi), _p(_vec(u, 2)), _p(geq))
    return geq


def time_factors(mode, omega, n):
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().orc_time_factors(int(mode), float(omega), int(n), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


# ---------------------------------------------------------------------------
# domain-level
# ---------------------------------------------------------------------------

class Domain:
    """A lattice with its stored post-collision state, advanced by orc_run.

    bc: per-axis boundary, either PERIODIC or BOUNCE_BACK, or a (lo, hi) pair.
    nu / D give omega_shear = 1/(3 nu + 1/2), omega_phi_diff = 1/(3 D + 1/2)
    (Sec. 6) unless the omegas are given directly.
    """

    def __init__(self, lattice, nx, ny, nz=1, bc=(PERIODIC, PERIODIC, PERIODIC), nu=None, omega_shear=None,
                 omega_bulk=1.0, omega_third=1.0, omega_fourth=1.0, D=None, omega_phi_diff=None,
                 omega_phi_high=1.0, force=(0.0, 0.0, 0.0), force_field=None, force_time=(TIME_CONSTANT, 0.0),
                 source=0.0, source_field=None, source_time=(TIME_CONSTANT, 0.0), d2q9_generic=False,
                 d2q5_printed_sign=False, nthreads=0, lorentz=0.0, wall_velocity=None, phi_walls=None,
                 viscous_heating=0.0):
        """wall_velocity: {(axis, side): (ux, uy, uz)} for moving bounce-back walls (side 0 = low, 1 = high);
        phi_walls: {(axis, side): value} for fixed-value scalar walls (other scalar walls: no flux);
        viscous_heating: c_h of the scalar source c_h (S:S) from the flow's strain rate."""
        if lattice not in (D3Q27, D3Q15):
            assert nz == 1
        self.lattice = lattice
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.q = num_dirs(lattice)
        self.d = num_dims(lattice)
        p = Params()
        p.lattice = lattice
        p.d2q9_generic = int(bool(d2q9_generic))
        p.d2q5_printed_sign = int(bool(d2q5_printed_sign))
        p.nthreads = int(nthreads)
        p.nx, p.ny, p.nz = nx, ny, nz
        for i in range(3):
            b = bc[i] if i < len(bc) else PERIODIC
            lo, hi = (b, b) if not isinstance(b, (tuple, list)) else b
            p.bc_lo[i], p.bc_hi[i] = lo, hi
        if omega_shear is None:
            omega_shear = 1.0 / (3.0 * nu + 0.5)
        if omega_phi_diff is None:
            omega_phi_diff = 1.0 / (3.0 * D + 0.5) if D is not None else 1.0
        p.omega_bulk, p.omega_shear, p.omega_third, p.omega_fourth = omega_bulk, omega_shear, omega_third, omega_fourth
        p.omega_phi_diff, p.omega_phi_high = omega_phi_diff, omega_phi_high
        for i in range(3):
            p.force[i] = force[i] if i < len(force) else 0.0
        self._ff = None
        if force_field is not None:
            self._ff = np.ascontiguousarray(force_field, dtype=np.float64).reshape(self.d, self.N)
            p.force_field = self._ff.ctypes.data
        p.force_time_mode, p.force_omega = force_time
        p.source = source
        self._sf = None
        if source_field is not None:
            self._sf = np.ascontiguousarray(source_field, dtype=np.float64).reshape(self.N)
            p.source_field = self._sf.ctypes.data
        p.source_time_mode, p.source_omega = source_time
        p.lorentz = lorentz
        for (ax, sd), uw in (wall_velocity or {}).items():
            for k in range(3):
                p.wall_u[(ax * 2 + sd) * 3 + k] = uw[k] if k < len(uw) else 0.0
        for (ax, sd), val in (phi_walls or {}).items():
            p.phi_wall[ax * 2 + sd] = 1
            p.phi_wall_value[ax * 2 + sd] = val
        p.viscous_heating = viscous_heating
        self.params = p
        self.f = np.zeros((self.q, self.N))
        self.g = np.zeros((5, self.N)) if lattice == D2Q9_D2Q5 else None
        self.step_count = 0

    # initial state: product-form equilibrium
    def init_equilibrium(self, rho=None, u=None, phi=None):
        rho = np.ones(self.N) if rho is None else np.asarray(rho, dtype=np.float64).reshape(self.N)
        u = np.zeros((self.d, self.N)) if u is None else np.asarray(u, dtype=np.float64).reshape(self.d, self.N)
        for node in range(self.N):
            self.f[:, node] = flow_equilibrium(self.lattice, rho[node], u[:, node])
        if self.g is not None:
            phi = np.zeros(self.N) if phi is None else np.asarray(phi, dtype=np.float64).reshape(self.N)
            for node in range(self.N):
                self.g[:, node] = scalar_equilibrium(phi[node], u[:2, node])
        self.step_count = 0

    def init_uniform(self, rho=1.0, u=(0.0, 0.0, 0.0), phi=0.0):
        """Equilibrium of one (rho, u, phi) at every node (computed once, broadcast)."""
        self.f[:] = flow_equilibrium(self.lattice, rho, u)[:, None]
        if self.g is not None:
            self.g[:] = scalar_equilibrium(phi, u[:2])[:, None]
        self.step_count = 0

    def run(self, nsteps):
        rc = lib().orc_run(ctypes.byref(self.params), _p(self.f), _p(self.g), int(self.step_count), int(nsteps))
        if rc != 0:
            raise MemoryError("orc_run failed")
        self.step_count += int(nsteps)

    def moments(self, kind=0):
        """(rho[N], u[d][N], phi[N] or None): kind 0 = output (eqs. 24, 42),
        kind 1 = half-forced (eqs. 25, 43)."""
        rho = np.zeros(self.N)
        u = np.zeros((self.d, self.N))
        phi = np.zeros(self.N) if self.g is not None else None
        lib().orc_moments(ctypes.byref(self.params), _p(self.f), _p(self.g), int(self.step_count), int(kind),
                          _p(rho), _p(u), _p(phi))
        return rho, u, phi

    def strain_rate_squared(self):
        """S:S [N] of the flow's strain rate (the viscous-heating source per unit
        coefficient) from the streamed populations of the stored state (D2Q9 flow)."""
        out = np.zeros(self.N)
        if lib().orc_strain_rate_field(ctypes.byref(self.params), _p(self.f), int(self.step_count), _p(out)) != 0:
            raise ValueError("strain rate: D2Q9 flow lattices only")
        return out

    def totals(self):
        """Mass, momentum (3) and scalar total of the stored state."""
        e = velocities(self.lattice)
        out = np.zeros(5)
        out[0] = self.f.sum()
        for i in range(3):
            out[1 + i] = (self.f * e[:, i][:, None]).sum()
        if self.g is not None:
            out[4] = self.g.sum()
        return out

    def grid(self, a):
        """View of a [N] array as [nz][ny][nx]."""
        nx, ny, nz = self.shape
        return np.asarray(a).reshape(nz, ny, nx)
