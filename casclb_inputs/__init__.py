"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the oracle.

This module holds none of the lattice Boltzmann arithmetic: it only draws
random numbers and evaluates the prescribed force/source patterns of the
workloads (sums of sinusoids).  Arrays follow the layout used everywhere in
this project: a field with `c` components over an (nx, ny, nz) lattice is a
float64 array [c][N], N = nx*ny*nz, x fastest (index x + nx*(y + ny*z)).

Workloads (the paper's analytic benchmarks scaled up; no dataset is involved):
  * ``poiseuille_channel``  D2Q9, 4 x 64, periodic x, walls on y, Fx = 1e-6,
    nu = 1/6, 20000 steps (body-force-driven Poiseuille flow of Sec. 6).
  * ``coupled_2d``          D2Q9 flow + D2Q5 scalar, 4096^2 periodic; force
    A(sin(2 pi x/L) cos(2 pi y/L), -cos(2 pi x/L) sin(2 pi y/L)) cos(w t),
    A = 1e-5, w = 2 pi / 10000; source B sin(2 pi x/L) sin(2 pi y/L),
    B = 1e-6; nu and D drawn from U[0.01, 0.1] (four-rolls-mill type forcing
    and a smooth source, Sec. 6).
  * ``duct_3d``             D3Q27 square duct 256^3, periodic x, walls on
    y and z, Fx = 1e-7, tau = 0.76 (square-duct flow of Sec. 6).
  * ``periodic_3d``         D3Q27 512^3 periodic; force = sum of 8 Fourier
    modes with integer wave vectors in {-4..4}^3 \\ {0}, amplitudes
    U[-1e-6, 1e-6] per component, phases U[0, 2 pi).
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

SEED = 0


def rng(seed: int = SEED) -> np.random.Generator:
    return np.random.default_rng(seed)


def coords(shape):
    """Integer node coordinates (x, y, z) as [3][N] int64, x fastest."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()]).astype(np.int64)


# ---------------------------------------------------------------------------
# force / source patterns
# ---------------------------------------------------------------------------

@dataclass
class FourierModes:
    """F(x) = sum_m a_m sin(2 pi k_m . x / L + theta_m), componentwise."""
    k: np.ndarray       # [M][3] integer wave vectors
    a: np.ndarray       # [M][3] amplitude vectors
    theta: np.ndarray   # [M] phases
    L: Tuple[int, int, int]

    def evaluate(self, pts: np.ndarray) -> np.ndarray:
        """pts [3][P] integer coordinates -> [3][P] force values."""
        pts = np.asarray(pts, dtype=np.float64)
        out = np.zeros((3, pts.shape[1]))
        for m in range(self.k.shape[0]):
            ph = 2.0 * np.pi * sum(self.k[m, i] * pts[i] / self.L[i] for i in range(3)) + self.theta[m]
            s = np.sin(ph)
            for i in range(3):
                out[i] += self.a[m, i] * s
        return out

    def field(self, shape, dtype=np.float64) -> np.ndarray:
        """[3][N] field over the whole lattice, evaluated plane by plane."""
        nx, ny, nz = shape
        out = np.empty((3, nx * ny * nz), dtype=dtype)
        plane = nx * ny
        xy = coords((nx, ny, 1))
        for z in range(nz):
            pts = np.vstack([xy[0], xy[1], np.full(plane, z)])
            out[:, z * plane:(z + 1) * plane] = self.evaluate(pts)
        return out


def fourier_modes(L=(512, 512, 512), nmodes=8, amp=1e-6, kmax=4, seed=SEED) -> FourierModes:
    g = rng(seed)
    ks = []
    while len(ks) < nmodes:
        k = g.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    a = g.uniform(-amp, amp, size=(nmodes, 3))
    theta = g.uniform(0.0, 2.0 * np.pi, size=nmodes)
    return FourierModes(np.array(ks, dtype=np.int64), a, theta, tuple(L))


def vortex_force_2d(shape, A=1e-5, pts: Optional[np.ndarray] = None) -> np.ndarray:
    """A (sin(2 pi x/L) cos(2 pi y/L), -cos(2 pi x/L) sin(2 pi y/L)) as [2][N] (or [2][P] at pts)."""
    nx, ny, _ = shape
    if pts is None:
        pts = coords(shape)
    x = 2.0 * np.pi * pts[0] / nx
    y = 2.0 * np.pi * pts[1] / ny
    return np.stack([A * np.sin(x) * np.cos(y), -A * np.cos(x) * np.sin(y)])


def product_source_2d(shape, B=1e-6, pts: Optional[np.ndarray] = None) -> np.ndarray:
    """B sin(2 pi x/L) sin(2 pi y/L) as [N] (or [P] at pts)."""
    nx, ny, _ = shape
    if pts is None:
        pts = coords(shape)
    return B * np.sin(2.0 * np.pi * pts[0] / nx) * np.sin(2.0 * np.pi * pts[1] / ny)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    lattice: str                      # "D2Q9", "D2Q9_D2Q5", "D3Q27"
    shape: Tuple[int, int, int]
    walls: Tuple[bool, bool, bool]    # halfway bounce-back walls on both ends of an axis
    nu: float
    steps: int
    force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    D: float = 0.0
    force_omega: float = 0.0          # > 0: force multiplied by cos(force_omega t)
    extra: dict = field(default_factory=dict)


def poiseuille_channel() -> Workload:
    return Workload("poiseuille_channel_4x64", "D2Q9", (4, 64, 1), (False, True, False), nu=1.0 / 6.0,
                    steps=20000, force=(1e-6, 0.0, 0.0))


def coupled_2d(L=4096, seed=SEED) -> Workload:
    g = rng(seed)
    nu, D = g.uniform(0.01, 0.1, size=2)
    return Workload(f"coupled_d2q9_d2q5_{L}x{L}", "D2Q9_D2Q5", (L, L, 1), (False, False, False), nu=float(nu),
                    steps=1000, D=float(D), force_omega=2.0 * np.pi / 10000.0, extra={"A": 1e-5, "B": 1e-6})


def duct_3d(n=256) -> Workload:
    tau = 0.76
    return Workload(f"duct_d3q27_{n}^3", "D3Q27", (n, n, n), (False, True, True), nu=(tau - 0.5) / 3.0,
                    steps=200, force=(1e-7, 0.0, 0.0))


def periodic_3d(n=512, seed=SEED) -> Workload:
    tau = 0.76
    return Workload(f"periodic_d3q27_{n}^3", "D3Q27", (n, n, n), (False, False, False), nu=(tau - 0.5) / 3.0,
                    steps=200, extra={"modes": fourier_modes((n, n, n), seed=seed)})


# ---------------------------------------------------------------------------
# random states for unit and parity tests
# ---------------------------------------------------------------------------

def smooth_fields(shape, d, amp_rho=0.02, amp_u=0.03, amp_phi=0.5, seed=SEED):
    """Seeded smooth (rho, u, phi) fields: a few low sinusoids plus a little noise.

    Returns rho [N], u [d][N], phi [N]."""
    g = rng(seed)
    pts = coords(shape).astype(np.float64)
    n = pts.shape[1]

    def smooth(amp):
        v = np.zeros(n)
        for _ in range(3):
            k = g.integers(1, 3, size=3)
            ph = g.uniform(0, 2 * np.pi)
            v += g.uniform(-amp, amp) * np.sin(sum(2 * np.pi * k[i] * pts[i] / shape[i] for i in range(3)) + ph)
        return v + 0.1 * amp * g.standard_normal(n)

    rho = 1.0 + smooth(amp_rho)
    u = np.stack([smooth(amp_u) for _ in range(d)])
    phi = smooth(amp_phi)
    return rho, u, phi


def smooth_fields_at(shape, pts, d, amp_rho=0.02, amp_u=0.03, amp_phi=0.5, seed=SEED):
    """Seeded smooth (rho, u, phi) evaluated at integer points pts [3][P] of a lattice of
    `shape` (three sinusoids per field, periodic on the lattice, no per-node noise), so
    that any sub-box gives the same values as the full lattice."""
    g = rng(seed)
    pts = np.asarray(pts, dtype=np.float64)

    def smooth(amp):
        v = np.zeros(pts.shape[1])
        for _ in range(3):
            k = g.integers(1, 3, size=3)
            ph = g.uniform(0, 2 * np.pi)
            a = g.uniform(-amp, amp)
            arg = sum(2 * np.pi * k[i] * pts[i] / shape[i] for i in range(3)) + ph
            v += a * np.sin(arg)
        return v

    rho = 1.0 + smooth(amp_rho)
    u = np.stack([smooth(amp_u) for _ in range(d)])
    phi = smooth(amp_phi)
    return rho, u, phi


def hartmann_batch(n=4096, U0=0.01, seed=SEED, nx_range=(4, 64), ny_range=(16, 256), ha_range=(0.0, 20.0),
                   nu_range=(0.02, 0.2)):
    """Seeded batch of independent Hartmann channels (Sec. 6 Hartmann flow as a parameter
    sweep): nx, ny uniform integers, Ha and nu uniform; driving force
    F_b = 2 rho nu U0 / L^2 (the Poiseuille force for centre-line velocity U0), Lorentz
    coefficient s = Ha^2 rho nu / L^2, L = ny / 2, rho = 1.  Returns a list of
    (nx, ny, nu, F_b, s, Ha)."""
    g = rng(seed)
    nx = g.integers(nx_range[0], nx_range[1] + 1, size=n)
    ny = g.integers(ny_range[0], ny_range[1] + 1, size=n)
    ha = g.uniform(*ha_range, size=n)
    nu = g.uniform(*nu_range, size=n)
    L = ny / 2.0
    fb = 2.0 * nu * U0 / L**2
    s = ha**2 * nu / L**2
    return [(int(nx[i]), int(ny[i]), float(nu[i]), float(fb[i]), float(s[i]), float(ha[i])) for i in range(n)]


def noise(shape_or_n, scale, seed=SEED):
    return scale * rng(seed).standard_normal(shape_or_n)


# ---------------------------------------------------------------------------
# warm-start problems: steady periodic flow + scalar under random smooth forcing
# ---------------------------------------------------------------------------

@dataclass
class WarmstartCase:
    """One periodic L x L D2Q9 + D2Q5 problem: force F [2][N], source S [N]
    (both sums of `nmodes` sinusoids with integer wave vectors, zero mean),
    viscosity nu and diffusivity D."""
    L: int
    nu: float
    D: float
    F: np.ndarray
    S: np.ndarray
    seed: int


def _wave_vectors(g, nmodes, kmin, kmax):
    ks = []
    while len(ks) < nmodes:
        k = g.integers(-kmax, kmax + 1, size=2)
        if kmin * kmin <= int(k @ k) <= kmax * kmax:
            ks.append(k)
    return np.array(ks, dtype=np.int64)


def _sinusoids(L, k, amp, theta):
    """sum_m amp[m] sin(2 pi k_m . x / L + theta_m) on the L x L grid, as [..., N] (x fastest)."""
    y, x = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    x = x.ravel().astype(np.float64)
    y = y.ravel().astype(np.float64)
    out = np.zeros(amp.shape[1:] + (L * L,))
    for m in range(k.shape[0]):
        s = np.sin(2.0 * np.pi * (k[m, 0] * x + k[m, 1] * y) / L + theta[m])
        out += amp[m][..., None] * s
    return out


def warmstart_case(seed, L=256, nu=None, D=None, nmodes=8, kmin=3, kmax=8, u_range=(0.005, 0.02),
                   phi_range=(0.5, 2.0), rate_range=(0.08, 0.2)):
    """Seeded problem of the warm-start study.  Wave vectors are integer with
    kmin <= |k| <= kmax (wavelengths L/8 .. L/3); per-mode amplitudes are drawn
    uniform in [-1, 1] and then scaled together so that the bound
    sum_m |a_m| / (nu |k_m|^2) of the steady (Stokes) speed equals a speed drawn
    from u_range (the force amplitudes this gives, 1e-6 .. 1e-4, keep the flow
    far below the lattice sound speed); the source likewise against D and
    phi_range.  nu and D are drawn from rate_range unless given."""
    g = rng(seed)
    if nu is None:
        nu = float(g.uniform(*rate_range))
    if D is None:
        D = float(g.uniform(*rate_range))
    kw = 2.0 * np.pi / L
    kf = _wave_vectors(g, nmodes, kmin, kmax)
    af = g.uniform(-1.0, 1.0, size=(nmodes, 2))
    tf = g.uniform(0.0, 2.0 * np.pi, size=nmodes)
    k2f = kw * kw * (kf**2).sum(axis=1)
    bound = (np.linalg.norm(af, axis=1) / (nu * k2f)).sum()
    af *= g.uniform(*u_range) / bound
    ks = _wave_vectors(g, nmodes, kmin, kmax)
    bs = g.uniform(-1.0, 1.0, size=nmodes)
    ts = g.uniform(0.0, 2.0 * np.pi, size=nmodes)
    k2s = kw * kw * (ks**2).sum(axis=1)
    bs *= g.uniform(*phi_range) / (np.abs(bs) / (D * k2s)).sum()
    F = _sinusoids(L, kf, af, tf)              # [2][N]
    S = _sinusoids(L, ks, bs[:, None], ts)[0]  # [N]
    return WarmstartCase(L, nu, D, F, S, seed)


def warmstart_group(seed, nslices, L=256, rate_range=(0.08, 0.2)):
    """`nslices` problems sharing one (nu, D) pair drawn from `seed` (a stack of
    slices for one solver context); slice i uses seed 1000 * seed + i."""
    g = rng(seed)
    nu, D = (float(v) for v in g.uniform(*rate_range, size=2))
    return [warmstart_case(1000 * seed + i, L=L, nu=nu, D=D) for i in range(nslices)]
