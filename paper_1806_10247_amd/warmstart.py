"""Learned warm start for steady periodic flow + scalar problems.

The lattice is initialised with the product-form equilibrium of an estimate
of the steady density rho, half-forced velocity u and half-sourced scalar phi
(converted to the populations' own moments, j = rho u - F/2 and phi - S/2)
and then iterated with the cascaded scheme until both residuals (velocity and
scalar, every K steps) fall below the tolerance, exactly as from a start from
rest: the estimate only moves the starting point, the converged answer is the
solver's.  The first few steps are each followed by a reset of the stored
moments to the estimate's (lb_reset_moments_device, keeping f - f_eq), which
gives the populations the non-equilibrium part that belongs to the
estimate's gradients; started at equilibrium they would launch a transient
that costs thousands of steps.

The estimate has two parts:
  1. coarse solves: the same problem on the L/2, L/4 and L/8 lattices under
     diffusive scaling (per halving dx x2, dt x4: force x8, source x4, same nu
     and D), each run to the tolerance (L/8 from rest, L/4 from the L/8
     solution, L/2 from the extrapolated L/4 and L/8 solutions:
     coarse_solutions); velocity, scalar and density deviation
     rescaled to the finer lattice (u/2, phi, (rho - mean)/4: the pressure
     scales as u^2) and upsampled (periodic Catmull-Rom).  The levels are
     combined by extrapolation on the L/2 lattice,
     f = f1 + a (f1 - f2) + b (f2 - f3).  Richardson's a = 1/3, b = 0 assumes
     an error exactly proportional to dx^2 (the scheme is second order in dx
     and, under diffusive scaling, its compressibility error is too); the
     weights used are fitted by least squares to the training solutions'
     largest scales (ExtrapolationFit), a pair per field.  This fixes the large
     scales, whose slow decay decides the iteration count;
  2. a U-Net (include/casclb_unet.h, bf16 matrix cores) that maps the force,
     source, rates and that guess to the remaining fine-lattice correction of
     all four fields, used only if it pays on validation problems (select()).
The density matters as much as the velocity: started from the exact steady
u and phi at uniform density, the pressure mismatch launches sound waves
whose slow viscous decay costs about half the steps of a cold start.
Every estimate is projected: means removed (mass, momentum and scalar totals
are conserved under zero-mean force and source, and a start from rest has
them at the rest values) and the Nyquist lines k_x = pi, k_y = pi removed
(the iteration leaves those modes unchanged, so any in an estimate would stay
in the converged state).

All field work runs on the GPU: restriction, prolongation, extrapolation,
projection, packing of the network's input and output and the initial
moments are kernels of include/casclb_warm.h, the solves and the network the
library's; torch tensors serve as device memory only.

Training data are steady solutions this solver produces: problems sharing
one (nu, D) pair run as the slices of one stacked 2D context (nz slices, one
launch per step), each slice's own residual checked at the end.  The weights
file holds the network's parameters, the fitted extrapolation weights and the
choices select() made (network on or off, reset cycles).

    python -m paper_1806_10247_amd.warmstart train --groups 64 --slices 16 --out weights.npz
    python -m paper_1806_10247_amd.warmstart select --weights weights.npz --out weights.npz
    python -m paper_1806_10247_amd.warmstart evaluate --weights weights.npz --cases 8
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import capi as C
from .solver import Solver

# feature / target scales (lattice units)
U0 = 0.01          # velocity scale
PHI0 = 1.0         # scalar scale
RHO0 = 3.0 * U0 * U0   # density-deviation scale (pressure ~ rho u^2, c_s^2 = 1/3)
K0 = 2.0 * math.pi * 5.0 / 256.0   # a mid wavenumber of the forcing (L = 256)
RATE_MID, RATE_HALF = 0.14, 0.06   # nu and D are mapped to (rate - mid) / half
RES = 0.02         # scale of the learned correction relative to U0 / PHI0
IN_CH, OUT_CH = 9, 4
LEVEL_IN_CH = 13   # features "levels": F (2), S, the two rates, h - q and q - o (u_x, u_y, phi, rho each)
CORRECTION_K2 = 5  # the network's correction keeps its modes with |k|^2 > 5: the largest scales are the guess's
RES_LOW = 5e-4     # scale of the low-mode correction (head "low") relative to U0 / PHI0 / RHO0
HEADS = ("full", "low")   # full: the correction outside the largest scales; low: only the modes 0 < |k|^2 <= 8


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# device field pipeline (include/casclb_warm.h); every array is a torch tensor
# on the GPU used only as memory, every operation a library kernel
# ---------------------------------------------------------------------------

def _ptr(t):
    return t.data_ptr() if t is not None else None


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _empty(*shape):
    import torch
    return torch.empty(*shape, dtype=torch.float64, device="cuda")


class Problems:
    """Force [2][B][L][L] and source [B][L][L] of B problems sharing (nu, D), on
    the device; `coarser()` gives the same problems on the L/2 lattice under
    diffusive scaling (dx x2, dt x4: force x8, source x4, block means)."""

    def __init__(self, L, nu, D, F, S, seeds=()):
        self.L, self.nu, self.D, self.F, self.S = L, nu, D, F, S
        self.B = S.numel() // (L * L)
        self.seeds = tuple(seeds)

    @classmethod
    def from_cases(cls, cases):
        import torch
        L = cases[0].L
        F = np.concatenate([c.F for c in cases], axis=1)
        S = np.concatenate([c.S for c in cases])
        return cls(L, cases[0].nu, cases[0].D, torch.from_numpy(np.ascontiguousarray(F)).cuda(),
                   torch.from_numpy(np.ascontiguousarray(S)).cuda(), [c.seed for c in cases])

    def coarser(self):
        Lc = self.L // 2
        F = _empty(2 * self.B * Lc * Lc)
        S = _empty(self.B * Lc * Lc)
        C.lb_warm_restrict(_ptr(self.F), 2 * self.B, self.L, 8.0, _ptr(F), _stream())
        C.lb_warm_restrict(_ptr(self.S), self.B, self.L, 4.0, _ptr(S), _stream())
        return Problems(Lc, self.nu, self.D, F, S, self.seeds)


class Fields:
    """(rho or rho - rho0 [B N], u [2][B N], phi [B N]) of B problems on an L x L
    lattice, device float64 (N = L^2, the node order of the solver)."""

    def __init__(self, L, B, rho=None, u=None, phi=None):
        n = B * L * L
        self.L, self.B = L, B
        self.buf = None
        if rho is None and u is None and phi is None:
            # one allocation, planes in the order rho, u_x, u_y, phi: plane-wise
            # operations on all fields are one launch
            self.buf = _empty(4 * n)
            rho, u, phi = self.buf[:n], self.buf[n:3 * n], self.buf[3 * n:]
        self.rho = rho if rho is not None else _empty(n)
        self.u = u if u is not None else _empty(2 * n)
        self.phi = phi if phi is not None else _empty(n)

    def planes(self):
        return ((self.rho, self.B), (self.u, 2 * self.B), (self.phi, self.B))

    def spans(self):
        """The planes as few (tensor, planes) runs as the storage allows: one
        run over all 4 B planes for Fields that own one allocation."""
        return ((self.buf, 4 * self.B),) if self.buf is not None else self.planes()

    def project(self, k2max=0):
        """Means and Nyquist lines (and the modes 0 < |k|^2 <= k2max) removed from
        every plane, in place."""
        for a, p in self.spans():
            C.lb_warm_project(_ptr(a), p, self.L, k2max, _stream())
        return self

    @classmethod
    def stack(cls, parts):
        """The problems of several Fields (same L) as one batch, in order."""
        import torch
        u = torch.cat([f.u.view(2, -1) for f in parts], dim=1).reshape(-1)
        return cls(parts[0].L, sum(f.B for f in parts), torch.cat([f.rho for f in parts]), u,
                   torch.cat([f.phi for f in parts]))

    def host(self):
        n = self.B * self.L * self.L
        return (self.rho.cpu().numpy(), self.u.cpu().numpy().reshape(2, n), self.phi.cpu().numpy())


# rescaling from the L/2 to the L lattice under diffusive scaling: density deviation, velocity, scalar
_LEVEL_SCALE = (0.25, 0.5, 1.0)


def prolong(f):
    """Fields on the 2L lattice from those on L, rescaled (u/2, (rho - .)/4)."""
    g = Fields(2 * f.L, f.B)
    for (a, p), (b, _), s in zip(f.planes(), g.planes(), _LEVEL_SCALE):
        C.lb_warm_prolong(_ptr(a), p, f.L, s, _ptr(b), _stream())
    return g


# Richardson's weight for a leading error proportional to dx^2, per field (density, velocity, scalar)
RICHARDSON = (1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0)
EXTRAPOLATION_K2 = 8   # the fitted extrapolation weights minimise the error in the modes 0 < |k|^2 <= 8


def _weights(w):
    return tuple(float(v) for v in (w if np.ndim(w) else (w, w, w)))


def extrapolate(f1, f2, w=RICHARDSON):
    """(1 + w) f1 - w P f2 on f1's lattice (f2 on the half-size lattice, P the
    rescaled prolongation), w per field (density, velocity, scalar) or one
    number.  w = 1/3 is Richardson's: the leading error, proportional to dx^2,
    is four times larger in f2.  Densities may carry any constant; remove it
    later."""
    g = prolong(f2)
    for (a, _), (b, _), wi in zip(f1.planes(), g.planes(), _weights(w)):
        C.lb_warm_axpby(a.numel(), 1.0 + wi, _ptr(a), -wi, _ptr(b), _ptr(b), _stream())
    return g


def richardson(f1, f2):
    return extrapolate(f1, f2, RICHARDSON)


def extrapolate3(f1, f2, f3, a, b):
    """(1 + a) f1 - a P f2 + b (P f2 - P P f3) on f1's lattice (f2 and f3 on the
    half- and quarter-size lattices, P the rescaled prolongation), per field
    (density, velocity, scalar) or one number each: the two-level combination
    plus a share b of the next coarser difference.  b = 0 is extrapolate()."""
    p2 = prolong(f2)
    p3 = prolong(prolong(f3))
    g = Fields(f1.L, f1.B)
    for (x, _), (y, _), (z, _), (o, _), ai, bi in zip(f1.planes(), p2.planes(), p3.planes(), g.planes(),
                                                      _weights(a), _weights(b)):
        C.lb_warm_axpby(x.numel(), 1.0 + ai, _ptr(x), bi - ai, _ptr(y), _ptr(o), _stream())
        C.lb_warm_axpby(x.numel(), 1.0, _ptr(o), -bi, _ptr(z), _ptr(o), _stream())
    return g


def guess_from_levels(f1, f2, w=RICHARDSON, f3=None, wb=None):
    """Fine-lattice guess (rho - rho0, u, phi) from the steady fields of the L/2
    (f1) and L/4 (f2) problems: extrapolation on the L/2 lattice with weights w
    (with f3, the L/8 fields, and wb: extrapolate3 with a = w, b = wb),
    prolongation, projection."""
    if f3 is not None and wb is not None:
        return prolong(extrapolate3(f1, f2, f3, w, wb)).project()
    return prolong(extrapolate(f1, f2, w)).project()


def _axpby(a, x, b, y, out):
    """out = a x + b y over every plane (Fields of the same shape), in as few
    launches as their storage allows."""
    runs = (x.spans(), y.spans(), out.spans()) if x.buf is not None and y.buf is not None and out.buf is not None \
        else (x.planes(), y.planes(), out.planes())
    for (p, _), (q, _), (r, _) in zip(*runs):
        C.lb_warm_axpby(p.numel(), a, _ptr(p), b, _ptr(q), _ptr(r), _stream())
    return out


def _copy(f):
    return _axpby(1.0, f, 0.0, f, Fields(f.L, f.B))


def _combine(a, x, b, y):
    """a x + b y, new Fields."""
    return _axpby(a, x, b, y, Fields(x.L, x.B))


def low_modes(f, k2max=EXTRAPOLATION_K2):
    """The part of f in the Fourier modes 0 < |k|^2 <= k2max (new Fields)."""
    return _combine(1.0, _copy(f).project(), -1.0, _copy(f).project(k2max))


class ExtrapolationFit:
    """Least-squares extrapolation weights from steady solutions.

    With two levels the fine-lattice guess with weight a is (1 + a) h - a q,
    h = P f1 and q = P P f2 (prolonged and projected L/2 and L/4 solutions);
    with three it is (1 + a) h - a q + b (q - o), o = P P P f3 (L/8), since
    prolongation and projection are linear.  Per field (density, velocity,
    scalar), the weights minimise the summed squared error against the fine
    solutions in the modes 0 < |k|^2 <= k2max, the largest scales, whose slow
    decay sets the iteration count: the normal equations of r = truth - h on
    the differences d1 = h - q (and d2 = q - o), all restricted to those
    modes.  Sums in float64 on the host, in the order the solutions are added."""

    def __init__(self, k2max=EXTRAPOLATION_K2, levels=2):
        if levels not in (2, 3):
            raise ValueError("two or three levels")
        self.k2max = k2max
        self.levels = levels
        nb = levels - 1
        self.gram = np.zeros((3, nb, nb))
        self.rhs = np.zeros((3, nb))
        self.count = 0

    def add(self, truth, f1, f2, keep=None, f3=None):
        """truth on the L lattice (projected in place), f1 / f2 (/ f3) the steady
        fields of the same B problems on the L/2 and L/4 (and L/8) lattices;
        keep selects problems."""
        h = prolong(f1).project()
        q = prolong(prolong(f2)).project()
        r = low_modes(_combine(1.0, truth.project(), -1.0, h), self.k2max)
        ds = [low_modes(_combine(1.0, h, -1.0, q), self.k2max)]
        if self.levels == 3:
            if f3 is None:
                raise ValueError("a three-level fit needs the L/8 fields")
            o = prolong(prolong(prolong(f3))).project()
            ds.append(low_modes(_combine(1.0, q, -1.0, o), self.k2max))
        keep = list(range(truth.B)) if keep is None else list(keep)
        n = truth.L * truth.L
        host = lambda a, p: a.cpu().numpy().reshape(p // truth.B, truth.B, n)[:, keep].ravel()
        for i, planes in enumerate(zip(r.planes(), *(d.planes() for d in ds))):
            (a, p), rest = planes[0], planes[1:]
            av = host(a, p)
            dv = [host(d, p) for d, _ in rest]
            for j, x in enumerate(dv):
                self.rhs[i, j] += float(np.dot(x, av))
                for k, y in enumerate(dv):
                    self.gram[i, j, k] += float(np.dot(x, y))
        self.count += len(keep)

    def weights(self):
        """(a per field) with two levels, ((a per field), (b per field)) with three."""
        if self.count == 0 or np.any(self.gram[:, 0, 0] <= 0.0):
            raise ValueError("extrapolation fit: no solutions with large-scale content")
        sol = np.array([np.linalg.solve(self.gram[i], self.rhs[i]) for i in range(3)])
        if self.levels == 2:
            return tuple(float(v) for v in sol[:, 0])
        return tuple(float(v) for v in sol[:, 0]), tuple(float(v) for v in sol[:, 1])


def guess_from_half(f1):
    """The guess from the L/2 solve alone (for comparison)."""
    return prolong(f1).project()


def features(probs, guess, out):
    """Network input [B][L][L][9] (float32, device): F/(nu K0^2 U0) (2),
    S/(D K0^2 PHI0), the two rates as constant channels, the guess u/U0 (2),
    phi/PHI0, (rho - rho0)/RHO0."""
    n = probs.B * probs.L * probs.L
    fs = 1.0 / (probs.nu * K0 * K0 * U0)
    ch = [dict(src=_ptr(probs.F), scale=fs), dict(src=_ptr(probs.F) + 8 * n, scale=fs),
          dict(src=_ptr(probs.S), scale=1.0 / (probs.D * K0 * K0 * PHI0)),
          dict(src=None, offset=(probs.nu - RATE_MID) / RATE_HALF),
          dict(src=None, offset=(probs.D - RATE_MID) / RATE_HALF),
          dict(src=_ptr(guess.u), scale=1.0 / U0), dict(src=_ptr(guess.u) + 8 * n, scale=1.0 / U0),
          dict(src=_ptr(guess.phi), scale=1.0 / PHI0), dict(src=_ptr(guess.rho), scale=1.0 / RHO0)]
    C.lb_warm_pack(ch, probs.B, probs.L * probs.L, _ptr(out), _stream())
    return out


_OUT_SCALE = (RES * U0, RES * U0, RES * PHI0, RES * RHO0)   # u_x, u_y, phi, rho channels


def _out_channels(guess, est, scales=None):
    n = guess.B * guess.L * guess.L
    srcs = (_ptr(guess.u), _ptr(guess.u) + 8 * n, _ptr(guess.phi), _ptr(guess.rho))
    dsts = (_ptr(est.u), _ptr(est.u) + 8 * n, _ptr(est.phi), _ptr(est.rho))
    return [dict(src=a, dst=b, scale=s) for a, b, s in zip(srcs, dsts, scales or _OUT_SCALE)]


def targets(truth, guess, out, scales=None):
    """The correction truth - guess, [B][L][L][4] float32 (device), channels
    (u_x, u_y, phi, density) divided by `scales` (default RES U0, RES U0,
    RES PHI0, RES RHO0); truth is projected in place."""
    truth.project()
    sc = scales or _OUT_SCALE
    n = guess.B * guess.L * guess.L
    diff = Fields(guess.L, guess.B)
    for (a, _), (b, _), (d, _) in zip(truth.planes(), guess.planes(), diff.planes()):
        C.lb_warm_axpby(a.numel(), 1.0, _ptr(a), -1.0, _ptr(b), _ptr(d), _stream())
    ch = [dict(src=_ptr(diff.u), scale=1.0 / sc[0]), dict(src=_ptr(diff.u) + 8 * n, scale=1.0 / sc[1]),
          dict(src=_ptr(diff.phi), scale=1.0 / sc[2]), dict(src=_ptr(diff.rho), scale=1.0 / sc[3])]
    C.lb_warm_pack(ch, guess.B, guess.L * guess.L, _ptr(out), _stream())
    return out


def level_differences(f1, f2, f3):
    """(h - q, q - o) on the fine lattice, h, q, o the prolonged and projected
    steady fields of the L/2, L/4 and L/8 problems: the differences between
    successive levels, of the size of the discretisation errors the
    extrapolation removes (the guess is (1 + a) h - a q + b (q - o)).  As
    prolongation and projection are linear, each difference is taken on the
    coarser lattice and prolonged once: h - q = P (f1 - P f2), q - o =
    P P (f2 - P f3), then projected."""
    d1 = prolong(_combine(1.0, f1, -1.0, prolong(f2))).project()
    d2 = prolong(prolong(_combine(1.0, f2, -1.0, prolong(f3)))).project()
    return d1, d2


def features_levels(probs, d1, d2, scales, out):
    """Network input of the "levels" features [B][L][L][13] (float32, device):
    F/(nu K0^2 U0) (2), S/(D K0^2 PHI0), the two rates as constant channels, then
    h - q and q - o as (u_x, u_y, phi, density) channels divided by `scales`
    (8 numbers, the channels' r.m.s. over the training solutions)."""
    n = probs.B * probs.L * probs.L
    fs = 1.0 / (probs.nu * K0 * K0 * U0)
    ch = [dict(src=_ptr(probs.F), scale=fs), dict(src=_ptr(probs.F) + 8 * n, scale=fs),
          dict(src=_ptr(probs.S), scale=1.0 / (probs.D * K0 * K0 * PHI0)),
          dict(src=None, offset=(probs.nu - RATE_MID) / RATE_HALF),
          dict(src=None, offset=(probs.D - RATE_MID) / RATE_HALF)]
    for d, sc in ((d1, scales[:4]), (d2, scales[4:])):
        ch += [dict(src=_ptr(d.u), scale=1.0 / sc[0]), dict(src=_ptr(d.u) + 8 * n, scale=1.0 / sc[1]),
               dict(src=_ptr(d.phi), scale=1.0 / sc[2]), dict(src=_ptr(d.rho), scale=1.0 / sc[3])]
    C.lb_warm_pack(ch, probs.B, probs.L * probs.L, _ptr(out), _stream())
    return out


def estimate(guess, y, k2max=None, scales=None):
    """The guess plus the network's correction y ([B][L][L][4] float32, device,
    channels times `scales`, default those of targets()), projected (means and
    Nyquist lines removed); the correction's modes with 0 < |k|^2 <= k2max
    (default CORRECTION_K2) are removed first, so the largest scales stay the
    multilevel guess's."""
    k2max = CORRECTION_K2 if k2max is None else k2max
    corr = Fields(guess.L, guess.B)
    chans = _out_channels(guess, corr, scales)
    for c in chans:
        c["src"] = None   # the correction alone
    C.lb_warm_unpack(_ptr(y), chans, guess.B, guess.L * guess.L, _stream())
    # the projected correction has no mean or Nyquist content and the guess is
    # projected: the sum needs no further projection
    return _axpby(1.0, guess, 1.0, corr.project(k2max), corr)


_OUT_SCALE_LOW = (RES_LOW * U0, RES_LOW * U0, RES_LOW * PHI0, RES_LOW * RHO0)


def targets_low(truth, guess, out, k2max=EXTRAPOLATION_K2):
    """The part of truth - guess in the modes 0 < |k|^2 <= k2max (the largest
    scales, whose slow decay sets the iteration count), [B][L][L][4] float32
    (device) in units of RES_LOW U0 (u), RES_LOW PHI0 (phi), RES_LOW RHO0
    (density); truth is projected in place."""
    low = low_modes(_combine(1.0, truth.project(), -1.0, guess), k2max)
    n = guess.B * guess.L * guess.L
    ch = [dict(src=_ptr(low.u), scale=1.0 / _OUT_SCALE_LOW[0]), dict(src=_ptr(low.u) + 8 * n, scale=1.0 / _OUT_SCALE_LOW[1]),
          dict(src=_ptr(low.phi), scale=1.0 / _OUT_SCALE_LOW[2]), dict(src=_ptr(low.rho), scale=1.0 / _OUT_SCALE_LOW[3])]
    C.lb_warm_pack(ch, guess.B, guess.L * guess.L, _ptr(out), _stream())
    return out


def estimate_low(guess, y, k2max=EXTRAPOLATION_K2):
    """The guess plus the modes 0 < |k|^2 <= k2max of the network's output y
    (units of targets_low), projected."""
    import torch

    zero = Fields(guess.L, guess.B, *(torch.zeros_like(a) for a, _ in guess.planes()))
    corr = Fields(guess.L, guess.B)
    n = guess.B * guess.L * guess.L
    srcs = (_ptr(zero.u), _ptr(zero.u) + 8 * n, _ptr(zero.phi), _ptr(zero.rho))
    dsts = (_ptr(corr.u), _ptr(corr.u) + 8 * n, _ptr(corr.phi), _ptr(corr.rho))
    C.lb_warm_unpack(_ptr(y), [dict(src=a, dst=b, scale=sc) for a, b, sc in zip(srcs, dsts, _OUT_SCALE_LOW)],
                     guess.B, guess.L * guess.L, _stream())
    return _combine(1.0, guess, 1.0, low_modes(corr, k2max)).project()


def apply_network(net, probs, guess, levels=None):
    """The estimate: the guess plus the network's correction, as net.head says;
    `levels` = (L/2, L/4, L/8 steady fields) for the "levels" features."""
    import torch

    if net.features == "levels":
        d1, d2 = level_differences(*levels)
        x = features_levels(probs, d1, d2, net.in_scale,
                            torch.empty(probs.B, probs.L, probs.L, LEVEL_IN_CH, dtype=torch.float32, device="cuda"))
    else:
        x = features(probs, guess, torch.empty(probs.B, probs.L, probs.L, IN_CH, dtype=torch.float32, device="cuda"))
    y = net.forward(x)
    if net.head == "low":
        return estimate_low(guess, y)
    return estimate(guess, y, net.correction_k2, net.out_scale)


def initial_state(probs, est, rho0=1.0, zero_momentum=True):
    """(rho, u, phi) for lb_init_equilibrium_device: the state whose own
    half-forced moments are the estimate (j = rho u - F/2, phi - S/2), with the
    total half-forced momentum of a start from rest (zero) when zero_momentum."""
    out = Fields(est.L, est.B)
    C.lb_warm_initial_state(_ptr(est.rho), _ptr(est.u), _ptr(est.phi), _ptr(probs.F), _ptr(probs.S), est.B,
                            est.L * est.L, rho0, zero_momentum, _ptr(out.rho), _ptr(out.u), _ptr(out.phi), _stream())
    return out


RESET_CYCLES = 5   # step + moment-reset cycles tried by select() before iterating


def reset_target(probs, est, rho0=1.0, zero_momentum=True):
    """The moments of the stored (post-collision) state that belong to the
    estimate: its density, the momentum rho u + F/2 of the written state (u the
    half-forced velocity; momentum change F over the step, half of it before
    the collision) and the scalar phi + S/2, as (rho, velocity, phi) for
    lb_reset_moments_device.  initial_state with the force and source negated
    computes exactly this (same momentum correction)."""
    F = _empty(probs.F.numel())
    S = _empty(probs.S.numel())
    C.lb_warm_axpby(F.numel(), -1.0, _ptr(probs.F), 0.0, _ptr(probs.F), _ptr(F), _stream())
    C.lb_warm_axpby(S.numel(), -1.0, _ptr(probs.S), 0.0, _ptr(probs.S), _ptr(S), _stream())
    return initial_state(Problems(probs.L, probs.nu, probs.D, F, S, probs.seeds), est, rho0, zero_momentum)


def _context(probs, storage, K):
    """One stacked context for the B problems of `probs` on the current torch
    stream, force and source handed over in device memory."""
    s = Solver("D2Q9_D2Q5", (probs.L, probs.L, probs.B), storage=storage, nu=probs.nu, D_phi=probs.D,
               residual_interval=K, stream=_stream())
    C.lb_set_force_field(s.ctx, _ptr(probs.F), C.LB_DTYPE_F64, C.LB_MEM_DEVICE)
    C.lb_set_source_field(s.ctx, _ptr(probs.S), C.LB_DTYPE_F64, C.LB_MEM_DEVICE)
    return s


def read_fields(s, probs):
    """Half-forced (rho, u, phi) of the context's current state, on the device."""
    f = Fields(probs.L, probs.B)
    C.lb_read_moments_device(s.ctx, C.LB_MOMENTS_HALF_FORCED, _ptr(f.rho), _ptr(f.u), _ptr(f.phi))
    return f


def run_to_steady(s, tol, max_steps, K):
    """Steps s (K at a time) until the velocity and scalar residuals are both
    below tol; returns (steps, r_u, r_phi)."""
    steps, r, rp = 0, math.inf, math.inf
    while steps < max_steps:
        s.step(K)
        steps += K
        r = s.residual()[0]
        rp = s.residual_scalar()
        if r < tol and rp < tol:
            break
    return steps, r, rp


def solve(probs, init=None, tol=1e-8, max_steps=400000, K=100, storage="f32", fields=False, reset=None, cycles=0):
    """Steps the problems (one stacked context) from rest, or from the state of
    `init` (Fields of rho, u, phi from initial_state), until both residuals are
    below tol.  With `reset` (Fields from reset_target), the first `cycles`
    steps are each followed by a reset of the stored moments to it
    (lb_reset_moments_device): the populations' non-equilibrium part adapts to
    the estimate's gradients while its moments stay.  Returns (steps including
    the cycles, seconds of stepping, r_u, r_phi, Fields of the final
    half-forced moments or None)."""
    with _context(probs, storage, K) as s:
        if init is None:
            s.init_equilibrium()
        else:
            C.lb_init_equilibrium_device(s.ctx, _ptr(init.rho), _ptr(init.u), _ptr(init.phi))
        s.synchronize()
        t0 = time.perf_counter()
        done = 0
        if reset is not None:
            for _ in range(cycles):
                s.step(1)
                C.lb_reset_moments_device(s.ctx, _ptr(reset.rho), _ptr(reset.u), _ptr(reset.phi))
                done += 1
        steps, r, rp = run_to_steady(s, tol, max_steps, K)
        seconds = time.perf_counter() - t0
        out = read_fields(s, probs) if fields else None
        s.synchronize()
        return steps + done, seconds, r, rp, out


def _slice_copy(src, dst, b):
    """Copies problem b of Fields src into problem b of Fields dst (same L, B)."""
    n = src.L * src.L
    for (a, p), (c, _) in zip(src.planes(), dst.planes()):
        per = p // src.B   # planes per problem (1, or 2 for u)
        for k in range(per):
            off = (k * src.B + b) * n
            C.lb_warm_axpby(n, 1.0, _ptr(a) + 8 * off, 0.0, _ptr(a) + 8 * off, _ptr(c) + 8 * off, _stream())


def solve_stack(probs, init=None, tol=1e-8, max_steps=400000, K=100, storage="f32", reset=None, cycles=0):
    """solve() for B independent problems stacked in one context, with each
    problem's own stopping rule: every K steps the residuals of each slice
    (velocity and scalar, as the library defines them, from the half-forced
    moments K steps apart) are checked, and a slice's fields are kept as they
    are at its first check below tol, exactly what a solve of that problem
    alone would return.  The stack runs until every slice has stopped or
    max_steps.  Returns (steps per slice including the cycles, -1 if it never
    converged; Fields of the kept states)."""
    import torch

    B, n = probs.B, probs.L * probs.L
    kept = Fields(probs.L, probs.B)
    done = np.full(B, -1, dtype=np.int64)
    with _context(probs, storage, 0) as s:
        if init is None:
            s.init_equilibrium()
        else:
            C.lb_init_equilibrium_device(s.ctx, _ptr(init.rho), _ptr(init.u), _ptr(init.phi))
        if reset is not None:
            for _ in range(cycles):
                s.step(1)
                C.lb_reset_moments_device(s.ctx, _ptr(reset.rho), _ptr(reset.u), _ptr(reset.phi))
        steps, prev = 0, None
        while steps < max_steps and (done < 0).any():
            s.step(K)
            steps += K
            f = read_fields(s, probs)
            if prev is not None:
                uu, up = f.u.view(2, B, n), prev.u.view(2, B, n)
                pp, pq = f.phi.view(B, n), prev.phi.view(B, n)
                ru = (uu - up).norm(dim=(0, 2)) / (K * uu.norm(dim=(0, 2)))
                rq = (pp - pq).norm(dim=1) / (K * pp.norm(dim=1))
                ok = ((ru < tol) & (rq < tol)).cpu().numpy()
                for b in np.nonzero(ok & (done < 0))[0]:
                    _slice_copy(f, kept, int(b))
                    done[b] = steps + (cycles if reset is not None else 0)
            prev = f
        s.synchronize()
    return done, kept


def coarse_solutions_stack(probs, tol=1e-8, K=100, w_coarse=RICHARDSON):
    """coarse_solutions (cascade, three levels) for the B problems of probs at
    once, each level one stacked solve_stack with per-problem stopping.
    Returns ((steps, Fields) of the L/2, L/4, L/8 levels)."""
    p1 = probs.coarser()
    p2 = p1.coarser()
    p3 = p2.coarser()
    n3, f3 = solve_stack(p3, tol=tol, K=K)
    n2, f2 = solve_stack(p2, initial_state(p2, guess_from_half(f3)), tol=tol, K=K)
    n1, f1 = solve_stack(p1, initial_state(p1, guess_from_levels(f2, f3, w_coarse)), tol=tol, K=K)
    return (n1, f1), (n2, f2), (n3, f3)


def slice_residuals(s, probs, K):
    """Per-slice residuals of a stacked context from two readouts K steps apart
    (bookkeeping of the training data; host norms)."""
    a = read_fields(s, probs).host()
    s.step(K)
    f = read_fields(s, probs)
    b = f.host()
    n = probs.L * probs.L
    out = []
    for z in range(probs.B):
        sl = slice(z * n, (z + 1) * n)
        ru = np.linalg.norm(b[1][:, sl] - a[1][:, sl]) / (K * np.linalg.norm(b[1][:, sl]))
        rq = np.linalg.norm(b[2][sl] - a[2][sl]) / (K * np.linalg.norm(b[2][sl]))
        out.append((float(ru), float(rq)))
    return f, out


def layer_shapes(levels, channels, cin, cout):
    """(Co, Ci) of the network's convolutions in parameter order (the
    architecture of include/casclb_unet.h)."""
    c = list(channels)[:levels]
    shapes = []
    for l in range(levels):
        shapes += [(c[l], cin if l == 0 else c[l - 1]), (c[l], c[l])]
    for l in range(levels - 2, -1, -1):
        shapes.append((c[l], c[l] + c[l + 1]))
    shapes.append((cout, c[0]))
    return shapes


class Surrogate:
    """The network on the GPU plus the device copies of its inputs."""

    def __init__(self, L=256, max_batch=16, levels=6, channels=(16, 32, 32, 48, 48, 48), stream=None,
                 features="guess"):
        import torch

        self.torch = torch
        self.L = L
        self.max_batch = max_batch
        cin = LEVEL_IN_CH if features == "levels" else IN_CH
        cfg = C.lb_unet_config_default(levels=levels, channels=channels, in_channels=cin, out_channels=OUT_CH,
                                       height=L, width=L, max_batch=max_batch,
                                       stream=stream if stream is not None else torch.cuda.current_stream().cuda_stream)
        self.cfg = dict(levels=levels, channels=list(channels), in_channels=cin, out_channels=OUT_CH, L=L)
        # "guess": F, S, rates and the multilevel guess (u, phi, rho) at fixed scales; "levels": F, S,
        # rates and the differences between the coarse levels, each divided by its r.m.s. (in_scale)
        self.features = features
        self.in_scale = [1.0] * 8
        self.out_scale = list(_OUT_SCALE)
        self.h = C.lb_unet_create(cfg)
        self.num_params = C.lb_unet_num_params(self.h)
        # the guess the network corrects: extrapolation weights of the two coarse levels
        self.extrapolation = RICHARDSON
        self.extrapolation_b = (0.0, 0.0, 0.0)   # the fine guess's share of the L/4 - L/8 difference
        self.extrapolation_coarse = RICHARDSON   # the L/4 and L/8 levels' weights for the L/2 start
        self.correction_k2 = CORRECTION_K2
        # whether the estimate adds the network's correction to the guess, and the step + moment-reset
        # cycles the iteration starts with (both chosen on validation problems)
        self.use_network = True
        self.reset_cycles = 0
        # residual the coarse levels are solved to (0: the fine solve's tolerance); the guess's
        # own error (~1e-4 in the largest scales) is far above a coarse level's at 1e-8
        self.coarse_tol = 0.0
        self.head = "full"       # what the network's output corrects (HEADS)
        self.meta = {}

    def close(self):
        if self.h:
            C.lb_unet_destroy(self.h)
            self.h = None

    def init_params(self, seed=0):
        """He-normal weights (std sqrt(2 / (9 Ci))), zero biases."""
        g = np.random.default_rng(seed)
        parts = []
        for co, ci in layer_shapes(self.cfg["levels"], self.cfg["channels"], self.cfg["in_channels"], OUT_CH):
            parts.append(g.standard_normal(co * 9 * ci) * math.sqrt(2.0 / (9 * ci)))
            parts.append(np.zeros(co))
        p = np.concatenate(parts)
        assert p.size == self.num_params
        self.set_params(p)

    def set_params(self, p):
        C.lb_unet_set_params(self.h, np.asarray(p, dtype=np.float32))

    def get_params(self):
        return C.lb_unet_get_params(self.h)

    def forward(self, x):
        """Network output for device inputs x [B][L][L][IN_CH] (float32 torch
        tensor) -> device tensor [B][L][L][OUT_CH], max_batch images per launch."""
        torch = self.torch
        x = x.contiguous()
        y = torch.empty(x.shape[:3] + (OUT_CH,), dtype=torch.float32, device="cuda")
        for i in range(0, x.shape[0], self.max_batch):
            b = min(self.max_batch, x.shape[0] - i)
            C.lb_unet_forward(self.h, x[i].data_ptr(), b, y[i].data_ptr())
        return y

    def train(self, X, Y, epochs, lr=2e-3, lr_end=1e-4, batch=None, seed=0, log_every=1):
        """Adam on the mean squared error over the normalised targets; X [N][L][L][IN_CH],
        Y [N][L][L][OUT_CH] (float32 device tensors); cosine learning-rate decay from
        lr to lr_end.  Returns the per-epoch mean losses."""
        torch = self.torch
        batch = batch or self.max_batch
        Xd, Yd = X.contiguous(), Y.contiguous()
        n = X.shape[0]
        g = np.random.default_rng(seed)
        steps_total = epochs * (n // batch)
        step = 0
        history = []
        for ep in range(epochs):
            order = g.permutation(n)
            losses = []
            for i in range(0, n - batch + 1, batch):
                idx = torch.from_numpy(order[i:i + batch]).cuda()
                xb = Xd.index_select(0, idx).contiguous()
                yb = Yd.index_select(0, idx).contiguous()
                a = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * step / max(1, steps_total)))
                losses.append(C.lb_unet_train_step(self.h, xb.data_ptr(), yb.data_ptr(), batch, a))
                step += 1
            history.append(float(np.mean(losses)))
            if log_every and (ep % log_every == 0 or ep == epochs - 1):
                _say(f"[warmstart] epoch {ep + 1}/{epochs}: loss {history[-1]:.4e}")
        return history

    def save(self, path, meta=None):
        np.savez(path, params=self.get_params(), config=json.dumps(self.cfg),
                 scales=np.array([U0, PHI0, K0, RATE_MID, RATE_HALF, RES, RHO0]), meta=json.dumps(meta or {}),
                 extrapolation=np.array(self.extrapolation), correction_k2=np.array(self.correction_k2),
                 use_network=np.array(self.use_network), reset_cycles=np.array(self.reset_cycles),
                 coarse_tol=np.array(self.coarse_tol),
                 extrapolation_coarse=np.array(self.extrapolation_coarse),
                 extrapolation_b=np.array(self.extrapolation_b), head=np.array(self.head),
                 features=np.array(self.features), in_scale=np.array(self.in_scale),
                 out_scale=np.array(self.out_scale))

    @classmethod
    def load(cls, path, max_batch=16):
        z = np.load(path, allow_pickle=False)
        cfg = json.loads(str(z["config"]))
        kind = str(z["features"]) if "features" in z.files else "guess"
        net = cls(L=cfg["L"], max_batch=max_batch, levels=cfg["levels"], channels=cfg["channels"], features=kind)
        net.set_params(z["params"])
        net.meta = json.loads(str(z["meta"]))
        if "extrapolation" in z.files:
            net.extrapolation = tuple(float(v) for v in z["extrapolation"])
        if "correction_k2" in z.files:
            net.correction_k2 = int(z["correction_k2"])
        if "use_network" in z.files:
            net.use_network = bool(z["use_network"])
        if "reset_cycles" in z.files:
            net.reset_cycles = int(z["reset_cycles"])
        if "coarse_tol" in z.files:
            net.coarse_tol = float(z["coarse_tol"])
        if "extrapolation_coarse" in z.files:
            net.extrapolation_coarse = tuple(float(v) for v in z["extrapolation_coarse"])
        if "extrapolation_b" in z.files:
            net.extrapolation_b = tuple(float(v) for v in z["extrapolation_b"])
        if "head" in z.files:
            net.head = str(z["head"])
        if "in_scale" in z.files:
            net.in_scale = [float(v) for v in z["in_scale"]]
        if "out_scale" in z.files:
            net.out_scale = [float(v) for v in z["out_scale"]]
        return net


def generate(groups, slices, L=256, first_seed=1, tol=1e-9, slice_tol=1e-8, coarse_tol=1e-8, K=100,
             extrapolation="fit"):
    """Network inputs and targets (device float32 tensors [M][L][L][9], [M][L][L][4])
    of `groups` x `slices` steady problems, the number of dropped slices and the
    weights {"fine": a, "fine_b": b, "coarse": w2}: a and b those of the
    three-level guess the targets correct (fitted to these solutions with
    ExtrapolationFit when extrapolation is "fit", else a = the weights given and
    b = 0), w2 those of the L/2 level's start (the L/4 and L/8 solutions fitted
    to the L/2 ones, two levels).  Without an L/8 level (L not a multiple of 32)
    the fine guess has two levels and b is 0.  Slices whose own residual misses
    slice_tol are dropped.  The coarse levels of each problem are solved on
    their own to coarse_tol, as the estimate solves them at inference."""
    import torch

    from casclb_inputs import warmstart_group
    solved = []
    three = L % 32 == 0
    fit = ExtrapolationFit(levels=3 if three else 2)
    fit_coarse = ExtrapolationFit()
    dropped = 0
    t0 = time.perf_counter()
    for gi in range(groups):
        cases = warmstart_group(first_seed + gi, slices, L=L)
        probs = Problems.from_cases(cases)
        with _context(probs, "f32", K) as s:
            s.init_equilibrium()
            steps, _, _ = run_to_steady(s, tol, 200000, K)
            truth, res = slice_residuals(s, probs, K)
        # each slice's coarse levels solved on their own, as at inference (a stacked
        # solve stops on the stack's residual and leaves some slices less converged)
        parts = [coarse_solutions(Problems.from_cases([c]), coarse_tol, K, level3=True) for c in cases]
        f1 = Fields.stack([p[0][4] for p in parts])
        f2 = Fields.stack([p[1][4] for p in parts])
        f3 = Fields.stack([p[2][4] for p in parts]) if parts[0][2] is not None else None
        keep = [i for i, (ru, rq) in enumerate(res) if ru < slice_tol and rq < slice_tol]
        dropped += probs.B - len(keep)
        if keep:
            fit.add(truth, f1, f2, keep, f3=f3)
            if f3 is not None:
                fit_coarse.add(_copy(f1), f2, f3, keep)
            solved.append((probs, truth, f1, f2, f3, keep))
        _say(f"[warmstart] group {gi + 1}/{groups} (nu {probs.nu:.3f}, D {probs.D:.3f}): {steps} steps, "
             f"worst slice residuals {max(r[0] for r in res):.1e} / {max(r[1] for r in res):.1e}, "
             f"{time.perf_counter() - t0:.0f} s")
    if isinstance(extrapolation, str):
        w, wb = fit.weights() if three else (fit.weights(), (0.0, 0.0, 0.0))
    else:
        w, wb = _weights(extrapolation), (0.0, 0.0, 0.0)
    _say(f"[warmstart] extrapolation weights a (density, velocity, scalar) {w[0]:.4f} {w[1]:.4f} {w[2]:.4f}, "
         f"b {wb[0]:.4f} {wb[1]:.4f} {wb[2]:.4f}")
    w2 = fit_coarse.weights() if fit_coarse.count else RICHARDSON
    _say(f"[warmstart] L/2 start weights (density, velocity, scalar) {w2[0]:.4f} {w2[1]:.4f} {w2[2]:.4f}")
    X, Y = [], []
    for probs, truth, f1, f2, f3, keep in solved:
        g = guess_from_levels(f1, f2, w, f3, wb)
        x = features(probs, g, torch.empty(probs.B, L, L, IN_CH, dtype=torch.float32, device="cuda"))
        y = targets(truth, g, torch.empty(probs.B, L, L, OUT_CH, dtype=torch.float32, device="cuda"))
        idx = torch.tensor(keep, dtype=torch.long, device="cuda")
        X.append(x.index_select(0, idx))
        Y.append(y.index_select(0, idx))
    return torch.cat(X), torch.cat(Y), dropped, dict(fine=w, fine_b=wb, coarse=w2)


def generate_stacked(groups, slices, net, L=256, first_seed=1, truth_tol=1e-9, K=100, log_every=16,
                     max_truth_steps=80000, features_kind="guess"):
    """Training data at scale: `groups` x `slices` problems (one (nu, D) pair
    per group), all levels of a group solved as stacked contexts with each
    problem's own stopping rule (solve_stack): the coarse cascade to 1e-8 with
    the weights of `net`, exactly as the estimate solves one problem, then the
    fine truth from that guess (with the reset cycles) to truth_tol.  Returns
    the network inputs X [M][L][L][9], the targets of both heads (full: truth -
    guess; low: its modes 0 < |k|^2 <= 8) [M][L][L][4] (float32 device
    tensors) and bookkeeping (steps per level, dropped problems, seconds)."""
    import torch

    from casclb_inputs import warmstart_group
    X, YF, YL = [], [], []
    steps = {"L/8": [], "L/4": [], "L/2": [], "fine": []}
    dropped = 0
    t0 = time.perf_counter()
    for gi in range(groups):
        probs = Problems.from_cases(warmstart_group(first_seed + gi, slices, L=L))
        (n1, f1), (n2, f2), (n3, f3) = coarse_solutions_stack(probs, 1e-8, K, net.extrapolation_coarse)
        g = guess_from_levels(f1, f2, net.extrapolation, f3, net.extrapolation_b)
        nt, truth = solve_stack(probs, initial_state(probs, g), tol=truth_tol, K=K, reset=reset_target(probs, g),
                                cycles=RESET_CYCLES, max_steps=max_truth_steps)
        keep = [b for b in range(probs.B) if min(n1[b], n2[b], n3[b], nt[b]) > 0]
        dropped += probs.B - len(keep)
        if keep:
            idx = torch.tensor(keep, dtype=torch.long, device="cuda")
            shape = (probs.B, L, L)
            if features_kind == "levels":
                d1, d2 = level_differences(f1, f2, f3)
                X.append(features_levels(probs, d1, d2, [1.0] * 8,
                                         torch.empty(*shape, LEVEL_IN_CH, dtype=torch.float32, device="cuda"))
                         .index_select(0, idx))
            else:
                X.append(features(probs, g, torch.empty(*shape, IN_CH, dtype=torch.float32, device="cuda"))
                         .index_select(0, idx))
            YL.append(targets_low(_copy(truth), g, torch.empty(*shape, OUT_CH, dtype=torch.float32, device="cuda"))
                      .index_select(0, idx))
            unit = [1.0] * 4 if features_kind == "levels" else None
            YF.append(targets(truth, g, torch.empty(*shape, OUT_CH, dtype=torch.float32, device="cuda"), unit)
                      .index_select(0, idx))
            for k, v in zip(("L/2", "L/4", "L/8", "fine"), (n1, n2, n3, nt)):
                steps[k] += [int(v[b]) for b in keep]
        if log_every and ((gi + 1) % log_every == 0 or gi + 1 == groups):
            _say(f"[warmstart] data: group {gi + 1}/{groups}, {sum(len(x) for x in X)} solutions, "
                 f"{dropped} dropped, {time.perf_counter() - t0:.0f} s")
    info = dict(samples=int(sum(x.shape[0] for x in X)), dropped=dropped, truth_tol=truth_tol,
                mean_steps={k: float(np.mean(v)) for k, v in steps.items()}, seconds=time.perf_counter() - t0,
                features=features_kind)
    X, YF, YL = torch.cat(X), torch.cat(YF), torch.cat(YL)
    if features_kind == "levels":
        # every level-difference input and every target channel divided by its r.m.s. over these solutions
        info["in_scale"] = [float(X[..., 5 + c].double().square().mean().sqrt()) for c in range(8)]
        info["out_scale"] = [float(YF[..., c].double().square().mean().sqrt()) for c in range(4)]
        for c in range(8):
            X[..., 5 + c] /= info["in_scale"][c]
        for c in range(4):
            YF[..., c] /= info["out_scale"][c]
    return X, YF, YL, info


def _low_error(a, b, k2max=EXTRAPOLATION_K2):
    """Relative l2 norm of the modes 0 < |k|^2 <= k2max of a - b against those of b
    (velocity and scalar), host norms."""
    d = low_modes(_combine(1.0, a, -1.0, b), k2max).host()
    r = low_modes(_copy(b), k2max).host()
    return [float(np.linalg.norm(d[1]) / np.linalg.norm(r[1])), float(np.linalg.norm(d[2]) / np.linalg.norm(r[2]))]


def compare_networks(nets, cases, tol=1e-8, K=100, base=None):
    """Per test case: the multilevel guess of `base` (the weights' coarse and
    extrapolation settings), the fine steps to tol from it with the reset
    cycles, from the same guess with each network's correction, and from the
    guess with its largest scales (0 < |k|^2 <= 8) replaced by those of the
    converged state (what a perfect low-mode correction would reach); the
    inference seconds of each network and the low-mode error of each estimate
    relative to the guess's.  Returns a list of dicts."""
    import torch

    base = base or nets[0]
    rows = []
    for c in cases:
        probs = Problems.from_cases([c])
        t0 = time.perf_counter()
        s1, s2, s3 = coarse_solutions(probs, tol, K, True, base.extrapolation_coarse, level3=True)
        g = guess_from_levels(s1[4], s2[4], base.extrapolation, s3[4], base.extrapolation_b)
        torch.cuda.synchronize()
        t_guess = time.perf_counter() - t0
        cold = solve(probs, None, tol=1e-10, K=K, storage="f64", fields=True, max_steps=800000)
        truth = cold[4].project()

        def run(e):
            return solve(probs, initial_state(probs, e), tol=tol, K=K, reset=reset_target(probs, e),
                         cycles=RESET_CYCLES)

        r_guess = run(g)
        low = low_modes(_combine(1.0, truth, -1.0, g))
        r_perfect = run(_combine(1.0, g, 1.0, low))
        r_all = run(_copy(truth))
        rest = _combine(1.0, _combine(1.0, truth, -1.0, g), -1.0, low)     # the error outside the largest scales
        r_rest = run(_combine(1.0, g, 1.0, rest))
        row = dict(seed=c.seed, guess_steps=r_guess[0], guess_s=r_guess[1], estimate_guess_s=t_guess,
                   perfect_low_steps=r_perfect[0], perfect_other_steps=r_rest[0], perfect_all_steps=r_all[0],
                   guess_low_error=_low_error(g, truth), networks=[])
        for net in nets:
            apply_network(net, probs, g, (s1[4], s2[4], s3[4]))           # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            est = apply_network(net, probs, g, (s1[4], s2[4], s3[4]))
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t1
            r = run(est)
            row["networks"].append(dict(steps=r[0], s=r[1], inference_s=t_inf, low_error=_low_error(est, truth)))
        rows.append(row)
        _say(f"[warmstart] test case {c.seed}: guess {r_guess[0]} steps, perfect largest scales {r_perfect[0]}, "
             f"perfect other scales {r_rest[0]}, exact state {r_all[0]}, "
             f"networks {[n['steps'] for n in row['networks']]}, low-mode error guess "
             f"{row['guess_low_error'][0]:.2e} networks {[round(n['low_error'][0], 4) for n in row['networks']]}")
    return rows


def compare_on_off(nets, cases, tol=1e-8, K=100, shipped=None):
    """Per case, one set of coarse solves shared by every variant: the fine
    steps to tol (and seconds of stepping) from rest, from the L/2 solve alone,
    from the Richardson combination, from the fitted multilevel guess without
    and with RESET_CYCLES reset cycles (the network off), and from the guess
    plus each network's correction with its reset cycles (the network on), with
    each network's inference seconds; with `shipped` (one of nets), also the
    wall-clock seconds of warm_solve with that weights file from the problem's
    definition to the converged state (coarse solves, inference, contexts and
    stepping) and of the cold solve likewise.  The coarse settings are those of
    nets[0].  Returns a list of dicts."""
    import torch

    base = nets[0]
    rows = []
    for c in cases:
        probs = Problems.from_cases([c])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s1, s2, s3 = coarse_solutions(probs, tol, K, True, base.extrapolation_coarse, level3=True)
        g = guess_from_levels(s1[4], s2[4], base.extrapolation, s3[4], base.extrapolation_b)
        torch.cuda.synchronize()
        t_guess = time.perf_counter() - t0
        cold = solve(probs, None, tol=tol, K=K)
        half = solve(probs, initial_state(probs, guess_from_half(s1[4])), tol=tol, K=K)
        rich = solve(probs, initial_state(probs, guess_from_levels(s1[4], s2[4], RICHARDSON)), tol=tol, K=K)
        plain = solve(probs, initial_state(probs, g), tol=tol, K=K)
        off = solve(probs, initial_state(probs, g), tol=tol, K=K, reset=reset_target(probs, g), cycles=RESET_CYCLES)
        row = dict(seed=c.seed, cold_steps=cold[0], cold_s=cold[1], coarse_steps=[s1[0], s2[0], s3[0]],
                   guess_estimate_s=t_guess, half_only_steps=half[0], richardson_steps=rich[0],
                   guess_steps=plain[0], off_steps=off[0], off_s=off[1], networks=[])
        levels = (s1[4], s2[4], s3[4])
        for net in nets:
            apply_network(net, probs, g, levels)           # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            est = apply_network(net, probs, g, levels)
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t1
            on = solve(probs, initial_state(probs, est), tol=tol, K=K, reset=reset_target(probs, est),
                       cycles=RESET_CYCLES)
            row["networks"].append(dict(steps=on[0], s=on[1], inference_s=t_inf))
        if shipped is not None:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            r = warm_solve(shipped, probs, tol, K)[0]
            torch.cuda.synchronize()
            row["shipped_end_to_end_s"] = time.perf_counter() - t2
            row["shipped_steps"] = r[0]
            t3 = time.perf_counter()
            solve(probs, None, tol=tol, K=K)
            torch.cuda.synchronize()
            row["cold_end_to_end_s"] = time.perf_counter() - t3
        rows.append(row)
        _say(f"[warmstart] case {c.seed}: cold {cold[0]}; L/2 guess {half[0]}; Richardson {rich[0]}; fitted guess "
             f"{plain[0]}, with cycles {off[0]}; networks with cycles {[n['steps'] for n in row['networks']]}")
    return rows


def scale_experiment(sizes, heads, epochs, base_weights, out_dir, slices=16, L=256, lr=5e-4, truth_tol=1e-9,
                     test_cases=8, features_kind="guess"):
    """Trains one network per (head, training-set size) on the first `size`
    solutions of one generated set, chooses network on/off on the validation
    problems (select) and compares all on the test problems; writes
    results.json and the weights of every network into out_dir."""
    import os

    import torch

    from casclb_inputs import warmstart_case
    os.makedirs(out_dir, exist_ok=True)
    base = Surrogate.load(base_weights)
    groups = -(-max(sizes) // slices)
    # group seeds from 1000 on: slice seeds 1000 g + i stay clear of the test (100000+) and
    # validation (200000+) problems
    X, YF, YL, info = generate_stacked(groups, slices, base, L=L, first_seed=1000, truth_tol=truth_tol,
                                       features_kind=features_kind)
    _say(f"[warmstart] {info}")
    results = dict(data=info, sizes=list(sizes), heads=list(heads), runs=[])
    nets = []
    for head in heads:
        Y = YL if head == "low" else YF
        for size, ep in zip(sizes, epochs):
            m = min(size, X.shape[0])
            net = Surrogate(L=L, features=features_kind)
            net.init_params(seed=0)
            for k in ("extrapolation", "extrapolation_b", "extrapolation_coarse", "correction_k2"):
                setattr(net, k, getattr(base, k))
            net.head = head
            if features_kind == "levels":
                net.in_scale, net.out_scale = info["in_scale"], info["out_scale"]
            t0 = time.perf_counter()
            hist = net.train(X[:m], Y[:m], ep, lr=lr, log_every=max(1, ep // 4))
            train_s = time.perf_counter() - t0
            val = select(net, [warmstart_case(s, L=L) for s in VALIDATION_SEEDS])
            meta = dict(samples=m, head=head, features=features_kind, epochs=ep, lr=lr, final_loss=hist[-1], losses=hist,
                        train_seconds=train_s,
                        validation_steps=val, use_network=net.use_network, reset_cycles=net.reset_cycles,
                        truth_tol=truth_tol)
            net.meta = meta
            path = os.path.join(out_dir, f"unet_{head}_{m}.npz")
            net.save(path, meta)
            results["runs"].append(dict(meta, weights=os.path.basename(path)))
            nets.append(net)
            _say(f"[warmstart] head {head}, {m} solutions: loss {hist[-1]:.3e}, network used: {net.use_network}")
    del X, YF, YL
    torch.cuda.empty_cache()
    results["test"] = compare_networks(nets, [warmstart_case(100000 + i, L=L) for i in range(test_cases)], base=base)
    with open(os.path.join(out_dir, "results.json"), "w") as f:
        json.dump(results, f)
    for n in nets:
        n.close()
    base.close()
    return results


def coarse_solutions(probs, tol=1e-8, K=100, cascade=True, w_coarse=RICHARDSON, level3=False):
    """Steady solutions of the L/2 and L/4 problems: solve() results (steps,
    seconds, r_u, r_phi, Fields) for each (and, with level3, of the L/8 problem
    as a third).  With cascade, each level starts from the coarser ones: the
    L/8 problem (when L is a multiple of 32) from rest, the L/4 one from the
    L/8 solution (guess_from_half), the L/2 one from the extrapolation of the
    L/4 and L/8 solutions with weights w_coarse (guess_from_levels); without
    an L/8 level the L/4 problem starts from rest and the L/2 one from the L/4
    solution.  Without cascade both start from rest.  Every start ends within
    the tolerance of the same steady state as long as each level resolves the
    forcing (its wave numbers below the Nyquist of the coarsest lattice: the
    iteration does not damp Nyquist modes); on these lattices a step costs
    about the same at every size (one wave's latency), so coarse steps saved
    are time saved."""
    p1 = probs.coarser()
    p2 = p1.coarser()
    s3 = None
    if cascade and probs.L % 32 == 0:
        p3 = p2.coarser()
        s3 = solve(p3, tol=tol, K=K, fields=True)
        s2 = solve(p2, initial_state(p2, guess_from_half(s3[4])), tol=tol, K=K, fields=True)
        init = initial_state(p1, guess_from_levels(s2[4], s3[4], w_coarse))
    else:
        s2 = solve(p2, tol=tol, K=K, fields=True)
        init = initial_state(p1, guess_from_half(s2[4])) if cascade else None
    s1 = solve(p1, init, tol=tol, K=K, fields=True)
    return (s1, s2, s3) if level3 else (s1, s2)


def coarse_tolerance(net, tol, coarse_tol=None):
    """The residual the coarse levels are solved to: coarse_tol if given, else
    the weights' setting, else the fine tolerance."""
    if coarse_tol is not None:
        return coarse_tol
    return net.coarse_tol if net.coarse_tol > 0 else tol


def warm_estimate(net, probs, tol=1e-8, K=100, parts=False, network=None, cascade=True, coarse_tol=None):
    """(estimate, multilevel guess, (L/2, L/4, L/8 steps; 0 without an L/8
    level), seconds of the coarse solves, resampling and inference) for the
    problems `probs`: the coarse levels are solved to coarse_tolerance(), the
    guess extrapolates them with net.extrapolation and net.extrapolation_b, the
    network adds its correction if `network` (default net.use_network), else
    the estimate is the guess.  With parts, also the guess from the L/2 solve
    alone and the two-level Richardson guess.  Estimates are Fields (rho - rho0,
    u, phi)."""
    import torch

    t0 = time.perf_counter()
    ct = coarse_tolerance(net, tol, coarse_tol)
    s1, s2, s3 = coarse_solutions(probs, ct, K, cascade, net.extrapolation_coarse, level3=True)
    g = guess_from_levels(s1[4], s2[4], net.extrapolation, s3[4] if s3 is not None else None, net.extrapolation_b)
    if net.use_network if network is None else network:
        est = apply_network(net, probs, g, (s1[4], s2[4], s3[4] if s3 is not None else None))
    else:
        est = g
    torch.cuda.synchronize()
    out = (est, g, (s1[0], s2[0], s3[0] if s3 is not None else 0), time.perf_counter() - t0)
    if parts:
        out = out + (guess_from_half(s1[4]), guess_from_levels(s1[4], s2[4], RICHARDSON))
    return out


def warm_solve(net, probs, tol=1e-8, K=100, fields=False, coarse_tol=None):
    """The warm start as the weights file configures it: warm_estimate, the
    initial state, net.reset_cycles cycles of one step and a moment reset to
    the estimate, then the iteration to tol.  Returns (solve() result, seconds
    of the estimate, coarse steps)."""
    est, _, csteps, t_est = warm_estimate(net, probs, tol, K, coarse_tol=coarse_tol)
    target = reset_target(probs, est) if net.reset_cycles else None
    return (solve(probs, initial_state(probs, est), tol=tol, K=K, fields=fields, reset=target,
                  cycles=net.reset_cycles), t_est, csteps)


def evaluate(net, cases, tol=1e-8, K=100):
    """Steps to tol from a cold start, from the L/2 guess alone, from the
    Richardson guess, from the guess with the network's extrapolation weights
    and from that guess plus the learned correction; returns a list of dicts
    (errors against the cold end state, relative L2 of the half-forced u, phi and
    the density deviation; seconds of the estimate with the network,
    estimate_s, and without, guess_estimate_s); reset_steps: from the estimate
    net.use_network selects, with RESET_CYCLES step + moment-reset cycles."""
    out = []
    for c in cases:
        probs = Problems.from_cases([c])
        est, g, csteps, t_est, g1, gr = warm_estimate(net, probs, tol, K, parts=True, network=True)
        t_guess_est = warm_estimate(net, probs, tol, K, network=False)[3]
        cold = solve(probs, None, tol=tol, K=K, fields=True)
        half_only = solve(probs, initial_state(probs, g1), tol=tol, K=K)
        rich_only = solve(probs, initial_state(probs, gr), tol=tol, K=K)
        guess_only = solve(probs, initial_state(probs, g), tol=tol, K=K)
        warm = solve(probs, initial_state(probs, est), tol=tol, K=K)
        chosen = est if net.use_network else g
        reset = solve(probs, initial_state(probs, chosen), tol=tol, K=K, reset=reset_target(probs, chosen),
                      cycles=RESET_CYCLES)
        rf, uf, pf = cold[4].host()
        rf = rf - rf.mean()

        def err(f):
            r, u, phi = f.host()
            return [float(np.linalg.norm(u - uf) / np.linalg.norm(uf)),
                    float(np.linalg.norm(phi - pf) / np.linalg.norm(pf)),
                    float(np.linalg.norm(r - rf) / np.linalg.norm(rf))]

        out.append(dict(seed=c.seed, nu=c.nu, D=c.D, cold_steps=cold[0], coarse_steps=list(csteps),
                        half_only_steps=half_only[0], richardson_steps=rich_only[0], coarse_only_steps=guess_only[0],
                        warm_steps=warm[0], reset_steps=reset[0], reset_s=reset[1], cold_s=cold[1],
                        estimate_s=t_est, guess_estimate_s=t_guess_est, coarse_only_s=guess_only[1],
                        warm_s=warm[1], half_guess_error=err(g1), richardson_error=err(gr), guess_error=err(g),
                        estimate_error=err(est)))
        e = out[-1]
        _say(f"[warmstart] case {c.seed}: cold {cold[0]} steps ({cold[1]:.2f} s); L/2 guess {half_only[0]}; "
             f"Richardson {rich_only[0]}; fitted extrapolation {guess_only[0]} (error u {e['guess_error'][0]:.1e}, "
             f"rho {e['guess_error'][2]:.1e}); + network {warm[0]} steps (error u {e['estimate_error'][0]:.1e}, "
             f"phi {e['estimate_error'][1]:.1e}, rho {e['estimate_error'][2]:.1e}); with {RESET_CYCLES} reset "
             f"cycles {reset[0]}; coarse steps {csteps}, "
             f"estimate {t_est:.3f} s")
    return out


VALIDATION_SEEDS = range(200000, 200008)   # problems for model selection, apart from training and test seeds


def select(net, cases, tol=1e-8, K=100):
    """Sets net.use_network and net.reset_cycles to the combination (network
    correction on or off, 0 or RESET_CYCLES step + moment-reset cycles) that
    steps `cases` to tol in the least total time, the network's inference
    (feature packing, forward pass, unpacking and projection) counted against
    the fine steps it saves.  Returns per case the steps of the four
    combinations [guess, guess + cycles, network, network + cycles] and the
    inference seconds."""
    import torch

    rows = []
    t = np.zeros(4)
    for c in cases:
        probs = Problems.from_cases([c])
        s1, s2, s3 = coarse_solutions(probs, tol, K, w_coarse=net.extrapolation_coarse, level3=True)
        g = guess_from_levels(s1[4], s2[4], net.extrapolation, s3[4] if s3 is not None else None,
                              net.extrapolation_b)
        for _ in range(1 if rows else 2):          # the first pass warms up, untimed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            est = apply_network(net, probs, g, (s1[4], s2[4], s3[4]))
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t0
        runs = []
        for e in (g, est):
            runs.append(solve(probs, initial_state(probs, e), tol=tol, K=K))
            runs.append(solve(probs, initial_state(probs, e), tol=tol, K=K, reset=reset_target(probs, e),
                              cycles=RESET_CYCLES))
        t += np.array([r[1] for r in runs]) + np.array([0.0, 0.0, t_inf, t_inf])
        rows.append([r[0] for r in runs] + [t_inf])
        _say(f"[warmstart] validation case {c.seed}: guess {runs[0][0]} steps, with {RESET_CYCLES} reset cycles "
             f"{runs[1][0]}; + network {runs[2][0]}, with cycles {runs[3][0]} ({t_inf:.4f} s inference)")
    best = int(np.argmin(t))
    net.use_network = best >= 2
    net.reset_cycles = RESET_CYCLES if best % 2 else 0
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--groups", type=int, default=64)
    tr.add_argument("--slices", type=int, default=16)
    tr.add_argument("--L", type=int, default=256)
    tr.add_argument("--epochs", type=int, default=60)
    tr.add_argument("--lr", type=float, default=5e-4)
    tr.add_argument("--lowpass-levels", type=int, default=0)
    tr.add_argument("--lowpass-weight", type=float, default=0.0)
    tr.add_argument("--out", required=True)
    tr.add_argument("--eval-cases", type=int, default=8)
    tr.add_argument("--richardson", action="store_true", help="Richardson's weights instead of fitted ones")
    tr.add_argument("--correction-k2", type=int, default=CORRECTION_K2)
    se = sub.add_parser("select", help="choose on validation problems whether the network's correction is used")
    se.add_argument("--weights", required=True)
    se.add_argument("--out", required=True)
    sc = sub.add_parser("scale", help="train at several training-set sizes and heads, compare on test problems")
    sc.add_argument("--weights", required=True, help="weights file whose guess settings the networks correct")
    sc.add_argument("--sizes", default="1024,5120,20480")
    sc.add_argument("--epochs", default="60,24,8")
    sc.add_argument("--heads", default="full")
    sc.add_argument("--slices", type=int, default=64)
    sc.add_argument("--truth-tol", type=float, default=1e-8)
    sc.add_argument("--test-cases", type=int, default=8)
    sc.add_argument("--out-dir", required=True)
    sc.add_argument("--features", default="guess", choices=("guess", "levels"))
    ev = sub.add_parser("evaluate")
    ev.add_argument("--weights", required=True)
    ev.add_argument("--cases", type=int, default=8)
    ev.add_argument("--L", type=int, default=256)
    args = ap.parse_args(argv)

    import torch

    torch.cuda.is_available()
    from casclb_inputs import warmstart_case
    if args.cmd == "train":
        X, Y, dropped, wts = generate(args.groups, args.slices, L=args.L,
                                      extrapolation=RICHARDSON if args.richardson else "fit")
        _say(f"[warmstart] {X.shape[0]} training solutions ({dropped} dropped)")
        net = Surrogate(L=args.L)
        net.init_params(seed=0)
        net.extrapolation = wts["fine"]
        net.extrapolation_b = wts["fine_b"]
        net.extrapolation_coarse = wts["coarse"]
        net.correction_k2 = args.correction_k2
        if args.lowpass_levels:
            C.lb_unet_set_lowpass_loss(net.h, args.lowpass_levels, args.lowpass_weight)
        t0 = time.perf_counter()
        hist = net.train(X, Y, args.epochs, lr=args.lr)
        train_s = time.perf_counter() - t0
        meta = dict(samples=int(X.shape[0]), dropped=int(dropped), groups=args.groups, slices=args.slices,
                    epochs=args.epochs, lr=args.lr, lowpass=[args.lowpass_levels, args.lowpass_weight],
                    final_loss=hist[-1], train_seconds=train_s, losses=hist, extrapolation=list(wts["fine"]),
                    extrapolation_b=list(wts["fine_b"]), extrapolation_coarse=list(wts["coarse"]),
                    correction_k2=args.correction_k2)
        meta["validation_steps"] = select(net, [warmstart_case(s, L=args.L) for s in VALIDATION_SEEDS])
        meta["use_network"] = net.use_network
        meta["reset_cycles"] = net.reset_cycles
        net.save(args.out, meta)
        cases = [warmstart_case(100000 + i, L=args.L) for i in range(args.eval_cases)]
        res = evaluate(net, cases)
        print(json.dumps(dict(meta=meta, eval=res)), flush=True)
        net.close()
    elif args.cmd == "scale":
        res = scale_experiment([int(v) for v in args.sizes.split(",")], args.heads.split(","),
                               [int(v) for v in args.epochs.split(",")], args.weights, args.out_dir,
                               slices=args.slices, truth_tol=args.truth_tol, test_cases=args.test_cases,
                               features_kind=args.features)
        print(json.dumps(dict(data=res["data"], runs=[{k: v for k, v in r.items() if k != "losses"}
                                                      for r in res["runs"]])), flush=True)
    elif args.cmd == "select":
        net = Surrogate.load(args.weights)
        meta = dict(net.meta)
        meta["validation_steps"] = select(net, [warmstart_case(s, L=net.L) for s in VALIDATION_SEEDS])
        meta["use_network"] = net.use_network
        meta["reset_cycles"] = net.reset_cycles
        net.save(args.out, meta)
        print(json.dumps(dict(use_network=net.use_network, reset_cycles=net.reset_cycles,
                              validation_steps=meta["validation_steps"])), flush=True)
        net.close()
    else:
        net = Surrogate.load(args.weights)
        cases = [warmstart_case(100000 + i, L=args.L) for i in range(args.cases)]
        print(json.dumps(evaluate(net, cases)), flush=True)
        net.close()


if __name__ == "__main__":
    main()
