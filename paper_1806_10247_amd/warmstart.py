"""Learned warm start for steady periodic flow + scalar problems.

The lattice is initialised with the product-form equilibrium of an estimate
of the steady density rho, half-forced velocity u and half-sourced scalar phi
(converted to the populations' own moments, j = rho u - F/2 and phi - S/2)
and then iterated with the cascaded scheme until both residuals (velocity and scalar,
every K steps) fall below the tolerance, exactly as from a cold start: the
estimate only moves the starting point, the converged answer is the solver's.

The estimate has two parts:
  1. a coarse solve: the same problem on the L/2 lattice under diffusive
     scaling (dx x2, dt x4: force x8, source x4, same nu and D), run to the
     tolerance (a quarter of the nodes, about a quarter of the steps), its
     u/2, phi and (rho - mean)/4 (the pressure scales as u^2) upsampled to
     L x L (periodic Catmull-Rom).  It fixes the large scales, whose slow
     decay dominates the iteration count;
  2. a U-Net (include/casclb_unet.h, bf16 matrix cores) that maps the force,
     source, rates and that upsampled guess to the remaining fine-lattice
     correction of all four fields.
The density matters as much as the velocity: started from the exact steady
u and phi at uniform density, the pressure mismatch launches sound waves
whose slow viscous decay costs about half the steps of a cold start.
The means of the estimate are removed (the density's is set to the rest
density): mass, momentum and scalar totals are conserved by the iteration
(zero-mean force and source), so this keeps the state the cold start
converges to.

Training data are steady solutions this solver produces: problems sharing
one (nu, D) pair run as the slices of one stacked 2D context (nz slices, one
launch per step), each slice's own residual checked at the end.

    python -m paper_1806_10247_amd.warmstart train --groups 48 --slices 16 --out weights.npz
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


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def features(case, guess):
    """Network input [L][L][9] (float32): F/(nu K0^2 U0) (2), S/(D K0^2 PHI0),
    the two rates as constant channels, and the coarse guess u/U0 (2), phi/PHI0,
    (rho - rho0)/RHO0.  guess = (rho - rho0 [N], u [2][N], phi [N])."""
    L = case.L
    rg, ug, pg = guess
    x = np.empty((L, L, IN_CH), dtype=np.float32)
    x[..., 0] = (case.F[0] / (case.nu * K0 * K0 * U0)).reshape(L, L)
    x[..., 1] = (case.F[1] / (case.nu * K0 * K0 * U0)).reshape(L, L)
    x[..., 2] = (case.S / (case.D * K0 * K0 * PHI0)).reshape(L, L)
    x[..., 3] = (case.nu - RATE_MID) / RATE_HALF
    x[..., 4] = (case.D - RATE_MID) / RATE_HALF
    x[..., 5] = (ug[0] / U0).reshape(L, L)
    x[..., 6] = (ug[1] / U0).reshape(L, L)
    x[..., 7] = (pg / PHI0).reshape(L, L)
    x[..., 8] = (rg / RHO0).reshape(L, L)
    return x


def targets(drho, u, phi, guess, L):
    """The correction to the coarse guess, [L][L][4] (float32): u (2) and phi in
    units of RES U0 / RES PHI0, the density deviation in units of RES RHO0."""
    rg, ug, pg = guess
    t = np.empty((L, L, OUT_CH), dtype=np.float32)
    t[..., 0] = ((u[0] - ug[0]) / (RES * U0)).reshape(L, L)
    t[..., 1] = ((u[1] - ug[1]) / (RES * U0)).reshape(L, L)
    t[..., 2] = ((phi - pg) / (RES * PHI0)).reshape(L, L)
    t[..., 3] = ((drho - rg) / (RES * RHO0)).reshape(L, L)
    return t


def fields(y, guess, L):
    """Warm-start estimate (rho - rho0 [N], u [2][N], phi [N]): the guess plus
    the network's correction y [L][L][4], means removed."""
    rg, ug, pg = guess
    y = np.asarray(y, dtype=np.float64).reshape(L * L, OUT_CH)
    u = ug + RES * U0 * np.stack([y[:, 0], y[:, 1]])
    phi = pg + RES * PHI0 * y[:, 2]
    drho = rg + RES * RHO0 * y[:, 3]
    return drho - drho.mean(), u - u.mean(axis=1, keepdims=True), phi - phi.mean()


# ---------------------------------------------------------------------------
# coarse solve
# ---------------------------------------------------------------------------

def downsample2(a, L):
    """2 x 2 block means of [..., L*L] fields (x fastest) -> [..., (L/2)^2]."""
    a = np.asarray(a)
    b = a.reshape(a.shape[:-1] + (L // 2, 2, L // 2, 2)).mean(axis=(-3, -1))
    return b.reshape(a.shape[:-1] + ((L // 2) ** 2,))


def upsample2(a, L):
    """Periodic Catmull-Rom interpolation of an (L/2)^2 field whose samples sit at
    fine positions 2X + 1/2 (block centres) onto the L x L fine nodes."""
    Lc = L // 2
    A = np.asarray(a, dtype=np.float64).reshape(Lc, Lc)

    def cr(p0, p1, p2, p3, t):
        return 0.5 * (2 * p1 + (p2 - p0) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t * t +
                      (3 * p1 - p0 - 3 * p2 + p3) * t ** 3)

    def along(A, ax):
        n = A.shape[ax]
        idx = np.arange(n)
        g = lambda k: np.take(A, (idx + k) % n, axis=ax)
        shape = list(A.shape)
        shape[ax] = 2 * n
        out = np.empty(shape)
        ev = [slice(None)] * A.ndim
        od = [slice(None)] * A.ndim
        ev[ax] = slice(0, None, 2)
        od[ax] = slice(1, None, 2)
        out[tuple(ev)] = cr(g(-2), g(-1), g(0), g(1), 0.75)   # fine 2X lies 3/4 past coarse X-1
        out[tuple(od)] = cr(g(-1), g(0), g(1), g(2), 0.25)    # fine 2X+1 lies 1/4 past coarse X
        return out

    return along(along(A, 0), 1).ravel()


def coarse_case(case):
    """The problem on the L/2 lattice under diffusive scaling."""
    from casclb_inputs import WarmstartCase
    return WarmstartCase(case.L // 2, case.nu, case.D, 8.0 * downsample2(case.F, case.L),
                         4.0 * downsample2(case.S, case.L), case.seed)


def guess_from_coarse(rc, uc, pc, L):
    """Fine-lattice guess (rho - rho0 [N], u [2][N], phi [N]) from the coarse steady
    density, half-forced velocity and scalar, means removed.  Under the diffusive
    scaling the coarse velocity is twice the fine one and the coarse density
    deviation (a pressure, ~ rho u^2 / c_s^2) four times."""
    ug = np.stack([upsample2(uc[0], L), upsample2(uc[1], L)]) / 2.0
    pg = upsample2(pc, L)
    rg = upsample2(np.asarray(rc) - np.mean(rc), L) / 4.0
    return rg - rg.mean(), ug - ug.mean(axis=1, keepdims=True), pg - pg.mean()


def initial_state(case, est, rho0=1.0):
    """(rho, u, phi) to hand to the equilibrium initialisation for the estimate
    est = (rho - rho0, half-forced u, half-sourced phi): the equilibrium's first
    moment is j = rho u - F/2 and its scalar phi - S/2 (eq. 25 and 43 read
    backwards), so the state's own half-forced moments are the estimate's."""
    drho, u, phi = est
    rho = rho0 + drho
    return rho, u - case.F / (2.0 * rho), phi - case.S / 2.0


def _context(cases, storage, K):
    L, nz = cases[0].L, len(cases)
    s = Solver("D2Q9_D2Q5", (L, L, nz), storage=storage, nu=cases[0].nu, D_phi=cases[0].D, residual_interval=K)
    s.set_force_field(np.concatenate([c.F for c in cases], axis=1))
    s.set_source_field(np.concatenate([c.S for c in cases]))
    return s


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


def steady_stack(cases, tol=1e-9, slice_tol=1e-8, max_steps=200000, K=100, storage="f32"):
    """Steady (rho, u, phi) of every case of one (nu, D) group, run as one stacked
    context.  Returns a list of (rho [N], u [2][N], phi [N], r_u, r_phi) per
    slice (half-forced moments); the per-slice residuals come from two readouts
    K steps apart."""
    L, nz = cases[0].L, len(cases)
    n = L * L
    with _context(cases, storage, K) as s:
        s.init_equilibrium()
        steps, r, rp = run_to_steady(s, tol, max_steps, K)
        _, u0, phi0 = s.moments(C.LB_MOMENTS_HALF_FORCED)
        s.step(K)
        rho1, u1, phi1 = s.moments(C.LB_MOMENTS_HALF_FORCED)
    out = []
    for z in range(nz):
        sl = slice(z * n, (z + 1) * n)
        ru = np.linalg.norm(u1[:, sl] - u0[:, sl]) / (K * np.linalg.norm(u1[:, sl]))
        rq = np.linalg.norm(phi1[sl] - phi0[sl]) / (K * np.linalg.norm(phi1[sl]))
        out.append((rho1[sl], u1[:, sl], phi1[sl], float(ru), float(rq)))
    return out, steps


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

    def __init__(self, L=256, max_batch=16, levels=6, channels=(16, 32, 32, 48, 48, 48), stream=None):
        import torch

        self.torch = torch
        self.L = L
        self.max_batch = max_batch
        cfg = C.lb_unet_config_default(levels=levels, channels=channels, in_channels=IN_CH, out_channels=OUT_CH,
                                       height=L, width=L, max_batch=max_batch,
                                       stream=stream if stream is not None else torch.cuda.current_stream().cuda_stream)
        self.cfg = dict(levels=levels, channels=list(channels), in_channels=IN_CH, out_channels=OUT_CH, L=L)
        self.h = C.lb_unet_create(cfg)
        self.num_params = C.lb_unet_num_params(self.h)

    def close(self):
        if self.h:
            C.lb_unet_destroy(self.h)
            self.h = None

    def init_params(self, seed=0):
        """He-normal weights (std sqrt(2 / (9 Ci))), zero biases."""
        g = np.random.default_rng(seed)
        parts = []
        for co, ci in layer_shapes(self.cfg["levels"], self.cfg["channels"], IN_CH, OUT_CH):
            parts.append(g.standard_normal(co * 9 * ci) * math.sqrt(2.0 / (9 * ci)))
            parts.append(np.zeros(co))
        p = np.concatenate(parts)
        assert p.size == self.num_params
        self.set_params(p)

    def set_params(self, p):
        C.lb_unet_set_params(self.h, np.asarray(p, dtype=np.float32))

    def get_params(self):
        return C.lb_unet_get_params(self.h)

    def predict(self, xs):
        """Network output for a batch of inputs [B][L][L][IN_CH] (numpy) -> numpy [B][L][L][OUT_CH]."""
        torch = self.torch
        xs = np.ascontiguousarray(xs, dtype=np.float32)
        out = np.empty(xs.shape[:3] + (OUT_CH,), dtype=np.float32)
        for i in range(0, xs.shape[0], self.max_batch):
            xb = torch.from_numpy(xs[i:i + self.max_batch]).cuda()
            yb = torch.empty(xb.shape[:3] + (OUT_CH,), dtype=torch.float32, device="cuda")
            C.lb_unet_forward(self.h, xb.data_ptr(), xb.shape[0], yb.data_ptr())
            out[i:i + xb.shape[0]] = yb.cpu().numpy()
        return out

    def train(self, X, Y, epochs, lr=2e-3, lr_end=1e-4, batch=None, seed=0, log_every=1):
        """Adam on the mean squared error over the normalised targets; X [N][L][L][IN_CH],
        Y [N][L][L][OUT_CH] (numpy, float32); cosine learning-rate decay from lr to lr_end.
        Returns the per-epoch mean losses."""
        torch = self.torch
        batch = batch or self.max_batch
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).cuda()
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
                 scales=np.array([U0, PHI0, K0, RATE_MID, RATE_HALF, RES, RHO0]), meta=json.dumps(meta or {}))

    @classmethod
    def load(cls, path, max_batch=16):
        z = np.load(path, allow_pickle=False)
        cfg = json.loads(str(z["config"]))
        net = cls(L=cfg["L"], max_batch=max_batch, levels=cfg["levels"], channels=cfg["channels"])
        net.set_params(z["params"])
        net.meta = json.loads(str(z["meta"]))
        return net


def solve_case(case, est=None, tol=1e-8, max_steps=400000, K=100, storage="f32", fields=False):
    """Steps from the state whose half-forced moments are the estimate
    est = (rho - rho0 [N], u [2][N], phi [N]) (None: rest) until both residuals
    are below tol; returns (steps, seconds, r_u, r_phi), plus the final
    half-forced (rho, u, phi) when `fields`."""
    with _context([case], storage, K) as s:
        if est is None:
            s.init_equilibrium()
        else:
            rho, u, phi = initial_state(case, est)
            s.init_equilibrium(rho=rho, u=u, phi=phi)
        s.synchronize()
        t0 = time.perf_counter()
        steps, r, rp = run_to_steady(s, tol, max_steps, K)
        out = (steps, time.perf_counter() - t0, r, rp)
        if fields:
            out = out + tuple(s.moments(C.LB_MOMENTS_HALF_FORCED))
        return out


def generate(groups, slices, L=256, first_seed=1, tol=1e-9, slice_tol=1e-8):
    """Features and targets of `groups` x `slices` steady problems (slices whose
    own residual misses slice_tol are dropped)."""
    from casclb_inputs import warmstart_group
    X, Y = [], []
    dropped = 0
    t0 = time.perf_counter()
    for gi in range(groups):
        cases = warmstart_group(first_seed + gi, slices, L=L)
        res, steps = steady_stack(cases, tol=tol, slice_tol=slice_tol)
        coarse, _ = steady_stack([coarse_case(c) for c in cases], tol=tol, slice_tol=slice_tol)
        for c, (rho, u, phi, ru, rq), (rc, uc, pc, _, _) in zip(cases, res, coarse):
            if ru < slice_tol and rq < slice_tol:
                g = guess_from_coarse(rc, uc, pc, L)
                X.append(features(c, g))
                Y.append(targets(rho - rho.mean(), u, phi, g, L))
            else:
                dropped += 1
        _say(f"[warmstart] group {gi + 1}/{groups} (nu {cases[0].nu:.3f}, D {cases[0].D:.3f}): {steps} steps, "
             f"worst slice residuals {max(r[3] for r in res):.1e} / {max(r[4] for r in res):.1e}, "
             f"{time.perf_counter() - t0:.0f} s")
    return np.stack(X), np.stack(Y), dropped


def warm_estimate(net, case, tol=1e-8, K=100):
    """(estimate, coarse-only guess, coarse steps, seconds of coarse solve + inference)."""
    t0 = time.perf_counter()
    cs = solve_case(coarse_case(case), None, tol=tol, K=K, fields=True)
    g = guess_from_coarse(cs[4], cs[5], cs[6], case.L)
    y = net.predict(features(case, g)[None])[0]
    return fields(y, g, case.L), g, cs[0], time.perf_counter() - t0


def evaluate(net, cases, tol=1e-8, K=100):
    """Steps to tol from a cold start, from the coarse guess alone, and from the
    coarse guess plus the learned correction; returns a list of dicts."""
    out = []
    for c in cases:
        est, g, csteps, t_est = warm_estimate(net, c, tol, K)
        cold = solve_case(c, None, tol=tol, K=K, fields=True)
        coarse_only = solve_case(c, g, tol=tol, K=K)
        warm = solve_case(c, est, tol=tol, K=K)
        rf, uf, pf = cold[4] - cold[4].mean(), cold[5], cold[6]
        err = lambda e: [float(np.linalg.norm(e[1] - uf) / np.linalg.norm(uf)),
                         float(np.linalg.norm(e[2] - pf) / np.linalg.norm(pf)),
                         float(np.linalg.norm(e[0] - rf) / np.linalg.norm(rf))]
        out.append(dict(seed=c.seed, nu=c.nu, D=c.D, cold_steps=cold[0], coarse_steps=csteps,
                        coarse_only_steps=coarse_only[0], warm_steps=warm[0], cold_s=cold[1], estimate_s=t_est,
                        coarse_only_s=coarse_only[1], warm_s=warm[1], guess_error=err(g), estimate_error=err(est)))
        _say(f"[warmstart] case {c.seed}: cold {cold[0]} steps ({cold[1]:.2f} s); coarse guess {coarse_only[0]} "
             f"(error u {out[-1]['guess_error'][0]:.1e}, rho {out[-1]['guess_error'][2]:.1e}); coarse + network {warm[0]} steps "
             f"(error u {out[-1]['estimate_error'][0]:.1e}, phi {out[-1]['estimate_error'][1]:.1e}, "
             f"rho {out[-1]['estimate_error'][2]:.1e}) + "
             f"{csteps} coarse steps, {t_est:.2f} s")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--groups", type=int, default=48)
    tr.add_argument("--slices", type=int, default=16)
    tr.add_argument("--L", type=int, default=256)
    tr.add_argument("--epochs", type=int, default=60)
    tr.add_argument("--lr", type=float, default=2e-3)
    tr.add_argument("--lowpass-levels", type=int, default=0)
    tr.add_argument("--lowpass-weight", type=float, default=0.0)
    tr.add_argument("--out", required=True)
    tr.add_argument("--eval-cases", type=int, default=8)
    ev = sub.add_parser("evaluate")
    ev.add_argument("--weights", required=True)
    ev.add_argument("--cases", type=int, default=8)
    ev.add_argument("--L", type=int, default=256)
    args = ap.parse_args(argv)

    import torch

    torch.cuda.is_available()
    from casclb_inputs import warmstart_case
    if args.cmd == "train":
        X, Y, dropped = generate(args.groups, args.slices, L=args.L)
        _say(f"[warmstart] {X.shape[0]} training solutions ({dropped} dropped)")
        net = Surrogate(L=args.L)
        net.init_params(seed=0)
        if args.lowpass_levels:
            C.lb_unet_set_lowpass_loss(net.h, args.lowpass_levels, args.lowpass_weight)
        t0 = time.perf_counter()
        hist = net.train(X, Y, args.epochs, lr=args.lr)
        train_s = time.perf_counter() - t0
        meta = dict(samples=int(X.shape[0]), dropped=int(dropped), groups=args.groups, slices=args.slices,
                    epochs=args.epochs, lr=args.lr, lowpass=[args.lowpass_levels, args.lowpass_weight],
                    final_loss=hist[-1], train_seconds=train_s, losses=hist)
        net.save(args.out, meta)
        cases = [warmstart_case(100000 + i, L=args.L) for i in range(args.eval_cases)]
        res = evaluate(net, cases)
        print(json.dumps(dict(meta=meta, eval=res)), flush=True)
        net.close()
    else:
        net = Surrogate.load(args.weights)
        cases = [warmstart_case(100000 + i, L=args.L) for i in range(args.cases)]
        print(json.dumps(evaluate(net, cases)), flush=True)
        net.close()


if __name__ == "__main__":
    main()
