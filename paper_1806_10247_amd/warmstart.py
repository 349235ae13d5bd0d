"""Learned warm start for steady periodic flow + scalar problems.

A U-Net (include/casclb_unet.h) maps the force field F, the source field S
and the two relaxation rates of a periodic D2Q9 + D2Q5 problem to an
estimate of the steady half-forced velocity u and half-sourced scalar phi.
The lattice is then initialised with the product-form equilibrium of that
estimate and iterated with the cascaded scheme until both residuals (velocity
and scalar, every K steps) fall below the tolerance, exactly as from a cold
start: the network only moves the starting point, the converged answer is
the solver's.

Training data are steady solutions this solver produces: problems sharing
one (nu, D) pair run as the slices of one stacked 2D context (nz slices, one
launch per step), each slice's own residual checked at the end.

    python -m paper_1806_10247_amd.warmstart train --groups 64 --slices 16 --out weights.npz
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
K0 = 2.0 * math.pi * 5.0 / 256.0   # a mid wavenumber of the forcing (L = 256)
RATE_MID, RATE_HALF = 0.14, 0.06   # nu and D are mapped to (rate - mid) / half
IN_CH, OUT_CH = 5, 3


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def features(case):
    """Network input [L][L][5] (float32): F/(nu K0^2 U0) (2), S/(D K0^2 PHI0),
    and the two rates as constant channels."""
    L = case.L
    x = np.empty((L, L, IN_CH), dtype=np.float32)
    x[..., 0] = (case.F[0] / (case.nu * K0 * K0 * U0)).reshape(L, L)
    x[..., 1] = (case.F[1] / (case.nu * K0 * K0 * U0)).reshape(L, L)
    x[..., 2] = (case.S / (case.D * K0 * K0 * PHI0)).reshape(L, L)
    x[..., 3] = (case.nu - RATE_MID) / RATE_HALF
    x[..., 4] = (case.D - RATE_MID) / RATE_HALF
    return x


def targets(u, phi, L):
    """[L][L][3] (float32) from u [2][N], phi [N]."""
    t = np.empty((L, L, OUT_CH), dtype=np.float32)
    t[..., 0] = (u[0] / U0).reshape(L, L)
    t[..., 1] = (u[1] / U0).reshape(L, L)
    t[..., 2] = (phi / PHI0).reshape(L, L)
    return t


def fields(y, L):
    """(u [2][N], phi [N]) float64 from a network output [L][L][3]."""
    y = np.asarray(y, dtype=np.float64).reshape(L * L, OUT_CH)
    return np.stack([y[:, 0] * U0, y[:, 1] * U0]), y[:, 2] * PHI0


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
    """Steady (u, phi) of every case of one (nu, D) group, run as one stacked
    context.  Returns a list of (u [2][N], phi [N], r_u, r_phi) per slice; the
    per-slice residuals come from two readouts K steps apart."""
    L, nz = cases[0].L, len(cases)
    n = L * L
    with _context(cases, storage, K) as s:
        s.init_equilibrium()
        steps, r, rp = run_to_steady(s, tol, max_steps, K)
        _, u0, phi0 = s.moments(C.LB_MOMENTS_HALF_FORCED)
        s.step(K)
        _, u1, phi1 = s.moments(C.LB_MOMENTS_HALF_FORCED)
    out = []
    for z in range(nz):
        sl = slice(z * n, (z + 1) * n)
        ru = np.linalg.norm(u1[:, sl] - u0[:, sl]) / (K * np.linalg.norm(u1[:, sl]))
        rq = np.linalg.norm(phi1[sl] - phi0[sl]) / (K * np.linalg.norm(phi1[sl]))
        out.append((u1[:, sl], phi1[sl], float(ru), float(rq)))
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

    def __init__(self, L=256, max_batch=16, levels=4, channels=(16, 32, 48, 96), stream=None):
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
        """Network output for a batch of inputs [B][L][L][5] (numpy) -> numpy [B][L][L][3]."""
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
        """Adam on the mean squared error over the normalised targets; X [N][L][L][5],
        Y [N][L][L][3] (numpy, float32); cosine learning-rate decay from lr to lr_end.
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
                 scales=np.array([U0, PHI0, K0, RATE_MID, RATE_HALF]), meta=json.dumps(meta or {}))

    @classmethod
    def load(cls, path, max_batch=16):
        z = np.load(path, allow_pickle=False)
        cfg = json.loads(str(z["config"]))
        net = cls(L=cfg["L"], max_batch=max_batch, levels=cfg["levels"], channels=cfg["channels"])
        net.set_params(z["params"])
        net.meta = json.loads(str(z["meta"]))
        return net


def solve_case(case, init=None, tol=1e-8, max_steps=400000, K=100, storage="f32", fields=False):
    """Steps from the equilibrium of `init` = (u [2][N], phi [N]) (None: rest)
    until both residuals are below tol; returns (steps, seconds, r_u, r_phi),
    plus the final half-forced (u, phi) when `fields`."""
    with _context([case], storage, K) as s:
        if init is None:
            s.init_equilibrium()
        else:
            s.init_equilibrium(u=init[0], phi=init[1])
        s.synchronize()
        t0 = time.perf_counter()
        steps, r, rp = run_to_steady(s, tol, max_steps, K)
        out = (steps, time.perf_counter() - t0, r, rp)
        if fields:
            _, u, phi = s.moments(C.LB_MOMENTS_HALF_FORCED)
            out = out + (u, phi)
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
        for c, (u, phi, ru, rq) in zip(cases, res):
            if ru < slice_tol and rq < slice_tol:
                X.append(features(c))
                Y.append(targets(u, phi, L))
            else:
                dropped += 1
        _say(f"[warmstart] group {gi + 1}/{groups} (nu {cases[0].nu:.3f}, D {cases[0].D:.3f}): {steps} steps, "
             f"worst slice residuals {max(r[2] for r in res):.1e} / {max(r[3] for r in res):.1e}, "
             f"{time.perf_counter() - t0:.0f} s")
    return np.stack(X), np.stack(Y), dropped


def evaluate(net, cases, tol=1e-8, K=100):
    """Cold and warm steps to tol for each case; returns a list of dicts."""
    out = []
    for c in cases:
        t0 = time.perf_counter()
        y = net.predict(features(c)[None])[0]
        t_pred = time.perf_counter() - t0
        u, phi = fields(y, c.L)
        cold = solve_case(c, None, tol=tol, K=K)
        warm = solve_case(c, (u, phi), tol=tol, K=K)
        out.append(dict(seed=c.seed, nu=c.nu, D=c.D, cold_steps=cold[0], warm_steps=warm[0], cold_s=cold[1],
                        warm_s=warm[1], predict_s=t_pred, cold_r=[cold[2], cold[3]], warm_r=[warm[2], warm[3]]))
        _say(f"[warmstart] case {c.seed}: cold {cold[0]} steps ({cold[1]:.2f} s), warm {warm[0]} steps "
             f"({warm[1]:.2f} s + {t_pred * 1e3:.1f} ms inference)")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--groups", type=int, default=64)
    tr.add_argument("--slices", type=int, default=16)
    tr.add_argument("--L", type=int, default=256)
    tr.add_argument("--epochs", type=int, default=30)
    tr.add_argument("--lr", type=float, default=2e-3)
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
        t0 = time.perf_counter()
        hist = net.train(X, Y, args.epochs, lr=args.lr)
        train_s = time.perf_counter() - t0
        meta = dict(samples=int(X.shape[0]), dropped=int(dropped), groups=args.groups, slices=args.slices,
                    epochs=args.epochs, lr=args.lr, final_loss=hist[-1], train_seconds=train_s, losses=hist)
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
