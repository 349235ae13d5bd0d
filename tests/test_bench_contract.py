"""Host-side parts of the benchmark's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_priming_ends_right_after_a_residual_check():
    """The timed region starts at a multiple of the residual interval, after at least
    one whole interval of untimed steps (so the graph used after every check exists)."""
    K = bench.RESIDUAL_INTERVAL
    for w in range(0, 3 * K + 7):
        p = bench.priming_steps(w)
        assert (w + p) % K == 0
        assert K < p <= 2 * K


def test_kernel_hash_covers_the_step_kernel_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0


def test_cpu_baseline_reports_the_contract_fields():
    """The oracle baseline: a positive rate in MLUPS, the thread count it used, its
    kind and the sample it was measured on, and the one-thread rate beside it."""
    r = bench.cpu_baseline(target_s=0.2, single_s=0.1)
    assert r["unit"] == "MLUPS" and r["kind"] == "oracle"
    assert r["value"] > 0 and r["single_thread_value"] > 0 and r["cores"] >= 1
    assert "256x256x16" in r["sample"] and "1 thread" in r["single_thread_sample"]
    assert r["nproc"] >= 1 and isinstance(r["cpu_model"], str)


def test_measured_traffic_reads_the_committed_counter_summary():
    value, path = bench.measured_traffic("step_d3q27_f32dev_duct256")
    assert path is not None and os.path.exists(path)
    assert value is None or value > 3.0e9    # HBM bytes per launch, near the 3.62e9 algorithmic ones
    assert bench.measured_traffic("no_such_kernel") == (None, None)


# ---------------------------------------------------------------------------
# the analytic comparators the benchmark reports errors against
# ---------------------------------------------------------------------------

def test_duct_startup_profile_against_the_oracle_and_its_limits():
    """Start-up profile of the duct (heat equation with a uniform source between
    walls): F t in the interior, symmetric, a layer at the walls; the FP64 oracle's
    D3Q27 duct from rest matches its interior exactly at t = steps + 1/2 (the
    half-forced velocity) and its whole cross-section to second order in the
    layer's resolution (error x 1/4 when sqrt(nu t) doubles)."""
    import numpy as np

    import oracle as O
    F, nu = 1e-7, (0.76 - 0.5) / 3
    errs = []
    for n, steps in ((48, 60), (96, 240)):
        ua = bench.duct_startup_profile(n, F, nu, steps + 0.5)
        assert np.allclose(ua, ua.T, rtol=0, atol=1e-20)
        assert abs(ua[n // 2, n // 2] / (F * (steps + 0.5)) - 1) < 1e-12     # untouched interior
        assert ua[0, n // 2] < 0.6 * ua[n // 2, n // 2]                      # wall layer
        d = O.Domain(O.D3Q27, 1, n, n, bc=(O.PERIODIC, O.BOUNCE_BACK, O.BOUNCE_BACK), nu=nu, force=(F, 0, 0))
        d.init_equilibrium()
        d.run(steps)
        _, u, _ = d.moments(1)
        ux = d.grid(u[0])[:, :, 0]
        assert abs(ux[n // 2, n // 2] / ua[n // 2, n // 2] - 1) < 1e-8
        errs.append(np.sqrt(((ux - ua) ** 2).sum() / (ua**2).sum()))
    assert errs[0] < 0.015 and 3.0 < errs[0] / errs[1] < 5.0, errs
    try:
        bench.duct_startup_profile(16, F, nu, 1000.0)
        raise AssertionError("thick layers must be refused")
    except ValueError:
        pass


def test_periodic_mode_projection_recovers_planted_amplitudes():
    """A velocity field built as the Stokes growth of the transverse part of a Fourier
    force gives zero error; scaling it by 1.01 gives 1%."""
    import numpy as np
    import torch

    from casclb_inputs import coords, fourier_modes
    n, nu, t = 16, 0.05, 30.5
    modes = fourier_modes((n, n, n), nmodes=3, amp=1e-6, kmax=2, seed=3)
    pts = coords((n, n, n))
    u = np.zeros((3, n**3))
    for km, am, th in zip(modes.k, modes.a, modes.theta):
        kv = np.asarray(km, dtype=np.float64)
        khat = kv / np.linalg.norm(kv)
        aperp = am - khat * (khat @ am)
        k2 = float((2 * np.pi * kv / n) @ (2 * np.pi * kv / n))
        ph = 2 * np.pi * (kv @ pts) / n + th
        u += aperp[:, None] * np.sin(ph)[None, :] * (1 - np.exp(-nu * k2 * t)) / (nu * k2)
    for scale, want in ((1.0, 0.0), (1.01, 0.01)):
        runs = {"f64": {"u": torch.from_numpy(scale * u), "steps_total": 30}}
        e = bench.periodic_modes_vs_analytic(torch, runs, modes, n, nu, dev="cpu")["f64"]
        assert abs(e["rel_l2_transverse_modes"] - want) < 1e-9, e


def test_coupled_mode_amplitudes_recover_planted_fields():
    import numpy as np
    import torch

    from casclb_inputs import coords, coupled_2d, product_source_2d, vortex_force_2d
    w = coupled_2d(64)
    k, t = 2 * np.pi / 64, 25.5
    lam, om, A, B = 2 * w.nu * k * k, w.force_omega, w.extra["A"], w.extra["B"]
    a = A * (lam * np.cos(om * t) + om * np.sin(om * t) - lam * np.exp(-lam * t)) / (lam**2 + om**2)
    lamp = 2 * w.D * k * k
    b = B * (1 - np.exp(-lamp * t)) / lamp
    pts = coords(w.shape)
    runs = {"f32": {"u": torch.from_numpy(1.02 * a * vortex_force_2d(w.shape, 1.0, pts)),
                    "phi": torch.from_numpy(0.99 * b * product_source_2d(w.shape, 1.0, pts)),
                    "workload": w, "steps_total": 25}}
    e = bench.coupled_vs_analytic(torch, runs, dev="cpu")["f32"]
    assert abs(e["velocity_amplitude_rel_err"] - 0.02) < 1e-9 and abs(e["scalar_amplitude_rel_err"] + 0.01) < 1e-9


def test_network_forward_bytes_count_each_activation_once():
    """The least HBM traffic of a forward pass, counted by hand for two small
    networks: one level (conv 1 reads the float32 input and writes c0, conv 2
    reads and writes c0, the output convolution reads c0 and writes float32) and
    two levels (plus the pooled copy, the coarse level's two convolutions and
    the decoder convolution that reads the skip and the half-resolution input)."""
    px = 2 * 8 * 8                                    # batch 2, 8 x 8
    one = px * (9 * 4 + 16 * 2) + px * (16 * 2 + 16 * 2) + px * (16 * 2 + 4 * 4)
    assert bench.unet_forward_bytes(1, (16,), 9, 4, 8, 8, 2) == one
    q = px // 4
    two = (px * (9 * 4 + 16 * 2) + px * (16 * 2 + 16 * 2) + q * 16 * 2      # level 0 and its pooled copy
           + q * (16 * 2 + 32 * 2) + q * (32 * 2 + 32 * 2)                  # level 1
           + px * (16 * 2 + 16 * 2) + q * 32 * 2                            # decoder at level 0
           + px * (16 * 2 + 4 * 4))                                         # output
    assert bench.unet_forward_bytes(2, (16, 32), 9, 4, 8, 8, 2) == two
