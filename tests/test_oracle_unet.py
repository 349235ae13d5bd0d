"""Pins of the float64 warm-start network oracle (oracle/unet.py) against brute
force, identities of the definitions and finite differences."""
import numpy as np
import pytest

from oracle import unet as U


def _rng(s):
    return np.random.default_rng(s)


def test_conv3x3_matches_brute_force_loops():
    g = _rng(1)
    n, h, w, ci, co = 2, 4, 5, 3, 2
    x = g.standard_normal((n, h, w, ci))
    wt = g.standard_normal((co, 3, 3, ci))
    b = g.standard_normal(co)
    y = U.conv3x3(x, wt, b)
    ref = np.zeros((n, h, w, co))
    for nn in range(n):
        for i in range(h):
            for j in range(w):
                for o in range(co):
                    s = b[o]
                    for a in range(3):
                        for c in range(3):
                            for k in range(ci):
                                s += wt[o, a, c, k] * x[nn, (i + a - 1) % h, (j + c - 1) % w, k]
                    ref[nn, i, j, o] = s
    assert np.abs(y - ref).max() < 1e-12


def test_conv3x3_delta_kernel_is_identity_and_shift():
    g = _rng(2)
    x = g.standard_normal((1, 6, 4, 2))
    w = np.zeros((2, 3, 3, 2))
    w[0, 1, 1, 0] = w[1, 1, 1, 1] = 1.0
    assert np.array_equal(U.conv3x3(x, w), x)
    # the tap (a, c) = (2, 0) reads x[i + 1, j - 1]
    w2 = np.zeros((1, 3, 3, 1))
    w2[0, 2, 0, 0] = 1.0
    y = U.conv3x3(x[..., :1], w2)
    assert np.array_equal(y[0, 2, 3, 0], x[0, 3, 2, 0])
    assert np.array_equal(y[0, 5, 0, 0], x[0, 0, 3, 0])   # wraps in both directions


def test_conv3x3_commutes_with_periodic_shifts():
    g = _rng(3)
    x = g.standard_normal((1, 8, 6, 3))
    w = g.standard_normal((4, 3, 3, 3))
    lhs = U.conv3x3(np.roll(x, (2, -1), axis=(1, 2)), w)
    rhs = np.roll(U.conv3x3(x, w), (2, -1), axis=(1, 2))
    assert np.abs(lhs - rhs).max() < 1e-12


def test_backward_operators_are_adjoints():
    g = _rng(4)
    x = g.standard_normal((2, 6, 8, 3))
    w = g.standard_normal((5, 3, 3, 3))
    gy = g.standard_normal((2, 6, 8, 5))
    # <conv(x), g> = <x, dgrad(g)> = <w, wgrad(g, x)>
    lhs = (U.conv3x3(x, w) * gy).sum()
    assert abs(lhs - (x * U.conv3x3_input_grad(gy, w)).sum()) < 1e-10 * abs(lhs)
    assert abs(lhs - (w * U.conv3x3_weight_grad(gy, x)).sum()) < 1e-10 * abs(lhs)
    p = g.standard_normal((2, 3, 4, 3))
    assert abs((U.avgpool2(x) * p).sum() - (x * U.avgpool2_grad(p)).sum()) < 1e-12
    q = g.standard_normal((2, 12, 16, 3))
    assert abs((U.upsample2(x) * q).sum() - (x * U.upsample2_grad(q)).sum()) < 1e-11


def test_avgpool_and_upsample_values():
    x = np.arange(16.0).reshape(1, 4, 4, 1)
    p = U.avgpool2(x)
    assert p[0, 0, 0, 0] == (0 + 1 + 4 + 5) / 4 and p[0, 1, 1, 0] == (10 + 11 + 14 + 15) / 4
    u = U.upsample2(p)
    assert u.shape == x.shape and u[0, 3, 2, 0] == p[0, 1, 1, 0]


def test_layer_shapes_and_parameter_count():
    shapes = U.layer_shapes(4, [16, 32, 48, 96], 5, 3)
    assert shapes == [(16, 5), (16, 16), (32, 16), (32, 32), (48, 32), (48, 48), (96, 48), (96, 96),
                      (48, 144), (32, 80), (16, 48), (3, 16)]
    net = U.UNet(4, [16, 32, 48, 96], 5, 3)
    assert net.num_params == sum(co * 9 * ci + co for co, ci in shapes)


@pytest.mark.parametrize("levels", [1, 3])
def test_network_gradient_matches_finite_differences(levels):
    """d/dp and d/dx of sum(c * net(p, x)) by central differences at random entries."""
    g = _rng(10 + levels)
    net = U.UNet(levels, [3, 4, 5], 2, 2)
    h = w = 8
    p = 0.4 * g.standard_normal(net.num_params)
    x = g.standard_normal((2, h, w, 2))
    cw = g.standard_normal((2, h, w, 2))
    f = lambda pp, xx: float((net.forward(pp, xx)[0] * cw).sum())
    y, cache = net.forward(p, x)
    gp, gx = net.backward(p, cache, cw)
    eps = 1e-6
    for idx in g.choice(net.num_params, 40, replace=False):
        e = np.zeros_like(p)
        e[idx] = eps
        fd = (f(p + e, x) - f(p - e, x)) / (2 * eps)
        assert abs(fd - gp[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, gp[idx])
    for _ in range(15):
        idx = tuple(int(g.integers(0, s)) for s in x.shape)
        e = np.zeros_like(x)
        e[idx] = eps
        fd = (f(p, x + e) - f(p, x - e)) / (2 * eps)
        assert abs(fd - gx[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, gx[idx])


def test_mse_gradient():
    g = _rng(20)
    y, t = g.standard_normal((2, 3, 4, 2)), g.standard_normal((2, 3, 4, 2))
    loss, gy = U.mse(y, t)
    assert abs(loss - ((y - t) ** 2).sum() / y.size) < 1e-15
    e = np.zeros_like(y)
    e[1, 2, 3, 0] = 1e-6
    fd = (U.mse(y + e, t)[0] - U.mse(y - e, t)[0]) / 2e-6
    assert abs(fd - gy[1, 2, 3, 0]) < 1e-9


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exactly g and g^2, so
    every step moves each parameter by lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.array([1.0, 2.0, 3.0])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 0.01
    for t in range(1, 6):
        p, m, v = U.adam_step(p, g, m, v, t, lr)
    want = np.array([1.0, 2.0, 3.0]) - 5 * lr * g / (np.abs(g) + 1e-8)
    assert np.abs(p - want).max() < 1e-12


def test_round_bf16():
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7, 1.0 + 3 * 2**-8, -3.140625, 1e-3])
    r = U.round_bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                  # tie, rounds to even (mantissa ...0)
    assert r[2] == 1.0 + 2**-7          # representable
    assert r[3] == 1.0 + 2**-6          # tie, rounds to even (up)
    assert r[4] == -3.140625
    assert abs(r[5] - 1e-3) <= 2**-9 * 1e-3
