"""Float64 reference of the warm-start surrogate network (test infrastructure only).

Not part of the product: only tests/, the package's smoke check and the
benchmark's CPU baseline may import it.  It shares no code with the HIP
library.  Everything is written from the definitions, in NHWC layout
(batch, row y, column x, channel), periodic (circular) in y and x:

  conv3x3      y[n,i,j,o] = b[o] + sum_{a,c in 0..2, k} w[o,a,c,k] x[n, i+a-1, j+c-1, k]
               (indices modulo H and W)
  relu         max(v, 0)
  avgpool2     y[n,i,j,k] = mean of x[n, 2i+a, 2j+c, k] over a, c in {0, 1}
  upsample2    y[n, 2i+a, 2j+c, k] = x[n, i, j, k] (nearest)
  concat       channels of the skip tensor first, then the up-sampled ones

Network (a U-Net over `levels` resolutions with feature widths `channels`):
  encoder level l: conv (in -> c_l) relu, conv (c_l -> c_l) relu = skip_l,
                   then avgpool2 into level l+1 (in = c_l there);
  bottom level L-1: its second conv output is the decoder state d_{L-1};
  decoder level l = L-2 .. 0: d_l = relu(conv(concat(skip_l, upsample2(d_{l+1}))))
                   (c_l + c_{l+1} -> c_l);
  output: conv (c_0 -> out_channels), no activation.
Parameters are one flat vector: per layer in the order above, w [Co][3][3][Ci]
then b [Co].

Loss: mean squared error over all output values.  Optimiser: Adam (Kingma &
Ba, 2015) with bias correction.  Gradients follow from the chain rule:
  conv3x3 input gradient  dx[n,i,j,k] = sum_{a,c,o} w[o,a,c,k] g[n, i-a+1, j-c+1, o]
  conv3x3 weight gradient dw[o,a,c,k] = sum_{n,i,j} g[n,i,j,o] x[n, i+a-1, j+c-1, k]
  bias gradient           db[o] = sum_{n,i,j} g[n,i,j,o]
  relu                    g * (y > 0)
  avgpool2                dx[n, 2i+a, 2j+c, k] = g[n,i,j,k] / 4
  upsample2               dx[n,i,j,k] = sum_{a,c} g[n, 2i+a, 2j+c, k]
"""
import numpy as np


def _shifted(x, a, c):
    """x[n, i + a - 1, j + c - 1, :] (periodic)."""
    return np.roll(x, shift=(1 - a, 1 - c), axis=(1, 2))


def conv3x3(x, w, b=None):
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for a in range(3):
        for c in range(3):
            y += _shifted(x, a, c) @ w[:, a, c, :].T
    return y if b is None else y + b


def conv3x3_input_grad(g, w):
    dx = np.zeros(g.shape[:3] + (w.shape[3],))
    for a in range(3):
        for c in range(3):
            # g[n, i - a + 1, j - c + 1, :] = roll by (a - 1, c - 1)
            dx += np.roll(g, shift=(a - 1, c - 1), axis=(1, 2)) @ w[:, a, c, :]
    return dx


def conv3x3_weight_grad(g, x):
    co, ci = g.shape[3], x.shape[3]
    dw = np.zeros((co, 3, 3, ci))
    gm = g.reshape(-1, co)
    for a in range(3):
        for c in range(3):
            dw[:, a, c, :] = gm.T @ _shifted(x, a, c).reshape(-1, ci)
    return dw


def relu(v):
    return np.maximum(v, 0.0)


def avgpool2(x):
    n, h, w, k = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, k).mean(axis=(2, 4))


def avgpool2_grad(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_grad(g):
    n, h, w, k = g.shape
    return g.reshape(n, h // 2, 2, w // 2, 2, k).sum(axis=(2, 4))


def layer_shapes(levels, channels, in_channels, out_channels):
    """(Co, Ci) of every conv layer, in parameter order."""
    c = list(channels)[:levels]
    shapes = []
    for l in range(levels):
        shapes.append((c[l], in_channels if l == 0 else c[l - 1]))
        shapes.append((c[l], c[l]))
    for l in range(levels - 2, -1, -1):
        shapes.append((c[l], c[l] + c[l + 1]))
    shapes.append((out_channels, c[0]))
    return shapes


class UNet:
    """Float64 network with the architecture of the module docstring."""

    def __init__(self, levels, channels, in_channels, out_channels):
        self.levels = levels
        self.channels = list(channels)[:levels]
        self.in_channels, self.out_channels = in_channels, out_channels
        self.shapes = layer_shapes(levels, channels, in_channels, out_channels)
        self.sizes = [co * 9 * ci + co for co, ci in self.shapes]
        self.num_params = int(sum(self.sizes))

    def unpack(self, p):
        out, off = [], 0
        for co, ci in self.shapes:
            w = p[off:off + co * 9 * ci].reshape(co, 3, 3, ci)
            off += co * 9 * ci
            b = p[off:off + co]
            off += co
            out.append((w, b))
        return out

    def forward(self, p, x, store=None):
        """Returns (output, cache).  `store` (default: identity) is applied to the
        input and to every activation the network keeps (the precision a storage
        format imposes); the output is not passed through it."""
        st = store if store is not None else (lambda a: a)
        L = self.levels
        layers = self.unpack(p)
        h = st(x)
        cache = {"x": h}
        li = 0
        skips = []
        for l in range(L):
            a1 = st(relu(conv3x3(h, *layers[li])))
            a2 = st(relu(conv3x3(a1, *layers[li + 1])))
            cache[("enc", l)] = (h, a1, a2)
            li += 2
            skips.append(a2)
            if l < L - 1:
                h = st(avgpool2(a2))
        d = skips[L - 1]
        for l in range(L - 2, -1, -1):
            cat = np.concatenate([skips[l], upsample2(d)], axis=3)
            d = st(relu(conv3x3(cat, *layers[li])))
            cache[("dec", l)] = (cat, d)
            li += 1
        y = conv3x3(d, *layers[li])
        cache["last"] = d
        return y, cache

    def backward(self, p, cache, gy, record=None):
        """Gradient of sum(gy * output) with respect to the flat parameters and the input.
        `record` (a list) receives every gradient array that multiplies weights or
        activations on the way back, in the order they are formed."""
        rec = record.append if record is not None else (lambda a: None)
        rec(gy)
        L = self.levels
        layers = self.unpack(p)
        grads = [None] * len(layers)
        li = len(layers) - 1
        d = cache["last"]
        grads[li] = (conv3x3_weight_grad(gy, d), gy.sum(axis=(0, 1, 2)))
        gd = conv3x3_input_grad(gy, layers[li][0])
        li -= 1
        gskip = [None] * L
        for l in range(0, L - 1):
            cat, dl = cache[("dec", l)]
            gpre = gd * (dl > 0)
            rec(gpre)
            grads[li] = (conv3x3_weight_grad(gpre, cat), gpre.sum(axis=(0, 1, 2)))
            gcat = conv3x3_input_grad(gpre, layers[li][0])
            cl = self.channels[l]
            gskip[l] = gcat[..., :cl]
            gd = upsample2_grad(gcat[..., cl:])
            li -= 1
        # gd is now the gradient of the bottom level's second activation
        gnext = gd
        for l in range(L - 1, -1, -1):
            h, a1, a2 = cache[("enc", l)]
            g2 = gnext if l == L - 1 else gskip[l] + gnext
            g2 = g2 * (a2 > 0)
            rec(g2)
            grads[li] = (conv3x3_weight_grad(g2, a1), g2.sum(axis=(0, 1, 2)))
            g1 = conv3x3_input_grad(g2, layers[li][0]) * (a1 > 0)
            rec(g1)
            grads[li - 1] = (conv3x3_weight_grad(g1, h), g1.sum(axis=(0, 1, 2)))
            gh = conv3x3_input_grad(g1, layers[li - 1][0])
            li -= 2
            if l > 0:
                gnext = avgpool2_grad(gh)
        flat = np.concatenate([np.concatenate([gw.ravel(), gb.ravel()]) for gw, gb in grads])
        return flat, gh


def mse(y, t):
    """Mean squared error and its gradient with respect to y."""
    d = y - t
    return float((d * d).mean()), 2.0 * d / d.size


def lowpass_mse(y, t, levels, weight):
    """weight * MSE of the (2^levels)-block means of y and t, and its gradient
    with respect to y (levels applications of avgpool2 and of its adjoint)."""
    py, pt = y, t
    for _ in range(levels):
        py, pt = avgpool2(py), avgpool2(pt)
    d = py - pt
    g = 2.0 * weight * d / d.size
    for _ in range(levels):
        g = avgpool2_grad(g)
    return weight * float((d * d).mean()), g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1**t)
    vhat = v / (1.0 - beta2**t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def round_bf16(a):
    """Round to bfloat16 (nearest, ties to even) through float32, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
