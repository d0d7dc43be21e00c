"""FP64 reference of the warm-start network (test infrastructure only).

The network is not part of the paper (its counterpart there is a Poisson
preconditioner, App. G); it is specified by the library's API: four 3x3
convolution layers on 64 x 64 fields, channels 3 -> 32 -> 32 -> 32 -> 1, the taps
of layer l spaced DILATION[l] = 1, 2, 4, 8 apart (receptive field 31 x 31), tanh
after the first three, zero padding along rows (eta), periodic padding along
columns (xi). Parameters are one flat vector: for each layer the weights
w[co][ci][3][3] followed by the bias b[co].

Written as plain loops over the nine taps with explicit padding, so that a
reader can check the index conventions by eye. Pinned by tests against a
closed-form impulse response and by central finite differences.
"""
from __future__ import annotations

import numpy as np

CHANNELS = [(3, 32), (32, 32), (32, 32), (32, 1)]
DILATION = [1, 2, 4, 8]
N_PARAMS = sum(co * ci * 9 + co for ci, co in CHANNELS)


def unpack(params):
    """List of (w [co][ci][3][3], b [co]) views of the flat parameter vector."""
    out, o = [], 0
    for ci, co in CHANNELS:
        w = params[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = params[o:o + co]
        o += co
        out.append((w, b))
    assert o == len(params)
    return out


def shifted(x, di, dj):
    """x[..., i + di, (j + dj) mod W] with zeros where i + di leaves the rows."""
    H = x.shape[-2]
    y = np.roll(x, -dj, axis=-1)               # periodic in the column index
    out = np.zeros_like(x)
    if di >= 0:
        out[..., :H - di, :] = y[..., di:, :]
    else:
        out[..., -di:, :] = y[..., :H + di, :]
    return out


def conv(x, w, b, d=1):
    """x [B][ci][H][W] -> [B][co][H][W]: b[co] + sum w[co][ci][di+1][dj+1] x[ci][i+d di][j+d dj]."""
    B, _, H, W = x.shape
    co = w.shape[0]
    y = np.zeros((B, co, H, W)) + b[None, :, None, None]
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            xs = shifted(x, d * di, d * dj)
            y += np.einsum("oc,bchw->bohw", w[:, :, di + 1, dj + 1], xs)
    return y


def conv_adjoint(g, w, d=1):
    """Adjoint of conv in x: gx[ci][i][j] = sum w[co][ci][di+1][dj+1] g[co][i-d di][j-d dj]."""
    B, _, H, W = g.shape
    ci = w.shape[1]
    gx = np.zeros((B, ci, H, W))
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            gx += shifted(np.einsum("oc,bohw->bchw", w[:, :, di + 1, dj + 1], g), -d * di, -d * dj)
    return gx


def forward(params, x):
    """Returns (output [B][1][H][W], list of layer outputs after activation)."""
    layers = unpack(params)
    acts = []
    h = x
    for l, (w, b) in enumerate(layers):
        h = conv(h, w, b, DILATION[l])
        if l < 3:
            h = np.tanh(h)
        acts.append(h)
    return h, acts


def loss(params, x, target):
    out, _ = forward(params, x)
    return float(np.mean((out - target) ** 2))


def grad(params, x, target):
    """Gradient of the mean squared error by reverse-mode differentiation."""
    layers = unpack(params)
    out, acts = forward(params, x)
    n = out.size
    g = 2.0 * (out - target) / n
    grads = []
    for l in range(3, -1, -1):
        w, _ = layers[l]
        d = DILATION[l]
        xin = x if l == 0 else acts[l - 1]
        gw = np.zeros_like(w)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                gw[:, :, di + 1, dj + 1] = np.einsum("bohw,bchw->oc", g, shifted(xin, d * di, d * dj))
        gb = g.sum(axis=(0, 2, 3))
        grads.append((gw, gb))
        if l > 0:
            g = conv_adjoint(g, w, d) * (1.0 - acts[l - 1] ** 2)
    grads.reverse()
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def adam(params, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) with bias correction."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
