"""Pins of the FP64 warm-start network reference (oracle/wsnet.py): parameter
count, closed-form impulse response with the padding rules, adjoint identity,
finite-difference gradients, first Adam step."""
import numpy as np
import pytest

from oracle import wsnet as N


def test_parameter_count():
    # 3*32*9+32 + 2*(32*32*9+32) + 32*9+1
    assert N.N_PARAMS == 19681


def test_impulse_response_padding():
    """One 3x3 layer on a unit impulse at the wall row, column 0: the output is the
    flipped stencil, wrapped across the periodic column seam and cut at the wall."""
    rng = np.random.default_rng(0)
    H, W = 6, 8
    w = rng.standard_normal((1, 1, 3, 3))
    x = np.zeros((1, 1, H, W))
    x[0, 0, 0, 0] = 1.0
    y = N.conv(x, w, np.zeros(1))[0, 0]
    expect = np.zeros((H, W))
    expect[0, 0] = w[0, 0, 1, 1]
    expect[0, 1] = w[0, 0, 1, 0]
    expect[0, W - 1] = w[0, 0, 1, 2]
    expect[1, 0] = w[0, 0, 0, 1]
    expect[1, 1] = w[0, 0, 0, 0]
    expect[1, W - 1] = w[0, 0, 0, 2]
    assert np.array_equal(y, expect)


def test_dilated_impulse_response():
    """Taps spaced d = 2 apart: the impulse at the wall row, column 1, lands on
    columns 3 and (1 - 2) mod W = W - 1 and on row 2; the taps reaching row -2 are cut."""
    rng = np.random.default_rng(3)
    H, W = 7, 8
    w = rng.standard_normal((1, 1, 3, 3))
    x = np.zeros((1, 1, H, W))
    x[0, 0, 0, 1] = 1.0
    y = N.conv(x, w, np.zeros(1), d=2)[0, 0]
    expect = np.zeros((H, W))
    expect[0, 1] = w[0, 0, 1, 1]
    expect[0, W - 1] = w[0, 0, 1, 2]          # y[j] picks x[j + 2]: j = W - 1 wraps to column 1
    expect[0, 3] = w[0, 0, 1, 0]
    expect[2, 1] = w[0, 0, 0, 1]
    expect[2, W - 1] = w[0, 0, 0, 2]
    expect[2, 3] = w[0, 0, 0, 0]
    assert np.array_equal(y, expect)
    assert N.DILATION == [1, 2, 4, 8]


@pytest.mark.parametrize("d", [1, 2, 4])
def test_adjoint_identity(d):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 9, 8))
    g = rng.standard_normal((2, 4, 9, 8))
    w = rng.standard_normal((4, 3, 3, 3))
    lhs = np.sum(N.conv(x, w, np.zeros(4), d) * g)
    rhs = np.sum(x * N.conv_adjoint(g, w, d))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gradient_finite_differences():
    rng = np.random.default_rng(2)
    p = 0.1 * rng.standard_normal(N.N_PARAMS)
    x = rng.standard_normal((2, 3, 10, 16))        # larger than the last layer's tap spacing
    t = rng.standard_normal((2, 1, 10, 16))
    g = N.grad(p, x, t)
    idx = rng.choice(N.N_PARAMS, 40, replace=False)
    idx = np.concatenate([idx, [0, 864, 895, N.N_PARAMS - 1]])    # first weight, layer-1 biases, last bias
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (N.loss(p + e, x, t) - N.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = N.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p, -0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8))
