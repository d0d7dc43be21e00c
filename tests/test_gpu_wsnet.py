"""The warm-start network kernels (qtt_ws_*) against the FP64 reference
oracle/wsnet.py: forward (FP32 and BF16 operands), squared-error gradient,
backward, Adam, and a short training run."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _setup(B=2, seed=0):
    import torch
    from paper_2507_05222_amd import qtt as Q, warmstart as W
    rng = np.random.default_rng(seed)
    ctx = Q.Context(0)
    p = W.init_params(seed) + 0.01 * rng.standard_normal(W.NPARAMS).astype(np.float32)
    x = rng.standard_normal((B, 3, 64, 64)).astype(np.float32)
    t = rng.standard_normal((B, 1, 64, 64)).astype(np.float32)
    net = W.Net(ctx, p)
    return torch, net, p.astype(np.float64), x, t


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_forward_matches_reference():
    from oracle import wsnet as N
    torch, net, p, x, _ = _setup()
    out, _ = net.forward(torch.from_numpy(x).cuda())
    ref, _ = N.forward(p, x.astype(np.float64))
    assert _rel(out.cpu().numpy(), ref) < 1e-5


def test_forward_bf16_within_budget():
    from oracle import wsnet as N
    torch, net, p, x, _ = _setup()
    out, _ = net.forward(torch.from_numpy(x).cuda(), bf16=True)
    ref, _ = N.forward(p, x.astype(np.float64))
    assert _rel(out.cpu().numpy(), ref) < 3e-2


def test_backward_matches_reference():
    from oracle import wsnet as N
    torch, net, p, x, t = _setup()
    loss = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    assert abs(loss - N.loss(p, x.astype(np.float64), t.astype(np.float64))) < 1e-5 * loss
    g = net.grads.cpu().numpy()
    gr = N.grad(p, x.astype(np.float64), t.astype(np.float64))
    assert _rel(g, gr) < 1e-4
    # every layer separately (the last layer's gradient dominates the norm)
    o = 0
    for ci, co in N.CHANNELS:
        k = co * ci * 9 + co
        assert _rel(g[o:o + k], gr[o:o + k]) < 1e-4, (ci, co)
        o += k


def test_adam_matches_reference():
    from oracle import wsnet as N
    torch, net, p, x, t = _setup()
    net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads.cpu().numpy().astype(np.float64)
    net.adam(1e-3)
    net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g2 = net.grads.cpu().numpy().astype(np.float64)
    net.adam(1e-3)
    q, m, v = N.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    q, m, v = N.adam(q, g2, m, v, 2, 1e-3)
    assert _rel(net.numpy_params(), q) < 1e-6


def test_training_reduces_loss():
    torch, net, p, x, _ = _setup(B=4, seed=3)
    xs = torch.from_numpy(x).cuda()
    # a smooth target that depends on the input: the local average of channel 0
    t = torch.nn.functional.avg_pool2d(xs[:, :1], 3, stride=1, padding=1)
    first = net.loss_grad(xs, t)
    for _ in range(60):
        net.loss_grad(xs, t)
        net.adam(3e-3)
    last = net.loss_grad(xs, t)
    assert last < 0.5 * first, (first, last)
