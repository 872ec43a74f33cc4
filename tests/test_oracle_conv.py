"""Pins for the oracle's 3-D convolution network and Adam step: library
routines (torch, float64, CPU) and central finite differences."""
import numpy as np
import pytest
import torch

import tomo_synth as ts  # noqa: F401  (keeps import order identical to other tests)


def _rand_net(rng, scale=0.2):
    shapes = [(16, 1, 3, 3, 3), (16,), (16, 16, 3, 3, 3), (16,), (1, 16, 3, 3, 3), (1,)]
    return [scale * rng.normal(size=s) for s in shapes]


@pytest.mark.parametrize("cin,cout,shape", [(1, 16, (5, 6, 7)), (16, 16, (4, 3, 5)), (16, 1, (6, 5, 4))])
def test_conv3d_matches_torch(ora, cin, cout, shape):
    rng = np.random.default_rng(cin * 100 + cout)
    x = rng.normal(size=(cin,) + shape)
    w = rng.normal(size=(cout, cin, 3, 3, 3))
    b = rng.normal(size=cout)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x)[None], torch.from_numpy(w),
                                     torch.from_numpy(b), padding=1)[0].numpy()
    np.testing.assert_allclose(ora.conv3d(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_conv3d_backward_matches_autograd(ora):
    rng = np.random.default_rng(3)
    x = rng.normal(size=(16, 4, 5, 6))
    w = rng.normal(size=(16, 16, 3, 3, 3))
    gout = rng.normal(size=(16, 4, 5, 6))
    tx = torch.from_numpy(x).requires_grad_(True)
    tw = torch.from_numpy(w).requires_grad_(True)
    tb = torch.zeros(16, dtype=torch.float64, requires_grad=True)
    out = torch.nn.functional.conv3d(tx[None], tw, tb, padding=1)[0]
    out.backward(torch.from_numpy(gout))
    gin, gw, gb = ora.conv3d_backward(x, w, gout)
    np.testing.assert_allclose(gin, tx.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gw, tw.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gb, tb.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_convnet_gradient_finite_differences(ora):
    """Parameter gradients of the MSE loss through the whole network against
    central differences (FP64)."""
    rng = np.random.default_rng(9)
    params = _rand_net(rng)
    r = rng.normal(size=(5, 4, 6))
    target = rng.normal(size=(5, 4, 6))
    _, grads = ora.mse_loss_and_grad(params, r, target)
    h = 1e-6
    for _ in range(24):
        k = rng.integers(0, len(params))
        flat = params[k].reshape(-1)
        j = rng.integers(0, flat.size)
        old = flat[j]
        flat[j] = old + h
        lp, _ = ora.mse_loss_and_grad(params, r, target)
        flat[j] = old - h
        lm, _ = ora.mse_loss_and_grad(params, r, target)
        flat[j] = old
        fd = (lp - lm) / (2 * h)
        an = grads[k].reshape(-1)[j]
        assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)), (k, j, fd, an)


def test_convnet_forward_matches_torch(ora):
    rng = np.random.default_rng(4)
    params = _rand_net(rng)
    r = rng.normal(size=(6, 5, 7))
    t = [torch.from_numpy(p) for p in params]
    h = torch.from_numpy(r)[None, None]
    h = torch.relu(torch.nn.functional.conv3d(h, t[0], t[1], padding=1))
    h = torch.relu(torch.nn.functional.conv3d(h, t[2], t[3], padding=1))
    h = torch.nn.functional.conv3d(h, t[4], t[5], padding=1)[0, 0].numpy()
    np.testing.assert_allclose(ora.convnet_forward(params, r), h, rtol=1e-12, atol=1e-12)


def test_adam_matches_torch(ora):
    rng = np.random.default_rng(2)
    params = _rand_net(rng)
    tparams = [torch.from_numpy(p.copy()).requires_grad_(True) for p in params]
    opt = torch.optim.Adam(tparams, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    for t in range(1, 6):
        grads = [rng.normal(size=p.shape) for p in params]
        for tp, g in zip(tparams, grads):
            tp.grad = torch.from_numpy(g.copy())
        opt.step()
        ora.adam_step(params, grads, m, v, t)
        for p, tp in zip(params, tparams):
            np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)
