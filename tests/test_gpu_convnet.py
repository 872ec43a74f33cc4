"""The preconditioner network's GPU kernels (forward on MFMA with BF16
activations, MSE gradient, Adam) against the FP64 oracle, and flexible CG
with the network inside tomo_cg_solve."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

BF16_REL = 2.0 ** -8  # relative rounding of a BF16 value (RNE gives half of this)


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def flat(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def unflat(v):
    shapes = [(16, 1, 3, 3, 3), (16,), (16, 16, 3, 3, 3), (16,), (1, 16, 3, 3, 3), (1,)]
    out, k = [], 0
    for s in shapes:
        m = int(np.prod(s))
        out.append(np.asarray(v[k:k + m], dtype=np.float64).reshape(s))
        k += m
    return out


def rand_params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return unflat(scale * rng.normal(size=7809))


def _abs_params(params):
    return [np.abs(p) for p in params]


@pytest.mark.parametrize("shape", [(19, 21, 37), (16, 16, 16), (5, 9, 33)])
def test_forward_matches_oracle(tomo, ora, shape):
    """Per voxel: |GPU - oracle| <= 8 * 2^-8 * (the same network with |w|,
    |b| and |x|), i.e. a few BF16 roundings through three layers, relative to
    the magnitudes that enter each sum."""
    params = rand_params(1)
    x = np.random.default_rng(2).normal(size=shape)
    net = tomo.ConvNet(shape)
    got = to_host(net.forward(to_dev(flat(params)), to_dev(x)))
    ref = ora.convnet_forward(params, x)
    bound = 8 * BF16_REL * ora.convnet_forward(_abs_params(params), np.abs(x)) + 1e-6
    err = np.abs(got - ref)
    assert np.all(err <= bound), f"{np.count_nonzero(err > bound)} of {err.size} exceed"
    assert np.linalg.norm(got - ref) <= 2e-2 * np.linalg.norm(ref)


def test_identity_network(tomo, ora):
    """The exact identity weights give N(r) = r up to one BF16 rounding."""
    r = np.random.default_rng(3).normal(size=(12, 10, 20))
    net = tomo.ConvNet(r.shape)
    got = to_host(net.forward(to_dev(flat(ora.identity_net(1.0))), to_dev(r)))
    np.testing.assert_allclose(got, r, rtol=2 * BF16_REL, atol=1e-7)


def test_loss_gradient_matches_oracle(tomo, ora):
    """MSE loss and all parameter gradients against FP64, norm-wise per
    tensor (BF16 activations and gradients: a few 2^-8 relative)."""
    shape = (11, 13, 18)
    params = rand_params(4)
    rng = np.random.default_rng(5)
    x = rng.normal(size=shape)
    target = rng.normal(size=shape)
    net = tomo.ConvNet(shape)
    loss, grad = net.loss_grad(to_dev(flat(params)), to_dev(x), to_dev(target))
    ref_loss, ref_grads = ora.mse_loss_and_grad(params, x, target)
    assert abs(loss - ref_loss) <= 2e-2 * ref_loss
    got = unflat(to_host(grad))
    for k, (gg, rr) in enumerate(zip(got, ref_grads)):
        assert np.linalg.norm(gg - rr) <= 5e-2 * np.linalg.norm(rr) + 1e-7, f"tensor {k}"


def test_backward_with_given_output_gradient(tomo, ora):
    """tomo_convnet_backward with an arbitrary d loss / d out against the
    oracle's back-propagation of the same gradient (same bound as above)."""
    shape = (9, 14, 21)
    params = rand_params(11)
    rng = np.random.default_rng(12)
    x = rng.normal(size=shape)
    gout = rng.normal(size=shape)
    net = tomo.ConvNet(shape)
    got = unflat(to_host(net.backward(to_dev(flat(params)), to_dev(x), to_dev(gout))))
    _, acts = ora.convnet_forward(params, x, keep=True)
    ref = ora.convnet_backward(params, acts, gout)
    for k, (gg, rr) in enumerate(zip(got, ref)):
        assert np.linalg.norm(gg - rr) <= 5e-2 * np.linalg.norm(rr) + 1e-7, f"tensor {k}"


def test_adam_matches_oracle(tomo, ora):
    import torch

    params = rand_params(6)
    pv = flat(params).astype(np.float32)
    p_d = to_dev(pv)
    m_d = torch.zeros_like(p_d)
    v_d = torch.zeros_like(p_d)
    m = [np.zeros_like(q) for q in params]
    v = [np.zeros_like(q) for q in params]
    work = unflat(pv.astype(np.float64))
    rng = np.random.default_rng(7)
    for t in range(1, 6):
        gf = rng.normal(size=7809).astype(np.float32)
        tomo.adam_step(p_d, to_dev(gf), m_d, v_d, t)
        ora.adam_step(work, unflat(gf.astype(np.float64)), m, v, t)
    np.testing.assert_allclose(to_host(p_d), flat(work), rtol=1e-6, atol=1e-7)


def test_training_steps_reduce_the_loss(tomo, ora):
    """A few Adam steps on one (r, A^-1 r)-like pair lower the MSE."""
    import torch

    shape = (16, 16, 16)
    rng = np.random.default_rng(8)
    x = rng.normal(size=shape)
    target = 0.5 * x + 0.1 * rng.normal(size=shape)
    p = to_dev(flat(rand_params(9, 0.05)))
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    net = tomo.ConvNet(shape)
    xd, td = to_dev(x), to_dev(target)
    first = None
    for t in range(1, 41):
        loss, g = net.loss_grad(p, xd, td)
        first = loss if first is None else first
        tomo.adam_step(p, g, m, v, t, lr=3e-3)
    assert loss < 0.5 * first


# ---------------------------------------------------------- flexible CG


def _problem(ora):
    wl = ts.tiny()
    y = ora.project(wl.geom, wl.x).astype(np.float32).astype(np.float64)
    return wl, y


def test_fcg_identity_network_tracks_cg(tomo, ora):
    wl, y = _problem(ora)
    dg = tomo.DeviceGeometry(wl.geom)
    _, rep_cg = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=8)
    net = to_dev(flat(ora.identity_net(1.0)))
    _, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=8, precond=net)
    assert rep["fell_back"] == -1 and rep["status"] == 0
    # z = r up to BF16 rounding: the iterates stay close to plain CG's
    np.testing.assert_allclose(rep["history"], rep_cg["history"], rtol=5e-2)
    # and the FP64 oracle's FCG with the exact identity is plain CG
    _, h_ora = ora.cg(ora.normal_operator(wl.geom, wl.lam_r), ora.rhs(wl.geom, y), n_iter=8)
    np.testing.assert_allclose(rep["history"], h_ora, rtol=5e-2)


def test_fcg_falls_back_when_z_is_not_a_descent_direction(tomo, ora):
    """z = -r gives z.r < 0 at once: the solver switches to plain CG before
    the first step and then follows plain CG."""
    wl, y = _problem(ora)
    dg = tomo.DeviceGeometry(wl.geom)
    net = to_dev(flat(ora.identity_net(-1.0)))
    _, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=10, precond=net)
    _, rep_cg = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=10)
    assert rep["fell_back"] == 0
    np.testing.assert_allclose(rep["history"], rep_cg["history"], rtol=1e-4)


def test_fcg_falls_back_after_the_stall_window(tomo, ora):
    """min_drop = 0.99 (the residual must fall 100x per step) makes every
    iteration a stall, forced from the host: the switch happens after exactly
    fallback_window = 3 iterations and the solve still converges."""
    wl, y = _problem(ora)
    dg = tomo.DeviceGeometry(wl.geom)
    net = to_dev(flat(ora.identity_net(1.0)))
    _, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=200, rtol=1e-3, precond=net,
                           min_drop=0.99, fallback_window=3)
    assert rep["fell_back"] == 3
    assert rep["status"] == 0 and rep["true_rel_res"] <= 1.1e-3


def test_fcg_rejects_multi_frame_cubes(tomo, ora):
    wl, y = _problem(ora)
    g = wl.geom
    gf = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, np.zeros(g.nviews, np.int32), 2)
    dg = tomo.DeviceGeometry(gf)
    net = to_dev(flat(ora.identity_net(1.0)))
    with pytest.raises(tomo.TomoError):
        tomo.cg_solve(dg, to_dev(y), lam_r=1e-2, max_iter=2, precond=net)
