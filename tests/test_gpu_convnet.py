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


GRAD_C = 2  # BF16 roundings allowed per gradient element (see _grad_bounds)


def _grad_bounds(ora, params, x, gabs_out):
    """Per-element magnitudes that bound the rounding of every parameter
    gradient: the forward and the back-propagation taken with |weights|,
    |biases|, |x| and a non-negative output-gradient magnitude, every ReLU
    replaced by the identity.  Each GPU gradient element is a sum over voxels
    of (data gradient) x (activation) products whose factors carry a few BF16
    roundings (2^-9 relative each, round to nearest: the stored activations,
    the stored data gradients, the forward's error), and the roundings of
    independent terms partly cancel, so its error stays within GRAD_C x 2^-8
    of the same sum taken over magnitudes (measured: 0.06 of that bound at
    worst); with the ReLUs as identities, a mask that rounding flips next to
    zero is covered too."""
    w1, b1, w2, b2, w3, b3 = [np.abs(p) for p in params]
    a0 = np.abs(np.asarray(x, dtype=np.float64))[None]
    a1 = ora.conv3d(a0, w1, b1)
    a2 = ora.conv3d(a1, w2, b2)
    g2, gw3, gb3 = ora.conv3d_backward(a2, w3, np.asarray(gabs_out, dtype=np.float64)[None])
    g1, gw2, gb2 = ora.conv3d_backward(a1, w2, g2)
    _, gw1, gb1 = ora.conv3d_backward(a0, w1, g1)
    return [gw1, gb1, gw2, gb2, gw3, gb3]


def _assert_grads_close(got, ref, mag, what):
    names = ["w1", "b1", "w2", "b2", "w3", "b3"]
    worst = 0.0
    for name, gg, rr, mm in zip(names, got, ref, mag):
        bound = GRAD_C * BF16_REL * mm + 1e-12
        err = np.abs(gg - rr)
        bad = err > bound
        worst = max(worst, float(np.max(err / bound)))
        if np.any(bad):
            k = np.unravel_index(np.argmax(err / bound), err.shape)
            raise AssertionError(f"{what} {name}: {np.count_nonzero(bad)} of {err.size} elements exceed "
                                 f"{GRAD_C} x 2^-8 of their magnitude sum; worst at {k}: gpu {gg[k]!r} "
                                 f"oracle {rr[k]!r} bound {bound[k]:.3e}")
    print(f"{what}: worst error / bound = {worst:.3f}", flush=True)


@pytest.mark.parametrize("shape,seed", [((11, 13, 18), 4), ((16, 16, 16), 14), ((7, 20, 33), 24)])
def test_loss_gradient_matches_oracle(tomo, ora, shape, seed):
    """MSE loss and every parameter-gradient element against FP64: the
    output gradient 2 (N(x) - t) / n carries the forward's error (at most
    8 x 2^-8 of the |.|-network, as the forward test bounds it), so its
    magnitude is 2 / n (|N(x) - t| + |.|-network), back-propagated as in
    _grad_bounds."""
    params = unflat(flat(rand_params(seed)).astype(np.float32))
    rng = np.random.default_rng(seed + 1)
    x = rng.normal(size=shape).astype(np.float32).astype(np.float64)
    target = rng.normal(size=shape).astype(np.float32).astype(np.float64)
    net = tomo.ConvNet(shape)
    loss, grad = net.loss_grad(to_dev(flat(params)), to_dev(x), to_dev(target))
    ref_loss, ref_grads = ora.mse_loss_and_grad(params, x, target)
    assert abs(loss - ref_loss) <= 2e-2 * ref_loss
    out_ref = ora.convnet_forward(params, x)
    out_abs = ora.convnet_forward(_abs_params(params), np.abs(x))
    gmag = 2.0 / x.size * (np.abs(out_ref - target) + 8 * BF16_REL * out_abs)
    _assert_grads_close(unflat(to_host(grad)), ref_grads, _grad_bounds(ora, params, x, gmag), "loss_grad")


@pytest.mark.parametrize("shape,seed", [((9, 14, 21), 11), ((12, 12, 40), 31)])
def test_backward_with_given_output_gradient(tomo, ora, shape, seed):
    """tomo_convnet_backward with an arbitrary d loss / d out against the
    oracle's back-propagation of the same gradient, element by element."""
    params = unflat(flat(rand_params(seed)).astype(np.float32))
    rng = np.random.default_rng(seed + 1)
    x = rng.normal(size=shape).astype(np.float32).astype(np.float64)
    gout = rng.normal(size=shape).astype(np.float32).astype(np.float64)
    net = tomo.ConvNet(shape)
    got = unflat(to_host(net.backward(to_dev(flat(params)), to_dev(x), to_dev(gout))))
    _, acts = ora.convnet_forward(params, x, keep=True)
    ref = ora.convnet_backward(params, acts, gout)
    _assert_grads_close(got, ref, _grad_bounds(ora, params, x, np.abs(gout)), "backward")


@pytest.mark.timeout(600)
def test_backward_at_training_size(tomo, ora):
    """Once at the training volume, 128^3, with the shipped network: the
    energy-norm training gradient's path (tomo_convnet_backward) element by
    element against the FP64 oracle, on a smooth unit-norm residual-like
    input (a blob field minus its mean)."""
    import os

    from paper_1103_5904_amd import precond as pc

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pflat = pc.load(os.path.join(root, "paper_1103_5904_amd", "precond_weights.npz"))
    pflat = pflat.detach().cpu().numpy().astype(np.float64)
    params = unflat(pflat)
    shape = (128, 128, 128)
    wl = ts.learned(2003)
    x = wl.x - wl.x.mean()
    x = (x / np.linalg.norm(x)).astype(np.float32).astype(np.float64)
    gout = np.random.default_rng(77).normal(size=shape).astype(np.float32).astype(np.float64) / 128.0 ** 1.5
    net = tomo.ConvNet(shape)
    got = unflat(to_host(net.backward(to_dev(pflat), to_dev(x), to_dev(gout))))
    _, acts = ora.convnet_forward(params, x, keep=True)
    ref = ora.convnet_backward(params, acts, gout)
    _assert_grads_close(got, ref, _grad_bounds(ora, params, x, np.abs(gout)), "backward 128^3")


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


def _bf16(a):
    """Round to BF16 (nearest, ties to even) through FP32, as the network's
    stored activations are."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    b = ((b + np.uint32(0x7FFF) + ((b >> 16) & np.uint32(1))) & np.uint32(0xFFFF0000)).astype(np.uint32)
    return b.view(np.float32).astype(np.float64)


def test_fcg_identity_network_tracks_cg(tomo, ora):
    """The exact identity weights make the network return its input rounded
    to BF16 (the stored activations), so the GPU's flexible CG is flexible CG
    with z = s bf16(r / s), s = ||r||: a preconditioner within 2^-9 of the
    identity.  Run in FP64, that model's residual history stays within
    0.54 x 2^-8 of plain CG's over these 8 iterations (the Polak-Ribiere
    recurrence amplifies the roundings, chaotically, to that size).  The GPU
    run realises the same roundings with FP32 vectors, so its history must
    lie within 2^-8 of the model's and within 2 x 2^-8 of plain CG's."""
    wl, y = _problem(ora)
    dg = tomo.DeviceGeometry(wl.geom)
    net = to_dev(flat(ora.identity_net(1.0)))
    _, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=8, precond=net)
    assert rep["fell_back"] == -1 and rep["status"] == 0
    A, b = ora.normal_operator(wl.geom, wl.lam_r), ora.rhs(wl.geom, y)

    def bf16_identity(r):
        s = float(np.sqrt(np.vdot(r, r)))
        return s * _bf16(r / s)

    _, h_model, fb = ora.fcg(A, b, bf16_identity, n_iter=8)
    assert fb == -1
    _, h_cg = ora.cg(A, b, n_iter=8)
    assert np.max(np.abs(h_model / h_cg - 1.0)) <= 0.6 * BF16_REL  # the model's own distance from CG
    dev_model = np.max(np.abs(rep["history"] / h_model - 1.0))
    dev_cg = np.max(np.abs(rep["history"] / h_cg - 1.0))
    print(f"FCG identity: deviation from the BF16 model {dev_model:.2e}, from plain CG {dev_cg:.2e}", flush=True)
    assert dev_model <= BF16_REL
    assert dev_cg <= 2 * BF16_REL


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
    assert rep["status"] == 0 and rep["true_rel_res"] <= 1e-3


def test_fcg_rejects_multi_frame_cubes(tomo, ora):
    wl, y = _problem(ora)
    g = wl.geom
    gf = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, np.zeros(g.nviews, np.int32), 2)
    dg = tomo.DeviceGeometry(gf)
    net = to_dev(flat(ora.identity_net(1.0)))
    with pytest.raises(tomo.TomoError):
        tomo.cg_solve(dg, to_dev(y), lam_r=1e-2, max_iter=2, precond=net)
