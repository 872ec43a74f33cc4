"""The autograd wrapper (forward P, backward P^T) on the differentiable
workload: 128^3 cube, 32 views of 256^2, lambda 1e-2."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import length_resolution, need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    tomo = need_gpu()
    import paper_1103_5904_amd.autograd as ag

    wl = ts.differentiable()
    dg = tomo.DeviceGeometry(wl.geom)
    return tomo, ag, wl, dg


def test_gradient_matches_oracle(setup, ora):
    """d/dx [0.5 ||P x - y||^2 + lambda ||D x||^2] = P^T (P x - y) + 2 lambda D^T D x,
    GPU autograd against the FP64 oracle per voxel.  Bound: the P^T bound
    (1e-4 of P^T|r|) plus the FP32 rounding of r (1e-6 of P^T(P|x| + |y|))
    plus 1e-5 of the prior's absolute stencil."""
    import torch

    tomo, ag, wl, dg = setup
    g = wl.geom
    xf = wl.x.astype(np.float32).astype(np.float64)
    y = ora.project(g, wl.extra["target_cube"]).astype(np.float32).astype(np.float64)
    x = to_dev(xf).requires_grad_(True)
    loss = ag.data_loss(x, dg, to_dev(y), wl.lam_r)
    loss.backward()
    got = to_host(x.grad)
    px = ora.project(g, xf)
    r = px - y
    ref = ora.backproject(g, r) + 2 * wl.lam_r * ora.laplacian6(xf)
    absx = np.abs(xf)
    # |(D^T D x)_v| <= 6 |x_v| + sum of |neighbours| (rolled copies over-count at the faces: still a bound)
    lap_abs = 6 * absx + sum(np.abs(np.roll(xf, s, a)) for a in range(3) for s in (1, -1))
    bound = (1e-4 * ora.backproject(g, np.abs(r)) + 1e-6 * ora.backproject(g, np.abs(px) + np.abs(y))
             + 1e-5 * 2 * wl.lam_r * lap_abs + length_resolution(g) * np.abs(r).max())
    err = np.abs(got - ref)
    assert np.all(err <= bound), f"{np.count_nonzero(err > bound)} voxels exceed the bound"
    # and the loss value itself
    ref_loss = 0.5 * float(r @ r) + wl.lam_r * sum(float(np.sum(np.diff(xf, axis=a) ** 2)) for a in range(3))
    assert abs(float(loss) - ref_loss) <= 1e-5 * ref_loss


def test_gradient_central_differences(setup, ora):
    """Central differences of the loss on 64 random voxels (h = 1e-3).  The
    loss is quadratic, so (L(x+h e) - L(x-h e)) / 2h equals the gradient up to
    rounding; only pixels whose rays cross voxel v change between the two
    evaluations, and their FP32 rounding bounds the error at ~1e-4 relative."""
    import torch

    tomo, ag, wl, dg = setup
    g = wl.geom
    y = to_dev(ora.project(g, wl.extra["target_cube"]))
    x = to_dev(wl.x).requires_grad_(True)
    ag.data_loss(x, dg, y, wl.lam_r).backward()
    grad = x.grad.detach().reshape(-1)
    rng = np.random.default_rng(600)
    nz, ny, nx = dg.cube_shape
    # voxels inside the region the views see, so the data term matters
    idx = rng.integers(0, g.nvox, 64)
    h = 1e-3
    worst = 0.0
    with torch.no_grad():
        xf = x.detach().reshape(-1)
        for v in idx:
            xp = xf.clone()
            xp[v] += h
            xm = xf.clone()
            xm[v] -= h
            lp = float(ag.data_loss(xp.reshape(dg.cube_shape), dg, y, wl.lam_r))
            lm = float(ag.data_loss(xm.reshape(dg.cube_shape), dg, y, wl.lam_r))
            fd = (lp - lm) / (2 * h)
            an = float(grad[v])
            scale = max(abs(an), 1e-3 * float(grad.abs().max()))
            worst = max(worst, abs(fd - an) / scale)
    assert worst <= 2e-3


def test_adjoint_identity_100_pairs(setup):
    """<P x, y> = <x, P^T y> on 100 random (x, y) pairs at full size."""
    import torch

    tomo, ag, wl, dg = setup
    g = wl.geom
    worst = 0.0
    for seed in range(500, 600):
        x, y = ts.random_pair(g.nvox, g.nrays, seed)
        xd, yd = to_dev(x), to_dev(y)
        px = tomo.project(dg, xd).double()
        pty = tomo.backproject(dg, yd).double()
        lhs = float(torch.dot(px, yd.double()))
        rhs = float(torch.dot(xd.double().ravel(), pty.ravel()))
        worst = max(worst, abs(lhs - rhs) / (float(torch.linalg.norm(px)) * float(np.linalg.norm(y))))
    assert worst <= 1e-5


def test_backward_of_a_composite(setup):
    """Autograd composes: d/dx sum(w * P x) = P^T w."""
    import torch

    tomo, ag, wl, dg = setup
    w = to_dev(np.random.default_rng(9).normal(size=wl.geom.nrays))
    x = to_dev(wl.x).requires_grad_(True)
    (ag.project(x, dg) * w).sum().backward()
    ref = tomo.backproject(dg, w)
    torch.cuda.synchronize()
    assert torch.allclose(x.grad, ref, rtol=1e-5, atol=1e-6 * float(ref.abs().max()))


def test_height_prior_and_gains(setup, ora):
    """The loss with two instruments (gains 0.7 and 1.6) and the
    height-weighted prior on the tiny problem: value against the oracle's
    criterion terms and gradient against its normal equations,
    grad = P^T G (G P x - y) + 2 lambda R D^T D R x."""
    tomo, ag, _, _ = setup
    wl = ts.tiny()
    g = wl.geom.subset(np.arange(wl.geom.nviews))
    g.gains = np.where(np.arange(g.nviews) < 4, 0.7, 1.6)
    h = (0.0, 0.0, 0.0, 0.0)
    dg = tomo.DeviceGeometry(g)
    xf = (wl.x * 1.1).astype(np.float32).astype(np.float64)
    y = ora.project(g, wl.x).astype(np.float32).astype(np.float64)
    x = to_dev(xf).requires_grad_(True)
    loss = ag.data_loss(x, dg, to_dev(y), wl.lam_r, height=h)
    loss.backward()
    got = to_host(x.grad)
    ref = ora.normal_operator(g, 2.0 * wl.lam_r, height=h)(xf) - ora.rhs(g, y)
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    r = ora.project(g, xf) - y
    hv = ora.voxel_heights(g, h)
    ref_loss = 0.5 * float(r @ r) + wl.lam_r * sum(float(np.sum(np.diff(hv * xf, axis=a) ** 2)) for a in range(3))
    assert abs(float(loss) - ref_loss) <= 1e-5 * ref_loss
