"""Host-side pieces of the preconditioner training: the exact network forms
of a linear filter and of the identity, and the linear-filter fit in the
energy norm, pinned against the FP64 oracle's network and a brute-force
minimisation on a tiny volume (no GPU)."""
import numpy as np
import pytest
import torch
from scipy import ndimage, optimize

from paper_1103_5904_amd import precond as pc


def unflat(v):
    out, k = [], 0
    for s in pc.SHAPES:
        m = int(np.prod(s))
        out.append(np.asarray(v[k:k + m], dtype=np.float64).reshape(s))
        k += m
    return out


def test_parameter_layout_matches_the_abi():
    assert sum(int(np.prod(s)) for s in pc.SHAPES) == 7809


@pytest.mark.parametrize("seed", [0, 1])
def test_linear_filter_params_is_exactly_the_filter(ora, seed):
    """The oracle's FP64 forward pass of linear_filter_params(h) is the zero-
    padded 3x3x3 cross-correlation with h (scipy), for signed h."""
    rng = np.random.default_rng(seed)
    h = rng.normal(size=(3, 3, 3))
    r = rng.normal(size=(7, 9, 11))
    got = ora.convnet_forward(unflat(pc.linear_filter_params(h)), r)
    ref = ndimage.correlate(r, h, mode="constant", cval=0.0)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_identity_params(ora):
    r = np.random.default_rng(2).normal(size=(5, 6, 7))
    got = ora.convnet_forward(unflat(pc.identity_params(0.37)), r)
    np.testing.assert_allclose(got, 0.37 * r, rtol=1e-13, atol=1e-15)


def test_tap_input_is_the_padded_shift():
    r = torch.randn(5, 6, 7, dtype=torch.float64)
    out = torch.empty_like(r)
    rp = torch.nn.functional.pad(r, (1, 1, 1, 1, 1, 1))
    for t in range(27):
        kz, ky, kx = t // 9, (t // 3) % 3, t % 3
        assert torch.equal(pc._tap_input(r, t, out), rp[kz:kz + 5, ky:ky + 6, kx:kx + 7])


def _tiny_spd(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.normal(size=(n, n))
    return B @ B.T / n + 0.5 * np.eye(n)


def test_linear_filter_fit_minimises_the_energy_error():
    """On a 4x5x6 volume with a random SPD matrix as A: the fitted filter is
    centro-symmetric, and no centro-symmetric filter found by a general
    minimiser (BFGS over the 14 free taps, brute-force energy from scipy's
    correlate and a dense solve for A^-1 r) has a lower energy-norm error
    sum_k ||h * r_k - A^-1 r_k||_A^2."""
    shape = (4, 5, 6)
    n = int(np.prod(shape))
    A = _tiny_spd(n, 3)
    rng = np.random.default_rng(4)
    rs = rng.normal(size=(3,) + shape)
    rs /= np.linalg.norm(rs.reshape(3, -1), axis=1)[:, None, None, None]

    def apply(v, out):
        out.copy_(torch.as_tensor(A @ v.reshape(-1).numpy()).reshape(v.shape))
        return out

    h = pc.fit_linear_filter(apply, torch.as_tensor(rs))
    np.testing.assert_allclose(h, h[::-1, ::-1, ::-1], rtol=0, atol=1e-12)
    e = [np.linalg.solve(A, r.reshape(-1)) for r in rs]

    def err(hf):
        tot = 0.0
        for r, ek in zip(rs, e):
            d = ndimage.correlate(r, hf.reshape(3, 3, 3), mode="constant").reshape(-1) - ek
            tot += d @ A @ d
        return tot

    E = np.zeros((27, 14))
    for t in range(27):
        E[t, min(t, 26 - t)] = 1.0
    best = optimize.minimize(lambda u: err(E @ u), np.zeros(14), method="BFGS", options={"gtol": 1e-10})
    assert err(h.ravel()) <= best.fun * (1 + 1e-9) + 1e-12
    np.testing.assert_allclose(h.ravel(), E @ best.x, rtol=1e-4, atol=1e-5)
