"""Training and evaluation of the learned CG preconditioner.

The paper names preconditioning as the untried remedy for slow CG
convergence (Sec. "Smooth Temporal Evolution").  Here a small 3-D
convolution network N stands in for the inverse of the normal operator
A = P^T P + lambda D^T D (Eq. stsrt) on residuals.

Training pairs come from the library's own plain CG: for iterate k of a
solve, the unit residual r_k / ||r_k|| and the CG correction
(x* - x_k) / ||r_k||, where x* is the same CG run to a tight tolerance.  The
network is fitted in the energy norm of A,

    L(z) = 0.5 (z - e)^T A (z - e),   z = N(r),

the error norm CG itself minimises, whose output gradient A (z - e) costs one
P and one P^T.  A Euclidean fit to e weights the smooth, weakly determined
modes of A^-1 above everything else, which no 3x3x3 stack can represent,
and gives a worse preconditioner than the identity.  Flexible CG then uses
z = ||r|| N(r / ||r||) (tomo_cg_solve with precond).

All arithmetic of the network, its gradient, the optimiser and A runs in
libtomo; this module schedules calls and does the few vector subtractions
and norms that glue them.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import tomo as _t

SHAPES = [(16, 1, 3, 3, 3), (16,), (16, 16, 3, 3, 3), (16,), (1, 16, 3, 3, 3), (1,)]


def identity_params(scale: float = 1.0) -> np.ndarray:
    """Flat parameters for which N(r) = scale * r exactly: the first layer
    splits r into (r, -r), the ReLUs keep r+ and r-, the middle layer passes
    them through and the last recombines scale * (r+ - r-)."""
    w1 = np.zeros(SHAPES[0])
    w1[0, 0, 1, 1, 1], w1[1, 0, 1, 1, 1] = 1.0, -1.0
    w2 = np.zeros(SHAPES[2])
    w2[0, 0, 1, 1, 1] = w2[1, 1, 1, 1, 1] = 1.0
    w3 = np.zeros(SHAPES[4])
    w3[0, 0, 1, 1, 1], w3[0, 1, 1, 1, 1] = scale, -scale
    return np.concatenate([w1.ravel(), np.zeros(16), w2.ravel(), np.zeros(16), w3.ravel(), np.zeros(1)])


class NormalOperator:
    """out = (P^T P + lambda D^T D) v on a one-frame geometry without masks,
    from tomo_project, tomo_backproject and tomo_apply_prior."""

    def __init__(self, dg: _t.DeviceGeometry, lam: float):
        if dg.nframes != 1 or dg.data_mask is not None or dg.map_mask is not None:
            raise ValueError("preconditioner training needs one frame and no masks")
        self.dg, self.lam = dg, float(lam)
        self.img = torch.empty(dg.npix, dtype=torch.float32, device="cuda")

    def __call__(self, v: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        _t.project(self.dg, v, out=self.img)
        _t.backproject(self.dg, self.img, out=out)
        _t.apply_prior(self.dg, v, self.lam, out=out, accumulate=True)
        return out


def linear_filter_params(h) -> np.ndarray:
    """Flat parameters for which N(r) = h * r exactly, for any 3x3x3 filter h
    (cross-correlation, zero padding): the first layer splits r into r+ and
    r-, the middle layer applies the positive and negative parts of h to each
    (four non-negative channels, which the ReLU leaves alone) and the last
    recombines h+ r+ - h- r+ - h+ r- + h- r-."""
    h = np.asarray(h, dtype=np.float64).reshape(3, 3, 3)
    hp, hm = np.maximum(h, 0.0), np.maximum(-h, 0.0)
    w1 = np.zeros(SHAPES[0])
    w1[0, 0, 1, 1, 1], w1[1, 0, 1, 1, 1] = 1.0, -1.0
    w2 = np.zeros(SHAPES[2])
    w2[0, 0], w2[1, 0], w2[2, 1], w2[3, 1] = hp, hm, hp, hm
    w3 = np.zeros(SHAPES[4])
    w3[0, 0:4, 1, 1, 1] = [1.0, -1.0, -1.0, 1.0]
    return np.concatenate([w1.ravel(), np.zeros(16), w2.ravel(), np.zeros(16), w3.ravel(), np.zeros(1)])


def _tap_input(r: torch.Tensor, t: int, out: torch.Tensor) -> torch.Tensor:
    """out[z, y, x] = r[z + dz, y + dy, x + dx] (zero outside the volume), the
    value tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) of a zero-padded 3x3x3
    cross-correlation reads; a pure copy."""
    dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
    n = r.shape
    out.zero_()
    src = tuple(slice(max(o, 0), m + min(o, 0)) for o, m in zip((dz, dy, dx), n))
    dst = tuple(slice(max(-o, 0), m + min(-o, 0)) for o, m in zip((dz, dy, dx), n))
    out[dst] = r[src]
    return out


def fit_linear_filter(A, residuals: torch.Tensor) -> np.ndarray:
    """The 3x3x3 filter h (centro-symmetric, so that r -> h * r is a
    symmetric operator) minimising sum_k ||h * r_k - A^-1 r_k||_A^2 over unit
    residuals r_k: the normal equations G h = c with
    G_ij = sum_k (S_i r_k)^T A (S_j r_k) and c_i = sum_k (S_i r_k)^T r_k, S_t the
    tap-t copy.  A(v, out) writes A v into out (a NormalOperator, or any
    symmetric positive definite operator on the residuals' device); costs 27
    applications of A per residual.  An offline step of training (run once
    by train_precond before the Adam steps), not part of any solve: its Gram
    products are plain torch GEMMs on the device, outside the library."""
    shape = residuals.shape[1:]
    S = torch.empty((27,) + tuple(shape), dtype=residuals.dtype, device=residuals.device)
    AS = torch.empty_like(S)
    G = np.zeros((27, 27))
    c = np.zeros(27)
    for r in residuals:
        for t in range(27):
            _tap_input(r, t, S[t])
            A(S[t], AS[t])
        Sf = S.reshape(27, -1).double()
        G += (Sf @ AS.reshape(27, -1).double().T).cpu().numpy()
        c += (Sf @ r.reshape(-1).double()).cpu().numpy()
    # centro-symmetric taps: h_t = h_{26 - t}; solve in the 14 free values
    E = np.zeros((27, 14))
    for t in range(27):
        E[t, min(t, 26 - t)] = 1.0
    Gs = E.T @ (0.5 * (G + G.T)) @ E
    return (E @ np.linalg.solve(Gs, E.T @ c)).reshape(3, 3, 3)


def noisy_data(dg: _t.DeviceGeometry, x_true: torch.Tensor, rel: float, seed: int) -> torch.Tensor:
    """y = P x + n with n ~ N(0, (rel * rms(P x))^2), drawn on the host from
    the seed (inputs, not method arithmetic)."""
    y = _t.project(dg, x_true)
    rms = float(torch.sqrt(torch.mean(y.double() ** 2)))
    noise = np.random.default_rng(seed).normal(0.0, rel * rms, dg.npix).astype(np.float32)
    return y + torch.as_tensor(noise, device=y.device)


def solve_pairs(dg: _t.DeviceGeometry, y: torch.Tensor, lam: float, k_record: int = 40,
                n_star: int = 300, rtol_star: float = 1e-6):
    """Training pairs from one problem: (r_k/||r_k||, (x* - x_k)/||r_k||),
    k = 0..k_record-1, on the volume's shape."""
    x_star, _ = _t.cg_solve(dg, y, lam_r=lam, max_iter=n_star, rtol=rtol_star, check_every=25)
    nv = dg.nvox
    rx = torch.empty((k_record, nv), dtype=torch.float32, device=y.device)
    rr = torch.empty((k_record, nv), dtype=torch.float32, device=y.device)
    _t.cg_solve(dg, y, lam_r=lam, max_iter=k_record - 1, record_x=rx, record_r=rr)
    norms = torch.linalg.norm(rr.double(), dim=1).clamp_min(1e-300)
    inv = (1.0 / norms).float()[:, None]
    inputs = (rr * inv).reshape((k_record,) + dg.cube_shape)
    targets = ((x_star.reshape(1, -1) - rx) * inv).reshape((k_record,) + dg.cube_shape)
    return inputs, targets


def train(dg: _t.DeviceGeometry, lam: float, inputs: torch.Tensor, targets: torch.Tensor,
          epochs: int = 2, lr: float = 3e-4, lr_final: float = 3e-5, seed: int = 0, log=None,
          init: np.ndarray | None = None, fit_pairs: slice = slice(0, 40, 4)):
    """Adam on the energy-norm error over the pairs (one pair per step, in a
    seeded random order, cosine learning-rate decay from lr to lr_final).
    Starts from the network form of the best linear 3x3x3 filter in the same
    norm (fit_linear_filter on the pairs fit_pairs selects), with 1e-3
    Gaussian noise on its zero weights so the spare channels can take part.
    Returns (params, energy-loss trace)."""
    A = NormalOperator(dg, lam)
    npairs = inputs.shape[0]
    shape = inputs.shape[1:]
    q = torch.empty(shape, dtype=torch.float32, device="cuda")
    if init is None:
        h = fit_linear_filter(A, inputs[:fit_pairs])
        init = linear_filter_params(h)
        init = init + 1e-3 * np.random.default_rng(seed).normal(size=init.shape) * (init == 0)
    params = torch.as_tensor(init.astype(np.float32), device="cuda").contiguous()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    net = _t.ConvNet(tuple(shape))
    grad = torch.empty_like(params)
    z = torch.empty(shape, dtype=torch.float32, device="cuda")
    d = torch.empty_like(z)
    rng = np.random.default_rng(seed)
    total = epochs * npairs
    trace = []
    acc = torch.zeros((), dtype=torch.float64, device="cuda")
    nacc = 0
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        for i in rng.permutation(npairs):
            step += 1
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * (step - 1) / total))
            net.forward(params, inputs[i], out=z)
            torch.sub(z, targets[i], out=d)
            A(d, q)  # d loss / d z
            net.backward(params, inputs[i], q, grad=grad)
            _t.adam_step(params, grad, m, v, step, lr=rate)
            acc += 0.5 * torch.dot(d.reshape(-1).double(), q.reshape(-1).double())
            nacc += 1
            if step % 200 == 0 or step == total:
                trace.append(float(acc) / nacc)
                acc.zero_()
                nacc = 0
                if log:
                    log(f"step {step}/{total}: energy error {trace[-1]:.4e} "
                        f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return params, trace


def time_to_tolerance(dg: _t.DeviceGeometry, y: torch.Tensor, lam: float, rtol: float,
                      params: torch.Tensor | None, max_iter: int = 1000, reps: int = 1):
    """Wall time (ms, median over reps) of tomo_cg_solve from entry to a
    confirmed true residual <= rtol, plain CG (params None) or flexible CG."""
    times = []
    rep = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = _t.cg_solve(dg, y, lam_r=lam, max_iter=max_iter, rtol=rtol, precond=params,
                             check_every=5)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(times)), rep


def save(path: str, params: torch.Tensor, meta: dict):
    np.savez(path, params=params.detach().cpu().numpy().astype(np.float32),
             meta=np.array(repr(meta)))


def load(path: str, device="cuda") -> torch.Tensor:
    with np.load(path, allow_pickle=False) as f:
        return torch.as_tensor(f["params"].astype(np.float32), device=device).contiguous()
