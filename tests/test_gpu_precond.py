"""The shipped learned preconditioner (trained by
python -m paper_1103_5904_amd.train_precond on seeds 1000-1049) against the
method without it: on held-out problems of the same family (128^3 blob
phantom, 28 views of 256x256, 1% noise, lambda 1e-2) flexible CG with the
network reaches a confirmed true relative residual of 1e-3 in fewer
iterations and less wall time than plain CG, without falling back."""
import ast
import os

import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import need_gpu

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1103_5904_amd", "precond_weights.npz")


@pytest.fixture(scope="module")
def setup():
    tomo = need_gpu()
    from paper_1103_5904_amd import precond as pc

    return tomo, pc, pc.load(WEIGHTS)


def test_weights_were_trained_on_other_seeds():
    with np.load(WEIGHTS, allow_pickle=False) as f:
        meta = ast.literal_eval(str(f["meta"]))
        assert f["params"].shape == (7809,) and np.all(np.isfinite(f["params"]))
    assert 1000 + meta["train_seeds"] <= 2003


@pytest.mark.parametrize("seed", [2003, 2004, 2006])
def test_learned_fcg_beats_plain_cg(setup, seed):
    import torch

    tomo, pc, net = setup
    wl = ts.learned(seed)
    dg = tomo.DeviceGeometry(wl.geom)
    y = pc.noisy_data(dg, torch.as_tensor(wl.x.astype(np.float32)).cuda(), wl.noise_rel, wl.noise_seed)
    pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, None)
    pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, net)
    t_plain, r_plain = pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, None, reps=5)
    t_net, r_net = pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, net, reps=5)
    print(f"seed {seed}: plain {r_plain['iters']} it {t_plain:.1f} ms, "
          f"learned {r_net['iters']} it {t_net:.1f} ms")
    for r in (r_plain, r_net):
        assert r["status"] == 0 and r["true_rel_res"] <= 1e-3
    assert r_net["fell_back"] == -1
    assert r_net["iters"] <= 0.85 * r_plain["iters"]
    assert t_net < t_plain
