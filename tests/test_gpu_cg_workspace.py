"""tomo_cg_solve with a caller-provided device workspace (tomo_cg_workspace_bytes):
the same kernels on the same buffers' contents, so the same iterates bit for
bit as the solve that takes stream-ordered scratch; a short workspace, a
misaligned one and a workspace with use_graph are refused before any work."""
import numpy as np
import pytest
import torch

import tomo_synth as ts
from _gpu_common import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def _problem(tomo, ora):
    wl = ts.tiny()
    y = ora.project(wl.geom, wl.x).astype(np.float32).astype(np.float64)
    return wl, tomo.DeviceGeometry(wl.geom), to_dev(y)


def _workspace(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def _same_solve(tomo, dg, y, ws, **kw):
    x0, r0 = tomo.cg_solve(dg, y, **kw)
    x1, r1 = tomo.cg_solve(dg, y, workspace=ws, **kw)
    assert r0["iters"] == r1["iters"] and r0["status"] == r1["status"]
    np.testing.assert_array_equal(r0["history"], r1["history"])
    np.testing.assert_array_equal(to_host(x0), to_host(x1))
    return r1


def test_workspace_solve_matches_scratch_solve(tomo, ora):
    wl, dg, y = _problem(tomo, ora)
    need = tomo.cg_workspace_bytes(dg, max_iter=20)
    nvox = int(np.prod(wl.geom.n))
    assert need >= 4 * 4 * nvox  # at least b, r, p and q
    # a workspace with room to spare, filled with garbage first
    ws = _workspace(need + 4096)
    ws.fill_(0xA5)
    rep = _same_solve(tomo, dg, y, ws, lam_r=wl.lam_r, max_iter=20)
    assert rep["iters"] == 20
    # exactly the queried size, twice in a row (the second sees the first's leftovers)
    ws = _workspace(need)
    for _ in range(2):
        _same_solve(tomo, dg, y, ws, lam_r=wl.lam_r, max_iter=20, rtol=1e-3, check_every=3)


def test_workspace_with_network_and_bricks(tomo, ora):
    """Flexible CG (identity network) and a tuning that walks bricks in P:
    the network's activations and P's bricked copy come from the workspace
    too."""
    from paper_1103_5904_amd import precond as pc

    wl, dg, y = _problem(tomo, ora)
    net = torch.as_tensor(pc.identity_params(1.0).astype(np.float32)).cuda()
    old = tomo.set_tuning(p_layout=3)
    try:
        tomo.autotune_clear()
        need_plain = tomo.cg_workspace_bytes(dg, max_iter=15)
        need = tomo.cg_workspace_bytes(dg, max_iter=15, precond=net)
        assert need > need_plain
        ws = _workspace(need)
        _same_solve(tomo, dg, y, ws, lam_r=wl.lam_r, max_iter=15, precond=net)
    finally:
        tomo.set_tuning(**old)


def test_workspace_refusals(tomo, ora):
    wl, dg, y = _problem(tomo, ora)
    need = tomo.cg_workspace_bytes(dg, max_iter=10)
    with pytest.raises(RuntimeError, match="needed"):
        tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=10, workspace=_workspace(need - 1))
    big = _workspace(need + 512)
    with pytest.raises(RuntimeError, match="aligned"):
        tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=10, workspace=big[8:])
    with pytest.raises(RuntimeError):
        tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=10, use_graph=True, workspace=big)
