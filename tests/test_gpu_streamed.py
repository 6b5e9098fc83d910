"""Boxes held in host memory, streamed through the GPU (rw_solve_bricks_streamed).

Per box the streamed solve runs the same kernels on the same data as the
device-resident one (a box's kernel path depends on its shape only), so x
and the per-box statistics must be bit-identical to rw_solve_bricks on the
same inputs, whatever the chunking; and both are checked against the oracle
on sampled boxes.
"""

import numpy as np
import pytest

import synth
from oracle import rw as orw

pytestmark = pytest.mark.gpu

KW = dict(beta=128.0, eps=1e-6, tol=1e-6)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2103_09564_amd as rwg
    assert torch.cuda.is_available()
    d = synth.stress_boxes(n=600, seed=21)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(d["x"].copy()).to(dev)
    st = rwg.solve_bricks(torch.from_numpy(d["g"]).to(dev), torch.from_numpy(d["mask"]).to(dev), xd,
                          d["shapes"], d["offsets"], **KW)
    torch.cuda.synchronize()
    return torch, rwg, d, xd.cpu(), rwg.stats_to_numpy(st)


def _host(torch, d, pinned):
    t = [torch.from_numpy(d[k].copy()) for k in ("g", "mask", "x")]
    return [v.pin_memory() for v in t] if pinned else t


@pytest.mark.parametrize("chunk, pinned", [(1_000_000, True), (3_000_000, False), (20_000, True), (0, True)])
def test_streamed_bit_identical_to_device_resident(env, chunk, pinned):
    torch, rwg, d, x_ref, st_ref = env
    print(f"streamed solve: 600 stress boxes, chunk_voxels={chunk}, pinned={pinned}", flush=True)
    g, m, x = _host(torch, d, pinned)
    st = rwg.stats_to_numpy(rwg.solve_bricks_streamed(g, m, x, d["shapes"], d["offsets"], chunk_voxels=chunk, **KW))
    assert torch.equal(x, x_ref)
    for k in ("status", "iters", "refine_steps", "true_rel_resid"):
        assert np.array_equal(st[k], st_ref[k]), k


def test_streamed_matches_oracle_on_sampled_boxes(env):
    torch, rwg, d, _, _ = env
    g, m, x = _host(torch, d, True)
    rwg.solve_bricks_streamed(g, m, x, d["shapes"], d["offsets"], chunk_voxels=2_000_000, **KW)
    xs = x.numpy()
    for i in (0, 137, 599):
        (nx, ny, nz), off = d["shapes"][i], int(d["offsets"][i])
        n = nx * ny * nz
        box = lambda a: a[off:off + n].reshape(nz, ny, nx)
        ref = orw.solve_box(box(d["g"]), box(d["mask"]), box(d["x"]).astype(np.float64), 128.0, 1e-6)
        assert np.max(np.abs(box(xs) - ref)) <= 1e-4


def test_streamed_argument_errors(env):
    torch, rwg, d, _, _ = env
    g, m, x = _host(torch, d, False)
    rev = d["offsets"][::-1].copy()
    with pytest.raises(rwg.RWError):
        rwg.solve_bricks_streamed(g, m, x, d["shapes"][::-1].copy(), rev, **KW)   # decreasing offsets
    with pytest.raises(ValueError):
        rwg.solve_bricks_streamed(g.cuda(), m, x, d["shapes"], d["offsets"], **KW)   # a device tensor
    shapes = d["shapes"][:2].copy()
    with pytest.raises(rwg.RWError):   # a box past the end of the buffers
        rwg.solve_bricks_streamed(g[:10], m[:10], x[:10], shapes, d["offsets"][:2], **KW)
    # no boxes: nothing happens
    rwg.solve_bricks_streamed(g, m, x, shapes[:0], d["offsets"][:0], **KW)


def test_streamed_three_rhs_and_fp64(env):
    """x interleaved [voxel][3] (the copies scale with nrhs) and the plain FP64
    path: still bit-identical to the device-resident solve."""
    torch, rwg, _, _, _ = env
    rng = np.random.default_rng(31)
    boxes = [synth.random_box(rng, s, dirichlet_frac=0.05) for s in [(9, 8, 7), (16, 5, 3), (20, 20, 20), (12, 30, 6)]]
    d = synth.from_boxes(boxes)
    R = 3
    xs = [np.where(d["mask"] != 0, rng.random(d["x"].size), 0.0).astype(np.float32) for _ in range(R)]
    x3 = np.stack(xs, axis=1).ravel()
    for kw in (dict(precision=rwg.PREC_MIXED, nrhs=R), dict(precision=rwg.PREC_FP64, nrhs=R)):
        print(f"streamed solve, 4 random boxes, {kw}", flush=True)
        xd = torch.from_numpy(x3.copy()).cuda()
        rwg.solve_bricks(torch.from_numpy(d["g"]).cuda(), torch.from_numpy(d["mask"]).cuda(), xd,
                         d["shapes"], d["offsets"], beta=128.0, eps=1e-6, tol=1e-7, **kw)
        torch.cuda.synchronize()
        xh = torch.from_numpy(x3.copy()).pin_memory()
        rwg.solve_bricks_streamed(torch.from_numpy(d["g"]).pin_memory(), torch.from_numpy(d["mask"]).pin_memory(),
                                  xh, d["shapes"], d["offsets"], chunk_voxels=3000, beta=128.0, eps=1e-6,
                                  tol=1e-7, **kw)
        assert torch.equal(xh, xd.cpu())
