"""GPU parity of the hierarchy at the paper's brick configuration (Section
IV-A/B: s = 32, e = 1.25, so 40^3 boxes with 4 + 4 voxels of expansion)
against ``oracle.hierarchy`` (FP64), through the C ABI.

* Tube twin (the 512^3 tube pipeline scaled to 128^3: 4 tubes, 3 levels, dt
  pruning at t_bin 0.49, hom off): FP64 box solves hold every level map to
  1e-6 and every brick decision exactly; mixed precision to 1e-4 at box
  tolerance 1e-6.  At the tube pipeline's own tolerance 1e-5 the relative
  residual stop leaves up to about 1e-3 in max norm (measured 9.7e-4 on a
  level-1 box, which starts from the coarsest level's sample): there the bar
  is 2e-3 (the error scales with the tolerance: 6.7e-5 at 1e-6), and the
  decisions and the Dice must still agree.
* Shell twin (the four-class shell volume at 128 x 128 x 64, 3 levels, K = 4
  so three right-hand sides per box, hom pruning at 0.3, dt off): FP64 to 1e-6
  with exact decisions; mixed to 1e-4, and the argmax labels equal wherever
  the oracle's top two classes differ by more than 1e-3.
* Per-brick replay at full size: the 512^3 tube pipeline in the configuration
  the benchmark times (4 levels, mixed, tol 1e-5).  For sampled solved
  level-0 bricks the oracle rebuilds each box from the GPU's own level-1 map
  (trilinear border samples and start values, rasterised labels) and solves
  it exactly; the GPU's core must match within the error bound of a solve
  stopped at relative residual 1e-5 (the bar is stated in the test).

uint16 volumes are normalised in FP32 on the GPU and in FP64 by the oracle;
a brick decision can then differ only if its statistic lies within about
1e-7 of a threshold, which does not happen on these volumes: the decisions
are required to be equal.
"""

import numpy as np
import pytest

import synth
from oracle import hierarchy as H

pytestmark = pytest.mark.gpu

S, E = 32, 1.25


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2103_09564_amd as rwg
    assert torch.cuda.is_available()
    return torch, rwg, rwg.context(0)


def _gpu(env, vol, seeds, levels, **kw):
    torch, rwg, ctx = env
    pyr = rwg.Pyramid(ctx, torch.from_numpy(vol).cuda(), levels)
    res = rwg.segment(pyr, seeds, **kw)
    torch.cuda.synchronize()
    maps = [res.level_map(l).cpu().numpy() for l in range(levels)]
    flags = [res.flags(l).cpu().numpy() for l in range(levels)]
    return res, maps, flags


def _flags_equal(gflags, ores, levels):
    for l in range(levels):
        reached = (gflags[l] & 1) != 0
        assert np.array_equal(reached, ores.computed[l]), f"level {l}: reached bricks differ"
        assert np.array_equal((gflags[l] & 2) != 0, ores.prunable[l] & ores.computed[l]), f"level {l}: prunable"


def _max_err(gmaps, ores, levels):
    return [float(np.max(np.abs(gmaps[l] - np.moveaxis(ores.maps[l], 0, -1)))) for l in range(levels)]


def _dice(a, b):
    return float(2.0 * np.sum(a & b) / max(1, np.sum(a) + np.sum(b)))


@pytest.fixture(scope="module")
def tube_twin():
    vol, seeds, tube = synth.tube_volume(n=128, n_tubes=4, n_fg=3, n_bg=40, seed=2)
    kw = dict(brick=S, expand=E, beta=128.0, eps=1e-6, n_classes=2, prune_hom=0, prune_dt=1, t_bin=0.49)
    p = H.Params(levels=3, brick=S, expand=E, beta=128.0, eps=1e-6, t_bin=0.49, prune_hom=False,
                 method="pcg", tol=1e-12)
    ores = H.segment(vol, seeds, p)
    # the configuration exercises pruning at both finer levels
    assert ores.computed[0].sum() < ores.computed[0].size and (ores.prunable[0] & ores.computed[0]).any()
    return vol, seeds, tube, kw, ores


def test_tube_twin_s32_fp64(env, tube_twin):
    vol, seeds, tube, kw, ores = tube_twin
    res, gmaps, gflags = _gpu(env, vol, seeds, 3, precision=0, tol=1e-12, **kw)
    _flags_equal(gflags, ores, 3)
    err = _max_err(gmaps, ores, 3)
    print(f"tube twin s=32 FP64: max |gpu - oracle| per level {err}", flush=True)
    assert max(err) <= 1e-6, err
    assert res.stats()["not_converged"] == [0, 0, 0]


@pytest.mark.parametrize("tol", [1e-6, 1e-5])
def test_tube_twin_s32_mixed(env, tube_twin, tol):
    vol, seeds, tube, kw, ores = tube_twin
    res, gmaps, gflags = _gpu(env, vol, seeds, 3, precision=1, tol=tol, **kw)
    _flags_equal(gflags, ores, 3)
    err = _max_err(gmaps, ores, 3)
    dg = _dice(gmaps[0][..., 0] > 0.5, tube > 0)
    do = _dice(ores.maps[0][0] > 0.5, tube > 0)
    print(f"tube twin s=32 mixed tol {tol}: max err per level {err}; Dice vs tubes GPU {dg:.4f} oracle {do:.4f}",
          flush=True)
    assert max(err) <= (1e-4 if tol <= 1e-6 else 2e-3), err
    # the same segmentation: Dice equal up to voxels near 0.5
    assert abs(dg - do) <= 1e-3


@pytest.fixture(scope="module")
def shell_twin():
    vol, lab, seeds, _ = synth.shell_volume(dims=(128, 128, 64), seed=5, n_per_class=20)
    kw = dict(brick=S, expand=E, beta=128.0, eps=1e-6, n_classes=4, prune_hom=1, prune_dt=0, t_hom=0.3)
    p = H.Params(levels=3, brick=S, expand=E, beta=128.0, eps=1e-6, n_classes=4, t_hom=0.3, prune_dt=False,
                 method="pcg", tol=1e-12)
    ores = H.segment(vol, seeds, p)
    assert (ores.prunable[0] & ores.computed[0]).any()
    return vol, lab, seeds, kw, ores


def test_shell_twin_k4_fp64(env, shell_twin):
    vol, lab, seeds, kw, ores = shell_twin
    res, gmaps, gflags = _gpu(env, vol, seeds, 3, precision=0, tol=1e-12, **kw)
    _flags_equal(gflags, ores, 3)
    err = _max_err(gmaps, ores, 3)
    print(f"shell twin K=4 FP64: max err per level {err}", flush=True)
    assert max(err) <= 1e-6, err


def test_shell_twin_k4_mixed_labels(env, shell_twin):
    vol, lab, seeds, kw, ores = shell_twin
    res, gmaps, gflags = _gpu(env, vol, seeds, 3, precision=1, tol=1e-6, **kw)
    _flags_equal(gflags, ores, 3)
    err = _max_err(gmaps, ores, 3)
    assert max(err) <= 1e-4, err
    probs = H.probabilities(ores, 0)
    top2 = np.sort(probs, axis=0)[-2:]
    clear = (top2[1] - top2[0]) > 1e-3
    glab = res.materialize(0, 0, prob=False, labels=True)[1].cpu().numpy()
    olab = H.labels(ores, 0)
    assert np.array_equal(glab[clear], olab[clear])
    acc_g, acc_o = float(np.mean(glab == lab)), float(np.mean(olab == lab))
    print(f"shell twin K=4 mixed: max err per level {err}; labels equal on {clear.mean():.5f} of voxels "
          f"with margin > 1e-3; accuracy vs truth GPU {acc_g:.4f} oracle {acc_o:.4f}", flush=True)


def test_shell_twin_k4_joint_and_per_class(env, shell_twin):
    """Below the coarsest level each class of a box is solved as a box of its
    own (one right-hand side) by default; rw_params.joint_classes = 1 solves
    the three together.  The same independent solves: the same decisions,
    level maps within 4e-5 of each other (two stops at relative residual
    1e-6) and both within 1e-4 of the oracle."""
    vol, lab, seeds, kw, ores = shell_twin
    rp, mp, fp = _gpu(env, vol, seeds, 3, precision=1, tol=1e-6, **kw)
    rj, mj, fj = _gpu(env, vol, seeds, 3, precision=1, tol=1e-6, joint_classes=1, **kw)
    for l in range(3):
        assert np.array_equal(fp[l], fj[l]), l
    diff = max(float(np.max(np.abs(mp[l] - mj[l]))) for l in range(3))
    print(f"shell twin K=4: per-class vs joint max diff {diff:.3e}", flush=True)
    assert diff <= 4e-5
    assert max(_max_err(mp, ores, 3)) <= 1e-4 and max(_max_err(mj, ores, 3)) <= 1e-4
    # a box's iterations are the most any of its classes took in both
    assert rp.stats()["solved"] == rj.stats()["solved"]


def test_tube_512_per_brick_replay(env):
    """Sampled level-0 bricks of the full-size tube pipeline, rebuilt by the
    oracle from the GPU's level-1 map and solved exactly.

    Bar: a box solved to relative residual tol = 1e-5 has an error of at most
    about cond * tol * ||x||; with the warm start from the parent sample the
    GPU error stays far below that.  The test requires 1e-4 on every sampled
    core voxel, the acceptance bar of the FP32 path."""
    torch, rwg, ctx = env
    vol, seeds, _ = synth.tube_volume(n=512, n_tubes=40, n_fg=20, n_bg=200, seed=2)
    levels = 4
    res, gmaps, gflags = _gpu(env, vol, seeds, levels, brick=S, expand=E, beta=128.0, eps=1e-6, tol=1e-5,
                              precision=1, n_classes=2, prune_hom=0, prune_dt=1, t_bin=0.49)
    d0 = vol.shape
    g0 = H.normalize(vol)
    lab0 = H.rasterize(seeds, 0, d0)
    up = H.upsample(gmaps[1][..., 0][None].astype(np.float64), d0)
    solved = np.argwhere((gflags[0] & 8) != 0)
    rng = np.random.default_rng(0)
    picks = solved[rng.choice(len(solved), min(32, len(solved)), replace=False)]
    p = H.Params(levels=levels, brick=S, expand=E, beta=128.0, eps=1e-6, method="pcg", tol=1e-12)
    errs = []
    for b in map(tuple, picks):
        core, box = H.brick_box(b, d0, S, E)
        xb = H._solve(g0[H._sl(box)], lab0[H._sl(box)], H.border_layer(box, d0), up[(slice(None),) + H._sl(box)], p)
        rel = tuple(slice(c0 - b0, c1 - b0) for (c0, c1), (b0, _) in zip(core, box))
        want = xb[0][rel]
        got = gmaps[0][H._sl(core)][..., 0]
        errs.append(float(np.max(np.abs(got - want))))
    print(f"tube 512 replay: {len(errs)} bricks, max err {max(errs):.3e}, median {np.median(errs):.3e}", flush=True)
    assert max(errs) <= 1e-4, errs
