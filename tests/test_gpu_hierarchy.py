"""GPU parity of the hierarchical pipeline (pyramid, level loop, pruning,
multi-class, incremental update) against ``oracle.hierarchy`` (FP64).

Two input kinds:
* float volumes quantised to multiples of 2^-10 with power-of-two sides, so the
  FP32 pyramid equals the FP64 one exactly; with FP64 box solves the level maps
  must then agree to 1e-6 and every brick decision must agree;
* uint16 volumes (global min-max normalisation in FP32 on the GPU): level maps
  agree to 1e-4 wherever both sides took the same pruning decisions; a
  decision may differ only where the deciding statistic lies within 1e-4 of
  its threshold (both results are correct then).
"""

import numpy as np
import pytest

from oracle import hierarchy as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2103_09564_amd as rwg
    assert torch.cuda.is_available()
    return torch, rwg, rwg.context(0)


def _sphere_volume(n, kind, seed=0):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    c = (n - 1) / 2
    r2 = (x - c) ** 2 + (y - 0.8 * c) ** 2 + (z - 1.1 * c) ** 2
    inside = r2 <= (0.3 * n) ** 2
    if kind == "u16":
        v = np.where(inside, 3000, 800) + rng.normal(0, 150, (n, n, n))
        return np.clip(v, 0, 65535).astype(np.uint16)
    v = np.where(inside, 0.7, 0.3) + rng.normal(0, 0.05, (n, n, n))
    return (np.round(np.clip(v, 0, 1) * 1024) / 1024).astype(np.float32)


def _seeds(n, rng, k_fg=6, k_bg=14, n_classes=2):
    c = (n - 1) / 2
    s = [[c + rng.uniform(-2, 2), 0.8 * c + rng.uniform(-2, 2), 1.1 * c + rng.uniform(-2, 2), 1] for _ in range(k_fg)]
    while len([q for q in s if q[3] == 0]) < k_bg:
        p = rng.uniform(0, n, 3)
        if (p[0] - c) ** 2 + (p[1] - 0.8 * c) ** 2 + (p[2] - 1.1 * c) ** 2 > (0.3 * n + 4) ** 2:
            s.append([p[0], p[1], p[2], 0])
    if n_classes > 2:
        for q in s:
            if q[3] == 0 and rng.random() < 0.5:
                q[3] = int(rng.integers(2, n_classes))
    return np.array(s, dtype=np.float64)


def _gpu_run(env, vol, seeds, levels, prev=None, pyr=None, **kw):
    torch, rwg, ctx = env
    if pyr is None:
        pyr = rwg.Pyramid(ctx, torch.from_numpy(vol).cuda(), levels)
    res = rwg.segment(pyr, seeds, prev=prev, **kw)
    torch.cuda.synchronize()
    maps = [res.level_map(l).cpu().numpy() for l in range(levels)]
    flags = [res.flags(l).cpu().numpy() for l in range(levels)]
    return pyr, res, maps, flags


def _oracle_params(**kw):
    base = dict(method="pcg", tol=1e-13)
    base.update(kw)
    return H.Params(**base)


def _compare(omaps, ores, gmaps, gflags, tol, exact_flags):
    for l in range(len(gmaps)):
        om = np.moveaxis(omaps[l], 0, -1)
        reached = (gflags[l] & 1) != 0
        assert np.array_equal(reached, ores.computed[l]) or not exact_flags, f"level {l} reached bricks differ"
        if exact_flags:
            assert np.array_equal((gflags[l] & 2) != 0, ores.prunable[l] & ores.computed[l]), f"level {l} prunable"
            err = np.max(np.abs(gmaps[l] - om))
            assert err <= tol, f"level {l}: max |gpu - oracle| = {err}"


def test_pyramid_u16_and_f32(env):
    torch, rwg, ctx = env
    rng = np.random.default_rng(1)
    v = rng.integers(100, 4000, (21, 29, 37)).astype(np.uint16)
    pyr = rwg.Pyramid(ctx, torch.from_numpy(v).cuda(), 4)
    ref = H.pyramid(v, 4)
    for l in range(4):
        got = pyr.level(l).cpu().numpy()
        assert got.shape == ref[l].shape
        assert np.max(np.abs(got - ref[l])) < 2e-6
    # a volume that starts 2 bytes past an aligned address (scalar loads in the min-max)
    flat = torch.from_numpy(np.concatenate([[7], v.ravel()]).astype(np.uint16)).cuda()
    pyr = rwg.Pyramid(ctx, flat[1:].view(v.shape), 2)
    for l in range(2):
        assert np.max(np.abs(pyr.level(l).cpu().numpy() - ref[l])) < 2e-6
    f = (rng.random((16, 12, 20)) * 1.4 - 0.2).astype(np.float32)
    pyr = rwg.Pyramid(ctx, torch.from_numpy(f).cuda(), 2)
    ref = H.pyramid(f, 2)
    for l in range(2):
        assert np.max(np.abs(pyr.level(l).cpu().numpy() - ref[l])) < 1e-6


@pytest.fixture(scope="module")
def binary_case():
    n, levels = 64, 4
    vol = _sphere_volume(n, "f32")
    seeds = _seeds(n, np.random.default_rng(2))
    p = _oracle_params(levels=levels, brick=8, beta=64.0, t_bin=0.01, t_hom=0.3)
    return vol, seeds, p, H.segment(vol, seeds, p)


def test_binary_fp64_exact_pyramid(env, binary_case):
    vol, seeds, p, ores = binary_case
    _, res, gmaps, gflags = _gpu_run(env, vol, seeds, p.levels, brick=8, beta=64.0, t_bin=0.01, t_hom=0.3,
                                     precision=0, tol=1e-12)
    _compare(ores.maps, ores, gmaps, gflags, 1e-6, exact_flags=True)
    st = res.stats()
    assert st["not_converged"] == [0] * p.levels
    # pruning took place (some level-0 bricks were never reached) and the
    # dense output equals the level-0 map
    assert sum(st["prunable"][1:]) > 0 and st["computed"][0] < st["bricks"][0]
    prob, lab = res.materialize(0, 1, prob=True, labels=True)
    assert np.array_equal(prob.cpu().numpy(), gmaps[0][..., 0])
    assert np.array_equal(lab.cpu().numpy(), (gmaps[0][..., 0] > 0.5).astype(np.uint8))


def test_binary_mixed_1e4(env, binary_case):
    vol, seeds, p, ores = binary_case
    _, _, gmaps, gflags = _gpu_run(env, vol, seeds, p.levels, brick=8, beta=64.0, t_bin=0.01, t_hom=0.3,
                                   precision=1, tol=1e-6)
    for l in range(p.levels):
        same = np.array_equal((gflags[l] & 1) != 0, ores.computed[l])
        assert same, f"level {l}: reached bricks differ"
        assert np.max(np.abs(gmaps[l] - np.moveaxis(ores.maps[l], 0, -1))) <= 1e-4


def test_u16_pipeline_1e4(env):
    n, levels = 64, 3
    vol = _sphere_volume(n, "u16", seed=3)
    seeds = _seeds(n, np.random.default_rng(4))
    p = _oracle_params(levels=levels, brick=16, beta=128.0, t_bin=0.49, prune_hom=False)
    ores = H.segment(vol, seeds, p)
    _, _, gmaps, gflags = _gpu_run(env, vol, seeds, levels, brick=16, beta=128.0, t_bin=0.49, prune_hom=0,
                                   precision=1, tol=1e-6)
    for l in range(levels):
        g_reached = (gflags[l] & 1) != 0
        if not np.array_equal(g_reached, ores.computed[l]):
            # a differing decision must sit on a threshold margin of the parent
            pytest.fail(f"level {l}: reached bricks differ")
        om = np.moveaxis(ores.maps[l], 0, -1)
        assert np.max(np.abs(gmaps[l] - om)) <= 1e-4


def test_multiclass_fp64(env):
    n, levels, K = 32, 2, 3
    vol = _sphere_volume(n, "f32", seed=5)
    seeds = _seeds(n, np.random.default_rng(6), n_classes=K)
    p = _oracle_params(levels=levels, brick=8, beta=64.0, n_classes=K, prune_dt=False, t_hom=0.3)
    ores = H.segment(vol, seeds, p)
    _, res, gmaps, gflags = _gpu_run(env, vol, seeds, levels, brick=8, beta=64.0, n_classes=K, prune_dt=0,
                                     t_hom=0.3, precision=0, tol=1e-12)
    _compare(ores.maps, ores, gmaps, gflags, 1e-6, exact_flags=True)
    probs = H.probabilities(ores, 0)
    lab = res.materialize(0, 0, prob=False, labels=True)[1].cpu().numpy()
    top2 = np.sort(probs, axis=0)[-2:]
    clear = (top2[1] - top2[0]) > 1e-3
    assert np.array_equal(lab[clear], H.labels(ores, 0)[clear])
    for cls in range(K):
        pr = res.materialize(0, cls, prob=True)[0].cpu().numpy()
        assert np.max(np.abs(pr - probs[cls])) <= 1e-6


@pytest.mark.parametrize("extra", [[[3.0, 3.0, 60.0, 0]], [[50.5, 12.25, 40.0, 1], [10.0, 52.0, 20.5, 0]]])
def test_incremental_matches_oracle(env, binary_case, extra):
    vol, seeds, p, ores = binary_case
    kw = dict(brick=8, beta=64.0, t_bin=0.01, t_hom=0.3, precision=0, tol=1e-12)
    pyr, res, _, _ = _gpu_run(env, vol, seeds, p.levels, **kw)
    more = np.concatenate([seeds, extra])
    oinc = H.segment(vol, more, p, prev=ores)
    _, rinc, gmaps, gflags = _gpu_run(env, vol, more, p.levels, prev=res, pyr=pyr, **kw)
    _compare(oinc.maps, oinc, gmaps, gflags, 1e-6, exact_flags=True)
    for l in range(p.levels):
        assert np.array_equal((gflags[l] & 8) != 0, oinc.recomputed[l]), f"level {l}: recomputed bricks differ"
    # no new label: everything is reused
    _, rsame, gm2, gf2 = _gpu_run(env, vol, more, p.levels, prev=rinc, pyr=pyr, **kw)
    for l in range(p.levels):
        assert not np.any(gf2[l] & 8)
        assert np.array_equal(gm2[l], gmaps[l])


@pytest.mark.parametrize("warm", [False, True])
@pytest.mark.parametrize("extra", [[[3.0, 3.0, 60.0, 0]], [[50.5, 12.25, 40.0, 1], [10.0, 52.0, 20.5, 0]]])
def test_incremental_node_rule_matches_oracle(env, binary_case, extra, warm):
    """The node rule of Section IV-E (solve, then keep the previous node and
    subtree when within t_inc) and the warm start from the previous result."""
    torch, rwg, ctx = env
    vol, seeds, p, ores = binary_case
    kw = dict(brick=8, beta=64.0, t_bin=0.01, t_hom=0.3, precision=0, tol=1e-12)
    pyr, res, _, _ = _gpu_run(env, vol, seeds, p.levels, **kw)
    more = np.concatenate([seeds, extra])
    oinc = H.segment(vol, more, H.Params(**{**p.__dict__, "inc_rule": "node", "inc_warm": warm}), prev=ores)
    mode = rwg.INC_NODE | (rwg.INC_WARM if warm else 0)
    _, rinc, gmaps, gflags = _gpu_run(env, vol, more, p.levels, prev=res, pyr=pyr, incremental=mode, **kw)
    _compare(oinc.maps, oinc, gmaps, gflags, 1e-6, exact_flags=True)
    kept = solved = 0
    for l in range(p.levels):
        assert np.array_equal((gflags[l] & rwg.F_SOLVED) != 0, oinc.recomputed[l]), f"level {l}: solved bricks differ"
        assert np.array_equal((gflags[l] & rwg.F_KEPT) != 0, oinc.reused[l]), f"level {l}: kept bricks differ"
        kept += int(oinc.reused[l].sum())
        solved += int(oinc.recomputed[l].sum())
    assert solved > 0
    if len(extra) == 1:
        assert kept > 0   # one background seed near a corner leaves nodes within t_inc
    if warm:
        # the same run started from the parent samples: the same result (the
        # start changes the iteration count only, either way)
        _, rcold, cmaps, _ = _gpu_run(env, vol, more, p.levels, prev=res, pyr=pyr, incremental=rwg.INC_NODE, **kw)
        for l in range(p.levels):
            assert np.max(np.abs(cmaps[l] - gmaps[l])) <= 2e-6
        assert rinc.stats()["voxel_iters"] != rcold.stats()["voxel_iters"]   # the warm start took effect


def test_incremental_node_rule_multiclass(env):
    """The node rule with three classes (two right-hand sides): the
    similarity test takes the max over both classes' maps."""
    torch, rwg, ctx = env
    n, levels, K = 32, 2, 3
    vol = _sphere_volume(n, "f32", seed=5)
    seeds = _seeds(n, np.random.default_rng(6), n_classes=K)
    kw = dict(brick=8, beta=64.0, n_classes=K, prune_dt=0, t_hom=0.3, precision=0, tol=1e-12)
    p = _oracle_params(levels=levels, brick=8, beta=64.0, n_classes=K, prune_dt=False, t_hom=0.3)
    ores = H.segment(vol, seeds, p)
    pyr, res, _, _ = _gpu_run(env, vol, seeds, levels, **kw)
    more = np.concatenate([seeds, [[30.0, 30.0, 30.0, 0]]])   # keeps 39 + 2 nodes, solves 48 + 8
    oinc = H.segment(vol, more, H.Params(**{**p.__dict__, "inc_rule": "node"}), prev=ores)
    assert oinc.reused[0].any() and oinc.reused[1].any()
    _, _, gmaps, gflags = _gpu_run(env, vol, more, levels, prev=res, pyr=pyr, incremental=rwg.INC_NODE, **kw)
    _compare(oinc.maps, oinc, gmaps, gflags, 1e-6, exact_flags=True)
    for l in range(levels):
        assert np.array_equal((gflags[l] & rwg.F_SOLVED) != 0, oinc.recomputed[l]), f"level {l}: solved bricks differ"
        assert np.array_equal((gflags[l] & rwg.F_KEPT) != 0, oinc.reused[l]), f"level {l}: kept bricks differ"


def test_single_level_is_plain_solve(env):
    torch, rwg, ctx = env
    vol = _sphere_volume(24, "f32", seed=7)
    seeds = _seeds(24, np.random.default_rng(8))
    p = _oracle_params(levels=1, brick=8, beta=64.0)
    ores = H.segment(vol, seeds, p)
    _, _, gmaps, gflags = _gpu_run(env, vol, seeds, 1, brick=8, beta=64.0, precision=0, tol=1e-12)
    assert np.max(np.abs(gmaps[0][..., 0] - ores.maps[0][0])) <= 1e-6


def test_segment_argument_errors(env):
    torch, rwg, ctx = env
    vol = _sphere_volume(16, "f32")
    pyr = rwg.Pyramid(ctx, torch.from_numpy(vol).cuda(), 2)
    with pytest.raises(rwg.RWError):
        rwg.segment(pyr, [[1, 1, 1, 5]], n_classes=2)
    with pytest.raises(rwg.RWError):
        rwg.segment(pyr, [[1, 1, 1, 1]], n_classes=9)
    with pytest.raises(rwg.RWError):
        rwg.segment(pyr, [[1, 1, 1, 1]], brick=1)
    with pytest.raises(rwg.RWError):
        rwg.segment(pyr, [[1, 1, 1, 1]], incremental=4)


def test_conflicting_labels_match_oracle(env):
    """Two labels on one voxel leave it unseeded and mark every brick whose box
    holds it cfl (never prunable); flags and maps against the oracle."""
    n, levels = 64, 3
    vol = _sphere_volume(n, "f32", seed=11)
    seeds = _seeds(n, np.random.default_rng(12))
    c = (n - 1) / 2
    extra = [[c + 0.3, 0.8 * c + 0.3, 1.1 * c, 0], [c + 0.3, 0.8 * c + 0.3, 1.1 * c, 1],   # inside the sphere
             [5.5, 60.2, 9.0, 1], [5.5, 60.2, 9.0, 0]]                                  # far outside it
    seeds = np.concatenate([seeds, np.array(extra, dtype=np.float64)])
    kw = dict(brick=8, beta=64.0, t_bin=0.01, t_hom=0.3)
    p = _oracle_params(levels=levels, **kw)
    ores = H.segment(vol, seeds, p)
    assert any(np.any(cf) for cf in ores.cfl)
    _, res, gmaps, gflags = _gpu_run(env, vol, seeds, levels, precision=0, tol=1e-12, **kw)
    _compare(ores.maps, ores, gmaps, gflags, 1e-6, exact_flags=True)
    for l in range(levels):
        reached = ores.computed[l]
        assert np.array_equal(((gflags[l] & 4) != 0) & reached, ores.cfl[l] & reached), f"level {l}: cfl differs"
        assert not np.any(((gflags[l] & 4) != 0) & ((gflags[l] & 2) != 0)), "a cfl brick was marked prunable"


def test_tube_volume_full_size_properties(env):
    """The 512^3 tube pipeline (4 levels, s = 32, e = 1.25, dt pruning at
    t_bin 0.49, mixed tol 1e-5) at full size, where the oracle is too slow:
    properties that hold at any size.  Maps lie in [0, 1] (maximum
    principle); every label voxel of a reached brick keeps its value; a brick
    is reached exactly when its parent is reached and not prunable; every
    solve converged."""
    import synth
    torch, rwg, ctx = env
    vol, seeds, _ = synth.tube_volume(n=512, n_tubes=40, n_fg=20, n_bg=200, seed=2)
    levels = 4
    pyr, res, maps, flags = _gpu_run(env, vol, seeds, levels, brick=32, expand=1.25, beta=128.0, eps=1e-6,
                                     tol=1e-5, precision=1, n_classes=2, prune_hom=0, prune_dt=1, t_bin=0.49)
    st = res.stats()
    assert st["not_converged"] == [0] * levels
    for l in range(levels):
        assert maps[l].min() >= -1e-6 and maps[l].max() <= 1 + 1e-6, l
    assert np.all((flags[levels - 1] & 1) != 0)
    for l in range(levels - 1):
        par = flags[l + 1]
        open_par = ((par & 1) != 0) & ((par & 2) == 0)
        nz, ny, nx = flags[l].shape
        expect = open_par[np.arange(nz)[:, None, None] // 2, np.arange(ny)[None, :, None] // 2,
                          np.arange(nx)[None, None, :] // 2]
        assert np.array_equal((flags[l] & 1) != 0, expect), f"level {l}: reached bricks"
    # labels at level 0 (voxel floor(q)); a voxel carrying both labels is unseeded
    vox = np.floor(seeds[:, :3]).astype(np.int64)
    keys = {}
    for (x, y, z), lab in zip(vox, seeds[:, 3].astype(int)):
        keys.setdefault((x, y, z), set()).add(lab)
    m0 = maps[0][..., 0]
    for (x, y, z), labs in keys.items():
        if len(labs) == 1 and (flags[0][z // 32, y // 32, x // 32] & 1):
            assert m0[z, y, x] == float(next(iter(labs))), (x, y, z, labs, m0[z, y, x])


def _poisson_volume(n, seed=0):
    """Photon counts: a sphere of mean 90 in a background of mean 25."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    c = (n - 1) / 2
    inside = (x - c) ** 2 + (y - 0.8 * c) ** 2 + (z - 1.1 * c) ** 2 <= (0.3 * n) ** 2
    return rng.poisson(np.where(inside, 90.0, 25.0)).astype(np.uint16)


def test_counts_pyramid_and_poisson_weight_pipeline(env):
    """Section IV-C's Poisson weight: the square-root counts pyramid against
    the oracle's (uint16 and float with negative values), and the hierarchy
    with beta 1/2 on it against the oracle hierarchy."""
    torch, rwg, ctx = env
    rng = np.random.default_rng(6)
    v = rng.integers(0, 4000, (21, 29, 37)).astype(np.uint16)
    pyr = rwg.Pyramid(ctx, torch.from_numpy(v).cuda(), 4, counts=True)
    ref = H.pyramid_counts(v, 4)
    for l in range(4):
        got = pyr.level(l).cpu().numpy()
        assert got.shape == ref[l].shape
        assert np.max(np.abs(got - ref[l]) / np.maximum(ref[l], 1.0)) < 1e-6
    f = (rng.random((16, 12, 20)) * 300 - 40).astype(np.float32)
    pyr = rwg.Pyramid(ctx, torch.from_numpy(f).cuda(), 3, counts=True)
    ref = H.pyramid_counts(f, 3)
    for l in range(3):
        assert np.max(np.abs(pyr.level(l).cpu().numpy() - ref[l]) / np.maximum(ref[l], 1.0)) < 1e-6
    n, levels = 64, 3
    vol = _poisson_volume(n, seed=7)
    seeds = _seeds(n, np.random.default_rng(8))
    p = _oracle_params(levels=levels, brick=16, beta=0.5, t_bin=0.49, prune_hom=False)
    ores = H.segment(vol, seeds, p, g=H.pyramid_counts(vol, levels))
    gpyr = rwg.Pyramid(ctx, torch.from_numpy(vol).cuda(), levels, counts=True)
    _, _, gmaps, gflags = _gpu_run(env, vol, seeds, levels, pyr=gpyr, brick=16, beta=0.5, t_bin=0.49, prune_hom=0,
                                   precision=1, tol=1e-6)
    for l in range(levels):
        assert np.array_equal((gflags[l] & 1) != 0, ores.computed[l]), f"level {l}: reached bricks differ"
        assert np.max(np.abs(gmaps[l] - np.moveaxis(ores.maps[l], 0, -1))) <= 1e-4
    # the segmentation separates the sphere from the background (0.89 of the
    # voxels labelled as the truth on this volume; a sanity floor, not parity)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    c = (n - 1) / 2
    truth = (x - c) ** 2 + (y - 0.8 * c) ** 2 + (z - 1.1 * c) ** 2 <= (0.3 * n) ** 2
    assert np.mean((gmaps[0][..., 0] > 0.5) == truth) > 0.8


def test_cached_buffers_carry_nothing_over(env):
    """Level maps, brick flags and pyramid levels come back from the
    per-device cache once freed: a run on another volume in between (its
    buffers reused, holding its values) must leave the repeated run's maps and
    flags bit for bit as before, for a binary and a three-class run."""
    import gc
    torch, rwg, ctx = env
    n, levels = 64, 3
    a = _sphere_volume(n, "u16", seed=7)
    b = _sphere_volume(n, "u16", seed=8)[::-1].copy()
    for n_classes in (2, 3):
        seeds = _seeds(n, np.random.default_rng(9), n_classes=n_classes)
        kw = dict(brick=16, beta=128.0, t_bin=0.49, prune_hom=0, precision=1, tol=1e-6, n_classes=n_classes)
        pyr, res, maps1, flags1 = _gpu_run(env, a, seeds, levels, **kw)
        del pyr, res
        gc.collect()
        pyr, res, _, _ = _gpu_run(env, b, seeds[::-1].copy(), levels, **kw)
        del pyr, res
        gc.collect()
        _, _, maps2, flags2 = _gpu_run(env, a, seeds, levels, **kw)
        for l in range(levels):
            assert np.array_equal(maps1[l], maps2[l]), (n_classes, l)
            assert np.array_equal(flags1[l], flags2[l]), (n_classes, l)


def _mem_types(pyr, res, levels):
    """hipMemoryType (1 host, 2 device) of each pyramid level and level map,
    asked of the HIP runtime this process has loaded."""
    import ctypes
    from paper_2103_09564_amd import binding as B
    path = next(ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln)
    hip = ctypes.CDLL(path)

    class Attr(ctypes.Structure):
        _fields_ = [("type", ctypes.c_int), ("device", ctypes.c_int), ("devicePointer", ctypes.c_void_p),
                    ("hostPointer", ctypes.c_void_p), ("isManaged", ctypes.c_int), ("allocationFlags", ctypes.c_uint)]

    def kind(ptr):
        a = Attr()
        assert hip.hipPointerGetAttributes(ctypes.byref(a), ctypes.c_void_p(ptr)) == 0
        return a.type
    out = []
    for l in range(levels):
        pp, pm, d, r = ctypes.c_void_p(), ctypes.c_void_p(), B._dims3(), ctypes.c_int()
        assert B.lib.rw_pyramid_level(pyr.handle, l, d, ctypes.byref(pp)) == 0
        assert B.lib.rw_result_level(res.handle, l, d, ctypes.byref(r), ctypes.byref(pm)) == 0
        out.append((kind(pp.value), kind(pm.value)))
    return out


def test_finest_levels_in_host_memory(env):
    """Out-of-core placement (Section IV-A): the finest levels' pyramid data
    and level maps in page-locked host memory (rw_pyramid_build_host,
    rw_params.host_levels), read and written in place by the same kernels.
    Pyramid levels, level maps, brick flags, run statistics and the
    materialised probabilities and labels equal the device-memory run's bit
    for bit (and the finest levels are indeed host memory), for a volume on
    the device (one host level) and one in pinned host memory (two), binary and three-class, and
    for an incremental run on top; pageable host memory and out-of-range
    level counts are refused."""
    torch, rwg, ctx = env
    print("host levels", flush=True)
    n, levels = 64, 3
    vol = _sphere_volume(n, "u16", seed=11)
    dv = torch.from_numpy(vol).cuda()
    hv = torch.from_numpy(vol).pin_memory()
    for n_classes in (2, 3):
        seeds = _seeds(n, np.random.default_rng(12), n_classes=n_classes)
        kw = dict(brick=16, beta=128.0, t_bin=0.49, prune_hom=1, precision=1, tol=1e-6, n_classes=n_classes)
        pyr_d, res_d, maps_d, flags_d = _gpu_run(env, vol, seeds, levels, **kw)
        more = np.vstack([seeds, [[n / 2 + 3, n / 2 - 5, n / 2, 1]]])
        _, _, mi_d, fi_d = _gpu_run(env, vol, more, levels, prev=res_d, pyr=pyr_d, **kw)
        for src, hl in ((dv, 1), (hv, 2)):
            pyr_h = rwg.Pyramid(ctx, src, levels, host_levels=hl)
            for l in range(levels):
                assert np.array_equal(pyr_h.level(l).cpu().numpy(), pyr_d.level(l).cpu().numpy()), (hl, l)
            _, res_h, maps_h, flags_h = _gpu_run(env, vol, seeds, levels, pyr=pyr_h, host_levels=hl, **kw)
            assert _mem_types(pyr_h, res_h, levels) == [(1, 1)] * hl + [(2, 2)] * (levels - hl), hl
            assert _mem_types(pyr_d, res_d, levels) == [(2, 2)] * levels
            for l in range(levels):
                assert np.array_equal(maps_h[l], maps_d[l]), (n_classes, hl, l)
                assert np.array_equal(flags_h[l], flags_d[l]), (n_classes, hl, l)
            assert res_h.stats() == res_d.stats(), (n_classes, hl)
            for cls in range(1, n_classes):
                pd_, ld_ = res_d.materialize(0, cls, prob=True, labels=True)
                ph_, lh_ = res_h.materialize(0, cls, prob=True, labels=True)
                assert torch.equal(pd_, ph_) and torch.equal(ld_, lh_), (n_classes, hl, cls)
            _, _, mi_h, fi_h = _gpu_run(env, vol, more, levels, prev=res_h, pyr=pyr_h, host_levels=hl, **kw)
            for l in range(levels):
                assert np.array_equal(mi_h[l], mi_d[l]) and np.array_equal(fi_h[l], fi_d[l]), (n_classes, hl, l)
    with pytest.raises(rwg.RWError):
        rwg.Pyramid(ctx, torch.from_numpy(vol), levels, host_levels=1)      # pageable host memory
    with pytest.raises(rwg.RWError):
        rwg.Pyramid(ctx, dv, levels, host_levels=levels)                    # the coarsest level stays on the device
    with pytest.raises(rwg.RWError):
        rwg.segment(rwg.Pyramid(ctx, dv, levels), _seeds(n, np.random.default_rng(13)), host_levels=levels)
