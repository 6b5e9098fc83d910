"""Pins of the oracle's hierarchical pipeline (CPU only)."""

import numpy as np
import pytest

from oracle import hierarchy as H
from oracle import rw


def test_downsample_matches_loops():
    rng = np.random.default_rng(0)
    a = rng.random((5, 3, 4))
    out = H.downsample2x(a)
    assert out.shape == (3, 2, 2)
    for z in range(3):
        for y in range(2):
            for x in range(2):
                vals = [a[zz, yy, xx] for zz in (2 * z, 2 * z + 1) for yy in (2 * y, 2 * y + 1)
                        for xx in (2 * x, 2 * x + 1) if zz < 5 and yy < 3 and xx < 4]
                assert abs(out[z, y, x] - sum(vals) / len(vals)) < 1e-15


def test_normalize():
    v = np.array([[[100, 300], [200, 500]]], dtype=np.uint16)
    assert np.allclose(H.normalize(v), [[[0.0, 0.5], [0.25, 1.0]]])
    f = np.array([[[-0.5, 0.25, 1.5]]], dtype=np.float32)
    assert np.allclose(H.normalize(f), [[[0.0, 0.25, 1.0]]])


def test_upsample_hand_values():
    # parent [0, 4] along x -> child centres at parent coords -0.25, 0.25, 0.75, 1.25
    p = np.array([0.0, 4.0]).reshape(1, 1, 1, 2)
    u = H.upsample(p, (1, 1, 4))
    assert np.allclose(u.ravel(), [0.0, 1.0, 3.0, 4.0], atol=1e-15)


def test_upsample_reproduces_linear_fields():
    Pz, Py, Px = 5, 6, 7
    z, y, x = np.meshgrid(np.arange(Pz), np.arange(Py), np.arange(Px), indexing="ij")
    f = 0.3 * x - 0.2 * y + 0.1 * z + 0.05
    u = H.upsample(f[None], (2 * Pz, 2 * Py, 2 * Px))[0]
    Z, Y, X = np.meshgrid(np.arange(2 * Pz), np.arange(2 * Py), np.arange(2 * Px), indexing="ij")
    fx = lambda c: (c + 0.5) / 2 - 0.5
    expect = 0.3 * fx(X) - 0.2 * fx(Y) + 0.1 * fx(Z) + 0.05
    inner = (slice(1, -1),) * 3        # clamping is active only on the outer layer
    assert np.max(np.abs(u[inner] - expect[inner])) < 1e-14
    c = H.upsample(np.full((1, 3, 3, 3), 0.7), (5, 6, 5))
    assert np.allclose(c, 0.7, atol=1e-15)


def test_rasterize_and_conflicts():
    seeds = np.array([[2.5, 0.2, 0.0, 1], [3.9, 1.9, 1.5, 0],   # level 1: both -> (z0,y0,x1)
                      [0.1, 0.1, 0.1, 1], [1.9, 0.0, 0.0, 1]])  # level 1: both -> (0,0,0), same label
    l0 = H.rasterize(seeds, 0, (4, 4, 4))
    assert l0[0, 0, 2] == 1 and l0[1, 1, 3] == 0 and l0[0, 0, 0] == 1 and l0[0, 0, 1] == 1
    l1 = H.rasterize(seeds, 1, (2, 2, 2))
    assert l1[0, 0, 1] == -2
    assert l1[0, 0, 0] == 1
    assert (l1 == -1).sum() == 6


def test_brick_box_hand_values():
    core, box = H.brick_box((0, 1, 0), (64, 64, 40), 32, 1.25)
    assert core == [(0, 32), (32, 64), (0, 32)]
    assert box == [(0, 36), (28, 64), (0, 36)]
    core, box = H.brick_box((0, 0, 1), (64, 64, 40), 32, 1.25)
    assert core[2] == (32, 40) and box[2] == (28, 40)


def test_prune_predicates_brute_force():
    p = H.Params(t_hom=0.3, t_bin=0.01)
    rng = np.random.default_rng(4)
    for _ in range(200):
        lo = rng.random()
        hi = lo + rng.random() * (1 - lo)
        x = rng.uniform(lo, hi, (1, 4, 4, 4))
        hom, dt = H.prune_tests(x, p)
        mn, mx = x.min(), x.max()
        assert hom == bool(mx - mn < 0.3)
        assert dt == bool(mn > 0.51 or mx < 0.49)


def _toy_volume(n=24, seed=0):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    c = (n - 1) / 2
    inside = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 <= (0.3 * n) ** 2
    v = np.where(inside, 3000, 800) + rng.normal(0, 100, (n, n, n))
    return np.clip(v, 0, 65535).astype(np.uint16)


def _toy_seeds(n=24):
    c = (n - 1) / 2
    fg = [[c + dx, c + dy, c, 1] for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
    bg = [[1.0, 1.0, 1.0, 0], [n - 2.0, n - 2.0, n - 2.0, 0], [1.0, n - 2.0, 2.0, 0], [n - 2.0, 1.0, n / 2, 0]]
    return np.array(fg + bg, dtype=np.float64)


def test_single_level_is_plain_solve():
    vol = _toy_volume(16)
    seeds = _toy_seeds(16)
    p = H.Params(levels=1, brick=8, beta=64.0)
    res = H.segment(vol, seeds, p)
    g = H.normalize(vol)
    lab = H.rasterize(seeds, 0, g.shape)
    x = np.where(lab == 1, 1.0, 0.0)
    plain = rw.solve_box(g, (lab >= 0).astype(np.uint8), x, 64.0, 1e-6)
    assert np.max(np.abs(res.maps[0][0] - plain)) < 1e-13


def test_one_brick_per_level_is_plain_solve_per_level():
    """With bricks covering whole levels no face is interior, so each level is
    solved with the user seeds only."""
    vol = _toy_volume(16)
    seeds = _toy_seeds(16)
    p = H.Params(levels=3, brick=16, beta=64.0, prune_hom=False, prune_dt=False)
    res = H.segment(vol, seeds, p)
    g = H.pyramid(vol, 3)
    for lvl in range(3):
        lab = H.rasterize(seeds, lvl, g[lvl].shape)
        x = np.where(lab == 1, 1.0, 0.0)
        plain = rw.solve_box(g[lvl], (lab >= 0).astype(np.uint8), x, 64.0, 1e-6)
        assert np.max(np.abs(res.maps[lvl][0] - plain)) < 1e-12


@pytest.fixture(scope="module")
def toy_run():
    vol = _toy_volume(24)
    seeds = _toy_seeds(24)
    p = H.Params(levels=3, brick=8, beta=64.0, t_bin=0.49, prune_hom=False, prune_dt=True)
    return vol, seeds, p, H.segment(vol, seeds, p)


def test_hierarchy_invariants(toy_run):
    vol, seeds, p, res = toy_run
    for lvl in range(3):
        m = res.maps[lvl]
        assert m.min() >= -1e-12 and m.max() <= 1 + 1e-12
    lab = H.rasterize(seeds, 0, res.dims[0])
    x0 = res.maps[0][0]
    comp = np.kron(res.computed[0], np.ones((8, 8, 8), bool))[:24, :24, :24]
    sel = (lab >= 0) & comp
    assert np.array_equal(x0[sel], (lab[sel] == 1).astype(float))
    # children are computed exactly where the parent was computed and not prunable
    for lvl in range(2):
        par = res.computed[lvl + 1] & ~res.prunable[lvl + 1]
        want = np.kron(par, np.ones((2, 2, 2), bool))[tuple(slice(0, n) for n in res.computed[lvl].shape)]
        assert np.array_equal(res.computed[lvl], want)
    # toy volume: the sphere is segmented
    g = H.normalize(vol)
    assert ((x0 > 0.5) == (g > 0.5)).mean() > 0.97


def test_incremental_no_new_seed_reuses_everything(toy_run):
    vol, seeds, p, res = toy_run
    again = H.segment(vol, seeds, p, prev=res)
    for lvl in range(3):
        assert np.array_equal(again.maps[lvl], res.maps[lvl])
        assert not again.recomputed[lvl].any()


def test_incremental_with_zero_threshold_equals_full_run(toy_run):
    vol, seeds, p, res = toy_run
    more = np.concatenate([seeds, [[20.0, 4.0, 12.0, 1]]])
    p0 = H.Params(**{**p.__dict__, "t_inc": 0.0})
    inc = H.segment(vol, more, p0, prev=res)
    full = H.segment(vol, more, p0)
    for lvl in range(3):
        assert np.array_equal(inc.computed[lvl], full.computed[lvl])
        assert np.max(np.abs(inc.maps[lvl] - full.maps[lvl])) < 1e-13


def test_incremental_recomputes_only_touched_bricks(toy_run):
    vol, seeds, p, res = toy_run
    more = np.concatenate([seeds, [[20.0, 4.0, 12.0, 1]]])
    inc = H.segment(vol, more, p, prev=res)
    full = H.segment(vol, more, p)
    # the brick holding the new seed is recomputed at level 0 if it is reached
    b = (12 // 8, 4 // 8, 20 // 8)
    if inc.computed[0][b]:
        assert inc.recomputed[0][b]
    assert inc.recomputed[0].sum() <= full.computed[0].sum()
    # reused results stay within t_inc-scale of a full recomputation
    assert np.max(np.abs(inc.maps[0] - full.maps[0])) < 0.2


def test_multiclass_hierarchy_sums_to_one():
    vol = _toy_volume(16)
    n = 16
    seeds = np.array([[7.5, 7.5, 7.5, 1], [1, 1, 1, 0], [14, 14, 14, 2], [1, 14, 7, 2], [14, 1, 3, 0]], float)
    p = H.Params(levels=2, brick=8, beta=64.0, n_classes=3, prune_hom=True, prune_dt=False)
    res = H.segment(vol, seeds, p)
    pr = H.probabilities(res, 0)
    assert pr.shape == (3, n, n, n)
    assert np.max(np.abs(pr.sum(axis=0) - 1)) < 1e-12
    lab = H.labels(res, 0)
    assert lab[7, 7, 7] == 1 and lab[14, 14, 14] == 2 and lab[1, 1, 1] == 0


def test_upsample_box_is_the_whole_upsample_restricted():
    """upsample_box equals the whole-level upsample on the box, for boxes on
    every edge (clamped taps) and in the interior, odd and even sizes."""
    rng = np.random.default_rng(3)
    parent = rng.random((2, 5, 7, 6))
    shape = (9, 13, 12)
    full = H.upsample(parent, shape)
    for box in [((0, 9), (0, 13), (0, 12)), ((0, 3), (5, 13), (7, 12)), ((4, 9), (1, 2), (0, 5)),
                ((3, 7), (6, 11), (2, 10))]:
        got = H.upsample_box(parent, shape, box)
        want = full[(slice(None),) + tuple(slice(a, b) for a, b in box)]
        assert got.shape == want.shape
        assert np.array_equal(got, want)


def test_upsample_box_from_a_crop_and_rasterize_box():
    rng = np.random.default_rng(4)
    parent = rng.random((3, 6, 5, 7))
    shape = (12, 9, 14)
    full = H.upsample(parent, shape)
    box = ((5, 12), (0, 4), (6, 11))
    # parent crop that covers the box's taps: child X -> parent (X + 1/2)/2 - 1/2
    origin = (2, 0, 2)
    crop = parent[:, 2:6, 0:3, 2:6]
    got = H.upsample_box(crop, shape, box, origin=origin, parent_shape=(6, 5, 7))
    assert np.array_equal(got, full[(slice(None),) + tuple(slice(a, b) for a, b in box)])
    with pytest.raises(ValueError):
        H.upsample_box(parent[:, 3:6], shape, box, origin=(3, 0, 0), parent_shape=(6, 5, 7))
    seeds = np.array([[6.2, 1.0, 7.9, 1], [6.7, 1.5, 7.1, 0], [10.0, 3.9, 11.5, 2], [0.5, 0.5, 0.5, 1],
                      [13.9, 8.9, 11.9, 3]])
    dims = (12, 9, 14)
    for lvl in (0, 1):
        d = tuple((n + (1 << lvl) - 1) >> lvl for n in dims)
        whole = H.rasterize(seeds, lvl, d)
        for b in [((0, d[0]), (0, d[1]), (0, d[2])), ((1, 4), (0, 3), (3, 7))]:
            sub = whole[tuple(slice(a, c) for a, c in b)]
            assert np.array_equal(H.rasterize_box(seeds, lvl, d, b), sub)


def test_normalize_with_a_global_range():
    v = np.array([[[100, 300], [200, 500]]], dtype=np.uint16)
    whole = H.normalize(v)
    part = H.normalize(v[:, :1, :], vrange=(100, 500))
    assert np.array_equal(part, whole[:, :1, :])
