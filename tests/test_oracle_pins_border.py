"""Pins of the oracle's box set-up and pruning decisions (CPU only).

* Section IV-A eq. (2) / Section IV-B eq. (3): which voxels of an expanded box
  carry continuous seeds and which parent value they take (a hand-worked
  case, and an end-to-end case where the answer is an affine field).
* Section IV-D1: hom/dt on binary and multi-class bricks against explicit
  loops and hand cases at the strict thresholds.
* Section IV-E (dirty-brick reading): the parent region whose change marks a
  brick dirty, against a hand-derived list of bricks.
* Section III-B: the Dirichlet energy on a hand-worked chain.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import hierarchy as H
from oracle import rw


@pytest.fixture(scope="module")
def border_case(golden_dir):
    with open(os.path.join(golden_dir, "border_s4_e15.json")) as f:
        return json.load(f)


def test_border_layer_and_parent_sample_hand_case(border_case):
    c = border_case
    d = tuple(c["level_dims_zyx"])
    core, box = H.brick_box(tuple(c["brick_index_zyx"]), d, c["brick"], c["expand"])
    assert [list(r) for r in core] == c["core_zyx"]
    assert [list(r) for r in box] == c["box_zyx"]
    border = H.border_layer(box, d)
    want = np.zeros(border.shape, bool)
    want[0, :, :] = True          # z low face (z = 3 is interior to the level)
    want[:, :, 0] = True          # x low face
    want[:, :, -1] = True         # x high face
    assert np.array_equal(border, want)
    assert int(border.sum()) == c["border_count"]

    P = np.array(c["parent_dims_zyx"])
    z, y, x = np.meshgrid(*(np.arange(n) for n in P), indexing="ij")
    parent = ((x ** 2 + 2 * y + z ** 2) / c["scale"])[None]
    up = H.upsample(parent, d)
    up_box = up[(slice(None),) + tuple(slice(a, b) for a, b in box)]
    XT, YT, ZT = (np.array(c[k]) for k in ("x_term", "y_term", "z_term"))
    hand = (XT[None, None, :] + YT[None, :, None] + ZT[:, None, None]) / c["scale"]
    assert up_box.shape[1:] == hand.shape
    assert np.max(np.abs(up_box[0] - hand)) < 1e-15

    # user labels: one on the border (overrides the sample), one inside,
    # a conflict on the border (keeps the sample) and one inside (unseeded)
    lab = np.full(border.shape, -1, np.int64)
    lab[0, 1, 2] = 1          # border, class 1 -> 1
    lab[2, 2, 2] = 0          # inside, class 0 -> 0
    lab[3, 1, 0] = -2         # border conflict -> parent sample
    lab[2, 1, 3] = -2         # inside conflict -> unseeded
    mask, xs = H.box_dirichlet(lab, border, up_box, 2)
    want_mask = want.copy()
    want_mask[2, 2, 2] = True
    assert np.array_equal(mask, want_mask)
    expect = hand.copy()
    expect[0, 1, 2] = 1.0
    expect[2, 2, 2] = 0.0
    assert np.max(np.abs(xs[0] - expect)) < 1e-15
    # three classes: a user label is 1 for its own class and 0 for the other
    up3 = np.stack([up_box[0], 0.5 * up_box[0]])
    lab3 = lab.copy()
    lab3[0, 1, 2] = 2
    m3, x3 = H.box_dirichlet(lab3, border, up3, 3)
    assert np.array_equal(m3, want_mask)
    assert x3[0][0, 1, 2] == 0.0 and x3[1][0, 1, 2] == 1.0
    assert x3[1][3, 1, 0] == 0.5 * hand[3, 1, 0]
    # warm start replaces only unseeded voxels
    start = np.full((1,) + border.shape, 0.25)
    mw, xw = H.box_dirichlet(lab, border, up_box, 2, start_box=start)
    assert np.array_equal(xw[0][want_mask], expect[want_mask])
    assert np.all(xw[0][~want_mask] == 0.25)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_interior_boxes_reproduce_affine_parent(axis):
    """beta = 0 (uniform weights).  Seeding the two faces of the coarsest
    level normal to `axis` with labels 0 and 1 makes its map affine along
    that axis.  Every level-0 box away from the volume faces then has all six
    faces seeded from an affine sample, so its discrete harmonic solution is
    that affine field: value ((X + 1/2)/2 - 1/2) / (n1 - 1) at child index X.
    A box sliced one voxel off, or along the wrong axis, fails."""
    dims = (16, 20, 24)                       # (z, y, x), level 0
    n1 = dims[axis] // 2
    other = [a for a in range(3) if a != axis]
    seeds = []
    for i in range(dims[other[0]] // 2):
        for j in range(dims[other[1]] // 2):
            for v, lab in ((0, 0), (n1 - 1, 1)):
                q = [0.0, 0.0, 0.0]           # (z, y, x) in level-0 units
                q[axis] = 2 * v + 0.5
                q[other[0]] = 2 * i + 0.5
                q[other[1]] = 2 * j + 0.5
                seeds.append([q[2], q[1], q[0], lab])
    seeds = np.array(seeds)
    vol = np.zeros(dims, np.float32)
    p = H.Params(levels=2, brick=4, expand=1.5, beta=0.0, eps=1e-6,
                 prune_hom=False, prune_dt=False)
    res = H.segment(vol, seeds, p)
    # the coarsest level is affine along the axis
    idx = np.arange(n1).reshape([-1 if a == axis else 1 for a in range(3)])
    assert np.max(np.abs(res.maps[1][0] - idx / (n1 - 1))) < 1e-12
    nb = H.brick_counts(dims, 4)
    X = np.arange(dims[axis]).reshape([-1 if a == axis else 1 for a in range(3)])
    field = np.broadcast_to(((X + 0.5) / 2 - 0.5) / (n1 - 1), dims)
    checked = 0
    for b in np.ndindex(nb):
        core, box = H.brick_box(b, dims, 4, 1.5)
        if any(lo == 0 or hi == d for (lo, hi), d in zip(box, dims)):
            continue
        assert res.computed[0][b]
        cs = H._sl(core)
        assert np.max(np.abs(res.maps[0][0][cs] - field[cs])) < 1e-12, b
        checked += 1
    assert checked == np.prod([n - 2 for n in nb])


def _loop_minmax(a):
    mn, mx = math.inf, -math.inf
    for v in np.asarray(a).ravel().tolist():
        mn = v if v < mn else mn
        mx = v if v > mx else mx
    return mn, mx


def test_binary_prune_tests_hand_cases_at_the_thresholds():
    p = H.Params(t_hom=0.25, t_bin=0.25, n_classes=2)
    c = lambda vals: np.array(vals, float).reshape(1, 1, 1, -1)
    assert H.prune_tests(c([0.25, 0.5]), p) == (False, False)      # range == t_hom: strict
    assert H.prune_tests(c([0.25, 0.375]), p) == (True, False)
    assert H.prune_tests(c([0.75, 0.875]), p) == (True, False)     # min - 0.5 == t_bin: strict
    assert H.prune_tests(c([0.875, 1.0]), p) == (True, True)       # foreground brick
    assert H.prune_tests(c([0.0, 0.125]), p) == (True, True)       # background brick
    assert H.prune_tests(c([0.0, 0.25]), p) == (False, False)      # 0.5 - max == t_bin: strict
    assert H.prune_tests(c([0.0, 1.0]), p) == (False, False)


def test_binary_prune_tests_against_loops():
    p = H.Params(t_hom=0.3, t_bin=0.01, n_classes=2)
    rng = np.random.default_rng(4)
    for _ in range(300):
        lo = rng.random()
        x = rng.uniform(lo, lo + rng.random() * (1 - lo), (1, 3, 4, 5))
        mn, mx = _loop_minmax(x[0])
        hom, dt = H.prune_tests(x, p)
        assert hom == (mx - mn < 0.3)
        assert dt == ((mn - 0.5 > 0.01) or (0.5 - mx > 0.01))


def test_multiclass_hom_includes_the_complement():
    """K = 3: both solved classes vary by 0.2 < t_hom, but together, so the
    complement 1 - x1 - x2 varies by 0.4 and the brick is not homogeneous."""
    p = H.Params(t_hom=0.3, n_classes=3)
    x1 = np.array([0.0, 0.1, 0.2]).reshape(1, 1, 3)
    m = np.stack([x1, x1])
    hom, dt = H.prune_tests(m, p)
    assert (hom, dt) == (False, False)
    # anti-correlated: complement constant 0.6, each class range 0.2 -> homogeneous
    m2 = np.stack([x1, 0.4 - x1])
    assert H.prune_tests(m2, p) == (True, False)
    # one class alone above t_hom
    m3 = np.stack([np.array([0.0, 0.35, 0.1]).reshape(1, 1, 3), 0.1 * np.ones((1, 1, 3))])
    assert H.prune_tests(m3, p)[0] is False
    # dt never applies to K > 2 (a brick entirely of class 1)
    m4 = np.stack([np.full((1, 1, 3), 0.95), np.full((1, 1, 3), 0.02)])
    assert H.prune_tests(m4, p) == (True, False)


def test_multiclass_prune_tests_against_loops():
    rng = np.random.default_rng(7)
    for K in (3, 4):
        p = H.Params(t_hom=0.3, n_classes=K)
        for _ in range(200):
            a = rng.random((K, 2, 3, 3)) ** rng.uniform(0.2, 5.0)
            a *= rng.uniform(0.0, 1.0, (K, 1, 1, 1))
            probs = a / a.sum(axis=0)
            core = probs[1:]
            ranges = []
            for k in range(K):
                cls = (1.0 - core.sum(axis=0)) if k == 0 else core[k - 1]
                mn, mx = _loop_minmax(cls)
                ranges.append(mx - mn)
            assert H.prune_tests(core, p) == (all(r < 0.3 for r in ranges), False)


# (expand, changed parent voxel (z, y, x), bricks per axis it reaches, bricks
# holding the new label's level-0 voxel (z, y, x) = (14, 2, 13)).  Level 0 is
# 16^3, s = 4.  The box of brick b along an axis and the parent voxels its
# trilinear sample reads (child X -> parent (X + 1/2)/2 - 1/2, two taps):
#   e = 1.5  (pads 1/1): [4b-1, 4b+5) -> 0..2, 1..4, 3..6, 5..7
#   e = 1.25 (pads 0/1): [4b, 4b+5)   -> 0..2, 1..4, 3..6, 5..7
#   e = 1.75 (pads 1/2): [4b-1, 4b+6) -> 0..3, 1..5, 3..7, 5..7
# (boxes clipped to [0, 16)).
DIRTY_CASES = [
    (1.5, (4, 2, 6), ((1, 2), (0, 1), (2, 3)), [(3, 0, 3)]),
    (1.25, (1, 3, 5), ((0, 1), (1, 2), (2, 3)), [(3, 0, 3)]),
    (1.75, (5, 0, 3), ((1, 2, 3), (0,), (0, 1, 2)), [(3, 0, 3), (3, 0, 2)]),
]


@pytest.mark.parametrize("expand,pv,reach,seed_bricks", DIRTY_CASES)
def test_dirty_rule_parent_region_hand_list(expand, pv, reach, seed_bricks):
    """Dirty-brick reading of Section IV-E: a change of the parent map at one
    parent voxel marks exactly the bricks whose box samples it, plus the
    bricks whose box holds the new label."""
    rng = np.random.default_rng(3)
    vol = (rng.random((16, 16, 16)) * 0.2 + 0.4).astype(np.float32)
    base = np.array([[1.5, 1.5, 1.5, 0], [14.5, 14.5, 14.5, 1], [3.5, 12.5, 8.5, 1]])
    new = np.array([[13.5, 2.5, 14.5, 0]])      # (x, y, z): level-0 voxel (z,y,x) = (14, 2, 13)
    p = H.Params(levels=2, brick=4, expand=expand, beta=32.0, prune_hom=False,
                 prune_dt=False, t_inc=0.01)
    seeds = np.concatenate([base, new])
    full = H.segment(vol, seeds, p)
    for delta, expect_region in ((0.05, True), (0.004, False)):
        prev = H.segment(vol, base, p)
        prev.maps[1] = full.maps[1].copy()
        prev.maps[1][(0,) + pv] += delta
        inc = H.segment(vol, seeds, p, prev=prev)
        want = np.zeros((4, 4, 4), bool)
        if expect_region:
            for bz in reach[0]:
                for by in reach[1]:
                    for bx in reach[2]:
                        want[bz, by, bx] = True
        for b in seed_bricks:
            want[b] = True
        assert np.array_equal(inc.recomputed[0], want), np.argwhere(inc.recomputed[0] != want)


def test_dirichlet_energy_hand_value():
    """Chain of 3 voxels, g = (0, 1/2, 1/2), beta = 4 ln 2, eps = 0: the two
    edge weights are 1/2 and 1; x = (0, 1, 3) gives D = (0.5*1 + 1*4)/2."""
    g = np.array([0.0, 0.5, 0.5]).reshape(1, 1, 3)
    x = np.array([0.0, 1.0, 3.0]).reshape(1, 1, 3)
    assert abs(rw.dirichlet_energy(g, x, 4 * math.log(2), 0.0) - 2.25) < 1e-15
    # the same along y and z
    assert abs(rw.dirichlet_energy(g.reshape(1, 3, 1), x.reshape(1, 3, 1), 4 * math.log(2), 0.0) - 2.25) < 1e-15
    assert abs(rw.dirichlet_energy(g.reshape(3, 1, 1), x.reshape(3, 1, 1), 4 * math.log(2), 0.0) - 2.25) < 1e-15
    # eps adds eps/2 * sum of squared differences
    assert abs(rw.dirichlet_energy(g, x, 4 * math.log(2), 0.125) - (2.25 + 0.0625 * 5)) < 1e-15
