"""Pins of the oracle's node rule for incremental runs (Section IV-E) and of
the warm start from the previous result.

The node rule solves a reached node, compares it with its previous version
and keeps the previous node and subtree when they are within t_inc and no
conflict involves a new label.  Checked here against what fixes it without
retyping it: an independent full run (at the coarsest level the rule's new
solution is the full run's), the two threshold limits (t_inc = 0 never
keeps, a huge t_inc keeps the whole previous tree) and the subtree property.
"""

import numpy as np
import pytest

from oracle import hierarchy as H
from test_oracle_hierarchy import _toy_seeds, _toy_volume


@pytest.fixture(scope="module")
def case():
    vol = _toy_volume(24)
    seeds = _toy_seeds(24)
    p = H.Params(levels=3, brick=8, beta=64.0, t_bin=0.49, prune_hom=False, prune_dt=True, inc_rule="node")
    prev = H.segment(vol, seeds, p)
    more = np.concatenate([seeds, [[20.0, 4.0, 12.0, 1], [3.0, 20.0, 18.0, 0]]])
    return vol, seeds, more, p, prev


def _with(p, **kw):
    return H.Params(**{**p.__dict__, **kw})


def _cfl_new(seeds, new, lvl, dims, p):
    lab = H.rasterize(seeds, lvl, dims)
    lab_new = H.rasterize(new, lvl, dims)
    nb = H.brick_counts(dims, p.brick)
    out = np.zeros(nb, dtype=bool)
    for b in np.ndindex(nb):
        _, box = H.brick_box(b, dims, p.brick, p.expand)
        sl = tuple(slice(lo, hi) for lo, hi in box)
        out[b] = bool(((lab[sl] == -2) & (lab_new[sl] != -1)).any())
    return out


def test_zero_threshold_keeps_nothing_and_equals_full_run(case):
    vol, _, more, p, prev = case
    p0 = _with(p, t_inc=0.0)
    inc = H.segment(vol, more, p0, prev=prev)
    full = H.segment(vol, more, p0)
    for lvl in range(p.levels):
        assert not inc.reused[lvl].any()
        assert np.array_equal(inc.computed[lvl], full.computed[lvl])
        assert np.array_equal(inc.recomputed[lvl], full.computed[lvl])
        assert np.max(np.abs(inc.maps[lvl] - full.maps[lvl])) < 1e-13


def test_huge_threshold_keeps_the_whole_previous_tree(case):
    vol, seeds, more, p, prev = case
    new = more[len(seeds):]
    assert not _cfl_new(more, new, p.levels - 1, prev.dims[p.levels - 1], p).any()
    inc = H.segment(vol, more, _with(p, t_inc=1e9), prev=prev)
    for lvl in range(p.levels):
        assert np.array_equal(inc.maps[lvl], prev.maps[lvl])
        assert np.array_equal(inc.computed[lvl], prev.computed[lvl])
        assert np.array_equal(inc.prunable[lvl], prev.prunable[lvl])
    # only the coarsest level is solved; every other reached brick is taken over
    for lvl in range(p.levels - 1):
        assert not inc.recomputed[lvl].any()
        assert np.array_equal(inc.reused[lvl], inc.computed[lvl])


@pytest.fixture(scope="module")
def wide():
    """Brick 4 on a 32^3 volume, two levels: 64 bricks at the coarsest level."""
    vol = _toy_volume(32, seed=3)
    seeds = _toy_seeds(32)
    p = H.Params(levels=2, brick=4, beta=64.0, t_bin=0.49, prune_hom=False, prune_dt=True, inc_rule="node")
    prev = H.segment(vol, seeds, p)
    more = np.concatenate([seeds, [[29.0, 29.0, 5.0, 0]]])  # changes 2 of the 64 coarse bricks by >= 0.01
    return vol, seeds, more, p, prev


def test_coarsest_decisions_match_an_independent_full_run(wide):
    vol, seeds, more, p, prev = wide
    top = p.levels - 1
    inc = H.segment(vol, more, p, prev=prev)
    full = H.segment(vol, more, _with(p, inc_rule="dirty"))       # no prev: plain full run
    cnew = _cfl_new(more, more[len(seeds):], top, prev.dims[top], p)
    nb = H.brick_counts(prev.dims[top], p.brick)
    for b in np.ndindex(nb):
        core, _ = H.brick_box(b, prev.dims[top], p.brick, p.expand)
        cs = (slice(None),) + tuple(slice(lo, hi) for lo, hi in core)
        diff = np.abs(full.maps[top][cs] - prev.maps[top][cs]).max()
        assert inc.reused[top][b] == (diff < p.t_inc and not cnew[b])
        want = prev.maps[top][cs] if inc.reused[top][b] else full.maps[top][cs]
        assert np.max(np.abs(inc.maps[top][cs] - want)) < 1e-13
    assert inc.reused[top].any() and not inc.reused[top].all()   # the case exercises both outcomes


def test_descendants_of_kept_nodes_are_copied_not_solved(case):
    vol, _, more, p, prev = case
    inc = H.segment(vol, more, p, prev=prev)
    for lvl in range(p.levels - 1):
        for b in np.ndindex(inc.computed[lvl].shape):
            pb = tuple(i // 2 for i in b)
            if not inc.computed[lvl][b]:
                continue
            core, _ = H.brick_box(b, prev.dims[lvl], p.brick, p.expand)
            cs = (slice(None),) + tuple(slice(lo, hi) for lo, hi in core)
            if inc.reused[lvl + 1][pb]:
                assert inc.reused[lvl][b] and not inc.recomputed[lvl][b]
                assert np.array_equal(inc.maps[lvl][cs], prev.maps[lvl][cs])
                assert inc.prunable[lvl][b] == prev.prunable[lvl][b]
            else:
                assert inc.recomputed[lvl][b]
    # children exist exactly under computed, non-prunable parents
    for lvl in range(p.levels - 1):
        par = inc.computed[lvl + 1] & ~inc.prunable[lvl + 1]
        want = np.kron(par, np.ones((2, 2, 2), bool))[tuple(slice(0, n) for n in inc.computed[lvl].shape)]
        assert np.array_equal(inc.computed[lvl], want)


def test_conflict_with_a_new_label_blocks_the_take_over(case):
    vol, seeds, _, p, prev = case
    # a new background seed on the voxel of an existing foreground seed: a
    # conflict that involves a new label in every box holding that voxel
    q = seeds[seeds[:, 3] == 1][0]
    more = np.concatenate([seeds, [[q[0], q[1], q[2], 0]]])
    inc = H.segment(vol, more, _with(p, t_inc=1e9), prev=prev)
    top = p.levels - 1
    cnew = _cfl_new(more, more[len(seeds):], top, prev.dims[top], p)
    assert cnew.any()
    assert np.array_equal(inc.reused[top], ~cnew)


@pytest.mark.parametrize("rule", ["dirty", "node"])
def test_warm_start_leaves_the_solution_unchanged(case, rule):
    vol, _, more, p, prev = case
    a = H.segment(vol, more, _with(p, inc_rule=rule, method="pcg", tol=1e-13), prev=prev)
    b = H.segment(vol, more, _with(p, inc_rule=rule, method="pcg", tol=1e-13, inc_warm=True), prev=prev)
    for lvl in range(p.levels):
        assert np.array_equal(a.computed[lvl], b.computed[lvl])
        assert np.max(np.abs(a.maps[lvl] - b.maps[lvl])) < 1e-9
