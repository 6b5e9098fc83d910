"""Oracle: hierarchical random walker over the LOD pyramid (TEST INFRASTRUCTURE).

Paper: arXiv 2103.09564.  Plain Python loops over bricks, float64.

* Section III-A: the pyramid.  Level 0 is the input volume; level l+1 is the
  2x2x2 mean of level l (partial blocks at odd edges average the voxels they
  have).  Intensities are normalised once on level 0 (uint16: global min-max
  to [0, 1]; float: clipped to [0, 1]).  For the Poisson-noise weight of
  Section IV-C the levels hold the mean counts instead, each replaced by its
  square root (``pyramid_counts``); solved with beta = 1/2.
* Section IV-A, eq. (1): the coarsest level is solved with the user seeds only.
  Here the coarsest level is solved as one domain (the whole level).
* Section IV-A, eq. (2) and Section IV-B, eq. (3): every finer brick (s^3
  voxels) is expanded to a box of side floor(e*s) (low pad floor((s_e-s)/2),
  high pad the rest, clipped to the volume).  The outermost voxel layer of
  the box, on faces interior to the volume, receives continuous seeds sampled
  from the parent level; user seeds rasterised into the box are 0/1 seeds and
  override those.  The solution is contracted back to the s^3 core.
* Sampling the parent (Section IV-A) and warm start (Section IV-D2): trilinear
  interpolation at cell centres, child voxel X -> parent coordinate
  (X + 1/2)/2 - 1/2, clamped at the volume edge.  The unseeded voxels of the
  box start from that sample (root level: 0).
* Rasterisation and conflicts (Section IV-A, IV-D1): a label at full-resolution
  position q lands in level-l voxel floor(q / 2^l).  A voxel hit by labels of
  different value is left unseeded and marks every box containing it as in
  conflict (cfl).
* Pruning (Section IV-D1): hom(n) = max - min < t_hom; dt(n) = min - 0.5 >
  t_bin or 0.5 - max > t_bin; prunable = (hom or dt) and not cfl.  Children of
  a prunable brick are not processed; their region keeps the upsampled
  parent value, and since every level map is complete, border sampling for a
  neighbour falls back to the nearest computed ancestor.
* Multi-class (Section III-B): classes 1..K-1 are solved as K-1 right-hand
  sides; class 0 is the complement.  hom must hold for every class; dt is a
  binary-segmentation test and only applies when K = 2.
* Incremental labelling (Section IV-E), as read here: level by level, a brick
  that the new run reaches is recomputed only if a newly added label lands
  in its box, if it was not computed in the previous result, or if the
  parent level map changed by at least t_inc (max abs difference) over the
  parent voxels the box samples; otherwise its previous core values and
  prunable flag are reused.  The coarsest level is recomputed iff any label
  was added.  This is the default ("dirty" rule).
* Incremental labelling, the paper's own node rule (inc_rule = "node",
  Section IV-E): every brick the new run reaches under a parent that was not
  taken over from the previous result is solved; if its new core is within
  t_inc of its previous core (max abs difference over the core voxels and
  classes) and no voxel of its box has a seed conflict involving a newly
  added label, the new node is discarded: the brick takes its previous core
  values and prunable flag, and every descendant it had in the previous
  result is taken over too (copied, not solved).  The coarsest level is
  always solved; each of its bricks is such a node.
* Warm start from the previous result (inc_warm, Section IV-E, after Grady):
  a brick solved in an incremental run starts its unseeded voxels from the
  previous result's map of the same level instead of the parent sample (the
  border values still come from the parent); the solution does not depend
  on the start.
"""

from dataclasses import dataclass, field
import numpy as np

from .rw import solve_box


@dataclass
class Params:
    beta: float = 128.0
    eps: float = 1e-6
    brick: int = 32          # s (Section IV-A)
    expand: float = 1.25     # e (Section IV-B)
    levels: int = 4          # pyramid levels including full resolution
    n_classes: int = 2       # K; binary = 2 (class 1 foreground)
    t_hom: float = 0.3       # Section IV-D1
    t_bin: float = 0.01      # Section IV-D1
    t_inc: float = 0.01      # Section IV-E
    prune_hom: bool = True
    prune_dt: bool = True
    inc_rule: str = "dirty"  # "dirty" or "node" (Section IV-E)
    inc_warm: bool = False   # incremental runs start solved boxes from the previous map
    method: str = "direct"   # per-box oracle solve
    tol: float = 1e-13       # used when method == "pcg"


@dataclass
class Result:
    params: Params
    dims: list                      # per level (Dz, Dy, Dx)
    maps: list                      # per level float64 (K-1, Dz, Dy, Dx)
    computed: list                  # per level bool (nbz, nby, nbx)
    prunable: list                  # per level bool (nbz, nby, nbx)
    cfl: list                       # per level bool (nbz, nby, nbx)
    recomputed: list = field(default_factory=list)   # per level bool (incremental)
    seeds: np.ndarray = None
    reused: list = field(default_factory=list)       # per level bool (node rule: taken over from prev)


def normalize(volume, vrange=None):
    """Level-0 intensities in [0, 1] (float64).  ``vrange`` = (min, max) of
    the whole uint16 volume when ``volume`` is only a part of it."""
    v = np.asarray(volume)
    if v.dtype == np.uint16:
        v = v.astype(np.float64)
        lo, hi = (v.min(), v.max()) if vrange is None else (float(vrange[0]), float(vrange[1]))
        return (v - lo) / (hi - lo) if hi > lo else np.zeros_like(v)
    return np.clip(v.astype(np.float64), 0.0, 1.0)


def downsample2x(a):
    """2x2x2 mean of the voxels each block has (Section III-A)."""
    a = np.asarray(a, dtype=np.float64)
    nz, ny, nx = a.shape
    out = np.zeros(((nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2))
    cnt = np.zeros_like(out)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                s = a[dz::2, dy::2, dx::2]
                out[:s.shape[0], :s.shape[1], :s.shape[2]] += s
                cnt[:s.shape[0], :s.shape[1], :s.shape[2]] += 1
    return out / cnt


def pyramid(volume, levels):
    g = [normalize(volume)]
    for _ in range(levels - 1):
        g.append(downsample2x(g[-1]))
    return g


def pyramid_counts(volume, levels):
    """Pyramid for the Poisson-noise weight (Section IV-C): the levels of
    the counts n (uint16 as is, float clipped below at 0; level l+1 the 2x2x2
    mean of level l), each replaced by sqrt(n).  The paper's weight
    exp(-(sqrt n_p - sqrt n_q)^2 / 2) is then the Gaussian weight of these
    values with beta = 1/2 (eps as in every solve here)."""
    n = np.asarray(volume)
    n = n.astype(np.float64) if n.dtype == np.uint16 else np.maximum(n.astype(np.float64), 0.0)
    c = [n]
    for _ in range(levels - 1):
        c.append(downsample2x(c[-1]))
    return [np.sqrt(a) for a in c]


def _axis_taps(n_child, n_parent):
    """Per child index X: (i0, i1, t) with value = (1-t)*p[i0] + t*p[i1]."""
    P = (np.arange(n_child) + 0.5) / 2.0 - 0.5
    P = np.clip(P, 0.0, n_parent - 1)
    i0 = np.floor(P).astype(np.int64)
    i0 = np.minimum(i0, max(n_parent - 2, 0))
    i1 = np.minimum(i0 + 1, n_parent - 1)
    t = P - i0
    return i0, i1, t


def upsample(parent, child_shape):
    """Trilinear sample of ``parent`` (.., Pz, Py, Px) at every child voxel."""
    parent = np.asarray(parent, dtype=np.float64)
    out = parent
    for axis, n in zip((-3, -2, -1), child_shape):
        i0, i1, t = _axis_taps(n, parent.shape[axis])
        a0 = np.take(out, i0, axis=axis)
        a1 = np.take(out, i1, axis=axis)
        shape = [1] * out.ndim
        shape[axis] = n
        tt = t.reshape(shape)
        out = (1.0 - tt) * a0 + tt * a1
    return out


def upsample_box(parent, child_shape, box, origin=(0, 0, 0), parent_shape=None):
    """``upsample(parent, child_shape)`` restricted to ``box`` ((lo, hi) per
    axis z, y, x): the same per-axis taps, evaluated only at the box's child
    voxels (for levels too large to upsample whole).  ``parent`` may be a
    crop of the parent level that starts at voxel ``origin`` of a level of
    spatial shape ``parent_shape`` (the taps follow the whole level); the
    crop must hold every parent voxel the box's taps use."""
    parent = np.asarray(parent, dtype=np.float64)
    if parent_shape is None:
        parent_shape = parent.shape[-3:]
    out = parent
    for axis, n, (lo, hi), o, npar in zip((-3, -2, -1), child_shape, box, origin, parent_shape):
        i0, i1, t = _axis_taps(n, npar)
        i0, i1, t = i0[lo:hi] - o, i1[lo:hi] - o, t[lo:hi]
        if i0.min() < 0 or i1.max() >= out.shape[axis]:
            raise ValueError("the parent crop does not cover the box")
        a0 = np.take(out, i0, axis=axis)
        a1 = np.take(out, i1, axis=axis)
        shape = [1] * out.ndim
        shape[axis] = hi - lo
        tt = t.reshape(shape)
        out = (1.0 - tt) * a0 + tt * a1
    return out


def rasterize(seeds, level, dims):
    """Level-l seed grid: -1 unseeded, k >= 0 class k, -2 conflict."""
    lab = np.full(dims, -1, dtype=np.int64)
    if seeds is None or len(seeds) == 0:
        return lab
    s = np.asarray(seeds, dtype=np.float64)
    f = 2.0 ** level
    vx = np.floor(s[:, 0] / f).astype(np.int64)
    vy = np.floor(s[:, 1] / f).astype(np.int64)
    vz = np.floor(s[:, 2] / f).astype(np.int64)
    for x, y, z, k in zip(vx, vy, vz, s[:, 3].astype(np.int64)):
        if not (0 <= z < dims[0] and 0 <= y < dims[1] and 0 <= x < dims[2]):
            continue
        cur = lab[z, y, x]
        if cur == -1:
            lab[z, y, x] = k
        elif cur >= 0 and cur != k:
            lab[z, y, x] = -2
    return lab


def rasterize_box(seeds, level, dims, box):
    """``rasterize(seeds, level, dims)`` restricted to ``box`` ((lo, hi) per
    axis z, y, x), without building the whole level's grid."""
    shape = tuple(hi - lo for lo, hi in box)
    lab = np.full(shape, -1, dtype=np.int64)
    if seeds is None or len(seeds) == 0:
        return lab
    s = np.asarray(seeds, dtype=np.float64)
    f = 2.0 ** level
    v = [np.floor(s[:, a] / f).astype(np.int64) for a in (2, 1, 0)]   # z, y, x
    inside = np.ones(len(s), dtype=bool)
    for a in range(3):
        inside &= (v[a] >= box[a][0]) & (v[a] < box[a][1]) & (v[a] >= 0) & (v[a] < dims[a])
    for i in np.flatnonzero(inside):
        z, y, x, k = v[0][i] - box[0][0], v[1][i] - box[1][0], v[2][i] - box[2][0], int(s[i, 3])
        cur = lab[z, y, x]
        if cur == -1:
            lab[z, y, x] = k
        elif cur >= 0 and cur != k:
            lab[z, y, x] = -2
    return lab


def brick_counts(dims, s):
    return tuple((d + s - 1) // s for d in dims)


def brick_box(b, dims, s, e):
    """Core and box of brick b=(bz,by,bx): lists of (lo, hi) per axis (z,y,x)."""
    se = int(np.floor(e * s))
    lo_pad = (se - s) // 2
    hi_pad = se - s - lo_pad
    core, box = [], []
    for bi, d in zip(b, dims):
        c0, c1 = bi * s, min((bi + 1) * s, d)
        core.append((c0, c1))
        box.append((max(c0 - lo_pad, 0), min(c1 + hi_pad, d)))
    return core, box


def _sl(r):
    return tuple(slice(a, b) for a, b in r)


def prune_tests(core_maps, p):
    """(hom, dt) of a contracted brick (Section IV-D1); core_maps (K-1, ...)."""
    K = p.n_classes
    if K == 2:
        x = core_maps[0]
        hom = (x.max() - x.min()) < p.t_hom
        dt = (x.min() - 0.5 > p.t_bin) or (0.5 - x.max() > p.t_bin)
        return bool(hom), bool(dt)
    comp = 1.0 - core_maps.sum(axis=0)
    allk = np.concatenate([comp[None], core_maps], axis=0)
    hom = all((c.max() - c.min()) < p.t_hom for c in allk)
    return bool(hom), False


def _prunable(core_maps, cfl, p):
    hom, dt = prune_tests(core_maps, p)
    return ((p.prune_hom and hom) or (p.prune_dt and dt)) and not cfl


def box_dirichlet(lab_box, border, up_box, n_classes, start_box=None):
    """Dirichlet data and start values of one box (Section IV-A eq. (2),
    Section IV-B eq. (3), Section IV-D2).

    lab_box: rasterised labels over the box (-1 none, -2 conflict, k class);
    border: the box's outer layer on faces interior to the level; up_box:
    the parent map sampled at the box voxels, (K-1, *box), or None (coarsest
    level).  A voxel is seeded when it carries a user label or lies on the
    border; a user label overrides the border sample (value 1 for its own
    class, 0 otherwise); a conflicting voxel carries no label, so on the
    border it keeps the parent sample.  Unseeded voxels start from the parent
    sample, or from ``start_box`` when given (warm start from a previous
    result).  Returns (mask, x) with x of shape (K-1, *box)."""
    seeded = lab_box >= 0
    mask = seeded | border
    x = np.zeros((n_classes - 1,) + lab_box.shape)
    for k in range(1, n_classes):
        xk = up_box[k - 1].copy() if up_box is not None else np.zeros(lab_box.shape)
        if start_box is not None:
            xk[~mask] = start_box[k - 1][~mask]
        xk[seeded] = (lab_box[seeded] == k).astype(np.float64)
        x[k - 1] = xk
    return mask, x


def _solve(g_box, lab_box, border, up_box, p, start_box=None):
    """One box: the Dirichlet problem of ``box_dirichlet`` solved per class;
    returns (K-1, *box)."""
    mask, x = box_dirichlet(lab_box, border, up_box, p.n_classes, start_box)
    out = np.zeros_like(x)
    for k in range(p.n_classes - 1):
        out[k] = solve_box(g_box, mask, x[k], p.beta, p.eps, method=p.method, tol=p.tol)
    return out


def segment(volume, seeds, p, prev=None, g=None):
    """Hierarchical random walker (eqs. 1-3 with pruning and Section IV-E).

    volume: level-0 array (uint16 or float); seeds: (n, 4) array of
    (x, y, z, label) with x, y, z in full-resolution voxel units.  ``g`` may
    pass a precomputed pyramid.  Returns a ``Result``.
    """
    if g is None:
        g = pyramid(volume, p.levels)
    if prev is not None and p.inc_rule == "node":
        return _segment_node_rule(g, seeds, p, prev)
    if p.inc_rule not in ("dirty", "node"):
        raise ValueError("inc_rule must be 'dirty' or 'node'")
    K = p.n_classes
    top = p.levels - 1
    dims = [gl.shape for gl in g]
    seeds = np.zeros((0, 4)) if seeds is None else np.asarray(seeds, dtype=np.float64)
    new_seeds = seeds
    if prev is not None:
        old = {tuple(r) for r in np.asarray(prev.seeds).tolist()}
        new_seeds = np.array([r for r in seeds.tolist() if tuple(r) not in old]).reshape(-1, 4)
    L = p.levels
    maps = [None] * L
    computed = [None] * L
    prunable = [None] * L
    cfl = [None] * L
    recomputed = [None] * L

    def cfl_grid(lab, d):
        nb = brick_counts(d, p.brick)
        c = np.zeros(nb, dtype=bool)
        conf = lab == -2
        for b in np.ndindex(nb):
            _, box = brick_box(b, d, p.brick, p.expand)
            c[b] = bool(conf[_sl(box)].any())
        return c

    # coarsest level: one domain, user seeds only (eq. 1)
    lab = rasterize(seeds, top, dims[top])
    cfl[top] = cfl_grid(lab, dims[top])
    nb = brick_counts(dims[top], p.brick)
    if prev is not None and len(new_seeds) == 0:
        maps[top] = prev.maps[top].copy()
        recomputed[top] = np.zeros(nb, dtype=bool)
    else:
        border = np.zeros(dims[top], dtype=bool)
        maps[top] = _solve(g[top], lab, border, None, p)
        recomputed[top] = np.ones(nb, dtype=bool)
    computed[top] = np.ones(nb, dtype=bool)
    prunable[top] = np.zeros(nb, dtype=bool)
    for b in np.ndindex(nb):
        core, _ = brick_box(b, dims[top], p.brick, p.expand)
        prunable[top][b] = _prunable(maps[top][(slice(None),) + _sl(core)], cfl[top][b], p)

    for lvl in range(top - 1, -1, -1):
        d = dims[lvl]
        up = upsample(maps[lvl + 1], d)
        maps[lvl] = up.copy()
        lab = rasterize(seeds, lvl, d)
        lab_new = rasterize(new_seeds, lvl, d) if prev is not None else None
        cfl[lvl] = cfl_grid(lab, d)
        nb = brick_counts(d, p.brick)
        computed[lvl] = np.zeros(nb, dtype=bool)
        prunable[lvl] = np.zeros(nb, dtype=bool)
        recomputed[lvl] = np.zeros(nb, dtype=bool)
        if prev is not None:
            change = np.abs(maps[lvl + 1] - prev.maps[lvl + 1]).max(axis=0)
        for b in np.ndindex(nb):
            pb = tuple(i // 2 for i in b)
            if not computed[lvl + 1][pb] or prunable[lvl + 1][pb]:
                continue
            core, box = brick_box(b, d, p.brick, p.expand)
            computed[lvl][b] = True
            if prev is not None and prev.computed[lvl][b]:
                new_in_box = bool((lab_new[_sl(box)] != -1).any())
                pr = [(max((lo - 1) // 2, 0), min(hi // 2, dp - 1) + 1)
                      for (lo, hi), dp in zip(box, dims[lvl + 1])]
                changed = bool(change[_sl(pr)].max() >= p.t_inc)
                if not new_in_box and not changed:
                    maps[lvl][(slice(None),) + _sl(core)] = prev.maps[lvl][(slice(None),) + _sl(core)]
                    prunable[lvl][b] = prev.prunable[lvl][b]
                    continue
            recomputed[lvl][b] = True
            start = prev.maps[lvl][(slice(None),) + _sl(box)] if prev is not None and p.inc_warm else None
            xb = _solve(g[lvl][_sl(box)], lab[_sl(box)], border_layer(box, d),
                        up[(slice(None),) + _sl(box)], p, start)
            rel = tuple(slice(c0 - b0, c1 - b0) for (c0, c1), (b0, _) in zip(core, box))
            maps[lvl][(slice(None),) + _sl(core)] = xb[(slice(None),) + rel]
            prunable[lvl][b] = _prunable(maps[lvl][(slice(None),) + _sl(core)], cfl[lvl][b], p)

    return Result(params=p, dims=dims, maps=maps, computed=computed, prunable=prunable,
                  cfl=cfl, recomputed=recomputed, seeds=seeds.copy())


def border_layer(box, d):
    """Outermost voxel layer of a box on faces interior to the level
    (Section IV-A eq. (2)); box: (lo, hi) per axis (z, y, x), d: level dims."""
    border = np.zeros(tuple(hi - lo for lo, hi in box), dtype=bool)
    for ax, ((lo, hi), dl) in enumerate(zip(box, d)):
        idx = [slice(None)] * 3
        if lo > 0:
            idx[ax] = 0
            border[tuple(idx)] = True
        if hi < dl:
            idx[ax] = -1
            border[tuple(idx)] = True
    return border


def _segment_node_rule(g, seeds, p, prev):
    """Incremental run with the paper's node rule (Section IV-E): solve a
    reached node, then keep the previous node and its subtree instead when
    the two cores are within t_inc and no conflict involves a new label."""
    K = p.n_classes
    top = p.levels - 1
    dims = [gl.shape for gl in g]
    seeds = np.zeros((0, 4)) if seeds is None else np.asarray(seeds, dtype=np.float64)
    old = {tuple(r) for r in np.asarray(prev.seeds).tolist()}
    new_seeds = np.array([r for r in seeds.tolist() if tuple(r) not in old]).reshape(-1, 4)
    L = p.levels
    maps, computed, prunable, cfl, recomputed, reused = ([None] * L for _ in range(6))

    def grids(lvl):
        d = dims[lvl]
        lab = rasterize(seeds, lvl, d)
        lab_new = rasterize(new_seeds, lvl, d)
        nb = brick_counts(d, p.brick)
        c = np.zeros(nb, dtype=bool)
        c_new = np.zeros(nb, dtype=bool)   # a conflict that involves a new label
        conf = lab == -2
        conf_new = conf & (lab_new != -1)
        for b in np.ndindex(nb):
            _, box = brick_box(b, d, p.brick, p.expand)
            c[b] = bool(conf[_sl(box)].any())
            c_new[b] = bool(conf_new[_sl(box)].any())
        return lab, nb, c, c_new

    def close(lvl, core):
        cs = (slice(None),) + _sl(core)
        return float(np.abs(maps[lvl][cs] - prev.maps[lvl][cs]).max()) < p.t_inc

    def take_over(lvl, b, core):
        cs = (slice(None),) + _sl(core)
        maps[lvl][cs] = prev.maps[lvl][cs]
        prunable[lvl][b] = prev.prunable[lvl][b]
        reused[lvl][b] = True

    # coarsest level: one domain (eq. 1); each brick is a node
    lab, nb, cfl[top], c_new = grids(top)
    start = prev.maps[top] if p.inc_warm else None
    maps[top] = _solve(g[top], lab, np.zeros(dims[top], dtype=bool), None, p, start)
    computed[top] = np.ones(nb, dtype=bool)
    recomputed[top] = np.ones(nb, dtype=bool)
    prunable[top] = np.zeros(nb, dtype=bool)
    reused[top] = np.zeros(nb, dtype=bool)
    for b in np.ndindex(nb):
        core, _ = brick_box(b, dims[top], p.brick, p.expand)
        if close(top, core) and not c_new[b]:
            take_over(top, b, core)
        else:
            prunable[top][b] = _prunable(maps[top][(slice(None),) + _sl(core)], cfl[top][b], p)

    for lvl in range(top - 1, -1, -1):
        d = dims[lvl]
        up = upsample(maps[lvl + 1], d)
        maps[lvl] = up.copy()
        lab, nb, cfl[lvl], c_new = grids(lvl)
        computed[lvl] = np.zeros(nb, dtype=bool)
        prunable[lvl] = np.zeros(nb, dtype=bool)
        recomputed[lvl] = np.zeros(nb, dtype=bool)
        reused[lvl] = np.zeros(nb, dtype=bool)
        for b in np.ndindex(nb):
            pb = tuple(i // 2 for i in b)
            if not computed[lvl + 1][pb] or prunable[lvl + 1][pb]:
                continue
            core, box = brick_box(b, d, p.brick, p.expand)
            computed[lvl][b] = True
            if reused[lvl + 1][pb] and prev.computed[lvl][b]:
                take_over(lvl, b, core)          # a descendant of a node taken over
                continue
            recomputed[lvl][b] = True
            start = prev.maps[lvl][(slice(None),) + _sl(box)] if p.inc_warm else None
            xb = _solve(g[lvl][_sl(box)], lab[_sl(box)], border_layer(box, d),
                        up[(slice(None),) + _sl(box)], p, start)
            rel = tuple(slice(c0 - b0, c1 - b0) for (c0, c1), (b0, _) in zip(core, box))
            maps[lvl][(slice(None),) + _sl(core)] = xb[(slice(None),) + rel]
            if prev.computed[lvl][b] and close(lvl, core) and not c_new[b]:
                take_over(lvl, b, core)
            else:
                prunable[lvl][b] = _prunable(maps[lvl][(slice(None),) + _sl(core)], cfl[lvl][b], p)

    return Result(params=p, dims=dims, maps=maps, computed=computed, prunable=prunable,
                  cfl=cfl, recomputed=recomputed, seeds=seeds.copy(), reused=reused)


def probabilities(res, level=0):
    """All K class probabilities at a level (class 0 = complement)."""
    m = res.maps[level]
    return np.concatenate([(1.0 - m.sum(axis=0))[None], m], axis=0)


def labels(res, level=0):
    """Argmax class per voxel, lowest index on ties (Section III-B)."""
    return np.argmax(probabilities(res, level), axis=0).astype(np.uint8)
