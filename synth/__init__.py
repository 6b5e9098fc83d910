"""Seeded synthetic inputs for the brick-local random-walker solve.

This module holds no part of the method's arithmetic: it only draws volumes,
seeds and Dirichlet data.  Both the oracle (``oracle/``) and the HIP path
(``paper_2103_09564_amd``) take their inputs from here; neither is imported.

Conventions: a box array is indexed ``a[z, y, x]`` (C order, x fastest); a
box shape is written (nx, ny, nz).  Dirichlet data ``x`` is float32 with the
seed values on seeded voxels (mask != 0) and the initial guess (0) elsewhere.

Workloads (all numpy ``default_rng(seed)``):

* ``plain_sphere``   -- a single 64^3 float volume: sphere of radius 20 at the
  centre (0.7) on 0.3, plus iid Gaussian noise sigma 0.05, clipped to [0, 1];
  foreground seeds a 5^3 block at the centre, background seeds all six faces.
* ``stress_boxes``   -- thousands of boxes of mixed shape drawn uniformly from
  {32^3, 32x32x17, 32x9x32, 5x32x32, 16^3}; intensities are uniform noise
  smoothed by a Gaussian (sigma 2) and min-max scaled per box; each face is a
  Dirichlet face with probability 1/2 with U[0,1] values (the first face drawn
  keeps shared edge voxels); 1 % of the other voxels are seeds with value 0
  or 1; a box with no seed at all is drawn again.
* ``blob_boxes``     -- 32^3 boxes with two Gaussian blobs (sigma 6,
  amplitudes 0.6 and 0.4) plus noise sigma 0.03; foreground seeds a 3^3 block
  at blob 1, background seeds a 3^3 block at blob 2 and all six faces; the
  ground-truth mask is blob 1 above half its maximum.
* ``cells_volume``   -- the paper's synthetic "cells" scenario (Section VI-B):
  spheres of diameter in [S/2, S] (S = structure size x volume side) placed
  at random until they cover the requested fraction of the volume, no centre
  inside another sphere; 0.7 inside on 0.3 plus iid Gaussian noise; a
  foreground seed at each centre and two background seeds per sphere at
  twice its radius from the centre, outside every sphere.
"""

import numpy as np
from scipy import ndimage

STRESS_SHAPES = ((32, 32, 32), (32, 32, 17), (32, 9, 32), (5, 32, 32), (16, 16, 16))


def plain_sphere(seed=1, n=64, radius=20.0, noise=0.05):
    rng = np.random.default_rng(seed)
    c = (n - 1) / 2.0
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    inside = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 <= radius ** 2
    g = np.where(inside, 0.7, 0.3) + rng.normal(0.0, noise, (n, n, n))
    g = np.clip(g, 0.0, 1.0).astype(np.float32)
    mask = np.zeros((n, n, n), dtype=np.uint8)
    xd = np.zeros((n, n, n), dtype=np.float32)
    face = (x == 0) | (x == n - 1) | (y == 0) | (y == n - 1) | (z == 0) | (z == n - 1)
    mask[face] = 1
    lo, hi = int(np.floor(c)) - 1, int(np.floor(c)) + 4     # indices 30..34 for n=64
    mask[lo:hi, lo:hi, lo:hi] = 1
    xd[lo:hi, lo:hi, lo:hi] = 1.0
    return g, mask, xd, inside


def _smooth_noise(rng, shape, sigma=2.0, pad=6):
    nx, ny, nz = shape
    a = rng.random((nz + 2 * pad, ny + 2 * pad, nx + 2 * pad)).astype(np.float64)
    a = ndimage.gaussian_filter(a, sigma=sigma, mode="reflect", truncate=3.0)
    a = a[pad:pad + nz, pad:pad + ny, pad:pad + nx]
    lo, hi = a.min(), a.max()
    return ((a - lo) / (hi - lo)).astype(np.float32)


def _stress_dirichlet(rng, shape):
    nx, ny, nz = shape
    while True:
        mask = np.zeros((nz, ny, nx), dtype=np.uint8)
        x = np.zeros((nz, ny, nx), dtype=np.float32)
        faces = [(2, 0), (2, nx - 1), (1, 0), (1, ny - 1), (0, 0), (0, nz - 1)]
        on_face = np.zeros((nz, ny, nx), dtype=bool)
        for axis, pos in faces:
            idx = [slice(None)] * 3
            idx[axis] = pos
            idx = tuple(idx)
            on_face[idx] = True
            if rng.random() < 0.5:
                vals = rng.random(mask[idx].shape).astype(np.float32)
                free = mask[idx] == 0
                x[idx] = np.where(free, vals, x[idx])
                mask[idx] = 1
        inner = ~on_face
        pick = inner & (rng.random((nz, ny, nx)) < 0.01)
        bern = (rng.random((nz, ny, nx)) < 0.5).astype(np.float32)
        mask[pick] = 1
        x[pick] = bern[pick]
        if mask.any():
            return mask, x


def stress_boxes(n=8192, seed=3, shapes=STRESS_SHAPES):
    """Mixed-shape boxes, concatenated.

    Returns dict with ``shapes`` (n,3 int32: nx, ny, nz), ``offsets`` (n int64),
    flat ``g`` float32, ``mask`` uint8, ``x`` float32 and ``boxes`` = list of
    (g, mask, x) views for the oracle.
    """
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(shapes), n)
    shp = np.array([shapes[i] for i in pick], dtype=np.int32).reshape(n, 3)
    sizes = shp.prod(axis=1).astype(np.int64)
    offsets = np.zeros(n, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    g = np.empty(total, dtype=np.float32)
    mask = np.empty(total, dtype=np.uint8)
    x = np.empty(total, dtype=np.float32)
    for b in range(n):
        s = tuple(int(v) for v in shp[b])
        gb = _smooth_noise(rng, s)
        mb, xb = _stress_dirichlet(rng, s)
        o, m = offsets[b], sizes[b]
        g[o:o + m] = gb.ravel()
        mask[o:o + m] = mb.ravel()
        x[o:o + m] = xb.ravel()
    return pack(shp, offsets, g, mask, x)


def pack(shapes, offsets, g, mask, x):
    boxes = []
    for (nx, ny, nz), o in zip(shapes, offsets):
        m = int(nx) * int(ny) * int(nz)
        sl = slice(int(o), int(o) + m)
        boxes.append((g[sl].reshape(nz, ny, nx), mask[sl].reshape(nz, ny, nx), x[sl].reshape(nz, ny, nx)))
    return dict(shapes=np.asarray(shapes, dtype=np.int32), offsets=np.asarray(offsets, dtype=np.int64),
                g=g, mask=mask, x=x, boxes=boxes)


def from_boxes(box_list):
    """Concatenate a list of (g, mask, x) box arrays (each [z,y,x])."""
    shapes = np.array([[b[0].shape[2], b[0].shape[1], b[0].shape[0]] for b in box_list], dtype=np.int32)
    sizes = shapes.prod(axis=1).astype(np.int64)
    offsets = np.zeros(len(box_list), dtype=np.int64)
    if len(box_list) > 1:
        offsets[1:] = np.cumsum(sizes)[:-1]
    g = np.concatenate([np.asarray(b[0], np.float32).ravel() for b in box_list]) if box_list else np.zeros(0, np.float32)
    mask = np.concatenate([np.asarray(b[1], np.uint8).ravel() for b in box_list]) if box_list else np.zeros(0, np.uint8)
    x = np.concatenate([np.asarray(b[2], np.float32).ravel() for b in box_list]) if box_list else np.zeros(0, np.float32)
    return pack(shapes, offsets, g, mask, x)


def blob_boxes(n=512, seed=4, size=32, sigma=6.0, noise=0.03):
    """Two-blob boxes; returns the packed dict plus ``gt`` (flat uint8)."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(size), np.arange(size), np.arange(size), indexing="ij")
    pts = np.stack([x, y, z], axis=-1).astype(np.float64)
    out, gts = [], []
    for _ in range(n):
        while True:
            c1 = rng.uniform(10.0, 21.0, 3)
            c2 = rng.uniform(10.0, 21.0, 3)
            if np.linalg.norm(c1 - c2) >= 8.0:
                break
        G1 = np.exp(-((pts - c1) ** 2).sum(-1) / (2 * sigma ** 2))
        G2 = np.exp(-((pts - c2) ** 2).sum(-1) / (2 * sigma ** 2))
        g = (0.6 * G1 + 0.4 * G2 + rng.normal(0.0, noise, G1.shape)).astype(np.float32)
        mask = np.zeros(g.shape, dtype=np.uint8)
        xd = np.zeros(g.shape, dtype=np.float32)
        mask[0, :, :] = mask[-1, :, :] = mask[:, 0, :] = mask[:, -1, :] = mask[:, :, 0] = mask[:, :, -1] = 1
        for c, v in ((c2, 0.0), (c1, 1.0)):
            cx, cy, cz = np.round(c).astype(int)
            mask[cz - 1:cz + 2, cy - 1:cy + 2, cx - 1:cx + 2] = 1
            xd[cz - 1:cz + 2, cy - 1:cy + 2, cx - 1:cx + 2] = v
        out.append((g, mask, xd))
        gts.append((G1 > 0.5).astype(np.uint8))
    d = from_boxes(out)
    d["gt"] = np.concatenate([t.ravel() for t in gts])
    return d


def random_box(rng, shape, dirichlet_frac=0.05, smooth=1.0):
    """Small random box for tests: smooth noise intensities, random seeds
    (at least one), values U[0,1]."""
    nx, ny, nz = shape
    g = rng.random((nz, ny, nx))
    if smooth > 0:
        g = ndimage.gaussian_filter(g, smooth, mode="reflect")
        g = (g - g.min()) / max(g.max() - g.min(), 1e-12)
    mask = (rng.random((nz, ny, nx)) < dirichlet_frac).astype(np.uint8)
    if not mask.any():
        mask.flat[rng.integers(0, mask.size)] = 1
    x = np.where(mask != 0, rng.random((nz, ny, nx)), 0.0)
    return g.astype(np.float32), mask, x.astype(np.float32)


# ---------------------------------------------------------------------------
# Hierarchical pipeline volumes
# ---------------------------------------------------------------------------

def _catmull_rom(ctrl, step=1.0):
    """Points along the uniform Catmull-Rom spline through all control points
    (end points reflected), spaced <= step voxels.  A union of balls of radius
    r >= 2 about points 1 voxel apart is within 0.07 voxel of the swept tube."""
    P = np.asarray(ctrl, np.float64)
    P = np.concatenate([2 * P[:1] - P[1:2], P, 2 * P[-1:] - P[-2:-1]])
    out = []
    for i in range(1, len(P) - 2):
        p0, p1, p2, p3 = P[i - 1], P[i], P[i + 1], P[i + 2]
        # oversample by the control polygon length so spacing stays below step
        n = int(np.ceil((np.linalg.norm(p1 - p0) + np.linalg.norm(p2 - p1) + np.linalg.norm(p3 - p2)) / step)) + 2
        t = np.linspace(0.0, 1.0, n, endpoint=(i == len(P) - 3))[:, None]
        t2, t3 = t * t, t * t * t
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * t3))
    return np.concatenate(out)


def _tube_voxels(shape, pts, r):
    """Flat indices (array [z, y, x], voxel centres at integer indices) of the
    voxels within distance r of any of the points (x, y, z); an index may
    repeat."""
    nz, ny, nx = shape
    R = int(np.ceil(r)) + 1
    o = np.arange(-R, R + 1)
    off = np.stack(np.meshgrid(o, o, o, indexing="ij"), -1).reshape(-1, 3)  # (dx, dy, dz)
    off = off[np.sum((off - 0.5) ** 2, axis=1) <= (r + 1.8) ** 2]           # cannot reach r otherwise
    off = off.astype(np.int32)
    p32 = pts.astype(np.float32)
    base = np.floor(p32).astype(np.int32)
    frac = p32 - base                                                       # point within its base voxel
    found = []
    for c in range(0, len(pts), 512):
        d = off[None, :, :].astype(np.float32) - frac[c:c + 512, None, :]
        hit = np.einsum("ijk,ijk->ij", d, d) <= r * r
        b = (base[c:c + 512, None, :] + off[None, :, :])[hit]
        ok = (b[:, 0] >= 0) & (b[:, 0] < nx) & (b[:, 1] >= 0) & (b[:, 1] < ny) & (b[:, 2] >= 0) & (b[:, 2] < nz)
        b = b[ok].astype(np.int64)
        found.append((b[:, 2] * ny + b[:, 1]) * nx + b[:, 0])
    return np.concatenate(found) if found else np.zeros(0, np.int64)


def _smooth_field(rng, n, sigma, coarse=4):
    """Gaussian-smoothed white noise rescaled to [-1, 1].  For a wide kernel
    the noise is drawn at 1/coarse resolution, smoothed with sigma/coarse and
    trilinearly resampled (the smoothed field is band-limited far below the
    coarse grid's Nyquist rate)."""
    import torch
    m = max(4, n // coarse)
    a = ndimage.gaussian_filter(rng.standard_normal((m, m, m)), sigma / coarse, mode="wrap")
    t = torch.from_numpy(a.astype(np.float32))[None, None]
    t = torch.nn.functional.interpolate(t, size=(n, n, n), mode="trilinear", align_corners=False)[0, 0]
    f = t.numpy()
    lo, hi = float(f.min()), float(f.max())
    return (2.0 * (f - lo) / (hi - lo) - 1.0).astype(np.float32)


def tube_volume(n=512, n_tubes=40, n_fg=20, n_bg=200, seed=2):
    """uint16 volume of random tubes on a textured background, with seeds.

    Tubes: Catmull-Rom centrelines through 5 control points U[32, n-32]^3
    (scaled for small n), radius U[2, 8], intensity U[2700, 3300] per tube.
    Background 800 + 200 s(p), s a Gaussian-smoothed (sigma n/32) white-noise
    field in [-1, 1]; then iid N(0, 150^2), clip to [0, 65535], round.
    Seeds (x, y, z, label) in voxel units where voxel k covers [k, k+1):
    n_fg foreground points (label 1), one on each of the first n_fg tube
    centrelines; n_bg background points (label 0) uniform in the volume,
    redrawn when closer than radius + 4 to a centreline.

    Returns (vol [z, y, x] uint16, seeds float64 [k, 4], tube index map uint8
    [z, y, x]: 0 background, t + 1 inside tube t, later tubes on top)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    lo, hi = 32.0 * n / 512.0, n - 32.0 * n / 512.0
    tube = np.zeros((n, n, n), dtype=np.uint8)
    vol = 800.0 + 200.0 * _smooth_field(rng, n, sigma=16.0 * n / 512.0)
    curves, radii = [], []
    for t in range(n_tubes):
        ctrl = rng.uniform(lo, hi, (5, 3))
        r = rng.uniform(2.0, 8.0)
        inten = rng.uniform(2700.0, 3300.0)
        pts = _catmull_rom(ctrl)
        idx = _tube_voxels(tube.shape, pts, r)
        vol.reshape(-1)[idx] = inten
        tube.reshape(-1)[idx] = t + 1
        curves.append(pts)
        radii.append(r)
    vol += rng.standard_normal((n, n, n), dtype=np.float32) * 150.0
    vol = np.rint(np.clip(vol, 0.0, 65535.0)).astype(np.uint16)
    seeds = []
    for t in range(min(n_fg, n_tubes)):
        p = curves[t][rng.integers(0, len(curves[t]))]
        seeds.append([p[0] + 0.5, p[1] + 0.5, p[2] + 0.5, 1])
    trees = [cKDTree(c) for c in curves]
    while len(seeds) < min(n_fg, n_tubes) + n_bg:
        q = rng.uniform(0.0, n, 3)
        if all(tr.query(q - 0.5)[0] > r + 4.0 for tr, r in zip(trees, radii)):
            seeds.append([q[0], q[1], q[2], 0])
    return vol, np.array(seeds, dtype=np.float64), tube


def _rotation(rng):
    """Uniform random 3-D rotation (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _lattice_noise(rng, dims, wavelength):
    """Trilinear interpolation of iid N(0, 1) values on a lattice of the given
    spacing (voxels), sampled at the voxel centres of dims = (nx, ny, nz);
    returns [z, y, x] float32."""
    import torch
    nx, ny, nz = dims
    cells = [int(np.ceil(d / wavelength)) + 2 for d in (nz, ny, nx)]
    lat = torch.from_numpy(rng.standard_normal(cells).astype(np.float32))
    # voxel i sits at lattice coordinate (i + 0.5) / wavelength
    axes = [(torch.arange(d, dtype=torch.float32) + 0.5) / float(wavelength) for d in (nz, ny, nx)]
    out = torch.zeros((nz, ny, nx))
    i0 = [a.floor().long() for a in axes]
    f = [a - a.floor() for a in axes]
    for dz in (0, 1):
        wz = (f[0] if dz else 1 - f[0])[:, None, None]
        for dy in (0, 1):
            wy = (f[1] if dy else 1 - f[1])[None, :, None]
            for dx in (0, 1):
                wx = (f[2] if dx else 1 - f[2])[None, None, :]
                out += wz * wy * wx * lat[(i0[0] + dz)[:, None, None], (i0[1] + dy)[None, :, None],
                                          (i0[2] + dx)[None, None, :]]
    return out.numpy()


def shell_volume(dims=(256, 256, 128), seed=5, n_per_class=50, margin=None, fbm_std=100.0):
    """uint16 volume of 4 classes: background (mean 500) and three nested
    ellipsoids E1 > E2 > E3 (common centre jittered by +-5 % of dims, common
    random rotation; semi-axes a1 = U[.35, .45] dims, a2 = a1 U[.6, .75],
    a3 = a2 U[.5, .7] per axis); class 1 = E1 \\ E2 (1500), 2 = E2 \\ E3 (2500),
    3 = E3 (3500).  Plus iid N(0, 250^2) and a 6-octave fBm of trilinear
    lattice noise (base wavelength 512 voxels, amplitude halved per octave,
    total std fbm_std); clip, round.

    Seeds: n_per_class points per class, each at least `margin` voxels from
    the class's region boundaries (ellipsoid-radius bound; default 8 voxels
    at a 1024-voxel short side, scaled with it, at least 2).  Returns
    (vol [z, y, x] uint16, labels [z, y, x] uint8, seeds float64 [k, 4],
    geometry dict for stroke drawing)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    D = np.array([nx, ny, nz], np.float64)
    if margin is None:
        margin = max(2.0, 8.0 * min(dims) / 1024.0)
    c = D / 2.0 + rng.uniform(-0.05, 0.05, 3) * D
    Q = _rotation(rng)
    a1 = rng.uniform(0.35, 0.45, 3) * D
    a2 = a1 * rng.uniform(0.6, 0.75, 3)
    a3 = a2 * rng.uniform(0.5, 0.7, 3)
    axes = [a1, a2, a3]
    labels = np.zeros((nz, ny, nx), np.uint8)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    for z in range(nz):
        # voxel centres at integer indices; ellipsoid frame coordinates u = Q^T (p - c)
        P = np.stack(np.broadcast_arrays(xs[None, :], ys[:, None], np.float64(z)), -1) - c
        u = P @ Q
        for k, a in enumerate(axes):
            inside = np.sum((u / a) ** 2, axis=-1) <= 1.0
            labels[z][inside] = k + 1
    means = np.array([500.0, 1500.0, 2500.0, 3500.0], np.float32)
    vol = means[labels]
    fbm = np.zeros((nz, ny, nx), np.float32)
    amp, var = 1.0, 0.0
    for o in range(6):
        fbm += amp * _lattice_noise(rng, dims, 512.0 / 2 ** o)
        var += amp * amp
        amp *= 0.5
    vol += fbm * np.float32(fbm_std / np.sqrt(var))   # lattice noise variance < 1: std <= fbm_std
    vol += rng.standard_normal((nz, ny, nx), dtype=np.float32) * 250.0
    vol = np.rint(np.clip(vol, 0.0, 65535.0)).astype(np.uint16)

    def rho(p):  # ellipsoid radii of points p (x, y, z) in index space, per ellipsoid
        u = (np.atleast_2d(p) - c) @ Q
        return [np.sqrt(np.sum((u / a) ** 2, axis=-1)) for a in axes]

    def clearance(p):  # lower bound of the distance to every ellipsoid surface
        return np.min([np.abs(r - 1.0) * a.min() for r, a in zip(rho(p), axes)], axis=0)

    seeds = []
    for cls in range(4):
        got, tries = 0, 0
        while got < n_per_class:
            tries += 1
            if tries > 1000:
                raise RuntimeError(f"class {cls}: too few voxels {margin} away from the boundaries")
            p = rng.uniform(0.0, 1.0, (4096, 3)) * (D - 1)
            q = np.rint(p).astype(np.int64)
            ok = (labels[q[:, 2], q[:, 1], q[:, 0]] == cls) & (clearance(q.astype(np.float64)) >= margin)
            for v in q[ok][: n_per_class - got]:
                seeds.append([v[0] + 0.5, v[1] + 0.5, v[2] + 0.5, cls])
                got += 1
    geo = dict(centre=c, rotation=Q, axes=axes, clearance=clearance, margin=margin)
    return vol, labels, np.array(seeds, np.float64), geo


def stroke(labels, geo, cls=2, length=2000, seed=6):
    """Self-avoiding 6-neighbour walk of `length` voxels inside class `cls`,
    every voxel at least geo["margin"] from the region boundaries (a walk that
    gets stuck starts again elsewhere).  Returns seeds (x, y, z, cls) at the
    voxel centres."""
    rng = np.random.default_rng(seed)
    margin = geo["margin"]
    nz, ny, nx = labels.shape
    steps = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])

    def ok(v):
        return (0 <= v[0] < nx and 0 <= v[1] < ny and 0 <= v[2] < nz and labels[v[2], v[1], v[0]] == cls
                and geo["clearance"](v.astype(np.float64))[0] >= margin)

    for _ in range(100000):
        start = np.array([rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)])
        if not ok(start):
            continue
        path, seen = [start], {tuple(start)}
        while len(path) < length:
            cand = [path[-1] + s for s in steps[rng.permutation(6)]]
            nxt = next((v for v in cand if tuple(v) not in seen and ok(v)), None)
            if nxt is None:
                break
            path.append(nxt)
            seen.add(tuple(nxt))
        if len(path) == length:
            p = np.array(path, np.float64) + 0.5
            return np.concatenate([p, np.full((length, 1), float(cls))], axis=1)
    raise RuntimeError("no self-avoiding walk of the requested length found")


def cells_volume(n=256, seed=11, structure=0.1, coverage=0.01, noise=0.1, max_spheres=10000):
    """Cells scenario: float32 volume [z, y, x] in [0, 1], seeds (x, y, z,
    label) in voxel units (voxel k covers [k, k+1)), and the ground truth
    (uint8, 1 inside a sphere).  Sphere diameters are U[S/2, S] with
    S = structure * n; spheres are added until at least ``coverage`` of the
    voxels is inside one (a centre may not fall inside an earlier sphere)."""
    rng = np.random.default_rng(seed)
    S = structure * n
    truth = np.zeros((n, n, n), dtype=np.uint8)
    centres, radii = [], []
    target = coverage * n ** 3
    count = 0
    tries = 0
    while count < target and len(centres) < max_spheres and tries < 50 * max_spheres:
        tries += 1
        r = rng.uniform(S / 4.0, S / 2.0)
        c = rng.uniform(r, n - r, 3)
        if any(np.sum((c - q) ** 2) < rq * rq for q, rq in zip(centres, radii)):
            continue
        lo = np.maximum(np.floor(c - r).astype(np.int64), 0)
        hi = np.minimum(np.ceil(c + r).astype(np.int64) + 1, n)
        zz, yy, xx = np.meshgrid(*(np.arange(lo[a], hi[a]) + 0.5 for a in (2, 1, 0)), indexing="ij")
        inside = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= r * r
        sub = truth[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        count += int(np.sum(inside & (sub == 0)))
        sub[inside] = 1
        centres.append(c)
        radii.append(r)
    vol = 0.3 + 0.4 * truth.astype(np.float32) + rng.standard_normal((n, n, n), dtype=np.float32) * noise
    vol = np.clip(vol, 0.0, 1.0).astype(np.float32)
    seeds = []
    for c, r in zip(centres, radii):
        seeds.append([c[0], c[1], c[2], 1])
        placed = 0
        for _ in range(100):
            if placed == 2:
                break
            d = rng.standard_normal(3)
            q = c + 2.0 * r * d / np.linalg.norm(d)
            if np.any(q < 0.0) or np.any(q >= n):
                continue
            if any(np.sum((q - c2) ** 2) <= r2 * r2 for c2, r2 in zip(centres, radii)):
                continue
            seeds.append([q[0], q[1], q[2], 0])
            placed += 1
    return vol, np.array(seeds, dtype=np.float64), truth


def _segment_mask(shape, a, b, r):
    """Voxels (centres at index + 0.5) within distance r of segment a-b:
    (lo, hi, mask) over the segment's bounding box, coordinates (x, y, z)."""
    n = np.array(shape[::-1])
    lo = np.maximum(np.floor(np.minimum(a, b) - r).astype(np.int64), 0)
    hi = np.minimum(np.ceil(np.maximum(a, b) + r).astype(np.int64) + 1, n)
    if np.any(hi <= lo):
        return lo, hi, None
    zz, yy, xx = np.meshgrid(*(np.arange(lo[k], hi[k]) + 0.5 for k in (2, 1, 0)), indexing="ij")
    p = np.stack([xx, yy, zz], -1)
    ab = b - a
    t = np.clip(((p - a) @ ab) / max(float(ab @ ab), 1e-12), 0.0, 1.0)
    d2 = np.sum((p - (a + t[..., None] * ab)) ** 2, axis=-1)
    return lo, hi, d2 <= r * r


def vessels_volume(n=256, seed=12, structure=0.1, coverage=0.01, noise=0.1, max_trees=200, min_radius=1.0):
    """Vessels scenario: trees of cylindrical segments with spheres at the
    branch points.  A tree starts at a random point of the volume border,
    heading inwards, with a diameter in [S/2, S] (S = structure * n); a
    segment is 5 radii long and then branches into two segments whose radii
    keep the cross-section area (r / sqrt 2), turned 35 degrees either side
    about a random axis normal to the parent; branches stop below
    `min_radius` or outside the volume.  Trees are added until `coverage` of
    the voxels is inside a vessel.  Labels: per segment two points on its
    centreline (foreground) and, for each, a point two radii away normal to
    the segment (background, dropped if it lands inside a vessel or outside
    the volume).  Intensities 0.7 in vessels, 0.3 elsewhere, plus Gaussian
    noise, clipped to [0, 1].  Returns (vol float32 [z, y, x], seeds float64
    (x, y, z, label), truth uint8)."""
    rng = np.random.default_rng(seed)
    S = structure * n
    truth = np.zeros((n, n, n), dtype=np.uint8)
    segs = []
    target = coverage * n ** 3
    count = 0

    def paint(a, b, r):
        nonlocal count
        lo, hi, m = _segment_mask(truth.shape, a, b, r)
        if m is None:
            return
        sub = truth[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        count += int(np.sum(m & (sub == 0)))
        sub[m] = 1

    def normal_to(d):
        v = rng.standard_normal(3)
        v -= (v @ d) * d
        return v / np.linalg.norm(v)

    trees = 0
    while count < target and trees < max_trees:
        trees += 1
        r0 = rng.uniform(S / 4.0, S / 2.0)
        face = rng.integers(0, 6)
        axis, side = face // 2, face % 2
        p = rng.uniform(0.0, n, 3)
        p[axis] = 0.0 if side == 0 else float(n)
        d = np.zeros(3)
        d[axis] = 1.0 if side == 0 else -1.0
        d = d + 0.3 * normal_to(d)
        d /= np.linalg.norm(d)
        stack = [(p, d, r0)]
        while stack and count < target:
            a, d, r = stack.pop()
            if r < min_radius:
                continue
            b = a + 5.0 * r * d
            paint(a, b, r)
            paint(b, b, r)                       # sphere at the branch point
            segs.append((a, b, r))
            if np.all(b >= 0) and np.all(b < n):
                ax = normal_to(d)
                c, s = np.cos(np.radians(35.0)), np.sin(np.radians(35.0))
                for sign in (1.0, -1.0):
                    dn = c * d + sign * s * ax
                    stack.append((b, dn / np.linalg.norm(dn), r / np.sqrt(2.0)))
    vol = 0.3 + 0.4 * truth.astype(np.float32) + rng.standard_normal((n, n, n), dtype=np.float32) * noise
    vol = np.clip(vol, 0.0, 1.0).astype(np.float32)
    seeds = []
    for a, b, r in segs:
        nrm = normal_to((b - a) / np.linalg.norm(b - a))
        for t in (0.25, 0.75):
            q = a + t * (b - a)
            if np.any(q < 0) or np.any(q >= n):
                continue
            seeds.append([q[0], q[1], q[2], 1])
            o = q + 2.0 * r * nrm
            oi = np.floor(o).astype(np.int64)
            if np.all(o >= 0) and np.all(o < n) and truth[oi[2], oi[1], oi[0]] == 0:
                seeds.append([o[0], o[1], o[2], 0])
    return vol, np.array(seeds, dtype=np.float64), truth


def shell_geometry(dims, seed=5):
    """The nested-shell geometry of ``shell_volume`` (same draws, same order):
    centre, rotation and semi-axes, plus a label function of voxel centres
    (integer indices, arrays of x, y, z) and the clearance bound."""
    rng = np.random.default_rng(seed)
    D = np.array(dims, np.float64)
    c = D / 2.0 + rng.uniform(-0.05, 0.05, 3) * D
    Q = _rotation(rng)
    a1 = rng.uniform(0.35, 0.45, 3) * D
    a2 = a1 * rng.uniform(0.6, 0.75, 3)
    a3 = a2 * rng.uniform(0.5, 0.7, 3)
    axes = [a1, a2, a3]

    def rho(p):
        u = (np.atleast_2d(p) - c) @ Q
        return [np.sqrt(np.sum((u / a) ** 2, axis=-1)) for a in axes]

    def label(p):
        r = rho(p)
        lab = np.zeros(len(r[0]), np.int64)
        for k in range(3):
            lab[r[k] <= 1.0] = k + 1
        return lab

    def clearance(p):
        return np.min([np.abs(r - 1.0) * a.min() for r, a in zip(rho(p), axes)], axis=0)

    return dict(centre=c, rotation=Q, axes=axes, label=label, clearance=clearance, rng=rng)


def shell_volume_device(dims=(2048, 2048, 1024), seed=5, n_per_class=50, margin=None, fbm_std=100.0,
                        device="cuda:0", slab=8):
    """The nested-shell recipe of ``shell_volume`` at sizes the host cannot
    draw quickly: the geometry and seeds come from numpy exactly as there
    (``shell_geometry``; seeds tested with the analytic labels), the noise
    from a seeded torch generator on ``device`` (so the volume differs from
    ``shell_volume``'s at the same seed but follows the same recipe), built
    ``slab`` z-planes at a time.  Returns (vol uint16 [z, y, x] tensor on the
    device, labels uint8 tensor on the device, seeds
    float64 [k, 4], geometry dict)."""
    import torch
    nx, ny, nz = dims
    geo = shell_geometry(dims, seed)
    rng = geo["rng"]
    if margin is None:
        margin = max(2.0, 8.0 * min(dims) / 1024.0)
    dev = torch.device(device)
    c = torch.tensor(geo["centre"], dtype=torch.float64, device=dev)
    Q = torch.tensor(geo["rotation"], dtype=torch.float64, device=dev)
    ax = [torch.tensor(a, dtype=torch.float64, device=dev) for a in geo["axes"]]
    # lattice values of the six fBm octaves (small; drawn on the host)
    octaves = []
    amp, var = 1.0, 0.0
    for o in range(6):
        wl = 512.0 / 2 ** o
        cells = [int(np.ceil(d / wl)) + 2 for d in (nz, ny, nx)]
        octaves.append((wl, amp, torch.from_numpy(rng.standard_normal(cells).astype(np.float32)).to(dev)))
        var += amp * amp
        amp *= 0.5
    fscale = float(fbm_std / np.sqrt(var))
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 1000003 + 17)
    means = torch.tensor([500.0, 1500.0, 2500.0, 3500.0], device=dev)
    vol = torch.empty((nz, ny, nx), dtype=torch.int16, device=dev)
    labels = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
    xs = torch.arange(nx, dtype=torch.float64, device=dev)
    ys = torch.arange(ny, dtype=torch.float64, device=dev)
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        zs = torch.arange(z0, z1, dtype=torch.float64, device=dev)
        P = torch.stack(torch.broadcast_tensors(xs[None, None, :], ys[None, :, None], zs[:, None, None]), -1) - c
        u = P @ Q
        lab = torch.zeros((z1 - z0, ny, nx), dtype=torch.uint8, device=dev)
        for k, a in enumerate(ax):
            lab[torch.sum((u / a) ** 2, dim=-1) <= 1.0] = k + 1
        del P, u
        labels[z0:z1] = lab
        v = means[lab.long()]
        fbm = torch.zeros((z1 - z0, ny, nx), dtype=torch.float32, device=dev)
        for wl, am, lat in octaves:
            coords = [(torch.arange(a0, a1, dtype=torch.float32, device=dev) + 0.5) / wl
                      for a0, a1 in ((z0, z1), (0, ny), (0, nx))]
            i0 = [t.floor().long() for t in coords]
            f = [t - t.floor() for t in coords]
            for dz in (0, 1):
                wz = (f[0] if dz else 1 - f[0])[:, None, None]
                for dy in (0, 1):
                    wy = (f[1] if dy else 1 - f[1])[None, :, None]
                    for dx in (0, 1):
                        wx = (f[2] if dx else 1 - f[2])[None, None, :]
                        fbm += am * wz * wy * wx * lat[(i0[0] + dz)[:, None, None], (i0[1] + dy)[None, :, None],
                                                       (i0[2] + dx)[None, None, :]]
        v = v + fbm * fscale
        v = v + torch.randn(v.shape, generator=gen, device=dev, dtype=torch.float32) * 250.0
        vu = torch.clamp(torch.round(v), 0.0, 65535.0).to(torch.int32)
        vol[z0:z1] = (vu - 65536 * (vu > 32767).to(torch.int32)).to(torch.int16)
        del v, fbm, vu, lab
    D = np.array(dims, np.float64)
    seeds = []
    for cls in range(4):
        got, tries = 0, 0
        while got < n_per_class:
            tries += 1
            if tries > 1000:
                raise RuntimeError(f"class {cls}: too few voxels {margin} away from the boundaries")
            q = np.rint(rng.uniform(0.0, 1.0, (4096, 3)) * (D - 1)).astype(np.int64)
            ok = (geo["label"](q.astype(np.float64)) == cls) & (geo["clearance"](q.astype(np.float64)) >= margin)
            for vq in q[ok][: n_per_class - got]:
                seeds.append([vq[0] + 0.5, vq[1] + 0.5, vq[2] + 0.5, cls])
                got += 1
    geo = dict(geo, margin=margin, dims=dims)
    del geo["rng"]
    return vol.view(torch.uint16), labels, np.array(seeds, np.float64), geo


def stroke_geo(geo, cls=2, length=2000, seed=6):
    """``stroke`` driven by the analytic labels of a shell geometry (for
    volumes whose label array stays on the device)."""
    rng = np.random.default_rng(seed)
    margin = geo["margin"]
    nx, ny, nz = geo["dims"]
    steps = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])

    def ok(v):
        return (0 <= v[0] < nx and 0 <= v[1] < ny and 0 <= v[2] < nz
                and geo["label"](v.astype(np.float64))[0] == cls
                and geo["clearance"](v.astype(np.float64))[0] >= margin)

    for _ in range(100000):
        start = np.array([rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)])
        if not ok(start):
            continue
        path, seen = [start], {tuple(start)}
        while len(path) < length:
            cand = [path[-1] + s for s in steps[rng.permutation(6)]]
            nxt = next((v for v in cand if tuple(v) not in seen and ok(v)), None)
            if nxt is None:
                break
            path.append(nxt)
            seen.add(tuple(nxt))
        if len(path) == length:
            p = np.array(path, np.float64) + 0.5
            return np.concatenate([p, np.full((length, 1), float(cls))], axis=1)
    raise RuntimeError("no self-avoiding walk of the requested length found")
