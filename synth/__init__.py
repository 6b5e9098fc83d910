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
