"""Pins of the Poisson-noise weight (Section IV-C) in the oracle: the weight
exp(-(sqrt n_p - sqrt n_q)^2 / 2) of the paper, built edge by edge into a
dense Laplacian and solved directly, against the oracle's box solve and
hierarchy on the square-root counts pyramid with beta = 1/2."""

import numpy as np

from oracle import hierarchy as H
from oracle import rw

EPS = 1e-6


def _poisson_dense_solve(n, seeded, xm, eps=EPS):
    """Dirichlet problem with the paper's Poisson weight, by brute force:
    every 6-neighbour edge written out, dense L, numpy solve."""
    nz, ny, nx = n.shape
    N = n.size
    idx = np.arange(N).reshape(n.shape)
    L = np.zeros((N, N))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for dz, dy, dx in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    zz, yy, xx = z + dz, y + dy, x + dx
                    if zz < nz and yy < ny and xx < nx:
                        a, b = idx[z, y, x], idx[zz, yy, xx]
                        w = np.exp(-0.5 * (np.sqrt(float(n[z, y, x])) - np.sqrt(float(n[zz, yy, xx]))) ** 2) + eps
                        L[a, a] += w
                        L[b, b] += w
                        L[a, b] -= w
                        L[b, a] -= w
    s = seeded.ravel() != 0
    u = ~s
    out = xm.astype(np.float64).ravel().copy()
    out[u] = np.linalg.solve(L[np.ix_(u, u)], -L[np.ix_(u, s)] @ out[s])
    return out.reshape(n.shape)


def test_poisson_weight_is_gaussian_of_sqrt_counts_by_brute_force():
    rng = np.random.default_rng(4)
    lam = np.where(rng.random((4, 5, 6)) < 0.5, 15.0, 60.0)
    n = rng.poisson(lam).astype(np.uint16)
    seeded = np.zeros(n.shape, np.uint8)
    seeded[0, 0, :] = 1
    seeded[-1, -1, :] = 1
    xm = np.zeros(n.shape)
    xm[-1, -1, :] = 1.0
    ref = _poisson_dense_solve(n, seeded, xm)
    g = H.pyramid_counts(n, 1)[0]
    got = rw.solve_box(g, seeded, xm, 0.5, EPS)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_pyramid_counts_closed_forms():
    c = np.full((5, 6, 7), 49, np.uint16)
    for lev in H.pyramid_counts(c, 3):
        assert np.allclose(lev, 7.0, rtol=0, atol=1e-14)
    # one 2x2x2 block of counts 1..8: the parent is sqrt of the mean count (4.5),
    # not the mean of the square roots
    b = np.arange(1, 9, dtype=np.uint16).reshape(2, 2, 2)
    p = H.pyramid_counts(b, 2)
    assert np.array_equal(p[0], np.sqrt(b.astype(np.float64)))
    assert abs(p[1][0, 0, 0] - np.sqrt(4.5)) < 1e-15
    assert abs(p[1][0, 0, 0] - np.sqrt(b.astype(np.float64)).mean()) > 1e-2
    # odd edges: the partial block averages the counts it has; float counts clip at 0
    f = np.array([[[4.0, -3.0, 16.0]]], np.float32)
    q = H.pyramid_counts(f, 2)
    assert np.allclose(q[0], [[[2.0, 0.0, 4.0]]]) and np.allclose(q[1], [[[np.sqrt(2.0), 4.0]]])


def test_single_level_poisson_hierarchy_is_plain_brute_force_solve():
    rng = np.random.default_rng(5)
    nz = ny = nx = 6
    z, y, x = np.meshgrid(*(np.arange(6),) * 3, indexing="ij")
    inside = (x - 2.5) ** 2 + (y - 2.5) ** 2 + (z - 2.5) ** 2 <= 4.0
    n = rng.poisson(np.where(inside, 80.0, 20.0)).astype(np.uint16)
    seeds = np.array([[2.5, 2.5, 2.5, 1], [0.5, 0.5, 0.5, 0], [5.5, 5.5, 5.5, 0], [0.5, 5.5, 3.0, 0]])
    p = H.Params(levels=1, brick=4, beta=0.5, eps=EPS)
    res = H.segment(n, seeds, p, g=H.pyramid_counts(n, 1))
    lab = H.rasterize(seeds, 0, (nz, ny, nx))
    ref = _poisson_dense_solve(n, (lab >= 0).astype(np.uint8), np.where(lab == 1, 1.0, 0.0))
    assert np.max(np.abs(res.maps[0][0] - ref)) < 1e-12
