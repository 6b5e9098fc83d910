"""Brute-force pins for the box solve (TEST INFRASTRUCTURE).

Paper: arXiv 2103.09564, Section III-B.  The random-walker solution x_u at an
unseeded voxel u is the probability that a random walker started at u, moving
to a 6-neighbour with probability proportional to the edge weight, first
reaches a seed, weighted by that seed's value (for 0/1 seeds: reaches a
foreground seed before a background seed).

These routines compute that probability without the Laplacian machinery of
``oracle.rw``: the transition matrix is built voxel by voxel with explicit
neighbour loops, so they pin the assembly and the solve of ``oracle.rw``.
Only for tiny boxes (a 4^3 box is 64 voxels).
"""

import numpy as np

from .rw import edge_weights

_NEIGHBOURS = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def _weight(g, beta, eps, a, b):
    """Weight of the edge between voxels a=(z,y,x) and b, read from the
    forward-edge arrays of ``edge_weights``."""
    wx, wy, wz = edge_weights(g, beta, eps)
    (za, ya, xa), (zb, yb, xb) = a, b
    if za != zb:
        return wz[min(za, zb), ya, xa]
    if ya != yb:
        return wy[za, min(ya, yb), xa]
    return wx[za, ya, min(xa, xb)]


def transition_matrix(g, beta, eps):
    """Dense random-walk transition matrix P = D^-1 W, by explicit loops."""
    g = np.asarray(g, dtype=np.float64)
    nz, ny, nx = g.shape
    n = g.size
    W = np.zeros((n, n))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = x + nx * (y + ny * z)
                for dx, dy, dz in _NEIGHBOURS:
                    X, Y, Z = x + dx, y + dy, z + dz
                    if 0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz:
                        j = X + nx * (Y + ny * Z)
                        W[i, j] = _weight(g, beta, eps, (z, y, x), (Z, Y, X))
    return W / W.sum(axis=1, keepdims=True)


def absorbing_chain(g, mask, x, beta, eps):
    """x_U = (I - P_UU)^-1 P_UM x_M with an explicit matrix inverse."""
    g = np.asarray(g)
    P = transition_matrix(g, beta, eps)
    m = np.asarray(mask).ravel() != 0
    U = np.flatnonzero(~m)
    M = np.flatnonzero(m)
    xm = np.asarray(x, dtype=np.float64).ravel()[M]
    N = np.linalg.inv(np.eye(U.size) - P[np.ix_(U, U)])
    out = np.array(x, dtype=np.float64).ravel()
    out[U] = N @ (P[np.ix_(U, M)] @ xm)
    return out.reshape(g.shape)


def monte_carlo(g, mask, x, beta, eps, start, n_walkers, rng, max_steps=1000000):
    """Monte-Carlo estimate of x at voxel ``start`` (flat index).

    Returns (mean, standard error).  Each walker moves until it first stands
    on a seeded voxel and reports that voxel's value.
    """
    g = np.asarray(g)
    P = transition_matrix(g, beta, eps)
    cdf = np.cumsum(P, axis=1)
    cdf[:, -1] = 1.0
    m = np.asarray(mask).ravel() != 0
    val = np.asarray(x, dtype=np.float64).ravel()
    pos = np.full(n_walkers, start, dtype=np.int64)
    done = m[pos].copy()
    result = np.where(done, val[pos], 0.0)
    steps = 0
    while not np.all(done) and steps < max_steps:
        act = np.flatnonzero(~done)
        u = rng.random(act.size)
        nxt = np.array([np.searchsorted(cdf[p], uu, side="right") for p, uu in zip(pos[act], u)])
        pos[act] = nxt
        hit = m[nxt]
        result[act[hit]] = val[nxt[hit]]
        done[act[hit]] = True
        steps += 1
    if not np.all(done):
        raise RuntimeError("walkers did not reach a seed")
    return float(result.mean()), float(result.std(ddof=1) / np.sqrt(n_walkers))
