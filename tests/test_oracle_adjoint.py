"""Pins of the oracle's adjoint gradients (CPU only): a closed form for the
1D chain and central finite differences of the oracle's own solve."""

import numpy as np

import synth
from oracle import rw, adjoint


def test_chain_closed_form_dbeta():
    """x_k = S_k/S with S_k = sum_{j<k} R_j, R_j = 1/w_j; differentiate."""
    rng = np.random.default_rng(2)
    n = 12
    gl = rng.random(n)
    beta, eps = 9.0, 1e-3
    g = gl.reshape(1, 1, n)
    mask = np.zeros((1, 1, n), np.uint8)
    mask[..., 0] = mask[..., -1] = 1
    x0 = np.zeros((1, 1, n))
    x0[..., -1] = 1.0
    x = rw.solve_box(g, mask, x0, beta, eps)
    c = rng.normal(size=n)                 # linear loss l = sum c_k x_k
    dl_dx = c.reshape(1, 1, n)
    _, dbeta, _ = adjoint.adjoint_gradients(g, mask, x, dl_dx, beta, eps)
    d2 = np.diff(gl) ** 2
    w = np.exp(-beta * d2) + eps
    R = 1.0 / w
    dR = d2 * (w - eps) / w ** 2           # dR/dbeta
    S = R.sum()
    dS = dR.sum()
    Sk = np.concatenate([[0.0], np.cumsum(R)])
    dSk = np.concatenate([[0.0], np.cumsum(dR)])
    dx = (dSk * S - Sk * dS) / S ** 2
    expect = float(np.sum(c[1:-1] * dx[1:-1]))
    assert abs(dbeta - expect) < 1e-12 * max(1.0, abs(expect))


def test_adjoint_matches_central_differences():
    rng = np.random.default_rng(7)
    g, m, x0 = synth.random_box(rng, (6, 5, 4), dirichlet_frac=0.15)
    g = g.astype(np.float64)
    beta, eps = 30.0, 1e-4
    y = (rng.random(g.shape) < 0.5).astype(np.float64)

    def loss(gg, bb):
        xs = rw.solve_box(gg, m, x0, bb, eps, method="dense")
        return adjoint.bce_loss(xs, y, m)[0]

    xs = rw.solve_box(g, m, x0, beta, eps, method="dense")
    _, dl_dx = adjoint.bce_loss(xs, y, m)
    dg, dbeta, _ = adjoint.adjoint_gradients(g, m, xs, dl_dx, beta, eps)
    h = 1e-5
    fd_beta = (loss(g, beta + h) - loss(g, beta - h)) / (2 * h)
    assert abs(dbeta - fd_beta) <= 1e-6 * max(abs(fd_beta), 1e-8)
    for v in rng.choice(g.size, 12, replace=False):
        gp = g.copy()
        gm = g.copy()
        gp.flat[v] += h
        gm.flat[v] -= h
        fd = (loss(gp, beta) - loss(gm, beta)) / (2 * h)
        assert abs(dg.flat[v] - fd) <= 1e-6 * max(abs(fd), 1e-6) + 1e-10


def test_bce_gradient_is_derivative():
    rng = np.random.default_rng(3)
    x = rng.uniform(0.01, 0.99, (4, 4, 4))
    y = (rng.random((4, 4, 4)) < 0.5).astype(float)
    m = (rng.random((4, 4, 4)) < 0.2).astype(np.uint8)
    _, gr = adjoint.bce_loss(x, y, m)
    h = 1e-6
    for v in range(0, 64, 7):
        xp = x.copy()
        xm = x.copy()
        xp.flat[v] += h
        xm.flat[v] -= h
        fd = (adjoint.bce_loss(xp, y, m)[0] - adjoint.bce_loss(xm, y, m)[0]) / (2 * h)
        assert abs(gr.flat[v] - fd) < 1e-7
