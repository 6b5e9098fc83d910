"""Oracle gradients of a loss on the random-walker solution (TEST INFRASTRUCTURE).

The paper (arXiv 2103.09564) has no gradient; this is derived from its
Dirichlet problem (Section III-B).  With L(w) x = 0 on the unseeded set U and
x fixed on M, differentiating along one edge weight w_e, e = (i, j), gives

    L_UU dx_U/dw_e = -[(e_i - e_j)(x_i - x_j)]_U .

For a loss l(x_U) let lambda solve the adjoint system L_UU lambda = dl/dx_U
(L_UU is symmetric) and extend lambda by 0 on M.  Then

    dl/dw_e = -(lambda_i - lambda_j)(x_i - x_j).

For the weight w = exp(-beta*(g_i - g_j)^2) + eps:
    dw/dbeta = -(g_i - g_j)^2 (w - eps)
    dw/dg_i  = -2 beta (g_i - g_j)(w - eps) = -dw/dg_j.
"""

import numpy as np
import scipy.sparse.linalg as spla

from .rw import edge_weights, edge_list, dirichlet_system


def bce_loss(x, y, mask, clamp=1e-6, count=None):
    """Mean binary cross-entropy over unseeded voxels and its gradient dl/dx.

    x is clamped to [clamp, 1-clamp]; the gradient is zero where the clamp is
    active.  ``count`` overrides the number of voxels the mean divides by
    (for a loss summed over many boxes).  Returns (loss, dl/dx).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    u = np.asarray(mask) == 0
    n = int(u.sum()) if count is None else count
    xc = np.clip(x, clamp, 1.0 - clamp)
    terms = -(y * np.log(xc) + (1.0 - y) * np.log(1.0 - xc))
    loss = float(terms[u].sum() / n)
    grad = (-y / xc + (1.0 - y) / (1.0 - xc)) / n
    grad = np.where(u & (x > clamp) & (x < 1.0 - clamp), grad, 0.0)
    return loss, grad


def adjoint_gradients(g, mask, x, dl_dx, beta, eps):
    """Gradient of l with respect to g (per voxel) and beta, float64.

    x: the converged full-box solution; dl_dx: dl/dx (values on seeded
    voxels are ignored).  Returns (dl_dg with the box shape, dl_dbeta,
    lambda with the box shape).
    """
    g = np.asarray(g, dtype=np.float64)
    A, _, U, M = dirichlet_system(g, mask, x, beta, eps)
    lam = np.zeros(g.size)
    rhs = np.asarray(dl_dx, dtype=np.float64).ravel()[U]
    if U.size and M.size:
        lam[U] = spla.spsolve(A.tocsc(), rhs)
    i, j, w = edge_list(g.shape, edge_weights(g, beta, eps))
    xf = np.asarray(x, dtype=np.float64).ravel()
    gf = g.ravel()
    dl_dw = -(lam[i] - lam[j]) * (xf[i] - xf[j])
    dg = gf[i] - gf[j]
    core = w - eps
    dl_dbeta = float(np.sum(dl_dw * (-(dg ** 2) * core)))
    dw_dgi = -2.0 * beta * dg * core
    grad = np.zeros(g.size)
    np.add.at(grad, i, dl_dw * dw_dgi)
    np.add.at(grad, j, -dl_dw * dw_dgi)
    return grad.reshape(g.shape), dl_dbeta, lam.reshape(g.shape)
