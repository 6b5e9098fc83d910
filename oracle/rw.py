"""Oracle: the random-walker Dirichlet problem on one box (TEST INFRASTRUCTURE).

Paper: Drees, Eilers & Jiang, arXiv 2103.09564, Section III-B.

A box is a 3D grid of nx*ny*nz voxels.  Arrays are indexed ``a[z, y, x]``
(C order), so the flat voxel index is ``x + nx*(y + ny*z)``.

* Graph: one vertex per voxel, edges between 6-neighbours *inside the box*
  (no edge leaves the box; volume faces are natural boundaries).
* Edge weight: w_pq = exp(-beta*(g_p - g_q)^2) + eps  (Section III-B gives the
  Gaussian term; the additive eps floor is the reading used throughout this
  project, it keeps the graph connected for any beta).
* Laplacian L = D - W with D_pp = sum_q w_pq.
* Dirichlet problem: minimise D(x) = 1/2 x^T L x with x fixed on the seeded
  set M.  Partitioning x = (x_U, x_M), the minimiser solves
        L_UU x_U = -L_UM x_M                                   (*)
  L_UU is an irreducibly diagonally dominant M-matrix when M is non-empty and
  eps > 0, so (*) has a unique solution; that solution is what this oracle
  returns (``solve_box``), computed by a sparse direct factorisation, a dense
  Cholesky factorisation, or textbook Jacobi-preconditioned CG (the solver the
  paper uses, Section V), each in float64.
* Multi-class (Section III-B, last paragraph): one solve per class with that
  class's seeds as foreground and all others as background; the label of a
  voxel is the class of largest probability.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.linalg as la


def edge_weights(g, beta, eps):
    """Forward edge weights of the 6-neighbour grid (Section III-B).

    Returns (wx, wy, wz): wx[z,y,x] joins (x,y,z)-(x+1,y,z), shape
    (nz,ny,nx-1); wy joins (x,y,z)-(x,y+1,z), shape (nz,ny-1,nx); wz joins
    (x,y,z)-(x,y,z+1), shape (nz-1,ny,nx).  float64.
    """
    g = np.asarray(g, dtype=np.float64)
    wx = np.exp(-beta * (g[:, :, 1:] - g[:, :, :-1]) ** 2) + eps
    wy = np.exp(-beta * (g[:, 1:, :] - g[:, :-1, :]) ** 2) + eps
    wz = np.exp(-beta * (g[1:, :, :] - g[:-1, :, :]) ** 2) + eps
    return wx, wy, wz


def edge_list(shape, weights):
    """All edges as (i, j, w) arrays with flat voxel indices i < j."""
    nz, ny, nx = shape
    idx = np.arange(nz * ny * nx).reshape(nz, ny, nx)
    wx, wy, wz = weights
    i = np.concatenate([idx[:, :, :-1].ravel(), idx[:, :-1, :].ravel(), idx[:-1, :, :].ravel()])
    j = np.concatenate([idx[:, :, 1:].ravel(), idx[:, 1:, :].ravel(), idx[1:, :, :].ravel()])
    w = np.concatenate([wx.ravel(), wy.ravel(), wz.ravel()])
    return i, j, w


def laplacian(g, beta, eps):
    """Sparse graph Laplacian L = D - W of the box (CSR, float64)."""
    g = np.asarray(g)
    n = g.size
    i, j, w = edge_list(g.shape, edge_weights(g, beta, eps))
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    vals = np.concatenate([-w, -w])
    deg = np.bincount(i, weights=w, minlength=n) + np.bincount(j, weights=w, minlength=n)
    L = sp.coo_matrix((np.concatenate([vals, deg]),
                       (np.concatenate([rows, np.arange(n)]), np.concatenate([cols, np.arange(n)]))),
                      shape=(n, n)).tocsr()
    return L


def dirichlet_system(g, mask, xm, beta, eps):
    """The system (*) of the module docstring.

    mask: nonzero where the voxel is seeded (set M); xm: array of the box
    shape whose values on M are the Dirichlet data.
    Returns (A = L_UU, b = -L_UM x_M, U, M) with U, M flat index arrays.
    """
    L = laplacian(g, beta, eps)
    m = np.asarray(mask).ravel() != 0
    U = np.flatnonzero(~m)
    M = np.flatnonzero(m)
    xM = np.asarray(xm, dtype=np.float64).ravel()[M]
    A = L[U][:, U].tocsr()
    b = -(L[U][:, M] @ xM)
    return A, b, U, M


def pcg(A, b, x0=None, tol=1e-13, max_iter=100000):
    """Textbook Jacobi-preconditioned conjugate gradients (Section V), float64.

    Stops when ||r||_2 <= tol * ||b||_2 (r the recursive residual) or after
    max_iter iterations.  Returns (x, iterations, final ||b-Ax||/||b||).
    """
    n = b.shape[0]
    d = A.diagonal()
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    z = r / d
    p = z.copy()
    rz = r @ z
    it = 0
    while it < max_iter and np.linalg.norm(r) > tol * bnorm:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = r / d
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, np.linalg.norm(b - A @ x) / bnorm


def solve_box(g, mask, x, beta, eps, method="direct", tol=1e-13, max_iter=100000):
    """Solution of the Dirichlet problem (*) on one box, float64.

    ``x`` carries the Dirichlet values on seeded voxels (and, for
    method='pcg', the initial guess elsewhere).  Returns the full box array:
    seeded voxels keep their value, unseeded ones get the solution.
    With no seeded voxel the problem has no unique solution and ``x`` is
    returned unchanged.
    """
    g = np.asarray(g)
    out = np.array(x, dtype=np.float64).reshape(g.shape)
    if not np.any(np.asarray(mask) != 0):
        return out
    A, b, U, M = dirichlet_system(g, mask, out, beta, eps)
    if U.size == 0:
        return out
    if method == "direct":
        xu = spla.spsolve(A.tocsc(), b)
    elif method == "dense":
        xu = la.cho_solve(la.cho_factor(A.toarray()), b)
    elif method == "pcg":
        xu, _, _ = pcg(A, b, x0=out.ravel()[U], tol=tol, max_iter=max_iter)
    else:
        raise ValueError(method)
    flat = out.ravel()
    flat[U] = xu
    return flat.reshape(g.shape)


def dirichlet_energy(g, x, beta, eps):
    """D(x) = 1/2 sum over edges w_pq (x_p - x_q)^2 (Section III-B)."""
    i, j, w = edge_list(np.asarray(g).shape, edge_weights(g, beta, eps))
    xf = np.asarray(x, dtype=np.float64).ravel()
    return 0.5 * float(np.sum(w * (xf[i] - xf[j]) ** 2))


def solve_multiclass(g, mask, labels, n_classes, beta, eps, method="direct", all_classes=False):
    """Multi-class random walker (Section III-B, last paragraph).

    mask: seeded voxels; labels: class index (0..n_classes-1) on seeded voxels.
    For each class k the seeds of class k are foreground (1) and all other
    seeds background (0).  Returns probs of shape (n_classes, *box) and the
    argmax labels (lowest class index wins ties).

    By default only classes 1..K-1 are solved and class 0 is the complement
    1 - sum_k x_k; this equals the separate solve because the Dirichlet data
    of all K problems sum to one and (*) is linear.  ``all_classes=True``
    solves all K problems separately.
    """
    g = np.asarray(g)
    labels = np.asarray(labels)
    probs = np.zeros((n_classes,) + g.shape)
    first = 0 if all_classes else 1
    for k in range(first, n_classes):
        xk = np.where(np.asarray(mask) != 0, (labels == k).astype(np.float64), 0.0)
        probs[k] = solve_box(g, mask, xk, beta, eps, method=method)
    if not all_classes:
        probs[0] = 1.0 - probs[1:].sum(axis=0)
    return probs, argmax_labels(probs)


def argmax_labels(probs):
    """Class of highest probability per voxel; ties go to the lowest index."""
    return np.argmax(probs, axis=0).astype(np.uint8)
