"""Pins of the oracle's box solve (CPU only).

Each test checks ``oracle.rw`` against something fixed by the paper's model
(Section III-B) or by mathematics, never against a retyped copy of itself:
hand-worked values, the series-resistor closed form of a 1D chain, discrete
harmonic polynomials, an independent brute force (absorbing Markov chain and
Monte-Carlo walkers), and invariants of the Dirichlet problem.
"""

import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import rw, brute


def _box_from_line(vals, axis):
    """Put a 1D array along axis 'x', 'y' or 'z' of a box ([z,y,x] layout)."""
    v = np.asarray(vals)
    shape = {"x": (1, 1, v.size), "y": (1, v.size, 1), "z": (v.size, 1, 1)}[axis]
    return v.reshape(shape)


def test_golden_chain(golden_dir):
    with open(os.path.join(golden_dir, "chain_ln2.json")) as f:
        gold = json.load(f)
    beta = math.log(2.0)
    for axis in "xyz":
        g = _box_from_line(gold["g"], axis)
        for case in gold["cases"]:
            wx, wy, wz = rw.edge_weights(g, beta, case["eps"])
            w = {"x": wx, "y": wy, "z": wz}[axis].ravel()
            assert np.allclose(w, case["weights"], rtol=0, atol=1e-15)
            # the other two axes have no edges in a line box
            assert sum(a.size for a in (wx, wy, wz)) == 2
            mask = _box_from_line([1, 0, 1], axis)
            x0 = _box_from_line([0.0, 0.0, 1.0], axis)
            for method in ("direct", "dense", "pcg"):
                x = rw.solve_box(g, mask, x0, beta, case["eps"], method=method)
                assert np.allclose(x.ravel(), case["x"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_chain_series_resistors(axis):
    """Potential drop along a chain is proportional to edge resistance 1/w."""
    rng = np.random.default_rng(11)
    n = 17
    gl = rng.random(n)
    beta, eps = 7.5, 1e-3
    g = _box_from_line(gl, axis)
    mask = np.zeros(n, dtype=np.uint8)
    mask[0] = mask[-1] = 1
    x0 = np.zeros(n)
    x0[-1] = 1.0
    x = rw.solve_box(g, _box_from_line(mask, axis), _box_from_line(x0, axis), beta, eps).ravel()
    R = 1.0 / (np.exp(-beta * np.diff(gl) ** 2) + eps)
    expect = np.concatenate([[0.0], np.cumsum(R)]) / R.sum()
    assert np.max(np.abs(x - expect)) < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_slab_reduces_to_chain(axis):
    """g varying along one axis only, 0/1 faces on that axis, free elsewhere:
    every line along the axis carries the chain profile."""
    rng = np.random.default_rng(12 + axis)
    shape = [5, 6, 7]
    n = shape[axis]
    prof = rng.random(n)
    bshape = [1, 1, 1]
    bshape[axis] = n
    g = np.broadcast_to(prof.reshape(bshape), shape).copy()
    mask = np.zeros(shape, dtype=np.uint8)
    x0 = np.zeros(shape)
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[axis] = 0
    hi[axis] = n - 1
    mask[tuple(lo)] = 1
    mask[tuple(hi)] = 1
    x0[tuple(hi)] = 1.0
    beta, eps = 20.0, 1e-6
    x = rw.solve_box(g, mask, x0, beta, eps)
    R = 1.0 / (np.exp(-beta * np.diff(prof) ** 2) + eps)
    expect = (np.concatenate([[0.0], np.cumsum(R)]) / R.sum()).reshape(bshape)
    assert np.max(np.abs(x - expect)) < 1e-12


HARMONIC = [
    lambda x, y, z: x + 2 * y - z,
    lambda x, y, z: x * y,
    lambda x, y, z: x * x - y * y,
    lambda x, y, z: x * y * z,
    lambda x, y, z: x * x + y * y - 2 * z * z,
]


@pytest.mark.parametrize("k", range(len(HARMONIC)))
def test_uniform_weights_harmonic_polynomial(k):
    """beta = 0 gives uniform weights; data from a discrete harmonic polynomial
    on all six faces is reproduced exactly inside."""
    nx, ny, nz = 7, 6, 5
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = HARMONIC[k](x.astype(float), y.astype(float), z.astype(float))
    f = (f - f.min()) / (f.max() - f.min())
    face = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
    g = np.random.default_rng(k).random((nz, ny, nx))
    xs = rw.solve_box(g, face.astype(np.uint8), np.where(face, f, 0.0), 0.0, 1e-6)
    assert np.max(np.abs(xs - f)) < 1e-13


def _boxes():
    rng = np.random.default_rng(21)
    return [synth.random_box(rng, s, dirichlet_frac=df)
            for s, df in [((6, 5, 4), 0.1), ((9, 9, 9), 0.03), ((12, 3, 7), 0.05), ((1, 1, 8), 0.2)]]


def test_direct_dense_pcg_agree():
    for g, m, x in _boxes():
        xd = rw.solve_box(g, m, x, 128.0, 1e-6, method="direct")
        xc = rw.solve_box(g, m, x, 128.0, 1e-6, method="dense")
        xp = rw.solve_box(g, m, x, 128.0, 1e-6, method="pcg", tol=1e-14)
        # both factorisations are backward stable: forward error <~ u * cond(A)
        A, _, _, _ = rw.dirichlet_system(g, m, x, 128.0, 1e-6)
        kappa = np.linalg.cond(A.toarray())
        assert np.max(np.abs(xd - xc)) < 1e-15 * kappa + 1e-13
        assert np.max(np.abs(xd - xp)) < 1e-13 * kappa + 1e-11


def test_absorbing_chain_matches_solve():
    rng = np.random.default_rng(5)
    g, m, x = synth.random_box(rng, (4, 4, 4), dirichlet_frac=0.15)
    for beta in (0.0, 10.0, 128.0):
        xa = brute.absorbing_chain(g, m, x, beta, 1e-6)
        xd = rw.solve_box(g, m, x, beta, 1e-6, method="dense")
        assert np.max(np.abs(xa - xd)) < 1e-12


def test_monte_carlo_walkers():
    rng = np.random.default_rng(6)
    g, m, x = synth.random_box(rng, (3, 3, 3), dirichlet_frac=0.0)
    m[...] = 0
    m[0, 0, 0] = m[2, 2, 2] = m[0, 2, 1] = 1
    x = np.zeros_like(x)
    x[2, 2, 2] = 1.0
    x[0, 2, 1] = 0.5
    beta, eps = 4.0, 1e-3
    xd = rw.solve_box(g, m, x, beta, eps)
    for start in (13, 5, 21):
        mean, se = brute.monte_carlo(g, m, x, beta, eps, start, 20000, np.random.default_rng(start))
        assert abs(mean - xd.ravel()[start]) < 5 * se + 1e-12


def test_invariants():
    for g, m, x in _boxes():
        beta, eps = 64.0, 1e-6
        x = x.astype(np.float64)
        xs = rw.solve_box(g, m, x, beta, eps)
        seeded = m != 0
        # rounding of a backward-stable solve: forward error <~ u * cond(A)
        A, _, _, _ = rw.dirichlet_system(g, m, x, beta, eps)
        tol = 1e-15 * np.linalg.cond(A.toarray()) + 1e-12
        # seeds fixed
        assert np.array_equal(xs[seeded], x[seeded].astype(np.float64))
        # maximum principle
        lo, hi = x[seeded].min(), x[seeded].max()
        assert xs[~seeded].min() >= lo - tol and xs[~seeded].max() <= hi + tol
        # mean-value property at every unseeded voxel
        wx, wy, wz = rw.edge_weights(g, beta, eps)
        num = np.zeros_like(xs)
        den = np.zeros_like(xs)
        num[:, :, :-1] += wx * xs[:, :, 1:]
        den[:, :, :-1] += wx
        num[:, :, 1:] += wx * xs[:, :, :-1]
        den[:, :, 1:] += wx
        num[:, :-1, :] += wy * xs[:, 1:, :]
        den[:, :-1, :] += wy
        num[:, 1:, :] += wy * xs[:, :-1, :]
        den[:, 1:, :] += wy
        num[:-1] += wz * xs[1:]
        den[:-1] += wz
        num[1:] += wz * xs[:-1]
        den[1:] += wz
        free = ~seeded & (den > 0)
        assert np.max(np.abs(xs[free] - num[free] / den[free])) < tol
        # symmetry x(1 - x_M) = 1 - x(x_M)
        xf = rw.solve_box(g, m, np.where(seeded, 1.0 - x, 0.0), beta, eps)
        assert np.max(np.abs(xf - (1.0 - xs))) < 10 * tol
        # superposition
        rng = np.random.default_rng(3)
        x2 = np.where(seeded, rng.random(x.shape), 0.0)
        xs2 = rw.solve_box(g, m, x2, beta, eps)
        xs12 = rw.solve_box(g, m, 0.3 * x + 0.7 * x2, beta, eps)
        assert np.max(np.abs(xs12 - (0.3 * xs + 0.7 * xs2))) < 10 * tol
        # energy minimality against random perturbations on the unseeded set
        e0 = rw.dirichlet_energy(g, xs, beta, eps)
        for _ in range(5):
            d = np.where(seeded, 0.0, rng.normal(0.0, 1e-3, x.shape))
            assert rw.dirichlet_energy(g, xs + d, beta, eps) >= e0


def test_multiclass_sums_to_one():
    rng = np.random.default_rng(8)
    g, m, _ = synth.random_box(rng, (7, 6, 5), dirichlet_frac=0.12)
    labels = rng.integers(0, 4, g.shape)
    pa, la = rw.solve_multiclass(g, m, labels, 4, 32.0, 1e-6, all_classes=True)
    pc, lc = rw.solve_multiclass(g, m, labels, 4, 32.0, 1e-6, all_classes=False)
    assert np.max(np.abs(pa.sum(axis=0) - 1.0)) < 1e-12
    assert np.max(np.abs(pa - pc)) < 1e-11
    assert np.array_equal(la, lc)
    # argmax is the class of the seed on seeded voxels
    seeded = m != 0
    assert np.array_equal(la[seeded], labels[seeded].astype(np.uint8))


def test_no_dirichlet_leaves_x():
    g = np.random.default_rng(1).random((3, 3, 3))
    x = np.full((3, 3, 3), 0.25)
    out = rw.solve_box(g, np.zeros((3, 3, 3), np.uint8), x, 1.0, 1e-6)
    assert np.array_equal(out, x)


def test_pcg_reaches_tolerance_and_counts():
    g, m, x = _boxes()[1]
    A, b, U, M = rw.dirichlet_system(g, m, x, 128.0, 1e-6)
    for tol in (1e-4, 1e-8, 1e-12):
        xu, it, rel = rw.pcg(A, b, tol=tol)
        assert rel <= 1.01 * tol and it > 0
