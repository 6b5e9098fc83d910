"""GPU gradients (adjoint solve + edge chain rule) against the oracle's FP64
adjoint and against central finite differences of the GPU forward solve.

Workload: boxes of the two-blob recipe (32^3, beta 64 learnable, g learnable),
loss = mean over unseeded voxels of BCE(clamp(x, 1e-6, 1-1e-6), y) with y the
blob-1 half-maximum mask.  Bar: gradients within 1e-3 relative: dl/dbeta as a
scalar; dl/dg per box in norm and per voxel, where each voxel must satisfy
|gpu - oracle| <= 1e-3 |oracle| + FLOOR * max_box |oracle| (FLOOR below: the
gradient is formed in FP32 from an FP32 adjoint solved to relative residual
1e-7, so voxels whose gradient cancels to near zero carry an absolute error of
that order of the box's largest gradient); and each of the 64 finite-difference
voxels on its own within 1e-3 relative plus the finite difference's own
truncation error, estimated from a second difference at h/2.
"""

import numpy as np
import pytest

import synth
from oracle import adjoint as oadj
from oracle import rw as orw

pytestmark = pytest.mark.gpu

BETA, EPS = 64.0, 1e-6
FLOOR = 1e-4


def _elementwise(dg, og, tag):
    """Per-voxel check; returns the worst ratio of error to allowance."""
    allow = 1e-3 * np.abs(og) + FLOOR * np.max(np.abs(og))
    ratio = np.abs(dg - og) / allow
    worst = float(ratio.max())
    assert worst <= 1.0, (tag, worst, int(np.argmax(ratio)))
    return worst


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2103_09564_amd as rwg
    assert torch.cuda.is_available()
    return torch, rwg


@pytest.fixture(scope="module")
def blobs():
    return synth.blob_boxes(n=6, seed=4)


def _bce(torch, x, y, u, count):
    xc = torch.clamp(x, 1e-6, 1 - 1e-6)
    t = -(y * torch.log(xc) + (1 - y) * torch.log(1 - xc))
    return (t * u).sum() / count


def test_adjoint_matches_oracle(env, blobs):
    torch, rwg = env
    d = blobs
    dev = torch.device("cuda:0")
    g = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    x = torch.from_numpy(d["x"]).to(dev)
    y = torch.from_numpy(d["gt"].astype(np.float64)).to(dev)
    u = (m == 0).double()
    count = float((d["mask"] == 0).sum())
    rwg.solve_bricks(g, m, x, d["shapes"], d["offsets"], beta=BETA, eps=EPS, tol=1e-7, precision=2,
                     refine_max=4, refine_tol=1e-10)
    xd = x.double().requires_grad_(True)
    loss = _bce(torch, xd, y, u, count)
    loss.backward()
    dl_dx = xd.grad.float().contiguous()
    dl_dg, dl_db, st = rwg.solve_bricks_adjoint(g, m, x, dl_dx, d["shapes"], d["offsets"], beta=BETA, eps=EPS,
                                                tol=1e-7)
    torch.cuda.synchronize()
    dg = dl_dg.cpu().numpy()
    db = float(dl_db.cpu()[0])
    # oracle, from its own forward solution and loss
    tot_db = 0.0
    for i, (gb, mb, xb) in enumerate(d["boxes"]):
        xo = orw.solve_box(gb, mb, xb, BETA, EPS, method="pcg", tol=1e-14)
        o = int(d["offsets"][i])
        yb = d["gt"][o:o + gb.size].reshape(gb.shape)
        _, grad = oadj.bce_loss(xo, yb, mb, count=count)
        og, odb, _ = oadj.adjoint_gradients(gb, mb, xo, grad, BETA, EPS)
        tot_db += odb
        rel = np.linalg.norm(dg[o:o + gb.size] - og.ravel()) / np.linalg.norm(og)
        assert rel <= 1e-3, (i, rel)
        worst = _elementwise(dg[o:o + gb.size], og.ravel(), i)
        print(f"blob box {i}: norm rel {rel:.2e}, worst per-voxel error/allowance {worst:.3f}", flush=True)
    assert abs(db - tot_db) <= 1e-3 * abs(tot_db), (db, tot_db)
    assert np.all(rwg.stats_to_numpy(st)["status"] == 0)


def test_rwsolve_autograd_and_finite_differences(env, blobs):
    """RWSolve backward (adjoint) against central differences (h = 1e-3) of
    the loss evaluated on FP64 GPU forward solves (plain FP64 PCG to 1e-13)."""
    torch, rwg = env
    d = blobs
    dev = torch.device("cuda:0")
    g0 = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    xdir = torch.from_numpy(d["x"]).to(dev)
    y = torch.from_numpy(d["gt"].astype(np.float64)).to(dev)
    u = (m == 0).double()
    count = float((d["mask"] == 0).sum())

    def loss64(g, beta):
        x = xdir.clone()
        x64 = torch.zeros(x.numel(), dtype=torch.float64, device=dev)
        rwg.solve_bricks(g, m, x, d["shapes"], d["offsets"], x64=x64, beta=float(beta), eps=EPS, tol=1e-13,
                         precision=0, max_iter=20000)
        return float(_bce(torch, x64, y, u, count))

    g = g0.clone().requires_grad_(True)
    beta = torch.tensor(BETA, dtype=torch.float64, requires_grad=True)
    x = rwg.RWSolve.apply(g, beta, m, xdir, d["shapes"], d["offsets"], EPS, 1e-12, 0)
    L = _bce(torch, x.double(), y, u, count)
    L.backward()
    ag = g.grad.detach().cpu().numpy()
    ab = float(beta.grad)
    h = 1e-3
    fd_b = (loss64(g0, BETA + h) - loss64(g0, BETA - h)) / (2 * h)
    assert abs(ab - fd_b) <= 1e-3 * abs(fd_b), (ab, fd_b)
    rng = np.random.default_rng(0)
    unk = np.flatnonzero(d["mask"] == 0)
    picks = rng.choice(unk, 64, replace=False)
    num = den = 0.0
    worst = 0.0
    for v in picks:
        def fd(step):
            gp = g0.clone()
            gm = g0.clone()
            gp[v] += step
            gm[v] -= step
            return (loss64(gp, BETA) - loss64(gm, BETA)) / (2 * step)
        f1, f2 = fd(h), fd(h / 2)
        trunc = 4.0 / 3.0 * abs(f1 - f2)     # error estimate of the h-difference (O(h^2))
        err = abs(ag[v] - f1)
        allow = 1e-3 * abs(f1) + trunc + 1e-12
        worst = max(worst, err / allow)
        assert err <= allow, (int(v), ag[v], f1, f2)
        num += (ag[v] - f1) ** 2
        den += f1 ** 2
    print(f"64 FD voxels: worst error/allowance {worst:.3f}, pooled RMS rel {np.sqrt(num / den):.2e}", flush=True)
    assert np.sqrt(num / den) <= 1e-3, np.sqrt(num / den)


def test_adjoint_on_resident_and_ragged_boxes(env):
    """Adjoint gradients on boxes small enough for the LDS-resident PCG and on
    ragged shapes, with a fixed random dl/dx, against the oracle."""
    torch, rwg = env
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(41)
    shapes = [(16, 16, 16), (32, 9, 32), (5, 32, 32), (13, 7, 19), (33, 31, 30)]
    boxes = [synth.random_box(rng, s, dirichlet_frac=0.04) for s in shapes]
    d = synth.from_boxes(boxes)
    g = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    x = torch.from_numpy(d["x"]).to(dev)
    beta = 96.0
    rwg.solve_bricks(g, m, x, d["shapes"], d["offsets"], beta=beta, eps=EPS, tol=1e-7, precision=2,
                     refine_max=4, refine_tol=1e-10)
    dl_dx_np = rng.standard_normal(d["x"].size).astype(np.float32)
    dl_dx = torch.from_numpy(dl_dx_np).to(dev)
    dl_dg, dl_db, st = rwg.solve_bricks_adjoint(g, m, x, dl_dx, d["shapes"], d["offsets"], beta=beta, eps=EPS,
                                                tol=1e-7)
    torch.cuda.synchronize()
    dg = dl_dg.cpu().numpy()
    tot = 0.0
    for i, (gb, mb, xb) in enumerate(boxes):
        o = int(d["offsets"][i])
        xo = orw.solve_box(gb, mb, xb, beta, EPS, method="pcg", tol=1e-14)
        og, odb, _ = oadj.adjoint_gradients(gb, mb, xo, dl_dx_np[o:o + gb.size].reshape(gb.shape), beta, EPS)
        tot += odb
        rel = np.linalg.norm(dg[o:o + gb.size] - og.ravel()) / np.linalg.norm(og)
        assert rel <= 1e-3, (shapes[i], rel)
        worst = _elementwise(dg[o:o + gb.size], og.ravel(), shapes[i])
        print(f"box {shapes[i]}: norm rel {rel:.2e}, worst per-voxel error/allowance {worst:.3f}", flush=True)
    assert abs(float(dl_db.cpu()[0]) - tot) <= 1e-3 * abs(tot)
    assert np.all(rwg.stats_to_numpy(st)["status"] == 0)
