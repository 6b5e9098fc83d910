"""Split boxes (RW_PATH_RESIDENT_SPLIT): boxes above 32768 voxels, such as the
40^3 boxes of the paper's brick configuration (s = 32, e = 1.25, Section
IV-B), solved by two workgroups per box that exchange partial sums and one
plane of z per CG iteration.  Against the FP64 oracle and against the same
boxes on the streaming kernels (rw_set_split_boxes(ctx, 0)), through the C
ABI.

Bars: max |x - oracle| <= 1e-4 at relative residual 1e-6 (the FP32 path's
bar), <= 1e-9 after FP64 refinement (which runs correction solves on the
split kernel); the split and streaming results, two stops at relative
residual 1e-6, within 4e-5 of each other (the bar between the other resident
kernels and the streaming ones); iteration counts within 5% (the same
Jacobi-PCG, rounded differently).
"""

import numpy as np
import pytest

import synth
from oracle import rw as orw

pytestmark = pytest.mark.gpu

BETA, EPS = 128.0, 1e-6
# (nx, ny, nz): the 40^3 box, clipped border boxes, an odd nz (halves of 17
# and 16 planes), a wide plane, a small upper half, and the narrowest plane
# the split takes (512 voxels)
SHAPES = [(40, 40, 40), (36, 40, 40), (40, 36, 33), (48, 40, 30), (40, 40, 21), (16, 32, 66)]


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2103_09564_amd as rwg
    assert torch.cuda.is_available()
    return torch, rwg, torch.device("cuda:0")


def _ref(box):
    g, m, x = box
    return orw.solve_box(g, m, x, BETA, EPS, method="pcg", tol=1e-14).ravel()


def _run(env, d, split=True, x64=False, **params):
    torch, rwg, dev = env
    ctx = rwg.Context(0)
    ctx.set_split_boxes(split)
    g = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    x = torch.from_numpy(d["x"]).to(dev)
    xd = torch.zeros(x.numel(), dtype=torch.float64, device=dev) if x64 else None
    st = rwg.solve_bricks(g, m, x, d["shapes"], d["offsets"], x64=xd, ctx=ctx, **params)
    torch.cuda.synchronize()
    plan = ctx.solve_plan(rwg.solve_params(**params), rwg.bricks_array(d["shapes"], d["offsets"]), d["g"].size)
    ctx.close()
    return x.cpu().numpy(), (xd.cpu().numpy() if x64 else None), rwg.stats_to_numpy(st), plan


@pytest.fixture(scope="module")
def boxes():
    rng = np.random.default_rng(41)
    bx = [synth.random_box(rng, s, dirichlet_frac=0.02) for s in SHAPES]
    return bx, synth.from_boxes(bx), [_ref(b) for b in bx]


def test_split_matches_oracle_and_streaming(env, boxes):
    print("split vs oracle and streaming", flush=True)
    _, rwg, _ = env
    bx, d, refs = boxes
    xs, _, ss, ps = _run(env, d, split=True, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    xw, _, sw, pw = _run(env, d, split=False, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    assert np.all(ps == rwg.PATH_RESIDENT_SPLIT), ps
    assert np.all((pw == rwg.PATH_STREAM) | (pw == rwg.PATH_STREAM_GLOBAL)), pw
    for i, ref in enumerate(refs):
        o, n = int(d["offsets"][i]), ref.size
        es = float(np.max(np.abs(xs[o:o + n] - ref)))
        ew = float(np.max(np.abs(xw[o:o + n] - ref)))
        print(SHAPES[i], "iters split", ss["iters"][i], "stream", sw["iters"][i], "err", es, ew, flush=True)
        assert es <= 1e-4, (SHAPES[i], ss[i])
        assert np.max(np.abs(xs[o:o + n] - xw[o:o + n])) <= 4e-5, (SHAPES[i], ss[i], sw[i])
        assert abs(int(ss["iters"][i]) - int(sw["iters"][i])) <= max(3, int(sw["iters"][i]) // 20), (ss[i], sw[i])
        assert ss["status"][i] in (0, 2), ss[i]
        assert ss["true_rel_resid"][i] <= 1e-5 * 1.0001, ss[i]


def test_split_refined_1e9(env, boxes):
    """MIXED_REFINE: FP64 residuals and FP32 correction solves, the latter on
    the split kernel too."""
    print("split refined", flush=True)
    bx, d, refs = boxes
    _, x64, st, _ = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-6, precision=2, refine_max=6,
                         refine_tol=1e-13, inner_tol=1e-4)
    for i, ref in enumerate(refs):
        o, n = int(d["offsets"][i]), ref.size
        assert np.max(np.abs(x64[o:o + n] - ref)) <= 1e-9, (SHAPES[i], st[i])
        assert st["refine_iters"][i] > 0, st[i]
    assert np.all(np.isin(st["status"], (0, 2))), st


def test_split_deterministic(env, boxes):
    """Both halves add the two partial sums in the same fixed order: repeated
    runs give the same bits, alone or beside other boxes."""
    print("split deterministic", flush=True)
    bx, d, _ = boxes
    x1, _, s1, _ = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    x2, _, s2, _ = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    assert np.array_equal(x1, x2) and np.array_equal(s1, s2)
    rng = np.random.default_rng(43)
    more = list(bx) + [synth.random_box(rng, s, dirichlet_frac=0.03) for s in [(32, 32, 32), (16, 16, 16)]]
    d3 = synth.from_boxes(more)
    x3, _, s3, _ = _run(env, d3, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    n = d["g"].size
    assert np.array_equal(x3[:n], x1)
    assert np.array_equal(s3["iters"][:len(bx)], s1["iters"])


def test_split_edge_cases(env):
    """No seed, zero Dirichlet data, seeds only in one half, the iteration cap
    and a non-finite g, on split boxes."""
    print("split edge cases", flush=True)
    rng = np.random.default_rng(45)
    a = synth.random_box(rng, (40, 40, 40), dirichlet_frac=0.02)
    nodir = (a[0], np.zeros_like(a[1]), a[2])
    zero = (a[0], a[1], np.where(a[1] != 0, 0.0, a[2]).astype(np.float32))
    # seeds only in the lower half (z < 20; arrays are [z, y, x])
    m1 = np.zeros_like(a[1])
    m1[:20] = a[1][:20]
    one_half = (a[0], m1, np.where(m1 != 0, a[2], 0.5).astype(np.float32))
    gb = a[0].copy()
    gb[30, 6, 7] = np.nan
    bad = (gb, a[1], a[2])
    d = synth.from_boxes([nodir, zero, one_half, a])
    x, _, st, plan = _run(env, d, beta=BETA, eps=EPS, tol=1e-7, precision=1)
    _, rwg, _ = env
    assert np.all(plan == rwg.PATH_RESIDENT_SPLIT), plan
    off = d["offsets"]
    n = a[0].size
    assert st["status"][0] == 5 and np.array_equal(x[off[0]:off[0] + n], nodir[2].ravel())
    assert st["status"][1] == 0 and np.all(x[off[1]:off[1] + n][a[1].ravel() == 0] == 0.0)
    for i in (2, 3):
        ref = _ref([nodir, zero, one_half, a][i])
        assert np.max(np.abs(x[off[i]:off[i] + n] - ref)) <= 1e-4, (i, st[i])
    d2 = synth.from_boxes([a, bad])
    x, _, st, _ = _run(env, d2, beta=BETA, eps=EPS, tol=1e-12, max_iter=3, precision=1, refine_max=0)
    assert st["status"][0] == 1 and st["iters"][0] == 3, st
    assert st["status"][1] == 4, st
