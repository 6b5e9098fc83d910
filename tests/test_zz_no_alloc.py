"""rw_solve_bricks_noalloc (the solve that allocates nothing, for callers that
cannot call hipMalloc) against rw_solve_bricks through the C ABI.

Both calls run the same kernels on the same boxes, so x, x64 and the stats
must agree bit for bit.  Two no-allocation calls in a row, the second on a
smaller batch, check that the shared device scratch (which keeps the last
call's contents) needs nothing cleared by the caller.  A batch beyond the
scratch is rejected before anything is queued.  Sampled boxes are also held
to the FP64 oracle (1e-4 for the mixed path)."""

import numpy as np
import pytest

import synth
from oracle import rw as orw

pytestmark = pytest.mark.gpu

BETA, EPS = 128.0, 1e-6


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2103_09564_amd as rwg
    assert torch.cuda.is_available()
    return torch, rwg, torch.device("cuda:0")


def _batch(seed, n, extra=()):
    rng = np.random.default_rng(seed)
    boxes = list(synth.stress_boxes(n=n, seed=seed)["boxes"])
    for s in extra:
        boxes.append(synth.random_box(rng, s, dirichlet_frac=0.03))
    return boxes, synth.from_boxes(boxes)


def _solve(env, d, noalloc, x64=False, **params):
    torch, rwg, dev = env
    ctx = rwg.context(0)
    g = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    x = torch.from_numpy(d["x"]).to(dev)
    xd = torch.zeros(x.numel(), dtype=torch.float64, device=dev) if x64 else None
    b = rwg.bricks_array(d["shapes"], d["offsets"])
    st = torch.zeros((len(b), rwg.STATS_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    p = rwg.solve_params(**params)
    if noalloc:
        ctx.rw_solve_bricks_noalloc(p, b, g, m, x, x64=xd, stats=st)
    else:
        ctx.rw_solve_bricks(p, b, g, m, x, x64=xd, stats=st)
    torch.cuda.synchronize()
    return x.cpu().numpy(), (xd.cpu().numpy() if x64 else None), rwg.stats_to_numpy(st)


def _same(a, b):
    xa, x64a, sa = a
    xb, x64b, sb = b
    assert np.array_equal(xa, xb)
    if x64a is not None:
        assert np.array_equal(x64a, x64b)
    for k in ("iters", "status", "refine_steps", "refine_iters", "rel_resid", "true_rel_resid"):
        assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("precision,x64", [(1, False), (2, True), (0, True)])
def test_noalloc_matches_solve_two_calls(env, precision, x64):
    print(f"noalloc precision={precision}", flush=True)
    params = dict(beta=BETA, eps=EPS, tol=1e-6, precision=precision, refine_max=2 if precision == 2 else 1)
    # first call: the stress shapes (both resident paths and the window
    # march for the odd boxes) and a wide box for the multi-workgroup domain
    # solver (its done flag read synchronously here); second call: a smaller
    # batch
    big = _batch(21, 24, extra=[(40, 40, 40), (7, 1, 9), (33, 2, 3), (48, 48, 40)])
    small = _batch(22, 6, extra=[(3, 4, 5)])
    for boxes, d in (big, small):
        ref = _solve(env, d, False, x64=x64, **params)
        got = _solve(env, d, True, x64=x64, **params)
        _same(ref, got)
        for i in (0, len(boxes) - 1):
            gb, mb, xb = boxes[i]
            want = orw.solve_box(gb, mb, xb, BETA, EPS, method="pcg", tol=1e-14).ravel()
            o, n = int(d["offsets"][i]), gb.size
            assert np.max(np.abs(got[0][o:o + n] - want)) <= 1e-4, (i, d["shapes"][i])


def test_noalloc_nrhs3(env):
    print("noalloc nrhs=3", flush=True)
    rng = np.random.default_rng(23)
    boxes = [synth.random_box(rng, s, dirichlet_frac=0.05) for s in [(32, 32, 17), (16, 16, 16), (20, 9, 11)]]
    d = synth.from_boxes(boxes)
    xs = [np.where(d["mask"] != 0, rng.random(d["x"].size), 0.0).astype(np.float32) for _ in range(3)]
    d3 = dict(d, x=np.stack(xs, axis=1).ravel())
    params = dict(beta=BETA, eps=EPS, tol=1e-6, precision=1, nrhs=3)
    _same(_solve(env, d3, False, **params), _solve(env, d3, True, **params))


def test_noalloc_rejects_batches_beyond_scratch(env):
    torch, rwg, dev = env
    print("noalloc over the limit", flush=True)
    cap = rwg.noalloc_scratch_bytes()
    n = cap // (32 ** 3 * 20) + 8     # 32^3 boxes: more than the scratch holds
    shapes = np.tile([32, 32, 32], (n, 1))
    offsets = np.arange(n, dtype=np.int64) * 32 ** 3
    nv = int(n * 32 ** 3)
    g = torch.zeros(nv, dtype=torch.float32, device=dev)
    m = torch.ones(nv, dtype=torch.uint8, device=dev)
    x = torch.zeros(nv, dtype=torch.float32, device=dev)
    with pytest.raises(rwg.RWError) as ei:
        rwg.context(0).rw_solve_bricks_noalloc(rwg.solve_params(), rwg.bricks_array(shapes, offsets), g, m, x)
    assert ei.value.code == rwg.RW_E_INVAL and "scratch" in str(ei.value)
