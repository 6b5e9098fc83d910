"""GPU parity of the batched box solve against the FP64 oracle, through the C ABI.

Tolerances: max |x_gpu - x_oracle| <= 1e-4 for the FP32 (mixed) path at
relative residual 1e-6, <= 1e-9 for the FP64-refined path and for the plain
FP64 path at relative residual 1e-12.  The oracle reference is the unique
solution of the box's Dirichlet problem (oracle.rw.solve_box; Jacobi-PCG to
1e-14, pinned against sparse/dense factorisations on the CPU).
"""

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


def _ref(box, beta=BETA, eps=EPS):
    g, m, x = box
    return orw.solve_box(g, m, x, beta, eps, method="pcg", tol=1e-14).ravel()


def _run(env, d, x64=False, **params):
    torch, rwg, dev = env
    g = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    x = torch.from_numpy(d["x"]).to(dev)
    xd = torch.zeros(x.numel(), dtype=torch.float64, device=dev) if x64 else None
    st = rwg.solve_bricks(g, m, x, d["shapes"], d["offsets"], x64=xd, **params)
    torch.cuda.synchronize()
    return x.cpu().numpy(), (xd.cpu().numpy() if x64 else None), rwg.stats_to_numpy(st)


def _mixed_set(seed=5):
    rng = np.random.default_rng(seed)
    boxes = list(synth.stress_boxes(n=10, seed=seed)["boxes"])
    for s in [(1, 1, 40), (3, 4, 5), (7, 1, 9), (33, 2, 3), (2, 31, 2), (40, 40, 40)]:
        boxes.append(synth.random_box(rng, s, dirichlet_frac=0.03))
    return boxes


@pytest.fixture(scope="module")
def mixed_set():
    boxes = _mixed_set()
    return boxes, synth.from_boxes(boxes), [_ref(b) for b in boxes]


def test_mixed_matches_oracle(env, mixed_set):
    boxes, d, refs = mixed_set
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    for i, ref in enumerate(refs):
        o, n = int(d["offsets"][i]), ref.size
        err = np.max(np.abs(x[o:o + n] - ref))
        assert err <= 1e-4, (i, d["shapes"][i], err, st[i])
        # boxes of the stress recipe meet tol in FP64 (possibly after refinement);
        # the extra random boxes include a weak-link chain (cond ~1e7) where an
        # FP32-stored x cannot reach tol relative to its tiny ||b||: STALLED is
        # the honest outcome there and the error bound above still holds.
        allowed = (0, 2) if i < 10 else (0, 2, 3)
        assert st["status"][i] in allowed, (i, st[i])
        if st["status"][i] in (0, 2):
            # MIXED refines only above stall_ratio (10) x tol
            assert st["true_rel_resid"][i] <= 1e-5 * 1.0001


def test_refined_matches_oracle_1e9(env, mixed_set):
    boxes, d, refs = mixed_set
    x, x64, st = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-6, precision=2,
                      refine_max=6, refine_tol=1e-13, inner_tol=1e-4)
    for i, ref in enumerate(refs):
        o, n = int(d["offsets"][i]), ref.size
        err = np.max(np.abs(x64[o:o + n] - ref))
        assert err <= 1e-9, (i, d["shapes"][i], err, st[i])
        assert np.max(np.abs(x[o:o + n] - ref)) <= 1e-6


def test_fp64_matches_oracle(env, mixed_set):
    boxes, d, refs = mixed_set
    _, x64, st = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-12, precision=0)
    for i, ref in enumerate(refs):
        o, n = int(d["offsets"][i]), ref.size
        err = np.max(np.abs(x64[o:o + n] - ref))
        assert err <= 1e-9, (i, d["shapes"][i], err, st[i])
        assert st["status"][i] == 0


def test_seeded_voxels_unchanged(env, mixed_set):
    boxes, d, refs = mixed_set
    x, _, _ = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    s = d["mask"] != 0
    assert np.array_equal(x[s], d["x"][s])


def test_edge_cases(env):
    rng = np.random.default_rng(9)
    # 0: no seed at all; 1: every voxel seeded; 2: zero Dirichlet data; 3: chain closed form;
    # 4: single unknown voxel
    g0, _, _ = synth.random_box(rng, (4, 5, 6))
    x0 = rng.random(g0.shape).astype(np.float32)
    nodir = (g0, np.zeros(g0.shape, np.uint8), x0)
    g1 = rng.random((3, 3, 3)).astype(np.float32)
    alls = (g1, np.ones(g1.shape, np.uint8), rng.random(g1.shape).astype(np.float32))
    g2, m2, _ = synth.random_box(rng, (6, 6, 6), dirichlet_frac=0.1)
    zero = (g2, m2, np.where(m2 != 0, 0.0, rng.random(g2.shape)).astype(np.float32))
    n = 25
    gl = rng.random(n).astype(np.float32)
    mc = np.zeros(n, np.uint8)
    mc[0] = mc[-1] = 1
    xc = np.zeros(n, np.float32)
    xc[-1] = 1.0
    chain = (gl.reshape(n, 1, 1), mc.reshape(n, 1, 1), xc.reshape(n, 1, 1))
    one = (np.array([[[0.1, 0.5, 0.9]]], np.float32), np.array([[[1, 0, 1]]], np.uint8),
           np.array([[[0.0, 0.3, 1.0]]], np.float32))
    boxes = [nodir, alls, zero, chain, one]
    d = synth.from_boxes(boxes)
    x, _, st = _run(env, d, beta=20.0, eps=1e-3, tol=1e-7, precision=1)
    off = d["offsets"]
    assert st["status"][0] == 5 and np.array_equal(x[off[0]:off[0] + g0.size], x0.ravel())
    assert st["status"][1] == 0 and st["iters"][1] == 0
    assert np.array_equal(x[off[1]:off[1] + 27], alls[2].ravel())
    assert st["status"][2] == 0 and np.all(x[off[2]:off[2] + 216][m2.ravel() == 0] == 0.0)
    w = np.exp(-20.0 * np.diff(gl.astype(np.float64)) ** 2) + 1e-3
    R = 1.0 / w
    expect = np.concatenate([[0.0], np.cumsum(R)]) / R.sum()
    assert np.max(np.abs(x[off[3]:off[3] + n] - expect)) <= 1e-4
    # the plain FP64 path reproduces the closed form to FP64 accuracy
    _, x64, st64 = _run(env, d, x64=True, beta=20.0, eps=1e-3, tol=1e-13, precision=0)
    assert np.max(np.abs(x64[off[3]:off[3] + n] - expect)) <= 1e-9
    assert st64["status"][0] == 5 and st64["status"][1] == 0
    w01 = np.exp(-20.0 * 0.16) + 1e-3
    w12 = np.exp(-20.0 * 0.16) + 1e-3
    assert abs(x[off[4] + 1] - (w01 * 0.0 + w12 * 1.0) / (w01 + w12)) < 1e-6


def test_iteration_cap_and_nonfinite(env):
    rng = np.random.default_rng(10)
    a = synth.random_box(rng, (12, 12, 12), dirichlet_frac=0.02)
    gb = a[0].copy()
    gb[3, 4, 5] = np.nan
    bad = (gb, a[1], a[2])
    d = synth.from_boxes([a, bad])
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-12, max_iter=1, precision=1, refine_max=0)
    assert st["status"][0] == 1 and st["iters"][0] == 1
    d2 = synth.from_boxes([bad])
    _, _, st2 = _run(env, d2, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    assert st2["status"][0] == 4


def test_multi_rhs_equals_separate(env):
    rng = np.random.default_rng(12)
    boxes = [synth.random_box(rng, s, dirichlet_frac=0.05) for s in [(9, 8, 7), (16, 5, 3), (20, 20, 20)]]
    d = synth.from_boxes(boxes)
    R = 3
    xs = [np.where(d["mask"] != 0, rng.random(d["x"].size), 0.0).astype(np.float32) for _ in range(R)]
    inter = np.stack(xs, axis=1).ravel()
    d3 = dict(d, x=inter)
    x3, _, st3 = _run(env, d3, beta=BETA, eps=EPS, tol=1e-7, precision=1, nrhs=3)
    x3 = x3.reshape(-1, R)
    for k in range(R):
        dk = dict(d, x=xs[k])
        xk, _, _ = _run(env, dk, beta=BETA, eps=EPS, tol=1e-7, precision=1)
        assert np.max(np.abs(x3[:, k] - xk)) < 1e-5
        for i, (g, m, _) in enumerate(boxes):
            o = int(d["offsets"][i])
            ref = orw.solve_box(g, m, xs[k][o:o + g.size].reshape(g.shape), BETA, EPS, method="pcg", tol=1e-14)
            assert np.max(np.abs(x3[o:o + g.size, k] - ref.ravel())) <= 1e-4


def test_deterministic_and_order_independent(env, mixed_set):
    boxes, d, _ = mixed_set
    xa, _, sa = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    xb, _, sb = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    assert np.array_equal(xa, xb) and np.array_equal(sa, sb)
    rev = synth.from_boxes(boxes[::-1])
    xr, _, sr = _run(env, rev, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    n = len(boxes)
    for i in range(n):
        j = n - 1 - i
        oi, oj, sz = int(d["offsets"][i]), int(rev["offsets"][j]), boxes[i][0].size
        assert np.array_equal(xa[oi:oi + sz], xr[oj:oj + sz])
        assert sa["iters"][i] == sr["iters"][j]


def test_plain_sphere_single_domain(env):
    g, m, x0, inside = synth.plain_sphere()
    d = synth.from_boxes([(g, m, x0)])
    ref = orw.solve_box(g, m, x0, BETA, EPS, method="pcg", tol=1e-13).ravel()
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    assert np.max(np.abs(x - ref)) <= 1e-4, st
    _, x64, st64 = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-6, precision=0)
    assert np.max(np.abs(x64 - ref)) <= 1e-4, st64
    # the sphere is segmented (sanity, not parity)
    assert ((x.reshape(g.shape) > 0.5) == inside).mean() > 0.99


def test_full_size_stress_sampled(env):
    """All 8192 mixed-shape boxes in one launch (the benchmark configuration);
    sampled boxes against the oracle, every box against its own residual."""
    d = synth.stress_boxes(n=8192, seed=3)
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    assert np.all(np.isin(st["status"], (0, 2))), np.unique(st["status"], return_counts=True)
    assert np.all(st["true_rel_resid"] <= 1e-5 * 1.0001)
    rng = np.random.default_rng(0)
    for i in rng.choice(len(d["boxes"]), 12, replace=False):
        ref = _ref(d["boxes"][i])
        o = int(d["offsets"][i])
        assert np.max(np.abs(x[o:o + ref.size] - ref)) <= 1e-4, (i, st[i])


def test_domain_solver_boxes(env):
    """Large single boxes (wide planes of >= 2^16 voxels, or >= 2^20 voxels)
    take the multi-workgroup solver, at most 64 per call, all of them in each
    launch; the rest of such a call runs the per-box kernels.  Every path
    against the oracle."""
    rng = np.random.default_rng(21)
    wide = synth.random_box(rng, (48, 48, 40), dirichlet_frac=0.02)
    tall = synth.random_box(rng, (32, 32, 1024), dirichlet_frac=0.05)
    d = synth.from_boxes([wide, tall])
    refs = [_ref(b) for b in (wide, tall)]
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    _, x64, st64 = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-6, precision=2,
                        refine_max=6, refine_tol=1e-13, inner_tol=1e-4)
    _, f64, stf = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-12, precision=0)
    for i, ref in enumerate(refs):
        o, n = int(d["offsets"][i]), ref.size
        assert st["status"][i] in (0, 2) and np.max(np.abs(x[o:o + n] - ref)) <= 1e-4, st[i]
        assert st64["status"][i] == 2 and np.max(np.abs(x64[o:o + n] - ref)) <= 1e-9, st64[i]
        assert stf["status"][i] == 0 and np.max(np.abs(f64[o:o + n] - ref)) <= 1e-9, stf[i]
        assert st["iters"][i] > 0 and stf["true_rel_resid"][i] <= 1e-12 * 1.01


def test_domain_solver_multi_rhs_and_cap(env):
    """65 wide boxes of 2^16+ voxels: the 64 largest share the domain
    solver's launches, the smallest goes to the global-memory march; nrhs = 2
    and 3 against per-rhs oracle solves, and boxes of the batched call against
    the same boxes solved one per call."""
    _, rwg, _ = env
    rng = np.random.default_rng(22)
    # sizes differ so that the boxes take different workgroup counts; the last is the smallest
    boxes = [synth.random_box(rng, (46, 46, 31 + (i % 5)), dirichlet_frac=0.03) for i in range(64)]
    boxes.append(synth.random_box(rng, (46, 46, 31), dirichlet_frac=0.03))
    d = synth.from_boxes(boxes)
    ctx = rwg.Context(0)
    plan = ctx.solve_plan(rwg.solve_params(beta=BETA, eps=EPS, tol=1e-7, precision=1),
                          rwg.bricks_array(d["shapes"], d["offsets"]), d["g"].size)
    ctx.close()
    assert int(np.sum(plan == rwg.PATH_DOMAIN)) == 64 and plan[64] != rwg.PATH_DOMAIN, plan
    for R in (2, 3):
        xs = [np.where(d["mask"] != 0, rng.random(d["x"].size), 0.0).astype(np.float32) for _ in range(R)]
        dR = dict(d, x=np.stack(xs, axis=1).ravel())
        xR, _, st = _run(env, dR, beta=BETA, eps=EPS, tol=1e-7, precision=1, nrhs=R)
        xR = xR.reshape(-1, R)
        assert np.all(np.isin(st["status"], (0, 2))), st
        for i in (0, 33, 63, 64):
            g, m, _ = boxes[i]
            o = int(d["offsets"][i])
            for k in range(R):
                ref = orw.solve_box(g, m, xs[k][o:o + g.size].reshape(g.shape), BETA, EPS, method="pcg",
                                    tol=1e-14)
                assert np.max(np.abs(xR[o:o + g.size, k] - ref.ravel())) <= 1e-4, (R, i, k)
    # same boxes solved one call per box agree with the batched call; the
    # iteration counts of the domain boxes are their own
    x1, _, s1 = _run(env, d, beta=BETA, eps=EPS, tol=1e-7, precision=1)
    for i in (3, 40, 64):
        di = synth.from_boxes([boxes[i]])
        xi, _, si = _run(env, di, beta=BETA, eps=EPS, tol=1e-7, precision=1)
        o = int(d["offsets"][i])
        assert np.max(np.abs(x1[o:o + boxes[i][0].size] - xi)) <= 1e-5
        if i < 64:
            assert s1["iters"][i] == si["iters"][0], (i, s1[i], si[0])


def test_resident_kernel_matches_oracle_and_streaming(env):
    """Boxes that fit one CU run an on-chip PCG (schedule 0): g and p, or p
    and the edge weights, in LDS, and p in LDS with the weights streamed
    from cache for boxes up to 32^3 (schedule 4: for every box that fits);
    schedule 1 forces the streaming kernels.  All against the oracle, on
    ragged sizes of every variant (slots past a box's end included)."""
    rng = np.random.default_rng(31)
    shapes = [(7, 13, 11), (31, 17, 33), (20, 20, 12), (3, 3, 3), (1, 1, 5), (32, 9, 32), (5, 32, 32),
              (16, 16, 16), (32, 32, 17), (9, 1, 40), (32, 32, 32), (30, 31, 33), (26, 29, 27)]
    boxes = [synth.random_box(rng, s, dirichlet_frac=0.03) for s in shapes]
    d = synth.from_boxes(boxes)
    refs = [_ref(b) for b in boxes]
    xr, _, sr = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1, schedule=0)
    xs, _, ss = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1, schedule=1)
    xg, _, sg = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1, schedule=4)
    _, x64, s64 = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-6, precision=2, refine_max=6,
                       refine_tol=1e-13, inner_tol=1e-4, schedule=0)
    _, x64g, s64g = _run(env, d, x64=True, beta=BETA, eps=EPS, tol=1e-6, precision=2, refine_max=6,
                         refine_tol=1e-13, inner_tol=1e-4, schedule=4)
    _, rwg, _ = env
    bricks = rwg.bricks_array(d["shapes"], d["offsets"])
    plan0 = rwg.context().solve_plan(rwg.solve_params(schedule=0), bricks, d["g"].size)
    plan4 = rwg.context().solve_plan(rwg.solve_params(schedule=4), bricks, d["g"].size)
    nv = np.prod(np.asarray(shapes), axis=1)
    # boxes above 10240 voxels (up to 32^3) take the streamed-weights kernel
    # by default, smaller ones keep the weights on chip (in registers up to
    # 5120 voxels, else in LDS); with schedule 4 every box up to 32768
    # voxels streams its weights
    assert np.all(plan0[nv > 10240] == rwg.PATH_RESIDENT_STREAMED), plan0
    assert np.all(plan0[nv <= 10240] == rwg.PATH_RESIDENT), plan0
    assert np.all(plan4 == rwg.PATH_RESIDENT_STREAMED), plan4
    for i, ref in enumerate(refs):
        o, n = int(d["offsets"][i]), ref.size
        assert np.max(np.abs(xr[o:o + n] - ref)) <= 1e-4, (shapes[i], sr[i])
        assert np.max(np.abs(xg[o:o + n] - ref)) <= 1e-4, (shapes[i], sg[i])
        # two stops at relative residual 1e-6 (each up to about 2e-5 from the
        # solution on the weak-link chain boxes) agree to the sum of the two
        assert np.max(np.abs(xr[o:o + n] - xs[o:o + n])) <= 4e-5, (shapes[i], sr[i], ss[i])
        assert np.max(np.abs(xg[o:o + n] - xs[o:o + n])) <= 4e-5, (shapes[i], sg[i], ss[i])
        assert np.max(np.abs(x64[o:o + n] - ref)) <= 1e-9, (shapes[i], s64[i])
        assert np.max(np.abs(x64g[o:o + n] - ref)) <= 1e-9, (shapes[i], s64g[i])
        assert abs(int(sr["iters"][i]) - int(ss["iters"][i])) <= max(3, ss["iters"][i] // 20), (sr[i], ss[i])
        assert abs(int(sg["iters"][i]) - int(ss["iters"][i])) <= max(3, ss["iters"][i] // 20), (sg[i], ss[i])
    assert np.all(np.isin(sg["status"], (0, 2))) and np.all(np.isin(s64g["status"], (0, 2)))
    assert np.all(np.isin(sr["status"], (0, 2))) and np.all(s64["status"] == 2) | np.all(np.isin(s64["status"], (0, 2)))


def test_four_voxel_layout_over_box_depths(env):
    """The streamed-weights kernel's four-voxel layout on 32 x 32 planes at
    every kind of depth: the smallest box it takes (nz = 11), the 17408-slot
    span whose last group belongs to half the threads (nz up to 17), the
    32768-slot span (nz 18 to 32); unused slots past each box's end.  Each
    box against the oracle, one launch per span."""
    print("four-voxel depths", flush=True)
    _, rwg, _ = env
    rng = np.random.default_rng(91)
    depths = (11, 14, 17, 18, 24, 31, 32)
    boxes = [synth.random_box(rng, (32, 32, nz), dirichlet_frac=0.02) for nz in depths]
    d = synth.from_boxes(boxes)
    plan = rwg.context().solve_plan(rwg.solve_params(), rwg.bricks_array(d["shapes"], d["offsets"]), d["g"].size)
    assert np.all(plan == rwg.PATH_RESIDENT_STREAMED), plan
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    off = d["offsets"]
    for i, b in enumerate(boxes):
        ref = _ref(b)
        err = np.max(np.abs(x[off[i]:off[i] + ref.size] - ref))
        assert err <= 1e-4, (depths[i], err, st[i])
        assert st["status"][i] in (0, 2) and st["true_rel_resid"][i] <= 1e-5 * 1.0001, (depths[i], st[i])
        # seeded voxels keep their values
        mk = b[1].ravel() != 0
        assert np.array_equal(x[off[i]:off[i] + ref.size][mk], b[2].ravel()[mk]), depths[i]


def test_streamed_weights_edge_cases(env):
    """The streamed-weights resident kernel on its special boxes: a non-finite
    g, the iteration cap, no seed, zero Dirichlet data, a single unknown
    voxel, 32x32-plane boxes next to other plane shapes (the four-voxel
    layout of 32 x 32 planes and the one-voxel layout with run-time
    neighbour offsets: the same FP32 arithmetic per voxel, FP64 sums in
    another order), and slots past the end of a box."""
    rng = np.random.default_rng(77)
    a = synth.random_box(rng, (32, 32, 20), dirichlet_frac=0.02)     # span 32768, 32x32 planes
    b = synth.random_box(rng, (32, 32, 12), dirichlet_frac=0.02)     # span 17408, 32x32 planes
    gb = a[0].copy()
    gb[5, 6, 7] = np.nan
    bad = (gb, a[1], a[2])
    nodir = (b[0], np.zeros_like(b[1]), b[2])
    zero = (b[0], b[1], np.where(b[1] != 0, 0.0, b[2]).astype(np.float32))
    one_m = np.ones_like(b[1])
    one_m[7, 3, 9] = 0
    one = (b[0], one_m, b[2])
    # iteration cap and non-finite
    d = synth.from_boxes([a, bad])
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-12, max_iter=3, precision=1, refine_max=0)
    assert st["status"][0] == 1 and st["iters"][0] == 3, st
    assert st["status"][1] == 4, st
    # no seed, zero data, one unknown voxel, against the oracle
    boxes = [nodir, zero, one, b]
    d = synth.from_boxes(boxes)
    _, rwg, _ = env
    plan = rwg.context().solve_plan(rwg.solve_params(), rwg.bricks_array(d["shapes"], d["offsets"]), d["g"].size)
    assert np.all(plan == rwg.PATH_RESIDENT_STREAMED), plan
    x, _, st = _run(env, d, beta=BETA, eps=EPS, tol=1e-7, precision=1)
    off = d["offsets"]
    assert st["status"][0] == 5 and np.array_equal(x[off[0]:off[0] + b[0].size], nodir[2].ravel())
    assert st["status"][1] == 0 and np.all(x[off[1]:off[1] + b[0].size][b[1].ravel() == 0] == 0.0)
    for i in (2, 3):
        ref = _ref(boxes[i])
        assert np.max(np.abs(x[off[i]:off[i] + ref.size] - ref)) <= 1e-4, (i, st[i])
    # 32x32-plane boxes alone (four-voxel layout in both launches) and with a
    # 31x33 box joining b's launch (one-voxel layout there): a's launch is the
    # same in both runs, bit for bit; b agrees to the FP64 sums' rounding
    c = synth.random_box(rng, (31, 33, 16), dirichlet_frac=0.02)
    d1 = synth.from_boxes([a, b])
    d2 = synth.from_boxes([a, b, c])
    p1 = rwg.context().solve_plan(rwg.solve_params(), rwg.bricks_array(d1["shapes"], d1["offsets"]), d1["g"].size)
    assert np.all(p1 == rwg.PATH_RESIDENT_STREAMED)
    x1, _, s1 = _run(env, d1, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    x2, _, s2 = _run(env, d2, beta=BETA, eps=EPS, tol=1e-6, precision=1)
    na, n = a[0].size, a[0].size + b[0].size
    assert np.array_equal(x1[:na], x2[:na]) and s1["iters"][0] == s2["iters"][0]
    assert np.max(np.abs(x1[na:n] - x2[na:n])) <= 1e-5 and abs(int(s1["iters"][1]) - int(s2["iters"][1])) <= 1
    ref_b = _ref(b)
    assert np.max(np.abs(x1[na:n] - ref_b)) <= 1e-4, s1[1]
    ref_c = _ref(c)
    assert np.max(np.abs(x2[n:n + ref_c.size] - ref_c)) <= 1e-4, s2[2]
