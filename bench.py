"""Benchmark: batched brick-local random-walker PCG on one MI355X.

Workload (the batching + precision stress configuration): 8192 boxes with
shapes drawn uniformly from {32^3, 32x32x17, 32x9x32, 5x32x32, 16^3},
Gaussian-smoothed noise intensities scaled to [0, 1] per box, random Dirichlet
faces and 1 % interior seeds (recipe in ``synth.stress_boxes``), beta 128,
eps 1e-6, per-box relative residual tolerance 1e-6.  All inputs are resident
in HBM before the timed region.

A step is one ``rw_solve_bricks`` call over all 8192 boxes (x reset to its
initial values first, inside the step).  The headline value is
voxel-iterations per second of the mixed-precision path (FP32 stencil and
vectors, FP64 reductions, FP64 true-residual check with refinement where it
misses tol): sum over boxes of (box voxels x PCG iterations executed, main +
correction solves) / seconds per step.  The plain-FP64 path runs on the same
workload for the mixed-vs-FP64 comparison.

Prints ONE JSON line.  --gpus N with N > 1 exits: this build targets one GPU.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
BYTES_PER_VOXEL_ITER = 28      # streaming formulation: read x, r, p, g; write x, r, p (FP32, one rhs)
SEGMENT_BYTES_PER_VOXEL_ITER = 16  # streamed-weights resident kernel: read w+x, w+y, w+z, 1/d per iteration
RESIDENT_BYTES_PER_VOXEL = 13  # weights-in-LDS kernel: read g, mask, x once per solve, write x once
BETA, EPS, TOL = 128.0, 1e-6, 1e-6
N_BOXES, SEED = 8192, 3
# workloads run only on request (--only NAME): minutes of GPU time
ON_REQUEST = ("shells_full", "memory_ceilings", "tubes_512_host_finest")
EXTRAS = ("plain_sphere_64", "tubes_512_hierarchy", "blobs_512x32_adjoint", "shells_hierarchy_incremental",
          "cells_256_ablation", "cells_brick_growth", "pruning_table_256", "stress_streamed_from_host")


# The sources that define, plan and launch the kernels of the headline
# workload (the resident and streaming PCG kernels, the init, check and
# finish phases, the box plan); the hierarchy and domain-solver sources do
# not touch them.
HOT_SOURCES = ("capi.hip", "common.h", "pcg.hip", "resident.hip")


def source_hash():
    """Hash of the library sources behind the headline workload's kernels."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2103_09564_amd", "csrc")
    for f in HOT_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(split):
    """HBM bytes of the dominant kernel from the committed counter summary, if
    it was taken on the current kernel sources (else None): of the 32^3 launch
    when the two streamed-weights launches run on streams of their own
    (`split`), else of the two launches together."""
    path = os.path.join(ROOT, "profiles", "k_pcg_resg4_stress8192.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("bench-traffic:"):
            rec = json.loads(line.split(":", 1)[1])
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("hbm_bytes_32cube_launch" if split else "hbm_bytes_streamed_launches")


def measure_ceilings(torch, rwg, ctx, reps=5):
    """Memory ceilings measured on this device with the library's probe
    kernels (16-byte loads from every CU): HBM read over a 4 GiB buffer (16x
    the 256 MB last-level cache), HBM copy of 2 GiB, and re-reads of a
    128 MiB buffer (32 passes in one launch) that stays in the last-level
    (Infinity) cache.  Best of `reps` launches, GB/s."""
    dev = torch.device("cuda:0")
    part = torch.empty(rwg.probe_blocks(), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def best(fn, nbytes):
        fn()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            ms.append(a.elapsed_time(b))
        return nbytes / (min(ms) * 1e-3) / 1e9, min(ms)

    big = torch.ones(1 << 30, dtype=torch.float32, device=dev)          # 4 GiB
    hbm_read = max(best(lambda: ctx.probe_read(big, 1, part, unroll=u, stream=stream), big.numel() * 4)[0]
                   for u in (4, 8, 16))
    del big
    src = torch.ones(1 << 29, dtype=torch.float32, device=dev)          # 2 GiB
    dst = torch.empty_like(src)
    hbm_copy, _ = best(lambda: ctx.probe_copy(dst, src, stream=stream), 2 * src.numel() * 4)
    del src, dst
    small = torch.ones(1 << 25, dtype=torch.float32, device=dev)        # 128 MiB
    passes = 32
    llc = max(best(lambda: ctx.probe_read(small, passes, part, unroll=u, stream=stream), passes * small.numel() * 4)[0]
              for u in (4, 8, 16))
    del small
    torch.cuda.synchronize()
    return {"hbm_read_GBps": hbm_read, "hbm_copy_GBps": hbm_copy, "llc_reread_GBps": llc,
            "note": "rw_probe_read / rw_probe_copy (16-byte loads, 2048 workgroups of 256 threads; reads with 4, 8 "
                    "or 16 loads in flight per thread, the best taken): read of 4 GiB, copy of 2 GiB (read + write "
                    "bytes), 32 re-reads of 128 MiB (last-level cache); best of 5 launches"}


def roofline_alone(torch, rwg, ctx, d, g, m, x, x0, stream, reps=3):
    """The dominant launch without the others beside it: the 32^3 boxes of
    the workload solved by themselves (same parameters, outside the timed
    steps; their offsets index the same arrays), the launch timed by the
    library's HIP events on its stream.  The kernel's own rate; in the timed
    step it shares the chip with the other launches."""
    import numpy as np
    sizes = d["shapes"].prod(axis=1)
    sel = np.where(sizes == 32 ** 3)[0]
    if len(sel) == 0:
        return None
    b = rwg.bricks_array(d["shapes"][sel], d["offsets"][sel])
    p = rwg.solve_params(beta=BETA, eps=EPS, tol=TOL, precision=rwg.PREC_MIXED, refine_max=1, inner_tol=1e-4)
    st = torch.empty((len(sel), 32), dtype=torch.uint8, device=g.device)
    x.copy_(x0)
    ctx.rw_solve_bricks(p, b, g, m, x, stats=st, stream=stream)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ms = []
    for _ in range(reps):
        x.copy_(x0)
        ctx.rw_solve_bricks(p, b, g, m, x, stats=st, stream=stream)
        ms.append(ctx.last_timing()["stream_ms"])
    ctx.set_timing(False)
    torch.cuda.synchronize()
    s = rwg.stats_to_numpy(st)
    vi = int(np.sum(sizes[sel] * s["iters"].astype(np.int64)))
    t = float(np.median(ms)) / 1e3
    ach = SEGMENT_BYTES_PER_VOXEL_ITER * vi / t / 1e9
    return {"boxes": int(len(sel)), "voxel_iters": vi, "ms": t * 1e3, "achieved": ach, "frac": ach / HBM_PEAK_GBS,
            "note": "the 32^3 boxes solved alone (median of 3 calls, outside the timed steps): the launch's own "
                    "rate at 16 B per voxel-iteration; in the timed step it shares the chip with the other launches"}


def probe_read_sweep(torch, rwg, ctx, reps=4):
    """Read bandwidth against buffer size: each buffer re-read in one probe
    launch (up to 64 passes, about 4 GiB in all), best of `reps` launches for
    4, 8 and 16 loads in flight per thread, GB/s.  Buffers up to 32 MiB stay
    in the XCDs' L2, those up to the 256 MB last-level cache in that cache."""
    dev = torch.device("cuda:0")
    part = torch.empty(rwg.probe_blocks(), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    rows = []
    for mib in (8, 16, 32, 64, 96, 128, 192, 256, 384, 512, 1024, 4096):
        buf = torch.ones(mib << 18, dtype=torch.float32, device=dev)
        passes = max(1, min(64, 4096 // mib))
        row = {"MiB": mib, "passes": passes}
        for u in (4, 8, 16):
            ms = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                ctx.probe_read(buf, passes, part, unroll=u, stream=stream)
                b.record(stream)
                b.synchronize()
                ms.append(a.elapsed_time(b))
            row[f"GBps_unroll{u}"] = passes * (mib << 20) / (min(ms) * 1e-3) / 1e9
        print(json.dumps(row), flush=True)
        rows.append(row)
        del buf
    return rows


def _oracle_worker(args):
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import rw as orw
    g, m, x, deadline = args
    if time.time() > deadline:
        return None
    with threadpool_limits(1):
        A, b, U, M = orw.dirichlet_system(g, m, x, BETA, EPS)
        xu, it, _ = orw.pcg(A, b, x0=np.asarray(x, np.float64).ravel()[U], tol=TOL)
    out = np.asarray(x, np.float64).ravel().copy()
    out[U] = xu
    return g.size * it, out


def _oracle_exact(args):
    from threadpoolctl import threadpool_limits
    from oracle import rw as orw
    g, m, x = args
    with threadpool_limits(1):
        return orw.solve_box(g, m, x, BETA, EPS, method="pcg", tol=1e-13).ravel()


def oracle_exact_sample(boxes, idx):
    """cpu_baseline leg: the exact solutions (oracle PCG to 1e-13) of the
    sampled boxes, for the error of each GPU path against the true answer."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(os.cpu_count() or 1, 16)) as pool:
        return dict(zip(idx, pool.map(_oracle_exact, [boxes[i] for i in idx], chunksize=1)))


def cpu_baseline(boxes, seconds=15.0):
    """The FP64 oracle (sparse Laplacian + Jacobi-PCG at the same tol) on a
    time-bounded sample of the same boxes, one box per process."""
    import multiprocessing as mp
    workers = min(os.cpu_count() or 1, 16)
    n = min(len(boxes), 4096)
    t0 = time.time()
    deadline = t0 + seconds
    vi, done, sols = 0, 0, {}
    with mp.get_context("fork").Pool(workers) as pool:
        for i, r in enumerate(pool.imap(_oracle_worker, [(b[0], b[1], b[2], deadline) for b in boxes[:n]],
                                        chunksize=1)):
            if r is None:
                continue
            vi += r[0]
            done += 1
            sols[i] = r[1]
    el = time.time() - t0
    return {"value": vi / el, "unit": "voxel-iters/s", "cores": workers, "kind": "oracle",
            "sample": f"first {done} of the {len(boxes)} boxes within a {seconds:.0f} s budget "
                      f"({el:.1f} s wall, FP64 scipy CSR + numpy Jacobi-PCG, tol {TOL:g}, "
                      f"one single-threaded process per core)"}, sols


# ---------------------------------------------------------------------------
# Further workloads (reported beside the headline, not part of it)
# ---------------------------------------------------------------------------

def _best_ms(torch, fn, reps):
    best = float("inf")
    out = None
    for _ in range(reps):
        out = None  # (the previous repetition's result is released outside the timed call)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) * 1e3)
    return best, out


def oracle_plain_solve(g, m, x):
    """cpu_baseline leg: exact reference of one box (FP64 oracle, tol 1e-13)."""
    from oracle import rw as orw
    t0 = time.time()
    ref = orw.solve_box(g, m, x, BETA, EPS, method="pcg", tol=1e-13).ravel()
    return ref, time.time() - t0


def bench_plain_sphere(torch, rwg, dev, cpu_leg):
    """64^3 sphere, one domain: FP64 to relative residual 1e-6 (the stated
    configuration) beside the mixed and mixed+refine paths."""
    import numpy as np
    import synth
    g, m, x0, inside = synth.plain_sphere()
    d = synth.from_boxes([(g, m, x0)])
    gd, md = torch.from_numpy(d["g"]).to(dev), torch.from_numpy(d["mask"]).to(dev)
    xd0 = torch.from_numpy(d["x"]).to(dev)
    x64 = torch.zeros(xd0.numel(), dtype=torch.float64, device=dev)
    ref, ref_s = oracle_plain_solve(g, m, x0) if cpu_leg else (None, None)
    runs = {"fp64_tol1e-6": dict(precision=0, tol=1e-6),
            "mixed_tol1e-6": dict(precision=1, tol=1e-6),
            "mixed_refine_tol1e-6": dict(precision=2, tol=1e-6, refine_max=4, refine_tol=1e-12)}
    out = {"workload": "plain sphere 64^3 float32 (radius 20, 0.7 on 0.3, noise 0.05), fg 5^3 centre block, "
                       "bg all faces, beta 128, eps 1e-6, one domain",
           "unknowns": int((m == 0).sum())}
    for name, kw in runs.items():
        xd = xd0.clone()

        def step():
            xd.copy_(xd0)
            return rwg.solve_bricks(gd, md, xd, d["shapes"], d["offsets"], x64=x64 if kw["precision"] != 1 else None,
                                    beta=BETA, eps=EPS, **kw)
        ms, st = _best_ms(torch, step, 3)
        s = rwg.stats_to_numpy(st)[0]
        sol = (x64.cpu().numpy() if kw["precision"] != 1 else xd.cpu().numpy().astype(np.float64))
        r = {"ms": ms, "iters": int(s["iters"]), "refine_iters": int(s["refine_iters"]),
             "status": rwg.STATUS_NAMES[int(s["status"])], "true_rel_resid": float(s["true_rel_resid"]),
             "voxel_iters_per_s": float(g.size * (int(s["iters"]) + int(s["refine_iters"])) / (ms / 1e3)),
             "dice_vs_sphere": float(2 * ((sol.reshape(g.shape) > 0.5) & inside).sum()
                                     / ((sol > 0.5).sum() + inside.sum()))}
        if ref is not None:
            r["max_abs_err_vs_oracle"] = float(np.max(np.abs(sol - ref)))
        out[name] = r
    if ref is not None:
        out["oracle_exact_s"] = ref_s
        # cpu_baseline leg: the oracle at the configuration's own tolerance (FP64, 1e-6)
        from oracle import rw as orw
        t0 = time.time()
        A, b_, U, M = orw.dirichlet_system(g, m, x0, BETA, EPS)
        _, it, _ = orw.pcg(A, b_, tol=1e-6)
        el = time.time() - t0
        out["cpu_oracle_tol1e-6"] = {"s": el, "iters": int(it), "voxel_iters_per_s": g.size * it / el,
                                     "cores": 1}
    return out


def bench_tubes(torch, rwg, ctx, n=512, n_tubes=40, levels=4):
    """Hierarchical pipeline on the random-tube volume (uint16, 4 levels,
    32^3 bricks expanded to 40^3, dt pruning at t_bin 0.49, mixed, tol 1e-5)."""
    import numpy as np
    import synth
    t0 = time.time()
    v, seeds, tube = synth.tube_volume(n=n, n_tubes=n_tubes, n_fg=20, n_bg=200, seed=2)
    gen_s = time.time() - t0
    vd = torch.from_numpy(v).to("cuda:0")
    kw = dict(brick=32, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=2, prune_hom=0,
              prune_dt=1, t_bin=0.49)
    pyr_ms, pyr = _best_ms(torch, lambda: rwg.Pyramid(ctx, vd, levels), 3)
    seg_ms, res = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), 3)
    st = res.stats()
    _, lab = res.materialize(0, 1, prob=False, labels=True)
    lb = lab.cpu().numpy().astype(bool)
    gt = (tube > 0) & (tube <= 20)
    vi = int(sum(st["voxel_iters"]))
    # the level solves under the other CG schedules of the 40^3 window
    # boxes: one sweep and one reduction per iteration (3), two sweeps (1)
    sched = {}
    for sc in (1, 3):
        ms, r = _best_ms(torch, lambda: rwg.segment(pyr, seeds, schedule=sc, **kw), 2)
        sched[str(sc)] = {"segment_ms": ms, "voxel_iters": int(sum(r.stats()["voxel_iters"])),
                          "max_abs_diff_vs_schedule_0": max(float((r.level_map(l) - res.level_map(l)).abs().max().item())
                                                            for l in range(levels))}
    # schedule 0 with the 40^3 boxes on the streaming window march instead of
    # split over two workgroups
    ctx.set_split_boxes(False)
    try:
        ms, r = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), 2)
    finally:
        ctx.set_split_boxes(True)
    sched["0_boxes_streaming"] = {
        "segment_ms": ms, "voxel_iters": int(sum(r.stats()["voxel_iters"])),
        "max_abs_diff_vs_schedule_0": max(float((r.level_map(l) - res.level_map(l)).abs().max().item())
                                          for l in range(levels))}
    return {"workload": f"tubes {n}^3 uint16, {n_tubes} tubes, 20 fg + 200 bg seeds, {levels} levels, s=32, e=1.25, "
                        "beta 128, dt pruning t_bin 0.49, mixed tol 1e-5",
            "pyramid_ms": pyr_ms, "segment_ms": seg_ms,
            "end_to_end_voxels_per_s": float(v.size / (seg_ms / 1e3)),
            "voxel_iters": vi, "voxel_iters_per_s": float(vi / (seg_ms / 1e3)),
            "per_level": {k: st[k] for k in ("bricks", "computed", "solved", "prunable", "voxel_iters", "max_iters",
                                             "not_converged")},
            "dice_vs_seeded_tubes": float(2 * (lb & gt).sum() / (lb.sum() + gt.sum())),
            "level_solve_schedules": sched, "generate_s": gen_s}


def bench_tubes_host(torch, rwg, ctx, n=512, n_tubes=40, levels=4):
    """The tube pipeline out of core: the volume in pinned host memory, the
    finest level's pyramid data and level map in page-locked host memory
    (rw_pyramid_build_host, rw_params.host_levels = 1), read and written in
    place by the kernels; against the same pipeline in device memory.  The
    level maps must agree bit for bit."""
    import synth
    v, seeds, _ = synth.tube_volume(n=n, n_tubes=n_tubes, n_fg=20, n_bg=200, seed=2)
    vh = torch.from_numpy(v).pin_memory()
    vd = vh.to("cuda:0")
    kw = dict(brick=32, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=2, prune_hom=0,
              prune_dt=1, t_bin=0.49)
    pd_ms, pyr_d = _best_ms(torch, lambda: rwg.Pyramid(ctx, vd, levels), 3)
    sd_ms, res_d = _best_ms(torch, lambda: rwg.segment(pyr_d, seeds, **kw), 3)
    ph_ms, pyr_h = _best_ms(torch, lambda: rwg.Pyramid(ctx, vh, levels, host_levels=1), 3)
    sh_ms, res_h = _best_ms(torch, lambda: rwg.segment(pyr_h, seeds, host_levels=1, **kw), 3)
    equal = all(bool(torch.equal(res_h.level_map(l), res_d.level_map(l))) for l in range(levels))
    host_bytes = v.size * 4 * 2      # level 0: g and the one-rhs map
    return {"workload": f"tubes {n}^3 uint16 in pinned host memory, level 0 (g and map) in page-locked host "
                        f"memory, {levels} levels, s=32, e=1.25, dt pruning, mixed tol 1e-5",
            "device": {"pyramid_ms": pd_ms, "segment_ms": sd_ms},
            "host_level0": {"pyramid_ms": ph_ms, "segment_ms": sh_ms, "host_bytes": host_bytes},
            "level_maps_equal": equal, "solved": res_h.stats()["solved"]}


def bench_blobs_adjoint(torch, rwg, dev, n=512, cpu_leg=False):
    """Forward (mixed + FP64 refinement) and adjoint on 512 two-blob 32^3
    boxes, beta 64; loss = mean BCE over unseeded voxels."""
    import synth
    d = synth.blob_boxes(n=n, seed=4)
    g = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    x0 = torch.from_numpy(d["x"]).to(dev)
    y = torch.from_numpy(d["gt"]).to(dev).float()
    u = (m == 0).float()
    x = x0.clone()
    kw = dict(beta=64.0, eps=EPS, tol=1e-6)

    def fwd():
        x.copy_(x0)
        return rwg.solve_bricks(g, m, x, d["shapes"], d["offsets"], precision=1, **kw)
    f_ms, st = _best_ms(torch, fwd, 3)
    xc = x.clamp(1e-6, 1 - 1e-6)
    dl_dx = ((xc - y) / (xc * (1 - xc)) * u / u.sum()).contiguous()
    b_ms, (dl_dg, dl_db, sta) = _best_ms(
        torch, lambda: rwg.solve_bricks_adjoint(g, m, x, dl_dx, d["shapes"], d["offsets"], **kw), 3)
    s, sa = rwg.stats_to_numpy(st), rwg.stats_to_numpy(sta)
    vox = 32 ** 3
    cpu = None
    if cpu_leg:
        # cpu_baseline leg: oracle forward (PCG, tol 1e-6) and adjoint (sparse direct) on 2 boxes
        from oracle import adjoint as oadj
        from oracle import rw as orw
        yh = d["gt"]
        t0 = time.time()
        for i in range(2):
            gb, mb, xb = d["boxes"][i]
            o = int(d["offsets"][i])
            xo = orw.solve_box(gb, mb, xb, 64.0, EPS, method="pcg", tol=1e-6)
            _, grad = oadj.bce_loss(xo, yh[o:o + gb.size].reshape(gb.shape), mb)
            oadj.adjoint_gradients(gb, mb, xo, grad, 64.0, EPS)
        el = time.time() - t0
        cpu = {"s_per_box": el / 2, "extrapolated_s_for_all": el / 2 * n, "cores": 1,
               "sample": "2 boxes, one process; the total is extrapolated"}
    return {"workload": f"{n} two-blob boxes 32^3, beta 64, forward mixed tol 1e-6 + adjoint tol 1e-6",
            "cpu_oracle": cpu,
            "forward_ms": f_ms, "adjoint_ms": b_ms,
            "forward_voxel_iters_per_s": float(vox * (s["iters"] + s["refine_iters"]).sum() / (f_ms / 1e3)),
            "adjoint_voxel_iters_per_s": float(vox * sa["iters"].sum() / (b_ms / 1e3)),
            "dl_dbeta": float(dl_db.item()), "dl_dg_norm": float(dl_dg.norm().item())}


def bench_shells(torch, rwg, ctx, dims=(256, 256, 128), levels=3):
    """Four-class nested-shell volume (3 right-hand sides per box, hom
    pruning t_hom 0.3, mixed tol 1e-5), then a 2000-voxel class-2 stroke
    solved incrementally."""
    import numpy as np
    import synth
    t0 = time.time()
    v, labels, seeds, geo = synth.shell_volume(dims=dims, seed=5)
    stroke = synth.stroke(labels, geo, cls=2, length=2000, seed=6)
    gen_s = time.time() - t0
    vd = torch.from_numpy(v).to("cuda:0")
    kw = dict(brick=32, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=4, prune_hom=1,
              prune_dt=0, t_hom=0.3)
    pyr_ms, pyr = _best_ms(torch, lambda: rwg.Pyramid(ctx, vd, levels), 2)
    full_ms, res = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), 2)
    more = np.concatenate([seeds, stroke])
    inc_ms, rinc = _best_ms(torch, lambda: rwg.segment(pyr, more, prev=res, **kw), 2)
    st, si = res.stats(), rinc.stats()
    _, lab = rinc.materialize(0, 0, prob=False, labels=True)
    acc = float((lab.cpu().numpy() == labels).mean())
    # incremental rules against a full run with every seed: the dirty-brick
    # rule (above), the node rule of Section IV-E, each with and without the
    # warm start from the previous result
    _, rfull = _best_ms(torch, lambda: rwg.segment(pyr, more, **kw), 1)
    lab_full = rfull.materialize(0, 0, prob=False, labels=True)[1].cpu().numpy()
    maps_full = [rfull.level_map(l) for l in range(levels)]
    rules = {}
    for name, mode in (("dirty", 0), ("dirty_warm", rwg.INC_WARM), ("node", rwg.INC_NODE),
                       ("node_warm", rwg.INC_NODE | rwg.INC_WARM)):
        ms, r = (inc_ms, rinc) if mode == 0 else _best_ms(
            torch, lambda: rwg.segment(pyr, more, prev=res, incremental=mode, **kw), 2)
        sr = r.stats()
        lb = r.materialize(0, 0, prob=False, labels=True)[1].cpu().numpy()
        rules[name] = {"incremental_ms": ms, "solved": sr["solved"], "voxel_iters": int(sum(sr["voxel_iters"])),
                       "kept": [int(((r.flags(l) & rwg.F_KEPT) != 0).sum().item()) for l in range(levels)],
                       "max_abs_diff_vs_full_run": max(float((r.level_map(l) - maps_full[l]).abs().max().item())
                                                       for l in range(levels)),
                       "label_agreement_vs_full_run": float((lb == lab_full).mean()),
                       "label_accuracy_vs_truth": float((lb == labels).mean())}
    # the three classes solved together in each box (weights shared, streaming kernels)
    joint_ms, rj = _best_ms(torch, lambda: rwg.segment(pyr, seeds, joint_classes=1, **kw), 2)
    joint = {"full_ms": joint_ms, "voxel_iters": int(sum(rj.stats()["voxel_iters"])),
             "max_abs_diff_vs_per_class": max(float((rj.level_map(l) - res.level_map(l)).abs().max().item())
                                              for l in range(levels))}
    return {"workload": f"nested shells {dims[0]}x{dims[1]}x{dims[2]} uint16, 4 classes (3 rhs), {levels} levels, "
                        "s=32, e=1.25, hom pruning t_hom 0.3, mixed tol 1e-5; then a 2000-voxel stroke (class 2)",
            "pyramid_ms": pyr_ms, "full_ms": full_ms, "incremental_ms": inc_ms, "joint_classes": joint,
            "full_voxel_iters_per_s": float(sum(st["voxel_iters"]) / (full_ms / 1e3)),
            "full_solved": st["solved"], "incremental_solved": si["solved"], "bricks": st["bricks"],
            "label_accuracy_vs_truth": acc, "incremental_rules": rules, "generate_s": gen_s}


def _replay_worker(args):
    """cpu_baseline leg: one level-0 box of the full-size shell run rebuilt
    by the oracle from the GPU's level-1 map and solved exactly."""
    from threadpoolctl import threadpool_limits
    from oracle import hierarchy as H
    vol_box, vrange, lab_box, border, up_box, p, rel = args
    with threadpool_limits(1):
        g_box = H.normalize(vol_box, vrange=vrange)
        xb = H._solve(g_box, lab_box, border, up_box, p)
    return xb[(slice(None),) + rel]


def bench_shells_full(torch, rwg, ctx, dims=(2048, 2048, 1024), levels=5, n_replay=256, cpu_leg=True):
    """The large multi-class incremental configuration at full size:
    2048 x 2048 x 1024 uint16 (8 GiB), four classes (background and three
    nested ellipsoidal shells, sigma 250 noise plus 1/f noise), 5 levels,
    s = 32, e = 1.25, three right-hand sides per box, hom pruning t_hom 0.3,
    mixed tol 1e-5; then a 2000-voxel class-2 stroke solved incrementally
    under the dirty-brick rule and the node rule.  The volume is generated
    on the device (``synth.shell_volume_device``).  cpu_baseline leg: sampled
    solved level-0 boxes of the full run rebuilt by the oracle from the
    GPU's level-1 map and solved exactly (max error of the GPU cores)."""
    import numpy as np
    import synth
    from oracle import hierarchy as H
    t0 = time.time()
    vol, labels, seeds, geo = synth.shell_volume_device(dims, seed=5, n_per_class=50)
    stroke = synth.stroke_geo(geo, cls=2, length=2000, seed=6)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    kw = dict(brick=32, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=4, prune_hom=1,
              prune_dt=0, t_hom=0.3)
    pyr_ms, pyr = _best_ms(torch, lambda: rwg.Pyramid(ctx, vol, levels), 1)
    print("bench.py: shells_full pyramid built", file=sys.stderr, flush=True)
    full_ms, res = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), 1)
    print("bench.py: shells_full full run done", file=sys.stderr, flush=True)
    more = np.concatenate([seeds, stroke])
    inc = {}
    for name, mode in (("dirty", 0), ("node", rwg.INC_NODE)):
        ms, r = _best_ms(torch, lambda: rwg.segment(pyr, more, prev=res, incremental=mode, **kw), 1)
        sr = r.stats()
        inc[name] = {"ms": ms, "solved": sr["solved"], "voxel_iters": int(sum(sr["voxel_iters"])),
                     "kept": [int(((r.flags(l) & rwg.F_KEPT) != 0).sum().item()) for l in range(levels)]}
        del r
        print(f"bench.py: shells_full incremental ({name}) done", file=sys.stderr, flush=True)
    # the three classes solved together in each box (weights shared, streaming kernels)
    jt_ms, rj = _best_ms(torch, lambda: rwg.segment(pyr, seeds, joint_classes=1, **kw), 1)

    # (levels 1.. only: a copy of level 0 is 51.5 GB; the 256x256x128 twin compares every level)
    joint = {"full_ms": jt_ms, "voxel_iters": int(sum(rj.stats()["voxel_iters"])),
             "max_abs_diff_vs_per_class_levels_1_up": max(
                 float((rj.level_map(l) - res.level_map(l)).abs().max().item()) for l in range(1, levels))}
    del rj
    print("bench.py: shells_full joint classes done", file=sys.stderr, flush=True)
    st = res.stats()
    lab = res.materialize(0, 0, prob=False, labels=True)[1]
    acc = float((lab == labels).float().mean().item())
    del lab
    out = {"workload": f"nested shells {dims[0]}x{dims[1]}x{dims[2]} uint16 (generated on the device), 4 classes "
                       f"(3 rhs), {levels} levels, s=32, e=1.25, hom pruning t_hom 0.3, mixed tol 1e-5; then a "
                       "2000-voxel class-2 stroke solved incrementally",
           "generate_s": gen_s, "pyramid_ms": pyr_ms, "full_ms": full_ms,
           "full_voxel_iters_per_s": float(sum(st["voxel_iters"]) / (full_ms / 1e3)),
           "end_to_end_voxels_per_s": float(np.prod(dims) / (full_ms / 1e3)),
           "bricks": st["bricks"], "full_computed": st["computed"], "full_solved": st["solved"],
           "full_not_converged": st["not_converged"], "full_max_iters": st["max_iters"],
           "label_accuracy_vs_truth": acc, "incremental": inc, "joint_classes": joint}
    if cpu_leg:
        # sampled solved level-0 boxes of the full run, replayed by the oracle
        import multiprocessing as mp
        p = H.Params(levels=levels, brick=32, expand=1.25, beta=BETA, eps=EPS, n_classes=4, method="pcg",
                     tol=1e-12)
        f0 = res.flags(0).cpu().numpy()
        solved = np.argwhere((f0 & rwg.F_SOLVED) != 0)
        rng = np.random.default_rng(0)
        picks = solved[rng.choice(len(solved), min(n_replay, len(solved)), replace=False)]
        v16 = vol.view(torch.int16)
        # the uint16 range of the whole volume (stored as int16 bits)
        vr = (int(min((v16[z:z + 64].to(torch.int32) & 0xFFFF).min().item() for z in range(0, dims[2], 64))),
              int(max((v16[z:z + 64].to(torch.int32) & 0xFFFF).max().item() for z in range(0, dims[2], 64))))
        m1 = res.level_map(1)
        m0 = res.level_map(0)
        d0 = (dims[2], dims[1], dims[0])
        d1 = tuple(m1.shape[:3])
        jobs, cores = [], []
        for b in map(tuple, picks):
            core, box = H.brick_box(b, d0, 32, 1.25)
            lo1 = tuple(max((lo - 1) // 2, 0) for lo, _ in box)
            hi1 = tuple(min(hi // 2 + 1, n) for (_, hi), n in zip(box, d1))
            crop = m1[lo1[0]:hi1[0], lo1[1]:hi1[1], lo1[2]:hi1[2]].permute(3, 0, 1, 2).cpu().numpy()
            up_box = H.upsample_box(crop, d0, box, origin=lo1, parent_shape=d1)
            vb = v16[box[0][0]:box[0][1], box[1][0]:box[1][1], box[2][0]:box[2][1]].cpu().numpy().view(np.uint16)
            lab_box = H.rasterize_box(seeds, 0, d0, box)
            rel = tuple(slice(c0 - b0, c1 - b0) for (c0, c1), (b0, _) in zip(core, box))
            jobs.append((vb, vr, lab_box, H.border_layer(box, d0), up_box, p, rel))
            cores.append(m0[core[0][0]:core[0][1], core[1][0]:core[1][1], core[2][0]:core[2][1]]
                         .permute(3, 0, 1, 2).cpu().numpy())
        del m0, m1
        t1 = time.time()
        workers = min(os.cpu_count() or 1, 16)
        with mp.get_context("fork").Pool(workers) as pool:
            refs = pool.map(_replay_worker, jobs, chunksize=1)
        errs = [float(np.max(np.abs(c - r))) for c, r in zip(cores, refs)]
        out["oracle_replay"] = {"bricks": len(errs), "max_abs_err": max(errs), "median_abs_err": float(np.median(errs)),
                                "cpu_s": time.time() - t1, "cores": workers,
                                "note": "level-0 boxes of the full run: oracle set-up from the GPU's level-1 map, "
                                        "FP64 PCG to 1e-12 per class; error of the GPU cores over the three classes"}
    return out


def bench_cells_ablation(torch, rwg, ctx, n=256, levels=4):
    """Ablations on the cells scenario (spheres covering 1 % of the volume,
    0.7 on 0.3 plus noise 0.1): brick size s in {16, 32, 64} (boxes 20^3,
    40^3, 80^3) with hom and dt pruning, and s = 32 with pruning off; time,
    bricks reached and solved per level, and Dice against the truth."""
    import numpy as np
    import synth
    t0 = time.time()
    v, seeds, truth = synth.cells_volume(n=n, seed=11)
    gen_s = time.time() - t0
    vd = torch.from_numpy(v).to("cuda:0")
    pyr = rwg.Pyramid(ctx, vd, levels)
    gt = truth.astype(bool)
    out = {"workload": f"cells {n}^3 float32, {int((seeds[:, 3] == 1).sum())} spheres (diameter 0.05-0.1 n, 1 % "
                       f"of the volume), 0.7 on 0.3, noise 0.1, {levels} levels, e=1.25, beta 128, t_hom 0.3, "
                       "t_bin 0.01, mixed tol 1e-5", "generate_s": gen_s}
    runs = [("s16_pruned", 16, 1), ("s32_pruned", 32, 1), ("s64_pruned", 64, 1), ("s32_unpruned", 32, 0)]
    for name, s, prune in runs:
        kw = dict(brick=s, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=2, prune_hom=prune,
                  prune_dt=prune, t_hom=0.3, t_bin=0.01)
        ms, res = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), 2)
        st = res.stats()
        _, lab = res.materialize(0, 1, prob=False, labels=True)
        lb = lab.cpu().numpy().astype(bool)
        out[name] = {"segment_ms": ms, "voxel_iters": int(sum(st["voxel_iters"])),
                     "per_level": {k: st[k] for k in ("bricks", "computed", "solved", "prunable")},
                     "dice_vs_truth": float(2 * (lb & gt).sum() / (lb.sum() + gt.sum()))}
    # incremental (Section IV-E): a first run misses one cell's seed, the
    # second adds it; the dirty-brick rule and the node rule, with and without
    # the warm start from the previous result, against the full s = 16 run
    kw = dict(brick=16, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=2, prune_hom=1,
              prune_dt=1, t_hom=0.3, t_bin=0.01)
    first = np.delete(seeds, np.flatnonzero(seeds[:, 3] == 1)[0], axis=0)
    _, r0 = _best_ms(torch, lambda: rwg.segment(pyr, first, **kw), 1)
    _, rfull = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), 1)
    lab_full = rfull.materialize(0, 1, prob=False, labels=True)[1].cpu().numpy()
    inc = {"brick": 16, "full_run_ms": out["s16_pruned"]["segment_ms"], "full_run_solved": rfull.stats()["solved"]}
    for name, mode in (("dirty", 0), ("dirty_warm", rwg.INC_WARM), ("node", rwg.INC_NODE),
                       ("node_warm", rwg.INC_NODE | rwg.INC_WARM)):
        ms, r = _best_ms(torch, lambda: rwg.segment(pyr, seeds, prev=r0, incremental=mode, **kw), 2)
        st = r.stats()
        lb = r.materialize(0, 1, prob=False, labels=True)[1].cpu().numpy()
        inc[name] = {"incremental_ms": ms, "solved": st["solved"], "voxel_iters": int(sum(st["voxel_iters"])),
                     "kept": [int(((r.flags(l) & rwg.F_KEPT) != 0).sum().item()) for l in range(levels)],
                     "label_agreement_vs_full_run": float((lb == lab_full).mean()),
                     "dice_vs_truth": float(2 * (lb.astype(bool) & gt).sum() / (lb.astype(bool).sum() + gt.sum()))}
    out["incremental_add_one_cell_seed"] = inc
    return out


def bench_pruning_table(torch, rwg, ctx, n=256, levels=4, reps=2):
    """The pruning ablation of Table IV on both synthetic scenarios (cells
    and vessels, structure size 0.1, 1 % foreground, 0.3 / 0.7 plus noise
    0.1): no pruning, hom only, dt only and both, each with the full run
    time, Dice against the truth, bricks solved, and the incremental run time
    of adding back one foreground label that a first run left out (Section
    V-B, the simulated editing step).  s = 32, e = 1.25, t_hom 0.3, t_bin
    0.01, mixed tol 1e-5.  The paper's table is over 1000^3 volumes; these
    are n^3."""
    import numpy as np
    import synth
    out = {"workload": f"cells and vessels {n}^3 float32, structure size 0.1, 1 % foreground, noise 0.1, {levels} "
                       "levels, s=32, e=1.25, beta 128, t_hom 0.3, t_bin 0.01, mixed tol 1e-5"}
    for scen, gen in (("cells", lambda: synth.cells_volume(n=n, seed=11)),
                      ("vessels", lambda: synth.vessels_volume(n=n, seed=12))):
        v, seeds, truth = gen()
        gt = truth.astype(bool)
        pyr = rwg.Pyramid(ctx, torch.from_numpy(v).to("cuda:0"), levels)
        rng = np.random.default_rng(5)
        drop = int(rng.choice(np.flatnonzero(seeds[:, 3] == 1)))
        first = np.delete(seeds, drop, axis=0)
        rows = {}
        for name, hom, dt in (("none", 0, 0), ("hom", 1, 0), ("dt", 0, 1), ("both", 1, 1)):
            kw = dict(brick=32, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=2, prune_hom=hom,
                      prune_dt=dt, t_hom=0.3, t_bin=0.01)
            ms, res = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), reps)
            st = res.stats()
            lb = res.materialize(0, 1, prob=False, labels=True)[1].cpu().numpy().astype(bool)
            _, r0 = _best_ms(torch, lambda: rwg.segment(pyr, first, **kw), 1)
            inc_ms, rinc = _best_ms(torch, lambda: rwg.segment(pyr, seeds, prev=r0, **kw), reps)
            rows[name] = {"full_ms": ms, "incremental_ms": inc_ms,
                          "dice_vs_truth": float(2 * (lb & gt).sum() / max(1, lb.sum() + gt.sum())),
                          "solved": st["solved"], "incremental_solved": rinc.stats()["solved"],
                          "voxel_iters": int(sum(st["voxel_iters"]))}
        out[scen] = {"labels": int(len(seeds)), "foreground_fraction": float(gt.mean()), "runs": rows}
    return out


def bench_cells_growth(torch, rwg, ctx, sizes=(64, 128, 256, 512)):
    """Active-brick growth (Section IV-D1): the same cells geometry scaled to
    n^3 voxels (structure and coverage relative to n, so the spheres' surface
    grows as n^2 = v^(2/3)), s = 16 with hom and dt pruning, levels chosen so
    that the coarsest level is 32^3.  Per size: level-0 bricks in all and
    reached, bricks solved, time; and the growth exponent of the reached
    level-0 bricks in v between successive sizes (2/3 for a surface)."""
    import numpy as np
    import synth
    rows = []
    for n in sizes:
        v, seeds, truth = synth.cells_volume(n=n, seed=11)
        levels = int(round(np.log2(n / 32))) + 1
        vd = torch.from_numpy(v).to("cuda:0")
        pyr = rwg.Pyramid(ctx, vd, levels)
        kw = dict(brick=16, expand=1.25, beta=BETA, eps=EPS, tol=1e-5, precision=1, n_classes=2, prune_hom=1,
                  prune_dt=1, t_hom=0.3, t_bin=0.01)
        ms, res = _best_ms(torch, lambda: rwg.segment(pyr, seeds, **kw), 2)
        st = res.stats()
        lb = res.materialize(0, 1, prob=False, labels=True)[1].cpu().numpy().astype(bool)
        gt = truth.astype(bool)
        rows.append({"n": n, "voxels": n ** 3, "levels": levels, "spheres": int((seeds[:, 3] == 1).sum()),
                     "level0_bricks": st["bricks"][0], "level0_reached": st["computed"][0],
                     "solved": st["solved"], "segment_ms": ms, "voxel_iters": int(sum(st["voxel_iters"])),
                     "dice_vs_truth": float(2 * (lb & gt).sum() / (lb.sum() + gt.sum()))})
        del vd, pyr, res
    for a, b in zip(rows, rows[1:]):
        dv = np.log(b["voxels"] / a["voxels"])
        b["reached_exponent_in_v"] = float(np.log(b["level0_reached"] / a["level0_reached"]) / dv)
        b["time_exponent_in_v"] = float(np.log(b["segment_ms"] / a["segment_ms"]) / dv)
    return {"workload": "cells geometry scaled to n^3, n in " + ", ".join(str(n) for n in sizes) +
                        "; s=16, e=1.25, hom and dt pruning, coarsest level 32^3, mixed tol 1e-5", "runs": rows}


def bench_streamed(torch, rwg, ctx, steps=3):
    """The 8192 stress boxes held in page-locked host memory and streamed
    through the GPU (rw_solve_bricks_streamed, default 2^24-voxel chunks, two lanes), against
    the same solve with the boxes resident in HBM.  The PCIe-inclusive rate."""
    import numpy as np
    import synth
    d = synth.stress_boxes(n=N_BOXES, seed=SEED)
    sizes = d["shapes"].prod(axis=1).astype(np.int64)
    gh, mh = torch.from_numpy(d["g"]).pin_memory(), torch.from_numpy(d["mask"]).pin_memory()
    x0 = torch.from_numpy(d["x"])
    xh = x0.clone().pin_memory()
    bricks = rwg.bricks_array(d["shapes"], d["offsets"])
    p = rwg.solve_params(beta=BETA, eps=EPS, tol=TOL, precision=rwg.PREC_MIXED, refine_max=1, inner_tol=1e-4)
    st = torch.empty((N_BOXES, 32), dtype=torch.uint8).pin_memory()
    s = torch.cuda.current_stream()

    def call():
        xh.copy_(x0)
        ctx.rw_solve_bricks_streamed(p, bricks, gh, mh, xh, stats=st, stream=s)
        s.synchronize()
    call()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    ms = (time.perf_counter() - t0) / steps * 1e3
    # the same boxes resident in HBM (x reset on the device inside the step)
    g, m, xd0 = gh.cuda(), mh.cuda(), x0.cuda()
    xd = xd0.clone()
    std = torch.empty((N_BOXES, 32), dtype=torch.uint8, device="cuda")

    def call_dev():
        xd.copy_(xd0)
        ctx.rw_solve_bricks(p, bricks, g, m, xd, stats=std, stream=s)
        s.synchronize()
    call_dev()
    t0 = time.perf_counter()
    for _ in range(steps):
        call_dev()
    ms_dev = (time.perf_counter() - t0) / steps * 1e3
    stn = rwg.stats_to_numpy(st)
    vox_it = int(np.sum(sizes * (stn["iters"].astype(np.int64) + stn["refine_iters"].astype(np.int64))))
    moved = int(sizes.sum()) * (4 + 1 + 4 + 4)   # g, mask, x in; x out
    return {"workload": "stress boxes (8192, 113.5M voxels) in page-locked host memory, 2^24-voxel chunks, two lanes, "
                        "mixed precision, tol 1e-6",
            "streamed_ms_per_call": ms, "device_resident_ms_per_call": ms_dev,
            "streamed_voxel_iters_per_s": vox_it / (ms / 1e3),
            "pcie_bytes_per_call": moved, "pcie_GBps_implied": moved / (ms / 1e3) / 1e9,
            "x_equal_to_device_resident": bool(torch.equal(xh, xd.cpu()))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--schedule", type=int, default=-1, help="CG schedule (rw_solve_params.schedule): -1 autotune the batch (rw_autotune) and run the tuned schedule (default), 0 library choice, 1 two-sweep streaming, 2 one-sweep streaming, 3 as 0 with 2, 4 streamed-weights resident wherever it fits")
    ap.add_argument("--no-extras", action="store_true", help="skip the further workloads (sphere, tubes, blobs, shells, cells)")
    ap.add_argument("--shells-dims", default="256,256,128", help="nested-shell volume dims nx,ny,nz")
    ap.add_argument("--only", choices=EXTRAS + ON_REQUEST, default=None,
                    help="run one further workload alone and print its JSON (for profiling; no headline line)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (boxes are independent; multi-GPU sharding "
              "is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2103_09564_amd as rwg

    dev = torch.device("cuda:0")
    shell_dims = tuple(int(t) for t in args.shells_dims.split(","))

    def extra(name, ctx):
        if name == "plain_sphere_64":
            return bench_plain_sphere(torch, rwg, dev, not args.no_cpu_baseline)
        if name == "tubes_512_hierarchy":
            return bench_tubes(torch, rwg, ctx)
        if name == "blobs_512x32_adjoint":
            return bench_blobs_adjoint(torch, rwg, dev, cpu_leg=not args.no_cpu_baseline)
        if name == "cells_256_ablation":
            return bench_cells_ablation(torch, rwg, ctx)
        if name == "cells_brick_growth":
            return bench_cells_growth(torch, rwg, ctx)
        if name == "pruning_table_256":
            return bench_pruning_table(torch, rwg, ctx)
        if name == "shells_full":
            return bench_shells_full(torch, rwg, ctx, cpu_leg=not args.no_cpu_baseline)
        if name == "memory_ceilings":
            return {"ceilings": measure_ceilings(torch, rwg, ctx), "read_sweep": probe_read_sweep(torch, rwg, ctx)}
        if name == "stress_streamed_from_host":
            return bench_streamed(torch, rwg, ctx)
        if name == "tubes_512_host_finest":
            return bench_tubes_host(torch, rwg, ctx)
        return bench_shells(torch, rwg, ctx, dims=shell_dims)

    if args.only:
        print(json.dumps({args.only: extra(args.only, rwg.Context(0))}), flush=True)
        return
    d = synth.stress_boxes(n=N_BOXES, seed=SEED)
    shapes, offsets = d["shapes"], d["offsets"]
    sizes = shapes.prod(axis=1).astype(np.int64)
    g = torch.from_numpy(d["g"]).to(dev)
    m = torch.from_numpy(d["mask"]).to(dev)
    x0 = torch.from_numpy(d["x"]).to(dev)
    x = x0.clone()
    ctx = rwg.Context(0)
    bricks = rwg.bricks_array(shapes, offsets)
    st = torch.empty((N_BOXES, 32), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    # the library's autotuner times its candidate schedules on this batch
    # (outside the timed region) and the timed steps run its winner
    tune = None
    sched = args.schedule
    if sched < 0:
        xw = torch.empty_like(x0)
        tune = {}
        for prec, name in ((rwg.PREC_MIXED, "mixed"), (rwg.PREC_FP64, "fp64")):
            if prec == rwg.PREC_FP64 and args.no_fp64:
                continue
            pt = rwg.solve_params(beta=BETA, eps=EPS, tol=TOL, precision=prec, refine_max=1, inner_tol=1e-4)
            tune[name] = ctx.autotune(pt, bricks, g, m, x0, xw, reps=2, stream=stream)
        del xw
        sched = rwg.SCHED_TUNED

    def run(prec, steps, warmup):
        p = rwg.solve_params(beta=BETA, eps=EPS, tol=TOL, precision=prec, refine_max=1, inner_tol=1e-4,
                             schedule=sched)
        for _ in range(warmup):
            x.copy_(x0)
            ctx.rw_solve_bricks(p, bricks, g, m, x, stats=st, stream=stream)
        torch.cuda.synchronize()
        # wall clock over the K timed steps; the PCG kernel's own duration comes
        # from the library's HIP events, recorded on the launch stream
        ctx.set_timing(True)
        tims = []
        t0 = time.perf_counter()
        for _ in range(steps):
            x.copy_(x0)
            ctx.rw_solve_bricks(p, bricks, g, m, x, stats=st, stream=stream)
            tims.append(ctx.last_timing())
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        ctx.set_timing(False)
        mean = {k: float(np.mean([t[k] for t in tims])) / 1e3 for k in tims[0]}
        s = rwg.stats_to_numpy(st)
        iters = s["iters"].astype(np.int64) + s["refine_iters"].astype(np.int64)
        vox_it = int(np.sum(sizes * iters))
        main = sizes * s["iters"].astype(np.int64)
        path = ctx.solve_plan(p, bricks, g.numel())
        # eager launches queued back to back against a captured graph of
        # the same solve (the x reset stays outside the graph)
        gs = torch.cuda.Stream()
        xg = x0.clone()
        with torch.cuda.stream(gs):
            graph = rwg.Graph(ctx, p, bricks, g, m, xg, stream=gs)
            for _ in range(warmup):
                xg.copy_(x0)
                graph.launch(stream=gs)
        gs.synchronize()
        tg0 = time.perf_counter()
        with torch.cuda.stream(gs):
            for _ in range(steps):
                xg.copy_(x0)
                graph.launch(stream=gs)
        gs.synchronize()
        graph_wall = (time.perf_counter() - tg0) / steps
        graph_same = bool(torch.equal(xg, x))
        graph.close()
        hbm = (path == rwg.PATH_STREAM) | (path == rwg.PATH_STREAM_GLOBAL)
        sw = path == rwg.PATH_RESIDENT_STREAMED
        lds = path == rwg.PATH_RESIDENT
        # the library runs two kernel groups concurrently: HBM-streaming and
        # streamed-weights boxes on one stream (stream_ms), LDS-resident boxes
        # on the other (resident_ms)
        return dict(wall=wall, kern=mean["pcg_ms"], t=mean, vox_it=vox_it, vox_it_main=int(main.sum()),
                    graph_wall=graph_wall, graph_same=graph_same, schedule=ctx.tuned_schedule(p, bricks),
                    res_vox=int(sizes[lds].sum()),
                    vox_it_a=int(main[hbm | sw].sum()), vox_it_sw=int(main[sw].sum()), vox_it_hbm=int(main[hbm].sum()),
                    vox_it_sw1=int(main[sw & (sizes > 17408)].sum()), vox_it_sw2=int(main[sw & (sizes <= 17408)].sum()),
                    vox_it_res=int(main[lds].sum()), n_hbm=int(hbm.sum()), n_sw=int(sw.sum()), n_res=int(lds.sum()),
                    stats=s, x=x.cpu().numpy())

    mixed = run(rwg.PREC_MIXED, args.steps, args.warmup)
    fp64 = None if args.no_fp64 else run(rwg.PREC_FP64, max(1, args.steps // 2), 1)

    value = mixed["vox_it"] / mixed["wall"]
    # Dominant kernel: the streamed-weights resident PCG (k_pcg_resg4, four
    # voxels per 16-byte load on 32 x 32 planes; the 32^3 and the 32x32x17
    # boxes form two launches), timed by the library's HIP
    # events on the stream it runs on.  When the two launches run concurrently
    # on streams of their own (stream2_ms > 0) the roofline is that of the
    # 32^3 launch alone; otherwise of the two together (one after the other on
    # one stream, with any HBM-streaming boxes).  Its algorithmic bytes: the
    # kernel keeps x, r and p on chip and must re-read, every iteration, the
    # 16 B per voxel of precomputed weights and 1/d (w+x, w+y, w+z, 1/d) that
    # its design streams from the cache hierarchy (segments of the boxes in
    # flight stay in the last-level cache, the rest comes from HBM).  The
    # 28 B streaming formulation is reported beside it as an equivalent only.
    t = mixed["t"]
    split = t.get("stream2_ms", 0.0) > 0
    vox_roof = mixed["vox_it_sw1"] if split else mixed["vox_it_a"]
    achieved = SEGMENT_BYTES_PER_VOXEL_ITER * vox_roof / t["stream_ms"] / 1e9 if t["stream_ms"] > 0 else 0.0
    stream_equiv = BYTES_PER_VOXEL_ITER * vox_roof / t["stream_ms"] / 1e9 if t["stream_ms"] > 0 else 0.0
    ceilings = measure_ceilings(torch, rwg, ctx)
    alone = roofline_alone(torch, rwg, ctx, d, g, m, x, x0, stream)
    # memory bytes of the whole PCG phase, each box at its kernel's own
    # algorithmic bytes (a cross-check that must stay below the HBM peak)
    n_res_vox = mixed["res_vox"]
    phase_bytes = (SEGMENT_BYTES_PER_VOXEL_ITER * mixed["vox_it_sw"] + BYTES_PER_VOXEL_ITER * mixed["vox_it_hbm"]
                   + RESIDENT_BYTES_PER_VOXEL * n_res_vox)
    traffic = traffic_from_profile(split)
    s = mixed["stats"]
    out = {
        "metric": "brick-PCG voxel-iters/s, %HBM peak; mixed vs plain FP64 at 1e-4 err",
        "value": value,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["wall"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "stress boxes: 8192 boxes, shapes U{32^3,32x32x17,32x9x32,5x32x32,16^3}, "
                               "beta 128, eps 1e-6, tol 1e-6, mixed FP32/FP64",
                   "n_boxes": N_BOXES, "voxels": int(sizes.sum()), "unknowns": int((d["mask"] == 0).sum()),
                   "tol": TOL, "precision": "mixed (FP32 vectors, FP64 reductions + FP64 true-residual check)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": ("k_pcg_resg4<512, 16> (streamed-weights resident PCG, the 32^3 boxes), main-solve "
                                "launch" if split else "k_pcg_resg4<512, 16> and <512, 9> (streamed-weights resident PCG, the 32^3 and "
                                "the 32x32x17 boxes one after the other on one stream), main-solve launches"),
                     "bytes_per_voxel_iter": SEGMENT_BYTES_PER_VOXEL_ITER,
                     "measured_ceilings": ceilings,
                     "alone": alone,
                     "frac_of_measured_hbm_read": achieved / ceilings["hbm_read_GBps"],
                     "frac_of_measured_llc_reread": achieved / ceilings["llc_reread_GBps"],
                     "streaming_equivalent": {"bytes_per_voxel_iter": BYTES_PER_VOXEL_ITER, "GBps": stream_equiv,
                                              "note": "what a kernel streaming x, r, p, g from HBM every iteration "
                                                      "would move at this rate; not this kernel's traffic"},
                     "note": "achieved = 16 B (the weights and 1/d the kernel re-reads every iteration) x its "
                             "voxel-iterations / its duration; the segments of the boxes in flight sit in the "
                             "last-level cache, so traffic (calibrated FETCH_SIZE + WRITE_SIZE per launch) is HBM "
                             "plus cache-hit bytes; the launch is bound by the cache loads it keeps in flight"},
        "solve": {"pcg_phase_ms": mixed["kern"] * 1e3, "voxel_iters": mixed["vox_it"],
                  "pcg_voxel_iters": mixed["vox_it_main"],
                  "pcg_phase_voxel_iters_per_s": mixed["vox_it_main"] / mixed["kern"],
                  "pcg_phase_memory_GBps": phase_bytes / mixed["kern"] / 1e9,
                  "pcg_phase_streaming_equivalent_GBps": BYTES_PER_VOXEL_ITER * mixed["vox_it_main"] / mixed["kern"] / 1e9,
                  "stream_group": {"boxes_streamed_weights": mixed["n_sw"], "boxes_hbm_streaming": mixed["n_hbm"],
                                   "voxel_iters": mixed["vox_it_a"], "ms": t["stream_ms"] * 1e3,
                                   "voxel_iters_per_s": (vox_roof / t["stream_ms"]) if t["stream_ms"] else None,
                                   "second_launch": ({"voxel_iters": mixed["vox_it_sw2"], "ms": t["stream2_ms"] * 1e3,
                                                      "voxel_iters_per_s": mixed["vox_it_sw2"] / t["stream2_ms"]}
                                                     if split else None),
                                   "note": ("ms times the 32^3 launch; the 32x32x17 launch runs beside it on a "
                                            "stream of its own (second_launch)" if split else
                                            "ms times all launches of the group, one after another")},
                  "lds_resident": {"boxes": mixed["n_res"], "voxel_iters": mixed["vox_it_res"],
                                   "ms": t["resident_ms"] * 1e3,
                                   "voxel_iters_per_s": mixed["vox_it_res"] / t["resident_ms"] if t["resident_ms"] else None,
                                   "note": "on-chip: p in LDS, the edge weights in registers (or LDS), x and r in "
                                           "registers; HBM is read once per solve, so no HBM roofline applies"},
                  "schedule": {"requested": "tuned" if args.schedule < 0 else args.schedule,
                               "ran": mixed["schedule"][0], "third_stream": mixed["schedule"][1],
                               "weights_in_registers": mixed["schedule"][2], "persistent": mixed["schedule"][3],
                               "autotune": tune},
                  "graph_replay": {"ms_per_step": mixed["graph_wall"] * 1e3,
                                   "x_equal_to_eager": mixed["graph_same"],
                                   "note": "the same solve captured once (rw_graph_create) and replayed K times"},
                  "mean_iters": float(s["iters"].mean()), "max_iters": int(s["iters"].max()),
                  "iters_by_shape": {f"{a}x{b}x{c}": {"boxes": int(sel.sum()), "mean_iters": float(s["iters"][sel].mean()),
                                                      "max_iters": int(s["iters"][sel].max())}
                                     for a, b, c in sorted({tuple(int(v) for v in r) for r in shapes})
                                     for sel in [(shapes[:, 0] == a) & (shapes[:, 1] == b) & (shapes[:, 2] == c)]},
                  "refined_boxes": int((s["refine_steps"] > 0).sum()),
                  "status_counts": {rwg.STATUS_NAMES[k]: int((s["status"] == k).sum()) for k in np.unique(s["status"])},
                  "max_true_rel_resid": float(s["true_rel_resid"].max()),
                  "bytes_note": "pcg_phase_memory_GBps: 16 B per voxel-iteration of streamed-weights boxes, 28 B of "
                                "HBM-streaming boxes, 13 B per voxel once for LDS-resident boxes, over the phase "
                                "time; pcg_phase_streaming_equivalent_GBps: 28 B for every voxel-iteration",
                  "source_hash": source_hash()},
    }
    if fp64 is not None:
        f = fp64["stats"]
        out["fp64_plain"] = {"value": fp64["vox_it"] / fp64["wall"], "ms_per_step": fp64["wall"] * 1e3,
                             "mean_iters": float(f["iters"].mean()),
                             "max_true_rel_resid": float(f["true_rel_resid"].max())}
        out["speedup_mixed_vs_fp64"] = fp64["wall"] / mixed["wall"]
    if not args.no_cpu_baseline:
        cb, sols = cpu_baseline(d["boxes"])
        out["cpu_baseline"] = cb
        err = {"mixed": 0.0}
        if fp64 is not None:
            err["fp64"] = 0.0
        for i, ref in sols.items():
            o, n = int(offsets[i]), int(sizes[i])
            err["mixed"] = max(err["mixed"], float(np.max(np.abs(mixed["x"][o:o + n] - ref))))
            if fp64 is not None:
                err["fp64"] = max(err["fp64"], float(np.max(np.abs(fp64["x"][o:o + n] - ref))))
        # against the exact solution (every 64th box): the "at 1e-4 error" of the metric
        idx = list(range(0, len(d["boxes"]), 64))
        exact = oracle_exact_sample(d["boxes"], idx)
        ex = {"mixed": 0.0}
        if fp64 is not None:
            ex["fp64"] = 0.0
        for i, ref in exact.items():
            o, n = int(offsets[i]), int(sizes[i])
            ex["mixed"] = max(ex["mixed"], float(np.max(np.abs(mixed["x"][o:o + n] - ref))))
            if fp64 is not None:
                ex["fp64"] = max(ex["fp64"], float(np.max(np.abs(fp64["x"][o:o + n] - ref))))
        out["max_abs_err_vs_exact"] = dict(ex, boxes=len(exact),
                                           note="oracle PCG to 1e-13 on every 64th box; both GPU paths at tol 1e-6")
        out["max_abs_diff_vs_oracle"] = dict(err, boxes=len(sols),
                                             note="oracle at the same tol 1e-6; both sides carry solver error")
    if not args.no_extras:
        extras = {}
        for name in EXTRAS:
            print(f"bench.py: {name}", file=sys.stderr, flush=True)
            try:
                extras[name] = extra(name, ctx)
            except Exception as e:  # a failing side workload must not hide the headline line
                extras[name] = {"error": f"{type(e).__name__}: {e}"}
        out["workloads"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
