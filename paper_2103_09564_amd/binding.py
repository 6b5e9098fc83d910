"""ctypes binding of librwseg (the C ABI in include/rwseg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Torch supplies device memory (``tensor.data_ptr()``) and the stream
(``torch.cuda.current_stream().cuda_stream``); no torch op runs on the data
inside these calls.  Importing this module fails loudly if librwseg.so has not
been built; there is no fallback implementation.
"""

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librwseg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as e; e.build()' "
        "or python -m paper_2103_09564_amd._build)")

lib = ctypes.CDLL(LIB_PATH)

RW_OK, RW_E_INVAL, RW_E_HIP, RW_E_NOMEM, RW_E_UNSUPPORTED = 0, -1, -2, -3, -4
PREC_FP64, PREC_MIXED, PREC_MIXED_REFINE = 0, 1, 2
ST_CONVERGED, ST_MAX_ITER, ST_REFINED, ST_STALLED, ST_NONFINITE, ST_NO_DIRICHLET = range(6)
STATUS_NAMES = ["CONVERGED", "MAX_ITER", "REFINED", "STALLED", "NONFINITE", "NO_DIRICHLET", "SYNC_LOST"]

BRICK_DTYPE = np.dtype([("nx", "<i4"), ("ny", "<i4"), ("nz", "<i4"), ("reserved", "<i4"), ("offset", "<i8")])
STATS_DTYPE = np.dtype([("iters", "<i4"), ("status", "<i4"), ("refine_steps", "<i4"), ("refine_iters", "<i4"),
                        ("rel_resid", "<f8"), ("true_rel_resid", "<f8")])
assert BRICK_DTYPE.itemsize == 24 and STATS_DTYPE.itemsize == 32


class SolveParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("eps", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32), ("nrhs", ctypes.c_int32),
                ("refine_max", ctypes.c_int32), ("refine_tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("stall_ratio", ctypes.c_double), ("schedule", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
lib.rw_version.restype = ctypes.c_int
lib.rw_solve_params_default.argtypes = [ctypes.POINTER(SolveParams)]
lib.rw_solve_params_default.restype = None
lib.rw_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(_vp)]
lib.rw_ctx_create.restype = ctypes.c_int
lib.rw_ctx_destroy.argtypes = [_vp]
lib.rw_ctx_destroy.restype = None
lib.rw_last_error.argtypes = [_vp]
lib.rw_last_error.restype = ctypes.c_char_p
lib.rw_solve_bricks.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]
lib.rw_solve_bricks.restype = ctypes.c_int
lib.rw_solve_bricks_noalloc.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp,
                                        _vp]
lib.rw_solve_bricks_noalloc.restype = ctypes.c_int
lib.rw_noalloc_scratch_bytes.argtypes = []
lib.rw_noalloc_scratch_bytes.restype = ctypes.c_size_t
lib.rw_solve_bricks_streamed.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp, _i64, _vp, _vp, _vp, _vp,
                                         _i64, _vp]
lib.rw_solve_bricks_streamed.restype = ctypes.c_int
lib.rw_solve_bricks_adjoint.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp, _i64, _vp, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _vp, _vp]
lib.rw_solve_bricks_adjoint.restype = ctypes.c_int
lib.rw_validate_solve.argtypes = [ctypes.POINTER(SolveParams), _i64, _vp, _i64]
lib.rw_validate_solve.restype = ctypes.c_int


class Timing(ctypes.Structure):
    _fields_ = [("init_ms", ctypes.c_float), ("pcg_ms", ctypes.c_float), ("finish_ms", ctypes.c_float),
                ("total_ms", ctypes.c_float), ("stream_ms", ctypes.c_float), ("resident_ms", ctypes.c_float),
                ("stream2_ms", ctypes.c_float)]


lib.rw_set_timing.argtypes = [_vp, ctypes.c_int]
lib.rw_set_timing.restype = ctypes.c_int
lib.rw_last_timing.argtypes = [_vp, ctypes.POINTER(Timing)]
lib.rw_last_timing.restype = ctypes.c_int
lib.rw_probe_blocks.argtypes = []
lib.rw_probe_blocks.restype = ctypes.c_int
lib.rw_probe_read.argtypes = [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int, _vp, _vp]
lib.rw_probe_read.restype = ctypes.c_int
lib.rw_probe_copy.argtypes = [_vp, _vp, _vp, _i64, _vp]
lib.rw_probe_copy.restype = ctypes.c_int
class TuneReport(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("best", ctypes.c_int32), ("schedule", ctypes.c_int32 * 8),
                ("third_stream", ctypes.c_int32 * 8), ("weights_in_registers", ctypes.c_int32 * 8),
                ("persistent", ctypes.c_int32 * 8), ("ms", ctypes.c_float * 8), ("key", ctypes.c_uint64),
                ("split_boxes", ctypes.c_int32 * 8)]


SCHED_TUNED = 5
lib.rw_autotune.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_int,
                            ctypes.POINTER(TuneReport), _vp]
lib.rw_autotune.restype = ctypes.c_int
lib.rw_set_plan_choices.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
lib.rw_set_plan_choices.restype = ctypes.c_int
lib.rw_set_split_boxes.argtypes = [_vp, ctypes.c_int]
lib.rw_set_split_boxes.restype = ctypes.c_int
lib.rw_tuned_schedule.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp] + [ctypes.POINTER(ctypes.c_int32)] * 5
lib.rw_tuned_schedule.restype = ctypes.c_int
lib.rw_graph_create.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                ctypes.POINTER(_vp)]
lib.rw_graph_create.restype = ctypes.c_int
lib.rw_graph_launch.argtypes = [_vp, _vp]
lib.rw_graph_launch.restype = ctypes.c_int
lib.rw_graph_free.argtypes = [_vp]
lib.rw_graph_free.restype = None
lib.rw_solve_plan.argtypes = [_vp, ctypes.POINTER(SolveParams), _i64, _vp, _i64, _vp]
lib.rw_solve_plan.restype = ctypes.c_int

PATH_STREAM, PATH_STREAM_GLOBAL, PATH_RESIDENT, PATH_DOMAIN, PATH_RESIDENT_STREAMED, PATH_RESIDENT_SPLIT = \
    0, 1, 2, 3, 4, 5


class RWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librwseg error {code}: {msg}")
        self.code = code


def version():
    return lib.rw_version()


def probe_blocks():
    """Workgroups of the memory probes (floats of their ``part`` output)."""
    return int(lib.rw_probe_blocks())


def noalloc_scratch_bytes():
    """Size of the fixed device scratch of rw_solve_bricks_noalloc."""
    return int(lib.rw_noalloc_scratch_bytes())


def validate_solve(params, bricks, n_voxels):
    """Host-only argument check (no GPU).  Returns (code, message)."""
    bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
    rc = lib.rw_validate_solve(ctypes.byref(params), len(bricks), bricks.ctypes.data_as(_vp), int(n_voxels))
    return rc, lib.rw_last_error(None).decode()


def solve_params(**kw):
    """rw_solve_params with the library defaults, overridden by ``kw``."""
    p = SolveParams()
    lib.rw_solve_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown solve parameter {k!r}")
        setattr(p, k, v)
    return p


def bricks_array(shapes, offsets):
    """Host rw_brick array from (n,3) shapes (nx, ny, nz) and (n,) offsets."""
    shapes = np.asarray(shapes).reshape(-1, 3)
    b = np.zeros(len(shapes), dtype=BRICK_DTYPE)
    b["nx"], b["ny"], b["nz"] = shapes[:, 0], shapes[:, 1], shapes[:, 2]
    b["offset"] = np.asarray(offsets, dtype=np.int64)
    return b


def _ptr(t):
    """Device pointer of a tensor; the library reads dense buffers, so views
    with gaps are rejected rather than read wrongly."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("librwseg takes contiguous tensors (call .contiguous() first)")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """An rw_ctx on one HIP device (owns the library's workspace)."""

    def __init__(self, device=0):
        h = _vp()
        rc = lib.rw_ctx_create(int(device), ctypes.byref(h))
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(None).decode())
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib.rw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(self.handle).decode())

    def rw_solve_bricks(self, params, bricks, g, mask, x, x64=None, stats=None, stream=None):
        """Queue rw_solve_bricks.  g, mask, x (and x64, stats) are device tensors;
        bricks a host BRICK_DTYPE array; stats a uint8 tensor of n*32 bytes."""
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        n_vox = g.numel()
        self._check(lib.rw_solve_bricks(self.handle, ctypes.byref(params), len(bricks),
                                        bricks.ctypes.data_as(_vp), n_vox, _ptr(g), _ptr(mask), _ptr(x),
                                        _ptr(x64), _ptr(stats), _stream(stream)))

    def rw_solve_bricks_noalloc(self, params, bricks, g, mask, x, x64=None, stats=None, stream=None):
        """Queue rw_solve_bricks_noalloc (same arguments as rw_solve_bricks;
        the workspace comes from the library's fixed device scratch)."""
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        n_vox = g.numel()
        self._check(lib.rw_solve_bricks_noalloc(self.handle, ctypes.byref(params), len(bricks),
                                                bricks.ctypes.data_as(_vp), n_vox, _ptr(g), _ptr(mask), _ptr(x),
                                                _ptr(x64), _ptr(stats), _stream(stream)))

    def rw_solve_bricks_streamed(self, params, bricks, g, mask, x, stats=None, chunk_voxels=0, stream=None):
        """Queue rw_solve_bricks_streamed.  g, mask, x (and stats) are HOST
        tensors (page-locked for overlapped copies); bricks a host
        BRICK_DTYPE array in increasing offset order."""
        for t in (g, mask, x) + ((stats,) if stats is not None else ()):
            if t.is_cuda or not t.is_contiguous():
                raise ValueError("streamed solve: g, mask, x and stats must be contiguous host tensors")
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        self._check(lib.rw_solve_bricks_streamed(self.handle, ctypes.byref(params), len(bricks),
                                                 bricks.ctypes.data_as(_vp), g.numel(), _ptr(g), _ptr(mask),
                                                 _ptr(x), _ptr(stats), int(chunk_voxels), _stream(stream)))

    def set_timing(self, enable=True):
        self._check(lib.rw_set_timing(self.handle, 1 if enable else 0))

    def last_timing(self):
        """Phase durations (ms) of the last timed solve; waits for its events."""
        t = Timing()
        self._check(lib.rw_last_timing(self.handle, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in Timing._fields_}

    def solve_plan(self, params, bricks, n_voxels):
        """Kernel path (PATH_*) of each brick, as an int32 numpy array."""
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        out = np.zeros(len(bricks), dtype=np.int32)
        self._check(lib.rw_solve_plan(self.handle, ctypes.byref(params), len(bricks), bricks.ctypes.data_as(_vp),
                                      int(n_voxels), out.ctypes.data_as(_vp)))
        return out

    def autotune(self, params, bricks, g, mask, x0, x_work, reps=3, stream=None):
        """Time the candidate schedules on this batch (rw_autotune; synchronises
        the stream) and record the fastest for SCHED_TUNED.  Returns the table
        as a dict."""
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        rep = TuneReport()
        self._check(lib.rw_autotune(self.handle, ctypes.byref(params), len(bricks), bricks.ctypes.data_as(_vp),
                                    g.numel(), _ptr(g), _ptr(mask), _ptr(x0), _ptr(x_work), int(reps),
                                    ctypes.byref(rep), _stream(stream)))
        n = rep.n_candidates
        return {"best": rep.best, "key": int(rep.key),
                "candidates": [{"schedule": rep.schedule[i], "third_stream": rep.third_stream[i],
                                "weights_in_registers": rep.weights_in_registers[i],
                                "persistent": rep.persistent[i], "split_boxes": rep.split_boxes[i],
                                "ms": rep.ms[i]}
                               for i in range(n)]}

    def set_plan_choices(self, third_stream=True, weights_in_registers=True, persistent=False):
        """rw_set_plan_choices for the next calls on this context."""
        self._check(lib.rw_set_plan_choices(self.handle, int(bool(third_stream)), int(bool(weights_in_registers)),
                                            int(bool(persistent))))

    def set_split_boxes(self, enable=True):
        """rw_set_split_boxes for the next calls on this context."""
        self._check(lib.rw_set_split_boxes(self.handle, int(bool(enable))))

    def tuned_schedule(self, params, bricks):
        """(schedule, third_stream, weights_in_registers, persistent, tuned) a
        SCHED_TUNED call would use."""
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        v = [ctypes.c_int32() for _ in range(5)]
        self._check(lib.rw_tuned_schedule(self.handle, ctypes.byref(params), len(bricks), bricks.ctypes.data_as(_vp),
                                          *[ctypes.byref(x) for x in v]))
        return v[0].value, v[1].value, v[2].value, v[3].value, bool(v[4].value)

    def probe_read(self, src, passes, part, unroll=8, stream=None):
        """Queue the read probe over tensor ``src`` (``passes`` times, ``unroll``
        loads in flight per thread); ``part`` a float32 device tensor of
        rw_probe_blocks() elements."""
        self._check(lib.rw_probe_read(self.handle, _ptr(src), src.numel() * src.element_size(), int(passes),
                                      int(unroll), _ptr(part), _stream(stream)))

    def probe_copy(self, dst, src, stream=None):
        """Queue a plain copy of tensor ``src`` into ``dst`` (same byte size)."""
        n = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != n:
            raise ValueError("probe_copy: dst and src differ in size")
        self._check(lib.rw_probe_copy(self.handle, _ptr(dst), _ptr(src), n, _stream(stream)))

    def rw_solve_bricks_adjoint(self, params, bricks, g, mask, x, dl_dx, dl_dg, dl_dbeta, lam=None,
                                stats=None, stream=None):
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        self._check(lib.rw_solve_bricks_adjoint(self.handle, ctypes.byref(params), len(bricks),
                                                bricks.ctypes.data_as(_vp), g.numel(), _ptr(g), _ptr(mask),
                                                _ptr(x), _ptr(dl_dx), _ptr(dl_dg), _ptr(dl_dbeta), _ptr(lam),
                                                _ptr(stats), _stream(stream)))


class Graph:
    """A captured rw_solve_bricks launch sequence (rw_graph_create); replay it
    with ``launch``.  ``stream`` must not be the null stream."""

    def __init__(self, ctx, params, bricks, g, mask, x, x64=None, stats=None, stream=None):
        bricks = np.ascontiguousarray(bricks, dtype=BRICK_DTYPE)
        h = _vp()
        rc = lib.rw_graph_create(ctx.handle, ctypes.byref(params), len(bricks), bricks.ctypes.data_as(_vp),
                                 g.numel(), _ptr(g), _ptr(mask), _ptr(x), _ptr(x64), _ptr(stats), _stream(stream),
                                 ctypes.byref(h))
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(ctx.handle).decode())
        self.handle = h
        self._keep = (g, mask, x, x64, stats)    # the graph reads and writes these buffers

    def launch(self, stream=None):
        rc = lib.rw_graph_launch(self.handle, _stream(stream))
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(None).decode())

    def close(self):
        if self.handle:
            lib.rw_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stats_to_numpy(stats_tensor):
    """Parse a device/host uint8 stats tensor into a STATS_DTYPE array."""
    raw = stats_tensor.detach().cpu().numpy().view(np.uint8).reshape(-1)
    return raw.view(STATS_DTYPE)


_default_ctx = {}


def context(device=0):
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def solve_bricks(g, mask, x, shapes, offsets, x64=None, stream=None, ctx=None, **params):
    """Solve all boxes; x is updated in place.  Returns the stats tensor
    (device, uint8 [n, 32]; parse with ``stats_to_numpy``)."""
    import torch
    ctx = ctx or context(g.device.index or 0)
    b = bricks_array(shapes, offsets)
    st = torch.empty((len(b), STATS_DTYPE.itemsize), dtype=torch.uint8, device=g.device)
    ctx.rw_solve_bricks(solve_params(**params), b, g, mask, x, x64=x64, stats=st, stream=stream)
    return st


def solve_bricks_streamed(g, mask, x, shapes, offsets, chunk_voxels=0, stream=None, ctx=None, device=0, **params):
    """Solve boxes held in host memory (x updated in place once the stream
    completes; this call synchronises it).  Returns the host stats tensor."""
    import torch
    ctx = ctx or context(device)
    b = bricks_array(shapes, offsets)
    st = torch.empty((len(b), STATS_DTYPE.itemsize), dtype=torch.uint8, pin_memory=g.is_pinned())
    ctx.rw_solve_bricks_streamed(solve_params(**params), b, g, mask, x, stats=st, chunk_voxels=chunk_voxels,
                                 stream=stream)
    if stream is None:
        torch.cuda.current_stream(device).synchronize()
    else:
        stream.synchronize()
    return st


def solve_bricks_adjoint(g, mask, x, dl_dx, shapes, offsets, lam=None, stream=None, ctx=None, **params):
    """Adjoint gradients: returns (dl_dg tensor, dl_dbeta 1-element float64 tensor, stats)."""
    import torch
    ctx = ctx or context(g.device.index or 0)
    b = bricks_array(shapes, offsets)
    dl_dg = torch.empty_like(g)
    dl_dbeta = torch.empty(1, dtype=torch.float64, device=g.device)
    st = torch.empty((len(b), STATS_DTYPE.itemsize), dtype=torch.uint8, device=g.device)
    ctx.rw_solve_bricks_adjoint(solve_params(**params), b, g, mask, x, dl_dx, dl_dg, dl_dbeta, lam=lam,
                                stats=st, stream=stream)
    return dl_dg, dl_dbeta, st


# ---------------------------------------------------------------------------
# Hierarchical segmentation (pyramid, rw_segment, results)
# ---------------------------------------------------------------------------

RW_U16, RW_F32 = 0, 1
MAX_LEVELS = 16
F_REACHED, F_PRUNABLE, F_CFL, F_SOLVED, F_KEPT = 1, 2, 4, 8, 16


class Params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("eps", ctypes.c_double), ("tol", ctypes.c_double),
                ("expand", ctypes.c_double), ("t_hom", ctypes.c_double), ("t_bin", ctypes.c_double),
                ("t_inc", ctypes.c_double), ("brick", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("n_classes", ctypes.c_int32), ("prune_hom", ctypes.c_int32),
                ("prune_dt", ctypes.c_int32), ("refine_max", ctypes.c_int32), ("incremental", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("joint_classes", ctypes.c_int32), ("host_levels", ctypes.c_int32)]


class Seed(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double),
                ("label", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_L = ctypes.c_int64 * MAX_LEVELS


class RunStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("reserved", ctypes.c_int32), ("bricks", _L), ("computed", _L),
                ("solved", _L), ("prunable", _L), ("voxel_iters", _L), ("box_voxels", _L),
                ("max_iters", ctypes.c_int32 * MAX_LEVELS), ("not_converged", ctypes.c_int32 * MAX_LEVELS)]

    def as_dict(self):
        n = self.levels
        return {k: [int(v) for v in getattr(self, k)[:n]] for k, _ in self._fields_[2:]}


_dims3 = ctypes.c_int64 * 3
lib.rw_params_default.argtypes = [ctypes.POINTER(Params)]
lib.rw_params_default.restype = None
lib.rw_pyramid_build.argtypes = [_vp, _vp, ctypes.c_int, _dims3, ctypes.c_int, ctypes.POINTER(_vp), _vp]
lib.rw_pyramid_build.restype = ctypes.c_int
lib.rw_pyramid_build_counts.argtypes = lib.rw_pyramid_build.argtypes
lib.rw_pyramid_build_counts.restype = ctypes.c_int
lib.rw_pyramid_build_host.argtypes = [_vp, _vp, ctypes.c_int, _dims3, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp),
                                      _vp]
lib.rw_pyramid_build_host.restype = ctypes.c_int
lib.rw_pyramid_free.argtypes = [_vp]
lib.rw_pyramid_free.restype = None
lib.rw_pyramid_level.argtypes = [_vp, ctypes.c_int, _dims3, ctypes.POINTER(_vp)]
lib.rw_pyramid_level.restype = ctypes.c_int
lib.rw_segment.argtypes = [_vp, _vp, _vp, _i64, ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp), _vp]
lib.rw_segment.restype = ctypes.c_int
lib.rw_result_free.argtypes = [_vp]
lib.rw_result_free.restype = None
lib.rw_result_stats.argtypes = [_vp, ctypes.POINTER(RunStats)]
lib.rw_result_stats.restype = ctypes.c_int
lib.rw_result_level.argtypes = [_vp, ctypes.c_int, _dims3, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_vp)]
lib.rw_result_level.restype = ctypes.c_int
lib.rw_result_flags.argtypes = [_vp, ctypes.c_int, _dims3, ctypes.POINTER(_vp)]
lib.rw_result_flags.restype = ctypes.c_int
lib.rw_result_materialize.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
lib.rw_result_materialize.restype = ctypes.c_int
for _f in ("rw_result_copy_level", "rw_result_copy_flags", "rw_pyramid_copy_level"):
    getattr(lib, _f).argtypes = [_vp, _vp, ctypes.c_int, _vp, _vp]
    getattr(lib, _f).restype = ctypes.c_int


# rw_params.incremental bits (runs with a previous result)
INC_NODE = 1   # the node rule of Section IV-E (else the dirty-brick rule)
INC_WARM = 2   # warm start of the solved boxes from the previous result


def params(**kw):
    """rw_params with the library defaults, overridden by ``kw``."""
    p = Params()
    lib.rw_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k!r}")
        setattr(p, k, v)
    return p


def seeds_array(seeds):
    """ctypes rw_seed array from an (n, 4) array of (x, y, z, label)."""
    s = np.asarray(seeds, dtype=np.float64).reshape(-1, 4)
    arr = (Seed * max(len(s), 1))()
    for i, (x, y, z, lab) in enumerate(s):
        arr[i] = Seed(float(x), float(y), float(z), int(lab), 0)
    return arr, len(s)


class Pyramid:
    """LOD pyramid on the device.  counts=False: normalised intensities
    (rw_pyramid_build); counts=True: square roots of the mean counts, for the
    Poisson weight with beta 0.5 (rw_pyramid_build_counts).  host_levels > 0:
    the finest host_levels levels in page-locked host memory
    (rw_pyramid_build_host; `volume` may then be a pinned CPU tensor)."""

    def __init__(self, ctx, volume, levels, stream=None, counts=False, host_levels=0):
        import torch
        self.ctx = ctx
        dt = {torch.uint16: RW_U16, torch.float32: RW_F32}.get(volume.dtype)
        if dt is None:
            raise TypeError("volume must be uint16 or float32")
        nz, ny, nx = volume.shape
        h = _vp()
        if host_levels:
            if counts:
                raise ValueError("host_levels is supported for the intensity pyramid only")
            ctx._check(lib.rw_pyramid_build_host(ctx.handle, _ptr(volume), dt, _dims3(nx, ny, nz), int(levels),
                                                 int(host_levels), ctypes.byref(h), _stream(stream)))
        else:
            build = lib.rw_pyramid_build_counts if counts else lib.rw_pyramid_build
            ctx._check(build(ctx.handle, _ptr(volume), dt, _dims3(nx, ny, nz), int(levels), ctypes.byref(h),
                             _stream(stream)))
        self.handle = h
        self.levels = levels
        self.device = volume.device if volume.is_cuda else torch.device("cuda", ctx.device)

    def level(self, l, stream=None):
        """Copy of pyramid level l as a (nz, ny, nx) float32 device tensor."""
        import torch
        d = _dims3()
        rc = lib.rw_pyramid_level(self.handle, int(l), d, None)
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(None).decode())
        nx, ny, nz = d
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device)
        self.ctx._check(lib.rw_pyramid_copy_level(self.ctx.handle, self.handle, int(l), _ptr(out), _stream(stream)))
        return out

    def close(self):
        if self.handle:
            lib.rw_pyramid_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Result:
    def __init__(self, ctx, handle, device):
        self.ctx, self.handle, self.device = ctx, handle, device

    def stats(self):
        st = RunStats()
        rc = lib.rw_result_stats(self.handle, ctypes.byref(st))
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(None).decode())
        return st.as_dict()

    def level_map(self, l, stream=None):
        """Copy of level map l as a (nz, ny, nx, K-1) float32 device tensor."""
        import torch
        d = _dims3()
        r = ctypes.c_int()
        rc = lib.rw_result_level(self.handle, int(l), d, ctypes.byref(r), None)
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(None).decode())
        nx, ny, nz = d
        out = torch.empty((nz, ny, nx, r.value), dtype=torch.float32, device=self.device)
        self.ctx._check(lib.rw_result_copy_level(self.ctx.handle, self.handle, int(l), _ptr(out), _stream(stream)))
        return out

    def flags(self, l, stream=None):
        """Copy of level l's brick flags as a (nbz, nby, nbx) uint8 device tensor."""
        import torch
        d = _dims3()
        rc = lib.rw_result_flags(self.handle, int(l), d, None)
        if rc != RW_OK:
            raise RWError(rc, lib.rw_last_error(None).decode())
        nx, ny, nz = d
        out = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.device)
        self.ctx._check(lib.rw_result_copy_flags(self.ctx.handle, self.handle, int(l), _ptr(out), _stream(stream)))
        return out

    def materialize(self, level=0, cls=1, prob=True, labels=False, stream=None):
        import torch
        d = _dims3()
        r = ctypes.c_int()
        lib.rw_result_level(self.handle, int(level), d, ctypes.byref(r), None)
        nx, ny, nz = d
        pr = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device) if prob else None
        lb = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.device) if labels else None
        self.ctx._check(lib.rw_result_materialize(self.ctx.handle, self.handle, int(level), int(cls), _ptr(pr),
                                                  _ptr(lb), _stream(stream)))
        return pr, lb

    def close(self):
        if self.handle:
            lib.rw_result_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def segment(pyramid, seeds, prev=None, stream=None, ctx=None, **kw):
    """Hierarchical segmentation of a Pyramid with (n, 4) seeds (x, y, z, label)."""
    ctx = ctx or pyramid.ctx
    arr, n = seeds_array(seeds)
    h = _vp()
    ctx._check(lib.rw_segment(ctx.handle, pyramid.handle, arr, n, ctypes.byref(params(**kw)),
                              prev.handle if prev is not None else None, ctypes.byref(h), _stream(stream)))
    return Result(ctx, h, pyramid.device)


# ---------------------------------------------------------------------------
# Differentiation: autograd wrapper around the batched solve and its adjoint
# ---------------------------------------------------------------------------

def _make_rwsolve():
    import torch

    class RWSolve(torch.autograd.Function):
        """x = rw(g, beta) for a batch of boxes, differentiable in g and beta.

        forward(g, beta, mask, x_dirichlet, shapes, offsets, eps, tol, precision):
        solves every box (x_dirichlet supplies the seeded values and the start);
        backward runs the library's adjoint (L_UU lambda = dl/dx_U and the
        edge-weight chain rule) and returns dl/dg (per voxel) and dl/dbeta.
        The Dirichlet values get no gradient.
        """

        @staticmethod
        def forward(fctx, g, beta, mask, x_dirichlet, shapes, offsets, eps=1e-6, tol=1e-8,
                    precision=PREC_MIXED_REFINE, adjoint_tol=1e-8):
            b = float(beta.detach().cpu()) if torch.is_tensor(beta) else float(beta)
            x = x_dirichlet.detach().clone()
            st = solve_bricks(g.detach(), mask, x, shapes, offsets, beta=b, eps=eps, tol=tol, precision=precision,
                              refine_max=4, refine_tol=tol)
            fctx.save_for_backward(g.detach(), x)
            fctx.meta = (mask, shapes, offsets, b, eps, adjoint_tol, torch.is_tensor(beta))
            fctx.solve_stats = st
            return x

        @staticmethod
        def backward(fctx, grad_x):
            g, x = fctx.saved_tensors
            mask, shapes, offsets, b, eps, atol, beta_is_tensor = fctx.meta
            dl_dg, dl_dbeta, _ = solve_bricks_adjoint(g, mask, x, grad_x.contiguous().float(), shapes, offsets,
                                                      beta=b, eps=eps, tol=atol)
            gb = dl_dbeta.reshape(()).to(torch.float32) if beta_is_tensor else None
            return dl_dg, gb, None, None, None, None, None, None, None, None

    return RWSolve


try:
    RWSolve = _make_rwsolve()
except ImportError:   # torch is only needed for the autograd wrapper
    RWSolve = None
