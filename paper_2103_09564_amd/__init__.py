"""MI355X-native brick-local random-walker segmentation (arXiv 2103.09564).

The compute path is librwseg.so (hand-written gfx950 HIP kernels behind the C
ABI in include/rwseg.h); ``binding`` marshals torch tensors into it.
"""

from .binding import (  # noqa: F401
    Context, RWError, SolveParams, BRICK_DTYPE, STATS_DTYPE, STATUS_NAMES,
    PREC_FP64, PREC_MIXED, PREC_MIXED_REFINE, PATH_STREAM, PATH_STREAM_GLOBAL, PATH_RESIDENT, PATH_DOMAIN,
    PATH_RESIDENT_STREAMED, PATH_RESIDENT_SPLIT,
    RW_OK, RW_E_INVAL, RW_E_HIP, RW_E_NOMEM, RW_E_UNSUPPORTED, noalloc_scratch_bytes, probe_blocks, Graph, SCHED_TUNED,
    bricks_array, context, solve_bricks, solve_bricks_adjoint, solve_bricks_streamed, solve_params, stats_to_numpy, validate_solve, version,
    Params, Pyramid, Result, params, segment, F_REACHED, F_PRUNABLE, F_CFL, F_SOLVED, F_KEPT, RWSolve,
    INC_NODE, INC_WARM,
)
