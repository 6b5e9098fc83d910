/*
 * rwseg.h -- C ABI of the MI355X (gfx950) brick-local random-walker library.
 *
 * Method: Drees, Eilers & Jiang, "Hierarchical Random Walker Segmentation for
 * Large Volumetric Biomedical Images", arXiv 2103.09564.
 *
 * Everything below takes plain pointers and sizes.  "dev" marks a device
 * (HBM) pointer, "host" a host pointer.  The caller owns every buffer it
 * passes and keeps it alive until the work queued on `stream` has finished;
 * the library never frees a caller buffer.  Library objects (rw_ctx,
 * rw_pyramid, rw_result) are opaque and freed only by their *_free/_destroy
 * call.  `stream` is a hipStream_t passed as void* (NULL = the null stream);
 * all device work is queued on it, asynchronously, unless a call says
 * otherwise.  Device stats and outputs are valid after a stream sync.
 *
 * Errors: every int-returning call returns RW_OK (0) or a negative RW_E_*
 * code; rw_last_error(ctx) gives a message.  Arguments are validated on the
 * host before anything is queued.  Per-brick numerical outcomes (iteration
 * cap, non-finite data, no Dirichlet voxel) are reported in rw_brick_stats and
 * never fail a call.  One rw_ctx per host thread.
 *
 * Box layout: a box of nx*ny*nz voxels is stored contiguously from its
 * element offset `offset`; voxel (i,j,k) sits at offset + i + nx*(j + ny*k).
 * With nrhs right-hand sides the per-voxel values are interleaved:
 * element (offset + v)*nrhs + c.
 */
#ifndef RWSEG_H
#define RWSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RW_VERSION 100

enum rw_error {
    RW_OK = 0,
    RW_E_INVAL = -1,        /* bad argument (message says which) */
    RW_E_HIP = -2,          /* a HIP runtime call failed */
    RW_E_NOMEM = -3,        /* device allocation failed */
    RW_E_UNSUPPORTED = -4   /* valid request this build does not implement */
};

enum rw_precision {
    RW_PREC_FP64 = 0,          /* plain FP64 PCG: vectors, weights, reductions in FP64 */
    RW_PREC_MIXED = 1,         /* FP32 stencil/vectors, FP64 dot products, FP64 true-residual
                                  check, and at most refine_max FP32 correction solves when the
                                  true residual exceeds stall_ratio * tol */
    RW_PREC_MIXED_REFINE = 2   /* as MIXED, then FP64 iterative refinement of an FP64 copy of x
                                  until the FP64 true relative residual <= refine_tol */
};

enum rw_status {
    RW_ST_CONVERGED = 0,     /* recursive ||r|| <= tol ||b|| (and, MIXED, FP64 true residual
                                <= stall_ratio * tol) */
    RW_ST_MAX_ITER = 1,      /* hit max_iter before tol */
    RW_ST_REFINED = 2,       /* FP32 solve stalled in FP64; refinement brought it within target */
    RW_ST_STALLED = 3,       /* refinement steps exhausted without meeting the target */
    RW_ST_NONFINITE = 4,     /* NaN/Inf met (input g or breakdown); x left as the last finite iterate */
    RW_ST_NO_DIRICHLET = 5,  /* box has no seeded voxel: problem has no unique solution, x untouched */
    RW_ST_SYNC_LOST = 6      /* the two workgroups of a split box (RW_PATH_RESIDENT_SPLIT) stopped
                                hearing from each other within a few seconds (a scheduling failure,
                                not a numerical one); x left as the last iterate */
};

/* One box (solve domain).  nx, ny, nz >= 1. */
typedef struct rw_brick {
    int32_t nx, ny, nz;
    int32_t reserved;        /* must be 0 */
    int64_t offset;          /* first voxel, in voxels, into g / mask / x */
} rw_brick;

/* Per-box result, written to device memory. */
typedef struct rw_brick_stats {
    int32_t iters;           /* PCG iterations of the main solve (max over rhs) */
    int32_t status;          /* rw_status (worst over rhs) */
    int32_t refine_steps;    /* FP64-residual correction solves run */
    int32_t refine_iters;    /* PCG iterations summed over those correction solves */
    double rel_resid;        /* final recursive ||r||/||b|| of the main solve (max over rhs) */
    double true_rel_resid;   /* FP64 ||b - L_UU x_U|| / ||b|| of the returned x (max over rhs);
                                0 if ||b|| = 0 */
} rw_brick_stats;

/* Parameters of the box solve (Section III-B; solver as in Section V). */
typedef struct rw_solve_params {
    double beta;             /* w = exp(-beta (g_p - g_q)^2) + eps, beta >= 0 */
    double eps;              /* eps >= 0 */
    double tol;              /* stop when ||r||_2 <= tol ||b||_2, b = -L_UM x_M; tol >= 0 */
    int32_t max_iter;        /* PCG iteration cap (the paper uses 5000) */
    int32_t precision;       /* rw_precision */
    int32_t nrhs;            /* 1..3 right-hand sides sharing g and the seed mask */
    int32_t refine_max;      /* max correction solves (MIXED: usually 1, MIXED_REFINE: e.g. 4) */
    double refine_tol;       /* MIXED_REFINE target FP64 true relative residual */
    double inner_tol;        /* relative tolerance of each FP32 correction solve */
    double stall_ratio;      /* MIXED: a box counts as stalled, and gets a correction solve, when
                                its FP64 true relative residual exceeds stall_ratio * tol (>= 1) */
    int32_t schedule;        /* CG iteration schedule: 0 library choice (MIXED with nrhs 1: boxes
                                up to 32^3 whose search direction fits one CU's LDS run resident,
                                RW_PATH_RESIDENT or RW_PATH_RESIDENT_STREAMED; the others stream
                                as in 1), 1 streaming, two sweeps and two
                                reductions per iteration (Hestenes-Stiefel), 2 streaming, one
                                sweep and one reduction (Chronopoulos-Gear; weights computed once
                                per iteration), 3 as 0 with the streaming boxes as in 2, 4 as 0
                                with every box that fits it on the streamed-weights resident
                                kernel (RW_PATH_RESIDENT_STREAMED), RW_SCHED_TUNED (5) the
                                schedule rw_autotune measured fastest for the batch.  Every
                                schedule is the same Jacobi-PCG iteration in exact arithmetic;
                                results differ by rounding (the one-sweep recurrence is the less
                                stable one on very ill-conditioned boxes). */
    int32_t reserved;        /* must be 0 */
} rw_solve_params;

/* rw_solve_params.schedule value: the schedule rw_autotune measured fastest
 * for this batch (its box shapes, nrhs and precision) on this context, or
 * schedule 0 when the batch was not tuned. */
#define RW_SCHED_TUNED 5

/* Fill *p with the defaults: beta 128, eps 1e-6, tol 1e-6, max_iter 5000,
 * MIXED, nrhs 1, refine_max 1, refine_tol 1e-13, inner_tol 1e-4, stall_ratio 10. */
void rw_solve_params_default(rw_solve_params* p);

typedef struct rw_ctx rw_ctx;

int rw_version(void);

/* Create a context on HIP device `hip_device`.  The context owns a device
 * workspace that grows on demand and is freed by rw_ctx_destroy, which also
 * frees the device's cached hierarchy buffers (see rw_result_free). */
int rw_ctx_create(int hip_device, rw_ctx** out);
void rw_ctx_destroy(rw_ctx* ctx);

/* Message of the last error on this context ("" if none).  The pointer is
 * valid until the next call on ctx.  ctx may be NULL (then: the last error
 * of rw_ctx_create on this thread). */
const char* rw_last_error(const rw_ctx* ctx);

/*
 * Batched brick-local random-walker solve (Section III-B, eq. rw(n, l, beta)
 * of Section IV-A applied to each box independently, as Section IV-D3 allows).
 *
 * For every box: weights w = exp(-beta (g_p - g_q)^2) + eps on all
 * 6-neighbour pairs inside the box, Laplacian L = D - W, and the Dirichlet
 * problem L_UU x_U = -L_UM x_M on the unseeded set U (mask == 0) with the
 * seeded values x_M (mask != 0) taken from x.  Solved by Jacobi-preconditioned
 * CG (Section V) starting from the values x holds on U.
 *
 *   bricks   host, n_bricks descriptors; boxes may not overlap
 *   n_voxels dev buffers below hold n_voxels voxels (every box must fit)
 *   g        dev float [n_voxels]          intensities (any range; beta applies as given)
 *   mask     dev uint8 [n_voxels]          nonzero = seeded (Dirichlet)
 *   x        dev float [n_voxels*nrhs]     in: x_M on seeded voxels, initial guess elsewhere;
 *                                          out: solution (seeded voxels unchanged)
 *   x64      dev double [n_voxels*nrhs] or NULL: if given, also receives the solution in FP64
 *            (MIXED_REFINE: the refined FP64 solution; its seeded entries are x_M)
 *   stats    dev rw_brick_stats [n_bricks] or NULL
 *
 * Returns RW_E_INVAL on bad descriptors/params; numerical outcomes go to stats.
 */
int rw_solve_bricks(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks,
                    const rw_brick* bricks, int64_t n_voxels, const float* g,
                    const uint8_t* mask, float* x, double* x64, rw_brick_stats* stats,
                    void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as rw_solve_bricks, with the same arguments, kernels and results,
 * that allocates nothing.  Its workspace (CG vectors, per-box state, the
 * device box list and the weight segments of the streamed-weights boxes) is
 * carved from a fixed device array of rw_noalloc_scratch_bytes() bytes
 * (64 MiB) that the library holds on each device from its first
 * rw_ctx_create there until the process ends; all kernels run on `stream`
 * (no side streams, no events, no phase timing).  A batch whose workspace
 * exceeds the array is rejected with RW_E_INVAL before anything is queued
 * (about 20 bytes per voxel and right-hand side for MIXED, 40 for FP64 or
 * when x64 is not given on MIXED_REFINE, plus 17 bytes per voxel of boxes on
 * the streamed-weights path and about 200 bytes per box: some fifty 32^3
 * boxes).  Every call on a device shares that device's array and leaves its
 * last contents there: calls that overlap on one device (on different
 * streams, or from different host threads) race and corrupt each other's
 * results; order them on one stream.  The box list is copied from host
 * memory on `stream`.  Host-side planning still uses the C++ heap.
 */
int rw_solve_bricks_noalloc(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks,
                            const rw_brick* bricks, int64_t n_voxels, const float* g,
                            const uint8_t* mask, float* x, double* x64, rw_brick_stats* stats,
                            void* stream);
size_t rw_noalloc_scratch_bytes(void);

/*
 * The same solve for boxes held in host memory, streamed through the GPU
 * (out-of-core brick queues; the paper's volumes reach hundreds of GB, more
 * than one GPU holds).  g, mask, x and stats have rw_solve_bricks' layout but
 * are HOST arrays; page-locked memory (hipHostMalloc) lets the copies run
 * asynchronously and overlap the solves, pageable memory works but copies
 * synchronously.  The boxes must be listed in increasing offset order without
 * overlap; runs of consecutive boxes whose voxel span is at most
 * chunk_voxels (0: 2^24; a larger box forms a chunk alone) go round two
 * lanes: chunk c is copied into lane c % 2's device staging set on a copy
 * stream, solved by that lane (lane 0: ctx on `stream`; lane 1: an internal
 * context with its own workspaces and stream), and its x
 * (and stats) copied back on a second copy stream, so copies in, solves of
 * consecutive chunks and copies out overlap.  Every chunk takes the kernel
 * variants the whole list would get, so per box the result is bit-identical
 * to rw_solve_bricks on the whole list, except where that call would leave
 * single-domain boxes beyond its cap of 64 to the window kernels (a chunk may
 * then run them on the domain solver: equal up to rounding).  No x64 output.  The call returns
 * once everything is queued: x and stats are complete when `stream` has
 * completed (every other stream is joined to it).  On an error part-way the
 * queued work finishes before the call returns.  The staging sets (about
 * 2 x (9 + 4 (nrhs - 1)) bytes per voxel of the largest chunk), page-locked
 * copies of the box lists and the lane context stay allocated on ctx.
 * Each chunk's solve ends with its slowest box: chunks much smaller than the
 * default leave the GPU idle in those tails.
 * Returns RW_E_INVAL on bad descriptors (as rw_solve_bricks, plus the order).
 */
int rw_solve_bricks_streamed(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks,
                             const rw_brick* bricks, int64_t n_voxels, const float* g,
                             const uint8_t* mask, float* x, rw_brick_stats* stats,
                             int64_t chunk_voxels, void* stream);

/*
 * Phase timing of rw_solve_bricks (tracing).  With timing enabled the next
 * solves record HIP events on their stream around each phase; rw_last_timing
 * waits for those events and returns the phase durations of the last solve
 * in milliseconds.  pcg_ms is the main PCG phase alone (the hot loop).  In
 * that phase two groups of kernels run concurrently on two streams (see
 * rw_solve_plan): the streaming boxes followed by the streamed-weights
 * resident boxes, and the boxes resident in LDS; stream_ms and resident_ms
 * are the durations of the two groups (0 for an empty group).  When the
 * streamed-weights boxes form two launches beside LDS-resident ones (and no
 * box streams), the second launch runs on a third stream, concurrently with
 * the first: stream_ms then times the first launch and stream2_ms the second.  In a one-rhs
 * MIXED or MIXED_REFINE solve the resident kernels compute their boxes'
 * start state themselves, inside pcg_ms; init_ms covers the other boxes.  In
 * a one-rhs MIXED solve each group's first FP64 check runs on its stream
 * right after the group, so it falls in pcg_ms (not in stream_ms or
 * resident_ms) and finish_ms keeps the rest of the check phase.
 */
typedef struct rw_timing {
    float init_ms;           /* Dirichlet init (r = -(L x)_U, z, p) of the non-resident boxes */
    float pcg_ms;            /* main PCG phase */
    float finish_ms;         /* FP64 true residual (when not done in pcg_ms), refinement, stats */
    float total_ms;
    float stream_ms;         /* main PCG: RW_PATH_STREAM* then RW_PATH_RESIDENT_STREAMED boxes
                                (only the first of two streamed-weights launches when stream2_ms > 0) */
    float resident_ms;       /* main PCG: RW_PATH_RESIDENT boxes */
    float stream2_ms;        /* main PCG: the second streamed-weights launch (boxes up to 17408 voxels)
                                when it runs on a stream of its own beside the first, else 0 */
} rw_timing;
int rw_set_timing(rw_ctx* ctx, int enable);
int rw_last_timing(rw_ctx* ctx, rw_timing* out);

/*
 * Autotuner (a batching pattern, not a step of the method).  Times candidate
 * schedules of rw_solve_bricks on this batch and records the fastest on ctx
 * for RW_SCHED_TUNED: for MIXED or MIXED_REFINE with one rhs schedule 0
 * (as is, without the second streamed-weights launch on a stream of its
 * own, with the small resident boxes' weights in LDS instead of registers,
 * with persistent resident grids, and, when the batch has boxes that split,
 * with those boxes streaming), schedule 4, schedule 3 and schedule 1;
 * otherwise schedules 1 and 2.  Each
 * candidate runs 1 + reps solves of the batch from x0 (dev, copied into
 * x_work before every run; both [n_voxels * nrhs]); the median of the reps
 * timed runs (HIP events on `stream`) ranks it.  params->schedule must be
 * 0..4 (ignored otherwise: every candidate sets it).  The call synchronises
 * `stream`.  out (host, may be NULL) receives the table.  A later tuning of
 * the same batch signature replaces the entry.  Results of every candidate
 * are equal up to rounding (they are the same Jacobi-PCG).
 */
typedef struct rw_tune_report {
    int32_t n_candidates;
    int32_t best;             /* index of the fastest candidate */
    int32_t schedule[8];      /* rw_solve_params.schedule of each candidate */
    int32_t third_stream[8];  /* 1: the second streamed-weights launch may take a stream of its own */
    int32_t weights_in_registers[8];  /* 1: small resident boxes keep their edge weights in registers
                                         (RW_PATH_RESIDENT, k_pcg_resr), 0: in LDS (k_pcg_resw) */
    int32_t persistent[8];    /* 1: the register- and LDS-resident launches are persistent grids (as many workgroups
                                 as the CUs hold, each taking boxes in launch order from a device
                                 counter), 0: one workgroup per box */
    float ms[8];              /* median milliseconds per solve */
    uint64_t key;             /* signature of the batch */
    int32_t split_boxes[8];   /* 1: boxes above 32768 voxels that fit run split over two
                                 workgroups (RW_PATH_RESIDENT_SPLIT), 0: they stream */
} rw_tune_report;
int rw_autotune(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                int64_t n_voxels, const float* g, const uint8_t* mask, const float* x0, float* x_work, int reps,
                rw_tune_report* out, void* stream);
/* The plan choices of the next calls on ctx (those the autotuner also
 * varies; a tuned entry's choices are applied on top): the second
 * streamed-weights launch may take a stream of its own (default 1), small
 * resident boxes keep their weights in registers (default 1), the register-
 * and LDS-resident launches run as persistent grids (default 0; the
 * streamed-weights launches always take one workgroup per box).  Each 0 or 1.  Results do not
 * depend on them: every box runs the same iteration in every plan. */
int rw_set_plan_choices(rw_ctx* ctx, int third_stream, int weights_in_registers, int persistent);
/* Whether boxes above 32768 voxels whose halves fit (RW_PATH_RESIDENT_SPLIT)
 * run split over two workgroups (enable = 1, the default) or on the
 * streaming kernels (0), for the next calls on ctx that carry no tuned plan.
 * Host-only.  RW_E_INVAL unless enable is 0 or 1. */
int rw_set_split_boxes(rw_ctx* ctx, int enable);

/* Host-only: the schedule and plan choices a RW_SCHED_TUNED call would run
 * for this batch (*tuned = 1 when ctx holds a measured entry for it, else 0
 * and the default); regs and persist may be NULL. */
int rw_tuned_schedule(const rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                      int32_t* schedule, int32_t* third_stream, int32_t* regs, int32_t* persist,
                      int32_t* tuned);

/*
 * Captured graph of one batched solve (a batching pattern, not a step of the
 * method): the whole launch sequence of rw_solve_bricks for these boxes,
 * buffers and params, recorded once with stream capture on `stream` (not
 * the null stream) and replayed by rw_graph_launch with no host planning and
 * no allocation.  Nothing runs at creation; each launch solves the boxes
 * from whatever g, mask and x (and x64, stats) hold then, exactly as
 * rw_solve_bricks would.  The graph owns its device workspace (allocated at
 * creation, like rw_solve_bricks' workspace) and the box list, so it does not
 * depend on ctx afterwards; the caller keeps the buffers alive while the
 * graph exists.  Replays of one graph must not overlap (they share its
 * workspace).  Errors: as rw_solve_bricks, plus RW_E_UNSUPPORTED for a batch
 * with single-domain boxes (that solver polls the host) and RW_E_HIP when
 * capture fails.  No phase timing inside a graph.
 */
typedef struct rw_graph rw_graph;
int rw_graph_create(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                    int64_t n_voxels, const float* g, const uint8_t* mask, float* x, double* x64,
                    rw_brick_stats* stats, void* stream, rw_graph** out);
int rw_graph_launch(rw_graph* graph, void* stream);
void rw_graph_free(rw_graph* graph);

/* Kernel path of a box in rw_solve_bricks. */
enum rw_path {
    RW_PATH_STREAM = 0,          /* one workgroup per box, vectors streamed from HBM, LDS window march */
    RW_PATH_STREAM_GLOBAL = 1,   /* the same without the LDS window (planes wider than it holds) */
    RW_PATH_RESIDENT = 2,        /* one workgroup per box, p in LDS, x and r in registers, the edge
                                    weights in registers (boxes up to 9216 voxels) or in LDS (up
                                    to 10240 voxels) */
    RW_PATH_DOMAIN = 3,          /* large box: many workgroups (every large box of the call in each launch), host-driven iteration */
    RW_PATH_RESIDENT_STREAMED = 4, /* one workgroup per box, p in LDS, r in registers; the edge
                                    weights and 1/d are computed once into a per-box buffer and
                                    re-read from cache each iteration (boxes up to 32768 voxels) */
    RW_PATH_RESIDENT_SPLIT = 5   /* two workgroups per box, one per half along z, each as
                                    RW_PATH_RESIDENT_STREAMED on its half; the halves exchange
                                    their partial sums and one plane of z per iteration through
                                    global memory (boxes above 32768 voxels whose halves hold at
                                    most 32768 and whose planes at most 2048) */
};

/*
 * Host-only: the kernel path rw_solve_bricks would take for each brick with
 * these params on ctx's device (caller order) into path[n_bricks] (host).
 * Validates like rw_solve_bricks; queues nothing.
 */
int rw_solve_plan(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                  int64_t n_voxels, int32_t* path);

/*
 * Host-only check of the arguments rw_solve_bricks would validate (params,
 * descriptors, buffer extents, overlap).  Needs no GPU and queues nothing.
 * Returns RW_OK or RW_E_INVAL; the message is in rw_last_error(NULL).
 */
int rw_validate_solve(const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                      int64_t n_voxels);

/*
 * Adjoint of rw_solve_bricks for gradients of a loss l(x) (derived from the
 * Dirichlet problem of Section III-B).  For each box solves
 * L_UU lambda = dl/dx_U (lambda = 0 on seeded voxels) with the same FP32 PCG
 * (params->tol, params->max_iter; nrhs must be 1), then, per edge e = (p,q),
 * dl/dw_e = -(lambda_p - lambda_q)(x_p - x_q) and
 *   dl_dg[p] += dl/dw_e * dw_e/dg_p,  dw/dg_p = -2 beta (g_p - g_q)(w - eps) = -dw/dg_q,
 *   dl_dbeta += dl/dw_e * (-(g_p - g_q)^2 (w - eps)).
 *
 *   x        dev float [n_voxels]   the converged forward solution
 *   dl_dx    dev float [n_voxels]   loss gradient (ignored on seeded voxels)
 *   dl_dg    dev float [n_voxels]   out: gradient w.r.t. g (every voxel, seeded included)
 *   dl_dbeta dev double [1]         out: gradient w.r.t. beta (FP64, summed over all boxes)
 *   lambda   dev float [n_voxels] or NULL: out, the adjoint solution
 *   stats    dev rw_brick_stats [n_bricks] or NULL: adjoint solve stats
 */
int rw_solve_bricks_adjoint(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks,
                            const rw_brick* bricks, int64_t n_voxels, const float* g,
                            const uint8_t* mask, const float* x, const float* dl_dx,
                            float* dl_dg, double* dl_dbeta, float* lambda,
                            rw_brick_stats* stats, void* stream);

/*
 * Memory-system probes (measurement, not a step of the method): the
 * ceilings the solve kernels are measured against on the device at hand.
 * rw_probe_read queues one kernel of rw_probe_blocks() workgroups that reads
 * the `bytes` at `src` (dev, 16-byte aligned, bytes a positive multiple of
 * 16) `passes` times with 16-byte loads, `unroll` (4, 8 or 16) of them in
 * flight per thread, and writes one float per workgroup to
 * `part` (dev float [rw_probe_blocks()]); a buffer well beyond the 256 MB
 * last-level cache measures HBM, a smaller one read many times that cache.
 * rw_probe_copy queues a plain copy of `bytes` from src to dst (dev, 16-byte
 * aligned, not overlapping).  Time them with events on `stream`.
 * Errors: RW_E_INVAL on a bad size, alignment or overlap.
 */
int rw_probe_blocks(void);
int rw_probe_read(rw_ctx* ctx, const void* src, int64_t bytes, int passes, int unroll, float* part,
                  void* stream);
int rw_probe_copy(rw_ctx* ctx, void* dst, const void* src, int64_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Hierarchical random walker over the LOD pyramid (Sections III-A and IV).
 * ------------------------------------------------------------------------ */

enum rw_dtype { RW_U16 = 0, RW_F32 = 1 };

typedef struct rw_pyramid rw_pyramid;
typedef struct rw_result rw_result;

#define RW_MAX_LEVELS 16

/*
 * Build the LOD pyramid (Section III-A) on the device: level 0 is the volume
 * normalised to [0,1] (uint16: global min-max; float: clipped), level l+1 is
 * the 2x2x2 mean of level l (partial blocks at odd edges average the voxels
 * they have; dims halve rounding up).  `vol` dev [nz][ny][nx] (x fastest);
 * dims = {nx, ny, nz}; 1 <= levels <= RW_MAX_LEVELS.  The pyramid owns its
 * device memory.  Work is queued on `stream`; the call returns after it is
 * queued.  Errors: RW_E_INVAL (dims, dtype, levels; `vol` not device memory
 * or page-locked host memory), RW_E_NOMEM.
 */
int rw_pyramid_build(rw_ctx* ctx, const void* vol, int dtype, const int64_t dims[3], int levels,
                     rw_pyramid** out, void* stream);

/*
 * Out-of-core pyramid (Section IV-A: the bricks a solve touches are small,
 * the volume need not fit in device memory).  As rw_pyramid_build, but
 * levels 0 .. host_levels - 1 (0 <= host_levels < levels) live in
 * page-locked, coherent host memory that the device's kernels read and write
 * in place over the host link; the coarser levels are in device memory.
 * `vol` may itself be page-locked host memory (hipHostMalloc, a pinned
 * tensor); pageable memory is rejected.  The levels equal rw_pyramid_build's
 * bit for bit.  Pair it with rw_params.host_levels for the level maps.
 * Errors: RW_E_INVAL (as rw_pyramid_build; host_levels), RW_E_NOMEM (host
 * or device memory).
 */
int rw_pyramid_build_host(rw_ctx* ctx, const void* vol, int dtype, const int64_t dims[3], int levels,
                          int host_levels, rw_pyramid** out, void* stream);

/*
 * The pyramid for the Poisson-noise weight of Section IV-C, where the edge
 * weight between voxels of counts n_p and n_q is exp(-(sqrt n_p - sqrt n_q)^2 / 2).
 * Level 0 holds the counts (uint16 as is; float clipped below at 0), level
 * l+1 the 2x2x2 mean of level l's counts (as in rw_pyramid_build), and then
 * every level is replaced by its square root.  With rw_params.beta = 0.5 the
 * library's weight exp(-beta dg^2) + eps is that weight (plus the eps floor).
 * Arguments, ownership and errors as for rw_pyramid_build.
 */
int rw_pyramid_build_counts(rw_ctx* ctx, const void* vol, int dtype, const int64_t dims[3], int levels,
                            rw_pyramid** out, void* stream);
/* Waits for the device, then hands the levels' buffers to a per-device cache
 * that the next pyramid or rw_segment of the same sizes takes them from (at
 * most 8 GiB per device are kept, the rest is freed; an allocation that
 * fails empties the cache first; rw_ctx_destroy empties it). */
void rw_pyramid_free(rw_pyramid* p);
/* Level accessor: dims = {nx, ny, nz} of the level, *data = float [nz][ny][nx]
 * (device memory, or page-locked host memory for the host levels of
 * rw_pyramid_build_host). */
int rw_pyramid_level(const rw_pyramid* p, int level, int64_t dims[3], const float** data);

/* A label (Section IV-A): a point in full-resolution voxel units (voxel k
 * covers [k, k+1)) with a class.  Binary segmentation: label 1 foreground,
 * 0 background.  K classes: label in [0, K). */
typedef struct rw_seed {
    double x, y, z;
    int32_t label;
    int32_t reserved;        /* must be 0 */
} rw_seed;

/* Parameters of the hierarchical run.  Paper defaults: brick 32 (Section
 * IV-A), expand 1.25 (IV-B), t_hom 0.3, t_bin 0.01 (IV-D1), t_inc 0.01 (IV-E). */
typedef struct rw_params {
    double beta, eps;        /* edge weights exp(-beta dg^2) + eps */
    double tol;              /* per-box PCG relative residual */
    double expand;           /* e: box side floor(e * brick) */
    double t_hom, t_bin, t_inc;
    int32_t brick;           /* s >= 2 */
    int32_t max_iter;
    int32_t precision;       /* rw_precision of the box solves */
    int32_t n_classes;       /* K in [2, 4]; K - 1 right-hand sides are solved */
    int32_t prune_hom, prune_dt;  /* enable the hom / dt tests (dt only for K = 2) */
    int32_t refine_max;
    int32_t incremental;     /* runs with prev: bit 0 the node rule (else the dirty-brick rule),
                                bit 1 warm start from prev (Section IV-E); 0 by default */
    int32_t schedule;        /* rw_solve_params.schedule of the level solves (0 by default) */
    int32_t joint_classes;   /* K > 2 with MIXED or MIXED_REFINE: 0 (default) solves each of the
                                K - 1 right-hand sides of a box below the coarsest level as a box
                                of its own (one right-hand side, so the resident and split
                                kernels take it; the results are the same solves); 1 solves
                                them together (the weights shared, streaming kernels).  The
                                coarsest level's domain always solves them together. */
    int32_t host_levels;     /* the level maps of levels 0 .. host_levels - 1 in page-locked host
                                memory (out of core, with rw_pyramid_build_host): the same
                                kernels read and write them in place, and the maps equal a
                                device-memory run's bit for bit; 0 (default) to levels - 1 */
} rw_params;

void rw_params_default(rw_params* p);

/* Per-run counters (host struct). */
typedef struct rw_run_stats {
    int32_t levels;
    int32_t reserved;
    int64_t bricks[RW_MAX_LEVELS];      /* bricks of each level */
    int64_t computed[RW_MAX_LEVELS];    /* bricks reached (solved or reused) */
    int64_t solved[RW_MAX_LEVELS];      /* boxes solved in this run */
    int64_t prunable[RW_MAX_LEVELS];    /* reached bricks whose children were pruned */
    int64_t voxel_iters[RW_MAX_LEVELS]; /* sum over solved boxes of box voxels x PCG iterations (a box with
                                           several right-hand sides: the most any of them took) */
    int64_t box_voxels[RW_MAX_LEVELS];  /* sum of solved box voxels */
    int32_t max_iters[RW_MAX_LEVELS];
    int32_t not_converged[RW_MAX_LEVELS];  /* solved boxes with status MAX_ITER / STALLED / NONFINITE */
} rw_run_stats;

/*
 * Hierarchical segmentation, eqs. (1)-(3) with pruning (Section IV-D1) and,
 * when `prev` is given, incremental reuse (Section IV-E):
 *  - coarsest level: one domain, user seeds only (eq. 1);
 *  - every finer brick whose parent brick was reached and is not prunable:
 *    box = brick expanded by floor(e*s) - s voxels (low side half, rounded
 *    down), clipped to the volume; the outer voxel layer on faces inside the
 *    volume is seeded with the trilinear sample (cell centres, clamped) of the
 *    parent level map; user seeds (rasterised to floor(q / 2^level),
 *    conflicting voxels left unseeded) override; the rest starts from that
 *    sample (Section IV-D2); the solution's s^3 core is kept;
 *  - prunable = (hom or dt) and not cfl (a conflict voxel in the box);
 *  - regions not reached keep the upsampled parent map (ancestor fallback);
 *  - incremental, dirty-brick rule (default): a reached brick is solved
 *    again only if a new label lands in its box, it was not reached in
 *    `prev`, or the parent level map moved by >= t_inc over the parent voxels
 *    its box samples; otherwise its previous core values and prunable flag
 *    are reused;
 *  - incremental, node rule (params->incremental bit 0; the rule of Section
 *    IV-E): the coarsest level and every brick reached under a parent that
 *    was not kept are solved; a solved brick that `prev` also reached is
 *    kept (flag bit 4) when its new core is within t_inc of the previous one
 *    (max abs difference) and no seed conflict in its box involves a newly
 *    added label: it takes its previous core and prunable flag, and its
 *    reached descendants in `prev` are copied, not solved;
 *  - warm start (params->incremental bit 1): solved boxes start their
 *    unseeded voxels from prev's map of the same level (the border still
 *    samples the parent).
 * `seeds` is a host array.  The run is queued on `stream` but the call
 * synchronises with it once per level (it reads back brick flags and
 * solver statistics to plan the next level).  *out owns its device memory.
 */
int rw_segment(rw_ctx* ctx, const rw_pyramid* pyr, const rw_seed* seeds, int64_t n_seeds,
               const rw_params* params, const rw_result* prev, rw_result** out, void* stream);
/* Waits for the device, then hands the result's level maps and flag arrays
 * to the per-device cache described at rw_pyramid_free. */
void rw_result_free(rw_result* r);
int rw_result_stats(const rw_result* r, rw_run_stats* out);
/* Level map: dims = {nx, ny, nz}, nrhs = K - 1, *map = float [voxel][nrhs]
 * (probabilities of classes 1..K-1; class 0 is the complement), in device
 * memory, or page-locked host memory for levels below rw_params.host_levels. */
int rw_result_level(const rw_result* r, int level, int64_t dims[3], int* nrhs, const float** map);
/* Brick flags of a level: nb = bricks per axis {x, y, z}, *flags = dev uint8
 * [nbz][nby][nbx]; bit 0 reached, bit 1 prunable, bit 2 seed conflict in the
 * box, bit 3 solved in this run, bit 4 kept from prev by the node rule (with
 * its subtree). */
int rw_result_flags(const rw_result* r, int level, int64_t nb[3], const uint8_t** flags);
/* Copies of the data behind the accessors above into caller device buffers,
 * queued on `stream`: a level map (float [voxel][K-1]), a level's brick flags
 * (uint8 [bricks]), a pyramid level (float [voxel]). */
int rw_result_copy_level(rw_ctx* ctx, const rw_result* r, int level, float* dst, void* stream);
int rw_result_copy_flags(rw_ctx* ctx, const rw_result* r, int level, uint8_t* dst, void* stream);
int rw_pyramid_copy_level(rw_ctx* ctx, const rw_pyramid* p, int level, float* dst, void* stream);
/*
 * Dense output of a level: prob (dev float [voxels] or NULL) receives the
 * probability of class `cls` (0 = complement); labels (dev uint8 [voxels] or
 * NULL) the argmax class, lowest index on ties (Section III-B).
 */
int rw_result_materialize(rw_ctx* ctx, const rw_result* r, int level, int cls, float* prob,
                          uint8_t* labels, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RWSEG_H */
