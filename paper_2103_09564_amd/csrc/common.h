// Internal declarations shared by the HIP sources of librwseg (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "rwseg.h"

// Library context (opaque to callers).
struct rw_ctx {
    int device = 0;
    size_t lds_limit = 0;        // LDS bytes one workgroup may allocate
    std::string err;
    void* ws = nullptr;          // solver vector workspace
    size_t ws_bytes = 0;
    void* bricks = nullptr;      // device BrickDev list
    size_t bricks_bytes = 0;
    void* aux = nullptr;         // per-box state / partials
    size_t aux_bytes = 0;
    void* hws = nullptr;         // hierarchy: packed boxes (g, mask, x)
    size_t hws_bytes = 0;
    void* hgeo = nullptr;        // hierarchy: box geometry, seed entries, per-box scalars
    size_t hgeo_bytes = 0;
    void* wts = nullptr;         // weight segments of the streamed-weights resident kernel
    size_t wts_bytes = 0;
    int timing = 0;              // record phase events in rw_solve_bricks
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // start, after init, after pcg, end
    int ev_valid = 0;
    // two side streams (default priority) that run the streaming and the
    // LDS-resident PCG kernels of one call concurrently, and their events
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t join[3] = {nullptr, nullptr, nullptr};
    // timing of the two kernel groups of the main PCG phase: streaming
    // start/end, resident start/end; gev_used bit 0 / bit 1 when recorded
    hipEvent_t gev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int gev_used = 0;
    // solves of boxes held in host memory: two device staging sets, a
    // host-to-device and a device-to-host copy stream (default priority)
    // and their events
    void* ooc = nullptr;
    size_t ooc_bytes = 0;
    hipStream_t cs[2] = {nullptr, nullptr};
    hipEvent_t cev[10] = {};   // per lane: filled, solved, copied back (3 x 3); start
    // page-locked staging of the per-chunk box lists (so that their upload
    // does not block the host), the slot of the current chunk, and an event
    // after the last upload that read it
    void* pin = nullptr;
    size_t pin_bytes = 0;
    void* list_stage = nullptr;
    hipEvent_t pin_ev = nullptr;
    // contexts with their own workspaces and compute streams (default
    // priority) for the streamed solve's lanes beyond the first, so that
    // consecutive chunks overlap on the GPU (up to three lanes)
    rw_ctx* twin[2] = {nullptr, nullptr};
    hipStream_t tstream[2] = {nullptr, nullptr};
    // plan choices fixed by the streamed solve for every chunk, as the whole
    // box list would make them: window columns (0: from the batch) and the
    // unaligned plane-march variant
    int plan_cols = 0;
    int plan_unaligned = 0;
    // keep both streamed-weights launches on one stream (the streamed solve's
    // lanes already run two solves at once)
    int plan_no_third = 0;
    // keep the weights of small resident boxes in LDS (k_pcg_resw) instead of
    // registers (k_pcg_resr): a tuning choice
    int plan_no_regs = 0;
    // resident launches as persistent grids taking boxes from a ticket
    // counter instead of one workgroup per box: a tuning choice
    int plan_persist = 0;
    // solve boxes above 32768 voxels on the streaming kernels instead of
    // splitting them over two workgroups: a tuning choice
    int plan_no_split = 0;
    // this device's copy of the static scratch of rw_solve_bricks_noalloc
    void* scratch = nullptr;
    // autotuned schedules: per batch signature (box shapes, nrhs,
    // precision) the fastest candidate rw_autotune measured
    struct Tuned {
        uint64_t key;
        int32_t schedule, no_third, no_regs, persist, no_split;
        float ms;
    };
    std::vector<Tuned> tuned;
};

namespace rwk {

// Error helpers (capi.hip): record the message on ctx (or the thread's
// create-error slot when ctx is NULL) and return `code`.
int fail(rw_ctx* ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int hip_fail(rw_ctx* ctx, hipError_t e, const char* what);
// Grow a device buffer to at least `bytes` (contents are not kept; syncs `s` first).
hipError_t grow(rw_ctx* ctx, void** buf, size_t* have, size_t bytes, hipStream_t s);

// No C++ exception crosses the ABI: host allocation failures map to
// RW_E_NOMEM, anything else thrown to RW_E_INVAL.
template <typename F>
inline int guarded(rw_ctx* ctx, F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(ctx, RW_E_NOMEM, "host allocation failed");
    } catch (const std::exception& ex) {
        return fail(ctx, RW_E_INVAL, "%s", ex.what());
    } catch (...) {
        return fail(ctx, RW_E_INVAL, "unexpected exception");
    }
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Device-side box descriptor, in launch order (largest boxes first); `slot`
// is the caller's brick index (where its stats go).
struct BrickDev {
    int32_t nx, ny, nz, slot;
    int64_t off;
    int64_t woff;  // streamed-weights resident kernel: start of the box's weight segment
};

// Per-box scalars carried between the phases of one solve (launch order).
struct BoxState {
    double rz[3], rr[3], bb[3];   // r.z, ||r||^2, ||b||^2 per rhs
    double nU, nM;                // unknown / seeded voxel counts
    double rel, true_rel;         // recursive and FP64 true relative residual
    int32_t iters, status, refine_steps, refine_iters;
    int32_t active;               // next k_pcg runs on this machine
    int32_t pending;              // a correction was solved and is to be applied
    int32_t checked, check_ok;    // true_rel is current for x (no correction applied since), and its verdict
};

struct SolveArgs {
    const BrickDev* bricks;
    const float* g;
    const uint8_t* mask;
    float* x;              // caller x (interleaved nrhs)
    double* x64;           // caller x64 or workspace (may be null when unused)
    void* r;               // workspace vectors, element type float or double
    void* z;
    void* p0;
    void* p1;
    void* xt;              // FP64 path: solution accumulator (double); unused otherwise
    float* dcorr;          // FP32 correction accumulator
    rw_brick_stats* stats;
    BoxState* state;       // [n_bricks], workspace
    double beta, eps, tol, refine_tol, inner_tol, stall_ratio;
    int32_t max_iter, precision, refine_max, want_x64;
    int32_t schedule;      // streaming kernels: 1 two-sweep Jacobi-PCG, 2 single-reduction (Chronopoulos-Gear)
    void* dom;             // multi-workgroup domain solver: scalar state and ticket
    double* dom_part;      // its per-workgroup partial sums
    float* wts;            // streamed-weights resident kernel: per-box weight segments
    int32_t fused_init;    // main solve: the resident kernels compute their boxes' start state
    int32_t early_check;   // main solve: 1 + may_refine: each kernel group's boxes get their first
                           // true-residual check on the group's stream as soon as the group ends
    uint32_t* tickets;     // persistent resident launches: one counter per launch of the plan (or null)
    int32_t dom_sync_poll; // domain solver: read its done flag synchronously (no page-locked slots or
                           // events; the solve that allocates nothing)
};

struct AdjointArgs {
    const BrickDev* bricks;
    const float* g;
    const uint8_t* mask;
    const float* x;
    const float* dl_dx;
    float* dl_dg;
    float* lambda;         // caller buffer or workspace
    float* r;
    float* z;
    float* p0;
    float* p1;
    double* beta_part;     // [n_bricks] per-box partial of dl/dbeta, in launch order
    rw_brick_stats* stats;
    double beta, eps, tol;
    int32_t max_iter;
};

// How the PCG kernel is split: boxes [0, n_dom) of the launch list run the
// multi-workgroup domain solver one after another (host copies in `host`),
// [n_dom, n_big) the global-memory march, [n_big, n) the LDS plane march with
// `cols` columns per thread (planes up to plane_max(cols) voxels).  use = 0:
// no plane march (n_big = n).
struct PlanePlan {
    int use;
    int cols;
    int plane_aligned;  // every window-march box has CH % (nx*ny) == 0 (CH = cols * 512)
    int64_t n_big;
    int64_t n_dom;
    const BrickDev* host;
    // Resident PCG (one rhs, FP32): boxes [n_res, n), in up to five launches
    // (largest box first within each): p in LDS with the weights streamed
    // from a per-box segment (boxes above and up to 17408 voxels), p and the
    // weights in LDS (boxes the registers do not hold), then p in LDS and the
    // weights in registers for larger and for small boxes (launched apart so
    // that their LDS size lets several workgroups share a CU).  Without
    // resident boxes n_res = n.
    int64_t n_res;
    int n_rl;
    struct ResLaunch {
        int64_t b0, b1;       // launch-list range
        int64_t max_voxels;   // largest box of the range
        int64_t max_plane;    // widest nx*ny of the range
        int kind;             // 1: weights-in-LDS kernel, 2: streamed-weights kernel, 3: weights in registers
        int px;               // 32 when every box of the range has 32 x 32 planes, else 0
    } rl[6];
    int64_t wts_elems;        // floats of weight segments the kind-2 boxes need (BrickDev::woff)
    // when set, the streaming and resident groups run on these two streams
    // (forked from and joined back into the caller's stream)
    hipStream_t side[3];
    hipEvent_t fork, join[3];
    // resident launches as persistent grids (SolveArgs::tickets)
    int persist;
    // the second streamed-weights launch runs on side[2] (two such launches,
    // weights-in-LDS launches beside them, no streaming boxes)
    int third;
    // main-solve group timing events (start/end streaming, start/end
    // resident, start/end of the launch on side[2]) or null
    hipEvent_t* gev;
};

// Resident PCG (resident.hip).
constexpr int kResThreads = 512;
constexpr int kResMaxVptW = 20;   // weights-in-LDS kernel: boxes up to 10240 voxels
constexpr int kResMaxVptR = 18;   // weights-in-registers kernel: boxes up to 9216 voxels
constexpr int kResSmallVox = 5120;  // the small weights group: at most 10 voxels per thread
constexpr int kResSpanG0 = 17408;   // streamed-weights kernel: voxel slots of its launches for
constexpr int kResSpanG1 = 32768;   // boxes up to 32 x 32 x 17 and up to 32^3
bool resident_w_fits(const BrickDev& b, size_t lds_limit);    // weights-in-LDS kernel
bool resident_r_fits(const BrickDev& b, size_t lds_limit);    // weights-in-registers kernel
bool resident_g_fits(const BrickDev& b, size_t lds_limit);    // streamed-weights kernel
int64_t resident_g_span(int64_t max_voxels);                  // its voxel slots per workgroup
int64_t resident_g_elems(const BrickDev& b, int64_t span);    // a box's weight segment, in floats
// ticket: null for one workgroup per box, else a counter (cleared by the
// launch) for a persistent grid that takes the boxes in order.
hipError_t launch_resident(const SolveArgs& a, int64_t b0, int64_t b1, int64_t max_voxels, int64_t max_plane,
                           int kind, int px, float* xt, int corr, uint32_t* ticket, hipStream_t s);
// Split boxes (two workgroups per box, one per half along z): boxes above
// kResSpanG1 voxels whose halves hold at most kResSpanG1 and whose planes at
// most kPairMaxPlane.  Their weight area (BrickDev::woff) holds the two
// halves' segments and a mailbox of kPairMailboxElems floats.
constexpr int kPairMaxPlane = 2048;
constexpr int64_t kPairMailboxElems = (512 + 8 * (kPairMaxPlane + kResThreads)) / 4;
bool resident_split_fits(const BrickDev& b, size_t lds_limit);
int64_t resident_split_elems(const BrickDev& b);
hipError_t launch_split(const SolveArgs& a, int64_t b0, int64_t b1, int64_t max_plane, float* xt, int corr,
                        hipStream_t s);

size_t plane_lds_bytes(int nrhs, bool fp64, int cols);

// Multi-workgroup domain solver (domain.hip).  A box goes there when it has at
// least kDomMinVox voxels and a plane too wide for the LDS march, or at least
// kDomBigVox voxels; at most kDomMaxBoxes boxes per call (the largest), all of
// them in each launch.
constexpr int64_t kDomMinVox = int64_t(1) << 16;
constexpr int64_t kDomBigVox = int64_t(1) << 20;
constexpr int kDomMaxBoxes = 64;
size_t domain_scratch_bytes(int64_t n_dom);  // scalar state and partials of n_dom boxes
void domain_bind(SolveArgs& a, void* scratch);
// Frees the hierarchy's cached level buffers of device `dev` (hier.hip; the
// current device must be dev).
void pool_trim(int dev);
// The phases of the per-box solve for the domain boxes [0, nd) of the launch
// list (host: their host descriptors), each over many workgroups per box.
// domain_pcg runs PCG from the state the init or check left, into xt
// (corr = 0: main solve, 1: correction solve), until every box is done; it
// reads a done flag every few iterations.
template <typename T, int R>
hipError_t domain_init(const SolveArgs& a, int nd, const BrickDev* host, hipStream_t s);
template <typename T, int R, typename XT>
hipError_t domain_pcg(const SolveArgs& a, int nd, const BrickDev* host, XT* xt, int corr, hipStream_t s);
template <int R, bool kRefine64>
hipError_t domain_check(const SolveArgs& a, int nd, const BrickDev* host, int may_refine, hipStream_t s);
template <int R, bool kRefine64>
hipError_t domain_apply(const SolveArgs& a, int nd, const BrickDev* host, hipStream_t s);
template <int R>
hipError_t domain_copy64(const SolveArgs& a, int nd, const BrickDev* host, int to64, hipStream_t s);
template <int R>
hipError_t domain_finish64(const SolveArgs& a, int nd, const BrickDev* host, hipStream_t s);
int plane_cols(int max_plane);
int plane_max(int cols);

// Memory-system probes (probe.hip): kProbeBlocks workgroups of 256 threads
// (eight per CU on 256 CUs) stream float4 loads over a buffer `passes` times
// (one float per workgroup to part), `unroll` (4, 8 or 16) loads in flight
// per thread, or copy it.
constexpr int kProbeBlocks = 2048;
hipError_t launch_probe_read(const void* src, int64_t bytes, int passes, int unroll, float* part, hipStream_t s);
hipError_t launch_probe_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);

// Launchers (pcg.hip).  Return a hipError_t.
// ev: optional events {after init, after main PCG} recorded on s (may be null).
hipError_t launch_solve(const SolveArgs& a, int64_t n_bricks, int nrhs, bool fp64, const PlanePlan& pp,
                        hipStream_t s, hipEvent_t* ev = nullptr);
// The adjoint reuses the solve kernels: `sa` carries the PCG view (r, z, p, state) of the workspace.
hipError_t launch_adjoint(const AdjointArgs& a, const SolveArgs& sa, int64_t n_bricks, double* dl_dbeta,
                          const PlanePlan& pp, hipStream_t s);

}  // namespace rwk
