// C ABI of librwseg: contexts, argument validation, workspace, launches.
// No C++ exception crosses the ABI; every entry point returns an rw_error.

#include "common.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

// Device scratch of rw_solve_bricks_noalloc: a fixed array in the code
// object, so that call allocates nothing.  Each device holds its own copy
// (until the process ends) at its own address, which rw_ctx_create looks up
// once per device; in host code `scratch` is only a stand-in for that
// address and is never passed to a kernel or copy.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

thread_local std::string g_create_err;

// Address of `scratch` on each device, looked up by the first context
// created on that device.
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

int rwk::fail(rw_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_err = buf;
    return code;
}

int rwk::hip_fail(rw_ctx* ctx, hipError_t e, const char* what) {
    return fail(ctx, e == hipErrorOutOfMemory ? RW_E_NOMEM : RW_E_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

// Grow a device buffer to at least `bytes` (contents are not kept).
hipError_t rwk::grow(rw_ctx* ctx, void** buf, size_t* have, size_t bytes, hipStream_t s) {
    if (*have >= bytes) return hipSuccess;
    if (*buf) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        e = hipFree(*buf);
        if (e != hipSuccess) return e;
        *buf = nullptr;
        *have = 0;
    }
    size_t want = bytes + bytes / 8;
    hipError_t e = hipMalloc(buf, want);
    if (e != hipSuccess) {
        *buf = nullptr;
        return e;
    }
    *have = want;
    return hipSuccess;
}

namespace {

using rwk::DevGuard;
using rwk::fail;
using rwk::grow;
using rwk::guarded;
using rwk::hip_fail;

int check_params(rw_ctx* ctx, const rw_solve_params* p) {
    if (!p) return fail(ctx, RW_E_INVAL, "params is NULL");
    if (!std::isfinite(p->beta) || p->beta < 0) return fail(ctx, RW_E_INVAL, "beta must be finite and >= 0");
    if (!std::isfinite(p->eps) || p->eps < 0) return fail(ctx, RW_E_INVAL, "eps must be finite and >= 0");
    if (!std::isfinite(p->tol) || p->tol < 0) return fail(ctx, RW_E_INVAL, "tol must be finite and >= 0");
    if (p->max_iter < 0) return fail(ctx, RW_E_INVAL, "max_iter must be >= 0");
    if (p->precision < RW_PREC_FP64 || p->precision > RW_PREC_MIXED_REFINE)
        return fail(ctx, RW_E_INVAL, "unknown precision %d", p->precision);
    if (p->nrhs < 1 || p->nrhs > 3) return fail(ctx, RW_E_INVAL, "nrhs must be 1, 2 or 3 (got %d)", p->nrhs);
    if (p->refine_max < 0 || p->refine_max > 64) return fail(ctx, RW_E_INVAL, "refine_max must be in [0, 64]");
    if (!std::isfinite(p->refine_tol) || p->refine_tol < 0) return fail(ctx, RW_E_INVAL, "refine_tol must be >= 0");
    if (!std::isfinite(p->inner_tol) || p->inner_tol < 0) return fail(ctx, RW_E_INVAL, "inner_tol must be >= 0");
    if (!std::isfinite(p->stall_ratio) || p->stall_ratio < 1) return fail(ctx, RW_E_INVAL, "stall_ratio must be >= 1");
    if (p->schedule < 0 || p->schedule > RW_SCHED_TUNED)
        return fail(ctx, RW_E_INVAL, "schedule must be 0, 1, 2, 3, 4 or RW_SCHED_TUNED (5)");
    return RW_OK;
}

// Schedule of the streaming kernels for a requested schedule (0, 1 and 4:
// two sweeps, 2 and 3: one sweep; 0, 3 and 4 also use the resident kernels).
int stream_schedule(int requested) { return requested == 2 || requested == 3 ? 2 : 1; }

// Signature of a batch for the tuned-schedule table: FNV-1a over the sorted
// (nx, ny, nz, count) histogram of its box shapes, nrhs and precision.
uint64_t batch_key(const rw_solve_params& p, int64_t n, const rw_brick* b) {
    std::vector<std::array<int32_t, 3>> sh((size_t)n);
    for (int64_t i = 0; i < n; ++i) sh[(size_t)i] = {b[i].nx, b[i].ny, b[i].nz};
    std::sort(sh.begin(), sh.end());
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    for (size_t i = 0; i < sh.size();) {
        size_t j = i;
        while (j < sh.size() && sh[j] == sh[i]) ++j;
        mix((uint64_t)(uint32_t)sh[i][0] | ((uint64_t)(uint32_t)sh[i][1] << 32));
        mix((uint64_t)(uint32_t)sh[i][2] | ((uint64_t)(j - i) << 32));
        i = j;
    }
    mix((uint64_t)p.nrhs | ((uint64_t)p.precision << 8));
    return h;
}

// The schedule a call runs: a tuned request takes the ctx's measured winner
// for its batch (the library's default, 0, when the batch was not tuned);
// *no_third is that winner's stream choice.
// Plan choices a schedule entry carries beside the schedule number.
struct PlanChoice {
    int no_third = 0;   // both streamed-weights launches on one stream
    int no_regs = 0;    // small resident boxes keep their weights in LDS
    int persist = 0;    // resident launches as persistent grids
    int no_split = 0;   // boxes above 32768 voxels stream instead of splitting
};

rw_solve_params resolve_schedule(const rw_ctx* ctx, const rw_solve_params& p, int64_t n, const rw_brick* b,
                                 PlanChoice* pc) {
    rw_solve_params q = p;
    pc->no_third = ctx->plan_no_third;
    pc->no_regs = ctx->plan_no_regs;
    pc->persist = ctx->plan_persist;
    pc->no_split = ctx->plan_no_split;
    if (p.schedule != RW_SCHED_TUNED) return q;
    q.schedule = 0;
    if (ctx->tuned.empty() || n == 0) return q;
    const uint64_t key = batch_key(p, n, b);
    for (const rw_ctx::Tuned& t : ctx->tuned)
        if (t.key == key) {
            q.schedule = t.schedule;
            pc->no_third = pc->no_third || t.no_third;
            pc->no_regs = pc->no_regs || t.no_regs;
            pc->persist = pc->persist || t.persist;
            pc->no_split = pc->no_split || t.no_split;
        }
    return q;
}

// Sets the context's plan choices for the duration of a call.
struct PlanScope {
    rw_ctx* ctx;
    int saved_third, saved_regs, saved_persist, saved_split;
    PlanScope(rw_ctx* c, const PlanChoice& pc)
        : ctx(c), saved_third(c->plan_no_third), saved_regs(c->plan_no_regs), saved_persist(c->plan_persist),
          saved_split(c->plan_no_split) {
        c->plan_no_third = pc.no_third;
        c->plan_no_regs = pc.no_regs;
        c->plan_persist = pc.persist;
        c->plan_no_split = pc.no_split;
    }
    ~PlanScope() {
        ctx->plan_no_third = saved_third;
        ctx->plan_no_regs = saved_regs;
        ctx->plan_persist = saved_persist;
        ctx->plan_no_split = saved_split;
    }
};

// Validate host descriptors and build the launch list (largest box first).
int build_list(rw_ctx* ctx, int64_t n, const rw_brick* bricks, int64_t n_voxels,
               std::vector<rwk::BrickDev>* out) {
    if (n < 0) return fail(ctx, RW_E_INVAL, "n_bricks < 0");
    if (n > 0 && !bricks) return fail(ctx, RW_E_INVAL, "bricks is NULL");
    if (n > (int64_t)0x7fffffff) return fail(ctx, RW_E_INVAL, "too many bricks (max 2^31-1)");
    if (n_voxels < 0) return fail(ctx, RW_E_INVAL, "n_voxels < 0");
    std::vector<std::pair<int64_t, int64_t>> spans;
    spans.reserve((size_t)n);
    out->resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const rw_brick& b = bricks[i];
        if (b.nx < 1 || b.ny < 1 || b.nz < 1)
            return fail(ctx, RW_E_INVAL, "brick %lld: dims %d x %d x %d must be >= 1", (long long)i, b.nx, b.ny, b.nz);
        if (b.reserved != 0) return fail(ctx, RW_E_INVAL, "brick %lld: reserved field must be 0", (long long)i);
        const int64_t nxy = (int64_t)b.nx * b.ny;
        if (nxy > (int64_t)0x7fffffff) return fail(ctx, RW_E_INVAL, "brick %lld: nx*ny too large", (long long)i);
        const int64_t vox = nxy * b.nz;
        if (b.offset < 0 || vox > n_voxels || b.offset > n_voxels - vox)
            return fail(ctx, RW_E_INVAL, "brick %lld: [%lld, %lld) outside the %lld-voxel buffers", (long long)i,
                        (long long)b.offset, (long long)(b.offset + vox), (long long)n_voxels);
        (*out)[(size_t)i] = rwk::BrickDev{b.nx, b.ny, b.nz, (int32_t)i, b.offset};
        spans.emplace_back(b.offset, b.offset + vox);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return fail(ctx, RW_E_INVAL, "bricks overlap in the voxel buffers");
    std::stable_sort(out->begin(), out->end(), [](const rwk::BrickDev& a, const rwk::BrickDev& b) {
        return (int64_t)a.nx * a.ny * a.nz > (int64_t)b.nx * b.ny * b.nz;
    });
    return RW_OK;
}

// Choose the PCG kernel split for this batch and move the boxes that are too
// wide for the LDS plane march to the front of the (largest-first) list.
// The few largest boxes (single domains) go to the multi-workgroup solver in
// front of the list; boxes that fit in one CU's LDS (one rhs, FP32, streaming
// schedule not forced) go to the resident kernel at the end.
// Window columns of a batch: from its widest plane that the window holds.
int plan_cols_of(const rw_ctx* ctx, const rw_brick* b, int64_t n, int nrhs, bool fp64) {
    int widest = 0;
    for (int64_t i = 0; i < n; ++i)
        if (b[i].nx * b[i].ny <= rwk::plane_max(4)) widest = std::max(widest, b[i].nx * b[i].ny);
    int cols = rwk::plane_cols(widest);
    if (rwk::plane_lds_bytes(nrhs, fp64, cols) > ctx->lds_limit) cols = 2;
    return cols;
}

// Kernel group of one box (the domain cap aside): 0 domain solver, 1 global
// march, 2 plane march, 3 and 4 resident (p in LDS, weights streamed) above
// and up to kResSpanG0 voxels, 5 resident (weights in LDS), 6 and 7 resident
// (weights in registers) above and up to kResSmallVox voxels, 8 split
// (two workgroups per box).
int group_of(const rw_ctx* ctx, int nx, int ny, int nz, int lim, bool res_ok, bool prefer_g, bool dom_left) {
    rwk::BrickDev b{};
    b.nx = nx;
    b.ny = ny;
    b.nz = nz;
    const int64_t nxy = (int64_t)nx * ny, vox = nxy * nz;
    const bool wide = nxy > lim;
    // (the domain kernels index voxels with 32-bit integers)
    const bool dom = vox < (int64_t(1) << 31) && (vox >= rwk::kDomBigVox || (wide && vox >= rwk::kDomMinVox));
    if (dom && dom_left) return 0;
    if (res_ok && prefer_g && rwk::resident_g_fits(b, ctx->lds_limit)) return vox > rwk::kResSpanG0 ? 3 : 4;
    if (res_ok && !ctx->plan_no_regs && rwk::resident_r_fits(b, ctx->lds_limit))
        return vox <= rwk::kResSmallVox ? 7 : 6;
    if (res_ok && rwk::resident_w_fits(b, ctx->lds_limit)) return 5;
    if (res_ok && rwk::resident_g_fits(b, ctx->lds_limit)) return vox > rwk::kResSpanG0 ? 3 : 4;
    if (res_ok && !ctx->plan_no_split && rwk::resident_split_fits(b, ctx->lds_limit)) return 8;
    return wide ? 1 : 2;
}

bool resident_ok(int nrhs, bool fp64, int schedule) {
    return nrhs == 1 && !fp64 && (schedule == 0 || schedule == 3 || schedule == 4);
}

rwk::PlanePlan plan_planes(const rw_ctx* ctx, std::vector<rwk::BrickDev>* list, int nrhs, bool fp64,
                           int schedule) {
    const int64_t n = (int64_t)list->size();
    rwk::PlanePlan pp{};
    pp.cols = 2;
    pp.n_big = pp.n_res = n;
    const bool res_ok = resident_ok(nrhs, fp64, schedule);
    const bool prefer_g = schedule == 4;
    int cols = ctx->plan_cols;
    if (cols == 0) {
        std::vector<rw_brick> hb(list->size());
        for (size_t i = 0; i < list->size(); ++i) hb[i] = rw_brick{(*list)[i].nx, (*list)[i].ny, (*list)[i].nz, 0, 0};
        cols = plan_cols_of(ctx, hb.data(), n, nrhs, fp64);
    }
    const bool use = rwk::plane_lds_bytes(nrhs, fp64, cols) <= ctx->lds_limit;
    const int lim = use ? rwk::plane_max(cols) : 0;
    // the list is largest-first
    std::vector<uint8_t> grp(list->size());
    int n_dom = 0;
    for (size_t i = 0; i < list->size(); ++i) {
        const rwk::BrickDev& b = (*list)[i];
        grp[i] = (uint8_t)group_of(ctx, b.nx, b.ny, b.nz, lim, res_ok, prefer_g, n_dom < rwk::kDomMaxBoxes);
        if (grp[i] == 0) ++n_dom;
    }
    std::vector<size_t> idx(list->size());
    std::iota(idx.begin(), idx.end(), size_t(0));
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return grp[a] < grp[b]; });
    std::vector<rwk::BrickDev> sorted(list->size());
    int64_t cnt[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t i = 0; i < idx.size(); ++i) {
        sorted[i] = (*list)[idx[i]];
        cnt[grp[idx[i]]] += 1;
    }
    list->swap(sorted);
    pp.use = use ? 1 : 0;
    pp.cols = cols;
    pp.n_dom = n_dom;
    pp.n_big = cnt[0] + cnt[1];
    pp.n_res = pp.n_big + cnt[2];
    pp.n_rl = 0;
    int64_t b0 = pp.n_res;
    pp.wts_elems = 0;
    // (the split boxes sort last; their launch comes first, with the other
    // streamed-weights launches)
    for (int gi = 3; gi <= 8; ++gi) {
        if (cnt[gi] == 0) continue;
        rwk::PlanePlan::ResLaunch& L = pp.rl[pp.n_rl++];
        L.b0 = b0;
        L.b1 = b0 + cnt[gi];
        L.kind = gi <= 4 ? 2 : gi == 5 ? 1 : gi == 8 ? 4 : 3;
        L.max_voxels = 0;
        L.max_plane = 0;
        L.px = 32;
        for (int64_t i = L.b0; i < L.b1; ++i) {
            const auto& b = (*list)[(size_t)i];
            L.max_voxels = std::max<int64_t>(L.max_voxels, (int64_t)b.nx * b.ny * b.nz);
            L.max_plane = std::max<int64_t>(L.max_plane, (int64_t)b.nx * b.ny);
            if (b.nx != 32 || b.ny != 32) L.px = 0;
        }
        if (L.kind == 2) {
            const int64_t span = rwk::resident_g_span(L.max_voxels);
            for (int64_t i = L.b0; i < L.b1; ++i) {
                auto& b = (*list)[(size_t)i];
                b.woff = pp.wts_elems;
                pp.wts_elems += rwk::resident_g_elems(b, span);
            }
        }
        if (L.kind == 4) {
            for (int64_t i = L.b0; i < L.b1; ++i) {
                auto& b = (*list)[(size_t)i];
                b.woff = pp.wts_elems;
                pp.wts_elems += rwk::resident_split_elems(b);
            }
        }
        b0 = L.b1;
    }
    pp.persist = ctx->plan_persist;
    pp.plane_aligned = ctx->plan_unaligned ? 0 : 1;
    for (int64_t i = pp.n_big; i < pp.n_res; ++i) {
        const auto& b = (*list)[(size_t)i];
        if ((int64_t)rwk::plane_max(cols) % ((int64_t)b.nx * b.ny) != 0) pp.plane_aligned = 0;
    }
    pp.host = list->data();
    return pp;
}

// Side streams and events for concurrent kernel groups (created once).
int attach_side_streams(rw_ctx* ctx, rwk::PlanePlan* pp) {
    if (!ctx->side[0]) {
        for (int i = 0; i < 3; ++i) {
            hipError_t e = hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join[i], hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(ctx, e, "creating side streams");
        }
        hipError_t e = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(ctx, e, "creating side-stream events");
    }
    pp->side[0] = ctx->side[0];
    pp->side[1] = ctx->side[1];
    pp->side[2] = ctx->side[2];
    int n_g = 0, n_w = 0, n_s = 0;
    for (int i = 0; i < pp->n_rl; ++i) (pp->rl[i].kind == 2 ? n_g : pp->rl[i].kind == 4 ? n_s : n_w) += 1;
    pp->third = n_g == 2 && n_s == 0 && n_w > 0 && pp->n_res == pp->n_dom && !ctx->plan_no_third ? 1 : 0;
    pp->fork = ctx->fork;
    pp->join[0] = ctx->join[0];
    pp->join[1] = ctx->join[1];
    pp->join[2] = ctx->join[2];
    return RW_OK;
}

// Weight segments of the streamed-weights resident boxes (none: null).
int bind_weights(rw_ctx* ctx, const rwk::PlanePlan& pp, rwk::SolveArgs* a, hipStream_t s) {
    a->wts = nullptr;
    if (pp.wts_elems == 0) return RW_OK;
    hipError_t e = grow(ctx, &ctx->wts, &ctx->wts_bytes, (size_t)pp.wts_elems * sizeof(float), s);
    if (e != hipSuccess) return hip_fail(ctx, e, "allocating weight segments");
    a->wts = (float*)ctx->wts;
    return RW_OK;
}

int upload_list(rw_ctx* ctx, const std::vector<rwk::BrickDev>& list, hipStream_t s) {
    size_t bytes = std::max<size_t>(list.size() * sizeof(rwk::BrickDev), 64);
    hipError_t e = grow(ctx, &ctx->bricks, &ctx->bricks_bytes, bytes, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "allocating brick list");
    if (!list.empty()) {
        // from a page-locked slot when the caller set one (the copy then
        // does not wait for the stream), else from the vector itself
        const void* src = list.data();
        if (ctx->list_stage) {
            std::memcpy(ctx->list_stage, list.data(), list.size() * sizeof(rwk::BrickDev));
            src = ctx->list_stage;
        }
        e = hipMemcpyAsync(ctx->bricks, src, list.size() * sizeof(rwk::BrickDev), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "uploading brick list");
    }
    return RW_OK;
}

// Workspace of one rw_solve_bricks call: the CG vectors (r, z, p0, p1 of
// the compute type, the FP32 correction buffer, an FP64 solution buffer when
// the caller gave none), the per-box state and domain-solver scratch, the
// device box list and the weight segments of the streamed-weights boxes.
// Offsets are from the start of each buffer; every part is 256-byte aligned.
struct SolveLayout {
    size_t nv, es, off_dcorr, off_x64, ws_bytes;   // vector workspace
    size_t state_bytes, tickets_off, aux_bytes;    // BoxState [n], domain scratch, launch tickets
    size_t list_bytes, wts_bytes;                  // BrickDev [n], weight segments
};

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// Ticket counters of the persistent resident launches (one per launch of a
// plan, at most six).
constexpr size_t kTicketBytes = 256;

SolveLayout solve_layout(const rw_solve_params& p, int64_t n_bricks, int64_t n_voxels, const double* x64,
                         const rwk::PlanePlan& pp) {
    SolveLayout L{};
    const bool fp64 = p.precision == RW_PREC_FP64;
    const bool need_x64 = fp64 || p.precision == RW_PREC_MIXED_REFINE;
    L.nv = (size_t)n_voxels * (size_t)p.nrhs;
    L.es = fp64 ? sizeof(double) : sizeof(float);
    size_t bytes = 4 * L.nv * L.es;
    L.off_dcorr = bytes;
    if (!fp64) bytes += L.nv * sizeof(float);
    L.off_x64 = up256(bytes);
    if (need_x64 && !x64) bytes = L.off_x64 + L.nv * sizeof(double);
    L.ws_bytes = up256(std::max<size_t>(bytes, 256));
    L.state_bytes = up256((size_t)n_bricks * sizeof(rwk::BoxState));
    L.tickets_off = up256(L.state_bytes + rwk::domain_scratch_bytes(pp.n_dom));
    L.aux_bytes = L.tickets_off + kTicketBytes;
    L.list_bytes = up256(std::max<size_t>((size_t)n_bricks * sizeof(rwk::BrickDev), 64));
    L.wts_bytes = up256((size_t)pp.wts_elems * sizeof(float));
    return L;
}

// Where a solve's workspace comes from.  Default: the context's buffers,
// grown on demand.  noalloc: the device's static scratch array (no
// allocation, no side stream or event; all kernels on `stream`).  ext: a
// buffer laid out by solve_layout that already holds the box list (a
// captured graph's own workspace); nothing is allocated or copied.
struct SolveMode {
    bool noalloc = false;
    char* ext = nullptr;
    size_t ext_bytes = 0;
};

size_t layout_total(const SolveLayout& L) { return L.ws_bytes + L.aux_bytes + L.list_bytes + L.wts_bytes; }

// rw_solve_bricks, rw_solve_bricks_noalloc and the captured graph's solve.
int solve_bricks_impl(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                      int64_t n_voxels, const float* g, const uint8_t* mask, float* x, double* x64,
                      rw_brick_stats* stats, void* stream, const SolveMode& mode) {
    const bool noalloc = mode.noalloc;
    int rc = check_params(ctx, params);
    if (rc) return rc;
    std::vector<rwk::BrickDev> list;
    rc = build_list(ctx, n_bricks, bricks, n_voxels, &list);
    if (rc) return rc;
    if (n_bricks == 0) return RW_OK;
    if (!g || !mask || !x) return fail(ctx, RW_E_INVAL, "g, mask and x must be non-NULL");
    PlanChoice pc;
    const rw_solve_params p = resolve_schedule(ctx, *params, n_bricks, bricks, &pc);
    PlanScope pls(ctx, pc);
    const int R = p.nrhs;
    const bool fp64 = p.precision == RW_PREC_FP64;
    const bool need_x64 = fp64 || p.precision == RW_PREC_MIXED_REFINE;
    hipStream_t s = (hipStream_t)stream;
    DevGuard dg(ctx->device);

    rwk::PlanePlan pp = plan_planes(ctx, &list, R, fp64, p.schedule);
    const SolveLayout L = solve_layout(p, n_bricks, n_voxels, x64, pp);
    char *w, *aux, *blist;
    float* wts = nullptr;
    if (mode.ext) {
        if (layout_total(L) > mode.ext_bytes) return fail(ctx, RW_E_INVAL, "workspace smaller than the batch's layout");
        w = mode.ext;
        aux = w + L.ws_bytes;
        blist = aux + L.aux_bytes;
        if (pp.wts_elems) wts = (float*)(blist + L.list_bytes);
        rc = attach_side_streams(ctx, &pp);
        if (rc) return rc;
    } else if (noalloc) {
        const size_t total = L.ws_bytes + L.aux_bytes + L.list_bytes + L.wts_bytes;
        if (total > kScratchBytes)
            return fail(ctx, RW_E_INVAL,
                        "rw_solve_bricks_noalloc: these boxes need %zu bytes of workspace, more than the "
                        "%zu-byte static scratch",
                        total, (size_t)kScratchBytes);
        if (!ctx->scratch) return fail(ctx, RW_E_HIP, "no static scratch address for device %d", ctx->device);
        char* base = (char*)ctx->scratch;
        w = base;
        aux = w + L.ws_bytes;
        blist = aux + L.aux_bytes;
        if (pp.wts_elems) wts = (float*)(blist + L.list_bytes);
        pp.side[0] = pp.side[1] = pp.side[2] = nullptr;  // one stream: the caller's
        pp.third = 0;
        pp.gev = nullptr;
        if (!list.empty()) {
            hipError_t e = hipMemcpyAsync(blist, list.data(), list.size() * sizeof(rwk::BrickDev),
                                          hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(ctx, e, "uploading brick list");
        }
    } else {
        hipError_t e = grow(ctx, &ctx->ws, &ctx->ws_bytes, L.ws_bytes, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "allocating solver workspace");
        e = grow(ctx, &ctx->aux, &ctx->aux_bytes, L.aux_bytes, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "allocating per-box state");
        rc = attach_side_streams(ctx, &pp);
        if (rc) return rc;
        rc = upload_list(ctx, list, s);
        if (rc) return rc;
        if (pp.wts_elems) {
            e = grow(ctx, &ctx->wts, &ctx->wts_bytes, L.wts_bytes, s);
            if (e != hipSuccess) return hip_fail(ctx, e, "allocating weight segments");
            wts = (float*)ctx->wts;
        }
        w = (char*)ctx->ws;
        aux = (char*)ctx->aux;
        blist = (char*)ctx->bricks;
    }

    const size_t nv = L.nv, es = L.es;
    rwk::SolveArgs a{};
    a.bricks = (const rwk::BrickDev*)blist;
    a.g = g;
    a.mask = mask;
    a.x = x;
    a.r = w;
    a.z = w + nv * es;
    a.p0 = w + 2 * nv * es;
    a.p1 = w + 3 * nv * es;
    a.dcorr = fp64 ? nullptr : (float*)(w + L.off_dcorr);
    double* x64buf = x64 ? x64 : (need_x64 ? (double*)(w + L.off_x64) : nullptr);
    a.x64 = x64buf;
    a.xt = x64buf;
    a.want_x64 = x64 ? 1 : 0;
    a.stats = stats;
    a.state = (rwk::BoxState*)aux;
    a.beta = p.beta;
    a.eps = p.eps;
    a.tol = p.tol;
    a.refine_tol = p.refine_tol;
    a.inner_tol = p.inner_tol;
    a.max_iter = p.max_iter;
    a.precision = p.precision;
    a.refine_max = p.refine_max;
    a.stall_ratio = p.stall_ratio;
    a.schedule = stream_schedule(p.schedule);
    rwk::domain_bind(a, aux + L.state_bytes);
    a.tickets = (uint32_t*)(aux + L.tickets_off);
    a.dom_sync_poll = noalloc ? 1 : 0;
    a.wts = wts;
    hipError_t e;
    hipEvent_t* ev = nullptr;
    const bool timed = ctx->timing && !noalloc && !mode.ext;
    if (timed) {
        for (int i = 0; i < 4; ++i)
            if (!ctx->ev[i]) {
                e = hipEventCreate(&ctx->ev[i]);
                if (e != hipSuccess) return hip_fail(ctx, e, "creating timing events");
            }
        for (int i = 0; i < 6; ++i)
            if (!ctx->gev[i]) {
                e = hipEventCreate(&ctx->gev[i]);
                if (e != hipSuccess) return hip_fail(ctx, e, "creating timing events");
            }
        e = hipEventRecord(ctx->ev[0], s);
        if (e != hipSuccess) return hip_fail(ctx, e, "recording timing event");
        ev = &ctx->ev[1];
        pp.gev = ctx->gev;
        // bit 0: streaming kernels or streamed-weights resident launches
        // (one stream), bit 1: the other resident launches
        bool any_g = false, any_lds = false;
        for (int i = 0; i < pp.n_rl; ++i) (pp.rl[i].kind == 2 || pp.rl[i].kind == 4 ? any_g : any_lds) = true;
        const bool res_path = R == 1 && !fp64;
        ctx->gev_used = (pp.n_res > pp.n_dom || (res_path && any_g) ? 1 : 0) | (res_path && any_lds ? 2 : 0) |
                        (res_path && pp.third ? 4 : 0);
    }
    e = rwk::launch_solve(a, n_bricks, R, fp64, pp, s, ev);
    if (e != hipSuccess) return hip_fail(ctx, e, "launching solve kernel");
    if (timed) {
        e = hipEventRecord(ctx->ev[3], s);
        if (e != hipSuccess) return hip_fail(ctx, e, "recording timing event");
        ctx->ev_valid = 1;
    }
    return RW_OK;
}

}  // namespace

extern "C" {

void rw_solve_params_default(rw_solve_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->beta = 128.0;
    p->eps = 1e-6;
    p->tol = 1e-6;
    p->max_iter = 5000;
    p->precision = RW_PREC_MIXED;
    p->nrhs = 1;
    p->refine_max = 1;
    p->refine_tol = 1e-13;
    p->inner_tol = 1e-4;
    p->stall_ratio = 10.0;
}

int rw_version(void) { return RW_VERSION; }

int rw_ctx_create(int hip_device, rw_ctx** out) {
    if (!out) return fail(nullptr, RW_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(nullptr, RW_E_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= n)
        return fail(nullptr, RW_E_INVAL, "device %d out of range (have %d)", hip_device, n);
    rw_ctx* c = new (std::nothrow) rw_ctx();
    if (!c) return fail(nullptr, RW_E_NOMEM, "host allocation failed");
    c->device = hip_device;
    int lds = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device);
    c->lds_limit = e == hipSuccess && lds > 0 ? (size_t)lds : 64 * 1024;
    // the device's copy of the no-allocation scratch, looked up once per
    // device with that device current
    if (hip_device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[hip_device]) {
            DevGuard dg(hip_device);
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                delete c;
                return fail(nullptr, RW_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            }
            g_scratch_ptr[hip_device] = ptr;
        }
        c->scratch = g_scratch_ptr[hip_device];
    }
    *out = c;
    return RW_OK;
}

void rw_ctx_destroy(rw_ctx* ctx) {
    if (!ctx) return;
    DevGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    rwk::pool_trim(ctx->device);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->bricks) (void)hipFree(ctx->bricks);
    if (ctx->aux) (void)hipFree(ctx->aux);
    if (ctx->hws) (void)hipFree(ctx->hws);
    if (ctx->hgeo) (void)hipFree(ctx->hgeo);
    if (ctx->wts) (void)hipFree(ctx->wts);
    if (ctx->ooc) (void)hipFree(ctx->ooc);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    if (ctx->pin_ev) (void)hipEventDestroy(ctx->pin_ev);
    for (int i = 0; i < 2; ++i) {
        if (ctx->tstream[i]) (void)hipStreamDestroy(ctx->tstream[i]);
        rw_ctx_destroy(ctx->twin[i]);
    }
    for (hipStream_t& c : ctx->cs)
        if (c) (void)hipStreamDestroy(c);
    for (hipEvent_t& e : ctx->cev)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i < 4; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    for (int i = 0; i < 6; ++i)
        if (ctx->gev[i]) (void)hipEventDestroy(ctx->gev[i]);
    for (int i = 0; i < 3; ++i) {
        if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
        if (ctx->join[i]) (void)hipEventDestroy(ctx->join[i]);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    delete ctx;
}

const char* rw_last_error(const rw_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int rw_set_plan_choices(rw_ctx* ctx, int third_stream, int weights_in_registers, int persistent) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    if ((third_stream | weights_in_registers | persistent) & ~1)
        return fail(ctx, RW_E_INVAL, "plan choices are 0 or 1");
    ctx->plan_no_third = third_stream ? 0 : 1;
    ctx->plan_no_regs = weights_in_registers ? 0 : 1;
    ctx->plan_persist = persistent;
    return RW_OK;
}

int rw_set_split_boxes(rw_ctx* ctx, int enable) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    if (enable & ~1) return fail(ctx, RW_E_INVAL, "enable is 0 or 1");
    ctx->plan_no_split = enable ? 0 : 1;
    return RW_OK;
}

int rw_set_timing(rw_ctx* ctx, int enable) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->timing = enable ? 1 : 0;
    ctx->ev_valid = 0;
    return RW_OK;
}

int rw_last_timing(rw_ctx* ctx, rw_timing* out) {
    if (!ctx || !out) return fail(ctx, RW_E_INVAL, "ctx and out must be non-NULL");
    if (!ctx->ev_valid) return fail(ctx, RW_E_INVAL, "no timed solve recorded (enable with rw_set_timing)");
    DevGuard dg(ctx->device);
    hipError_t e = hipEventSynchronize(ctx->ev[3]);
    float t[3] = {0, 0, 0};
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventElapsedTime(&t[i], ctx->ev[i], ctx->ev[i + 1]);
    if (e != hipSuccess) return hip_fail(ctx, e, "reading timing events");
    out->init_ms = t[0];
    out->pcg_ms = t[1];
    out->finish_ms = t[2];
    out->total_ms = t[0] + t[1] + t[2];
    out->stream_ms = out->resident_ms = out->stream2_ms = 0.0f;
    float* dst[3] = {&out->stream_ms, &out->resident_ms, &out->stream2_ms};
    for (int gidx = 0; gidx < 3 && e == hipSuccess; ++gidx)
        if (ctx->gev_used & (1 << gidx)) e = hipEventElapsedTime(dst[gidx], ctx->gev[2 * gidx], ctx->gev[2 * gidx + 1]);
    if (e != hipSuccess) return hip_fail(ctx, e, "reading timing events");
    return RW_OK;
}

int rw_validate_solve(const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                      int64_t n_voxels) {
    return guarded(nullptr, [&]() -> int {
    g_create_err.clear();
    int rc = check_params(nullptr, params);
    if (rc) return rc;
    std::vector<rwk::BrickDev> list;
    return build_list(nullptr, n_bricks, bricks, n_voxels, &list);
    });
}

int rw_solve_plan(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                  int64_t n_voxels, int32_t* path) {
    return guarded(ctx, [&]() -> int {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    int rc = check_params(ctx, params);
    if (rc) return rc;
    std::vector<rwk::BrickDev> list;
    rc = build_list(ctx, n_bricks, bricks, n_voxels, &list);
    if (rc) return rc;
    if (n_bricks > 0 && !path) return fail(ctx, RW_E_INVAL, "path is NULL");
    PlanChoice pc;
    const rw_solve_params pe = resolve_schedule(ctx, *params, n_bricks, bricks, &pc);
    PlanScope pls(ctx, pc);
    const rwk::PlanePlan pp = plan_planes(ctx, &list, pe.nrhs, pe.precision == RW_PREC_FP64, pe.schedule);
    for (int64_t i = 0; i < n_bricks; ++i) {
        const int32_t slot = list[(size_t)i].slot;
        path[slot] = i < pp.n_dom ? RW_PATH_DOMAIN
                     : i < pp.n_big ? RW_PATH_STREAM_GLOBAL
                     : i < pp.n_res ? RW_PATH_STREAM
                                      : RW_PATH_RESIDENT;
        for (int k = 0; k < pp.n_rl; ++k)
            if (i >= pp.rl[k].b0 && i < pp.rl[k].b1 && (pp.rl[k].kind == 2 || pp.rl[k].kind == 4))
                path[slot] = pp.rl[k].kind == 2 ? RW_PATH_RESIDENT_STREAMED : RW_PATH_RESIDENT_SPLIT;
    }
    return RW_OK;
    });
}

int rw_solve_bricks(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                    int64_t n_voxels, const float* g, const uint8_t* mask, float* x, double* x64,
                    rw_brick_stats* stats, void* stream) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    return guarded(ctx, [&] {
        return solve_bricks_impl(ctx, params, n_bricks, bricks, n_voxels, g, mask, x, x64, stats, stream, SolveMode{});
    });
}

int rw_solve_bricks_noalloc(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                            int64_t n_voxels, const float* g, const uint8_t* mask, float* x, double* x64,
                            rw_brick_stats* stats, void* stream) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    return guarded(ctx, [&] {
        SolveMode mode;
        mode.noalloc = true;
        return solve_bricks_impl(ctx, params, n_bricks, bricks, n_voxels, g, mask, x, x64, stats, stream, mode);
    });
}

size_t rw_noalloc_scratch_bytes(void) { return (size_t)kScratchBytes; }

// lanes of the streamed solve: context, compute stream and staging set
// (three lanes measured slower than two: each solve forks onto two side
// streams, and a process has four hardware queues)
static constexpr int kLanes = 2;

int rw_solve_bricks_streamed(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                             int64_t n_voxels, const float* g, const uint8_t* mask, float* x,
                             rw_brick_stats* stats, int64_t chunk_voxels, void* stream) {
    return guarded(ctx, [&]() -> int {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (n_bricks < 0 || n_voxels < 0) return fail(ctx, RW_E_INVAL, "n_bricks and n_voxels must be >= 0");
    if (n_bricks == 0) return RW_OK;
    if (!bricks || !g || !mask || !x) return fail(ctx, RW_E_INVAL, "bricks, g, mask and x must be non-NULL");
    // a tuned request takes the whole list's tuned schedule for every chunk
    PlanChoice pc_all;
    const rw_solve_params presolved = resolve_schedule(ctx, *params, n_bricks, bricks, &pc_all);
    params = &presolved;
    PlanScope pls(ctx, pc_all);
    const int R = params->nrhs;
    // default: 2^24 voxels, large enough that a chunk fills the GPU with
    // several waves of boxes (each chunk's solve ends with its slowest box)
    if (chunk_voxels <= 0) chunk_voxels = (int64_t)1 << 24;
    // chunks: runs of consecutive boxes (in increasing offset order) whose
    // voxel span stays within chunk_voxels; a larger box is a chunk alone
    auto vox = [&](int64_t i) { return (int64_t)bricks[i].nx * bricks[i].ny * bricks[i].nz; };
    std::vector<int64_t> cut{0};
    int64_t span_max = 0, boxes_max = 0;
    for (int64_t i = 0; i < n_bricks; ++i) {
        if (bricks[i].nx < 1 || bricks[i].ny < 1 || bricks[i].nz < 1 || bricks[i].offset < 0 ||
            bricks[i].offset + vox(i) > n_voxels)
            return fail(ctx, RW_E_INVAL, "brick %lld does not fit the %lld voxels", (long long)i, (long long)n_voxels);
        if (i > 0 && bricks[i].offset < bricks[i - 1].offset + vox(i - 1))
            return fail(ctx, RW_E_INVAL, "streamed boxes must be in increasing offset order without overlap (brick %lld)",
                        (long long)i);
        const int64_t c0 = cut.back();
        if (i > c0 && bricks[i].offset + vox(i) - bricks[c0].offset > chunk_voxels) cut.push_back(i);
    }
    cut.push_back(n_bricks);
    const int64_t nc = (int64_t)cut.size() - 1;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t b0 = cut[c], b1 = cut[c + 1];
        span_max = std::max(span_max, bricks[b1 - 1].offset + vox(b1 - 1) - bricks[b0].offset);
        boxes_max = std::max(boxes_max, b1 - b0);
    }
    hipStream_t s = (hipStream_t)stream;
    DevGuard dg(ctx->device);
    if (!ctx->cs[0]) {
        for (int i = 0; i < 2; ++i) {
            hipError_t e = hipStreamCreateWithFlags(&ctx->cs[i], hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(ctx, e, "creating copy streams");
        }
        for (hipEvent_t& ev : ctx->cev) {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(ctx, e, "creating copy events");
        }
        hipError_t e = hipEventCreateWithFlags(&ctx->pin_ev, hipEventDisableTiming);
        for (int i = 0; i < kLanes - 1 && e == hipSuccess; ++i)
            e = hipStreamCreateWithFlags(&ctx->tstream[i], hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(ctx, e, "creating copy events");
    }
    for (int i = 0; i < kLanes - 1; ++i)
        if (!ctx->twin[i]) {
            rc = rw_ctx_create(ctx->device, &ctx->twin[i]);
            if (rc) return fail(ctx, rc, "creating a lane's solve context: %s", rw_last_error(nullptr));
        }
    // page-locked box-list slots, one per chunk (a slot per BrickDev list,
    // 256-byte aligned); an earlier call's uploads from them are waited for
    {
        hipError_t e = hipEventSynchronize(ctx->pin_ev);
        const size_t want = (size_t)n_bricks * sizeof(rwk::BrickDev) + (size_t)nc * 256 + 256;
        if (e == hipSuccess && ctx->pin_bytes < want) {
            if (ctx->pin) e = hipHostFree(ctx->pin);
            ctx->pin = nullptr;
            ctx->pin_bytes = 0;
            if (e == hipSuccess) e = hipHostMalloc(&ctx->pin, want, hipHostMallocDefault);
            if (e == hipSuccess) ctx->pin_bytes = want;
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "allocating page-locked box lists");
    }
    // staging set k: g float [span], x float [span * R], stats [boxes], mask uint8 [span]
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t bg = up((size_t)span_max * 4), bx = up((size_t)span_max * R * 4),
                 bs = up((size_t)boxes_max * sizeof(rw_brick_stats)), bm = up((size_t)span_max);
    const size_t set = bg + bx + bs + bm;
    // nothing of an earlier call may still use the staging sets
    hipError_t e = hipStreamSynchronize(ctx->cs[0]);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->cs[1]);
    if (e == hipSuccess) e = grow(ctx, &ctx->ooc, &ctx->ooc_bytes, kLanes * set, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "allocating staging buffers");
    char* base = (char*)ctx->ooc;
    auto G = [&](int k) { return (float*)(base + k * set); };
    auto X = [&](int k) { return (float*)(base + k * set + bg); };
    auto S = [&](int k) { return (rw_brick_stats*)(base + k * set + bg + bx); };
    auto M = [&](int k) { return (uint8_t*)(base + k * set + bg + bx + bs); };
    hipEvent_t* h2d = &ctx->cev[0];     // [kLanes] staging set k filled
    hipEvent_t* done = &ctx->cev[3];    // [kLanes] staging set k solved
    hipEvent_t* d2h = &ctx->cev[6];     // [kLanes] staging set k copied back
    hipEvent_t start = ctx->cev[9];
    // on a failure part-way, the copies already queued finish before returning
    auto drain = [&](int code) {
        for (rw_ctx* c : {ctx, ctx->twin[0], ctx->twin[1]})
            if (c) c->plan_cols = c->plan_unaligned = c->plan_no_third = 0;
        (void)hipStreamSynchronize(ctx->cs[0]);
        (void)hipStreamSynchronize(ctx->cs[1]);
        for (hipStream_t t : ctx->tstream)
            if (t) (void)hipStreamSynchronize(t);
        (void)hipEventRecord(ctx->pin_ev, s);
        return code;
    };
    auto span_of = [&](int64_t c, int64_t* off) {
        *off = bricks[cut[c]].offset;
        return bricks[cut[c + 1] - 1].offset + vox(cut[c + 1] - 1) - *off;
    };
    auto fill = [&](int64_t c, int k) -> hipError_t {
        int64_t off;
        const int64_t n = span_of(c, &off);
        hipError_t r = hipMemcpyAsync(G(k), g + off, (size_t)n * 4, hipMemcpyHostToDevice, ctx->cs[0]);
        if (r == hipSuccess) r = hipMemcpyAsync(M(k), mask + off, (size_t)n, hipMemcpyHostToDevice, ctx->cs[0]);
        if (r == hipSuccess)
            r = hipMemcpyAsync(X(k), x + off * R, (size_t)n * R * 4, hipMemcpyHostToDevice, ctx->cs[0]);
        if (r == hipSuccess) r = hipEventRecord(h2d[k], ctx->cs[0]);
        return r;
    };
    // chunk c is solved by lane c % kLanes: its context, its stream (lane
    // 0: the caller's context and stream) and its staging set
    rw_ctx* C[kLanes] = {ctx};
    hipStream_t SS[kLanes] = {s};
    for (int i = 1; i < kLanes; ++i) {
        C[i] = ctx->twin[i - 1];
        SS[i] = ctx->tstream[i - 1];
    }
    // every chunk takes the window columns and plane-march variant of the
    // whole list, so that each box runs the kernel it runs in one call
    {
        const bool fp64 = params->precision == RW_PREC_FP64;
        const int cols = plan_cols_of(ctx, bricks, n_bricks, R, fp64);
        const int lim = rwk::plane_lds_bytes(R, fp64, cols) <= ctx->lds_limit ? rwk::plane_max(cols) : 0;
        const bool res_ok = resident_ok(R, fp64, params->schedule);
        int unaligned = 0;
        for (int64_t i = 0; i < n_bricks; ++i)
            if (group_of(ctx, bricks[i].nx, bricks[i].ny, bricks[i].nz, lim, res_ok, params->schedule == 4, false) == 2 &&
                (int64_t)rwk::plane_max(cols) % ((int64_t)bricks[i].nx * bricks[i].ny) != 0)
                unaligned = 1;
        for (rw_ctx* c : C) {
            c->plan_cols = cols;
            c->plan_unaligned = unaligned;
            c->plan_no_third = 1;
        }
    }
    auto unplan = [&] {
        for (rw_ctx* c : C) c->plan_cols = c->plan_unaligned = c->plan_no_third = 0;
    };
    e = hipEventRecord(start, s);
    for (hipStream_t t : {ctx->cs[0], ctx->cs[1]})
        if (e == hipSuccess) e = hipStreamWaitEvent(t, start, 0);
    for (int i = 1; i < kLanes && e == hipSuccess; ++i) e = hipStreamWaitEvent(SS[i], start, 0);
    for (int64_t c = 0; c < std::min<int64_t>(nc, kLanes) && e == hipSuccess; ++c) e = fill(c, (int)c);
    if (e != hipSuccess) return drain(hip_fail(ctx, e, "queuing host-to-device copies"));
    std::vector<rw_brick> rb;
    char* slot = (char*)ctx->pin;
    for (int64_t c = 0; c < nc; ++c) {
        const int k = (int)(c % kLanes);
        int64_t off;
        const int64_t n = span_of(c, &off);
        rb.assign(bricks + cut[c], bricks + cut[c + 1]);
        for (rw_brick& b : rb) b.offset -= off;
        e = hipStreamWaitEvent(SS[k], h2d[k], 0);
        if (e != hipSuccess) return drain(hip_fail(ctx, e, "ordering the solve after its copies"));
        C[k]->list_stage = slot;
        rc = rw_solve_bricks(C[k], params, (int64_t)rb.size(), rb.data(), n, G(k), M(k), X(k), nullptr,
                             stats ? S(k) : nullptr, SS[k]);
        C[k]->list_stage = nullptr;
        slot += ((rb.size() * sizeof(rwk::BrickDev) + 255) & ~size_t(255));
        if (rc) {
            if (k) ctx->err = C[k]->err;
            return drain(rc);
        }
        e = hipEventRecord(done[k], SS[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(ctx->cs[1], done[k], 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(x + off * R, X(k), (size_t)n * R * 4, hipMemcpyDeviceToHost, ctx->cs[1]);
        if (e == hipSuccess && stats)
            e = hipMemcpyAsync(stats + cut[c], S(k), rb.size() * sizeof(rw_brick_stats), hipMemcpyDeviceToHost,
                               ctx->cs[1]);
        if (e == hipSuccess) e = hipEventRecord(d2h[k], ctx->cs[1]);
        // the set is refilled once its results are out
        if (e == hipSuccess && c + kLanes < nc) {
            e = hipStreamWaitEvent(ctx->cs[0], d2h[k], 0);
            if (e == hipSuccess) e = fill(c + kLanes, k);
        }
        if (e != hipSuccess) return drain(hip_fail(ctx, e, "queuing copies"));
    }
    unplan();
    e = hipStreamWaitEvent(s, d2h[(nc - 1) % kLanes], 0);
    if (e == hipSuccess) e = hipEventRecord(ctx->pin_ev, s);
    if (e != hipSuccess) return drain(hip_fail(ctx, e, "joining the copy stream"));
    return RW_OK;
    });
}

int rw_solve_bricks_adjoint(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks,
                            const rw_brick* bricks, int64_t n_voxels, const float* g, const uint8_t* mask,
                            const float* x, const float* dl_dx, float* dl_dg, double* dl_dbeta,
                            float* lambda, rw_brick_stats* stats, void* stream) {
    return guarded(ctx, [&]() -> int {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (params->nrhs != 1) return fail(ctx, RW_E_UNSUPPORTED, "adjoint supports nrhs = 1 only");
    std::vector<rwk::BrickDev> list;
    rc = build_list(ctx, n_bricks, bricks, n_voxels, &list);
    if (rc) return rc;
    if (!dl_dbeta) return fail(ctx, RW_E_INVAL, "dl_dbeta must be non-NULL");
    if (n_bricks > 0 && (!g || !mask || !x || !dl_dx || !dl_dg))
        return fail(ctx, RW_E_INVAL, "g, mask, x, dl_dx and dl_dg must be non-NULL");
    hipStream_t s = (hipStream_t)stream;
    DevGuard dg(ctx->device);
    const size_t nv = (size_t)n_voxels;
    size_t bytes = 4 * nv * sizeof(float);
    const size_t off_lam = bytes;
    if (!lambda) bytes += nv * sizeof(float);
    hipError_t e = grow(ctx, &ctx->ws, &ctx->ws_bytes, std::max<size_t>(bytes, 256), s);
    if (e != hipSuccess) return hip_fail(ctx, e, "allocating adjoint workspace");
    PlanChoice pc;
    const rw_solve_params pe = resolve_schedule(ctx, *params, n_bricks, bricks, &pc);
    PlanScope pls(ctx, pc);
    rwk::PlanePlan pp = plan_planes(ctx, &list, 1, false, pe.schedule);
    const size_t state_bytes = ((size_t)n_bricks * sizeof(rwk::BoxState) + 255) & ~size_t(255);
    const size_t part_bytes = ((size_t)n_bricks * sizeof(double) + 255) & ~size_t(255);
    const size_t tickets_off = up256(state_bytes + part_bytes + rwk::domain_scratch_bytes(pp.n_dom));
    e = grow(ctx, &ctx->aux, &ctx->aux_bytes, tickets_off + kTicketBytes, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "allocating adjoint partials");
    rc = attach_side_streams(ctx, &pp);
    if (rc) return rc;
    rc = upload_list(ctx, list, s);
    if (rc) return rc;
    char* w = (char*)ctx->ws;
    rwk::AdjointArgs a{};
    a.bricks = (const rwk::BrickDev*)ctx->bricks;
    a.g = g;
    a.mask = mask;
    a.x = x;
    a.dl_dx = dl_dx;
    a.dl_dg = dl_dg;
    a.r = (float*)w;
    a.z = (float*)(w + nv * 4);
    a.p0 = (float*)(w + 2 * nv * 4);
    a.p1 = (float*)(w + 3 * nv * 4);
    a.lambda = lambda ? lambda : (float*)(w + off_lam);
    a.beta_part = (double*)((char*)ctx->aux + state_bytes);
    a.stats = stats;
    a.beta = params->beta;
    a.eps = params->eps;
    a.tol = params->tol;
    a.max_iter = params->max_iter;
    rwk::SolveArgs sa{};
    sa.bricks = a.bricks;
    sa.g = g;
    sa.mask = mask;
    sa.r = a.r;
    sa.z = a.z;
    sa.p0 = a.p0;
    sa.p1 = a.p1;
    sa.state = (rwk::BoxState*)ctx->aux;
    sa.beta = a.beta;
    sa.eps = a.eps;
    sa.tol = a.tol;
    sa.inner_tol = a.tol;
    sa.max_iter = a.max_iter;
    sa.precision = RW_PREC_MIXED;
    sa.schedule = stream_schedule(pe.schedule);
    rwk::domain_bind(sa, (char*)ctx->aux + state_bytes + part_bytes);
    sa.tickets = (uint32_t*)((char*)ctx->aux + tickets_off);
    rc = bind_weights(ctx, pp, &sa, s);
    if (rc) return rc;
    e = rwk::launch_adjoint(a, sa, n_bricks, dl_dbeta, pp, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "launching adjoint kernels");
    return RW_OK;
    });
}

int rw_probe_blocks(void) { return rwk::kProbeBlocks; }

int rw_probe_read(rw_ctx* ctx, const void* src, int64_t bytes, int passes, int unroll, float* part, void* stream) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    if (!src || !part) return fail(ctx, RW_E_INVAL, "src and part must be non-NULL");
    if (bytes <= 0 || bytes % 16 != 0 || ((uintptr_t)src & 15) != 0)
        return fail(ctx, RW_E_INVAL, "bytes must be a positive multiple of 16 and src 16-byte aligned");
    if (passes < 1) return fail(ctx, RW_E_INVAL, "passes must be >= 1");
    if (unroll != 4 && unroll != 8 && unroll != 16) return fail(ctx, RW_E_INVAL, "unroll must be 4, 8 or 16");
    DevGuard dg(ctx->device);
    hipError_t e = rwk::launch_probe_read(src, bytes, passes, unroll, part, (hipStream_t)stream);
    return e == hipSuccess ? RW_OK : hip_fail(ctx, e, "launching the read probe");
}

int rw_probe_copy(rw_ctx* ctx, void* dst, const void* src, int64_t bytes, void* stream) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    if (!src || !dst) return fail(ctx, RW_E_INVAL, "src and dst must be non-NULL");
    if (bytes <= 0 || bytes % 16 != 0 || ((uintptr_t)src & 15) != 0 || ((uintptr_t)dst & 15) != 0)
        return fail(ctx, RW_E_INVAL, "bytes must be a positive multiple of 16 and both buffers 16-byte aligned");
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes) return fail(ctx, RW_E_INVAL, "src and dst overlap");
    DevGuard dg(ctx->device);
    hipError_t e = rwk::launch_probe_copy(dst, src, bytes, (hipStream_t)stream);
    return e == hipSuccess ? RW_OK : hip_fail(ctx, e, "launching the copy probe");
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate schedules of one batch and keeps the fastest.
// ---------------------------------------------------------------------------

int rw_autotune(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                int64_t n_voxels, const float* g, const uint8_t* mask, const float* x0, float* x_work, int reps,
                rw_tune_report* out, void* stream) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    return guarded(ctx, [&]() -> int {
        int rc = check_params(ctx, params);
        if (rc) return rc;
        if (params->schedule == RW_SCHED_TUNED) return fail(ctx, RW_E_INVAL, "tune a concrete schedule (0..4)");
        if (n_bricks < 1 || !x0 || !x_work || reps < 1 || reps > 64)
            return fail(ctx, RW_E_INVAL, "need n_bricks >= 1, x0, x_work and 1 <= reps <= 64");
        if (x0 == x_work) return fail(ctx, RW_E_INVAL, "x0 and x_work must differ");
        std::vector<rwk::BrickDev> list;
        rc = build_list(ctx, n_bricks, bricks, n_voxels, &list);
        if (rc) return rc;
        // candidates: the resident plans (MIXED, one rhs) with and without
        // the third stream, every fitting box on the streamed-weights kernel,
        // and the streaming schedules (two sweeps; one sweep)
        struct Cand {
            int schedule, no_third, no_regs, persist, no_split;
        };
        std::vector<Cand> cands;
        if (params->nrhs == 1 && params->precision != RW_PREC_FP64) {
            cands = {{0, 0, 0, 0, 0}, {0, 1, 0, 0, 0}, {0, 0, 1, 0, 0}, {0, 0, 0, 1, 0},
                     {4, 0, 0, 0, 0}, {3, 0, 0, 0, 0}, {1, 0, 0, 0, 0}};
            // with split boxes in the batch: the default plan with them streaming
            bool any_split = false;
            for (const auto& b : list) any_split = any_split || rwk::resident_split_fits(b, ctx->lds_limit);
            if (any_split) cands.push_back({0, 0, 0, 0, 1});
        } else {
            cands = {{1, 0, 0, 0, 0}, {2, 0, 0, 0, 0}};
        }
        hipStream_t s = (hipStream_t)stream;
        DevGuard dg(ctx->device);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return hip_fail(ctx, e, "creating tuning events");
        }
        const size_t xbytes = (size_t)n_voxels * params->nrhs * sizeof(float);
        const int saved_timing = ctx->timing;
        ctx->timing = 0;
        std::vector<float> med(cands.size(), 0.0f);
        rc = RW_OK;
        for (size_t c = 0; c < cands.size() && rc == RW_OK; ++c) {
            rw_solve_params q = *params;
            q.schedule = cands[c].schedule;
            PlanChoice pc;
            pc.no_third = cands[c].no_third;
            pc.no_regs = cands[c].no_regs;
            pc.persist = cands[c].persist;
            pc.no_split = cands[c].no_split;
            PlanScope pls(ctx, pc);
            std::vector<float> t;
            for (int r = 0; r <= reps && rc == RW_OK; ++r) {   // run 0 warms up
                e = hipMemcpyAsync(x_work, x0, xbytes, hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                if (e != hipSuccess) {
                    rc = hip_fail(ctx, e, "resetting x for a tuning run");
                    break;
                }
                rc = solve_bricks_impl(ctx, &q, n_bricks, bricks, n_voxels, g, mask, x_work, nullptr, nullptr, stream,
                                       SolveMode{});
                if (rc) break;
                float ms = 0.0f;
                e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) rc = hip_fail(ctx, e, "timing a tuning run");
                if (r > 0) t.push_back(ms);
            }
            if (rc == RW_OK) {
                std::sort(t.begin(), t.end());
                med[c] = t[t.size() / 2];
            }
        }
        ctx->timing = saved_timing;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        size_t best = 0;
        for (size_t c = 1; c < cands.size(); ++c)
            if (med[c] < med[best]) best = c;
        const uint64_t key = batch_key(*params, n_bricks, bricks);
        bool found = false;
        for (rw_ctx::Tuned& t : ctx->tuned)
            if (t.key == key) {
                t = rw_ctx::Tuned{key, cands[best].schedule, cands[best].no_third, cands[best].no_regs,
                                  cands[best].persist, cands[best].no_split, med[best]};
                found = true;
            }
        if (!found)
            ctx->tuned.push_back(rw_ctx::Tuned{key, cands[best].schedule, cands[best].no_third,
                                               cands[best].no_regs, cands[best].persist, cands[best].no_split,
                                               med[best]});
        if (out) {
            std::memset(out, 0, sizeof(*out));
            out->n_candidates = (int32_t)cands.size();
            out->best = (int32_t)best;
            out->key = key;
            for (size_t c = 0; c < cands.size(); ++c) {
                out->schedule[c] = cands[c].schedule;
                out->third_stream[c] = cands[c].no_third ? 0 : 1;
                out->weights_in_registers[c] = cands[c].no_regs ? 0 : 1;
                out->persistent[c] = cands[c].persist;
                out->split_boxes[c] = cands[c].no_split ? 0 : 1;
                out->ms[c] = med[c];
            }
        }
        return RW_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Captured graphs of one batched solve.
// ---------------------------------------------------------------------------

struct rw_graph {
    int device = 0;
    void* ws = nullptr;          // the graph's own workspace (box list included)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void graph_release(rw_graph* gr) {
    if (!gr) return;
    DevGuard dg(gr->device);
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    if (gr->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(gr->ws);
    }
    delete gr;
}

extern "C" {

int rw_graph_create(rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                    int64_t n_voxels, const float* g, const uint8_t* mask, float* x, double* x64,
                    rw_brick_stats* stats, void* stream, rw_graph** out) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    if (!out) return fail(ctx, RW_E_INVAL, "out is NULL");
    *out = nullptr;
    return guarded(ctx, [&]() -> int {
        int rc = check_params(ctx, params);
        if (rc) return rc;
        std::vector<rwk::BrickDev> list;
        rc = build_list(ctx, n_bricks, bricks, n_voxels, &list);
        if (rc) return rc;
        if (n_bricks == 0) return fail(ctx, RW_E_INVAL, "a graph needs at least one box");
        if (!g || !mask || !x) return fail(ctx, RW_E_INVAL, "g, mask and x must be non-NULL");
        PlanChoice pc;
        const rw_solve_params p = resolve_schedule(ctx, *params, n_bricks, bricks, &pc);
        PlanScope pls(ctx, pc);
        const bool fp64 = p.precision == RW_PREC_FP64;
        rwk::PlanePlan pp = plan_planes(ctx, &list, p.nrhs, fp64, p.schedule);
        if (pp.n_dom > 0)
            return fail(ctx, RW_E_UNSUPPORTED,
                        "a batch with single-domain boxes (the domain solver polls the host) cannot be captured");
        const SolveLayout L = solve_layout(p, n_bricks, n_voxels, x64, pp);
        hipStream_t s = (hipStream_t)stream;
        DevGuard dg(ctx->device);
        rw_graph* gr = new rw_graph();
        gr->device = ctx->device;
        hipError_t e = hipMalloc(&gr->ws, layout_total(L));
        if (e != hipSuccess) {
            graph_release(gr);
            return hip_fail(ctx, e, "allocating the graph's workspace");
        }
        // the box list goes into the workspace once, before the capture
        char* blist = (char*)gr->ws + L.ws_bytes + L.aux_bytes;
        e = hipMemcpy(blist, list.data(), list.size() * sizeof(rwk::BrickDev), hipMemcpyHostToDevice);
        rc = e == hipSuccess ? attach_side_streams(ctx, &pp) : hip_fail(ctx, e, "uploading the box list");
        if (rc) {
            graph_release(gr);
            return rc;
        }
        const int saved_timing = ctx->timing;
        ctx->timing = 0;
        e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            ctx->timing = saved_timing;
            graph_release(gr);
            return hip_fail(ctx, e, "beginning stream capture (the stream must not be the null stream)");
        }
        SolveMode mode;
        mode.ext = (char*)gr->ws;
        mode.ext_bytes = layout_total(L);
        rc = solve_bricks_impl(ctx, &p, n_bricks, bricks, n_voxels, g, mask, x, x64, stats, stream, mode);
        e = hipStreamEndCapture(s, &gr->graph);
        ctx->timing = saved_timing;
        if (rc == RW_OK && e != hipSuccess) rc = hip_fail(ctx, e, "ending stream capture");
        if (rc == RW_OK) {
            e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(ctx, e, "instantiating the graph");
        }
        if (rc) {
            graph_release(gr);
            return rc;
        }
        *out = gr;
        return RW_OK;
    });
}

int rw_graph_launch(rw_graph* gr, void* stream) {
    if (!gr || !gr->exec) return fail(nullptr, RW_E_INVAL, "graph is NULL");
    DevGuard dg(gr->device);
    hipError_t e = hipGraphLaunch(gr->exec, (hipStream_t)stream);
    return e == hipSuccess ? RW_OK : fail(nullptr, RW_E_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
}

void rw_graph_free(rw_graph* gr) { graph_release(gr); }

int rw_tuned_schedule(const rw_ctx* ctx, const rw_solve_params* params, int64_t n_bricks, const rw_brick* bricks,
                      int32_t* schedule, int32_t* third_stream, int32_t* regs, int32_t* persist,
                      int32_t* tuned) {
    if (!ctx || !params || !schedule || !third_stream || !tuned || n_bricks < 0 || (n_bricks > 0 && !bricks))
        return fail(nullptr, RW_E_INVAL, "bad arguments");
    rw_solve_params q = *params;
    q.schedule = RW_SCHED_TUNED;
    PlanChoice pc;
    const rw_solve_params r = resolve_schedule(ctx, q, n_bricks, bricks, &pc);
    *schedule = r.schedule;
    *third_stream = pc.no_third ? 0 : 1;
    if (regs) *regs = pc.no_regs ? 0 : 1;
    if (persist) *persist = pc.persist;
    *tuned = 0;
    for (const rw_ctx::Tuned& t : ctx->tuned)
        if (n_bricks > 0 && t.key == batch_key(*params, n_bricks, bricks)) *tuned = 1;
    return RW_OK;
}

}  // extern "C"
