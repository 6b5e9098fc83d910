// Resident Jacobi-PCG for boxes that fit on one compute unit (one
// right-hand side, FP32 vectors, FP64 reductions; Section III-B system,
// Section V solver).
//
// The streaming kernels read g and the CG vectors from HBM in every sweep.
// A box of up to 32^3 voxels keeps its search direction p in the LDS of one
// CU instead, and each thread keeps its own voxels' x, r and q = L_UU p in
// registers (thread t owns voxels t + k * NT, so every LDS access of a wave
// is to consecutive words).  The edge weights are computed once per solve:
// into LDS beside p for boxes up to 10240 voxels (k_pcg_resw), or into a
// per-box segment of a global buffer that stays in the Infinity Cache for
// larger ones (k_pcg_resg).  Per iteration:
//   p = z + beta p        (own voxels, in place in LDS)        barrier
//   q = d p - sum_nb w p_nb, sigma = p.q
//   reduce sigma -> alpha;  x += alpha p, r -= alpha q, z = r/d
//   reduce r.z, ||r||^2 -> beta, convergence test
// The iteration is the same Jacobi-PCG as the streaming kernels (same start
// state, same stopping rule), so the paths are interchangeable per box.

#include "common.h"

#include <algorithm>

namespace rwk {

namespace {


template <int NT, int N>
__device__ __forceinline__ void res_block_sum(double (&v)[N], double* red) {
    constexpr int W = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = v[k];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        v[k] = s;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[w * N + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i) s += red[i * N + k];
        v[k] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ bool res_finite(double v) { return isfinite(v); }

struct ResWeight {
    float c, eps;  // c = -beta * log2(e)
    __device__ __forceinline__ float operator()(float a, float b) const {
        const float d = a - b;
        return __builtin_amdgcn_exp2f(c * d * d) + eps;
    }
};

}  // namespace

// Start state of a main solve computed by a resident kernel itself (the
// init phase computes it for the other boxes, with the same rules): on
// unknown voxels r0 = sum_nb w x_nb - d x (every in-box neighbour; x on
// unknown voxels is the caller's guess), written to the r workspace, and
// b = the seeded neighbours' part of that sum; rho = r0.z0, ||r0||^2,
// ||b||^2 and the unknown / seeded counts are reduced over the workgroup.
//
// res_start_finish takes each thread's partial sums {r.z, r.r, b.b,
// unknown, seeded}, reduces them (red holds at least 5 * NT / 64 doubles),
// resets P[0, nv) to 0 once every thread's reads of it are done and writes
// the box's BoxState.  With no seed, no unknown or b = 0 (then x_U = 0 and
// r = 0, written here) there is nothing to iterate and it returns false.
template <int NT>
__device__ bool res_start_finish(double (&sum)[5], int nv, const uint8_t* m, float* xb, float* rw, float* P,
                                 double* red, BoxState& st, double& rz, double& rr, double& bb) {
    res_block_sum<NT, 5>(sum, red);  // its barriers order every read of P before the reset below
    for (int v = threadIdx.x; v < nv; v += NT) P[v] = 0.0f;
    const double nU = sum[3], nM = sum[4];
    const bool allzero = sum[2] == 0.0;
    const bool act = nM > 0.0 && nU > 0.0 && !allzero;
    const bool zero_sol = nM > 0.0 && nU > 0.0 && allzero;  // ||b|| = 0: x_U = 0, no iterations
    rz = zero_sol ? 0.0 : sum[0];
    rr = zero_sol ? 0.0 : sum[1];
    bb = sum[2];
    if (zero_sol)
        for (int v = threadIdx.x; v < nv; v += NT)
            if (m[v] == 0) xb[v] = rw[v] = 0.0f;
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) st.rz[c] = st.rr[c] = st.bb[c] = 0.0;
        st.rz[0] = rz;
        st.rr[0] = rr;
        st.bb[0] = bb;
        st.nU = nU;
        st.nM = nM;
        st.rel = 0.0;
        st.true_rel = 0.0;
        st.iters = st.refine_steps = st.refine_iters = 0;
        st.status = nM == 0.0 ? RW_ST_NO_DIRICHLET : RW_ST_CONVERGED;
        st.active = act ? 1 : 0;
        st.pending = 0;
        st.checked = 0;
    }
    __syncthreads();  // P reset and r written before any thread reads them
    // every lane holds the same sums; said so, the caller's exit on it stays
    // uniform and the segment offsets after it stay scalar
    return __builtin_amdgcn_readfirstlane(act ? 1 : 0) != 0;
}

// P[v] for v in [lo, hi): x[v] on the box when with_x, 0 elsewhere.  U
// slots per thread at a time, their loads (clamped into the box) issued
// before any is used.
template <int NT, int U>
__device__ __forceinline__ void res_fill_p(float* P, const float* xb, int lo, int hi, int nv, bool with_x) {
    for (int v0 = lo + (int)threadIdx.x; v0 < hi; v0 += U * NT) {
        float xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * NT;
            xv[u] = xb[min(max(v, 0), nv - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * NT;
            if (v < hi) P[v] = with_x && v >= 0 && v < nv ? xv[u] : 0.0f;
        }
    }
}

// A box's weights pass over the slots v in [lo, hi) (thread t: lo + t +
// k * NT), U slots at a time: every global load of the U (g and the mask at
// the voxel and its six neighbours, indices clamped into the box) is issued
// before any is used, so a thread keeps them in flight together.  Per
// slot: the forward weights w+x, w+y, w+z (0 toward neighbours outside the
// box and on slots outside it) and, when need_d or start, the diagonal d
// (all six edge weights); out(v, wx, wy, wz, d, unknown) stores them.  On
// a main solve (start set; P holds x, with zero pads) also the start-state
// terms of each voxel: on an unknown one r0 = sum_nb w x_nb - d x -> rw[v]
// and its parts of the sums {r.z, r.r, b.b, unknown, seeded}, with z0 =
// r0 / d and b the seeded neighbours' part of the sum; on a seeded one
// r = 0.
template <int NT, int U, typename Out>
__device__ __forceinline__ void res_weights_pass(int lo, int hi, int nx, int ny, int nz, const float* g,
                                                 const uint8_t* m, const ResWeight& W, bool need_d, bool start,
                                                 const float* P, float* rw, double (&sum)[5], Out out) {
    const int nxy = nx * ny, nv = nxy * nz;
    for (int v0 = lo + (int)threadIdx.x; v0 < hi; v0 += U * NT) {
        int c[U];
        bool in[U][6];
        float gc[U], gn[U][6];
        uint8_t mc[U], mn[U][6];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * NT;
            c[u] = v >= 0 && v < nv ? v : 0;
            const int kz = c[u] / nxy, rem = c[u] - kz * nxy, j = rem / nx, i = rem - j * nx;
            const int no[6] = {1, -1, nx, -nx, nxy, -nxy};
            in[u][0] = i + 1 < nx;
            in[u][1] = i > 0;
            in[u][2] = j + 1 < ny;
            in[u][3] = j > 0;
            in[u][4] = kz + 1 < nz;
            in[u][5] = kz > 0;
            gc[u] = g[c[u]];
            mc[u] = m[c[u]];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int nb = in[u][e] ? c[u] + no[e] : c[u];
                gn[u][e] = g[nb];
                mn[u][e] = m[nb];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * NT;
            const bool inb = v >= 0 && v < nv;
            float w[6];  // +x, -x, +y, -y, +z, -z
#pragma unroll
            for (int e = 0; e < 6; ++e) w[e] = 0.0f;
            if (inb) {
                if (in[u][0]) w[0] = W(gc[u], gn[u][0]);
                if (in[u][2]) w[2] = W(gc[u], gn[u][2]);
                if (in[u][4]) w[4] = W(gc[u], gn[u][4]);
                if (need_d || start) {
                    if (in[u][1]) w[1] = W(gn[u][1], gc[u]);
                    if (in[u][3]) w[3] = W(gn[u][3], gc[u]);
                    if (in[u][5]) w[5] = W(gn[u][5], gc[u]);
                }
            }
            const float d = ((w[0] + w[2]) + w[4]) + w[1] + w[3] + w[5];
            const bool unk = inb && mc[u] == 0;
            if (v < hi) out(v, w[0], w[2], w[4], d, unk);
            if (start && inb) {
                const int no[6] = {1, -1, nx, -nx, nxy, -nxy};
                float acc = 0.0f, bs = 0.0f;  // sum_nb w x_nb, and over the seeded neighbours only
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    const float xr = P[v + no[e]];  // inside P's pads for every slot of the box
                    const float xn = in[u][e] ? xr : 0.0f;
                    acc += w[e] * xn;
                    if (mn[u][e] != 0) bs += w[e] * xn;
                }
                const float r0 = unk ? acc - d * P[v] : 0.0f;
                rw[v] = r0;
                if (unk) {
                    sum[0] += (double)r0 * (double)(r0 * __builtin_amdgcn_rcpf(d));
                    sum[1] += (double)r0 * (double)r0;
                    sum[2] += (double)bs * (double)bs;
                }
                sum[3] += unk ? 1.0 : 0.0;  // both counts updated: no run-time index into sum
                sum[4] += unk ? 0.0 : 1.0;
            }
        }
    }
}

// Boxes up to 10240 voxels: one workgroup of NT threads per box (VPT = most
// voxels a thread owns; thread t owns voxels t + k * NT, so every LDS access
// of a wave is to consecutive words).  LDS holds four arrays, p and the
// weights w+x, w+y, w+z of the edges to the +x, +y and +z neighbours (0
// where that neighbour is not in the box), computed once per solve.  Each
// array has nx*ny zero pads before the box and nx*ny + 1 after it, so every
// neighbour address v + offset is inside it; the unused voxel slots of a
// thread map to the element just past the box.  A voxel's other three
// weights are its -x, -y, -z neighbours' forward weights, so the stencil is
// six multiply-adds with no exponential and no mask.  x, r, d, 1/d and
// q = L_UU p stay in registers.  xt: x (main solve) or the correction
// accumulator (corr = 1).
template <int NT, int VPT>
__device__ __forceinline__ void resw_box(const SolveArgs& a, float* xt, int corr, int ib) {
    extern __shared__ __align__(16) float w_lds[];
    __shared__ double red[(NT / 64) * 5];  // block sums of up to 5 values (the start state)
    constexpr int NC = (VPT + 31) / 32;  // unknown-voxel bits
    BoxState& st = a.state[ib];
    const bool fused = a.fused_init && !corr;  // this kernel computes the start state
    if (!fused && !st.active) return;
    const BrickDev bd = a.bricks[ib];
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz, nxy = nx * ny, nv = nxy * nz;
    const int L = nv + 2 * nxy + 1;  // array stride (box and pads)
    float* const P = w_lds + nxy;
    float* const WX = P + L;
    float* const WY = WX + L;
    float* const WZ = WY + L;
    const float* g = a.g + bd.off;
    const uint8_t* m = a.mask + bd.off;
    float* xb = xt + bd.off;
    const float* rb = (const float*)a.r + bd.off;
    const ResWeight W{(float)(-a.beta * 1.4426950408889634), (float)a.eps};

    // Main solve: P holds x (pads 0) while the weights are computed, and
    // the start state is computed in the same pass.  Otherwise P starts at 0.
    res_fill_p<NT, 4>(P, xb, -nxy, nv + nxy + 1, nv, fused);
    if (fused) __syncthreads();
    float* const rw = (float*)a.r + bd.off;
    double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // r.z, r.r, b.b, unknown, seeded
    // forward weights from g (global loads of the voxel and its neighbours)
    res_weights_pass<NT, 4>(-nxy, nv + nxy + 1, nx, ny, nz, g, m, W, false, fused, P, rw, sum,
                            [&](int v, float wx, float wy, float wz, float, bool) {
                                WX[v] = wx;
                                WY[v] = wy;
                                WZ[v] = wz;
                            });
    double rz, rr, bb;
    if (fused) {
        if (!res_start_finish<NT>(sum, nv, m, xb, rw, P, red, st, rz, rr, bb))
            return;  // nothing to iterate (state and x written)
    } else {
        rz = st.rz[0];
        rr = st.rr[0];
        bb = st.bb[0];
    }
    float x[VPT], r[VPT], id[VPT], d[VPT], q[VPT];
    unsigned unk[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) unk[c] = 0u;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v0 = threadIdx.x + k * NT;
        const int v = v0 < nv ? v0 : nv - 1;
        const bool u = v0 < nv && m[v] == 0;
        const float xv = xb[v], rv = rb[v];
        x[k] = u ? xv : 0.0f;
        r[k] = u ? rv : 0.0f;
        unk[k >> 5] |= (u ? 1u : 0u) << (k & 31);
    }
    auto isu = [&](int k) { return (unk[k >> 5] >> (k & 31)) & 1u; };
    auto slot = [&](int tb, int k) { const int v0 = tb + k * NT; return v0 < nv ? v0 : nv; };
    int off_y = nx, off_z = nxy;
    __syncthreads();
    // d = the six weights of the voxel (its own forward ones and its
    // neighbours' forward ones toward it); static
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = slot(threadIdx.x, k);
        const float dd = WX[v] + WY[v] + WZ[v] + WX[v - 1] + WY[v - off_y] + WZ[v - off_z];
        d[k] = isu(k) ? dd : 0.0f;
        id[k] = isu(k) ? __builtin_amdgcn_rcpf(dd) : 0.0f;
    }

    const double tol = corr ? a.inner_tol : a.tol;
    const double tol2 = tol * tol;
    double betac = 0.0;
    int it = 0, flags = 0;
    for (;;) {
        if (rr <= tol2 * bb) break;
        if (it >= a.max_iter) {
            flags = 2;
            break;
        }
        // opaque copies: per-voxel addresses stay inside the loop
        int tb = threadIdx.x;
        asm volatile("" : "+v"(tb));
        asm volatile("" : "+v"(off_y));
        asm volatile("" : "+v"(off_z));
        const float be = it == 0 ? 0.0f : (float)betac;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = slot(tb, k);
            const float pn = r[k] * id[k] + be * P[v];
            P[v] = isu(k) ? pn : 0.0f;
        }
        __syncthreads();
        double sig = 0.0;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = slot(tb, k);
            const float pv = P[v];
            const float acc = WX[v] * P[v + 1] + WX[v - 1] * P[v - 1] + WY[v] * P[v + off_y] +
                              WY[v - off_y] * P[v - off_y] + WZ[v] * P[v + off_z] + WZ[v - off_z] * P[v - off_z];
            q[k] = isu(k) ? d[k] * pv - acc : 0.0f;
            sig += (double)pv * (double)q[k];
        }
        double s1[1] = {sig};
        res_block_sum<NT, 1>(s1, red);
        sig = s1[0];
        const double alpha = rz / sig;
        if (!res_finite(alpha) || !(sig > 0.0)) {
            flags = 1;
            break;
        }
        const float al = (float)alpha;
        double acc2[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = slot(tb, k);
            // p, q, r and 1/d are 0 on seeded and unused slots, so these stay 0
            x[k] += al * P[v];
            r[k] -= al * q[k];
            const float z = r[k] * id[k];
            acc2[0] += (double)r[k] * (double)z;
            acc2[1] += (double)r[k] * (double)r[k];
        }
        res_block_sum<NT, 2>(acc2, red);
        ++it;
        if (!res_finite(acc2[0]) || !res_finite(acc2[1])) {
            flags = 1;
            break;
        }
        betac = acc2[0] / rz;
        rz = acc2[0];
        rr = acc2[1];
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = threadIdx.x + k * NT;
        if (isu(k)) xb[v] = x[k];
    }
    if (threadIdx.x == 0) {
        st.rz[0] = rz;
        st.rr[0] = rr;
        if (corr) {
            st.refine_iters += it;
        } else {
            st.iters = it;
            st.rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            if (flags & 2) st.status = RW_ST_MAX_ITER;
        }
        if (flags & 1) st.status = RW_ST_NONFINITE;
        st.pending = corr && !(flags & 1) ? 1 : 0;
    }
}

// One workgroup per box.
template <int NT, int VPT>
__global__ __launch_bounds__(NT) void k_pcg_resw(SolveArgs a, float* xt, int corr, int base, int, uint32_t*) {
    resw_box<NT, VPT>(a, xt, corr, base + (int)blockIdx.x);
}

// Persistent grid: its workgroups take the boxes [base, end) in launch order
// (largest first) from the ticket counter until none is left.  A kernel of
// its own, so that the loop does not cost the one-box kernel registers.
template <int NT, int VPT>
__global__ __launch_bounds__(NT) void k_pcg_resw_q(SolveArgs a, float* xt, int corr, int base, int end,
                                             uint32_t* ticket) {
    __shared__ int s_ib;
    for (;;) {
        __syncthreads();  // the previous box's last LDS reads are done
        if (threadIdx.x == 0) s_ib = base + (int)atomicAdd(ticket, 1u);
        __syncthreads();
        const int ib = s_ib;
        if (ib >= end) return;
        resw_box<NT, VPT>(a, xt, corr, ib);
    }
}


// Boxes up to kResMaxVptR * 512 voxels (e.g. 16^3, 5x32x32): the
// weights-in-registers kernel.  Each thread computes, once per solve, all six
// edge weights of each of its voxels (thread t owns voxels t + k * NT) from
// g and keeps them in registers with d, 1/d, x, r, p and q; the LDS holds
// only p (with nx*ny zero pads on both sides and one past the box, where the
// unused slots of a thread point).  Per iteration a voxel then touches the
// LDS seven times (its p written once, six neighbours read), against sixteen
// in k_pcg_resw, which keeps the forward weights in LDS: the weights-in-LDS
// kernel is bound by LDS bandwidth, this one by arithmetic.  On a seeded or
// unused slot every weight, d and 1/d are 0, so p, q and r stay 0 there.
// The edge weight is symmetric in its two voxels, so a voxel's backward
// weights equal its neighbours' forward ones bit for bit, and the stencil
// sums in the same order as k_pcg_resw.
template <int NT, int VPT>
__device__ __forceinline__ void resr_box(const SolveArgs& a, float* xt, int corr, int ib) {
    extern __shared__ __align__(16) float pr_lds[];
    __shared__ double red[(NT / 64) * 5];  // block sums of up to 5 values (the start state)
    constexpr int NC = (VPT + 31) / 32;  // unknown-voxel bits
    constexpr int U = VPT > 10 ? 1 : 2;  // voxels per thread whose loads are issued together
    BoxState& st = a.state[ib];
    const bool fused = a.fused_init && !corr;  // this kernel computes the start state
    if (!fused && !st.active) return;
    const BrickDev bd = a.bricks[ib];
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz, nxy = nx * ny, nv = nxy * nz;
    float* const P = pr_lds + nxy;
    const float* g = a.g + bd.off;
    const uint8_t* m = a.mask + bd.off;
    float* xb = xt + bd.off;
    float* const rw = (float*)a.r + bd.off;
    const ResWeight W{(float)(-a.beta * 1.4426950408889634), (float)a.eps};

    // Main solve: P holds x (pads 0) while the weights and the start state
    // are computed.  Otherwise P starts at 0.
    constexpr int span = NT * VPT;  // voxel slots: a thread's unused ones (v >= nv) are LDS slots of their own
    res_fill_p<NT, 4>(P, xb, -nxy, span + nxy, nv, fused);
    if (fused) __syncthreads();
    // above 10 voxels per thread d is not kept but summed from the six
    // weights in every pass (the same sum in the same order, so the same
    // value): one register per voxel less, which 18 voxels per thread need
    constexpr bool kKeepD = VPT <= 10;
    float x[VPT], r[VPT], q[VPT], p[VPT], d[kKeepD ? VPT : 1], id[VPT], w[6][VPT];
    unsigned unk[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) unk[c] = 0u;
    double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // r.z, r.r, b.b, unknown, seeded
    // weights (and, main solve, start state) U voxels at a time, every
    // global load of the U (g and mask at the voxel and its six neighbours,
    // indices clamped into the box) issued before any is used
#pragma unroll
    for (int k0 = 0; k0 < VPT; k0 += U) {
        int c[U];
        bool in[U][6];
        float gc[U], gn[U][6];
        uint8_t mc[U], mn[U][6];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u < VPT) {
                const int v = threadIdx.x + (k0 + u) * NT;
                c[u] = v < nv ? v : 0;
                const int kz = c[u] / nxy, rem = c[u] - kz * nxy, j = rem / nx, i = rem - j * nx;
                const int no[6] = {1, -1, nx, -nx, nxy, -nxy};
                in[u][0] = i + 1 < nx;
                in[u][1] = i > 0;
                in[u][2] = j + 1 < ny;
                in[u][3] = j > 0;
                in[u][4] = kz + 1 < nz;
                in[u][5] = kz > 0;
                gc[u] = g[c[u]];
                mc[u] = m[c[u]];
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    const int nb = in[u][e] ? c[u] + no[e] : c[u];
                    gn[u][e] = g[nb];
                    mn[u][e] = m[nb];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u;
            if (k < VPT) {
                const int v = threadIdx.x + k * NT;
                const bool inb = v < nv;
                const bool uk = inb && mc[u] == 0;
                float we[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) we[e] = inb && in[u][e] ? W(gc[u], gn[u][e]) : 0.0f;
                const float dd = ((we[0] + we[2]) + we[4]) + we[1] + we[3] + we[5];
                float xv = 0.0f, r0 = 0.0f;
                if (fused) {
                    if (inb) {
                        const int no[6] = {1, -1, nx, -nx, nxy, -nxy};
                        float acc = 0.0f, bs = 0.0f;  // sum_nb w x_nb, and over the seeded neighbours only
#pragma unroll
                        for (int e = 0; e < 6; ++e) {
                            const float xr = P[v + no[e]];  // inside P's pads for every voxel of the box
                            const float xn = in[u][e] ? xr : 0.0f;
                            acc += we[e] * xn;
                            if (mn[u][e] != 0) bs += we[e] * xn;
                        }
                        xv = P[v];
                        r0 = uk ? acc - dd * xv : 0.0f;
                        rw[v] = r0;
                        if (uk) {
                            sum[0] += (double)r0 * (double)(r0 * __builtin_amdgcn_rcpf(dd));
                            sum[1] += (double)r0 * (double)r0;
                            sum[2] += (double)bs * (double)bs;
                        }
                        sum[3] += uk ? 1.0 : 0.0;
                        sum[4] += uk ? 0.0 : 1.0;
                    }
                } else {
                    const int cv = inb ? v : nv - 1;
                    xv = xb[cv];
                    r0 = rw[cv];
                }
#pragma unroll
                for (int e = 0; e < 6; ++e) w[e][k] = uk ? we[e] : 0.0f;
                if constexpr (kKeepD) d[k] = uk ? dd : 0.0f;
                id[k] = uk ? __builtin_amdgcn_rcpf(dd) : 0.0f;
                x[k] = uk ? xv : 0.0f;
                r[k] = uk ? r0 : 0.0f;
                unk[k >> 5] |= (uk ? 1u : 0u) << (k & 31);
            }
        }
    }
    double rz, rr, bb;
    if (fused) {
        if (!res_start_finish<NT>(sum, nv, m, xb, rw, P, red, st, rz, rr, bb))
            return;  // nothing to iterate (state and x written)
    } else {
        rz = st.rz[0];
        rr = st.rr[0];
        bb = st.bb[0];
    }
    auto isu = [&](int k) { return (unk[k >> 5] >> (k & 31)) & 1u; };
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        q[k] = r[k] * id[k];  // z0
        p[k] = 0.0f;
    }

    const double tol = corr ? a.inner_tol : a.tol;
    const double tol2 = tol * tol;
    double betac = 0.0;
    int it = 0, flags = 0;
    for (;;) {
        if (rr <= tol2 * bb) break;
        if (it >= a.max_iter) {
            flags = 2;
            break;
        }
        // one base per neighbour direction, fresh for each pass (opaque
        // copies); slot k is base + k * NT, an immediate offset, so no
        // per-voxel address is kept
        int tb = threadIdx.x;
        asm volatile("" : "+v"(tb));
        float* const Pt = P + tb;
        const float be = it == 0 ? 0.0f : (float)betac;
        // p = z + beta p (0 on seeded and unused slots)
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            p[k] = q[k] + be * p[k];
            Pt[k * NT] = p[k];
        }
        __syncthreads();
        int t2 = threadIdx.x, oy = nx, oz = nxy;
        asm volatile("" : "+v"(t2));
        asm volatile("" : "+v"(oy));
        asm volatile("" : "+v"(oz));
        const float* const Q0 = P + t2;
        const float* const Qyp = Q0 + oy;
        const float* const Qym = Q0 - oy;
        const float* const Qzp = Q0 + oz;
        const float* const Qzm = Q0 - oz;
        double sig = 0.0;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const float acc = w[0][k] * Q0[k * NT + 1] + w[1][k] * Q0[k * NT - 1] + w[2][k] * Qyp[k * NT] +
                              w[3][k] * Qym[k * NT] + w[4][k] * Qzp[k * NT] + w[5][k] * Qzm[k * NT];
            float dk;
            if constexpr (kKeepD) dk = d[k];
            else dk = ((w[0][k] + w[2][k]) + w[4][k]) + w[1][k] + w[3][k] + w[5][k];
            q[k] = dk * p[k] - acc;
            sig += (double)p[k] * (double)q[k];
        }
        double s1[1] = {sig};
        res_block_sum<NT, 1>(s1, red);
        sig = s1[0];
        const double alpha = rz / sig;
        if (!res_finite(alpha) || !(sig > 0.0)) {
            flags = 1;
            break;
        }
        const float al = (float)alpha;
        double acc2[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            // p, q, r and 1/d are 0 on seeded and unused slots, so these stay 0
            x[k] += al * p[k];
            r[k] -= al * q[k];
            const float z = r[k] * id[k];
            q[k] = z;
            acc2[0] += (double)r[k] * (double)z;
            acc2[1] += (double)r[k] * (double)r[k];
        }
        res_block_sum<NT, 2>(acc2, red);
        ++it;
        if (!res_finite(acc2[0]) || !res_finite(acc2[1])) {
            flags = 1;
            break;
        }
        betac = acc2[0] / rz;
        rz = acc2[0];
        rr = acc2[1];
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = threadIdx.x + k * NT;
        if (isu(k)) xb[v] = x[k];
    }
    if (threadIdx.x == 0) {
        st.rz[0] = rz;
        st.rr[0] = rr;
        if (corr) {
            st.refine_iters += it;
        } else {
            st.iters = it;
            st.rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            if (flags & 2) st.status = RW_ST_MAX_ITER;
        }
        if (flags & 1) st.status = RW_ST_NONFINITE;
        st.pending = corr && !(flags & 1) ? 1 : 0;
    }
}

// One workgroup per box.
template <int NT, int VPT>
__global__ __launch_bounds__(NT) void k_pcg_resr(SolveArgs a, float* xt, int corr, int base, int, uint32_t*) {
    resr_box<NT, VPT>(a, xt, corr, base + (int)blockIdx.x);
}

// Persistent grid: its workgroups take the boxes [base, end) in launch order
// (largest first) from the ticket counter until none is left.  A kernel of
// its own, so that the loop does not cost the one-box kernel registers.
template <int NT, int VPT>
__global__ __launch_bounds__(NT) void k_pcg_resr_q(SolveArgs a, float* xt, int corr, int base, int end,
                                             uint32_t* ticket) {
    __shared__ int s_ib;
    for (;;) {
        __syncthreads();  // the previous box's last LDS reads are done
        if (threadIdx.x == 0) s_ib = base + (int)atomicAdd(ticket, 1u);
        __syncthreads();
        const int ib = s_ib;
        if (ib >= end) return;
        resr_box<NT, VPT>(a, xt, corr, ib);
    }
}


// Variant for boxes whose search direction alone fits in one CU's LDS (up
// to 32768 voxels, e.g. 32^3): LDS holds p only (4 B per voxel, pads as
// above).  The forward weights w+x, w+y, w+z and 1/d are computed once per
// launch into the box's segment of a global buffer and read back in every
// iteration; a box's segment stays in the last-level cache while its
// workgroup iterates, so an iteration reads about 16 B per voxel from there
// and computes no exponential.  x, r and q (q holds z between iterations)
// stay in registers.
//
// Segment of a box (floats): arrays WX, WY, WZ, ID of stride
// T = nx*ny + NT*VPT, each nx*ny zeros, the box, then zeros up to NT*VPT.
// Thread t owns the slots t + k*NT, k < VPT, of which those >= nv are
// unused: they read LDS pads and segment zeros (p = 0, 1/d = 0), so no
// address is clamped.  1/d = 0 also marks seeded voxels, whose r is kept
// at 0.
//
// The forward weights (and 1/d) are loaded G voxels ahead of their use (a
// two-group register ring, pinned with scheduling barriers), so a wave keeps
// 3G loads to the Infinity Cache in flight instead of waiting on each
// voxel's weights.  The backward weights are lines the same or a
// neighbouring lane or wave has just brought into L1; they are loaded when
// their group is computed, before the next group's forward loads, so that
// waiting for them (loads complete in order) leaves those in flight.
// Segment accesses are buffer instructions on one resource for the
// segment: a per-voxel byte offset in a VGPR and the array (and neighbour)
// offset in an SGPR, so no 64-bit address is formed or kept per voxel.
// The resource's size bounds every access to the segment.
struct SegBuf {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ float ld(unsigned vo, int so) const {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)vo, so, 0));
    }
};

// Workgroup barrier that orders LDS only (global loads stay in flight).
__device__ __forceinline__ void res_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int NT, int N>
__device__ __forceinline__ void res_block_sum_lds(double (&v)[N], double* red) {
    constexpr int W = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = v[k];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        v[k] = s;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[w * N + k] = v[k];
    }
    res_lds_barrier();
    // lane k < N adds value k over the waves (wave order); every lane then
    // reads the N totals from those lanes (uniform: no VGPR holds them)
    double s = 0.0;
    if (lane < N) {
#pragma unroll
        for (int i = 0; i < W; ++i) s += red[i * N + lane];
    }
    const unsigned long long sb = (unsigned long long)__double_as_longlong(s);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const unsigned lo = __builtin_amdgcn_readlane((unsigned)sb, k);
        const unsigned hi = __builtin_amdgcn_readlane((unsigned)(sb >> 32), k);
        v[k] = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
    res_lds_barrier();
}

template <int NT, int VPT, int G>
__device__ __forceinline__ void resg_box(const SolveArgs& a, float* xt, int corr, int ib) {
    extern __shared__ __align__(16) float p_lds[];
    __shared__ double red[(NT / 64) * 5];  // block sums of up to 5 values (the start state)
    constexpr int NG = (VPT + G - 1) / G;
    BoxState& st = a.state[ib];
    const bool fused = a.fused_init && !corr;  // this kernel computes the start state
    if (!fused && !st.active) return;
    const BrickDev bd = a.bricks[ib];
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz, nxy = nx * ny, nv = nxy * nz;
    constexpr int span = NT * VPT;
    const int T = nxy + span;  // stride of the segment arrays
    float* P = p_lds + nxy;
    const float* g = a.g + bd.off;
    const uint8_t* m = a.mask + bd.off;
    float* const xb = xt + bd.off;
    const float* rb = (const float*)a.r + bd.off;
    float* const seg = a.wts + bd.woff;
    float* const WX = seg + nxy;
    float* const WY = WX + T;
    float* const WZ = WY + T;
    float* const ID = WZ + T;
    const ResWeight W{(float)(-a.beta * 1.4426950408889634), (float)a.eps};

    // Main solve: P holds x (pads 0) while the weights are computed, and
    // the start state is computed in the same pass from the weights in
    // registers.  Otherwise P starts at 0.
    res_fill_p<NT, 8>(P, xb, -nxy, span + nxy, nv, fused);
    if (fused) __syncthreads();
    float* const rw = (float*)a.r + bd.off;
    double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // r.z, r.r, b.b, unknown, seeded
    // weights (0 toward neighbours outside the box) and 1/d (0 on seeded
    // voxels); pads and unused slots are 0
    res_weights_pass<NT, 8>(-nxy, span, nx, ny, nz, g, m, W, true, fused, P, rw, sum,
                            [&](int v, float wx, float wy, float wz, float d, bool unk) {
                                WX[v] = wx;
                                WY[v] = wy;
                                WZ[v] = wz;
                                ID[v] = unk ? __builtin_amdgcn_rcpf(d) : 0.0f;
                            });
    // 0x00020000: raw 32-bit buffer (third descriptor word for this chip family)
    const SegBuf sb{__builtin_amdgcn_make_buffer_rsrc(seg, 0, (int)(4 * (4 * T)), 0x00020000)};
    // byte offsets of the arrays (from voxel 0 of WX) and of the backward
    // neighbours: uniform (stated, so that no copy of them computed in the
    // weights loop above, whose trip count differs per lane, is taken as
    // per-lane)
    const int sWX = __builtin_amdgcn_readfirstlane(4 * nxy), sWY = __builtin_amdgcn_readfirstlane(sWX + 4 * T),
              sWZ = __builtin_amdgcn_readfirstlane(sWY + 4 * T), sID = __builtin_amdgcn_readfirstlane(sWZ + 4 * T);
    const int sWXm = sWX - 4, sWYm = __builtin_amdgcn_readfirstlane(sWY - 4 * nx),
              sWZm = __builtin_amdgcn_readfirstlane(sWZ - 4 * nxy);

    float x[VPT], r[VPT], q[VPT];
    double rz, rr, bb;
    if (fused) {
        // its barriers also make the weights written above visible to the workgroup
        if (!res_start_finish<NT>(sum, nv, m, xb, rw, P, red, st, rz, rr, bb))
            return;  // nothing to iterate (state and x written)
    }
    {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v0 = threadIdx.x + k * NT;
            const int v = v0 < nv ? v0 : nv - 1;
            const bool u = v0 < nv && m[v] == 0;
            const float rv = rb[v], xv = xb[v];
            r[k] = u ? rv : 0.0f;
            x[k] = u ? xv : 0.0f;
        }
        if (!fused) {
            // the weights written above are read by other threads of the workgroup
            __syncthreads();
            rz = st.rz[0];
            rr = st.rr[0];
            bb = st.bb[0];
        }
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) q[k] = r[k] * sb.ld(4u * (unsigned)(threadIdx.x + k * NT), sID);  // start z

    const double tol = corr ? a.inner_tol : a.tol;
    const double tol2 = tol * tol;
    double betac = 0.0;
    float wr[2][G][3];  // forward weights of two groups of voxels
    float ir[2][G];     // 1/d of two groups
    int it = 0, flags = 0;
    for (;;) {
        if (rr <= tol2 * bb) break;
        if (it >= a.max_iter) {
            flags = 2;
            break;
        }
        // opaque copies: per-voxel addresses stay inside the loop
        int tb = threadIdx.x, oy = nx, oz = nxy;
        asm volatile("" : "+v"(tb));
        asm volatile("" : "+v"(oy));
        asm volatile("" : "+v"(oz));
        // byte offsets of a group's slots, from an opaque per-group base (so
        // that the compiler keeps no per-slot offset beyond its group)
        const unsigned o0 = 4u * (unsigned)tb;
        auto group_base = [&](int gi, unsigned ob) {
            unsigned og = ob + 4u * (unsigned)(gi * G * NT);
            asm volatile("" : "+v"(og));
            return og;
        };
        // forward weights (from the Infinity Cache: issued a group ahead)
        auto load_w = [&](int gi, float (&w)[G][3]) {
            const unsigned og = group_base(gi, o0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (gi * G + j < VPT) {
                    const unsigned o = og + 4u * (unsigned)(j * NT);
                    w[j][0] = sb.ld(o, sWX);
                    w[j][1] = sb.ld(o, sWY);
                    w[j][2] = sb.ld(o, sWZ);
                }
            }
        };
        // backward weights: lines the forward loads of this or a neighbouring
        // lane or wave just brought into L1, loaded when the group is computed
        auto load_b = [&](int gi, float (&w)[G][3]) {
            const unsigned og = group_base(gi, o0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (gi * G + j < VPT) {
                    const unsigned o = og + 4u * (unsigned)(j * NT);
                    w[j][0] = sb.ld(o, sWXm);
                    w[j][1] = sb.ld(o, sWYm);
                    w[j][2] = sb.ld(o, sWZm);
                }
            }
        };
        auto load_i = [&](int gi, float (&w)[G], unsigned ob) {
            const unsigned og = group_base(gi, ob);
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (gi * G + j < VPT) w[j] = sb.ld(og + 4u * (unsigned)(j * NT), sID);
        };
        load_w(0, wr[0]);
        const float be = it == 0 ? 0.0f : (float)betac;
        float* const Pt = P + tb;
        // p = z + beta p (z = 0 and p = 0 on seeded and unused slots), in
        // groups of 8 so that the compiler does not read all p first
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            Pt[k * NT] = q[k] + be * Pt[k * NT];
            if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        res_lds_barrier();
        const float* const Pxm = Pt - 1;
        const float* const Pym = Pt - oy;
        const float* const Pyp = Pt + oy;
        const float* const Pzm = Pt - oz;
        const float* const Pzp = Pt + oz;
        double sig = 0.0;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            // this group's backward loads go first: waiting for them must not
            // wait for the next group's forward loads (loads complete in order)
            float wb[G][3];
            load_b(gi, wb);
            __builtin_amdgcn_sched_barrier(0);
            if (gi + 1 < NG) load_w(gi + 1, wr[(gi + 1) & 1]);
            else load_i(0, ir[0], o0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int k = gi * G + j;
                if (k < VPT) {
                    const float wxp = wr[gi & 1][j][0], wyp = wr[gi & 1][j][1], wzp = wr[gi & 1][j][2];
                    const float wxm = wb[j][0], wym = wb[j][1], wzm = wb[j][2];
                    const float d = ((wxp + wxm) + (wyp + wym)) + (wzp + wzm);
                    const float pv = Pt[k * NT];
                    const float acc = wxp * Pxm[k * NT + 2] + wxm * Pxm[k * NT] + wyp * Pyp[k * NT] +
                                      wym * Pym[k * NT] + wzp * Pzp[k * NT] + wzm * Pzm[k * NT];
                    q[k] = d * pv - acc;  // masked in the update below
                    sig += (double)pv * (double)q[k];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        double s1[1] = {sig};
        res_block_sum_lds<NT, 1>(s1, red);
        sig = s1[0];
        const double alpha = rz / sig;
        if (!res_finite(alpha) || !(sig > 0.0)) {
            flags = 1;
            break;
        }
        const float al = (float)alpha;
        double acc2[2] = {0.0, 0.0};
        // fresh opaque copy: no per-voxel address lives across the reduction
        int t3 = threadIdx.x;
        asm volatile("" : "+v"(t3));
        const unsigned o3 = 4u * (unsigned)t3;
        const float* const P3 = P + t3;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            if (gi + 1 < NG) load_i(gi + 1, ir[(gi + 1) & 1], o3);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int k = gi * G + j;
                if (k < VPT) {
                    const float id = ir[gi & 1][j];
                    const float pv = P3[k * NT];
                    // p = 0 on seeded and unused slots; r stays 0 there (1/d = 0)
                    x[k] += al * pv;
                    // pin the update here: sunk below the reduction it would
                    // keep every p value of the pass live
                    asm volatile("" : "+v"(x[k]));
                    const float rn = r[k] - al * q[k];
                    r[k] = id != 0.0f ? rn : 0.0f;
                    const float z = r[k] * id;
                    q[k] = z;
                    acc2[0] += (double)r[k] * (double)z;
                    acc2[1] += (double)r[k] * (double)r[k];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        res_block_sum_lds<NT, 2>(acc2, red);
        ++it;
        if (!res_finite(acc2[0]) || !res_finite(acc2[1])) {
            flags = 1;
            break;
        }
        betac = acc2[0] / rz;
        rz = acc2[0];
        rr = acc2[1];
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = threadIdx.x + k * NT;
        if (v < nv && m[v] == 0) xb[v] = x[k];
    }
    if (threadIdx.x == 0) {
        st.rz[0] = rz;
        st.rr[0] = rr;
        if (corr) {
            st.refine_iters += it;
        } else {
            st.iters = it;
            st.rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            if (flags & 2) st.status = RW_ST_MAX_ITER;
        }
        if (flags & 1) st.status = RW_ST_NONFINITE;
        st.pending = corr && !(flags & 1) ? 1 : 0;
    }
}

// One workgroup per box.
template <int NT, int VPT, int G>
__global__ __launch_bounds__(NT) void k_pcg_resg(SolveArgs a, float* xt, int corr, int base, int, uint32_t*) {
    resg_box<NT, VPT, G>(a, xt, corr, base + (int)blockIdx.x);
}

// Launches with 32 x 32 planes: each thread owns four consecutive voxels per
// group, voxels 4 (t + NT j) + i (i < 4, j < NGR, t + NT j < NG, the span's
// NG groups), so p, the weights and 1/d move as 16-byte loads: per group one
// LDS load of p, two scalar ones (the x neighbours outside the group) and
// four of the y and z neighbour groups, three forward-weight loads, one
// backward x weight and two backward y and z groups from the segment.  The
// iteration is the one of resg_box, voxel for voxel in the same order of
// operations; only the per-thread FP64 partial sums run over other voxels.
// When NG is not a multiple of NT the last group belongs to the first
// NG mod NT threads, a whole number of waves.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct SegBuf4 {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ float4 ld(unsigned vo, int so) const {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)vo, so, 0);
        return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
    }
    __device__ __forceinline__ float ld1(unsigned vo, int so) const {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)vo, so, 0));
    }
};

__device__ __forceinline__ float f4c(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

template <int NT, int NGR, int NG>
__device__ __forceinline__ void resg4_box(const SolveArgs& a, float* xt, int corr, int ib) {
    extern __shared__ __align__(16) float p_lds[];
    __shared__ double red[(NT / 64) * 5];
    constexpr int PX = 32, NXY = PX * PX;
    static_assert(NGR == (NG + NT - 1) / NT && (NG % NT) % 64 == 0, "groups per thread, whole waves in the last");
    constexpr int span = 4 * NG;
    BoxState& st = a.state[ib];
    const bool fused = a.fused_init && !corr;
    if (!fused && !st.active) return;
    const BrickDev bd = a.bricks[ib];
    const int nz = bd.nz, nv = NXY * nz;
    const int T = NXY + span;
    float* const P = p_lds + NXY;
    float4* const P4 = (float4*)P;  // group k of the box: voxels 4k .. 4k + 3
    const float* g = a.g + bd.off;
    const uint8_t* m = a.mask + bd.off;
    float* const xb = xt + bd.off;
    const float* rb = (const float*)a.r + bd.off;
    float* const seg = a.wts + bd.woff;
    float* const WX = seg + NXY;
    float* const WY = WX + T;
    float* const WZ = WY + T;
    float* const ID = WZ + T;
    const ResWeight W{(float)(-a.beta * 1.4426950408889634), (float)a.eps};

    res_fill_p<NT, 8>(P, xb, -NXY, span + NXY, nv, fused);
    if (fused) __syncthreads();
    float* const rw = (float*)a.r + bd.off;
    double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    res_weights_pass<NT, 8>(-NXY, span, PX, PX, nz, g, m, W, true, fused, P, rw, sum,
                            [&](int v, float wx, float wy, float wz, float d, bool unk) {
                                WX[v] = wx;
                                WY[v] = wy;
                                WZ[v] = wz;
                                ID[v] = unk ? __builtin_amdgcn_rcpf(d) : 0.0f;
                            });
    // (the segment, its arrays 16-byte aligned: its offset in the weight
    // buffer is a whole number of 256-byte lines, and nx*ny and the stride
    // are multiples of four floats)
    const SegBuf4 sb{__builtin_amdgcn_make_buffer_rsrc(seg, 0, (int)(4 * (4 * T)), 0x00020000)};
    const int sWX = __builtin_amdgcn_readfirstlane(4 * NXY), sWY = __builtin_amdgcn_readfirstlane(sWX + 4 * T),
              sWZ = __builtin_amdgcn_readfirstlane(sWY + 4 * T), sID = __builtin_amdgcn_readfirstlane(sWZ + 4 * T);
    const int sWXm = sWX - 4, sWYm = __builtin_amdgcn_readfirstlane(sWY - 4 * PX),
              sWZm = __builtin_amdgcn_readfirstlane(sWZ - 4 * NXY);

    float4 x[NGR], r[NGR], q[NGR];
    double rz, rr, bb;
    if (fused) {
        if (!res_start_finish<NT>(sum, nv, m, xb, rw, P, red, st, rz, rr, bb)) return;
    }
    {
#pragma unroll
        for (int j = 0; j < NGR; ++j) {
            float rv4[4], xv4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v0 = 4 * ((int)threadIdx.x + j * NT) + i;
                const int v = v0 < nv ? v0 : nv - 1;
                const bool u = v0 < nv && m[v] == 0;
                const float rv = rb[v], xv = xb[v];
                rv4[i] = u ? rv : 0.0f;
                xv4[i] = u ? xv : 0.0f;
            }
            r[j] = make_float4(rv4[0], rv4[1], rv4[2], rv4[3]);
            x[j] = make_float4(xv4[0], xv4[1], xv4[2], xv4[3]);
            if ((j & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
        if (!fused) {
            __syncthreads();
            rz = st.rz[0];
            rr = st.rr[0];
            bb = st.bb[0];
        }
    }
#pragma unroll
    for (int j = 0; j < NGR; ++j) {
        const float4 id = sb.ld(16u * (unsigned)(threadIdx.x + j * NT), sID);
        q[j] = make_float4(r[j].x * id.x, r[j].y * id.y, r[j].z * id.z, r[j].w * id.w);  // start z
    }

    const double tol = corr ? a.inner_tol : a.tol;
    const double tol2 = tol * tol;
    double betac = 0.0;
    float4 wr[2][3];  // forward weights of two groups
    float4 ir[2];     // 1/d of two groups
    // this thread owns group NGR - 1 (the loads of a group it does not own
    // stay inside the segment and go unused)
    const bool last = NG % NT == 0 || (int)threadIdx.x < NG % NT;
    int it = 0, flags = 0;
    for (;;) {
        if (rr <= tol2 * bb) break;
        if (it >= a.max_iter) {
            flags = 2;
            break;
        }
        int tb = threadIdx.x;
        asm volatile("" : "+v"(tb));
        const unsigned o0 = 16u * (unsigned)tb;
        auto group_base = [&](int j, unsigned ob) {
            unsigned og = ob + 16u * (unsigned)(j * NT);
            asm volatile("" : "+v"(og));
            return og;
        };
        auto load_w = [&](int j, float4 (&w)[3]) {
            const unsigned og = group_base(j, o0);
            w[0] = sb.ld(og, sWX);
            w[1] = sb.ld(og, sWY);
            w[2] = sb.ld(og, sWZ);
        };
        load_w(0, wr[0]);
        const float be = it == 0 ? 0.0f : (float)betac;
        float4* const Pt = P4 + tb;
#pragma unroll
        for (int j = 0; j < NGR; ++j) {
            if (j == NGR - 1 && !last) continue;
            const float4 pv = Pt[j * NT];
            Pt[j * NT] = make_float4(q[j].x + be * pv.x, q[j].y + be * pv.y, q[j].z + be * pv.z, q[j].w + be * pv.w);
            if ((j & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
        res_lds_barrier();
        const float* const Ps = P + 4 * tb;  // first voxel of group 0
        double sig = 0.0;
#pragma unroll
        for (int j = 0; j < NGR; ++j) {
            // this group's backward loads first, then the next group's forward ones
            const unsigned og = group_base(j, o0);
            const float wxm0 = sb.ld1(og, sWXm);
            const float4 wym = sb.ld(og, sWYm);
            const float4 wzm = sb.ld(og, sWZm);
            __builtin_amdgcn_sched_barrier(0);
            if (j + 1 < NGR) load_w(j + 1, wr[(j + 1) & 1]);
            else ir[0] = sb.ld(o0, sID);
            __builtin_amdgcn_sched_barrier(0);
            if (j == NGR - 1 && !last) continue;
            const float4 wx = wr[j & 1][0], wy = wr[j & 1][1], wz = wr[j & 1][2];
            const float4 pv = Pt[j * NT];
            const float pxm = Ps[4 * j * NT - 1], pxp = Ps[4 * j * NT + 4];
            const float4 pym = Pt[j * NT - PX / 4], pyp = Pt[j * NT + PX / 4];
            const float4 pzm = Pt[j * NT - NXY / 4], pzp = Pt[j * NT + NXY / 4];
            float qv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float wxp = f4c(wx, i), wyp = f4c(wy, i), wzp = f4c(wz, i);
                const float wxmi = i == 0 ? wxm0 : f4c(wx, i - 1);
                const float wymi = f4c(wym, i), wzmi = f4c(wzm, i);
                const float d = ((wxp + wxmi) + (wyp + wymi)) + (wzp + wzmi);
                const float p0 = f4c(pv, i);
                const float pl = i == 0 ? pxm : f4c(pv, i - 1);
                const float pr = i == 3 ? pxp : f4c(pv, i + 1);
                const float acc = wxp * pr + wxmi * pl + wyp * f4c(pyp, i) + wymi * f4c(pym, i) + wzp * f4c(pzp, i) +
                                  wzmi * f4c(pzm, i);
                qv[i] = d * p0 - acc;  // masked in the update below
                sig += (double)p0 * (double)qv[i];
            }
            q[j] = make_float4(qv[0], qv[1], qv[2], qv[3]);
            __builtin_amdgcn_sched_barrier(0);
        }
        double s1[1] = {sig};
        res_block_sum_lds<NT, 1>(s1, red);
        sig = s1[0];
        const double alpha = rz / sig;
        if (!res_finite(alpha) || !(sig > 0.0)) {
            flags = 1;
            break;
        }
        const float al = (float)alpha;
        double acc2[2] = {0.0, 0.0};
        int t3 = threadIdx.x;
        asm volatile("" : "+v"(t3));
        const unsigned o3 = 16u * (unsigned)t3;
        const float4* const P3 = P4 + t3;
#pragma unroll
        for (int j = 0; j < NGR; ++j) {
            if (j + 1 < NGR) ir[(j + 1) & 1] = sb.ld(group_base(j + 1, o3), sID);
            __builtin_amdgcn_sched_barrier(0);
            if (j == NGR - 1 && !last) continue;
            const float4 id = ir[j & 1];
            const float4 pv = P3[j * NT];
            x[j] = make_float4(x[j].x + al * pv.x, x[j].y + al * pv.y, x[j].z + al * pv.z, x[j].w + al * pv.w);
            asm volatile("" : "+v"(x[j].x), "+v"(x[j].y), "+v"(x[j].z), "+v"(x[j].w));
            float rn[4], zn[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float idi = f4c(id, i);
                const float rr0 = f4c(r[j], i) - al * f4c(q[j], i);
                rn[i] = idi != 0.0f ? rr0 : 0.0f;
                zn[i] = rn[i] * idi;
                acc2[0] += (double)rn[i] * (double)zn[i];
                acc2[1] += (double)rn[i] * (double)rn[i];
            }
            r[j] = make_float4(rn[0], rn[1], rn[2], rn[3]);
            q[j] = make_float4(zn[0], zn[1], zn[2], zn[3]);
            __builtin_amdgcn_sched_barrier(0);
        }
        res_block_sum_lds<NT, 2>(acc2, red);
        ++it;
        if (!res_finite(acc2[0]) || !res_finite(acc2[1])) {
            flags = 1;
            break;
        }
        betac = acc2[0] / rz;
        rz = acc2[0];
        rr = acc2[1];
    }
    int te = (int)threadIdx.x;
    asm volatile("" : "+v"(te));
#pragma unroll
    for (int j = 0; j < NGR; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = 4 * (te + j * NT) + i;
            if (v < nv && m[v] == 0) xb[v] = f4c(x[j], i);
        }
    }
    if (threadIdx.x == 0) {
        st.rz[0] = rz;
        st.rr[0] = rr;
        if (corr) {
            st.refine_iters += it;
        } else {
            st.iters = it;
            st.rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            if (flags & 2) st.status = RW_ST_MAX_ITER;
        }
        if (flags & 1) st.status = RW_ST_NONFINITE;
        st.pending = corr && !(flags & 1) ? 1 : 0;
    }
}

template <int NT, int NGR, int NG>
__global__ __launch_bounds__(NT) void k_pcg_resg4(SolveArgs a, float* xt, int corr, int base, int, uint32_t*) {
    resg4_box<NT, NGR, NG>(a, xt, corr, base + (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Split boxes: two workgroups per box (k_pcg_res2).
//
// A 40^3 box (a brick of 32^3 expanded by 1.25, Section IV-B) needs 250 KB
// for p alone, more than one CU's LDS.  Cut along z, each half (up to 32768
// voxels) fits the streamed-weights layout above: p of the half in LDS, x, r
// and q in registers, the half's edge weights and 1/d in a segment of its
// own.  The upper half's voxels take slots 0.., the lower half's end at the
// last slot, so that the other half's plane at the cut falls in the LDS pad
// below (upper) or above (lower) the slots, and every stencil access is as
// in k_pcg_resg.  Per CG iteration the halves exchange two messages through
// a per-box mailbox in global memory: their parts of p.q (giving alpha), then
// their parts of r.z and ||r||^2 with z on their plane at the cut (giving
// beta; each half then forms the other's new p at the cut itself, with the
// same fused multiply-add, so the halo needs no message of its own).  Both
// halves add the two parts in the same order and so take the same decisions
// (convergence, breakdown, iteration cap) and leave together.
//
// Mailbox words are written and read with device-scope atomic accesses; a
// message's stores are complete (s_waitcnt) before its flag is written, and
// its words are read after the flag is seen, so no cache is flushed.  A
// message n >= 1 sits in buffer n & 1: the start message (odd) and each
// iteration's p.q (even) and r.z message (odd) with the plane; a buffer is
// written again only after the other half has answered the message in
// between, by which time it has read the first.

struct PairBox {
    char* base;
    __device__ uint32_t* flag(int h) const { return (uint32_t*)(base + 128 * h); }
    __device__ uint64_t* part(int h, int b) const { return (uint64_t*)(base + 256 + 64 * (2 * h + b)); }
    // z at the cut, then one spare word per thread
    __device__ uint32_t* plane(int h) const { return (uint32_t*)(base + 512 + 4 * (kPairMaxPlane + kResThreads) * h); }
};
static_assert(512 + 8 * (kPairMaxPlane + kResThreads) <= kPairMailboxElems * 4, "mailbox size");

__device__ __forceinline__ void dev_st(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t dev_ld(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dev_st64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t dev_ld64(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls of the other half's flag before a half gives up (a few seconds).
constexpr uint32_t kPairSpin = 1u << 22;

// Message n of half h: the NV sums v (equal on every thread) go out and the
// other half's come back in o (equal on every thread); the plane stores of
// this message were issued before the call.  Every wave polls the other
// half's flag itself (a uniform loop); false on every thread when some wave
// saw no answer within kPairSpin polls.
template <int NV>
__device__ __forceinline__ bool pair_exchange(const PairBox& mb, int h, uint32_t n, const double (&v)[NV],
                                              double (&o)[NV]) {
    const int b = (int)(n & 1u);
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) dev_st64(mb.part(h, b) + k, (uint64_t)__double_as_longlong(v[k]));
    __builtin_amdgcn_s_waitcnt(0);  // this thread's mailbox stores have completed
    __syncthreads();                // and every thread's
    if (threadIdx.x == 0) dev_st(mb.flag(h), n);
    int late = 0;
    for (uint32_t spins = 0; __builtin_amdgcn_readfirstlane(dev_ld(mb.flag(h ^ 1))) < n;) {
        if (++spins > kPairSpin) {
            late = 1;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    // (no early return: a branch out of the caller's iteration here costs
    // that loop registers; the caller stops at its next convergence test)
    const bool lost = __syncthreads_or(late) != 0;
    for (int k = 0; k < NV; ++k) {
        const double w = __longlong_as_double((long long)dev_ld64(mb.part(h ^ 1, b) + k));
        o[k] = lost ? 0.0 : w;
    }
    return !lost;
}

// Floats of one half's segment (four arrays of nxy + span) and of a split
// box's weight area (two halves and the mailbox).
__host__ __device__ inline int64_t split_half_elems(int64_t nxy) {
    return (4 * (nxy + kResSpanG1) + 63) & ~int64_t(63);
}

template <int NT, int VPT, int G>
__device__ __forceinline__ void res2_half(const SolveArgs& a, float* xt, int corr, int ib, int h) {
    extern __shared__ __align__(16) float p_lds[];
    __shared__ double red[(NT / 64) * 5];
    constexpr int NG = (VPT + G - 1) / G;
    constexpr int span = NT * VPT;
    constexpr int U = 8;  // slots per thread at a time in the weights pass
    constexpr int kPlaneSlots = (kPairMaxPlane + NT - 1) / NT;  // a thread's slots on a plane at the cut
    static_assert(span == kResSpanG1, "split halves use the 32768-slot layout");
    BoxState& st = a.state[ib];
    const bool fused = a.fused_init && !corr;
    if (!fused && !st.active) return;  // both halves read the same flag
    const BrickDev bd = a.bricks[ib];
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz, nxy = nx * ny;
    const int z0 = (nz + 1) >> 1;           // planes of the lower half
    const int zh = h ? nz - z0 : z0;        // planes of this half
    const int nv = nxy * zh;                // its voxels
    const int S = h ? 0 : span - nv;        // slot of its first voxel
    const int goff = h ? z0 * nxy : 0;      // box voxel of its first voxel
    const int hb = h ? -nxy : span;         // slots of the other half's plane at the cut (the halo)
    const int bs = h ? 0 : span - nxy;      // slots of this half's plane at the cut
    const int T = nxy + span;
    float* P = p_lds + nxy;
    // the half's voxel v (slot v + S) is box voxel goff + v
    const float* g = a.g + bd.off + goff;
    const uint8_t* m = a.mask + bd.off + goff;
    float* const xb = xt + bd.off + goff;
    float* const rw = (float*)a.r + bd.off + goff;
    const int64_t he = split_half_elems(nxy);
    float* const seg = a.wts + bd.woff + h * he;
    float* const WX = seg + nxy;
    float* const WY = WX + T;
    float* const WZ = WY + T;
    float* const ID = WZ + T;
    const PairBox mb{(char*)(a.wts + bd.woff + 2 * he)};
    const ResWeight W{(float)(-a.beta * 1.4426950408889634), (float)a.eps};
    // local voxels with x in P for the start state: the half and the halo
    const int vlo = h ? -nxy : 0, vhi = h ? nv : nv + nxy;

    // P over [-nxy, span + nxy): x of the half's voxels and of the halo for
    // a main solve's start state, 0 elsewhere
    for (int s = -nxy + (int)threadIdx.x; s < span + nxy; s += NT) {
        const int v = s - S;
        float xv = 0.0f;
        if (fused && v >= vlo && v < vhi) xv = xb[v];
        P[s] = xv;
    }
    if (fused) __syncthreads();
    double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // r.z, r.r, b.b, unknown, seeded
    // Weights pass over the slots [-nxy, span) (thread t: -nxy + t + k * NT),
    // U at a time with all their loads issued first: the forward weights
    // w+x, w+y, w+z (0 toward neighbours outside the box and on slots
    // outside the half) and 1/d (0 on seeded voxels and outside the half);
    // in the upper half's pad plane, the weight of the edge across the cut.
    // A main solve also forms the start state (r0 = sum_nb w x_nb - d x, the
    // sums) as res_weights_pass does; neighbours across the cut are in box.
    for (int s0 = -nxy + (int)threadIdx.x; s0 < span; s0 += U * NT) {
        int c[U];
        bool in[U][6];
        float gc[U], gn[U][6];
        uint8_t mc[U], mn[U][6];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + u * NT;
            const int v = s - S;
            // a voxel of the half, the upper half's pad plane, or (unused
            // slots) voxel 0
            c[u] = v >= 0 && v < nv ? v : (h && s < 0 ? v : 0);
            const int kz = c[u] >= 0 ? c[u] / nxy : -1, rem = c[u] - kz * nxy, j = rem / nx, i = rem - j * nx;
            const int no[6] = {1, -1, nx, -nx, nxy, -nxy};
            in[u][0] = i + 1 < nx;
            in[u][1] = i > 0;
            in[u][2] = j + 1 < ny;
            in[u][3] = j > 0;
            in[u][4] = kz + 1 < zh || !h;  // (the lower half's top plane faces the upper half)
            in[u][5] = kz > 0 || (h && kz == 0);  // (the upper half's first plane faces the lower half)
            gc[u] = g[c[u]];
            mc[u] = m[c[u]];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int nb = in[u][e] ? c[u] + no[e] : c[u];
                gn[u][e] = g[nb];
                mn[u][e] = m[nb];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + u * NT;
            const int v = s - S;
            const bool inb = v >= 0 && v < nv;
            float w[6];  // +x, -x, +y, -y, +z, -z
#pragma unroll
            for (int e = 0; e < 6; ++e) w[e] = 0.0f;
            if (inb) {
#pragma unroll
                for (int e = 0; e < 6; e += 2)
                    if (in[u][e]) w[e] = W(gc[u], gn[u][e]);
#pragma unroll
                for (int e = 1; e < 6; e += 2)
                    if (in[u][e]) w[e] = W(gn[u][e], gc[u]);
            } else if (h && s < 0) {
                w[4] = W(gc[u], gn[u][4]);  // the edge across the cut
            }
            const float d = ((w[0] + w[2]) + w[4]) + w[1] + w[3] + w[5];
            const bool unk = inb && mc[u] == 0;
            if (s < span) {
                WX[s] = w[0];
                WY[s] = w[2];
                WZ[s] = w[4];
                ID[s] = unk ? __builtin_amdgcn_rcpf(d) : 0.0f;
            }
            if (fused && inb) {
                const int no[6] = {1, -1, nx, -nx, nxy, -nxy};
                float acc = 0.0f, bs2 = 0.0f;  // sum_nb w x_nb, and over the seeded neighbours only
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    const float xr = P[s + no[e]];
                    const float xn = in[u][e] ? xr : 0.0f;
                    acc += w[e] * xn;
                    if (mn[u][e] != 0) bs2 += w[e] * xn;
                }
                const float r0 = unk ? acc - d * P[s] : 0.0f;
                rw[v] = r0;
                if (unk) {
                    sum[0] += (double)r0 * (double)(r0 * __builtin_amdgcn_rcpf(d));
                    sum[1] += (double)r0 * (double)r0;
                    sum[2] += (double)bs2 * (double)bs2;
                }
                sum[3] += unk ? 1.0 : 0.0;
                sum[4] += unk ? 0.0 : 1.0;
            }
        }
    }
    res_block_sum<NT, 5>(sum, red);  // its barriers also publish rw and the segment to the workgroup

    // a correction solve starts from the box's state (read before the start
    // message: the lower half rewrites it when it ends)
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (!fused) {
        rz = st.rz[0];
        rr = st.rr[0];
        bb = st.bb[0];
    }
    // x, r and the start z on this half's slots; z on its plane at the cut
    // goes to the other half with the start sums
    float x[VPT], r[VPT], q[VPT];
    uint32_t* const pl_out = mb.plane(h);
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int s = threadIdx.x + k * NT;
        const int v0 = s - S;
        const int v = v0 < 0 ? 0 : v0 < nv ? v0 : nv - 1;
        const uint8_t mv = m[v];
        const float rv = rw[v], xv = xb[v];
        const bool u = v0 >= 0 && v0 < nv && mv == 0;
        r[k] = u ? rv : 0.0f;
        x[k] = u ? xv : 0.0f;
    }
    // 0x00020000: raw 32-bit buffer (third descriptor word for this chip family)
    const SegBuf sb{__builtin_amdgcn_make_buffer_rsrc(seg, 0, (int)(4 * (4 * T)), 0x00020000)};
    const int sWX = __builtin_amdgcn_readfirstlane(4 * nxy), sWY = __builtin_amdgcn_readfirstlane(sWX + 4 * T),
              sWZ = __builtin_amdgcn_readfirstlane(sWY + 4 * T), sID = __builtin_amdgcn_readfirstlane(sWZ + 4 * T);
    const int sWXm = sWX - 4, sWYm = __builtin_amdgcn_readfirstlane(sWY - 4 * nx),
              sWZm = __builtin_amdgcn_readfirstlane(sWZ - 4 * nxy);
    // start z (the 1/d of unused and seeded slots is 0)
#pragma unroll
    for (int k = 0; k < VPT; ++k) q[k] = r[k] * sb.ld(4u * (unsigned)(threadIdx.x + k * NT), sID);
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        if (k < kPlaneSlots || k >= VPT - kPlaneSlots) {
            const unsigned o = (unsigned)((int)threadIdx.x + k * NT - bs);
            dev_st(pl_out + (o < (unsigned)nxy ? o : (unsigned)(kPairMaxPlane + threadIdx.x)), __float_as_uint(q[k]));
        }
    }
    double tot[5];
    {
        double o[5];
        if (!pair_exchange<5>(mb, h, 1u, sum, o)) {
            if (threadIdx.x == 0 && h == 0) {
                st.status = RW_ST_SYNC_LOST;
                st.active = 0;
                st.pending = 0;
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) tot[k] = h == 0 ? sum[k] + o[k] : o[k] + sum[k];
    }
    if (fused) {
        // reset P (the halo held the other half's x) and settle the box's
        // state as res_start_finish does, on the two halves' sums
        for (int s = -nxy + (int)threadIdx.x; s < span + nxy; s += NT) P[s] = 0.0f;
        const double nU = tot[3], nM = tot[4];
        const bool allzero = tot[2] == 0.0;
        const bool act = nM > 0.0 && nU > 0.0 && !allzero;
        const bool zero_sol = nM > 0.0 && nU > 0.0 && allzero;
        rz = zero_sol ? 0.0 : tot[0];
        rr = zero_sol ? 0.0 : tot[1];
        bb = tot[2];
        if (zero_sol)
            for (int v = threadIdx.x; v < nv; v += NT)
                if (m[v] == 0) xb[v] = rw[v] = 0.0f;
        if (threadIdx.x == 0 && h == 0) {
            for (int cc = 0; cc < 3; ++cc) st.rz[cc] = st.rr[cc] = st.bb[cc] = 0.0;
            st.rz[0] = rz;
            st.rr[0] = rr;
            st.bb[0] = bb;
            st.nU = nU;
            st.nM = nM;
            st.rel = 0.0;
            st.true_rel = 0.0;
            st.iters = st.refine_steps = st.refine_iters = 0;
            st.status = nM == 0.0 ? RW_ST_NO_DIRICHLET : RW_ST_CONVERGED;
            st.active = act ? 1 : 0;
            st.pending = 0;
            st.checked = 0;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(act ? 1 : 0)) return;
    }

    uint32_t* const pl_in = mb.plane(h ^ 1);

    const double tol = corr ? a.inner_tol : a.tol;
    const double tol2 = tol * tol;
    double betac = 0.0;
    float wr[2][G][3];
    float ir[2][G];
    int it = 0, flags = 0;
    uint32_t msg = 1;
    for (;;) {
        if (flags & 4) break;  // the other half stopped answering
        if (rr <= tol2 * bb) break;
        if (it >= a.max_iter) {
            flags = 2;
            break;
        }
        int tb = threadIdx.x, oy = nx, oz = nxy;
        asm volatile("" : "+v"(tb));
        asm volatile("" : "+v"(oy));
        asm volatile("" : "+v"(oz));
        const unsigned o0 = 4u * (unsigned)tb;
        auto group_base = [&](int gi, unsigned ob) {
            unsigned og = ob + 4u * (unsigned)(gi * G * NT);
            asm volatile("" : "+v"(og));
            return og;
        };
        auto load_w = [&](int gi, float (&w)[G][3]) {
            const unsigned og = group_base(gi, o0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (gi * G + j < VPT) {
                    const unsigned o = og + 4u * (unsigned)(j * NT);
                    w[j][0] = sb.ld(o, sWX);
                    w[j][1] = sb.ld(o, sWY);
                    w[j][2] = sb.ld(o, sWZ);
                }
            }
        };
        auto load_b = [&](int gi, float (&w)[G][3]) {
            const unsigned og = group_base(gi, o0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (gi * G + j < VPT) {
                    const unsigned o = og + 4u * (unsigned)(j * NT);
                    w[j][0] = sb.ld(o, sWXm);
                    w[j][1] = sb.ld(o, sWYm);
                    w[j][2] = sb.ld(o, sWZm);
                }
            }
        };
        auto load_i = [&](int gi, float (&w)[G], unsigned ob) {
            const unsigned og = group_base(gi, ob);
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (gi * G + j < VPT) w[j] = sb.ld(og + 4u * (unsigned)(j * NT), sID);
        };
        load_w(0, wr[0]);
        const float be = it == 0 ? 0.0f : (float)betac;
        float* const Pt = P + tb;
        // p = z + beta p on this half's slots and, from the other half's z,
        // on its plane at the cut (the halo), with the multiply-add that half
        // uses there
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            Pt[k * NT] = __builtin_fmaf(be, Pt[k * NT], q[k]);
            if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        for (int i = tb; i < nxy; i += NT)
            P[hb + i] = __builtin_fmaf(be, P[hb + i], __uint_as_float(dev_ld(pl_in + i)));
        res_lds_barrier();
        const float* const Pxm = Pt - 1;
        const float* const Pym = Pt - oy;
        const float* const Pyp = Pt + oy;
        const float* const Pzm = Pt - oz;
        const float* const Pzp = Pt + oz;
        double sig = 0.0;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            float wb[G][3];
            load_b(gi, wb);
            __builtin_amdgcn_sched_barrier(0);
            if (gi + 1 < NG) load_w(gi + 1, wr[(gi + 1) & 1]);
            else load_i(0, ir[0], o0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int k = gi * G + j;
                if (k < VPT) {
                    const float wxp = wr[gi & 1][j][0], wyp = wr[gi & 1][j][1], wzp = wr[gi & 1][j][2];
                    const float wxm = wb[j][0], wym = wb[j][1], wzm = wb[j][2];
                    const float d = ((wxp + wxm) + (wyp + wym)) + (wzp + wzm);
                    const float pv = Pt[k * NT];
                    const float acc = wxp * Pxm[k * NT + 2] + wxm * Pxm[k * NT] + wyp * Pyp[k * NT] +
                                      wym * Pym[k * NT] + wzp * Pzp[k * NT] + wzm * Pzm[k * NT];
                    q[k] = d * pv - acc;  // masked in the update below
                    sig += (double)pv * (double)q[k];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        double s1[1] = {sig};
        res_block_sum_lds<NT, 1>(s1, red);
        {
            double o1[1];
            flags |= pair_exchange<1>(mb, h, ++msg, s1, o1) ? 0 : 4;
            sig = h == 0 ? s1[0] + o1[0] : o1[0] + s1[0];
        }
        const double alpha = rz / sig;
        if (!res_finite(alpha) || !(sig > 0.0)) {
            flags |= 1;
            break;
        }
        const float al = (float)alpha;
        double acc2[2] = {0.0, 0.0};
        int t3 = threadIdx.x;
        asm volatile("" : "+v"(t3));
        const unsigned o3 = 4u * (unsigned)t3;
        const float* const P3 = P + t3;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            if (gi + 1 < NG) load_i(gi + 1, ir[(gi + 1) & 1], o3);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int k = gi * G + j;
                if (k < VPT) {
                    const float id = ir[gi & 1][j];
                    const float pv = P3[k * NT];
                    x[k] += al * pv;
                    asm volatile("" : "+v"(x[k]));
                    const float rn = r[k] - al * q[k];
                    r[k] = id != 0.0f ? rn : 0.0f;
                    const float z = r[k] * id;
                    q[k] = z;
                    acc2[0] += (double)r[k] * (double)z;
                    acc2[1] += (double)r[k] * (double)r[k];
                    // z on this half's plane at the cut, for the other
                    // half's p there (only the first and last slots of a
                    // thread can be on it)
                    if (k < kPlaneSlots || k >= VPT - kPlaneSlots) {
                        // (slots off the plane write the thread's spare word: no branch)
                        const unsigned o = (unsigned)(t3 + k * NT - bs);
                        dev_st(pl_out + (o < (unsigned)nxy ? o : (unsigned)(kPairMaxPlane + t3)), __float_as_uint(z));
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        res_block_sum_lds<NT, 2>(acc2, red);
        ++it;
        {
            double o2[2];
            flags |= pair_exchange<2>(mb, h, ++msg, acc2, o2) ? 0 : 4;
            for (int k = 0; k < 2; ++k) acc2[k] = h == 0 ? acc2[k] + o2[k] : o2[k] + acc2[k];
        }
        if (!res_finite(acc2[0]) || !res_finite(acc2[1])) {
            flags |= 1;
            break;
        }
        betac = acc2[0] / rz;
        rz = acc2[0];
        rr = acc2[1];
    }
    // (an opaque index: addresses and mask bytes of the start are not kept
    // across the iteration for these stores)
    int te = (int)threadIdx.x - S;
    asm volatile("" : "+v"(te));
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = te + k * NT;
        if (v >= 0 && v < nv && m[v] == 0) xb[v] = x[k];
    }
    if (threadIdx.x == 0 && h == 0) {
        st.rz[0] = rz;
        st.rr[0] = rr;
        if (corr) {
            st.refine_iters += it;
        } else {
            st.iters = it;
            st.rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            if (flags & 2) st.status = RW_ST_MAX_ITER;
        }
        if (flags & 1) st.status = RW_ST_NONFINITE;
        if (flags & 4) st.status = RW_ST_SYNC_LOST;
        st.pending = corr && !(flags & 5) ? 1 : 0;
    }
}

// Workgroups b and b + 8 of each group of 16 are the lower and upper half of
// one box (consecutive workgroups go to different XCDs, these two to the
// same one).
template <int NT, int VPT, int G>
__global__ __launch_bounds__(NT) void k_pcg_res2(SolveArgs a, float* xt, int corr, int base, int n) {
    const int b = (int)blockIdx.x;
    const int i = (b >> 4) * 8 + (b & 7);
    if (i >= n) return;
    res2_half<NT, VPT, G>(a, xt, corr, base + i, (b >> 3) & 1);
}

// Clears the mailbox flags of boxes [base, base + gridDim.x) (a kernel, so
// that the sequence is valid inside a captured graph).
__global__ void k_pair_clear(SolveArgs a, int base) {
    const BrickDev bd = a.bricks[base + (int)blockIdx.x];
    const int64_t he = split_half_elems((int64_t)bd.nx * bd.ny);
    const PairBox mb{(char*)(a.wts + bd.woff + 2 * he)};
    if (threadIdx.x < 2) dev_st(mb.flag((int)threadIdx.x), 0u);
}


// Elements of each LDS array of the weights kernel for the largest box of a
// launch: the box, nx*ny pad elements before it and nx*ny + 1 after it (the
// unused voxel slots of a thread map to the element just past the box, whose
// +z neighbour is the last one).
int64_t resident_lds_elems(int64_t voxels, int64_t plane) { return voxels + 2 * plane + 1; }
bool resident_w_fits(const BrickDev& b, size_t lds_limit) {
    const int64_t nxy = (int64_t)b.nx * b.ny, nv = nxy * b.nz;
    return nv <= (int64_t)kResMaxVptW * kResThreads &&
           (size_t)resident_lds_elems(nv, nxy) * sizeof(float4) + 1024 <= lds_limit;
}

// The weights-in-registers kernel: p alone in LDS, at most kResMaxVptR voxels
// per thread; its LDS array holds every voxel slot of the launch (threads x
// voxels per thread, as launch_resident picks them) and nx*ny pads on both
// sides.
static int64_t resident_r_vpt(int64_t max_voxels) {
    const int64_t v = (max_voxels + kResThreads - 1) / kResThreads;
    return v <= 4 ? 4 : v <= 8 ? 8 : v <= 10 ? 10 : kResMaxVptR;
}
static int64_t resident_r_lds_elems(int64_t max_voxels, int64_t plane) {
    return resident_r_vpt(max_voxels) * kResThreads + 2 * plane;
}
bool resident_r_fits(const BrickDev& b, size_t lds_limit) {
    const int64_t nxy = (int64_t)b.nx * b.ny, nv = nxy * b.nz;
    return nv <= (int64_t)kResMaxVptR * kResThreads &&
           (size_t)resident_r_lds_elems(nv, nxy) * sizeof(float) + 1024 <= lds_limit;
}

// Voxel slots (threads x voxels per thread) of a streamed-weights launch
// whose largest box has max_voxels voxels (0: too large).
int64_t resident_g_span(int64_t max_voxels) {
    if (max_voxels <= kResSpanG0) return kResSpanG0;
    if (max_voxels <= kResSpanG1) return kResSpanG1;
    return 0;
}

static size_t resident_g_lds(int64_t span, int64_t plane) { return (size_t)(span + 2 * plane) * sizeof(float); }

bool resident_g_fits(const BrickDev& b, size_t lds_limit) {
    const int64_t nxy = (int64_t)b.nx * b.ny, nv = nxy * b.nz;
    const int64_t span = resident_g_span(nv);
    return span > 0 && resident_g_lds(span, nxy) + 1024 <= lds_limit;
}

int64_t resident_g_elems(const BrickDev& b, int64_t span) {
    const int64_t nxy = (int64_t)b.nx * b.ny;
    return (4 * (nxy + span) + 63) & ~int64_t(63);  // four arrays, whole 256-byte lines
}

// Boxes [b0, b1) of the launch list, all eligible for the kernel `kind`
// (1: weights and p in LDS, 2: p in LDS and weights in a global buffer,
// 3: p in LDS and weights in registers),
// largest first; px = 32 when every box has 32 x 32 planes.
// Clears a launch's ticket counter (a kernel, not a memset, so that the
// sequence stays valid inside a captured graph).
__global__ void k_clear_ticket(uint32_t* t) {
    if (threadIdx.x == 0) *t = 0u;
}

hipError_t launch_resident(const SolveArgs& a, int64_t b0, int64_t b1, int64_t max_voxels, int64_t max_plane,
                           int kind, int px, float* xt, int corr, uint32_t* ticket, hipStream_t s) {
    if (b1 <= b0) return hipSuccess;
    const size_t lds = kind == 2   ? resident_g_lds(resident_g_span(max_voxels), max_plane)
                       : kind == 3 ? (size_t)resident_r_lds_elems(max_voxels, max_plane) * sizeof(float)
                                   : (size_t)resident_lds_elems(max_voxels, max_plane) * sizeof(float4);
    auto go1 = [&](auto kern, int nt) -> hipError_t {
        if (lds > 48 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        int64_t n = b1 - b0;
        if (ticket) {
            // persistent: as many workgroups as the CUs hold at once
            int per_cu = 0, cus = 0, dev = 0;
            hipError_t e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds);
            if (e != hipSuccess) return e;
            n = std::min<int64_t>(n, (int64_t)std::max(per_cu, 1) * std::max(cus, 1));
            hipLaunchKernelGGL(k_clear_ticket, dim3(1), dim3(64), 0, s, ticket);
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)n), dim3(nt), lds, s, a, xt, corr, (int)b0, (int)b1, ticket);
        return hipGetLastError();
    };
    // the one-box kernel, or its persistent twin when a ticket is given
    auto go = [&](auto kern, auto kern_q, int nt) -> hipError_t { return ticket ? go1(kern_q, nt) : go1(kern, nt); };
    if (kind == 2) {
        // the plan sized each box's weight segment for this launch's span
        if (!a.wts) return hipErrorInvalidValue;
        const int64_t span = resident_g_span(max_voxels);
        // 512 threads; 32 x 32 planes: four voxels per 16-byte load (k_pcg_resg4,
        // 34 or 64 voxels per thread); other planes one voxel per load, the
        // forward weights issued 8 voxels ahead (34 per thread) or 5 (64 per
        // thread, where three register arrays leave room for no more)
        constexpr int nt = kResThreads;
        // one workgroup per box only: a persistent twin of this kernel would
        // spill registers (its box loop keeps values live across boxes)
        if (ticket) return hipErrorInvalidValue;
        constexpr int ng0 = kResSpanG0 / 4, ng1 = kResSpanG1 / 4;
        if (span == kResSpanG0)
            return px == 32 ? go1(k_pcg_resg4<nt, (ng0 + nt - 1) / nt, ng0>, nt)
                            : go1(k_pcg_resg<nt, kResSpanG0 / nt, 8>, nt);
        if (span == kResSpanG1)
            return px == 32 ? go1(k_pcg_resg4<nt, ng1 / nt, ng1>, nt)
                            : go1(k_pcg_resg<nt, kResSpanG1 / nt, 5>, nt);
        return hipErrorInvalidValue;
    }
    const int nt = kResThreads;
    const int64_t vpt = (max_voxels + nt - 1) / nt;
    if (kind == 1) {
        if (vpt <= 10) return go(k_pcg_resw<kResThreads, 10>, k_pcg_resw_q<kResThreads, 10>, nt);
        if (vpt <= kResMaxVptW) return go(k_pcg_resw<kResThreads, kResMaxVptW>, k_pcg_resw_q<kResThreads, kResMaxVptW>, nt);
    }
    if (kind == 3) {
        if (vpt <= 4) return go(k_pcg_resr<kResThreads, 4>, k_pcg_resr_q<kResThreads, 4>, nt);
        if (vpt <= 8) return go(k_pcg_resr<kResThreads, 8>, k_pcg_resr_q<kResThreads, 8>, nt);
        if (vpt <= 10) return go(k_pcg_resr<kResThreads, 10>, k_pcg_resr_q<kResThreads, 10>, nt);
        if (vpt <= kResMaxVptR) return go(k_pcg_resr<kResThreads, kResMaxVptR>, k_pcg_resr_q<kResThreads, kResMaxVptR>, nt);
    }
    return hipErrorInvalidValue;
}

bool resident_split_fits(const BrickDev& b, size_t lds_limit) {
    const int64_t nxy = (int64_t)b.nx * b.ny, nv = nxy * b.nz;
    const int64_t z0 = (b.nz + 1) / 2;
    return nv > kResSpanG1 && b.nz >= 2 && nxy >= kResThreads && nxy <= kPairMaxPlane && nxy * z0 <= kResSpanG1 &&
           (size_t)(kResSpanG1 + 2 * nxy) * sizeof(float) + 1024 <= lds_limit;
}

int64_t resident_split_elems(const BrickDev& b) {
    return 2 * split_half_elems((int64_t)b.nx * b.ny) + ((kPairMailboxElems + 63) & ~int64_t(63));
}

hipError_t launch_split(const SolveArgs& a, int64_t b0, int64_t b1, int64_t max_plane, float* xt, int corr,
                        hipStream_t s) {
    if (b1 <= b0) return hipSuccess;
    if (!a.wts || max_plane > kPairMaxPlane) return hipErrorInvalidValue;
    const int64_t n = b1 - b0;
    hipLaunchKernelGGL(k_pair_clear, dim3((unsigned)n), dim3(64), 0, s, a, (int)b0);
    constexpr int nt = kResThreads;
    auto k = k_pcg_res2<nt, kResSpanG1 / nt, 4>;
    const size_t lds = (size_t)(kResSpanG1 + 2 * max_plane) * sizeof(float);
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // 16 workgroups for each group of 8 boxes (a box's halves are b and b + 8)
    hipLaunchKernelGGL(k, dim3((unsigned)(16 * ((n + 7) / 8))), dim3(nt), lds, s, a, xt, corr, (int)b0, (int)n);
    return hipGetLastError();
}

}  // namespace rwk
