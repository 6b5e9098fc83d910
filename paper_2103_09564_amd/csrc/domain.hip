// Multi-workgroup solve of large boxes (single domains such as the coarsest
// pyramid level or a plain volume solve, and the boxes of large bricks):
// every phase of the per-box solve (Dirichlet init, Jacobi-PCG, FP64 true
// residual, correction set-up and apply; Section III-B system, Section V
// solver) spread over up to kDomMaxWG workgroups of kDomThreads threads per
// box (grid-stride over the box's voxels).  The domain boxes of a call (the
// first nd of its list) share each launch: box j takes the next dom_wgs
// workgroups, and has its own scalar state, ticket and partials.
//
// Each voxel's stencil is evaluated branch-free: out-of-box neighbours are
// replaced by the voxel itself with weight 0, so all loads of a voxel are in
// flight together.  Workgroup sums go to a partials array; the last workgroup
// to finish (ticket counter) adds them in workgroup order and writes the
// scalars, so every result is deterministic.
//
// One CG iteration is two launches (for every domain box of the call):
//   A(n): p_new = z + beta_n p_old, partial sigma = p_new . L_UU p_new;
//         last workgroup: alpha_n = rho_n / sigma (breakdown test)
//   B(n): x += alpha p, r -= alpha L_UU p, z = r / d, partial r.z, ||r||^2;
//         last workgroup: convergence test, beta_{n+1}, state n+1
// The scalar state of iteration n lives in slot n & 1; the host reads the
// done flag every few iterations (one read behind the queued launches) and
// stops launching.

#include "common.h"

#include <algorithm>
#include <map>

namespace rwk {

constexpr int kDomThreads = 256;
constexpr int kDomWaves = kDomThreads / 64;
constexpr int kDomMaxWG = 2048;
constexpr int kDomPart = 12;  // doubles per workgroup partial record

struct DomState {
    double rz[3], rr[3], beta[3], alpha[3];
    int32_t done[3];
    int32_t all_done, iters, flags;
};

struct DomCtl {
    DomState s[2];
    uint32_t ticket;
    int32_t pad[3];
};

// Scratch layout: a table (the workgroup prefix of each domain box in the two
// launch kinds, int32 [2][kDomMaxBoxes + 1], and the every-box-done word at
// byte 2048) in its first 4 KB, then per domain box DomCtl (padded to
// 512 B) and partials [kDomMaxWG][kDomPart].
constexpr size_t kDomTableBytes = 4096;
constexpr size_t kDomDoneOff = 2048;
constexpr size_t kDomBoxBytes = 512 + (size_t)kDomMaxWG * kDomPart * sizeof(double);
size_t domain_scratch_bytes(int64_t n_dom) {
    return kDomTableBytes + (size_t)std::max<int64_t>(n_dom, 1) * kDomBoxBytes;
}
static_assert(2 * (kDomMaxBoxes + 1) * sizeof(int32_t) <= kDomDoneOff, "domain table size");
__host__ __device__ inline DomCtl* dom_ctl(void* dom, int j) {
    return (DomCtl*)((char*)dom + kDomTableBytes + (size_t)j * kDomBoxBytes);
}

void domain_bind(SolveArgs& a, void* scratch) {
    static_assert(sizeof(DomCtl) <= 512, "DomCtl exceeds its scratch");
    a.dom = scratch;
    a.dom_part = nullptr;  // (per box: after its DomCtl)
}

// Workgroups of a domain box in a launch: kind 0 (the phases) one voxel per
// thread and pass, kind 1 (the PCG launches) kVpt.
constexpr int kDomPcgWG = 1024;
constexpr int kVpt = 2;
__host__ __device__ inline int dom_wgs(int64_t nv, int kind) {
    const int64_t per = kind ? (int64_t)kVpt * kDomThreads : (int64_t)kDomThreads;
    const int64_t cap = kind ? kDomPcgWG : kDomMaxWG;
    const int64_t g = (nv + per - 1) / per;
    return (int)(g < 1 ? 1 : g > cap ? cap : g);
}

namespace {

template <typename T>
struct DWeight;
template <>
struct DWeight<float> {
    float c, eps;  // c = -beta * log2(e)
    __device__ DWeight(double beta, double e) : c((float)(-beta * 1.4426950408889634)), eps((float)e) {}
    __device__ __forceinline__ float operator()(float a, float b) const {
        const float d = a - b;
        return __builtin_amdgcn_exp2f(c * d * d) + eps;
    }
};
template <>
struct DWeight<double> {
    double nb, eps;
    __device__ DWeight(double beta, double e) : nb(-beta), eps(e) {}
    __device__ __forceinline__ double operator()(double a, double b) const {
        const double d = a - b;
        return exp(nb * d * d) + eps;
    }
};

__device__ __forceinline__ float drecip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double drecip(double d) { return 1.0 / d; }

// The six neighbours of flat box voxel v; absent ones point at v itself.
struct Nb {
    int u[6];
    bool h[6];
};

__device__ __forceinline__ Nb neighbours(int v, int nx, int ny, int nz) {
    const int nxy = nx * ny;
    const int k = v / nxy, r0 = v - k * nxy, j = r0 / nx, i = r0 - j * nx;
    Nb n;
    n.h[0] = i > 0;
    n.h[1] = i + 1 < nx;
    n.h[2] = j > 0;
    n.h[3] = j + 1 < ny;
    n.h[4] = k > 0;
    n.h[5] = k + 1 < nz;
    n.u[0] = n.h[0] ? v - 1 : v;
    n.u[1] = n.h[1] ? v + 1 : v;
    n.u[2] = n.h[2] ? v - nx : v;
    n.u[3] = n.h[3] ? v + nx : v;
    n.u[4] = n.h[4] ? v - nxy : v;
    n.u[5] = n.h[5] ? v + nxy : v;
    return n;
}

// Edge weights of voxel v to its neighbours (0 where absent); returns the diagonal.
template <typename T>
__device__ __forceinline__ T stencil_weights(const float* __restrict__ g, int v, const Nb& n, const DWeight<T>& W,
                                             T (&w)[6]) {
    const T gc = (T)g[v];
    T gn[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) gn[q] = (T)g[n.u[q]];
    T d = T(0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        w[q] = n.h[q] ? W(gc, gn[q]) : T(0);
        d += w[q];
    }
    return d;
}

// This workgroup's share of a launch over the domain boxes [0, nd): box ib,
// workgroup w of the box's G, the box's scalar state and partials.
struct DomView {
    int ib, w, G;
    DomCtl* ctl;
    double* part;
};
// Every wave reads the launch's prefix table (lane l: box l's first
// workgroup) and takes the last box that starts at or before this workgroup.
__device__ __forceinline__ DomView dom_view(const SolveArgs& a, int nd, int kind) {
    const int32_t* pre = (const int32_t*)a.dom + kind * (kDomMaxBoxes + 1);
    const int lane = threadIdx.x & 63, b = (int)blockIdx.x;
    const int lo = lane < nd ? pre[lane] : 0x7fffffff;
    const int hi = lane < nd ? pre[lane + 1] : 0;
    const unsigned long long m = __ballot(lo <= b);  // bit 0 always set (pre[0] = 0)
    const int j = 63 - __clzll(m);
    const int l0 = __shfl(lo, j, 64), l1 = __shfl(hi, j, 64);
    DomCtl* c = dom_ctl(a.dom, j);
    return DomView{j, b - l0, l1 - l0, c, (double*)((char*)c + 512)};
}

template <int N>
__device__ __forceinline__ void wg_sum(double (&v)[N], double* red) {
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
        for (int i = 0; i < kDomWaves; ++i) s += red[i * N + k];
        v[k] = s;
    }
    __syncthreads();
}

// Store this workgroup's sums, take a ticket; in the last workgroup to arrive
// return true with the sums over all workgroups (fixed order) in v.
template <int N>
__device__ __forceinline__ bool last_wg_sum(double (&v)[N], const DomView& dv, double* red) {
    __shared__ int last;
    DomCtl* ctl = dv.ctl;
    double* part = dv.part;
    wg_sum<N>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) part[dv.w * kDomPart + k] = v[k];
        __threadfence();
        const uint32_t t = atomicAdd(&ctl->ticket, 1u);
        last = t == (uint32_t)dv.G - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double s[N];
#pragma unroll
    for (int k = 0; k < N; ++k) s[k] = 0.0;
    // thread t adds workgroups t, t + 256, ... in order; then the fixed tree of wg_sum
    for (int w = threadIdx.x; w < dv.G; w += kDomThreads) {
#pragma unroll
        for (int k = 0; k < N; ++k) s[k] += __builtin_nontemporal_load(&part[w * kDomPart + k]);
    }
    wg_sum<N>(s, red);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = s[k];
    if (threadIdx.x == 0) ctl->ticket = 0u;
    return true;
}

// Ticket without sums: true in the last workgroup to arrive.
__device__ __forceinline__ bool last_wg(const DomView& dv) {
    __shared__ int last;
    DomCtl* ctl = dv.ctl;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t t = atomicAdd(&ctl->ticket, 1u);
        last = t == (uint32_t)dv.G - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    if (threadIdx.x == 0) ctl->ticket = 0u;
    return true;
}

__device__ __forceinline__ bool fin(double v) { return isfinite(v); }

#define RW_DOM_LOOP(dv, v, nv) for (int v = (dv).w * kDomThreads + threadIdx.x; v < (nv); v += (dv).G * kDomThreads)

}  // namespace

// ---------------------------------------------------------------------------
// Dirichlet init (the multi-workgroup form of the per-box init): r = -(L x)_U,
// z = r/d, p = 0, sums r.z, ||r||^2, ||b||^2, |U|, |M|; the FP64 path copies x
// into its FP64 solution buffer.
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ __launch_bounds__(kDomThreads) void k_dinit(SolveArgs a, int nd) {
    __shared__ double red[kDomWaves * kDomPart];
    const DomView dv = dom_view(a, nd, 0);
    const int ib = dv.ib;
    const BrickDev b = a.bricks[ib];
    const int nv = b.nx * b.ny * b.nz;
    double s[3 * R + 2];
#pragma unroll
    for (int k = 0; k < 3 * R + 2; ++k) s[k] = 0.0;
    const DWeight<T> W(a.beta, a.eps);
    const float* g = a.g + b.off;
    const uint8_t* m = a.mask + b.off;
    const float* x = a.x + b.off * R;
    T* r = (T*)a.r + b.off * R;
    T* z = (T*)a.z + b.off * R;
    T* p0 = (T*)a.p0 + b.off * R;
    T* p1 = (T*)a.p1 + b.off * R;
    RW_DOM_LOOP(dv, v, nv) {
        if (sizeof(T) == 8) {
            double* xt = (double*)a.xt + b.off * R;
#pragma unroll
            for (int k = 0; k < R; ++k) xt[v * R + k] = (double)x[v * R + k];
        }
        if (m[v] == 0) {
            const Nb n = neighbours(v, b.nx, b.ny, b.nz);
            T w[6];
            bool sm[6];
            T xn[6][R], xv[R];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                sm[q] = m[n.u[q]] != 0;
#pragma unroll
                for (int k = 0; k < R; ++k) xn[q][k] = (T)x[n.u[q] * R + k];
            }
#pragma unroll
            for (int k = 0; k < R; ++k) xv[k] = (T)x[v * R + k];
            const T d = stencil_weights<T>(g, v, n, W, w);
            const T id = drecip(d);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                T acc = T(0), accm = T(0);
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    acc += w[q] * xn[q][k];
                    accm += w[q] * (sm[q] ? xn[q][k] : T(0));
                }
                const T rv = acc - d * xv[k];
                const T zv = rv * id;
                r[v * R + k] = rv;
                z[v * R + k] = zv;
                p0[v * R + k] = T(0);
                p1[v * R + k] = T(0);
                s[k] += (double)rv * (double)zv;
                s[R + k] += (double)rv * (double)rv;
                s[2 * R + k] += (double)accm * (double)accm;
            }
            s[3 * R] += 1.0;
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                r[v * R + k] = T(0);
                z[v * R + k] = T(0);
                p0[v * R + k] = T(0);
                p1[v * R + k] = T(0);
            }
            s[3 * R + 1] += 1.0;
        }
    }
    if (!last_wg_sum<3 * R + 2>(s, dv, red)) return;
    if (threadIdx.x == 0) {
        BoxState& st = a.state[ib];
        const double nU = s[3 * R], nM = s[3 * R + 1];
        bool allzero = true;
        for (int k = 0; k < 3; ++k) st.rz[k] = st.rr[k] = st.bb[k] = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const bool zero = s[2 * R + k] == 0.0;
            allzero = allzero && zero;
            // ||b|| = 0 for an rhs: its solution is x_U = 0 (k_dzero), no iterations
            st.rz[k] = zero ? 0.0 : s[k];
            st.rr[k] = zero ? 0.0 : s[R + k];
            st.bb[k] = s[2 * R + k];
        }
        st.nU = nU;
        st.nM = nM;
        st.rel = 0.0;
        st.true_rel = 0.0;
        st.iters = st.refine_steps = st.refine_iters = 0;
        st.status = nM == 0.0 ? RW_ST_NO_DIRICHLET : RW_ST_CONVERGED;
        st.active = (nM > 0.0 && nU > 0.0 && !allzero) ? 1 : 0;
        st.pending = 0;
        st.checked = 0;
    }
}

// Right-hand sides with ||b|| = 0: x_U = r = z = 0 for them.
template <typename T, int R>
__global__ __launch_bounds__(kDomThreads) void k_dzero(SolveArgs a, int nd) {
    const DomView dv = dom_view(a, nd, 0);
    const int ib = dv.ib;
    const BoxState& st = a.state[ib];
    if (!(st.nM > 0.0 && st.nU > 0.0)) return;
    bool any = false;
#pragma unroll
    for (int k = 0; k < R; ++k) any = any || st.bb[k] == 0.0;
    if (!any) return;
    const BrickDev b = a.bricks[ib];
    const int nv = b.nx * b.ny * b.nz;
    T* xt = (sizeof(T) == 8 ? (T*)a.xt : (T*)a.x) + b.off * R;
    T* r = (T*)a.r + b.off * R;
    T* z = (T*)a.z + b.off * R;
    RW_DOM_LOOP(dv, v, nv) {
        if (a.mask[b.off + v] != 0) continue;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (st.bb[k] == 0.0) {
                xt[v * R + k] = T(0);
                r[v * R + k] = T(0);
                z[v * R + k] = T(0);
            }
    }
}

// ---------------------------------------------------------------------------
// Jacobi-PCG
// ---------------------------------------------------------------------------

// Ticket counters to 0 (device memory is not cleared when allocated); one
// workgroup per domain box.
__global__ void k_dreset(SolveArgs a) {
    if (threadIdx.x == 0) dom_ctl(a.dom, (int)blockIdx.x)->ticket = 0u;
}

// The PCG kernels spread a box over at most kDomPcgWG workgroups, kVpt voxels
// per thread and pass.  Each launch starts by adding the previous launch's
// per-workgroup partials in workgroup order (every workgroup gets the same
// scalars; kernel boundaries make the partials visible); workgroup 0 records
// the scalar state.
// Sum of per-workgroup partials part[w * stride + k], w < G, k < N, in order.
template <int N>
__device__ __forceinline__ void sum_partials(const double* part, int stride, int G, double (&out)[N], double* red) {
    double v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = 0.0;
    for (int w = threadIdx.x; w < G; w += kDomThreads) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += part[w * stride + k];
    }
    wg_sum<N>(v, red);
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = v[k];
}

// Slot layout of a box's PCG partials: A (sigma) [G][3], B (r.z, ||r||^2) [G][6].
__device__ __forceinline__ double* part_a(const DomView& dv) { return dv.part; }
__device__ __forceinline__ double* part_b(const DomView& dv) { return dv.part + kDomPcgWG * 3; }

// State for A(0) (slot 1, and slot 0) from the box state (init or check).
template <int R>
__global__ void k_dstart(SolveArgs a) {
    if (threadIdx.x != 0) return;
    const int ib = (int)blockIdx.x;
    const BoxState& st = a.state[ib];
    DomCtl* ctl = dom_ctl(a.dom, ib);
    DomState s{};
#pragma unroll
    for (int k = 0; k < R; ++k) {
        s.rz[k] = st.rz[k];
        s.rr[k] = st.rr[k];
    }
    s.all_done = st.active ? 0 : 1;
    ctl->s[0] = s;
    ctl->s[1] = s;
    ctl->ticket = 0u;
}

// A(it): scalars of iteration it from B(it-1)'s partials (A(0): from the
// start state), convergence test; then p_new = z + beta p_old and the
// partials of sigma = p_new . L_UU p_new.
template <typename T, int R>
__global__ __launch_bounds__(kDomThreads) void k_dA(SolveArgs a, int nd, int it, double tol, int max_iter,
                                                    const T* __restrict__ z, const T* __restrict__ pold,
                                                    T* __restrict__ pnew) {
    __shared__ double red[kDomWaves * kDomPart];
    const DomView dv = dom_view(a, nd, 1);
    const int ib = dv.ib;
    DomCtl* ctl = dv.ctl;
    const volatile DomState* prev = &ctl->s[(it + 1) & 1];
    DomState* out = &ctl->s[it & 1];
    const bool lead = dv.w == 0 && threadIdx.x == 0;
    if (prev->all_done) {
        if (lead) *out = *(const DomState*)prev;
        return;
    }
    double rz[R], rr[R];
    if (it == 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            rz[k] = prev->rz[k];
            rr[k] = prev->rr[k];
        }
    } else {
        double s2[2 * R];
        sum_partials<2 * R>(part_b(dv), 6, dv.G, s2, red);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            rz[k] = s2[k];
            rr[k] = s2[R + k];
        }
    }
    const double* bb = a.state[ib].bb;
    bool all = true;
    int flags = prev->flags;
    T be[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const bool was = it > 0 && prev->done[k];
        const double prz = prev->rz[k], prr = prev->rr[k];
        if (!was && (!fin(rz[k]) || !fin(rr[k]))) flags |= 1;
        if (was) {
            rz[k] = prz;
            rr[k] = prr;
        }
        const bool dn = was || rr[k] <= tol * tol * bb[k];
        const double bk = (it == 0 || dn) ? 0.0 : rz[k] / prz;
        be[k] = (T)bk;
        all = all && dn;
        if (lead) {
            out->done[k] = dn ? 1 : 0;
            out->beta[k] = bk;
            out->rz[k] = rz[k];
            out->rr[k] = rr[k];
        }
    }
    if (!all && it >= max_iter) flags |= 2;
    const int fin_ = (all || flags) ? 1 : 0;
    if (lead) {
        out->all_done = fin_;
        out->iters = it;
        out->flags = flags;
    }
    if (fin_) return;
    const BrickDev b = a.bricks[ib];
    const int nv = b.nx * b.ny * b.nz;
    const DWeight<T> W(a.beta, a.eps);
    const T* zb = z + b.off * R;
    const T* pb = pold + b.off * R;
    const float* gb = a.g + b.off;
    const uint8_t* mb = a.mask + b.off;
    T* nb = pnew + b.off * R;
    double sig[R];
#pragma unroll
    for (int k = 0; k < R; ++k) sig[k] = 0.0;
    const int stride = dv.G * kDomThreads;
    for (int v0 = dv.w * kDomThreads + threadIdx.x; v0 < nv; v0 += kVpt * stride) {
        // all loads of the kVpt voxels first (clamped in-box indices), then compute
        int vv[kVpt];
        bool use[kVpt];
        Nb n[kVpt];
        T pn[kVpt][6][R], pv[kVpt][R], w[kVpt][6], d[kVpt];
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            const int v = v0 + j * stride;
            vv[j] = v < nv ? v : nv - 1;
            use[j] = v < nv && mb[vv[j]] == 0;
            n[j] = neighbours(vv[j], b.nx, b.ny, b.nz);
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int k = 0; k < R; ++k)
                    pn[j][q][k] = zb[n[j].u[q] * R + k] + be[k] * pb[n[j].u[q] * R + k];
#pragma unroll
            for (int k = 0; k < R; ++k) pv[j][k] = zb[vv[j] * R + k] + be[k] * pb[vv[j] * R + k];
            d[j] = stencil_weights<T>(gb, vv[j], n[j], W, w[j]);
        }
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            if (!use[j]) continue;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < 6; ++q) acc += w[j][q] * pn[j][q][k];
                const T qv = d[j] * pv[j][k] - acc;
                sig[k] += (double)pv[j][k] * (double)qv;
                nb[vv[j] * R + k] = pv[j][k];
            }
        }
    }
    wg_sum<R>(sig, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) part_a(dv)[dv.w * 3 + k] = sig[k];
    }
}

// B(it): alpha from A(it)'s partials (breakdown test); x += alpha p,
// r -= alpha L_UU p, z = r / d and the partials of r.z, ||r||^2.
template <typename T, int R, typename XT>
__global__ __launch_bounds__(kDomThreads) void k_dB(SolveArgs a, int nd, int it, XT* xt, const T* __restrict__ p) {
    __shared__ double red[kDomWaves * kDomPart];
    const DomView dv = dom_view(a, nd, 1);
    const int ib = dv.ib;
    DomCtl* ctl = dv.ctl;
    const volatile DomState* cur = &ctl->s[it & 1];
    if (cur->all_done) return;
    double sig[R];
    sum_partials<R>(part_a(dv), 3, dv.G, sig, red);
    T al[R];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const bool dn = cur->done[k];
        const double alpha = dn ? 0.0 : cur->rz[k] / sig[k];
        if (!dn && (!(sig[k] > 0.0) || !fin(alpha))) bad = true;
        al[k] = (T)alpha;
    }
    if (bad) {
        // breakdown: stop with the current iterate
        if (dv.w == 0 && threadIdx.x == 0) {
            DomState s = *(const DomState*)cur;
            s.flags |= 1;
            s.all_done = 1;
            ctl->s[it & 1] = s;
            ctl->s[(it + 1) & 1] = s;
        }
        return;
    }
    const BrickDev b = a.bricks[ib];
    const int nv = b.nx * b.ny * b.nz;
    const DWeight<T> W(a.beta, a.eps);
    const T* pb = p + b.off * R;
    T* rb = (T*)a.r + b.off * R;
    T* zb = (T*)a.z + b.off * R;
    XT* xb = xt + b.off * R;
    const float* gb = a.g + b.off;
    const uint8_t* mb = a.mask + b.off;
    double arz[R], arr[R];
#pragma unroll
    for (int k = 0; k < R; ++k) arz[k] = arr[k] = 0.0;
    const int stride = dv.G * kDomThreads;
    for (int v0 = dv.w * kDomThreads + threadIdx.x; v0 < nv; v0 += kVpt * stride) {
        int vv[kVpt];
        bool use[kVpt];
        Nb n[kVpt];
        T pn[kVpt][6][R], pv[kVpt][R], rv0[kVpt][R], xv0[kVpt][R], w[kVpt][6], d[kVpt];
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            const int v = v0 + j * stride;
            vv[j] = v < nv ? v : nv - 1;
            use[j] = v < nv && mb[vv[j]] == 0;
            n[j] = neighbours(vv[j], b.nx, b.ny, b.nz);
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int k = 0; k < R; ++k) pn[j][q][k] = pb[n[j].u[q] * R + k];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                pv[j][k] = pb[vv[j] * R + k];
                rv0[j][k] = rb[vv[j] * R + k];
                xv0[j][k] = (T)xb[vv[j] * R + k];
            }
            d[j] = stencil_weights<T>(gb, vv[j], n[j], W, w[j]);
        }
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            if (!use[j]) continue;
            const T id = drecip(d[j]);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < 6; ++q) acc += w[j][q] * pn[j][q][k];
                const T qv = d[j] * pv[j][k] - acc;
                const T rv = rv0[j][k] - al[k] * qv;
                const T zv = rv * id;
                xb[vv[j] * R + k] = (XT)(xv0[j][k] + al[k] * pv[j][k]);
                rb[vv[j] * R + k] = rv;
                zb[vv[j] * R + k] = zv;
                arz[k] += (double)rv * (double)zv;
                arr[k] += (double)rv * (double)rv;
            }
        }
    }
    double s2[2 * R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        s2[k] = arz[k];
        s2[R + k] = arr[k];
    }
    wg_sum<2 * R>(s2, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) part_b(dv)[dv.w * 6 + k] = s2[k];
    }
}

// Final scalars into the box state (as the per-box PCG kernel leaves it).
template <int R>
__global__ void k_dend(SolveArgs a, int slot, int corr) {
    if (threadIdx.x != 0) return;
    const int ib = (int)blockIdx.x;
    const DomState s = dom_ctl(a.dom, ib)->s[slot];
    BoxState& st = a.state[ib];
    if (!st.active) return;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        st.rz[k] = s.rz[k];
        st.rr[k] = s.rr[k];
    }
    if (corr) {
        st.refine_iters += s.iters;
    } else {
        st.iters = s.iters;
        double rel = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (st.bb[k] > 0.0) rel = fmax(rel, sqrt(s.rr[k] / st.bb[k]));
        st.rel = rel;
        if (s.flags & 2) st.status = RW_ST_MAX_ITER;
    }
    if (s.flags & 1) st.status = RW_ST_NONFINITE;
    st.pending = corr && !(s.flags & 1) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// FP64 true residual r64 = b - L_UU x with FP64 weights, of xs (float x or
// double x64).  kMode 0 (check): r <- (float)r64; the last workgroup takes
// the refinement decision.  kMode 1 (FP64 finish): x <- (float)x64 on U; the
// last workgroup stores the true relative residual.
// ---------------------------------------------------------------------------
template <int R, typename XS, int kMode>
__global__ __launch_bounds__(kDomThreads) void k_dresid(SolveArgs a, int nd, const XS* __restrict__ xs,
                                                        int may_refine, int refine64) {
    __shared__ double red[kDomWaves * kDomPart];
    const DomView dv = dom_view(a, nd, 0);
    const int ib = dv.ib;
    const BoxState& st0 = a.state[ib];
    const bool solved = st0.nM > 0.0 && st0.nU > 0.0 && st0.status != RW_ST_NONFINITE;
    const BrickDev b = a.bricks[ib];
    const int nv = b.nx * b.ny * b.nz;
    const uint8_t* m = a.mask + b.off;
    const XS* x = xs + b.off * R;
    if (kMode == 1) {
        RW_DOM_LOOP(dv, v, nv) {
            if (m[v] != 0) continue;
#pragma unroll
            for (int k = 0; k < R; ++k) a.x[(b.off + v) * R + k] = (float)x[v * R + k];
        }
    }
    if (!solved) {
        if (kMode == 0 && dv.w == 0 && threadIdx.x == 0) a.state[ib].active = 0;
        return;
    }
    double q[2 * R];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) q[k] = 0.0;
    const DWeight<double> W(a.beta, a.eps);
    RW_DOM_LOOP(dv, v, nv) {
        if (m[v] != 0) continue;
        const Nb n = neighbours(v, b.nx, b.ny, b.nz);
        bool sm[6];
        double xn[6][R], xv[R];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            sm[j] = m[n.u[j]] != 0;
#pragma unroll
            for (int k = 0; k < R; ++k) xn[j][k] = (double)x[n.u[j] * R + k];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) xv[k] = (double)x[v * R + k];
        double w[6];
        const double d = stencil_weights<double>(a.g + b.off, v, n, W, w);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            double acc = 0.0, accm = 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                acc += w[j] * xn[j][k];
                accm += w[j] * (sm[j] ? xn[j][k] : 0.0);
            }
            const double rv = acc - d * xv[k];
            q[k] += rv * rv;
            q[R + k] += accm * accm;
            if (kMode == 0) ((float*)a.r)[(b.off + v) * R + k] = (float)rv;
        }
    }
    if (!last_wg_sum<2 * R>(q, dv, red)) return;
    if (threadIdx.x != 0) return;
    BoxState& st = a.state[ib];
    double tr = 0.0;
    bool ok = true;
    const double target = refine64 ? a.refine_tol : a.tol * a.stall_ratio;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (q[R + k] > 0.0) tr = fmax(tr, sqrt(q[k] / q[R + k]));
        if (q[k] > target * target * q[R + k]) ok = false;
    }
    st.true_rel = tr;
    if (kMode == 0) {
        const bool refine = may_refine && !ok && st.refine_steps < a.refine_max;
        st.active = refine ? 1 : 0;
        if (!may_refine && st.refine_steps > 0 && st.status == RW_ST_CONVERGED)
            st.status = ok ? RW_ST_REFINED : RW_ST_STALLED;
    }
}

// Correction system L_UU d = r64 (r holds r64 in FP32): z = r/d, p = 0, d = 0;
// seeded voxels all 0; ||b||^2 = ||r||^2.  Only when the check set `active`.
template <int R>
__global__ __launch_bounds__(kDomThreads) void k_dexplicit(SolveArgs a, int nd) {
    __shared__ double red[kDomWaves * kDomPart];
    const DomView dv = dom_view(a, nd, 0);
    const int ib = dv.ib;
    if (!a.state[ib].active) return;
    const BrickDev b = a.bricks[ib];
    const int nv = b.nx * b.ny * b.nz;
    double e[2 * R];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) e[k] = 0.0;
    const DWeight<float> W(a.beta, a.eps);
    float* r = (float*)a.r + b.off * R;
    float* z = (float*)a.z + b.off * R;
    float* p0 = (float*)a.p0 + b.off * R;
    float* p1 = (float*)a.p1 + b.off * R;
    float* dc = a.dcorr + b.off * R;
    RW_DOM_LOOP(dv, v, nv) {
        if (a.mask[b.off + v] == 0) {
            const Nb n = neighbours(v, b.nx, b.ny, b.nz);
            float w[6];
            const float id = drecip(stencil_weights<float>(a.g + b.off, v, n, W, w));
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const float rv = r[v * R + k];
                const float zv = rv * id;
                z[v * R + k] = zv;
                p0[v * R + k] = 0.0f;
                p1[v * R + k] = 0.0f;
                dc[v * R + k] = 0.0f;
                e[k] += (double)rv * (double)zv;
                e[R + k] += (double)rv * (double)rv;
            }
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                r[v * R + k] = 0.0f;
                z[v * R + k] = 0.0f;
                p0[v * R + k] = 0.0f;
                p1[v * R + k] = 0.0f;
                dc[v * R + k] = 0.0f;
            }
        }
    }
    if (!last_wg_sum<2 * R>(e, dv, red)) return;
    if (threadIdx.x == 0) {
        BoxState& st = a.state[ib];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            st.rz[k] = e[k];
            st.rr[k] = st.bb[k] = e[R + k];
        }
    }
}

// x (MIXED) or x64 (MIXED_REFINE) += d on U when a correction is pending.
template <int R, bool kRefine64>
__global__ __launch_bounds__(kDomThreads) void k_dapply(SolveArgs a, int nd) {
    const DomView dv = dom_view(a, nd, 0);
    const int ib = dv.ib;
    if (!a.state[ib].pending) return;
    const BrickDev b = a.bricks[ib];
    const int nv = b.nx * b.ny * b.nz;
    RW_DOM_LOOP(dv, v, nv) {
        if (a.mask[b.off + v] != 0) continue;
        const int64_t o = (b.off + v) * R;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (kRefine64) a.x64[o + k] += (double)a.dcorr[o + k];
            else a.x[o + k] += a.dcorr[o + k];
        }
    }
    if (!last_wg(dv)) return;
    if (threadIdx.x == 0) {
        BoxState& st = a.state[ib];
        st.refine_steps += 1;
        st.pending = 0;
    }
}

// to64: x64 = x on every voxel; else x = (float)x64 on U.
template <int R>
__global__ __launch_bounds__(kDomThreads) void k_dcopy64(SolveArgs a, int nd, int to64) {
    const DomView dv = dom_view(a, nd, 0);
    const BrickDev b = a.bricks[dv.ib];
    const int nv = b.nx * b.ny * b.nz;
    RW_DOM_LOOP(dv, v, nv) {
        const int64_t o = (b.off + v) * R;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (to64) a.x64[o + k] = (double)a.x[o + k];
            else if (a.mask[b.off + v] == 0) a.x[o + k] = (float)a.x64[o + k];
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Workgroups of a launch over the domain boxes [0, nd) (host copies in host).
static unsigned dom_total(const BrickDev* host, int nd, int kind) {
    int64_t g = 0;
    for (int j = 0; j < nd; ++j) g += dom_wgs((int64_t)host[j].nx * host[j].ny * host[j].nz, kind);
    return (unsigned)std::max<int64_t>(g, 1);
}

// The every-box-done word: 1 when every domain box's state in `slot` is done.
__global__ void k_dall(SolveArgs a, int nd, int slot) {
    int all = 1;
    for (int j = threadIdx.x; j < nd; j += blockDim.x) all &= dom_ctl(a.dom, j)->s[slot].all_done != 0 ? 1 : 0;
    all = __syncthreads_and(all);
    if (threadIdx.x == 0) *(int32_t*)((char*)a.dom + kDomDoneOff) = all;
}

// The prefix table of the domain boxes [0, nd) for both launch kinds (one
// thread), as the host sums them in dom_total.
__global__ void k_dtable(SolveArgs a, int nd) {
    if (threadIdx.x != 0) return;
    int32_t* pre = (int32_t*)a.dom;
    for (int kind = 0; kind < 2; ++kind) {
        int32_t acc = 0;
        pre[kind * (kDomMaxBoxes + 1)] = 0;
        for (int j = 0; j < nd; ++j) {
            const BrickDev b = a.bricks[j];
            acc += dom_wgs((int64_t)b.nx * b.ny * b.nz, kind);
            pre[kind * (kDomMaxBoxes + 1) + j + 1] = acc;
        }
    }
}

template <typename T, int R>
hipError_t domain_init(const SolveArgs& a, int nd, const BrickDev* host, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    const unsigned G = dom_total(host, nd, 0);
    hipLaunchKernelGGL(k_dtable, dim3(1), dim3(64), 0, s, a, nd);
    hipLaunchKernelGGL(k_dreset, dim3((unsigned)nd), dim3(64), 0, s, a);
    hipLaunchKernelGGL((k_dinit<T, R>), dim3(G), dim3(kDomThreads), 0, s, a, nd);
    hipLaunchKernelGGL((k_dzero<T, R>), dim3(G), dim3(kDomThreads), 0, s, a, nd);
    return hipGetLastError();
}

// Page-locked slots and events for the done-flag reads of domain_pcg, per
// host thread and device, created on first use and kept for the thread's
// lifetime; null when they cannot be had.
struct DomPoll {
    int32_t* flag = nullptr;  // [2], page-locked
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool tried = false;
};
static DomPoll* dom_poll() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    thread_local std::map<int, DomPoll> polls;
    DomPoll& p = polls[dev];
    if (!p.tried) {
        p.tried = true;
        void* h = nullptr;
        bool ok = hipHostMalloc(&h, 64, hipHostMallocDefault) == hipSuccess;
        if (ok) p.flag = (int32_t*)h;
        for (int i = 0; i < 2 && ok; ++i) ok = hipEventCreateWithFlags(&p.ev[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            p.flag = nullptr;
        }
    }
    return p.flag ? &p : nullptr;
}

template <typename T, int R, typename XT>
hipError_t domain_pcg(const SolveArgs& a, int nd, const BrickDev* host, XT* xt, int corr, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    const unsigned G = dom_total(host, nd, 1);
    const double tol = corr ? a.inner_tol : a.tol;
    T* z = (T*)a.z;
    T* p0 = (T*)a.p0;
    T* p1 = (T*)a.p1;
    int32_t* done_word = (int32_t*)((char*)a.dom + kDomDoneOff);
    // (the table again: the adjoint's solve reaches this without the init)
    hipLaunchKernelGGL(k_dtable, dim3(1), dim3(64), 0, s, a, nd);
    hipLaunchKernelGGL(k_dstart<R>, dim3((unsigned)nd), dim3(64), 0, s, a);
    // The done flag (every box done) is read after the first iteration and
    // every `poll` iterations: copied into page-locked memory behind the
    // launches, and waited for only after the next `poll` iterations are
    // queued, so the device does not idle while the host reads it.
    // Iterations queued past the end are no-ops (A and B return at once for a
    // box whose state is done).  Without the page-locked slots the flag is
    // read synchronously, and so is it in the solve that allocates nothing.
    DomPoll* pl = a.dom_sync_poll ? nullptr : dom_poll();
    auto finished = [&](bool* out) -> hipError_t {
        int32_t f = 0;
        hipError_t e = hipMemcpyAsync(&f, done_word, sizeof(f), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        *out = f != 0;
        return e;
    };
    const int poll = 16;
    int it = 0, checks = 0, pending = -1;
    for (;; ++it) {
        T* pold = (it & 1) ? p1 : p0;
        T* pnew = (it & 1) ? p0 : p1;
        hipLaunchKernelGGL((k_dA<T, R>), dim3(G), dim3(kDomThreads), 0, s, a, nd, it, tol, a.max_iter, z, pold,
                           pnew);
        if (it >= a.max_iter) break;  // A(max_iter) records the final state
        hipLaunchKernelGGL((k_dB<T, R, XT>), dim3(G), dim3(kDomThreads), 0, s, a, nd, it, xt, (const T*)pnew);
        if (it == 0 || (it + 1) % poll == 0) {
            hipLaunchKernelGGL(k_dall, dim3(1), dim3(64), 0, s, a, nd, it & 1);
            bool done = false;
            if (!pl) {
                hipError_t e = finished(&done);
                if (e != hipSuccess) return e;
            } else {
                // check `checks` goes to slot checks & 1, whose last use (check
                // checks - 2) was waited for at check checks - 1
                const int slot = checks++ & 1;
                hipError_t e =
                    hipMemcpyAsync(&pl->flag[slot], done_word, sizeof(int32_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipEventRecord(pl->ev[slot], s);
                if (e == hipSuccess && pending >= 0) {
                    e = hipEventSynchronize(pl->ev[pending]);
                    done = e == hipSuccess && pl->flag[pending] != 0;
                }
                if (e != hipSuccess) return e;
                pending = slot;
            }
            if (done) break;
        }
    }
    // slot it & 1 holds each box's final scalars (written by A(it), or carried there)
    hipLaunchKernelGGL(k_dend<R>, dim3((unsigned)nd), dim3(64), 0, s, a, it & 1, corr);
    return hipGetLastError();
}

template <int R, bool kRefine64>
hipError_t domain_check(const SolveArgs& a, int nd, const BrickDev* host, int may_refine, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    const unsigned G = dom_total(host, nd, 0);
    if (kRefine64)
        hipLaunchKernelGGL((k_dresid<R, double, 0>), dim3(G), dim3(kDomThreads), 0, s, a, nd,
                           (const double*)a.x64, may_refine, 1);
    else
        hipLaunchKernelGGL((k_dresid<R, float, 0>), dim3(G), dim3(kDomThreads), 0, s, a, nd, (const float*)a.x,
                           may_refine, 0);
    if (may_refine) hipLaunchKernelGGL((k_dexplicit<R>), dim3(G), dim3(kDomThreads), 0, s, a, nd);
    return hipGetLastError();
}

template <int R, bool kRefine64>
hipError_t domain_apply(const SolveArgs& a, int nd, const BrickDev* host, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_dapply<R, kRefine64>), dim3(dom_total(host, nd, 0)), dim3(kDomThreads), 0, s, a, nd);
    return hipGetLastError();
}

template <int R>
hipError_t domain_copy64(const SolveArgs& a, int nd, const BrickDev* host, int to64, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_dcopy64<R>), dim3(dom_total(host, nd, 0)), dim3(kDomThreads), 0, s, a, nd, to64);
    return hipGetLastError();
}

template <int R>
hipError_t domain_finish64(const SolveArgs& a, int nd, const BrickDev* host, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_dresid<R, double, 1>), dim3(dom_total(host, nd, 0)), dim3(kDomThreads), 0, s, a, nd,
                       (const double*)a.xt, 0, 0);
    return hipGetLastError();
}

#define RW_DOM_INST_R(R)                                                                                     \
    template hipError_t domain_init<float, R>(const SolveArgs&, int, const BrickDev*, hipStream_t);          \
    template hipError_t domain_init<double, R>(const SolveArgs&, int, const BrickDev*, hipStream_t);         \
    template hipError_t domain_pcg<float, R, float>(const SolveArgs&, int, const BrickDev*, float*, int,     \
                                                    hipStream_t);                                            \
    template hipError_t domain_pcg<double, R, double>(const SolveArgs&, int, const BrickDev*, double*, int,  \
                                                      hipStream_t);                                          \
    template hipError_t domain_check<R, false>(const SolveArgs&, int, const BrickDev*, int, hipStream_t);    \
    template hipError_t domain_check<R, true>(const SolveArgs&, int, const BrickDev*, int, hipStream_t);     \
    template hipError_t domain_apply<R, false>(const SolveArgs&, int, const BrickDev*, hipStream_t);         \
    template hipError_t domain_apply<R, true>(const SolveArgs&, int, const BrickDev*, hipStream_t);          \
    template hipError_t domain_copy64<R>(const SolveArgs&, int, const BrickDev*, int, hipStream_t);          \
    template hipError_t domain_finish64<R>(const SolveArgs&, int, const BrickDev*, hipStream_t);
RW_DOM_INST_R(1)
RW_DOM_INST_R(2)
RW_DOM_INST_R(3)

}  // namespace rwk
