// Multi-workgroup Jacobi-PCG for one large box (a single domain such as the
// coarsest pyramid level or a plain volume solve): the same iteration as the
// per-box kernels (Section III-B system, Section V solver), spread over up to
// kDomMaxWG workgroups.  Each CG iteration is two launches:
//   A(it): gamma/beta from the partial sums of B(it-1), convergence test;
//          p_new = z + beta p_old, sigma = p_new . L_UU p_new (per-WG partials)
//   B(it): alpha = gamma / sigma; x += alpha p, r -= alpha L_UU p, z = r/d,
//          per-WG partials of r.z and ||r||^2
// Every workgroup sums the partials in workgroup order, so all of them get the
// same scalars bit for bit and the result is deterministic.  Workgroup 0 keeps
// the scalars in a two-slot state (slot it & 1); the host polls the done flag
// every few iterations.

#include "common.h"

#include <algorithm>

namespace rwk {

constexpr int kDomThreads = 256;
constexpr int kDomMaxWG = 1024;

struct DomState {
    double rz[3], rr[3], beta[3];
    int32_t done[3];
    int32_t all_done, iters, flags, pad;
};

template <typename T>
__device__ __forceinline__ T dom_weight(T a, T b, double beta, double eps);
template <>
__device__ __forceinline__ float dom_weight<float>(float a, float b, double beta, double eps) {
    const float d = a - b;
    return __builtin_amdgcn_exp2f((float)(-beta * 1.4426950408889634) * d * d) + (float)eps;
}
template <>
__device__ __forceinline__ double dom_weight<double>(double a, double b, double beta, double eps) {
    const double d = a - b;
    return exp(-beta * d * d) + eps;
}

// Workgroup sum of N doubles, identical on every thread.
template <int N>
__device__ __forceinline__ void dom_block_sum(double (&v)[N], double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = v[k];
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        v[k] = s;
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) red[w * N + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (int i = 0; i < kDomThreads / 64; ++i) s += red[i * N + k];
        v[k] = s;
    }
    __syncthreads();
}

// Sum of per-workgroup partials part[w * N + k], w < G, in order.
template <int N>
__device__ __forceinline__ void dom_sum_partials(const double* part, int G, double (&out)[N], double* red) {
    double v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = 0.0;
    for (int w = threadIdx.x; w < G; w += kDomThreads)
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += part[w * N + k];
    dom_block_sum<N>(v, red);
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = v[k];
}

// Stencil of voxel v (box-relative) on an operand given by op(u): returns d and acc.
template <typename T, int N, typename Op>
__device__ __forceinline__ void dom_stencil(const BrickDev& b, const float* __restrict__ g, int v, double beta,
                                            double eps, Op op, T& d, T (&acc)[N]) {
    const int nx = b.nx, nxy = b.nx * b.ny;
    const int k = v / nxy, r0 = v - k * nxy, j = r0 / nx, i = r0 - j * nx;
    const T gc = (T)g[v];
    d = T(0);
#pragma unroll
    for (int a = 0; a < N; ++a) acc[a] = T(0);
    auto nb = [&](int u) {
        const T w = dom_weight<T>(gc, (T)g[u], beta, eps);
        d += w;
        T o[N];
        op(u, o);
#pragma unroll
        for (int a = 0; a < N; ++a) acc[a] += w * o[a];
    };
    if (i > 0) nb(v - 1);
    if (i + 1 < nx) nb(v + 1);
    if (j > 0) nb(v - nx);
    if (j + 1 < b.ny) nb(v + nx);
    if (k > 0) nb(v - nxy);
    if (k + 1 < b.nz) nb(v + nxy);
}

__device__ __forceinline__ bool dom_finite(double v) { return isfinite(v); }
__device__ __forceinline__ float dom_recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double dom_recip(double d) { return 1.0 / d; }

// Start: state slot 1 (read by A(0)) from the box's BoxState.
template <int R>
__global__ void k_dom_start(const BoxState* st, DomState* ds) {
    if (threadIdx.x != 0) return;
    DomState s{};
#pragma unroll
    for (int k = 0; k < R; ++k) {
        s.rz[k] = st->rz[k];
        s.rr[k] = st->rr[k];
    }
    s.all_done = st->active ? 0 : 1;
    ds[1] = s;
    ds[0] = s;
}

template <typename T, int R>
__global__ __launch_bounds__(kDomThreads) void k_dom_A(SolveArgs a, int ib, int it, double tol, int max_iter,
                                                       const T* __restrict__ z, const T* __restrict__ pold,
                                                       T* __restrict__ pnew) {
    __shared__ double red[(kDomThreads / 64) * 2 * 3];
    DomState* ds = (DomState*)a.dom;
    const DomState* prev = ds + ((it + 1) & 1);
    DomState* out = ds + (it & 1);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (prev->all_done) {
        if (lead) *out = *prev;
        return;
    }
    const BrickDev b = a.bricks[ib];
    const int G = gridDim.x;
    double rz[R], rr[R];
    if (it == 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            rz[k] = prev->rz[k];
            rr[k] = prev->rr[k];
        }
    } else {
        double s2[2 * R];
        dom_sum_partials<2 * R>(a.dom_partB, G, s2, red);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            rz[k] = s2[k];
            rr[k] = s2[R + k];
        }
    }
    bool all = true;
    int flags = prev->flags;
    double be64[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const bool was = it > 0 && prev->done[k];
        const bool dn = was || rr[k] <= tol * tol * a.state[ib].bb[k];
        const double prz = prev->rz[k];
        be64[k] = (it == 0 || dn) ? 0.0 : rz[k] / prz;
        if (!dom_finite(rz[k]) || !dom_finite(rr[k])) flags |= 1;
        if (was) {
            rz[k] = prz;
            rr[k] = prev->rr[k];
        }
        all = all && dn;
        if (lead) {
            out->done[k] = dn ? 1 : 0;
            out->beta[k] = be64[k];
        }
    }
    if (!all && it >= max_iter) flags |= 2;
    const int fin = (all || flags) ? 1 : 0;
    if (lead) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            out->rz[k] = rz[k];
            out->rr[k] = rr[k];
        }
        out->all_done = fin;
        out->iters = it;
        out->flags = flags;
    }
    if (fin) return;
    const T* zb = z + b.off * R;
    const T* pb = pold + b.off * R;
    T* nbp = pnew + b.off * R;
    const float* gb = a.g + b.off;
    const uint8_t* mb = a.mask + b.off;
    const int nv = b.nx * b.ny * b.nz;
    T be[R];
#pragma unroll
    for (int k = 0; k < R; ++k) be[k] = (T)be64[k];
    double sig[R];
#pragma unroll
    for (int k = 0; k < R; ++k) sig[k] = 0.0;
    for (int v = blockIdx.x * kDomThreads + threadIdx.x; v < nv; v += G * kDomThreads) {
        if (mb[v] != 0) continue;
        T d, acc[R];
        dom_stencil<T, R>(b, gb, v, a.beta, a.eps,
                          [&](int u, T (&o)[R]) {
#pragma unroll
                              for (int k = 0; k < R; ++k) o[k] = zb[u * R + k] + be[k] * pb[u * R + k];
                          },
                          d, acc);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T pv = zb[v * R + k] + be[k] * pb[v * R + k];
            const T q = d * pv - acc[k];
            sig[k] += (double)pv * (double)q;
            nbp[v * R + k] = pv;
        }
    }
    dom_block_sum<R>(sig, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < R; ++k) a.dom_partA[blockIdx.x * R + k] = sig[k];
}

template <typename T, int R, typename XT>
__global__ __launch_bounds__(kDomThreads) void k_dom_B(SolveArgs a, int ib, int it, XT* __restrict__ xt,
                                                       const T* __restrict__ p, T* __restrict__ r, T* __restrict__ z) {
    __shared__ double red[(kDomThreads / 64) * 2 * 3];
    DomState* ds = (DomState*)a.dom;
    DomState cur = ds[it & 1];
    if (cur.all_done) return;
    const BrickDev b = a.bricks[ib];
    const int G = gridDim.x;
    double sig[R];
    dom_sum_partials<R>(a.dom_partA, G, sig, red);
    T al[R];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const double alpha = cur.done[k] ? 0.0 : cur.rz[k] / sig[k];
        if (!cur.done[k] && (!(sig[k] > 0.0) || !dom_finite(alpha))) bad = true;
        al[k] = bad ? T(0) : (T)alpha;
    }
    if (bad) {
        // breakdown: record and stop (x keeps the last finite iterate)
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            cur.flags |= 1;
            cur.all_done = 1;
            ds[it & 1] = cur;
            ds[(it + 1) & 1] = cur;
        }
        return;
    }
    const T* pb = p + b.off * R;
    T* rb = r + b.off * R;
    T* zb = z + b.off * R;
    XT* xb = xt + b.off * R;
    const float* gb = a.g + b.off;
    const uint8_t* mb = a.mask + b.off;
    const int nv = b.nx * b.ny * b.nz;
    double s2[2 * R];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) s2[k] = 0.0;
    for (int v = blockIdx.x * kDomThreads + threadIdx.x; v < nv; v += G * kDomThreads) {
        if (mb[v] != 0) continue;
        T d, acc[R];
        dom_stencil<T, R>(b, gb, v, a.beta, a.eps,
                          [&](int u, T (&o)[R]) {
#pragma unroll
                              for (int k = 0; k < R; ++k) o[k] = pb[u * R + k];
                          },
                          d, acc);
        const T id = dom_recip(d);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T pv = pb[v * R + k];
            const T q = d * pv - acc[k];
            xb[v * R + k] = (XT)((T)xb[v * R + k] + al[k] * pv);
            const T rv = rb[v * R + k] - al[k] * q;
            const T zv = rv * id;
            rb[v * R + k] = rv;
            zb[v * R + k] = zv;
            s2[k] += (double)rv * (double)zv;
            s2[R + k] += (double)rv * (double)rv;
        }
    }
    dom_block_sum<2 * R>(s2, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) a.dom_partB[blockIdx.x * 2 * R + k] = s2[k];
}

// End: final scalars back into the box's BoxState (stats and the next phases).
template <int R>
__global__ void k_dom_end(SolveArgs a, int ib, int slot, int corr) {
    if (threadIdx.x != 0) return;
    const DomState s = ((DomState*)a.dom)[slot];
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

// Scratch layout: two DomState slots (256 B), partials A [kDomMaxWG][3],
// partials B [kDomMaxWG][6].
size_t domain_scratch_bytes() { return 256 + (size_t)kDomMaxWG * 9 * sizeof(double); }

void domain_bind(SolveArgs& a, void* scratch) {
    static_assert(2 * sizeof(DomState) <= 256, "DomState slots exceed their scratch");
    char* c = (char*)scratch;
    a.dom = c;
    a.dom_partA = (double*)(c + 256);
    a.dom_partB = a.dom_partA + kDomMaxWG * 3;
}

// One box, launch index ib, host copy of its descriptor bd.
template <typename T, int R, typename XT>
hipError_t domain_pcg(const SolveArgs& a, int ib, const BrickDev& bd, XT* xt, int corr, hipStream_t s) {
    const int64_t nv = (int64_t)bd.nx * bd.ny * bd.nz;
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(kDomMaxWG, (nv + 2 * kDomThreads - 1) / (2 * kDomThreads)));
    const double tol = corr ? a.inner_tol : a.tol;
    T* r = (T*)a.r;
    T* z = (T*)a.z;
    T* p0 = (T*)a.p0;
    T* p1 = (T*)a.p1;
    hipLaunchKernelGGL(k_dom_start<R>, dim3(1), dim3(64), 0, s, a.state + ib, (DomState*)a.dom);
    DomState* dsp = (DomState*)a.dom;
    const int poll = 16;
    int it = 0;
    for (; it <= a.max_iter; ++it) {
        T* pold = (it & 1) ? p1 : p0;
        T* pnew = (it & 1) ? p0 : p1;
        hipLaunchKernelGGL((k_dom_A<T, R>), dim3(G), dim3(kDomThreads), 0, s, a, ib, it, tol, a.max_iter, z, pold,
                           pnew);
        hipLaunchKernelGGL((k_dom_B<T, R, XT>), dim3(G), dim3(kDomThreads), 0, s, a, ib, it, xt, pnew, r, z);
        if (it == 0 || (it + 1) % poll == 0) {
            int32_t done = 0;
            hipError_t e = hipMemcpyAsync(&done, &dsp[it & 1].all_done, sizeof(done), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            if (done) break;
        }
    }
    if (it > a.max_iter) it = a.max_iter;
    // the state slot of the last A launch holds the final scalars
    hipLaunchKernelGGL(k_dom_end<R>, dim3(1), dim3(64), 0, s, a, ib, it & 1, corr);
    return hipGetLastError();
}

#define RW_DOM_INST(T, R, XT) \
    template hipError_t domain_pcg<T, R, XT>(const SolveArgs&, int, const BrickDev&, XT*, int, hipStream_t);
RW_DOM_INST(float, 1, float)
RW_DOM_INST(float, 2, float)
RW_DOM_INST(float, 3, float)
RW_DOM_INST(double, 1, double)
RW_DOM_INST(double, 2, double)
RW_DOM_INST(double, 3, double)

}  // namespace rwk
