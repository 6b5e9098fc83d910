// Batched brick-local random-walker solve: matrix-free Jacobi-PCG on gfx950.
//
// Method (arXiv 2103.09564, Section III-B): on each box, edge weights
// w = exp(-beta (g_p - g_q)^2) + eps between 6-neighbours inside the box,
// Laplacian L = D - W, and the Dirichlet problem L_UU x_U = -L_UM x_M.
// Solver (Section V): conjugate gradients with the Jacobi preconditioner.
//
// Layout of the work: one workgroup per box, launched largest box first so
// the hardware dispatcher balances uneven boxes (longest-processing-time
// order).  Inside a workgroup each thread owns whole z-columns of the box and
// marches along z, keeping the z-neighbours of the stencil in registers; the
// in-plane neighbours are re-read through L1/L2.  The matrix is never
// stored: weights are recomputed from g in every sweep and the right-hand
// side b = -L_UM x_M is folded into the initial residual r = -(L x)_U.
//
// Per CG iteration two sweeps and two workgroup reductions:
//   sweep A:  p_new = z + beta p_old (p double-buffered), q = L_UU p_new,
//             sigma = p_new . q                       -> alpha = rho / sigma
//   sweep B:  q = L_UU p_new again, x += alpha p, r -= alpha q, z = r / d,
//             rho' = r . z, ||r||^2                   -> beta = rho' / rho
// Dot products are accumulated in FP64 on every path; vectors and weights are
// FP32 on the mixed path and FP64 on the plain-FP64 path.  Reductions have a
// fixed order, so results do not depend on batch order or scheduling.
//
// Mixed path afterwards (precision pattern, not from the paper): the true
// residual b - L_UU x_U is recomputed in FP64 with FP64 weights; where it
// misses the target, FP32 correction solves L_UU d = r64 are run and added to
// x (MIXED) or to an FP64 copy of x (MIXED_REFINE, iterative refinement).

#include "common.h"

#include <math.h>

namespace rwk {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename T>
struct Weight;

template <>
struct Weight<float> {
    float c;    // -beta * log2(e)
    float eps;
    __device__ __forceinline__ float operator()(float a, float b) const {
        const float d = a - b;
        return __builtin_amdgcn_exp2f(c * d * d) + eps;
    }
};

template <>
struct Weight<double> {
    double nb;  // -beta
    double eps;
    __device__ __forceinline__ double operator()(double a, double b) const {
        const double d = a - b;
        return exp(nb * d * d) + eps;
    }
};

template <typename T>
__device__ __forceinline__ Weight<T> make_weight(double beta, double eps);
template <>
__device__ __forceinline__ Weight<float> make_weight<float>(double beta, double eps) {
    return Weight<float>{(float)(-beta * 1.4426950408889634), (float)eps};
}
template <>
__device__ __forceinline__ Weight<double> make_weight<double>(double beta, double eps) {
    return Weight<double>{-beta, eps};
}

template <typename T>
__device__ __forceinline__ T recip(T d) { return T(1) / d; }
template <>
__device__ __forceinline__ float recip<float>(float d) { return __builtin_amdgcn_rcpf(d); }

struct Box {
    int64_t off;
    int nx, ny, nz, nxy;
};

template <typename T, int N>
struct Val {
    T a[N];
};

// Sum N doubles over the workgroup; every thread receives the same bits.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = v[k];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        v[k] = s;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[wave * N + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += red[w * N + k];
        v[k] = s;
    }
    __syncthreads();
}

// Column march over a box.  For every voxel v, `load(u)` gives the N operand
// values of voxel u; for unknown voxels `visit_u(v, d, acc, self)` receives the
// diagonal d = sum of the 6 in-box weights, acc = sum_nb w * operand(nb) and
// the voxel's own operand; seeded voxels get `visit_m(v, self)`.
template <typename T, int N, typename Load, typename VisitU, typename VisitM>
__device__ __forceinline__ void march(const Box& b, const float* __restrict__ g,
                                      const uint8_t* __restrict__ m, const Weight<T>& W,
                                      Load load, VisitU visit_u, VisitM visit_m) {
    for (int c = threadIdx.x; c < b.nxy; c += kThreads) {
        const int j = c / b.nx, i = c - j * b.nx;
        const bool hxm = i > 0, hxp = i + 1 < b.nx, hym = j > 0, hyp = j + 1 < b.ny;
        int64_t v = b.off + c;
        T g0 = (T)g[v];
        Val<T, N> s0 = load(v), sm;
#pragma unroll
        for (int k = 0; k < N; ++k) sm.a[k] = T(0);
        T wzm = T(0);
        for (int kz = 0; kz < b.nz; ++kz, v += b.nxy) {
            const bool hzp = kz + 1 < b.nz;
            T gu = T(0), wzp = T(0);
            Val<T, N> su;
#pragma unroll
            for (int k = 0; k < N; ++k) su.a[k] = T(0);
            if (hzp) {
                gu = (T)g[v + b.nxy];
                su = load(v + b.nxy);
                wzp = W(g0, gu);
            }
            if (m[v] == 0) {
                T d = wzm + wzp;
                Val<T, N> acc;
#pragma unroll
                for (int k = 0; k < N; ++k) acc.a[k] = wzm * sm.a[k] + wzp * su.a[k];
                auto nb = [&](int64_t u) {
                    const T w = W(g0, (T)g[u]);
                    d += w;
                    const Val<T, N> o = load(u);
#pragma unroll
                    for (int k = 0; k < N; ++k) acc.a[k] += w * o.a[k];
                };
                if (hxm) nb(v - 1);
                if (hxp) nb(v + 1);
                if (hym) nb(v - b.nx);
                if (hyp) nb(v + b.nx);
                visit_u(v, d, acc, s0);
            } else {
                visit_m(v, s0);
            }
            sm = s0;
            s0 = su;
            wzm = wzp;
            g0 = gu;
        }
    }
}

// Plain loop over the voxels of a box (pointwise sweeps).
template <typename F>
__device__ __forceinline__ void each_voxel(const Box& b, F f) {
    const int64_t n = (int64_t)b.nxy * b.nz;
    for (int64_t t = threadIdx.x; t < n; t += kThreads) f(b.off + t);
}

template <typename T, int R>
struct Vecs {
    T* r;
    T* z;
    T* p[2];
};

// Dirichlet init: r = -(L x)_U, b = -L_UM x_M, z = r/d, p = 0; x read from
// the caller's float array.  Returns sums (rz, rr, bb per rhs, nU, nM).
template <typename T, int R>
__device__ void init_implicit(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                              const float* __restrict__ x, Vecs<T, R> V, const Weight<T>& W,
                              double (&rz)[R], double (&rr)[R], double (&bb)[R], double& nU,
                              double& nM) {
    auto load = [&](int64_t u) {
        Val<T, 2 * R> o;
        const bool s = m[u] != 0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T xv = (T)x[u * R + k];
            o.a[k] = xv;
            o.a[R + k] = s ? xv : T(0);
        }
        return o;
    };
    auto vu = [&](int64_t v, T d, const Val<T, 2 * R>& acc, const Val<T, 2 * R>& self) {
        const T id = recip(d);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T rv = acc.a[k] - d * self.a[k];
            const T zv = rv * id;
            V.r[v * R + k] = rv;
            V.z[v * R + k] = zv;
            V.p[0][v * R + k] = T(0);
            rz[k] += (double)rv * (double)zv;
            rr[k] += (double)rv * (double)rv;
            bb[k] += (double)acc.a[R + k] * (double)acc.a[R + k];
        }
        nU += 1.0;
    };
    auto vm = [&](int64_t v, const Val<T, 2 * R>&) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            V.r[v * R + k] = T(0);
            V.z[v * R + k] = T(0);
            V.p[0][v * R + k] = T(0);
        }
        nM += 1.0;
    };
    march<T, 2 * R>(b, g, m, W, load, vu, vm);
}

// Explicit-RHS init (correction and adjoint solves): r holds the right-hand
// side on U on entry; z = r/d, p = 0, target = 0.  Seeded voxels: r = z = p =
// target = 0.  rr doubles as ||b||^2.
template <typename T, int R, typename XT>
__device__ void init_explicit(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                              Vecs<T, R> V, XT* __restrict__ tgt, const Weight<T>& W,
                              double (&rz)[R], double (&rr)[R]) {
    auto load = [&](int64_t) {
        Val<T, 1> o;
        o.a[0] = T(0);
        return o;
    };
    auto vu = [&](int64_t v, T d, const Val<T, 1>&, const Val<T, 1>&) {
        const T id = recip(d);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T rv = V.r[v * R + k];
            const T zv = rv * id;
            V.z[v * R + k] = zv;
            V.p[0][v * R + k] = T(0);
            tgt[v * R + k] = XT(0);
            rz[k] += (double)rv * (double)zv;
            rr[k] += (double)rv * (double)rv;
        }
    };
    auto vm = [&](int64_t v, const Val<T, 1>&) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            V.r[v * R + k] = T(0);
            V.z[v * R + k] = T(0);
            V.p[0][v * R + k] = T(0);
            tgt[v * R + k] = XT(0);
        }
    };
    march<T, 1>(b, g, m, W, load, vu, vm);
}

// FP64 true residual r64 = b - L_UU x_U = sum_nb w (x_nb - x_v) with FP64
// weights, of a candidate x (float or double, seeded entries = x_M).  Writes
// r64 (rounded) into rout when given.
template <int R, typename XS, typename RT>
__device__ void true_residual(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                              const XS* __restrict__ xs, RT* __restrict__ rout, double beta, double eps,
                              double (&rr)[R], double (&bb)[R]) {
    const Weight<double> W = make_weight<double>(beta, eps);
    auto load = [&](int64_t u) {
        Val<double, 2 * R> o;
        const bool s = m[u] != 0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double xv = (double)xs[u * R + k];
            o.a[k] = xv;
            o.a[R + k] = s ? xv : 0.0;
        }
        return o;
    };
    auto vu = [&](int64_t v, double d, const Val<double, 2 * R>& acc, const Val<double, 2 * R>& self) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double rv = acc.a[k] - d * self.a[k];
            rr[k] += rv * rv;
            bb[k] += acc.a[R + k] * acc.a[R + k];
            if (rout) rout[v * R + k] = (RT)rv;
        }
    };
    auto vm = [&](int64_t, const Val<double, 2 * R>&) {};
    march<double, 2 * R>(b, g, m, W, load, vu, vm);
}

// Sweep A: p_new = z + beta p_old, sigma = p_new . L_UU p_new.
template <typename T, int R>
__device__ void sweep_pq(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                         const T* __restrict__ z, const T* __restrict__ pold, T* __restrict__ pnew,
                         const T (&bk)[R], const Weight<T>& W, double (&sig)[R]) {
    auto load = [&](int64_t u) {
        Val<T, R> o;
#pragma unroll
        for (int k = 0; k < R; ++k) o.a[k] = z[u * R + k] + bk[k] * pold[u * R + k];
        return o;
    };
    auto vu = [&](int64_t v, T d, const Val<T, R>& acc, const Val<T, R>& self) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T q = d * self.a[k] - acc.a[k];
            sig[k] += (double)self.a[k] * (double)q;
            pnew[v * R + k] = self.a[k];
        }
    };
    auto vm = [&](int64_t v, const Val<T, R>&) {
#pragma unroll
        for (int k = 0; k < R; ++k) pnew[v * R + k] = T(0);
    };
    march<T, R>(b, g, m, W, load, vu, vm);
}

// Sweep B: q = L_UU p, x += alpha p, r -= alpha q, z = r/d, rho' and ||r||^2.
template <typename T, int R, typename XT>
__device__ void sweep_update(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                             const T* __restrict__ p, Vecs<T, R> V, XT* __restrict__ xt,
                             const T (&al)[R], const Weight<T>& W, double (&rz)[R], double (&rr)[R]) {
    auto load = [&](int64_t u) {
        Val<T, R> o;
#pragma unroll
        for (int k = 0; k < R; ++k) o.a[k] = p[u * R + k];
        return o;
    };
    auto vu = [&](int64_t v, T d, const Val<T, R>& acc, const Val<T, R>& self) {
        const T id = recip(d);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T q = d * self.a[k] - acc.a[k];
            xt[v * R + k] = (XT)((T)xt[v * R + k] + al[k] * self.a[k]);
            const T rv = V.r[v * R + k] - al[k] * q;
            const T zv = rv * id;
            V.r[v * R + k] = rv;
            V.z[v * R + k] = zv;
            rz[k] += (double)rv * (double)zv;
            rr[k] += (double)rv * (double)rv;
        }
    };
    auto vm = [&](int64_t, const Val<T, R>&) {};
    march<T, R>(b, g, m, W, load, vu, vm);
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// Jacobi-PCG from an initialised state (r, z, p[0] = 0).  Returns iterations;
// sets *nonfinite on breakdown.  done[k] marks rhs that met tol.
template <typename T, int R, typename XT>
__device__ int pcg_loop(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                        Vecs<T, R> V, XT* __restrict__ xt, const Weight<T>& W, double (&rz)[R],
                        double (&rr)[R], const double (&bb)[R], double tol, int max_iter,
                        bool* nonfinite, bool* hit_cap, double* red) {
    double betac[R];
#pragma unroll
    for (int k = 0; k < R; ++k) betac[k] = 0.0;
    const double tol2 = tol * tol;
    int it = 0;
    *nonfinite = false;
    *hit_cap = false;
    for (;;) {
        bool done[R];
        bool all = true;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            done[k] = rr[k] <= tol2 * bb[k];
            all = all && done[k];
        }
        if (all) break;
        if (it >= max_iter) {
            *hit_cap = true;
            break;
        }
        T* pold = V.p[it & 1];
        T* pnew = V.p[(it + 1) & 1];
        T bk[R];
#pragma unroll
        for (int k = 0; k < R; ++k) bk[k] = done[k] ? T(0) : (T)betac[k];
        double sig[R];
#pragma unroll
        for (int k = 0; k < R; ++k) sig[k] = 0.0;
        sweep_pq<T, R>(b, g, m, V.z, pold, pnew, bk, W, sig);
        block_sum<R>(sig, red);
        T al[R];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double a = done[k] ? 0.0 : rz[k] / sig[k];
            if (!done[k] && (!finite(a) || !(sig[k] > 0.0))) bad = true;
            al[k] = bad ? T(0) : (T)a;
        }
        if (bad) {
            *nonfinite = true;
            break;
        }
        double rzn[R], rrn[R], acc[2 * R];
#pragma unroll
        for (int k = 0; k < R; ++k) rzn[k] = rrn[k] = 0.0;
        sweep_update<T, R, XT>(b, g, m, pnew, V, xt, al, W, rzn, rrn);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            acc[k] = rzn[k];
            acc[R + k] = rrn[k];
        }
        block_sum<2 * R>(acc, red);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (done[k]) continue;
            if (!finite(acc[k]) || !finite(acc[R + k])) bad = true;
            betac[k] = acc[k] / rz[k];
            rz[k] = acc[k];
            rr[k] = acc[R + k];
        }
        ++it;
        if (bad) {
            *nonfinite = true;
            break;
        }
    }
    return it;
}

template <typename T, int R>
__global__ __launch_bounds__(kThreads) void k_solve(SolveArgs a) {
    __shared__ double red[kWaves * 4 * 3];
    const BrickDev bd = a.bricks[blockIdx.x];
    const Box b{bd.off, bd.nx, bd.ny, bd.nz, bd.nx * bd.ny};
    const Weight<T> W = make_weight<T>(a.beta, a.eps);
    Vecs<T, R> V{(T*)a.r, (T*)a.z, {(T*)a.p0, (T*)a.p1}};
    constexpr bool kF64 = sizeof(T) == 8;

    double rz[R], rr[R], bb[R], nU = 0.0, nM = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) rz[k] = rr[k] = bb[k] = 0.0;
    init_implicit<T, R>(b, a.g, a.mask, a.x, V, W, rz, rr, bb, nU, nM);
    {
        double s[3 * R + 2];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            s[k] = rz[k];
            s[R + k] = rr[k];
            s[2 * R + k] = bb[k];
        }
        s[3 * R] = nU;
        s[3 * R + 1] = nM;
        block_sum<3 * R + 2>(s, red);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            rz[k] = s[k];
            rr[k] = s[R + k];
            bb[k] = s[2 * R + k];
        }
        nU = s[3 * R];
        nM = s[3 * R + 1];
    }

    rw_brick_stats st{};
    st.status = RW_ST_CONVERGED;
    T* xt;
    if constexpr (kF64) {
        xt = (T*)a.xt;
        each_voxel(b, [&](int64_t v) {
#pragma unroll
            for (int k = 0; k < R; ++k) xt[v * R + k] = (T)a.x[v * R + k];
        });
    } else {
        xt = (T*)a.x;
    }
    bool bzero = true;
#pragma unroll
    for (int k = 0; k < R; ++k) bzero = bzero && (bb[k] == 0.0);

    if (nM == 0.0) {
        st.status = RW_ST_NO_DIRICHLET;
    } else if (nU > 0.0) {
        bool nonfinite = false, cap = false;
        // ||b|| = 0 for an rhs: its solution is x_U = 0 (no iterations)
        bool anyzero = false;
#pragma unroll
        for (int k = 0; k < R; ++k) anyzero = anyzero || (bb[k] == 0.0);
        if (anyzero) {
            const double* bbp = bb;
            each_voxel(b, [&](int64_t v) {
                if (a.mask[v] == 0) {
#pragma unroll
                    for (int k = 0; k < R; ++k)
                        if (bbp[k] == 0.0) {
                            xt[v * R + k] = T(0);
                            V.r[v * R + k] = T(0);
                            V.z[v * R + k] = T(0);
                        }
                }
            });
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (bb[k] == 0.0) rr[k] = rz[k] = 0.0;
            __syncthreads();
        }
        if (!bzero) {
            st.iters = pcg_loop<T, R, T>(b, a.g, a.mask, V, xt, W, rz, rr, bb, a.tol, a.max_iter,
                                         &nonfinite, &cap, red);
        }
        double rel = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (bb[k] > 0.0) rel = fmax(rel, sqrt(rr[k] / bb[k]));
        st.rel_resid = rel;
        if (nonfinite) st.status = RW_ST_NONFINITE;
        else if (cap) st.status = RW_ST_MAX_ITER;
    }
    __syncthreads();

    // FP64 true residual of the result; mixed path: refinement.
    if (nM > 0.0 && nU > 0.0 && st.status != RW_ST_NONFINITE) {
        if constexpr (kF64) {
            double r2[R], b2[R], q[2 * R];
#pragma unroll
            for (int k = 0; k < R; ++k) r2[k] = b2[k] = 0.0;
            true_residual<R, T, float>(b, a.g, a.mask, xt, (float*)nullptr, a.beta, a.eps, r2, b2);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                q[k] = r2[k];
                q[R + k] = b2[k];
            }
            block_sum<2 * R>(q, red);
            double tr = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (q[R + k] > 0.0) tr = fmax(tr, sqrt(q[k] / q[R + k]));
            st.true_rel_resid = tr;
        } else {
            const bool refine64 = a.precision == RW_PREC_MIXED_REFINE;
            const double target = refine64 ? a.refine_tol : a.tol;
            double* x64 = a.x64;
            if (refine64) {
                each_voxel(b, [&](int64_t v) {
#pragma unroll
                    for (int k = 0; k < R; ++k) x64[v * R + k] = (double)a.x[v * R + k];
                });
                __syncthreads();
            }
            int steps = 0, riters = 0;
            double tr = 0.0;
            for (;;) {
                double r2[R], b2[R], q[2 * R];
#pragma unroll
                for (int k = 0; k < R; ++k) r2[k] = b2[k] = 0.0;
                if (refine64)
                    true_residual<R, double, T>(b, a.g, a.mask, x64, V.r, a.beta, a.eps, r2, b2);
                else
                    true_residual<R, float, T>(b, a.g, a.mask, a.x, V.r, a.beta, a.eps, r2, b2);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    q[k] = r2[k];
                    q[R + k] = b2[k];
                }
                block_sum<2 * R>(q, red);
                tr = 0.0;
                bool ok = true;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    if (q[R + k] > 0.0) tr = fmax(tr, sqrt(q[k] / q[R + k]));
                    if (q[k] > target * target * q[R + k]) ok = false;
                }
                if (ok || steps >= a.refine_max) break;
                // correction solve L_UU d = r64 in FP32, from d = 0
                double crz[R], crr[R], cbb[R], e[2 * R];
#pragma unroll
                for (int k = 0; k < R; ++k) crz[k] = crr[k] = 0.0;
                init_explicit<T, R, float>(b, a.g, a.mask, V, a.dcorr, W, crz, crr);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    e[k] = crz[k];
                    e[R + k] = crr[k];
                }
                block_sum<2 * R>(e, red);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    crz[k] = e[k];
                    crr[k] = cbb[k] = e[R + k];
                }
                bool nf = false, cap = false;
                riters += pcg_loop<T, R, float>(b, a.g, a.mask, V, a.dcorr, W, crz, crr, cbb,
                                                a.inner_tol, a.max_iter, &nf, &cap, red);
                __syncthreads();
                if (nf) break;
                if (refine64) {
                    each_voxel(b, [&](int64_t v) {
                        if (a.mask[v] == 0) {
#pragma unroll
                            for (int k = 0; k < R; ++k) x64[v * R + k] += (double)a.dcorr[v * R + k];
                        }
                    });
                } else {
                    each_voxel(b, [&](int64_t v) {
                        if (a.mask[v] == 0) {
#pragma unroll
                            for (int k = 0; k < R; ++k) a.x[v * R + k] += a.dcorr[v * R + k];
                        }
                    });
                }
                __syncthreads();
                ++steps;
            }
            st.true_rel_resid = tr;
            st.refine_steps = steps;
            st.refine_iters = riters;
            if (steps > 0 && st.status == RW_ST_CONVERGED) {
                bool ok = tr <= target;
                st.status = ok ? RW_ST_REFINED : RW_ST_STALLED;
            }
            if (refine64) {
                each_voxel(b, [&](int64_t v) {
                    if (a.mask[v] == 0) {
#pragma unroll
                        for (int k = 0; k < R; ++k) a.x[v * R + k] = (float)x64[v * R + k];
                    }
                });
            }
        }
    }
    // outputs
    if constexpr (kF64) {
        each_voxel(b, [&](int64_t v) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double xv = (double)xt[v * R + k];
                if (a.mask[v] == 0) a.x[v * R + k] = (float)xv;
                if (a.want_x64) a.x64[v * R + k] = xv;
            }
        });
    } else if (a.want_x64 && a.precision != RW_PREC_MIXED_REFINE) {
        each_voxel(b, [&](int64_t v) {
#pragma unroll
            for (int k = 0; k < R; ++k) a.x64[v * R + k] = (double)a.x[v * R + k];
        });
    }
    if (threadIdx.x == 0 && a.stats) a.stats[bd.slot] = st;
}

// Adjoint: L_UU lambda = dl/dx_U (FP32 PCG), then the edge gradient in
// gather form (every voxel sums over its own edges; no atomics).
__global__ __launch_bounds__(kThreads) void k_adjoint(AdjointArgs a) {
    __shared__ double red[kWaves * 4 * 3];
    const BrickDev bd = a.bricks[blockIdx.x];
    const Box b{bd.off, bd.nx, bd.ny, bd.nz, bd.nx * bd.ny};
    const Weight<float> W = make_weight<float>(a.beta, a.eps);
    Vecs<float, 1> V{a.r, a.z, {a.p0, a.p1}};
    // rhs into r (U only), count seeds
    double cnt[1] = {0.0};
    each_voxel(b, [&](int64_t v) {
        const bool u = a.mask[v] == 0;
        a.r[v] = u ? a.dl_dx[v] : 0.0f;
        if (!u) cnt[0] += 1.0;
    });
    block_sum<1>(cnt, red);
    rw_brick_stats st{};
    double rz[1] = {0.0}, rr[1] = {0.0};
    init_explicit<float, 1, float>(b, a.g, a.mask, V, a.lambda, W, rz, rr);
    double e[2] = {rz[0], rr[0]};
    block_sum<2>(e, red);
    rz[0] = e[0];
    rr[0] = e[1];
    double bb[1] = {rr[0]};
    if (cnt[0] == 0.0) {
        st.status = RW_ST_NO_DIRICHLET;
    } else if (bb[0] > 0.0) {
        bool nf = false, cap = false;
        st.iters = pcg_loop<float, 1, float>(b, a.g, a.mask, V, a.lambda, W, rz, rr, bb, a.tol,
                                             a.max_iter, &nf, &cap, red);
        st.rel_resid = sqrt(rr[0] / bb[0]);
        st.status = nf ? RW_ST_NONFINITE : (cap ? RW_ST_MAX_ITER : RW_ST_CONVERGED);
    }
    __syncthreads();
    // gradient sweep
    const float beta = (float)a.beta, eps = (float)a.eps;
    double db[1] = {0.0};
    for (int c = threadIdx.x; c < b.nxy; c += kThreads) {
        const int j = c / b.nx, i = c - j * b.nx;
        for (int kz = 0; kz < b.nz; ++kz) {
            const int64_t v = b.off + c + (int64_t)kz * b.nxy;
            const float gv = a.g[v], lv = a.lambda[v], xv = a.x[v];
            float acc = 0.0f;
            auto edge = [&](int64_t u, bool fwd) {
                const float dg = gv - a.g[u];
                const float core = W(gv, a.g[u]) - eps;
                const float dldw = -(lv - a.lambda[u]) * (xv - a.x[u]);
                acc += dldw * (-2.0f * beta * dg * core);
                if (fwd) db[0] += (double)dldw * (double)(-(dg * dg) * core);
            };
            if (i > 0) edge(v - 1, false);
            if (i + 1 < b.nx) edge(v + 1, true);
            if (j > 0) edge(v - b.nx, false);
            if (j + 1 < b.ny) edge(v + b.nx, true);
            if (kz > 0) edge(v - b.nxy, false);
            if (kz + 1 < b.nz) edge(v + b.nxy, true);
            a.dl_dg[v] = acc;
        }
    }
    block_sum<1>(db, red);
    if (threadIdx.x == 0) {
        a.beta_part[blockIdx.x] = db[0];
        if (a.stats) a.stats[bd.slot] = st;
    }
}

// Sum the per-box dl/dbeta partials in launch order (deterministic).
__global__ __launch_bounds__(kThreads) void k_sum_partials(const double* part, int64_t n, double* out) {
    __shared__ double red[kWaves];
    double s[1] = {0.0};
    // fixed assignment of partials to threads, fixed tree: deterministic
    for (int64_t i = threadIdx.x; i < n; i += kThreads) s[0] += part[i];
    block_sum<1>(s, red);
    if (threadIdx.x == 0) *out = s[0];
}

hipError_t launch_solve(const SolveArgs& a, int64_t n, int nrhs, bool fp64, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((unsigned)n), block(kThreads);
    if (fp64) {
        switch (nrhs) {
            case 1: hipLaunchKernelGGL((k_solve<double, 1>), grid, block, 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_solve<double, 2>), grid, block, 0, s, a); break;
            case 3: hipLaunchKernelGGL((k_solve<double, 3>), grid, block, 0, s, a); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (nrhs) {
            case 1: hipLaunchKernelGGL((k_solve<float, 1>), grid, block, 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_solve<float, 2>), grid, block, 0, s, a); break;
            case 3: hipLaunchKernelGGL((k_solve<float, 3>), grid, block, 0, s, a); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_adjoint(const AdjointArgs& a, int64_t n, double* dl_dbeta, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_adjoint, dim3((unsigned)n), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, s, a.beta_part, n, dl_dbeta);
    return hipGetLastError();
}

}  // namespace rwk
