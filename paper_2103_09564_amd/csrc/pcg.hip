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

constexpr int kThreads = 512;
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
template <typename T>
struct Val<T, 0> {};

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

// Plane march with in-plane exchange through LDS (boxes whose z-plane has at
// most C*kThreads voxels).  Thread t owns the columns t + q*kThreads, q < C,
// and walks them along z.  Per plane k: the operand (N values, e.g. p) and g
// of plane k+1 go to one of three rotating LDS plane buffers, one barrier,
// then every voxel of plane k reads its 4 in-plane neighbours from LDS and its
// 2 z-neighbours from registers.  Global loads run two planes ahead of the
// compute (operand, g, mask and NX private extras such as x and r), so each
// wave keeps several loads in flight while it computes.  Only unknown voxels
// are visited: visit_u(v, d, acc, self, extras).
template <typename T, int N, int NX, int C, typename Load, typename LoadX, typename VisitU>
__device__ __forceinline__ void plane_march(const Box& b, const float* __restrict__ g,
                                            const uint8_t* __restrict__ m, const Weight<T>& W,
                                            T* __restrict__ lds, Load load, LoadX loadx, VisitU visit_u) {
    const int nxy = b.nxy;
    const int sb = (N + 1) * nxy;
    int col[C];
    unsigned fl[C];  // 1 valid, 2 x-, 4 x+, 8 y-, 16 y+
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const int c = threadIdx.x + q * kThreads;
        col[q] = c;
        fl[q] = 0;
        if (c < nxy) {
            const int j = c / b.nx, i = c - j * b.nx;
            fl[q] = 1u | (i > 0 ? 2u : 0u) | (i + 1 < b.nx ? 4u : 0u) | (j > 0 ? 8u : 0u) |
                    (j + 1 < b.ny ? 16u : 0u);
        }
    }
    Val<T, N> sm[C], s0[C], su[C], sn[C];
    Val<T, NX> x0[C], xu[C], xn[C];
    T g0[C], gu[C], gn[C], wzm[C];
    unsigned m0[C], mu[C], mn[C];
    const int64_t off = b.off;
#pragma unroll
    for (int q = 0; q < C; ++q) {
#pragma unroll
        for (int a = 0; a < N; ++a) sm[q].a[a] = s0[q].a[a] = su[q].a[a] = sn[q].a[a] = T(0);
        g0[q] = gu[q] = gn[q] = wzm[q] = T(0);
        m0[q] = mu[q] = mn[q] = 1u;
        if (fl[q]) {
            const int64_t v = off + col[q];
            s0[q] = load(v);
            g0[q] = (T)g[v];
            m0[q] = m[v];
            x0[q] = loadx(v);
            if (b.nz > 1) {
                su[q] = load(v + nxy);
                gu[q] = (T)g[v + nxy];
                mu[q] = m[v + nxy];
                xu[q] = loadx(v + nxy);
            }
#pragma unroll
            for (int a = 0; a < N; ++a) lds[a * nxy + col[q]] = s0[q].a[a];
            lds[N * nxy + col[q]] = g0[q];
        }
    }
    for (int k = 0; k < b.nz; ++k) {
        const int64_t base = off + (int64_t)k * nxy;
        const bool h1 = k + 1 < b.nz, h2 = k + 2 < b.nz;
#pragma unroll
        for (int q = 0; q < C; ++q) {
#pragma unroll
            for (int a = 0; a < N; ++a) sn[q].a[a] = T(0);
            gn[q] = T(0);
            mn[q] = 1u;
            if (fl[q] && h2) {
                const int64_t u = base + 2 * nxy + col[q];
                sn[q] = load(u);
                gn[q] = (T)g[u];
                mn[q] = m[u];
                xn[q] = loadx(u);
            }
        }
        if (h1) {
            T* Lw = lds + ((k + 1) % 3) * sb;
#pragma unroll
            for (int q = 0; q < C; ++q) {
                if (fl[q]) {
#pragma unroll
                    for (int a = 0; a < N; ++a) Lw[a * nxy + col[q]] = su[q].a[a];
                    Lw[N * nxy + col[q]] = gu[q];
                }
            }
        }
        __syncthreads();
        const T* L = lds + (k % 3) * sb;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            if (!fl[q]) continue;
            const T wzp = h1 ? W(g0[q], gu[q]) : T(0);
            if (m0[q] == 0) {
                T d = wzm[q] + wzp;
                Val<T, N> acc;
#pragma unroll
                for (int a = 0; a < N; ++a) acc.a[a] = wzm[q] * sm[q].a[a] + wzp * su[q].a[a];
                const T gc = g0[q];
                auto nb = [&](int cc) {
                    const T w = W(gc, L[N * nxy + cc]);
                    d += w;
#pragma unroll
                    for (int a = 0; a < N; ++a) acc.a[a] += w * L[a * nxy + cc];
                };
                if (fl[q] & 2u) nb(col[q] - 1);
                if (fl[q] & 4u) nb(col[q] + 1);
                if (fl[q] & 8u) nb(col[q] - b.nx);
                if (fl[q] & 16u) nb(col[q] + b.nx);
                visit_u(base + col[q], d, acc, s0[q], x0[q]);
            }
            wzm[q] = wzp;
            sm[q] = s0[q];
            s0[q] = su[q];
            su[q] = sn[q];
            g0[q] = gu[q];
            gu[q] = gn[q];
            m0[q] = mu[q];
            mu[q] = mn[q];
            x0[q] = xu[q];
            xu[q] = xn[q];
        }
    }
    __syncthreads();
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
            V.p[1][v * R + k] = T(0);
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
            V.p[1][v * R + k] = T(0);
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
            V.p[1][v * R + k] = T(0);
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
            V.p[1][v * R + k] = T(0);
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
template <typename T, int R, int C>
__device__ void sweep_pq(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                         const T* __restrict__ z, const T* __restrict__ pold, T* __restrict__ pnew,
                         const T (&bk)[R], const Weight<T>& W, double (&sig)[R], T* lds, bool plane) {
    auto load = [&](int64_t u) {
        Val<T, R> o;
#pragma unroll
        for (int k = 0; k < R; ++k) o.a[k] = z[u * R + k] + bk[k] * pold[u * R + k];
        return o;
    };
    if (plane) {
        auto nox = [&](int64_t) { return Val<T, 0>{}; };
        auto vp = [&](int64_t v, T d, const Val<T, R>& acc, const Val<T, R>& self, const Val<T, 0>&) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T q = d * self.a[k] - acc.a[k];
                sig[k] += (double)self.a[k] * (double)q;
                pnew[v * R + k] = self.a[k];
            }
        };
        plane_march<T, R, 0, C>(b, g, m, W, lds, load, nox, vp);
        return;
    }
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
template <typename T, int R, int C, typename XT>
__device__ void sweep_update(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                             const T* __restrict__ p, Vecs<T, R> V, XT* __restrict__ xt,
                             const T (&al)[R], const Weight<T>& W, double (&rz)[R], double (&rr)[R],
                             T* lds, bool plane) {
    auto load = [&](int64_t u) {
        Val<T, R> o;
#pragma unroll
        for (int k = 0; k < R; ++k) o.a[k] = p[u * R + k];
        return o;
    };
    if (plane) {
        auto lx = [&](int64_t u) {
            Val<T, 2 * R> o;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                o.a[k] = (T)xt[u * R + k];
                o.a[R + k] = V.r[u * R + k];
            }
            return o;
        };
        auto vp = [&](int64_t v, T d, const Val<T, R>& acc, const Val<T, R>& self, const Val<T, 2 * R>& ex) {
            const T id = recip(d);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T q = d * self.a[k] - acc.a[k];
                xt[v * R + k] = (XT)(ex.a[k] + al[k] * self.a[k]);
                const T rv = ex.a[R + k] - al[k] * q;
                const T zv = rv * id;
                V.r[v * R + k] = rv;
                V.z[v * R + k] = zv;
                rz[k] += (double)rv * (double)zv;
                rr[k] += (double)rv * (double)rv;
            }
        };
        plane_march<T, R, 2 * R, C>(b, g, m, W, lds, load, lx, vp);
        return;
    }
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
// flags breakdown / the iteration cap.  done[k] marks rhs that met tol.
struct LoopEnd {
    int iters;
    int flags;  // 1: non-finite / breakdown, 2: iteration cap
};

template <typename T, int R, int C, bool kPlane, typename XT>
__device__ LoopEnd pcg_loop(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                            Vecs<T, R> V, XT* __restrict__ xt, const Weight<T>& W, double (&rz)[R],
                            double (&rr)[R], const double (&bb)[R], double tol, int max_iter, double* red,
                            T* lds) {
    double betac[R];
#pragma unroll
    for (int k = 0; k < R; ++k) betac[k] = 0.0;
    const double tol2 = tol * tol;
    int it = 0;
    int flags = 0;
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
            flags = 2;
            break;
        }
        // select, not index: a dynamically indexed pointer pair would live in scratch
        T* pold = (it & 1) ? V.p[1] : V.p[0];
        T* pnew = (it & 1) ? V.p[0] : V.p[1];
        T bk[R];
#pragma unroll
        for (int k = 0; k < R; ++k) bk[k] = done[k] ? T(0) : (T)betac[k];
        double sig[R];
#pragma unroll
        for (int k = 0; k < R; ++k) sig[k] = 0.0;
        sweep_pq<T, R, C>(b, g, m, V.z, pold, pnew, bk, W, sig, lds, kPlane);
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
            flags = 1;
            break;
        }
        double rzn[R], rrn[R], acc[2 * R];
#pragma unroll
        for (int k = 0; k < R; ++k) rzn[k] = rrn[k] = 0.0;
        sweep_update<T, R, C, XT>(b, g, m, pnew, V, xt, al, W, rzn, rrn, lds, kPlane);
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
            flags = 1;
            break;
        }
    }
    return LoopEnd{it, flags};
}

// ---------------------------------------------------------------------------
// Kernels.  A solve is a short sequence of launches over the same box list
// (one workgroup per box, launch order = largest box first); per-box scalars
// travel between them in BoxState.  Splitting the phases keeps the register
// budget of the hot PCG kernel to what its two sweeps need.
// ---------------------------------------------------------------------------

template <typename T, int R>
__device__ __forceinline__ Vecs<T, R> vecs(const SolveArgs& a) {
    return Vecs<T, R>{(T*)a.r, (T*)a.z, {(T*)a.p0, (T*)a.p1}};
}

__device__ __forceinline__ Box box_of(const BrickDev& bd) {
    return Box{bd.off, bd.nx, bd.ny, bd.nz, bd.nx * bd.ny};
}

// Phase 1: Dirichlet init, per-box decision (no seed / no unknown / zero rhs).
template <typename T, int R>
__global__ __launch_bounds__(kThreads) void k_init(SolveArgs a) {
    __shared__ double red[kWaves * 12];
    const BrickDev bd = a.bricks[blockIdx.x];
    const Box b = box_of(bd);
    const Weight<T> W = make_weight<T>(a.beta, a.eps);
    Vecs<T, R> V = vecs<T, R>(a);
    double rz[R], rr[R], bb[R], nU = 0.0, nM = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) rz[k] = rr[k] = bb[k] = 0.0;
    init_implicit<T, R>(b, a.g, a.mask, a.x, V, W, rz, rr, bb, nU, nM);
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
    T* xt = sizeof(T) == 8 ? (T*)a.xt : (T*)a.x;
    if (sizeof(T) == 8) {
        each_voxel(b, [&](int64_t v) {
#pragma unroll
            for (int k = 0; k < R; ++k) xt[v * R + k] = (T)a.x[v * R + k];
        });
    }
    nU = s[3 * R];
    nM = s[3 * R + 1];
    bool allzero = true, anyzero = false;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        allzero = allzero && s[2 * R + k] == 0.0;
        anyzero = anyzero || s[2 * R + k] == 0.0;
    }
    if (nM > 0.0 && nU > 0.0 && anyzero) {
        // ||b|| = 0 for an rhs: its solution is x_U = 0, no iterations
        __syncthreads();
        each_voxel(b, [&](int64_t v) {
            if (a.mask[v] == 0) {
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (s[2 * R + k] == 0.0) {
                        xt[v * R + k] = T(0);
                        V.r[v * R + k] = T(0);
                        V.z[v * R + k] = T(0);
                    }
            }
        });
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (s[2 * R + k] == 0.0) s[k] = s[R + k] = 0.0;
    }
    if (threadIdx.x == 0) {
        BoxState& st = a.state[blockIdx.x];
        for (int k = 0; k < 3; ++k) st.rz[k] = st.rr[k] = st.bb[k] = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            st.rz[k] = s[k];
            st.rr[k] = s[R + k];
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
    }
}

// Phase 2: the PCG loop on every active box.  corr = 0: main solve into xt
// (x, or the FP64 accumulator on the FP64 path); corr = 1: FP32 correction
// solve into dcorr from the state init_explicit left (tolerance inner_tol).
template <typename T, int R, int C, bool kPlane, typename XT>
__global__ __launch_bounds__(kThreads) void k_pcg(SolveArgs a, XT* xt, int corr, int base) {
    __shared__ double red[kWaves * 12];
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const int ib = base + blockIdx.x;
    BoxState& st = a.state[ib];
    if (!st.active) return;
    const BrickDev bd = a.bricks[ib];
    const Box b = box_of(bd);
    const Weight<T> W = make_weight<T>(a.beta, a.eps);
    Vecs<T, R> V = vecs<T, R>(a);
    double rz[R], rr[R], bb[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        rz[k] = st.rz[k];
        rr[k] = st.rr[k];
        bb[k] = st.bb[k];
    }
    const LoopEnd e = pcg_loop<T, R, C, kPlane, XT>(b, a.g, a.mask, V, xt, W, rz, rr, bb,
                                                    corr ? a.inner_tol : a.tol, a.max_iter, red,
                                                    reinterpret_cast<T*>(dyn_lds));
    if (threadIdx.x == 0) {
        if (corr) {
            st.refine_iters += e.iters;
        } else {
            st.iters = e.iters;
            double rel = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (bb[k] > 0.0) rel = fmax(rel, sqrt(rr[k] / bb[k]));
            st.rel = rel;
            if (e.flags & 2) st.status = RW_ST_MAX_ITER;
        }
        if (e.flags & 1) st.status = RW_ST_NONFINITE;
        st.pending = corr && !(e.flags & 1) ? 1 : 0;
    }
}

// Phase 3: FP64 true residual of the current solution (x, or x64 when
// refine64), relative to ||b||.  With may_refine, a box whose residual misses
// its target (stall_ratio*tol for MIXED, refine_tol for MIXED_REFINE) gets the
// correction system L_UU d = r64 initialised (r <- r64, z, p, d = 0) and is
// marked active for the next k_pcg(corr = 1).
template <int R, bool kRefine64>
__global__ __launch_bounds__(kThreads) void k_check(SolveArgs a, int may_refine) {
    __shared__ double red[kWaves * 12];
    BoxState& st = a.state[blockIdx.x];
    const bool solved = st.nM > 0.0 && st.nU > 0.0 && st.status != RW_ST_NONFINITE;
    if (!solved) {
        if (threadIdx.x == 0) st.active = 0;
        return;
    }
    const BrickDev bd = a.bricks[blockIdx.x];
    const Box b = box_of(bd);
    Vecs<float, R> V = vecs<float, R>(a);
    double r2[R], b2[R], q[2 * R];
#pragma unroll
    for (int k = 0; k < R; ++k) r2[k] = b2[k] = 0.0;
    if (kRefine64)
        true_residual<R, double, float>(b, a.g, a.mask, a.x64, V.r, a.beta, a.eps, r2, b2);
    else
        true_residual<R, float, float>(b, a.g, a.mask, a.x, V.r, a.beta, a.eps, r2, b2);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        q[k] = r2[k];
        q[R + k] = b2[k];
    }
    block_sum<2 * R>(q, red);
    const double target = kRefine64 ? a.refine_tol : a.tol * a.stall_ratio;
    double tr = 0.0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (q[R + k] > 0.0) tr = fmax(tr, sqrt(q[k] / q[R + k]));
        if (q[k] > target * target * q[R + k]) ok = false;
    }
    const bool refine = may_refine && !ok && st.refine_steps < a.refine_max;
    if (refine) {
        const Weight<float> W = make_weight<float>(a.beta, a.eps);
        double crz[R], crr[R], e[2 * R];
#pragma unroll
        for (int k = 0; k < R; ++k) crz[k] = crr[k] = 0.0;
        __syncthreads();
        init_explicit<float, R, float>(b, a.g, a.mask, V, a.dcorr, W, crz, crr);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            e[k] = crz[k];
            e[R + k] = crr[k];
        }
        block_sum<2 * R>(e, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                st.rz[k] = e[k];
                st.rr[k] = st.bb[k] = e[R + k];
            }
        }
    }
    if (threadIdx.x == 0) {
        st.true_rel = tr;
        st.active = refine ? 1 : 0;
        if (!may_refine && st.refine_steps > 0 && st.status == RW_ST_CONVERGED)
            st.status = ok ? RW_ST_REFINED : RW_ST_STALLED;
    }
}

// Phase 4: add the correction d to x (MIXED) or to x64 (MIXED_REFINE).
template <int R, bool kRefine64>
__global__ __launch_bounds__(kThreads) void k_apply(SolveArgs a) {
    BoxState& st = a.state[blockIdx.x];
    if (!st.pending) return;
    const Box b = box_of(a.bricks[blockIdx.x]);
    each_voxel(b, [&](int64_t v) {
        if (a.mask[v] == 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (kRefine64) a.x64[v * R + k] += (double)a.dcorr[v * R + k];
                else a.x[v * R + k] += a.dcorr[v * R + k];
            }
        }
    });
    if (threadIdx.x == 0) {
        st.refine_steps += 1;
        st.pending = 0;
    }
}

// Copy x into the FP64 accumulator (MIXED_REFINE start) or back (end).
template <int R>
__global__ __launch_bounds__(kThreads) void k_copy64(SolveArgs a, int to64) {
    const Box b = box_of(a.bricks[blockIdx.x]);
    each_voxel(b, [&](int64_t v) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (to64) a.x64[v * R + k] = (double)a.x[v * R + k];
            else if (a.mask[v] == 0) a.x[v * R + k] = (float)a.x64[v * R + k];
        }
    });
}

// FP64 path end: true residual of the FP64 solution (stats), x <- (float)x64.
template <int R>
__global__ __launch_bounds__(kThreads) void k_finish64(SolveArgs a) {
    __shared__ double red[kWaves * 12];
    BoxState& st = a.state[blockIdx.x];
    const Box b = box_of(a.bricks[blockIdx.x]);
    const double* xt = (const double*)a.xt;
    if (st.nM > 0.0 && st.nU > 0.0 && st.status != RW_ST_NONFINITE) {
        double r2[R], b2[R], q[2 * R];
#pragma unroll
        for (int k = 0; k < R; ++k) r2[k] = b2[k] = 0.0;
        true_residual<R, double, float>(b, a.g, a.mask, xt, (float*)nullptr, a.beta, a.eps, r2, b2);
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
        if (threadIdx.x == 0) st.true_rel = tr;
    }
    each_voxel(b, [&](int64_t v) {
        if (a.mask[v] == 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) a.x[v * R + k] = (float)xt[v * R + k];
        }
    });
}

// Last phase: stats in caller order, optional FP64 copy of the result.
template <int R>
__global__ __launch_bounds__(kThreads) void k_stats(SolveArgs a, int copy64) {
    const BrickDev bd = a.bricks[blockIdx.x];
    if (copy64) {
        const Box b = box_of(bd);
        each_voxel(b, [&](int64_t v) {
#pragma unroll
            for (int k = 0; k < R; ++k) a.x64[v * R + k] = (double)a.x[v * R + k];
        });
    }
    if (threadIdx.x == 0 && a.stats) {
        const BoxState& st = a.state[blockIdx.x];
        rw_brick_stats o{};
        o.iters = st.iters;
        o.status = st.status;
        o.refine_steps = st.refine_steps;
        o.refine_iters = st.refine_iters;
        o.rel_resid = st.rel;
        o.true_rel_resid = st.true_rel;
        a.stats[bd.slot] = o;
    }
}

// Adjoint phases: rhs dl/dx on U -> explicit init; PCG into lambda; gradient.
__global__ __launch_bounds__(kThreads) void k_adj_init(AdjointArgs a, SolveArgs sa) {
    __shared__ double red[kWaves * 12];
    const Box b = box_of(a.bricks[blockIdx.x]);
    const Weight<float> W = make_weight<float>(a.beta, a.eps);
    Vecs<float, 1> V{a.r, a.z, {a.p0, a.p1}};
    double cnt[1] = {0.0};
    each_voxel(b, [&](int64_t v) {
        const bool u = a.mask[v] == 0;
        a.r[v] = u ? a.dl_dx[v] : 0.0f;
        if (!u) cnt[0] += 1.0;
    });
    block_sum<1>(cnt, red);   // barrier: r complete before init_explicit reads it
    double rz[1] = {0.0}, rr[1] = {0.0};
    init_explicit<float, 1, float>(b, a.g, a.mask, V, a.lambda, W, rz, rr);
    double e[2] = {rz[0], rr[0]};
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        BoxState& st = sa.state[blockIdx.x];
        st.rz[0] = e[0];
        st.rr[0] = st.bb[0] = e[1];
        st.nM = cnt[0];
        st.nU = (double)b.nxy * b.nz - cnt[0];
        st.iters = st.refine_steps = st.refine_iters = 0;
        st.rel = st.true_rel = 0.0;
        st.status = cnt[0] == 0.0 ? RW_ST_NO_DIRICHLET : RW_ST_CONVERGED;
        st.active = (cnt[0] > 0.0 && e[1] > 0.0) ? 1 : 0;
        st.pending = 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_adj_grad(AdjointArgs a, SolveArgs sa) {
    __shared__ double red[kWaves * 12];
    const BrickDev bd = a.bricks[blockIdx.x];
    const Box b = box_of(bd);
    const Weight<float> W = make_weight<float>(a.beta, a.eps);
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
        const BoxState& st = sa.state[blockIdx.x];
        if (a.stats) {
            rw_brick_stats o{};
            o.iters = st.iters;
            o.status = st.status;
            o.rel_resid = st.bb[0] > 0.0 ? sqrt(st.rr[0] / st.bb[0]) : 0.0;
            a.stats[bd.slot] = o;
        }
    }
}

// Sum the per-box dl/dbeta partials in launch order (deterministic).
__global__ __launch_bounds__(kThreads) void k_sum_partials(const double* part, int64_t n, double* out) {
    __shared__ double red[kWaves];
    double s[1] = {0.0};
    for (int64_t i = threadIdx.x; i < n; i += kThreads) s[0] += part[i];
    block_sum<1>(s, red);
    if (threadIdx.x == 0) *out = s[0];
}

// In k_pcg the adjoint keeps rr in st.rr; its final relative residual is read
// back by k_adj_grad from the same state.

// ---------------------------------------------------------------------------
// Launch sequences.
// ---------------------------------------------------------------------------

#define RW_TRY(...)                           \
    do {                                      \
        hipError_t e_ = (__VA_ARGS__);        \
        if (e_ != hipSuccess) return e_;      \
    } while (0)

// The box list is ordered so that boxes whose z-plane exceeds the LDS plane
// march (nx*ny > C*kThreads) come first: [0, n_big) run the global-memory
// march, [n_big, n) the LDS plane march, each kernel compiled for one path.
template <typename T, int R, int C, typename XT>
static hipError_t launch_pcg_plane(const SolveArgs& a, int64_t n, int64_t n_big, XT* xt, int corr, size_t lds,
                                   hipStream_t s) {
    if (n_big > 0)
        hipLaunchKernelGGL((k_pcg<T, R, C, false, XT>), dim3((unsigned)n_big), dim3(kThreads), 0, s, a, xt, corr, 0);
    if (n > n_big) {
        auto k = k_pcg<T, R, C, true, XT>;
        if (lds > 48 * 1024)
            RW_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k, dim3((unsigned)(n - n_big)), dim3(kThreads), lds, s, a, xt, corr, (int)n_big);
    }
    return hipGetLastError();
}

template <typename T, int R, typename XT>
static hipError_t launch_pcg_c(const SolveArgs& a, int64_t n, XT* xt, int corr, const PlanePlan& pp, hipStream_t s) {
    const size_t lds = pp.use ? (size_t)3 * (R + 1) * pp.cols * kThreads * sizeof(T) : 0;
    const int64_t n_big = pp.use ? pp.n_big : n;
    return pp.cols == 2 ? launch_pcg_plane<T, R, 2, XT>(a, n, n_big, xt, corr, lds, s)
                        : launch_pcg_plane<T, R, 4, XT>(a, n, n_big, xt, corr, lds, s);
}

template <int R>
static hipError_t launch_mixed(const SolveArgs& a, int64_t n, const PlanePlan& pp, hipStream_t s) {
    const dim3 grid((unsigned)n), blk(kThreads);
    hipLaunchKernelGGL((k_init<float, R>), grid, blk, 0, s, a);
    RW_TRY(launch_pcg_c<float, R, float>(a, n, a.x, 0, pp, s));
    const bool r64 = a.precision == RW_PREC_MIXED_REFINE;
    if (r64) hipLaunchKernelGGL((k_copy64<R>), grid, blk, 0, s, a, 1);
    for (int step = 0; step < a.refine_max; ++step) {
        if (r64) hipLaunchKernelGGL((k_check<R, true>), grid, blk, 0, s, a, 1);
        else hipLaunchKernelGGL((k_check<R, false>), grid, blk, 0, s, a, 1);
        RW_TRY(launch_pcg_c<float, R, float>(a, n, a.dcorr, 1, pp, s));
        if (r64) hipLaunchKernelGGL((k_apply<R, true>), grid, blk, 0, s, a);
        else hipLaunchKernelGGL((k_apply<R, false>), grid, blk, 0, s, a);
    }
    if (r64) hipLaunchKernelGGL((k_check<R, true>), grid, blk, 0, s, a, 0);
    else hipLaunchKernelGGL((k_check<R, false>), grid, blk, 0, s, a, 0);
    if (r64) hipLaunchKernelGGL((k_copy64<R>), grid, blk, 0, s, a, 0);
    hipLaunchKernelGGL((k_stats<R>), grid, blk, 0, s, a, (a.want_x64 && !r64) ? 1 : 0);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_fp64(const SolveArgs& a, int64_t n, const PlanePlan& pp, hipStream_t s) {
    const dim3 grid((unsigned)n), blk(kThreads);
    hipLaunchKernelGGL((k_init<double, R>), grid, blk, 0, s, a);
    RW_TRY(launch_pcg_c<double, R, double>(a, n, (double*)a.xt, 0, pp, s));
    hipLaunchKernelGGL((k_finish64<R>), grid, blk, 0, s, a);
    hipLaunchKernelGGL((k_stats<R>), grid, blk, 0, s, a, 0);
    return hipGetLastError();
}

size_t plane_lds_bytes(int nrhs, bool fp64, int cols) {
    return (size_t)3 * (nrhs + 1) * cols * kThreads * (fp64 ? 8 : 4);
}

int plane_cols(int max_plane) { return max_plane <= 2 * kThreads ? 2 : 4; }

int plane_max(int cols) { return cols * kThreads; }

hipError_t launch_solve(const SolveArgs& a, int64_t n, int nrhs, bool fp64, const PlanePlan& pp, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (fp64) {
        switch (nrhs) {
            case 1: return launch_fp64<1>(a, n, pp, s);
            case 2: return launch_fp64<2>(a, n, pp, s);
            case 3: return launch_fp64<3>(a, n, pp, s);
        }
    } else {
        switch (nrhs) {
            case 1: return launch_mixed<1>(a, n, pp, s);
            case 2: return launch_mixed<2>(a, n, pp, s);
            case 3: return launch_mixed<3>(a, n, pp, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(const AdjointArgs& a, const SolveArgs& sa, int64_t n, double* dl_dbeta, const PlanePlan& pp,
                          hipStream_t s) {
    if (n > 0) {
        const dim3 grid((unsigned)n), blk(kThreads);
        hipLaunchKernelGGL(k_adj_init, grid, blk, 0, s, a, sa);
        RW_TRY(launch_pcg_c<float, 1, float>(sa, n, a.lambda, 0, pp, s));
        hipLaunchKernelGGL(k_adj_grad, grid, blk, 0, s, a, sa);
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, s, a.beta_part, n, dl_dbeta);
    return hipGetLastError();
}

}  // namespace rwk
