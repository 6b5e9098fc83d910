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

#include <algorithm>
#include <type_traits>

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

// Workgroup barrier that orders LDS only.  The march loops keep global loads
// for later chunks in flight across their per-step barriers; __syncthreads()
// would wait for those (its release fence covers global memory too).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// 1 or 0 in T from integer bit operations (a select here can turn into a
// branch around the multiplied exponential).
template <typename T>
__device__ __forceinline__ T unit_or_zero(bool h);
template <>
__device__ __forceinline__ float unit_or_zero<float>(bool h) {
    return __uint_as_float((0u - (unsigned)h) & 0x3f800000u);
}
template <>
__device__ __forceinline__ double unit_or_zero<double>(bool h) {
    return __longlong_as_double((0ll - (long long)h) & 0x3ff0000000000000ll);
}

// Register-ring depth of the window march (3: loads two chunks ahead, 4: three).
#ifndef RW_WINDOW_RING
#define RW_WINDOW_RING 3
#endif
constexpr int kRing = RW_WINDOW_RING;

// Window march: the box is walked as a flat array in chunks of CH = C*kThreads
// consecutive voxels (thread t handles voxels t + q*kThreads of each chunk, so
// every load is coalesced and every thread is busy whatever the box shape).
// A ring of four LDS chunk buffers holds chunks c-1, c, c+1 while chunk c is
// computed, so all six stencil neighbours (+-1, +-nx, +-nx*ny; requires
// nx*ny <= CH) are read from LDS.  Global loads of raw operand values, g, the
// seed mask and NX private extras (e.g. x and r) run three chunks ahead in a
// four-deep register ring that is rotated by unrolling, not by copying.
// prep(raw) turns the raw loads into the N operand values written to LDS.
// Only unknown voxels are visited: visit_u(v, d, acc, self, extras).
template <typename T, int RN, int NX>
struct Slot {
    Val<T, RN> raw;
    Val<T, NX> ex;
    T g;
    unsigned m;
};

// kAligned: the chunk holds a whole number of z-planes (CH % (nx*ny) == 0),
// so each thread keeps its (i, j) from chunk to chunk and advances k by
// CH / (nx*ny): the x and y neighbour tests are computed once.
template <typename T, int N, int RN, int NX, int C, bool kAligned, typename LoadRaw, typename Prep, typename LoadX,
          typename VisitU>
__device__ __forceinline__ void window_march(const Box& b, const float* __restrict__ g,
                                             const uint8_t* __restrict__ m, const Weight<T>& W,
                                             T* __restrict__ lds, LoadRaw loadraw, Prep prep, LoadX loadx,
                                             VisitU visit_u) {
    // box-relative 32-bit indices on uniform base pointers (scalar base + vector offset loads)
    const float* __restrict__ gb = g + b.off;
    const uint8_t* __restrict__ mb = m + b.off;
    constexpr int CH = C * kThreads;
    constexpr int LOG = __builtin_ctz(CH);
    static_assert((1 << LOG) == CH, "chunk must be a power of two");
    constexpr int BS = (N + 1) * CH;
    const int nv = b.nxy * b.nz;
    const int NC = (nv + CH - 1) / CH;
    const int dk = CH / b.nxy, rem = CH - dk * b.nxy, dj = rem / b.nx, di = rem - dj * b.nx;
    int vi[C], ii[C], jj[C], kk[C];
    unsigned xy[C];  // kAligned: bits 0..3 = neighbour -x, +x, -y, +y inside the box
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const int v = q * kThreads + threadIdx.x;
        vi[q] = v;
        kk[q] = v / b.nxy;
        const int r = v - kk[q] * b.nxy;
        jj[q] = r / b.nx;
        ii[q] = r - jj[q] * b.nx;
        xy[q] = (ii[q] > 0 ? 1u : 0u) | (ii[q] + 1 < b.nx ? 2u : 0u) | (jj[q] > 0 ? 4u : 0u) |
                (jj[q] + 1 < b.ny ? 8u : 0u);
    }
    using S = Slot<T, RN, NX>;
    S r0[C], r1[C], r2[C], r3[C];
    (void)r3;
    auto load_chunk = [&](int c, S (&Sl)[C]) {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int v = c * CH + q * kThreads + threadIdx.x;
            if (v < nv) {
                Sl[q].raw = loadraw(v);
                Sl[q].ex = loadx(v);
                Sl[q].g = (T)gb[v];
                Sl[q].m = mb[v];
            }
        }
    };
    auto write_chunk = [&](int c, const S (&Sl)[C]) {
        T* L = lds + (c & 3) * BS;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int v = c * CH + q * kThreads + threadIdx.x;
            if (v < nv) {
                const Val<T, N> op = prep(Sl[q].raw);
                const int o = q * kThreads + threadIdx.x;
#pragma unroll
                for (int a = 0; a < N; ++a) L[a * CH + o] = op.a[a];
                L[N * CH + o] = Sl[q].g;
            }
        }
    };
    auto compute_chunk = [&](const S (&Sl)[C]) {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int v = vi[q];
            if (v < nv && Sl[q].m == 0) {
                const T* self = lds + ((v >> LOG) & 3) * BS + (v & (CH - 1));
                const T gc = Sl[q].g;
                T d = T(0);
                Val<T, N> acc, sv;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    acc.a[a] = T(0);
                    sv.a[a] = self[a * CH];
                }
                // Every neighbour slot is read (the ring wraps, so u outside
                // the box still lands in the LDS ring, which holds finite
                // values) and its weight is multiplied by 0 or 1: branches
                // around the exponentials would serialise the LDS reads.
                auto nb = [&](int u, bool h) {
                    const T* p = lds + ((u >> LOG) & 3) * BS + (u & (CH - 1));
                    const T w = W(gc, p[N * CH]) * unit_or_zero<T>(h);
                    d += w;
#pragma unroll
                    for (int a = 0; a < N; ++a) acc.a[a] += w * p[a * CH];
                };
                if constexpr (kAligned) {
                    nb(v - 1, xy[q] & 1u);
                    nb(v + 1, xy[q] & 2u);
                    nb(v - b.nx, xy[q] & 4u);
                    nb(v + b.nx, xy[q] & 8u);
                } else {
                    nb(v - 1, ii[q] > 0);
                    nb(v + 1, ii[q] + 1 < b.nx);
                    nb(v - b.nx, jj[q] > 0);
                    nb(v + b.nx, jj[q] + 1 < b.ny);
                }
                nb(v - b.nxy, kk[q] > 0);
                nb(v + b.nxy, kk[q] + 1 < b.nz);
                visit_u(v, d, acc, sv, Sl[q].ex);
            }
            vi[q] = v + CH;
            kk[q] += dk;
            if constexpr (!kAligned) {
                ii[q] += di;
                jj[q] += dj;
                if (ii[q] >= b.nx) {
                    ii[q] -= b.nx;
                    jj[q] += 1;
                }
                if (jj[q] >= b.ny) {
                    jj[q] -= b.ny;
                    kk[q] += 1;
                }
            }
        }
    };
    if constexpr (kRing == 4) {
        auto step = [&](int c, S (&s0)[C], S (&s1)[C], S (&s3)[C]) {
            if (c + 3 < NC) load_chunk(c + 3, s3);
            if (c + 1 < NC) write_chunk(c + 1, s1);
            lds_barrier();
            compute_chunk(s0);
        };
        load_chunk(0, r0);
        if (NC > 1) load_chunk(1, r1);
        if (NC > 2) load_chunk(2, r2);
        write_chunk(0, r0);
        for (int c = 0; c < NC; c += 4) {
            step(c, r0, r1, r3);
            if (c + 1 >= NC) break;
            step(c + 1, r1, r2, r0);
            if (c + 2 >= NC) break;
            step(c + 2, r2, r3, r1);
            if (c + 3 >= NC) break;
            step(c + 3, r3, r0, r2);
        }
    } else {
        // three-deep register ring: loads run two chunks ahead
        auto step = [&](int c, S (&s0)[C], S (&s1)[C], S (&s2)[C]) {
            if (c + 2 < NC) load_chunk(c + 2, s2);
            if (c + 1 < NC) write_chunk(c + 1, s1);
            lds_barrier();
            compute_chunk(s0);
        };
        load_chunk(0, r0);
        if (NC > 1) load_chunk(1, r1);
        write_chunk(0, r0);
        for (int c = 0; c < NC; c += 3) {
            step(c, r0, r1, r2);
            if (c + 1 >= NC) break;
            step(c + 1, r1, r2, r0);
            if (c + 2 >= NC) break;
            step(c + 2, r2, r0, r1);
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

// The same true residual as a flat pass over the box's voxels (the check
// phase): thread t takes voxels t + k * kThreads, U at a time, and issues
// every load of the U (g, the seed mask and x at the voxel and its six
// neighbours, indices clamped into the box) before using any, so a thread
// keeps them in flight together instead of waiting plane by plane.  Each
// voxel computes its six weights itself.
template <int R, typename XS, typename RT>
__device__ void true_residual_flat(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                                   const XS* __restrict__ xs, RT* __restrict__ rout, double beta, double eps,
                                   double (&rr)[R], double (&bb)[R]) {
    constexpr int U = R == 1 ? 3 : 2;  // within 128 VGPRs: two workgroups per CU
    const Weight<double> W = make_weight<double>(beta, eps);
    const int nx = b.nx, ny = b.ny, nz = b.nz, nxy = b.nxy;
    const int64_t nv = (int64_t)nxy * nz;
    const float* __restrict__ gb = g + b.off;
    const uint8_t* __restrict__ mb = m + b.off;
    const XS* __restrict__ xb = xs + b.off * R;
    for (int64_t v0 = threadIdx.x; v0 < nv; v0 += (int64_t)U * kThreads) {
        bool in[U][6];
        float gc[U], gn[U][6];
        uint8_t mc[U], mn[U][6];
        XS xc[U][R], xn[U][6][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = v0 + (int64_t)u * kThreads;
            const int64_t c = v < nv ? v : 0;
            const int64_t kz = c / nxy;
            const int rem = (int)(c - kz * nxy), j = rem / nx, i = rem - j * nx;
            const int64_t no[6] = {1, -1, nx, -nx, nxy, -nxy};
            in[u][0] = i + 1 < nx;
            in[u][1] = i > 0;
            in[u][2] = j + 1 < ny;
            in[u][3] = j > 0;
            in[u][4] = kz + 1 < nz;
            in[u][5] = kz > 0;
            gc[u] = gb[c];
            mc[u] = mb[c];
#pragma unroll
            for (int k = 0; k < R; ++k) xc[u][k] = xb[c * R + k];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int64_t nb = in[u][e] ? c + no[e] : c;
                gn[u][e] = gb[nb];
                mn[u][e] = mb[nb];
#pragma unroll
                for (int k = 0; k < R; ++k) xn[u][e][k] = xb[nb * R + k];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = v0 + (int64_t)u * kThreads;
            if (v >= nv || mc[u] != 0) continue;
            double d = 0.0, acc[R], acm[R];
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] = acm[k] = 0.0;
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                if (!in[u][e]) continue;
                const double w = W((double)gc[u], (double)gn[u][e]);
                d += w;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const double xv = (double)xn[u][e][k];
                    acc[k] += w * xv;
                    if (mn[u][e] != 0) acm[k] += w * xv;
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double rv = acc[k] - d * (double)xc[u][k];
                rr[k] += rv * rv;
                bb[k] += acm[k] * acm[k];
                if (rout) rout[(b.off + v) * R + k] = (RT)rv;
            }
        }
    }
}

// Sweep A: p_new = z + beta p_old, sigma = p_new . L_UU p_new.
template <typename T, int R, int C, bool kAligned>
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
        const T* __restrict__ zb = z + b.off * R;
        const T* __restrict__ pb = pold + b.off * R;
        T* __restrict__ nb_ = pnew + b.off * R;
        auto raw = [&](int u) {
            Val<T, 2 * R> o;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                o.a[k] = zb[u * R + k];
                o.a[R + k] = pb[u * R + k];
            }
            return o;
        };
        auto prep = [&](const Val<T, 2 * R>& o) {
            Val<T, R> p;
#pragma unroll
            for (int k = 0; k < R; ++k) p.a[k] = o.a[k] + bk[k] * o.a[R + k];
            return p;
        };
        auto nox = [&](int) { return Val<T, 0>{}; };
        auto vp = [&](int v, T d, const Val<T, R>& acc, const Val<T, R>& self, const Val<T, 0>&) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T q = d * self.a[k] - acc.a[k];
                sig[k] += (double)self.a[k] * (double)q;
                nb_[v * R + k] = self.a[k];
            }
        };
        window_march<T, R, 2 * R, 0, C, kAligned>(b, g, m, W, lds, raw, prep, nox, vp);
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
template <typename T, int R, int C, bool kAligned, typename XT>
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
        const T* __restrict__ pbb = p + b.off * R;
        T* __restrict__ rb = V.r + b.off * R;
        T* __restrict__ zb = V.z + b.off * R;
        XT* __restrict__ xb = xt + b.off * R;
        auto ld = [&](int u) {
            Val<T, R> o;
#pragma unroll
            for (int k = 0; k < R; ++k) o.a[k] = pbb[u * R + k];
            return o;
        };
        auto lx = [&](int u) {
            Val<T, 2 * R> o;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                o.a[k] = (T)xb[u * R + k];
                o.a[R + k] = rb[u * R + k];
            }
            return o;
        };
        auto vp = [&](int v, T d, const Val<T, R>& acc, const Val<T, R>& self, const Val<T, 2 * R>& ex) {
            const T id = recip(d);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T q = d * self.a[k] - acc.a[k];
                xb[v * R + k] = (XT)(ex.a[k] + al[k] * self.a[k]);
                const T rv = ex.a[R + k] - al[k] * q;
                const T zv = rv * id;
                rb[v * R + k] = rv;
                zb[v * R + k] = zv;
                rz[k] += (double)rv * (double)zv;
                rr[k] += (double)rv * (double)rv;
            }
        };
        auto prep = [&](const Val<T, R>& o) { return o; };
        window_march<T, R, R, 2 * R, C, kAligned>(b, g, m, W, lds, ld, prep, lx, vp);
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

template <typename T, int R, int C, bool kPlane, bool kAligned, typename XT>
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
        sweep_pq<T, R, C, kAligned>(b, g, m, V.z, pold, pnew, bk, W, sig, lds, kPlane);
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
        sweep_update<T, R, C, kAligned, XT>(b, g, m, pnew, V, xt, al, W, rzn, rrn, lds, kPlane);
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
// Single-reduction CG (Chronopoulos-Gear) for the window path.
//
// Mathematically the Jacobi-PCG above, reordered so that one stencil sweep
// and one workgroup reduction make an iteration: with z = r/d, w = L_UU z and
// the recurrence s = L_UU p,
//   beta_i  = gamma_i / gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})
//   p = z + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   z = r/d,  w = L_UU z,  gamma = r.z,  delta = w.z,  ||r||^2      (one reduction)
// so the edge weights (and d) are computed once per iteration instead of
// twice.  Storage: V.r = r, V.z = w, V.p[0] = p, V.p[1] = s.
// ---------------------------------------------------------------------------

template <typename T, int R>
struct CgRaw {
    T x[R], r[R], p[R], s[R], w[R];
    T g;
    unsigned m;
};

template <typename T>
struct CgCarry {
    T w[6];
    T d;
    unsigned mk;  // bit 0: unknown voxel; bits 1..6: neighbour -x,+x,-y,+y,-z,+z present
};

// One CG-CG iteration over the box.  Pipeline per step c (chunks of CH
// voxels, thread t owning voxels t + q*kThreads of each chunk):
//   (a) global loads of chunk c+4 into a four-deep register ring,
//   (b) g of chunk c+3 into the LDS g-ring,
//   (c) stage 1, chunk c+1: the six weights and d (g of chunks c..c+2 from
//       LDS), the pointwise updates of p, s, x, r and z = r/d; z goes to the
//       LDS z-ring, weights and d stay in registers,
//   (d) barrier,
//   (e) stage 2, chunk c: w = d z - sum_nb w_nb z_nb from the z-ring; delta.
// Rings of four chunks make every LDS write land in a slot no thread can
// still be reading (one barrier per step).
template <typename T, int R, int C, typename XT>
__device__ void cgcg_sweep(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                           Vecs<T, R> V, XT* __restrict__ xt, const T (&al)[R], const T (&be)[R],
                           const Weight<T>& W, T* __restrict__ lds, double (&gam)[R], double (&del)[R],
                           double (&rr)[R]) {
    constexpr int CH = C * kThreads;
    constexpr int RING = 4 * CH;
    constexpr int RM = RING - 1;
    T* __restrict__ Gr = lds;
    T* __restrict__ Zr = lds + RING;
    const int nv = b.nxy * b.nz;
    const int NC = (nv + CH - 1) / CH;
    const int nx = b.nx, ny = b.ny, nz = b.nz, nxy = b.nxy;
    const float* __restrict__ gb = g + b.off;
    const uint8_t* __restrict__ mb = m + b.off;
    XT* __restrict__ xb = xt + b.off * R;
    T* __restrict__ rb = V.r + b.off * R;
    T* __restrict__ pb = V.p[0] + b.off * R;
    T* __restrict__ sb = V.p[1] + b.off * R;
    T* __restrict__ wb = V.z + b.off * R;
    const int dk = CH / nxy, rem = CH - dk * nxy, dj = rem / nx, di = rem - dj * nx;
    int ii[C], jj[C], kk[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const int v = q * kThreads + threadIdx.x;
        kk[q] = v / nxy;
        const int r0 = v - kk[q] * nxy;
        jj[q] = r0 / nx;
        ii[q] = r0 - jj[q] * nx;
    }
    using Raw = CgRaw<T, R>;
    using Car = CgCarry<T>;
    Raw q0[C], q1[C], q2[C], q3[C];
    Car k0[C], k1[C];

    auto load = [&](int c, Raw (&S)[C]) {
        if (c >= NC) return;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const unsigned v = (unsigned)(c * CH + q * kThreads) + threadIdx.x;
            if (v < (unsigned)nv) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    S[q].x[k] = (T)xb[v * R + k];
                    S[q].r[k] = rb[v * R + k];
                    S[q].p[k] = pb[v * R + k];
                    S[q].s[k] = sb[v * R + k];
                    S[q].w[k] = wb[v * R + k];
                }
                S[q].g = (T)gb[v];
                S[q].m = mb[v];
            }
        }
    };
    auto write_g = [&](int c, const Raw (&S)[C]) {
        if (c >= NC) return;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const unsigned v = (unsigned)(c * CH + q * kThreads) + threadIdx.x;
            if (v < (unsigned)nv) Gr[v & RM] = S[q].g;
        }
    };
    auto stage1 = [&](int c, const Raw (&S)[C], Car (&K)[C]) {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const unsigned v = (unsigned)(c * CH + q * kThreads) + threadIdx.x;
            K[q].mk = 0u;
            if (c < NC && v < (unsigned)nv) {
                const int vm = (int)(v & RM);
                if (S[q].m == 0) {
                    const T gc = S[q].g;
                    const bool f0 = ii[q] > 0, f1 = ii[q] + 1 < nx, f2 = jj[q] > 0, f3 = jj[q] + 1 < ny,
                               f4 = kk[q] > 0, f5 = kk[q] + 1 < nz;
                    const T w0 = f0 ? W(gc, Gr[(vm - 1) & RM]) : T(0);
                    const T w1 = f1 ? W(gc, Gr[(vm + 1) & RM]) : T(0);
                    const T w2 = f2 ? W(gc, Gr[(vm - nx) & RM]) : T(0);
                    const T w3 = f3 ? W(gc, Gr[(vm + nx) & RM]) : T(0);
                    const T w4 = f4 ? W(gc, Gr[(vm - nxy) & RM]) : T(0);
                    const T w5 = f5 ? W(gc, Gr[(vm + nxy) & RM]) : T(0);
                    const T d = ((w0 + w1) + (w2 + w3)) + (w4 + w5);
                    const T id = recip(d);
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const T zi = S[q].r[k] * id;
                        const T pn = zi + be[k] * S[q].p[k];
                        const T sn = S[q].w[k] + be[k] * S[q].s[k];
                        const T rn = S[q].r[k] - al[k] * sn;
                        const T zn = rn * id;
                        pb[v * R + k] = pn;
                        sb[v * R + k] = sn;
                        xb[v * R + k] = (XT)(S[q].x[k] + al[k] * pn);
                        rb[v * R + k] = rn;
                        Zr[k * RING + vm] = zn;
                        gam[k] += (double)rn * (double)zn;
                        rr[k] += (double)rn * (double)rn;
                    }
                    K[q].w[0] = w0;
                    K[q].w[1] = w1;
                    K[q].w[2] = w2;
                    K[q].w[3] = w3;
                    K[q].w[4] = w4;
                    K[q].w[5] = w5;
                    K[q].d = d;
                    K[q].mk = 1u | (f0 ? 2u : 0u) | (f1 ? 4u : 0u) | (f2 ? 8u : 0u) | (f3 ? 16u : 0u) |
                              (f4 ? 32u : 0u) | (f5 ? 64u : 0u);
                } else {
#pragma unroll
                    for (int k = 0; k < R; ++k) Zr[k * RING + vm] = T(0);
                }
            }
            ii[q] += di;
            jj[q] += dj;
            kk[q] += dk;
            if (ii[q] >= nx) {
                ii[q] -= nx;
                jj[q] += 1;
            }
            if (jj[q] >= ny) {
                jj[q] -= ny;
                kk[q] += 1;
            }
        }
    };
    auto stage2 = [&](int c, const Car (&K)[C]) {
        if (c < 0) return;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const unsigned mk = K[q].mk;
            if (mk & 1u) {
                const unsigned v = (unsigned)(c * CH + q * kThreads) + threadIdx.x;
                const int vm = (int)(v & RM);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T* Z = Zr + k * RING;
                    T acc = T(0);
                    if (mk & 2u) acc += K[q].w[0] * Z[(vm - 1) & RM];
                    if (mk & 4u) acc += K[q].w[1] * Z[(vm + 1) & RM];
                    if (mk & 8u) acc += K[q].w[2] * Z[(vm - nx) & RM];
                    if (mk & 16u) acc += K[q].w[3] * Z[(vm + nx) & RM];
                    if (mk & 32u) acc += K[q].w[4] * Z[(vm - nxy) & RM];
                    if (mk & 64u) acc += K[q].w[5] * Z[(vm + nxy) & RM];
                    const T zc = Z[vm];
                    const T wn = K[q].d * zc - acc;
                    wb[v * R + k] = wn;
                    del[k] += (double)wn * (double)zc;
                }
            }
        }
    };
    // step c: load c+4, g of c+3, stage 1 on c+1, barrier, stage 2 on c
    auto step = [&](int c, Raw (&S1)[C], Raw (&S3)[C], Raw (&S4)[C], Car (&Kin)[C], Car (&Kout)[C]) {
        load(c + 4, S4);
        write_g(c + 3, S3);
        stage1(c + 1, S1, Kout);
        lds_barrier();
        stage2(c, Kin);
    };
    load(0, q0);
    load(1, q1);
    load(2, q2);
    write_g(0, q0);
    write_g(1, q1);
    lds_barrier();
    // steps c = -1 .. NC-1; raw ring slot of chunk j is j mod 4, carry slot j mod 2
    for (int c = -1; c < NC; c += 4) {
        step(c, q0, q2, q3, k1, k0);
        if (c + 1 >= NC) break;
        step(c + 1, q1, q3, q0, k0, k1);
        if (c + 2 >= NC) break;
        step(c + 2, q2, q0, q1, k1, k0);
        if (c + 3 >= NC) break;
        step(c + 3, q3, q1, q2, k0, k1);
    }
    __syncthreads();
}

// w0 = L_UU z0 in place over z (V.z), delta0 = z.w0.  Every voxel's z is
// loaded three chunks before its w is written, so the in-place update is safe.
template <typename T, int R, int C>
__device__ void cgcg_init_w(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m, Vecs<T, R> V,
                            const Weight<T>& W, T* lds, double (&del)[R]) {
    T* __restrict__ zb = V.z + b.off * R;
    auto raw = [&](int u) {
        Val<T, R> o;
#pragma unroll
        for (int k = 0; k < R; ++k) o.a[k] = zb[u * R + k];
        return o;
    };
    auto prep = [&](const Val<T, R>& o) { return o; };
    auto nox = [&](int) { return Val<T, 0>{}; };
    auto vp = [&](int v, T d, const Val<T, R>& acc, const Val<T, R>& self, const Val<T, 0>&) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T w = d * self.a[k] - acc.a[k];
            del[k] += (double)self.a[k] * (double)w;
            zb[v * R + k] = w;
        }
    };
    window_march<T, R, R, 0, C, false>(b, g, m, W, lds, raw, prep, nox, vp);
}

template <typename T, int R, int C, typename XT>
__device__ LoopEnd cgcg_loop(const Box& b, const float* __restrict__ g, const uint8_t* __restrict__ m,
                             Vecs<T, R> V, XT* __restrict__ xt, const Weight<T>& W, double (&gam)[R],
                             double (&rr)[R], const double (&bb)[R], double tol, int max_iter, double* red,
                             T* lds) {
    const double tol2 = tol * tol;
    int it = 0, flags = 0;
    bool done[R];
    bool all = true;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        done[k] = rr[k] <= tol2 * bb[k];
        all = all && done[k];
    }
    if (all) return LoopEnd{0, 0};
    if (max_iter <= 0) return LoopEnd{0, 2};
    double del[R];
#pragma unroll
    for (int k = 0; k < R; ++k) del[k] = 0.0;
    cgcg_init_w<T, R, C>(b, g, m, V, W, lds, del);
    block_sum<R>(del, red);
    double alpha[R], beta[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        alpha[k] = done[k] ? 0.0 : gam[k] / del[k];
        beta[k] = 0.0;
        if (!done[k] && !(del[k] > 0.0 && finite(alpha[k]))) flags = 1;
    }
    if (flags) return LoopEnd{0, flags};
    for (;;) {
        T al[R], be[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            al[k] = done[k] ? T(0) : (T)alpha[k];
            be[k] = done[k] ? T(0) : (T)beta[k];
        }
        double acc[3 * R], gn[R], dn[R], rn[R];
#pragma unroll
        for (int k = 0; k < R; ++k) gn[k] = dn[k] = rn[k] = 0.0;
        cgcg_sweep<T, R, C, XT>(b, g, m, V, xt, al, be, W, lds, gn, dn, rn);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            acc[k] = gn[k];
            acc[R + k] = dn[k];
            acc[2 * R + k] = rn[k];
        }
        block_sum<3 * R>(acc, red);
        ++it;
        bool alld = true;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (done[k]) continue;
            const double g1 = acc[k], d1 = acc[R + k], r1 = acc[2 * R + k];
            const double b1 = g1 / gam[k];
            const double den = d1 - b1 * g1 / alpha[k];
            rr[k] = r1;
            gam[k] = g1;
            if (!finite(r1) || !finite(g1)) flags = 1;
            done[k] = r1 <= tol2 * bb[k];
            if (!done[k]) {
                if (!(den > 0.0)) flags = 1;
                beta[k] = b1;
                alpha[k] = g1 / den;
                if (!finite(alpha[k])) flags = 1;
            }
            alld = alld && done[k];
        }
        if (flags) break;
        if (alld) break;
        if (it >= max_iter) {
            flags = 2;
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
__global__ __launch_bounds__(kThreads) void k_init(SolveArgs a, int base) {
    const int ib = base + blockIdx.x;
    __shared__ double red[kWaves * 12];
    const BrickDev bd = a.bricks[ib];
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
        BoxState& st = a.state[ib];
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
        st.checked = 0;
    }
}

// Phase 2: the PCG loop on every active box.  corr = 0: main solve into xt
// (x, or the FP64 accumulator on the FP64 path); corr = 1: FP32 correction
// solve into dcorr from the state init_explicit left (tolerance inner_tol).
template <typename T, int R, int C, bool kPlane, int kSched, typename XT, bool kAligned = false>
__device__ __forceinline__ void pcg_box(SolveArgs a, XT* xt, int corr, int base) {
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
    const double tol = corr ? a.inner_tol : a.tol;
    if constexpr (kPlane) {
        // the window march reads ring slots of chunks outside the box (with
        // weight 0): start from a ring of finite values
        T* L = reinterpret_cast<T*>(dyn_lds);
        for (int i = threadIdx.x; i < 4 * (R + 1) * C * kThreads; i += kThreads) L[i] = T(0);
        __syncthreads();
    }
    LoopEnd e;
    if constexpr (kPlane && kSched == 2)
        e = cgcg_loop<T, R, C, XT>(b, a.g, a.mask, V, xt, W, rz, rr, bb, tol, a.max_iter, red,
                                   reinterpret_cast<T*>(dyn_lds));
    else if constexpr (kPlane)
        e = pcg_loop<T, R, C, true, kAligned, XT>(b, a.g, a.mask, V, xt, W, rz, rr, bb, tol, a.max_iter, red,
                                        reinterpret_cast<T*>(dyn_lds));
    else
        e = pcg_loop<T, R, C, false, false, XT>(b, a.g, a.mask, V, xt, W, rz, rr, bb, tol, a.max_iter, red,
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

template <typename T, int R, int C, bool kPlane, int kSched, typename XT>
__global__ __launch_bounds__(kThreads) void k_pcg(SolveArgs a, XT* xt, int corr, int base) {
    pcg_box<T, R, C, kPlane, kSched, XT>(a, xt, corr, base);
}

// The window-march kernel of the common case (FP32, one rhs, two-sweep
// schedule, planes up to 1024 voxels) held to 128 VGPRs so that two
// 512-thread workgroups share a CU.
template <int C, bool kAligned>
__global__ __launch_bounds__(kThreads, 4) void k_pcg_w1(SolveArgs a, float* xt, int corr, int base) {
    pcg_box<float, 1, C, true, 1, float, kAligned>(a, xt, corr, base);
}

// Phase 3: FP64 true residual of the current solution (x, or x64 when
// refine64), relative to ||b||.  With may_refine, a box whose residual misses
// its target (stall_ratio*tol for MIXED, refine_tol for MIXED_REFINE) gets the
// correction system L_UU d = r64 initialised (r <- r64, z, p, d = 0) and is
// marked active for the next k_pcg(corr = 1).
template <int R, bool kRefine64>
__global__ __launch_bounds__(kThreads) void k_check(SolveArgs a, int may_refine, int base) {
    const int ib = base + blockIdx.x;
    __shared__ double red[kWaves * 12];
    BoxState& st = a.state[ib];
    const bool solved = st.nM > 0.0 && st.nU > 0.0 && st.status != RW_ST_NONFINITE;
    if (!solved) {
        if (threadIdx.x == 0) st.active = 0;
        return;
    }
    // x unchanged since this box's last check (no correction applied): its
    // true residual and verdict stand; only a retried correction needs the pass
    if (st.checked) {
        const bool ok = st.check_ok != 0;
        if (!(may_refine && !ok && st.refine_steps < a.refine_max)) {
            if (threadIdx.x == 0) {
                st.active = 0;
                if (!may_refine && st.refine_steps > 0 && st.status == RW_ST_CONVERGED)
                    st.status = ok ? RW_ST_REFINED : RW_ST_STALLED;
            }
            return;
        }
    }
    const BrickDev bd = a.bricks[ib];
    const Box b = box_of(bd);
    Vecs<float, R> V = vecs<float, R>(a);
    double r2[R], b2[R], q[2 * R];
#pragma unroll
    for (int k = 0; k < R; ++k) r2[k] = b2[k] = 0.0;
    if (kRefine64)
        true_residual_flat<R, double, float>(b, a.g, a.mask, a.x64, V.r, a.beta, a.eps, r2, b2);
    else
        true_residual_flat<R, float, float>(b, a.g, a.mask, a.x, V.r, a.beta, a.eps, r2, b2);
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
        st.checked = 1;
        st.check_ok = ok ? 1 : 0;
        st.active = refine ? 1 : 0;
        if (!may_refine && st.refine_steps > 0 && st.status == RW_ST_CONVERGED)
            st.status = ok ? RW_ST_REFINED : RW_ST_STALLED;
    }
}

// Phase 4: add the correction d to x (MIXED) or to x64 (MIXED_REFINE).
template <int R, bool kRefine64>
__global__ __launch_bounds__(kThreads) void k_apply(SolveArgs a, int base) {
    const int ib = base + blockIdx.x;
    BoxState& st = a.state[ib];
    if (!st.pending) return;
    const Box b = box_of(a.bricks[ib]);
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
        st.checked = 0;
    }
}

// Copy x into the FP64 accumulator (MIXED_REFINE start) or back (end).
template <int R>
__global__ __launch_bounds__(kThreads) void k_copy64(SolveArgs a, int to64, int base) {
    const int ib = base + blockIdx.x;
    const Box b = box_of(a.bricks[ib]);
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
__global__ __launch_bounds__(kThreads) void k_finish64(SolveArgs a, int base) {
    const int ib = base + blockIdx.x;
    __shared__ double red[kWaves * 12];
    BoxState& st = a.state[ib];
    const Box b = box_of(a.bricks[ib]);
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
__global__ __launch_bounds__(kThreads) void k_stats(SolveArgs a, int copy64, int copy_from) {
    const BrickDev bd = a.bricks[blockIdx.x];
    if (copy64 && (int)blockIdx.x >= copy_from) {
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
        st.checked = 0;
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

// The box list is ordered so that the large single domains come first (the
// multi-workgroup solver), then boxes whose z-plane exceeds the LDS plane
// march (nx*ny > C*kThreads, global-memory march), then the rest (LDS plane
// march), each kernel compiled for one path.
template <typename T, int R, int C, typename XT>
static hipError_t launch_pcg_plane(const SolveArgs& a, int64_t n, int64_t n_big, XT* xt, int corr, size_t lds,
                                   const PlanePlan& pp, hipStream_t s) {
    RW_TRY((domain_pcg<T, R, XT>(a, (int)pp.n_dom, pp.host, xt, corr, s)));
    const int64_t n_stream_end = std::min<int64_t>(n, pp.n_res);
    constexpr bool kRes = std::is_same<T, float>::value && std::is_same<XT, float>::value && R == 1;
    // streamed-weights resident launches share the streaming kernel's stream;
    // the other resident launches run on a second stream, concurrently
    bool any_g = false, any_lds = false;
    if (kRes && n > pp.n_res)
        for (int i = 0; i < pp.n_rl; ++i) (pp.rl[i].kind == 2 || pp.rl[i].kind == 4 ? any_g : any_lds) = true;
    const bool any_str = n_stream_end > pp.n_dom;
    const bool on_a = any_str || any_g;
    const bool fork = on_a && any_lds && pp.side[0] != nullptr;
    hipStream_t s_str = s, s_res = s;
    // a second streamed-weights launch (the boxes up to 17408 voxels) runs on
    // a third stream, so that it need not wait for the first one's tail
    const bool third = kRes && fork && pp.third && pp.side[2] != nullptr;
    hipStream_t s_g2 = s;
    if (fork) {
        RW_TRY(hipEventRecord(pp.fork, s));
        RW_TRY(hipStreamWaitEvent(pp.side[0], pp.fork, 0));
        RW_TRY(hipStreamWaitEvent(pp.side[1], pp.fork, 0));
        s_str = pp.side[0];
        s_res = pp.side[1];
        s_g2 = s_str;
        if (third) {
            RW_TRY(hipStreamWaitEvent(pp.side[2], pp.fork, 0));
            s_g2 = pp.side[2];
        }
    }
    hipEvent_t* tev = corr == 0 ? pp.gev : nullptr;
    if (tev && on_a) RW_TRY(hipEventRecord(tev[0], s_str));
    if (n_big > pp.n_dom)
        hipLaunchKernelGGL((k_pcg<T, R, C, false, 1, XT>), dim3((unsigned)(n_big - pp.n_dom)), dim3(kThreads), 0,
                           s_str, a, xt, corr, (int)pp.n_dom);
    if (n_stream_end > n_big) {
        auto k = a.schedule == 2 ? k_pcg<T, R, C, true, 2, XT> : k_pcg<T, R, C, true, 1, XT>;
        if constexpr (kRes && C == 2)
            if (a.schedule != 2) k = pp.plane_aligned ? k_pcg_w1<C, true> : k_pcg_w1<C, false>;
        if (lds > 48 * 1024)
            RW_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k, dim3((unsigned)(n_stream_end - n_big)), dim3(kThreads), lds, s_str, a, xt, corr,
                           (int)n_big);
    }
    if constexpr (kRes) {
        // split boxes first: the largest, two workgroups each
        for (int i = 0; i < pp.n_rl; ++i)
            if (pp.rl[i].kind == 4)
                RW_TRY(launch_split(a, pp.rl[i].b0, pp.rl[i].b1, pp.rl[i].max_plane, xt, corr, s_str));
        int k = 0;
        for (int i = 0; i < pp.n_rl; ++i)
            if (pp.rl[i].kind == 2) {
                const bool second = third && k++ == 1;   // on the third stream, timed on its own
                if (second && tev) RW_TRY(hipEventRecord(tev[4], s_g2));
                // (the streamed-weights kernel's persistent twin spills registers:
                // one workgroup per box for it)
                RW_TRY(launch_resident(a, pp.rl[i].b0, pp.rl[i].b1, pp.rl[i].max_voxels, pp.rl[i].max_plane, 2,
                                       pp.rl[i].px, xt, corr, nullptr, second ? s_g2 : s_str));
                if (second && tev) RW_TRY(hipEventRecord(tev[5], s_g2));
            }
    }
    if (tev && on_a) RW_TRY(hipEventRecord(tev[1], s_str));
    if (third) {
        // the stream group ends when both launches have
        RW_TRY(hipEventRecord(pp.join[2], s_g2));
        RW_TRY(hipStreamWaitEvent(s_str, pp.join[2], 0));
    }
    // first true-residual check of a group's boxes, on its stream, while the
    // other group may still run (the check phase skips them afterwards)
    const bool early = kRes && corr == 0 && a.early_check > 0;
    auto check_range = [&](int64_t b0, int64_t b1, hipStream_t st) {
        if (b1 > b0)
            hipLaunchKernelGGL((k_check<1, false>), dim3((unsigned)(b1 - b0)), dim3(kThreads), 0, st, a,
                               a.early_check - 1, (int)b0);
    };
    if (early) {
        check_range(pp.n_dom, n_stream_end, s_str);
        for (int i = 0; i < pp.n_rl; ++i)
            if (pp.rl[i].kind == 2 || pp.rl[i].kind == 4) check_range(pp.rl[i].b0, pp.rl[i].b1, s_str);
    }
    if constexpr (kRes) {
        if (tev && any_lds) RW_TRY(hipEventRecord(tev[2], s_res));
        for (int i = 0; i < pp.n_rl; ++i)
            if (pp.rl[i].kind != 2 && pp.rl[i].kind != 4)
                RW_TRY(launch_resident(a, pp.rl[i].b0, pp.rl[i].b1, pp.rl[i].max_voxels, pp.rl[i].max_plane,
                                       pp.rl[i].kind, pp.rl[i].px, xt, corr, pp.persist ? a.tickets + i : nullptr,
                                       s_res));
        if (tev && any_lds) RW_TRY(hipEventRecord(tev[3], s_res));
        if (early)
            for (int i = 0; i < pp.n_rl; ++i)
                if (pp.rl[i].kind != 2 && pp.rl[i].kind != 4) check_range(pp.rl[i].b0, pp.rl[i].b1, s_res);
    }
    if (fork) {
        RW_TRY(hipEventRecord(pp.join[0], s_str));
        RW_TRY(hipEventRecord(pp.join[1], s_res));
        RW_TRY(hipStreamWaitEvent(s, pp.join[0], 0));
        RW_TRY(hipStreamWaitEvent(s, pp.join[1], 0));
    }
    return hipGetLastError();
}

template <typename T, int R, typename XT>
static hipError_t launch_pcg_c(const SolveArgs& a, int64_t n, XT* xt, int corr, const PlanePlan& pp, hipStream_t s) {
    const size_t lds = pp.use ? plane_lds_bytes(R, sizeof(T) == 8, pp.cols) : 0;
    const int64_t n_big = pp.use ? pp.n_big : n;
    return pp.cols == 2 ? launch_pcg_plane<T, R, 2, XT>(a, n, n_big, xt, corr, lds, pp, s)
                        : launch_pcg_plane<T, R, 4, XT>(a, n, n_big, xt, corr, lds, pp, s);
}

// Per-box phase kernels cover boxes [nd, n) with one workgroup each; the
// domain boxes [0, nd) run the multi-workgroup phases one after another.
template <int R>
static hipError_t launch_mixed(const SolveArgs& a, int64_t n, const PlanePlan& pp, hipStream_t s, hipEvent_t* ev) {
    const int nd = (int)pp.n_dom;
    const dim3 grid((unsigned)(n - nd)), blk(kThreads);
    const bool rest = n > nd;
    const bool r64 = a.precision == RW_PREC_MIXED_REFINE;
    // the resident kernels [n_res, n) compute their boxes' start state in the
    // main solve themselves; the init phase covers the others
    const int64_t n_init = R == 1 ? std::max<int64_t>(pp.n_res, nd) : n;
    if (n_init > nd) hipLaunchKernelGGL((k_init<float, R>), dim3((unsigned)(n_init - nd)), blk, 0, s, a, nd);
    RW_TRY((domain_init<float, R>(a, nd, pp.host, s)));
    if (ev) RW_TRY(hipEventRecord(ev[0], s));
    SolveArgs am = a;
    am.fused_init = 1;
    // one rhs, FP32 x checked: each kernel group's boxes are checked as soon
    // as the group ends (the check below then skips them)
    am.early_check = R == 1 && !r64 ? 1 + (a.refine_max > 0 ? 1 : 0) : 0;
    RW_TRY(launch_pcg_c<float, R, float>(am, n, a.x, 0, pp, s));
    if (ev) RW_TRY(hipEventRecord(ev[1], s));
    if (r64) {
        if (rest) hipLaunchKernelGGL((k_copy64<R>), grid, blk, 0, s, a, 1, nd);
        RW_TRY(domain_copy64<R>(a, nd, pp.host, 1, s));
    }
    auto check = [&](int may_refine) -> hipError_t {
        if (rest) {
            if (r64) hipLaunchKernelGGL((k_check<R, true>), grid, blk, 0, s, a, may_refine, nd);
            else hipLaunchKernelGGL((k_check<R, false>), grid, blk, 0, s, a, may_refine, nd);
        }
        RW_TRY(r64 ? domain_check<R, true>(a, nd, pp.host, may_refine, s)
                   : domain_check<R, false>(a, nd, pp.host, may_refine, s));
        return hipGetLastError();
    };
    for (int step = 0; step < a.refine_max; ++step) {
        RW_TRY(check(1));
        RW_TRY(launch_pcg_c<float, R, float>(a, n, a.dcorr, 1, pp, s));
        if (rest) {
            if (r64) hipLaunchKernelGGL((k_apply<R, true>), grid, blk, 0, s, a, nd);
            else hipLaunchKernelGGL((k_apply<R, false>), grid, blk, 0, s, a, nd);
        }
        RW_TRY(r64 ? domain_apply<R, true>(a, nd, pp.host, s) : domain_apply<R, false>(a, nd, pp.host, s));
    }
    RW_TRY(check(0));
    if (r64) {
        if (rest) hipLaunchKernelGGL((k_copy64<R>), grid, blk, 0, s, a, 0, nd);
        RW_TRY(domain_copy64<R>(a, nd, pp.host, 0, s));
    }
    const int copy = (a.want_x64 && !r64) ? 1 : 0;
    if (copy)
        RW_TRY(domain_copy64<R>(a, nd, pp.host, 1, s));
    hipLaunchKernelGGL((k_stats<R>), dim3((unsigned)n), blk, 0, s, a, copy, nd);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_fp64(const SolveArgs& a, int64_t n, const PlanePlan& pp, hipStream_t s, hipEvent_t* ev) {
    const int nd = (int)pp.n_dom;
    const dim3 grid((unsigned)(n - nd)), blk(kThreads);
    const bool rest = n > nd;
    if (rest) hipLaunchKernelGGL((k_init<double, R>), grid, blk, 0, s, a, nd);
    RW_TRY((domain_init<double, R>(a, nd, pp.host, s)));
    if (ev) RW_TRY(hipEventRecord(ev[0], s));
    RW_TRY(launch_pcg_c<double, R, double>(a, n, (double*)a.xt, 0, pp, s));
    if (ev) RW_TRY(hipEventRecord(ev[1], s));
    if (rest) hipLaunchKernelGGL((k_finish64<R>), grid, blk, 0, s, a, nd);
    RW_TRY(domain_finish64<R>(a, nd, pp.host, s));
    hipLaunchKernelGGL((k_stats<R>), dim3((unsigned)n), blk, 0, s, a, 0, nd);
    return hipGetLastError();
}

size_t plane_lds_bytes(int nrhs, bool fp64, int cols) {
    return (size_t)4 * (nrhs + 1) * cols * kThreads * (fp64 ? 8 : 4);
}

int plane_cols(int max_plane) { return max_plane <= 2 * kThreads ? 2 : 4; }
// LDS of the window march: four chunk buffers of (nrhs operands + g).

int plane_max(int cols) { return cols * kThreads; }

hipError_t launch_solve(const SolveArgs& a, int64_t n, int nrhs, bool fp64, const PlanePlan& pp, hipStream_t s,
                        hipEvent_t* ev) {
    if (n == 0) return hipSuccess;
    if (fp64) {
        switch (nrhs) {
            case 1: return launch_fp64<1>(a, n, pp, s, ev);
            case 2: return launch_fp64<2>(a, n, pp, s, ev);
            case 3: return launch_fp64<3>(a, n, pp, s, ev);
        }
    } else {
        switch (nrhs) {
            case 1: return launch_mixed<1>(a, n, pp, s, ev);
            case 2: return launch_mixed<2>(a, n, pp, s, ev);
            case 3: return launch_mixed<3>(a, n, pp, s, ev);
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
