// LDS/register-resident Jacobi-PCG for boxes that fit on one compute unit
// (one right-hand side, FP32 vectors, FP64 reductions; Section III-B system,
// Section V solver).
//
// The streaming kernels read g and the CG vectors from HBM in every sweep.  A
// box of up to ~20k voxels fits in the LDS of one CU instead: g and the
// search direction p live in LDS (8 B per voxel), and each thread keeps its
// own voxels' x, r, 1/d and q = L_UU p in registers (thread t owns voxels
// t + k * NT, so every LDS access of a wave is to consecutive words).  HBM is
// touched only to load the box and to store x at the end, so the iteration
// runs at LDS speed.  Per iteration:
//   p = r/d + beta p      (own voxels, in place in LDS)        barrier
//   q = d p - sum_nb w p_nb, sigma = p.q  (weights recomputed from g in LDS)
//   reduce sigma -> alpha;  x += alpha p, r -= alpha q, z = r/d
//   reduce r.z, ||r||^2 -> beta, convergence test
// The iteration is the same Jacobi-PCG as the streaming kernels (same start
// state, same stopping rule), so the two are interchangeable per box.

#include "common.h"

#include <algorithm>

namespace rwk {

namespace {

// Per-voxel code: bits 0..5 neighbour -x,+x,-y,+y,-z,+z inside the box, bit 6 unknown.
constexpr unsigned kUnknown = 64u;

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

// 1.0f if bit b of c is set, else 0.0f (integer arithmetic only).
__device__ __forceinline__ float bitf(unsigned c, int b) {
    return __uint_as_float((0u - ((c >> b) & 1u)) & 0x3f800000u);
}

// Neighbour offsets of the six stencil directions.
__device__ __forceinline__ void nb_offsets(int nx, int nxy, int (&o)[6]) {
    o[0] = -1;
    o[1] = 1;
    o[2] = -nx;
    o[3] = nx;
    o[4] = -nxy;
    o[5] = nxy;
}

}  // namespace

// One workgroup of NT threads per box; VPT = most voxels a thread owns.
// xt: x (main solve) or the correction accumulator (corr = 1).
//
// LDS holds (g, p) pairs for the box with nx*ny zero pairs before it and
// nx*ny + 1 after it, so every neighbour address v + offset is inside the
// array (pairs that are not in-box neighbours get weight 0).  One 8-byte LDS read per
// neighbour fetches both g and p.
template <int NT, int VPT>
__global__ __launch_bounds__(NT) void k_pcg_res(SolveArgs a, float* xt, int corr, int base) {
    extern __shared__ __align__(16) float2 gp_lds[];
    __shared__ double red[(NT / 64) * 2];
    constexpr int NC = (VPT + 3) / 4;  // 8-bit codes, four per word
    const int ib = base + blockIdx.x;
    BoxState& st = a.state[ib];
    if (!st.active) return;
    const BrickDev bd = a.bricks[ib];
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz, nxy = nx * ny, nv = nxy * nz;
    float2* gp = gp_lds + nxy;
    const float* g = a.g + bd.off;
    const uint8_t* m = a.mask + bd.off;
    float* xb = xt + bd.off;
    const float* rb = (const float*)a.r + bd.off;
    const ResWeight W{(float)(-a.beta * 1.4426950408889634), (float)a.eps};
    int off[6];
    nb_offsets(nx, nxy, off);

    for (int v = (int)threadIdx.x - nxy; v <= nv + nxy; v += NT) gp[v] = make_float2(v >= 0 && v < nv ? g[v] : 0.0f, 0.0f);
    // Per-voxel arrays are only ever updated with selects, never under a
    // branch: a conditional update of one element makes the compiler carry
    // the whole array through the branch (and copy it).  Voxel slots past the
    // end of the box have code 0 and use the first pad pair in LDS (p = 0
    // there is rewritten with 0) and the last voxel for global loads.
    float x[VPT], r[VPT], id[VPT], q[VPT];
    unsigned code[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) code[c] = 0u;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v0 = threadIdx.x + k * NT;
        const int v = v0 < nv ? v0 : nv - 1;  // global index
        const int kz = v / nxy, rem = v - kz * nxy, j = rem / nx, i = rem - j * nx;
        const bool u = v0 < nv && m[v] == 0;
        const unsigned c = (i > 0 ? 1u : 0u) | (i + 1 < nx ? 2u : 0u) | (j > 0 ? 4u : 0u) | (j + 1 < ny ? 8u : 0u) |
                           (kz > 0 ? 16u : 0u) | (kz + 1 < nz ? 32u : 0u) | kUnknown;
        const float xv = xb[v], rv = rb[v];
        x[k] = u ? xv : 0.0f;
        r[k] = u ? rv : 0.0f;
        code[k >> 2] |= (u ? c : 0u) << ((k & 3) * 8);
    }
    auto cd = [&](int k) { return (code[k >> 2] >> ((k & 3) * 8)) & 0xffu; };
    auto slot = [&](int tb, int k) { const int v0 = tb + k * NT; return v0 < nv ? v0 : nv; };  // LDS index
    __syncthreads();
    // 1/d of own unknown voxels (d = sum of the in-box weights; static)
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = slot(threadIdx.x, k);
        const unsigned c = cd(k);
        const float gc = gp[v].x;
        float d = 0.0f;
#pragma unroll
        for (int q6 = 0; q6 < 6; ++q6) d += W(gc, gp[v + off[q6]].x) * bitf(c, q6);
        id[k] = (c & kUnknown) ? __builtin_amdgcn_rcpf(d) : 0.0f;
    }

    double rz = st.rz[0], rr = st.rr[0];
    const double bb = st.bb[0];
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
        // opaque copies: keep per-voxel addresses and neighbour masks inside
        // the loop (hoisting them all would cost VPT * 7 registers and VPT * 6
        // lane masks)
        int tb = threadIdx.x;
        asm volatile("" : "+v"(tb));
#pragma unroll
        for (int c = 0; c < NC; ++c) asm volatile("" : "+v"(code[c]));
        const float be = it == 0 ? 0.0f : (float)betac;
        // p = z + beta p on own unknown voxels (seeded voxels keep p = 0)
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = slot(tb, k);
            const float pn = r[k] * id[k] + be * gp[v].y;
            gp[v].y = (cd(k) & kUnknown) ? pn : 0.0f;
        }
        __syncthreads();
        // q = L_UU p at an own voxel (0 on seeded and unused slots, where p = 0)
        auto apply = [&](int v, unsigned c, float& pv) {
            const float2 self = gp[v];
            float d = 0.0f, acc = 0.0f;
#pragma unroll
            for (int q6 = 0; q6 < 6; ++q6) {
                const float2 nb = gp[v + off[q6]];
                // weight times a 0/1 factor, not a select: a select lets the
                // compiler branch around the exp, which serialises the loads
                const float w = W(self.x, nb.x) * bitf(c, q6);
                d += w;
                acc += w * nb.y;
            }
            pv = self.y;
            return (c & kUnknown) ? d * self.y - acc : 0.0f;
        };
        double sig = 0.0;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            float pv;
            q[k] = apply(slot(tb, k), cd(k), pv);
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
            x[k] += al * gp[v].y;
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
        if (cd(k) & kUnknown) xb[v] = x[k];
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

// Variant for smaller boxes: LDS holds (p, w+x, w+y, w+z) per voxel, the
// weights of the edges to the +x, +y and +z neighbours (0 where that
// neighbour is not in the box), computed once per solve; the pads (as in the
// (g, p) kernel) are all 0.
// A voxel's other three weights are its -x, -y, -z neighbours' forward
// weights, so the stencil is six multiply-adds with no exponential and no
// mask.  16 bytes of LDS per voxel instead of 8.
template <int NT, int VPT>
__global__ __launch_bounds__(NT) void k_pcg_resw(SolveArgs a, float* xt, int corr, int base) {
    extern __shared__ __align__(16) float4 wp_lds[];
    __shared__ double red[(NT / 64) * 2];
    constexpr int NC = (VPT + 31) / 32;  // unknown-voxel bits
    const int ib = base + blockIdx.x;
    BoxState& st = a.state[ib];
    if (!st.active) return;
    const BrickDev bd = a.bricks[ib];
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz, nxy = nx * ny, nv = nxy * nz;
    float4* wp = wp_lds + nxy;
    const float* g = a.g + bd.off;
    const uint8_t* m = a.mask + bd.off;
    float* xb = xt + bd.off;
    const float* rb = (const float*)a.r + bd.off;
    const ResWeight W{(float)(-a.beta * 1.4426950408889634), (float)a.eps};

    // forward weights from g (global loads of the voxel and its +x, +y, +z neighbours)
    for (int v = (int)threadIdx.x - nxy; v <= nv + nxy; v += NT) {
        float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (v >= 0 && v < nv) {
            const int kz = v / nxy, rem = v - kz * nxy, j = rem / nx, i = rem - j * nx;
            const float gc = g[v];
            if (i + 1 < nx) e.y = W(gc, g[v + 1]);
            if (j + 1 < ny) e.z = W(gc, g[v + nx]);
            if (kz + 1 < nz) e.w = W(gc, g[v + nxy]);
        }
        wp[v] = e;
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
    int off_x = 1, off_y = nx, off_z = nxy;
    __syncthreads();
    // d = the six weights of the voxel (its own forward ones and its
    // neighbours' forward ones toward it); static
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = slot(threadIdx.x, k);
        const float4 self = wp[v];
        const float dd = self.y + self.z + self.w + wp[v - off_x].y + wp[v - off_y].z + wp[v - off_z].w;
        d[k] = isu(k) ? dd : 0.0f;
        id[k] = isu(k) ? __builtin_amdgcn_rcpf(dd) : 0.0f;
    }

    double rz = st.rz[0], rr = st.rr[0];
    const double bb = st.bb[0];
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
            const float pn = r[k] * id[k] + be * wp[v].x;
            wp[v].x = isu(k) ? pn : 0.0f;
        }
        __syncthreads();
        double sig = 0.0;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = slot(tb, k);
            const float4 self = wp[v];
            const float2 mx = *reinterpret_cast<const float2*>(&wp[v - off_x]);  // p, w+x of v - 1
            const float4 my = wp[v - off_y];
            const float4 mz = wp[v - off_z];
            const float acc = self.y * wp[v + off_x].x + self.z * wp[v + off_y].x + self.w * wp[v + off_z].x +
                              mx.y * mx.x + my.z * my.x + mz.w * mz.x;
            q[k] = isu(k) ? d[k] * self.x - acc : 0.0f;
            sig += (double)self.x * (double)q[k];
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
            x[k] += al * wp[v].x;
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

// Dynamic LDS of a launch, in elements: the largest box, nx*ny pad elements
// before it and nx*ny + 1 after it (the unused voxel slots of a thread map
// to the element just past the box, whose +z neighbour is the last one).
int64_t resident_lds_elems(int64_t voxels, int64_t plane) { return voxels + 2 * plane + 1; }
size_t resident_lds_bytes(int64_t voxels, int64_t plane) { return (size_t)resident_lds_elems(voxels, plane) * sizeof(float2); }

bool resident_fits(const BrickDev& b, size_t lds_limit) {
    const int64_t nxy = (int64_t)b.nx * b.ny, nv = nxy * b.nz;
    // beside the small static reduction array
    return nv <= (int64_t)kResMaxVpt * kResThreads && resident_lds_bytes(nv, nxy) + 1024 <= lds_limit;
}

bool resident_w_fits(const BrickDev& b, size_t lds_limit) {
    const int64_t nxy = (int64_t)b.nx * b.ny, nv = nxy * b.nz;
    return nv <= (int64_t)kResMaxVptW * kResThreads &&
           (size_t)resident_lds_elems(nv, nxy) * sizeof(float4) + 1024 <= lds_limit;
}

// Boxes [b0, b1) of the launch list, all eligible for the kernel `kind`
// (0: g and p in LDS, 1: weights and p in LDS), largest first.
hipError_t launch_resident(const SolveArgs& a, int64_t b0, int64_t b1, int64_t max_voxels, int64_t max_plane,
                           int kind, float* xt, int corr, hipStream_t s) {
    if (b1 <= b0) return hipSuccess;
    const size_t lds = kind == 1 ? (size_t)resident_lds_elems(max_voxels, max_plane) * sizeof(float4)
                                 : resident_lds_bytes(max_voxels, max_plane);
    const dim3 grid((unsigned)(b1 - b0));
    auto go = [&](auto kern) -> hipError_t {
        if (lds > 48 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, grid, dim3(kResThreads), lds, s, a, xt, corr, (int)b0);
        return hipGetLastError();
    };
    const int64_t vpt = (max_voxels + kResThreads - 1) / kResThreads;
    if (kind == 1) {
        if (vpt <= 10) return go(k_pcg_resw<kResThreads, 10>);
        if (vpt <= kResMaxVptW) return go(k_pcg_resw<kResThreads, kResMaxVptW>);
        return hipErrorInvalidValue;
    }
    if (vpt <= 4) return go(k_pcg_res<kResThreads, 4>);
    if (vpt <= 10) return go(k_pcg_res<kResThreads, 10>);
    if (vpt <= 20) return go(k_pcg_res<kResThreads, 20>);
    if (vpt <= kResMaxVpt) return go(k_pcg_res<kResThreads, kResMaxVpt>);
    return hipErrorInvalidValue;
}

}  // namespace rwk
