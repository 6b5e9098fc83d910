// Hierarchical random walker over the LOD pyramid (arXiv 2103.09564,
// Sections III-A and IV): pyramid build, the level loop with border seeds from
// the parent level, pruning, multi-class and incremental reuse.
//
// Device data of a run: one dense map per level, float [voxel][K-1]
// (classes 1..K-1; class 0 is the complement), and one flag byte per brick.
// Boxes of a level are packed into a workspace (g, seed mask, x), solved by the
// batched box solver (rw_solve_bricks), and their cores scattered back into
// the level map.  The host plans each level from the parent level's brick
// flags (one small read-back per level) and handles the few labels.

#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <tuple>
#include <vector>

struct rw_pyramid {
    int device = 0;
    int levels = 0;
    int64_t dims[RW_MAX_LEVELS][3] = {};   // x, y, z
    float* data[RW_MAX_LEVELS] = {};
    bool host[RW_MAX_LEVELS] = {};         // level in page-locked host memory
};

namespace rwk {
struct LevelRes {
    int64_t dims[3] = {0, 0, 0};   // x, y, z
    int64_t nb[3] = {0, 0, 0};
    float* map = nullptr;
    uint8_t* flags = nullptr;
    size_t map_bytes = 0, flags_bytes = 0;
    bool host = false;             // map in page-locked host memory
};
}  // namespace rwk

struct rw_result {
    int device = 0;
    rw_params params{};
    int levels = 0;
    int R = 1;
    rwk::LevelRes lv[RW_MAX_LEVELS];
    std::vector<rw_seed> seeds;
    rw_run_stats stats{};
};

namespace rwk {

constexpr int kHThreads = 256;
enum : uint8_t { F_REACHED = 1, F_PRUNABLE = 2, F_CFL = 4, F_SOLVED = 8, F_KEPT = 16 };

// Geometry of one packed box of a level (level voxel coordinates).
struct BoxGeo {
    int32_t x0, y0, z0;        // box origin
    int32_t nx, ny, nz;        // box dims
    int32_t cx0, cy0, cz0;     // core origin
    int32_t cnx, cny, cnz;     // core dims
    int32_t faces;             // Dirichlet layer from the parent: bit 0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi, 4 z-lo, 5 z-hi
    int32_t brick;             // brick linear index at the level
    int64_t off;               // packed offset (voxels)
};

struct SeedEntry {
    int64_t v;                 // packed voxel index
    int32_t label;
    int32_t pad;
};

// ---- pyramid ---------------------------------------------------------------

// Global min and max of a uint16 volume: grid-stride, 8 voxels per 16-byte
// load (when the volume is 16-byte aligned), then wave and workgroup
// reductions and one atomic pair per workgroup (a launch has at most
// kMinMaxBlocks workgroups, so the atomics stay few).
constexpr int kMinMaxBlocks = 2048;

__global__ __launch_bounds__(256) void k_minmax_u16(const uint16_t* __restrict__ v, int64_t n, int aligned16,
                                                    unsigned* mm) {
    __shared__ unsigned red[2][4];
    unsigned lo = 0xffffu, hi = 0u;
    const int64_t n8 = aligned16 ? n / 8 : 0;
    const uint4* v8 = reinterpret_cast<const uint4*>(v);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n8; i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 q = v8[i];
        const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned a = w[k] & 0xffffu, b = w[k] >> 16;
            lo = min(lo, min(a, b));
            hi = max(hi, max(a, b));
        }
    }
    for (int64_t i = n8 * 8 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned a = v[i];
        lo = min(lo, a);
        hi = max(hi, a);
    }
    for (int o = 32; o >= 1; o >>= 1) {
        lo = min(lo, (unsigned)__shfl_xor(lo, o, 64));
        hi = max(hi, (unsigned)__shfl_xor(hi, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = lo;
        red[1][threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)blockDim.x / 64; ++w) {
            lo = min(lo, red[0][w]);
            hi = max(hi, red[1][w]);
        }
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}

__global__ void k_normalize_u16(const uint16_t* __restrict__ v, int64_t n, const unsigned* mm, float* __restrict__ g) {
    const float lo = (float)mm[0], range = (float)mm[1] - (float)mm[0];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] = range > 0.0f ? ((float)v[i] - lo) / range : 0.0f;
}

__global__ void k_clip_f32(const float* __restrict__ v, int64_t n, float* __restrict__ g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] = fminf(fmaxf(v[i], 0.0f), 1.0f);
}

// Counts pyramid (Poisson weight): level 0 = the counts as float (uint16 as
// is, float clipped below at 0); after the mean downsampling every level is
// replaced by its square root.
__global__ void k_counts_u16(const uint16_t* __restrict__ v, int64_t n, float* __restrict__ g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] = (float)v[i];
}

__global__ void k_counts_f32(const float* __restrict__ v, int64_t n, float* __restrict__ g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] = fmaxf(v[i], 0.0f);
}

__global__ void k_sqrt_inplace(float* __restrict__ g, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] = sqrtf(g[i]);
}

// Parent voxel = mean of the child voxels its 2x2x2 block holds.
__global__ void k_downsample(const float* __restrict__ c, int64_t cx, int64_t cy, int64_t cz, float* __restrict__ p,
                             int64_t px, int64_t py, int64_t pz) {
    const int64_t n = px * py * pz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % px, y = (i / px) % py, z = i / (px * py);
        float s = 0.0f;
        int cnt = 0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const int64_t X = 2 * x + dx, Y = 2 * y + dy, Z = 2 * z + dz;
                    if (X < cx && Y < cy && Z < cz) {
                        s += c[X + cx * (Y + cy * Z)];
                        ++cnt;
                    }
                }
        p[i] = s / (float)cnt;
    }
}

// ---- level maps ------------------------------------------------------------

// Trilinear taps at cell centres: child index X -> parent coordinate
// (X + 1/2)/2 - 1/2, clamped to [0, n-1].
__device__ __forceinline__ void taps(int64_t X, int64_t n, int64_t& i0, int64_t& i1, float& t) {
    float P = ((float)X + 0.5f) * 0.5f - 0.5f;
    P = fminf(fmaxf(P, 0.0f), (float)(n - 1));
    int64_t a = (int64_t)floorf(P);
    a = a > n - 2 ? n - 2 : a;
    a = a < 0 ? 0 : a;
    i0 = a;
    i1 = a + 1 < n ? a + 1 : n - 1;
    t = P - (float)a;
}

// One workgroup per row (Y, Z) of the child map (grid cy x cz).  The
// workgroup first blends, for every parent x of the row, the four parent
// rows its y and z taps select (in LDS, up to kUpRow parent voxels at a
// time), then each child voxel takes the two x taps from LDS: every parent
// value is loaded once per row instead of eight times per voxel.
constexpr int kUpRow = 1024;  // parent voxels of a row blended at a time

template <int R>
__global__ void k_upsample(const float* __restrict__ pm, int64_t px, int64_t py, int64_t pz, float* __restrict__ cm,
                           int64_t cx, int64_t cy, int64_t cz) {
    __shared__ float yz[kUpRow * R];
    const int64_t Y = blockIdx.x, Z = blockIdx.y;
    int64_t y0, y1, z0, z1;
    float ty, tz;
    taps(Y, py, y0, y1, ty);
    taps(Z, pz, z0, z1, tz);
    const float* r00 = pm + px * (y0 + py * z0) * R;
    const float* r10 = pm + px * (y1 + py * z0) * R;
    const float* r01 = pm + px * (y0 + py * z1) * R;
    const float* r11 = pm + px * (y1 + py * z1) * R;
    float* out = cm + cx * (Y + cy * Z) * R;
    // windows of W children: a child X takes parent x floor(X/2 - 1/4) and
    // the next, so the window [X0, X0 + W) needs at most (W - 1)/2 + 3 <=
    // kUpRow parent voxels from the first child's first tap on
    constexpr int64_t W = 2 * (kUpRow - 4);
    for (int64_t X0 = 0; X0 < cx; X0 += W) {
        int64_t a0, a1;
        float t0;
        taps(X0, px, a0, a1, t0);
        const int64_t na = std::min<int64_t>(kUpRow, px - a0);
        const int64_t X1 = std::min<int64_t>(cx, X0 + W);
        __syncthreads();  // the previous window's readers are done
        for (int64_t q = threadIdx.x; q < na * R; q += blockDim.x) {
            const int64_t e = a0 * R + q;
            const float c0 = (1.0f - ty) * r00[e] + ty * r10[e];
            const float c1 = (1.0f - ty) * r01[e] + ty * r11[e];
            yz[q] = (1.0f - tz) * c0 + tz * c1;
        }
        __syncthreads();
        for (int64_t X = X0 + threadIdx.x; X < X1; X += blockDim.x) {
            int64_t x0, x1;
            float tx;
            taps(X, px, x0, x1, tx);
#pragma unroll
            for (int k = 0; k < R; ++k)
                out[X * R + k] = (1.0f - tx) * yz[(x0 - a0) * R + k] + tx * yz[(x1 - a0) * R + k];
        }
    }
}

// One workgroup per box: gather g, set the Dirichlet layer on border faces,
// x = trilinear sample of the parent level map (border values and warm
// start), or 0 on the coarsest level (pm == nullptr).  The parent map is read
// directly, so cores already written into this level's map never leak into
// another box's border.
//
// ps = 0: one packed box per box, x interleaved [voxel][class].  ps > 0 (the
// per-class layout): the packed boxes repeat once per class at strides of ps
// voxels, g and the mask copied into each, x of class c in copy c, so that
// each class solves as a box of its own.
template <int R>
__global__ void k_setup(const BoxGeo* __restrict__ geo, const float* __restrict__ glev, int64_t Dx, int64_t Dy,
                        const float* __restrict__ pm, int64_t px, int64_t py, int64_t pz,
                        const float* __restrict__ warm, float* __restrict__ gb, uint8_t* __restrict__ mb,
                        float* __restrict__ xb, int64_t ps) {
    const BoxGeo b = geo[blockIdx.x];
    const int nxy = b.nx * b.ny, n = nxy * b.nz;  // (box voxels fit 32 bits)
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int k = t / nxy, rem = t - k * nxy, j = rem / b.nx, i = rem - j * b.nx;
        const int64_t X = b.x0 + i, Y = b.y0 + j, Z = b.z0 + k;
        const int64_t L = X + Dx * (Y + Dy * Z);
        const int64_t v = b.off + t;
        const float gv = glev[L];
        const bool border = ((b.faces & 1) && i == 0) || ((b.faces & 2) && i == b.nx - 1) ||
                            ((b.faces & 4) && j == 0) || ((b.faces & 8) && j == b.ny - 1) ||
                            ((b.faces & 16) && k == 0) || ((b.faces & 32) && k == b.nz - 1);
        // the border takes the parent sample; with a warm map (a previous
        // result of this level) the unseeded voxels start from it instead
        const bool from_warm = warm && !border;
        int64_t x0 = 0, x1 = 0, y0 = 0, y1 = 0, z0 = 0, z1 = 0;
        float tx = 0.0f, ty = 0.0f, tz = 0.0f;
        if (pm && !from_warm) {
            taps(X, px, x0, x1, tx);
            taps(Y, py, y0, y1, ty);
            taps(Z, pz, z0, z1, tz);
        }
#pragma unroll
        for (int c = 0; c < R; ++c) {
            float xv = 0.0f;
            if (from_warm) {
                xv = warm[L * R + c];
            } else if (pm) {
                auto P = [&](int64_t a, int64_t bb, int64_t cc) { return pm[(a + px * (bb + py * cc)) * R + c]; };
                const float c00 = (1.0f - tx) * P(x0, y0, z0) + tx * P(x1, y0, z0);
                const float c10 = (1.0f - tx) * P(x0, y1, z0) + tx * P(x1, y1, z0);
                const float c01 = (1.0f - tx) * P(x0, y0, z1) + tx * P(x1, y0, z1);
                const float c11 = (1.0f - tx) * P(x0, y1, z1) + tx * P(x1, y1, z1);
                const float c0 = (1.0f - ty) * c00 + ty * c10;
                const float c1 = (1.0f - ty) * c01 + ty * c11;
                xv = (1.0f - tz) * c0 + tz * c1;
            }
            if (ps) {
                gb[c * ps + v] = gv;
                mb[c * ps + v] = border ? 1 : 0;
                xb[c * ps + v] = xv;
            } else {
                xb[v * R + c] = xv;
            }
        }
        if (!ps) {
            gb[v] = gv;
            mb[v] = border ? 1 : 0;
        }
    }
}

// User seeds override: x = [label == class] for classes 1..K-1.
// (ps as in k_setup)
template <int R>
__global__ void k_seeds(const SeedEntry* __restrict__ e, int64_t n, uint8_t* __restrict__ mb, float* __restrict__ xb,
                        int64_t ps) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const SeedEntry s = e[i];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        if (ps) mb[c * ps + s.v] = 1;
        xb[ps ? c * ps + s.v : s.v * R + c] = s.label == c + 1 ? 1.0f : 0.0f;
    }
    if (!ps) mb[s.v] = 1;
}

// Keep the box solution's core (eq. 3, contraction).
// (ps as in k_setup)
template <int R>
__global__ void k_contract(const BoxGeo* __restrict__ geo, const float* __restrict__ xb, int64_t Dx, int64_t Dy,
                           float* __restrict__ lmap, int64_t ps) {
    const BoxGeo b = geo[blockIdx.x];
    const int64_t n = (int64_t)b.cnx * b.cny * b.cnz;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int i = (int)(t % b.cnx), j = (int)((t / b.cnx) % b.cny), k = (int)(t / ((int64_t)b.cnx * b.cny));
        const int X = b.cx0 + i, Y = b.cy0 + j, Z = b.cz0 + k;
        const int64_t L = X + Dx * (Y + Dy * (int64_t)Z);
        const int64_t v = b.off + (X - b.x0) + (int64_t)b.nx * ((Y - b.y0) + (int64_t)b.ny * (Z - b.z0));
#pragma unroll
        for (int c = 0; c < R; ++c) lmap[L * R + c] = xb[ps ? c * ps + v : v * R + c];
    }
}

// Reuse a previous result's core (incremental update).
template <int R>
__global__ void k_copy_core(const BoxGeo* __restrict__ geo, const float* __restrict__ src, int64_t Dx, int64_t Dy,
                            float* __restrict__ dst) {
    const BoxGeo b = geo[blockIdx.x];
    const int64_t n = (int64_t)b.cnx * b.cny * b.cnz;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int i = (int)(t % b.cnx), j = (int)((t / b.cnx) % b.cny), k = (int)(t / ((int64_t)b.cnx * b.cny));
        const int64_t L = (b.cx0 + i) + Dx * ((b.cy0 + j) + Dy * (int64_t)(b.cz0 + k));
#pragma unroll
        for (int c = 0; c < R; ++c) dst[L * R + c] = src[L * R + c];
    }
}

// Block-wide float min / max.
__device__ __forceinline__ void block_minmax(float& lo, float& hi, float* red) {
    for (int o = 32; o >= 1; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * w] = lo;
        red[2 * w + 1] = hi;
    }
    __syncthreads();
    lo = red[0];
    hi = red[1];
    for (int i = 1; i < nw; ++i) {
        lo = fminf(lo, red[2 * i]);
        hi = fmaxf(hi, red[2 * i + 1]);
    }
    __syncthreads();
}

// Pruning tests on a brick core of the level map (Section IV-D1):
// hom = max - min < t_hom (every class, the complement included, when K > 2),
// dt = min - 0.5 > t_bin or 0.5 - max > t_bin (K = 2 only);
// prunable = (hom or dt) and not cfl.  One workgroup per brick.
template <int R>
__global__ void k_prune(const BoxGeo* __restrict__ geo, const float* __restrict__ lmap, int64_t Dx, int64_t Dy,
                        float t_hom, float t_bin, int use_hom, int use_dt, uint8_t* __restrict__ flags) {
    __shared__ float red[2 * 16];
    const BoxGeo b = geo[blockIdx.x];
    const int64_t n = (int64_t)b.cnx * b.cny * b.cnz;
    float lo[R + 1], hi[R + 1];
#pragma unroll
    for (int c = 0; c <= R; ++c) {
        lo[c] = INFINITY;
        hi[c] = -INFINITY;
    }
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int i = (int)(t % b.cnx), j = (int)((t / b.cnx) % b.cny), k = (int)(t / ((int64_t)b.cnx * b.cny));
        const int64_t L = (b.cx0 + i) + Dx * ((b.cy0 + j) + Dy * (int64_t)(b.cz0 + k));
        float sum = 0.0f;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const float v = lmap[L * R + c];
            sum += v;
            lo[c] = fminf(lo[c], v);
            hi[c] = fmaxf(hi[c], v);
        }
        lo[R] = fminf(lo[R], 1.0f - sum);
        hi[R] = fmaxf(hi[R], 1.0f - sum);
    }
    bool hom = true;
#pragma unroll
    for (int c = 0; c <= R; ++c) {
        block_minmax(lo[c], hi[c], red);
        if (c < R || R > 1) hom = hom && (hi[c] - lo[c] < t_hom);
    }
    const bool dt = R == 1 && ((lo[0] - 0.5f > t_bin) || (0.5f - hi[0] > t_bin));
    if (threadIdx.x == 0) {
        uint8_t f = flags[b.brick];
        const bool prunable = ((use_hom && hom) || (use_dt && dt)) && !(f & F_CFL);
        flags[b.brick] = prunable ? (uint8_t)(f | F_PRUNABLE) : (uint8_t)(f & ~F_PRUNABLE);
    }
}

// Incremental: max |new - old| of the parent level map over the parent voxels
// a box samples, [(lo-1)/2, hi/2] per axis, clamped.  One workgroup per box.
// Max abs difference of two maps of one level over each box's core (all
// classes): the similarity test of the node rule.
template <int R>
__global__ void k_core_change(const BoxGeo* __restrict__ geo, const float* __restrict__ a, const float* __restrict__ b_,
                              int64_t Dx, int64_t Dy, float* __restrict__ out) {
    __shared__ float red[2 * 16];
    const BoxGeo b = geo[blockIdx.x];
    const int64_t n = (int64_t)b.cnx * b.cny * b.cnz;
    float m = 0.0f, dummy = 0.0f;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int i = (int)(t % b.cnx), j = (int)((t / b.cnx) % b.cny), k = (int)(t / ((int64_t)b.cnx * b.cny));
        const int64_t L = (b.cx0 + i) + Dx * ((b.cy0 + j) + Dy * (int64_t)(b.cz0 + k));
#pragma unroll
        for (int c = 0; c < R; ++c) m = fmaxf(m, fabsf(a[L * R + c] - b_[L * R + c]));
    }
    float lo = -m;
    block_minmax(lo, dummy, red);
    if (threadIdx.x == 0) out[blockIdx.x] = -lo;
}

template <int R>
__global__ void k_parent_change(const BoxGeo* __restrict__ geo, const float* __restrict__ pn, const float* __restrict__ po,
                                int64_t Px, int64_t Py, int64_t Pz, float* __restrict__ out) {
    __shared__ float red[2 * 16];
    const BoxGeo b = geo[blockIdx.x];
    auto lo_of = [](int a) { return a - 1 >= 0 ? (a - 1) / 2 : 0; };
    const int64_t ax = lo_of(b.x0), ay = lo_of(b.y0), az = lo_of(b.z0);
    const int64_t bx = std::min<int64_t>((b.x0 + b.nx) / 2, Px - 1), by = std::min<int64_t>((b.y0 + b.ny) / 2, Py - 1),
                  bz = std::min<int64_t>((b.z0 + b.nz) / 2, Pz - 1);
    const int64_t sx = bx - ax + 1, sy = by - ay + 1, sz = bz - az + 1;
    float m = 0.0f, dummy = 0.0f;
    for (int64_t t = threadIdx.x; t < sx * sy * sz; t += blockDim.x) {
        const int64_t X = ax + t % sx, Y = ay + (t / sx) % sy, Z = az + t / (sx * sy);
        const int64_t L = X + Px * (Y + Py * Z);
#pragma unroll
        for (int c = 0; c < R; ++c) m = fmaxf(m, fabsf(pn[L * R + c] - po[L * R + c]));
    }
    float lo = -m;
    block_minmax(lo, dummy, red);
    if (threadIdx.x == 0) out[blockIdx.x] = -lo;
}

template <int R>
__global__ void k_materialize(const float* __restrict__ lmap, int64_t n, int cls, float* __restrict__ prob,
                              uint8_t* __restrict__ labels) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float v[R + 1];
        float sum = 0.0f;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            v[c + 1] = lmap[i * R + c];
            sum += v[c + 1];
        }
        v[0] = 1.0f - sum;
        if (prob) prob[i] = v[cls];
        if (labels) {
            int best = 0;
#pragma unroll
            for (int c = 1; c <= R; ++c)
                if (v[c] > v[best]) best = c;
            labels[i] = (uint8_t)best;
        }
    }
}

static unsigned grid_for(int64_t n, int threads) {
    const int64_t g = (n + threads - 1) / threads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// The buffers of freed results and pyramids (level maps, brick flags,
// pyramid levels) are kept per device for the next allocation of the same
// size, since hipFree synchronises the device and a run allocates two buffers
// per level: at most kPoolBytes per device are kept, the rest is freed.  An
// allocation that fails empties the device's cache and is tried once more;
// rw_ctx_destroy empties it too.  The cache is never destroyed (no hipFree
// at process exit).
constexpr size_t kPoolBytes = size_t(8) << 30;
struct BufPool {
    std::mutex mu;
    std::multimap<std::pair<int, size_t>, void*> idle;  // (device, bytes) -> buffer
    std::map<int, size_t> held;                         // idle bytes per device
};
static BufPool& buf_pool() {
    static BufPool* p = new BufPool();
    return *p;
}
// Frees the idle buffers of `dev` (the current device).
void pool_trim(int dev) {
    BufPool& P = buf_pool();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto it = P.idle.begin(); it != P.idle.end();) {
        if (it->first.first == dev) {
            (void)hipFree(it->second);
            it = P.idle.erase(it);
        } else {
            ++it;
        }
    }
    P.held[dev] = 0;
}
// A buffer of `bytes` on `dev` (the current device): a cached one of that
// size, else hipMalloc.
static hipError_t pool_alloc(int dev, void** out, size_t bytes) {
    BufPool& P = buf_pool();
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto it = P.idle.find({dev, bytes});
        if (it != P.idle.end()) {
            *out = it->second;
            P.held[dev] -= bytes;
            P.idle.erase(it);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        pool_trim(dev);
        e = hipMalloc(out, bytes);
    }
    return e;
}
// Returns a buffer no queued work uses any more (the caller has synchronised).
static void pool_release(int dev, void* p, size_t bytes) {
    if (!p) return;
    BufPool& P = buf_pool();
    std::lock_guard<std::mutex> g(P.mu);
    if (P.held[dev] + bytes > kPoolBytes) {
        (void)hipFree(p);
        return;
    }
    P.idle.insert({{dev, bytes}, p});
    P.held[dev] += bytes;
}

// ---- host planning ------------------------------------------------------------

struct LevelGeo {
    int64_t D[3];    // x, y, z
    int64_t nb[3];
};

// Brick b (bx, by, bz) -> box geometry (core and expanded box, clipped).
// Page-locked host memory that kernels read and write in place, for levels
// larger than device memory (Section IV-A: bricks are small, the volume need
// not be).  Coherent: every device access goes to host memory, so no XCD's
// cache keeps a stale copy between kernels.
static hipError_t host_alloc(void** out, size_t bytes) {
    *out = nullptr;
    return hipHostMalloc(out, std::max<size_t>(bytes, 4), hipHostMallocMapped | hipHostMallocCoherent);
}

// Whether kernels may read p: device memory or page-locked host memory
// (pageable host memory would fault the device).
static bool device_readable(const void* p) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeHost || at.type == hipMemoryTypeManaged;
}

static BoxGeo brick_box(const LevelGeo& L, int s, double e, int64_t bx, int64_t by, int64_t bz) {
    const int se = (int)std::floor(e * s);
    const int lo_pad = (se - s) / 2, hi_pad = se - s - lo_pad;
    BoxGeo g{};
    const int64_t bi[3] = {bx, by, bz};
    int32_t c0[3], c1[3], b0[3], b1[3];
    for (int a = 0; a < 3; ++a) {
        c0[a] = (int32_t)(bi[a] * s);
        c1[a] = (int32_t)std::min<int64_t>((bi[a] + 1) * s, L.D[a]);
        b0[a] = std::max(c0[a] - lo_pad, 0);
        b1[a] = (int32_t)std::min<int64_t>(c1[a] + hi_pad, L.D[a]);
    }
    g.x0 = b0[0]; g.y0 = b0[1]; g.z0 = b0[2];
    g.nx = b1[0] - b0[0]; g.ny = b1[1] - b0[1]; g.nz = b1[2] - b0[2];
    g.cx0 = c0[0]; g.cy0 = c0[1]; g.cz0 = c0[2];
    g.cnx = c1[0] - c0[0]; g.cny = c1[1] - c0[1]; g.cnz = c1[2] - c0[2];
    g.faces = 0;
    for (int a = 0; a < 3; ++a) {
        if (b0[a] > 0) g.faces |= 1 << (2 * a);
        if (b1[a] < L.D[a]) g.faces |= 2 << (2 * a);
    }
    g.brick = (int32_t)(bx + L.nb[0] * (by + L.nb[1] * bz));
    return g;
}

static bool in_box(const BoxGeo& g, int64_t X, int64_t Y, int64_t Z) {
    return X >= g.x0 && X < g.x0 + g.nx && Y >= g.y0 && Y < g.y0 + g.ny && Z >= g.z0 && Z < g.z0 + g.nz;
}

// Level-l label grid, sparse: voxel linear index -> class, or -2 (conflict).
static std::map<int64_t, int> rasterize(const std::vector<rw_seed>& seeds, int level, const LevelGeo& L) {
    std::map<int64_t, int> lab;
    const double f = std::ldexp(1.0, level);
    for (const rw_seed& s : seeds) {
        const int64_t X = (int64_t)std::floor(s.x / f), Y = (int64_t)std::floor(s.y / f),
                      Z = (int64_t)std::floor(s.z / f);
        if (X < 0 || Y < 0 || Z < 0 || X >= L.D[0] || Y >= L.D[1] || Z >= L.D[2]) continue;
        const int64_t v = X + L.D[0] * (Y + L.D[1] * Z);
        auto it = lab.find(v);
        if (it == lab.end()) lab[v] = s.label;
        else if (it->second >= 0 && it->second != s.label) it->second = -2;
    }
    return lab;
}

// Bricks whose (expanded, clipped) box contains voxel (X, Y, Z).
template <typename F>
static void bricks_containing(const LevelGeo& L, int s, double e, int64_t X, int64_t Y, int64_t Z, F f) {
    const int se = (int)std::floor(e * s);
    const int pad = std::max((se - s) / 2, se - s - (se - s) / 2);
    const int64_t P[3] = {X, Y, Z};
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = std::max<int64_t>(0, (P[a] - pad) / s - 1);
        hi[a] = std::min<int64_t>(L.nb[a] - 1, (P[a] + pad) / s + 1);
    }
    for (int64_t bz = lo[2]; bz <= hi[2]; ++bz)
        for (int64_t by = lo[1]; by <= hi[1]; ++by)
            for (int64_t bx = lo[0]; bx <= hi[0]; ++bx) {
                const BoxGeo g = brick_box(L, s, e, bx, by, bz);
                if (in_box(g, X, Y, Z)) f(g.brick);
            }
}

struct Planner {
    rw_ctx* ctx;
    hipStream_t s;
    int R;
    const rw_params* p;

    int ensure(void** buf, size_t* have, size_t bytes) {
        hipError_t e = grow(ctx, buf, have, std::max<size_t>(bytes, 256), s);
        return e == hipSuccess ? RW_OK : hip_fail(ctx, e, "allocating hierarchy workspace");
    }
};

template <typename T>
static int upload(rw_ctx* ctx, void* dst, const std::vector<T>& v, hipStream_t s) {
    if (v.empty()) return RW_OK;
    hipError_t e = hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    return e == hipSuccess ? RW_OK : hip_fail(ctx, e, "uploading hierarchy plan");
}

#define H_TRY(x)                     \
    do {                             \
        int rc_ = (x);               \
        if (rc_ != RW_OK) return rc_; \
    } while (0)
#define H_HIP(x, what)                                   \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

template <int R>
static void launch_setup(const BoxGeo* geo, int64_t n, const float* glev, int64_t Dx, int64_t Dy, const float* pm,
                         const int64_t* PD, const float* warm, float* gb, uint8_t* mb, float* xb, int64_t ps,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_setup<R>, dim3((unsigned)n), dim3(kHThreads), 0, s, geo, glev, Dx, Dy, pm, PD ? PD[0] : 0,
                       PD ? PD[1] : 0, PD ? PD[2] : 0, warm, gb, mb, xb, ps);
}

// Solve the listed boxes of a level and scatter their cores into lmap.
// `geos` are the boxes (host); `entries` the seed overrides per packed voxel;
// `warm` (or null): a previous map of this level to start the unseeded
// voxels from.
template <int R>
static int solve_boxes(rw_ctx* ctx, hipStream_t s, const rw_params& P, const LevelGeo& L, const float* glev,
                       float* lmap, const float* pmap, const int64_t* PD, std::vector<BoxGeo>& geos,
                       const std::map<int64_t, int>& lab, rw_run_stats* st, int level, const float* warm) {
    const int top = pmap == nullptr;
    // each class a box of its own below the coarsest level (rw_params.joint_classes)
    const bool per_class = R > 1 && P.precision != RW_PREC_FP64 && !top && P.joint_classes == 0;
    const int64_t maxv_batch = ((int64_t)1 << 28) / (per_class ? R : 1);   // voxels per batch
    size_t i0 = 0;
    while (i0 < geos.size()) {
        // batch [i0, i1)
        int64_t nv = 0;
        size_t i1 = i0;
        while (i1 < geos.size()) {
            const int64_t v = (int64_t)geos[i1].nx * geos[i1].ny * geos[i1].nz;
            if (i1 > i0 && nv + v > maxv_batch) break;
            geos[i1].off = nv;
            nv += v;
            ++i1;
        }
        const int64_t nb = (int64_t)(i1 - i0);
        // seed entries of this batch
        std::vector<SeedEntry> ent;
        std::map<int32_t, size_t> brick_to_box;
        for (size_t i = i0; i < i1; ++i) brick_to_box[geos[i].brick] = i;
        for (const auto& kv : lab) {
            if (kv.second < 0) continue;
            const int64_t v = kv.first;
            const int64_t X = v % L.D[0], Y = (v / L.D[0]) % L.D[1], Z = v / (L.D[0] * L.D[1]);
            auto add = [&](int32_t brick) {
                auto it = brick_to_box.find(brick);
                if (it == brick_to_box.end()) return;
                const BoxGeo& g = geos[it->second];
                const int64_t pv = g.off + (X - g.x0) + (int64_t)g.nx * ((Y - g.y0) + (int64_t)g.ny * (Z - g.z0));
                ent.push_back(SeedEntry{pv, kv.second, 0});
            };
            if (top) add(geos[i0].brick);
            else bricks_containing(L, P.brick, P.expand, X, Y, Z, add);
        }
        // workspace: g f32, x f32 * R, mask u8 | geo, seed entries, stats
        // (per class: g and the mask once per class too, copy c at c * nv)
        const int64_t ps = per_class ? nv : 0;
        const int64_t ncopy = per_class ? R : 1;
        const size_t bx = ((size_t)nv * R * 4 + 255) & ~size_t(255);
        const size_t bg = ((size_t)nv * ncopy * 4 + 255) & ~size_t(255);
        const size_t bm = ((size_t)nv * ncopy + 255) & ~size_t(255);
        H_HIP(grow(ctx, &ctx->hws, &ctx->hws_bytes, bx + bg + bm, s), "allocating packed boxes");
        char* w = (char*)ctx->hws;
        float* xb = (float*)w;
        float* gb = (float*)(w + bx);
        uint8_t* mb = (uint8_t*)(w + bx + bg);
        const size_t gg = ((size_t)nb * sizeof(BoxGeo) + 255) & ~size_t(255);
        const size_t ge = ((ent.size() + 1) * sizeof(SeedEntry) + 255) & ~size_t(255);
        const size_t gs = (size_t)nb * ncopy * sizeof(rw_brick_stats);
        H_HIP(grow(ctx, &ctx->hgeo, &ctx->hgeo_bytes, gg + ge + gs, s), "allocating box geometry");
        BoxGeo* dgeo = (BoxGeo*)ctx->hgeo;
        SeedEntry* dent = (SeedEntry*)((char*)ctx->hgeo + gg);
        rw_brick_stats* dst = (rw_brick_stats*)((char*)ctx->hgeo + gg + ge);
        std::vector<BoxGeo> part(geos.begin() + i0, geos.begin() + i1);
        H_TRY(upload(ctx, dgeo, part, s));
        H_TRY(upload(ctx, dent, ent, s));
        launch_setup<R>(dgeo, nb, glev, L.D[0], L.D[1], pmap, PD, warm, gb, mb, xb, ps, s);
        if (!ent.empty())
            hipLaunchKernelGGL(k_seeds<R>, dim3(grid_for((int64_t)ent.size(), kHThreads)), dim3(kHThreads), 0, s, dent,
                               (int64_t)ent.size(), mb, xb, ps);
        H_HIP(hipGetLastError(), "launching box setup");
        // batched box solve (per class: class c of box i is box c * nb + i)
        std::vector<rw_brick> br((size_t)(nb * ncopy));
        for (int64_t c = 0; c < ncopy; ++c)
            for (int64_t i = 0; i < nb; ++i)
                br[(size_t)(c * nb + i)] = rw_brick{part[(size_t)i].nx, part[(size_t)i].ny, part[(size_t)i].nz, 0,
                                                     c * ps + part[(size_t)i].off};
        rw_solve_params sp;
        rw_solve_params_default(&sp);
        sp.beta = P.beta;
        sp.eps = P.eps;
        sp.tol = P.tol;
        sp.max_iter = P.max_iter;
        sp.precision = P.precision;
        sp.nrhs = per_class ? 1 : R;
        sp.refine_max = P.refine_max;
        sp.schedule = P.schedule;
        H_TRY(rw_solve_bricks(ctx, &sp, nb * ncopy, br.data(), nv * ncopy, gb, mb, xb, nullptr, dst, s));
        hipLaunchKernelGGL(k_contract<R>, dim3((unsigned)nb), dim3(kHThreads), 0, s, dgeo, xb, L.D[0], L.D[1], lmap,
                           ps);
        H_HIP(hipGetLastError(), "launching contraction");
        // stats (the workspaces are reused by the next batch: sync)
        std::vector<rw_brick_stats> hs((size_t)(nb * ncopy));
        H_HIP(hipMemcpyAsync(hs.data(), dst, hs.size() * sizeof(rw_brick_stats), hipMemcpyDeviceToHost, s),
              "reading solver stats");
        H_HIP(hipStreamSynchronize(s), "synchronising level");
        for (int64_t i = 0; i < nb; ++i) {
            // a box's sweeps and status over its classes, as a joint solve reports them
            int32_t it = 0, rit = 0;
            bool bad = false;
            for (int64_t c = 0; c < ncopy; ++c) {
                const rw_brick_stats& q = hs[(size_t)(c * nb + i)];
                it = std::max(it, q.iters);
                rit = std::max(rit, q.refine_iters);
                bad = bad || q.status == RW_ST_MAX_ITER || q.status == RW_ST_STALLED || q.status == RW_ST_NONFINITE ||
                      q.status == RW_ST_SYNC_LOST;
            }
            const int64_t v = (int64_t)part[(size_t)i].nx * part[(size_t)i].ny * part[(size_t)i].nz;
            st->voxel_iters[level] += v * (int64_t)(it + rit);
            st->box_voxels[level] += v;
            st->max_iters[level] = std::max(st->max_iters[level], it);
            if (bad) st->not_converged[level] += 1;
        }
        st->solved[level] += nb;
        i0 = i1;
    }
    return RW_OK;
}

template <int R>
static int run_prune(rw_ctx* ctx, hipStream_t s, const rw_params& P, const LevelGeo& L, const float* lmap,
                     const std::vector<BoxGeo>& geos, uint8_t* dflags) {
    if (geos.empty()) return RW_OK;
    const size_t gg = geos.size() * sizeof(BoxGeo);
    H_HIP(grow(ctx, &ctx->hgeo, &ctx->hgeo_bytes, gg, s), "allocating box geometry");
    H_TRY(upload(ctx, ctx->hgeo, geos, s));
    hipLaunchKernelGGL(k_prune<R>, dim3((unsigned)geos.size()), dim3(kHThreads), 0, s, (const BoxGeo*)ctx->hgeo, lmap,
                       L.D[0], L.D[1], (float)P.t_hom, (float)P.t_bin, P.prune_hom, P.prune_dt, dflags);
    H_HIP(hipGetLastError(), "launching prune test");
    H_HIP(hipStreamSynchronize(s), "synchronising prune");
    return RW_OK;
}

template <int R>
static int segment_impl(rw_ctx* ctx, const rw_pyramid* pyr, const std::vector<rw_seed>& seeds, const rw_params& P,
                        const rw_result* prev, rw_result* res, hipStream_t s) {
    const int Lv = pyr->levels, top = Lv - 1;
    rw_run_stats& st = res->stats;
    st.levels = Lv;
    std::vector<rw_seed> newseeds;
    if (prev) {
        auto key = [](const rw_seed& a) { return std::make_tuple(a.x, a.y, a.z, a.label); };
        std::set<std::tuple<double, double, double, int>> old;
        for (const rw_seed& q : prev->seeds) old.insert(key(q));
        for (const rw_seed& q : seeds)
            if (!old.count(key(q))) newseeds.push_back(q);
    }
    std::vector<LevelGeo> LG((size_t)Lv);
    for (int l = 0; l < Lv; ++l) {
        for (int a = 0; a < 3; ++a) {
            LG[(size_t)l].D[a] = pyr->dims[l][a];
            LG[(size_t)l].nb[a] = (pyr->dims[l][a] + P.brick - 1) / P.brick;
        }
        rwk::LevelRes& lr = res->lv[l];
        for (int a = 0; a < 3; ++a) {
            lr.dims[a] = LG[(size_t)l].D[a];
            lr.nb[a] = LG[(size_t)l].nb[a];
        }
        const int64_t nvox = lr.dims[0] * lr.dims[1] * lr.dims[2];
        const int64_t nbr = lr.nb[0] * lr.nb[1] * lr.nb[2];
        st.bricks[l] = nbr;
        lr.map_bytes = (size_t)nvox * R * sizeof(float);
        lr.flags_bytes = (size_t)nbr;
        lr.host = l < P.host_levels;
        if (lr.host) H_HIP(host_alloc((void**)&lr.map, lr.map_bytes), "allocating level map in host memory");
        else H_HIP(pool_alloc(res->device, (void**)&lr.map, lr.map_bytes), "allocating level map");
        H_HIP(pool_alloc(res->device, (void**)&lr.flags, lr.flags_bytes), "allocating brick flags");
        H_HIP(hipMemsetAsync(lr.flags, 0, (size_t)nbr, s), "clearing brick flags");
    }
    auto all_bricks = [&](int l) {
        std::vector<BoxGeo> v;
        const LevelGeo& L = LG[(size_t)l];
        for (int64_t bz = 0; bz < L.nb[2]; ++bz)
            for (int64_t by = 0; by < L.nb[1]; ++by)
                for (int64_t bx = 0; bx < L.nb[0]; ++bx) v.push_back(brick_box(L, P.brick, P.expand, bx, by, bz));
        return v;
    };
    auto cfl_bricks = [&](int l, const std::map<int64_t, int>& lab, std::vector<uint8_t>& hflags) {
        const LevelGeo& L = LG[(size_t)l];
        for (const auto& kv : lab) {
            if (kv.second != -2) continue;
            const int64_t v = kv.first;
            const int64_t X = v % L.D[0], Y = (v / L.D[0]) % L.D[1], Z = v / (L.D[0] * L.D[1]);
            bricks_containing(L, P.brick, P.expand, X, Y, Z, [&](int32_t b) { hflags[(size_t)b] |= F_CFL; });
        }
    };
    // Node rule (Section IV-E): conflicts that involve a newly added label
    const bool node = prev && (P.incremental & 1);
    const float* no_warm = nullptr;
    auto warm_of = [&](int l) { return prev && (P.incremental & 2) ? (const float*)prev->lv[l].map : no_warm; };
    auto cfl_new = [&](int l, const std::map<int64_t, int>& lab) {
        const LevelGeo& L = LG[(size_t)l];
        std::vector<uint8_t> c((size_t)(L.nb[0] * L.nb[1] * L.nb[2]), 0);
        for (const auto& kv : rasterize(newseeds, l, L)) {
            auto it = lab.find(kv.first);
            if (it == lab.end() || it->second != -2) continue;
            const int64_t v = kv.first;
            const int64_t X = v % L.D[0], Y = (v / L.D[0]) % L.D[1], Z = v / (L.D[0] * L.D[1]);
            bricks_containing(L, P.brick, P.expand, X, Y, Z, [&](int32_t b) { c[(size_t)b] = 1; });
        }
        return c;
    };
    // After a node-rule level is solved and prune-tested: every solved brick
    // that the previous result also reached is compared with its previous
    // core; within t_inc and no conflict with a new label, the previous core
    // and prunable flag replace the new ones and the brick is marked kept
    // (its previous subtree is taken over level by level below).
    auto take_over = [&](int l, const std::vector<BoxGeo>& solved, const std::vector<uint8_t>& prevflags,
                         const std::vector<uint8_t>& cnew) -> int {
        const LevelGeo& L = LG[(size_t)l];
        rwk::LevelRes& lr = res->lv[l];
        const int64_t nbr = L.nb[0] * L.nb[1] * L.nb[2];
        std::vector<BoxGeo> cand;
        for (const BoxGeo& g : solved)
            if (prevflags[(size_t)g.brick] & F_REACHED) cand.push_back(g);
        if (cand.empty()) return RW_OK;
        const size_t gg = (cand.size() * sizeof(BoxGeo) + 255) & ~size_t(255);
        H_HIP(grow(ctx, &ctx->hgeo, &ctx->hgeo_bytes, gg + cand.size() * sizeof(float), s), "allocating box geometry");
        H_TRY(upload(ctx, ctx->hgeo, cand, s));
        float* dch = (float*)((char*)ctx->hgeo + gg);
        hipLaunchKernelGGL(k_core_change<R>, dim3((unsigned)cand.size()), dim3(kHThreads), 0, s,
                           (const BoxGeo*)ctx->hgeo, lr.map, prev->lv[l].map, L.D[0], L.D[1], dch);
        H_HIP(hipGetLastError(), "launching core change test");
        std::vector<float> ch(cand.size());
        std::vector<uint8_t> f((size_t)nbr);
        H_HIP(hipMemcpyAsync(ch.data(), dch, ch.size() * sizeof(float), hipMemcpyDeviceToHost, s), "reading change test");
        H_HIP(hipMemcpyAsync(f.data(), lr.flags, (size_t)nbr, hipMemcpyDeviceToHost, s), "reading flags");
        H_HIP(hipStreamSynchronize(s), "synchronising change test");
        std::vector<BoxGeo> keep;
        for (size_t i = 0; i < cand.size(); ++i) {
            const size_t b = (size_t)cand[i].brick;
            if ((double)ch[i] < P.t_inc && !cnew[b]) {
                keep.push_back(cand[i]);
                f[b] = (uint8_t)((f[b] & ~F_PRUNABLE) | (prevflags[b] & F_PRUNABLE) | F_KEPT);
            }
        }
        if (keep.empty()) return RW_OK;
        H_HIP(grow(ctx, &ctx->hgeo, &ctx->hgeo_bytes, keep.size() * sizeof(BoxGeo), s), "allocating box geometry");
        H_TRY(upload(ctx, ctx->hgeo, keep, s));
        hipLaunchKernelGGL(k_copy_core<R>, dim3((unsigned)keep.size()), dim3(kHThreads), 0, s,
                           (const BoxGeo*)ctx->hgeo, prev->lv[l].map, L.D[0], L.D[1], lr.map);
        H_HIP(hipGetLastError(), "launching take-over copy");
        H_HIP(hipMemcpyAsync(lr.flags, f.data(), (size_t)nbr, hipMemcpyHostToDevice, s), "uploading flags");
        H_HIP(hipStreamSynchronize(s), "synchronising take-over");   // f is host memory of this scope
        return RW_OK;
    };

    // ---- coarsest level: one domain, user seeds only (eq. 1)
    {
        const LevelGeo& L = LG[(size_t)top];
        rwk::LevelRes& lr = res->lv[top];
        const int64_t nbr = L.nb[0] * L.nb[1] * L.nb[2];
        auto lab = rasterize(seeds, top, L);
        std::vector<uint8_t> hflags((size_t)nbr, F_REACHED);
        cfl_bricks(top, lab, hflags);
        const bool reuse = prev && !node && newseeds.empty();
        if (reuse) {
            H_HIP(hipMemcpyAsync(lr.map, prev->lv[top].map, (size_t)(L.D[0] * L.D[1] * L.D[2]) * R * sizeof(float),
                                 hipMemcpyDeviceToDevice, s),
                  "copying previous coarsest level");
        } else {
            for (auto& f : hflags) f |= F_SOLVED;
            BoxGeo g{};
            g.nx = (int32_t)L.D[0];
            g.ny = (int32_t)L.D[1];
            g.nz = (int32_t)L.D[2];
            g.cnx = g.nx;
            g.cny = g.ny;
            g.cnz = g.nz;
            g.brick = 0;
            std::vector<BoxGeo> one{g};
            H_TRY(solve_boxes<R>(ctx, s, P, L, pyr->data[top], lr.map, nullptr, nullptr, one, lab, &st, top,
                                 warm_of(top)));
        }
        H_HIP(hipMemcpyAsync(lr.flags, hflags.data(), (size_t)nbr, hipMemcpyHostToDevice, s), "uploading flags");
        H_TRY(run_prune<R>(ctx, s, P, L, lr.map, all_bricks(top), lr.flags));
        if (node) {
            std::vector<uint8_t> pf((size_t)nbr);
            H_HIP(hipMemcpyAsync(pf.data(), prev->lv[top].flags, (size_t)nbr, hipMemcpyDeviceToHost, s),
                  "reading previous flags");
            H_HIP(hipStreamSynchronize(s), "synchronising flags");
            H_TRY(take_over(top, all_bricks(top), pf, cfl_new(top, lab)));
        }
        st.computed[top] = nbr;
    }

    // ---- finer levels (eqs. 2-3)
    for (int l = top - 1; l >= 0; --l) {
        const LevelGeo& L = LG[(size_t)l];
        const LevelGeo& PL = LG[(size_t)l + 1];
        rwk::LevelRes& lr = res->lv[l];
        const rwk::LevelRes& pr = res->lv[l + 1];
        const int64_t nbr = L.nb[0] * L.nb[1] * L.nb[2];
        if (L.D[2] > 65535) return fail(ctx, RW_E_UNSUPPORTED, "levels deeper than 65535 planes are not supported");
        hipLaunchKernelGGL(k_upsample<R>, dim3((unsigned)L.D[1], (unsigned)L.D[2]), dim3(kHThreads), 0, s, pr.map,
                           PL.D[0], PL.D[1], PL.D[2], lr.map, L.D[0], L.D[1], L.D[2]);
        H_HIP(hipGetLastError(), "launching upsample");
        std::vector<uint8_t> pflags((size_t)(PL.nb[0] * PL.nb[1] * PL.nb[2]));
        H_HIP(hipMemcpyAsync(pflags.data(), pr.flags, pflags.size(), hipMemcpyDeviceToHost, s), "reading parent flags");
        std::vector<uint8_t> prevflags;
        if (prev) {
            prevflags.resize((size_t)nbr);
            H_HIP(hipMemcpyAsync(prevflags.data(), prev->lv[l].flags, (size_t)nbr, hipMemcpyDeviceToHost, s),
                  "reading previous flags");
        }
        H_HIP(hipStreamSynchronize(s), "synchronising level");
        auto lab = rasterize(seeds, l, L);
        std::vector<uint8_t> hflags((size_t)nbr, 0);
        cfl_bricks(l, lab, hflags);
        std::vector<BoxGeo> reached;
        for (int64_t bz = 0; bz < L.nb[2]; ++bz)
            for (int64_t by = 0; by < L.nb[1]; ++by)
                for (int64_t bx = 0; bx < L.nb[0]; ++bx) {
                    const int64_t pb = bx / 2 + PL.nb[0] * (by / 2 + PL.nb[1] * (bz / 2));
                    const uint8_t f = pflags[(size_t)pb];
                    if ((f & F_REACHED) && !(f & F_PRUNABLE)) reached.push_back(brick_box(L, P.brick, P.expand, bx, by, bz));
                }
        std::vector<BoxGeo> solve, reuse;
        if (!prev) {
            solve = reached;
        } else if (node) {
            // descendants of kept nodes are taken over; every other reached brick is solved
            for (const BoxGeo& g : reached) {
                const int64_t bx = g.brick % L.nb[0], by = (g.brick / L.nb[0]) % L.nb[1], bz = g.brick / (L.nb[0] * L.nb[1]);
                const int64_t pb = bx / 2 + PL.nb[0] * (by / 2 + PL.nb[1] * (bz / 2));
                if ((pflags[(size_t)pb] & F_KEPT) && (prevflags[(size_t)g.brick] & F_REACHED)) reuse.push_back(g);
                else solve.push_back(g);
            }
        } else {
            std::vector<uint8_t> newin((size_t)nbr, 0);
            auto nl = rasterize(newseeds, l, L);
            for (const auto& kv : nl) {
                const int64_t v = kv.first;
                const int64_t X = v % L.D[0], Y = (v / L.D[0]) % L.D[1], Z = v / (L.D[0] * L.D[1]);
                bricks_containing(L, P.brick, P.expand, X, Y, Z, [&](int32_t b) { newin[(size_t)b] = 1; });
            }
            std::vector<BoxGeo> cand;
            for (const BoxGeo& g : reached) {
                if ((prevflags[(size_t)g.brick] & F_REACHED) && !newin[(size_t)g.brick]) cand.push_back(g);
                else solve.push_back(g);
            }
            if (!cand.empty()) {
                const size_t gg = (cand.size() * sizeof(BoxGeo) + 255) & ~size_t(255);
                H_HIP(grow(ctx, &ctx->hgeo, &ctx->hgeo_bytes, gg + cand.size() * sizeof(float), s),
                      "allocating box geometry");
                H_TRY(upload(ctx, ctx->hgeo, cand, s));
                float* dch = (float*)((char*)ctx->hgeo + gg);
                hipLaunchKernelGGL(k_parent_change<R>, dim3((unsigned)cand.size()), dim3(kHThreads), 0, s,
                                   (const BoxGeo*)ctx->hgeo, pr.map, prev->lv[l + 1].map, PL.D[0], PL.D[1], PL.D[2], dch);
                H_HIP(hipGetLastError(), "launching change test");
                std::vector<float> ch(cand.size());
                H_HIP(hipMemcpyAsync(ch.data(), dch, ch.size() * sizeof(float), hipMemcpyDeviceToHost, s),
                      "reading change test");
                H_HIP(hipStreamSynchronize(s), "synchronising change test");
                for (size_t i = 0; i < cand.size(); ++i) {
                    if ((double)ch[i] >= P.t_inc) solve.push_back(cand[i]);
                    else reuse.push_back(cand[i]);
                }
            }
        }
        for (const BoxGeo& g : reached) hflags[(size_t)g.brick] |= F_REACHED;
        for (const BoxGeo& g : solve) hflags[(size_t)g.brick] |= F_SOLVED;
        for (const BoxGeo& g : reuse)
            hflags[(size_t)g.brick] |= (uint8_t)((prevflags[(size_t)g.brick] & F_PRUNABLE) | (node ? F_KEPT : 0));
        H_HIP(hipMemcpyAsync(lr.flags, hflags.data(), (size_t)nbr, hipMemcpyHostToDevice, s), "uploading flags");
        H_HIP(hipStreamSynchronize(s), "synchronising flags");   // hflags is host memory of this scope
        if (!reuse.empty()) {
            H_HIP(grow(ctx, &ctx->hgeo, &ctx->hgeo_bytes, reuse.size() * sizeof(BoxGeo), s), "allocating box geometry");
            H_TRY(upload(ctx, ctx->hgeo, reuse, s));
            hipLaunchKernelGGL(k_copy_core<R>, dim3((unsigned)reuse.size()), dim3(kHThreads), 0, s,
                               (const BoxGeo*)ctx->hgeo, prev->lv[l].map, L.D[0], L.D[1], lr.map);
            H_HIP(hipGetLastError(), "launching reuse copy");
            H_HIP(hipStreamSynchronize(s), "synchronising reuse copy");
        }
        if (!solve.empty()) {
            // largest boxes first is done by the solver; keep brick order here
            H_TRY(solve_boxes<R>(ctx, s, P, L, pyr->data[l], lr.map, pr.map, PL.D, solve, lab, &st, l, warm_of(l)));
            H_TRY(run_prune<R>(ctx, s, P, L, lr.map, solve, lr.flags));
            if (node) H_TRY(take_over(l, solve, prevflags, cfl_new(l, lab)));
        }
        st.computed[l] = (int64_t)reached.size();
    }
    // prunable counts
    for (int l = 0; l < Lv; ++l) {
        std::vector<uint8_t> f((size_t)(res->lv[l].nb[0] * res->lv[l].nb[1] * res->lv[l].nb[2]));
        H_HIP(hipMemcpyAsync(f.data(), res->lv[l].flags, f.size(), hipMemcpyDeviceToHost, s), "reading flags");
        H_HIP(hipStreamSynchronize(s), "synchronising");
        for (uint8_t v : f) st.prunable[l] += (v & F_REACHED) && (v & F_PRUNABLE) ? 1 : 0;
    }
    return RW_OK;
}

}  // namespace rwk

using namespace rwk;

static void free_result_mem(rw_result* r) {
    for (int l = 0; l < RW_MAX_LEVELS; ++l) {
        if (r->lv[l].host) (void)hipHostFree(r->lv[l].map);
        else pool_release(r->device, r->lv[l].map, r->lv[l].map_bytes);
        pool_release(r->device, r->lv[l].flags, r->lv[l].flags_bytes);
        r->lv[l].map = nullptr;
        r->lv[l].flags = nullptr;
    }
}

extern "C" {

void rw_params_default(rw_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->beta = 128.0;
    p->eps = 1e-6;
    p->tol = 1e-5;
    p->expand = 1.25;
    p->t_hom = 0.3;
    p->t_bin = 0.01;
    p->t_inc = 0.01;
    p->brick = 32;
    p->max_iter = 5000;
    p->precision = RW_PREC_MIXED;
    p->n_classes = 2;
    p->prune_hom = 1;
    p->prune_dt = 1;
    p->refine_max = 1;
}

// counts = 0: normalised intensities (rw_pyramid_build); 1: square roots of
// the mean counts (rw_pyramid_build_counts).
static int pyramid_build(rw_ctx* ctx, const void* vol, int dtype, const int64_t dims[3], int levels, int counts,
                         int host_levels, rw_pyramid** out, void* stream) {
    return rwk::guarded(ctx, [&]() -> int {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    if (!out) return fail(ctx, RW_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!vol || !dims) return fail(ctx, RW_E_INVAL, "vol and dims must be non-NULL");
    if (dtype != RW_U16 && dtype != RW_F32) return fail(ctx, RW_E_INVAL, "dtype must be RW_U16 or RW_F32");
    if (levels < 1 || levels > RW_MAX_LEVELS) return fail(ctx, RW_E_INVAL, "levels must be in [1, %d]", RW_MAX_LEVELS);
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > (1 << 20)) return fail(ctx, RW_E_INVAL, "dims must be in [1, 2^20]");
    if (host_levels < 0 || host_levels >= levels)
        return fail(ctx, RW_E_INVAL, "host_levels must be in [0, levels - 1]");
    hipStream_t s = (hipStream_t)stream;
    DevGuard dg(ctx->device);
    if (!device_readable(vol))
        return fail(ctx, RW_E_INVAL, "vol must be device memory or page-locked host memory");
    rw_pyramid* p = new (std::nothrow) rw_pyramid();
    if (!p) return fail(ctx, RW_E_NOMEM, "host allocation failed");
    p->device = ctx->device;
    p->levels = levels;
    for (int l = 0; l < levels; ++l)
        for (int a = 0; a < 3; ++a) p->dims[l][a] = l == 0 ? dims[a] : (p->dims[l - 1][a] + 1) / 2;
    for (int l = 0; l < levels; ++l) {
        const int64_t n = p->dims[l][0] * p->dims[l][1] * p->dims[l][2];
        p->host[l] = l < host_levels;
        hipError_t e = p->host[l] ? host_alloc((void**)&p->data[l], (size_t)n * sizeof(float))
                                  : pool_alloc(p->device, (void**)&p->data[l], (size_t)n * sizeof(float));
        if (e != hipSuccess) {
            rw_pyramid_free(p);
            return hip_fail(ctx, e, "allocating pyramid level");
        }
    }
    const int64_t n0 = dims[0] * dims[1] * dims[2];
    const int T = 256;
    if (counts) {
        if (dtype == RW_U16)
            hipLaunchKernelGGL(k_counts_u16, dim3(grid_for(n0, T)), dim3(T), 0, s, (const uint16_t*)vol, n0,
                               p->data[0]);
        else
            hipLaunchKernelGGL(k_counts_f32, dim3(grid_for(n0, T)), dim3(T), 0, s, (const float*)vol, n0, p->data[0]);
    } else if (dtype == RW_U16) {
        unsigned init[2] = {0xffffu, 0u};
        unsigned* mm = nullptr;
        hipError_t e = pool_alloc(p->device, (void**)&mm, sizeof(init));
        if (e == hipSuccess) e = hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            const unsigned gmm = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kMinMaxBlocks, (n0 / 8 + 255) / 256));
            const int al16 = ((uintptr_t)vol & 15u) == 0 ? 1 : 0;
            hipLaunchKernelGGL(k_minmax_u16, dim3(gmm), dim3(256), 0, s, (const uint16_t*)vol, n0, al16, mm);
            hipLaunchKernelGGL(k_normalize_u16, dim3(grid_for(n0, T)), dim3(T), 0, s, (const uint16_t*)vol, n0, mm,
                               p->data[0]);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) pool_release(p->device, mm, sizeof(init));
        else if (mm) (void)hipFree(mm);
        if (e != hipSuccess) {
            rw_pyramid_free(p);
            return hip_fail(ctx, e, "normalising volume");
        }
    } else {
        hipLaunchKernelGGL(k_clip_f32, dim3(grid_for(n0, T)), dim3(T), 0, s, (const float*)vol, n0, p->data[0]);
    }
    for (int l = 1; l < levels; ++l) {
        const int64_t n = p->dims[l][0] * p->dims[l][1] * p->dims[l][2];
        hipLaunchKernelGGL(k_downsample, dim3(grid_for(n, T)), dim3(T), 0, s, p->data[l - 1], p->dims[l - 1][0],
                           p->dims[l - 1][1], p->dims[l - 1][2], p->data[l], p->dims[l][0], p->dims[l][1], p->dims[l][2]);
    }
    if (counts)
        for (int l = 0; l < levels; ++l) {
            const int64_t n = p->dims[l][0] * p->dims[l][1] * p->dims[l][2];
            hipLaunchKernelGGL(k_sqrt_inplace, dim3(grid_for(n, T)), dim3(T), 0, s, p->data[l], n);
        }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        rw_pyramid_free(p);
        return hip_fail(ctx, e, "building pyramid");
    }
    *out = p;
    return RW_OK;
    });
}

int rw_pyramid_build(rw_ctx* ctx, const void* vol, int dtype, const int64_t dims[3], int levels, rw_pyramid** out,
                     void* stream) {
    return pyramid_build(ctx, vol, dtype, dims, levels, 0, 0, out, stream);
}

int rw_pyramid_build_host(rw_ctx* ctx, const void* vol, int dtype, const int64_t dims[3], int levels,
                          int host_levels, rw_pyramid** out, void* stream) {
    return pyramid_build(ctx, vol, dtype, dims, levels, 0, host_levels, out, stream);
}

int rw_pyramid_build_counts(rw_ctx* ctx, const void* vol, int dtype, const int64_t dims[3], int levels,
                            rw_pyramid** out, void* stream) {
    return pyramid_build(ctx, vol, dtype, dims, levels, 1, 0, out, stream);
}

void rw_pyramid_free(rw_pyramid* p) {
    if (!p) return;
    DevGuard dg(p->device);
    (void)hipDeviceSynchronize();
    for (int l = 0; l < p->levels; ++l) {
        if (p->host[l]) (void)hipHostFree(p->data[l]);
        else pool_release(p->device, p->data[l], (size_t)(p->dims[l][0] * p->dims[l][1] * p->dims[l][2]) * sizeof(float));
    }
    delete p;
}

int rw_pyramid_level(const rw_pyramid* p, int level, int64_t dims[3], const float** data) {
    if (!p || level < 0 || level >= p->levels) return fail(nullptr, RW_E_INVAL, "bad pyramid or level");
    if (dims)
        for (int a = 0; a < 3; ++a) dims[a] = p->dims[level][a];
    if (data) *data = p->data[level];
    return RW_OK;
}

int rw_segment(rw_ctx* ctx, const rw_pyramid* pyr, const rw_seed* seeds, int64_t n_seeds, const rw_params* params,
               const rw_result* prev, rw_result** out, void* stream) {
    return rwk::guarded(ctx, [&]() -> int {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    if (!out) return fail(ctx, RW_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!pyr || !params) return fail(ctx, RW_E_INVAL, "pyramid and params must be non-NULL");
    if (n_seeds < 0 || (n_seeds > 0 && !seeds)) return fail(ctx, RW_E_INVAL, "bad seed array");
    const rw_params& P = *params;
    if (P.n_classes < 2 || P.n_classes > 4) return fail(ctx, RW_E_INVAL, "n_classes must be in [2, 4]");
    if (P.brick < 2 || P.brick > 1024) return fail(ctx, RW_E_INVAL, "brick must be in [2, 1024]");
    if (!(P.expand >= 1.0) || P.expand > 4.0) return fail(ctx, RW_E_INVAL, "expand must be in [1, 4]");
    if (!(P.t_hom >= 0) || !(P.t_bin >= 0) || !(P.t_inc >= 0)) return fail(ctx, RW_E_INVAL, "thresholds must be >= 0");
    if (P.incremental < 0 || P.incremental > 3) return fail(ctx, RW_E_INVAL, "incremental must be in 0..3");
    if (P.schedule < 0 || P.schedule > RW_SCHED_TUNED) return fail(ctx, RW_E_INVAL, "schedule must be in 0..5");
    if (P.joint_classes != 0 && P.joint_classes != 1) return fail(ctx, RW_E_INVAL, "joint_classes must be 0 or 1");
    if (P.host_levels < 0 || P.host_levels >= pyr->levels)
        return fail(ctx, RW_E_INVAL, "host_levels must be in [0, levels - 1]");
    for (int64_t i = 0; i < n_seeds; ++i) {
        const rw_seed& q = seeds[i];
        if (!std::isfinite(q.x) || !std::isfinite(q.y) || !std::isfinite(q.z))
            return fail(ctx, RW_E_INVAL, "seed %lld has a non-finite coordinate", (long long)i);
        if (q.label < 0 || q.label >= P.n_classes)
            return fail(ctx, RW_E_INVAL, "seed %lld: label %d outside [0, %d)", (long long)i, q.label, P.n_classes);
    }
    if (prev) {
        if (prev->levels != pyr->levels || prev->R != P.n_classes - 1 || prev->params.brick != P.brick ||
            prev->params.expand != P.expand)
            return fail(ctx, RW_E_INVAL, "prev was computed with a different pyramid or brick layout");
        for (int l = 0; l < pyr->levels; ++l)
            for (int a = 0; a < 3; ++a)
                if (prev->lv[l].dims[a] != pyr->dims[l][a]) return fail(ctx, RW_E_INVAL, "prev dims differ");
    }
    rw_result* r = new (std::nothrow) rw_result();
    if (!r) return fail(ctx, RW_E_NOMEM, "host allocation failed");
    r->device = ctx->device;
    r->params = P;
    r->levels = pyr->levels;
    r->R = P.n_classes - 1;
    try {
        r->seeds.assign(seeds, seeds + n_seeds);
    } catch (...) {
        delete r;
        throw;
    }
    hipStream_t s = (hipStream_t)stream;
    DevGuard dg(ctx->device);
    const int rc = rwk::guarded(ctx, [&]() -> int {
        switch (r->R) {
            case 1: return segment_impl<1>(ctx, pyr, r->seeds, P, prev, r, s);
            case 2: return segment_impl<2>(ctx, pyr, r->seeds, P, prev, r, s);
            case 3: return segment_impl<3>(ctx, pyr, r->seeds, P, prev, r, s);
        }
        return RW_OK;
    });
    if (rc != RW_OK) {
        (void)hipStreamSynchronize(s);
        free_result_mem(r);
        delete r;
        return rc;
    }
    *out = r;
    return RW_OK;
    });
}

void rw_result_free(rw_result* r) {
    if (!r) return;
    DevGuard dg(r->device);
    (void)hipDeviceSynchronize();
    free_result_mem(r);
    delete r;
}

int rw_result_stats(const rw_result* r, rw_run_stats* out) {
    if (!r || !out) return fail(nullptr, RW_E_INVAL, "result and out must be non-NULL");
    *out = r->stats;
    return RW_OK;
}

int rw_result_level(const rw_result* r, int level, int64_t dims[3], int* nrhs, const float** map) {
    if (!r || level < 0 || level >= r->levels) return fail(nullptr, RW_E_INVAL, "bad result or level");
    if (dims)
        for (int a = 0; a < 3; ++a) dims[a] = r->lv[level].dims[a];
    if (nrhs) *nrhs = r->R;
    if (map) *map = r->lv[level].map;
    return RW_OK;
}

int rw_result_flags(const rw_result* r, int level, int64_t nb[3], const uint8_t** flags) {
    if (!r || level < 0 || level >= r->levels) return fail(nullptr, RW_E_INVAL, "bad result or level");
    if (nb)
        for (int a = 0; a < 3; ++a) nb[a] = r->lv[level].nb[a];
    if (flags) *flags = r->lv[level].flags;
    return RW_OK;
}

static int copy_out(rw_ctx* ctx, void* dst, const void* src, size_t bytes, void* stream, int device) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    if (!dst) return fail(ctx, RW_E_INVAL, "dst is NULL");
    DevGuard dg(device);
    // (the source may be a level in page-locked host memory)
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, (hipStream_t)stream);
    return e == hipSuccess ? RW_OK : hip_fail(ctx, e, "copying out");
}

int rw_result_copy_level(rw_ctx* ctx, const rw_result* r, int level, float* dst, void* stream) {
    if (!r || level < 0 || level >= r->levels) return fail(ctx, RW_E_INVAL, "bad result or level");
    const int64_t n = r->lv[level].dims[0] * r->lv[level].dims[1] * r->lv[level].dims[2];
    return copy_out(ctx, dst, r->lv[level].map, (size_t)n * r->R * sizeof(float), stream, r->device);
}

int rw_result_copy_flags(rw_ctx* ctx, const rw_result* r, int level, uint8_t* dst, void* stream) {
    if (!r || level < 0 || level >= r->levels) return fail(ctx, RW_E_INVAL, "bad result or level");
    const int64_t n = r->lv[level].nb[0] * r->lv[level].nb[1] * r->lv[level].nb[2];
    return copy_out(ctx, dst, r->lv[level].flags, (size_t)n, stream, r->device);
}

int rw_pyramid_copy_level(rw_ctx* ctx, const rw_pyramid* p, int level, float* dst, void* stream) {
    if (!p || level < 0 || level >= p->levels) return fail(ctx, RW_E_INVAL, "bad pyramid or level");
    const int64_t n = p->dims[level][0] * p->dims[level][1] * p->dims[level][2];
    return copy_out(ctx, dst, p->data[level], (size_t)n * sizeof(float), stream, p->device);
}

int rw_result_materialize(rw_ctx* ctx, const rw_result* r, int level, int cls, float* prob, uint8_t* labels,
                          void* stream) {
    if (!ctx) return fail(nullptr, RW_E_INVAL, "ctx is NULL");
    ctx->err.clear();
    if (!r || level < 0 || level >= r->levels) return fail(ctx, RW_E_INVAL, "bad result or level");
    if (cls < 0 || cls > r->R) return fail(ctx, RW_E_INVAL, "class %d outside [0, %d]", cls, r->R);
    const int64_t n = r->lv[level].dims[0] * r->lv[level].dims[1] * r->lv[level].dims[2];
    hipStream_t s = (hipStream_t)stream;
    DevGuard dg(ctx->device);
    const int T = 256;
    switch (r->R) {
        case 1: hipLaunchKernelGGL(k_materialize<1>, dim3(grid_for(n, T)), dim3(T), 0, s, r->lv[level].map, n, cls, prob, labels); break;
        case 2: hipLaunchKernelGGL(k_materialize<2>, dim3(grid_for(n, T)), dim3(T), 0, s, r->lv[level].map, n, cls, prob, labels); break;
        case 3: hipLaunchKernelGGL(k_materialize<3>, dim3(grid_for(n, T)), dim3(T), 0, s, r->lv[level].map, n, cls, prob, labels); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RW_OK : hip_fail(ctx, e, "launching materialize");
}

}  // extern "C"
