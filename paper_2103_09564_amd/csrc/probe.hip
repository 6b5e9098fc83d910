// Memory-system probes: the ceilings the solve kernels are measured against.
//
// These are not steps of the method.  They measure, on the device at hand,
// what a plain stream of 16-byte loads (and a plain copy) reaches from HBM
// and, for a buffer small enough to stay in the last-level (Infinity) cache,
// from that cache, so that a kernel's bytes per second can be set against a
// measured ceiling as well as the vendor figure.

#include "common.h"

namespace rwk {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;   // the copy's loads in flight per thread

// Each thread reads float4 elements i = t + k * T (T = all threads of the
// grid), U of them with their loads issued together, `passes` times over
// the buffer; per workgroup one float (the sum, so the loads stay live) goes
// to part[blockIdx.x].
template <int U>
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const float4* __restrict__ src, int64_t n4, int passes,
                                                            float* __restrict__ part) {
    __shared__ float red[kProbeThreads / 64];
    const int64_t T = (int64_t)gridDim.x * kProbeThreads;
    const int64_t t0 = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    float acc = 0.0f;
    for (int pass = 0; pass < passes; ++pass) {
        int64_t i = t0;
        for (; i + (U - 1) * T < n4; i += U * T) {
            float4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = src[i + u * T];
#pragma unroll
            for (int u = 0; u < U; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
        }
        for (; i < n4; i += T) {
            const float4 v = src[i];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < kProbeThreads / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(float4* __restrict__ dst, const float4* __restrict__ src,
                                                            int64_t n4) {
    const int64_t T = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + (kProbeUnroll - 1) * T < n4; i += kProbeUnroll * T) {
        float4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) v[u] = src[i + u * T];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) dst[i + u * T] = v[u];
    }
    for (; i < n4; i += T) dst[i] = src[i];
}

}  // namespace

hipError_t launch_probe_read(const void* src, int64_t bytes, int passes, int unroll, float* part, hipStream_t s) {
    const int64_t n4 = bytes / 16;
    if (unroll == 4)
        hipLaunchKernelGGL(k_probe_read<4>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, (const float4*)src, n4,
                           passes, part);
    else if (unroll == 8)
        hipLaunchKernelGGL(k_probe_read<8>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, (const float4*)src, n4,
                           passes, part);
    else if (unroll == 16)
        hipLaunchKernelGGL(k_probe_read<16>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, (const float4*)src, n4,
                           passes, part);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_probe_copy(void* dst, const void* src, int64_t bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_copy, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, (float4*)dst, (const float4*)src,
                       bytes / 16);
    return hipGetLastError();
}

}  // namespace rwk
