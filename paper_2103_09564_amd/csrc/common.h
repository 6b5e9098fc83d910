// Internal declarations shared by the HIP sources of librwseg (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "rwseg.h"

namespace rwk {

// Device-side box descriptor, in launch order (largest boxes first); `slot`
// is the caller's brick index (where its stats go).
struct BrickDev {
    int32_t nx, ny, nz, slot;
    int64_t off;
};

struct SolveArgs {
    const BrickDev* bricks;
    const float* g;
    const uint8_t* mask;
    float* x;              // caller x (interleaved nrhs)
    double* x64;           // caller x64 or workspace (may be null when unused)
    void* r;               // workspace vectors, element type float or double
    void* z;
    void* p0;
    void* p1;
    void* xt;              // FP64 path: solution accumulator (double); unused otherwise
    float* dcorr;          // FP32 correction accumulator
    rw_brick_stats* stats;
    double beta, eps, tol, refine_tol, inner_tol;
    int32_t max_iter, precision, refine_max, want_x64;
};

struct AdjointArgs {
    const BrickDev* bricks;
    const float* g;
    const uint8_t* mask;
    const float* x;
    const float* dl_dx;
    float* dl_dg;
    float* lambda;         // caller buffer or workspace
    float* r;
    float* z;
    float* p0;
    float* p1;
    double* beta_part;     // [n_bricks] per-box partial of dl/dbeta, in launch order
    rw_brick_stats* stats;
    double beta, eps, tol;
    int32_t max_iter;
};

// Launchers (pcg.hip).  Return a hipError_t.
hipError_t launch_solve(const SolveArgs& a, int64_t n_bricks, int nrhs, bool fp64, hipStream_t s);
hipError_t launch_adjoint(const AdjointArgs& a, int64_t n_bricks, double* dl_dbeta, hipStream_t s);

}  // namespace rwk
