// Time transform of Algorithm 1 as a GEMM on the matrix cores:
//   Y[k][s] = sum_t V[k][t] X[t][s],  k, t < N_t,  s < M (all spatial nodes).
// V (DCT-VIII or DST-I) is symmetric and orthogonal, so the same kernel applies
// V and V^{-1} = V. Optional epilogue: per-block partials of r.Y and q.Y for
// the PCG scalars (summed by the kernels that consume them).
#pragma once

#include "device_util.h"
#include "plan.h"

namespace mfg {

enum DotMode { DOT_NONE = 0, DOT_INIT = 1, DOT_STD = 2, DOT_FLEX = 3 };

// Precision of the matrix-core products.
enum GemmMode { GM_F64 = 0, GM_F32 = 1, GM_F16 = 2, GM_BF16 = 3 };

// X (float64 or float32) -> Y (float64 or float32).
// `name` labels the launch for the profiler (a string literal).
template <typename TX, typename TY>
void tgemm(const Plan& P, int mode, const TX* X, TY* Y, int dotmode, const double* r,
           const double* q, hipStream_t s, const char* name);

}  // namespace mfg
