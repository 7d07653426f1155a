// Time transform of Algorithm 1 as a GEMM on the matrix cores:
//   Y[k][s] = sum_t V[k][t] X[t][s],  k, t < N_t,  s < M (all spatial nodes).
// V (DCT-VIII or DST-I) is symmetric and orthogonal, so the same kernel applies
// V and V^{-1} = V. Optional epilogue: per-block partials of r.Y and q.Y for
// the PCG scalars (summed by the kernels that consume them).
#pragma once

#include "batch_args.h"
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

// The forward pass of the mixed-precision preconditioner fused: the time GEMM
// of r (N_t <= 128) and the forward row transforms along axis 1 of length 256,
// written to the float32 intermediate; one block per axis-0 row (all time
// slices and all 256 nodes), the output staged through LDS. It computes the
// bits of the separate kernels (the same operand scaling groups, row pairs and
// transform arithmetic). Whether the plan can take it:
bool fused_fwd_ok(const Plan& P);
// Whether a PCG iteration can also run its update in the fused forward pass.
bool fused_upd_ok(const Plan& P);

// The inverse pass fused (row transforms along axis 1 of length 256, then the
// inverse time GEMM with its dot products, N_t <= 128, one 16-node tile per
// wave): reads the intermediate ra.data, writes z and the r.z (z.q) partials
// exactly as the separate kernels. Returns the number of partials.
bool fused_inv_ok(const Plan& P);
int launch_rows_tgemm_inv(const Plan& P, int mode, const RowsArgs<float>& ra, double* z,
                          int dotmode, const double* r, const double* q, hipStream_t s);
// ua: also apply the conjugate gradient update first (r is then ua->r, and the
// kernel leaves the r.r stopping test to a later launch); nullptr: none.
void launch_tgemm_rows_fwd(const Plan& P, int mode, const double* r, float* tmp,
                           const RowsArgs<float>& ra, const UpdArgs* ua, hipStream_t s);

}  // namespace mfg
