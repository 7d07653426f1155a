// Vector kernels of the (flexible) preconditioned conjugate gradient method
// (Sections 3-4) with device-resident scalars and deterministic reductions,
// and the initial Chambolle-Pock point.
#include "device_util.h"
#include "plan.h"

namespace mfg {

namespace {

constexpr int kThreads = 256;

int grid_for(long long n, int max_blocks) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

// x = 0, r = b, b.b -> S_BB; resets the status scalars.
__global__ __launch_bounds__(kThreads) void k_pcg_init(long long n, const double* __restrict__ b,
                                                       double* __restrict__ x,
                                                       double* __restrict__ r, RedBuf rb) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = b[i];
    x[i] = 0.0;
    r[i] = v;
    acc[0] += v * v;
  }
  double tot[1];
  if (reduce_commit<1>(acc, rb, T_BB, gridDim.x, tot) && threadIdx.x == 0) {
    const double bb = tot[0];
    rb.scal[S_BB] = bb;
    rb.scal[S_RR] = bb;
    rb.scal[S_BAD] = finite_d(bb) ? 0.0 : 2.0;
    rb.scal[S_DONE] = (bb == 0.0) ? 1.0 : 0.0;
  }
}

// x += alpha p; r -= alpha q; r.r -> S_RR; S_DONE when r.r <= rtol^2 b.b.
__global__ __launch_bounds__(kThreads) void k_update(long long n, double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q, RedBuf rb) {
  const double alpha = rb.scal[S_ALPHA];
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc[0] += ri * ri;
  }
  double tot[1];
  if (reduce_commit<1>(acc, rb, T_RR, gridDim.x, tot) && threadIdx.x == 0) {
    const double rr = tot[0];
    rb.scal[S_RR] = rr;
    if (!finite_d(rr)) rb.scal[S_BAD] = 2.0;
    if (rr <= rb.scal[S_TOL2] * rb.scal[S_BB]) rb.scal[S_DONE] = 1.0;
  }
}

// ||b - Ax||^2 -> S_AUX0, ||b||^2 -> S_AUX1.
__global__ __launch_bounds__(kThreads) void k_residual(long long n, const double* __restrict__ b,
                                                       const double* __restrict__ Ax, RedBuf rb) {
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double bi = b[i];
    const double d = bi - Ax[i];
    acc[0] += d * d;
    acc[1] += bi * bi;
  }
  double tot[2];
  if (reduce_commit<2>(acc, rb, T_AUX, gridDim.x, tot) && threadIdx.x == 0) {
    rb.scal[S_AUX0] = tot[0];
    rb.scal[S_AUX1] = tot[1];
  }
}

__global__ __launch_bounds__(kThreads) void k_fill(double* __restrict__ x, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ __launch_bounds__(64) void k_set_scalar(double* scal, int slot, double v) {
  if (threadIdx.x == 0) scal[slot] = v;
}

// xi = 0; y = ybar = (m0 at every slice, w = 0).
__global__ __launch_bounds__(kThreads) void k_cp_init(Geom g, const double* __restrict__ m0,
                                                      double* __restrict__ xi,
                                                      double* __restrict__ y,
                                                      double* __restrict__ ybar) {
  const long long tot = g.n * (1 + g.ncomp);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = (i < g.n) ? m0[i % g.M] : 0.0;
    xi[i] = 0.0;
    y[i] = v;
    ybar[i] = v;
  }
}

}  // namespace

void launch_pcg_init(const Plan& P, const double* b, double* x, double* r, double rtol,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, s, P.red.scal, (int)S_TOL2, rtol * rtol);
  hipLaunchKernelGGL(k_pcg_init, dim3(grid_for(P.g.n, P.red.max_blocks)), dim3(kThreads), 0, s,
                     P.g.n, b, x, r, P.red);
}

void launch_update(const Plan& P, double* x, double* r, const double* p, const double* q,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(grid_for(P.g.n, P.red.max_blocks)), dim3(kThreads), 0, s,
                     P.g.n, x, r, p, q, P.red);
}

void launch_residual(const Plan& P, const double* b, const double* Ax, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for(P.g.n, P.red.max_blocks)), dim3(kThreads), 0, s,
                     P.g.n, b, Ax, P.red);
}

void launch_fill(double* x, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, x, n, v);
}

void launch_cp_init(const Plan& P, double* xi, double* y, double* ybar, hipStream_t s) {
  hipLaunchKernelGGL(k_cp_init, dim3(grid_for(P.g.n * (1 + P.g.ncomp), P.red.max_blocks)),
                     dim3(kThreads), 0, s, P.g, (const double*)P.m0, xi, y, ybar);
}

}  // namespace mfg
