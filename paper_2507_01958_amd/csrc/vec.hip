// Vector kernels of the (flexible) preconditioned conjugate gradient method
// (Sections 3-4) with device-resident scalars and deterministic two-stage
// reductions, and the initial Chambolle-Pock point.
#include "device_util.h"
#include "plan.h"

namespace mfg {

namespace {

constexpr int kThreads = 256;

int grid_for(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > kStreamGrid) b = kStreamGrid;
  return (int)b;
}

// x = 0, r = b; partial b.b.
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
  reduce_store<1>(acc, rb, T_BB);
}

// x += alpha p; r -= alpha q; partial r.r.
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
  reduce_store<1>(acc, rb, T_RR);
}

// partials of ||b - Ax||^2 and ||b||^2.
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
  reduce_store<2>(acc, rb, T_AUX);
}

// Sum the partials of one site in block order (single block) and apply `op`.
__global__ __launch_bounds__(256) void k_finish(RedBuf rb, int site, int nblocks, int op) {
  __shared__ double sh[2 * 16];
  const double* part = rb.partials + (size_t)site * kSlotsPerSite * rb.max_blocks;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    v[0] += part[b];
    v[1] += part[(size_t)rb.max_blocks + b];
  }
  block_sum<2>(v, sh);
  if (threadIdx.x != 0) return;
  double* S = rb.scal;
  const double a = v[0], c = v[1];
  switch (op) {
    case OP_BB:
      S[S_BB] = a;
      S[S_RR] = a;
      S[S_BAD] = finite_d(a) ? 0.0 : 2.0;
      S[S_DONE] = (a == 0.0) ? 1.0 : 0.0;
      break;
    case OP_PQ:
      S[S_PQ] = a;
      if (!finite_d(a)) {
        S[S_BAD] = 2.0;
        S[S_ALPHA] = 0.0;
      } else if (!(a > 0.0)) {
        S[S_BAD] = 1.0;
        S[S_ALPHA] = 0.0;
      } else {
        S[S_ALPHA] = S[S_RHO] / a;
      }
      break;
    case OP_RR:
      S[S_RR] = a;
      if (!finite_d(a)) S[S_BAD] = 2.0;
      if (a <= S[S_TOL2] * S[S_BB]) S[S_DONE] = 1.0;
      break;
    case OP_RZ_INIT:
    case OP_RZ_STD:
    case OP_RZ_FLEX:
      if (!finite_d(a) || !finite_d(c)) {
        S[S_BAD] = 2.0;
      } else if (!(a > 0.0)) {
        S[S_BAD] = 1.0;
      } else if (op == OP_RZ_INIT) {
        S[S_RHO] = a;
        S[S_BETA] = 0.0;
      } else {
        const double rho = S[S_RHO];
        S[S_BETA] = (op == OP_RZ_FLEX) ? -S[S_ALPHA] * c / rho : a / rho;
        S[S_RHO] = a;
      }
      break;
    case OP_DM:
      S[S_DM] = a;
      break;
    case OP_AUX:
      S[S_AUX0] = a;
      S[S_AUX1] = c;
      break;
    default:
      break;
  }
}

__global__ __launch_bounds__(kThreads) void k_fill(double* __restrict__ x, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ __launch_bounds__(64) void k_set_scalars(double* scal, double tol2) {
  if (threadIdx.x == 0) {
    scal[S_TOL2] = tol2;
    scal[S_BAD] = 0.0;
    scal[S_DONE] = 0.0;
  }
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

void launch_finish(const Plan& P, int site, int nblocks, int op, hipStream_t s) {
  ProfScope ps(P, "finish", s);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, P.red, site, nblocks, op);
}

void launch_pcg_init(const Plan& P, const double* b, double* x, double* r, double rtol,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, P.red.scal, rtol * rtol);
  const int grid = grid_for(P.g.n);
  {
    ProfScope ps(P, "pcg_init", s);
    hipLaunchKernelGGL(k_pcg_init, dim3(grid), dim3(kThreads), 0, s, P.g.n, b, x, r, P.red);
  }
  launch_finish(P, T_BB, grid, OP_BB, s);
}

void launch_update(const Plan& P, double* x, double* r, const double* p, const double* q,
                   hipStream_t s) {
  const int grid = grid_for(P.g.n);
  {
    ProfScope ps(P, "update", s);
    hipLaunchKernelGGL(k_update, dim3(grid), dim3(kThreads), 0, s, P.g.n, x, r, p, q, P.red);
  }
  launch_finish(P, T_RR, grid, OP_RR, s);
}

void launch_residual(const Plan& P, const double* b, const double* Ax, hipStream_t s) {
  const int grid = grid_for(P.g.n);
  {
    ProfScope ps(P, "residual", s);
    hipLaunchKernelGGL(k_residual, dim3(grid), dim3(kThreads), 0, s, P.g.n, b, Ax, P.red);
  }
  launch_finish(P, T_AUX, grid, OP_AUX, s);
}

void launch_fill(double* x, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, x, n, v);
}

void launch_cp_init(const Plan& P, double* xi, double* y, double* ybar, hipStream_t s) {
  ProfScope ps(P, "cp_init", s);
  hipLaunchKernelGGL(k_cp_init, dim3(grid_for(P.g.n * (1 + P.g.ncomp))), dim3(kThreads), 0, s,
                     P.g, (const double*)P.m0, xi, y, ybar);
}

}  // namespace mfg
