// Vector kernels of the (flexible) preconditioned conjugate gradient method
// (Sections 3-4) with device-resident scalars and deterministic two-stage
// reductions, and the initial Chambolle-Pock point.
//
// Each kernel body is a device function of (arguments, block id, block count):
// the single-instance kernels call it with blockIdx/gridDim, the batched
// kernels (batch.hip) with the block's place inside its instance.
#include "batch_args.h"
#include "device_util.h"
#include "pcg_update.h"
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

}  // namespace

// r = b (the residual of x = 0, which the first update writes); partial b.b;
// block 0 resets the PCG status.
__device__ void pcg_init_body(const InitArgs& a, int bid, int nb) {
  if (bid == 0 && threadIdx.x == 0) {
    double* S = a.rb.scal;
    S[S_TOL2] = a.tol2;
    S[S_BAD] = 0.0;
    S[S_DONE] = 0.0;
    S[S_ITS] = 0.0;
  }
  double acc[1] = {0.0};
  for (long long i = (long long)bid * blockDim.x + threadIdx.x; i < a.n;
       i += (long long)nb * blockDim.x) {
    const double v = a.b[i];
    a.r[i] = v;
    acc[0] += v * v;
  }
  reduce_store<1>(acc, a.rb, T_BB, bid);
}

// x += alpha p; r -= alpha q (alpha: pcg_alpha); partial r.r. Skipped once
// the solve is done.
__device__ void update_body(const UpdArgs& a, int bid, int nb) {
  if (a.done && *a.done != 0.0) return;
  const double alpha = pcg_alpha(a, bid);
  double acc[1] = {0.0};
  // explicit fused multiply-adds, so the operations do not depend on the
  // compiler's contraction choices in this kernel; the first update of a solve
  // (x = 0) writes x without reading it
  // (x, r, p, q are distinct buffers: every load of an element is issued
  // before its stores)
  double* __restrict__ x = a.x;
  double* __restrict__ r = a.r;
  const double* __restrict__ p = a.p;
  const double* __restrict__ q = a.q;
  const long long i0 = (long long)bid * blockDim.x + threadIdx.x, di = (long long)nb * blockDim.x;
  if (a.first) {
    for (long long i = i0; i < a.n; i += di) {
      const double pv = p[i], qv = q[i], rv = r[i];
      x[i] = alpha * pv;
      const double ri = __builtin_fma(-alpha, qv, rv);
      r[i] = ri;
      acc[0] += ri * ri;
    }
  } else {
    for (long long i = i0; i < a.n; i += di) {
      const double pv = p[i], qv = q[i], rv = r[i], xv = x[i];
      x[i] = __builtin_fma(alpha, pv, xv);
      const double ri = __builtin_fma(-alpha, qv, rv);
      r[i] = ri;
      acc[0] += ri * ri;
    }
  }
  reduce_store<1>(acc, a.rb, T_RR, bid);
}

// Sum the partials of one site (one block of kFinishThreads) and apply `op`.
// Thread t adds entries t, t + T, t + 2T, ... in order (T threads); the loads
// are issued kFinishDepth at a time so that a site of 32768 partials takes two
// rounds of memory latency rather than one per entry. Only OP_AUX reads the
// second slot.
__device__ void finish_body(const FinishArgs& f) {
  const RedBuf& rb = f.rb;
  if (f.done && *f.done != 0.0) return;
  __shared__ double sh[2 * 16];
  const double* part = rb.partials + (size_t)f.site * kSlotsPerSite * rb.max_blocks;
  const int nslot = (f.op == OP_AUX) ? 2 : 1;
  const int T = blockDim.x;
  double v[2] = {0.0, 0.0};
  for (int k = 0; k < nslot; ++k) {
    const double* pk = part + (size_t)k * rb.max_blocks;
    double acc = 0.0;
    for (int b0 = threadIdx.x; b0 < f.nblocks; b0 += T * kFinishDepth) {
      double t[kFinishDepth];
#pragma unroll
      for (int u = 0; u < kFinishDepth; ++u) {
        const int b = b0 + u * T;
        t[u] = (b < f.nblocks) ? pk[b] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kFinishDepth; ++u) acc += t[u];
    }
    v[k] = acc;
  }
  block_sum<2>(v, sh);
  if (threadIdx.x != 0) return;
  double* S = rb.scal;
  const double a = v[0], c = v[1];
  switch (f.op) {
    case OP_BB:
      S[S_BB] = a;
      S[S_RR] = a;
      S[S_BAD] = finite_d(a) ? 0.0 : 2.0;
      S[S_DONE] = (a == 0.0) ? 1.0 : 0.0;
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

namespace {

__global__ __launch_bounds__(kThreads) void k_pcg_init(InitArgs a) {
  pcg_init_body(a, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kThreads) void k_update(UpdArgs a) {
  update_body(a, blockIdx.x, gridDim.x);
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
  reduce_store<2>(acc, rb, T_AUX, blockIdx.x);
}

__global__ __launch_bounds__(kFinishThreads) void k_finish(FinishArgs f) { finish_body(f); }

__global__ __launch_bounds__(kThreads) void k_fill(double* __restrict__ x, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

// Per-slice sums of the m block of y (blocks 0..N_t-1) and of m0 (block N_t),
// each in a fixed order.
__global__ __launch_bounds__(kThreads) void k_slice_mass(Geom g, const double* __restrict__ y,
                                                         const double* __restrict__ m0,
                                                         double* __restrict__ sums) {
  const int b = blockIdx.x;
  const double* src = (b < g.nt) ? y + (size_t)b * g.M : m0;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < g.M; i += blockDim.x) v[0] += src[i];
  __shared__ double sh[16];
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) sums[b] = v[0];
}

// max_t |sums[t] - sums[N_t]| * hd (hd = h^d, the cell measure).
__global__ __launch_bounds__(kThreads) void k_mass_drift(int nt, const double* __restrict__ sums,
                                                         double hd, double* __restrict__ out) {
  double mx = 0.0;
  for (int t = threadIdx.x; t < nt; t += blockDim.x) mx = fmax(mx, fabs(sums[t] - sums[nt]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  __shared__ double sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, sh[w]);
    *out = mx * hd;
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

FinishArgs finish_args(const Plan& P, int site, int nblocks, int op) {
  FinishArgs f;
  f.rb = P.red;
  f.site = site;
  f.nblocks = nblocks;
  f.op = op;
  f.done = P.pcg_done;
  return f;
}

void launch_finish(const Plan& P, int site, int nblocks, int op, hipStream_t s) {
  ProfScope ps(P, "finish", s);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishThreads), 0, s,
                     finish_args(P, site, nblocks, op));
}

InitArgs pcg_init_args(const Plan& P, const double* b, double* r, double rtol) {
  return InitArgs{P.g.n, b, r, P.red, rtol * rtol};
}

int pcg_init_grid(const Plan& P) { return grid_for(P.g.n); }

void launch_pcg_init(const Plan& P, const double* b, double* r, double rtol, hipStream_t s) {
  const int grid = pcg_init_grid(P);
  {
    ProfScope ps(P, "pcg_init", s);
    hipLaunchKernelGGL(k_pcg_init, dim3(grid), dim3(kThreads), 0, s,
                       pcg_init_args(P, b, r, rtol));
  }
  launch_finish(P, T_BB, grid, OP_BB, s);
}

UpdArgs update_args(const Plan& P, double* x, double* r, const double* p, const double* q,
                    bool first) {
  return UpdArgs{P.g.n, x, r, p, q, P.red, P.pcg_done, P.pq_blocks, P.rz_blocks, first ? 1 : 0};
}

int update_grid(const Plan& P) { return grid_for(P.g.n); }

void launch_update(const Plan& P, double* x, double* r, const double* p, const double* q,
                   bool first, hipStream_t s) {
  const int grid = update_grid(P);
  {
    ProfScope ps(P, "update", s);
    hipLaunchKernelGGL(k_update, dim3(grid), dim3(kThreads), 0, s,
                       update_args(P, x, r, p, q, first));
  }
  // the r.r partials are summed by the stopping test of the next
  // preconditioner application (its forward time transform)
  P.rr_blocks = grid;
}

void launch_residual(const Plan& P, const double* b, const double* Ax, hipStream_t s) {
  const int grid = grid_for(P.g.n);
  {
    ProfScope ps(P, "residual", s);
    hipLaunchKernelGGL(k_residual, dim3(grid), dim3(kThreads), 0, s, P.g.n, b, Ax, P.red);
  }
  launch_finish(P, T_AUX, grid, OP_AUX, s);
}

void launch_mass_drift(const Plan& P, const double* y, hipStream_t s) {
  const Geom& g = P.g;
  // N_t + 1 sums in the T_AUX partials (4 * max_blocks >= 4097 slots)
  double* sums = P.red.partials + (size_t)T_AUX * kSlotsPerSite * P.red.max_blocks;
  const double hd = 1.0 / (g.ih1 * (g.has0 ? g.ih0 : 1.0));
  hipLaunchKernelGGL(k_slice_mass, dim3(g.nt + 1), dim3(kThreads), 0, s, g, y,
                     (const double*)P.m0, sums);
  hipLaunchKernelGGL(k_mass_drift, dim3(1), dim3(kThreads), 0, s, g.nt, (const double*)sums, hd,
                     P.red.scal + S_MASS);
}

void launch_fill(double* x, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, x, n, v);
}

void launch_cp_init(const Plan& P, double* xi, double* y, double* ybar, hipStream_t s) {
  ProfScope ps(P, "cp_init", s);
  hipLaunchKernelGGL(k_cp_init, dim3(grid_for(P.g.n * (1 + P.g.ncomp))), dim3(kThreads), 0, s,
                     P.g, (const double*)P.m0, xi, y, ybar);
}

// ---- batched launches (args / offsets are device arrays, see batch_args.h) ----
namespace {

__global__ __launch_bounds__(kThreads) void k_update_batch(const UpdArgs* A, const int* off,
                                                           int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  update_body(A[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

// one block per instance
__global__ __launch_bounds__(kFinishThreads) void k_finish_batch(const FinishArgs* F) {
  finish_body(F[blockIdx.x]);
}

// Per instance: load the step sizes of CP iteration S_CPIT from the schedule
// table sched[(i * maxit + it) * 3 + {sigma, tau, theta}] and advance S_CPIT.
__global__ __launch_bounds__(64) void k_cp_advance_batch(double* scal, int stride, int ninst,
                                                         const double* sched, int maxit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* S = scal + (size_t)i * stride;
  int it = (int)S[S_CPIT];
  if (it >= maxit) it = maxit - 1;
  const double* e = sched + ((size_t)i * maxit + it) * 3;
  S[S_SIGMA] = e[0];
  S[S_TAU] = e[1];
  S[S_THETA] = e[2];
  S[S_CPIT] = (double)(it + 1);
}

}  // namespace

void launch_update_batch(const UpdArgs* A, const int* off, int ninst, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_update_batch, dim3(total), dim3(kThreads), 0, s, A, off, ninst);
}

void launch_finish_batch(const FinishArgs* F, int ninst, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_batch, dim3(ninst), dim3(kFinishThreads), 0, s, F);
}

void launch_cp_advance_batch(double* scal, int stride, int ninst, const double* sched, int maxit,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_cp_advance_batch, dim3((ninst + 63) / 64), dim3(64), 0, s, scal, stride,
                     ninst, sched, maxit);
}

}  // namespace mfg
