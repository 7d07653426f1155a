// Reverse sweep of the Chambolle-Pock iteration (mfg_cp_adjoint).
//
// Forward step l (Section 3, eq. pasosChamPock; sigma, tau, theta from the
// Section 5 schedule):
//   z = xi + sigma ybar;  b = Cr z - sigma dr(m0);  u = A^{-1} b;  xi' = Cr^T u;
//   v = y - tau xi';  y' = prox(v; V);  ybar' = y' + theta (y' - y).
// Reverse step, given the adjoints (g_xi', g_y', g_ybar') of the new state:
//   g_y' += (1 + theta) g_ybar';  g_v = J_prox^T g_y';  g_V += J_{prox,V}^T g_y';
//   g_y = -theta g_ybar' + g_v;   g_xi' -= tau g_v;
//   g_u = Cr g_xi';  g_b = A^{-1} g_u (A symmetric: the same PCG);
//   g_z = Cr^T g_b;  g_m0 -= (sigma/dt) g_b[slice 0];  g_xi = g_z;  g_ybar = sigma g_z;
// and the initial point y_0 = ybar_0 = (m0 at every slice, w = 0) adds the
// m-parts of g_y_0 + g_ybar_0, summed over slices, to g_m0.
//
// Prox Jacobian (implicit function theorem on h'(m) = 0, active branch m > 0,
// s = m + tau, a = |w~|^2, g = a/s^3 + 2 c2 m + c1 + 1/tau with the cell's
// coupling coefficients, the terminal cost included on the last slice):
//   dm/dmbar = 1/(tau g), dm/dV = -1/g, dm/dwbar_c = chi_c w~_c/(s^2 g),
//   dw_c = (tau/s^2) w~_c dm + (m/s) chi_c dwbar_c   (chi_c: wbar_c strictly
//   inside its half-line); zero on the inactive branch.
#include "device_util.h"
#include "plan.h"
#include "prox_cell.h"

namespace mfg {

namespace {

constexpr int kThreads = 256;

int grid_for(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (int)b;
}

// The root m is recomputed with the forward prox's own code (prox_cell.h), so
// it is reproduced exactly.

// Fused reverse of extrapolation + prox + (v = y - tau xi') for one step.
// In place: gy <- g_y (previous iterate), gxi <- g_xi' - tau g_v. gVc[p] is the
// cell's contribution to g_V (summed over slices by k_sum_slices).
__global__ __launch_bounds__(kThreads) void k_adj_prox(Geom g, double* __restrict__ gy,
                                                       const double* __restrict__ gyb,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ Vpot,
                                                       const double* __restrict__ VT,
                                                       double tau, double theta,
                                                       double* __restrict__ gxi,
                                                       double* __restrict__ gVc) {
  const long long n = g.n;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int rem = (int)((unsigned)p % (unsigned)g.M);  // n < 2^31
    const bool lastslice = (unsigned)p >= (unsigned)(g.nt - 1) * (unsigned)g.M;
    const double c1 = lastslice ? g.c1T : g.c1;
    double wb[4], wt[4], gyn[5], gv[5];
    double a = 0.0;
    for (int c = 0; c < g.ncomp; ++c) {
      const double x = v[(size_t)(c + 1) * n + p];
      wb[c] = x;
      wt[c] = (c & 1) ? fmin(x, 0.0) : fmax(x, 0.0);
      a += wt[c] * wt[c];
    }
    const double m = prox_root(v[p], a, lastslice ? VT[rem] : Vpot[rem], tau, c1, g.c2);
    for (int c = 0; c <= g.ncomp; ++c) {
      const size_t o = (size_t)c * n + p;
      gyn[c] = gy[o] + (1.0 + theta) * gyb[o];
    }
    double gV = 0.0;
    if (m > 0.0) {
      const double s = m + tau;
      const double gpp = a / (s * s * s) + 2.0 * g.c2 * m + c1 + 1.0 / tau;
      double gm_tot = gyn[0];
      for (int c = 0; c < g.ncomp; ++c) gm_tot += gyn[1 + c] * (tau / (s * s)) * wt[c];
      gv[0] = gm_tot / (tau * gpp);
      gV = -gm_tot / gpp;
      for (int c = 0; c < g.ncomp; ++c) {
        const bool inside = (c & 1) ? (wb[c] < 0.0) : (wb[c] > 0.0);
        gv[1 + c] = inside ? gm_tot * wt[c] / (s * s * gpp) + gyn[1 + c] * (m / s) : 0.0;
      }
    } else {
      for (int c = 0; c <= g.ncomp; ++c) gv[c] = 0.0;
    }
    for (int c = 0; c <= g.ncomp; ++c) {
      const size_t o = (size_t)c * n + p;
      gy[o] = -theta * gyb[o] + gv[c];
      gxi[o] -= tau * gv[c];
    }
    gVc[p] = gV;
  }
}

// out[s] += sum_t in[t * M + s] (one thread per node: a fixed summation order).
__global__ __launch_bounds__(kThreads) void k_sum_slices(int M, int nt,
                                                         const double* __restrict__ in,
                                                         const double* __restrict__ in2,
                                                         double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= M) return;
  double acc = 0.0;
  for (int t = 0; t < nt; ++t) {
    acc += in[(size_t)t * M + s];
    if (in2) acc += in2[(size_t)t * M + s];
  }
  out[s] += acc;
}

// y[i] = a x[i] + b y[i] over n entries.
__global__ __launch_bounds__(kThreads) void k_axpby(long long n, double a,
                                                    const double* __restrict__ x, double b,
                                                    double* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

}  // namespace

void launch_adj_prox(const Plan& P, double* gy, const double* gyb, const double* v, double tau,
                     double theta, double* gxi, double* gVc, hipStream_t s) {
  ProfScope ps(P, "adj_prox", s);
  hipLaunchKernelGGL(k_adj_prox, dim3(grid_for(P.g.n)), dim3(kThreads), 0, s, P.g, gy, gyb, v,
                     (const double*)P.V, (const double*)P.VT, tau, theta, gxi, gVc);
}

void launch_sum_slices(const Plan& P, const double* in, const double* in2, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_sum_slices, dim3((P.g.M + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     P.g.M, P.g.nt, in, in2, out);
}

void launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kThreads), 0, s, n, a, x, b, y);
}

}  // namespace mfg
