// Space-time stencils of the discrete constraint (Section 2, Section 3):
//   Cr y     (eq. ABC, first block row eliminated),
//   Cr^T u,
//   A u = Cr Cr^T u (eq. largeA),
// plus the per-cell proximal step (Section 3) and the fused
// back-projection + prox + extrapolation of one Chambolle-Pock iteration.
//
// One-axis operators, with h the spacing of the axis:
//   K:   (2u_i - u_{i+1} - u_{i-1}) / h^2     (periodic mod N; Neumann by the
//        half-sample reflection, i.e. the Section 4.3 matrix with corners 1)
//   D^1 w (even flux component):  w_i - w_{i-1}     (Neumann: w_{N-1} and w_{-1}
//        do not enter, the printed D^1 has a zero last column)
//   D^2 w (odd flux component):   w_{i+1} - w_i     (Neumann: w_0 and w_N do not
//        enter, zero first column)
//   (D^1)^T u = u_i - u_{i+1},  (D^2)^T u = u_{i-1} - u_i (both vanish across a
//        Neumann boundary under the reflection).
// B = [D^1_x, D^2_x, D^1_y, D^2_y] / h and L = nu K + I/dt (Section 3).
#include "batch_args.h"
#include "device_util.h"
#include "plan.h"
#include "prox_cell.h"

namespace mfg {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ size_t at(const Geom& g, int t, int i0, int i1) {
  return (size_t)t * g.M + (size_t)i0 * g.n1 + i1;
}

// The per-cell stencils below are specialised on the axis count (HAS0: d = 2)
// and the boundary types (BC: bit 0 set when axis 1 is Neumann, bit 1 when
// axis 0 is; periodic otherwise) so the cell loops carry no branches on them;
// *_dispatch picks the specialisation once per block.

// (K v)(i0, i1) in slice t of v.
template <bool HAS0, int BC>
__device__ __forceinline__ double Kop(const double* __restrict__ v, const Geom& g, int t, int i0,
                                      int i1) {
  const double c = v[at(g, t, i0, i1)];
  double r = (2.0 * c - v[at(g, t, i0, nbr1(i1 + 1, g.n1, BC & 1))] -
              v[at(g, t, i0, nbr1(i1 - 1, g.n1, BC & 1))]) * g.ih1sq;
  if (HAS0)
    r += (2.0 * c - v[at(g, t, nbr1(i0 + 1, g.n0, BC & 2), i1)] -
          v[at(g, t, nbr1(i0 - 1, g.n0, BC & 2), i1)]) * g.ih0sq;
  return r;
}

// (D^1 w)_i and (D^2 w)_i along one axis for the value accessor f(index).
// Neumann: the terms that do not enter are loaded from a valid index and
// dropped by a select, so no load sits behind a branch.
template <bool NEU, class F>
__device__ __forceinline__ double D1w(F f, int i, int n) {
  if (!NEU) return f(i) - f(i == 0 ? n - 1 : i - 1);
  const double a = f(i <= n - 2 ? i : n - 2), b = f(i >= 1 ? i - 1 : 0);
  return (i <= n - 2 ? a : 0.0) - (i >= 1 ? b : 0.0);
}
template <bool NEU, class F>
__device__ __forceinline__ double D2w(F f, int i, int n) {
  if (!NEU) return f(i + 1 == n ? 0 : i + 1) - f(i);
  const double a = f(i <= n - 2 ? i + 1 : n - 1), b = f(i >= 1 ? i : 0);
  return (i <= n - 2 ? a : 0.0) - (i >= 1 ? b : 0.0);
}

// Calls F<HAS0, BC>::run(args...) for the geometry's axis count and boundaries.
template <template <bool, int> class F, class... A>
__device__ __forceinline__ void geom_dispatch(const Geom& g, A&&... args) {
  if (g.has0) {
    switch (g.bcm) {
      case 0: F<true, 0>::run(args...); break;
      case 1: F<true, 1>::run(args...); break;
      case 2: F<true, 2>::run(args...); break;
      default: F<true, 3>::run(args...);
    }
  } else {
    if (g.bcm & 1) F<false, 1>::run(args...);
    else F<false, 0>::run(args...);
  }
}

// b = Cr (xi + sigma ybar) - sigma [t==0] m0/dt. With ybar == nullptr this is
// b = Cr xi (apply_C). ZM: z = xi + sigma ybar read ready-made from zin.
//
// Logical block lb owns the cells sb * 256 + threadIdx.x (+ k * nsp * 256) of
// a slice (spatial block sb = lb % nsp) and walks a chunk of a.tc slices
// (chunk lb / nsp); each thread keeps its cell's z_t of the m-component for the
// next slice's -z_{t-1}/dt term, so only the chunk's first slice reads slice
// t-1. The single-plan launch spreads logical blocks over the XCDs in
// contiguous ranges, so the blocks that read a row's neighbour rows share an L2.
constexpr int kRhsMaxSpatial = 8192;

__host__ __device__ inline int rhs_nsp(const Geom& g) {
  const int nsp = (g.M + kThreads - 1) / kThreads;
  return nsp < kRhsMaxSpatial ? nsp : kRhsMaxSpatial;
}

// One cell's column of b over slices [t0, t1).
template <bool HASBAR, bool ZM, bool HAS0, int BC>
__device__ __forceinline__ void rhs_column(const RhsArgs& a, int rem, int t0, int t1,
                                           double& acc) {
  const Geom& g = a.g;
  const double* __restrict__ xi = ZM ? a.zin : a.xi;
  const double* __restrict__ ybar = a.ybar;
  double* __restrict__ b = a.b;
  const double sigma = a.sigma_dev ? *a.sigma_dev : a.sigma;
  const long long n = g.n;
  const int i0 = rem / g.n1, i1 = rem - i0 * g.n1;
  const int row = i0 * g.n1;
  constexpr bool NEU1 = (BC & 1) != 0, NEU0 = (BC & 2) != 0;
  const int j1p = row + nbr1(i1 + 1, g.n1, NEU1), j1m = row + nbr1(i1 - 1, g.n1, NEU1);
  const int j0p = nbr1(i0 + 1, g.n0, NEU0) * g.n1 + i1, j0m = nbr1(i0 - 1, g.n0, NEU0) * g.n1 + i1;
  auto z = [&](int c, size_t idx) -> double {
    const size_t k = (size_t)c * n + idx;
    // one rounding (fma), as where z is formed by the back-projection
    return (HASBAR && !ZM) ? __builtin_fma(sigma, ybar[k], xi[k]) : xi[k];
  };
  double zprev = t0 >= 1 ? z(0, (size_t)(t0 - 1) * g.M + rem) : 0.0;
  for (int t = t0; t < t1; ++t) {
    const size_t base = (size_t)t * g.M;
    // m-part: L z_t - [t>=1] z_{t-1}/dt
    const double zc = z(0, base + rem);
    double Kz = (2.0 * zc - z(0, base + j1p) - z(0, base + j1m)) * g.ih1sq;
    if (HAS0) Kz += (2.0 * zc - z(0, base + j0p) - z(0, base + j0m)) * g.ih0sq;
    double r = g.nu * Kz + zc * g.idt;
    if (t >= 1) r -= zprev * g.idt;
    // flux part: sum_c B_c w^(c)_t
    {
      constexpr int ce = HAS0 ? 3 : 1, co = HAS0 ? 4 : 2;
      auto fe = [&](int j) { return z(ce, base + row + j); };
      auto fo = [&](int j) { return z(co, base + row + j); };
      r += (D1w<NEU1>(fe, i1, g.n1) + D2w<NEU1>(fo, i1, g.n1)) * g.ih1;
    }
    if (HAS0) {
      auto fe = [&](int i) { return z(1, base + (size_t)i * g.n1 + i1); };
      auto fo = [&](int i) { return z(2, base + (size_t)i * g.n1 + i1); };
      r += (D1w<NEU0>(fe, i0, g.n0) + D2w<NEU0>(fo, i0, g.n0)) * g.ih0;
    }
    if (HASBAR && t == 0) r -= sigma * a.m0[rem] * g.idt;
    b[base + rem] = r;
    if (HASBAR) acc += r * r;
    zprev = zc;
  }
}

template <bool HASBAR, bool ZM, bool HAS0, int BC>
__device__ void rhs_cells(const RhsArgs& a, int lb, int nb, double& acc) {
  (void)nb;
  const Geom g = a.g;
  const int nsp = rhs_nsp(g);
  const int chunk = lb / nsp;
  const int t0 = chunk * a.tc, t1 = min(g.nt, t0 + a.tc);
  for (int rem = (lb - chunk * nsp) * kThreads + (int)threadIdx.x; rem < g.M;
       rem += nsp * kThreads)
    rhs_column<HASBAR, ZM, HAS0, BC>(a, rem, t0, t1, acc);
}

template <bool HASBAR, bool ZM>
struct RhsCells {
  template <bool HAS0, int BC>
  struct F {
    __device__ static void run(const RhsArgs& a, int bid, int nb, double& acc) {
      rhs_cells<HASBAR, ZM, HAS0, BC>(a, bid, nb, acc);
    }
  };
};

template <bool HASBAR>
__device__ void rhs_finish(const RhsArgs& a, int bid, double (&acc)[1]) {
  if (HASBAR && a.init) {
    // PCG start: x = 0 (written by the first update), r = b, b.b partials,
    // status reset
    if (bid == 0 && threadIdx.x == 0) {
      double* S = a.rb.scal;
      S[S_TOL2] = a.tol2_dev ? *a.tol2_dev : a.tol2;
      S[S_BAD] = 0.0;
      S[S_DONE] = 0.0;
      S[S_ITS] = 0.0;
    }
    reduce_store<1>(acc, a.rb, T_BB, bid);
  }
}

// Batched form: the z source and the geometry are chosen per instance.
template <bool HASBAR>
__device__ void rhs_body(const RhsArgs& a, int bid, int nb) {
  double acc[1] = {0.0};
  if (HASBAR && a.zin && (!a.zmode_dev || *a.zmode_dev != 0.0))
    geom_dispatch<RhsCells<HASBAR, true>::template F>(a.g, a, bid, nb, acc[0]);
  else
    geom_dispatch<RhsCells<HASBAR, false>::template F>(a.g, a, bid, nb, acc[0]);
  rhs_finish<HASBAR>(a, bid, acc);
}

// LDS-tiled right-hand side (b = Cr z - sigma [t==0] m0/dt with z = zin, or
// z = xi + sigma ybar formed with one rounding). A block owns a TI x TJ spatial
// tile and walks a chunk of a.tc time slices; per slice every component of z
// on the tile plus a one-node halo (wrapped or mirrored at the boundary, as
// nbr1 picks the neighbour) is staged in LDS with coalesced loads, and the
// loads of slice t+1 are issued into registers before slice t is computed.
// Each z value is read from global memory once per block (plus the halo), the
// neighbours come from LDS, and each thread keeps its cells' m-component of
// slice t for the next slice's -z_{t-1}/dt term. The per-cell arithmetic is
// that of rhs_column, term for term.
constexpr int kRThreads = 512;  // threads of a tiled right-hand-side block

template <bool HAS0>
struct RTile {
  static constexpr int TI = HAS0 ? 16 : 1;     // tile rows (axis 0)
  static constexpr int TJ = HAS0 ? 64 : 512;   // tile columns (axis 1)
  static constexpr int H0 = HAS0 ? 1 : 0;      // halo rows
  static constexpr int SI = TI + 2 * H0, SJ = TJ + 2;
  static constexpr int NS = SI * SJ;           // staged values per component
  static constexpr int NC = HAS0 ? 5 : 3;      // components of z
  static constexpr int NPER = (NS + kRThreads - 1) / kRThreads;
  static constexpr int CPT = TI * TJ / kRThreads;  // cells per thread
};

// ZMODE: 1 z read from zin, 0 z = xi + sigma ybar, -1 chosen per block (batched).
// LDS of a tiled right-hand-side block (the d = 2 tile, the larger one)
constexpr int kRhsLds = RTile<true>::NC * RTile<true>::NS;
static_assert(RTile<false>::NC * RTile<false>::NS <= kRhsLds, "d = 1 tile exceeds the LDS size");

template <int ZMODE, bool HAS0, int BC>
__device__ void rhs_tile_body(const RhsArgs& a, int lb, double& acc, double* lds) {
  using R = RTile<HAS0>;
  constexpr bool NEU1 = (BC & 1) != 0, NEU0 = (BC & 2) != 0;
  const Geom& g = a.g;
  const bool zm = ZMODE == 1 || (ZMODE < 0 && a.zin && (!a.zmode_dev || *a.zmode_dev != 0.0));
  const double* __restrict__ src = zm ? a.zin : a.xi;
  const double* __restrict__ ybar = a.ybar;
  double* __restrict__ b = a.b;
  const double sigma = a.sigma_dev ? *a.sigma_dev : a.sigma;
  const long long n = g.n;
  const int tiles1 = (g.n1 + R::TJ - 1) / R::TJ;
  const int tiles0 = HAS0 ? (g.n0 + R::TI - 1) / R::TI : 1;
  const int tile = lb % (tiles0 * tiles1), chunk = lb / (tiles0 * tiles1);
  const int i0 = (tile / tiles1) * R::TI, j0 = (tile % tiles1) * R::TJ;
  const int t_lo = chunk * a.tc, t_hi = min(g.nt, t_lo + a.tc);
  auto Zs = reinterpret_cast<double (*)[R::NS]>(lds);  // Zs[component][staged value]
  // staged element e of this thread: byte offset within a slice (32 bits: a
  // slice of M < 2^28 cells, checked by the plan), so the loads take a uniform
  // base and a 32-bit per-lane offset
  unsigned off[R::NPER];
  bool has[R::NPER];
#pragma unroll
  for (int e = 0; e < R::NPER; ++e) {
    const int idx = threadIdx.x + kRThreads * e;
    has[e] = idx < R::NS;
    off[e] = 0u;
    if (has[e]) {
      const int ii = idx / R::SJ - R::H0, jj = idx % R::SJ - 1;
      const int gi = HAS0 ? nbr_tile(i0 + ii, g.n0, NEU0) : 0;
      const int gj = nbr_tile(j0 + jj, g.n1, NEU1);
      off[e] = (unsigned)(gi * g.n1 + gj) * 8u;
    }
  }
  double rz[R::NC][R::NPER], ry[ZMODE == 1 ? 1 : R::NC][R::NPER];
  auto issue = [&](int t) {
    const size_t base = (size_t)t * g.M;
#pragma unroll
    for (int c = 0; c < R::NC; ++c) {
      // uniform slice base per component, 32-bit byte offsets per element
      const char* __restrict__ zc_ = reinterpret_cast<const char*>(src + (size_t)c * n + base);
      const char* __restrict__ yc_ =
          ZMODE == 1 ? nullptr : reinterpret_cast<const char*>(ybar + (size_t)c * n + base);
#pragma unroll
      for (int e = 0; e < R::NPER; ++e)
        if (has[e]) {
          rz[c][e] = *reinterpret_cast<const double*>(zc_ + off[e]);
          if constexpr (ZMODE != 1) {
            if (!zm) ry[c][e] = *reinterpret_cast<const double*>(yc_ + off[e]);
          }
        }
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int c = 0; c < R::NC; ++c)
#pragma unroll
      for (int e = 0; e < R::NPER; ++e)
        if (has[e]) {
          double v = rz[c][e];
          // one rounding (fma), as where z is formed by the back-projection
          if constexpr (ZMODE != 1) {
            if (!zm) v = __builtin_fma(sigma, ry[c][e], v);
          }
          Zs[c][threadIdx.x + kRThreads * e] = v;
        }
  };
  double zprev[R::CPT];
  // the m-component of slice t_lo - 1 at this thread's cells
#pragma unroll
  for (int k = 0; k < R::CPT; ++k) {
    const int idx = threadIdx.x + kRThreads * k;
    const int ii = idx / R::TJ, jj = idx % R::TJ;
    zprev[k] = 0.0;
    if (t_lo >= 1 && i0 + ii < g.n0 && j0 + jj < g.n1) {
      const size_t o = (size_t)(t_lo - 1) * g.M + (size_t)(i0 + ii) * g.n1 + j0 + jj;
      zprev[k] = zm ? src[o] : __builtin_fma(sigma, ybar[o], src[o]);
    }
  }
  constexpr int C1 = HAS0 ? 1 : 0, C2 = HAS0 ? 2 : 0;   // axis-0 flux components
  constexpr int CE = HAS0 ? 3 : 1, CO = HAS0 ? 4 : 2;   // axis-1 flux components
  if (t_lo < t_hi) issue(t_lo);
  for (int t = t_lo; t < t_hi; ++t) {
    commit();
    __syncthreads();
    if (t + 1 < t_hi) issue(t + 1);
#pragma unroll
    for (int k = 0; k < R::CPT; ++k) {
      const int idx = threadIdx.x + kRThreads * k;
      const int ii = idx / R::TJ, jj = idx % R::TJ;
      const int gi = i0 + ii, gj = j0 + jj;
      if (gi < g.n0 && gj < g.n1) {
        const int c = (ii + R::H0) * R::SJ + jj + 1;
        const double* Z0 = Zs[0];
        const double zc = Z0[c];
        double Kz = (2.0 * zc - Z0[c + 1] - Z0[c - 1]) * g.ih1sq;
        if (HAS0) Kz += (2.0 * zc - Z0[c + R::SJ] - Z0[c - R::SJ]) * g.ih0sq;
        double r = g.nu * Kz + zc * g.idt;
        if (t >= 1) r -= zprev[k] * g.idt;
        {
          const double* E = Zs[CE];
          const double* O = Zs[CO];
          // D^1 w_e = w_i - w_{i-1}, D^2 w_o = w_{i+1} - w_i (Neumann: the
          // terms across the boundary do not enter)
          const double d1 = NEU1 ? (gj <= g.n1 - 2 ? E[c] : 0.0) - (gj >= 1 ? E[c - 1] : 0.0)
                                 : E[c] - E[c - 1];
          const double d2 = NEU1 ? (gj <= g.n1 - 2 ? O[c + 1] : 0.0) - (gj >= 1 ? O[c] : 0.0)
                                 : O[c + 1] - O[c];
          r += (d1 + d2) * g.ih1;
        }
        if (HAS0) {
          const double* E = Zs[C1];
          const double* O = Zs[C2];
          const double d1 = NEU0 ? (gi <= g.n0 - 2 ? E[c] : 0.0) - (gi >= 1 ? E[c - R::SJ] : 0.0)
                                 : E[c] - E[c - R::SJ];
          const double d2 = NEU0 ? (gi <= g.n0 - 2 ? O[c + R::SJ] : 0.0) - (gi >= 1 ? O[c] : 0.0)
                                 : O[c + R::SJ] - O[c];
          r += (d1 + d2) * g.ih0;
        }
        const int rem = gi * g.n1 + gj;
        if (t == 0) r -= sigma * a.m0[rem] * g.idt;
        b[(size_t)t * g.M + rem] = r;
        acc += r * r;
        zprev[k] = zc;
      }
    }
    __syncthreads();
  }
}

template <bool HAS0, int BC>
struct RhsTileBatch {
  __device__ static void run(const RhsArgs& a, int lb, double& acc, double* lds) {
    rhs_tile_body<-1, HAS0, BC>(a, lb, acc, lds);
  }
};

// Batched form of the tiled right-hand side: z source and geometry per instance.
__device__ void rhs_tile_batch_body(const RhsArgs& a, int bid) {
  __shared__ double lds[kRhsLds];
  double acc[1] = {0.0};
  geom_dispatch<RhsTileBatch>(a.g, a, bid, acc[0], lds);
  rhs_finish<true>(a, bid, acc);
}

// Components of Cr^T u at one cell: out[0] = m-part, out[1+c] = B_c^T u_t.
template <bool HAS0, int BC>
__device__ __forceinline__ void CT_cell(const Geom& g, const double* __restrict__ u, int t, int i0,
                                        int i1, double* out) {
  const double uc = u[at(g, t, i0, i1)];
  double m = g.nu * Kop<HAS0, BC>(u, g, t, i0, i1) + uc * g.idt;
  if (t <= g.nt - 2) m -= u[at(g, t + 1, i0, i1)] * g.idt;
  out[0] = m;
  {
    constexpr int cb1 = HAS0 ? 2 : 0;
    const double up = u[at(g, t, i0, nbr1(i1 + 1, g.n1, BC & 1))];
    const double um = u[at(g, t, i0, nbr1(i1 - 1, g.n1, BC & 1))];
    out[1 + cb1] = (uc - up) * g.ih1;
    out[2 + cb1] = (um - uc) * g.ih1;
  }
  if (HAS0) {
    const double up = u[at(g, t, nbr1(i0 + 1, g.n0, BC & 2), i1)];
    const double um = u[at(g, t, nbr1(i0 - 1, g.n0, BC & 2), i1)];
    out[1] = (uc - up) * g.ih0;
    out[2] = (um - uc) * g.ih0;
  }
}

template <bool HAS0, int BC>
struct ApplyCT {
  __device__ static void run(const Geom& g, const double* __restrict__ u,
                             double* __restrict__ y) {
    constexpr int NC = HAS0 ? 4 : 2;
    const long long n = g.n;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
      // n < 2^31 (checked by the plan): 32-bit index arithmetic
      const unsigned pu = (unsigned)p;
      const int t = (int)(pu / (unsigned)g.M);
      const int rem = (int)(pu - (unsigned)t * (unsigned)g.M);
      const int i0 = (int)((unsigned)rem / (unsigned)g.n1), i1 = rem - i0 * g.n1;
      double out[5];
      CT_cell<HAS0, BC>(g, u, t, i0, i1, out);
#pragma unroll
      for (int c = 0; c <= NC; ++c) y[(size_t)c * n + p] = out[c];
    }
  }
};

__global__ __launch_bounds__(kThreads) void k_apply_CT(Geom g, const double* __restrict__ u,
                                                       double* __restrict__ y) {
  geom_dispatch<ApplyCT>(g, g, u, y);
}

// (A u)_t = K g_t + ((1 + [t>=1]) u_t - s_t)/dt^2 with
//   g_t = nu^2 K u_t + (2 nu/dt + 2) u_t - (nu/dt) s_t,   s_t = u_{t-1} + u_{t+1},
// which is eq. largeA with C = L^2 + B B^T = nu^2 K^2 + (2nu/dt) K + I/dt^2 + 2K
// (B B^T = 2K, eq. precstead) and the off-diagonal blocks -L/dt.
//
// Each block owns a TI x TJ spatial tile and a chunk of time slices and walks
// the chunk in time, keeping slices t-1, t, t+1 (tile plus a 2-node halo) in an
// LDS ring, so every slice is read once per block; g is staged in LDS on the
// tile plus a 1-node halo. In FUSE mode the input is the PCG direction formed on
// the fly, p = z + beta p_old (p = z on the first iteration), written to p_new
// by the block that owns the node; p_old and p_new are different buffers, so
// halo reads never see a value updated by a neighbouring block.
constexpr int kTJ = 64;
// BIG = 0, 1, 2: 16-, 32- or 64-row tiles for 256-, 512- or 1024-thread blocks
// (larger tiles: smaller halo share, barriers amortised over more work).
template <bool HAS0, int BIG = 0>
struct Tile {
  static constexpr int NT = 256 << BIG;  // threads per block
  static constexpr int TI = HAS0 ? (16 << BIG) : 1;   // tile rows (axis 0)
  static constexpr int HI = HAS0 ? 2 : 0;    // halo rows of the u slots
  static constexpr int GH = HAS0 ? 1 : 0;    // halo rows of g
  static constexpr int SI = TI + 2 * HI;
  static constexpr int SJ = kTJ + 4;
  static constexpr int GI = TI + 2 * GH;
  static constexpr int GJ = kTJ + 2;
};

template <bool HAS0, bool FUSE, int BIG = 0>
__device__ void aat_body(const AatArgs& a, int bid, int nb) {
  if (a.done && *a.done != 0.0) return;
  using C = Tile<HAS0, BIG>;
  const Geom g = a.g;
  const double* __restrict__ src = a.src;
  const double* __restrict__ pold = a.pold;
  double* __restrict__ pnew = a.pnew;
  double* __restrict__ q = a.q;
  const RedBuf rb = a.rb;
  const int tc = a.tc, first = a.first, reduce = a.reduce;
  __shared__ double U[3][C::SI * C::SJ];
  __shared__ double G[C::GI * C::GJ];
  const int tiles1 = (g.n1 + kTJ - 1) / kTJ;
  const int tiles0 = HAS0 ? (g.n0 + C::TI - 1) / C::TI : 1;
  const int nchunk = (g.nt + tc - 1) / tc;
  const int blk = xcd_remap(bid, nb);
  const int tile = blk / nchunk, chunk = blk - tile * nchunk;
  const int i0 = (tile / tiles1) * C::TI, j0 = (tile % tiles1) * kTJ;
  (void)tiles0;
  const int t_lo = chunk * tc;
  const int t_hi = (t_lo + tc < g.nt) ? t_lo + tc : g.nt;
  // PCG direction form: beta from the r.z (z.q) partials of the last
  // preconditioner application; a breakdown there (r.z not positive or not
  // finite) ends the solve.
  double beta = 0.0;
  if (FUSE && a.nrz > 0) {
    double f[2];
    fold_partials<2>(rb, T_RZ, a.nrz, f);
    const int bad = (!finite_d(f[0]) || !finite_d(f[1])) ? 2 : (!(f[0] > 0.0) ? 1 : 0);
    if (bad) {
      if (bid == 0 && threadIdx.x == 0) {
        rb.scal[S_BAD] = (double)bad;
        rb.scal[S_DONE] = 1.0;
      }
      return;
    }
    if (!first) {
      const double rho = rb.scal[S_RHO];
      beta = a.flex ? -rb.scal[S_ALPHA] * f[1] / rho : f[0] / rho;
    }
    if (bid == 0 && threadIdx.x == 0) rb.scal[S_BETA] = beta;
  }
  const double c1 = 2.0 * g.nu * g.idt + 2.0, c2 = g.nu * g.idt, nu2 = g.nu * g.nu;

  // Slot loads are split into issue (global loads into registers) and commit
  // (combine, publish p_new, store to LDS), so the loads of slice t+2 are in
  // flight while slice t is being computed.
  constexpr int NS = C::SI * C::SJ;
  constexpr int NPER = (NS + C::NT - 1) / C::NT;
  double rz[NPER], rp[NPER];
  auto issue = [&](int t) {
#pragma unroll
    for (int e = 0; e < NPER; ++e) {
      const int idx = threadIdx.x + C::NT * e;
      rz[e] = 0.0;
      rp[e] = 0.0;
      if (idx < NS && t >= 0 && t < g.nt) {
        const int ii = idx / C::SJ - C::HI, jj = idx % C::SJ - 2;
        const int gi = HAS0 ? nbr_tile(i0 + ii, g.n0, g.bcm & 2) : 0;
        const int gj = nbr_tile(j0 + jj, g.n1, g.bcm & 1);
        const size_t o = (size_t)t * g.M + (size_t)gi * g.n1 + gj;
        rz[e] = src[o];
        if (FUSE && !first) rp[e] = pold[o];
      }
    }
  };
  auto commit = [&](int t, double* dst) {
#pragma unroll
    for (int e = 0; e < NPER; ++e) {
      const int idx = threadIdx.x + C::NT * e;
      if (idx < NS) {
        const double v = FUSE ? rz[e] + beta * rp[e] : rz[e];
        if (FUSE && t >= t_lo && t < t_hi) {
          const int ii = idx / C::SJ - C::HI, jj = idx % C::SJ - 2;
          if (ii >= 0 && ii < C::TI && jj >= 0 && jj < kTJ && i0 + ii < g.n0 && j0 + jj < g.n1)
            pnew[(size_t)t * g.M + (size_t)(i0 + ii) * g.n1 + j0 + jj] = v;
        }
        dst[idx] = v;
      }
    }
  };

  double acc = 0.0;
  int sp = 0, sc = 1, sn = 2;
  issue(t_lo - 1);
  commit(t_lo - 1, U[sp]);
  issue(t_lo);
  commit(t_lo, U[sc]);
  issue(t_lo + 1);
  for (int t = t_lo; t < t_hi; ++t) {
    commit(t + 1, U[sn]);
    __syncthreads();
    if (t + 1 < t_hi) issue(t + 2);
    const double* Up = U[sp];
    const double* Uc = U[sc];
    const double* Un = U[sn];
    for (int idx = threadIdx.x; idx < C::GI * C::GJ; idx += blockDim.x) {
      const int gi = idx / C::GJ, gj = idx - gi * C::GJ;
      const int c = (gi - C::GH + C::HI) * C::SJ + gj + 1;
      const double u = Uc[c];
      double Ku = (2.0 * u - Uc[c + 1] - Uc[c - 1]) * g.ih1sq;
      if (HAS0) Ku += (2.0 * u - Uc[c + C::SJ] - Uc[c - C::SJ]) * g.ih0sq;
      G[idx] = nu2 * Ku + c1 * u - c2 * (Up[c] + Un[c]);
    }
    __syncthreads();
    const double diag = (t >= 1) ? 2.0 : 1.0;
    for (int idx = threadIdx.x; idx < C::TI * kTJ; idx += blockDim.x) {
      const int ii = idx / kTJ, jj = idx - ii * kTJ;
      if (i0 + ii < g.n0 && j0 + jj < g.n1) {
        const int gc = (ii + C::GH) * C::GJ + jj + 1;
        const double gv = G[gc];
        double Kg = (2.0 * gv - G[gc + 1] - G[gc - 1]) * g.ih1sq;
        if (HAS0) Kg += (2.0 * gv - G[gc + C::GJ] - G[gc - C::GJ]) * g.ih0sq;
        const int c = (ii + C::HI) * C::SJ + jj + 2;
        const double u = Uc[c];
        const double val = Kg + (diag * u - (Up[c] + Un[c])) * g.idt2;
        q[(size_t)t * g.M + (size_t)(i0 + ii) * g.n1 + j0 + jj] = val;
        acc += u * val;
      }
    }
    __syncthreads();
    const int tmp = sp;
    sp = sc;
    sc = sn;
    sn = tmp;
  }
  if (reduce) {
    double v[1] = {acc};
    reduce_store<1>(v, rb, T_PQ, bid);
  }
}

// The per-cell prox of Section 3 is prox_cell (prox_cell.h): the coupling's
// coefficients are g.c2 and, per slice, (g.c1, V) or, on the last slice,
// (g.c1T, VT).
__global__ __launch_bounds__(kThreads) void k_prox(Geom g, const double* __restrict__ v,
                                                   const double* __restrict__ Vpot,
                                                   const double* __restrict__ VT, double tau,
                                                   double* __restrict__ y) {
  const long long n = g.n;
  const unsigned last = (unsigned)(g.nt - 1) * (unsigned)g.M;  // n < 2^31
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int rem = (int)((unsigned)p % (unsigned)g.M);
    const bool lastslice = (unsigned)p >= last;
    const double Vc = lastslice ? VT[rem] : Vpot[rem];
    const double c1 = lastslice ? g.c1T : g.c1;
    double w[4];
    for (int c = 0; c < g.ncomp; ++c) w[c] = v[(size_t)(c + 1) * n + p];
    const bool qg = g.q != 2.0;
    const double m =
        g.has0 ? (qg ? prox_cell<4, true>(v[p], w, Vc, tau, c1, g.c2, g.q, g.qp)
                     : prox_cell<4>(v[p], w, Vc, tau, c1, g.c2))
               : (qg ? prox_cell<2, true>(v[p], w, Vc, tau, c1, g.c2, g.q, g.qp)
                     : prox_cell<2>(v[p], w, Vc, tau, c1, g.c2));
    y[p] = m;
    for (int c = 0; c < g.ncomp; ++c) y[(size_t)(c + 1) * n + p] = w[c];
  }
}

// VT = V - w mbar with w = 1/(beta dt): the last slice's potential once the
// terminal cost G/dt = (m^2/2 - mbar m)/(beta dt) is folded in (w = 0 without it).
__global__ __launch_bounds__(kThreads) void k_terminal_potential(int M, const double* __restrict__ V,
                                                                 const double* __restrict__ mbar,
                                                                 double w,
                                                                 double* __restrict__ VT) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x)
    VT[i] = (w == 0.0) ? V[i] : V[i] - w * mbar[i];
}

// Value function of the scheme (MFG_T^2_h) from the multiplier lam of the
// reduced constraint: u^k = -lam_k for k < N_t and u^{N_t} = g(m^{N_t}) =
// (m^{N_t} - mbar)/beta (ib = 1/beta; 0 without a terminal cost). u holds
// N_t + 1 slices.
__global__ __launch_bounds__(kThreads) void k_value(Geom g, const double* __restrict__ lam,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ mbar, double ib,
                                                    double* __restrict__ u) {
  const long long n = g.n, tot = n + g.M;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < tot;
       p += (long long)gridDim.x * blockDim.x) {
    if (p < n) {
      u[p] = -lam[p];
    } else {
      const long long i = p - n;
      u[p] = (ib == 0.0) ? 0.0 : (y[n - g.M + i] - mbar[i]) * ib;
    }
  }
}

// Residual of the discrete HJB equation of (MFG_T^2_h) at cell (t, i0, i1):
//   R = (u^t - u^{t+1})/dt + nu K u^t + |P_K(-[D_h u^t])|^2 / 2 - f(x, m^{t+1}),
// where -[D_h u] is the flux part of Cr^T u (B_c^T u per component) and
// f = c2 m^2 + c1 m + V; u has N_t + 1 slices, m is the primal's first block.
template <bool HAS0, int BC>
struct HjbCells {
  __device__ static void run(const Geom& g, const double* __restrict__ y,
                             const double* __restrict__ u, const double* __restrict__ Vpot,
                             double* __restrict__ R) {
    const long long n = g.n;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
      const unsigned pu = (unsigned)p;  // n < 2^31
      const int t = (int)(pu / (unsigned)g.M);
      const int rem = (int)(pu - (unsigned)t * (unsigned)g.M);
      const int i0 = (int)((unsigned)rem / (unsigned)g.n1), i1 = rem - i0 * g.n1;
      const double uc = u[at(g, t, i0, i1)];
      double ham = 0.0;
      {
        const double up = u[at(g, t, i0, nbr1(i1 + 1, g.n1, BC & 1))];
        const double um = u[at(g, t, i0, nbr1(i1 - 1, g.n1, BC & 1))];
        const double e = fmax((uc - up) * g.ih1, 0.0), o = fmin((um - uc) * g.ih1, 0.0);
        ham += e * e + o * o;
      }
      if (HAS0) {
        const double up = u[at(g, t, nbr1(i0 + 1, g.n0, BC & 2), i1)];
        const double um = u[at(g, t, nbr1(i0 - 1, g.n0, BC & 2), i1)];
        const double e = fmax((uc - up) * g.ih0, 0.0), o = fmin((um - uc) * g.ih0, 0.0);
        ham += e * e + o * o;
      }
      const double m = y[p];
      const double f = (g.c2 * m + g.c1) * m + Vpot[rem];
      // Hamiltonian |P_K(-D u)|^q'/q' (ham holds the squared norm)
      const double hq = g.qp == 2.0 ? 0.5 * ham : pow(ham, 0.5 * g.qp) / g.qp;
      R[p] = (uc - u[p + g.M]) * g.idt + g.nu * Kop<HAS0, BC>(u, g, t, i0, i1) + hq - f;
    }
  }
};

__global__ __launch_bounds__(kThreads) void k_hjb(Geom g, const double* __restrict__ y,
                                                  const double* __restrict__ u,
                                                  const double* __restrict__ Vpot,
                                                  double* __restrict__ R) {
  geom_dispatch<HjbCells>(g, g, y, u, Vpot, R);
}

// One CP iteration after the projection solve:
//   xi' = Cr^T u;  y' = prox_{tau phi}(y - tau xi');  ybar = y' + theta (y' - y);
// partial ||m' - m||^2 reduced into the device scalar S_DM.
// QG: general exponent q' of the Hamiltonian (prox_cell).
template <bool HAS0, int BC, bool QG>
struct BackprojCellsQ {
  __device__ static void run(const BackprojArgs& a, int bid, int nb, double tau, double theta,
                             double sig_next, double& acc) {
    constexpr int NC = HAS0 ? 4 : 2;
    const Geom& g = a.g;
    const double* __restrict__ u = a.u;
    double* __restrict__ xi = a.xi;
    double* __restrict__ y = a.y;
    double* __restrict__ ybar = a.ybar;
    const double* __restrict__ Vpot = a.V;
    const double* __restrict__ VT = a.VT;
    double* __restrict__ vout = a.vout;
    double* __restrict__ zout = a.zout;
    const long long n = g.n;
    for (long long p = (long long)bid * blockDim.x + threadIdx.x; p < n;
         p += (long long)nb * blockDim.x) {
      // n < 2^31 (checked by the plan): 32-bit index arithmetic
      const unsigned pu = (unsigned)p;
      const int t = (int)(pu / (unsigned)g.M);
      const int rem = (int)(pu - (unsigned)t * (unsigned)g.M);
      const int i0 = (int)((unsigned)rem / (unsigned)g.n1), i1 = rem - i0 * g.n1;
      double x[5], yo[5], w[4];
      CT_cell<HAS0, BC>(g, u, t, i0, i1, x);
#pragma unroll
      for (int c = 0; c <= NC; ++c) yo[c] = y[(size_t)c * n + p];
#pragma unroll
      for (int c = 0; c < NC; ++c) w[c] = yo[1 + c] - tau * x[1 + c];
      const double mbar = yo[0] - tau * x[0];
      if (vout) {
        vout[p] = mbar;
#pragma unroll
        for (int c = 0; c < NC; ++c) vout[(size_t)(c + 1) * n + p] = w[c];
      }
      const bool lastslice = t == g.nt - 1;
      const double m = prox_cell<NC, QG>(mbar, w, lastslice ? VT[rem] : Vpot[rem], tau,
                                         lastslice ? g.c1T : g.c1, g.c2, g.q, g.qp);
      // streaming stores: the new state is read again only by the next step
      const double mb = m + theta * (m - yo[0]);
      __builtin_nontemporal_store(m, &y[p]);
#pragma unroll
      for (int c = 0; c < NC; ++c) __builtin_nontemporal_store(w[c], &y[(size_t)(c + 1) * n + p]);
      if (zout) {
        // one rounding (fma), as where the right-hand side forms z from xi, ybar
        __builtin_nontemporal_store(__builtin_fma(sig_next, mb, x[0]), &zout[p]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double wb = w[c] + theta * (w[c] - yo[1 + c]);
          __builtin_nontemporal_store(__builtin_fma(sig_next, wb, x[1 + c]),
                                      &zout[(size_t)(c + 1) * n + p]);
        }
      } else {
#pragma unroll
        for (int c = 0; c <= NC; ++c) __builtin_nontemporal_store(x[c], &xi[(size_t)c * n + p]);
        __builtin_nontemporal_store(mb, &ybar[p]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
          __builtin_nontemporal_store(w[c] + theta * (w[c] - yo[1 + c]),
                                      &ybar[(size_t)(c + 1) * n + p]);
      }
      const double dm = m - yo[0];
      acc += dm * dm;
    }
  }
};

template <bool HAS0, int BC>
using BackprojCells = BackprojCellsQ<HAS0, BC, false>;

// GEO: 0 = geometry chosen per block (batched form, q' = 2), else
// 1 + 4 HAS0 + BC; QG: general exponent q'.
template <int GEO, bool QG = false>
__device__ void backproj_body(const BackprojArgs& a, int bid, int nb) {
  const double tau = a.tau_dev ? *a.tau_dev : a.tau;
  const double theta = a.theta_dev ? *a.theta_dev : a.theta;
  const double sig_next = a.zout ? (a.sigma_dev ? *a.sigma_dev : a.sigma) / theta : 0.0;
  if (a.zflag && bid == 0 && threadIdx.x == 0) *a.zflag = a.zout ? 1.0 : 0.0;
  double acc[1] = {0.0};
  if constexpr (GEO == 0)
    geom_dispatch<BackprojCells>(a.g, a, bid, nb, tau, theta, sig_next, acc[0]);
  else
    BackprojCellsQ<((GEO - 1) & 4) != 0, (GEO - 1) & 3, QG>::run(a, bid, nb, tau, theta,
                                                                 sig_next, acc[0]);
  reduce_store<1>(acc, a.rb, T_DM, bid);
}

// Single-plan form, one specialisation per geometry. Logical blocks in
// contiguous ranges per XCD: the blocks that read a row's neighbour rows of u
// (and slice t+1) mostly share an L2.
template <int GEO, bool QG>
__global__ __launch_bounds__(kThreads) void k_backproj_prox(BackprojArgs a) {
  backproj_body<GEO, QG>(a, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

__global__ __launch_bounds__(kThreads) void k_backproj_prox_batch(const BackprojArgs* A,
                                                                  const int* off, int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  const BackprojArgs a = A[i];
  backproj_body<0>(a, blockIdx.x - off[i], off[i + 1] - off[i]);
}

// Single-plan form: one specialisation per z source and geometry (chosen on
// the host), so each carries only its own path's registers.
template <bool HASBAR, bool ZM, bool HAS0, int BC>
__global__ __launch_bounds__(kThreads) void k_rhs(RhsArgs a) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  double acc[1] = {0.0};
  rhs_cells<HASBAR, ZM, HAS0, BC>(a, lb, gridDim.x, acc[0]);
  rhs_finish<HASBAR>(a, lb, acc);
}

template <bool HASBAR, bool ZM>
void rhs_launch(const RhsArgs& a, int grid, hipStream_t s) {
  const dim3 gd(grid), bd(kThreads);
  if (a.g.has0) {
    switch (a.g.bcm) {
      case 0: hipLaunchKernelGGL((k_rhs<HASBAR, ZM, true, 0>), gd, bd, 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_rhs<HASBAR, ZM, true, 1>), gd, bd, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_rhs<HASBAR, ZM, true, 2>), gd, bd, 0, s, a); break;
      default: hipLaunchKernelGGL((k_rhs<HASBAR, ZM, true, 3>), gd, bd, 0, s, a);
    }
  } else {
    if (a.g.bcm & 1) hipLaunchKernelGGL((k_rhs<HASBAR, ZM, false, 1>), gd, bd, 0, s, a);
    else hipLaunchKernelGGL((k_rhs<HASBAR, ZM, false, 0>), gd, bd, 0, s, a);
  }
}

__global__ __launch_bounds__(kRThreads) void k_rhs_batch(const RhsArgs* A, const int* off,
                                                         int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  const RhsArgs a = A[i];  // one copy of the instance's arguments for every specialisation
  rhs_tile_batch_body(a, blockIdx.x - off[i]);
}

// Single-plan tiled right-hand side, one specialisation per z source and geometry.
template <int ZMODE, bool HAS0, int BC>
__global__ __launch_bounds__(kRThreads) void k_rhs_tile(RhsArgs a) {
  __shared__ double lds[kRhsLds];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  double acc[1] = {0.0};
  rhs_tile_body<ZMODE, HAS0, BC>(a, lb, acc[0], lds);
  rhs_finish<true>(a, lb, acc);
}

template <int ZMODE>
void rhs_tile_launch(const RhsArgs& a, int grid, hipStream_t s) {
  const dim3 gd(grid), bd(kRThreads);
  if (a.g.has0) {
    switch (a.g.bcm) {
      case 0: hipLaunchKernelGGL((k_rhs_tile<ZMODE, true, 0>), gd, bd, 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_rhs_tile<ZMODE, true, 1>), gd, bd, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_rhs_tile<ZMODE, true, 2>), gd, bd, 0, s, a); break;
      default: hipLaunchKernelGGL((k_rhs_tile<ZMODE, true, 3>), gd, bd, 0, s, a);
    }
  } else {
    if (a.g.bcm & 1) hipLaunchKernelGGL((k_rhs_tile<ZMODE, false, 1>), gd, bd, 0, s, a);
    else hipLaunchKernelGGL((k_rhs_tile<ZMODE, false, 0>), gd, bd, 0, s, a);
  }
}

template <bool HAS0, bool FUSE, int BIG>
__global__ __launch_bounds__((Tile<HAS0, BIG>::NT)) void k_AAt_tile(AatArgs a) {
  aat_body<HAS0, FUSE, BIG>(a, blockIdx.x, gridDim.x);
}

// Batched launches use the default tile (32 rows for d = 2): one block size
// for every instance.
constexpr int kBatchBig = 1;
static_assert(kBatchBig == Tune{}.aat_big, "batched and single-plan default A tiles differ");

template <bool HAS0>
__global__ __launch_bounds__((Tile<HAS0, HAS0 ? kBatchBig : 0>::NT)) void k_AAt_batch(
    const AatArgs* A, const int* off, int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  aat_body<HAS0, true, HAS0 ? kBatchBig : 0>(A[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

// Persistent form of the batched A phase over a tile queue: a resident grid
// whose blocks take virtual block ids (instance tiles in the batch's order) from
// a device counter until every one is taken; each runs the batched kernel's
// body with that id, so the results are the same bits. The counter starts at 0
// (k_queue_reset, a kernel so the step can be recorded in a graph); every block
// leaves once the counter passes `total`.
__global__ void k_queue_reset(int* q) {
  if (threadIdx.x == 0) *q = 0;
}

template <bool HAS0>
__global__ __launch_bounds__((Tile<HAS0, HAS0 ? kBatchBig : 0>::NT)) void k_AAt_batch_queue(
    const AatArgs* A, const int* off, int ninst, int total, int* queue) {
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(queue, 1);
    __syncthreads();  // also: the previous tile's LDS reads are over
    const int vb = next;
    __syncthreads();  // `next` is read before thread 0 takes the next id
    if (vb >= total) return;
    const int i = batch_instance(off, ninst, vb);
    aat_body<HAS0, true, HAS0 ? kBatchBig : 0>(A[i], vb - off[i], off[i + 1] - off[i]);
  }
}

// One thread per node up to `cap` blocks (grid-stride beyond that).
int grid_for(long long n, int cap = kStreamGrid) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// Time-chunk length of the tiled A kernel: enough blocks to fill the chip.
// The grid also stays within the reduction's partial-sum capacity.
int aat_chunk(const Geom& g, int ntile, int max_blocks, int want) {
  long long tc = ((long long)g.nt * ntile) / 1024;
  if (want > 0) tc = want;  // tuned
  if (tc < 1) tc = 1;
  if (tc > 64) tc = 64;
  const long long need = ((long long)g.nt * ntile + max_blocks - 1) / max_blocks;
  if (tc < need) tc = need;
  // the last chunk of a tile may be partial: grow tc until ntile * ceil(nt / tc)
  // fits (ends by tc = nt, where the grid is ntile <= 1024 blocks)
  while (tc < g.nt && (long long)ntile * ((g.nt + tc - 1) / tc) > max_blocks) ++tc;
  return (int)tc;
}

template <bool HAS0, int BIG = 0>
int aat_shape(const Plan& P, int* tc_out) {
  const Geom& g = P.g;
  constexpr int TI = Tile<HAS0, BIG>::TI;
  const int ntile = ((g.n0 + TI - 1) / TI) * ((g.n1 + kTJ - 1) / kTJ);
  const int tc = aat_chunk(g, ntile, P.red.max_blocks, P.tune.aat_tc);
  *tc_out = tc;
  return ntile * ((g.nt + tc - 1) / tc);
}

template <bool HAS0, bool FUSE, int BIG>
void aat_launch_t(const Plan& P, const double* src, const double* pold, double* pnew, double* q,
                  bool first, bool reduce, hipStream_t s) {
  int tc;
  const int grid = aat_shape<HAS0, BIG>(P, &tc);
  // inside a PCG solve, the direction form takes beta from the r.z partials
  const int nrz = (FUSE && P.pcg_done) ? P.rz_blocks : 0;
  const AatArgs a{P.g,    src, pold, pnew, q, P.red, tc, first ? 1 : 0, reduce ? 1 : 0,
                  P.pcg_done, nrz, pcg_flexible(P) ? 1 : 0};
  {
    ProfScope ps(P, FUSE ? "aat_fused" : "aat", s);
    hipLaunchKernelGGL((k_AAt_tile<HAS0, FUSE, BIG>), dim3(grid), dim3(Tile<HAS0, BIG>::NT), 0, s,
                       a);
  }
  // the p.q partials are summed by the update that consumes them
  if (reduce) P.pq_blocks = grid;
}

template <bool HAS0, bool FUSE>
void aat_launch(const Plan& P, const double* src, const double* pold, double* pnew, double* q,
                bool first, bool reduce, hipStream_t s) {
  if constexpr (HAS0) {
    if (P.tune.aat_big == 1) {
      aat_launch_t<HAS0, FUSE, 1>(P, src, pold, pnew, q, first, reduce, s);
      return;
    }
    if (P.tune.aat_big == 2) {
      aat_launch_t<HAS0, FUSE, 2>(P, src, pold, pnew, q, first, reduce, s);
      return;
    }
  }
  aat_launch_t<HAS0, FUSE, 0>(P, src, pold, pnew, q, first, reduce, s);
}

}  // namespace

// Time slices per block of the right-hand-side kernel: about 4096 blocks (at
// most 4096 + 8192, so the b.b partials of a PCG start stay few). A function of
// the geometry only, so batched and single-plan runs sum b.b in the same order.
static int rhs_tc(const Plan& P) {
  const Geom& g = P.g;
  const long long nsp = rhs_nsp(g);
  long long tc = P.tune.rhs_tc > 0 ? P.tune.rhs_tc : (nsp * g.nt + 4095) / 4096;
  // the grid stays within the reduction's partial-sum capacity
  while (tc < g.nt && nsp * ((g.nt + tc - 1) / tc) > P.red.max_blocks) ++tc;
  return (int)(tc < 1 ? 1 : tc > g.nt ? g.nt : tc);
}

// Tiled right-hand side: spatial tiles and time slices per block (about 2048
// blocks, within the partial-sum capacity). A function of the geometry only,
// so batched and single-plan runs sum b.b in the same order.
static int rhs_tiles(const Geom& g) {
  if (g.has0)
    return ((g.n0 + RTile<true>::TI - 1) / RTile<true>::TI) *
           ((g.n1 + RTile<true>::TJ - 1) / RTile<true>::TJ);
  return (g.n1 + RTile<false>::TJ - 1) / RTile<false>::TJ;
}

static int rhs_tile_tc(const Plan& P) {
  const Geom& g = P.g;
  const long long nt_ = g.nt, tiles = rhs_tiles(g);
  long long tc = P.tune.rhs_tc > 0 ? P.tune.rhs_tc : (tiles * nt_ + 2047) / 2048;
  while (tc < nt_ && tiles * ((nt_ + tc - 1) / tc) > P.red.max_blocks) ++tc;
  return (int)(tc < 1 ? 1 : tc > nt_ ? nt_ : tc);
}

RhsArgs rhs_args(const Plan& P, const double* xi, const double* ybar, double sigma,
                 const double* sigma_dev, double* b, const double* zin,
                 const double* zmode_dev) {
  return RhsArgs{P.g,  xi,    ybar, sigma,   sigma_dev,    P.m0, b, zin, zmode_dev, 0,
                 P.red, 0.0, nullptr, rhs_tile_tc(P)};
}

int rhs_grid(const Plan& P) {
  const int tc = rhs_tile_tc(P);
  return rhs_tiles(P.g) * ((P.g.nt + tc - 1) / tc);
}

void launch_rhs(const Plan& P, const double* xi, const double* ybar, double sigma,
                const double* m0, double* b, hipStream_t s, const double* zin, double init_rtol) {
  RhsArgs a = rhs_args(P, xi, ybar, sigma, nullptr, b, zin);
  a.m0 = m0;
  a.init = init_rtol >= 0.0 ? 1 : 0;
  a.tol2 = init_rtol * init_rtol;
  const int grid = rhs_grid(P);
  {
    ProfScope ps(P, "rhs", s);
    if (zin) rhs_tile_launch<1>(a, grid, s);
    else rhs_tile_launch<0>(a, grid, s);
  }
  if (a.init) launch_finish(P, T_BB, grid, OP_BB, s);
}

void launch_apply_C(const Plan& P, const double* y, double* b, hipStream_t s) {
  ProfScope ps(P, "apply_C", s);
  const RhsArgs a{P.g,   y,   nullptr, 0.0, nullptr,       nullptr, b, nullptr, nullptr, 0,
                  P.red, 0.0, nullptr, rhs_tc(P)};
  const int tc = rhs_tc(P);
  rhs_launch<false, false>(a, rhs_nsp(P.g) * ((P.g.nt + tc - 1) / tc), s);
}

void launch_apply_CT(const Plan& P, const double* u, double* y, hipStream_t s) {
  ProfScope ps(P, "apply_CT", s);
  hipLaunchKernelGGL(k_apply_CT, dim3(grid_for(P.g.n, 1 << 20)), dim3(kThreads), 0, s,
                     P.g, u, y);
}

void launch_AAt(const Plan& P, const double* u, double* q, bool reduce_pq, hipStream_t s) {
  if (P.g.has0) aat_launch<true, false>(P, u, nullptr, nullptr, q, false, reduce_pq, s);
  else aat_launch<false, false>(P, u, nullptr, nullptr, q, false, reduce_pq, s);
}

void launch_pdir_AAt(const Plan& P, const double* z, const double* pold, double* pnew, double* q,
                     bool first, hipStream_t s) {
  if (P.g.has0) aat_launch<true, true>(P, z, pold, pnew, q, first, true, s);
  else aat_launch<false, true>(P, z, pold, pnew, q, first, true, s);
}

void launch_prox(const Plan& P, const double* v, double tau, double* y, hipStream_t s) {
  ProfScope ps(P, "prox", s);
  hipLaunchKernelGGL(k_prox, dim3(grid_for(P.g.n, 1 << 20)), dim3(kThreads), 0, s, P.g,
                     v, (const double*)P.V, (const double*)P.VT, tau, y);
}

void launch_terminal_potential(const Plan& P, hipStream_t s) {
  const double w = P.beta > 0.0 ? 1.0 / (P.beta * P.g.dt) : 0.0;
  hipLaunchKernelGGL(k_terminal_potential, dim3(grid_for(P.g.M)), dim3(kThreads), 0, s, P.g.M,
                     (const double*)P.V, (const double*)P.mbar, w, P.VT);
}

void launch_value(const Plan& P, const double* lam, const double* y, double* u, hipStream_t s) {
  const double ib = P.beta > 0.0 ? 1.0 / P.beta : 0.0;
  hipLaunchKernelGGL(k_value, dim3(grid_for(P.g.n + P.g.M)), dim3(kThreads), 0, s, P.g, lam, y,
                     (const double*)P.mbar, ib, u);
}

void launch_hjb_residual(const Plan& P, const double* y, const double* u, double* R,
                         hipStream_t s) {
  ProfScope ps(P, "hjb_residual", s);
  hipLaunchKernelGGL(k_hjb, dim3(grid_for(P.g.n)), dim3(kThreads), 0, s, P.g, y, u,
                     (const double*)P.V, R);
}

BackprojArgs backproj_args(const Plan& P, const double* u, double* xi, double* y, double* ybar,
                           double tau, double theta, const double* tau_dev,
                           const double* theta_dev, double* vout) {
  return BackprojArgs{P.g,      u,         xi,   y,       ybar,    P.V,     P.VT,   tau,    theta,
                      tau_dev,  theta_dev, P.red, vout, nullptr, 0.0, nullptr, nullptr};
}

int backproj_grid(const Plan& P) { return grid_for(P.g.n, P.red.max_blocks); }

template <bool QG>
void backproj_launch(const Geom& g, const BackprojArgs& a, int grid, hipStream_t s) {
  const dim3 gd(grid), bd(kThreads);
  switch (1 + 4 * (g.has0 ? 1 : 0) + g.bcm) {
    case 1: hipLaunchKernelGGL((k_backproj_prox<1, QG>), gd, bd, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_backproj_prox<2, QG>), gd, bd, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_backproj_prox<5, QG>), gd, bd, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_backproj_prox<6, QG>), gd, bd, 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_backproj_prox<7, QG>), gd, bd, 0, s, a); break;
    default: hipLaunchKernelGGL((k_backproj_prox<8, QG>), gd, bd, 0, s, a);
  }
}

void launch_backproj_prox(const Plan& P, const double* u, double* xi, double* y, double* ybar,
                          double tau, double theta, hipStream_t s, double* vout, double* zout,
                          double sigma) {
  const int grid = backproj_grid(P);
  {
    ProfScope ps(P, "backproj_prox", s);
    BackprojArgs a = backproj_args(P, u, xi, y, ybar, tau, theta, nullptr, nullptr, vout);
    a.zout = zout;
    a.sigma = sigma;
    if (P.g.q != 2.0) backproj_launch<true>(P.g, a, grid, s);
    else backproj_launch<false>(P.g, a, grid, s);
  }
  launch_finish(P, T_DM, grid, OP_DM, s);
}

// ---- batched launches (args / offsets are device arrays, see batch_args.h) ----
AatArgs aat_args(const Plan& P, const double* z, const double* pold, double* pnew, double* q,
                 bool first, const double* done, int* grid) {
  int tc;
  *grid = P.g.has0 ? aat_shape<true, kBatchBig>(P, &tc) : aat_shape<false>(P, &tc);
  // nrz is filled in once the inverse time GEMM's grid is known
  return AatArgs{P.g, z, pold, pnew, q, P.red, tc, first ? 1 : 0, 1, done, 0,
                 pcg_flexible(P) ? 1 : 0};
}

int aat_queue_grid(bool has0) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const hipError_t e =
      has0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_AAt_batch_queue<true>,
                                                          Tile<true, kBatchBig>::NT, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_AAt_batch_queue<false>,
                                                          Tile<false, 0>::NT, 0);
  if (e != hipSuccess || per < 1) return 0;
  return cus * per;
}

void launch_aat_batch(bool has0, const AatArgs* A, const int* off, int ninst, int total,
                      hipStream_t s, int* queue, int qgrid) {
  if (queue && qgrid > 0) {
    const int grid = qgrid < total ? qgrid : total;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, queue);
    if (has0)
      hipLaunchKernelGGL(k_AAt_batch_queue<true>, dim3(grid), dim3(Tile<true, kBatchBig>::NT), 0,
                         s, A, off, ninst, total, queue);
    else
      hipLaunchKernelGGL(k_AAt_batch_queue<false>, dim3(grid), dim3(Tile<false, 0>::NT), 0, s,
                         A, off, ninst, total, queue);
    return;
  }
  if (has0)
    hipLaunchKernelGGL(k_AAt_batch<true>, dim3(total), dim3(Tile<true, kBatchBig>::NT), 0, s, A,
                       off, ninst);
  else
    hipLaunchKernelGGL(k_AAt_batch<false>, dim3(total), dim3(Tile<false, 0>::NT), 0, s, A, off,
                       ninst);
}

void launch_rhs_batch(const RhsArgs* A, const int* off, int ninst, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_batch, dim3(total), dim3(kRThreads), 0, s, A, off, ninst);
}

void launch_backproj_batch(const BackprojArgs* A, const int* off, int ninst, int total,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_backproj_prox_batch, dim3(total), dim3(kThreads), 0, s, A, off, ninst);
}

}  // namespace mfg
