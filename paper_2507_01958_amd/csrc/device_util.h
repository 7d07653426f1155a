// Device helpers: neighbour index maps, wave64 / block reductions and the
// deterministic last-block reduction.
#pragma once

#include "mfg_internal.h"

namespace mfg {



// Neighbour index along an axis of n nodes. Periodic: indices mod n (Section 2).
// Neumann: half-sample reflection (-1 -> 0, n -> n-1), which reproduces the
// Section 4.3 Laplacian whose corner entries are 1, and makes the transposed
// one-sided differences vanish at the boundary.
__device__ __forceinline__ int nbr(int p, int n, int neumann) {
  if (neumann) {
    if (p < 0) p = -1 - p;
    else if (p >= n) p = 2 * n - 1 - p;
    p = p < 0 ? 0 : (p >= n ? n - 1 : p);
    return p;
  }
  p %= n;
  return p < 0 ? p + n : p;
}

// nbr for a tile row or column p >= -2 whose value is needed only when
// p <= n + 1 (two-node halo of a tile that may run past the end of the axis):
// exact there, some valid index beyond (no division). Needs n >= 2.
__device__ __forceinline__ int nbr_tile(int p, int n, int neumann) {
  if (p < 0) return neumann ? -1 - p : p + n;
  if (p < n) return p;
  if (p >= n + 2) return 0;
  return neumann ? 2 * n - 1 - p : p - n;
}

// nbr for a direct neighbour of a node, p in [-1, n] (no division).
__device__ __forceinline__ int nbr1(int p, int n, int neumann) {
  if (p < 0) return neumann ? 0 : n - 1;
  if (p >= n) return neumann ? n - 1 : 0;
  return p;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum NV values over the block; the result is valid in thread 0 only.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * 16 + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[k * 16 + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Store this block's partial sums (slot k of `site` at index bid, the block's
// id within its instance).
// A later kernel (a one-block finisher, or the consumer through
// fold_partials) sums them after the producing kernel has completed, so no
// device-scope fence is needed here (on a multi-XCD part such a fence writes
// back the whole L2 of the XCD).
template <int NV>
__device__ __forceinline__ void reduce_store(double (&v)[NV], const RedBuf& rb, int site,
                                             int bid) {
  static_assert(NV <= kSlotsPerSite, "too many reduction slots");
  __shared__ double sh[NV * 16];
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0) {
    double* part = rb.partials + (size_t)site * kSlotsPerSite * rb.max_blocks;
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(size_t)k * rb.max_blocks + bid] = v[k];
  }
}

__device__ __forceinline__ bool finite_d(double x) { return __builtin_isfinite(x); }

// The sums of slots 0..NV-1 of a site's first n partials, formed inside the
// kernel that consumes them (in place of a one-block finisher launch between
// producer and consumer). Wave 0 adds entries lane, lane + 64, ... in order
// and combines the 64 lane sums by a butterfly, so the result depends only on
// n: every block, whatever its size, gets the same bits. Broadcast to the
// block through LDS; every thread of the block must call it.
template <int NV>
__device__ __forceinline__ void fold_partials(const RedBuf& rb, int site, int n,
                                              double (&out)[NV]) {
  __shared__ double sh[NV];
  if (threadIdx.x < 64) {
    const double* part = rb.partials + (size_t)site * kSlotsPerSite * rb.max_blocks;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < n; b += 64) {
#pragma unroll
      for (int k = 0; k < NV; ++k) v[k] += part[(size_t)k * rb.max_blocks + b];
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) sh[k] = v[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = sh[k];
  __syncthreads();
}

// The PCG stopping test on r.r, taken by the kernel that next reads r (the
// preconditioner's first pass) instead of a finisher launch. Every block sums
// the n partials (same bits everywhere); block 0 records r.r, counts the
// iteration and sets S_DONE on convergence (r.r <= tol^2 b.b), a non-finite
// r.r or an earlier breakdown. Returns true when the solve is over. Every
// thread of the block must call it.
__device__ __forceinline__ bool rr_check(const RedBuf& rb, int n, int bid) {
  double rr[1];
  fold_partials<1>(rb, T_RR, n, rr);
  const double* S = rb.scal;
  const bool bad = !finite_d(rr[0]);
  const bool done = bad || S[S_BAD] != 0.0 || rr[0] <= S[S_TOL2] * S[S_BB];
  if (bid == 0 && threadIdx.x == 0) {
    double* Sw = rb.scal;
    Sw[S_RR] = rr[0];
    Sw[S_ITS] += 1.0;
    if (bad) Sw[S_BAD] = 2.0;
    if (done) Sw[S_DONE] = 1.0;
  }
  return done;
}

// XCD-aware block order: blocks b and b+8 run on the same XCD, so map them to
// neighbouring logical tiles (shared cache lines and halos stay in one L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int full = nb & ~7;
  if (b >= full) return b;
  const int per = full >> 3;
  return (b & 7) * per + (b >> 3);
}

}  // namespace mfg
