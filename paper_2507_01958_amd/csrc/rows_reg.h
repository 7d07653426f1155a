// Row transforms of Algorithm 2 on the register path (axis 1 of length N = 64,
// 128 or 256, contiguous in memory), shared by the row kernels and the fused
// time-GEMM + row-transform kernel.
//
// Two real rows are transformed as one complex line. The rows of a line are
// those of time slices 2 tp and 2 tp + 1 at the same axis-0 index i0
// (line = tp n0 + i0), so a block that owns every time slice of one i0 row
// pairs them the same way as the row kernels do, and both give the same bits.
// The multiply-adds of the transforms are written as explicit fused
// multiply-adds, so the arithmetic does not depend on the kernel the helpers
// are compiled into.
#pragma once

#include "fft_reg.h"

namespace mfg {

template <typename T>
__device__ __forceinline__ const T* tw_table(const Axis& ax);
template <>
__device__ __forceinline__ const double* tw_table<double>(const Axis& ax) { return ax.tw; }
template <>
__device__ __forceinline__ const float* tw_table<float>(const Axis& ax) { return ax.twf; }
template <typename T>
__device__ __forceinline__ const T* ct_table(const Axis& ax);
template <>
__device__ __forceinline__ const double* ct_table<double>(const Axis& ax) { return ax.ct; }
template <>
__device__ __forceinline__ const float* ct_table<float>(const Axis& ax) { return ax.ctf; }

// Makhoul's even/odd reordering of a DCT-II input: position n of the complex
// FFT's input takes element dct_perm(n) of the line.
__device__ __forceinline__ int dct_perm(int n, int N) {
  return (2 * n < N) ? 2 * n : 2 * (N - 1 - n) + 1;
}

// The two rows of register-path line `line` (rows are (t, i0) at t n0 + i0,
// nt = nrows / n0 slices).
struct RowPair {
  int ra, rb;
  bool hasa, hasb;
};
__device__ __forceinline__ RowPair row_pair(int line, int nrows, int n0) {
  const int nt = nrows / n0;
  const int tp = line / n0, i0 = line - tp * n0;
  const int ta = 2 * tp, tb = ta + 1;
  return RowPair{ta * n0 + i0, tb * n0 + i0, ta < nt, tb < nt};
}

// Lines of the register path for nrows = nt n0 rows.
__host__ __device__ inline int reg_lines(int nrows, int n0) {
  const int nt = nrows / n0;
  return ((nt + 1) / 2) * n0;
}

// Forward real transform of one line along the contiguous axis: the DHT
// (periodic) or DCT-II (Neumann, input read in Makhoul order), spectra in
// natural order. Split in two so a caller can synchronise between them (and
// reuse the loads' source as the exchange area): rows_fwd_load takes the
// thread's 16 inputs, ld(n) returning the two rows' elements n as a complex
// value (row a real part, row b imaginary part); rows_fwd_xform transforms
// them and calls st(k, a, b) with the two rows' spectra at k. lds: the line's
// exchange area of fft4; zb: its pairing buffer (Shape::L2 elements). Called by
// every thread of the block.
template <typename T, int N, class LD>
__device__ __forceinline__ void rows_fwd_load(LD ld, bool dct, int p, C2<T> (&v)[16]) {
  using Sh = fftr::Shape<T, N>;
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int n = p + Sh::N2 * n1;
    v[n1] = ld(dct ? dct_perm(n, N) : n);
  }
}

template <typename T, int N, class ST>
__device__ __forceinline__ void rows_fwd_xform(C2<T> (&v)[16], ST st, bool dct, C2<T>* lds,
                                               C2<T>* zb, int p, const T* __restrict__ tw,
                                               const T* __restrict__ ct) {
  using Sh = fftr::Shape<T, N>;
  fftr::fft4<T, N, -1>(v, lds, p, tw);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) zb[p + Sh::N2 * m] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = p + Sh::N2 * m;
    const int kr = k ? N - k : 0;
    const C2<T> z = v[m], zr = zb[kr];
    const T pp = z.x, q = z.y, r = zr.x, s = zr.y;
    T oa, ob;
    if (!dct) {
      oa = (T)0.5 * ((pp + r) - (q - s));
      ob = (T)0.5 * ((q + s) + (pp - r));
    } else {
      const T c = ct[2 * k], sn = ct[2 * k + 1];
      oa = (T)0.5 * fftr::ffma(c, pp + r, sn * (q - s));
      ob = (T)0.5 * fftr::ffma(c, q + s, sn * (r - pp));
    }
    st(k, oa, ob);
  }
}

template <typename T, int N, class LD, class ST>
__device__ __forceinline__ void rows_fwd_line(LD ld, ST st, bool dct, C2<T>* lds, C2<T>* zb,
                                              int p, const T* __restrict__ tw,
                                              const T* __restrict__ ct) {
  C2<T> v[16];
  rows_fwd_load<T, N>(ld, dct, p, v);
  rows_fwd_xform<T, N>(v, st, dct, lds, zb, p, tw, ct);
}

// Inverse real transform of one line along the contiguous axis (times N):
// spectra in, the two rows' values out in v (register m holds position
// n = p + Shape::N2 m of the complex line; with DCT-II it goes to element
// dct_perm(n) of the rows). The complex input of the inverse FFT is formed
// from the pair (k, N - k): DHT: Re F = (H[k] + H[N-k])/2,
// Im F = (H[N-k] - H[k])/2; DCT-II: V[k] = exp(i pi k/(2N)) (C[k] - i C[N-k]).
// ld(k) returns the two rows' spectra at k (row a real part, row b imaginary
// part). lds: the line's exchange area of fft4. Called by every thread of the
// block.
template <typename T, int N, class LD>
__device__ __forceinline__ void rows_inv_line(LD ld, bool dct, C2<T>* lds, int p,
                                              const T* __restrict__ tw,
                                              const T* __restrict__ ct, C2<T> (&v)[16]) {
  using Sh = fftr::Shape<T, N>;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = p + Sh::N2 * m;
    const int kr = k ? N - k : 0;
    const C2<T> cz = ld(k), rz = ld(kr);
    const T ca = cz.x, cb = cz.y;
    T ra_ = rz.x, rb_ = rz.y;
    if (!dct) {
      const T fa_re = (T)0.5 * (ca + ra_), fa_im = (T)0.5 * (ra_ - ca);
      const T fb_re = (T)0.5 * (cb + rb_), fb_im = (T)0.5 * (rb_ - cb);
      v[m] = C2<T>{fa_re - fb_im, fa_im + fb_re};
    } else {
      if (k == 0) {
        ra_ = (T)0;
        rb_ = (T)0;
      }
      const T c = ct[2 * k], sn = ct[2 * k + 1];
      v[m].x = fftr::ffma(c, ca, sn * ra_) - fftr::ffma(sn, cb, -(c * rb_));
      v[m].y = fftr::ffma(sn, ca, -(c * ra_)) + fftr::ffma(c, cb, sn * rb_);
    }
  }
  fftr::fft4<T, N, +1>(v, lds, p, tw);
}

}  // namespace mfg
