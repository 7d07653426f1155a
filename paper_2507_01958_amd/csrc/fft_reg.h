// Register-resident complex FFTs for the spatial transforms of Algorithm 2 on
// axes of length N = 64, 128 or 256.
//
// Four-step form N = N1 * N2 with N1 = 16 and N2 = N / 16 threads per line:
// thread p of a line holds the 16 elements x[p + N2 n1] (n1 = 0..15), takes a
// 16-point DFT in registers, multiplies by W_N^(p k1), and exchanges through
// LDS once; then each thread takes 16 / N2 DFTs of length N2 (over n2, for
// k1 = p + N2 h) and ends up holding X[p + N2 m], m = 0..15 -- the same
// distribution as its input, so a forward and an inverse transform chain
// without further data movement. X[k] = sum_n x[n] exp(SIGN 2 pi i n k / N),
// unnormalised.
//
// LDS layout of the exchange: per line, element (k1, n2) at k1 * S + n2 with
// row stride S and line stride L; the pairing buffer (element k of a line at
// k, line stride L2). They were chosen, by exhaustive count over the lanes of
// each access, to be free of bank conflicts for 16-byte (float64 complex) and
// 8-byte (float32 complex) accesses served 128 bytes (32 banks of 4 bytes) at
// a time, which is how gfx950 behaves for these accesses (the hardware's
// SQ_LDS_BANK_CONFLICT counter reads zero on them and flagged an earlier
// layout that was conflict-free only for 256 bytes at a time).
#pragma once

#include "mfg_internal.h"

namespace mfg {

template <typename T>
struct C2 {
  T x, y;
};

namespace fftr {

template <typename T>
__device__ __forceinline__ C2<T> add(C2<T> a, C2<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ C2<T> sub(C2<T> a, C2<T> b) {
  return {a.x - b.x, a.y - b.y};
}
// a b + c with one rounding (written out, so the result does not depend on
// the compiler's contraction choices in the kernel it is compiled into)
__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a * (c + i s)
template <typename T>
__device__ __forceinline__ C2<T> mul(C2<T> a, T c, T s) {
  return {ffma(a.x, c, -(a.y * s)), ffma(a.x, s, a.y * c)};
}
// a * (SIGN i)
template <int SIGN, typename T>
__device__ __forceinline__ C2<T> rot90(C2<T> a) {
  return SIGN < 0 ? C2<T>{a.y, -a.x} : C2<T>{-a.y, a.x};
}

// cos and sin of 2 pi m / 16, m = 0..7 (exact values: cos(pi/8) =
// sqrt(2 + sqrt 2)/2, sin(pi/8) = sqrt(2 - sqrt 2)/2, cos(pi/4) = sqrt(2)/2).
constexpr double kC1 = 0.92387953251128675612818318939678829;
constexpr double kS1 = 0.38268343236508977172845998403039887;
constexpr double kR2 = 0.70710678118654752440084436210484904;

// a * exp(SIGN 2 pi i m / 16), m a compile-time constant after unrolling.
template <int SIGN, typename T>
__device__ __forceinline__ C2<T> w16(C2<T> a, int m) {
  const T sg = (T)SIGN;
  switch (m) {
    case 0: return a;
    case 1: return mul(a, (T)kC1, sg * (T)kS1);
    case 2: return mul(a, (T)kR2, sg * (T)kR2);
    case 3: return mul(a, (T)kS1, sg * (T)kC1);
    case 4: return rot90<SIGN>(a);
    case 5: return mul(a, -(T)kS1, sg * (T)kC1);
    case 6: return mul(a, -(T)kR2, sg * (T)kR2);
    default: return mul(a, -(T)kC1, sg * (T)kS1);
  }
}

// In-place DFT of R = 1, 2, 4, 8, 16 points, natural order in and out.
template <int R, int SIGN, typename T>
__device__ __forceinline__ void dft(C2<T>* v) {
  if constexpr (R == 2) {
    const C2<T> a = v[0];
    v[0] = add(a, v[1]);
    v[1] = sub(a, v[1]);
  } else if constexpr (R == 4) {
    const C2<T> t0 = add(v[0], v[2]), t1 = sub(v[0], v[2]);
    const C2<T> t2 = add(v[1], v[3]), t3 = rot90<SIGN>(sub(v[1], v[3]));
    v[0] = add(t0, t2);
    v[2] = sub(t0, t2);
    v[1] = add(t1, t3);
    v[3] = sub(t1, t3);
  } else if constexpr (R >= 8) {
    C2<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<R / 2, SIGN>(e);
    dft<R / 2, SIGN>(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const C2<T> t = w16<SIGN>(o[k], (16 / R) * k);
      v[k] = add(e[k], t);
      v[k + R / 2] = sub(e[k], t);
    }
  }
}

// LF selects the thread mapping: false, p fastest (thread = line * N2 + p; the
// row transforms, where a line is contiguous in memory); true, line fastest
// (thread = p * LPB + line; the column solves, where the lines of a block are
// adjacent columns, so one load instruction covers whole 128-byte row
// segments). Each mapping has its own conflict-free strides.
template <typename T, int N, bool LF = false>
struct Shape {
  static constexpr int N1 = 16;
  static constexpr int N2 = N / 16;          // threads per line
  static constexpr int NT = sizeof(T) == 8 ? 128 : 256;  // threads per block
  static constexpr int LPB = NT / N2;        // complex lines per block
  static constexpr int S = LF ? N2 : N2 + 1;
  static constexpr int L = LF ? N + 1 : 16 * S + (N2 == 16 ? 0 : N2);
  static constexpr int L2 = LF ? N + 1 : N + ((N2 == 16 && sizeof(T) == 8) ? 0 : N2);
  static constexpr int BUF = LPB * (L > L2 ? L : L2);  // complex elements of LDS
  __device__ static __forceinline__ int line(int tid) { return LF ? tid % LPB : tid / N2; }
  __device__ static __forceinline__ int pos(int tid) { return LF ? tid / LPB : tid % N2; }
};

// True for the axis lengths with a register path.
__host__ __device__ constexpr bool has_reg_path(int N) { return N == 64 || N == 128 || N == 256; }

// Four-step FFT of one line: v[n1] = x[p + N2 n1] in, v[m] = X[p + N2 m] out.
// lds: this line's exchange area (Shape::L complex elements); tw: cos/sin of
// 2 pi m / N, m = 0..N-1 (interleaved). Called by every thread of the block
// (contains a barrier); the caller synchronises before reusing lds.
template <typename T, int N, int SIGN, bool LF = false>
__device__ __forceinline__ void fft4(C2<T>* v, C2<T>* lds, int p, const T* __restrict__ tw) {
  using Sh = Shape<T, N, LF>;
  dft<16, SIGN>(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) {
    const int m = p * k1;
    v[k1] = mul(v[k1], tw[2 * m], (T)SIGN * tw[2 * m + 1]);
  }
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) lds[k1 * Sh::S + p] = v[k1];
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 16 / Sh::N2; ++h) {
    C2<T> b[Sh::N2];
    const int k1 = p + Sh::N2 * h;
#pragma unroll
    for (int n2 = 0; n2 < Sh::N2; ++n2) b[n2] = lds[k1 * Sh::S + n2];
    dft<Sh::N2, SIGN>(b);
#pragma unroll
    for (int k2 = 0; k2 < Sh::N2; ++k2) v[h + (16 / Sh::N2) * k2] = b[k2];
  }
}

}  // namespace fftr
}  // namespace mfg
