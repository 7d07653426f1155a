// Parallel-in-time preconditioner P^{-1} of eq. pstrec:
//   P^{-1} = (V^T (x) T^{-1}) (I (x) Lambda_1 + Lambda_t (x) Lambda_2)^{-1} (V (x) T)
// Algorithm 1: the time transform V (DCT-VIII for l = 1, DST-I for l = 2) is a
// dense N_t x N_t matrix applied to every spatial node: a GEMM on the matrix
// cores. Algorithm 2: per time step k the spatial system
// (C-hat + lambda_k L-hat) x = y is diagonalised by a real transform T along
// each axis and divided entrywise by
//   S = nu^2 R^2 + 2R + (nu lambda_k/dt) R + lambda_k/dt^2,
//   R = lambda_x/dx^2 + lambda_y/dy^2.
// T is the discrete Hartley transform on a periodic axis (its basis vectors
// cos + sin diagonalise the symmetric circulant Laplacian with the DFT's
// eigenvalues, and it is real and self-inverse up to 1/N), and the DCT-II on a
// Neumann axis. Both are computed from one complex FFT per pair of real lines
// (DCT-II by Makhoul's even/odd reordering), with a mixed-radix (4, 2, 3)
// Stockham FFT staged in LDS.
#include "batch_args.h"
#include "device_util.h"
#include "fft_reg.h"
#include "rows_reg.h"
#include "plan.h"
#include "tgemm.h"

namespace mfg {

namespace {

constexpr int kLoadBatch = 8;  // global loads per thread issued before their LDS stores

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, T c, T s) {
  return {a.x * c - a.y * s, a.x * s + a.y * c};
}

// Complex FFT of nlines lines of length ax.N held in LDS buffer a (b is the
// ping-pong partner). sign = -1 forward, +1 inverse (unnormalised). Returns the
// buffer that holds the result. Must be called by the whole block.
template <typename T>
__device__ C2<T>* fft_lds(C2<T>* a, C2<T>* b, int nlines, const Axis& ax, const T* tw, int sign) {
  const int N = ax.N;
  const T sg = (T)sign;
  int Ns = 1;
  for (int ps = 0; ps < ax.npass; ++ps) {
    const int R = ax.radix[ps];
    const int nb = N / R;
    const int tws = N / (Ns * R);
    const int total = nlines * nb;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int line = idx / nb;
      const int j = idx - line * nb;
      const C2<T>* in = a + line * N;
      C2<T>* out = b + line * N;
      const int k = j % Ns;
      const int base = (j / Ns) * Ns * R + k;
      if (R == 4) {
        C2<T> v0 = in[j], v1 = in[j + nb], v2 = in[j + 2 * nb], v3 = in[j + 3 * nb];
        if (k) {
          const int m = k * tws;
          v1 = cmul(v1, tw[2 * m], sg * tw[2 * m + 1]);
          v2 = cmul(v2, tw[4 * m], sg * tw[4 * m + 1]);
          v3 = cmul(v3, tw[6 * m], sg * tw[6 * m + 1]);
        }
        const C2<T> t0 = {v0.x + v2.x, v0.y + v2.y};
        const C2<T> t1 = {v0.x - v2.x, v0.y - v2.y};
        const C2<T> t2 = {v1.x + v3.x, v1.y + v3.y};
        const C2<T> d = {v1.x - v3.x, v1.y - v3.y};
        const C2<T> t3 = {-sg * d.y, sg * d.x};  // (sign i) * d
        out[base] = {t0.x + t2.x, t0.y + t2.y};
        out[base + Ns] = {t1.x + t3.x, t1.y + t3.y};
        out[base + 2 * Ns] = {t0.x - t2.x, t0.y - t2.y};
        out[base + 3 * Ns] = {t1.x - t3.x, t1.y - t3.y};
      } else if (R == 2) {
        C2<T> v0 = in[j], v1 = in[j + nb];
        if (k) {
          const int m = k * tws;
          v1 = cmul(v1, tw[2 * m], sg * tw[2 * m + 1]);
        }
        out[base] = {v0.x + v1.x, v0.y + v1.y};
        out[base + Ns] = {v0.x - v1.x, v0.y - v1.y};
      } else {  // R == 3
        C2<T> v0 = in[j], v1 = in[j + nb], v2 = in[j + 2 * nb];
        if (k) {
          const int m = k * tws;
          v1 = cmul(v1, tw[2 * m], sg * tw[2 * m + 1]);
          v2 = cmul(v2, tw[4 * m], sg * tw[4 * m + 1]);
        }
        const T h = (T)0.8660254037844386467637231707529362;  // sqrt(3)/2
        const C2<T> s = {v1.x + v2.x, v1.y + v2.y};
        const C2<T> d = {v1.x - v2.x, v1.y - v2.y};
        const C2<T> m0 = {v0.x - (T)0.5 * s.x, v0.y - (T)0.5 * s.y};
        const C2<T> rot = {-sg * h * d.y, sg * h * d.x};  // (sign i sqrt3/2) d
        out[base] = {v0.x + s.x, v0.y + s.y};
        out[base + Ns] = {m0.x + rot.x, m0.y + rot.y};
        out[base + 2 * Ns] = {m0.x - rot.x, m0.y - rot.y};
      }
    }
    __syncthreads();
    C2<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// Makhoul's reordering for the DCT-II: v[n] = x[perm(n)].
// Real spectra of the two packed real lines from their complex FFT Z.
// DHT: H_a = (p + r - q + s)/2, H_b = (q + s + p - r)/2 with Z[k] = p + iq,
// Z[N-k] = r + is.  DCT-II: C = Re(e^{-i pi k/(2N)} V[k]) of each line.
template <typename T>
__device__ void post_forward(const C2<T>* Z, C2<T>* out, int nlines, const Axis& ax, const T* ct) {
  const int N = ax.N;
  for (int idx = threadIdx.x; idx < nlines * N; idx += blockDim.x) {
    const int line = idx / N, k = idx - line * N;
    const int kr = (k == 0) ? 0 : N - k;
    const C2<T> a = Z[line * N + k], b = Z[line * N + kr];
    const T p = a.x, q = a.y, r = b.x, s = b.y;
    C2<T> o;
    if (ax.kind == 0) {
      o.x = (T)0.5 * ((p + r) - (q - s));
      o.y = (T)0.5 * ((q + s) + (p - r));
    } else {
      const T c = ct[2 * k], sn = ct[2 * k + 1];
      o.x = (T)0.5 * (c * (p + r) + sn * (q - s));
      o.y = (T)0.5 * (c * (q + s) + sn * (r - p));
    }
    out[line * N + k] = o;
  }
  __syncthreads();
}

// Complex spectrum for the inverse DCT-II of two packed real spectra:
// V[k] = e^{i pi k/(2N)} (C[k] - i C[N-k]) per line, Z = V_a + i V_b.
template <typename T>
__device__ void pre_inverse_dct(const C2<T>* Cin, C2<T>* Z, int nlines, const Axis& ax,
                                const T* ct) {
  const int N = ax.N;
  for (int idx = threadIdx.x; idx < nlines * N; idx += blockDim.x) {
    const int line = idx / N, k = idx - line * N;
    const C2<T> cur = Cin[line * N + k];
    const C2<T> rev = (k == 0) ? C2<T>{(T)0, (T)0} : Cin[line * N + N - k];
    const T c = ct[2 * k], sn = ct[2 * k + 1];
    C2<T> o;
    o.x = c * cur.x + sn * rev.x - (sn * cur.y - c * rev.y);
    o.y = (sn * cur.x - c * rev.x) + c * cur.y + sn * rev.y;
    Z[line * N + k] = o;
  }
  __syncthreads();
}

// Inverse real transform of spectra held in `buf` (re = line a, im = line b);
// returns the buffer with the (unnormalised, times N) spatial lines in natural
// order for the DHT, or in Makhoul order for the DCT (caller applies dct_perm).
template <typename T>
__device__ C2<T>* inverse_real(C2<T>* buf, C2<T>* other, int nlines, const Axis& ax,
                               const T* tw, const T* ct) {
  if (ax.kind == 0) {
    C2<T>* z = fft_lds<T>(buf, other, nlines, ax, tw, -1);
    C2<T>* o = (z == buf) ? other : buf;
    post_forward<T>(z, o, nlines, ax, ct);
    return o;
  }
  pre_inverse_dct<T>(buf, other, nlines, ax, ct);
  return fft_lds<T>(other, buf, nlines, ax, tw, +1);
}

// Copy the axis' twiddle (cos/sin 2 pi m/N) and DCT (cos/sin pi k/2N) tables
// into LDS; returns pointers through tw and ct.
template <typename T>
__device__ void stage_tables(const Axis& ax, T* lds, const T*& tw, const T*& ct) {
  const int N = ax.N;
  const T* gtw = tw_table<T>(ax);
  const T* gct = ct_table<T>(ax);
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
    lds[i] = gtw[i];
    lds[2 * N + i] = gct[i];
  }
  tw = lds;
  ct = lds + 2 * N;
}



__device__ __forceinline__ double shift_symbol(const SolveCtx& sc, double R, double lt) {
  return sc.nu * sc.nu * R * R + 2.0 * R + (sc.nu * lt * sc.idt) * R + lt * sc.idt2;
}

// Transforms along the contiguous axis (length N = ax.N) of nrows rows.
// mode 0: forward; 1: inverse; 2: forward, divide by S (d = 1), inverse.
template <typename T>
__device__ void rows_body(const RowsArgs<T>& a, int bid) {
  if (a.done && *a.done != 0.0) return;
  T* __restrict__ data = a.data;
  const int nrows = a.nrows, mode = a.mode, lpb = a.lpb, n0 = a.n0;
  const Axis& ax = a.ax;
  const SolveCtx& sc = a.sc;
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = ax.N;
  C2<T>* A = reinterpret_cast<C2<T>*>(smem);
  C2<T>* B = A + lpb * N;
  const T *tw, *ct;
  stage_tables<T>(ax, reinterpret_cast<T*>(B + lpb * N), tw, ct);
  const int line0 = bid * lpb;
  int nl = (nrows + 1) / 2 - line0;
  if (nl > lpb) nl = lpb;
  const bool dct = (ax.kind == 1);
  // load: batches of kLoadBatch elements per thread in flight before the LDS
  // stores (blockDim.x == 256)
  {
    const int total = nl * N;
    for (int base = 0; base < total; base += 256 * kLoadBatch) {
      T va[kLoadBatch], vb[kLoadBatch];
#pragma unroll
      for (int e = 0; e < kLoadBatch; ++e) {
        const int idx = base + threadIdx.x + 256 * e;
        va[e] = (T)0;
        vb[e] = (T)0;
        if (idx < total) {
          const int l = idx / N, n = idx - l * N;
          const int ra = 2 * (line0 + l), rb = ra + 1;
          const int src = (mode != 1 && dct) ? dct_perm(n, N) : n;
          va[e] = data[(size_t)ra * N + src];
          if (rb < nrows) vb[e] = data[(size_t)rb * N + src];
        }
      }
#pragma unroll
      for (int e = 0; e < kLoadBatch; ++e) {
        const int idx = base + threadIdx.x + 256 * e;
        if (idx < total) A[idx] = C2<T>{va[e], vb[e]};
      }
    }
  }
  __syncthreads();
  C2<T>* res;
  if (mode == 1) {
    res = inverse_real<T>(A, B, nl, ax, tw, ct);
  } else {
    C2<T>* z = fft_lds<T>(A, B, nl, ax, tw, -1);
    C2<T>* o = (z == A) ? B : A;
    post_forward<T>(z, o, nl, ax, ct);
    if (mode == 0) {
      res = o;
    } else {
      // divide (d = 1: rows are time slices, n0 == 1)
      for (int idx = threadIdx.x; idx < nl * N; idx += blockDim.x) {
        const int l = idx / N, k = idx - l * N;
        const int ra = 2 * (line0 + l), rb = ra + 1;
        const double R = sc.lam1[k];
        const double sa = shift_symbol(sc, R, sc.lam_t[ra / n0]);
        const double sb = (rb < nrows) ? shift_symbol(sc, R, sc.lam_t[rb / n0]) : 1.0;
        C2<T> v = o[idx];
        v.x = (T)((double)v.x * (sc.norm / sa));
        v.y = (T)((double)v.y * (sc.norm / sb));
        o[idx] = v;
      }
      __syncthreads();
      res = inverse_real<T>(o, (o == A) ? B : A, nl, ax, tw, ct);
    }
  }
  // store
  const bool permute_out = (mode != 0) && dct;
  for (int idx = threadIdx.x; idx < nl * N; idx += blockDim.x) {
    const int l = idx / N, n = idx - l * N;
    const int ra = 2 * (line0 + l), rb = ra + 1;
    const int dst = permute_out ? dct_perm(n, N) : n;
    const C2<T> v = res[idx];
    data[(size_t)ra * N + dst] = v.x;
    if (rb < nrows) data[(size_t)rb * N + dst] = v.y;
  }
}

// Transform along axis 0 (stride n1), divide by S, inverse along axis 0, for
// cw columns of one time slice per block (d = 2).
template <typename T>
__device__ void cols_body(const ColsArgs<T>& a, int bid, int nb) {
  if (a.done && *a.done != 0.0) return;
  T* __restrict__ data = a.data;
  const Geom& g = a.g;
  const Axis& ax = a.ax;
  const int cw = a.cw;
  const SolveCtx& sc = a.sc;
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = ax.N;  // == n0
  const int nlines = cw / 2;
  C2<T>* A = reinterpret_cast<C2<T>*>(smem);
  C2<T>* B = A + nlines * N;
  const T *tw, *ct;
  stage_tables<T>(ax, reinterpret_cast<T*>(B + nlines * N), tw, ct);
  const int ncb = (g.n1 + cw - 1) / cw;
  const int blk = xcd_remap(bid, nb);
  const int t = blk / ncb;
  const int j0 = (blk - t * ncb) * cw;
  const bool dct = (ax.kind == 1);
  T* slice = data + (size_t)t * g.M;
  {
    const int total = N * cw;
    for (int base = 0; base < total; base += 256 * kLoadBatch) {
      T v[kLoadBatch];
#pragma unroll
      for (int e = 0; e < kLoadBatch; ++e) {
        const int idx = base + threadIdx.x + 256 * e;
        v[e] = (T)0;
        if (idx < total) {
          const int i = idx / cw, jj = idx - i * cw;
          const int j = j0 + jj;
          if (j < g.n1) v[e] = slice[(size_t)i * g.n1 + j];
        }
      }
#pragma unroll
      for (int e = 0; e < kLoadBatch; ++e) {
        const int idx = base + threadIdx.x + 256 * e;
        if (idx < total) {
          const int i = idx / cw, jj = idx - i * cw;
          // position along the line: Makhoul order for the DCT (inverse of
          // dct_perm: element i goes to position n with perm(n) = i)
          const int n = dct ? ((i & 1) ? (N - 1 - (i >> 1)) : (i >> 1)) : i;
          T* dst = reinterpret_cast<T*>(&A[(jj >> 1) * N + n]);
          dst[jj & 1] = v[e];
        }
      }
    }
  }
  __syncthreads();
  C2<T>* z = fft_lds<T>(A, B, nlines, ax, tw, -1);
  C2<T>* o = (z == A) ? B : A;
  post_forward<T>(z, o, nlines, ax, ct);
  const double lt = sc.lam_t[t];
  for (int idx = threadIdx.x; idx < nlines * N; idx += blockDim.x) {
    const int l = idx / N, k = idx - l * N;
    const int ja = j0 + 2 * l, jb = ja + 1;
    const double R0 = sc.lam0[k];
    const double sa = (ja < g.n1) ? shift_symbol(sc, R0 + sc.lam1[ja], lt) : 1.0;
    const double sb = (jb < g.n1) ? shift_symbol(sc, R0 + sc.lam1[jb], lt) : 1.0;
    C2<T> v = o[idx];
    v.x = (T)((double)v.x * (sc.norm / sa));
    v.y = (T)((double)v.y * (sc.norm / sb));
    o[idx] = v;
  }
  __syncthreads();
  C2<T>* res = inverse_real<T>(o, (o == A) ? B : A, nlines, ax, tw, ct);
  for (int idx = threadIdx.x; idx < N * cw; idx += blockDim.x) {
    const int i = idx / cw, jj = idx - i * cw;
    const int j = j0 + jj;
    if (j >= g.n1) continue;
    int n;
    if (dct) n = (i & 1) ? (N - 1 - (i >> 1)) : (i >> 1);
    else n = i;
    const C2<T> v = res[(jj >> 1) * N + n];
    slice[(size_t)i * g.n1 + j] = (jj & 1) ? v.y : v.x;
  }
}

// ---- register path (axis length 64, 128 or 256; see fft_reg.h) ----
// A complex line packs two real lines (real and imaginary parts); thread p of
// line l holds the elements p + N2 m. Threads of lines past the end take part
// in the barriers with zeros and store nothing.

template <typename T>
using V2 = T __attribute__((ext_vector_type(2)));

// Forward real transform along the contiguous axis: DHT (periodic) or DCT-II
// (Neumann, input read in Makhoul order), spectra stored in natural order.
template <typename T, int N>
__device__ void rows_fwd_reg(const RowsArgs<T>& a, int bid, C2<T>* lds) {
  using Sh = fftr::Shape<T, N>;
  const int l = threadIdx.x / Sh::N2, p = threadIdx.x % Sh::N2;
  const RowPair rp = row_pair(bid * Sh::LPB + l, a.nrows, a.n0);
  T* __restrict__ data = a.data;
  // n < 2^31: 32-bit offsets
  auto ld = [&](int n) {
    return C2<T>{rp.hasa ? data[(unsigned)rp.ra * N + n] : (T)0,
                 rp.hasb ? data[(unsigned)rp.rb * N + n] : (T)0};
  };
  auto st = [&](int k, T oa, T ob) {
    if (rp.hasa) data[(unsigned)rp.ra * N + k] = oa;
    if (rp.hasb) data[(unsigned)rp.rb * N + k] = ob;
  };
  rows_fwd_line<T, N>(ld, st, a.ax.kind == 1, lds + l * Sh::L, lds + l * Sh::L2, p,
                      tw_table<T>(a.ax), ct_table<T>(a.ax));
}

// Inverse real transform along the contiguous axis (rows_inv_line), lines out
// in natural order.
template <typename T, int N>
__device__ void rows_inv_reg(const RowsArgs<T>& a, int bid, C2<T>* lds) {
  using Sh = fftr::Shape<T, N>;
  const int l = threadIdx.x / Sh::N2, p = threadIdx.x % Sh::N2;
  const RowPair rp = row_pair(bid * Sh::LPB + l, a.nrows, a.n0);
  const int ra = rp.ra, rb = rp.rb;
  const bool hasa = rp.hasa, hasb = rp.hasb;
  const bool dct = a.ax.kind == 1;
  T* __restrict__ data = a.data;
  C2<T> v[16];
  // n < 2^31: 32-bit offsets
  rows_inv_line<T, N>(
      [&](int k) {
        return C2<T>{hasa ? data[(unsigned)ra * N + k] : (T)0,
                     hasb ? data[(unsigned)rb * N + k] : (T)0};
      },
      dct, lds + l * Sh::L, p, tw_table<T>(a.ax), ct_table<T>(a.ax), v);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int n = p + Sh::N2 * m;
    const int dst = dct ? dct_perm(n, N) : n;
    if (hasa) data[(unsigned)ra * N + dst] = v[m].x;
    if (hasb) data[(unsigned)rb * N + dst] = v[m].y;
  }
}

// 1/x from the hardware reciprocal refined by Newton steps (two in float64,
// one in float32): within an ulp of the correctly rounded quotient.
template <typename T>
__device__ __forceinline__ T recip(T x);
template <>
__device__ __forceinline__ double recip<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <>
__device__ __forceinline__ float recip<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// The shifted symbol of Algorithm 2 for one time slice as a polynomial in R:
// S = nu^2 R^2 + (2 + nu lambda_t/dt) R + lambda_t/dt^2 (> 0), and the scale
// norm / S applied to a spectral coefficient.
template <typename T>
struct SliceSymbol {
  T a2, b, c, norm;
  __device__ SliceSymbol(const SolveCtx& sc, double lt)
      : a2((T)(sc.nu * sc.nu)), b((T)(2.0 + sc.nu * lt * sc.idt)), c((T)(lt * sc.idt2)),
        norm((T)sc.norm) {}
  __device__ __forceinline__ T inv(T R) const {
    return norm * recip<T>(fma(fma(a2, R, b), R, c));
  }
};

// Column solve along axis 0 (length N = n0, stride n1) of one time slice:
// forward transform, division by S, inverse transform; two real columns per
// complex line. Periodic: DFT with the two columns' spectra separated by
// Z_a = (Z[k] + conj Z[N-k])/2, Z_b = (Z[k] - conj Z[N-k])/(2i) (S is even in
// k). Neumann: DCT-II via Makhoul's reordering; both C[k] and C[N-k] are
// formed from the pair (Z[k], Z[N-k]) so the inverse input needs no second
// exchange.
// One column tile of the register path: two columns (ja, ja + 1) of slice t
// per line, 2 LPB adjacent columns per tile.
struct ColTile {
  int t, ja;
  bool hasa, hasb, pair_ld;
};

template <typename T, int N>
__device__ __forceinline__ ColTile col_tile(const ColsArgs<T>& a, int blk) {
  using Sh = fftr::Shape<T, N, true>;
  const Geom& g = a.g;
  const int l = Sh::line(threadIdx.x);
  const int cw = 2 * Sh::LPB;
  const int ncb = (g.n1 + cw - 1) / cw;
  ColTile c;
  c.t = blk / ncb;
  c.ja = (blk - c.t * ncb) * cw + 2 * l;
  c.hasa = c.ja < g.n1;
  c.hasb = c.ja + 1 < g.n1;
  c.pair_ld = c.hasb && ((g.n1 & 1) == 0);  // 2-element aligned vector access
  return c;
}

// The tile's inputs.
template <typename T, int N>
__device__ __forceinline__ void cols_load(const ColsArgs<T>& a, const ColTile& c,
                                          C2<T> (&v)[16]) {
  using Sh = fftr::Shape<T, N, true>;
  const int p = Sh::pos(threadIdx.x);
  const bool dct = a.ax.kind == 1;
  const unsigned n1s = (unsigned)a.g.n1;
  const T* __restrict__ slice = a.data + (size_t)c.t * a.g.M;
  // 32-bit offsets within the slice (M < 2^31); the column-pair test is
  // uniform, so each form is one straight run of loads
  if (c.pair_ld) {
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
      const int n = p + Sh::N2 * n1;
      const unsigned o = (unsigned)(dct ? dct_perm(n, N) : n) * n1s + (unsigned)c.ja;
      const V2<T> w = *reinterpret_cast<const V2<T>*>(slice + o);
      v[n1] = C2<T>{w.x, w.y};
    }
  } else {
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
      const int n = p + Sh::N2 * n1;
      const unsigned o = (unsigned)(dct ? dct_perm(n, N) : n) * n1s + (unsigned)c.ja;
      v[n1].x = c.hasa ? slice[o] : (T)0;
      v[n1].y = c.hasb ? slice[o + 1] : (T)0;
    }
  }
}

template <typename T, int N>
__device__ __forceinline__ void cols_store(const ColsArgs<T>& a, const ColTile& c,
                                           const C2<T> (&v)[16]) {
  using Sh = fftr::Shape<T, N, true>;
  const int p = Sh::pos(threadIdx.x);
  const bool dct = a.ax.kind == 1;
  const unsigned n1s = (unsigned)a.g.n1;
  T* __restrict__ slice = a.data + (size_t)c.t * a.g.M;
  if (c.pair_ld) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int n = p + Sh::N2 * m;
      const unsigned o = (unsigned)(dct ? dct_perm(n, N) : n) * n1s + (unsigned)c.ja;
      *reinterpret_cast<V2<T>*>(slice + o) = V2<T>{v[m].x, v[m].y};
    }
  } else {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int n = p + Sh::N2 * m;
      const unsigned o = (unsigned)(dct ? dct_perm(n, N) : n) * n1s + (unsigned)c.ja;
      if (c.hasa) slice[o] = v[m].x;
      if (c.hasb) slice[o + 1] = v[m].y;
    }
  }
}

// Forward transform, division by S, inverse transform of the tile's lines in
// registers (exchanges through lds; called by every thread of the block; the
// caller synchronises before lds is used again).
template <typename T, int N>
__device__ __forceinline__ void cols_xform(const ColsArgs<T>& a, const ColTile& c,
                                           C2<T> (&v)[16], C2<T>* lds) {
  using Sh = fftr::Shape<T, N, true>;
  const SolveCtx& sc = a.sc;
  const int l = Sh::line(threadIdx.x), p = Sh::pos(threadIdx.x);
  const bool dct = a.ax.kind == 1;
  const T* __restrict__ tw = tw_table<T>(a.ax);
  const int t = c.t, ja = c.ja, jb = ja + 1;
  const bool hasa = c.hasa, hasb = c.hasb;
  fftr::fft4<T, N, -1, true>(v, lds + l * Sh::L, p, tw);
  __syncthreads();
  C2<T>* zb = lds + l * Sh::L2;
#pragma unroll
  for (int m = 0; m < 16; ++m) zb[p + Sh::N2 * m] = v[m];
  __syncthreads();
  const SliceSymbol<T> sym(sc, sc.lam_t[t]);
  const T l1a = hasa ? (T)sc.lam1[ja] : (T)0, l1b = hasb ? (T)sc.lam1[jb] : (T)0;
  const T* __restrict__ ct = ct_table<T>(a.ax);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = p + Sh::N2 * m;
    const int kr = k ? N - k : 0;
    const C2<T> z = v[m], zr = zb[kr];
    const T R0 = (T)sc.lam0[k];
    const T ia = sym.inv(R0 + l1a);
    const T ib = sym.inv(R0 + l1b);
    if (!dct) {
      // W = Z_a ia + i Z_b ib = (Z + conj Zr)/2 ia + (Z - conj Zr)/2 ib
      const C2<T> sp = {(T)0.5 * (z.x + zr.x), (T)0.5 * (z.y - zr.y)};
      const C2<T> sm = {(T)0.5 * (z.x - zr.x), (T)0.5 * (z.y + zr.y)};
      v[m] = C2<T>{fftr::ffma(sp.x, ia, sm.x * ib), fftr::ffma(sp.y, ia, sm.y * ib)};
    } else {
      const T pp = z.x, q = z.y, r = zr.x, s = zr.y;
      const T c = ct[2 * k], sn = ct[2 * k + 1];
      const T ca = (T)0.5 * fftr::ffma(c, pp + r, sn * (q - s)) * ia;
      const T cb = (T)0.5 * fftr::ffma(c, q + s, sn * (r - pp)) * ib;
      T rca = (T)0, rcb = (T)0;
      if (k) {
        const T Rr = (T)sc.lam0[kr];
        const T ira = sym.inv(Rr + l1a);
        const T irb = sym.inv(Rr + l1b);
        const T cr = ct[2 * kr], snr = ct[2 * kr + 1];
        rca = (T)0.5 * fftr::ffma(cr, r + pp, snr * (s - q)) * ira;
        rcb = (T)0.5 * fftr::ffma(cr, s + q, snr * (pp - r)) * irb;
      }
      v[m].x = fftr::ffma(c, ca, sn * rca) - fftr::ffma(sn, cb, -(c * rcb));
      v[m].y = fftr::ffma(sn, ca, -(c * rca)) + fftr::ffma(c, cb, sn * rcb);
    }
  }
  __syncthreads();
  fftr::fft4<T, N, +1, true>(v, lds + l * Sh::L, p, tw);
}

template <typename T, int N>
__device__ void cols_reg(const ColsArgs<T>& a, int bid, int nb, C2<T>* lds) {
  const ColTile c = col_tile<T, N>(a, xcd_remap(bid, nb));
  C2<T> v[16];
  cols_load<T, N>(a, c, v);
  cols_xform<T, N>(a, c, v, lds);
  cols_store<T, N>(a, c, v);
}

// The float64 LDS-path bodies are compiled once, as functions of their own,
// and called by both the single-plan and the batched kernels: inlined into
// each, the compiler contracted their multiply-adds differently, and batched
// runs must take exactly the single-plan arithmetic.
template <typename T>
__device__ __noinline__ void rows_body_call(const RowsArgs<T>& a, int bid) {
  rows_body<T>(a, bid);
}
template <typename T>
__device__ __noinline__ void cols_body_call(const ColsArgs<T>& a, int bid, int nb) {
  cols_body<T>(a, bid, nb);
}

template <typename T>
__device__ __forceinline__ void rows_entry(const RowsArgs<T>& a, int bid) {
  if constexpr (sizeof(T) == 8) rows_body_call<T>(a, bid);
  else rows_body<T>(a, bid);
}
template <typename T>
__device__ __forceinline__ void cols_entry(const ColsArgs<T>& a, int bid, int nb) {
  if constexpr (sizeof(T) == 8) cols_body_call<T>(a, bid, nb);
  else cols_body<T>(a, bid, nb);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rows(RowsArgs<T> a) {
  rows_entry<T>(a, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rows_batch(const RowsArgs<T>* A, const int* off,
                                                    int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  rows_entry<T>(A[i], blockIdx.x - off[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cols_solve(ColsArgs<T> a) {
  cols_entry<T>(a, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cols_batch(const ColsArgs<T>* A, const int* off,
                                                    int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  cols_entry<T>(A[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

// Register path, one kernel per axis length (mode 0: forward, 1: inverse).
template <typename T, int N>
__device__ __forceinline__ void rows_reg(const RowsArgs<T>& a, int bid) {
  if (a.done && *a.done != 0.0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem);
  if (a.mode == 0) rows_fwd_reg<T, N>(a, bid, lds);
  else rows_inv_reg<T, N>(a, bid, lds);
}

template <typename T, int N>
__device__ __forceinline__ void cols_reg_entry(const ColsArgs<T>& a, int bid, int nb) {
  if (a.done && *a.done != 0.0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cols_reg<T, N>(a, bid, nb, reinterpret_cast<C2<T>*>(smem));
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_rows_reg(RowsArgs<T> a) {
  rows_reg<T, N>(a, blockIdx.x);
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_rows_reg_batch(const RowsArgs<T>* A, const int* off,
                                                        int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  const RowsArgs<T> a = A[i];
  rows_reg<T, N>(a, blockIdx.x - off[i]);
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_cols_reg(ColsArgs<T> a) {
  cols_reg_entry<T, N>(a, blockIdx.x, gridDim.x);
}


template <typename T, int N>
__global__ __launch_bounds__(256) void k_cols_reg_batch(const ColsArgs<T>* A, const int* off,
                                                        int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  const ColsArgs<T> a = A[i];
  cols_reg_entry<T, N>(a, blockIdx.x - off[i], off[i + 1] - off[i]);
}

// Launch the row / column kernels of size class cls (0: LDS Stockham path,
// else the register path of that axis length).
template <typename T>
void launch_rows_cls(int cls, dim3 grid, dim3 block, size_t shm, hipStream_t s,
                     const RowsArgs<T>& a) {
  switch (cls) {
    case 64: hipLaunchKernelGGL((k_rows_reg<T, 64>), grid, block, shm, s, a); break;
    case 128: hipLaunchKernelGGL((k_rows_reg<T, 128>), grid, block, shm, s, a); break;
    case 256: hipLaunchKernelGGL((k_rows_reg<T, 256>), grid, block, shm, s, a); break;
    default: hipLaunchKernelGGL(k_rows<T>, grid, block, shm, s, a);
  }
}

template <typename T>
void launch_cols_cls(int cls, dim3 grid, dim3 block, size_t shm, hipStream_t s,
                     const ColsArgs<T>& a) {
  switch (cls) {
    case 64: hipLaunchKernelGGL((k_cols_reg<T, 64>), grid, block, shm, s, a); break;
    case 128: hipLaunchKernelGGL((k_cols_reg<T, 128>), grid, block, shm, s, a); break;
    case 256: hipLaunchKernelGGL((k_cols_reg<T, 256>), grid, block, shm, s, a); break;
    default: hipLaunchKernelGGL(k_cols_solve<T>, grid, block, shm, s, a);
  }
}

struct SpatialShape {
  int lpb, nrows, rblocks, cw, cblocks;
  int rreg, creg;          // size class: 0 (LDS path) or the axis length (register path)
  int rthreads, cthreads;  // block sizes
  size_t rshm, cshm;
};

SolveCtx solve_ctx(const Plan& P) {
  SolveCtx sc;
  sc.lam_t = P.lam_t;
  sc.lam0 = P.g.has0 ? P.ax0.lam : nullptr;
  sc.lam1 = P.ax1.lam;
  sc.nu = P.g.nu;
  sc.idt = P.g.idt;
  sc.idt2 = P.g.idt2;
  sc.norm = 1.0 / ((double)P.g.n0 * (double)P.g.n1);
  return sc;
}

// Launch shapes of the spatial solves (row transforms and column solves).
template <typename T>
SpatialShape spatial_shape(const Plan& P) {
  const Geom& g = P.g;
  SpatialShape sh{};
  const int N1 = g.n1;
  const int nrows = g.nt * g.n0;
  const int nlines = (nrows + 1) / 2;
  sh.nrows = nrows;
  const bool use_reg = P.tune.fft_reg != 0;
  sh.rreg = (use_reg && g.has0 && fftr::has_reg_path(N1)) ? N1 : 0;
  if (sh.rreg) {
    // register path: lines pair the time slices 2 tp, 2 tp + 1 (rows_reg.h)
    const int rlines = reg_lines(nrows, g.n0);
    int lpb = 0, buf = 0;
    switch (N1) {
      case 64: lpb = fftr::Shape<T, 64>::LPB; buf = fftr::Shape<T, 64>::BUF; break;
      case 128: lpb = fftr::Shape<T, 128>::LPB; buf = fftr::Shape<T, 128>::BUF; break;
      default: lpb = fftr::Shape<T, 256>::LPB; buf = fftr::Shape<T, 256>::BUF; break;
    }
    sh.lpb = lpb;
    sh.rblocks = (rlines + lpb - 1) / lpb;
    sh.rthreads = fftr::Shape<T, 64>::NT;
    sh.rshm = (size_t)buf * sizeof(C2<T>);
  } else {
    int lpb = P.tune.rows_elems / N1;
    if (lpb < 1) lpb = 1;
    if (lpb > 32) lpb = 32;
    if (lpb > nlines) lpb = nlines;
    // keep dynamic LDS (two buffers + tables) within 64 KB
    const int lpb_max =
        (int)((65536 - 4 * (size_t)N1 * sizeof(T)) / (2 * (size_t)N1 * sizeof(C2<T>)));
    if (lpb > lpb_max) lpb = lpb_max;
    if (lpb < 1) lpb = 1;
    sh.lpb = lpb;
    sh.rblocks = (nlines + lpb - 1) / lpb;
    sh.rthreads = 256;
    sh.rshm = 2 * (size_t)lpb * N1 * sizeof(C2<T>) + 4 * (size_t)N1 * sizeof(T);
  }
  if (g.has0) {
    sh.creg = (use_reg && fftr::has_reg_path(g.n0)) ? g.n0 : 0;
    if (sh.creg) {
      int lines = 0, buf = 0;
      switch (g.n0) {
        case 64: lines = fftr::Shape<T, 64, true>::LPB; buf = fftr::Shape<T, 64, true>::BUF; break;
        case 128: lines = fftr::Shape<T, 128, true>::LPB; buf = fftr::Shape<T, 128, true>::BUF; break;
        default: lines = fftr::Shape<T, 256, true>::LPB; buf = fftr::Shape<T, 256, true>::BUF; break;
      }
      sh.cw = 2 * lines;
      sh.cthreads = fftr::Shape<T, 64>::NT;
      sh.cshm = (size_t)buf * sizeof(C2<T>);
    } else {
      int lines = P.tune.cols_lines;
      const int lmax =
          (int)((65536 - 4 * (size_t)g.n0 * sizeof(T)) / (2 * (size_t)g.n0 * sizeof(C2<T>)));
      if (lines > lmax) lines = lmax;
      if (lines < 1) lines = 1;
      sh.cw = 2 * lines;
      sh.cthreads = 256;
      sh.cshm = 2 * (size_t)lines * g.n0 * sizeof(C2<T>) + 4 * (size_t)g.n0 * sizeof(T);
    }
    sh.cblocks = g.nt * ((g.n1 + sh.cw - 1) / sh.cw);
  }
  return sh;
}

template <typename T>
RowsArgs<T> rows_args(const Plan& P, const SpatialShape& sh, T* data, int mode,
                      const double* done) {
  return RowsArgs<T>{data,        sh.nrows, P.ax1, mode, sh.lpb, solve_ctx(P),
                     P.g.has0 ? P.g.n0 : 1, done, (mode != 2) ? sh.rreg : 0};
}

template <typename T>
ColsArgs<T> cols_args(const Plan& P, const SpatialShape& sh, T* data, const double* done) {
  return ColsArgs<T>{data, P.g, P.ax0, sh.cw, solve_ctx(P), done, sh.creg};
}

// skip_fwd / skip_inv: the forward / inverse row transforms are done by the
// fused forward / inverse pass.
template <typename T>
void spatial_solves(const Plan& P, T* data, hipStream_t s, bool skip_fwd = false,
                    bool skip_inv = false) {
  const Geom& g = P.g;
  const SpatialShape sh = spatial_shape<T>(P);
  if (!g.has0) {
    ProfScope ps(P, sizeof(T) == 8 ? "rows_solve_f64" : "rows_solve_f32", s);
    hipLaunchKernelGGL(k_rows<T>, dim3(sh.rblocks), dim3(256), sh.rshm, s,
                       rows_args<T>(P, sh, data, 2, P.pcg_done));
    return;
  }
  if (!skip_fwd) {
    ProfScope ps(P, sizeof(T) == 8 ? "rows_fwd_f64" : "rows_fwd_f32", s);
    launch_rows_cls<T>(sh.rreg, dim3(sh.rblocks), dim3(sh.rthreads), sh.rshm, s,
                       rows_args<T>(P, sh, data, 0, P.pcg_done));
  }
  {
    ProfScope ps(P, sizeof(T) == 8 ? "cols_solve_f64" : "cols_solve_f32", s);
    launch_cols_cls<T>(sh.creg, dim3(sh.cblocks), dim3(sh.cthreads), sh.cshm, s,
                       cols_args<T>(P, sh, data, P.pcg_done));
  }
  if (skip_inv) return;
  ProfScope ps(P, sizeof(T) == 8 ? "rows_inv_f64" : "rows_inv_f32", s);
  launch_rows_cls<T>(sh.rreg, dim3(sh.rblocks), dim3(sh.rthreads), sh.rshm, s,
                     rows_args<T>(P, sh, data, 1, P.pcg_done));
}

}  // namespace

namespace {

int mixed_mode(const Plan& P) {
  return P.precision == MFG_MIXED_FP32 ? GM_F32
         : (P.precision == MFG_MIXED_FP16 ? GM_F16 : GM_BF16);
}

const char* const kFwdNames[4] = {"tgemm_f64_fwd", "tgemm_f32_fwd", "tgemm_f16_fwd",
                                  "tgemm_bf16_fwd"};
const char* const kInvNames[4] = {"tgemm_f64_inv", "tgemm_f32_inv", "tgemm_f16_inv",
                                  "tgemm_bf16_inv"};
const char* const kFusedNames[4] = {"", "tgemm_rows_f32_fwd", "tgemm_rows_f16_fwd",
                                    "tgemm_rows_bf16_fwd"};
const char* const kUpdFusedNames[4] = {"", "update_tgemm_rows_f32_fwd",
                                       "update_tgemm_rows_f16_fwd", "update_tgemm_rows_bf16_fwd"};
const char* const kInvFusedNames[4] = {"", "rows_tgemm_f32_inv", "rows_tgemm_f16_inv",
                                       "rows_tgemm_bf16_inv"};

// Spatial solves after the forward pass (its row transforms done when
// fwd_fused) and the inverse pass (z, with the dot partials of dotmode).
void mixed_tail(const Plan& P, int mode, float* tmp, double* z, int dotmode, const double* r,
                const double* q, bool fwd_fused, hipStream_t s) {
  const int gate = P.rr_gate;  // stopping test of the inverse pass (0: none)
  P.rr_gate = 0;
  const bool inv_fused = fused_inv_ok(P);
  spatial_solves<float>(P, tmp, s, fwd_fused, inv_fused);
  P.rr_gate = gate;
  if (inv_fused) {
    int parts;
    {
      ProfScope ps(P, kInvFusedNames[mode], s);
      parts = launch_rows_tgemm_inv(P, mode,
                                    rows_args<float>(P, spatial_shape<float>(P), tmp, 1,
                                                     P.pcg_done),
                                    z, dotmode, r, q, s);
    }
    if (dotmode != DOT_NONE) P.rz_blocks = parts;
  } else {
    tgemm<float, double>(P, mode, tmp, z, dotmode, r, q, s, kInvNames[mode]);
  }
  P.rr_gate = 0;
}

}  // namespace

void launch_precond(const Plan& P, const double* r, double* z, bool fused_dots,
                    const double* q, hipStream_t s) {
  int dotmode = DOT_NONE;
  if (fused_dots)
    dotmode = (q == nullptr) ? DOT_INIT : (pcg_flexible(P) ? DOT_FLEX : DOT_STD);
  // inside the PCG loop the forward transform takes the r.r stopping test
  // over the update's partials (no finisher launch between them)
  P.rr_gate = (fused_dots && q != nullptr && P.pcg_done) ? P.rr_blocks : 0;
  if (P.precision == MFG_FP64) {
    double* tmp = P.tmp;
    tgemm<double, double>(P, GM_F64, r, tmp, DOT_NONE, nullptr, nullptr, s, "tgemm_f64_fwd");
    P.rr_gate = 0;
    spatial_solves<double>(P, tmp, s);
    tgemm<double, double>(P, GM_F64, tmp, z, dotmode, r, q, s, "tgemm_f64_inv");
    return;
  }
  // mixed: float32 intermediate and spatial solves; time transform in the
  // plan's matrix-core precision
  const int mode = mixed_mode(P);
  float* tmp = reinterpret_cast<float*>(P.tmp);
  const bool fwd_fused = fused_fwd_ok(P);
  if (fwd_fused) {
    ProfScope ps(P, kFusedNames[mode], s);
    launch_tgemm_rows_fwd(P, mode, r, tmp,
                          rows_args<float>(P, spatial_shape<float>(P), tmp, 0, P.pcg_done),
                          nullptr, s);
  } else {
    tgemm<double, float>(P, mode, r, tmp, DOT_NONE, nullptr, nullptr, s, kFwdNames[mode]);
  }
  P.rr_gate = 0;
  mixed_tail(P, mode, tmp, z, dotmode, r, q, fwd_fused, s);
}

// One PCG iteration's update and preconditioning: x += alpha p, r -= alpha q
// (r.r partials), then z = P^{-1} r (r.r stopping test first) with the fused
// r.z (and z.q) partials. Where the fused forward pass applies, the update
// runs inside it and the stopping test moves to the inverse time transform
// (the spatial solves of the last iteration run before it sets the flag; their
// output is not used).
void launch_update_precond(const Plan& P, double* x, double* r, const double* p,
                           const double* q, double* z, bool first, hipStream_t s) {
  if (!fused_upd_ok(P)) {
    launch_update(P, x, r, p, q, first, s);
    launch_precond(P, r, z, true, q, s);
    return;
  }
  const int mode = mixed_mode(P);
  float* tmp = reinterpret_cast<float*>(P.tmp);
  const UpdArgs ua = update_args(P, x, r, p, q, first);
  {
    ProfScope ps(P, kUpdFusedNames[mode], s);
    launch_tgemm_rows_fwd(P, mode, r, tmp,
                          rows_args<float>(P, spatial_shape<float>(P), tmp, 0, P.pcg_done), &ua,
                          s);
  }
  P.rr_blocks = P.g.n0;  // one r.r partial per block (axis-0 row)
  P.rr_gate = P.rr_blocks;
  mixed_tail(P, mode, tmp, z, pcg_flexible(P) ? DOT_FLEX : DOT_STD, r, q, true, s);
}

// ---- batched spatial solves (float32 data in the mixed modes, float64 in FP64) ----
template <typename T>
int batch_rows_args(const Plan& P, T* data, int mode, const double* done, RowsArgs<T>* out,
                    int* blocks, size_t* shm, int* threads) {
  const SpatialShape sh = spatial_shape<T>(P);
  *out = rows_args<T>(P, sh, data, mode, done);
  *blocks = sh.rblocks;
  *shm = sh.rshm;
  *threads = sh.rthreads;
  return sh.rreg;
}

template <typename T>
int batch_cols_args(const Plan& P, T* data, const double* done, ColsArgs<T>* out, int* blocks,
                    size_t* shm, int* threads) {
  const SpatialShape sh = spatial_shape<T>(P);
  *out = cols_args<T>(P, sh, data, done);
  *blocks = sh.cblocks;
  *shm = sh.cshm;
  *threads = sh.cthreads;
  return sh.creg;
}

// the block size is that of the size class (every instance of a launch has it)
template <typename T>
void launch_rows_batch(int cls, const RowsArgs<T>* a, const int* off, int ninst, int total,
                       size_t shm, int threads, hipStream_t s) {
  const dim3 g(total), b(threads);
  switch (cls) {
    case 64: hipLaunchKernelGGL((k_rows_reg_batch<T, 64>), g, b, shm, s, a, off, ninst); break;
    case 128: hipLaunchKernelGGL((k_rows_reg_batch<T, 128>), g, b, shm, s, a, off, ninst); break;
    case 256: hipLaunchKernelGGL((k_rows_reg_batch<T, 256>), g, b, shm, s, a, off, ninst); break;
    default: hipLaunchKernelGGL(k_rows_batch<T>, g, b, shm, s, a, off, ninst);
  }
}

template <typename T>
void launch_cols_batch(int cls, const ColsArgs<T>* a, const int* off, int ninst, int total,
                       size_t shm, int threads, hipStream_t s) {
  const dim3 g(total), b(threads);
  switch (cls) {
    case 64: hipLaunchKernelGGL((k_cols_reg_batch<T, 64>), g, b, shm, s, a, off, ninst); break;
    case 128: hipLaunchKernelGGL((k_cols_reg_batch<T, 128>), g, b, shm, s, a, off, ninst); break;
    case 256: hipLaunchKernelGGL((k_cols_reg_batch<T, 256>), g, b, shm, s, a, off, ninst); break;
    default: hipLaunchKernelGGL(k_cols_batch<T>, g, b, shm, s, a, off, ninst);
  }
}

#define MFG_BATCH_SPATIAL(T)                                                                    \
  template int batch_rows_args<T>(const Plan&, T*, int, const double*, RowsArgs<T>*, int*,      \
                                  size_t*, int*);                                               \
  template int batch_cols_args<T>(const Plan&, T*, const double*, ColsArgs<T>*, int*, size_t*,  \
                                  int*);                                                        \
  template void launch_rows_batch<T>(int, const RowsArgs<T>*, const int*, int, int, size_t, int, \
                                     hipStream_t);                                              \
  template void launch_cols_batch<T>(int, const ColsArgs<T>*, const int*, int, int, size_t, int, \
                                     hipStream_t);
MFG_BATCH_SPATIAL(float)
MFG_BATCH_SPATIAL(double)
#undef MFG_BATCH_SPATIAL

}  // namespace mfg
