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
#include "plan.h"
#include "tgemm.h"

namespace mfg {

namespace {

template <typename T>
struct C2 {
  T x, y;
};

constexpr int kLoadBatch = 8;  // global loads per thread issued before their LDS stores

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
__device__ __forceinline__ int dct_perm(int n, int N) {
  return (2 * n < N) ? 2 * n : 2 * (N - 1 - n) + 1;
}

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

template <typename T>
__global__ __launch_bounds__(256) void k_rows(RowsArgs<T> a) {
  rows_body<T>(a, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rows_batch(const RowsArgs<T>* A, const int* off,
                                                    int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  rows_body<T>(A[i], blockIdx.x - off[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cols_solve(ColsArgs<T> a) {
  cols_body<T>(a, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cols_batch(const ColsArgs<T>* A, const int* off,
                                                    int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  cols_body<T>(A[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

struct SpatialShape {
  int lpb, nrows, rblocks, cw, cblocks;
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
  int lpb = P.tune.rows_elems / N1;
  if (lpb < 1) lpb = 1;
  if (lpb > 32) lpb = 32;
  const int nrows = g.nt * g.n0;
  const int nlines = (nrows + 1) / 2;
  if (lpb > nlines) lpb = nlines;
  // keep dynamic LDS (two buffers + tables) within 64 KB
  const int lpb_max = (int)((65536 - 4 * (size_t)N1 * sizeof(T)) / (2 * (size_t)N1 * sizeof(C2<T>)));
  if (lpb > lpb_max) lpb = lpb_max;
  if (lpb < 1) lpb = 1;
  sh.lpb = lpb;
  sh.nrows = nrows;
  sh.rblocks = (nlines + lpb - 1) / lpb;
  sh.rshm = 2 * (size_t)lpb * N1 * sizeof(C2<T>) + 4 * (size_t)N1 * sizeof(T);
  if (g.has0) {
    int lines = P.tune.cols_lines;
    const int lmax =
        (int)((65536 - 4 * (size_t)g.n0 * sizeof(T)) / (2 * (size_t)g.n0 * sizeof(C2<T>)));
    if (lines > lmax) lines = lmax;
    if (lines < 1) lines = 1;
    sh.cw = 2 * lines;
    sh.cblocks = g.nt * ((g.n1 + sh.cw - 1) / sh.cw);
    sh.cshm = 2 * (size_t)lines * g.n0 * sizeof(C2<T>) + 4 * (size_t)g.n0 * sizeof(T);
  }
  return sh;
}

template <typename T>
RowsArgs<T> rows_args(const Plan& P, const SpatialShape& sh, T* data, int mode,
                      const double* done) {
  return RowsArgs<T>{data, sh.nrows, P.ax1, mode, sh.lpb, solve_ctx(P), P.g.has0 ? P.g.n0 : 1,
                     done};
}

template <typename T>
ColsArgs<T> cols_args(const Plan& P, const SpatialShape& sh, T* data, const double* done) {
  return ColsArgs<T>{data, P.g, P.ax0, sh.cw, solve_ctx(P), done};
}

template <typename T>
void spatial_solves(const Plan& P, T* data, hipStream_t s) {
  const Geom& g = P.g;
  const SpatialShape sh = spatial_shape<T>(P);
  if (!g.has0) {
    ProfScope ps(P, sizeof(T) == 8 ? "rows_solve_f64" : "rows_solve_f32", s);
    hipLaunchKernelGGL(k_rows<T>, dim3(sh.rblocks), dim3(256), sh.rshm, s,
                       rows_args<T>(P, sh, data, 2, nullptr));
    return;
  }
  {
    ProfScope ps(P, sizeof(T) == 8 ? "rows_fwd_f64" : "rows_fwd_f32", s);
    hipLaunchKernelGGL(k_rows<T>, dim3(sh.rblocks), dim3(256), sh.rshm, s,
                       rows_args<T>(P, sh, data, 0, nullptr));
  }
  {
    ProfScope ps(P, sizeof(T) == 8 ? "cols_solve_f64" : "cols_solve_f32", s);
    hipLaunchKernelGGL(k_cols_solve<T>, dim3(sh.cblocks), dim3(256), sh.cshm, s,
                       cols_args<T>(P, sh, data, nullptr));
  }
  ProfScope ps(P, sizeof(T) == 8 ? "rows_inv_f64" : "rows_inv_f32", s);
  hipLaunchKernelGGL(k_rows<T>, dim3(sh.rblocks), dim3(256), sh.rshm, s,
                     rows_args<T>(P, sh, data, 1, nullptr));
}

}  // namespace

void launch_precond(const Plan& P, const double* r, double* z, bool fused_dots,
                    const double* q, hipStream_t s) {
  int dotmode = DOT_NONE;
  if (fused_dots)
    dotmode = (q == nullptr) ? DOT_INIT : (P.precision == MFG_FP64 ? DOT_STD : DOT_FLEX);
  if (P.precision == MFG_FP64) {
    double* tmp = P.tmp;
    tgemm<double, double>(P, GM_F64, r, tmp, DOT_NONE, nullptr, nullptr, s, "tgemm_f64_fwd");
    spatial_solves<double>(P, tmp, s);
    tgemm<double, double>(P, GM_F64, tmp, z, dotmode, r, q, s, "tgemm_f64_inv");
    return;
  }
  // mixed: float32 intermediate and spatial solves; time transform in the
  // plan's matrix-core precision
  const int mode = P.precision == MFG_MIXED_FP32 ? GM_F32
                   : (P.precision == MFG_MIXED_FP16 ? GM_F16 : GM_BF16);
  float* tmp = reinterpret_cast<float*>(P.tmp);
  static const char* fwd_names[4] = {"tgemm_f64_fwd", "tgemm_f32_fwd", "tgemm_f16_fwd",
                                     "tgemm_bf16_fwd"};
  static const char* inv_names[4] = {"tgemm_f64_inv", "tgemm_f32_inv", "tgemm_f16_inv",
                                     "tgemm_bf16_inv"};
  tgemm<double, float>(P, mode, r, tmp, DOT_NONE, nullptr, nullptr, s, fwd_names[mode]);
  spatial_solves<float>(P, tmp, s);
  tgemm<float, double>(P, mode, tmp, z, dotmode, r, q, s, inv_names[mode]);
}

// ---- batched spatial solves: float32 data (mixed precision) ----
void batch_rows_args(const Plan& P, float* data, int mode, const double* done, void* out,
                     int* blocks, size_t* shm) {
  const SpatialShape sh = spatial_shape<float>(P);
  *reinterpret_cast<RowsArgs<float>*>(out) = rows_args<float>(P, sh, data, mode, done);
  *blocks = sh.rblocks;
  *shm = sh.rshm;
}

void batch_cols_args(const Plan& P, float* data, const double* done, void* out, int* blocks,
                     size_t* shm) {
  const SpatialShape sh = spatial_shape<float>(P);
  *reinterpret_cast<ColsArgs<float>*>(out) = cols_args<float>(P, sh, data, done);
  *blocks = sh.cblocks;
  *shm = sh.cshm;
}

void launch_rows_batch_f32(const void* A, const int* off, int ninst, int total, size_t shm,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_rows_batch<float>, dim3(total), dim3(256), shm, s,
                     reinterpret_cast<const RowsArgs<float>*>(A), off, ninst);
}

void launch_cols_batch_f32(const void* A, const int* off, int ninst, int total, size_t shm,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_cols_batch<float>, dim3(total), dim3(256), shm, s,
                     reinterpret_cast<const ColsArgs<float>*>(A), off, ninst);
}

}  // namespace mfg
