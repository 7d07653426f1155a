// Time transform of Algorithm 1 on the gfx950 matrix cores (see tgemm.h).
//
// k_tgemm64: float64 products (v_mfma_f64_16x16x4f64). A block has 4 waves,
//   each owning CB blocks of 16 spatial nodes; the block covers KB*16 output
//   rows. V is staged through LDS in chunks of 16 time rows and, like the X
//   operands, fetched into registers one chunk ahead of its use.
// k_tgemm_lp: float32 / float16 / bfloat16 products with float32 accumulation
//   (v_mfma_f32_16x16x4f32, v_mfma_f32_16x16x16f16, v_mfma_f32_16x16x16bf16_1k)
//   for N_t <= 128: the whole of V sits in LDS (row k contiguous in t, the
//   matrix-core A layout) and the block's X operands for every t sit in
//   registers. For float16 the block's inputs are first scaled by a power of
//   two that maps their largest magnitude to about 2^14 (range of float16),
//   and the products are scaled back exactly.
// V is symmetric (V[k][t] = V[t][k] for the DCT-VIII and the DST-I), which the
// LDS staging uses to read it with unit stride.
#include "tgemm.h"

namespace mfg {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

template <int KB, int CB, typename TX, typename TY>
__global__ __launch_bounds__(256) void k_tgemm64(const double* __restrict__ Vt,
                                                 const TX* __restrict__ X, TY* __restrict__ Y,
                                                 int nt, int M, int ncolblk, int dotmode,
                                                 const double* __restrict__ rvec,
                                                 const double* __restrict__ qvec, RedBuf rb) {
  constexpr int KW = KB * 16;
  constexpr int TK = 16;
  constexpr int VPER = TK * KW / 256;
  __shared__ double Vs[TK * KW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cbk = blockIdx.x % ncolblk, kc = blockIdx.x / ncolblk;
  const int kbase = kc * KW;
  const int col0 = (cbk * 4 + wave) * CB * 16 + (lane & 15);
  const int kq = lane >> 4;
  v4d acc[CB][KB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc[cb][kb] = (v4d){0.0, 0.0, 0.0, 0.0};
  double vreg[VPER];
  double xn[CB][4];
  auto fetch = [&](int t0) {
#pragma unroll
    for (int e = 0; e < VPER; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int r = idx / KW, kk = idx - r * KW;
      const int t = t0 + r, k = kbase + kk;
      vreg[e] = (t < nt && k < nt) ? Vt[(size_t)t * nt + k] : 0.0;
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int t = t0 + 4 * ks + kq;
        const int col = col0 + cb * 16;
        xn[cb][ks] = (t < nt && col < M) ? (double)X[(size_t)t * M + col] : 0.0;
      }
  };
  const int nchunk = (nt + TK - 1) / TK;
  fetch(0);
  for (int c = 0; c < nchunk; ++c) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < VPER; ++e) Vs[threadIdx.x + 256 * e] = vreg[e];
    double xc[CB][4];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) xc[cb][ks] = xn[cb][ks];
    __syncthreads();
    if (c + 1 < nchunk) fetch((c + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const double a = Vs[(4 * ks + kq) * KW + kb * 16 + (lane & 15)];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[cb][kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xc[cb][ks], acc[cb][kb], 0, 0, 0);
      }
  }
  double dots[2] = {0.0, 0.0};
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = col0 + cb * 16;
    if (col >= M) continue;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int jr = 0; jr < 4; ++jr) {
        // v_mfma_f64_16x16x4f64 result: register jr of lane l holds row
        // (l / 16) + 4 jr, column l % 16
        const int k = kbase + kb * 16 + kq + 4 * jr;
        if (k < nt) {
          const size_t o = (size_t)k * M + col;
          const double v = acc[cb][kb][jr];
          Y[o] = (TY)v;
          if (dotmode != DOT_NONE) {
            dots[0] += rvec[o] * v;
            if (dotmode == DOT_FLEX) dots[1] += qvec[o] * v;
          }
        }
      }
  }
  if (dotmode != DOT_NONE) reduce_store<2>(dots, rb, T_RZ);
}

__device__ __forceinline__ short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (short)(u >> 16);
}

template <int MODE>
struct LpTraits;
template <>
struct LpTraits<GM_F32> {
  using VT = float;
  static constexpr int KSTEP = 4;
};
template <>
struct LpTraits<GM_F16> {
  using VT = _Float16;
  static constexpr int KSTEP = 16;
};
template <>
struct LpTraits<GM_BF16> {
  using VT = unsigned short;
  static constexpr int KSTEP = 16;
};

// NTP: N_t padded to a multiple of 16 (<= 128). The block covers 4 waves x CB
// blocks of 16 nodes and all N_t output rows.
template <int MODE, int NTP, int CB, typename TX, typename TY>
__global__ __launch_bounds__(256) void k_tgemm_lp(const typename LpTraits<MODE>::VT* __restrict__ Vg,
                                                  const TX* __restrict__ X, TY* __restrict__ Y,
                                                  int nt, int M, int dotmode,
                                                  const double* __restrict__ rvec,
                                                  const double* __restrict__ qvec, RedBuf rb) {
  using VT = typename LpTraits<MODE>::VT;
  constexpr int KSTEP = LpTraits<MODE>::KSTEP;
  constexpr int NKS = NTP / KSTEP;  // k-steps
  constexpr int NKB = NTP / 16;     // output row blocks
  constexpr int PER = KSTEP / 4;    // operand values per lane per k-step (1 or 4)
  __shared__ __align__(16) VT Vs[NTP * NTP];  // Vs[k * NTP + t] = V[k][t]
  __shared__ float smax[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int col0 = (blockIdx.x * 4 + wave) * CB * 16 + (lane & 15);
  // stage V (symmetric: row k read with unit stride in t)
  for (int idx = threadIdx.x; idx < NTP * NTP; idx += 256) {
    const int k = idx / NTP, t = idx - k * NTP;
    VT v;
    if (k < nt && t < nt) v = Vg[(size_t)k * nt + t];
    else v = (VT)0;
    Vs[idx] = v;
  }
  // operands: t = KSTEP*ks + PER*kq + j
  float xs[CB][NKS][PER];
  float amax = 0.0f;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = col0 + cb * 16;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int t = KSTEP * ks + PER * kq + j;
        const float v = (t < nt && col < M) ? (float)X[(size_t)t * M + col] : 0.0f;
        xs[cb][ks][j] = v;
        amax = fmaxf(amax, fabsf(v));
      }
  }
  float scale = 1.0f, unscale = 1.0f;
  if (MODE == GM_F16) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) smax[wave] = amax;
  }
  __syncthreads();
  if (MODE == GM_F16) {
    const float bm = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
    if (bm > 0.0f && __builtin_isfinite(bm)) {
      int e;
      frexpf(bm, &e);             // bm < 2^e
      e = e < -100 ? -100 : e;    // keep 2^(14 - e) finite in float32
      scale = ldexpf(1.0f, 14 - e);
      unscale = ldexpf(1.0f, e - 14);
    }
  }
  v4f acc[CB][NKB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) acc[cb][kb] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    if constexpr (MODE == GM_F32) {
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        const float a = Vs[(kb * 16 + (lane & 15)) * NTP + KSTEP * ks + PER * kq];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xs[cb][ks][0], acc[cb][kb], 0, 0, 0);
      }
    } else if constexpr (MODE == GM_F16) {
      v4h b[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) b[cb][j] = (_Float16)(xs[cb][ks][j] * scale);
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        const v4h a = *reinterpret_cast<const v4h*>(
            &Vs[(kb * 16 + (lane & 15)) * NTP + KSTEP * ks + PER * kq]);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b[cb], acc[cb][kb], 0, 0, 0);
      }
    } else {
      v4s b[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) b[cb][j] = f2bf(xs[cb][ks][j]);
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        const v4s a = *reinterpret_cast<const v4s*>(
            &Vs[(kb * 16 + (lane & 15)) * NTP + KSTEP * ks + PER * kq]);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[cb], acc[cb][kb], 0, 0, 0);
      }
    }
  }
  double dots[2] = {0.0, 0.0};
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = col0 + cb * 16;
    if (col >= M) continue;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int jr = 0; jr < 4; ++jr) {
        // float32-accumulating 16x16 results: register jr of lane l holds row
        // 4 (l / 16) + jr, column l % 16
        const int k = kb * 16 + 4 * kq + jr;
        if (k < nt) {
          const size_t o = (size_t)k * M + col;
          const double v = (double)(acc[cb][kb][jr] * unscale);
          Y[o] = (TY)v;
          if (dotmode != DOT_NONE) {
            dots[0] += rvec[o] * v;
            if (dotmode == DOT_FLEX) dots[1] += qvec[o] * v;
          }
        }
      }
  }
  if (dotmode != DOT_NONE) reduce_store<2>(dots, rb, T_RZ);
}

template <int MODE, int NTP, typename TX, typename TY>
int lp_launch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
              hipStream_t s) {
  constexpr int CB = 2;
  const int M = P.g.M;
  const int grid = (M + 64 * CB - 1) / (64 * CB);
  const void* V = (MODE == GM_F32) ? (const void*)P.Vt32
                  : (MODE == GM_F16) ? (const void*)P.Vt16 : (const void*)P.Vtbf;
  hipLaunchKernelGGL((k_tgemm_lp<MODE, NTP, CB, TX, TY>), dim3(grid), dim3(256), 0, s,
                     (const typename LpTraits<MODE>::VT*)V, X, Y, P.g.nt, M, dotmode, r, q, P.red);
  return grid;
}

template <int MODE, typename TX, typename TY>
int lp_dispatch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
                hipStream_t s) {
  const int nt = P.g.nt;
  if (nt <= 16) return lp_launch<MODE, 16>(P, X, Y, dotmode, r, q, s);
  if (nt <= 32) return lp_launch<MODE, 32>(P, X, Y, dotmode, r, q, s);
  if (nt <= 64) return lp_launch<MODE, 64>(P, X, Y, dotmode, r, q, s);
  if (nt <= 96) return lp_launch<MODE, 96>(P, X, Y, dotmode, r, q, s);
  return lp_launch<MODE, 128>(P, X, Y, dotmode, r, q, s);
}

template <int KB, int CB, typename TX, typename TY>
int f64_launch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
               hipStream_t s) {
  const int nt = P.g.nt, M = P.g.M;
  const int ncolblk = (M + 64 * CB - 1) / (64 * CB);
  const int nkc = (nt + KB * 16 - 1) / (KB * 16);
  const int grid = ncolblk * nkc;
  hipLaunchKernelGGL((k_tgemm64<KB, CB, TX, TY>), dim3(grid), dim3(256), 0, s, P.Vt64, X, Y, nt,
                     M, ncolblk, dotmode, r, q, P.red);
  return grid;
}

}  // namespace

template <typename TX, typename TY>
void tgemm(const Plan& P, int mode, const TX* X, TY* Y, int dotmode, const double* r,
           const double* q, hipStream_t s) {
  const int nt = P.g.nt;
  int grid;
  if (mode != GM_F64 && nt <= 128) {
    if (mode == GM_F32) grid = lp_dispatch<GM_F32>(P, X, Y, dotmode, r, q, s);
    else if (mode == GM_F16) grid = lp_dispatch<GM_F16>(P, X, Y, dotmode, r, q, s);
    else grid = lp_dispatch<GM_BF16>(P, X, Y, dotmode, r, q, s);
  } else if (nt <= 32) {
    grid = f64_launch<2, 2>(P, X, Y, dotmode, r, q, s);
  } else if (nt <= 64) {
    grid = f64_launch<4, 2>(P, X, Y, dotmode, r, q, s);
  } else {
    grid = f64_launch<8, 2>(P, X, Y, dotmode, r, q, s);
  }
  if (dotmode != DOT_NONE) launch_finish(P, T_RZ, grid, finish_op(dotmode), s);
}

template void tgemm<double, double>(const Plan&, int, const double*, double*, int, const double*,
                                    const double*, hipStream_t);
template void tgemm<double, float>(const Plan&, int, const double*, float*, int, const double*,
                                   const double*, hipStream_t);
template void tgemm<float, double>(const Plan&, int, const float*, double*, int, const double*,
                                   const double*, hipStream_t);

}  // namespace mfg
