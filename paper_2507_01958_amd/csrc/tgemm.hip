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
#include <type_traits>

#include "batch_args.h"
#include "pcg_update.h"
#include "rows_reg.h"
#include "tgemm.h"

namespace mfg {

namespace {

// Whether a GEMM block has nothing to do: the solve is over, or the r.r check
// folded into the forward transform (nrr > 0) ends it now.
template <typename TX, typename TY>
__device__ __forceinline__ bool gemm_skip(const GemmArgs<TX, TY>& ga, int bid) {
  if (ga.done && *ga.done != 0.0) return true;
  return ga.nrr > 0 && rr_check(ga.rb, ga.nrr, bid);
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

template <int KB, int CB, typename TX, typename TY>
__device__ void tgemm64_body(const GemmArgs<TX, TY>& ga, int bid) {
  if (gemm_skip(ga, bid)) return;
  const double* __restrict__ Vt = static_cast<const double*>(ga.V);
  const TX* __restrict__ X = ga.X;
  TY* __restrict__ Y = ga.Y;
  const int nt = ga.nt, M = ga.M, ncolblk = ga.ncolblk, dotmode = ga.dotmode;
  const double* __restrict__ rvec = ga.rvec;
  const double* __restrict__ qvec = ga.qvec;
  const RedBuf rb = ga.rb;
  constexpr int KW = KB * 16;
  constexpr int TK = 16;
  constexpr int VPER = TK * KW / 256;
  __shared__ double Vs[TK * KW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cbk = bid % ncolblk, kc = bid / ncolblk;
  const int kbase = kc * KW;
  const int col0 = (cbk * 4 + wave) * CB * 16 + (lane & 15);
  const int kq = lane >> 4;
  v4d acc[CB][KB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc[cb][kb] = (v4d){0.0, 0.0, 0.0, 0.0};
  double vreg[VPER];
  // prefetched operands stay in their input type until used, so a float input
  // is not converted (and waited for) right after its load is issued
  TX xn[CB][4];
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
        xn[cb][ks] = (t < nt && col < M) ? X[(size_t)t * M + col] : TX(0);
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
      for (int ks = 0; ks < 4; ++ks) xc[cb][ks] = (double)xn[cb][ks];
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
  if (dotmode != DOT_NONE) reduce_store<2>(dots, rb, T_RZ, bid);
}

template <int KB, int CB, typename TX, typename TY>
__global__ __launch_bounds__(256) void k_tgemm64(GemmArgs<TX, TY> a) {
  tgemm64_body<KB, CB, TX, TY>(a, blockIdx.x);
}

template <int KB, int CB>
__global__ __launch_bounds__(256) void k_tgemm64_batch(const GemmArgs<double, double>* A,
                                                       const int* off, int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  tgemm64_body<KB, CB, double, double>(A[i], blockIdx.x - off[i]);
}

constexpr int pow2_floor(int c) {
  int m = 1;
  while (m * 2 <= c) m *= 2;
  return m;
}

// LDS copy of the low-precision V (row r = output row k, V[r][t] for
// t < NTP): the 16-byte chunks c < P of row r (P the largest power of two
// <= chunks per row) are stored at c ^ (r & (P - 1)), a permutation within the
// row, so that the 16 lanes of a matrix-core A-operand read (16 consecutive
// rows, the same chunk) fall on distinct banks instead of one.
template <int NTP, typename VT>
struct VsLayout {
  static constexpr int EPC = 16 / (int)sizeof(VT);  // elements per chunk
  static constexpr int C = NTP / EPC;                // chunks per row
  static constexpr int P = pow2_floor(C);
  __device__ static __forceinline__ int swz(int r, int c) { return c < P ? (c ^ (r & (P - 1))) : c; }
  __device__ static __forceinline__ int idx(int r, int t) {
    return r * NTP + swz(r, t / EPC) * EPC + (t % EPC);
  }
  // destination chunk of source chunk i of the row-major copy
  __device__ static __forceinline__ int chunk(int i) {
    const int r = i / C;
    return r * C + swz(r, i - r * C);
  }
};

__device__ __forceinline__ short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (short)(u >> 16);
}

template <int MODE>
struct LpTraits;
template <>
struct LpTraits<GM_F32> {
  // float32 accuracy from float16 products: V as 2 NTP rows (hi, then lo) of
  // float16, operands split the same way per k-step (see kVSplitScale)
  using VT = _Float16;
  static constexpr int KSTEP = 16;
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

// Pieces of the low-precision time GEMM (N_t <= 128), shared by k_tgemm_lp and
// the fused time-GEMM + row-transform kernel so both compute the same bits.
// NTP: N_t padded to a multiple of 16 (<= 128); a wave owns CB blocks of 16
// nodes (columns col0 + 16 cb) and all NTP output rows.
template <int MODE, int NTP>
struct LpShape {
  using VT = typename LpTraits<MODE>::VT;
  static constexpr int KSTEP = LpTraits<MODE>::KSTEP;
  static constexpr int NKS = NTP / KSTEP;  // k-steps
  static constexpr int NKB = NTP / 16;     // output row blocks
  static constexpr int PER = KSTEP / 4;    // operand values per lane per k-step (1 or 4)
  static constexpr bool SPLIT = MODE == GM_F32;      // hi / lo float16 terms
  static constexpr bool SCALED = MODE == GM_F16 || SPLIT;  // power-of-2 operand scale
  static constexpr int VROWS = SPLIT ? 2 * NTP : NTP;
};

// Operands of the wave's CB tiles (t = KSTEP ks + PER kq + j); returns their
// largest magnitude.
template <int MODE, int NTP, int CB, typename TX>
__device__ __forceinline__ float lp_load(const TX* __restrict__ X, int nt, int M, int col0,
                                         int kq, float (&xs)[CB][LpShape<MODE, NTP>::NKS]
                                                            [LpShape<MODE, NTP>::PER]) {
  using L = LpShape<MODE, NTP>;
  float amax = 0.0f;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = col0 + cb * 16;
#pragma unroll
    for (int ks = 0; ks < L::NKS; ++ks)
#pragma unroll
      for (int j = 0; j < L::PER; ++j) {
        const int t = L::KSTEP * ks + L::PER * kq + j;
        const float v = (t < nt && col < M) ? (float)X[(size_t)t * M + col] : 0.0f;
        xs[cb][ks][j] = v;
        amax = fmaxf(amax, fabsf(v));
      }
  }
  return amax;
}

// V (zero-padded NTP x NTP copy, row k = V[k][.]; with SPLIT the lo rows
// follow) into LDS with 16-byte copies by nthreads threads.
template <int MODE, int NTP>
__device__ __forceinline__ void lp_stage_v(const typename LpShape<MODE, NTP>::VT* Vg,
                                           typename LpShape<MODE, NTP>::VT* Vs, int nthreads) {
  using L = LpShape<MODE, NTP>;
  constexpr int NV16 = L::VROWS * NTP * (int)sizeof(typename L::VT) / 16;
  const uint4* src = reinterpret_cast<const uint4*>(Vg);
  uint4* dst = reinterpret_cast<uint4*>(Vs);
  for (int i = threadIdx.x; i < NV16; i += nthreads)
    dst[VsLayout<NTP, typename L::VT>::chunk(i)] = src[i];
}

// Operand scale and the output's unscale from the largest operand magnitude
// bm of the scaling group: a power of two mapping bm to about 2^14 (float16
// range); V's split scale is undone with it.
template <int MODE, int NTP>
__device__ __forceinline__ void lp_scales(float bm, float& scale, float& unscale) {
  using L = LpShape<MODE, NTP>;
  const float vunscale = L::SPLIT ? (float)(1.0 / kVSplitScale) : 1.0f;
  scale = 1.0f;
  unscale = vunscale;
  if (L::SCALED && bm > 0.0f && __builtin_isfinite(bm)) {
    int e;
    frexpf(bm, &e);             // bm < 2^e
    e = e < -100 ? -100 : e;    // keep 2^(14 - e) finite in float32
    scale = ldexpf(1.0f, 14 - e);
    unscale = ldexpf(1.0f, e - 14) * vunscale;
  }
}

// The matrix-core products: acc[cb][kb] (rows 16 kb + 4 (lane / 16) + jr,
// column lane % 16 of tile cb) = sum over t of V[row][t] x_t (scaled).
template <int MODE, int NTP, int CB>
__device__ __forceinline__ void lp_mma(const typename LpShape<MODE, NTP>::VT* Vs,
                                       const float (&xs)[CB][LpShape<MODE, NTP>::NKS]
                                                        [LpShape<MODE, NTP>::PER],
                                       float scale, int lane,
                                       v4f (&acc)[CB][LpShape<MODE, NTP>::NKB]) {
  using L = LpShape<MODE, NTP>;
  using VT = typename L::VT;
  constexpr int KSTEP = L::KSTEP, PER = L::PER;
  const int kq = lane >> 4;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int kb = 0; kb < L::NKB; ++kb) acc[cb][kb] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < L::NKS; ++ks) {
    if constexpr (L::SPLIT) {
      // x s = hi + lo exactly up to lo's rounding (x s is float32, hi float16)
      v4h bh[CB], bl[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float xv = xs[cb][ks][j] * scale;
          const _Float16 h = (_Float16)xv;
          bh[cb][j] = h;
          bl[cb][j] = (_Float16)(xv - (float)h);
        }
#pragma unroll
      for (int kb = 0; kb < L::NKB; ++kb) {
        const int r = kb * 16 + (lane & 15), t = KSTEP * ks + PER * kq;
        const v4h ah = *reinterpret_cast<const v4h*>(&Vs[VsLayout<NTP, VT>::idx(r, t)]);
        const v4h al = *reinterpret_cast<const v4h*>(&Vs[VsLayout<NTP, VT>::idx(r + NTP, t)]);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh[cb], acc[cb][kb], 0, 0, 0);
          acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl[cb], acc[cb][kb], 0, 0, 0);
          acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh[cb], acc[cb][kb], 0, 0, 0);
        }
      }
    } else if constexpr (MODE == GM_F16) {
      v4h b[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) b[cb][j] = (_Float16)(xs[cb][ks][j] * scale);
#pragma unroll
      for (int kb = 0; kb < L::NKB; ++kb) {
        const v4h a = *reinterpret_cast<const v4h*>(
            &Vs[VsLayout<NTP, VT>::idx(kb * 16 + (lane & 15), KSTEP * ks + PER * kq)]);
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
      for (int kb = 0; kb < L::NKB; ++kb) {
        const v4s a = *reinterpret_cast<const v4s*>(
            &Vs[VsLayout<NTP, VT>::idx(kb * 16 + (lane & 15), KSTEP * ks + PER * kq)]);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[cb], acc[cb][kb], 0, 0, 0);
      }
    }
  }
}

// The block covers WPB waves x CB blocks of 16 nodes and all N_t output rows;
// the operand scale is the block's.
template <int MODE, int NTP, int CB, typename TX, typename TY, int WPB = 4>
__device__ void tgemm_lp_body(const GemmArgs<TX, TY>& ga, int bid) {
  if (gemm_skip(ga, bid)) return;
  using L = LpShape<MODE, NTP>;
  using VT = typename L::VT;
  const VT* __restrict__ Vg = static_cast<const VT*>(ga.V);
  TY* __restrict__ Y = ga.Y;
  const int nt = ga.nt, M = ga.M, dotmode = ga.dotmode;
  const double* __restrict__ rvec = ga.rvec;
  const double* __restrict__ qvec = ga.qvec;
  const RedBuf rb = ga.rb;
  __shared__ __align__(16) VT Vs[L::VROWS * NTP];  // Vs[k * NTP + t] = V[k][t] (+ lo rows)
  __shared__ float smax[WPB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int col0 = (bid * WPB + wave) * CB * 16 + (lane & 15);
  float xs[CB][L::NKS][L::PER];
  float amax = lp_load<MODE, NTP, CB>(ga.X, nt, M, col0, kq, xs);
  // stage V after the operand loads are in flight
  lp_stage_v<MODE, NTP>(Vg, Vs, WPB * 64);
  if (L::SCALED) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) smax[wave] = amax;
  }
  __syncthreads();
  float bm = 0.0f;
  if (L::SCALED) {
    bm = smax[0];
#pragma unroll
    for (int w = 1; w < WPB; ++w) bm = fmaxf(bm, smax[w]);
  }
  float scale, unscale;
  lp_scales<MODE, NTP>(bm, scale, unscale);
  v4f acc[CB][L::NKB];
  lp_mma<MODE, NTP, CB>(Vs, xs, scale, lane, acc);
  double dots[2] = {0.0, 0.0};
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = col0 + cb * 16;
    if (col >= M) continue;
#pragma unroll
    for (int kb = 0; kb < L::NKB; ++kb)
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
  if (dotmode != DOT_NONE) reduce_store<2>(dots, rb, T_RZ, bid);
}

template <int MODE, int NTP, int CB, typename TX, typename TY, int WPB>
__global__ __launch_bounds__(WPB * 64) void k_tgemm_lp(GemmArgs<TX, TY> a) {
  tgemm_lp_body<MODE, NTP, CB, TX, TY, WPB>(a, blockIdx.x);
}

// Raw buffer access (a range-checked vector memory descriptor): a load beyond
// `bytes` returns 0 and a store beyond it is dropped, so code at the ragged end
// of an array needs no branch (branches around loads and stores leave the
// compiler unsure how many are outstanding, and it then waits for all).
typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
  // third descriptor word of a raw (untyped, stride 0) buffer on gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t rs, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u32, v), rs, (int)off, 0, 0);
}

// The conjugate gradient update of the wave's tiles (x += alpha p, r -= alpha q,
// the same multiply-adds as the update kernel), adding r.r to rr; the new r
// values are the GEMM operands (as lp_load reads them). Returns their largest
// magnitude. The elements go in groups of one k-step (PER values per tile);
// the loads of group g + 1 are issued before group g is computed and stored,
// so a wave keeps two groups of loads in flight. Elements with t >= N_t lie
// beyond the descriptors' range: they read 0 (a zero operand, as lp_load's)
// and their stores are dropped. Requires NTP M 8 < 2^31 bytes (the caller
// checks). FIRST: x = 0 before the update (written, not read). XUPD = false:
// only r (x += alpha p is left to XStream).
template <int MODE, int NTP, int CB, bool FIRST, bool XUPD = true>
__device__ __forceinline__ float upd_load(const UpdArgs& a, double alpha, int nt, int M, int col0,
                                          int kq, float (&xs)[CB][LpShape<MODE, NTP>::NKS]
                                                             [LpShape<MODE, NTP>::PER],
                                          double& rr) {
  using L = LpShape<MODE, NTP>;
  constexpr int G = CB * L::PER;  // elements per group
  const unsigned bytes = (unsigned)nt * (unsigned)M * 8u;
  const __amdgpu_buffer_rsrc_t xr = buf_rsrc(a.x, bytes), rr_ = buf_rsrc(a.r, bytes);
  const __amdgpu_buffer_rsrc_t pr = buf_rsrc(a.p, bytes), qr = buf_rsrc(a.q, bytes);
  auto off = [&](int ks, int e) {
    const int cb = e / L::PER, j = e % L::PER;
    const int t = L::KSTEP * ks + L::PER * kq + j, col = col0 + cb * 16;
    return ((unsigned)t * (unsigned)M + (unsigned)col) * 8u;
  };
  double pb[2][G], qb[2][G], rb[2][G], xb[2][G];
  auto load = [&](int ks, int buf) {
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const unsigned o = off(ks, e);
      if (XUPD) pb[buf][e] = buf_ld(pr, o);
      qb[buf][e] = buf_ld(qr, o);
      rb[buf][e] = buf_ld(rr_, o);
      if (XUPD && !FIRST) xb[buf][e] = buf_ld(xr, o);
    }
  };
  float amax = 0.0f;
  load(0, 0);
#pragma unroll
  for (int ks = 0; ks < L::NKS; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < L::NKS) load(ks + 1, cur ^ 1);
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const unsigned o = off(ks, e);
      if (XUPD)
        buf_st(xr, o, FIRST ? alpha * pb[cur][e] : __builtin_fma(alpha, pb[cur][e], xb[cur][e]));
      const double ri = __builtin_fma(-alpha, qb[cur][e], rb[cur][e]);
      buf_st(rr_, o, ri);
      rr += ri * ri;
      const float v = (float)ri;
      xs[e / L::PER][ks][e % L::PER] = v;
      amax = fmaxf(amax, fabsf(v));
    }
  }
  return amax;
}

// x += alpha p of the fused kernel's column (one 16-node tile, CB = 1) by
// ranges of k-steps whose loads are issued before one of the kernel's
// LDS-only phases (products, tile, row loads, transforms) and whose stores
// follow it, so most of this third of the update's traffic overlaps the
// computation. The ranges (bound(c), c = 0..5) give each phase what its free
// registers hold (1/8 of the k-steps during the products and the transforms,
// 2/8 during the tile phases); the last quarter follows the transforms. The
// same multiply-add as the update kernel; t >= N_t lies beyond the
// descriptors' range.
template <int MODE, int NTP, bool FIRST>
struct XStream {
  using L = LpShape<MODE, NTP>;
  static constexpr int bound(int c) {
    return c == 0 ? 0 : c == 1 ? L::NKS / 8 : c == 2 ? 3 * L::NKS / 8
                      : c == 3 ? 5 * L::NKS / 8 : c == 4 ? 6 * L::NKS / 8 : L::NKS;
  }
  __amdgpu_buffer_rsrc_t xr, pr;
  double alpha;
  int M, col0, kq;
  double xb[L::NKS][L::PER], pb[L::NKS][L::PER];
  __device__ __forceinline__ unsigned off(int ks, int j) const {
    const int t = L::KSTEP * ks + L::PER * kq + j;
    return ((unsigned)t * (unsigned)M + (unsigned)col0) * 8u;
  }
  // the compiler's scheduler keeps each range's loads at their place (hoisted
  // into the products, they would hold registers there)
  template <int C>
  __device__ __forceinline__ void load() {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = bound(C); ks < bound(C + 1); ++ks)
#pragma unroll
      for (int j = 0; j < L::PER; ++j) {
        const unsigned o = off(ks, j);
        pb[ks][j] = buf_ld(pr, o);
        if (!FIRST) xb[ks][j] = buf_ld(xr, o);
      }
    __builtin_amdgcn_sched_barrier(0);
  }
  template <int C>
  __device__ __forceinline__ void store() {
#pragma unroll
    for (int ks = bound(C); ks < bound(C + 1); ++ks)
#pragma unroll
      for (int j = 0; j < L::PER; ++j) {
        const double pv = pb[ks][j];
        buf_st(xr, off(ks, j), FIRST ? alpha * pv : __builtin_fma(alpha, pv, xb[ks][j]));
      }
  }
};

// Fused forward pass (time GEMM + row transforms along axis 1, N = 256): the
// block owns axis-0 row bid, all 256 nodes (16 waves x one tile of 16) and all
// time slices. The operands are scaled per group of gwaves waves, the columns
// the separate GEMM's blocks cover. The output goes to LDS (rows of
// kFusedStride floats: 4 rows apart, the four row groups of a wave's
// accumulator stores, lie 16 banks apart); each of the 64 lines (slices 2 tp,
// 2 tp + 1) loads its two rows, and after a barrier the same LDS serves the
// row transforms' exchanges.
constexpr int kFusedThreads = 1024;
constexpr int kFusedN = 256;
constexpr int kFusedStride = kFusedN + 4;

// LDS of the fused forward pass: V during the products, then the output tile,
// then the row transforms' exchange areas, in one space of BYTES.
template <int MODE, int NTP>
struct FusedFwdLds {
  using L = LpShape<MODE, NTP>;
  using Sh = fftr::Shape<float, kFusedN>;
  static constexpr int LINES = kFusedThreads / Sh::N2;  // 64 lines: up to 128 time slices
  static constexpr int TILE_BYTES = NTP * kFusedStride * 4;
  static constexpr int VS_BYTES = L::VROWS * NTP * (int)sizeof(typename L::VT);
  static constexpr int SCR_BYTES =
      LINES * (Sh::L > Sh::L2 ? Sh::L : Sh::L2) * (int)sizeof(C2<float>);
  static constexpr int A1 = TILE_BYTES > VS_BYTES ? TILE_BYTES : VS_BYTES;
  static constexpr int BYTES = A1 > SCR_BYTES ? A1 : SCR_BYTES;
};

// XM: 0 no update; 1 the update with x = 0 before it (x written, not read);
// 2 the update. smem: FusedFwdLds bytes; smax: one float per wave; twc: the
// row transform's twiddles (2 N floats) and DCT post-twiddles (2 N floats),
// staged from global memory so the transform phase issues no global loads
// (which would also wait for the x chunk's loads in flight).
template <int MODE, int NTP, int XM>
__device__ __forceinline__ void tgemm_rows_fwd_body(const GemmArgs<double, float>& ga,
                                                    const RowsArgs<float>& ra, const UpdArgs& ua,
                                                    int gwaves, unsigned char* smem, float* smax,
                                                    float* twc) {
  const int bid = blockIdx.x;
  using L = LpShape<MODE, NTP>;
  using VT = typename L::VT;
  using Sh = fftr::Shape<float, kFusedN>;
  constexpr int CB = 1, WAVES = kFusedThreads / 64;
  static_assert(WAVES * CB * 16 == kFusedN, "a block covers one row of 256 nodes");
  static_assert(2 * FusedFwdLds<MODE, NTP>::LINES >= 128, "one pass transforms every slice");
  static_assert(kFusedThreads == 4 * kFusedN, "one thread per staged table entry");
  VT* Vs = reinterpret_cast<VT*>(smem);              // V during the products,
  float* tile = reinterpret_cast<float*>(smem);      // then the output tile,
  C2<float>* scr = reinterpret_cast<C2<float>*>(smem);  // then the exchange areas
  const int nt = ga.nt, M = ga.M;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kq = lane >> 4;
  const int i0 = bid;
  const int col0 = i0 * kFusedN + wave * 16 + (lane & 15);
  const bool dct = ra.ax.kind == 1;
  float xs[CB][L::NKS][L::PER];
  float amax;
  // x += alpha p streamed through the compute phases (XS), or with r in the
  // first phase (the float32 split: its products and conversions leave no
  // registers for the streamed ranges)
  constexpr bool XS = XM != 0 && MODE != GM_F32;
  XStream<MODE, NTP, XM == 1> xst;
  if constexpr (XM != 0) {
    const double alpha = pcg_alpha(ua, bid);
    double rr[1] = {0.0};
    amax = upd_load<MODE, NTP, CB, XM == 1, !XS>(ua, alpha, nt, M, col0, kq, xs, rr[0]);
    lp_stage_v<MODE, NTP>(static_cast<const VT*>(ga.V), Vs, kFusedThreads);
    reduce_store<1>(rr, ua.rb, T_RR, bid);
    const unsigned bytes = (unsigned)nt * (unsigned)M * 8u;
    xst.xr = buf_rsrc(ua.x, bytes);
    xst.pr = buf_rsrc(ua.p, bytes);
    xst.alpha = alpha;
    xst.M = M;
    xst.col0 = col0;
    xst.kq = kq;
  } else {
    amax = lp_load<MODE, NTP, CB>(ga.X, nt, M, col0, kq, xs);
    lp_stage_v<MODE, NTP>(static_cast<const VT*>(ga.V), Vs, kFusedThreads);
  }
  if (L::SCALED) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) smax[wave] = amax;
  }
  __syncthreads();
  // table entry of this thread (written to LDS before the transforms; loaded
  // here, after the update's registers are free)
  float tcv = 0.0f;
  if (threadIdx.x < 2 * kFusedN) tcv = tw_table<float>(ra.ax)[threadIdx.x];
  else if (dct) tcv = ct_table<float>(ra.ax)[threadIdx.x - 2 * kFusedN];
  if constexpr (XS) xst.template load<0>();
  float bm = 0.0f;
  if (L::SCALED) {
    const int g0 = (wave / gwaves) * gwaves;
    bm = smax[g0];
    for (int w = 1; w < gwaves; ++w) bm = fmaxf(bm, smax[g0 + w]);
  }
  float scale, unscale;
  lp_scales<MODE, NTP>(bm, scale, unscale);
  v4f acc[CB][L::NKB];
  lp_mma<MODE, NTP, CB>(Vs, xs, scale, lane, acc);
  if constexpr (XS) {
    xst.template store<0>();
    xst.template load<1>();
  }
  __syncthreads();  // V is no longer read: its LDS takes the output tile
#pragma unroll
  for (int kb = 0; kb < L::NKB; ++kb)
#pragma unroll
    for (int jr = 0; jr < 4; ++jr)
      tile[(kb * 16 + 4 * kq + jr) * kFusedStride + wave * 16 + (lane & 15)] =
          acc[0][kb][jr] * unscale;
  twc[threadIdx.x] = tcv;
  __syncthreads();
  if constexpr (XS) {
    xst.template store<1>();
    xst.template load<2>();
  }
  const int l = threadIdx.x / Sh::N2, p = threadIdx.x % Sh::N2;
  // rows of slices 2 l and 2 l + 1 (tile rows 2 l, 2 l + 1)
  const RowPair rp = row_pair(l * ra.n0 + i0, ra.nrows, ra.n0);
  const float* ta = tile + (2 * l) * kFusedStride;
  const float* tb = ta + kFusedStride;
  C2<float> v[16];
  rows_fwd_load<float, kFusedN>(
      [&](int n) { return C2<float>{rp.hasa ? ta[n] : 0.0f, rp.hasb ? tb[n] : 0.0f}; }, dct, p,
      v);
  __syncthreads();  // the tile is read: its LDS takes the exchange areas
  if constexpr (XS) {
    xst.template store<2>();
    xst.template load<3>();
  }
  float* __restrict__ out = ra.data;
  rows_fwd_xform<float, kFusedN>(
      v,
      [&](int k, float oa, float ob) {
        if (rp.hasa) out[(unsigned)rp.ra * kFusedN + k] = oa;  // n < 2^31
        if (rp.hasb) out[(unsigned)rp.rb * kFusedN + k] = ob;
      },
      dct, scr + l * Sh::L, scr + l * Sh::L2, p, twc, twc + 2 * kFusedN);
  if constexpr (XS) {
    xst.template store<3>();
    xst.template load<4>();
    xst.template store<4>();
  }
}

// UPD: the block first applies the conjugate gradient update to its columns
// (ua; x, r and the r.r partials are written as by the update kernel) and
// takes the new r as the GEMM operand.
template <int MODE, int NTP, bool UPD>
__global__ __launch_bounds__(kFusedThreads) void k_tgemm_rows_fwd(GemmArgs<double, float> ga,
                                                                  RowsArgs<float> ra, UpdArgs ua,
                                                                  int gwaves) {
  if (gemm_skip(ga, blockIdx.x)) return;
  __shared__ __align__(16) unsigned char smem[FusedFwdLds<MODE, NTP>::BYTES];
  __shared__ float smax[kFusedThreads / 64];
  __shared__ float twc[4 * kFusedN];
  if constexpr (UPD) {
    if (ua.first) tgemm_rows_fwd_body<MODE, NTP, 1>(ga, ra, ua, gwaves, smem, smax, twc);
    else tgemm_rows_fwd_body<MODE, NTP, 2>(ga, ra, ua, gwaves, smem, smax, twc);
  } else {
    tgemm_rows_fwd_body<MODE, NTP, 0>(ga, ra, ua, gwaves, smem, smax, twc);
  }
}

// Fused inverse pass (row transforms along axis 1, N = 256, then the inverse
// time GEMM with its r.z (and z.q) partials): the block owns axis-0 row bid.
// Its 64 lines (slices 2 tp, 2 tp + 1) load their spectra from the float32
// intermediate and take the inverse transform, exchanging through LDS; the
// rows then go to an LDS tile in the same space (rows of kInvStride floats:
// the tile's column reads by the four row groups of a wave lie 16 banks
// apart), each wave (one tile of 16 nodes) takes its operands from it, V
// replaces the tile, and the products
// and the epilogue follow the separate GEMM with one 16-node tile per wave:
// operands scaled per group of gwaves waves, each group's partials formed in
// the same order and stored at the index of the separate kernel's block
// (gpr groups per row), so both give the same bits.
constexpr int kInvStride = kFusedStride;

template <int MODE, int NTP>
__global__ __launch_bounds__(kFusedThreads) void k_rows_tgemm_inv(GemmArgs<float, double> ga,
                                                                  RowsArgs<float> ra, int gwaves,
                                                                  int gpr) {
  const int bid = blockIdx.x;
  if (gemm_skip(ga, bid)) return;
  using L = LpShape<MODE, NTP>;
  using VT = typename L::VT;
  using Sh = fftr::Shape<float, kFusedN>;
  constexpr int WAVES = kFusedThreads / 64;
  static_assert(WAVES * 16 == kFusedN, "a block covers one row of 256 nodes");
  constexpr int LINES = kFusedThreads / Sh::N2;
  static_assert(2 * LINES >= 128, "one pass transforms every time slice");
  constexpr int TILE_BYTES = 2 * LINES * kInvStride * 4;
  constexpr int VS_BYTES = L::VROWS * NTP * (int)sizeof(VT);
  constexpr int SCR_BYTES = LINES * (Sh::L > Sh::L2 ? Sh::L : Sh::L2) * (int)sizeof(C2<float>);
  constexpr int A1 = TILE_BYTES > VS_BYTES ? TILE_BYTES : VS_BYTES;
  constexpr int A_BYTES = A1 > SCR_BYTES ? A1 : SCR_BYTES;
  __shared__ __align__(16) unsigned char smem[A_BYTES];
  __shared__ float smax[WAVES];
  __shared__ double dsum[2][WAVES];
  C2<float>* scr = reinterpret_cast<C2<float>*>(smem);  // exchange areas,
  float* tile = reinterpret_cast<float*>(smem);         // then the rows,
  VT* Vs = reinterpret_cast<VT*>(smem);                 // then V
  const int nt = ga.nt, M = ga.M;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kq = lane >> 4;
  const int i0 = bid;
  // inverse row transforms of slices 2 l, 2 l + 1
  const bool dct = ra.ax.kind == 1;
  const int l = threadIdx.x / Sh::N2, p = threadIdx.x % Sh::N2;
  const RowPair rp = row_pair(l * ra.n0 + i0, ra.nrows, ra.n0);
  {
    const float* __restrict__ in = ra.data;
    C2<float> v[16];
    rows_inv_line<float, kFusedN>(
        [&](int k) {
          return C2<float>{rp.hasa ? in[(unsigned)rp.ra * kFusedN + k] : 0.0f,
                           rp.hasb ? in[(unsigned)rp.rb * kFusedN + k] : 0.0f};
        },
        dct, scr + l * Sh::L, p, tw_table<float>(ra.ax), ct_table<float>(ra.ax), v);
    __syncthreads();  // the exchanges are over: their LDS takes the rows
    float* ta = tile + (2 * l) * kInvStride;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int n = p + Sh::N2 * m;
      const int dst = dct ? dct_perm(n, kFusedN) : n;
      ta[dst] = v[m].x;
      ta[kInvStride + dst] = v[m].y;
    }
  }
  __syncthreads();
  // the wave's operands (t = KSTEP ks + PER kq + j; zero beyond N_t)
  float xs[1][L::NKS][L::PER];
  float amax = 0.0f;
#pragma unroll
  for (int ks = 0; ks < L::NKS; ++ks)
#pragma unroll
    for (int j = 0; j < L::PER; ++j) {
      const int t = L::KSTEP * ks + L::PER * kq + j;
      const float v = t < nt ? tile[t * kInvStride + wave * 16 + (lane & 15)] : 0.0f;
      xs[0][ks][j] = v;
      amax = fmaxf(amax, fabsf(v));
    }
  __syncthreads();  // the tile is read: V takes its LDS
  lp_stage_v<MODE, NTP>(static_cast<const VT*>(ga.V), Vs, kFusedThreads);
  if (L::SCALED) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) smax[wave] = amax;
  }
  __syncthreads();
  float bm = 0.0f;
  if (L::SCALED) {
    const int g0 = (wave / gwaves) * gwaves;
    bm = smax[g0];
    for (int w = 1; w < gwaves; ++w) bm = fmaxf(bm, smax[g0 + w]);
  }
  float scale, unscale;
  lp_scales<MODE, NTP>(bm, scale, unscale);
  v4f acc[1][L::NKB];
  lp_mma<MODE, NTP, 1>(Vs, xs, scale, lane, acc);
  // epilogue: z and the dot partials
  const int dotmode = ga.dotmode;
  const double* __restrict__ rvec = ga.rvec;
  const double* __restrict__ qvec = ga.qvec;
  double* __restrict__ Y = ga.Y;
  const int col = i0 * kFusedN + wave * 16 + (lane & 15);
  double dots[2] = {0.0, 0.0};
#pragma unroll
  for (int kb = 0; kb < L::NKB; ++kb)
#pragma unroll
    for (int jr = 0; jr < 4; ++jr) {
      const int k = kb * 16 + 4 * kq + jr;
      if (k < nt) {
        const size_t o = (size_t)k * M + col;
        const double v = (double)(acc[0][kb][jr] * unscale);
        Y[o] = v;
        if (dotmode != DOT_NONE) {
          dots[0] += rvec[o] * v;
          if (dotmode == DOT_FLEX) dots[1] += qvec[o] * v;
        }
      }
    }
  if (dotmode != DOT_NONE) {
    // as reduce_store over the separate kernel's block of gwaves waves: the
    // wave sums, then the group's waves added in order from zero
#pragma unroll
    for (int k = 0; k < 2; ++k) dots[k] = wave_sum(dots[k]);
    if (lane == 0) {
      dsum[0][wave] = dots[0];
      dsum[1][wave] = dots[1];
    }
    __syncthreads();
    if (threadIdx.x < gpr) {
      const int g = threadIdx.x;
      double* part = ga.rb.partials + (size_t)T_RZ * kSlotsPerSite * ga.rb.max_blocks;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        double sum = 0.0;
        for (int w = 0; w < gwaves; ++w) sum += dsum[k][g * gwaves + w];
        part[(size_t)k * ga.rb.max_blocks + i0 * gpr + g] = sum;
      }
    }
  }
}

template <int MODE, int NTP, int CB, typename TX, typename TY, int WPB>
__global__ __launch_bounds__(WPB * 64) void k_tgemm_lp_batch(const GemmArgs<TX, TY>* A,
                                                             const int* off, int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  tgemm_lp_body<MODE, NTP, CB, TX, TY, WPB>(A[i], blockIdx.x - off[i]);
}

// Low-precision products for N_t > 128 (k_tgemm_lps). V (the table of the
// plan's precision, row k contiguous in t, zero-padded to ldv = N_t rounded up
// to 128) is too large for LDS, so it is staged in chunks of TK = 32 time rows:
// a block covers KB*16 output rows and 4 waves x CB tiles of 16 spatial nodes,
// and walks t with the next chunk of V and of its operands fetched into
// registers while the current one is multiplied. The float16 operands are
// scaled per wave and chunk by a power of two that maps the chunk's largest
// magnitude to about 2^14; when that scale changes the accumulators are
// rescaled by the (exact) power-of-two ratio, so they always hold the sum in
// units of the current scale. Blocks of one column block run on one XCD
// (their operand reads share that L2).
constexpr int kLpsTK = 32;           // time rows per chunk
// padded LDS row of 36 halves (18 words): the 16 rows of an A-operand read
// (8 bytes per lane) fall on distinct bank pairs
constexpr int kLpsTKP = kLpsTK + 4;

template <int MODE, int KB, int CB, typename TX, typename TY>
__device__ void tgemm_lps_body(const GemmArgs<TX, TY>& ga, int bid, int nb) {
  if (gemm_skip(ga, bid)) return;
  using VT = typename LpTraits<MODE>::VT;
  constexpr bool SPLIT = MODE == GM_F32;
  constexpr bool SCALED = MODE == GM_F16 || SPLIT;
  constexpr int WPB = 4, KW = KB * 16, TK = kLpsTK, TKP = kLpsTKP, NKS = TK / 16;
  constexpr int NV = SPLIT ? 2 : 1;                  // V terms (hi, lo)
  constexpr int CHUNK16 = NV * KW * TK * 2 / 16;     // 16-byte pieces per V chunk
  constexpr int VPT = CHUNK16 / (WPB * 64);          // per thread
  static_assert(CHUNK16 % (WPB * 64) == 0, "V chunk must split evenly over the block");
  const VT* __restrict__ Vg = static_cast<const VT*>(ga.V);
  const TX* __restrict__ X = ga.X;
  TY* __restrict__ Y = ga.Y;
  const int nt = ga.nt, M = ga.M, ldv = ga.ldv, dotmode = ga.dotmode;
  const int nkc = ldv / KW;
  const int logical = xcd_remap(bid, nb);
  const int cbk = logical / nkc, kc = logical - cbk * nkc;
  const int kbase = kc * KW;
  __shared__ __align__(16) VT Vs[NV * KW * TKP];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4, cl = lane & 15;
  const int col0 = (cbk * WPB + wave) * CB * 16 + cl;
  // V chunk pieces: piece i covers row (i / 4) of term (i / (4 KW)) and 8
  // consecutive t (16 bytes)
  uint4 vreg[VPT];
  TX xn[CB][NKS][4];
  auto fetch = [&](int t0) {
#pragma unroll
    for (int e = 0; e < VPT; ++e) {
      const int i = threadIdx.x + WPB * 64 * e;
      const int term = i / (4 * KW), rem = i - term * 4 * KW;
      const int r = rem >> 2, q = rem & 3;
      const size_t src = ((size_t)term * ldv + kbase + r) * ldv + t0 + 8 * q;
      vreg[e] = *reinterpret_cast<const uint4*>(Vg + src);
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int t = t0 + 16 * ks + 4 * kq + j;
          const int col = col0 + cb * 16;
          xn[cb][ks][j] = (t < nt && col < M) ? X[(size_t)t * M + col] : TX(0);
        }
  };
  v4f acc[CB][KB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc[cb][kb] = (v4f){0.f, 0.f, 0.f, 0.f};
  float scale = 0.0f;  // current operand scale (0: none chosen yet)
  const int nchunk = (nt + TK - 1) / TK;
  fetch(0);
  for (int c = 0; c < nchunk; ++c) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < VPT; ++e) {
      const int i = threadIdx.x + WPB * 64 * e;
      const int term = i / (4 * KW), rem = i - term * 4 * KW;
      const int r = rem >> 2, q = rem & 3;
      // two 8-byte stores: the padded rows (72 bytes) are 8-byte aligned only
      uint2* d = reinterpret_cast<uint2*>(&Vs[(term * KW + r) * TKP + 8 * q]);
      d[0] = make_uint2(vreg[e].x, vreg[e].y);
      d[1] = make_uint2(vreg[e].z, vreg[e].w);
    }
    float xc[CB][NKS][4];
    float amax = 0.0f;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          xc[cb][ks][j] = (float)xn[cb][ks][j];
          amax = fmaxf(amax, fabsf(xc[cb][ks][j]));
        }
    __syncthreads();
    if (c + 1 < nchunk) fetch((c + 1) * TK);
    if constexpr (SCALED) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
      if (amax > 0.0f && __builtin_isfinite(amax)) {
        int e;
        frexpf(amax, &e);           // amax < 2^e
        e = e < -100 ? -100 : e;    // keep 2^(14 - e) finite in float32
        const float sn = ldexpf(1.0f, 14 - e);
        if (scale != 0.0f && sn != scale) {
          const float ratio = sn / scale;  // a power of two: exact
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) acc[cb][kb] *= ratio;
        }
        scale = sn;
      }
    }
    const float sc = (SCALED && scale != 0.0f) ? scale : 1.0f;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      if constexpr (SPLIT) {
        v4h bh[CB], bl[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float xv = xc[cb][ks][j] * sc;
            const _Float16 h = (_Float16)xv;
            bh[cb][j] = h;
            bl[cb][j] = (_Float16)(xv - (float)h);
          }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const int r = kb * 16 + cl;
          const v4h ah = *reinterpret_cast<const v4h*>(&Vs[r * TKP + 16 * ks + 4 * kq]);
          const v4h al = *reinterpret_cast<const v4h*>(&Vs[(KW + r) * TKP + 16 * ks + 4 * kq]);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh[cb], acc[cb][kb], 0, 0, 0);
            acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl[cb], acc[cb][kb], 0, 0, 0);
            acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh[cb], acc[cb][kb], 0, 0, 0);
          }
        }
      } else if constexpr (MODE == GM_F16) {
        v4h b[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int j = 0; j < 4; ++j) b[cb][j] = (_Float16)(xc[cb][ks][j] * sc);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const v4h a =
              *reinterpret_cast<const v4h*>(&Vs[(kb * 16 + cl) * TKP + 16 * ks + 4 * kq]);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[cb][kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b[cb], acc[cb][kb], 0, 0, 0);
        }
      } else {
        v4s b[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int j = 0; j < 4; ++j) b[cb][j] = f2bf(xc[cb][ks][j]);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const v4s a =
              *reinterpret_cast<const v4s*>(&Vs[(kb * 16 + cl) * TKP + 16 * ks + 4 * kq]);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[cb][kb] =
                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[cb], acc[cb][kb], 0, 0, 0);
        }
      }
    }
  }
  const float vunscale = SPLIT ? (float)(1.0 / kVSplitScale) : 1.0f;
  const float unscale = ((SCALED && scale != 0.0f) ? 1.0f / scale : 1.0f) * vunscale;
  double dots[2] = {0.0, 0.0};
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = col0 + cb * 16;
    if (col >= M) continue;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int jr = 0; jr < 4; ++jr) {
        // float32-accumulating 16x16 results: register jr of lane l holds row
        // 4 (l / 16) + jr, column l % 16
        const int k = kbase + kb * 16 + 4 * kq + jr;
        if (k < nt) {
          const size_t o = (size_t)k * M + col;
          const double v = (double)(acc[cb][kb][jr] * unscale);
          Y[o] = (TY)v;
          if (dotmode != DOT_NONE) {
            dots[0] += ga.rvec[o] * v;
            if (dotmode == DOT_FLEX) dots[1] += ga.qvec[o] * v;
          }
        }
      }
  }
  if (dotmode != DOT_NONE) reduce_store<2>(dots, ga.rb, T_RZ, bid);
}

template <int MODE, int KB, int CB, typename TX, typename TY>
__global__ __launch_bounds__(256) void k_tgemm_lps(GemmArgs<TX, TY> a) {
  tgemm_lps_body<MODE, KB, CB, TX, TY>(a, blockIdx.x, gridDim.x);
}

template <int MODE, int KB, int CB, typename TX, typename TY>
__global__ __launch_bounds__(256) void k_tgemm_lps_batch(const GemmArgs<TX, TY>* A,
                                                         const int* off, int ninst) {
  const int i = batch_instance(off, ninst, blockIdx.x);
  tgemm_lps_body<MODE, KB, CB, TX, TY>(A[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

// the streaming kernel's shape: 8 x 16 output rows per block; one 16-node tile
// per wave for the float32 split of float64 operands, two otherwise
template <int MODE, typename TX>
constexpr int lps_cb() {
  return (MODE == GM_F32 && sizeof(TX) == 8) ? 1 : 2;
}
constexpr int kLpsKB = 8;

// Streaming persistent form for N_t <= 128 (NTP = N_t rounded up to 16):
// each block stages all of V in LDS once; each wave then streams 16-node
// column tiles (tile w, w + #waves, ...) with two operand register sets, so
// the global loads of the next tile are in flight while the current one is
// multiplied and stored. float16 / bfloat16 operands are scaled per tile by a
// power of two from the tile's largest magnitude (a wave-level reduction).
// LDS layout: float64 Vs[t][k] (V is symmetric; the f64 A operand is one k
// per lane); low precision the swizzled row-major copy of VsLayout.
template <int MODE>
struct StreamTraits;
template <>
struct StreamTraits<GM_F64> {
  using VT = double;
  static constexpr int KSTEP = 4;
};
template <>
struct StreamTraits<GM_F32> {
  using VT = float;
  static constexpr int KSTEP = 16;
};
template <>
struct StreamTraits<GM_F16> {
  using VT = _Float16;
  static constexpr int KSTEP = 16;
};
template <>
struct StreamTraits<GM_BF16> {
  using VT = unsigned short;
  static constexpr int KSTEP = 16;
};

template <int MODE, int NTP>
struct StreamShape {
  static constexpr int KSTEP = StreamTraits<MODE>::KSTEP;
  static constexpr int PER = KSTEP / 4;   // operand values per lane per step
  static constexpr int NKS = NTP / KSTEP;  // steps
  static constexpr int NKB = NTP / 16;     // 16-row output blocks
  static constexpr int NX = NKS * PER;     // operand values per lane per tile
};

// Operands of one 16-column tile: x[ks * PER + j] = X[t][col], t = KSTEP ks +
// PER kq + j (zero outside the matrix).
template <int MODE, int NTP, typename TX, int NXA>
__device__ __forceinline__ void stream_load(TX (&x)[NXA], const TX* __restrict__ X, int tile,
                                            int nt, int M, int kq, int cl) {
  using Sh = StreamShape<MODE, NTP>;
  const int col = tile * 16 + cl;
  const bool cv = col < M;
#pragma unroll
  for (int ks = 0; ks < Sh::NKS; ++ks)
#pragma unroll
    for (int j = 0; j < Sh::PER; ++j) {
      const int t = Sh::KSTEP * ks + Sh::PER * kq + j;
      x[ks * Sh::PER + j] = (cv && t < nt) ? X[(size_t)t * M + col] : (TX)0;
    }
}

// Multiply one tile, store it and accumulate the dot products.
template <int MODE, int NTP, typename TX, typename TY, int NXA>
__device__ __forceinline__ void stream_tile(const TX (&x)[NXA],
                                            const typename StreamTraits<MODE>::VT* Vs, int tile,
                                            const GemmArgs<TX, TY>& ga, int lane,
                                            double (&dots)[2]) {
  using Sh = StreamShape<MODE, NTP>;
  using VT = typename StreamTraits<MODE>::VT;
  const int nt = ga.nt, M = ga.M, dotmode = ga.dotmode;
  const int kq = lane >> 4, cl = lane & 15;
  const int col = tile * 16 + cl;
  // The A operands of step ks + 1 are read from LDS while step ks multiplies;
  // a scheduling barrier per step keeps the compiler from hoisting every
  // step's reads (which would exhaust the register file).
  if constexpr (MODE == GM_F64) {
    v4d acc[Sh::NKB];
#pragma unroll
    for (int kb = 0; kb < Sh::NKB; ++kb) acc[kb] = (v4d){0.0, 0.0, 0.0, 0.0};
    double a[2][Sh::NKB];
#pragma unroll
    for (int kb = 0; kb < Sh::NKB; ++kb) a[0][kb] = Vs[kq * NTP + kb * 16 + cl];
#pragma unroll
    for (int ks = 0; ks < Sh::NKS; ++ks) {
      if (ks + 1 < Sh::NKS) {
#pragma unroll
        for (int kb = 0; kb < Sh::NKB; ++kb)
          a[(ks + 1) & 1][kb] = Vs[(4 * (ks + 1) + kq) * NTP + kb * 16 + cl];
      }
#pragma unroll
      for (int kb = 0; kb < Sh::NKB; ++kb)
        acc[kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks & 1][kb], (double)x[ks], acc[kb], 0,
                                                       0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (col < M) {
#pragma unroll
      for (int kb = 0; kb < Sh::NKB; ++kb)
#pragma unroll
        for (int jr = 0; jr < 4; ++jr) {
          // f64 result layout: row (l / 16) + 4 jr, column l % 16
          const int k = kb * 16 + kq + 4 * jr;
          if (k < nt) {
            const size_t o = (size_t)k * M + col;
            const double v = acc[kb][jr];
            ga.Y[o] = (TY)v;
            if (dotmode != DOT_NONE) {
              dots[0] += ga.rvec[o] * v;
              if (dotmode == DOT_FLEX) dots[1] += ga.qvec[o] * v;
            }
          }
        }
    }
  } else {
    float scale = 1.0f, unscale = 1.0f;
    if constexpr (MODE == GM_F16) {
      float amax = 0.0f;
#pragma unroll
      for (int i = 0; i < Sh::NX; ++i) amax = fmaxf(amax, fabsf((float)x[i]));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
      if (amax > 0.0f && __builtin_isfinite(amax)) {
        int e;
        frexpf(amax, &e);
        e = e < -100 ? -100 : e;
        scale = ldexpf(1.0f, 14 - e);
        unscale = ldexpf(1.0f, e - 14);
      }
    }
    v4f acc[Sh::NKB];
#pragma unroll
    for (int kb = 0; kb < Sh::NKB; ++kb) acc[kb] = (v4f){0.f, 0.f, 0.f, 0.f};
    // 16 bytes of A per lane and step: 4 floats, or 4 x 16 bits (low half used)
    using AT = typename std::conditional<MODE == GM_F32, v4f, uint2>::type;
    AT a[2][Sh::NKB];
#pragma unroll
    for (int kb = 0; kb < Sh::NKB; ++kb)
      a[0][kb] = *reinterpret_cast<const AT*>(&Vs[VsLayout<NTP, VT>::idx(kb * 16 + cl, 4 * kq)]);
#pragma unroll
    for (int ks = 0; ks < Sh::NKS; ++ks) {
      if (ks + 1 < Sh::NKS) {
#pragma unroll
        for (int kb = 0; kb < Sh::NKB; ++kb)
          a[(ks + 1) & 1][kb] = *reinterpret_cast<const AT*>(
              &Vs[VsLayout<NTP, VT>::idx(kb * 16 + cl, Sh::KSTEP * (ks + 1) + 4 * kq)]);
      }
      if constexpr (MODE == GM_F32) {
#pragma unroll
        for (int kb = 0; kb < Sh::NKB; ++kb)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks & 1][kb][j], (float)x[ks * 4 + j],
                                                           acc[kb], 0, 0, 0);
      } else if constexpr (MODE == GM_F16) {
        v4h b;
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = (_Float16)((float)x[ks * 4 + j] * scale);
#pragma unroll
        for (int kb = 0; kb < Sh::NKB; ++kb) {
          v4h av;
          __builtin_memcpy(&av, &a[ks & 1][kb], sizeof(av));
          acc[kb] = __builtin_amdgcn_mfma_f32_16x16x16f16(av, b, acc[kb], 0, 0, 0);
        }
      } else {
        v4s b;
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = f2bf((float)x[ks * 4 + j]);
#pragma unroll
        for (int kb = 0; kb < Sh::NKB; ++kb) {
          v4s av;
          __builtin_memcpy(&av, &a[ks & 1][kb], sizeof(av));
          acc[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b, acc[kb], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (col < M) {
#pragma unroll
      for (int kb = 0; kb < Sh::NKB; ++kb)
#pragma unroll
        for (int jr = 0; jr < 4; ++jr) {
          // float32-accumulating 16x16 results: row 4 (l / 16) + jr, column l % 16
          const int k = kb * 16 + 4 * kq + jr;
          if (k < nt) {
            const size_t o = (size_t)k * M + col;
            const double v = (double)(acc[kb][jr] * unscale);
            ga.Y[o] = (TY)v;
            if (dotmode != DOT_NONE) {
              dots[0] += ga.rvec[o] * v;
              if (dotmode == DOT_FLEX) dots[1] += ga.qvec[o] * v;
            }
          }
        }
    }
  }
}

template <int MODE, int NTP, int WAVES, typename TX, typename TY>
__global__ __launch_bounds__(WAVES * 64) void k_tgemm_stream(GemmArgs<TX, TY> ga) {
  if (gemm_skip(ga, (int)blockIdx.x)) return;
  using VT = typename StreamTraits<MODE>::VT;
  using Sh = StreamShape<MODE, NTP>;
  constexpr int NT = WAVES * 64;
  __shared__ __align__(16) VT Vs[NTP * NTP];
  {
    constexpr int NV16 = NTP * NTP * (int)sizeof(VT) / 16;
    const uint4* src = reinterpret_cast<const uint4*>(ga.V);
    uint4* dst = reinterpret_cast<uint4*>(Vs);
    for (int i = threadIdx.x; i < NV16; i += NT)
      dst[MODE == GM_F64 ? i : VsLayout<NTP, VT>::chunk(i)] = src[i];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4, cl = lane & 15;
  const int ntiles = (ga.M + 15) / 16;
  const int stride = gridDim.x * WAVES;
  double dots[2] = {0.0, 0.0};
  TX xa[Sh::NX], xb[Sh::NX];
  int tile = blockIdx.x * WAVES + wave;
  if (tile < ntiles) stream_load<MODE, NTP>(xa, ga.X, tile, ga.nt, ga.M, kq, cl);
  while (tile < ntiles) {
    int next = tile + stride;
    if (next < ntiles) stream_load<MODE, NTP>(xb, ga.X, next, ga.nt, ga.M, kq, cl);
    stream_tile<MODE, NTP>(xa, Vs, tile, ga, lane, dots);
    tile = next;
    if (tile >= ntiles) break;
    next = tile + stride;
    if (next < ntiles) stream_load<MODE, NTP>(xa, ga.X, next, ga.nt, ga.M, kq, cl);
    stream_tile<MODE, NTP>(xb, Vs, tile, ga, lane, dots);
    tile = next;
  }
  if (ga.dotmode != DOT_NONE) reduce_store<2>(dots, ga.rb, T_RZ, blockIdx.x);
}

template <int MODE, int NTP, typename TX, typename TY>
int stream_launch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r,
                  const double* q, hipStream_t s) {
  const int M = P.g.M;
  const int ntiles = (M + 15) / 16;
  // 4 waves a block; float64: one block per CU (V takes up to 128 KB of LDS,
  // each wave has a SIMD's whole register file); low precision: two blocks
  constexpr int WAVES = 4;
  const int per_cu = (MODE == GM_F64) ? 1 : 2;
  int grid = P.num_cus * per_cu;
  const int need = (ntiles + WAVES - 1) / WAVES;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  const void* V = (MODE == GM_F64) ? (const void*)P.Vp64
                  : (MODE == GM_F32) ? (const void*)P.Vp32
                  : (MODE == GM_F16) ? (const void*)P.Vp16 : (const void*)P.Vpbf;
  const GemmArgs<TX, TY> a{V, X, Y, P.g.nt, M, 0, dotmode, r, q, P.red, P.pcg_done, P.rr_gate};
  hipLaunchKernelGGL((k_tgemm_stream<MODE, NTP, WAVES, TX, TY>), dim3(grid), dim3(WAVES * 64), 0,
                     s, a);
  return grid;
}

template <int MODE, typename TX, typename TY>
int pers_dispatch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r,
                  const double* q, hipStream_t s) {
  switch (P.ntp) {
    case 16: return stream_launch<MODE, 16>(P, X, Y, dotmode, r, q, s);
    case 32: return stream_launch<MODE, 32>(P, X, Y, dotmode, r, q, s);
    case 48: return stream_launch<MODE, 48>(P, X, Y, dotmode, r, q, s);
    case 64: return stream_launch<MODE, 64>(P, X, Y, dotmode, r, q, s);
    case 80: return stream_launch<MODE, 80>(P, X, Y, dotmode, r, q, s);
    case 96: return stream_launch<MODE, 96>(P, X, Y, dotmode, r, q, s);
    case 112: return stream_launch<MODE, 112>(P, X, Y, dotmode, r, q, s);
    default: return stream_launch<MODE, 128>(P, X, Y, dotmode, r, q, s);
  }
}

const void* lp_table(const Plan& P, int mode) {
  return (mode == GM_F32) ? (const void*)P.Vp16s
         : (mode == GM_F16) ? (const void*)P.Vp16 : (const void*)P.Vpbf;
}

template <int MODE, int NTP, int CB, int WPB, typename TX, typename TY>
int lp_launch_cb(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
                 hipStream_t s) {
  const int M = P.g.M;
  const int grid = (M + 16 * WPB * CB - 1) / (16 * WPB * CB);
  const GemmArgs<TX, TY> a{lp_table(P, MODE), X, Y, P.g.nt, M, 0, dotmode, r, q, P.red,
                           P.pcg_done, P.rr_gate};
  hipLaunchKernelGGL((k_tgemm_lp<MODE, NTP, CB, TX, TY, WPB>), dim3(grid), dim3(WPB * 64), 0, s,
                     a);
  return grid;
}

// Launch shape by direction: forward (float64 in) or inverse (float64 out).
template <int MODE, int NTP, typename TX, typename TY>
int lp_launch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
              hipStream_t s) {
  const bool fwd = std::is_same<TX, double>::value;
  const int cb = fwd ? P.tune.lp_cb : P.tune.lp_cb_i;
  const int waves = fwd ? P.tune.lp_waves : P.tune.lp_waves_i;
  if (waves == 8) {
    if (cb == 1) return lp_launch_cb<MODE, NTP, 1, 8>(P, X, Y, dotmode, r, q, s);
    return lp_launch_cb<MODE, NTP, 2, 8>(P, X, Y, dotmode, r, q, s);
  }
  if (cb == 1) return lp_launch_cb<MODE, NTP, 1, 4>(P, X, Y, dotmode, r, q, s);
  return lp_launch_cb<MODE, NTP, 2, 4>(P, X, Y, dotmode, r, q, s);
}

template <int MODE, typename TX, typename TY>
int lp_dispatch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
                hipStream_t s) {
  switch (P.ntp) {
    case 16: return lp_launch<MODE, 16>(P, X, Y, dotmode, r, q, s);
    case 32: return lp_launch<MODE, 32>(P, X, Y, dotmode, r, q, s);
    case 48: return lp_launch<MODE, 48>(P, X, Y, dotmode, r, q, s);
    case 64: return lp_launch<MODE, 64>(P, X, Y, dotmode, r, q, s);
    case 80: return lp_launch<MODE, 80>(P, X, Y, dotmode, r, q, s);
    case 96: return lp_launch<MODE, 96>(P, X, Y, dotmode, r, q, s);
    case 112: return lp_launch<MODE, 112>(P, X, Y, dotmode, r, q, s);
    default: return lp_launch<MODE, 128>(P, X, Y, dotmode, r, q, s);
  }
}

template <int KB, int CB, typename TX, typename TY>
int f64_launch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
               hipStream_t s) {
  const int nt = P.g.nt, M = P.g.M;
  const int ncolblk = (M + 64 * CB - 1) / (64 * CB);
  const int nkc = (nt + KB * 16 - 1) / (KB * 16);
  const int grid = ncolblk * nkc;
  const GemmArgs<TX, TY> a{P.Vt64, X, Y, nt, M, ncolblk, dotmode, r, q, P.red, P.pcg_done,
                           P.rr_gate};
  hipLaunchKernelGGL((k_tgemm64<KB, CB, TX, TY>), dim3(grid), dim3(256), 0, s, a);
  return grid;
}


template <int MODE, typename TX, typename TY>
int lps_launch(const Plan& P, const TX* X, TY* Y, int dotmode, const double* r, const double* q,
               hipStream_t s) {
  // the float32 split of float64 operands (its forward transform) takes one
  // 16-node tile per wave: its prefetched registers would otherwise leave one
  // wave per SIMD (221 against 275 us at 64^2 x 2048); float16 and bfloat16
  // keep two (117 against 147 us)
  constexpr int KB = kLpsKB, CB = lps_cb<MODE, TX>();
  const int M = P.g.M;
  const int ncolblk = (M + 4 * CB * 16 - 1) / (4 * CB * 16);
  const int grid = ncolblk * (P.ntps / (KB * 16));
  GemmArgs<TX, TY> a{P.Vs_lp, X, Y, P.g.nt, M, ncolblk, dotmode, r, q, P.red, P.pcg_done,
                     P.rr_gate};
  a.ldv = P.ntps;
  hipLaunchKernelGGL((k_tgemm_lps<MODE, KB, CB, TX, TY>), dim3(grid), dim3(256), 0, s, a);
  return grid;
}

template <typename TX, typename TY>
int tgemm_launch(const Plan& P, int mode, const TX* X, TY* Y, int dotmode, const double* r,
                 const double* q, hipStream_t s) {
  const int nt = P.g.nt;
  if constexpr (!std::is_same<TX, double>::value || !std::is_same<TY, double>::value) {
    if (mode != GM_F64 && P.ntp == 0 && P.ntps > 0 && P.tune.lp_stream) {
      if (mode == GM_F32) return lps_launch<GM_F32>(P, X, Y, dotmode, r, q, s);
      if (mode == GM_F16) return lps_launch<GM_F16>(P, X, Y, dotmode, r, q, s);
      return lps_launch<GM_BF16>(P, X, Y, dotmode, r, q, s);
    }
  }
  if (P.ntp > 0 && P.tune.tgemm_pers) {
    if (mode == GM_F64) return pers_dispatch<GM_F64>(P, X, Y, dotmode, r, q, s);
    if (mode == GM_F32) return pers_dispatch<GM_F32>(P, X, Y, dotmode, r, q, s);
    if (mode == GM_F16) return pers_dispatch<GM_F16>(P, X, Y, dotmode, r, q, s);
    return pers_dispatch<GM_BF16>(P, X, Y, dotmode, r, q, s);
  }
  if (mode != GM_F64 && P.ntp > 0) {
    if (mode == GM_F32) return lp_dispatch<GM_F32>(P, X, Y, dotmode, r, q, s);
    if (mode == GM_F16) return lp_dispatch<GM_F16>(P, X, Y, dotmode, r, q, s);
    return lp_dispatch<GM_BF16>(P, X, Y, dotmode, r, q, s);
  }
  if (P.tune.f64_cb == 1) {
    if (nt <= 32) return f64_launch<2, 1>(P, X, Y, dotmode, r, q, s);
    if (nt <= 64) return f64_launch<4, 1>(P, X, Y, dotmode, r, q, s);
    return f64_launch<8, 1>(P, X, Y, dotmode, r, q, s);
  }
  if (nt <= 32) return f64_launch<2, 2>(P, X, Y, dotmode, r, q, s);
  if (nt <= 64) return f64_launch<4, 2>(P, X, Y, dotmode, r, q, s);
  return f64_launch<8, 2>(P, X, Y, dotmode, r, q, s);
}

}  // namespace

template <typename TX, typename TY>
void tgemm(const Plan& P, int mode, const TX* X, TY* Y, int dotmode, const double* r,
           const double* q, hipStream_t s, const char* name) {
  int grid;
  {
    ProfScope ps(P, name, s);
    grid = tgemm_launch(P, mode, X, Y, dotmode, r, q, s);
  }
  // the r.z (and z.q) partials are summed by the kernels that consume them
  if (dotmode != DOT_NONE) P.rz_blocks = grid;
}

template void tgemm<double, double>(const Plan&, int, const double*, double*, int,
                                    const double*, const double*, hipStream_t, const char*);
template void tgemm<double, float>(const Plan&, int, const double*, float*, int,
                                    const double*, const double*, hipStream_t, const char*);
template void tgemm<float, double>(const Plan&, int, const float*, double*, int,
                                    const double*, const double*, hipStream_t, const char*);

bool fused_fwd_ok(const Plan& P) {
  return P.tune.fuse_fwd && P.precision != MFG_FP64 && P.g.has0 && P.g.n1 == kFusedN &&
         P.tune.fft_reg && P.ntp > 0 && !P.tune.tgemm_pers;
}

bool fused_upd_ok(const Plan& P) {
  // the update addresses its vectors through 32-bit byte offsets
  return P.tune.fuse_upd && P.pcg_done && fused_fwd_ok(P) &&
         (long long)P.ntp * P.g.M * 8 < (1LL << 31);
}

template <int MODE, bool UPD>
void fused_dispatch(const Plan& P, const GemmArgs<double, float>& ga, const RowsArgs<float>& ra,
                    const UpdArgs& ua, int gwaves, hipStream_t s) {
  const dim3 g(P.g.n0), b(kFusedThreads);
#define MFG_FUSED(NTPV)                                                                  \
  case NTPV:                                                                             \
    hipLaunchKernelGGL((k_tgemm_rows_fwd<MODE, NTPV, UPD>), g, b, 0, s, ga, ra, ua, gwaves); \
    break;
  switch (P.ntp) {
    MFG_FUSED(16)
    MFG_FUSED(32)
    MFG_FUSED(48)
    MFG_FUSED(64)
    MFG_FUSED(80)
    MFG_FUSED(96)
    MFG_FUSED(112)
    default: MFG_FUSED(128)
  }
#undef MFG_FUSED
}

void launch_tgemm_rows_fwd(const Plan& P, int mode, const double* r, float* tmp,
                           const RowsArgs<float>& ra, const UpdArgs* ua, hipStream_t s) {
  // operands scaled in the separate forward GEMM's groups: lp_waves x lp_cb
  // tiles of 16 nodes, i.e. that many waves of this kernel
  const int gwaves = (P.tune.lp_waves == 8 ? 8 : 4) * (P.tune.lp_cb == 1 ? 1 : 2);
  // with the update the stopping test is left to a later kernel (nrr = 0)
  const GemmArgs<double, float> ga{lp_table(P, mode), r,       tmp,     P.g.nt,     P.g.M,
                                   0,                 DOT_NONE, nullptr, nullptr,    P.red,
                                   P.pcg_done,        ua ? 0 : P.rr_gate};
  const UpdArgs u = ua ? *ua : UpdArgs{};
  if (ua) {
    if (mode == GM_F32) fused_dispatch<GM_F32, true>(P, ga, ra, u, gwaves, s);
    else if (mode == GM_F16) fused_dispatch<GM_F16, true>(P, ga, ra, u, gwaves, s);
    else fused_dispatch<GM_BF16, true>(P, ga, ra, u, gwaves, s);
  } else {
    if (mode == GM_F32) fused_dispatch<GM_F32, false>(P, ga, ra, u, gwaves, s);
    else if (mode == GM_F16) fused_dispatch<GM_F16, false>(P, ga, ra, u, gwaves, s);
    else fused_dispatch<GM_BF16, false>(P, ga, ra, u, gwaves, s);
  }
}

bool fused_inv_ok(const Plan& P) {
  return P.tune.fuse_inv && P.precision != MFG_FP64 && P.g.has0 && P.g.n1 == kFusedN &&
         P.tune.fft_reg && P.ntp > 0 && !P.tune.tgemm_pers && P.tune.lp_cb_i == 1;
}

template <int MODE>
void fused_inv_dispatch(const Plan& P, const GemmArgs<float, double>& ga,
                        const RowsArgs<float>& ra, int gwaves, int gpr, hipStream_t s) {
  const dim3 g(P.g.n0), b(kFusedThreads);
#define MFG_FUSED_INV(NTPV)                                                                \
  case NTPV:                                                                               \
    hipLaunchKernelGGL((k_rows_tgemm_inv<MODE, NTPV>), g, b, 0, s, ga, ra, gwaves, gpr);  \
    break;
  switch (P.ntp) {
    MFG_FUSED_INV(16)
    MFG_FUSED_INV(32)
    MFG_FUSED_INV(48)
    MFG_FUSED_INV(64)
    MFG_FUSED_INV(80)
    MFG_FUSED_INV(96)
    MFG_FUSED_INV(112)
    default: MFG_FUSED_INV(128)
  }
#undef MFG_FUSED_INV
}

int launch_rows_tgemm_inv(const Plan& P, int mode, const RowsArgs<float>& ra, double* z,
                          int dotmode, const double* r, const double* q, hipStream_t s) {
  // the separate inverse GEMM's blocks: lp_waves_i tiles of 16 nodes (one per
  // wave here), gpr of them per row of 256 nodes
  const int gwaves = P.tune.lp_waves_i == 8 ? 8 : 4;
  const int gpr = kFusedN / (16 * gwaves);
  const GemmArgs<float, double> ga{lp_table(P, mode), ra.data, z,       P.g.nt,     P.g.M,
                                   0,                 dotmode, r,       q,          P.red,
                                   P.pcg_done,        P.rr_gate};
  if (mode == GM_F32) fused_inv_dispatch<GM_F32>(P, ga, ra, gwaves, gpr, s);
  else if (mode == GM_F16) fused_inv_dispatch<GM_F16>(P, ga, ra, gwaves, gpr, s);
  else fused_inv_dispatch<GM_BF16>(P, ga, ra, gwaves, gpr, s);
  return P.g.n0 * gpr;
}

// ---- batched low-precision time GEMM (one N_t padding class per launch) ----
template <typename TX, typename TY>
GemmArgs<TX, TY> batch_gemm_args(const Plan& P, int mode, const TX* X, TY* Y, int dotmode,
                                 const double* r, const double* q, const double* done,
                                 int* blocks) {
  // batched plans use one shape for both directions (the forward one)
  const int cb = P.tune.lp_cb == 1 ? 1 : 2;
  const int cols = 16 * (P.tune.lp_waves == 8 ? 8 : 4) * cb;
  *blocks = (P.g.M + cols - 1) / cols;
  return GemmArgs<TX, TY>{lp_table(P, mode), X, Y, P.g.nt, P.g.M, 0, dotmode, r, q, P.red, done,
                          0};
}

template <int MODE, int CB, int WPB, typename TX, typename TY>
void lp_batch_dispatch(int ntp, const GemmArgs<TX, TY>* A, const int* off, int ninst, int total,
                       hipStream_t s) {
#define MFG_LPB(NTPV)                                                                     \
  case NTPV:                                                                              \
    hipLaunchKernelGGL((k_tgemm_lp_batch<MODE, NTPV, CB, TX, TY, WPB>), dim3(total),     \
                       dim3(WPB * 64), 0, s, A, off, ninst);                              \
    break;
  switch (ntp) {
    MFG_LPB(16)
    MFG_LPB(32)
    MFG_LPB(48)
    MFG_LPB(64)
    MFG_LPB(80)
    MFG_LPB(96)
    MFG_LPB(112)
    default:
      hipLaunchKernelGGL((k_tgemm_lp_batch<MODE, 128, CB, TX, TY, WPB>), dim3(total),
                         dim3(WPB * 64), 0, s, A, off, ninst);
  }
#undef MFG_LPB
}

template <int MODE, typename TX, typename TY>
void lp_batch_cb(int ntp, int cb, int waves, const GemmArgs<TX, TY>* A, const int* off, int ninst,
                 int total, hipStream_t s) {
  if (waves == 8) {
    if (cb == 1) lp_batch_dispatch<MODE, 1, 8>(ntp, A, off, ninst, total, s);
    else lp_batch_dispatch<MODE, 2, 8>(ntp, A, off, ninst, total, s);
  } else {
    if (cb == 1) lp_batch_dispatch<MODE, 1, 4>(ntp, A, off, ninst, total, s);
    else lp_batch_dispatch<MODE, 2, 4>(ntp, A, off, ninst, total, s);
  }
}

template <typename TX, typename TY>
void launch_gemm_batch(int mode, int ntp, int cb, int waves, const GemmArgs<TX, TY>* A,
                       const int* off, int ninst, int total, hipStream_t s) {
  if (mode == GM_F32) lp_batch_cb<GM_F32>(ntp, cb, waves, A, off, ninst, total, s);
  else if (mode == GM_F16) lp_batch_cb<GM_F16>(ntp, cb, waves, A, off, ninst, total, s);
  else lp_batch_cb<GM_BF16>(ntp, cb, waves, A, off, ninst, total, s);
}

// ---- batched streaming low-precision time GEMM (N_t > 128) ----
template <typename TX, typename TY>
GemmArgs<TX, TY> batch_gemm_lps_args(const Plan& P, int mode, const TX* X, TY* Y, int dotmode,
                                     const double* r, const double* q, const double* done,
                                     int* blocks) {
  const int cb = mode == GM_F32 ? (sizeof(TX) == 8 ? lps_cb<GM_F32, double>()
                                                   : lps_cb<GM_F32, float>())
                                : 2;
  const int M = P.g.M;
  const int ncolblk = (M + 4 * cb * 16 - 1) / (4 * cb * 16);
  *blocks = ncolblk * (P.ntps / (kLpsKB * 16));
  GemmArgs<TX, TY> a{P.Vs_lp, X, Y, P.g.nt, M, ncolblk, dotmode, r, q, P.red, done, 0};
  a.ldv = P.ntps;
  return a;
}

template <typename TX, typename TY>
void launch_gemm_lps_batch(int mode, const GemmArgs<TX, TY>* A, const int* off, int ninst,
                           int total, hipStream_t s) {
  const dim3 g(total), b(256);
  if (mode == GM_F32)
    hipLaunchKernelGGL((k_tgemm_lps_batch<GM_F32, kLpsKB, lps_cb<GM_F32, TX>(), TX, TY>), g, b,
                       0, s, A, off, ninst);
  else if (mode == GM_F16)
    hipLaunchKernelGGL((k_tgemm_lps_batch<GM_F16, kLpsKB, lps_cb<GM_F16, TX>(), TX, TY>), g, b,
                       0, s, A, off, ninst);
  else
    hipLaunchKernelGGL((k_tgemm_lps_batch<GM_BF16, kLpsKB, lps_cb<GM_BF16, TX>(), TX, TY>), g,
                       b, 0, s, A, off, ninst);
}

template GemmArgs<double, float> batch_gemm_lps_args(const Plan&, int, const double*, float*, int,
                                                     const double*, const double*,
                                                     const double*, int*);
template GemmArgs<float, double> batch_gemm_lps_args(const Plan&, int, const float*, double*, int,
                                                     const double*, const double*,
                                                     const double*, int*);
template void launch_gemm_lps_batch(int, const GemmArgs<double, float>*, const int*, int, int,
                                    hipStream_t);
template void launch_gemm_lps_batch(int, const GemmArgs<float, double>*, const int*, int, int,
                                    hipStream_t);

// ---- batched float64 time GEMM (one (KB, CB) class per launch) ----
GemmArgs<double, double> batch_gemm64_args(const Plan& P, const double* X, double* Y, int dotmode,
                                           const double* r, const double* q, const double* done,
                                           int* blocks, int* kb, int* cb) {
  // the single-plan choice of f64_launch (any N_t: the k rows come in chunks)
  const int nt = P.g.nt, M = P.g.M;
  *kb = nt <= 32 ? 2 : (nt <= 64 ? 4 : 8);
  *cb = P.tune.f64_cb == 1 ? 1 : 2;
  const int ncolblk = (M + 64 * *cb - 1) / (64 * *cb);
  *blocks = ncolblk * ((nt + *kb * 16 - 1) / (*kb * 16));
  return GemmArgs<double, double>{P.Vt64, X, Y, nt, M, ncolblk, dotmode, r, q, P.red, done, 0};
}

void launch_gemm64_batch(int kb, int cb, const GemmArgs<double, double>* A, const int* off,
                         int ninst, int total, hipStream_t s) {
  const dim3 g(total), b(256);
  if (cb == 1) {
    if (kb == 2) hipLaunchKernelGGL((k_tgemm64_batch<2, 1>), g, b, 0, s, A, off, ninst);
    else if (kb == 4) hipLaunchKernelGGL((k_tgemm64_batch<4, 1>), g, b, 0, s, A, off, ninst);
    else hipLaunchKernelGGL((k_tgemm64_batch<8, 1>), g, b, 0, s, A, off, ninst);
  } else {
    if (kb == 2) hipLaunchKernelGGL((k_tgemm64_batch<2, 2>), g, b, 0, s, A, off, ninst);
    else if (kb == 4) hipLaunchKernelGGL((k_tgemm64_batch<4, 2>), g, b, 0, s, A, off, ninst);
    else hipLaunchKernelGGL((k_tgemm64_batch<8, 2>), g, b, 0, s, A, off, ninst);
  }
}

template GemmArgs<double, float> batch_gemm_args(const Plan&, int, const double*, float*, int,
                                                 const double*, const double*, const double*,
                                                 int*);
template GemmArgs<float, double> batch_gemm_args(const Plan&, int, const float*, double*, int,
                                                 const double*, const double*, const double*,
                                                 int*);
template void launch_gemm_batch(int, int, int, int, const GemmArgs<double, float>*, const int*,
                                int, int, hipStream_t);
template void launch_gemm_batch(int, int, int, int, const GemmArgs<float, double>*, const int*,
                                int, int, hipStream_t);

}  // namespace mfg
