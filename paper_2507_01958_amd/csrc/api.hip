// C ABI entry points (include/mfg.h): plan construction, operators, PCG and
// the Chambolle-Pock driver.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <utility>
#include <string>
#include <vector>

#include "plan.h"

namespace mfg {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(MFG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

static bool size_ok(int N) {
  if (N < 4 || N > kMaxAxisN) return false;
  int n = N;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

void radices(int N, int* r, int* np) {
  int n = N, k = 0;
  while (n % 4 == 0) { r[k++] = 4; n /= 4; }
  while (n % 2 == 0) { r[k++] = 2; n /= 2; }
  while (n % 3 == 0) { r[k++] = 3; n /= 3; }
  *np = k;
}

template <typename T>
static int dalloc(Plan& P, T** ptr, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(T) + 256);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MFG_ERR_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  P.dev_allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return MFG_OK;
}

template <typename T>
static int upload(Plan& P, T** dst, const std::vector<T>& h) {
  int rc = dalloc(P, dst, h.size());
  if (rc) return rc;
  HIP_TRY(hipMemcpy(*dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return MFG_OK;
}

static unsigned short to_bf16(float f) {
  unsigned int u;
  std::memcpy(&u, &f, 4);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest even
  return (unsigned short)(u >> 16);
}

// One spatial axis: FFT plan, twiddles, DCT post-twiddles and the eigenvalues
// of the one-axis negative Laplacian divided by h^2 (Algorithm 2).
static int build_axis(Plan& P, Axis& ax, int N, bool neumann, double h) {
  ax.N = N;
  radices(N, ax.radix, &ax.npass);
  ax.kind = neumann ? 1 : 0;
  std::vector<double> tw(2 * N), ct(2 * N), lam(N);
  std::vector<float> twf(2 * N), ctf(2 * N);
  const double pi = 3.14159265358979323846264338327950288;
  for (int m = 0; m < N; ++m) {
    tw[2 * m] = std::cos(2.0 * pi * m / N);
    tw[2 * m + 1] = std::sin(2.0 * pi * m / N);
    ct[2 * m] = std::cos(pi * m / (2.0 * N));
    ct[2 * m + 1] = std::sin(pi * m / (2.0 * N));
    const double ev = neumann ? 2.0 - 2.0 * std::cos(pi * m / N) : 2.0 - 2.0 * std::cos(2.0 * pi * m / N);
    lam[m] = ev / (h * h);
  }
  for (int i = 0; i < 2 * N; ++i) {
    twf[i] = (float)tw[i];
    ctf[i] = (float)ct[i];
  }
  double *dtw, *dct, *dlam;
  float *dtwf, *dctf;
  int rc;
  if ((rc = upload(P, &dtw, tw)) || (rc = upload(P, &dct, ct)) || (rc = upload(P, &dlam, lam)) ||
      (rc = upload(P, &dtwf, twf)) || (rc = upload(P, &dctf, ctf)))
    return rc;
  ax.tw = dtw;
  ax.ct = dct;
  ax.lam = dlam;
  ax.twf = dtwf;
  ax.ctf = dctf;
  return MFG_OK;
}

static int check_fields(const Plan& P, const double* V, const double* m0, bool need_both) {
  const int M = P.g.M;
  std::vector<double> h(M);
  if (V) {
    HIP_TRY(hipMemcpy(h.data(), V, M * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < M; ++i)
      if (!std::isfinite(h[i])) return fail(MFG_ERR_NONFINITE, "V has a non-finite entry");
  } else if (need_both) {
    return fail(MFG_ERR_INVALID_ARG, "V is NULL");
  }
  if (m0) {
    HIP_TRY(hipMemcpy(h.data(), m0, M * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < M; ++i) {
      if (!std::isfinite(h[i])) return fail(MFG_ERR_NONFINITE, "m0 has a non-finite entry");
      if (h[i] < 0.0) return fail(MFG_ERR_INVALID_ARG, "m0 has a negative entry");
    }
  } else if (need_both) {
    return fail(MFG_ERR_INVALID_ARG, "m0 is NULL");
  }
  return MFG_OK;
}

static void release(Plan& P) {
  if (P.stream) (void)hipStreamSynchronize(P.stream);
  else (void)hipDeviceSynchronize();
  for (auto& r : P.prof.pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : P.prof.pool) (void)hipEventDestroy(e);
  P.prof.pending.clear();
  P.prof.pool.clear();
  for (void* p : P.dev_allocs) (void)hipFree(p);
  for (void* p : P.host_allocs) (void)hipHostFree(p);
  P.dev_allocs.clear();
  P.host_allocs.clear();
}

// MFG_TUNE="key=value,..." overrides launch-shape choices (see Tune).
static void read_tune_env(Tune& t) {
  const char* env = std::getenv("MFG_TUNE");
  if (!env) return;
  std::string str(env);
  size_t pos = 0;
  while (pos < str.size()) {
    size_t end = str.find(',', pos);
    if (end == std::string::npos) end = str.size();
    const std::string kv = str.substr(pos, end - pos);
    const size_t eq = kv.find('=');
    if (eq != std::string::npos) {
      const std::string k = kv.substr(0, eq);
      const int v = std::atoi(kv.c_str() + eq + 1);
      if (k == "f64_cb" && (v == 1 || v == 2)) t.f64_cb = v;
      else if (k == "lp_cb" && (v == 1 || v == 2)) t.lp_cb = v;
      else if (k == "lp_waves" && (v == 4 || v == 8)) t.lp_waves = v;
      else if (k == "lp_cb_i" && (v == 1 || v == 2)) t.lp_cb_i = v;
      else if (k == "lp_waves_i" && (v == 4 || v == 8)) t.lp_waves_i = v;
      else if (k == "rows_elems" && v >= 64 && v <= 8192) t.rows_elems = v;
      else if (k == "cols_lines" && v >= 1 && v <= 16) t.cols_lines = v;
      else if (k == "tgemm_pers" && (v == 0 || v == 1)) t.tgemm_pers = v;
      else if (k == "fft_reg" && (v == 0 || v == 1)) t.fft_reg = v;
      else if (k == "aat_tc" && v >= 0 && v <= 64) t.aat_tc = v;
      else if (k == "aat_big" && v >= 0 && v <= 2) t.aat_big = v;
      else if (k == "flex" && (v >= -1 && v <= 1)) t.flex = v;
      else if (k == "lp_stream" && (v == 0 || v == 1)) t.lp_stream = v;
      else if (k == "rhs_tc" && v >= 0 && v <= 64) t.rhs_tc = v;
      else if (k == "fuse_fwd" && (v == 0 || v == 1)) t.fuse_fwd = v;
      else if (k == "fuse_upd" && (v == 0 || v == 1)) t.fuse_upd = v;
      else if (k == "fuse_inv" && (v == 0 || v == 1)) t.fuse_inv = v;
      else if (k == "batch_queue" && (v == 0 || v == 1)) t.batch_queue = v;
    }
    pos = end + 1;
  }
}

bool axis_neumann(const mfg_problem_t* pb, int a) {
  switch (pb->bc) {
    case MFG_BC_NEUMANN: return true;
    case MFG_BC_PERIODIC_X_NEUMANN_Y: return a == 1;
    case MFG_BC_NEUMANN_X_PERIODIC_Y: return a == 0;
    default: return false;
  }
}

double axis_spacing(const mfg_problem_t* pb, int a) {
  const double L = pb->hi[a] - pb->lo[a];
  return axis_neumann(pb, a) ? L / (pb->n[a] + 1) : L / pb->n[a];
}

// Validate the problem and fill the plan's geometry and scalars (no device
// allocation, no table).
int setup_problem(Plan& P, const mfg_problem_t* pb, hipStream_t stream) {
  if (!pb) return fail(MFG_ERR_INVALID_ARG, "problem is NULL");
  if (pb->d != 1 && pb->d != 2) return fail(MFG_ERR_INVALID_ARG, "d must be 1 or 2");
  for (int a = 0; a < pb->d; ++a) {
    if (pb->n[a] < 4) return fail(MFG_ERR_INVALID_ARG, "each axis needs at least 4 nodes");
    if (!size_ok(pb->n[a]))
      return fail(MFG_ERR_UNSUPPORTED, "axis sizes must be 2^a 3^b and at most 1024");
    if (!(pb->hi[a] > pb->lo[a]) || !std::isfinite(pb->hi[a] - pb->lo[a]))
      return fail(MFG_ERR_INVALID_ARG, "domain needs hi > lo");
  }
  if (pb->nt < 2 || pb->nt > kMaxNt) return fail(MFG_ERR_INVALID_ARG, "nt must be in [2, 4096]");
  {
    // the kernels index cells of an n-vector with 32-bit arithmetic
    const long long ncell = (long long)pb->nt * pb->n[0] * (pb->d == 2 ? pb->n[1] : 1);
    if (ncell >= (1LL << 31))
      return fail(MFG_ERR_UNSUPPORTED, "grid too large: N_t times the spatial nodes must be below 2^31");
  }
  if (!(pb->T > 0.0) || !std::isfinite(pb->T)) return fail(MFG_ERR_INVALID_ARG, "T must be > 0");
  if (pb->bc < MFG_BC_PERIODIC || pb->bc > MFG_BC_NEUMANN_X_PERIODIC_Y)
    return fail(MFG_ERR_INVALID_ARG, "unknown boundary condition");
  if (pb->d == 1 && pb->bc > MFG_BC_NEUMANN)
    return fail(MFG_ERR_INVALID_ARG, "a boundary type per axis needs d = 2");
  if (!(pb->nu >= 0.0) || !std::isfinite(pb->nu)) return fail(MFG_ERR_INVALID_ARG, "nu must be >= 0");
  if (!(pb->qprime >= 1.2 && pb->qprime <= 6.0))
    return fail(MFG_ERR_UNSUPPORTED, "q' must lie in [1.2, 6]");
  if (!(pb->gamma > 0.0) || !std::isfinite(pb->gamma))
    return fail(MFG_ERR_INVALID_ARG, "gamma must be > 0");
  if (pb->l != 1 && pb->l != 2) return fail(MFG_ERR_INVALID_ARG, "l must be 1 or 2");
  if (pb->precision < MFG_FP64 || pb->precision > MFG_MIXED_BF16)
    return fail(MFG_ERR_INVALID_ARG, "unknown precision");
  if (pb->coupling < MFG_F_LINEAR || pb->coupling > MFG_F_POTENTIAL)
    return fail(MFG_ERR_INVALID_ARG, "unknown coupling");
  if (!(pb->beta >= 0.0) || !std::isfinite(pb->beta))
    return fail(MFG_ERR_INVALID_ARG, "beta must be >= 0 (0: no terminal cost)");

  P.pb = *pb;
  P.stream = stream;
  HIP_TRY(hipGetDevice(&P.device));
  {
    int ncu = 0;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P.device));
    P.num_cus = ncu > 0 ? ncu : 256;
  }
  P.precision = pb->precision;
  P.l = pb->l;
  P.gamma = pb->gamma;
  Geom& g = P.g;
  auto spacing = [&](int a) { return axis_spacing(pb, a); };
  // internal axis 1 (j) is y when d = 2 and x when d = 1; axis 0 (i) is x
  g.bcm = pb->d == 2 ? (axis_neumann(pb, 1) ? 1 : 0) | (axis_neumann(pb, 0) ? 2 : 0)
                     : (axis_neumann(pb, 0) ? 1 : 0);
  g.nt = pb->nt;
  g.nu = pb->nu;
  g.dt = pb->T / pb->nt;
  g.idt = 1.0 / g.dt;
  g.idt2 = g.idt * g.idt;
  if (pb->d == 2) {
    g.n0 = pb->n[0];
    g.n1 = pb->n[1];
    g.has0 = 1;
    const double h0 = spacing(0), h1 = spacing(1);
    g.ih0 = 1.0 / h0;
    g.ih1 = 1.0 / h1;
    g.ih0sq = g.ih0 * g.ih0;
    g.ih1sq = g.ih1 * g.ih1;
    g.ncomp = 4;
    g.cb1 = 2;
  } else {
    g.n0 = 1;
    g.n1 = pb->n[0];
    g.has0 = 0;
    const double h1 = spacing(0);
    g.ih0 = 0.0;
    g.ih0sq = 0.0;
    g.ih1 = 1.0 / h1;
    g.ih1sq = g.ih1 * g.ih1;
    g.ncomp = 2;
    g.cb1 = 0;
  }
  g.M = g.n0 * g.n1;
  g.n = (long long)g.nt * g.M;
  // coupling f = c2 m^2 + c1 m + V; the terminal cost adds 1/(beta dt) to the
  // last slice's linear coefficient
  g.qp = pb->qprime;
  g.q = pb->qprime == 2.0 ? 2.0 : pb->qprime / (pb->qprime - 1.0);
  g.c2 = pb->coupling == MFG_F_QUADRATIC ? 0.5 : 0.0;
  g.c1 = pb->coupling == MFG_F_LINEAR ? 1.0 : 0.0;
  g.c1T = pb->beta > 0.0 ? g.c1 + 1.0 / (pb->beta * g.dt) : g.c1;
  P.beta = pb->beta;
  return MFG_OK;
}

static int build_plan(Plan& P, const mfg_problem_t* pb, const double* V, const double* m0,
                      hipStream_t stream) {
  int rc = setup_problem(P, pb, stream);
  if (rc) return rc;
  const Geom& g = P.g;
  const bool neu = pb->bc == MFG_BC_NEUMANN;
  auto spacing = [&](int a) {
    const double L = pb->hi[a] - pb->lo[a];
    return neu ? L / (pb->n[a] + 1) : L / pb->n[a];
  };
  // V and m0 may come from work queued on the caller's stream
  if (stream) HIP_TRY(hipStreamSynchronize(stream));
  else HIP_TRY(hipDeviceSynchronize());
  rc = check_fields(P, V, m0, true);
  if (rc) return rc;

  // problem data; the terminal target starts at zero
  if ((rc = dalloc(P, &P.V, g.M)) || (rc = dalloc(P, &P.m0, g.M)) ||
      (rc = dalloc(P, &P.mbar, g.M)) || (rc = dalloc(P, &P.VT, g.M)))
    return rc;
  HIP_TRY(hipMemcpy(P.V, V, g.M * sizeof(double), hipMemcpyDeviceToDevice));
  HIP_TRY(hipMemcpy(P.m0, m0, g.M * sizeof(double), hipMemcpyDeviceToDevice));
  HIP_TRY(hipMemset(P.mbar, 0, g.M * sizeof(double)));
  launch_terminal_potential(P, nullptr);
  HIP_TRY(hipGetLastError());

  // time transform (eq. eigs and the DCT-VIII / DST-I of Section 4.1)
  const int nt = g.nt;
  const double pi = 3.14159265358979323846264338327950288;
  std::vector<double> Vm((size_t)nt * nt), Vt((size_t)nt * nt), lt(nt);
  for (int k = 1; k <= nt; ++k) {
    lt[k - 1] = 2.0 - 2.0 * std::cos(pi * (k - 1 + 0.5 * P.l) / (nt + 0.5 * P.l));
    for (int j = 1; j <= nt; ++j) {
      double v;
      if (P.l == 1)
        v = std::sqrt(4.0 / (2 * nt + 1)) *
            std::cos(pi * (double)((2 * k - 1) * (2 * j - 1)) / (2.0 * (2 * nt + 1)));
      else
        v = std::sqrt(2.0 / (nt + 1)) * std::sin(pi * (double)(k * j) / (nt + 1.0));
      Vm[(size_t)(k - 1) * nt + (j - 1)] = v;
    }
  }
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < nt; ++k) Vt[(size_t)t * nt + k] = Vm[(size_t)k * nt + t];
  std::vector<float> Vt32(Vt.size());
  std::vector<_Float16> Vt16(Vt.size());
  std::vector<unsigned short> Vtbf(Vt.size());
  for (size_t i = 0; i < Vt.size(); ++i) {
    Vt32[i] = (float)Vt[i];
    Vt16[i] = (_Float16)Vt[i];
    Vtbf[i] = to_bf16((float)Vt[i]);
  }
  if (nt <= 128) {
    const int ntp = (nt + 15) / 16 * 16;
    P.ntp = ntp;
    std::vector<float> p32((size_t)ntp * ntp, 0.0f);
    std::vector<_Float16> p16((size_t)ntp * ntp, (_Float16)0.0f);
    std::vector<_Float16> p16s(2 * (size_t)ntp * ntp, (_Float16)0.0f);
    std::vector<unsigned short> pbf((size_t)ntp * ntp, 0);
    std::vector<double> p64((size_t)ntp * ntp, 0.0);
    for (int k = 0; k < nt; ++k)
      for (int t = 0; t < nt; ++t) {
        const double v = Vm[(size_t)k * nt + t];
        p64[(size_t)t * ntp + k] = v;
        p32[(size_t)k * ntp + t] = (float)v;
        p16[(size_t)k * ntp + t] = (_Float16)v;
        const _Float16 hi = (_Float16)(v * kVSplitScale);
        p16s[(size_t)k * ntp + t] = hi;
        p16s[((size_t)ntp + k) * ntp + t] = (_Float16)(v * kVSplitScale - (double)hi);
        pbf[(size_t)k * ntp + t] = to_bf16((float)v);
      }
    if ((rc = upload(P, &P.Vp64, p64)) || (rc = upload(P, &P.Vp32, p32)) ||
        (rc = upload(P, &P.Vp16, p16)) || (rc = upload(P, &P.Vp16s, p16s)) ||
        (rc = upload(P, &P.Vpbf, pbf)))
      return rc;
  }
  if (nt > 128 && P.precision != MFG_FP64) {
    // streaming low-precision V (row k contiguous in t), only the table of the
    // plan's precision
    const int ns = (nt + 127) / 128 * 128;
    P.ntps = ns;
    if (P.precision == MFG_MIXED_BF16) {
      std::vector<unsigned short> tb((size_t)ns * ns, 0);
      for (int k = 0; k < nt; ++k)
        for (int t = 0; t < nt; ++t) tb[(size_t)k * ns + t] = to_bf16((float)Vm[(size_t)k * nt + t]);
      unsigned short* d = nullptr;
      if ((rc = upload(P, &d, tb))) return rc;
      P.Vs_lp = d;
    } else {
      const bool split = P.precision == MFG_MIXED_FP32;
      std::vector<_Float16> th((size_t)(split ? 2 : 1) * ns * ns, (_Float16)0.0f);
      for (int k = 0; k < nt; ++k)
        for (int t = 0; t < nt; ++t) {
          const double v = Vm[(size_t)k * nt + t];
          if (split) {
            const _Float16 hi = (_Float16)(v * kVSplitScale);
            th[(size_t)k * ns + t] = hi;
            th[((size_t)ns + k) * ns + t] = (_Float16)(v * kVSplitScale - (double)hi);
          } else {
            th[(size_t)k * ns + t] = (_Float16)v;
          }
        }
      _Float16* d = nullptr;
      if ((rc = upload(P, &d, th))) return rc;
      P.Vs_lp = d;
    }
  }
  if ((rc = upload(P, &P.Vt64, Vt)) || (rc = upload(P, &P.Vt32, Vt32)) ||
      (rc = upload(P, &P.Vt16, Vt16)) || (rc = upload(P, &P.Vtbf, Vtbf)) ||
      (rc = upload(P, &P.lam_t, lt)))
    return rc;

  // spatial axes
  if (g.has0) {
    if ((rc = build_axis(P, P.ax0, g.n0, axis_neumann(&P.pb, 0), axis_spacing(&P.pb, 0))))
      return rc;
    if ((rc = build_axis(P, P.ax1, g.n1, axis_neumann(&P.pb, 1), axis_spacing(&P.pb, 1))))
      return rc;
  } else {
    if ((rc = build_axis(P, P.ax1, g.n1, axis_neumann(&P.pb, 0), axis_spacing(&P.pb, 0))))
      return rc;
  }

  // workspace
  const size_t n = (size_t)g.n;
  if ((rc = dalloc(P, &P.r, n)) || (rc = dalloc(P, &P.z, n)) || (rc = dalloc(P, &P.p, n)) ||
      (rc = dalloc(P, &P.p2, n)) ||
      (rc = dalloc(P, &P.q, n)) || (rc = dalloc(P, &P.tmp, n)) || (rc = dalloc(P, &P.b, n)) ||
      (rc = dalloc(P, &P.u, n)) || (rc = dalloc(P, &P.zn, (size_t)n * (1 + g.ncomp))))
    return rc;
  P.red.max_blocks = 32768;
  {
    // the time-transform GEMM reduces one partial per block
    const long long colblk = (g.M + 63) / 64;
    const long long kchunks = (((g.nt + 15) / 16) + 7) / 8;
    if (colblk * kchunks > P.red.max_blocks)
      return fail(MFG_ERR_UNSUPPORTED, "grid too large for the time-transform reduction");
  }
  if ((rc = dalloc(P, &P.red.partials, (size_t)T_COUNT * kSlotsPerSite * P.red.max_blocks)) ||
      (rc = dalloc(P, &P.red.scal, S_COUNT)))
    return rc;
  HIP_TRY(hipMemset(P.red.scal, 0, S_COUNT * sizeof(double)));
  void* hs = nullptr;
  HIP_TRY(hipHostMalloc(&hs, S_COUNT * sizeof(double), hipHostMallocDefault));
  P.host_allocs.push_back(hs);
  P.host_scal = static_cast<double*>(hs);
  // launch shapes: defaults, then a tuned choice cached for this key, then
  // explicit MFG_TUNE overrides
  {
    Tune t;
    if (tune_lookup(P, &t)) {
      keep_untuned(P.tune, t);
      P.tune = t;
    }
  }
  read_tune_env(P.tune);
  HIP_TRY(hipDeviceSynchronize());
  return MFG_OK;
}

static hipEvent_t pool_event(Plan& P) {
  if (!P.prof.pool.empty()) {
    hipEvent_t e = P.prof.pool.back();
    P.prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Resolve pending event pairs into the per-kernel totals (synchronises).
static void prof_flush(const Plan& Pc) {
  Plan& P = const_cast<Plan&>(Pc);
  if (P.prof.pending.empty()) return;
  (void)hipStreamSynchronize(P.stream);
  for (auto& r : P.prof.pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& a = P.prof.acc[r.name];
      a.first += 1;
      a.second += ms;
    }
    P.prof.pool.push_back(r.a);
    P.prof.pool.push_back(r.b);
  }
  P.prof.pending.clear();
}

int prof_begin(const Plan& Pc, const char* name, hipStream_t s) {
  Plan& P = const_cast<Plan&>(Pc);
  if (!P.prof.on) return -1;
  if (P.prof.pending.size() >= 4096) prof_flush(P);
  Profiler::Rec r{name, pool_event(P), pool_event(P)};
  if (!r.a || !r.b) return -1;
  (void)hipEventRecord(r.a, s);
  P.prof.pending.push_back(r);
  return (int)P.prof.pending.size() - 1;
}

void prof_end(const Plan& Pc, int id, hipStream_t s) {
  Plan& P = const_cast<Plan&>(Pc);
  if (id < 0 || id >= (int)P.prof.pending.size()) return;
  (void)hipEventRecord(P.prof.pending[id].b, s);
}

int read_scalars(Plan& P) {
  HIP_TRY(hipMemcpyAsync(P.host_scal, P.red.scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                         P.stream));
  HIP_TRY(hipStreamSynchronize(P.stream));
  return MFG_OK;
}

// PCG from x = 0, or from the x it is given when warm (the residual is then
// r = b - A x, and the first update adds to x) (flexible form where
// pcg_flexible says so). Iterations are
// launched in chunks without a host round trip: every kernel of an iteration
// tests the device `done` flag (set by the r.r stopping test on convergence,
// breakdown or a non-finite value) and returns at once when it is set, so
// launching past convergence only costs launch latency. The first chunk is as
// long as the previous solve on this plan; later ones are single iterations.
// r_ready: the start (r = b, b.b, status reset) was already done by the
// kernel that formed b (b is then not needed).
int run_pcg(Plan& P, const double* b, double* x, double rtol, int maxit, int* iters_out,
            double* relres_rec, double* relres_true, bool r_ready, bool warm) {
  hipStream_t s = P.stream;
  P.pcg_done = P.red.scal + S_DONE;
  if (!r_ready) launch_pcg_init(P, b, P.r, rtol, s);
  if (warm) {
    // r = b - A x0 (b.b and the status come from the start above)
    launch_AAt(P, x, P.q, false, s);
    launch_axpby(P.g.n, -1.0, P.q, 1.0, P.r, s);
  }
  launch_precond(P, P.r, P.z, true, nullptr, s);
  double* pold = P.p2;
  double* pnew = P.p;
  int k = 0, rc = MFG_OK;
  int chunk = std::max(1, P.last_pcg_its);
  while (true) {
    const int todo = std::min(chunk, maxit - k);
    for (int j = 0; j < todo; ++j) {
      ++k;
      launch_pdir_AAt(P, P.z, pold, pnew, P.q, k == 1, s);
      launch_update_precond(P, x, P.r, pnew, P.q, P.z, k == 1 && !warm, s);
      std::swap(pold, pnew);
    }
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) {
      P.pcg_done = nullptr;
      return fail(MFG_ERR_HIP, std::string("PCG launch failed: ") + hipGetErrorString(le));
    }
    if ((rc = read_scalars(P))) {
      P.pcg_done = nullptr;
      return rc;
    }
    if (P.host_scal[S_DONE] != 0.0 || k >= maxit) break;
    chunk = 1;
  }
  P.pcg_done = nullptr;
  const double bad = P.host_scal[S_BAD];
  if (bad == 2.0) return fail(MFG_ERR_NONFINITE, "non-finite value in PCG");
  if (bad == 1.0) return fail(MFG_ERR_BREAKDOWN, "PCG breakdown (p.Ap or r.z not positive)");
  const bool conv = P.host_scal[S_DONE] != 0.0;
  const int its = (int)P.host_scal[S_ITS];
  const double bb = P.host_scal[S_BB];
  // b = 0: done before the first update, which would have written x
  if (conv && its == 0) launch_fill(x, P.g.n, 0.0, s);
  P.last_pcg_its = its;
  if (iters_out) *iters_out = its;
  if (relres_rec) *relres_rec = (bb > 0.0) ? std::sqrt(P.host_scal[S_RR] / bb) : 0.0;
  if (relres_true) {
    launch_AAt(P, x, P.p, false, s);
    launch_residual(P, b, P.p, s);
    if ((rc = read_scalars(P))) return rc;
    const double b2 = P.host_scal[S_AUX1];
    *relres_true = (b2 > 0.0) ? std::sqrt(P.host_scal[S_AUX0] / b2) : 0.0;
  }
  if (!conv) return fail(MFG_ERR_NOT_CONVERGED, "PCG reached maxit without converging");
  return MFG_OK;
}

// One Chambolle-Pock iteration (eq. pasosChamPock, Section 5 schedule) on the
// state; vout (optional) receives the prox input v = y - tau xi'. Inside a
// multi-step call the right-hand side only needs z = xi + sigma ybar: z_in, the
// previous step left it in P.zn (st->xi, st->ybar are stale); z_out, store it
// there for the next step instead of xi' and ybar'. The first step of a call
// reads the state and the last one writes it back, so the caller sees the
// same state either way, and 10 n-vectors of traffic per step are saved.
static int cp_step(Plan& P, mfg_state_t* st, double rtol, int maxit, int* its, double* rel,
                   double* vout, bool z_in = false, bool z_out = false) {
  hipStream_t s = P.stream;
  // the right-hand side goes straight into the PCG residual and starts the
  // solve (from the previous projection's solution with a warm start)
  launch_rhs(P, st->xi, st->ybar, st->sigma, P.m0, P.r, s, z_in ? P.zn : nullptr, rtol);
  int rc = run_pcg(P, nullptr, P.u, rtol, maxit, its, rel, nullptr, true,
                   P.warm_start && P.u_valid);
  if (rc && rc != MFG_ERR_NOT_CONVERGED) {
    P.u_valid = false;
    return rc;
  }
  P.u_valid = true;
  const double theta = 1.0 / std::sqrt(1.0 + 2.0 * P.gamma * st->tau);
  launch_backproj_prox(P, P.u, st->xi, st->y, st->ybar, st->tau, theta, s, vout,
                       z_out ? P.zn : nullptr, st->sigma);
  HIP_TRY(hipGetLastError());
  st->tau *= theta;
  st->sigma /= theta;
  st->theta = theta;
  st->iter += 1;
  return rc;
}

// Reverse sweep with recomputation from checkpoints (see adjoint.hip).
static int run_cp_adjoint(Plan& P, const mfg_state_t* ckpts, int every, int n_iter,
                          const double* gy_final, double rtol, int maxit, double* g_m0,
                          double* g_V) {
  hipStream_t s = P.stream;
  const long long n = P.g.n;
  const long long np = n * (1 + P.g.ncomp);
  const int M = P.g.M;
  std::vector<void*> mine;
  auto alloc = [&](double** ptr, long long count) -> int {
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)count * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MFG_ERR_OOM, "adjoint workspace allocation failed");
    }
    mine.push_back(p);
    *ptr = static_cast<double*>(p);
    return MFG_OK;
  };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    for (void* p : mine) (void)hipFree(p);
  };
  double *tape, *sx, *sy, *sb, *gxi, *gy, *gyb, *gVc, *gb;
  int rc;
  if ((rc = alloc(&tape, (long long)every * np)) || (rc = alloc(&sx, np)) ||
      (rc = alloc(&sy, np)) || (rc = alloc(&sb, np)) || (rc = alloc(&gxi, np)) ||
      (rc = alloc(&gy, np)) || (rc = alloc(&gyb, np)) || (rc = alloc(&gVc, n)) ||
      (rc = alloc(&gb, n))) {
    cleanup();
    return rc;
  }
  launch_fill(gxi, np, 0.0, s);
  launch_fill(gyb, np, 0.0, s);
  launch_fill(g_m0, M, 0.0, s);
  launch_fill(g_V, M, 0.0, s);
  HIP_TRY(hipMemcpyAsync(gy, gy_final, np * sizeof(double), hipMemcpyDeviceToDevice, s));
  const int nseg = (n_iter + every - 1) / every;
  std::vector<double> sig(every), ta(every), th(every);
  int final_rc = MFG_OK;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int cnt = std::min(every, n_iter - seg * every);
    // recompute the segment's forward steps from its checkpoint, taping v
    mfg_state_t st = ckpts[seg];
    HIP_TRY(hipMemcpyAsync(sx, st.xi, np * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(sy, st.y, np * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(sb, st.ybar, np * sizeof(double), hipMemcpyDeviceToDevice, s));
    st.xi = sx;
    st.y = sy;
    st.ybar = sb;
    for (int j = 0; j < cnt; ++j) {
      sig[j] = st.sigma;
      ta[j] = st.tau;
      int its;
      double rel;
      rc = cp_step(P, &st, rtol, maxit, &its, &rel, tape + (size_t)j * np);
      if (rc == MFG_ERR_NOT_CONVERGED) final_rc = rc;
      else if (rc) { cleanup(); return rc; }
      th[j] = st.theta;
    }
    // reverse steps of the segment
    for (int j = cnt - 1; j >= 0; --j) {
      launch_adj_prox(P, gy, gyb, tape + (size_t)j * np, ta[j], th[j], gxi, gVc, s);
      launch_sum_slices(P, gVc, nullptr, g_V, s);
      launch_apply_C(P, gxi, P.b, s);
      int its;
      double rel;
      rc = run_pcg(P, P.b, gb, rtol, maxit, &its, &rel, nullptr);
      if (rc == MFG_ERR_NOT_CONVERGED) final_rc = rc;
      else if (rc) { cleanup(); return rc; }
      launch_apply_CT(P, gb, gxi, s);
      launch_axpby(np, sig[j], gxi, 0.0, gyb, s);
      launch_axpby(M, -sig[j] * P.g.idt, gb, 1.0, g_m0, s);
    }
  }
  // initial point: y_0 = ybar_0 = (m0 at every slice, w = 0)
  launch_sum_slices(P, gy, gyb, g_m0, s);
  HIP_TRY(hipGetLastError());
  cleanup();
  if (final_rc) return fail(final_rc, "some PCG solve reached maxit");
  return MFG_OK;
}

}  // namespace mfg

using mfg::fail;

extern "C" {

int mfg_plan(const mfg_problem_t* pb, const double* V, const double* m0, hipStream_t stream,
             mfg_plan_t* out) {
  if (!out) return fail(MFG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  mfg_plan_s* h = new (std::nothrow) mfg_plan_s();
  if (!h) return fail(MFG_ERR_OOM, "host allocation failed");
  int rc = mfg::build_plan(h->P, pb, V, m0, stream);
  if (rc) {
    std::string msg = mfg::g_last_error;
    mfg::release(h->P);
    delete h;
    mfg::g_last_error = msg;
    return rc;
  }
  *out = h;
  return MFG_OK;
}

int mfg_destroy(mfg_plan_t plan) {
  if (!plan) return MFG_OK;
  mfg::release(plan->P);
  delete plan;
  return MFG_OK;
}

int mfg_set_stream(mfg_plan_t plan, hipStream_t stream) {
  if (!plan) return fail(MFG_ERR_INVALID_ARG, "plan is NULL");
  plan->P.stream = stream;
  return MFG_OK;
}

int mfg_set_data(mfg_plan_t plan, const double* V, const double* m0) {
  if (!plan) return fail(MFG_ERR_INVALID_ARG, "plan is NULL");
  mfg::Plan& P = plan->P;
  HIP_TRY(hipStreamSynchronize(P.stream));
  int rc = mfg::check_fields(P, V, m0, false);
  if (rc) return rc;
  if (V) {
    HIP_TRY(hipMemcpyAsync(P.V, V, P.g.M * sizeof(double), hipMemcpyDeviceToDevice, P.stream));
    mfg::launch_terminal_potential(P, P.stream);
    HIP_TRY(hipGetLastError());
  }
  if (m0)
    HIP_TRY(hipMemcpyAsync(P.m0, m0, P.g.M * sizeof(double), hipMemcpyDeviceToDevice, P.stream));
  return MFG_OK;
}

int mfg_set_target(mfg_plan_t plan, const double* mbar) {
  if (!plan || !mbar) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  mfg::Plan& P = plan->P;
  if (!(P.beta > 0.0)) return fail(MFG_ERR_INVALID_ARG, "the problem has no terminal cost (beta = 0)");
  HIP_TRY(hipStreamSynchronize(P.stream));
  {
    std::vector<double> h(P.g.M);
    HIP_TRY(hipMemcpy(h.data(), mbar, P.g.M * sizeof(double), hipMemcpyDeviceToHost));
    for (double x : h)
      if (!std::isfinite(x)) return fail(MFG_ERR_NONFINITE, "mbar has a non-finite entry");
  }
  HIP_TRY(hipMemcpyAsync(P.mbar, mbar, P.g.M * sizeof(double), hipMemcpyDeviceToDevice, P.stream));
  mfg::launch_terminal_potential(P, P.stream);
  HIP_TRY(hipGetLastError());
  return MFG_OK;
}

int mfg_value_function(mfg_plan_t plan, const mfg_state_t* st, double pcg_rtol, int pcg_maxit,
                       double* u) {
  if (!plan || !st || !st->xi || !st->y || !u) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (!(pcg_rtol >= 0.0) || pcg_maxit < 1)
    return fail(MFG_ERR_INVALID_ARG, "need rtol >= 0, maxit >= 1");
  mfg::Plan& P = plan->P;
  // the multiplier: A lam = Cr xi (least-squares solution of Cr^T lam = xi)
  mfg::launch_apply_C(P, st->xi, P.b, P.stream);
  int its = 0;
  double rel = 0.0;
  P.u_valid = false;  // P.u now holds the multiplier, not a projection's solution
  const int rc = mfg::run_pcg(P, P.b, P.u, pcg_rtol, pcg_maxit, &its, &rel, nullptr);
  if (rc && rc != MFG_ERR_NOT_CONVERGED) return rc;
  mfg::launch_value(P, P.u, st->y, u, P.stream);
  HIP_TRY(hipGetLastError());
  if (rc) return fail(rc, "the multiplier's PCG solve reached maxit");
  return MFG_OK;
}

int mfg_hjb_residual(mfg_plan_t plan, const double* y, const double* u, double* R) {
  if (!plan || !y || !u || !R) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  mfg::launch_hjb_residual(plan->P, y, u, R, plan->P.stream);
  HIP_TRY(hipGetLastError());
  return MFG_OK;
}

int mfg_set_warm_start(mfg_plan_t plan, int enable) {
  if (!plan) return fail(MFG_ERR_INVALID_ARG, "plan is NULL");
  plan->P.warm_start = enable != 0;
  return MFG_OK;
}

int mfg_prox(mfg_plan_t plan, const double* v, double tau, double* y) {
  if (!plan || !v || !y) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(MFG_ERR_INVALID_ARG, "tau must be > 0");
  mfg::launch_prox(plan->P, v, tau, y, plan->P.stream);
  HIP_TRY(hipGetLastError());
  return MFG_OK;
}

int mfg_apply_AAt(mfg_plan_t plan, const double* u, double* q) {
  if (!plan || !u || !q) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (u == q) return fail(MFG_ERR_INVALID_ARG, "u and q must not alias");
  mfg::launch_AAt(plan->P, u, q, false, plan->P.stream);
  HIP_TRY(hipGetLastError());
  return MFG_OK;
}

int mfg_apply_C(mfg_plan_t plan, const double* y, double* b) {
  if (!plan || !y || !b) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  mfg::launch_apply_C(plan->P, y, b, plan->P.stream);
  HIP_TRY(hipGetLastError());
  return MFG_OK;
}

int mfg_apply_CT(mfg_plan_t plan, const double* u, double* y) {
  if (!plan || !u || !y) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  mfg::launch_apply_CT(plan->P, u, y, plan->P.stream);
  HIP_TRY(hipGetLastError());
  return MFG_OK;
}

int mfg_precond(mfg_plan_t plan, const double* r, double* z) {
  if (!plan || !r || !z) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (r == z) return fail(MFG_ERR_INVALID_ARG, "r and z must not alias");
  mfg::launch_precond(plan->P, r, z, false, nullptr, plan->P.stream);
  HIP_TRY(hipGetLastError());
  return MFG_OK;
}

int mfg_pcg(mfg_plan_t plan, const double* b, double* u, double rtol, int maxit, int* iters,
            double* relres) {
  if (!plan || !b || !u) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (b == u) return fail(MFG_ERR_INVALID_ARG, "b and u must not alias");
  if (!(rtol >= 0.0) || maxit < 1) return fail(MFG_ERR_INVALID_ARG, "need rtol >= 0, maxit >= 1");
  return mfg::run_pcg(plan->P, b, u, rtol, maxit, iters, nullptr, relres);
}

int mfg_cp_init(mfg_plan_t plan, mfg_state_t* st) {
  if (!plan || !st || !st->xi || !st->y || !st->ybar)
    return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  mfg::launch_cp_init(plan->P, st->xi, st->y, st->ybar, plan->P.stream);
  HIP_TRY(hipGetLastError());
  plan->P.u_valid = false;  // the first projection starts from zero
  st->sigma = 1.0;
  st->tau = 1.0;
  st->theta = 1.0;
  st->iter = 0;
  return MFG_OK;
}

int mfg_cp_solve(mfg_plan_t plan, mfg_state_t* st, int n_iter, double pcg_rtol, int pcg_maxit,
                 mfg_stats_t* stats) {
  if (!plan || !st || !st->xi || !st->y || !st->ybar)
    return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (n_iter < 0 || pcg_maxit < 1 || !(pcg_rtol >= 0.0))
    return fail(MFG_ERR_INVALID_ARG, "bad iteration arguments");
  if (!(st->sigma > 0.0) || !(st->tau > 0.0)) return fail(MFG_ERR_INVALID_ARG, "bad step sizes");
  mfg::Plan& P = plan->P;
  // ||m' - m||^2 of each step is copied to pinned host memory in stream order
  // (no host wait between steps) and read once at the end
  // (and the mass drift, when asked for)
  double* dm_host = nullptr;
  const bool want_dm = stats && (stats->dm || stats->mass_drift) && n_iter > 0;
  if (want_dm &&
      hipHostMalloc(reinterpret_cast<void**>(&dm_host), 2 * (size_t)n_iter * sizeof(double)) !=
          hipSuccess) {
    (void)hipGetLastError();
    return fail(MFG_ERR_OOM, "pinned statistics buffer");
  }
  int final_rc = MFG_OK, rc = MFG_OK;
  for (int it = 0; it < n_iter; ++it) {
    int its = 0;
    double rel = 0.0;
    rc = mfg::cp_step(P, st, pcg_rtol, pcg_maxit, &its, &rel, nullptr, it > 0, it + 1 < n_iter);
    if (rc == MFG_ERR_NOT_CONVERGED) final_rc = rc;
    else if (rc) break;
    rc = MFG_OK;
    if (stats) {
      if (stats->pcg_iters) stats->pcg_iters[it] = its;
      if (stats->pcg_relres) stats->pcg_relres[it] = rel;
      if (dm_host && hipMemcpyAsync(dm_host + it, P.red.scal + mfg::S_DM, sizeof(double),
                                    hipMemcpyDeviceToHost, P.stream) != hipSuccess) {
        rc = fail(MFG_ERR_HIP, "statistics copy failed");
        break;
      }
      if (dm_host && stats->mass_drift) {
        mfg::launch_mass_drift(P, st->y, P.stream);
        if (hipMemcpyAsync(dm_host + n_iter + it, P.red.scal + mfg::S_MASS, sizeof(double),
                           hipMemcpyDeviceToHost, P.stream) != hipSuccess) {
          rc = fail(MFG_ERR_HIP, "statistics copy failed");
          break;
        }
      }
    }
  }
  if (dm_host) {
    if (hipStreamSynchronize(P.stream) != hipSuccess && !rc)
      rc = fail(MFG_ERR_HIP, "stream synchronisation failed");
    if (!rc)
      for (int it = 0; it < n_iter; ++it) {
        if (stats->dm) stats->dm[it] = std::sqrt(dm_host[it]);
        if (stats->mass_drift) stats->mass_drift[it] = dm_host[n_iter + it];
      }
    (void)hipHostFree(dm_host);
  }
  if (rc) {
    // a step after the first may have left xi and ybar only in the z hand-off
    // buffer: the state is marked unusable
    st->iter = -1;
    return rc;
  }
  if (final_rc) return fail(final_rc, "some PCG solve reached maxit");
  return MFG_OK;
}

// Section 5: the loop ends after the first iteration whose change in m is
// below cp_tol; iteration l+1 solves to min(1e-4, max(1e-6, 1e-4 r_l)) with
// r_l the change of the iteration before it (1e-4 for the first of the call).
// Every step writes xi and ybar (no z hand-off: whether another step follows
// is known only after its change has been read back).
int mfg_cp_solve_tol(mfg_plan_t plan, mfg_state_t* st, int max_iter, double cp_tol,
                     int pcg_maxit, int* n_done, mfg_stats_t* stats) {
  if (!plan || !st || !st->xi || !st->y || !st->ybar)
    return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (max_iter < 0 || pcg_maxit < 1 || !(cp_tol >= 0.0) || !std::isfinite(cp_tol))
    return fail(MFG_ERR_INVALID_ARG, "bad iteration arguments");
  if (!(st->sigma > 0.0) || !(st->tau > 0.0)) return fail(MFG_ERR_INVALID_ARG, "bad step sizes");
  mfg::Plan& P = plan->P;
  if (n_done) *n_done = 0;
  int final_rc = MFG_OK, rc = MFG_OK;
  double r_prev = -1.0;
  for (int it = 0; it < max_iter; ++it) {
    const double tol = (r_prev < 0.0) ? 1e-4 : std::min(1e-4, std::max(1e-6, 1e-4 * r_prev));
    int its = 0;
    double rel = 0.0;
    rc = mfg::cp_step(P, st, tol, pcg_maxit, &its, &rel, nullptr);
    if (rc == MFG_ERR_NOT_CONVERGED) final_rc = rc;
    else if (rc) break;
    if ((rc = mfg::read_scalars(P))) break;
    const double r = std::sqrt(P.host_scal[mfg::S_DM]);
    if (n_done) *n_done = it + 1;
    if (stats) {
      if (stats->pcg_iters) stats->pcg_iters[it] = its;
      if (stats->pcg_relres) stats->pcg_relres[it] = rel;
      if (stats->dm) stats->dm[it] = r;
      if (stats->mass_drift) {
        mfg::launch_mass_drift(P, st->y, P.stream);
        if ((rc = mfg::read_scalars(P))) break;
        stats->mass_drift[it] = P.host_scal[mfg::S_MASS];
      }
    }
    r_prev = r;
    if (r <= cp_tol) break;
  }
  if (rc) return rc;
  if (final_rc) return fail(final_rc, "some PCG solve reached maxit");
  return MFG_OK;
}

int mfg_cp_adjoint(mfg_plan_t plan, const mfg_state_t* ckpts, int n_ckpt, int every, int n_iter,
                   const double* gy_final, double pcg_rtol, int pcg_maxit, double* g_m0,
                   double* g_V) {
  if (!plan || !ckpts || !gy_final || !g_m0 || !g_V)
    return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (n_iter < 0 || every < 1 || n_ckpt < 1 || (long long)n_ckpt * every < n_iter ||
      pcg_maxit < 1 || !(pcg_rtol >= 0.0))
    return fail(MFG_ERR_INVALID_ARG, "bad checkpoint or iteration arguments");
  for (int k = 0; k < n_ckpt; ++k)
    if (!ckpts[k].xi || !ckpts[k].y || !ckpts[k].ybar)
      return fail(MFG_ERR_INVALID_ARG, "checkpoint with NULL vectors");
  if (plan->P.warm_start)
    return fail(MFG_ERR_INVALID_ARG,
                "the reverse sweep recomputes steps from checkpoints with cold PCG starts: "
                "disable the warm start for the forward run and the gradient");
  if (plan->P.pb.qprime != 2.0)
    return fail(MFG_ERR_UNSUPPORTED, "the reverse sweep differentiates the q' = 2 prox only");
  return mfg::run_cp_adjoint(plan->P, ckpts, every, n_iter, gy_final, pcg_rtol, pcg_maxit, g_m0,
                             g_V);
}

int mfg_profile(mfg_plan_t plan, int enable) {
  if (!plan) return fail(MFG_ERR_INVALID_ARG, "plan is NULL");
  mfg::Plan& P = plan->P;
  mfg::prof_flush(P);
  if (enable) P.prof.acc.clear();
  P.prof.on = enable != 0;
  return MFG_OK;
}

int mfg_profile_report(mfg_plan_t plan, char* buf, int len) {
  if (!plan || !buf || len < 3) return fail(MFG_ERR_INVALID_ARG, "bad arguments");
  mfg::Plan& P = plan->P;
  mfg::prof_flush(P);
  std::string out = "{";
  bool first = true;
  char tmp[256];
  for (auto& kv : P.prof.acc) {
    std::snprintf(tmp, sizeof(tmp), "%s\"%s\": {\"calls\": %ld, \"total_ms\": %.6f}",
                  first ? "" : ", ", kv.first.c_str(), kv.second.first, kv.second.second);
    out += tmp;
    first = false;
  }
  out += "}";
  if ((int)out.size() + 1 > len) return fail(MFG_ERR_INVALID_ARG, "buffer too small");
  std::memcpy(buf, out.c_str(), out.size() + 1);
  return MFG_OK;
}

int mfg_autotune(mfg_plan_t plan, int effort) {
  if (!plan || (effort != 1 && effort != 2)) return fail(MFG_ERR_INVALID_ARG, "bad arguments");
  return mfg::autotune(plan->P, effort, true);
}

const char* mfg_last_error(void) { return mfg::g_last_error.c_str(); }

const char* mfg_version(void) { return "mfg 0.1 (gfx950)"; }

}  // extern "C"
