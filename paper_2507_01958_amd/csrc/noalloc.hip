// mfg_pcg_noalloc: the PCG solve of mfg_pcg (Sections 3-4) for callers that
// cannot allocate device memory. There is no plan: the problem statement is
// read on every call, and the preconditioner's tables (eqs. eigs, lambda1,
// lambda2 and the transforms of Algorithms 1 and 2) and the PCG workspace are
// carved from a file-scope device array that each GPU holds for the life of
// the process. The kernels are those of mfg_pcg.
#include <mutex>

#include "device_util.h"
#include "plan.h"

namespace mfg {

// The scratch array: 64 MiB per GPU. A call needs 6 n-vectors of float64
// workspace, 8 MiB of reduction partials and under 1 MiB of tables, so
// problems up to n = N_t N_x N_y = 2^20 cells fit.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};
int g_last_its[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up once per device,
// with that device current). In host code the array's name is only a host-side
// stand-in, so every use below goes through this pointer.
int scratch_of(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MFG_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MFG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MFG_OK;
}

// Bump allocation of 256-byte aligned pieces of the scratch array.
struct Carver {
  unsigned char* base;
  size_t used = 0;
  bool ok = true;
  template <typename T>
  T* take(size_t count) {
    const size_t start = (used + 255) & ~size_t(255);
    const size_t bytes = count * sizeof(T);
    if (start + bytes > kScratchBytes) {
      ok = false;
      return nullptr;
    }
    used = start + bytes;
    return reinterpret_cast<T*>(base + start);
  }
};

__device__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}

struct TimeTables {
  int nt, l, ntp;
  double* Vt64;
  double* lam_t;
  double* Vp64;
  float* Vp32;
  _Float16* Vp16;
  _Float16* Vp16s;
  unsigned short* Vpbf;
};

// The same tables as a plan builds: V of Section 4.1 (DCT-VIII for l = 1,
// DST-I for l = 2, orthonormal and symmetric), its eigenvalues (eq. eigs) and
// the zero-padded low-precision copies, one entry (k, t) per thread.
__global__ void k_time_tables(TimeTables a) {
  const int nt = a.nt, ntp = a.ntp;
  const double pi = 3.14159265358979323846264338327950288;
  const long long total = (long long)ntp * ntp;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / ntp), t = (int)(e % ntp);
    double v = 0.0;
    if (k < nt && t < nt) {
      if (a.l == 1)
        v = sqrt(4.0 / (2 * nt + 1)) *
            cos(pi * (double)((2 * k + 1) * (2 * t + 1)) / (2.0 * (2 * nt + 1)));
      else
        v = sqrt(2.0 / (nt + 1)) * sin(pi * (double)((k + 1) * (t + 1)) / (nt + 1.0));
      a.Vt64[(size_t)t * nt + k] = v;
      if (t == 0) a.lam_t[k] = 2.0 - 2.0 * cos(pi * (k + 0.5 * a.l) / (nt + 0.5 * a.l));
    }
    a.Vp64[(size_t)t * ntp + k] = v;
    a.Vp32[(size_t)k * ntp + t] = (float)v;
    a.Vp16[(size_t)k * ntp + t] = (_Float16)v;
    const _Float16 hi = (_Float16)(v * kVSplitScale);
    a.Vp16s[(size_t)k * ntp + t] = hi;
    a.Vp16s[((size_t)ntp + k) * ntp + t] = (_Float16)(v * kVSplitScale - (double)hi);
    a.Vpbf[(size_t)k * ntp + t] = bf16_rne((float)v);
  }
}

struct AxisTables {
  int N, neumann;
  double ih2;  // 1/h^2
  double *tw, *ct, *lam;
  float *twf, *ctf;
};

// Twiddles cos/sin(2 pi m/N), DCT post-twiddles cos/sin(pi m/(2N)) and the
// eigenvalues of the one-axis negative Laplacian over h^2 (Algorithm 2).
__global__ void k_axis_tables(AxisTables a) {
  const double pi = 3.14159265358979323846264338327950288;
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < a.N; m += gridDim.x * blockDim.x) {
    const double c = cos(2.0 * pi * m / a.N), s = sin(2.0 * pi * m / a.N);
    const double cc = cos(pi * m / (2.0 * a.N)), cs = sin(pi * m / (2.0 * a.N));
    a.tw[2 * m] = c;
    a.tw[2 * m + 1] = s;
    a.ct[2 * m] = cc;
    a.ct[2 * m + 1] = cs;
    a.twf[2 * m] = (float)c;
    a.twf[2 * m + 1] = (float)s;
    a.ctf[2 * m] = (float)cc;
    a.ctf[2 * m + 1] = (float)cs;
    const double ev = a.neumann ? 2.0 - 2.0 * cos(pi * m / a.N) : 2.0 - 2.0 * cos(2.0 * pi * m / a.N);
    a.lam[m] = ev * a.ih2;
  }
}

void carve_axis(Carver& C, Axis& ax, int N, bool neumann, double h, hipStream_t s) {
  ax.N = N;
  radices(N, ax.radix, &ax.npass);
  ax.kind = neumann ? 1 : 0;
  AxisTables t{N, neumann ? 1 : 0, 1.0 / (h * h), C.take<double>(2 * N), C.take<double>(2 * N),
               C.take<double>(N), C.take<float>(2 * N), C.take<float>(2 * N)};
  if (!C.ok) return;
  hipLaunchKernelGGL(k_axis_tables, dim3((N + 255) / 256), dim3(256), 0, s, t);
  ax.tw = t.tw;
  ax.ct = t.ct;
  ax.lam = t.lam;
  ax.twf = t.twf;
  ax.ctf = t.ctf;
}

}  // namespace

}  // namespace mfg

using mfg::fail;

extern "C" int mfg_pcg_noalloc(const mfg_problem_t* pb, const double* b, double* u, double rtol,
                               int maxit, hipStream_t stream, int* iters, double* relres) {
  using namespace mfg;
  if (!pb || !b || !u) return fail(MFG_ERR_INVALID_ARG, "NULL argument");
  if (b == u) return fail(MFG_ERR_INVALID_ARG, "b and u must not alias");
  if (!(rtol >= 0.0) || maxit < 1) return fail(MFG_ERR_INVALID_ARG, "need rtol >= 0, maxit >= 1");
  Plan P;
  int rc = setup_problem(P, pb, stream);
  if (rc) return rc;
  const Geom& g = P.g;
  if (g.nt > 128)
    return fail(MFG_ERR_UNSUPPORTED, "mfg_pcg_noalloc serves N_t <= 128");
  unsigned char* base = nullptr;
  if ((rc = scratch_of(P.device, &base))) return rc;
  Carver C{base};
  // tables
  const int nt = g.nt, ntp = (nt + 15) / 16 * 16;
  P.ntp = ntp;
  TimeTables tt{nt, P.l, ntp, C.take<double>((size_t)nt * nt), C.take<double>(nt),
                C.take<double>((size_t)ntp * ntp), C.take<float>((size_t)ntp * ntp),
                C.take<_Float16>((size_t)ntp * ntp), C.take<_Float16>(2 * (size_t)ntp * ntp),
                C.take<unsigned short>((size_t)ntp * ntp)};
  // workspace: r, z, p (two buffers), q and the preconditioner intermediate;
  // the reduction partials and scalars
  const size_t n = (size_t)g.n;
  P.r = C.take<double>(n);
  P.z = C.take<double>(n);
  P.p = C.take<double>(n);
  P.p2 = C.take<double>(n);
  P.q = C.take<double>(n);
  P.tmp = C.take<double>(n);
  P.red.max_blocks = 32768;
  P.red.partials = C.take<double>((size_t)T_COUNT * kSlotsPerSite * P.red.max_blocks);
  P.red.scal = C.take<double>(S_COUNT);
  if (!C.ok)
    return fail(MFG_ERR_UNSUPPORTED,
                "problem too large for the no-allocation entry point (64 MiB of scratch: "
                "about 2^20 cells)");
  {
    const long long colblk = (g.M + 63) / 64;
    const long long kchunks = (((g.nt + 15) / 16) + 7) / 8;
    if (colblk * kchunks > P.red.max_blocks)
      return fail(MFG_ERR_UNSUPPORTED, "grid too large for the time-transform reduction");
  }
  hipStream_t s = stream;
  hipLaunchKernelGGL(k_time_tables, dim3((ntp * ntp + 255) / 256), dim3(256), 0, s, tt);
  P.Vt64 = tt.Vt64;
  P.lam_t = tt.lam_t;
  P.Vp64 = tt.Vp64;
  P.Vp32 = tt.Vp32;
  P.Vp16 = tt.Vp16;
  P.Vp16s = tt.Vp16s;
  P.Vpbf = tt.Vpbf;
  if (g.has0) {
    carve_axis(C, P.ax0, g.n0, axis_neumann(pb, 0), axis_spacing(pb, 0), s);
    carve_axis(C, P.ax1, g.n1, axis_neumann(pb, 1), axis_spacing(pb, 1), s);
  } else {
    carve_axis(C, P.ax1, g.n1, axis_neumann(pb, 0), axis_spacing(pb, 0), s);
  }
  if (!C.ok) return fail(MFG_ERR_UNSUPPORTED, "problem too large for the no-allocation entry point");
  // the scalar block starts at zero on every call (earlier calls left theirs)
  launch_fill(P.red.scal, S_COUNT, 0.0, s);
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MFG_ERR_HIP, std::string("table launch: ") + hipGetErrorString(e));
  }
  double host_scal[S_COUNT] = {};
  P.host_scal = host_scal;
  P.last_pcg_its = g_last_its[P.device];
  rc = run_pcg(P, b, u, rtol, maxit, iters, nullptr, relres);
  g_last_its[P.device] = P.last_pcg_its;
  return rc;
}
