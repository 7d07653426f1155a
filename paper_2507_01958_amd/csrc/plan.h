// Host-side plan object behind mfg_plan_t.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "mfg_internal.h"

struct mfg_plan_s;

namespace mfg {

// Launch-shape choices of the kernels that have more than one (set by the
// autotuner or the MFG_TUNE environment variable, "key=value,...").
struct Tune {
  int f64_cb = 1;    // time GEMM (float64): 16-node column blocks per wave
  int lp_cb = 1;     // time GEMM (low precision): column blocks per wave, forward
  int lp_waves = 8;  // time GEMM (low precision): waves per block (4 or 8), forward
  int lp_cb_i = 1;     // ... the same two for the inverse transform
  int lp_waves_i = 8;
  int rows_elems = 1024;  // row transforms: complex elements per block
  int cols_lines = 4;     // column solves: complex lines (column pairs) per block
  int tgemm_pers = 0;     // persistent time GEMM (whole V in LDS) when N_t <= 128
  int fft_reg = 1;        // register-resident FFTs for axis lengths 64, 128, 256
  int aat_tc = 0;         // A kernel: time slices per block (0: chosen from the grid)
  int aat_big = 1;        // A kernel (d = 2): 16 << aat_big tile rows, 256 << aat_big threads
  // PCG update with the mixed-precision preconditioner: 1 flexible
  // (Polak-Ribiere), 0 standard, -1 by precision (standard for float32, whose
  // preconditioner is symmetric to float32 rounding; flexible for float16 and
  // bfloat16)
  int flex = -1;
  // time GEMM with low-precision products also when N_t > 128 (V streamed
  // through LDS); 0: float64 products there
  int lp_stream = 1;
  // right-hand-side kernel: time slices walked per block (0: chosen from the
  // geometry alone; not autotuned, so batched and single-plan runs agree)
  int rhs_tc = 0;
  // forward preconditioner pass fused (time GEMM + row transforms) where it
  // applies (mixed modes, axis 1 of 256 nodes, N_t <= 128); 0: separate kernels
  int fuse_fwd = 1;
  // inside PCG, the update (x += alpha p, r -= alpha q) runs in the fused
  // forward pass too; 0: its own kernel
  int fuse_upd = 1;
  // inverse pass fused (row transforms + inverse time GEMM) where it applies
  // (as fuse_fwd, and one 16-node tile per wave in the inverse GEMM)
  int fuse_inv = 1;
  // batched solves: the A phase as a persistent grid over a tile queue
  // (0: one block per instance tile)
  int batch_queue = 0;
};

// Optional per-kernel timing with HIP events recorded on the plan's stream
// around each launch (enabled by mfg_profile). Event pairs are resolved when a
// report is requested or when many are pending.
struct Profiler {
  bool on = false;
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<long, double>> acc;  // name -> (calls, total ms)
};

struct Plan {
  mfg_problem_t pb{};
  Tune tune{};
  mutable Profiler prof;
  // Device flag that the kernels of a PCG loop test to skip their work once
  // the solve has converged (set only while mfg_pcg / a CP step iterates).
  const double* pcg_done = nullptr;
  int last_pcg_its = 0;  // iterations of the previous solve (launch chunking)
  // CP projections start PCG from the previous projection's solution (kept in
  // u) when warm_start is set and u holds one (u_valid)
  bool warm_start = false, u_valid = false;
  // Grids of the last launches that stored p.q and r.z partials: the update
  // and the A kernel sum that many partials themselves.
  mutable int pq_blocks = 0, rz_blocks = 0;
  // r.r partials of the last update (rr_blocks), and the count the next time
  // GEMM launch folds its stopping test over (rr_gate; 0: none)
  mutable int rr_blocks = 0, rr_gate = 0;
  Geom g{};
  int precision = MFG_FP64;
  int l = 1;
  double gamma = 0.0;
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cus = 256;

  // problem data (plan-owned copies)
  double* V = nullptr;   // M
  double* m0 = nullptr;  // M
  // terminal cost g = (m - mbar)/beta (beta = 0: none): the target density and
  // the last slice's potential VT = V - mbar/(beta dt)
  double beta = 0.0;
  double* mbar = nullptr;  // M
  double* VT = nullptr;    // M

  // time transform (Algorithm 1): Vt[t][k] = V[k][t] (V is symmetric)
  double* Vt64 = nullptr;
  float* Vt32 = nullptr;
  _Float16* Vt16 = nullptr;
  unsigned short* Vtbf = nullptr;
  double* lam_t = nullptr;  // N_t eigenvalues (eq. eigs)
  // V zero-padded to ntp x ntp (ntp = N_t rounded up to 16, when N_t <= 128)
  // for the low-precision kernels, which copy it to LDS with 16-byte loads
  int ntp = 0;
  double* Vp64 = nullptr;  // float64 copy: Vp64[t * ntp + k] = V[k][t]
  float* Vp32 = nullptr;
  _Float16* Vp16 = nullptr;
  // float32-accurate split for the blocked float32 kernel: rows 0..ntp-1 the
  // float16 rounding hi of 2^8 V, rows ntp..2ntp-1 the float16 rounding of
  // 2^8 V - hi
  _Float16* Vp16s = nullptr;
  unsigned short* Vpbf = nullptr;
  // N_t > 128: the low-precision V of the plan's precision for the streaming
  // kernel, V[k][t] at k * ntps + t, zero-padded to ntps (N_t rounded up to
  // 128); the float32 split stores the lo rows after the hi rows
  int ntps = 0;
  const void* Vs_lp = nullptr;

  // spatial transforms (Algorithm 2)
  Axis ax0{}, ax1{};

  // workspace (n-vectors)
  double *r = nullptr, *z = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr;
  double *tmp = nullptr;  // preconditioner intermediate (float64 or float32 view)
  double *b = nullptr, *u = nullptr;
  // z = xi + sigma ybar handed from one CP step's back-projection to the next
  // step's right-hand side inside one multi-step call ((1 + 2d) n values)
  double *zn = nullptr;
  RedBuf red{};
  double* host_scal = nullptr;  // pinned mirror of red.scal

  std::vector<void*> dev_allocs;
  std::vector<void*> host_allocs;
};

// Record the start / end of a launch for the profiler (no-op when disabled).
int prof_begin(const Plan& P, const char* name, hipStream_t s);
void prof_end(const Plan& P, int id, hipStream_t s);

struct ProfScope {
  const Plan& P;
  hipStream_t s;
  int id;
  ProfScope(const Plan& p, const char* name, hipStream_t st) : P(p), s(st), id(prof_begin(p, name, st)) {}
  ~ProfScope() { prof_end(P, id, s); }
};

// Whether PCG takes the flexible update on this plan.
inline bool pcg_flexible(const Plan& P) {
  if (P.precision == MFG_FP64) return false;
  if (P.tune.flex >= 0) return P.tune.flex != 0;
  return P.precision != MFG_MIXED_FP32;
}

// api.hip: validate a problem and fill the plan's geometry (no allocation);
// PCG on the plan's workspace (r_ready: the start r = b, b.b, status reset was
// already done by the kernel that formed b); copy the device scalars to
// P.host_scal (synchronises the plan's stream).
int setup_problem(Plan& P, const mfg_problem_t* pb, hipStream_t stream);
// Copy the Tune fields that are not launch shapes (method choices, settings).
void keep_untuned(const Tune& from, Tune& to);
// Boundary type of axis a of the problem (0 = x, 1 = y): true for Neumann.
bool axis_neumann(const mfg_problem_t* pb, int a);
// Spacing of axis a (Section 2): (b - a)/N periodic, (b - a)/(N + 1) Neumann.
double axis_spacing(const mfg_problem_t* pb, int a);
int run_pcg(Plan& P, const double* b, double* x, double rtol, int maxit, int* iters_out,
            double* relres_rec, double* relres_true, bool r_ready = false, bool warm = false);
int read_scalars(Plan& P);
int fail(int code, const std::string& msg);
// Radix sequence (4s, then 2s, then 3s) of a spatial FFT of length N.
void radices(int N, int* r, int* np);

// Launch-shape autotuner (tune.hip): cached choice for the plan's key, and
// measurement of the candidates (allow_pers = false excludes the persistent
// time GEMM, which batched launches do not use).
bool tune_lookup(const Plan& P, Tune* out);
void batch_shape(Tune& t);
int autotune(Plan& P, int effort, bool allow_pers);

}  // namespace mfg

struct mfg_plan_s {
  mfg::Plan P;
};
