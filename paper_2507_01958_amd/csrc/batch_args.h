// Argument blocks of the kernels that run both for one plan and batched over
// many plans in one launch. A batched launch takes a device array of these
// (one per instance) plus block offsets: instance i owns blocks
// [off[i], off[i+1]) and runs the same body with its local block id, so a
// batched run performs exactly the arithmetic of the single-plan run.
#pragma once

#include "mfg_internal.h"

namespace mfg {

// Solve context of Algorithm 2: eigenvalue tables and constants of S.
struct SolveCtx {
  const double* lam_t;  // time eigenvalues (eq. eigs)
  const double* lam0;   // axis-0 eigenvalues / h0^2 (nullptr when absent)
  const double* lam1;   // axis-1 eigenvalues / h1^2
  double nu, idt, idt2;
  double norm;          // 1 / (N0 N1)
};

// `done` (batched runs only, else null): the instance's converged flag; the
// PCG-loop bodies return at once when it is set.
struct InitArgs {
  long long n;
  const double* b;
  double* r;
  RedBuf rb;
  double tol2;  // (rtol)^2 for the status reset
};

// npq, nrz: partial counts of the p.q site (the A kernel's grid) and of the
// r.z site (the inverse time GEMM's grid), summed by each block.
struct UpdArgs {
  long long n;
  double* x;
  double* r;
  const double* p;
  const double* q;
  RedBuf rb;
  const double* done;
  int npq, nrz;
  int first;  // first iteration: x = alpha p (x is not read; the solve starts at 0)
};

struct FinishArgs {
  RedBuf rb;
  int site, nblocks, op;
  const double* done;
};

// nrz > 0 (PCG direction form): partial count of the r.z site, from which each
// block forms beta (flex: the flexible formula).
struct AatArgs {
  Geom g;
  const double* src;   // u, or z when forming p = z + beta p_old
  const double* pold;
  double* pnew;
  double* q;
  RedBuf rb;
  int tc, first, reduce;
  const double* done;
  int nrz, flex;
};

// Step sizes either by value or from device memory (pointer non-null).
// zin (optional): z = xi + sigma ybar as written by the previous step's
// back-projection, read in place of xi and ybar; with zmode_dev set (batched
// runs) only while *zmode_dev != 0.
// init (PCG start fused into the right-hand side): b is the PCG residual r
// (the solve starts at x = 0), block partials of b.b go to the T_BB site and
// block 0 resets the PCG status with tol2 = rtol^2 (by value or from tol2_dev).
// tc: time slices per block (each block owns 256 consecutive cells of a slice
// and walks tc slices; the grid is ceil(M / 256) * ceil(N_t / tc) blocks).
struct RhsArgs {
  Geom g;
  const double* xi;
  const double* ybar;
  double sigma;
  const double* sigma_dev;
  const double* m0;
  double* b;
  const double* zin;
  const double* zmode_dev;
  int init;
  RedBuf rb;
  double tol2;
  const double* tol2_dev;
  int tc;
};

struct BackprojArgs {
  Geom g;
  const double* u;
  double* xi;
  double* y;
  double* ybar;
  const double* V;
  const double* VT;  // potential of the last time slice (terminal cost folded in)
  double tau, theta;
  const double* tau_dev;
  const double* theta_dev;
  RedBuf rb;
  double* vout;
  // zout (optional): in place of xi' and ybar', store z = xi' + sigma' ybar'
  // with sigma' = sigma / theta, the input of the next step's right-hand side
  // (sigma by value or from sigma_dev); zflag (batched runs): set to 1 when z
  // is stored, 0 when xi' and ybar' are.
  double* zout;
  double sigma;
  const double* sigma_dev;
  double* zflag;
};

template <typename T>
struct RowsArgs {
  T* data;
  int nrows;
  Axis ax;
  int mode, lpb;
  SolveCtx sc;
  int n0;
  const double* done;
  int reg;  // register path (fft_reg.h) for axis lengths 64, 128, 256
};

template <typename T>
struct ColsArgs {
  T* data;
  Geom g;
  Axis ax;
  int cw;
  SolveCtx sc;
  const double* done;
  int reg;
};

template <typename TX, typename TY>
struct GemmArgs {
  const void* V;   // float64 Vt (chunked kernel) or the padded copy (low precision)
  const TX* X;
  TY* Y;
  int nt, M, ncolblk, dotmode;
  const double* rvec;
  const double* qvec;
  RedBuf rb;
  const double* done;
  int nrr;  // > 0: first take the PCG r.r check over that many partials
  int ldv;  // row stride of the streamed low-precision V table (N_t > 128)
};

// Instance that owns block b of a batched launch (off[0] = 0 <= b < off[ninst]).
__device__ __forceinline__ int batch_instance(const int* off, int ninst, int b) {
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- host-side builders and batched launchers (defined next to each kernel) ----
struct Plan;
InitArgs pcg_init_args(const Plan& P, const double* b, double* r, double rtol);
int pcg_init_grid(const Plan& P);
UpdArgs update_args(const Plan& P, double* x, double* r, const double* p, const double* q,
                    bool first);
int update_grid(const Plan& P);
FinishArgs finish_args(const Plan& P, int site, int nblocks, int op);
RhsArgs rhs_args(const Plan& P, const double* xi, const double* ybar, double sigma,
                 const double* sigma_dev, double* b, const double* zin = nullptr,
                 const double* zmode_dev = nullptr);
int rhs_grid(const Plan& P);
BackprojArgs backproj_args(const Plan& P, const double* u, double* xi, double* y, double* ybar,
                           double tau, double theta, const double* tau_dev,
                           const double* theta_dev, double* vout);
int backproj_grid(const Plan& P);
AatArgs aat_args(const Plan& P, const double* z, const double* pold, double* pnew, double* q,
                 bool first, const double* done, int* grid);
// return the size class of the instance's launch (0: LDS path, else N); T is
// the preconditioner's intermediate (float in the mixed modes, double in FP64)
template <typename T>
int batch_rows_args(const Plan& P, T* data, int mode, const double* done, RowsArgs<T>* out,
                    int* blocks, size_t* shm, int* threads);
template <typename T>
int batch_cols_args(const Plan& P, T* data, const double* done, ColsArgs<T>* out, int* blocks,
                    size_t* shm, int* threads);
template <typename TX, typename TY>
GemmArgs<TX, TY> batch_gemm_args(const Plan& P, int mode, const TX* X, TY* Y, int dotmode,
                                 const double* r, const double* q, const double* done,
                                 int* blocks);

// streaming low-precision time GEMM (N_t > 128); the block count differs
// between directions (the float32 split's forward takes one tile per wave)
template <typename TX, typename TY>
GemmArgs<TX, TY> batch_gemm_lps_args(const Plan& P, int mode, const TX* X, TY* Y, int dotmode,
                                     const double* r, const double* q, const double* done,
                                     int* blocks);
template <typename TX, typename TY>
void launch_gemm_lps_batch(int mode, const GemmArgs<TX, TY>* A, const int* off, int ninst,
                           int total, hipStream_t s);
// float64 time GEMM: the (KB, CB) class of the instance's launch in kb, cb
GemmArgs<double, double> batch_gemm64_args(const Plan& P, const double* X, double* Y, int dotmode,
                                           const double* r, const double* q, const double* done,
                                           int* blocks, int* kb, int* cb);
void launch_gemm64_batch(int kb, int cb, const GemmArgs<double, double>* A, const int* off,
                         int ninst, int total, hipStream_t s);

void launch_update_batch(const UpdArgs* A, const int* off, int ninst, int total, hipStream_t s);
void launch_finish_batch(const FinishArgs* F, int ninst, hipStream_t s);
void launch_cp_advance_batch(double* scal, int stride, int ninst, const double* sched, int maxit,
                             hipStream_t s);
// queue != nullptr: the persistent form over a tile queue (queue: one device
// int; qgrid: resident blocks, aat_queue_grid; 0 = not available).
void launch_aat_batch(bool has0, const AatArgs* A, const int* off, int ninst, int total,
                      hipStream_t s, int* queue = nullptr, int qgrid = 0);
int aat_queue_grid(bool has0);
void launch_rhs_batch(const RhsArgs* A, const int* off, int ninst, int total, hipStream_t s);
void launch_backproj_batch(const BackprojArgs* A, const int* off, int ninst, int total,
                           hipStream_t s);
template <typename T>
void launch_rows_batch(int cls, const RowsArgs<T>* A, const int* off, int ninst, int total,
                       size_t shm, int threads, hipStream_t s);
template <typename T>
void launch_cols_batch(int cls, const ColsArgs<T>* A, const int* off, int ninst, int total,
                       size_t shm, int threads, hipStream_t s);
template <typename TX, typename TY>
void launch_gemm_batch(int mode, int ntp, int cb, int waves, const GemmArgs<TX, TY>* A,
                       const int* off, int ninst, int total, hipStream_t s);

}  // namespace mfg
