// Internal declarations shared by the HIP translation units of libmfg.
//
// Internal axes: a space-time n-vector is [t][i0][i1] with i1 contiguous.
// For d = 2, axis 0 is x (N_x nodes, stride N_y) and axis 1 is y (N_y nodes,
// stride 1); flux components 0,1 act along x and 2,3 along y. For d = 1 the
// single axis x is stored as axis 1 (n0 = 1) and its components are 0,1.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/mfg.h"

namespace mfg {

constexpr int kMaxPass = 16;
constexpr int kMaxAxisN = 1024;
constexpr int kMaxNt = 4096;
constexpr int kSlotsPerSite = 4;  // reduction values per site

// Geometry and constants of one problem, passed by value to kernels.
struct Geom {
  int n0, n1;      // internal axis sizes (n0 = 1 when d = 1)
  int nt, M;       // time steps, nodes per slice
  long long n;     // nt * M
  int has0;        // axis 0 present (d = 2)
  int bcm;         // Neumann axes: bit 0 axis 1 (j), bit 1 axis 0 (i); else periodic
  int ncomp;       // 2d flux components
  int cb1;         // first flux component acting along axis 1 (2 if d=2, 0 if d=1)
  double ih0, ih1;     // 1/h per axis (0 when absent)
  double ih0sq, ih1sq; // 1/h^2 per axis (0 when absent)
  double nu, dt, idt, idt2;
  // coupling f(x, m) = c2 m^2 + c1 m + V(x); on the last time slice the
  // terminal cost g = (m - mbar)/beta makes the linear coefficient c1T
  // (= c1 + 1/(beta dt), or c1 without a terminal cost) and the potential VT
  double c2, c1, c1T;
  // Hamiltonian |p|^q'/q' (eq. power_hamiltonian): qp = q', q = q'/(q' - 1)
  // the exponent of the flux cost b-hat
  double q, qp;
};

// Deterministic two-level reduction: per-block partials, then a sum in a fixed
// order, by a one-block finisher kernel or inside the kernel that consumes it.
struct RedBuf {
  double* partials;   // [slot][block]
  double* scal;       // device scalar block
  int max_blocks;
};

// Device scalar slots.
enum ScalarSlot {
  S_RHO = 0,    // r.z of the current iterate
  S_PQ = 1,     // p.q
  S_ALPHA = 2,
  S_BETA = 3,
  S_RR = 4,     // r.r
  S_BB = 5,     // b.b
  S_ZQ = 6,     // z.q (flexible beta)
  S_DONE = 7,   // 1 when converged
  S_TOL2 = 8,   // (rtol ||b||)^2 threshold factor rtol^2 (set by host)
  S_BAD = 9,    // 1: breakdown, 2: non-finite
  S_DM = 10,    // ||m' - m||^2 of the last CP step
  S_AUX0 = 11,
  S_AUX1 = 12,
  S_ITS = 13,   // PCG iterations done (counted by the r.r stopping test)
  S_SIGMA = 14, // CP step sizes of the current iteration (graph-driven runs)
  S_TAU = 15,
  S_THETA = 16,
  S_CPIT = 17,  // CP iterations done (graph-driven runs)
  S_ZMODE = 18, // 1 while the right-hand side's input z is in the plan's buffer
  S_MASS = 19,  // mass drift of the primal iterate (statistics)
  S_COUNT = 24
};

enum ReduceSite { T_BB = 0, T_PQ = 1, T_RR = 2, T_RZ = 3, T_DM = 4, T_AUX = 5, T_COUNT = 8 };

// What the finisher does with the summed partials of a site.
// (p.q, r.z and r.r are summed by their consumers: the update, the A kernel
// and the preconditioner's forward time transform.)
enum FinishOp {
  OP_BB = 0,        // b.b -> S_BB, S_RR; S_DONE if zero; S_BAD if non-finite
  OP_DM = 6,        // -> S_DM
  OP_AUX = 7        // -> S_AUX0, S_AUX1
};

constexpr int kStreamGrid = 2048;  // blocks of the streaming kernels
constexpr int kFinishThreads = 1024;  // threads of a one-block finisher (16 waves)
constexpr int kFinishDepth = 16;     // partials each finisher thread loads at once

// The float32 time transform of the blocked kernel runs on the float16 matrix
// cores at float32 accuracy: operands and V are split into a float16 term and
// a float16 remainder, and three products (hi hi, hi lo, lo hi; the lo lo term
// is below float32 rounding) accumulate in float32. V is scaled by 2^8 before
// the split so that its remainder stays in the float16 normal range.
constexpr double kVSplitScale = 256.0;

// One spatial transform axis (Algorithm 2): real-to-real transform built on a
// complex Stockham FFT of length N with two real lines packed per complex one.
struct Axis {
  int N;
  int npass;
  int radix[kMaxPass];
  int kind;            // 0: discrete Hartley (periodic), 1: DCT-II (Neumann)
  const double* tw;    // cos/sin(2 pi m / N), interleaved, m < N
  const float* twf;
  const double* ct;    // cos/sin(pi k / (2N)), interleaved, k < N
  const float* ctf;
  const double* lam;   // eigenvalue of the negative Laplacian / h^2 at frequency k
};

struct Plan;

// ---- launchers (each defined in its .hip file) ----
// stencil.hip
// zin (optional): z = xi + sigma ybar stored by the previous back-projection;
// init_rtol >= 0: b is the PCG residual of x = 0 and the kernel also does the
// PCG start (b.b, status reset with tolerance init_rtol)
void launch_rhs(const Plan& P, const double* xi, const double* ybar, double sigma,
                const double* m0, double* b, hipStream_t s, const double* zin = nullptr,
                double init_rtol = -1.0);
void launch_apply_C(const Plan& P, const double* y, double* b, hipStream_t s);
void launch_apply_CT(const Plan& P, const double* u, double* y, hipStream_t s);
void launch_AAt(const Plan& P, const double* u, double* q, bool reduce_pq, hipStream_t s);
void launch_pdir_AAt(const Plan& P, const double* z, const double* pold, double* pnew, double* q,
                     bool first, hipStream_t s);
void launch_prox(const Plan& P, const double* v, double tau, double* y, hipStream_t s);
// VT = V - mbar/(beta dt) (V without a terminal cost)
void launch_terminal_potential(const Plan& P, hipStream_t s);
// value function from the multiplier lam: u[k] = -lam[k] (k < N_t), u[N_t] = g(m^{N_t})
void launch_value(const Plan& P, const double* lam, const double* y, double* u, hipStream_t s);
void launch_hjb_residual(const Plan& P, const double* y, const double* u, double* R,
                         hipStream_t s);
// vout (optional): stores v = y - tau xi' (the prox input) for the reverse sweep;
// zout (optional): stores z = xi' + (sigma / theta) ybar' in place of xi', ybar'
void launch_backproj_prox(const Plan& P, const double* u, double* xi, double* y, double* ybar,
                          double tau, double theta, hipStream_t s, double* vout = nullptr,
                          double* zout = nullptr, double sigma = 0.0);
// vec.hip
// r = b, b.b, PCG status reset (the solve starts at x = 0: the first update
// writes x)
void launch_pcg_init(const Plan& P, const double* b, double* r, double rtol, hipStream_t s);
void launch_update(const Plan& P, double* x, double* r, const double* p, const double* q,
                   bool first, hipStream_t s);
void launch_residual(const Plan& P, const double* b, const double* Ax, hipStream_t s);
void launch_finish(const Plan& P, int site, int nblocks, int op, hipStream_t s);
void launch_fill(double* x, long long n, double v, hipStream_t s);
void launch_cp_init(const Plan& P, double* xi, double* y, double* ybar, hipStream_t s);
// max over time slices of |h^d sum_i m^{t+1}_i - h^d sum_i m0_i| for the m block
// of y, into the device scalar S_MASS
void launch_mass_drift(const Plan& P, const double* y, hipStream_t s);
// adjoint.hip
void launch_adj_prox(const Plan& P, double* gy, const double* gyb, const double* v, double tau,
                     double theta, double* gxi, double* gVc, hipStream_t s);
void launch_sum_slices(const Plan& P, const double* in, const double* in2, double* out,
                       hipStream_t s);
void launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t s);
// precond.hip
void launch_update_precond(const Plan& P, double* x, double* r, const double* p,
                           const double* q, double* z, bool first, hipStream_t s);
void launch_precond(const Plan& P, const double* r, double* z, bool fused_dots,
                    const double* q, hipStream_t s);

}  // namespace mfg
