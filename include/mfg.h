/*
 * mfg.h -- C ABI of the MI355X (gfx950) solver for time-dependent variational
 * mean field games, after Ljosheim, Kalise, Pearson and Silva,
 * "Parallel-in-Time Preconditioning for Time-Dependent Variational Mean Field
 * Games" (arXiv 2507.01958).
 *
 * The library runs the paper's Chambolle-Pock iteration (Section 3,
 * eq. pasosChamPock) on the finite-difference discretisation (Section 2,
 * problem VMFG_h): a per-cell proximal step on the cost b-hat + F, then the
 * projection onto the discrete Fokker-Planck constraint (eq. CC*), which is a
 * conjugate-gradient solve with the reduced matrix of eq. largeA,
 * preconditioned by the parallel-in-time operator of eq. pstrec
 * (Algorithms 1 and 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All vector arguments are DEVICE pointers to contiguous float64 arrays on
 *   the GPU that was current when the plan was made, unless stated otherwise.
 *   The caller owns them; the library never frees or keeps them.
 * - Sizes: M = N_x * N_y (N_y = 1 when d = 1), n = N_t * M, and a primal
 *   vector holds (1 + 2d) n values.
 * - Layout: an n-vector is [t][i][j] with j fastest (time slice t, node (i, j)).
 *   A primal vector is the block m (n values) followed by the 2d flux blocks
 *   w^(c) (n values each, c = 0..2d-1; even c is the non-negative and odd c the
 *   non-positive half-line of the cone K of Section 2; c = 0, 1 act along x,
 *   c = 2, 3 along y). Slice t of m holds m^{t+1}; slice t of w holds w^t; the
 *   initial density m^0 = m0 is eliminated (Section 2.1: 5 N_t N_x N_y
 *   unknowns when d = 2).
 * - Every call is asynchronous on the plan's stream, except outputs written to
 *   host pointers (iteration counts, residuals, statistics), which synchronise
 *   the stream before returning.
 * - Return value: MFG_OK or an mfg_status_t error code; nothing is thrown
 *   across the ABI. On error the contents of output buffers are unspecified
 *   and mfg_last_error() describes the failure (thread-local string).
 * - A plan is not thread-safe; different plans are independent.
 */
#ifndef MFG_H
#define MFG_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFG_OK = 0,
  MFG_ERR_INVALID_ARG = 1,   /* bad shape, parameter or pointer */
  MFG_ERR_UNSUPPORTED = 2,   /* valid but not implemented (q' out of range, FFT size) */
  MFG_ERR_NOT_CONVERGED = 3, /* PCG hit maxit; iters/relres are still filled */
  MFG_ERR_BREAKDOWN = 4,     /* non-positive curvature or r.z in PCG */
  MFG_ERR_NONFINITE = 5,     /* NaN or Inf met in an input or a residual */
  MFG_ERR_HIP = 6,           /* a HIP runtime call failed */
  MFG_ERR_OOM = 7            /* device allocation failed */
} mfg_status_t;

/* Boundary conditions: periodic (the torus of Section 2) or Neumann (the
 * no-flux problem MFG_Omega with the Section 4.3 matrices), on every axis or,
 * for d = 2, one type per axis (Section 4.3: the spatial solver allows
 * different conditions in x and y; each axis takes its own spacing, one-axis
 * operators and transform, DFT or DCT-II). */
typedef enum {
  MFG_BC_PERIODIC = 0,
  MFG_BC_NEUMANN = 1,
  MFG_BC_PERIODIC_X_NEUMANN_Y = 2, /* d = 2 only */
  MFG_BC_NEUMANN_X_PERIODIC_Y = 3  /* d = 2 only */
} mfg_bc_t;

/* Coupling f(x, m) of the running cost F = integral of f dm (Section 2.1):
 * LINEAR f = m + V(x); QUADRATIC f = m^2/2 + V(x), the crowd-aversion coupling
 * of Problem 1 (Section 5.1, where V = -(sin 2 pi y + sin 2 pi x + cos 4 pi x)/2);
 * POTENTIAL f = V(x), independent of m (Problem 2 of Section 5.2 has V = 0). */
typedef enum { MFG_F_LINEAR = 0, MFG_F_QUADRATIC = 1, MFG_F_POTENTIAL = 2 } mfg_coupling_t;

/* Arithmetic of the preconditioner inside PCG. The outer PCG recurrences,
 * the reduced-matrix products, the right-hand side and the prox are float64
 * in every mode. MIXED modes run the spatial solves (Algorithm 2) in float32
 * and the time transform (Algorithm 1) on the matrix cores with float16/
 * bfloat16 inputs (or float32 operands carried as two float16 terms) and
 * float32 accumulation. With float16 and bfloat16 PCG takes its flexible
 * (Polak-Ribiere) form; with float32 the preconditioner is symmetric to
 * float32 rounding and PCG keeps the standard form. Up to N_t = 128 the
 * low-precision time transform holds all of V in LDS; for longer horizons it
 * streams V through LDS in chunks of 32 time rows, with the float16 operands
 * scaled per chunk by powers of two. */
typedef enum {
  MFG_FP64 = 0,
  MFG_MIXED_FP32 = 1,  /* time transform at fp32 accuracy (fp32 operands split into two fp16
                          terms, three fp16 matrix-core products, fp32 accumulate), spatial
                          solves fp32 */
  MFG_MIXED_FP16 = 2,  /* time transform fp16 inputs / fp32 accumulate */
  MFG_MIXED_BF16 = 3   /* time transform bf16 inputs / fp32 accumulate */
} mfg_precision_t;

/* Problem statement (Sections 1-2, Section 5 setup). */
typedef struct {
  int d;             /* space dimension, 1 or 2 */
  int n[2];          /* N_x, N_y: nodes per axis (interior nodes if Neumann);
                        n[1] is ignored when d = 1. Each must be >= 4 and of
                        the form 2^a 3^b (spatial transform sizes). */
  int nt;            /* N_t time steps, 2 <= N_t <= 4096; N_t times the
                        spatial node count must be below 2^31 */
  double T;          /* horizon T > 0; dt = T / N_t */
  double lo[2], hi[2]; /* domain [a,b] x [c,d]: periodic dx = (b-a)/N_x,
                          Neumann dx = (b-a)/(N_x+1) (Section 2), per axis */
  int bc;            /* mfg_bc_t */
  double nu;         /* viscosity nu >= 0 */
  double qprime;     /* Hamiltonian |p|^q'/q' (eq. power_hamiltonian), 1.2 <= q' <= 6
                        (2 in the paper's experiments); the flux cost is then
                        |w|^q/(q m^(q-1)) with q = q'/(q'-1). mfg_cp_adjoint
                        needs q' = 2. */
  double gamma;      /* strong-convexity constant of the accelerated CP
                        step sizes (Section 5); > 0 */
  int l;             /* time preconditioner of eq. prec: 1 = DCT-VIII (exact
                        at nu = 0), 2 = DST-I */
  int precision;     /* mfg_precision_t */
  int coupling;      /* mfg_coupling_t (0: f = m + V) */
  double beta;       /* terminal cost g(x, m) = (m - mbar(x))/beta of Section 5.2
                        when beta > 0 (it enters the objective as G/dt on the last
                        time slice, G the primitive of g); 0: g = 0. mbar is set by
                        mfg_set_target and is zero until then. */
} mfg_problem_t;

typedef struct mfg_plan_s* mfg_plan_t;

/* Build a plan: validate the problem, compute the grid constants and the
 * eigenvalue / transform tables (eqs. eigs, lambda1, lambda2) and allocate the
 * plan's workspace (about 8 n-vectors plus one primal vector). V (the potential
 * of the coupling, M values) and m0 (initial density, M values, >= 0 and
 * finite) are device pointers; the plan copies them after synchronising
 * `stream` (work queued there may produce them). stream may be 0 (the null
 * stream). */
int mfg_plan(const mfg_problem_t* pb, const double* V, const double* m0,
             hipStream_t stream, mfg_plan_t* out);

/* Release a plan and its workspace (synchronises its stream). */
int mfg_destroy(mfg_plan_t plan);

/* Replace the stream that later calls run on. */
int mfg_set_stream(mfg_plan_t plan, hipStream_t stream);

/* Replace the potential V and/or the initial density m0 (device pointers, M
 * values; NULL keeps the current one). */
int mfg_set_data(mfg_plan_t plan, const double* V, const double* m0);

/* Target density mbar of the terminal cost g = (m - mbar)/beta (Section 5.2):
 * device pointer, M finite values, copied. MFG_ERR_INVALID_ARG if the problem
 * has no terminal cost (beta = 0). */
int mfg_set_target(mfg_plan_t plan, const double* mbar);

/* Proximal step of Section 3: y = prox_{tau phi}(v) for phi = B-hat + F (+ G/dt
 * on the last time slice), cell by cell, with F the primitive of the coupling
 * f (mfg_coupling_t), G that of the terminal cost, and b-hat(m, w) = |w|^2/(2m)
 * on the cone. v, y: primal vectors; y may alias v. tau > 0. */
int mfg_prox(mfg_plan_t plan, const double* v, double tau, double* y);

/* q = A u with A = Cr Cr^T the reduced matrix of eq. largeA (u, q: n-vectors;
 * must not alias). */
int mfg_apply_AAt(mfg_plan_t plan, const double* u, double* q);

/* b = Cr y: the reduced constraint matrix of eq. ABC (first block row
 * eliminated) applied to a primal vector y; b is an n-vector. The constant
 * part m0/dt of the constraint is not included. */
int mfg_apply_C(mfg_plan_t plan, const double* y, double* b);

/* y = Cr^T u (u: n-vector, y: primal vector). */
int mfg_apply_CT(mfg_plan_t plan, const double* u, double* y);

/* z = P^{-1} r with P the preconditioner of eq. prec applied through
 * eq. pstrec (Algorithm 1 along time, Algorithm 2 per time step). Exact (to
 * rounding) in MFG_FP64, approximate in the MIXED modes. r, z: n-vectors, must
 * not alias. */
int mfg_precond(mfg_plan_t plan, const double* r, double* z);

/* Preconditioned CG on A u = b from u = 0 (Sections 3-4): stops when the
 * recursively updated residual satisfies ||r||_2 <= rtol ||b||_2 or after
 * maxit iterations (flexible update with the float16/bfloat16 preconditioner).
 * b, u: n-vectors (must not alias). iters (host, may be NULL): iterations
 * done. relres (host, may be NULL): if non-NULL, the TRUE float64 relative
 * residual ||b - A u|| / ||b|| is computed (one extra product) and stored.
 * Returns MFG_ERR_NOT_CONVERGED if maxit was reached. */
int mfg_pcg(mfg_plan_t plan, const double* b, double* u, double rtol, int maxit,
            int* iters, double* relres);

/* Warm start of the CP projections (enable != 0): each PCG solve of
 * mfg_cp_solve / mfg_cp_solve_tol starts from the previous projection's
 * solution on this plan instead of zero (the residual is then b - A u_prev;
 * the stopping rule stays ||r|| <= rtol ||b||). The first projection after
 * mfg_cp_init starts from zero. Off by default, as in the paper's setup, and
 * not used by batched solves; mfg_cp_adjoint refuses to run while it is on
 * (its recomputed steps start cold). */
int mfg_set_warm_start(mfg_plan_t plan, int enable);

/* Chambolle-Pock state (Section 3, Section 5 schedule). The three vectors are
 * caller-owned device primal vectors ((1+2d) n values each): the dual variable
 * xi, the primal y = (m, w) and its extrapolation ybar. sigma, tau, theta are
 * the current step sizes; iter counts completed iterations. Copying the
 * vectors and the scalars is a complete checkpoint. */
typedef struct {
  double* xi;
  double* y;
  double* ybar;
  double sigma, tau, theta;
  long iter;
} mfg_state_t;

/* Per-iteration statistics of mfg_cp_solve; every pointer is a HOST array of
 * at least n_iter entries, or NULL to skip it. */
typedef struct {
  int* pcg_iters;     /* PCG iterations of each projection */
  double* pcg_relres; /* final recursive relative residual of each PCG */
  double* dm;         /* ||m_{l+1} - m_l||_2 */
  double* mass_drift; /* max over time slices t of |h^d sum_i m^{t+1}_i - h^d sum_i m0_i|
                         for the primal iterate y after the iteration (h^d the cell
                         measure); its projection conserves the mass up to the PCG
                         residual, y itself up to the CP convergence. Costs one
                         read of the m block per iteration. */
} mfg_stats_t;

/* Initial point: xi = 0, y = ybar = (m0 at every time slice, w = 0),
 * sigma = tau = theta = 1, iter = 0. */
int mfg_cp_init(mfg_plan_t plan, mfg_state_t* st);

/* Run n_iter accelerated Chambolle-Pock iterations (eq. pasosChamPock):
 *   xi <- Cr^T A^{-1} (Cr (xi + sigma ybar) - sigma dr)        (eq. CC*)
 *   y' <- prox_{tau phi}(y - tau xi);  theta = (1 + 2 gamma tau)^{-1/2}
 *   ybar <- y' + theta (y' - y);  tau <- theta tau;  sigma <- sigma / theta
 * with each A-solve done by PCG to pcg_rtol (at most pcg_maxit iterations,
 * zero initial guess). The state is updated in place. stats may be NULL.
 * Between the iterations of one call, xi and ybar are kept only through
 * z = xi + sigma ybar in plan workspace (the right-hand side needs nothing
 * else); the last iteration writes them back, so the state after the call is
 * bitwise that of n_iter single-iteration calls. If the call fails with an
 * error other than MFG_ERR_NOT_CONVERGED, the state's vectors are unspecified
 * and st->iter is set to -1 (the state must be re-initialised).
 * Returns MFG_ERR_NOT_CONVERGED (after finishing all iterations) if some PCG
 * solve hit pcg_maxit. */
int mfg_cp_solve(mfg_plan_t plan, mfg_state_t* st, int n_iter, double pcg_rtol,
                 int pcg_maxit, mfg_stats_t* stats);

/* Chambolle-Pock iterations as in mfg_cp_solve, with the stopping and
 * inner-tolerance rules of Section 5: iteration l+1 solves its projection by
 * PCG to the relative residual min(1e-4, max(1e-6, 1e-4 r_l)), where
 * r_l = ||m_l - m_{l-1}||_2 is the change made by the iteration before it
 * (1e-4 for the first iteration of the call), and the loop ends after the
 * first iteration with r <= cp_tol, or after max_iter iterations. The paper
 * takes cp_tol = 1e-4 ||m0||_2. *n_done (HOST, may be NULL) receives the
 * number of iterations run; stats arrays need max_iter entries, of which the
 * first *n_done are written. Reads the change back to the host after every
 * iteration. MFG_ERR_NOT_CONVERGED (after the loop) if some PCG solve hit
 * pcg_maxit. */
int mfg_cp_solve_tol(mfg_plan_t plan, mfg_state_t* st, int max_iter, double cp_tol,
                     int pcg_maxit, int* n_done, mfg_stats_t* stats);

/* Reverse-mode gradient through n_iter Chambolle-Pock iterations started at
 * mfg_cp_init: given gy = dJ/dy_N (device primal vector) for a scalar J of the
 * final primal iterate, writes dJ/dm0 and dJ/dV (device, M values each).
 * The iteration (eq. pasosChamPock with the Section 5 schedule, the prox of
 * Section 3 through its implicit-function derivative, the projection eq. CC*)
 * is differentiated exactly; each reverse step needs one solve with the
 * symmetric matrix of eq. largeA, done by the same PCG (pcg_rtol, pcg_maxit;
 * use the forward run's values, so the recomputed forward steps reproduce it).
 * ckpts[k] must hold the state after k*every iterations (ckpts[0] is the
 * initial point, as after mfg_cp_init), n_ckpt*every >= n_iter; the
 * checkpoints are read, not modified. Allocates (every + 6) primal vectors of
 * workspace for the call. MFG_ERR_NOT_CONVERGED if some solve reached maxit
 * (outputs still written). */
int mfg_cp_adjoint(mfg_plan_t plan, const mfg_state_t* ckpts, int n_ckpt, int every, int n_iter,
                   const double* gy, double pcg_rtol, int pcg_maxit, double* g_m0,
                   double* g_V);

/* Value function of the discrete MFG system (Section 2, scheme MFG_T^2_h)
 * read off a Chambolle-Pock state: the multiplier lam of the reduced
 * constraint solves A lam = Cr xi (eq. largeA; PCG to pcg_rtol, at most
 * pcg_maxit iterations, from zero), and u^k = -lam_k for k < N_t, u^{N_t} =
 * g(x, m^{N_t}) (0 without a terminal cost). At a fixed point of the
 * iteration this u and the state's (m, w) satisfy the scheme: the HJB
 * equation (see mfg_hjb_residual) and w^k = m^{k+1} P_K(-[D_h u^k]).
 * u: device array of (N_t + 1) M values, [k][i][j]. MFG_ERR_NOT_CONVERGED if
 * the solve reached pcg_maxit (u still written). */
int mfg_value_function(mfg_plan_t plan, const mfg_state_t* st, double pcg_rtol, int pcg_maxit,
                       double* u);

/* Residual of the HJB equation of (MFG_T^2_h) per cell, for k = 0..N_t-1:
 *   R^k = (u^k - u^{k+1})/dt + nu K u^k + |P_K(-[D_h u^k])|^2 / 2 - f(x, m^{k+1}),
 * K the negative discrete Laplacian, -[D_h u] the four one-sided differences of
 * Section 2 (zero across a Neumann boundary), f the coupling. It vanishes where
 * m > 0 and is <= 0 where m = 0 at a solution. y: primal vector (its m block is
 * used), u: (N_t + 1) M values as from mfg_value_function, R: n-vector. */
int mfg_hjb_residual(mfg_plan_t plan, const double* y, const double* u, double* R);

/* Autotune the plan's launch shapes (how the preconditioner passes split
 * work among thread blocks: rows per block of the row transforms, column
 * pairs per block of the column solves, column blocks per wave and the
 * persistent form of the time GEMM), timing candidates with HIP events on the
 * plan's stream; results are unchanged up to the summation order of the dot
 * products. effort 1: use the choice cached for this (d, grid, N_t, bc,
 * precision, l, GPU architecture) if any, else measure; 2: measure again.
 * The choice is cached for the process and applied to later plans of the
 * same key; if the environment variable MFG_TUNE_CACHE names a file it is
 * read from and appended to. Overwrites the plan's workspace; synchronises. */
int mfg_autotune(mfg_plan_t plan, int effort);

/* ---- Batches of independent problems -------------------------------------
 * Many problems solved together (for instance a parameter sweep over nu, V or
 * m0, or independent problems of different sizes): every phase of a
 * Chambolle-Pock step runs as ONE kernel launch over all instances, and the
 * step, up to a fixed number of PCG iterations, is recorded once into a HIP
 * graph and replayed. Each instance performs exactly the arithmetic of
 * mfg_cp_solve on its own plan with the same arguments, so its iterates are
 * bitwise identical to a single-plan run. */
typedef struct mfg_batch_s* mfg_batch_t;

/* Build a batch of count >= 1 plans. pbs[i], V[i], m0[i] are as for mfg_plan
 * (V and m0 arrays are host arrays of device pointers). Requirements: d = 2,
 * q' = 2 (MFG_ERR_UNSUPPORTED otherwise) and one precision shared by all
 * instances (MFG_ERR_INVALID_ARG otherwise); any N_t (above 128 the MIXED
 * precisions take the streaming time transform, which MFG_TUNE lp_stream=0
 * would switch off: MFG_ERR_UNSUPPORTED then). The instances' plans use `stream`; batched
 * solves run on an internal stream ordered after and before `stream` with
 * events. */
int mfg_plan_batch(const mfg_problem_t* pbs, const double* const* V, const double* const* m0,
                   int count, hipStream_t stream, mfg_batch_t* out);

/* Plan of instance i (owned by the batch: do not destroy). It accepts every
 * single-plan call (mfg_cp_init, mfg_cp_solve, mfg_cp_adjoint, ...). */
int mfg_batch_plan(mfg_batch_t batch, int i, mfg_plan_t* out);

/* mfg_autotune for every instance (the persistent time GEMM excluded), then
 * rebuild the batched launches. */
int mfg_batch_autotune(mfg_batch_t batch, int effort);

/* Release the batch and its plans. */
int mfg_batch_destroy(mfg_batch_t batch);

/* n_iter Chambolle-Pock iterations on every instance (states: host array of
 * count states, each as for mfg_cp_solve). use_graph != 0 replays a recorded
 * HIP graph for each step after the first one of the batch's life; 0 issues
 * the same launches eagerly. pcg_iters (host, may be NULL): n_iter * count
 * entries, [iteration][instance]. Returns MFG_ERR_NOT_CONVERGED (after all
 * iterations) if some solve reached pcg_maxit. On any other error every
 * state's vectors are unspecified and its iter is set to -1. */
int mfg_batch_cp_solve(mfg_batch_t batch, mfg_state_t* states, int n_iter, double pcg_rtol,
                       int pcg_maxit, int use_graph, int* pcg_iters);

/* Per-kernel timing: enable != 0 starts recording a HIP event pair on the
 * plan's stream around every kernel launch of the plan (totals reset); 0
 * stops. Recording adds host work per launch but does not change what the
 * kernels do. */
int mfg_profile(mfg_plan_t plan, int enable);

/* Write the recorded per-kernel totals as a JSON object
 * {"kernel": {"calls": n, "total_ms": t}, ...} into buf (len bytes, host
 * memory); synchronises the plan's stream. MFG_ERR_INVALID_ARG if buf is too
 * small. */
int mfg_profile_report(mfg_plan_t plan, char* buf, int len);

/* ---- Without device allocation ------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * mfg_pcg_noalloc solves A u = b as mfg_pcg does (same kernels, same stopping
 * rule; the tables are computed on the device, so results agree with mfg_pcg
 * to rounding), for the problem *pb, with no plan. It allocates nothing: the
 * preconditioner's tables, the PCG workspace (6 n-vectors) and the reduction
 * buffers live in a 64 MiB device array of the library that each GPU it runs
 * on holds until the process ends. Limits: N_t <= 128 and about 2^20 cells
 * (n = N_t N_x N_y), MFG_ERR_UNSUPPORTED beyond. b, u: device n-vectors (must
 * not alias); runs on `stream` (0: the null stream) of the current device and
 * synchronises it (iters, relres as for mfg_pcg). Every call on a GPU uses
 * that GPU's one array and overwrites what the previous call left there:
 * calls that overlap on one GPU (other threads, other streams) race and must
 * be serialised by the caller. */
int mfg_pcg_noalloc(const mfg_problem_t* pb, const double* b, double* u, double rtol, int maxit,
                    hipStream_t stream, int* iters, double* relres);

/* Human-readable description of the last error on this thread. */
const char* mfg_last_error(void);

/* Library version string. */
const char* mfg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MFG_H */
