// Host-side plan object behind mfg_plan_t.
#pragma once

#include <string>
#include <vector>

#include "mfg_internal.h"

struct mfg_plan_s;

namespace mfg {

struct Plan {
  mfg_problem_t pb{};
  Geom g{};
  int precision = MFG_FP64;
  int l = 1;
  double gamma = 0.0;
  hipStream_t stream = nullptr;
  int device = 0;

  // problem data (plan-owned copies)
  double* V = nullptr;   // M
  double* m0 = nullptr;  // M

  // time transform (Algorithm 1): Vt[t][k] = V[k][t] (V is symmetric)
  double* Vt64 = nullptr;
  float* Vt32 = nullptr;
  _Float16* Vt16 = nullptr;
  unsigned short* Vtbf = nullptr;
  double* lam_t = nullptr;  // N_t eigenvalues (eq. eigs)

  // spatial transforms (Algorithm 2)
  Axis ax0{}, ax1{};

  // workspace (n-vectors)
  double *r = nullptr, *z = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr;
  double *tmp = nullptr;  // preconditioner intermediate (float64 or float32 view)
  double *b = nullptr, *u = nullptr;
  double *xi_tmp = nullptr;
  RedBuf red{};
  double* host_scal = nullptr;  // pinned mirror of red.scal

  std::vector<void*> dev_allocs;
  std::vector<void*> host_allocs;
};

}  // namespace mfg

struct mfg_plan_s {
  mfg::Plan P;
};
