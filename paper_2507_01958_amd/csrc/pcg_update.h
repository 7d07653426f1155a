// The step length of the conjugate gradient update (x += alpha p, r -= alpha q)
// from the device-resident partial sums, shared by the update kernel and the
// fused update + forward preconditioner kernel so both take the same alpha.
#pragma once

#include "batch_args.h"
#include "device_util.h"

namespace mfg {

// alpha = r.z / p.q from the partials of both sites (breakdown, p.q not
// positive or not finite: alpha = 0 and S_BAD, which ends the solve at the next
// r.r check). Block 0 records p.q, alpha and rho = r.z for the next direction.
// r.z = 0 means r = 0 (a warm start at the solution): a zero step, not a
// breakdown; the next r.r test ends the solve. Every thread of the block must
// call it.
__device__ __forceinline__ double pcg_alpha(const UpdArgs& a, int bid) {
  double pq[1], rz[1];
  fold_partials<1>(a.rb, T_PQ, a.npq, pq);
  fold_partials<1>(a.rb, T_RZ, a.nrz, rz);
  const int bad = !finite_d(pq[0]) ? 2 : (!(pq[0] > 0.0) && rz[0] != 0.0 ? 1 : 0);
  const double alpha = (bad || rz[0] == 0.0) ? 0.0 : rz[0] / pq[0];
  if (bid == 0 && threadIdx.x == 0) {
    double* S = a.rb.scal;
    S[S_PQ] = pq[0];
    S[S_ALPHA] = alpha;
    S[S_RHO] = rz[0];
    if (bad) S[S_BAD] = (double)bad;
  }
  return alpha;
}

}  // namespace mfg
