// Per-cell proximal step of Section 3 for a coupling that is a polynomial in m
// (Section 2.1; the two problems of Section 5), first for q' = 2 (the
// Hamiltonian |p|^2/2), then for a general exponent q':
//   f(x, m) = c2 m^2 + c1 m + V(x),   F = c2 m^3/3 + c1 m^2/2 + V m,
// with a terminal cost g = (m - mbar)/beta folded into the last time slice's
// c1 (+1/(beta dt)) and V (-mbar/(beta dt)) by the caller.
//
// prox(mbar, wbar) minimises |w|^2/(2m) + F(m) + (|m - mbar|^2 + |w - wbar|^2)/(2 tau)
// over m >= 0, w in the cone K. For fixed m the flux is w = m/(m + tau) w~ with
// w~ = P_K(wbar); with a = |w~|^2 the scalar problem has the increasing
// derivative h'(m) = -a/(2(m+tau)^2) + c2 m^2 + (c1 + 1/tau) m + V - mbar/tau.
// m = 0 when h'(0) >= 0, i.e. 2 tau^2 V - 2 tau mbar - a >= 0. Otherwise:
// * c2 = 0: h' is concave; Newton from the root for a = 0,
//   max(0, (mbar - tau V)/(1 + tau c1)), rises monotonically: iterate while an
//   update still increases m (at most 64 updates).
// * c2 > 0: the root lies between lo, the root of Q(m) = c2 m^2 + (c1 + 1/tau) m
//   + V - mbar/tau, and hi, the root of Q - a/(2 tau^2) (closed forms); Newton
//   from lo keeps that bracket (each iterate replaces lo or hi by the sign of
//   h'), takes the midpoint when a step leaves it, and stops when the iterate
//   no longer moves or the bracket cannot be split (at most 100 steps).
//
// General exponent: with the Hamiltonian |p|^q'/q' (eq. power_hamiltonian) the
// flux cost is |w|^q/(q m^(q-1)), q = q'/(q' - 1). For fixed m the flux is
// w = m s w~/a with a = |w~| and s the root of phi(s) = tau s^(q-1) + m s - a
// in (0, min(a/m, s_max)], s_max = (a/tau)^(1/(q-1)), and
// h'(m) = -s^q/q' + c2 m^2 + c1 m + V - (mbar - m)/tau is increasing, with
// h''(m) = (q-1) s^q/(tau (q-1) s^(q-2) + m) + 2 c2 m + c1 + 1/tau. m = 0 when
// h'(0) = -s_max^q/q' + V - mbar/tau >= 0. Otherwise the root lies between the
// roots of Q (lo) and of Q - s_max^q/q' (hi); Newton's method on h' keeps that
// bracket (midpoint when a step leaves it), each h'(m) taking s from Newton's
// method on phi in its own bracket, warm-started from the previous s. Both stop
// when the iterate no longer moves or the bracket cannot be split (at most 100
// outer and 100 inner steps). Solving in m keeps m accurate where it is small
// against a/s.
#pragma once

#include <hip/hip_runtime.h>

namespace mfg {

// Non-negative root of c2 m^2 + B m + C (c2 > 0, B > 0), 0 when C >= 0,
// without cancellation.
__device__ __forceinline__ double quad_root(double c2, double B, double C) {
  if (!(C < 0.0)) return 0.0;
  return -2.0 * C / (B + sqrt(B * B - 4.0 * c2 * C));
}

// h'(0) >= 0: the minimiser is m = 0, w = 0.
__device__ __forceinline__ bool prox_inactive(double mbar, double a, double V, double tau) {
  return 2.0 * tau * tau * V - 2.0 * tau * mbar - a >= 0.0;
}

// Root m of h' on the active branch (h'(0) < 0) for a = |w~|^2.
__device__ __forceinline__ double prox_root_active(double mbar, double a, double V, double tau,
                                                   double c1, double c2) {
  const double B = c1 + 1.0 / tau;
  if (c2 == 0.0) {
    double m = fmax(0.0, (mbar - tau * V) / (1.0 + tau * c1));
    for (int it = 0; it < 64; ++it) {
      const double s = m + tau;
      const double hp = -a / (2.0 * s * s) + B * m + V - mbar / tau;
      const double hpp = a / (s * s * s) + B;
      const double mn = m - hp / hpp;
      if (!(mn > m)) break;
      m = mn;
    }
    return m;
  }
  const double C = V - mbar / tau;
  double lo = quad_root(c2, B, C);
  double hi = quad_root(c2, B, C - a / (2.0 * tau * tau));
  double m = lo;
  for (int it = 0; it < 100; ++it) {
    const double s = m + tau;
    const double hp = -a / (2.0 * s * s) + (c2 * m + B) * m + C;
    const double hpp = a / (s * s * s) + 2.0 * c2 * m + B;
    if (hp < 0.0) lo = m;
    else if (hp > 0.0) hi = m;
    else break;  // a root, or a non-finite value
    double mn = m - hp / hpp;
    if (!(mn > lo && mn < hi)) {
      mn = 0.5 * (lo + hi);
      if (!(mn > lo && mn < hi)) break;
    }
    if (mn == m) break;
    m = mn;
  }
  return m;
}

// Root m of the scalar problem for a = |w~|^2 (0 on the inactive branch).
__device__ __forceinline__ double prox_root(double mbar, double a, double V, double tau,
                                            double c1, double c2) {
  if (prox_inactive(mbar, a, V, tau)) return 0.0;
  return prox_root_active(mbar, a, V, tau, c1, c2);
}

// General exponent q != 2 of b-hat (qp = q' its conjugate): the prox for the
// cone projection w~ of the flux with a = |w~| > 0. Returns m (0 on the
// inactive branch) and the factor f with w = f w~.
__device__ __forceinline__ double prox_general(double mbar, double a, double V, double tau,
                                               double c1, double c2, double q, double qp,
                                               double* f) {
  const double B = c1 + 1.0 / tau, C = V - mbar / tau;
  const double smax = exp(log(a / tau) / (q - 1.0));
  const double hmax = exp(q * log(smax)) / qp;
  *f = 0.0;
  if (-hmax + C >= 0.0) return 0.0;
  auto root_Q = [&](double Cc) { return c2 > 0.0 ? quad_root(c2, B, Cc) : fmax(0.0, -Cc / B); };
  double s = smax;
  // s(m): root of tau s^(q-1) + m s - a, warm-started from the previous s
  auto s_of = [&](double m) {
    const double cap = m > 0.0 ? fmin(a / m, smax) : smax;
    double lo = 0.0, hi = cap;
    double x = fmin(s, cap);
    for (int it = 0; it < 100; ++it) {
      const double xq2 = exp((q - 2.0) * log(x));   // x^(q-2)
      const double ph = tau * xq2 * x + m * x - a;
      if (ph < 0.0) lo = x;
      else if (ph > 0.0) hi = x;
      else break;
      double xn = x - ph / (tau * (q - 1.0) * xq2 + m);
      if (!(xn > lo && xn < hi)) {
        xn = 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) break;
      }
      if (xn == x) break;
      x = xn;
    }
    s = x;
    return x;
  };
  double lo = root_Q(C), hi = root_Q(C - hmax);
  double m = lo;
  for (int it = 0; it < 100; ++it) {
    const double sv = s_of(m);
    const double sq2 = exp((q - 2.0) * log(sv));   // s^(q-2)
    const double sq = sq2 * sv * sv;
    const double hp = -sq / qp + (c2 * m + B) * m + C;
    if (hp < 0.0) lo = m;
    else if (hp > 0.0) hi = m;
    else break;  // a root, or a non-finite value
    const double hpp = (q - 1.0) * sq / (tau * (q - 1.0) * sq2 + m) + 2.0 * c2 * m + B;
    double mn = m - hp / hpp;
    if (!(mn > lo && mn < hi)) {
      mn = 0.5 * (lo + hi);
      if (!(mn > lo && mn < hi)) break;
    }
    if (mn == m) break;
    m = mn;
  }
  const double sv = s_of(m);
  *f = m * sv / a;
  return m;
}

// Full cell prox: projects w in place onto the cone, then scales it by
// m/(m + tau) (sets it to zero on the inactive branch); returns m. QG: a
// general exponent q of b-hat (qp = q'); otherwise q = 2 and the closed-form
// reduction above (q, qp unused). Separate instantiations keep the general
// path's registers out of the q = 2 kernels.
template <int NC, bool QG = false>
__device__ __forceinline__ double prox_cell(double mbar, double* w, double V, double tau,
                                            double c1, double c2, double q = 2.0,
                                            double qp = 2.0) {
  double a = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double v = w[c];
    v = (c & 1) ? fmin(v, 0.0) : fmax(v, 0.0);
    w[c] = v;
    a += v * v;
  }
  if constexpr (QG) {
    double f = 0.0, m;
    if (a > 0.0) {
      m = prox_general(mbar, sqrt(a), V, tau, c1, c2, q, qp, &f);
    } else {
      // w = 0: the non-negative root of c2 m^2 + (c1 + 1/tau) m + V - mbar/tau
      const double B = c1 + 1.0 / tau, C = V - mbar / tau;
      m = c2 > 0.0 ? quad_root(c2, B, C) : fmax(0.0, -C / B);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] *= f;
    return m;
  } else {
    (void)q;
    (void)qp;
  }
  if (prox_inactive(mbar, a, V, tau)) {
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = 0.0;
    return 0.0;
  }
  const double m = prox_root_active(mbar, a, V, tau, c1, c2);
  const double f = m / (m + tau);
#pragma unroll
  for (int c = 0; c < NC; ++c) w[c] *= f;
  return m;
}

}  // namespace mfg
