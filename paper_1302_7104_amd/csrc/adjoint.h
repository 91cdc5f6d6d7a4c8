// Device helpers of the discrete adjoint shared by the adjoint kernels: the
// Jacobian of the equilibrium, the moment cotangent map and the derivatives of
// the MWB term (with the tie and kink conventions).
#pragma once

#include <type_traits>

#include "common.h"

namespace pclb {

// Jacobian of the equilibrium (Eq. feq) with respect to (rho, u_x, u_y, E)
// at one state, applied to cotangents one velocity at a time.
struct FeqJac {
  EqCoef c;
  double rho, ux, uy;
  double F[NK + 1], Fp[NK + 1];              // F_k(E) and dF_k/dE
  double A0u, A1u, A2u;                      // dA_n / d(u^2)
  double A0E, A1E, A2E, A3E, A4E;            // dA_n / dE
};

PCLB_HD inline void feq_jac_setup(const Tables& T, double rho, double ux, double uy, double E,
                                     FeqJac& J) {
  eq_setup(T, rho, ux, uy, E, J.c);
  J.rho = rho;
  J.ux = ux;
  J.uy = uy;
  J.F[1] = weight_k<0>(E); J.F[2] = weight_k<1>(E); J.F[3] = weight_k<2>(E); J.F[4] = weight_k<3>(E);
  J.Fp[1] = weight_k_prime<0>(E); J.Fp[2] = weight_k_prime<1>(E);
  J.Fp[3] = weight_k_prime<2>(E); J.Fp[4] = weight_k_prime<3>(E);
  J.F[0] = 1.0 - 8.0 * (((J.F[1] + J.F[2]) + J.F[3]) + J.F[4]);
  J.Fp[0] = -8.0 * (((J.Fp[1] + J.Fp[2]) + J.Fp[3]) + J.Fp[4]);
  const double iE = 1.0 / E, iE2 = iE * iE, iE3 = iE2 * iE;
  const double a = 0.5 * (ux * ux + uy * uy) * iE, g = 1.0 - a;
  J.A0u = -0.5 * g * iE;
  J.A1u = -0.5 * iE2;
  J.A2u = -0.25 * iE3;
  J.A0E = a * g * iE;
  J.A1E = (2.0 * a - 1.0) * iE2;
  J.A2E = 0.5 * (a - 2.0 * g) * iE3;
  J.A3E = -0.5 * iE2 * iE2;
  J.A4E = -(1.0 / 6.0) * iE2 * iE3;
}

// G += l * d f^eq_q / d(rho, u_x, u_y, E) for velocity q = (k, d).
template <int Q>
PCLB_HD inline void feq_jac_accum(const FeqJac& J, double l, double G[4]) {
  constexpr int k = k_of(Q), d = d_of(Q);
  double w;
  if (Q == 0) w = 0.0;
  else w = speed(k) * (d < 4 ? J.c.p[d & 3] : -J.c.p[d & 3]);
  const EqCoef& c = J.c;
  const double P = c.A0 + w * (c.A1 + w * (c.A2 + w * (c.A3 + w * c.A4)));
  const double Pw = c.A1 + w * (2.0 * c.A2 + w * (3.0 * c.A3 + w * 4.0 * c.A4));
  const double Pu = J.A0u + w * (J.A1u + w * J.A2u);
  const double PE = J.A0E + w * (J.A1E + w * (J.A2E + w * (J.A3E + w * J.A4E)));
  const double rFk = J.rho * J.F[k];
  G[0] += l * J.F[k] * P;
  G[1] += l * rFk * (Pw * vx_q(Q) + Pu * 2.0 * J.ux);
  G[2] += l * rFk * (Pw * vy_q(Q) + Pu * 2.0 * J.uy);
  G[3] += l * J.rho * (J.Fp[k] * P + J.F[k] * PE);
}

// (G_rho, G_ux, G_uy, G_E) -> cotangents of M = (rho, j_x, j_y, eps) through
// u = j / rho, E = eps / rho - u^2 / 2.
PCLB_HD inline void to_moment_cotangent(double rho, double ux, double uy, double E,
                                           const double G[4], double gM[4]) {
  const double ir = 1.0 / rho;
  gM[0] = G[0] - (G[1] * ux + G[2] * uy) * ir + G[3] * (0.5 * (ux * ux + uy * uy) - E) * ir;
  gM[1] = (G[1] - G[3] * ux) * ir;
  gM[2] = (G[2] - G[3] * uy) * ir;
  gM[3] = G[3] * ir;
}

// Derivatives of T = |C| d1 + K h(d1, d2), d1 = c - u1, d2 = u1 - u2,
// h = (d1 - d2)|d1| / (|d1| + |d2|), with respect to (c, u1, u2).  T is not
// differentiable where d1 or d2 vanishes; a difference within `eps` times the
// stencil's magnitude counts as zero there, so that rounding noise does not
// pick the branch.  sgn(0) = 0; at d1 = d2 = 0, (dh/dd1, dh/dd2) = (1, 0).
template <class A>
struct MwbDT {
  A dc, du1, du2;
};
using MwbD = MwbDT<double>;

PCLB_HD inline double absv(double x) { return __builtin_fabs(x); }
PCLB_HD inline float absv(float x) { return __builtin_fabsf(x); }
PCLB_HD inline double recipv(double x) { return 1.0 / x; }
// the hardware reciprocal (1 ulp): the derivative of an FP32 state's step
// needs no more
PCLB_HD inline float recipv(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;   // host emulation of the device arithmetic (tests only)
#endif
}

// In the arithmetic type A: double for FP64 states, float for FP32 states
// (the tie threshold of FP32 states is far above float rounding).
template <class A>
PCLB_HD inline MwbDT<A> mwb_grad_t(A aC, A K, A c, A u1, A u2, A eps) {
  const A zero = 0, one = 1;
  A d1 = c - u1, d2 = u1 - u2;
  const A thr = eps * (absv(c) + absv(u1) + absv(u2));
  if (absv(d1) <= thr) d1 = zero;
  if (absv(d2) <= thr) d2 = zero;
  const A a1 = absv(d1), a2 = absv(d2), D = a1 + a2;
  A h1 = one, h2 = zero;
  if (D != zero) {
    const A s1 = d1 > zero ? one : (d1 < zero ? -one : zero);
    const A s2 = d2 > zero ? one : (d2 < zero ? -one : zero);
    const A iD = recipv(D), iD2 = iD * iD;
    h1 = a1 * iD + (d1 - d2) * s1 * a2 * iD2;
    h2 = -a1 * iD - (d1 - d2) * a1 * s2 * iD2;
  }
  MwbDT<A> r;
  r.dc = aC + K * h1;
  r.du1 = -aC - K * h1 + K * h2;
  r.du2 = -K * h2;
  return r;
}

PCLB_HD inline MwbD mwb_grad(double aC, double K, double c, double u1, double u2, double eps) {
  return mwb_grad_t<double>(aC, K, c, u1, u2, eps);
}

template <class R>
PCLB_HD inline double fetch_f(const R* __restrict__ f, const R* __restrict__ ghost, int q, int i,
                                 int j, int nr, int nth, size_t plane) {
  if (i < 0) return (double)ghost[ghost_index(0, -1 - i, q, j, nth)];
  if (i >= nr) return (double)ghost[ghost_index(1, i - nr, q, j, nth)];
  return (double)f[q * plane + (size_t)i * nth + j];
}

template <int Q, class Fn>
PCLB_HD inline void static_for_q(Fn&& fn) {
  if constexpr (Q < NQ) {
    fn(std::integral_constant<int, Q>{});
    static_for_q<Q + 1>(fn);
  }
}

}  // namespace pclb
