// Discrete adjoint of the combined-scheme step (the method's Eq.
// combined_scheme differentiated by hand; the paper has no adjoint).
//
// lam_t(m) = e lam(m) + sum_a gM_a(m) phi_a(q)                (relaxation + f^eq)
//          - sum_{n : m in stencil_q(n)} lam_q(n) dT_q(n)/df_q(m)   (MWB, gather form)
//          + ghost-layer terms for the two rows next to each wall,
// with phi(q) = (1, v_qx, v_qy, v_q^2/2) and gM the cotangent of the four
// linear moments M = (rho, j_x, j_y, eps) of node m.
//
// Every array below is indexed with compile-time indices only, so that the
// kernels keep their working set in registers (no private scratch memory).
#include <type_traits>

#include "common.h"
#include "launch.h"

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

__device__ inline void feq_jac_setup(const Tables& T, double rho, double ux, double uy, double E,
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
__device__ inline void feq_jac_accum(const FeqJac& J, double l, double G[4]) {
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
__device__ inline void to_moment_cotangent(double rho, double ux, double uy, double E,
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
struct MwbD {
  double dc, du1, du2;
};
__device__ inline MwbD mwb_grad(double aC, double K, double c, double u1, double u2, double eps) {
  double d1 = c - u1, d2 = u1 - u2;
  const double thr = eps * (fabs(c) + fabs(u1) + fabs(u2));
  if (fabs(d1) <= thr) d1 = 0.0;
  if (fabs(d2) <= thr) d2 = 0.0;
  const double a1 = fabs(d1), a2 = fabs(d2), D = a1 + a2;
  double h1 = 1.0, h2 = 0.0;
  if (D != 0.0) {
    const double s1 = d1 > 0.0 ? 1.0 : (d1 < 0.0 ? -1.0 : 0.0);
    const double s2 = d2 > 0.0 ? 1.0 : (d2 < 0.0 ? -1.0 : 0.0);
    const double iD = 1.0 / D, iD2 = iD * iD;
    h1 = a1 * iD + (d1 - d2) * s1 * a2 * iD2;
    h2 = -a1 * iD - (d1 - d2) * a1 * s2 * iD2;
  }
  MwbD r;
  r.dc = aC + K * h1;
  r.du1 = -aC - K * h1 + K * h2;
  r.du2 = -K * h2;
  return r;
}

// Tie threshold per storage precision: a few hundred ulps of the stored values
// (rounding differences of f^eq scale with sum |f| / rho, up to about 16 here).
template <class R> struct TieEps;
template <> struct TieEps<double> { static constexpr double value = 1e-13; };
template <> struct TieEps<float> { static constexpr double value = 1e-5; };

template <class R>
__device__ inline double fetch_f(const R* __restrict__ f, const R* __restrict__ ghost, int q, int i,
                                 int j, int nr, int nth, size_t plane) {
  if (i < 0) return (double)ghost[ghost_index(0, -1 - i, q, j, nth)];
  if (i >= nr) return (double)ghost[ghost_index(1, i - nr, q, j, nth)];
  return (double)f[q * plane + (size_t)i * nth + j];
}

template <int Q, class Fn>
__device__ inline void static_for_q(Fn&& fn) {
  if constexpr (Q < NQ) {
    fn(std::integral_constant<int, Q>{});
    static_for_q<Q + 1>(fn);
  }
}

// ---------------------------------------------------------------------------
// Ghost adjoint: cotangents of the ghost distributions from the MWB terms of
// the two real rows next to each wall, pulled back through f^eq, the boundary
// kind and the linear extrapolation to the moments of those two rows.
// gm[((side * 2 + s) * 4 + a) * nth + j], s = 0 the row next to the wall.
template <class R>
__global__ void __launch_bounds__(128) ghost_adjoint_kernel(Tables T, BCdev bc, const R* __restrict__ f,
                                                            const R* __restrict__ lam,
                                                            const R* __restrict__ ghost,
                                                            double* __restrict__ gm) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int side = blockIdx.y;
  if (j >= T.nth) return;
  const int nr = T.nr, nth = T.nth;
  const size_t plane = (size_t)nr * nth;
  const int i0 = side == 0 ? 0 : nr - 1, i1 = side == 0 ? 1 : nr - 2;
  const int gsgn = side == 0 ? -1 : 1;     // direction from the wall row into the ghosts
  const double ct = T.cth[j], st = T.sth[j];
  const int kind = bc.kind[side];
  constexpr double TE = TieEps<R>::value;
  // macroscopic state of the two real rows
  double m0[4], m1[4];
  {
    double fl[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) fl[q] = (double)f[q * plane + (size_t)i0 * nth + j];
    node_macros(fl, m0[0], m0[1], m0[2], m0[3]);
#pragma unroll
    for (int q = 0; q < NQ; ++q) fl[q] = (double)f[q * plane + (size_t)i1 * nth + j];
    node_macros(fl, m1[0], m1[1], m1[2], m1[3]);
  }
  // ghost states exactly as the forward ghost kernel builds them
  double gs0[4], gs1[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gs0[a] = 2.0 * m0[a] - m1[a];
    gs1[a] = 2.0 * gs0[a] - m0[a];
  }
  if (kind == 0) {
    const double w0 = bc.p[side][0] * bc.rg[side][0], w1 = bc.p[side][0] * bc.rg[side][1];
    gs0[1] = -w0 * st; gs0[2] = w0 * ct;
    gs1[1] = -w1 * st; gs1[2] = w1 * ct;
  }
  double Gm0[4] = {0, 0, 0, 0}, Gm1[4] = {0, 0, 0, 0};
  if (kind != 1) {                     // inflow ghosts do not depend on the state
    FeqJac J0, J1;
    feq_jac_setup(T, gs0[0], gs0[1], gs0[2], gs0[3], J0);
    feq_jac_setup(T, gs1[0], gs1[1], gs1[2], gs1[3], J1);
    double G0[4] = {0, 0, 0, 0}, G1[4] = {0, 0, 0, 0};
    static_for_q<1>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      const double vr = vx_q(q) * ct + vy_q(q) * st;
      const bool upwind_is_ghost = side == 0 ? (vr >= 0.0) : (vr < 0.0);
      if (upwind_is_ghost) {
        const double aC = fabs(vr * T.dt_dr), K = aC * (1.0 - aC);
        const double fw = fetch_f(f, ghost, q, i0, j, nr, nth, plane);
        const double f1 = fetch_f(f, ghost, q, i1, j, nr, nth, plane);
        const double g0 = fetch_f(f, ghost, q, i0 + gsgn, j, nr, nth, plane);
        const double g1 = fetch_f(f, ghost, q, i0 + 2 * gsgn, j, nr, nth, plane);
        const double lw = (double)lam[q * plane + (size_t)i0 * nth + j];
        const double l1 = (double)lam[q * plane + (size_t)i1 * nth + j];
        const MwbD a = mwb_grad(aC, K, fw, g0, g1, TE);   // wall row: u1 = ghost 0, u2 = ghost 1
        const MwbD b = mwb_grad(aC, K, f1, fw, g0, TE);   // next row: u2 = ghost 0
        feq_jac_accum<q>(J0, -lw * a.du1 - l1 * b.du2, G0);
        feq_jac_accum<q>(J1, -lw * a.du2, G1);
      }
    });
    // ghost 0 = 2 m0 - m1, ghost 1 = 3 m0 - 2 m1 for the extrapolated components
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const bool extrap = (a == 0 || a == 3) || kind == 2;
      if (extrap) {
        Gm0[a] = 2.0 * G0[a] + 3.0 * G1[a];
        Gm1[a] = -G0[a] - 2.0 * G1[a];
      }
    }
  }
  double gM0[4], gM1[4];
  to_moment_cotangent(m0[0], m0[1], m0[2], m0[3], Gm0, gM0);
  to_moment_cotangent(m1[0], m1[1], m1[2], m1[3], Gm1, gM1);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gm[((size_t)(side * 2 + 0) * 4 + a) * nth + j] = gM0[a];
    gm[((size_t)(side * 2 + 1) * 4 + a) * nth + j] = gM1[a];
  }
}

// ---------------------------------------------------------------------------
// Node adjoint: one thread per node m, gather over every output whose stencil
// holds m.
template <class R>
__global__ void __launch_bounds__(128) adjoint_node_kernel(Tables T, const R* __restrict__ f,
                                                           const R* __restrict__ lam,
                                                           const R* __restrict__ ghost,
                                                           const double* __restrict__ gm,
                                                           R* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= T.nth) return;
  const int nr = T.nr, nth = T.nth;
  const size_t plane = (size_t)nr * nth;
  const size_t c0 = (size_t)i * nth + j;
  const double e = T.e;
  constexpr double TE = TieEps<R>::value;
  // moment cotangent of this node from the relaxation's f^eq
  double gM[4];
  {
    double fl[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) fl[q] = (double)f[q * plane + c0];
    double rho, ux, uy, E;
    node_macros(fl, rho, ux, uy, E);
    FeqJac J;
    feq_jac_setup(T, rho, ux, uy, E, J);
    double G[4] = {0, 0, 0, 0};
    static_for_q<0>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      feq_jac_accum<q>(J, (1.0 - e) * (double)lam[q * plane + c0], G);
    });
    to_moment_cotangent(rho, ux, uy, E, G, gM);
  }
  if (i <= 1) {
#pragma unroll
    for (int a = 0; a < 4; ++a) gM[a] += gm[((size_t)i * 4 + a) * nth + j];
  }
  if (i >= nr - 2) {
    const int s = nr - 1 - i;
#pragma unroll
    for (int a = 0; a < 4; ++a) gM[a] += gm[((size_t)(2 + s) * 4 + a) * nth + j];
  }
  int jj[5];
  double cs[5], sn[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    int t = j + s - 2;
    t = t < 0 ? t + nth : (t >= nth ? t - nth : t);
    jj[s] = t;
    cs[s] = T.cth[t];
    sn[s] = T.sth[t];
  }
  const double sth_row = T.dt_dth * T.rinv[i];
  out[c0] = (R)(e * (double)lam[c0] + gM[0]);      // rest velocity: no convection
#pragma unroll 1
  for (int q = 1; q < NQ; ++q) {
    const int k = k_of(q), d = d_of(q);
    const double vx = speed(k) * cos_d(d), vy = speed(k) * sin_d(d);
    const double lq = (double)lam[q * plane + c0];
    double acc = e * lq + gM[0] + gM[1] * vx + gM[2] * vy + gM[3] * 0.5 * speed(k) * speed(k);
    // radial gather (the upwind side is fixed along the ray)
    {
      const double vr = vx * cs[2] + vy * sn[2];
      const double aC = fabs(vr * T.dt_dr), K = aC * (1.0 - aC);
      const bool back = vr >= 0.0;
      const double r0 = fetch_f(f, ghost, q, i - 2, j, nr, nth, plane);
      const double r1 = fetch_f(f, ghost, q, i - 1, j, nr, nth, plane);
      const double r2 = fetch_f(f, ghost, q, i, j, nr, nth, plane);
      const double r3 = fetch_f(f, ghost, q, i + 1, j, nr, nth, plane);
      const double r4 = fetch_f(f, ghost, q, i + 2, j, nr, nth, plane);
      // m as centre
      acc -= lq * mwb_grad(aC, K, r2, back ? r1 : r3, back ? r0 : r4, TE).dc;
      // m as first upwind neighbour of n1 = i + 1 (backward) or i - 1 (forward)
      const int n1 = back ? i + 1 : i - 1;
      if (n1 >= 0 && n1 < nr) {
        const MwbD g = back ? mwb_grad(aC, K, r3, r2, r1, TE) : mwb_grad(aC, K, r1, r2, r3, TE);
        acc -= (double)lam[q * plane + (size_t)n1 * nth + j] * g.du1;
      }
      // m as second upwind neighbour of n2 = i + 2 (backward) or i - 2 (forward)
      const int n2 = back ? i + 2 : i - 2;
      if (n2 >= 0 && n2 < nr) {
        const MwbD g = back ? mwb_grad(aC, K, r4, r3, r2, TE) : mwb_grad(aC, K, r0, r1, r2, TE);
        acc -= (double)lam[q * plane + (size_t)n2 * nth + j] * g.du2;
      }
    }
    // azimuthal gather: output n = j + s - 2 with its own upwind side
    {
      const R* fp = f + q * plane + (size_t)i * nth;
      const R* lp = lam + q * plane + (size_t)i * nth;
      const double t0 = fp[jj[0]], t1 = fp[jj[1]], t2 = fp[jj[2]], t3 = fp[jj[3]], t4 = fp[jj[4]];
      double vt, aC, K;
      // s = 0: n = j - 2 uses m only when its upwind side is forward (m = u2)
      vt = -vx * sn[0] + vy * cs[0];
      if (vt < 0.0) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= (double)lp[jj[0]] * mwb_grad(aC, K, t0, t1, t2, TE).du2;
      }
      // s = 1: n = j - 1, forward (m = u1)
      vt = -vx * sn[1] + vy * cs[1];
      if (vt < 0.0) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= (double)lp[jj[1]] * mwb_grad(aC, K, t1, t2, t3, TE).du1;
      }
      // s = 2: n = m (m is the centre)
      vt = -vx * sn[2] + vy * cs[2];
      aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
      acc -= lq * (vt >= 0.0 ? mwb_grad(aC, K, t2, t1, t0, TE) : mwb_grad(aC, K, t2, t3, t4, TE)).dc;
      // s = 3: n = j + 1, backward (m = u1)
      vt = -vx * sn[3] + vy * cs[3];
      if (vt >= 0.0) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= (double)lp[jj[3]] * mwb_grad(aC, K, t3, t2, t1, TE).du1;
      }
      // s = 4: n = j + 2, backward (m = u2)
      vt = -vx * sn[4] + vy * cs[4];
      if (vt >= 0.0) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= (double)lp[jj[4]] * mwb_grad(aC, K, t4, t3, t2, TE).du2;
      }
    }
    out[q * plane + c0] = (R)acc;
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the initial equilibrium: dJ/d(rho, u_r, u_theta, T) per node.
template <class R>
__global__ void __launch_bounds__(128) adjoint_init_kernel(Tables T, const R* __restrict__ lam,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ ur,
                                                           const double* __restrict__ ut,
                                                           const double* __restrict__ Tt,
                                                           double* d_rho, double* d_ur,
                                                           double* d_ut, double* d_T) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const size_t c0 = (size_t)i * T.nth + j;
  const double ct = T.cth[j], st = T.sth[j];
  const double a = ur[c0], b = ut[c0];
  const double ux = a * ct - b * st, uy = a * st + b * ct;
  FeqJac J;
  feq_jac_setup(T, rho[c0], ux, uy, Tt[c0], J);
  double G[4] = {0, 0, 0, 0};
  static_for_q<0>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    feq_jac_accum<q>(J, (double)lam[q * plane + c0], G);
  });
  d_rho[c0] = G[0];
  d_ur[c0] = G[1] * ct + G[2] * st;
  d_ut[c0] = -G[1] * st + G[2] * ct;
  d_T[c0] = G[3];
}

template <class R>
hipError_t launch_adjoint(const Tables& T, const BCdev& bc, const void* f, const void* lam,
                          void* lam_out, void* ghost, void* /*unused*/, double* gm, hipStream_t s) {
  hipError_t e = launch_ghost<R>(T, bc, f, ghost, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ghost_adjoint_kernel<R>, dim3((T.nth + 127) / 128, 2), dim3(128), 0, s, T, bc,
                     (const R*)f, (const R*)lam, (const R*)ghost, gm);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_node_kernel<R>, dim3((T.nth + 127) / 128, T.nr), dim3(128), 0, s, T,
                     (const R*)f, (const R*)lam, (const R*)ghost, (const double*)gm, (R*)lam_out);
  return hipGetLastError();
}

template <class R>
hipError_t launch_adjoint_init(const Tables& T, const void* lam, const double* rho,
                               const double* ur, const double* ut, const double* Tt, double* d_rho,
                               double* d_ur, double* d_ut, double* d_T, hipStream_t s) {
  hipLaunchKernelGGL(adjoint_init_kernel<R>, dim3((T.nth + 127) / 128, T.nr), dim3(128), 0, s, T,
                     (const R*)lam, rho, ur, ut, Tt, d_rho, d_ur, d_ut, d_T);
  return hipGetLastError();
}

template hipError_t launch_adjoint<float>(const Tables&, const BCdev&, const void*, const void*, void*,
                                          void*, void*, double*, hipStream_t);
template hipError_t launch_adjoint<double>(const Tables&, const BCdev&, const void*, const void*, void*,
                                           void*, void*, double*, hipStream_t);
template hipError_t launch_adjoint_init<float>(const Tables&, const void*, const double*, const double*,
                                               const double*, const double*, double*, double*, double*,
                                               double*, hipStream_t);
template hipError_t launch_adjoint_init<double>(const Tables&, const void*, const double*, const double*,
                                                const double*, const double*, double*, double*, double*,
                                                double*, hipStream_t);

}  // namespace pclb
