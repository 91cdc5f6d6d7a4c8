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

#include "adjoint.h"
#include "common.h"
#include "launch.h"

namespace pclb {

// ---------------------------------------------------------------------------
// Ghost adjoint: cotangents of the ghost distributions from the MWB terms of
// the two real rows next to each wall, pulled back through f^eq, the boundary
// kind and the linear extrapolation to the moments of those two rows.
// gm[((side * 2 + s) * 4 + a) * nth + j], s = 0 the row next to the wall.
template <class R>
__global__ void __launch_bounds__(128) ghost_adjoint_kernel(Tables T, BCdev bc, const R* __restrict__ f,
                                                            const R* __restrict__ lam,
                                                            const R* __restrict__ ghost,
                                                            double tie, double* __restrict__ gm) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int side = blockIdx.y;
  if (j >= T.nth) return;
  const int nr = T.nr, nth = T.nth;
  const size_t plane = (size_t)nr * nth;
  const int i0 = side == 0 ? 0 : nr - 1, i1 = side == 0 ? 1 : nr - 2;
  const int gsgn = side == 0 ? -1 : 1;     // direction from the wall row into the ghosts
  const double ct = T.cth[j], st = T.sth[j];
  const int kind = bc.kind[side];
  const double TE = tie;
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
                                                           double tie, R* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= T.nth) return;
  const int nr = T.nr, nth = T.nth;
  const size_t plane = (size_t)nr * nth;
  const size_t c0 = (size_t)i * nth + j;
  const double e = T.e;
  // MWB derivatives in the state's precision
  using A = R;
  const A TEa = (A)tie;
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
      acc -= lq * (double)mwb_grad_t<A>((A)aC, (A)K, (A)r2, (A)(back ? r1 : r3), (A)(back ? r0 : r4), TEa).dc;
      // m as first upwind neighbour of n1 = i + 1 (backward) or i - 1 (forward)
      const int n1 = back ? i + 1 : i - 1;
      if (n1 >= 0 && n1 < nr) {
        const MwbDT<A> g = back ? mwb_grad_t<A>((A)aC, (A)K, (A)r3, (A)r2, (A)r1, TEa)
                                : mwb_grad_t<A>((A)aC, (A)K, (A)r1, (A)r2, (A)r3, TEa);
        acc -= (double)lam[q * plane + (size_t)n1 * nth + j] * (double)g.du1;
      }
      // m as second upwind neighbour of n2 = i + 2 (backward) or i - 2 (forward)
      const int n2 = back ? i + 2 : i - 2;
      if (n2 >= 0 && n2 < nr) {
        const MwbDT<A> g = back ? mwb_grad_t<A>((A)aC, (A)K, (A)r4, (A)r3, (A)r2, TEa)
                                : mwb_grad_t<A>((A)aC, (A)K, (A)r0, (A)r1, (A)r2, TEa);
        acc -= (double)lam[q * plane + (size_t)n2 * nth + j] * (double)g.du2;
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
        acc -= (double)lp[jj[0]] * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t0, (A)t1, (A)t2, TEa).du2;
      }
      // s = 1: n = j - 1, forward (m = u1)
      vt = -vx * sn[1] + vy * cs[1];
      if (vt < 0.0) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= (double)lp[jj[1]] * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t1, (A)t2, (A)t3, TEa).du1;
      }
      // s = 2: n = m (m is the centre)
      vt = -vx * sn[2] + vy * cs[2];
      aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
      acc -= lq * (double)(vt >= 0.0 ? mwb_grad_t<A>((A)aC, (A)K, (A)t2, (A)t1, (A)t0, TEa)
                                      : mwb_grad_t<A>((A)aC, (A)K, (A)t2, (A)t3, (A)t4, TEa)).dc;
      // s = 3: n = j + 1, backward (m = u1)
      vt = -vx * sn[3] + vy * cs[3];
      if (vt >= 0.0) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= (double)lp[jj[3]] * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t3, (A)t2, (A)t1, TEa).du1;
      }
      // s = 4: n = j + 2, backward (m = u2)
      vt = -vx * sn[4] + vy * cs[4];
      if (vt >= 0.0) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= (double)lp[jj[4]] * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t4, (A)t3, (A)t2, TEa).du2;
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
                          void* lam_out, void* ghost, double* gm, double tie, hipStream_t s) {
  hipError_t e = launch_ghost<R>(T, bc, f, ghost, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ghost_adjoint_kernel<R>, dim3((T.nth + 127) / 128, 2), dim3(128), 0, s, T, bc,
                     (const R*)f, (const R*)lam, (const R*)ghost, tie, gm);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_node_kernel<R>, dim3((T.nth + 127) / 128, T.nr), dim3(128), 0, s, T,
                     (const R*)f, (const R*)lam, (const R*)ghost, (const double*)gm, tie, (R*)lam_out);
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
                                          void*, double*, double, hipStream_t);
template hipError_t launch_adjoint<double>(const Tables&, const BCdev&, const void*, const void*, void*,
                                           void*, double*, double, hipStream_t);
template hipError_t launch_adjoint_init<float>(const Tables&, const void*, const double*, const double*,
                                               const double*, const double*, double*, double*, double*,
                                               double*, hipStream_t);
template hipError_t launch_adjoint_init<double>(const Tables&, const void*, const double*, const double*,
                                                const double*, const double*, double*, double*, double*,
                                                double*, hipStream_t);

}  // namespace pclb
