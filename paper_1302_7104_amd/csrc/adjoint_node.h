// Discrete adjoint of the combined-scheme step: the per-column ghost adjoint
// and the per-node adjoint (the method's Eq. combined_scheme differentiated by
// hand; the paper has no adjoint).  Shared by the adjoint kernels and by the
// host emulation of the device arithmetic that the CPU tests run.
//
// lam_t(m) = e lam(m) + sum_a gM_a(m) phi_a(q)                (relaxation + f^eq)
//          - sum_{n : m in stencil_q(n)} lam_q(n) dT_q(n)/df_q(m)   (MWB, gather form)
//          + ghost-layer terms for the two rows next to each wall,
// with phi(q) = (1, v_qx, v_qy, v_q^2/2) and gM the cotangent of the four
// linear moments M = (rho, j_x, j_y, eps) of node m.
//
// Every array below is indexed with compile-time indices only, so that the
// kernels keep their working set in registers (no private scratch memory).
#pragma once

#include "adjoint.h"

namespace pclb {

// ---------------------------------------------------------------------------
// Ghost adjoint of one column j of wall `side`: cotangents of the ghost
// distributions from the MWB terms of the two real rows next to the wall,
// pulled back through f^eq, the boundary kind and the linear extrapolation to
// the moments of those two rows.
// gm[((side * 2 + s) * 4 + a) * nth + j], s = 0 the row next to the wall.
template <class R>
PCLB_HD inline void ghost_adjoint_column(const Tables& T, const BCdev& bc, const R* __restrict__ f,
                                         const R* __restrict__ lam, const R* __restrict__ ghost,
                                         double tie, int side, int j, double* __restrict__ gm) {
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
    const unsigned rb = rback_bits(octant_of(j, nth, T.nf));
    static_for_q<1>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      const double vr = vx_q(q) * ct + vy_q(q) * st;
      const bool back = (rb >> d_of(q)) & 1u;
      const bool upwind_is_ghost = side == 0 ? back : !back;
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
// Node adjoint of node (i, j): gather over every output whose stencil holds
// the node.
// SECTOR: the grid is a sector (n_f < 8) whose ends rotate the direction
// index; without it the rotations are compiled out.
template <class R, bool SECTOR = true>
PCLB_HD inline void adjoint_node(const Tables& T, const R* __restrict__ f, const R* __restrict__ lam,
                                 const R* __restrict__ ghost, const double* __restrict__ gm,
                                 double tie, int i, int j, R* __restrict__ out) {
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
  // the five columns around j; across an end of a sector a column holds the
  // velocity whose direction index is rotated (Sec. II.C): rot[s] is the
  // rotation of this node's velocity index to the one read there
  int jj[5], rot[5];
  double cs[5], sn[5];
  const int s_lo = T.nf & 7, s_hi = (8 - T.nf) & 7;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    int t = j + s - 2;
    rot[s] = !SECTOR ? 0 : t < 0 ? s_lo : (t >= nth ? s_hi : 0);
    t = t < 0 ? t + nth : (t >= nth ? t - nth : t);
    jj[s] = t;
    cs[s] = T.cth[t];
    sn[s] = T.sth[t];
  }
  const double sth_row = T.dt_dth * T.rinv[i];
  // upwind sides of this column (radial) and of the five columns around it
  // (azimuthal), from their octants
  const unsigned rb = rback_bits(octant_of(j, nth, T.nf));
  unsigned tbs[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) tbs[s] = tback_bits(octant_of(jj[s], nth, T.nf));
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
      const bool back = (rb >> d) & 1u;
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
    // azimuthal gather: output n = j + s - 2 with its own upwind side.  Seen
    // from this column, n's velocity is qs[s] (q rotated where n lies across
    // an end of a sector) and the values around it are those of plane q
    // continued through the azimuthal ghosts, i.e. plane qs[s] at column jj[s]
    {
      const size_t row = (size_t)i * nth;
      int qs[5], ds[5];
      double t[5], wx[5], wy[5];
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        qs[s] = rot[s] ? rot_q(q, rot[s]) : q;
        ds[s] = d_of(qs[s]);
        t[s] = (double)f[qs[s] * plane + row + jj[s]];
        wx[s] = rot[s] ? speed(k) * cos_d(ds[s]) : vx;
        wy[s] = rot[s] ? speed(k) * sin_d(ds[s]) : vy;
      }
      auto lam_at = [&](int s) { return (double)lam[qs[s] * plane + row + jj[s]]; };
      double vt, aC, K;
      // s = 0: n = j - 2 uses m only when its upwind side is forward (m = u2)
      vt = -wx[0] * sn[0] + wy[0] * cs[0];
      if (!((tbs[0] >> ds[0]) & 1u)) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= lam_at(0) * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t[0], (A)t[1], (A)t[2], TEa).du2;
      }
      // s = 1: n = j - 1, forward (m = u1)
      vt = -wx[1] * sn[1] + wy[1] * cs[1];
      if (!((tbs[1] >> ds[1]) & 1u)) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= lam_at(1) * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t[1], (A)t[2], (A)t[3], TEa).du1;
      }
      // s = 2: n = m (m is the centre)
      vt = -vx * sn[2] + vy * cs[2];
      aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
      acc -= lq * (double)(((tbs[2] >> d) & 1u) ? mwb_grad_t<A>((A)aC, (A)K, (A)t[2], (A)t[1], (A)t[0], TEa)
                                      : mwb_grad_t<A>((A)aC, (A)K, (A)t[2], (A)t[3], (A)t[4], TEa)).dc;
      // s = 3: n = j + 1, backward (m = u1)
      vt = -wx[3] * sn[3] + wy[3] * cs[3];
      if ((tbs[3] >> ds[3]) & 1u) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= lam_at(3) * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t[3], (A)t[2], (A)t[1], TEa).du1;
      }
      // s = 4: n = j + 2, backward (m = u2)
      vt = -wx[4] * sn[4] + wy[4] * cs[4];
      if ((tbs[4] >> ds[4]) & 1u) {
        aC = fabs(vt * sth_row); K = aC * (1.0 - aC);
        acc -= lam_at(4) * (double)mwb_grad_t<A>((A)aC, (A)K, (A)t[4], (A)t[3], (A)t[2], TEa).du2;
      }
    }
    out[q * plane + c0] = (R)acc;
  }
}

}  // namespace pclb
