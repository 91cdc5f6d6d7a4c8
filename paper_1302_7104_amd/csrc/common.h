// Device-side building blocks of the polar FDLB step (gfx950).
//
// Velocity model: Sec. II.A of Lin et al. (arXiv:1302.7104), Eq. DVM1, with
// the speeds (0, 1, 2.92, 2.99, 4.49) and the octagon row of Table I.
// Numbering: q = 0 rest; q = 1 + 8(k-1) + d for speed group k = 1..4 and
// direction d = 0..7 at angle d*pi/4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

// Every helper below is also compiled for the host, where a CPU emulation of
// the per-node update runs the same arithmetic for the CPU test-suite.
#define PCLB_HD __host__ __device__

namespace pclb {

constexpr int NQ = 33;
constexpr int NK = 4;
constexpr int ND = 8;
constexpr double RSQRT2 = 0.70710678118654752440084436210485;

__host__ __device__ constexpr double speed(int k) {
  return k == 0 ? 0.0 : k == 1 ? 1.0 : k == 2 ? 2.92 : k == 3 ? 2.99 : 4.49;
}
// cos and sin of d*pi/4, exact where they are 0 or +-1.
__host__ __device__ constexpr double cos_d(int d) {
  return d == 0 ? 1.0 : d == 1 ? RSQRT2 : d == 2 ? 0.0 : d == 3 ? -RSQRT2
       : d == 4 ? -1.0 : d == 5 ? -RSQRT2 : d == 6 ? 0.0 : RSQRT2;
}
__host__ __device__ constexpr double sin_d(int d) {
  return d == 0 ? 0.0 : d == 1 ? RSQRT2 : d == 2 ? 1.0 : d == 3 ? RSQRT2
       : d == 4 ? 0.0 : d == 5 ? -RSQRT2 : d == 6 ? -1.0 : -RSQRT2;
}
__host__ __device__ constexpr int qidx(int k, int d) { return 1 + ND * (k - 1) + d; }
__host__ __device__ constexpr int k_of(int q) { return q == 0 ? 0 : 1 + (q - 1) / ND; }
__host__ __device__ constexpr int d_of(int q) { return q == 0 ? 0 : (q - 1) % ND; }
__host__ __device__ constexpr double vx_q(int q) { return speed(k_of(q)) * cos_d(d_of(q)); }
__host__ __device__ constexpr double vy_q(int q) { return speed(k_of(q)) * sin_d(d_of(q)); }
__host__ __device__ constexpr double v2_q(int q) { return speed(k_of(q)) * speed(k_of(q)); }

// Weights F_k(E) of the octagon model (Eqs. F_k with the first row of Table I,
// B = (B0, B1, B2, B3, B4) = (8, -1/4, 1, -6, 48), suffixes {k+l} = mod{k+l, 4})
// as polynomials F_k(E) = E (c0 + E (c1 + E (c2 + E c3))):
//   c0 = B1 e3 / den, c1 = B2 e2 / den, c2 = B3 e1 / den, c3 = B4 / den,
// e1, e2, e3 the elementary symmetric sums of the other three v_l^2 and
// den = v_k^2 prod_l (v_k^2 - v_l^2).  Evaluated at compile time.
struct WeightPoly {
  double c[NK][4];
};
constexpr WeightPoly make_weight_poly() {
  WeightPoly w{};
  const double B1 = -0.25, B2 = 1.0, B3 = -6.0, B4 = 48.0;
  double x[NK + 1] = {};
  for (int k = 0; k <= NK; ++k) x[k] = speed(k) * speed(k);
  for (int k = 1; k <= NK; ++k) {
    int o[3] = {};
    for (int l = 1; l <= 3; ++l) o[l - 1] = (k + l <= NK) ? k + l : k + l - NK;
    const double a = x[o[0]], b = x[o[1]], c = x[o[2]];
    const double den = x[k] * (x[k] - a) * (x[k] - b) * (x[k] - c);
    w.c[k - 1][0] = B1 * a * b * c / den;
    w.c[k - 1][1] = B2 * (a * b + b * c + c * a) / den;
    w.c[k - 1][2] = B3 * (a + b + c) / den;
    w.c[k - 1][3] = B4 / den;
  }
  return w;
}
template <int K, int N> struct WC {
  static constexpr double v = make_weight_poly().c[K][N];
};
// F_k(E) for k = K + 1.
template <int K>
__host__ __device__ inline double weight_k(double E) {
  return E * (WC<K, 0>::v + E * (WC<K, 1>::v + E * (WC<K, 2>::v + E * WC<K, 3>::v)));
}
// dF_k/dE for k = K + 1.
template <int K>
__host__ __device__ inline double weight_k_prime(double E) {
  return WC<K, 0>::v + E * (2.0 * WC<K, 1>::v + E * (3.0 * WC<K, 2>::v + E * 4.0 * WC<K, 3>::v));
}

// 1/x in double.  On the device: the hardware reciprocal refined by two
// Newton steps (within an ulp or two of the IEEE quotient, at a fraction of
// the division sequence's cost; every FP64 division of the step is one of
// these).  The host emulation divides.
PCLB_HD inline double recip_d(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
#else
  return 1.0 / x;
#endif
}

// Everything a step launch needs besides the state buffers.
struct Tables {
  int32_t nr, nth;
  int32_t nf;          // theta covers 2 pi nf / 8 (8: the full annulus)
  double dt_dr;        // dt / dr
  double dt_dth;       // dt / dtheta
  double e;            // exp(-dt / tau), computed on the host in double
  const double* cth;   // cos(theta_j), j = 0..nth-1
  const double* sth;   // sin(theta_j)
  const double* rinv;  // 1 / r_i, i = 0..nr-1
  const double* wA;    // quadrature weight r_i w_i dr dtheta of row i
  int32_t n_mixed;     // strips of the strip kernel that contain an octant boundary
  int32_t scheme;      // convection scheme (SCH_* below)
};

// Convection schemes (Sec. II.B; the comparison of Sec. III.A, Figs. 5-6).
constexpr int SCH_MWB = 0, SCH_WB = 1, SCH_LW = 2, SCH_UPWIND2 = 3;

// Radial boundary description as the kernels see it.
struct BCdev {
  int32_t kind[2];     // PCLB_WALL / PCLB_INFLOW / PCLB_EXTRAPOLATE
  int32_t neq[2];      // 1: ghosts also take the wall row's f - f^eq
  double p[2][4];
  double rg[2][2];     // radius of ghost layer 0 (next to the wall) and 1, per side
};

// Ghost layers: ghost[((side * 2 + layer) * NQ + q) * nth + j], layer 0 at
// r = R1 - dr (inner) or R2 + dr (outer), layer 1 one spacing further out.
__host__ __device__ inline size_t ghost_index(int side, int layer, int q, int j, int nth) {
  return ((size_t)(side * 2 + layer) * NQ + q) * (size_t)nth + j;
}

// ---------------------------------------------------------------------------
// Equilibrium (Eq. feq) in the factorised form used on the device:
//   f^eq_{k,d} = rho F_k(E) P(w),  w = v_k (u . e_d),
//   P(w) = A0 + A1 w + A2 w^2 + A3 w^3 + A4 w^4,
//   A0 = 1 - a + a^2/2, A1 = g / E, A2 = g / (2E^2), A3 = 1/(6E^3), A4 = 1/(24E^4),
//   a = u^2 / (2E), g = 1 - a.
// Moments, equilibrium and relaxation run in double for both state types:
// the weights have opposite signs at the nearly equal speeds 2.92 and 2.99
// and P(w) cancels for w against the flow, so that float arithmetic here
// loses several digits per step (measured: 1e-4 relative after 100 steps),
// while rounding only the relaxed value to float keeps the FP32 state within
// about 1e-6 of the FP64 trajectory.
struct EqCoef {
  double rF[NK + 1];   // rho F_k
  double A0, A1, A2, A3, A4;
  double p[4];         // u . e_d for d = 0..3 (d + 4 is the negative)
};

PCLB_HD inline void eq_setup(const Tables&, double rho, double ux, double uy, double E,
                             EqCoef& c) {
  double iE = recip_d(E);
  const double F1 = weight_k<0>(E), F2 = weight_k<1>(E), F3 = weight_k<2>(E), F4 = weight_k<3>(E);
  c.rF[1] = rho * F1;
  c.rF[2] = rho * F2;
  c.rF[3] = rho * F3;
  c.rF[4] = rho * F4;
  c.rF[0] = rho * (1.0 - 8.0 * (((F1 + F2) + F3) + F4));
  double u2 = ux * ux + uy * uy;
  double a = 0.5 * u2 * iE;
  double g = 1.0 - a;
  double iE2 = iE * iE;
  c.A0 = g + 0.5 * a * a;
  c.A1 = g * iE;
  c.A2 = 0.5 * g * iE2;
  c.A3 = iE2 * iE * (1.0 / 6.0);
  c.A4 = iE2 * iE2 * (1.0 / 24.0);
  c.p[0] = ux;
  c.p[1] = (ux + uy) * RSQRT2;
  c.p[2] = uy;
  c.p[3] = (uy - ux) * RSQRT2;
}

PCLB_HD inline double eq_val(const EqCoef& c, int k, int d) {
  double pd = d < 4 ? c.p[d] : -c.p[d - 4];
  double w = speed(k) * pd;
  return c.rF[k] * (c.A0 + w * (c.A1 + w * (c.A2 + w * (c.A3 + w * c.A4))));
}

// Linear moments of one node, rho, j = sum f v and eps = sum f v^2 (halved at
// the end), summed per pair of opposite directions (d, d+4), d = 0..3: with
// sp_k = f_{k,d} + f_{k,d+4} and sm_k = f_{k,d} - f_{k,d+4},
//   rho_d = sum_k sp_k, j_d = sum_k v_k e_d sm_k, eps_d = sum_k v_k^2 sp_k
// the four partials are then added in the order d = 0, 1, 2, 3 and the rest
// velocity last.  Every kernel sums in exactly this order.
PCLB_HD inline void d4_partial(int d4, const double* fp, const double* fm, double* P) {
  double r = 0.0, jx = 0.0, jy = 0.0, eps = 0.0;
#pragma unroll
  for (int k = 1; k <= NK; ++k) {
    const double sp = fp[k - 1] + fm[k - 1];
    const double sm = fp[k - 1] - fm[k - 1];
    r += sp;
    // a zero component adds nothing (skipping it leaves every sum unchanged
    // and saves the constants and operations in the kernels, where d4 is
    // known at compile time)
    if (cos_d(d4) != 0.0) jx += (speed(k) * cos_d(d4)) * sm;
    if (sin_d(d4) != 0.0) jy += (speed(k) * sin_d(d4)) * sm;
    eps += (speed(k) * speed(k)) * sp;
  }
  P[0] = r;
  P[1] = jx;
  P[2] = jy;
  P[3] = eps;
}

// rho, u, E (Eqs. moment1-moment3: E = eps / (2 rho) - u^2 / 2) from the four
// pair partials P[d][0..3] and the rest velocity's value f0.
PCLB_HD inline void combine_partials(const double P[4][4], double f0, double& rho, double& ux,
                                     double& uy, double& E) {
  const double r = (((P[0][0] + P[1][0]) + P[2][0]) + P[3][0]) + f0;
  const double jx = ((P[0][1] + P[1][1]) + P[2][1]) + P[3][1];
  const double jy = ((P[0][2] + P[1][2]) + P[2][2]) + P[3][2];
  const double eps = ((P[0][3] + P[1][3]) + P[2][3]) + P[3][3];
  rho = r;
  const double ir = recip_d(r);
  ux = jx * ir;
  uy = jy * ir;
  E = 0.5 * eps * ir - 0.5 * (ux * ux + uy * uy);
}

PCLB_HD inline void node_partials(const double* f, double P[4][4]) {
  for (int d4 = 0; d4 < 4; ++d4) {
    double fp[NK], fm[NK];
    for (int k = 1; k <= NK; ++k) {
      fp[k - 1] = f[qidx(k, d4)];
      fm[k - 1] = f[qidx(k, d4 + 4)];
    }
    d4_partial(d4, fp, fm, P[d4]);
  }
}

PCLB_HD inline void node_macros(const double* f, double& rho, double& ux, double& uy, double& E) {
  double P[4][4];
  node_partials(f, P);
  combine_partials(P, f[0], rho, ux, uy, E);
}

// Relaxed values of the opposite pair (k, d) and (k, d + 4), d = 0..3
// (Eq. operator1_new): f^eq + (f - f^eq) e written as e f + (1 - e) f^eq,
// with f^eq = rho F_k P(+-w) and P split into its even and odd parts in
// w = v_k pd, pd = u . e_d (the caller passes c.p[d], or its negative to hand
// the pair over in the order (d + 4, d); negation is exact, so both orders
// give the same two values).  In double: the caller rounds once, after the
// convection terms.  one_m_e = 1 - e.
template <int K>
PCLB_HD inline void relax_pair(const EqCoef& c, double e, double one_m_e, double pd, double fp,
                               double fm, double& rp, double& rm) {
  const double w = speed(K) * pd;
  const double w2 = w * w;
  const double ev = c.A0 + w2 * (c.A2 + w2 * c.A4);
  const double od = w * (c.A1 + w2 * c.A3);
  const double s = one_m_e * c.rF[K];
  const double gp = s * (ev + od), gm = s * (ev - od);
  rp = fma(fp, e, gp);
  rm = fma(fm, e, gm);
}

// The rest velocity: (1 - e) rho F_0 A0 + e f_0.
PCLB_HD inline double relax_rest_share(const EqCoef& c, double one_m_e) {
  return one_m_e * (c.rF[0] * c.A0);
}

template <class R>
PCLB_HD inline R relax_rest(double s0, double e, double f0) {
  return (R)fma(f0, e, s0);
}

// Upwind sides.  The radial and azimuthal components of direction d at angle
// theta are v_k cos(d pi/4 - theta) and v_k sin(d pi/4 - theta); a velocity is
// upwind-backward (its stencil lies at lower index) where its component is
// >= 0.  Inside the octant (m pi/4, (m+1) pi/4] of theta the pattern of signs
// depends only on d - m: relative to the octant, directions 7, 0, 1, 2 are
// radially backward and 1, 2, 3, 4 azimuthally backward.  The octant of
// column j follows from exact integer arithmetic, theta_j = (j+1) 2 pi / nth,
// so the side is exact even at the columns on the axes theta = m pi/4, where
// one component of four directions vanishes and its computed value is
// rounding noise: such a column takes the sides of the octant below it (the
// limit of the signs as theta approaches the axis from below).  The term of
// that component has |C| ~ 1e-17 there, so the choice moves no result
// beyond that size.
PCLB_HD inline int octant_of(int j, int nth, int nf) {
  // theta_j = (j+1) dtheta with dtheta = 2 pi nf / (8 nth): the octant m
  // with theta_j in (m pi/4, (m+1) pi/4]
  return (int)(((long long)nf * (j + 1) - 1) / nth);
}

// Azimuthal boundary condition of a sector 0 < theta <= 2 pi nf / 8 (Sec.
// II.C, Fig. 3): a ghost column before the first real one holds the values
// of the column nth places later with the direction index advanced by nf,
// a ghost column after the last holds those nth places earlier with it
// moved back by nf (8 - nf modulo 8).  rot_q returns the velocity whose
// plane is read: speed unchanged, direction d -> (d + s) mod 8; the rest
// velocity is unchanged.  With nf = 8 both rotations are the identity.
PCLB_HD inline int rot_q(int q, int s) {
  return q == 0 ? 0 : 1 + ((q - 1) & ~7) + (((q - 1) + s) & 7);
}
PCLB_HD inline unsigned rot8(unsigned bits, int m) {
  return ((bits << m) | (bits >> (8 - m))) & 0xffu;
}
constexpr unsigned RBACK_OCT0 = 0x87u;   // relative directions 0, 1, 2, 7
constexpr unsigned TBACK_OCT0 = 0x1eu;   // relative directions 1, 2, 3, 4
PCLB_HD inline unsigned rback_bits(int oct) { return rot8(RBACK_OCT0, oct); }
PCLB_HD inline unsigned tback_bits(int oct) { return rot8(TBACK_OCT0, oct); }

// Direction geometry of one theta column: for each direction d, the upwind
// sides (bit d set = backward) and, per d mod 4, |v_r| dt/dr and
// |v_theta| dt/dtheta per unit speed.  The Courant numbers of velocity (k, d)
// are v_k * ar[d mod 4] and v_k * at[d mod 4] / r.
template <class R> struct DirGeom {
  R ar[4], at[4];
  unsigned rback, tback;
};
template <class R>
PCLB_HD inline void dir_geometry(double ct, double st, int oct, double dt_dr, double dt_dth,
                                 DirGeom<R>& g) {
  g.rback = rback_bits(oct);
  g.tback = tback_bits(oct);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const double vr = cos_d(d) * ct + sin_d(d) * st;     // v_r / v_k
    const double vt = sin_d(d) * ct - cos_d(d) * st;     // v_theta / v_k
    g.ar[d] = (R)(fabs(vr) * dt_dr);
    g.at[d] = (R)(fabs(vt) * dt_dth);
  }
}
// |C| and |C|(1 - |C|) from the speed and the per-unit-speed factor.
template <class R>
PCLB_HD inline void courant(R vk, R a, R& aC, R& K) {
  aC = vk * a;
  K = aC - aC * aC;
}

// ---------------------------------------------------------------------------
// MWB convection term (Eq. MWB Scheme) in the division-free form, written with
// the upwind differences d1 = c - u1 and d2 = u1 - u2 (u1 one node upwind, u2
// two nodes upwind):
//   T = |C| d1 + |C|(1-|C|) (d1 - d2) |d1| / (|d1| + |d2|),
// which equals [C + C(1-|C|)(1-S(eta))(1-eta)/2] delta for either sign of C,
// and whose limiter part is 0 when d1 = d2 = 0.
//
// Limiter part (d1 - d2) |d1| / (|d1| + |d2|).  Double on the device: the
// weight |d1| / (|d1| + |d2|) with recip_d (the IEEE division sequence cost
// 0.4 ms of a 5 ms FP64 step), capped at 1; the denominator is guarded so
// that d1 = d2 = 0 gives 0.  Float on the device: the weight from
// the hardware reciprocal, saturated to [0, 1] by the VALU clamp, which also
// sends the 0 * inf of d1 = d2 = 0 to 0.  The host emulation divides.
template <class R>
PCLB_HD inline R mwb_lim(R d1, R d2);
template <>
PCLB_HD inline double mwb_lim<double>(double d1, double d2) {
  const double a1 = fabs(d1), a2 = fabs(d2);
  const double s = fmax(a1 + a2, 2.2250738585072014e-308);
#if defined(__HIP_DEVICE_COMPILE__)
  return (d1 - d2) * fmin(a1 * recip_d(s), 1.0);
#else
  // host emulation of the device arithmetic (tests only)
  return (d1 - d2) * a1 / s;
#endif
}
template <>
PCLB_HD inline float mwb_lim<float>(float d1, float d2) {
  const float a1 = fabsf(d1), a2 = fabsf(d2);
#if defined(__HIP_DEVICE_COMPILE__)
  const float w = __builtin_amdgcn_fmed3f(a1 * __builtin_amdgcn_rcpf(a1 + a2), 0.0f, 1.0f);
#else
  // host emulation of the device arithmetic (tests only)
  const float den = a1 + a2;
  const float w = den == 0.0f ? 0.0f : fminf(a1 * (1.0f / den), 1.0f);
#endif
  return (d1 - d2) * w;
}

template <class R>
PCLB_HD inline R mwb_term(R absC, R K, R c, R u1, R u2) {
  const R d1 = c - u1;
  const R d2 = u1 - u2;
  return absC * d1 + K * mwb_lim<R>(d1, d2);
}

// rel - T_r - T_theta for one velocity from the radial differences (d1r, d2r)
// with (aCr, Kr) and the azimuthal ones (d1t, d2t) with (aCt, Kt).  The two
// MWB terms are formed in the state type (each is a Courant number times an
// upwind difference, far smaller than f); they are subtracted from the relaxed
// value in double, and the new f is rounded once to the state type.  (Four
// float operations at the size of f would round four times.)
template <class R>
PCLB_HD inline R mwb_update_d(double rel, R aCr, R Kr, R d1r, R d2r, R aCt, R Kt, R d1t, R d2t) {
  const R tr = aCr * d1r + Kr * mwb_lim<R>(d1r, d2r);
  const R tt = aCt * d1t + Kt * mwb_lim<R>(d1t, d2t);
  return (R)((rel - (double)tr) - (double)tt);
}

// The convection term of each scheme in the same upwind form: with
// |C| = aC, K = |C|(1 - |C|), d1 = c - u1, d2 = u1 - u2 and the downwind
// difference dw = w1 - c (w1 one node downwind),
//   MWB:                 aC d1 + K (d1 - d2) |d1| / (|d1| + |d2|)
//   Warming-Beam:        aC d1 + K/2 (d1 - d2)       (the MWB bracket with S = 0)
//   Lax-Wendroff:        aC d1 + K/2 (dw - d1)
//   second-order upwind: aC d1 + aC/2 (d1 - d2)
// (each equals the scheme's printed or textbook form for either sign of C).
// The upwind schemes' term from the differences alone (not Lax-Wendroff).
template <int SCH, class R>
PCLB_HD inline R conv_term_d(R aC, R K, R d1, R d2) {
  static_assert(SCH != SCH_LW, "Lax-Wendroff needs the downwind neighbour");
  if constexpr (SCH == SCH_WB) return aC * d1 + (R)0.5 * K * (d1 - d2);
  else if constexpr (SCH == SCH_UPWIND2) return aC * d1 + (R)0.5 * aC * (d1 - d2);
  else return aC * d1 + K * mwb_lim<R>(d1, d2);
}

template <int SCH, class R>
PCLB_HD inline R conv_term(R aC, R K, R c, R u1, R u2, R w1) {
  const R d1 = c - u1, d2 = u1 - u2;
  if constexpr (SCH == SCH_LW) return aC * d1 + (R)0.5 * K * ((w1 - c) - d1);
  else return conv_term_d<SCH, R>(aC, K, d1, d2);
}

// rel - T_r - T_theta of an upwind scheme from the differences, as
// mwb_update_d (the same rounding as velocity_update for that scheme).
template <int SCH, class R>
PCLB_HD inline R scheme_update_d(double rel, R aCr, R Kr, R d1r, R d2r, R aCt, R Kt, R d1t, R d2t) {
  if constexpr (SCH == SCH_MWB) {
    return mwb_update_d<R>(rel, aCr, Kr, d1r, d2r, aCt, Kt, d1t, d2t);
  } else {
    const R tr = conv_term_d<SCH, R>(aCr, Kr, d1r, d2r);
    const R tt = conv_term_d<SCH, R>(aCt, Kt, d1t, d2t);
    return (R)((rel - (double)tr) - (double)tt);
  }
}

// The same from the centre value c and the upwind neighbours.
template <class R>
PCLB_HD inline R mwb_update(double rel, R c, R aCr, R Kr, R u1r, R u2r, R aCt, R Kt, R u1t, R u2t) {
  return mwb_update_d<R>(rel, aCr, Kr, c - u1r, u1r - u2r, aCt, Kt, c - u1t, u1t - u2t);
}

// Compile-time loop over the speeds k = K..NK.
template <int K, class Fn>
PCLB_HD inline void for_k(Fn&& fn) {
  if constexpr (K <= NK) {
    fn(std::integral_constant<int, K>{});
    for_k<K + 1>(fn);
  }
}

// New value of velocity q (direction d) of one node from its relaxed value
// rel (double), its centre value c and the Courant factors, the neighbours
// read through row(q, di) / col(q, dj): the scheme's two convection terms in
// the state type, subtracted in double, one rounding.
template <class R, int SCH, class RowFn, class ColFn>
PCLB_HD inline R velocity_update(const DirGeom<R>& G, int d, int q, double rel, R c, R aCr, R Kr,
                                 R aCt, R Kt, RowFn& row, ColFn& col) {
  const int sr = ((G.rback >> d) & 1u) ? -1 : 1;   // upwind offset in r
  const int sc = ((G.tback >> d) & 1u) ? -1 : 1;   // upwind offset in theta
  if constexpr (SCH == SCH_MWB) {
    return mwb_update<R>(rel, c, aCr, Kr, row(q, sr), row(q, 2 * sr), aCt, Kt, col(q, sc),
                         col(q, 2 * sc));
  } else {
    // the downwind neighbours only matter to Lax-Wendroff
    const R wr = SCH == SCH_LW ? row(q, -sr) : c;
    const R wt = SCH == SCH_LW ? col(q, -sc) : c;
    const R tr = conv_term<SCH, R>(aCr, Kr, c, row(q, sr), row(q, 2 * sr), wr);
    const R tt = conv_term<SCH, R>(aCt, Kt, c, col(q, sc), col(q, 2 * sc), wt);
    return (R)((rel - (double)tr) - (double)tt);
  }
}

// ---------------------------------------------------------------------------
// Combined-scheme update of one node (Eq. combined_scheme): centre values fc,
// radial neighbours row(q, di) at rows i+di (di = -2, -1, 1, 2; ghost rows
// included) and azimuthal neighbours col(q, dj) at columns j+dj of row i.
// put(q, value) receives f_q at t + dt as soon as it is computed (so that a
// kernel can store it at once instead of holding all 33 results).
template <class R, int SCH = SCH_MWB, class RowFn, class ColFn, class PutFn>
PCLB_HD inline void node_update_put(const Tables& T, int i, int j, const R* fc, RowFn row,
                                    ColFn col, PutFn put) {
  const double ct = T.cth[j], st = T.sth[j];
  double fd[NQ];
  for (int q = 0; q < NQ; ++q) fd[q] = (double)fc[q];
  double rho, ux, uy, E;
  node_macros(fd, rho, ux, uy, E);
  EqCoef ec;
  eq_setup(T, rho, ux, uy, E, ec);
  const double e = T.e, ome = 1.0 - T.e;
  put(0, relax_rest<R>(relax_rest_share(ec, ome), e, fd[0]));   // rest velocity: no convection
  DirGeom<R> G;
  dir_geometry(ct, st, octant_of(j, T.nth, T.nf), T.dt_dr, T.dt_dth, G);
  const R rinv = (R)T.rinv[i];
  R atr[4];
  for (int d = 0; d < 4; ++d) atr[d] = G.at[d] * rinv;
  // direction pairs outer, speeds inner
#pragma unroll
  for (int d4 = 0; d4 < 4; ++d4) {
    for_k<1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      double rel[2];
      relax_pair<k>(ec, e, ome, ec.p[d4], fd[qidx(k, d4)], fd[qidx(k, d4 + 4)], rel[0], rel[1]);
      R aCr, Kr, aCt, Kt;
      courant<R>((R)speed(k), G.ar[d4], aCr, Kr);
      courant<R>((R)speed(k), atr[d4], aCt, Kt);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = qidx(k, d4 + 4 * h);
        put(q, velocity_update<R, SCH>(G, d4 + 4 * h, q, rel[h], fc[q], aCr, Kr, aCt, Kt, row, col));
      }
    });
  }
}

// The same with the results in res[0..NQ-1].
template <class R, int SCH = SCH_MWB, class RowFn, class ColFn>
PCLB_HD inline void node_update(const Tables& T, int i, int j, const R* fc, RowFn row, ColFn col,
                                R* res) {
  node_update_put<R, SCH>(T, i, j, fc, row, col, [&](int q, R v) { res[q] = v; });
}

// Ghost layers of one wall and column (Sec. II.C, radial boundary condition):
// from the macroscopic state of the wall row (f0) and the next row (f1),
// extrapolate rho and E linearly and recursively (ghost0 = 2 row0 - row1,
// ghost1 = 2 ghost0 - row0), set u per boundary kind, and return f^eq of
// both ghost states in g0 and g1; with bc.neq the non-equilibrium part
// f - f^eq of the wall row is added to both (the non-equilibrium boundary
// condition the paper cites for Sec. II.C), in double, rounded once.
template <class R>
PCLB_HD inline void ghost_column(const Tables& T, const BCdev& bc, int side, double ct, double st,
                                 const R* f0, const R* f1, R* g0, R* g1) {
  double m[2][4];
  double fl[NQ];
  for (int q = 0; q < NQ; ++q) fl[q] = (double)f0[q];
  node_macros(fl, m[0][0], m[0][1], m[0][2], m[0][3]);
  for (int q = 0; q < NQ; ++q) fl[q] = (double)f1[q];
  node_macros(fl, m[1][0], m[1][1], m[1][2], m[1][3]);
  double prev[4] = {m[0][0], m[0][1], m[0][2], m[0][3]};
  double pprev[4] = {m[1][0], m[1][1], m[1][2], m[1][3]};
  const int kind = bc.kind[side];
  const bool neq = bc.neq[side] != 0;
  EqCoef c0;
  if (neq) {
    const double ux0 = m[0][1], uy0 = m[0][2];
    eq_setup(T, m[0][0], ux0, uy0, m[0][3], c0);
  }
  // f - f^eq of the wall row, velocity q
  auto neq0 = [&](int q) -> double {
    if (!neq) return 0.0;
    const double fe = q == 0 ? c0.rF[0] * c0.A0 : eq_val(c0, k_of(q), d_of(q));
    return (double)f0[q] - fe;
  };
  for (int layer = 0; layer < 2; ++layer) {
    double g[4];
    for (int a = 0; a < 4; ++a) g[a] = 2.0 * prev[a] - pprev[a];
    for (int a = 0; a < 4; ++a) { pprev[a] = prev[a]; prev[a] = g[a]; }
    double rho = g[0], ux = g[1], uy = g[2], E = g[3];
    if (kind == 0) {                   // WALL: u_r = 0, u_theta = omega r_g
      const double ut = bc.p[side][0] * bc.rg[side][layer];
      ux = -ut * st;
      uy = ut * ct;
    } else if (kind == 1) {            // INFLOW
      rho = bc.p[side][0];
      ux = bc.p[side][1] * ct - bc.p[side][2] * st;
      uy = bc.p[side][1] * st + bc.p[side][2] * ct;
      E = bc.p[side][3];
    }                                  // EXTRAPOLATE keeps the extrapolated u
    EqCoef c;
    eq_setup(T, rho, ux, uy, E, c);
    R* out = layer == 0 ? g0 : g1;
    out[0] = (R)(c.rF[0] * c.A0 + neq0(0));
    for (int k = 1; k <= NK; ++k)
      for (int d = 0; d < ND; ++d) out[qidx(k, d)] = (R)(eq_val(c, k, d) + neq0(qidx(k, d)));
  }
}

}  // namespace pclb
