// The double and triple octagon models (Sec. II.A: Eq. DVM1 with N_i = 16 or
// 24 directions per speed, the weights of Table I's second and third rows):
// radial ghost layers, step, initial state, fields and diagnostics for 65 and
// 97 velocities.  One thread per node, the velocities visited in runtime loops
// (the velocity count makes fully unrolled code, as the octagon kernels use,
// impractical), every neighbour read from global memory.  The arithmetic per
// velocity is the octagon's: moments and equilibrium in double, f^eq =
// rho F_k P(w), the relaxation e f + (1 - e) f^eq, the scheme's two convection
// terms (conv_term) in the state type, one rounding.  Upwind sides follow the
// signs of the computed velocity components (a component that vanishes exactly
// has |C| of the order of the rounding there, so its side moves no result
// beyond that size).  State layout f[q][i][j] with q = 1 + N_i (k - 1) + d;
// ghost layers ghost[side][layer][q][j] with 1 + 4 N_i planes.
#include "common.h"
#include "diag.h"
#include "launch.h"
#include "strip_common.h"

namespace pclb {

namespace {

// cos and sin of 2 pi d / N for d = 0..N-1 (N a multiple of 8), formed at
// compile time: the angle is split into o eighths of the circle and a
// remainder x in [0, pi/4), whose series are summed to full double precision
// (the 14th term is below 1e-40), then rotated by the o eighths.
constexpr double CPI = 3.14159265358979323846;
constexpr double series_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double series_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
constexpr void dir_cs(int d, int N, double& c, double& s) {
  const int n = N / 8, o = d / n, m = d % n;
  const double x = CPI / 4.0 * m / n;
  const double a = m == 0 ? 1.0 : series_cos(x), b = m == 0 ? 0.0 : series_sin(x);
  const double h = RSQRT2;
  switch (o) {
    case 0: c = a; s = b; break;
    case 1: c = (a - b) * h; s = (a + b) * h; break;
    case 2: c = -b; s = a; break;
    case 3: c = -(a + b) * h; s = (a - b) * h; break;
    case 4: c = -a; s = -b; break;
    case 5: c = (b - a) * h; s = -(a + b) * h; break;
    case 6: c = b; s = -a; break;
    default: c = (a + b) * h; s = (b - a) * h;
  }
}
template <int NI> struct Dirs {
  double c[NI], s[NI];
  constexpr Dirs() : c(), s() {
    for (int d = 0; d < NI; ++d) dir_cs(d, NI, c[d], s[d]);
  }
};
// compile-time checks of the tables against values known to 20 digits, and
// of |e_d| = 1 for every direction
constexpr double cabs(double x) { return x < 0 ? -x : x; }
template <int NI> constexpr bool unit_dirs() {
  const Dirs<NI> t{};
  for (int d = 0; d < NI; ++d)
    if (cabs(t.c[d] * t.c[d] + t.s[d] * t.s[d] - 1.0) > 4.5e-16) return false;
  return true;
}
static_assert(cabs(Dirs<16>().c[1] - 0.92387953251128675613) < 2.3e-16, "cos(pi/8)");
static_assert(cabs(Dirs<16>().s[1] - 0.38268343236508977173) < 1.2e-16, "sin(pi/8)");
static_assert(cabs(Dirs<16>().c[13] - 0.38268343236508977173) < 1.2e-16, "cos(13 pi/8)");
static_assert(cabs(Dirs<16>().s[13] + 0.92387953251128675613) < 2.3e-16, "sin(13 pi/8)");
static_assert(cabs(Dirs<24>().c[1] - 0.96592582628906828675) < 2.3e-16, "cos(pi/12)");
static_assert(cabs(Dirs<24>().s[2] - 0.5) < 1.2e-16, "sin(pi/6)");
static_assert(cabs(Dirs<24>().c[10] + 0.86602540378443864676) < 2.3e-16, "cos(5 pi/6)");
static_assert(cabs(Dirs<24>().s[17] + 0.96592582628906828675) < 2.3e-16, "sin(17 pi/12)");
static_assert(unit_dirs<16>() && unit_dirs<24>(), "unit directions");

__constant__ Dirs<16> DIRS16 = Dirs<16>();
__constant__ Dirs<24> DIRS24 = Dirs<24>();
template <int NI> __device__ inline const Dirs<NI>& dirs();
template <> __device__ inline const Dirs<16>& dirs<16>() { return DIRS16; }
template <> __device__ inline const Dirs<24>& dirs<24>() { return DIRS24; }

// Weights F_k(E) of Table I's row for N_i (Eqs. F_k), as polynomials
// E (c0 + E (c1 + E (c2 + E c3))) with coefficients formed at compile time
// (the octagon's construction with that row's B1..B4); F_0 = 1 - B0 sum F_k.
struct RowB {
  double b0, b1, b2, b3, b4;
};
template <int NI> constexpr RowB row_b();
template <> constexpr RowB row_b<16>() { return {16.0, -1.0 / 8.0, 0.5, -3.0, 24.0}; }
template <> constexpr RowB row_b<24>() { return {24.0, -1.0 / 12.0, 1.0 / 3.0, -2.0, 16.0}; }
// coefficient N of F_k, k = K + 1
template <int NI> constexpr double row_coef(int K, int N) {
  const RowB B = row_b<NI>();
  double x[NK + 1] = {};
  for (int k = 0; k <= NK; ++k) x[k] = speed(k) * speed(k);
  const int k = K + 1;
  int o[3] = {};
  for (int l = 1; l <= 3; ++l) o[l - 1] = (k + l <= NK) ? k + l : k + l - NK;
  const double a = x[o[0]], b = x[o[1]], c = x[o[2]];
  const double den = x[k] * (x[k] - a) * (x[k] - b) * (x[k] - c);
  return N == 0 ? B.b1 * a * b * c / den
       : N == 1 ? B.b2 * (a * b + b * c + c * a) / den
       : N == 2 ? B.b3 * (a + b + c) / den
       : B.b4 / den;
}
template <int NI, int K, int N> struct RC {
  static constexpr double v = row_coef<NI>(K, N);
};
template <int NI, int K>
__device__ inline double row_weight(double E) {
  return E * (RC<NI, K, 0>::v + E * (RC<NI, K, 1>::v + E * (RC<NI, K, 2>::v + E * RC<NI, K, 3>::v)));
}

template <int NI> constexpr int nq_of() { return 1 + NK * NI; }

// Equilibrium coefficients of one node in the octagon kernels' factorised
// form (Eq. feq: f^eq = rho F_k P(w), P(w) = A0 + A1 w + ... + A4 w^4,
// w = v_k u . e_d) with this model's weights; the relaxation of an opposite
// pair (d, d + N_i/2) then goes through relax_pair, whose even and odd parts
// of P serve both members.
template <int NI>
__device__ inline void eq_models(double rho, double ux, double uy, double E, EqCoef& c) {
  const double F1 = row_weight<NI, 0>(E), F2 = row_weight<NI, 1>(E);
  const double F3 = row_weight<NI, 2>(E), F4 = row_weight<NI, 3>(E);
  c.rF[1] = rho * F1;
  c.rF[2] = rho * F2;
  c.rF[3] = rho * F3;
  c.rF[4] = rho * F4;
  c.rF[0] = rho * (1.0 - row_b<NI>().b0 * (((F1 + F2) + F3) + F4));
  const double iE = recip_d(E), u2 = ux * ux + uy * uy, a = 0.5 * u2 * iE, g = 1.0 - a;
  const double iE2 = iE * iE;
  c.A0 = g + 0.5 * a * a;
  c.A1 = g * iE;
  c.A2 = 0.5 * g * iE2;
  c.A3 = iE2 * iE * (1.0 / 6.0);
  c.A4 = iE2 * iE2 * (1.0 / 24.0);
  c.p[0] = ux;   // the Cartesian velocity (u . e_d is formed per direction)
  c.p[1] = uy;
  c.p[2] = c.p[3] = 0.0;
}

// f^eq of the pair (K, d) and (K, d + N_i/2), pd = u . e_d.
template <int K>
__device__ inline void feq_pair(const EqCoef& c, double pd, double& fp, double& fm) {
  const double w = speed(K) * pd, w2 = w * w;
  const double ev = c.A0 + w2 * (c.A2 + w2 * c.A4);
  const double od = w * (c.A1 + w2 * c.A3);
  fp = c.rF[K] * (ev + od);
  fm = c.rF[K] * (ev - od);
}

// fn(k, d, qp, qm) for every opposite pair: speed group k as a compile-time
// constant, direction d = 0 .. N_i/2 - 1 in a runtime loop (outer), planes qp
// of (k, d) and qm of (k, d + N_i/2).  The direction's constants are loaded
// once for its four speeds, and the eight velocities' loads of one iteration
// are in flight together.
template <int NI, class Fn>
__device__ inline void for_each_pair(Fn&& fn) {
#pragma unroll 1
  for (int d = 0; d < NI / 2; ++d) {
    for_k<1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int qp = 1 + NI * (k - 1) + d;
      fn(kc, d, qp, qp + NI / 2);
    });
  }
}

// Moment partials of the opposite pair (d, d + N_i/2) over the four speeds,
// from the pair's values fp[k-1] (direction d) and fm[k-1] (d + N_i/2): with
// sp = fp + fm and sm = fp - fm, P = (sum sp, sum v_k c_d sm, sum v_k s_d sm,
// sum v_k^2 sp), speeds in order.
template <int NI>
__device__ inline void pair_partial(int d, const double* fp, const double* fm, double* P) {
  const double cd = dirs<NI>().c[d], sd = dirs<NI>().s[d];
  double r = 0.0, jx = 0.0, jy = 0.0, eps = 0.0;
#pragma unroll
  for (int k = 1; k <= NK; ++k) {
    const double sp = fp[k - 1] + fm[k - 1], sm = fp[k - 1] - fm[k - 1];
    r += sp;
    jx += (speed(k) * cd) * sm;
    jy += (speed(k) * sd) * sm;
    eps += (speed(k) * speed(k)) * sp;
  }
  P[0] = r;
  P[1] = jx;
  P[2] = jy;
  P[3] = eps;
}

// rho, u, E from the sums of the pair partials (taken in pair order) and the
// rest velocity's value, added last (Eqs. moment1-moment3).
__device__ inline void moments_from_sums(double r, double jx, double jy, double eps, double f0,
                                         double& rho, double& ux, double& uy, double& E) {
  rho = r + f0;
  const double ir = recip_d(rho);
  ux = jx * ir;
  uy = jy * ir;
  E = 0.5 * eps * ir - 0.5 * (ux * ux + uy * uy);
}

// rho, u, E of one node from its values get(q): pair partials in the order
// d = 0 .. N_i/2 - 1, then the rest velocity (every kernel of these models
// sums in exactly this order); jeps, if given, receives rho u_x, rho u_y and
// the energy density sum f v^2 / 2; fin becomes false if a value is not
// finite.
template <int NI, class Get>
__device__ inline void moments_of(Get get, double& rho, double& ux, double& uy, double& E,
                                  double* jeps = nullptr, bool* fin = nullptr) {
  double r = 0.0, jx = 0.0, jy = 0.0, eps = 0.0;
  bool ok = true;
#pragma unroll 1
  for (int d = 0; d < NI / 2; ++d) {
    double fp[NK], fm[NK], P[4];
#pragma unroll
    for (int k = 1; k <= NK; ++k) {
      const int qp = 1 + NI * (k - 1) + d;
      fp[k - 1] = get(qp);
      fm[k - 1] = get(qp + NI / 2);
      if (fin) ok = ok && isfinite(fp[k - 1]) && isfinite(fm[k - 1]);
    }
    pair_partial<NI>(d, fp, fm, P);
    r += P[0];
    jx += P[1];
    jy += P[2];
    eps += P[3];
  }
  const double f0 = get(0);
  if (fin) *fin = ok && isfinite(f0);
  moments_from_sums(r, jx, jy, eps, f0, rho, ux, uy, E);
  if (jeps) {
    jeps[0] = jx;
    jeps[1] = jy;
    jeps[2] = 0.5 * eps;
  }
}

__device__ inline size_t gidx(int side, int layer, int q, int j, int nth, int nq) {
  return ((size_t)(side * 2 + layer) * nq + q) * (size_t)nth + j;
}

// The velocity whose plane a ghost column beyond the ends of a sector reads
// (Sec. II.C, Fig. 3): direction d -> (d + s) mod N_i, speed unchanged.
template <int NI>
__device__ inline int rotq(int q, int s) {
  if (q == 0 || s == 0) return q;
  const int k = (q - 1) / NI, d = (q - 1) % NI;
  return 1 + NI * k + (d + s) % NI;
}

// Radial ghost layers (Sec. II.C): rho, u, E of the two rows next to the wall
// extrapolated linearly and recursively, u set per boundary kind, f^eq of the
// ghost state stored; with bc.neq the wall row's f - f^eq is added.
template <class R, int NI>
__global__ void __launch_bounds__(256) models_ghost_kernel(Tables T, BCdev bc, const R* __restrict__ f,
                                                           R* __restrict__ ghost) {
  constexpr int NQM = nq_of<NI>();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int side = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const int i0 = side == 0 ? 0 : T.nr - 1, i1 = side == 0 ? 1 : T.nr - 2;
  const R* f0 = f + (size_t)i0 * T.nth + j;
  const R* f1 = f + (size_t)i1 * T.nth + j;
  double m[2][4];
  moments_of<NI>([&](int q) { return (double)f0[q * plane]; }, m[0][0], m[0][1], m[0][2], m[0][3]);
  moments_of<NI>([&](int q) { return (double)f1[q * plane]; }, m[1][0], m[1][1], m[1][2], m[1][3]);
  const double ct = T.cth[j], st = T.sth[j];
  const bool neq = bc.neq[side] != 0;
  EqCoef c0{};
  if (neq) eq_models<NI>(m[0][0], m[0][1], m[0][2], m[0][3], c0);
  double prev[4] = {m[0][0], m[0][1], m[0][2], m[0][3]};
  double pprev[4] = {m[1][0], m[1][1], m[1][2], m[1][3]};
  const int kind = bc.kind[side];
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
    eq_models<NI>(rho, ux, uy, E, c);
    const double nv0 = neq ? (double)f0[0] - c0.rF[0] * c0.A0 : 0.0;
    ghost[gidx(side, layer, 0, j, T.nth, NQM)] = (R)(c.rF[0] * c.A0 + nv0);
    for_each_pair<NI>([&](auto kc, int d, int qp, int qm) {
      constexpr int k = decltype(kc)::value;
      const double cd = dirs<NI>().c[d], sd = dirs<NI>().s[d];
      double ep, em, np = 0.0, nm = 0.0;
      feq_pair<k>(c, ux * cd + uy * sd, ep, em);
      if (neq) {
        double wp, wm;
        feq_pair<k>(c0, c0.p[0] * cd + c0.p[1] * sd, wp, wm);
        np = (double)f0[qp * plane] - wp;
        nm = (double)f0[qm * plane] - wm;
      }
      ghost[gidx(side, layer, qp, j, T.nth, NQM)] = (R)(ep + np);
      ghost[gidx(side, layer, qm, j, T.nth, NQM)] = (R)(em + nm);
    });
  }
}

// Eq. combined_scheme for every velocity of node (i, j): direction pairs
// outer, speeds inner (the octagon node kernel's order).  The Courant factors
// are formed as there: per direction |v_r| dt/dr and |v_theta| dt/dtheta per
// unit speed rounded to the state type, then times 1/r and the speed.
template <class R, int NI, int SCH, bool SECTOR>
__global__ void __launch_bounds__(256) models_step_kernel(Tables T, const R* __restrict__ f,
                                                          R* __restrict__ out,
                                                          const R* __restrict__ ghost) {
  constexpr int NQM = nq_of<NI>(), NH = NI / 2;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const int nr = T.nr, nth = T.nth;
  if (j >= nth) return;
  const size_t plane = (size_t)nr * nth;
  const size_t rowoff = (size_t)i * nth, c0 = rowoff + j;
  double rho, ux, uy, E;
  moments_of<NI>([&](int q) { return (double)f[q * plane + c0]; }, rho, ux, uy, E);
  EqCoef ec;
  eq_models<NI>(rho, ux, uy, E, ec);
  const double e = T.e, ome = 1.0 - T.e;
  const double ct = T.cth[j], st = T.sth[j];
  const R rinv = (R)T.rinv[i];
  // azimuthal neighbour columns, wrapped around the ring; on a sector a
  // wrapped column reads the direction rotated by n_f (low end) or back
  // (high end)
  const int jm1 = j >= 1 ? j - 1 : j - 1 + nth, jm2 = j >= 2 ? j - 2 : j - 2 + nth;
  const int jp1 = j + 1 < nth ? j + 1 : j + 1 - nth, jp2 = j + 2 < nth ? j + 2 : j + 2 - nth;
  const int s_lo = T.nf % NI, s_hi = (NI - T.nf % NI) % NI;
  const int rm1 = j >= 1 ? 0 : s_lo, rm2 = j >= 2 ? 0 : s_lo;
  const int rp1 = j + 1 < nth ? 0 : s_hi, rp2 = j + 2 < nth ? 0 : s_hi;
  auto azi = [&](int q, int dj) -> R {
    const int t = dj == -1 ? jm1 : dj == -2 ? jm2 : dj == 1 ? jp1 : jp2;
    int qq = q;
    if constexpr (SECTOR) qq = rotq<NI>(q, dj == -1 ? rm1 : dj == -2 ? rm2 : dj == 1 ? rp1 : rp2);
    return f[qq * plane + rowoff + t];
  };
  auto rad = [&](int q, int di) -> R {
    const int ii = i + di;
    if (ii < 0) return ghost[gidx(0, -1 - ii, q, j, nth, NQM)];
    if (ii >= nr) return ghost[gidx(1, ii - nr, q, j, nth, NQM)];
    return f[q * plane + c0 + (ptrdiff_t)di * nth];
  };
  out[c0] = relax_rest<R>(relax_rest_share(ec, ome), e, (double)f[c0]);   // rest velocity: no convection
  // update of one velocity q with centre value c, relaxed value rel, upwind
  // offsets sr, sc and Courant factors
  auto update = [&](int q, R c, double rel, int sr, int sc, R aCr, R Kr, R aCt, R Kt) {
    const R wr = SCH == SCH_LW ? rad(q, -sr) : c;   // downwind: Lax-Wendroff only
    const R wt = SCH == SCH_LW ? azi(q, -sc) : c;
    const R tr = conv_term<SCH, R>(aCr, Kr, c, rad(q, sr), rad(q, 2 * sr), wr);
    const R tt = conv_term<SCH, R>(aCt, Kt, c, azi(q, sc), azi(q, 2 * sc), wt);
    out[q * plane + c0] = (R)((rel - (double)tr) - (double)tt);
  };
#pragma unroll 1
  for (int d = 0; d < NH; ++d) {
    const double cd = dirs<NI>().c[d], sd = dirs<NI>().s[d];
    const double pd = ux * cd + uy * sd;
    const double vr = cd * ct + sd * st, vt = sd * ct - cd * st;   // per unit speed
    const R ar = (R)(fabs(vr) * T.dt_dr), at = (R)(fabs(vt) * T.dt_dth) * rinv;
    // upwind sides: backward (stencil at lower index) where the component is
    // >= 0; the opposite direction has the negated components
    const int srp = vr >= 0.0 ? -1 : 1, scp = vt >= 0.0 ? -1 : 1;
    const int srm = -vr >= 0.0 ? -1 : 1, scm = -vt >= 0.0 ? -1 : 1;
    for_k<1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int qp = 1 + NI * (k - 1) + d, qm = qp + NH;
      const R cp = f[qp * plane + c0], cm = f[qm * plane + c0];
      double rp, rm;
      relax_pair<k>(ec, e, ome, pd, (double)cp, (double)cm, rp, rm);
      R aCr, Kr, aCt, Kt;
      courant<R>((R)speed(k), ar, aCr, Kr);
      courant<R>((R)speed(k), at, aCt, Kt);
      update(qp, cp, rp, srp, scp, aCr, Kr, aCt, Kt);
      update(qm, cm, rm, srm, scm, aCr, Kr, aCt, Kt);
    });
  }
}

// f = f^eq(rho, u, T), u given in polar components (Eq. feq).
template <class R, int NI>
__global__ void __launch_bounds__(256) models_init_kernel(Tables T, const double* __restrict__ rho,
                                                          const double* __restrict__ ur,
                                                          const double* __restrict__ ut,
                                                          const double* __restrict__ Tt,
                                                          R* __restrict__ f, int* __restrict__ bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const size_t c0 = (size_t)i * T.nth + j;
  const double r = rho[c0], a = ur[c0], b = ut[c0], E = Tt[c0];
  if (!(r > 0.0) || !(E > 0.0) || !isfinite(r) || !isfinite(E) || !isfinite(a) || !isfinite(b))
    atomicOr(bad, 1);
  const double ct = T.cth[j], st = T.sth[j];
  const double ux = a * ct - b * st, uy = a * st + b * ct;
  EqCoef c;
  eq_models<NI>(r, ux, uy, E, c);
  f[c0] = (R)(c.rF[0] * c.A0);
  for_each_pair<NI>([&](auto kc, int d, int qp, int qm) {
    double ep, em;
    feq_pair<decltype(kc)::value>(c, ux * dirs<NI>().c[d] + uy * dirs<NI>().s[d], ep, em);
    f[qp * plane + c0] = (R)ep;
    f[qm * plane + c0] = (R)em;
  });
}

// rho, u_r, u_theta, T of every node (null outputs skipped).
template <class R, int NI>
__global__ void __launch_bounds__(256) models_fields_kernel(Tables T, const R* __restrict__ f,
                                                            double* rho, double* ur, double* ut,
                                                            double* Tt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const size_t c0 = (size_t)i * T.nth + j;
  double r, ux, uy, E;
  moments_of<NI>([&](int q) { return (double)f[q * plane + c0]; }, r, ux, uy, E);
  const double ct = T.cth[j], st = T.sth[j];
  if (rho) rho[c0] = r;
  if (ur) ur[c0] = ux * ct + uy * st;
  if (ut) ut[c0] = -ux * st + uy * ct;
  if (Tt) Tt[c0] = E;
}

// Diagnostics partials in the octagon's slot layout (mass, momentum x, y and
// energy as compensated (sum, error) pairs, min rho, min T, non-finite node
// count), one slot row per block; the fixed-order final pass is shared.
template <class R, int NI>
__global__ void __launch_bounds__(DIAG_BLOCK) models_diag_kernel(Tables T, const R* __restrict__ f,
                                                                 double* __restrict__ partial) {
  const size_t plane = (size_t)T.nr * T.nth;
  TwoS acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  double rmin = INFINITY, tmin = INFINITY, bad = 0.0;
  for (size_t n = (size_t)blockIdx.x * DIAG_BLOCK + threadIdx.x; n < plane;
       n += (size_t)gridDim.x * DIAG_BLOCK) {
    const int i = (int)(n / T.nth);
    double rho, ux, uy, E, je[3];
    bool fin;
    moments_of<NI>([&](int q) { return (double)f[q * plane + n]; }, rho, ux, uy, E, je, &fin);
    if (!fin) { bad += 1.0; continue; }
    const double w = T.wA[i];
    two_add(acc[0], rho * w);
    two_add(acc[1], je[0] * w);
    two_add(acc[2], je[1] * w);
    two_add(acc[3], je[2] * w);
    rmin = fmin(rmin, rho);
    tmin = fmin(tmin, E);
  }
  diag_block_reduce(acc, rmin, tmin, bad, partial);
}

// ---------------------------------------------------------------------------
// Strip form of the step (full annulus, n_theta a multiple of 64, every
// convection scheme: the ring holds both radial sides of a node and the halo
// both azimuthal ones, so Lax-Wendroff's downwind neighbour is at hand), the
// design of the octagon's FP64 strip kernel for N_i/2 direction pairs: a workgroup of N_i/2 wavefronts owns a strip of 64 theta columns
// (one per lane) and marches in r over a chunk of rows; wave W owns the pair
// (W, W + N_i/2), eight velocities, and wave 0 also the rest velocity.  Each
// owned velocity keeps a ring of MS_RING rows in registers: six (i-2 .. i+3
// at row i, the load of a row issued two rows before its first use) for the
// double octagon, five (i-2 .. i+2, one row before) for the triple octagon,
// whose twelve waves have 168 registers each; the row loop is unrolled
// MS_RING times so the roles rotate at compile time.  Per row the waves
// exchange their pair partials through LDS (one barrier, double-buffered by
// row parity), each builds the node's equilibrium from their sum in pair
// order, and updates its velocities with the node kernel's arithmetic, so the
// two forms agree bit for bit.  Azimuthal neighbours come from the adjacent
// lanes (ds_bpermute); the two columns beyond each end of the strip from a
// halo read one row ahead (one load per lane: lane v the pair left of the
// strip for velocity v, lane 8 + v the pair right of it).

template <class R> struct Pair2;
template <> struct Pair2<float> { using T = float2; };
template <> struct Pair2<double> { using T = double2; };

// a where m is all ones, b where it is zero (a select on the bits: a plain
// select between two ring slots lets the compiler select their addresses
// and keep the ring in scratch memory)
__device__ inline float ms_pick(uint64_t m, float a, float b) {
  return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, a) & (uint32_t)m) |
                                       (__builtin_bit_cast(uint32_t, b) & ~(uint32_t)m));
}
__device__ inline double ms_pick(uint64_t m, double a, double b) {
  return __builtin_bit_cast(double, (__builtin_bit_cast(uint64_t, a) & m) | (__builtin_bit_cast(uint64_t, b) & ~m));
}

// d: this wave's direction pair (wave-uniform; one copy of the code serves
// every wave, so that no wave holds another's values)
template <class R, int NI, int MS_RING, int SCH>
__device__ inline void ms_march(const Tables& T, const R* __restrict__ f, R* __restrict__ out,
                                const R* __restrict__ ghost, int d, int j0, int i0, int i1,
                                double* lds) {
  constexpr int NQM = nq_of<NI>(), NH = NI / 2, NV = 2 * NK;
  const int nr = T.nr, nth = T.nth;
  const size_t plane = (size_t)nr * nth;
  const int lane = threadIdx.x & 63, j = j0 + lane;
  auto qv = [&](int v) { return 1 + NI * (v >> 1) + d + NH * (v & 1); };   // v = 2 (k-1) + h
  const double cd = dirs<NI>().c[d], sd = dirs<NI>().s[d];
  const double ct = T.cth[j], st = T.sth[j];
  const double vr = cd * ct + sd * st, vt = sd * ct - cd * st;   // per unit speed, direction d
  const R ar = (R)(fabs(vr) * T.dt_dr), at0 = (R)(fabs(vt) * T.dt_dth);
  const double e = T.e, ome = 1.0 - T.e;
  // per member h (direction d, then d + N_i/2, whose components are negated)
  uint64_t rm[2];
  int a1[2], a2[2], eb[2], dn[2], ebd[2];
  bool e1[2], e2[2], ed[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double svr = h ? -vr : vr, svt = h ? -vt : vt;
    rm[h] = svr >= 0.0 ? ~0ull : 0ull;      // radially upwind-backward
    const bool tb = svt >= 0.0;             // azimuthally upwind-backward
    const int sc = tb ? -1 : 1;
    a1[h] = (lane + sc) & 63;
    a2[h] = (lane + 2 * sc) & 63;
    eb[h] = tb ? 0 : 8;
    e1[h] = tb ? lane == 0 : lane == 63;
    e2[h] = tb ? lane == 1 : lane == 62;
    // the downwind neighbour (Lax-Wendroff only): the other adjacent lane,
    // the halo of the other side at the strip's downwind end
    dn[h] = (lane - sc) & 63;
    ebd[h] = tb ? 8 : 0;
    ed[h] = tb ? lane == 63 : lane == 0;
  }
  const bool left_lane = (lane & 15) < 8;
  auto load = [&](int v, int row) -> R {
    if (row < 0) return ghost[gidx(0, -1 - row, qv(v), j, nth, NQM)];
    if (row >= nr) return ghost[gidx(1, row - nr, qv(v), j, nth, NQM)];
    return f[qv(v) * plane + (size_t)row * nth + j];
  };
  auto halo = [&](int row) -> typename Pair2<R>::T {
    const int hl = lane & 15, v = hl & 7;
    int c = hl < 8 ? j0 - 2 : j0 + 64;
    c = c < 0 ? c + nth : (c >= nth ? c - nth : c);
    return *reinterpret_cast<const typename Pair2<R>::T*>(f + qv(v) * plane + (size_t)row * nth + c);
  };
  R S[MS_RING][NV];
  const int last = i1 + 1;   // the furthest row any update of the chunk reads
#pragma unroll
  for (int s = 0; s < MS_RING; ++s) {
    const int row = i0 - 2 + s;
#pragma unroll
    for (int v = 0; v < NV; ++v) S[s][v] = row <= last ? load(v, row) : (R)0;
  }
  const bool rest = d == 0;   // wave 0 also owns the rest velocity
  double r0 = 0.0;
  if (rest) r0 = (double)f[(size_t)i0 * nth + j];
  auto hv = halo(i0);
  for (int ib = i0; ib < i1; ib += MS_RING) {
#pragma unroll
    for (int u = 0; u < MS_RING; ++u) {
      const int i = ib + u;
      if (i >= i1) break;
      auto slot = [&](int sl, int v) -> R { return S[(u + sl) % MS_RING][v]; };
      const auto hcur = hv;
      if (i + 1 < i1) hv = halo(i + 1);
      double rcur = r0;
      if (rest && i + 1 < i1) r0 = (double)f[(size_t)(i + 1) * nth + j];
      // pair partials, exchanged through LDS: buf[(p * 4 + a) * 64 + lane],
      // the rest value at buf[NH * 4 * 64 + lane]
      double* buf = lds + (i & 1) * ((NH * 4 + 1) * 64);
      {
        double fp[NK], fm[NK], P[4];
#pragma unroll
        for (int k = 1; k <= NK; ++k) {
          fp[k - 1] = (double)slot(2, 2 * (k - 1));
          fm[k - 1] = (double)slot(2, 2 * (k - 1) + 1);
        }
        pair_partial<NI>(d, fp, fm, P);
#pragma unroll
        for (int a = 0; a < 4; ++a) buf[(d * 4 + a) * 64 + lane] = P[a];
      }
      if (rest) buf[NH * 4 * 64 + lane] = rcur;
      __syncthreads();
      rcur = buf[NH * 4 * 64 + lane];
      double r = 0.0, jx = 0.0, jy = 0.0, eps = 0.0;
      // (not unrolled: all N_i/2 partials in flight at once would take
      // 4 N_i registers)
#pragma unroll 1
      for (int p = 0; p < NH; ++p) {
        r += buf[(p * 4 + 0) * 64 + lane];
        jx += buf[(p * 4 + 1) * 64 + lane];
        jy += buf[(p * 4 + 2) * 64 + lane];
        eps += buf[(p * 4 + 3) * 64 + lane];
      }
      double rho, ux, uy, E;
      moments_from_sums(r, jx, jy, eps, rcur, rho, ux, uy, E);
      EqCoef ec;
      eq_models<NI>(rho, ux, uy, E, ec);
      const size_t c0 = (size_t)i * nth + j;
      if (rest) out[c0] = relax_rest<R>(relax_rest_share(ec, ome), e, rcur);
      // halo by role: H1 the column next to the strip (j0 - 1 / j0 + 64), H2
      // the one beyond it (j0 - 2 / j0 + 65)
      const R H1 = left_lane ? hcur.y : hcur.x, H2 = left_lane ? hcur.x : hcur.y;
      const R rinv = (R)T.rinv[i];
      const R at = at0 * rinv;
      const double pd = ux * cd + uy * sd;
      for_k<1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int v0 = 2 * (k - 1);
        double rel[2];
        relax_pair<k>(ec, e, ome, pd, (double)slot(2, v0), (double)slot(2, v0 + 1), rel[0], rel[1]);
        R aCr, Kr, aCt, Kt;
        courant<R>((R)speed(k), ar, aCr, Kr);
        courant<R>((R)speed(k), at, aCt, Kt);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int v = v0 + h;
          const R c = slot(2, v);
          const R u1r = ms_pick(rm[h], slot(1, v), slot(3, v));
          const R u2r = ms_pick(rm[h], slot(0, v), slot(4, v));
          const R z1 = __shfl(c, a1[h]), z2 = __shfl(c, a2[h]);
          const R g1 = __shfl(H1, eb[h] + v), g2 = __shfl(H2, eb[h] + v);
          const R u1t = e1[h] ? g1 : z1;
          const R u2t = e1[h] ? g2 : (e2[h] ? g1 : z2);
          R w1r = c, w1t = c;
          if constexpr (SCH == SCH_LW) {
            w1r = ms_pick(rm[h], slot(3, v), slot(1, v));
            const R zd = __shfl(c, dn[h]), gd = __shfl(H1, ebd[h] + v);
            w1t = ed[h] ? gd : zd;
          }
          const R tr = conv_term<SCH, R>(aCr, Kr, c, u1r, u2r, w1r);
          const R tt = conv_term<SCH, R>(aCt, Kt, c, u1t, u2t, w1t);
          out[qv(v) * plane + c0] = (R)((rel[h] - (double)tr) - (double)tt);
        }
      });
      // look-ahead: row i + MS_RING - 2 into the slot of row i - 2
      const int row = i + MS_RING - 2;
      if (row <= last) {
#pragma unroll
        for (int v = 0; v < NV; ++v) S[u % MS_RING][v] = load(v, row);
      }
    }
  }
}

template <class R, int NI, int RING, int SCH>
__global__ void __launch_bounds__(64 * (NI / 2))
models_strip_kernel(Tables T, const R* __restrict__ f, R* __restrict__ out,
                    const R* __restrict__ ghost, int chunk) {
  __shared__ double lds[2 * ((NI / 2) * 4 + 1) * 64];
  const int nstrip = T.nth / 64;
  const int item = strip::work_item(1);
  const int strip_i = item % nstrip, ck = item / nstrip;
  const int j0 = strip_i * 64;
  const int i0 = ck * chunk, i1 = min(i0 + chunk, T.nr);
  ms_march<R, NI, RING, SCH>(T, f, out, ghost, __builtin_amdgcn_readfirstlane(threadIdx.x / 64), j0, i0,
                             i1, lds);
}

}  // namespace

template <class R>
hipError_t launch_models_ghost(const Tables& T, int ni, const BCdev& bc, const void* f, void* ghost,
                               hipStream_t s) {
  const dim3 grid((T.nth + 255) / 256, 2);
  if (ni == 16)
    hipLaunchKernelGGL((models_ghost_kernel<R, 16>), grid, dim3(256), 0, s, T, bc, (const R*)f, (R*)ghost);
  else
    hipLaunchKernelGGL((models_ghost_kernel<R, 24>), grid, dim3(256), 0, s, T, bc, (const R*)f, (R*)ghost);
  return hipGetLastError();
}

template <class R, int NI, int SCH>
void launch_models_step_sch(const Tables& T, dim3 grid, const R* f, R* out, const R* gh, hipStream_t s) {
  if (T.nf == NI)
    hipLaunchKernelGGL((models_step_kernel<R, NI, SCH, false>), grid, dim3(256), 0, s, T, f, out, gh);
  else
    hipLaunchKernelGGL((models_step_kernel<R, NI, SCH, true>), grid, dim3(256), 0, s, T, f, out, gh);
}

template <class R, int NI>
void launch_models_step_ni(const Tables& T, dim3 grid, const R* f, R* out, const R* gh, hipStream_t s) {
  switch (T.scheme) {
    case SCH_WB: launch_models_step_sch<R, NI, SCH_WB>(T, grid, f, out, gh, s); break;
    case SCH_LW: launch_models_step_sch<R, NI, SCH_LW>(T, grid, f, out, gh, s); break;
    case SCH_UPWIND2: launch_models_step_sch<R, NI, SCH_UPWIND2>(T, grid, f, out, gh, s); break;
    default: launch_models_step_sch<R, NI, SCH_MWB>(T, grid, f, out, gh, s);
  }
}

// The strip form serves the double octagon (six-row ring) and float states of
// the triple octagon, whose twelve waves per workgroup must fit in 168
// registers each: with a five-row ring (the look-ahead row issued one row
// before its first use) the float form does; the double form spills.
bool models_strip_supported(const Tables& T, int ni, int precision) {
  // every scheme: the ring holds both radial sides and the halo both
  // azimuthal ones
  return (ni == 16 || (ni == 24 && precision == 32)) && T.nf == ni && T.nth >= 64 && T.nth % 64 == 0;
}

template <class R, int NI, int RING>
void launch_models_strip_sch(const Tables& T, dim3 grid, const R* f, R* out, const R* gh, int chunk,
                             hipStream_t s) {
  const dim3 block(64 * (NI / 2));
  switch (T.scheme) {
    case SCH_WB:
      hipLaunchKernelGGL((models_strip_kernel<R, NI, RING, SCH_WB>), grid, block, 0, s, T, f, out, gh, chunk);
      break;
    case SCH_LW:
      hipLaunchKernelGGL((models_strip_kernel<R, NI, RING, SCH_LW>), grid, block, 0, s, T, f, out, gh, chunk);
      break;
    case SCH_UPWIND2:
      hipLaunchKernelGGL((models_strip_kernel<R, NI, RING, SCH_UPWIND2>), grid, block, 0, s, T, f, out, gh,
                         chunk);
      break;
    default:
      hipLaunchKernelGGL((models_strip_kernel<R, NI, RING, SCH_MWB>), grid, block, 0, s, T, f, out, gh, chunk);
  }
}

template <class R>
hipError_t launch_models_step(const Tables& T, int ni, const void* f, void* out, const void* ghost,
                              const StripTune& tune, bool strip, hipStream_t s) {
  constexpr int prec = std::is_same<R, float>::value ? 32 : 64;
  if (strip && models_strip_supported(T, ni, prec)) {
    int chunk = tune.chunk > 0 ? tune.chunk : 32;
    const int strips = T.nth / 64;
    while (tune.chunk <= 0 && chunk > 8 && (long)strips * ((T.nr + chunk - 1) / chunk) < 4096) chunk /= 2;
    const dim3 grid(strips * ((T.nr + chunk - 1) / chunk));
    if (ni == 16)
      launch_models_strip_sch<R, 16, 6>(T, grid, (const R*)f, (R*)out, (const R*)ghost, chunk, s);
    else if constexpr (prec == 32)
      launch_models_strip_sch<R, 24, 5>(T, grid, (const R*)f, (R*)out, (const R*)ghost, chunk, s);
    return hipGetLastError();
  }
  const dim3 grid((T.nth + 255) / 256, T.nr);
  if (ni == 16) launch_models_step_ni<R, 16>(T, grid, (const R*)f, (R*)out, (const R*)ghost, s);
  else launch_models_step_ni<R, 24>(T, grid, (const R*)f, (R*)out, (const R*)ghost, s);
  return hipGetLastError();
}

template <class R>
hipError_t launch_models_init(const Tables& T, int ni, const double* rho, const double* ur,
                              const double* ut, const double* Tt, void* f, int* bad, hipStream_t s) {
  const dim3 grid((T.nth + 255) / 256, T.nr);
  if (ni == 16)
    hipLaunchKernelGGL((models_init_kernel<R, 16>), grid, dim3(256), 0, s, T, rho, ur, ut, Tt, (R*)f, bad);
  else
    hipLaunchKernelGGL((models_init_kernel<R, 24>), grid, dim3(256), 0, s, T, rho, ur, ut, Tt, (R*)f, bad);
  return hipGetLastError();
}

template <class R>
hipError_t launch_models_fields(const Tables& T, int ni, const void* f, double* rho, double* ur,
                                double* ut, double* Tt, hipStream_t s) {
  const dim3 grid((T.nth + 255) / 256, T.nr);
  if (ni == 16)
    hipLaunchKernelGGL((models_fields_kernel<R, 16>), grid, dim3(256), 0, s, T, (const R*)f, rho, ur, ut, Tt);
  else
    hipLaunchKernelGGL((models_fields_kernel<R, 24>), grid, dim3(256), 0, s, T, (const R*)f, rho, ur, ut, Tt);
  return hipGetLastError();
}

template <class R>
hipError_t launch_models_diag(const Tables& T, int ni, const void* f, double* partial, double step,
                              double* out, hipStream_t s) {
  const int nb = diag_blocks();
  if (ni == 16)
    hipLaunchKernelGGL((models_diag_kernel<R, 16>), dim3(nb), dim3(DIAG_BLOCK), 0, s, T, (const R*)f, partial);
  else
    hipLaunchKernelGGL((models_diag_kernel<R, 24>), dim3(nb), dim3(DIAG_BLOCK), 0, s, T, (const R*)f, partial);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_diag_final(partial, nb, step, out, s);
}

#define PCLB_INST(R)                                                                               \
  template hipError_t launch_models_ghost<R>(const Tables&, int, const BCdev&, const void*, void*, \
                                             hipStream_t);                                         \
  template hipError_t launch_models_step<R>(const Tables&, int, const void*, void*, const void*,   \
                                            const StripTune&, bool, hipStream_t);                  \
  template hipError_t launch_models_init<R>(const Tables&, int, const double*, const double*,      \
                                            const double*, const double*, void*, int*, hipStream_t); \
  template hipError_t launch_models_fields<R>(const Tables&, int, const void*, double*, double*,   \
                                              double*, double*, hipStream_t);                      \
  template hipError_t launch_models_diag<R>(const Tables&, int, const void*, double*, double,      \
                                            double*, hipStream_t);
PCLB_INST(float)
PCLB_INST(double)
#undef PCLB_INST

}  // namespace pclb
