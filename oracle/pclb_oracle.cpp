// Plain FP64 reference implementation (the "oracle") of the polar-coordinate
// finite-difference lattice Boltzmann step of Lin, Xu, Zhang, Li and Succi,
// "Polar coordinate lattice Boltzmann modeling of compressible flows"
// (arXiv:1302.7104): analytic BGK relaxation plus Modified Warming-Beam
// (MWB) convection, combined additively from the state at time t.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg load this library.  The product path (the HIP
// library) never links, loads or calls it, and the two share no code, header,
// table or constant generator.
//
// Style: slow, plain loops in double precision, each function following one
// passage of the paper in the paper's order and notation.  OpenMP is used only
// to spread independent rows / velocity planes over host cores.
//
// Layout of every distribution array exchanged with the caller: f[q][i][j],
// q = 0..32 the discrete velocity, i = 0..nr-1 the radial node, j = 0..nth-1
// the azimuthal node (fastest).  Field arrays are [i][j].
//
// Velocity numbering: q = 0 is the rest velocity (speed group k = 0); for
// k = 1..4 and direction i = 1..8, q = 1 + 8(k-1) + (i-1).
//
// Readings of the paper that this file takes (each one is listed with its
// evidence in the design notes of the repository):
//  * velocities are fixed in the Cartesian frame; their polar components at
//    angle theta are v_r = v_x cos(theta) + v_y sin(theta) and
//    v_theta = -v_x sin(theta) + v_y cos(theta);
//  * full annulus (N_f = N_i = 8): the azimuthal ghost copy keeps the
//    velocity index unchanged;
//  * nodes r_i = R1 + i dr (i = 0..nr-1, dr = (R2-R1)/(nr-1)) and
//    theta_j = (j+1) dtheta (dtheta = 2 pi / nth);
//  * the combined scheme evaluates all three terms from f at time t;
//  * the MWB bracket uses (1 - |C|) and is evaluated in the division-free form
//    of the switch, which is 0 when both upwind differences vanish; C = 0
//    counts as C >= 0;
//  * radial ghost nodes hold the equilibrium of linearly extrapolated density
//    and temperature; the velocity there is set per boundary kind.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int NK = 4;             // non-zero speed groups (Sec. II.A)
constexpr int NI = 8;             // directions per group, octagon model
constexpr int NQ = 1 + NK * NI;   // 33 discrete velocities of the octagon
constexpr int NQ_MAX = 1 + NK * 24;   // 97: the triple octagon
constexpr double PI = 3.14159265358979323846;

// Speeds v_0..v_4 (Sec. II.A, after Eq. DVM1).
const double VK[NK + 1] = {0.0, 1.0, 2.92, 2.99, 4.49};

// Table I: (N_i, B0, B1, B2, B3, B4) for the octagon, double and triple octagon.
struct TableRow { int ni; double b0, b1, b2, b3, b4; };
const TableRow TABLE1[3] = {
    {8, 8.0, -0.25, 1.0, -6.0, 48.0},
    {16, 16.0, -1.0 / 8.0, 0.5, -3.0, 24.0},
    {24, 24.0, -1.0 / 12.0, 1.0 / 3.0, -2.0, 16.0},
};

// Eq. DVM1 for N_i directions per speed (8 octagon, 16 double, 24 triple
// octagon): v_kix = v_k cos[2 pi (i-1)/N_i], v_kiy = v_k sin[...];
// q = 1 + N_i (k-1) + (i-1), q = 0 the rest velocity.
struct Velocities {
  int ni, nq;
  double vx[NQ_MAX], vy[NQ_MAX];
  int k[NQ_MAX];
  explicit Velocities(int n) : ni(n), nq(1 + NK * n) {
    vx[0] = 0.0; vy[0] = 0.0; k[0] = 0;
    for (int kk = 1; kk <= NK; ++kk)
      for (int i = 1; i <= ni; ++i) {
        int q = 1 + ni * (kk - 1) + (i - 1);
        double phi = 2.0 * PI * (i - 1) / ni;
        vx[q] = VK[kk] * std::cos(phi);
        vy[q] = VK[kk] * std::sin(phi);
        k[q] = kk;
      }
  }
};
const Velocities VELS[3] = {Velocities(8), Velocities(16), Velocities(24)};
// the model of a grid (its N_i) and its Table I row
inline const Velocities& vel_of(int ni) { return ni == 24 ? VELS[2] : ni == 16 ? VELS[1] : VELS[0]; }
inline const TableRow& row_of(int ni) { return ni == 24 ? TABLE1[2] : ni == 16 ? TABLE1[1] : TABLE1[0]; }
// the octagon, for the node-level helpers that take no grid
const Velocities& V = VELS[0];

// ---------------------------------------------------------------------------
// Forward-mode dual numbers, used only to differentiate the equilibrium and
// the MWB term for the adjoint.  abs() uses sgn(0) = 0.
template <int N> struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int n = 0; n < N; ++n) d[n] = 0; }
  Dual(double x) : v(x) { for (int n = 0; n < N; ++n) d[n] = 0; }
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int n = 0; n < N; ++n) r.d[n] = a.d[n] + b.d[n]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int n = 0; n < N; ++n) r.d[n] = a.d[n] - b.d[n]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int n = 0; n < N; ++n) r.d[n] = -a.d[n]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int n = 0; n < N; ++n) r.d[n] = a.d[n] * b.v + a.v * b.d[n]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int n = 0; n < N; ++n) r.d[n] = (a.d[n] * b.v - a.v * b.d[n]) / (b.v * b.v);
  return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N> dabs(const Dual<N>& a) {
  double s = a.v > 0 ? 1.0 : (a.v < 0 ? -1.0 : 0.0);
  Dual<N> r; r.v = std::fabs(a.v); for (int n = 0; n < N; ++n) r.d[n] = s * a.d[n]; return r; }
inline double dabs(double a) { return std::fabs(a); }
inline double val(double a) { return a; }
template <int N> double val(const Dual<N>& a) { return a.v; }

// ---------------------------------------------------------------------------
// Eq. mod: mod{a,b} = a if a <= b, else a - b.
inline int modab(int a, int b) { return a <= b ? a : a - b; }

// Eqs. F_k (Sec. II.A) with the Table I row of the chosen model:
//   F_k = [B4 E^4 + B3 (x_{k+1}+x_{k+2}+x_{k+3}) E^3
//          + B2 (x_{k+1}x_{k+2} + x_{k+2}x_{k+3} + x_{k+3}x_{k+1}) E^2
//          + B1 x_{k+1}x_{k+2}x_{k+3} E]
//         / [x_k (x_k - x_{k+1})(x_k - x_{k+2})(x_k - x_{k+3})],  x = v^2,
//   F_0 = 1 - B0 (F_1 + F_2 + F_3 + F_4).
template <class T> void weights(const T& E, const TableRow& tb, T F[NK + 1]) {
  double x[NK + 1];
  for (int k = 0; k <= NK; ++k) x[k] = VK[k] * VK[k];
  T sum = T(0.0);
  for (int k = 1; k <= NK; ++k) {
    int k1 = modab(k + 1, NK), k2 = modab(k + 2, NK), k3 = modab(k + 3, NK);
    double den = x[k] * (x[k] - x[k1]) * (x[k] - x[k2]) * (x[k] - x[k3]);
    T E2 = E * E, E3 = E2 * E, E4 = E3 * E;
    T num = tb.b4 * E4 + tb.b3 * (x[k1] + x[k2] + x[k3]) * E3 +
            tb.b2 * (x[k1] * x[k2] + x[k2] * x[k3] + x[k3] * x[k1]) * E2 +
            tb.b1 * (x[k1] * x[k2] * x[k3]) * E;
    F[k] = num / den;
    sum = sum + F[k];
  }
  F[0] = 1.0 - tb.b0 * sum;
}

// Eq. feq: the polynomial equilibrium of velocity q of the set W for
// (rho, u, E), with the weights F of W's Table I row.
template <class T>
T feq_q(const Velocities& W, const T& rho, const T& ux, const T& uy, const T& E,
        const T F[NK + 1], int q) {
  T u2 = ux * ux + uy * uy;
  T w = W.vx[q] * ux + W.vy[q] * uy;          // v_ki . u
  T one_m = 1.0 - u2 / (2.0 * E);             // (1 - u^2 / 2E)
  T E2 = E * E;
  T br = (1.0 - u2 / (2.0 * E) + (u2 * u2) / (8.0 * E2))
       + (w / E) * one_m
       + ((w * w) / (2.0 * E2)) * one_m
       + (w * w * w) / (6.0 * E2 * E)
       + (w * w * w * w) / (24.0 * E2 * E2);
  return rho * F[W.k[q]] * br;
}
template <class T>
T feq_q(const T& rho, const T& ux, const T& uy, const T& E, const T F[NK + 1], int q) {
  return feq_q(V, rho, ux, uy, E, F, q);
}

template <class T>
void feq_all(const Velocities& W, const T& rho, const T& ux, const T& uy, const T& E, T* out) {
  T F[NK + 1];
  weights(E, row_of(W.ni), F);
  for (int q = 0; q < W.nq; ++q) out[q] = feq_q(W, rho, ux, uy, E, F, q);
}
template <class T>
void feq_all(const T& rho, const T& ux, const T& uy, const T& E, T* out) {
  feq_all(V, rho, ux, uy, E, out);
}

// Eqs. moment1-moment3: rho = sum f, rho u = sum f v,
// rho E = sum (1/2) f (v - u).(v - u), over the velocity set W.
void macros(const Velocities& W, const double* f, double& rho, double& ux, double& uy, double& E) {
  rho = 0; double jx = 0, jy = 0;
  for (int q = 0; q < W.nq; ++q) { rho += f[q]; jx += f[q] * W.vx[q]; jy += f[q] * W.vy[q]; }
  ux = jx / rho; uy = jy / rho;
  double e2 = 0;
  for (int q = 0; q < W.nq; ++q) {
    double cx = W.vx[q] - ux, cy = W.vy[q] - uy;
    e2 += 0.5 * f[q] * (cx * cx + cy * cy);
  }
  E = e2 / rho;
}
void macros(const double* f, double& rho, double& ux, double& uy, double& E) {
  macros(V, f, rho, ux, uy, E);
}

// The same macroscopic fields written as a function of the four linear
// moments M = (rho, rho u_x, rho u_y, sum (1/2) f v.v); used to differentiate.
template <class T> void macros_of_M(const T M[4], T& rho, T& ux, T& uy, T& E) {
  rho = M[0]; ux = M[1] / rho; uy = M[2] / rho;
  E = M[3] / rho - 0.5 * (ux * ux + uy * uy);
}

// Sec. II.B, Eqs. WB_Scheme_2 / MWB Scheme.  With the upwind difference
// delta (backward when C >= 0, forward otherwise), the next one upwind
// delta' = eta delta, and S(eta) = (|eta| - 1)/(|eta| + 1), the scheme
// subtracts [C + (1/2) C (1-|C|)(1-S(eta))(1-eta)] delta.  Since
//   (1/2)(1 - S(eta))(1 - eta) delta = (delta - delta') |delta| / (|delta| + |delta'|)
// for every delta != 0, the term is evaluated in that division-free form, with
// the ratio taken as 0 when |delta| + |delta'| = 0 (the limit delta -> 0 of the
// eta-form, whose whole bracket then multiplies a vanishing delta).  This is
// the one canonical form of the switch: the eta-form loses digits in
// 1 - S(eta) when |eta| >> 1.  psi holds psi_{j-2..j+2}.  s_mode = 1 replaces
// S by 0, which turns the bracket into the plain Warming-Beam one:
// C delta + (1/2) C (1-|C|)(delta - delta').
template <class T> void upwind_differences(double C, const T psi[5], T& delta, T& dprime) {
  if (C >= 0) { delta = psi[2] - psi[1]; dprime = psi[1] - psi[0]; }
  else        { delta = psi[3] - psi[2]; dprime = psi[4] - psi[3]; }
}

template <class T> T mwb_term(double C, const T psi[5], int s_mode) {
  T delta, dprime;
  upwind_differences(C, psi, delta, dprime);
  const double K = C * (1.0 - std::fabs(C));
  if (s_mode) return C * delta + 0.5 * K * (delta - dprime);
  T den = dabs(delta) + dabs(dprime);
  if (val(den) == 0.0) return T(0.0);
  return C * delta + K * ((delta - dprime) * dabs(delta) / den);
}

// The same term written with eta and S(eta) exactly as printed (0 when
// delta = 0).  Kept only to pin the division-free form against the printed one.
double mwb_term_eta(double C, const double psi[5]) {
  double delta, dprime;
  upwind_differences(C, psi, delta, dprime);
  if (delta == 0.0) return 0.0;
  double eta = dprime / delta;
  double S = (std::fabs(eta) - 1.0) / (std::fabs(eta) + 1.0);
  return (C + 0.5 * C * (1.0 - std::fabs(C)) * (1.0 - S) * (1.0 - eta)) * delta;
}

// The convection term T = psi_j^n - psi_j^{n+1} of one sweep for each scheme
// the paper compares (Sec. II.B; Sec. III.A, Figs. 5 and 6), psi holding
// psi_{j-2..j+2}:
//  0 MWB: Eq. MWB Scheme (mwb_term);
//  1 Warming-Beam, Eq. WB_Scheme_1 as printed;
//  2 Lax-Wendroff: Eq. Taylor expansion with both derivatives taken by
//    central differences (the paper names the scheme without printing it);
//  3 second-order upwind: Eq. Taylor expansion cut after the first-order
//    term, the derivative from Eq. upwind scheme_1 (forward Euler in time).
double convection_term(int scheme, double C, const double psi[5]) {
  const double pm2 = psi[0], pm1 = psi[1], p0 = psi[2], pp1 = psi[3], pp2 = psi[4];
  switch (scheme) {
    case 1:
      if (C >= 0) return C * (p0 - pm1) + 0.5 * C * (1.0 - C) * (p0 - 2.0 * pm1 + pm2);
      return C * (pp1 - p0) - 0.5 * C * (1.0 + C) * (p0 - 2.0 * pp1 + pp2);
    case 2:
      return 0.5 * C * (pp1 - pm1) - 0.5 * C * C * (pp1 - 2.0 * p0 + pm1);
    case 3:
      if (C >= 0) return C * (3.0 * p0 - 4.0 * pm1 + pm2) / 2.0;
      return -C * (3.0 * p0 - 4.0 * pp1 + pp2) / 2.0;
    default:
      return mwb_term<double>(C, psi, 0);
  }
}

// Partial derivatives of mwb_term with respect to psi_{j-2..j+2}, written as
// derivatives of the term in (delta, delta') mapped back to the stencil.
//
// The term is not differentiable where delta or delta' vanishes.  The
// derivative convention (a reading: the paper has no adjoint):
//  * a difference whose size is at most tie_eps times the stencil's magnitude
//    |psi| summed over its three nodes counts as exactly zero, so that the
//    rounding of the state does not pick the branch (the caller passes the
//    threshold that suits the precision the state was computed in);
//  * sgn(0) = 0 inside |.|; with delta = 0 and delta' != 0 this gives
//    dh/d(delta) = dh/d(delta') = 0 for h = (delta - delta')|delta|/(|delta| + |delta'|),
//    the mean of the two one-sided derivatives (what a central difference
//    across the kink sees);
//  * with delta = delta' = 0, (dh/d(delta), dh/d(delta')) = (1, 0), the exact
//    one-sided derivative for a perturbation of any single stencil node.
// Elsewhere the derivatives come from forward-mode differentiation of the
// division-free form.
constexpr double KINK_H[2] = {1.0, 0.0};

void mwb_grad(double C, const double psi[5], double tie_eps, double g[5]) {
  for (int n = 0; n < 5; ++n) g[n] = 0;
  const bool back = C >= 0;
  double delta, dprime;
  upwind_differences(C, psi, delta, dprime);
  double mag = back ? std::fabs(psi[0]) + std::fabs(psi[1]) + std::fabs(psi[2])
                    : std::fabs(psi[2]) + std::fabs(psi[3]) + std::fabs(psi[4]);
  double thr = tie_eps * mag;
  if (std::fabs(delta) <= thr) delta = 0.0;
  if (std::fabs(dprime) <= thr) dprime = 0.0;
  double K = C * (1.0 - std::fabs(C));
  double dd, ddp;   // d term / d delta, d term / d delta'
  if (delta == 0.0) {
    double h1 = dprime == 0.0 ? KINK_H[0] : 0.0, h2 = dprime == 0.0 ? KINK_H[1] : 0.0;
    dd = C + K * h1;
    ddp = K * h2;
  } else {
    Dual<2> D(delta), Dp(dprime);
    D.d[0] = 1.0;
    Dp.d[1] = 1.0;
    Dual<2> h = (D - Dp) * dabs(D) / (dabs(D) + dabs(Dp));
    Dual<2> t = C * D + K * h;
    dd = t.d[0];
    ddp = t.d[1];
  }
  if (back) { g[2] += dd; g[1] += -dd + ddp; g[0] += -ddp; }
  else      { g[3] += dd - ddp; g[2] += -dd; g[4] += ddp; }
}

}  // namespace

// Grid, time step and radial boundary description.
//   bc_kind: 0 = WALL (p[0] = angular velocity omega; u = (0, omega r) at the
//   ghost nodes), 1 = INFLOW (p = rho, u_r, u_theta, T prescribed at the ghost
//   nodes), 2 = EXTRAPOLATE (u_r, u_theta extrapolated like rho and T).
//   side 0 = inner (r = R1), side 1 = outer (r = R2).
//   terms: bit 0 relaxation, bit 1 radial convection, bit 2 azimuthal
//   convection (7 = the combined scheme; other values only for tests).
struct OrGrid {
  int32_t nr, nth;
  double r1, r2, tau, dt;
  int32_t bc_kind[2];
  double bc_par[2][4];
  int32_t terms;
  int32_t nf;   // N_f: theta covers 0 < theta <= 2 pi N_f / N_i (N_i = 8; 8 = full annulus)
  int32_t scheme;  // convection: 0 MWB (Eq. MWB Scheme), 1 Warming-Beam (Eq. WB_Scheme_1),
                   // 2 Lax-Wendroff, 3 second-order upwind (Sec. II.B, Sec. III.A Figs. 5-6)
  int32_t relax;   // relaxation: 0 analytic (Eq. operator1_new), 1 forward Euler (Eq. operator1_old)
  int32_t ni;      // N_i: 8 octagon, 16 double, 24 triple octagon (Table I); 1 + 4 N_i velocities
};

namespace {

struct Geometry {
  int nr, nth;
  double dr, dth;
  std::vector<double> r, ct, st;
  explicit Geometry(const OrGrid& g) : nr(g.nr), nth(g.nth) {
    dr = (g.r2 - g.r1) / (nr - 1);
    dth = 2.0 * PI * g.nf / (g.ni * (double)nth);   // Sec. II.C: 2 pi N_f / (N_i N_theta)
    r.resize(nr + 4);                      // r of rows -2..nr+1
    for (int i = -2; i < nr + 2; ++i) r[i + 2] = g.r1 + i * dr;
    ct.resize(nth); st.resize(nth);
    for (int j = 0; j < nth; ++j) {
      double th = (j + 1) * dth;
      ct[j] = std::cos(th); st[j] = std::sin(th);
    }
  }
  double rr(int i) const { return r[i + 2]; }
};

// Ghost-padded copy of one step's distribution: rows -2..nr+1, cols -2..nth+1.
struct Padded {
  int nr, nth, W, H;
  std::vector<double> a;
  Padded(int nr_, int nth_, int nq) : nr(nr_), nth(nth_), W(nth_ + 4), H(nr_ + 4),
                                      a((size_t)nq * (nr_ + 4) * (nth_ + 4), 0.0) {}
  double& at(int q, int i, int j) { return a[((size_t)q * H + (i + 2)) * W + (j + 2)]; }
  double at(int q, int i, int j) const { return a[((size_t)q * H + (i + 2)) * W + (j + 2)]; }
};

inline size_t idx(const OrGrid& g, int q, int i, int j) {
  return ((size_t)q * g.nr + i) * g.nth + j;
}

// The relaxation of one value over a step (Sec. II.B): Eq. operator1_new
// (relax = 0) or Eq. operator1_old (relax = 1).
double relax_value(const OrGrid& g, double f, double feq) {
  if (g.relax == 1) return f - g.dt / g.tau * (f - feq);
  return feq + (f - feq) * std::exp(-g.dt / g.tau);
}

// mod{a, b} of Sec. II.B: a for a <= b, a - b above (a in 1..2b).
inline int paper_mod(int a, int b) { return a <= b ? a : a - b; }

// Sec. II.C, azimuthal boundary condition (Fig. 3): the distribution of
// velocity q at column jv, where jv may lie up to two columns outside
// 0..nth-1, is that of column jv + nth with direction index mod{i + N_f, N_i}
// (jv < 0), or of column jv - nth with mod{i - N_f + N_i, N_i} (jv >= nth);
// i = 1..N_i is the paper's direction index, q = 1 + N_i (k - 1) + (i - 1).
// Sets the real column and the velocity read there.
void azimuthal_source(const OrGrid& g, int q, int jv, int& q_src, int& j_src) {
  const Velocities& VG = vel_of(g.ni);
  q_src = q;
  j_src = jv;
  if (jv >= 0 && jv < g.nth) return;
  int i_dir = q == 0 ? 0 : (q - 1) % VG.ni + 1;
  int i_src = i_dir;
  if (jv < 0) {
    j_src = jv + g.nth;
    if (q != 0) i_src = paper_mod(i_dir + g.nf, VG.ni);
  } else {
    j_src = jv - g.nth;
    if (q != 0) i_src = paper_mod(i_dir - g.nf + VG.ni, VG.ni);
  }
  if (q != 0) q_src = q - i_dir + i_src;
}

// Macroscopic fields (rho, u_x, u_y, E) of every real node.
void all_macros(const OrGrid& g, const double* f, std::vector<double>& m) {
  const Velocities& VG = vel_of(g.ni);
  m.assign((size_t)4 * g.nr * g.nth, 0.0);
  size_t n = (size_t)g.nr * g.nth;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < g.nr; ++i)
    for (int j = 0; j < g.nth; ++j) {
      double fl[NQ_MAX];
      for (int q = 0; q < VG.nq; ++q) fl[q] = f[idx(g, q, i, j)];
      size_t c = (size_t)i * g.nth + j;
      macros(VG, fl, m[c], m[n + c], m[2 * n + c], m[3 * n + c]);
    }
}

// Sec. II.C, radial boundary condition.  Given the macroscopic fields of the
// two real rows next to one wall, return (rho, u_x, u_y, E) at the two ghost
// rows.  rho and T (= E) are extrapolated linearly and recursively:
// rho(ghost1) = 2 rho(row0) - rho(row1), rho(ghost2) = 2 rho(ghost1) - rho(row0).
// The velocity follows the boundary kind.  T is used as E since gamma = 2.
template <class T>
void ghost_macros(const OrGrid& g, int side, double rg1, double rg2, double ct, double st,
                  const T m0[4], const T m1[4], T out1[4], T out2[4]) {
  // m0: row adjacent to the wall, m1: next row inward; each (rho, ux, uy, E).
  int kind = g.bc_kind[side] & 15;     // the NONEQ flag (16) does not change the state
  const double* p = g.bc_par[side];
  T rho1 = 2.0 * m0[0] - m1[0];
  T rho2 = 2.0 * rho1 - m0[0];
  T E1 = 2.0 * m0[3] - m1[3];
  T E2 = 2.0 * E1 - m0[3];
  T ur1, ut1, ur2, ut2;
  if (kind == 0) {            // WALL: u_r = 0, u_theta = omega r at the ghost node
    ur1 = T(0.0); ut1 = T(p[0] * rg1);
    ur2 = T(0.0); ut2 = T(p[0] * rg2);
  } else if (kind == 1) {     // INFLOW: everything prescribed
    rho1 = T(p[0]); rho2 = T(p[0]);
    ur1 = T(p[1]); ur2 = T(p[1]);
    ut1 = T(p[2]); ut2 = T(p[2]);
    E1 = T(p[3]); E2 = T(p[3]);
  } else {                    // EXTRAPOLATE: polar velocity components too
    T ur_0 = m0[1] * ct + m0[2] * st, ut_0 = -m0[1] * st + m0[2] * ct;
    T ur_1 = m1[1] * ct + m1[2] * st, ut_1 = -m1[1] * st + m1[2] * ct;
    ur1 = 2.0 * ur_0 - ur_1; ut1 = 2.0 * ut_0 - ut_1;
    ur2 = 2.0 * ur1 - ur_0;  ut2 = 2.0 * ut1 - ut_0;
  }
  out1[0] = rho1; out1[1] = ur1 * ct - ut1 * st; out1[2] = ur1 * st + ut1 * ct; out1[3] = E1;
  out2[0] = rho2; out2[1] = ur2 * ct - ut2 * st; out2[2] = ur2 * st + ut2 * ct; out2[3] = E2;
}

// Fill the padded array for one step: real nodes, the periodic azimuthal
// ghosts (Sec. II.C, azimuthal boundary condition: azimuthal_source) and the
// radial equilibrium ghosts.  Returns the number of ghost nodes whose
// extrapolated rho or T is not positive.
int build_padded(const OrGrid& g, const Geometry& geo, const double* f,
                 const std::vector<double>& m, Padded& P) {
  const Velocities& VG = vel_of(g.ni);
#pragma omp parallel for schedule(static)
  for (int q = 0; q < VG.nq; ++q)
    for (int i = 0; i < g.nr; ++i)
      for (int j = 0; j < g.nth; ++j) P.at(q, i, j) = f[idx(g, q, i, j)];
  // azimuthal ghosts: i_theta <= 0 takes i_theta + N_theta, i_theta > N_theta
  // takes i_theta - N_theta, each with its rotated direction index
  for (int q = 0; q < VG.nq; ++q)
    for (int i = 0; i < g.nr; ++i)
      for (int jv : {-2, -1, g.nth, g.nth + 1}) {
        int qs, js;
        azimuthal_source(g, q, jv, qs, js);
        P.at(q, i, jv) = f[idx(g, qs, i, js)];
      }
  const size_t n = (size_t)g.nr * g.nth;
  int bad = 0;
  for (int side = 0; side < 2; ++side) {
    int i0 = side == 0 ? 0 : g.nr - 1;     // row next to the wall
    int i1 = side == 0 ? 1 : g.nr - 2;     // next row inward
    int ig1 = side == 0 ? -1 : g.nr;       // first ghost row
    int ig2 = side == 0 ? -2 : g.nr + 1;   // second ghost row
    for (int j = 0; j < g.nth; ++j) {
      double m0[4], m1[4], o1[4], o2[4];
      for (int a = 0; a < 4; ++a) {
        m0[a] = m[a * n + (size_t)i0 * g.nth + j];
        m1[a] = m[a * n + (size_t)i1 * g.nth + j];
      }
      ghost_macros<double>(g, side, geo.rr(ig1), geo.rr(ig2), geo.ct[j], geo.st[j], m0, m1, o1, o2);
      if (!(o1[0] > 0) || !(o1[3] > 0) || !(o2[0] > 0) || !(o2[3] > 0)) ++bad;
      double fe1[NQ_MAX], fe2[NQ_MAX];
      feq_all(VG, o1[0], o1[1], o1[2], o1[3], fe1);
      feq_all(VG, o2[0], o2[1], o2[2], o2[3], fe2);
      // non-equilibrium boundary (flag 16): both ghost layers also take the
      // wall row's f - f^eq
      double fneq[NQ_MAX] = {0};
      if (g.bc_kind[side] & 16) {
        double fw[NQ_MAX], few[NQ_MAX];
        for (int q = 0; q < VG.nq; ++q) fw[q] = f[idx(g, q, i0, j)];
        feq_all(VG, m0[0], m0[1], m0[2], m0[3], few);
        for (int q = 0; q < VG.nq; ++q) fneq[q] = fw[q] - few[q];
      }
      for (int q = 0; q < VG.nq; ++q) {
        P.at(q, ig1, j) = fe1[q] + fneq[q];
        P.at(q, ig2, j) = fe2[q] + fneq[q];
      }
    }
  }
  return bad;
}

inline double vr_of(const Velocities& W, int q, double ct, double st) { return W.vx[q] * ct + W.vy[q] * st; }
inline double vt_of(const Velocities& W, int q, double ct, double st) { return -W.vx[q] * st + W.vy[q] * ct; }

}  // namespace

// ===========================================================================
// C ABI used by the Python test wrapper.
extern "C" {


int or_num_velocities() { return NQ; }

void or_velocities(double* vx, double* vy, int32_t* k) {
  for (int q = 0; q < NQ; ++q) { vx[q] = V.vx[q]; vy[q] = V.vy[q]; k[q] = V.k[q]; }
}

// F_0..F_4 for one of the three Table I rows (0 octagon, 1 double, 2 triple).
void or_weights(double E, int32_t row, double* F) {
  double Fl[NK + 1];
  weights(E, TABLE1[row], Fl);
  for (int k = 0; k <= NK; ++k) F[k] = Fl[k];
}

void or_feq(double rho, double ux, double uy, double E, double* out) {
  feq_all(rho, ux, uy, E, out);
}

// out = (rho, u_x, u_y, E) of one node.
void or_macros(const double* f, double* out) {
  macros(f, out[0], out[1], out[2], out[3]);
}

// Analytic relaxation of one node (Eq. operator1_new) over a step dt.
void or_relax_node(const double* f, double dt, double tau, double* out) {
  double rho, ux, uy, E, fe[NQ];
  macros(f, rho, ux, uy, E);
  feq_all(rho, ux, uy, E, fe);
  double e = std::exp(-dt / tau);
  for (int q = 0; q < NQ; ++q) out[q] = fe[q] + (f[q] - fe[q]) * e;
}

double or_mwb_term(double C, const double* psi, int32_t s_mode) {
  return mwb_term<double>(C, psi, s_mode);
}

double or_mwb_term_eta(double C, const double* psi) { return mwb_term_eta(C, psi); }

double or_convection_term(int32_t scheme, double C, const double* psi) {
  return convection_term(scheme, C, psi);
}

void or_mwb_grad(double C, const double* psi, double tie_eps, double* g) {
  mwb_grad(C, psi, tie_eps, g);
}


// Eq. combined_scheme applied nsteps times: f_out = f after nsteps steps.
// f_in and f_out may alias.  Returns the number of ghost nodes that had a
// non-positive extrapolated density or temperature (0 in a healthy run).
int or_step(const OrGrid* gp, const double* f_in, double* f_out, int32_t nsteps) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
  size_t tot = (size_t)VG.nq * g.nr * g.nth;
  std::vector<double> cur(f_in, f_in + tot), m;
  Padded P(g.nr, g.nth, VG.nq);
  int bad = 0;
  for (int s = 0; s < nsteps; ++s) {
    all_macros(g, cur.data(), m);                 // moments of every real node
    bad += build_padded(g, geo, cur.data(), m, P);  // theta ghosts, radial ghosts
    size_t n = (size_t)g.nr * g.nth;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < g.nr; ++i) {
      double r = geo.rr(i);
      for (int j = 0; j < g.nth; ++j) {
        size_t c = (size_t)i * g.nth + j;
        double fe[NQ_MAX];
        feq_all(VG, m[c], m[n + c], m[2 * n + c], m[3 * n + c], fe);
        for (int q = 0; q < VG.nq; ++q) {
          double ft = P.at(q, i, j);
          double out = 0.0;
          if (g.terms & 1) out += relax_value(g, ft, fe[q]);   // Eqs. operator1_new / _old
          else out += ft;
          double Cr = vr_of(VG, q, geo.ct[j], geo.st[j]) * g.dt / geo.dr;
          double Ct = vt_of(VG, q, geo.ct[j], geo.st[j]) * g.dt / (r * geo.dth);
          if (g.terms & 2) {
            double psi[5] = {P.at(q, i - 2, j), P.at(q, i - 1, j), ft, P.at(q, i + 1, j), P.at(q, i + 2, j)};
            out -= convection_term(g.scheme, Cr, psi);
          }
          if (g.terms & 4) {
            double psi[5] = {P.at(q, i, j - 2), P.at(q, i, j - 1), ft, P.at(q, i, j + 1), P.at(q, i, j + 2)};
            out -= convection_term(g.scheme, Ct, psi);
          }
          f_out[idx(g, q, i, j)] = out;
        }
      }
    }
#pragma omp parallel for schedule(static)
    for (int q = 0; q < VG.nq; ++q) {
      const size_t b = (size_t)q * g.nr * g.nth, e = b + (size_t)g.nr * g.nth;
      std::copy(f_out + b, f_out + e, cur.begin() + b);
    }
  }
  if (nsteps == 0) std::copy(cur.begin(), cur.end(), f_out);
  return bad;
}

// One step of Eq. combined_scheme evaluated only at the listed nodes
// (nodes[2n] = i, nodes[2n+1] = j); out[n*33 + q] receives f_q at time t + dt.
// Same arithmetic as or_step, restricted to the cross-shaped neighbourhood of
// each node, so that very large grids can be sampled.
void or_step_sample(const OrGrid* gp, const double* f, const int32_t* nodes, int32_t count,
                    double* out) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
#pragma omp parallel for schedule(dynamic)
  for (int n = 0; n < count; ++n) {
    const int i = nodes[2 * n], j = nodes[2 * n + 1];
    auto node_f = [&](int ii, int jj, double fl[NQ_MAX]) {
      for (int q = 0; q < VG.nq; ++q) fl[q] = f[idx(g, q, ii, jj)];
    };
    // macroscopic fields of any real node
    auto mac = [&](int ii, int jj, double m[4]) {
      double fl[NQ_MAX];
      node_f(ii, jj, fl);
      macros(VG, fl, m[0], m[1], m[2], m[3]);
    };
    // f_q at row ii (possibly a ghost row) of a real column jj, or at a real
    // row ii of a column up to two places beyond the ends (azimuthal ghosts)
    auto value = [&](int q, int ii, int jj) -> double {
      if (jj < 0 || jj >= g.nth) {
        int qs, js;
        azimuthal_source(g, q, jj, qs, js);
        return f[idx(g, qs, ii, js)];
      }
      if (ii >= 0 && ii < g.nr) return f[idx(g, q, ii, jj)];
      int side = ii < 0 ? 0 : 1;
      int i0 = side == 0 ? 0 : g.nr - 1, i1 = side == 0 ? 1 : g.nr - 2;
      int ig1 = side == 0 ? -1 : g.nr, ig2 = side == 0 ? -2 : g.nr + 1;
      double m0[4], m1[4], o1[4], o2[4];
      mac(i0, jj, m0);
      mac(i1, jj, m1);
      ghost_macros<double>(g, side, geo.rr(ig1), geo.rr(ig2), geo.ct[jj], geo.st[jj], m0, m1, o1, o2);
      const double* o = (ii == ig1) ? o1 : o2;
      double F[NK + 1];
      weights(o[3], row_of(g.ni), F);
      double v = feq_q(VG, o[0], o[1], o[2], o[3], F, q);
      if (g.bc_kind[side] & 16) {                    // + f - f^eq of the wall row
        double Fw[NK + 1];
        weights(m0[3], row_of(g.ni), Fw);
        v += f[idx(g, q, i0, jj)] - feq_q(VG, m0[0], m0[1], m0[2], m0[3], Fw, q);
      }
      return v;
    };
    double m[4];
    mac(i, j, m);
    double fe[NQ_MAX];
    feq_all(VG, m[0], m[1], m[2], m[3], fe);
    double r = geo.rr(i);
    for (int q = 0; q < VG.nq; ++q) {
      double ft = f[idx(g, q, i, j)];
      double res = relax_value(g, ft, fe[q]);
      double Cr = vr_of(VG, q, geo.ct[j], geo.st[j]) * g.dt / geo.dr;
      double Ct = vt_of(VG, q, geo.ct[j], geo.st[j]) * g.dt / (r * geo.dth);
      double pr[5], pt[5];
      for (int s = 0; s < 5; ++s) {
        pr[s] = value(q, i - 2 + s, j);
        pt[s] = value(q, i, j - 2 + s);
      }
      res -= convection_term(g.scheme, Cr, pr);
      res -= convection_term(g.scheme, Ct, pt);
      out[(size_t)n * VG.nq + q] = res;
    }
  }
}

// f = f^eq of given fields; u is given in polar components (u_r, u_theta) at
// each node and turned into Cartesian ones with the node's angle.
void or_init_feq(const OrGrid* gp, const double* rho, const double* ur, const double* ut,
                 const double* T, double* f) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
  for (int i = 0; i < g.nr; ++i)
    for (int j = 0; j < g.nth; ++j) {
      size_t c = (size_t)i * g.nth + j;
      double ux = ur[c] * geo.ct[j] - ut[c] * geo.st[j];
      double uy = ur[c] * geo.st[j] + ut[c] * geo.ct[j];
      double fe[NQ_MAX];
      feq_all(VG, rho[c], ux, uy, T[c], fe);
      for (int q = 0; q < VG.nq; ++q) f[idx(g, q, i, j)] = fe[q];
    }
}

// rho, u_r, u_theta, T fields of a distribution (any output may be null).
void or_fields(const OrGrid* gp, const double* f, double* rho, double* ur, double* ut, double* T) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
  for (int i = 0; i < g.nr; ++i)
    for (int j = 0; j < g.nth; ++j) {
      double fl[NQ_MAX], r_, ux, uy, E;
      for (int q = 0; q < VG.nq; ++q) fl[q] = f[idx(g, q, i, j)];
      macros(VG, fl, r_, ux, uy, E);
      size_t c = (size_t)i * g.nth + j;
      if (rho) rho[c] = r_;
      if (ur) ur[c] = ux * geo.ct[j] + uy * geo.st[j];
      if (ut) ut[c] = -ux * geo.st[j] + uy * geo.ct[j];
      if (T) T[c] = E;
    }
}

// Conserved totals over the annulus with the trapezoidal rule in r (weight
// 1/2 on the two wall rows) and the rectangle rule in theta:
// out = {mass, P_x, P_y, total energy, min rho, min T, non-finite count, 0}.
// Sums are accumulated in long double.
void or_diagnostics(const OrGrid* gp, const double* f, double* out) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
  long double mass = 0, px = 0, py = 0, en = 0;
  double rmin = INFINITY, tmin = INFINITY, bad = 0;
  for (int i = 0; i < g.nr; ++i) {
    double w = (i == 0 || i == g.nr - 1) ? 0.5 : 1.0;
    double dA = geo.rr(i) * w * geo.dr * geo.dth;
    for (int j = 0; j < g.nth; ++j) {
      double fl[NQ_MAX];
      long double rho = 0, jx = 0, jy = 0, eps = 0;
      bool fin = true;
      for (int q = 0; q < VG.nq; ++q) {
        fl[q] = f[idx(g, q, i, j)];
        if (!std::isfinite(fl[q])) fin = false;
        rho += fl[q]; jx += fl[q] * VG.vx[q]; jy += fl[q] * VG.vy[q];
        eps += 0.5L * fl[q] * (VG.vx[q] * VG.vx[q] + VG.vy[q] * VG.vy[q]);
      }
      if (!fin) { bad += 1; continue; }
      mass += rho * dA; px += jx * dA; py += jy * dA; en += eps * dA;
      double r_, ux, uy, E;
      macros(VG, fl, r_, ux, uy, E);
      rmin = std::min(rmin, r_); tmin = std::min(tmin, E);
    }
  }
  out[0] = (double)mass; out[1] = (double)px; out[2] = (double)py; out[3] = (double)en;
  out[4] = rmin; out[5] = tmin; out[6] = bad; out[7] = 0;
}

// One step of the discrete adjoint: lam_out = (d Phi / d f |_{f_t})^T lam_next,
// where Phi is the combined-scheme step of or_step (with terms = 7), including
// the dependence of the radial ghost nodes on the two real rows next to each
// wall.  Reverse-mode, written as a scatter from each output node to the inputs
// it depends on.  tie_eps is the relative size below which an upwind
// difference counts as zero (the derivative convention of mwb_grad): 1e-13
// suits a state computed in double precision.
int or_adjoint_step(const OrGrid* gp, const double* f_t, const double* lam_next, double tie_eps,
                    double* lam_out) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  // the adjoint of the combined MWB step of the octagon with equilibrium ghosts only
  if (g.scheme != 0 || g.terms != 7 || (g.bc_kind[0] & 16) || (g.bc_kind[1] & 16) || g.ni != 8)
    return -1;
  Geometry geo(g);
  size_t tot = (size_t)VG.nq * g.nr * g.nth, n = (size_t)g.nr * g.nth;
  std::vector<double> m;
  all_macros(g, f_t, m);
  Padded P(g.nr, g.nth, VG.nq);
  build_padded(g, geo, f_t, m, P);
  // d(relaxed f)/df = e + (1 - e) df^eq/df for both relaxations: Eq.
  // operator1_new has e = exp(-dt/tau), Eq. operator1_old e = 1 - dt/tau
  double e = g.relax == 1 ? 1.0 - g.dt / g.tau : std::exp(-g.dt / g.tau);

  // adjoint of the four linear moments of every real node
  std::vector<double> gM((size_t)4 * n, 0.0);
  // adjoint of the radial ghost distributions: [q][row slot 0..3][j] with
  // slots (-2, -1, nr, nr+1)
  std::vector<double> gG((size_t)VG.nq * 4 * g.nth, 0.0);
  std::fill(lam_out, lam_out + tot, 0.0);

  // (1) relaxation: lam_out += e lam; f^eq path into the node's moments.
#pragma omp parallel for schedule(static)
  for (int i = 0; i < g.nr; ++i)
    for (int j = 0; j < g.nth; ++j) {
      size_t c = (size_t)i * g.nth + j;
      double fl[NQ_MAX];
      for (int q = 0; q < VG.nq; ++q) fl[q] = f_t[idx(g, q, i, j)];
      Dual<4> M[4];
      M[0] = 0; M[1] = 0; M[2] = 0; M[3] = 0;
      double Mv[4] = {0, 0, 0, 0};
      for (int q = 0; q < VG.nq; ++q) {
        Mv[0] += fl[q]; Mv[1] += fl[q] * VG.vx[q]; Mv[2] += fl[q] * VG.vy[q];
        Mv[3] += 0.5 * fl[q] * (VG.vx[q] * VG.vx[q] + VG.vy[q] * VG.vy[q]);
      }
      for (int a = 0; a < 4; ++a) { M[a] = Dual<4>(Mv[a]); M[a].d[a] = 1.0; }
      Dual<4> rho, ux, uy, E, fe[NQ_MAX];
      macros_of_M(M, rho, ux, uy, E);
      feq_all(VG, rho, ux, uy, E, fe);
      double acc[4] = {0, 0, 0, 0};
      for (int q = 0; q < VG.nq; ++q) {
        double lam = lam_next[idx(g, q, i, j)];
        lam_out[idx(g, q, i, j)] += e * lam;
        for (int a = 0; a < 4; ++a) acc[a] += (1.0 - e) * lam * fe[q].d[a];
      }
      for (int a = 0; a < 4; ++a) gM[a * n + c] += acc[a];
    }

  // (2) convection terms, one velocity plane at a time.  Across the ends of a
  // sector a stencil of plane q reads (and so scatters into) other planes of
  // the same speed, so the threads take one speed each, its planes in turn.
#pragma omp parallel for schedule(dynamic)
  for (int kk = 0; kk <= NK; ++kk)
  for (int q = kk == 0 ? 0 : 1 + NI * (kk - 1); q < (kk == 0 ? 1 : 1 + NI * kk); ++q) {
    for (int i = 0; i < g.nr; ++i) {
      double r = geo.rr(i);
      for (int j = 0; j < g.nth; ++j) {
        double lam = lam_next[idx(g, q, i, j)];
        double Cr = vr_of(VG, q, geo.ct[j], geo.st[j]) * g.dt / geo.dr;
        double Ct = vt_of(VG, q, geo.ct[j], geo.st[j]) * g.dt / (r * geo.dth);
        double psi[5], gr[5];
        for (int s = 0; s < 5; ++s) psi[s] = P.at(q, i - 2 + s, j);
        mwb_grad(Cr, psi, tie_eps, gr);
        for (int s = 0; s < 5; ++s) {
          int ii = i - 2 + s;
          double v = -lam * gr[s];
          if (v == 0.0) continue;
          if (ii >= 0 && ii < g.nr) lam_out[idx(g, q, ii, j)] += v;
          else {
            int slot = ii == -2 ? 0 : ii == -1 ? 1 : ii == g.nr ? 2 : 3;
            gG[((size_t)q * 4 + slot) * g.nth + j] += v;
          }
        }
        for (int s = 0; s < 5; ++s) psi[s] = P.at(q, i, j - 2 + s);
        mwb_grad(Ct, psi, tie_eps, gr);
        for (int s = 0; s < 5; ++s) {
          int qs, js;                    // where the stencil's value was read
          azimuthal_source(g, q, j - 2 + s, qs, js);
          lam_out[idx(g, qs, i, js)] += -lam * gr[s];
        }
      }
    }
  }

  // (3) radial ghosts depend on the moments of the two real rows by each wall.
  for (int side = 0; side < 2; ++side) {
    int i0 = side == 0 ? 0 : g.nr - 1, i1 = side == 0 ? 1 : g.nr - 2;
    int ig1 = side == 0 ? -1 : g.nr, ig2 = side == 0 ? -2 : g.nr + 1;
    int s1 = side == 0 ? 1 : 2, s2 = side == 0 ? 0 : 3;
    for (int j = 0; j < g.nth; ++j) {
      Dual<8> M0[4], M1[4], m0[4], m1[4], o1[4], o2[4];
      for (int a = 0; a < 4; ++a) {
        double v0 = 0, v1 = 0;
        for (int q = 0; q < VG.nq; ++q) {
          double ph = a == 0 ? 1.0 : a == 1 ? VG.vx[q] : a == 2 ? VG.vy[q]
                    : 0.5 * (VG.vx[q] * VG.vx[q] + VG.vy[q] * VG.vy[q]);
          v0 += ph * f_t[idx(g, q, i0, j)];
          v1 += ph * f_t[idx(g, q, i1, j)];
        }
        M0[a] = Dual<8>(v0); M0[a].d[a] = 1.0;
        M1[a] = Dual<8>(v1); M1[a].d[4 + a] = 1.0;
      }
      macros_of_M(M0, m0[0], m0[1], m0[2], m0[3]);
      macros_of_M(M1, m1[0], m1[1], m1[2], m1[3]);
      ghost_macros<Dual<8>>(g, side, geo.rr(ig1), geo.rr(ig2), geo.ct[j], geo.st[j], m0, m1, o1, o2);
      Dual<8> fe1[NQ_MAX], fe2[NQ_MAX];
      feq_all(VG, o1[0], o1[1], o1[2], o1[3], fe1);
      feq_all(VG, o2[0], o2[1], o2[2], o2[3], fe2);
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int q = 0; q < VG.nq; ++q) {
        double l1 = gG[((size_t)q * 4 + s1) * g.nth + j];
        double l2 = gG[((size_t)q * 4 + s2) * g.nth + j];
        for (int d = 0; d < 8; ++d) acc[d] += l1 * fe1[q].d[d] + l2 * fe2[q].d[d];
      }
      for (int a = 0; a < 4; ++a) {
        gM[a * n + (size_t)i0 * g.nth + j] += acc[a];
        gM[a * n + (size_t)i1 * g.nth + j] += acc[4 + a];
      }
    }
  }

  // (4) moments are linear in f: M_a = sum_q phi_a(q) f_q.
#pragma omp parallel for schedule(static)
  for (int i = 0; i < g.nr; ++i)
    for (int j = 0; j < g.nth; ++j) {
      size_t c = (size_t)i * g.nth + j;
      for (int q = 0; q < VG.nq; ++q) {
        double ph3 = 0.5 * (VG.vx[q] * VG.vx[q] + VG.vy[q] * VG.vy[q]);
        lam_out[idx(g, q, i, j)] += gM[c] + gM[n + c] * VG.vx[q] + gM[2 * n + c] * VG.vy[q] +
                                    gM[3 * n + c] * ph3;
      }
    }
  return 0;
}

// Adjoint of or_init_feq: given lam = dJ/df at the initial state, return
// dJ/d(rho, u_r, u_theta, T) per node.
void or_adjoint_init(const OrGrid* gp, const double* rho, const double* ur, const double* ut,
                     const double* T, const double* lam, double* d_rho, double* d_ur,
                     double* d_ut, double* d_T) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
  for (int i = 0; i < g.nr; ++i)
    for (int j = 0; j < g.nth; ++j) {
      size_t c = (size_t)i * g.nth + j;
      Dual<4> R(rho[c]), Ur(ur[c]), Ut(ut[c]), TT(T[c]);
      R.d[0] = 1; Ur.d[1] = 1; Ut.d[2] = 1; TT.d[3] = 1;
      Dual<4> ux = Ur * geo.ct[j] - Ut * geo.st[j];
      Dual<4> uy = Ur * geo.st[j] + Ut * geo.ct[j];
      Dual<4> fe[NQ_MAX];
      feq_all(VG, R, ux, uy, TT, fe);
      double acc[4] = {0, 0, 0, 0};
      for (int q = 0; q < VG.nq; ++q) {
        double l = lam[idx(g, q, i, j)];
        for (int a = 0; a < 4; ++a) acc[a] += l * fe[q].d[a];
      }
      d_rho[c] = acc[0]; d_ur[c] = acc[1]; d_ut[c] = acc[2]; d_T[c] = acc[3];
    }
}

// Sec. IV, Eqs. M_relative, M_absolute, D_relative, D_absolute: the moments
// M_m and the central moments M*_m (velocities relative to the node's flow
// velocity u) of f, and their departures from equilibrium Delta_m = M_m(f -
// f^eq) and Delta*_m = M*_m(f - f^eq), f^eq taken at the node's own rho, u,
// E.  Components in the polar basis (e_r, e_theta) of the node, 12 per kind:
//   M_2: rr, r theta, theta theta;  M_3: rrr, rr theta, r theta theta,
//   theta theta theta;  M_{3,1}: r, theta;  M_{4,2}: rr, r theta, theta theta,
// where M_{3,1} = sum (1/2) f |v|^2 v and M_{4,2} = sum (1/2) f |v|^2 v v.
// out[((kind * 12 + comp) * nr + i) * nth + j], kind 0 = M, 1 = M*, 2 = Delta,
// 3 = Delta*.
// The non-equilibrium fields of one node (i, j): acc[kind][12] as or_noneq.
static void noneq_node(const OrGrid& g, const Geometry& geo, const double* f, int i, int j,
                       double acc[4][12]) {
  const Velocities& VG = vel_of(g.ni);
  double fl[NQ_MAX], fe[NQ_MAX];
  for (int q = 0; q < VG.nq; ++q) fl[q] = f[idx(g, q, i, j)];
  double rho, ux, uy, E;
  macros(VG, fl, rho, ux, uy, E);
  feq_all(VG, rho, ux, uy, E, fe);
  const double ct = geo.ct[j], st = geo.st[j];
  const double ur = ux * ct + uy * st, ut = -ux * st + uy * ct;
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 12; ++c) acc[a][c] = 0.0;
  for (int q = 0; q < VG.nq; ++q) {
    const double vr = vr_of(VG, q, ct, st), vt = vt_of(VG, q, ct, st);
    for (int kind = 0; kind < 4; ++kind) {
      const double w = kind < 2 ? fl[q] : fl[q] - fe[q];       // f, or f - f^eq
      const bool central = kind % 2 == 1;
      const double a = central ? vr - ur : vr;                  // r component
      const double b = central ? vt - ut : vt;                  // theta component
      const double h = 0.5 * (a * a + b * b);                   // |v|^2 / 2
      double* o = acc[kind];
      o[0] += w * a * a;  o[1] += w * a * b;  o[2] += w * b * b;
      o[3] += w * a * a * a;  o[4] += w * a * a * b;  o[5] += w * a * b * b;  o[6] += w * b * b * b;
      o[7] += w * h * a;  o[8] += w * h * b;
      o[9] += w * h * a * a;  o[10] += w * h * a * b;  o[11] += w * h * b * b;
    }
  }
}

// Sec. IV, Eqs. M_relative, M_absolute, D_relative, D_absolute: the moments
// M_m and the central moments M*_m (velocities relative to the node's flow
// velocity u) of f, and their departures from equilibrium Delta_m = M_m(f -
// f^eq) and Delta*_m = M*_m(f - f^eq), f^eq taken at the node's own rho, u,
// E.  Components in the polar basis (e_r, e_theta) of the node, 12 per kind:
//   M_2: rr, r theta, theta theta;  M_3: rrr, rr theta, r theta theta,
//   theta theta theta;  M_{3,1}: r, theta;  M_{4,2}: rr, r theta, theta theta,
// where M_{3,1} = sum (1/2) f |v|^2 v and M_{4,2} = sum (1/2) f |v|^2 v v.
// out[((kind * 12 + comp) * nr + i) * nth + j], kind 0 = M, 1 = M*, 2 = Delta,
// 3 = Delta*.
void or_noneq(const OrGrid* gp, const double* f, double* out) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
  const size_t n = (size_t)g.nr * g.nth;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < g.nr; ++i)
    for (int j = 0; j < g.nth; ++j) {
      double acc[4][12];
      noneq_node(g, geo, f, i, j, acc);
      const size_t cidx = (size_t)i * g.nth + j;
      for (int kind = 0; kind < 4; ++kind)
        for (int c = 0; c < 12; ++c) out[((size_t)kind * 12 + c) * n + cidx] = acc[kind][c];
    }
}

// The same at the listed nodes only (nodes[2n] = i, nodes[2n+1] = j):
// out[(n * 4 + kind) * 12 + comp].
void or_noneq_sample(const OrGrid* gp, const double* f, const int32_t* nodes, int32_t count,
                     double* out) {
  const OrGrid& g = *gp;
  const Velocities& VG = vel_of(g.ni);
  Geometry geo(g);
#pragma omp parallel for schedule(static)
  for (int n = 0; n < count; ++n) {
    double acc[4][12];
    noneq_node(g, geo, f, nodes[2 * n], nodes[2 * n + 1], acc);
    for (int kind = 0; kind < 4; ++kind)
      for (int c = 0; c < 12; ++c) out[((size_t)n * 4 + kind) * 12 + c] = acc[kind][c];
  }
}

int or_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
