// Device-side building blocks of the polar FDLB step (gfx950).
//
// Velocity model: Sec. II.A of Lin et al. (arXiv:1302.7104), Eq. DVM1, with
// the speeds (0, 1, 2.92, 2.99, 4.49) and the octagon row of Table I.
// Numbering: q = 0 rest; q = 1 + 8(k-1) + d for speed group k = 1..4 and
// direction d = 0..7 at angle d*pi/4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Everything a step launch needs besides the state buffers.
struct Tables {
  int32_t nr, nth;
  double dt_dr;        // dt / dr
  double dt_dth;       // dt / dtheta
  double e;            // exp(-dt / tau), computed on the host in double
  double fc[NK][4];    // F_k(E) = E (c0 + E (c1 + E (c2 + E c3))), k = 1..4 at [k-1]
  const double* cth;   // cos(theta_j), j = 0..nth-1
  const double* sth;   // sin(theta_j)
  const double* rinv;  // 1 / r_i, i = 0..nr-1
  const double* wA;    // quadrature weight r_i w_i dr dtheta of row i
};

// Radial boundary description as the kernels see it.
struct BCdev {
  int32_t kind[2];     // PCLB_WALL / PCLB_INFLOW / PCLB_EXTRAPOLATE
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
struct EqCoef {
  double rF[NK + 1];   // rho F_k
  double A0, A1, A2, A3, A4;
  double p[4];         // u . e_d for d = 0..3 (d + 4 is the negative)
};

__device__ inline void eq_setup(const Tables& T, double rho, double ux, double uy, double E,
                                EqCoef& c) {
  double iE = 1.0 / E;
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    double F = E * (T.fc[k][0] + E * (T.fc[k][1] + E * (T.fc[k][2] + E * T.fc[k][3])));
    c.rF[k + 1] = rho * F;
    sum += F;
  }
  c.rF[0] = rho * (1.0 - 8.0 * sum);
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

__device__ inline double eq_val(const EqCoef& c, int k, int d) {
  double pd = d < 4 ? c.p[d] : -c.p[d - 4];
  double w = speed(k) * pd;
  return c.rF[k] * (c.A0 + w * (c.A1 + w * (c.A2 + w * (c.A3 + w * c.A4))));
}

// Linear moments of one node: rho, j_x, j_y and eps = sum f v^2 / 2; then the
// macroscopic u and E = eps / rho - u^2 / 2 (Eqs. moment1-moment3).
__device__ inline void node_macros(const double* f, double& rho, double& ux, double& uy,
                                   double& E) {
  double r = 0.0, jx = 0.0, jy = 0.0, eps = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    r += f[q];
    jx += f[q] * vx_q(q);
    jy += f[q] * vy_q(q);
    eps += f[q] * v2_q(q);
  }
  rho = r;
  double ir = 1.0 / r;
  ux = jx * ir;
  uy = jy * ir;
  E = 0.5 * eps * ir - 0.5 * (ux * ux + uy * uy);
}

// ---------------------------------------------------------------------------
// MWB convection term (Eq. MWB Scheme) in the division-free form, written with
// the upwind neighbours u1 (one node upwind) and u2 (two nodes upwind):
//   T = |C| d1 + |C|(1-|C|) (d1 - d2) |d1| / (|d1| + |d2|),  d1 = c - u1,
//   d2 = u1 - u2,
// which equals [C + C(1-|C|)(1-S(eta))(1-eta)/2] delta for either sign of C,
// and is 0 in the limiter part when d1 = d2 = 0.
template <class R> struct Lim;
template <> struct Lim<double> {
  __device__ static inline double ratio(double num, double den) {
    return num / fmax(den, 2.2250738585072014e-308);
  }
};
template <> struct Lim<float> {
  __device__ static inline float ratio(float num, float den) {
    return num * __builtin_amdgcn_rcpf(fmaxf(den, 1.17549435e-38f));
  }
};

template <class R>
__device__ inline R mwb_term(R absC, R K, R c, R u1, R u2) {
  R d1 = c - u1;
  R d2 = u1 - u2;
  R den = (d1 < R(0) ? -d1 : d1) + (d2 < R(0) ? -d2 : d2);
  R lim = Lim<R>::ratio((d1 - d2) * (d1 < R(0) ? -d1 : d1), den);
  return absC * d1 + K * lim;
}

}  // namespace pclb
