// Forward kernels of the polar FDLB step: radial ghost layers, the per-node
// reference step, initial equilibrium, macroscopic fields and diagnostics.
// Sec. II of Lin et al. (arXiv:1302.7104).
#include "common.h"
#include "diag.h"
#include "launch.h"

namespace pclb {

// ---------------------------------------------------------------------------
// Radial ghost layers (Sec. II.C, radial boundary condition): from the two
// real rows next to a wall take rho, u, E; extrapolate rho and E linearly and
// recursively (ghost0 = 2 row0 - row1, ghost1 = 2 ghost0 - row0); set the
// velocity per boundary kind; store f^eq of the ghost state.
template <class R>
__global__ void __launch_bounds__(256) ghost_kernel(Tables T, BCdev bc, const R* __restrict__ f,
                                                    R* __restrict__ ghost) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int side = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const int i0 = side == 0 ? 0 : T.nr - 1;
  const int i1 = side == 0 ? 1 : T.nr - 2;
  R f0[NQ], f1[NQ], g0[NQ], g1[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    f0[q] = f[q * plane + (size_t)i0 * T.nth + j];
    f1[q] = f[q * plane + (size_t)i1 * T.nth + j];
  }
  ghost_column<R>(T, bc, side, T.cth[j], T.sth[j], f0, f1, g0, g1);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    ghost[ghost_index(side, 0, q, j, T.nth)] = g0[q];
    ghost[ghost_index(side, 1, q, j, T.nth)] = g1[q];
  }
}

// ---------------------------------------------------------------------------
// Reference step: one thread per node, neighbours read straight from global
// memory (Eq. combined_scheme).  Used for small grids and as a cross-check of
// the strip kernel.
template <class R>
__device__ inline R fetch(const R* __restrict__ f, const R* __restrict__ ghost, int q, int i, int j,
                          int nr, int nth, size_t plane) {
  if (i < 0) return ghost[ghost_index(0, -1 - i, q, j, nth)];
  if (i >= nr) return ghost[ghost_index(1, i - nr, q, j, nth)];
  return f[q * plane + (size_t)i * nth + j];
}

template <class R, int SCH, bool SECTOR>
__device__ inline void node_step_at(const Tables& T, const R* __restrict__ f, R* __restrict__ out,
                                    const R* __restrict__ ghost, int i, int j) {
  const int nr = T.nr, nth = T.nth;
  const size_t plane = (size_t)nr * nth;
  const size_t c0 = (size_t)i * nth + j;
  R fc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) fc[q] = f[q * plane + c0];
  auto row = [&](int q, int di) { return fetch(f, ghost, q, i + di, j, nr, nth, plane); };
  // theta neighbours; across the ends of a sector the direction index rotates
  auto col = [&](int q, int dj) {
    int t = j + dj, qq = q;
    if constexpr (SECTOR) {
      const int s_lo = T.nf & 7, s_hi = (8 - T.nf) & 7;
      if (t < 0) {
        t += nth;
        qq = rot_q(q, s_lo);
      } else if (t >= nth) {
        t -= nth;
        qq = rot_q(q, s_hi);
      }
    } else {
      t = t < 0 ? t + nth : (t >= nth ? t - nth : t);
    }
    return f[qq * plane + (size_t)i * nth + t];
  };
  // each result is stored as soon as it is computed: holding all 33 (with the
  // centre values and the neighbours in flight) kept the kernel at one wave
  // per SIMD
  node_update_put<R, SCH>(T, i, j, fc, row, col, [&](int q, R v) { out[q * plane + c0] = v; });
}

// Three waves per SIMD: the FP64 kernel then keeps 168 VGPRs and spills 24
// of them to scratch, which is still faster than two waves without spills
// (6.3 against 6.8 ms per step at 4096 x 8192; four waves: 8.9 ms).
#ifndef PCLB_NODE_WAVES
#define PCLB_NODE_WAVES 3
#endif
template <class R, int SCH, bool SECTOR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PCLB_NODE_WAVES, PCLB_NODE_WAVES)))
step_node_kernel(Tables T, const R* __restrict__ f, R* __restrict__ out,
                 const R* __restrict__ ghost) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= T.nth) return;
  node_step_at<R, SCH, SECTOR>(T, f, out, ghost, blockIdx.y, j);
}

template <class R, int SCH>
void launch_node_sch(const Tables& T, dim3 grid, const R* f, R* out, const R* ghost, hipStream_t s) {
  if (T.nf == 8)
    hipLaunchKernelGGL((step_node_kernel<R, SCH, false>), grid, dim3(256), 0, s, T, f, out, ghost);
  else
    hipLaunchKernelGGL((step_node_kernel<R, SCH, true>), grid, dim3(256), 0, s, T, f, out, ghost);
}

// ---------------------------------------------------------------------------
// f = f^eq(rho, u, T) with u given in polar components (Eq. feq).
template <class R>
__global__ void __launch_bounds__(256) init_kernel(Tables T, const double* __restrict__ rho,
                                                   const double* __restrict__ ur,
                                                   const double* __restrict__ ut,
                                                   const double* __restrict__ Tt,
                                                   R* __restrict__ f, int* __restrict__ bad) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const size_t c0 = (size_t)i * T.nth + j;
  double r = rho[c0], a = ur[c0], b = ut[c0], E = Tt[c0];
  if (!(r > 0.0) || !(E > 0.0) || !isfinite(r) || !isfinite(E) || !isfinite(a) || !isfinite(b))
    atomicOr(bad, 1);
  double ct = T.cth[j], st = T.sth[j];
  double ux = a * ct - b * st, uy = a * st + b * ct;
  EqCoef c;
  eq_setup(T, r, ux, uy, E, c);
  f[c0] = (R)(c.rF[0] * c.A0);
#pragma unroll
  for (int k = 1; k <= NK; ++k)
#pragma unroll
    for (int d = 0; d < ND; ++d) f[qidx(k, d) * plane + c0] = (R)eq_val(c, k, d);
}

// ---------------------------------------------------------------------------
// Macroscopic fields (rho, u_r, u_theta, T) of every node; null outputs skipped.
template <class R>
__global__ void __launch_bounds__(256) fields_kernel(Tables T, const R* __restrict__ f,
                                                     double* rho, double* ur, double* ut,
                                                     double* Tt) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const size_t c0 = (size_t)i * T.nth + j;
  double fl[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) fl[q] = (double)f[q * plane + c0];
  double r, ux, uy, E;
  node_macros(fl, r, ux, uy, E);
  double ct = T.cth[j], st = T.sth[j];
  if (rho) rho[c0] = r;
  if (ur) ur[c0] = ux * ct + uy * st;
  if (ut) ut[c0] = -ux * st + uy * ct;
  if (Tt) Tt[c0] = E;
}

// ---------------------------------------------------------------------------
// Non-equilibrium fields of Sec. IV (Eqs. M_relative, M_absolute, D_relative,
// D_absolute): per node the moments M_m and central moments M*_m of f and
// their departures from equilibrium Delta_m = M_m(f - f^eq), Delta*_m =
// M*_m(f - f^eq), m in {2, 3, (3,1), (4,2)}, in the node's polar basis, 12
// components per kind (rr, r theta, theta theta; rrr, rr theta, r theta theta,
// theta theta theta; r, theta; rr, r theta, theta theta).  f^eq is summed from
// the discrete equilibrium of the node's rho, u, E.  All in double.  The kinds
// selected by the bit mask go to out in the order M, M*, Delta, Delta*.
//
// Every component is a moment of order 2 to 4 in the polar velocity
// components, so the kernel sums the 15 polar moments up to order four once,
// P[n][m] = sum_q w_q a^(n-m) b^m (a = v . e_r, b = v . e_theta), for w = f
// and for w = f - f^eq, and forms the central ones from them with the
// binomial sum over (a - u_r)^i (b - u_theta)^j.  Each rounding is relative to
// a term of the sum over q of |w_q| (|v_q| + |u|)^order.
namespace noneq {

constexpr int NM = 15;                                    // moments of order 0..4
__host__ __device__ constexpr int mo(int n, int m) { return n * (n + 1) / 2 + m; }
// binomial coefficients C(n, k), n <= 4
__device__ constexpr double BINOM[5][5] = {
    {1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};

// P += t w and P_d += t w_d over the 15 monomials t = a^(n-m) b^m
__device__ __forceinline__ void polar_add(double a, double b, double w, double wd,
                                          double (&Pf)[NM], double (&Pd)[NM]) {
  double pa[5], pb[5];
  pa[0] = pb[0] = 1.0;
#pragma unroll
  for (int p = 1; p < 5; ++p) {
    pa[p] = pa[p - 1] * a;
    pb[p] = pb[p - 1] * b;
  }
#pragma unroll
  for (int n = 0; n <= 4; ++n)
#pragma unroll
    for (int m = 0; m <= n; ++m) {
      const double t = pa[n - m] * pb[m];
      Pf[mo(n, m)] += t * w;
      Pd[mo(n, m)] += t * wd;
    }
}

// sum_q w (a - sr)^I (b - st)^J from the polar moments; pr[p] = (-sr)^p,
// pt[p] = (-st)^p
template <int I, int J>
__device__ __forceinline__ double shifted(const double (&P)[NM], const double (&pr)[5],
                                          const double (&pt)[5]) {
  double acc = 0.0;
#pragma unroll
  for (int k = I; k >= 0; --k)
#pragma unroll
    for (int l = J; l >= 0; --l)
      acc += (BINOM[I][k] * BINOM[J][l]) * (pr[I - k] * pt[J - l]) * P[mo(k + l, l)];
  return acc;
}

// the 12 components of one kind, about (sr, st)
__device__ __forceinline__ void components(const double (&P)[NM], double sr, double st,
                                           double (&o)[12]) {
  double pr[5], pt[5];
  pr[0] = pt[0] = 1.0;
#pragma unroll
  for (int p = 1; p < 5; ++p) {
    pr[p] = pr[p - 1] * -sr;
    pt[p] = pt[p - 1] * -st;
  }
  const double s20 = shifted<2, 0>(P, pr, pt), s11 = shifted<1, 1>(P, pr, pt), s02 = shifted<0, 2>(P, pr, pt);
  const double s30 = shifted<3, 0>(P, pr, pt), s21 = shifted<2, 1>(P, pr, pt);
  const double s12 = shifted<1, 2>(P, pr, pt), s03 = shifted<0, 3>(P, pr, pt);
  const double s40 = shifted<4, 0>(P, pr, pt), s31 = shifted<3, 1>(P, pr, pt), s22 = shifted<2, 2>(P, pr, pt);
  const double s13 = shifted<1, 3>(P, pr, pt), s04 = shifted<0, 4>(P, pr, pt);
  o[0] = s20;  o[1] = s11;  o[2] = s02;
  o[3] = s30;  o[4] = s21;  o[5] = s12;  o[6] = s03;
  o[7] = 0.5 * (s30 + s12);   // sum w |c|^2/2 c_r
  o[8] = 0.5 * (s21 + s03);
  o[9] = 0.5 * (s40 + s22);   // sum w |c|^2/2 c_r c_r
  o[10] = 0.5 * (s31 + s13);
  o[11] = 0.5 * (s22 + s04);
}

}  // namespace noneq

template <class R>
__global__ void __launch_bounds__(256) noneq_kernel(Tables T, const R* __restrict__ f, int kinds,
                                                    double* __restrict__ out) {
  using namespace noneq;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= T.nth) return;
  const size_t plane = (size_t)T.nr * T.nth;
  const size_t c0 = (size_t)i * T.nth + j;
  R fl[NQ];                    // the node's values in the state's type
#pragma unroll
  for (int q = 0; q < NQ; ++q) fl[q] = f[q * plane + c0];
  double rho, ux, uy, E;
  {
    double fd[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) fd[q] = (double)fl[q];
    node_macros(fd, rho, ux, uy, E);
  }
  const double f0 = (double)fl[0];
  EqCoef ec;
  eq_setup(T, rho, ux, uy, E, ec);
  const double ct = T.cth[j], st = T.sth[j];
  double Pf[NM], Pd[NM];
#pragma unroll
  for (int m = 1; m < NM; ++m) Pf[m] = Pd[m] = 0.0;
  Pf[0] = f0;                                   // the rest velocity: order 0 only
  Pd[0] = f0 - ec.rF[0] * ec.A0;
  // speeds in a loop (a bounded working set: unrolled, the scheduler keeps
  // every velocity's products live at once), directions unrolled
#pragma unroll 1
  for (int k = 1; k <= NK; ++k) {
    const double vk = k == 1 ? speed(1) : k == 2 ? speed(2) : k == 3 ? speed(3) : speed(4);
    const double rFk = k == 1 ? ec.rF[1] : k == 2 ? ec.rF[2] : k == 3 ? ec.rF[3] : ec.rF[4];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double w = (double)(k == 1 ? fl[1 + d] : k == 2 ? fl[9 + d] : k == 3 ? fl[17 + d] : fl[25 + d]);
      const double x = vk * (d < 4 ? ec.p[d] : -ec.p[d - 4]);
      const double fe = rFk * (ec.A0 + x * (ec.A1 + x * (ec.A2 + x * (ec.A3 + x * ec.A4))));
      // polar components of e_d at this node, times the speed
      const double ea = cos_d(d) * ct + sin_d(d) * st, eb = sin_d(d) * ct - cos_d(d) * st;
      polar_add(vk * ea, vk * eb, w, w - fe, Pf, Pd);
    }
  }
  const double ur = ux * ct + uy * st, ut = -ux * st + uy * ct;
  int slot = 0;
#pragma unroll
  for (int kind = 0; kind < 4; ++kind) {
    if (!((kinds >> kind) & 1)) continue;
    const bool central = kind & 1;
    double o[12];
    if (kind < 2) components(Pf, central ? ur : 0.0, central ? ut : 0.0, o);
    else components(Pd, central ? ur : 0.0, central ? ut : 0.0, o);
#pragma unroll
    for (int c = 0; c < 12; ++c)   // not read again here: nontemporal
      __builtin_nontemporal_store(o[c], out + ((size_t)slot * 12 + c) * plane + c0);
    ++slot;
  }
}

// ---------------------------------------------------------------------------
// Diagnostics of the octagon state (reduction helpers in diag.h).
template <class R>
__global__ void __launch_bounds__(DIAG_BLOCK) diag_partial_kernel(Tables T, const R* __restrict__ f,
                                                                  double* __restrict__ partial) {
  const size_t plane = (size_t)T.nr * T.nth;
  TwoS acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  double rmin = INFINITY, tmin = INFINITY, bad = 0.0;
  for (size_t n = (size_t)blockIdx.x * DIAG_BLOCK + threadIdx.x; n < plane;
       n += (size_t)gridDim.x * DIAG_BLOCK) {
    int i = (int)(n / T.nth);
    double fl[NQ];
    bool fin = true;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      fl[q] = (double)f[q * plane + n];
      fin = fin && isfinite(fl[q]);
    }
    if (!fin) { bad += 1.0; continue; }
    double rho = 0, jx = 0, jy = 0, eps = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      rho += fl[q]; jx += fl[q] * vx_q(q); jy += fl[q] * vy_q(q); eps += fl[q] * v2_q(q);
    }
    eps *= 0.5;
    double w = T.wA[i];
    two_add(acc[0], rho * w);
    two_add(acc[1], jx * w);
    two_add(acc[2], jy * w);
    two_add(acc[3], eps * w);
    double ir = 1.0 / rho;
    double ux = jx * ir, uy = jy * ir;
    double E = eps * ir - 0.5 * (ux * ux + uy * uy);
    rmin = fmin(rmin, rho);
    tmin = fmin(tmin, E);
  }
  diag_block_reduce(acc, rmin, tmin, bad, partial);
}

// Final pass: one wavefront.  Lane l merges the partial rows l, l + 64,
// l + 128, ... in that order, then the lanes' results meet in a butterfly of
// fixed shape (offsets 32, 16, ..., 1), so the sums are the same on every run.
__global__ void __launch_bounds__(64) diag_final_kernel(const double* __restrict__ partial, int nb,
                                                        double step, double* __restrict__ out) {
  const int lane = threadIdx.x;
  TwoS acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  double rmin = INFINITY, tmin = INFINITY, bad = 0.0;
  for (int b = lane; b < nb; b += 64) {
    const double* p = partial + (size_t)b * DIAG_SLOTS;
    for (int a = 0; a < 4; ++a) acc[a] = two_merge(acc[a], TwoS{p[2 * a], p[2 * a + 1]});
    rmin = fmin(rmin, p[8]);
    tmin = fmin(tmin, p[9]);
    bad += p[10];
  }
  for (int o = 32; o > 0; o >>= 1) {
    for (int a = 0; a < 4; ++a) {
      const TwoS other{__shfl_xor(acc[a].s, o), __shfl_xor(acc[a].c, o)};
      // the lower lane of each pair keeps its own sum first, so both lanes
      // of a pair form the same result
      acc[a] = (lane & o) ? two_merge(other, acc[a]) : two_merge(acc[a], other);
    }
    rmin = fmin(rmin, __shfl_xor(rmin, o));
    tmin = fmin(tmin, __shfl_xor(tmin, o));
    const double ob = __shfl_xor(bad, o);
    bad = (lane & o) ? ob + bad : bad + ob;
  }
  if (lane == 0) {
    for (int a = 0; a < 4; ++a) out[a] = acc[a].s + acc[a].c;
    out[4] = rmin;
    out[5] = tmin;
    out[6] = bad;
    out[7] = step;
  }
}

// ---------------------------------------------------------------------------
// Launchers (host side).
template <class R>
hipError_t launch_ghost(const Tables& T, const BCdev& bc, const void* f, void* ghost, hipStream_t s) {
  dim3 grid((T.nth + 255) / 256, 2);
  hipLaunchKernelGGL(ghost_kernel<R>, grid, dim3(256), 0, s, T, bc, (const R*)f, (R*)ghost);
  return hipGetLastError();
}

template <class R>
hipError_t launch_step_node(const Tables& T, const void* f, void* out, const void* ghost, hipStream_t s) {
  dim3 grid((T.nth + 255) / 256, T.nr);
  const R* fi = (const R*)f;
  const R* gh = (const R*)ghost;
  switch (T.scheme) {
    case SCH_WB: launch_node_sch<R, SCH_WB>(T, grid, fi, (R*)out, gh, s); break;
    case SCH_LW: launch_node_sch<R, SCH_LW>(T, grid, fi, (R*)out, gh, s); break;
    case SCH_UPWIND2: launch_node_sch<R, SCH_UPWIND2>(T, grid, fi, (R*)out, gh, s); break;
    default: launch_node_sch<R, SCH_MWB>(T, grid, fi, (R*)out, gh, s);
  }
  return hipGetLastError();
}

template <class R>
hipError_t launch_init(const Tables& T, const double* rho, const double* ur, const double* ut,
                       const double* Tt, void* f, int* bad, hipStream_t s) {
  dim3 grid((T.nth + 255) / 256, T.nr);
  hipLaunchKernelGGL(init_kernel<R>, grid, dim3(256), 0, s, T, rho, ur, ut, Tt, (R*)f, bad);
  return hipGetLastError();
}

template <class R>
hipError_t launch_fields(const Tables& T, const void* f, double* rho, double* ur, double* ut,
                         double* Tt, hipStream_t s) {
  dim3 grid((T.nth + 255) / 256, T.nr);
  hipLaunchKernelGGL(fields_kernel<R>, grid, dim3(256), 0, s, T, (const R*)f, rho, ur, ut, Tt);
  return hipGetLastError();
}

__global__ void zero_int_kernel(int* p) { if (threadIdx.x == 0) *p = 0; }

hipError_t launch_zero_int(int* p, hipStream_t s) {
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

template <class R>
hipError_t launch_noneq(const Tables& T, const void* f, int kinds, double* out, hipStream_t s) {
  dim3 grid((T.nth + 255) / 256, T.nr);
  hipLaunchKernelGGL(noneq_kernel<R>, grid, dim3(256), 0, s, T, (const R*)f, kinds, out);
  return hipGetLastError();
}

int diag_blocks() { return 1024; }
int diag_slots() { return DIAG_SLOTS; }

template <class R>
hipError_t launch_diag(const Tables& T, const void* f, double* partial, double step, double* out,
                       hipStream_t s) {
  int nb = diag_blocks();
  hipLaunchKernelGGL(diag_partial_kernel<R>, dim3(nb), dim3(DIAG_BLOCK), 0, s, T, (const R*)f, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_diag_final(partial, nb, step, out, s);
}

hipError_t launch_diag_final(const double* partial, int nb, double step, double* out, hipStream_t s) {
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, s, partial, nb, step, out);
  return hipGetLastError();
}

#define PCLB_INST(R)                                                                              \
  template hipError_t launch_ghost<R>(const Tables&, const BCdev&, const void*, void*, hipStream_t); \
  template hipError_t launch_step_node<R>(const Tables&, const void*, void*, const void*, hipStream_t); \
  template hipError_t launch_init<R>(const Tables&, const double*, const double*, const double*,  \
                                     const double*, void*, int*, hipStream_t);                    \
  template hipError_t launch_fields<R>(const Tables&, const void*, double*, double*, double*,     \
                                       double*, hipStream_t);                                     \
  template hipError_t launch_diag<R>(const Tables&, const void*, double*, double, double*, hipStream_t); \
  template hipError_t launch_noneq<R>(const Tables&, const void*, int, double*, hipStream_t);
PCLB_INST(float)
PCLB_INST(double)
#undef PCLB_INST

}  // namespace pclb
