// Adjoint kernels of the combined-scheme step: one thread per wall column
// (ghost adjoint) and one thread per node (node adjoint); the arithmetic is
// in adjoint_node.h.
#include <type_traits>

#include "adjoint_node.h"
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
  if (j >= T.nth) return;
  ghost_adjoint_column<R>(T, bc, f, lam, ghost, tie, blockIdx.y, j, gm);
}

// ---------------------------------------------------------------------------
// Node adjoint: one thread per node m, gather over every output whose stencil
// holds m.
template <class R, bool SECTOR>
__global__ void __launch_bounds__(128) adjoint_node_kernel(Tables T, const R* __restrict__ f,
                                                           const R* __restrict__ lam,
                                                           const R* __restrict__ ghost,
                                                           const double* __restrict__ gm,
                                                           double tie, R* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= T.nth) return;
  adjoint_node<R, SECTOR>(T, f, lam, ghost, gm, tie, blockIdx.y, j, out);
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
                          void* lam_out, void* ghost, double* gm, double tie,
                          const StripTune& tune, bool strip, hipStream_t s) {
  hipError_t e = launch_ghost<R>(T, bc, f, ghost, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ghost_adjoint_kernel<R>, dim3((T.nth + 127) / 128, 2), dim3(128), 0, s, T, bc,
                     (const R*)f, (const R*)lam, (const R*)ghost, tie, gm);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (strip && adjoint_strip_supported(T, std::is_same<R, float>::value ? 32 : 64))
    return launch_adjoint_strip<R>(T, f, lam, lam_out, ghost, gm, tie, tune, s);
  const dim3 grid((T.nth + 127) / 128, T.nr);
  if (T.nf == 8)
    hipLaunchKernelGGL((adjoint_node_kernel<R, false>), grid, dim3(128), 0, s, T, (const R*)f,
                       (const R*)lam, (const R*)ghost, (const double*)gm, tie, (R*)lam_out);
  else
    hipLaunchKernelGGL((adjoint_node_kernel<R, true>), grid, dim3(128), 0, s, T, (const R*)f,
                       (const R*)lam, (const R*)ghost, (const double*)gm, tie, (R*)lam_out);
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
                                          void*, double*, double, const StripTune&, bool, hipStream_t);
template hipError_t launch_adjoint<double>(const Tables&, const BCdev&, const void*, const void*, void*,
                                           void*, double*, double, const StripTune&, bool, hipStream_t);
template hipError_t launch_adjoint_init<float>(const Tables&, const void*, const double*, const double*,
                                               const double*, const double*, double*, double*, double*,
                                               double*, hipStream_t);
template hipError_t launch_adjoint_init<double>(const Tables&, const void*, const double*, const double*,
                                                const double*, const double*, double*, double*, double*,
                                                double*, hipStream_t);

}  // namespace pclb
