// Deterministic diagnostics reduction shared by the diagnostics kernels:
// compensated (TwoSum) per-thread sums, a block tree of (sum, error) pairs
// into one slot row per block, and a one-block fixed-order final pass
// (launch_diag_final).
#pragma once

#include <hip/hip_runtime.h>

namespace pclb {

struct TwoS {
  double s, c;
};
__device__ inline void two_add(TwoS& a, double x) {
  double s = a.s + x;
  double bb = s - a.s;
  double err = (a.s - (s - bb)) + (x - bb);
  a.s = s;
  a.c += err;
}
__device__ inline TwoS two_merge(TwoS a, TwoS b) {
  TwoS r = a;
  two_add(r, b.s);
  r.c += b.c;
  return r;
}

constexpr int DIAG_BLOCK = 256;
constexpr int DIAG_SLOTS = 11;   // 4 x (sum, err), min rho, min T, bad count

// Block reduction of the per-thread partials into partial[blockIdx.x][0..10];
// every thread of the block calls it.
__device__ inline void diag_block_reduce(const TwoS acc[4], double rmin, double tmin, double bad,
                                         double* __restrict__ partial) {
  __shared__ double sh[DIAG_SLOTS][DIAG_BLOCK];
  for (int a = 0; a < 4; ++a) { sh[2 * a][threadIdx.x] = acc[a].s; sh[2 * a + 1][threadIdx.x] = acc[a].c; }
  sh[8][threadIdx.x] = rmin;
  sh[9][threadIdx.x] = tmin;
  sh[10][threadIdx.x] = bad;
  __syncthreads();
  for (int w = DIAG_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      int o = threadIdx.x + w;
      for (int a = 0; a < 4; ++a) {
        TwoS x{sh[2 * a][threadIdx.x], sh[2 * a + 1][threadIdx.x]};
        TwoS y{sh[2 * a][o], sh[2 * a + 1][o]};
        TwoS z = two_merge(x, y);
        sh[2 * a][threadIdx.x] = z.s;
        sh[2 * a + 1][threadIdx.x] = z.c;
      }
      sh[8][threadIdx.x] = fmin(sh[8][threadIdx.x], sh[8][o]);
      sh[9][threadIdx.x] = fmin(sh[9][threadIdx.x], sh[9][o]);
      sh[10][threadIdx.x] += sh[10][o];
    }
    __syncthreads();
  }
  if (threadIdx.x < DIAG_SLOTS) partial[(size_t)blockIdx.x * DIAG_SLOTS + threadIdx.x] = sh[threadIdx.x][0];
}

// out[0..7] = mass, momentum x, y, energy, min rho, min T, non-finite nodes,
// step, from nb slot rows of partials.
hipError_t launch_diag_final(const double* partial, int nb, double step, double* out, hipStream_t s);

}  // namespace pclb
