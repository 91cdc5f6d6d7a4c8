// Strip kernel of the combined-scheme step (Eq. combined_scheme) for FP64
// storage, full annulus, MWB scheme (and the three schemes it is compared
// with: Warming-Beam, Lax-Wendroff and second-order upwind).  A workgroup owns a
// strip of 64 theta columns (one per lane; n_theta a multiple of 64) and
// marches in r over a chunk of rows.  Four wavefronts share the strip, wave W owning the direction
// pair (W, W + 4): the eight velocities (k, W) and (k, W + 4), k = 1..4, and
// wave 0 also the rest velocity.  For each owned velocity a wave keeps six
// rows in registers, i-2 .. i+3 at row i: the radial stencil of either upwind
// side (rows i-2 .. i+2) and one row of look-ahead, so every f value of the
// chunk is read from HBM once and every load is issued two rows before its
// first use.  The ring's roles rotate at compile time (the row loop is
// unrolled six times), so no register is moved.
//
// Per row: each wave forms the moment partials of its pair (d4_partial), the
// partials meet in LDS (one barrier per row, double-buffered by row parity),
// and every wave builds the node's equilibrium from their fixed-order sum
// (combine_partials, eq_setup) and updates its own velocities with the same
// arithmetic as the node kernel (relax_pair, courant, the scheme's terms), so both
// kernels give the same FP64 result bit for bit.  Azimuthal neighbours come
// from the adjacent lanes (ds_bpermute of the centre row); the two columns
// beyond each end of the strip come from a halo read one row ahead with one
// 16-byte load per lane (lane v: the pair left of the strip for velocity v,
// lane 8 + v: the pair right of it), which the edge lanes fetch with
// ds_bpermute as well.
#include <type_traits>

#include "common.h"
#include "launch.h"
#include "strip_common.h"

namespace pclb {

namespace {

using namespace strip;

constexpr int S64_WAVES = 4;   // one wave per direction pair
constexpr int S64_NV = 8;      // velocities per wave
constexpr int S64_RING = 6;    // rows i-2 .. i+3

struct S64Ctx {
  const double* f;
  double* out;
  const double* ghost;
  size_t plane;
  int nr, nth, j, lane;
};

// Plane of the wave's velocity v = 2 (k - 1) + h: direction W + 4 h, speed k.
template <int W>
__device__ constexpr int s64_q(int v) {
  return qidx((v >> 1) + 1, W + 4 * (v & 1));
}

// Velocity q at row `row` of this lane's column: rows beyond the walls from
// the ghost layers.  Only rows -2 .. nr + 1 are ever asked for.
__device__ inline double s64_load(const S64Ctx& X, int q, int row) {
  if (row < 0) return X.ghost[ghost_index(0, -1 - row, q, X.j, X.nth)];
  if (row >= X.nr) return X.ghost[ghost_index(1, row - X.nr, q, X.j, X.nth)];
  return X.f[q * X.plane + (size_t)row * X.nth + X.j];
}

// Halo of row `row` (a real row): lane v < 8 reads velocity v's pair of
// columns (j0 - 2, j0 - 1), lane 8 + v the pair (j0 + 64, j0 + 65), wrapped
// around the ring; the other lanes repeat lane (lane mod 16)'s read.
template <int W>
__device__ inline double2 s64_halo(const S64Ctx& X, int j0, int row) {
  const int hl = X.lane & 15, v = hl & 7;
  int c = hl < 8 ? j0 - 2 : j0 + 64;
  c = c < 0 ? c + X.nth : (c >= X.nth ? c - X.nth : c);
  return *reinterpret_cast<const double2*>(X.f + s64_q<W>(v) * X.plane + (size_t)row * X.nth + c);
}

// a where m is all ones, b where it is zero, formed on the bits: a plain
// select between two ring slots lets the compiler select their addresses and
// keep the ring in scratch memory
__device__ inline double pick(uint64_t m, double a, double b) {
  return __builtin_bit_cast(double, (__builtin_bit_cast(uint64_t, a) & m) | (__builtin_bit_cast(uint64_t, b) & ~m));
}

template <int W, int SCH>
__device__ inline void s64_march(const Tables& T, const S64Ctx& X, int j0, int i0, int i1,
                                 double* lds) {
  constexpr int d4 = W;
  const int lane = X.lane;
  // geometry of the column: Courant factors per unit speed and upwind sides
  DirGeom<double> G;
  dir_geometry(T.cth[X.j], T.sth[X.j], octant_of(X.j, X.nth, ND), T.dt_dr, T.dt_dth, G);
  const double e = T.e, ome = 1.0 - T.e;
  // per member h of the pair: radial upwind side (all ones where backward),
  // the lanes one and two upwind in theta, the halo lane base of the upwind
  // side (0: left pairs, 8: right pairs), and whether this lane's u1 lies
  // beyond the strip (e1) or its u2 is the first column beyond it (e2)
  uint64_t rm[2];
  int a1[2], a2[2], eb[2], dn[2], ebd[2];
  bool e1[2], e2[2], ed[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    rm[h] = ((G.rback >> (d4 + 4 * h)) & 1u) ? ~0ull : 0ull;
    const bool tb = (G.tback >> (d4 + 4 * h)) & 1u;
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
  const bool left_lane = (lane & 15) < 8;   // lanes holding a left halo pair
  // the ring: S[s][v] holds row (i - 2 + s) at slot (u + s) mod 6 of row i = ib + u
  double S[S64_RING][S64_NV];
  const int last = i1 + 1;   // the furthest row any update of the chunk reads
#pragma unroll
  for (int s = 0; s < S64_RING; ++s) {
    const int row = i0 - 2 + s;
#pragma unroll
    for (int v = 0; v < S64_NV; ++v) S[s][v] = row <= last ? s64_load(X, s64_q<W>(v), row) : 0.0;
  }
  double r0 = 0.0;
  if constexpr (W == 0) r0 = X.f[(size_t)i0 * X.nth + X.j];
  double2 hv = s64_halo<W>(X, j0, i0);
  for (int ib = i0; ib < i1; ib += S64_RING) {
#pragma unroll
    for (int u = 0; u < S64_RING; ++u) {
      const int i = ib + u;
      if (i >= i1) break;
      auto slot = [&](int s, int v) -> double { return S[(u + s) % S64_RING][v]; };
      // next row's halo and rest value, issued before this row's work
      const double2 hcur = hv;
      if (i + 1 < i1) hv = s64_halo<W>(X, j0, i + 1);
      double rcur = r0;
      if constexpr (W == 0) {
        if (i + 1 < i1) r0 = X.f[(size_t)(i + 1) * X.nth + X.j];
      }
      // moment partials of the pair (d4, d4 + 4), exchanged through LDS
      double P[4][4];
      {
        double fp[NK], fm[NK];
#pragma unroll
        for (int k = 1; k <= NK; ++k) {
          fp[k - 1] = slot(2, 2 * (k - 1));
          fm[k - 1] = slot(2, 2 * (k - 1) + 1);
        }
        d4_partial(d4, fp, fm, P[d4]);
      }
      double* buf = lds + (i & 1) * (17 * 64);
#pragma unroll
      for (int a = 0; a < 4; ++a) buf[(d4 * 4 + a) * 64 + lane] = P[d4][a];
      if constexpr (W == 0) buf[16 * 64 + lane] = rcur;
      __syncthreads();
      if constexpr (W != 0) rcur = buf[16 * 64 + lane];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        if (d == d4) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a) P[d][a] = buf[(d * 4 + a) * 64 + lane];
      }
      double rho, ux, uy, E;
      combine_partials(P, rcur, rho, ux, uy, E);
      EqCoef ec;
      eq_setup(T, rho, ux, uy, E, ec);
      const size_t c0 = (size_t)i * X.nth + X.j;
      if constexpr (W == 0)
        __builtin_nontemporal_store(relax_rest<double>(relax_rest_share(ec, ome), e, rcur), X.out + c0);
      // halo by role: H1 the column next to the strip (j0 - 1 / j0 + 64), H2
      // the one beyond it (j0 - 2 / j0 + 65)
      const double H1 = left_lane ? hcur.y : hcur.x, H2 = left_lane ? hcur.x : hcur.y;
      const double rinv = T.rinv[i];
      const double atr = G.at[d4] * rinv;
#pragma unroll
      for (int k = 1; k <= NK; ++k) {
        const int v0 = 2 * (k - 1);
        double rel[2];
        // relax_pair needs its speed at compile time
        switch (k) {
          case 1: relax_pair<1>(ec, e, ome, ec.p[d4], slot(2, v0), slot(2, v0 + 1), rel[0], rel[1]); break;
          case 2: relax_pair<2>(ec, e, ome, ec.p[d4], slot(2, v0), slot(2, v0 + 1), rel[0], rel[1]); break;
          case 3: relax_pair<3>(ec, e, ome, ec.p[d4], slot(2, v0), slot(2, v0 + 1), rel[0], rel[1]); break;
          default: relax_pair<4>(ec, e, ome, ec.p[d4], slot(2, v0), slot(2, v0 + 1), rel[0], rel[1]);
        }
        double aCr, Kr, aCt, Kt;
        courant<double>(speed(k), G.ar[d4], aCr, Kr);
        courant<double>(speed(k), atr, aCt, Kt);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int v = v0 + h;
          const double c = slot(2, v);
          const double u1r = pick(rm[h], slot(1, v), slot(3, v));
          const double u2r = pick(rm[h], slot(0, v), slot(4, v));
          // azimuthal neighbours: adjacent lanes; the strip's edge lanes take
          // velocity v's halo of their upwind side
          const double z1 = __shfl(c, a1[h]), z2 = __shfl(c, a2[h]);
          const double g1 = __shfl(H1, eb[h] + v), g2 = __shfl(H2, eb[h] + v);
          const double u1t = e1[h] ? g1 : z1;
          const double u2t = e1[h] ? g2 : (e2[h] ? g1 : z2);
          double res;
          if constexpr (SCH == SCH_LW) {
            const double w1r = pick(rm[h], slot(3, v), slot(1, v));
            const double zd = __shfl(c, dn[h]), gd = __shfl(H1, ebd[h] + v);
            const double w1t = ed[h] ? gd : zd;
            const double tr = conv_term<SCH_LW, double>(aCr, Kr, c, u1r, u2r, w1r);
            const double tt = conv_term<SCH_LW, double>(aCt, Kt, c, u1t, u2t, w1t);
            res = (rel[h] - tr) - tt;
          } else {
            res = scheme_update_d<SCH, double>(rel[h], aCr, Kr, c - u1r, u1r - u2r, aCt, Kt, c - u1t,
                                               u1t - u2t);
          }
          __builtin_nontemporal_store(res, X.out + s64_q<W>(v) * X.plane + c0);
        }
      }
      // look-ahead: row i + 4 into the slot of row i - 2
      const int row = i + 4;
      if (row <= last) {
#pragma unroll
        for (int v = 0; v < S64_NV; ++v) S[u % S64_RING][v] = s64_load(X, s64_q<W>(v), row);
      }
    }
  }
}

template <int SCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
step_strip64_kernel(Tables T, const double* __restrict__ f, double* __restrict__ out,
                    const double* __restrict__ ghost, int chunk, int xcd_order) {
  __shared__ double lds[2 * 17 * 64];
  const int nstrip = T.nth / WAVE;
  const int item = work_item(xcd_order);
  const int strip = item % nstrip, ck = item / nstrip;
  const int j0 = strip * WAVE;
  const int i0 = ck * chunk, i1 = min(i0 + chunk, T.nr);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const S64Ctx X{f, out, ghost, (size_t)T.nr * T.nth, T.nr, T.nth, j0 + lane, lane};
  switch (w) {
    case 0: s64_march<0, SCH>(T, X, j0, i0, i1, lds); break;
    case 1: s64_march<1, SCH>(T, X, j0, i0, i1, lds); break;
    case 2: s64_march<2, SCH>(T, X, j0, i0, i1, lds); break;
    default: s64_march<3, SCH>(T, X, j0, i0, i1, lds);
  }
}

}  // namespace

bool strip64_supported(const Tables& T) {
  // full annulus, whole strips, every scheme (the ring holds both radial
  // sides and the halo both azimuthal ones)
  return T.nf == ND && T.nth >= WAVE && T.nth % WAVE == 0;
}

hipError_t launch_step_strip64(const Tables& T, const void* f, void* out, const void* ghost,
                               const StripTune& tune, hipStream_t s) {
  int chunk = tune.chunk > 0 ? tune.chunk : 32;
  const int strips = T.nth / WAVE;
  while (tune.chunk <= 0 && chunk > 8 && (long)strips * ((T.nr + chunk - 1) / chunk) < 4096) chunk /= 2;
  const int chunks = (T.nr + chunk - 1) / chunk;
  const int order = tune.order < 0 ? 1 : tune.order;
  const dim3 grid(strips * chunks), block(S64_WAVES * WAVE);
  const double* fi = (const double*)f;
  const double* gh = (const double*)ghost;
  double* fo = (double*)out;
  if (T.scheme == SCH_WB)
    hipLaunchKernelGGL((step_strip64_kernel<SCH_WB>), grid, block, 0, s, T, fi, fo, gh, chunk, order);
  else if (T.scheme == SCH_UPWIND2)
    hipLaunchKernelGGL((step_strip64_kernel<SCH_UPWIND2>), grid, block, 0, s, T, fi, fo, gh, chunk, order);
  else if (T.scheme == SCH_LW)
    hipLaunchKernelGGL((step_strip64_kernel<SCH_LW>), grid, block, 0, s, T, fi, fo, gh, chunk, order);
  else
    hipLaunchKernelGGL((step_strip64_kernel<SCH_MWB>), grid, block, 0, s, T, fi, fo, gh, chunk, order);
  return hipGetLastError();
}

}  // namespace pclb
