// Strip form of the adjoint step for FP32 states (full annulus, MWB, n_theta
// a multiple of 64).  The node kernel gathers, for each node m and velocity,
// the derivatives of the six convection stencils that contain m and so
// evaluates every stencil's derivative three times; here every stencil is
// differentiated once, by the lane that owns its centre, and its three
// products with the cotangent of its output are handed to the nodes they
// belong to:
//   lam_t(m) = e lam(m) + sum_a gM_a(m) phi_a(q)
//            - sum over stencils n holding m of lam_q(n) dT_q(n)/df_q(m).
//
// A workgroup owns a strip of 64 theta columns (one per lane) and the rows
// [i0, i1) of a chunk; eight wavefronts share it, wave W + 4 KH owning the
// four velocities of direction pair (W, W + 4) with speeds 2 KH + 1 and
// 2 KH + 2 (wave 0 also the rest velocity).  The march visits the stencil
// rows i0 - 2 .. i1 + 1: the radial stencils of the two rows on either side
// of the chunk also reach into it.  Per velocity a wave keeps six rows of f
// (i-2 .. i+3) and three rows of pending results, whose meaning depends on
// the lane's radial upwind side:
//   backward (stencil i, i-1, i-2): slots = rows (i-2, i-1, i), the lowest
//     complete after stencil row i;
//   forward  (stencil i, i+1, i+2): slots = rows (i, i+1, i+2), the lowest
//     complete after stencil row i.
// Either way stencil row i adds dc to the slot of row i, du1 to the middle
// slot and du2 to the remaining one, and the lowest slot is stored.
//
// Per owned row the waves exchange their moment partials through LDS (the
// Jacobian of f^eq needs the node's moments), then the partial cotangents of
// the moments (G = sum_q (1 - e) lam_q df^eq_q/d(rho, u, E)), two barriers
// per row; the partials of a direction pair are added speed half by speed
// half, so the moments may differ from the forward kernels' in the last
// bit.  Azimuthally, lane j differentiates its own stencil (neighbours from
// the adjacent lanes and a halo read one row ahead, as in the forward
// kernel) and the products travel to the lanes one and two columns upwind;
// the stencils centred in the two columns beyond each end of the strip that
// reach into it are differentiated by the halo lanes (lane v: the left pair
// of velocity v, lane 4 + v: the right pair).
//
// The derivatives, their products with the cotangents, the lane exchange and
// the pending results are in the state's precision (the products are
// rounded to float before they are summed, about 1e-7 of the largest
// cotangent around an entry); the relaxation and f^eq parts are in FP64.
// An FP64 form of the same kernel needs more than 256 registers per lane, so
// FP64 states keep the node kernel.
#include <type_traits>

#include "adjoint.h"
#include "common.h"
#include "launch.h"
#include "strip_common.h"

namespace pclb {

namespace {

using namespace strip;

constexpr int AS_WAVES = 8;
constexpr int AS_NV = 4;       // velocities per wave
constexpr int AS_RING = 6;     // rows i-2 .. i+3 of f
constexpr int AS_LDS_A = 33 * 64;   // moment partials (8 x 4) and the rest velocity
constexpr int AS_LDS_B = 32 * 64;   // cotangent partials (8 x 4)

template <class R>
struct AsCtx {
  const R* f;
  const R* lam;
  R* out;
  const R* ghost;
  const double* gm;
  size_t plane;
  int nr, nth, j, lane;
};

template <class R>
using Pair = std::conditional_t<std::is_same_v<R, float>, float2, double2>;

// Plane of the wave's velocity v = 2 (k - 2 KH - 1) + h: direction W + 4 h,
// speed k.
template <int W, int KH>
__device__ constexpr int as_q(int v) {
  return qidx(2 * KH + (v >> 1) + 1, W + 4 * (v & 1));
}

// Velocity q at row `row` of this lane's column (rows -2 .. nr + 1; beyond
// the walls from the ghost layers).
template <class R>
__device__ inline R as_f(const AsCtx<R>& X, int q, int row) {
  if (row < 0) return X.ghost[ghost_index(0, -1 - row, q, X.j, X.nth)];
  if (row >= X.nr) return X.ghost[ghost_index(1, row - X.nr, q, X.j, X.nth)];
  return X.f[q * X.plane + (size_t)row * X.nth + X.j];
}

template <class R>
__device__ inline Pair<R> as_pair(const R* base, size_t off) {
  return *reinterpret_cast<const Pair<R>*>(base + off);
}

// a where m is all ones, b where it is zero, formed on the bits (a select
// between ring slots would let the compiler select their addresses and keep
// the ring in scratch memory)
__device__ inline double pick(uint64_t m, double a, double b) {
  return __builtin_bit_cast(double, (__builtin_bit_cast(uint64_t, a) & m) | (__builtin_bit_cast(uint64_t, b) & ~m));
}
__device__ inline float pick(uint64_t m, float a, float b) {
  const uint32_t m32 = (uint32_t)m;
  return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, a) & m32) | (__builtin_bit_cast(uint32_t, b) & ~m32));
}

__device__ inline int wrapc(int c, int nth) { return c < 0 ? c + nth : (c >= nth ? c - nth : c); }

template <class R, int W, int KH>
__device__ inline void as_march(const Tables& T, const AsCtx<R>& X, int j0, int i0, int i1,
                                double tie, double* ldsA, double* ldsB) {
  using A = R;                    // arithmetic of the MWB derivatives
  constexpr int d4 = W;
  const int lane = X.lane, nr = X.nr, nth = X.nth;
  const A TEa = (A)tie;
  const double e = T.e, ome = 1.0 - T.e;
  DirGeom<double> G;
  dir_geometry(T.cth[X.j], T.sth[X.j], octant_of(X.j, nth, ND), T.dt_dr, T.dt_dth, G);
  // per member h of the pair: radial upwind side (mask of ones where
  // backward), the azimuthal one, the lanes one and two upwind in theta, the
  // halo lane base of the upwind side, and whether u1 (e1) or u2 (e2) of
  // this lane's own stencil lies beyond the strip
  uint64_t rm[2];
  bool tbk[2], e1[2], e2[2];
  int a1[2], a2[2], eb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    rm[h] = ((G.rback >> (d4 + 4 * h)) & 1u) ? ~0ull : 0ull;
    const bool tb = (G.tback >> (d4 + 4 * h)) & 1u;
    tbk[h] = tb;
    const int sc = tb ? -1 : 1;
    a1[h] = (lane + sc) & 63;
    a2[h] = (lane + 2 * sc) & 63;
    eb[h] = tb ? 0 : 4;
    e1[h] = tb ? lane == 0 : lane == 63;
    e2[h] = tb ? lane == 1 : lane == 62;
  }
  // halo lanes: hs = 0 the pair left of the strip (far j0 - 2, near j0 - 1),
  // 1 the pair right of it (near j0 + 64, far j0 + 65), for velocity hv
  const int hl = lane & 7, hv = hl & 3, hs = hl >> 2;
  const int hdir = d4 + 4 * (hv & 1);
  const double hvk = speed(2 * KH + (hv >> 1) + 1);
  const int cnear = wrapc(hs ? j0 + 64 : j0 - 1, nth), cfar = wrapc(hs ? j0 + 65 : j0 - 2, nth);
  // |v_theta| dt/dtheta per unit speed of the pair's directions in the two
  // halo columns, as dir_geometry forms it, and whether their stencils reach
  // into the strip (left: forward upwind, right: backward upwind)
  const double at_near = fabs(sin_d(d4) * T.cth[cnear] - cos_d(d4) * T.sth[cnear]) * T.dt_dth;
  const double at_far = fabs(sin_d(d4) * T.cth[cfar] - cos_d(d4) * T.sth[cfar]) * T.dt_dth;
  const bool tb_near = (tback_bits(octant_of(cnear, nth, ND)) >> hdir) & 1u;
  const bool tb_far = (tback_bits(octant_of(cfar, nth, ND)) >> hdir) & 1u;
  const bool in_near = hs ? tb_near : !tb_near, in_far = hs ? tb_far : !tb_far;
  // halo pair offsets within a row: outer (far, near) pair and the strip's
  // edge pair on the same side
  const int co = hs ? wrapc(j0 + 64, nth) : wrapc(j0 - 2, nth);
  const int ci = hs ? j0 + 62 : j0;
  const size_t hplane = (size_t)as_q<W, KH>(hv) * X.plane;

  const int s0 = i0 - 2, s1 = i1 + 1;        // stencil rows visited
  const int flast = min(i1 + 3, nr + 1);     // the furthest f row read
  auto real = [&](int i) { return i >= 0 && i < nr; };
  auto owned = [&](int i) { return i >= i0 && i < i1; };

  // the f ring: S[s][v] holds row (i - 2 + s) at slot (u + s) mod 6 of row i = ib + u
  A S[AS_RING][AS_NV];
#pragma unroll
  for (int s = 0; s < AS_RING; ++s) {
    const int row = s0 - 2 + s;
#pragma unroll
    for (int v = 0; v < AS_NV; ++v)
      S[s][v] = (row >= -2 && row <= flast) ? as_f(X, as_q<W, KH>(v), row) : (A)0;
  }
  // cotangents of the current and the next stencil row
  A Ln[AS_NV], Lc[AS_NV];
  A l0n = 0, l0c = 0;                        // rest velocity (wave 0)
#pragma unroll
  for (int v = 0; v < AS_NV; ++v) Ln[v] = real(s0) ? X.lam[as_q<W, KH>(v) * X.plane + (size_t)s0 * nth + X.j] : (A)0;
  // halo of the next owned row: f outer pair, f edge pair, lambda outer pair
  Pair<R> hfo{}, hfi{}, hlo{};
  auto load_halo = [&](int row) {
    const size_t rb = hplane + (size_t)row * nth;
    hfo = as_pair(X.f, rb + co);
    hfi = as_pair(X.f, rb + ci);
    hlo = as_pair(X.lam, rb + co);
  };
  // pending results: Acc[(u + s) mod 3] is slot s at row ib + u
  A Acc[3][AS_NV];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int v = 0; v < AS_NV; ++v) Acc[s][v] = (A)0;

  for (int ib = s0; ib <= s1; ib += AS_RING) {
#pragma unroll
    for (int u = 0; u < AS_RING; ++u) {
      const int i = ib + u;
      if (i > s1) break;
      auto slot = [&](int s, int v) -> A { return S[(u + s) % AS_RING][v]; };
      A* A0 = Acc[u % 3];
      A* A1 = Acc[(u + 1) % 3];
      A* A2 = Acc[(u + 2) % 3];
      // cotangents of this row; the next row's issued now
#pragma unroll
      for (int v = 0; v < AS_NV; ++v) Lc[v] = Ln[v];
      const bool nxt = real(i + 1) && i + 1 <= s1;
#pragma unroll
      for (int v = 0; v < AS_NV; ++v)
        Ln[v] = nxt ? X.lam[as_q<W, KH>(v) * X.plane + (size_t)(i + 1) * nth + X.j] : (A)0;
      if constexpr (W == 0 && KH == 0) {
        l0c = l0n;
        l0n = owned(i + 1) ? X.lam[(size_t)(i + 1) * nth + X.j] : (A)0;
      }
      const Pair<R> cfo = hfo, cfi = hfi, clo = hlo;
      if (owned(i + 1)) load_halo(i + 1);

      if (owned(i)) {
        // ---- moments of the node (exchange 1) and the Jacobian of f^eq
        double* bA = ldsA + (i & 1) * AS_LDS_A;
        {
          // this wave's share of the pair partial (as d4_partial, two speeds)
          double pr = 0.0, pjx = 0.0, pjy = 0.0, pe = 0.0;
#pragma unroll
          for (int kk = 0; kk < 2; ++kk) {
            const int k = 2 * KH + kk + 1;
            const double fpv = (double)slot(2, 2 * kk), fmv = (double)slot(2, 2 * kk + 1);
            const double sp = fpv + fmv, sm = fpv - fmv;
            pr += sp;
            if (cos_d(d4) != 0.0) pjx += (speed(k) * cos_d(d4)) * sm;
            if (sin_d(d4) != 0.0) pjy += (speed(k) * sin_d(d4)) * sm;
            pe += (speed(k) * speed(k)) * sp;
          }
          const int wv = W * 2 + KH;
          bA[(wv * 4 + 0) * 64 + lane] = pr;
          bA[(wv * 4 + 1) * 64 + lane] = pjx;
          bA[(wv * 4 + 2) * 64 + lane] = pjy;
          bA[(wv * 4 + 3) * 64 + lane] = pe;
        }
        double r0 = 0.0;
        if constexpr (W == 0 && KH == 0) {
          r0 = (double)X.f[(size_t)i * nth + X.j];
          bA[32 * 64 + lane] = r0;
        }
        __syncthreads();
        if constexpr (W != 0 || KH != 0) r0 = bA[32 * 64 + lane];
        double P[4][4];
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
          for (int a = 0; a < 4; ++a)
            P[d][a] = bA[((d * 2 + 0) * 4 + a) * 64 + lane] + bA[((d * 2 + 1) * 4 + a) * 64 + lane];
        double rho, ux, uy, E;
        combine_partials(P, r0, rho, ux, uy, E);
        double Gm[4];
        {
          FeqJac J;
          feq_jac_setup(T, rho, ux, uy, E, J);
          double Gp[4] = {0.0, 0.0, 0.0, 0.0};
          if constexpr (W == 0 && KH == 0) feq_jac_accum<0>(J, ome * (double)l0c, Gp);
          for_v<0, AS_NV>([&](auto vc) {
            constexpr int v = decltype(vc)::value;
            feq_jac_accum<as_q<W, KH>(v)>(J, ome * (double)Lc[v], Gp);
          });
          // ---- cotangent partials (exchange 2), summed in wave order
          double* bB = ldsB + (i & 1) * AS_LDS_B;
#pragma unroll
          for (int a = 0; a < 4; ++a) bB[((W * 2 + KH) * 4 + a) * 64 + lane] = Gp[a];
          __syncthreads();
          double Gs[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            double g = bB[a * 64 + lane];
#pragma unroll
            for (int wv = 1; wv < AS_WAVES; ++wv) g += bB[(wv * 4 + a) * 64 + lane];
            Gs[a] = g;
          }
          to_moment_cotangent(rho, ux, uy, E, Gs, Gm);
        }
        // the ghost layers' share of the two rows next to each wall
        if (i <= 1) {
#pragma unroll
          for (int a = 0; a < 4; ++a) Gm[a] += X.gm[((size_t)i * 4 + a) * nth + X.j];
        }
        if (i >= nr - 2) {
          const int s = nr - 1 - i;
#pragma unroll
          for (int a = 0; a < 4; ++a) Gm[a] += X.gm[((size_t)(2 + s) * 4 + a) * nth + X.j];
        }
        if constexpr (W == 0 && KH == 0) X.out[(size_t)i * nth + X.j] = (R)(e * (double)l0c + Gm[0]);

        // ---- halo lanes: the stencils centred beyond the strip's ends
        const double rinv = T.rinv[i];
        const bool left = hs == 0;
        const A o_near = left ? cfo.y : cfo.x, o_far = left ? cfo.x : cfo.y;
        const A i_near = left ? cfi.x : cfi.y, i_next = left ? cfi.y : cfi.x;
        const A l_near = left ? clo.y : clo.x, l_far = left ? clo.x : clo.y;
        A xe, xn;
        {
          const double cn = hvk * (at_near * rinv), cf = hvk * (at_far * rinv);
          const MwbDT<A> gn = mwb_grad_t<A>((A)cn, (A)(cn - cn * cn), o_near, i_near, i_next, TEa);
          const MwbDT<A> gf = mwb_grad_t<A>((A)cf, (A)(cf - cf * cf), o_far, o_near, i_near, TEa);
          const A tn1 = in_near ? l_near * gn.du1 : (A)0;
          const A tn2 = in_near ? l_near * gn.du2 : (A)0;
          const A tf2 = in_far ? l_far * gf.du2 : (A)0;
          xe = tn1 + tf2;      // to the edge column (lane 0 or 63)
          xn = tn2;            // to the next one (lane 1 or 62)
        }
        // halo f values by role for the own stencils of the edge lanes
        const A H1 = o_near, H2 = o_far;
        const double atr = G.at[d4] * rinv;

        for_v<0, AS_NV>([&](auto vc) {
          constexpr int v = decltype(vc)::value;
          constexpr int h = v & 1, k = 2 * KH + (v >> 1) + 1;
          constexpr int q = as_q<W, KH>(v);
          const A lq = Lc[v];
          A loc = (A)(e * (double)lq + Gm[0] + Gm[1] * vx_q(q) + Gm[2] * vy_q(q) + Gm[3] * 0.5 * v2_q(q));
          // own azimuthal stencil
          const A c = slot(2, v);
          const A z1 = __shfl(c, a1[h]), z2 = __shfl(c, a2[h]);
          const A g1 = __shfl(H1, eb[h] + v), g2 = __shfl(H2, eb[h] + v);
          const A u1t = e1[h] ? g1 : z1;
          const A u2t = e1[h] ? g2 : (e2[h] ? g1 : z2);
          double aCt, Kt;
          courant<double>(speed(k), atr, aCt, Kt);
          const MwbDT<A> gt = mwb_grad_t<A>((A)aCt, (A)Kt, c, u1t, u2t, TEa);
          loc -= lq * gt.dc;
          const A t1 = lq * gt.du1, t2 = lq * gt.du2;
          const A sb1 = tbk[h] ? t1 : (A)0, sf1 = tbk[h] ? (A)0 : t1;
          const A sb2 = tbk[h] ? t2 : (A)0, sf2 = tbk[h] ? (A)0 : t2;
          // products from the stencils one and two columns away in the strip
          A rcv = 0;
          {
            const A p1b = __shfl(sb1, (lane + 1) & 63), p1f = __shfl(sf1, (lane - 1) & 63);
            const A p2b = __shfl(sb2, (lane + 2) & 63), p2f = __shfl(sf2, (lane - 2) & 63);
            rcv += lane == 63 ? (A)0 : p1b;
            rcv += lane == 0 ? (A)0 : p1f;
            rcv += lane >= 62 ? (A)0 : p2b;
            rcv += lane <= 1 ? (A)0 : p2f;
          }
          // and from the halo lanes' stencils beyond the ends
          {
            const A le = __shfl(xe, v), ln = __shfl(xn, v);
            const A re = __shfl(xe, 4 + v), rn = __shfl(xn, 4 + v);
            rcv += lane == 0 ? le : (lane == 63 ? re : (A)0);
            rcv += lane == 1 ? ln : (lane == 62 ? rn : (A)0);
          }
          loc -= rcv;
          // into the slot of row i: the highest where radially backward
          A2[v] += pick(rm[h], loc, (A)0);
          A0[v] += pick(rm[h], (A)0, loc);
        });
      }

      // ---- radial stencils of row i (every real row of the march)
      if (real(i)) {
        for_v<0, AS_NV>([&](auto vc) {
          constexpr int v = decltype(vc)::value;
          constexpr int h = v & 1, k = 2 * KH + (v >> 1) + 1;
          double aCr, Kr;
          courant<double>(speed(k), G.ar[d4], aCr, Kr);
          const A c = slot(2, v);
          const A u1 = pick(rm[h], slot(1, v), slot(3, v));
          const A u2 = pick(rm[h], slot(0, v), slot(4, v));
          const MwbDT<A> g = mwb_grad_t<A>((A)aCr, (A)Kr, c, u1, u2, TEa);
          const A lq = Lc[v];
          const A tdc = lq * g.dc, t1 = lq * g.du1, t2 = lq * g.du2;
          A0[v] -= pick(rm[h], t2, tdc);
          A1[v] -= t1;
          A2[v] -= pick(rm[h], tdc, t2);
        });
      }

      // ---- the lowest slot is complete: row i - 2 (backward) or i (forward)
      for_v<0, AS_NV>([&](auto vc) {
        constexpr int v = decltype(vc)::value;
        constexpr int h = v & 1;
        const int row = rm[h] ? i - 2 : i;
        if (owned(row)) __builtin_nontemporal_store((R)A0[v], X.out + as_q<W, KH>(v) * X.plane + (size_t)row * nth + X.j);
        A0[v] = (A)0;
      });

      // look-ahead: row i + 4 into the slot of row i - 2
      const int row = i + 4;
      if (row <= flast) {
#pragma unroll
        for (int v = 0; v < AS_NV; ++v) S[u % AS_RING][v] = as_f(X, as_q<W, KH>(v), row);
      }
    }
  }
}

template <class R>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
adjoint_strip_kernel(Tables T, const R* __restrict__ f, const R* __restrict__ lam,
                     const R* __restrict__ ghost, const double* __restrict__ gm, double tie,
                     R* __restrict__ out, int chunk, int xcd_order) {
  __shared__ double ldsA[2 * AS_LDS_A];
  __shared__ double ldsB[2 * AS_LDS_B];
  const int nstrip = T.nth / WAVE;
  const int item = work_item(xcd_order);
  const int strip = item % nstrip, ck = item / nstrip;
  const int j0 = strip * WAVE;
  const int i0 = ck * chunk, i1 = min(i0 + chunk, T.nr);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const AsCtx<R> X{f, lam, out, ghost, gm, (size_t)T.nr * T.nth, T.nr, T.nth, j0 + lane, lane};
  switch (w) {
    case 0: as_march<R, 0, 0>(T, X, j0, i0, i1, tie, ldsA, ldsB); break;
    case 1: as_march<R, 1, 0>(T, X, j0, i0, i1, tie, ldsA, ldsB); break;
    case 2: as_march<R, 2, 0>(T, X, j0, i0, i1, tie, ldsA, ldsB); break;
    case 3: as_march<R, 3, 0>(T, X, j0, i0, i1, tie, ldsA, ldsB); break;
    case 4: as_march<R, 0, 1>(T, X, j0, i0, i1, tie, ldsA, ldsB); break;
    case 5: as_march<R, 1, 1>(T, X, j0, i0, i1, tie, ldsA, ldsB); break;
    case 6: as_march<R, 2, 1>(T, X, j0, i0, i1, tie, ldsA, ldsB); break;
    default: as_march<R, 3, 1>(T, X, j0, i0, i1, tie, ldsA, ldsB);
  }
}

}  // namespace

bool adjoint_strip_supported(const Tables& T, int precision) {
  // FP32 states only: the FP64 form of this kernel needs more than 256
  // registers per lane
  return precision == 32 && T.nf == ND && T.scheme == SCH_MWB && T.nth >= WAVE && T.nth % WAVE == 0;
}

template <class R>
hipError_t launch_adjoint_strip(const Tables& T, const void* f, const void* lam, void* lam_out,
                                const void* ghost, const double* gm, double tie,
                                const StripTune& tune, hipStream_t s) {
  // 64-row chunks: four stencil rows of every chunk are visited twice
  // (0.81 ms per FP32 adjoint step at 1024 x 2048, 0.83 with 32 rows)
  const int chunk = tune.chunk > 0 ? tune.chunk : 64;
  const int strips = T.nth / WAVE, chunks = (T.nr + chunk - 1) / chunk;
  const int order = tune.order < 0 ? 1 : tune.order;
  hipLaunchKernelGGL(adjoint_strip_kernel<R>, dim3(strips * chunks), dim3(AS_WAVES * WAVE), 0, s, T,
                     (const R*)f, (const R*)lam, (const R*)ghost, gm, tie, (R*)lam_out, chunk, order);
  return hipGetLastError();
}

template hipError_t launch_adjoint_strip<float>(const Tables&, const void*, const void*, void*,
                                                const void*, const double*, double,
                                                const StripTune&, hipStream_t);
// FP64 states take the node kernel (adjoint_strip_supported)
template <>
hipError_t launch_adjoint_strip<double>(const Tables&, const void*, const void*, void*, const void*,
                                        const double*, double, const StripTune&, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace pclb
