// Strip kernel of the combined-scheme step (Eq. combined_scheme) for FP32
// storage.  A workgroup owns a strip of 64 consecutive theta columns (one per
// lane, the strip aligned to 64 columns so that every load and store covers
// whole cache lines) and marches in r over a chunk of rows.  For each velocity
// a wavefront keeps in registers the three rows its radial MWB stencil needs
// (centre and the two upwind neighbours) and one row of look-ahead, so every
// f value of the chunk is read from HBM once and every load is issued two
// rows before its first use.  The azimuthal neighbours come from the adjacent
// lanes (ds_bpermute); the two columns beyond the strip on the upwind side
// are read per row for all velocities of a wave with one load (lane v holds
// velocity v's pair).
//
// Per row: moments, equilibrium and analytic relaxation in double (Eqs.
// moment1-3, F_k, feq, operator1_new), the radial and azimuthal MWB terms in
// float, one store per velocity, the look-ahead loads.  The kernel is
// templated on the convection scheme: the two upwind schemes the paper
// compares MWB with (Warming-Beam and second-order upwind) use the same
// stencil and differences, with their own terms (conv_term_d).
//
// Register slots by role.  The radial velocity components of the opposite
// directions d and d+4 have opposite signs, so on almost every strip one
// member of each pair is upwind-backward (u1 at row i-1) on all 64 lanes and
// the other upwind-forward.  A wave on such a strip ("uniform") holds each
// pair as (backward member, forward member) and picks the planes it reads and
// writes with scalar offsets, so that its hot loop has no per-lane selects.
// Strips where a sign changes inside the strip run the same code with lane
// selects ("mixed").  Both round exactly like the node kernel.  The upwind
// sides are those of the column's octant (octant_of), so a strip is uniform
// exactly when all its columns lie in one octant: when n_theta is a multiple
// of 512 every strip is.
#include <type_traits>

#include "common.h"
#include "launch.h"
#include "strip_common.h"

namespace pclb {

namespace {

using namespace strip;

// The state is addressed through buffer resources, one per speed k, whose
// base is plane 8(k-1): velocity (k, d) is plane 1 + d of resource k-1 and
// the rest velocity plane 0 of resource 0.  A plane is selected by a scalar
// offset, the lane's position by a 32-bit vector offset; every offset that
// addresses data stays below 2^31 (checked by strip_supported).
struct StripCtx {
  __amdgpu_buffer_rsrc_t fin[NK], fout[NK], gh;
  const float* fb;          // the input state (halo rows of uniform waves)
  size_t plane;             // values per plane
  uint32_t plane_bytes;
  int nr, nth;
  int col;                  // this lane's column
  uint32_t col4;            // its byte offset within a row
  bool store;               // this lane's column exists (the last strip may be ragged)
  double e, ome;            // exp(-dt/tau) and 1 - exp(-dt/tau)
  // azimuthal halo: byte offsets within a row of the columns the edge lanes read
  uint32_t hl4, hr4;        // pair (j0-2, j0-1) for lane 0, pair (j0+64, j0+65) for lane 63
  uint32_t hu1_4, hu2_4;    // mixed strips: u1 of lanes 0 / 63, u2 of lanes 0, 1 / 62, 63
  bool edge_l, edge_r;      // lane 0, lane 63
  bool e2l, e2r;            // lanes 0 and 1, lanes 62 and 63
  bool halo_pairs;          // the 8-byte halo loads apply (uniform waves)
};

// Work split: a strip is processed by NSPLIT wavefronts of one workgroup.
// Wave W owns the direction pairs d4 = D40 .. D40 + D4N - 1 and, for each,
// the velocities (k, d4) and (k, d4 + 4), k = 1..4; wave 0 also owns the rest
// velocity.  Per row every wave forms the moment partials of its pairs, the
// partials meet in LDS, and every wave then builds the same equilibrium from
// their sum and updates its own velocities.
template <int NSPLIT, int W>
struct Own {
  static constexpr int D4N = 4 / NSPLIT;       // direction pairs per wave
  static constexpr int D40 = W * D4N;          // first pair of this wave
  static constexpr int NV = 8 * D4N;           // velocities per wave (rest excluded)
  // slot v = (pl * 4 + (k - 1)) * 2 + h: pair d4 = D40 + pl, speed k, member h
  static constexpr int pl_of(int v) { return v >> 3; }
  static constexpr int k_of_v(int v) { return ((v >> 1) & 3) + 1; }
  static constexpr int h_of(int v) { return v & 1; }
};

// Per-wave role table.  Member h of pair pl is direction d4 + 4 (h ^ swap):
// in a uniform wave member 0 is the backward one on every lane; in a mixed
// wave swap = 0 and the roles are per lane.
template <int D4N>
struct Roles {
  uint32_t soff[D4N][2];    // byte offset of member h's plane within its resource
  int qb[D4N][2];           // 1 + direction of member h (its plane within the resource)
  double sg[D4N];           // +1, or -1 when the members are swapped
  bool tb[D4N][2];          // uniform waves: member h is azimuthally upwind-backward
};

// Load of a slot's velocity (speed K, plane qb of resource K-1) at row `row`;
// voff is the byte offset of this lane's column in that row (or OOB).  With
// EDGE, rows beyond the walls come from the ghost layers.
template <bool EDGE, int K>
__device__ inline float load_slot(const StripCtx& X, uint32_t soff, int qb, int row, uint32_t voff,
                                  bool on) {
  if constexpr (EDGE) {
    if (row < 0 || row >= X.nr) {
      const int side = row < 0 ? 0 : 1, layer = row < 0 ? -1 - row : row - X.nr;
      const int q = qb + ND * (K - 1);
      const uint32_t off = on ? (uint32_t)ghost_index(side, layer, q, X.col, X.nth) * 4u : OOB;
      return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(X.gh, off, 0, 0));
    }
  }
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(X.fin[K - 1], voff, soff, 0));
}

template <int K>
__device__ inline void store_slot(const StripCtx& X, uint32_t soff, uint32_t voff, float v) {
  // the b32 builtins move raw 32-bit words: pass the float's bits
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), X.fout[K - 1], voff, soff, STORE_NT);
}

__device__ inline uint32_t row_off(const StripCtx& X, int row, bool on) {
  return on ? (uint32_t)(row * X.nth) * 4u + X.col4 : OOB;
}

// Azimuthal halo of one velocity at row `row` (a real row).  Uniform waves:
// the edge lane on the upwind side reads the two columns beyond the strip in
// one 8-byte load, (lo, hi) = (j0-2, j0-1) on the left, (j0+64, j0+65) on the
// right.  Mixed waves: lanes 0 / 63 read their u1 into `lo`, lanes 0, 1 /
// 62, 63 their u2 into `hi`.  Every other lane reads nothing (value 0).
template <int K, bool UNI>
__device__ inline void load_halo(const StripCtx& X, uint32_t soff, int row, bool tb, bool on,
                                 float& lo, float& hi) {
  const uint32_t rb = (uint32_t)(row * X.nth) * 4u;
  if constexpr (UNI) {
    const bool act = on && (tb ? X.edge_l : X.edge_r);
    const uint32_t voff = act ? rb + (tb ? X.hl4 : X.hr4) : OOB;
    const auto r = __builtin_amdgcn_raw_buffer_load_b64(X.fin[K - 1], voff, soff, 0);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
  } else {
    const uint32_t v1 = on && (X.edge_l || X.edge_r) ? rb + X.hu1_4 : OOB;
    const uint32_t v2 = on && (X.e2l || X.e2r) ? rb + X.hu2_4 : OOB;
    lo = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(X.fin[K - 1], v1, soff, 0));
    hi = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(X.fin[K - 1], v2, soff, 0));
  }
}

// One output row i.  For every owned velocity the slots A, B, C hold three
// consecutive rows in increasing order: (i-2, i-1, i) when the upwind side is
// i-1 ("backward"), (i, i+1, i+2) otherwise; a ring of NS = 4 slots holds one
// more row of look-ahead.  After the velocity's terms are computed, the lowest
// slot A is refilled with row (lowest + NS), and the caller rotates the roles
// by one slot for the next row.  A load is thus issued NS - 2 rows before the
// row that first uses it.  more1: row i+1 is in the chunk (rest velocity,
// halo); moreN: row i+NS-2 is (look-ahead rows).
//
// Azimuthal halo of uniform waves: lane v holds in (hlo, hhi) the two columns
// beyond the strip on slot v's upwind side at row i; the pair for row i+1 is
// read with one load for all slots at the start of the row (hp: lane v's
// pointer to that pair in row 0), and each slot takes its pair with
// readlane.  Mixed waves keep one pair of registers per slot (HA, HB).
template <int NSPLIT, int W, bool EDGE, bool UNI, int NS, int SCH>
__device__ inline void strip_row(const Tables& T, const StripCtx& X, const DirGeom<float>& G,
                                 const Roles<4 / NSPLIT>& RL, int i, int ir, float rinv_lane,
                                 bool more, bool moreN, const int* ta,
                                 float& r0, float* A, float* B, float* C, float* HA, float* HB,
                                 float& hlo, float& hhi, const float* hp, double* lds) {
  using O = Own<NSPLIT, W>;
  const int lane = threadIdx.x & 63;
  float nlo = 0.0f, nhi = 0.0f;
  if constexpr (UNI) {
    // every lane loads (lanes past the slots read the first two values of a
    // real row, which nobody uses), so that no branch splits the wave here
    const int hrow = more ? i + 1 : i;
    const float2 t = *reinterpret_cast<const float2*>(hp + (size_t)hrow * X.nth);
    nlo = t.x;
    nhi = t.y;
  }
  // backward role of slot v: fixed in a uniform wave, per lane otherwise
  auto back = [&](int v) -> bool {
    if constexpr (UNI) return O::h_of(v) == 0;
    else return (G.rback >> (O::D40 + O::pl_of(v) + 4 * O::h_of(v))) & 1u;
  };
  // moment partials of the owned direction pairs
  double P[4][4];
#pragma unroll
  for (int pl = 0; pl < O::D4N; ++pl) {
    double f0[NK], f1[NK];
#pragma unroll
    for (int k = 1; k <= NK; ++k) {
      const int v0 = (pl * 4 + (k - 1)) * 2, v1 = v0 + 1;
      f0[k - 1] = (double)(back(v0) ? C[v0] : A[v0]);
      f1[k - 1] = (double)(back(v1) ? C[v1] : A[v1]);
    }
    double* Pd = P[O::D40 + pl];
    d4_partial(O::D40 + pl, f0, f1, Pd);
    if constexpr (UNI) {            // f0 - f1 was taken with the members swapped
      Pd[1] *= RL.sg[pl];
      Pd[2] *= RL.sg[pl];
    }
  }
  double rest = (double)r0;            // wave 0's; the others read it from LDS
  if constexpr (NSPLIT > 1) {
    // lds[(d * 4 + a) * 64 + lane] and the rest velocity at lds[16 * 64 + lane],
    // double-buffered by row parity
    double* buf = lds + (i & 1) * (17 * 64);
#pragma unroll
    for (int pl = 0; pl < O::D4N; ++pl)
#pragma unroll
      for (int a = 0; a < 4; ++a) buf[((O::D40 + pl) * 4 + a) * 64 + lane] = P[O::D40 + pl][a];
    if constexpr (W == 0) buf[16 * 64 + lane] = rest;
    __syncthreads();
    if constexpr (W != 0) rest = buf[16 * 64 + lane];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      if (d >= O::D40 && d < O::D40 + O::D4N) continue;
#pragma unroll
      for (int a = 0; a < 4; ++a) P[d][a] = buf[(d * 4 + a) * 64 + lane];
    }
  }
  double rho, ux, uy, E;
  combine_partials(P, rest, rho, ux, uy, E);
  EqCoef ec;
  eq_setup(T, rho, ux, uy, E, ec);
  // 1/r of this row from lane (i - i_begin) of rinv_lane: a table load here
  // would be waited for in order behind every look-ahead load and store in
  // flight
  const float rinv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rinv_lane), ir));
  const uint32_t ovoff = X.store ? (uint32_t)(i * X.nth) * 4u + X.col4 : OOB;
  const uint32_t vb = row_off(X, i + NS - 2, moreN), vf = row_off(X, i + NS, moreN);
  if constexpr (W == 0) {            // rest velocity: relaxation only, one row ahead
    const float res = relax_rest<float>(relax_rest_share(ec, X.ome), X.e, (double)r0);
    store_slot<1>(X, 0, ovoff, res);
    r0 = load_slot<EDGE, 1>(X, 0, 0, i + 1, row_off(X, i + 1, more), more);
  }
  for_v<0, O::NV / 2>([&](auto pc) {
    constexpr int pk = decltype(pc)::value;     // (pair, k) index
    constexpr int pl = pk >> 2, k = (pk & 3) + 1;
    constexpr int d4 = O::D40 + pl;
    constexpr int v0 = pk * 2, v1 = pk * 2 + 1;
    const bool b0 = back(v0), b1 = back(v1);
    const float c0 = b0 ? C[v0] : A[v0];
    const float c1 = b1 ? C[v1] : A[v1];
    double rel[2];
    // with the members swapped the odd coefficients change sign, exactly
    const double sg = UNI ? RL.sg[pl] : 1.0;
    relax_pair<k>(ec, X.e, X.ome, sg * ec.p[d4], (double)c0, (double)c1, rel[0], rel[1]);
    float aCr, Kr, aCt, Kt;
    courant<float>((float)speed(k), G.ar[d4], aCr, Kr);
    courant<float>((float)speed(k), G.at[d4] * rinv, aCt, Kt);
    auto one = [&](auto vv, bool bk, float c, double rl) {
      constexpr int v = decltype(vv)::value;
      constexpr int h = O::h_of(v);
      // azimuthal differences.  Uniform waves: d1 from the upwind lane (the
      // edge lane from the halo), d2 is the upwind lane's d1 (the edge lane's
      // from the halo pair).  Mixed waves: both neighbours from the lanes one
      // and two upwind, the edge lanes from their halo values.
      float d1t, d2t;
      if constexpr (UNI) {
        const bool tb = RL.tb[pl][h];
        const bool edge = tb ? X.edge_l : X.edge_r;
        const float lo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hlo), v));
        const float hi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hhi), v));
        const float fix1 = tb ? hi : lo, fix2 = tb ? lo : hi;
        const float z = lane_from(c, ta[v]);
        const float u1t = edge ? fix1 : z;
        d1t = c - u1t;
        const float dz = lane_from(d1t, ta[v]);
        d2t = edge ? fix1 - fix2 : dz;
      } else {
        const bool tb = (G.tback >> (O::D40 + O::pl_of(v) + 4 * O::h_of(v))) & 1u;
        const bool e1 = tb ? X.edge_l : X.edge_r, e2 = tb ? X.e2l : X.e2r;
        const float z1 = lane_from(c, ta[v]);
        const float z2 = lane_from(c, (ta[v] << 1) - (lane << 2));
        const float u1t = e1 ? HA[v] : z1;
        const float u2t = e2 ? HB[v] : z2;
        d1t = c - u1t;
        d2t = u1t - u2t;
      }
      const float u1r = B[v];
      const float d1r = c - u1r, d2r = u1r - (bk ? A[v] : C[v]);
      const float res = scheme_update_d<SCH, float>(rl, aCr, Kr, d1r, d2r, aCt, Kt, d1t, d2t);
      store_slot<k>(X, RL.soff[pl][h], ovoff, res);
      A[v] = load_slot<EDGE, k>(X, RL.soff[pl][h], RL.qb[pl][h], bk ? i + NS - 2 : i + NS,
                                bk ? vb : vf, moreN);
      if constexpr (!UNI) load_halo<k, false>(X, RL.soff[pl][h], i + 1, false, more, HA[v], HB[v]);
    };
    one(std::integral_constant<int, v0>{}, b0, c0, rel[0]);
    one(std::integral_constant<int, v1>{}, b1, c1, rel[1]);
  });
  if constexpr (UNI) {
    hlo = nlo;
    hhi = nhi;
  }
}

template <int NSPLIT, int W, bool EDGE, bool UNI, int NS, int SCH>
__device__ inline void strip_march(const Tables& T, const StripCtx& X, const DirGeom<float>& G,
                                   const Roles<4 / NSPLIT>& RL, int i_begin, int i_end,
                                   double* lds) {
  using O = Own<NSPLIT, W>;
  static_assert(NS == 3 || NS == 4, "ring of three or four rows");
  float S[NS][O::NV];
  float HA[UNI ? 1 : O::NV], HB[UNI ? 1 : O::NV];   // mixed waves: halo of the row, per slot
  float hlo = 0.0f, hhi = 0.0f;                       // uniform waves: lane v holds slot v's pair
  const float* hp = X.fb;
  // ds_bpermute byte address of the azimuthally upwind lane, per slot
  int ta[O::NV];
  const int lane = threadIdx.x & (WAVE - 1);
  // 1/r of the chunk's rows, lane l holding row i_begin + l (chunks have at
  // most 64 rows)
  const float rinv_lane = i_begin + lane < X.nr ? (float)T.rinv[i_begin + lane] : 0.0f;
  float r0 = 0.0f;
  if constexpr (W == 0) r0 = load_slot<EDGE, 1>(X, 0, 0, i_begin, row_off(X, i_begin, true), true);
  if constexpr (UNI) {
    // the first halo pair is loaded before the ring, so that at the loop's
    // head it is as old as in later iterations (the compiler's wait counting
    // merges both)
    for_v<0, O::NV>([&](auto vc) {
      constexpr int v = decltype(vc)::value;
      constexpr int pl = O::pl_of(v), h = O::h_of(v), k = O::k_of_v(v);
      if (lane == v)
        hp = X.fb + (size_t)(RL.qb[pl][h] + ND * (k - 1)) * X.plane +
             (RL.tb[pl][h] ? X.hl4 : X.hr4) / 4u;
    });
    const float2 t = *reinterpret_cast<const float2*>(hp + (size_t)i_begin * X.nth);
    hlo = t.x;
    hhi = t.y;
  }
  for_v<0, O::NV>([&](auto vc) {
    constexpr int v = decltype(vc)::value;
    constexpr int pl = O::pl_of(v), h = O::h_of(v), k = O::k_of_v(v);
    const int qb = RL.qb[pl][h];
    const int d = qb - 1;                       // direction of the slot's velocity
    ta[v] = (((G.tback >> d) & 1u) ? lane - 1 : lane + 1) << 2;
    if constexpr (!UNI) load_halo<k, false>(X, RL.soff[pl][h], i_begin, false, true, HA[v], HB[v]);
  });
  // the ring, one slot of every velocity after the other, so that the
  // look-ahead slot is loaded last
  for_v<0, NS>([&](auto sc) {
    constexpr int sl = decltype(sc)::value;
    // look-ahead slot sl >= 3 is first used at row i_begin + sl - 2
    const bool on = sl < 3 || i_begin + sl - 2 < i_end;
    for_v<0, O::NV>([&](auto vc) {
      constexpr int v = decltype(vc)::value;
      constexpr int pl = O::pl_of(v), h = O::h_of(v), k = O::k_of_v(v);
      const int qb = RL.qb[pl][h];
      const bool bk = UNI ? h == 0 : ((G.rback >> (qb - 1)) & 1u);
      const int row = (bk ? i_begin - 2 : i_begin) + sl;
      S[sl][v] = load_slot<EDGE, k>(X, RL.soff[pl][h], qb, row, row_off(X, row, on), on);
    });
  });
  if constexpr (NS == 4) {
    // four rows per iteration with the slot roles rotated at compile time, so
    // the ring needs no register moves (a move of a register whose load is in
    // flight would wait for that load and undo the look-ahead)
    // (whole groups of four rows run without a per-row condition, so that the
    // compiler's wait counting sees every row's loads; the last rows of a
    // chunk whose length is not a multiple of four follow with one)
    int i = i_begin;
    for (; i + NS <= i_end; i += NS) {
      for_v<0, NS>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        const int iu = i + u;
        strip_row<NSPLIT, W, EDGE, UNI, NS, SCH>(T, X, G, RL, iu, iu - i_begin, rinv_lane,
                                            iu + 1 < i_end, iu + NS - 2 < i_end, ta, r0,
                                            S[u % NS], S[(u + 1) % NS], S[(u + 2) % NS], HA, HB,
                                            hlo, hhi, hp, lds);
      });
    }
    for_v<0, NS - 1>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const int iu = i + u;
      if (iu < i_end)
        strip_row<NSPLIT, W, EDGE, UNI, NS, SCH>(T, X, G, RL, iu, iu - i_begin, rinv_lane,
                                            iu + 1 < i_end, iu + NS - 2 < i_end, ta, r0,
                                            S[u % NS], S[(u + 1) % NS], S[(u + 2) % NS], HA, HB,
                                            hlo, hhi, hp, lds);
    });
  } else {
    // one row per iteration, the ring rotated by register moves (its loads
    // are one row ahead and waited for at the next row's start anyway)
    for (int i = i_begin; i < i_end; ++i) {
      strip_row<NSPLIT, W, EDGE, UNI, NS, SCH>(T, X, G, RL, i, i - i_begin, rinv_lane, i + 1 < i_end,
                                          i + 1 < i_end, ta, r0,
                                          S[0], S[1], S[2], HA, HB, hlo, hhi, hp, lds);
      for_v<0, O::NV>([&](auto vc) {
        constexpr int v = decltype(vc)::value;
        const float t = S[0][v];
        S[0][v] = S[1][v];
        S[1][v] = S[2][v];
        S[2][v] = t;
      });
    }
  }
}

template <int NSPLIT, int W, bool MIXED, int SCH, int NS = MIXED ? 3 : 4>
__device__ inline void strip_wave(const Tables& T, const StripCtx& X, const DirGeom<float>& G,
                                  int i_begin, int i_end, double* lds) {
  using O = Own<NSPLIT, W>;
  // Roles of the owned pairs: uniform when, on every lane of the wave, exactly
  // one member of each pair is radially backward, the same member on all
  // lanes, and each member has the same azimuthal upwind side on all lanes
  // (and the two halo columns on each side are adjacent in memory).
  Roles<O::D4N> RL;
  bool uni = X.halo_pairs;
#pragma unroll
  for (int pl = 0; pl < O::D4N; ++pl) {
    const int d4 = O::D40 + pl;
    const uint64_t all = ~0ull;
    const uint64_t b0 = __ballot((G.rback >> d4) & 1u);
    const uint64_t b1 = __ballot((G.rback >> (d4 + 4)) & 1u);
    const uint64_t t0 = __ballot((G.tback >> d4) & 1u);
    const uint64_t t1 = __ballot((G.tback >> (d4 + 4)) & 1u);
    const bool swap = b0 == 0 && b1 == all;
    uni = uni && ((b0 == all && b1 == 0) || swap) && (t0 == 0 || t0 == all) &&
          (t1 == 0 || t1 == all);
    RL.sg[pl] = swap ? -1.0 : 1.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int qb = 1 + d4 + 4 * (h ^ (swap ? 1 : 0));
      RL.qb[pl][h] = qb;
      RL.soff[pl][h] = (uint32_t)qb * X.plane_bytes;
      RL.tb[pl][h] = (h ^ (swap ? 1 : 0)) ? t1 == all : t0 == all;
    }
  }
  // the chunk reads rows i_begin-2 .. i_end+1; only chunks next to a wall
  // touch the ghost layers
  const bool edge = i_begin < 2 || i_end + 1 >= X.nr;
  // Strips where every wave is uniform run in the launch without the mixed
  // code (which needs more registers); the others in the mixed launch.
  const bool all_uni = __syncthreads_and(uni ? 1 : 0) != 0;
  if (all_uni == MIXED) return;
  if constexpr (!MIXED) {
    if (edge) strip_march<NSPLIT, W, true, true, NS, SCH>(T, X, G, RL, i_begin, i_end, lds);
    else strip_march<NSPLIT, W, false, true, NS, SCH>(T, X, G, RL, i_begin, i_end, lds);
    return;
  }
  if (uni) {
    if (edge) strip_march<NSPLIT, W, true, true, NS, SCH>(T, X, G, RL, i_begin, i_end, lds);
    else strip_march<NSPLIT, W, false, true, NS, SCH>(T, X, G, RL, i_begin, i_end, lds);
  } else {
#pragma unroll
    for (int pl = 0; pl < O::D4N; ++pl) {       // mixed: members in natural order
      RL.sg[pl] = 1.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int qb = 1 + O::D40 + pl + 4 * h;
        RL.qb[pl][h] = qb;
        RL.soff[pl][h] = (uint32_t)qb * X.plane_bytes;
        RL.tb[pl][h] = false;
      }
    }
    if (edge) strip_march<NSPLIT, W, true, false, NS, SCH>(T, X, G, RL, i_begin, i_end, lds);
    else strip_march<NSPLIT, W, false, false, NS, SCH>(T, X, G, RL, i_begin, i_end, lds);
  }
}

}  // namespace

// Two waves per SIMD (at most 256 registers per lane): left to itself the
// compiler spends a few accumulation registers beyond that on the uniform
// variant and drops to one wave.
template <int NSPLIT, bool MIXED, int SCH>
__global__ void __launch_bounds__(WAVE * NSPLIT) __attribute__((amdgpu_waves_per_eu(2)))
step_strip_kernel(Tables T, const float* __restrict__ f, float* __restrict__ out,
                  const float* __restrict__ ghost, int chunk_rows, int n_strips, int xcd_order) {
  __shared__ double lds[NSPLIT > 1 ? 2 * 17 * 64 : 1];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = threadIdx.x >> 6;                     // wave within the group
  const int w_item = work_item(xcd_order);
  const int strip = w_item % n_strips;
  const int chunk = w_item / n_strips;
  const int nr = T.nr, nth = T.nth;
  const int i_begin = chunk * chunk_rows;
  const int i_end = min(nr, i_begin + chunk_rows);    // every block has i_begin < nr

  StripCtx X;
  const size_t plane = (size_t)nr * nth;
  X.plane_bytes = (uint32_t)(plane * 4);
#pragma unroll
  for (int k = 1; k <= NK; ++k) {
    X.fin[k - 1] = make_rsrc(f + ND * (k - 1) * plane);
    X.fout[k - 1] = make_rsrc(out + ND * (k - 1) * plane);
  }
  X.gh = make_rsrc(ghost);
  X.fb = f;
  X.plane = plane;
  X.nr = nr;
  X.nth = nth;
  // column of this lane (periodic) and whether it stores an output
  const int j0 = strip * WAVE;
  const int jout = j0 + lane;                          // past nth only in a ragged last strip
  X.col = jout % nth;
  X.col4 = (uint32_t)X.col * 4u;
  X.store = jout < nth;
  // azimuthal halo columns (periodic)
  auto wrap = [&](int c) { return ((c % nth) + nth) % nth; };
  X.edge_l = lane == 0;
  X.edge_r = lane == WAVE - 1;
  X.e2l = lane <= 1;
  X.e2r = lane >= WAVE - 2;
  X.hl4 = (uint32_t)wrap(j0 - 2) * 4u;
  X.hr4 = (uint32_t)wrap(j0 + WAVE) * 4u;
  X.hu1_4 = (uint32_t)(lane == 0 ? wrap(j0 - 1) : wrap(j0 + WAVE)) * 4u;
  X.hu2_4 = (uint32_t)(lane == 0 ? wrap(j0 - 2)
                                 : lane == 1 ? wrap(j0 - 1)
                                             : lane == WAVE - 2 ? wrap(j0 + WAVE) : wrap(j0 + WAVE + 1)) *
            4u;
  // the 8-byte halo loads need both pairs adjacent and 8-byte aligned
  X.halo_pairs = (nth % 2 == 0) && wrap(j0 - 2) + 1 == wrap(j0 - 1) &&
                 wrap(j0 + WAVE) + 1 == wrap(j0 + WAVE + 1);
  X.e = T.e;
  X.ome = 1.0 - T.e;
  DirGeom<float> G;
  dir_geometry(T.cth[X.col], T.sth[X.col], octant_of(X.col, nth, T.nf), T.dt_dr, T.dt_dth, G);
  if constexpr (NSPLIT == 1) {
    strip_wave<1, 0, MIXED, SCH>(T, X, G, i_begin, i_end, lds);
  } else if constexpr (NSPLIT == 2) {
    if (w == 0) strip_wave<2, 0, MIXED, SCH>(T, X, G, i_begin, i_end, lds);
    else strip_wave<2, 1, MIXED, SCH>(T, X, G, i_begin, i_end, lds);
  } else {
    if (w == 0) strip_wave<4, 0, MIXED, SCH>(T, X, G, i_begin, i_end, lds);
    else if (w == 1) strip_wave<4, 1, MIXED, SCH>(T, X, G, i_begin, i_end, lds);
    else if (w == 2) strip_wave<4, 2, MIXED, SCH>(T, X, G, i_begin, i_end, lds);
    else strip_wave<4, 3, MIXED, SCH>(T, X, G, i_begin, i_end, lds);
  }
}

template <class R>
bool strip_supported(const Tables& T) {
  // every offset that addresses data (at most 8 planes past a resource base,
  // plus the lane offset, kept below 9 planes) must stay below 2^31, the OOB
  // marker; the lanes of one strip must be distinct columns
  const double plane_bytes = 4.0 * T.nr * (double)T.nth;
  // the strip kernel wraps theta without rotating the velocity index (full
  // annulus only) and carries the upwind schemes (MWB, Warming-Beam and
  // second-order upwind), not Lax-Wendroff, whose downwind neighbour its
  // ring does not hold
  return std::is_same<R, float>::value && T.nf == 8 && T.scheme != SCH_LW && T.nth >= WAVE &&
         9.0 * plane_bytes < 2147483647.0;
}

int strip_default_chunk(const Tables& T) {
  // enough (strip, chunk) workgroups to fill 256 CUs several times over
  const int strips = n_strips(T.nth);
  int chunk = 32;
  while (chunk > 8 && (long)strips * ((T.nr + chunk - 1) / chunk) < 4096) chunk /= 2;
  return chunk;
}

// Strips whose lanes' columns (taken modulo n_theta, as the kernel takes
// them, so that a ragged last strip counts its wrapped lanes) lie in more
// than one octant (host side): with the upwind sides taken from the octants
// every other strip is uniform.
int strip_mixed_count(int nth, int nf) {
  int n = 0;
  for (int j0 = 0; j0 < nth; j0 += WAVE) {
    const int oct = octant_of(j0, nth, nf);
    for (int l = 1; l < WAVE; ++l)
      if (octant_of((j0 + l) % nth, nth, nf) != oct) {
        ++n;
        break;
      }
  }
  return n;
}

// strips whose waves are all uniform, then (if any strip straddles an octant
// boundary, or has its halo columns apart) the others, in a second launch
// over the same grid in which the uniform strips return at once
template <int SCH>
hipError_t launch_strip_sch(const Tables& T, const float* fi, float* fo, const float* gh, int chunk_rows,
                            int strips, int order, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((step_strip_kernel<2, false, SCH>), dim3(blocks), dim3(2 * WAVE), 0, s, T, fi, fo,
                     gh, chunk_rows, strips, order);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (T.n_mixed > 0 || T.nth % 2 != 0) {
    hipLaunchKernelGGL((step_strip_kernel<2, true, SCH>), dim3(blocks), dim3(2 * WAVE), 0, s, T, fi, fo,
                       gh, chunk_rows, strips, order);
    e = hipGetLastError();
  }
  return e;
}

template <class R>
hipError_t launch_step_strip(const Tables& T, const void* f, void* out, const void* ghost,
                             const StripTune& tune, hipStream_t s) {
  if (!strip_supported<R>(T)) return hipErrorNotSupported;
  const int chunk_rows = tune.chunk > 0 ? tune.chunk : strip_default_chunk(T);
  if (chunk_rows > WAVE) return hipErrorInvalidValue;   // 1/r of a chunk is held one row per lane
  const int order = tune.order >= 0 ? (tune.order ? 1 : 0) : 1;
  const int strips = n_strips(T.nth);
  const int chunks = (T.nr + chunk_rows - 1) / chunk_rows;
  const int blocks = strips * chunks;
  const float* fi = (const float*)f;
  float* fo = (float*)out;
  const float* gh = (const float*)ghost;
  switch (T.scheme) {
    case SCH_WB: return launch_strip_sch<SCH_WB>(T, fi, fo, gh, chunk_rows, strips, order, blocks, s);
    case SCH_UPWIND2:
      return launch_strip_sch<SCH_UPWIND2>(T, fi, fo, gh, chunk_rows, strips, order, blocks, s);
    default: return launch_strip_sch<SCH_MWB>(T, fi, fo, gh, chunk_rows, strips, order, blocks, s);
  }
}

template bool strip_supported<float>(const Tables&);
template bool strip_supported<double>(const Tables&);
template hipError_t launch_step_strip<float>(const Tables&, const void*, void*, const void*,
                                             const StripTune&, hipStream_t);
template hipError_t launch_step_strip<double>(const Tables&, const void*, void*, const void*,
                                              const StripTune&, hipStream_t);

}  // namespace pclb
