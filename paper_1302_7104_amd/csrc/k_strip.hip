// Strip kernel of the combined-scheme step (Eq. combined_scheme) for FP32
// storage: every wavefront owns a strip of 64 consecutive theta columns and
// marches in r over a chunk of rows, keeping for each velocity the three
// values its radial MWB stencil needs (centre and the two upwind neighbours)
// in registers.  Each f value of the chunk is read from HBM once; the theta
// neighbours come from the adjacent lanes (ds_bpermute), so only 4 of the 64
// lanes (2 on each side) are halo columns that produce no output.
//
// Per row: 33 loads issued one row ahead, moments and equilibrium in double
// (Eqs. moment1-3, F_k, feq), analytic relaxation (Eq. operator1_new), the
// radial and azimuthal MWB terms in float, 33 stores.
#include <type_traits>

#include "common.h"
#include "launch.h"

namespace pclb {

namespace {

constexpr int WAVE = 64;
constexpr int HALO = 2;
constexpr int OUT_COLS = WAVE - 2 * HALO;     // 60 output columns per strip
// word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format)
constexpr int BUF_DWORD3 = 0x00020000;
constexpr int NXCD = 8;   // accelerator dies; workgroups are dealt to them round-robin

template <int Q, class Fn>
__device__ inline void for_q(Fn&& fn) {
  if constexpr (Q < NQ) {
    fn(std::integral_constant<int, Q>{});
    for_q<Q + 1>(fn);
  }
}

// The state is addressed through buffer resources: planes 0..10, 11..21 and
// 22..32 each from their own base, a plane selected by a scalar offset
// q' * plane_bytes, the lane's position by a 32-bit vector offset.  Every
// offset stays below 2^31 (checked by strip_supported).
constexpr int PLANES_PER_DESC = 11;
constexpr int NDESC = 3;

struct StripCtx {
  __amdgpu_buffer_rsrc_t fin[NDESC], fout[NDESC], gh;
  uint32_t plane_bytes;
  int nr, nth;
  int col;
  bool store;
  double e, ome;
  int bp_b1, bp_b2, bp_f1, bp_f2;   // ds_bpermute byte addresses of lanes -1, -2, +1, +2
};

template <int Q>
__device__ inline uint32_t plane_off(const StripCtx& X) {
  return (uint32_t)(Q % PLANES_PER_DESC) * X.plane_bytes;
}

// Value of velocity Q at row `row` of this lane's column: the state for real
// rows; with EDGE, rows beyond the walls come from the ghost layers (and rows
// past the last ghost layer, read only after a chunk's last row, are clamped).
template <bool EDGE, int Q>
__device__ inline float load_f(const StripCtx& X, int row) {
  if constexpr (EDGE) {
    row = min(row, X.nr + 1);
    if (row < 0 || row >= X.nr) {
      const int side = row < 0 ? 0 : 1, layer = row < 0 ? -1 - row : row - X.nr;
      const uint32_t off = (uint32_t)ghost_index(side, layer, Q, X.col, X.nth) * 4u;
      return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(X.gh, off, 0, 0));
    }
  }
  const uint32_t voff = (uint32_t)(row * X.nth + X.col) * 4u;
  return __uint_as_float(
      __builtin_amdgcn_raw_buffer_load_b32(X.fin[Q / PLANES_PER_DESC], voff, plane_off<Q>(X), 0));
}

template <int Q>
__device__ inline void store_f(const StripCtx& X, uint32_t voff, float v) {
  // the b32 builtins move raw 32-bit words: pass the float's bits
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), X.fout[Q / PLANES_PER_DESC], voff,
                                        plane_off<Q>(X), 0);
}

__device__ inline float lane_from(float v, int byte_addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
}

// Work split: a strip of 64 columns is processed by NSPLIT wavefronts of one
// workgroup.  Wave W owns the direction pairs d = W*(4/NSPLIT) .. and, for each,
// the velocities (k, d) and (k, d+4), k = 1..4; wave 0 also owns the rest
// velocity.  Per row every wave forms the moment partials of its pairs, the
// partials meet in LDS, and every wave then builds the same equilibrium from
// their sum and updates its own velocities.
template <int NSPLIT, int W>
struct Own {
  static constexpr int D4N = 4 / NSPLIT;       // direction pairs per wave
  static constexpr int D40 = W * D4N;          // first pair of this wave
  static constexpr int NV = 8 * D4N;           // velocities per wave (rest excluded)
  // local slot v -> velocity: v = (pair * 4 + (k - 1)) * 2 + h
  static constexpr int q_of(int v) {
    return qidx(((v >> 1) & 3) + 1, D40 + (v >> 3) + 4 * (v & 1));
  }
};

template <int V, int N, class Fn>
__device__ inline void for_v(Fn&& fn) {
  if constexpr (V < N) {
    fn(std::integral_constant<int, V>{});
    for_v<V + 1, N>(fn);
  }
}

// One output row i.  For every owned velocity the slots A, B, C hold three
// consecutive rows in increasing order: (i-2, i-1, i) when the upwind side is
// i-1 ("backward"), (i, i+1, i+2) otherwise.  After the velocity's terms are
// computed, the lowest slot A is refilled with row (lowest + 3), so that the
// roles rotate A <- B <- C <- A from one row to the next.
template <int NSPLIT, int W, bool EDGE>
__device__ inline void strip_row(const Tables& T, const StripCtx& X, const DirGeom<float>& G, int i,
                                 bool more, float& r0, float* A, float* B, float* C, double* lds) {
  using O = Own<NSPLIT, W>;
  const unsigned rback = G.rback, tback = G.tback;
  // moment partials of the owned direction pairs
  double P[4][4];
#pragma unroll
  for (int p = 0; p < O::D4N; ++p) {
    double fp[NK], fm[NK];
#pragma unroll
    for (int k = 1; k <= NK; ++k) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int v = (p * 4 + (k - 1)) * 2 + h;
        const int d = O::D40 + p + 4 * h;
        const float c = ((rback >> d) & 1u) ? C[v] : A[v];
        (h ? fm : fp)[k - 1] = (double)c;
      }
    }
    d4_partial(O::D40 + p, (W == 0 && p == 0) ? (double)r0 : 0.0, fp, fm, P[O::D40 + p]);
  }
  if constexpr (NSPLIT > 1) {
    // lds[(d * 4 + a) * 64 + lane], double-buffered by row parity
    double* buf = lds + (i & 1) * (16 * 64);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < O::D4N; ++p)
#pragma unroll
      for (int a = 0; a < 4; ++a) buf[((O::D40 + p) * 4 + a) * 64 + lane] = P[O::D40 + p][a];
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      if (d >= O::D40 && d < O::D40 + O::D4N) continue;
#pragma unroll
      for (int a = 0; a < 4; ++a) P[d][a] = buf[(d * 4 + a) * 64 + lane];
    }
  }
  double rho, ux, uy, E;
  combine_partials(P, rho, ux, uy, E);
  EqCoef ec;
  eq_setup(T, rho, ux, uy, E, ec);
  const float rinv = (float)T.rinv[i];
  const uint32_t ovoff = (uint32_t)(i * X.nth + X.col) * 4u;
  if constexpr (W == 0) {            // rest velocity: relaxation only
    const float res = relax_rest<float>(ec, X.e, X.ome, r0);
    if (X.store) store_f<0>(X, ovoff, res);
    if (more) r0 = load_f<EDGE, 0>(X, i + 1);
  }
  for_v<0, O::NV / 2>([&](auto pc) {
    constexpr int pk = decltype(pc)::value;     // (pair, k) index
    constexpr int p = pk >> 2, k = (pk & 3) + 1;
    constexpr int d4 = O::D40 + p;
    constexpr int vp = pk * 2, vm = pk * 2 + 1;
    constexpr int qp = qidx(k, d4), qm = qidx(k, d4 + 4);
    const bool bp = (rback >> d4) & 1u, bm = (rback >> (d4 + 4)) & 1u;
    const float cp = bp ? C[vp] : A[vp];
    const float cm = bm ? C[vm] : A[vm];
    float rel[2];
    relax_pair<float>(ec, X.e, X.ome, k, d4, cp, cm, rel[0], rel[1]);
    float aCr, Kr, aCt, Kt;
    courant<float>((float)speed(k), G.ar[d4], aCr, Kr);
    courant<float>((float)speed(k), G.at[d4] * rinv, aCt, Kt);
    auto one = [&](auto vv, auto qq, bool back, float c, float rl) {
      constexpr int v = decltype(vv)::value;
      constexpr int q = decltype(qq)::value;
      constexpr int d = d_of(q);
      const bool tb = (tback >> d) & 1u;
      const float t1 = lane_from(c, tb ? X.bp_b1 : X.bp_f1);
      const float t2 = lane_from(c, tb ? X.bp_b2 : X.bp_f2);
      const float res = mwb_update<float>(rl, c, aCr, Kr, B[v], back ? A[v] : C[v], aCt, Kt, t1, t2);
      if (X.store) store_f<q>(X, ovoff, res);
      if (more) A[v] = load_f<EDGE, q>(X, back ? i + 1 : i + 3);
    };
    one(std::integral_constant<int, vp>{}, std::integral_constant<int, qp>{}, bp, cp, rel[0]);
    one(std::integral_constant<int, vm>{}, std::integral_constant<int, qm>{}, bm, cm, rel[1]);
  });
}

template <int NSPLIT, int W, bool EDGE>
__device__ inline void strip_march(const Tables& T, const StripCtx& X, const DirGeom<float>& G,
                                   int i_begin, int i_end, double* lds) {
  using O = Own<NSPLIT, W>;
  float S0[O::NV], S1[O::NV], S2[O::NV];
  float r0 = 0.0f;
  if constexpr (W == 0) r0 = load_f<EDGE, 0>(X, i_begin);
  for_v<0, O::NV>([&](auto vc) {
    constexpr int v = decltype(vc)::value;
    constexpr int q = O::q_of(v);
    constexpr int d = d_of(q);
    const int base = ((G.rback >> d) & 1u) ? i_begin - 2 : i_begin;
    S0[v] = load_f<EDGE, q>(X, base);
    S1[v] = load_f<EDGE, q>(X, base + 1);
    S2[v] = load_f<EDGE, q>(X, base + 2);
  });
  for (int i = i_begin; i < i_end; i += 3) {
    strip_row<NSPLIT, W, EDGE>(T, X, G, i, i + 1 < i_end, r0, S0, S1, S2, lds);
    if (i + 1 >= i_end) break;
    strip_row<NSPLIT, W, EDGE>(T, X, G, i + 1, i + 2 < i_end, r0, S1, S2, S0, lds);
    if (i + 2 >= i_end) break;
    strip_row<NSPLIT, W, EDGE>(T, X, G, i + 2, i + 3 < i_end, r0, S2, S0, S1, lds);
  }
}

template <int NSPLIT, int W>
__device__ inline void strip_wave(const Tables& T, const StripCtx& X, const DirGeom<float>& G,
                                  int i_begin, int i_end, double* lds) {
  // the chunk reads rows i_begin-2 .. i_end+1; only chunks next to a wall
  // touch the ghost layers
  if (i_begin < 2 || i_end + 1 >= X.nr) strip_march<NSPLIT, W, true>(T, X, G, i_begin, i_end, lds);
  else strip_march<NSPLIT, W, false>(T, X, G, i_begin, i_end, lds);
}

}  // namespace

template <int NSPLIT>
__global__ void __launch_bounds__(WAVE * NSPLIT)
step_strip_kernel(Tables T, const float* __restrict__ f, float* __restrict__ out,
                  const float* __restrict__ ghost, int chunk_rows, int n_strips, int xcd_order) {
  __shared__ double lds[NSPLIT > 1 ? 2 * 16 * 64 : 1];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = threadIdx.x >> 6;                     // wave within the group
  // Work item w runs over strips first, then chunks.  With xcd_order the
  // workgroups dealt to one XCD take a contiguous range of work items, so
  // that strips next to each other in theta (which read the same cache lines
  // at their common edge) and the chunks above and below them share that
  // XCD's L2.
  int w_item = blockIdx.x;
  if (xcd_order) {
    const int nb = gridDim.x, per = nb / NXCD, extra = nb % NXCD;
    const int x = blockIdx.x % NXCD, local = blockIdx.x / NXCD;
    w_item = x * per + min(x, extra) + local;
  }
  const int strip = w_item % n_strips;
  const int chunk = w_item / n_strips;
  const int nr = T.nr, nth = T.nth;
  const int i_begin = chunk * chunk_rows;
  const int i_end = min(nr, i_begin + chunk_rows);    // every block has i_begin < nr

  StripCtx X;
  const size_t plane = (size_t)nr * nth;
  X.plane_bytes = (uint32_t)(plane * 4);
#pragma unroll
  for (int b = 0; b < NDESC; ++b) {
    X.fin[b] = __builtin_amdgcn_make_buffer_rsrc((void*)(f + b * PLANES_PER_DESC * plane), 0,
                                                 0x7fffffff, BUF_DWORD3);
    X.fout[b] = __builtin_amdgcn_make_buffer_rsrc((void*)(out + b * PLANES_PER_DESC * plane), 0,
                                                  0x7fffffff, BUF_DWORD3);
  }
  X.gh = __builtin_amdgcn_make_buffer_rsrc((void*)ghost, 0, 0x7fffffff, BUF_DWORD3);
  X.nr = nr;
  X.nth = nth;
  // column of this lane (periodic) and whether it stores an output
  const int jout = strip * OUT_COLS + lane - HALO;     // may be -2 .. nth+1
  int col = jout % nth;
  X.col = col < 0 ? col + nth : col;
  X.store = lane >= HALO && lane < WAVE - HALO && jout < nth;
  X.e = T.e;
  X.ome = 1.0 - T.e;
  X.bp_b1 = (lane - 1) << 2;
  X.bp_b2 = (lane - 2) << 2;
  X.bp_f1 = (lane + 1) << 2;
  X.bp_f2 = (lane + 2) << 2;
  DirGeom<float> G;
  dir_geometry(T.cth[X.col], T.sth[X.col], T.dt_dr, T.dt_dth, G);
  if constexpr (NSPLIT == 1) {
    strip_wave<1, 0>(T, X, G, i_begin, i_end, lds);
  } else if constexpr (NSPLIT == 2) {
    if (w == 0) strip_wave<2, 0>(T, X, G, i_begin, i_end, lds);
    else strip_wave<2, 1>(T, X, G, i_begin, i_end, lds);
  } else {
    if (w == 0) strip_wave<4, 0>(T, X, G, i_begin, i_end, lds);
    else if (w == 1) strip_wave<4, 1>(T, X, G, i_begin, i_end, lds);
    else if (w == 2) strip_wave<4, 2>(T, X, G, i_begin, i_end, lds);
    else strip_wave<4, 3>(T, X, G, i_begin, i_end, lds);
  }
}

template <class R>
bool strip_supported(const Tables& T) {
  // every buffer offset (10 planes + the lane offset) must stay below 2^31
  const double plane_bytes = 4.0 * T.nr * (double)T.nth;
  return std::is_same<R, float>::value && T.nth >= WAVE &&
         (double)PLANES_PER_DESC * plane_bytes < 2147483647.0;
}

int strip_default_chunk(const Tables& T) {
  // enough (strip, chunk) workgroups to fill 256 CUs several times over
  const int strips = (T.nth + OUT_COLS - 1) / OUT_COLS;
  int chunk = 32;
  while (chunk > 8 && (long)strips * ((T.nr + chunk - 1) / chunk) < 4096) chunk /= 2;
  return chunk;
}

template <class R>
hipError_t launch_step_strip(const Tables& T, const void* f, void* out, const void* ghost,
                             const StripTune& tune, hipStream_t s) {
  if (!strip_supported<R>(T)) return hipErrorNotSupported;
  const int chunk_rows = tune.chunk > 0 ? tune.chunk : strip_default_chunk(T);
  const int split = tune.split > 0 ? tune.split : 2;
  const int order = tune.order >= 0 ? (tune.order ? 1 : 0) : 1;
  const int strips = (T.nth + OUT_COLS - 1) / OUT_COLS;
  const int chunks = (T.nr + chunk_rows - 1) / chunk_rows;
  const int blocks = strips * chunks;
  const float* fi = (const float*)f;
  float* fo = (float*)out;
  const float* gh = (const float*)ghost;
  if (split == 1)
    hipLaunchKernelGGL(step_strip_kernel<1>, dim3(blocks), dim3(WAVE), 0, s, T, fi, fo, gh, chunk_rows, strips, order);
  else if (split == 2)
    hipLaunchKernelGGL(step_strip_kernel<2>, dim3(blocks), dim3(2 * WAVE), 0, s, T, fi, fo, gh, chunk_rows, strips, order);
  else if (split == 4)
    hipLaunchKernelGGL(step_strip_kernel<4>, dim3(blocks), dim3(4 * WAVE), 0, s, T, fi, fo, gh, chunk_rows, strips, order);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template bool strip_supported<float>(const Tables&);
template bool strip_supported<double>(const Tables&);
template hipError_t launch_step_strip<float>(const Tables&, const void*, void*, const void*,
                                             const StripTune&, hipStream_t);
template hipError_t launch_step_strip<double>(const Tables&, const void*, void*, const void*,
                                              const StripTune&, hipStream_t);

}  // namespace pclb
