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
constexpr int WAVES_PER_BLOCK = 4;
// word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format)
constexpr int BUF_DWORD3 = 0x00020000;

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

// One output row i.  For every moving velocity the slots A, B, C hold three
// consecutive rows in increasing order: (i-2, i-1, i) when the upwind side is
// i-1 ("backward"), (i, i+1, i+2) otherwise.  After the velocity's terms are
// computed, the lowest slot A is refilled with row (lowest + 3), so that the
// roles rotate A <- B <- C <- A from one row to the next.
template <bool EDGE>
__device__ inline void strip_row(const Tables& T, const StripCtx& X, const DirGeom<float>& G, int i,
                                 float& r0, float* A, float* B, float* C) {
  const unsigned rback = G.rback, tback = G.tback;
  // moments (Eqs. moment1-3) in double
  double rho, ux, uy, E;
  {
    double fd[NQ];
    fd[0] = (double)r0;
    for_q<1>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int d = d_of(q);
      fd[q] = (double)(((rback >> d) & 1u) ? C[q] : A[q]);
    });
    node_macros(fd, rho, ux, uy, E);
  }
  EqCoef ec;
  eq_setup(T, rho, ux, uy, E, ec);
  const float rinv = (float)T.rinv[i];
  float atr[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) atr[d] = G.at[d] * rinv;
  const uint32_t ovoff = (uint32_t)(i * X.nth + X.col) * 4u;
  // rest velocity: relaxation only
  {
    const float res = relax_rest<float>(ec, X.e, X.ome, r0);
    if (X.store) store_f<0>(X, ovoff, res);
    r0 = load_f<EDGE, 0>(X, i + 1);
  }
  for_q<1>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int k = k_of(q), d = d_of(q);
    if constexpr (d < 4) {
      constexpr int qm = q + 4;
      const bool bp = (rback >> d) & 1u, bm = (rback >> (d + 4)) & 1u;
      const float cp = bp ? C[q] : A[q];
      const float cm = bm ? C[qm] : A[qm];
      float rel[2];
      relax_pair<float>(ec, X.e, X.ome, k, d, cp, cm, rel[0], rel[1]);
      float aCr, Kr, aCt, Kt;
      courant<float>((float)speed(k), G.ar[d], aCr, Kr);
      courant<float>((float)speed(k), atr[d], aCt, Kt);
      auto one = [&](auto qq, bool back, float c, float rl) {
        constexpr int Q = decltype(qq)::value;
        constexpr int D = d_of(Q);
        const bool tb = (tback >> D) & 1u;
        const float t1 = lane_from(c, tb ? X.bp_b1 : X.bp_f1);
        const float t2 = lane_from(c, tb ? X.bp_b2 : X.bp_f2);
        const float res = mwb_update<float>(rl, c, aCr, Kr, B[Q], back ? A[Q] : C[Q], aCt, Kt, t1, t2);
        if (X.store) store_f<Q>(X, ovoff, res);
        A[Q] = load_f<EDGE, Q>(X, back ? i + 1 : i + 3);
      };
      one(std::integral_constant<int, q>{}, bp, cp, rel[0]);
      one(std::integral_constant<int, qm>{}, bm, cm, rel[1]);
    }
  });
}

template <bool EDGE>
__device__ inline void strip_march(const Tables& T, const StripCtx& X, const DirGeom<float>& G,
                                   int i_begin, int i_end) {
  float S0[NQ], S1[NQ], S2[NQ];
  float r0 = load_f<EDGE, 0>(X, i_begin);
  for_q<1>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int d = d_of(q);
    const int base = ((G.rback >> d) & 1u) ? i_begin - 2 : i_begin;
    S0[q] = load_f<EDGE, q>(X, base);
    S1[q] = load_f<EDGE, q>(X, base + 1);
    S2[q] = load_f<EDGE, q>(X, base + 2);
  });
  for (int i = i_begin; i < i_end; i += 3) {
    strip_row<EDGE>(T, X, G, i, r0, S0, S1, S2);
    if (i + 1 >= i_end) break;
    strip_row<EDGE>(T, X, G, i + 1, r0, S1, S2, S0);
    if (i + 2 >= i_end) break;
    strip_row<EDGE>(T, X, G, i + 2, r0, S2, S0, S1);
  }
}

}  // namespace

__global__ void __launch_bounds__(WAVE * WAVES_PER_BLOCK)
step_strip_kernel(Tables T, const float* __restrict__ f, float* __restrict__ out,
                  const float* __restrict__ ghost, int chunk_rows, int n_strips) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wave = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  const int strip = wave % n_strips;
  const int chunk = wave / n_strips;
  const int nr = T.nr, nth = T.nth;
  const int i_begin = chunk * chunk_rows;
  if (i_begin >= nr) return;                          // whole wave exits together
  const int i_end = min(nr, i_begin + chunk_rows);

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
  // the chunk reads rows i_begin-2 .. i_end+2 (the last two only as
  // look-ahead); only chunks next to a wall touch the ghost layers
  if (i_begin < 2 || i_end + 2 >= nr) strip_march<true>(T, X, G, i_begin, i_end);
  else strip_march<false>(T, X, G, i_begin, i_end);
}

template <class R>
bool strip_supported(const Tables& T) {
  // every buffer offset (10 planes + the lane offset) must stay below 2^31
  const double plane_bytes = 4.0 * T.nr * (double)T.nth;
  return std::is_same<R, float>::value && T.nth >= WAVE &&
         (double)PLANES_PER_DESC * plane_bytes < 2147483647.0;
}

int strip_default_chunk(const Tables& T) {
  // enough (strip, chunk) waves to fill 256 CUs several times over
  const int strips = (T.nth + OUT_COLS - 1) / OUT_COLS;
  int chunk = 128;
  while (chunk > 16 && (long)strips * ((T.nr + chunk - 1) / chunk) < 8192) chunk /= 2;
  return chunk;
}

template <class R>
hipError_t launch_step_strip(const Tables& T, const void* f, void* out, const void* ghost,
                             int chunk_rows, hipStream_t s) {
  if (!strip_supported<R>(T)) return hipErrorNotSupported;
  if (chunk_rows <= 0) chunk_rows = strip_default_chunk(T);
  const int strips = (T.nth + OUT_COLS - 1) / OUT_COLS;
  const int chunks = (T.nr + chunk_rows - 1) / chunk_rows;
  const long waves = (long)strips * chunks;
  const int blocks = (int)((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
  hipLaunchKernelGGL(step_strip_kernel, dim3(blocks), dim3(WAVE * WAVES_PER_BLOCK), 0, s, T,
                     (const float*)f, (float*)out, (const float*)ghost, chunk_rows, strips);
  return hipGetLastError();
}

template bool strip_supported<float>(const Tables&);
template bool strip_supported<double>(const Tables&);
template hipError_t launch_step_strip<float>(const Tables&, const void*, void*, const void*, int, hipStream_t);
template hipError_t launch_step_strip<double>(const Tables&, const void*, void*, const void*, int, hipStream_t);

}  // namespace pclb
