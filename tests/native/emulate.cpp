// Host emulation of the device step and adjoint step (test infrastructure):
// runs the shared per-node arithmetic of the HIP kernels (node_update,
// ghost_column, ghost_adjoint_column, adjoint_node) on the CPU, so that the
// CPU test-suite can check the device math against the oracle without a GPU.
// Loaded by tests/test_device_math.py.
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../paper_1302_7104_amd/csrc/adjoint_node.h"
#include "../../paper_1302_7104_amd/csrc/common.h"

using namespace pclb;

namespace {

struct Setup {
  std::vector<double> cth, sth, rinv, wA;
  Tables T{};
  BCdev bc{};
  Setup(int nr, int nth, int nf, double r1, double r2, double tau, double dt, const int32_t* kind,
        const double* par, int scheme = SCH_MWB, int relax = 0)
      : cth(nth), sth(nth), rinv(nr), wA(nr) {
    const double PI = 3.14159265358979323846;
    const double dr = (r2 - r1) / (nr - 1), dth = 2.0 * PI * nf / (8.0 * nth);
    for (int j = 0; j < nth; ++j) {
      cth[j] = std::cos((j + 1) * dth);
      sth[j] = std::sin((j + 1) * dth);
    }
    for (int i = 0; i < nr; ++i) rinv[i] = 1.0 / (r1 + i * dr);
    T.nr = nr;
    T.nth = nth;
    T.nf = nf;
    T.dt_dr = dt / dr;
    T.dt_dth = dt / dth;
    T.e = relax == 1 ? 1.0 - dt / tau : std::exp(-dt / tau);
    T.scheme = scheme;
    T.cth = cth.data();
    T.sth = sth.data();
    T.rinv = rinv.data();
    T.wA = wA.data();
    for (int s = 0; s < 2; ++s) {
      bc.kind[s] = kind[s] & 15;
      bc.neq[s] = (kind[s] & 16) ? 1 : 0;
      for (int a = 0; a < 4; ++a) bc.p[s][a] = par[4 * s + a];
    }
    bc.rg[0][0] = r1 - dr; bc.rg[0][1] = r1 - 2.0 * dr;
    bc.rg[1][0] = r2 + dr; bc.rg[1][1] = r2 + 2.0 * dr;
  }
};

template <class R>
void fill_ghosts(const Setup& S, const R* cur, std::vector<R>& ghost) {
  const int nr = S.T.nr, nth = S.T.nth;
  const size_t plane = (size_t)nr * nth;
  ghost.assign(4 * NQ * (size_t)nth, R(0));
  for (int side = 0; side < 2; ++side) {
    const int i0 = side == 0 ? 0 : nr - 1, i1 = side == 0 ? 1 : nr - 2;
    for (int j = 0; j < nth; ++j) {
      R f0[NQ], f1[NQ], g0[NQ], g1[NQ];
      for (int q = 0; q < NQ; ++q) {
        f0[q] = cur[q * plane + (size_t)i0 * nth + j];
        f1[q] = cur[q * plane + (size_t)i1 * nth + j];
      }
      ghost_column<R>(S.T, S.bc, side, S.cth[j], S.sth[j], f0, f1, g0, g1);
      for (int q = 0; q < NQ; ++q) {
        ghost[ghost_index(side, 0, q, j, nth)] = g0[q];
        ghost[ghost_index(side, 1, q, j, nth)] = g1[q];
      }
    }
  }
}

template <class R>
void run(int nr, int nth, int nf, double r1, double r2, double tau, double dt, const int32_t* kind,
         const double* par, const R* fin, R* fout, int nsteps, int scheme, int relax) {
  Setup S(nr, nth, nf, r1, r2, tau, dt, kind, par, scheme, relax);
  const Tables& T = S.T;
  const std::vector<double>& cth = S.cth;
  const std::vector<double>& sth = S.sth;
  const size_t plane = (size_t)nr * nth;
  std::vector<R> cur(fin, fin + NQ * plane), nxt(NQ * plane), ghost;
  for (int s = 0; s < nsteps; ++s) {
    fill_ghosts<R>(S, cur.data(), ghost);
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nth; ++j) {
        R fc[NQ], res[NQ];
        for (int q = 0; q < NQ; ++q) fc[q] = cur[q * plane + (size_t)i * nth + j];
        auto row = [&](int q, int di) -> R {
          const int ii = i + di;
          if (ii < 0) return ghost[ghost_index(0, -1 - ii, q, j, nth)];
          if (ii >= nr) return ghost[ghost_index(1, ii - nr, q, j, nth)];
          return cur[q * plane + (size_t)ii * nth + j];
        };
        // theta neighbours, the direction index rotated across the ends of a
        // sector (identity for the full annulus)
        auto col = [&](int q, int dj) -> R {
          int t = j + dj, qq = q;
          if (t < 0) { t += nth; qq = rot_q(q, nf & 7); }
          else if (t >= nth) { t -= nth; qq = rot_q(q, (8 - nf) & 7); }
          return cur[qq * plane + (size_t)i * nth + t];
        };
        switch (scheme) {
          case SCH_WB: node_update<R, SCH_WB>(T, i, j, fc, row, col, res); break;
          case SCH_LW: node_update<R, SCH_LW>(T, i, j, fc, row, col, res); break;
          case SCH_UPWIND2: node_update<R, SCH_UPWIND2>(T, i, j, fc, row, col, res); break;
          default: node_update<R, SCH_MWB>(T, i, j, fc, row, col, res);
        }
        for (int q = 0; q < NQ; ++q) nxt[q * plane + (size_t)i * nth + j] = res[q];
      }
    cur.swap(nxt);
  }
  for (size_t n = 0; n < cur.size(); ++n) fout[n] = cur[n];
}

template <class R>
void adjoint(int nr, int nth, int nf, double r1, double r2, double tau, double dt,
             const int32_t* kind, const double* par, double tie, const R* f, const R* lam, R* out) {
  Setup S(nr, nth, nf, r1, r2, tau, dt, kind, par);
  std::vector<R> ghost;
  fill_ghosts<R>(S, f, ghost);
  std::vector<double> gm(16 * (size_t)nth, 0.0);
  for (int side = 0; side < 2; ++side)
    for (int j = 0; j < nth; ++j)
      ghost_adjoint_column<R>(S.T, S.bc, f, lam, ghost.data(), tie, side, j, gm.data());
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nth; ++j) adjoint_node<R>(S.T, f, lam, ghost.data(), gm.data(), tie, i, j, out);
}

}  // namespace

// nf: theta covers 2 pi nf / 8 (8: the full annulus)
extern "C" int emu_adjoint_step(int32_t nr, int32_t nth, double r1, double r2, double tau, double dt,
                                const int32_t* kind, const double* par, int32_t precision,
                                double tie, const void* f, const void* lam, void* out, int32_t nf) {
  if (precision == 64)
    adjoint<double>(nr, nth, nf, r1, r2, tau, dt, kind, par, tie, (const double*)f,
                    (const double*)lam, (double*)out);
  else
    adjoint<float>(nr, nth, nf, r1, r2, tau, dt, kind, par, tie, (const float*)f,
                   (const float*)lam, (float*)out);
  return 0;
}

// scheme: SCH_*; relax: 0 analytic, 1 forward Euler
extern "C" int emu_steps(int32_t nr, int32_t nth, double r1, double r2, double tau, double dt,
                         const int32_t* kind, const double* par, int32_t precision,
                         const void* fin, void* fout, int32_t nsteps, int32_t nf, int32_t scheme,
                         int32_t relax) {
  if (precision == 64)
    run<double>(nr, nth, nf, r1, r2, tau, dt, kind, par, (const double*)fin, (double*)fout, nsteps,
                scheme, relax);
  else
    run<float>(nr, nth, nf, r1, r2, tau, dt, kind, par, (const float*)fin, (float*)fout, nsteps,
               scheme, relax);
  return 0;
}
