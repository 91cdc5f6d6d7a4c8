// Driver for an AddressSanitizer / UndefinedBehaviorSanitizer host build of
// the device arithmetic (test infrastructure, built with hipcc for the host
// only and run by tests/test_sanitizers.py): runs the emulated step and
// adjoint step of tests/native/emulate.cpp in both precisions with each
// radial boundary kind, on the full annulus and on sectors, and every
// convection scheme with forward-Euler relaxation.
#include <cmath>
#include <cstdio>
#include <vector>

#include "emulate.cpp"

template <class R>
static double run_case(const int32_t* kind, const double* par, int prec, int nf) {
  const int nr = 9, nth = 70, NQ = 33;
  const size_t ns = (size_t)NQ * nr * nth;
  std::vector<R> f(ns), fo(ns), lam(ns), lo(ns);
  // a smooth positive state: f^eq-like magnitudes with a ripple
  for (size_t q = 0; q < ns; ++q) f[q] = (R)(0.02 * (1.0 + 0.1 * std::sin(0.01 * (double)q)));
  for (size_t q = 0; q < ns; ++q) lam[q] = (R)std::cos(0.003 * (double)q);
  for (int sch = 1; sch < 4; ++sch)
    emu_steps(nr, nth, 0.5, 1.5, 2e-3, 1e-3, kind, par, prec, f.data(), fo.data(), 2, nf, sch, 1);
  emu_steps(nr, nth, 0.5, 1.5, 2e-3, 1e-3, kind, par, prec, f.data(), fo.data(), 2, nf, 0, 0);
  emu_adjoint_step(nr, nth, 0.5, 1.5, 2e-3, 1e-3, kind, par, prec, prec == 64 ? 1e-13 : 1e-6,
                   fo.data(), lam.data(), lo.data(), nf);
  return (double)fo[ns / 2] + (double)lo[ns / 3];
}

int main() {
  const int32_t kinds[3][2] = {{0, 0}, {1, 2}, {2, 1}};
  const double par[8] = {1.1, 0.05, 0.0, 1.0, 0.9, -0.03, 0.1, 0.95};
  double sink = 0;
  for (const auto& k : kinds)
    for (int nf : {8, 1, 3}) {
      sink += run_case<double>(k, par, 64, nf);
      sink += run_case<float>(k, par, 32, nf);
    }
  std::printf("ok %.6e\n", sink);
  return 0;
}
