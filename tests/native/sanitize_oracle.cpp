// Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
// oracle (test infrastructure, built and run by tests/test_sanitizers.py):
// calls every exported oracle routine on small grids with each radial
// boundary kind, on the full annulus and on sectors, and on states that take
// the error paths (a non-finite value, a non-positive ghost temperature).
// Exits non-zero, through the sanitizers, on any invalid access or undefined
// operation.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

struct OrGrid {
  int32_t nr, nth;
  double r1, r2, tau, dt;
  int32_t bc_kind[2];
  double bc_par[2][4];
  int32_t terms;
  int32_t nf;
  int32_t scheme, relax;
  int32_t ni;
};

extern "C" {
int or_num_velocities();
void or_velocities(double* vx, double* vy, int32_t* k);
void or_weights(double E, int32_t row, double* F);
void or_feq(double rho, double ux, double uy, double E, double* out);
void or_macros(const double* f, double* out);
void or_relax_node(const double* f, double dt, double tau, double* out);
double or_mwb_term(double C, const double* psi, int32_t s_mode);
double or_mwb_term_eta(double C, const double* psi);
void or_mwb_grad(double C, const double* psi, double tie_eps, double* g);
int or_step(const OrGrid* g, const double* f_in, double* f_out, int32_t nsteps);
void or_step_sample(const OrGrid* g, const double* f, const int32_t* nodes, int32_t count, double* out);
void or_init_feq(const OrGrid* g, const double* rho, const double* ur, const double* ut,
                 const double* T, double* f);
void or_fields(const OrGrid* g, const double* f, double* rho, double* ur, double* ut, double* T);
void or_diagnostics(const OrGrid* g, const double* f, double* out);
int or_adjoint_step(const OrGrid* g, const double* f_t, const double* lam_next, double tie_eps,
                    double* out);
void or_adjoint_init(const OrGrid* g, const double* rho, const double* ur, const double* ut,
                     const double* T, const double* lam, double* d_rho, double* d_ur, double* d_ut,
                     double* d_T);
void or_noneq(const OrGrid* g, const double* f, double* out);
void or_noneq_sample(const OrGrid* g, const double* f, const int32_t* nodes, int32_t count,
                     double* out);
}

int main() {
  const int NQ = or_num_velocities();
  double sink = 0;
  {
    std::vector<double> vx(NQ), vy(NQ), F(5);
    std::vector<int32_t> k(NQ);
    or_velocities(vx.data(), vy.data(), k.data());
    for (int row = 0; row < 3; ++row) or_weights(1.1, row, F.data());
    std::vector<double> fe(NQ), rel(NQ), mac(4);
    or_feq(1.2, 0.1, -0.2, 1.3, fe.data());
    or_macros(fe.data(), mac.data());
    or_relax_node(fe.data(), 1e-3, 2e-3, rel.data());
    // stencils psi_{j-2..j+2}: flat, smooth, a kink, one-sided ties
    const double psis[4][5] = {{1, 1, 1, 1, 1}, {1, 2, 4, 3, 2}, {0.5, 1, 1, 2, 2}, {1, 1, 2, 3, 3}};
    for (const auto& p : psis)
      for (double C : {-0.4, 0.0, 0.3}) {
        double g[5];
        sink += or_mwb_term(C, p, 0) + or_mwb_term(C, p, 1) + or_mwb_term_eta(C, p);
        or_mwb_grad(C, p, 1e-13, g);
        sink += g[0] + g[1] + g[2] + g[3] + g[4];
      }
  }
  const int nr = 9, nth = 40;
  const size_t n = (size_t)nr * nth, ns = (size_t)NQ * n;
  const int32_t kinds[3][2] = {{0, 0}, {1, 2}, {2, 1}};
  for (const auto& kd : kinds)
  for (int nf : {8, 1, 3}) {
    OrGrid g{nr, nth, 0.5, 1.5, 2e-3, 1e-3, {kd[0], kd[1]}, {{0.2, 0, 0, 0}, {1.05, 0.02, 0.01, 0.95}}, 7, nf,
             0, nf == 3 ? 1 : 0, 8};
    if (kd[0] == 1) { g.bc_par[0][0] = 1.1; g.bc_par[0][1] = 0.05; g.bc_par[0][2] = 0.0; g.bc_par[0][3] = 1.0; }
    std::vector<double> rho(n), ur(n), ut(n), T(n);
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nth; ++j) {
        const size_t c = (size_t)i * nth + j;
        rho[c] = 1.0 + 0.05 * std::sin(0.3 * i + 0.2 * j);
        ur[c] = 0.02 * std::cos(0.1 * j);
        ut[c] = 0.1 * std::sin(0.4 * i);
        T[c] = 1.0 + 0.03 * std::cos(0.5 * i - 0.3 * j);
      }
    std::vector<double> f(ns), f1(ns), lam(ns), lo(ns), d(8), nq(4 * 12 * n);
    or_init_feq(&g, rho.data(), ur.data(), ut.data(), T.data(), f.data());
    if (or_step(&g, f.data(), f1.data(), 3) != 0) return 2;
    const int32_t nodes[] = {0, 0, nr - 1, nth - 1, 4, 17};
    std::vector<double> smp(3 * NQ), nqs(3 * 4 * 12);
    or_step_sample(&g, f1.data(), nodes, 3, smp.data());
    or_fields(&g, f1.data(), rho.data(), ur.data(), nullptr, T.data());
    or_diagnostics(&g, f1.data(), d.data());
    for (size_t q = 0; q < ns; ++q) lam[q] = std::sin(0.001 * (double)q);
    if (or_adjoint_step(&g, f1.data(), lam.data(), 1e-13, lo.data()) != 0) return 4;
    // every convection scheme through the step and the sampled step
    for (int sch = 1; sch < 4; ++sch) {
      OrGrid gs = g;
      gs.scheme = sch;
      std::vector<double> fs(ns);
      if (or_step(&gs, f.data(), fs.data(), 2) != 0) return 5;
      or_step_sample(&gs, f.data(), nodes, 3, smp.data());
      sink += fs[ns / 4] + smp[1];
      if (or_adjoint_step(&gs, f1.data(), lam.data(), 1e-13, lo.data()) != -1) return 6;
    }
    std::vector<double> dr(n), du(n), dv(n), dT(n);
    or_adjoint_init(&g, rho.data(), ur.data(), ut.data(), T.data(), lam.data(), dr.data(), du.data(),
                    dv.data(), dT.data());
    or_noneq(&g, f1.data(), nq.data());
    or_noneq_sample(&g, f1.data(), nodes, 3, nqs.data());
    sink += f1[ns / 2] + lo[ns / 3] + d[0] + dr[5] + nq[7] + nqs[11] + smp[2];
    // error paths: a non-finite value is counted; a non-positive ghost state
    // makes or_step report bad ghosts
    f1[17] = NAN;
    or_diagnostics(&g, f1.data(), d.data());
    if (d[6] < 1) return 3;
    for (int q = 0; q < NQ; ++q)
      for (int j = 0; j < nth; ++j) f[((size_t)q * nr + 0) * nth + j] = q == 0 ? -1.0 : 0.0;
    (void)or_step(&g, f.data(), f1.data(), 1);
  }
  std::printf("ok %.6e\n", sink);
  return 0;
}
