// C ABI of libpclb.so: context, validation, geometry and weight tables, and
// launch orchestration of the polar FDLB step (see include/pclb.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>

#include "../../include/pclb.h"
#include "common.h"
#include "launch.h"

using namespace pclb;

// Scratch of pclb_step_static: the radial ghost layers (4 * (1 + 4 n_i) *
// n_theta elements of the state type) in a file-scope device array, so that the entry
// point needs no allocation.  Every GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the per-device
// address hipGetSymbolAddress returns (the array's name is a host-side
// stand-in, not a device address).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

struct pclb_ctx {
  pclb_config cfg{};
  int device = 0;
  double dr = 0, dth = 0;
  Tables T{};
  BCdev bc{};
  void* f[2] = {nullptr, nullptr};
  int cur = 0;
  bool bound = false;
  hipStream_t stream = nullptr;
  int64_t steps = 0;
  StripTune tune;               // strip kernel launch shape
  double tie = 0;               // adjoint tie threshold
  // context-owned device memory
  double* d_geom = nullptr;     // cth[nth], sth[nth], rinv[nr], wA[nr]
  void* d_ghost = nullptr;      // 4 * nq * nth elements of the state type, nq = 1 + 4 n_i
  double* d_partial = nullptr;  // diagnostics partials
  double* d_diag = nullptr;     // 8 doubles for the synchronizing variant
  int* d_flag = nullptr;        // init validation flag
  double* d_gm = nullptr;       // adjoint: ghost moment cotangents 2*2*4*nth
  void* d_scratch = nullptr;    // this device's copy of the static scratch array
  // pclb_step_graph: the executable graph of `gsteps` steps starting from
  // buffer `gcur`, captured on `gstream` (a non-blocking stream of the
  // context) at configuration stamp `gstamp`; `stamp` moves with every
  // pclb_set_bc and pclb_bind, which change what the kernels are given
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t gsteps = 0;
  int gcur = -1;
  uint64_t gstamp = 0, stamp = 1;
  std::string err;
};

namespace {

thread_local std::string g_create_error;

constexpr double PI = 3.14159265358979323846;

size_t elem_size(const pclb_ctx* c) { return c->cfg.precision == 32 ? 4 : 8; }

int fail(pclb_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return code;
}

int hip_fail(pclb_ctx* c, hipError_t e, const char* where) {
  return fail(c, PCLB_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// velocities of the model: the rest velocity and n_i directions per speed
int model_nq(int ni) { return 1 + NK * ni; }
bool model_ok(int ni) { return ni == 8 || ni == 16 || ni == 24; }

// theta increment of Sec. II.C: 2 pi n_f / (n_i n_theta)
double sector_dth(const pclb_config* c) { return 2.0 * PI * c->n_f / ((double)c->n_i * c->n_theta); }

int validate(const pclb_config* c, std::string& why) {
  if (!c) { why = "null config"; return PCLB_EINVAL; }
  if (!(c->r1 > 0.0) || !(c->r2 > c->r1)) { why = "need 0 < r1 < r2"; return PCLB_EINVAL; }
  if (c->n_r < 4) { why = "n_r must be >= 4"; return PCLB_EINVAL; }
  if (c->n_theta < 8) { why = "n_theta must be >= 8"; return PCLB_EINVAL; }
  if ((int64_t)c->n_r * c->n_theta > (int64_t)1 << 31) { why = "grid too large"; return PCLB_EINVAL; }
  if (!(c->tau > 0.0) || !std::isfinite(c->tau)) { why = "tau must be > 0"; return PCLB_EINVAL; }
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) { why = "dt must be > 0"; return PCLB_EINVAL; }
  if (!model_ok(c->n_i)) { why = "n_i must be 8, 16 or 24 (Table I)"; return PCLB_EINVAL; }
  if (c->n_f < 1 || c->n_f > c->n_i) { why = "n_f must be in 1..n_i (theta covers 2 pi n_f / n_i)"; return PCLB_EINVAL; }
  if (c->precision != 32 && c->precision != 64) { why = "precision must be 32 or 64"; return PCLB_EINVAL; }
  if (c->fp64_collision != 1) {
    why = "fp64_collision must be 1 (float collision is not offered: it loses accuracy and no time)";
    return PCLB_EINVAL;
  }
  if (c->kernel < 0 || c->kernel > 2) { why = "unknown kernel selection"; return PCLB_EINVAL; }
  if (c->strip_chunk < 0 || c->strip_chunk > 64 || c->strip_order < 0 || c->strip_order > 2) {
    why = "strip launch shape out of range (strip_chunk 0-64, strip_order 0-2)";
    return PCLB_EINVAL;
  }
  if (!(c->adjoint_tie >= 0.0) || !(c->adjoint_tie < 1e-2)) {
    why = "adjoint_tie must be in [0, 1e-2)";
    return PCLB_EINVAL;
  }
  if (c->scheme < PCLB_SCHEME_MWB || c->scheme > PCLB_SCHEME_UPWIND2) { why = "unknown scheme"; return PCLB_EINVAL; }
  if (c->relaxation != PCLB_RELAX_ANALYTIC && c->relaxation != PCLB_RELAX_EULER) {
    why = "unknown relaxation";
    return PCLB_EINVAL;
  }
  double dr = (c->r2 - c->r1) / (c->n_r - 1);
  double dth = sector_dth(c);
  double vmax = speed(NK);
  double cr = vmax * c->dt / dr, ct = vmax * c->dt / (c->r1 * dth);
  if (cr > 1.0 || ct > 1.0) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "Courant numbers max|C_r| = %.4g, max|C_theta| = %.4g exceed 1", cr, ct);
    why = buf;
    return PCLB_ECFL;
  }
  return PCLB_OK;
}

// The strip kernels march one workgroup per (64-column strip, chunk of at
// least 8 rows); with fewer than 512 such workgroups a grid leaves most of
// the GPU idle and the one-thread-per-node kernel is faster (measured: 25
// against 50 us per FP32 step at 64 x 128, 31 against 43 at 256 x 512; the
// strip kernel wins from 512 x 1024 on, 55 against 78 us).  Only the
// automatic choice looks at this; an explicit PCLB_KERNEL_STRIP is obeyed
// wherever the strip kernel can run.
bool strip_pays(const pclb_ctx* c) {
  const pclb_config& g = c->cfg;
  return g.kernel == PCLB_KERNEL_STRIP ||
         (int64_t)((g.n_theta + 63) / 64) * ((g.n_r + 7) / 8) >= 512;
}

template <class R>
hipError_t do_step(pclb_ctx* c, const void* in, void* out, void* ghost) {
  if (c->cfg.n_i != 8) {
    hipError_t e = launch_models_ghost<R>(c->T, c->cfg.n_i, c->bc, in, ghost, c->stream);
    if (e != hipSuccess) return e;
    const bool strip = (c->cfg.kernel == PCLB_KERNEL_STRIP || c->cfg.kernel == PCLB_KERNEL_AUTO) && strip_pays(c);
    return launch_models_step<R>(c->T, c->cfg.n_i, in, out, ghost, c->tune, strip, c->stream);
  }
  hipError_t e = launch_ghost<R>(c->T, c->bc, in, ghost, c->stream);
  if (e != hipSuccess) return e;
  int kern = c->cfg.kernel;
  if ((kern == PCLB_KERNEL_STRIP || kern == PCLB_KERNEL_AUTO) && strip_pays(c)) {
    if constexpr (std::is_same<R, float>::value) {
      if (strip_supported<R>(c->T)) return launch_step_strip<R>(c->T, in, out, ghost, c->tune, c->stream);
    } else {
      if (strip64_supported(c->T)) return launch_step_strip64(c->T, in, out, ghost, c->tune, c->stream);
    }
  }
  return launch_step_node<R>(c->T, in, out, ghost, c->stream);
}

hipError_t step_once(pclb_ctx* c, const void* in, void* out, void* ghost) {
  return c->cfg.precision == 32 ? do_step<float>(c, in, out, ghost)
                                : do_step<double>(c, in, out, ghost);
}

size_t ghost_bytes(const pclb_ctx* c) { return 4 * (size_t)model_nq(c->cfg.n_i) * c->cfg.n_theta * elem_size(c); }

}  // namespace

extern "C" {

double pclb_cfl_dt(const pclb_config* cfg, double cfl) {
  if (!cfg || !(cfg->r1 > 0) || !(cfg->r2 > cfg->r1) || cfg->n_r < 2 || cfg->n_theta < 1 ||
      !model_ok(cfg->n_i) || cfg->n_f < 1 || cfg->n_f > cfg->n_i || !(cfl > 0))
    return -1.0;
  double dr = (cfg->r2 - cfg->r1) / (cfg->n_r - 1);
  double dth = sector_dth(cfg);
  return cfl * std::fmin(dr, cfg->r1 * dth) / speed(NK);
}

int pclb_create(const pclb_config* cfg, pclb_ctx** out) {
  if (!out) return fail(nullptr, PCLB_EINVAL, "null output pointer");
  *out = nullptr;
  std::string why;
  int rc = validate(cfg, why);
  if (rc != PCLB_OK) return fail(nullptr, rc, why);
  pclb_ctx* c = new (std::nothrow) pclb_ctx();
  if (!c) return fail(nullptr, PCLB_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  // launch shape of the strip kernel (results do not depend on it)
  c->tune.chunk = cfg->strip_chunk;
  c->tune.order = cfg->strip_order == PCLB_ORDER_PLAIN ? 0 : 1;
  c->tie = cfg->adjoint_tie > 0.0 ? cfg->adjoint_tie : (cfg->precision == 64 ? 1e-13 : 1e-6);
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) { delete c; return fail(nullptr, PCLB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e)); }
  const int nr = cfg->n_r, nth = cfg->n_theta;
  c->dr = (cfg->r2 - cfg->r1) / (nr - 1);
  c->dth = sector_dth(cfg);
  // geometry tables: node angles theta_j = (j+1) dtheta, radii r_i = R1 + i dr
  std::string host_err;
  size_t ngeom = 2 * (size_t)nth + 2 * (size_t)nr;
  double* h = new (std::nothrow) double[ngeom];
  if (!h) { delete c; return fail(nullptr, PCLB_ENOMEM, "host allocation failed"); }
  for (int j = 0; j < nth; ++j) {
    double th = (j + 1) * c->dth;
    h[j] = std::cos(th);
    h[nth + j] = std::sin(th);
  }
  for (int i = 0; i < nr; ++i) {
    double r = cfg->r1 + i * c->dr;
    h[2 * nth + i] = 1.0 / r;
    double w = (i == 0 || i == nr - 1) ? 0.5 : 1.0;
    h[2 * nth + nr + i] = r * w * c->dr * c->dth;
  }
  // this device's address of the static scratch array (used by pclb_step_static)
  e = hipGetSymbolAddress(&c->d_scratch, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    delete[] h;
    delete c;
    return fail(nullptr, PCLB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  size_t es = cfg->precision == 32 ? 4 : 8;
  bool ok = hipMalloc(&c->d_geom, ngeom * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_ghost, 4 * (size_t)model_nq(cfg->n_i) * nth * es) == hipSuccess &&
            hipMalloc(&c->d_partial, (size_t)diag_blocks() * diag_slots() * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_diag, 8 * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_flag, sizeof(int)) == hipSuccess &&
            hipMalloc(&c->d_gm, 16 * (size_t)nth * sizeof(double)) == hipSuccess;

  if (!ok) {
    delete[] h;
    pclb_destroy(c);
    return fail(nullptr, PCLB_ENOMEM, "device allocation of context tables failed");
  }
  e = hipMemcpy(c->d_geom, h, ngeom * sizeof(double), hipMemcpyHostToDevice);
  delete[] h;

  if (e != hipSuccess) { pclb_destroy(c); return fail(nullptr, PCLB_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e)); }
  Tables& T = c->T;
  T.nr = nr;
  T.nth = nth;
  T.nf = cfg->n_f;
  T.dt_dr = cfg->dt / c->dr;
  T.dt_dth = cfg->dt / c->dth;
  // both relaxations are f^eq + (f - f^eq) e: Eq. operator1_new with
  // e = exp(-dt/tau), Eq. operator1_old with e = 1 - dt/tau
  T.e = cfg->relaxation == PCLB_RELAX_EULER ? 1.0 - cfg->dt / cfg->tau : std::exp(-cfg->dt / cfg->tau);
  T.scheme = cfg->scheme;
  T.cth = c->d_geom;
  T.sth = c->d_geom + nth;
  T.rinv = c->d_geom + 2 * nth;
  T.wA = c->d_geom + 2 * nth + nr;
  T.n_mixed = cfg->n_i == 8 ? strip_mixed_count(nth, cfg->n_f) : 0;
  for (int s = 0; s < 2; ++s) {
    c->bc.kind[s] = PCLB_WALL;
    c->bc.neq[s] = 0;
    for (int a = 0; a < 4; ++a) c->bc.p[s][a] = 0.0;
  }
  c->bc.rg[0][0] = cfg->r1 - c->dr;
  c->bc.rg[0][1] = cfg->r1 - 2.0 * c->dr;
  c->bc.rg[1][0] = cfg->r2 + c->dr;
  c->bc.rg[1][1] = cfg->r2 + 2.0 * c->dr;
  *out = c;
  return PCLB_OK;
}

void pclb_destroy(pclb_ctx* c) {
  if (!c) return;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->d_geom) (void)hipFree(c->d_geom);
  if (c->d_ghost) (void)hipFree(c->d_ghost);
  if (c->d_partial) (void)hipFree(c->d_partial);
  if (c->d_diag) (void)hipFree(c->d_diag);
  if (c->d_flag) (void)hipFree(c->d_flag);
  if (c->d_gm) (void)hipFree(c->d_gm);
  delete c;
}

const char* pclb_last_error(const pclb_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

int pclb_bind(pclb_ctx* c, void* f0, void* f1, void* stream) {
  if (!c) return PCLB_EINVAL;
  if (!f0 || !f1 || f0 == f1) return fail(c, PCLB_EINVAL, "two distinct non-null buffers are required");
  c->f[0] = f0;
  c->f[1] = f1;
  c->cur = 0;
  c->stream = (hipStream_t)stream;
  c->bound = true;
  c->steps = 0;
  ++c->stamp;
  return PCLB_OK;
}

int pclb_set_bc(pclb_ctx* c, int32_t side, int32_t kind, const double p[4]) {
  if (!c) return PCLB_EINVAL;
  if (side < 0 || side > 1) return fail(c, PCLB_EINVAL, "side must be 0 (inner) or 1 (outer)");
  const int neq = (kind & PCLB_BC_NONEQ) ? 1 : 0;
  kind &= ~PCLB_BC_NONEQ;
  if (kind < PCLB_WALL || kind > PCLB_EXTRAPOLATE) return fail(c, PCLB_EINVAL, "unknown boundary kind");
  double q[4] = {0, 0, 0, 0};
  if (kind != PCLB_EXTRAPOLATE) {
    if (!p) return fail(c, PCLB_EINVAL, "boundary parameters required");
    for (int a = 0; a < 4; ++a) q[a] = p[a];
  }
  for (int a = 0; a < 4; ++a)
    if (!std::isfinite(q[a])) return fail(c, PCLB_EINVAL, "non-finite boundary parameter");
  if (kind == PCLB_INFLOW && (!(q[0] > 0.0) || !(q[3] > 0.0)))
    return fail(c, PCLB_EINVAL, "inflow density and temperature must be > 0");
  c->bc.kind[side] = kind;
  c->bc.neq[side] = neq;
  for (int a = 0; a < 4; ++a) c->bc.p[side][a] = q[a];
  ++c->stamp;
  return PCLB_OK;
}

int pclb_init_state(pclb_ctx* c, const double* rho, const double* ur, const double* ut, const double* T) {
  if (!c) return PCLB_EINVAL;
  if (!c->bound) return fail(c, PCLB_ESTATE, "bind buffers first");
  if (!rho || !ur || !ut || !T) return fail(c, PCLB_EINVAL, "null field pointer");
  hipError_t e = launch_zero_int(c->d_flag, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "flag reset");
  const int ni = c->cfg.n_i;
  if (ni != 8)
    e = c->cfg.precision == 32
            ? launch_models_init<float>(c->T, ni, rho, ur, ut, T, c->f[c->cur], c->d_flag, c->stream)
            : launch_models_init<double>(c->T, ni, rho, ur, ut, T, c->f[c->cur], c->d_flag, c->stream);
  else
    e = c->cfg.precision == 32
            ? launch_init<float>(c->T, rho, ur, ut, T, c->f[c->cur], c->d_flag, c->stream)
            : launch_init<double>(c->T, rho, ur, ut, T, c->f[c->cur], c->d_flag, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "init launch");
  int flag = 0;
  e = hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "init sync");
  c->steps = 0;
  if (flag) return fail(c, PCLB_EINVAL, "initial fields need rho > 0, T > 0 and finite values");
  return PCLB_OK;
}

int pclb_step(pclb_ctx* c, int64_t n) {
  if (!c) return PCLB_EINVAL;
  if (!c->bound) return fail(c, PCLB_ESTATE, "bind buffers first");
  if (n < 0) return fail(c, PCLB_EINVAL, "negative step count");
  for (int64_t s = 0; s < n; ++s) {
    hipError_t e = step_once(c, c->f[c->cur], c->f[1 - c->cur], c->d_ghost);
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
    c->cur = 1 - c->cur;
    ++c->steps;
  }
  return PCLB_OK;
}

int pclb_step_static(pclb_ctx* c, int64_t n) {
  if (!c) return PCLB_EINVAL;
  if (!c->bound) return fail(c, PCLB_ESTATE, "bind buffers first");
  if (n < 0) return fail(c, PCLB_EINVAL, "negative step count");
  if (ghost_bytes(c) > STATIC_SCRATCH_BYTES) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "ghost layers need %zu bytes, above the %zu-byte static scratch (n_theta <= %zu "
                  "at this precision and n_i)",
                  ghost_bytes(c), STATIC_SCRATCH_BYTES, STATIC_SCRATCH_BYTES / (4 * model_nq(c->cfg.n_i) * elem_size(c)));
    return fail(c, PCLB_EINVAL, buf);
  }
  for (int64_t s = 0; s < n; ++s) {
    hipError_t e = step_once(c, c->f[c->cur], c->f[1 - c->cur], c->d_scratch);
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
    c->cur = 1 - c->cur;
    ++c->steps;
  }
  return PCLB_OK;
}

int pclb_step_graph(pclb_ctx* c, int64_t n) {
  if (!c) return PCLB_EINVAL;
  if (!c->bound) return fail(c, PCLB_ESTATE, "bind buffers first");
  if (n < 0 || n > 100000) return fail(c, PCLB_EINVAL, "step count must be in 0..100000");
  if (n == 0) return PCLB_OK;
  hipError_t e = hipSuccess;
  if (!c->gexec || c->gsteps != n || c->gcur != c->cur || c->gstamp != c->stamp) {
    if (c->gexec) {
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
    if (!c->gstream) {
      e = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(c, e, "capture stream");
    }
    // record n steps on the capture stream (nothing runs), buffers alternating
    // from the current one
    hipStream_t keep = c->stream;
    c->stream = c->gstream;
    e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      c->stream = keep;
      return hip_fail(c, e, "begin capture");
    }
    int cur = c->cur;
    hipError_t le = hipSuccess;
    for (int64_t k = 0; k < n && le == hipSuccess; ++k) {
      le = step_once(c, c->f[cur], c->f[1 - cur], c->d_ghost);
      cur = 1 - cur;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->gstream, &g);
    c->stream = keep;
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(c, le, "step launch under capture");
    }
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->gexec = nullptr;
      return hip_fail(c, e, "graph instantiate");
    }
    c->gsteps = n;
    c->gcur = c->cur;
    c->gstamp = c->stamp;
  }
  e = hipGraphLaunch(c->gexec, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "graph launch");
  if (n & 1) c->cur = 1 - c->cur;
  c->steps += n;
  return PCLB_OK;
}

int pclb_step_into(pclb_ctx* c, const void* f_in, void* f_out) {
  if (!c) return PCLB_EINVAL;
  if (!f_in || !f_out || f_in == f_out) return fail(c, PCLB_EINVAL, "distinct non-null buffers required");
  hipError_t e = step_once(c, f_in, f_out, c->d_ghost);
  if (e != hipSuccess) return hip_fail(c, e, "step launch");
  return PCLB_OK;
}

int pclb_current(const pclb_ctx* c, int32_t* which) {
  if (!c || !which) return PCLB_EINVAL;
  *which = c->cur;
  return PCLB_OK;
}

int pclb_step_count(const pclb_ctx* c, int64_t* steps) {
  if (!c || !steps) return PCLB_EINVAL;
  *steps = c->steps;
  return PCLB_OK;
}

int pclb_moments_of(pclb_ctx* c, const void* f, double* rho, double* ur, double* ut, double* T,
                    double* diag8) {
  if (!c) return PCLB_EINVAL;
  if (!f) return fail(c, PCLB_EINVAL, "null state buffer");
  hipError_t e = hipSuccess;
  const int ni = c->cfg.n_i;
  const bool f32 = c->cfg.precision == 32;
  if (rho || ur || ut || T) {
    if (ni != 8)
      e = f32 ? launch_models_fields<float>(c->T, ni, f, rho, ur, ut, T, c->stream)
              : launch_models_fields<double>(c->T, ni, f, rho, ur, ut, T, c->stream);
    else
      e = f32 ? launch_fields<float>(c->T, f, rho, ur, ut, T, c->stream)
              : launch_fields<double>(c->T, f, rho, ur, ut, T, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "fields launch");
  if (diag8) {
    const double step = (double)c->steps;
    if (ni != 8)
      e = f32 ? launch_models_diag<float>(c->T, ni, f, c->d_partial, step, diag8, c->stream)
              : launch_models_diag<double>(c->T, ni, f, c->d_partial, step, diag8, c->stream);
    else
      e = f32 ? launch_diag<float>(c->T, f, c->d_partial, step, diag8, c->stream)
              : launch_diag<double>(c->T, f, c->d_partial, step, diag8, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "diagnostics launch");
  }
  return PCLB_OK;
}

int pclb_moments(pclb_ctx* c, double* rho, double* ur, double* ut, double* T, double* diag8) {
  if (!c) return PCLB_EINVAL;
  if (!c->bound) return fail(c, PCLB_ESTATE, "bind buffers first");
  return pclb_moments_of(c, c->f[c->cur], rho, ur, ut, T, diag8);
}

int pclb_moments_host(pclb_ctx* c, double* diag8_host) {
  if (!c) return PCLB_EINVAL;
  if (!diag8_host) return fail(c, PCLB_EINVAL, "null output");
  int rc = pclb_moments(c, nullptr, nullptr, nullptr, nullptr, c->d_diag);
  if (rc != PCLB_OK) return rc;
  hipError_t e = hipMemcpyAsync(diag8_host, c->d_diag, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics copy");
  if (diag8_host[6] != 0.0) return fail(c, PCLB_ENONFINITE, "non-finite distribution values found");
  return PCLB_OK;
}

int pclb_noneq(pclb_ctx* c, const void* f, int32_t kinds, double* out) {
  if (!c) return PCLB_EINVAL;
  if (kinds <= 0 || kinds > PCLB_NONEQ_ALL) return fail(c, PCLB_EINVAL, "kinds must be a nonzero mask of PCLB_NONEQ_*");
  if (!out) return fail(c, PCLB_EINVAL, "null output");
  if (c->cfg.n_i != 8) return fail(c, PCLB_EINVAL, "non-equilibrium moments are built for the octagon (n_i = 8) only");
  if (!f) {
    if (!c->bound) return fail(c, PCLB_ESTATE, "bind buffers first");
    f = c->f[c->cur];
  }
  hipError_t e = c->cfg.precision == 32 ? launch_noneq<float>(c->T, f, kinds, out, c->stream)
                                        : launch_noneq<double>(c->T, f, kinds, out, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "non-equilibrium launch");
  return PCLB_OK;
}

int pclb_adjoint_step(pclb_ctx* c, const void* f_t, const void* lam_next, void* lam_out) {
  if (!c) return PCLB_EINVAL;
  if (!f_t || !lam_next || !lam_out || lam_out == lam_next || lam_out == f_t)
    return fail(c, PCLB_EINVAL, "three non-null buffers, lam_out distinct from the inputs");
  if (c->cfg.scheme != PCLB_SCHEME_MWB) return fail(c, PCLB_EINVAL, "the adjoint covers the MWB scheme only");
  if (c->cfg.n_i != 8) return fail(c, PCLB_EINVAL, "the adjoint covers the octagon (n_i = 8) only");
  if (c->bc.neq[0] || c->bc.neq[1])
    return fail(c, PCLB_EINVAL, "the adjoint covers equilibrium ghost layers only (no PCLB_BC_NONEQ)");
  // the strip form where it applies and, unless asked for, where the grid
  // gives it enough workgroups
  const int kern = c->cfg.kernel;
  const bool strip = kern == PCLB_KERNEL_STRIP || (kern == PCLB_KERNEL_AUTO && strip_pays(c));
  hipError_t e = c->cfg.precision == 32
                     ? launch_adjoint<float>(c->T, c->bc, f_t, lam_next, lam_out, c->d_ghost, c->d_gm,
                                             c->tie, c->tune, strip, c->stream)
                     : launch_adjoint<double>(c->T, c->bc, f_t, lam_next, lam_out, c->d_ghost, c->d_gm,
                                              c->tie, c->tune, strip, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint launch");
  return PCLB_OK;
}

int pclb_adjoint_init(pclb_ctx* c, const void* lam0, const double* rho, const double* ur,
                      const double* ut, const double* T, double* d_rho, double* d_ur, double* d_ut,
                      double* d_T) {
  if (!c) return PCLB_EINVAL;
  if (!lam0 || !rho || !ur || !ut || !T || !d_rho || !d_ur || !d_ut || !d_T)
    return fail(c, PCLB_EINVAL, "null pointer");
  if (c->cfg.n_i != 8) return fail(c, PCLB_EINVAL, "the adjoint covers the octagon (n_i = 8) only");
  hipError_t e = c->cfg.precision == 32
                     ? launch_adjoint_init<float>(c->T, lam0, rho, ur, ut, T, d_rho, d_ur, d_ut, d_T, c->stream)
                     : launch_adjoint_init<double>(c->T, lam0, rho, ur, ut, T, d_rho, d_ur, d_ut, d_T, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint init launch");
  return PCLB_OK;
}

}  // extern "C"
