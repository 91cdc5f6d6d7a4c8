// Host-side launchers of the kernels (one per kernel family, templated on the
// storage type: float for precision 32, double for precision 64).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace pclb {

template <class R>
hipError_t launch_ghost(const Tables& T, const BCdev& bc, const void* f, void* ghost, hipStream_t s);
template <class R>
hipError_t launch_step_node(const Tables& T, const void* f, void* out, const void* ghost, hipStream_t s);
// Launch shape of the strip kernel; zero fields take the defaults.  None of
// them changes the results.
struct StripTune {
  int chunk = 0;   // rows marched by one workgroup
  int order = -1;  // 1: XCD-contiguous workgroup order, 0: plain order
};
// Strips of the strip kernel that contain an octant boundary (host side).
int strip_mixed_count(int nth, int nf);
template <class R>
hipError_t launch_step_strip(const Tables& T, const void* f, void* out, const void* ghost,
                             const StripTune& tune, hipStream_t s);
template <class R>
bool strip_supported(const Tables& T);
// The FP64 strip kernel (full annulus, MWB, n_theta a multiple of 64).
bool strip64_supported(const Tables& T);
hipError_t launch_step_strip64(const Tables& T, const void* f, void* out, const void* ghost,
                               const StripTune& tune, hipStream_t s);
template <class R>
hipError_t launch_init(const Tables& T, const double* rho, const double* ur, const double* ut,
                       const double* Tt, void* f, int* bad, hipStream_t s);
template <class R>
hipError_t launch_fields(const Tables& T, const void* f, double* rho, double* ur, double* ut,
                         double* Tt, hipStream_t s);
template <class R>
hipError_t launch_diag(const Tables& T, const void* f, double* partial, double step, double* out,
                       hipStream_t s);
hipError_t launch_zero_int(int* p, hipStream_t s);
template <class R>
hipError_t launch_noneq(const Tables& T, const void* f, int kinds, double* out, hipStream_t s);
int diag_blocks();
int diag_slots();
hipError_t launch_diag_final(const double* partial, int nb, double step, double* out, hipStream_t s);

// The double and triple octagon (n_i = 16 or 24 directions per speed): ghost
// layers of 1 + 4 n_i planes, the per-node step of every scheme, initial
// state, fields and diagnostics.
template <class R>
hipError_t launch_models_ghost(const Tables& T, int ni, const BCdev& bc, const void* f, void* ghost,
                               hipStream_t s);
// strip: the strip form may be used (full annulus, MWB, n_theta a multiple of 64)
template <class R>
hipError_t launch_models_step(const Tables& T, int ni, const void* f, void* out, const void* ghost,
                              const StripTune& tune, bool strip, hipStream_t s);
template <class R>
hipError_t launch_models_init(const Tables& T, int ni, const double* rho, const double* ur,
                              const double* ut, const double* Tt, void* f, int* bad, hipStream_t s);
template <class R>
hipError_t launch_models_fields(const Tables& T, int ni, const void* f, double* rho, double* ur,
                                double* ut, double* Tt, hipStream_t s);
template <class R>
hipError_t launch_models_diag(const Tables& T, int ni, const void* f, double* partial, double step,
                              double* out, hipStream_t s);

// Adjoint.  strip: the strip form of the node adjoint where it applies.
template <class R>
hipError_t launch_adjoint(const Tables& T, const BCdev& bc, const void* f, const void* lam,
                          void* lam_out, void* ghost, double* gm, double tie,
                          const StripTune& tune, bool strip, hipStream_t s);
// The strip adjoint (FP32 states, full annulus, MWB, n_theta a multiple of 64).
bool adjoint_strip_supported(const Tables& T, int precision);
template <class R>
hipError_t launch_adjoint_strip(const Tables& T, const void* f, const void* lam, void* lam_out,
                                const void* ghost, const double* gm, double tie,
                                const StripTune& tune, hipStream_t s);
template <class R>
hipError_t launch_adjoint_init(const Tables& T, const void* lam, const double* rho,
                               const double* ur, const double* ut, const double* Tt, double* d_rho,
                               double* d_ur, double* d_ut, double* d_T, hipStream_t s);

}  // namespace pclb
