/*
 * pclb.h — C ABI of the MI355X polar-coordinate FDLB library (libpclb.so).
 *
 * The library advances the 33 discrete-velocity distributions f_q of the
 * octagon velocity model (Lin, Xu, Zhang, Li, Succi, "Polar coordinate lattice
 * Boltzmann modeling of compressible flows", arXiv:1302.7104, Sec. II.A,
 * Eq. DVM1 and Table I row 1), or the 65 and 97 of the double and triple
 * octagon (Table I rows 2 and 3, pclb_config.n_i = 16 and 24), on an annulus
 * R1 <= r <= R2 or a sector of it (Sec. II.C) with the combined scheme of
 * Sec. II.B (Eq. combined_scheme): analytic BGK relaxation (Eq.
 * operator1_new) plus the Modified Warming-Beam convection terms in r and
 * theta (Eq. MWB Scheme with the switch S(eta) = (|eta|-1)/(|eta|+1)), all
 * evaluated from f at time t.  Boundaries: periodic in theta (Sec. II.C,
 * azimuthal boundary condition, with the direction rotation of a sector), and
 * two radial ghost layers per wall holding equilibria of linearly
 * extrapolated density and temperature (Sec. II.C, radial boundary
 * condition).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Distribution arrays are structure-of-arrays f[q][i][j] with
 *    q = 0..4 n_i (q = 0 rest; q = 1 + n_i(k-1) + d for speed group k = 1..4
 *    and direction d = 0..n_i-1 at angle 2 pi d / n_i; the octagon: q = 0..32,
 *    angle d*pi/4), i = 0..n_r-1 radial (r_i = R1 + i*dr,
 *    dr = (R2-R1)/(n_r-1)), j = 0..n_theta-1 azimuthal (theta_j =
 *    (j+1)*dtheta, dtheta = 2 pi n_f / (n_i n_theta)), j fastest.  Element
 *    type: float when the context was created with precision 32, double
 *    with precision 64.
 *  - Field arrays (rho, u_r, u_theta, T and their cotangents) are double
 *    [n_r][n_theta].  Velocities are polar components at each node.
 *    T is the temperature, equal to the internal energy E since gamma = 2
 *    (Sec. II.A).
 *  - All pointers passed to entry points that launch kernels are DEVICE
 *    pointers of the context's device and stay owned by the caller.  Work is
 *    enqueued on the stream given to pclb_bind and is asynchronous unless the
 *    entry point says it synchronizes.
 *  - Every entry point returns PCLB_OK (0) or a negative PCLB_E* code; no C++
 *    exception crosses the ABI.  pclb_last_error() describes the last failure.
 */
#ifndef PCLB_H
#define PCLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pclb_ctx pclb_ctx;

enum {
  PCLB_OK = 0,
  PCLB_EINVAL = -1,      /* bad argument or configuration */
  PCLB_ECFL = -2,        /* a Courant number exceeds 1 (outside the monotone range) */
  PCLB_EDEVICE = -3,     /* HIP runtime or launch failure */
  PCLB_ENOMEM = -4,      /* device allocation failed */
  PCLB_ESTATE = -5,      /* call not valid in the context's current state */
  PCLB_ENONFINITE = -6   /* non-finite distribution found by a diagnostic */
};

/* Radial boundary kinds (Sec. II.C, radial boundary condition). */
enum {
  PCLB_WALL = 0,         /* p[0] = angular velocity omega: u = (0, omega r) at the ghosts */
  PCLB_INFLOW = 1,       /* p = (rho, u_r, u_theta, T) prescribed at the ghosts */
  PCLB_EXTRAPOLATE = 2,  /* u_r, u_theta extrapolated linearly like rho and T */
  /* Flag to OR into a kind: the ghost layers take f^eq of their state plus
   * the non-equilibrium part f - f^eq of the row next to the wall, instead of
   * f^eq alone (the non-equilibrium boundary condition Sec. II.C cites).
   * pclb_adjoint_step refuses contexts that use it. */
  PCLB_BC_NONEQ = 16
};

/* Kernel selection for pclb_step / pclb_step_into.  Both kernels give the
 * same result bit for bit.  The strip kernel runs float states of the full
 * annulus (n_f = 8) with an upwind scheme (MWB, Warming-Beam, second-order
 * upwind) and n_theta >= 64 whose planes it can address with 32-bit offsets;
 * its strips of 64 columns that straddle an octant boundary theta = m pi/4
 * (none when n_theta is a multiple of 512) run in a second launch of a
 * variant that selects upwind sides per lane.  Its double form runs double
 * states of the full annulus with any scheme and n_theta a multiple of 64.
 * Everything else (sectors, float Lax-Wendroff, other grids) runs on the
 * node kernel, whatever is asked.  The
 * double and triple octagon have kernels of their own: a strip form for the
 * double octagon and for float states of the triple octagon on the full
 * annulus with the MWB scheme and n_theta a multiple of 64 (chosen as above),
 * and a per-node form (one thread per node, velocities in a loop) for
 * everything else; both give the same result bit for bit. */
enum {
  PCLB_KERNEL_AUTO = 0,    /* the strip kernel when the grid allows it and gives it at least
                              512 workgroups (64-column strips times chunks of 8 rows), else
                              the node kernel */
  PCLB_KERNEL_NODE = 1,    /* one thread per node, neighbours read from global memory */
  PCLB_KERNEL_STRIP = 2    /* r-marching 64-column theta strips with a register ring */
};

/* Convection scheme (pclb_config.scheme): the paper's MWB scheme and the three
 * it is compared with (Sec. II.B; Sec. III.A, Figs. 5 and 6).  All run on
 * the strip kernels except Lax-Wendroff for float octagon states, whose
 * stencil reaches downwind beyond what that kernel's ring holds (it runs on
 * the node kernel); only MWB has an adjoint. */
enum {
  PCLB_SCHEME_MWB = 0,     /* Eq. MWB Scheme with S(eta) = (|eta| - 1) / (|eta| + 1) */
  PCLB_SCHEME_WB = 1,      /* Warming-Beam, Eq. WB_Scheme_1 */
  PCLB_SCHEME_LW = 2,      /* Lax-Wendroff: Eq. Taylor expansion with central differences */
  PCLB_SCHEME_UPWIND2 = 3  /* second-order upwind, Eq. upwind scheme_1, Euler in time */
};

/* Relaxation over a step (pclb_config.relaxation), Sec. II.B. */
enum {
  PCLB_RELAX_ANALYTIC = 0, /* Eq. operator1_new: f^eq + (f - f^eq) exp(-dt/tau) */
  PCLB_RELAX_EULER = 1     /* Eq. operator1_old: f - dt/tau (f - f^eq) */
};

/* Workgroup order of the strip kernel (pclb_config.strip_order). */
enum {
  PCLB_ORDER_DEFAULT = 0,
  PCLB_ORDER_XCD = 1,      /* each accelerator die runs a contiguous range of strips */
  PCLB_ORDER_PLAIN = 2     /* workgroup index order */
};

typedef struct pclb_config {
  int32_t n_r;           /* radial nodes, >= 4 */
  int32_t n_theta;       /* azimuthal nodes, >= 8 */
  double r1, r2;         /* annulus radii, 0 < r1 < r2 */
  double tau;            /* relaxation time (Eq. FDLBM), > 0 */
  double dt;             /* time step, > 0 */
  int32_t n_i;           /* directions per speed group (Eq. DVM1, Table I): 8
                            (octagon, 33 velocities), 16 (double octagon, 65) or
                            24 (triple octagon, 97).  Non-equilibrium moments and
                            the adjoint cover n_i = 8 only */
  int32_t n_f;           /* N_f of Sec. II.C, 1..n_i: theta covers 0 < theta <= 2 pi n_f / n_i,
                            dtheta = 2 pi n_f / (n_i n_theta), and for n_f < n_i the
                            azimuthal ghosts rotate the direction index by n_f
                            (Fig. 3); n_f = n_i is the full annulus */
  int32_t precision;     /* 32: float storage and convection; 64: double throughout */
  int32_t fp64_collision;/* 1: moments, equilibrium and relaxation in double for
                            either precision.  The only accepted value: float
                            collision of a float state drifts from the double
                            trajectory by 1e-4 relative within 100 steps (the
                            speed-2.92 and speed-2.99 weights nearly cancel) and
                            saves no time on this GPU, whose double vector rate
                            equals its non-packed float rate */
  int32_t kernel;        /* PCLB_KERNEL_* */
  /* Launch shape of the strip kernel; 0 selects the default.  None of these
   * changes any result. */
  int32_t strip_chunk;   /* rows marched by one workgroup, 1..64 */
  int32_t strip_order;   /* PCLB_ORDER_* */
  double adjoint_tie;    /* relative size below which an upwind difference
                            counts as zero in pclb_adjoint_step; 0 selects the
                            default of the precision (1e-13 for 64, 1e-6 for
                            32); must be >= 0 and < 1e-2 */
  int32_t scheme;        /* PCLB_SCHEME_*; 0 is the paper's combined scheme */
  int32_t relaxation;    /* PCLB_RELAX_* */
} pclb_config;

/* Courant-number time step: dt = cfl * min(dr, r1*dtheta) / 4.49, 4.49 being
 * the largest speed of the velocity set (Sec. II.A).  Returns a negative
 * value if cfg describes no valid grid. */
double pclb_cfl_dt(const pclb_config* cfg, double cfl);

/* Validate cfg and create a context on the current HIP device.  Checks
 * r1 > 0, r2 > r1, n_r >= 4, n_theta >= 8, tau > 0, dt > 0, n_i in {8, 16, 24},
 * n_f in 1..n_i,
 * precision in {32, 64}, fp64_collision = 1, the launch-shape fields,
 * adjoint_tie, scheme and relaxation in range (PCLB_EINVAL), and
 * max |C_r|, |C_theta| <= 1 (the
 * monotone range of Sec. II.B, Eqs. varphi_0-varphi2e) -> PCLB_ECFL.  Allocates the
 * context's small device tables and scratch (ghost layers, reduction
 * partials).  *out is owned by the caller until pclb_destroy.  Both radial
 * boundaries start as WALL with omega = 0. */
int pclb_create(const pclb_config* cfg, pclb_ctx** out);

/* Free the context's device tables and scratch.  NULL is accepted. */
void pclb_destroy(pclb_ctx* ctx);

/* Text of the last failure on ctx (or of the last failed pclb_create when ctx
 * is NULL).  Static lifetime until the next call on the same context. */
const char* pclb_last_error(const pclb_ctx* ctx);

/* Bind two caller-owned device buffers of (1 + 4 n_i)*n_r*n_theta elements
 * each (33, 65 or 97 planes; the ping-pong pair) and the HIP stream (a
 * hipStream_t, NULL = default stream) on which every later call enqueues its
 * work.  Buffer 0 becomes current. */
int pclb_bind(pclb_ctx* ctx, void* f0, void* f1, void* stream);

/* Set the radial boundary of side 0 (inner, r = R1) or 1 (outer, r = R2):
 * kind is PCLB_WALL, PCLB_INFLOW or PCLB_EXTRAPOLATE, optionally ORed with
 * PCLB_BC_NONEQ; p as listed with the kinds (ignored for EXTRAPOLATE).
 * PCLB_EINVAL for an unknown side or kind, a missing or non-finite p, or an
 * inflow density or temperature <= 0.  Host-side only; takes effect from
 * the next launch. */
int pclb_set_bc(pclb_ctx* ctx, int32_t side, int32_t kind, const double p[4]);

/* f = f^eq(rho, u, T) on every node of the current buffer (Eq. feq with the
 * weights of Eqs. F_k), from device field arrays; resets the step counter.
 * Synchronizes the stream and returns PCLB_EINVAL if any rho <= 0, T <= 0 or
 * non-finite input was found. */
int pclb_init_state(pclb_ctx* ctx, const double* rho, const double* u_r,
                    const double* u_theta, const double* T);

/* Advance n >= 0 steps of Eq. combined_scheme on the bound buffers: per step
 * one radial-ghost launch and one fused step launch, then the buffers swap.
 * Asynchronous. */
int pclb_step(pclb_ctx* ctx, int64_t n);

/* pclb_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same steps, bit for bit, with the radial ghost layers held in a static
 * scratch array of the library (16 MiB per GPU, reserved while the library is
 * loaded) instead of the context's buffer.  Calls no allocating routine.
 * Returns PCLB_EINVAL if the ghost layers (4 * (1 + 4 n_i) * n_theta elements
 * of the state type) exceed the array: for the octagon n_theta > 31775 at
 * precision 32 or n_theta > 15887 at precision 64 (65 and 97 velocities:
 * 16131 and 10810 at precision 32, half that at 64).  Every call on one GPU, from any context,
 * uses that GPU's one array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must not be issued. */
int pclb_step_static(pclb_ctx* ctx, int64_t n);

/* pclb_step as one HIP graph launch (for small grids, whose steps are
 * dominated by launch overhead): the first call captures the n steps'
 * kernel launches from the current buffer into a graph on a stream of the
 * context and instantiates it; later calls with the same n, the same current
 * buffer and no pclb_set_bc or pclb_bind in between replay it; anything else
 * captures again.  The same steps as pclb_step, bit for bit.  PCLB_EINVAL for
 * n outside 0..100000; PCLB_EDEVICE if capture, instantiation or launch
 * fails.  Asynchronous on the bound stream. */
int pclb_step_graph(pclb_ctx* ctx, int64_t n);

/* One step from an arbitrary caller buffer f_in to f_out (both device
 * buffers of the context's element type and size; they must not overlap).
 * Used by checkpoint-recompute.  Does not touch the bound buffers or the step
 * counter. */
int pclb_step_into(pclb_ctx* ctx, const void* f_in, void* f_out);

/* Which bound buffer (0 or 1) holds the current state. */
int pclb_current(const pclb_ctx* ctx, int32_t* which);

/* Number of steps taken since pclb_init_state (or since binding). */
int pclb_step_count(const pclb_ctx* ctx, int64_t* steps);

/* Macroscopic fields of the current state (Eqs. moment1-moment3): any of the
 * four device field pointers may be NULL.  If diag8 (device, 8 doubles) is not
 * NULL it receives {mass, P_x, P_y, total energy, min rho, min T,
 * non-finite node count, step count}, the integrals taken with r dr dtheta,
 * the trapezoidal rule in r and the rectangle rule in theta, accumulated in
 * double with compensated (TwoSum) partial sums and a fixed-order second
 * pass (bitwise reproducible).  Asynchronous. */
int pclb_moments(pclb_ctx* ctx, double* rho, double* u_r, double* u_theta, double* T,
                 double* diag8);

/* Same diagnostics for an arbitrary state buffer f. */
int pclb_moments_of(pclb_ctx* ctx, const void* f, double* rho, double* u_r, double* u_theta,
                    double* T, double* diag8);

/* Synchronizing variant: diagnostics of the current state copied to the host
 * array diag8_host.  Returns PCLB_ENONFINITE if any node is non-finite. */
int pclb_moments_host(pclb_ctx* ctx, double* diag8_host);

/* Non-equilibrium fields of Sec. IV (Eqs. M_relative, M_absolute, D_relative,
 * D_absolute), the mask bits of pclb_noneq. */
enum {
  PCLB_NONEQ_M = 1,       /* moments M_m = sum f v...v */
  PCLB_NONEQ_MSTAR = 2,   /* central moments M*_m = sum f (v-u)...(v-u) */
  PCLB_NONEQ_DELTA = 4,   /* Delta_m = M_m(f - f^eq) */
  PCLB_NONEQ_DSTAR = 8,   /* Delta*_m = M*_m(f - f^eq) */
  PCLB_NONEQ_ALL = 15
};

/* The non-equilibrium fields of f (the current state if f is NULL) for
 * m in {2, 3, (3,1), (4,2)} with M_{3,1} = sum (1/2) f |v|^2 v and
 * M_{4,2} = sum (1/2) f |v|^2 v v, u the node's flow velocity and f^eq the
 * discrete equilibrium of the node's rho, u, E (summed from the 33 values,
 * not from closed forms).  out is a device array of doubles
 * [n_kinds][12][n_r][n_theta]: the kinds selected by `kinds` in the order
 * M, M*, Delta, Delta*, and per kind the 12 components in the node's polar
 * basis (e_r, e_theta): M_2 rr, r theta, theta theta; M_3 rrr, rr theta,
 * r theta theta, theta theta theta; M_{3,1} r, theta; M_{4,2} rr, r theta,
 * theta theta.  Computed in double.  Asynchronous.  PCLB_EINVAL for an empty
 * or unknown mask or a null out. */
int pclb_noneq(pclb_ctx* ctx, const void* f, int32_t kinds, double* out);

/* One step of the discrete adjoint of Eq. combined_scheme (not in the paper):
 * lam_out = (d Phi / d f at f_t)^T lam_next, where Phi is the step of
 * pclb_step including the dependence of the radial ghost layers on the two
 * real rows next to each wall.  The MWB switch is differentiated piecewise:
 * an upwind difference within adjoint_tie times the stencil's magnitude
 * (|f| summed over its three nodes) counts as zero, sgn(0) = 0, and where
 * both upwind differences vanish the derivatives of
 * (delta - delta')|delta|/(|delta|+|delta'|) with respect to (delta, delta')
 * are (1, 0).  All three buffers hold the context's element type and do
 * not overlap.  Asynchronous.  Float states of the full annulus with
 * n_theta a multiple of 64 take a strip form of the adjoint where the
 * context's kernel choice would take the strip kernel for pclb_step
 * (PCLB_KERNEL_STRIP, or PCLB_KERNEL_AUTO on a large enough grid; default
 * chunk 64 rows); it rounds the products of derivatives and cotangents to
 * float before summing them, so its result may differ from the node
 * kernel's by an ulp or two of float. */
int pclb_adjoint_step(pclb_ctx* ctx, const void* f_t, const void* lam_next, void* lam_out);

/* Adjoint of pclb_init_state: from lam0 = dJ/df at f = f^eq(fields), write
 * dJ/d(rho, u_r, u_theta, T) (device double fields; outputs overwritten). */
int pclb_adjoint_init(pclb_ctx* ctx, const void* lam0, const double* rho, const double* u_r,
                      const double* u_theta, const double* T, double* d_rho, double* d_u_r,
                      double* d_u_theta, double* d_T);

#ifdef __cplusplus
}
#endif

#endif /* PCLB_H */
