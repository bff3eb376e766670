/*
 * lbmwb.h -- C ABI of the MI355X (gfx950) library for the well-balanced
 * phase-field lattice Boltzmann step of Ju, Liu, Yan, Bao, Sun and Guo,
 * "A well-balanced lattice Boltzmann model for binary fluids based on the
 * incompressible phase-field theory" (arXiv 2311.10827).
 *
 * One time step updates two D2Q9 populations on a 2-D grid:
 *   - the order-parameter population, the paper's f_i (Sec. 2.3.1, eq. BGK),
 *     whose equilibrium carries no velocity; convection u.grad(phi) enters as
 *     a source term F_i plus half its time derivative (eqs. H_i, F_i);
 *   - the pressure/velocity population, the paper's g_i (Sec. 2.3.2,
 *     eq. BGK-NS), driven by the potential-form force F = -phi grad(mu) + G.
 * Names in this header follow the paper: "f" is always the order-parameter
 * population and "g" the hydrodynamic one.
 *
 * Conventions
 *   - Lattice units, delta_x = delta_t = 1, c_s^2 = 1/3.
 *   - Velocity order: 0 rest; 1 (+1,0); 2 (0,+1); 3 (-1,0); 4 (0,-1);
 *     5 (+1,+1); 6 (-1,+1); 7 (-1,-1); 8 (+1,-1).
 *   - Fields are row-major [ny][nx], x fastest; cell (i, j) is at x = i, y = j.
 *   - Phase A is the paper's "l" phase (phi_A), phase B its "v" phase.
 *
 * Memory and streams
 *   - The library never allocates or frees device memory.  The caller
 *     allocates the state (lbm_state_bytes) and workspace
 *     (lbm_workspace_bytes) buffers on the device, keeps them alive for the
 *     context's lifetime and owns them; the context only borrows them.
 *   - Every call is ordered on the HIP stream given to lbm_init and does not
 *     block the host, except where a function says it synchronises.
 *   - A context is not thread-safe.  Pointer arguments marked "device" must
 *     be device memory of the GPU current at lbm_init.
 *
 * Errors: every int-returning function returns LBM_OK (0) or a negative code;
 * lbm_strerror() names it and lbm_last_error() gives the context's detail
 * text.  No C++ exception crosses this interface.
 */
#ifndef LBMWB_H
#define LBMWB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)     /* bad argument: size, relaxation time <= 1/2, rho <= 0, ... */
#define LBM_EHIP (-2)       /* a HIP runtime call or kernel launch failed */
#define LBM_ENONFINITE (-3) /* diagnostics saw NaN/Inf or a non-positive density */
#define LBM_ESTATE (-4)     /* call made in the wrong state */

enum { LBM_PERIODIC = 0, LBM_WALL = 1 };

/* Viscosity across the interface (lbm_params.nu_form). */
enum { LBM_NU_LINEAR = 0, LBM_NU_INVERSE = 1, LBM_NU_EXP = 2 };

/* Collision operator (lbm_params.collision). */
enum { LBM_BGK = 0, LBM_MRT = 1 };

/* Storage of the FP32 rest population's low word (lbm_params.lo_format). */
enum { LBM_LO_AUTO = 0, LBM_LO_16 = 1, LBM_LO_32 = 2 };

/*
 * Problem parameters, in the paper's notation.
 *   phi_A, phi_B   order parameter of the two bulk phases (Sec. 2.1, eq. bulk_energy).
 *   rho_A, rho_B   densities; rho is linear in phi between them (Sec. 2.3.2,
 *                  sentence before eq. vis).
 *   nu_A, nu_B     kinematic viscosities; tau_g = 1/2 + nu / c_s^2 per cell
 *                  (Sec. 2.3.2), with nu(phi) chosen by nu_form.
 *   kappa, beta    gradient and double-well coefficients (eqs. energy_function,
 *                  bulk_energy).  With use_sigma_W = 1 they are derived from the
 *                  surface tension sigma and interface width W instead
 *                  (eqs. beta, suiface_tension).
 *   M, alpha       mobility and the equilibrium's free parameter;
 *                  tau_f = 1/2 + M / (c_s^2 alpha) (Sec. 2.3.1, eq. mobility).
 *   use_tau        0: the relaxation times follow from M, alpha, nu_A, nu_B as
 *                  above.  1: tau_f, tau_gA, tau_gB are given instead and
 *                  alpha = M / (c_s^2 (tau_f - 1/2)) (eq. mobility solved for
 *                  alpha) and nu_A,B = c_s^2 (tau_gA,B - 1/2) (Sec. 2.3.2)
 *                  are derived from them; the alpha, nu_A, nu_B fields are
 *                  then ignored.  Each tau must exceed 1/2.
 *   tau_f, tau_gA, tau_gB   the relaxation times, read only with use_tau = 1.
 *   gx, gy         body force G added to the interfacial force (Sec. 2.3.2).
 *   bc_x, bc_y     LBM_PERIODIC, or LBM_WALL: half-way bounce-back for both
 *                  populations, and phi, mu mirrored across the wall in the
 *                  finite-difference stencils (the paper's tests are periodic).
 *   precision      64: populations stored and updated in FP64.
 *                  32: populations stored and updated in FP32; the rest
 *                      population of f, of order one, is held as an
 *                      unevaluated pair hi + lo (hi an FP32 word, lo an
 *                      FP32 word or a 16-bit fraction of ulp(hi), about
 *                      2^-40 relative: lo_format) offset by (phi_A + phi_B) / 2, the
 *                      others are small deviations
 *                      from the rest equilibrium; diagnostics stay FP64.
 *   diag_every     0: no diagnostics inside lbm_step; k > 0: a fused FP64
 *                  diagnostic pass every k steps (see lbm_step).
 *   kernel_path    0: automatic: two steps per launch (as 3) for an FP32
 *                  state on a periodic grid that does not fit the GPU's
 *                  last-level cache; else the fused kernel when the grid
 *                  gives its launch enough workgroups (at least 512 strips
 *                  of 256 x 8 cells), else the two kernels;
 *                  1: the phi/mu pass and the collide-stream pass as two
 *                  kernels; 2: one fused kernel per step (phi and mu kept
 *                  on chip); 3: two steps per launch (the intermediate
 *                  state kept on chip, only every second state written to
 *                  memory), FP32 on grids periodic in both directions
 *                  only; a step due for diagnostics, and the last of an
 *                  odd count, runs as in 2.  All give the same results bit
 *                  for bit.
 *   nu_form        how nu varies across the interface (Sec. 2.3.2).  With the
 *                  phase-A fraction s = (phi - phi_B)/(phi_A - phi_B):
 *                  LBM_NU_LINEAR:  nu linear in phi (eq. vis, the paper's
 *                                  choice);
 *                  LBM_NU_INVERSE: 1/nu = s/nu_A + (1 - s)/nu_B;
 *                  LBM_NU_EXP:     ln nu = s ln nu_A + (1 - s) ln nu_B.
 *                  The paper names the last two as alternatives without
 *                  writing them out; s is not clamped.  1/nu vanishes at
 *                  s = -nu_A/(nu_B - nu_A) when nu_A < nu_B (and mirrored),
 *                  so the inverse form needs phi to stay that close to the
 *                  bulk values.
 *   collision      LBM_BGK: single relaxation time for both populations, as
 *                  in the paper (eqs. BGK, BGK-NS).
 *                  LBM_MRT: multiple relaxation times, the extension the paper
 *                  names (Sec. 2.3) without giving it: the non-equilibrium
 *                  part is relaxed in the orthogonal D2Q9 moment basis of
 *                  Lallemand and Luo, m = (rho, e, eps, j_x, q_x, j_y, q_y,
 *                  p_xx, p_xy).  f: phi and j at 1/tau_f (the mobility is
 *                  unchanged), e, eps, q, (p_xx, p_xy) at mrt_f[0..3]; the
 *                  source is added as in BGK.  g: j, p_xx, p_xy at
 *                  1/tau_g(phi) (the viscosity is unchanged), (rho, e, eps)
 *                  together at mrt_g[0], q at mrt_g[1]; the forcing of eq.
 *                  GGi enters as M^-1 (I - S/2) M G~.  rho, e and eps of g
 *                  share one rate because p is recovered from
 *                  sum_{i!=0} g_i = (8 rho + e - eps)/9.  Every rate must lie
 *                  in (0, 2); with all rates equal to the BGK ones the result
 *                  is the BGK step.
 *   lo_format      FP32 only (ignored for precision 64): the storage of the
 *                  low word lo of the rest population's pair hi + lo.
 *                  LBM_LO_AUTO: 16 bits for states above 1 GiB that run
 *                  one step per launch (where the step is bound by HBM
 *                  traffic), an FP32 word below and with two steps per
 *                  launch (lbm_derived.two_step);
 *                  LBM_LO_16: always the 16-bit fraction of ulp(hi);
 *                  LBM_LO_32: always an FP32 word.  The state size does not
 *                  depend on it.
 */
typedef struct lbm_params {
  int32_t nx, ny;
  int32_t bc_x, bc_y;
  int32_t precision;
  int32_t use_sigma_W;
  double phi_A, phi_B;
  double rho_A, rho_B;
  double nu_A, nu_B;
  double kappa, beta;
  double sigma, W;
  double M, alpha;
  double gx, gy;
  int32_t diag_every;
  int32_t kernel_path;
  int32_t nu_form;
  int32_t collision;
  double mrt_f[4];
  double mrt_g[2];
  int32_t lo_format;
  int32_t use_tau;
  double tau_f, tau_gA, tau_gB;
} lbm_params;

/* Derived constants (lattice units). */
typedef struct lbm_derived {
  double kappa, beta;     /* as used by the step */
  double sigma, W;        /* surface tension and width implied by kappa, beta */
  double tau_f;           /* 1/2 + M / (c_s^2 alpha), or as given (use_tau) */
  double tau_gA, tau_gB;  /* 1/2 + nu_A / c_s^2, 1/2 + nu_B / c_s^2, or as given */
  double alpha;           /* as given, or M / (c_s^2 (tau_f - 1/2)) (use_tau) */
  double nu_A, nu_B;      /* as given, or c_s^2 (tau_g - 1/2) (use_tau) */
  int32_t lo16;           /* 1 if an FP32 state keeps the low word in 16 bits */
  int32_t two_step;       /* 1 if lbm_step runs two steps per launch where it
                           * can (kernel_path 3, or 0 for an FP32 state on a
                           * grid periodic in both directions larger than the
                           * GPU's last-level cache) */
} lbm_derived;

/*
 * FP64 diagnostics of the pre-collision state at time `step`.
 * source_sum = sum_x (3/2 S(n) - 1/2 S(n-1)) with S = u.grad(phi); the next
 * step changes sum_x phi by exactly -source_sum (the zeroth moment of the
 * source, Sec. 2.3.1, eq. sumfeqandF).  Sums and extrema are reduced in a
 * fixed order, so they are bitwise reproducible.
 */
typedef struct lbm_diag {
  double sum_phi;
  double source_sum;
  double kinetic_energy;  /* 1/2 sum_x rho |u|^2 (Sec. 3.1) */
  double max_u;           /* max_x |u| */
  double min_rho, max_rho;
  double mu_min, mu_max;
  double phi_min, phi_max;
  double max_div_u;       /* max_x |d_x u_x + d_y u_y|, each derivative the
                           * isotropic gradient of Sec. 2.3.2 (eq. gradient)
                           * with the stencils' wrap or mirrored wall ghosts;
                           * the recovered equations are incompressible.
                           * Formed by lbm_moments only: -1 from
                           * lbm_last_diag */
  double laplace_dP;      /* mean of P^ = p + phi mu - psi(phi), psi the
                           * double well of Sec. 2.1 (eq. bulk_energy), over
                           * the bulk-A cells minus its mean over the bulk-B
                           * cells: the jump that equals sigma / R across a
                           * drop at mechanical equilibrium.  With the
                           * phase-A fraction s = (phi - phi_B) /
                           * (phi_A - phi_B), bulk A is s >= max(s) - 0.01
                           * and bulk B s <= min(s) + 0.01.  0 unless both
                           * sets are non-empty and disjoint.  Formed by
                           * lbm_moments only */
  int64_t n_nonfinite;    /* cells whose phi, mu, u or p is not finite */
  int64_t n_bulk_A, n_bulk_B; /* cells in the two bulk sets (0 from
                               * lbm_last_diag) */
  int64_t step;
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Validate `p` and fill `out`.  LBM_EINVAL on: nx, ny < 1; a plane of more
 * than 2^31 - 1 cells; bc not 0/1; precision not 32/64; phi_A == phi_B;
 * rho_A, rho_B <= 0; nu_A, nu_B <= 0; M <= 0; alpha <= 0; kappa or beta
 * < 0 (or sigma, W <= 0 with use_sigma_W); diag_every < 0; kernel_path not
 * 0..3, or 3 with precision 64 or a wall; nu_form not one of LBM_NU_*; collision not LBM_BGK or LBM_MRT; with
 * LBM_MRT, an MRT rate outside (0, 2); lo_format not one of LBM_LO_*;
 * use_tau not 0/1; with use_tau, a relaxation time <= 1/2 or not finite. */
int lbm_derive(const lbm_params* p, lbm_derived* out);

/* Bytes the caller must allocate for the state and the workspace (0 if `p`
 * is invalid).  The state holds two population buffers, two source planes
 * (S_prev, and S of a two-step launch) and the phi and mu planes; its layout is private to the library (256-byte aligned
 * planes).  The workspace holds reduction partials. */
size_t lbm_state_bytes(const lbm_params* p);
size_t lbm_workspace_bytes(const lbm_params* p);

/*
 * Create a context and write the initial state (time 0):
 *   f = f^eq(phi0, mu(phi0)) (Sec. 2.3.1, eq. H_i),
 *   g = g^eq(p = 0, u0) (Sec. 2.3.2, eq. G_i),
 *   previous-step source = S(0) computed from that state.
 * phi0: device, FP64 [ny][nx], required.  ux0, uy0: device, FP64 [ny][nx], or
 * NULL for zero.  state, workspace: device buffers of at least the sizes
 * above, 256-byte aligned.  stream: a hipStream_t, or NULL for the null
 * stream.  On success *out owns host-side resources until lbm_destroy.
 */
int lbm_init(lbm_ctx** out, const lbm_params* p, void* state, void* workspace,
             const double* phi0, const double* ux0, const double* uy0, void* stream);

/*
 * Advance n >= 0 time steps.  A step computes phi = sum_i f_i (Sec. 2.3.1,
 * eq. order-parameter) and mu (eq. chemical_potencial with the isotropic
 * Laplacian of Sec. 2.3.2, eq. Laplace), then collides and pull-streams both
 * populations (Sec. 2.3.1, eq. BGK; Sec. 2.3.2, eqs. BGK-NS, G_i, Siu, GGi
 * and the u, p recovery), in one kernel or two, or two steps in one kernel
 * (kernel_path).  Asynchronous.  With diag_every = k > 0 every k-th step also reduces the
 * diagnostics of its pre-collision state; a pass that found a non-finite
 * value or rho <= 0 makes a later lbm_step (or lbm_last_diag) return
 * LBM_ENONFINITE once that pass has completed on the device.
 */
int lbm_step(lbm_ctx* ctx, int64_t n);

/*
 * lbm_step for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * steps, kernels and results as lbm_step, bit for bit, but the diagnostic
 * reductions of diag_every > 0 use a scratch array the library holds on each
 * GPU for the life of the process (4 MiB, set up by lbm_init on the GPU
 * current there) instead of the context's workspace, and the call allocates
 * nothing.  Limit: a grid whose diagnostic partials, first-level reduction
 * and result exceed 4 MiB (8 + 1024 + 1 blocks of 11 doubles per strip of
 * the fused step, or per 64 x 4 tile of the two-kernel step: e.g. 16384^2
 * fused is 3.0 MB, 4096^2 two-kernel 5.9 MB) gets LBM_EINVAL with the sizes
 * in lbm_last_error, and no step is taken.  LBM_ESTATE while step timing
 * (lbm_timing) is on, since it records new events.  LBM_EHIP if lbm_init
 * could not set the scratch up.  All contexts on one GPU share its scratch:
 * calls that overlap (different streams, or threads) race on it; calls on
 * one stream are ordered.  Otherwise as lbm_step.
 */
int lbm_step_noalloc(lbm_ctx* ctx, int64_t n);

/* Number of steps taken since lbm_init (or the step given to lbm_set_state). */
int64_t lbm_step_count(const lbm_ctx* ctx);

/*
 * Moments of the current pre-collision state: phi = sum_i f_i (Sec. 2.3.1,
 * eq. order-parameter); mu (Sec. 2.1, eq. chemical_potencial, with the
 * isotropic Laplacian of Sec. 2.3.2, eq. Laplace); u from
 * rho u = sum_i c_i g_i + F/2 and p from the non-rest g, u.grad(rho)/2 and
 * rho s_0(u) (Sec. 2.3.2, the macroscopic subequations, with
 * F = -phi grad(mu) + G and the isotropic gradients of eq. gradient); rho
 * linear in phi (Sec. 2.3.2, before eq. vis).
 * Each output is device FP64 [ny][nx] or NULL.  If diag is not NULL it
 * receives the diagnostics (host struct), max_div_u and laplace_dP
 * included; that makes the call synchronise the stream.  With diag, the
 * fields among phi, mu, ux, uy, p that are NULL are staged in the state's
 * idle population buffer (the one the next step overwrites), so no memory
 * beyond the state is needed.  Does not advance time.
 */
int lbm_moments(lbm_ctx* ctx, double* phi, double* mu, double* ux, double* uy, double* p,
                double* rho, lbm_diag* diag);

/* Diagnostics of the latest fused diagnostic pass of lbm_step (host
 * struct).  Synchronises the stream.  LBM_ESTATE if no pass ran yet;
 * LBM_ENONFINITE if that pass saw a non-finite value or rho <= 0 (the struct
 * is still filled). */
int lbm_last_diag(lbm_ctx* ctx, lbm_diag* diag);

/*
 * Copy the pre-collision populations and the previous-step source of the
 * periodic window [x0, x0 + w) x [y0, y0 + h) (coordinates taken modulo
 * nx, ny) into device FP64 arrays f [9][h][w], g [9][h][w], Sp [h][w]; any
 * may be NULL.  Requires 1 <= w <= nx, 1 <= h <= ny.
 */
int lbm_get_state(lbm_ctx* ctx, int32_t x0, int32_t y0, int32_t w, int32_t h, double* f,
                  double* g, double* Sp);

/* Replace the whole state by pre-collision populations f, g [9][ny][nx]
 * and previous-step source Sp [ny][nx] (device FP64), and set the step
 * counter to `step`. */
int lbm_set_state(lbm_ctx* ctx, const double* f, const double* g, const double* Sp,
                  int64_t step);

/* Step timing with HIP events recorded around each step's kernels on the
 * context's stream.  lbm_timing(ctx, 1) starts recording (clearing earlier
 * records), 0 stops.  lbm_kernel_times synchronises and returns the summed
 * milliseconds of the timed steps and their number. */
int lbm_timing(lbm_ctx* ctx, int enable);
int lbm_kernel_times(lbm_ctx* ctx, double* ms_step, int64_t* steps);

/* Bandwidth probe: copy `bytes` (a multiple of 16) from src to dst on
 * `stream` with a plain streaming kernel (device pointers, 16-byte aligned,
 * non-overlapping). */
int lbm_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Checkpoints.  A snapshot holds the raw state (one population buffer and
 * the previous-step source plane, in the storage precision) plus two scratch
 * planes for that state's phi and mu: restoring it reproduces the following
 * steps bit for bit.  dst/src: device buffers of lbm_snapshot_bytes(ctx)
 * bytes, 256-byte aligned.  lbm_restore also sets the step counter.
 * ---------------------------------------------------------------------- */
#define LBM_SNAPSHOT_HAS_PHI_MU 1
size_t lbm_snapshot_bytes(const lbm_ctx* ctx);
int lbm_snapshot(lbm_ctx* ctx, void* dst);
int lbm_restore(lbm_ctx* ctx, const void* src, int64_t step);
/* One step from snapshot src into snapshot dst (distinct buffers), without
 * touching the context's own state or step counter.  The state in dst equals
 * what lbm_step followed by lbm_snapshot gives, bit for bit; src's phi and mu
 * planes are left holding the phi and mu of src (LBM_SNAPSHOT_HAS_PHI_MU).
 * Lets a caller recompute a segment of states without copies. */
int lbm_step_into(lbm_ctx* ctx, void* src, void* dst);

/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of the step.  The paper defines the forward step
 * only (Sec. 2.3); these functions give the exact transpose of its Jacobian.
 *
 * The state at time n is s_n = (f, g, S_prev): pre-collision populations and
 * the previous-step source.  An adjoint lambda has the same layout as
 * lbm_get_state's outputs packed together: 19 dense planes [ny][nx]
 * (f_0..f_8, g_0..g_8, S_prev) in the storage precision (double for
 * precision 64, float for 32), device memory.  The arithmetic is in the
 * storage precision, like the forward step's; parameter gradients
 * accumulate in FP64.  The adjoint follows the step the context was made
 * for: either viscosity law (nu_form) and either collision (for MRT the
 * moment-space relaxation M^-1 S M is symmetric, so its transpose is the
 * same operator).
 *
 * Parameter gradients accumulate in the adjoint workspace for
 * theta = (kappa, beta, alpha, tau_f, nu_A, nu_B), each taken as independent;
 * lbm_adjoint_theta returns them in that basis or in the basis
 * (kappa, beta, M, tau_f, tau_gA, tau_gB) of the mobility and the
 * relaxation times.  The MRT rates mrt_f, mrt_g are constants, not
 * differentiated.
 * ---------------------------------------------------------------------- */

/* Bytes of the adjoint workspace (7 planes plus parameter partials). */
size_t lbm_adjoint_workspace_bytes(const lbm_params* p);
/* Attach a device workspace (256-byte aligned) and zero the parameter
 * gradient.  Required before the other adjoint calls (else LBM_ESTATE). */
int lbm_adjoint_attach(lbm_ctx* ctx, void* adj_workspace);
/* state: a snapshot of s_n (lbm_snapshot / lbm_step_into).  Map
 * lam_in = dL/ds_{n+1} to lam_out = dL/ds_n and add dL/dtheta of this step.
 * lam_in and lam_out must not overlap.  flags: LBM_SNAPSHOT_HAS_PHI_MU if the
 * snapshot's phi/mu planes are valid (it was the source of lbm_step_into),
 * else 0 and they are recomputed into it. */
int lbm_adjoint_step(lbm_ctx* ctx, void* state, const void* lam_in, void* lam_out, int flags);
/* One checkpoint segment of the backward pass: snaps[0] holds s_k; the
 * other L - 1 snapshots receive s_{k+1}..s_{k+L-1} (lbm_step_into), then the
 * L adjoint steps run in reverse from lam = dL/ds_{k+L}, ping-ponging with
 * tmp.  *which = 0 if dL/ds_k ends in lam, 1 if in tmp.  snaps: host array of
 * L distinct device snapshot pointers. */
int lbm_adjoint_segment(lbm_ctx* ctx, void* const* snaps, int L, void* lam, void* tmp,
                        int* which);
/* state: a snapshot of s_0 made by lbm_init from phi0 with no initial
 * velocity (else LBM_ESTATE).  Map lam0 = dL/ds_0 to dphi0 = dL/dphi0
 * (device FP64 [ny][nx]) and add dL/dtheta of the initialisation.
 * scratch: a device buffer of the adjoint's size, distinct from lam0. */
int lbm_adjoint_init(lbm_ctx* ctx, const void* state, const double* phi0, const void* lam0,
                     void* scratch, double* dphi0);
/* Copy the accumulated parameter gradient to out[6] (host; synchronises)
 * and, if reset != 0, zero it.  basis LBM_THETA_NATIVE:
 * dL/d(kappa, beta, alpha, tau_f, nu_A, nu_B) with the six independent.
 * basis LBM_THETA_TAU: dL/d(kappa, beta, M, tau_f, tau_gA, tau_gB) with those
 * six independent, by the chain rule through alpha = M / (c_s^2 (tau_f - 1/2))
 * (Sec. 2.3.1, eq. mobility) and nu = c_s^2 (tau_g - 1/2) (Sec. 2.3.2), at
 * the context's parameters.  LBM_EINVAL for another basis. */
enum { LBM_THETA_NATIVE = 0, LBM_THETA_TAU = 1 };
int lbm_adjoint_theta(lbm_ctx* ctx, int basis, double* out, int reset);

/* Release the context's host resources (not the caller's buffers). */
int lbm_destroy(lbm_ctx* ctx);

const char* lbm_strerror(int code);
/* Detail text of the context's most recent failure ("" if none). */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBMWB_H */
