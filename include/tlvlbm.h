/*
 * tlvlbm.h -- C ABI of the MI355X (gfx950) implementation of the
 * total-Lagrangian vectorial lattice Boltzmann method for finite-strain
 * hyperelasticity with curved boundaries (J. Feng, X. Chu).
 *
 * One context owns one lattice (D2Q4x6 or D3Q6x12) on one GPU: the
 * vector populations, the displacement history, the cut-link tables of an
 * embedded level-set geometry, and the scratch of the compatibility
 * projection.  All compute runs in HIP kernels on the context's stream.
 *
 * Common conventions
 *  - State ordering U = (v_1..v_D, F_11, F_12, .., F_DD), F row-major
 *    (Sec. 2.2, Eq. 11); M = D + D^2 components.
 *  - Lattice directions q = 0..2D-1 ordered (+e1, -e1, +e2, -e2, +e3, -e3);
 *    the opposite direction is q ^ 1 (Sec. 2.3, Eq. 20).
 *  - Grid nodes sit at origin + (i + 1/2) dx; the linear node index is
 *    x + nx*(y + ny*z).  Field arrays crossing the ABI are planar,
 *    [component][node] over ALL grid nodes, in double precision; values at
 *    inactive nodes are ignored on input and written as 0 on output.
 *  - Pointers: every array argument may be host memory or device memory
 *    (detected with hipPointerGetAttributes).  Inputs are borrowed for the
 *    duration of the call; the library copies what it keeps.  Outputs are
 *    caller-owned; calls that write outputs return after the data is in
 *    place (they synchronise the context stream).
 *  - Errors: status codes only; nothing throws across the ABI.  Device
 *    failures detected during stepping (J <= 0, non-finite state, Newton
 *    failure) are sticky: every later call returns the same code until
 *    tlvlbm_set_state or tlvlbm_put_state.  tlvlbm_last_error() gives text.
 *  - Call order: create -> [set_levelset] -> [set_boundary]* -> set_state ->
 *    step / moments / get_state.  Out-of-order calls return
 *    TLVLBM_ERR_CALL_ORDER.
 */
#ifndef TLVLBM_H
#define TLVLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tlvlbm_ctx tlvlbm_ctx;

typedef enum {
  TLVLBM_OK = 0,
  TLVLBM_ERR_INVALID_ARG = 1,
  TLVLBM_ERR_OUT_OF_MEMORY = 2,
  TLVLBM_ERR_DEVICE = 3,
  TLVLBM_ERR_NONPOSITIVE_J = 4, /* admissibility J = det F > 0 violated (Sec. 2.1, Eq. 3) */
  TLVLBM_ERR_NEWTON = 5,        /* Neumann normal-image solve failed (Sec. 3.4) */
  TLVLBM_ERR_NONFINITE = 6,
  TLVLBM_ERR_CALL_ORDER = 7
} tlvlbm_status;

typedef enum { TLVLBM_D2Q4x6 = 2, TLVLBM_D3Q6x12 = 3 } tlvlbm_lattice;
typedef enum { TLVLBM_FP32 = 0, TLVLBM_FP64 = 1 } tlvlbm_precision;
typedef enum { TLVLBM_BC_DIRICHLET_VELOCITY = 1, TLVLBM_BC_NEUMANN_TRACTION = 2 } tlvlbm_bc_type;
typedef enum {
  TLVLBM_RAMP_CONST = 0,   /* s(t) = 1 */
  TLVLBM_RAMP_SIN2 = 1,    /* s(t) = sin^2(pi t / (2 T_r)) for t < T_r, else 1 (Sec. 4.3, Eq. 71) */
  TLVLBM_RAMP_HALFCOS = 2, /* s(t) = (1 - cos(pi t / T_r)) / 2 for t < T_r, else 1 (Sec. 5.3, Eq. 88) */
  TLVLBM_RAMP_LINEAR = 3   /* s(t) = t / T_r for t < T_r, else 1 */
} tlvlbm_ramp;

/* Cartesian grid.  Nodes at origin + (i + 1/2) dx.  Bit A of periodic_mask
 * makes axis A periodic.  A non-periodic axis needs a level set whose outer
 * node layers are inactive (every lattice neighbour of an active node must
 * exist). */
typedef struct {
  int32_t n[3];
  double dx;
  double origin[3];
  uint32_t periodic_mask;
} tlvlbm_grid;

/* Material law; P = dW/dF (Sec. 2.1, Eq. 4).
 * law 0: compressible neo-Hookean (Sec. 4.1, Eq. 62),
 *   W = mu/2 (|F|^2 - D) - (mu + lambda/2) ln J + lambda/4 (J^2 - 1).
 * law 1: the same solid reinforced by one family of fibres along the unit
 *   reference direction a0 (an anisotropic law as the outlook of Sec. 6
 *   names): W += k1/2 (|F a0|^2 - 1)^2, k1 >= 0; a0 is normalised.
 * law 2: law 1 (k1 = 0: law 0) with one viscoelastic Maxwell branch, the
 *   history-dependent extension that Sec. 6 names as a local node update:
 *   an overstress Q in the second Piola stress, P = P_eq(F) + F Q, relaxing
 *   as dQ/dt + Q / tau = beta dS_0/dt with S_0 = mu (I - C^{-1}),
 *   C = F^T F, advanced once per step by the midpoint rule on its
 *   convolution, Q^{n+1} = xi^2 Q^n + beta xi (S_0^{n+1} - S_0^n),
 *   xi = exp(-dt / (2 tau)).  beta >= 0; tau >= 0 (0: no overstress;
 *   INFINITY: the glassy limit, a neo-Hookean solid of shear modulus
 *   mu (1 + beta) from an undeformed start).  Every active node keeps the
 *   branch's history (D(D+1)/2 FP64 values), started relaxed at F0 by
 *   tlvlbm_set_state.
 * k1 and a0 are read for laws 1 and 2, beta and tau for law 2 only. */
typedef struct {
  int32_t law;
  double mu, lambda;
  double k1;
  double a0[3];
  double beta, tau;
} tlvlbm_material;

/* Run options (tlvlbm_default_options fills the paper's settings of
 * Sec. 4.1: omega = 1.8, gamma = 0, theta_F = 1, projection every 20 steps,
 * projection relaxed by 20 damped Jacobi sweeps of weight 2/3). */
typedef struct {
  double omega;       /* BGK relaxation, 0 < omega <= 2 (Sec. 2.4, Eq. 29) */
  double gamma;       /* velocity damping source B = (-gamma v, 0) (Sec. 4.1) */
  double theta_F;     /* repair weight, 0 < theta_F <= 1 (Sec. 3.5, Eq. 60) */
  double cg_rtol;     /* projection CG stop: ||r|| <= rtol max(||b||, ||r0||) (CG vectors are
                         FP64 in both builds); <= 0: 1e-14 (FP64 build), 1e-8 (FP32 build) */
  int32_t proj_every; /* projection cadence in steps when Neumann links exist; 0 disables */
  int32_t cg_maxit;   /* projection CG iteration cap; <= 0: 20 sqrt(active nodes) + 100 */
  int32_t precision;  /* tlvlbm_precision of the populations and bulk arithmetic */
  int32_t track_u;    /* 1: carry the displacement quadrature (Eq. 34); 0: not; -1: auto
                         (on whenever a level set is set) */
  void *stream;       /* hipStream_t for all work; NULL = default stream */
  int32_t cg_multigrid; /* exact mode: 1: CG preconditioned by one geometric multigrid V-cycle per
                           iteration (aggregation of 2^D blocks, damped Jacobi); 0: plain CG */
  int32_t proj_sweeps;  /* projection solver (Sec. 3.5).  > 0: that many damped Jacobi sweeps
                           x <- x + proj_weight (b - K x) / diag(K) on the normal equations,
                           started from the current displacement (the paper's relaxation; default
                           20); 0: exact minimiser (CG to cg_rtol) */
  double proj_weight;   /* Jacobi damping weight, 0 < proj_weight <= 1 (default 2/3) */
  /* Device memory of the context.  When dev_alloc is set, every device buffer
   * the context keeps (populations, displacement history, cut-link tables,
   * projection and multigrid workspace, reverse-mode arena) comes from
   * dev_alloc(bytes, alloc_user) and goes back through dev_free(ptr,
   * alloc_user) -- for example a framework's caching allocator; dev_alloc
   * returns NULL when it cannot allocate (TLVLBM_ERR_OUT_OF_MEMORY) and must
   * return memory usable on `stream`.  dev_free is required with dev_alloc.
   * The library calls them from the thread that makes the API call; memory
   * is released only after the context's stream is synchronised.  NULL
   * (default): hipMalloc / hipFree.  Call-scoped staging of host arrays and
   * the batch's tile lists always use hipMalloc. */
  void *(*dev_alloc)(size_t bytes, void *alloc_user);
  void (*dev_free)(void *ptr, void *alloc_user);
  void *alloc_user;
} tlvlbm_options;

/* Boundary condition attached to a boundary identifier (Sec. 3.1).
 * Value at boundary point X_b and time t:
 *   s(t) * ( a + G (X_b - X0) + p_radial e_R + p_normal N_b ),
 * e_R = (X_b - X0)/|X_b - X0|, N_b the outward unit normal (Eq. 38),
 * G row-major 3x3 (the leading D x D block is used).
 * DIRICHLET_VELOCITY imposes v_D at t^n + dt/2 (Sec. 3.3, Eqs. 44-45); with
 * given_as_displacement the value is u_D and v_D = d u_D/dt (Sec. 2.1, Eq. 9),
 * plus the ramped rotation of `twist` below.
 * NEUMANN_TRACTION imposes the nominal traction P N = T at t^n + dt/2
 * (Sec. 3.4, Eqs. 46-56). */
typedef struct {
  int32_t type;  /* tlvlbm_bc_type */
  int32_t ramp;  /* tlvlbm_ramp */
  double T_r;
  int32_t given_as_displacement;
  double a[3];
  double G[9];
  double p_radial;
  double p_normal;
  double X0[3];
  double twist;  /* displacement-given Dirichlet only: adds the rigid rotation
                    (R(s(t) twist) - I)(X_b - X0) in the (e1, e2) plane, angle
                    twist (radians) about the e3 axis through X0 (the tube of
                    Sec. 5.3, Eq. 87); v_D is its time derivative */
} tlvlbm_bc;

typedef struct {
  int64_t active_nodes;
  int64_t cut_links;
  int64_t dirichlet_links;
  int64_t neumann_links;
  int64_t cg_iterations;   /* cumulative */
  int64_t newton_failures; /* cumulative */
  int64_t projections;     /* cumulative */
  int64_t step;            /* time level n of the stored state */
  int64_t lsq_linear_fallbacks;
} tlvlbm_stats_t;

/* Fill options with the defaults listed above. */
void tlvlbm_default_options(tlvlbm_options *opt);

/* Create a context.  lattice selects D; rho0 > 0 divides the stress flux
 * (Phi_A^{v_i} = -P_iA / rho0, Sec. 2.2, Eq. 13 with the density restored);
 * dt > 0 sets the lattice speed c = dx / dt (Sec. 2.3).  opt may be NULL
 * (defaults).  On success *out owns all device memory of the context. */
tlvlbm_status tlvlbm_create(const tlvlbm_grid *grid, tlvlbm_lattice lattice, const tlvlbm_material *mat,
                            double rho0, double dt, const tlvlbm_options *opt, tlvlbm_ctx **out);
tlvlbm_status tlvlbm_destroy(tlvlbm_ctx *ctx);

/* Embed a body by node samples of a level set, phi <= 0 inside (Sec. 3.1,
 * Eq. 36).  phi[N] (double), bid[N] (uint8, may be NULL = 0) boundary
 * identifiers, read at the outside node of each cut link.  Builds, on the GPU:
 * the active mask, the compacted cut-link table (prefix scan over sign changes,
 * ordered by (bid, node, q)), cut fractions by FP64 bisection of the cubic
 * along-link interpolant of phi (Eq. 37), normals from central-difference
 * gradients of phi interpolated to X_b (Eq. 38), and the static weighted
 * least-squares tangent-derivative weights of every link (Eqs. 49-52).
 * Returns INVALID_ARG if an active node lacks a lattice neighbour. */
tlvlbm_status tlvlbm_set_levelset(tlvlbm_ctx *ctx, const double *phi, const uint8_t *bid);

/* Attach a boundary condition to identifier bid (copied). */
tlvlbm_status tlvlbm_set_boundary(tlvlbm_ctx *ctx, uint8_t bid, const tlvlbm_bc *bc);

/* Body acceleration b(X, t) = s(t) g(X) (Sec. 2.1, Eq. 5).  It enters the
 * source B = (b - gamma v, 0) of the first-order system (Eq. 12): in the
 * state recovery (Eq. 28) and the collision (Eqs. 29-30) of step n with
 * t = t^n, and in the second-order initialisation through B0 (Eqs. 32-33)
 * when set before tlvlbm_set_state.
 *   g     [D][N] FP64 planar, host or device (copied; NULL removes the field)
 *   ramp  tlvlbm_ramp kind of s(t), T_r its time (> 0 unless CONST)
 * A new field takes effect at the next step; a caller that needs a general
 * b(X, t) sets it before each step(1).  Contexts with a body acceleration
 * have no reverse mode (TLVLBM_ERR_INVALID_ARG). */
tlvlbm_status tlvlbm_set_body_force(tlvlbm_ctx *ctx, const double *g, int32_t ramp, double T_r);

/* Thermal stretch th(X) per node, the thermal distortion through which the
 * outlook introduces thermoelasticity (Sec. 6): the temperature field,
 * advanced by the caller, enters as the isotropic stretch of the split
 * F = F_e (th I) with the energy th^D W(F_e) per reference volume, so the
 * law (neo-Hookean, or with fibres) at node X becomes
 *   P(F) = th^(D-1) P_W(F / th)
 * in the bulk update, the traction closure's Newton solve, the
 * initialisation and the stress output.
 *   th  [N] FP64, host or device (copied; every value > 0 and finite, else
 *       TLVLBM_ERR_INVALID_ARG); NULL removes the field
 * A new field takes effect at the next step (a caller that advances the
 * temperature sets it between steps); set before tlvlbm_set_state it enters
 * the initialisation, whose second-order terms take th as locally uniform.
 * Not with a Maxwell branch (law 2), and no reverse mode
 * (TLVLBM_ERR_INVALID_ARG). */
tlvlbm_status tlvlbm_set_thermal_stretch(tlvlbm_ctx *ctx, const double *th);

/* Replace the material (e.g. for finite-difference sweeps).  The stored
 * populations are kept.  When the old or the new material has a Maxwell
 * branch (law 2), the branch's history starts anew: tlvlbm_step returns
 * CALL_ORDER until the next tlvlbm_set_state (or tlvlbm_put_history and
 * tlvlbm_put_state). */
tlvlbm_status tlvlbm_set_material(tlvlbm_ctx *ctx, const tlvlbm_material *mat);

/* Initial state (Sec. 2.1, Eq. 6).  U0[M][N]; u0[D][N] or NULL (zero);
 * dU0[D][M][N] = d U0 / d X_A or NULL (zero gradients).  Populations are
 * initialised to second order, f_q = feq(U0) - dt/2 (d_t + c e_qA d_A)
 * feq(U0) with d_t U0 = B0 - Phi'_A(U0) d_A U0 (Sec. 2.4, Eqs. 32-33), and
 * the history so that u^0 = u0 (Eq. 34).  Resets the step counter to 0 and
 * clears sticky errors.  Returns NONPOSITIVE_J if det F0 <= 0 at an active
 * node. */
tlvlbm_status tlvlbm_set_state(tlvlbm_ctx *ctx, const double *U0, const double *u0, const double *dU0);

/* Advance n time steps of Algorithm 1 (Sec. 3.6): state recovery (Eq. 28),
 * compatibility projection and population repair when Neumann links exist
 * and step % proj_every == 0 (Sec. 3.5, Eqs. 57-61), local BGK collision
 * with source (Eqs. 29-30), displacement quadrature (Eq. 34), streaming
 * (Eq. 31) and cut-link reconstruction (Eqs. 41-56).  Returns after one
 * status read at the end of the n steps; device failures are reported as
 * NONPOSITIVE_J / NONFINITE / NEWTON. */
tlvlbm_status tlvlbm_step(tlvlbm_ctx *ctx, int64_t n);

/* Recovered state of the current time level: U_out[M][N] (Eq. 28),
 * u_out[D][N] displacement (Eq. 34; zero when not tracked), J_out[N]
 * (det F).  Any output may be NULL. */
tlvlbm_status tlvlbm_moments(tlvlbm_ctx *ctx, double *U_out, double *u_out, double *J_out);

/* The same moments in the context's precision: U_out[M][N] and J_out[N] as
 * float for a TLVLBM_FP32 context (double for TLVLBM_FP64), the values
 * tlvlbm_moments returns rounded once to that precision; u_out[D][N] stays
 * FP64 (the displacement history is FP64 in both builds).  Host or device;
 * any output may be NULL. */
tlvlbm_status tlvlbm_moments_native(tlvlbm_ctx *ctx, void *U_out, double *u_out, void *J_out);

/* Stress of the current time level (the final diagnostics of Algorithm 1):
 * first Piola P_out[D*D][N] of the recovered F with the material law (with
 * a Maxwell branch: its history as the next collision uses it; with a
 * thermal stretch: the node's stretch) and Cauchy
 * stress sigma_out[D*D][N] = J^{-1} P F^T (Sec. 2.4, Eq. 35), row-major
 * components, FP64, host or device; zero at inactive nodes.  Either may be
 * NULL. */
tlvlbm_status tlvlbm_stress(tlvlbm_ctx *ctx, double *P_out, double *sigma_out);

/* Raw state for checkpoint/resume: pre-collision populations f^n as
 * [2D][M][N] and the displacement history u*^n as [D][N] (either may be
 * NULL), plus the step index.  The history of a Maxwell branch is not part
 * of it (tlvlbm_get_history / tlvlbm_put_history): tlvlbm_put_state keeps
 * the branch's history as it is, and on a law-2 context that has none yet
 * (no set_state, no put_history) returns CALL_ORDER. */
tlvlbm_status tlvlbm_get_state(tlvlbm_ctx *ctx, double *f, double *ustar, int64_t *step);
tlvlbm_status tlvlbm_put_state(tlvlbm_ctx *ctx, const double *f, const double *ustar, int64_t step);

/* The Maxwell branch's history (law 2) for checkpoint/resume: per node
 * R = xi^2 Q^n - beta xi S_0^n (the overstress Q and the shear stress S_0 of
 * the last committed step, xi = exp(-dt/(2 tau))), D(D+1)/2 packed symmetric
 * components (2D: 00, 01, 11; 3D: 00, 01, 02, 11, 12, 22) as [D(D+1)/2][N]
 * FP64, host or device; values at inactive nodes are not used.  A history
 * is meaningful only with the beta, tau, mu and dt it was taken with.
 * INVALID_ARG without a branch; get: CALL_ORDER before set_state or
 * put_history. */
tlvlbm_status tlvlbm_get_history(tlvlbm_ctx *ctx, double *R);
tlvlbm_status tlvlbm_put_history(tlvlbm_ctx *ctx, const double *R);

/* Cut-link table (host or device outputs, length = stats.cut_links): node,
 * outgoing direction q, cut fraction eta, normal N_b [L][3], boundary id.
 * Any output may be NULL. */
tlvlbm_status tlvlbm_get_links(tlvlbm_ctx *ctx, int64_t *node, int32_t *q, double *eta, double *Nb,
                               int32_t *bid);

tlvlbm_status tlvlbm_stats(tlvlbm_ctx *ctx, tlvlbm_stats_t *out);

/* Block until all work of the context's stream is done. */
tlvlbm_status tlvlbm_synchronize(tlvlbm_ctx *ctx);

/* Text of the last error on this context (never NULL). */
const char *tlvlbm_last_error(const tlvlbm_ctx *ctx);

/* ---- Reverse mode (project extension, not in the paper) ------------------
 * Gradient of a linear functional of the moments after n steps,
 *   L = sum_i sum_r dLdU[r][i] U_r(i) + sum_i sum_k dLdu[k][i] u_k(i)
 * (U, u exactly as tlvlbm_moments returns them), with respect to the
 * material parameters and the initial data, by the discrete adjoint of the
 * step (collision, streaming, cut-link closures including the Neumann
 * Newton solve, the compatibility projection and the second-order
 * initialisation; Secs. 2.4, 3.2-3.5).
 *  - Precondition: the state is the one set by tlvlbm_set_state (no step
 *    since).  The call advances the context n steps, as tlvlbm_step does,
 *    and leaves it there.
 *  - U0, dU0: the arrays given to tlvlbm_set_state ([M][nodes],
 *    [D][M][nodes] or NULL); the initialisation's transpose needs them.
 *  - dLdU [M][nodes], dLdu [D][nodes]: FP64, host or device, either may be
 *    NULL (dLdu requires the displacement quadrature).
 *  - grad_mat[2] (host): dL/dmu, dL/dlambda.  grad_v0, grad_u0 [D][nodes]
 *    FP64 host or device, or NULL: dL/dv0 (the velocity rows of U0) and
 *    dL/du0; F0 and dU0 are held fixed.
 *  - segment: the schedule.  > 0: a checkpoint of the stored field (Q M + D
 *    node planes) every `segment` steps; each segment is recomputed once
 *    with its tape.  0: the last steps keep their tape from the first pass
 *    (as many as 60% of the free device memory holds: all of them for
 *    short runs), and only the steps before them are checkpointed and
 *    recomputed, in segments of about sqrt(steps x checkpoint / tape step).
 *    < 0: as 0 with at most -segment taped final steps.  Tape per step:
 *    D x D planes of F - I over the 32-node chunks that hold active nodes
 *    (population precision), F^r likewise on projection steps, and u at the
 *    Neumann stencil nodes (FP64).  TLVLBM_ERR_OUT_OF_MEMORY if checkpoints
 *    and tape do not fit.  When a quarter of the remaining memory holds
 *    them, the projection solutions of the checkpointed steps are kept
 *    (FP64, active tiles) and replayed by the recomputation.  This memory
 *    stays with the context (reused by the next call with the same n and
 *    segment) until tlvlbm_destroy or a call of another shape.  Every
 *    schedule gives bit-identical results.  Work: one forward pass, one
 *    recomputation of the checkpointed steps without projection solves, one
 *    reverse pass (the transposed projection sweeps on projection steps).
 *  - Errors: the forward's errors; TLVLBM_ERR_CALL_ORDER without a fresh
 *    state; TLVLBM_ERR_INVALID_ARG with a body acceleration or a Maxwell
 *    branch (law 2).  A failure leaves the context in an error state. */
tlvlbm_status tlvlbm_adjoint_step(tlvlbm_ctx *ctx, int64_t n, const double *U0, const double *dU0,
                                  const double *dLdU, const double *dLdu, double *grad_mat, double *grad_v0,
                                  double *grad_u0, int64_t segment);

/* The same reverse mode in two calls, for losses that depend on the final
 * state (their dLdU, dLdu are known only after the forward run) and for
 * several gradients of one run:
 *
 * tlvlbm_adjoint_record: the first pass of tlvlbm_adjoint_step alone.  From
 * the state of tlvlbm_set_state (no step since), advance n steps as
 * tlvlbm_step does, keeping checkpoints and the tape of the final steps
 * (schedule `segment` as above), and device copies of U0 and dU0 (the arrays
 * given to tlvlbm_set_state: [M][nodes], [D][M][nodes] or NULL).  The
 * context ends at step n; tlvlbm_moments reads the final state.
 *
 * tlvlbm_adjoint_backward: the reverse pass of the recorded run for
 * L = sum dLdU . U + dLdu . u over the final moments (as above; either may
 * be NULL): grad_mat[2] (host) = dL/d(mu, lambda); grad_v0, grad_u0
 * [D][nodes] as above; grad_dU0 [D][M][nodes] = dL/d dU0, the gradient with
 * respect to the initial gradient data of the second-order initialisation
 * (Sec. 2.4, Eqs. 32-33; U0 held fixed).  A caller whose dU0 is a function
 * of v0 (for instance a difference operator applied to it) obtains the total
 * velocity gradient as grad_v0 + (that operator)^T grad_dU0.  Any output may
 * be NULL; outputs are host or device FP64.  Segments are recomputed from
 * their checkpoints; the context returns to the end of the run, and the
 * record stays valid: the call may be repeated with other dLdU, dLdu.
 * TLVLBM_ERR_CALL_ORDER without a record, or when the context changed after
 * it (a step, a new state, material, boundary condition, level set or body
 * force).  Every call gives the same result bit for bit as
 * tlvlbm_adjoint_step on the same inputs. */
tlvlbm_status tlvlbm_adjoint_record(tlvlbm_ctx *ctx, int64_t n, const double *U0, const double *dU0,
                                    int64_t segment);
tlvlbm_status tlvlbm_adjoint_backward(tlvlbm_ctx *ctx, const double *dLdU, const double *dLdu, double *grad_mat,
                                      double *grad_v0, double *grad_u0, double *grad_dU0);

/* ---- Many instances (project extension, not in the paper) ---------------
 * Independent contexts of the same lattice and precision, sharing one
 * non-default stream, at the same step, each with a level set and state.
 *
 * tlvlbm_step_each advances every context n steps with per-instance
 * launches of the single-instance kernels (the reference for the batched
 * path).
 *
 * tlvlbm_batch_create builds tile lists over all instances; tlvlbm_batch_step
 * then runs every phase of Algorithm 1 as ONE launch over all instances
 * (bulk update, cut links, every projection/CG kernel with per-instance
 * scalars and segmented reductions) and replays captured hipGraphs: with
 * the Jacobi projection (proj_sweeps > 0) a whole projection cycle
 * (projection step and the proj_every - 1 steps after it) from one graph;
 * with the exact projection, whose CG polls its convergence from the host,
 * the steps between projections.  The batch borrows the contexts:
 * they must outlive it, and single-instance calls on them while the batch is
 * in use are not allowed (the batch keeps its own copy of their buffer
 * roles).  Results equal the per-instance path up to floating-point
 * summation order.  Errors of any instance are reported (and made sticky on
 * that context).  The projection phases run over every instance, so either
 * all instances have Neumann links or none has (TLVLBM_ERR_INVALID_ARG for a
 * mixed set: the projection belongs to lattices with Neumann links only).
 * The batched bulk update runs every law (0, 1, 2), the thermal stretch and
 * the body acceleration, each instance with its own material, history,
 * field and ramp: the whole batch takes the most general update one of its
 * instances needs (reinforced for fibres or a body acceleration, whose
 * extra terms vanish where an instance has none; the branch's update, with
 * no overstress where an instance has no branch; the stretched update, with
 * th = 1 where there is no field).  A batch holding both a Maxwell branch
 * and a thermal stretch is refused (TLVLBM_ERR_INVALID_ARG; no update
 * covers both; tlvlbm_step_each takes them). */
typedef struct tlvlbm_batch tlvlbm_batch;
tlvlbm_status tlvlbm_step_each(tlvlbm_ctx *const *ctxs, int32_t n, int64_t steps);
tlvlbm_status tlvlbm_batch_create(tlvlbm_ctx *const *ctxs, int32_t n, tlvlbm_batch **out);
tlvlbm_status tlvlbm_batch_step(tlvlbm_batch *b, int64_t steps);
/* 0 disables graph replay (every launch issued from the host) */
tlvlbm_status tlvlbm_batch_set_graph(tlvlbm_batch *b, int32_t use_graph);
/* Tile configuration of the batched node kernels (bulk update, moments):
 * spans of tile_width nodes (64, 128 or 256; one workgroup each) of an
 * instance's node order, aligned to tile_width, that hold active nodes, in
 * order 0 (instance by instance) or 1 (round robin over the instances).  tlvlbm_batch_create picks the configuration
 * by timing the bulk kernel over each of the six on the batch's own state
 * (3 timed launches each; u* and u are saved and restored, no step is
 * taken); tlvlbm_batch_autotune repeats that with `reps` timed launches;
 * tlvlbm_batch_set_tiles forces one.  Results do not depend on the
 * configuration (the per-node arithmetic is the same).
 * tlvlbm_batch_get_tiles: the configuration in use and, in ms[6] (may be
 * NULL), the mean time per launch of each candidate, index order * 3 +
 * (0, 1, 2 for widths 64, 128, 256).  Errors: TLVLBM_ERR_INVALID_ARG for
 * other widths or orders; device errors as for tlvlbm_batch_step. */
tlvlbm_status tlvlbm_batch_autotune(tlvlbm_batch *b, int32_t reps);
tlvlbm_status tlvlbm_batch_set_tiles(tlvlbm_batch *b, int32_t tile_width, int32_t order);
tlvlbm_status tlvlbm_batch_get_tiles(const tlvlbm_batch *b, int32_t *tile_width, int32_t *order, double *ms);
tlvlbm_status tlvlbm_batch_destroy(tlvlbm_batch *b);
const char *tlvlbm_batch_last_error(const tlvlbm_batch *b);

/* ---- Without device allocation ------------------------------------------
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the cut-link table
 * that tlvlbm_set_levelset builds and tlvlbm_get_links returns, computed
 * straight from a level set with no allocation at all.
 *  - grid, lattice: as for tlvlbm_create; phi [N] FP64 and bid [N] uint8
 *    (NULL: identifier 0) node samples as for tlvlbm_set_levelset, in device
 *    memory.
 *  - Outputs (device memory, caller-owned, `capacity` records each): node
 *    [cap] int64, q [cap] int32 (required); eta [cap] FP64, Nb [cap][3] FP64,
 *    bid_out [cap] int32 (each may be NULL).  Same records, same order
 *    (bid, node, q) and the same values bit for bit as tlvlbm_get_links after
 *    tlvlbm_set_levelset.  *n_links (host) receives the number of cut links.
 *  - stream: hipStream_t of the work (NULL: default); returns after the
 *    results are in place (synchronises the stream).
 *  - Workspace: one fixed device array of the library (about 66 KiB, held by
 *    every GPU the library runs on until the process ends), which limits
 *    the grid to TLVLBM_NOALLOC_MAX_NODES nodes.  Calls that overlap on one
 *    GPU (several host threads or streams) race on it.
 *  - Errors: TLVLBM_ERR_INVALID_ARG for a larger grid, host-memory arrays, a
 *    missing required pointer, an active node without a lattice neighbour,
 *    or more links than `capacity` (then *n_links holds the count needed and
 *    no record is written); TLVLBM_ERR_DEVICE for a device failure. */
#define TLVLBM_NOALLOC_MAX_NODES (8192LL * 2048LL)
tlvlbm_status tlvlbm_cut_links_noalloc(const tlvlbm_grid *grid, tlvlbm_lattice lattice, const double *phi,
                                       const uint8_t *bid, int64_t capacity, int64_t *node, int32_t *q, double *eta,
                                       double *Nb, int32_t *bid_out, int64_t *n_links, void *stream);

/* Size in bytes of one population buffer (for bandwidth accounting). */
size_t tlvlbm_population_bytes(const tlvlbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
