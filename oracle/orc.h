/*
 * FP64 CPU oracle for the total-Lagrangian vectorial lattice Boltzmann method
 * (Feng & Chu, "Total-Lagrangian vectorial lattice Boltzmann method for
 * finite-strain hyperelasticity with curved boundaries").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header or constant with the GPU library.
 *
 * Conventions (all arrays are caller-owned, host memory, double precision):
 *   D      spatial dimension (2 or 3); Q = 2D lattice directions; M = D + D*D.
 *   state  U = (v_1..v_D, F_11, F_12, .., F_DD), F row-major (Sec. 2.2, Eq. 11).
 *   dirs   q = 0..Q-1 ordered (+e1, -e1, +e2, -e2, +e3, -e3); opp(q) = q ^ 1.
 *   nodes  X_i = origin + (i + 1/2) dx, linear index x + nx*(y + ny*z).
 *   planar field arrays are [component][node] over ALL grid nodes.
 *
 * Parity notes: functions whose result has no independent pin are marked
 * "parity unpinned" in orc.c; every other function is pinned by tests that
 * do not re-type its formula.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes (same numeric meaning as the product library, defined here
 * independently) */
enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_MEM = 2, ORC_ERR_J = 4,
       ORC_ERR_NEWTON = 5, ORC_ERR_NONFINITE = 6, ORC_ERR_ORDER = 7 };

enum { ORC_BC_NONE = 0, ORC_BC_DIRICHLET = 1, ORC_BC_NEUMANN = 2 };
enum { ORC_RAMP_CONST = 0, ORC_RAMP_SIN2 = 1, ORC_RAMP_HALFCOS = 2,
       ORC_RAMP_LINEAR = 3 };

/* ---- point maps (Sec. 2.1, Eq. 4; Sec. 4.1, Eq. 62) ---------------------- */
int  orc_piola(int D, double mu, double lam, const double *F, double *P);
int  orc_piola_jvp(int D, double mu, double lam, const double *F,
                   const double *dF, double *dP);
/* the same maps for the fibre-reinforced law W += k1/2 (|F a0|^2 - 1)^2
 * (a0 used as given: pass a unit vector) */
int  orc_piola_law(int D, double mu, double lam, double k1, const double *a0, const double *F, double *P);
int  orc_piola_law_jvp(int D, double mu, double lam, double k1, const double *a0, const double *F,
                       const double *dF, double *dP);
int  orc_cauchy(int D, double mu, double lam, const double *F, double *sigma);
double orc_energy(int D, double mu, double lam, const double *F);
/* fluxes Phi[A][M] (Eq. 13) and equilibria feq[q][M] (Eq. 24) */
void orc_flux(int D, double mu, double lam, double rho0, const double *U,
              double *Phi);
void orc_feq(int D, double c, double mu, double lam, double rho0,
             const double *U, double *feq);
void orc_feq_jvp(int D, double c, double mu, double lam, double rho0,
                 const double *U, const double *Z, double *dfeq);

/* ---- cut-link local solves (Sec. 3.4) ------------------------------------ */
/* weighted LSQ tangent-derivative weights (Eqs. 49-52).  xi[npts][D] are
 * normalised offsets (X_m - X_b)/dx, tang[(D-1)][D] unit tangents.  Writes
 * w[(D-1)][npts].  Returns 2 (quadratic basis), 1 (linear fallback) or 0. */
int orc_lsq_weights(int D, int npts, const double *xi, const double *tang,
                    double dx, double *w);
/* Newton solve of R(h) = P(h (x) N + G_t) N - T = 0 (Eqs. 53-56).
 * Gt = sum_alpha g_alpha (x) t_alpha (DxD row-major).  Returns 1 on
 * convergence, 0 on failure; h holds the last admissible iterate. */
int orc_newton(int D, double mu, double lam, const double *N, const double *Gt,
               const double *T, const double *h0, double tol, double *h,
               int *iters);

/* ---- the simulation ------------------------------------------------------ */
typedef struct orc_sim orc_sim;

orc_sim *orc_create(int D, const int *n, double dx, const double *origin,
                    int periodic_mask, double mu, double lam, double rho0,
                    double dt, double omega, double gamma, double theta_F,
                    int proj_every);
void orc_destroy(orc_sim *s);
/* Compatibility projection solver (Sec. 3.5).  sweeps > 0: that many damped
 * Jacobi sweeps of weight `weight` on the normal equations, started from the
 * current displacement (the default, ORC_PROJ_SWEEPS sweeps of weight
 * ORC_PROJ_WEIGHT); sweeps = 0: the exact minimiser (CG to stagnation). */
#define ORC_PROJ_SWEEPS 20
#define ORC_PROJ_WEIGHT (2.0 / 3.0)
int  orc_set_projection(orc_sim *s, int sweeps, double weight);
/* body acceleration b(X, t) = s(t) g(X) (Sec. 2.1, Eq. 5), entering
 * B = (b - gamma v, 0) in the recovery, the collision and the initialisation
 * (Eqs. 28-33); g [D][N] planar (copied) or NULL to clear; s(t) a ramp of
 * kind `ramp` and time T_r, evaluated at t^n for step n. */
int  orc_set_body_force(orc_sim *s, const double *g, int ramp, double T_r);
/* fibre reinforcement W += k1/2 (|F a0|^2 - 1)^2 along the reference
 * direction a0 (normalised; k1 = 0 restores the neo-Hookean law) */
int  orc_set_fibres(orc_sim *s, double k1, const double *a0);
/* one viscoelastic (Maxwell) branch on top of the law (the history-dependent
 * extension of Sec. 6): P = P_eq(F) + F Q, dQ/dt + Q/tau = beta dS_0/dt,
 * S_0 = mu (I - C^{-1}); per-node history started relaxed at orc_set_state
 * (call before it).  beta >= 0; tau >= 0 (0: no overstress, INFINITY: the
 * glassy limit).  No reverse mode with a branch (ORC_ERR_ARG). */
int  orc_set_viscous(orc_sim *s, double beta, double tau);
/* thermal stretch th [N] (copied; every value > 0; NULL removes it): the
 * law at node i becomes P(F) = th_i^(D-1) P_W(F / th_i), the thermal
 * distortion F = F_e (th I) of thermoelasticity (Sec. 6), the temperature
 * field advanced by the caller.  Takes effect at the next step, and in the
 * initialisation when set before orc_set_state (whose second-order terms
 * take th as locally uniform).  Not with a Maxwell branch and no reverse
 * mode (ORC_ERR_ARG). */
int  orc_set_thermal(orc_sim *s, const double *th);
int  orc_thermal_piola(int D, double mu, double lam, double k1, const double *a0, double th,
                       const double *F, double *P);
int  orc_thermal_piola_jvp(int D, double mu, double lam, double k1, const double *a0, double th,
                           const double *F, const double *dF, double *dP);
/* the branch's history (Q^n, S_0^n) of every node, planar [D*D][N] each */
int  orc_get_viscous(orc_sim *s, double *Qh, double *S0h);
/* point maps of the branch with a given history, and a material point driven
 * along F[0..n] [n+1][D*D] one step dt apart (P [n+1][D*D]) */
int  orc_visco_piola(int D, double mu, double lam, double beta, double xi,
                     const double *Qh, const double *S0h, const double *F, double *P);
int  orc_visco_piola_jvp(int D, double mu, double lam, double beta, double xi,
                         const double *Qh, const double *S0h, const double *F,
                         const double *dF, double *dP);
int  orc_visco_path(int D, double mu, double lam, double beta, double tau, double dt,
                    int64_t n, const double *F, double *P);
/* phi[N] node samples (phi <= 0 inside, Eq. 36); bid[N] boundary ids. */
int  orc_set_levelset(orc_sim *s, const double *phi, const uint8_t *bid);
/* boundary value s(t) (a + G (X - X0) + p_radial e_R + p_normal N_b) */
int  orc_set_bc(orc_sim *s, int bid, int type, int ramp, double T_r,
                int given_as_displacement, const double *a, const double *G,
                double p_radial, double p_normal, const double *X0);
/* displacement-given Dirichlet only: add the ramped rigid rotation
 * (R(s(t) twist) - I)(X - X0) in the (e1, e2) plane (Sec. 5.3, Eq. 87) */
int  orc_set_bc_twist(orc_sim *s, int bid, double twist);
/* boundary data of identifier bid at X (normal Nb), time t: val = imposed
 * velocity or traction, disp (may be NULL) = prescribed displacement */
int  orc_bc_data(orc_sim *s, int bid, const double *X, const double *Nb, double t, double *val, double *disp);
/* U0[M][N]; u0[D][N] or NULL; dU0[D][M][N] (d/dX_A of U0) or NULL */
int  orc_set_state(orc_sim *s, const double *U0, const double *u0,
                   const double *dU0);
int  orc_step(orc_sim *s, int64_t nsteps);
/* U[M][N] (recovered, Eq. 28), u[D][N] (Eq. 34), J[N]; any may be NULL */
int  orc_moments(orc_sim *s, double *U, double *u, double *J);
/* first Piola P[D*D][N] (with each node's law and history) and Cauchy
 * stress sigma[D*D][N] = J^{-1} P F^T (Eq. 35) of the current state; either
 * may be NULL */
int  orc_stress(orc_sim *s, double *P, double *sigma);
/* pre-collision populations f^n as [Q][M][N] */
int  orc_get_f(orc_sim *s, double *f);
int  orc_put_f(orc_sim *s, const double *f, const double *ustar, int64_t step);
/* post-collision populations f* of the last completed step, [Q][M][N] */
int  orc_get_fs(orc_sim *s, double *f);
int64_t orc_num_active(orc_sim *s);
int64_t orc_num_links(orc_sim *s);
/* link records in (bid, node, q) order: node[L], q[L], eta[L], Nb[L][3],
 * bid[L]; any pointer may be NULL */
int  orc_get_links(orc_sim *s, int64_t *node, int32_t *q, double *eta,
                   double *Nb, int32_t *bid);
/* stats[0]=newton iterations, [1]=newton failures, [2]=cg iterations,
 *      [3]=projections, [4]=step, [5]=status */
void orc_stats(orc_sim *s, int64_t *stats);
/* projection-only entry for pins: given F[D*D][N] (planar) and a warm start
 * u[D][N], solve the edge least-squares problem of Eq. 57 in place. */
int  orc_project(orc_sim *s, const double *F, double *u, double rtol,
                 int64_t *iters);
/* the projection with the Dirichlet cut-link anchors evaluated at time t */
int  orc_project_anchored(orc_sim *s, const double *F, double *u, double t, double rtol, int64_t *iters);
/* Reverse mode (project extension; the paper has no adjoint).  From the state
 * set by orc_set_state, advance nsteps steps (as orc_step does) and return
 * the gradient of L = sum_m dLdU(m).U(m) + dLdu(m).u(m) over the moments
 * after the last step: grad_mat[2] = dL/d(mu, lambda), grad_v0[D][N] =
 * dL/dv0 and grad_u0[D][N] = dL/du0 for the v0 (velocity rows of U0) and u0
 * of orc_set_state (F0 and dU0 held fixed), and grad_dU0[D][M][N] = dL/d dU0,
 * the gradient with respect to the spatial-gradient data of the
 * initialisation (Eqs. 32-33; U0 held fixed).  dLdU[M][N], dLdu[D][N] and
 * any output may be NULL.  ORC_ERR_ORDER unless the state is the one set by
 * orc_set_state. */
int  orc_adjoint(orc_sim *s, int64_t nsteps, const double *dLdU,
                 const double *dLdu, double *grad_mat, double *grad_v0,
                 double *grad_u0, double *grad_dU0);
/* OpenMP threads used by the oracle */
int  orc_num_threads(void);
/* compatible gradient of Eq. 59 (planar in/out) */
int  orc_compatible_F(orc_sim *s, const double *u, const double *F,
                      double *Fc);

#ifdef __cplusplus
}
#endif
#endif
