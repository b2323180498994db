/*
 * FP64 CPU oracle for the total-Lagrangian vectorial LBM (Feng & Chu).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously-correct reference that
 * the GPU path is checked against.  Only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the GPU
 * library.  Dense arrays, AoS populations f[node][q][r], plain loops, OpenMP
 * over nodes, no fusion: the update follows Algorithm 1 (Sec. 3.6) phase by
 * phase.
 *
 * Readings where the paper is silent or ambiguous are stated at the point of
 * use and listed with the design notes of the repository.
 *
 * Parity status of the functions below: every function is pinned by the
 * CPU test-suite (closed forms, printed values, invariants, brute force),
 * except the level-set cubic-interpolant bisection order details and the
 * Newton backtracking schedule, whose *results* are pinned (exact root /
 * closed-form circle intersection) but whose iteration counts are
 * "parity unpinned".
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD 3
#define MAXQ 6
#define MAXM 12
#define LSQ_RADIUS 2.5   /* stencil radius in lattice units (reading) */
#define LSQ_MAXPTS 1024

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                        */
/* ------------------------------------------------------------------------ */

/* lattice direction components: q = 2A (+e_A), 2A+1 (-e_A) (Sec. 2.3, Eq. 20) */
static int e_of(int q, int A) { return (q / 2 == A) ? ((q & 1) ? -1 : 1) : 0; }

static double det_n(int D, const double *F) {
  if (D == 2) return F[0] * F[3] - F[1] * F[2];
  return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]);
}

/* cofactor matrix, cof(F) = J F^{-T} */
static void cof_n(int D, const double *F, double *C) {
  if (D == 2) {
    C[0] = F[3]; C[1] = -F[2]; C[2] = -F[1]; C[3] = F[0];
    return;
  }
  C[0] = F[4] * F[8] - F[5] * F[7];
  C[1] = F[5] * F[6] - F[3] * F[8];
  C[2] = F[3] * F[7] - F[4] * F[6];
  C[3] = F[2] * F[7] - F[1] * F[8];
  C[4] = F[0] * F[8] - F[2] * F[6];
  C[5] = F[1] * F[6] - F[0] * F[7];
  C[6] = F[1] * F[5] - F[2] * F[4];
  C[7] = F[2] * F[3] - F[0] * F[5];
  C[8] = F[0] * F[4] - F[1] * F[3];
}

/* solve a small dense system A x = b (n <= 12) by Gaussian elimination with
 * partial pivoting; returns 0 if singular */
static int gauss_solve(int n, const double *Ain, const double *bin, double *x) {
  double A[12 * 12], b[12];
  memcpy(A, Ain, sizeof(double) * n * n);
  memcpy(b, bin, sizeof(double) * n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
    if (A[p * n + k] == 0.0) return 0;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
      }
      double t = b[k]; b[k] = b[p]; b[p] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      double l = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
      b[i] -= l * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
    x[i] = s / A[i * n + i];
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* constitutive point maps                                                    */
/* ------------------------------------------------------------------------ */

/* Compressible neo-Hookean energy (Sec. 4.1, Eq. 62). */
double orc_energy(int D, double mu, double lam, const double *F) {
  double J = det_n(D, F), f2 = 0.0;
  for (int k = 0; k < D * D; ++k) f2 += F[k] * F[k];
  return 0.5 * mu * (f2 - D) - (mu + 0.5 * lam) * log(J) + 0.25 * lam * (J * J - 1.0);
}

/* First Piola stress P = dW/dF of Eq. 62 (Sec. 2.1, Eq. 4):
 *   P = mu (F - F^{-T}) + (lam/2)(J^2 - 1) F^{-T}.
 * Returns ORC_ERR_J when J <= 0 (Eq. 3). */
int orc_piola(int D, double mu, double lam, const double *F, double *P) {
  double C[9], J = det_n(D, F);
  if (!(J > 0.0)) {
    for (int k = 0; k < D * D; ++k) P[k] = NAN;
    return ORC_ERR_J;
  }
  cof_n(D, F, C);
  for (int k = 0; k < D * D; ++k) {
    double FiT = C[k] / J;
    P[k] = mu * (F[k] - FiT) + 0.5 * lam * (J * J - 1.0) * FiT;
  }
  return ORC_OK;
}

/* Tangent action dP = C : dF (Sec. 2.1, Eq. 4), differentiated from the
 * Piola map above:
 *   dP = mu dF + (mu - lam/2 (J^2-1)) F^{-T} dF^T F^{-T}
 *        + lam J^2 tr(F^{-1} dF) F^{-T}. */
int orc_piola_jvp(int D, double mu, double lam, const double *F, const double *dF,
                  double *dP) {
  double C[9], FiT[9], J = det_n(D, F);
  if (!(J > 0.0)) return ORC_ERR_J;
  cof_n(D, F, C);
  for (int k = 0; k < D * D; ++k) FiT[k] = C[k] / J;
  double tr = 0.0; /* tr(F^{-1} dF) = sum_ij FiT_ij dF_ij */
  for (int k = 0; k < D * D; ++k) tr += FiT[k] * dF[k];
  double a = mu - 0.5 * lam * (J * J - 1.0);
  for (int i = 0; i < D; ++i)
    for (int A = 0; A < D; ++A) {
      double s = 0.0; /* (F^{-T} dF^T F^{-T})_iA = sum_jk FiT_ij dF_kj FiT_kA */
      for (int j = 0; j < D; ++j)
        for (int k = 0; k < D; ++k) s += FiT[i * D + j] * dF[k * D + j] * FiT[k * D + A];
      dP[i * D + A] = mu * dF[i * D + A] + a * s + lam * J * J * tr * FiT[i * D + A];
    }
  return ORC_OK;
}

/* Material of a simulation: the neo-Hookean solid of Eq. 62, optionally
 * reinforced by one family of fibres along the unit reference direction a0
 * (the anisotropic law the paper's outlook names, Sec. 6):
 *   W = W_NH(F) + (k1/2) (I4 - 1)^2,  I4 = |F a0|^2,
 *   P = P_NH + 2 k1 (I4 - 1) (F a0) (x) a0,
 *   dP = dP_NH + 2 k1 [2 ((F a0).(dF a0)) (F a0) (x) a0 + (I4 - 1) (dF a0) (x) a0].
 * k1 = 0 is the paper's law.
 *
 * Optionally one viscoelastic (Maxwell) branch, the history-dependent law the
 * outlook names as a local node update (Sec. 6).  The branch adds an
 * overstress Q to the second Piola stress, P = P_eq(F) + F Q, driven by the
 * shear part of the neo-Hookean second Piola stress S_0 = mu (I - C^{-1})
 * (C = F^T F) through the relaxation equation
 *   dQ/dt + Q / tau = beta dS_0/dt,
 * i.e. Q(t) = beta int exp(-(t - s)/tau) dS_0/ds ds.  The convolution over one
 * step taken by the midpoint rule gives the second-order update
 *   Q^{n+1} = xi^2 Q^n + beta xi (S_0^{n+1} - S_0^n),  xi = exp(-dt/(2 tau)).
 * At a node the map F -> P therefore depends on the history (Qh, S0h) =
 * (Q^n, S_0^n) of the last committed step:
 *   Q(F) = xi^2 Qh + beta xi (S_0(F) - S0h),   P(F) = P_eq(F) + F Q(F),
 * and its tangent at frozen history is
 *   dP = dP_eq + dF Q(F) + beta xi F dS_0,  dS_0 = mu C^{-1} dC C^{-1},
 *   dC = dF^T F + F^T dF.
 * tau -> infinity (xi = 1) from an undeformed start gives the neo-Hookean
 * solid with shear modulus mu (1 + beta); tau -> 0 (xi = 0) the equilibrium
 * law.  Qh = NULL: no branch.
 *
 * Optionally a thermal stretch th > 0 at the node, the thermal distortion
 * the outlook names for thermoelasticity (Sec. 6): the temperature field,
 * advanced by whatever solves for it, enters as the isotropic stretch
 * F_th = th I of the multiplicative split F = F_e F_th, with the energy per
 * reference volume det(F_th) W(F_e).  Then
 *   P(F) = th^(D-1) P_W(F / th),
 * P_W the stress of the law above, and its tangent is
 *   dP = th^(D-1) dP_W(F / th; dF / th).
 * th = 1: no stretch. */
typedef struct {
  double mu, lam, k1, a0[3];
  double beta, xi;
  const double *Qh, *S0h; /* D x D history of the node, or NULL */
  double th;              /* thermal stretch of the node (1: none) */
} orc_mat;

static orc_mat nh_mat(double mu, double lam) {
  orc_mat m = {mu, lam, 0.0, {0.0, 0.0, 0.0}, 0.0, 0.0, NULL, NULL, 1.0};
  return m;
}

/* S_0 = mu (I - C^{-1}), C^{-1}_AB = sum_i F^{-T}_iA F^{-T}_iB */
static void visco_S0(int D, double mu, const double *F, double *S0, double *Ci) {
  double C[9], J = det_n(D, F);
  cof_n(D, F, C);
  for (int A = 0; A < D; ++A)
    for (int B = 0; B < D; ++B) {
      double s = 0.0;
      for (int i = 0; i < D; ++i) s += C[i * D + A] * C[i * D + B];
      s /= J * J;
      if (Ci) Ci[A * D + B] = s;
      S0[A * D + B] = mu * ((A == B ? 1.0 : 0.0) - s);
    }
}

/* overstress Q(F) with the node's history */
static void visco_Q(int D, const orc_mat *m, const double *F, double *Qv, double *Ci) {
  double S0[9];
  visco_S0(D, m->mu, F, S0, Ci);
  for (int k = 0; k < D * D; ++k) Qv[k] = m->xi * m->xi * m->Qh[k] + m->beta * m->xi * (S0[k] - m->S0h[k]);
}

static int mat_piola_w(int D, const orc_mat *m, const double *F, double *P) {
  int st = orc_piola(D, m->mu, m->lam, F, P);
  if (st) return st;
  if (m->k1 != 0.0) {
    double fa[3] = {0.0, 0.0, 0.0}, I4 = 0.0;
    for (int i = 0; i < D; ++i) {
      for (int A = 0; A < D; ++A) fa[i] += F[i * D + A] * m->a0[A];
      I4 += fa[i] * fa[i];
    }
    for (int i = 0; i < D; ++i)
      for (int A = 0; A < D; ++A) P[i * D + A] += 2.0 * m->k1 * (I4 - 1.0) * fa[i] * m->a0[A];
  }
  if (m->Qh) {
    double Qv[9];
    visco_Q(D, m, F, Qv, NULL);
    for (int i = 0; i < D; ++i)
      for (int A = 0; A < D; ++A) {
        double s = 0.0;
        for (int B = 0; B < D; ++B) s += F[i * D + B] * Qv[B * D + A];
        P[i * D + A] += s;
      }
  }
  return ORC_OK;
}

static int mat_piola_jvp_w(int D, const orc_mat *m, const double *F, const double *dF, double *dP) {
  int st = orc_piola_jvp(D, m->mu, m->lam, F, dF, dP);
  if (st) return st;
  if (m->k1 != 0.0) {
    double fa[3] = {0.0, 0.0, 0.0}, dfa[3] = {0.0, 0.0, 0.0}, I4 = 0.0, dI = 0.0;
    for (int i = 0; i < D; ++i) {
      for (int A = 0; A < D; ++A) {
        fa[i] += F[i * D + A] * m->a0[A];
        dfa[i] += dF[i * D + A] * m->a0[A];
      }
      I4 += fa[i] * fa[i];
      dI += fa[i] * dfa[i];
    }
    for (int i = 0; i < D; ++i)
      for (int A = 0; A < D; ++A)
        dP[i * D + A] += 2.0 * m->k1 * (2.0 * dI * fa[i] + (I4 - 1.0) * dfa[i]) * m->a0[A];
  }
  if (m->Qh) {
    double Qv[9], Ci[9], dC[9], W[9], dS0[9];
    visco_Q(D, m, F, Qv, Ci);
    for (int A = 0; A < D; ++A)
      for (int B = 0; B < D; ++B) {
        double s = 0.0;
        for (int i = 0; i < D; ++i) s += dF[i * D + A] * F[i * D + B] + F[i * D + A] * dF[i * D + B];
        dC[A * D + B] = s;
      }
    for (int A = 0; A < D; ++A) /* W = C^{-1} dC */
      for (int B = 0; B < D; ++B) {
        double s = 0.0;
        for (int K = 0; K < D; ++K) s += Ci[A * D + K] * dC[K * D + B];
        W[A * D + B] = s;
      }
    for (int A = 0; A < D; ++A) /* dS0 = mu W C^{-1} */
      for (int B = 0; B < D; ++B) {
        double s = 0.0;
        for (int K = 0; K < D; ++K) s += W[A * D + K] * Ci[K * D + B];
        dS0[A * D + B] = m->mu * s;
      }
    for (int i = 0; i < D; ++i)
      for (int A = 0; A < D; ++A) {
        double s = 0.0;
        for (int B = 0; B < D; ++B)
          s += dF[i * D + B] * Qv[B * D + A] + m->beta * m->xi * F[i * D + B] * dS0[B * D + A];
        dP[i * D + A] += s;
      }
  }
  return ORC_OK;
}

/* the law at a node with its thermal stretch (see orc_mat) */
static int mat_piola(int D, const orc_mat *m, const double *F, double *P) {
  if (m->th == 1.0) return mat_piola_w(D, m, F, P);
  double Fe[9] = {0.0};
  for (int k = 0; k < D * D; ++k) Fe[k] = F[k] / m->th;
  int st = mat_piola_w(D, m, Fe, P);
  const double sc = pow(m->th, D - 1);
  for (int k = 0; k < D * D; ++k) P[k] *= sc;
  return st;
}

static int mat_piola_jvp(int D, const orc_mat *m, const double *F, const double *dF, double *dP) {
  if (m->th == 1.0) return mat_piola_jvp_w(D, m, F, dF, dP);
  double Fe[9] = {0.0}, dFe[9] = {0.0};
  for (int k = 0; k < D * D; ++k) {
    Fe[k] = F[k] / m->th;
    dFe[k] = dF[k] / m->th;
  }
  int st = mat_piola_jvp_w(D, m, Fe, dFe, dP);
  const double sc = pow(m->th, D - 1);
  for (int k = 0; k < D * D; ++k) dP[k] *= sc;
  return st;
}

/* advance a node's history with the deformation F the step used:
 * (Qh, S0h) <- (Q(F), S_0(F)) */
static void visco_commit(int D, const orc_mat *m, const double *F, double *Qh, double *S0h) {
  double Qv[9], S0[9];
  visco_Q(D, m, F, Qv, NULL);
  visco_S0(D, m->mu, F, S0, NULL);
  for (int k = 0; k < D * D; ++k) {
    Qh[k] = Qv[k];
    S0h[k] = S0[k];
  }
}

/* exported forms of the Maxwell-branch maps (pins) */
int orc_visco_piola(int D, double mu, double lam, double beta, double xi, const double *Qh, const double *S0h,
                    const double *F, double *P) {
  orc_mat m = {mu, lam, 0.0, {0.0, 0.0, 0.0}, beta, xi, Qh, S0h, 1.0};
  return mat_piola(D, &m, F, P);
}

int orc_visco_piola_jvp(int D, double mu, double lam, double beta, double xi, const double *Qh, const double *S0h,
                        const double *F, const double *dF, double *dP) {
  orc_mat m = {mu, lam, 0.0, {0.0, 0.0, 0.0}, beta, xi, Qh, S0h, 1.0};
  return mat_piola_jvp(D, &m, F, dF, dP);
}

/* a material point driven along F[0..n] (one step apart): history started
 * relaxed at F[0] (Q = 0, S0h = S_0(F[0])); at each step the stress of the
 * current F with the stored history, then the history advance, the order a
 * lattice node takes them in */
int orc_visco_path(int D, double mu, double lam, double beta, double tau, double dt, int64_t n, const double *F,
                   double *P) {
  double Qh[9] = {0.0}, S0h[9];
  if (!(tau >= 0.0) || !(dt > 0.0)) return ORC_ERR_ARG;
  const double xi = exp(-dt / (2.0 * tau));
  visco_S0(D, mu, F, S0h, NULL);
  orc_mat m = {mu, lam, 0.0, {0.0, 0.0, 0.0}, beta, xi, Qh, S0h, 1.0};
  for (int64_t k = 0; k <= n; ++k) {
    const double *Fk = F + (size_t)k * D * D;
    int st = mat_piola(D, &m, Fk, P + (size_t)k * D * D);
    if (st) return st;
    visco_commit(D, &m, Fk, Qh, S0h);
  }
  return ORC_OK;
}

/* exported forms of the law with a thermal stretch (pins) */
int orc_thermal_piola(int D, double mu, double lam, double k1, const double *a0, double th, const double *F,
                      double *P) {
  if (!(th > 0.0)) return ORC_ERR_ARG;
  orc_mat m = {mu, lam, k1, {a0[0], a0[1], D == 3 ? a0[2] : 0.0}, 0.0, 0.0, NULL, NULL, th};
  return mat_piola(D, &m, F, P);
}

int orc_thermal_piola_jvp(int D, double mu, double lam, double k1, const double *a0, double th, const double *F,
                          const double *dF, double *dP) {
  if (!(th > 0.0)) return ORC_ERR_ARG;
  orc_mat m = {mu, lam, k1, {a0[0], a0[1], D == 3 ? a0[2] : 0.0}, 0.0, 0.0, NULL, NULL, th};
  return mat_piola_jvp(D, &m, F, dF, dP);
}

/* exported forms of the material maps (law with fibres) */
int orc_piola_law(int D, double mu, double lam, double k1, const double *a0, const double *F, double *P) {
  orc_mat m = {mu, lam, k1, {a0[0], a0[1], D == 3 ? a0[2] : 0.0}, 0.0, 0.0, NULL, NULL, 1.0};
  return mat_piola(D, &m, F, P);
}

int orc_piola_law_jvp(int D, double mu, double lam, double k1, const double *a0, const double *F,
                      const double *dF, double *dP) {
  orc_mat m = {mu, lam, k1, {a0[0], a0[1], D == 3 ? a0[2] : 0.0}, 0.0, 0.0, NULL, NULL, 1.0};
  return mat_piola_jvp(D, &m, F, dF, dP);
}

/* Cauchy stress sigma = J^{-1} P F^T (Sec. 2.4, Eq. 35). */
int orc_cauchy(int D, double mu, double lam, const double *F, double *sigma) {
  double P[9];
  int st = orc_piola(D, mu, lam, F, P);
  if (st) return st;
  double J = det_n(D, F);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int A = 0; A < D; ++A) s += P[i * D + A] * F[j * D + A];
      sigma[i * D + j] = s / J;
    }
  return ORC_OK;
}

/* Fluxes Phi_A(U) (Sec. 2.2, Eq. 13): Phi_A^{v_i} = -P_iA / rho0,
 * Phi_A^{F_iB} = -delta_AB v_i.  Layout Phi[A*M + r]. */
static void flux_m(int D, const orc_mat *m, double rho0, const double *U, double *Phi) {
  int M = D + D * D;
  double P[9];
  mat_piola(D, m, U + D, P);
  for (int A = 0; A < D; ++A)
    for (int r = 0; r < M; ++r) {
      double val;
      if (r < D) {
        val = -P[r * D + A] / rho0;
      } else {
        int i = (r - D) / D, B = (r - D) % D;
        val = (A == B) ? -U[i] : 0.0;
      }
      Phi[A * M + r] = val;
    }
}

/* Equilibrium populations (Sec. 2.3, Eq. 24):
 * feq_q = (1/2D) [ U + (D/c) e_qA Phi_A(U) ].  Layout feq[q*M + r]. */
static void feq_m(int D, double c, const orc_mat *m, double rho0, const double *U, double *feq) {
  int M = D + D * D, Q = 2 * D;
  double Phi[MAXD * MAXM];
  flux_m(D, m, rho0, U, Phi);
  for (int q = 0; q < Q; ++q)
    for (int r = 0; r < M; ++r) {
      double s = 0.0;
      for (int A = 0; A < D; ++A) s += e_of(q, A) * Phi[A * M + r];
      feq[q * M + r] = (U[r] + (double)D / c * s) / (2.0 * D);
    }
}

/* Flux Jacobian action (Sec. 2.2, Eq. 18) */
static void flux_jvp(int D, const orc_mat *m, double rho0, const double *U, const double *Z, double *dPhi) {
  int M = D + D * D;
  double dP[9];
  mat_piola_jvp(D, m, U + D, Z + D, dP);
  for (int A = 0; A < D; ++A)
    for (int r = 0; r < M; ++r) {
      double val;
      if (r < D) {
        val = -dP[r * D + A] / rho0;
      } else {
        int i = (r - D) / D, B = (r - D) % D;
        val = (A == B) ? -Z[i] : 0.0;
      }
      dPhi[A * M + r] = val;
    }
}

/* Equilibrium derivative (Sec. 2.3, Eq. 27). */
static void feq_jvp_m(int D, double c, const orc_mat *m, double rho0, const double *U, const double *Z,
                      double *dfeq) {
  int M = D + D * D, Q = 2 * D;
  double dPhi[MAXD * MAXM];
  flux_jvp(D, m, rho0, U, Z, dPhi);
  for (int q = 0; q < Q; ++q)
    for (int r = 0; r < M; ++r) {
      double s = 0.0;
      for (int A = 0; A < D; ++A) s += e_of(q, A) * dPhi[A * M + r];
      dfeq[q * M + r] = (Z[r] + (double)D / c * s) / (2.0 * D);
    }
}

/* exported forms for the neo-Hookean law */
void orc_flux(int D, double mu, double lam, double rho0, const double *U, double *Phi) {
  orc_mat m = nh_mat(mu, lam);
  flux_m(D, &m, rho0, U, Phi);
}

void orc_feq(int D, double c, double mu, double lam, double rho0, const double *U, double *feq) {
  orc_mat m = nh_mat(mu, lam);
  feq_m(D, c, &m, rho0, U, feq);
}

void orc_feq_jvp(int D, double c, double mu, double lam, double rho0, const double *U, const double *Z,
                 double *dfeq) {
  orc_mat m = nh_mat(mu, lam);
  feq_jvp_m(D, c, &m, rho0, U, Z, dfeq);
}

/* ------------------------------------------------------------------------ */
/* Neumann local solves                                                       */
/* ------------------------------------------------------------------------ */

/* Weighted LSQ quadratic fit and tangent-derivative weights (Sec. 3.4,
 * Eqs. 49-52).  Basis (normalised coordinates xi):
 *   2D: 1, xi1, xi2, xi1^2/2, xi1 xi2, xi2^2/2                (Eq. 50)
 *   3D: 1, xi1, xi2, xi3, xi1^2/2, xi2^2/2, xi3^2/2, xi1xi2, xi1xi3, xi2xi3
 * Weights W_m = 1/(1 + |xi_m|^2) and the linear fallback (fewer than twice
 * as many points as basis terms, or a scaled Cholesky pivot below 1e-10) are
 * readings: the paper gives neither.  Row alpha of w is
 *   [0, t_alpha/dx, 0...] (A^T W A)^{-1} A^T W                  (Eq. 51). */
static int lsq_basis(int D, int quad, const double *xi, double *row) {
  int k = 0;
  row[k++] = 1.0;
  for (int A = 0; A < D; ++A) row[k++] = xi[A];
  if (quad) {
    if (D == 2) {
      row[k++] = 0.5 * xi[0] * xi[0];
      row[k++] = xi[0] * xi[1];
      row[k++] = 0.5 * xi[1] * xi[1];
    } else {
      row[k++] = 0.5 * xi[0] * xi[0];
      row[k++] = 0.5 * xi[1] * xi[1];
      row[k++] = 0.5 * xi[2] * xi[2];
      row[k++] = xi[0] * xi[1];
      row[k++] = xi[0] * xi[2];
      row[k++] = xi[1] * xi[2];
    }
  }
  return k;
}

int orc_lsq_weights(int D, int npts, const double *xi, const double *tang, double dx,
                    double *w) {
  for (int quad = 1; quad >= 0; --quad) {
    int nb = quad ? (D == 2 ? 6 : 10) : D + 1;
    if (npts < (quad ? 2 * nb : nb)) continue;
    double *A = (double *)malloc(sizeof(double) * npts * nb);
    double *W = (double *)malloc(sizeof(double) * npts);
    double N[10 * 10];
    for (int m = 0; m < npts; ++m) {
      lsq_basis(D, quad, xi + m * D, A + m * nb);
      double r2 = 0.0;
      for (int a = 0; a < D; ++a) r2 += xi[m * D + a] * xi[m * D + a];
      W[m] = 1.0 / (1.0 + r2);
    }
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        double s = 0.0;
        for (int m = 0; m < npts; ++m) s += A[m * nb + i] * W[m] * A[m * nb + j];
        N[i * nb + j] = s;
      }
    /* conditioning test on the Jacobi-scaled normal matrix */
    double Ns[10 * 10], sc[10];
    for (int i = 0; i < nb; ++i) sc[i] = 1.0 / sqrt(N[i * nb + i]);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) Ns[i * nb + j] = N[i * nb + j] * sc[i] * sc[j];
    int ok = 1;
    for (int k = 0; k < nb && ok; ++k) {
      double d = Ns[k * nb + k];
      for (int p = 0; p < k; ++p) d -= Ns[k * nb + p] * Ns[k * nb + p];
      if (!(d >= 1e-10)) { ok = 0; break; }
      Ns[k * nb + k] = sqrt(d);
      for (int i = k + 1; i < nb; ++i) {
        double s = Ns[i * nb + k];
        for (int p = 0; p < k; ++p) s -= Ns[i * nb + p] * Ns[k * nb + p];
        Ns[i * nb + k] = s / Ns[k * nb + k];
      }
    }
    if (ok) {
      for (int al = 0; al < D - 1; ++al) {
        double e[10] = {0}, z[10];
        for (int a = 0; a < D; ++a) e[1 + a] = tang[al * D + a] / dx;
        if (!gauss_solve(nb, N, e, z)) { ok = 0; break; }
        for (int m = 0; m < npts; ++m) {
          double s = 0.0;
          for (int j = 0; j < nb; ++j) s += A[m * nb + j] * z[j];
          w[al * npts + m] = W[m] * s;
        }
      }
    }
    free(A);
    free(W);
    if (ok) return quad ? 2 : 1;
  }
  return 0;
}

static void build_Fb(int D, const double *h, const double *N, const double *Gt, double *F) {
  for (int i = 0; i < D; ++i)
    for (int A = 0; A < D; ++A) F[i * D + A] = h[i] * N[A] + Gt[i * D + A];
}

/* R(h) = P(F_b(h)) N - T (Eqs. 54, 56); returns 0 if det F_b <= 0 */
static int newton_residual(int D, const orc_mat *m, const double *N, const double *Gt, const double *T,
                           const double *h, double *R) {
  double F[9], P[9];
  build_Fb(D, h, N, Gt, F);
  if (!(det_n(D, F) > 0.0)) return 0;
  mat_piola(D, m, F, P);
  for (int i = 0; i < D; ++i) {
    double s = 0.0;
    for (int A = 0; A < D; ++A) s += P[i * D + A] * N[A];
    R[i] = s - T[i];
  }
  for (int i = 0; i < D; ++i)
    if (!isfinite(R[i])) return 0;
  return 1;
}

/* Local Newton for the normal image h (Sec. 3.4, Eqs. 53-56).  The Jacobian
 * dR_i/dh_k = N_A C_iAkB N_B is the acoustic tensor Q(N; F_b) of Eq. 19,
 * evaluated with the tangent action; the paper's finite-difference Jacobian
 * reaches the same root.  Trial states are accepted only with det F_b > 0
 * and a decreasing residual (halving, at most 10 times). */
static int newton_m(int D, const orc_mat *m, const double *N, const double *Gt, const double *T,
                    const double *h0, double tol, double *h, int *iters) {
  double R[3], Rt[3], ht[3], Qm[9], dh[3], F[9];
  for (int i = 0; i < D; ++i) h[i] = h0[i];
  if (iters) *iters = 0;
  if (!newton_residual(D, m, N, Gt, T, h, R)) return 0;
  double thr = tol * (m->mu > 1.0 ? m->mu : 1.0);
  for (int it = 0; it <= 30; ++it) {
    double rinf = 0.0, r2 = 0.0;
    for (int i = 0; i < D; ++i) {
      rinf = fmax(rinf, fabs(R[i]));
      r2 += R[i] * R[i];
    }
    if (iters) *iters = it;
    if (rinf <= thr) return 1;
    if (it == 30) break;
    build_Fb(D, h, N, Gt, F);
    for (int k = 0; k < D; ++k) {
      double dF[9], dP[9];
      for (int i = 0; i < D; ++i)
        for (int A = 0; A < D; ++A) dF[i * D + A] = (i == k ? 1.0 : 0.0) * N[A];
      mat_piola_jvp(D, m, F, dF, dP);
      for (int i = 0; i < D; ++i) {
        double s = 0.0;
        for (int A = 0; A < D; ++A) s += dP[i * D + A] * N[A];
        Qm[i * D + k] = s;
      }
    }
    double mR[3];
    for (int i = 0; i < D; ++i) mR[i] = -R[i];
    if (!gauss_solve(D, Qm, mR, dh)) return 0;
    double step = 1.0;
    int accepted = 0;
    for (int ls = 0; ls <= 10; ++ls) {
      for (int i = 0; i < D; ++i) ht[i] = h[i] + step * dh[i];
      if (newton_residual(D, m, N, Gt, T, ht, Rt)) {
        double rt2 = 0.0, rtinf = 0.0;
        for (int i = 0; i < D; ++i) {
          rt2 += Rt[i] * Rt[i];
          rtinf = fmax(rtinf, fabs(Rt[i]));
        }
        if (rt2 < r2 || rtinf <= thr) {
          accepted = 1;
          break;
        }
      }
      step *= 0.5;
    }
    if (!accepted) return 0;
    for (int i = 0; i < D; ++i) {
      h[i] = ht[i];
      R[i] = Rt[i];
    }
  }
  return 0;
}

int orc_newton(int D, double mu, double lam, const double *N, const double *Gt, const double *T,
               const double *h0, double tol, double *h, int *iters) {
  orc_mat m = nh_mat(mu, lam);
  return newton_m(D, &m, N, Gt, T, h0, tol, h, iters);
}

/* ------------------------------------------------------------------------ */
/* the simulation                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
  int type, ramp, disp;
  double Tr, a[3], G[9], p, pn, X0[3];
  double tw; /* rigid rotation angle about e3 through X0 (displacement-given Dirichlet) */
} orc_bc;

typedef struct {
  int64_t m, mminus, out;
  int q, bid, basis;
  double eta, N[3], Xb[3], t[2][3];
  int npts;
  int64_t *pts;
  double *w; /* [(D-1)][npts] */
} orc_link;

struct orc_sim {
  int D, Q, M;
  int n[3], per[3];
  int64_t N;
  double dx, org[3];
  double mu, lam, rho0, dt, c, omega, gamma, theta;
  double k1, a0[3]; /* fibre reinforcement (k1 = 0: the paper's law) */
  int proj_every;
  int proj_sweeps;    /* > 0: damped Jacobi sweeps per projection solve; 0: exact minimiser */
  double proj_weight; /* Jacobi damping weight */
  int64_t step;
  int status, have_state, has_ls;
  uint8_t *act;
  double *f, *fs, *ustar, *u, *U;
  int64_t nl;
  orc_link *links;
  orc_bc bc[256];
  int64_t st_newton_it, st_newton_fail, st_cg_it, st_proj;
  /* initial data of the last orc_set_state (kept for the reverse mode) */
  double *U0, *u0, *dU0;
  int64_t init_step;
  /* body acceleration b(X, t) = s(t) g(X) (Eq. 5): g [N][D] or NULL */
  double *bf;
  int bf_ramp;
  double bf_Tr;
  /* Maxwell branch (orc_set_viscous): history [N][D*D] of every node, or NULL */
  double vbeta, vtau, vxi;
  double *Qh, *S0h;
  /* thermal stretch of every node (orc_set_thermal) [N], or NULL */
  double *th;
};

static void coords(const orc_sim *s, int64_t i, int *c) {
  c[0] = (int)(i % s->n[0]);
  c[1] = (int)((i / s->n[0]) % s->n[1]);
  c[2] = (int)(i / ((int64_t)s->n[0] * s->n[1]));
}

/* node at integer offset o from node i; periodic wrap on periodic axes,
 * -1 outside a non-periodic box */
static int64_t nbr_off(const orc_sim *s, int64_t i, const int *o) {
  int c[3];
  coords(s, i, c);
  for (int A = 0; A < 3; ++A) {
    int v = c[A] + (A < s->D ? o[A] : 0);
    if (v < 0 || v >= s->n[A]) {
      if (!s->per[A]) return -1;
      v = ((v % s->n[A]) + s->n[A]) % s->n[A];
    }
    c[A] = v;
  }
  return c[0] + (int64_t)s->n[0] * (c[1] + (int64_t)s->n[1] * c[2]);
}

static int64_t nbr_q(const orc_sim *s, int64_t i, int q, int mult) {
  int o[3] = {0, 0, 0};
  o[q / 2] = e_of(q, q / 2) * mult;
  return nbr_off(s, i, o);
}

static void node_pos(const orc_sim *s, int64_t i, double *X) {
  int c[3];
  coords(s, i, c);
  for (int A = 0; A < 3; ++A) X[A] = s->org[A] + (c[A] + 0.5) * s->dx;
}

orc_sim *orc_create(int D, const int *n, double dx, const double *origin, int periodic_mask,
                    double mu, double lam, double rho0, double dt, double omega,
                    double gamma, double theta_F, int proj_every) {
  if (D != 2 && D != 3) return NULL;
  if (!(dx > 0) || !(dt > 0) || !(rho0 > 0) || !(omega > 0 && omega <= 2)) return NULL;
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  s->D = D;
  s->Q = 2 * D;
  s->M = D + D * D;
  s->N = 1;
  for (int A = 0; A < 3; ++A) {
    s->n[A] = (A < D) ? n[A] : 1;
    s->per[A] = (A < D) ? ((periodic_mask >> A) & 1) : 1;
    s->org[A] = (A < D && origin) ? origin[A] : 0.0;
    s->N *= s->n[A];
  }
  s->dx = dx;
  s->dt = dt;
  s->c = dx / dt; /* lattice speed c = dx/dt (Sec. 2.3) */
  s->mu = mu;
  s->lam = lam;
  s->rho0 = rho0;
  s->omega = omega;
  s->gamma = gamma;
  s->theta = theta_F;
  s->proj_every = proj_every;
  s->proj_sweeps = ORC_PROJ_SWEEPS;
  s->proj_weight = ORC_PROJ_WEIGHT;
  s->act = (uint8_t *)malloc((size_t)s->N);
  if (!s->act) {
    orc_destroy(s);
    return NULL;
  }
  memset(s->act, 1, (size_t)s->N);
  return s;
}

/* population and field storage is allocated on first use, so that geometry
 * queries on large grids need only the active mask */
static int alloc_fields(orc_sim *s) {
  if (s->f) return ORC_OK;
  size_t nf = (size_t)s->N * s->Q * s->M;
  s->f = (double *)calloc(nf, sizeof(double));
  s->fs = (double *)calloc(nf, sizeof(double));
  s->ustar = (double *)calloc((size_t)s->N * s->D, sizeof(double));
  s->u = (double *)calloc((size_t)s->N * s->D, sizeof(double));
  s->U = (double *)calloc((size_t)s->N * s->M, sizeof(double));
  if (!s->f || !s->fs || !s->ustar || !s->u || !s->U) return ORC_ERR_MEM;
  return ORC_OK;
}

static void free_links(orc_sim *s) {
  for (int64_t l = 0; l < s->nl; ++l) {
    free(s->links[l].pts);
    free(s->links[l].w);
  }
  free(s->links);
  s->links = NULL;
  s->nl = 0;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free_links(s);
  free(s->f);
  free(s->fs);
  free(s->ustar);
  free(s->u);
  free(s->U);
  free(s->U0);
  free(s->u0);
  free(s->dU0);
  free(s->bf);
  free(s->th);
  free(s->Qh);
  free(s->S0h);
  free(s->act);
  free(s);
}

/* level-set gradient at a node by central differences (one-sided at a
 * non-periodic box edge) */
static void phi_grad(const orc_sim *s, const double *phi, int64_t i, double *g) {
  for (int A = 0; A < s->D; ++A) {
    int o[3] = {0, 0, 0};
    o[A] = 1;
    int64_t ip = nbr_off(s, i, o);
    o[A] = -1;
    int64_t im = nbr_off(s, i, o);
    if (ip >= 0 && im >= 0) g[A] = (phi[ip] - phi[im]) / (2.0 * s->dx);
    else if (ip >= 0) g[A] = (phi[ip] - phi[i]) / s->dx;
    else if (im >= 0) g[A] = (phi[i] - phi[im]) / s->dx;
    else g[A] = 0.0;
  }
}

/* cut fraction by bisection of phi along the link (Sec. 3.1, Eq. 37).  phi
 * along the link is the cubic Lagrange interpolant of the samples at link
 * parameters -1, 0, 1, 2 (linear when an outer sample lies outside the box):
 * a reading, the paper only names bisection of phi. */
static double cut_fraction(const orc_sim *s, const double *phi, int64_t m, int q) {
  int64_t o1 = nbr_q(s, m, q, 1), om = nbr_q(s, m, q, -1), o2 = nbr_q(s, m, q, 2);
  double p0 = phi[m], p1 = phi[o1];
  int cubic = (om >= 0 && o2 >= 0);
  double pm = cubic ? phi[om] : 0.0, p2 = cubic ? phi[o2] : 0.0;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 80; ++it) {
    double x = 0.5 * (lo + hi), val;
    if (cubic) {
      val = -pm * x * (x - 1.0) * (x - 2.0) / 6.0 + p0 * (x + 1.0) * (x - 1.0) * (x - 2.0) / 2.0 -
            p1 * (x + 1.0) * x * (x - 2.0) / 2.0 + p2 * (x + 1.0) * x * (x - 1.0) / 6.0;
    } else {
      val = p0 + (p1 - p0) * x;
    }
    if (val <= 0.0) lo = x;
    else hi = x;
  }
  double eta = 0.5 * (lo + hi);
  return eta < 0.0 ? 0.0 : (eta > 1.0 ? 1.0 : eta);
}

static int cmp_link(const void *a, const void *b) {
  const orc_link *x = (const orc_link *)a, *y = (const orc_link *)b;
  if (x->bid != y->bid) return x->bid < y->bid ? -1 : 1;
  if (x->m != y->m) return x->m < y->m ? -1 : 1;
  return x->q - y->q;
}

/* Active nodes and cut links (Sec. 3.1, Eqs. 36-39; link sets of Sec. 3.6). */
int orc_set_levelset(orc_sim *s, const double *phi, const uint8_t *bid) {
  int D = s->D;
  free_links(s);
  for (int64_t i = 0; i < s->N; ++i) s->act[i] = (phi[i] <= 0.0);
  /* every lattice neighbour of an active node must exist */
  for (int64_t i = 0; i < s->N; ++i) {
    if (!s->act[i]) continue;
    for (int q = 0; q < s->Q; ++q)
      if (nbr_q(s, i, q, 1) < 0) return ORC_ERR_ARG;
  }
  int64_t cnt = 0;
  for (int64_t i = 0; i < s->N; ++i) {
    if (!s->act[i]) continue;
    for (int q = 0; q < s->Q; ++q)
      if (!s->act[nbr_q(s, i, q, 1)]) ++cnt;
  }
  s->links = (orc_link *)calloc(cnt ? cnt : 1, sizeof(orc_link));
  s->nl = cnt;
  int64_t l = 0;
  for (int64_t i = 0; i < s->N; ++i) {
    if (!s->act[i]) continue;
    for (int q = 0; q < s->Q; ++q) {
      int64_t o = nbr_q(s, i, q, 1);
      if (s->act[o]) continue;
      orc_link *L = &s->links[l++];
      L->m = i;
      L->q = q;
      L->out = o;
      L->bid = bid ? bid[o] : 0; /* identifier read at the outside node */
      int64_t mm = nbr_q(s, i, q, -1);
      L->mminus = (mm >= 0 && s->act[mm]) ? mm : i; /* Eq. 43 fallback */
    }
  }
  qsort(s->links, (size_t)cnt, sizeof(orc_link), cmp_link);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < cnt; ++k) {
    orc_link *L = &s->links[k];
    int q = L->q, A = q / 2, sg = e_of(q, A);
    L->eta = cut_fraction(s, phi, L->m, q);
    double X[3], g0[3], g1[3], nrm = 0.0;
    node_pos(s, L->m, X);
    for (int a = 0; a < 3; ++a) L->Xb[a] = X[a] + (a == A ? sg * L->eta * s->dx : 0.0);
    /* normal: normalised linear interpolation of node gradients (Eq. 38) */
    phi_grad(s, phi, L->m, g0);
    phi_grad(s, phi, L->out, g1);
    for (int a = 0; a < D; ++a) {
      L->N[a] = (1.0 - L->eta) * g0[a] + L->eta * g1[a];
      nrm += L->N[a] * L->N[a];
    }
    nrm = sqrt(nrm);
    if (nrm > 0.0) {
      for (int a = 0; a < D; ++a) L->N[a] /= nrm;
    } else {
      for (int a = 0; a < D; ++a) L->N[a] = (a == A) ? sg : 0.0;
    }
    /* tangent frame */
    if (D == 2) {
      L->t[0][0] = -L->N[1];
      L->t[0][1] = L->N[0];
    } else {
      int k0 = 0;
      for (int a = 1; a < 3; ++a)
        if (fabs(L->N[a]) < fabs(L->N[k0])) k0 = a;
      double t1[3] = {0, 0, 0}, dd;
      t1[k0] = 1.0;
      dd = L->N[k0];
      double n1 = 0.0;
      for (int a = 0; a < 3; ++a) {
        t1[a] -= dd * L->N[a];
        n1 += t1[a] * t1[a];
      }
      n1 = sqrt(n1);
      for (int a = 0; a < 3; ++a) L->t[0][a] = t1[a] / n1;
      L->t[1][0] = L->N[1] * L->t[0][2] - L->N[2] * L->t[0][1];
      L->t[1][1] = L->N[2] * L->t[0][0] - L->N[0] * L->t[0][2];
      L->t[1][2] = L->N[0] * L->t[0][1] - L->N[1] * L->t[0][0];
    }
    /* LSQ stencil: active nodes within LSQ_RADIUS of X_b (reading) */
    double xi[LSQ_MAXPTS * 3];
    int64_t pts[LSQ_MAXPTS];
    int np = 0;
    int R = 4;
    for (int oz = (D == 3 ? -R : 0); oz <= (D == 3 ? R : 0); ++oz)
      for (int oy = -R; oy <= R; ++oy)
        for (int ox = -R; ox <= R; ++ox) {
          int o[3] = {ox, oy, oz};
          double xr[3], r2 = 0.0;
          for (int a = 0; a < D; ++a) {
            xr[a] = o[a] - (a == A ? sg * L->eta : 0.0);
            r2 += xr[a] * xr[a];
          }
          if (r2 > LSQ_RADIUS * LSQ_RADIUS) continue;
          int64_t j = nbr_off(s, L->m, o);
          if (j < 0 || !s->act[j]) continue;
          for (int a = 0; a < D; ++a) xi[np * D + a] = xr[a];
          pts[np++] = j;
        }
    L->npts = np;
    L->pts = (int64_t *)malloc(sizeof(int64_t) * (np ? np : 1));
    memcpy(L->pts, pts, sizeof(int64_t) * np);
    L->w = (double *)calloc((size_t)(D - 1) * (np ? np : 1), sizeof(double));
    double tg[6];
    for (int al = 0; al < D - 1; ++al)
      for (int a = 0; a < D; ++a) tg[al * D + a] = L->t[al][a];
    L->basis = orc_lsq_weights(D, np, xi, tg, s->dx, L->w);
  }
  s->has_ls = 1;
  s->have_state = 0;
  return ORC_OK;
}

int orc_set_fibres(orc_sim *s, double k1, const double *a0) {
  double n = 0.0;
  for (int A = 0; A < s->D; ++A) n += a0[A] * a0[A];
  if (!(k1 >= 0.0) || (k1 > 0.0 && !(n > 0.0))) return ORC_ERR_ARG;
  s->k1 = k1;
  for (int A = 0; A < 3; ++A) s->a0[A] = (A < s->D && n > 0.0) ? a0[A] / sqrt(n) : 0.0;
  return ORC_OK;
}

int orc_set_viscous(orc_sim *s, double beta, double tau) {
  if (!(beta >= 0.0) || !(tau >= 0.0) || s->th) return ORC_ERR_ARG;
  if (!s->Qh) {
    s->Qh = (double *)calloc((size_t)s->N * s->D * s->D, sizeof(double));
    s->S0h = (double *)calloc((size_t)s->N * s->D * s->D, sizeof(double));
    if (!s->Qh || !s->S0h) return ORC_ERR_MEM;
  }
  s->vbeta = beta;
  s->vtau = tau;
  s->vxi = exp(-s->dt / (2.0 * tau)); /* tau = 0: 0; tau = inf: 1 */
  s->have_state = 0;                  /* the history starts at orc_set_state */
  return ORC_OK;
}

int orc_get_viscous(orc_sim *s, double *Qh, double *S0h) {
  int DD = s->D * s->D;
  if (!s->Qh) return ORC_ERR_ARG;
  for (int64_t i = 0; i < s->N; ++i)
    for (int k = 0; k < DD; ++k) {
      if (Qh) Qh[(size_t)k * s->N + i] = s->act[i] ? s->Qh[(size_t)i * DD + k] : 0.0;
      if (S0h) S0h[(size_t)k * s->N + i] = s->act[i] ? s->S0h[(size_t)i * DD + k] : 0.0;
    }
  return ORC_OK;
}

int orc_set_thermal(orc_sim *s, const double *th) {
  if (!th) {
    free(s->th);
    s->th = NULL;
    return ORC_OK;
  }
  if (s->Qh) return ORC_ERR_ARG;
  for (int64_t i = 0; i < s->N; ++i)
    if (!(th[i] > 0.0) || !isfinite(th[i])) return ORC_ERR_ARG;
  if (!s->th) s->th = (double *)malloc(sizeof(double) * (size_t)s->N);
  if (!s->th) return ORC_ERR_MEM;
  memcpy(s->th, th, sizeof(double) * (size_t)s->N);
  return ORC_OK;
}

int orc_set_body_force(orc_sim *s, const double *g, int ramp, double T_r) {
  free(s->bf);
  s->bf = NULL;
  if (!g) return ORC_OK;
  s->bf = (double *)malloc(sizeof(double) * (size_t)s->N * s->D);
  if (!s->bf) return ORC_ERR_MEM;
  for (int64_t i = 0; i < s->N; ++i)
    for (int a = 0; a < s->D; ++a) s->bf[i * s->D + a] = g[(size_t)a * s->N + i];
  s->bf_ramp = ramp;
  s->bf_Tr = T_r;
  return ORC_OK;
}

int orc_set_projection(orc_sim *s, int sweeps, double weight) {
  if (sweeps < 0 || !(weight > 0.0 && weight <= 1.0)) return ORC_ERR_ARG;
  s->proj_sweeps = sweeps;
  s->proj_weight = weight;
  return ORC_OK;
}

int orc_set_bc(orc_sim *s, int bid, int type, int ramp, double T_r, int disp, const double *a,
               const double *G, double p_radial, double p_normal, const double *X0) {
  if (bid < 0 || bid > 255) return ORC_ERR_ARG;
  orc_bc *b = &s->bc[bid];
  memset(b, 0, sizeof(*b));
  b->type = type;
  b->ramp = ramp;
  b->Tr = T_r;
  b->disp = disp;
  b->p = p_radial;
  b->pn = p_normal;
  for (int k = 0; k < 3; ++k) {
    b->a[k] = a ? a[k] : 0.0;
    b->X0[k] = X0 ? X0[k] : 0.0;
  }
  for (int k = 0; k < 9; ++k) b->G[k] = G ? G[k] : 0.0;
  return ORC_OK;
}

int orc_set_bc_twist(orc_sim *s, int bid, double twist) {
  if (bid < 0 || bid > 255) return ORC_ERR_ARG;
  orc_bc *b = &s->bc[bid];
  if (twist != 0.0 && !(b->type == ORC_BC_DIRICHLET && b->disp)) return ORC_ERR_ARG;
  b->tw = twist;
  return ORC_OK;
}

/* loading factor s(t) and its derivative: sine-squared ramp (Sec. 4.3,
 * Eq. 71), half-cosine ramp (Sec. 5.3, Eq. 88), linear ramp, constant */
static void ramp_eval(int kind, double Tr, double t, double *sv, double *dsv) {
  *sv = 1.0;
  *dsv = 0.0;
  if (kind == ORC_RAMP_SIN2 && t < Tr) {
    double a = M_PI * t / (2.0 * Tr);
    *sv = sin(a) * sin(a);
    *dsv = M_PI / (2.0 * Tr) * sin(M_PI * t / Tr);
  } else if (kind == ORC_RAMP_HALFCOS && t < Tr) {
    *sv = 0.5 * (1.0 - cos(M_PI * t / Tr));
    *dsv = 0.5 * M_PI / Tr * sin(M_PI * t / Tr);
  } else if (kind == ORC_RAMP_LINEAR && t < Tr) {
    *sv = t / Tr;
    *dsv = 1.0 / Tr;
  }
}

/* time integral S(t) of the loading factor, S(0) = 0 */
static double ramp_integral(int kind, double Tr, double t) {
  double tc = (t < Tr) ? t : Tr, S;
  if (kind == ORC_RAMP_SIN2) S = 0.5 * tc - Tr / (2.0 * M_PI) * sin(M_PI * tc / Tr);
  else if (kind == ORC_RAMP_HALFCOS) S = 0.5 * tc - Tr / (2.0 * M_PI) * sin(M_PI * tc / Tr);
  else if (kind == ORC_RAMP_LINEAR) S = 0.5 * tc * tc / Tr;
  else return t;
  return S + (t - tc);
}

/* prescribed boundary value at (X, t): s(t) (a + G (X - X0) + p e_R + pn N_b)
 * with e_R the unit vector from X0; a displacement-given Dirichlet value is
 * imposed through its rate v_D = d u_D / dt (Sec. 2.1, Eq. 9) */
static void bc_value(const orc_bc *b, int D, const double *X, const double *Nb, double t,
                     double *val) {
  double sv, dsv, base[3], d[3], r = 0.0;
  ramp_eval(b->ramp, b->Tr, t, &sv, &dsv);
  for (int a = 0; a < D; ++a) {
    d[a] = X[a] - b->X0[a];
    r += d[a] * d[a];
  }
  r = sqrt(r);
  for (int i = 0; i < D; ++i) {
    double s = b->a[i];
    for (int A = 0; A < D; ++A) s += b->G[i * 3 + A] * d[A];
    if (b->p != 0.0 && r > 0.0) s += b->p * d[i] / r;
    s += b->pn * Nb[i];
    base[i] = s;
  }
  double fac = (b->type == ORC_BC_DIRICHLET && b->disp) ? dsv : sv;
  for (int i = 0; i < D; ++i) val[i] = fac * base[i];
  if (b->type == ORC_BC_DIRICHLET && b->disp && b->tw != 0.0) {
    /* velocity of the ramped rotation u = (R(s tw) - I) d (Sec. 5.3, Eq. 87) */
    double al = sv * b->tw, da = dsv * b->tw;
    val[0] += da * (-sin(al) * d[0] - cos(al) * d[1]);
    val[1] += da * (cos(al) * d[0] - sin(al) * d[1]);
  }
}

/* prescribed Dirichlet displacement u_D(X, t): the value itself when the
 * condition is given as a displacement, otherwise the time integral of the
 * prescribed velocity from the reference configuration at t = 0 */
static void bc_displacement(const orc_bc *b, int D, const double *X, const double *Nb, double t,
                            double *val) {
  double sv, dsv;
  ramp_eval(b->ramp, b->Tr, t, &sv, &dsv);
  orc_bc tmp = *b;
  tmp.type = ORC_BC_NEUMANN; /* returns s(t) * base */
  tmp.ramp = ORC_RAMP_CONST;
  bc_value(&tmp, D, X, Nb, t, val); /* base */
  double fac = b->disp ? sv : ramp_integral(b->ramp, b->Tr, t);
  for (int i = 0; i < D; ++i) val[i] *= fac;
  if (b->disp && b->tw != 0.0) {
    double al = sv * b->tw, d0 = X[0] - b->X0[0], d1 = X[1] - b->X0[1];
    val[0] += (cos(al) - 1.0) * d0 - sin(al) * d1;
    val[1] += sin(al) * d0 + (cos(al) - 1.0) * d1;
  }
}

/* boundary data of identifier bid at point X (normal Nb) and time t: the
 * imposed velocity (Dirichlet) or traction (Neumann) and, for Dirichlet, the
 * prescribed displacement; exposed so that tests can check the data itself */
int orc_bc_data(orc_sim *s, int bid, const double *X, const double *Nb, double t, double *val, double *disp) {
  if (!s || bid < 0 || bid > 255 || !X || !Nb || !val) return ORC_ERR_ARG;
  const orc_bc *b = &s->bc[bid];
  bc_value(b, s->D, X, Nb, t, val);
  if (disp) bc_displacement(b, s->D, X, Nb, t, disp);
  return ORC_OK;
}

/* material of node m of the simulation with the given (mu, lambda); with a
 * Maxwell branch it carries the node's history (m < 0: none) */
static orc_mat sim_mat(const orc_sim *s, double mu, double lam, int64_t m) {
  orc_mat mat = {mu, lam, s->k1, {s->a0[0], s->a0[1], s->a0[2]}, 0.0, 0.0, NULL, NULL, 1.0};
  if (s->th && m >= 0) mat.th = s->th[m];
  if (s->Qh && m >= 0) {
    size_t o = (size_t)m * s->D * s->D;
    mat.beta = s->vbeta;
    mat.xi = s->vxi;
    mat.Qh = s->Qh + o;
    mat.S0h = s->S0h + o;
  }
  return mat;
}

/* body acceleration at node i and time t (zero without a field) */
static void body_acc(const orc_sim *s, int64_t i, double t, double *b) {
  for (int a = 0; a < s->D; ++a) b[a] = 0.0;
  if (!s->bf) return;
  double sv, dsv;
  ramp_eval(s->bf_ramp, s->bf_Tr, t, &sv, &dsv);
  for (int a = 0; a < s->D; ++a) b[a] = sv * s->bf[i * s->D + a];
}

/* Second-order initialisation (Sec. 2.4, Eqs. 32-33):
 *   f_q = feq(U0) - dt/2 (dt + c e_qA d_A) feq(U0),
 *   dt U0 = B0 - Phi'_A(U0) d_A U0,
 * with the directional derivatives taken through the equilibrium derivative
 * of Eq. 27.  With no gradients supplied the spatial terms vanish. */
/* populations of one node from U0 and its derivatives dA[A*M + r] */
static void init_node(const orc_sim *s, int64_t node, double mu, double lam, const double *U, const double *dA,
                      const double *b0, double *f) {
  int D = s->D, M = s->M, Q = s->Q;
  double Ut[MAXM], feq[MAXQ * MAXM], dPhi[MAXD * MAXM];
  const orc_mat mat = sim_mat(s, mu, lam, node);
  /* B0 = (b0 - gamma v0, 0): body acceleration and velocity damping */
  for (int r = 0; r < M; ++r) Ut[r] = (r < D) ? b0[r] - s->gamma * U[r] : 0.0;
  for (int A = 0; A < D; ++A) {
    flux_jvp(D, &mat, s->rho0, U, dA + A * M, dPhi);
    for (int r = 0; r < M; ++r) Ut[r] -= dPhi[A * M + r];
  }
  feq_m(D, s->c, &mat, s->rho0, U, feq);
  for (int q = 0; q < Q; ++q) {
    double Z[MAXM], dfeq[MAXQ * MAXM];
    for (int r = 0; r < M; ++r) {
      double s2 = Ut[r];
      for (int A = 0; A < D; ++A) s2 += s->c * e_of(q, A) * dA[A * M + r];
      Z[r] = s2;
    }
    feq_jvp_m(D, s->c, &mat, s->rho0, U, Z, dfeq);
    for (int r = 0; r < M; ++r) f[q * M + r] = feq[q * M + r] - 0.5 * s->dt * dfeq[q * M + r];
  }
}

static void keep_initial_data(orc_sim *s, const double *U0, const double *u0, const double *dU0) {
  size_t NM = (size_t)s->N * s->M;
  free(s->U0);
  free(s->u0);
  free(s->dU0);
  s->U0 = (double *)malloc(sizeof(double) * NM);
  s->u0 = (double *)calloc((size_t)s->N * s->D, sizeof(double));
  s->dU0 = (double *)calloc(NM * s->D, sizeof(double));
  if (!s->U0 || !s->u0 || !s->dU0) return;
  memcpy(s->U0, U0, sizeof(double) * NM);
  if (u0) memcpy(s->u0, u0, sizeof(double) * (size_t)s->N * s->D);
  if (dU0) memcpy(s->dU0, dU0, sizeof(double) * NM * s->D);
}

int orc_set_state(orc_sim *s, const double *U0, const double *u0, const double *dU0) {
  int D = s->D, M = s->M, Q = s->Q;
  int err = 0;
  /* without a level set every node is active: all axes must then wrap */
  if (!s->has_ls)
    for (int A = 0; A < D; ++A)
      if (!s->per[A]) return ORC_ERR_ARG;
  if (alloc_fields(s)) return ORC_ERR_MEM;
#pragma omp parallel for reduction(| : err)
  for (int64_t i = 0; i < s->N; ++i) {
    double *f = s->f + (size_t)i * Q * M;
    if (!s->act[i]) {
      memset(f, 0, sizeof(double) * Q * M);
      for (int a = 0; a < D; ++a) s->ustar[i * D + a] = 0.0;
      continue;
    }
    double U[MAXM], dA[MAXD * MAXM];
    for (int r = 0; r < M; ++r) U[r] = U0[(size_t)r * s->N + i];
    if (!(det_n(D, U + D) > 0.0)) {
      err |= 1;
      continue;
    }
    for (int A = 0; A < D; ++A)
      for (int r = 0; r < M; ++r)
        dA[A * M + r] = dU0 ? dU0[((size_t)A * M + r) * s->N + i] : 0.0;
    double b0[MAXD];
    body_acc(s, i, s->step * s->dt, b0);
    if (s->Qh) { /* the branch starts relaxed at F0: Q = 0, S0h = S_0(F0) */
      double *Qh = s->Qh + (size_t)i * D * D, *S0h = s->S0h + (size_t)i * D * D;
      for (int k = 0; k < D * D; ++k) Qh[k] = 0.0;
      visco_S0(D, s->mu, U + D, S0h, NULL);
    }
    init_node(s, i, s->mu, s->lam, U, dA, b0, f);
    for (int a = 0; a < D; ++a) {
      double u0a = u0 ? u0[(size_t)a * s->N + i] : 0.0;
      s->ustar[i * D + a] = u0a - 0.5 * s->dt * U[a]; /* so that u^0 = u0 (Eq. 34) */
    }
  }
  if (err) return ORC_ERR_J;
  keep_initial_data(s, U0, u0, dU0);
  s->step = 0;
  s->init_step = 0;
  s->status = ORC_OK;
  s->have_state = 1;
  return ORC_OK;
}

/* State recovery (Eq. 28) with the velocity-proportional damping source
 * B = (-gamma v, 0) of Sec. 4.1.  The half-step source makes the recovered
 * velocity implicit; its closed form v = sum_q f^v / (1 + gamma dt/2) is a
 * reading (the paper is silent). */
/* U^n = sum_q f_q + dt/2 B^n (Eq. 28) with B^n = (b^n - gamma v^n, 0): the
 * damping part is implicit in v^n */
static int recover(orc_sim *s) {
  int D = s->D, M = s->M, Q = s->Q;
  int err = 0;
  const double tn = s->step * s->dt;
#pragma omp parallel for reduction(| : err)
  for (int64_t i = 0; i < s->N; ++i) {
    if (!s->act[i]) continue;
    const double *f = s->f + (size_t)i * Q * M;
    double *U = s->U + (size_t)i * M;
    for (int r = 0; r < M; ++r) {
      double acc = 0.0;
      for (int q = 0; q < Q; ++q) acc += f[q * M + r];
      U[r] = acc;
    }
    double b[MAXD];
    body_acc(s, i, tn, b);
    for (int a = 0; a < D; ++a) U[a] = (U[a] + 0.5 * s->dt * b[a]) / (1.0 + 0.5 * s->gamma * s->dt);
    for (int r = 0; r < M; ++r)
      if (!isfinite(U[r])) err |= 2;
    if (!(det_n(D, U + D) > 0.0)) err |= 1;
    for (int a = 0; a < D; ++a) s->u[i * D + a] = s->ustar[i * D + a] + 0.5 * s->dt * U[a];
  }
  if (err & 2) return ORC_ERR_NONFINITE;
  if (err & 1) return ORC_ERR_J;
  return ORC_OK;
}

/* ---- compatibility projection (Sec. 3.5) -------------------------------- */

/* right-hand side of the normal equations of the edge least-squares problem
 * (Eq. 57): for the edge l -> m = l + e_A the target difference is
 * r = (dx/2) [(F_m - I) + (F_l - I)] e_A ; b_m = sum_in r - sum_out r. */
static void proj_rhs(const orc_sim *s, const double *Unm, int comp, double *b) {
  int D = s->D, M = s->M;
#pragma omp parallel for
  for (int64_t m = 0; m < s->N; ++m) {
    if (!s->act[m]) {
      b[m] = 0.0;
      continue;
    }
    double acc = 0.0;
    const double *Fm = Unm + (size_t)m * M + D;
    for (int A = 0; A < D; ++A) {
      int64_t lp = nbr_q(s, m, 2 * A, 1), lm = nbr_q(s, m, 2 * A + 1, 1);
      double d = (comp == A) ? 1.0 : 0.0;
      if (lm >= 0 && s->act[lm]) {
        const double *Fl = Unm + (size_t)lm * M + D;
        acc += 0.5 * s->dx * (Fm[comp * D + A] + Fl[comp * D + A] - 2.0 * d);
      }
      if (lp >= 0 && s->act[lp]) {
        const double *Fl = Unm + (size_t)lp * M + D;
        acc -= 0.5 * s->dx * (Fm[comp * D + A] + Fl[comp * D + A] - 2.0 * d);
      }
    }
    b[m] = acc;
  }
}

/* graph Laplacian of the active-node graph: (L x)_m = sum_{l~m} (x_m - x_l) */
static void graph_lap(const orc_sim *s, const double *x, double *y) {
#pragma omp parallel for
  for (int64_t m = 0; m < s->N; ++m) {
    if (!s->act[m]) {
      y[m] = 0.0;
      continue;
    }
    double acc = 0.0;
    for (int q = 0; q < s->Q; ++q) {
      int64_t l = nbr_q(s, m, q, 1);
      if (l >= 0 && s->act[l]) acc += x[m] - x[l];
    }
    y[m] = acc;
  }
}

static double dot_act(const orc_sim *s, const double *a, const double *b) {
  double acc = 0.0;
#pragma omp parallel for reduction(+ : acc)
  for (int64_t m = 0; m < s->N; ++m)
    if (s->act[m]) acc += a[m] * b[m];
  return acc;
}

/* Exact minimiser of the edge least-squares problem by conjugate gradients,
 * warm-started from the current displacement.
 *
 * Null mode (Sec. 3.5 allows a gauge condition or prescribed displacement
 * anchors): every Dirichlet cut link (m, q) adds the anchor relation
 *   u^c_m + (F_m - I)(X_b - X_m) = u_D(X_b, t^n)
 * with unit weight, which makes the normal matrix L + A definite on every
 * connected component that touches a Dirichlet boundary.  On components
 * without anchors CG from x0 stays in x0 + range(L), which fixes the constant
 * to the mean of the warm start (the gauge).  anc_n[m] counts anchors of node
 * m and anc_s[m*D + i] sums their targets; both may be NULL. */
static int64_t proj_jacobi(orc_sim *s, const double *Unm, double *u, const int *anc_n, const double *anc_s);

static int64_t proj_solve(orc_sim *s, const double *Unm, double *u /* [N][D] */, double rtol,
                          const int *anc_n, const double *anc_s) {
  if (s->proj_sweeps > 0) return proj_jacobi(s, Unm, u, anc_n, anc_s);
  int64_t N = s->N, its = 0;
  double *b = (double *)malloc(sizeof(double) * N), *x = (double *)malloc(sizeof(double) * N);
  double *r = (double *)malloc(sizeof(double) * N), *p = (double *)malloc(sizeof(double) * N);
  double *Ap = (double *)malloc(sizeof(double) * N);
  int64_t nact = 0;
  for (int64_t m = 0; m < N; ++m) nact += s->act[m];
  int64_t maxit = 10 * nact + 100;
  for (int comp = 0; comp < s->D; ++comp) {
    proj_rhs(s, Unm, comp, b);
    if (anc_n)
      for (int64_t m = 0; m < N; ++m) b[m] += anc_s[m * s->D + comp];
    for (int64_t m = 0; m < N; ++m) x[m] = s->act[m] ? u[m * s->D + comp] : 0.0;
    graph_lap(s, x, Ap);
    if (anc_n)
      for (int64_t m = 0; m < N; ++m) Ap[m] += anc_n[m] * x[m];
    for (int64_t m = 0; m < N; ++m) {
      r[m] = s->act[m] ? b[m] - Ap[m] : 0.0;
      p[m] = r[m];
    }
    double bb = dot_act(s, b, b), rr = dot_act(s, r, r);
    double thr = rtol * rtol * (bb > rr ? bb : rr);
    int64_t k = 0;
    while (rr > thr && k < maxit) {
      graph_lap(s, p, Ap);
      if (anc_n)
        for (int64_t m = 0; m < N; ++m) Ap[m] += anc_n[m] * p[m];
      double pAp = dot_act(s, p, Ap);
      if (!(pAp > 0.0)) break;
      double alpha = rr / pAp;
      for (int64_t m = 0; m < N; ++m) {
        x[m] += alpha * p[m];
        r[m] -= alpha * Ap[m];
      }
      double rr2 = dot_act(s, r, r);
      double beta = rr2 / rr;
      rr = rr2;
      for (int64_t m = 0; m < N; ++m) p[m] = r[m] + beta * p[m];
      ++k;
    }
    its += k;
    for (int64_t m = 0; m < N; ++m)
      if (s->act[m]) u[m * s->D + comp] = x[m];
  }
  free(b); free(x); free(r); free(p); free(Ap);
  return its;
}

/* diagonal of the normal matrix K = graph Laplacian + anchor counts */
static double proj_diag(const orc_sim *s, const int *anc_n, int64_t m) {
  double d = anc_n ? anc_n[m] : 0;
  for (int q = 0; q < s->Q; ++q) {
    int64_t l = nbr_q(s, m, q, 1);
    if (l >= 0 && s->act[l]) d += 1.0;
  }
  return d;
}

/* Damped Jacobi relaxation of the same normal equations (Sec. 3.5: the
 * paper relaxes them by damped Jacobi iterations on the active-node graph,
 * started from the current displacement): per component, proj_sweeps sweeps
 *   x <- x + w (b - K x) / diag(K)
 * with w = proj_weight.  A node with a zero diagonal (no active neighbour and
 * no anchor) has no edge relation and keeps its value. */
static int64_t proj_jacobi(orc_sim *s, const double *Unm, double *u, const int *anc_n, const double *anc_s) {
  int64_t N = s->N;
  double *b = (double *)malloc(sizeof(double) * N), *x = (double *)malloc(sizeof(double) * N);
  double *Kx = (double *)malloc(sizeof(double) * N);
  for (int comp = 0; comp < s->D; ++comp) {
    proj_rhs(s, Unm, comp, b);
    if (anc_n)
      for (int64_t m = 0; m < N; ++m) b[m] += anc_s[m * s->D + comp];
    for (int64_t m = 0; m < N; ++m) x[m] = s->act[m] ? u[m * s->D + comp] : 0.0;
    for (int k = 0; k < s->proj_sweeps; ++k) {
      graph_lap(s, x, Kx);
#pragma omp parallel for
      for (int64_t m = 0; m < N; ++m) {
        if (!s->act[m]) continue;
        double d = proj_diag(s, anc_n, m);
        if (d == 0.0) continue;
        double kx = Kx[m] + (anc_n ? anc_n[m] * x[m] : 0.0);
        u[m * s->D + comp] = x[m] + s->proj_weight * (b[m] - kx) / d;
      }
      for (int64_t m = 0; m < N; ++m)
        if (s->act[m]) x[m] = u[m * s->D + comp];
    }
  }
  free(b); free(x); free(Kx);
  return (int64_t)s->proj_sweeps * s->D;
}

/* anchor counts and target sums from the Dirichlet cut links at time t */
static void proj_anchors(orc_sim *s, const double *Unm, double t, int **anc_n, double **anc_s) {
  int D = s->D, M = s->M;
  *anc_n = NULL;
  *anc_s = NULL;
  int any = 0;
  for (int64_t l = 0; l < s->nl; ++l)
    if (s->bc[s->links[l].bid].type == ORC_BC_DIRICHLET) any = 1;
  if (!any) return;
  int *n = (int *)calloc((size_t)s->N, sizeof(int));
  double *a = (double *)calloc((size_t)s->N * D, sizeof(double));
  for (int64_t l = 0; l < s->nl; ++l) {
    const orc_link *L = &s->links[l];
    const orc_bc *b = &s->bc[L->bid];
    if (b->type != ORC_BC_DIRICHLET) continue;
    double uD[3];
    bc_displacement(b, D, L->Xb, L->N, t, uD);
    const double *Fm = Unm + (size_t)L->m * M + D;
    int A = L->q / 2, sg = e_of(L->q, A);
    double off = sg * L->eta * s->dx; /* X_b - X_m along axis A */
    n[L->m] += 1;
    for (int i = 0; i < D; ++i) a[L->m * D + i] += uD[i] - (Fm[i * D + A] - (i == A ? 1.0 : 0.0)) * off;
  }
  *anc_n = n;
  *anc_s = a;
}

/* compatible deformation gradient F^c = I + grad_dx u^c (Eq. 59): centred
 * differences where both axis neighbours are active, one-sided where only one
 * is, and the evolved column kept where neither is (reading). */
static void compat_F(const orc_sim *s, const double *u, const double *Unm, double *Fc) {
  int D = s->D, M = s->M;
#pragma omp parallel for
  for (int64_t m = 0; m < s->N; ++m) {
    if (!s->act[m]) continue;
    for (int A = 0; A < D; ++A) {
      int64_t lp = nbr_q(s, m, 2 * A, 1), lm = nbr_q(s, m, 2 * A + 1, 1);
      int hp = (lp >= 0 && s->act[lp]), hm = (lm >= 0 && s->act[lm]);
      for (int i = 0; i < D; ++i) {
        double g;
        if (hp && hm) g = (u[lp * D + i] - u[lm * D + i]) / (2.0 * s->dx);
        else if (hp) g = (u[lp * D + i] - u[m * D + i]) / s->dx;
        else if (hm) g = (u[m * D + i] - u[lm * D + i]) / s->dx;
        else {
          Fc[(size_t)m * D * D + i * D + A] = Unm[(size_t)m * M + D + i * D + A];
          continue;
        }
        Fc[(size_t)m * D * D + i * D + A] = (i == A ? 1.0 : 0.0) + g;
      }
    }
  }
}

#define PROJ_RTOL 1e-15

/* ---- cut links (Secs. 3.2-3.4) ------------------------------------------ */

/* boundary deformation gradient of a Neumann link (Sec. 3.4): tangent images
 * g_a = t_a + sum_m w_a,m u_m (Eqs. 48-52) from the current displacement,
 * then the normal image h from the local Newton solve (Eqs. 53-56), and
 * F_b = h (x) N + sum_a g_a (x) t_a.  Returns 0 (with F_b = I) when the root
 * is not admissible. */
static int neumann_Fb(orc_sim *s, const orc_link *L, double th, int count, double *Gt, double *Fb) {
  int D = s->D, M = s->M;
  const orc_bc *b = &s->bc[L->bid];
  double T[3], h0[3], h[3];
  for (int k = 0; k < 9; ++k) Gt[k] = 0.0;
  for (int al = 0; al < D - 1; ++al) {
    double g[3];
    for (int i = 0; i < D; ++i) {
      double acc = L->t[al][i];
      for (int k = 0; k < L->npts; ++k) acc += L->w[al * L->npts + k] * s->u[L->pts[k] * D + i];
      g[i] = acc;
    }
    for (int i = 0; i < D; ++i)
      for (int B = 0; B < D; ++B) Gt[i * D + B] += g[i] * L->t[al][B];
  }
  bc_value(b, D, L->Xb, L->N, th, T);
  /* initial guess h0 = F_m N_b from the link's active node (reading) */
  const double *Fm = s->U + (size_t)L->m * M + D;
  for (int i = 0; i < D; ++i) {
    double acc = 0.0;
    for (int B = 0; B < D; ++B) acc += Fm[i * D + B] * L->N[B];
    h0[i] = acc;
  }
  int its = 0;
  const orc_mat mat = sim_mat(s, s->mu, s->lam, L->m);
  int conv = newton_m(D, &mat, L->N, Gt, T, h0, 1e-12, h, &its);
  if (count) {
#pragma omp atomic
    s->st_newton_it += its;
    if (!conv) {
#pragma omp atomic
      s->st_newton_fail += 1;
    }
  }
  build_Fb(D, h, L->N, Gt, Fb);
  if (!(det_n(D, Fb) > 0.0)) {
    for (int k = 0; k < D * D; ++k) Fb[k] = (k % (D + 1) == 0) ? 1.0 : 0.0;
    return 0;
  }
  return 1;
}

static int close_link(orc_sim *s, const orc_link *L, double tn) {
  int D = s->D, M = s->M, Q = s->Q;
  const orc_bc *b = &s->bc[L->bid];
  int qo = L->q, qi = qo ^ 1, A = qo / 2, sg = e_of(qo, A);
  double d[3] = {0, 0, 0};
  d[A] = -sg; /* incoming direction d = -e (Eq. 39) */
  double Dsign[MAXM], S[MAXM];
  double th = tn + 0.5 * s->dt; /* boundary data at t^n + dt/2 */
  int ok = 1;
  if (b->type == ORC_BC_DIRICHLET) {
    /* Eqs. 44-45: D_D = diag(-I_D, I_D2), S^v = v_b/D, S^F_iB = -d_B v_b,i / c */
    double vb[3];
    bc_value(b, D, L->Xb, L->N, th, vb);
    for (int r = 0; r < M; ++r) {
      if (r < D) {
        Dsign[r] = -1.0;
        S[r] = vb[r] / D;
      } else {
        int i = (r - D) / D, B = (r - D) % D;
        Dsign[r] = 1.0;
        S[r] = -d[B] * vb[i] / s->c;
      }
    }
  } else if (b->type == ORC_BC_NEUMANN) {
    double Gt[9], Fb[9], Pb[9];
    ok = neumann_Fb(s, L, th, 1, Gt, Fb);
    const orc_mat mat = sim_mat(s, s->mu, s->lam, L->m);
    mat_piola(D, &mat, Fb, Pb);
    /* Eqs. 46-47: D_N = diag(I_D, -I_D2), S^v_i = -d_A P_b,iA / c,
     * S^F_iB = F_b,iB / D ; the density divides the stress flux */
    for (int r = 0; r < M; ++r) {
      if (r < D) {
        double acc = 0.0;
        for (int B = 0; B < D; ++B) acc += d[B] * Pb[r * D + B];
        Dsign[r] = 1.0;
        S[r] = -acc / (s->rho0 * s->c);
      } else {
        Dsign[r] = -1.0;
        S[r] = Fb[r - D] / D;
      }
    }
  } else {
    return 0; /* link without a boundary condition */
  }
  /* cut-link interpolation (Eqs. 42-43) */
  const double *fs_m = s->fs + (size_t)L->m * Q * M;
  const double *fs_mm = s->fs + (size_t)L->mminus * Q * M;
  double *fn = s->f + (size_t)L->m * Q * M + qi * M;
  double eta = L->eta;
  for (int r = 0; r < M; ++r) {
    double fo = fs_m[qo * M + r]; /* f*_{-d}(X_f) */
    double fi = fs_m[qi * M + r]; /* f*_{d}(X_f)  */
    if (eta >= 0.5) {
      fn[r] = (Dsign[r] * fo + S[r]) / (2.0 * eta) + (1.0 - 1.0 / (2.0 * eta)) * fi;
    } else {
      fn[r] = Dsign[r] * (2.0 * eta * fo + (1.0 - 2.0 * eta) * fs_mm[qo * M + r]) + S[r];
    }
  }
  return ok ? 1 : -1;
}

/* projection + repair (first block of Algorithm 1 guarded by C^N) */
static void project_pre(orc_sim *s, double tn) {
  int D = s->D, M = s->M, Q = s->Q;
  int *anc_n;
  double *anc_s;
  proj_anchors(s, s->U, tn, &anc_n, &anc_s);
  s->st_cg_it += proj_solve(s, s->U, s->u, PROJ_RTOL, anc_n, anc_s);
  free(anc_n);
  free(anc_s);
  double *Fc = (double *)malloc(sizeof(double) * (size_t)s->N * D * D);
  compat_F(s, s->u, s->U, Fc);
#pragma omp parallel for
  for (int64_t m = 0; m < s->N; ++m) {
    if (!s->act[m]) continue;
    double *U = s->U + (size_t)m * M;
    for (int a = 0; a < D; ++a) s->ustar[m * D + a] = s->u[m * D + a] - 0.5 * s->dt * U[a];
    double Ur[MAXM], fe0[MAXQ * MAXM], fe1[MAXQ * MAXM];
    for (int r = 0; r < M; ++r) Ur[r] = U[r];
    for (int k = 0; k < D * D; ++k)
      Ur[D + k] = (1.0 - s->theta) * U[D + k] + s->theta * Fc[(size_t)m * D * D + k];
    const orc_mat mat = sim_mat(s, s->mu, s->lam, m);
    feq_m(D, s->c, &mat, s->rho0, U, fe0);
    feq_m(D, s->c, &mat, s->rho0, Ur, fe1);
    double *f = s->f + (size_t)m * Q * M;
    for (int k = 0; k < Q * M; ++k) f[k] += fe1[k] - fe0[k]; /* Eq. 61 */
    for (int r = 0; r < M; ++r) U[r] = Ur[r];
  }
  free(Fc);
}

int orc_step(orc_sim *s, int64_t nsteps) {
  int D = s->D, M = s->M, Q = s->Q;
  if (!s->have_state) return ORC_ERR_ORDER;
  if (s->status) return s->status;
  int has_neu = 0;
  for (int64_t l = 0; l < s->nl; ++l)
    if (s->bc[s->links[l].bid].type == ORC_BC_NEUMANN) has_neu = 1;
  for (int64_t l = 0; l < s->nl; ++l)
    if (s->bc[s->links[l].bid].type == ORC_BC_NONE) return ORC_ERR_ARG;
  for (int64_t it = 0; it < nsteps; ++it) {
    double tn = s->step * s->dt;
    int st = recover(s);
    if (st) {
      s->status = st;
      return st;
    }
    int proj = has_neu && s->proj_every > 0 && (s->step % s->proj_every == 0);
    if (proj) {
      project_pre(s, tn);
      s->st_proj++;
    }
    /* local collision (Eq. 29) with source weights w_q = 1/(4D) (Eq. 30),
     * and the displacement history advance (Eq. 34) */
#pragma omp parallel for
    for (int64_t m = 0; m < s->N; ++m) {
      if (!s->act[m]) continue;
      const double *U = s->U + (size_t)m * M;
      double feq[MAXQ * MAXM], B[MAXM], b[MAXD];
      const orc_mat mat = sim_mat(s, s->mu, s->lam, m);
      feq_m(D, s->c, &mat, s->rho0, U, feq);
      body_acc(s, m, tn, b);
      for (int r = 0; r < M; ++r) B[r] = (r < D) ? b[r] - s->gamma * U[r] : 0.0;
      const double *f = s->f + (size_t)m * Q * M;
      double *fs = s->fs + (size_t)m * Q * M;
      for (int q = 0; q < Q; ++q)
        for (int r = 0; r < M; ++r)
          fs[q * M + r] = f[q * M + r] + s->omega * (feq[q * M + r] - f[q * M + r]) +
                          s->dt * (2.0 - s->omega) * B[r] / (4.0 * D);
      for (int a = 0; a < D; ++a) s->ustar[m * D + a] = s->u[m * D + a] + 0.5 * s->dt * U[a];
      /* the Maxwell branch commits the deformation this collision used (the
       * repaired one on a projection step); the cut-link closures of the
       * step, which follow, see the advanced history (reading) */
      if (s->Qh) visco_commit(D, &mat, U + D, s->Qh + (size_t)m * D * D, s->S0h + (size_t)m * D * D);
    }
    if (proj) {
      /* second displacement projection with the repaired F; the history reset
       * u* = u^c + dt/2 v advances the reset displacement as the collision
       * loop does (reading of the sign in Algorithm 1) */
      int *anc_n;
      double *anc_s;
      proj_anchors(s, s->U, tn, &anc_n, &anc_s);
      s->st_cg_it += proj_solve(s, s->U, s->u, PROJ_RTOL, anc_n, anc_s);
      free(anc_n);
      free(anc_s);
#pragma omp parallel for
      for (int64_t m = 0; m < s->N; ++m) {
        if (!s->act[m]) continue;
        for (int a = 0; a < D; ++a)
          s->ustar[m * D + a] = s->u[m * D + a] + 0.5 * s->dt * s->U[(size_t)m * M + a];
      }
    }
    /* streaming on interior links (Eq. 31) */
#pragma omp parallel for
    for (int64_t m = 0; m < s->N; ++m) {
      if (!s->act[m]) continue;
      for (int q = 0; q < Q; ++q) {
        int64_t l = nbr_q(s, m, q, 1);
        if (!s->act[l]) continue;
        memcpy(s->f + (size_t)l * Q * M + q * M, s->fs + (size_t)m * Q * M + q * M,
               sizeof(double) * M);
      }
    }
    /* cut-link reconstruction */
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t l = 0; l < s->nl; ++l)
      if (close_link(s, &s->links[l], tn) < 0) bad = 1;
    s->step++;
    if (bad) {
      s->status = ORC_ERR_NEWTON;
      return ORC_ERR_NEWTON;
    }
  }
  return ORC_OK;
}

int orc_moments(orc_sim *s, double *Uo, double *uo, double *Jo) {
  int D = s->D, M = s->M;
  if (!s->have_state) return ORC_ERR_ORDER;
  int st = recover(s);
  for (int64_t i = 0; i < s->N; ++i) {
    const double *U = s->U + (size_t)i * M;
    int a = s->act[i];
    if (Uo)
      for (int r = 0; r < M; ++r) Uo[(size_t)r * s->N + i] = a ? U[r] : 0.0;
    if (uo)
      for (int k = 0; k < D; ++k) uo[(size_t)k * s->N + i] = a ? s->u[i * D + k] : 0.0;
    if (Jo) Jo[i] = a ? det_n(D, U + D) : 0.0;
  }
  return st;
}

/* stress of the current state at every active node: P = P(F) with the
 * node's law (and the history of the Maxwell branch as the next collision
 * would use it), sigma = J^{-1} P F^T (Sec. 2.4, Eq. 35); planar [D*D][N],
 * zero at inactive nodes; either may be NULL */
int orc_stress(orc_sim *s, double *Po, double *So) {
  int D = s->D, M = s->M;
  if (!s->have_state) return ORC_ERR_ORDER;
  int st = recover(s);
  for (int64_t i = 0; i < s->N; ++i) {
    double P[9] = {0.0}, sg[9] = {0.0};
    if (s->act[i]) {
      const double *F = s->U + (size_t)i * M + D;
      const orc_mat mat = sim_mat(s, s->mu, s->lam, i);
      if (mat_piola(D, &mat, F, P)) st = st ? st : ORC_ERR_J;
      double J = det_n(D, F);
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          double acc = 0.0;
          for (int A = 0; A < D; ++A) acc += P[a * D + A] * F[b * D + A];
          sg[a * D + b] = acc / J;
        }
    }
    for (int k = 0; k < D * D; ++k) {
      if (Po) Po[(size_t)k * s->N + i] = P[k];
      if (So) So[(size_t)k * s->N + i] = sg[k];
    }
  }
  return st;
}

int orc_get_f(orc_sim *s, double *fo) {
  int M = s->M, Q = s->Q;
  for (int64_t i = 0; i < s->N; ++i)
    for (int q = 0; q < Q; ++q)
      for (int r = 0; r < M; ++r)
        fo[((size_t)q * M + r) * s->N + i] = s->act[i] ? s->f[(size_t)i * Q * M + q * M + r] : 0.0;
  return ORC_OK;
}

int orc_put_f(orc_sim *s, const double *fi, const double *ustar, int64_t step) {
  int M = s->M, Q = s->Q, D = s->D;
  if (alloc_fields(s)) return ORC_ERR_MEM;
  for (int64_t i = 0; i < s->N; ++i) {
    for (int q = 0; q < Q; ++q)
      for (int r = 0; r < M; ++r)
        s->f[(size_t)i * Q * M + q * M + r] = fi[((size_t)q * M + r) * s->N + i];
    for (int a = 0; a < D; ++a) s->ustar[i * D + a] = ustar ? ustar[(size_t)a * s->N + i] : 0.0;
  }
  s->step = step;
  s->init_step = -1;
  s->have_state = 1;
  s->status = ORC_OK;
  return ORC_OK;
}

int64_t orc_num_active(orc_sim *s) {
  int64_t c = 0;
  for (int64_t i = 0; i < s->N; ++i) c += s->act[i];
  return c;
}

int64_t orc_num_links(orc_sim *s) { return s->nl; }

int orc_get_links(orc_sim *s, int64_t *node, int32_t *q, double *eta, double *Nb, int32_t *bid) {
  for (int64_t l = 0; l < s->nl; ++l) {
    const orc_link *L = &s->links[l];
    if (node) node[l] = L->m;
    if (q) q[l] = L->q;
    if (eta) eta[l] = L->eta;
    if (Nb)
      for (int a = 0; a < 3; ++a) Nb[l * 3 + a] = a < s->D ? L->N[a] : 0.0;
    if (bid) bid[l] = L->bid;
  }
  return ORC_OK;
}

void orc_stats(orc_sim *s, int64_t *st) {
  st[0] = s->st_newton_it;
  st[1] = s->st_newton_fail;
  st[2] = s->st_cg_it;
  st[3] = s->st_proj;
  st[4] = s->step;
  st[5] = s->status;
}

int orc_project(orc_sim *s, const double *F, double *u, double rtol, int64_t *iters) {
  int D = s->D, M = s->M;
  double *Unm = (double *)calloc((size_t)s->N * M, sizeof(double));
  double *uu = (double *)malloc(sizeof(double) * (size_t)s->N * D);
  for (int64_t i = 0; i < s->N; ++i) {
    for (int k = 0; k < D * D; ++k) Unm[(size_t)i * M + D + k] = F[(size_t)k * s->N + i];
    for (int a = 0; a < D; ++a) uu[i * D + a] = u[(size_t)a * s->N + i];
  }
  int64_t its = proj_solve(s, Unm, uu, rtol, NULL, NULL);
  if (iters) *iters = its;
  for (int64_t i = 0; i < s->N; ++i)
    for (int a = 0; a < D; ++a) u[(size_t)a * s->N + i] = uu[i * D + a];
  free(Unm);
  free(uu);
  return ORC_OK;
}

/* the same projection with the anchors of the Dirichlet cut links at time t
 * (the relation u^c_m + (F_m - I)(X_b - X_m) = u_D(X_b, t) per link), as the
 * step applies it */
int orc_project_anchored(orc_sim *s, const double *F, double *u, double t, double rtol, int64_t *iters) {
  int D = s->D, M = s->M;
  double *Unm = (double *)calloc((size_t)s->N * M, sizeof(double));
  double *uu = (double *)malloc(sizeof(double) * (size_t)s->N * D);
  for (int64_t i = 0; i < s->N; ++i) {
    for (int k = 0; k < D * D; ++k) Unm[(size_t)i * M + D + k] = F[(size_t)k * s->N + i];
    for (int a = 0; a < D; ++a) uu[i * D + a] = u[(size_t)a * s->N + i];
  }
  int *anc_n;
  double *anc_s;
  proj_anchors(s, Unm, t, &anc_n, &anc_s);
  int64_t its = proj_solve(s, Unm, uu, rtol, anc_n, anc_s);
  free(anc_n);
  free(anc_s);
  if (iters) *iters = its;
  for (int64_t i = 0; i < s->N; ++i)
    for (int a = 0; a < D; ++a) u[(size_t)a * s->N + i] = uu[i * D + a];
  free(Unm);
  free(uu);
  return ORC_OK;
}

int orc_compatible_F(orc_sim *s, const double *u, const double *F, double *Fc) {
  int D = s->D, M = s->M;
  double *Unm = (double *)calloc((size_t)s->N * M, sizeof(double));
  double *uu = (double *)malloc(sizeof(double) * (size_t)s->N * D);
  double *Fcn = (double *)calloc((size_t)s->N * D * D, sizeof(double));
  for (int64_t i = 0; i < s->N; ++i) {
    for (int k = 0; k < D * D; ++k) Unm[(size_t)i * M + D + k] = F[(size_t)k * s->N + i];
    for (int a = 0; a < D; ++a) uu[i * D + a] = u[(size_t)a * s->N + i];
  }
  compat_F(s, uu, Unm, Fcn);
  for (int64_t i = 0; i < s->N; ++i)
    for (int k = 0; k < D * D; ++k) Fc[(size_t)k * s->N + i] = s->act[i] ? Fcn[(size_t)i * D * D + k] : 0.0;
  free(Unm);
  free(uu);
  free(Fcn);
  return ORC_OK;
}

/* post-collision populations f* of the last completed step, [Q][M][N] */
int orc_get_fs(orc_sim *s, double *fo) {
  int M = s->M, Q = s->Q;
  if (!s->fs) return ORC_ERR_ORDER;
  for (int64_t i = 0; i < s->N; ++i)
    for (int q = 0; q < Q; ++q)
      for (int r = 0; r < M; ++r)
        fo[((size_t)q * M + r) * s->N + i] = s->act[i] ? s->fs[(size_t)i * Q * M + q * M + r] : 0.0;
  return ORC_OK;
}

/* number of OpenMP threads the oracle runs with */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ======================================================================== */
/* Reverse mode (project extension: the paper has no adjoint)               */
/* ======================================================================== */
/* Gradient of a linear functional of the moments after nsteps steps,
 *   L = sum_m dLdU(m) . U(m) + dLdu(m) . u(m),
 * with respect to the material parameters (mu, lambda), the initial velocity
 * v0 and the initial displacement u0 given to orc_set_state, by the discrete
 * adjoint of orc_step.  Written to be checked by eye, not to be fast:
 *  - the transpose of every nonlinear point map is formed column by column
 *    from its tangent (the JVP applied to unit vectors);
 *  - the Piola map and the equilibrium are linear in (mu, lambda) and the
 *    second-order initialisation is quadratic in them, so a central
 *    difference with unit step gives their parameter derivatives exactly (up
 *    to rounding); the initialisation is affine in v0, so a unit difference
 *    gives its v0 derivative;
 *  - the forward trajectory is stored whole and each step is recomputed by
 *    the forward code itself;
 *  - the projection's CG solve is differentiated as the exact solution map
 *    x = x0 + K^+ (b - K x0) of a warm-started CG on the semi-definite
 *    normal matrix K (graph Laplacian + anchors): b_bar = K^+ x_bar and
 *    x0_bar = (I - K K^+) x_bar, the projection onto the constants of the
 *    connected components without anchors. */

/* out[r] = sum_{q,s} lam[q*M+s] d feq_{q,s} / d U_r */
static void feq_vjp(const orc_sim *s, double mu, double lam, const double *U, const double *lq,
                    double *out) {
  int M = s->M, Q = s->Q;
  for (int r = 0; r < M; ++r) {
    double e[MAXM] = {0}, d[MAXQ * MAXM], acc = 0.0;
    e[r] = 1.0;
    const orc_mat mat = sim_mat(s, mu, lam, -1);
    feq_jvp_m(s->D, s->c, &mat, s->rho0, U, e, d);
    for (int k = 0; k < Q * M; ++k) acc += lq[k] * d[k];
    out[r] = acc;
  }
}

/* sum_k lq[k] d feq_k / d(mu, lambda), by the exact unit central difference */
static void feq_dp(const orc_sim *s, const double *U, const double *lq, double *g) {
  int QM = s->Q * s->M;
  double a[MAXQ * MAXM], b[MAXQ * MAXM];
  orc_feq(s->D, s->c, s->mu + 1.0, s->lam, s->rho0, U, a);
  orc_feq(s->D, s->c, s->mu - 1.0, s->lam, s->rho0, U, b);
  double gm = 0.0, gl = 0.0;
  for (int k = 0; k < QM; ++k) gm += lq[k] * 0.5 * (a[k] - b[k]);
  orc_feq(s->D, s->c, s->mu, s->lam + 1.0, s->rho0, U, a);
  orc_feq(s->D, s->c, s->mu, s->lam - 1.0, s->rho0, U, b);
  for (int k = 0; k < QM; ++k) gl += lq[k] * 0.5 * (a[k] - b[k]);
  g[0] += gm;
  g[1] += gl;
}

/* W : dP/dF as a matrix: out_kB = sum_iA W_iA dP_iA/dF_kB */
static void piola_vjp(int D, const orc_mat *m, const double *F, const double *W, double *out) {
  for (int k = 0; k < D * D; ++k) {
    double E[9] = {0}, dP[9], acc = 0.0;
    E[k] = 1.0;
    mat_piola_jvp(D, m, F, E, dP);
    for (int j = 0; j < D * D; ++j) acc += W[j] * dP[j];
    out[k] = acc;
  }
}

/* W : dP/d(mu, lambda), exact unit central difference (the fibre term does
 * not depend on mu, lambda) */
static void piola_dp(int D, double mu, double lam, const double *F, const double *W, double *g) {
  double a[9], b[9], gm = 0.0, gl = 0.0;
  orc_piola(D, mu + 1.0, lam, F, a);
  orc_piola(D, mu - 1.0, lam, F, b);
  for (int k = 0; k < D * D; ++k) gm += W[k] * 0.5 * (a[k] - b[k]);
  orc_piola(D, mu, lam + 1.0, F, a);
  orc_piola(D, mu, lam - 1.0, F, b);
  for (int k = 0; k < D * D; ++k) gl += W[k] * 0.5 * (a[k] - b[k]);
  g[0] += gm;
  g[1] += gl;
}

/* K x = graph Laplacian + anchor diagonal (the forward solve's matrix) */
static void apply_K(const orc_sim *s, const int *anc_n, const double *x, double *y) {
  graph_lap(s, x, y);
  if (anc_n)
    for (int64_t m = 0; m < s->N; ++m) y[m] += anc_n[m] * x[m];
}

/* y = K^+ rhs for rhs orthogonal to the null space of K (plain CG from 0) */
static void cg_pinv(const orc_sim *s, const int *anc_n, const double *rhs, double *y) {
  int64_t N = s->N, nact = 0;
  double *r = (double *)malloc(sizeof(double) * N), *p = (double *)malloc(sizeof(double) * N);
  double *Ap = (double *)malloc(sizeof(double) * N);
  for (int64_t m = 0; m < N; ++m) {
    nact += s->act[m];
    y[m] = 0.0;
    r[m] = s->act[m] ? rhs[m] : 0.0;
    p[m] = r[m];
  }
  double rr = dot_act(s, r, r), thr = 1e-30 * rr;
  for (int64_t k = 0; k < 10 * nact + 100 && rr > thr; ++k) {
    apply_K(s, anc_n, p, Ap);
    double pAp = dot_act(s, p, Ap);
    if (!(pAp > 0.0)) break;
    double alpha = rr / pAp;
    for (int64_t m = 0; m < N; ++m) {
      y[m] += alpha * p[m];
      r[m] -= alpha * Ap[m];
    }
    double rr2 = dot_act(s, r, r), beta = rr2 / rr;
    rr = rr2;
    for (int64_t m = 0; m < N; ++m) p[m] = r[m] + beta * p[m];
  }
  free(r); free(p); free(Ap);
}

/* connected components of the active graph; anch[c] = 1 when a node of
 * component c carries an anchor */
static int64_t components(const orc_sim *s, const int *anc_n, int64_t *comp, uint8_t **anch) {
  int64_t N = s->N, nc = 0;
  int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (N ? N : 1));
  for (int64_t m = 0; m < N; ++m) comp[m] = -1;
  for (int64_t m0 = 0; m0 < N; ++m0) {
    if (!s->act[m0] || comp[m0] >= 0) continue;
    int64_t top = 0;
    stack[top++] = m0;
    comp[m0] = nc;
    while (top) {
      int64_t m = stack[--top];
      for (int q = 0; q < s->Q; ++q) {
        int64_t l = nbr_q(s, m, q, 1);
        if (l >= 0 && s->act[l] && comp[l] < 0) {
          comp[l] = nc;
          stack[top++] = l;
        }
      }
    }
    ++nc;
  }
  free(stack);
  *anch = (uint8_t *)calloc(nc ? nc : 1, 1);
  if (anc_n)
    for (int64_t m = 0; m < N; ++m)
      if (s->act[m] && anc_n[m]) (*anch)[comp[m]] = 1;
  return nc;
}

/* adjoint of u = x0 + K^+ (b - K x0) per component of u ([N][D]):
 * y = K^+ ubar (the b adjoint), x0bar = ubar - K y */
static void solve_adj(const orc_sim *s, const int *anc_n, const int64_t *comp, const uint8_t *anch,
                      int64_t nc, const double *ubar, double *y, double *x0bar) {
  int D = s->D;
  int64_t N = s->N;
  double *rhs = (double *)malloc(sizeof(double) * N), *yc = (double *)malloc(sizeof(double) * N);
  double *sum = (double *)calloc(nc ? nc : 1, sizeof(double));
  int64_t *cnt = (int64_t *)calloc(nc ? nc : 1, sizeof(int64_t));
  for (int64_t m = 0; m < N; ++m)
    if (s->act[m]) cnt[comp[m]]++;
  for (int i = 0; i < D; ++i) {
    for (int64_t c = 0; c < nc; ++c) sum[c] = 0.0;
    for (int64_t m = 0; m < N; ++m)
      if (s->act[m]) sum[comp[m]] += ubar[m * D + i];
    for (int64_t m = 0; m < N; ++m) {
      double pm = 0.0; /* projection onto the null space of K */
      if (s->act[m] && !anch[comp[m]]) pm = sum[comp[m]] / (double)cnt[comp[m]];
      rhs[m] = s->act[m] ? ubar[m * D + i] - pm : 0.0;
      x0bar[m * D + i] = pm;
    }
    cg_pinv(s, anc_n, rhs, yc);
    for (int64_t m = 0; m < N; ++m) y[m * D + i] = yc[m];
  }
  free(rhs); free(yc); free(sum); free(cnt);
}

/* adjoint of proj_jacobi per component of u ([N][D]): the sweep
 * x' = x + w Dg^-1 (b - K x) has the transpose  xbar = (I - w K Dg^-1) x'bar,
 * bbar += w Dg^-1 x'bar (K symmetric); y receives bbar, x0bar the adjoint of
 * the starting displacement */
static void jacobi_adj(const orc_sim *s, const int *anc_n, const double *ubar, double *y, double *x0bar) {
  int D = s->D;
  int64_t N = s->N;
  double *z = (double *)malloc(sizeof(double) * N), *w = (double *)malloc(sizeof(double) * N);
  double *Kw = (double *)malloc(sizeof(double) * N);
  for (int i = 0; i < D; ++i) {
    for (int64_t m = 0; m < N; ++m) {
      z[m] = s->act[m] ? ubar[m * D + i] : 0.0;
      y[m * D + i] = 0.0;
    }
    for (int k = 0; k < s->proj_sweeps; ++k) {
      for (int64_t m = 0; m < N; ++m) {
        double d = s->act[m] ? proj_diag(s, anc_n, m) : 0.0;
        w[m] = d > 0.0 ? z[m] / d : 0.0;
        y[m * D + i] += s->proj_weight * w[m];
      }
      apply_K(s, anc_n, w, Kw);
      for (int64_t m = 0; m < N; ++m)
        if (s->act[m]) z[m] -= s->proj_weight * Kw[m];
    }
    for (int64_t m = 0; m < N; ++m) x0bar[m * D + i] = s->act[m] ? z[m] : 0.0;
  }
  free(z); free(w); free(Kw);
}

/* transpose of proj_rhs: Fbar[m*D*D + i*D + A] += d b / d F_m,iA applied to y */
static void proj_rhs_T(const orc_sim *s, const double *y, double *Fbar) {
  int D = s->D;
  for (int64_t m = 0; m < s->N; ++m) {
    if (!s->act[m]) continue;
    for (int A = 0; A < D; ++A) {
      int64_t lp = nbr_q(s, m, 2 * A, 1), lm = nbr_q(s, m, 2 * A + 1, 1);
      for (int i = 0; i < D; ++i) {
        double w = 0.5 * s->dx * y[m * D + i];
        if (lm >= 0 && s->act[lm]) {
          Fbar[(size_t)m * D * D + i * D + A] += w;
          Fbar[(size_t)lm * D * D + i * D + A] += w;
        }
        if (lp >= 0 && s->act[lp]) {
          Fbar[(size_t)m * D * D + i * D + A] -= w;
          Fbar[(size_t)lp * D * D + i * D + A] -= w;
        }
      }
    }
  }
}

/* transpose of the F dependence of proj_anchors' target sums */
static void anchors_T(const orc_sim *s, const double *y, double *Fbar) {
  int D = s->D;
  for (int64_t l = 0; l < s->nl; ++l) {
    const orc_link *L = &s->links[l];
    if (s->bc[L->bid].type != ORC_BC_DIRICHLET) continue;
    int A = L->q / 2, sg = e_of(L->q, A);
    double off = sg * L->eta * s->dx;
    for (int i = 0; i < D; ++i) Fbar[(size_t)L->m * D * D + i * D + A] -= off * y[L->m * D + i];
  }
}

/* transpose of compat_F: u-part into ubar, kept columns into Fbar */
static void compat_F_T(const orc_sim *s, const double *Fcbar, double *ubar, double *Fbar) {
  int D = s->D;
  for (int64_t m = 0; m < s->N; ++m) {
    if (!s->act[m]) continue;
    for (int A = 0; A < D; ++A) {
      int64_t lp = nbr_q(s, m, 2 * A, 1), lm = nbr_q(s, m, 2 * A + 1, 1);
      int hp = (lp >= 0 && s->act[lp]), hm = (lm >= 0 && s->act[lm]);
      for (int i = 0; i < D; ++i) {
        double g = Fcbar[(size_t)m * D * D + i * D + A];
        if (hp && hm) {
          ubar[lp * D + i] += g / (2.0 * s->dx);
          ubar[lm * D + i] -= g / (2.0 * s->dx);
        } else if (hp) {
          ubar[lp * D + i] += g / s->dx;
          ubar[m * D + i] -= g / s->dx;
        } else if (hm) {
          ubar[m * D + i] += g / s->dx;
          ubar[lm * D + i] -= g / s->dx;
        } else {
          Fbar[(size_t)m * D * D + i * D + A] += g;
        }
      }
    }
  }
}

/* adjoint of one Neumann link's source S (Eqs. 46-47 with the F_b of
 * neumann_Fb) given Sbar; accumulates into ubar ([N][D]) and gmat */
static void neumann_adj(orc_sim *s, const orc_link *L, double th, const double *Sbar, double *ubar,
                        double *gmat) {
  int D = s->D;
  int qo = L->q, A0 = qo / 2, sg = e_of(qo, A0);
  double d[3] = {0, 0, 0};
  d[A0] = -sg;
  double Gt[9], Fb[9], W[9], Fbb[9], hb[3], Qm[9], z[3], Gtb[9];
  neumann_Fb(s, L, th, 0, Gt, Fb);
  /* S^v_i = -sum_B d_B P_iB / (rho0 c), S^F_iB = F_b,iB / D */
  for (int i = 0; i < D; ++i)
    for (int B = 0; B < D; ++B) W[i * D + B] = -Sbar[i] * d[B] / (s->rho0 * s->c);
  const orc_mat mat = sim_mat(s, s->mu, s->lam, -1);
  piola_vjp(D, &mat, Fb, W, Fbb);
  for (int k = 0; k < D * D; ++k) Fbb[k] += Sbar[D + k] / D;
  piola_dp(D, s->mu, s->lam, Fb, W, gmat);
  /* F_b = h (x) N + Gt : h_bar = Fb_bar N, Gt_bar = Fb_bar */
  for (int i = 0; i < D; ++i) {
    double acc = 0.0;
    for (int B = 0; B < D; ++B) acc += Fbb[i * D + B] * L->N[B];
    hb[i] = acc;
  }
  /* implicit function theorem on R(h, Gt, p) = P(F_b) N - T = 0:
   * z = Q^{-T} h_bar, Gt_bar -= (dR/dGt)^T z, p_bar -= (dR/dp)^T z */
  for (int k = 0; k < D; ++k) {
    double dF[9], dP[9];
    for (int i = 0; i < D; ++i)
      for (int A = 0; A < D; ++A) dF[i * D + A] = (i == k ? 1.0 : 0.0) * L->N[A];
    mat_piola_jvp(D, &mat, Fb, dF, dP);
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int A = 0; A < D; ++A) acc += dP[i * D + A] * L->N[A];
      Qm[k * D + i] = acc; /* row k of Q^T */
    }
  }
  if (!gauss_solve(D, Qm, hb, z)) return;
  double zN[9], gz[2] = {0.0, 0.0};
  for (int i = 0; i < D; ++i)
    for (int A = 0; A < D; ++A) zN[i * D + A] = z[i] * L->N[A];
  piola_vjp(D, &mat, Fb, zN, Gtb);
  for (int k = 0; k < D * D; ++k) Gtb[k] = Fbb[k] - Gtb[k];
  piola_dp(D, s->mu, s->lam, Fb, zN, gz);
  gmat[0] -= gz[0];
  gmat[1] -= gz[1];
  /* Gt = sum_a g_a (x) t_a, g_a = t_a + sum_k w_a,k u_pts(k) */
  for (int al = 0; al < D - 1; ++al) {
    double gb[3];
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int B = 0; B < D; ++B) acc += Gtb[i * D + B] * L->t[al][B];
      gb[i] = acc;
    }
    for (int k = 0; k < L->npts; ++k)
      for (int i = 0; i < D; ++i) ubar[L->pts[k] * D + i] += L->w[al * L->npts + k] * gb[i];
  }
}

int orc_adjoint(orc_sim *s, int64_t nsteps, const double *dLdU, const double *dLdu, double *grad_mat,
                double *grad_v0, double *grad_u0, double *grad_dU0) {
  int D = s->D, M = s->M, Q = s->Q;
  int64_t N = s->N;
  if (!s->have_state || s->init_step != s->step || !s->U0) return ORC_ERR_ORDER;
  if (s->status) return s->status;
  if (nsteps < 0 || s->Qh || s->th) return ORC_ERR_ARG; /* no reverse mode through a branch or a stretch */
  int has_neu = 0, has_dir = 0;
  for (int64_t l = 0; l < s->nl; ++l) {
    int t = s->bc[s->links[l].bid].type;
    if (t == ORC_BC_NEUMANN) has_neu = 1;
    if (t == ORC_BC_DIRICHLET) has_dir = 1;
  }
  const size_t nf = (size_t)N * Q * M, nd = (size_t)N * D;
  const int64_t k0 = s->step;
  /* forward trajectory X^k = (f^k, u*^k), k = k0 .. k0 + nsteps - 1 */
  double *trf = (double *)malloc(sizeof(double) * nf * (nsteps ? nsteps : 1));
  double *trs = (double *)malloc(sizeof(double) * nd * (nsteps ? nsteps : 1));
  if (!trf || !trs) {
    free(trf); free(trs);
    return ORC_ERR_MEM;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    memcpy(trf + nf * k, s->f, sizeof(double) * nf);
    memcpy(trs + nd * k, s->ustar, sizeof(double) * nd);
    int st = orc_step(s, 1);
    if (st) {
      free(trf); free(trs);
      return st;
    }
  }
  double *lf = (double *)calloc(nf, sizeof(double)), *lfs = (double *)calloc(nf, sizeof(double));
  double *lus = (double *)calloc(nd, sizeof(double)), *ub = (double *)calloc(nd, sizeof(double));
  double *ubc = (double *)calloc(nd, sizeof(double)), *y = (double *)calloc(nd, sizeof(double));
  double *x0b = (double *)calloc(nd, sizeof(double));
  double *Ua = (double *)calloc((size_t)N * M, sizeof(double)), *Ur = (double *)calloc((size_t)N * M, sizeof(double));
  double *Fcb = (double *)calloc((size_t)N * D * D, sizeof(double));
  double *Frb = (double *)calloc((size_t)N * D * D, sizeof(double));
  double *Uab = (double *)calloc((size_t)N * M, sizeof(double));
  int64_t *comp = (int64_t *)malloc(sizeof(int64_t) * N);
  uint8_t *anch = NULL;
  int64_t nc = 0;
  double gmat[2] = {0.0, 0.0};
  const double kap = 1.0 + 0.5 * s->gamma * s->dt, sig = s->dt * (2.0 - s->omega) / (4.0 * D);
  /* seeds: U = R(f) with v = sum f^v / kappa, u = u* + dt/2 v */
  for (int64_t m = 0; m < N; ++m) {
    if (!s->act[m]) continue;
    for (int r = 0; r < M; ++r) {
      double g = dLdU ? dLdU[(size_t)r * N + m] : 0.0;
      if (r < D && dLdu) g += 0.5 * s->dt * dLdu[(size_t)r * N + m];
      if (r < D) g /= kap;
      for (int q = 0; q < Q; ++q) lf[(size_t)m * Q * M + q * M + r] = g;
    }
    for (int a = 0; a < D; ++a) lus[m * D + a] = dLdu ? dLdu[(size_t)a * N + m] : 0.0;
  }
  /* anchor counts depend on the links only (the targets are not needed) */
  int *an = NULL;
  {
    double *as = NULL;
    if (has_dir) proj_anchors(s, s->U, 0.0, &an, &as);
    free(as);
    nc = components(s, an, comp, &anch);
  }
  int status = ORC_OK;
  for (int64_t k = nsteps - 1; k >= 0 && !status; --k) {
    const int64_t stp = k0 + k;
    const double th = stp * s->dt + 0.5 * s->dt;
    const int proj = has_neu && s->proj_every > 0 && (stp % s->proj_every == 0);
    /* recompute step stp */
    memcpy(s->f, trf + nf * k, sizeof(double) * nf);
    memcpy(s->ustar, trs + nd * k, sizeof(double) * nd);
    s->step = stp;
    recover(s);
    memcpy(Ua, s->U, sizeof(double) * N * M);
    memcpy(s->f, trf + nf * k, sizeof(double) * nf);
    s->step = stp;
    status = orc_step(s, 1); /* s->fs, s->u (closure input), s->U (U^r) */
    if (status) break;
    memcpy(Ur, s->U, sizeof(double) * N * M);
    /* streaming transpose: fs(m, q) went to f(m + e_q, q) */
    memset(lfs, 0, sizeof(double) * nf);
    for (int64_t m = 0; m < N; ++m) {
      if (!s->act[m]) continue;
      for (int q = 0; q < Q; ++q) {
        int64_t l = nbr_q(s, m, q, 1);
        if (!s->act[l]) continue;
        for (int r = 0; r < M; ++r)
          lfs[(size_t)m * Q * M + q * M + r] += lf[(size_t)l * Q * M + q * M + r];
      }
    }
    /* cut-link transpose (Eqs. 42-47) */
    memset(ubc, 0, sizeof(double) * nd);
    for (int64_t l = 0; l < s->nl; ++l) {
      const orc_link *L = &s->links[l];
      const orc_bc *b = &s->bc[L->bid];
      int qo = L->q, qi = qo ^ 1;
      const double *ln = lf + (size_t)L->m * Q * M + qi * M;
      double Dsign[MAXM], Sb[MAXM], eta = L->eta;
      for (int r = 0; r < M; ++r) {
        int vrow = r < D;
        Dsign[r] = (b->type == ORC_BC_DIRICHLET) ? (vrow ? -1.0 : 1.0) : (vrow ? 1.0 : -1.0);
      }
      for (int r = 0; r < M; ++r) {
        double g = ln[r];
        if (eta >= 0.5) {
          lfs[(size_t)L->m * Q * M + qo * M + r] += Dsign[r] / (2.0 * eta) * g;
          lfs[(size_t)L->m * Q * M + qi * M + r] += (1.0 - 1.0 / (2.0 * eta)) * g;
          Sb[r] = g / (2.0 * eta);
        } else {
          lfs[(size_t)L->m * Q * M + qo * M + r] += Dsign[r] * 2.0 * eta * g;
          lfs[(size_t)L->mminus * Q * M + qo * M + r] += Dsign[r] * (1.0 - 2.0 * eta) * g;
          Sb[r] = g;
        }
      }
      if (b->type == ORC_BC_NEUMANN) neumann_adj(s, L, th, Sb, ubc, gmat);
    }
    /* collision, displacement history and (on projection steps) repair and
     * projections, in reverse */
    memset(Uab, 0, sizeof(double) * N * M);
    if (!proj) {
      for (size_t k2 = 0; k2 < nd; ++k2) ub[k2] = ubc[k2] + lus[k2];
#pragma omp parallel
      {
        double gl[2] = {0.0, 0.0};
#pragma omp for
        for (int64_t m = 0; m < N; ++m) {
          if (!s->act[m]) continue;
          const double *U = Ua + (size_t)m * M, *ls = lfs + (size_t)m * Q * M;
          double yv[MAXM], *Ub = Uab + (size_t)m * M;
          feq_vjp(s, s->mu, s->lam, U, ls, yv);
          feq_dp(s, U, ls, gl);
          for (int r = 0; r < M; ++r) {
            double src = 0.0;
            if (r < D)
              for (int q = 0; q < Q; ++q) src += -s->gamma * ls[q * M + r];
            Ub[r] = s->omega * yv[r] + sig * src;
          }
          for (int a = 0; a < D; ++a) Ub[a] += 0.5 * s->dt * (lus[m * D + a] + ub[m * D + a]);
        }
#pragma omp critical
        {
          gmat[0] += s->omega * gl[0];
          gmat[1] += s->omega * gl[1];
        }
      }
      for (int64_t m = 0; m < N; ++m)
        for (int q = 0; q < Q; ++q)
          for (int r = 0; r < M; ++r) {
            size_t o = (size_t)m * Q * M + q * M + r;
            lf[o] = s->act[m] ? (1.0 - s->omega) * lfs[o] : 0.0;
          }
    } else {
      /* second solve: u^cc = solve(F^r, warm start u^c); u* = u^cc + dt/2 v */
      for (size_t k2 = 0; k2 < nd; ++k2) ub[k2] = ubc[k2] + lus[k2];
      if (s->proj_sweeps > 0) jacobi_adj(s, an, ub, y, x0b);
      else solve_adj(s, an, comp, anch, nc, ub, y, x0b);
      memset(Frb, 0, sizeof(double) * (size_t)N * D * D);
      proj_rhs_T(s, y, Frb);
      if (an) anchors_T(s, y, Frb);
      memcpy(ubc, x0b, sizeof(double) * nd); /* u^c adjoint so far */
      memset(Fcb, 0, sizeof(double) * (size_t)N * D * D);
      double gl[2] = {0.0, 0.0}, gr[2] = {0.0, 0.0};
      for (int64_t m = 0; m < N; ++m) {
        if (!s->act[m]) continue;
        const double *U = Ua + (size_t)m * M, *UR = Ur + (size_t)m * M;
        double *ls = lfs + (size_t)m * Q * M, *l1 = lf + (size_t)m * Q * M;
        double yv[MAXM], Urb[MAXM], *Ub = Uab + (size_t)m * M;
        /* collision with U^r */
        feq_vjp(s, s->mu, s->lam, UR, ls, yv);
        feq_dp(s, UR, ls, gl);
        for (int r = 0; r < M; ++r) {
          double src = 0.0;
          if (r < D)
            for (int q = 0; q < Q; ++q) src += -s->gamma * ls[q * M + r];
          Urb[r] = s->omega * yv[r] + sig * src;
        }
        for (int a = 0; a < D; ++a) Urb[a] += 0.5 * s->dt * lus[m * D + a];
        for (int k2 = 0; k2 < D * D; ++k2) Urb[D + k2] += Frb[(size_t)m * D * D + k2];
        for (int k2 = 0; k2 < Q * M; ++k2) l1[k2] = (1.0 - s->omega) * ls[k2];
        /* repair f' = f + feq(U^r) - feq(U) (Eq. 61) */
        feq_vjp(s, s->mu, s->lam, UR, l1, yv);
        for (int r = 0; r < M; ++r) Urb[r] += yv[r];
        feq_vjp(s, s->mu, s->lam, U, l1, yv);
        for (int r = 0; r < M; ++r) Ub[r] -= yv[r];
        feq_dp(s, UR, l1, gr);
        {
          double gneg[2] = {0.0, 0.0};
          feq_dp(s, U, l1, gneg);
          gr[0] -= gneg[0];
          gr[1] -= gneg[1];
        }
        /* U^r = (v, (1 - theta) F + theta F^c) */
        for (int a = 0; a < D; ++a) Ub[a] += Urb[a];
        for (int k2 = 0; k2 < D * D; ++k2) {
          Ub[D + k2] += (1.0 - s->theta) * Urb[D + k2];
          Fcb[(size_t)m * D * D + k2] = s->theta * Urb[D + k2];
        }
      }
      gmat[0] += s->omega * gl[0] + gr[0];
      gmat[1] += s->omega * gl[1] + gr[1];
      /* F^c = compat(u^c, F) */
      memset(Frb, 0, sizeof(double) * (size_t)N * D * D);
      compat_F_T(s, Fcb, ubc, Frb);
      /* first solve: u^c = solve(F, warm start u) */
      if (s->proj_sweeps > 0) jacobi_adj(s, an, ubc, y, x0b);
      else solve_adj(s, an, comp, anch, nc, ubc, y, x0b);
      proj_rhs_T(s, y, Frb);
      if (an) anchors_T(s, y, Frb);
      for (int64_t m = 0; m < N; ++m) {
        if (!s->act[m]) continue;
        for (int k2 = 0; k2 < D * D; ++k2) Uab[(size_t)m * M + D + k2] += Frb[(size_t)m * D * D + k2];
        for (int a = 0; a < D; ++a) {
          ub[m * D + a] = x0b[m * D + a];
          Uab[(size_t)m * M + a] += 0.5 * s->dt * ub[m * D + a];
        }
      }
    }
    /* recovery transpose: U = R(f), v = sum f^v / kappa; u = u* + dt/2 v */
    for (int64_t m = 0; m < N; ++m) {
      if (!s->act[m]) continue;
      for (int r = 0; r < M; ++r) {
        double g = Uab[(size_t)m * M + r];
        if (r < D) g /= kap;
        for (int q = 0; q < Q; ++q) lf[(size_t)m * Q * M + q * M + r] += g;
      }
      for (int a = 0; a < D; ++a) lus[m * D + a] = ub[m * D + a];
    }
  }
  /* initialisation transpose (Eqs. 32-33) and u*^0 = u0 - dt/2 v0 */
  if (!status) {
    double gi[2] = {0.0, 0.0};
    for (int64_t m = 0; m < N; ++m) {
      if (grad_v0)
        for (int a = 0; a < D; ++a) grad_v0[(size_t)a * N + m] = 0.0;
      if (grad_u0)
        for (int a = 0; a < D; ++a) grad_u0[(size_t)a * N + m] = 0.0;
      if (grad_dU0)
        for (int k2 = 0; k2 < D * M; ++k2) grad_dU0[(size_t)k2 * N + m] = 0.0;
      if (!s->act[m]) continue;
      double U[MAXM], dA[MAXD * MAXM], f0[MAXQ * MAXM], f1[MAXQ * MAXM];
      const double *l0 = lf + (size_t)m * Q * M;
      for (int r = 0; r < M; ++r) U[r] = s->U0[(size_t)r * N + m];
      for (int A = 0; A < D; ++A)
        for (int r = 0; r < M; ++r) dA[A * M + r] = s->dU0[((size_t)A * M + r) * N + m];
      double b0[MAXD];
      body_acc(s, m, s->init_step * s->dt, b0);
      init_node(s, -1, s->mu, s->lam, U, dA, b0, f0);
      for (int a = 0; a < D; ++a) {
        double acc = 0.0;
        U[a] += 1.0;
        init_node(s, -1, s->mu, s->lam, U, dA, b0, f1);
        U[a] -= 1.0;
        for (int k2 = 0; k2 < Q * M; ++k2) acc += l0[k2] * (f1[k2] - f0[k2]);
        if (grad_v0) grad_v0[(size_t)a * N + m] = acc - 0.5 * s->dt * lus[m * D + a];
        if (grad_u0) grad_u0[(size_t)a * N + m] = lus[m * D + a];
      }
      /* the populations are affine in the gradient data dU0 (Eqs. 32-33):
       * unit differences are exact */
      if (grad_dU0)
        for (int k2 = 0; k2 < D * M; ++k2) {
          double acc = 0.0;
          dA[k2] += 1.0;
          init_node(s, -1, s->mu, s->lam, U, dA, b0, f1);
          dA[k2] -= 1.0;
          for (int k3 = 0; k3 < Q * M; ++k3) acc += l0[k3] * (f1[k3] - f0[k3]);
          grad_dU0[(size_t)k2 * N + m] = acc;
        }
      init_node(s, -1, s->mu + 1.0, s->lam, U, dA, b0, f0);
      init_node(s, -1, s->mu - 1.0, s->lam, U, dA, b0, f1);
      for (int k2 = 0; k2 < Q * M; ++k2) gi[0] += l0[k2] * 0.5 * (f0[k2] - f1[k2]);
      init_node(s, -1, s->mu, s->lam + 1.0, U, dA, b0, f0);
      init_node(s, -1, s->mu, s->lam - 1.0, U, dA, b0, f1);
      for (int k2 = 0; k2 < Q * M; ++k2) gi[1] += l0[k2] * 0.5 * (f0[k2] - f1[k2]);
    }
    gmat[0] += gi[0];
    gmat[1] += gi[1];
    if (grad_mat) {
      grad_mat[0] = gmat[0];
      grad_mat[1] = gmat[1];
    }
  }
  /* leave the simulation at the end of the trajectory */
  if (!status && nsteps > 0) {
    memcpy(s->f, trf + nf * (nsteps - 1), sizeof(double) * nf);
    memcpy(s->ustar, trs + nd * (nsteps - 1), sizeof(double) * nd);
    s->step = k0 + nsteps - 1;
    status = orc_step(s, 1);
  }
  free(trf); free(trs); free(lf); free(lfs); free(lus); free(ub); free(ubc); free(y); free(x0b);
  free(Ua); free(Ur); free(Fcb); free(Frb); free(Uab); free(comp); free(anch); free(an);
  return status;
}
