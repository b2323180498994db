// Constitutive laws of the lattice update as register-level policies.
//
// The bulk update, the initialisation and the traction closure evaluate the
// first Piola stress node by node: the law stays a local material-point
// operation, and laws with internal variables update them at the node
// (Sec. 6).  A law is a type with
//   body                 the instantiation also applies a body acceleration
//   Node                 the law's per-node internal variables, in registers
//   load(p, node, S, n)  read them (planes of stride S)
//   stress(p, F, n, P)   P(F) in FP64 at the loaded internal variables;
//                        returns J (the caller flags J <= 0)
//   tangent(p, F, n, dF, dP)  its directional derivative at frozen
//                        internal variables
//   commit(p, n, node, S)  advance the internal variables with the
//                        deformation of the last stress evaluation (the one
//                        the collision used)
// NeoHookean is the paper's law (Eq. 62); Reinforced adds one fibre family
// (k1 > 0) and takes a body acceleration; Viscoelastic adds one Maxwell
// branch with per-node history to Reinforced; Thermal gives Reinforced a
// per-node thermal stretch.
#pragma once
#include <hip/hip_runtime.h>

#include "tl_internal.hpp"
#include "tl_math.hpp"

namespace tl {

// packed symmetric index: 2D (00, 01, 11), 3D (00, 01, 02, 11, 12, 22)
template <int D> __host__ __device__ constexpr int sym_idx(int A, int B) {
  return A <= B ? (A * (2 * D - A + 1)) / 2 + (B - A) : (B * (2 * D - B + 1)) / 2 + (A - B);
}
template <int D> constexpr int sym_n() { return D * (D + 1) / 2; }

// the shear part of the neo-Hookean second Piola stress, S_0 = mu (I - C^{-1})
// (packed), and C^{-1} = F^{-1} F^{-T} (full, optional)
template <int D>
__host__ __device__ __forceinline__ void shear_S0(const double *F, double mu, double *S0, double *Ci) {
  double G[D * D];
  cofactor<D>(F, G);
  const double J = det<D>(F);
  const double r = 1.0 / (J * J);
#pragma unroll
  for (int A = 0; A < D; ++A)
#pragma unroll
    for (int B = A; B < D; ++B) {
      double c = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) c += G[i * D + A] * G[i * D + B];
      c *= r;
      S0[sym_idx<D>(A, B)] = mu * ((A == B ? 1.0 : 0.0) - c);
      if (Ci) Ci[A * D + B] = Ci[B * D + A] = c;
    }
}

// Maxwell branch: overstress Q(F) = R + beta xi S_0(F) in the second Piola
// stress, P += F Q; S0 receives S_0(F)
template <int D>
__host__ __device__ __forceinline__ void maxwell_add(const double *F, const Par &p, const double *R, double *P,
                                                     double *S0) {
  shear_S0<D>(F, p.mu, S0, nullptr);
  double Qv[sym_n<D>()];
#pragma unroll
  for (int k = 0; k < sym_n<D>(); ++k) Qv[k] = R[k] + p.vbx * S0[k];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int A = 0; A < D; ++A) {
      double s = 0.0;
#pragma unroll
      for (int B = 0; B < D; ++B) s += F[i * D + B] * Qv[sym_idx<D>(B, A)];
      P[i * D + A] += s;
    }
}

// its tangent at frozen R: dP += dF Q + beta xi F dS_0,
// dS_0 = mu C^{-1} dC C^{-1}, dC = dF^T F + F^T dF
template <int D>
__host__ __device__ __forceinline__ void maxwell_tangent_add(const double *F, const double *dF, const Par &p,
                                                             const double *R, double *dP) {
  double S0[sym_n<D>()], Ci[D * D], W[D * D], dS[D * D];
  shear_S0<D>(F, p.mu, S0, Ci);
#pragma unroll
  for (int A = 0; A < D; ++A)  // W = C^{-1} dC
#pragma unroll
    for (int B = 0; B < D; ++B) {
      double s = 0.0;
#pragma unroll
      for (int K = 0; K < D; ++K) {
        double dC = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) dC += dF[i * D + K] * F[i * D + B] + F[i * D + K] * dF[i * D + B];
        s += Ci[A * D + K] * dC;
      }
      W[A * D + B] = s;
    }
#pragma unroll
  for (int A = 0; A < D; ++A)  // dS_0 = mu W C^{-1}
#pragma unroll
    for (int B = 0; B < D; ++B) {
      double s = 0.0;
#pragma unroll
      for (int K = 0; K < D; ++K) s += W[A * D + K] * Ci[K * D + B];
      dS[A * D + B] = p.mu * s;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int A = 0; A < D; ++A) {
      double s = 0.0;
#pragma unroll
      for (int B = 0; B < D; ++B) {
        const int k = sym_idx<D>(B, A);
        s += dF[i * D + B] * (R[k] + p.vbx * S0[k]) + p.vbx * F[i * D + B] * dS[B * D + A];
      }
      dP[i * D + A] += s;
    }
}

template <int D> struct NeoHookean {
  static constexpr bool body = false;
  struct Node {};
  __device__ static void load(const Par &, int64_t, int64_t, Node &) {}
  __host__ __device__ static double stress(const Par &p, const double *F, Node &, double *P) {
    return piola<D>(F, p.mu, p.lam, P);
  }
  __device__ static void tangent(const Par &p, const double *F, const Node &, const double *dF, double *dP) {
    piola_tangent<D>(F, dF, p.mu, p.lam, dP);
  }
  __device__ static void commit(const Par &, const Node &, int64_t, int64_t) {}
};

template <int D> struct Reinforced {
  static constexpr bool body = true;
  struct Node {};
  __device__ static void load(const Par &, int64_t, int64_t, Node &) {}
  __host__ __device__ static double stress(const Par &p, const double *F, Node &, double *P) {
    const double J = piola<D>(F, p.mu, p.lam, P);
    if (p.k1 != 0.0) fibre_add<D>(F, p.k1, p.a0, P);
    return J;
  }
  __device__ static void tangent(const Par &p, const double *F, const Node &, const double *dF, double *dP) {
    piola_tangent<D>(F, dF, p.mu, p.lam, dP);
    if (p.k1 != 0.0) fibre_tangent_add<D>(F, dF, p.k1, p.a0, dP);
  }
  __device__ static void commit(const Par &, const Node &, int64_t, int64_t) {}
};

// Maxwell branch on the reinforced solid (an instance of a batch without a
// branch has no history planes: R = 0 and beta xi = 0, so Q = 0 and nothing
// is committed): P = P_eq(F) + F Q,
// dQ/dt + Q / tau = beta dS_0/dt, advanced per step by the midpoint rule on
// its convolution, Q^{n+1} = xi^2 Q^n + beta xi (S_0^{n+1} - S_0^n) with
// xi = exp(-dt / (2 tau)).  The node keeps R = xi^2 Q^n - beta xi S_0^n, so
// that Q(F) = R + beta xi S_0(F) and the commit after the step is
// R' = xi^2 R + beta xi (xi^2 - 1) S_0(F).
template <int D> struct Viscoelastic {
  static constexpr bool body = true;
  struct Node {
    double R[sym_n<D>()], S0[sym_n<D>()];
  };
  __device__ static void load(const Par &p, int64_t node, int64_t S, Node &n) {
#pragma unroll
    for (int k = 0; k < sym_n<D>(); ++k) n.R[k] = p.hist ? p.hist[(size_t)k * S + node] : 0.0;
  }
  __host__ __device__ static double stress(const Par &p, const double *F, Node &n, double *P) {
    typename Reinforced<D>::Node e;
    const double J = Reinforced<D>::stress(p, F, e, P);
    maxwell_add<D>(F, p, n.R, P, n.S0);
    return J;
  }
  __device__ static void tangent(const Par &p, const double *F, const Node &n, const double *dF, double *dP) {
    typename Reinforced<D>::Node e;
    Reinforced<D>::tangent(p, F, e, dF, dP);
    maxwell_tangent_add<D>(F, dF, p, n.R, dP);
  }
  __device__ static void commit(const Par &p, const Node &n, int64_t node, int64_t S) {
    if (!p.hist) return;
    const double c = p.vbx * (p.vxi2 - 1.0);
#pragma unroll
    for (int k = 0; k < sym_n<D>(); ++k) p.hist[(size_t)k * S + node] = p.vxi2 * n.R[k] + c * n.S0[k];
  }
};

// Thermal distortion (Sec. 6 names it for thermoelasticity): the temperature
// field, advanced by the caller, enters as the isotropic stretch th of the
// split F = F_e (th I) with the energy th^D W(F_e) per reference volume, so
// P(F) = th^(D-1) P_W(F / th) and dP = th^(D-1) dP_W(F / th; dF / th).  The
// node's th is one FP64 plane of stride S (p.thf; none: th = 1, as for the
// instances of a batch that have no field).
template <int D> struct Thermal {
  static constexpr bool body = true;
  struct Node {
    double th;
  };
  __device__ static void load(const Par &p, int64_t node, int64_t, Node &n) { n.th = p.thf ? p.thf[node] : 1.0; }
  __host__ __device__ static double stress(const Par &p, const double *F, Node &n, double *P) {
    double Fe[D * D];
#pragma unroll
    for (int k = 0; k < D * D; ++k) Fe[k] = F[k] / n.th;
    typename Reinforced<D>::Node e;
    const double Je = Reinforced<D>::stress(p, Fe, e, P);
    const double sc = D == 3 ? n.th * n.th : n.th;
#pragma unroll
    for (int k = 0; k < D * D; ++k) P[k] *= sc;
    return Je * sc * n.th;  // J = det F = th^D det F_e
  }
  __device__ static void tangent(const Par &p, const double *F, const Node &n, const double *dF, double *dP) {
    double Fe[D * D], dFe[D * D];
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
      Fe[k] = F[k] / n.th;
      dFe[k] = dF[k] / n.th;
    }
    typename Reinforced<D>::Node e;
    Reinforced<D>::tangent(p, Fe, e, dFe, dP);
    const double sc = D == 3 ? n.th * n.th : n.th;
#pragma unroll
    for (int k = 0; k < D * D; ++k) dP[k] *= sc;
  }
  __device__ static void commit(const Par &, const Node &, int64_t, int64_t) {}
};

// The context's law at one node for the paths that are not specialised
// (initialisation, traction closure, stress output): the elastic part, plus
// the Maxwell branch when R (the node's packed internal variables) is given,
// at the node's thermal stretch th (1: none).
template <int D> __host__ __device__ __forceinline__ double law_piola(const double *F, const Par &p, const double *R,
                                                                      double *P, double th = 1.0) {
  if (th != 1.0) {
    typename Thermal<D>::Node n{th};
    return Thermal<D>::stress(p, F, n, P);
  }
  typename Reinforced<D>::Node e;
  const double J = Reinforced<D>::stress(p, F, e, P);
  if (R) {
    double S0[sym_n<D>()];
    maxwell_add<D>(F, p, R, P, S0);
  }
  return J;
}

template <int D>
__device__ __forceinline__ void law_tangent(const double *F, const double *dF, const Par &p, const double *R,
                                            double *dP, double th = 1.0) {
  if (th != 1.0) {
    const typename Thermal<D>::Node n{th};
    Thermal<D>::tangent(p, F, n, dF, dP);
    return;
  }
  typename Reinforced<D>::Node e;
  Reinforced<D>::tangent(p, F, e, dF, dP);
  if (R) maxwell_tangent_add<D>(F, dF, p, R, dP);
}

// the node's thermal stretch (1 without a field)
template <int D> __device__ __forceinline__ double law_theta(const Par &p, int64_t node) {
  return p.thf ? p.thf[node] : 1.0;
}

// the node's internal variables (false: the law has none)
template <int D> __device__ __forceinline__ bool law_load(const Par &p, int64_t node, int64_t S, double *R) {
  if (!p.hist) return false;
#pragma unroll
  for (int k = 0; k < sym_n<D>(); ++k) R[k] = p.hist[(size_t)k * S + node];
  return true;
}

}  // namespace tl
