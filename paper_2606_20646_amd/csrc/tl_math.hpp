// Device-side point maps of the total-Lagrangian vectorial LBM.
//
// Everything here is register-resident, templated on the dimension D and the
// arithmetic type T.  Matrices are row-major D x D arrays.
#pragma once
#include <hip/hip_runtime.h>

namespace tl {

template <int D> struct Lat {
  static constexpr int Q = 2 * D;      // axis velocity set (Sec. 2.3, Eq. 20)
  static constexpr int M = D + D * D;  // state components (Sec. 2.2, Eq. 11)
};

// determinant and cofactor matrix cof(F) = det(F) F^{-T}
template <int D, typename T> __host__ __device__ __forceinline__ T det(const T *F) {
  if constexpr (D == 2) {
    return F[0] * F[3] - F[1] * F[2];
  } else {
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
  }
}

template <int D, typename T> __host__ __device__ __forceinline__ void cofactor(const T *F, T *C) {
  if constexpr (D == 2) {
    C[0] = F[3];
    C[1] = -F[2];
    C[2] = -F[1];
    C[3] = F[0];
  } else {
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
}

// First Piola stress of the compressible neo-Hookean solid (Sec. 4.1,
// Eq. 62; P = dW/dF, Sec. 2.1, Eq. 4):
//   P = mu (F - F^{-T}) + lambda/2 (J^2 - 1) F^{-T}.
// Returns J; the caller flags J <= 0.
template <int D, typename T>
__host__ __device__ __forceinline__ T piola(const T *F, T mu, T lam, T *P) {
  T C[D * D];
  cofactor<D>(F, C);
  const T J = det<D>(F);
  const T rJ = T(1) / J;
  const T a = mu * rJ;
  const T b = T(0.5) * lam * (J * J - T(1)) * rJ;
#pragma unroll
  for (int k = 0; k < D * D; ++k) P[k] = mu * F[k] + (b - a) * C[k];
  return J;
}

// Tangent action dP = C : dF (Sec. 2.1, Eq. 4; Sec. 2.2, Eq. 18):
//   dP = mu dF + (mu - lambda/2 (J^2-1)) F^{-T} dF^T F^{-T}
//        + lambda J^2 tr(F^{-1} dF) F^{-T}.
template <int D, typename T>
__device__ __forceinline__ void piola_tangent(const T *F, const T *dF, T mu, T lam, T *dP) {
  T C[D * D], G[D * D];
  cofactor<D>(F, C);
  const T J = det<D>(F);
  const T rJ = T(1) / J;
#pragma unroll
  for (int k = 0; k < D * D; ++k) G[k] = C[k] * rJ;  // F^{-T}
  T tr = T(0);
#pragma unroll
  for (int k = 0; k < D * D; ++k) tr += G[k] * dF[k];
  const T a = mu - T(0.5) * lam * (J * J - T(1));
  const T b = lam * J * J * tr;
#pragma unroll
  for (int i = 0; i < D; ++i) {
#pragma unroll
    for (int A = 0; A < D; ++A) {
      T s = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T w = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) w += dF[k * D + j] * G[k * D + A];
        s += G[i * D + j] * w;
      }
      dP[i * D + A] = mu * dF[i * D + A] + a * s + b * G[i * D + A];
    }
  }
}

// Fibre reinforcement of the neo-Hookean solid (the anisotropic law named in
// the paper's outlook, Sec. 6): W += k1/2 (I4 - 1)^2 with I4 = |F a0|^2 for a
// unit reference fibre direction a0.  Adds to P and to the tangent action:
//   P  += 2 k1 (I4 - 1) (F a0) (x) a0,
//   dP += 2 k1 [2 ((F a0).(dF a0)) (F a0) + (I4 - 1) dF a0] (x) a0.
template <int D, typename T>
__host__ __device__ __forceinline__ void fibre_add(const T *F, T k1, const double *a0, T *P) {
  T fa[D], I4 = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T s = T(0);
#pragma unroll
    for (int A = 0; A < D; ++A) s += F[i * D + A] * T(a0[A]);
    fa[i] = s;
    I4 += s * s;
  }
  const T c = T(2) * k1 * (I4 - T(1));
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int A = 0; A < D; ++A) P[i * D + A] += c * fa[i] * T(a0[A]);
}

template <int D, typename T>
__device__ __forceinline__ void fibre_tangent_add(const T *F, const T *dF, T k1, const double *a0, T *dP) {
  T fa[D], dfa[D], I4 = T(0), dI = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T s = T(0), ds = T(0);
#pragma unroll
    for (int A = 0; A < D; ++A) {
      s += F[i * D + A] * T(a0[A]);
      ds += dF[i * D + A] * T(a0[A]);
    }
    fa[i] = s;
    dfa[i] = ds;
    I4 += s * s;
    dI += s * ds;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T w = T(2) * k1 * (T(2) * dI * fa[i] + (I4 - T(1)) * dfa[i]);
#pragma unroll
    for (int A = 0; A < D; ++A) dP[i * D + A] += w * T(a0[A]);
  }
}

// Flux entry Phi_A^r of the conservative system (Sec. 2.2, Eq. 13) given the
// stress P (already divided by rho0 in the velocity rows by the caller).
template <int D, typename T>
__device__ __forceinline__ T flux_entry(int A, int r, const T *v, const T *Prho) {
  if (r < D) return -Prho[r * D + A];
  const int i = (r - D) / D, B = (r - D) % D;
  return (A == B) ? -v[i] : T(0);
}

}  // namespace tl
