// Device helpers shared by the forward and reverse kernels: grid
// neighbourhoods, boundary data and the local Newton solve of the Neumann
// closure (all FP64, register resident).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "tl_internal.hpp"
#include "tl_law.hpp"
#include "tl_math.hpp"

namespace tl {

// ------------------------------------------------------------ grid helpers

struct C3 {
  int x, y, z;
};

__device__ __forceinline__ C3 coords_of(const Geo &g, int64_t i) {
  C3 c;
  c.x = (int)(i % g.nx);
  c.y = (int)((i / g.nx) % g.ny);
  c.z = (int)(i / ((int64_t)g.nx * g.ny));
  return c;
}

// node at integer offset (ox, oy, oz): periodic wrap, -1 outside a non-periodic box
__device__ __forceinline__ int64_t node_at(const Geo &g, C3 c, int ox, int oy, int oz) {
  int v[3] = {c.x + ox, c.y + oy, c.z + oz};
  const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    if (v[A] < 0 || v[A] >= n[A]) {
      if (!((g.per >> A) & 1)) return -1;
      v[A] = ((v[A] % n[A]) + n[A]) % n[A];
    }
  }
  return v[0] + (int64_t)g.nx * (v[1] + (int64_t)g.ny * v[2]);
}

__device__ __forceinline__ int64_t node_dir(const Geo &g, C3 c, int q, int mult) {
  const int A = q / 2, sg = (q & 1) ? -1 : 1;
  return node_at(g, c, A == 0 ? sg * mult : 0, A == 1 ? sg * mult : 0, A == 2 ? sg * mult : 0);
}

// node X + e_q of node i when that neighbour exists (the caller has checked
// bit q of the neighbour mask): fixed offsets in a box without periodic axes
__device__ __forceinline__ int64_t nb_index(const Geo &g, int64_t i, int q) {
  if (g.per) return node_dir(g, coords_of(g, i), q, 1);
  const int64_t nxy = (int64_t)g.nx * g.ny;
  const int64_t off = (q < 2) ? 1 : (q < 4 ? (int64_t)g.nx : nxy);
  return (q & 1) ? i - off : i + off;
}

// gv[al][i] += sum_k w_al,k u_i(point k) over the LSQ stencil of link l
// (Eqs. 48-52), points in order.  The loads of 8 points are issued together
// (a sequential loop would wait for every index and then every value in
// turn); the accumulation order is the sequential one.  slot(k) gives the
// displacement index of point k, uval(j, i) component i there.
template <int D, typename SlotF, typename UF>
__device__ __forceinline__ void lsq_gather(const Links &L, int64_t l, int np, SlotF slot, UF uval,
                                           double (&gv)[D - 1][D]) {
  constexpr int B = 8;
  for (int k0 = 0; k0 < np; k0 += B) {
    // past the last point the loads repeat point np - 1 (always valid) and
    // are not accumulated: no load sits behind a branch
    int64_t jj[B];
#pragma unroll
    for (int t = 0; t < B; ++t) jj[t] = slot(k0 + t < np ? k0 + t : np - 1);
    double uu[B][D], ww[B][D - 1];
#pragma unroll
    for (int t = 0; t < B; ++t) {
      const int k = k0 + t < np ? k0 + t : np - 1;
#pragma unroll
      for (int i = 0; i < D; ++i) uu[t][i] = uval(jj[t], i);
#pragma unroll
      for (int al = 0; al < D - 1; ++al) ww[t][al] = L.sw[lsq_w(L, l, al, k)];
    }
#pragma unroll
    for (int t = 0; t < B; ++t)
      if (k0 + t < np)
#pragma unroll
        for (int al = 0; al < D - 1; ++al)
#pragma unroll
          for (int i = 0; i < D; ++i) gv[al][i] += ww[t][al] * uu[t][i];
  }
}

// ------------------------------------------------- boundary data (FP64)

__host__ __device__ __forceinline__ void ramp_eval(int kind, double Tr, double t, double &s, double &ds) {
  s = 1.0;
  ds = 0.0;
  if (t < Tr) {
    if (kind == TLVLBM_RAMP_SIN2) {
      const double a = M_PI * t / (2.0 * Tr);
      s = sin(a) * sin(a);
      ds = M_PI / (2.0 * Tr) * sin(M_PI * t / Tr);
    } else if (kind == TLVLBM_RAMP_HALFCOS) {
      s = 0.5 * (1.0 - cos(M_PI * t / Tr));
      ds = 0.5 * M_PI / Tr * sin(M_PI * t / Tr);
    } else if (kind == TLVLBM_RAMP_LINEAR) {
      s = t / Tr;
      ds = 1.0 / Tr;
    }
  }
}

// integral of the loading factor from 0 to t
__host__ __device__ __forceinline__ double ramp_int(int kind, double Tr, double t) {
  if (kind == TLVLBM_RAMP_CONST) return t;
  const double tc = t < Tr ? t : Tr;
  double S;
  if (kind == TLVLBM_RAMP_LINEAR) S = 0.5 * tc * tc / Tr;
  else S = 0.5 * tc - Tr / (2.0 * M_PI) * sin(M_PI * tc / Tr);  // sin^2 and half-cosine
  return S + (t - tc);
}

// ramped rigid rotation of a displacement-given Dirichlet condition about the
// e3 axis through X0: u += (R(alpha) - I) d, v += alpha' R'(alpha) d with
// alpha = s(t) tw, d = (X - X0) in the (e1, e2) plane
__device__ __forceinline__ void twist_add(const BC &b, const double *X, double s, double ds, bool velocity,
                                          double *val) {
  if (b.tw == 0.0) return;
  const double al = s * b.tw, c = cos(al), sn = sin(al);
  const double dx = X[0] - b.X0[0], dy = X[1] - b.X0[1];
  if (velocity) {
    const double da = ds * b.tw;
    val[0] += da * (-sn * dx - c * dy);
    val[1] += da * (c * dx - sn * dy);
  } else {
    val[0] += (c - 1.0) * dx - sn * dy;
    val[1] += sn * dx + (c - 1.0) * dy;
  }
}

template <int D> __device__ __forceinline__ void bc_base(const BC &b, const double *X, const double *N, double *val) {
  double d[3], r = 0.0;
  for (int a = 0; a < D; ++a) {
    d[a] = X[a] - b.X0[a];
    r += d[a] * d[a];
  }
  r = sqrt(r);
  for (int i = 0; i < D; ++i) {
    double s = b.a[i];
    for (int A = 0; A < D; ++A) s += b.G[i * 3 + A] * d[A];
    if (b.pr != 0.0 && r > 0.0) s += b.pr * d[i] / r;
    s += b.pn * N[i];
    val[i] = s;
  }
}

// small dense solve A x = b (D <= 3) by the adjugate, x = cof(A)^T b / det A:
// fixed register arrays (no dynamically indexed pivoting); false when det A
// is zero or not finite
template <int D> __device__ inline bool solve_small(const double *A, const double *b, double *x) {
  double C[D * D];
  cofactor<D>(A, C);
  const double dA = det<D>(A);
  if (!(dA != 0.0) || !isfinite(dA)) return false;
  const double r = 1.0 / dA;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s += C[j * D + i] * b[j];
    x[i] = s * r;
  }
  return true;
}

// stress and tangent action of the elastic material in FP64 (neo-Hookean,
// plus the fibre term when p.k1 > 0)
template <int D> __host__ __device__ __forceinline__ double mat_piola(const double *F, const Par &p, double *P) {
  return law_piola<D>(F, p, nullptr, P);
}

template <int D>
__device__ __forceinline__ void mat_tangent(const double *F, const double *dF, const Par &p, double *dP) {
  law_tangent<D>(F, dF, p, nullptr, dP);
}

// R(h) = P(h (x) N + Gt) N - T (Eqs. 54, 56) with the law of the link's
// node (Hn: its internal variables, or null; th: its thermal stretch);
// false if det F_b <= 0
template <int D>
__device__ inline bool nm_residual(const double *h, const double *N, const double *Gt, const double *Tb, const Par &p,
                            double *R, const double *Hn = nullptr, double th = 1.0) {
  double F[D * D], P[D * D];
  for (int i = 0; i < D; ++i)
    for (int a = 0; a < D; ++a) F[i * D + a] = h[i] * N[a] + Gt[i * D + a];
  if (!(det<D>(F) > 0.0)) return false;
  law_piola<D>(F, p, Hn, P, th);
  for (int i = 0; i < D; ++i) {
    double s = 0.0;
    for (int a = 0; a < D; ++a) s += P[i * D + a] * N[a];
    R[i] = s - Tb[i];
    if (!__builtin_isfinite(R[i])) return false;
  }
  return true;
}

// Local Newton for the normal image h (Eqs. 53-56) in FP64, Jacobian
// dR/dh = Q(N; F_b) (acoustic tensor, Eq. 19) from the tangent action;
// accepts only det F_b > 0 with a decreasing residual (<= 10 halvings).
template <int D>
__device__ inline bool newton_h(const double *N, const double *Gt, const double *Tb, const Par &p, double tol,
                         double *h, const double *Hn = nullptr, double th = 1.0) {
  double R[D], Rt[D], ht[D];
  if (!nm_residual<D>(h, N, Gt, Tb, p, R, Hn, th)) return false;
  const double thr = tol * (p.mu > 1.0 ? p.mu : 1.0);
  for (int it = 0; it <= 30; ++it) {
    double rinf = 0.0, r2 = 0.0;
    for (int i = 0; i < D; ++i) {
      rinf = fmax(rinf, fabs(R[i]));
      r2 += R[i] * R[i];
    }
    if (rinf <= thr) return true;
    if (it == 30) break;
    double F[D * D], Qm[D * D], dh[D], mR[D];
    for (int i = 0; i < D; ++i)
      for (int a = 0; a < D; ++a) F[i * D + a] = h[i] * N[a] + Gt[i * D + a];
    for (int k = 0; k < D; ++k) {
      double dF[D * D], dP[D * D];
      for (int i = 0; i < D; ++i)
        for (int a = 0; a < D; ++a) dF[i * D + a] = (i == k) ? N[a] : 0.0;
      law_tangent<D>(F, dF, p, Hn, dP, th);
      for (int i = 0; i < D; ++i) {
        double s = 0.0;
        for (int a = 0; a < D; ++a) s += dP[i * D + a] * N[a];
        Qm[i * D + k] = s;
      }
    }
    for (int i = 0; i < D; ++i) mR[i] = -R[i];
    if (!solve_small<D>(Qm, mR, dh)) return false;
    double step = 1.0;
    bool acc = false;
    for (int ls = 0; ls <= 10; ++ls) {
      for (int i = 0; i < D; ++i) ht[i] = h[i] + step * dh[i];
      if (nm_residual<D>(ht, N, Gt, Tb, p, Rt, Hn, th)) {
        double rt2 = 0.0, rtinf = 0.0;
        for (int i = 0; i < D; ++i) {
          rt2 += Rt[i] * Rt[i];
          rtinf = fmax(rtinf, fabs(Rt[i]));
        }
        if (rt2 < r2 || rtinf <= thr) {
          acc = true;
          break;
        }
      }
      step *= 0.5;
    }
    if (!acc) return false;
    for (int i = 0; i < D; ++i) {
      h[i] = ht[i];
      R[i] = Rt[i];
    }
  }
  return false;
}

}  // namespace tl
