// Reverse mode of the TL-VLBM update on gfx950 (project extension: the
// paper has no adjoint).
//
// For L = sum dLdU . U + dLdu . u over the moments after n steps, the
// gradient with respect to (mu, lambda), the initial velocity v0 and the
// initial displacement u0 is accumulated by the discrete adjoint of the
// forward kernels, in the forward's own storage: the adjoint of the stored
// field (post-collision populations plus the populations the cut links
// deposit at outside nodes) lives in SoA planes.  The forward bulk kernel
// pulls f*_q(X - e_q); its transpose reads the adjoint at its own node and
// pushes to X - e_q.  The cut-link transposes run first, in three passes
// whose write targets are unique per link within a pass.
//
// The forward is checkpointed every `seg` steps (full stored field); each
// segment is recomputed once with a per-step tape of the recovered state
// (v, F - I), the repaired F of projection steps and the displacement seen
// by the cut links, then reversed.
//
// Transposes of the point maps use the major symmetry of the hyperelastic
// tangent (C_iAkB = C_kBiA): the adjoint of dF -> dP(F)[dF] is the same
// map, so the forward tangent routine serves both directions.  The
// projection is differentiated through its solver: the damped Jacobi
// sweeps are transposed sweep by sweep; the exact mode's warm-started CG is
// differentiated as its exact solution map u = u0 + K^+ (b - K u0):
// b_bar = K^+ u_bar, u0_bar = (I - K K^+) u_bar, the mean of u_bar over each
// connected component without anchors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "tl_device.hpp"
#include "tl_internal.hpp"
#include "tl_math.hpp"

namespace tl {
namespace {

constexpr int AT = 256;

struct AdjPar {
  double om, sig, inv_damp, hdt, i2D, i2c, irho, mu, lam, gamma, c, dt, theta, dx;
  double k1, a0[3];  // fibre term of the material (k1 = 0: none)
};

// node X - e_q (periodic wrap; for an embedded body the neighbour exists)
__device__ __forceinline__ int64_t minus_eq(const Geo &g, int x, int y, int z, int q) {
  const int A = q >> 1, s = (q & 1) ? -1 : 1;
  if (A == 0) {
    x -= s;
    x = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
  } else if (A == 1) {
    y -= s;
    y = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
  } else {
    z -= s;
    z = z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z);
  }
  return x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
}

// two block sums added into slot[0..1] (one writer per slot: deterministic)
__device__ __forceinline__ void block_acc2(double a, double b, double *slot) {
  __shared__ double sh[AT / 64][2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  if (lane == 0) {
    sh[wid][0] = a;
    sh[wid][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
      s0 += sh[w][0];
      s1 += sh[w][1];
    }
    slot[0] += s0;
    slot[1] += s1;
  }
}

// Ub += a sum_q feq'_q(U)^T lam_q (equilibrium derivative, Sec. 2.3, Eq. 27)
// and (gm, gl) += a sum_q lam_q . d feq_q / d(mu, lambda).  With
// mu_A = sum_q e_qA lam_q:  v_bar_i = S_vi/(2D) - mu_A[F_iA]/(2c),
// F_bar = S_F/(2D) - dP(F)[W]/(2 c rho0), W_iA = mu_A[v_i].
// The F-row part: CW = -a/(2 c rho0) dP(F)[W] and the parameter terms
// (gm, gl) += -a/(2 c rho0) W : dP/d(mu, lambda), as two contractions:
// dP/dmu = F - F^{-T}, dP/dlambda = (J^2 - 1)/2 F^{-T} (the fibre term has no
// mu, lambda).
template <int D>
__device__ __forceinline__ void vjp_tangent(const double *F, const double *W, const AdjPar &p, double a, double *CW,
                                            double &gm, double &gl) {
  const double cf = -a * p.i2c * p.irho;
  {
    double C[D * D];
    cofactor<D>(F, C);
    const double J = det<D>(F), rJ = 1.0 / J;
    double wf = 0.0, wg = 0.0;
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
      wf += W[k] * F[k];
      wg += W[k] * (C[k] * rJ);
    }
    gm += cf * (wf - wg);
    gl += cf * (0.5 * (J * J - 1.0) * wg);
  }
  piola_tangent<D>(F, W, p.mu, p.lam, CW);
  if (p.k1 != 0.0) fibre_tangent_add<D>(F, W, p.k1, p.a0, CW);
#pragma unroll
  for (int k = 0; k < D * D; ++k) CW[k] *= cf;
}

// Phi'_A(U)^T x for the flux of Eq. 13 at deformation F: velocity rows
// -x[F_kA]; deformation rows -dP(F)[x_v (x) e_A] / rho0 (the tangent's major
// symmetry turns the transpose into the tangent action)
template <int D>
__device__ __forceinline__ void flux_T(const double *x, int A, const double *F, const AdjPar &p, double *out) {
  double W[D * D], CW[D * D];
#pragma unroll
  for (int k = 0; k < D; ++k) out[k] = -x[D + k * D + A];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int B = 0; B < D; ++B) W[i * D + B] = (B == A) ? x[i] : 0.0;
  piola_tangent<D>(F, W, p.mu, p.lam, CW);
  if (p.k1 != 0.0) fibre_tangent_add<D>(F, W, p.k1, p.a0, CW);
#pragma unroll
  for (int k = 0; k < D * D; ++k) out[D + k] = -CW[k] * p.irho;
}

// lam holds the adjoint populations in their storage type E (register
// pressure: 2D·M values); the arithmetic is FP64.
template <int D, typename E>
__device__ __forceinline__ void feq_vjp(const E (&lam)[2 * D][D + D * D], const double *F, const AdjPar &p,
                                        double a, double *Ub, double &gm, double &gl) {
  constexpr int Q = 2 * D, M = D + D * D;
  double W[D * D];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) s += double(lam[q][r]);
    Ub[r] += a * p.i2D * s;
  }
#pragma unroll
  for (int A = 0; A < D; ++A) {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const double m = double(lam[2 * A][r]) - double(lam[2 * A + 1][r]);
      if (r < D) {
        W[r * D + A] = m;
      } else {
        const int i = (r - D) / D, B = (r - D) % D;
        if (B == A) Ub[i] -= a * p.i2c * m;
      }
    }
  }
  double CW[D * D];
  vjp_tangent<D>(F, W, p, a, CW, gm, gl);
#pragma unroll
  for (int k = 0; k < D * D; ++k) Ub[D + k] += CW[k];
}

template <int D, typename T>
__device__ __forceinline__ void load_adj(const T *__restrict__ L, const Geo &g, int64_t node,
                                         T (&lam)[2 * D][D + D * D]) {
  constexpr int Q = 2 * D, M = D + D * D;
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int r = 0; r < M; ++r) lam[q][r] = L[(size_t)(q * M + r) * g.S + node];
}

// push lam_f = (1 - omega) lam_fs + R^T Ub to the pull slots X - e_q
template <int D, typename T>
__device__ __forceinline__ void push_adj(T *__restrict__ Lin, const Geo &g, const AdjPar &p, int x, int y, int z,
                                         const T (&lam)[2 * D][D + D * D], const double *Ub) {
  constexpr int Q = 2 * D, M = D + D * D;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t dst = minus_eq(g, x, y, z, q);
#pragma unroll
    for (int r = 0; r < M; ++r)
      Lin[(size_t)(q * M + r) * g.S + dst] =
          T((1.0 - p.om) * double(lam[q][r]) + Ub[r] * (r < D ? p.inv_damp : 1.0));
  }
}

// tape planes (F - I of every step, F^r of projection steps) hold one slot
// per node of the chunk list, cpos[i / CHUNK] * CHUNK + i % CHUNK, plane stride ts
// (without a chunk list: the node index, stride S)
__device__ __forceinline__ int64_t tslot(const int32_t *__restrict__ cpos, int64_t node) {
  return cpos ? (int64_t)cpos[node / CHUNK] * CHUNK + (node % CHUNK) : node;
}

template <int D, typename T>
__device__ __forceinline__ void tape_F(const T *__restrict__ tape, int64_t ts, int64_t slot, double *F) {
#pragma unroll
  for (int k = 0; k < D * D; ++k) F[k] = double(tape[(size_t)k * ts + slot]) + ((k % (D + 1) == 0) ? 1.0 : 0.0);
}

// ------------------------------------------------------------------ seeds
// adjoint of the final moments: U = R(f) (v = sum f^v / (1 + gamma dt/2)),
// u = u* + dt/2 v
template <int D, typename T, bool MASK, bool TRACK>
__global__ __launch_bounds__(AT) void k_adj_seed(T *__restrict__ Lin, Geo g, AdjPar p,
                                                 const uint8_t *__restrict__ act, const double *__restrict__ dLdU,
                                                 const double *__restrict__ dLdu, double *__restrict__ lus) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, row = blockIdx.y;
  if (x >= g.nx) return;
  const int64_t node = x + (int64_t)g.nx * row;
  if (MASK && !act[node]) return;
  const int y = row % g.ny, z = row / g.ny;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    double v = dLdU ? dLdU[(size_t)r * g.N + node] : 0.0;
    if (r < D) {
      if (TRACK && dLdu) v += p.hdt * dLdu[(size_t)r * g.N + node];
      v *= p.inv_damp;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) Lin[(size_t)(q * M + r) * g.S + minus_eq(g, x, y, z, q)] = T(v);
  }
  if (TRACK)
#pragma unroll
    for (int i = 0; i < D; ++i) lus[(size_t)i * g.S + node] = dLdu ? dLdu[(size_t)i * g.N + node] : 0.0;
}

// ------------------------------------------------- bulk transpose (plain)
// collision (Eq. 29) with the damping source, recovery (Eq. 28) and the
// displacement history (Eq. 34): u = u* + dt/2 v, u*' = u + dt/2 v.
// CH: embedded bodies, over the list of CHUNK-node chunks that hold active
// nodes (64 / CHUNK chunks per wavefront, as the forward update); else one block
// per (row, x range).
template <int D, typename T, bool MASK, bool TRACK, bool CH = false>
__global__ __launch_bounds__(AT, 3) void k_adj_bulk(const T *__restrict__ Lout, T *__restrict__ Lin, Geo g, AdjPar p,
                                                 const uint8_t *__restrict__ act, const T *__restrict__ tape,
                                                 int64_t ts, const double *__restrict__ ubc,
                                                 double *__restrict__ lus, double *__restrict__ gblk,
                                                 const int32_t *__restrict__ chunks = nullptr, int nchunks = 0) {
  constexpr int Q = 2 * D, M = D + D * D;
  int x, row;
  bool live;
  int64_t slot = 0;
  if constexpr (CH) {
    const int ch = blockIdx.x * (AT / CHUNK) + (int)(threadIdx.x / CHUNK);
    const int64_t i = ch < nchunks ? (int64_t)chunks[ch] * CHUNK + (threadIdx.x % CHUNK) : g.N;
    live = i < g.N;
    x = live ? (int)(i % g.nx) : 0;
    row = live ? (int)(i / g.nx) : 0;
    slot = (int64_t)ch * CHUNK + (threadIdx.x % CHUNK);
  } else {
    x = blockIdx.x * blockDim.x + threadIdx.x;
    row = blockIdx.y;
    live = x < g.nx;
  }
  const int64_t node = x + (int64_t)g.nx * row;
  if constexpr (!CH) slot = node;
  double gm = 0.0, gl = 0.0;
  if (live && (!MASK || act[node])) {
    // the feq' transpose of feq_vjp (a = omega), arranged so that only the
    // velocity rows of lam stay in registers: the F rows stream through one
    // at a time and are pushed as soon as their U_bar is complete
    const int y = row % g.ny, z = row / g.ny;
    const double a = p.om;
    int64_t dst[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) dst[q] = minus_eq(g, x, y, z, q);
    T lv[Q][D];
    double Sv[D], W[D * D], Ubv[D];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < D; ++i) lv[q][i] = Lout[(size_t)(q * M + i) * g.S + node];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s += double(lv[q][i]);
      Sv[i] = s;
      Ubv[i] = a * p.i2D * s;
#pragma unroll
      for (int A = 0; A < D; ++A) W[i * D + A] = double(lv[2 * A][i]) - double(lv[2 * A + 1][i]);
    }
    double CW[D * D];
    {
      double F[D * D];
      tape_F<D, T>(tape, ts, slot, F);
      vjp_tangent<D>(F, W, p, a, CW, gm, gl);
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
      const int r = D + k, i = k / D, B = k % D;
      T lr[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) lr[q] = Lout[(size_t)(q * M + r) * g.S + node];
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s += double(lr[q]);
      const double ub = a * p.i2D * s + CW[k];
      Ubv[i] -= a * p.i2c * (double(lr[2 * B]) - double(lr[2 * B + 1]));
#pragma unroll
      for (int q = 0; q < Q; ++q) Lin[(size_t)(q * M + r) * g.S + dst[q]] = T((1.0 - p.om) * double(lr[q]) + ub);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) Ubv[i] -= p.sig * p.gamma * Sv[i];
    if (TRACK) {
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const double lu = lus[(size_t)i * g.S + node];
        const double ub = ubc[(size_t)i * g.S + node] + lu;
        Ubv[i] += p.hdt * (lu + ub);
        lus[(size_t)i * g.S + node] = ub;
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < D; ++i)
        Lin[(size_t)(q * M + i) * g.S + dst[q]] = T((1.0 - p.om) * double(lv[q][i]) + Ubv[i] * p.inv_damp);
  }
  block_acc2(gm, gl, gblk + 2 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x));
}

// ------------------------------------------- bulk transpose (projection)
// phase 1: collision with U^r and the repair f += feq(U^r) - feq(U) (Eq. 61)
// in reverse; U^r = (v, (1 - theta) F + theta F^c) (Eq. 60).  Leaves the
// partial adjoint of the recovered state in UaB and that of F^c in Fcb.
template <int D, typename T>
__global__ __launch_bounds__(AT) void k_adj_rep1(const T *__restrict__ Lout, Geo g, AdjPar p,
                                                 const uint8_t *__restrict__ act, const T *__restrict__ tape,
                                                 const T *__restrict__ tapeFr, int64_t ts,
                                                 const int32_t *__restrict__ cpos, const double *__restrict__ Frb,
                                                 const double *__restrict__ lus, double *__restrict__ UaB,
                                                 double *__restrict__ Fcb, double *__restrict__ gblk) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, row = blockIdx.y;
  const int64_t node = x + (int64_t)g.nx * row;
  double gm = 0.0, gl = 0.0;
  if (x < g.nx && act[node]) {
    T lam[Q][M];
    double Fa[D * D], Fr[D * D], Ur[M], Ua[M];
    load_adj<D, T>(Lout, g, node, lam);
    const int64_t slot = tslot(cpos, node);
    tape_F<D, T>(tape, ts, slot, Fa);
#pragma unroll
    for (int k = 0; k < D * D; ++k) Fr[k] = double(tapeFr[(size_t)k * ts + slot]) + ((k % (D + 1) == 0) ? 1.0 : 0.0);
#pragma unroll
    for (int r = 0; r < M; ++r) {
      Ur[r] = 0.0;
      Ua[r] = 0.0;
    }
    // omega feq'(U^r) (collision) + (1 - omega) feq'(U^r) (repair)
    feq_vjp<D>(lam, Fr, p, 1.0, Ur, gm, gl);
    feq_vjp<D>(lam, Fa, p, -(1.0 - p.om), Ua, gm, gl);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s += double(lam[q][i]);
      Ur[i] += -p.sig * p.gamma * s + p.hdt * lus[(size_t)i * g.S + node];
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) Ur[D + k] += Frb[(size_t)k * g.S + node];
#pragma unroll
    for (int i = 0; i < D; ++i) UaB[(size_t)i * g.S + node] = Ua[i] + Ur[i];
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
      UaB[(size_t)(D + k) * g.S + node] = Ua[D + k] + (1.0 - p.theta) * Ur[D + k];
      Fcb[(size_t)k * g.S + node] = p.theta * Ur[D + k];
    }
  }
  block_acc2(gm, gl, gblk + 2 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x));
}

// phase 2: the recovered state's adjoint is complete (kept columns, first
// projection, u = u* + dt/2 v): push lam_f
template <int D, typename T>
__global__ __launch_bounds__(AT) void k_adj_rep2(const T *__restrict__ Lout, T *__restrict__ Lin, Geo g, AdjPar p,
                                                 const uint8_t *__restrict__ act, const double *__restrict__ UaB,
                                                 const double *__restrict__ Fext, const double *__restrict__ x0b,
                                                 double *__restrict__ lus) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, row = blockIdx.y;
  if (x >= g.nx) return;
  const int64_t node = x + (int64_t)g.nx * row;
  if (!act[node]) return;
  const int y = row % g.ny, z = row / g.ny;
  T lam[Q][M];
  double Ub[M];
  load_adj<D, T>(Lout, g, node, lam);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double ub = x0b[(size_t)i * g.S + node];
    Ub[i] = UaB[(size_t)i * g.S + node] + p.hdt * ub;
    lus[(size_t)i * g.S + node] = ub;
  }
#pragma unroll
  for (int k = 0; k < D * D; ++k) Ub[D + k] = UaB[(size_t)(D + k) * g.S + node] + Fext[(size_t)k * g.S + node];
  push_adj<D, T>(Lin, g, p, x, y, z, lam, Ub);
}

// ------------------------------------------------- cut-link transposes
// Interpolated closure (Eqs. 42-43): for eta >= 1/2
//   f_in = (Dg f*_out(m) + S)/(2 eta) + (1 - 1/(2 eta)) f*_in(m),
// else f_in = Dg (2 eta f*_out(m) + (1 - 2 eta) f*_out(m^-)) + S.  The adjoint
// of the deposited value sits in the pull slot of the outside node.
// PASS 1 sets lam(m, q_out) (no pull reads it) and differentiates the
// Neumann source; PASS 2 adds to lam(m, q_in), PASS 3 to lam(m^-, q_out).
template <int D, typename T, int PASS, bool NEU>
__global__ __launch_bounds__(64) void k_adj_link(T *__restrict__ Lb, Links L, int64_t b0, int64_t b1, BC bc, Geo g,
                                                 Par par, double th, const T *__restrict__ tapeU,
                                                 const T *__restrict__ tapeFr, int64_t ts,
                                                 const int32_t *__restrict__ cpos, const double *__restrict__ tapeu,
                                                 const int32_t *__restrict__ sc, int64_t nu,
                                                 double *__restrict__ gbar, double *__restrict__ glink) {
  constexpr int M = D + D * D;
  const int64_t l = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= b1) return;
  const int64_t m = L.node[l], mm = L.mminus[l], o = L.out[l];
  const int qo = L.q[l], qi = qo ^ 1, A = qo / 2;
  const double sg = (qo & 1) ? -1.0 : 1.0;
  const double eta = L.eta[l];
  double lg[M];
#pragma unroll
  for (int r = 0; r < M; ++r) lg[r] = double(Lb[(size_t)(qi * M + r) * g.S + o]);
  // (read all M targets, then write them: the M slots of one link are
  // distinct, and interleaved loads and stores through one pointer would be
  // issued one row at a time)
  if constexpr (PASS == 2) {
    if (eta >= 0.5) {
      T cur[M];
#pragma unroll
      for (int r = 0; r < M; ++r) cur[r] = Lb[(size_t)(qi * M + r) * g.S + m];
#pragma unroll
      for (int r = 0; r < M; ++r) Lb[(size_t)(qi * M + r) * g.S + m] = T(double(cur[r]) + (1.0 - 0.5 / eta) * lg[r]);
    }
    return;
  }
  if constexpr (PASS == 3) {
    if (eta < 0.5 && mm != m) {
      T cur[M];
#pragma unroll
      for (int r = 0; r < M; ++r) cur[r] = Lb[(size_t)(qo * M + r) * g.S + mm];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const double Dg = NEU ? (r < D ? 1.0 : -1.0) : (r < D ? -1.0 : 1.0);
        Lb[(size_t)(qo * M + r) * g.S + mm] = T(double(cur[r]) + Dg * (1.0 - 2.0 * eta) * lg[r]);
      }
    }
    return;
  }
  // PASS 1
#pragma unroll
  for (int r = 0; r < M; ++r) {
    const double Dg = NEU ? (r < D ? 1.0 : -1.0) : (r < D ? -1.0 : 1.0);
    double v = (eta >= 0.5) ? Dg * 0.5 / eta * lg[r] : Dg * 2.0 * eta * lg[r];
    if (eta < 0.5 && mm == m) v += Dg * (1.0 - 2.0 * eta) * lg[r];
    Lb[(size_t)(qo * M + r) * g.S + m] = T(v);
  }
  if constexpr (NEU) {
    // forward state of the link: tangent images from the LSQ weights applied
    // to u (Eqs. 48-52), the Newton root h (Eqs. 53-56), F_b = h (x) N + Gt
    double N[3], Xb[3], Tb[3], Gt[D * D];
    for (int a = 0; a < 3; ++a) {
      N[a] = L.Nb[l * 3 + a];
      Xb[a] = L.Xb[l * 3 + a];
    }
    for (int k = 0; k < D * D; ++k) Gt[k] = 0.0;
    const int np = L.npts[l];
    double gv[D - 1][D];
    for (int al = 0; al < D - 1; ++al)
      for (int i = 0; i < D; ++i) gv[al][i] = L.tang[l * 6 + al * 3 + i];
    // the tape holds u at the Neumann stencil nodes only
    lsq_gather<D>(
        L, l, np, [&](int k) { return (int64_t)sc[lsq_i(L, l, k)]; },
        [&](int64_t t, int i) { return tapeu[(size_t)i * nu + t]; }, gv);
    for (int al = 0; al < D - 1; ++al)
      for (int i = 0; i < D; ++i)
        for (int B = 0; B < D; ++B) Gt[i * D + B] += gv[al][i] * L.tang[l * 6 + al * 3 + B];
    double s, ds;
    ramp_eval(bc.ramp, bc.Tr, th, s, ds);
    bc_base<D>(bc, Xb, N, Tb);
    for (int i = 0; i < D; ++i) Tb[i] *= s;
    double h[D], Fm[D * D];
    const int64_t slot = tslot(cpos, m);
    if (tapeFr)
      for (int k = 0; k < D * D; ++k) Fm[k] = double(tapeFr[(size_t)k * ts + slot]) + ((k % (D + 1) == 0) ? 1.0 : 0.0);
    else
      tape_F<D, T>(tapeU, ts, slot, Fm);
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int B = 0; B < D; ++B) acc += Fm[i * D + B] * N[B];
      h[i] = acc;
    }
    newton_h<D>(N, Gt, Tb, par, 1e-12, h);
    double Fb[D * D];
    for (int i = 0; i < D; ++i)
      for (int B = 0; B < D; ++B) Fb[i * D + B] = h[i] * N[B] + Gt[i * D + B];
    // source adjoint: S^v_i = sg P_b,iA / (rho0 c), S^F = (F_b - I)/D (Eqs. 46-47)
    const double cS = (eta >= 0.5) ? 0.5 / eta : 1.0;
    double W[D * D], CW[D * D], Fbb[D * D], Pm[D * D], Pl[D * D];
    for (int i = 0; i < D; ++i)
      for (int B = 0; B < D; ++B) W[i * D + B] = (B == A) ? sg * cS * lg[i] * par.inv_rho0 / par.c : 0.0;
    mat_tangent<D>(Fb, W, par, CW);
    piola<D>(Fb, 1.0, 0.0, Pm);
    piola<D>(Fb, 0.0, 1.0, Pl);
    double gm = 0.0, gl = 0.0;
    for (int k = 0; k < D * D; ++k) {
      Fbb[k] = CW[k] + cS * lg[D + k] / D;
      gm += W[k] * Pm[k];
      gl += W[k] * Pl[k];
    }
    // implicit function theorem on R(h) = P(F_b) N - T = 0: z = Q^{-T} h_bar
    // (Q the acoustic tensor, Eq. 19), Gt_bar = F_b_bar - dP[z (x) N],
    // p_bar -= dP/dp : (z (x) N)
    double hb[D], Qt[D * D], z[D];
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int B = 0; B < D; ++B) acc += Fbb[i * D + B] * N[B];
      hb[i] = acc;
    }
    for (int k = 0; k < D; ++k) {
      double dF[D * D], dP[D * D];
      for (int i = 0; i < D; ++i)
        for (int a = 0; a < D; ++a) dF[i * D + a] = (i == k) ? N[a] : 0.0;
      mat_tangent<D>(Fb, dF, par, dP);
      for (int i = 0; i < D; ++i) {
        double acc = 0.0;
        for (int a = 0; a < D; ++a) acc += dP[i * D + a] * N[a];
        Qt[k * D + i] = acc;  // (Q^T)_ki = Q_ik
      }
    }
    if (!solve_small<D>(Qt, hb, z))
      for (int i = 0; i < D; ++i) z[i] = 0.0;
    double zN[D * D], CzN[D * D];
    for (int i = 0; i < D; ++i)
      for (int a = 0; a < D; ++a) zN[i * D + a] = z[i] * N[a];
    mat_tangent<D>(Fb, zN, par, CzN);
    for (int k = 0; k < D * D; ++k) {
      gm -= zN[k] * Pm[k];
      gl -= zN[k] * Pl[k];
    }
    for (int al = 0; al < D - 1; ++al)
      for (int i = 0; i < D; ++i) {
        double acc = 0.0;
        for (int B = 0; B < D; ++B) acc += (Fbb[i * D + B] - CzN[i * D + B]) * L.tang[l * 6 + al * 3 + B];
        gbar[l * 6 + al * 3 + i] = acc;
      }
    glink[2 * l] += gm;
    glink[2 * l + 1] += gl;
  }
}

// u_bar at the LSQ stencil nodes: sum over (link, point) entries of
// w_alpha,k g_bar_alpha (sorted entries: deterministic)
template <int D>
__global__ __launch_bounds__(AT) void k_adj_ugather(int64_t ns, const int64_t *__restrict__ sn,
                                                    const int64_t *__restrict__ so, const int32_t *__restrict__ el,
                                                    const double *__restrict__ ew, Geo g,
                                                    const double *__restrict__ gbar, double *__restrict__ ubc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ns) return;
  double acc[D];
  for (int i = 0; i < D; ++i) acc[i] = 0.0;
  // entries in order, 4 at a time with every load unconditional (entries
  // past the last repeat it and are not accumulated)
  const int64_t e0 = so[t], e1 = so[t + 1];
  for (int64_t e = e0; e < e1; e += 4) {
    int64_t ll[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ll[k] = el[e + k < e1 ? e + k : e1 - 1];
    double wk[4][D - 1], gb[4][D - 1][D];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t ek = e + k < e1 ? e + k : e1 - 1;
#pragma unroll
      for (int al = 0; al < D - 1; ++al) {
        wk[k][al] = ew[(size_t)ek * (D - 1) + al];
#pragma unroll
        for (int i = 0; i < D; ++i) gb[k][al][i] = gbar[ll[k] * 6 + al * 3 + i];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (e + k < e1)
#pragma unroll
        for (int al = 0; al < D - 1; ++al)
#pragma unroll
          for (int i = 0; i < D; ++i) acc[i] += wk[k][al] * gb[k][al][i];
  }
  for (int i = 0; i < D; ++i) ubc[(size_t)i * g.S + sn[t]] = acc[i];
}

// --------------------------------------------------- projection transposes
// x0_bar = projection of u_bar onto the null space of K, CG right-hand side
// b = u_bar - x0_bar, start x = 0
template <int D>
__global__ __launch_bounds__(AT) void k_pi_apply(Geo g, const uint8_t *__restrict__ act,
                                                 const int32_t *__restrict__ comp, const double *__restrict__ mean,
                                                 const double *__restrict__ ua, const double *__restrict__ ub,
                                                 double *__restrict__ x0b, double *__restrict__ b,
                                                 double *__restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const bool a = act[i];
  const int32_t c = a ? comp[i] : -1;
  for (int k = 0; k < D; ++k) {
    const size_t o = (size_t)k * g.S + i;
    const double u = a ? ua[o] + (ub ? ub[o] : 0.0) : 0.0;
    const double pm = c >= 0 ? mean[(size_t)c * D + k] : 0.0;
    x0b[o] = pm;
    b[o] = a ? u - pm : 0.0;
    x[o] = 0.0;
  }
}

// transpose of the projection's damped Jacobi sweeps (Sec. 3.5).  A sweep
// x' = x + om D^+ (b - K x) (deg = diag K, D^+ = 1/deg where deg > 0 and 0
// else, K symmetric) has the transpose z -> z - om K D^+ z, b_bar += om D^+ z.
// In the scaled variable w = D^+ z one transposed sweep is
//   b_bar += om w,  w <- (1 - om) w + om/deg sum_{active nbrs} w_j,
// the forward sweep with b = 0; afterwards z = deg w, and z passes unchanged
// through nodes with deg = 0.
// degree and active neighbours of node i from its neighbour mask (bit q:
// X + e_q active, bit 6: X active); 0 for an inactive node
template <int D>
__device__ __forceinline__ int jac_degree(const Geo &g, const uint8_t *__restrict__ nbm,
                                          const uint8_t *__restrict__ anc_n, int64_t i, int64_t *nb) {
  const unsigned m = nbm[i];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) nb[q] = -1;
  if (!(m & 64u)) return 0;
#pragma unroll
  for (int q = 0; q < 2 * D; ++q)
    if ((m >> q) & 1u) nb[q] = nb_index(g, i, q);
  return (anc_n ? anc_n[i] : 0) + __builtin_popcount(m & ((1u << (2 * D)) - 1u));
}

// seed: z = ua + ub; w = D^+ z, zk = z where deg = 0 (else 0), b_bar = 0
template <int D>
__global__ __launch_bounds__(AT) void k_jacT_seedw(Geo g, const uint8_t *__restrict__ nbm,
                                                   const uint8_t *__restrict__ anc_n, const double *__restrict__ ua,
                                                   const double *__restrict__ ub, double *__restrict__ w,
                                                   double *__restrict__ zk, double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int64_t nb[2 * D];
  const int deg = jac_degree<D>(g, nbm, anc_n, i, nb);
  const bool a = (nbm[i] & 64u) != 0;
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S + i;
    const double z = a ? ua[o] + (ub ? ub[o] : 0.0) : 0.0;
    w[o] = deg ? z / double(deg) : 0.0;
    zk[o] = deg ? 0.0 : z;
    y[o] = 0.0;
  }
}

// one transposed sweep over the active tiles (XCD-contiguous tile ranges,
// as the forward sweep)
template <int D>
__global__ __launch_bounds__(AT) void k_jacT_sweep(Geo g, const uint8_t *__restrict__ nbm,
                                                   const uint8_t *__restrict__ anc_n, const double *__restrict__ win,
                                                   double *__restrict__ wout, double *__restrict__ y, double om,
                                                   const int32_t *__restrict__ tiles, int ntile, int per) {
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= ntile) return;
  const int64_t i = (tiles ? (int64_t)tiles[t] : (int64_t)t) * AT + threadIdx.x;
  if (i >= g.N || !(nbm[i] & 64u)) return;
  int64_t nb[2 * D];
  const int deg = jac_degree<D>(g, nbm, anc_n, i, nb);
  // unconditional loads (a missing neighbour reads the node itself and adds
  // an exact zero): all of them in flight together
  int64_t at[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) at[q] = nb[q] >= 0 ? nb[q] : i;
  double wi[D], yi[D], wn[D][2 * D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S;
    wi[c] = win[o + i];
    yi[c] = y[o + i];
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) wn[c][q] = win[o + at[q]];
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S;
    y[o + i] = yi[c] + om * wi[c];
    if (deg == 0) {
      wout[o + i] = 0.0;
      continue;
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) s += nb[q] >= 0 ? wn[c][q] : 0.0;
    wout[o + i] = (1.0 - om) * wi[c] + om * s / double(deg);
  }
}

// z = deg w + zk (the start's adjoint) on the tiles' active nodes
template <int D>
__global__ __launch_bounds__(AT) void k_jacT_final(Geo g, const uint8_t *__restrict__ nbm,
                                                   const uint8_t *__restrict__ anc_n, const double *__restrict__ w,
                                                   double *__restrict__ zk, const int32_t *__restrict__ tiles,
                                                   int ntile) {
  const int t = blockIdx.x;
  if (t >= ntile) return;
  const int64_t i = (tiles ? (int64_t)tiles[t] : (int64_t)t) * AT + threadIdx.x;
  if (i >= g.N || !(nbm[i] & 64u)) return;
  int64_t nb[2 * D];
  const int deg = jac_degree<D>(g, nbm, anc_n, i, nb);
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S + i;
    zk[o] += double(deg) * w[o];
  }
}

// transpose of the edge least-squares right-hand side (Eq. 57):
// F_bar_iA(m) (+)= dx/2 ([m-e_A act] (y_m - y_{m-e_A}) + [m+e_A act] (y_{m+e_A} - y_m))
template <int D, bool ADD>
__global__ __launch_bounds__(AT) void k_adj_rhsT(Geo g, const uint8_t *__restrict__ act, const double *__restrict__ y,
                                                 double *__restrict__ Fb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N || !act[i]) return;
  const C3 cc = coords_of(g, i);
  const double hdx = 0.5 * g.dx;
  for (int A = 0; A < D; ++A) {
    const int64_t lp = node_dir(g, cc, 2 * A, 1), lm = node_dir(g, cc, 2 * A + 1, 1);
    const bool hp = lp >= 0 && act[lp], hm = lm >= 0 && act[lm];
    for (int c = 0; c < D; ++c) {
      const size_t o = (size_t)c * g.S;
      double v = 0.0;
      if (hm) v += y[o + i] - y[o + lm];
      if (hp) v += y[o + lp] - y[o + i];
      double *t = Fb + (size_t)(c * D + A) * g.S + i;
      *t = ADD ? *t + hdx * v : hdx * v;
    }
  }
}

// transpose of the anchor targets u_D - (F_m - I)(X_b - X_m): F_bar_iA(m) -= off y_i(m)
template <int D>
__global__ __launch_bounds__(64) void k_adj_anchT(Links L, int64_t b0, int64_t b1, Geo g, const double *__restrict__ y,
                                                  double *__restrict__ Fb) {
  const int64_t l = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= b1) return;
  const int64_t m = L.node[l];
  const int q = L.q[l], A = q / 2;
  const double off = ((q & 1) ? -1.0 : 1.0) * L.eta[l] * g.dx;
  for (int i = 0; i < D; ++i) atomicAdd(&Fb[(size_t)(i * D + A) * g.S + m], -off * y[(size_t)i * g.S + m]);
}

// transpose of F^c = I + grad_dx u^c (Eq. 59; centred, one-sided next to a
// cut, evolved column kept when neither neighbour is active), gathered at
// node j; kept columns pass to Fext; ucb = x0b + grad^T Fcb
template <int D>
__global__ __launch_bounds__(AT) void k_adj_compatT(Geo g, const uint8_t *__restrict__ act,
                                                    const double *__restrict__ Fcb, const double *__restrict__ x0b,
                                                    double *__restrict__ ucb, double *__restrict__ Fext) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= g.N || !act[j]) return;
  const C3 cc = coords_of(g, j);
  const double idx = 1.0 / g.dx;
  double acc[D];
  for (int i = 0; i < D; ++i) acc[i] = x0b[(size_t)i * g.S + j];
  for (int A = 0; A < D; ++A) {
    const int64_t lp = node_dir(g, cc, 2 * A, 1), lm = node_dir(g, cc, 2 * A + 1, 1);
    const bool hp = lp >= 0 && act[lp], hm = lm >= 0 && act[lm];
    double clm = 0.0, clp = 0.0;  // j as the +A neighbour of lm, as the -A neighbour of lp
    if (hm) {
      const int64_t l2 = node_dir(g, coords_of(g, lm), 2 * A + 1, 1);
      clm = (l2 >= 0 && act[l2]) ? 0.5 * idx : idx;
    }
    if (hp) {
      const int64_t l2 = node_dir(g, coords_of(g, lp), 2 * A, 1);
      clp = (l2 >= 0 && act[l2]) ? -0.5 * idx : -idx;
    }
    const double cj = (hp && !hm) ? -idx : ((hm && !hp) ? idx : 0.0);
    for (int i = 0; i < D; ++i) {
      const size_t o = (size_t)(i * D + A) * g.S;
      if (hm) acc[i] += clm * Fcb[o + lm];
      if (hp) acc[i] += clp * Fcb[o + lp];
      acc[i] += cj * Fcb[o + j];
      Fext[o + j] = (!hp && !hm) ? Fcb[o + j] : 0.0;
    }
  }
  for (int i = 0; i < D; ++i) ucb[(size_t)i * g.S + j] = acc[i];
}

// --------------------------------------------- initialisation transpose
// f^0_q = feq(U0) - dt/2 feq'(U0)[Z_q], Z_q = U0_t + c e_qA d_A U0,
// U0_t = B0 - Phi'_A(U0) d_A U0 (Sec. 2.4, Eqs. 32-33).  f^0 is affine in
// v0 with slope (1 + gamma dt/2) feq'(U0); its (mu, lambda) derivative has
// three parts: feq, the equilibrium derivative and U0_t.
template <int D, typename T, bool MASK, bool TRACK>
__global__ __launch_bounds__(AT) void k_adj_init(const T *__restrict__ Lin, Geo g, AdjPar p,
                                                 const uint8_t *__restrict__ act, const double *__restrict__ U0,
                                                 const double *__restrict__ dU0, const double *__restrict__ lus,
                                                 double *__restrict__ gv0, double *__restrict__ gu0,
                                                 double *__restrict__ gdU0, double *__restrict__ gblk) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, row = blockIdx.y;
  const int64_t node = x + (int64_t)g.nx * row;
  double gm = 0.0, gl = 0.0;
  if (x < g.nx) {
    if (!MASK || act[node]) {
      const int y = row % g.ny, z = row / g.ny;
      double lam[Q][M], F[D * D], G[M];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t src = minus_eq(g, x, y, z, q);
#pragma unroll
        for (int r = 0; r < M; ++r) lam[q][r] = double(Lin[(size_t)(q * M + r) * g.S + src]);
      }
#pragma unroll
      for (int k = 0; k < D * D; ++k) F[k] = U0[(size_t)(D + k) * g.N + node];
#pragma unroll
      for (int r = 0; r < M; ++r) G[r] = 0.0;
      feq_vjp<D>(lam, F, p, 1.0, G, gm, gl);
      for (int i = 0; i < D; ++i) {
        const double lu = TRACK ? lus[(size_t)i * g.S + node] : 0.0;
        if (gv0) gv0[(size_t)i * g.N + node] = (1.0 + p.gamma * p.hdt) * G[i] - p.hdt * lu;
        if (gu0) gu0[(size_t)i * g.N + node] = lu;
      }
      if (gdU0) {
        // f_q = feq(U0) - dt/2 feq'_q(U0)[Z_q] with Z_q = B0 - sum_A Phi'_A d_A U0
        // + c e_qA d_A U0 (Eqs. 32-33) is affine in the gradient data:
        // dL/d(d_A U0) = -dt/2 sum_q (c e_qA w_q - Phi'_A^T w_q),
        // w_q = feq'_q^T lam_q = lam_q/(2D) + e_q Phi'_Aq^T lam_q/(2c)
        double gd[D][M];
#pragma unroll
        for (int A = 0; A < D; ++A)
#pragma unroll
          for (int r = 0; r < M; ++r) gd[A][r] = 0.0;
        for (int q = 0; q < Q; ++q) {
          const int Aq = q / 2;
          const double sg = (q & 1) ? -1.0 : 1.0;
          double w[M], t[M];
          flux_T<D>(lam[q], Aq, F, p, t);
#pragma unroll
          for (int r = 0; r < M; ++r) w[r] = lam[q][r] * p.i2D + sg * p.i2c * t[r];
          for (int A = 0; A < D; ++A) {
            flux_T<D>(w, A, F, p, t);
#pragma unroll
            for (int r = 0; r < M; ++r) gd[A][r] -= p.hdt * ((A == Aq ? p.c * sg * w[r] : 0.0) - t[r]);
          }
        }
        for (int A = 0; A < D; ++A)
          for (int r = 0; r < M; ++r) gdU0[((size_t)A * M + r) * g.N + node] = gd[A][r];
      }
      if (dU0) {
        double dA[D][M];
        for (int A = 0; A < D; ++A)
          for (int r = 0; r < M; ++r) dA[A][r] = dU0[((size_t)A * M + r) * g.N + node];
        // -dt/2 sum_q lam_q . (d feq'_q / dp)[Z_q]: only the v rows depend on
        // the parameters, through dP(F0)[Z_q,F] with
        // Z_q,F_iB = d_B v_i + c e_qA d_A F_iB
        for (int q = 0; q < Q; ++q) {
          const int A = q / 2;
          const double sg = (q & 1) ? -1.0 : 1.0;
          double Zf[D * D], dPm[D * D], dPl[D * D];
          for (int i = 0; i < D; ++i)
            for (int B = 0; B < D; ++B) Zf[i * D + B] = dA[B][i] + p.c * sg * dA[A][D + i * D + B];
          piola_tangent<D>(F, Zf, 1.0, 0.0, dPm);
          piola_tangent<D>(F, Zf, 0.0, 1.0, dPl);
          for (int i = 0; i < D; ++i) {
            const double cf = -p.hdt * lam[q][i] * p.i2c * sg * (-p.irho);
            gm += cf * dPm[i * D + A];
            gl += cf * dPl[i * D + A];
          }
        }
        // -dt/2 G . dU0_t/dp, dU0_t,v_i/dp = sum_A (d dP/dp)(F0)[d_A F]_iA / rho0
        for (int A = 0; A < D; ++A) {
          double dPm[D * D], dPl[D * D];
          piola_tangent<D>(F, dA[A] + D, 1.0, 0.0, dPm);
          piola_tangent<D>(F, dA[A] + D, 0.0, 1.0, dPl);
          for (int i = 0; i < D; ++i) {
            gm -= p.hdt * G[i] * dPm[i * D + A] * p.irho;
            gl -= p.hdt * G[i] * dPl[i * D + A] * p.irho;
          }
        }
      }
    } else {
      for (int i = 0; i < D; ++i) {
        if (gv0) gv0[(size_t)i * g.N + node] = 0.0;
        if (gu0) gu0[(size_t)i * g.N + node] = 0.0;
      }
      if (gdU0)
        for (int k = 0; k < D * (D + D * D); ++k) gdU0[(size_t)k * g.N + node] = 0.0;
    }
  }
  block_acc2(gm, gl, gblk + 2 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x));
}

// ------------------------------------------------------------------ host

inline void grid_of(const Geo &g, dim3 &grid, dim3 &block) {
  const int bx = g.nx >= 256 ? 256 : ((g.nx + 63) / 64) * 64;
  block = dim3(bx, 1, 1);
  grid = dim3((g.nx + bx - 1) / bx, g.ny * g.nz, 1);
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// device allocations of one reverse run, released on every exit path
// hands out the arena's blocks in request order (same order every call),
// reallocating a block that is too small
struct Pool {
  AdjArena *a;
  tlvlbm_ctx *c;
  size_t next = 0;
  template <typename X> hipError_t get(X **out, size_t bytes, hipStream_t st, bool zero = true) {
    bytes = bytes ? bytes : 16;
    if (next < a->blk.size() && a->bytes[next] < bytes) {
      dfree(c, a->blk[next]);
      a->blk[next] = nullptr;
      a->bytes[next] = 0;
    }
    if (next >= a->blk.size()) {
      a->blk.push_back(nullptr);
      a->bytes.push_back(0);
    }
    if (!a->blk[next]) {
      void *q = nullptr;
      const hipError_t e = dmalloc(c, &q, bytes);
      if (e != hipSuccess) return e;
      a->blk[next] = q;
      a->bytes[next] = bytes;
    }
    *out = (X *)a->blk[next++];
    return zero ? hipMemsetAsync(*out, 0, bytes, st) : hipSuccess;
  }
};

void arena_release(tlvlbm_ctx *c, AdjArena *a) {
  for (void *q : a->blk)
    if (q) dfree(c, q);
  a->blk.clear();
  a->bytes.clear();
  a->key[0] = a->key[1] = -1;
  a->avail = 0;
}

struct Run {
  tlvlbm_ctx *c;
  AdjPar ap;
  dim3 grid, block;
  size_t nblk = 0;
  bool neu = false, dir = false;
  // adjoint fields
  void *La = nullptr, *Lb = nullptr;
  double *lus = nullptr, *ubc = nullptr, *gbar = nullptr, *glink = nullptr, *gblk = nullptr, *ginit = nullptr;
  // projection
  double *UaB = nullptr, *Fcb = nullptr, *Fext = nullptr, *Frb = nullptr, *x0b = nullptr, *ucb = nullptr;
  // stencil gather
  int64_t ns = 0;
  int64_t *sn = nullptr, *so = nullptr;
  int32_t *el = nullptr, *sc = nullptr;
  double *ew = nullptr;
  // tape layout
  int64_t ts = 0;
  const int32_t *cpos = nullptr;
};

template <int D, typename T> void launch_link_pass(Run &R, int pass, double th, const TapeStep &tp) {
  tlvlbm_ctx *c = R.c;
  for (int b = 0; b < 256; ++b) {
    const int64_t b0 = c->bid_begin[b], b1 = c->bid_end[b];
    if (b1 <= b0) continue;
    const bool neu = c->bcs[b].type == TLVLBM_BC_NEUMANN_TRACTION;
    const unsigned nb = nblocks(b1 - b0, 64);
    const T *tU = (const T *)tp.U, *tF = (const T *)tp.Fr;
    const double *tu = (const double *)tp.u;
#define TL_LINK(P, NN)                                                                                         \
  hipLaunchKernelGGL((k_adj_link<D, T, P, NN>), nb, 64, 0, c->st, (T *)R.La, c->L, b0, b1, c->bcs[b], c->geo, \
                     c->par, th, tU, tF, R.ts, R.cpos, tu, R.sc, R.ns, R.gbar, R.glink)
    if (pass == 1) {
      if (neu) TL_LINK(1, true);
      else TL_LINK(1, false);
    } else if (pass == 2) {
      if (neu) TL_LINK(2, true);
      else TL_LINK(2, false);
    } else {
      if (neu) TL_LINK(3, true);
      else TL_LINK(3, false);
    }
#undef TL_LINK
  }
}

// exact mode: x0b = null-space part of (ua + ub); CG workspace b = the
// rest, x = 0; then x = K^+ b.  Jacobi mode: the transposed sweeps.
template <int D> int solve_adj(Run &R, const double *ua, const double *ub) {
  tlvlbm_ctx *c = R.c;
  CG &w = c->cg;
  const Geo &g = c->geo;
  const Gauge &G = *c->gauge;
  if (c->proj_sweeps > 0) {
    // Jacobi mode: the sweeps transposed in reverse order; y (the right-hand
    // side's adjoint) in w.x, the start's adjoint in x0b
    const uint8_t *an = R.dir ? G.anc_n : nullptr;
    const unsigned nb = nblocks(g.N, AT);
    const int nt = w.tiles ? w.ntiles : (int)nb;
    const int per = (nt + 7) / 8;
    double *wa = (double *)w.p0, *wb = (double *)w.r;
    if (!w.nbm) return TLVLBM_ERR_DEVICE;
    hipLaunchKernelGGL((k_jacT_seedw<D>), nb, AT, 0, c->st, g, w.nbm, an, ua, ub, wa, R.x0b, (double *)w.x);
    for (int k = 0; k < c->proj_sweeps; ++k) {
      hipLaunchKernelGGL((k_jacT_sweep<D>), (unsigned)(per * 8), AT, 0, c->st, g, w.nbm, an, (const double *)wa,
                         wb, (double *)w.x, c->proj_weight, w.tiles, nt, per);
      std::swap(wa, wb);
    }
    hipLaunchKernelGGL((k_jacT_final<D>), (unsigned)nt, AT, 0, c->st, g, w.nbm, an, (const double *)wa, R.x0b,
                       w.tiles, nt);
    return hipGetLastError() == hipSuccess ? TLVLBM_OK : TLVLBM_ERR_DEVICE;
  }
  gauge_means(c, ua, ub, G.mean);
  hipLaunchKernelGGL((k_pi_apply<D>), nblocks(g.N, AT), AT, 0, c->st, g, c->act, G.comp, G.mean, ua, ub, R.x0b,
                     (double *)w.b, (double *)w.x);
  if (!R.dir) return run_cg_given(c, nullptr);
  // the anchor counts go where the forward keeps them (one captured CG
  // graph serves both directions)
  if (hipMemcpyAsync(w.anc_n, G.anc_n, g.N, hipMemcpyDeviceToDevice, c->st) != hipSuccess) return TLVLBM_ERR_DEVICE;
  return run_cg_given(c, w.anc_n);
}

template <int D> void anchors_T(Run &R, const double *y, double *Fb) {
  tlvlbm_ctx *c = R.c;
  for (int b = 0; b < 256; ++b) {
    const int64_t b0 = c->bid_begin[b], b1 = c->bid_end[b];
    if (b1 <= b0 || c->bcs[b].type != TLVLBM_BC_DIRICHLET_VELOCITY) continue;
    hipLaunchKernelGGL((k_adj_anchT<D>), nblocks(b1 - b0, 64), 64, 0, c->st, c->L, b0, b1, c->geo, y, Fb);
  }
}

// reverse of step k: R.La holds the adjoint of that step's output, the
// result (adjoint of its input) goes to R.Lb; then the two swap
template <int D, typename T> int reverse_step(Run &R, int64_t k, const TapeStep &tp) {
  tlvlbm_ctx *c = R.c;
  const Geo &g = c->geo;
  const double th = k * c->par.dt + 0.5 * c->par.dt;
  const bool proj = is_projection_step(c, k);
  if (c->L.n) {
    launch_link_pass<D, T>(R, 1, th, tp);
    launch_link_pass<D, T>(R, 2, th, tp);
    launch_link_pass<D, T>(R, 3, th, tp);
  }
  if (R.ns)
    hipLaunchKernelGGL((k_adj_ugather<D>), nblocks(R.ns, AT), AT, 0, c->st, R.ns, R.sn, R.so, R.el, R.ew, g,
                       R.gbar, R.ubc);
  const T *Lout = (const T *)R.La;
  T *Lin = (T *)R.Lb;
  if (!proj) {
    const T *tU = (const T *)tp.U;
    if (c->act && c->chunks) {
      const unsigned nb = (unsigned)((c->nchunks + AT / CHUNK - 1) / (AT / CHUNK));
      if (c->track_u)
        hipLaunchKernelGGL((k_adj_bulk<D, T, true, true, true>), nb, AT, 0, c->st, Lout, Lin, g, R.ap, c->act, tU,
                           R.ts, R.ubc, R.lus, R.gblk, c->chunks, c->nchunks);
      else
        hipLaunchKernelGGL((k_adj_bulk<D, T, true, false, true>), nb, AT, 0, c->st, Lout, Lin, g, R.ap, c->act, tU,
                           R.ts, R.ubc, R.lus, R.gblk, c->chunks, c->nchunks);
    } else if (c->act) {
      if (c->track_u)
        hipLaunchKernelGGL((k_adj_bulk<D, T, true, true>), R.grid, R.block, 0, c->st, Lout, Lin, g, R.ap, c->act, tU,
                           R.ts, R.ubc, R.lus, R.gblk);
      else
        hipLaunchKernelGGL((k_adj_bulk<D, T, true, false>), R.grid, R.block, 0, c->st, Lout, Lin, g, R.ap, c->act,
                           tU, R.ts, R.ubc, R.lus, R.gblk);
    } else {
      if (c->track_u)
        hipLaunchKernelGGL((k_adj_bulk<D, T, false, true>), R.grid, R.block, 0, c->st, Lout, Lin, g, R.ap, c->act,
                           tU, R.ts, R.ubc, R.lus, R.gblk);
      else
        hipLaunchKernelGGL((k_adj_bulk<D, T, false, false>), R.grid, R.block, 0, c->st, Lout, Lin, g, R.ap, c->act,
                           tU, R.ts, R.ubc, R.lus, R.gblk);
    }
  } else {
    CG &w = c->cg;
    // second projection (u from F^r, warm start u^c) and u* = u + dt/2 v
    int s = solve_adj<D>(R, R.ubc, R.lus);
    if (s) return s;
    hipLaunchKernelGGL((k_adj_rhsT<D, false>), nblocks(g.N, AT), AT, 0, c->st, g, c->act, (const double *)w.x, R.Frb);
    anchors_T<D>(R, (const double *)w.x, R.Frb);
    hipLaunchKernelGGL((k_adj_rep1<D, T>), R.grid, R.block, 0, c->st, Lout, g, R.ap, c->act, (const T *)tp.U,
                       (const T *)tp.Fr, R.ts, R.cpos, R.Frb, R.lus, R.UaB, R.Fcb, R.gblk);
    hipLaunchKernelGGL((k_adj_compatT<D>), nblocks(g.N, AT), AT, 0, c->st, g, c->act, R.Fcb, R.x0b, R.ucb, R.Fext);
    // first projection (u^c from F, warm start u)
    s = solve_adj<D>(R, R.ucb, nullptr);
    if (s) return s;
    hipLaunchKernelGGL((k_adj_rhsT<D, true>), nblocks(g.N, AT), AT, 0, c->st, g, c->act, (const double *)w.x, R.Fext);
    anchors_T<D>(R, (const double *)w.x, R.Fext);
    hipLaunchKernelGGL((k_adj_rep2<D, T>), R.grid, R.block, 0, c->st, Lout, Lin, g, R.ap, c->act, R.UaB, R.Fext,
                       R.x0b, R.lus);
  }
  std::swap(R.La, R.Lb);
  return hipGetLastError() == hipSuccess ? TLVLBM_OK : TLVLBM_ERR_DEVICE;
}

// host preparation: the transposed LSQ stencils of the Neumann links
// transposed LSQ stencils of the Neumann links (built once per geometry and
// set of conditions, kept in the context): a counting sort by node keeps the
// (link, point) order within each node, so the gather is deterministic
int stencil_transpose(tlvlbm_ctx *c) {
  const int64_t nl = c->L.n, N = c->geo.N;
  const int D = c->D;
  std::vector<int32_t> lnp(nl), sidx((size_t)nl * c->L.kmax);
  std::vector<double> sw((size_t)nl * c->L.kmax * (D - 1));
  if (nl) {
    if (hipMemcpy(lnp.data(), c->L.npts, nl * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(sidx.data(), c->L.sidx, sidx.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(sw.data(), c->L.sw, sw.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return TLVLBM_ERR_DEVICE;
  }
  std::vector<uint8_t> is_neu(nl, 0);
  for (int b = 0; b < 256; ++b)
    for (int64_t l = c->bid_begin[b]; l < c->bid_end[b]; ++l)
      is_neu[l] = c->bcs[b].type == TLVLBM_BC_NEUMANN_TRACTION;
  std::vector<int64_t> cnt(N + 1, 0);
  for (int64_t l = 0; l < nl; ++l)
    if (is_neu[l])
      for (int k = 0; k < lnp[l]; ++k) cnt[sidx[lsq_i(c->L, l, k)] + 1]++;
  std::vector<int64_t> sn, so;
  for (int64_t j = 0; j < N; ++j)
    if (cnt[j + 1]) sn.push_back(j);
  for (int64_t j = 0; j < N; ++j) cnt[j + 1] += cnt[j];
  const int64_t ne = cnt[N];
  std::vector<int32_t> el(ne), ek(ne);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t l = 0; l < nl; ++l)
    if (is_neu[l])
      for (int k = 0; k < lnp[l]; ++k) {
        const int64_t e = pos[sidx[lsq_i(c->L, l, k)]]++;
        el[e] = (int32_t)l;
        ek[e] = k;
      }
  for (int64_t j : sn) so.push_back(cnt[j]);
  so.push_back(ne);
  // tangent weights in entry order; compact tape index of every stencil slot
  std::vector<double> ew((size_t)ne * (D - 1));
  for (int64_t e = 0; e < ne; ++e)
    for (int al = 0; al < D - 1; ++al) ew[(size_t)e * (D - 1) + al] = sw[lsq_w(c->L, el[e], al, ek[e])];
  std::vector<int32_t> sc(sidx.size(), 0);
  {
    std::vector<int32_t> at(N, -1);
    for (size_t t = 0; t < sn.size(); ++t) at[sn[t]] = (int32_t)t;
    for (int64_t l = 0; l < nl; ++l)
      if (is_neu[l])
        for (int k = 0; k < lnp[l]; ++k) sc[lsq_i(c->L, l, k)] = at[sidx[lsq_i(c->L, l, k)]];
  }
  StencilT *T = new (std::nothrow) StencilT();
  if (!T) return TLVLBM_ERR_OUT_OF_MEMORY;
  T->ns = (int64_t)sn.size();
  if (T->ns) {
    if (dmalloc(c, &T->sn, sn.size() * sizeof(int64_t)) || dmalloc(c, &T->so, so.size() * sizeof(int64_t)) ||
        dmalloc(c, &T->el, el.size() * sizeof(int32_t)) || dmalloc(c, &T->ek, ek.size() * sizeof(int32_t)) ||
        dmalloc(c, &T->ew, ew.size() * sizeof(double)) || dmalloc(c, &T->sc, sc.size() * sizeof(int32_t)) ||
        hipMemcpy(T->sn, sn.data(), sn.size() * sizeof(int64_t), hipMemcpyHostToDevice) ||
        hipMemcpy(T->so, so.data(), so.size() * sizeof(int64_t), hipMemcpyHostToDevice) ||
        hipMemcpy(T->el, el.data(), el.size() * sizeof(int32_t), hipMemcpyHostToDevice) ||
        hipMemcpy(T->ek, ek.data(), ek.size() * sizeof(int32_t), hipMemcpyHostToDevice) ||
        hipMemcpy(T->ew, ew.data(), ew.size() * sizeof(double), hipMemcpyHostToDevice) ||
        hipMemcpy(T->sc, sc.data(), sc.size() * sizeof(int32_t), hipMemcpyHostToDevice)) {
      for (void *p : {(void *)T->sn, (void *)T->so, (void *)T->el, (void *)T->ek, (void *)T->ew, (void *)T->sc})
        dfree(c, p);
      delete T;
      return TLVLBM_ERR_OUT_OF_MEMORY;
    }
  }
  c->stT = T;
  return TLVLBM_OK;
}

// projection solutions of recorded step k: stored by the first pass (mode 1),
// replayed by the recomputation (mode 2)
inline void rec_xs(const AdjRec &rec, int64_t k, TapeStep &tp, int mode) {
  tp.xs[0] = tp.xs[1] = nullptr;
  tp.xmode = 0;
  if (rec.xstore && rec.pidx[k] >= 0) {
    tp.xs[0] = rec.xstore + (size_t)(2 * rec.pidx[k]) * rec.xslot;
    tp.xs[1] = rec.xstore + (size_t)(2 * rec.pidx[k] + 1) * rec.xslot;
    tp.xmode = mode;
  }
}

// the launch geometry and flags of a reverse run (the same in the record and
// the backward call)
template <int D, typename T> void run_setup(Run &R, tlvlbm_ctx *c) {
  const Geo &g = c->geo;
  const Par &pp = c->par;
  R.c = c;
  R.ap = AdjPar{pp.omega,
                pp.dt * (2.0 - pp.omega) / (4.0 * D),
                1.0 / (1.0 + 0.5 * pp.gamma * pp.dt),
                0.5 * pp.dt,
                1.0 / (2.0 * D),
                0.5 / pp.c,
                pp.inv_rho0,
                pp.mu,
                pp.lam,
                pp.gamma,
                pp.c,
                pp.dt,
                c->theta,
                g.dx,
                pp.k1,
                {pp.a0[0], pp.a0[1], pp.a0[2]}};
  grid_of(g, R.grid, R.block);
  // per-block parameter-gradient slots: row blocks and chunk blocks
  R.nblk = std::max((size_t)R.grid.x * R.grid.y, (size_t)(c->nchunks + AT / CHUNK - 1) / (AT / CHUNK));
  for (int b = 0; b < 256; ++b) {
    if (c->bid_end[b] <= c->bid_begin[b]) continue;
    if (c->bcs[b].type == TLVLBM_BC_NEUMANN_TRACTION) R.neu = true;
    if (c->bcs[b].type == TLVLBM_BC_DIRICHLET_VELOCITY) R.dir = true;
  }
  R.ts = tape_stride(c);
  R.cpos = (c->act && c->chunks) ? c->cpos : nullptr;
}

// sizes of the checkpoint and tape blocks
struct TapeSizes {
  size_t plane, dplane, tplane, ck_bytes, tapeu_bytes, tape_bytes, trF_bytes;
  int64_t nu;
};

template <int D, typename T> TapeSizes tape_sizes(const Run &R, tlvlbm_ctx *c) {
  constexpr int Q = 2 * D, M = D + D * D;
  TapeSizes z;
  z.plane = (size_t)c->geo.S * sizeof(T);
  z.dplane = (size_t)c->geo.S * sizeof(double);
  z.nu = (R.neu && c->stT) ? c->stT->ns : 0;
  z.tplane = (size_t)R.ts * sizeof(T);
  z.ck_bytes = (size_t)Q * M * z.plane + (c->track_u ? D * z.dplane : 0);
  z.tapeu_bytes = (size_t)D * std::max<int64_t>(z.nu, 1) * sizeof(double);
  z.tape_bytes = (size_t)D * D * z.tplane + (R.neu ? z.tapeu_bytes : 0);
  z.trF_bytes = (size_t)D * D * z.tplane;
  return z;
}

// First pass of the reverse mode: n forward steps from the fresh state with
// checkpoints of the stored field and the tape of the final steps, leaving
// the context at step n.  Everything the backward pass needs stays in the
// context's arena and record.
template <int D, typename T>
tlvlbm_status record_t(tlvlbm_ctx *c, int64_t n, const double *U0, const double *dU0, int64_t seg,
                       std::string &err) {
  constexpr int Q = 2 * D, M = D + D * D;
  const Geo &g = c->geo;
  hipStream_t st = c->st;
  if (!c->arena) c->arena = new AdjArena();
  if (!c->rec) c->rec = new AdjRec();
  AdjRec &rec = *c->rec;
  rec.valid = false;
  Pool pool{c->arena, c};
  Run R;
  run_setup<D, T>(R, c);
  const bool track = c->track_u;
  // projection tables first: rebuilding them frees the transposed stencils,
  // which the tape below refers to, so no step of this call may rebuild them
  if (c->act && (R.neu || R.dir) && (!c->gauge || c->aux_stale)) {
    const int s = proj_aux_build(c);
    if (s) return (tlvlbm_status)s;
  }
  // transposed Neumann stencils: the gather of u_bar, and the nodes whose
  // displacement the tape keeps
  if (c->act && R.neu && !c->stT) {
    const int s = stencil_transpose(c);
    if (s) return (tlvlbm_status)s;
  }
  // tape: F - I of every step and F^r of projection steps in chunk slots
  // (population precision), u at the Neumann stencil nodes (FP64)
  const TapeSizes z = tape_sizes<D, T>(R, c);
  const size_t plane = z.plane, dplane = z.dplane;
  const bool has_proj = R.neu && c->proj_every > 0;
  auto nproj_in = [&](int64_t k0, int64_t k1) {
    int64_t np = 0;
    for (int64_t k = k0; k < k1; ++k) np += is_projection_step(c, k) ? 1 : 0;
    return np;
  };
  // Schedule.  With a caller's segment length: checkpoints every seg steps,
  // each segment recomputed once with its tape.  By default the last `tail`
  // steps keep their tape from the first pass (as many as 60% of the free
  // device memory holds; at most -seg of them for seg < 0) and only the
  // steps before them are checkpointed and recomputed, in segments of
  // ~sqrt(steps * checkpoint / tape step).
  const int64_t seg_arg = seg;
  AdjArena &ar = *c->arena;
  int64_t tail = 0;
  size_t avail = 0;
  const size_t init_bytes = (size_t)M * g.N * sizeof(double) + (dU0 ? (size_t)D * M * g.N * sizeof(double) : 0);
  if (ar.key[0] != n || ar.key[1] != seg_arg) {
    arena_release(c, &ar);
    size_t fixed = 2 * (size_t)Q * M * plane + 2 * (size_t)D * dplane + 2 * z.ck_bytes + init_bytes +
                   (size_t)D * M * dplane;
    if (R.neu) fixed += (size_t)(M + 3 * D * D + 2 * D) * dplane;
    if (z.nu) fixed += (size_t)z.nu * (3 * 8 + 8 * (D + 1)) + (size_t)c->L.n * c->L.kmax * 4;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
    if (seg_arg <= 0 && fr > fixed) {
      const double per_step = (double)z.tape_bytes + (has_proj ? (double)z.trF_bytes / c->proj_every : 0.0);
      tail = std::min<int64_t>(n, (int64_t)(0.6 * (double)(fr - fixed) / per_step));
      if (seg_arg < 0) tail = std::min<int64_t>(tail, -seg_arg);
      tail = std::max<int64_t>(tail, 0);
    }
    const int64_t head = n - tail;
    if (seg_arg <= 0) {
      seg = (int64_t)std::ceil(std::sqrt((double)std::max<int64_t>(head, 1) * (double)z.ck_bytes /
                                         (double)z.tape_bytes));
      seg = std::max<int64_t>(1, std::min<int64_t>(seg, std::max<int64_t>(head, 1)));
    }
    const int64_t nck_ = head > 0 ? (head + seg - 1) / seg : 0;
    const int64_t nps = has_proj ? seg / c->proj_every + 2 : 0;
    size_t need = fixed + (size_t)(nck_ + 1) * z.ck_bytes + (head > 0 ? (size_t)seg * z.tape_bytes : 0) +
                  (head > 0 ? (size_t)nps * z.trF_bytes : 0) + (size_t)tail * z.tape_bytes +
                  (size_t)nproj_in(head, n) * z.trF_bytes;
    if (fr && need > fr) {
      err = "adjoint: checkpoints and tape do not fit in device memory (lower the step count or pass a segment length)";
      return TLVLBM_ERR_OUT_OF_MEMORY;
    }
    ar.avail = fr > need ? fr - need : 0;
    ar.key[0] = n;
    ar.key[1] = seg_arg;
    ar.seg = seg;
    ar.tail = tail;
  }
  seg = ar.seg;
  tail = ar.tail;
  avail = ar.avail;
  const int64_t head = n - tail;
  const int64_t nck = head > 0 ? (head + seg - 1) / seg : 0;
  if (R.neu || R.dir) {
    const int s = ensure_cg(c);
    if (s) return (tlvlbm_status)s;
  }
  // the initial data, kept for the initialisation's transpose
  {
    DevIn dU0d, ddU0;
    if (dU0d.take(U0, (size_t)M * g.N * sizeof(double), st) ||
        ddU0.take(dU0, (size_t)D * M * g.N * sizeof(double), st))
      return TLVLBM_ERR_OUT_OF_MEMORY;
    if (pool.get(&rec.U0, (size_t)M * g.N * sizeof(double), st, false) ||
        hipMemcpyAsync(rec.U0, dU0d.ptr, (size_t)M * g.N * sizeof(double), hipMemcpyDeviceToDevice, st))
      return TLVLBM_ERR_OUT_OF_MEMORY;
    rec.dU0 = nullptr;
    if (dU0 && (pool.get(&rec.dU0, (size_t)D * M * g.N * sizeof(double), st, false) ||
                hipMemcpyAsync(rec.dU0, ddU0.ptr, (size_t)D * M * g.N * sizeof(double), hipMemcpyDeviceToDevice,
                               st)))
      return TLVLBM_ERR_OUT_OF_MEMORY;
    if (hipStreamSynchronize(st) != hipSuccess) return TLVLBM_ERR_DEVICE;  // before the DevIn copies go
  }
  // forward with checkpoints
  rec.ckf.assign(nck + 1, nullptr);
  rec.cku.assign(nck + 1, nullptr);
  for (int64_t s = 0; s <= nck; ++s) {
    if (pool.get(&rec.ckf[s], (size_t)Q * M * plane, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
    if (track && pool.get(&rec.cku[s], (size_t)D * dplane, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
  }
  auto save = [&](int64_t s) -> bool {
    if (hipMemcpyAsync(rec.ckf[s], c->fB, (size_t)Q * M * plane, hipMemcpyDeviceToDevice, st)) return false;
    if (track && hipMemcpyAsync(rec.cku[s], c->ustar, (size_t)D * dplane, hipMemcpyDeviceToDevice, st)) return false;
    return true;
  };
  // the projection solutions of the first pass are kept (active tiles, FP64)
  // when they fit in a quarter of the free memory, so that the recomputation
  // replays them instead of solving again
  const int64_t nproj = nproj_in(0, head);
  rec.xstore = nullptr;
  rec.xslot = 0;
  if (nproj && c->cg.tiles) {
    rec.xslot = (size_t)D * c->cg.ntiles * 256;
    const size_t xbytes = (size_t)nproj * 2 * rec.xslot * sizeof(double);
    if (xbytes <= avail / 4 && pool.get(&rec.xstore, xbytes, st, false)) rec.xstore = nullptr;
  }
  rec.pidx.assign(n, -1);
  for (int64_t k = 0, p = 0; k < head; ++k)
    if (is_projection_step(c, k)) rec.pidx[k] = p++;
  // the tail's tape, written by the first pass
  char *tailU = nullptr, *tailu = nullptr, *tailF = nullptr;
  rec.ttp.assign((size_t)tail, TapeStep{});
  if (tail > 0) {
    const int64_t ntp = nproj_in(head, n);
    if (pool.get(&tailU, (size_t)tail * D * D * z.tplane, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
    if (R.neu && z.nu && pool.get(&tailu, (size_t)tail * z.tapeu_bytes, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
    if (ntp && pool.get(&tailF, (size_t)ntp * z.trF_bytes, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
    int64_t ip = 0;
    for (int64_t k = head; k < n; ++k) {
      TapeStep &tp = rec.ttp[k - head];
      tp.U = tailU + (size_t)(k - head) * D * D * z.tplane;
      tp.u = (R.neu && z.nu) ? tailu + (size_t)(k - head) * z.tapeu_bytes : nullptr;
      tp.un = c->stT ? c->stT->sn : nullptr;
      tp.nu = z.nu;
      tp.Fr = is_projection_step(c, k) ? tailF + (size_t)(ip++) * z.trF_bytes : nullptr;
    }
  }
  rec.n = n;
  rec.seg = seg;
  rec.tail = tail;
  rec.nck = nck;
  for (int64_t k = 0; k < n; ++k) {
    if (k < head && k % seg == 0 && !save(k / seg)) return TLVLBM_ERR_DEVICE;
    TapeStep tp{};
    if (k >= head) tp = rec.ttp[k - head];
    rec_xs(rec, k, tp, 1);
    const int s = step_once(c, &tp);
    if (s) return (tlvlbm_status)s;
  }
  if (!save(nck)) return TLVLBM_ERR_DEVICE;
  {
    const tlvlbm_status s = check_flag(c);
    if (s) return s;
  }
  rec.pool_next = pool.next;
  rec.valid = true;
  return TLVLBM_OK;
}

// Backward pass: the gradient of L = sum dLdU . U + dLdu . u over the final
// moments of the recorded run, with respect to (mu, lambda), v0, u0 and the
// initial gradient data dU0.  The recorded segments are recomputed from
// their checkpoints; the context returns to the end of the trajectory.
template <int D, typename T>
tlvlbm_status backward_t(tlvlbm_ctx *c, const double *dLdU, const double *dLdu, double *gmat, double *gv0,
                         double *gu0, double *gdU0, std::string &err) {
  constexpr int Q = 2 * D, M = D + D * D;
  const Geo &g = c->geo;
  hipStream_t st = c->st;
  AdjRec &rec = *c->rec;
  Pool pool{c->arena, c};
  pool.next = rec.pool_next;
  Run R;
  run_setup<D, T>(R, c);
  const bool track = c->track_u;
  const TapeSizes z = tape_sizes<D, T>(R, c);
  const size_t plane = z.plane, dplane = z.dplane;
  const bool has_proj = R.neu && c->proj_every > 0;
  const int64_t n = rec.n, seg = rec.seg, tail = rec.tail, head = n - tail, nck = rec.nck;
  const int64_t nproj_seg = has_proj ? seg / c->proj_every + 2 : 0;
  auto restore = [&](int64_t s) -> bool {
    if (hipMemcpyAsync(c->fB, rec.ckf[s], (size_t)Q * M * plane, hipMemcpyDeviceToDevice, st)) return false;
    if (track && hipMemcpyAsync(c->ustar, rec.cku[s], (size_t)D * dplane, hipMemcpyDeviceToDevice, st)) return false;
    return true;
  };
  DevIn dLU, dLu;
  if (dLU.take(dLdU, (size_t)M * g.N * sizeof(double), st) || dLu.take(dLdu, (size_t)D * g.N * sizeof(double), st))
    return TLVLBM_ERR_OUT_OF_MEMORY;
  // adjoint buffers
  if (pool.get(&R.La, (size_t)Q * M * plane, st) || pool.get(&R.Lb, (size_t)Q * M * plane, st) ||
      pool.get(&R.lus, (size_t)D * dplane, st) || pool.get(&R.ubc, (size_t)D * dplane, st) ||
      pool.get(&R.gbar, (size_t)std::max<int64_t>(c->L.n, 1) * 6 * sizeof(double), st) ||
      pool.get(&R.glink, (size_t)std::max<int64_t>(c->L.n, 1) * 2 * sizeof(double), st) ||
      pool.get(&R.gblk, R.nblk * 2 * sizeof(double), st) || pool.get(&R.ginit, R.nblk * 2 * sizeof(double), st))
    return TLVLBM_ERR_OUT_OF_MEMORY;
  if (R.neu) {
    if (pool.get(&R.UaB, (size_t)M * dplane, st) || pool.get(&R.Fcb, (size_t)D * D * dplane, st) ||
        pool.get(&R.Fext, (size_t)D * D * dplane, st) || pool.get(&R.Frb, (size_t)D * D * dplane, st) ||
        pool.get(&R.x0b, (size_t)D * dplane, st) || pool.get(&R.ucb, (size_t)D * dplane, st))
      return TLVLBM_ERR_OUT_OF_MEMORY;
  }
  if (c->act) {
    // (the record builds them when Neumann links exist: no tape refers to
    // them otherwise, and the projection tables are current)
    if (!c->stT) {
      const int s = stencil_transpose(c);
      if (s) return (tlvlbm_status)s;
    }
    R.ns = c->stT->ns;
    R.sn = c->stT->sn;
    R.so = c->stT->so;
    R.el = c->stT->el;
    R.ew = c->stT->ew;
    R.sc = c->stT->sc;
  }
  // per-step tape of one segment
  char *tapeU = nullptr, *tapeu = nullptr, *tapeF = nullptr;
  if (head > 0) {
    if (pool.get(&tapeU, (size_t)seg * D * D * z.tplane, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
    if (R.neu && pool.get(&tapeu, (size_t)seg * z.tapeu_bytes, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
    if (nproj_seg && pool.get(&tapeF, (size_t)nproj_seg * z.trF_bytes, st, false)) return TLVLBM_ERR_OUT_OF_MEMORY;
  }
  // seeds
  {
    const double *gU = (const double *)dLU.ptr, *gu = (const double *)dLu.ptr;
    if (c->act) {
      if (track)
        hipLaunchKernelGGL((k_adj_seed<D, T, true, true>), R.grid, R.block, 0, st, (T *)R.La, g, R.ap, c->act, gU, gu,
                           R.lus);
      else
        hipLaunchKernelGGL((k_adj_seed<D, T, true, false>), R.grid, R.block, 0, st, (T *)R.La, g, R.ap, c->act, gU,
                           gu, R.lus);
    } else {
      if (track)
        hipLaunchKernelGGL((k_adj_seed<D, T, false, true>), R.grid, R.block, 0, st, (T *)R.La, g, R.ap, c->act, gU,
                           gu, R.lus);
      else
        hipLaunchKernelGGL((k_adj_seed<D, T, false, false>), R.grid, R.block, 0, st, (T *)R.La, g, R.ap, c->act, gU,
                           gu, R.lus);
    }
  }
  // the tail in reverse from the first pass's tape, then the head's
  // segments in reverse: recompute with the tape, then reverse each step
  const int64_t st_proj0 = c->st_proj;
  for (int64_t k = n - 1; k >= head; --k) {
    const int e = reverse_step<D, T>(R, k, rec.ttp[k - head]);
    if (e) return (tlvlbm_status)e;
  }
  for (int64_t s = nck - 1; s >= 0; --s) {
    const int64_t k0 = s * seg, k1 = std::min<int64_t>(head, k0 + seg);
    if (!restore(s)) return TLVLBM_ERR_DEVICE;
    c->step = k0;
    std::vector<TapeStep> tps(k1 - k0);
    int64_t ip = 0;
    for (int64_t k = k0; k < k1; ++k) {
      TapeStep &tp = tps[k - k0];
      tp.U = tapeU + (size_t)(k - k0) * D * D * z.tplane;
      // (no stencil node: no Neumann link reads the displacement)
      tp.u = (R.neu && R.ns) ? tapeu + (size_t)(k - k0) * z.tapeu_bytes : nullptr;
      tp.un = R.sn;
      tp.nu = R.ns;
      tp.Fr = nullptr;
      rec_xs(rec, k, tp, 2);
      if (is_projection_step(c, k)) {
        if (ip >= nproj_seg) return TLVLBM_ERR_INVALID_ARG;
        tp.Fr = tapeF + (size_t)(ip++) * z.trF_bytes;
      }
      const int e = step_once(c, &tp);
      if (e) return (tlvlbm_status)e;
    }
    for (int64_t k = k1 - 1; k >= k0; --k) {
      const int e = reverse_step<D, T>(R, k, tps[k - k0]);
      if (e) return (tlvlbm_status)e;
    }
  }
  c->st_proj = st_proj0;  // recomputation is not counted as progress
  // initialisation transpose
  DevOut ov, ou, od;
  if (ov.take(gv0, (size_t)D * g.N * sizeof(double)) || ou.take(gu0, (size_t)D * g.N * sizeof(double)) ||
      od.take(gdU0, (size_t)D * M * g.N * sizeof(double)))
    return TLVLBM_ERR_OUT_OF_MEMORY;
  {
    const double *u0p = rec.U0, *du0p = rec.dU0;
    double *pv = (double *)ov.ptr, *pu = (double *)ou.ptr, *pd = (double *)od.ptr;
    if (c->act) {
      if (track)
        hipLaunchKernelGGL((k_adj_init<D, T, true, true>), R.grid, R.block, 0, st, (const T *)R.La, g, R.ap, c->act,
                           u0p, du0p, R.lus, pv, pu, pd, R.ginit);
      else
        hipLaunchKernelGGL((k_adj_init<D, T, true, false>), R.grid, R.block, 0, st, (const T *)R.La, g, R.ap, c->act,
                           u0p, du0p, R.lus, pv, pu, pd, R.ginit);
    } else {
      if (track)
        hipLaunchKernelGGL((k_adj_init<D, T, false, true>), R.grid, R.block, 0, st, (const T *)R.La, g, R.ap, c->act,
                           u0p, du0p, R.lus, pv, pu, pd, R.ginit);
      else
        hipLaunchKernelGGL((k_adj_init<D, T, false, false>), R.grid, R.block, 0, st, (const T *)R.La, g, R.ap,
                           c->act, u0p, du0p, R.lus, pv, pu, pd, R.ginit);
    }
  }
  if (hipGetLastError() != hipSuccess) return TLVLBM_ERR_DEVICE;
  if (ov.finish(st) || ou.finish(st) || od.finish(st)) return TLVLBM_ERR_DEVICE;
  // parameter gradient: fixed-order host sum of the per-block and per-link slots
  std::vector<double> hb(R.nblk * 2), hi(R.nblk * 2), hl((size_t)std::max<int64_t>(c->L.n, 1) * 2);
  if (hipMemcpyAsync(hb.data(), R.gblk, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(hi.data(), R.ginit, hi.size() * sizeof(double), hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(hl.data(), R.glink, hl.size() * sizeof(double), hipMemcpyDeviceToHost, st))
    return TLVLBM_ERR_DEVICE;
  // back to the end of the trajectory
  if (!restore(nck)) return TLVLBM_ERR_DEVICE;
  c->step = n;
  if (hipStreamSynchronize(st) != hipSuccess) return TLVLBM_ERR_DEVICE;
  double gsum[2] = {0.0, 0.0};
  for (size_t b = 0; b < R.nblk; ++b)
    for (int k = 0; k < 2; ++k) gsum[k] += hb[2 * b + k];
  for (size_t l = 0; l < (size_t)c->L.n; ++l)
    for (int k = 0; k < 2; ++k) gsum[k] += hl[2 * l + k];
  for (size_t b = 0; b < R.nblk; ++b)
    for (int k = 0; k < 2; ++k) gsum[k] += hi[2 * b + k];
  if (gmat) {
    gmat[0] = gsum[0];
    gmat[1] = gsum[1];
  }
  (void)err;
  return check_flag(c);
}

}  // namespace
}  // namespace tl

using namespace tl;

namespace {

tlvlbm_status adjoint_fail(tlvlbm_ctx *c, tlvlbm_status s, const std::string &err, const char *what) {
  if (s) {
    c->status = s;
    if (c->rec) c->rec->valid = false;
    try {
      c->err = err.empty() ? std::string(what) : err;
    } catch (...) {
    }
  }
  return s;
}

tlvlbm_status record_call(tlvlbm_ctx *c, int64_t n, const double *U0, const double *dU0, int64_t segment) {
  if (!c->have_state || !c->fresh) {
    c->err = "adjoint: the state must be the one set by tlvlbm_set_state (no step since)";
    return TLVLBM_ERR_CALL_ORDER;
  }
  if (c->bf) {
    c->err = "adjoint: no reverse mode with a body acceleration";
    return TLVLBM_ERR_INVALID_ARG;
  }
  if (c->visco) {
    c->err = "adjoint: no reverse mode through a Maxwell branch";
    return TLVLBM_ERR_INVALID_ARG;
  }
  if (c->par.thf) {
    c->err = "adjoint: no reverse mode with a thermal stretch";
    return TLVLBM_ERR_INVALID_ARG;
  }
  std::string err;
  tlvlbm_status s;
  try {
    if (c->D == 2)
      s = c->prec ? record_t<2, double>(c, n, U0, dU0, segment, err) : record_t<2, float>(c, n, U0, dU0, segment, err);
    else
      s = c->prec ? record_t<3, double>(c, n, U0, dU0, segment, err) : record_t<3, float>(c, n, U0, dU0, segment, err);
  } catch (...) {
    err = "adjoint: host allocation failed";
    s = TLVLBM_ERR_OUT_OF_MEMORY;
  }
  c->fresh = false;
  return adjoint_fail(c, s, err, "adjoint record failed");
}

tlvlbm_status backward_call(tlvlbm_ctx *c, const double *dLdU, const double *dLdu, double *grad_mat, double *grad_v0,
                            double *grad_u0, double *grad_dU0) {
  if (!c->rec || !c->rec->valid || c->step != c->rec->n) {
    c->err = "adjoint: no recorded run ending at the current state (tlvlbm_adjoint_record, no change since)";
    return TLVLBM_ERR_CALL_ORDER;
  }
  std::string err;
  tlvlbm_status s;
  try {
    if (c->D == 2)
      s = c->prec ? backward_t<2, double>(c, dLdU, dLdu, grad_mat, grad_v0, grad_u0, grad_dU0, err)
                  : backward_t<2, float>(c, dLdU, dLdu, grad_mat, grad_v0, grad_u0, grad_dU0, err);
    else
      s = c->prec ? backward_t<3, double>(c, dLdU, dLdu, grad_mat, grad_v0, grad_u0, grad_dU0, err)
                  : backward_t<3, float>(c, dLdU, dLdu, grad_mat, grad_v0, grad_u0, grad_dU0, err);
  } catch (...) {
    err = "adjoint: host allocation failed";
    s = TLVLBM_ERR_OUT_OF_MEMORY;
  }
  return adjoint_fail(c, s, err, "adjoint backward failed");
}

}  // namespace

extern "C" tlvlbm_status tlvlbm_adjoint_record(tlvlbm_ctx *c, int64_t n, const double *U0, const double *dU0,
                                               int64_t segment) {
  if (!c || n < 0 || !U0) return TLVLBM_ERR_INVALID_ARG;
  if (c->status) return (tlvlbm_status)c->status;
  return record_call(c, n, U0, dU0, segment);
}

extern "C" tlvlbm_status tlvlbm_adjoint_backward(tlvlbm_ctx *c, const double *dLdU, const double *dLdu,
                                                 double *grad_mat, double *grad_v0, double *grad_u0,
                                                 double *grad_dU0) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  if (c->status) return (tlvlbm_status)c->status;
  return backward_call(c, dLdU, dLdu, grad_mat, grad_v0, grad_u0, grad_dU0);
}

extern "C" tlvlbm_status tlvlbm_adjoint_step(tlvlbm_ctx *c, int64_t n, const double *U0, const double *dU0,
                                        const double *dLdU, const double *dLdu, double *grad_mat, double *grad_v0,
                                        double *grad_u0, int64_t segment) {
  if (!c || n < 0 || !U0) return TLVLBM_ERR_INVALID_ARG;
  if (c->status) return (tlvlbm_status)c->status;
  const tlvlbm_status s = record_call(c, n, U0, dU0, segment);
  if (s) return s;
  return backward_call(c, dLdU, dLdu, grad_mat, grad_v0, grad_u0, nullptr);
}
