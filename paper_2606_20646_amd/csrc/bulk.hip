// Bulk kernels of the TL-VLBM update on gfx950.
//
// Storage.  Populations live in structure-of-arrays planes, plane (q, r) at
// offset (q*M + r) * S, node x fastest.  The stored field between steps is the
// post-collision, pre-streaming population f*, so one fused kernel pulls
// f*_q(X - e_q) (streaming, Sec. 2.4, Eq. 31), recovers the state (Eq. 28),
// collides (Eq. 29) and writes f*(X) for the next step: one read and one write
// of every population per step.  A population that would have to come from
// outside the body (missing direction of a cut link) is deposited by the
// cut-link kernel into the pull slot of the outside (inactive) node, so the
// bulk kernel never branches on geometry.
//
// Precision.  Populations are stored shifted by the equilibrium of a uniform
// reference state (0, Fref), g = f - feq(0, Fref) (the initial deformation
// gradient at the first active node; I for a body at rest).  The stored
// values and their sums (v, F - Fref) then have the magnitude of the
// dynamics, not of the static deformation and its stress: a deformed
// lattice with a weak wave on it keeps the wave's digits in FP32.  The
// recovered F and its stress are formed in FP64 registers and the stress
// enters the equilibrium as the difference P(F)/rho0 - P(Fref)/rho0, so the
// FP32 arithmetic of the collision also acts on dynamic-scale values.
#include "tl_device.hpp"
#include "tl_internal.hpp"
#include "tl_math.hpp"

// Tuning knobs (compile-time): non-temporal population loads / stores, and a
// minimum number of waves per SIMD for the fused kernel (caps VGPRs).
#ifndef TL_NT_LOAD
#define TL_NT_LOAD 1
#endif
#ifndef TL_NT_STORE
#define TL_NT_STORE 1
#endif
// The periodic update fits 168 VGPRs without spills at 3 waves per SIMD;
// the embedded (chunked) updates run fastest at their natural allocation.
#ifndef TL_BULK_WAVES
#define TL_BULK_WAVES 3
#endif
// embedded bodies: minimum waves per SIMD of the chunked and batched updates
#ifndef TL_CHUNK_WAVES
#define TL_CHUNK_WAVES 1
#endif

namespace tl {

template <typename T> __device__ __forceinline__ T ld_pop(const T *p) {
#if TL_NT_LOAD
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

template <typename T> __device__ __forceinline__ void st_pop(T *p, T v) {
#if TL_NT_STORE
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

__device__ __forceinline__ int wrap_m(int v, int n) { return v < 0 ? v + n : v; }
__device__ __forceinline__ int wrap_p(int v, int n) { return v >= n ? v - n : v; }

// node index of X - e_q (periodic wrap; for active nodes of an embedded body
// the neighbour always exists, see set_levelset)
template <int q>
__device__ __forceinline__ int64_t pull_src(const Geo &g, int x, int y, int z) {
  int xs = x, ys = y, zs = z;
  if constexpr (q == 0) xs = wrap_m(x - 1, g.nx);
  if constexpr (q == 1) xs = wrap_p(x + 1, g.nx);
  if constexpr (q == 2) ys = wrap_m(y - 1, g.ny);
  if constexpr (q == 3) ys = wrap_p(y + 1, g.ny);
  if constexpr (q == 4) zs = wrap_m(z - 1, g.nz);
  if constexpr (q == 5) zs = wrap_p(z + 1, g.nz);
  return xs + (int64_t)g.nx * (ys + (int64_t)g.ny * zs);
}

template <int D, typename T, int q, int M>
__device__ __forceinline__ void load_dir(const T *__restrict__ fin, const Geo &g, int x, int y, int z,
                                         T (&f)[2 * D][M]) {
  const int64_t s = pull_src<q>(g, x, y, z);
#pragma unroll
  for (int r = 0; r < M; ++r) f[q][r] = ld_pop(fin + (size_t)(q * M + r) * g.S + s);
}

template <int D, typename T, int M>
__device__ __forceinline__ void pull_all(const T *__restrict__ fin, const Geo &g, int x, int y, int z,
                                         T (&f)[2 * D][M]) {
  load_dir<D, T, 0>(fin, g, x, y, z, f);
  load_dir<D, T, 1>(fin, g, x, y, z, f);
  load_dir<D, T, 2>(fin, g, x, y, z, f);
  load_dir<D, T, 3>(fin, g, x, y, z, f);
  if constexpr (D == 3) {
    load_dir<D, T, 4>(fin, g, x, y, z, f);
    load_dir<D, T, 5>(fin, g, x, y, z, f);
  }
}

template <typename T> __device__ __forceinline__ bool finite_(T v) { return __builtin_isfinite(v); }

// Fused pull-stream + state recovery + (optional projection repair) + BGK
// collision with source + displacement quadrature (Algorithm 1, bulk loops).
// TAPE: also store the recovered (pre-repair) F - I to the tape planes of
// the reverse mode, plane k at tape[k * ts + tslot].
template <int D, typename T, bool MASK, bool TRACK, bool REPAIR, bool TAPE = false, class L = NeoHookean<D>>
__device__ __forceinline__ void bulk_node(const T *__restrict__ fin, T *__restrict__ fout, const Geo &g,
                                          const Par &p, const uint8_t *__restrict__ act, double *__restrict__ ustar,
                                          double *__restrict__ ubuf, const T *__restrict__ Frp,
                                          int *__restrict__ flag, int x, int row, T *__restrict__ tape = nullptr,
                                          const T *__restrict__ bf = nullptr, T bs = T(0), int64_t tslot = 0,
                                          int64_t ts = 0) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = x + (int64_t)g.nx * row;
  if constexpr (MASK) {
    if (!act[node]) return;
  }
  T f[Q][M];
  pull_all<D, T, M>(fin, g, x, y, z, f);

  // state recovery with the half-step source (Eq. 28): B = (b - gamma v, 0)
  // with the damping implicit, v = (sum_q f^v + dt/2 b) / (1 + gamma dt / 2)
  T dU[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    T s = f[0][r];
#pragma unroll
    for (int q = 1; q < Q; ++q) s += f[q][r];
    dU[r] = s;
  }
  const T dt = T(p.dt);
  const T inv_damp = T(1) / (T(1) + T(0.5) * T(p.gamma) * dt);
  T bacc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) bacc[i] = (L::body && bf) ? bs * bf[(size_t)i * g.S + node] : T(0);
  // the sums are v and F - Fref (populations stored about the reference
  // state); F and its stress P(F) in FP64, which enters the equilibrium as
  // the difference P(F)/rho0 - Pref
  T v[D];
#pragma unroll
  for (int i = 0; i < D; ++i) v[i] = (L::body ? dU[i] + T(0.5) * dt * bacc[i] : dU[i]) * inv_damp;
  double F[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) F[k] = p.Fref[k] + double(dU[D + k]);
  if constexpr (TAPE) {
    if (tape) {
#pragma unroll
      for (int k = 0; k < D * D; ++k) tape[(size_t)k * ts + tslot] = T(F[k] - ((k % (D + 1) == 0) ? 1.0 : 0.0));
    }
  }
  const T inv2c = T(0.5) / T(p.c);
  const T om = T(p.omega);
  const T srcw = dt * (T(2) - om) / T(4 * D);
  double Fr[D * D];
  if constexpr (REPAIR) {
    // population repair f += feq(v, F^r) - feq(v, F) (Sec. 3.5, Eq. 61),
    // deformation rows here, velocity rows with the stress below; the
    // repaired planes hold F^r - I
#pragma unroll
    for (int k = 0; k < D * D; ++k) Fr[k] = double(Frp[(size_t)k * g.S + node]) + ((k % (D + 1) == 0) ? 1.0 : 0.0);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k = 0; k < D * D; ++k) f[q][D + k] += T((Fr[k] - F[k]) / (2 * D));
#pragma unroll
    for (int k = 0; k < D * D; ++k) dU[D + k] = T(Fr[k] - p.Fref[k]);
  }

  // BGK collision with source weights 1/(4D) (Eqs. 29-30) in the stored
  // variables: feq_q(U) - feq_q(0, Fref) = (v, F - Fref)/(2D)
  // + e_qA (Phi_A(U) - Phi_A(0, Fref)) / (2c).
  // The isotropic part (v, F - Fref)/(2D) once per row, rounded from FP64:
  // 1/(2D) has no exact FP32 value in 3D, and a rounded factor would bias
  // the zeroth moment of every collision by the same relative amount.
  // The deformation rows need v and F but not the stress: they are stored
  // first, which frees their registers before the stress is formed.
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    const int r = D + k, i = k / D, B = k % D;
    const T iso = T(double(dU[r]) * (1.0 / (2 * D)));
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int A = q / 2;
      const T sg = (q & 1) ? T(-1) : T(1);
      const T phi = (A == B) ? -v[i] : T(0);
      const T feq = iso + sg * inv2c * phi;
      const T out = f[q][r] + om * (feq - f[q][r]);
      st_pop(fout + (size_t)(q * M + r) * g.S + node, out);
    }
  }

  // the first Piola stress in FP64 (law L), which enters the equilibrium as
  // the difference P(F)/rho0 - Pref, and the velocity rows
  typename L::Node law;  // the law's internal variables at the node
  L::load(p, node, g.S, law);
  double P[D * D];
  double J = L::stress(p, F, law, P);
  bool bad = !(J > 0.0);
  if constexpr (REPAIR) {
    double P1[D * D];
    const double J1 = L::stress(p, Fr, law, P1);
    bad |= !(J1 > 0.0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int A = q / 2;
      const double sg = (q & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int i = 0; i < D; ++i) f[q][i] += T(sg * (0.5 / p.c) * (-(P1[i * D + A] - P[i * D + A]) * p.inv_rho0));
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) P[k] = P1[k];
    J = J1;
  }
  T dP[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) dP[k] = T(P[k] * p.inv_rho0 - p.Pref[k]);
  // internal variables advance with the deformation the collision uses
  L::commit(p, law, node, g.S);
#pragma unroll
  for (int r = 0; r < D; ++r) {
    const T iso = T(double(v[r]) * (1.0 / (2 * D)));
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int A = q / 2;
      const T sg = (q & 1) ? T(-1) : T(1);
      const T feq = iso + sg * inv2c * (-dP[r * D + A]);
      T out = f[q][r] + om * (feq - f[q][r]);
      out += srcw * (L::body ? bacc[r] - T(p.gamma) * v[r] : -T(p.gamma) * v[r]);
      st_pop(fout + (size_t)(q * M + r) * g.S + node, out);
    }
  }

  if constexpr (TRACK) {
    // trapezoidal displacement quadrature (Eq. 34), FP64 in both builds
    const double hdt = 0.5 * p.dt;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double uu;
      if constexpr (REPAIR) {
        uu = ubuf[(size_t)i * g.S + node];
      } else {
        uu = ustar[(size_t)i * g.S + node] + hdt * double(v[i]);
        ubuf[(size_t)i * g.S + node] = uu;
      }
      ustar[(size_t)i * g.S + node] = uu + hdt * double(v[i]);
    }
  }
  double chk = J;
#pragma unroll
  for (int i = 0; i < D; ++i) chk += double(v[i]);
  if (bad || !finite_(chk)) atomicOr(flag, finite_(chk) ? FLAG_J : FLAG_NONFINITE);
}

// The single-instance kernel keeps the update inline: routed through the
// device function above, the compiler schedules its address arithmetic
// differently and the kernel runs 2.6% slower at 256^3 (measured).  The two
// bodies are kept identical (a CPU test compares them).
template <int D, typename T, bool MASK, bool TRACK, bool REPAIR, class L = NeoHookean<D>>
__global__ __launch_bounds__(256, TL_BULK_WAVES) void k_bulk(const T *__restrict__ fin, T *__restrict__ fout, Geo g, Par p,
                                               const uint8_t *__restrict__ act, double *__restrict__ ustar,
                                               double *__restrict__ ubuf, const T *__restrict__ Frp,
                                               int *__restrict__ flag, const T *__restrict__ bf, T bs) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int row = blockIdx.y;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = x + (int64_t)g.nx * row;
  if constexpr (MASK) {
    if (!act[node]) return;
  }
  T f[Q][M];
  pull_all<D, T, M>(fin, g, x, y, z, f);

  // state recovery with the half-step source (Eq. 28): B = (b - gamma v, 0)
  // with the damping implicit, v = (sum_q f^v + dt/2 b) / (1 + gamma dt / 2)
  T dU[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    T s = f[0][r];
#pragma unroll
    for (int q = 1; q < Q; ++q) s += f[q][r];
    dU[r] = s;
  }
  const T dt = T(p.dt);
  const T inv_damp = T(1) / (T(1) + T(0.5) * T(p.gamma) * dt);
  T bacc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) bacc[i] = (L::body && bf) ? bs * bf[(size_t)i * g.S + node] : T(0);
  // the sums are v and F - Fref (populations stored about the reference
  // state); F and its stress P(F) in FP64, which enters the equilibrium as
  // the difference P(F)/rho0 - Pref
  T v[D];
#pragma unroll
  for (int i = 0; i < D; ++i) v[i] = (L::body ? dU[i] + T(0.5) * dt * bacc[i] : dU[i]) * inv_damp;
  double F[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) F[k] = p.Fref[k] + double(dU[D + k]);
  const T inv2c = T(0.5) / T(p.c);
  const T om = T(p.omega);
  const T srcw = dt * (T(2) - om) / T(4 * D);
  double Fr[D * D];
  if constexpr (REPAIR) {
    // population repair f += feq(v, F^r) - feq(v, F) (Sec. 3.5, Eq. 61),
    // deformation rows here, velocity rows with the stress below; the
    // repaired planes hold F^r - I
#pragma unroll
    for (int k = 0; k < D * D; ++k) Fr[k] = double(Frp[(size_t)k * g.S + node]) + ((k % (D + 1) == 0) ? 1.0 : 0.0);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k = 0; k < D * D; ++k) f[q][D + k] += T((Fr[k] - F[k]) / (2 * D));
#pragma unroll
    for (int k = 0; k < D * D; ++k) dU[D + k] = T(Fr[k] - p.Fref[k]);
  }

  // BGK collision with source weights 1/(4D) (Eqs. 29-30) in the stored
  // variables: feq_q(U) - feq_q(0, Fref) = (v, F - Fref)/(2D)
  // + e_qA (Phi_A(U) - Phi_A(0, Fref)) / (2c).
  // The isotropic part (v, F - Fref)/(2D) once per row, rounded from FP64:
  // 1/(2D) has no exact FP32 value in 3D, and a rounded factor would bias
  // the zeroth moment of every collision by the same relative amount.
  // The deformation rows need v and F but not the stress: they are stored
  // first, which frees their registers before the stress is formed.
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    const int r = D + k, i = k / D, B = k % D;
    const T iso = T(double(dU[r]) * (1.0 / (2 * D)));
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int A = q / 2;
      const T sg = (q & 1) ? T(-1) : T(1);
      const T phi = (A == B) ? -v[i] : T(0);
      const T feq = iso + sg * inv2c * phi;
      const T out = f[q][r] + om * (feq - f[q][r]);
      st_pop(fout + (size_t)(q * M + r) * g.S + node, out);
    }
  }

  // the first Piola stress in FP64 (law L), which enters the equilibrium as
  // the difference P(F)/rho0 - Pref, and the velocity rows
  typename L::Node law;  // the law's internal variables at the node
  L::load(p, node, g.S, law);
  double P[D * D];
  double J = L::stress(p, F, law, P);
  bool bad = !(J > 0.0);
  if constexpr (REPAIR) {
    double P1[D * D];
    const double J1 = L::stress(p, Fr, law, P1);
    bad |= !(J1 > 0.0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int A = q / 2;
      const double sg = (q & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int i = 0; i < D; ++i) f[q][i] += T(sg * (0.5 / p.c) * (-(P1[i * D + A] - P[i * D + A]) * p.inv_rho0));
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) P[k] = P1[k];
    J = J1;
  }
  T dP[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) dP[k] = T(P[k] * p.inv_rho0 - p.Pref[k]);
  // internal variables advance with the deformation the collision uses
  L::commit(p, law, node, g.S);
#pragma unroll
  for (int r = 0; r < D; ++r) {
    const T iso = T(double(v[r]) * (1.0 / (2 * D)));
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int A = q / 2;
      const T sg = (q & 1) ? T(-1) : T(1);
      const T feq = iso + sg * inv2c * (-dP[r * D + A]);
      T out = f[q][r] + om * (feq - f[q][r]);
      out += srcw * (L::body ? bacc[r] - T(p.gamma) * v[r] : -T(p.gamma) * v[r]);
      st_pop(fout + (size_t)(q * M + r) * g.S + node, out);
    }
  }

  if constexpr (TRACK) {
    // trapezoidal displacement quadrature (Eq. 34), FP64 in both builds
    const double hdt = 0.5 * p.dt;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double uu;
      if constexpr (REPAIR) {
        uu = ubuf[(size_t)i * g.S + node];
      } else {
        uu = ustar[(size_t)i * g.S + node] + hdt * double(v[i]);
        ubuf[(size_t)i * g.S + node] = uu;
      }
      ustar[(size_t)i * g.S + node] = uu + hdt * double(v[i]);
    }
  }
  double chk = J;
#pragma unroll
  for (int i = 0; i < D; ++i) chk += double(v[i]);
  if (bad || !finite_(chk)) atomicOr(flag, finite_(chk) ? FLAG_J : FLAG_NONFINITE);
}

// the same update recording the recovered state on the reverse-mode tape
template <int D, typename T, bool MASK, bool TRACK, bool REPAIR, class L = NeoHookean<D>>
__global__ __launch_bounds__(256) void k_bulk_tape(const T *__restrict__ fin, T *__restrict__ fout, Geo g, Par p,
                                                   const uint8_t *__restrict__ act, double *__restrict__ ustar,
                                                   double *__restrict__ ubuf, const T *__restrict__ Frp,
                                                   int *__restrict__ flag, T *__restrict__ tape,
                                                   const T *__restrict__ bf, T bs) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  bulk_node<D, T, MASK, TRACK, REPAIR, true, L>(fin, fout, g, p, act, ustar, ubuf, Frp, flag, x,
                                                   (int)blockIdx.y, tape, bf, bs,
                                                   x + (int64_t)g.nx * blockIdx.y, g.S);
}

// Embedded bodies: the same update over the list of CHUNK-node chunks (of
// the node order) that hold active nodes, 64 / CHUNK chunks per wavefront;
// inactive nodes of a chunk return at once (MASK).
template <int D, typename T, bool TRACK, bool REPAIR, class L>
__global__ __launch_bounds__(256, TL_CHUNK_WAVES) void k_bulk_chunks(const T *__restrict__ fin, T *__restrict__ fout,
                                                                    Geo g, Par p, const uint8_t *__restrict__ act,
                                                                    double *__restrict__ ustar,
                                                                    double *__restrict__ ubuf,
                                                                    const T *__restrict__ Frp, int *__restrict__ flag,
                                                                    const T *__restrict__ bf, T bs,
                                                                    const int32_t *__restrict__ chunks, int nchunks) {
  const int ch = blockIdx.x * (256 / CHUNK) + (int)(threadIdx.x / CHUNK);
  if (ch >= nchunks) return;
  const int64_t i = (int64_t)chunks[ch] * CHUNK + (threadIdx.x % CHUNK);
  if (i >= g.N) return;
  const int x = (int)(i % g.nx), row = (int)(i / g.nx);
  bulk_node<D, T, true, TRACK, REPAIR, false, L>(fin, fout, g, p, act, ustar, ubuf, Frp, flag, x, row, nullptr,
                                                    bf, bs);
}

// the chunked update recording the recovered state on the reverse-mode tape
template <int D, typename T, bool TRACK, bool REPAIR, class L>
__global__ __launch_bounds__(256, TL_CHUNK_WAVES) void k_bulk_chunks_tape(
    const T *__restrict__ fin, T *__restrict__ fout, Geo g, Par p, const uint8_t *__restrict__ act,
    double *__restrict__ ustar, double *__restrict__ ubuf, const T *__restrict__ Frp, int *__restrict__ flag,
    T *__restrict__ tape, const int32_t *__restrict__ chunks, int nchunks) {
  const int ch = blockIdx.x * (256 / CHUNK) + (int)(threadIdx.x / CHUNK);
  if (ch >= nchunks) return;
  const int64_t i = (int64_t)chunks[ch] * CHUNK + (threadIdx.x % CHUNK);
  if (i >= g.N) return;
  const int x = (int)(i % g.nx), row = (int)(i / g.nx);
  // tape slot of chunk ch, position i % CHUNK
  bulk_node<D, T, true, TRACK, REPAIR, true, L>(fin, fout, g, p, act, ustar, ubuf, Frp, flag, x, row, tape,
                                                  nullptr, T(0), (int64_t)ch * CHUNK + (threadIdx.x % CHUNK),
                                                  (int64_t)nchunks * CHUNK);
}

// Batched bulk update: one block per tile (instance, row, first x) of the
// tile list; every instance keeps its own geometry, material and buffers.
// the body-acceleration ramp of instance I at the batch's current step
// (read on the device, so that replays of captured steps advance it)
template <typename T> __device__ __forceinline__ T batch_body_scale(const Inst &I, const int64_t *step) {
  if (!I.bf) return T(0);
  double sv, dsv;
  ramp_eval(I.bf_ramp, I.bf_Tr, *step * I.p.dt, sv, dsv);
  return T(sv);
}

template <int D, typename T, bool REPAIR, class L = NeoHookean<D>>
__global__ __launch_bounds__(256, TL_CHUNK_WAVES) void k_bulk_batch(const Inst *__restrict__ insts,
                                                                   const int4 *__restrict__ tiles,
                                                                   const int64_t *__restrict__ step) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const int64_t node = (int64_t)t.y * blockDim.x + threadIdx.x;
  if (node >= I.g.N) return;
  const int row = (int)(node / I.g.nx), x = (int)(node - (int64_t)row * I.g.nx);
  bulk_node<D, T, true, true, REPAIR, false, L>((const T *)I.fin, (T *)I.fout, I.g, I.p, I.act,
                                                (double *)I.ustar, (double *)I.ubuf, (const T *)I.Fr, I.flag, x, row,
                                                nullptr, (const T *)I.bf, batch_body_scale<T>(I, step));
}

// Pull f^n and write moments: v (damping-corrected), F, u = u* + dt/2 v, J.
// Output planes have stride ostride; any output may be null.
template <int D, typename T, typename O, bool MASK, bool DEV = false>
__device__ __forceinline__ void moments_node(const T *__restrict__ fin, const Geo &g, const Par &p,
                                             const uint8_t *__restrict__ act, const double *__restrict__ ustar,
                                             O *__restrict__ Vo, O *__restrict__ Fo, double *__restrict__ uo,
                                             O *__restrict__ Jo, int64_t ostride, int x, int row,
                                             const T *__restrict__ bf = nullptr, T bs = T(0)) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = x + (int64_t)g.nx * row;
  if (MASK && !act[node]) {
    for (int i = 0; i < D; ++i) {
      if (Vo) Vo[(size_t)i * ostride + node] = O(0);
      if (uo) uo[(size_t)i * ostride + node] = 0.0;
    }
    if (Fo)
      for (int k = 0; k < D * D; ++k) Fo[(size_t)k * ostride + node] = O(0);
    if (Jo) Jo[node] = O(0);
    return;
  }
  T f[Q][M];
  pull_all<D, T, M>(fin, g, x, y, z, f);
  T dU[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    T s = f[0][r];
#pragma unroll
    for (int q = 1; q < Q; ++q) s += f[q][r];
    dU[r] = s;
  }
  const T inv_damp = T(1) / (T(1) + T(0.5) * T(p.gamma) * T(p.dt));
  T v[D];
  double F[D * D];
#pragma unroll
  for (int i = 0; i < D; ++i)
    v[i] = (bf ? dU[i] + T(0.5) * T(p.dt) * (bs * bf[(size_t)i * g.S + node]) : dU[i]) * inv_damp;
#pragma unroll
  for (int k = 0; k < D * D; ++k) F[k] = p.Fref[k] + double(dU[D + k]);  // stored about (0, Fref)
  if (Vo)
    for (int i = 0; i < D; ++i) Vo[(size_t)i * ostride + node] = O(v[i]);
  if (Fo)  // DEV: F - I (the projection's planes), else F
    for (int k = 0; k < D * D; ++k)
      Fo[(size_t)k * ostride + node] = O(DEV ? F[k] - ((k % (D + 1) == 0) ? 1.0 : 0.0) : F[k]);
  if (uo)
    for (int i = 0; i < D; ++i)
      uo[(size_t)i * ostride + node] = ustar ? ustar[(size_t)i * g.S + node] + 0.5 * p.dt * double(v[i]) : 0.0;
  if (Jo) Jo[node] = O(det<D>(F));
}

template <int D, typename T, typename O, bool MASK, bool DEV = false>
__global__ __launch_bounds__(256) void k_moments(const T *__restrict__ fin, Geo g, Par p,
                                                  const uint8_t *__restrict__ act, const double *__restrict__ ustar,
                                                  O *__restrict__ Vo, O *__restrict__ Fo, double *__restrict__ uo,
                                                  O *__restrict__ Jo, int64_t ostride, const T *__restrict__ bf,
                                                  T bs) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  moments_node<D, T, O, MASK, DEV>(fin, g, p, act, ustar, Vo, Fo, uo, Jo, ostride, x, (int)blockIdx.y, bf, bs);
}

// Stress of the current time level: P of the recovered F with the node's
// law and sigma = J^{-1} P F^T (Sec. 2.4, Eq. 35), planar [D*D][N] FP64;
// zero at inactive nodes
template <int D, typename T, bool MASK>
__global__ __launch_bounds__(256) void k_stress(const T *__restrict__ fin, Geo g, Par p,
                                                 const uint8_t *__restrict__ act, double *__restrict__ Po,
                                                 double *__restrict__ So) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int row = blockIdx.y;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = x + (int64_t)g.nx * row;
  double P[D * D], sg[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) P[k] = sg[k] = 0.0;
  if (!MASK || act[node]) {
    T f[Q][M];
    pull_all<D, T, M>(fin, g, x, y, z, f);
    double F[D * D];
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
      T s = f[0][D + k];
#pragma unroll
      for (int q = 1; q < Q; ++q) s += f[q][D + k];
      F[k] = p.Fref[k] + double(s);
    }
    double Hn[sym_n<D>()];
    const double J = law_piola<D>(F, p, law_load<D>(p, node, g.S, Hn) ? Hn : nullptr, P, law_theta<D>(p, node));
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        double s = 0.0;
#pragma unroll
        for (int A = 0; A < D; ++A) s += P[a * D + A] * F[b * D + A];
        sg[a * D + b] = s / J;
      }
  }
  if (Po)
    for (int k = 0; k < D * D; ++k) Po[(size_t)k * g.N + node] = P[k];
  if (So)
    for (int k = 0; k < D * D; ++k) So[(size_t)k * g.N + node] = sg[k];
}

// batched projection inputs: v, F into each instance's workspace, u = u* + dt/2 v
template <int D, typename T>
__global__ __launch_bounds__(256) void k_moments_batch(const Inst *__restrict__ insts,
                                                        const int4 *__restrict__ tiles,
                                                        const int64_t *__restrict__ step) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const int64_t node = (int64_t)t.y * blockDim.x + threadIdx.x;
  if (node >= I.g.N) return;
  const int row = (int)(node / I.g.nx), x = (int)(node - (int64_t)row * I.g.nx);
  moments_node<D, T, T, true, true>((const T *)I.fin, I.g, I.p, I.act, (const double *)I.ustar, (T *)I.V, (T *)I.Fm,
                                    (double *)I.ubuf, (T *)nullptr, I.g.S, x, row, (const T *)I.bf,
                                    batch_body_scale<T>(I, step));
}

// Second-order initialisation (Sec. 2.4, Eqs. 32-33) in FP64, stored
// reverse-streamed: the value for direction q of node X goes to the pull slot
// X - e_q, so that the first bulk pull reads f^0_q(X).
template <int D, typename T, bool MASK>
__global__ __launch_bounds__(256) void k_init(T *__restrict__ fout, Geo g, Par p, const uint8_t *__restrict__ act,
                                               const double *__restrict__ U0, const double *__restrict__ u0,
                                               const double *__restrict__ dU0, double *__restrict__ ustar,
                                               int *__restrict__ flag, const T *__restrict__ bf, double bs) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int row = blockIdx.y;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = x + (int64_t)g.nx * row;
  if (MASK && !act[node]) return;
  double U[M], dA[D][M], Ut[M];
#pragma unroll
  for (int r = 0; r < M; ++r) U[r] = U0[(size_t)r * g.N + node];
#pragma unroll
  for (int A = 0; A < D; ++A)
#pragma unroll
    for (int r = 0; r < M; ++r) dA[A][r] = dU0 ? dU0[((size_t)A * M + r) * g.N + node] : 0.0;
  const double *F = U + D;
  double P[D * D];
  if (!(det<D>(F) > 0.0)) {
    atomicOr(flag, FLAG_J);
    return;
  }
  // a Maxwell branch starts relaxed at F0: Q^0 = 0, S_0^0 = S_0(F0), i.e.
  // R = -beta xi S_0(F0)
  double Hn[sym_n<D>()];
  const double *hn = nullptr;
  if (p.hist) {
    shear_S0<D>(F, p.mu, Hn, nullptr);
#pragma unroll
    for (int k = 0; k < sym_n<D>(); ++k) {
      Hn[k] = -p.vbx * Hn[k];
      p.hist[(size_t)k * g.S + node] = Hn[k];
    }
    hn = Hn;
  }
  // the node's thermal stretch, taken as locally uniform in the
  // second-order terms (its gradient does not enter them)
  const double th = law_theta<D>(p, node);
  law_piola<D>(F, p, hn, P, th);
  // d_t U0 = B0 - Phi'_A(U0) d_A U0, B0 = (b0 - gamma v0, 0)
#pragma unroll
  for (int r = 0; r < M; ++r)
    Ut[r] = (r < D) ? (bf ? bs * double(bf[(size_t)r * g.S + node]) : 0.0) - p.gamma * U[r] : 0.0;
#pragma unroll
  for (int A = 0; A < D; ++A) {
    double dP[D * D];
    law_tangent<D>(F, dA[A] + D, p, hn, dP, th);
#pragma unroll
    for (int i = 0; i < D; ++i) Ut[i] += dP[i * D + A] * p.inv_rho0;  // -(-dP)
#pragma unroll
    for (int i = 0; i < D; ++i) Ut[D + i * D + A] += dA[A][i];        // -(-dv_i)
  }
  const double c = p.c, inv2D = 1.0 / (2 * D);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int A = q / 2;
    const double sg = (q & 1) ? -1.0 : 1.0;
    double Z[M], dP[D * D];
#pragma unroll
    for (int r = 0; r < M; ++r) Z[r] = Ut[r] + c * sg * dA[A][r];
    law_tangent<D>(F, Z + D, p, hn, dP, th);
    int xs = x, ys = y, zs = z;  // X - e_q
    if (A == 0) xs = (x - (int)sg + g.nx) % g.nx;
    if (A == 1) ys = (y - (int)sg + g.ny) % g.ny;
    if (A == 2) zs = (z - (int)sg + g.nz) % g.nz;
    const int64_t dst = xs + (int64_t)g.nx * (ys + (int64_t)g.ny * zs);
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double phi, dphi;
      if (r < D) {
        phi = -P[r * D + A] * p.inv_rho0;
        dphi = -dP[r * D + A] * p.inv_rho0;
      } else {
        const int i = (r - D) / D, B = (r - D) % D;
        phi = (A == B) ? -U[i] : 0.0;
        dphi = (A == B) ? -Z[i] : 0.0;
      }
      const double feq = U[r] * inv2D + sg * phi / (2.0 * c);
      const double dfeq = Z[r] * inv2D + sg * dphi / (2.0 * c);
      // stored about the reference state (0, Fref)
      const double fv = feq - 0.5 * p.dt * dfeq - pop_shift<D>(p, q, r);
      fout[(size_t)(q * M + r) * g.S + dst] = T(fv);
    }
  }
  if (ustar)
#pragma unroll
    for (int i = 0; i < D; ++i)
      ustar[(size_t)i * g.S + node] = (u0 ? u0[(size_t)i * g.N + node] : 0.0) - 0.5 * p.dt * U[i];
}

// raw pre-collision populations f^n (unshifted) [Q][M][N] and u*^n [D][N]
template <int D, typename T, bool MASK>
__global__ __launch_bounds__(256) void k_get_f(const T *__restrict__ fin, Geo g, Par p,
                                                const uint8_t *__restrict__ act, const double *__restrict__ ustar,
                                                double *__restrict__ fo, double *__restrict__ uso) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int row = blockIdx.y;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = x + (int64_t)g.nx * row;
  const bool on = !MASK || act[node];
  if (fo) {
    T f[Q][M];
    if (on) pull_all<D, T, M>(fin, g, x, y, z, f);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        fo[((size_t)q * M + r) * g.N + node] = on ? double(f[q][r]) + pop_shift<D>(p, q, r) : 0.0;
      }
  }
  if (uso)
    for (int i = 0; i < D; ++i) uso[(size_t)i * g.N + node] = (on && ustar) ? ustar[(size_t)i * g.S + node] : 0.0;
}

template <int D, typename T, bool MASK>
__global__ __launch_bounds__(256) void k_put_f(T *__restrict__ fout, Geo g, Par p, const uint8_t *__restrict__ act,
                                                const double *__restrict__ fi, const double *__restrict__ usi,
                                                double *__restrict__ ustar) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int row = blockIdx.y;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = x + (int64_t)g.nx * row;
  if (MASK && !act[node]) return;
  if (fi) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int A = q / 2, sg = (q & 1) ? -1 : 1;
      int xs = x, ys = y, zs = z;
      if (A == 0) xs = (x - sg + g.nx) % g.nx;
      if (A == 1) ys = (y - sg + g.ny) % g.ny;
      if (A == 2) zs = (z - sg + g.nz) % g.nz;
      const int64_t dst = xs + (int64_t)g.nx * (ys + (int64_t)g.ny * zs);
#pragma unroll
      for (int r = 0; r < M; ++r) {
        fout[(size_t)(q * M + r) * g.S + dst] = T(fi[((size_t)q * M + r) * g.N + node] - pop_shift<D>(p, q, r));
      }
    }
  }
  if (ustar)
    for (int i = 0; i < D; ++i) ustar[(size_t)i * g.S + node] = usi ? usi[(size_t)i * g.N + node] : 0.0;
}

// ------------------------------------------------------------------ launchers

static inline void grid_of(const Geo &g, dim3 &grid, dim3 &block) {
  int bx = g.nx >= 256 ? 256 : ((g.nx + 63) / 64) * 64;
  block = dim3(bx, 1, 1);
  grid = dim3((g.nx + bx - 1) / bx, g.ny * g.nz, 1);
}

// body acceleration scale s(t^n) of the current step (0 without a field)
template <typename T> static T body_scale(const tlvlbm_ctx *c) {
  if (!c->bf) return T(0);
  double sv, dsv;
  ramp_eval(c->bf_ramp, c->bf_Tr, c->step * c->par.dt, sv, dsv);
  return T(sv);
}

template <int D, typename T, class L> static void bulk_plain_t(tlvlbm_ctx *c, bool repair) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  const T *fin = (const T *)c->fB;
  T *fout = (T *)c->fA;
  double *us = (double *)c->ustar, *ub = (double *)c->ubuf;
  const T *Fr = (const T *)c->cg.Fr;
  const T *bf = (const T *)c->bf;
  const T bs = body_scale<T>(c);
  if (c->act && c->chunks) {
    // embedded body: only the chunks holding active nodes
    const unsigned nb = (unsigned)((c->nchunks + 256 / CHUNK - 1) / (256 / CHUNK));
    if (repair)
      hipLaunchKernelGGL((k_bulk_chunks<D, T, true, true, L>), nb, 256, 0, c->st, fin, fout, c->geo, c->par,
                         c->act, us, ub, Fr, c->d_flag, bf, bs, c->chunks, c->nchunks);
    else if (c->track_u)
      hipLaunchKernelGGL((k_bulk_chunks<D, T, true, false, L>), nb, 256, 0, c->st, fin, fout, c->geo, c->par,
                         c->act, us, ub, Fr, c->d_flag, bf, bs, c->chunks, c->nchunks);
    else
      hipLaunchKernelGGL((k_bulk_chunks<D, T, false, false, L>), nb, 256, 0, c->st, fin, fout, c->geo, c->par,
                         c->act, us, ub, Fr, c->d_flag, bf, bs, c->chunks, c->nchunks);
    return;
  }
  if (repair) {
    hipLaunchKernelGGL((k_bulk<D, T, true, true, true, L>), grid, block, 0, c->st, fin, fout, c->geo, c->par,
                       c->act, us, ub, Fr, c->d_flag, bf, bs);
  } else if (c->act) {
    if (c->track_u)
      hipLaunchKernelGGL((k_bulk<D, T, true, true, false, L>), grid, block, 0, c->st, fin, fout, c->geo, c->par,
                         c->act, us, ub, Fr, c->d_flag, bf, bs);
    else
      hipLaunchKernelGGL((k_bulk<D, T, true, false, false, L>), grid, block, 0, c->st, fin, fout, c->geo, c->par,
                         c->act, us, ub, Fr, c->d_flag, bf, bs);
  } else {
    if (c->track_u)
      hipLaunchKernelGGL((k_bulk<D, T, false, true, false, L>), grid, block, 0, c->st, fin, fout, c->geo, c->par,
                         c->act, us, ub, Fr, c->d_flag, bf, bs);
    else
      hipLaunchKernelGGL((k_bulk<D, T, false, false, false, L>), grid, block, 0, c->st, fin, fout, c->geo,
                         c->par, c->act, us, ub, Fr, c->d_flag, bf, bs);
  }
}

// the forward of the reverse mode (no body acceleration: refused there; the
// fibre law in the Reinforced instantiation; no history-dependent law)
template <int D, typename T, class L> static void bulk_tape_t(tlvlbm_ctx *c, bool repair, void *tape) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  const T *fin = (const T *)c->fB;
  T *fout = (T *)c->fA;
  double *us = (double *)c->ustar, *ub = (double *)c->ubuf;
  const T *Fr = (const T *)c->cg.Fr;
  T *tp = (T *)tape;
  const T *nb = nullptr;
  if (c->act && c->chunks) {
    const unsigned nblk = (unsigned)((c->nchunks + 256 / CHUNK - 1) / (256 / CHUNK));
    if (repair)
      hipLaunchKernelGGL((k_bulk_chunks_tape<D, T, true, true, L>), nblk, 256, 0, c->st, fin, fout, c->geo,
                         c->par, c->act, us, ub, Fr, c->d_flag, tp, c->chunks, c->nchunks);
    else if (c->track_u)
      hipLaunchKernelGGL((k_bulk_chunks_tape<D, T, true, false, L>), nblk, 256, 0, c->st, fin, fout, c->geo,
                         c->par, c->act, us, ub, Fr, c->d_flag, tp, c->chunks, c->nchunks);
    else
      hipLaunchKernelGGL((k_bulk_chunks_tape<D, T, false, false, L>), nblk, 256, 0, c->st, fin, fout, c->geo,
                         c->par, c->act, us, ub, Fr, c->d_flag, tp, c->chunks, c->nchunks);
    return;
  }
  if (repair)
    hipLaunchKernelGGL((k_bulk_tape<D, T, true, true, true, L>), grid, block, 0, c->st, fin, fout, c->geo, c->par,
                       c->act, us, ub, Fr, c->d_flag, tp, nb, T(0));
  else if (c->act && c->track_u)
    hipLaunchKernelGGL((k_bulk_tape<D, T, true, true, false, L>), grid, block, 0, c->st, fin, fout, c->geo, c->par,
                       c->act, us, ub, Fr, c->d_flag, tp, nb, T(0));
  else if (c->act)
    hipLaunchKernelGGL((k_bulk_tape<D, T, true, false, false, L>), grid, block, 0, c->st, fin, fout, c->geo,
                       c->par, c->act, us, ub, Fr, c->d_flag, tp, nb, T(0));
  else if (c->track_u)
    hipLaunchKernelGGL((k_bulk_tape<D, T, false, true, false, L>), grid, block, 0, c->st, fin, fout, c->geo,
                       c->par, c->act, us, ub, Fr, c->d_flag, tp, nb, T(0));
  else
    hipLaunchKernelGGL((k_bulk_tape<D, T, false, false, false, L>), grid, block, 0, c->st, fin, fout, c->geo,
                       c->par, c->act, us, ub, Fr, c->d_flag, tp, nb, T(0));
}

template <int D, typename T> static void bulk_t(tlvlbm_ctx *c, bool repair, void *tape, bool taped) {
  // one instantiation per law: the paper's, the reinforced solid (fibres,
  // body acceleration) and the Maxwell branch (the reverse mode refuses it)
  const bool ext = c->bf || c->par.k1 != 0.0;
  if (tape || taped) {
    if (ext) bulk_tape_t<D, T, Reinforced<D>>(c, repair, tape);
    else bulk_tape_t<D, T, NeoHookean<D>>(c, repair, tape);
    return;
  }
  if (c->par.hist) bulk_plain_t<D, T, Viscoelastic<D>>(c, repair);
  else if (c->par.thf) bulk_plain_t<D, T, Thermal<D>>(c, repair);
  else if (ext) bulk_plain_t<D, T, Reinforced<D>>(c, repair);
  else bulk_plain_t<D, T, NeoHookean<D>>(c, repair);
}

void launch_bulk(tlvlbm_ctx *c, bool repair, void *tape, bool taped) {
  if (c->D == 2) {
    if (c->prec) bulk_t<2, double>(c, repair, tape, taped);
    else bulk_t<2, float>(c, repair, tape, taped);
  } else {
    if (c->prec) bulk_t<3, double>(c, repair, tape, taped);
    else bulk_t<3, float>(c, repair, tape, taped);
  }
}

template <int D, typename T>
static void moments_t(tlvlbm_ctx *c, double *U, double *u, double *J, bool to_scratch) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  const double *us = c->track_u ? (const double *)c->ustar : nullptr;
  const T *bf = (const T *)c->bf;
  const T bs = body_scale<T>(c);
  if (to_scratch) {
    // projection inputs: v, F into the CG workspace, u into the u buffer
    if (c->act)
      hipLaunchKernelGGL((k_moments<D, T, T, true, true>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par, c->act,
                         us, (T *)c->cg.V, (T *)c->cg.Fm, (double *)c->ubuf, (T *)nullptr, (int64_t)c->geo.S, bf, bs);
    else
      hipLaunchKernelGGL((k_moments<D, T, T, false, true>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par,
                         c->act, us, (T *)c->cg.V, (T *)c->cg.Fm, (double *)c->ubuf, (T *)nullptr, (int64_t)c->geo.S, bf,
                         bs);
    return;
  }
  double *Vo = U, *Fo = U ? U + (size_t)D * c->geo.N : nullptr;
  if (c->act)
    hipLaunchKernelGGL((k_moments<D, T, double, true>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par,
                       c->act, us, Vo, Fo, u, J, (int64_t)c->geo.N, bf, bs);
  else
    hipLaunchKernelGGL((k_moments<D, T, double, false>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par,
                       c->act, us, Vo, Fo, u, J, (int64_t)c->geo.N, bf, bs);
}

// moments in the population precision (v and F as stored, J), u in FP64
template <int D, typename T> static void moments_native_t(tlvlbm_ctx *c, void *U, double *u, void *J) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  const double *us = c->track_u ? (const double *)c->ustar : nullptr;
  const T *bf = (const T *)c->bf;
  const T bs = body_scale<T>(c);
  T *Vo = (T *)U, *Fo = U ? (T *)U + (size_t)D * c->geo.N : nullptr;
  if (c->act)
    hipLaunchKernelGGL((k_moments<D, T, T, true>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par, c->act, us,
                       Vo, Fo, u, (T *)J, (int64_t)c->geo.N, bf, bs);
  else
    hipLaunchKernelGGL((k_moments<D, T, T, false>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par, c->act,
                       us, Vo, Fo, u, (T *)J, (int64_t)c->geo.N, bf, bs);
}

void launch_moments_native(tlvlbm_ctx *c, void *U, double *u, void *J) {
  if (c->D == 2) {
    if (c->prec) moments_native_t<2, double>(c, U, u, J);
    else moments_native_t<2, float>(c, U, u, J);
  } else {
    if (c->prec) moments_native_t<3, double>(c, U, u, J);
    else moments_native_t<3, float>(c, U, u, J);
  }
}

void launch_pull_moments(tlvlbm_ctx *c, double *U, double *u, double *J, bool to_scratch) {
  if (c->D == 2) {
    if (c->prec) moments_t<2, double>(c, U, u, J, to_scratch);
    else moments_t<2, float>(c, U, u, J, to_scratch);
  } else {
    if (c->prec) moments_t<3, double>(c, U, u, J, to_scratch);
    else moments_t<3, float>(c, U, u, J, to_scratch);
  }
}

template <int D, typename T> static void stress_t(tlvlbm_ctx *c, double *P, double *S) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  if (c->act)
    hipLaunchKernelGGL((k_stress<D, T, true>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par, c->act, P, S);
  else
    hipLaunchKernelGGL((k_stress<D, T, false>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par, c->act, P,
                       S);
}

void launch_stress(tlvlbm_ctx *c, double *P, double *S) {
  if (c->D == 2) {
    if (c->prec) stress_t<2, double>(c, P, S);
    else stress_t<2, float>(c, P, S);
  } else {
    if (c->prec) stress_t<3, double>(c, P, S);
    else stress_t<3, float>(c, P, S);
  }
}

template <int D, typename T>
static void init_t(tlvlbm_ctx *c, const double *U0, const double *u0, const double *dU0) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  double *us = c->track_u ? (double *)c->ustar : nullptr;
  if (c->act)
    hipLaunchKernelGGL((k_init<D, T, true>), grid, block, 0, c->st, (T *)c->fB, c->geo, c->par, c->act, U0, u0, dU0,
                       us, c->d_flag, (const T *)c->bf, double(body_scale<T>(c)));
  else
    hipLaunchKernelGGL((k_init<D, T, false>), grid, block, 0, c->st, (T *)c->fB, c->geo, c->par, c->act, U0, u0,
                       dU0, us, c->d_flag, (const T *)c->bf, double(body_scale<T>(c)));
}

void launch_init(tlvlbm_ctx *c, const double *U0, const double *u0, const double *dU0) {
  if (c->D == 2) {
    if (c->prec) init_t<2, double>(c, U0, u0, dU0);
    else init_t<2, float>(c, U0, u0, dU0);
  } else {
    if (c->prec) init_t<3, double>(c, U0, u0, dU0);
    else init_t<3, float>(c, U0, u0, dU0);
  }
}

template <int D, typename T> static void getf_t(tlvlbm_ctx *c, double *f, double *us) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  const double *ust = c->track_u ? (const double *)c->ustar : nullptr;
  if (c->act)
    hipLaunchKernelGGL((k_get_f<D, T, true>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par, c->act, ust, f,
                       us);
  else
    hipLaunchKernelGGL((k_get_f<D, T, false>), grid, block, 0, c->st, (const T *)c->fB, c->geo, c->par, c->act, ust, f,
                       us);
}

// caller planes [k][N] (FP64) into context planes [k][S] (population precision)
template <typename T>
__global__ __launch_bounds__(256) void k_planes_in(const double *__restrict__ src, T *__restrict__ dst, int64_t N,
                                                   int64_t S, int k) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N)
    for (int c = 0; c < k; ++c) dst[(size_t)c * S + i] = T(src[(size_t)c * N + i]);
}

void launch_planes_in(tlvlbm_ctx *c, const double *src, void *dst, int k) {
  const unsigned nb = (unsigned)((c->geo.N + 255) / 256);
  if (c->prec)
    hipLaunchKernelGGL((k_planes_in<double>), nb, 256, 0, c->st, src, (double *)dst, c->geo.N, c->geo.S, k);
  else
    hipLaunchKernelGGL((k_planes_in<float>), nb, 256, 0, c->st, src, (float *)dst, c->geo.N, c->geo.S, k);
}

void launch_get_f(tlvlbm_ctx *c, double *f, double *ustar) {
  if (c->D == 2) {
    if (c->prec) getf_t<2, double>(c, f, ustar);
    else getf_t<2, float>(c, f, ustar);
  } else {
    if (c->prec) getf_t<3, double>(c, f, ustar);
    else getf_t<3, float>(c, f, ustar);
  }
}

template <int D, typename T> static void putf_t(tlvlbm_ctx *c, const double *f, const double *us) {
  dim3 grid, block;
  grid_of(c->geo, grid, block);
  double *ust = c->track_u ? (double *)c->ustar : nullptr;
  if (c->act)
    hipLaunchKernelGGL((k_put_f<D, T, true>), grid, block, 0, c->st, (T *)c->fB, c->geo, c->par, c->act, f, us, ust);
  else
    hipLaunchKernelGGL((k_put_f<D, T, false>), grid, block, 0, c->st, (T *)c->fB, c->geo, c->par, c->act, f, us, ust);
}

void launch_put_f(tlvlbm_ctx *c, const double *f, const double *ustar) {
  if (c->D == 2) {
    if (c->prec) putf_t<2, double>(c, f, ustar);
    else putf_t<2, float>(c, f, ustar);
  } else {
    if (c->prec) putf_t<3, double>(c, f, ustar);
    else putf_t<3, float>(c, f, ustar);
  }
}

}  // namespace tl

namespace tl {

// batched launchers: tiles are (instance, k) pairs, nodes k tw .. (k + 1) tw - 1 of the instance
template <int D, typename T>
static void bulk_batch_t(const Inst *insts, const int4 *tiles, int ntiles, bool repair, int tw, hipStream_t st,
                         int law, const int64_t *step) {
  // law 3: the Maxwell branch for the whole batch (no overstress on
  // instances without one); 2: the thermal stretch (th = 1 on instances
  // without a field); 1: the reinforced law (its fibre term vanishes on
  // instances with k1 = 0); 0: the neo-Hookean law
  if (law == 3) {
    if (repair)
      hipLaunchKernelGGL((k_bulk_batch<D, T, true, Viscoelastic<D>>), ntiles, tw, 0, st, insts, tiles, step);
    else
      hipLaunchKernelGGL((k_bulk_batch<D, T, false, Viscoelastic<D>>), ntiles, tw, 0, st, insts, tiles, step);
    return;
  }
  if (law == 2) {
    if (repair)
      hipLaunchKernelGGL((k_bulk_batch<D, T, true, Thermal<D>>), ntiles, tw, 0, st, insts, tiles, step);
    else
      hipLaunchKernelGGL((k_bulk_batch<D, T, false, Thermal<D>>), ntiles, tw, 0, st, insts, tiles, step);
    return;
  }
  if (law == 1) {
    if (repair)
      hipLaunchKernelGGL((k_bulk_batch<D, T, true, Reinforced<D>>), ntiles, tw, 0, st, insts, tiles, step);
    else
      hipLaunchKernelGGL((k_bulk_batch<D, T, false, Reinforced<D>>), ntiles, tw, 0, st, insts, tiles, step);
    return;
  }
  if (repair)
    hipLaunchKernelGGL((k_bulk_batch<D, T, true>), ntiles, tw, 0, st, insts, tiles, step);
  else
    hipLaunchKernelGGL((k_bulk_batch<D, T, false>), ntiles, tw, 0, st, insts, tiles, step);
}

// tw: nodes per tile = threads per workgroup (<= 256)
void launch_bulk_batch(int D, int prec, const Inst *insts, const int4 *tiles, int ntiles, bool repair, int tw,
                       hipStream_t st, int law, const int64_t *step) {
  if (D == 2) {
    if (prec) bulk_batch_t<2, double>(insts, tiles, ntiles, repair, tw, st, law, step);
    else bulk_batch_t<2, float>(insts, tiles, ntiles, repair, tw, st, law, step);
  } else {
    if (prec) bulk_batch_t<3, double>(insts, tiles, ntiles, repair, tw, st, law, step);
    else bulk_batch_t<3, float>(insts, tiles, ntiles, repair, tw, st, law, step);
  }
}

void launch_moments_batch(int D, int prec, const Inst *insts, const int4 *tiles, int ntiles, int tw,
                          hipStream_t st, const int64_t *step) {
  if (D == 2) {
    if (prec) hipLaunchKernelGGL((k_moments_batch<2, double>), ntiles, tw, 0, st, insts, tiles, step);
    else hipLaunchKernelGGL((k_moments_batch<2, float>), ntiles, tw, 0, st, insts, tiles, step);
  } else {
    if (prec) hipLaunchKernelGGL((k_moments_batch<3, double>), ntiles, tw, 0, st, insts, tiles, step);
    else hipLaunchKernelGGL((k_moments_batch<3, float>), ntiles, tw, 0, st, insts, tiles, step);
  }
}

}  // namespace tl
