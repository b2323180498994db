// Geometric multigrid preconditioner for the compatibility projection's
// normal matrix (Sec. 3.5, Eq. 57): K = graph Laplacian of the active nodes
// plus the anchor counts of Dirichlet cut links.
//
// Levels aggregate 2 x 2 (x 2) blocks of the level below.  A coarse operator
// is half the Galerkin product P^T K P with the piecewise-constant
// prolongation P: edge weights sum the fine edges crossing between two
// blocks, anchors sum over the block, and the factor 1/2 makes the coarse
// correction that of the cell-centred Laplacian on the coarse lattice (the
// plain Galerkin product is twice too stiff for constant prolongation, in 2D
// and in 3D).  Every coarse operator is again a weighted graph Laplacian on
// axis neighbours, stored as D float weight planes (exact: multiples of
// powers of 1/2) and a diagonal.  The V-cycle uses damped Jacobi (the same
// sweeps before and after the coarse correction, so the preconditioner is
// symmetric) and Jacobi sweeps on the coarsest level; it is applied to all D
// displacement components at once.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tl_internal.hpp"

namespace tl {

namespace {

constexpr int MT = 256;

// ---------------------------------------------------------------- kernels

template <int D>
__device__ __forceinline__ double apply_K(const MGView &L, const double *x, int64_t i, int x0, int y0, int z0,
                                          int c) {
  const size_t o = (size_t)c * L.stride;
  double s = (double)L.d[i] * x[o + i];
  const int n[3] = {L.nx, L.ny, L.nz};
  const int cc[3] = {x0, y0, z0};
#pragma unroll
  for (int A = 0; A < D; ++A) {
    const int64_t st = A == 0 ? 1 : (A == 1 ? (int64_t)L.nx : (int64_t)L.nx * L.ny);
    const bool per = (L.per >> A) & 1;
    // edge to +A (weight stored at i)
    const float wp = L.w[(size_t)A * L.N + i];
    if (wp != 0.0f) {
      const int64_t j = (cc[A] + 1 < n[A]) ? i + st : i - (int64_t)(n[A] - 1) * st;
      s -= (double)wp * x[o + j];
    }
    // edge from -A (weight stored at the neighbour)
    int64_t j = -1;
    if (cc[A] > 0) j = i - st;
    else if (per) j = i + (int64_t)(n[A] - 1) * st;
    if (j >= 0) {
      const float wm = L.w[(size_t)A * L.N + j];
      if (wm != 0.0f) s -= (double)wm * x[o + j];
    }
  }
  return s;
}

__device__ __forceinline__ void xyz_of(const MGView &L, int64_t i, int &x, int &y, int &z) {
  x = (int)(i % L.nx);
  y = (int)((i / L.nx) % L.ny);
  z = (int)(i / ((int64_t)L.nx * L.ny));
}

// xout = first ? om b / d : xin + om (b - K xin) / d  (tiles: 256-node tiles
// holding active nodes; null = all)
template <int D>
__global__ __launch_bounds__(MT) void k_mg_smooth(MGView L, const double *__restrict__ b, const double *__restrict__ xin,
                                                  double *__restrict__ xout, double om, int first,
                                                  const double *__restrict__ scal, const int32_t *__restrict__ tiles) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int64_t i = (tiles ? (int64_t)tiles[blockIdx.x] : (int64_t)blockIdx.x) * MT + threadIdx.x;
  if (i >= L.N) return;
  const float d = L.d[i];
  if (d == 0.0f) {
    for (int c = 0; c < D; ++c) xout[(size_t)c * L.stride + i] = 0.0;
    return;
  }
  const double id = 1.0 / (double)d;
  if (first) {
    for (int c = 0; c < D; ++c) xout[(size_t)c * L.stride + i] = om * b[(size_t)c * L.stride + i] * id;
    return;
  }
  int x, y, z;
  xyz_of(L, i, x, y, z);
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * L.stride + i;
    xout[o] = xin[o] + om * (b[o] - apply_K<D>(L, xin, i, x, y, z, c)) * id;
  }
}

// bc(C) = sum over the children f of C of (b - K x)(f)
template <int D>
__global__ __launch_bounds__(MT) void k_mg_restrict(MGView F, MGView Cg, const double *__restrict__ b,
                                                    const double *__restrict__ x, double *__restrict__ bc,
                                                    const double *__restrict__ scal) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (I >= Cg.N) return;
  int cx, cy, cz;
  xyz_of(Cg, I, cx, cy, cz);
  double acc[D];
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int fx = 2 * cx + dx, fy = 2 * cy + dy, fz = 2 * cz + dz;
        if (fx >= F.nx || fy >= F.ny || fz >= F.nz) continue;
        const int64_t f = fx + (int64_t)F.nx * (fy + (int64_t)F.ny * fz);
        if (F.d[f] == 0.0f) continue;
        for (int c = 0; c < D; ++c)
          acc[c] += b[(size_t)c * F.stride + f] - apply_K<D>(F, x, f, fx, fy, fz, c);
      }
  for (int c = 0; c < D; ++c) bc[(size_t)c * Cg.stride + I] = acc[c];
}

// x(f) += xc(parent(f)) on nodes with a non-zero diagonal
template <int D>
__global__ __launch_bounds__(MT) void k_mg_prolong(MGView F, MGView Cg, const double *__restrict__ xc,
                                                   double *__restrict__ x, const double *__restrict__ scal,
                                                   const int32_t *__restrict__ tiles) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int64_t i = (tiles ? (int64_t)tiles[blockIdx.x] : (int64_t)blockIdx.x) * MT + threadIdx.x;
  if (i >= F.N || F.d[i] == 0.0f) return;
  int fx, fy, fz;
  xyz_of(F, i, fx, fy, fz);
  const int64_t I = (fx >> 1) + (int64_t)Cg.nx * ((fy >> 1) + (int64_t)Cg.ny * (fz >> 1));
  for (int c = 0; c < D; ++c) x[(size_t)c * F.stride + i] += xc[(size_t)c * Cg.stride + I];
}

inline unsigned nb(int64_t n) { return (unsigned)((n + MT - 1) / MT); }

// the coarsest level (at most CT nodes): all Jacobi sweeps in one block, in LDS
constexpr int CT = 512;
template <int D>
__global__ __launch_bounds__(CT) void k_mg_coarse(MGView L, const double *__restrict__ b, double *__restrict__ x,
                                                  double om, int nsweep, const double *__restrict__ scal) {
  if (scal && scal[S_DONE] != 0.0) return;
  __shared__ double xs[2][D][CT];
  const int i = threadIdx.x;
  const bool on = i < L.N;
  const double d = on ? (double)L.d[i] : 0.0;
  double bi[D];
  for (int c = 0; c < D; ++c) {
    bi[c] = (on && d != 0.0) ? b[(size_t)c * L.stride + i] : 0.0;
    xs[0][c][i] = (d != 0.0) ? om * bi[c] / d : 0.0;
  }
  int x0 = 0, y0 = 0, z0 = 0;
  if (on) {
    x0 = i % L.nx;
    y0 = (i / L.nx) % L.ny;
    z0 = i / (L.nx * L.ny);
  }
  __syncthreads();
  int cur = 0;
  for (int s = 1; s < nsweep; ++s) {
    if (on && d != 0.0) {
      for (int c = 0; c < D; ++c) {
        double kx = d * xs[cur][c][i];
        const int n[3] = {L.nx, L.ny, L.nz};
        const int cc[3] = {x0, y0, z0};
        for (int A = 0; A < D; ++A) {
          const int st = A == 0 ? 1 : (A == 1 ? L.nx : L.nx * L.ny);
          const float wp = L.w[(size_t)A * L.N + i];
          if (wp != 0.0f) kx -= (double)wp * xs[cur][c][(cc[A] + 1 < n[A]) ? i + st : i - (n[A] - 1) * st];
          int j = -1;
          if (cc[A] > 0) j = i - st;
          else if ((L.per >> A) & 1) j = i + (n[A] - 1) * st;
          if (j >= 0) {
            const float wm = L.w[(size_t)A * L.N + j];
            if (wm != 0.0f) kx -= (double)wm * xs[cur][c][j];
          }
        }
        xs[cur ^ 1][c][i] = xs[cur][c][i] + om * (bi[c] - kx) / d;
      }
    } else {
      for (int c = 0; c < D; ++c) xs[cur ^ 1][c][i] = 0.0;
    }
    __syncthreads();
    cur ^= 1;
  }
  if (on)
    for (int c = 0; c < D; ++c) x[(size_t)c * L.stride + i] = xs[cur][c][i];
}

// per-tile sums of ua (+ ub) over the nodes of components without anchors
template <int D>
__global__ __launch_bounds__(MT) void k_gauge_tiles(const int32_t *__restrict__ cn, Geo g, const double *__restrict__ ua,
                                                    const double *__restrict__ ub, double *__restrict__ tpart) {
  __shared__ double sh[MT / 64][D];
  const int32_t j = cn[(size_t)blockIdx.x * MT + threadIdx.x];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = 0; i < D; ++i) {
    double v = 0.0;
    if (j >= 0) v = ua[(size_t)i * g.S + j] + (ub ? ub[(size_t)i * g.S + j] : 0.0);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wid][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < D) {
    double s = 0.0;
    for (int w = 0; w < MT / 64; ++w) s += sh[w][threadIdx.x];
    tpart[(size_t)blockIdx.x * D + threadIdx.x] = s;
  }
}

// component means from the tile sums (one block per component, fixed order)
template <int D>
__global__ __launch_bounds__(MT) void k_gauge_comp(const int64_t *__restrict__ ct, const int64_t *__restrict__ cnt,
                                                   const double *__restrict__ tpart, double *__restrict__ mean) {
  __shared__ double sh[MT / 64][D];
  const int c = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = 0; i < D; ++i) {
    double v = 0.0;
    for (int64_t t = ct[c] + threadIdx.x; t < ct[c + 1]; t += MT) v += tpart[t * D + i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wid][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < D) {
    double s = 0.0;
    for (int w = 0; w < MT / 64; ++w) s += sh[w][threadIdx.x];
    mean[(size_t)c * D + threadIdx.x] = s / double(cnt[c]);
  }
}

template <int D>
__global__ __launch_bounds__(MT) void k_gauge_shift(Geo g, const int32_t *__restrict__ comp,
                                                    const double *__restrict__ mean, const double *__restrict__ mean0,
                                                    double *__restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const int32_t c = comp[i];
  if (c < 0) return;
  for (int k = 0; k < D; ++k) x[(size_t)k * g.S + i] -= mean[(size_t)c * D + k] - mean0[(size_t)c * D + k];
}

// smoothing sweeps on level l: result in lev.x (b = lev.b); `cold` starts from 0
// sweeps on level l from lev.x (or from 0 when cold); the result is left in
// lev.x, or written to `out` by the last sweep
template <int D>
void sweeps(MG &mg, int l, int n, bool cold, hipStream_t st, const double *scal, double *out = nullptr) {
  MGLevel &L = mg.lev[l];
  const int32_t *tl = l == 0 ? mg.tiles : nullptr;
  const unsigned grid = tl ? (unsigned)mg.ntiles : nb(L.v.N);
  for (int s = 0; s < n; ++s) {
    double *dst = (out && s == n - 1) ? out : L.t;
    hipLaunchKernelGGL((k_mg_smooth<D>), grid, MT, 0, st, L.v, L.b, L.x, dst, mg.omega, (cold && s == 0) ? 1 : 0,
                       scal, tl);
    if (dst == L.t) std::swap(L.x, L.t);
  }
}

template <int D> void vcycle(MG &mg, int l, hipStream_t st, const double *scal, double *out) {
  const int last = (int)mg.lev.size() - 1;
  MGLevel &F = mg.lev[l];
  if (l == last) {
    if (F.v.N <= CT)
      hipLaunchKernelGGL((k_mg_coarse<D>), 1, CT, 0, st, F.v, F.b, out ? out : F.x, mg.omega, mg.nu_coarse, scal);
    else
      sweeps<D>(mg, l, mg.nu_coarse, true, st, scal, out);
    return;
  }
  MGLevel &Cg = mg.lev[l + 1];
  const int32_t *tl = l == 0 ? mg.tiles : nullptr;
  sweeps<D>(mg, l, mg.nu, true, st, scal);
  hipLaunchKernelGGL((k_mg_restrict<D>), nb(Cg.v.N), MT, 0, st, F.v, Cg.v, F.b, F.x, Cg.b, scal);
  vcycle<D>(mg, l + 1, st, scal, nullptr);
  hipLaunchKernelGGL((k_mg_prolong<D>), tl ? (unsigned)mg.ntiles : nb(F.v.N), MT, 0, st, F.v, Cg.v, Cg.x, F.x, scal,
                     tl);
  sweeps<D>(mg, l, mg.nu, false, st, scal, out);
}


// ------------------------------------------- batched (level-synchronous) V-cycle
// tiles: (instance, block of MT nodes of the level); each instance's level
// data in tab[inst*lmax + level].  Sweep sources and targets: phase 0 A <- b
// (cold), 1 B <- A, 2 A <- B, 3 z <- A (last post sweep of the finest level).

template <int D>
__global__ __launch_bounds__(MT) void k_bmg_smooth(const BMGLev *__restrict__ tab, int lmax, int l,
                                                   const int4 *__restrict__ tiles, int phase, double om,
                                                   const Inst *__restrict__ insts) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  if (((const double *)I.scal)[S_DONE] != 0.0) return;
  const BMGLev &Lv = tab[(size_t)t.x * lmax + l];
  const MGView &L = Lv.v;
  const int64_t i = (int64_t)t.y * MT + threadIdx.x;
  if (i >= L.N) return;
  const double *src = phase == 1 || phase == 3 ? Lv.A : Lv.B;
  double *dst = phase == 0 || phase == 2 ? Lv.A : (phase == 1 ? Lv.B : (double *)I.z);
  const float d = L.d[i];
  if (d == 0.0f) {
    for (int c = 0; c < D; ++c) dst[(size_t)c * L.stride + i] = 0.0;
    return;
  }
  const double id = 1.0 / (double)d;
  if (phase == 0) {
    for (int c = 0; c < D; ++c) dst[(size_t)c * L.stride + i] = om * Lv.b[(size_t)c * L.stride + i] * id;
    return;
  }
  int x, y, z;
  xyz_of(L, i, x, y, z);
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * L.stride + i;
    dst[o] = src[o] + om * (Lv.b[o] - apply_K<D>(L, src, i, x, y, z, c)) * id;
  }
}

// level l+1 right-hand side = restricted residual of level l (from B)
template <int D>
__global__ __launch_bounds__(MT) void k_bmg_restrict(const BMGLev *__restrict__ tab, int lmax, int l,
                                                     const int4 *__restrict__ tiles, const Inst *__restrict__ insts) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  if (((const double *)I.scal)[S_DONE] != 0.0) return;
  const BMGLev &Fl = tab[(size_t)t.x * lmax + l], &Cl = tab[(size_t)t.x * lmax + l + 1];
  const MGView &F = Fl.v, &Cg = Cl.v;
  const int64_t Ic = (int64_t)t.y * MT + threadIdx.x;
  if (Ic >= Cg.N) return;
  int cx, cy, cz;
  xyz_of(Cg, Ic, cx, cy, cz);
  double acc[D];
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int fx = 2 * cx + dx, fy = 2 * cy + dy, fz = 2 * cz + dz;
        if (fx >= F.nx || fy >= F.ny || fz >= F.nz) continue;
        const int64_t f = fx + (int64_t)F.nx * (fy + (int64_t)F.ny * fz);
        if (F.d[f] == 0.0f) continue;
        for (int c = 0; c < D; ++c)
          acc[c] += Fl.b[(size_t)c * F.stride + f] - apply_K<D>(F, Fl.B, f, fx, fy, fz, c);
      }
  for (int c = 0; c < D; ++c) Cl.b[(size_t)c * Cg.stride + Ic] = acc[c];
}

// B_l += B_{l+1}(parent)
template <int D>
__global__ __launch_bounds__(MT) void k_bmg_prolong(const BMGLev *__restrict__ tab, int lmax, int l,
                                                    const int4 *__restrict__ tiles, const Inst *__restrict__ insts) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  if (((const double *)I.scal)[S_DONE] != 0.0) return;
  const BMGLev &Fl = tab[(size_t)t.x * lmax + l], &Cl = tab[(size_t)t.x * lmax + l + 1];
  const MGView &F = Fl.v, &Cg = Cl.v;
  const int64_t i = (int64_t)t.y * MT + threadIdx.x;
  if (i >= F.N || F.d[i] == 0.0f) return;
  int fx, fy, fz;
  xyz_of(F, i, fx, fy, fz);
  const int64_t Ic = (fx >> 1) + (int64_t)Cg.nx * ((fy >> 1) + (int64_t)Cg.ny * (fz >> 1));
  for (int c = 0; c < D; ++c) Fl.B[(size_t)c * F.stride + i] += Cl.B[(size_t)c * Cg.stride + Ic];
}

// coarsest level of every instance (one block each): Jacobi sweeps in LDS,
// result to B (or z when the finest level is the coarsest)
template <int D>
__global__ __launch_bounds__(CT) void k_bmg_coarse(const BMGLev *__restrict__ tab, int lmax,
                                                   const int *__restrict__ last, double om, int nsweep,
                                                   const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  if (((const double *)I.scal)[S_DONE] != 0.0) return;
  const int l = last[blockIdx.x];
  const BMGLev &Lv = tab[(size_t)blockIdx.x * lmax + l];
  const MGView &L = Lv.v;
  __shared__ double xs[2][D][CT];
  const int i = threadIdx.x;
  const bool on = i < L.N;
  const double d = on ? (double)L.d[i] : 0.0;
  double bi[D];
  for (int c = 0; c < D; ++c) {
    bi[c] = (on && d != 0.0) ? Lv.b[(size_t)c * L.stride + i] : 0.0;
    xs[0][c][i] = (d != 0.0) ? om * bi[c] / d : 0.0;
  }
  int x0 = 0, y0 = 0, z0 = 0;
  if (on) {
    x0 = i % L.nx;
    y0 = (i / L.nx) % L.ny;
    z0 = i / (L.nx * L.ny);
  }
  __syncthreads();
  int cur = 0;
  for (int s = 1; s < nsweep; ++s) {
    if (on && d != 0.0) {
      for (int c = 0; c < D; ++c) {
        double kx = d * xs[cur][c][i];
        const int n[3] = {L.nx, L.ny, L.nz};
        const int cc[3] = {x0, y0, z0};
        for (int A = 0; A < D; ++A) {
          const int st = A == 0 ? 1 : (A == 1 ? L.nx : L.nx * L.ny);
          const float wp = L.w[(size_t)A * L.N + i];
          if (wp != 0.0f) kx -= (double)wp * xs[cur][c][(cc[A] + 1 < n[A]) ? i + st : i - (n[A] - 1) * st];
          int j = -1;
          if (cc[A] > 0) j = i - st;
          else if ((L.per >> A) & 1) j = i + (n[A] - 1) * st;
          if (j >= 0) {
            const float wm = L.w[(size_t)A * L.N + j];
            if (wm != 0.0f) kx -= (double)wm * xs[cur][c][j];
          }
        }
        xs[cur ^ 1][c][i] = xs[cur][c][i] + om * (bi[c] - kx) / d;
      }
    } else {
      for (int c = 0; c < D; ++c) xs[cur ^ 1][c][i] = 0.0;
    }
    __syncthreads();
    cur ^= 1;
  }
  double *out = l == 0 ? (double *)I.z : Lv.B;
  if (on)
    for (int c = 0; c < D; ++c) out[(size_t)c * L.stride + i] = xs[cur][c][i];
}

template <int D> void batch_vcycle_t(const BatchMG &bm, const Inst *insts, int ninst, hipStream_t st) {
  const int L = bm.lmax;
  // descent: pre-smoothing and restriction on the levels above each
  // instance's coarsest
  for (int l = 0; l + 1 < L; ++l) {
    if (!bm.nsm[l]) continue;
    hipLaunchKernelGGL((k_bmg_smooth<D>), bm.nsm[l], MT, 0, st, bm.tab, L, l, bm.sm[l], 0, bm.omega, insts);
    hipLaunchKernelGGL((k_bmg_smooth<D>), bm.nsm[l], MT, 0, st, bm.tab, L, l, bm.sm[l], 1, bm.omega, insts);
    if (bm.nrs[l + 1])
      hipLaunchKernelGGL((k_bmg_restrict<D>), bm.nrs[l + 1], MT, 0, st, bm.tab, L, l, bm.rs[l + 1], insts);
  }
  hipLaunchKernelGGL((k_bmg_coarse<D>), ninst, CT, 0, st, bm.tab, L, bm.last, bm.omega, bm.nu_coarse, insts);
  // ascent: prolongation and post-smoothing
  for (int l = L - 2; l >= 0; --l) {
    if (!bm.nsm[l]) continue;
    hipLaunchKernelGGL((k_bmg_prolong<D>), bm.nsm[l], MT, 0, st, bm.tab, L, l, bm.sm[l], insts);
    hipLaunchKernelGGL((k_bmg_smooth<D>), bm.nsm[l], MT, 0, st, bm.tab, L, l, bm.sm[l], 2, bm.omega, insts);
    hipLaunchKernelGGL((k_bmg_smooth<D>), bm.nsm[l], MT, 0, st, bm.tab, L, l, bm.sm[l], l == 0 ? 3 : 1, bm.omega,
                       insts);
  }
}
}  // namespace

namespace {

void gauge_free(tlvlbm_ctx *c, Gauge *G) {
  if (!G) return;
  for (void *p : {(void *)G->comp, (void *)G->cn, (void *)G->ct, (void *)G->ccnt, (void *)G->tpart,
                  (void *)G->mean, (void *)G->mean0, (void *)G->anc_n})
    dfree(c, p);
  delete G;
}

void mg_free(tlvlbm_ctx *c, MG *mg) {
  if (!mg) return;
  for (MGLevel &L : mg->lev) {
    for (void *p : {(void *)L.w, (void *)L.d, (void *)L.x, (void *)L.t}) dfree(c, p);
    if (L.b) dfree(c, L.b);  // level 0 borrows the CG residual only inside mg_apply
  }
  delete mg;
}

// components of the active graph (breadth-first over lattice neighbours)
// and the tile lists of those without anchors
int gauge_build(tlvlbm_ctx *c, const std::vector<uint8_t> &act, const std::vector<float> &anc, Gauge **out) {
  const Geo &g = c->geo;
  const int D = c->D;
  const int64_t N = g.N;
  std::vector<int32_t> cid(N, -1);
  std::vector<int64_t> stack;
  int32_t nc = 0;
  const int n3[3] = {g.nx, g.ny, g.nz};
  for (int64_t s0 = 0; s0 < N; ++s0) {
    if (!act[s0] || cid[s0] >= 0) continue;
    cid[s0] = nc;
    stack.assign(1, s0);
    while (!stack.empty()) {
      const int64_t m = stack.back();
      stack.pop_back();
      const int cc[3] = {(int)(m % g.nx), (int)((m / g.nx) % g.ny), (int)(m / ((int64_t)g.nx * g.ny))};
      for (int q = 0; q < 2 * D; ++q) {
        int v[3] = {cc[0], cc[1], cc[2]};
        const int A = q / 2;
        v[A] += (q & 1) ? -1 : 1;
        if (v[A] < 0 || v[A] >= n3[A]) {
          if (!((g.per >> A) & 1)) continue;
          v[A] = (v[A] + n3[A]) % n3[A];
        }
        const int64_t j = v[0] + (int64_t)g.nx * (v[1] + (int64_t)g.ny * v[2]);
        if (act[j] && cid[j] < 0) {
          cid[j] = nc;
          stack.push_back(j);
        }
      }
    }
    ++nc;
  }
  std::vector<uint8_t> anch(nc, 0);
  for (int64_t m = 0; m < N; ++m)
    if (act[m] && anc[m] > 0.0f) anch[cid[m]] = 1;
  std::vector<int32_t> uidx(nc, -1);
  int32_t nu = 0;
  for (int32_t k = 0; k < nc; ++k)
    if (!anch[k]) uidx[k] = nu++;
  std::vector<int32_t> comp(N, -1);
  std::vector<std::vector<int32_t>> members(nu);
  for (int64_t m = 0; m < N; ++m)
    if (act[m] && uidx[cid[m]] >= 0) {
      comp[m] = uidx[cid[m]];
      members[comp[m]].push_back((int32_t)m);
    }
  std::vector<int32_t> cn;
  std::vector<int64_t> ct(nu + 1, 0), ccnt(nu + 1, 0);
  for (int32_t k = 0; k < nu; ++k) {
    ct[k] = (int64_t)(cn.size() / MT);
    ccnt[k] = (int64_t)members[k].size();
    cn.insert(cn.end(), members[k].begin(), members[k].end());
    while (cn.size() % MT) cn.push_back(-1);
  }
  ct[nu] = (int64_t)(cn.size() / MT);
  std::vector<uint8_t> an(N, 0);
  for (int64_t m = 0; m < N; ++m) an[m] = (uint8_t)anc[m];
  Gauge *G = new (std::nothrow) Gauge();
  if (!G) return TLVLBM_ERR_OUT_OF_MEMORY;
  G->nu = nu;
  G->ntile = ct[nu];
  const size_t ncn = std::max<size_t>(cn.size(), 1);
  if (dmalloc(c, &G->comp, N * sizeof(int32_t)) || dmalloc(c, &G->cn, ncn * sizeof(int32_t)) ||
      dmalloc(c, &G->ct, ct.size() * sizeof(int64_t)) || dmalloc(c, &G->ccnt, ccnt.size() * sizeof(int64_t)) ||
      dmalloc(c, &G->tpart, ((size_t)G->ntile + 1) * D * sizeof(double)) ||
      dmalloc(c, &G->mean, ((size_t)nu + 1) * D * sizeof(double)) ||
      dmalloc(c, &G->mean0, ((size_t)nu + 1) * D * sizeof(double)) || dmalloc(c, &G->anc_n, N)) {
    gauge_free(c, G);
    return TLVLBM_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(G->comp, comp.data(), N * sizeof(int32_t), hipMemcpyHostToDevice) ||
      (cn.size() && hipMemcpy(G->cn, cn.data(), cn.size() * sizeof(int32_t), hipMemcpyHostToDevice)) ||
      hipMemcpy(G->ct, ct.data(), ct.size() * sizeof(int64_t), hipMemcpyHostToDevice) ||
      hipMemcpy(G->ccnt, ccnt.data(), ccnt.size() * sizeof(int64_t), hipMemcpyHostToDevice) ||
      hipMemcpy(G->anc_n, an.data(), N, hipMemcpyHostToDevice)) {
    gauge_free(c, G);
    return TLVLBM_ERR_DEVICE;
  }
  *out = G;
  return TLVLBM_OK;
}

int mg_build(tlvlbm_ctx *c, const std::vector<uint8_t> &act, const std::vector<float> &anc, MG **out);

}  // namespace

void proj_aux_free(tlvlbm_ctx *c) {
  if (c->cg.pcg_graph) (void)hipGraphExecDestroy(c->cg.pcg_graph);
  c->cg.pcg_graph = nullptr;
  if (c->stT) {
    for (void *p : {(void *)c->stT->sn, (void *)c->stT->so, (void *)c->stT->el, (void *)c->stT->ek,
                    (void *)c->stT->ew, (void *)c->stT->sc})
      dfree(c, p);
    delete c->stT;
    c->stT = nullptr;
  }
  gauge_free(c, c->gauge);
  c->gauge = nullptr;
  mg_free(c, c->mg);
  c->mg = nullptr;
}

// Host-side preparation of the projection (once per geometry and
// boundary-condition set): active mask and anchor counts, the components
// without anchors, and the multigrid hierarchy when it is enabled.
int proj_aux_build(tlvlbm_ctx *c) {
  const Geo &g = c->geo;
  const int64_t N = g.N;
  std::vector<uint8_t> act(N, 1);
  if (c->act && hipMemcpy(act.data(), c->act, N, hipMemcpyDeviceToHost) != hipSuccess) return TLVLBM_ERR_DEVICE;
  std::vector<float> anc(N, 0.0f);
  {
    const int64_t nl = c->L.n;
    std::vector<int64_t> node(nl);
    if (nl && hipMemcpy(node.data(), c->L.node, nl * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
      return TLVLBM_ERR_DEVICE;
    for (int b = 0; b < 256; ++b)
      if (c->bcs[b].type == TLVLBM_BC_DIRICHLET_VELOCITY)
        for (int64_t l = c->bid_begin[b]; l < c->bid_end[b]; ++l) anc[node[l]] += 1.0f;
  }
  proj_aux_free(c);
  // 256-node tiles that hold active nodes: the single-instance CG and the
  // finest multigrid sweeps skip the rest
  {
    std::vector<int32_t> tiles;
    for (int64_t t = 0; t * 256 < N; ++t) {
      bool any = false;
      for (int64_t i = t * 256; i < std::min<int64_t>(N, t * 256 + 256) && !any; ++i) any = act[i] != 0;
      if (any) tiles.push_back((int32_t)t);
    }
    if (c->cg.tiles) dfree(c, c->cg.tiles);
    c->cg.tiles = nullptr;
    c->cg.ntiles = 0;
    if (c->cg.jt) dfree(c, c->cg.jt);
    c->cg.jt = nullptr;
    c->cg.njt = 0;
    // 2D: the tiles of the fused Jacobi sweeps
    std::vector<int32_t> jt;
    if (c->D == 2 && active_tiles2(g, act.data(), jt) && !jt.empty()) {
      if (dmalloc(c, &c->cg.jt, jt.size() * sizeof(int32_t)) != hipSuccess) return TLVLBM_ERR_OUT_OF_MEMORY;
      if (hipMemcpy(c->cg.jt, jt.data(), jt.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
        return TLVLBM_ERR_DEVICE;
      c->cg.njt = (int)jt.size();
    }
    // neighbour masks of the active-node graph: the Jacobi sweeps read one
    // byte per node instead of the seven activity flags and coordinates
    std::vector<uint8_t> nbm(N, 0);
    const int64_t nxy = (int64_t)g.nx * g.ny;
    for (int64_t i = 0; i < N; ++i) {
      if (!act[i]) continue;
      const int c3[3] = {(int)(i % g.nx), (int)((i / g.nx) % g.ny), (int)(i / nxy)};
      const int n3[3] = {g.nx, g.ny, g.nz};
      uint8_t m = 64;
      for (int q = 0; q < 2 * c->D; ++q) {
        int v[3] = {c3[0], c3[1], c3[2]};
        const int A = q / 2;
        v[A] += (q & 1) ? -1 : 1;
        if (v[A] < 0 || v[A] >= n3[A]) {
          if (!((g.per >> A) & 1)) continue;
          v[A] = (v[A] + n3[A]) % n3[A];
        }
        if (act[v[0] + (int64_t)g.nx * (v[1] + (int64_t)g.ny * v[2])]) m |= (uint8_t)(1u << q);
      }
      nbm[i] = m;
    }
    if (c->cg.nbm) dfree(c, c->cg.nbm);
    c->cg.nbm = nullptr;
    if (dmalloc(c, &c->cg.nbm, N) != hipSuccess) return TLVLBM_ERR_OUT_OF_MEMORY;
    if (hipMemcpy(c->cg.nbm, nbm.data(), N, hipMemcpyHostToDevice) != hipSuccess) return TLVLBM_ERR_DEVICE;
    if (!tiles.empty()) {
      if (dmalloc(c, &c->cg.tiles, tiles.size() * sizeof(int32_t)) != hipSuccess) return TLVLBM_ERR_OUT_OF_MEMORY;
      if (hipMemcpy(c->cg.tiles, tiles.data(), tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
        return TLVLBM_ERR_DEVICE;
      c->cg.ntiles = (int)tiles.size();
    }
  }
  int s = gauge_build(c, act, anc, &c->gauge);
  if (s) return s;
  if (c->cg_multigrid && c->proj_sweeps == 0) {  // the exact mode's preconditioner
    s = mg_build(c, act, anc, &c->mg);
    if (s) return s;
  }
  c->aux_stale = false;
  return TLVLBM_OK;
}

void gauge_means(tlvlbm_ctx *c, const double *ua, const double *ub, double *mean) {
  const Gauge &G = *c->gauge;
  if (!G.nu) return;
  if (c->D == 2) {
    hipLaunchKernelGGL((k_gauge_tiles<2>), (unsigned)G.ntile, MT, 0, c->st, G.cn, c->geo, ua, ub, G.tpart);
    hipLaunchKernelGGL((k_gauge_comp<2>), (unsigned)G.nu, MT, 0, c->st, G.ct, G.ccnt, G.tpart, mean);
  } else {
    hipLaunchKernelGGL((k_gauge_tiles<3>), (unsigned)G.ntile, MT, 0, c->st, G.cn, c->geo, ua, ub, G.tpart);
    hipLaunchKernelGGL((k_gauge_comp<3>), (unsigned)G.nu, MT, 0, c->st, G.ct, G.ccnt, G.tpart, mean);
  }
}

void gauge_restore(tlvlbm_ctx *c, double *x, const double *mean0) {
  const Gauge &G = *c->gauge;
  if (!G.nu) return;
  gauge_means(c, x, nullptr, G.mean);
  if (c->D == 2)
    hipLaunchKernelGGL((k_gauge_shift<2>), nb(c->geo.N), MT, 0, c->st, c->geo, G.comp, G.mean, mean0, x);
  else
    hipLaunchKernelGGL((k_gauge_shift<3>), nb(c->geo.N), MT, 0, c->st, c->geo, G.comp, G.mean, mean0, x);
}

namespace {

// multigrid hierarchy from the active mask and the anchor counts
int mg_build(tlvlbm_ctx *c, const std::vector<uint8_t> &act, const std::vector<float> &anc, MG **out) {
  const Geo &g = c->geo;
  const int D = c->D;
  const int64_t N = g.N;
  MG *mg = new (std::nothrow) MG();
  if (!mg) return TLVLBM_ERR_OUT_OF_MEMORY;
  mg->omega = 2.0 / 3.0;
  mg->nu = 2;
  mg->nu_coarse = 40;
  // level 0: unit weights between active neighbours
  struct HL {
    int n[3], per;
    std::vector<float> w, a;
  };
  std::vector<HL> H;
  {
    HL h;
    h.n[0] = g.nx;
    h.n[1] = g.ny;
    h.n[2] = g.nz;
    h.per = g.per;
    h.w.assign((size_t)D * N, 0.0f);
    h.a = anc;
    for (int64_t i = 0; i < N; ++i) {
      if (!act[i]) continue;
      const int cc[3] = {(int)(i % g.nx), (int)((i / g.nx) % g.ny), (int)(i / ((int64_t)g.nx * g.ny))};
      for (int A = 0; A < D; ++A) {
        int v[3] = {cc[0], cc[1], cc[2]};
        if (++v[A] >= h.n[A]) {
          if (!((g.per >> A) & 1) || h.n[A] == 1) continue;
          v[A] = 0;
        }
        const int64_t j = v[0] + (int64_t)g.nx * (v[1] + (int64_t)g.ny * v[2]);
        if (j != i && act[j]) h.w[(size_t)A * N + i] = 1.0f;
      }
    }
    H.push_back(std::move(h));
  }
  // coarser levels: half the Galerkin product with constant prolongation
  while (H.size() < 16) {
    const HL &f = H.back();
    int64_t nf = (int64_t)f.n[0] * f.n[1] * f.n[2];
    bool coarsen = nf > 512;
    for (int A = 0; A < D; ++A) coarsen = coarsen && f.n[A] >= 2;
    if (!coarsen) break;
    HL h;
    for (int A = 0; A < 3; ++A) h.n[A] = A < D ? (f.n[A] + 1) / 2 : 1;
    h.per = f.per;
    const int64_t nc = (int64_t)h.n[0] * h.n[1] * h.n[2];
    h.w.assign((size_t)D * nc, 0.0f);
    h.a.assign(nc, 0.0f);
    for (int64_t i = 0; i < nf; ++i) {
      const int cc[3] = {(int)(i % f.n[0]), (int)((i / f.n[0]) % f.n[1]), (int)(i / ((int64_t)f.n[0] * f.n[1]))};
      const int pc[3] = {cc[0] / 2, cc[1] / 2, cc[2] / 2};
      const int64_t I = pc[0] + (int64_t)h.n[0] * (pc[1] + (int64_t)h.n[1] * pc[2]);
      h.a[I] += 0.5f * f.a[i];
      for (int A = 0; A < D; ++A) {
        const float w = f.w[(size_t)A * nf + i];
        if (w == 0.0f) continue;
        int v[3] = {cc[0], cc[1], cc[2]};
        if (++v[A] >= f.n[A]) v[A] = 0;  // stored only where the edge exists
        int q[3] = {v[0] / 2, v[1] / 2, v[2] / 2};
        if (q[A] == pc[A]) continue;  // inside one block
        // the edge joins block I to its +A neighbour (wrapping)
        h.w[(size_t)A * nc + I] += 0.5f * w;
      }
    }
    H.push_back(std::move(h));
  }
  // upload
  mg->lev.resize(H.size());
  for (size_t l = 0; l < H.size(); ++l) {
    HL &h = H[l];
    MGLevel &L = mg->lev[l];
    const int64_t n = (int64_t)h.n[0] * h.n[1] * h.n[2];
    std::vector<float> d(n, 0.0f);
    for (int64_t i = 0; i < n; ++i) {
      const int cc[3] = {(int)(i % h.n[0]), (int)((i / h.n[0]) % h.n[1]), (int)(i / ((int64_t)h.n[0] * h.n[1]))};
      float s = h.a[i];
      for (int A = 0; A < D; ++A) {
        s += h.w[(size_t)A * n + i];
        int v[3] = {cc[0], cc[1], cc[2]};
        if (--v[A] < 0) {
          if (!((h.per >> A) & 1)) continue;
          v[A] = h.n[A] - 1;
        }
        const int64_t j = v[0] + (int64_t)h.n[0] * (v[1] + (int64_t)h.n[1] * v[2]);
        s += h.w[(size_t)A * n + j];
      }
      d[i] = s;
    }
    L.v.nx = h.n[0];
    L.v.ny = h.n[1];
    L.v.nz = h.n[2];
    L.v.per = h.per;
    L.v.N = n;
    L.v.stride = l == 0 ? g.S : n;
    float *w = nullptr, *dd = nullptr;
    if (dmalloc(c, &w, (size_t)D * n * sizeof(float)) != hipSuccess ||
        dmalloc(c, &dd, (size_t)n * sizeof(float)) != hipSuccess) {
      if (w) dfree(c, w);
      mg_free(c, mg);
      return TLVLBM_ERR_OUT_OF_MEMORY;
    }
    L.w = w;
    L.d = dd;
    L.v.w = w;
    L.v.d = dd;
    if (hipMemcpy(w, h.w.data(), (size_t)D * n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dd, d.data(), (size_t)n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      mg_free(c, mg);
      return TLVLBM_ERR_DEVICE;
    }
    const size_t vb = (size_t)D * L.v.stride * sizeof(double);
    if (dmalloc(c, &L.x, vb) != hipSuccess || dmalloc(c, &L.t, vb) != hipSuccess ||
        (l > 0 && dmalloc(c, &L.b, vb) != hipSuccess)) {
      mg_free(c, mg);
      return TLVLBM_ERR_OUT_OF_MEMORY;
    }
    if (hipMemset(L.x, 0, vb) != hipSuccess || hipMemset(L.t, 0, vb) != hipSuccess ||
        (l > 0 && hipMemset(L.b, 0, vb) != hipSuccess)) {
      mg_free(c, mg);
      return TLVLBM_ERR_DEVICE;
    }
  }
  *out = mg;
  return TLVLBM_OK;
}

}  // namespace

// z = M^{-1} r (one V-cycle); r and z are [D][S] FP64 planes
void mg_apply(tlvlbm_ctx *c, const double *r, double *z, const double *scal) {
  MG &mg = *c->mg;
  MGLevel &L0 = mg.lev[0];
  double *b_own = L0.b;
  L0.b = const_cast<double *>(r);
  mg.tiles = c->cg.tiles;
  mg.ntiles = c->cg.ntiles;
  if (c->D == 2) vcycle<2>(mg, 0, c->st, scal, z);
  else vcycle<3>(mg, 0, c->st, scal, z);
  L0.b = b_own;
}

void batch_vcycle(int D, const BatchMG &bm, const Inst *insts, int ninst, hipStream_t st) {
  if (D == 2) batch_vcycle_t<2>(bm, insts, ninst, st);
  else batch_vcycle_t<3>(bm, insts, ninst, st);
}

void batch_mg_free(BatchMG &bm) {
  for (void *p : {(void *)bm.tab, (void *)bm.last}) (void)hipFree(p);
  for (int4 *p : bm.sm) (void)hipFree(p);
  for (int4 *p : bm.rs) (void)hipFree(p);
  bm = BatchMG();
}

}  // namespace tl
