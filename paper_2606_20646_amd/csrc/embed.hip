// Embedded-boundary kernels of the TL-VLBM update on gfx950:
//  - cut-link construction from level-set samples (Sec. 3.1),
//  - cut-link reconstruction, velocity Dirichlet and nominal-traction Neumann
//    (Secs. 3.2-3.4),
//  - compatibility projection by conjugate gradients (Sec. 3.5).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "tl_device.hpp"
#include "tl_internal.hpp"
#include "tl_math.hpp"

namespace tl {

#define HIP_OK(x)                                   \
  do {                                              \
    if ((x) != hipSuccess) return TLVLBM_ERR_DEVICE; \
  } while (0)

// ----------------------------------------------------------- active mask

template <int D>
__global__ void k_active(const double *__restrict__ phi, Geo g, uint8_t *__restrict__ act, int *flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  act[i] = phi[i] <= 0.0;
}

// every lattice neighbour of an active node must exist; count cut links per bid
template <int D>
__global__ void k_check_hist(Geo g, const uint8_t *__restrict__ act, const uint8_t *__restrict__ bid, int *flag,
                             unsigned *hist) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N || !act[i]) return;
  const C3 c = coords_of(g, i);
  for (int q = 0; q < 2 * D; ++q) {
    const int64_t o = node_dir(g, c, q, 1);
    if (o < 0) {
      atomicOr(flag, FLAG_ARG);
      return;
    }
    if (!act[o]) atomicAdd(&hist[bid ? bid[o] : 0], 1u);
  }
}

// number of cut links of node i whose outside node carries identifier b
template <int D>
__global__ void k_count(Geo g, const uint8_t *__restrict__ act, const uint8_t *__restrict__ bid, int b,
                        int *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int k = 0;
  if (act[i]) {
    const C3 c = coords_of(g, i);
    for (int q = 0; q < 2 * D; ++q) {
      const int64_t o = node_dir(g, c, q, 1);
      if (o >= 0 && !act[o] && (bid ? bid[o] : 0) == b) ++k;
    }
  }
  cnt[i] = k;
}

// ------------------------------------------------ exclusive prefix scan
// three phases: per-block totals, scan of totals (one block), local rescan

constexpr int SCAN_T = 256, SCAN_V = 8, SCAN_CH = SCAN_T * SCAN_V;

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t &total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int64_t a = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[SCAN_T - 1];
  int64_t ex = sh[t] - v;
  __syncthreads();
  return ex;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_tot(const int *__restrict__ cnt, int64_t n, int64_t *__restrict__ tot) {
  __shared__ int64_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH + threadIdx.x * SCAN_V;
  int64_t s = 0;
  for (int k = 0; k < SCAN_V; ++k)
    if (base + k < n) s += cnt[base + k];
  int64_t total;
  block_excl_scan(s, sh, total);
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_tot2(int64_t *__restrict__ tot, int64_t nb, int64_t *__restrict__ grand) {
  __shared__ int64_t sh[SCAN_T];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += SCAN_T) {
    const int64_t i = b0 + threadIdx.x;
    int64_t v = (i < nb) ? tot[i] : 0;
    int64_t total;
    int64_t ex = block_excl_scan(v, sh, total);
    if (i < nb) tot[i] = carry + ex;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int *__restrict__ cnt, int64_t n,
                                                       const int64_t *__restrict__ tot, int64_t *__restrict__ off) {
  __shared__ int64_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH + threadIdx.x * SCAN_V;
  int64_t s = 0;
  for (int k = 0; k < SCAN_V; ++k)
    if (base + k < n) s += cnt[base + k];
  int64_t total;
  int64_t ex = block_excl_scan(s, sh, total) + tot[blockIdx.x];
  for (int k = 0; k < SCAN_V; ++k)
    if (base + k < n) {
      off[base + k] = ex;
      ex += cnt[base + k];
    }
}

// compacted link records of identifier b, in (node, q) order
template <int D>
__global__ void k_scatter(Geo g, const uint8_t *__restrict__ act, const uint8_t *__restrict__ bid, int b,
                          const int *__restrict__ cnt, const int64_t *__restrict__ off, int64_t base, Links L) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N || cnt[i] == 0) return;
  const C3 c = coords_of(g, i);
  int64_t k = base + off[i];
  for (int q = 0; q < 2 * D; ++q) {
    const int64_t o = node_dir(g, c, q, 1);
    if (o >= 0 && !act[o] && (bid ? bid[o] : 0) == b) {
      L.node[k] = i;
      L.out[k] = o;
      L.q[k] = q;
      L.bid[k] = b;
      ++k;
    }
  }
}

// ---------------------------------------------- link geometry (FP64)

__device__ double phi_grad_axis(const Geo &g, const double *phi, C3 c, int64_t i, int A) {
  const int64_t ip = node_at(g, c, A == 0, A == 1, A == 2);
  const int64_t im = node_at(g, c, -(A == 0), -(A == 1), -(A == 2));
  if (ip >= 0 && im >= 0) return (phi[ip] - phi[im]) / (2.0 * g.dx);
  if (ip >= 0) return (phi[ip] - phi[i]) / g.dx;
  if (im >= 0) return (phi[i] - phi[im]) / g.dx;
  return 0.0;
}

// Cut fraction eta: bisection of the cubic interpolant of phi through the
// link parameters -1, 0, 1, 2 (linear when an outer sample is missing)
// (Sec. 3.1, Eq. 37) and the unit normal N_b from the level-set gradient
// (Eq. 38) of the link (m, q) with outside node o; mb = the node behind m
// (-1 if none).  Shared by the context's link tables and the allocation-free
// table of tlvlbm_cut_links_noalloc.
template <int D>
__device__ __forceinline__ double link_eta_normal(const Geo &g, const double *__restrict__ phi, int64_t m, int64_t o,
                                                  int q, int64_t mb, double *N) {
  const int A = q / 2, sg = (q & 1) ? -1 : 1;
  const C3 cm = coords_of(g, m), co = coords_of(g, o);
  const int64_t o2 = node_dir(g, co, q, 1);
  const double p0 = phi[m], p1 = phi[o];
  const bool cubic = (mb >= 0 && o2 >= 0);
  const double pm = cubic ? phi[mb] : 0.0, p2 = cubic ? phi[o2] : 0.0;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 80; ++it) {
    const double s = 0.5 * (lo + hi);
    double val;
    if (cubic) {
      // Lagrange basis on the nodes -1, 0, 1, 2
      const double lm = -s * (s - 1.0) * (s - 2.0) / 6.0;
      const double l0 = (s + 1.0) * (s - 1.0) * (s - 2.0) / 2.0;
      const double l1 = -(s + 1.0) * s * (s - 2.0) / 2.0;
      const double l2 = (s + 1.0) * s * (s - 1.0) / 6.0;
      val = pm * lm + p0 * l0 + p1 * l1 + p2 * l2;
    } else {
      val = p0 + s * (p1 - p0);
    }
    if (val <= 0.0) lo = s;
    else hi = s;
  }
  double eta = 0.5 * (lo + hi);
  eta = eta < 0.0 ? 0.0 : (eta > 1.0 ? 1.0 : eta);
  double nrm = 0.0;
  for (int a = 0; a < 3; ++a) N[a] = 0.0;
  for (int a = 0; a < D; ++a) {
    const double gm = phi_grad_axis(g, phi, cm, m, a), go = phi_grad_axis(g, phi, co, o, a);
    N[a] = (1.0 - eta) * gm + eta * go;
    nrm += N[a] * N[a];
  }
  nrm = sqrt(nrm);
  if (nrm > 0.0) {
    for (int a = 0; a < D; ++a) N[a] /= nrm;
  } else {
    for (int a = 0; a < D; ++a) N[a] = (a == A) ? sg : 0.0;
  }
  return eta;
}

// link geometry of the context's table: eta, N_b, X_b, the tangent frame and
// the upstream node m^- of the eta < 1/2 branch (Eq. 43)
template <int D>
__global__ void k_link_geom(Geo g, const double *__restrict__ phi, const uint8_t *__restrict__ act, Links L) {
  const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= L.n) return;
  const int64_t m = L.node[l], o = L.out[l];
  const int q = L.q[l], A = q / 2, sg = (q & 1) ? -1 : 1;
  const C3 cm = coords_of(g, m);
  const int64_t mb = node_dir(g, cm, q, -1);
  double N[3];
  const double eta = link_eta_normal<D>(g, phi, m, o, q, mb, N);
  L.eta[l] = eta;
  const double X[3] = {g.ox + (cm.x + 0.5) * g.dx, g.oy + (cm.y + 0.5) * g.dx, g.oz + (cm.z + 0.5) * g.dx};
  for (int a = 0; a < 3; ++a) {
    L.Nb[l * 3 + a] = N[a];
    L.Xb[l * 3 + a] = X[a] + ((a == A) ? sg * eta * g.dx : 0.0);
  }
  double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
  if (D == 2) {
    t1[0] = -N[1];
    t1[1] = N[0];
  } else {
    int k0 = 0;
    for (int a = 1; a < 3; ++a)
      if (fabs(N[a]) < fabs(N[k0])) k0 = a;
    const double dd = N[k0];
    double n1 = 0.0;
    for (int a = 0; a < 3; ++a) {
      t1[a] = ((a == k0) ? 1.0 : 0.0) - dd * N[a];
      n1 += t1[a] * t1[a];
    }
    n1 = sqrt(n1);
    for (int a = 0; a < 3; ++a) t1[a] /= n1;
    t2[0] = N[1] * t1[2] - N[2] * t1[1];
    t2[1] = N[2] * t1[0] - N[0] * t1[2];
    t2[2] = N[0] * t1[1] - N[1] * t1[0];
  }
  for (int a = 0; a < 3; ++a) {
    L.tang[l * 6 + a] = t1[a];
    L.tang[l * 6 + 3 + a] = t2[a];
  }
  L.mminus[l] = (mb >= 0 && act[mb]) ? mb : m;
}

// quadratic (or linear) LSQ basis row in normalised coordinates (Eq. 50)
template <int D> __device__ __forceinline__ int lsq_row(const double *xi, bool quad, double *a) {
  int k = 0;
  a[k++] = 1.0;
  for (int d = 0; d < D; ++d) a[k++] = xi[d];
  if (quad) {
    if (D == 2) {
      a[k++] = 0.5 * xi[0] * xi[0];
      a[k++] = xi[0] * xi[1];
      a[k++] = 0.5 * xi[1] * xi[1];
    } else {
      a[k++] = 0.5 * xi[0] * xi[0];
      a[k++] = 0.5 * xi[1] * xi[1];
      a[k++] = 0.5 * xi[2] * xi[2];
      a[k++] = xi[0] * xi[1];
      a[k++] = xi[0] * xi[2];
      a[k++] = xi[1] * xi[2];
    }
  }
  return k;
}

// Static weighted-LSQ tangent-derivative weights per link (Eqs. 49-52):
// stencil = active nodes within 2.5 dx of X_b, weights 1/(1 + |xi|^2),
// quadratic basis, linear fallback when there are fewer than twice as many
// points as terms or a Jacobi-scaled Cholesky pivot drops below 1e-10.
template <int D>
__global__ void k_link_lsq(Geo g, const uint8_t *__restrict__ act, Links L, int *flag) {
  const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= L.n) return;
  const int64_t m = L.node[l];
  const int q = L.q[l], A = q / 2, sg = (q & 1) ? -1 : 1;
  const double eta = L.eta[l];
  const C3 cm = coords_of(g, m);
  int np = 0;
  const int R = 4;
  for (int oz = (D == 3 ? -R : 0); oz <= (D == 3 ? R : 0); ++oz)
    for (int oy = -R; oy <= R; ++oy)
      for (int ox = -R; ox <= R; ++ox) {
        const int o[3] = {ox, oy, oz};
        double r2 = 0.0;
        for (int a = 0; a < D; ++a) {
          const double xr = o[a] - ((a == A) ? sg * eta : 0.0);
          r2 += xr * xr;
        }
        if (r2 > LSQ_RADIUS * LSQ_RADIUS) continue;
        const int64_t j = node_at(g, cm, ox, oy, oz);
        if (j < 0 || !act[j]) continue;
        if (np >= L.kmax) {
          atomicOr(flag, FLAG_STENCIL);
          L.npts[l] = 0;
          L.basis[l] = 0;
          return;
        }
        L.sidx[lsq_i(L, l, np)] = (int32_t)j;
        ++np;
      }
  L.npts[l] = np;
  // normalised coordinates of the stencil, in stencil order
  double xs[KMAX3 * 3];
  {
    int cnt = 0;
    for (int oz = (D == 3 ? -R : 0); oz <= (D == 3 ? R : 0); ++oz)
      for (int oy = -R; oy <= R; ++oy)
        for (int ox = -R; ox <= R; ++ox) {
          const int o[3] = {ox, oy, oz};
          double r2 = 0.0, xr[3];
          for (int a = 0; a < D; ++a) {
            xr[a] = o[a] - ((a == A) ? sg * eta : 0.0);
            r2 += xr[a] * xr[a];
          }
          if (r2 > LSQ_RADIUS * LSQ_RADIUS) continue;
          const int64_t j = node_at(g, cm, ox, oy, oz);
          if (j < 0 || !act[j]) continue;
          for (int a = 0; a < D; ++a) xs[cnt * D + a] = xr[a];
          ++cnt;
        }
  }
  const double *tg = L.tang + l * 6;
  for (int quad = 1; quad >= 0; --quad) {
    const int nb = quad ? (D == 2 ? 6 : 10) : D + 1;
    if (np < (quad ? 2 * nb : nb)) continue;
    double Nm[100];
    for (int k = 0; k < nb * nb; ++k) Nm[k] = 0.0;
    for (int k = 0; k < np; ++k) {
      double a[10], r2 = 0.0;
      lsq_row<D>(xs + k * D, quad, a);
      for (int d = 0; d < D; ++d) r2 += xs[k * D + d] * xs[k * D + d];
      const double W = 1.0 / (1.0 + r2);
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) Nm[i * nb + j] += a[i] * W * a[j];
    }
    // Jacobi-scaled Cholesky pivot test
    double Ls[100], sc[10];
    for (int i = 0; i < nb; ++i) sc[i] = 1.0 / sqrt(Nm[i * nb + i]);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) Ls[i * nb + j] = Nm[i * nb + j] * sc[i] * sc[j];
    bool ok = true;
    for (int k = 0; k < nb && ok; ++k) {
      double d = Ls[k * nb + k];
      for (int p = 0; p < k; ++p) d -= Ls[k * nb + p] * Ls[k * nb + p];
      if (!(d >= 1e-10)) {
        ok = false;
        break;
      }
      Ls[k * nb + k] = sqrt(d);
      for (int i = k + 1; i < nb; ++i) {
        double s = Ls[i * nb + k];
        for (int p = 0; p < k; ++p) s -= Ls[i * nb + p] * Ls[k * nb + p];
        Ls[i * nb + k] = s / Ls[k * nb + k];
      }
    }
    if (!ok) continue;
    // z = Nm^{-1} e_t through the scaled factor: Nm = S^-1 Ls Ls^T S^-1
    for (int al = 0; al < D - 1; ++al) {
      double y[10], z[10];
      for (int i = 0; i < nb; ++i) y[i] = 0.0;
      for (int d = 0; d < D; ++d) y[1 + d] = tg[al * 3 + d] / g.dx;
      for (int i = 0; i < nb; ++i) y[i] *= sc[i];
      for (int i = 0; i < nb; ++i) {  // forward
        double s = y[i];
        for (int p = 0; p < i; ++p) s -= Ls[i * nb + p] * z[p];
        z[i] = s / Ls[i * nb + i];
      }
      for (int i = nb - 1; i >= 0; --i) {  // backward
        double s = z[i];
        for (int p = i + 1; p < nb; ++p) s -= Ls[p * nb + i] * y[p];
        y[i] = s / Ls[i * nb + i];
      }
      for (int i = 0; i < nb; ++i) y[i] *= sc[i];
      for (int k = 0; k < np; ++k) {
        double a[10], r2 = 0.0, s = 0.0;
        lsq_row<D>(xs + k * D, quad, a);
        for (int d = 0; d < D; ++d) r2 += xs[k * D + d] * xs[k * D + d];
        for (int j = 0; j < nb; ++j) s += a[j] * y[j];
        L.sw[lsq_w(L, l, al, k)] = s / (1.0 + r2);
      }
    }
    L.basis[l] = quad ? 2 : 1;
    return;
  }
  L.basis[l] = 0;
  for (int al = 0; al < D - 1; ++al)
    for (int k = 0; k < np; ++k) L.sw[lsq_w(L, l, al, k)] = 0.0;
}

// ----------------------------------------------------- cut-link closure

// The populations a closure reads, all loaded before any write: f*_out(m)
// and, for eta >= 1/2, f*_in(m), else f*_out(m^-).  The closure writes only
// the pull slot of the outside node, which no link reads, so the loads can
// all be in flight together (interleaved with the writes through the same
// pointer they would be issued one row at a time).
template <int D, typename T>
__device__ __forceinline__ void closure_reads(const T *__restrict__ f, const Geo &g, int64_t m, int64_t mm, int qo,
                                              double eta, T (&fo)[D + D * D], T (&fx)[D + D * D]) {
  constexpr int M = D + D * D;
  const int qi = qo ^ 1;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    fo[r] = f[(size_t)(qo * M + r) * g.S + m];
    fx[r] = (eta >= 0.5) ? f[(size_t)(qi * M + r) * g.S + m] : f[(size_t)(qo * M + r) * g.S + mm];
  }
}

// Velocity Dirichlet (Sec. 3.3, Eqs. 44-45) with cut-link interpolation
// (Sec. 3.2, Eqs. 42-43).  f holds post-collision populations (shifted); the
// reconstructed incoming population is written to the pull slot of the
// outside node.  One thread per link.
template <int D, typename T>
__device__ __forceinline__ void cut_dirichlet_link(T *__restrict__ f, const Links &L, int64_t l, const BC &bc,
                                                   const Geo &g, const Par &p, double th) {
  constexpr int M = D + D * D;
  const int64_t m = L.node[l], mm = L.mminus[l], o = L.out[l];
  const int qo = L.q[l], qi = qo ^ 1, A = qo / 2;
  const double sg = (qo & 1) ? -1.0 : 1.0;
  const double eta = L.eta[l];
  double Xb[3], N[3], vb[3];
  for (int a = 0; a < 3; ++a) {
    Xb[a] = L.Xb[l * 3 + a];
    N[a] = L.Nb[l * 3 + a];
  }
  double s, ds;
  ramp_eval(bc.ramp, bc.Tr, th, s, ds);
  bc_base<D>(bc, Xb, N, vb);
  const double fac = bc.disp ? ds : s;
  for (int i = 0; i < D; ++i) vb[i] *= fac;
  twist_add(bc, Xb, s, ds, true, vb);
  const T ie = T(1.0 / (2.0 * eta));
  const T e2 = T(2.0 * eta);
  T fo[M], fx[M];
  closure_reads<D, T>(f, g, m, mm, qo, eta, fo, fx);
#pragma unroll
  for (int r = 0; r < M; ++r) {
    T Dg, S;
    if (r < D) {
      Dg = T(-1);
      S = T(vb[r] / D);
    } else {
      const int i = (r - D) / D, B = (r - D) % D;
      Dg = T(1);
      // -d_B v_i / c with d = -e_{q_out}; the shifts of q_out and q_in cancel
      // in both row kinds (Dg = -1 on velocity rows, whose shift is odd in q)
      S = (B == A) ? T(sg * vb[i] / p.c) : T(0);
    }
    T out;
    if (eta >= 0.5) out = (Dg * fo[r] + S) * ie + (T(1) - ie) * fx[r];
    else out = Dg * (e2 * fo[r] + (T(1) - e2) * fx[r]) + S;
    f[(size_t)(qi * M + r) * g.S + o] = out;
  }
}

// Nominal-traction Neumann (Sec. 3.4, Eqs. 46-56) with cut-link
// interpolation.  Tangent images from the static LSQ weights applied to the
// displacement u (Eqs. 48-52); normal image by the local Newton; the
// boundary state enters the deformation-gradient rows, the Piola flux the
// velocity rows.
template <int D, typename T>
__device__ __forceinline__ void cut_neumann_link(T *__restrict__ f, const Links &L, int64_t l, const BC &bc,
                                                 const Geo &g, const Par &p, double th, const double *__restrict__ u,
                                                 int *__restrict__ flag, unsigned long long *__restrict__ nfail) {
  constexpr int Q = 2 * D, M = D + D * D;
  const int64_t m = L.node[l], mm = L.mminus[l], o = L.out[l];
  const int qo = L.q[l], qi = qo ^ 1, A = qo / 2;
  const double sg = (qo & 1) ? -1.0 : 1.0;
  const double eta = L.eta[l];
  double Xb[3], N[3], Tb[3];
  for (int a = 0; a < 3; ++a) {
    Xb[a] = L.Xb[l * 3 + a];
    N[a] = L.Nb[l * 3 + a];
  }
  // sum_alpha g_alpha (x) t_alpha with g_alpha = t_alpha + sum_k w_alpha,k u_k
  // (one pass over the stencil for both tangents)
  double Gt[D * D];
  for (int k = 0; k < D * D; ++k) Gt[k] = 0.0;
  const int np = L.npts[l];
  double gv[D - 1][D];
  for (int al = 0; al < D - 1; ++al)
    for (int i = 0; i < D; ++i) gv[al][i] = L.tang[l * 6 + al * 3 + i];
  lsq_gather<D>(
      L, l, np, [&](int k) { return (int64_t)L.sidx[lsq_i(L, l, k)]; },
      [&](int64_t j, int i) { return u[(size_t)i * g.S + j]; }, gv);
  for (int al = 0; al < D - 1; ++al)
    for (int i = 0; i < D; ++i)
      for (int B = 0; B < D; ++B) Gt[i * D + B] += gv[al][i] * L.tang[l * 6 + al * 3 + B];
  double s, ds;
  ramp_eval(bc.ramp, bc.Tr, th, s, ds);
  bc_base<D>(bc, Xb, N, Tb);
  for (int i = 0; i < D; ++i) Tb[i] *= s;
  // initial guess h0 = F_m N with F_m = sum_q f*_q^F(m) (collision keeps the
  // F moment since the source has no F rows; stored about Fref)
  double h[D];
  {
    double Fm[D * D];
    for (int k = 0; k < D * D; ++k) {
      double acc = p.Fref[k];
      for (int qq = 0; qq < Q; ++qq) acc += double(f[(size_t)(qq * M + D + k) * g.S + m]);
      Fm[k] = acc;
    }
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int B = 0; B < D; ++B) acc += Fm[i * D + B] * N[B];
      h[i] = acc;
    }
  }
  // the law of node m (with a Maxwell branch: its history after this step's
  // collision)
  double Hn[sym_n<D>()];
  const double *hn = law_load<D>(p, m, g.S, Hn) ? Hn : nullptr;
  const double ths = law_theta<D>(p, m);  // the node's thermal stretch
  const bool conv = newton_h<D>(N, Gt, Tb, p, 1e-12, h, hn, ths);
  if (!conv) atomicAdd(nfail, 1ull);
  double Fb[D * D], Pb[D * D];
  for (int i = 0; i < D; ++i)
    for (int a = 0; a < D; ++a) Fb[i * D + a] = h[i] * N[a] + Gt[i * D + a];
  if (!(det<D>(Fb) > 0.0)) {
    atomicOr(flag, FLAG_NEWTON);
    for (int k = 0; k < D * D; ++k) Fb[k] = (k % (D + 1) == 0) ? 1.0 : 0.0;
  }
  law_piola<D>(Fb, p, hn, Pb, ths);
  const T ie = T(1.0 / (2.0 * eta));
  const T e2 = T(2.0 * eta);
  T fo[M], fx[M];
  closure_reads<D, T>(f, g, m, mm, qo, eta, fo, fx);
#pragma unroll
  for (int r = 0; r < M; ++r) {
    T Dg, S;
    // sources in the stored variables g = f - feq(0, Fref): the closure
    // g_in = Dg g_out + S holds with S = S_f + Dg g_shift(q_out) - g_shift(q_in)
    if (r < D) {
      Dg = T(1);
      // -d_A P_b,iA / (rho0 c), d = -e_{q_out}, plus twice the shift of q_out
      S = T(sg * (Pb[r * D + A] * p.inv_rho0 - p.Pref[r * D + A]) / p.c);
    } else {
      const int k = r - D;
      Dg = T(-1);
      // F_b/D less twice the shift Fref/(2D)
      S = T((Fb[k] - p.Fref[k]) / D);
    }
    T out;
    if (eta >= 0.5) out = (Dg * fo[r] + S) * ie + (T(1) - ie) * fx[r];
    else out = Dg * (e2 * fo[r] + (T(1) - e2) * fx[r]) + S;
    f[(size_t)(qi * M + r) * g.S + o] = out;
  }
}

// --------------------------------------------------------- projection

// anchors of the projection null mode: each Dirichlet cut link adds
// u_m = u_D(X_b, t) - (F_m - I)(X_b - X_m) with unit weight
template <int D, typename T>
__device__ __forceinline__ void anchor_link(const Links &L, int64_t l, const BC &bc, const Geo &g, double t,
                                            const T *__restrict__ Fm, int *__restrict__ anc_n,
                                            double *__restrict__ anc_s) {
  const int64_t m = L.node[l];
  const int q = L.q[l], A = q / 2;
  const double sg = (q & 1) ? -1.0 : 1.0;
  double Xb[3], N[3], uD[3];
  for (int a = 0; a < 3; ++a) {
    Xb[a] = L.Xb[l * 3 + a];
    N[a] = L.Nb[l * 3 + a];
  }
  double s, ds;
  ramp_eval(bc.ramp, bc.Tr, t, s, ds);
  bc_base<D>(bc, Xb, N, uD);
  const double fac = bc.disp ? s : ramp_int(bc.ramp, bc.Tr, t);
  for (int i = 0; i < D; ++i) uD[i] *= fac;
  twist_add(bc, Xb, s, ds, false, uD);
  const double off = sg * L.eta[l] * g.dx;
  atomicAdd(&anc_n[m], 1);
  for (int i = 0; i < D; ++i) {
    const double Fi = double(Fm[(size_t)(i * D + A) * g.S + m]);  // F - I
    atomicAdd(&anc_s[(size_t)i * g.S + m], uD[i] - Fi * off);
  }
}

// right-hand side of the normal equations of the edge least-squares problem
// (Eq. 57) plus the anchor targets
template <int D, typename T>
__device__ __forceinline__ void cg_rhs_node(const Geo &g, const uint8_t *__restrict__ act, const T *__restrict__ Fm,
                                            const double *__restrict__ anc_s, double *__restrict__ b, int64_t i) {
  if (i >= g.N) return;
  if (!act[i]) {
    for (int c = 0; c < D; ++c) b[(size_t)c * g.S + i] = double(0);
    return;
  }
  const C3 cc = coords_of(g, i);
  const double hdx = double(0.5 * g.dx);
  for (int c = 0; c < D; ++c) {
    double acc = anc_s ? anc_s[(size_t)c * g.S + i] : double(0);
    for (int A = 0; A < D; ++A) {
      const int64_t lp = node_dir(g, cc, 2 * A, 1), lm = node_dir(g, cc, 2 * A + 1, 1);
      const double Fi = Fm[(size_t)(c * D + A) * g.S + i];
      if (lm >= 0 && act[lm]) acc += hdx * (Fi + Fm[(size_t)(c * D + A) * g.S + lm]);
      if (lp >= 0 && act[lp]) acc -= hdx * (Fi + Fm[(size_t)(c * D + A) * g.S + lp]);
    }
    b[(size_t)c * g.S + i] = acc;
  }
}

// the same right-hand side on an active node from its neighbour mask (bit q:
// X + e_q active, bit 6: X active), every load issued before any use; a
// missing neighbour reads the node itself and contributes an exact zero
template <int D, typename T>
__device__ __forceinline__ void cg_rhs_node_m(const Geo &g, const uint8_t *__restrict__ nbm,
                                              const T *__restrict__ Fm, const double *__restrict__ anc_s,
                                              double *__restrict__ b, int64_t i) {
  if (i >= g.N) return;
  const unsigned m = nbm[i];
  if (!(m & 64u)) return;
  int64_t lp[D], lm[D];
#pragma unroll
  for (int A = 0; A < D; ++A) {
    lp[A] = ((m >> (2 * A)) & 1u) ? nb_index(g, i, 2 * A) : i;
    lm[A] = ((m >> (2 * A + 1)) & 1u) ? nb_index(g, i, 2 * A + 1) : i;
  }
  double Fi[D * D], Fp[D * D], Fn[D * D], as[D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    const int A = k % D;
    Fi[k] = double(Fm[(size_t)k * g.S + i]);
    Fp[k] = double(Fm[(size_t)k * g.S + lp[A]]);
    Fn[k] = double(Fm[(size_t)k * g.S + lm[A]]);
  }
#pragma unroll
  for (int c = 0; c < D; ++c) as[c] = anc_s ? anc_s[(size_t)c * g.S + i] : 0.0;
  const double hdx = double(0.5 * g.dx);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double acc = as[c];
#pragma unroll
    for (int A = 0; A < D; ++A) {
      const int k = c * D + A;
      acc += ((m >> (2 * A + 1)) & 1u) ? hdx * (Fi[k] + Fn[k]) : 0.0;
      acc -= ((m >> (2 * A)) & 1u) ? hdx * (Fi[k] + Fp[k]) : 0.0;
    }
    b[(size_t)c * g.S + i] = acc;
  }
}

// block partials: up to PSTRIDE doubles per block
constexpr int PSTRIDE = 16;

constexpr int CG_T = 256;

// Reductions: every block writes its partial sums to partial[blk*PSTRIDE + k]
// (no fence, no atomic); a one-block finalize kernel launched next sums the
// partials in a fixed order (deterministic) and updates the CG scalars.  A
// device-scope release fence per block would write back the whole L2 of its
// XCD, which made each reduction cost far more than the sweep it ends.
template <int K>
__device__ __forceinline__ void block_store(double (&v)[K], double *partial, int blk) {
  __shared__ double sh[CG_T / 64][PSTRIDE];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sh[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < CG_T / 64; ++w) s += sh[w][threadIdx.x];
    partial[blk * PSTRIDE + threadIdx.x] = s;
  }
}

// totals of the K partial sums over nblk blocks (one block of FIN_T threads)
constexpr int FIN_T = 1024;
template <int K>
__device__ __forceinline__ void block_totals(const double *partial, int nblk, double *tot) {
  __shared__ double sh[FIN_T / 64][PSTRIDE];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += FIN_T)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += partial[b * PSTRIDE + k];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = acc[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sh[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
      for (int w = 0; w < FIN_T / 64; ++w) t += sh[w][k];
      tot[k] = t;
    }
}

// r = b - A x, p = r, rr and bb (A = active-graph Laplacian + anchors)
template <int D, typename T>
__device__ __forceinline__ void cg_init_blk(const Geo &g, const uint8_t *__restrict__ act,
                                            const uint8_t *__restrict__ anc_n, const double *__restrict__ b,
                                            const double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
                                            double *partial, int blk, int slot) {
  const int64_t i = blk * (int64_t)CG_T + threadIdx.x;
  double v[2 * D];
  for (int k = 0; k < 2 * D; ++k) v[k] = 0.0;
  if (i < g.N) {
    if (act[i]) {
      const C3 cc = coords_of(g, i);
      int64_t nb[2 * D];
      int deg = anc_n ? anc_n[i] : 0;
      for (int q = 0; q < 2 * D; ++q) {
        nb[q] = node_dir(g, cc, q, 1);
        if (nb[q] >= 0 && !act[nb[q]]) nb[q] = -1;
        if (nb[q] >= 0) ++deg;
      }
      for (int c = 0; c < D; ++c) {
        double ax = double(deg) * x[(size_t)c * g.S + i];
        for (int q = 0; q < 2 * D; ++q)
          if (nb[q] >= 0) ax -= x[(size_t)c * g.S + nb[q]];
        const double bi = b[(size_t)c * g.S + i];
        const double ri = bi - ax;
        r[(size_t)c * g.S + i] = ri;
        p[(size_t)c * g.S + i] = ri;
        v[c] = double(ri) * double(ri);
        v[D + c] = double(bi) * double(bi);
      }
    } else {
      for (int c = 0; c < D; ++c) {
        r[(size_t)c * g.S + i] = double(0);
        p[(size_t)c * g.S + i] = double(0);
      }
    }
  }
  block_store<2 * D>(v, partial, slot);
}

template <int D> __device__ __forceinline__ void cg_init_fin(const double *tot, double *scal, double rtol) {
  {
    bool all = true;
    for (int c = 0; c < D; ++c) {
      const double rr = tot[c], bb = tot[D + c];
      scal[S_RR + c] = rr;
      scal[S_BB + c] = bb;
      scal[S_THR + c] = rtol * rtol * (bb > rr ? bb : rr);
      scal[S_BETA + c] = 0.0;
      scal[S_ITS + c] = 0.0;
      const bool act_c = rr > scal[S_THR + c];
      scal[S_ACT + c] = act_c ? 1.0 : 0.0;
      all = all && !act_c;
    }
    scal[S_DONE] = all ? 1.0 : 0.0;
  }
}

// p_new = r + beta p_old (recomputed at neighbours), Ap = A p_new, p.Ap
template <int D, typename T>
__device__ __forceinline__ void cg_Ap_blk(const Geo &g, const uint8_t *__restrict__ act,
                                          const uint8_t *__restrict__ anc_n, const double *__restrict__ r,
                                          const double *__restrict__ pold, double *__restrict__ pnew, double *__restrict__ Ap,
                                          double *partial, const double *scal, int blk, int slot) {
  if (scal[S_DONE] != 0.0) return;
  const int64_t i = blk * (int64_t)CG_T + threadIdx.x;
  double v[D];
  for (int k = 0; k < D; ++k) v[k] = 0.0;
  double beta[D];
  for (int c = 0; c < D; ++c) beta[c] = double(scal[S_BETA + c]);
  if (i < g.N && act[i]) {
    const C3 cc = coords_of(g, i);
    int64_t nb[2 * D];
    int deg = anc_n ? anc_n[i] : 0;
    for (int q = 0; q < 2 * D; ++q) {
      nb[q] = node_dir(g, cc, q, 1);
      if (nb[q] >= 0 && !act[nb[q]]) nb[q] = -1;
      if (nb[q] >= 0) ++deg;
    }
    for (int c = 0; c < D; ++c) {
      const size_t o = (size_t)c * g.S;
      const double pi = r[o + i] + beta[c] * pold[o + i];
      double ap = double(deg) * pi;
      for (int q = 0; q < 2 * D; ++q)
        if (nb[q] >= 0) ap -= r[o + nb[q]] + beta[c] * pold[o + nb[q]];
      pnew[o + i] = pi;
      Ap[o + i] = ap;
      v[c] = double(pi) * double(ap);
    }
  } else if (i < g.N) {
    for (int c = 0; c < D; ++c) {
      pnew[(size_t)c * g.S + i] = double(0);
      Ap[(size_t)c * g.S + i] = double(0);
    }
  }
  block_store<D>(v, partial, slot);
}

template <int D> __device__ __forceinline__ void cg_Ap_fin(const double *tot, double *scal, bool pc) {
  {
    for (int c = 0; c < D; ++c) {
      const bool on = scal[S_ACT + c] != 0.0 && tot[c] > 0.0;
      scal[S_ALPHA + c] = on ? scal[(pc ? S_RZ : S_RR) + c] / tot[c] : 0.0;
      if (!on) scal[S_ACT + c] = 0.0;
    }
  }
}

// x += alpha p, r -= alpha Ap, rr_new, beta, convergence
template <int D, typename T>
__device__ __forceinline__ void cg_update_blk(const Geo &g, const uint8_t *__restrict__ act, double *__restrict__ x,
                                              double *__restrict__ r, const double *__restrict__ p, const double *__restrict__ Ap,
                                              double *partial, const double *scal, int blk, int slot) {
  if (scal[S_DONE] != 0.0) return;
  const int64_t i = blk * (int64_t)CG_T + threadIdx.x;
  double v[D];
  for (int k = 0; k < D; ++k) v[k] = 0.0;
  if (i < g.N && act[i]) {
    for (int c = 0; c < D; ++c) {
      const size_t o = (size_t)c * g.S;
      const double al = double(scal[S_ALPHA + c]);
      x[o + i] += al * p[o + i];
      const double ri = r[o + i] - al * Ap[o + i];
      r[o + i] = ri;
      v[c] = double(ri) * double(ri);
    }
  }
  block_store<D>(v, partial, slot);
}

template <int D> __device__ __forceinline__ void cg_update_fin(const double *tot, double *scal, bool pc) {
  {
    bool all = true;
    for (int c = 0; c < D; ++c) {
      if (scal[S_ACT + c] != 0.0) {
        scal[S_ITS + c] += 1.0;
        const double rr2 = tot[c];
        if (!pc) scal[S_BETA + c] = rr2 / scal[S_RR + c];
        scal[S_RR + c] = rr2;
        if (!(rr2 > scal[S_THR + c])) scal[S_ACT + c] = 0.0;
      } else {
        scal[S_BETA + c] = 0.0;
      }
      all = all && (scal[S_ACT + c] == 0.0);
    }
    scal[S_DONE] = all ? 1.0 : 0.0;
  }
}

// one damped Jacobi sweep of the projection's normal equations (Sec. 3.5):
// xout = xin + om (b - K xin) / diag(K), K = active-graph Laplacian plus the
// anchor counts.  Inactive nodes and nodes with a zero diagonal (no active
// neighbour, no anchor: no edge relation) copy xin.
template <int D>
__device__ __forceinline__ void jacobi_node(const Geo &g, const uint8_t *__restrict__ act,
                                            const uint8_t *__restrict__ anc_n, const double *__restrict__ b,
                                            const double *__restrict__ xin, double *__restrict__ xout, double om,
                                            int64_t i) {
  if (i >= g.N) return;
  int deg = 0;
  int64_t nb[2 * D];
  if (act[i]) {
    const C3 cc = coords_of(g, i);
    deg = anc_n ? anc_n[i] : 0;
    for (int q = 0; q < 2 * D; ++q) {
      nb[q] = node_dir(g, cc, q, 1);
      if (nb[q] >= 0 && !act[nb[q]]) nb[q] = -1;
      if (nb[q] >= 0) ++deg;
    }
  }
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S;
    const double xi = xin[o + i];
    if (deg == 0) {
      xout[o + i] = xi;
      continue;
    }
    double kx = double(deg) * xi;
    for (int q = 0; q < 2 * D; ++q)
      if (nb[q] >= 0) kx -= xin[o + nb[q]];
    xout[o + i] = xi + om * (b[o + i] - kx) / double(deg);
  }
}

// one component of one node's damped Jacobi update: node value xi,
// right-hand side bi, neighbour values xn[q] (used where bit q of the mask m
// says X + e_q is active), diagonal deg > 0
template <int D>
__device__ __forceinline__ double jacobi_upd(double xi, double bi, const double *xn, unsigned m, int deg, double om) {
  double kx = double(deg) * xi;
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) kx -= ((m >> q) & 1u) ? xn[q] : 0.0;
  return xi + om * (bi - kx) / double(deg);
}

// the same sweep from the precomputed neighbour mask (bit q: X + e_q active,
// bit 6: X active); the same operations in the same order
template <int D>
__device__ __forceinline__ void jacobi_node_m(const Geo &g, const uint8_t *__restrict__ nbm,
                                              const uint8_t *__restrict__ anc_n, const double *__restrict__ b,
                                              const double *__restrict__ xin, double *__restrict__ xout, double om,
                                              int64_t i) {
  if (i >= g.N) return;
  const unsigned m = nbm[i];
  // an inactive node has no edges: no active node reads it, and neither
  // buffer's value there is used, so it is skipped (the copies of the
  // result skip it too)
  if (!(m & 64u)) return;
  int64_t nb[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) nb[q] = -1;
  const int deg = (anc_n ? anc_n[i] : 0) + __builtin_popcount(m & ((1u << (2 * D)) - 1u));
#pragma unroll
  for (int q = 0; q < 2 * D; ++q)
    if ((m >> q) & 1u) nb[q] = nb_index(g, i, q);
  // every load unconditional (a missing neighbour reads the node itself and
  // contributes an exact zero), so that all of them are in flight together
  int64_t at[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) at[q] = nb[q] >= 0 ? nb[q] : i;
  double xi[D], bi[D], xn[D][2 * D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S;
    xi[c] = xin[o + i];
    bi[c] = b[o + i];
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) xn[c][q] = xin[o + at[q]];
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S;
    xout[o + i] = deg == 0 ? xi[c] : jacobi_upd<D>(xi[c], bi[c], xn[c], m, deg, om);
  }
}

// JT_NS or fewer damped Jacobi sweeps of a 2D grid fused in LDS.  The tile
// (tx, ty) of JT x JT nodes and a halo of ns nodes (wrapped on periodic
// axes) are staged once; sweep s updates the active nodes at least s nodes
// inside the staged square, whose four neighbours then hold the values of
// sweep s - 1, so after ns sweeps the tile holds exactly what ns separate
// sweeps give, and only the tile is written.  Every update is jacobi_upd,
// as in jacobi_node_m.  Staged nodes outside a non-periodic grid, and
// inactive ones, are never read: no mask bit points at them.
constexpr int JT_W = JT + 2 * JT_NS;
constexpr int JT_OWN = (JT_W * JT_W + CG_T - 1) / CG_T;  // staged nodes per thread
static_assert(JT_NS >= 1 && JT_W < 256 && JT_W * JT_W * 16 <= 65536,
              "fused sweeps: 1 <= JT_NS, the staged square within the LDS of one workgroup");
__device__ __forceinline__ void jacobi_tile2(const Geo &g, const uint8_t *__restrict__ nbm,
                                             const uint8_t *__restrict__ anc_n, const double *__restrict__ b,
                                             const double *__restrict__ xin, double *__restrict__ xout, double om,
                                             int tx, int ty, int ns, double2 *sx) {
  const int W = JT + 2 * ns, R = W * W;
  const int gx0 = tx * JT - ns, gy0 = ty * JT - ns;
  const size_t S = (size_t)g.S;
  int pos[JT_OWN];       // lx | ly << 8 of the staged node, -1: none
  unsigned md[JT_OWN];   // neighbour mask | diagonal << 8 (0: inactive)
  int64_t gi[JT_OWN];    // its node (0 where it has none)
  double b0[JT_OWN], b1[JT_OWN], n0[JT_OWN], n1[JT_OWN];
  bool in[JT_OWN];
#pragma unroll
  for (int j = 0; j < JT_OWN; ++j) {
    const int r = (int)threadIdx.x + j * CG_T;
    const int lx = r % W, ly = r / W;
    pos[j] = r < R ? lx | (ly << 8) : -1;
    int gx = gx0 + lx, gy = gy0 + ly;
    in[j] = r < R;
    if (gx < 0 || gx >= g.nx) {
      if (g.per & 1) gx = ((gx % g.nx) + g.nx) % g.nx;
      else in[j] = false;
    }
    if (gy < 0 || gy >= g.ny) {
      if (g.per & 2) gy = ((gy % g.ny) + g.ny) % g.ny;
      else in[j] = false;
    }
    gi[j] = in[j] ? gx + (int64_t)g.nx * gy : 0;
  }
  // every load issued before any is used (node 0 stands in where a staged
  // position has no node), so that all of them are in flight together
  unsigned mm[JT_OWN], an[JT_OWN];
  double x0[JT_OWN], x1[JT_OWN];
#pragma unroll
  for (int j = 0; j < JT_OWN; ++j) {
    mm[j] = nbm[gi[j]];
    an[j] = anc_n ? anc_n[gi[j]] : 0u;
    b0[j] = b[gi[j]];
    b1[j] = b[S + gi[j]];
    x0[j] = xin[gi[j]];
    x1[j] = xin[S + gi[j]];
  }
#pragma unroll
  for (int j = 0; j < JT_OWN; ++j) {
    const bool a = in[j] && (mm[j] & 64u);
    md[j] = a ? (mm[j] | ((an[j] + (unsigned)__builtin_popcount(mm[j] & 15u)) << 8)) : 0u;
    if (pos[j] >= 0) sx[(int)threadIdx.x + j * CG_T] = a ? make_double2(x0[j], x1[j]) : make_double2(0.0, 0.0);
    n0[j] = n1[j] = 0.0;
  }
  __syncthreads();
  for (int s = 1; s <= ns; ++s) {
    bool up[JT_OWN];
#pragma unroll
    for (int j = 0; j < JT_OWN; ++j) {
      const int r = (int)threadIdx.x + j * CG_T;
      const int lx = pos[j] & 255, ly = pos[j] >> 8;
      const int deg = (int)(md[j] >> 8);
      up[j] = pos[j] >= 0 && deg > 0 && lx >= s && lx < W - s && ly >= s && ly < W - s;
      // no branch around the reads: a position that is not updated reads
      // an interior one instead (its result is dropped)
      const int rc = up[j] ? r : W + 1;
      const double2 c0 = sx[rc], e = sx[rc + 1], w = sx[rc - 1], n = sx[rc + W], o = sx[rc - W];
      const double xa[4] = {e.x, w.x, n.x, o.x}, xb[4] = {e.y, w.y, n.y, o.y};
      const unsigned m = md[j] & 255u;
      const int dg = up[j] ? deg : 1;
      n0[j] = jacobi_upd<2>(c0.x, b0[j], xa, m, dg, om);
      n1[j] = jacobi_upd<2>(c0.y, b1[j], xb, m, dg, om);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < JT_OWN; ++j)
      if (up[j]) sx[(int)threadIdx.x + j * CG_T] = make_double2(n0[j], n1[j]);
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < JT_OWN; ++j) {
    const int lx = pos[j] & 255, ly = pos[j] >> 8;
    if (pos[j] < 0 || !(md[j] & 64u) || lx < ns || lx >= ns + JT || ly < ns || ly >= ns + JT) continue;
    // the tile proper: no wrap (a last tile's columns or rows past the grid
    // are wrapped copies and are not written)
    if (tx * JT + lx - ns >= g.nx || ty * JT + ly - ns >= g.ny) continue;
    const double2 v = sx[(int)threadIdx.x + j * CG_T];
    xout[gi[j]] = v.x;
    xout[S + gi[j]] = v.y;
  }
}

// compatible gradient F^c = I + grad_dx u^c (Eq. 59) and F^r = (1-theta) F +
// theta F^c (Eq. 60): centred differences, one-sided next to a cut, the
// evolved column kept when neither neighbour is active.  The projection's
// deformation planes (evolved F, repaired F^r) hold F - I: the deviation keeps
// its digits in the FP32 build, where a stored F = I + small loses them.
template <int D, typename T>
__device__ __forceinline__ void gradF_node(const Geo &g, const uint8_t *__restrict__ act, const double *__restrict__ u,
                                           const T *__restrict__ Fm, T *__restrict__ Fr, double theta, int64_t i) {
  if (i >= g.N || !act[i]) return;
  const C3 cc = coords_of(g, i);
  for (int A = 0; A < D; ++A) {
    const int64_t lp = node_dir(g, cc, 2 * A, 1), lm = node_dir(g, cc, 2 * A + 1, 1);
    const bool hp = lp >= 0 && act[lp], hm = lm >= 0 && act[lm];
    for (int c = 0; c < D; ++c) {
      const size_t o = (size_t)c * g.S;
      const double Fe = Fm[(size_t)(c * D + A) * g.S + i];
      double Fc;
      if (hp && hm) Fc = (u[o + lp] - u[o + lm]) / (2.0 * g.dx);
      else if (hp) Fc = (u[o + lp] - u[o + i]) / g.dx;
      else if (hm) Fc = (u[o + i] - u[o + lm]) / g.dx;
      else {
        Fr[(size_t)(c * D + A) * g.S + i] = T(Fe);
        continue;
      }
      Fr[(size_t)(c * D + A) * g.S + i] = T((1.0 - theta) * Fe + theta * Fc);
    }
  }
}

// u = x, u* = x + dt/2 v  (advance = true) or x - dt/2 v
template <int D, typename T>
__device__ __forceinline__ void ureset_node(const Geo &g, const uint8_t *__restrict__ act, const double *__restrict__ x,
                                            const T *__restrict__ V, double *__restrict__ u,
                                            double *__restrict__ us, double hdt, int64_t i) {
  if (i >= g.N || !act[i]) return;
  for (int c = 0; c < D; ++c) {
    const size_t o = (size_t)c * g.S;
    u[o + i] = x[o + i];
    us[o + i] = x[o + i] + hdt * double(V[o + i]);
  }
}

// ------------------------------------------------- single-instance kernels

template <int D, typename T>
// Links [b0, b1) may span several boundary identifiers of one type (the
// table is ordered by identifier); each link reads its condition from bcs.
__global__ __launch_bounds__(256) void k_cut_dirichlet(T *__restrict__ f, Links L, int64_t b0, int64_t b1,
                                                        const BC *__restrict__ bcs, Geo g, Par p, double th) {
  const int64_t l = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l < b1) cut_dirichlet_link<D, T>(f, L, l, bcs[L.bid[l]], g, p, th);
}

template <int D, typename T>
__global__ __launch_bounds__(128) void k_cut_neumann(T *__restrict__ f, Links L, int64_t b0, int64_t b1,
                                                      const BC *__restrict__ bcs, Geo g, Par p, double th,
                                                      const double *__restrict__ u, int *__restrict__ flag,
                                                      unsigned long long *__restrict__ nfail) {
  const int64_t l = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l < b1) cut_neumann_link<D, T>(f, L, l, bcs[L.bid[l]], g, p, th, u, flag, nfail);
}

// both kinds in one launch (links sorted by identifier, so a wavefront
// mostly holds one kind); the two closures read and write disjoint slots
template <int D, typename T>
__global__ __launch_bounds__(128) void k_cut_mixed(T *__restrict__ f, Links L, int64_t b0, int64_t b1,
                                                    const BC *__restrict__ bcs, Geo g, Par p, double th,
                                                    const double *__restrict__ u, int *__restrict__ flag,
                                                    unsigned long long *__restrict__ nfail) {
  const int64_t l = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= b1) return;
  const BC &bc = bcs[L.bid[l]];
  if (bc.type == TLVLBM_BC_DIRICHLET_VELOCITY) cut_dirichlet_link<D, T>(f, L, l, bc, g, p, th);
  else cut_neumann_link<D, T>(f, L, l, bc, g, p, th, u, flag, nfail);
}

template <int D, typename T>
__global__ void k_anchor(Links L, int64_t b0, int64_t b1, BC bc, Geo g, double t, const T *__restrict__ Fm,
                         int *__restrict__ anc_n, double *__restrict__ anc_s) {
  const int64_t l = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l < b1) anchor_link<D, T>(L, l, bc, g, t, Fm, anc_n, anc_s);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_cg_rhs(Geo g, const uint8_t *__restrict__ act, const T *__restrict__ Fm,
                                                 const double *__restrict__ anc_s, double *__restrict__ b) {
  cg_rhs_node<D, T>(g, act, Fm, anc_s, b, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// over the active tiles with the neighbour masks (nodes outside the tiles
// keep b, which nothing reads there)
template <int D, typename T>
__global__ __launch_bounds__(CG_T) void k_cg_rhs_tiles(Geo g, const uint8_t *__restrict__ nbm,
                                                        const T *__restrict__ Fm, const double *__restrict__ anc_s,
                                                        double *__restrict__ b, const int32_t *__restrict__ tiles,
                                                        int ntile) {
  if ((int)blockIdx.x >= ntile) return;
  cg_rhs_node_m<D, T>(g, nbm, Fm, anc_s, b, (int64_t)tiles[blockIdx.x] * CG_T + threadIdx.x);
}

template <int D, typename T>
__global__ __launch_bounds__(CG_T) void k_cg_init(Geo g, const uint8_t *__restrict__ act,
                                                   const uint8_t *__restrict__ anc_n, const double *__restrict__ b,
                                                   const double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ p, double *partial,
                                                   const int32_t *__restrict__ tiles) {
  cg_init_blk<D, T>(g, act, anc_n, b, x, r, p, partial, tiles ? tiles[blockIdx.x] : blockIdx.x, blockIdx.x);
}

template <int D, typename T>
__global__ __launch_bounds__(CG_T) void k_cg_Ap(Geo g, const uint8_t *__restrict__ act,
                                                 const uint8_t *__restrict__ anc_n, const double *__restrict__ r,
                                                 const double *__restrict__ pold, double *__restrict__ pnew,
                                                 double *__restrict__ Ap, double *partial, const double *scal,
                                                 const int32_t *__restrict__ tiles) {
  cg_Ap_blk<D, T>(g, act, anc_n, r, pold, pnew, Ap, partial, scal, tiles ? tiles[blockIdx.x] : blockIdx.x,
                  blockIdx.x);
}

template <int D, typename T>
__global__ __launch_bounds__(CG_T) void k_cg_update(Geo g, const uint8_t *__restrict__ act, double *__restrict__ x,
                                                     double *__restrict__ r, const double *__restrict__ p,
                                                     const double *__restrict__ Ap, double *partial,
                                                     const double *scal, const int32_t *__restrict__ tiles) {
  cg_update_blk<D, T>(g, act, x, r, p, Ap, partial, scal, tiles ? tiles[blockIdx.x] : blockIdx.x, blockIdx.x);
}

// r.z for the preconditioned iteration
template <int D>
__global__ __launch_bounds__(CG_T) void k_cg_dot(Geo g, const uint8_t *__restrict__ act, const double *__restrict__ r,
                                                  const double *__restrict__ z, double *partial, const double *scal,
                                                  const int32_t *__restrict__ tiles) {
  if (scal[S_DONE] != 0.0) return;
  const int64_t i = (tiles ? tiles[blockIdx.x] : (int64_t)blockIdx.x) * CG_T + threadIdx.x;
  double v[D];
  for (int c = 0; c < D; ++c) v[c] = 0.0;
  if (i < g.N && (!act || act[i]))
    for (int c = 0; c < D; ++c) v[c] = r[(size_t)c * g.S + i] * z[(size_t)c * g.S + i];
  block_store<D>(v, partial, blockIdx.x);
}

// beta = (r.z)_new / (r.z)_old for the preconditioned iteration
template <int D> __device__ __forceinline__ void cg_rz_fin(const double *tot, double *scal, bool first) {
  for (int c = 0; c < D; ++c) {
    const double rz = tot[c];
    scal[S_BETA + c] = (!first && scal[S_ACT + c] != 0.0 && scal[S_RZ + c] != 0.0) ? rz / scal[S_RZ + c] : 0.0;
    scal[S_RZ + c] = rz;
  }
}

// finalize of a CG reduction (one block): OP 0 init, 1 p.Ap, 2 update,
// 3 r.z (4: r.z of the initial residual); PC: preconditioned iteration
template <int D, int OP, bool PC>
__device__ __forceinline__ void cg_fin(const double *partial, int nblk, double *scal, double rtol) {
  if (OP != 0 && OP != 4 && scal[S_DONE] != 0.0) return;
  __shared__ double tot[PSTRIDE];
  block_totals<(OP == 0 ? 2 * D : D)>(partial, nblk, tot);
  if (threadIdx.x == 0) {
    if (OP == 0) cg_init_fin<D>(tot, scal, rtol);
    else if (OP == 1) cg_Ap_fin<D>(tot, scal, PC);
    else if (OP == 2) cg_update_fin<D>(tot, scal, PC);
    else cg_rz_fin<D>(tot, scal, OP == 4);
  }
}

template <int D, int OP, bool PC = false>
__global__ __launch_bounds__(FIN_T) void k_cg_fin(const double *partial, int nblk, double *scal, double rtol) {
  cg_fin<D, OP, PC>(partial, nblk, scal, rtol);
}

// one block per instance
template <int D, int OP, bool PC = false>
__global__ __launch_bounds__(FIN_T) void k_cg_fin_batch(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  cg_fin<D, OP, PC>(I.partial, I.nblk, I.scal, I.rtol);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_gradF(Geo g, const uint8_t *__restrict__ act, const double *__restrict__ u,
                                                const T *__restrict__ Fm, T *__restrict__ Fr, double theta,
                                                const int32_t *__restrict__ tiles) {
  gradF_node<D, T>(g, act, u, Fm, Fr, theta,
                   (tiles ? (int64_t)tiles[blockIdx.x] : (int64_t)blockIdx.x) * 256 + threadIdx.x);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_ureset(Geo g, const uint8_t *__restrict__ act, const double *__restrict__ x,
                                                 const T *__restrict__ V, double *__restrict__ u, double *__restrict__ us,
                                                 double hdt, const int32_t *__restrict__ tiles) {
  ureset_node<D, T>(g, act, x, V, u, us, hdt,
                    (tiles ? (int64_t)tiles[blockIdx.x] : (int64_t)blockIdx.x) * 256 + threadIdx.x);
}

// Workgroups go to the 8 XCDs round robin (block b to XCD b % 8): block b
// takes tile (b % 8) * per + b / 8, so that each XCD sweeps one contiguous
// range of tiles and finds the neighbour rows and planes of x in its own L2.
constexpr int NXCD = 8;
template <int D>
__global__ __launch_bounds__(CG_T) void k_jacobi(Geo g, const uint8_t *__restrict__ nbm,
                                                 const uint8_t *__restrict__ anc_n, const double *__restrict__ b,
                                                 const double *__restrict__ xin, double *__restrict__ xout, double om,
                                                 const int32_t *__restrict__ tiles, int ntile, int per) {
  const int t = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  if (t >= ntile) return;
  const int64_t blk = tiles ? (int64_t)tiles[t] : (int64_t)t;
  jacobi_node_m<D>(g, nbm, anc_n, b, xin, xout, om, blk * CG_T + threadIdx.x);
}

// fused 2D sweeps over the tiles jt (the XCD-aware order of k_jacobi)
__global__ __launch_bounds__(CG_T) void k_jacobi_fused2(Geo g, const uint8_t *__restrict__ nbm,
                                                        const uint8_t *__restrict__ anc_n,
                                                        const double *__restrict__ b, const double *__restrict__ xin,
                                                        double *__restrict__ xout, double om,
                                                        const int32_t *__restrict__ jt, int njt, int per, int ns) {
  __shared__ double2 sx[JT_W * JT_W];
  const int t = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  if (t >= njt) return;
  const int32_t p = jt[t];
  jacobi_tile2(g, nbm, anc_n, b, xin, xout, om, p & 0xffff, p >> 16, ns, sx);
}

template <int D>
__global__ __launch_bounds__(CG_T) void k_copy_planes(Geo g, const double *__restrict__ src, double *__restrict__ dst,
                                                      const int32_t *__restrict__ tiles,
                                                      const uint8_t *__restrict__ nbm) {
  const int64_t blk = tiles ? (int64_t)tiles[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t i = blk * CG_T + threadIdx.x;
  if (i < g.N && (nbm[i] & 64u))
    for (int c = 0; c < D; ++c) dst[(size_t)c * g.S + i] = src[(size_t)c * g.S + i];
}

// copy of the displacement planes (FP64) into or out of the solver iterate,
// over the 256-node tiles that hold active nodes (tiles == null: all nodes;
// nothing reads either buffer outside the tiles)
template <int D>
__global__ __launch_bounds__(256) void k_copy_u(Geo g, const double *__restrict__ src, double *__restrict__ dst,
                                                 const int32_t *__restrict__ tiles) {
  const int64_t i = (tiles ? (int64_t)tiles[blockIdx.x] : (int64_t)blockIdx.x) * 256 + threadIdx.x;
  if (i < g.N) {
    double v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = src[(size_t)c * g.S + i];
#pragma unroll
    for (int c = 0; c < D; ++c) dst[(size_t)c * g.S + i] = v[c];
  }
}

// default CG tolerance: 1e-14 for FP64 populations, 1e-8 for FP32 ones (the
// FP32 deformation gradient carries ~1e-7 relative rounding already)
double cg_default_rtol(int prec) { return prec ? 1e-14 : 1e-8; }

// default CG iteration cap: 20 sqrt(active nodes) + 100 (CG needs
// O(sqrt(cond)) = O(grid diameter) iterations on the active-node graph)
int64_t cg_default_maxit(int64_t nactive) {
  int64_t r = 1;
  while (r * r < nactive) ++r;
  return 20 * r + 100;
}

// ------------------------------------------------------------ host side

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <int D> static int build_links_t(tlvlbm_ctx *c, const double *phi, const uint8_t *bid, std::string &err) {
  const Geo &g = c->geo;
  hipStream_t st = c->st;
  hipLaunchKernelGGL((k_active<D>), nblk(g.N, 256), 256, 0, st, phi, g, c->act, c->d_flag);
  unsigned *hist = nullptr;
  HIP_OK(dmalloc(c, &hist, 256 * sizeof(unsigned)));
  HIP_OK(hipMemsetAsync(hist, 0, 256 * sizeof(unsigned), st));
  HIP_OK(hipMemsetAsync(c->d_flag, 0, sizeof(int), st));
  hipLaunchKernelGGL((k_check_hist<D>), nblk(g.N, 256), 256, 0, st, g, c->act, bid, c->d_flag, hist);
  unsigned hh[256];
  int flag = 0;
  HIP_OK(hipMemcpyAsync(hh, hist, sizeof(hh), hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  dfree(c, hist);
  if (flag & FLAG_ARG) {
    err = "an active node has no lattice neighbour (non-periodic axis needs an inactive frame)";
    return TLVLBM_ERR_INVALID_ARG;
  }
  int64_t total = 0;
  for (int b = 0; b < 256; ++b) total += hh[b];
  Links &L = c->L;
  L.n = total;
  L.kmax = (D == 2) ? KMAX2 : KMAX3;
  const int64_t n = total > 0 ? total : 1;
  HIP_OK(dmalloc(c, &L.node, n * 8));
  HIP_OK(dmalloc(c, &L.out, n * 8));
  HIP_OK(dmalloc(c, &L.mminus, n * 8));
  HIP_OK(dmalloc(c, &L.q, n * 4));
  HIP_OK(dmalloc(c, &L.bid, n * 4));
  HIP_OK(dmalloc(c, &L.npts, n * 4));
  HIP_OK(dmalloc(c, &L.basis, n * 4));
  HIP_OK(dmalloc(c, &L.eta, n * 8));
  HIP_OK(dmalloc(c, &L.Nb, n * 24));
  HIP_OK(dmalloc(c, &L.Xb, n * 24));
  HIP_OK(dmalloc(c, &L.tang, n * 48));
  HIP_OK(dmalloc(c, &L.sidx, n * L.kmax * 4));
  HIP_OK(dmalloc(c, &L.sw, n * 2 * L.kmax * 8));
  // per-identifier compaction by prefix scan over link counts
  int *cnt = nullptr;
  int64_t *off = nullptr, *tot = nullptr, *grand = nullptr;
  const int64_t nb = (g.N + SCAN_CH - 1) / SCAN_CH;
  HIP_OK(dmalloc(c, &cnt, g.N * sizeof(int)));
  HIP_OK(dmalloc(c, &off, g.N * sizeof(int64_t)));
  HIP_OK(dmalloc(c, &tot, nb * sizeof(int64_t)));
  HIP_OK(dmalloc(c, &grand, sizeof(int64_t)));
  int64_t base = 0;
  for (int b = 0; b < 256; ++b) {
    c->bid_begin[b] = c->bid_end[b] = base;
    if (!hh[b]) continue;
    hipLaunchKernelGGL((k_count<D>), nblk(g.N, 256), 256, 0, st, g, c->act, bid, b, cnt);
    hipLaunchKernelGGL(k_scan_tot, (unsigned)nb, SCAN_T, 0, st, cnt, g.N, tot);
    hipLaunchKernelGGL(k_scan_tot2, 1, SCAN_T, 0, st, tot, nb, grand);
    hipLaunchKernelGGL(k_scan_apply, (unsigned)nb, SCAN_T, 0, st, cnt, g.N, tot, off);
    hipLaunchKernelGGL((k_scatter<D>), nblk(g.N, 256), 256, 0, st, g, c->act, bid, b, cnt, off, base, L);
    int64_t gsum = 0;
    HIP_OK(hipMemcpyAsync(&gsum, grand, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (gsum != (int64_t)hh[b]) {
      err = "cut-link compaction count mismatch";
      return TLVLBM_ERR_DEVICE;
    }
    base += gsum;
    c->bid_end[b] = base;
  }
  dfree(c, cnt);
  dfree(c, off);
  dfree(c, tot);
  dfree(c, grand);
  if (total > 0) {
    hipLaunchKernelGGL((k_link_geom<D>), nblk(total, 128), 128, 0, st, g, phi, c->act, L);
    hipLaunchKernelGGL((k_link_lsq<D>), nblk(total, 64), 64, 0, st, g, c->act, L, c->d_flag);
  }
  HIP_OK(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (flag & FLAG_STENCIL) {
    err = "LSQ stencil exceeds its capacity";
    return TLVLBM_ERR_DEVICE;
  }
  HIP_OK(hipGetLastError());
  return TLVLBM_OK;
}

int build_links(tlvlbm_ctx *c, const double *phi, const uint8_t *bid, std::string &err) {
  return c->D == 2 ? build_links_t<2>(c, phi, bid, err) : build_links_t<3>(c, phi, bid, err);
}

// device copy of the boundary conditions (after tlvlbm_set_boundary),
// ordered on the context's stream behind the steps already queued
static int sync_bcs(tlvlbm_ctx *c) {
  if (!c->d_bcs && dmalloc(c, &c->d_bcs, sizeof(c->bcs)) != hipSuccess) return TLVLBM_ERR_OUT_OF_MEMORY;
  if (c->bcs_dirty) {
    if (hipMemcpyAsync(c->d_bcs, c->bcs, sizeof(c->bcs), hipMemcpyHostToDevice, c->st) != hipSuccess)
      return TLVLBM_ERR_DEVICE;
    c->bcs_dirty = false;
  }
  return TLVLBM_OK;
}

// one launch per run of consecutive boundary identifiers of one type (the
// links of a run are contiguous in the table), so that e.g. both walls of a
// tube close in one Neumann launch
template <int D, typename T> static int cutlinks_t(tlvlbm_ctx *c, double tn) {
  const double th = (double(c->step) + 0.5) * c->par.dt;  // t^n + dt/2, same rounding as the batched path
  const int s = sync_bcs(c);
  if (s) return s;
  // both kinds present: one launch over every link
  bool any_dir = false, any_neu = false;
  int64_t lo = -1, hi = -1;
  for (int b = 0; b < 256; ++b) {
    if (c->bid_end[b] <= c->bid_begin[b]) continue;
    if (c->bcs[b].type == TLVLBM_BC_DIRICHLET_VELOCITY) any_dir = true;
    else any_neu = true;
    if (lo < 0) lo = c->bid_begin[b];
    hi = c->bid_end[b];
  }
  if (any_dir && any_neu && hi - lo == c->L.n) {
    hipLaunchKernelGGL((k_cut_mixed<D, T>), nblk(hi - lo, 128), 128, 0, c->st, (T *)c->fA, c->L, lo, hi,
                       (const BC *)c->d_bcs, c->geo, c->par, th, (const double *)c->ubuf, c->d_flag,
                       (unsigned long long *)c->d_newton_fail);
    return TLVLBM_OK;
  }
  int b = 0;
  while (b < 256) {
    if (c->bid_end[b] <= c->bid_begin[b]) {
      ++b;
      continue;
    }
    const int type = c->bcs[b].type;
    const int64_t b0 = c->bid_begin[b];
    int64_t b1 = c->bid_end[b];
    int e = b + 1;
    for (; e < 256; ++e) {
      if (c->bid_end[e] <= c->bid_begin[e]) continue;
      if (c->bcs[e].type != type || c->bid_begin[e] != b1) break;
      b1 = c->bid_end[e];
    }
    if (type == TLVLBM_BC_DIRICHLET_VELOCITY)
      hipLaunchKernelGGL((k_cut_dirichlet<D, T>), nblk(b1 - b0, 256), 256, 0, c->st, (T *)c->fA, c->L, b0, b1,
                         (const BC *)c->d_bcs, c->geo, c->par, th);
    else
      hipLaunchKernelGGL((k_cut_neumann<D, T>), nblk(b1 - b0, 128), 128, 0, c->st, (T *)c->fA, c->L, b0, b1,
                         (const BC *)c->d_bcs, c->geo, c->par, th, (const double *)c->ubuf, c->d_flag,
                         (unsigned long long *)c->d_newton_fail);
    b = e;
  }
  return TLVLBM_OK;
}

// the displacement at the Neumann stencil nodes, for the reverse-mode tape
__global__ __launch_bounds__(256) void k_gather_u(const double *__restrict__ u, int64_t S, int D,
                                                  const int64_t *__restrict__ un, int64_t nu,
                                                  double *__restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nu) return;
  const int64_t j = un[t];
  for (int i = 0; i < D; ++i) out[(size_t)i * nu + t] = u[(size_t)i * S + j];
}

// chunk slots of whole planes, for the reverse-mode tape
template <typename T>
__global__ __launch_bounds__(256) void k_tape_gather(const T *__restrict__ src, int64_t S, int64_t N,
                                                     const int32_t *__restrict__ chunks, int64_t nslot, int planes,
                                                     T *__restrict__ dst) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslot) return;
  const int64_t node = (int64_t)chunks[s / CHUNK] * CHUNK + (s % CHUNK);
  if (node >= N) return;
  for (int k = 0; k < planes; ++k) dst[(size_t)k * nslot + s] = src[(size_t)k * S + node];
}

void launch_tape_gather(tlvlbm_ctx *c, const void *src, void *dst, int planes) {
  const int64_t ns = (int64_t)c->nchunks * CHUNK;
  if (c->prec)
    hipLaunchKernelGGL(k_tape_gather<double>, nblk(ns, 256), 256, 0, c->st, (const double *)src, c->geo.S, c->geo.N,
                       c->chunks, ns, planes, (double *)dst);
  else
    hipLaunchKernelGGL(k_tape_gather<float>, nblk(ns, 256), 256, 0, c->st, (const float *)src, c->geo.S, c->geo.N,
                       c->chunks, ns, planes, (float *)dst);
}

void launch_gather_u(tlvlbm_ctx *c, const int64_t *un, int64_t nu, double *out) {
  hipLaunchKernelGGL(k_gather_u, nblk(nu, 256), 256, 0, c->st, (const double *)c->ubuf, c->geo.S, c->D, un, nu,
                     out);
}

int launch_cutlinks(tlvlbm_ctx *c, double tn) {
  if (c->D == 2) return c->prec ? cutlinks_t<2, double>(c, tn) : cutlinks_t<2, float>(c, tn);
  return c->prec ? cutlinks_t<3, double>(c, tn) : cutlinks_t<3, float>(c, tn);
}

template <int D, typename T> static int cg_alloc(tlvlbm_ctx *c) {
  CG &w = c->cg;
  if (w.x) return TLVLBM_OK;
  // CG vectors are FP64 in both builds (a few node planes; FP32 vectors
  // stall well above the tolerance on large graphs)
  const size_t plane = (size_t)c->geo.S * sizeof(T), dplane = (size_t)c->geo.S * sizeof(double);
  void **vec[] = {&w.x, &w.r, &w.p0, &w.p1, &w.Ap, &w.b, &w.anc_s, &w.z};
  for (void **pp : vec) {
    HIP_OK(dmalloc(c, pp, D * dplane));
    HIP_OK(hipMemsetAsync(*pp, 0, D * dplane, c->st));
  }
  HIP_OK(dmalloc(c, &w.V, D * plane));
  HIP_OK(dmalloc(c, &w.Fm, D * D * plane));
  HIP_OK(dmalloc(c, &w.Fr, D * D * plane));
  HIP_OK(hipMemsetAsync(w.Fr, 0, D * D * plane, c->st));
  HIP_OK(dmalloc(c, &w.anc_n, c->geo.S));
  HIP_OK(dmalloc(c, &w.anc_i, c->geo.S * sizeof(int)));
  w.nblk = (int)nblk(c->geo.N, CG_T);
  HIP_OK(dmalloc(c, &w.partial, (size_t)w.nblk * PSTRIDE * sizeof(double)));
  HIP_OK(dmalloc(c, &w.scal, S_NSCAL * sizeof(double)));
  return TLVLBM_OK;
}

// anchors accumulate in int32 then narrow to uint8 counts
template <int D, typename T>
__global__ void k_anchor_narrow(Geo g, const int *__restrict__ ai, uint8_t *__restrict__ an) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < g.N) an[i] = (uint8_t)ai[i];
}

template <int D, typename T> static int cg_run(tlvlbm_ctx *c, const uint8_t *anc_n);

// Preconditioned CG (one multigrid V-cycle per iteration) on the workspace:
// right-hand side w.b, start and result w.x; the same per-component scalars
// and stopping rule as the plain iteration (relative residual ||r||).
template <int D, typename T> static int pcg_run(tlvlbm_ctx *c, const uint8_t *anc_n, double rtol) {
  CG &w = c->cg;
  const Geo &g = c->geo;
  hipStream_t st = c->st;
  if (!c->mg || !c->gauge || c->aux_stale) {
    const int s = proj_aux_build(c);
    if (s) return s;
  }
  // the preconditioner moves the constants of components without anchors,
  // which plain CG from the warm start keeps: restore them afterwards
  gauge_means(c, (const double *)w.x, nullptr, c->gauge->mean0);
  double *r = (double *)w.r, *z = (double *)w.z;
  const int nt = w.tiles ? w.ntiles : w.nblk;
  hipLaunchKernelGGL((k_cg_init<D, T>), nt, CG_T, 0, st, g, c->act, anc_n, (const double *)w.b,
                     (const double *)w.x, r, (double *)w.p0, w.partial, w.tiles);
  hipLaunchKernelGGL((k_cg_fin<D, 0>), 1, FIN_T, 0, st, w.partial, nt, w.scal, rtol);
  mg_apply(c, r, z, nullptr);
  hipLaunchKernelGGL((k_cg_dot<D>), nt, CG_T, 0, st, g, c->act, (const double *)r, (const double *)z, w.partial,
                     (const double *)w.scal, w.tiles);
  hipLaunchKernelGGL((k_cg_fin<D, 4, true>), 1, FIN_T, 0, st, w.partial, nt, w.scal, 0.0);
  const int64_t maxit = c->cg_maxit > 0 ? c->cg_maxit : cg_default_maxit(c->nactive);
  // PCG_BATCH iterations between convergence polls (even, so that the p
  // ping-pong returns to p0); every kernel returns at once after convergence
  constexpr int PCG_BATCH = 8;
  auto body = [&]() {
    double *pa = (double *)w.p0, *pb = (double *)w.p1;
    for (int k = 0; k < PCG_BATCH; ++k) {
      hipLaunchKernelGGL((k_cg_Ap<D, T>), nt, CG_T, 0, st, g, c->act, anc_n, (const double *)z, pa, pb,
                         (double *)w.Ap, w.partial, w.scal, w.tiles);
      hipLaunchKernelGGL((k_cg_fin<D, 1, true>), 1, FIN_T, 0, st, w.partial, nt, w.scal, 0.0);
      hipLaunchKernelGGL((k_cg_update<D, T>), nt, CG_T, 0, st, g, c->act, (double *)w.x, r, pb,
                         (const double *)w.Ap, w.partial, w.scal, w.tiles);
      hipLaunchKernelGGL((k_cg_fin<D, 2, true>), 1, FIN_T, 0, st, w.partial, nt, w.scal, 0.0);
      mg_apply(c, r, z, w.scal);
      hipLaunchKernelGGL((k_cg_dot<D>), nt, CG_T, 0, st, g, c->act, (const double *)r, (const double *)z,
                         w.partial, (const double *)w.scal, w.tiles);
      hipLaunchKernelGGL((k_cg_fin<D, 3, true>), 1, FIN_T, 0, st, w.partial, nt, w.scal, 0.0);
      std::swap(pa, pb);
    }
  };
  // the batch is launch-bound (about 45 small kernels per iteration): replay
  // it from a graph captured once per hierarchy and anchor set (not on the
  // legacy default stream, which cannot be captured)
  const bool use_graph = st != nullptr;
  if (use_graph && (!w.pcg_graph || w.pcg_key != (const void *)anc_n)) {
    if (w.pcg_graph) (void)hipGraphExecDestroy(w.pcg_graph);
    w.pcg_graph = nullptr;
    hipGraph_t gr = nullptr;
    HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    body();
    HIP_OK(hipStreamEndCapture(st, &gr));
    const hipError_t e = hipGraphInstantiate(&w.pcg_graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
      w.pcg_graph = nullptr;
      return TLVLBM_ERR_DEVICE;
    }
    w.pcg_key = (const void *)anc_n;
  }
  for (int64_t it = 0; it < maxit; it += PCG_BATCH) {
    if (use_graph) HIP_OK(hipGraphLaunch(w.pcg_graph, st));
    else body();
    HIP_OK(hipMemcpyAsync(c->hscal, w.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (c->hscal[S_DONE] != 0.0) break;
  }
  gauge_restore(c, (double *)w.x, c->gauge->mean0);
  HIP_OK(hipMemcpyAsync(c->hscal, w.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int k = 0; k < D; ++k) c->st_cg += (int64_t)c->hscal[S_ITS + k];
  return TLVLBM_OK;
}

// the projection's damped Jacobi relaxation (Sec. 3.5) on the workspace:
// right-hand side w.b, start and result w.x (w.r is the second sweep
// buffer); proj_sweeps sweeps of weight proj_weight over the active tiles
template <int D> static int jacobi_run(tlvlbm_ctx *c, const uint8_t *anc_n) {
  CG &w = c->cg;
  const Geo &g = c->geo;
  hipStream_t st = c->st;
  if (!c->gauge || c->aux_stale) {
    const int s = proj_aux_build(c);
    if (s) return s;
  }
  if (!w.nbm) return TLVLBM_ERR_DEVICE;
  const unsigned nt = w.tiles ? (unsigned)w.ntiles : nblk(g.N, CG_T);
  const int per = (int)((nt + NXCD - 1) / NXCD);
  double *a = (double *)w.x, *bb = (double *)w.r;
  if (D == 2 && w.jt) {
    // up to JT_NS sweeps per launch, staged in LDS
    const int per2 = (w.njt + NXCD - 1) / NXCD;
    for (int left = c->proj_sweeps; left > 0;) {
      const int ns = std::min(left, JT_NS);
      hipLaunchKernelGGL(k_jacobi_fused2, (unsigned)(per2 * NXCD), CG_T, 0, st, g, w.nbm, anc_n,
                         (const double *)w.b, (const double *)a, bb, c->proj_weight, w.jt, w.njt, per2, ns);
      std::swap(a, bb);
      left -= ns;
    }
  } else {
    for (int k = 0; k < c->proj_sweeps; ++k) {
      hipLaunchKernelGGL((k_jacobi<D>), (unsigned)(per * NXCD), CG_T, 0, st, g, w.nbm, anc_n, (const double *)w.b,
                         (const double *)a, bb, c->proj_weight, w.tiles, (int)nt, per);
      std::swap(a, bb);
    }
  }
  if (a != (double *)w.x)
    hipLaunchKernelGGL((k_copy_planes<D>), nt, CG_T, 0, st, g, (const double *)a, (double *)w.x, w.tiles, w.nbm);
  c->st_cg += (int64_t)c->proj_sweeps * D;
  return hipGetLastError() == hipSuccess ? TLVLBM_OK : TLVLBM_ERR_DEVICE;
}

template <int D, typename T> static int cg_solve(tlvlbm_ctx *c, const T *F, double t) {
  CG &w = c->cg;
  const Geo &g = c->geo;
  hipStream_t st = c->st;
  // anchors from the Dirichlet cut links
  bool any_dir = false;
  for (int b = 0; b < 256; ++b)
    if (c->bid_end[b] > c->bid_begin[b] && c->bcs[b].type == TLVLBM_BC_DIRICHLET_VELOCITY) any_dir = true;
  const uint8_t *anc_n = nullptr;
  const double *anc_s = nullptr;
  if (any_dir) {
    int *ai = w.anc_i;
    HIP_OK(hipMemsetAsync(ai, 0, g.N * sizeof(int), st));
    HIP_OK(hipMemsetAsync(w.anc_s, 0, D * (size_t)g.S * sizeof(double), st));
    for (int b = 0; b < 256; ++b) {
      const int64_t b0 = c->bid_begin[b], b1 = c->bid_end[b];
      if (b1 <= b0 || c->bcs[b].type != TLVLBM_BC_DIRICHLET_VELOCITY) continue;
      hipLaunchKernelGGL((k_anchor<D, T>), nblk(b1 - b0, 128), 128, 0, st, c->L, b0, b1, c->bcs[b], g, t, F, ai,
                         (double *)w.anc_s);
    }
    hipLaunchKernelGGL((k_anchor_narrow<D, T>), nblk(g.N, 256), 256, 0, st, g, ai, w.anc_n);
    anc_n = w.anc_n;
    anc_s = (const double *)w.anc_s;
  }
  if (w.nbm && w.tiles)
    hipLaunchKernelGGL((k_cg_rhs_tiles<D, T>), (unsigned)w.ntiles, CG_T, 0, st, g, w.nbm, F, anc_s, (double *)w.b,
                       w.tiles, w.ntiles);
  else
    hipLaunchKernelGGL((k_cg_rhs<D, T>), nblk(g.N, 256), 256, 0, st, g, c->act, F, anc_s, (double *)w.b);
  if (c->proj_sweeps > 0) return jacobi_run<D>(c, anc_n);
  return cg_run<D, T>(c, anc_n);
}

// CG iterations on the workspace: right-hand side w.b, start and result w.x,
// matrix = active-graph Laplacian + anchor counts anc_n (may be null)
template <int D, typename T> static int cg_run(tlvlbm_ctx *c, const uint8_t *anc_n) {
  CG &w = c->cg;
  const Geo &g = c->geo;
  hipStream_t st = c->st;
  const double rtol = c->cg_rtol > 0 ? c->cg_rtol : cg_default_rtol(c->prec);
  if (!c->gauge || c->aux_stale) {
    const int s = proj_aux_build(c);
    if (s) return s;
  }
  if (c->cg_multigrid) return pcg_run<D, T>(c, anc_n, rtol);
  const int nt = w.tiles ? w.ntiles : w.nblk;
  hipLaunchKernelGGL((k_cg_init<D, T>), nt, CG_T, 0, st, g, c->act, anc_n, (const double *)w.b,
                     (const double *)w.x, (double *)w.r, (double *)w.p0, w.partial, w.tiles);
  hipLaunchKernelGGL((k_cg_fin<D, 0>), 1, FIN_T, 0, st, w.partial, nt, w.scal, rtol);
  const int64_t maxit = c->cg_maxit > 0 ? c->cg_maxit : cg_default_maxit(c->nactive);
  double *pa = (double *)w.p0, *pb = (double *)w.p1;
  int64_t it = 0;
  while (it < maxit) {
    const int64_t batch = std::min<int64_t>(32, maxit - it);
    for (int64_t k = 0; k < batch; ++k) {
      hipLaunchKernelGGL((k_cg_Ap<D, T>), nt, CG_T, 0, st, g, c->act, anc_n, (const double *)w.r, pa, pb,
                         (double *)w.Ap, w.partial, w.scal, w.tiles);
      hipLaunchKernelGGL((k_cg_fin<D, 1>), 1, FIN_T, 0, st, w.partial, nt, w.scal, 0.0);
      hipLaunchKernelGGL((k_cg_update<D, T>), nt, CG_T, 0, st, g, c->act, (double *)w.x, (double *)w.r, pb,
                         (const double *)w.Ap, w.partial, w.scal, w.tiles);
      hipLaunchKernelGGL((k_cg_fin<D, 2>), 1, FIN_T, 0, st, w.partial, nt, w.scal, 0.0);
      std::swap(pa, pb);
    }
    it += batch;
    HIP_OK(hipMemcpyAsync(c->hscal, w.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (c->hscal[S_DONE] != 0.0) break;
  }
  HIP_OK(hipMemcpyAsync(c->hscal, w.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int k = 0; k < D; ++k) c->st_cg += (int64_t)c->hscal[S_ITS + k];
  return TLVLBM_OK;
}

// first == true: projection before collision (u^c from F^n, then F^r);
// first == false: projection after the repaired collision (u from F^r),
// followed by the displacement reset.
// copies of the CG solution on the active tiles: pack (dir 0) to a store
// [D][ntiles*256], or unpack (dir 1) from it
template <int D>
__global__ __launch_bounds__(256) void k_xstore(Geo g, const int32_t *__restrict__ tiles, int ntiles,
                                                 double *__restrict__ x, double *__restrict__ store, int dir) {
  const int64_t i = (int64_t)tiles[blockIdx.x] * 256 + threadIdx.x;
  if (i >= g.N) return;
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x, ps = (size_t)ntiles * 256;
  for (int c = 0; c < D; ++c) {
    if (dir) x[(size_t)c * g.S + i] = store[c * ps + o];
    else store[c * ps + o] = x[(size_t)c * g.S + i];
  }
}

// the projection's solve, or (mode 2) its solution replayed from a store
// written by an earlier run of the same step (mode 1)
template <int D, typename T> static int solve_or_replay(tlvlbm_ctx *c, const T *F, double tn, double *store, int mode) {
  CG &w = c->cg;
  if (mode == 2 && store && w.tiles) {
    hipLaunchKernelGGL((k_xstore<D>), w.ntiles, 256, 0, c->st, c->geo, w.tiles, w.ntiles, (double *)w.x, store, 1);
    return TLVLBM_OK;
  }
  const int st = cg_solve<D, T>(c, F, tn);
  if (st) return st;
  if (mode == 1 && store && w.tiles)
    hipLaunchKernelGGL((k_xstore<D>), w.ntiles, 256, 0, c->st, c->geo, w.tiles, w.ntiles, (double *)w.x, store, 0);
  return TLVLBM_OK;
}

template <int D, typename T>
static int projection_t(tlvlbm_ctx *c, bool first, double tn, double *store, int mode) {
  int st = cg_alloc<D, T>(c);
  if (st) return st;
  CG &w = c->cg;
  const Geo &g = c->geo;
  // projection tables (tiles, masks, components) current before any launch
  // that uses them
  if (!c->gauge || c->aux_stale) {
    st = proj_aux_build(c);
    if (st) return st;
  }
  // the node-wise kernels around the solve run over the active tiles
  const int32_t *tl = w.tiles;
  const unsigned nt = tl ? (unsigned)w.ntiles : nblk(g.N, 256);
  if (first) {
    launch_pull_moments(c, nullptr, nullptr, nullptr, true);  // v, F, u^n
    hipLaunchKernelGGL((k_copy_u<D>), nt, 256, 0, c->st, g, (const double *)c->ubuf, (double *)w.x, tl);
    st = solve_or_replay<D, T>(c, (const T *)w.Fm, tn, store, mode);
    if (st) return st;
    hipLaunchKernelGGL((k_copy_u<D>), nt, 256, 0, c->st, g, (const double *)w.x, (double *)c->ubuf, tl);
    hipLaunchKernelGGL((k_gradF<D, T>), nt, 256, 0, c->st, g, c->act, (const double *)w.x, (const T *)w.Fm,
                       (T *)w.Fr, c->theta, tl);
  } else {
    hipLaunchKernelGGL((k_copy_u<D>), nt, 256, 0, c->st, g, (const double *)c->ubuf, (double *)w.x, tl);
    st = solve_or_replay<D, T>(c, (const T *)w.Fr, tn, store, mode);
    if (st) return st;
    hipLaunchKernelGGL((k_ureset<D, T>), nt, 256, 0, c->st, g, c->act, (const double *)w.x, (const T *)w.V,
                       (double *)c->ubuf, (double *)c->ustar, 0.5 * c->par.dt, tl);
  }
  HIP_OK(hipGetLastError());
  return TLVLBM_OK;
}

int run_cg_given(tlvlbm_ctx *c, const uint8_t *anc_n) {
  if (c->D == 2) return c->prec ? cg_run<2, double>(c, anc_n) : cg_run<2, float>(c, anc_n);
  return c->prec ? cg_run<3, double>(c, anc_n) : cg_run<3, float>(c, anc_n);
}

int run_projection(tlvlbm_ctx *c, bool first, double tn, double *store, int mode) {
  if (c->D == 2)
    return c->prec ? projection_t<2, double>(c, first, tn, store, mode)
                   : projection_t<2, float>(c, first, tn, store, mode);
  return c->prec ? projection_t<3, double>(c, first, tn, store, mode)
                 : projection_t<3, float>(c, first, tn, store, mode);
}

}  // namespace tl

// ===================================================== batched launches
// Tiles:  node tiles (instance, block of 256 grid nodes), link tiles
// (segment, first link).  A segment is one boundary identifier of one
// instance (contiguous link range, one condition).  Every block works on one
// instance, so CG reductions are segmented by instance with the same
// deterministic last-block scheme as the single-instance solver.

namespace tl {

template <int D, typename T>
__global__ __launch_bounds__(64) void k_cut_batch(const Inst *__restrict__ insts, const Seg *__restrict__ segs,
                                                  const int4 *__restrict__ tiles, const int64_t *__restrict__ step) {
  const int4 t = tiles[blockIdx.x];
  const Seg &sg = segs[t.x];
  const Inst &I = insts[sg.inst];
  const int64_t l = sg.b0 + t.y + threadIdx.x;
  if (l >= sg.b1) return;
  const double th = (double(*step) + 0.5) * I.p.dt;
  if (sg.type == TLVLBM_BC_DIRICHLET_VELOCITY)
    cut_dirichlet_link<D, T>((T *)I.fout, I.L, l, sg.bc, I.g, I.p, th);
  else
    cut_neumann_link<D, T>((T *)I.fout, I.L, l, sg.bc, I.g, I.p, th, (const double *)I.ubuf, I.flag, I.nfail);
}

template <int D, typename T>
__global__ __launch_bounds__(64) void k_anchor_batch(const Inst *__restrict__ insts, const Seg *__restrict__ segs,
                                                     const int4 *__restrict__ tiles, const int64_t *__restrict__ step,
                                                     int useFr) {
  const int4 t = tiles[blockIdx.x];
  const Seg &sg = segs[t.x];
  if (sg.type != TLVLBM_BC_DIRICHLET_VELOCITY) return;
  const Inst &I = insts[sg.inst];
  const int64_t l = sg.b0 + t.y + threadIdx.x;
  if (l >= sg.b1) return;
  const double tn = double(*step) * I.p.dt;
  anchor_link<D, T>(I.L, l, sg.bc, I.g, tn, (const T *)(useFr ? I.Fr : I.Fm), I.anc_i, (double *)I.anc_s);
}

// per-node utilities over node tiles: 0 zero anchors, 1 narrow anchors,
// 2 x <- u, 3 u <- x
template <int D, typename T>
__global__ __launch_bounds__(256) void k_node_util_batch(const Inst *__restrict__ insts,
                                                         const int4 *__restrict__ tiles, int op) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const int64_t i = t.y * (int64_t)256 + threadIdx.x;
  if (i >= I.g.N) return;
  if (op == 0) {
    if (I.anc_i) I.anc_i[i] = 0;
    for (int c = 0; c < D; ++c) ((double *)I.anc_s)[(size_t)c * I.g.S + i] = 0.0;
  } else if (op == 1) {
    if (I.anc_n) I.anc_n[i] = (uint8_t)I.anc_i[i];
  } else if (op == 2) {
    for (int c = 0; c < D; ++c) ((double *)I.x)[(size_t)c * I.g.S + i] = ((const double *)I.ubuf)[(size_t)c * I.g.S + i];
  } else {
    for (int c = 0; c < D; ++c) ((double *)I.ubuf)[(size_t)c * I.g.S + i] = ((const double *)I.x)[(size_t)c * I.g.S + i];
  }
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_cg_rhs_batch(const Inst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles, int useFr, int anchored) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  cg_rhs_node<D, T>(I.g, I.act, (const T *)(useFr ? I.Fr : I.Fm), anchored ? (const double *)I.anc_s : nullptr,
                    (double *)I.b, t.y * (int64_t)256 + threadIdx.x);
}

template <int D, typename T>
__global__ __launch_bounds__(CG_T) void k_cg_init_batch(const Inst *__restrict__ insts,
                                                        const int4 *__restrict__ tiles, int anchored) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  cg_init_blk<D, T>(I.g, I.act, anchored ? I.anc_n : nullptr, (const double *)I.b, (const double *)I.x,
                    (double *)I.r, (double *)I.p0, I.partial, t.y, t.y);
}

template <int D, typename T>
__global__ __launch_bounds__(CG_T) void k_cg_Ap_batch(const Inst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles, int pp, int anchored,
                                                      int precond) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const double *pold = (const double *)(pp ? I.p1 : I.p0);
  double *pnew = (double *)(pp ? I.p0 : I.p1);
  cg_Ap_blk<D, T>(I.g, I.act, anchored ? I.anc_n : nullptr, (const double *)(precond ? I.z : I.r), pold, pnew,
                  (double *)I.Ap, I.partial, I.scal, t.y, t.y);
}

// r.z per instance (batched preconditioned iteration)
template <int D>
__global__ __launch_bounds__(CG_T) void k_cg_dot_batch(const Inst *__restrict__ insts,
                                                       const int4 *__restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  if (((const double *)I.scal)[S_DONE] != 0.0) return;
  const int64_t i = (int64_t)t.y * CG_T + threadIdx.x;
  double v[D];
  for (int c = 0; c < D; ++c) v[c] = 0.0;
  if (i < I.g.N && I.act[i])
    for (int c = 0; c < D; ++c)
      v[c] = ((const double *)I.r)[(size_t)c * I.g.S + i] * ((const double *)I.z)[(size_t)c * I.g.S + i];
  block_store<D>(v, I.partial, t.y);
}

template <int D, typename T>
__global__ __launch_bounds__(CG_T) void k_cg_update_batch(const Inst *__restrict__ insts,
                                                          const int4 *__restrict__ tiles, int pp) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const double *pnew = (const double *)(pp ? I.p0 : I.p1);
  cg_update_blk<D, T>(I.g, I.act, (double *)I.x, (double *)I.r, pnew, (const double *)I.Ap, I.partial, I.scal,
                      t.y, t.y);
}

// batched Jacobi sweep: dir 0 reads x and writes r, dir 1 the reverse;
// copy: x = r
template <int D>
__global__ __launch_bounds__(CG_T) void k_jacobi_batch(const Inst *__restrict__ insts, const int4 *__restrict__ tiles,
                                                       int dir, int anchored, double om) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const double *xin = (const double *)(dir ? I.r : I.x);
  double *xout = (double *)(dir ? I.x : I.r);
  if (I.nbm)
    jacobi_node_m<D>(I.g, I.nbm, anchored ? I.anc_n : nullptr, (const double *)I.b, xin, xout, om,
                     (int64_t)t.y * CG_T + threadIdx.x);
  else
    jacobi_node<D>(I.g, I.act, anchored ? I.anc_n : nullptr, (const double *)I.b, xin, xout, om,
                   (int64_t)t.y * CG_T + threadIdx.x);
}

// fused 2D sweeps of the batch: tiles (instance, tx, ty) in the XCD-aware
// order of k_jacobi; dir as in k_jacobi_batch
__global__ __launch_bounds__(CG_T) void k_jacobi_fused2_batch(const Inst *__restrict__ insts,
                                                              const int4 *__restrict__ jt, int njt, int per, int dir,
                                                              int anchored, double om, int ns) {
  __shared__ double2 sx[JT_W * JT_W];
  const int t = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  if (t >= njt) return;
  const int4 q = jt[t];
  const Inst &I = insts[q.x];
  const double *xin = (const double *)(dir ? I.r : I.x);
  double *xout = (double *)(dir ? I.x : I.r);
  jacobi_tile2(I.g, I.nbm, anchored ? I.anc_n : nullptr, (const double *)I.b, xin, xout, om, q.y, q.z, ns, sx);
}

template <int D>
__global__ __launch_bounds__(CG_T) void k_jacobi_copy_batch(const Inst *__restrict__ insts,
                                                            const int4 *__restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const int64_t i = (int64_t)t.y * CG_T + threadIdx.x;
  // the sweeps over the neighbour masks skip inactive nodes: copy active ones
  if (i < I.g.N && (!I.nbm || (I.nbm[i] & 64u)))
    for (int c = 0; c < D; ++c)
      ((double *)I.x)[(size_t)c * I.g.S + i] = ((const double *)I.r)[(size_t)c * I.g.S + i];
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_gradF_batch(const Inst *__restrict__ insts, const int4 *__restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  gradF_node<D, T>(I.g, I.act, (const double *)I.x, (const T *)I.Fm, (T *)I.Fr, I.theta,
                   t.y * (int64_t)256 + threadIdx.x);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_ureset_batch(const Inst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  ureset_node<D, T>(I.g, I.act, (const double *)I.x, (const T *)I.V, (double *)I.ubuf, (double *)I.ustar, 0.5 * I.p.dt,
                    t.y * (int64_t)256 + threadIdx.x);
}

// end of a batched step: swap every instance's population buffers and
// advance the device step counter
__global__ void k_step_end(Inst *__restrict__ insts, int n, int64_t *__restrict__ step) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    void *a = insts[k].fin;
    insts[k].fin = insts[k].fout;
    insts[k].fout = a;
  }
  if (k == 0) step[0] += 1;
}

// number of instances whose CG is still running
__global__ void k_cg_pending(const Inst *__restrict__ insts, int n, int *__restrict__ pending) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && insts[k].scal[S_DONE] == 0.0) atomicAdd(pending, 1);
}

template <int D, typename T>
static void batch_kernels_t(BatchOp op, const BatchArgs &a) {
  hipStream_t st = a.st;
  switch (op) {
    case BatchOp::Cut:
      hipLaunchKernelGGL((k_cut_batch<D, T>), a.nlt, 64, 0, st, a.insts, a.segs, a.ltiles, a.step);
      break;
    case BatchOp::Anchor:
      hipLaunchKernelGGL((k_anchor_batch<D, T>), a.nlt, 64, 0, st, a.insts, a.segs, a.ltiles, a.step, a.flagA);
      break;
    case BatchOp::ZeroAnchor:
    case BatchOp::NarrowAnchor:
    case BatchOp::XfromU:
    case BatchOp::UfromX: {
      const int code = op == BatchOp::ZeroAnchor ? 0 : op == BatchOp::NarrowAnchor ? 1 : op == BatchOp::XfromU ? 2 : 3;
      hipLaunchKernelGGL((k_node_util_batch<D, T>), a.nct, 256, 0, st, a.insts, a.ctiles, code);
      break;
    }
    case BatchOp::Rhs:
      hipLaunchKernelGGL((k_cg_rhs_batch<D, T>), a.nct, 256, 0, st, a.insts, a.ctiles, a.flagA, a.flagB);
      break;
    case BatchOp::CgInit:
      hipLaunchKernelGGL((k_cg_init_batch<D, T>), a.nct, CG_T, 0, st, a.insts, a.ctiles, a.flagB);
      hipLaunchKernelGGL((k_cg_fin_batch<D, 0>), a.ninst, FIN_T, 0, st, a.insts);
      break;
    case BatchOp::CgAp:
      hipLaunchKernelGGL((k_cg_Ap_batch<D, T>), a.nct, CG_T, 0, st, a.insts, a.ctiles, a.flagA, a.flagB, 0);
      hipLaunchKernelGGL((k_cg_fin_batch<D, 1>), a.ninst, FIN_T, 0, st, a.insts);
      break;
    case BatchOp::PcAp:
      hipLaunchKernelGGL((k_cg_Ap_batch<D, T>), a.nct, CG_T, 0, st, a.insts, a.ctiles, a.flagA, a.flagB, 1);
      hipLaunchKernelGGL((k_cg_fin_batch<D, 1, true>), a.ninst, FIN_T, 0, st, a.insts);
      break;
    case BatchOp::PcUpdate:
      hipLaunchKernelGGL((k_cg_update_batch<D, T>), a.nct, CG_T, 0, st, a.insts, a.ctiles, a.flagA);
      hipLaunchKernelGGL((k_cg_fin_batch<D, 2, true>), a.ninst, FIN_T, 0, st, a.insts);
      break;
    case BatchOp::PcDot:
    case BatchOp::PcDotFirst:
      hipLaunchKernelGGL((k_cg_dot_batch<D>), a.nct, CG_T, 0, st, a.insts, a.ctiles);
      if (op == BatchOp::PcDot)
        hipLaunchKernelGGL((k_cg_fin_batch<D, 3, true>), a.ninst, FIN_T, 0, st, a.insts);
      else
        hipLaunchKernelGGL((k_cg_fin_batch<D, 4, true>), a.ninst, FIN_T, 0, st, a.insts);
      break;
    case BatchOp::PcInit:
      break;
    case BatchOp::CgUpdate:
      hipLaunchKernelGGL((k_cg_update_batch<D, T>), a.nct, CG_T, 0, st, a.insts, a.ctiles, a.flagA);
      hipLaunchKernelGGL((k_cg_fin_batch<D, 2>), a.ninst, FIN_T, 0, st, a.insts);
      break;
    case BatchOp::GradF:
      hipLaunchKernelGGL((k_gradF_batch<D, T>), a.nct, 256, 0, st, a.insts, a.ctiles);
      break;
    case BatchOp::Jacobi:
      hipLaunchKernelGGL((k_jacobi_batch<D>), a.nct, CG_T, 0, st, a.insts, a.ctiles, a.flagA, a.flagB, a.om);
      break;
    case BatchOp::JacobiFused:
      if (D == 2) {
        const int per = (a.njt + NXCD - 1) / NXCD;
        hipLaunchKernelGGL(k_jacobi_fused2_batch, (unsigned)(per * NXCD), CG_T, 0, st, a.insts, a.jtiles, a.njt, per,
                           a.flagA, a.flagB, a.om, a.nsw);
      }
      break;
    case BatchOp::JacobiCopy:
      hipLaunchKernelGGL((k_jacobi_copy_batch<D>), a.nct, CG_T, 0, st, a.insts, a.ctiles);
      break;
    case BatchOp::UReset:
      hipLaunchKernelGGL((k_ureset_batch<D, T>), a.nct, 256, 0, st, a.insts, a.ctiles);
      break;
    case BatchOp::StepEnd:
      hipLaunchKernelGGL(k_step_end, (a.ninst + 63) / 64, 64, 0, st, a.insts, a.ninst, a.step);
      break;
    case BatchOp::Pending:
      hipLaunchKernelGGL(k_cg_pending, (a.ninst + 63) / 64, 64, 0, st, a.insts, a.ninst, a.pending);
      break;
  }
}

void launch_batch(int D, int prec, BatchOp op, const BatchArgs &a) {
  if (D == 2) {
    if (prec) batch_kernels_t<2, double>(op, a);
    else batch_kernels_t<2, float>(op, a);
  } else {
    if (prec) batch_kernels_t<3, double>(op, a);
    else batch_kernels_t<3, float>(op, a);
  }
}

int ensure_cg(tlvlbm_ctx *c) {
  if (c->D == 2) return c->prec ? cg_alloc<2, double>(c) : cg_alloc<2, float>(c);
  return c->prec ? cg_alloc<3, double>(c) : cg_alloc<3, float>(c);
}

}  // namespace tl

// --------------------------------------------- allocation-free link table
// tlvlbm_cut_links_noalloc: the cut-link table of a level set without any
// device allocation.  Its workspace (per-identifier link histogram, error
// flag, chunk totals of the prefix scan) is one fixed device array of the
// library, `scratch`, held by every GPU the library runs on until the
// process ends; the activity test phi <= 0 is evaluated where needed, so no
// node-sized buffer exists.  Host code reaches the array only through the
// address hipGetSymbolAddress returns on each device.

namespace tl {
namespace {

constexpr int NA_CHUNKS = 8192;  // chunk totals: at most NA_CHUNKS * SCAN_CH nodes
constexpr size_t NA_TOT = 0, NA_GRAND = NA_TOT + sizeof(int64_t) * NA_CHUNKS, NA_HIST = NA_GRAND + 256,
                 NA_FLAG = NA_HIST + 256 * sizeof(unsigned), NA_BYTES = NA_FLAG + 256;
constexpr int NA_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

std::mutex na_mutex;
void *na_ptr[NA_MAX_DEVICES] = {nullptr};

// the array's address on the current device (looked up once per device)
hipError_t na_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NA_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(na_mutex);
  if (!na_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    na_ptr[dev] = p;
  }
  *out = na_ptr[dev];
  return hipSuccess;
}

__device__ __forceinline__ bool na_active(const double *__restrict__ phi, int64_t i) { return phi[i] <= 0.0; }

__global__ void k_na_clear(unsigned *hist, int *flag) {
  hist[threadIdx.x] = 0u;
  if (threadIdx.x == 0) *flag = 0;
}

// every lattice neighbour of an active node must exist; cut links per bid
template <int D>
__global__ void k_na_hist(Geo g, const double *__restrict__ phi, const uint8_t *__restrict__ bid, int *flag,
                          unsigned *hist) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N || !na_active(phi, i)) return;
  const C3 c = coords_of(g, i);
  for (int q = 0; q < 2 * D; ++q) {
    const int64_t o = node_dir(g, c, q, 1);
    if (o < 0) {
      atomicOr(flag, FLAG_ARG);
      return;
    }
    if (!na_active(phi, o)) atomicAdd(&hist[bid ? bid[o] : 0], 1u);
  }
}

// cut links of node i whose outside node carries identifier b
template <int D>
__device__ __forceinline__ int na_count(const Geo &g, const double *__restrict__ phi, const uint8_t *__restrict__ bid,
                                        int b, int64_t i) {
  if (i >= g.N || !na_active(phi, i)) return 0;
  const C3 c = coords_of(g, i);
  int k = 0;
  for (int q = 0; q < 2 * D; ++q) {
    const int64_t o = node_dir(g, c, q, 1);
    if (o >= 0 && !na_active(phi, o) && (bid ? bid[o] : 0) == b) ++k;
  }
  return k;
}

// link count of every chunk of SCAN_CH nodes
template <int D>
__global__ __launch_bounds__(SCAN_T) void k_na_chunk(Geo g, const double *__restrict__ phi,
                                                     const uint8_t *__restrict__ bid, int b, int64_t *tot) {
  __shared__ int64_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH + threadIdx.x * SCAN_V;
  int64_t s = 0;
  for (int k = 0; k < SCAN_V; ++k) s += na_count<D>(g, phi, bid, b, base + k);
  int64_t total;
  block_excl_scan(s, sh, total);
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// records of identifier b in (node, q) order: chunk offset (scanned totals)
// plus the block-local exclusive scan of the per-thread counts
template <int D>
__global__ __launch_bounds__(SCAN_T) void k_na_scatter(Geo g, const double *__restrict__ phi,
                                                       const uint8_t *__restrict__ bid, int b,
                                                       const int64_t *__restrict__ tot, int64_t base_out, int64_t cap,
                                                       int64_t *__restrict__ node, int32_t *__restrict__ qo,
                                                       int32_t *__restrict__ bo) {
  __shared__ int64_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH + threadIdx.x * SCAN_V;
  int cnt[SCAN_V];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_V; ++k) {
    cnt[k] = na_count<D>(g, phi, bid, b, base + k);
    s += cnt[k];
  }
  int64_t total;
  int64_t ex = block_excl_scan(s, sh, total) + tot[blockIdx.x] + base_out;
  for (int k = 0; k < SCAN_V; ++k) {
    if (!cnt[k]) continue;
    const int64_t i = base + k;
    const C3 c = coords_of(g, i);
    for (int q = 0; q < 2 * D; ++q) {
      const int64_t o = node_dir(g, c, q, 1);
      if (o >= 0 && !na_active(phi, o) && (bid ? bid[o] : 0) == b) {
        if (ex < cap) {
          node[ex] = i;
          qo[ex] = q;
          if (bo) bo[ex] = b;
        }
        ++ex;
      }
    }
  }
}

template <int D>
__global__ void k_na_geom(Geo g, const double *__restrict__ phi, int64_t n, const int64_t *__restrict__ node,
                          const int32_t *__restrict__ qo, double *__restrict__ eta, double *__restrict__ Nb) {
  const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= n) return;
  const int64_t m = node[l];
  const int q = qo[l];
  const C3 cm = coords_of(g, m);
  const int64_t o = node_dir(g, cm, q, 1), mb = node_dir(g, cm, q, -1);
  double N[3];
  const double e = link_eta_normal<D>(g, phi, m, o, q, mb, N);
  if (eta) eta[l] = e;
  if (Nb)
    for (int a = 0; a < 3; ++a) Nb[l * 3 + a] = N[a];
}

template <int D>
tlvlbm_status na_links_t(const Geo &g, const double *phi, const uint8_t *bid, int64_t cap, int64_t *node, int32_t *q,
                         double *eta, double *Nb, int32_t *bo, int64_t *n_links, hipStream_t st,
                         unsigned char *ws) {
  int64_t *tot = (int64_t *)(ws + NA_TOT), *grand = (int64_t *)(ws + NA_GRAND);
  unsigned *hist = (unsigned *)(ws + NA_HIST);
  int *flag = (int *)(ws + NA_FLAG);
  const int64_t nb = (g.N + SCAN_CH - 1) / SCAN_CH;
  // the workspace keeps the last call's contents: clear what starts at zero
  hipLaunchKernelGGL(k_na_clear, 1, 256, 0, st, hist, flag);
  hipLaunchKernelGGL((k_na_hist<D>), nblk(g.N, 256), 256, 0, st, g, phi, bid, flag, hist);
  unsigned hh[256];
  int fl = 0;
  if (hipMemcpyAsync(hh, hist, sizeof(hh), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return TLVLBM_ERR_DEVICE;
  if (fl & FLAG_ARG) return TLVLBM_ERR_INVALID_ARG;
  int64_t total = 0;
  for (int b = 0; b < 256; ++b) total += hh[b];
  *n_links = total;
  if (total > cap) return TLVLBM_ERR_INVALID_ARG;
  int64_t base = 0;
  for (int b = 0; b < 256; ++b) {
    if (!hh[b]) continue;
    hipLaunchKernelGGL((k_na_chunk<D>), (unsigned)nb, SCAN_T, 0, st, g, phi, bid, b, tot);
    hipLaunchKernelGGL(k_scan_tot2, 1, SCAN_T, 0, st, tot, nb, grand);
    hipLaunchKernelGGL((k_na_scatter<D>), (unsigned)nb, SCAN_T, 0, st, g, phi, bid, b, tot, base, cap, node, q, bo);
    base += hh[b];
  }
  if (total > 0)
    hipLaunchKernelGGL((k_na_geom<D>), nblk(total, 128), 128, 0, st, g, phi, total, node, q, eta, Nb);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return TLVLBM_ERR_DEVICE;
  return TLVLBM_OK;
}

}  // namespace
}  // namespace tl

extern "C" tlvlbm_status tlvlbm_cut_links_noalloc(const tlvlbm_grid *grid, tlvlbm_lattice lattice, const double *phi,
                                                  const uint8_t *bid, int64_t capacity, int64_t *node, int32_t *q,
                                                  double *eta, double *Nb, int32_t *bid_out, int64_t *n_links,
                                                  void *stream) {
  using namespace tl;
  if (!grid || !phi || !node || !q || !n_links || capacity < 0) return TLVLBM_ERR_INVALID_ARG;
  if (lattice != TLVLBM_D2Q4x6 && lattice != TLVLBM_D3Q6x12) return TLVLBM_ERR_INVALID_ARG;
  *n_links = 0;
  const int D = (int)lattice;
  Geo g{};
  int64_t N = 1;
  for (int a = 0; a < 3; ++a) {
    const int na = a < D ? grid->n[a] : 1;
    if (na < 1) return TLVLBM_ERR_INVALID_ARG;
    N *= na;
  }
  if (!(grid->dx > 0) || N > (int64_t)NA_CHUNKS * SCAN_CH) return TLVLBM_ERR_INVALID_ARG;
  // inputs and outputs in device memory (nothing is staged: staging would allocate)
  for (const void *p : {(const void *)phi, (const void *)bid, (const void *)node, (const void *)q, (const void *)eta,
                        (const void *)Nb, (const void *)bid_out})
    if (p && !is_device_ptr(p)) return TLVLBM_ERR_INVALID_ARG;
  g.nx = grid->n[0];
  g.ny = grid->n[1];
  g.nz = D == 3 ? grid->n[2] : 1;
  g.per = (int)(grid->periodic_mask & ((1u << D) - 1)) | (D == 2 ? 4 : 0);
  g.N = N;
  g.S = N;
  g.dx = grid->dx;
  g.ox = grid->origin[0];
  g.oy = grid->origin[1];
  g.oz = D == 3 ? grid->origin[2] : 0.0;
  void *ws = nullptr;
  if (na_scratch(&ws) != hipSuccess) return TLVLBM_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  return D == 2 ? na_links_t<2>(g, phi, bid, capacity, node, q, eta, Nb, bid_out, n_links, st, (unsigned char *)ws)
                : na_links_t<3>(g, phi, bid, capacity, node, q, eta, Nb, bid_out, n_links, st, (unsigned char *)ws);
}
