// C ABI of the tlvlbm runtime: context lifetime, host/device argument
// marshalling, call-order checks and the step loop of Algorithm 1.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "tl_device.hpp"
#include "tl_internal.hpp"

using namespace tl;

// extra elements between population planes of large grids (tuning knob)
#ifndef TL_PLANE_PAD
#define TL_PLANE_PAD 0
#endif

namespace {

tlvlbm_status fail(tlvlbm_ctx *c, tlvlbm_status s, const char *msg) {
  if (c) {
    try {
      c->err = msg;
    } catch (...) {
    }
  }
  return s;
}

tlvlbm_status dev_fail(tlvlbm_ctx *c, hipError_t e, const char *where) {
  if (c) {
    try {
      c->err = std::string(where) + ": " + hipGetErrorString(e);
    } catch (...) {
    }
  }
  return e == hipErrorOutOfMemory ? TLVLBM_ERR_OUT_OF_MEMORY : TLVLBM_ERR_DEVICE;
}

#define CHK(expr, where)                   \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return dev_fail(c, e_, where); \
  } while (0)

__global__ void k_count_active(const uint8_t *act, int64_t n, unsigned long long *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool a = i < n && act[i];
  const unsigned long long b = __ballot(a);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(out, (unsigned long long)__popcll(b));
}

tlvlbm_status read_flag(tlvlbm_ctx *c) {
  int flag = 0;
  CHK(hipMemcpyAsync(c->h_flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->st), "flag read");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  flag = *c->h_flag;
  if (flag & FLAG_NONFINITE) return fail(c, TLVLBM_ERR_NONFINITE, "non-finite state");
  if (flag & FLAG_J) return fail(c, TLVLBM_ERR_NONPOSITIVE_J, "det F <= 0 at an active node");
  if (flag & FLAG_NEWTON) return fail(c, TLVLBM_ERR_NEWTON, "Neumann normal-image solve left det F_b <= 0");
  return TLVLBM_OK;
}

bool has_neumann(const tlvlbm_ctx *c) {
  for (int b = 0; b < 256; ++b)
    if (c->bid_end[b] > c->bid_begin[b] && c->bcs[b].type == TLVLBM_BC_NEUMANN_TRACTION) return true;
  return false;
}

// launches of one step of Algorithm 1 (no host synchronisation except inside
// the projection's CG convergence polling)
}  // namespace

namespace tl {

// law 0: neo-Hookean; law 1: with fibres (k1 >= 0, a0 not zero); law 2:
// law 1 (or law 0 when k1 = 0) with a Maxwell branch (beta >= 0, tau >= 0)
static bool material_ok(const tlvlbm_material *m) {
  if (!m || m->law < 0 || m->law > 2) return false;
  if (m->law >= 1) {
    const double n = m->a0[0] * m->a0[0] + m->a0[1] * m->a0[1] + m->a0[2] * m->a0[2];
    if (!(m->k1 >= 0) || (m->law == 1 && !(n > 0)) || (m->k1 > 0 && !(n > 0))) return false;
  }
  if (m->law == 2 && (!(m->beta >= 0) || !(m->tau >= 0))) return false;
  return true;
}

static void set_material_par(tlvlbm_ctx *c, const tlvlbm_material *m) {
  Par &p = c->par;
  const int D = c->D;
  p.mu = m->mu;
  p.lam = m->lambda;
  p.k1 = m->law >= 1 ? m->k1 : 0.0;
  double n = 0.0;
  for (int a = 0; a < D; ++a) n += m->a0[a] * m->a0[a];
  for (int a = 0; a < 3; ++a) p.a0[a] = (p.k1 > 0 && a < D) ? m->a0[a] / std::sqrt(n) : 0.0;
  c->visco = m->law == 2;
  c->vbeta = c->visco ? m->beta : 0.0;
  c->vtau = c->visco ? m->tau : 0.0;
  p.hist = nullptr;  // attached by set_state
  p.thf = c->thf;    // the thermal stretch stays with the context
}

// branch constants beta xi and xi^2, xi = exp(-dt / (2 tau)) (tau = 0: 0,
// tau = infinity: 1)
static void set_branch_par(tlvlbm_ctx *c) {
  const double xi = c->visco ? std::exp(-c->par.dt / (2.0 * c->vtau)) : 0.0;
  c->par.vbx = c->vbeta * xi;
  c->par.vxi2 = xi * xi;
}

tlvlbm_status check_flag(tlvlbm_ctx *c) { return read_flag(c); }

hipError_t dmalloc_v(tlvlbm_ctx *c, void **p, size_t bytes) {
  *p = nullptr;
  if (c && c->dev_alloc) {
    *p = c->dev_alloc(bytes ? bytes : 1, c->alloc_user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void dfree(tlvlbm_ctx *c, void *p) {
  if (!p) return;
  if (c && c->dev_alloc) {
    // a caching allocator may hand the block out at once: the context's
    // queued work must be done with it first (hipFree waits by itself)
    (void)hipStreamSynchronize(c->st);
    c->dev_free(p, c->alloc_user);
    return;
  }
  (void)hipFree(p);
}

// stress of the material on the host (the reference state's equilibrium: a
// constant of the stored representation, so the thermal stretch, which may
// change between steps, stays out of it)
static double mat_piola_host(int D, const double *F, const Par &p, double *P) {
  return D == 2 ? mat_piola<2>(F, p, P) : mat_piola<3>(F, p, P);
}

bool is_projection_step(const tlvlbm_ctx *c, int64_t step) {
  return has_neumann(c) && c->proj_every > 0 && (step % c->proj_every == 0);
}

// One step of Algorithm 1.  With a tape, the recovered state, the repaired
// deformation gradient (projection steps) and the displacement seen by the
// cut links are recorded for the reverse mode.
int step_once(tlvlbm_ctx *c, const TapeStep *tp) {
  const double tn = c->step * c->par.dt;
  const bool proj = is_projection_step(c, c->step);
  const size_t plane = (size_t)c->geo.S * c->esz;
  if (proj) {
    int s = run_projection(c, true, tn, tp ? tp->xs[0] : nullptr, tp ? tp->xmode : 0);
    if (s) return s;
    launch_bulk(c, true, tp ? tp->U : nullptr, tp != nullptr);
    if (tp && tp->Fr) {
      if (c->act && c->chunks) launch_tape_gather(c, c->cg.Fr, tp->Fr, c->D * c->D);
      else CHK(hipMemcpyAsync(tp->Fr, c->cg.Fr, (size_t)c->D * c->D * plane, hipMemcpyDeviceToDevice, c->st), "tape");
    }
    s = run_projection(c, false, tn, tp ? tp->xs[1] : nullptr, tp ? tp->xmode : 0);
    if (s) return s;
    ++c->st_proj;
  } else {
    launch_bulk(c, false, tp ? tp->U : nullptr, tp != nullptr);
  }
  if (c->L.n) {
    const int s = launch_cutlinks(c, tn);
    if (s) return s;
  }
  if (tp && tp->u) {
    if (tp->un) {
      if (tp->nu) launch_gather_u(c, tp->un, tp->nu, (double *)tp->u);
    } else {
      CHK(hipMemcpyAsync(tp->u, c->ubuf, (size_t)c->D * c->geo.S * sizeof(double), hipMemcpyDeviceToDevice, c->st),
          "tape");
    }
  }
  std::swap(c->fA, c->fB);
  ++c->step;
  return TLVLBM_OK;
}

}  // namespace tl

extern "C" {

void tlvlbm_default_options(tlvlbm_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->omega = 1.8;
  o->gamma = 0.0;
  o->theta_F = 1.0;
  o->cg_rtol = 0.0;
  o->proj_every = 20;
  o->cg_maxit = 0;
  o->cg_multigrid = 1;
  o->proj_sweeps = 20;
  o->proj_weight = 2.0 / 3.0;
  o->precision = TLVLBM_FP32;
  o->track_u = -1;
  o->stream = nullptr;
}

tlvlbm_status tlvlbm_create(const tlvlbm_grid *grid, tlvlbm_lattice lattice, const tlvlbm_material *mat, double rho0,
                            double dt, const tlvlbm_options *opt, tlvlbm_ctx **out) {
  if (!out) return TLVLBM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!grid || !mat || (lattice != TLVLBM_D2Q4x6 && lattice != TLVLBM_D3Q6x12)) return TLVLBM_ERR_INVALID_ARG;
  if (!(rho0 > 0) || !(dt > 0) || !(grid->dx > 0) || !material_ok(mat)) return TLVLBM_ERR_INVALID_ARG;
  tlvlbm_options o;
  tlvlbm_default_options(&o);
  if (opt) o = *opt;
  if (!(o.omega > 0 && o.omega <= 2) || !(o.theta_F > 0 && o.theta_F <= 1)) return TLVLBM_ERR_INVALID_ARG;
  if (o.precision != TLVLBM_FP32 && o.precision != TLVLBM_FP64) return TLVLBM_ERR_INVALID_ARG;
  if (o.proj_sweeps < 0 || !(o.proj_weight > 0 && o.proj_weight <= 1)) return TLVLBM_ERR_INVALID_ARG;
  if (!o.dev_alloc != !o.dev_free) return TLVLBM_ERR_INVALID_ARG;
  const int D = (int)lattice;
  int64_t N = 1;
  for (int a = 0; a < 3; ++a) {
    const int na = a < D ? grid->n[a] : 1;
    if (na < 1) return TLVLBM_ERR_INVALID_ARG;
    N *= na;
  }
  if (N >= (int64_t(1) << 31)) return TLVLBM_ERR_INVALID_ARG;
  tlvlbm_ctx *c = new (std::nothrow) tlvlbm_ctx();
  if (!c) return TLVLBM_ERR_OUT_OF_MEMORY;
  c->D = D;
  c->Q = 2 * D;
  c->M = D + D * D;
  c->prec = o.precision;
  c->esz = o.precision ? 8 : 4;
  c->geo.nx = grid->n[0];
  c->geo.ny = grid->n[1];
  c->geo.nz = D == 3 ? grid->n[2] : 1;
  c->geo.per = (int)(grid->periodic_mask & ((1u << D) - 1)) | (D == 2 ? 4 : 0);
  c->geo.N = N;
  // plane stride: whole 256-element rows, plus TL_PLANE_PAD elements on large
  // grids (measured on MI355X at 256^3: no padding is fastest)
  int64_t S = (N + 255) / 256 * 256;
  if (S >= (int64_t(1) << 20)) S += TL_PLANE_PAD;
  c->geo.S = S;
  c->geo.dx = grid->dx;
  c->geo.ox = grid->origin[0];
  c->geo.oy = grid->origin[1];
  c->geo.oz = D == 3 ? grid->origin[2] : 0.0;
  set_material_par(c, mat);
  for (int k = 0; k < 9; ++k) {
    c->par.Fref[k] = (k < D * D && k % (D + 1) == 0) ? 1.0 : 0.0;
    c->par.Pref[k] = 0.0;
  }
  c->par.inv_rho0 = 1.0 / rho0;
  c->par.dt = dt;
  c->par.c = grid->dx / dt;
  set_branch_par(c);
  c->par.omega = o.omega;
  c->par.gamma = o.gamma;
  c->theta = o.theta_F;
  c->cg_rtol = o.cg_rtol;
  c->proj_every = o.proj_every;
  c->cg_maxit = o.cg_maxit;
  c->cg_multigrid = o.cg_multigrid ? 1 : 0;
  c->proj_sweeps = o.proj_sweeps;
  c->proj_weight = o.proj_weight;
  c->track_opt = o.track_u;
  c->track_u = o.track_u == 1;
  c->st = (hipStream_t)o.stream;
  c->dev_alloc = o.dev_alloc;
  c->dev_free = o.dev_free;
  c->alloc_user = o.alloc_user;
  const size_t fb = (size_t)c->Q * c->M * (size_t)S * c->esz;
  if (dmalloc(c, &c->fA, fb) != hipSuccess || dmalloc(c, &c->fB, fb) != hipSuccess ||
      dmalloc(c, &c->d_flag, sizeof(int)) != hipSuccess ||
      dmalloc(c, &c->d_newton_fail, sizeof(int64_t)) != hipSuccess ||
      hipHostMalloc((void **)&c->h_flag, sizeof(int)) != hipSuccess ||
      hipHostMalloc((void **)&c->hscal, 64 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    tlvlbm_destroy(c);
    return TLVLBM_ERR_OUT_OF_MEMORY;
  }
  if (hipMemsetAsync(c->d_flag, 0, sizeof(int), c->st) != hipSuccess ||
      hipMemsetAsync(c->d_newton_fail, 0, sizeof(int64_t), c->st) != hipSuccess) {
    tlvlbm_destroy(c);
    return TLVLBM_ERR_DEVICE;
  }
  c->nactive = N;
  *out = c;
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_destroy(tlvlbm_ctx *c) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  if (c->st) (void)hipStreamSynchronize(c->st);
  else (void)hipDeviceSynchronize();
  void *ptrs[] = {c->fA, c->fB, c->ustar, c->ubuf, c->act, c->d_flag, c->d_newton_fail, c->L.node, c->L.out,
                  c->L.mminus, c->L.q, c->L.bid, c->L.npts, c->L.basis, c->L.eta, c->L.Nb, c->L.Xb, c->L.tang,
                  c->L.sidx, c->L.sw, c->cg.x, c->cg.r, c->cg.p0, c->cg.p1, c->cg.Ap, c->cg.b, c->cg.V, c->cg.Fm,
                  c->cg.Fr, c->cg.anc_n, c->cg.anc_i, c->cg.anc_s, c->cg.partial, c->cg.scal, c->cg.z, c->cg.tiles,
                  c->cg.jt, c->cg.nbm, c->bf, c->chunks, c->cpos, c->d_bcs, c->hist, c->thf};
  for (void *p : ptrs)
    if (p) dfree(c, p);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  if (c->hscal) (void)hipHostFree(c->hscal);
  proj_aux_free(c);
  if (c->arena) {
    for (void *q : c->arena->blk)
      if (q) dfree(c, q);
    delete c->arena;
  }
  delete c->rec;
  delete c;
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_set_levelset(tlvlbm_ctx *c, const double *phi, const uint8_t *bid) {
  if (!c || !phi) return TLVLBM_ERR_INVALID_ARG;
  rec_invalidate(c);
  try {
    if (c->has_ls) return fail(c, TLVLBM_ERR_CALL_ORDER, "level set already set");
    const int64_t N = c->geo.N;
    DevIn dphi, dbid;
    CHK(dphi.take(phi, N * sizeof(double), c->st), "phi upload");
    CHK(dbid.take(bid, N, c->st), "bid upload");
    CHK(dmalloc(c, &c->act, N), "mask alloc");
    std::string err;
    int s = build_links(c, (const double *)dphi.ptr, (const uint8_t *)dbid.ptr, err);
    if (s) return fail(c, (tlvlbm_status)s, err.c_str());
    unsigned long long *cnt = nullptr;
    CHK(dmalloc(c, &cnt, sizeof(unsigned long long)), "count alloc");
    CHK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), c->st), "count clear");
    hipLaunchKernelGGL(k_count_active, (unsigned)((N + 255) / 256), 256, 0, c->st, c->act, N, cnt);
    unsigned long long na = 0;
    CHK(hipMemcpyAsync(&na, cnt, sizeof(na), hipMemcpyDeviceToHost, c->st), "count read");
    CHK(hipStreamSynchronize(c->st), "synchronize");
    dfree(c, cnt);
    c->nactive = (int64_t)na;
    {
      // CHUNK-node chunks holding active nodes, in node order
      std::vector<uint8_t> act(N);
      CHK(hipMemcpy(act.data(), c->act, N, hipMemcpyDeviceToHost), "mask read");
      std::vector<int32_t> ch;
      c->first_active = 0;
      for (int64_t i = 0; i < N; ++i)
        if (act[i]) {
          c->first_active = i;
          break;
        }
      for (int64_t k = 0; k * CHUNK < N; ++k) {
        bool any = false;
        for (int64_t i = k * CHUNK; i < std::min<int64_t>(N, k * CHUNK + CHUNK) && !any; ++i) any = act[i] != 0;
        if (any) ch.push_back((int32_t)k);
      }
      if (!ch.empty()) {
        CHK(dmalloc(c, &c->chunks, ch.size() * sizeof(int32_t)), "chunk alloc");
        CHK(hipMemcpy(c->chunks, ch.data(), ch.size() * sizeof(int32_t), hipMemcpyHostToDevice), "chunk upload");
        std::vector<int32_t> pos((size_t)((N + CHUNK - 1) / CHUNK), -1);
        for (size_t k = 0; k < ch.size(); ++k) pos[ch[k]] = (int32_t)k;
        CHK(dmalloc(c, &c->cpos, pos.size() * sizeof(int32_t)), "chunk position alloc");
        CHK(hipMemcpy(c->cpos, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice), "chunk position upload");
      }
      c->nchunks = (int)ch.size();
    }
    c->has_ls = true;
    c->have_state = false;
    if (c->track_opt == -1) c->track_u = true;
    return TLVLBM_OK;
  } catch (...) {
    return fail(c, TLVLBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

tlvlbm_status tlvlbm_set_boundary(tlvlbm_ctx *c, uint8_t bid, const tlvlbm_bc *bc) {
  if (!c || !bc) return TLVLBM_ERR_INVALID_ARG;
  rec_invalidate(c);
  if (bc->type != TLVLBM_BC_DIRICHLET_VELOCITY && bc->type != TLVLBM_BC_NEUMANN_TRACTION)
    return fail(c, TLVLBM_ERR_INVALID_ARG, "unknown boundary type");
  if (bc->ramp < 0 || bc->ramp > 3 || (bc->ramp != TLVLBM_RAMP_CONST && !(bc->T_r > 0)))
    return fail(c, TLVLBM_ERR_INVALID_ARG, "bad ramp");
  BC &b = c->bcs[bid];
  b.type = bc->type;
  b.ramp = bc->ramp;
  b.disp = bc->given_as_displacement ? 1 : 0;
  b.Tr = bc->T_r;
  for (int k = 0; k < 3; ++k) {
    b.a[k] = bc->a[k];
    b.X0[k] = bc->X0[k];
  }
  for (int k = 0; k < 9; ++k) b.G[k] = bc->G[k];
  b.pr = bc->p_radial;
  b.pn = bc->p_normal;
  if (bc->twist != 0.0 && !(bc->type == TLVLBM_BC_DIRICHLET_VELOCITY && bc->given_as_displacement))
    return fail(c, TLVLBM_ERR_INVALID_ARG, "twist needs a displacement-given Dirichlet condition");
  b.tw = bc->twist;
  c->bc_set[bid] = true;
  c->bcs_dirty = true;
  c->aux_stale = true;  // projection anchors and components follow the conditions
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_set_body_force(tlvlbm_ctx *c, const double *g, int32_t ramp, double T_r) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  rec_invalidate(c);
  if (ramp < 0 || ramp > 3 || (ramp != TLVLBM_RAMP_CONST && !(T_r > 0)))
    return fail(c, TLVLBM_ERR_INVALID_ARG, "bad ramp");
  try {
    if (!g) {
      dfree(c, c->bf);
      c->bf = nullptr;
      return TLVLBM_OK;
    }
    const size_t plane = (size_t)c->geo.S * c->esz;
    if (!c->bf) {
      CHK(dmalloc(c, &c->bf, (size_t)c->D * plane), "body force alloc");
      CHK(hipMemsetAsync(c->bf, 0, (size_t)c->D * plane, c->st), "body force clear");
    }
    DevIn dg;
    CHK(dg.take(g, (size_t)c->D * c->geo.N * sizeof(double), c->st), "body force upload");
    launch_planes_in(c, (const double *)dg.ptr, c->bf, c->D);
    CHK(hipGetLastError(), "body force convert");
    CHK(hipStreamSynchronize(c->st), "body force");
    c->bf_ramp = ramp;
    c->bf_Tr = T_r;
    return TLVLBM_OK;
  } catch (...) {
    return fail(c, TLVLBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

tlvlbm_status tlvlbm_set_thermal_stretch(tlvlbm_ctx *c, const double *th) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  rec_invalidate(c);
  try {
    if (!th) {
      dfree(c, c->thf);
      c->thf = nullptr;
      c->par.thf = nullptr;
      return TLVLBM_OK;
    }
    if (c->visco) return fail(c, TLVLBM_ERR_INVALID_ARG, "a thermal stretch does not combine with a Maxwell branch");
    const int64_t N = c->geo.N;
    std::vector<double> h((size_t)N);
    CHK(hipMemcpyAsync(h.data(), th, (size_t)N * sizeof(double), hipMemcpyDefault, c->st), "thermal stretch read");
    CHK(hipStreamSynchronize(c->st), "synchronize");
    for (int64_t i = 0; i < N; ++i)
      if (!(h[i] > 0.0) || !std::isfinite(h[i]))
        return fail(c, TLVLBM_ERR_INVALID_ARG, "the thermal stretch must be positive and finite at every node");
    if (!c->thf) CHK(dmalloc(c, &c->thf, (size_t)c->geo.S * sizeof(double)), "thermal stretch alloc");
    CHK(hipMemcpyAsync(c->thf, h.data(), (size_t)N * sizeof(double), hipMemcpyHostToDevice, c->st),
        "thermal stretch upload");
    CHK(hipStreamSynchronize(c->st), "synchronize");
    c->par.thf = c->thf;
    return TLVLBM_OK;
  } catch (...) {
    return fail(c, TLVLBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

tlvlbm_status tlvlbm_set_material(tlvlbm_ctx *c, const tlvlbm_material *m) {
  if (!c || !material_ok(m)) return TLVLBM_ERR_INVALID_ARG;
  if (m->law == 2 && c->thf) return fail(c, TLVLBM_ERR_INVALID_ARG, "a Maxwell branch does not combine with a thermal stretch");
  rec_invalidate(c);
  // a Maxwell branch (before or after) starts its history at set_state
  if (c->visco || m->law == 2) {
    c->have_state = false;
    c->hist_set = false;
  }
  set_material_par(c, m);
  set_branch_par(c);
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_set_state(tlvlbm_ctx *c, const double *U0, const double *u0, const double *dU0) {
  if (!c || !U0) return TLVLBM_ERR_INVALID_ARG;
  rec_invalidate(c);
  try {
    if (!c->has_ls)
      for (int a = 0; a < c->D; ++a)
        if (!((c->geo.per >> a) & 1))
          return fail(c, TLVLBM_ERR_INVALID_ARG, "without a level set every axis must be periodic");
    for (int b = 0; b < 256; ++b)
      if (c->bid_end[b] > c->bid_begin[b] && !c->bc_set[b])
        return fail(c, TLVLBM_ERR_CALL_ORDER, "a boundary identifier with cut links has no condition");
    if (has_neumann(c) && !c->track_u)
      return fail(c, TLVLBM_ERR_INVALID_ARG, "Neumann links need the displacement quadrature (track_u)");
    const int64_t N = c->geo.N, S = c->geo.S;
    const int D = c->D, M = c->M;
    if (c->track_u && !c->ustar) {
      CHK(dmalloc(c, &c->ustar, (size_t)D * S * sizeof(double)), "u* alloc");
      CHK(dmalloc(c, &c->ubuf, (size_t)D * S * sizeof(double)), "u alloc");
      CHK(hipMemsetAsync(c->ubuf, 0, (size_t)D * S * sizeof(double), c->st), "u clear");
    }
    // the Maxwell branch's history (the initialisation starts it at F0)
    c->par.hist = nullptr;
    if (c->visco) {
      if (!c->hist) CHK(dmalloc(c, &c->hist, (size_t)(D * (D + 1) / 2) * S * sizeof(double)), "history alloc");
      c->par.hist = c->hist;
      c->hist_set = true;  // the initialisation writes it
    }
    DevIn dU, du, ddU;
    CHK(dU.take(U0, (size_t)M * N * sizeof(double), c->st), "U0 upload");
    CHK(du.take(u0, (size_t)D * N * sizeof(double), c->st), "u0 upload");
    CHK(ddU.take(dU0, (size_t)D * M * N * sizeof(double), c->st), "dU0 upload");
    // reference state of the stored populations: (0, F0) at the first active
    // node, with its stress under the current material
    {
      double Fr[9] = {0.0}, Pr[9] = {0.0};
      CHK(hipMemcpy2DAsync(Fr, sizeof(double), (const double *)dU.ptr + (size_t)D * N + c->first_active,
                           (size_t)N * sizeof(double), sizeof(double), (size_t)D * D, hipMemcpyDeviceToHost, c->st),
          "reference state read");
      CHK(hipStreamSynchronize(c->st), "synchronize");
      bool ok = true;
      for (int k = 0; k < D * D; ++k) ok = ok && std::isfinite(Fr[k]);
      const double J = ok ? mat_piola_host(D, Fr, c->par, Pr) : 0.0;
      if (!(J > 0.0) || !std::isfinite(J)) {
        for (int k = 0; k < D * D; ++k) {
          Fr[k] = (k % (D + 1) == 0) ? 1.0 : 0.0;
          Pr[k] = 0.0;
        }
      }
      for (int k = 0; k < 9; ++k) {
        c->par.Fref[k] = k < D * D ? Fr[k] : 0.0;
        c->par.Pref[k] = k < D * D ? Pr[k] * c->par.inv_rho0 : 0.0;
      }
    }
    const size_t fb = (size_t)c->Q * M * (size_t)S * c->esz;
    CHK(hipMemsetAsync(c->fB, 0, fb, c->st), "population clear");
    CHK(hipMemsetAsync(c->fA, 0, fb, c->st), "population clear");
    CHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->st), "flag clear");
    c->step = 0;  // the initial state is at t = 0 (body acceleration b(X, 0))
    launch_init(c, (const double *)dU.ptr, (const double *)du.ptr, (const double *)ddU.ptr);
    CHK(hipGetLastError(), "init launch");
    tlvlbm_status s = read_flag(c);
    if (s) return s;
    // host-side preparation of the projection (tiles, components, multigrid
    // hierarchy) happens here, not inside the first projection step
    if (has_neumann(c) && c->proj_every > 0 && (!c->gauge || c->aux_stale)) {
      int e = ensure_cg(c);
      if (!e) e = proj_aux_build(c);
      if (e) return fail(c, (tlvlbm_status)e, "projection setup failed");
    }
    c->step = 0;
    c->status = TLVLBM_OK;
    c->have_state = true;
    c->fresh = true;
    return TLVLBM_OK;
  } catch (...) {
    return fail(c, TLVLBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

tlvlbm_status tlvlbm_step(tlvlbm_ctx *c, int64_t n) {
  if (!c || n < 0) return TLVLBM_ERR_INVALID_ARG;
  if (!c->have_state) return fail(c, TLVLBM_ERR_CALL_ORDER, "step before set_state");
  if (c->status) return (tlvlbm_status)c->status;
  if (n > 0) rec_invalidate(c);
  for (int64_t k = 0; k < n; ++k) {
    c->fresh = false;
    const int s = step_once(c);
    if (s) return (tlvlbm_status)(c->status = s);
  }
  CHK(hipGetLastError(), "step launch");
  tlvlbm_status s = read_flag(c);
  c->status = s;
  return s;
}

tlvlbm_status tlvlbm_step_each(tlvlbm_ctx *const *ctxs, int32_t nctx, int64_t n) {
  if (!ctxs || nctx < 1 || n < 0) return TLVLBM_ERR_INVALID_ARG;
  for (int i = 0; i < nctx; ++i) {
    if (!ctxs[i]) return TLVLBM_ERR_INVALID_ARG;
    rec_invalidate(ctxs[i]);
    if (!ctxs[i]->have_state) return fail(ctxs[i], TLVLBM_ERR_CALL_ORDER, "step before set_state");
    if (ctxs[i]->status) return (tlvlbm_status)ctxs[i]->status;
  }
  for (int64_t k = 0; k < n; ++k)
    for (int i = 0; i < nctx; ++i) {
      ctxs[i]->fresh = false;
      const int s = step_once(ctxs[i]);
      if (s) return (tlvlbm_status)(ctxs[i]->status = s);
    }
  tlvlbm_status worst = TLVLBM_OK;
  for (int i = 0; i < nctx; ++i) {
    tlvlbm_ctx *c = ctxs[i];
    CHK(hipGetLastError(), "step launch");
    const tlvlbm_status s = read_flag(c);
    c->status = s;
    if (s) worst = s;
  }
  return worst;
}

tlvlbm_status tlvlbm_moments(tlvlbm_ctx *c, double *U_out, double *u_out, double *J_out) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  if (!c->have_state) return fail(c, TLVLBM_ERR_CALL_ORDER, "moments before set_state");
  const int64_t N = c->geo.N;
  DevOut U, u, J;
  CHK(U.take(U_out, (size_t)c->M * N * sizeof(double)), "U alloc");
  CHK(u.take(u_out, (size_t)c->D * N * sizeof(double)), "u alloc");
  CHK(J.take(J_out, (size_t)N * sizeof(double)), "J alloc");
  if (u.ptr && !c->track_u) CHK(hipMemsetAsync(u.ptr, 0, (size_t)c->D * N * sizeof(double), c->st), "u clear");
  launch_pull_moments(c, (double *)U.ptr, c->track_u ? (double *)u.ptr : nullptr, (double *)J.ptr, false);
  CHK(hipGetLastError(), "moments launch");
  CHK(U.finish(c->st), "U copy");
  CHK(u.finish(c->st), "u copy");
  CHK(J.finish(c->st), "J copy");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_moments_native(tlvlbm_ctx *c, void *U_out, double *u_out, void *J_out) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  if (!c->have_state) return fail(c, TLVLBM_ERR_CALL_ORDER, "moments before set_state");
  const int64_t N = c->geo.N;
  DevOut U, u, J;
  CHK(U.take(U_out, (size_t)c->M * N * c->esz), "U alloc");
  CHK(u.take(u_out, (size_t)c->D * N * sizeof(double)), "u alloc");
  CHK(J.take(J_out, (size_t)N * c->esz), "J alloc");
  if (u.ptr && !c->track_u) CHK(hipMemsetAsync(u.ptr, 0, (size_t)c->D * N * sizeof(double), c->st), "u clear");
  launch_moments_native(c, U.ptr, c->track_u ? (double *)u.ptr : nullptr, J.ptr);
  CHK(hipGetLastError(), "moments launch");
  CHK(U.finish(c->st), "U copy");
  CHK(u.finish(c->st), "u copy");
  CHK(J.finish(c->st), "J copy");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_stress(tlvlbm_ctx *c, double *P_out, double *sigma_out) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  if (!c->have_state) return fail(c, TLVLBM_ERR_CALL_ORDER, "stress before set_state");
  const int64_t N = c->geo.N;
  const size_t bytes = (size_t)c->D * c->D * N * sizeof(double);
  DevOut P, S;
  CHK(P.take(P_out, bytes), "P alloc");
  CHK(S.take(sigma_out, bytes), "sigma alloc");
  launch_stress(c, (double *)P.ptr, (double *)S.ptr);
  CHK(hipGetLastError(), "stress launch");
  CHK(P.finish(c->st), "P copy");
  CHK(S.finish(c->st), "sigma copy");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_get_state(tlvlbm_ctx *c, double *f, double *ustar, int64_t *step) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  if (!c->have_state) return fail(c, TLVLBM_ERR_CALL_ORDER, "get_state before set_state");
  const int64_t N = c->geo.N;
  DevOut F, U;
  CHK(F.take(f, (size_t)c->Q * c->M * N * sizeof(double)), "f alloc");
  CHK(U.take(ustar, (size_t)c->D * N * sizeof(double)), "u* alloc");
  launch_get_f(c, (double *)F.ptr, (double *)U.ptr);
  CHK(hipGetLastError(), "get_state launch");
  CHK(F.finish(c->st), "f copy");
  CHK(U.finish(c->st), "u* copy");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  if (step) *step = c->step;
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_get_history(tlvlbm_ctx *c, double *R) {
  if (!c || !R) return TLVLBM_ERR_INVALID_ARG;
  if (!c->visco) return fail(c, TLVLBM_ERR_INVALID_ARG, "get_history: the material has no Maxwell branch");
  if (!c->hist_set) return fail(c, TLVLBM_ERR_CALL_ORDER, "get_history before set_state or put_history");
  const int64_t N = c->geo.N, S = c->geo.S;
  const int K = c->D * (c->D + 1) / 2;
  CHK(hipMemcpy2DAsync(R, (size_t)N * sizeof(double), c->hist, (size_t)S * sizeof(double), (size_t)N * sizeof(double),
                       (size_t)K, hipMemcpyDefault, c->st),
      "history copy");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_put_history(tlvlbm_ctx *c, const double *R) {
  if (!c || !R) return TLVLBM_ERR_INVALID_ARG;
  if (!c->visco) return fail(c, TLVLBM_ERR_INVALID_ARG, "put_history: the material has no Maxwell branch");
  rec_invalidate(c);
  const int64_t N = c->geo.N, S = c->geo.S;
  const int K = c->D * (c->D + 1) / 2;
  if (!c->hist) CHK(dmalloc(c, &c->hist, (size_t)K * S * sizeof(double)), "history alloc");
  CHK(hipMemcpy2DAsync(c->hist, (size_t)S * sizeof(double), R, (size_t)N * sizeof(double), (size_t)N * sizeof(double),
                       (size_t)K, hipMemcpyDefault, c->st),
      "history copy");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  c->par.hist = c->hist;
  c->hist_set = true;
  c->fresh = false;
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_put_state(tlvlbm_ctx *c, const double *f, const double *ustar, int64_t step) {
  if (!c || !f || step < 0) return TLVLBM_ERR_INVALID_ARG;
  if (c->visco && !c->hist_set)
    return fail(c, TLVLBM_ERR_CALL_ORDER, "put_state: a Maxwell branch needs its history first (put_history)");
  rec_invalidate(c);
  {
    const int64_t N = c->geo.N;
    if (c->track_u && !c->ustar) {
      CHK(dmalloc(c, &c->ustar, (size_t)c->D * c->geo.S * sizeof(double)), "u* alloc");
      CHK(dmalloc(c, &c->ubuf, (size_t)c->D * c->geo.S * sizeof(double)), "u alloc");
      CHK(hipMemsetAsync(c->ubuf, 0, (size_t)c->D * c->geo.S * sizeof(double), c->st), "u clear");
    }
    DevIn F, U;
    CHK(F.take(f, (size_t)c->Q * c->M * N * sizeof(double), c->st), "f upload");
    CHK(U.take(ustar, (size_t)c->D * N * sizeof(double), c->st), "u* upload");
    launch_put_f(c, (const double *)F.ptr, (const double *)U.ptr);
    CHK(hipGetLastError(), "put_state launch");
    CHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->st), "flag clear");
    CHK(hipStreamSynchronize(c->st), "synchronize");
  }
  c->fresh = false;
  c->step = step;
  c->status = TLVLBM_OK;
  c->have_state = true;
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_get_links(tlvlbm_ctx *c, int64_t *node, int32_t *q, double *eta, double *Nb, int32_t *bid) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  const size_t n = (size_t)c->L.n;
  if (!n) return TLVLBM_OK;
  struct Item {
    void *dst;
    const void *src;
    size_t bytes;
  } items[] = {{node, c->L.node, n * 8}, {q, c->L.q, n * 4}, {eta, c->L.eta, n * 8}, {Nb, c->L.Nb, n * 24},
               {bid, c->L.bid, n * 4}};
  for (auto &it : items)
    if (it.dst) CHK(hipMemcpyAsync(it.dst, it.src, it.bytes, hipMemcpyDefault, c->st), "link copy");
  CHK(hipStreamSynchronize(c->st), "synchronize");
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_stats(tlvlbm_ctx *c, tlvlbm_stats_t *o) {
  if (!c || !o) return TLVLBM_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->active_nodes = c->nactive;
  o->cut_links = c->L.n;
  for (int b = 0; b < 256; ++b) {
    const int64_t k = c->bid_end[b] - c->bid_begin[b];
    if (k <= 0) continue;
    if (c->bcs[b].type == TLVLBM_BC_NEUMANN_TRACTION) o->neumann_links += k;
    else if (c->bcs[b].type == TLVLBM_BC_DIRICHLET_VELOCITY) o->dirichlet_links += k;
  }
  o->cg_iterations = c->st_cg;
  o->projections = c->st_proj;
  o->step = c->step;
  int64_t nf = 0;
  if (hipMemcpy(&nf, c->d_newton_fail, sizeof(nf), hipMemcpyDeviceToHost) != hipSuccess)
    return TLVLBM_ERR_DEVICE;
  o->newton_failures = nf;
  if (c->L.n) {
    std::vector<int32_t> basis(c->L.n);
    if (hipMemcpy(basis.data(), c->L.basis, c->L.n * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return TLVLBM_ERR_DEVICE;
    for (int32_t b : basis) o->lsq_linear_fallbacks += (b == 1);
  }
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_synchronize(tlvlbm_ctx *c) {
  if (!c) return TLVLBM_ERR_INVALID_ARG;
  CHK(hipStreamSynchronize(c->st), "synchronize");
  return TLVLBM_OK;
}

const char *tlvlbm_last_error(const tlvlbm_ctx *c) {
  if (!c) return "null context";
  return c->err.c_str();
}

size_t tlvlbm_population_bytes(const tlvlbm_ctx *c) {
  if (!c) return 0;
  return (size_t)c->Q * c->M * (size_t)c->geo.N * c->esz;
}

}  // extern "C"
