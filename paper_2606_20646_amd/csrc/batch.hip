// Batched launch of many independent TL-VLBM instances (project extension):
// every phase of Algorithm 1 runs as one tile-list kernel over all instances,
// the projection's Jacobi sweeps run over all instances at once (the exact
// mode's CG keeps per-instance scalars with segmented reductions), and
// stretches of steps without projection are replayed from a hipGraph.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tl_internal.hpp"

using namespace tl;

struct tlvlbm_batch {
  std::vector<tlvlbm_ctx *> c;
  int D = 0, prec = 0, proj_every = 0;
  int sweeps = 0;       // projection: damped Jacobi sweeps (0: CG)
  double jw = 0.0;      // Jacobi weight
  hipStream_t st = nullptr;
  std::vector<Inst> h_inst;
  Inst *d_inst = nullptr;
  int4 *d_btiles = nullptr, *d_ctiles = nullptr, *d_ltiles = nullptr;
  int nbt = 0, nct = 0, nlt = 0;
  // 2D: tiles (instance, tx, ty) of the fused Jacobi sweeps (none: one
  // launch per sweep)
  int4 *d_jtiles = nullptr;
  int njt = 0;
  // node-kernel tiles: spans of tw nodes of an instance's node order (aligned
  // to tw) holding active nodes, in order
  // `torder` (0: instance by instance, 1: round robin over the instances);
  // chosen by batch_autotune
  int tw = 256, torder = 0;
  double tune_ms[2][3] = {};
  std::vector<std::vector<uint8_t>> act;  // host copies of the activity masks
  Seg *d_segs = nullptr;
  int64_t *d_step = nullptr;
  int *d_pending = nullptr, *h_pending = nullptr;
  int *h_flags = nullptr;
  bool any_neu = false, any_dir = false;
  // bulk update of the batch: 0 neo-Hookean, 1 reinforced (an instance has
  // fibres or a body acceleration), 2 thermal stretch (an instance has a
  // field; it covers both), 3 Maxwell branch (an instance has one; it covers
  // 1, not 2: a batch with both is refused)
  int law = 0;
  int64_t step = 0, maxit = 0;
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  int glen = 0;
  // a whole projection cycle (projection step + proj_every - 1 plain steps)
  // captured once, in the Jacobi mode (no host decisions inside it)
  hipGraphExec_t gcycle = nullptr;
  bool capturing = false;
  bool use_mg = false;  // every instance has a multigrid hierarchy: batched V-cycles
  BatchMG bmg;
  std::string err;
};

namespace {

tlvlbm_status bfail(tlvlbm_batch *b, tlvlbm_status s, const char *m) {
  if (b) {
    try {
      b->err = m;
    } catch (...) {
    }
  }
  return s;
}

#define BCHK(expr, what)                                                 \
  do {                                                                   \
    if ((expr) != hipSuccess) return bfail(b, TLVLBM_ERR_DEVICE, what); \
  } while (0)

BatchArgs args_of(tlvlbm_batch *b) {
  BatchArgs a{};
  a.st = b->st;
  a.insts = b->d_inst;
  a.ninst = (int)b->c.size();
  a.segs = b->d_segs;
  a.ltiles = b->d_ltiles;
  a.nlt = b->nlt;
  a.ctiles = b->d_ctiles;
  a.nct = b->nct;
  a.jtiles = b->d_jtiles;
  a.njt = b->njt;
  a.step = b->d_step;
  a.pending = b->d_pending;
  a.om = b->jw;
  return a;
}

void run(tlvlbm_batch *b, BatchOp op, int fa = 0, int fb = 0, int nsw = 0) {
  BatchArgs a = args_of(b);
  a.flagA = fa;
  a.flagB = fb;
  a.nsw = nsw;
  launch_batch(b->D, b->prec, op, a);
}

tlvlbm_status pcg_batch(tlvlbm_batch *b, int anch);

tlvlbm_status cg_batch(tlvlbm_batch *b, int useFr) {
  const int anch = b->any_dir ? 1 : 0;
  if (anch) {
    run(b, BatchOp::ZeroAnchor);
    if (b->nlt) run(b, BatchOp::Anchor, useFr);
    run(b, BatchOp::NarrowAnchor);
  }
  run(b, BatchOp::Rhs, useFr, anch);
  if (b->sweeps > 0) {
    // damped Jacobi relaxation: launches alternate x -> r and r -> x (2D:
    // up to JT_NS sweeps per launch, staged in LDS)
    int dir = 0;
    for (int k = 0; k < b->sweeps;) {
      const int ns = b->njt ? std::min(b->sweeps - k, JT_NS) : 1;
      run(b, b->njt ? BatchOp::JacobiFused : BatchOp::Jacobi, dir, anch, ns);
      dir ^= 1;
      k += ns;
    }
    if (dir) run(b, BatchOp::JacobiCopy);
    if (!b->capturing)
      for (tlvlbm_ctx *c : b->c) c->st_cg += (int64_t)b->sweeps * c->D;
    return TLVLBM_OK;
  }
  if (b->use_mg) return pcg_batch(b, anch);
  run(b, BatchOp::CgInit, 0, anch);
  int pp = 0;
  for (int64_t it = 0; it < b->maxit;) {
    const int64_t k = std::min<int64_t>(32, b->maxit - it);
    for (int64_t j = 0; j < k; ++j) {
      run(b, BatchOp::CgAp, pp, anch);
      run(b, BatchOp::CgUpdate, pp);
      pp ^= 1;
    }
    it += k;
    BCHK(hipMemsetAsync(b->d_pending, 0, sizeof(int), b->st), "pending clear");
    run(b, BatchOp::Pending);
    BCHK(hipMemcpyAsync(b->h_pending, b->d_pending, sizeof(int), hipMemcpyDeviceToHost, b->st), "pending read");
    BCHK(hipStreamSynchronize(b->st), "synchronize");
    if (*b->h_pending == 0) break;
  }
  return TLVLBM_OK;
}

// preconditioned CG over all instances: one batched V-cycle per iteration;
// the constants of components without anchors are restored per instance
// afterwards (as in the single-instance solver)
tlvlbm_status pcg_batch(tlvlbm_batch *b, int anch) {
  const int ni = (int)b->c.size();
  for (tlvlbm_ctx *c : b->c) gauge_means(c, (const double *)c->cg.x, nullptr, c->gauge->mean0);
  run(b, BatchOp::CgInit, 0, anch);
  batch_vcycle(b->D, b->bmg, b->d_inst, ni, b->st);
  run(b, BatchOp::PcDotFirst);
  int pp = 0;
  for (int64_t it = 0; it < b->maxit;) {
    for (int j = 0; j < 8; ++j) {
      run(b, BatchOp::PcAp, pp, anch);
      run(b, BatchOp::PcUpdate, pp);
      batch_vcycle(b->D, b->bmg, b->d_inst, ni, b->st);
      run(b, BatchOp::PcDot);
      pp ^= 1;
    }
    it += 8;
    BCHK(hipMemsetAsync(b->d_pending, 0, sizeof(int), b->st), "pending clear");
    run(b, BatchOp::Pending);
    BCHK(hipMemcpyAsync(b->h_pending, b->d_pending, sizeof(int), hipMemcpyDeviceToHost, b->st), "pending read");
    BCHK(hipStreamSynchronize(b->st), "synchronize");
    if (*b->h_pending == 0) break;
  }
  for (tlvlbm_ctx *c : b->c) gauge_restore(c, (double *)c->cg.x, c->gauge->mean0);
  return TLVLBM_OK;
}

void plain_step(tlvlbm_batch *b) {
  launch_bulk_batch(b->D, b->prec, b->d_inst, b->d_btiles, b->nbt, false, b->tw, b->st, b->law, b->d_step);
  if (b->nlt) run(b, BatchOp::Cut);
  run(b, BatchOp::StepEnd);
}

tlvlbm_status projection_step(tlvlbm_batch *b) {
  launch_moments_batch(b->D, b->prec, b->d_inst, b->d_btiles, b->nbt, b->tw, b->st, b->d_step);
  run(b, BatchOp::XfromU);
  tlvlbm_status s = cg_batch(b, 0);
  if (s) return s;
  run(b, BatchOp::UfromX);
  run(b, BatchOp::GradF);
  launch_bulk_batch(b->D, b->prec, b->d_inst, b->d_btiles, b->nbt, true, b->tw, b->st, b->law, b->d_step);
  run(b, BatchOp::XfromU);
  s = cg_batch(b, 1);
  if (s) return s;
  run(b, BatchOp::UReset);
  if (b->nlt) run(b, BatchOp::Cut);
  run(b, BatchOp::StepEnd);
  return TLVLBM_OK;
}

// spans k W .. (k + 1) W - 1 of an instance's node order that hold active
// nodes, as (instance, k); the spans are aligned to W nodes in every plane,
// so their loads and stores start on a cache line; order 0: instance by
// instance, 1: round robin over the instances (tile r of each, then r + 1)
std::vector<int4> node_tiles(const tlvlbm_batch *b, int W, int order) {
  const int ni = (int)b->c.size();
  std::vector<std::vector<int4>> per(ni);
  for (int k = 0; k < ni; ++k) {
    const Geo &g = b->c[k]->geo;
    const std::vector<uint8_t> &a = b->act[k];
    for (int64_t s = 0; s < g.N; s += W) {
      bool any = a.empty();
      for (int64_t i = s; i < std::min<int64_t>(g.N, s + W) && !any; ++i) any = a[(size_t)i] != 0;
      if (any) per[k].push_back(make_int4(k, (int)(s / W), 0, 0));
    }
  }
  std::vector<int4> t;
  if (order == 0) {
    for (auto &v : per) t.insert(t.end(), v.begin(), v.end());
  } else {
    size_t most = 0;
    for (auto &v : per) most = std::max(most, v.size());
    for (size_t r = 0; r < most; ++r)
      for (auto &v : per)
        if (r < v.size()) t.push_back(v[r]);
  }
  return t;
}

tlvlbm_status set_tiles(tlvlbm_batch *b, const std::vector<int4> &t, int W, int order) {
  int4 *d = nullptr;
  BCHK(hipMalloc(&d, std::max<size_t>(1, t.size()) * sizeof(int4)), "tile alloc");
  if (!t.empty() && hipMemcpyAsync(d, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice, b->st) != hipSuccess) {
    (void)hipFree(d);
    return bfail(b, TLVLBM_ERR_DEVICE, "tile upload");
  }
  BCHK(hipStreamSynchronize(b->st), "synchronize");
  if (b->d_btiles) (void)hipFree(b->d_btiles);
  b->d_btiles = d;
  b->nbt = (int)t.size();
  b->tw = W;
  b->torder = order;
  if (b->gexec) {  // the captured steps hold the old tiles
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->glen = 0;
  }
  if (b->gcycle) {
    (void)hipGraphExecDestroy(b->gcycle);
    b->gcycle = nullptr;
  }
  return TLVLBM_OK;
}

// Time the bulk kernel over every tile configuration (reps launches each,
// after one untimed) on the batch's own state and keep the fastest.  The
// kernel reads the populations and rewrites the displacement history in
// place, so u* and u of every instance are saved first and restored after
// every launch: no step is taken and the state is unchanged.
tlvlbm_status batch_autotune(tlvlbm_batch *b, int reps) {
  const int ni = (int)b->c.size();
  const int widths[3] = {64, 128, 256};
  std::vector<void *> keep(2 * ni, nullptr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int4 *dt = nullptr;
  tlvlbm_status res = TLVLBM_OK;
  auto restore = [&]() {
    for (int k = 0; k < ni; ++k) {
      const size_t bytes = (size_t)b->D * b->c[k]->geo.S * sizeof(double);
      if (keep[2 * k] && hipMemcpyAsync(b->c[k]->ustar, keep[2 * k], bytes, hipMemcpyDeviceToDevice, b->st))
        return false;
      if (keep[2 * k + 1] && hipMemcpyAsync(b->c[k]->ubuf, keep[2 * k + 1], bytes, hipMemcpyDeviceToDevice, b->st))
        return false;
    }
    return true;
  };
  double best = 1e300;
  int bw = b->tw, bo = b->torder;
  do {
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    for (int k = 0; ok && k < ni; ++k) {
      const size_t bytes = (size_t)b->D * b->c[k]->geo.S * sizeof(double);
      void *src[2] = {b->c[k]->ustar, b->c[k]->ubuf};
      for (int j = 0; ok && j < 2; ++j) {
        if (!src[j]) continue;
        ok = hipMalloc(&keep[2 * k + j], bytes) == hipSuccess &&
             hipMemcpyAsync(keep[2 * k + j], src[j], bytes, hipMemcpyDeviceToDevice, b->st) == hipSuccess;
      }
    }
    if (!ok) {
      res = bfail(b, TLVLBM_ERR_OUT_OF_MEMORY, "autotune: no room for the saved displacement history");
      break;
    }
    for (int order = 0; order < 2 && res == TLVLBM_OK; ++order)
      for (int wi = 0; wi < 3 && res == TLVLBM_OK; ++wi) {
        const std::vector<int4> t = node_tiles(b, widths[wi], order);
        if (dt) (void)hipFree(dt);
        dt = nullptr;
        if (hipMalloc(&dt, std::max<size_t>(1, t.size()) * sizeof(int4)) != hipSuccess ||
            (!t.empty() &&
             hipMemcpyAsync(dt, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice, b->st) != hipSuccess)) {
          res = bfail(b, TLVLBM_ERR_DEVICE, "autotune: tile upload");
          break;
        }
        double tot = 0.0;
        for (int r = 0; r <= reps; ++r) {
          float ms = 0.0f;
          if (hipEventRecord(e0, b->st) != hipSuccess) res = TLVLBM_ERR_DEVICE;
          launch_bulk_batch(b->D, b->prec, b->d_inst, dt, (int)t.size(), false, widths[wi], b->st, b->law, b->d_step);
          if (hipEventRecord(e1, b->st) != hipSuccess || !restore() || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            res = TLVLBM_ERR_DEVICE;
          if (res) break;
          if (r > 0) tot += ms;
        }
        if (res) {
          res = bfail(b, res, "autotune: timing");
          break;
        }
        b->tune_ms[order][wi] = tot / std::max(reps, 1);
        if (b->tune_ms[order][wi] < best) {
          best = b->tune_ms[order][wi];
          bw = widths[wi];
          bo = order;
        }
      }
  } while (false);
  if (hipStreamSynchronize(b->st) != hipSuccess && !res) res = bfail(b, TLVLBM_ERR_DEVICE, "autotune: synchronize");
  if (dt) (void)hipFree(dt);
  for (void *p : keep)
    if (p) (void)hipFree(p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (res) return res;
  return set_tiles(b, node_tiles(b, bw, bo), bw, bo);
}

// capture glen plain steps once; replayed for every such stretch
tlvlbm_status ensure_graph(tlvlbm_batch *b, int len) {
  if (b->gexec && b->glen == len) return TLVLBM_OK;
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  hipGraph_t g = nullptr;
  BCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal), "graph capture");
  for (int k = 0; k < len; ++k) plain_step(b);
  BCHK(hipStreamEndCapture(b->st, &g), "graph capture end");
  BCHK(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  b->glen = len;
  return TLVLBM_OK;
}

// capture one projection cycle: the projection step (Jacobi sweeps: a fixed
// sequence of launches, no polls, no memsets) and the proj_every - 1 plain
// steps after it; replayed for every whole cycle
tlvlbm_status ensure_cycle_graph(tlvlbm_batch *b) {
  if (b->gcycle) return TLVLBM_OK;
  hipGraph_t g = nullptr;
  BCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal), "graph capture");
  b->capturing = true;
  tlvlbm_status s = projection_step(b);
  for (int k = 1; k < b->proj_every && !s; ++k) plain_step(b);
  b->capturing = false;
  const hipError_t e = hipStreamEndCapture(b->st, &g);
  if (s || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return s ? s : bfail(b, TLVLBM_ERR_DEVICE, "graph capture end");
  }
  const hipError_t ei = hipGraphInstantiate(&b->gcycle, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    b->gcycle = nullptr;
    return bfail(b, TLVLBM_ERR_DEVICE, "graph instantiate");
  }
  return TLVLBM_OK;
}

}  // namespace

extern "C" {

tlvlbm_status tlvlbm_batch_create(tlvlbm_ctx *const *ctxs, int32_t n, tlvlbm_batch **out) {
  if (!ctxs || n < 1 || !out) return TLVLBM_ERR_INVALID_ARG;
  *out = nullptr;
  tlvlbm_batch *b = new (std::nothrow) tlvlbm_batch();
  if (!b) return TLVLBM_ERR_OUT_OF_MEMORY;
  try {
    const tlvlbm_ctx *c0 = ctxs[0];
    if (!c0) {
      delete b;
      return TLVLBM_ERR_INVALID_ARG;
    }
    b->D = c0->D;
    b->prec = c0->prec;
    b->st = c0->st;
    b->proj_every = c0->proj_every;
    b->sweeps = c0->proj_sweeps;
    b->jw = c0->proj_weight;
    b->step = c0->step;
    b->use_graph = b->st != nullptr;  // no stream capture on the legacy default stream
    std::vector<Seg> segs;
    std::vector<int4> bt, ct, lt;
    int n_neu = 0;  // instances with Neumann links (those the projection runs on)
    bool any_visco = false, any_thermal = false;
    for (int k = 0; k < n; ++k) {
      tlvlbm_ctx *c = ctxs[k];
      if (!c || c->D != b->D || c->prec != b->prec || c->st != b->st || c->proj_every != b->proj_every ||
          c->proj_sweeps != b->sweeps || c->proj_weight != b->jw || c->step != b->step || !c->have_state ||
          !c->has_ls || !c->track_u || c->status || (c->visco && !c->hist_set)) {
        delete b;
        return TLVLBM_ERR_INVALID_ARG;
      }
      if (ensure_cg(c)) {
        delete b;
        return TLVLBM_ERR_OUT_OF_MEMORY;
      }
      b->c.push_back(c);
      Inst I{};
      I.g = c->geo;
      I.p = c->par;
      I.theta = c->theta;
      I.rtol = c->cg_rtol > 0 ? c->cg_rtol : cg_default_rtol(c->prec);
      I.fin = c->fB;
      I.fout = c->fA;
      I.act = c->act;
      I.ustar = c->ustar;
      I.ubuf = c->ubuf;
      I.L = c->L;
      I.x = c->cg.x;
      I.r = c->cg.r;
      I.p0 = c->cg.p0;
      I.p1 = c->cg.p1;
      I.Ap = c->cg.Ap;
      I.b = c->cg.b;
      I.V = c->cg.V;
      I.Fm = c->cg.Fm;
      I.Fr = c->cg.Fr;
      I.anc_s = c->cg.anc_s;
      I.z = c->cg.z;
      I.anc_n = c->cg.anc_n;
      I.nbm = c->cg.nbm;
      I.anc_i = c->cg.anc_i;
      I.partial = c->cg.partial;
      I.scal = c->cg.scal;
      I.nblk = c->cg.nblk;
      I.flag = c->d_flag;
      I.nfail = (unsigned long long *)c->d_newton_fail;
      I.bf = c->bf;
      I.bf_ramp = c->bf_ramp;
      I.bf_Tr = c->bf_Tr;
      b->h_inst.push_back(I);
      if (c->par.k1 != 0.0 || c->bf) b->law = std::max(b->law, 1);
      if (c->par.thf) any_thermal = true;
      if (c->visco) any_visco = true;
      {
        // activity mask on the host for the node-tile lists (empty: all active)
        std::vector<uint8_t> a;
        if (c->act) {
          a.resize((size_t)c->geo.N);
          if (hipMemcpy(a.data(), c->act, a.size(), hipMemcpyDeviceToHost) != hipSuccess) {
            tlvlbm_batch_destroy(b);
            return TLVLBM_ERR_DEVICE;
          }
        }
        b->act.push_back(std::move(a));
      }
      for (int blk = 0; blk < c->cg.nblk; ++blk) ct.push_back(make_int4(k, blk, 0, 0));
      bool inst_neu = false;
      for (int bid = 0; bid < 256; ++bid) {
        const int64_t b0 = c->bid_begin[bid], b1 = c->bid_end[bid];
        if (b1 <= b0) continue;
        if (c->bcs[bid].type == TLVLBM_BC_NEUMANN_TRACTION) inst_neu = true;
        Seg s{};
        s.inst = k;
        s.type = c->bcs[bid].type;
        s.b0 = b0;
        s.b1 = b1;
        s.bc = c->bcs[bid];
        if (s.type == TLVLBM_BC_NEUMANN_TRACTION) b->any_neu = true;
        if (s.type == TLVLBM_BC_DIRICHLET_VELOCITY) b->any_dir = true;
        for (int64_t o = 0; o < b1 - b0; o += 64) lt.push_back(make_int4((int)segs.size(), (int)o, 0, 0));
        segs.push_back(s);
      }
      n_neu += inst_neu ? 1 : 0;
      b->maxit = std::max<int64_t>(b->maxit, c->cg_maxit > 0 ? c->cg_maxit : cg_default_maxit(c->nactive));
    }
    // The projection phases run over every instance of the batch, and the
    // projection belongs only to lattices with Neumann links (Sec. 3.5):
    // instances with and without them cannot share a batch.
    if (n_neu != 0 && n_neu != n) {
      tlvlbm_batch_destroy(b);
      return TLVLBM_ERR_INVALID_ARG;
    }
    // one bulk update serves the batch: a Maxwell branch and a thermal
    // stretch have none in common
    if (any_visco && any_thermal) {
      tlvlbm_batch_destroy(b);
      return TLVLBM_ERR_INVALID_ARG;
    }
    if (any_visco) b->law = 3;
    else if (any_thermal) b->law = 2;
    bt = node_tiles(b, b->tw, b->torder);
    b->nbt = (int)bt.size();
    b->nct = (int)ct.size();
    b->nlt = (int)lt.size();
    // batched multigrid when every instance carries a hierarchy
    b->use_mg = b->any_neu;
    for (tlvlbm_ctx *c : b->c) b->use_mg = b->use_mg && c->mg && c->gauge && !c->aux_stale && c->mg->nu == 2;
    if (b->use_mg) {
      BatchMG &bm = b->bmg;
      int lmax = 0;
      for (tlvlbm_ctx *c : b->c) lmax = std::max<int>(lmax, (int)c->mg->lev.size());
      bm.lmax = lmax;
      bm.omega = b->c[0]->mg->omega;
      bm.nu_coarse = b->c[0]->mg->nu_coarse;
      std::vector<BMGLev> tab((size_t)n * lmax);
      std::vector<int> last(n);
      std::vector<std::vector<int4>> sm(lmax), rs(lmax);
      for (int k = 0; k < n; ++k) {
        const MG &mg = *b->c[k]->mg;
        const int nl = (int)mg.lev.size();
        last[k] = nl - 1;
        for (int l = 0; l < nl; ++l) {
          const MGLevel &L = mg.lev[l];
          BMGLev &T = tab[(size_t)k * lmax + l];
          T.v = L.v;
          T.b = l == 0 ? (double *)b->c[k]->cg.r : L.b;
          T.A = L.x;
          T.B = L.t;
          const int nblk = (int)((L.v.N + 255) / 256);
          for (int blk = 0; blk < nblk; ++blk) {
            if (l < nl - 1) sm[l].push_back(make_int4(k, blk, 0, 0));
            if (l >= 1) rs[l].push_back(make_int4(k, blk, 0, 0));
          }
        }
      }
      bool ok = hipMalloc(&bm.tab, tab.size() * sizeof(BMGLev)) == hipSuccess &&
                hipMalloc(&bm.last, n * sizeof(int)) == hipSuccess &&
                hipMemcpy(bm.tab, tab.data(), tab.size() * sizeof(BMGLev), hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(bm.last, last.data(), n * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
      bm.sm.assign(lmax, nullptr);
      bm.rs.assign(lmax, nullptr);
      bm.nsm.assign(lmax, 0);
      bm.nrs.assign(lmax, 0);
      for (int l = 0; l < lmax && ok; ++l) {
        bm.nsm[l] = (int)sm[l].size();
        bm.nrs[l] = (int)rs[l].size();
        if (bm.nsm[l])
          ok = hipMalloc(&bm.sm[l], sm[l].size() * sizeof(int4)) == hipSuccess &&
               hipMemcpy(bm.sm[l], sm[l].data(), sm[l].size() * sizeof(int4), hipMemcpyHostToDevice) == hipSuccess;
        if (ok && bm.nrs[l])
          ok = hipMalloc(&bm.rs[l], rs[l].size() * sizeof(int4)) == hipSuccess &&
               hipMemcpy(bm.rs[l], rs[l].data(), rs[l].size() * sizeof(int4), hipMemcpyHostToDevice) == hipSuccess;
      }
      if (!ok) {
        tlvlbm_batch_destroy(b);
        return TLVLBM_ERR_OUT_OF_MEMORY;
      }
    }
    if (hipMalloc(&b->d_inst, n * sizeof(Inst)) != hipSuccess ||
        hipMalloc(&b->d_btiles, std::max<size_t>(1, bt.size()) * sizeof(int4)) != hipSuccess ||
        hipMalloc(&b->d_ctiles, ct.size() * sizeof(int4)) != hipSuccess ||
        hipMalloc(&b->d_ltiles, std::max<size_t>(1, lt.size()) * sizeof(int4)) != hipSuccess ||
        hipMalloc(&b->d_segs, std::max<size_t>(1, segs.size()) * sizeof(Seg)) != hipSuccess ||
        hipMalloc(&b->d_step, sizeof(int64_t)) != hipSuccess || hipMalloc(&b->d_pending, sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&b->h_pending, sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&b->h_flags, n * sizeof(int)) != hipSuccess) {
      tlvlbm_batch_destroy(b);
      return TLVLBM_ERR_OUT_OF_MEMORY;
    }
    hipStream_t st = b->st;
    if (hipMemcpyAsync(b->d_inst, b->h_inst.data(), n * sizeof(Inst), hipMemcpyHostToDevice, st) != hipSuccess ||
        (bt.size() &&
         hipMemcpyAsync(b->d_btiles, bt.data(), bt.size() * sizeof(int4), hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(b->d_ctiles, ct.data(), ct.size() * sizeof(int4), hipMemcpyHostToDevice, st) != hipSuccess ||
        (lt.size() &&
         hipMemcpyAsync(b->d_ltiles, lt.data(), lt.size() * sizeof(int4), hipMemcpyHostToDevice, st) != hipSuccess) ||
        (segs.size() &&
         hipMemcpyAsync(b->d_segs, segs.data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(b->d_step, &b->step, sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      tlvlbm_batch_destroy(b);
      return TLVLBM_ERR_DEVICE;
    }
    // 2D Jacobi projection: the tiles of the fused sweeps, instance by
    // instance (every instance needs its neighbour masks)
    if (b->D == 2 && b->any_neu && b->sweeps > 0) {
      std::vector<int4> jt;
      std::vector<int32_t> one;
      bool ok = true;
      for (int k = 0; k < n && ok; ++k) {
        const tlvlbm_ctx *c = b->c[k];
        ok = c->cg.nbm != nullptr &&
             active_tiles2(c->geo, b->act[k].empty() ? nullptr : b->act[k].data(), one);
        for (int32_t p : one) jt.push_back(make_int4(k, p & 0xffff, p >> 16, 0));
      }
      if (ok && !jt.empty()) {
        if (hipMalloc(&b->d_jtiles, jt.size() * sizeof(int4)) != hipSuccess) {
          tlvlbm_batch_destroy(b);
          return TLVLBM_ERR_OUT_OF_MEMORY;
        }
        if (hipMemcpy(b->d_jtiles, jt.data(), jt.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess) {
          tlvlbm_batch_destroy(b);
          return TLVLBM_ERR_DEVICE;
        }
        b->njt = (int)jt.size();
      }
    }
    // tile configuration of the node kernels, timed on this batch
    const tlvlbm_status ts = batch_autotune(b, 3);
    if (ts) {
      tlvlbm_batch_destroy(b);
      return ts;
    }
    *out = b;
    return TLVLBM_OK;
  } catch (...) {
    delete b;
    return TLVLBM_ERR_OUT_OF_MEMORY;
  }
}

tlvlbm_status tlvlbm_batch_autotune(tlvlbm_batch *b, int32_t reps) {
  if (!b || reps < 1) return TLVLBM_ERR_INVALID_ARG;
  return batch_autotune(b, reps);
}

tlvlbm_status tlvlbm_batch_set_tiles(tlvlbm_batch *b, int32_t tile_width, int32_t order) {
  if (!b || (tile_width != 64 && tile_width != 128 && tile_width != 256) || (order != 0 && order != 1))
    return TLVLBM_ERR_INVALID_ARG;
  return set_tiles(b, node_tiles(b, tile_width, order), tile_width, order);
}

tlvlbm_status tlvlbm_batch_get_tiles(const tlvlbm_batch *b, int32_t *tile_width, int32_t *order, double *ms) {
  if (!b) return TLVLBM_ERR_INVALID_ARG;
  if (tile_width) *tile_width = b->tw;
  if (order) *order = b->torder;
  if (ms)
    for (int o = 0; o < 2; ++o)
      for (int w = 0; w < 3; ++w) ms[o * 3 + w] = b->tune_ms[o][w];
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_batch_set_graph(tlvlbm_batch *b, int32_t use_graph) {
  if (!b) return TLVLBM_ERR_INVALID_ARG;
  b->use_graph = use_graph != 0 && b->st != nullptr;
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_batch_step(tlvlbm_batch *b, int64_t n) {
  if (!b || n < 0) return TLVLBM_ERR_INVALID_ARG;
  for (auto *c : b->c)
    if (c->status) return bfail(b, (tlvlbm_status)c->status, "an instance holds a sticky error");
  if (n > 0)
    for (auto *c : b->c) rec_invalidate(c);
  const int pe = b->proj_every;
  int64_t k = 0;
  while (k < n) {
    const bool proj = b->any_neu && pe > 0 && (b->step % pe == 0);
    if (proj && b->use_graph && b->sweeps > 0 && pe > 1 && n - k >= pe) {
      // a whole cycle from one graph
      tlvlbm_status s = ensure_cycle_graph(b);
      if (s) return s;
      BCHK(hipGraphLaunch(b->gcycle, b->st), "graph launch");
      for (tlvlbm_ctx *c : b->c) c->st_cg += 2 * (int64_t)b->sweeps * c->D;
      b->step += pe;
      k += pe;
      continue;
    }
    if (proj) {
      tlvlbm_status s = projection_step(b);
      if (s) return s;
      ++b->step;
      ++k;
      continue;
    }
    // plain steps until the next projection step (or the end)
    int64_t run_len = n - k;
    if (b->any_neu && pe > 0) run_len = std::min<int64_t>(run_len, pe - (b->step % pe));
    const int glen = (b->any_neu && pe > 1) ? pe - 1 : 20;
    if (b->use_graph && run_len == glen) {
      tlvlbm_status s = ensure_graph(b, glen);
      if (s) return s;
      BCHK(hipGraphLaunch(b->gexec, b->st), "graph launch");
    } else {
      for (int64_t j = 0; j < run_len; ++j) plain_step(b);
    }
    b->step += run_len;
    k += run_len;
  }
  BCHK(hipGetLastError(), "batch launch");
  // keep the contexts' view of their buffers and step in sync
  const int ni = (int)b->c.size();
  for (int i = 0; i < ni; ++i) {
    tlvlbm_ctx *c = b->c[i];
    if (n & 1) std::swap(c->fA, c->fB);
    c->step = b->step;
    c->fresh = false;
    BCHK(hipMemcpyAsync(b->h_flags + i, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, b->st), "flag read");
  }
  BCHK(hipStreamSynchronize(b->st), "synchronize");
  tlvlbm_status worst = TLVLBM_OK;
  for (int i = 0; i < ni; ++i) {
    const int f = b->h_flags[i];
    tlvlbm_status s = (f & FLAG_NONFINITE) ? TLVLBM_ERR_NONFINITE
                      : (f & FLAG_J)       ? TLVLBM_ERR_NONPOSITIVE_J
                      : (f & FLAG_NEWTON)  ? TLVLBM_ERR_NEWTON
                                           : TLVLBM_OK;
    if (s) {
      b->c[i]->status = s;
      worst = s;
    }
  }
  if (worst) return bfail(b, worst, "an instance reported a device failure");
  return TLVLBM_OK;
}

tlvlbm_status tlvlbm_batch_destroy(tlvlbm_batch *b) {
  if (!b) return TLVLBM_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(b->st);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->gcycle) (void)hipGraphExecDestroy(b->gcycle);
  batch_mg_free(b->bmg);
  void *ptrs[] = {b->d_inst, b->d_btiles, b->d_ctiles, b->d_ltiles, b->d_jtiles, b->d_segs, b->d_step, b->d_pending};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (b->h_pending) (void)hipHostFree(b->h_pending);
  if (b->h_flags) (void)hipHostFree(b->h_flags);
  delete b;
  return TLVLBM_OK;
}

const char *tlvlbm_batch_last_error(const tlvlbm_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
