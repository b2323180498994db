// Internal types of the tlvlbm runtime (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tlvlbm.h"

namespace tl {

// sticky device error bits
enum : int { FLAG_J = 1, FLAG_NONFINITE = 2, FLAG_NEWTON = 4, FLAG_ARG = 8, FLAG_STENCIL = 16 };

// maximum LSQ stencil (active nodes within 2.5 dx of X_b; at most 21 lattice
// points fit in 2D and 81 in 3D)
constexpr int KMAX2 = 24;
// nodes per chunk of the embedded-body chunk list (a divisor of 64: one
// wavefront covers 64 / CHUNK chunks)
#ifndef TL_CHUNK
#define TL_CHUNK 32
#endif
constexpr int CHUNK = TL_CHUNK;
constexpr int KMAX3 = 88;
constexpr double LSQ_RADIUS = 2.5;
// 2D projection sweeps fused in LDS: tiles of JT x JT nodes, JT_NS sweeps per
// launch (the staged halo is JT_NS nodes wide)
constexpr int JT = 32;
#ifndef TL_JACOBI_FUSE
#define TL_JACOBI_FUSE 5
#endif
constexpr int JT_NS = TL_JACOBI_FUSE;

// grid geometry passed by value to kernels
struct Geo {
  int nx, ny, nz;
  int per;      // periodic bit mask
  int64_t N;    // nodes
  int64_t S;    // plane stride (elements) of population and node-field planes
  double dx, ox, oy, oz;
};

// scalar parameters of the bulk update
struct Par {
  double mu, lam, inv_rho0, dt, c, omega, gamma;
  double k1, a0[3];  // fibre reinforcement (k1 = 0: the neo-Hookean law of Eq. 62)
  // Reference state (0, Fref) of the stored populations: every kernel keeps
  // g_q = f_q - feq_q(0, Fref), whose moments are (v, F - Fref) and whose
  // magnitudes are those of the dynamics rather than of the static stress.
  // Pref = P(Fref) / rho0 with the material of tlvlbm_set_state (a constant
  // of the representation: a later material change keeps it).
  double Fref[9], Pref[9];
  // Maxwell branch (law 2): beta xi and xi^2 with xi = exp(-dt / (2 tau)),
  // and the node's internal variables R = xi^2 Q^n - beta xi S_0^n in
  // D(D+1)/2 FP64 planes of stride S (packed symmetric, sym_idx); null: no
  // branch
  double vbx, vxi2;
  double *hist;
  // thermal stretch of every node (one FP64 plane of stride S), or null
  const double *thf;
};

// stored-population shift feq_q^r(0, Fref) of direction q, row r:
// velocity rows -e_qA Pref_iA / (2c), deformation rows Fref / (2D)
template <int D> __host__ __device__ __forceinline__ double pop_shift(const Par &p, int q, int r) {
  if (r < D) return ((q & 1) ? 0.5 : -0.5) * p.Pref[r * D + q / 2] / p.c;
  return p.Fref[r - D] / (2 * D);
}

// cut-link table (device SoA), ordered by (bid, node, q)
struct Links {
  int64_t n = 0;
  int kmax = 0;
  int64_t *node = nullptr, *out = nullptr, *mminus = nullptr;
  int32_t *q = nullptr, *bid = nullptr, *npts = nullptr, *basis = nullptr;
  double *eta = nullptr, *Nb = nullptr /*[n][3]*/, *Xb = nullptr /*[n][3]*/, *tang = nullptr /*[n][2][3]*/;
  // LSQ stencils, point-major so that adjacent links (one per lane) read
  // adjacent words: node of point k of link l at sidx[k*n + l], weight of
  // tangent al at sw[(al*kmax + k)*n + l] (see lsq_i, lsq_w)
  int32_t *sidx = nullptr; /*[kmax][n]*/
  double *sw = nullptr;    /*[2][kmax][n]*/
};

__host__ __device__ inline size_t lsq_i(const Links &L, int64_t l, int k) { return (size_t)k * L.n + l; }
__host__ __device__ inline size_t lsq_w(const Links &L, int64_t l, int al, int k) {
  return ((size_t)al * L.kmax + k) * L.n + l;
}

// boundary condition by value (mirrors tlvlbm_bc)
struct BC {
  int type, ramp, disp;
  double Tr, a[3], G[9], pr, pn, X0[3], tw;
};

// scalar slots of the CG state (device doubles, per component)
enum { S_RR = 0, S_BB = 4, S_THR = 8, S_ALPHA = 12, S_BETA = 16, S_ACT = 20, S_ITS = 24, S_DONE = 28, S_RZ = 32,
       S_NSCAL = 36 };

// one multigrid level (device view passed by value to kernels)
struct MGView {
  int nx, ny, nz, per;
  int64_t N, stride;  // nodes, plane stride of the level's vectors
  const float *w;     // [D][N] weight of the edge to the +A neighbour
  const float *d;     // [N] diagonal (edge weights + anchors)
};
struct MGLevel {
  MGView v{};
  float *w = nullptr, *d = nullptr;
  double *b = nullptr, *x = nullptr, *t = nullptr;  // [D][stride]
};
struct MG {
  std::vector<MGLevel> lev;
  double omega = 2.0 / 3.0;
  int nu = 2, nu_coarse = 40;
  const int32_t *tiles = nullptr;  // finest level: active 256-node tiles (the CG's)
  int ntiles = 0;
};

// connected components of the active graph that carry no anchor: the
// projection determines u there only up to a constant (the gauge)
struct Gauge {
  int64_t nu = 0, ntile = 0;   // such components; tiles of 256 of their nodes
  int32_t *comp = nullptr;     // [N] component index, -1 elsewhere
  int32_t *cn = nullptr;       // [ntile*256] node of each tile slot, -1 padding
  int64_t *ct = nullptr;       // [nu+1] first tile of each component
  int64_t *ccnt = nullptr;     // [nu] node count
  double *tpart = nullptr;     // [ntile][D] tile sums
  double *mean = nullptr, *mean0 = nullptr;  // [nu][D]
  uint8_t *anc_n = nullptr;    // [N] anchor counts (Dirichlet cut links per node)
};

// LSQ stencils of the Neumann links transposed to their nodes (reverse
// mode): node sn[t] receives entries so[t] .. so[t+1]-1 = (link el, point ek)
struct StencilT {
  int64_t ns = 0;                       // distinct stencil nodes of the Neumann links
  int64_t *sn = nullptr, *so = nullptr; // their node indices (sorted), entry offsets
  int32_t *el = nullptr, *ek = nullptr; // per entry: link, point
  double *ew = nullptr;                 // per entry: the D - 1 tangent weights
  int32_t *sc = nullptr;                // per stencil slot lsq_i(l, k): index into sn
};

// device blocks of the reverse mode, kept between calls of the same shape
// (step count, segment length): repeated gradient evaluations allocate once
struct AdjArena {
  std::vector<void *> blk;
  std::vector<size_t> bytes;
  int64_t key[2] = {-1, -1};  // (steps, requested segment length)
  size_t avail = 0;  // free memory beyond the fixed needs when first sized
  int64_t seg = 1, tail = 0;  // the schedule chosen for that key
};

// projection / CG workspace
struct CG {
  void *x = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *Ap = nullptr, *b = nullptr;  // [D][S] FP64
  void *z = nullptr;                                // preconditioned residual [D][S] FP64
  void *V = nullptr, *Fm = nullptr, *Fr = nullptr;  // v [D][S], F - I [D2][S], F^r - I [D2][S]  (T)
  uint8_t *anc_n = nullptr;                         // anchors per node
  int *anc_i = nullptr;                             // anchor counting scratch
  void *anc_s = nullptr;                            // anchor target sums [D][S] (FP64)
  double *partial = nullptr;                        // [nblk][16] block partial sums
  int32_t *tiles = nullptr;                         // 256-node tiles holding active nodes
  int ntiles = 0;
  uint8_t *nbm = nullptr;  // per node: bit q = neighbour X + e_q active, bit 6 = node active
  int32_t *jt = nullptr;   // 2D: JT x JT tiles holding active nodes (tx | ty << 16)
  int njt = 0;
  hipGraphExec_t pcg_graph = nullptr;               // captured batch of preconditioned iterations
  const void *pcg_key = nullptr;                    // anchor array it was captured with
  double *scal = nullptr;                           // device scalars
  int nblk = 0;
};

struct AdjRec;  // a recorded forward run of the reverse mode (below)

// Per-instance descriptor of a batched launch (device memory).  fin/fout are
// swapped on the device at the end of every step, so the ping-pong of every
// instance needs no upload (and replays correctly from a graph).
struct Inst {
  Geo g;
  Par p;
  double theta, rtol;
  void *fin, *fout;
  uint8_t *act;
  void *ustar, *ubuf;  // displacement history u*, u: FP64 in both builds
  Links L;
  // projection workspace
  void *x, *r, *p0, *p1, *Ap, *b, *V, *Fm, *Fr, *anc_s;
  void *z;  // preconditioned residual (batched multigrid)
  uint8_t *anc_n;
  uint8_t *nbm;  // neighbour masks of the projection graph (null: from act)
  int *anc_i;
  double *partial, *scal;
  int nblk;  // node tiles of 256 of this instance (CG reductions)
  int *flag;
  unsigned long long *nfail;
  // body acceleration b = s(t) g: g planes in the population precision
  // (null: none) and the ramp s
  const void *bf;
  int bf_ramp;
  double bf_Tr;
};

// one boundary identifier of one instance: a contiguous link range
struct Seg {
  int inst, type;
  int64_t b0, b1;
  BC bc;
};

enum class BatchOp { Cut, Anchor, ZeroAnchor, NarrowAnchor, XfromU, UfromX, Rhs, CgInit, CgAp, CgUpdate, GradF,
                     UReset, StepEnd, Pending, PcInit, PcAp, PcUpdate, PcDot, PcDotFirst, Jacobi, JacobiCopy,
                     JacobiFused };

// one multigrid level of one instance in a batched V-cycle: the view and the
// level's vectors (b: right-hand side, A and B: the two sweep buffers; the
// level's result is in B)
struct BMGLev {
  MGView v;
  double *b, *A, *B;
};

// level-synchronous batched V-cycle over instances with different depths
struct BatchMG {
  int lmax = 0;                         // deepest hierarchy
  BMGLev *tab = nullptr;                // device [ninst][lmax]
  int *last = nullptr;                  // device [ninst] coarsest level index
  double omega = 2.0 / 3.0;
  int nu_coarse = 40;
  std::vector<int4 *> sm;               // per level: (inst, block) tiles of the levels above an instance's coarsest
  std::vector<int> nsm;
  std::vector<int4 *> rs;               // per level l >= 1: tiles of level-l nodes that receive a restriction
  std::vector<int> nrs;
};
void batch_vcycle(int D, const BatchMG &bm, const Inst *insts, int ninst, hipStream_t st);
void batch_mg_free(BatchMG &bm);

struct BatchArgs {
  hipStream_t st;
  Inst *insts;
  int ninst;
  const Seg *segs;
  const int4 *ltiles;  // link tiles (segment, first link)
  int nlt;
  const int4 *ctiles;  // node tiles (instance, block of 256)
  int nct;
  int64_t *step;       // device step counter
  int *pending;
  int flagA, flagB;
  const int4 *jtiles;  // 2D tiles of the fused sweeps (instance, tx, ty)
  int njt;
  int nsw;             // sweeps of one fused launch
  double om;           // Jacobi weight (projection sweeps)
};

// JT x JT tiles of a 2D grid that hold an active node, row by row, packed
// tx | ty << 16 (act null: every node active); false when the grid has more
// tiles per axis than the packing holds
inline bool active_tiles2(const Geo &g, const uint8_t *act, std::vector<int32_t> &out) {
  out.clear();
  const int tnx = (g.nx + JT - 1) / JT, tny = (g.ny + JT - 1) / JT;
  if (g.nz != 1 || tnx > 65535 || tny > 32767) return false;
  std::vector<uint8_t> hit((size_t)tnx * tny, act ? 0 : 1);
  if (act)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x)
        if (act[x + (int64_t)g.nx * y]) hit[(size_t)(y / JT) * tnx + x / JT] = 1;
  for (int ty = 0; ty < tny; ++ty)
    for (int tx = 0; tx < tnx; ++tx)
      if (hit[(size_t)ty * tnx + tx]) out.push_back(tx | (ty << 16));
  return true;
}

// host or device arguments crossing the ABI
inline bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// device view of a borrowed input array (copied when it lives on the host)
struct DevIn {
  const void *ptr = nullptr;
  void *owned = nullptr;
  ~DevIn() {
    if (owned) (void)hipFree(owned);
  }
  hipError_t take(const void *src, size_t bytes, hipStream_t st) {
    if (!src) return hipSuccess;
    if (is_device_ptr(src)) {
      ptr = src;
      return hipSuccess;
    }
    hipError_t e = hipMalloc(&owned, bytes);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(owned, src, bytes, hipMemcpyHostToDevice, st);
    ptr = owned;
    return e;
  }
};

// device target for a caller output (staged when it lives on the host)
struct DevOut {
  void *user = nullptr, *ptr = nullptr, *owned = nullptr;
  size_t bytes = 0;
  ~DevOut() {
    if (owned) (void)hipFree(owned);
  }
  hipError_t take(void *dst, size_t b) {
    user = dst;
    bytes = b;
    if (!dst) return hipSuccess;
    if (is_device_ptr(dst)) {
      ptr = dst;
      return hipSuccess;
    }
    hipError_t e = hipMalloc(&owned, b);
    ptr = owned;
    return e;
  }
  hipError_t finish(hipStream_t st) {
    if (owned && user) return hipMemcpyAsync(user, owned, bytes, hipMemcpyDeviceToHost, st);
    return hipSuccess;
  }
};

void launch_batch(int D, int prec, BatchOp op, const BatchArgs &a);
// batched node kernels over tiles of tw nodes of one row (tw <= 256 threads)
void launch_bulk_batch(int D, int prec, const Inst *insts, const int4 *tiles, int ntiles, bool repair, int tw,
                       hipStream_t st, int law, const int64_t *step);
void launch_moments_batch(int D, int prec, const Inst *insts, const int4 *tiles, int ntiles, int tw,
                          hipStream_t st, const int64_t *step);
int ensure_cg(tlvlbm_ctx *c);
int64_t cg_default_maxit(int64_t nactive);
double cg_default_rtol(int prec);

}  // namespace tl

struct tlvlbm_ctx {
  int D = 0, Q = 0, M = 0, prec = 0;
  tl::Geo geo{};
  tl::Par par{};
  double theta = 1.0, cg_rtol = 0.0;
  int proj_every = 20, cg_maxit = 0, track_opt = -1;
  int cg_multigrid = 1;        // 1: multigrid-preconditioned CG, 0: plain CG
  int proj_sweeps = 20;        // > 0: damped Jacobi sweeps per projection solve; 0: exact solve
  double proj_weight = 2.0 / 3.0;
  tl::MG *mg = nullptr;        // preconditioner hierarchy (built on first use)
  tl::Gauge *gauge = nullptr;  // components without anchors (built on first use)
  tl::StencilT *stT = nullptr; // transposed Neumann stencils (reverse mode, built on first use)
  tl::AdjArena *arena = nullptr; // reverse-mode device memory (kept until destroy or a new shape)
  tl::AdjRec *rec = nullptr;     // the forward run recorded for the backward pass
  // caller's device allocator (tlvlbm_options); null: hipMalloc / hipFree
  void *(*dev_alloc)(size_t, void *) = nullptr;
  void (*dev_free)(void *, void *) = nullptr;
  void *alloc_user = nullptr;
  bool aux_stale = true;       // boundary conditions changed since the build
  bool track_u = false;
  hipStream_t st = nullptr;
  size_t esz = 4;
  void *fA = nullptr, *fB = nullptr;  // population planes (Q*M planes of stride S)
  // embedded bodies: the CHUNK-node chunks of the node order that hold active
  // nodes (one wavefront each); the bulk update skips the rest
  int32_t *chunks = nullptr;
  int nchunks = 0;
  // position of every CHUNK-node block in the chunk list (-1: not listed);
  // the reverse-mode tape stores chunk slots cpos[i / CHUNK] * CHUNK + i % CHUNK
  int32_t *cpos = nullptr;
  // body acceleration b(X, t) = s(t) g(X) (Eq. 5): g in D planes of the
  // population precision (null: none), s a ramp
  void *bf = nullptr;
  int bf_ramp = 0;
  double bf_Tr = 1.0;
  // Maxwell branch of law 2 (beta, tau) and its history planes (kept
  // allocated once made; par.hist points at them while the law has a branch)
  bool visco = false;
  double vbeta = 0.0, vtau = 0.0;
  double *hist = nullptr;
  bool hist_set = false;  // the planes hold the branch's history (set_state or put_history)
  double *thf = nullptr;  // thermal stretch plane [S] (par.thf while set)
  // displacement history u* and u (Eq. 34): D FP64 planes each in both
  // builds (a quadrature over thousands of steps; FP32 sums lose ~1e-5)
  void *ustar = nullptr, *ubuf = nullptr;
  uint8_t *act = nullptr;  // active mask (nullptr: all active)
  int64_t first_active = 0;  // first active node in node order (the reference state is read there)
  bool has_ls = false, have_state = false;
  bool fresh = false;  // state is the one set by set_state (no step since)
  int64_t nactive = 0;
  tl::Links L;
  int64_t bid_begin[256] = {0}, bid_end[256] = {0};
  bool bc_set[256] = {false};
  tl::BC bcs[256];
  tl::BC *d_bcs = nullptr;  // device copy for the cut-link launches (refreshed when bcs_dirty)
  bool bcs_dirty = true;
  tl::CG cg;
  double *hscal = nullptr;  // pinned host mirror for scalars
  int *d_flag = nullptr;
  int *h_flag = nullptr;
  int64_t *d_newton_fail = nullptr;
  int status = TLVLBM_OK;
  std::string err;
  int64_t step = 0;
  int64_t st_cg = 0, st_proj = 0, st_lin = 0;
};

namespace tl {
// device memory kept by a context: through its allocator hooks when set
hipError_t dmalloc_v(tlvlbm_ctx *c, void **p, size_t bytes);
void dfree(tlvlbm_ctx *c, void *p);
template <typename X> inline hipError_t dmalloc(tlvlbm_ctx *c, X **p, size_t bytes) {
  return dmalloc_v(c, (void **)p, bytes);
}
// launchers (bulk.hip)
// taped: the kernels of the reverse mode's forward (the same update through
// the shared device function, recording the tape when tape is not null), so
// that steps with and without a tape round identically
void launch_bulk(tlvlbm_ctx *c, bool repair, void *tape = nullptr, bool taped = false);
void launch_pull_moments(tlvlbm_ctx *c, double *U, double *u, double *J, bool to_scratch);
void launch_moments_native(tlvlbm_ctx *c, void *U, double *u, void *J);
void launch_init(tlvlbm_ctx *c, const double *U0, const double *u0, const double *dU0);
void launch_get_f(tlvlbm_ctx *c, double *f, double *ustar);
void launch_planes_in(tlvlbm_ctx *c, const double *src, void *dst, int k);
void launch_put_f(tlvlbm_ctx *c, const double *f, const double *ustar);
void launch_stress(tlvlbm_ctx *c, double *P, double *sigma);
// launchers (embed.hip)
int build_links(tlvlbm_ctx *c, const double *phi_d, const uint8_t *bid_d, std::string &err);
int launch_cutlinks(tlvlbm_ctx *c, double tn);
// store/mode: 0 solve; 1 solve and keep the solution on the active tiles in
// store; 2 take the solution from store instead of solving
int run_projection(tlvlbm_ctx *c, bool first, double tn, double *store = nullptr, int mode = 0);
// CG on the projection workspace with a given right-hand side (w.b) and start (w.x)
int run_cg_given(tlvlbm_ctx *c, const uint8_t *anc_n);
// projection helpers (mg.hip): components and anchors, multigrid hierarchy
int proj_aux_build(tlvlbm_ctx *c);
void proj_aux_free(tlvlbm_ctx *c);
void mg_apply(tlvlbm_ctx *c, const double *r, double *z, const double *scal);
// per-component means of ua (+ ub) over the components without anchors
void gauge_means(tlvlbm_ctx *c, const double *ua, const double *ub, double *mean);
// x -= mean(x) - mean0 on those components
void gauge_restore(tlvlbm_ctx *c, double *x, const double *mean0);
// reverse-mode tape of one step: recovered state (v, F - I) [M planes],
// repaired F [D*D planes, projection steps], displacement seen by the cut
// links [D planes]; any may be null
struct TapeStep {
  void *U, *Fr;   // recovered (v, F - I) and repaired F, population precision
  void *u;        // displacement seen by the cut links, FP64: u[i * nu + t] at
                  // node un[t] (the Neumann stencil nodes), or whole planes
  const int64_t *un = nullptr;
  int64_t nu = 0;
  double *xs[2];  // projection solutions of the step (see run_projection)
  int xmode;
};
// A forward run recorded by tlvlbm_adjoint_record: the schedule, the arena
// blocks of its checkpoints, of the tape of its final steps and of the
// projection solutions, and device copies of the initial data.  Valid until
// the context changes (a step, a new state, material or boundary, another
// record); the backward pass leaves it valid.
struct AdjRec {
  bool valid = false;
  int64_t n = 0, seg = 1, tail = 0, nck = 0;
  size_t pool_next = 0;  // first arena block after the record's
  std::vector<void *> ckf, cku;
  std::vector<TapeStep> ttp;
  double *xstore = nullptr;
  size_t xslot = 0;
  std::vector<int64_t> pidx;
  double *U0 = nullptr, *dU0 = nullptr;
};
inline void rec_invalidate(tlvlbm_ctx *c) {
  if (c->rec) c->rec->valid = false;
}

// reverse-mode tape planes: one slot per node of the chunk list (embedded
// bodies) or per node
inline int64_t tape_stride(const tlvlbm_ctx *c) {
  return (c->act && c->chunks) ? (int64_t)c->nchunks * CHUNK : (int64_t)c->geo.S;
}
// dst[k * tape_stride + slot] = src[k * S + node] for k < planes (embed.hip)
void launch_tape_gather(tlvlbm_ctx *c, const void *src, void *dst, int planes);
// out[i * nu + t] = u_i at node un[t] (embed.hip)
void launch_gather_u(tlvlbm_ctx *c, const int64_t *un, int64_t nu, double *out);
// one step of Algorithm 1 (api.hip)
int step_once(tlvlbm_ctx *c, const TapeStep *tp = nullptr);
bool is_projection_step(const tlvlbm_ctx *c, int64_t step);
// reads (and synchronises on) the device error flags
tlvlbm_status check_flag(tlvlbm_ctx *c);
}  // namespace tl
