// C ABI of libbddc.so: context management and the orchestration of setup, apply
// and preconditioned CG.  Every step of the numerical path runs in the HIP
// kernels of kernels.hip; this file only allocates, uploads the host plan,
// launches and reads back status words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "bddc_internal.h"
#include "kernels.h"

using namespace bddc;

namespace {
constexpr double COARSE_CG_TOL = 1e-13;   // coarse CG: relative residual
constexpr int COARSE_CG_MAXIT = 2000;
}  // namespace

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// status of the device status word (bits DEV_*)
int device_status_error(int w) {
  if (w & DEV_WAIT_GAVE_UP)
    return fail(BDDC_EHIP, "a device-side wait (triangular-solve task or coarse-CG grid barrier) gave up (wait_polls limit)");
  return fail(BDDC_ENOCONV, "the coarse CG stopped at its iteration limit or broke down");
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(BDDC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Extreme eigenvalues of a symmetric tridiagonal matrix by Sturm bisection.
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    double off = i ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int k) {
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < d.size(); ++i) {
    double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < d.size() ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (sturm_count(d, e, mid) > k) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// CG-Lanczos tridiagonal from the CG coefficients: T[k,k] = 1/alpha_k +
// beta_{k-1}/alpha_{k-1}, T[k,k+1] = sqrt(beta_k)/alpha_k.
double lanczos_cond(const std::vector<double>& alpha, const std::vector<double>& beta) {
  const size_t m = alpha.size();
  if (m == 0) return 1.0;
  std::vector<double> d(m), e(m ? m - 1 : 0);
  for (size_t k = 0; k < m; ++k) {
    d[k] = 1.0 / alpha[k] + (k ? beta[k - 1] / alpha[k - 1] : 0.0);
    if (k + 1 < m) e[k] = std::sqrt(std::max(beta[k], 0.0)) / alpha[k];
  }
  double lmin = tridiag_eig(d, e, 0), lmax = tridiag_eig(d, e, int(m) - 1);
  return lmin > 0 ? lmax / lmin : INFINITY;
}

struct TimedFamily {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;   // eager launches (pooled events)
  std::vector<float> durations;                             // collected, not yet reported
};

// event pair recorded inside a captured graph (owned by the graph)
struct GraphTimed {
  std::string family;
  hipEvent_t b, e;
};

}  // namespace

struct bddc_ctx {
  Plan plan;
  hipStream_t st = nullptr;
  bool fp32 = false;                // local factors and triangular solves in FP32
  bool pc32 = false;                // interface form: preconditioner matrices in FP32
  bool rho_scaling = false;         // coefficient-aware weights instead of 1/kappa
  bool coarse_cg = false;           // coarse problem by CG instead of the dense factor / inverse
  int32_t *ac_rowptr = nullptr, *ac_fcol = nullptr, *ac_fsrc = nullptr;   // full CSR of A_c (coarse CG)
  double* ac_fval = nullptr;        // its values
  int ac_nfull = 0;
  double* ccg_work = nullptr;       // coarse CG vectors (7 n_c)
  bool use_graph = false;
  bool iface = true;                // interface-restricted CG (see bddc.h)
  MeshDevHost mesh{};
  std::vector<void*> allocs;
  int64_t dev_bytes = 0;
  int cus = 256;
  int grid_trsv = 1024;
  int wg_per_cu = 4;
  double *tune_b = nullptr, *tune_x = nullptr;

  double* theta = nullptr;
  int32_t *rowptr = nullptr, *col = nullptr;
  double* val = nullptr;
  uint8_t* kappa = nullptr;
  MatDesc* mats = nullptr;
  int32_t *gmap = nullptr, *lmap = nullptr, *avg_of = nullptr;
  double *wgt = nullptr, *avg_coef = nullptr, *dsc = nullptr, *wd = nullptr;
  void* tiles = nullptr;
  void* dinv = nullptr;
  double *app = nullptr, *sainv = nullptr, *sainve = nullptr, *aci = nullptr;
  int32_t *rc = nullptr, *cinv_ptr = nullptr, *cinv = nullptr, *inv_ptr = nullptr, *inv = nullptr;
  int32_t *ac_src_ptr = nullptr, *ac_src = nullptr, *ac_row = nullptr, *ac_col = nullptr, *ac_diag = nullptr;
  double *ac_val = nullptr, *dc = nullptr;
  double *ctiles = nullptr, *cdinv = nullptr;
  MatDesc* cmat = nullptr;
  MatDesc cmat_host{};
  int Tc = 0;
  int32_t *t_fwd_rr = nullptr, *t_bwd_rr = nullptr, *t_fwd_ii = nullptr, *t_bwd_ii = nullptr;
  int32_t *t_symfin = nullptr, *tinfo = nullptr, *trows_op = nullptr, *trows_pc = nullptr;
  int32_t *ifc_g = nullptr, *ifc_l = nullptr, *ifc_slotz = nullptr, *ifc_slotf = nullptr;   // interface dofs
  double *ifc_dsc = nullptr, *ifc_wd = nullptr;
  int32_t *fcol = nullptr, *fcol_ii = nullptr, *lrow_rr = nullptr, *lrow_ii = nullptr;   // factor envelopes
  int32_t *bptr = nullptr, *brows = nullptr, *btile = nullptr;   // rows of each factor column in the envelope
  int32_t *iptr = nullptr, *irows = nullptr, *itile0 = nullptr, *itile1 = nullptr;   // interior block
  EnvRow* envrow = nullptr;                     // envelope storage of each tile row
  std::vector<MatDesc> mats_dev;                // host image of the device descriptors
  double* xg = nullptr;                        // inverses of the trailing factor blocks
  double *sg = nullptr, *hg = nullptr;         // interface form: Schur complements, X^T X (+ border rows)
  float* hg32 = nullptr;                       // X^T X (+ border rows) in FP32 (pc32, instead of hg)
  double *symp = nullptr, *rowp = nullptr;     // their column / row partial products
  double *zpad = nullptr, *fpad = nullptr;     // D^{-1} z (+ corners) and W D r in padded rows
  double *cxg = nullptr, *cainv = nullptr;   // explicit coarse inverse
  double* upart = nullptr;   // u_c as csplit column-split partials (the coarse CG: one vector)
  int csplit = 1;
  double *sploc = nullptr, *cpp = nullptr;
  int max_loclen = 1;
  void* pub_local = nullptr;   // 4 * n_vec entries of the local precision
  unsigned* tickets = nullptr;
  int* fready = nullptr;            // per tile ready words of the persistent factorisation
  int wait_polls = 1 << 22;         // polls of a published value (or a coarse-CG grid barrier) before a wait gives up
  int coarse_maxit = COARSE_CG_MAXIT;
  int sym_lds_cols = SYM_LDS_COLS;     // interface mat-vec: columns summed in LDS (test limit)
  int sym_row_pieces = SYM_ROW_PIECES; // interface mat-vec: row pieces kept in LDS (test limit)
  unsigned* fticket = nullptr;
  void* static_scratch = nullptr;   // this device's fixed workspace (bddc_apply_noalloc)
  double *part = nullptr, *gbuf = nullptr, *mu = nullptr, *coef = nullptr, *ww = nullptr, *v12 = nullptr;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *tmp = nullptr;
  double *part_a = nullptr, *part_b = nullptr, *part_c = nullptr, *scal = nullptr;
  PcgScalars* sc = nullptr;
  int* err = nullptr;
  double t_setup_ms = 0.0;
  double factor_ms = 0.0;           // GPU time of the batched local factorisation at setup

  // HIP graphs of chunks of PCG iterations (use_graph): graph k holds iterations
  // [k*GRAPH_CHUNK, (k+1)*GRAPH_CHUNK) of a solve, replayed on gst, which is
  // joined to the ctx stream with events.  The iterate lives in xw so that the
  // captured kernel arguments stay valid from one solve to the next.
  static constexpr int GRAPH_CHUNK = 4;
  hipStream_t gst = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<hipGraphExec_t> graphs;      // index 2k: untimed, 2k+1: with timing events
  std::vector<hipGraph_t> graph_defs;
  std::vector<std::vector<GraphTimed>> graph_timed;
  double* xw = nullptr;
  // mapped pinned host memory: the word the iteration sets when the solve ends,
  // and the scalars read back at the end of a CG segment (5 + 3 MAX_PCG_IT)
  int* hdone = nullptr;
  int* hdone_dev = nullptr;
  double* hback = nullptr;
  double* hback_dev = nullptr;
  hipEvent_t snap_ev[2] = {nullptr, nullptr};

  bool timing = false;
  std::map<std::string, TimedFamily> fam;
  std::vector<hipEvent_t> event_pool;

  ~bddc_ctx() {
    for (hipGraphExec_t g : graphs)
      if (g) hipGraphExecDestroy(g);
    for (hipGraph_t g : graph_defs)
      if (g) hipGraphDestroy(g);
    for (auto& v : graph_timed)
      for (auto& gt : v) {
        hipEventDestroy(gt.b);
        hipEventDestroy(gt.e);
      }
    if (ev_in) hipEventDestroy(ev_in);
    for (hipEvent_t e : snap_ev)
      if (e) hipEventDestroy(e);
    if (hdone) hipHostFree(hdone);
    if (hback) hipHostFree(hback);
    if (ev_out) hipEventDestroy(ev_out);
    if (gst) hipStreamDestroy(gst);
    for (auto& kv : fam)
      for (auto& pr : kv.second.pending) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
      }
    for (hipEvent_t e : event_pool) hipEventDestroy(e);
    for (void* a : allocs) hipFree(a);
  }

  template <typename T>
  int alloc(T*& ptr, int64_t count) {
    ptr = nullptr;
    if (count <= 0) count = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, size_t(count) * sizeof(T));
    if (e != hipSuccess) return fail(BDDC_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    allocs.push_back(p);
    dev_bytes += count * int64_t(sizeof(T));
    ptr = static_cast<T*>(p);
    return BDDC_OK;
  }
  template <typename T>
  int upload(T*& ptr, const std::vector<T>& host) {
    int rc_ = alloc(ptr, int64_t(host.size()));
    if (rc_) return rc_;
    if (!host.empty()) HIP_TRY(hipMemcpyAsync(ptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return BDDC_OK;
  }

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
  }
  // event pair around a launch of a named family when timing is on
  // Event pairs around launches of a named family when timing is on.  Inside a
  // graph capture the events become nodes of the graph (fresh events owned by it).
  std::vector<GraphTimed>* capture_timed = nullptr;
  std::vector<GraphTimed> graph_pending;
  hipEvent_t begin(const char* name) {
    if (!timing) return nullptr;
    hipEvent_t e = nullptr;
    if (capture_timed) hipEventCreate(&e);
    else e = get_event();
    hipEventRecord(e, st);
    return e;
  }
  // a start/stop pair that the kernel dispatch itself records (the kernel's own
  // duration, without the queue gap in front of it)
  void kernel_events(const char* name, hipEvent_t* b, hipEvent_t* e) {
    *b = *e = nullptr;
    if (!timing || capture_timed) return;
    *b = get_event();
    *e = get_event();
    fam[name].pending.push_back({*b, *e});
  }
  void end(const char* name, hipEvent_t b) {
    if (!timing || !b) return;
    hipEvent_t e = nullptr;
    if (capture_timed) {
      hipEventCreate(&e);
      hipEventRecord(e, st);
      capture_timed->push_back({name, b, e});
      return;
    }
    e = get_event();
    hipEventRecord(e, st);
    fam[name].pending.push_back({b, e});
  }
  void collect() {
    hipStreamSynchronize(st);
    for (auto& kv : fam) {
      for (auto& pr : kv.second.pending) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, pr.first, pr.second);
        kv.second.durations.push_back(ms);
        event_pool.push_back(pr.first);
        event_pool.push_back(pr.second);
      }
      kv.second.pending.clear();
    }
    for (auto& gt : graph_pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, gt.b, gt.e) == hipSuccess) fam[gt.family].durations.push_back(ms);
    }
    graph_pending.clear();
  }
};

namespace {

TrsvArgs base_args(bddc_ctx* c) {
  TrsvArgs a;
  std::memset(&a, 0, sizeof(a));
  a.mats = c->mats;
  a.tiles = c->tiles;
  a.dinv = c->dinv;
  a.gmap = c->gmap;
  a.wd = c->wd;
  a.dsc = c->dsc;
  a.rowptr = c->rowptr;
  a.colind = c->col;
  a.vals = c->val;
  a.werr = c->err + 3;
  a.spin = c->wait_polls;
  return a;
}

void* pub_slot(bddc_ctx* c, int i) {
  const size_t es = c->fp32 ? sizeof(float) : sizeof(double);
  return static_cast<char*>(c->pub_local) + size_t(i) * size_t(c->plan.n_vec) * es;
}

// Buffers of one preconditioner application that start over at every call.
struct ApplyWs {
  void* pub_local;      // 4 * n_vec entries of the local precision
  unsigned* tickets;    // 8 counters
};

int trsv_grid(bddc_ctx* c, int ntasks) { return std::max(1, std::min(ntasks, c->grid_trsv)); }
// Interior passes: one chain of tile rows per subdomain, each task waiting on the
// previous rows of its own chain; about four tasks in flight per chain keep
// every chain busy, and more workgroups only add polling traffic (measured on
// the 64^3 workload: 64 chains, 256 workgroups beat 512 and 768).
int trsv_grid_ii(bddc_ctx* c, int ntasks) {
  const int want = std::max(c->cus, 4 * c->plan.nsubs);
  return std::max(1, std::min(ntasks, std::min(want, c->grid_trsv)));
}

// z = M^{-1} r (paper Sec. 2): v1 + v2 through the forward solve, the coarse
// problem and the backward solve, then v3 on subdomain interiors.
// ws: where the per-application buffers live (published solutions, tickets);
// NULL: the ctx's own.  With ws no event is recorded.
void enqueue_apply(bddc_ctx* c, const double* r, double* z, const int* done, const ApplyWs* ws = nullptr) {
  const Plan& P = c->plan;
  hipStream_t st = c->st;
  ApplyWs own{c->pub_local, c->tickets};
  const ApplyWs& W = ws ? *ws : own;
  const bool events = ws == nullptr;
  auto slot = [&](int i) -> void* {
    const size_t es = c->fp32 ? sizeof(float) : sizeof(double);
    return static_cast<char*>(W.pub_local) + size_t(i) * size_t(P.n_vec) * es;
  };
  hipEvent_t ea = events ? c->begin("apply") : nullptr;
  if (c->fp32) launch_fill_sentinel<float>(static_cast<float*>(W.pub_local), 4 * P.n_vec, st);
  else launch_fill_sentinel<double>(static_cast<double*>(W.pub_local), 4 * P.n_vec, st);
  launch_fill<unsigned>(W.tickets, 0u, 8, st);

  // forward solve with A_RR: t = L^{-1} D W_i R_i r, border partials W^T t
  TrsvArgs a = base_args(c);
  a.done = done;
  a.tasks = c->t_fwd_rr;
  a.fcol = c->fcol;
  a.ntasks = int(P.fwd_rr.size() / 2);
  a.ticket = W.tickets + 0;
  a.sol = slot(0);
  a.rin = r;
  a.part = c->part;
  {
    hipEvent_t k0 = nullptr, k1 = nullptr;
    if (events) c->kernel_events("trsv_fwd_rr", &k0, &k1);
    launch_trsv(TRSV_FWD_RR, c->fp32, a, trsv_grid(c, a.ntasks), st, k0, k1);
  }

  if (P.n_coarse > 0) {
    launch_coarse_prep(c->mats, P.nsubs, c->part, c->sainv, c->sainve, c->gmap, c->wgt, r, c->gbuf, c->mu, done, nullptr,
                       0, 0, st);
    // u_c = A_c^{-1} r_c: the explicit inverse (column-split partials), or the coarse CG
    if (c->coarse_cg)
      launch_coarse_cg(c->ac_rowptr, c->ac_fcol, c->ac_fval, c->ac_nfull, c->dc, P.n_coarse, c->cinv_ptr, c->cinv,
                       c->gbuf, c->upart, c->ccg_work, COARSE_CG_TOL, c->coarse_maxit, c->wait_polls, done,
                       c->err + 3, st);
    else
      launch_coarse_gemv(c->cainv, P.n_coarse, c->csplit, c->cinv_ptr, c->cinv, c->gbuf, c->upart, done, st);
    launch_coarse_coef(c->mats, P.nsubs, c->rc, c->upart, P.n_coarse, c->csplit, c->mu, c->sainv, c->sainve,
                       c->wgt, c->coef, c->ww, done, st);
  }
  // backward solve: D L^{-T} (t + W coef) = z_R + Phi_R u (weighted)
  a = base_args(c);
  a.done = done;
  a.tasks = c->t_bwd_rr;
  a.lrow = c->lrow_rr;
  a.bptr = c->bptr;
  a.brows = c->brows;
  a.btile = c->btile;
  a.ntasks = int(P.bwd_rr.size() / 2);
  a.ticket = W.tickets + 1;
  a.sol = slot(1);
  a.src = slot(0);
  a.coef = c->coef;
  a.ww = c->ww;
  {
    hipEvent_t k0 = nullptr, k1 = nullptr;
    if (events) c->kernel_events("trsv_bwd_rr", &k0, &k1);
    launch_trsv(TRSV_BWD_RR, c->fp32, a, trsv_grid(c, a.ntasks), st, k0, k1);
  }
  // v1 + v2 = sum_i R_i^T W_i w_i
  launch_gather_v12(c->inv_ptr, c->inv, c->ww, c->kappa, c->v12, z, P.n_free, done, st);
  // v3: interior solves of r1 = r - A (v1 + v2)
  a = base_args(c);
  a.done = done;
  a.tasks = c->t_fwd_ii;
  a.fcol = c->fcol_ii;
  a.ntasks = int(P.fwd_ii.size() / 2);
  a.ticket = W.tickets + 2;
  a.sol = slot(2);
  a.rin = r;
  a.v12 = c->v12;
  {
    hipEvent_t k0 = nullptr, k1 = nullptr;
    if (events) c->kernel_events("trsv_fwd_ii", &k0, &k1);
    launch_trsv(TRSV_FWD_II, c->fp32, a, trsv_grid_ii(c, a.ntasks), st, k0, k1);
  }
  a = base_args(c);
  a.done = done;
  a.tasks = c->t_bwd_ii;
  a.lrow = c->lrow_ii;
  a.iptr = c->iptr;
  a.irows = c->irows;
  a.itile0 = c->itile0;
  a.itile1 = c->itile1;
  a.ntasks = int(P.bwd_ii.size() / 2);
  a.ticket = W.tickets + 3;
  a.sol = slot(3);
  a.src = slot(2);
  a.zout = z;
  a.base = c->v12;
  {
    hipEvent_t k0 = nullptr, k1 = nullptr;
    if (events) c->kernel_events("trsv_bwd_ii", &k0, &k1);
    launch_trsv(TRSV_BWD_II, c->fp32, a, trsv_grid_ii(c, a.ntasks), st, k0, k1);
  }
  if (events) c->end("apply", ea);
}

IfcArgs ifc_args(bddc_ctx* c) {
  IfcArgs a;
  std::memset(&a, 0, sizeof(a));
  a.g = c->ifc_g;
  a.l = c->ifc_l;
  a.slotz = c->ifc_slotz;
  a.slotf = c->ifc_slotf;
  a.dsc = c->ifc_dsc;
  a.wd = c->ifc_wd;
  a.n = int64_t(c->plan.ifc_g.size());
  a.sc = c->sc;
  a.sploc = c->sploc;
  a.r = c->r;
  a.z = c->z;
  a.p = c->p;
  a.q = c->q;
  a.zpad = c->zpad;
  a.fpad = c->fpad;
  return a;
}

IfaceArgs iface_args(bddc_ctx* c) {
  IfaceArgs a;
  std::memset(&a, 0, sizeof(a));
  a.mats = c->mats;
  a.tinfo = c->tinfo;
  a.ntiles = c->plan.n_sg;
  a.nwg = int(std::min<int64_t>(c->grid_trsv, c->plan.n_sg));
  a.rowp = c->rowp;
  a.check_it = -1;
  a.sc = c->sc;
  a.part = c->symp;
  a.dsc = c->dsc;
  a.wd = c->wd;
  a.wgt = c->wgt;
  a.sploc = c->sploc;
  a.ww = c->ww;
  a.lds_cols = c->sym_lds_cols;
  a.row_pieces = c->sym_row_pieces;
  return a;
}

// Interface preconditioner (v1 + v2 restricted to interface dofs) on an
// interface residual r (its f = W D r already in the padded input fpad): the
// products of X^T X and of the constraint rows W_G^T X with f, the coarse
// problem, then x = X^T X f + X^T W_G coef weighted into ww, gathered into z
// (interface entries) with the partial sums of r.z.  check_it >= 0: the
// mat-vec first takes the convergence decision of that CG iteration.
void enqueue_apply_iface(bddc_ctx* c, const double* r, double* z, double* part_rz, const int* done,
                         int check_it = -1) {
  const Plan& P = c->plan;
  hipStream_t st = c->st;
  hipEvent_t ea = c->begin("apply");
  IfaceArgs a = iface_args(c);
  a.m = c->pc32 ? static_cast<const void*>(c->hg32) : c->hg;
  a.m32 = c->pc32 ? 1 : 0;
  a.trows = c->trows_pc;
  a.xpad = c->fpad;
  a.check_it = check_it;
  a.hdone = check_it >= 0 ? c->hdone_dev : nullptr;
  a.part_rr = c->part_b;
  a.nparts_rr = ifc_blocks(int64_t(P.ifc_g.size()));
  {
    hipEvent_t k0, k1;
    c->kernel_events("pc", &k0, &k1);
    launch_sym_mv(a, st, k0, k1);
  }
  if (P.n_coarse > 0) {
    launch_coarse_prep(c->mats, P.nsubs, nullptr, c->sainv, c->sainve, c->gmap, c->wgt, r, c->gbuf, c->mu, done,
                       c->rowp, a.ntiles, a.nwg, st);
    if (c->coarse_cg)
      launch_coarse_cg(c->ac_rowptr, c->ac_fcol, c->ac_fval, c->ac_nfull, c->dc, P.n_coarse, c->cinv_ptr, c->cinv,
                       c->gbuf, c->upart, c->ccg_work, COARSE_CG_TOL, c->coarse_maxit, c->wait_polls, done,
                       c->err + 3, st);
    else
      launch_coarse_gemv(c->cainv, P.n_coarse, c->csplit, c->cinv_ptr, c->cinv, c->gbuf, c->upart, done, st);
    launch_coarse_coef(c->mats, P.nsubs, c->rc, c->upart, P.n_coarse, c->csplit, c->mu, c->sainv, c->sainve,
                       c->wgt, c->coef, c->ww, done, st);
  }
  a.coef = c->coef;
  a.tasks = c->t_symfin;
  a.ntasks = int(P.symfin.size() / 2);
  launch_pc_finish(a, st);
  {
    IfcArgs g = ifc_args(c);
    g.ww = c->ww;
    g.r = const_cast<double*>(r);
    g.z = z;
    g.part_out = part_rz;
    launch_gather_z_ifc(g, st);
  }
  c->end("apply", ea);
}

// q = S p with p = z + beta p (iteration it), partial sums of p.q into part_pq:
// S z from the explicit local Schur complements, then q = S z + beta q
void enqueue_schur(bddc_ctx* c, int it, bool fresh, const double* part_rz, double* part_pq) {
  const Plan& P = c->plan;
  hipStream_t st = c->st;
  hipEvent_t e = c->begin("schur");
  IfaceArgs a = iface_args(c);
  a.m = c->sg;
  a.trows = c->trows_op;
  a.xpad = c->zpad;
  {
    hipEvent_t k0, k1;
    c->kernel_events("op", &k0, &k1);
    launch_sym_mv(a, st, k0, k1);
  }
  a.tasks = c->t_symfin;
  a.ntasks = int(P.symfin.size() / 2);
  launch_op_finish(a, st);
  {
    IfcArgs g = ifc_args(c);
    g.it = it;
    g.fresh = fresh ? 1 : 0;
    g.part_in = part_rz;
    g.part_out = part_pq;
    launch_gather_sp_ifc(g, st);
  }
  c->end("schur", e);
}

// x = P_I b: interior solves of b, zero on the interface
// (zero: optional vector set to zero by the same first launch)
void enqueue_interior_guess(bddc_ctx* c, const double* b, double* x, double* zero = nullptr) {
  const Plan& P = c->plan;
  hipStream_t st = c->st;
  launch_reset(c->fp32, pub_slot(c, 2), 2 * P.n_vec, nullptr, 0, c->tickets, nullptr, st, c->kappa, x, zero,
               P.n_free);
  TrsvArgs a = base_args(c);
  a.tasks = c->t_fwd_ii;
  a.fcol = c->fcol_ii;
  a.ntasks = int(P.fwd_ii.size() / 2);
  a.ticket = c->tickets + 2;
  a.sol = pub_slot(c, 2);
  a.rin = b;
  hipEvent_t k0, k1;
  c->kernel_events("trsv_fwd_ii", &k0, &k1);
  launch_trsv(TRSV_FWD_II, c->fp32, a, trsv_grid_ii(c, a.ntasks), st, k0, k1);
  a = base_args(c);
  a.tasks = c->t_bwd_ii;
  a.lrow = c->lrow_ii;
  a.iptr = c->iptr;
  a.irows = c->irows;
  a.itile0 = c->itile0;
  a.itile1 = c->itile1;
  a.ntasks = int(P.bwd_ii.size() / 2);
  a.ticket = c->tickets + 3;
  a.sol = pub_slot(c, 3);
  a.src = pub_slot(c, 2);
  a.zout = x;
  c->kernel_events("trsv_bwd_ii", &k0, &k1);
  launch_trsv(TRSV_BWD_II, c->fp32, a, trsv_grid_ii(c, a.ntasks), st, k0, k1);
}

// one PCG iteration it (fresh: first of a segment, p = z)
void enqueue_iteration(bddc_ctx* c, double* x, int it, bool fresh) {
  hipStream_t st = c->st;
  const int64_t n = c->plan.n_free;
  const int* done = &c->sc->done;
  if (c->iface) {
    enqueue_schur(c, it, fresh, c->part_c, c->part_a);
  } else {
    hipEvent_t e = c->begin("spmv");
    launch_pcg_dir(c->rowptr, c->col, c->val, c->z, c->p, c->q, c->part_c, c->part_a, c->sc, it, fresh ? 1 : 0, n,
                   st);
    c->end("spmv", e);
  }
  if (c->iface) {
    IfcArgs g = ifc_args(c);
    g.x = x;
    g.it = it;
    g.part_in = c->part_a;
    g.part_out = c->part_b;
    launch_pcg_update_ifc(g, st);
    // the preconditioner's mat-vec takes this iteration's convergence decision
    enqueue_apply_iface(c, c->r, c->z, c->part_c, done, it);
  } else {
    launch_pcg_update(x, c->r, c->p, c->q, c->part_a, c->part_b, c->sc, it, n, st);
    launch_pcg_check(c->part_b, c->sc, it, c->hdone_dev, st);
    enqueue_apply(c, c->r, c->z, done);
    launch_dot(c->r, c->z, c->part_c, n, done, st);
  }
}

// Replays (capturing on first use) the graph of iterations
// [k*GRAPH_CHUNK, (k+1)*GRAPH_CHUNK); x must be c->xw.
int launch_chunk_graph(bddc_ctx* c, double* x, int k) {
  if (!c->gst) {
    HIP_TRY(hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  }
  const int slot = k;
  if (int(c->graphs.size()) <= slot) {
    c->graphs.resize(slot + 1, nullptr);
    c->graph_defs.resize(slot + 1, nullptr);
    c->graph_timed.resize(slot + 1);
  }
  if (!c->graphs[slot]) {
    hipStream_t user = c->st;
    c->st = c->gst;
    hipError_t e = hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int i = 0; i < bddc_ctx::GRAPH_CHUNK; ++i) {
        const int it = k * bddc_ctx::GRAPH_CHUNK + i;
        enqueue_iteration(c, x, it, it == 0);
      }
    }
    hipGraph_t g = nullptr;
    if (e == hipSuccess) e = hipStreamEndCapture(c->gst, &g);
    c->st = user;
    if (e != hipSuccess) return fail(BDDC_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    HIP_TRY(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    c->graph_defs[slot] = g;
    c->graphs[slot] = ex;
  }
  HIP_TRY(hipEventRecord(c->ev_in, c->st));
  HIP_TRY(hipStreamWaitEvent(c->gst, c->ev_in, 0));
  HIP_TRY(hipGraphLaunch(c->graphs[slot], c->gst));
  HIP_TRY(hipEventRecord(c->ev_out, c->gst));
  HIP_TRY(hipStreamWaitEvent(c->st, c->ev_out, 0));
  return BDDC_OK;
}

// out = xt + P_I (b - A xt) on interior dofs, xt on the interface (xt is zero on
// interior dofs); out may be xt itself
void enqueue_interior_complete(bddc_ctx* c, const double* b, const double* xt, double* out) {
  const Plan& P = c->plan;
  hipStream_t st = c->st;
  if (out != xt) hipMemcpyAsync(out, xt, P.n_free * sizeof(double), hipMemcpyDeviceToDevice, st);
  launch_reset(c->fp32, pub_slot(c, 2), 2 * P.n_vec, nullptr, 0, c->tickets, nullptr, st);
  TrsvArgs a = base_args(c);
  a.tasks = c->t_fwd_ii;
  a.fcol = c->fcol_ii;
  a.ntasks = int(P.fwd_ii.size() / 2);
  a.ticket = c->tickets + 2;
  a.sol = pub_slot(c, 2);
  a.rin = b;
  a.v12 = xt;
  hipEvent_t k0, k1;
  c->kernel_events("trsv_fwd_ii", &k0, &k1);
  launch_trsv(TRSV_FWD_II, c->fp32, a, trsv_grid_ii(c, a.ntasks), st, k0, k1);
  a = base_args(c);
  a.tasks = c->t_bwd_ii;
  a.lrow = c->lrow_ii;
  a.iptr = c->iptr;
  a.irows = c->irows;
  a.itile0 = c->itile0;
  a.itile1 = c->itile1;
  a.ntasks = int(P.bwd_ii.size() / 2);
  a.ticket = c->tickets + 3;
  a.sol = pub_slot(c, 3);
  a.src = pub_slot(c, 2);
  a.zout = out;
  a.base = xt;
  c->kernel_events("trsv_bwd_ii", &k0, &k1);
  launch_trsv(TRSV_BWD_II, c->fp32, a, trsv_grid_ii(c, a.ntasks), st, k0, k1);
}

int do_setup(bddc_ctx* c, const bddc_coefficients* coef) {
  Plan& P = c->plan;
  hipStream_t st = c->st;
  int rc_;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  c->cus = prop.multiProcessorCount;
  c->grid_trsv = std::max(64, c->cus * c->wg_per_cu);

  // coefficients
  if ((rc_ = c->alloc(c->theta, P.n_el))) return rc_;
  HIP_TRY(hipMemcpyAsync(c->theta, coef->theta, size_t(P.n_el) * sizeof(double),
                         coef->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if ((rc_ = c->alloc(c->err, 4))) return rc_;
  launch_fill<int>(c->err, 0, 4, st);
  launch_check_theta(c->theta, P.n_el, c->err, st);

  // plan arrays
  if ((rc_ = c->upload(c->rowptr, P.rowptr))) return rc_;
  if ((rc_ = c->alloc(c->col, P.nnz))) return rc_;
  if ((rc_ = c->alloc(c->val, P.nnz))) return rc_;
  if ((rc_ = c->upload(c->kappa, P.kappa))) return rc_;
  // descriptors with device copies of the envelope tables (uploaded below)
  if ((rc_ = c->upload(c->fcol, P.fcol))) return rc_;
  if ((rc_ = c->upload(c->envrow, P.envrow))) return rc_;
  c->mats_dev = P.subs;
  for (auto& D : c->mats_dev) {
    D.env = c->envrow + D.vec_off / NB;
  }
  if ((rc_ = c->upload(c->mats, c->mats_dev))) return rc_;
  if ((rc_ = c->upload(c->gmap, P.gmap))) return rc_;
  if ((rc_ = c->upload(c->lmap, P.lmap))) return rc_;
  if ((rc_ = c->upload(c->avg_of, P.avg_of))) return rc_;
  if ((rc_ = c->upload(c->wgt, P.weight))) return rc_;
  if ((rc_ = c->upload(c->avg_coef, P.avg_coef))) return rc_;
  if ((rc_ = c->alloc(c->dsc, P.n_loc))) return rc_;
  if ((rc_ = c->alloc(c->wd, P.n_loc))) return rc_;
  if ((rc_ = c->upload(c->rc, P.rc))) return rc_;
  if ((rc_ = c->upload(c->cinv_ptr, P.cinv_ptr))) return rc_;
  if ((rc_ = c->upload(c->cinv, P.cinv))) return rc_;
  if ((rc_ = c->upload(c->inv_ptr, P.inv_ptr))) return rc_;
  if ((rc_ = c->upload(c->inv, P.inv))) return rc_;
  if ((rc_ = c->upload(c->ac_src_ptr, P.ac_src_ptr))) return rc_;
  if ((rc_ = c->upload(c->ac_src, P.ac_src))) return rc_;
  if ((rc_ = c->upload(c->ac_row, P.ac_row))) return rc_;
  if ((rc_ = c->upload(c->ac_col, P.ac_col))) return rc_;
  if ((rc_ = c->upload(c->ac_diag, P.ac_diag))) return rc_;
  if ((rc_ = c->upload(c->t_fwd_rr, P.fwd_rr))) return rc_;
  if ((rc_ = c->upload(c->t_bwd_rr, P.bwd_rr))) return rc_;
  if ((rc_ = c->upload(c->t_fwd_ii, P.fwd_ii))) return rc_;
  if ((rc_ = c->upload(c->t_bwd_ii, P.bwd_ii))) return rc_;
  if ((rc_ = c->upload(c->tinfo, P.tinfo))) return rc_;
  if ((rc_ = c->upload(c->trows_op, P.trows_op))) return rc_;
  if ((rc_ = c->upload(c->trows_pc, P.trows_pc))) return rc_;
  if ((rc_ = c->upload(c->ifc_g, P.ifc_g))) return rc_;
  if ((rc_ = c->upload(c->ifc_l, P.ifc_l))) return rc_;
  if ((rc_ = c->upload(c->ifc_slotz, P.ifc_slotz))) return rc_;
  if ((rc_ = c->upload(c->ifc_slotf, P.ifc_slotf))) return rc_;
  if ((rc_ = c->upload(c->fcol_ii, P.fcol_ii))) return rc_;
  if ((rc_ = c->upload(c->lrow_rr, P.lrow_rr))) return rc_;
  if ((rc_ = c->upload(c->bptr, P.bptr))) return rc_;
  if ((rc_ = c->upload(c->brows, P.brows))) return rc_;
  if ((rc_ = c->upload(c->btile, P.btile))) return rc_;
  if ((rc_ = c->upload(c->iptr, P.iptr))) return rc_;
  if ((rc_ = c->upload(c->irows, P.irows))) return rc_;
  if ((rc_ = c->upload(c->itile0, P.itile0))) return rc_;
  if ((rc_ = c->upload(c->itile1, P.itile1))) return rc_;
  if ((rc_ = c->upload(c->lrow_ii, P.lrow_ii))) return rc_;
  if ((rc_ = c->upload(c->t_symfin, P.symfin))) return rc_;

  // global matrix
  launch_assemble_csr(c->mesh, c->theta, c->rowptr, c->col, c->val, P.n_free, c->err, st);

  // local matrices, tiles zero-filled first
  const int64_t tile_elems = P.n_tiles * NB * NB;
  const int64_t dinv_elems = P.n_dinv * NB * NB;
  if (c->fp32) {
    float *t, *d;
    if ((rc_ = c->alloc(t, tile_elems))) return rc_;
    if ((rc_ = c->alloc(d, dinv_elems))) return rc_;
    launch_fill<float>(t, 0.f, tile_elems, st);
    c->tiles = t;
    c->dinv = d;
    float* pl;
    if ((rc_ = c->alloc(pl, 4 * P.n_vec))) return rc_;
    c->pub_local = pl;
  } else {
    double *t, *d;
    if ((rc_ = c->alloc(t, tile_elems))) return rc_;
    if ((rc_ = c->alloc(d, dinv_elems))) return rc_;
    launch_fill<double>(t, 0.0, tile_elems, st);
    c->tiles = t;
    c->dinv = d;
    double* pl;
    if ((rc_ = c->alloc(pl, 4 * P.n_vec))) return rc_;
    c->pub_local = pl;
  }
  const int64_t small = int64_t(P.nsubs) * MAX_NCI * MAX_NCI;
  if ((rc_ = c->alloc(c->app, small))) return rc_;
  if ((rc_ = c->alloc(c->sainv, small))) return rc_;
  if ((rc_ = c->alloc(c->sainve, small))) return rc_;
  if ((rc_ = c->alloc(c->aci, small))) return rc_;
  launch_fill<double>(c->app, 0.0, small, st);
  launch_fill<double>(c->aci, 0.0, small, st);
  int max_ni = 1;
  for (auto& D : P.subs) max_ni = std::max(max_ni, int(D.n_i));
  if (c->rho_scaling) {
    double* rho;
    if ((rc_ = c->alloc(rho, P.n_loc))) return rc_;
    launch_rho_weights(c->mesh, c->theta, c->mats, P.nsubs, max_ni, c->gmap, c->inv_ptr, c->inv, P.n_free, rho,
                       c->wgt, st);
  }
  launch_local_assembly(c->mesh, c->theta, c->mats, P.nsubs, max_ni, c->gmap, c->lmap, c->wgt, c->dsc, c->wd,
                        c->avg_of, c->avg_coef, c->tiles, c->fp32, c->app, c->err + 1, st);
  if ((rc_ = c->alloc(c->ifc_dsc, int64_t(P.ifc_l.size()) + 1))) return rc_;
  if ((rc_ = c->alloc(c->ifc_wd, int64_t(P.ifc_l.size()) + 1))) return rc_;
  launch_ifc_setup(c->ifc_l, c->dsc, c->wd, c->ifc_dsc, c->ifc_wd, int64_t(P.ifc_g.size()), st);
  hipEvent_t f0 = nullptr, f1 = nullptr;
  HIP_TRY(hipEventCreate(&f0));
  HIP_TRY(hipEventCreate(&f1));
  HIP_TRY(hipEventRecord(f0, st));
  {
    // one persistent launch factors every local matrix (two workgroups per CU:
    // each holds two tiles in LDS)
    int32_t* ftasks = nullptr;
    if ((rc_ = c->upload(ftasks, P.factor_tasks))) return rc_;
    if ((rc_ = c->alloc(c->fready, P.n_tiles))) return rc_;
    if ((rc_ = c->alloc(c->fticket, 1))) return rc_;
    launch_factor_persistent(c->mats, c->tiles, c->dinv, c->fp32, c->fcol, ftasks, int(P.factor_tasks.size() / 3),
                             c->fticket, c->fready, P.n_tiles, 2 * c->cus, c->err + 1, st);
  }
  HIP_TRY(hipEventRecord(f1, st));
  if ((rc_ = c->alloc(c->cpp, small))) return rc_;
  launch_local_small(c->mats, P.nsubs, c->tiles, c->fp32, c->app, c->sainv, c->sainve, c->aci, c->cpp, c->err + 1,
                     st);
  if (c->iface) {
    if ((rc_ = c->alloc(c->xg, P.n_xg * NB * NB))) return rc_;
    launch_trailing_inverse(c->mats, P.nsubs, P.maxTG, static_cast<const double*>(c->tiles),
                            static_cast<const double*>(c->dinv), c->xg, st);
    if ((rc_ = c->alloc(c->sg, P.n_sg * NB * NB))) return rc_;
    if (c->pc32) {
      if ((rc_ = c->alloc(c->hg32, P.n_sg * NB * NB))) return rc_;
    } else if ((rc_ = c->alloc(c->hg, P.n_sg * NB * NB))) {
      return rc_;
    }
    if ((rc_ = c->alloc(c->symp, P.n_sg * NB))) return rc_;
    if ((rc_ = c->alloc(c->rowp, P.n_sg * NB))) return rc_;
    launch_sym_build(SYM_OP, c->mats, P.nsubs, P.maxTS, static_cast<const double*>(c->tiles), c->xg, c->cpp, c->sg,
                     false, st);
    launch_sym_build(SYM_PC, c->mats, P.nsubs, P.maxTS, static_cast<const double*>(c->tiles), c->xg, c->cpp,
                     c->pc32 ? static_cast<void*>(c->hg32) : c->hg, c->pc32, st);
  }

  // coarse problem
  const int nc = P.n_coarse;
  c->Tc = (nc + NB - 1) / NB;
  std::memset(&c->cmat_host, 0, sizeof(MatDesc));
  c->cmat_host.T = c->Tc;
  c->cmat_host.Tx = c->Tc;
  c->cmat_host.n_R = nc;
  std::vector<MatDesc> cm(1, c->cmat_host);
  if ((rc_ = c->upload(c->cmat, cm))) return rc_;
  if ((rc_ = c->alloc(c->ac_val, int64_t(P.ac_row.size())))) return rc_;
  if (c->coarse_cg) {
    // CSR of the full symmetric A_c over its stored lower-triangle entries
    struct FE { int32_t r, q, e; };
    std::vector<FE> fe;
    for (size_t e = 0; e < P.ac_row.size(); ++e) {
      fe.push_back({P.ac_row[e], P.ac_col[e], int32_t(e)});
      if (P.ac_row[e] != P.ac_col[e]) fe.push_back({P.ac_col[e], P.ac_row[e], int32_t(e)});
    }
    std::sort(fe.begin(), fe.end(), [](const FE& x, const FE& y) { return x.r != y.r ? x.r < y.r : x.q < y.q; });
    std::vector<int32_t> rp(nc + 1, 0), fc, fs;
    for (const FE& f : fe) {
      ++rp[f.r + 1];
      fc.push_back(f.q);
      fs.push_back(f.e);
    }
    for (int p = 0; p < nc; ++p) rp[p + 1] += rp[p];
    if ((rc_ = c->upload(c->ac_rowptr, rp))) return rc_;
    if ((rc_ = c->upload(c->ac_fcol, fc))) return rc_;
    if ((rc_ = c->upload(c->ac_fsrc, fs))) return rc_;
    c->ac_nfull = int(fs.size());
    if ((rc_ = c->alloc(c->ac_fval, int64_t(fs.size())))) return rc_;
    if ((rc_ = c->alloc(c->ccg_work, 7 * int64_t(nc) + 3 * 64 + 8))) return rc_;
  }
  if ((rc_ = c->alloc(c->dc, nc))) return rc_;
  // (the coarse CG needs no dense coarse factor)
  if ((rc_ = c->alloc(c->ctiles, c->coarse_cg ? 1 : tri_tile(c->Tc, 0) * NB * NB))) return rc_;
  if ((rc_ = c->alloc(c->cdinv, c->coarse_cg ? 1 : int64_t(c->Tc) * NB * NB))) return rc_;
  if (nc > 0 && c->coarse_cg) {
    launch_coarse_assembly(c->ac_src_ptr, c->ac_src, c->ac_row, c->ac_col, c->ac_diag, int(P.ac_row.size()), nc,
                           c->aci, c->ac_val, c->dc, nullptr, c->err + 2, st);
    launch_coarse_cg_matrix(c->ac_fsrc, c->ac_val, c->ac_fval, c->ac_nfull, st);
    if ((rc_ = c->alloc(c->upart, nc))) return rc_;
  } else if (nc > 0) {
    launch_fill<double>(c->ctiles, 0.0, tri_tile(c->Tc, 0) * NB * NB, st);
    launch_pad_identity(c->cmat, 1, c->ctiles, false, st);
    launch_coarse_assembly(c->ac_src_ptr, c->ac_src, c->ac_row, c->ac_col, c->ac_diag, int(P.ac_row.size()), nc,
                           c->aci, c->ac_val, c->dc, c->ctiles, c->err + 2, st);
    {
      std::vector<int32_t> ct;
      std::string terr;
      if ((rc_ = make_factor_tasks(cm, nullptr, ct, terr))) return fail(rc_, terr);
      int32_t* ctasks = nullptr;
      int* cready = nullptr;
      if ((rc_ = c->upload(ctasks, ct))) return rc_;
      if ((rc_ = c->alloc(cready, tri_tile(c->Tc, 0)))) return rc_;
      launch_factor_persistent(c->cmat, c->ctiles, c->cdinv, false, nullptr, ctasks, int(ct.size() / 3), c->fticket,
                               cready, tri_tile(c->Tc, 0), 2 * c->cus, c->err + 2, st);
    }
    {
      // A_c^{-1} = D X^T X D, X = inverse of the coarse Cholesky factor
      if ((rc_ = c->alloc(c->cxg, tri_tile(c->Tc, 0) * NB * NB))) return rc_;
      if ((rc_ = c->alloc(c->cainv, int64_t(nc) * nc))) return rc_;
      c->csplit = (nc + COARSE_SPLIT_COLS - 1) / COARSE_SPLIT_COLS;
      if ((rc_ = c->alloc(c->upart, int64_t(c->csplit) * nc))) return rc_;
      launch_trailing_inverse(c->cmat, 1, c->Tc, c->ctiles, c->cdinv, c->cxg, st);
      launch_coarse_inverse(c->cxg, c->dc, nc, c->cainv, st);
    }
  }

  // apply and PCG work space
  if ((rc_ = c->alloc(c->tickets, 8))) return rc_;
  if ((rc_ = c->alloc(c->part, (P.n_vec / NB + 1) * MAX_NCI))) return rc_;
  if ((rc_ = c->alloc(c->gbuf, int64_t(P.rc.size()) + 1))) return rc_;
  if ((rc_ = c->alloc(c->mu, int64_t(P.nsubs) * MAX_NCI))) return rc_;
  if ((rc_ = c->alloc(c->coef, int64_t(P.nsubs) * MAX_NCI))) return rc_;
  if ((rc_ = c->alloc(c->ww, P.n_loc))) return rc_;
  if ((rc_ = c->alloc(c->v12, P.n_free))) return rc_;
  launch_fill<double>(c->coef, 0.0, int64_t(P.nsubs) * MAX_NCI, st);
  if ((rc_ = c->alloc(c->r, P.n_free))) return rc_;
  if ((rc_ = c->alloc(c->z, P.n_free))) return rc_;
  if ((rc_ = c->alloc(c->p, P.n_free))) return rc_;
  if ((rc_ = c->alloc(c->q, P.n_free))) return rc_;
  if ((rc_ = c->alloc(c->tmp, P.n_free))) return rc_;
  if ((rc_ = c->alloc(c->part_a, VEC_GRID))) return rc_;
  if ((rc_ = c->alloc(c->part_b, VEC_GRID))) return rc_;
  if ((rc_ = c->alloc(c->part_c, VEC_GRID))) return rc_;
  if ((rc_ = c->alloc(c->sc, 1))) return rc_;
  if ((rc_ = c->alloc(c->xw, P.n_free))) return rc_;
  if ((rc_ = c->alloc(c->zpad, P.n_symrows * NB + 1))) return rc_;
  if ((rc_ = c->alloc(c->fpad, P.n_symrows * NB + 1))) return rc_;
  launch_fill<double>(c->zpad, 0.0, P.n_symrows * NB + 1, st);
  launch_fill<double>(c->fpad, 0.0, P.n_symrows * NB + 1, st);
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->hdone), sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
  HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->hdone_dev), c->hdone, 0));
  *c->hdone = 0;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->hback), (6 + 3 * size_t(MAX_PCG_IT)) * sizeof(double),
                        hipHostMallocMapped | hipHostMallocCoherent));
  HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->hback_dev), c->hback, 0));
  for (int i = 0; i < 2; ++i) HIP_TRY(hipEventCreateWithFlags(&c->snap_ev[i], hipEventDisableTiming));
  if ((rc_ = c->alloc(c->sploc, P.n_loc))) return rc_;
  for (auto& D : P.subs) c->max_loclen = std::max(c->max_loclen, int(D.T * NB + D.n_P));
  if ((rc_ = c->alloc(c->scal, 8))) return rc_;

  HIP_TRY(hipGetLastError());
  int herr[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(herr, c->err, sizeof(herr), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, f0, f1));
    c->factor_ms = ms;
    hipEventDestroy(f0);
    hipEventDestroy(f1);
  }
  if (herr[0] & 1) return fail(BDDC_ENOTSPD, "conductivity must be positive and finite");
  if (herr[0] & 4) return fail(BDDC_EINVAL, "internal: CSR row count mismatch");
  if ((herr[1] | herr[2]) & 8) return fail(BDDC_EHIP, "a factorisation task waited too long for a tile it reads");
  if (herr[1]) return fail(BDDC_ENOTSPD, "a local factorisation met a non-positive pivot (flags " +
                                            std::to_string(herr[1]) + ")");
  if (herr[2]) return fail(BDDC_ENOTSPD, "the coarse matrix is not positive definite (flags " +
                                            std::to_string(herr[2]) + ")");
  return BDDC_OK;
}

int check_ctx(bddc_ctx* c) {
  if (!c) return fail(BDDC_EINVAL, "ctx is NULL");
  return BDDC_OK;
}

}  // namespace

extern "C" {

int bddc_plan_stats(const bddc_mesh* mesh, const bddc_partition* part, uint32_t constraints, int64_t stats[8]) {
  if (!stats) return fail(BDDC_EINVAL, "stats is NULL");
  Plan P;
  std::string err;
  int rc_ = make_plan(mesh, part, constraints, P, err);
  if (rc_) return fail(rc_, err);
  int64_t sum_ni = 0;
  for (auto& D : P.subs) sum_ni += D.n_i;
  stats[0] = P.n_free;
  stats[1] = P.nsubs;
  stats[2] = P.n_coarse;
  stats[3] = P.n_corner_classes;
  stats[4] = P.n_edge_classes;
  stats[5] = P.n_face_classes;
  stats[6] = sum_ni;
  stats[7] = P.max_nci;
  return BDDC_OK;
}

int bddc_setup(const bddc_mesh* mesh, const bddc_partition* part, const bddc_coefficients* coef,
               uint32_t constraints, const bddc_options* opts, bddc_ctx** out) {
  const double t0 = now_ms();
  if (!out) return fail(BDDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!coef || !coef->theta) return fail(BDDC_EINVAL, "coefficients are NULL");
  if (!opts) return fail(BDDC_EINVAL, "options are NULL");
  if (opts->local_bits != 32 && opts->local_bits != 64) return fail(BDDC_EINVAL, "local_bits must be 32 or 64");
  if (opts->nb_override != 0 && opts->nb_override != NB) return fail(BDDC_ENOTIMPL, "only 64-wide tiles are built");
  if (opts->flags &
      ~(BDDC_SETUP_KEEP_ON_ERROR | BDDC_SETUP_FULL_SPACE | BDDC_SETUP_RHO_SCALING | BDDC_SETUP_COARSE_CG))
    return fail(BDDC_EINVAL, "unknown options.flags bits");
  bddc_ctx* c = new (std::nothrow) bddc_ctx();
  if (!c) return fail(BDDC_ENOMEM, "host allocation failed");
  std::string err;
  int rc_ = make_plan(mesh, part, constraints, c->plan, err);
  if (rc_) {
    delete c;
    return fail(rc_, err);
  }
  if (coef->on_device != 0 && coef->on_device != 1) {
    delete c;
    return fail(BDDC_EINVAL, "coefficients.on_device must be 0 or 1");
  }
  if (!coef->on_device) {
    for (int64_t e = 0; e < c->plan.n_el; ++e)
      if (!(coef->theta[e] > 0.0) || !std::isfinite(coef->theta[e])) {
        delete c;
        return fail(BDDC_ENOTSPD, "conductivity must be positive and finite (element " + std::to_string(e) + ")");
      }
  }
  c->st = static_cast<hipStream_t>(opts->stream);
  // the fixed workspace of bddc_apply_noalloc on the current device (looked up
  // once per device; a failed lookup only disables that entry point)
  if (static_scratch_address(&c->static_scratch) != 0) c->static_scratch = nullptr;
  c->use_graph = opts->use_graph != 0;
  c->rho_scaling = (opts->flags & BDDC_SETUP_RHO_SCALING) != 0;
  c->coarse_cg = (opts->flags & BDDC_SETUP_COARSE_CG) != 0;
  c->iface = !(opts->flags & BDDC_SETUP_FULL_SPACE);
  // the interface mat-vec packs a tile's row distance and its column into 8
  // bits each: at most IFACE_MAX_TS tile rows per subdomain; larger boxes
  // iterate on the whole space
  for (auto& D : c->plan.subs)
    if (sym_tile_rows(D) > IFACE_MAX_TS) c->iface = false;
  // FP32 local solves: on the whole space the local factors and triangular
  // solves are FP32 (the operator there is the FP64 global matrix).  The
  // interface operator and the interior solves come from the local factors and
  // must be exact, so the interface form keeps FP64 factors and applies the
  // preconditioner's local solves, its explicit matrices, in FP32.
  const bool local32 = opts->local_bits == 32;
  c->fp32 = local32 && !c->iface;
  c->pc32 = local32 && c->iface;
  c->mesh.dim = c->plan.dim;
  for (int a = 0; a < 3; ++a) {
    c->mesh.nel[a] = int(c->plan.nel[a]);
    c->mesh.h[a] = 1.0 / double(c->plan.nel[a]);
  }
  rc_ = do_setup(c, coef);
  if (rc_) {
    hipStreamSynchronize(c->st);
    if ((opts->flags & BDDC_SETUP_KEEP_ON_ERROR) && rc_ == BDDC_ENOTSPD) {
      *out = c;
      return rc_;
    }
    delete c;
    return rc_;
  }
  c->t_setup_ms = now_ms() - t0;
  *out = c;
  return BDDC_OK;
}

int bddc_apply(bddc_ctx* c, const double* r, double* z) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!r || !z || r == z) return fail(BDDC_EINVAL, "r and z must be distinct non-NULL device pointers");
  enqueue_apply(c, r, z, nullptr);
  HIP_TRY(hipGetLastError());
  return BDDC_OK;
}

int bddc_apply_noalloc(bddc_ctx* c, const double* r, double* z) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!r || !z || r == z) return fail(BDDC_EINVAL, "r and z must be distinct non-NULL device pointers");
  if (!c->static_scratch) return fail(BDDC_EHIP, "the fixed device workspace has no address on this device");
  const Plan& P = c->plan;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t es = c->fp32 ? sizeof(float) : sizeof(double);
  const size_t b_pub = up(size_t(4) * size_t(P.n_vec) * es);
  const size_t need = b_pub + up(8 * sizeof(unsigned));
  if (need > STATIC_SCRATCH_BYTES)
    return fail(BDDC_EINVAL, "this problem needs " + std::to_string(need) + " bytes of apply workspace; the fixed "
                             "workspace of bddc_apply_noalloc holds " + std::to_string(STATIC_SCRATCH_BYTES));
  char* base = static_cast<char*>(c->static_scratch);
  ApplyWs ws{base, reinterpret_cast<unsigned*>(base + b_pub)};
  enqueue_apply(c, r, z, nullptr, &ws);
  HIP_TRY(hipGetLastError());
  return BDDC_OK;
}

int bddc_spmv(bddc_ctx* c, const double* x, double* y) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!x || !y || x == y) return fail(BDDC_EINVAL, "x and y must be distinct non-NULL device pointers");
  hipEvent_t e = c->begin("spmv");
  launch_spmv(c->rowptr, c->col, c->val, x, y, c->plan.n_free, c->st);
  c->end("spmv", e);
  HIP_TRY(hipGetLastError());
  return BDDC_OK;
}

int bddc_elem_grad(bddc_ctx* c, const double* lam, const double* u, double* g) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!lam || !u || !g) return fail(BDDC_EINVAL, "NULL pointer");
  launch_elem_grad(c->mesh, lam, u, g, c->plan.n_el, c->st);
  HIP_TRY(hipGetLastError());
  return BDDC_OK;
}

int bddc_pcg_solve(bddc_ctx* c, const double* b, double* x, double rtol, int32_t maxit, int32_t flags,
                   bddc_pcg_info* info) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!b || !x || b == x) return fail(BDDC_EINVAL, "b and x must be distinct non-NULL device pointers");
  if (!(rtol > 0.0) || !(rtol < 1.0)) return fail(BDDC_EINVAL, "rtol must be in (0, 1)");
  if (maxit < 0 || maxit > MAX_PCG_IT) return fail(BDDC_EINVAL, "maxit must be in [0, 8192]");
  if (flags & ~BDDC_X0_GIVEN) return fail(BDDC_EINVAL, "unknown solve flags");
  const double t0 = now_ms();
  const Plan& P = c->plan;
  hipStream_t st = c->st;
  const int64_t n = P.n_free;
  int* done = &c->sc->done;
  const bool iface = c->iface;
  double* const x_user = x;
  if (c->use_graph) {
    // iterate in the ctx-owned buffer so that captured graphs stay valid
    if (flags & BDDC_X0_GIVEN) HIP_TRY(hipMemcpyAsync(c->xw, x_user, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    x = c->xw;
  }
  if (iface) {
    // interface unknowns: x holds the interface part (interior zero) during the
    // iteration; the residual lives on interface dofs (z, p and q are only
    // touched on interface dofs, and the first iteration of a segment does not
    // read p or q)
    if (flags & BDDC_X0_GIVEN) {
      launch_zero_interior(c->kappa, x, n, st);
      enqueue_interior_complete(c, b, x, c->tmp);
    } else {
      enqueue_interior_guess(c, b, c->tmp, x);
    }
    launch_residual(c->rowptr, c->col, c->val, c->tmp, b, c->r, c->part_a, c->part_b, n, st, c->kappa);
  } else {
    if (!(flags & BDDC_X0_GIVEN)) enqueue_interior_guess(c, b, x);
    launch_residual(c->rowptr, c->col, c->val, x, b, c->r, c->part_a, c->part_b, n, st);
  }
  launch_pcg_init(c->part_a, c->part_b, c->sc, rtol * rtol, st);

  struct HostScalars { double tol2, bb, rr0; int done, iters; } hs{};
  int devstat = 0;   // device status word (DEV_* bits) read back with the scalars
  std::vector<double> alphas, betas;
  int it = 0;            // iteration slot
  int restarts = 0;
  int status = BDDC_OK;
  double relres_true = 0.0, relres_rec = 0.0;
  bool fresh = true;
  int seg_start = 0;
  volatile int* const hdone = c->hdone;
  for (;;) {
    *hdone = 0;   // nothing of this ctx is in flight here
    // (re)start: z = M^{-1} r, rz
    if (iface) {
      launch_reset(false, nullptr, 0, nullptr, 0, c->tickets, done, st);
      launch_scatter_f_ifc(ifc_args(c), st);
      enqueue_apply_iface(c, c->r, c->z, c->part_c, done);
    } else {
      enqueue_apply(c, c->r, c->z, done);
      launch_dot(c->r, c->z, c->part_c, n, done, st);
    }
    // Iterations are queued at most two steps (one iteration eagerly, one graph
    // chunk with graphs) ahead of the last step the host has seen complete, and
    // no further once the iteration has set the host's end-of-solve word; the
    // kernels of a converged solve return at once.
    int pending = 0, slot_w = 0, slot_r = 0;
    for (;;) {
      while (pending < 2 && it < maxit && !*hdone) {
        // per-kernel timing needs eager launches (events are not captured into graphs)
        if (c->use_graph && !c->timing && fresh == (it == 0) && it % bddc_ctx::GRAPH_CHUNK == 0 &&
            it + bddc_ctx::GRAPH_CHUNK <= maxit && seg_start == 0) {
          if (int rc_ = launch_chunk_graph(c, x, it / bddc_ctx::GRAPH_CHUNK)) return rc_;
          it += bddc_ctx::GRAPH_CHUNK;
        } else {
          enqueue_iteration(c, x, it, fresh);
          ++it;
        }
        fresh = false;
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(c->snap_ev[slot_w], st));
        slot_w ^= 1;
        ++pending;
      }
      if (pending == 0 || *hdone) break;
      HIP_TRY(hipEventSynchronize(c->snap_ev[slot_r]));
      slot_r ^= 1;
      --pending;
    }
    // interior values of x (interface form) and the true residual, then every
    // scalar the host needs, in one readback
    if (iface) enqueue_interior_complete(c, b, x, x);
    launch_residual(c->rowptr, c->col, c->val, x, b, c->tmp, c->part_a, c->part_b, n, st);
    launch_finish_dot(c->part_a, c->scal, st);
    launch_pack_readback(c->sc, c->scal, c->err + 3, 0, it, c->hback_dev, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    const double* hb = c->hback;
    std::memcpy(&hs, hb, sizeof(hs));
    const int iters = hs.iters;
    std::memcpy(&devstat, hb + 5, sizeof(int));
    if (iters > seg_start && restarts == 0) {
      alphas.assign(hb + 6, hb + 6 + iters);
      betas.assign(hb + 6 + it, hb + 6 + it + iters - 1);
    }
    const double rr = iters > 0 ? hb[6 + 2 * it + iters - 1] : hs.rr0;
    if (devstat) break;
    relres_rec = hs.bb > 0 ? std::sqrt(rr / hs.bb) : 0.0;
    relres_true = hs.bb > 0 ? std::sqrt(hb[4] / hs.bb) : 0.0;
    if (hs.done == 2) { status = BDDC_EBREAKDOWN; break; }
    if (hs.done == 1 && relres_true <= rtol) { status = BDDC_OK; break; }
    if (it >= maxit) { status = BDDC_ENOCONV; break; }
    if (restarts >= 3) { status = BDDC_ENOCONV; break; }
    // residual replacement: r = b - A x, restart the directions
    ++restarts;
    launch_residual(c->rowptr, c->col, c->val, x, b, c->r, c->part_a, c->part_b, n, st,
                    iface ? c->kappa : nullptr);
    if (iface) launch_zero_interior(c->kappa, x, n, st);
    launch_pcg_init(c->part_a, c->part_b, c->sc, rtol * rtol, st);
    // keep the iteration count across the restart
    fresh = true;
    seg_start = it;
    launch_fill<int>(&c->sc->iters, it, 1, st);
  }
  if (x != x_user) HIP_TRY(hipMemcpyAsync(x_user, x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (c->timing) c->collect();
  if (info) {
    info->iters = hs.iters;
    info->relres_true = relres_true;
    info->relres_rec = relres_rec;
    info->cond_est = lanczos_cond(alphas, betas);
    info->t_setup_ms = c->t_setup_ms;
    info->t_solve_ms = now_ms() - t0;
  }
  if (devstat) {
    launch_fill<int>(c->err + 3, 0, 1, st);
    HIP_TRY(hipStreamSynchronize(st));
    return device_status_error(devstat);
  }
  if (status == BDDC_EBREAKDOWN) return fail(status, "CG breakdown: (p, A p) <= 0, (r, z) <= 0 or NaN");
  if (status == BDDC_ENOCONV) return fail(status, "maximum iterations reached");
  return BDDC_OK;
}

int bddc_query(bddc_ctx* c, int64_t* n_free, int32_t* n_sub, int32_t* n_coarse, int64_t* dev_bytes) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (n_free) *n_free = c->plan.n_free;
  if (n_sub) *n_sub = c->plan.nsubs;
  if (n_coarse) *n_coarse = c->plan.n_coarse;
  if (dev_bytes) *dev_bytes = c->dev_bytes;
  return BDDC_OK;
}

int bddc_setup_stats(bddc_ctx* c, double* factor_flops, double* factor_ms) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (factor_flops) *factor_flops = c->plan.factor_flops;
  if (factor_ms) *factor_ms = c->factor_ms;
  return BDDC_OK;
}

int bddc_set_timing(bddc_ctx* c, int32_t enabled) {
  if (int rc_ = check_ctx(c)) return rc_;
  c->collect();
  c->timing = enabled != 0;
  return BDDC_OK;
}

int bddc_kernel_time(bddc_ctx* c, const char* family, int64_t* launches, double* total_ms) {
  if (int rc_ = check_ctx(c)) return rc_;
  static const char* known[] = {"trsv_fwd_rr", "trsv_bwd_rr", "trsv_fwd_ii", "trsv_bwd_ii", "op", "pc",
                                "schur", "spmv", "apply"};
  bool ok = false;
  for (const char* k : known) ok |= family && std::strcmp(family, k) == 0;
  if (!ok) return fail(BDDC_EINVAL, "unknown kernel family");
  c->collect();
  auto it = c->fam.find(family);
  int64_t n = 0;
  double tot = 0.0;
  if (it != c->fam.end()) {
    // launches that returned at once because the solve had already converged
    // (queued ahead of the host's convergence check) are not counted
    float mx = 0.f;
    for (float d : it->second.durations) mx = std::max(mx, d);
    for (float d : it->second.durations)
      if (d >= 0.2f * mx) {
        ++n;
        tot += d;
      }
    it->second.durations.clear();
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = tot;
  return BDDC_OK;
}

int64_t bddc_debug_read(bddc_ctx* c, const char* what, int32_t sub, double* out, int64_t cap) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!what || !out || sub < 0 || sub >= c->plan.nsubs) return fail(BDDC_EINVAL, "bad debug_read arguments");
  HIP_TRY(hipStreamSynchronize(c->st));
  const MatDesc& D = c->plan.subs[sub];
  const std::string w(what);
  const int64_t es = c->fp32 ? 4 : 8;
  auto tile_to_double = [&](int64_t tile_index, std::vector<double>& buf) -> int {
    buf.resize(NB * NB);
    if (c->fp32) {
      std::vector<float> f(NB * NB);
      HIP_TRY(hipMemcpy(f.data(), static_cast<char*>(c->tiles) + tile_index * NB * NB * es, NB * NB * es,
                        hipMemcpyDeviceToHost));
      for (int i = 0; i < NB * NB; ++i) buf[i] = f[i];
    } else {
      HIP_TRY(hipMemcpy(buf.data(), static_cast<char*>(c->tiles) + tile_index * NB * NB * es, NB * NB * es,
                        hipMemcpyDeviceToHost));
    }
    return BDDC_OK;
  };
  std::vector<double> res;
  if (w == "sizes") {
    res = {double(D.n_R), double(D.n_I), double(D.n_A), double(D.n_P), double(D.T), double(D.n_i)};
  } else if (w == "factor") {
    const int64_t n = int64_t(D.T) * NB;
    res.assign(n * n, 0.0);
    std::vector<double> t;
    for (int i = 0; i < D.T; ++i)
      for (int j = 0; j <= i; ++j) {
        if (int rc_ = tile_to_double(env_tile(D, i, j), t)) return rc_;
        for (int r = 0; r < NB; ++r)
          for (int q = 0; q < NB; ++q) res[(i * NB + r) * n + j * NB + q] = t[r * NB + q];
      }
  } else if (w == "border" || w == "schur") {
    if (D.n_ci == 0) return 0;
    std::vector<double> t;
    if (w == "schur") {
      if (int rc_ = tile_to_double(env_tile(D, D.T, D.T), t)) return rc_;
      res = t;
    } else {
      const int64_t n = int64_t(D.T) * NB;
      res.assign(NB * n, 0.0);
      for (int j = 0; j < D.T; ++j) {
        if (int rc_ = tile_to_double(env_tile(D, D.T, j), t)) return rc_;
        for (int r = 0; r < NB; ++r)
          for (int q = 0; q < NB; ++q) res[r * n + j * NB + q] = t[r * NB + q];
      }
    }
  } else if (w == "aci") {
    res.resize(MAX_NCI * MAX_NCI);
    HIP_TRY(hipMemcpy(res.data(), c->aci + int64_t(sub) * MAX_NCI * MAX_NCI, res.size() * 8, hipMemcpyDeviceToHost));
  } else if (w == "gmap") {
    res.resize(D.n_i);
    for (int a = 0; a < D.n_i; ++a) res[a] = c->plan.gmap[D.loc_off + a];
  } else if (w == "envelope") {
    // per tile row k < T: first tile column of the factor's envelope (all rows),
    // then the same over the interior rows (rows k < TI only)
    const int64_t base = D.vec_off / NB;
    res.resize(2 * int64_t(D.T));
    for (int k = 0; k < D.T; ++k) {
      res[k] = c->plan.fcol[base + k];
      res[D.T + k] = c->plan.fcol_ii[base + k];
    }
  } else if (w == "dscale") {
    res.resize(D.n_i);
    HIP_TRY(hipMemcpy(res.data(), c->dsc + D.loc_off, res.size() * 8, hipMemcpyDeviceToHost));
  } else {
    return fail(BDDC_EINVAL, "unknown debug_read item");
  }
  const int64_t m = std::min<int64_t>(cap, int64_t(res.size()));
  std::memcpy(out, res.data(), size_t(m) * sizeof(double));
  return m;
}

namespace {
void drop_graphs(bddc_ctx* c) {
  hipStreamSynchronize(c->st);
  if (c->gst) hipStreamSynchronize(c->gst);
  for (auto& g : c->graphs)
    if (g) hipGraphExecDestroy(g);
  for (auto& g : c->graph_defs)
    if (g) hipGraphDestroy(g);
  for (auto& v : c->graph_timed)
    for (auto& gt : v) {
      hipEventDestroy(gt.b);
      hipEventDestroy(gt.e);
    }
  c->graphs.clear();
  c->graph_defs.clear();
  c->graph_timed.clear();
  c->graph_pending.clear();
}
}  // namespace

int bddc_set_limit(bddc_ctx* c, const char* what, int32_t value) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!what) return fail(BDDC_EINVAL, "limit name is NULL");
  const std::string w(what);
  if (w == "wait_polls") {
    drop_graphs(c);   // captured kernel arguments hold the old limit
    c->wait_polls = value;
  } else if (w == "coarse_cg_maxit") {
    if (value < 0) return fail(BDDC_EINVAL, "coarse_cg_maxit must be >= 0");
    drop_graphs(c);
    c->coarse_maxit = value;
  } else if (w == "sym_lds_cols") {
    if (value < 0 || value > SYM_LDS_COLS) return fail(BDDC_EINVAL, "sym_lds_cols must be in [0, 64]");
    drop_graphs(c);
    c->sym_lds_cols = value;
  } else if (w == "sym_row_pieces") {
    if (value < 0 || value > SYM_ROW_PIECES) return fail(BDDC_EINVAL, "sym_row_pieces must be in [0, 28]");
    drop_graphs(c);
    c->sym_row_pieces = value;
  } else {
    return fail(BDDC_EINVAL, "unknown limit (wait_polls, coarse_cg_maxit, sym_lds_cols, sym_row_pieces)");
  }
  return BDDC_OK;
}

int bddc_sync(bddc_ctx* c) {
  if (int rc_ = check_ctx(c)) return rc_;
  int w = 0;
  HIP_TRY(hipMemcpyAsync(&w, c->err + 3, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (w) {
    launch_fill<int>(c->err + 3, 0, 1, c->st);
    HIP_TRY(hipStreamSynchronize(c->st));
    return device_status_error(w);
  }
  return BDDC_OK;
}

int bddc_set_tuning(bddc_ctx* c, int32_t wg_per_cu) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (wg_per_cu < 1 || wg_per_cu > 16) return fail(BDDC_EINVAL, "wg_per_cu must be in [1, 16]");
  drop_graphs(c);
  c->wg_per_cu = wg_per_cu;
  c->grid_trsv = std::max(64, c->cus * wg_per_cu);
  return BDDC_OK;
}

int bddc_autotune(bddc_ctx* c, const int32_t* cand, int32_t ncand, int32_t iters, int32_t* best, double* ms_out) {
  if (int rc_ = check_ctx(c)) return rc_;
  if (!cand || ncand < 1 || iters < 1 || iters > 256) return fail(BDDC_EINVAL, "bad autotune arguments");
  for (int i = 0; i < ncand; ++i)
    if (cand[i] < 1 || cand[i] > 16) return fail(BDDC_EINVAL, "candidates must be in [1, 16]");
  const int64_t n = c->plan.n_free;
  if (!c->tune_b) {
    if (int rc_ = c->alloc(c->tune_b, n)) return rc_;
    if (int rc_ = c->alloc(c->tune_x, n)) return rc_;
    launch_fill<double>(c->tune_b, 1.0, n, c->st);
  }
  const bool timing = c->timing;
  c->timing = false;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best_ms = 1e300;
  int best_v = c->wg_per_cu;
  for (int i = 0; i < ncand; ++i) {
    if (int rc_ = bddc_set_tuning(c, cand[i])) return rc_;
    bddc_pcg_info info;
    double ms_i = 1e300;
    for (int rep = 0; rep < 2; ++rep) {   // the first run captures graphs and warms caches
      HIP_TRY(hipEventRecord(e0, c->st));
      int rc_ = bddc_pcg_solve(c, c->tune_b, c->tune_x, 1e-30, iters, 0, &info);
      if (rc_ != BDDC_OK && rc_ != BDDC_ENOCONV) return rc_;
      HIP_TRY(hipEventRecord(e1, c->st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1) ms_i = ms;
    }
    if (ms_out) ms_out[i] = ms_i;
    if (ms_i < best_ms) {
      best_ms = ms_i;
      best_v = cand[i];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->timing = timing;
  if (best) *best = best_v;
  return bddc_set_tuning(c, best_v);
}

void bddc_destroy(bddc_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->st);
  delete c;
}

const char* bddc_strerror(int code) {
  switch (code) {
    case BDDC_OK: return "success";
    case BDDC_EINVAL: return "invalid argument";
    case BDDC_ENOTSPD: return "matrix not symmetric positive definite";
    case BDDC_ENOMEM: return "out of memory";
    case BDDC_EHIP: return "HIP runtime error";
    case BDDC_ENOCONV: return "no convergence within maxit";
    case BDDC_EBREAKDOWN: return "CG breakdown";
    case BDDC_ENOTIMPL: return "not implemented";
    default: return "unknown status";
  }
}

const char* bddc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
