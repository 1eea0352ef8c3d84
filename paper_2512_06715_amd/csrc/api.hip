// Host side of the C ABI: argument checks, workspace carving, setup
// orchestration, the block-by-block solve driver with HIP graphs.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "internal.h"
#include "pdhg.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base((char *)b) {}
  template <typename T>
  T *take(int64_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += sizeof(T) * (size_t)(count > 0 ? count : 1);
    return p;
  }
};

unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + PDHG_BLOCK - 1) / PDHG_BLOCK); }

}  // namespace

struct pdhg_handle {
  int64_t m = 0, n = 0, nnz = 0;
  pdhg_opts o{};
  int on_device = 0;
  hipStream_t hs = nullptr;
  hipStream_t user = nullptr;
  hipEvent_t ev = nullptr;
  bool hip_failed = false;
  double setup_s = 0.0;

  int32_t *rp, *ci, *cp, *ri, *long_rows, *long_cols, *scan_tmp, *tmp_next;
  double *v, *vt, *b0, *c0, *l0, *u0, *b, *c, *l, *u, *Dr, *Dc;
  uint8_t *kind, *vk;
  double *X[2], *Y[2], *AX[2], *XS, *YS, *XL, *YL, *XA, *YA, *AXA, *ATY, *ATYA;
  float *vf = nullptr, *vtf = nullptr, *bf = nullptr, *cf = nullptr, *lf = nullptr,
        *uf = nullptr;
  float *Xf[2] = {nullptr, nullptr}, *Yf[2] = {nullptr, nullptr}, *AXf[2] = {nullptr, nullptr};
  float *XSf = nullptr, *YSf = nullptr;
  double *part_dx2, *part_dy, *part_rows, *part_cols, *scratch;
  int nscratch = 0;
  CtlState *st;
  int *err;
  int n_long_rows = 0, n_long_cols = 0, nblk_rows = 0, nblk_cols = 0;
  int tpb_rows = 1, tpb_cols = 1, grid_rows = 1, grid_cols = 1;
  CtlState *host_st = nullptr;

  struct Graph {
    hipGraphExec_t exec = nullptr;
    int period = 0;
    double tol = 0;
    int64_t max_iter = 0;
  } graph[2];
};

namespace {

size_t layout(pdhg_handle *h, void *base) {
  Carver cv(base);
  int64_t m = h->m, n = h->n, nnz = h->nnz;
  h->rp = cv.take<int32_t>(m + 1);
  h->ci = cv.take<int32_t>(nnz);
  h->cp = cv.take<int32_t>(n + 1);
  h->ri = cv.take<int32_t>(nnz);
  h->long_rows = cv.take<int32_t>(m);
  h->long_cols = cv.take<int32_t>(n);
  h->scan_tmp = cv.take<int32_t>(scan_tmp_ints(n + 1));
  h->tmp_next = cv.take<int32_t>(n + 1);
  h->v = cv.take<double>(nnz);
  h->vt = cv.take<double>(nnz);
  h->b0 = cv.take<double>(m);
  h->b = cv.take<double>(m);
  h->Dr = cv.take<double>(m);
  h->c0 = cv.take<double>(n);
  h->l0 = cv.take<double>(n);
  h->u0 = cv.take<double>(n);
  h->c = cv.take<double>(n);
  h->l = cv.take<double>(n);
  h->u = cv.take<double>(n);
  h->Dc = cv.take<double>(n);
  h->kind = cv.take<uint8_t>(m);
  h->vk = cv.take<uint8_t>(n);
  for (int q = 0; q < 2; q++) {
    h->X[q] = cv.take<double>(n);
    h->Y[q] = cv.take<double>(m);
    h->AX[q] = cv.take<double>(m);
  }
  h->XS = cv.take<double>(n);
  h->YS = cv.take<double>(m);
  h->XL = cv.take<double>(n);
  h->YL = cv.take<double>(m);
  h->XA = cv.take<double>(n);
  h->YA = cv.take<double>(m);
  h->AXA = cv.take<double>(m);
  h->ATY = cv.take<double>(n);
  h->ATYA = cv.take<double>(n);
  int64_t nbr = nblk(m), nbc = nblk(n);
  h->part_dx2 = cv.take<double>(nbc + n);
  h->part_dy = cv.take<double>(2 * (nbr + m));
  h->part_rows = cv.take<double>(nbr * EV_ROWQ);
  h->part_cols = cv.take<double>(nbc * EV_COLQ);
  h->nscratch = 5 * 1024;
  h->scratch = cv.take<double>(h->nscratch);
  h->st = cv.take<CtlState>(1);
  h->err = cv.take<int>(1);
  if (h->o.precision == PDHG_MIXED) {
    h->vf = cv.take<float>(nnz);
    h->vtf = cv.take<float>(nnz);
    h->bf = cv.take<float>(m);
    h->cf = cv.take<float>(n);
    h->lf = cv.take<float>(n);
    h->uf = cv.take<float>(n);
    for (int q = 0; q < 2; q++) {
      h->Xf[q] = cv.take<float>(n);
      h->Yf[q] = cv.take<float>(m);
      h->AXf[q] = cv.take<float>(m);
    }
    h->XSf = cv.take<float>(n);
    h->YSf = cv.take<float>(m);
  }
  return cv.off + 256;
}

int check_opts(const pdhg_opts *o) {
  if (!(o->tol > 0.0)) return fail(PDHG_ERR_ARG, "tol must be > 0");
  if (o->max_iter < 0) return fail(PDHG_ERR_ARG, "max_iter must be >= 0");
  if (o->precision != PDHG_FP64 && o->precision != PDHG_MIXED)
    return fail(PDHG_ERR_ARG, "precision must be PDHG_FP64 or PDHG_MIXED");
  if (o->eval_period < 1) return fail(PDHG_ERR_ARG, "eval_period must be >= 1");
  if (o->step_mode != 0 && o->step_mode != 1) return fail(PDHG_ERR_ARG, "step_mode must be 0 or 1");
  if (o->scaling_iters < 0) return fail(PDHG_ERR_ARG, "scaling_iters must be >= 0");
  if (o->unroll_iters < 0) return fail(PDHG_ERR_ARG, "unroll_iters must be >= 0");
  if (!(o->pw_theta >= 0.0 && o->pw_theta <= 1.0)) return fail(PDHG_ERR_ARG, "pw_theta must be in [0, 1]");
  if (o->tiles_per_block < 0) return fail(PDHG_ERR_ARG, "tiles_per_block must be >= 0");
  return PDHG_OK;
}

int check_lp_shape(const pdhg_lp *lp) {
  if (!lp) return fail(PDHG_ERR_ARG, "lp is null");
  if (lp->m <= 0 || lp->n <= 0) return fail(PDHG_ERR_ARG, "m and n must be positive");
  if (lp->nnz < 0 || lp->nnz > 0x7fffffffLL || lp->m >= 0x7fffffffLL || lp->n >= 0x7fffffffLL)
    return fail(PDHG_ERR_ARG, "sizes must fit in int32");
  if (!lp->row_ptr || !lp->row_kind || !lp->b || !lp->c || !lp->l || !lp->u ||
      (lp->nnz > 0 && (!lp->col_idx || !lp->val)))
    return fail(PDHG_ERR_ARG, "null array in lp");
  return PDHG_OK;
}

// Full validation of host-resident input, before any device call.
int validate_host(const pdhg_lp *lp) {
  int64_t m = lp->m, n = lp->n, nnz = lp->nnz;
  const int32_t *rp = lp->row_ptr, *ci = lp->col_idx;
  if (rp[0] != 0) return fail(PDHG_ERR_CSR, "row_ptr[0] = %d, expected 0", rp[0]);
  for (int64_t i = 0; i < m; i++) {
    if (rp[i + 1] < rp[i]) return fail(PDHG_ERR_CSR, "row_ptr decreases at row %lld", (long long)i);
    if (rp[i + 1] > nnz) return fail(PDHG_ERR_CSR, "row_ptr[%lld] exceeds nnz", (long long)(i + 1));
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
      if (ci[k] < 0 || ci[k] >= n)
        return fail(PDHG_ERR_CSR, "column %d out of range in row %lld", ci[k], (long long)i);
      if (k > rp[i] && ci[k] <= ci[k - 1])
        return fail(PDHG_ERR_CSR, "columns of row %lld not strictly ascending", (long long)i);
    }
  }
  if (rp[m] != nnz) return fail(PDHG_ERR_CSR, "row_ptr[m] = %d, expected nnz = %lld", rp[m], (long long)nnz);
  for (int64_t i = 0; i < m; i++)
    if (lp->row_kind[i] > 1) return fail(PDHG_ERR_ARG, "row_kind[%lld] = %d", (long long)i, lp->row_kind[i]);
  for (int64_t j = 0; j < n; j++) {
    double lj = lp->l[j], uj = lp->u[j];
    if (isnan(lj) || isnan(uj) || lj > uj || lj == INFINITY || uj == -INFINITY)
      return fail(PDHG_ERR_BOUNDS, "invalid bounds at column %lld", (long long)j);
  }
  for (int64_t k = 0; k < nnz; k++)
    if (!isfinite(lp->val[k])) return fail(PDHG_ERR_NONFINITE, "non-finite A entry %lld", (long long)k);
  for (int64_t i = 0; i < m; i++)
    if (!isfinite(lp->b[i])) return fail(PDHG_ERR_NONFINITE, "non-finite b[%lld]", (long long)i);
  for (int64_t j = 0; j < n; j++)
    if (!isfinite(lp->c[j])) return fail(PDHG_ERR_NONFINITE, "non-finite c[%lld]", (long long)j);
  return PDHG_OK;
}

#define HC(call)                                                                          \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      h->hip_failed = true;                                                               \
      return fail(PDHG_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));           \
    }                                                                                     \
  } while (0)

#define HK()                                                                              \
  do {                                                                                    \
    hipError_t e_ = hipGetLastError();                                                    \
    if (e_ != hipSuccess) {                                                               \
      h->hip_failed = true;                                                               \
      return fail(PDHG_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_));       \
    }                                                                                     \
  } while (0)

hipMemcpyKind in_kind(const pdhg_handle *h) {
  return h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}

template <typename T>
IterView<T> iter_view(pdhg_handle *h);

template <>
IterView<double> iter_view<double>(pdhg_handle *h) {
  IterView<double> w{};
  w.m = h->m;
  w.n = h->n;
  w.rp = h->rp;
  w.ci = h->ci;
  w.cp = h->cp;
  w.ri = h->ri;
  w.v = h->v;
  w.vt = h->vt;
  w.b = h->b;
  w.c = h->c;
  w.l = h->l;
  w.u = h->u;
  w.kind = h->kind;
  w.vk = h->vk;
  for (int q = 0; q < 2; q++) {
    w.X[q] = h->X[q];
    w.Y[q] = h->Y[q];
    w.AX[q] = h->AX[q];
  }
  w.XS = h->XS;
  w.YS = h->YS;
  w.nblk_rows = h->nblk_rows;
  w.nblk_cols = h->nblk_cols;
  w.long_rows = h->long_rows;
  w.long_cols = h->long_cols;
  w.n_long_rows = h->n_long_rows;
  w.n_long_cols = h->n_long_cols;
  w.tpb_rows = h->tpb_rows;
  w.tpb_cols = h->tpb_cols;
  w.grid_rows = h->grid_rows;
  w.grid_cols = h->grid_cols;
  w.part_dx2 = h->part_dx2;
  w.part_dy = h->part_dy;
  w.adaptive = h->o.step_mode == 0;
  return w;
}

template <>
IterView<float> iter_view<float>(pdhg_handle *h) {
  IterView<float> w{};
  w.m = h->m;
  w.n = h->n;
  w.rp = h->rp;
  w.ci = h->ci;
  w.cp = h->cp;
  w.ri = h->ri;
  w.v = h->vf;
  w.vt = h->vtf;
  w.b = h->bf;
  w.c = h->cf;
  w.l = h->lf;
  w.u = h->uf;
  w.kind = h->kind;
  w.vk = h->vk;
  for (int q = 0; q < 2; q++) {
    w.X[q] = h->Xf[q];
    w.Y[q] = h->Yf[q];
    w.AX[q] = h->AXf[q];
  }
  w.XS = h->XSf;
  w.YS = h->YSf;
  w.nblk_rows = h->nblk_rows;
  w.nblk_cols = h->nblk_cols;
  w.long_rows = h->long_rows;
  w.long_cols = h->long_cols;
  w.n_long_rows = h->n_long_rows;
  w.n_long_cols = h->n_long_cols;
  w.tpb_rows = h->tpb_rows;
  w.tpb_cols = h->tpb_cols;
  w.grid_rows = h->grid_rows;
  w.grid_cols = h->grid_cols;
  w.part_dx2 = h->part_dx2;
  w.part_dy = h->part_dy;
  w.adaptive = h->o.step_mode == 0;
  return w;
}

template <typename T>
EvalView<T> eval_view(pdhg_handle *h) {
  EvalView<T> e{};
  IterView<T> w = iter_view<T>(h);
  e.m = h->m;
  e.n = h->n;
  e.rp = h->rp;
  e.ci = h->ci;
  e.cp = h->cp;
  e.ri = h->ri;
  e.v = h->v;
  e.vt = h->vt;
  e.b = h->b;
  e.c = h->c;
  e.l = h->l;
  e.u = h->u;
  e.Dr = h->Dr;
  e.Dc = h->Dc;
  e.kind = h->kind;
  e.vk = h->vk;
  for (int q = 0; q < 2; q++) {
    e.X[q] = w.X[q];
    e.Y[q] = w.Y[q];
    e.AX[q] = w.AX[q];
  }
  e.XS = w.XS;
  e.YS = w.YS;
  e.XA = h->XA;
  e.YA = h->YA;
  e.AXA = h->AXA;
  e.ATY = h->ATY;
  e.ATYA = h->ATYA;
  e.XL = h->XL;
  e.YL = h->YL;
  e.nblk_rows = h->nblk_rows;
  e.nblk_cols = h->nblk_cols;
  e.part_rows = h->part_rows;
  e.part_cols = h->part_cols;
  e.use_average = h->o.use_average;
  e.restart = h->o.restart;
  e.pw_theta = h->o.pw_update ? h->o.pw_theta : 0.0;
  return e;
}

int read_state(pdhg_handle *h) {
  HC(hipMemcpyAsync(h->host_st, h->st, sizeof(CtlState), hipMemcpyDeviceToHost, h->hs));
  HC(hipStreamSynchronize(h->hs));
  return PDHG_OK;
}

// Record one block (period attempts + evaluation) as a graph.
template <typename T>
int capture_block(pdhg_handle *h, int slot, int period, double tol, int64_t max_iter) {
  auto &g = h->graph[slot];
  if (g.exec && g.period == period && g.tol == tol && g.max_iter == max_iter) return PDHG_OK;
  if (g.exec) {
    HC(hipGraphExecDestroy(g.exec));
    g.exec = nullptr;
  }
  IterView<T> w = iter_view<T>(h);
  EvalView<T> e = eval_view<T>(h);
  hipGraph_t graph;
  HC(hipStreamBeginCapture(h->hs, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < period; i++) launch_attempt<T>(w, h->st, max_iter, h->hs);
  launch_evaluate_ll<T>(e, h->long_rows, h->n_long_rows, h->long_cols, h->n_long_cols, h->st, tol,
                        max_iter, h->hs);
  HC(hipStreamEndCapture(h->hs, &graph));
  HK();
  HC(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
  HC(hipGraphDestroy(graph));
  g.period = period;
  g.tol = tol;
  g.max_iter = max_iter;
  return PDHG_OK;
}

// Run attempts in blocks until the device reports done; the start point must
// already be initialised (launch_init_point) or carried over.
// stall_evals > 0: return with *status_out = 0 when the reported relative KKT
// error has not dropped below 0.9 of its best value for that many evaluations.
template <typename T>
int run_blocks(pdhg_handle *h, double tol, int64_t max_iter, double t_start, int *status_out,
               int stall_evals = 0) {
  IterView<T> w = iter_view<T>(h);
  EvalView<T> e = eval_view<T>(h);
  const int slot = sizeof(T) == 4 ? 1 : 0;
  const int P = h->o.eval_period;
  launch_evaluate_ll<T>(e, h->long_rows, h->n_long_rows, h->long_cols, h->n_long_cols, h->st, tol,
                        max_iter, h->hs);
  HK();
  int rc = read_state(h);
  if (rc) return rc;
  double best = h->host_st->rel_kkt;
  int since = 0;
  while (!h->host_st->done) {
    int64_t k = h->host_st->k;
    int64_t nb = std::min<int64_t>(P, max_iter - k);
    if (nb == P && h->o.use_graph) {
      rc = capture_block<T>(h, slot, P, tol, max_iter);
      if (rc) return rc;
      HC(hipGraphLaunch(h->graph[slot].exec, h->hs));
    } else {
      for (int64_t i = 0; i < nb; i++) launch_attempt<T>(w, h->st, max_iter, h->hs);
      launch_evaluate_ll<T>(e, h->long_rows, h->n_long_rows, h->long_cols, h->n_long_cols, h->st,
                            tol, max_iter, h->hs);
      HK();
    }
    rc = read_state(h);
    if (rc) return rc;
    const CtlState *s = h->host_st;
    if (h->o.verbose)
      fprintf(stderr,
              "pdhg k=%lld kkt=%.3e (p %.2e d %.2e g %.2e) obj=%.10g eta=%.3e omega=%.3e "
              "restarts=%lld\n",
              s->k, s->rel_kkt, s->rel_p, s->rel_d, s->rel_gap, s->pobj, s->eta, s->omega,
              s->restarts);
    if (!s->done && now_s() - t_start > h->o.time_limit_s) {
      *status_out = PDHG_TIME_LIMIT;
      return PDHG_OK;
    }
    if (s->rel_kkt < 0.9 * best) {
      best = s->rel_kkt;
      since = 0;
    } else if (stall_evals > 0 && ++since >= stall_evals && !s->done) {
      *status_out = 0;
      return PDHG_OK;
    }
  }
  *status_out = h->host_st->status;
  return PDHG_OK;
}

int enter(pdhg_handle *h) {
  if (h->hip_failed) return fail(PDHG_ERR_HIP, "handle unusable after an earlier HIP error");
  HC(hipEventRecord(h->ev, h->user));
  HC(hipStreamWaitEvent(h->hs, h->ev, 0));
  return PDHG_OK;
}

int leave(pdhg_handle *h) {
  HC(hipEventRecord(h->ev, h->hs));
  HC(hipStreamWaitEvent(h->user, h->ev, 0));
  return PDHG_OK;
}

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

void pdhg_default_opts(pdhg_opts *o) {
  memset(o, 0, sizeof *o);
  o->tol = 1e-4;
  o->max_iter = 10000000;
  o->time_limit_s = 1e30;
  o->precision = PDHG_FP64;
  o->eval_period = 64;
  o->step_mode = 0;
  o->fixed_eta = 0.0;
  o->fixed_omega = 0.0;
  o->scaling_iters = 10;
  o->pock_chambolle = 1;
  o->restart = 1;
  o->use_average = 1;
  o->unroll_iters = 0;
  o->checkpoint_every = 50;
  o->use_graph = 1;
  o->verbose = 0;
  o->polish_tol = 0.0;
  o->pw_update = 1;
  o->pw_theta = 0.5;
}

const char *pdhg_last_error(void) { return g_err.c_str(); }

int pdhg_workspace_bytes(const pdhg_lp *lp, const pdhg_opts *opts, size_t *bytes) {
  int rc = check_lp_shape(lp);
  if (rc) return rc;
  if (!opts || !bytes) return fail(PDHG_ERR_ARG, "null argument");
  rc = check_opts(opts);
  if (rc) return rc;
  pdhg_handle tmp;
  tmp.m = lp->m;
  tmp.n = lp->n;
  tmp.nnz = lp->nnz;
  tmp.o = *opts;
  *bytes = layout(&tmp, nullptr);
  return PDHG_OK;
}

int pdhg_setup(const pdhg_lp *lp, const pdhg_opts *opts, void *workspace, size_t ws_bytes,
               void *stream, pdhg_handle **out) {
  if (!out) return fail(PDHG_ERR_ARG, "handle pointer is null");
  *out = nullptr;
  int rc = check_lp_shape(lp);
  if (rc) return rc;
  if (!opts) return fail(PDHG_ERR_ARG, "opts is null");
  rc = check_opts(opts);
  if (rc) return rc;
  if (!lp->on_device) {
    rc = validate_host(lp);
    if (rc) return rc;
  }
  size_t need = 0;
  pdhg_workspace_bytes(lp, opts, &need);
  if (!workspace || ws_bytes < need)
    return fail(PDHG_ERR_OOM, "workspace of %zu bytes, need %zu", ws_bytes, need);

  double t0 = now_s();
  pdhg_handle *h = new pdhg_handle();
  h->m = lp->m;
  h->n = lp->n;
  h->nnz = lp->nnz;
  h->o = *opts;
  h->on_device = lp->on_device;
  h->user = (hipStream_t)stream;
  layout(h, (void *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255));
  h->nblk_rows = (int)nblk(h->m);
  h->nblk_cols = (int)nblk(h->n);
  auto cleanup = [&](int code) {
    pdhg_destroy(h);
    return code;
  };
#define SC(call)                                                                            \
  do {                                                                                      \
    int r_ = (call);                                                                        \
    if (r_) return cleanup(r_);                                                             \
  } while (0)
  auto setup_body = [&]() -> int {
    HC(hipStreamCreateWithFlags(&h->hs, hipStreamNonBlocking));
    HC(hipEventCreateWithFlags(&h->ev, hipEventDisableTiming));
    HC(hipHostMalloc((void **)&h->host_st, sizeof(CtlState), hipHostMallocDefault));
    int r = enter(h);
    if (r) return r;
    int64_t m = h->m, n = h->n, nnz = h->nnz;
    hipMemcpyKind kd = in_kind(h);
    HC(hipMemcpyAsync(h->rp, lp->row_ptr, sizeof(int32_t) * (m + 1), kd, h->hs));
    if (nnz) {
      HC(hipMemcpyAsync(h->ci, lp->col_idx, sizeof(int32_t) * nnz, kd, h->hs));
      HC(hipMemcpyAsync(h->v, lp->val, sizeof(double) * nnz, kd, h->hs));
    }
    HC(hipMemcpyAsync(h->kind, lp->row_kind, m, kd, h->hs));
    HC(hipMemcpyAsync(h->b0, lp->b, sizeof(double) * m, kd, h->hs));
    HC(hipMemcpyAsync(h->c0, lp->c, sizeof(double) * n, kd, h->hs));
    HC(hipMemcpyAsync(h->l0, lp->l, sizeof(double) * n, kd, h->hs));
    HC(hipMemcpyAsync(h->u0, lp->u, sizeof(double) * n, kd, h->hs));
    if (h->on_device) {
      HC(hipMemsetAsync(h->err, 0, sizeof(int), h->hs));
      launch_validate(h->rp, h->ci, h->v, h->kind, h->b0, h->c0, h->l0, h->u0, m, n, nnz, h->err,
                      h->hs);
      HK();
      int herr = 0;
      HC(hipMemcpyAsync(&herr, h->err, sizeof(int), hipMemcpyDeviceToHost, h->hs));
      HC(hipStreamSynchronize(h->hs));
      if (herr & VERR_CSR) return fail(PDHG_ERR_CSR, "matrix is not canonical CSR");
      if (herr & VERR_KIND) return fail(PDHG_ERR_ARG, "row_kind entry not 0 or 1");
      if (herr & VERR_BOUNDS) return fail(PDHG_ERR_BOUNDS, "invalid variable bounds");
      if (herr & VERR_NONFINITE) return fail(PDHG_ERR_NONFINITE, "non-finite entry in A, b or c");
    }
    launch_var_kind(h->l0, h->u0, n, h->vk, h->hs);
    launch_transpose(h->rp, h->ci, h->v, m, n, nnz, h->cp, h->ri, h->vt, h->tmp_next, h->scan_tmp,
                     h->hs);
    HK();
    // scaling: rs in YA (m), cs in XA (n)
    launch_fill(h->Dr, 1.0, m, h->hs);
    launch_fill(h->Dc, 1.0, n, h->hs);
    int passes = h->o.scaling_iters + (h->o.pock_chambolle ? 1 : 0);
    for (int it = 0; it < passes; it++)
      launch_scale_pass(h->rp, h->ci, h->v, h->cp, h->ri, h->vt, m, n,
                        it == h->o.scaling_iters ? 1 : 0, h->YA, h->XA, h->Dr, h->Dc, h->hs);
    launch_scale_vectors(h->b0, h->c0, h->l0, h->u0, h->Dr, h->Dc, m, n, h->b, h->c, h->l, h->u,
                         h->hs);
    HK();
    // long rows and columns (handled by a workgroup each in the iteration)
    std::vector<int32_t> hp(std::max(m, n) + 1);
    std::vector<int32_t> lr, lc;
    HC(hipMemcpyAsync(hp.data(), h->rp, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost, h->hs));
    HC(hipStreamSynchronize(h->hs));
    for (int64_t i = 0; i < m; i++)
      if (hp[i + 1] - hp[i] > PDHG_LONG_SEG) lr.push_back((int32_t)i);
    HC(hipMemcpyAsync(hp.data(), h->cp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, h->hs));
    HC(hipStreamSynchronize(h->hs));
    for (int64_t j = 0; j < n; j++)
      if (hp[j + 1] - hp[j] > PDHG_LONG_SEG) lc.push_back((int32_t)j);
    h->n_long_rows = (int)lr.size();
    h->n_long_cols = (int)lc.size();
    h->tpb_rows = h->o.tiles_per_block > 0
                      ? h->o.tiles_per_block
                      : std::max(1, (h->nblk_rows + PDHG_TARGET_GROUPS - 1) / PDHG_TARGET_GROUPS);
    h->tpb_cols = h->o.tiles_per_block > 0
                      ? h->o.tiles_per_block
                      : std::max(1, (h->nblk_cols + PDHG_TARGET_GROUPS - 1) / PDHG_TARGET_GROUPS);
    h->grid_rows = h->n_long_rows + (h->nblk_rows + h->tpb_rows - 1) / h->tpb_rows;
    h->grid_cols = h->n_long_cols + (h->nblk_cols + h->tpb_cols - 1) / h->tpb_cols;
    if (!lr.empty())
      HC(hipMemcpyAsync(h->long_rows, lr.data(), sizeof(int32_t) * lr.size(), hipMemcpyHostToDevice,
                        h->hs));
    if (!lc.empty())
      HC(hipMemcpyAsync(h->long_cols, lc.data(), sizeof(int32_t) * lc.size(), hipMemcpyHostToDevice,
                        h->hs));
    launch_init_ctl(h->v, nnz, h->b, h->c, h->b0, h->c0, m, n, h->scratch, h->nscratch, h->st,
                    h->o.step_mode, h->o.step_mode == 1 ? h->o.fixed_eta : 0.0, h->o.fixed_omega,
                    h->hs);
    if (h->o.precision == PDHG_MIXED) {
      launch_cast_f32(h->v, h->vf, nnz, h->hs);
      launch_cast_f32(h->vt, h->vtf, nnz, h->hs);
      launch_cast_f32(h->b, h->bf, m, h->hs);
      launch_cast_f32(h->c, h->cf, n, h->hs);
      launch_cast_f32(h->l, h->lf, n, h->hs);
      launch_cast_f32(h->u, h->uf, n, h->hs);
    }
    HK();
    HC(hipStreamSynchronize(h->hs));
    r = leave(h);
    if (r) return r;
    return PDHG_OK;
  };
  SC(setup_body());
#undef SC
  h->setup_s = now_s() - t0;
  *out = h;
  return PDHG_OK;
}

int pdhg_solve(pdhg_handle *h, const double *x0, const double *y0, double *x, double *y,
               pdhg_info *info) {
  if (!h || !x || !y || !info) return fail(PDHG_ERR_ARG, "null argument");
  int rc = enter(h);
  if (rc) return rc;
  double t0 = now_s();
  memset(info, 0, sizeof *info);
  // stage host start vectors in the average buffers (free before the first evaluation)
  const double *dx0 = x0, *dy0 = y0;
  if (!h->on_device) {
    if (x0) {
      HC(hipMemcpyAsync(h->XA, x0, sizeof(double) * h->n, hipMemcpyHostToDevice, h->hs));
      dx0 = h->XA;
    }
    if (y0) {
      HC(hipMemcpyAsync(h->YA, y0, sizeof(double) * h->m, hipMemcpyHostToDevice, h->hs));
      dy0 = h->YA;
    }
  }
  int status = 0;
  bool final_fp32 = false;
  int64_t attempts_fp32 = 0;
  EvalView<double> e = eval_view<double>(h);
  if (h->o.precision == PDHG_FP64) {
    launch_init_point<double>(e, h->long_rows, h->n_long_rows, dx0, dy0, h->st, h->AXA, h->hs);
    HK();
    rc = run_blocks<double>(h, h->o.tol, h->o.max_iter, t0, &status);
    if (rc) return rc;
  } else {
    // FP32 phase: FP32 matrix, iterates and SpMVs; FP64 evaluation and control
    EvalView<float> ef = eval_view<float>(h);
    double tol32 = h->o.polish_tol > h->o.tol ? h->o.polish_tol : h->o.tol;
    launch_init_point<float>(ef, h->long_rows, h->n_long_rows, dx0, dy0, h->st, h->AXA, h->hs);
    HK();
    rc = run_blocks<float>(h, tol32, h->o.max_iter, t0, &status, 300);
    if (rc) return rc;
    attempts_fp32 = h->host_st->k;
    final_fp32 = true;
    bool polish = (status == 0) || (status == PDHG_OPTIMAL && tol32 > h->o.tol);
    if (polish) {
      // FP64 refinement from the FP32 iterate
      launch_switch_to_fp64(ef, e, h->long_rows, h->n_long_rows, h->st, h->hs);
      HK();
      rc = run_blocks<double>(h, h->o.tol, h->o.max_iter, t0, &status);
      if (rc) return rc;
      final_fp32 = false;
    }
  }
  // unscale into the caller's arrays
  if (h->on_device) {
    if (final_fp32)
      launch_unscale<float>(eval_view<float>(h), h->st, x, y, h->hs);
    else
      launch_unscale<double>(e, h->st, x, y, h->hs);
    HK();
  } else {
    if (final_fp32)
      launch_unscale<float>(eval_view<float>(h), h->st, h->ATYA, h->AXA, h->hs);
    else
      launch_unscale<double>(e, h->st, h->ATYA, h->AXA, h->hs);
    HK();
    HC(hipMemcpyAsync(x, h->ATYA, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(y, h->AXA, sizeof(double) * h->m, hipMemcpyDeviceToHost, h->hs));
  }
  rc = read_state(h);
  if (rc) return rc;
  const CtlState *s = h->host_st;
  info->status = status;
  info->which = s->which;
  info->attempts = s->k;
  info->attempts_fp32 = attempts_fp32;
  info->accepted = s->accepted;
  info->restarts = s->restarts;
  info->primal_obj = s->pobj;
  info->dual_obj = s->dobj;
  info->rel_primal = s->rel_p;
  info->rel_dual = s->rel_d;
  info->rel_gap = s->rel_gap;
  info->rel_kkt = s->rel_kkt;
  info->eta = s->eta;
  info->omega = s->omega;
  info->setup_s = h->setup_s;
  info->solve_s = now_s() - t0;
  return leave(h);
}

int pdhg_solve_batch(pdhg_handle *const *, int, const pdhg_instance *, int, double *const *,
                     double *const *, pdhg_info *) {
  return fail(PDHG_ERR_STATE, "batched solve not available in this build");
}

int pdhg_backward(pdhg_handle *, double, double *, double *) {
  return fail(PDHG_ERR_STATE, "backward not available in this build");
}

void pdhg_destroy(pdhg_handle *h) {
  if (!h) return;
  for (auto &g : h->graph)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (h->hs) {
    (void)hipStreamSynchronize(h->hs);
    (void)hipStreamDestroy(h->hs);
  }
  if (h->ev) (void)hipEventDestroy(h->ev);
  if (h->host_st) (void)hipHostFree(h->host_st);
  delete h;
}

int pdhg_export_setup(pdhg_handle *h, uint8_t *var_kind, int32_t *colptr, int32_t *rowidx,
                      double *valT, double *val_s, double *Dr, double *Dc) {
  if (!h) return fail(PDHG_ERR_ARG, "null handle");
  int rc = enter(h);
  if (rc) return rc;
  auto d2h = [&](void *dst, const void *src, size_t bytes) -> int {
    if (dst) HC(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->hs));
    return PDHG_OK;
  };
  if ((rc = d2h(var_kind, h->vk, h->n))) return rc;
  if ((rc = d2h(colptr, h->cp, sizeof(int32_t) * (h->n + 1)))) return rc;
  if ((rc = d2h(rowidx, h->ri, sizeof(int32_t) * h->nnz))) return rc;
  if ((rc = d2h(valT, h->vt, sizeof(double) * h->nnz))) return rc;
  if ((rc = d2h(val_s, h->v, sizeof(double) * h->nnz))) return rc;
  if ((rc = d2h(Dr, h->Dr, sizeof(double) * h->m))) return rc;
  if ((rc = d2h(Dc, h->Dc, sizeof(double) * h->n))) return rc;
  HC(hipStreamSynchronize(h->hs));
  return leave(h);
}

int pdhg_spmv(pdhg_handle *h, int transpose, const double *x, double *out) {
  if (!h || !x || !out) return fail(PDHG_ERR_ARG, "null argument");
  int rc = enter(h);
  if (rc) return rc;
  int64_t nin = transpose ? h->m : h->n, nout = transpose ? h->n : h->m;
  double *din = transpose ? h->YA : h->XA;
  double *dout = transpose ? h->ATYA : h->AXA;
  HC(hipMemcpyAsync(din, x, sizeof(double) * nin, hipMemcpyHostToDevice, h->hs));
  if (transpose)
    launch_spmv(h->cp, h->ri, h->vt, h->n, din, dout, h->hs);
  else
    launch_spmv(h->rp, h->ci, h->v, h->m, din, dout, h->hs);
  HK();
  HC(hipMemcpyAsync(out, dout, sizeof(double) * nout, hipMemcpyDeviceToHost, h->hs));
  HC(hipStreamSynchronize(h->hs));
  return leave(h);
}

}  // extern "C"

namespace {
template <typename T>
int time_kernels(pdhg_handle *h, int attempts, double *ms) {
  IterView<T> w = iter_view<T>(h);
  hipEvent_t ev[4];
  for (auto &e : ev) HC(hipEventCreate(&e));
  double acc[4] = {0, 0, 0, 0};
  for (int a = 0; a < attempts; a++) {
    HC(hipEventRecord(ev[0], h->hs));
    launch_primal<T>(w, h->st, h->hs);
    HC(hipEventRecord(ev[1], h->hs));
    launch_dual<T>(w, h->st, h->hs);
    HC(hipEventRecord(ev[2], h->hs));
    launch_control<T>(w, h->st, h->hs);
    HC(hipEventRecord(ev[3], h->hs));
    HK();
    HC(hipEventSynchronize(ev[3]));
    float t;
    for (int q = 0; q < 3; q++) {
      HC(hipEventElapsedTime(&t, ev[q], ev[q + 1]));
      acc[q] += t;
    }
    HC(hipEventElapsedTime(&t, ev[0], ev[3]));
    acc[3] += t;
  }
  for (auto &e : ev) HC(hipEventDestroy(e));
  for (int q = 0; q < 4; q++) ms[q] = acc[q] / attempts;
  return PDHG_OK;
}
}  // namespace

extern "C" int pdhg_time_kernels(pdhg_handle *h, int attempts, double *ms_out) {
  if (!h || !ms_out || attempts < 1) return fail(PDHG_ERR_ARG, "bad argument");
  int rc = enter(h);
  if (rc) return rc;
  rc = h->o.precision == PDHG_MIXED ? time_kernels<float>(h, attempts, ms_out)
                                    : time_kernels<double>(h, attempts, ms_out);
  if (rc) return rc;
  return leave(h);
}
