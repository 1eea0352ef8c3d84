// Host side of the C ABI: argument checks, workspace carving, setup
// orchestration, and the block-by-block driver that replays iteration blocks
// as HIP graphs over a group of instances (one for pdhg_solve, many for
// pdhg_solve_batch).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <stddef.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
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

// ---------------------------------------------------------------------------
// The no-allocation batch (pdhg_solve_batch_static) carves its workspace out
// of this file-scope device array instead of a caller's buffer: at most
// PDHG_STATIC_SCRATCH_BYTES (pdhg.h), held by each GPU the library runs on
// until the process ends.  In host code the name `scratch` is only a
// stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device (static_scratch), and only that
// address is passed on.
#define PDHG_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[PDHG_STATIC_SCRATCH_BYTES];

std::mutex g_static_mu;                          // one no-allocation batch at a time
CtlState g_static_states[PDHG_STATIC_MAX_BATCH];  // its host mirror of the control states
std::mutex g_symbol_mu;
void *g_scratch_ptr[PDHG_MAX_DEVICES];           // device address of `scratch`, per device

// The current device's address of `scratch` (looked up on its first use).
int static_scratch(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= PDHG_MAX_DEVICES)
    return fail(PDHG_ERR_HIP, "no usable current device for the no-allocation scratch");
  std::lock_guard<std::mutex> lk(g_symbol_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PDHG_ERR_HIP, "hipGetSymbolAddress of the scratch array failed on device %d: %s",
                  dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PDHG_OK;
}

// Bump allocator over a caller's workspace; with base == nullptr it only
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

int nblk(int64_t n) { return (int)std::max<int64_t>(1, (n + PDHG_BLOCK - 1) / PDHG_BLOCK); }

// Device tables of an instance group: the Inst arrays the kernels read and
// the prefix tables of every launch shape, with room for `cap` instances.
struct GroupDev {
  int cap = 0;
  Inst<double> *d64 = nullptr;
  Inst<float> *d32 = nullptr;
  int32_t *pre = nullptr;         // 6 * (cap + 1)
  CtlState *dstates = nullptr;    // gathered states
  CtlState *hstates = nullptr;    // host mirror (pinned, except in the no-allocation batch)
  bool graphs = true;             // false: blocks are launched directly, never captured
};

void carve_group(Carver &cv, GroupDev &gd, int cap) {
  gd.cap = cap;
  gd.d64 = cv.take<Inst<double>>(cap);
  gd.d32 = cv.take<Inst<float>>(cap);
  gd.pre = cv.take<int32_t>(6 * (cap + 1));
  gd.dstates = cv.take<CtlState>(cap);
}

// Per-instance buffers: iterates of both precisions, evaluation vectors,
// partials and the control state.
struct IterBufs {
  double *X[2], *Y[2], *AX[2], *XS, *YS;
  float *Xf[2], *Yf[2], *AXf[2], *XSf, *YSf;
  double *XL, *YL, *XA, *YA, *AXA, *ATY, *ATYA;
  double *part_dx2, *part_dy, *ctl_stage, *ev_stage, *part_rows, *part_cols;
  CtlState *st;
};

void carve_iter(Carver &cv, IterBufs &b, int64_t m, int64_t n, int grid_rows, int grid_cols,
                bool mixed) {
  for (int q = 0; q < 2; q++) {
    b.X[q] = cv.take<double>(n);
    b.Y[q] = cv.take<double>(m);
    b.AX[q] = cv.take<double>(m);
  }
  b.XS = cv.take<double>(n);
  b.YS = cv.take<double>(m);
  for (int q = 0; q < 2; q++) {
    b.Xf[q] = mixed ? cv.take<float>(n) : nullptr;
    b.Yf[q] = mixed ? cv.take<float>(m) : nullptr;
    b.AXf[q] = mixed ? cv.take<float>(m) : nullptr;
  }
  b.XSf = mixed ? cv.take<float>(n) : nullptr;
  b.YSf = mixed ? cv.take<float>(m) : nullptr;
  b.XL = cv.take<double>(n);
  b.YL = cv.take<double>(m);
  b.XA = cv.take<double>(n);
  b.YA = cv.take<double>(m);
  b.AXA = cv.take<double>(m);
  b.ATY = cv.take<double>(n);
  b.ATYA = cv.take<double>(n);
  b.part_dx2 = cv.take<double>(grid_cols);
  b.part_dy = cv.take<double>(2 * (int64_t)grid_rows);
  b.ctl_stage = cv.take<double>(3 * PDHG_CTL_SPLIT);
  b.ev_stage = cv.take<double>((EV_ROWQ + EV_COLQ) * PDHG_CTL_SPLIT);
  b.part_rows = cv.take<double>((int64_t)nblk(m) * EV_ROWQ);
  b.part_cols = cv.take<double>((int64_t)nblk(n) * EV_COLQ);
  b.st = cv.take<CtlState>(1);
}

}  // namespace

struct pdhg_handle {
  int64_t m = 0, n = 0, nnz = 0;
  pdhg_opts o{};
  int on_device = 0;
  double obj_offset = 0.0;  // added to the reported objectives only
  int stream_nt[2] = {1, 1};  // attempt kernels' load policy per precision (FP64, FP32)
  // the iterate buffers and control state hold a solve's state (pdhg_solve
  // initialises them; setup leaves the iterate part of the state unset)
  bool state_ready = false;
  hipStream_t hs = nullptr;
  hipStream_t user = nullptr;
  hipEvent_t ev = nullptr;
  bool hip_failed = false;
  double setup_s = 0.0;

  // preprocessed problem (shared by every instance built on this handle)
  int32_t *rp, *ci, *cp, *ri, *long_rows, *long_cols, *scan_tmp, *tmp_next;
  double *v, *vt, *b0, *c0, *l0, *u0, *b, *c, *l, *u, *Dr, *Dc;
  float *vf = nullptr, *vtf = nullptr, *bf = nullptr, *cf = nullptr, *lf = nullptr,
        *uf = nullptr;
  uint8_t *kind, *vk;
  // 16-bit tile-relative structure of A (rows) and A' (columns), used by the
  // attempt kernels when `compact` (every tile fits)
  uint16_t *rofs, *cofs, *cix16, *rix16;
  int32_t *tb_rows, *tb_cols;
  bool compact = false;
  // locality ordering: caller's index of each internal row / column and the
  // internal index of each caller column (all null without reordering)
  int32_t *rperm = nullptr, *cperm = nullptr, *cinv = nullptr;
  int32_t *perm_buf = nullptr;
  std::vector<int32_t> h_rperm, h_cperm;  // host copies
  // implied bounds for the dual bound: device (scaled, internal order) and
  // host (caller's order, original units), and the caller's l, u
  double *ilo = nullptr, *ihi = nullptr;
  std::vector<double> h_ilo, h_ihi, h_l, h_u;
  bool impl_valid = false;
  // the dual bound's repair interval of each row: device (scaled, internal
  // order) and host (caller's order, original units)
  double *rylo = nullptr, *ryhi = nullptr;
  std::vector<double> h_ylo, h_yhi;
  // the same repair for c = 0 (the Farkas test): per row, bit 0 keeps y >= 0
  // and bit 1 keeps y <= 0 (the intervals' ends are 0 or infinite)
  uint8_t *fyk = nullptr;
  std::vector<uint8_t> h_fyk;
  bool rep_valid = false;
  // c'x is bounded below on the implied box (setup's b, c): no direction of
  // its recession cone improves the objective, so the ray test is skipped
  bool obj_bounded = false;
  double bound_allow = 0.0;
  double *scratch;
  int nscratch = 0;
  int *err;
  int n_long_rows = 0, n_long_cols = 0, nblk_rows = 0, nblk_cols = 0;
  int tpb_rows = 1, tpb_cols = 1;
  int grid_rows[2] = {1, 1}, grid_cols[2] = {1, 1};  // attempt grids: [FP64, FP32]
  int long_seg = PDHG_LONG_SEG;  // SpMV partition (chosen by the autotuner or the options)
  int direct = 0;
  std::vector<int32_t> hrp, hcp;  // host copies of the row / column pointers

  // unrolled mode: checkpoints (x, y, Ax) every ur_C steps, masks of one
  // segment, adjoint vectors, and the forward's step sizes
  double *ckpt = nullptr, *XB = nullptr, *YB = nullptr, *H = nullptr, *BB = nullptr,
         *CB = nullptr, *XK = nullptr;
  uint64_t *mask_x = nullptr, *mask_y = nullptr;
  int64_t ur_K = 0, ur_C = 0;
  double ur_eta = 0, ur_omega = 0;
  bool ur_valid = false;

  // feasibility polishing (pdhg_polish): the polished primal and dual points
  // (caller's order, original space), discarded outputs, a zero vector and
  // the bounds with their finite entries zeroed (scaled space)
  double *pol_x = nullptr, *pol_y = nullptr, *pol_xd = nullptr, *pol_yd = nullptr,
         *pol_zero = nullptr, *pol_lz = nullptr, *pol_uz = nullptr;

  // the handle's own instance (pdhg_solve) and its cached block graphs
  IterBufs it{};
  GroupDev grp{};
  struct Slot {
    hipGraphExec_t exec = nullptr;
    int period = 0;
    double tol = 0;
    int64_t max_iter = 0;
    int version = 0;
  } graph[2];
};

namespace {

typedef pdhg_handle::Slot GraphSlot;

void partition(pdhg_handle *h) {
  h->nblk_rows = nblk(h->m);
  h->nblk_cols = nblk(h->n);
  h->tpb_rows = h->o.tiles_per_block > 0
                    ? h->o.tiles_per_block
                    : std::max(1, (h->nblk_rows + PDHG_TARGET_GROUPS - 1) / PDHG_TARGET_GROUPS);
  h->tpb_cols = h->o.tiles_per_block > 0
                    ? h->o.tiles_per_block
                    : std::max(1, (h->nblk_cols + PDHG_TARGET_GROUPS - 1) / PDHG_TARGET_GROUPS);
}

void set_grids(pdhg_handle *h) {
  for (int q = 0; q < 2; q++) {
    int64_t tile = PDHG_TILE;
    int tr = (int)((h->m + tile - 1) / tile), tc = (int)((h->n + tile - 1) / tile);
    h->grid_rows[q] = h->n_long_rows + (tr + h->tpb_rows - 1) / h->tpb_rows;
    h->grid_cols[q] = h->n_long_cols + (tc + h->tpb_cols - 1) / h->tpb_cols;
  }
}

size_t layout(pdhg_handle *h, void *base) {
  Carver cv(base);
  int64_t m = h->m, n = h->n, nnz = h->nnz;
  bool mixed = h->o.precision == PDHG_MIXED;
  partition(h);
  h->rp = cv.take<int32_t>(m + 1);
  h->ci = cv.take<int32_t>(std::max<int64_t>(nnz, 1));  // the attempt kernels may read entry 0 of an empty matrix
  h->cp = cv.take<int32_t>(n + 1);
  h->ri = cv.take<int32_t>(std::max<int64_t>(nnz, 1));
  h->long_rows = cv.take<int32_t>(m);
  h->long_cols = cv.take<int32_t>(n);
  h->rofs = cv.take<uint16_t>(m);
  h->cofs = cv.take<uint16_t>(n);
  // index and value arrays: two entries past the last nonzero, which the
  // paired loads of the attempt kernels may read
  h->cix16 = cv.take<uint16_t>(nnz + 2);
  h->rix16 = cv.take<uint16_t>(nnz + 2);
  h->tb_rows = cv.take<int32_t>(nblk(m));
  h->tb_cols = cv.take<int32_t>(nblk(n));
  h->scan_tmp = cv.take<int32_t>(scan_tmp_ints(n + 1));
  h->tmp_next = cv.take<int32_t>(n + 1);
  h->v = cv.take<double>(nnz + 2);
  h->vt = cv.take<double>(nnz + 2);
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
  h->perm_buf = h->o.reorder ? cv.take<int32_t>(m + 2 * n) : nullptr;
  h->ilo = cv.take<double>(n);
  h->ihi = cv.take<double>(n);
  h->rylo = cv.take<double>(m);
  h->ryhi = cv.take<double>(m);
  h->fyk = cv.take<uint8_t>(m);
  if (mixed) {
    h->vf = cv.take<float>(nnz + 2);
    h->vtf = cv.take<float>(nnz + 2);
    h->bf = cv.take<float>(m);
    h->cf = cv.take<float>(n);
    h->lf = cv.take<float>(n);
    h->uf = cv.take<float>(n);
  }
  h->nscratch = 5 * 1024;
  h->scratch = cv.take<double>(h->nscratch);
  h->err = cv.take<int>(1);
  // worst-case grids: every row and column long
  int gr = (int)std::min<int64_t>(m + h->nblk_rows, 0x7fffffff);
  int gc = (int)std::min<int64_t>(n + h->nblk_cols, 0x7fffffff);
  carve_iter(cv, h->it, m, n, gr, gc, mixed);
  carve_group(cv, h->grp, 1);
  h->pol_x = cv.take<double>(n);
  h->pol_y = cv.take<double>(m);
  h->pol_xd = cv.take<double>(n);
  h->pol_yd = cv.take<double>(m);
  h->pol_zero = cv.take<double>(std::max(m, n));
  h->pol_lz = cv.take<double>(n);
  h->pol_uz = cv.take<double>(n);
  if (h->o.unroll_iters > 0) {
    int64_t K = h->o.unroll_iters;
    int64_t C = h->o.checkpoint_every > 0 ? std::min<int64_t>(h->o.checkpoint_every, K) : K;
    int64_t S = (K + C - 1) / C;
    h->ur_K = K;
    h->ur_C = C;
    h->ckpt = cv.take<double>(S * (n + 2 * m));
    h->mask_x = cv.take<uint64_t>(C * ((n + 63) / 64));
    h->mask_y = cv.take<uint64_t>(C * ((m + 63) / 64));
    h->XB = cv.take<double>(n);
    h->YB = cv.take<double>(m);
    h->H = cv.take<double>(n);
    h->BB = cv.take<double>(m);
    h->CB = cv.take<double>(n);
    h->XK = cv.take<double>(n);
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
  if (o->long_seg < 0) return fail(PDHG_ERR_ARG, "long_seg must be >= 0");
  if (o->reorder != 0 && o->reorder != 1) return fail(PDHG_ERR_ARG, "reorder must be 0 or 1");
  if (o->compact_index != 0 && o->compact_index != 1)
    return fail(PDHG_ERR_ARG, "compact_index must be 0 or 1");
  if (o->infeas_every < 0) return fail(PDHG_ERR_ARG, "infeas_every must be >= 0");
  if (o->polish_pw_update != 0 && o->polish_pw_update != 1)
    return fail(PDHG_ERR_ARG, "polish_pw_update must be 0 or 1");
  if (o->fp32_stall_evals < 0) return fail(PDHG_ERR_ARG, "fp32_stall_evals must be >= 0");
  if (!(o->dinf_tol >= 0.0) || !isfinite(o->dinf_tol))
    return fail(PDHG_ERR_ARG, "dinf_tol must be finite and >= 0");
  if (o->batch_pack != 0 && o->batch_pack != 1) return fail(PDHG_ERR_ARG, "batch_pack must be 0 or 1");
  if (o->stream_nt < -1 || o->stream_nt > 1)
    return fail(PDHG_ERR_ARG, "stream_nt must be -1, 0 or 1");
  if (o->polish_fp32_matrix != 0 && o->polish_fp32_matrix != 1)
    return fail(PDHG_ERR_ARG, "polish_fp32_matrix must be 0 or 1");
  if (o->unroll_iters > 0 && o->precision != PDHG_FP64)
    return fail(PDHG_ERR_ARG, "unrolled mode runs in FP64");
  if (o->unroll_iters > 0 && o->checkpoint_every < 0)
    return fail(PDHG_ERR_ARG, "checkpoint_every must be >= 0");
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
  if (!isfinite(lp->obj_offset)) return fail(PDHG_ERR_NONFINITE, "obj_offset is not finite");
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

#define RC(call)       \
  do {                 \
    int r_ = (call);   \
    if (r_) return r_; \
  } while (0)

// A caller-order vector src (host or device memory) into internal order:
// dst[i] = src[perm[i]] (device), staged through `staging` (cnt doubles) when
// src is host memory.  perm null: a plain copy.
int to_internal(pdhg_handle *h, double *dst, const double *src, int src_on_device,
                const int32_t *perm, int64_t cnt, double *staging) {
  hipMemcpyKind kd = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (!perm) {
    HC(hipMemcpyAsync(dst, src, sizeof(double) * cnt, kd, h->hs));
    return PDHG_OK;
  }
  const double *from = src;
  if (!src_on_device) {
    HC(hipMemcpyAsync(staging, src, sizeof(double) * cnt, hipMemcpyHostToDevice, h->hs));
    from = staging;
  }
  launch_gather_f64(dst, from, perm, cnt, h->hs);
  HK();
  return PDHG_OK;
}

// An internal-order device vector into the caller's order: dst[perm[i]] = src[i].
int to_caller(pdhg_handle *h, double *dst, const double *src, const int32_t *perm, int64_t cnt) {
  if (perm)
    launch_scatter_f64(dst, src, perm, cnt, h->hs);
  else
    launch_copy_f64(dst, src, cnt, h->hs);
  HK();
  return PDHG_OK;
}

// Relabel the scaled problem by the locality ordering: the CSR of P A Q' is
// built on the host from the scaled matrix, its transpose on the device by
// the setup kernel, and every problem vector is gathered into the new order.
int reorder_problem(pdhg_handle *h) {
  const int64_t m = h->m, n = h->n, nnz = h->nnz;
  std::vector<int32_t> rp(m + 1), ci(std::max<int64_t>(nnz, 1));
  std::vector<double> v(std::max<int64_t>(nnz, 1));
  HC(hipMemcpyAsync(rp.data(), h->rp, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost, h->hs));
  if (nnz) {
    HC(hipMemcpyAsync(ci.data(), h->ci, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(v.data(), h->v, sizeof(double) * nnz, hipMemcpyDeviceToHost, h->hs));
  }
  HC(hipStreamSynchronize(h->hs));
  std::vector<int32_t> cp, ri, ro, co, prp, pci;
  std::vector<double> none, pv;
  transpose_csr(m, n, rp.data(), ci.data(), nullptr, cp, ri, none);
  rcm_order(m, n, rp.data(), ci.data(), cp.data(), ri.data(), ro, co);
  std::vector<int32_t> cinv(n);
  for (int64_t j = 0; j < n; j++) cinv[co[j]] = (int32_t)j;
  permute_csr(m, rp.data(), ci.data(), v.data(), ro, cinv, prp, pci, pv);
  h->rperm = h->perm_buf;
  h->cperm = h->perm_buf + m;
  h->cinv = h->perm_buf + m + n;
  HC(hipMemcpyAsync(h->rperm, ro.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, h->hs));
  HC(hipMemcpyAsync(h->cperm, co.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, h->hs));
  HC(hipMemcpyAsync(h->cinv, cinv.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, h->hs));
  HC(hipMemcpyAsync(h->rp, prp.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, h->hs));
  if (nnz) {
    HC(hipMemcpyAsync(h->ci, pci.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, h->hs));
    HC(hipMemcpyAsync(h->v, pv.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, h->hs));
  }
  launch_transpose(h->rp, h->ci, h->v, m, n, nnz, h->cp, h->ri, h->vt, h->tmp_next, h->scan_tmp,
                   h->hs);
  HK();
  double *tr = h->it.YA, *tc = h->it.XA;  // free until the first solve
  for (double *a : {h->b0, h->b, h->Dr}) {
    launch_copy_f64(tr, a, m, h->hs);
    launch_gather_f64(a, tr, h->rperm, m, h->hs);
  }
  for (double *a : {h->c0, h->l0, h->u0, h->c, h->l, h->u, h->Dc}) {
    launch_copy_f64(tc, a, n, h->hs);
    launch_gather_f64(a, tc, h->cperm, n, h->hs);
  }
  HC(hipMemcpyAsync(tr, h->kind, m, hipMemcpyDeviceToDevice, h->hs));
  launch_gather_u8(h->kind, (const uint8_t *)tr, h->rperm, m, h->hs);
  HC(hipMemcpyAsync(tc, h->vk, n, hipMemcpyDeviceToDevice, h->hs));
  launch_gather_u8(h->vk, (const uint8_t *)tc, h->cperm, n, h->hs);
  HK();
  HC(hipStreamSynchronize(h->hs));  // the host arrays go out of scope
  h->h_rperm = std::move(ro);
  h->h_cperm = std::move(co);
  return PDHG_OK;
}

// The dual bound's repair interval of each row, in the caller's order and
// units: a column with one nonzero a_ij and an infinite bound on a side
// needs its reduced cost c_j - a_ij y_i to keep a sign (>= 0 for an infinite
// upper bound, <= 0 for an infinite lower one), a half-line for y_i with end
// t = c_j / a_ij moved inward by 2^-40 |t|; the row's interval is the
// intersection of its half-lines with y_i >= 0 on >= rows (no repair when
// it is empty).  lo, hi: l, u tightened by the implied bounds.
void repair_intervals(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                      const uint8_t *kind, const double *c, const double *lo, const double *hi,
                      std::vector<double> &ylo, std::vector<double> &yhi) {
  std::vector<int32_t> cnt(n, 0);
  std::vector<int64_t> row(n, 0);
  std::vector<double> val(n, 0.0);
  for (int64_t i = 0; i < m; i++)
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      cnt[ci[k]]++;
      row[ci[k]] = i;
      val[ci[k]] = v[k];
    }
  ylo.assign(m, -INFINITY);
  yhi.assign(m, INFINITY);
  for (int64_t i = 0; i < m; i++)
    if (kind[i] == 1) ylo[i] = 0.0;
  const double margin = std::ldexp(1.0, -40);
  for (int64_t j = 0; j < n; j++) {
    if (cnt[j] != 1 || val[j] == 0.0) continue;
    const int64_t i = row[j];
    const double a = val[j], t = c[j] / a;
    const double below = t - margin * std::fabs(t), above = t + margin * std::fabs(t);
    if (std::isinf(hi[j])) {  // a y_i <= c_j
      if (a > 0.0)
        yhi[i] = std::fmin(yhi[i], below);
      else
        ylo[i] = std::fmax(ylo[i], above);
    }
    if (std::isinf(lo[j])) {  // a y_i >= c_j
      if (a > 0.0)
        ylo[i] = std::fmax(ylo[i], above);
      else
        yhi[i] = std::fmin(yhi[i], below);
    }
  }
  for (int64_t i = 0; i < m; i++)
    if (ylo[i] > yhi[i]) {
      ylo[i] = kind[i] == 1 ? 0.0 : -INFINITY;
      yhi[i] = INFINITY;
    }
}

// Implied bounds of the caller's problem (original order and units), from
// the host copy of the LP; the longest column sets the rounding allowance of
// the dual bound.
int setup_implied_bounds(pdhg_handle *h, const pdhg_lp *lp) {
  const int64_t m = h->m, n = h->n, nnz = h->nnz;
  std::vector<int32_t> rp, ci;
  std::vector<double> v, b;
  std::vector<uint8_t> kind;
  const int32_t *prp = lp->row_ptr, *pci = lp->col_idx;
  const double *pv = lp->val, *pb = lp->b;
  const uint8_t *pk = lp->row_kind;
  h->h_l.resize(n);
  h->h_u.resize(n);
  if (h->on_device) {
    rp.resize(m + 1);
    ci.resize(std::max<int64_t>(nnz, 1));
    v.resize(std::max<int64_t>(nnz, 1));
    b.resize(m);
    kind.resize(m);
    HC(hipMemcpyAsync(rp.data(), lp->row_ptr, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost,
                      h->hs));
    if (nnz) {
      HC(hipMemcpyAsync(ci.data(), lp->col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost,
                        h->hs));
      HC(hipMemcpyAsync(v.data(), lp->val, sizeof(double) * nnz, hipMemcpyDeviceToHost, h->hs));
    }
    HC(hipMemcpyAsync(b.data(), lp->b, sizeof(double) * m, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(kind.data(), lp->row_kind, m, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(h->h_l.data(), lp->l, sizeof(double) * n, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(h->h_u.data(), lp->u, sizeof(double) * n, hipMemcpyDeviceToHost, h->hs));
    HC(hipStreamSynchronize(h->hs));
    prp = rp.data();
    pci = ci.data();
    pv = v.data();
    pb = b.data();
    pk = kind.data();
  } else {
    std::copy(lp->l, lp->l + n, h->h_l.begin());
    std::copy(lp->u, lp->u + n, h->h_u.begin());
  }
  h->h_ilo = h->h_l;
  h->h_ihi = h->h_u;
  implied_bounds(m, prp, pci, pv, pk, pb, 64, h->h_ilo.data(), h->h_ihi.data());
  std::vector<double> hc(n);
  if (h->on_device) {
    HC(hipMemcpyAsync(hc.data(), lp->c, sizeof(double) * n, hipMemcpyDeviceToHost, h->hs));
    HC(hipStreamSynchronize(h->hs));
  } else {
    std::copy(lp->c, lp->c + n, hc.begin());
  }
  repair_intervals(m, n, prp, pci, pv, pk, hc.data(), h->h_ilo.data(), h->h_ihi.data(), h->h_ylo,
                   h->h_yhi);
  {
    std::vector<double> zero(n, 0.0), flo, fhi;
    repair_intervals(m, n, prp, pci, pv, pk, zero.data(), h->h_ilo.data(), h->h_ihi.data(), flo,
                     fhi);
    h->h_fyk.assign(m, 0);
    for (int64_t i = 0; i < m; i++)
      h->h_fyk[i] = (uint8_t)((flo[i] == 0.0 ? 1 : 0) | (fhi[i] == 0.0 ? 2 : 0));
  }
  // every feasible x lies in the implied box, so every ray of the feasible
  // set lies in the box's recession cone; c'd >= 0 there when each term
  // c_j x_j is bounded below on [lo_j, hi_j]
  h->obj_bounded = true;
  for (int64_t j = 0; j < n && h->obj_bounded; j++) {
    const bool flo = isfinite(h->h_ilo[j]), fhi = isfinite(h->h_ihi[j]);
    const double cj = hc[j];
    h->obj_bounded = (flo && fhi) || cj == 0.0 || (cj > 0.0 && flo) || (cj < 0.0 && fhi);
  }
  std::vector<int64_t> clen(n, 0);
  int64_t kmax = 0;
  for (int64_t k = 0; k < nnz; k++) kmax = std::max(kmax, ++clen[pci[k]]);
  h->bound_allow = 2.0 * (double)(n + m + kmax + 4) * std::ldexp(1.0, -53);
  return PDHG_OK;
}

// The implied bounds on the device: internal order, scaled like l and u.
int upload_implied_bounds(pdhg_handle *h) {
  const int64_t n = h->n;
  double *tl = h->it.XA, *tu = h->it.ATY, *tg = h->it.ATYA;  // free during setup
  HC(hipMemcpyAsync(tl, h->h_ilo.data(), sizeof(double) * n, hipMemcpyHostToDevice, h->hs));
  HC(hipMemcpyAsync(tu, h->h_ihi.data(), sizeof(double) * n, hipMemcpyHostToDevice, h->hs));
  if (h->cperm) {
    launch_gather_f64(tg, tl, h->cperm, n, h->hs);
    launch_copy_f64(tl, tg, n, h->hs);
    launch_gather_f64(tg, tu, h->cperm, n, h->hs);
    launch_copy_f64(tu, tg, n, h->hs);
  }
  // (the scaled-c output of this launcher goes to the free buffer tg)
  launch_scale_vectors(nullptr, tl, tl, tu, h->Dr, h->Dc, 0, n, nullptr, tg, h->ilo, h->ihi, h->hs);
  HK();
  // repair intervals: internal order, divided by the row factors (exact)
  const int64_t m = h->m;
  std::vector<double> dr(m), lo(m), hi(m);
  HC(hipMemcpyAsync(dr.data(), h->Dr, sizeof(double) * m, hipMemcpyDeviceToHost, h->hs));
  HC(hipStreamSynchronize(h->hs));
  for (int64_t i = 0; i < m; i++) {
    const int64_t r = h->rperm ? h->h_rperm[i] : i;
    lo[i] = h->h_ylo[r] / dr[i];
    hi[i] = h->h_yhi[r] / dr[i];
  }
  HC(hipMemcpyAsync(h->rylo, lo.data(), sizeof(double) * m, hipMemcpyHostToDevice, h->hs));
  HC(hipMemcpyAsync(h->ryhi, hi.data(), sizeof(double) * m, hipMemcpyHostToDevice, h->hs));
  std::vector<uint8_t> fk(m);
  for (int64_t i = 0; i < m; i++) fk[i] = h->h_fyk[h->rperm ? h->h_rperm[i] : i];
  HC(hipMemcpyAsync(h->fyk, fk.data(), m, hipMemcpyHostToDevice, h->hs));
  HC(hipStreamSynchronize(h->hs));  // the host arrays go out of scope; keep setup ordered
  h->impl_valid = true;
  h->rep_valid = true;
  return PDHG_OK;
}

// The 16-bit form of the final (scaled, reordered) structure, kept when
// every tile of both matrices fits it.
int build_compact(pdhg_handle *h) {
  h->compact = false;
  if (!h->o.compact_index) return PDHG_OK;
  HC(hipMemsetAsync(h->err, 0, sizeof(int), h->hs));
  launch_compact(h->rp, h->ci, h->m, h->rofs, h->cix16, h->tb_rows, h->err, h->hs);
  launch_compact(h->cp, h->ri, h->n, h->cofs, h->rix16, h->tb_cols, h->err, h->hs);
  HK();
  int herr = 0;
  HC(hipMemcpyAsync(&herr, h->err, sizeof(int), hipMemcpyDeviceToHost, h->hs));
  HC(hipStreamSynchronize(h->hs));
  h->compact = herr == 0;
  return PDHG_OK;
}

// Load policy of the attempt kernels' streams per iteration precision
// (stream_nt[0] FP64, [1] FP32): non-temporal when the larger of the two
// attempt kernels moves at least three quarters of the 256 MiB Infinity
// Cache, so that L2 keeps the gathered windows; ordinary loads below, whose
// lines the Infinity Cache can hold for the next launch.  The bytes are the
// kernels' own storage form (structure, values, the gathered vector, the
// streamed, written and folded vectors).
void set_stream_policy(pdhg_handle *h) {
  const double m = (double)h->m, n = (double)h->n, nnz = (double)h->nnz;
  auto structure = [&](double r) {
    return h->compact ? 2 * r + 8 * ceil(r / PDHG_TILE) + 2 * nnz : 4 * (r + 1) + 4 * nnz;
  };
  for (int f = 0; f < 2; f++) {
    const double vb = f ? 4.0 : 8.0;
    const double primal = structure(n) + vb * nnz + vb * m + 7 * vb * n;
    const double dual = structure(m) + vb * nnz + vb * n + 7 * vb * m + m;
    const bool big = std::max(primal, dual) >= 0.75 * 256.0 * 1024 * 1024;
    h->stream_nt[f] = h->o.stream_nt < 0 ? (big ? 1 : 0) : h->o.stream_nt;
  }
}

// Rows and columns longer than the partition's threshold get a workgroup each.
int build_long_lists(pdhg_handle *h) {
  std::vector<int32_t> lr, lc;
  for (int64_t i = 0; i < h->m; i++)
    if (h->hrp[i + 1] - h->hrp[i] > h->long_seg) lr.push_back((int32_t)i);
  for (int64_t j = 0; j < h->n; j++)
    if (h->hcp[j + 1] - h->hcp[j] > h->long_seg) lc.push_back((int32_t)j);
  h->n_long_rows = (int)lr.size();
  h->n_long_cols = (int)lc.size();
  if (!lr.empty())
    HC(hipMemcpyAsync(h->long_rows, lr.data(), sizeof(int32_t) * lr.size(), hipMemcpyHostToDevice,
                      h->hs));
  if (!lc.empty())
    HC(hipMemcpyAsync(h->long_cols, lc.data(), sizeof(int32_t) * lc.size(), hipMemcpyHostToDevice,
                      h->hs));
  HC(hipStreamSynchronize(h->hs));
  set_grids(h);
  return PDHG_OK;
}

int apply_partition(pdhg_handle *h, int tpb, int direct, int long_seg) {
  h->tpb_rows = h->tpb_cols = tpb;
  h->direct = direct;
  h->long_seg = long_seg;
  return build_long_lists(h);
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

// ---------------------------------------------------------------------------
// instance views

// Scaled problem vectors of one instance; defaults are the handle's.
struct InstData {
  const double *b, *c, *l, *u;
  const float *bf, *cf, *lf, *uf;
  const uint8_t *vk;
};

InstData base_data(const pdhg_handle *h) {
  return InstData{h->b, h->c, h->l, h->u, h->bf, h->cf, h->lf, h->uf, h->vk};
}

template <typename T>
void fill_common(Inst<T> &I, const pdhg_handle *h, const InstData &d, const IterBufs &b) {
  IterView<T> &w = I.w;
  EvalView<T> &e = I.e;
  w.m = e.m = h->m;
  w.n = e.n = h->n;
  w.rp = e.rp = h->rp;
  w.ci = e.ci = h->ci;
  w.cp = e.cp = h->cp;
  w.ri = e.ri = h->ri;
  w.kind = e.kind = h->kind;
  w.vk = e.vk = d.vk;
  w.nblk_rows = e.nblk_rows = h->nblk_rows;
  w.nblk_cols = e.nblk_cols = h->nblk_cols;
  w.long_rows = h->long_rows;
  w.long_cols = h->long_cols;
  w.n_long_rows = h->n_long_rows;
  w.n_long_cols = h->n_long_cols;
  w.tpb_rows = h->tpb_rows;
  w.tpb_cols = h->tpb_cols;
  w.grid_rows = h->grid_rows[sizeof(T) == 4];
  w.grid_cols = h->grid_cols[sizeof(T) == 4];
  w.part_dx2 = b.part_dx2;
  w.part_dy = b.part_dy;
  w.ctl_stage = b.ctl_stage;
  w.adaptive = h->o.step_mode == 0;
  w.long_seg = e.long_seg = h->long_seg;
  w.direct = h->direct;
  w.rofs = h->compact ? h->rofs : nullptr;
  w.cofs = h->compact ? h->cofs : nullptr;
  w.cix16 = h->compact ? h->cix16 : nullptr;
  w.rix16 = h->compact ? h->rix16 : nullptr;
  w.tb_rows = h->compact ? h->tb_rows : nullptr;
  w.tb_cols = h->compact ? h->tb_cols : nullptr;
  e.v = h->v;
  e.vt = h->vt;
  e.b = d.b;
  e.c = d.c;
  e.l = d.l;
  e.u = d.u;
  e.Dr = h->Dr;
  e.Dc = h->Dc;
  e.rperm = h->rperm;
  e.cperm = h->cperm;
  e.XA = b.XA;
  e.YA = b.YA;
  e.AXA = b.AXA;
  e.ATY = b.ATY;
  e.ATYA = b.ATYA;
  e.XL = b.XL;
  e.YL = b.YL;
  e.part_rows = b.part_rows;
  e.part_cols = b.part_cols;
  e.ev_stage = b.ev_stage;
  e.xbest = sizeof(T) == 4 ? b.X[0] : nullptr;
  e.ilo = h->impl_valid ? h->ilo : nullptr;
  e.ihi = h->impl_valid ? h->ihi : nullptr;
  e.rylo = h->rep_valid ? h->rylo : nullptr;
  e.ryhi = h->rep_valid ? h->ryhi : nullptr;
  e.bound_allow = h->bound_allow;
  e.ybest = sizeof(T) == 4 ? b.Y[0] : nullptr;
  e.use_average = h->o.use_average;
  e.term = 0;
  e.restart = h->o.restart;
  e.pw_theta = h->o.pw_update ? h->o.pw_theta : 0.0;
  e.hold_k = 0;
  e.infeas_period = (long long)h->o.eval_period * h->o.infeas_every;
  e.dinf_tol = h->obj_bounded ? 0.0 : h->o.dinf_tol;
  I.st = b.st;
  I.x0 = I.y0 = nullptr;
  I.xout = I.yout = nullptr;
  I.fyk = h->impl_valid ? h->fyk : nullptr;
}

template <typename T>
Inst<T> make_inst(const pdhg_handle *h, const InstData &d, const IterBufs &b);

template <>
Inst<double> make_inst<double>(const pdhg_handle *h, const InstData &d, const IterBufs &b) {
  Inst<double> I{};
  fill_common(I, h, d, b);
  I.w.v = h->v;
  I.w.vt = h->vt;
  I.w.v32 = h->vf;  // null unless the handle is mixed
  I.w.vt32 = h->vtf;
  I.w.b = d.b;
  I.w.c = d.c;
  I.w.l = d.l;
  I.w.u = d.u;
  for (int q = 0; q < 2; q++) {
    I.w.X[q] = I.e.X[q] = b.X[q];
    I.w.Y[q] = I.e.Y[q] = b.Y[q];
    I.w.AX[q] = I.e.AX[q] = b.AX[q];
  }
  I.w.XS = I.e.XS = b.XS;
  I.w.YS = I.e.YS = b.YS;
  return I;
}

template <>
Inst<float> make_inst<float>(const pdhg_handle *h, const InstData &d, const IterBufs &b) {
  Inst<float> I{};
  fill_common(I, h, d, b);
  I.w.v = h->vf;
  I.w.vt = h->vtf;
  I.w.b = d.bf;
  I.w.c = d.cf;
  I.w.l = d.lf;
  I.w.u = d.uf;
  for (int q = 0; q < 2; q++) {
    I.w.X[q] = I.e.X[q] = b.Xf[q];
    I.w.Y[q] = I.e.Y[q] = b.Yf[q];
    I.w.AX[q] = I.e.AX[q] = b.AXf[q];
  }
  I.w.XS = I.e.XS = b.XSf;
  I.w.YS = I.e.YS = b.YSf;
  return I;
}

template <typename T>
Inst<T> *dev_insts(GroupDev &gd);
template <>
Inst<double> *dev_insts<double>(GroupDev &gd) {
  return gd.d64;
}
template <>
Inst<float> *dev_insts<float>(GroupDev &gd) {
  return gd.d32;
}

// Upload the active instances and the prefix tables of every launch shape.
template <typename T>
int upload_group(pdhg_handle *h, GroupDev &gd, const std::vector<Inst<T>> &all,
                 const std::vector<int> &act, Groups &g) {
  int na = (int)act.size();
  int c1 = gd.cap + 1;
  std::vector<Inst<T>> sel(na);
  std::vector<int32_t> pre(6 * c1, 0);
  for (int k = 0; k < na; k++) {
    const Inst<T> &I = all[act[k]];
    sel[k] = I;
    int cnt[6] = {I.w.grid_cols, I.w.grid_rows, I.e.nblk_rows, I.e.nblk_cols, I.w.n_long_rows,
                  I.w.n_long_cols};
    for (int s = 0; s < 6; s++) pre[s * c1 + k + 1] = pre[s * c1 + k] + cnt[s];
  }
  HC(hipMemcpyAsync(dev_insts<T>(gd), sel.data(), sizeof(Inst<T>) * na, hipMemcpyHostToDevice,
                    h->hs));
  HC(hipMemcpyAsync(gd.pre, pre.data(), sizeof(int32_t) * pre.size(), hipMemcpyHostToDevice, h->hs));
  HC(hipStreamSynchronize(h->hs));  // the host staging vectors go out of scope
  const int32_t *p = gd.pre;
  g.ninst = na;
  g.p_primal = p;
  g.p_dual = p + c1;
  g.p_rows = p + 2 * c1;
  g.p_cols = p + 3 * c1;
  g.p_lrows = p + 4 * c1;
  g.p_lcols = p + 5 * c1;
  g.n_primal = pre[na];
  g.n_dual = pre[c1 + na];
  g.n_rows = pre[2 * c1 + na];
  g.n_cols = pre[3 * c1 + na];
  g.n_lrows = pre[4 * c1 + na];
  g.n_lcols = pre[5 * c1 + na];
  g.compact = 1;
  for (int k = 0; k < na; k++) g.compact = g.compact && sel[k].w.cix16 != nullptr;
  g.nt = h->stream_nt[sizeof(T) == 4];
  g.v32 = sizeof(T) == 8;
  for (int k = 0; k < na; k++) g.v32 = g.v32 && sel[k].w.use_v32 && sel[k].w.v32 && sel[k].w.vt32;
  g.interleave = na > 1;
  for (int k = 1; k < na && g.interleave; k++) {
    const IterView<T> &a = sel[0].w, &b = sel[k].w;
    g.interleave = a.rp == b.rp && a.cp == b.cp && a.v == b.v && a.vt == b.vt &&
                   a.grid_rows == b.grid_rows && a.grid_cols == b.grid_cols &&
                   a.tpb_rows == b.tpb_rows && a.tpb_cols == b.tpb_cols &&
                   a.n_long_rows == b.n_long_rows && a.n_long_cols == b.n_long_cols &&
                   a.long_seg == b.long_seg && a.direct == b.direct;
  }
  // shared-matrix instances walked a pack at a time (same tiles, partials and
  // bits as one at a time)
  const IterView<T> &w0 = sel[0].w;
  g.pack = (g.interleave && g.compact && !g.v32 && h->o.batch_pack && w0.tpb_rows == 1 &&
            w0.tpb_cols == 1 && !w0.direct && !w0.mask_x && !w0.mask_y)
               ? PDHG_PACK
               : 0;
  if (g.pack) {
    const int npk = (na + PDHG_PACK - 1) / PDHG_PACK;
    const int64_t tr = (w0.m + PDHG_TILE - 1) / PDHG_TILE, tc = (w0.n + PDHG_TILE - 1) / PDHG_TILE;
    g.n_primal_pack = (int)(w0.n_long_cols * (int64_t)na + tc * npk);
    g.n_dual_pack = (int)(w0.n_long_rows * (int64_t)na + tr * npk);
  }
  return PDHG_OK;
}

int read_states(pdhg_handle *h, GroupDev &gd, int na, bool fp32) {
  if (fp32)
    launch_gather_states<float>(gd.d32, na, gd.dstates, h->hs);
  else
    launch_gather_states<double>(gd.d64, na, gd.dstates, h->hs);
  HK();
  HC(hipMemcpyAsync(gd.hstates, gd.dstates, sizeof(CtlState) * na, hipMemcpyDeviceToHost, h->hs));
  HC(hipStreamSynchronize(h->hs));
  return PDHG_OK;
}

// Record one block (period attempts + evaluation) as a graph.  `version`
// identifies the group tables the graph was taken with.
template <typename T>
int capture(pdhg_handle *h, GraphSlot &gs, const Inst<T> *dI, const Groups &g, int period,
            double tol, int64_t max_iter, int version) {
  if (gs.exec && gs.period == period && gs.tol == tol && gs.max_iter == max_iter &&
      gs.version == version)
    return PDHG_OK;
  if (gs.exec) {
    HC(hipGraphExecDestroy(gs.exec));
    gs.exec = nullptr;
  }
  hipGraph_t graph;
  HC(hipStreamBeginCapture(h->hs, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < period; i++) launch_attempt<T>(dI, g, h->hs);
  launch_evaluate<T>(dI, g, tol, max_iter, h->hs);
  HC(hipStreamEndCapture(h->hs, &graph));
  HK();
  HC(hipGraphInstantiate(&gs.exec, graph, nullptr, nullptr, 0));
  HC(hipGraphDestroy(graph));
  gs.period = period;
  gs.tol = tol;
  gs.max_iter = max_iter;
  gs.version = version;
  return PDHG_OK;
}

// Drive a group of instances in blocks of `period` attempts plus an
// evaluation until every instance is done.  `active` lists the instances
// (indices into `all`, start points already initialised).  On return
// status[i] holds each one's status, 0 for an instance stopped because its
// relative KKT error had not dropped below 0.9 of its best value for
// `stall_evals` evaluations (0 disables that test), or, with drift_test,
// had drifted to 10x above a start point within 10x of the tolerance that
// it never improved on.  With reuse_graph the
// slot's graph is kept if it was taken with the same tables.
template <typename T>
int run_group(pdhg_handle *h, GroupDev &gd, const std::vector<Inst<T>> &all,
              std::vector<int> active, double tol, int64_t max_iter, double t_start,
              int stall_evals, GraphSlot &gs, bool reuse_graph, std::vector<int> &status,
              std::vector<CtlState> &final_state, bool drift_test = true) {
  const int P = h->o.eval_period;
  const bool fp32 = sizeof(T) == 4;
  std::vector<double> best(all.size(), INFINITY), first(all.size(), INFINITY);
  std::vector<int> since(all.size(), 0);
  long long evals = 0;
  Groups g{};
  int version = reuse_graph ? gs.version : gs.version + 1;
  RC(upload_group<T>(h, gd, all, active, g));
  const Inst<T> *dI = dev_insts<T>(gd);
  launch_evaluate<T>(dI, g, tol, max_iter, h->hs);
  HK();
  for (;;) {
    RC(read_states(h, gd, (int)active.size(), fp32));
    std::vector<int> still;
    bool timeout = now_s() - t_start > h->o.time_limit_s;
    int64_t kmin = INT64_MAX;
    for (size_t q = 0; q < active.size(); q++) {
      int i = active[q];
      const CtlState &s = gd.hstates[q];
      final_state[i] = s;
      if (h->o.verbose && active.size() == 1)
        fprintf(stderr,
                "pdhg k=%lld kkt=%.3e (p %.2e d %.2e g %.2e) obj=%.10g eta=%.3e omega=%.3e "
                "restarts=%lld\n",
                s.k, s.rel_kkt, s.rel_p, s.rel_d, s.rel_gap, s.pobj, s.eta, s.omega, s.restarts);
      if (s.done) {
        status[i] = s.status;
        continue;
      }
      if (timeout) {
        status[i] = PDHG_TIME_LIMIT;
        continue;
      }
      if (first[i] == INFINITY) first[i] = s.rel_kkt;
      if (s.rel_kkt < 0.9 * best[i]) {
        best[i] = s.rel_kkt;
        since[i] = 0;
      } else if (stall_evals > 0 &&
                 (++since[i] >= stall_evals ||
                  (drift_test && best[i] == first[i] && first[i] <= 10.0 * tol &&
                   s.rel_kkt > 10.0 * first[i]))) {
        // stalled, or drifting away from a start point that was near the target
        // and has not been improved on (the next phase starts from the best point)
        status[i] = 0;
        continue;
      }
      still.push_back(i);
      kmin = std::min<int64_t>(kmin, s.k);
    }
    if (h->o.verbose && active.size() > 1 && !still.empty() && ++evals % 64 == 0) {
      double worst = 0.0;
      for (int i : still) worst = std::max(worst, final_state[i].rel_kkt);
      fprintf(stderr, "pdhg batch: %d of %zu instances running, fewest attempts %lld, largest kkt %.3e\n",
              (int)still.size(), all.size(), (long long)kmin, worst);
    }
    if (still.empty()) break;
    if (still.size() != active.size()) {
      active.swap(still);
      RC(upload_group<T>(h, gd, all, active, g));
      version++;
    }
    int64_t nb = std::min<int64_t>(P, max_iter - kmin);
    if (nb < 1) nb = 1;
    if (nb == P && h->o.use_graph && gd.graphs) {
      RC(capture<T>(h, gs, dI, g, P, tol, max_iter, version));
      HC(hipGraphLaunch(gs.exec, h->hs));
    } else {
      for (int64_t i = 0; i < nb; i++) launch_attempt<T>(dI, g, h->hs);
      launch_evaluate<T>(dI, g, tol, max_iter, h->hs);
      HK();
    }
  }
  return PDHG_OK;
}

void fill_info(pdhg_info *info, const CtlState &s, int status, int64_t attempts_fp32,
               double setup_s, double solve_s, double obj_offset) {
  memset(info, 0, sizeof *info);
  info->status = status;
  info->which = s.which;
  info->attempts = s.k;
  info->attempts_fp32 = attempts_fp32;
  info->accepted = s.accepted;
  info->restarts = s.restarts;
  info->primal_obj = s.pobj + obj_offset;
  info->dual_obj = s.dobj + obj_offset;
  info->rel_primal = s.rel_p;
  info->rel_dual = s.rel_d;
  info->rel_gap = s.rel_gap;
  info->rel_kkt = s.rel_kkt;
  info->eta = s.eta;
  info->omega = s.omega;
  info->setup_s = setup_s;
  info->solve_s = solve_s;
  info->dual_bound = s.dual_bound + obj_offset;  // -INFINITY stays -INFINITY
}

// Solve a group of prepared instances (start points and result pointers set)
// with the precision of handle h's options.
int solve_group(pdhg_handle *h, GroupDev &gd, std::vector<Inst<double>> &i64,
                std::vector<Inst<float>> &i32, GraphSlot *gslots, bool reuse, double t0,
                std::vector<int> &status, std::vector<CtlState> &fin,
                std::vector<int64_t> &att32, std::vector<int> &final_fp32) {
  const int B = (int)i64.size();
  std::vector<int> all(B);
  for (int i = 0; i < B; i++) all[i] = i;
  status.assign(B, 0);
  fin.assign(B, CtlState{});
  att32.assign(B, 0);
  final_fp32.assign(B, 0);
  Groups g{};
  if (h->o.precision == PDHG_FP64) {
    RC(upload_group<double>(h, gd, i64, all, g));
    launch_init_point<double>(gd.d64, g, h->hs);
    HK();
    return run_group<double>(h, gd, i64, all, h->o.tol, h->o.max_iter, t0, 0, gslots[0], reuse,
                             status, fin);
  }
  // FP32 phase: FP32 matrix, iterates and SpMVs; FP64 evaluation and control
  double tol32 = h->o.polish_tol > h->o.tol ? h->o.polish_tol : h->o.tol;
  RC(upload_group<float>(h, gd, i32, all, g));
  launch_init_point<float>(gd.d32, g, h->hs);
  HK();
  RC(run_group<float>(h, gd, i32, all, tol32, h->o.max_iter, t0, h->o.fp32_stall_evals, gslots[1], reuse, status,
                      fin));
  std::vector<int> polish;
  for (int i = 0; i < B; i++) {
    att32[i] = fin[i].k;
    final_fp32[i] = 1;
    // stalled, reached polish_tol, or NaN / Inf in the FP32 iterates (an
    // overflow, e.g. on an unbounded LP): the FP64 phase goes on from the
    // best point
    if (status[i] == 0 || status[i] == PDHG_NUMERICAL ||
        (status[i] == PDHG_OPTIMAL && tol32 > h->o.tol))
      polish.push_back(i);
  }
  if (polish.empty()) return PDHG_OK;
  // FP64 refinement from the FP32 iterates (both tables describe the same
  // instances); optionally with the primal weight held where the FP32 phase
  // left it
  if (!h->o.polish_pw_update)
    for (int i : polish) i64[i].e.pw_theta = 0.0;
  // the FP64 phase's attempt kernels on the FP32 matrix values (its
  // evaluation keeps the FP64 matrix): their rounding (2^-24 relative per
  // entry) moves the fixed point by about 1e-7 relative, so only for
  // tolerances of 1e-6 and above, and an instance whose relative KKT error
  // stalls there (twice the FP32 phase's window: near the tolerance the
  // FP64 phase improves slowly but steadily) goes on with the FP64 values
  const bool v32 = h->o.polish_fp32_matrix && h->o.tol >= 1e-6;
  if (v32)
    for (int i : polish) i64[i].w.use_v32 = 1;
  RC(upload_group<float>(h, gd, i32, polish, g));
  Groups g64{};
  RC(upload_group<double>(h, gd, i64, polish, g64));
  launch_switch_to_fp64(gd.d32, gd.d64, g64, h->hs);
  HK();
  std::vector<int> st2(B, 0);
  std::vector<CtlState> fin2(B);
  RC(run_group<double>(h, gd, i64, polish, h->o.tol, h->o.max_iter, t0,
                       v32 ? 2 * h->o.fp32_stall_evals : 0, gslots[0], reuse && B == 1 && !v32, st2,
                       fin2, false));
  std::vector<int> again;
  for (int i : polish) {
    status[i] = st2[i];
    fin[i] = fin2[i];
    final_fp32[i] = 0;
    if (v32 && st2[i] == 0) again.push_back(i);
  }
  if (again.empty()) return PDHG_OK;
  for (int i : again) i64[i].w.use_v32 = 0;
  std::vector<int> st3(B, 0);
  std::vector<CtlState> fin3(B);
  RC(run_group<double>(h, gd, i64, again, h->o.tol, h->o.max_iter, t0, 0, gslots[0], false, st3,
                       fin3));
  for (int i : again) {
    status[i] = st3[i];
    fin[i] = fin3[i];
  }
  return PDHG_OK;
}

// Unscale every instance's result from the precision its solve ended in.
// The safe dual bound of each instance's reported point, computed once after
// the solve in the precision the instance finished in, into fin[].
int bound_group(pdhg_handle *h, GroupDev &gd, std::vector<Inst<double>> &i64,
                std::vector<Inst<float>> &i32, const std::vector<int> &final_fp32,
                std::vector<CtlState> &fin) {
  std::vector<int> a64, a32;
  for (int i = 0; i < (int)i64.size(); i++) (final_fp32[i] ? a32 : a64).push_back(i);
  Groups g{};
  for (int pass = 0; pass < 2; pass++) {
    const std::vector<int> &act = pass ? a32 : a64;
    if (act.empty()) continue;
    if (pass) {
      RC(upload_group<float>(h, gd, i32, act, g));
      launch_bound<float>(gd.d32, g, h->hs);
    } else {
      RC(upload_group<double>(h, gd, i64, act, g));
      launch_bound<double>(gd.d64, g, h->hs);
    }
    HK();
    RC(read_states(h, gd, (int)act.size(), pass == 1));
    for (size_t k = 0; k < act.size(); k++) fin[act[k]].dual_bound = gd.hstates[k].dual_bound;
  }
  return PDHG_OK;
}

int unscale_group(pdhg_handle *h, GroupDev &gd, std::vector<Inst<double>> &i64,
                  std::vector<Inst<float>> &i32, const std::vector<int> &final_fp32) {
  std::vector<int> a64, a32;
  for (int i = 0; i < (int)i64.size(); i++) (final_fp32[i] ? a32 : a64).push_back(i);
  Groups g{};
  if (!a64.empty()) {
    RC(upload_group<double>(h, gd, i64, a64, g));
    launch_unscale<double>(gd.d64, g, h->hs);
    HK();
  }
  if (!a32.empty()) {
    RC(upload_group<float>(h, gd, i32, a32, g));
    launch_unscale<float>(gd.d32, g, h->hs);
    HK();
  }
  return PDHG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// SpMV partition autotuner

// Average time of one attempt (both SpMV-fused kernels and the step control)
// under the handle's current partition, from its own start point.
template <typename T>
int time_attempts(pdhg_handle *h, int warm, int reps, double *ms) {
  InstData d = base_data(h);
  std::vector<Inst<T>> one{make_inst<T>(h, d, h->it)};
  std::vector<int> act{0};
  Groups g{};
  RC(upload_group<T>(h, h->grp, one, act, g));
  const Inst<T> *dI = dev_insts<T>(h->grp);
  launch_init_point<T>(dI, g, h->hs);
  for (int i = 0; i < warm; i++) launch_attempt<T>(dI, g, h->hs);
  HK();
  hipEvent_t e0, e1;
  HC(hipEventCreate(&e0));
  HC(hipEventCreate(&e1));
  HC(hipEventRecord(e0, h->hs));
  for (int i = 0; i < reps; i++) launch_attempt<T>(dI, g, h->hs);
  HC(hipEventRecord(e1, h->hs));
  HK();
  HC(hipEventSynchronize(e1));
  float t = 0.f;
  HC(hipEventElapsedTime(&t, e0, e1));
  HC(hipEventDestroy(e0));
  HC(hipEventDestroy(e1));
  *ms = t / reps;
  return PDHG_OK;
}

struct Partition {
  int tpb, direct, long_seg;
};

// Choices already made in this process, by matrix signature.
std::mutex g_tune_mu;
std::map<std::tuple<int64_t, int64_t, int64_t, int, uint64_t>, Partition> g_tune_cache;

uint64_t pointer_checksum(const std::vector<int32_t> &p) {
  uint64_t hsh = 1469598103934665603ull;
  size_t step = std::max<size_t>(1, p.size() / 4096);
  for (size_t i = 0; i < p.size(); i += step) hsh = (hsh ^ (uint64_t)(uint32_t)p[i]) * 1099511628211ull;
  return hsh ^ (uint64_t)(uint32_t)p.back();
}

// Time every candidate partition for a few attempts and keep the fastest.
int autotune(pdhg_handle *h) {
  auto key = std::make_tuple(h->m, h->n, h->nnz, h->o.precision,
                             pointer_checksum(h->hrp) ^ (pointer_checksum(h->hcp) << 1));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end())
      return apply_partition(h, it->second.tpb, it->second.direct, it->second.long_seg);
  }
  const int tpbs[] = {1, 2, 4};
  const int directs[] = {0, 1};
  const int segs[] = {32, 64, 256};
  Partition best{1, 0, PDHG_LONG_SEG};
  double best_ms = INFINITY;
  for (int tpb : tpbs)
    for (int dr : directs)
      for (int ls : segs) {
        RC(apply_partition(h, tpb, dr, ls));
        double ms = 0.0;
        if (h->o.precision == PDHG_MIXED)
          RC(time_attempts<float>(h, 3, 20, &ms));
        else
          RC(time_attempts<double>(h, 3, 20, &ms));
        if (ms < best_ms) {
          best_ms = ms;
          best = Partition{tpb, dr, ls};
        }
      }
  RC(apply_partition(h, best.tpb, best.direct, best.long_seg));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best;
  return PDHG_OK;
}

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
  o->tiles_per_block = 0;
  o->autotune = 0;
  o->spmv_direct = 0;
  o->long_seg = 0;
  o->reorder = 1;
  o->compact_index = 1;
  o->infeas_every = 4;
  o->polish_pw_update = 1;
  o->fp32_stall_evals = 300;
  o->dinf_tol = 1e-8;
  o->batch_pack = 0;
  o->stream_nt = -1;
  o->polish_fp32_matrix = 1;
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
  h->obj_offset = lp->obj_offset;
  h->user = (hipStream_t)stream;
  layout(h, (void *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255));
  auto setup_body = [&]() -> int {
    HC(hipStreamCreateWithFlags(&h->hs, hipStreamNonBlocking));
    HC(hipEventCreateWithFlags(&h->ev, hipEventDisableTiming));
    HC(hipHostMalloc((void **)&h->grp.hstates, sizeof(CtlState), hipHostMallocDefault));
    RC(enter(h));
    int64_t m = h->m, n = h->n, nnz = h->nnz;
    hipMemcpyKind kd = h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
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
    RC(setup_implied_bounds(h, lp));
    launch_var_kind(h->l0, h->u0, n, h->vk, h->hs);
    launch_transpose(h->rp, h->ci, h->v, m, n, nnz, h->cp, h->ri, h->vt, h->tmp_next, h->scan_tmp,
                     h->hs);
    HK();
    // scaling: row factors in YA (m), column factors in XA (n)
    launch_fill(h->Dr, 1.0, m, h->hs);
    launch_fill(h->Dc, 1.0, n, h->hs);
    int passes = h->o.scaling_iters + (h->o.pock_chambolle ? 1 : 0);
    for (int it = 0; it < passes; it++)
      launch_scale_pass(h->rp, h->ci, h->v, h->cp, h->ri, h->vt, m, n,
                        it == h->o.scaling_iters ? 1 : 0, h->it.YA, h->it.XA, h->Dr, h->Dc, h->hs);
    launch_scale_vectors(h->b0, h->c0, h->l0, h->u0, h->Dr, h->Dc, m, n, h->b, h->c, h->l, h->u,
                         h->hs);
    HK();
    if (h->o.reorder) RC(reorder_problem(h));
    RC(build_compact(h));
    set_stream_policy(h);
    RC(upload_implied_bounds(h));
    // long rows and columns (handled by a workgroup each in the iteration)
    h->hrp.resize(m + 1);
    h->hcp.resize(n + 1);
    HC(hipMemcpyAsync(h->hrp.data(), h->rp, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(h->hcp.data(), h->cp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, h->hs));
    HC(hipStreamSynchronize(h->hs));
    h->direct = h->o.spmv_direct;
    h->long_seg = h->o.long_seg > 0 ? h->o.long_seg : PDHG_LONG_SEG;
    RC(build_long_lists(h));
    launch_init_ctl(h->v, nnz, h->b, h->c, h->b0, h->c0, m, n, h->scratch, h->nscratch, h->it.st,
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
    if (h->o.autotune) RC(autotune(h));
    return leave(h);
  };
  rc = setup_body();
  if (rc) {
    pdhg_destroy(h);
    return rc;
  }
  h->setup_s = now_s() - t0;
  *out = h;
  return PDHG_OK;
}

}  // extern "C"

namespace {

// ||A^||_2 by power iteration on A'A from the all-ones direction (the same
// iteration as the reference definition of the unrolled step size).
int power_norm(pdhg_handle *h, int iters, double *est) {
  int64_t m = h->m, n = h->n;
  double *z = h->it.XA, *w = h->it.YA, *q = h->it.ATYA;
  launch_fill(z, 1.0 / sqrt((double)n), n, h->hs);
  HK();
  *est = 0.0;
  for (int it = 0; it < iters; it++) {
    launch_spmv(h->rp, h->ci, h->v, m, z, w, h->hs);
    launch_spmv(h->cp, h->ri, h->vt, n, w, q, h->hs);
    double *dn = launch_sumsq(q, n, h->scratch, h->nscratch, h->hs);
    HK();
    double qn2 = 0.0;
    HC(hipMemcpyAsync(&qn2, dn, sizeof(double), hipMemcpyDeviceToHost, h->hs));
    HC(hipStreamSynchronize(h->hs));
    double qn = sqrt(qn2);
    *est = sqrt(qn);
    if (qn == 0.0) break;
    launch_axpby(z, q, 1.0 / qn, 0.0, n, h->hs);
    HK();
  }
  return PDHG_OK;
}

template <typename F>
int write_state_field(pdhg_handle *h, size_t offset, const F &value) {
  HC(hipMemcpyAsync((char *)h->it.st + offset, &value, sizeof(F), hipMemcpyHostToDevice, h->hs));
  HC(hipStreamSynchronize(h->hs));
  return PDHG_OK;
}

// The instance of the unrolled mode: fixed steps, no restarts, no average.
Inst<double> unrolled_inst(pdhg_handle *h) {
  Inst<double> I = make_inst<double>(h, base_data(h), h->it);
  I.w.adaptive = 0;
  I.e.restart = 0;
  I.e.use_average = 0;
  return I;
}

int solve_unrolled(pdhg_handle *h, const double *dx0, const double *dy0, double *xo, double *yo,
                   pdhg_info *info, double t0) {
  const int64_t K = h->ur_K, C = h->ur_C, m = h->m, n = h->n;
  double eta = h->o.fixed_eta;
  if (!(eta > 0.0)) {
    double nrm = 0.0;
    RC(power_norm(h, 50, &nrm));
    eta = nrm > 0.0 ? 0.9 / nrm : 1.0;
  }
  RC(write_state_field(h, offsetof(CtlState, eta0), eta));
  std::vector<Inst<double>> one{unrolled_inst(h)};
  one[0].x0 = dx0;
  one[0].y0 = dy0;
  one[0].xout = xo;
  one[0].yout = yo;
  std::vector<int> act{0};
  Groups g{};
  RC(upload_group<double>(h, h->grp, one, act, g));
  const Inst<double> *dI = h->grp.d64;
  launch_init_point<double>(dI, g, h->hs);
  HK();
  const int64_t S = (K + C - 1) / C;
  hipGraphExec_t exec = nullptr;
  for (int64_t s = 0; s < S; s++) {
    double *ck = h->ckpt + s * (n + 2 * m);
    launch_checkpoint<double>(dI, g, ck, ck + n, ck + n + m, 0, h->hs);
    int64_t steps = std::min<int64_t>(C, K - s * C);
    if (steps == C && h->o.use_graph) {
      if (!exec) {
        hipGraph_t graph;
        HC(hipStreamBeginCapture(h->hs, hipStreamCaptureModeThreadLocal));
        for (int64_t i = 0; i < C; i++) launch_attempt<double>(dI, g, h->hs);
        HC(hipStreamEndCapture(h->hs, &graph));
        HK();
        HC(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        HC(hipGraphDestroy(graph));
      }
      HC(hipGraphLaunch(exec, h->hs));
    } else {
      for (int64_t i = 0; i < steps; i++) launch_attempt<double>(dI, g, h->hs);
      HK();
    }
  }
  if (exec) HC(hipGraphExecDestroy(exec));
  // x_K for the adjoint's seed; the y and Ax copies land in scratch
  launch_checkpoint<double>(dI, g, h->XK, h->YB, h->BB, 0, h->hs);
  launch_evaluate<double>(dI, g, 0.0, K, h->hs);
  launch_unscale<double>(dI, g, h->hs);
  HK();
  RC(read_states(h, h->grp, 1, false));
  const CtlState &st = h->grp.hstates[0];
  h->ur_eta = st.eta;
  h->ur_omega = st.omega;
  h->ur_valid = true;
  fill_info(info, st, PDHG_ITER_LIMIT, 0, h->setup_s, now_s() - t0, h->obj_offset);
  return PDHG_OK;
}

int backward_unrolled(pdhg_handle *h, double gv, double *grad_b, double *grad_c) {
  const int64_t K = h->ur_K, C = h->ur_C, m = h->m, n = h->n;
  const int64_t wx = (n + 63) / 64, wy = (m + 63) / 64, S = (K + C - 1) / C;
  // seed: dV/dx_K = c^, dV/dc^ (direct) = x_K
  launch_copy_f64(h->XB, h->c, n, h->hs);
  launch_fill(h->YB, 0.0, m, h->hs);
  launch_fill(h->BB, 0.0, m, h->hs);
  launch_copy_f64(h->CB, h->XK, n, h->hs);
  HK();
  AdjView a{};
  a.m = m;
  a.n = n;
  a.rp = h->rp;
  a.ci = h->ci;
  a.cp = h->cp;
  a.ri = h->ri;
  a.v = h->v;
  a.vt = h->vt;
  a.long_rows = h->long_rows;
  a.long_cols = h->long_cols;
  a.n_long_rows = h->n_long_rows;
  a.n_long_cols = h->n_long_cols;
  a.nblk_rows = h->nblk_rows;
  a.nblk_cols = h->nblk_cols;
  a.long_seg = h->long_seg;
  a.XB = h->XB;
  a.YB = h->YB;
  a.H = h->H;
  a.BB = h->BB;
  a.CB = h->CB;
  a.tau = h->ur_eta / h->ur_omega;
  a.sigma = h->ur_eta * h->ur_omega;
  std::vector<int> act{0};
  for (int64_t s = S - 1; s >= 0; s--) {
    int64_t steps = std::min<int64_t>(C, K - s * C);
    // recompute the segment from its checkpoint, recording the masks
    launch_fill_u64(h->mask_x, steps * wx, h->hs);
    launch_fill_u64(h->mask_y, steps * wy, h->hs);
    std::vector<Inst<double>> one{unrolled_inst(h)};
    one[0].w.mask_x = h->mask_x;
    one[0].w.mask_y = h->mask_y;
    one[0].w.mask_k0 = s * C;
    Groups g{};
    RC(upload_group<double>(h, h->grp, one, act, g));
    const Inst<double> *dI = h->grp.d64;
    double *ck = h->ckpt + s * (n + 2 * m);
    launch_checkpoint<double>(dI, g, ck, ck + n, ck + n + m, 1, h->hs);
    HK();
    RC(write_state_field(h, offsetof(CtlState, k), (long long)(s * C)));
    for (int64_t i = 0; i < steps; i++) launch_attempt<double>(dI, g, h->hs);
    HK();
    // reverse sweep over the segment
    for (int64_t k = steps - 1; k >= 0; k--) {
      a.mask_x = h->mask_x + k * wx;
      a.mask_y = h->mask_y + k * wy;
      launch_adjoint_step(a, h->hs);
    }
    HK();
  }
  // back to the original space: dV/db = Dr b-bar, dV/dc = Dc c-bar (internal
  // order in AXA / ATYA), then into the caller's order
  double *tb = h->it.AXA, *tc = h->it.ATYA;
  launch_scale_vectors(h->BB, h->CB, h->CB, h->CB, h->Dr, h->Dc, m, n, tb, tc, h->H, h->XB,
                       h->hs);
  launch_axpby(tb, tb, gv, 0.0, m, h->hs);
  launch_axpby(tc, tc, gv, 0.0, n, h->hs);
  double *ob = h->on_device ? grad_b : h->it.YA;
  double *oc = h->on_device ? grad_c : h->it.XA;
  RC(to_caller(h, ob, tb, h->rperm, m));
  RC(to_caller(h, oc, tc, h->cperm, n));
  HK();
  if (!h->on_device) {
    HC(hipMemcpyAsync(grad_b, ob, sizeof(double) * m, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(grad_c, oc, sizeof(double) * n, hipMemcpyDeviceToHost, h->hs));
  }
  HC(hipStreamSynchronize(h->hs));
  return PDHG_OK;
}

}  // namespace

extern "C" {

int pdhg_solve(pdhg_handle *h, const double *x0, const double *y0, double *x, double *y,
               pdhg_info *info) {
  if (!h || !x || !y || !info) return fail(PDHG_ERR_ARG, "null argument");
  RC(enter(h));
  double t0 = now_s();
  // host start vectors are staged in the average buffers (free until the first evaluation)
  const double *dx0 = x0, *dy0 = y0;
  if (!h->on_device) {
    if (x0) {
      HC(hipMemcpyAsync(h->it.XA, x0, sizeof(double) * h->n, hipMemcpyHostToDevice, h->hs));
      dx0 = h->it.XA;
    }
    if (y0) {
      HC(hipMemcpyAsync(h->it.YA, y0, sizeof(double) * h->m, hipMemcpyHostToDevice, h->hs));
      dy0 = h->it.YA;
    }
  }
  double *xo = h->on_device ? x : h->it.ATYA;
  double *yo = h->on_device ? y : h->it.AXA;
  if (h->ur_K > 0) {
    RC(solve_unrolled(h, dx0, dy0, xo, yo, info, t0));
    if (!h->on_device) {
      HC(hipMemcpyAsync(x, xo, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->hs));
      HC(hipMemcpyAsync(y, yo, sizeof(double) * h->m, hipMemcpyDeviceToHost, h->hs));
    }
    HC(hipStreamSynchronize(h->hs));
    h->state_ready = true;
    info->solve_s = now_s() - t0;
    return leave(h);
  }
  InstData d = base_data(h);
  std::vector<Inst<double>> i64{make_inst<double>(h, d, h->it)};
  std::vector<Inst<float>> i32{make_inst<float>(h, d, h->it)};
  i64[0].x0 = i32[0].x0 = dx0;
  i64[0].y0 = i32[0].y0 = dy0;
  i64[0].xout = i32[0].xout = xo;
  i64[0].yout = i32[0].yout = yo;
  std::vector<int> status, final_fp32;
  std::vector<CtlState> fin;
  std::vector<int64_t> att32;
  RC(solve_group(h, h->grp, i64, i32, h->graph, true, t0, status, fin, att32, final_fp32));
  RC(bound_group(h, h->grp, i64, i32, final_fp32, fin));
  RC(unscale_group(h, h->grp, i64, i32, final_fp32));
  if (!h->on_device) {
    HC(hipMemcpyAsync(x, xo, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(y, yo, sizeof(double) * h->m, hipMemcpyDeviceToHost, h->hs));
  }
  HC(hipStreamSynchronize(h->hs));
  h->state_ready = true;
  fill_info(info, fin[0], status[0], h->o.precision == PDHG_MIXED ? att32[0] : 0, h->setup_s,
            now_s() - t0, h->obj_offset);
  return leave(h);
}

}  // extern "C"

namespace {

// One FP64 solve of a variant of the handle's problem on its own buffers:
// data d (scaled), norms of b0 / c0 (original space) for the relative
// measures, start (x0, y0) and results (xo, yo) in the caller's order and
// original space, termination on e.term.  The polish steps are adaptive
// whatever opts.step_mode, test no infeasibility and keep no dual bound.
int polish_solve(pdhg_handle *h, const InstData &d, const double *b0, const double *c0,
                 const double *x0, const double *y0, int term, double tol, int64_t max_iter,
                 double omega0, double t0, double *xo, double *yo, CtlState &fin, int &status) {
  Inst<double> I = make_inst<double>(h, d, h->it);
  I.w.adaptive = 1;
  I.e.term = term;
  I.e.ilo = I.e.ihi = nullptr;
  I.e.rylo = I.e.ryhi = nullptr;
  I.fyk = nullptr;
  I.e.infeas_period = 0;
  I.e.dinf_tol = 0.0;
  I.x0 = x0;
  I.y0 = y0;
  I.xout = xo;
  I.yout = yo;
  launch_init_ctl(h->v, h->nnz, d.b, d.c, b0, c0, h->m, h->n, h->scratch, h->nscratch, I.st, 0,
                  0.0, omega0, h->hs);
  HK();
  std::vector<Inst<double>> one{I};
  std::vector<int> act{0}, st(1, 0);
  std::vector<CtlState> f(1);
  Groups g{};
  RC(upload_group<double>(h, h->grp, one, act, g));
  launch_init_point<double>(h->grp.d64, g, h->hs);
  HK();
  RC(run_group<double>(h, h->grp, one, act, tol, max_iter, t0, 0, h->graph[0], false, st, f));
  launch_unscale<double>(h->grp.d64, g, h->hs);
  HK();
  fin = f[0];
  status = st[0];
  return PDHG_OK;
}

}  // namespace

extern "C" int pdhg_polish(pdhg_handle *h, const double *x, const double *y, double tol,
                           int64_t max_iter, double omega, double *x_out, double *y_out,
                           pdhg_info *info) {
  if (!h || !x || !y || !x_out || !y_out || !info) return fail(PDHG_ERR_ARG, "null argument");
  if (!(tol > 0.0)) return fail(PDHG_ERR_ARG, "tol must be > 0");
  if (!(omega >= 0.0) || !std::isfinite(omega)) return fail(PDHG_ERR_ARG, "omega must be >= 0");
  if (h->ur_K > 0) return fail(PDHG_ERR_STATE, "no feasibility polishing in the unrolled mode");
  RC(enter(h));
  const double t0 = now_s();
  const int64_t m = h->m, n = h->n;
  if (max_iter <= 0) max_iter = h->o.max_iter;
  // the point, staged in device memory (caller's order, original space)
  const double *dx = x, *dy = y;
  if (!h->on_device) {
    HC(hipMemcpyAsync(h->pol_xd, x, sizeof(double) * n, hipMemcpyHostToDevice, h->hs));
    HC(hipMemcpyAsync(h->pol_yd, y, sizeof(double) * m, hipMemcpyHostToDevice, h->hs));
    dx = h->pol_xd;
    dy = h->pol_yd;
  }
  launch_fill(h->pol_zero, 0.0, std::max(m, n), h->hs);
  launch_zero_finite(h->l, h->pol_lz, n, h->hs);
  launch_zero_finite(h->u, h->pol_uz, n, h->hs);
  HK();
  const double om = omega > 0.0 ? omega : 0.0;
  // 1. primal feasibility: c = 0, from (x, 0), until the relative primal
  //    residual is at most tol; its x is kept (in pol_x)
  InstData dp = base_data(h);
  dp.c = h->pol_zero;
  CtlState f1{}, f2{}, f3{};
  int s1 = 0, s2 = 0, s3 = 0;
  RC(polish_solve(h, dp, h->b0, h->pol_zero, dx, nullptr, 1, tol, max_iter, om, t0, h->pol_x,
                  h->pol_y, f1, s1));
  // 2. dual feasibility: b = 0 and the finite bounds 0 (the same dual cone of
  //    reduced costs), from (0, y), until the relative dual residual is at
  //    most tol; its y is kept (in pol_y)
  InstData dd = base_data(h);
  dd.b = h->pol_zero;
  dd.l = h->pol_lz;
  dd.u = h->pol_uz;
  RC(polish_solve(h, dd, h->pol_zero, h->c0, nullptr, dy, 2, tol, max_iter, om, t0, h->pol_xd,
                  h->pol_y, f2, s2));
  // 3. the combined point on the original problem: one evaluation (no
  //    attempt), then its dual bound and unscaled result
  double *xo = h->on_device ? x_out : h->it.ATYA;
  double *yo = h->on_device ? y_out : h->it.AXA;
  {
    InstData d = base_data(h);
    Inst<double> I = make_inst<double>(h, d, h->it);
    I.x0 = h->pol_x;
    I.y0 = h->pol_y;
    I.xout = xo;
    I.yout = yo;
    launch_init_ctl(h->v, h->nnz, d.b, d.c, h->b0, h->c0, m, n, h->scratch, h->nscratch, I.st, 0,
                    0.0, om, h->hs);
    HK();
    std::vector<Inst<double>> i64{I};
    std::vector<Inst<float>> i32;
    std::vector<int> act{0}, st(1, 0), final_fp32{0};
    std::vector<CtlState> fin(1);
    Groups g{};
    RC(upload_group<double>(h, h->grp, i64, act, g));
    launch_init_point<double>(h->grp.d64, g, h->hs);
    HK();
    RC(run_group<double>(h, h->grp, i64, act, h->o.tol, 0, t0, 0, h->graph[0], false, st, fin));
    RC(bound_group(h, h->grp, i64, i32, final_fp32, fin));
    RC(unscale_group(h, h->grp, i64, i32, final_fp32));
    f3 = fin[0];
    s3 = st[0];
  }
  if (!h->on_device) {
    HC(hipMemcpyAsync(x_out, xo, sizeof(double) * n, hipMemcpyDeviceToHost, h->hs));
    HC(hipMemcpyAsync(y_out, yo, sizeof(double) * m, hipMemcpyDeviceToHost, h->hs));
  }
  HC(hipStreamSynchronize(h->hs));
  (void)s3;
  fill_info(info, f3, f3.rel_kkt <= h->o.tol ? PDHG_OPTIMAL : PDHG_ITER_LIMIT, 0, h->setup_s,
            now_s() - t0, h->obj_offset);
  info->attempts = f1.k + f2.k;
  info->accepted = f1.accepted + f2.accepted;
  info->restarts = f1.restarts + f2.restarts;
  info->eta = f1.eta;
  info->omega = f1.omega;
  // either step stopped short of tol (attempt limit or no progress): the
  // point's residuals say how far it got
  (void)s1;
  (void)s2;
  return leave(h);
}

// ---------------------------------------------------------------------------
// batched solve

namespace {

struct BatchPlan {
  std::vector<IterBufs> it;
  // per-instance problem vectors that differ from the base (nullptr: shared)
  std::vector<double *> b0, c0, l0, u0, b, c, l, u;
  std::vector<float *> bf, cf, lf, uf;
  std::vector<uint8_t *> vk;
  std::vector<int32_t *> fix_idx;
  std::vector<double *> fix_val;
  std::vector<double *> xo, yo;  // staging for host results
  std::vector<double *> x0, y0;  // staging for host warm starts
  GroupDev gd;
};

size_t batch_layout(pdhg_handle *const *hs, const pdhg_instance *inst, int batch, void *base,
                    BatchPlan &P) {
  Carver cv(base);
  P.it.assign(batch, IterBufs{});
  std::vector<double *> nd(batch, nullptr);
  std::vector<float *> nf(batch, nullptr);
  P.b0 = P.c0 = P.l0 = P.u0 = P.b = P.c = P.l = P.u = nd;
  P.bf = P.cf = P.lf = P.uf = nf;
  P.vk.assign(batch, nullptr);
  P.fix_idx.assign(batch, nullptr);
  P.fix_val.assign(batch, nullptr);
  P.xo = P.yo = P.x0 = P.y0 = nd;
  for (int k = 0; k < batch; k++) {
    const pdhg_handle *h = hs[inst[k].base];
    int64_t m = h->m, n = h->n;
    bool mixed = h->o.precision == PDHG_MIXED;
    carve_iter(cv, P.it[k], m, n, std::max(h->grid_rows[0], h->grid_rows[1]),
               std::max(h->grid_cols[0], h->grid_cols[1]), mixed);
    if (inst[k].b) {
      P.b0[k] = cv.take<double>(m);
      P.b[k] = cv.take<double>(m);
      if (mixed) P.bf[k] = cv.take<float>(m);
    }
    if (inst[k].c) {
      P.c0[k] = cv.take<double>(n);
      P.c[k] = cv.take<double>(n);
      if (mixed) P.cf[k] = cv.take<float>(n);
    }
    if (inst[k].l || inst[k].u || inst[k].n_fix > 0) {
      P.l0[k] = cv.take<double>(n);
      P.u0[k] = cv.take<double>(n);
      P.l[k] = cv.take<double>(n);
      P.u[k] = cv.take<double>(n);
      P.vk[k] = cv.take<uint8_t>(n);
      if (mixed) {
        P.lf[k] = cv.take<float>(n);
        P.uf[k] = cv.take<float>(n);
      }
    }
    if (inst[k].n_fix > 0) {
      P.fix_idx[k] = cv.take<int32_t>(inst[k].n_fix);
      P.fix_val[k] = cv.take<double>(inst[k].n_fix);
    }
    if (!h->on_device) {
      P.xo[k] = cv.take<double>(n);
      P.yo[k] = cv.take<double>(m);
      if (inst[k].x0) P.x0[k] = cv.take<double>(n);
      if (inst[k].y0) P.y0[k] = cv.take<double>(m);
    }
  }
  carve_group(cv, P.gd, batch);
  return cv.off + 256;
}

int check_batch(pdhg_handle *const *handles, int n_handles, const pdhg_instance *inst, int batch) {
  if (!handles || n_handles < 1 || !inst || batch < 1)
    return fail(PDHG_ERR_ARG, "empty batch or null arguments");
  for (int i = 0; i < n_handles; i++) {
    if (!handles[i]) return fail(PDHG_ERR_ARG, "null handle %d", i);
    if (handles[i]->o.precision != handles[0]->o.precision)
      return fail(PDHG_ERR_ARG, "all handles of a batch must use the same precision");
  }
  for (int k = 0; k < batch; k++) {
    if (inst[k].base < 0 || inst[k].base >= n_handles)
      return fail(PDHG_ERR_ARG, "instance %d: base %d out of range", k, inst[k].base);
    if (inst[k].n_fix < 0 || (inst[k].n_fix > 0 && (!inst[k].fix_idx || !inst[k].fix_val)))
      return fail(PDHG_ERR_ARG, "instance %d: bad fixings", k);
    if (!(inst[k].omega0 >= 0.0 && std::isfinite(inst[k].omega0)) ||
        !(inst[k].eta0 >= 0.0 && std::isfinite(inst[k].eta0)))
      return fail(PDHG_ERR_ARG, "instance %d: omega0 and eta0 must be finite and >= 0", k);
    if (inst[k].hold_omega < 0) return fail(PDHG_ERR_ARG, "instance %d: hold_omega < 0", k);
    const pdhg_handle *h = handles[inst[k].base];
    if (!h->on_device)
      for (int64_t q = 0; q < inst[k].n_fix; q++)
        if (inst[k].fix_idx[q] < 0 || inst[k].fix_idx[q] >= h->n || !isfinite(inst[k].fix_val[q]))
          return fail(PDHG_ERR_ARG, "instance %d: fixing %lld out of range or not finite", k,
                      (long long)q);
  }
  return PDHG_OK;
}

struct PinnedStates {
  CtlState *p = nullptr;
  ~PinnedStates() {
    if (p) (void)hipHostFree(p);
  }
};

}  // namespace

extern "C" {

int pdhg_batch_workspace_bytes(pdhg_handle *const *handles, int n_handles,
                               const pdhg_instance *inst, int batch, size_t *bytes) {
  int rc = check_batch(handles, n_handles, inst, batch);
  if (rc) return rc;
  if (!bytes) return fail(PDHG_ERR_ARG, "null argument");
  BatchPlan P;
  *bytes = batch_layout(handles, inst, batch, nullptr, P);
  return PDHG_OK;
}

}  // extern "C"

namespace {

// The batched solve on a workspace already checked to be large enough
// (ws: 256-byte aligned).  hstates: the host mirror of the batch's control
// states (batch entries; null: pinned memory allocated here).  graphs: false
// launches every block directly (no graph is captured or instantiated).
int solve_batch_on(pdhg_handle *const *handles, int n_handles, const pdhg_instance *inst,
                   int batch, void *ws, double *const *x, double *const *y, pdhg_info *infos,
                   CtlState *hstates, bool graphs) {
  int rc = PDHG_OK;
  BatchPlan P;
  batch_layout(handles, inst, batch, ws, P);
  P.gd.graphs = graphs;
  pdhg_handle *h = handles[0];  // the batch runs on this handle's stream
  for (int i = 0; i < n_handles; i++) RC(enter(handles[i]));
  for (int i = 1; i < n_handles; i++) {
    pdhg_handle *hi = handles[i];
    if (hipStreamSynchronize(hi->hs) != hipSuccess) return fail(PDHG_ERR_HIP, "stream sync failed");
  }
  double t0 = now_s();
  PinnedStates pin;
  if (hstates) {
    P.gd.hstates = hstates;
  } else {
    HC(hipHostMalloc((void **)&pin.p, sizeof(CtlState) * batch, hipHostMallocDefault));
    P.gd.hstates = pin.p;
  }
  std::vector<Inst<double>> i64(batch);
  std::vector<Inst<float>> i32(batch);
  const bool mixed = h->o.precision == PDHG_MIXED;
  for (int k = 0; k < batch; k++) {
    const pdhg_instance &q = inst[k];
    pdhg_handle *hb = handles[q.base];
    int64_t m = hb->m, n = hb->n;
    hipMemcpyKind kd = hb->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    IterBufs &ib = P.it[k];
    InstData d = base_data(hb);
    if (q.b) {  // b^ = Dr b
      RC(to_internal(h, P.b0[k], q.b, hb->on_device, hb->rperm, m, ib.YA));
      launch_scale_vectors(P.b0[k], nullptr, nullptr, nullptr, hb->Dr, hb->Dc, m, 0, P.b[k], nullptr,
                           nullptr, nullptr, h->hs);
      d.b = P.b[k];
      if (mixed) {
        launch_cast_f32(P.b[k], P.bf[k], m, h->hs);
        d.bf = P.bf[k];
      }
    }
    const double *l0 = hb->l0, *u0 = hb->u0;
    if (P.l0[k]) {  // bounds: overrides, then fixings l = u = value
      if (q.l)
        RC(to_internal(h, P.l0[k], q.l, hb->on_device, hb->cperm, n, ib.XA));
      else
        HC(hipMemcpyAsync(P.l0[k], hb->l0, sizeof(double) * n, hipMemcpyDeviceToDevice, h->hs));
      if (q.u)
        RC(to_internal(h, P.u0[k], q.u, hb->on_device, hb->cperm, n, ib.XA));
      else
        HC(hipMemcpyAsync(P.u0[k], hb->u0, sizeof(double) * n, hipMemcpyDeviceToDevice, h->hs));
      if (q.n_fix > 0) {  // caller's column indices, mapped through the ordering
        HC(hipMemcpyAsync(P.fix_idx[k], q.fix_idx, sizeof(int32_t) * q.n_fix, kd, h->hs));
        HC(hipMemcpyAsync(P.fix_val[k], q.fix_val, sizeof(double) * q.n_fix, kd, h->hs));
        launch_fix_bounds(P.l0[k], P.u0[k], P.fix_idx[k], P.fix_val[k], q.n_fix, hb->cinv, n,
                          h->hs);
      }
      launch_var_kind(P.l0[k], P.u0[k], n, P.vk[k], h->hs);
      l0 = P.l0[k];
      u0 = P.u0[k];
    }
    if (q.c) RC(to_internal(h, P.c0[k], q.c, hb->on_device, hb->cperm, n, ib.XA));
    if (q.c || P.l0[k]) {
      // c^ = Dc c, l^ = l / Dc, u^ = u / Dc; untouched outputs go to free buffers
      launch_scale_vectors(nullptr, q.c ? P.c0[k] : hb->c0, l0, u0, hb->Dr, hb->Dc, 0, n, nullptr,
                           q.c ? P.c[k] : ib.XA, P.l0[k] ? P.l[k] : ib.XL,
                           P.l0[k] ? P.u[k] : ib.ATY, h->hs);
      if (q.c) {
        d.c = P.c[k];
        if (mixed) {
          launch_cast_f32(P.c[k], P.cf[k], n, h->hs);
          d.cf = P.cf[k];
        }
      }
      if (P.l0[k]) {
        d.l = P.l[k];
        d.u = P.u[k];
        d.vk = P.vk[k];
        if (mixed) {
          launch_cast_f32(P.l[k], P.lf[k], n, h->hs);
          launch_cast_f32(P.u[k], P.uf[k], n, h->hs);
          d.lf = P.lf[k];
          d.uf = P.uf[k];
        }
      }
    }
    HK();
    // initial step size, primal weight and the norms of this instance's b and c
    const double eta0 = q.eta0 > 0.0 ? q.eta0 : (hb->o.step_mode == 1 ? hb->o.fixed_eta : 0.0);
    const double omega0 = q.omega0 > 0.0 ? q.omega0 : hb->o.fixed_omega;
    launch_init_ctl(hb->v, hb->nnz, d.b, d.c, q.b ? P.b0[k] : hb->b0, q.c ? P.c0[k] : hb->c0, m, n,
                    hb->scratch, hb->nscratch, ib.st, hb->o.step_mode, eta0, omega0, h->hs);
    HK();
    HC(hipStreamSynchronize(h->hs));  // the base's scratch is reused by the next instance
    i64[k] = make_inst<double>(hb, d, ib);
    i32[k] = make_inst<float>(hb, d, ib);
    if (q.b || q.l || q.u) {  // the base's implied bounds assume its b, l, u
      i64[k].e.ilo = i64[k].e.ihi = nullptr;
      i32[k].e.ilo = i32[k].e.ihi = nullptr;
    }
    // the Farkas intervals come from the base's box: a fixing can bound a
    // column whose missing bound made one (a penalty slack fixed to 0), and
    // the clamp would then zero the very duals a certificate needs, so such
    // instances test y as it is
    if (q.b || q.l || q.u || q.n_fix > 0) i64[k].fyk = i32[k].fyk = nullptr;
    i64[k].e.hold_k = i32[k].e.hold_k = q.hold_omega;  // weight held for these attempts
    if (q.b || q.c || q.l || q.u) {  // and its repair intervals those and its c
      i64[k].e.rylo = i64[k].e.ryhi = nullptr;
      i32[k].e.rylo = i32[k].e.ryhi = nullptr;
      i64[k].e.dinf_tol = i32[k].e.dinf_tol = hb->o.dinf_tol;  // and so does the ray-test skip
    }
    const double *wx = q.x0, *wy = q.y0;  // warm start, caller's order
    if (!hb->on_device) {
      if (q.x0) {
        HC(hipMemcpyAsync(P.x0[k], q.x0, sizeof(double) * n, hipMemcpyHostToDevice, h->hs));
        wx = P.x0[k];
      }
      if (q.y0) {
        HC(hipMemcpyAsync(P.y0[k], q.y0, sizeof(double) * m, hipMemcpyHostToDevice, h->hs));
        wy = P.y0[k];
      }
    }
    i64[k].x0 = i32[k].x0 = wx;
    i64[k].y0 = i32[k].y0 = wy;
    double *xo = hb->on_device ? x[k] : P.xo[k];
    double *yo = hb->on_device ? y[k] : P.yo[k];
    i64[k].xout = i32[k].xout = xo;
    i64[k].yout = i32[k].yout = yo;
  }
  std::vector<int> status, final_fp32;
  std::vector<CtlState> fin;
  std::vector<int64_t> att32;
  GraphSlot gs[2];
  rc = solve_group(h, P.gd, i64, i32, gs, false, t0, status, fin, att32, final_fp32);
  for (auto &g : gs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (rc) return rc;
  RC(bound_group(h, P.gd, i64, i32, final_fp32, fin));
  RC(unscale_group(h, P.gd, i64, i32, final_fp32));
  for (int k = 0; k < batch; k++) {
    pdhg_handle *hb = handles[inst[k].base];
    if (!hb->on_device) {
      HC(hipMemcpyAsync(x[k], P.xo[k], sizeof(double) * hb->n, hipMemcpyDeviceToHost, h->hs));
      HC(hipMemcpyAsync(y[k], P.yo[k], sizeof(double) * hb->m, hipMemcpyDeviceToHost, h->hs));
    }
  }
  HC(hipStreamSynchronize(h->hs));
  double dt = now_s() - t0;
  for (int k = 0; k < batch; k++)
    fill_info(&infos[k], fin[k], status[k], mixed ? att32[k] : 0, handles[inst[k].base]->setup_s,
              dt, handles[inst[k].base]->obj_offset);
  for (int i = 0; i < n_handles; i++) RC(leave(handles[i]));
  return PDHG_OK;
}

}  // namespace

extern "C" {

int pdhg_solve_batch(pdhg_handle *const *handles, int n_handles, const pdhg_instance *inst,
                     int batch, void *workspace, size_t ws_bytes, double *const *x,
                     double *const *y, pdhg_info *infos) {
  int rc = check_batch(handles, n_handles, inst, batch);
  if (rc) return rc;
  if (!x || !y || !infos) return fail(PDHG_ERR_ARG, "null output arrays");
  for (int k = 0; k < batch; k++)
    if (!x[k] || !y[k]) return fail(PDHG_ERR_ARG, "instance %d: null output", k);
  BatchPlan P;
  size_t need = batch_layout(handles, inst, batch, nullptr, P);
  if (!workspace || ws_bytes < need)
    return fail(PDHG_ERR_OOM, "batch workspace of %zu bytes, need %zu", ws_bytes, need);
  return solve_batch_on(handles, n_handles, inst, batch,
                        (void *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255), x, y, infos,
                        nullptr, true);
}

int pdhg_solve_batch_static(pdhg_handle *const *handles, int n_handles,
                            const pdhg_instance *inst, int batch, double *const *x,
                            double *const *y, pdhg_info *infos) {
  int rc = check_batch(handles, n_handles, inst, batch);
  if (rc) return rc;
  if (!x || !y || !infos) return fail(PDHG_ERR_ARG, "null output arrays");
  for (int k = 0; k < batch; k++)
    if (!x[k] || !y[k]) return fail(PDHG_ERR_ARG, "instance %d: null output", k);
  if (batch > PDHG_STATIC_MAX_BATCH)
    return fail(PDHG_ERR_OOM, "no-allocation batch of %d instances, at most %d", batch,
                PDHG_STATIC_MAX_BATCH);
  BatchPlan P;
  size_t need = batch_layout(handles, inst, batch, nullptr, P);
  if (need > PDHG_STATIC_SCRATCH_BYTES)
    return fail(PDHG_ERR_OOM, "no-allocation batch needs %zu bytes of scratch, at most %zu",
                need, (size_t)PDHG_STATIC_SCRATCH_BYTES);
  void *ptr = nullptr;
  RC(static_scratch(&ptr));
  std::lock_guard<std::mutex> lk(g_static_mu);  // one call at a time per process
  return solve_batch_on(handles, n_handles, inst, batch, ptr, x, y, infos, g_static_states,
                        false);
}

int pdhg_backward(pdhg_handle *h, double grad_value, double *grad_b, double *grad_c) {
  if (!h || !grad_b || !grad_c) return fail(PDHG_ERR_ARG, "null argument");
  if (!h->ur_valid)
    return fail(PDHG_ERR_STATE, "backward needs a preceding unrolled solve (opts.unroll_iters > 0)");
  RC(enter(h));
  RC(backward_unrolled(h, grad_value, grad_b, grad_c));
  return leave(h);
}

int pdhg_update(pdhg_handle *h, const double *b, const double *c) {
  if (!h) return fail(PDHG_ERR_ARG, "null handle");
  if (!h->on_device) {
    for (int64_t i = 0; b && i < h->m; i++)
      if (!isfinite(b[i])) return fail(PDHG_ERR_NONFINITE, "non-finite b[%lld]", (long long)i);
    for (int64_t j = 0; c && j < h->n; j++)
      if (!isfinite(c[j])) return fail(PDHG_ERR_NONFINITE, "non-finite c[%lld]", (long long)j);
  }
  RC(enter(h));
  if (b) {
    RC(to_internal(h, h->b0, b, h->on_device, h->rperm, h->m, h->it.YA));
    h->impl_valid = false;  // they were derived from the old right-hand side
    h->rep_valid = false;
    h->obj_bounded = false;
  }
  if (c) {
    RC(to_internal(h, h->c0, c, h->on_device, h->cperm, h->n, h->it.XA));
    h->rep_valid = false;  // the repair intervals come from the old costs
    h->obj_bounded = false;
  }
  launch_scale_vectors(h->b0, h->c0, h->l0, h->u0, h->Dr, h->Dc, h->m, h->n, h->b, h->c, h->l,
                       h->u, h->hs);
  launch_init_ctl(h->v, h->nnz, h->b, h->c, h->b0, h->c0, h->m, h->n, h->scratch, h->nscratch,
                  h->it.st, h->o.step_mode, h->o.step_mode == 1 ? h->o.fixed_eta : 0.0,
                  h->o.fixed_omega, h->hs);
  if (h->o.precision == PDHG_MIXED) {
    launch_cast_f32(h->b, h->bf, h->m, h->hs);
    launch_cast_f32(h->c, h->cf, h->n, h->hs);
  }
  HK();
  HC(hipStreamSynchronize(h->hs));
  h->ur_valid = false;
  return leave(h);
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
  if (h->grp.hstates) (void)hipHostFree(h->grp.hstates);
  delete h;
}

int pdhg_export_setup(pdhg_handle *h, uint8_t *var_kind, int32_t *colptr, int32_t *rowidx,
                      double *valT, double *val_s, double *Dr, double *Dc) {
  if (!h) return fail(PDHG_ERR_ARG, "null handle");
  RC(enter(h));
  auto d2h = [&](void *dst, const void *src, size_t bytes) -> int {
    if (dst) HC(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->hs));
    return PDHG_OK;
  };
  const int64_t m = h->m, n = h->n, nnz = h->nnz;
  if (!h->rperm) {
    RC(d2h(var_kind, h->vk, n));
    RC(d2h(colptr, h->cp, sizeof(int32_t) * (n + 1)));
    RC(d2h(rowidx, h->ri, sizeof(int32_t) * nnz));
    RC(d2h(valT, h->vt, sizeof(double) * nnz));
    RC(d2h(val_s, h->v, sizeof(double) * nnz));
    RC(d2h(Dr, h->Dr, sizeof(double) * m));
    RC(d2h(Dc, h->Dc, sizeof(double) * n));
    HC(hipStreamSynchronize(h->hs));
    return leave(h);
  }
  // the internal problem relabelled back into the caller's order (values are
  // moved, never recomputed, so this is the scaled problem exactly)
  std::vector<int32_t> prp(m + 1), pci(std::max<int64_t>(nnz, 1));
  std::vector<double> pv(std::max<int64_t>(nnz, 1)), dr(m), dc(n);
  std::vector<uint8_t> vk(n);
  RC(d2h(prp.data(), h->rp, sizeof(int32_t) * (m + 1)));
  RC(d2h(pci.data(), h->ci, sizeof(int32_t) * nnz));
  RC(d2h(pv.data(), h->v, sizeof(double) * nnz));
  RC(d2h(dr.data(), h->Dr, sizeof(double) * m));
  RC(d2h(dc.data(), h->Dc, sizeof(double) * n));
  RC(d2h(vk.data(), h->vk, n));
  HC(hipStreamSynchronize(h->hs));
  std::vector<int32_t> rp, ci, cp, ri;
  std::vector<double> v, vt;
  unpermute_csr(m, prp.data(), pci.data(), pv.data(), h->h_rperm, h->h_cperm, rp, ci, v);
  if (val_s) std::copy(v.begin(), v.begin() + nnz, val_s);
  if (colptr || rowidx || valT) {
    transpose_csr(m, n, rp.data(), ci.data(), v.data(), cp, ri, vt);
    if (colptr) std::copy(cp.begin(), cp.end(), colptr);
    if (rowidx) std::copy(ri.begin(), ri.begin() + nnz, rowidx);
    if (valT) std::copy(vt.begin(), vt.begin() + nnz, valT);
  }
  for (int64_t i = 0; i < m; i++)
    if (Dr) Dr[h->h_rperm[i]] = dr[i];
  for (int64_t j = 0; j < n; j++) {
    if (Dc) Dc[h->h_cperm[j]] = dc[j];
    if (var_kind) var_kind[h->h_cperm[j]] = vk[j];
  }
  return leave(h);
}

int pdhg_export_fp32(pdhg_handle *h, float *val_s, float *valT, float *b, float *c, float *l,
                     float *u) {
  if (!h) return fail(PDHG_ERR_ARG, "null handle");
  if (h->o.precision != PDHG_MIXED) return fail(PDHG_ERR_STATE, "no FP32 copies in FP64 mode");
  RC(enter(h));
  const int64_t m = h->m, n = h->n, nnz = h->nnz;
  std::vector<float> vf(std::max<int64_t>(nnz, 1)), vtf(std::max<int64_t>(nnz, 1)), bf(m), cf(n),
      lf(n), uf(n);
  std::vector<int32_t> prp(m + 1), pci(std::max<int64_t>(nnz, 1)), pcp(n + 1),
      pri(std::max<int64_t>(nnz, 1));
  auto d2h = [&](void *dst, const void *src, size_t bytes) -> int {
    HC(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->hs));
    return PDHG_OK;
  };
  if (nnz) {
    RC(d2h(vf.data(), h->vf, sizeof(float) * nnz));
    RC(d2h(vtf.data(), h->vtf, sizeof(float) * nnz));
    RC(d2h(pci.data(), h->ci, sizeof(int32_t) * nnz));
    RC(d2h(pri.data(), h->ri, sizeof(int32_t) * nnz));
  }
  RC(d2h(prp.data(), h->rp, sizeof(int32_t) * (m + 1)));
  RC(d2h(pcp.data(), h->cp, sizeof(int32_t) * (n + 1)));
  RC(d2h(bf.data(), h->bf, sizeof(float) * m));
  RC(d2h(cf.data(), h->cf, sizeof(float) * n));
  RC(d2h(lf.data(), h->lf, sizeof(float) * n));
  RC(d2h(uf.data(), h->uf, sizeof(float) * n));
  HC(hipStreamSynchronize(h->hs));
  if (!h->rperm) {
    if (val_s) std::copy(vf.begin(), vf.begin() + nnz, val_s);
    if (valT) std::copy(vtf.begin(), vtf.begin() + nnz, valT);
    if (b) std::copy(bf.begin(), bf.end(), b);
    if (c) std::copy(cf.begin(), cf.end(), c);
    if (l) std::copy(lf.begin(), lf.end(), l);
    if (u) std::copy(uf.begin(), uf.end(), u);
    return leave(h);
  }
  // relabelled back into the caller's order through double (exact both ways)
  auto back = [&](int64_t rows, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                  const std::vector<float> &val, const std::vector<int32_t> &ro,
                  const std::vector<int32_t> &co, float *out) {
    std::vector<double> wide(val.begin(), val.end());
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    unpermute_csr(rows, ptr.data(), idx.data(), wide.data(), ro, co, rp, ci, v);
    for (int64_t k = 0; k < nnz; k++) out[k] = (float)v[k];
  };
  if (val_s) back(m, prp, pci, vf, h->h_rperm, h->h_cperm, val_s);
  if (valT) back(n, pcp, pri, vtf, h->h_cperm, h->h_rperm, valT);
  for (int64_t i = 0; i < m; i++)
    if (b) b[h->h_rperm[i]] = bf[i];
  for (int64_t j = 0; j < n; j++) {
    if (c) c[h->h_cperm[j]] = cf[j];
    if (l) l[h->h_cperm[j]] = lf[j];
    if (u) u[h->h_cperm[j]] = uf[j];
  }
  return leave(h);
}

int pdhg_spmv(pdhg_handle *h, int transpose, const double *x, double *out) {
  if (!h || !x || !out) return fail(PDHG_ERR_ARG, "null argument");
  RC(enter(h));
  int64_t nin = transpose ? h->m : h->n, nout = transpose ? h->n : h->m;
  double *din = transpose ? h->it.YA : h->it.XA;
  double *dout = transpose ? h->it.ATYA : h->it.AXA;
  const std::vector<int32_t> &pin = transpose ? h->h_rperm : h->h_cperm;
  const std::vector<int32_t> &pout = transpose ? h->h_cperm : h->h_rperm;
  std::vector<double> xin, yout;
  const double *src = x;
  if (h->rperm) {  // caller's order <-> internal order on the host
    xin.resize(nin);
    for (int64_t q = 0; q < nin; q++) xin[q] = x[pin[q]];
    src = xin.data();
    yout.resize(nout);
  }
  HC(hipMemcpyAsync(din, src, sizeof(double) * nin, hipMemcpyHostToDevice, h->hs));
  if (transpose)
    launch_spmv(h->cp, h->ri, h->vt, h->n, din, dout, h->hs);
  else
    launch_spmv(h->rp, h->ci, h->v, h->m, din, dout, h->hs);
  HK();
  HC(hipMemcpyAsync(h->rperm ? yout.data() : out, dout, sizeof(double) * nout,
                    hipMemcpyDeviceToHost, h->hs));
  HC(hipStreamSynchronize(h->hs));
  if (h->rperm)
    for (int64_t q = 0; q < nout; q++) out[pout[q]] = yout[q];
  return leave(h);
}

}  // extern "C"

namespace {
template <typename T>
int time_kernels(pdhg_handle *h, int attempts, double *ms, const double *flush = nullptr,
                 int64_t flush_n = 0) {
  InstData d = base_data(h);
  std::vector<Inst<T>> one{make_inst<T>(h, d, h->it)};
  std::vector<int> act{0};
  Groups g{};
  RC(upload_group<T>(h, h->grp, one, act, g));
  const Inst<T> *dI = dev_insts<T>(h->grp);
  if (!h->state_ready) {
    // no solve has set the iterates and the control state (the buffer
    // index, steps, weights): start from the zero point, a few attempts in
    launch_init_point<T>(dI, g, h->hs);
    for (int i = 0; i < 16; i++) launch_attempt<T>(dI, g, h->hs);
    HK();
    h->state_ready = true;
  }
  // the start/stop events of each kernel carry its dispatch's own timestamps
  hipEvent_t ev[6];
  for (auto &e : ev) HC(hipEventCreate(&e));
  double acc[4] = {0, 0, 0, 0};
  for (int a = 0; a < attempts; a++) {
    // cold caches: reading flush_n doubles evicts the previous attempt's
    // lines from L2 and the Infinity Cache (clean lines, no write-back)
    if (flush) launch_sumsq(flush, flush_n, h->scratch, h->nscratch, h->hs);
    launch_primal<T>(dI, g, h->hs, ev[0], ev[1]);
    launch_dual<T>(dI, g, h->hs, ev[2], ev[3]);
    launch_control<T>(dI, g, h->hs, ev[4], ev[5]);
    HK();
    HC(hipEventSynchronize(ev[5]));
    float t;
    for (int q = 0; q < 3; q++) {
      HC(hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]));
      acc[q] += t;
    }
    HC(hipEventElapsedTime(&t, ev[0], ev[5]));
    acc[3] += t;
  }
  for (auto &e : ev) HC(hipEventDestroy(e));
  for (int q = 0; q < 4; q++) ms[q] = acc[q] / attempts;
  return PDHG_OK;
}
}  // namespace

extern "C" int pdhg_implied_bounds(pdhg_handle *h, double *lo, double *hi) {
  if (!h || !lo || !hi) return fail(PDHG_ERR_ARG, "null argument");
  const std::vector<double> &a = h->impl_valid ? h->h_ilo : h->h_l;
  const std::vector<double> &b = h->impl_valid ? h->h_ihi : h->h_u;
  std::copy(a.begin(), a.end(), lo);
  std::copy(b.begin(), b.end(), hi);
  return PDHG_OK;
}

extern "C" int pdhg_locality_order(int64_t m, int64_t n, const int32_t *row_ptr,
                                   const int32_t *col_idx, int32_t *row_order,
                                   int32_t *col_order) {
  if (m <= 0 || n <= 0 || !row_ptr || !row_order || !col_order)
    return fail(PDHG_ERR_ARG, "bad argument");
  if (row_ptr[0] != 0) return fail(PDHG_ERR_CSR, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < m; i++) {
    if (row_ptr[i + 1] < row_ptr[i]) return fail(PDHG_ERR_CSR, "row_ptr not monotone");
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
      if (col_idx[k] < 0 || col_idx[k] >= n || (k > row_ptr[i] && col_idx[k] <= col_idx[k - 1]))
        return fail(PDHG_ERR_CSR, "column indices out of range or not ascending in row %lld",
                    (long long)i);
  }
  std::vector<int32_t> cp, ri, ro, co;
  std::vector<double> none;
  transpose_csr(m, n, row_ptr, col_idx, nullptr, cp, ri, none);
  rcm_order(m, n, row_ptr, col_idx, cp.data(), ri.data(), ro, co);
  std::copy(ro.begin(), ro.end(), row_order);
  std::copy(co.begin(), co.end(), col_order);
  return PDHG_OK;
}

extern "C" int pdhg_get_partition(pdhg_handle *h, int *out) {
  if (!h || !out) return fail(PDHG_ERR_ARG, "null argument");
  out[0] = h->tpb_rows;
  out[1] = h->direct;
  out[2] = h->long_seg;
  out[3] = h->n_long_rows + h->n_long_cols;
  out[4] = h->compact ? 1 : 0;
  out[5] = h->stream_nt[0];
  out[6] = h->stream_nt[1];
  return PDHG_OK;
}

extern "C" int pdhg_time_kernels(pdhg_handle *h, int attempts, double *ms_out) {
  if (!h || !ms_out || attempts < 1) return fail(PDHG_ERR_ARG, "bad argument");
  RC(enter(h));
  int rc = h->o.precision == PDHG_MIXED ? time_kernels<float>(h, attempts, ms_out)
                                        : time_kernels<double>(h, attempts, ms_out);
  if (rc) return rc;
  return leave(h);
}

extern "C" int pdhg_time_kernels_cold(pdhg_handle *h, int attempts, const void *flush,
                                      size_t flush_bytes, double *ms_out) {
  if (!h || !ms_out || attempts < 1 || !flush || flush_bytes < 8)
    return fail(PDHG_ERR_ARG, "bad argument");
  RC(enter(h));
  const double *f = (const double *)flush;
  const int64_t fn = (int64_t)(flush_bytes / 8);
  int rc = h->o.precision == PDHG_MIXED ? time_kernels<float>(h, attempts, ms_out, f, fn)
                                        : time_kernels<double>(h, attempts, ms_out, f, fn);
  if (rc) return rc;
  return leave(h);
}

// ---------------------------------------------------------------------------
// merge-path SpMV

namespace {

#define HCN(call)                                                                  \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(PDHG_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
  } while (0)

int merge_sizes_ok(int64_t m, int64_t nnz) {
  if (m < 0 || nnz < 0 || m + nnz >= 0x7fffffffLL)
    return fail(PDHG_ERR_ARG, "m and nnz must be >= 0 with m + nnz < 2^31");
  return PDHG_OK;
}

template <typename T>
int spmv_merge_call(int64_t m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                    const T *val, const T *x, T *y, void *ws, size_t ws_bytes, void *stream) {
  RC(merge_sizes_ok(m, nnz));
  if (m == 0) return PDHG_OK;
  if (!row_ptr || !y || !ws || (nnz > 0 && (!col_idx || !val || !x)))
    return fail(PDHG_ERR_ARG, "null argument");
  if (((uintptr_t)ws & 255) != 0) return fail(PDHG_ERR_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < merge_workspace_bytes(m, nnz))
    return fail(PDHG_ERR_OOM, "workspace of %zu bytes, need %zu", ws_bytes,
                merge_workspace_bytes(m, nnz));
  launch_spmv_merge<T>(row_ptr, col_idx, val, x, y, m, nnz, ws, (hipStream_t)stream);
  HCN(hipGetLastError());
  return PDHG_OK;
}

}  // namespace

extern "C" int pdhg_spmv_merge_workspace_bytes(int64_t m, int64_t nnz, size_t *bytes) {
  RC(merge_sizes_ok(m, nnz));
  if (!bytes) return fail(PDHG_ERR_ARG, "null argument");
  *bytes = merge_workspace_bytes(m, nnz);
  return PDHG_OK;
}

extern "C" int pdhg_spmv_merge_plan(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                                    const int32_t *col_idx, void *ws, size_t ws_bytes,
                                    void *stream) {
  RC(merge_sizes_ok(m, nnz));
  if (n < 0) return fail(PDHG_ERR_ARG, "n must be >= 0");
  if (m == 0) return PDHG_OK;
  if (!row_ptr || !ws || (nnz > 0 && !col_idx)) return fail(PDHG_ERR_ARG, "null argument");
  if (((uintptr_t)ws & 255) != 0) return fail(PDHG_ERR_ARG, "workspace must be 256-byte aligned");
  const size_t need = merge_workspace_bytes(m, nnz);
  if (ws_bytes < need) return fail(PDHG_ERR_OOM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  // the structure check writes its flag into the carry-value area, which
  // the SpMV overwrites before reading
  const size_t nwg = (size_t)merge_workgroups(m, nnz);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  int *bad = (int *)((char *)ws + up(4 * (nwg + 1)) + up(4 * nwg));
  HCN(hipMemsetAsync(bad, 0, sizeof(int), s));
  launch_merge_check(row_ptr, col_idx, m, n, nnz, bad, s);
  HCN(hipGetLastError());
  int hbad = 1;
  HCN(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HCN(hipStreamSynchronize(s));
  if (hbad) return fail(PDHG_ERR_CSR, "row_ptr or col_idx is not a canonical CSR structure");
  launch_merge_plan(row_ptr, m, nnz, ws, s);
  HCN(hipGetLastError());
  return PDHG_OK;
}

extern "C" int pdhg_spmv_merge_f64(int64_t m, int64_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_idx, const double *val, const double *x,
                                   double *y, void *ws, size_t ws_bytes, void *stream) {
  return spmv_merge_call<double>(m, nnz, row_ptr, col_idx, val, x, y, ws, ws_bytes, stream);
}

extern "C" int pdhg_spmv_merge_f32(int64_t m, int64_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_idx, const float *val, const float *x,
                                   float *y, void *ws, size_t ws_bytes, void *stream) {
  return spmv_merge_call<float>(m, nnz, row_ptr, col_idx, val, x, y, ws, ws_bytes, stream);
}

namespace {

template <typename T>
int time_merge(pdhg_handle *h, int attempts, char *ws, double *ms) {
  const bool f32 = sizeof(T) == 4;
  const T *v = f32 ? (const T *)h->vf : (const T *)h->v;
  const T *vt = f32 ? (const T *)h->vtf : (const T *)h->vt;
  const IterBufs &b = h->it;
  // A' y into the average's buffer (n), A x into the next A x buffer (m)
  const T *xin = f32 ? (const T *)b.Xf[0] : (const T *)b.X[0];
  const T *yin = f32 ? (const T *)b.Yf[0] : (const T *)b.Y[0];
  T *aty = f32 ? (T *)b.XSf : (T *)b.XS;
  T *ax = f32 ? (T *)b.AXf[1] : (T *)b.AX[1];
  char *wsT = ws, *wsA = ws + merge_workspace_bytes(h->n, h->nnz);
  launch_merge_plan(h->cp, h->n, h->nnz, wsT, h->hs);
  launch_merge_plan(h->rp, h->m, h->nnz, wsA, h->hs);
  HK();
  hipEvent_t ev[4];
  for (auto &e : ev) HC(hipEventCreate(&e));
  double acc[2] = {0, 0};
  for (int a = 0; a < attempts; a++) {
    HC(hipEventRecord(ev[0], h->hs));
    launch_spmv_merge<T>(h->cp, h->ri, vt, yin, aty, h->n, h->nnz, wsT, h->hs);
    HC(hipEventRecord(ev[1], h->hs));
    HC(hipEventRecord(ev[2], h->hs));
    launch_spmv_merge<T>(h->rp, h->ci, v, xin, ax, h->m, h->nnz, wsA, h->hs);
    HC(hipEventRecord(ev[3], h->hs));
    HK();
    HC(hipEventSynchronize(ev[3]));
    float t;
    HC(hipEventElapsedTime(&t, ev[0], ev[1]));
    acc[0] += t;
    HC(hipEventElapsedTime(&t, ev[2], ev[3]));
    acc[1] += t;
  }
  for (auto &e : ev) HC(hipEventDestroy(e));
  ms[0] = acc[0] / attempts;
  ms[1] = acc[1] / attempts;
  return PDHG_OK;
}

}  // namespace

extern "C" int pdhg_time_spmv_merge(pdhg_handle *h, int attempts, void *ws, size_t ws_bytes,
                                    double *ms_out) {
  if (!h || !ms_out || !ws || attempts < 1) return fail(PDHG_ERR_ARG, "bad argument");
  if (((uintptr_t)ws & 255) != 0) return fail(PDHG_ERR_ARG, "workspace must be 256-byte aligned");
  const size_t need = merge_workspace_bytes(h->n, h->nnz) + merge_workspace_bytes(h->m, h->nnz);
  if (ws_bytes < need) return fail(PDHG_ERR_OOM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  RC(enter(h));
  int rc = h->o.precision == PDHG_MIXED ? time_merge<float>(h, attempts, (char *)ws, ms_out)
                                        : time_merge<double>(h, attempts, (char *)ws, ms_out);
  if (rc) return rc;
  return leave(h);
}
