// PDHG control, evaluation and bookkeeping kernels.
//
// One attempt is k_primal and k_dual (attempt.hip) followed by
//   k_control  step-size test, accept/reject by flipping the buffer index
// Every 'eval_period' attempts an evaluation computes the KKT error of the
// current and the averaged iterate, decides termination and restarts.
// All control state lives in device memory so that a block of attempts can be
// replayed as one HIP graph; the host reads the state only between blocks.
//
// Every kernel is grouped: one launch serves all instances of a batch.  A
// workgroup finds its instance by a binary search of the launch's prefix
// table, after the XCD remapping, so each XCD walks contiguous blocks of one
// instance.  A single solve is a group of one.
#include "device.h"

#include <hip/hip_ext.h>

#include <math.h>

namespace {

// Step-size control of one attempt (PDLP adaptive rule):
//   ebar = ||dz||_omega^2 / (2 |dy' A dx|),  accept iff eta <= ebar,
//   eta <- min((1 - (k+1)^-0.3) ebar, (1 + (k+1)^-0.6) eta),  k = attempts so far.
// PDHG_CTL_SPLIT workgroups per instance each sum a fixed slice of the
// attempt kernels' partials; the last one to finish (device-scope ticket)
// adds the slice sums in slice order and takes the decision.  The sums do
// not depend on which workgroup finishes last.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_control(const Inst<T> *__restrict__ I) {
  __shared__ double r[3];
  __shared__ int last;
  const int inst = blockIdx.x / PDHG_CTL_SPLIT, part = blockIdx.x % PDHG_CTL_SPLIT;
  const AS_C Inst<T> &in = cin(I)[inst];
  CtlState *gst = in.st;
  const int64_t nc = in.w.grid_cols, nr = in.w.grid_rows;
  // an instance with few partials (up to PDHG_CTL_SOLO of each kind) is
  // reduced and decided by its first workgroup alone: no slice sums, fences
  // or ticket; the others return
  const bool solo = nc <= PDHG_CTL_SOLO && nr <= PDHG_CTL_SOLO;
  if (solo && part != 0) return;
  const int nsplit = solo ? 1 : PDHG_CTL_SPLIT;
  const int64_t c0 = nc * part / nsplit, c1 = nc * (part + 1) / nsplit;
  const int64_t r0 = nr * part / nsplit, r1 = nr * (part + 1) / nsplit;
  const AS_G double *px = gin((const double *)in.w.part_dx2), *py = gin((const double *)in.w.part_dy);
  double v[3] = {0.0, 0.0, 0.0};
  {
    constexpr int CH = 4;
    double a[CH], d[CH], e[CH];
    for (int64_t b0 = 0; b0 < c1 - c0 || b0 < r1 - r0; b0 += CH * PDHG_BLOCK) {
#pragma unroll
      for (int q = 0; q < CH; q++) {
        int64_t bx = c0 + b0 + q * PDHG_BLOCK + threadIdx.x;
        int64_t by = r0 + b0 + q * PDHG_BLOCK + threadIdx.x;
        a[q] = bx < c1 ? px[bx] : 0.0;
        d[q] = by < r1 ? py[by] : 0.0;
        e[q] = by < r1 ? py[nr + by] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < CH; q++) {
        v[0] += a[q];
        v[1] += d[q];
        v[2] += e[q];
      }
    }
  }
  block_reduce<3, PDHG_BLOCK>(v, 0u, r);
  __shared__ double sl[3 * PDHG_CTL_SPLIT];
  __shared__ unsigned long long sw[sizeof(CtlState) / 8];
  if (solo) {
    if (threadIdx.x < sizeof(CtlState) / 8)
      sw[threadIdx.x] = gin((const unsigned long long *)gst)[threadIdx.x];
    if (threadIdx.x < 3) sl[threadIdx.x] = r[threadIdx.x];
    __syncthreads();
  } else {
    double *stage = in.w.ctl_stage;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < 3; q++) stage[3 * part + q] = r[q];
      __threadfence();  // the slice sums are visible before the ticket counts them
      last = atomicAdd(&gst->ticket, 1) == PDHG_CTL_SPLIT - 1;
    }
    __syncthreads();
    if (!last) return;
    // last workgroup: every lane fetches one slice sum or one state word after
    // its acquire fence (one round trip), then lane 0 combines them in order
    __threadfence();
    if (threadIdx.x < 3 * PDHG_CTL_SPLIT) sl[threadIdx.x] = gin((const double *)stage)[threadIdx.x];
    else if (threadIdx.x - 3 * PDHG_CTL_SPLIT < sizeof(CtlState) / 8)
      sw[threadIdx.x - 3 * PDHG_CTL_SPLIT] =
          gin((const unsigned long long *)gst)[threadIdx.x - 3 * PDHG_CTL_SPLIT];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double dx2 = 0.0, dy2 = 0.0, inter = 0.0;
  for (int p = 0; p < nsplit; p++) {
    dx2 += sl[3 * p];
    dy2 += sl[3 * p + 1];
    inter += sl[3 * p + 2];
  }
  CtlState st;
  {
    unsigned long long *dst = (unsigned long long *)&st;
    for (int q = 0; q < (int)(sizeof(CtlState) / 8); q++) dst[q] = sw[q];
  }
  st.ticket = 0;
  double eta = st.eta, omega = st.omega;
  long long k = st.k + 1;
  if (st.pending > 0.0) st.fresh = 0;  // this attempt's kernels folded it
  st.pending = 0.0;
  int accept = 1;
  double eta_new = eta;
  if (in.w.adaptive) {
    double nz = omega * dx2 + dy2 / omega;
    double ebar = (inter != 0.0) ? nz / (2.0 * fabs(inter)) : INFINITY;
    double kk = (double)(k + 1);
    double e1 = (1.0 - pow(kk, -0.3)) * ebar;
    double e2 = (1.0 + pow(kk, -0.6)) * eta;
    accept = (eta <= ebar);
    eta_new = e1 < e2 ? e1 : e2;
  }
  if (accept) {
    st.cur ^= 1;
    st.pending = eta;
    st.wsum += eta;
    st.accepted += 1;
  }
  st.eta = eta_new;
  st.k = k;
  st.dx2 = dx2;
  st.dy2 = dy2;
  st.inter = inter;
  store_state(gst, st);
}

// ---------------------------------------------------------------------------
// evaluation kernels (FP64)

__device__ inline bool have_avg(const CtlState *st, int use_average) {
  return use_average && st->wsum > 0.0;
}

// instance, its local block and its views for a launch over 256-row blocks
#define GROUP_BLOCK(pre)                                    \
  const int b = xcd_remap(blockIdx.x, gridDim.x);           \
  const int inst = find_inst(g.pre, g.ninst, b);            \
  const int lb = b - g.pre[inst];                           \
  const EvalView<T> &e = I[inst].e;                         \
  const CtlState *st = I[inst].st;                          \
  (void)st;                                                 \
  (void)lb;

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_avg_cols(const Inst<T> *__restrict__ I, Groups g) {
  GROUP_BLOCK(p_cols)
  if (!have_avg(st, e.use_average)) return;
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (j >= e.n) return;
  double pend = st->pending;
  T xs = e.XS[j];
  if (pend > 0.0) {
    xs = (st->fresh ? (T)0 : xs) + (T)pend * e.X[st->cur][j];
    e.XS[j] = xs;
  }
  e.XA[j] = (double)xs / st->wsum;
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_avg_rows(const Inst<T> *__restrict__ I, Groups g) {
  GROUP_BLOCK(p_rows)
  if (!have_avg(st, e.use_average)) return;
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= e.m) return;
  double pend = st->pending;
  T ys = e.YS[i];
  if (pend > 0.0) {
    ys = (st->fresh ? (T)0 : ys) + (T)pend * e.Y[st->cur][i];
    e.YS[i] = ys;
  }
  e.YA[i] = (double)ys / st->wsum;
}

// FP64 products of the evaluation (and of the start point):
//   SP_ATY   ATY  = A' y_cur   (columns)
//   SP_AXA   AXA  = A x_avg    (rows, skipped without an average)
//   SP_ATYA  ATYA = A' y_avg   (columns, skipped without an average)
//   SP_AX0   AXA  = A x_0      (rows; start point in buffer 0 of the iterate type)
enum { SP_ATY = 0, SP_AXA = 1, SP_ATYA = 2, SP_AX0 = 3 };

template <typename T>
struct SpmvSel {
  const int32_t *ptr, *idx;
  const double *v;
  int64_t rows;
  const T *xt;       // iterate-typed input or null
  const double *xd;  // FP64 input or null
  double *out;
  bool skip;
};

template <typename T>
__device__ inline SpmvSel<T> spmv_sel(const EvalView<T> &e, const CtlState *st, int mode) {
  SpmvSel<T> s;
  bool rowsA = (mode == SP_AXA || mode == SP_AX0);
  s.ptr = rowsA ? e.rp : e.cp;
  s.idx = rowsA ? e.ci : e.ri;
  s.v = rowsA ? e.v : e.vt;
  s.rows = rowsA ? e.m : e.n;
  s.xt = mode == SP_ATY ? e.Y[st->cur] : (mode == SP_AX0 ? e.X[0] : nullptr);
  s.xd = mode == SP_AXA ? e.XA : (mode == SP_ATYA ? e.YA : nullptr);
  s.out = mode == SP_ATY ? e.ATY : (mode == SP_ATYA ? e.ATYA : e.AXA);
  s.skip = (mode == SP_AXA || mode == SP_ATYA) && !have_avg(st, e.use_average);
  return s;
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_eval_spmv(const Inst<T> *__restrict__ I, Groups g,
                                                          int mode) {
  const bool rowsA = (mode == SP_AXA || mode == SP_AX0);
  const int32_t *pre = rowsA ? g.p_rows : g.p_cols;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = find_inst(pre, g.ninst, b);
  const int lb = b - pre[inst];
  SpmvSel<T> s = spmv_sel(I[inst].e, I[inst].st, mode);
  if (s.skip) return;
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= s.rows) return;
  int a = s.ptr[i], z = s.ptr[i + 1];
  if (z - a > I[inst].e.long_seg) return;
  double acc = 0.0;
  if (s.xt)
    for (int k = a; k < z; k++) acc += s.v[k] * (double)s.xt[s.idx[k]];
  else
    for (int k = a; k < z; k++) acc += s.v[k] * s.xd[s.idx[k]];
  s.out[i] = acc;
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_eval_spmv_long(const Inst<T> *__restrict__ I,
                                                               Groups g, int mode) {
  const bool rowsA = (mode == SP_AXA || mode == SP_AX0);
  const int32_t *pre = rowsA ? g.p_lrows : g.p_lcols;
  const int b = blockIdx.x;
  const int inst = find_inst(pre, g.ninst, b);
  const int lb = b - pre[inst];
  const IterView<T> &w = I[inst].w;
  SpmvSel<T> s = spmv_sel(I[inst].e, I[inst].st, mode);
  if (s.skip) return;
  int64_t i = rowsA ? w.long_rows[lb] : w.long_cols[lb];
  int a = s.ptr[i], z = s.ptr[i + 1];
  double acc[1] = {0.0};
  if (s.xt)
    for (int k = a + threadIdx.x; k < z; k += PDHG_BLOCK) acc[0] += s.v[k] * (double)s.xt[s.idx[k]];
  else
    for (int k = a + threadIdx.x; k < z; k += PDHG_BLOCK) acc[0] += s.v[k] * s.xd[s.idx[k]];
  double tot[1];
  block_reduce<1>(acc, 0u, tot);
  if (threadIdx.x == 0) s.out[i] = tot[0];
}

// Row dots of the evaluation, one 256-row tile of a FP64 CSR matrix per
// workgroup: s0 = sum_k v[k] x0[idx[k]] and, when x1 is given,
// s1 = sum_k v[k] x1[idx[k]], for this lane's row i, in CSR order with each
// product rounded on its own.  The tile's indices and values are loaded once
// and both products staged in LDS (tiles past EV_TILE_CAP nonzeros use
// per-lane loops).  `mine` is false for rows longer than long_seg, whose
// products a workgroup of their own computes beforehand.  Every lane must
// call it; lds holds 2 (EV_TILE_CAP + PDHG_BLOCK) doubles.
// 1024 staged products per tile keep the two buffers at 20 KB, which allows
// 7 workgroups per CU (2048 products, 37 KB, allowed 4 and was 10-19% slower
// on 7.2M nonzeros, although fewer tiles fell back to per-lane loops)
#define EV_TILE_CAP (4 * PDHG_BLOCK)
template <typename X0>
__device__ inline void eval_rowdots(const int32_t *ptr_, const int32_t *idx_, const double *v_,
                                    const X0 *x0_, const double *x1_, int64_t i, bool valid,
                                    int base, int top, int long_seg, double *lds, double &s0,
                                    double &s1, bool &mine) {
  const AS_G int32_t *ptr = gin(ptr_), *idx = gin(idx_);
  const AS_G double *v = gin(v_), *x1 = gin(x1_);
  const AS_G X0 *x0 = gin(x0_);
  const int cnt = top - base;
  const bool two = x1_ != nullptr;
  double *lds1 = lds + EV_TILE_CAP + PDHG_BLOCK;
  int rs = 0, re = 0;
  s0 = s1 = 0.0;
  if (cnt <= EV_TILE_CAP) {
    for (int k0 = 0; k0 < cnt; k0 += 4 * PDHG_BLOCK) {
      int id[4];
      double vv[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int k = k0 + q * PDHG_BLOCK + (int)threadIdx.x;
        int kc = base + (k < cnt ? k : cnt - 1);
        id[q] = __builtin_nontemporal_load(idx + kc);
        vv[q] = __builtin_nontemporal_load(v + kc);
      }
      if (k0 == 0 && valid) {
        rs = ptr[i];
        re = ptr[i + 1];
      }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int k = k0 + q * PDHG_BLOCK + (int)threadIdx.x;
        int slot = k < cnt ? k : EV_TILE_CAP + (int)threadIdx.x;
        lds[slot] = __dmul_rn(vv[q], (double)x0[id[q]]);
        if (two) lds1[slot] = __dmul_rn(vv[q], x1[id[q]]);
      }
    }
    if (cnt == 0 && valid) {
      rs = ptr[i];
      re = ptr[i + 1];
    }
    __syncthreads();
    mine = valid && (re - rs <= long_seg);
    if (mine) {
      for (int k = rs - base; k < re - base; k++) s0 += lds[k];
      if (two)
        for (int k = rs - base; k < re - base; k++) s1 += lds1[k];
    }
    __syncthreads();
  } else {
    if (valid) {
      rs = ptr[i];
      re = ptr[i + 1];
    }
    mine = valid && (re - rs <= long_seg);
    if (mine)
      for (int k = rs; k < re; k++) {
        s0 += __dmul_rn(v[k], (double)x0[idx[k]]);
        if (two) s1 += __dmul_rn(v[k], x1[idx[k]]);
      }
  }
}

// Row-space KKT pieces for the current point and the average, with A x_avg
// computed here (and kept for a restart to the average):
// [0] ||r_p||^2 scaled [1] ||r_p||^2 unscaled [2] ||r_p||_inf unscaled
// [3] b'y [4] ||y - y_last||^2, then the same five for the average.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_eval_rows(const Inst<T> *__restrict__ I, Groups g) {
  __shared__ double lds[2 * (EV_TILE_CAP + PDHG_BLOCK)];
  GROUP_BLOCK(p_rows)
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  bool avg = have_avg(st, e.use_average);
  double axa = 0.0;
  if (avg) {
    int64_t r0 = (int64_t)lb * PDHG_BLOCK, rend = r0 + PDHG_BLOCK < e.m ? r0 + PDHG_BLOCK : e.m;
    double unused;
    bool mine;
    eval_rowdots<double>(e.rp, e.ci, e.v, e.XA, nullptr, i, i < e.m, e.rp[r0], e.rp[rend],
                         e.long_seg, lds, axa, unused, mine);
    if (i < e.m) {
      if (mine)
        e.AXA[i] = axa;
      else
        axa = e.AXA[i];  // long row: its own workgroup computed it
    }
  }
  double q[EV_ROWQ];
#pragma unroll
  for (int t = 0; t < EV_ROWQ; t++) q[t] = 0.0;
  if (i < e.m) {
    int cur = st->cur;
    double bi = gin(e.b)[i], dr = gin(e.Dr)[i], yl = gin((const double *)e.YL)[i];
    bool ge = gin(e.kind)[i] == 1;
#pragma unroll
    for (int p = 0; p < 2; p++) {
      if (p == 1 && !avg) break;
      double yi = p ? gin((const double *)e.YA)[i] : (double)gin((const T *)e.Y[cur])[i];
      double axi = p ? axa : (double)gin((const T *)e.AX[cur])[i];
      double r = bi - axi;
      if (ge && r < 0.0) r = 0.0;
      double ru = r / dr;
      q[5 * p + 0] = r * r;
      q[5 * p + 1] = ru * ru;
      q[5 * p + 2] = fabs(ru);
      q[5 * p + 3] = bi * yi;
      q[5 * p + 4] = (yi - yl) * (yi - yl);
    }
  }
  double out[EV_ROWQ];
  block_reduce<EV_ROWQ>(q, (1u << 2) | (1u << 7), out);
  if (threadIdx.x == 0)
    for (int t = 0; t < EV_ROWQ; t++) e.part_rows[(int64_t)t * e.nblk_rows + lb] = out[t];
}

__device__ inline double proj_lambda(uint8_t vk, double lam) {
  if (vk == VK_FREE) return 0.0;
  if (vk == VK_LOWER) return lam > 0.0 ? lam : 0.0;
  if (vk == VK_UPPER) return lam < 0.0 ? lam : 0.0;
  return lam;
}

__device__ inline double bound_term(uint8_t vk, double lam, double l, double u) {
  double t = 0.0;
  if (lam > 0.0 && (vk == VK_LOWER || vk == VK_BOXED || vk == VK_FIXED)) t += l * lam;
  if (lam < 0.0 && (vk == VK_UPPER || vk == VK_BOXED || vk == VK_FIXED)) t += u * lam;
  return t;
}

// Column-space KKT pieces, with A'y and A'y_avg computed here:
// [0] ||r_d||^2 scaled [1] ||r_d||^2 unscaled
// [2] ||r_d||_inf unscaled [3] bound part of the dual objective [4] c'x
// [5] ||x - x_last||^2, then the same six for the average.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_eval_cols(const Inst<T> *__restrict__ I, Groups g) {
  __shared__ double lds[2 * (EV_TILE_CAP + PDHG_BLOCK)];
  GROUP_BLOCK(p_cols)
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  bool avg = have_avg(st, e.use_average);
  double aty[2];
  {
    int64_t c0 = (int64_t)lb * PDHG_BLOCK, cend = c0 + PDHG_BLOCK < e.n ? c0 + PDHG_BLOCK : e.n;
    bool mine;
    eval_rowdots<T>(e.cp, e.ri, e.vt, e.Y[st->cur], avg ? e.YA : nullptr, j, j < e.n, e.cp[c0],
                    e.cp[cend], e.long_seg, lds, aty[0], aty[1], mine);
    if (j < e.n && !mine) {  // long column: its own workgroup computed the sums
      aty[0] = e.ATY[j];
      if (avg) aty[1] = e.ATYA[j];
    }
  }
  double q[EV_COLQ];
#pragma unroll
  for (int t = 0; t < EV_COLQ; t++) q[t] = 0.0;
  if (j < e.n) {
    int cur = st->cur;
    double cj = gin(e.c)[j], dc = gin(e.Dc)[j], lj = gin(e.l)[j], uj = gin(e.u)[j];
    double xl = gin((const double *)e.XL)[j];
    uint8_t vk = gin(e.vk)[j];
#pragma unroll
    for (int p = 0; p < 2; p++) {  // constant indices keep q in registers
      if (p == 1 && !avg) break;
      double xj = p ? gin((const double *)e.XA)[j] : (double)gin((const T *)e.X[cur])[j];
      double lam = cj - aty[p];
      double pl = proj_lambda(vk, lam);
      double rd = lam - pl;
      double rdu = rd / dc;
      q[6 * p + 0] = rd * rd;
      q[6 * p + 1] = rdu * rdu;
      q[6 * p + 2] = fabs(rdu);
      q[6 * p + 3] = bound_term(vk, pl, lj, uj);
      q[6 * p + 4] = cj * xj;
      q[6 * p + 5] = (xj - xl) * (xj - xl);
    }
  }
  double out[EV_COLQ];
  block_reduce<EV_COLQ>(q, (1u << 2) | (1u << 8), out);
  if (threadIdx.x == 0)
    for (int t = 0; t < EV_COLQ; t++) e.part_cols[(int64_t)t * e.nblk_cols + lb] = out[t];
}

struct PointKKT {
  double komega, rel_kkt, pobj, dobj, rel_p, rel_d, rel_g, sp2, sd2, gap, dl_x, dl_y;
};

__device__ inline PointKKT point_kkt(const double *rq, const double *cq, double omega, double nb,
                                     double nc) {
  PointKKT p;
  p.sp2 = rq[0];
  p.sd2 = cq[0];
  p.pobj = cq[4];
  p.dobj = rq[3] + cq[3];
  p.gap = fabs(p.pobj - p.dobj);
  p.komega = sqrt(omega * p.sp2 + p.sd2 / omega + p.gap * p.gap);
  p.rel_p = sqrt(rq[1]) / (1.0 + nb);
  p.rel_d = sqrt(cq[1]) / (1.0 + nc);
  p.rel_g = p.gap / (1.0 + fabs(p.pobj) + fabs(p.dobj));
  double r = p.rel_p;
  if (p.rel_d > r) r = p.rel_d;
  if (p.rel_g > r) r = p.rel_g;
  p.rel_kkt = r;
  p.dl_x = sqrt(cq[5]);
  p.dl_y = sqrt(rq[4]);
  return p;
}

// Termination (relative KKT on the original problem), restart decision on
// the scaled KKT_omega (restart at the better of current and average when it
// fell to 0.2 of the last restart's, or to 0.8 with no progress since the
// previous evaluation, or after 0.36 of all attempts), primal-weight update.
// PDHG_CTL_SPLIT workgroups per instance reduce fixed slices of the
// evaluation partials; the last to finish combines the slices in slice order
// and takes the decisions.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_eval_control(const Inst<T> *__restrict__ I,
                                                             double tol, long long max_iter) {
  constexpr unsigned ROWMAX = (1u << 2) | (1u << 7), COLMAX = (1u << 2) | (1u << 8);
  constexpr int NQ = EV_ROWQ + EV_COLQ;
  __shared__ double r[NQ];
  __shared__ int last;
  const int inst = blockIdx.x / PDHG_CTL_SPLIT, part = blockIdx.x % PDHG_CTL_SPLIT;
  const AS_C Inst<T> &in = cin(I)[inst];
  const AS_C EvalView<T> &e = in.e;
  CtlState *gst = in.st;
  const int64_t nbr = e.nblk_rows, nbc = e.nblk_cols;
  const int64_t r0 = nbr * part / PDHG_CTL_SPLIT, r1 = nbr * (part + 1) / PDHG_CTL_SPLIT;
  const int64_t c0 = nbc * part / PDHG_CTL_SPLIT, c1 = nbc * (part + 1) / PDHG_CTL_SPLIT;
  reduce_partials<EV_ROWQ, PDHG_BLOCK>(e.part_rows + r0, r1 - r0, nbr, ROWMAX, r);
  reduce_partials<EV_COLQ, PDHG_BLOCK>(e.part_cols + c0, c1 - c0, nbc, COLMAX, r + EV_ROWQ);
  double *stage = e.ev_stage;
  if (threadIdx.x == 0) {
    for (int q = 0; q < NQ; q++) stage[NQ * part + q] = r[q];
    __threadfence();  // the slice results are visible before the ticket counts them
    last = atomicAdd(&gst->ticket, 1) == PDHG_CTL_SPLIT - 1;
  }
  __syncthreads();
  if (!last) return;
  // last workgroup: the slice results and the state words fetched in
  // parallel after the acquire fence, then combined in slice order by lane 0
  constexpr int NS = NQ * PDHG_CTL_SPLIT, NW = NS + (int)(sizeof(CtlState) / 8);
  static_assert(NW <= 2 * PDHG_BLOCK, "two words per lane");
  __shared__ double sl[NS];
  __shared__ unsigned long long sw[sizeof(CtlState) / 8];
  __threadfence();
  {
    const AS_G unsigned long long *src_s = gin((const unsigned long long *)stage);
    const AS_G unsigned long long *src_w = gin((const unsigned long long *)gst);
    const int t0 = threadIdx.x, t1 = threadIdx.x + PDHG_BLOCK;
    unsigned long long a0 = t0 < NS ? src_s[t0] : (t0 < NW ? src_w[t0 - NS] : 0ull);
    unsigned long long a1 = t1 < NS ? src_s[t1] : (t1 < NW ? src_w[t1 - NS] : 0ull);
    if (t0 < NS) sl[t0] = __longlong_as_double((long long)a0);
    else if (t0 < NW) sw[t0 - NS] = a0;
    if (t1 < NS) sl[t1] = __longlong_as_double((long long)a1);
    else if (t1 < NW) sw[t1 - NS] = a1;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double rq[EV_ROWQ], cq[EV_COLQ];
  for (int q = 0; q < NQ; q++) {
    bool mx = q < EV_ROWQ ? ((ROWMAX >> q) & 1) : ((COLMAX >> (q - EV_ROWQ)) & 1);
    double a = 0.0;
    for (int p = 0; p < PDHG_CTL_SPLIT; p++) {
      double t = sl[NQ * p + q];
      a = mx ? fmax(a, t) : a + t;
    }
    if (q < EV_ROWQ)
      rq[q] = a;
    else
      cq[q - EV_ROWQ] = a;
  }
  CtlState stv;
  {
    unsigned long long *dst = (unsigned long long *)&stv;
    for (int q = 0; q < (int)(sizeof(CtlState) / 8); q++) dst[q] = sw[q];
  }
  stv.ticket = 0;
  CtlState *st = &stv;
  bool avg = e.use_average && st->wsum > 0.0;
  double omega = st->omega;
  PointKKT pc = point_kkt(rq, cq, omega, st->nb, st->nc);
  PointKKT pa = pc;
  if (avg) pa = point_kkt(rq + 5, cq + 6, omega, st->nb, st->nc);
  long long k = st->k;
  if (st->pending > 0.0) st->fresh = 0;  // the average kernels folded it
  st->pending = 0.0;
  st->have_avg = avg;
  st->restart_flag = 0;
  if (st->init_pending) {
    st->kkt_last = pc.komega;
    st->init_pending = 0;
  }
  const PointKKT *rep = &pc;
  int which = 0;
  // the tested quantity: the relative KKT error, or for feasibility
  // polishing one relative residual alone
  const double tc = e.term == 1 ? pc.rel_p : (e.term == 2 ? pc.rel_d : pc.rel_kkt);
  const double ta = e.term == 1 ? pa.rel_p : (e.term == 2 ? pa.rel_d : pa.rel_kkt);
  if (!isfinite(pc.rel_kkt)) {
    st->done = 1;
    st->status = 4;
  } else if (tc <= tol) {
    st->done = 1;
    st->status = 1;
  } else if (avg && ta <= tol) {
    st->done = 1;
    st->status = 1;
    which = 1;
    rep = &pa;
  } else if (k >= max_iter) {
    st->done = 1;
    st->status = 2;
  } else if (e.restart && k > 0) {
    bool cand_avg = avg && pa.komega < pc.komega;
    const PointKKT *cd = cand_avg ? &pa : &pc;
    double kc = cd->komega;
    bool do_restart = (kc <= 0.2 * st->kkt_last) ||
                      (kc <= 0.8 * st->kkt_last && kc > st->kkt_prev) ||
                      ((double)(k - st->last_restart) >= 0.36 * (double)k);
    st->kkt_prev = kc;
    if (do_restart) {
      st->restart_flag = cand_avg ? 2 : 1;
      double dx = cd->dl_x, dy = cd->dl_y;
      double th = k < e.hold_k ? 0.0 : e.pw_theta;
      if (th > 0.0 && dx > 1e-10 && dy > 1e-10)
        omega = exp(th * log(dy / dx) + (1.0 - th) * log(omega));
      st->omega = omega;
      st->kkt_last = sqrt(omega * cd->sp2 + cd->sd2 / omega + cd->gap * cd->gap);
      st->kkt_prev = INFINITY;
      st->wsum = 0.0;
      st->fresh = 1;
      st->last_restart = k;
      st->restarts += 1;
      rep = cd;
    }
  }
  st->which = which;
  st->stash = 0;
  if (e.xbest && rep->rel_kkt < st->best_kkt) {  // FP32 phase: new best point
    st->stash = 1;
    st->best_kkt = rep->rel_kkt;
  }
  st->pobj = rep->pobj;
  st->dobj = rep->dobj;
  st->rel_p = rep->rel_p;
  st->rel_d = rep->rel_d;
  st->rel_gap = rep->rel_g;
  st->rel_kkt = rep->rel_kkt;
  store_state(gst, stv);
}

// FP32 phase: keep the evaluated current iterate when it is the best so far
// (in FP64, in the buffers the FP64 phase starts from).
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_stash_cols(const Inst<T> *__restrict__ I, Groups g) {
  GROUP_BLOCK(p_cols)
  if (!e.xbest || !st->stash) return;
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (j >= e.n) return;
  // the evaluated point: the average when it was reported or restarted to
  e.xbest[j] = (st->which || st->restart_flag == 2) ? e.XA[j] : (double)e.X[st->cur][j];
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_stash_rows(const Inst<T> *__restrict__ I, Groups g) {
  GROUP_BLOCK(p_rows)
  if (!e.ybest || !st->stash) return;
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= e.m) return;
  e.ybest[i] = (st->which || st->restart_flag == 2) ? e.YA[i] : (double)e.Y[st->cur][i];
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_restart_cols(const Inst<T> *__restrict__ I,
                                                             Groups g) {
  GROUP_BLOCK(p_cols)
  int f = st->restart_flag;
  if (f == 0) return;
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (j >= e.n) return;
  T *x = e.X[st->cur];
  if (f == 2) x[j] = (T)e.XA[j];
  e.XL[j] = (double)x[j];
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_restart_rows(const Inst<T> *__restrict__ I,
                                                             Groups g) {
  GROUP_BLOCK(p_rows)
  int f = st->restart_flag;
  if (f == 0) return;
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= e.m) return;
  T *y = e.Y[st->cur];
  if (f == 2) {
    y[i] = (T)e.YA[i];
    e.AX[st->cur][i] = (T)e.AXA[i];
  }
  e.YL[i] = (double)y[i];
}

// ---------------------------------------------------------------------------
// certificate of primal infeasibility, every infeas_period attempts (FP64)
//
// Farkas: with y_i >= 0 on >= rows and a box [lo, hi] holding every feasible
// x (l, u tightened by the implied bounds), a feasible x would give
// b'y <= sum_j (A'y)_j x_j <= sum_j max over [lo_j, hi_j] of (A'y)_j x_j.
// So b'y + sum_j min(lambda_j lo_j, lambda_j hi_j) > 0 with lambda = -A'y,
// beyond its rounding allowance, proves that no feasible x exists.  The sum
// is the safe bound's for c = 0 (same sign rule and allowance), taken at the
// current y, which the iteration keeps projected.  The test runs after the
// evaluation's decisions and before its restart copies, and is skipped
// (uniformly) when the instance is done or k is not a multiple of the period.
//
// Dual infeasibility (PDLP's ray test, a tolerance test): the primal
// displacement since the last restart, d = Dc (x - XL), certifies an
// improving ray when c'd < 0 and the largest violation of (A d)_i = 0 on =
// rows, (A d)_i >= 0 on >= rows and of d_j in the recession cone of
// [lo_j, hi_j] is at most dinf_tol (-c'd).  In the scaled problem
// (A d)_i = (A^ d^)_i / Dr_i and c_j d_j = c^_j d^_j exactly.  On an
// unbounded LP the iterates move by a fixed ray per step once their
// projections stop changing, and a restart inside that phase makes d an
// exact multiple of it.  Tested after the primal certificate.

// y of the Farkas test: projected on >= rows, then clamped into the repair
// interval for c = 0 (any such y is a candidate certificate)
__device__ inline double farkas_y(double y, uint8_t kind, uint8_t fk) {
  if (kind == 1 && y < 0.0) y = 0.0;
  if (fk & 1) y = fmax(y, 0.0);
  if (fk & 2) y = fmin(y, 0.0);
  return y;
}

template <typename T>
__device__ inline bool infeas_due(const EvalView<T> &e, const CtlState *st) {
  return e.infeas_period > 0 && !st->done && st->k > 0 && st->k % e.infeas_period == 0;
}

// Rows: partials [0] b'y, [1] sum |b_i y_i|, [2] largest violation of the
// row's cone by A d (ray test, over the FP64 matrix).  A row of up to
// INFEAS_LANE_ROW entries is summed by its own lane; a longer one by the
// whole wave, one such row after the other (lanes stride its entries, a
// butterfly sums them), so a few thousand-entry rows do not hold a wave
// for thousands of dependent loads.
#define INFEAS_LANE_ROW 64
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_infeas_rows(const Inst<T> *__restrict__ I,
                                                            Groups g) {
  GROUP_BLOCK(p_rows)
  if (!infeas_due(e, st)) return;
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  double q[3] = {0.0, 0.0, 0.0};
  const bool ray = e.dinf_tol > 0.0;
  const AS_G int32_t *rp = gin(e.rp), *ci = gin(e.ci);
  const AS_G double *v = gin(e.v), *xl = gin((const double *)e.XL);
  const AS_G T *x = gin((const T *)e.X[st->cur]);
  int a = 0, z = 0;
  uint8_t ki = 0;
  double s = 0.0;
  if (i < e.m) {
    ki = gin(e.kind)[i];
    const double yi = farkas_y((double)gin((const T *)e.Y[st->cur])[i], ki,
                               I[inst].fyk ? gin(I[inst].fyk)[i] : (uint8_t)0);
    double t = __dmul_rn(gin(e.b)[i], yi);
    q[0] = t;
    q[1] = fabs(t);
    if (ray) {
      a = rp[i];
      z = rp[i + 1];
      if (z - a <= INFEAS_LANE_ROW)
        for (int k = a; k < z; k++) {
          const int32_t j = ci[k];
          s += __dmul_rn(v[k], (double)x[j] - xl[j]);
        }
    }
  }
  if (ray) {
    // long rows of this wave, in lane order (the loop is uniform per wave)
    uint64_t pend = __ballot(i < e.m && z - a > INFEAS_LANE_ROW);
    const int lane = threadIdx.x & 63;
    while (pend) {
      const int src = __ffsll((unsigned long long)pend) - 1;
      pend &= pend - 1;
      const int ra = __shfl(a, src), rz = __shfl(z, src);
      double part = 0.0;
      for (int k = ra + lane; k < rz; k += 64) {
        const int32_t j = ci[k];
        part += __dmul_rn(v[k], (double)x[j] - xl[j]);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
      if (lane == src) s = part;
    }
    if (i < e.m) {
      const double r = s / gin(e.Dr)[i];
      // non-finite counts as infinite (fmax would drop a NaN)
      q[2] = !isfinite(r) ? INFINITY : ki == 0 ? fabs(r) : fmax(-r, 0.0);
    }
  }
  double out[3];
  block_reduce<3>(q, 4u, out);
  if (threadIdx.x == 0)
    for (int t = 0; t < 3; t++) e.part_rows[(int64_t)t * e.nblk_rows + lb] = out[t];
}

// Columns, one lane per column: lambda_j = -sum_i a_ij y_i in ascending row
// order, its error bound, and the term as in the safe bound (c = 0).
// Partials [0] terms, [1] magnitudes, [2] needed infinite bounds; for the
// ray test [3] c'd and [4] the largest violation of the bounds' recession
// cones by d.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_infeas_cols(const Inst<T> *__restrict__ I,
                                                            Groups g) {
  GROUP_BLOCK(p_cols)
  if (!infeas_due(e, st)) return;
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (j < e.n) {
    const AS_G int32_t *cp = gin(e.cp), *ri = gin(e.ri);
    const AS_G double *vt = gin(e.vt);
    const AS_G T *y = gin((const T *)e.Y[st->cur]);
    const AS_G uint8_t *kind = gin(e.kind);
    const AS_G uint8_t *fyk = I[inst].fyk ? gin(I[inst].fyk) : nullptr;
    const int a = cp[j], z = cp[j + 1];
    double s = 0.0, sa = 0.0;
    for (int k = a; k < z; k++) {
      const int32_t i = ri[k];
      const double yi = farkas_y((double)y[i], kind[i], fyk ? fyk[i] : (uint8_t)0);
      double pr = __dmul_rn(vt[k], yi);
      s += pr;
      sa += fabs(pr);
    }
    const double lam = 0.0 - s;
    const double err = 2.0 * (double)(z - a + 2) * 0x1p-53 * sa;
    double lo = gin(e.l)[j], hi = gin(e.u)[j];
    if (e.ilo) {
      lo = fmax(lo, gin(e.ilo)[j]);
      hi = fmin(hi, gin(e.ihi)[j]);
    }
    if (fabs(lam) > err || err == 0.0) {
      if (lam != 0.0) {
        double bnd = lam > 0.0 ? lo : hi;
        if (isinf(bnd)) {
          q[2] = 1.0;
        } else {
          q[0] = __dmul_rn(lam, bnd);
          q[1] = fabs(bnd) * sa;
        }
      }
    } else if (isinf(lo) || isinf(hi)) {
      q[2] = 1.0;
    } else {
      q[0] = fmin(__dmul_rn(lam, lo), __dmul_rn(lam, hi));
      q[1] = fmax(fabs(lo), fabs(hi)) * sa;
    }
    if (e.dinf_tol > 0.0) {
      const double dh = (double)gin((const T *)e.X[st->cur])[j] - gin((const double *)e.XL)[j];
      const double d = __dmul_rn(gin(e.Dc)[j], dh);
      q[3] = __dmul_rn(gin(e.c)[j], dh);
      const bool flo = isfinite(lo), fhi = isfinite(hi);
      q[4] = !isfinite(d)  ? INFINITY
             : flo && fhi ? fabs(d)
             : flo        ? fmax(-d, 0.0)
             : fhi        ? fmax(d, 0.0)
                          : 0.0;
    }
  }
  double out[5];
  block_reduce<5>(q, 16u, out);
  if (threadIdx.x == 0)
    for (int t = 0; t < 5; t++) e.part_cols[(int64_t)t * e.nblk_cols + lb] = out[t];
}

// One workgroup per instance: the values in fixed order.  A positive Farkas
// value ends the solve with the current iterate as the certificate; else a
// passing ray test ends it with the ray (returned as x).
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_infeas_finish(const Inst<T> *__restrict__ I) {
  const EvalView<T> &e = I[blockIdx.x].e;
  CtlState *st = I[blockIdx.x].st;
  if (!infeas_due(e, st)) return;
  double r[3], c[5];
  reduce_partials<3, PDHG_BLOCK>(e.part_rows, e.nblk_rows, e.nblk_rows, 4u, r);
  reduce_partials<5, PDHG_BLOCK>(e.part_cols, e.nblk_cols, e.nblk_cols, 16u, c);
  if (threadIdx.x != 0) return;
  int status = 0;
  if (c[2] == 0.0 && (r[0] + c[0]) - e.bound_allow * (r[1] + c[1]) > 0.0)
    status = 5;  // PDHG_PRIMAL_INFEASIBLE
  else if (e.dinf_tol > 0.0 && c[3] < 0.0 && fmax(r[2], c[4]) <= e.dinf_tol * -c[3])
    status = 6;  // PDHG_DUAL_INFEASIBLE
  if (status) {
    st->done = 1;
    st->status = status;
    st->which = 0;
    st->restart_flag = 0;
  }
}

// ---------------------------------------------------------------------------
// safe dual bound of the reported point, once after the solve (FP64)
//
// Weak duality: for any y~ with y~_i >= 0 on >= rows, every feasible x has
// c'x >= b'y~ + sum_j lambda_j x_j >= b'y~ + sum_j min(lambda_j lo_j,
// lambda_j hi_j), lambda = c - A'y~, with [lo, hi] = [l, u] tightened by the
// implied bounds.  y~ is the reported y, projected on >= rows and clamped
// into the row's repair interval (which keeps the reduced costs of
// single-entry columns with an infinite bound sign-feasible).  In the scaled
// problem every term equals its unscaled counterpart exactly (power-of-two
// factors).

// Rows: y~ into YL (the restart anchor, unused after the solve); partials
// [0] b'y~, [1] sum |b_i y~_i|.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_bound_rows(const Inst<T> *__restrict__ I,
                                                           Groups g) {
  GROUP_BLOCK(p_rows)
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  double q[2] = {0.0, 0.0};
  if (i < e.m) {
    double yi = st->which ? gin((const double *)e.YA)[i] : (double)gin((const T *)e.Y[st->cur])[i];
    if (gin(e.kind)[i] == 1 && yi < 0.0) yi = 0.0;
    if (e.rylo) yi = fmin(fmax(yi, gin(e.rylo)[i]), gin(e.ryhi)[i]);
    gout(e.YL)[i] = yi;
    double t = __dmul_rn(gin(e.b)[i], yi);
    q[0] = t;
    q[1] = fabs(t);
  }
  double out[2];
  block_reduce<2>(q, 0u, out);
  if (threadIdx.x == 0) {
    e.part_rows[lb] = out[0];
    e.part_rows[(int64_t)e.nblk_rows + lb] = out[1];
  }
}

// Columns, one lane per column: lambda_j = c_j - sum_i a_ij y~_i in the
// stored transpose's (ascending row) order, each product rounded on its
// own, and its rounding error bound err = 2 (k + 2) 2^-53 (|c_j| +
// sum_i |a_ij y~_i|) over the column's k entries.  With |lambda_j| > err (or
// err = 0) its sign is certain and the term is lambda_j times the bound that
// sign selects; otherwise the term is min(lambda_j lo_j, lambda_j hi_j) with
// both bounds finite.  A needed infinite bound is counted.  Partials [0] sum
// of terms, [1] sum of B_j (|c_j| + sum_i |a_ij y~_i|) with B_j the bound
// used (the larger magnitude when both), [2] count of needed infinite bounds.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_bound_cols(const Inst<T> *__restrict__ I,
                                                           Groups g) {
  GROUP_BLOCK(p_cols)
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  double q[3] = {0.0, 0.0, 0.0};
  if (j < e.n) {
    const AS_G int32_t *cp = gin(e.cp), *ri = gin(e.ri);
    const AS_G double *vt = gin(e.vt), *yt = gin((const double *)e.YL);
    const int a = cp[j], z = cp[j + 1];
    double s = 0.0, sa = 0.0;
    for (int k = a; k < z; k++) {
      double pr = __dmul_rn(vt[k], yt[ri[k]]);
      s += pr;
      sa += fabs(pr);
    }
    const double cj = gin(e.c)[j];
    const double lam = cj - s, mag = fabs(cj) + sa;
    const double err = 2.0 * (double)(z - a + 2) * 0x1p-53 * mag;
    double lo = gin(e.l)[j], hi = gin(e.u)[j];
    if (e.ilo) {
      lo = fmax(lo, gin(e.ilo)[j]);
      hi = fmin(hi, gin(e.ihi)[j]);
    }
    if (fabs(lam) > err || err == 0.0) {
      if (lam != 0.0) {
        double bnd = lam > 0.0 ? lo : hi;
        if (isinf(bnd)) {
          q[2] = 1.0;
        } else {
          q[0] = __dmul_rn(lam, bnd);
          q[1] = fabs(bnd) * mag;
        }
      }
    } else if (isinf(lo) || isinf(hi)) {
      q[2] = 1.0;
    } else {
      q[0] = fmin(__dmul_rn(lam, lo), __dmul_rn(lam, hi));
      q[1] = fmax(fabs(lo), fabs(hi)) * mag;
    }
  }
  double out[3];
  block_reduce<3>(q, 0u, out);
  if (threadIdx.x == 0)
    for (int t = 0; t < 3; t++) e.part_cols[(int64_t)t * e.nblk_cols + lb] = out[t];
}

// One workgroup per instance: the partials in fixed order, then
// bound = b'y~ + sum of terms - bound_allow (sum |b_i y~_i| + sum of the
// magnitudes), or -infinity when a needed bound is infinite.
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_bound_finish(const Inst<T> *__restrict__ I) {
  const EvalView<T> &e = I[blockIdx.x].e;
  CtlState *st = I[blockIdx.x].st;
  double r[2], c[3];
  reduce_partials<2, PDHG_BLOCK>(e.part_rows, e.nblk_rows, e.nblk_rows, 0u, r);
  reduce_partials<3, PDHG_BLOCK>(e.part_cols, e.nblk_cols, e.nblk_cols, 0u, c);
  if (threadIdx.x == 0)
    st->dual_bound = c[2] > 0.0 ? -INFINITY : (r[0] + c[0]) - e.bound_allow * (r[1] + c[1]);
}

// Start point: x = proj_[l,u](x0 / Dc) (0 if no x0), y = proj_Y(y0 / Dr).
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_init_cols(const Inst<T> *__restrict__ I, Groups g) {
  GROUP_BLOCK(p_cols)
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (j >= e.n) return;
  const double *x0 = I[inst].x0;
  double xv = x0 ? x0[e.cperm ? e.cperm[j] : j] / e.Dc[j] : 0.0;
  xv = clamp_box<double>(xv, e.l[j], e.u[j]);
  e.X[0][j] = (T)xv;
  e.XL[j] = (double)(T)xv;
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_init_rows(const Inst<T> *__restrict__ I, Groups g) {
  GROUP_BLOCK(p_rows)
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= e.m) return;
  const double *y0 = I[inst].y0;
  double yv = y0 ? y0[e.rperm ? e.rperm[i] : i] / e.Dr[i] : 0.0;
  if (e.kind[i] == 1 && yv < 0.0) yv = 0.0;
  e.Y[0][i] = (T)yv;
  e.YL[i] = (double)(T)yv;
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_ax_to_iter(const Inst<T> *__restrict__ I, Groups g) {
  GROUP_BLOCK(p_rows)
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i < e.m) e.AX[0][i] = (T)e.AXA[i];
}

template <typename T>
__global__ void k_init_state(const Inst<T> *__restrict__ I) {
  CtlState *st = I[blockIdx.x].st;
  st->cur = 0;
  st->fresh = 1;
  st->pending = 0.0;
  st->wsum = 0.0;
  st->k = 0;
  st->accepted = 0;
  st->restarts = 0;
  st->last_restart = 0;
  st->kkt_prev = INFINITY;
  st->kkt_last = INFINITY;
  st->done = 0;
  st->status = 0;
  st->which = 0;
  st->restart_flag = 0;
  st->have_avg = 0;
  st->init_pending = 1;
  st->ticket = 0;
  st->best_kkt = INFINITY;
  st->dual_bound = -INFINITY;  // computed after the solve
  st->stash = 0;
  st->eta = st->eta0;
  st->omega = st->omega0;
}

// FP32 -> FP64 hand-over of the mixed-precision solve: the FP32 phase's
// current iterate becomes the FP64 start point; attempts, accepted steps,
// restarts, the step size and the primal weight carry over, the average and
// the restart reference start afresh.
__global__ __launch_bounds__(PDHG_BLOCK) void k_switch_cols(const Inst<float> *__restrict__ If,
                                                            const Inst<double> *__restrict__ I,
                                                            Groups g) {
  typedef double T;
  GROUP_BLOCK(p_cols)
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (j >= e.n) return;
  (void)If;
  e.XL[j] = e.X[0][j];  // X[0] holds the FP32 phase's best point
}

__global__ __launch_bounds__(PDHG_BLOCK) void k_switch_rows(const Inst<float> *__restrict__ If,
                                                            const Inst<double> *__restrict__ I,
                                                            Groups g) {
  typedef double T;
  GROUP_BLOCK(p_rows)
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= e.m) return;
  (void)If;
  e.YL[i] = e.Y[0][i];  // Y[0] holds the FP32 phase's best point
}

__global__ void k_switch_state(const Inst<double> *__restrict__ I) {
  CtlState *st = I[blockIdx.x].st;
  st->cur = 0;
  st->fresh = 1;
  st->pending = 0.0;
  st->wsum = 0.0;
  st->done = 0;
  st->status = 0;
  st->which = 0;
  st->restart_flag = 0;
  st->kkt_prev = INFINITY;
  st->init_pending = 1;
  st->last_restart = st->k;
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_unscale_cols(const Inst<T> *__restrict__ I,
                                                             Groups g) {
  GROUP_BLOCK(p_cols)
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (j >= e.n) return;
  double xv = st->which ? e.XA[j] : (double)e.X[st->cur][j];
  if (st->status == 6) xv = (double)e.X[st->cur][j] - e.XL[j];  // the ray
  I[inst].xout[e.cperm ? e.cperm[j] : j] = e.Dc[j] * xv;
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_unscale_rows(const Inst<T> *__restrict__ I,
                                                             Groups g) {
  GROUP_BLOCK(p_rows)
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= e.m) return;
  double yv = st->which ? e.YA[i] : (double)e.Y[st->cur][i];
  if (st->status == 5)  // the certificate itself: y as the Farkas test took it
    yv = farkas_y(yv, e.kind[i], I[inst].fyk ? I[inst].fyk[i] : (uint8_t)0);
  I[inst].yout[e.rperm ? e.rperm[i] : i] = e.Dr[i] * yv;
}

// ---------------------------------------------------------------------------
// adjoint of unrolled PDHG
//
// Forward step k (fixed tau, sigma; masks Mx, My of that step):
//   x' = P(x - tau c + tau A'y),  y' = P(y + sigma b - sigma A (2x' - x)).
// Its transpose, applied to the adjoints (xb, yb) of (x', y'):
//   g  = My .* yb                      (rows)
//   t  = A' g,  xb' = xb - 2 sigma t,  h = Mx .* xb'
//   xb <- sigma t + h,  cb -= tau h    (columns)
//   yb <- g + tau A h,  bb += sigma g  (rows)
// Two kernels per step: the column kernel gathers g = My .* yb on the fly.

__device__ inline bool mask_bit(const uint64_t *mask, int64_t i) {
  return (mask[i >> 6] >> (i & 63)) & 1ull;
}

__device__ inline void adj_col(const AdjView &a, int64_t j, double t) {
  double xb = a.XB[j] - 2.0 * a.sigma * t;
  double h = mask_bit(a.mask_x, j) ? xb : 0.0;
  a.XB[j] = a.sigma * t + h;
  a.CB[j] -= a.tau * h;
  a.H[j] = h;
}

__global__ __launch_bounds__(PDHG_BLOCK) void k_adj_cols(AdjView a) {
  int b = blockIdx.x;
  if (b < a.n_long_cols) {
    int64_t j = a.long_cols[b];
    double acc[1] = {0.0};
    for (int k = a.cp[j] + threadIdx.x; k < a.cp[j + 1]; k += PDHG_BLOCK) {
      int64_t i = a.ri[k];
      if (mask_bit(a.mask_y, i)) acc[0] += a.vt[k] * a.YB[i];
    }
    double tot[1];
    block_reduce<1>(acc, 0u, tot);
    if (threadIdx.x == 0) adj_col(a, j, tot[0]);
    return;
  }
  int64_t j = (int64_t)(b - a.n_long_cols) * PDHG_BLOCK + threadIdx.x;
  if (j >= a.n) return;
  int s = a.cp[j], e = a.cp[j + 1];
  if (e - s > a.long_seg) return;
  double t = 0.0;
  for (int k = s; k < e; k++) {
    int64_t i = a.ri[k];
    if (mask_bit(a.mask_y, i)) t += a.vt[k] * a.YB[i];
  }
  adj_col(a, j, t);
}

__device__ inline void adj_row(const AdjView &a, int64_t i, double s) {
  double g = mask_bit(a.mask_y, i) ? a.YB[i] : 0.0;
  a.YB[i] = g + a.tau * s;
  a.BB[i] += a.sigma * g;
}

__global__ __launch_bounds__(PDHG_BLOCK) void k_adj_rows(AdjView a) {
  int b = blockIdx.x;
  if (b < a.n_long_rows) {
    int64_t i = a.long_rows[b];
    double acc[1] = {0.0};
    for (int k = a.rp[i] + threadIdx.x; k < a.rp[i + 1]; k += PDHG_BLOCK) acc[0] += a.v[k] * a.H[a.ci[k]];
    double tot[1];
    block_reduce<1>(acc, 0u, tot);
    if (threadIdx.x == 0) adj_row(a, i, tot[0]);
    return;
  }
  int64_t i = (int64_t)(b - a.n_long_rows) * PDHG_BLOCK + threadIdx.x;
  if (i >= a.m) return;
  int s = a.rp[i], e = a.rp[i + 1];
  if (e - s > a.long_seg) return;
  double acc = 0.0;
  for (int k = s; k < e; k++) acc += a.v[k] * a.H[a.ci[k]];
  adj_row(a, i, acc);
}

__global__ void k_fill_u64(uint64_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_copy_f64(double *__restrict__ d, const double *__restrict__ s, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// y = alpha x + beta y
__global__ void k_axpby(double *y, const double *x, double alpha, double beta, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = alpha * x[i] + beta * y[i];
}

__global__ __launch_bounds__(PDHG_BLOCK) void k_sumsq_partials(const double *x, int64_t n,
                                                               double *part) {
  double q[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * PDHG_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * PDHG_BLOCK)
    q[0] += x[i] * x[i];
  double out[1];
  block_reduce<1>(q, 0u, out);
  if (threadIdx.x == 0) part[blockIdx.x] = out[0];
}

__global__ __launch_bounds__(CTL_BLOCK) void k_sumsq_finish(double *part, int np, double *out) {
  __shared__ double r[1];
  reduce_partials<1>(part, np, 0, 0u, r);
  if (threadIdx.x == 0) *out = r[0];
}

// Save (restore = 0) the current iterate x, y, Ax of each instance, or put a
// saved one back as the current iterate (restore = 1).
template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_checkpoint_cols(const Inst<T> *__restrict__ I,
                                                                Groups g, double *cx,
                                                                int restore) {
  GROUP_BLOCK(p_cols)
  int64_t j = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (j >= e.n) return;
  if (restore)
    e.X[0][j] = (T)cx[j];
  else
    cx[j] = (double)e.X[st->cur][j];
}

template <typename T>
__global__ __launch_bounds__(PDHG_BLOCK) void k_checkpoint_rows(const Inst<T> *__restrict__ I,
                                                                Groups g, double *cy, double *cax,
                                                                int restore) {
  GROUP_BLOCK(p_rows)
  int64_t i = (int64_t)lb * PDHG_BLOCK + threadIdx.x;
  if (i >= e.m) return;
  if (restore) {
    e.Y[0][i] = (T)cy[i];
    e.AX[0][i] = (T)cax[i];
  } else {
    cy[i] = (double)e.Y[st->cur][i];
    cax[i] = (double)e.AX[st->cur][i];
  }
}

template <typename T>
__global__ void k_restore_state(const Inst<T> *__restrict__ I) {
  CtlState *st = I[blockIdx.x].st;
  st->cur = 0;
  st->pending = 0.0;
}

// ---------------------------------------------------------------------------
// setup reductions for the initial step size and primal weight

__global__ __launch_bounds__(PDHG_BLOCK) void k_norm_partials(const double *v, int64_t nnz,
                                                              const double *b, const double *c,
                                                              const double *b0, const double *c0,
                                                              int64_t m, int64_t n,
                                                              double *part, int nparts) {
  // [0] max|v| [1] ||b||^2 [2] ||c||^2 [3] ||b0||^2 [4] ||c0||^2
  double q[5] = {0, 0, 0, 0, 0};
  int64_t stride = (int64_t)gridDim.x * PDHG_BLOCK;
  for (int64_t k = (int64_t)blockIdx.x * PDHG_BLOCK + threadIdx.x; k < nnz; k += stride)
    q[0] = fmax(q[0], fabs(v[k]));
  for (int64_t i = (int64_t)blockIdx.x * PDHG_BLOCK + threadIdx.x; i < m; i += stride) {
    q[1] += b[i] * b[i];
    q[3] += b0[i] * b0[i];
  }
  for (int64_t j = (int64_t)blockIdx.x * PDHG_BLOCK + threadIdx.x; j < n; j += stride) {
    q[2] += c[j] * c[j];
    q[4] += c0[j] * c0[j];
  }
  double out[5];
  block_reduce<5>(q, 1u, out);
  if (threadIdx.x == 0)
    for (int t = 0; t < 5; t++) part[t * nparts + blockIdx.x] = out[t];
}

__global__ __launch_bounds__(CTL_BLOCK) void k_init_ctl(const double *part, int nparts,
                                                        double fixed_eta, double fixed_omega,
                                                        CtlState *st) {
  __shared__ double r[5];
  reduce_partials<5>(part, nparts, nparts, 1u, r);
  if (threadIdx.x != 0) return;
  double amax = r[0], nbs = sqrt(r[1]), ncs = sqrt(r[2]);
  st->nb = sqrt(r[3]);
  st->nc = sqrt(r[4]);
  st->ticket = 0;
  st->eta0 = (fixed_eta > 0.0) ? fixed_eta : (amax > 0.0 ? 1.0 / amax : 1.0);
  if (fixed_omega > 0.0)
    st->omega0 = fixed_omega;
  else
    st->omega0 = (ncs > 1e-10 && nbs > 1e-10) ? ncs / nbs : 1.0;
}

template <typename T>
__global__ void k_gather_states(const Inst<T> *__restrict__ I, int n, CtlState *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *I[i].st;
}

__global__ void k_spmv_plain(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ v, int64_t rows,
                             const double *__restrict__ x, double *__restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double acc = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++) acc += v[k] * x[ci[k]];
  y[i] = acc;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

template <typename T>
void launch_control(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0,
                    hipEvent_t t1) {
  const unsigned grid = grid_of(g.ninst * PDHG_CTL_SPLIT);
  if (t0)
    hipExtLaunchKernelGGL(k_control<T>, dim3(grid), dim3(PDHG_BLOCK), 0, s, t0, t1, 0, I);
  else
    k_control<T><<<grid, PDHG_BLOCK, 0, s>>>(I);
}

template <typename T>
void launch_attempt(const Inst<T> *I, const Groups &g, hipStream_t s) {
  launch_primal<T>(I, g, s);
  launch_dual<T>(I, g, s);
  launch_control<T>(I, g, s);
}

template <typename T>
static void launch_products(const Inst<T> *I, const Groups &g, int mode, hipStream_t s) {
  bool rowsA = (mode == SP_AXA || mode == SP_AX0);
  k_eval_spmv<T><<<grid_of(rowsA ? g.n_rows : g.n_cols), PDHG_BLOCK, 0, s>>>(I, g, mode);
  int nl = rowsA ? g.n_lrows : g.n_lcols;
  if (nl) k_eval_spmv_long<T><<<grid_of(nl), PDHG_BLOCK, 0, s>>>(I, g, mode);
}

template <typename T>
void launch_evaluate(const Inst<T> *I, const Groups &g, double tol, int64_t max_iter,
                     hipStream_t s) {
  k_avg_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
  k_avg_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
  // long rows and columns first (a workgroup each); the row and column
  // kernels compute the other products themselves
  if (g.n_lcols) {
    k_eval_spmv_long<T><<<grid_of(g.n_lcols), PDHG_BLOCK, 0, s>>>(I, g, SP_ATY);
    k_eval_spmv_long<T><<<grid_of(g.n_lcols), PDHG_BLOCK, 0, s>>>(I, g, SP_ATYA);
  }
  if (g.n_lrows) k_eval_spmv_long<T><<<grid_of(g.n_lrows), PDHG_BLOCK, 0, s>>>(I, g, SP_AXA);
  k_eval_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
  k_eval_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
  k_eval_control<T><<<grid_of(g.ninst * PDHG_CTL_SPLIT), PDHG_BLOCK, 0, s>>>(I, tol, (long long)max_iter);
  k_infeas_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
  k_infeas_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
  k_infeas_finish<T><<<grid_of(g.ninst), PDHG_BLOCK, 0, s>>>(I);
  k_restart_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
  k_restart_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
  if (sizeof(T) == 4) {
    k_stash_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
    k_stash_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
  }
}

template <typename T>
void launch_bound(const Inst<T> *I, const Groups &g, hipStream_t s) {
  k_bound_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
  k_bound_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
  k_bound_finish<T><<<grid_of(g.ninst), PDHG_BLOCK, 0, s>>>(I);
}

template <typename T>
void launch_init_point(const Inst<T> *I, const Groups &g, hipStream_t s) {
  k_init_state<T><<<grid_of(g.ninst), 1, 0, s>>>(I);
  k_init_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
  k_init_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
  launch_products<T>(I, g, SP_AX0, s);
  k_ax_to_iter<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
}

void launch_switch_to_fp64(const Inst<float> *If, const Inst<double> *Id, const Groups &g,
                           hipStream_t s) {
  k_switch_cols<<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(If, Id, g);
  k_switch_rows<<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(If, Id, g);
  k_switch_state<<<grid_of(g.ninst), 1, 0, s>>>(Id);
  launch_products<double>(Id, g, SP_AX0, s);
  k_ax_to_iter<double><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(Id, g);
}

template <typename T>
void launch_unscale(const Inst<T> *I, const Groups &g, hipStream_t s) {
  k_unscale_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g);
  k_unscale_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g);
}

void launch_init_ctl(const double *v, int64_t nnz, const double *b, const double *c,
                     const double *b0, const double *c0, int64_t m, int64_t n, double *scratch,
                     int nscratch, CtlState *st, int step_mode, double fixed_eta,
                     double fixed_omega, hipStream_t s) {
  int np = nscratch / 5;
  if (np > 1024) np = 1024;
  (void)step_mode;
  k_norm_partials<<<np, PDHG_BLOCK, 0, s>>>(v, nnz, b, c, b0, c0, m, n, scratch, np);
  k_init_ctl<<<1, CTL_BLOCK, 0, s>>>(scratch, np, fixed_eta, fixed_omega, st);
}

void launch_adjoint_step(const AdjView &a, hipStream_t s) {
  k_adj_cols<<<grid_of(a.n_long_cols + a.nblk_cols), PDHG_BLOCK, 0, s>>>(a);
  k_adj_rows<<<grid_of(a.n_long_rows + a.nblk_rows), PDHG_BLOCK, 0, s>>>(a);
}

void launch_fill_u64(uint64_t *p, int64_t n, hipStream_t s) {
  k_fill_u64<<<grid_for(n), PDHG_BLOCK, 0, s>>>(p, n);
}

void launch_copy_f64(double *dst, const double *src, int64_t n, hipStream_t s) {
  k_copy_f64<<<grid_for(n), PDHG_BLOCK, 0, s>>>(dst, src, n);
}

void launch_axpby(double *y, const double *x, double alpha, double beta, int64_t n,
                  hipStream_t s) {
  k_axpby<<<grid_for(n), PDHG_BLOCK, 0, s>>>(y, x, alpha, beta, n);
}

// ||x||^2 into scratch[nscratch - 1] (device); partials use the rest.
double *launch_sumsq(const double *x, int64_t n, double *scratch, int nscratch, hipStream_t s) {
  int np = nscratch - 1 < 1024 ? nscratch - 1 : 1024;
  k_sumsq_partials<<<np, PDHG_BLOCK, 0, s>>>(x, n, scratch);
  k_sumsq_finish<<<1, CTL_BLOCK, 0, s>>>(scratch, np, scratch + nscratch - 1);
  return scratch + nscratch - 1;
}

template <typename T>
void launch_checkpoint(const Inst<T> *I, const Groups &g, double *cx, double *cy, double *cax,
                       int restore, hipStream_t s) {
  k_checkpoint_cols<T><<<grid_of(g.n_cols), PDHG_BLOCK, 0, s>>>(I, g, cx, restore);
  k_checkpoint_rows<T><<<grid_of(g.n_rows), PDHG_BLOCK, 0, s>>>(I, g, cy, cax, restore);
  if (restore) k_restore_state<T><<<grid_of(g.ninst), 1, 0, s>>>(I);
}

template <typename T>
void launch_gather_states(const Inst<T> *I, int n, CtlState *out, hipStream_t s) {
  k_gather_states<T><<<(n + 63) / 64, 64, 0, s>>>(I, n, out);
}

void launch_spmv(const int32_t *rp, const int32_t *ci, const double *v, int64_t rows,
                 const double *x, double *y, hipStream_t s) {
  k_spmv_plain<<<grid_for(rows), PDHG_BLOCK, 0, s>>>(rp, ci, v, rows, x, y);
}

#define INST(T)                                                                            \
  template void launch_control<T>(const Inst<T> *, const Groups &, hipStream_t, hipEvent_t,   \
                                  hipEvent_t);                                             \
  template void launch_attempt<T>(const Inst<T> *, const Groups &, hipStream_t);           \
  template void launch_evaluate<T>(const Inst<T> *, const Groups &, double, int64_t,       \
                                   hipStream_t);                                           \
  template void launch_init_point<T>(const Inst<T> *, const Groups &, hipStream_t);        \
  template void launch_bound<T>(const Inst<T> *, const Groups &, hipStream_t);             \
  template void launch_unscale<T>(const Inst<T> *, const Groups &, hipStream_t);            \
  template void launch_gather_states<T>(const Inst<T> *, int, CtlState *, hipStream_t);        \
  template void launch_checkpoint<T>(const Inst<T> *, const Groups &, double *, double *,    \
                                     double *, int, hipStream_t);
INST(double)
INST(float)
