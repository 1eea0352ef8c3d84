// The two kernels of one PDHG attempt (Chambolle-Pock step of the paper's
// "PDHG Background" section, box projection on x, sign-cone projection on
// >= rows, PDLP adaptive step), each an SpMV with the projection fused:
//   k_primal   x' = proj_[l,u](x - tau (c - A'y))            (row-dot over A')
//   k_dual     y' = proj_Y(y + sigma (b - (2 A x' - A x)))   (row-dot over A,
//              A x' cached for the next attempt)
// Both write per-workgroup partials of the step-size test; the control kernel
// (iterate.hip) reduces them.  Every kernel is grouped: one launch serves all
// instances of a batch.
#include "device.h"

#include <hip/hip_ext.h>

namespace {

// Both kernels walk tiles of PDHG_TILE rows of a CSR matrix (A for the dual
// step, the stored A' for the primal step).  A tile's nonzeros are one
// contiguous range, so the workgroup streams column indices and values with
// consecutive lanes on consecutive nonzeros (coalesced), forms the products
// with the gathered vector into LDS, and each lane then sums its own row from
// LDS in CSR order.  Tiles whose nonzeros do not fit the LDS buffer fall back
// to one lane per row (as does the `direct` partition).  Rows longer than
// `long_seg` get a workgroup each (the first blocks of the instance).  Each
// workgroup covers `tpb` consecutive tiles and writes one partial per reduced
// quantity.

#define TILE_CAP (8 * PDHG_TILE)  // nonzeros of a tile staged in LDS
#define TILE_U 4       // nonzeros per lane loaded before their gathers

// Streams read exactly once per launch: with NT they bypass the cache
// hierarchy's reuse policy so that L2 keeps the gathered vector windows
// (when a launch's bytes exceed the Infinity Cache); without it they are
// ordinary loads, whose lines the Infinity Cache can still hold for the
// next launch (when they fit).
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const AS_G T *p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Iterate stores of the attempt kernels.
template <typename T>
__device__ __forceinline__ void st_out(AS_G T *p, T v) {
  *p = v;
}

// Products are rounded on their own (never fused into the sum), so the
// LDS-staged and the per-row paths give bit-identical row sums.
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }

// The structure of one tile: 32-bit CSR (ptr, idx), or with C the 16-bit
// tile-relative form (row ends `ofs` counted from the tile's first nonzero,
// indices `ix16` counted from the tile's smallest index `tb`).  Row i of the
// tile is lane threadIdx.x.
template <bool C, bool NT>
struct TileIx {
  const AS_G int32_t *ptr, *idx;
  const AS_G uint16_t *ofs, *ix16;
  int tb;
  // index of nonzero k: streamed (read once per launch) or cached
  __device__ __forceinline__ int col_stream(int k) const {
    if constexpr (C)
      return tb + (int)ld_stream<NT>(ix16 + k);
    else
      return ld_stream<NT>(idx + k);
  }
  __device__ __forceinline__ int col(int k) const {
    if constexpr (C)
      return tb + (int)ix16[k];
    else
      return idx[k];
  }
  // nonzero range [rs, re) of this lane's row i; base = the tile's first
  __device__ __forceinline__ void bounds(int64_t i, int base, int &rs, int &re) const {
    if constexpr (C) {
      const bool first = threadIdx.x == 0;
      const int prev = ofs[first ? i : i - 1];  // always an entry of this tile
      re = base + (int)ofs[i];
      rs = first ? base : base + prev;
    } else {
      rs = ptr[i];
      re = ptr[i + 1];
    }
  }
};

// Dot product s = sum_k v[k] x[idx[k]] of this lane's row i (rows r0 + lane of
// a PDHG_TILE-row tile whose nonzeros are [base, top)), summed in CSR order.  The
// row's bounds are loaded here, after the tile's index/value stream has been
// issued, so the gathers wait only on that stream.  `mine` returns whether
// the row is valid and short enough to be this tile's.  Every lane of the
// workgroup must call it.
template <typename T>
struct Pair;
template <>
struct Pair<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

// LDS staging of a tile's products from the 16-bit structure, two nonzeros
// per load: pair p covers entries a0 + 2p and a0 + 2p + 1 with a0 the even
// entry at or below the tile's first, so each lane reads one aligned 32-bit
// word of indices and one aligned pair of values (the index and value arrays
// hold two entries past the last nonzero) and writes both products as one
// aligned LDS pair at slot 2p.  The caller's rows read from lds + (base - a0).
// Entries outside the tile (at most the one before its first and the one
// after its last) gather x at the tile's smallest index, and no row reads
// their slots; lanes past the last pair repeat it and write the same values.
// The lane's row bounds (rs, re) are loaded after the first loads of the
// stream.
template <typename T, typename V, bool NT>
__device__ __forceinline__ void stage_pairs(const TileIx<true, NT> &ix, const AS_G V *v,
                                            const AS_G T *x, int base, int top, T *lds, int64_t i,
                                            bool valid, int &rs, int &re) {
  typedef typename Pair<T>::type T2;
  typedef typename Pair<V>::type V2;
  const int a0 = base & ~1;
  const int npair = (top - a0 + 1) >> 1;
  const AS_G uint32_t *iw = (const AS_G uint32_t *)(ix.ix16 + a0);
  const AS_G V2 *vw = (const AS_G V2 *)(v + a0);
  constexpr int TP = TILE_U / 2;
  for (int p0 = 0; p0 < npair; p0 += TP * PDHG_TILE) {
    uint32_t w[TP];
    V2 vv[TP];
#pragma unroll
    for (int q = 0; q < TP; q++) {
      int p = p0 + q * PDHG_TILE + (int)threadIdx.x;
      int pc = p < npair ? p : npair - 1;
      w[q] = ld_stream<NT>(iw + pc);
      vv[q] = ld_stream<NT>(vw + pc);
    }
    if (p0 == 0 && valid) ix.bounds(i, base, rs, re);
#pragma unroll
    for (int q = 0; q < TP; q++) {
      int p = p0 + q * PDHG_TILE + (int)threadIdx.x;
      int pc = p < npair ? p : npair - 1;
      int e = a0 + 2 * pc;  // absolute entry of the pair's first
      int c0 = e >= base ? ix.tb + (int)(w[q] & 0xffffu) : ix.tb;
      int c1 = e + 1 < top ? ix.tb + (int)(w[q] >> 16) : ix.tb;
      T2 pr;
      pr.x = mul_rn((T)vv[q].x, x[c0]);
      pr.y = mul_rn((T)vv[q].y, x[c1]);
      *(T2 *)(lds + 2 * pc) = pr;
    }
  }
}

template <typename T, typename V, bool C, bool NT>
__device__ __forceinline__ T tile_rowdot(const TileIx<C, NT> &ix, const AS_G V *v, const AS_G T *x,
                                         int64_t i, bool valid, int base, int top, int long_seg,
                                         T *lds, int direct, bool &mine) {
  const int cnt = top - base;
  T s = 0;
  int rs = 0, re = 0;
  if (C && !direct && cnt <= TILE_CAP) {
    const int off = base & 1;  // slot of the tile's first entry
    if constexpr (C) {
      if (cnt > 0)
        stage_pairs<T, V, NT>(ix, v, x, base, top, lds, i, valid, rs, re);
      else if (valid)
        ix.bounds(i, base, rs, re);
    }
    __syncthreads();
    mine = valid && (re - rs <= long_seg);
    if (mine)
      for (int k = rs - base + off; k < re - base + off; k++) s += lds[k];
    __syncthreads();
  } else if (!direct && cnt <= TILE_CAP) {
    for (int k0 = 0; k0 < cnt; k0 += TILE_U * PDHG_TILE) {
      int id[TILE_U];
      V vv[TILE_U];
#pragma unroll
      for (int q = 0; q < TILE_U; q++) {
        int k = k0 + q * PDHG_TILE + (int)threadIdx.x;
        int kc = base + (k < cnt ? k : cnt - 1);
        id[q] = ix.col_stream(kc);
        vv[q] = ld_stream<NT>(v + kc);
      }
      if (k0 == 0 && valid) ix.bounds(i, base, rs, re);
#pragma unroll
      for (int q = 0; q < TILE_U; q++) {
        int k = k0 + q * PDHG_TILE + (int)threadIdx.x;
        // lanes past the tile write a slot of their own past the staged range
        lds[k < cnt ? k : TILE_CAP + (int)threadIdx.x] = mul_rn((T)vv[q], x[id[q]]);
      }
    }
    if (cnt == 0 && valid) ix.bounds(i, base, rs, re);
    __syncthreads();
    mine = valid && (re - rs <= long_seg);
    if (mine)
      for (int k = rs - base; k < re - base; k++) s += lds[k];
    __syncthreads();
  } else {
    if (valid) ix.bounds(i, base, rs, re);
    mine = valid && (re - rs <= long_seg);
    if (mine) {
      for (int k0 = rs; k0 < re; k0 += TILE_U) {
        int id[TILE_U];
        V vv[TILE_U];
#pragma unroll
        for (int q = 0; q < TILE_U; q++) {
          int kc = k0 + q < re ? k0 + q : re - 1;
          id[q] = ix.col(kc);
          vv[q] = v[kc];
        }
#pragma unroll
        for (int q = 0; q < TILE_U; q++) {
          T p = mul_rn((T)vv[q], x[id[q]]);
          if (k0 + q < re) s += p;
        }
      }
    }
  }
  return s;
}

// One long row (a workgroup of its own): FP64 sum of the products.
template <typename T, typename V>
__device__ __forceinline__ double long_rowdot(const AS_G int32_t *idx, const AS_G V *v,
                                              const AS_G T *x, int s, int e) {
  double acc[1] = {0.0};
  for (int k = s + threadIdx.x; k < e; k += PDHG_TILE)
    acc[0] += (double)mul_rn((T)v[k], x[idx[k]]);
  double tot[1];
  block_reduce<1, PDHG_TILE>(acc, 0u, tot);
  return tot[0];
}

// Bit-packed mask of one wave's 64 consecutive rows (tile rows are
// 64-aligned); bits are OR-ed in, so long rows can add theirs separately.
__device__ inline void record_mask(uint64_t *mask, int64_t row0_of_wave, bool bit) {
  uint64_t bits = __ballot(bit);
  if ((threadIdx.x & 63) == 0 && bits) atomicOr((unsigned long long *)&mask[row0_of_wave >> 6],
                                                 (unsigned long long)bits);
}

__device__ inline void record_bit(uint64_t *mask, int64_t row) {
  atomicOr((unsigned long long *)&mask[row >> 6], 1ull << (row & 63));
}

// Folds the previous iterate into the running sum of the average when an
// accepted weight is pending.  It does not depend on the row's product, so
// the tile's workgroup folds every row of the tile, long ones included (in
// the finish step of its own rows, separately for the long ones): every
// element of the sums is read and written by one lane of one workgroup per
// launch, never by the long row's own workgroup.
template <typename T>
__device__ __forceinline__ void fold_sum(AS_G T *sum, int64_t i, T prev, T v, double pend,
                                         int fresh) {
  if (pend > 0.0) st_out(sum + i, (fresh ? (T)0 : prev) + (T)pend * v);
}

// Primal update of column j from t = (A'y)_j; returns whether the pre-clamp
// value lies strictly inside the box.  With xs, also folds x_j into the sum.
template <typename T>
__device__ __forceinline__ bool primal_finish(int64_t j, T t, T tau, T xj, T cj, T lj, T uj,
                                              AS_G T *xn, AS_G T *xs, T xsj, double pend,
                                              int fresh, double &d2) {
  T xt = xj - tau * (cj - t);
  T xv = clamp_box<T>(xt, lj, uj);
  st_out(xn + j, xv);
  double d = (double)xv - (double)xj;
  d2 += d * d;
  if (xs) fold_sum<T>(xs, j, xsj, xj, pend, fresh);
  return xt > lj && xt < uj;
}

// Matrix values the attempt kernels multiply: the iterates' own precision,
// or with FP64 iterates and V = float the FP32 copies, widened exactly (the
// mixed path's FP64 phase).
template <typename V, typename T>
__device__ __forceinline__ const AS_G V *vals(const AS_C IterView<T> &w, bool transpose) {
  if constexpr (sizeof(V) == sizeof(T))
    return gin((const V *)(transpose ? w.vt : w.v));
  else
    return gin(transpose ? w.vt32 : w.v32);
}

// Long column lb of an instance (a workgroup of its own): its row-dot over
// the stored transpose in FP64, then the primal update by lane 0.
template <typename T, typename V>
__device__ __forceinline__ void primal_long(const AS_C IterView<T> &w, const AS_C CtlState *st,
                                            int lb, uint64_t *mask) {
  const int cur = st->cur;
  const T tau = (T)(st->eta / st->omega);
  const AS_G T *x = gin((const T *)w.X[cur]), *y = gin((const T *)w.Y[cur]);
  const AS_G T *c = gin(w.c), *l = gin(w.l), *u = gin(w.u);
  AS_G T *xn = gout(w.X[cur ^ 1]);
  int64_t j = gin(w.long_cols)[lb];
  const AS_C int32_t *cpc = cin(w.cp);
  double t = long_rowdot<T, V>(gin(w.ri), vals<V>(w, true), y, cpc[j], cpc[j + 1]);
  if (threadIdx.x == 0) {
    double dd = 0.0;
    bool in = primal_finish<T>(j, (T)t, tau, x[j], c[j], l[j], u[j], xn, nullptr, (T)0, 0.0, 0, dd);
    gout(w.part_dx2)[lb] = dd;
    if (mask && in) record_bit(mask, j);
  }
}

template <typename T, bool C, bool NT, typename V>
__global__ __launch_bounds__(PDHG_TILE) __attribute__((amdgpu_waves_per_eu(8))) void k_primal(const Inst<T> *__restrict__ I, Groups g) {
  __shared__ __align__(16) T lds[TILE_CAP + PDHG_TILE];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = g.interleave ? b % g.ninst : find_inst_u(g.p_primal, g.ninst, b);
  const int lb = g.interleave ? b / g.ninst : b - cin(g.p_primal)[inst];
  const AS_C IterView<T> &w = cin(I)[inst].w;
  const AS_C CtlState *st = cin(cin(I)[inst].st);
  const int cur = st->cur;
  const T tau = (T)(st->eta / st->omega);
  const double pend = st->pending;
  const int fresh = st->fresh;
  const bool fold_read = pend > 0.0 && !fresh;
  const int64_t n = w.n;
  const AS_G int32_t *cp = gin(w.cp), *ri = gin(w.ri);
  const AS_G V *vt = vals<V>(w, true);
  const AS_G T *c = gin(w.c), *l = gin(w.l), *u = gin(w.u);
  const AS_G T *x = gin((const T *)w.X[cur]), *y = gin((const T *)w.Y[cur]);
  AS_G T *xn = gout(w.X[cur ^ 1]);
  AS_G T *xs = gout(w.XS);
  uint64_t *mask = w.mask_x ? w.mask_x + (st->k - w.mask_k0) * ((n + 63) >> 6) : nullptr;
  double d2[1] = {0.0};
  if (lb < w.n_long_cols) {
    primal_long<T, V>(w, st, lb, mask);
    return;
  }
  const int tpb = w.tpb_cols, long_seg = w.long_seg, direct = w.direct;
  int64_t t0 = (int64_t)(lb - w.n_long_cols) * tpb;
  int64_t ntiles = (n + PDHG_TILE - 1) / PDHG_TILE;
  int64_t t1 = t0 + tpb < ntiles ? t0 + tpb : ntiles;
  const AS_C int32_t *cpc = cin(w.cp);
  for (int64_t t = t0; t < t1; t++) {
    int64_t r0 = t * PDHG_TILE;
    int64_t rend = r0 + PDHG_TILE < n ? r0 + PDHG_TILE : n;
    int64_t j = r0 + threadIdx.x;
    // the column's own loads go out with the tile bounds, before the SpMV
    int base = cpc[r0], top = cpc[rend];
    T xj = 0, cj = 0, lj = 0, uj = 0, xsj = 0;
    if (j < n) {
      xj = x[j];
      cj = ld_stream<NT>(c + j);
      lj = ld_stream<NT>(l + j);
      uj = ld_stream<NT>(u + j);
      if (fold_read) xsj = xs[j];
    }
    const TileIx<C, NT> ix{cp, ri, gin(w.cofs), gin(w.rix16), C ? cin(w.tb_cols)[t] : 0};
    bool mine;
    T s = tile_rowdot<T, V, C, NT>(ix, vt, y, j, j < n, base, top, long_seg, lds, direct, mine);
    bool in = false;
    if (mine)
      in = primal_finish<T>(j, s, tau, xj, cj, lj, uj, xn, xs, xsj, pend, fresh, d2[0]);
    else if (j < n)
      fold_sum<T>(xs, j, xsj, xj, pend, fresh);  // long column
    if (mask) record_mask(mask, j & ~(int64_t)63, in);
  }
  double out[1];
  block_reduce<1, PDHG_TILE>(d2, 0u, out);
  if (threadIdx.x == 0) gout(w.part_dx2)[lb] = out[0];
}

// Dual update of row i from s = (A x')_i; returns whether the dual is
// unprojected (equality row or value > 0).
template <typename T>
__device__ __forceinline__ bool dual_finish(int64_t i, T s, T sigma, T yi, T axi, T bi, uint8_t ki,
                                            AS_G T *yn, AS_G T *axn, AS_G T *ys, T ysi,
                                            double pend, int fresh, double &dy2, double &inter) {
  T yv = yi + sigma * (bi - (s + s - axi));
  bool in = (ki == 0) || (yv > (T)0);
  if (ki == 1 && yv < (T)0) yv = (T)0;
  st_out(yn + i, yv);
  st_out(axn + i, s);
  double dy = (double)yv - (double)yi;
  dy2 += dy * dy;
  inter += dy * ((double)s - (double)axi);
  if (ys) fold_sum<T>(ys, i, ysi, yi, pend, fresh);
  return in;
}

// Long row lb of an instance: its row-dot over A in FP64, then the dual
// update by lane 0.
template <typename T, typename V>
__device__ __forceinline__ void dual_long(const AS_C IterView<T> &w, const AS_C CtlState *st,
                                          int lb, uint64_t *mask) {
  const int cur = st->cur;
  const T sigma = (T)(st->eta * st->omega);
  const AS_G T *xn = gin((const T *)w.X[cur ^ 1]);
  const AS_G T *y = gin((const T *)w.Y[cur]), *ax = gin((const T *)w.AX[cur]), *bb = gin(w.b);
  AS_G T *yn = gout(w.Y[cur ^ 1]), *axn = gout(w.AX[cur ^ 1]);
  int64_t i = gin(w.long_rows)[lb];
  const AS_C int32_t *rpc = cin(w.rp);
  double t = long_rowdot<T, V>(gin(w.ci), vals<V>(w, false), xn, rpc[i], rpc[i + 1]);
  if (threadIdx.x == 0) {
    double acc[2] = {0.0, 0.0};
    bool in = dual_finish<T>(i, (T)t, sigma, y[i], ax[i], bb[i], gin(w.kind)[i], yn, axn, nullptr,
                             (T)0, 0.0, 0, acc[0], acc[1]);
    gout(w.part_dy)[lb] = acc[0];
    gout(w.part_dy)[w.grid_rows + lb] = acc[1];
    if (mask && in) record_bit(mask, i);
  }
}

template <typename T, bool C, bool NT, typename V>
__global__ __launch_bounds__(PDHG_TILE) __attribute__((amdgpu_waves_per_eu(8))) void k_dual(const Inst<T> *__restrict__ I, Groups g) {
  __shared__ __align__(16) T lds[TILE_CAP + PDHG_TILE];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = g.interleave ? b % g.ninst : find_inst_u(g.p_dual, g.ninst, b);
  const int lb = g.interleave ? b / g.ninst : b - cin(g.p_dual)[inst];
  const AS_C IterView<T> &w = cin(I)[inst].w;
  const AS_C CtlState *st = cin(cin(I)[inst].st);
  const int cur = st->cur;
  const T sigma = (T)(st->eta * st->omega);
  const double pend = st->pending;
  const int fresh = st->fresh;
  const bool fold_read = pend > 0.0 && !fresh;
  const int64_t m = w.m;
  const AS_G int32_t *rp = gin(w.rp), *ci = gin(w.ci);
  const AS_G V *v = vals<V>(w, false);
  const AS_G T *bb = gin(w.b);
  const AS_G uint8_t *kind = gin(w.kind);
  const AS_G T *xn = gin((const T *)w.X[cur ^ 1]);
  const AS_G T *y = gin((const T *)w.Y[cur]), *ax = gin((const T *)w.AX[cur]);
  AS_G T *yn = gout(w.Y[cur ^ 1]), *axn = gout(w.AX[cur ^ 1]), *ys = gout(w.YS);
  uint64_t *mask = w.mask_y ? w.mask_y + (st->k - w.mask_k0) * ((m + 63) >> 6) : nullptr;
  const int64_t G = w.grid_rows;
  double acc[2] = {0.0, 0.0};
  if (lb < w.n_long_rows) {
    dual_long<T, V>(w, st, lb, mask);
    return;
  }
  const int tpb = w.tpb_rows, long_seg = w.long_seg, direct = w.direct;
  int64_t t0 = (int64_t)(lb - w.n_long_rows) * tpb;
  int64_t ntiles = (m + PDHG_TILE - 1) / PDHG_TILE;
  int64_t t1 = t0 + tpb < ntiles ? t0 + tpb : ntiles;
  const AS_C int32_t *rpc = cin(w.rp);
  for (int64_t t = t0; t < t1; t++) {
    int64_t r0 = t * PDHG_TILE;
    int64_t rend = r0 + PDHG_TILE < m ? r0 + PDHG_TILE : m;
    int64_t i = r0 + threadIdx.x;
    int base = rpc[r0], top = rpc[rend];
    T yi = 0, axi = 0, bi = 0, ysi = 0;
    uint8_t ki = 0;
    if (i < m) {
      yi = y[i];
      axi = ax[i];
      bi = ld_stream<NT>(bb + i);
      ki = kind[i];
      if (fold_read) ysi = ys[i];
    }
    const TileIx<C, NT> ix{rp, ci, gin(w.rofs), gin(w.cix16), C ? cin(w.tb_rows)[t] : 0};
    bool mine;
    T s = tile_rowdot<T, V, C, NT>(ix, v, xn, i, i < m, base, top, long_seg, lds, direct, mine);
    bool in = false;
    if (mine)
      in = dual_finish<T>(i, s, sigma, yi, axi, bi, ki, yn, axn, ys, ysi, pend, fresh, acc[0],
                          acc[1]);
    else if (i < m)
      fold_sum<T>(ys, i, ysi, yi, pend, fresh);  // long row
    if (mask) record_mask(mask, i & ~(int64_t)63, in);
  }
  double out[2];
  block_reduce<2, PDHG_TILE>(acc, 0u, out);
  if (threadIdx.x == 0) {
    gout(w.part_dy)[lb] = out[0];
    gout(w.part_dy)[G + lb] = out[1];
  }
}

// ---------------------------------------------------------------------------
// Multi-instance tiles: instances that share one matrix (branch-and-bound
// variants of one LP, g.pack > 0) are walked NB at a time.  A workgroup
// applies one tile of the shared matrix to a pack of NB instances: the
// tile's 16-bit indices and values are staged in LDS once, then each lane
// walks its own row in CSR order, four entries at a time, gathering the pack's
// NB vectors together (4 NB independent loads in flight per lane).  Each
// product is rounded on its own and the row sum starts at zero and adds them
// in CSR order, as in the single-instance kernels, so every instance gets
// the same bits either way.  Long rows and columns keep a workgroup per
// instance (the first n_long * ninst blocks); the tiles follow tile-major,
// the packs of one tile next to each other on one XCD.

// Stage the raw structure of a tile (indices relative to its smallest one,
// values) in LDS, two entries per load as in stage_pairs; entry e of the
// tile sits at slot e - a0, a0 = base & ~1.
template <typename T>
__device__ __forceinline__ void stage_structure(const AS_G uint16_t *ix16, const AS_G T *v,
                                                int base, int top, uint16_t *sidx, T *sval) {
  typedef typename Pair<T>::type T2;
  const int a0 = base & ~1;
  const int npair = (top - a0 + 1) >> 1;
  const AS_G uint32_t *iw = (const AS_G uint32_t *)(ix16 + a0);
  const AS_G T2 *vw = (const AS_G T2 *)(v + a0);
  constexpr int TP = TILE_U / 2;
  for (int p0 = 0; p0 < npair; p0 += TP * PDHG_TILE) {
    uint32_t w[TP];
    T2 vv[TP];
#pragma unroll
    for (int q = 0; q < TP; q++) {
      int p = p0 + q * PDHG_TILE + (int)threadIdx.x;
      int pc = p < npair ? p : npair - 1;
      w[q] = ld_stream<true>(iw + pc);
      vv[q] = ld_stream<true>(vw + pc);
    }
#pragma unroll
    for (int q = 0; q < TP; q++) {
      int p = p0 + q * PDHG_TILE + (int)threadIdx.x;
      int pc = p < npair ? p : npair - 1;
      *(uint32_t *)(sidx + 2 * pc) = w[q];
      *(T2 *)(sval + 2 * pc) = vv[q];
    }
  }
}

// Row sums s[q] = sum_k v[k] x_q[idx[k]] of this lane's row (entries [rs, re)
// of the tile staged from a0) for the pack's instances q < nq, in CSR order.
// Without staging (a tile past the LDS buffer) the entries come from global
// memory.
template <typename T, int NB>
__device__ __forceinline__ void pack_rowdot(const uint16_t *sidx, const T *sval, bool staged,
                                            const AS_G uint16_t *ix16, const AS_G T *v, int tb,
                                            int a0, int rs, int re, const AS_G T *const (&x)[NB],
                                            int nq, T (&s)[NB]) {
#pragma unroll
  for (int q = 0; q < NB; q++) s[q] = 0;
  for (int k0 = rs; k0 < re; k0 += TILE_U) {
    int id[TILE_U];
    T vv[TILE_U];
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      int k = k0 + u < re ? k0 + u : re - 1;
      id[u] = tb + (int)(staged ? sidx[k - a0] : ix16[k]);
      vv[u] = staged ? sval[k - a0] : v[k];
    }
    T gx[TILE_U][NB];
#pragma unroll
    for (int u = 0; u < TILE_U; u++)
#pragma unroll
      for (int q = 0; q < NB; q++) gx[u][q] = q < nq ? x[q][id[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < TILE_U; u++)
      if (k0 + u < re) {
#pragma unroll
        for (int q = 0; q < NB; q++) s[q] += mul_rn(vv[u], gx[u][q]);
      }
  }
}

template <typename T, int NB>
__global__ __launch_bounds__(PDHG_TILE) void k_primal_pack(const Inst<T> *__restrict__ I, Groups g) {
  __shared__ __align__(16) uint16_t sidx[TILE_CAP + 4];
  __shared__ __align__(16) T sval[TILE_CAP + 4];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const AS_C IterView<T> &w0 = cin(I)[0].w;  // the shared matrix and partition
  const int nlong = w0.n_long_cols;
  if (b < nlong * g.ninst) {
    const int inst = b % g.ninst;
    primal_long<T, T>(cin(I)[inst].w, cin(cin(I)[inst].st), b / g.ninst, nullptr);
    return;
  }
  const int npk = (g.ninst + NB - 1) / NB;
  const int tb_ = b - nlong * g.ninst;
  const int64_t t = tb_ / npk;
  const int q0 = (tb_ % npk) * NB;
  const int nq = g.ninst - q0 < NB ? g.ninst - q0 : NB;
  const int64_t n = w0.n;
  const int64_t r0 = t * PDHG_TILE;
  const int64_t rend = r0 + PDHG_TILE < n ? r0 + PDHG_TILE : n;
  const int64_t j = r0 + threadIdx.x;
  const bool valid = j < n;
  const AS_C int32_t *cpc = cin(w0.cp);
  const int base = cpc[r0], top = cpc[rend];
  const int tbase = cin(w0.tb_cols)[t];
  // the pack's step sizes, iterates and the column's own values
  T tau[NB], xj[NB], cj[NB], lj[NB], uj[NB], xsj[NB];
  const AS_G T *y[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) {
    xj[q] = cj[q] = lj[q] = uj[q] = xsj[q] = 0;
    tau[q] = 0;
    y[q] = nullptr;
    if (q < nq) {
      const AS_C IterView<T> &w = cin(I)[q0 + q].w;
      const AS_C CtlState *st = cin(cin(I)[q0 + q].st);
      const int cur = st->cur;
      tau[q] = (T)(st->eta / st->omega);
      y[q] = gin((const T *)w.Y[cur]);
      if (valid) {
        xj[q] = gin((const T *)w.X[cur])[j];
        cj[q] = ld_stream<true>(gin(w.c) + j);
        lj[q] = ld_stream<true>(gin(w.l) + j);
        uj[q] = ld_stream<true>(gin(w.u) + j);
        if (st->pending > 0.0 && !st->fresh) xsj[q] = gin((const T *)w.XS)[j];
      }
    }
  }
  const bool staged = top - base <= TILE_CAP;
  if (staged && top > base) stage_structure<T>(gin(w0.rix16), gin(w0.vt), base, top, sidx, sval);
  int rs = 0, re = 0;
  if (valid) {
    const TileIx<true, true> ix{nullptr, nullptr, gin(w0.cofs), gin(w0.rix16), tbase};
    ix.bounds(j, base, rs, re);
  }
  __syncthreads();
  const bool mine = valid && (re - rs <= w0.long_seg);
  T sum[NB];
  pack_rowdot<T, NB>(sidx, sval, staged, gin(w0.rix16), gin(w0.vt), tbase, base & ~1, rs,
                     mine ? re : rs, y, nq, sum);
  double d2[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) {
    d2[q] = 0.0;
    if (q < nq && valid) {
      const AS_C IterView<T> &w = cin(I)[q0 + q].w;
      const AS_C CtlState *st = cin(cin(I)[q0 + q].st);
      const int cur = st->cur;
      AS_G T *xn = gout(w.X[cur ^ 1]);
      AS_G T *xs = gout(w.XS);
      if (mine)
        primal_finish<T>(j, sum[q], tau[q], xj[q], cj[q], lj[q], uj[q], xn, xs, xsj[q],
                         st->pending, st->fresh, d2[q]);
      else
        fold_sum<T>(xs, j, xsj[q], xj[q], st->pending, st->fresh);  // long column
    }
  }
  double out[NB];
  block_reduce<NB, PDHG_TILE>(d2, 0u, out);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NB; q++)
      if (q < nq) gout(cin(I)[q0 + q].w.part_dx2)[nlong + t] = out[q];
}

template <typename T, int NB>
__global__ __launch_bounds__(PDHG_TILE) void k_dual_pack(const Inst<T> *__restrict__ I, Groups g) {
  __shared__ __align__(16) uint16_t sidx[TILE_CAP + 4];
  __shared__ __align__(16) T sval[TILE_CAP + 4];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const AS_C IterView<T> &w0 = cin(I)[0].w;
  const int nlong = w0.n_long_rows;
  if (b < nlong * g.ninst) {
    const int inst = b % g.ninst;
    dual_long<T, T>(cin(I)[inst].w, cin(cin(I)[inst].st), b / g.ninst, nullptr);
    return;
  }
  const int npk = (g.ninst + NB - 1) / NB;
  const int tb_ = b - nlong * g.ninst;
  const int64_t t = tb_ / npk;
  const int q0 = (tb_ % npk) * NB;
  const int nq = g.ninst - q0 < NB ? g.ninst - q0 : NB;
  const int64_t m = w0.m;
  const int64_t r0 = t * PDHG_TILE;
  const int64_t rend = r0 + PDHG_TILE < m ? r0 + PDHG_TILE : m;
  const int64_t i = r0 + threadIdx.x;
  const bool valid = i < m;
  const AS_C int32_t *rpc = cin(w0.rp);
  const int base = rpc[r0], top = rpc[rend];
  const int tbase = cin(w0.tb_rows)[t];
  T yi[NB], axi[NB], bi[NB], ysi[NB];
  uint8_t ki = 0;
  const AS_G T *xn[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) {
    yi[q] = axi[q] = bi[q] = ysi[q] = 0;
    xn[q] = nullptr;
    if (q < nq) {
      const AS_C IterView<T> &w = cin(I)[q0 + q].w;
      const AS_C CtlState *st = cin(cin(I)[q0 + q].st);
      const int cur = st->cur;
      xn[q] = gin((const T *)w.X[cur ^ 1]);
      if (valid) {
        yi[q] = gin((const T *)w.Y[cur])[i];
        axi[q] = gin((const T *)w.AX[cur])[i];
        bi[q] = ld_stream<true>(gin(w.b) + i);
        if (st->pending > 0.0 && !st->fresh) ysi[q] = gin((const T *)w.YS)[i];
      }
    }
  }
  if (valid) ki = gin(w0.kind)[i];
  const bool staged = top - base <= TILE_CAP;
  if (staged && top > base) stage_structure<T>(gin(w0.cix16), gin(w0.v), base, top, sidx, sval);
  int rs = 0, re = 0;
  if (valid) {
    const TileIx<true, true> ix{nullptr, nullptr, gin(w0.rofs), gin(w0.cix16), tbase};
    ix.bounds(i, base, rs, re);
  }
  __syncthreads();
  const bool mine = valid && (re - rs <= w0.long_seg);
  T sum[NB];
  pack_rowdot<T, NB>(sidx, sval, staged, gin(w0.cix16), gin(w0.v), tbase, base & ~1, rs,
                     mine ? re : rs, xn, nq, sum);
  double acc[2 * NB];
#pragma unroll
  for (int q = 0; q < NB; q++) {
    acc[2 * q] = acc[2 * q + 1] = 0.0;
    if (q < nq && valid) {
      const AS_C IterView<T> &w = cin(I)[q0 + q].w;
      const AS_C CtlState *st = cin(cin(I)[q0 + q].st);
      const int cur = st->cur;
      const T sigma = (T)(st->eta * st->omega);
      AS_G T *yn = gout(w.Y[cur ^ 1]), *axn = gout(w.AX[cur ^ 1]), *ys = gout(w.YS);
      if (mine)
        dual_finish<T>(i, sum[q], sigma, yi[q], axi[q], bi[q], ki, yn, axn, ys, ysi[q],
                       st->pending, st->fresh, acc[2 * q], acc[2 * q + 1]);
      else
        fold_sum<T>(ys, i, ysi[q], yi[q], st->pending, st->fresh);  // long row
    }
  }
  double out[2 * NB];
  block_reduce<2 * NB, PDHG_TILE>(acc, 0u, out);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NB; q++)
      if (q < nq) {
        const AS_C IterView<T> &w = cin(I)[q0 + q].w;
        gout(w.part_dy)[nlong + t] = out[2 * q];
        gout(w.part_dy)[w.grid_rows + nlong + t] = out[2 * q + 1];
      }
}

}  // namespace

// With events, the kernel is launched through hipExtLaunchKernelGGL, whose
// start/stop events take the dispatch's own timestamps (the kernel's
// duration, without launch gaps).
template <typename T, bool C, bool NT, typename V>
void launch_primal_v(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0,
                     hipEvent_t t1) {
  if (t0)
    hipExtLaunchKernelGGL(k_primal<T, C, NT, V>, dim3(grid_of(g.n_primal)), dim3(PDHG_TILE), 0, s,
                          t0, t1, 0, I, g);
  else
    k_primal<T, C, NT, V><<<grid_of(g.n_primal), PDHG_TILE, 0, s>>>(I, g);
}

// FP64 iterates on the FP32 matrix values when the group asks for them
template <typename T, bool C, bool NT>
void launch_primal_as(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0,
                      hipEvent_t t1) {
  if (sizeof(T) == 8 && g.v32)
    launch_primal_v<T, C, NT, float>(I, g, s, t0, t1);
  else
    launch_primal_v<T, C, NT, T>(I, g, s, t0, t1);
}

template <typename T, bool C, bool NT, typename V>
void launch_dual_v(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0,
                   hipEvent_t t1) {
  if (t0)
    hipExtLaunchKernelGGL(k_dual<T, C, NT, V>, dim3(grid_of(g.n_dual)), dim3(PDHG_TILE), 0, s, t0,
                          t1, 0, I, g);
  else
    k_dual<T, C, NT, V><<<grid_of(g.n_dual), PDHG_TILE, 0, s>>>(I, g);
}

template <typename T, bool C, bool NT>
void launch_dual_as(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0,
                    hipEvent_t t1) {
  if (sizeof(T) == 8 && g.v32)
    launch_dual_v<T, C, NT, float>(I, g, s, t0, t1);
  else
    launch_dual_v<T, C, NT, T>(I, g, s, t0, t1);
}

template <typename T>
void launch_primal(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0,
                   hipEvent_t t1) {
  if (g.pack) {
    if (t0)
      hipExtLaunchKernelGGL(k_primal_pack<T, PDHG_PACK>, dim3(grid_of(g.n_primal_pack)),
                            dim3(PDHG_TILE), 0, s, t0, t1, 0, I, g);
    else
      k_primal_pack<T, PDHG_PACK><<<grid_of(g.n_primal_pack), PDHG_TILE, 0, s>>>(I, g);
    return;
  }
  if (g.compact)
    g.nt ? launch_primal_as<T, true, true>(I, g, s, t0, t1)
         : launch_primal_as<T, true, false>(I, g, s, t0, t1);
  else
    g.nt ? launch_primal_as<T, false, true>(I, g, s, t0, t1)
         : launch_primal_as<T, false, false>(I, g, s, t0, t1);
}

template <typename T>
void launch_dual(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (g.pack) {
    if (t0)
      hipExtLaunchKernelGGL(k_dual_pack<T, PDHG_PACK>, dim3(grid_of(g.n_dual_pack)),
                            dim3(PDHG_TILE), 0, s, t0, t1, 0, I, g);
    else
      k_dual_pack<T, PDHG_PACK><<<grid_of(g.n_dual_pack), PDHG_TILE, 0, s>>>(I, g);
    return;
  }
  if (g.compact)
    g.nt ? launch_dual_as<T, true, true>(I, g, s, t0, t1)
         : launch_dual_as<T, true, false>(I, g, s, t0, t1);
  else
    g.nt ? launch_dual_as<T, false, true>(I, g, s, t0, t1)
         : launch_dual_as<T, false, false>(I, g, s, t0, t1);
}

#define INST(T)                                                                             \
  template void launch_primal<T>(const Inst<T> *, const Groups &, hipStream_t, hipEvent_t,    \
                                 hipEvent_t);                                              \
  template void launch_dual<T>(const Inst<T> *, const Groups &, hipStream_t, hipEvent_t,      \
                               hipEvent_t);
INST(double)
INST(float)
