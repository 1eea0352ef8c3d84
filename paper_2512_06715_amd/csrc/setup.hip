// One-time preprocessing kernels: validation, bound kinds, transpose,
// power-of-two diagonal scaling.  Everything here is integer work or exact
// floating-point work (comparisons, power-of-two factors), so the results are
// bit-identical to any correct sequential implementation of the same steps.
#include "internal.h"

#include <math.h>

namespace {

inline unsigned grid_for(int64_t n, int per_block = PDHG_BLOCK) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g > 0 ? g : 1);
}

// ---------------------------------------------------------------------------
// validation

__global__ void k_validate_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const double *__restrict__ v, const uint8_t *__restrict__ kind,
                                const double *__restrict__ b, int64_t m, int64_t n, int64_t nnz,
                                int *err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    if (rp[0] != 0 || (int64_t)rp[m] != nnz) atomicOr(err, VERR_CSR);
  }
  if (i >= m) return;
  int bits = 0;
  int64_t s = rp[i], e = rp[i + 1];
  if (s < 0 || e < s || e > nnz) {
    atomicOr(err, VERR_CSR);
    return;
  }
  int32_t prev = -1;
  for (int64_t k = s; k < e; k++) {
    int32_t c = ci[k];
    if (c < 0 || c >= n || c <= prev) bits |= VERR_CSR;
    prev = c;
    if (!isfinite(v[k])) bits |= VERR_NONFINITE;
  }
  if (kind[i] > 1) bits |= VERR_KIND;
  if (!isfinite(b[i])) bits |= VERR_NONFINITE;
  if (bits) atomicOr(err, bits);
}

__global__ void k_validate_cols(const double *__restrict__ c, const double *__restrict__ l,
                                const double *__restrict__ u, int64_t n, int *err) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int bits = 0;
  double lj = l[j], uj = u[j];
  if (isnan(lj) || isnan(uj) || lj > uj || lj == INFINITY || uj == -INFINITY) bits |= VERR_BOUNDS;
  if (!isfinite(c[j])) bits |= VERR_NONFINITE;
  if (bits) atomicOr(err, bits);
}

__global__ void k_var_kind(const double *__restrict__ l, const double *__restrict__ u, int64_t n,
                           uint8_t *__restrict__ vk) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  bool lf = isfinite(l[j]), uf = isfinite(u[j]);
  uint8_t k;
  if (lf && uf)
    k = (l[j] == u[j]) ? VK_FIXED : VK_BOXED;
  else if (lf)
    k = VK_LOWER;
  else if (uf)
    k = VK_UPPER;
  else
    k = VK_FREE;
  vk[j] = k;
}

// ---------------------------------------------------------------------------
// integer helpers

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_copy_i32(int32_t *__restrict__ d, const int32_t *__restrict__ s, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

__global__ void k_fill_f64(double *p, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// A bound vector with its finite entries set to zero (infinite ones kept).
__global__ void k_zero_finite(const double *src, double *dst, int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) dst[j] = isfinite(src[j]) ? 0.0 : src[j];
}

__global__ void k_cast_f32(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (float)s[i];  // round to nearest even
}

// Inclusive scan, level 1: 1024 elements per block (4 per thread).
__global__ void k_scan_blocks(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                              int64_t len, int32_t *__restrict__ totals) {
  __shared__ int32_t lds[PDHG_BLOCK];
  int t = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * (4 * PDHG_BLOCK) + 4 * t;
  int32_t a[4];
  for (int q = 0; q < 4; q++) a[q] = (base + q < len) ? in[base + q] : 0;
  a[1] += a[0];
  a[2] += a[1];
  a[3] += a[2];
  int32_t tsum = a[3];
  lds[t] = tsum;
  __syncthreads();
  for (int off = 1; off < PDHG_BLOCK; off <<= 1) {
    int32_t add = (t >= off) ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int32_t excl = lds[t] - tsum;
  for (int q = 0; q < 4; q++)
    if (base + q < len) out[base + q] = a[q] + excl;
  if (t == PDHG_BLOCK - 1) totals[blockIdx.x] = lds[t];
}

// Level 2: exclusive scan of the block totals by one workgroup, in chunks.
__global__ void k_scan_totals(int32_t *totals, int64_t nt) {
  __shared__ int32_t lds[PDHG_BLOCK];
  __shared__ int32_t carry;
  int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nt; c0 += PDHG_BLOCK) {
    int32_t val = (c0 + t < nt) ? totals[c0 + t] : 0;
    lds[t] = val;
    __syncthreads();
    for (int off = 1; off < PDHG_BLOCK; off <<= 1) {
      int32_t add = (t >= off) ? lds[t - off] : 0;
      __syncthreads();
      lds[t] += add;
      __syncthreads();
    }
    int32_t incl = lds[t];
    if (c0 + t < nt) totals[c0 + t] = carry + incl - val;
    __syncthreads();
    if (t == PDHG_BLOCK - 1) carry += incl;
    __syncthreads();
  }
}

__global__ void k_scan_add(int32_t *__restrict__ out, int64_t len,
                           const int32_t *__restrict__ totals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] += totals[i / (4 * PDHG_BLOCK)];
}

// ---------------------------------------------------------------------------
// transpose

__global__ void k_col_count(const int32_t *__restrict__ ci, int64_t nnz, int32_t *cnt1) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt1[ci[k] + 1], 1);
}

__global__ void k_scatter(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const double *__restrict__ v, int64_t m, int32_t *next,
                          int32_t *__restrict__ ri, double *__restrict__ vt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
    int32_t slot = atomicAdd(&next[ci[k]], 1);
    ri[slot] = (int32_t)i;
    vt[slot] = v[k];
  }
}

// Short columns: insertion sort of (row, value) by row, one thread each.
__global__ void k_sort_short(const int32_t *__restrict__ cp, int64_t n, int32_t *__restrict__ ri,
                             double *__restrict__ vt) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int64_t s = cp[j], e = cp[j + 1];
  if (e - s > PDHG_SORT_SHORT) return;
  for (int64_t a = s + 1; a < e; a++) {
    int32_t key = ri[a];
    double val = vt[a];
    int64_t b = a - 1;
    while (b >= s && ri[b] > key) {
      ri[b + 1] = ri[b];
      vt[b + 1] = vt[b];
      b--;
    }
    ri[b + 1] = key;
    vt[b + 1] = val;
  }
}

// Long columns: one workgroup per column, bitonic network in its all-ascending
// form (the first comparator of each merge stage pairs i with the mirror
// element), so comparisons with partners past the end are skipped and the
// network still sorts a segment of any length in place in global memory.
__global__ void k_sort_long(const int32_t *__restrict__ cp, int64_t n, int32_t *ri, double *vt) {
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    int64_t s = cp[j], e = cp[j + 1];
    int64_t len = e - s;
    if (len <= PDHG_SORT_SHORT) continue;
    int32_t *key = ri + s;
    double *val = vt + s;
    int64_t p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (int64_t blk = 2; blk <= p2; blk <<= 1) {
      for (int64_t d = blk >> 1; d > 0; d >>= 1) {
        for (int64_t i = threadIdx.x; i < p2; i += blockDim.x) {
          int64_t partner;
          if (d == (blk >> 1))
            partner = (i & ~(blk - 1)) + (blk - 1 - (i & (blk - 1)));  // mirror
          else
            partner = i ^ d;
          if (partner > i && partner < len) {
            if (key[i] > key[partner]) {
              int32_t tk = key[i];
              key[i] = key[partner];
              key[partner] = tk;
              double tv = val[i];
              val[i] = val[partner];
              val[partner] = tv;
            }
          }
        }
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// scaling

// Power of two nearest to sqrt(M) on a log scale: with M = nu 2^E,
// nu in [0.5,1), the exponent is floor(E/2).  M = 0 gives 1.
__device__ inline double pow2_sqrt(double M) {
  if (!(M > 0.0)) return 1.0;
  int E;
  frexp(M, &E);
  int k = (E >= 0) ? E / 2 : -((-E + 1) / 2);
  return ldexp(1.0, k);
}

__global__ void k_row_stat(const int32_t *__restrict__ rp, const double *__restrict__ v,
                           int64_t m, int pc, double *__restrict__ rs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double acc = 0.0;
  for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
    double a = fabs(v[k]);
    if (pc)
      acc = acc + a;
    else if (a > acc)
      acc = a;
  }
  rs[i] = pow2_sqrt(acc);
}

__global__ void k_rescale_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               double *__restrict__ v, int64_t m, const double *__restrict__ rs,
                               const double *__restrict__ cs, double *__restrict__ Dr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double r = rs[i];
  for (int64_t k = rp[i]; k < rp[i + 1]; k++) v[k] = v[k] / r / cs[ci[k]];
  Dr[i] = Dr[i] / r;
}

__global__ void k_rescale_cols(const int32_t *__restrict__ cp, const int32_t *__restrict__ ri,
                               double *__restrict__ vt, int64_t n, const double *__restrict__ rs,
                               const double *__restrict__ cs, double *__restrict__ Dc) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = cs[j];
  for (int64_t k = cp[j]; k < cp[j + 1]; k++) vt[k] = vt[k] / rs[ri[k]] / s;
  Dc[j] = Dc[j] / s;
}

__global__ void k_scale_rows_vec(const double *__restrict__ b0, const double *__restrict__ Dr,
                                 int64_t m, double *__restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = Dr[i] * b0[i];
}

__global__ void k_scale_cols_vec(const double *__restrict__ c0, const double *__restrict__ l0,
                                 const double *__restrict__ u0, const double *__restrict__ Dc,
                                 int64_t n, double *__restrict__ c, double *__restrict__ l,
                                 double *__restrict__ u) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double d = Dc[j];
  c[j] = d * c0[j];
  l[j] = l0[j] / d;
  u[j] = u0[j] / d;
}

__global__ void k_fix_bounds(double *l, double *u, const int32_t *__restrict__ idx,
                             const double *__restrict__ val, int64_t nfix,
                             const int32_t *__restrict__ inv, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nfix) return;
  int64_t j = idx[k];
  if (j < 0 || j >= n) return;  // out-of-range fixings are ignored
  if (inv) j = inv[j];
  l[j] = val[k];
  u[j] = val[k];
}

// 16-bit tile-relative structure of a CSR matrix, one workgroup per tile of
// PDHG_TILE rows: rofs[i] = ptr[i + 1] - ptr[r0] (r0 the tile's first row),
// ix16[k] = idx[k] - tb[t], tb[t] = the smallest index of the tile's
// nonzeros.  A tile with more than 65535 nonzeros or an index span above
// 65535 sets *fail and leaves the arrays incomplete.
__global__ __launch_bounds__(PDHG_BLOCK) void k_compact(const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ idx,
                                                        int64_t rows, uint16_t *rofs,
                                                        uint16_t *ix16, int32_t *tb, int *fail) {
  static_assert(PDHG_BLOCK == PDHG_TILE, "one lane per tile row");
  __shared__ int smin[PDHG_BLOCK], smax[PDHG_BLOCK];
  const int64_t t = blockIdx.x, r0 = t * PDHG_TILE;
  const int64_t rend = r0 + PDHG_TILE < rows ? r0 + PDHG_TILE : rows;
  const int base = ptr[r0], top = ptr[rend];
  int mn = 0x7fffffff, mx = -1;
  for (int k = base + (int)threadIdx.x; k < top; k += PDHG_BLOCK) {
    mn = min(mn, idx[k]);
    mx = max(mx, idx[k]);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int h = PDHG_BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + h]);
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + h]);
    }
    __syncthreads();
  }
  mn = top > base ? smin[0] : 0;
  mx = top > base ? smax[0] : 0;
  if (top - base > 65535 || mx - mn > 65535) {
    if (threadIdx.x == 0) atomicOr(fail, 1);
    return;
  }
  if (threadIdx.x == 0) tb[t] = mn;
  for (int k = base + (int)threadIdx.x; k < top; k += PDHG_BLOCK) ix16[k] = (uint16_t)(idx[k] - mn);
  const int64_t i = r0 + threadIdx.x;
  if (i < rend) rofs[i] = (uint16_t)(ptr[i + 1] - base);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

void launch_fix_bounds(double *l, double *u, const int32_t *idx, const double *val, int64_t nfix,
                       const int32_t *inv, int64_t n, hipStream_t s) {
  if (nfix > 0) k_fix_bounds<<<grid_for(nfix), PDHG_BLOCK, 0, s>>>(l, u, idx, val, nfix, inv, n);
}

void launch_validate(const int32_t *rp, const int32_t *ci, const double *v, const uint8_t *kind,
                     const double *b, const double *c, const double *l, const double *u,
                     int64_t m, int64_t n, int64_t nnz, int *err, hipStream_t s) {
  k_validate_rows<<<grid_for(m), PDHG_BLOCK, 0, s>>>(rp, ci, v, kind, b, m, n, nnz, err);
  k_validate_cols<<<grid_for(n), PDHG_BLOCK, 0, s>>>(c, l, u, n, err);
}

void launch_var_kind(const double *l, const double *u, int64_t n, uint8_t *vk, hipStream_t s) {
  k_var_kind<<<grid_for(n), PDHG_BLOCK, 0, s>>>(l, u, n, vk);
}

int64_t scan_tmp_ints(int64_t len) { return (len + 4 * PDHG_BLOCK - 1) / (4 * PDHG_BLOCK) + 1; }

static void inclusive_scan(const int32_t *in, int32_t *out, int64_t len, int32_t *totals,
                           hipStream_t s) {
  int64_t nb = (len + 4 * PDHG_BLOCK - 1) / (4 * PDHG_BLOCK);
  k_scan_blocks<<<(unsigned)nb, PDHG_BLOCK, 0, s>>>(in, out, len, totals);
  k_scan_totals<<<1, PDHG_BLOCK, 0, s>>>(totals, nb);
  k_scan_add<<<grid_for(len), PDHG_BLOCK, 0, s>>>(out, len, totals);
}

void launch_transpose(const int32_t *rp, const int32_t *ci, const double *v, int64_t m, int64_t n,
                      int64_t nnz, int32_t *cp, int32_t *ri, double *vt, int32_t *tmp_next,
                      int32_t *scan_tmp, hipStream_t s) {
  // column counts shifted by one, then an inclusive scan gives the pointers
  k_fill_i32<<<grid_for(n + 1), PDHG_BLOCK, 0, s>>>(tmp_next, 0, n + 1);
  k_col_count<<<grid_for(nnz), PDHG_BLOCK, 0, s>>>(ci, nnz, tmp_next);
  inclusive_scan(tmp_next, cp, n + 1, scan_tmp, s);
  k_copy_i32<<<grid_for(n), PDHG_BLOCK, 0, s>>>(tmp_next, cp, n);
  k_scatter<<<grid_for(m), PDHG_BLOCK, 0, s>>>(rp, ci, v, m, tmp_next, ri, vt);
  k_sort_short<<<grid_for(n), PDHG_BLOCK, 0, s>>>(cp, n, ri, vt);
  k_sort_long<<<1024, PDHG_BLOCK, 0, s>>>(cp, n, ri, vt);
}

void launch_scale_pass(int32_t *rp, int32_t *ci, double *v, int32_t *cp, int32_t *ri, double *vt,
                       int64_t m, int64_t n, int pc, double *rs, double *cs, double *Dr,
                       double *Dc, hipStream_t s) {
  k_row_stat<<<grid_for(m), PDHG_BLOCK, 0, s>>>(rp, v, m, pc, rs);
  k_row_stat<<<grid_for(n), PDHG_BLOCK, 0, s>>>(cp, vt, n, pc, cs);
  k_rescale_rows<<<grid_for(m), PDHG_BLOCK, 0, s>>>(rp, ci, v, m, rs, cs, Dr);
  k_rescale_cols<<<grid_for(n), PDHG_BLOCK, 0, s>>>(cp, ri, vt, n, rs, cs, Dc);
}

void launch_scale_vectors(const double *b0, const double *c0, const double *l0, const double *u0,
                          const double *Dr, const double *Dc, int64_t m, int64_t n, double *b,
                          double *c, double *l, double *u, hipStream_t s) {
  k_scale_rows_vec<<<grid_for(m), PDHG_BLOCK, 0, s>>>(b0, Dr, m, b);
  k_scale_cols_vec<<<grid_for(n), PDHG_BLOCK, 0, s>>>(c0, l0, u0, Dc, n, c, l, u);
}

void launch_compact(const int32_t *ptr, const int32_t *idx, int64_t rows, uint16_t *rofs,
                    uint16_t *ix16, int32_t *tb, int *fail, hipStream_t s) {
  int64_t tiles = (rows + PDHG_TILE - 1) / PDHG_TILE;
  k_compact<<<(unsigned)(tiles > 0 ? tiles : 1), PDHG_BLOCK, 0, s>>>(ptr, idx, rows, rofs, ix16,
                                                                      tb, fail);
}

void launch_fill(double *p, double v, int64_t n, hipStream_t s) {
  k_fill_f64<<<grid_for(n), PDHG_BLOCK, 0, s>>>(p, v, n);
}

void launch_zero_finite(const double *src, double *dst, int64_t n, hipStream_t s) {
  k_zero_finite<<<grid_for(n), PDHG_BLOCK, 0, s>>>(src, dst, n);
}

void launch_copy_i32(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s) {
  k_copy_i32<<<grid_for(n), PDHG_BLOCK, 0, s>>>(dst, src, n);
}

void launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
  k_cast_f32<<<grid_for(n), PDHG_BLOCK, 0, s>>>(src, dst, n);
}
