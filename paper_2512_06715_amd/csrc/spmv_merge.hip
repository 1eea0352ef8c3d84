// Merge-path CSR SpMV, y = A x: the load-balanced alternative to the
// row-split tiles of the attempt kernels.  The rows' ends and the nonzeros
// form one merged sequence of m + nnz items; every workgroup takes an equal
// share of it (MP_ITEMS items) and every lane an equal share of that
// (MP_IPT items), whatever the row lengths, so a long row is split between
// lanes and workgroups instead of getting a workgroup of its own.
//
// A plan kernel finds once per matrix structure where each workgroup's
// share starts (a binary search on the merge path per workgroup).  The SpMV
// kernel stages its share's products and row ends in LDS, each lane walks
// its items (a binary search in LDS for its start), and a lane's partial
// sum of a row that began before it is completed from the earlier lanes'
// carries in lane order; a row that began in an earlier workgroup gets that
// workgroup's carry from a short fix-up kernel.  No atomics: the sums of a
// row are added in a fixed order, so repeated runs give the same bits.
#include "device.h"

#include <hip/hip_runtime.h>

namespace {

#define MP_THREADS 256
#define MP_IPT 8
#define MP_ITEMS (MP_THREADS * MP_IPT)

__device__ __forceinline__ double mp_mul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float mp_mul(float a, float b) { return __fmul_rn(a, b); }

// Rows ended before diagonal d of the merge path of the row ends re[0, m)
// and the nonzero indices 0 .. nnz-1: the largest i with re[i-1] <= d - i
// (a row end goes first when no nonzero of its row remains).
__device__ int64_t merge_split(const int32_t *re, int64_t m, int64_t nnz, int64_t d) {
  int64_t lo = d - nnz > 0 ? d - nnz : 0, hi = d < m ? d : m;
  while (lo < hi) {
    int64_t p = (lo + hi) >> 1;
    if ((int64_t)re[p] <= d - p - 1)
      lo = p + 1;
    else
      hi = p;
  }
  return lo;
}

// CSR structure check of the plan: row_ptr[0] = 0, nondecreasing, row_ptr[m]
// = nnz, column indices in [0, n).  Any violation sets *bad.
__global__ void k_merge_check(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              int64_t m, int64_t n, int64_t nnz, int *bad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool odd = false;
  if (t == 0) odd = rp[0] != 0 || (int64_t)rp[m] != nnz;
  if (t < m) odd = odd || rp[t + 1] < rp[t];
  if (t < nnz) odd = odd || ci[t] < 0 || (int64_t)ci[t] >= n;
  if (odd) *bad = 1;
}

// start[w] = rows ended before workgroup w's first item, w = 0 .. nwg.
__global__ void k_merge_plan(const int32_t *__restrict__ rp, int64_t m, int64_t nnz, int nwg,
                             int32_t *start) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w > nwg) return;
  int64_t d = (int64_t)w * MP_ITEMS;
  if (d > m + nnz) d = m + nnz;
  start[w] = (int32_t)merge_split(rp + 1, m, nnz, d);
}

template <typename T>
__global__ __launch_bounds__(MP_THREADS) void k_spmv_merge(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const T *__restrict__ v,
    const T *__restrict__ x, T *__restrict__ y, int64_t m, int64_t nnz,
    const int32_t *__restrict__ start, int32_t *carry_row, T *carry_val) {
  __shared__ T s_prod[MP_ITEMS];
  __shared__ int32_t s_re[MP_ITEMS];
  __shared__ int32_t s_crow[MP_THREADS];
  __shared__ T s_cval[MP_THREADS];
  const int w = blockIdx.x;
  const int64_t d0 = (int64_t)w * MP_ITEMS;
  const int64_t d1 = d0 + MP_ITEMS < m + nnz ? d0 + MP_ITEMS : m + nnz;
  const int64_t i0 = start[w], i1 = start[w + 1];
  const int64_t k0 = d0 - i0, k1 = d1 - i1;
  const int nrow = (int)(i1 - i0), nk = (int)(k1 - k0);
  const int tid = threadIdx.x;
  // the share's products (consecutive lanes on consecutive nonzeros) and row ends
  for (int q0 = 0; q0 < nk; q0 += 4 * MP_THREADS) {
    int id[4];
    T vv[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      int q = q0 + u * MP_THREADS + tid;
      int qc = q < nk ? q : nk - 1;
      id[u] = ci[k0 + qc];
      vv[u] = v[k0 + qc];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      int q = q0 + u * MP_THREADS + tid;
      if (q < nk) s_prod[q] = mp_mul(vv[u], x[id[u]]);
    }
  }
  for (int q = tid; q < nrow; q += MP_THREADS) s_re[q] = rp[i0 + 1 + q] - (int32_t)k0;
  __syncthreads();
  // this lane's items [dt, de) of the share, starting at local row ti, nonzero tk
  const int len = (int)(d1 - d0);
  const int dt = tid * MP_IPT < len ? tid * MP_IPT : len;
  const int de = dt + MP_IPT < len ? dt + MP_IPT : len;
  int lo = dt - nk > 0 ? dt - nk : 0, hi = dt < nrow ? dt : nrow;
  while (lo < hi) {
    int p = (lo + hi) >> 1;
    if (s_re[p] <= dt - p - 1)
      lo = p + 1;
    else
      hi = p;
  }
  int ti = lo, tk = dt - lo;
  T sum = 0, first_val = 0;
  int first_row = -1;
#pragma unroll
  for (int q = 0; q < MP_IPT; q++) {
    if (dt + q < de) {
      if (ti < nrow && s_re[ti] <= tk) {  // the end of row ti
        if (first_row < 0) {
          first_row = ti;
          first_val = sum;
        } else {
          y[i0 + ti] = sum;  // the row began in this lane
        }
        sum = 0;
        ti++;
      } else {
        sum += s_prod[tk];
        tk++;
      }
    }
  }
  s_crow[tid] = ti;  // the row this lane stops in, with its partial sum
  s_cval[tid] = sum;
  __syncthreads();
  if (first_row >= 0) {
    // earlier lanes that stopped in this row hold its beginning: add their
    // partial sums in lane order, then this lane's
    int t = tid - 1;
    while (t >= 0 && s_crow[t] == first_row) t--;
    T tot = 0;
    for (int u = t + 1; u < tid; u++) tot += s_cval[u];
    y[i0 + first_row] = tot + first_val;
  }
  if (tid == MP_THREADS - 1) {
    // every lane ends at or before the share's end, where row i1 is current:
    // the lanes that stopped in row i1 hold its part in this workgroup
    int t = MP_THREADS - 1;
    while (t >= 0 && s_crow[t] == nrow) t--;
    T tot = 0;
    for (int u = t + 1; u < MP_THREADS; u++) tot += s_cval[u];
    carry_row[w] = (int32_t)i1;
    carry_val[w] = tot;
  }
}

// Rows that span workgroups: the first workgroup of each run of equal carry
// rows adds the run's carries, in workgroup order, to the value the row's
// last workgroup wrote.
template <typename T>
__global__ void k_spmv_merge_fix(const int32_t *__restrict__ carry_row,
                                 const T *__restrict__ carry_val, int nwg, int64_t m, T *y) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwg) return;
  const int32_t r = carry_row[w];
  if (r >= m || (w > 0 && carry_row[w - 1] == r)) return;
  T tot = 0;
  for (int u = w; u < nwg && carry_row[u] == r; u++) tot += carry_val[u];
  y[r] = y[r] + tot;
}

}  // namespace

int merge_workgroups(int64_t m, int64_t nnz) { return (int)((m + nnz + MP_ITEMS - 1) / MP_ITEMS); }

size_t merge_workspace_bytes(int64_t m, int64_t nnz) {
  const size_t nwg = (size_t)merge_workgroups(m, nnz);
  // start[nwg + 1], carry_row[nwg], carry_val[nwg] (8 bytes each), 256-byte aligned
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return up(4 * (nwg + 1)) + up(4 * nwg) + up(8 * nwg);
}

void launch_merge_check(const int32_t *rp, const int32_t *ci, int64_t m, int64_t n, int64_t nnz,
                        int *bad, hipStream_t s) {
  const int64_t len = (m > nnz ? m : nnz) + 1;
  k_merge_check<<<grid_for(len), PDHG_BLOCK, 0, s>>>(rp, ci, m, n, nnz, bad);
}

void launch_merge_plan(const int32_t *rp, int64_t m, int64_t nnz, void *ws, hipStream_t s) {
  const int nwg = merge_workgroups(m, nnz);
  k_merge_plan<<<grid_for(nwg + 1), PDHG_BLOCK, 0, s>>>(rp, m, nnz, nwg, (int32_t *)ws);
}

template <typename T>
void launch_spmv_merge(const int32_t *rp, const int32_t *ci, const T *v, const T *x, T *y,
                       int64_t m, int64_t nnz, void *ws, hipStream_t s) {
  const int nwg = merge_workgroups(m, nnz);
  if (nwg == 0) return;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char *base = (char *)ws;
  const int32_t *start = (const int32_t *)base;
  int32_t *crow = (int32_t *)(base + up(4 * ((size_t)nwg + 1)));
  T *cval = (T *)(base + up(4 * ((size_t)nwg + 1)) + up(4 * (size_t)nwg));
  k_spmv_merge<T><<<nwg, MP_THREADS, 0, s>>>(rp, ci, v, x, y, m, nnz, start, crow, cval);
  k_spmv_merge_fix<T><<<grid_for(nwg), PDHG_BLOCK, 0, s>>>(crow, cval, nwg, m, y);
}

template void launch_spmv_merge<double>(const int32_t *, const int32_t *, const double *,
                                        const double *, double *, int64_t, int64_t, void *,
                                        hipStream_t);
template void launch_spmv_merge<float>(const int32_t *, const int32_t *, const float *,
                                       const float *, float *, int64_t, int64_t, void *,
                                       hipStream_t);
