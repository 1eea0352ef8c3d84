// Locality ordering of the scaled problem.
//
// The attempt kernels gather x by the column indices of A's rows and y by the
// row indices of A's columns.  In the order a model is written (for the UC
// relaxation: period-major blocks of buses, lines and units) the entries of
// neighbouring rows point far apart, so the lanes of one wave touch many
// cache lines per gather.  The solver therefore works on P A Q' with P, Q
// from a reverse Cuthill-McKee ordering of the bipartite graph whose nodes
// are the rows and the columns of A and whose edges are its nonzeros (rows
// and columns are ordered together, so a band of rows meets a band of
// columns).  It is a pure relabelling: every vector is stored in the new
// order and mapped back at the boundary, and no value is recomputed.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace {

// Rows 0..m-1 and columns m..m+n-1 of the bipartite graph of A.
struct Graph {
  int64_t m, n;
  const int32_t *rp, *ci, *cp, *ri;
  int64_t deg(int64_t u) const { return u < m ? rp[u + 1] - rp[u] : cp[u - m + 1] - cp[u - m]; }
  template <typename F>
  void nbrs(int64_t u, F f) const {
    if (u < m) {
      for (int32_t k = rp[u]; k < rp[u + 1]; k++) f(m + ci[k]);
    } else {
      int64_t j = u - m;
      for (int32_t k = cp[j]; k < cp[j + 1]; k++) f((int64_t)ri[k]);
    }
  }
};

// Breadth-first levels from `root` over the nodes not yet numbered; returns
// the depth of the last level and leaves its nodes in `last`.  `stamp` marks
// the nodes seen by search `tag` without clearing between searches.
int bfs_last_level(const Graph &g, int64_t root, const std::vector<uint8_t> &done,
                   std::vector<int32_t> &stamp, int32_t tag, std::vector<int64_t> &queue,
                   std::vector<int64_t> &last) {
  queue.clear();
  queue.push_back(root);
  stamp[root] = tag;
  size_t head = 0;
  int depth = 0;
  while (true) {
    size_t level_end = queue.size();
    last.assign(queue.begin() + head, queue.end());
    while (head < level_end) {
      int64_t u = queue[head++];
      g.nbrs(u, [&](int64_t w) {
        if (!done[w] && stamp[w] != tag) {
          stamp[w] = tag;
          queue.push_back(w);
        }
      });
    }
    if (queue.size() == level_end) break;
    depth++;
  }
  return depth;
}

}  // namespace

// Reverse Cuthill-McKee order of the rows and columns of an m x n CSR
// matrix (with its transpose cp/ri).  Each connected component starts from a
// pseudo-peripheral node (George-Liu: move to a minimum-degree node of the
// farthest level while the eccentricity grows); neighbours are numbered by
// increasing degree, ties by index.  Out: row_order[i] = original row of
// position i, col_order[j] = original column of position j.
void rcm_order(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *cp,
               const int32_t *ri, std::vector<int32_t> &row_order, std::vector<int32_t> &col_order) {
  const Graph g{m, n, rp, ci, cp, ri};
  const int64_t N = m + n;
  // nodes by (degree, index): counting sort
  int64_t maxdeg = 0;
  for (int64_t u = 0; u < N; u++) maxdeg = std::max(maxdeg, g.deg(u));
  std::vector<int64_t> cnt(maxdeg + 2, 0), by_deg(N);
  for (int64_t u = 0; u < N; u++) cnt[g.deg(u) + 1]++;
  for (int64_t d = 0; d <= maxdeg; d++) cnt[d + 1] += cnt[d];
  for (int64_t u = 0; u < N; u++) by_deg[cnt[g.deg(u)]++] = u;

  std::vector<uint8_t> done(N, 0);
  std::vector<int32_t> stamp(N, -1);
  std::vector<int64_t> order, queue, last, nb;
  order.reserve(N);
  int32_t tag = 0;
  for (int64_t s : by_deg) {
    if (done[s]) continue;
    int64_t root = s;
    int ecc = bfs_last_level(g, root, done, stamp, tag++, queue, last);
    for (int it = 0; it < 8; it++) {
      int64_t best = last[0];
      for (int64_t w : last)
        if (g.deg(w) < g.deg(best) || (g.deg(w) == g.deg(best) && w < best)) best = w;
      int e2 = bfs_last_level(g, best, done, stamp, tag++, queue, last);
      if (e2 <= ecc) break;
      root = best;
      ecc = e2;
    }
    size_t head = order.size();
    order.push_back(root);
    done[root] = 1;
    while (head < order.size()) {
      int64_t u = order[head++];
      nb.clear();
      g.nbrs(u, [&](int64_t w) {
        if (!done[w]) {
          done[w] = 1;
          nb.push_back(w);
        }
      });
      std::sort(nb.begin(), nb.end(), [&](int64_t a, int64_t b) {
        int64_t da = g.deg(a), db = g.deg(b);
        return da != db ? da < db : a < b;
      });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  row_order.clear();
  col_order.clear();
  row_order.reserve(m);
  col_order.reserve(n);
  for (int64_t q = N - 1; q >= 0; q--) {
    int64_t u = order[q];
    if (u < m)
      row_order.push_back((int32_t)u);
    else
      col_order.push_back((int32_t)(u - m));
  }
}

// P A Q' in CSR with ascending columns in each row: row i is original row
// row_order[i], column j original column col_order[j] (cinv = its inverse).
void permute_csr(int64_t m, const int32_t *rp, const int32_t *ci, const double *v,
                 const std::vector<int32_t> &row_order, const std::vector<int32_t> &cinv,
                 std::vector<int32_t> &prp, std::vector<int32_t> &pci, std::vector<double> &pv) {
  prp.assign(m + 1, 0);
  for (int64_t i = 0; i < m; i++) {
    int32_t r = row_order[i];
    prp[i + 1] = prp[i] + (rp[r + 1] - rp[r]);
  }
  pci.resize(prp[m]);
  pv.resize(prp[m]);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < m; i++) {
    int32_t r = row_order[i];
    row.clear();
    for (int32_t k = rp[r]; k < rp[r + 1]; k++) row.emplace_back(cinv[ci[k]], v[k]);
    std::sort(row.begin(), row.end(),
              [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                return a.first < b.first;
              });
    for (size_t q = 0; q < row.size(); q++) {
      pci[prp[i] + q] = row[q].first;
      pv[prp[i] + q] = row[q].second;
    }
  }
}

// The inverse relabelling of permute_csr: the original CSR (ascending
// columns) from the permuted one.
void unpermute_csr(int64_t m, const int32_t *prp, const int32_t *pci, const double *pv,
                   const std::vector<int32_t> &row_order, const std::vector<int32_t> &col_order,
                   std::vector<int32_t> &rp, std::vector<int32_t> &ci, std::vector<double> &v) {
  rp.assign(m + 1, 0);
  for (int64_t i = 0; i < m; i++) rp[row_order[i] + 1] = prp[i + 1] - prp[i];
  for (int64_t r = 0; r < m; r++) rp[r + 1] += rp[r];
  ci.resize(rp[m]);
  v.resize(rp[m]);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < m; i++) {
    int32_t r = row_order[i];
    row.clear();
    for (int32_t k = prp[i]; k < prp[i + 1]; k++) row.emplace_back(col_order[pci[k]], pv[k]);
    std::sort(row.begin(), row.end(),
              [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                return a.first < b.first;
              });
    for (size_t q = 0; q < row.size(); q++) {
      ci[rp[r] + q] = row[q].first;
      v[rp[r] + q] = row[q].second;
    }
  }
}

// Host transpose of a CSR matrix (rows ascending within each column); v may
// be null for the structure alone.
void transpose_csr(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                   std::vector<int32_t> &cp, std::vector<int32_t> &ri, std::vector<double> &vt) {
  cp.assign(n + 1, 0);
  for (int64_t k = 0; k < rp[m]; k++) cp[ci[k] + 1]++;
  for (int64_t j = 0; j < n; j++) cp[j + 1] += cp[j];
  ri.resize(std::max<int64_t>(rp[m], 1));
  if (v) vt.resize(std::max<int64_t>(rp[m], 1));
  std::vector<int32_t> next(cp.begin(), cp.end() - 1);
  for (int64_t i = 0; i < m; i++)
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      int32_t q = next[ci[k]]++;
      ri[q] = (int32_t)i;
      if (v) vt[q] = v[k];
    }
}

// ---------------------------------------------------------------------------
// device relabelling of vectors

namespace {

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + PDHG_BLOCK - 1) / PDHG_BLOCK;
  return (unsigned)(g > 0 ? g : 1);
}

template <typename T>
__global__ void k_gather(T *__restrict__ dst, const T *__restrict__ src,
                         const int32_t *__restrict__ order, int64_t cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) dst[i] = src[order[i]];
}

template <typename T>
__global__ void k_scatter(T *__restrict__ dst, const T *__restrict__ src,
                          const int32_t *__restrict__ order, int64_t cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) dst[order[i]] = src[i];
}

}  // namespace

void launch_gather_f64(double *dst, const double *src, const int32_t *order, int64_t cnt,
                       hipStream_t s) {
  if (cnt > 0) k_gather<double><<<grid_for(cnt), PDHG_BLOCK, 0, s>>>(dst, src, order, cnt);
}

void launch_gather_u8(uint8_t *dst, const uint8_t *src, const int32_t *order, int64_t cnt,
                      hipStream_t s) {
  if (cnt > 0) k_gather<uint8_t><<<grid_for(cnt), PDHG_BLOCK, 0, s>>>(dst, src, order, cnt);
}

void launch_scatter_f64(double *dst, const double *src, const int32_t *order, int64_t cnt,
                        hipStream_t s) {
  if (cnt > 0) k_scatter<double><<<grid_for(cnt), PDHG_BLOCK, 0, s>>>(dst, src, order, cnt);
}
