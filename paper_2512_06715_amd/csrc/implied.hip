// Implied variable bounds for the safe dual bound (host code).
//
// The dual bound b'y + sum_j min over [lo_j, hi_j] of lambda_j x_j (weak
// duality) is -infinity as soon as a variable without a finite bound on the
// needed side has a nonzero reduced cost, which with approximate duals is the
// rule for free variables (the bus angles of the UC relaxation).  Bound
// propagation over the rows gives them finite bounds that every feasible
// point satisfies: with the other variables of a row at the ends of their
// bounds, a >= row (and an = row in both directions) bounds each variable.
#include <cmath>
#include <cstdint>

#include "internal.h"

// Sweeps over the rows in index order, each using the bounds found before it
// (also within the sweep), until a sweep adds nothing or `passes` sweeps
// have run.  Only infinite bounds are replaced.  A derived bound
// r = (b_i - sum over the other entries of t_k) / a_j becomes r - w (lower) or
// r + w (upper) with w = 2 (len + 2) 2^-53 (|b_i| + sum |t_k|) / |a_j| +
// 4 2^-53 |r| (len = the row's entries, t_k its finite activity terms).  The
// computed r carries the rounding of the products, the row sum, the removal
// of the own term, the subtraction from b_i and the division, below
// 2 (len + 2) 2^-53 (|b_i| + sum |t_k|) / |a_j| + 2^-53 |r| even where the
// terms cancel, and the second part of w also covers the rounding of r -+ w.
// A non-finite r or w gives no bound.  lo, hi hold l, u on entry.  Returns
// how many bounds became finite.
int64_t implied_bounds(int64_t m, const int32_t *rp, const int32_t *ci, const double *v,
                       const uint8_t *kind, const double *b, int passes, double *lo, double *hi) {
  const double eps = std::ldexp(1.0, -53);
  int64_t made = 0;
  for (int sweep = 0; sweep < passes; sweep++) {
    const int64_t made0 = made;
    for (int64_t i = 0; i < m; i++) {
      // activity range of the row: finite parts, their magnitudes and the
      // number of infinite terms
      double act_lo = 0.0, act_hi = 0.0, mag_lo = 0.0, mag_hi = 0.0;
      int64_t inf_lo = 0, inf_hi = 0;
      const int64_t len = rp[i + 1] - rp[i];
      for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
        const double a = v[k], L = lo[ci[k]], U = hi[ci[k]];
        const double t_lo = a > 0.0 ? a * L : a * U, t_hi = a > 0.0 ? a * U : a * L;
        if (std::isinf(t_lo)) {
          inf_lo++;
        } else {
          act_lo += t_lo;
          mag_lo += std::fabs(t_lo);
        }
        if (std::isinf(t_hi)) {
          inf_hi++;
        } else {
          act_hi += t_hi;
          mag_hi += std::fabs(t_hi);
        }
      }
      for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
        const int32_t j = ci[k];
        const double a = v[k], L = lo[j], U = hi[j];
        if (a == 0.0) continue;
        const double t_lo = a > 0.0 ? a * L : a * U, t_hi = a > 0.0 ? a * U : a * L;
        // row >= b: a x_j >= b - (largest activity of the other entries)
        if (inf_hi - (std::isinf(t_hi) ? 1 : 0) == 0) {
          const double r = (b[i] - (act_hi - (std::isinf(t_hi) ? 0.0 : t_hi))) / a;
          const double w = 2.0 * (double)(len + 2) * eps * (std::fabs(b[i]) + mag_hi) /
                                std::fabs(a) +
                            4.0 * eps * std::fabs(r);
          if (std::isfinite(r) && std::isfinite(w)) {
            if (a > 0.0 && std::isinf(lo[j])) {
              lo[j] = r - w;
              made++;
            }
            if (a < 0.0 && std::isinf(hi[j])) {
              hi[j] = r + w;
              made++;
            }
          }
        }
        // an equality row is also <= b: a x_j <= b - (smallest activity of the others)
        if (kind[i] == 0 && inf_lo - (std::isinf(t_lo) ? 1 : 0) == 0) {
          const double r = (b[i] - (act_lo - (std::isinf(t_lo) ? 0.0 : t_lo))) / a;
          const double w = 2.0 * (double)(len + 2) * eps * (std::fabs(b[i]) + mag_lo) /
                                std::fabs(a) +
                            4.0 * eps * std::fabs(r);
          if (std::isfinite(r) && std::isfinite(w)) {
            if (a > 0.0 && std::isinf(hi[j])) {
              hi[j] = r + w;
              made++;
            }
            if (a < 0.0 && std::isinf(lo[j])) {
              lo[j] = r - w;
              made++;
            }
          }
        }
      }
    }
    if (made == made0) break;
  }
  return made;
}
