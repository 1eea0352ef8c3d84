/*
 * FP64 CPU oracle for the restarted PDHG (PDLP-style) LP solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark call this code.  It shares nothing with
 * the HIP library: no headers, helpers or tables.
 *
 * Problem:   min c'x  s.t.  a_i'x = b_i (eq rows),  a_i'x >= b_i (ge rows),
 *            l <= x <= u.
 * This is the LP pair of the paper's "PDHG Background" section with the
 * sign reading that agrees with its Lagrangian and update equations
 * (primal rows are >=, duals y >= 0), widened to equality rows and to a
 * box [l, u] instead of x >= 0.  Lagrangian L(x,y) = c'x - y'(Ax - b).
 *
 * Everything is written as plain scalar loops in the order the algorithm
 * states; sums run sequentially in index order.  Compile with
 * -ffp-contract=off so no multiply-add is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_CSR (-2)
#define ORC_ERR_BOUNDS (-3)
#define ORC_ERR_NONFINITE (-4)

#define ST_OPTIMAL 1
#define ST_ITER_LIMIT 2
#define ST_NUMERICAL 4
#define ST_PRIMAL_INFEASIBLE 5
#define ST_DUAL_INFEASIBLE 6

enum { VK_FREE = 0, VK_LOWER = 1, VK_UPPER = 2, VK_BOXED = 3, VK_FIXED = 4 };

/* ------------------------------------------------------------------ */
/* input validation and bound kinds                                     */

int orc_validate(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                 const double *v, const uint8_t *kind, const double *b,
                 const double *c, const double *l, const double *u) {
  if (m <= 0 || n <= 0) return ORC_ERR_ARG;
  if (rp[0] != 0) return ORC_ERR_CSR;
  for (int64_t i = 0; i < m; i++) {
    if (rp[i + 1] < rp[i]) return ORC_ERR_CSR;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
      if (ci[k] < 0 || ci[k] >= n) return ORC_ERR_CSR;
      if (k > rp[i] && ci[k] <= ci[k - 1]) return ORC_ERR_CSR;
    }
  }
  for (int64_t i = 0; i < m; i++)
    if (kind[i] > 1) return ORC_ERR_ARG;
  for (int64_t j = 0; j < n; j++) {
    if (isnan(l[j]) || isnan(u[j])) return ORC_ERR_BOUNDS;
    if (l[j] > u[j]) return ORC_ERR_BOUNDS;
    if (l[j] == INFINITY || u[j] == -INFINITY) return ORC_ERR_BOUNDS;
  }
  for (int64_t k = 0; k < rp[m]; k++)
    if (!isfinite(v[k])) return ORC_ERR_NONFINITE;
  for (int64_t i = 0; i < m; i++)
    if (!isfinite(b[i])) return ORC_ERR_NONFINITE;
  for (int64_t j = 0; j < n; j++)
    if (!isfinite(c[j])) return ORC_ERR_NONFINITE;
  return ORC_OK;
}

/* 0 free, 1 lower bound only, 2 upper bound only, 3 both (l<u), 4 fixed */
void orc_var_kind(int64_t n, const double *l, const double *u, uint8_t *out) {
  for (int64_t j = 0; j < n; j++) {
    int lf = isfinite(l[j]), uf = isfinite(u[j]);
    if (lf && uf)
      out[j] = (l[j] == u[j]) ? VK_FIXED : VK_BOXED;
    else if (lf)
      out[j] = VK_LOWER;
    else if (uf)
      out[j] = VK_UPPER;
    else
      out[j] = VK_FREE;
  }
}

/* CSR of A^T by counting sort: rows ascending inside each column. */
void orc_transpose(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                   const double *v, int32_t *cp, int32_t *ri, double *vt) {
  int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t j = 0; j <= n; j++) cp[j] = 0;
  for (int64_t k = 0; k < rp[m]; k++) cp[ci[k] + 1] += 1;
  for (int64_t j = 0; j < n; j++) cp[j + 1] += cp[j];
  for (int64_t j = 0; j < n; j++) next[j] = cp[j];
  for (int64_t i = 0; i < m; i++)
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
      int64_t slot = next[ci[k]]++;
      ri[slot] = (int32_t)i;
      vt[slot] = v[k];
    }
  free(next);
}

/* ------------------------------------------------------------------ */
/* diagonal preconditioning                                              */

/* The power of two nearest to sqrt(M) on a log scale.  With M = nu * 2^E,
 * nu in [0.5, 1): sqrt(M) = sqrt(nu) 2^(E/2), and log2 sqrt(M) lies in
 * [E/2 - 1/2, E/2) for even E and in [(E-1)/2, (E-1)/2 + 1/2) for odd E,
 * so the nearest integer exponent is floor(E/2) in both cases (a tie at
 * E/2 - 1/2 goes up).  M = 0 (an empty row or column) gives 1. */
double orc_pow2_sqrt(double M) {
  if (!(M > 0.0)) return 1.0;
  int E;
  frexp(M, &E);
  int k = (E >= 0) ? E / 2 : -((-E + 1) / 2);
  return ldexp(1.0, k);
}

/* In place: A <- diag(1/r) A diag(1/s) for ruiz_iters Ruiz infinity-norm
 * passes, then (if pc) one Pock-Chambolle pass with alpha = 1.  Every
 * factor is a power of two, so each rescale is exact.  Dr, Dc accumulate
 * so that A_scaled = diag(Dr) A diag(Dc). */
void orc_scale(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
               double *v, int ruiz_iters, int pc, double *Dr, double *Dc) {
  double *rs = (double *)malloc(sizeof(double) * (size_t)m);
  double *cs = (double *)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < m; i++) Dr[i] = 1.0;
  for (int64_t j = 0; j < n; j++) Dc[j] = 1.0;
  int passes = ruiz_iters + (pc ? 1 : 0);
  for (int it = 0; it < passes; it++) {
    int is_pc = (it == ruiz_iters);
    for (int64_t i = 0; i < m; i++) rs[i] = 0.0;
    for (int64_t j = 0; j < n; j++) cs[j] = 0.0;
    for (int64_t i = 0; i < m; i++)
      for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
        double a = fabs(v[k]);
        if (is_pc) {
          rs[i] += a;
          cs[ci[k]] += a;
        } else {
          if (a > rs[i]) rs[i] = a;
          if (a > cs[ci[k]]) cs[ci[k]] = a;
        }
      }
    for (int64_t i = 0; i < m; i++) rs[i] = orc_pow2_sqrt(rs[i]);
    for (int64_t j = 0; j < n; j++) cs[j] = orc_pow2_sqrt(cs[j]);
    for (int64_t i = 0; i < m; i++)
      for (int64_t k = rp[i]; k < rp[i + 1]; k++) v[k] = v[k] / rs[i] / cs[ci[k]];
    for (int64_t i = 0; i < m; i++) Dr[i] = Dr[i] / rs[i];
    for (int64_t j = 0; j < n; j++) Dc[j] = Dc[j] / cs[j];
  }
  free(rs);
  free(cs);
}

/* ------------------------------------------------------------------ */
/* small helpers on plain arrays                                         */

static void spmv(int64_t m, const int32_t *rp, const int32_t *ci, const double *v,
                 const double *x, double *out) {
  for (int64_t i = 0; i < m; i++) {
    double s = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) s += v[k] * x[ci[k]];
    out[i] = s;
  }
}

static double dot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t j = 0; j < n; j++) s += a[j] * b[j];
  return s;
}

static double clampd(double x, double lo, double hi) {
  if (x < lo) return lo;
  if (x > hi) return hi;
  return x;
}

/* Projection of a reduced cost lambda_j onto the cone the dual allows for
 * variable kind vk: free -> {0}, lower-only -> [0, inf), upper-only ->
 * (-inf, 0], boxed and fixed -> R. */
static double proj_lambda(uint8_t vk, double lam) {
  switch (vk) {
    case VK_FREE: return 0.0;
    case VK_LOWER: return lam > 0.0 ? lam : 0.0;
    case VK_UPPER: return lam < 0.0 ? lam : 0.0;
    default: return lam;
  }
}

/* Bound term of the dual objective for a projected reduced cost:
 * l * max(lam,0) - u * max(-lam,0) over the finite bounds. */
static double bound_term(uint8_t vk, double lam, double l, double u) {
  double t = 0.0;
  if (lam > 0.0 && (vk == VK_LOWER || vk == VK_BOXED || vk == VK_FIXED)) t += l * lam;
  if (lam < 0.0 && (vk == VK_UPPER || vk == VK_BOXED || vk == VK_FIXED)) t += u * lam;
  return t;
}

/* KKT pieces of a point, given Ax and A'y already formed.
 * Row weights wr and column weights wc turn scaled residuals into
 * unscaled ones (pass NULL for none): residual_i / wr_i, lambda_j / wc_j.
 * out: [0] ||r_p||^2, [1] ||r_d||^2, [2] primal obj, [3] dual obj,
 *      [4] ||r_p||_inf, [5] ||r_d||_inf */
static void kkt_pieces(int64_t m, int64_t n, const uint8_t *kind, const uint8_t *vk,
                       const double *b, const double *c, const double *l,
                       const double *u, const double *x, const double *y,
                       const double *Ax, const double *ATy, const double *wr,
                       const double *wc, double *out) {
  double rp2 = 0.0, rpi = 0.0, rd2 = 0.0, rdi = 0.0, pobj = 0.0, dobj = 0.0;
  for (int64_t i = 0; i < m; i++) {
    double r = b[i] - Ax[i];
    if (kind[i] == 1 && r < 0.0) r = 0.0;
    if (wr) r = r / wr[i];
    rp2 += r * r;
    if (fabs(r) > rpi) rpi = fabs(r);
    dobj += b[i] * y[i];
  }
  for (int64_t j = 0; j < n; j++) {
    double lam = c[j] - ATy[j];
    double pl = proj_lambda(vk[j], lam);
    double rd = lam - pl;
    double rdu = wc ? rd / wc[j] : rd;
    rd2 += rdu * rdu;
    if (fabs(rdu) > rdi) rdi = fabs(rdu);
    dobj += bound_term(vk[j], pl, l[j], u[j]);
    pobj += c[j] * x[j];
  }
  out[0] = rp2;
  out[1] = rd2;
  out[2] = pobj;
  out[3] = dobj;
  out[4] = rpi;
  out[5] = rdi;
}

/* ------------------------------------------------------------------ */
/* independent KKT checker on the unscaled problem                        */

/* out: [0] rel_p [1] rel_d [2] rel_gap [3] rel_kkt [4] primal obj
 *      [5] dual obj [6] ||r_p||_2 [7] ||r_d||_2 [8] |gap| [9] ||r_p||_inf
 *      [10] ||r_d||_inf [11] max bound violation [12] max cone violation of y
 * The primal residual also counts bound violations of x; the dual residual
 * also counts negative y on >= rows.  Relative measures:
 *   rel_p = ||r_p||/(1+||b||), rel_d = ||r_d||/(1+||c||),
 *   rel_gap = |pobj - dobj| / (1 + |pobj| + |dobj|). */
void orc_kkt(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
             const double *v, const uint8_t *kind, const double *b, const double *c,
             const double *l, const double *u, const double *x, const double *y,
             double *out) {
  double *Ax = (double *)malloc(sizeof(double) * (size_t)m);
  double *ATy = (double *)calloc((size_t)n, sizeof(double));
  uint8_t *vk = (uint8_t *)malloc((size_t)n);
  orc_var_kind(n, l, u, vk);
  spmv(m, rp, ci, v, x, Ax);
  for (int64_t i = 0; i < m; i++)
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) ATy[ci[k]] += v[k] * y[i];
  double pc[6];
  kkt_pieces(m, n, kind, vk, b, c, l, u, x, y, Ax, ATy, NULL, NULL, pc);
  double bv = 0.0, bv2 = 0.0, cv = 0.0, cv2 = 0.0;
  for (int64_t j = 0; j < n; j++) {
    double e = 0.0;
    if (x[j] < l[j]) e = l[j] - x[j];
    if (x[j] > u[j]) e = x[j] - u[j];
    bv2 += e * e;
    if (e > bv) bv = e;
  }
  for (int64_t i = 0; i < m; i++)
    if (kind[i] == 1 && y[i] < 0.0) {
      cv2 += y[i] * y[i];
      if (-y[i] > cv) cv = -y[i];
    }
  double nb = sqrt(dot(m, b, b)), nc = sqrt(dot(n, c, c));
  double rpn = sqrt(pc[0] + bv2), rdn = sqrt(pc[1] + cv2);
  double gap = fabs(pc[2] - pc[3]);
  out[0] = rpn / (1.0 + nb);
  out[1] = rdn / (1.0 + nc);
  out[2] = gap / (1.0 + fabs(pc[2]) + fabs(pc[3]));
  out[3] = out[0];
  if (out[1] > out[3]) out[3] = out[1];
  if (out[2] > out[3]) out[3] = out[2];
  out[4] = pc[2];
  out[5] = pc[3];
  out[6] = rpn;
  out[7] = rdn;
  out[8] = gap;
  out[9] = pc[4] > bv ? pc[4] : bv;
  out[10] = pc[5] > cv ? pc[5] : cv;
  out[11] = bv;
  out[12] = cv;
  free(Ax);
  free(ATy);
  free(vk);
}

/* ------------------------------------------------------------------ */
/* restarted, adaptive-step PDHG                                          */

typedef struct {
  double tol;          /* relative KKT target */
  int64_t max_iter;    /* attempts */
  int eval_period;     /* attempts between evaluations */
  int step_mode;       /* 0 adaptive, 1 constant (eta = fixed_eta) */
  double fixed_eta;    /* constant mode; <= 0 means 0.9/||A||_2 (power iteration) */
  int ruiz_iters;
  int pock_chambolle;
  int restart;         /* 1: restart scheme on */
  int use_average;     /* 1: weighted average is a restart/termination candidate */
  double omega0;       /* <= 0: ||c||/||b|| rule */
  double pw_theta;     /* primal-weight smoothing; 0 keeps omega */
  int infeas_every;    /* > 0: every this many evaluations, test y for a
                          certificate of primal infeasibility */
  const double *ilo, *ihi;  /* bounds every feasible x satisfies (original
                               space; NULL: l, u) for that test and the next */
  double dinf_eps;     /* > 0: at the same evaluations, test the primal
                          displacement since the last restart as a ray
                          certifying dual infeasibility, with this tolerance */
  double *trace;       /* nullable: one record of ORC_TRACE_LEN doubles per
                          evaluation, at most trace_cap records (see below) */
  int64_t trace_cap;
  int term;            /* the quantity held to tol: 0 the relative KKT error,
                          1 the relative primal residual, 2 the relative dual
                          residual (feasibility polishing) */
} orc_opts;

/* Evaluation trace (instrumentation only; it changes no arithmetic).  Record
 * r of o->trace: [0] attempts k, [1] KKT_omega of the current iterate,
 * [2] KKT_omega of the average (-1 without one), [3] KKT_omega of the last
 * restart point and [4] the previous evaluation's candidate (both as the
 * restart decision sees them; +inf when none), [5] 1 if the evaluation
 * restarted, [6] 1 if the candidate was the average, [7] omega after the
 * evaluation, [8] KKT_omega of the new restart point (the reference of the
 * next decisions; -1 without a restart).  Records past trace_cap are
 * dropped; info[15] counts all of them. */
#define ORC_TRACE_LEN 9

/* info: [0] status [1] attempts [2] accepted [3] restarts [4] pobj [5] dobj
 *       [6] rel_p [7] rel_d [8] rel_gap [9] rel_kkt [10] eta [11] omega
 *       [12] returned point (0 current, 1 average) [13] initial eta
 *       [14] initial omega [15] evaluation records (the trace below) */

typedef struct {
  int64_t m, n;
  const int32_t *rp, *ci, *cp, *ri;
  const double *v, *vt;
  const uint8_t *kind, *vk;
  const double *b, *c, *l, *u;       /* scaled data */
  const double *Dr, *Dc;
  double nb, nc;                     /* unscaled ||b||, ||c|| */
} scaled_lp;

/* Scaled-space KKT_omega for restarts and unscaled relative KKT for
 * termination, both from one pass.  out: [0] KKT_omega, [1] rel_kkt,
 * [2] pobj, [3] dobj, [4] rel_p, [5] rel_d, [6] rel_gap, [7] ||r_p||^2,
 * [8] ||r_d||^2, [9] gap (scaled space pieces for KKT_omega) */
static void evaluate(const scaled_lp *P, const double *x, const double *y,
                     const double *Ax, const double *ATy, double omega, double *out) {
  double sc[6], us[6];
  kkt_pieces(P->m, P->n, P->kind, P->vk, P->b, P->c, P->l, P->u, x, y, Ax, ATy,
             NULL, NULL, sc);
  kkt_pieces(P->m, P->n, P->kind, P->vk, P->b, P->c, P->l, P->u, x, y, Ax, ATy,
             P->Dr, P->Dc, us);
  double gap = fabs(sc[2] - sc[3]);
  out[0] = sqrt(omega * sc[0] + sc[1] / omega + gap * gap);
  double rel_p = sqrt(us[0]) / (1.0 + P->nb);
  double rel_d = sqrt(us[1]) / (1.0 + P->nc);
  double rel_g = gap / (1.0 + fabs(sc[2]) + fabs(sc[3]));
  double r = rel_p;
  if (rel_d > r) r = rel_d;
  if (rel_g > r) r = rel_g;
  out[1] = r;
  out[2] = sc[2];
  out[3] = sc[3];
  out[4] = rel_p;
  out[5] = rel_d;
  out[6] = rel_g;
  out[7] = sc[0];
  out[8] = sc[1];
  out[9] = gap;
}

static void spmv_t(const scaled_lp *P, const double *y, double *out) {
  spmv(P->n, P->cp, P->ri, P->vt, y, out);
}

/* ||A||_2 estimate: power iteration on A'A from the all-ones vector. */
double orc_power_norm(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                      const double *v, int iters) {
  double *z = (double *)malloc(sizeof(double) * (size_t)n);
  double *w = (double *)malloc(sizeof(double) * (size_t)m);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  double nrm = sqrt((double)n), est = 0.0;
  for (int64_t j = 0; j < n; j++) z[j] = 1.0 / nrm;
  for (int it = 0; it < iters; it++) {
    spmv(m, rp, ci, v, z, w);
    for (int64_t j = 0; j < n; j++) q[j] = 0.0;
    for (int64_t i = 0; i < m; i++)
      for (int64_t k = rp[i]; k < rp[i + 1]; k++) q[ci[k]] += v[k] * w[i];
    double qn = sqrt(dot(n, q, q));
    est = sqrt(qn);
    if (qn == 0.0) break;
    for (int64_t j = 0; j < n; j++) z[j] = q[j] / qn;
  }
  free(z);
  free(w);
  free(q);
  return est;
}

int64_t orc_bound_repair(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                         const double *v, const uint8_t *kind, const double *c,
                         const double *lo, const double *hi, double *ylo, double *yhi);

/* Certificate of primal infeasibility (Farkas): for y with y_i >= 0 on >= rows
 * and a box [lo, hi] that holds every feasible x, feasibility would give
 * b'y <= y'Ax = sum_j (A'y)_j x_j <= sum_j max over [lo_j, hi_j] of
 * (A'y)_j x_j; so b'y + sum_j min(lambda_j lo_j, lambda_j hi_j) > 0 with
 * lambda = -A'y proves that no feasible x exists.  This is the safe bound's
 * sum for c = 0 (same sign rule and allowance), on the scaled problem.  Any
 * such y will do, so y is first clamped into the safe bound's repair
 * intervals for c = 0 (ylo, yhi; nullable): a row whose single-entry column
 * has an infinite bound on the side lambda_j would need gets the sign (or
 * the zero) that keeps lambda_j usable.  The intervals' ends are 0 or
 * infinite, so the scaling leaves them unchanged.  Returns the value lowered
 * by the allowance, or -INFINITY when a needed bound is infinite. */
static double homogeneous_certificate(const scaled_lp *P, const double *y, const double *lo,
                                      const double *hi, const double *ylo, const double *yhi) {
  const int64_t m = P->m, n = P->n;
  const double eps = ldexp(1.0, -53);
  double by = 0.0, byabs = 0.0, terms = 0.0, sabs = 0.0;
  int64_t kmax = 0, ninf = 0;
  for (int64_t i = 0; i < m; i++) {
    double yi = (P->kind[i] == 1 && y[i] < 0.0) ? 0.0 : y[i];
    if (ylo) yi = fmin(fmax(yi, ylo[i]), yhi[i]);
    double t = P->b[i] * yi;
    by += t;
    byabs += fabs(t);
  }
  for (int64_t j = 0; j < n; j++) {
    double s = 0.0, sa = 0.0;
    for (int32_t k = P->cp[j]; k < P->cp[j + 1]; k++) {
      int32_t i = P->ri[k];
      double yi = (P->kind[i] == 1 && y[i] < 0.0) ? 0.0 : y[i];
      if (ylo) yi = fmin(fmax(yi, ylo[i]), yhi[i]);
      double pr = P->vt[k] * yi;
      s += pr;
      sa += fabs(pr);
    }
    int64_t len = P->cp[j + 1] - P->cp[j];
    if (len > kmax) kmax = len;
    const double lam = 0.0 - s;
    const double err = 2.0 * (double)(len + 2) * eps * sa;
    if (fabs(lam) > err || err == 0.0) {
      if (lam == 0.0) continue;
      const double bnd = lam > 0.0 ? lo[j] : hi[j];
      if (isinf(bnd)) {
        ninf++;
        continue;
      }
      terms += lam * bnd;
      sabs += fabs(bnd) * sa;
    } else if (isinf(lo[j]) || isinf(hi[j])) {
      ninf++;
    } else {
      terms += fmin(lam * lo[j], lam * hi[j]);
      sabs += fmax(fabs(lo[j]), fabs(hi[j])) * sa;
    }
  }
  if (ninf) return -INFINITY;
  return (by + terms) - 2.0 * (double)(n + m + kmax + 4) * eps * (byabs + sabs);
}

/* Certificate of dual infeasibility (the primal has an improving ray): a
 * direction d with c'd < 0 along which every constraint stays satisfied,
 * i.e. (A d)_i = 0 on = rows, (A d)_i >= 0 on >= rows, and d_j in the
 * recession cone of [lo_j, hi_j] (d_j = 0 where both ends are finite,
 * d_j >= 0 where only lo_j is, d_j <= 0 where only hi_j is).  This is the
 * test of PDLP, the PDHG variant the paper builds on; an approximate one:
 * d passes when c'd < 0 and the largest violation is at most eps (-c'd),
 * both homogeneous in d.  It is evaluated on the original problem.  The
 * candidate is the primal iterate's displacement since the last restart,
 * d^ = x - xl in the scaled space, d = Dc d^; on an unbounded LP the
 * iterates move by a fixed ray per step once the projections stop changing.
 * In the original space (A d)_i = (sum_k a^_ik d^_k) / Dr_i and
 * c_j d_j = c^_j d^_j (power-of-two factors).  lo, hi: the scaled box of
 * the infeasibility test (only their finiteness matters).  On success the
 * unscaled d is written to ray and 1 is returned. */
static int ray_certificate(const scaled_lp *P, const double *x, const double *xl,
                           const double *lo, const double *hi, double eps, double *ray) {
  const int64_t m = P->m, n = P->n;
  double cd = 0.0, worst = 0.0;
  for (int64_t j = 0; j < n; j++) {
    const double dh = x[j] - xl[j];
    const double d = P->Dc[j] * dh;
    cd += P->c[j] * dh;
    double viol = 0.0;
    if (!isfinite(d))
      viol = INFINITY;  /* an overflowed direction is no certificate */
    else if (isfinite(lo[j]) && isfinite(hi[j]))
      viol = fabs(d);
    else if (isfinite(lo[j]))
      viol = d < 0.0 ? -d : 0.0;
    else if (isfinite(hi[j]))
      viol = d > 0.0 ? d : 0.0;
    if (viol > worst) worst = viol;
  }
  for (int64_t i = 0; i < m; i++) {
    double s = 0.0;
    for (int32_t k = P->rp[i]; k < P->rp[i + 1]; k++) s += P->v[k] * (x[P->ci[k]] - xl[P->ci[k]]);
    const double r = s / P->Dr[i];
    const double viol = !isfinite(r) ? INFINITY : P->kind[i] == 0 ? fabs(r) : (r < 0.0 ? -r : 0.0);
    if (viol > worst) worst = viol;
  }
  if (!(cd < 0.0) || !(worst <= eps * -cd)) return 0;
  for (int64_t j = 0; j < n; j++) ray[j] = P->Dc[j] * (x[j] - xl[j]);
  return 1;
}

int orc_pdhg(int64_t m, int64_t n, const int32_t *rp0, const int32_t *ci0,
             const double *v0, const uint8_t *kind, const double *b0, const double *c0,
             const double *l0, const double *u0, const orc_opts *o, const double *x0,
             const double *y0, double *x_out, double *y_out, double *info) {
  int64_t nnz = rp0[m];
  /* scaled copies */
  double *v = (double *)malloc(sizeof(double) * (size_t)nnz);
  memcpy(v, v0, sizeof(double) * (size_t)nnz);
  double *Dr = (double *)malloc(sizeof(double) * (size_t)m);
  double *Dc = (double *)malloc(sizeof(double) * (size_t)n);
  orc_scale(m, n, rp0, ci0, v, o->ruiz_iters, o->pock_chambolle, Dr, Dc);
  int32_t *cp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *ri = (int32_t *)malloc(sizeof(int32_t) * (size_t)nnz);
  double *vt = (double *)malloc(sizeof(double) * (size_t)nnz);
  orc_transpose(m, n, rp0, ci0, v, cp, ri, vt);
  double *b = (double *)malloc(sizeof(double) * (size_t)m);
  double *c = (double *)malloc(sizeof(double) * (size_t)n);
  double *l = (double *)malloc(sizeof(double) * (size_t)n);
  double *u = (double *)malloc(sizeof(double) * (size_t)n);
  uint8_t *vk = (uint8_t *)malloc((size_t)n);
  orc_var_kind(n, l0, u0, vk);
  for (int64_t i = 0; i < m; i++) b[i] = Dr[i] * b0[i];
  for (int64_t j = 0; j < n; j++) {
    c[j] = Dc[j] * c0[j];
    l[j] = l0[j] / Dc[j];
    u[j] = u0[j] / Dc[j];
  }
  scaled_lp P = {m, n, rp0, ci0, cp, ri, v, vt, kind, vk, b, c, l, u, Dr, Dc,
                 sqrt(dot(m, b0, b0)), sqrt(dot(n, c0, c0))};

  size_t N8 = sizeof(double) * (size_t)n, M8 = sizeof(double) * (size_t)m;
  double *x = malloc(N8), *y = malloc(M8), *Ax = malloc(M8), *ATy = malloc(N8);
  double *xn = malloc(N8), *yn = malloc(M8), *Axn = malloc(M8);
  double *xs = malloc(N8), *ys = malloc(M8);
  double *xa = malloc(N8), *ya = malloc(M8), *Axa = malloc(M8), *ATya = malloc(N8);
  double *xl = malloc(N8), *yl = malloc(M8);
  double *ray = malloc(N8);

  /* start point: clamp(0 or x0) into the box; y0 projected onto the cone */
  for (int64_t j = 0; j < n; j++) x[j] = clampd(x0 ? x0[j] / Dc[j] : 0.0, l[j], u[j]);
  for (int64_t i = 0; i < m; i++) {
    double yi = y0 ? y0[i] / Dr[i] : 0.0;
    if (kind[i] == 1 && yi < 0.0) yi = 0.0;
    y[i] = yi;
  }
  spmv(m, rp0, ci0, v, x, Ax);
  spmv_t(&P, y, ATy);

  /* step size and primal weight */
  double amax = 0.0;
  for (int64_t k = 0; k < nnz; k++)
    if (fabs(v[k]) > amax) amax = fabs(v[k]);
  double eta;
  if (o->step_mode == 1)
    eta = o->fixed_eta > 0.0 ? o->fixed_eta : 0.9 / orc_power_norm(m, n, rp0, ci0, v, 50);
  else
    eta = amax > 0.0 ? 1.0 / amax : 1.0;  /* no nonzero: 1 */
  double omega;
  if (o->omega0 > 0.0)
    omega = o->omega0;
  else {
    double nc = sqrt(dot(n, c, c)), nb = sqrt(dot(m, b, b));
    omega = (nc > 1e-10 && nb > 1e-10) ? nc / nb : 1.0;
  }
  info[13] = eta;
  info[14] = omega;

  /* the box of the infeasibility test, scaled */
  double *blo = (double *)malloc(N8), *bhi = (double *)malloc(N8);
  /* the repair intervals of the Farkas test (c = 0) over the same box */
  double *fylo = (double *)malloc(M8 > 0 ? M8 : 8), *fyhi = (double *)malloc(M8 > 0 ? M8 : 8);
  {
    double *zero = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    orc_bound_repair(m, n, rp0, ci0, v0, kind, zero, o->ilo ? o->ilo : l0,
                     o->ihi ? o->ihi : u0, fylo, fyhi);
    free(zero);
  }
  for (int64_t j = 0; j < n; j++) {
    blo[j] = (o->ilo ? o->ilo[j] : l0[j]) / Dc[j];
    bhi[j] = (o->ihi ? o->ihi[j] : u0[j]) / Dc[j];
  }
  double ev[10], eva[10];
  evaluate(&P, x, y, Ax, ATy, omega, ev);
  double kkt_last = ev[0], kkt_prev = INFINITY;
  memcpy(xl, x, N8);
  memcpy(yl, y, M8);
  double wsum = 0.0;
  int64_t k = 0, accepted = 0, restarts = 0, last_restart = 0;
  int status = 0, which = 0;
  int P_eval = o->eval_period > 0 ? o->eval_period : 64;
  int64_t ntrace = 0;

  for (;;) {
    if (k % P_eval == 0 || k >= o->max_iter) {
      /* ---- evaluation: termination on the unscaled problem ---- */
      spmv_t(&P, y, ATy);
      evaluate(&P, x, y, Ax, ATy, omega, ev);
      int have_avg = o->use_average && wsum > 0.0;
      if (have_avg) {
        for (int64_t j = 0; j < n; j++) xa[j] = xs[j] / wsum;
        for (int64_t i = 0; i < m; i++) ya[i] = ys[i] / wsum;
        spmv(m, rp0, ci0, v, xa, Axa);
        spmv_t(&P, ya, ATya);
        evaluate(&P, xa, ya, Axa, ATya, omega, eva);
      }
      if (getenv("ORC_TRACE"))
        fprintf(stderr, "k=%lld cur kkt=%.3e (p %.2e d %.2e g %.2e) komega=%.3e avg kkt=%.3e komega=%.3e eta=%.3e omega=%.3e last=%.3e\n",
                (long long)k, ev[1], ev[4], ev[5], ev[6], ev[0], have_avg ? eva[1] : -1.0,
                have_avg ? eva[0] : -1.0, eta, omega, kkt_last);
      if (!isfinite(ev[1])) {
        status = ST_NUMERICAL;
        break;
      }
      /* the tested measure: [1] relative KKT, [4] primal, [5] dual residual */
      const int tq = o->term == 1 ? 4 : (o->term == 2 ? 5 : 1);
      if (ev[tq] <= o->tol) {
        status = ST_OPTIMAL;
        which = 0;
        break;
      }
      if (have_avg && eva[tq] <= o->tol) {
        status = ST_OPTIMAL;
        which = 1;
        break;
      }
      if (k >= o->max_iter) {
        status = ST_ITER_LIMIT;
        which = 0;
        break;
      }
      if (o->infeas_every > 0 && k > 0 && (k / P_eval) % o->infeas_every == 0 &&
          homogeneous_certificate(&P, y, blo, bhi, fylo, fyhi) > 0.0) {
        status = ST_PRIMAL_INFEASIBLE;
        which = 0;
        break;
      }
      if (o->infeas_every > 0 && o->dinf_eps > 0.0 && k > 0 && (k / P_eval) % o->infeas_every == 0 &&
          ray_certificate(&P, x, xl, blo, bhi, o->dinf_eps, ray)) {
        status = ST_DUAL_INFEASIBLE;
        which = 0;
        break;
      }
      /* ---- restart decision on the scaled KKT_omega ---- */
      double *rec = (o->trace && ntrace < o->trace_cap) ? o->trace + ORC_TRACE_LEN * ntrace : NULL;
      ntrace++;
      if (rec) {
        rec[0] = (double)k;
        rec[1] = ev[0];
        rec[2] = have_avg ? eva[0] : -1.0;
        rec[3] = kkt_last;
        rec[4] = kkt_prev;
        rec[5] = 0.0;
        rec[6] = 0.0;
        rec[7] = omega;
        rec[8] = -1.0;
      }
      if (o->restart && k > 0) {
        int cand_avg = have_avg && eva[0] < ev[0];
        double kc = cand_avg ? eva[0] : ev[0];
        int do_restart = (kc <= 0.2 * kkt_last) ||
                         (kc <= 0.8 * kkt_last && kc > kkt_prev) ||
                         ((double)(k - last_restart) >= 0.36 * (double)k);
        kkt_prev = kc;
        if (rec) rec[6] = cand_avg;
        if (do_restart) {
          if (cand_avg) {
            memcpy(x, xa, N8);
            memcpy(y, ya, M8);
            memcpy(Ax, Axa, M8);
            memcpy(ATy, ATya, N8);
            memcpy(ev, eva, sizeof ev);
          }
          double dx = 0.0, dy = 0.0;
          for (int64_t j = 0; j < n; j++) dx += (x[j] - xl[j]) * (x[j] - xl[j]);
          for (int64_t i = 0; i < m; i++) dy += (y[i] - yl[i]) * (y[i] - yl[i]);
          dx = sqrt(dx);
          dy = sqrt(dy);
          if (o->pw_theta > 0.0 && dx > 1e-10 && dy > 1e-10)
            omega = exp(o->pw_theta * log(dy / dx) + (1.0 - o->pw_theta) * log(omega));
          memcpy(xl, x, N8);
          memcpy(yl, y, M8);
          kkt_last = sqrt(omega * ev[7] + ev[8] / omega + ev[9] * ev[9]);
          kkt_prev = INFINITY;
          wsum = 0.0;
          last_restart = k;
          restarts++;
          if (rec) {
            rec[5] = 1.0;
            rec[7] = omega;
            rec[8] = kkt_last;
          }
        }
      }
    }

    /* ---- one attempt ---- */
    double tau = eta / omega, sigma = eta * omega;
    for (int64_t j = 0; j < n; j++) xn[j] = clampd(x[j] - tau * (c[j] - ATy[j]), l[j], u[j]);
    spmv(m, rp0, ci0, v, xn, Axn);
    for (int64_t i = 0; i < m; i++) {
      double yi = y[i] + sigma * (b[i] - (2.0 * Axn[i] - Ax[i]));
      if (kind[i] == 1 && yi < 0.0) yi = 0.0;
      yn[i] = yi;
    }
    k++;
    int accept = 1;
    double eta_used = eta;
    if (o->step_mode == 0) {
      double dx2 = 0.0, dy2 = 0.0, inter = 0.0;
      for (int64_t j = 0; j < n; j++) dx2 += (xn[j] - x[j]) * (xn[j] - x[j]);
      for (int64_t i = 0; i < m; i++) {
        dy2 += (yn[i] - y[i]) * (yn[i] - y[i]);
        inter += (yn[i] - y[i]) * (Axn[i] - Ax[i]);
      }
      double nz = omega * dx2 + dy2 / omega;
      double ebar = (inter != 0.0) ? nz / (2.0 * fabs(inter)) : INFINITY;
      double kk = (double)(k + 1);
      double e1 = (1.0 - pow(kk, -0.3)) * ebar;
      double e2 = (1.0 + pow(kk, -0.6)) * eta;
      accept = (eta <= ebar);
      eta = e1 < e2 ? e1 : e2;
    }
    if (accept) {
      double *t;
      t = x; x = xn; xn = t;
      t = y; y = yn; yn = t;
      t = Ax; Ax = Axn; Axn = t;
      spmv_t(&P, y, ATy);
      if (wsum == 0.0) {
        for (int64_t j = 0; j < n; j++) xs[j] = eta_used * x[j];
        for (int64_t i = 0; i < m; i++) ys[i] = eta_used * y[i];
      } else {
        for (int64_t j = 0; j < n; j++) xs[j] += eta_used * x[j];
        for (int64_t i = 0; i < m; i++) ys[i] += eta_used * y[i];
      }
      wsum += eta_used;
      accepted++;
    }
  }

  const double *xr = which ? xa : x, *yr = which ? ya : y;
  const double *er = which ? eva : ev;
  for (int64_t j = 0; j < n; j++) x_out[j] = status == ST_DUAL_INFEASIBLE ? ray[j] : Dc[j] * xr[j];
  for (int64_t i = 0; i < m; i++) {
    double yv = yr[i];
    if (status == ST_PRIMAL_INFEASIBLE) {  /* the certificate as the test took it */
      if (kind[i] == 1 && yv < 0.0) yv = 0.0;
      yv = fmin(fmax(yv, fylo[i]), fyhi[i]);
    }
    y_out[i] = Dr[i] * yv;
  }
  info[0] = status;
  info[1] = (double)k;
  info[2] = (double)accepted;
  info[3] = (double)restarts;
  info[4] = er[2];
  info[5] = er[3];
  info[6] = er[4];
  info[7] = er[5];
  info[8] = er[6];
  info[9] = er[1];
  info[10] = eta;
  info[11] = omega;
  info[12] = which;
  info[15] = (double)ntrace;

  free(v); free(Dr); free(Dc); free(cp); free(ri); free(vt);
  free(b); free(c); free(l); free(u); free(vk);
  free(x); free(y); free(Ax); free(ATy); free(xn); free(yn); free(Axn);
  free(xs); free(ys); free(xa); free(ya); free(Axa); free(ATya); free(xl); free(yl);
  free(ray); free(blo); free(bhi); free(fylo); free(fyhi);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* unrolled PDHG and its forward-mode derivative                          */

/* K fixed steps (tau = eta/omega, sigma = eta*omega) from x = clamp(0),
 * y = 0 on the scaled problem, no restarts and no averaging.
 * Returns V = c'x_K (original space) and, for a direction (db, dc) in the
 * original space, dV = dc'x_K + c'dx_K via the tangent recursion
 *   dx' = Mx .* (dx - tau dc^ + tau A^T dy)
 *   dy' = My .* (dy + sigma db^ - sigma A (2 dx' - dx))
 * with Mx = 1 where the pre-clamp value is strictly inside (l^, u^) and
 * My = 1 on equality rows and on >= rows whose pre-projection value > 0.
 * x_out, y_out (nullable) receive the unscaled x_K, y_K.
 * mask_flips_out (nullable) counts pre-clamp values within 1e-12 relative of a
 * bound (diagnostic for finite differences). */
int orc_unrolled(int64_t m, int64_t n, const int32_t *rp0, const int32_t *ci0,
                 const double *v0, const uint8_t *kind, const double *b0,
                 const double *c0, const double *l0, const double *u0, int ruiz_iters,
                 int pc, int64_t K, double eta, double omega, const double *db0,
                 const double *dc0, double *V_out, double *dV_out, double *x_out,
                 double *y_out) {
  int64_t nnz = rp0[m];
  double *v = malloc(sizeof(double) * (size_t)nnz);
  memcpy(v, v0, sizeof(double) * (size_t)nnz);
  double *Dr = malloc(sizeof(double) * (size_t)m), *Dc = malloc(sizeof(double) * (size_t)n);
  orc_scale(m, n, rp0, ci0, v, ruiz_iters, pc, Dr, Dc);
  int32_t *cp = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *ri = malloc(sizeof(int32_t) * (size_t)nnz);
  double *vt = malloc(sizeof(double) * (size_t)nnz);
  orc_transpose(m, n, rp0, ci0, v, cp, ri, vt);
  size_t N8 = sizeof(double) * (size_t)n, M8 = sizeof(double) * (size_t)m;
  double *b = malloc(M8), *c = malloc(N8), *l = malloc(N8), *u = malloc(N8);
  double *db = malloc(M8), *dc = malloc(N8);
  for (int64_t i = 0; i < m; i++) {
    b[i] = Dr[i] * b0[i];
    db[i] = db0 ? Dr[i] * db0[i] : 0.0;
  }
  for (int64_t j = 0; j < n; j++) {
    c[j] = Dc[j] * c0[j];
    dc[j] = dc0 ? Dc[j] * dc0[j] : 0.0;
    l[j] = l0[j] / Dc[j];
    u[j] = u0[j] / Dc[j];
  }
  double *x = malloc(N8), *y = calloc((size_t)m, sizeof(double));
  double *dx = calloc((size_t)n, sizeof(double)), *dy = calloc((size_t)m, sizeof(double));
  double *ATy = malloc(N8), *ATdy = malloc(N8), *xe = malloc(N8), *dxe = malloc(N8);
  double *Axe = malloc(M8), *Adxe = malloc(M8);
  for (int64_t j = 0; j < n; j++) x[j] = clampd(0.0, l[j], u[j]);
  double tau = eta / omega, sigma = eta * omega;
  for (int64_t k = 0; k < K; k++) {
    spmv(n, cp, ri, vt, y, ATy);
    spmv(n, cp, ri, vt, dy, ATdy);
    for (int64_t j = 0; j < n; j++) {
      double xt = x[j] - tau * (c[j] - ATy[j]);
      double xn = clampd(xt, l[j], u[j]);
      int inside = (xt > l[j]) && (xt < u[j]);
      double dxn = inside ? (dx[j] - tau * dc[j] + tau * ATdy[j]) : 0.0;
      xe[j] = 2.0 * xn - x[j];
      dxe[j] = 2.0 * dxn - dx[j];
      x[j] = xn;
      dx[j] = dxn;
    }
    spmv(m, rp0, ci0, v, xe, Axe);
    spmv(m, rp0, ci0, v, dxe, Adxe);
    for (int64_t i = 0; i < m; i++) {
      double yt = y[i] + sigma * (b[i] - Axe[i]);
      int free_row = (kind[i] == 0) || (yt > 0.0);
      y[i] = free_row ? yt : 0.0;
      dy[i] = free_row ? (dy[i] + sigma * db[i] - sigma * Adxe[i]) : 0.0;
    }
  }
  *V_out = dot(n, c, x);
  *dV_out = dot(n, dc, x) + dot(n, c, dx);
  if (x_out)
    for (int64_t j = 0; j < n; j++) x_out[j] = Dc[j] * x[j];
  if (y_out)
    for (int64_t i = 0; i < m; i++) y_out[i] = Dr[i] * y[i];
  free(v); free(Dr); free(Dc); free(cp); free(ri); free(vt);
  free(b); free(c); free(l); free(u); free(db); free(dc);
  free(x); free(y); free(dx); free(dy); free(ATy); free(ATdy); free(xe); free(dxe);
  free(Axe); free(Adxe);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* implied bounds and the safe dual bound                                 */

/* Feasibility-based bound propagation over the rows (an = row gives
 * a'x >= b and a'x <= b, a >= row only the first): with the other variables
 * at the ends of their current bounds, each row bounds each of its
 * variables.  Sweeps run over the rows in index order and use bounds found
 * earlier in the same sweep.  Only infinite bounds are replaced, and a
 * derived bound r = (b_i - sum over the others of t_k) / a_j is widened to
 * r -+ w with w = 2 (len + 2) 2^-53 (|b_i| + sum |t_k|) / |a_j| + 4 2^-53 |r|
 * (len = the row's entries, t_k the finite activity terms), which exceeds
 * the rounding of r even where the terms cancel; a non-finite r or w gives
 * no bound.  lo, hi: in the bounds l, u; out the implied bounds.  Returns
 * the number of bounds made finite. */
int64_t orc_implied_bounds(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                           const double *v, const uint8_t *kind, const double *b,
                           int passes, double *lo, double *hi) {
  const double eps = ldexp(1.0, -53);
  int64_t made = 0;
  (void)n;
  for (int pass = 0; pass < passes; pass++) {
    int64_t before = made;
    for (int64_t i = 0; i < m; i++) {
      /* activity bounds of row i: finite parts, their magnitudes and counts of
       * infinite terms */
      double minf = 0.0, maxf = 0.0, mina = 0.0, maxa = 0.0;
      int64_t mininf = 0, maxinf = 0;
      const int64_t len = rp[i + 1] - rp[i];
      for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
        double a = v[k], L = lo[ci[k]], U = hi[ci[k]];
        double tmin = a > 0.0 ? a * L : a * U, tmax = a > 0.0 ? a * U : a * L;
        if (isinf(tmin)) mininf++; else { minf += tmin; mina += fabs(tmin); }
        if (isinf(tmax)) maxinf++; else { maxf += tmax; maxa += fabs(tmax); }
      }
      for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
        int32_t j = ci[k];
        double a = v[k], L = lo[j], U = hi[j];
        if (a == 0.0) continue;
        double tmin = a > 0.0 ? a * L : a * U, tmax = a > 0.0 ? a * U : a * L;
        /* a'x >= b: a_j x_j >= b - (max activity of the others).  The
         * computed r carries the rounding of the products, the row sum, the
         * removal of the own term, the subtraction from b and the division:
         * below 2 (len + 2) 2^-53 (|b_i| + sum |t_k|) / |a_j| + 2^-53 |r|;
         * w exceeds it, and 4 2^-53 |r| also covers the rounding of r -+ w */
        int64_t oinf = maxinf - (isinf(tmax) ? 1 : 0);
        if (oinf == 0) {
          double r = (b[i] - (maxf - (isinf(tmax) ? 0.0 : tmax))) / a;
          double w = 2.0 * (double)(len + 2) * eps * (fabs(b[i]) + maxa) / fabs(a) +
                     4.0 * eps * fabs(r);
          if (isfinite(r) && isfinite(w)) {
            if (a > 0.0 && isinf(lo[j])) { lo[j] = r - w; made++; }
            if (a < 0.0 && isinf(hi[j])) { hi[j] = r + w; made++; }
          }
        }
        if (kind[i] == 0) { /* a'x <= b: a_j x_j <= b - (min activity of the others) */
          int64_t oinf2 = mininf - (isinf(tmin) ? 1 : 0);
          if (oinf2 == 0) {
            double r = (b[i] - (minf - (isinf(tmin) ? 0.0 : tmin))) / a;
            double w = 2.0 * (double)(len + 2) * eps * (fabs(b[i]) + mina) / fabs(a) +
                       4.0 * eps * fabs(r);
            if (isfinite(r) && isfinite(w)) {
              if (a > 0.0 && isinf(hi[j])) { hi[j] = r + w; made++; }
              if (a < 0.0 && isinf(lo[j])) { lo[j] = r - w; made++; }
            }
          }
        }
      }
    }
    if (made == before) break;
  }
  return made;
}

/* Dual repair for the bound (reading of the safe-bound row): a column with a
 * single nonzero a_ij whose bound on one side is infinite (a penalty slack
 * with no upper limit) constrains y_i: u_j = +inf needs
 * lambda_j = c_j - a_ij y_i >= 0, l_j = -inf needs lambda_j <= 0.  Each such
 * constraint is a half-line for y_i with end t = c_j / a_ij, moved inward by
 * 2^-40 |t| so that the repaired lambda_j clears its rounding error; the
 * interval of row i is the intersection of its half-lines (and of y_i >= 0
 * on >= rows).  An empty intersection gives no repair.  lo, hi are the
 * bounds used for the bound (l, u tightened by the implied ones).  Returns
 * the number of rows whose interval is narrower than the sign constraint. */
int64_t orc_bound_repair(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                         const double *v, const uint8_t *kind, const double *c,
                         const double *lo, const double *hi, double *ylo, double *yhi) {
  int64_t *cnt = calloc((size_t)n, sizeof(int64_t));
  int64_t *row = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  double *val = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < m; i++)
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      cnt[ci[k]]++;
      row[ci[k]] = i;
      val[ci[k]] = v[k];
    }
  for (int64_t i = 0; i < m; i++) {
    ylo[i] = kind[i] == 1 ? 0.0 : -INFINITY;
    yhi[i] = INFINITY;
  }
  const double margin = ldexp(1.0, -40);
  for (int64_t j = 0; j < n; j++) {
    if (cnt[j] != 1 || val[j] == 0.0) continue;
    const int64_t i = row[j];
    const double a = val[j], t = c[j] / a;
    /* u_j = +inf: a y_i <= c_j; l_j = -inf: a y_i >= c_j */
    if (isinf(hi[j])) {
      if (a > 0.0) yhi[i] = fmin(yhi[i], t - margin * fabs(t));
      else ylo[i] = fmax(ylo[i], t + margin * fabs(t));
    }
    if (isinf(lo[j])) {
      if (a > 0.0) ylo[i] = fmax(ylo[i], t + margin * fabs(t));
      else yhi[i] = fmin(yhi[i], t - margin * fabs(t));
    }
  }
  int64_t fin = 0;
  for (int64_t i = 0; i < m; i++) {
    if (ylo[i] > yhi[i]) {
      ylo[i] = kind[i] == 1 ? 0.0 : -INFINITY;
      yhi[i] = INFINITY;
    }
    if (yhi[i] < INFINITY || ylo[i] > (kind[i] == 1 ? 0.0 : -INFINITY)) fin++;
  }
  free(cnt);
  free(row);
  free(val);
  return fin;
}

/* A lower bound on the LP optimum from any y (weak duality).  With ytil the
 * y projected on y_i >= 0 for >= rows and clamped into [ylo_i, yhi_i] (any
 * such ytil will do; ylo/yhi may be NULL), every feasible x has
 *   c'x = b'ytil + ytil'(Ax - b) + lambda'x >= b'ytil + sum_j lambda_j x_j,
 * lambda = c - A'ytil, and x_j in [lo_j, hi_j] bounds the last sum from below
 * by min(lambda_j lo_j, lambda_j hi_j).  lambda_j is computed as
 * c_j - sum_i a_ij ytil_i in ascending i, each product rounded on its own;
 * its rounding error is below err_j = 2 (k_j + 2) eps (|c_j| + sum_i
 * |a_ij ytil_i|) (k_j entries in column j, eps = 2^-53).  Its sign is taken
 * as known when |lambda_j| > err_j (or err_j = 0): the term is lambda_j times
 * the bound that sign selects.  Otherwise the term is min(lambda_j lo_j,
 * lambda_j hi_j) with both bounds finite.  A needed infinite bound makes the
 * bound -INFINITY.  The computed value is lowered by 2 (K + 4) eps S with
 * K = n + m + (longest column) and S = sum_i |b_i ytil_i| + sum_j B_j (|c_j|
 * + sum_i |a_ij ytil_i|), B_j the bound used (both: the larger magnitude),
 * which exceeds the rounding error of everything summed.  out: [0] bound,
 * [1] value before the allowance, [2] the allowance, [3] number of needed
 * infinite bounds, [4] number of rows whose y the repair changed. */
void orc_safe_bound(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                    const double *v, const uint8_t *kind, const double *b, const double *c,
                    const double *lo, const double *hi, const double *ylo, const double *yhi,
                    const double *y, double *out) {
  double *aty = calloc((size_t)n, sizeof(double));
  double *atyabs = calloc((size_t)n, sizeof(double));
  int64_t *clen = calloc((size_t)n, sizeof(int64_t));
  double by = 0.0, byabs = 0.0;
  int64_t repaired = 0;
  for (int64_t i = 0; i < m; i++) {
    double yi = (kind[i] == 1 && y[i] < 0.0) ? 0.0 : y[i];
    if (ylo && yhi) {
      double yc = fmin(fmax(yi, ylo[i]), yhi[i]);
      if (yc != yi) repaired++;
      yi = yc;
    }
    double t = b[i] * yi;
    by += t;
    byabs += fabs(t);
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      double p = v[k] * yi;
      aty[ci[k]] += p;
      atyabs[ci[k]] += fabs(p);
      clen[ci[k]]++;
    }
  }
  const double eps = ldexp(1.0, -53);
  double terms = 0.0, sabs = 0.0;
  int64_t ninf = 0, kmax = 0;
  for (int64_t j = 0; j < n; j++) {
    if (clen[j] > kmax) kmax = clen[j];
    const double lam = c[j] - aty[j];
    const double mag = fabs(c[j]) + atyabs[j];
    const double err = 2.0 * (double)(clen[j] + 2) * eps * mag;
    if (fabs(lam) > err || err == 0.0) {
      if (lam == 0.0) continue;
      const double bnd = lam > 0.0 ? lo[j] : hi[j];
      if (isinf(bnd)) {
        ninf++;
        continue;
      }
      terms += lam * bnd;
      sabs += fabs(bnd) * mag;
    } else if (isinf(lo[j]) || isinf(hi[j])) {
      ninf++;
    } else {
      terms += fmin(lam * lo[j], lam * hi[j]);
      sabs += fmax(fabs(lo[j]), fabs(hi[j])) * mag;
    }
  }
  double val = by + terms;
  double allow = 2.0 * (double)(n + m + kmax + 4) * eps * (byabs + sabs);
  out[0] = ninf ? -INFINITY : val - allow;
  out[1] = val;
  out[2] = allow;
  out[3] = (double)ninf;
  out[4] = (double)repaired;
  free(aty);
  free(atyabs);
  free(clen);
}
