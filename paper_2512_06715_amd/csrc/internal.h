// Internal declarations shared by the HIP translation units of libpdhg.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PDHG_BLOCK 256
// rows / columns longer than this are handled by a workgroup each
#define PDHG_LONG_SEG 64
// tile groups per launch above which a workgroup takes several tiles
#define PDHG_TARGET_GROUPS 65536
// columns longer than this are sorted with a workgroup during the transpose
#define PDHG_SORT_SHORT 32

enum { VK_FREE = 0, VK_LOWER = 1, VK_UPPER = 2, VK_BOXED = 3, VK_FIXED = 4 };

// Error bits raised by the device-side validation kernels.
enum { VERR_CSR = 1, VERR_BOUNDS = 2, VERR_NONFINITE = 4, VERR_KIND = 8 };

// Control state of one solve.  Lives in device memory; the control kernels
// own it and the host only reads it between iteration blocks.
struct CtlState {
  double eta, omega;      // current step size and primal weight
  double pending;         // weight of the accepted iterate not yet folded into the sums
  double wsum;            // sum of weights in the current restart epoch
  double kkt_last;        // KKT_omega of the last restart point
  double kkt_prev;        // KKT_omega of the previous evaluation's candidate
  double nb, nc;          // ||b||, ||c|| of the original problem
  double eta0, omega0;
  // report of the last evaluation (for the point the solve would return)
  double pobj, dobj, rel_p, rel_d, rel_gap, rel_kkt;
  // last attempt's reduced partials (diagnostics)
  double dx2, dy2, inter;
  long long k, accepted, restarts, last_restart;
  int cur;                // buffer index of the current iterate
  int fresh;              // 1: the next fold starts the sums afresh
  int done, status, which;
  int restart_flag;       // 0 none, 1 restart at current, 2 restart to average
  int have_avg;
  int init_pending;       // 1: the next evaluation records the restart reference
};

// One precision's view of the scaled problem and iterates.
template <typename T>
struct IterView {
  int64_t m, n;
  const int32_t *rp, *ci, *cp, *ri;
  const T *v, *vt;
  const T *b, *c, *l, *u;
  const uint8_t *kind, *vk;
  T *X[2], *Y[2], *AX[2];
  T *XS, *YS;
  int nblk_rows, nblk_cols;      // 256-row tiles
  const int32_t *long_rows, *long_cols;
  int n_long_rows, n_long_cols;
  int tpb_rows, tpb_cols;        // tiles per workgroup
  int grid_rows, grid_cols;      // long segments + tile groups
  double *part_dx2;              // [grid_cols]
  double *part_dy;               // [2 * grid_rows]
  int adaptive;
};

// FP64 evaluation view (always FP64 matrix); iterates of type T.
template <typename T>
struct EvalView {
  int64_t m, n;
  const int32_t *rp, *ci, *cp, *ri;
  const double *v, *vt;
  const double *b, *c, *l, *u, *Dr, *Dc;
  const uint8_t *kind, *vk;
  T *X[2], *Y[2], *AX[2];
  T *XS, *YS;
  double *XA, *YA, *AXA, *ATY, *ATYA, *XL, *YL;
  int nblk_rows, nblk_cols;
  double *part_rows;             // [nblk_rows * EV_ROWQ]
  double *part_cols;             // [nblk_cols * EV_COLQ]
  int use_average, restart;
  double pw_theta;               // 0 keeps the primal weight
};

#define EV_ROWQ 10
#define EV_COLQ 12

// ---------------------------------------------------------------------------
// launchers (setup.hip)
void launch_validate(const int32_t *rp, const int32_t *ci, const double *v,
                     const uint8_t *kind, const double *b, const double *c,
                     const double *l, const double *u, int64_t m, int64_t n,
                     int64_t nnz, int *err, hipStream_t s);
void launch_var_kind(const double *l, const double *u, int64_t n, uint8_t *vk,
                     hipStream_t s);
void launch_transpose(const int32_t *rp, const int32_t *ci, const double *v,
                      int64_t m, int64_t n, int64_t nnz, int32_t *cp, int32_t *ri,
                      double *vt, int32_t *tmp_next, int32_t *scan_tmp, hipStream_t s);
int64_t scan_tmp_ints(int64_t len);
void launch_scale_pass(int32_t *rp, int32_t *ci, double *v, int32_t *cp, int32_t *ri,
                       double *vt, int64_t m, int64_t n, int pc, double *rs, double *cs,
                       double *Dr, double *Dc, hipStream_t s);
void launch_scale_vectors(const double *b0, const double *c0, const double *l0,
                          const double *u0, const double *Dr, const double *Dc,
                          int64_t m, int64_t n, double *b, double *c, double *l,
                          double *u, hipStream_t s);
void launch_fill(double *p, double v, int64_t n, hipStream_t s);
void launch_copy_i32(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s);
void launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// launchers (iterate.hip)
template <typename T>
void launch_attempt(const IterView<T> &w, CtlState *st, int64_t max_iter, hipStream_t s);
template <typename T>
void launch_primal(const IterView<T> &w, CtlState *st, hipStream_t s);
template <typename T>
void launch_dual(const IterView<T> &w, CtlState *st, hipStream_t s);
template <typename T>
void launch_control(const IterView<T> &w, CtlState *st, hipStream_t s);
template <typename T>
void launch_evaluate_ll(const EvalView<T> &e, const int32_t *long_rows, int n_long_rows,
                        const int32_t *long_cols, int n_long_cols, CtlState *st, double tol,
                        int64_t max_iter, hipStream_t s);
template <typename T>
void launch_init_point(const EvalView<T> &e, const int32_t *long_rows, int n_long_rows,
                       const double *x0, const double *y0, CtlState *st, double *ax_tmp,
                       hipStream_t s);
void launch_switch_to_fp64(const EvalView<float> &ef, const EvalView<double> &ed,
                           const int32_t *long_rows, int n_long_rows, CtlState *st,
                           hipStream_t s);
template <typename T>
void launch_unscale(const EvalView<T> &e, const CtlState *st, double *x, double *y,
                    hipStream_t s);
void launch_init_ctl(const double *v, int64_t nnz, const double *b, const double *c,
                     const double *b0, const double *c0, int64_t m, int64_t n,
                     double *scratch, int nscratch, CtlState *st, int step_mode,
                     double fixed_eta, double fixed_omega, hipStream_t s);
void launch_spmv(const int32_t *rp, const int32_t *ci, const double *v, int64_t rows,
                 const double *x, double *y, hipStream_t s);
