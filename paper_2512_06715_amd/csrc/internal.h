// Internal declarations shared by the HIP translation units of libpdhg.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#define PDHG_BLOCK 256
// rows of one tile of the attempt kernels (and their workgroup size)
#ifndef PDHG_TILE
#define PDHG_TILE 256
#endif
// workgroups per instance of the step-control kernel
#define PDHG_CTL_SPLIT 16
// partials of each kind (attempt workgroups) up to which one control
// workgroup reduces an instance alone
#define PDHG_CTL_SOLO 4096
// instances per workgroup of the attempt kernels when instances share a matrix
#define PDHG_PACK 4
// default length above which a row / column is handled by a workgroup
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
  double best_kkt;        // FP32 phase: lowest KKT of an evaluated current iterate
  double dual_bound;      // weak-duality lower bound from the reported point's y
  long long k, accepted, restarts, last_restart;
  int cur;                // buffer index of the current iterate
  int fresh;              // 1: the next fold starts the sums afresh
  int done, status, which;
  int restart_flag;       // 0 none, 1 restart at current, 2 restart to average
  int have_avg;
  int init_pending;       // 1: the next evaluation records the restart reference
  int ticket;             // step-control workgroups done with the current attempt
  int stash;              // FP32 phase: the evaluated current iterate is a new best
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
  double *ctl_stage;             // [3 * PDHG_CTL_SPLIT] slice sums of the step control
  int adaptive;
  int long_seg;                  // rows longer than this get a workgroup each
  int direct;                    // 1: per-row loops instead of LDS-staged tiles
  // 16-bit tile-relative form of both matrices' structure (null when some
  // tile does not fit): per row, the end of its nonzeros counted from the
  // tile's first nonzero; per nonzero, its index minus the tile's smallest
  // one; per tile, that smallest index
  const uint16_t *rofs, *cofs, *cix16, *rix16;
  const int32_t *tb_rows, *tb_cols;
  // unrolled-mode recording: when non-null, attempt k - mask_k0 writes its
  // projection masks (bit j: pre-clamp x strictly inside the box; bit i:
  // equality row or pre-projection y > 0) into words [(k - mask_k0) * words]
  uint64_t *mask_x, *mask_y;
  int64_t mask_k0;
  // FP32 copies of the matrix values (mixed handles; null otherwise), which
  // FP64 iterates multiply when use_v32 is set (the mixed path's FP64 phase
  // with opts.polish_fp32_matrix)
  const float *v32, *vt32;
  int use_v32;
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
  double *ev_stage;              // [(EV_ROWQ + EV_COLQ) * PDHG_CTL_SPLIT] slice results
  // FP32 phase: the best evaluated iterate, kept in FP64 (the FP64 phase's
  // start buffers); null in the FP64 views
  double *xbest, *ybest;
  // implied bounds (scaled, internal order) for the dual bound; null: use l, u
  const double *ilo, *ihi;
  // the dual bound's repair interval of each row (scaled, internal order);
  // null: no repair
  const double *rylo, *ryhi;
  double bound_allow;            // rounding allowance factor 2 (n + m + longest column + 4) 2^-53
  int use_average, restart;
  double pw_theta;               // 0 keeps the primal weight
  long long hold_k;              // no primal-weight update before this attempt
  long long infeas_period;       // attempts between infeasibility tests (0: none)
  double dinf_tol;               // tolerance of the ray test at those (0: no ray test)
  int long_seg;
  // caller's index of each internal row / column (null: same order)
  const int32_t *rperm, *cperm;
  // the quantity the termination test holds to the tolerance: 0 the relative
  // KKT error, 1 the relative primal residual, 2 the relative dual residual
  // (feasibility polishing)
  int term;
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
void launch_compact(const int32_t *ptr, const int32_t *idx, int64_t rows, uint16_t *rofs,
                    uint16_t *ix16, int32_t *tb, int *fail, hipStream_t s);
void launch_scale_pass(int32_t *rp, int32_t *ci, double *v, int32_t *cp, int32_t *ri,
                       double *vt, int64_t m, int64_t n, int pc, double *rs, double *cs,
                       double *Dr, double *Dc, hipStream_t s);
void launch_scale_vectors(const double *b0, const double *c0, const double *l0,
                          const double *u0, const double *Dr, const double *Dc,
                          int64_t m, int64_t n, double *b, double *c, double *l,
                          double *u, hipStream_t s);
void launch_fill(double *p, double v, int64_t n, hipStream_t s);
// dst[j] = 0 where src[j] is finite, src[j] (an infinite bound) elsewhere
void launch_zero_finite(const double *src, double *dst, int64_t n, hipStream_t s);
// merge-path SpMV (spmv_merge.hip)
int merge_workgroups(int64_t m, int64_t nnz);
size_t merge_workspace_bytes(int64_t m, int64_t nnz);
void launch_merge_check(const int32_t *rp, const int32_t *ci, int64_t m, int64_t n, int64_t nnz,
                        int *bad, hipStream_t s);
void launch_merge_plan(const int32_t *rp, int64_t m, int64_t nnz, void *ws, hipStream_t s);
template <typename T>
void launch_spmv_merge(const int32_t *rp, const int32_t *ci, const T *v, const T *x, T *y,
                       int64_t m, int64_t nnz, void *ws, hipStream_t s);

void launch_fix_bounds(double *l, double *u, const int32_t *idx, const double *val, int64_t nfix,
                       const int32_t *inv, int64_t n,
                       hipStream_t s);
void launch_copy_i32(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s);
void launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t s);

// implied bounds by row propagation (implied.hip)
int64_t implied_bounds(int64_t m, const int32_t *rp, const int32_t *ci, const double *v,
                       const uint8_t *kind, const double *b, int passes, double *lo, double *hi);

// locality ordering (reorder.hip)
void rcm_order(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *cp,
               const int32_t *ri, std::vector<int32_t> &row_order, std::vector<int32_t> &col_order);
void permute_csr(int64_t m, const int32_t *rp, const int32_t *ci, const double *v,
                 const std::vector<int32_t> &row_order, const std::vector<int32_t> &cinv,
                 std::vector<int32_t> &prp, std::vector<int32_t> &pci, std::vector<double> &pv);
void unpermute_csr(int64_t m, const int32_t *prp, const int32_t *pci, const double *pv,
                   const std::vector<int32_t> &row_order, const std::vector<int32_t> &col_order,
                   std::vector<int32_t> &rp, std::vector<int32_t> &ci, std::vector<double> &v);
void transpose_csr(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                   std::vector<int32_t> &cp, std::vector<int32_t> &ri, std::vector<double> &vt);
// dst[i] = src[order[i]] (gather) / dst[order[i]] = src[i] (scatter)
void launch_gather_f64(double *dst, const double *src, const int32_t *order, int64_t cnt,
                       hipStream_t s);
void launch_gather_u8(uint8_t *dst, const uint8_t *src, const int32_t *order, int64_t cnt,
                      hipStream_t s);
void launch_scatter_f64(double *dst, const double *src, const int32_t *order, int64_t cnt,
                        hipStream_t s);

// One instance of a (possibly batched) solve: views of its problem data and
// iterates, its control state, start point and result buffers.
template <typename T>
struct Inst {
  IterView<T> w;
  EvalView<T> e;
  CtlState *st;
  const double *x0, *y0;  // start point, original space (device) or null
  double *xout, *yout;    // unscaled result (device)
  // Farkas repair per row, bit 0 y >= 0, bit 1 y <= 0 (nullable); last, so
  // the fields the attempt kernels read keep their offsets
  const uint8_t *fyk;
};

// Block-to-instance maps of a grouped launch: exclusive prefix sums of each
// instance's block count for every kernel shape (device memory, ninst + 1
// entries); the totals are the grid sizes.
struct Groups {
  int ninst;
  const int32_t *p_primal, *p_dual;  // attempt kernels
  const int32_t *p_rows, *p_cols;    // one block per 256 rows / columns
  const int32_t *p_lrows, *p_lcols;  // one block per long row / column
  int n_primal, n_dual, n_rows, n_cols, n_lrows, n_lcols;
  // 1: every instance has the same matrix and attempt grids; the attempt
  // kernels then number blocks tile-major (block b is local block b / ninst
  // of instance b % ninst), so the instances' blocks of one tile run back to
  // back on one XCD and its L2 serves the shared matrix tile once
  int interleave;
  // 1: every instance has the 16-bit structure; the attempt kernels read it
  int compact;
  // > 0: instances sharing one matrix (interleave, 16-bit structure, one
  // tile per workgroup, LDS-staged tiles, no mask recording) are walked
  // PDHG_PACK at a time by the pack kernels, whose grids are these
  int pack;
  int n_primal_pack, n_dual_pack;
  // 1: the attempt kernels stream the matrix and the read-once vectors with
  // non-temporal loads; 0: ordinary loads
  int nt;
  // 1: FP64 iterates multiply the FP32 matrix values (every instance has
  // use_v32 set)
  int v32;
};

// ---------------------------------------------------------------------------
// launchers (iterate.hip); every launch covers all instances of the group
template <typename T>
void launch_primal(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
template <typename T>
void launch_dual(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
template <typename T>
void launch_control(const Inst<T> *I, const Groups &g, hipStream_t s, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
template <typename T>
void launch_attempt(const Inst<T> *I, const Groups &g, hipStream_t s);
template <typename T>
void launch_evaluate(const Inst<T> *I, const Groups &g, double tol, int64_t max_iter,
                     hipStream_t s);
template <typename T>
void launch_bound(const Inst<T> *I, const Groups &g, hipStream_t s);
template <typename T>
void launch_init_point(const Inst<T> *I, const Groups &g, hipStream_t s);
void launch_switch_to_fp64(const Inst<float> *If, const Inst<double> *Id, const Groups &g,
                           hipStream_t s);
template <typename T>
void launch_unscale(const Inst<T> *I, const Groups &g, hipStream_t s);
// Adjoint of unrolled PDHG (FP64): one reverse step with the masks of the
// forward step it undoes.
struct AdjView {
  int64_t m, n;
  const int32_t *rp, *ci, *cp, *ri;
  const double *v, *vt;
  const int32_t *long_rows, *long_cols;
  int n_long_rows, n_long_cols;
  int nblk_rows, nblk_cols;
  int long_seg;
  const uint64_t *mask_x, *mask_y;  // this step's masks
  double *XB, *YB, *H, *BB, *CB;     // x-bar, y-bar, h, b-bar, c-bar
  double tau, sigma;
};
void launch_adjoint_step(const AdjView &a, hipStream_t s);
void launch_fill_u64(uint64_t *p, int64_t n, hipStream_t s);
void launch_copy_f64(double *dst, const double *src, int64_t n, hipStream_t s);
void launch_axpby(double *y, const double *x, double alpha, double beta, int64_t n,
                  hipStream_t s);
double *launch_sumsq(const double *x, int64_t n, double *scratch, int nscratch, hipStream_t s);
template <typename T>
void launch_checkpoint(const Inst<T> *I, const Groups &g, double *cx, double *cy, double *cax,
                       int restore, hipStream_t s);

template <typename T>
void launch_gather_states(const Inst<T> *I, int n, CtlState *out, hipStream_t s);
void launch_init_ctl(const double *v, int64_t nnz, const double *b, const double *c,
                     const double *b0, const double *c0, int64_t m, int64_t n,
                     double *scratch, int nscratch, CtlState *st, int step_mode,
                     double fixed_eta, double fixed_omega, hipStream_t s);
void launch_spmv(const int32_t *rp, const int32_t *ci, const double *v, int64_t rows,
                 const double *x, double *y, hipStream_t s);
