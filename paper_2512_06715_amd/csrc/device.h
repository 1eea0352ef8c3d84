// Device helpers shared by the iteration kernels (attempt.hip, iterate.hip).
#pragma once
#include "internal.h"

#include <math.h>

namespace {

// Address spaces.  Pointers read out of the instance tables are generic; the
// attempt kernels cast them so that the compiler emits global (vector) and
// scalar loads instead of flat ones, whose shared wait counter serialises
// the otherwise independent load streams.  Instance tables, control states
// and CSR pointers are not written while an attempt kernel runs, so their
// uniform reads may go through the scalar path.
#define AS_G __attribute__((address_space(1)))
#define AS_C __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const AS_G T *gin(const T *p) {
  return (const AS_G T *)p;
}
template <typename T>
__device__ __forceinline__ AS_G T *gout(T *p) {
  return (AS_G T *)p;
}
template <typename T>
__device__ __forceinline__ const AS_C T *cin(const T *p) {
  return (const AS_C T *)p;
}


inline unsigned grid_of(int n) { return (unsigned)(n > 0 ? n : 1); }
inline unsigned grid_for(int64_t n) {
  int64_t g = (n + PDHG_BLOCK - 1) / PDHG_BLOCK;
  return (unsigned)(g > 0 ? g : 1);
}

// The hardware hands consecutive workgroups to the 8 XCDs in turn.  Map them
// so that each XCD works on one contiguous range of logical blocks, which keeps
// the gathered vector windows of neighbouring rows inside one L2.
__device__ inline int xcd_remap(int b, int nb) {
  int xcd = b & 7, local = b >> 3;
  int per = nb >> 3, rem = nb & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Instance owning logical block b: the largest i with pre[i] <= b.
__device__ inline int find_inst(const int32_t *pre, int ninst, int b) {
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pre[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename T>
__device__ inline T clamp_box(T x, T lo, T hi) {
  // explicit comparisons keep NaN visible (fmin/fmax would drop it)
  return x < lo ? lo : (x > hi ? hi : x);
}

// Deterministic block reduction of NQ doubles (fixed shuffle tree, then the
// waves in order).  Bit q of maxmask selects max instead of sum.
template <int NQ, int BS = PDHG_BLOCK>
__device__ inline void block_reduce(double (&v)[NQ], unsigned maxmask, double *out) {
  __shared__ double lds[BS / 64][NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    double a = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_down(a, off, 64);
      a = ((maxmask >> q) & 1) ? fmax(a, o) : a + o;
    }
    v[q] = a;
  }
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; q++) lds[wid][q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      double a = lds[0][q];
      for (int w = 1; w < BS / 64; w++)
        a = ((maxmask >> q) & 1) ? fmax(a, lds[w][q]) : a + lds[w][q];
      out[q] = a;
    }
  }
  __syncthreads();
}

// Sum (or max) of `cnt` partials with stride `stride`, one workgroup of BS
// threads, fixed order: lane t combines partials t, t + BS, t + 2 BS, ... in
// that order, then the block tree combines the lanes.  Loads go out CH per
// lane at a time before any of them is used.
#define CTL_BLOCK 1024
static_assert(sizeof(CtlState) % 8 == 0, "the state is copied in 8-byte words");
// Whole-state write-back (8-byte words) from one lane.
__device__ inline void store_state(CtlState *dst, const CtlState &s) {
  AS_G unsigned long long *d = gout((unsigned long long *)dst);
  const unsigned long long *w = (const unsigned long long *)&s;
#pragma unroll
  for (int q = 0; q < (int)(sizeof(CtlState) / 8); q++) d[q] = w[q];
}

template <int NQ, int BS = CTL_BLOCK>
__device__ inline void reduce_partials(const double *p, int64_t cnt, int64_t stride,
                                       unsigned maxmask, double *out) {
  constexpr int CH = NQ >= 8 ? 2 : 16 / NQ;
  const AS_G double *pg = gin(p);
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) v[q] = 0.0;
  for (int64_t b0 = 0; b0 < cnt; b0 += CH * BS) {
    double a[CH][NQ];
#pragma unroll
    for (int c = 0; c < CH; c++) {
      int64_t b = b0 + c * BS + threadIdx.x;
      int64_t bc = b < cnt ? b : cnt - 1;
#pragma unroll
      for (int q = 0; q < NQ; q++) a[c][q] = pg[q * stride + bc];
    }
#pragma unroll
    for (int c = 0; c < CH; c++) {
      bool ok = b0 + c * BS + threadIdx.x < cnt;
#pragma unroll
      for (int q = 0; q < NQ; q++)
        v[q] = ((maxmask >> q) & 1) ? fmax(v[q], ok ? a[c][q] : v[q]) : v[q] + (ok ? a[c][q] : 0.0);
    }
  }
  block_reduce<NQ, BS>(v, maxmask, out);
}

// Instance owning logical block b (uniform): the largest i with pre[i] <= b.
__device__ inline int find_inst_u(const int32_t *pre, int ninst, int b) {
  const AS_C int32_t *p = cin(pre);
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (p[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace
