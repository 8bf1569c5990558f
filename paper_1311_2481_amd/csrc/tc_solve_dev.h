// Device helpers shared by the banded-solve kernels (tc_solve.hip) and the
// fused adjoint sweeps (tc_adjoint_pc.hip): complex arithmetic, factor
// addressing, the operator rows, the running elimination and the lane
// layout of the four-sweep kernels.
#pragma once
#include "tc_internal.h"

namespace tc {

__device__ __forceinline__ cd cz() { return cd{0.0, 0.0}; }
__device__ __forceinline__ cd cfma(cd acc, double w, cd v) { return cd{fma(w, v.x, acc.x), fma(w, v.y, acc.y)}; }
__device__ __forceinline__ cd cnfma(cd acc, double w, cd v) { return cd{fma(-w, v.x, acc.x), fma(-w, v.y, acc.y)}; }
__device__ __forceinline__ cd cmuls(cd v, double w) { return cd{v.x * w, v.y * w}; }
// i * w * v
__device__ __forceinline__ cd cimul(cd v, double w) { return cd{-w * v.y, w * v.x}; }

__device__ __forceinline__ const double* facp(const double* fac, const Dims& d, int op, int j) {
  return fac + ((int64_t)(op * d.n_r + j) * NFAC) * d.ndm;
}

// Row j of operator op in natural column order: entry k multiplies node j+k-4.
// Evaluated without contraction, like the elimination below, so that the
// sweeps that rebuild factors on the fly reproduce the stored ones exactly.
__device__ __forceinline__ void operator_row(const double* rc, const Dims& d, int op, int j, double a, double b,
                                             double* row) {
#pragma clang fp contract(off)
  const double* R = rc + (int64_t)j * RC_N;
  const int M = d.n_r - 1;
  const bool wall = (j == 0 || j == M);
  if (op == OP_P) {
    if (wall) {
      if (j == M && a == 0.0 && b == 0.0) {
        for (int k = 0; k < NB9; ++k) row[k] = (k == HW) ? 1.0 : 0.0;
      } else {
        const double s = (j == 0) ? d.s0 : d.sM;
        for (int k = 0; k < NB9; ++k) row[k] = s * R[RC_W1 + k];
      }
      return;
    }
  } else if (wall) {
    for (int k = 0; k < NB9; ++k) row[k] = (k == HW) ? 1.0 : 0.0;
    return;
  }
  for (int k = 0; k < NB9; ++k) row[k] = R[RC_W2 + k] + R[RC_W1 + k] * R[RC_IR];
  double diag = -(a * a) * R[RC_IR2] - b * b;
  if (op == OP_HP) diag += -(1.0 + 2.0 * a) * R[RC_IR2] - 1.5 / d.dt;
  if (op == OP_HM) diag += -(1.0 - 2.0 * a) * R[RC_IR2] - 1.5 / d.dt;
  if (op == OP_HZ) diag += -1.5 / d.dt;
  row[HW] += diag;
}

// Running factorization of one operator in its processing order (ascending
// rows for P, descending for the Helmholtz operators): U[q] is the U-row of
// the row q+1 places earlier, its inverse pivot in U[q][0] and the 4
// entries after the pivot in U[q][1..4].
struct Elim {
  double U[4][5];
  __device__ __forceinline__ void reset() {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 5; ++c) U[q][c] = 0.0;
  }
  // Next row: ip = its place in processing order, row its entries in
  // processing column order (entry HW on the diagonal).  Gives the
  // multipliers of the 4 previous rows (mult[q-1]: the row q places
  // earlier, the eliminated entry times that row's inverse pivot), leaves
  // the row's pivot and the entries after it in row[HW .. HW+4] and its
  // inverse pivot and those entries in U[0].
  __device__ __forceinline__ void next(double (&row)[NB9], int ip, double (&mult)[4]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int q = 4; q >= 1; --q) {
      double m = 0.0;
      if (ip - q >= 0) {
        m = row[HW - q] * U[q - 1][0];
#pragma unroll
        for (int c = 1; c < 5; ++c) row[HW - q + c] -= m * U[q - 1][c];
      }
      mult[q - 1] = m;
    }
#pragma unroll
    for (int q = 3; q >= 1; --q)
#pragma unroll
      for (int c = 0; c < 5; ++c) U[q][c] = U[q - 1][c];
    U[0][0] = 1.0 / row[HW];
#pragma unroll
    for (int c = 1; c < 5; ++c) U[0][c] = row[HW + c];
  }
  // multipliers of row j of operator op (processing place ip)
  __device__ __forceinline__ void row_mult(const double* rc, const Dims& d, int op, int j, int ip, double a, double b,
                                           double (&mult)[4]) {
    double nat[NB9], row[NB9];
    operator_row(rc, d, op, j, a, b, nat);
#pragma unroll
    for (int c = 0; c < NB9; ++c) row[c] = (op != OP_P) ? nat[NB9 - 1 - c] : nat[c];
    next(row, ip, mult);
  }
};

// ------------------------------------------------------------------ lane layout
// Lane layout: one mode per lane.  A wave holds 32 mode pairs: lanes 0-31
// take slot +l, lanes 32-63 slot -l of the same (|l|, n), so both halves
// load the same factor words in the same instruction (one fetch) and every
// state access is two contiguous 32-element runs.  The -l lanes of |l| = 0
// are idle (that slot is the +l one).
struct Lane1 {
  int dm;          // distinct mode (factor column)
  int64_t o;       // plane offset of the slot
  double a, b;
  bool zero_mode;
};

__device__ __forceinline__ bool make_lane1(const Dims& d, Lane1& L) {
  const int half = threadIdx.x >> 5;
  L.dm = blockIdx.x * 32 + (threadIdx.x & 31);
  if (L.dm >= d.ndm) return false;
  const int labs = L.dm / d.mt, n = L.dm - labs * d.mt;
  if (half == 1 && labs == 0) return false;
  const int s = half ? d.mz - labs : labs;
  L.o = (int64_t)s * d.mt + n;
  L.a = n * d.kt;
  L.b = (half ? -labs : labs) * d.kz;
  L.zero_mode = (labs == 0 && n == 0);
  return true;
}

}  // namespace tc
