// Argument block and launcher of the direct (dense Cholesky) solve of the
// reduced camera system (device pointers only; FP64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ba.h"
#include "ba_internal.h"

namespace ba {

constexpr int DENSE_NB = 64;       // panel width of the blocked factorisation
constexpr int DENSE_BROWS = 256;   // rows per partial sum of the back substitution
constexpr int DENSE_MAX_CAMS = 2048;  // n = 9 n_c <= 18432 unknowns (2.7 GB of storage)

struct DenseArgs {
  int nc;
  int64_t nnzb;
  int64_t ld;       // leading dimension of the dense storage (multiple of DENSE_NB)
  double* A;        // [(9 nc + 1) * ld]: lower triangle of S, then b_S in row 9 nc
  double* Linv;     // [panels][DENSE_NB][DENSE_NB] inverses of the diagonal factors
  double* part;     // [ceil(9 nc / DENSE_BROWS)][DENSE_NB] back-substitution partials
  double* resid;    // [nc][2] per-camera |r|^2, |b|^2
  double* x;        // [9 nc] the solution (camera step)
  const double *b, *Sdiag;
  const void* S;    // upper off-diagonal blocks (precision T)
  const int32_t *S_ptr, *S_col, *blk_row, *T_ptr, *T_blk, *T_src;
  ba_step_info* info;
  int* error;
};

// bytes of the dense storage for nc cameras: A, Linv, part, resid
inline size_t dense_ld(int nc) { return (size_t)((9 * nc + DENSE_NB - 1) / DENSE_NB) * DENSE_NB; }

template <typename T>
hipError_t launch_dense_solve(const DenseArgs& a, hipStream_t s);

}  // namespace ba
