// Pose graph optimisation (Sec. IV-D, Eq. 4 and 5): kernel arguments and
// launchers.  A pose is stored in a 10-value camera row [t q 0 0 0] so that
// the damping, the block-Jacobi PCG, the retraction and the acceptance of the
// bundle-adjustment step serve the pose graph unchanged; the kernels here
// produce the reduced system directly (no points to eliminate) and the
// candidate's cost and model reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ba_internal.h"

namespace ba {

constexpr int PGO_CHUNK = 256;     // edges per workgroup of the per-edge kernels
constexpr int PGO_REC = 48;        // doubles per edge record: A = J^T Omega J (36), b = J^T Omega r (6)
constexpr int PGO_ASM_THREADS = 128;

struct PgoEdgeArgs {
  int64_t m;
  const double *T, *omega;  // caller's [m][7], [m][36] or null (identity)
  double *pg_T, *pg_om;     // stored [m][8], [m][36]
  DevScalars* dev;
};

struct PgoLinArgs {
  int64_t m;
  const int32_t *ei, *ej;
  const double *cams, *T, *om;
  double* rec;  // [m][PGO_REC]
  double *part_cost, *part_gmax;
};

// one workgroup per stored upper block (row a = blk_row[k], column S_col[k]);
// the block's edges are code[ptr[k] .. ptr[k+1]) = 2 e + s, s = 1 when the
// row's pose is the edge's first pose zeta_i (its Jacobian is -J), in
// ascending edge order
struct PgoAsmArgs {
  const int32_t *blk_row, *S_col, *ptr, *code;
  const uint8_t* fixed;
  const double* rec;
  void* S;  // off-diagonal blocks (precision T)
  double *Sdiag, *gc, *bS, *diagU;
  const int32_t* blk_pos;  // streamed PCG plans: copy of each upper block (else null)
  void* SI;
};

struct PgoCandArgs {
  int64_t m;
  const int32_t *ei, *ej;
  const double *cams_new, *T, *om, *rec, *dx;
  double *part_cost_new, *part_pred;
};

hipError_t launch_pgo_set_edges(const PgoEdgeArgs&, hipStream_t);
hipError_t launch_pgo_linearize(const PgoLinArgs&, hipStream_t);
template <typename T> hipError_t launch_pgo_assemble(const PgoAsmArgs&, int64_t nnzb, hipStream_t);
hipError_t launch_pgo_candidate(const PgoCandArgs&, hipStream_t);

inline int pgo_chunks(int64_t m) { return (int)((m + PGO_CHUNK - 1) / PGO_CHUNK); }

}  // namespace ba
