// Argument blocks and launchers of the implicit-function adjoint kernels
// (device pointers only; FP64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ba_internal.h"

namespace ba {

struct AdjTangentArgs {
  int nc;
  const uint8_t* fixed;
  const double *cams, *gL_cams;  // [nc][10] stored rows and their loss gradient
  double* gt;                    // [nc][9] tangent gradient
};

struct AdjObsArgs {
  int64_t no;
  const int32_t *o_cam, *o_pt;
  const uint8_t* fixed;
  const double *o_xy, *o_w, *cams, *pts;
  double *A, *J, *r;
};

struct AdjPointArgs {
  const int32_t *chunk_ptr, *chunk_pt, *pt_ptr, *o_pt;
  const double* A;
  double *Vinv, *Y;
  GridSync* gs;
  int* error;
};

struct AdjCameraArgs {
  const int32_t *cam_ptr, *cam_obs, *o_pt;
  const uint8_t* fixed;
  const double *A, *Y, *gL_pts, *gt;
  double *U, *b;
};

struct AdjSchurArgs {
  const int32_t *slot_blk, *slot_pb, *slot_pe, *slot_lead, *pair_x, *pair_y, *blk_row, *S_ptr;
  const double *A, *Y, *U;
  double *S, *Sdiag;
};

struct AdjBackArgs {
  const int32_t *chunk_ptr, *chunk_pt, *pt_ptr, *o_cam, *o_pt;
  const int64_t* o_orig;
  const double *A, *J, *r, *o_w, *Vinv, *vc, *gL_pts;
  double *vp, *dLdx, *dLdw;
};

struct AdjStatArgs {
  int nc, np;
  const int32_t *cam_ptr, *cam_obs, *pt_ptr;
  const double *J, *r, *o_w;
  double* stat;  // [2]: max |gradient component|, max |single term| (zeroed by the caller)
};

hipError_t launch_adj_stationarity(const AdjStatArgs&, hipStream_t);
hipError_t launch_adj_tangent(const AdjTangentArgs&, hipStream_t);
hipError_t launch_adj_obs(const AdjObsArgs&, hipStream_t);
hipError_t launch_adj_points(const AdjPointArgs&, int nchunk, LongChunks, hipStream_t);
hipError_t launch_adj_camera(const AdjCameraArgs&, int nc, hipStream_t);
hipError_t launch_adj_schur(const AdjSchurArgs&, int nwg, hipStream_t);
hipError_t launch_adj_backsub(const AdjBackArgs&, int nchunk, LongChunks, hipStream_t);

}  // namespace ba
