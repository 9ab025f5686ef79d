// Kernel argument blocks and launchers (device pointers only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ba.h"
#include "ba_internal.h"

namespace ba {

struct LinArgs {
  const int32_t *chunk_ptr, *chunk_pt, *pt_ptr, *o_cam, *o_pt;
  const uint8_t* fixed;
  const double *o_xy, *o_w, *cams, *pts;
  double huber;
  double* w;
  void* J;
  double *V, *gp, *part_cost, *part_gmax;
  double* rec;  // per observation: r, w, e (the residual lives only here)
  // point elimination of the same pass (damping with the current lambda)
  double dmin, dmax;
  double *Vinv, *ep;
  DevScalars* dev;
  GridSync* gs;
};

struct DampArgs {
  int np;
  const double *V, *gp;
  double dmin, dmax;
  double *Vinv, *ep;
  DevScalars* dev;
  GridSync* gs;
};

struct PointQArgs {
  int64_t no;
  const int32_t* o_pt;
  const double *w, *Vinv, *ep;
  void* J;      // reads Jp of each row, writes Q, w into it
  double* rec;  // writes e = Jp ep
};

struct SchurArgs {
  int nwg;       // workgroups of the slot table
  int rec_unit;  // first 64-byte unit of the records, counted from J
  // stab: step table in 64-byte units from J (rows, or records for the y
  // side of self pairs; -1: no pair)
  const int32_t *slot_blk, *slot_lead, *blk_row, *S_ptr, *stab, *swptr;
  const void* J;
  void* S;
  double* Sdiag;
  // camera vectors from the self pairs of the diagonal blocks
  double *gc, *bS, *diagU;
  // streamed PCG plans: each upper off-diagonal block also written to its
  // streamed copy blk_pos[e], padded to SI_STRIDE values (null otherwise)
  const int32_t* blk_pos = nullptr;
  void* SI = nullptr;
};

struct CamFinishArgs {
  double* Sdiag;  // undamped on entry, damped on exit
  const double* diagU;
  double dmin, dmax;
  double* Minv;
  DevScalars* dev;
  double* Linv;   // optional: inverse Cholesky factors (lower, [nc][81])
  const double* gc;  // optional: bS -= gc (completes the right-hand side)
  double* bS;
};

struct PcgArgs {
  int nc, maxiter;
  double rtol;
  const int32_t *S_ptr, *T_ptr, *wg_row, *item_ptr, *item_e, *item_code, *ucol_ptr, *ucol;
  const void* S;
  const double *Sdiag, *Minv, *b;
  double* x;
  double *zring, *partA, *partB;  // (maxiter + 1) slots each
  ba_step_info* info;
  GridSync* gs;
  int* error;
  // streamed plans (mixed precision; wg_row is then the streamed
  // decomposition): per-workgroup upper blocks, their local columns and FP32
  // copies; the columns, exchange slots, incoming slots per row and sending
  // workgroups; exchange ring (maxiter + 2 slots of rstride doubles) and
  // flags (maxiter + 2 per workgroup)
  const int32_t* sitem_ptr = nullptr;
  const int32_t* sitem_col = nullptr;
  const void* SI = nullptr;
  const int32_t *vcol_ptr = nullptr, *vcol = nullptr, *vbase = nullptr;
  const int32_t *in_ptr = nullptr, *in_off = nullptr, *src_ptr = nullptr, *src = nullptr;
  int64_t rstride = 0;
  double *rring = nullptr, *rflag = nullptr;
};

struct BackArgs {
  const int32_t *chunk_ptr, *chunk_pt, *pt_ptr, *o_cam, *o_pt;
  const void* J;
  const double *w, *dc, *gp, *Vinv, *pts;
  double *dp, *pts_new, *part_pred;
};

struct RetractArgs {
  int nc;
  const uint8_t* fixed;
  const double *cams, *dc, *gc;
  double *cams_new, *part_linc;
};

struct CostArgs {
  const int32_t *chunk_ptr, *o_cam, *o_pt;
  const double *o_xy, *o_w, *cams, *pts;
  double huber;
  double* part_cost_new;
};

struct FinalArgs {
  int nchunk, ncamblk, nc;
  const double *part_cost_new, *part_pred, *part_linc, *part_gmax, *gc;
  double lambda_min, lambda_max;
  DevScalars* dev;
  ba_step_info* info;
  double* stage;  // [4][FINAL_STAGE_MAX]: per-workgroup partials of the first stage
  int nstage;     // workgroups of the first stage
};

struct ObsArgs {
  int64_t no;
  const int64_t* o_orig;
  const double *xy, *w;
  double *o_xy, *o_w;
  DevScalars* dev;
};

// Row permutation of a FP64 table: gather (dst row i = src row map[i]) or
// scatter (dst row map[i] = src row i), copying the first `width` values of
// rows of src_stride / dst_stride values.
struct PermArgs {
  int n;
  const int32_t* map;
  bool gather;
  const double* src;
  double* dst;
  int src_stride, dst_stride, width;
};

template <typename T> hipError_t launch_linearize(const LinArgs&, int nchunk, LongChunks, hipStream_t);
hipError_t launch_permute_rows(const PermArgs&, hipStream_t);
hipError_t launch_reduce_cost(const double* part, int n, DevScalars* dev, hipStream_t);
hipError_t launch_damp_points(const DampArgs&, hipStream_t);
template <typename T> hipError_t launch_point_q(const PointQArgs&, hipStream_t);
template <typename T> hipError_t launch_schur_pairs(const SchurArgs&, int nwg, hipStream_t);
template <typename T> hipError_t launch_camera_finish(const CamFinishArgs&, int nc, hipStream_t);
template <typename T> int pcg_max_grid(bool resident, bool pipelined, bool stream = false);
template <typename T>
hipError_t launch_pcg(const PcgArgs&, int grid, bool resident, bool pipelined, hipStream_t);
template <typename T> hipError_t launch_backsub(const BackArgs&, int nchunk, LongChunks, hipStream_t);
hipError_t launch_retract_cameras(const RetractArgs&, int nblk, hipStream_t);
hipError_t launch_candidate_cost(const CostArgs&, int nchunk, hipStream_t);
hipError_t launch_finalize(FinalArgs, hipStream_t);
hipError_t launch_set_observations(const ObsArgs&, hipStream_t);

}  // namespace ba
