// Internal structures shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ba.h"

namespace ba {

constexpr int D = 9;            // camera tangent size (6 pose + f, k1, k2)
// One row of NJ values (precision T) per observation: Jc 2x9 at [0, 18),
// Jp 2x3 at [JP, JP + 6) (written by the linearisation), the Schur factor
// Q = w Jp Vinv (2x3) at [JQ, JQ + 6), the weight w at JW and one zero
// (written by the point elimination): a 128-byte line in mixed precision,
// so one Schur pair reads two lines, and each kernel writes whole 32-byte
// sectors.
constexpr int NJ = 32;
constexpr int JP = 18;
constexpr int JQ = 24;
constexpr int JW = 30;
constexpr int CHUNK = 256;      // observations per point-aligned chunk (= its block size)
constexpr int SCHUR_THREADS = 256;
constexpr int SCHUR_LANES = 3;         // lanes per pair chunk (3 block columns each)
constexpr int SCHUR_WAVE_SLOTS = 21;   // pair chunks per wavefront (63 lanes)
constexpr int SCHUR_WAVES = SCHUR_THREADS / 64;
constexpr int SCHUR_SLOTS = SCHUR_WAVES * SCHUR_WAVE_SLOTS;  // 84 pair chunks per workgroup
constexpr int SCHUR_ROWS = 2 * SCHUR_WAVE_SLOTS;  // staged observation rows per wavefront step
constexpr int SCHUR_CHUNK = 16;        // target pairs per chunk
constexpr int CAM_THREADS = 128;
constexpr int PCG_THREADS = 1024;
constexpr int PCG_RMAX = 48;          // block rows owned by one PCG workgroup
constexpr int PCG_MAX_GRID = 256;     // PCG workgroups (one per compute unit)
constexpr int PCG_GROUPS = PCG_THREADS / 9;  // 9-lane groups of a PCG workgroup
constexpr int PCG_IPG = 3;            // register-resident items per lane group
constexpr int ZSTRIDE = 16;           // doubles per block column in a PCG exchange slot
constexpr int PART_STRIDE = 16;       // doubles per workgroup partial (one 128-byte line)
constexpr int PCG_ZCOLS = 768;        // distinct block columns one PCG workgroup may touch
constexpr int ITEM_TRANS = 1 << 16;   // PCG item flags: transposed upper block,
constexpr int ITEM_DIAG = 1 << 17;    //   diagonal block (FP64, indexed by camera)
constexpr int BARRIER_FANIN = 16;
constexpr int MAX_BARRIER_GROUPS = 128;
// Chunks holding one point seen more than CHUNK times (their own kernels
// take them; the chunk kernels skip them).
struct LongChunks {
  const int32_t* idx;  // device: chunk indices
  int n;
};
constexpr int FINAL_STAGE_MAX = 256;  // workgroups of the first acceptance-reduction stage
constexpr int SI_STRIDE = 84;         // values per block of the streamed PCG copy of S (81 + zeros:
                                      // 16-byte aligned blocks in FP32)
constexpr int STREAM_RMAX = 96;       // block rows owned by one streamed-PCG workgroup
constexpr int STREAM_COLS = 448;      // distinct upper block columns of one streamed-PCG workgroup
constexpr int STREAM_IN_MAX = 2048;   // received column sums of a streamed-PCG workgroup listed in LDS

// Host-side symbolic analysis of the observation pattern (computed once per
// problem; the paper caches its sparse-product table the same way, Sec. IV-B-1).
struct Plan {
  int32_t nc = 0, np = 0;
  int64_t no = 0;
  // observations sorted by (point, camera, original index): "positions"
  std::vector<int32_t> o_cam, o_pt;
  std::vector<int64_t> o_orig;       // original index of each position
  std::vector<int32_t> pt_ptr;       // [np+1] position range of each point
  std::vector<int32_t> chunk_ptr;    // [nchunk+1] position range of each chunk
  std::vector<int32_t> chunk_pt;     // [nchunk+1] point range of each chunk
  std::vector<int32_t> long_chunk;   // chunks with more than CHUNK positions (one point each)
  std::vector<int32_t> cam_ptr;      // [nc+1]
  std::vector<int32_t> cam_obs;      // positions grouped by camera
  std::vector<int32_t> S_ptr, S_col; // upper block pattern, diagonal first in each row
  std::vector<int32_t> T_ptr, T_blk, T_src;  // for row b: upper blocks (a,b), a < b
  // observation pairs (x, y) that feed each S block: camera(x) = row, camera(y)
  // = column, same point; grouped by block, ascending x within a block
  std::vector<int32_t> pair_x, pair_y;
  // Schur workgroups: SCHUR_SLOTS chunk slots each; slot -> (block, pair range,
  // number of slots of the block when this slot is the block's first, else 0)
  std::vector<int32_t> slot_blk, slot_pb, slot_pe, slot_lead;
  // the same chunks as wavefront steps: wavefront v of Schur workgroup g
  // runs steps [swptr[4g + v], swptr[4g + v + 1]); step t lists the pair of
  // each of the wavefront's 21 slots, stab[SCHUR_ROWS t + 2s] = x,
  // stab[SCHUR_ROWS t + 2s + 1] = y, or -2 - x for a self pair (x, x), or
  // -1 twice when slot s has no pair at that step (uploaded in 64-byte
  // units of the observation rows and records)
  std::vector<int32_t> stab, swptr;
  std::vector<int32_t> blk_row;  // block -> its row (camera a)
  // PCG workgroup decomposition: workgroup g owns rows [pcg_row[g],
  // pcg_row[g+1]); its (row, block) items in row order with block index and
  // code (local column | flags), and the distinct block columns it reads.
  // pcg_resident: every lane group has at most PCG_IPG items.
  std::vector<int32_t> pcg_row, item_ptr, item_e, item_code, ucol_ptr, ucol;
  // streamed plans (not pcg_resident) have a decomposition of their own,
  // balanced by upper blocks: workgroup g owns rows [srow[g], srow[g+1]);
  // its upper off-diagonal blocks, in row order, are the streamed items
  // sitem_ptr[g] .. sitem_ptr[g+1] (numbered globally, each with an FP32
  // copy SI), item i in block column vcol[vcol_ptr[g] + sitem_col[i]];
  // blk_pos[e] is the item of upper block e (-1 for diagonal blocks).  The
  // column sums for other workgroups' rows go to exchange slot
  // vbase[g] + 9 j (doubles; each workgroup's slots start on a 128-byte
  // line) of a ring slot of rstride doubles; row b adds the slots
  // in_off[in_ptr[b] .. in_ptr[b+1]) (ascending sending workgroup), and
  // workgroup g waits for the workgroups src[src_ptr[g] .. src_ptr[g+1]).
  std::vector<int32_t> srow, sitem_ptr, sitem_col, blk_pos, vcol_ptr, vcol, vbase;
  std::vector<int32_t> in_ptr, in_off, src_ptr, src;
  int64_t rstride = 0;
  int32_t sgrid = 0, max_vcol = 0;
  // camera co-visibility graph (both directions of every off-diagonal block):
  // neighbours of camera i are nbr[nbr_ptr[i] .. nbr_ptr[i+1]), through block
  // nbr_blk; nbr_rev is the slot of the same block in the neighbour's list
  std::vector<int32_t> nbr_ptr, nbr, nbr_blk, nbr_rev;
  int32_t max_ucol = 0, pcg_grid = 0;
  bool pcg_resident = false;
  int64_t nnzb = 0, n_pairs = 0;
  int32_t n_schur_wg = 0;
  int32_t max_track = 0;
};

// Allocation-free binding: the fixed device scratch every such problem on a
// GPU shares (ba_problem_bind_static), and its address on `device` (the
// current device), resolved once per device.
constexpr size_t STATIC_SCRATCH_BYTES = BA_STATIC_SCRATCH_BYTES;
hipError_t static_scratch(int device, void** ptr);

// Reverse Cuthill-McKee order of the cameras (order[c] = internal index of
// camera c); the indices must be in range.
std::vector<int32_t> camera_order(int32_t nc, int32_t np, int64_t no, const int32_t* cidx,
                                  const int32_t* pidx);

// Builds the plan; returns an empty string or an error message.
std::string build_plan(int32_t nc, int32_t np, int64_t no, const int32_t* cidx, const int32_t* pidx,
                       Plan* out);

struct DevScalars {
  double F;        // cost at the current parameters
  double lambda;   // damping of the next step
  int32_t error;   // bit flags set by kernels (see ERR_*)
  int32_t pad;
};

// per-camera flags of the `fixed` array: the whole camera held fixed (gauge
// anchor; its Jacobian block is zero), or only its intrinsics (the 6-DoF
// pose-only camera: Jacobian columns f, k1, k2 zero, so its reduced rows
// and its step in those components are exactly zero)
enum : uint8_t { FIXED_CAMERA = 1, FIXED_INTRINSICS = 2 };

enum : int32_t {
  ERR_NONFINITE_OBS = 1,
  ERR_BAD_WEIGHT = 2,
  ERR_POINT_BLOCK = 4,    // a damped 3x3 point block was not positive definite
  ERR_CAMERA_BLOCK = 8,   // a diagonal Schur block was not positive definite
  ERR_BARRIER = 16,       // the PCG grid barrier timed out
};

struct GridSync {
  unsigned count;
  unsigned gen;
  unsigned pad_[62];
  struct {
    unsigned count;
    unsigned pad_[63];
  } group[MAX_BARRIER_GROUPS];
};

// Device pointers carved out of the caller's workspace.
struct Buffers {
  // plan
  int32_t *o_cam, *o_pt, *pt_ptr, *chunk_ptr, *chunk_pt, *cam_ptr, *cam_obs, *long_chunk;
  int32_t *S_ptr, *S_col, *T_ptr, *T_blk, *T_src;
  int32_t *pair_x, *pair_y, *slot_blk, *slot_pb, *slot_pe, *slot_lead, *blk_row, *stab, *swptr;
  int32_t *pcg_row, *item_ptr, *item_e, *item_code, *ucol_ptr, *ucol;
  int32_t *srow, *sitem_ptr, *sitem_col, *blk_pos, *vcol_ptr, *vcol, *vbase;
  int32_t *in_ptr, *in_off, *src_ptr, *src;
  void* SI;  // streamed plans: [n_sitems][SI_STRIDE] (precision T)
  int64_t* o_orig;
  uint8_t* fixed;
  // observations (sorted by position)
  double *o_xy, *o_w;
  // parameters: [0] current, [1] candidate
  double *cams[2], *pts[2];
  // linearisation: w per observation; r [no][2] is the adjoint's residual
  // at the solution (the step's residual is in rec)
  double *r, *w;
  void* J;  // float or double [no][NJ] (layout above)
  // [no][8] FP64 per observation: r0, r1, w, 0 (linearisation), then
  // e = Jp ep: e0, e1, 0, 0 (point elimination); the camera vectors of the
  // Schur kernel's self pairs read it
  double* rec;
  double *V, *gp, *gc, *diagU;
  // damped quantities
  double *Vinv, *ep;
  void* S;  // float or double [nnzb][81]; diagonal blocks live in Sdiag
  double *Sdiag, *bS, *Minv;  // FP64 diagonal blocks (damped in place), rhs, block-Jacobi inverse
  // step
  double *x, *dp;
  // partial sums
  double *part_cost, *part_cost_new, *part_pred, *part_gmax, *part_linc, *part_stage;
  double *zring, *partA, *partB;  // PCG exchange rings, one slot per iteration
  double *rring, *rflag;          // streamed plans: column-sum exchange slots and flags
  // direct solve (BA_SOLVER_CHOLESKY): dense lower triangle of S with b_S as
  // an extra row, inverses of the diagonal factors, partial sums, residuals
  double *dA, *dLinv, *dpart, *dresid;
  DevScalars* dev;
  ba_step_info* dinfo;
  GridSync* gsync;
  // implicit-function adjoint (only with enable_backward; FP64)
  double *adjA, *adjJ, *adjY;  // per position: [78] w (J^T J + C), [24] J, [27] W V^-1
  double *adjU;                // [nc][81] exact camera blocks
  double* adjS;                // [nnzb][81] reduced matrix (aliases S in FP64 mode)
  double *adj_gt, *adj_vc, *adj_vp;  // tangent loss gradient, adjoint vector
  DevScalars* adj_dev;         // lambda = 0 and the adjoint's error flags
  double* adj_stat;            // [2] stationarity check: max |g_i|, max |term|
  ba_step_info* adj_info;
  // learned preconditioner (only with BA_PRECOND_LEARNED)
  double *pcLinv, *pcMinvL;    // [nc][81] inverse Cholesky factors, learned blocks
  float* pc_params;            // network parameters
  short* pc_wbf16;             // BF16 copies of the input and message-layer weights
  int32_t *nbr_ptr, *nbr, *nbr_blk, *nbr_rev;
  float *gX, *gE, *gw;         // network inputs
  float* gact;                 // activations (inference)
  // pose graphs: edge endpoints, measurements [m][8], information [m][36],
  // per-edge records (A, b), and each stored block's edge list
  int32_t *pg_ei, *pg_ej, *pg_ptr, *pg_code;
  double *pg_T, *pg_om, *pg_rec;
  // camera reordering: internal index of every caller camera; the adjoint's
  // dL/dcams in internal order
  int32_t* cam_perm;
  double* adj_gcam;
};

}  // namespace ba

struct ba_problem {
  ba_options opt;
  ba::Plan plan;
  ba::Buffers b{};
  hipStream_t stream = nullptr;
  int device = -1;
  void* workspace = nullptr;
  size_t ws_bytes = 0;
  size_t ws_needed = 0;
  bool bound = false, have_obs = false, have_params = false;
  bool lin_valid = false;
  int cur = 0;  // which parameter buffer is current
  int nchunk = 0, cam_blocks = 0;
  int pcg_grid = 0;
  double lambda = 1e-4;
  double cg_rtol = 1e-4;
  int32_t cg_maxiter = 250;
  bool profiling = false;
  hipEvent_t ev[BA_NUM_PHASES][2] = {};
  double phase_ms[BA_NUM_PHASES] = {};
  int64_t phase_n[BA_NUM_PHASES] = {};
  bool phase_used[BA_NUM_PHASES] = {};
  bool adj_grid_ok = false;  // the FP64 standard PCG fits the plan's grid
  bool gnn_ready = false;    // learned preconditioner parameters are set
  bool have_system = false;  // a step has formed the reduced system
  int32_t rec_unit = 0;      // records' first 64-byte unit counted from J
  size_t rec_off = 0;        // byte offset of the records from J (workspace layout)
  uint32_t profile_mask = 0;  // phases bracketed by events while profiling
  ba_step_info* hinfo = nullptr;     // pinned host staging
  ba::DevScalars* hscal = nullptr;   // pinned host staging
  // the Schur step table in 64-byte units (computed at creation)
  std::vector<int32_t> stab_units;
  // bound to the device's static scratch (ba_problem_bind_static): staging
  // in the handle itself instead of pinned buffers
  bool static_ws = false;
  ba_step_info hinfo_local{};
  ba::DevScalars hscal_local{};
  // pose graph (ba_pgo_create): n_edges edges i -> j; the camera rows hold
  // the poses and the plan is that of two observations per edge; pg_ptr /
  // pg_code list each stored block's edges (2 e + 1 when the block's row is
  // the edge's first pose, else 2 e)
  bool pgo = false;
  int64_t n_edges = 0;
  std::vector<int32_t> pg_ei, pg_ej, pg_ptr, pg_code;
  // cameras renumbered (reverse Cuthill-McKee) for the plan: cam_perm[c] is
  // the internal index of caller camera c, cam_inv its inverse; every
  // camera-indexed device buffer is in internal order and the entry points
  // translate.  x_* give the block pattern in caller order for ba_export:
  // upper blocks (a, b), a <= b, diagonal first; block k is internal block
  // x_blk[k], transposed when x_tr[k]
  bool reordered = false;
  std::vector<int32_t> cam_perm, cam_inv;
  std::vector<int64_t> x_ptr;
  std::vector<int32_t> x_col, x_blk;
  std::vector<uint8_t> x_tr;
};
