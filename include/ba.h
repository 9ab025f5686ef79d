/*
 * ba.h -- C ABI of the MI355X (gfx950) bundle-adjustment hot path.
 *
 * One Levenberg-Marquardt iteration of bundle adjustment ("Bundle Adjustment
 * in the Eager Mode", Alg. 1 and Eq. 2): per-observation reprojection
 * residuals and Jacobian blocks (Eq. 1, Sec. III-C), block-sparse J^T J and
 * J^T r assembly (Sec. IV-B-1, IV-B-2), clamped diagonal damping (Sec.
 * IV-B-3), the Schur complement of the damped system onto the cameras, a
 * block-Jacobi preconditioned conjugate-gradient solve (Sec. IV-C-2),
 * back-substitution of the points and the trust-region acceptance of the
 * step (Sec. V).
 *
 * Conventions shared by every entry point
 *  - Pointers marked "device" address memory on the GPU the problem was bound
 *    to; "host" pointers address ordinary CPU memory.  Sizes are element
 *    counts unless named *_bytes.
 *  - Camera rows are 10 float64: [tx ty tz qx qy qz qw f k1 k2]; the pose maps
 *    world to camera, Y = R(q) X + t, q a unit quaternion stored scalar-last;
 *    pixel = f (1 + k1 s + k2 s^2) (-Y_x/Y_z, -Y_y/Y_z), s the squared norm of
 *    the normalised coordinates (the projection of Eq. 1 with the BAL camera
 *    used by the paper's benchmark).  Points are 3 float64 in world frame.
 *  - Camera steps use the 9-dimensional tangent (rho, phi, df, dk1, dk2):
 *    T <- Exp(rho, phi) T on SE(3) (left update; the pose gradient space has 6
 *    degrees of freedom, Sec. III-C footnote), intrinsics additive.  With
 *    cam_dof 6 the intrinsics are constants and the step is the pose part.
 *  - The library owns no device memory: the caller provides one device
 *    workspace (ba_problem_bind) and keeps it alive until destroy.  The
 *    library allocates only small pinned host staging buffers.
 *  - All device work is enqueued on the stream given to ba_problem_bind.  A
 *    handle is not thread-safe; one problem per stream.
 *  - Errors are returned as ba_status; nothing aborts.  ba_last_error() gives a
 *    message for the calling thread's most recent failure.
 */
#ifndef BA_H
#define BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_problem ba_problem;

typedef enum {
  BA_OK = 0,
  BA_EINVAL = -1,        /* bad argument: null pointer, size, index out of range,
                            non-finite observation, weight <= 0, short workspace */
  BA_ENUMERIC = -2,      /* non-finite cost or a non-positive-definite block at
                            the current parameters; parameters are unchanged */
  BA_EHIP = -3,          /* a HIP runtime call failed */
  BA_ENOTCONV = -4,      /* ba_solve: damping reached lambda_max on a rejected step */
  BA_ESTATE = -5,        /* call out of order (not bound, no observations, ...) */
  BA_EUNSUPPORTED = -6   /* option or problem shape this build does not handle */
} ba_status;

enum { BA_FP64 = 0, BA_MIXED = 1 };

/* Solver options.  Defaults (ba_default_options) follow the paper's minimum
 * example (Sec. V: PCG(tol=1e-4, maxiter=250), TrustRegion(up=2, down=1/16));
 * the values the paper leaves open (initial damping, clamp range, lambda
 * bounds) are this library's choice. */
typedef struct {
  int32_t cam_dof;     /* camera tangent size: 9 (pose + f, k1, k2), or 6 (pose
                          only, intrinsics held at their set values; the
                          9-wide exports then carry zeros in columns 6-8) */
  int32_t precision;   /* BA_FP64: every stored quantity FP64.
                          BA_MIXED: Jacobian blocks and the reduced camera
                          matrix stored FP32 (arithmetic stays FP64; costs,
                          reductions, point blocks and CG vectors are FP64) */
  double huber_delta;  /* > 0: Huber loss on the squared residual norm with this
                          threshold in pixels; <= 0: plain squared loss */
  double cg_rtol;      /* PCG stops when |b - S x| <= cg_rtol |b| (relative) */
  int32_t cg_maxiter;  /* and after at most this many iterations */
  double lambda0, lambda_min, lambda_max;
  double diag_min, diag_max; /* clamp range of the damped diagonal */
  int32_t cg_variant;  /* BA_CG_PIPELINED: one grid synchronisation per CG
                          iteration (same iterates in exact arithmetic; relative
                          residuals below ~1e-10 may not be attainable);
                          BA_CG_STANDARD: the textbook recurrence, two per
                          iteration */
  int32_t enable_backward; /* nonzero: the workspace also holds the FP64 buffers
                              of ba_backward (about 1 KB per observation) */
  double adjoint_rtol;     /* relative residual of ba_backward's PCG solve */
  int32_t precond;         /* BA_PRECOND_BLOCK_JACOBI, or BA_PRECOND_LEARNED: the
                              block-Jacobi blocks corrected by the camera-graph
                              network (ba_set_gnn_params); until parameters are
                              set, and whenever its PCG fails (breaks down, or
                              ends with a non-finite relative residual or one
                              >= 1), the step uses plain block-Jacobi */
  double adjoint_grad_tol; /* ba_backward requires a stationary theta:
                              max_i |g_i| <= adjoint_grad_tol * max_k,i |w_k (J_k^T r_k)_i|
                              (the gradient against the scale of its terms) */
  int32_t linear_solver;   /* BA_SOLVER_PCG: block-Jacobi PCG on the reduced
                              camera system (Sec. IV-C-2); BA_SOLVER_CHOLESKY:
                              the paper's factorisation alternative (Sec.
                              IV-C-1) on the same system, assembled dense in
                              FP64 (at most 2048 cameras; the workspace grows
                              by 8 (9 n_cams)^2 bytes); cg_* are then unused
                              and cg_rel_resid reports |b - S x| / |b| */
  int32_t camera_order;    /* BA_ORDER_BANDWIDTH: the library renumbers the
                              cameras internally (reverse Cuthill-McKee order of
                              their co-visibility graph) so that the reduced
                              matrix's blocks lie near its diagonal and the
                              PCG's workgroups exchange with few others; every
                              entry point still takes and returns cameras in
                              the caller's order.  BA_ORDER_GIVEN: the caller's
                              order is used as is */
} ba_options;

enum { BA_SOLVER_PCG = 0, BA_SOLVER_CHOLESKY = 1 };

enum { BA_ORDER_BANDWIDTH = 0, BA_ORDER_GIVEN = 1 };

enum { BA_PRECOND_BLOCK_JACOBI = 0, BA_PRECOND_LEARNED = 1 };

enum { BA_CG_PIPELINED = 0, BA_CG_STANDARD = 1 };

/* Per-iteration report (host struct). */
typedef struct {
  double cost_before;   /* F(theta) = 1/2 sum_k w_k rho(|r_k|^2) */
  double cost_after;    /* F(theta (+) delta) */
  double lambda_used;   /* damping of this step */
  double lambda_next;   /* damping after the trust-region update */
  double cg_rel_resid;  /* final |b - S x| / |b| of the PCG */
  double pred;          /* predicted reduction of the Gauss-Newton model */
  double grad_inf;      /* max-norm of the gradient J^T W r at theta */
  int32_t accepted;     /* 1 if theta moved */
  int32_t cg_iters;
  int32_t cg_breakdown; /* 1 if p^T S p <= 0 stopped the PCG */
  int32_t status;       /* ba_status of the step */
  int32_t precond_used; /* 0 block-Jacobi, 1 learned, 2 learned then block-Jacobi
                           (the learned PCG failed, see ba_options.precond) */
  int32_t stop_reason;  /* ba_solve, on its last step: BA_STOP_* (BA_STOP_NONE on
                           every other step and from ba_lm_step) */
} ba_step_info;

/* Why ba_solve stopped (ba_step_info.stop_reason of its last step). */
enum {
  BA_STOP_NONE = 0,
  BA_STOP_MAX_ITERS = 1,   /* max_iters ran out before another rule held */
  BA_STOP_PLATEAU = 2,     /* plateau_steps iterations with relative decrease < tol */
  BA_STOP_GRADIENT = 3,    /* |g|_inf <= 1e-12 (1 + F) at the step's linearisation point */
  BA_STOP_LAMBDA_MAX = 4,  /* a step was rejected at lambda_max (BA_ENOTCONV) */
  BA_STOP_ERROR = 5        /* a step failed; its status is the return value */
};

/* Fills *opt with the defaults: cam_dof 9, BA_FP64, squared loss, cg_rtol 1e-4,
 * cg_maxiter 250, lambda0 1e-4, lambda in [1e-12, 1e12], clamp [1e-6, 1e32],
 * BA_CG_PIPELINED, backward disabled, adjoint_rtol 1e-10, block-Jacobi,
 * adjoint_grad_tol 1e-6, BA_SOLVER_PCG, BA_ORDER_BANDWIDTH. */
void ba_default_options(ba_options* opt);

/* Creates a problem from the observation pattern: observation k sees point
 * pt_idx[k] in camera cam_idx[k] (the index tensors of Sec. V's minimum
 * example).  cam_idx, pt_idx: host int32 arrays of n_obs entries; copied.
 * Runs the symbolic analysis once (the cached sparsity structure of
 * Sec. IV-B-1): observation ordering, the block pattern of the reduced camera
 * matrix and the table of observation pairs that feed each block.  No device
 * work is done.  Errors: BA_EINVAL for sizes <= 0 or indices out of range,
 * BA_EUNSUPPORTED for cam_dof other than 9 or 6 (6 with the learned
 * preconditioner or the adjoint).  A point may be seen any number of times
 * (points seen more than 256 times take their own kernels). */
ba_status ba_problem_create(const ba_options* opt, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                            const int32_t* cam_idx, const int32_t* pt_idx, ba_problem** out);

/* Exact device workspace size in bytes needed by ba_problem_bind. */
ba_status ba_problem_workspace_bytes(const ba_problem* p, size_t* bytes);

/* Binds the caller's device workspace (>= workspace_bytes, 256-byte aligned)
 * and HIP stream (hipStream_t, NULL = default stream) on the current device,
 * and uploads the symbolic structure.  The workspace stays owned by the
 * caller and must outlive the problem.  Errors: BA_EINVAL (null/short/
 * misaligned workspace), BA_EHIP. */
ba_status ba_problem_bind(ba_problem* p, void* workspace, size_t bytes, void* hip_stream);

/* Sets the observed pixels.  obs_xy: device float64 [n_obs][2] (x, y) in the
 * creation order; obs_w: device float64 [n_obs] per-observation weights
 * omega_k > 0, or NULL for all ones.  Copied (the caller may free them).
 * Errors: BA_EINVAL for non-finite pixels or weights <= 0 (checked with one
 * stream synchronisation). */
ba_status ba_set_observations(ba_problem* p, const double* obs_xy, const double* obs_w);

/* Marks cameras whose parameters stay fixed (gauge anchors): mask_host is a
 * host uint8 array of n_cams entries, nonzero = fixed; NULL clears. */
ba_status ba_set_fixed_cameras(ba_problem* p, const uint8_t* mask_host);

/* Sets / reads the parameters theta: cams device float64 [n_cams][10], pts
 * device float64 [n_pts][3].  set copies and invalidates the linearisation. */
ba_status ba_set_params(ba_problem* p, const double* cams, const double* pts);
ba_status ba_get_params(const ba_problem* p, double* cams, double* pts);

/* Damping for the next step, and PCG stopping rule overrides (rtol >= 0,
 * maxiter >= 1); rtol = 0 with a fixed maxiter pins the CG iteration count. */
ba_status ba_set_lambda(ba_problem* p, double lambda);
ba_status ba_get_lambda(const ba_problem* p, double* lambda);
ba_status ba_set_cg(ba_problem* p, double rtol, int32_t maxiter);

/* One LM iteration (Alg. 1): linearise at theta unless the previous step was
 * rejected (then the linearisation is reused), damp, reduce onto the cameras,
 * PCG, back-substitute, evaluate the candidate, accept or reject and update
 * lambda (accept iff F' < F, F' finite and pred > 0; ratio > 0.75 halves
 * lambda, ratio <= 0.25 or a rejection multiplies it by 16).  info: host, may
 * be NULL.  Synchronises the stream once.  Errors: BA_ESTATE before
 * bind/observations/params, BA_ENUMERIC (theta and lambda unchanged). */
ba_status ba_lm_step(ba_problem* p, ba_step_info* info);

/* Repeats ba_lm_step until max_iters iterations, or plateau_steps consecutive
 * iterations with relative decrease (F - F')/F < rel_decrease_tol (a rejected
 * step decreases by 0; Sec. V, StopOnPlateau), or |g|_inf <= 1e-12 (1 + F) at
 * a step's linearisation point.  The rules are tested after every step in
 * the order: rejection at lambda_max, plateau, gradient, max_iters.  infos:
 * host array of max_iters entries or NULL; the last entry's stop_reason says
 * which rule ended the solve.  *iters_done (host, may be NULL) receives the
 * number of iterations run.  Returns BA_ENOTCONV when a step is rejected at
 * lambda_max (its damping was lambda_max already), or a failing step's
 * status. */
ba_status ba_solve(ba_problem* p, int32_t max_iters, double rel_decrease_tol, int32_t plateau_steps,
                   ba_step_info* infos, int32_t* iters_done);

/* Gradient of a loss L(theta*) of the optimum with respect to the observed
 * pixels and the per-observation weights: the implicit-function adjoint of
 * the stationarity condition sum_k w_k J_k^T r_k = 0 (the solver inside a
 * bilevel learning pipeline, Sec. VI-D and App. A).  With H the exact Hessian
 * of delta -> F(theta* (+) delta) at 0 (Gauss-Newton term plus the projection
 * curvature weighted by the residuals) and v = H^-1 dL/dtheta (tangent):
 *   dL/dx_k = w_k J_k v,   dL/dw_k = -r_k . (J_k v).
 * H v = dL/dtheta is solved exactly like the LM system (points eliminated,
 * the same pair table, block-Jacobi PCG with the standard recurrence to
 * adjoint_rtol within cg_maxiter iterations), in FP64 whatever the precision.
 *   dL_dcams: device float64 [n_cams][10], dL/d(stored camera row); its
 *             component along the quaternion's own direction is ignored (the
 *             gradient is taken along the retraction); fixed cameras ignored;
 *   dL_dpts:  device float64 [n_pts][3];
 *   dL_dobs:  device float64 [n_obs][2] output, creation order;
 *   dL_dw:    device float64 [n_obs] output, or NULL;
 *   info:     host, may be NULL: cg_iters, cg_rel_resid, status.
 * theta must be a stationary point (run ba_solve first): the gradient at
 * theta is checked first (adjoint_grad_tol) and a non-stationary theta is
 * refused with BA_ENOTCONV before anything is written.  Squared loss only
 * (huber_delta <= 0).  Overwrites the intermediate quantities of the last
 * ba_lm_step (ba_export then shows the adjoint's), and the next ba_lm_step
 * re-linearises.  Synchronises the stream.  Errors: BA_ESTATE (not bound /
 * enable_backward not set at creation), BA_EUNSUPPORTED (Huber loss),
 * BA_EINVAL (null pointer), BA_ENOTCONV (theta not stationary: nothing
 * written; or the PCG did not reach adjoint_rtol: outputs written),
 * BA_ENUMERIC (H not positive definite on a point or camera block: not at a
 * minimum), BA_EHIP. */
ba_status ba_backward(ba_problem* p, const double* dL_dcams, const double* dL_dpts, double* dL_dobs,
                      double* dL_dw, ba_step_info* info);

/* ---- learned correction of the block-Jacobi preconditioner ----------------
 * The paper preconditions its PCG with a diagonal (block) preconditioner
 * (Sec. IV-C-2).  With BA_PRECOND_LEARNED each 9x9 block is corrected from
 * the camera co-visibility graph of the reduced system: with S_ii = L_i L_i^T,
 * S^_ij = L_i^-1 S_ij L_j^-T, E_i = sum_j S^_ij S^_ij^T and a_ij = |S^_ij|_F,
 * node inputs [upper(E_i), log(1 + tr E_i), log(1 + deg_i)] pass through an
 * input layer and BA_GNN_LAYERS message-passing layers (weighted mean of the
 * neighbours, weights a_ij / sum_j a_ij, width BA_GNN_HIDDEN, ReLU) to 45
 * outputs o_i; C_i = strict lower(o_i) + diag(exp(o_i diag)) and
 * M_i = L_i^-T C_i C_i^T L_i^-1 (SPD; zero outputs give block-Jacobi).
 * Parameters: one float32 vector of ba_gnn_num_params() values, in the order
 * W_in [64][47], b_in [64], per layer W_s [64][64], W_m [64][64], b [64],
 * W_out [45][64], b_out [45] (row-major, output index first). */
enum { BA_GNN_FEATURES = 47, BA_GNN_HIDDEN = 64, BA_GNN_OUTPUTS = 45, BA_GNN_LAYERS = 3 };
int64_t ba_gnn_num_params(void);

/* Copies the network parameters (device float32, ba_gnn_num_params values)
 * into the problem; NULL returns to plain block-Jacobi.  Requires
 * precond == BA_PRECOND_LEARNED at creation. */
ba_status ba_set_gnn_params(ba_problem* p, const float* params);

/* Training graphs.  A graph holds the network inputs of one reduced camera
 * system (node features, E_i, neighbour weights) and the activations of a
 * training pass, in a caller-provided device workspace.  ba_graph_create
 * takes the camera pattern of a problem created with BA_PRECOND_LEARNED;
 * ba_graph_build fills the inputs from that problem's most recent step (its
 * damped reduced system), enqueued on the problem's stream. */
typedef struct ba_graph ba_graph;
ba_status ba_graph_create(const ba_problem* p, ba_graph** out);
ba_status ba_graph_workspace_bytes(const ba_graph* g, size_t* bytes);
ba_status ba_graph_bind(ba_graph* g, void* workspace, size_t bytes, void* hip_stream);
ba_status ba_graph_build(ba_graph* g, ba_problem* p);
/* Training loss of the graph's system for the given parameters,
 *   loss = (1/n) sum_i tr(Mh_i G_i Mh_i) - 2 tr(Mh_i) + 9,
 *   Mh_i = C_i C_i^T, G_i = I + E_i
 * (the squared Frobenius distance of the block-normalised preconditioned
 * operator to the identity, by block rows), and its gradient ADDED to grad
 * (device float32).  *loss (host) receives the loss.  Synchronises the
 * graph's stream. */
ba_status ba_gnn_loss_grad(ba_graph* g, const float* params, float* grad, double* loss);
/* One Adam step on device float32 vectors of n values (m, v: moments; step
 * counts from 1) with the gradient grad_scale * grad (e.g. 1 / number of
 * summed systems: the mean over a batch), on the given stream. */
ba_status ba_gnn_adam(int64_t n, float* params, const float* grad, float* m, float* v, int32_t step,
                      float lr, float beta1, float beta2, float eps, float grad_scale, void* hip_stream);
void ba_graph_destroy(ba_graph* g);

/* Host snapshot of (theta, lambda) for checkpoint / resume.  With host_blob ==
 * NULL, *bytes receives the size; otherwise *bytes must be at least that. */
ba_status ba_get_state(const ba_problem* p, void* host_blob, size_t* bytes);
ba_status ba_set_state(ba_problem* p, const void* host_blob, size_t bytes);

/* Reads an intermediate quantity of the most recent step into host memory
 * (for inspection and tests), in creation order for per-observation fields:
 *   BA_X_RESIDUAL  float64 [n_obs][2]   r_k = pixel - observation
 *   BA_X_WEIGHT    float64 [n_obs]      w_k = omega_k rho'(|r_k|^2)
 *   BA_X_JC        float64 [n_obs][2][9]
 *   BA_X_JP        float64 [n_obs][2][3]
 *   BA_X_COST      float64 [1]          F at the linearisation point
 *   BA_X_GRAD_C    float64 [n_cams][9]; BA_X_GRAD_P float64 [n_pts][3]
 *   BA_X_V         float64 [n_pts][3][3] undamped point blocks
 *   BA_X_S_PTR     int64 [n_cams+1]; BA_X_S_COL int32 [nnzb]
 *   BA_X_S         float64 [nnzb][9][9] reduced camera matrix, upper blocks
 *   BA_X_BS        float64 [n_cams][9]  its right-hand side
 *   BA_X_DC        float64 [n_cams][9]; BA_X_DP float64 [n_pts][3] the step
 *   BA_X_ADJ_VC    float64 [n_cams][9]; BA_X_ADJ_VP float64 [n_pts][3] the
 *                  adjoint vector v of the last ba_backward
 *   BA_X_PRECOND   float64 [n_cams][9][9] the preconditioner blocks of the
 *                  last step (learned blocks when the network ran)
 *   BA_X_PLAN      int64 [4] how the problem runs: the PCG layout (0 block
 *                  values held in registers, 1 stored blocks read per
 *                  (row, block) item, 2 upper blocks streamed once per
 *                  product), its workgroups, the Schur pair count and the
 *                  Schur workgroups (no device work)
 * bytes must equal the field's size.  Synchronises the stream. */
enum {
  BA_X_RESIDUAL = 1, BA_X_WEIGHT, BA_X_JC, BA_X_JP, BA_X_COST, BA_X_GRAD_C, BA_X_GRAD_P,
  BA_X_V, BA_X_S_PTR, BA_X_S_COL, BA_X_S, BA_X_BS, BA_X_DC, BA_X_DP, BA_X_ADJ_VC, BA_X_ADJ_VP,
  BA_X_PRECOND, BA_X_PLAN
};
ba_status ba_export(const ba_problem* p, int32_t field, void* host_dst, size_t bytes);

/* Per-phase timing with HIP events recorded on the problem's stream around
 * every kernel launch of ba_lm_step (off by default).  Phases:
 *   0 linearise (residuals, Jacobian blocks, point blocks), 1 cost reduction,
 *   2 point damping and inverses, 3 per-observation Schur factors,
 *   4 camera gradient / right-hand side, 5 Schur blocks from the pair table,
 *   6 diagonal damping and block-Jacobi factors, 7 PCG, 8 back-substitution,
 *   9 camera retraction, 10 candidate cost, 11 acceptance, 12 learned
 *   preconditioner (graph features and network).
 * ba_get_phase_times writes, for the first n phases, the summed milliseconds
 * (ms_out) and the number of launches (launches_out, may be NULL) since
 * profiling was last enabled. */
enum { BA_NUM_PHASES = 13 };
ba_status ba_set_profiling(ba_problem* p, int32_t enable);
/* As ba_set_profiling, but events are recorded only around the phases whose
 * bit (1 << phase) is set in mask (0: off); fewer events disturb the timed
 * steps less.  ba_set_profiling(p, 1) is ba_set_profiling_mask(p, all). */
ba_status ba_set_profiling_mask(ba_problem* p, uint32_t mask);
ba_status ba_get_phase_times(const ba_problem* p, double* ms_out, int64_t* launches_out, int32_t n);

/* Number of stored upper blocks of the reduced camera matrix (incl. diagonal). */
ba_status ba_problem_nnzb(const ba_problem* p, int64_t* nnzb);

/* Allocation-free binding, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): binds p, like ba_problem_bind, but to a fixed device scratch
 * array of BA_STATIC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends, instead of a caller workspace.  Allocates
 * nothing (no hipMalloc, hipFree or pinned host memory: the host staging
 * lives in the handle).  All problems bound this way on one GPU share that
 * GPU's array: binding another takes it over (the earlier handle's calls
 * then return BA_ESTATE), and calls that overlap on one GPU race.  Errors:
 * BA_EINVAL (ba_problem_workspace_bytes above BA_STATIC_SCRATCH_BYTES),
 * BA_ESTATE (already bound), BA_EHIP. */
#define BA_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
ba_status ba_problem_bind_static(ba_problem* p, void* hip_stream);

/* ---- pose graph optimisation (Sec. IV-D, Eq. 4 and 5) ----------------------
 * Z* = argmin 1/2 sum_e r_e^T Omega_e r_e over poses zeta, one residual per
 * edge e = (i, j): r_e = Log(zeta_i^-1 zeta_j T_e^-1) in R^6 (translation
 * part first), T_e the measured relative pose zeta_i^-1 zeta_j.  Poses and
 * measurements are 7 float64 [tx ty tz qx qy qz qw] (unit quaternion,
 * scalar last) for the transform [R(q) t; 0 1]; steps are the 6-vector
 * (rho, phi) of the left update zeta <- Exp(rho, phi) zeta.  A pose graph is
 * a ba_problem: the same LM iteration (ba_lm_step, ba_solve: linearise,
 * clamped damping, block-Jacobi PCG or dense Cholesky, retraction,
 * acceptance, damping update) runs on the 6x6-block system
 * H = sum J^T Omega J, g = sum J^T Omega r directly (nothing to eliminate),
 * the blocks held as 9x9 camera blocks with zero rows and columns 6-8.
 * Also valid on pose graphs: ba_problem_workspace_bytes, ba_problem_bind,
 * ba_problem_bind_static, ba_set_fixed_cameras (the mask fixes poses: gauge
 * anchors), ba_set_lambda, ba_get_lambda, ba_set_cg, ba_get_state,
 * ba_set_state (no points), ba_problem_nnzb, the profiling calls (phases 0
 * linearise, 1 cost, 5 block assembly, 6, 7, 9 retraction, 10 candidate,
 * 11) and ba_export of BA_X_COST, BA_X_GRAD_C, BA_X_S_PTR, BA_X_S_COL, BA_X_S,
 * BA_X_BS, BA_X_DC (9-wide rows, the last 3 entries zero), BA_X_PRECOND and
 * BA_X_PLAN.  The observation and point entry points return BA_EINVAL. */

/* Creates a pose graph of n_poses poses and n_edges edges ei[e] -> ej[e]
 * (host int32 arrays, copied; several edges may join the same two poses).
 * opt: cam_dof is ignored; huber_delta must be <= 0, precond block-Jacobi
 * and enable_backward 0 (else BA_EUNSUPPORTED).  Errors: BA_EINVAL (sizes
 * <= 0, endpoint out of range, an edge from a pose to itself),
 * BA_EUNSUPPORTED (more than 2^29 edges, options above). */
ba_status ba_pgo_create(const ba_options* opt, int32_t n_poses, int64_t n_edges, const int32_t* ei,
                        const int32_t* ej, ba_problem** out);
/* Measurements: T device float64 [n_edges][7]; omega device float64
 * [n_edges][6][6] information matrices (row-major, in the (rho, phi) order
 * of r), or NULL for identities.  Copied.  Errors: BA_EINVAL for non-finite
 * values, a quaternion with | |q|^2 - 1 | > 1e-10, or an information matrix
 * that is not exactly symmetric or has a diagonal entry <= 0 (one stream
 * synchronisation). */
ba_status ba_pgo_set_edges(ba_problem* p, const double* T, const double* omega);
/* Sets / reads the poses: device float64 [n_poses][7].  set copies and
 * invalidates the linearisation; a retracted pose carries a renormalised
 * quaternion of either sign. */
ba_status ba_pgo_set_poses(ba_problem* p, const double* poses);
ba_status ba_pgo_get_poses(const ba_problem* p, double* poses);

void ba_problem_destroy(ba_problem* p);
const char* ba_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BA_H */
