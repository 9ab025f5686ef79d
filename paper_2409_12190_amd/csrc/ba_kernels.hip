// gfx950 kernels of one Levenberg-Marquardt iteration of bundle adjustment.
//
// Data layout (HBM):
//   observations sorted by (point, camera): "positions"; per position x the
//   pixel o_xy[2x..2x+1] (FP64), weight o_w[x], camera o_cam[x], point o_pt[x];
//   Jacobian blocks J[x][24] = Jc (2x9 row-major) then Jp (2x3), stored in
//   the precision T (double in FP64 mode, float in mixed mode);
//   residual r[2x..] and Gauss-Newton weight w[x] in FP64;
//   point blocks V[j][6] (upper triangle xx xy xz yy yz zz), gradients gp[j][3],
//   gc[a][9]; reduced camera matrix S[e][81] (T, upper block pattern);
//   PCG vectors FP64 [n_cams][9].
//
// Every reduction is done in a fixed order (workgroup trees, then one final
// workgroup, or a fixed-order sum over per-workgroup partials), so results
// are bitwise reproducible from run to run.
#include "ba_device.h"
#include "ba_internal.h"
#include "ba_kernels.h"
#include "ba_reduce.h"

namespace ba {

template <typename T>
__device__ __forceinline__ void load_J(const T* __restrict__ J, double Jc[2][9], double Jp[2][3]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int m = 0; m < 9; ++m) Jc[i][m] = (double)J[i * 9 + m];
#pragma unroll
    for (int m = 0; m < 3; ++m) Jp[i][m] = (double)J[JP + i * 3 + m];
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Jc and Jp into an observation row (values [0, 24): whole 16-byte stores;
// rows are 16-byte aligned)
__device__ __forceinline__ void store_row(float* J, const double Jc[2][9], const double Jp[2][3]) {
  float v[24];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int m = 0; m < 9; ++m) v[i * 9 + m] = (float)Jc[i][m];
#pragma unroll
    for (int m = 0; m < 3; ++m) v[JP + i * 3 + m] = (float)Jp[i][m];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    f32x4 t;
    t.x = v[4 * k];
    t.y = v[4 * k + 1];
    t.z = v[4 * k + 2];
    t.w = v[4 * k + 3];
    *reinterpret_cast<f32x4*>(J + 4 * k) = t;
  }
}

__device__ __forceinline__ void store_row(double* J, const double Jc[2][9], const double Jp[2][3]) {
  double v[24];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int m = 0; m < 9; ++m) v[i * 9 + m] = Jc[i][m];
#pragma unroll
    for (int m = 0; m < 3; ++m) v[JP + i * 3 + m] = Jp[i][m];
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    f64x2 t;
    t.x = v[2 * k];
    t.y = v[2 * k + 1];
    *reinterpret_cast<f64x2*>(J + 2 * k) = t;
  }
}

// Q, w and a zero into values [JQ, NJ) of an observation row
__device__ __forceinline__ void store_q(float* J, const double Q[6], double w) {
  f32x4 t;
  t.x = (float)Q[0];
  t.y = (float)Q[1];
  t.z = (float)Q[2];
  t.w = (float)Q[3];
  *reinterpret_cast<f32x4*>(J + JQ) = t;
  t.x = (float)Q[4];
  t.y = (float)Q[5];
  t.z = (float)w;
  t.w = 0.0f;
  *reinterpret_cast<f32x4*>(J + JQ + 4) = t;
}

__device__ __forceinline__ void store_q(double* J, const double Q[6], double w) {
  f64x2 t;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    t.x = Q[2 * k];
    t.y = Q[2 * k + 1];
    *reinterpret_cast<f64x2*>(J + JQ + 2 * k) = t;
  }
  t.x = w;
  t.y = 0.0;
  *reinterpret_cast<f64x2*>(J + JW) = t;
}

__device__ __forceinline__ void load_sym3(const double* __restrict__ s, double M[3][3]) {
  M[0][0] = s[0]; M[0][1] = s[1]; M[0][2] = s[2];
  M[1][0] = s[1]; M[1][1] = s[3]; M[1][2] = s[4];
  M[2][0] = s[2]; M[2][1] = s[4]; M[2][2] = s[5];
}

// ---------------------------------------------------------------------------
// damped point block V*_j = V_j + lambda clamp(diag V_j) (Eq. 2 with the
// clamp of Sec. IV-B-3), its inverse (adjugate / determinant, FP64) and
// ep_j = V*_j^-1 gp_j; the determinant test flags a block that is not
// positive definite.  Returns the inverse as its upper triangle.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void damp_point(const double v[6], const double g[3], double lam, double dmin,
                                           double dmax, double vi[6], double e[3], int* error) {
  const double m00 = v[0] + lam * fmin(fmax(v[0], dmin), dmax);
  const double m11 = v[3] + lam * fmin(fmax(v[3], dmin), dmax);
  const double m22 = v[5] + lam * fmin(fmax(v[5], dmin), dmax);
  const double m01 = v[1], m02 = v[2], m12 = v[4];
  const double c00 = m11 * m22 - m12 * m12;
  const double c01 = m02 * m12 - m01 * m22;
  const double c02 = m01 * m12 - m02 * m11;
  const double c11 = m00 * m22 - m02 * m02;
  const double c12 = m01 * m02 - m00 * m12;
  const double c22 = m00 * m11 - m01 * m01;
  const double det = m00 * c00 + m01 * c01 + m02 * c02;
  if (!(det > 0.0) || !isfinite(det)) atomicOr(error, (int)ERR_POINT_BLOCK);
  const double id = 1.0 / det;
  vi[0] = c00 * id; vi[1] = c01 * id; vi[2] = c02 * id;
  vi[3] = c11 * id; vi[4] = c12 * id; vi[5] = c22 * id;
  e[0] = (c00 * g[0] + c01 * g[1] + c02 * g[2]) * id;
  e[1] = (c01 * g[0] + c11 * g[1] + c12 * g[2]) * id;
  e[2] = (c02 * g[0] + c12 * g[1] + c22 * g[2]) * id;
}

// the PCG grid barrier of this step starts from a clean state (threads
// 0..MAX_BARRIER_GROUPS of the first workgroup)
__device__ __forceinline__ void reset_grid_sync(GridSync* gs, int j) {
  if (j <= MAX_BARRIER_GROUPS) {
    if (j == 0) {
      gs->count = 0u;
      gs->gen = 0u;
    } else {
      gs->group[j - 1].count = 0u;
    }
  }
}

// Q_x = w Jp_x V*^-1 and e_x = Jp_x ep_j of one observation
__device__ __forceinline__ void point_factors(const double Jp[2][3], double w, const double vi[6],
                                              const double ep[3], double Q[6], double e[2]) {
  double Vi[3][3];
  load_sym3(vi, Vi);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int m = 0; m < 3; ++m) Q[3 * i + m] = w * (Jp[i][0] * Vi[0][m] + Jp[i][1] * Vi[1][m] + Jp[i][2] * Vi[2][m]);
    e[i] = Jp[i][0] * ep[0] + Jp[i][1] * ep[1] + Jp[i][2] * ep[2];
  }
}

__device__ __forceinline__ void store_rec(double* rec, double r0, double r1, double w, double e0, double e1) {
  f64x2* rc = reinterpret_cast<f64x2*>(rec);
  f64x2 t;
  t.x = r0;
  t.y = r1;
  rc[0] = t;
  t.x = w;
  t.y = 0.0;
  rc[1] = t;
  t.x = e0;
  t.y = e1;
  rc[2] = t;
  t.x = 0.0;
  t.y = 0.0;
  rc[3] = t;
}

// ---------------------------------------------------------------------------
// observation pass: residual, Jacobian blocks, robust weight, cost, the
// point-keyed blocks V_j = sum w Jp^T Jp, gp_j = sum w Jp^T r (Alg. 1 first
// two lines; Sec. IV-A-2 batched Jacobian values), and, with the current
// lambda, the point elimination: V*_j^-1, ep_j and per observation the Schur
// factor Q_x and e_x.  One workgroup per point-aligned chunk; segmented sums
// in LDS, fixed order.  Every observation row and record is written whole.
// ---------------------------------------------------------------------------
// Observation x of the linearisation: residual, robust weight and cost,
// Jacobian row (written with w) and its 9 terms of the point sums (upper V_j,
// then gp_j).
template <typename T>
__device__ __forceinline__ void lin_observation(const LinArgs& a, int x, double (&Jp)[2][3], double& rx,
                                                double& ry, double& w, double& cost, double (&sv)[9]) {
  const int ci = a.o_cam[x];
  const int pj = a.o_pt[x];
  const Camera cam = load_camera(a.cams + 10 * (size_t)ci);
  const double* P = a.pts + 3 * (size_t)pj;
  double Jc[2][9];
  const Proj pr = project_jac(cam, v3(P[0], P[1], P[2]), Jc, Jp);
  rx = pr.px - a.o_xy[2 * (size_t)x];
  ry = pr.py - a.o_xy[2 * (size_t)x + 1];
  double drho;
  const double rho = robust_rho(rx * rx + ry * ry, a.huber, &drho);
  const double om = a.o_w[x];
  w = om * drho;
  cost = 0.5 * om * rho;
  const uint8_t fx = a.fixed[ci];
  if (fx & FIXED_CAMERA) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int m = 0; m < 9; ++m) Jc[i][m] = 0.0;
  } else if (fx & FIXED_INTRINSICS) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int m = 6; m < 9; ++m) Jc[i][m] = 0.0;
  }
  a.w[x] = w;
  store_row(reinterpret_cast<T*>(a.J) + (size_t)x * NJ, Jc, Jp);
  sv[0] = w * (Jp[0][0] * Jp[0][0] + Jp[1][0] * Jp[1][0]);
  sv[1] = w * (Jp[0][0] * Jp[0][1] + Jp[1][0] * Jp[1][1]);
  sv[2] = w * (Jp[0][0] * Jp[0][2] + Jp[1][0] * Jp[1][2]);
  sv[3] = w * (Jp[0][1] * Jp[0][1] + Jp[1][1] * Jp[1][1]);
  sv[4] = w * (Jp[0][1] * Jp[0][2] + Jp[1][1] * Jp[1][2]);
  sv[5] = w * (Jp[0][2] * Jp[0][2] + Jp[1][2] * Jp[1][2]);
  sv[6] = w * (Jp[0][0] * rx + Jp[1][0] * ry);
  sv[7] = w * (Jp[0][1] * rx + Jp[1][1] * ry);
  sv[8] = w * (Jp[0][2] * rx + Jp[1][2] * ry);
}

// The point-elimination factors of observation x from Jp as stored
// (precision T), like every other reader of the row: both sides of the Schur
// pair product and the right-hand side then use one rounding of Jp, which
// keeps the reduced system symmetric.
template <typename T>
__device__ __forceinline__ void lin_factors(const LinArgs& a, int x, const double (&Jp)[2][3], double rx,
                                            double ry, double w, const double (&pv)[6], const double (&pe)[3]) {
  double Jq[2][3], Q[6], e[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int m = 0; m < 3; ++m) Jq[i][m] = (double)(T)Jp[i][m];
  point_factors(Jq, w, pv, pe, Q, e);
  store_q(reinterpret_cast<T*>(a.J) + (size_t)x * NJ, Q, w);
  store_rec(a.rec + 8 * (size_t)x, rx, ry, w, e[0], e[1]);
}

// A chunk holding one point seen more than CHUNK times: each thread takes
// the point's observations t, t + CHUNK, ... and sums their terms in that
// order; the threads' partials are then added in a fixed order.  The
// observations' Jp, r and w for the factors are read back from the row and
// the weight array.
// red: CHUNK / 64 doubles; lds: 3 CHUNK / 64 + 9 doubles (reductions, then
// the point's factors handed to every thread).
template <typename T>
__device__ void linearize_long_track(const LinArgs& a, int c, int x0, int x1, double* red, double* lds) {
  double* const bc = lds + 3 * (CHUNK / 64);
  const int t = threadIdx.x, j = a.chunk_pt[c];
  double cost = 0.0, sv[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) sv[q] = 0.0;
  for (int x = x0 + t; x < x1; x += CHUNK) {
    double Jp[2][3], rx, ry, w, cx, so[9];
    lin_observation<T>(a, x, Jp, rx, ry, w, cx, so);
    a.rec[8 * (size_t)x] = rx;
    a.rec[8 * (size_t)x + 1] = ry;
    cost += cx;
#pragma unroll
    for (int q = 0; q < 9; ++q) sv[q] += so[q];
  }
  for (int q = 0; q < 9; q += 3) block_sum3(sv[q], sv[q + 1], sv[q + 2], lds);
  double gmax = 0.0;
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) a.V[6 * (size_t)j + q] = sv[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a.gp[3 * (size_t)j + q] = sv[6 + q];
    gmax = fmax(fabs(sv[6]), fmax(fabs(sv[7]), fabs(sv[8])));
    double vi[6], ep[3];
    damp_point(sv, sv + 6, a.dev->lambda, a.dmin, a.dmax, vi, ep, &a.dev->error);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      a.Vinv[6 * (size_t)j + q] = vi[q];
      bc[q] = vi[q];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a.ep[3 * (size_t)j + q] = ep[q];
      bc[6 + q] = ep[q];
    }
  }
  __syncthreads();
  double pv[6], pe[3];
#pragma unroll
  for (int q = 0; q < 6; ++q) pv[q] = bc[q];
#pragma unroll
  for (int q = 0; q < 3; ++q) pe[q] = bc[6 + q];
  const T* Jall = reinterpret_cast<const T*>(a.J);
  for (int x = x0 + t; x < x1; x += CHUNK) {
    double Jp[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int m = 0; m < 3; ++m) Jp[i][m] = (double)Jall[(size_t)x * NJ + JP + 3 * i + m];
    lin_factors<T>(a, x, Jp, a.rec[8 * (size_t)x], a.rec[8 * (size_t)x + 1], a.w[x], pv, pe);
  }
  const double tot = block_sum(cost, red);
  const double gm = block_max(gmax, red);
  if (t == 0) {
    a.part_cost[c] = tot;
    a.part_gmax[c] = gm;
  }
}

template <typename T>
__global__ __launch_bounds__(CHUNK) void k_linearize(LinArgs a) {
  __shared__ double sh[9][CHUNK];
  __shared__ double red[CHUNK / 64];
  const int c = blockIdx.x;
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1];
  const int t = threadIdx.x;
  const int x = x0 + t;
  if (c == 0) reset_grid_sync(a.gs, t);
  if (x1 - x0 > CHUNK) return;  // one long track: k_linearize_long
  double cost = 0.0;
  double Jp[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  double rx = 0.0, ry = 0.0, w = 0.0;
  int pj = 0;
  if (x < x1) {
    pj = a.o_pt[x];
    double sv[9];
    lin_observation<T>(a, x, Jp, rx, ry, w, cost, sv);
#pragma unroll
    for (int q = 0; q < 9; ++q) sh[q][t] = sv[q];
  }
  __syncthreads();
  double gmax = 0.0;
  const int j0 = a.chunk_pt[c], j1 = a.chunk_pt[c + 1];
  const double lam = a.dev->lambda;
  // a chunk holds at most CHUNK points: one per thread
  const int j = j0 + t;
  double vi[6], ep[3];
  if (j < j1) {
    double s[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q] = 0.0;
    const int lo = a.pt_ptr[j] - x0, hi = a.pt_ptr[j + 1] - x0;
    for (int y = lo; y < hi; ++y)
#pragma unroll
      for (int q = 0; q < 9; ++q) s[q] += sh[q][y];
#pragma unroll
    for (int q = 0; q < 6; ++q) a.V[6 * (size_t)j + q] = s[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a.gp[3 * (size_t)j + q] = s[6 + q];
    gmax = fmax(fabs(s[6]), fmax(fabs(s[7]), fabs(s[8])));
    damp_point(s, s + 6, lam, a.dmin, a.dmax, vi, ep, &a.dev->error);
#pragma unroll
    for (int q = 0; q < 6; ++q) a.Vinv[6 * (size_t)j + q] = vi[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a.ep[3 * (size_t)j + q] = ep[q];
  }
  __syncthreads();  // the observation sums are consumed: sh holds the points now
  if (j < j1) {
#pragma unroll
    for (int q = 0; q < 6; ++q) sh[q][t] = vi[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) sh[6 + q][t] = ep[q];
  }
  __syncthreads();
  if (x < x1) {
    const int k = pj - j0;
    double pv[6], pe[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) pv[q] = sh[q][k];
#pragma unroll
    for (int q = 0; q < 3; ++q) pe[q] = sh[6 + q][k];
    lin_factors<T>(a, x, Jp, rx, ry, w, pv, pe);
  }
  const double tot = block_sum(cost, red);
  const double gm = block_max(gmax, red);
  if (t == 0) {
    a.part_cost[c] = tot;
    a.part_gmax[c] = gm;
  }
}

// The chunks of one point seen more than CHUNK times (one workgroup each).
template <typename T>
__global__ __launch_bounds__(CHUNK) void k_linearize_long(LinArgs a, const int32_t* chunks) {
  __shared__ double red[CHUNK / 64];
  __shared__ double lds[3 * (CHUNK / 64) + 9];
  const int c = chunks[blockIdx.x];
  linearize_long_track<T>(a, c, a.chunk_ptr[c], a.chunk_ptr[c + 1], red, lds);
}

// F = sum of the chunk partials (fixed order), and the gradient max over points.
__global__ __launch_bounds__(1024) void k_reduce_cost(const double* __restrict__ part, int n,
                                                      DevScalars* dev) {
  __shared__ double red[16];
  const double F = block_sum_array4(part, n, red);
  if (threadIdx.x == 0) dev->F = F;
}

// ---------------------------------------------------------------------------
// damping of the point blocks and their inverses (Eq. 2 with the clamp of
// Sec. IV-B-3): V*_j = V_j + lambda clamp(diag V_j), Vinv_j = V*_j^-1 by the
// adjugate, ep_j = Vinv_j gp_j.  One thread per point, FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_damp_points(DampArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  reset_grid_sync(a.gs, j);
  if (j >= a.np) return;
  double v[6], g[3], vi[6], e[3];
#pragma unroll
  for (int q = 0; q < 6; ++q) v[q] = a.V[6 * (size_t)j + q];
#pragma unroll
  for (int q = 0; q < 3; ++q) g[q] = a.gp[3 * (size_t)j + q];
  damp_point(v, g, a.dev->lambda, a.dmin, a.dmax, vi, e, &a.dev->error);
#pragma unroll
  for (int q = 0; q < 6; ++q) a.Vinv[6 * (size_t)j + q] = vi[q];
#pragma unroll
  for (int q = 0; q < 3; ++q) a.ep[3 * (size_t)j + q] = e[q];
}

// ---------------------------------------------------------------------------
// per-observation factor of the Schur product: Q_x = w_x Jp_x Vinv_j (2x3),
// stored in the Jacobian precision into the observation's row with w, and
// e_x = Jp_x ep_j (FP64, for the Schur right-hand side) into its record
// (one thread per observation).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_point_q(PointQArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.no) return;
  T* row = reinterpret_cast<T*>(a.J) + (size_t)x * NJ;
  const int j = a.o_pt[x];
  double Jq[2][3], vi[6], pe[3], Q[6], e[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int m = 0; m < 3; ++m) Jq[i][m] = (double)row[JP + 3 * i + m];
#pragma unroll
  for (int q = 0; q < 6; ++q) vi[q] = a.Vinv[6 * (size_t)j + q];
#pragma unroll
  for (int q = 0; q < 3; ++q) pe[q] = a.ep[3 * (size_t)j + q];
  const double w = a.w[x];
  point_factors(Jq, w, vi, pe, Q, e);
  store_q(row, Q, w);
  f64x2* rc = reinterpret_cast<f64x2*>(a.rec + 8 * (size_t)x + 4);
  f64x2 t;
  t.x = e[0];
  t.y = e[1];
  rc[0] = t;
  t.x = 0.0;
  t.y = 0.0;
  rc[1] = t;
}

// ---------------------------------------------------------------------------
// Schur blocks from the pair table (Sec. IV-B-1 numeric phase on the cached
// table): for block (a, b) and pairs (x, y) sharing a point, x in camera a,
// y in camera b,
//   S_ab  = -sum Jc_x^T (Q_x (w_y Jp_y)^T) Jc_y                  (a < b)
//   S_aa' = sum Jc_x^T ([x = y] w_x I - Q_x (w_y Jp_y)^T) Jc_y   (undamped)
// Each workgroup holds SCHUR_SLOTS chunk slots, SCHUR_WAVE_SLOTS per
// wavefront; SCHUR_LANES = 3 lanes share a chunk, lane k accumulating
// columns 3k..3k+2 of the block (27 values) in registers.  A wavefront
// advances its 21 chunks in lockstep steps: at each step the whole
// wavefront stages the two observation rows of every chunk's current pair
// in LDS with contiguous 16-byte loads (8 lanes per 128-byte row), the next
// step's rows being in flight while the current pair is multiplied out of
// LDS; so every row costs one cache line instead of a broadcast load per
// value.  The chunks of one block sit in consecutive slots of one workgroup
// and are summed in slot order through LDS: no atomics, fixed summation
// order.  Off-diagonal blocks go to S (precision T); diagonal blocks, still
// to be damped, to the FP64 buffer Sdiag.  The self pairs (x, x) of a
// diagonal block visit every observation of its camera once, so the same
// lanes also form the camera vectors
//   gc_a = sum w Jc^T r,  diagU_a = diag(sum w Jc^T Jc),
//   bS_a + gc_a = sum w Jc^T e,  e = Jp ep_j,
// from the observation's FP64 record, staged in place of the (repeated) y
// row: this saves a pass over the observations in camera order.
// ---------------------------------------------------------------------------
template <typename T> struct SchurStage {
  static constexpr int ROW_BYTES = NJ * (int)sizeof(T);          // 128 or 256
  static constexpr int PIECES = ROW_BYTES / 16;                   // 16-byte pieces per row
  static constexpr int EPP = 16 / (int)sizeof(T);                 // values per piece
  static constexpr int LOADS = (SCHUR_ROWS * PIECES + 63) / 64;   // staging loads per lane
  // room for every piece the lanes move (rows past SCHUR_ROWS included), so
  // that the LDS stores need no lane-dependent branch: such a branch inside
  // the lockstep loop lets the compiler restructure it into a divergent nest
  static constexpr int WAVE_BYTES = LOADS * 64 * 16;
};

constexpr int SCHUR_PART_BYTES = SCHUR_SLOTS * 81 * 8;
constexpr int schur_lds_bytes(int stage) { return stage > SCHUR_PART_BYTES ? stage : SCHUR_PART_BYTES; }

// piece p of staged row r lives at piece p ^ (slot & 7): the rows of the
// wavefront's slots start in different banks
__device__ __forceinline__ int stage_piece(int r, int p) { return p ^ ((r >> 1) & 7); }

template <typename T>
__device__ __forceinline__ T stage_val(const unsigned char* st, int r, int e) {
  constexpr int EPP = SchurStage<T>::EPP;
  return *reinterpret_cast<const T*>(st + r * SchurStage<T>::ROW_BYTES + stage_piece(r, e / EPP) * 16 +
                                     (e % EPP) * (int)sizeof(T));
}

// 16-byte piece p of staged row r, as EPP values
template <typename T>
__device__ __forceinline__ void stage_piece_vals(const unsigned char* st, int r, int p, T* out) {
  const unsigned char* src = st + r * SchurStage<T>::ROW_BYTES + stage_piece(r, p) * 16;
  if constexpr (sizeof(T) == 4) {
    const f32x4 t = *reinterpret_cast<const f32x4*>(src);
    out[0] = t.x;
    out[1] = t.y;
    out[2] = t.z;
    out[3] = t.w;
  } else {
    const f64x2 t = *reinterpret_cast<const f64x2*>(src);
    out[0] = t.x;
    out[1] = t.y;
  }
}

// acc[r][c] += (Jc_x^T M Jc_y)[r][c0 + c],
// M = [x = y] w_y I - w_y Q_x Jp_y^T
template <typename T>
__device__ __forceinline__ void pair_update(double (&acc)[9][3], const T (&jx)[20], const T (&q)[8],
                                            const T (&jy)[6], const T (&py)[6], double w, bool self) {
  double M[2][2];
#pragma unroll
  for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2)
      M[i2][k2] = -w * ((double)q[3 * i2] * (double)py[3 * k2] + (double)q[3 * i2 + 1] * (double)py[3 * k2 + 1] +
                        (double)q[3 * i2 + 2] * (double)py[3 * k2 + 2]);
  if (self) {
    M[0][0] += w;
    M[1][1] += w;
  }
  double g0[3], g1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double a0 = (double)jy[c], a1 = (double)jy[3 + c];
    g0[c] = M[0][0] * a0 + M[0][1] * a1;
    g1[c] = M[1][0] * a0 + M[1][1] * a1;
  }
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const double j0 = (double)jx[r], j1 = (double)jx[9 + r];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = fma(j1, g1[c], fma(j0, g0[c], acc[r][c]));
  }
}

template <typename T>
__global__ __launch_bounds__(SCHUR_THREADS) void k_schur_pairs(SchurArgs a) {
  using SS = SchurStage<T>;
  // staging rows during the steps; per slot the 81 block values afterwards,
  // then (diagonal blocks) the camera vectors
  __shared__ __align__(16) unsigned char lds[schur_lds_bytes(SCHUR_WAVES * SS::WAVE_BYTES)];
  double(*part)[81] = reinterpret_cast<double(*)[81]>(lds);
  // workgroups are dispatched round-robin over the 8 XCDs: XCD k takes the
  // k-th contiguous range of slot workgroups, so that neighbouring rows (which
  // read the same observations) share that XCD's L2
  const int per = (a.nwg + 7) / 8;
  const int lw = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (lw >= a.nwg) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = lane / SCHUR_LANES;              // slot within the wavefront (s < 21 computes)
  const int c0 = 3 * (lane - SCHUR_LANES * s);
  const bool computes = s < SCHUR_WAVE_SLOTS;
  const int slot = wave * SCHUR_WAVE_SLOTS + s;  // slot within the workgroup
  const size_t sbase = (size_t)lw * SCHUR_SLOTS;
  unsigned char* st = lds + wave * SS::WAVE_BYTES;
  const unsigned char* __restrict__ Jb = reinterpret_cast<const unsigned char*>(a.J);

  // per slot, for the reduction: number of chunks when the slot leads its
  // block (else 0) and the destination: block e of S, or -1 - row for the
  // diagonal block of camera row (Sdiag)
  __shared__ int slot_n[SCHUR_SLOTS], slot_dst[SCHUR_SLOTS], slot_pn[SCHUR_SLOTS];
  bool diag_slot = false;
  if (computes) {
    const int e = a.slot_blk[sbase + slot];
    int row = 0;
    if (e >= 0) {
      row = a.blk_row[e];
      // (a camera without observations has an empty diagonal block: zeros)
      diag_slot = a.S_ptr[row] == e;
    }
    if (c0 == 0) {
      const int n = a.slot_lead[sbase + slot];
      slot_n[slot] = n;
      slot_dst[slot] = diag_slot ? -1 - row : e;
      if (a.SI && n > 0 && !diag_slot) slot_pn[slot] = a.blk_pos[e];
    }
  }
  const int t0 = a.swptr[(size_t)lw * SCHUR_WAVES + wave];
  const int nt = a.swptr[(size_t)lw * SCHUR_WAVES + wave + 1] - t0;
  const int* __restrict__ tab = a.stab + (size_t)t0 * SCHUR_ROWS;

  // staging: lane `lane` moves piece (64 k + lane) % PIECES of row
  // (64 k + lane) / PIECES for k < LOADS.  Every load is issued without a
  // branch (a slot without a pair reads unit 0, rows past SCHUR_ROWS repeat
  // the last one, a record's pieces past its end read the next records), so
  // the compiler's wait counting keeps the next step's loads in flight
  // across the multiplication of the current one.
  int code[SS::LOADS];
  f32x4 buf[SS::LOADS];
  auto fetch_codes = [&](int t) {
#pragma unroll
    for (int k = 0; k < SS::LOADS; ++k) {
      const int r = min((64 * k + lane) / SS::PIECES, SCHUR_ROWS - 1);
      code[k] = tab[(size_t)t * SCHUR_ROWS + r];
    }
  };
  auto fetch_rows = [&]() {
#pragma unroll
    for (int k = 0; k < SS::LOADS; ++k) {
      const int p = (64 * k + lane) % SS::PIECES;
      buf[k] = *reinterpret_cast<const f32x4*>(Jb + (size_t)max(code[k], 0) * 64 + p * 16);
    }
  };
  auto stage_rows = [&]() {
#pragma unroll
    for (int k = 0; k < SS::LOADS; ++k) {
      const int q = 64 * k + lane, r = q / SS::PIECES, p = q % SS::PIECES;
      *reinterpret_cast<f32x4*>(st + r * SS::ROW_BYTES + stage_piece(r, p) * 16) = buf[k];
    }
  };

  double acc[9][3];
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = 0.0;
  double vg[3] = {0.0, 0.0, 0.0}, vb[3] = {0.0, 0.0, 0.0}, vu[3] = {0.0, 0.0, 0.0};

  const int ys = min(2 * s + 1, SCHUR_ROWS - 1);  // this lane's y code (lane 63 reads a valid one)
  if (nt > 0) {
    fetch_codes(0);
    fetch_rows();
    int ycode = computes ? tab[ys] : -1;
    fetch_codes(min(1, nt - 1));
    stage_rows();
    for (int t = 0; t < nt; ++t) {
      // rows of step t + 1 in flight, codes of step t + 2 requested (steps
      // past the last repeat it: loaded, never staged)
      fetch_rows();
      fetch_codes(min(t + 2, nt - 1));
      const int yn = tab[(size_t)min(t + 1, nt - 1) * SCHUR_ROWS + ys];
      const int ycode_next = computes ? yn : -1;
      __builtin_amdgcn_wave_barrier();
      if (computes && ycode != -1) {
        const bool self = ycode >= a.rec_unit;
        const int rx = 2 * s, ry = self ? rx : rx + 1;
        T jx[20], q[8], jy[6], py[6];
#pragma unroll
        for (int p = 0; p < 20 / SS::EPP; ++p) stage_piece_vals<T>(st, rx, p, jx + p * SS::EPP);
#pragma unroll
        for (int p = 0; p < 8 / SS::EPP; ++p) stage_piece_vals<T>(st, rx, JQ / SS::EPP + p, q + p * SS::EPP);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          jy[c] = stage_val<T>(st, ry, c0 + c);
          jy[3 + c] = stage_val<T>(st, ry, 9 + c0 + c);
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) py[m] = stage_val<T>(st, ry, JP + m);
        const double w = (double)stage_val<T>(st, ry, JW);
        pair_update<T>(acc, jx, q, jy, py, w, self);
        if (self) {
          // the record r0, r1, w, 0, e0, e1 staged in row rx + 1 (FP64)
          double rv[6];
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            const f64x2 v = *reinterpret_cast<const f64x2*>(st + (rx + 1) * SS::ROW_BYTES + stage_piece(rx + 1, p) * 16);
            rv[2 * p] = v.x;
            rv[2 * p + 1] = v.y;
          }
          const double r0 = rv[0], r1 = rv[1], wx = rv[2], e0 = rv[4], e1 = rv[5];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double j0 = (double)jy[c], j1 = (double)jy[3 + c];
            vg[c] += wx * (j0 * r0 + j1 * r1);
            vb[c] += wx * (j0 * e0 + j1 * e1);
            vu[c] += wx * (j0 * j0 + j1 * j1);
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (t + 1 < nt) stage_rows();
      ycode = ycode_next;
    }
  }
  __syncthreads();  // the staging area becomes the partial-sum area
  if (computes) {
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) part[slot][r * 9 + c0 + c] = acc[r][c];
  }
  __syncthreads();
  // every lead slot sums its block's chunk partials in slot order
  for (int t = threadIdx.x; t < SCHUR_SLOTS * 81; t += blockDim.x) {
    const int sl = t / 81, qq = t - 81 * (t / 81);
    const int n = slot_n[sl];
    if (n == 0) continue;
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += part[sl + k][qq];
    const int dst = slot_dst[sl];
    if (dst < 0) {
      a.Sdiag[81 * (size_t)(-1 - dst) + qq] = v;
    } else {
      reinterpret_cast<T*>(a.S)[81 * (size_t)dst + qq] = (T)v;
      if (a.SI) {
        T* si = reinterpret_cast<T*>(a.SI);
        const size_t pn = (size_t)slot_pn[sl] * SI_STRIDE;
        si[pn + qq] = (T)v;
        if (qq < SI_STRIDE - 81) si[pn + 81 + qq] = (T)0;
      }
    }
  }
  // camera vectors of the diagonal blocks, through the same LDS
  if (!__syncthreads_or(diag_slot)) return;
  if (diag_slot)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      part[slot][c0 + c] = vg[c];
      part[slot][9 + c0 + c] = vb[c];
      part[slot][18 + c0 + c] = vu[c];
    }
  __syncthreads();
  for (int t = threadIdx.x; t < SCHUR_SLOTS * 27; t += blockDim.x) {
    const int sl = t / 27, qq = t - 27 * (t / 27);
    const int n = slot_n[sl], dst = slot_dst[sl];
    if (n == 0 || dst >= 0) continue;
    const size_t row = (size_t)(-1 - dst);
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += part[sl + k][qq];
    if (qq < 9) a.gc[9 * row + qq] = v;
    else if (qq < 18) a.bS[9 * row + (qq - 9)] = v;  // - gc, added by the camera finish
    else a.diagU[9 * row + (qq - 18)] = v;
  }
}

// ---------------------------------------------------------------------------
// diagonal blocks: S_aa = Sdiag_a + lambda clamp(diagU_a) (Eq. 2 damping with
// the clamp of Sec. IV-B-3), kept in FP64 (damped in place), and the block-Jacobi
// preconditioner Minv_a = S_aa^-1 by Cholesky in FP64 (one workgroup per
// camera; the factorisation by one lane).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_camera_finish(CamFinishArgs a) {
  __shared__ double Sd[81];
  const int cam = blockIdx.x;
  const double lam = a.dev->lambda;
  // right-hand side of the reduced system: bS = -gc + sum w Jc^T Jp ep
  if (a.gc && threadIdx.x < 9) a.bS[9 * (size_t)cam + threadIdx.x] -= a.gc[9 * (size_t)cam + threadIdx.x];
  for (int q = threadIdx.x; q < 81; q += blockDim.x) {
    double v = a.Sdiag[81 * (size_t)cam + q];
    const int r = q / 9;
    if (q == 10 * r) v += lam * fmin(fmax(a.diagU[9 * (size_t)cam + r], a.dmin), a.dmax);
    Sd[q] = v;
    a.Sdiag[81 * (size_t)cam + q] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double L[81];
    for (int q = 0; q < 81; ++q) L[q] = Sd[q];
    bool ok = true;
    for (int k = 0; k < 9; ++k) {
      double d = L[k * 9 + k];
      for (int m = 0; m < k; ++m) d -= L[k * 9 + m] * L[k * 9 + m];
      if (!(d > 0.0)) {
        ok = false;
        d = 1.0;
      }
      d = sqrt(d);
      L[k * 9 + k] = d;
      for (int i2 = k + 1; i2 < 9; ++i2) {
        double s = L[i2 * 9 + k];
        for (int m = 0; m < k; ++m) s -= L[i2 * 9 + m] * L[k * 9 + m];
        L[i2 * 9 + k] = s / d;
      }
    }
    if (!ok) atomicOr(&a.dev->error, (int)ERR_CAMERA_BLOCK);
    double Li[81];
    for (int q = 0; q < 81; ++q) Li[q] = 0.0;
    for (int i2 = 0; i2 < 9; ++i2) {
      Li[i2 * 9 + i2] = 1.0 / L[i2 * 9 + i2];
      for (int k = i2 + 1; k < 9; ++k) {
        double s = 0.0;
        for (int m = i2; m < k; ++m) s += L[k * 9 + m] * Li[m * 9 + i2];
        Li[k * 9 + i2] = -s / L[k * 9 + k];
      }
    }
    if (a.Linv)
      for (int q = 0; q < 81; ++q) a.Linv[81 * (size_t)cam + q] = Li[q];
    double* Mi = a.Minv + 81 * (size_t)cam;
    for (int r = 0; r < 9; ++r)
      for (int cc = 0; cc < 9; ++cc) Mi[r * 9 + cc] = lt_times(Li, Li, r, cc);
  }
}

// ---------------------------------------------------------------------------
// back-substitution and the predicted reduction (one workgroup per chunk):
//   dp_j = Vinv_j (-gp_j - sum_x w_x Jp_x^T Jc_x dc_{c_x}),
//   pred partials: gp_j . dp_j and sum_x w_x |Jc_x dc + Jp_x dp_j|^2,
//   candidate points p'_j = p_j + dp_j.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(CHUNK) void k_backsub(BackArgs a) {
  __shared__ double tk[3][CHUNK];
  __shared__ double red[CHUNK / 64];
  const int c = blockIdx.x;
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1];
  if (x1 - x0 > CHUNK) return;  // one long track: k_backsub_long
  const int t = threadIdx.x, x = x0 + t;
  const T* __restrict__ Jall = reinterpret_cast<const T*>(a.J);
  double Jc[2][9], Jp[2][3], w = 0.0, ec0 = 0.0, ec1 = 0.0;
  int j = -1;
  if (x < x1) {
    j = a.o_pt[x];
    load_J(Jall + (size_t)x * NJ, Jc, Jp);
    w = a.w[x];
    const double* dc = a.dc + 9 * (size_t)a.o_cam[x];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      ec0 += Jc[0][m] * dc[m];
      ec1 += Jc[1][m] * dc[m];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) tk[m][t] = w * (Jp[0][m] * ec0 + Jp[1][m] * ec1);
  }
  __syncthreads();
  double lin = 0.0;
  const int j0 = a.chunk_pt[c], j1 = a.chunk_pt[c + 1];
  for (int jj = j0 + t; jj < j1; jj += blockDim.x) {
    const double* g = a.gp + 3 * (size_t)jj;
    double s0 = -g[0], s1 = -g[1], s2 = -g[2];
    const int lo = a.pt_ptr[jj] - x0, hi = a.pt_ptr[jj + 1] - x0;
    for (int y = lo; y < hi; ++y) {
      s0 -= tk[0][y];
      s1 -= tk[1][y];
      s2 -= tk[2][y];
    }
    const double* vi = a.Vinv + 6 * (size_t)jj;
    const double d0 = vi[0] * s0 + vi[1] * s1 + vi[2] * s2;
    const double d1 = vi[1] * s0 + vi[3] * s1 + vi[4] * s2;
    const double d2 = vi[2] * s0 + vi[4] * s1 + vi[5] * s2;
    double* dp = a.dp + 3 * (size_t)jj;
    dp[0] = d0; dp[1] = d1; dp[2] = d2;
    const double* P = a.pts + 3 * (size_t)jj;
    double* Pn = a.pts_new + 3 * (size_t)jj;
    Pn[0] = P[0] + d0; Pn[1] = P[1] + d1; Pn[2] = P[2] + d2;
    lin += g[0] * d0 + g[1] * d1 + g[2] * d2;
  }
  __syncthreads();
  double quad = 0.0;
  if (x < x1) {
    const double* dp = a.dp + 3 * (size_t)j;
    const double e0 = ec0 + Jp[0][0] * dp[0] + Jp[0][1] * dp[1] + Jp[0][2] * dp[2];
    const double e1 = ec1 + Jp[1][0] * dp[0] + Jp[1][1] * dp[1] + Jp[1][2] * dp[2];
    quad = w * (e0 * e0 + e1 * e1);
  }
  const double ql = block_sum(quad, red);
  const double ll = block_sum(lin, red);
  if (t == 0) {
    a.part_pred[2 * (size_t)c] = ql;
    a.part_pred[2 * (size_t)c + 1] = ll;
  }
}

// The chunks of one point seen more than CHUNK times: each thread takes the
// point's observations t, t + CHUNK, ... (sums in that order, then over the
// threads in a fixed order); thread 0 forms dp.
template <typename T>
__global__ __launch_bounds__(CHUNK) void k_backsub_long(BackArgs a, const int32_t* chunks) {
  __shared__ double red[CHUNK / 64];
  __shared__ double lds[3 * (CHUNK / 64) + 3];
  const int c = chunks[blockIdx.x];
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1], j = a.chunk_pt[c], t = threadIdx.x;
  const T* __restrict__ Jall = reinterpret_cast<const T*>(a.J);
  auto cam_term = [&](int x, double (&Jp)[2][3], double& w, double& ec0, double& ec1) {
    double Jc[2][9];
    load_J(Jall + (size_t)x * NJ, Jc, Jp);
    w = a.w[x];
    const double* dc = a.dc + 9 * (size_t)a.o_cam[x];
    ec0 = 0.0;
    ec1 = 0.0;
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      ec0 += Jc[0][m] * dc[m];
      ec1 += Jc[1][m] * dc[m];
    }
  };
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int x = x0 + t; x < x1; x += CHUNK) {
    double Jp[2][3], w, ec0, ec1;
    cam_term(x, Jp, w, ec0, ec1);
    s0 += w * (Jp[0][0] * ec0 + Jp[1][0] * ec1);
    s1 += w * (Jp[0][1] * ec0 + Jp[1][1] * ec1);
    s2 += w * (Jp[0][2] * ec0 + Jp[1][2] * ec1);
  }
  block_sum3(s0, s1, s2, lds);
  double* const dpl = lds + 3 * (CHUNK / 64);
  double lin = 0.0;
  if (t == 0) {
    const double* g = a.gp + 3 * (size_t)j;
    const double r0 = -g[0] - s0, r1 = -g[1] - s1, r2 = -g[2] - s2;
    const double* vi = a.Vinv + 6 * (size_t)j;
    const double d0 = vi[0] * r0 + vi[1] * r1 + vi[2] * r2;
    const double d1 = vi[1] * r0 + vi[3] * r1 + vi[4] * r2;
    const double d2 = vi[2] * r0 + vi[4] * r1 + vi[5] * r2;
    double* dp = a.dp + 3 * (size_t)j;
    dp[0] = d0; dp[1] = d1; dp[2] = d2;
    const double* P = a.pts + 3 * (size_t)j;
    double* Pn = a.pts_new + 3 * (size_t)j;
    Pn[0] = P[0] + d0; Pn[1] = P[1] + d1; Pn[2] = P[2] + d2;
    lin = g[0] * d0 + g[1] * d1 + g[2] * d2;
    dpl[0] = d0; dpl[1] = d1; dpl[2] = d2;
  }
  __syncthreads();
  const double d0 = dpl[0], d1 = dpl[1], d2 = dpl[2];
  double quad = 0.0;
  for (int x = x0 + t; x < x1; x += CHUNK) {
    double Jp[2][3], w, ec0, ec1;
    cam_term(x, Jp, w, ec0, ec1);
    const double e0 = ec0 + Jp[0][0] * d0 + Jp[0][1] * d1 + Jp[0][2] * d2;
    const double e1 = ec1 + Jp[1][0] * d0 + Jp[1][1] * d1 + Jp[1][2] * d2;
    quad += w * (e0 * e0 + e1 * e1);
  }
  const double ql = block_sum(quad, red);
  const double ll = block_sum(lin, red);
  if (t == 0) {
    a.part_pred[2 * (size_t)c] = ql;
    a.part_pred[2 * (size_t)c + 1] = ll;
  }
}

// candidate cameras theta' = Exp(dc) theta (fixed cameras copied) and the
// partials of gc . dc (one thread per camera).
__global__ __launch_bounds__(256) void k_retract_cameras(RetractArgs a) {
  __shared__ double red[4];
  const int cam = blockIdx.x * blockDim.x + threadIdx.x;
  double lin = 0.0;
  if (cam < a.nc) {
    const double* src = a.cams + 10 * (size_t)cam;
    double* dst = a.cams_new + 10 * (size_t)cam;
    const double* dc = a.dc + 9 * (size_t)cam;
    if (a.fixed[cam] & FIXED_CAMERA) {
      for (int q = 0; q < 10; ++q) dst[q] = src[q];
    } else {
      retract_camera(src, dc, dst);
    }
    const double* g = a.gc + 9 * (size_t)cam;
    for (int m = 0; m < 9; ++m) lin += g[m] * dc[m];
  }
  const double s = block_sum(lin, red);
  if (threadIdx.x == 0) a.part_linc[blockIdx.x] = s;
}

// cost at the candidate (one workgroup per chunk)
__global__ __launch_bounds__(CHUNK) void k_candidate_cost(CostArgs a) {
  __shared__ double red[CHUNK / 64];
  const int c = blockIdx.x;
  double cost = 0.0;
  // (more than one pass only in the chunk of a point seen more than CHUNK times)
  for (int x = a.chunk_ptr[c] + threadIdx.x; x < a.chunk_ptr[c + 1]; x += CHUNK) {
    const Camera cam = load_camera(a.cams + 10 * (size_t)a.o_cam[x]);
    const double* P = a.pts + 3 * (size_t)a.o_pt[x];
    const Proj pr = project(cam, v3(P[0], P[1], P[2]));
    const double rx = pr.px - a.o_xy[2 * (size_t)x], ry = pr.py - a.o_xy[2 * (size_t)x + 1];
    double drho;
    const double rho = robust_rho(rx * rx + ry * ry, a.huber, &drho);
    cost += 0.5 * a.o_w[x] * rho;
  }
  const double s = block_sum(cost, red);
  if (threadIdx.x == 0) a.part_cost_new[c] = s;
}

// acceptance reduction, first stage: workgroup w reduces a contiguous slice
// of the chunk partials (candidate cost, the two predicted-reduction terms,
// gradient max) and of gc (max |.|) into stage[q][w]; fixed order
__global__ __launch_bounds__(256) void k_final_stage(FinalArgs a) {
  __shared__ double red[4];
  const int w = blockIdx.x, G = gridDim.x;
  const int lo = (int)((int64_t)a.nchunk * w / G), hi = (int)((int64_t)a.nchunk * (w + 1) / G);
  double f = 0.0, q = 0.0, lp = 0.0, gm = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    f += a.part_cost_new[i];
    q += a.part_pred[2 * (size_t)i];
    lp += a.part_pred[2 * (size_t)i + 1];
    gm = fmax(gm, a.part_gmax[i]);
  }
  const int n9 = 9 * a.nc;
  const int glo = (int)((int64_t)n9 * w / G), ghi = (int)((int64_t)n9 * (w + 1) / G);
  for (int i = glo + threadIdx.x; i < ghi; i += blockDim.x) gm = fmax(gm, fabs(a.gc[i]));
  f = block_sum(f, red);
  q = block_sum(q, red);
  lp = block_sum(lp, red);
  gm = block_max(gm, red);
  if (threadIdx.x == 0) {
    a.stage[w] = f;
    a.stage[FINAL_STAGE_MAX + w] = q;
    a.stage[2 * FINAL_STAGE_MAX + w] = lp;
    a.stage[3 * FINAL_STAGE_MAX + w] = gm;
  }
}

// acceptance and the trust-region damping update (one workgroup, from the
// first stage's partials)
__global__ __launch_bounds__(256) void k_finalize(FinalArgs a) {
  __shared__ double red[4];
  const double Fn = block_sum_array(a.stage, a.nstage, red);
  const double q = block_sum_array(a.stage + FINAL_STAGE_MAX, a.nstage, red);
  const double lp = block_sum_array(a.stage + 2 * FINAL_STAGE_MAX, a.nstage, red);
  const double lc = block_sum_array(a.part_linc, a.ncamblk, red);
  double gm = 0.0;
  for (int i = threadIdx.x; i < a.nstage; i += blockDim.x) gm = fmax(gm, a.stage[3 * FINAL_STAGE_MAX + i]);
  gm = block_max(gm, red);
  if (threadIdx.x == 0) {
    DevScalars* dev = a.dev;
    const double F = dev->F;
    const double lam = dev->lambda;
    const double pred = -(lc + lp) - 0.5 * q;
    const bool accept = isfinite(Fn) && Fn < F && pred > 0.0;
    const double ratio = (F - Fn) / pred;
    double ln = lam;
    if (!accept || ratio <= 0.25) ln = fmin(16.0 * lam, a.lambda_max);
    else if (ratio > 0.75) ln = fmax(0.5 * lam, a.lambda_min);
    dev->lambda = ln;
    if (accept) dev->F = Fn;
    ba_step_info* info = a.info;
    info->cost_before = F;
    info->cost_after = Fn;
    info->lambda_used = lam;
    info->lambda_next = ln;
    info->pred = pred;
    info->grad_inf = gm;
    info->accepted = accept ? 1 : 0;
    info->status = 0;
  }
}

// caller-order <-> internal-order rows (cameras renumbered by the plan)
__global__ __launch_bounds__(256) void k_permute_rows(PermArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int si = a.gather ? a.map[i] : i, di = a.gather ? i : a.map[i];
  const double* s = a.src + (size_t)si * a.src_stride;
  double* d = a.dst + (size_t)di * a.dst_stride;
  for (int k = 0; k < a.width; ++k) d[k] = s[k];
}

// gather the caller's observations into position order, with validation
__global__ __launch_bounds__(256) void k_set_observations(ObsArgs a) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= a.no) return;
  const int64_t k = a.o_orig[x];
  const double px = a.xy[2 * k], py = a.xy[2 * k + 1];
  const double w = a.w ? a.w[k] : 1.0;
  if (!isfinite(px) || !isfinite(py)) atomicOr(&a.dev->error, (int)ERR_NONFINITE_OBS);
  if (!(w > 0.0) || !isfinite(w)) atomicOr(&a.dev->error, (int)ERR_BAD_WEIGHT);
  a.o_xy[2 * x] = px;
  a.o_xy[2 * x + 1] = py;
  a.o_w[x] = w;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
hipError_t launch_linearize(const LinArgs& a, int nchunk, LongChunks lc, hipStream_t s) {
  hipLaunchKernelGGL(k_linearize<T>, dim3(nchunk), dim3(CHUNK), 0, s, a);
  if (lc.n > 0) hipLaunchKernelGGL(k_linearize_long<T>, dim3(lc.n), dim3(CHUNK), 0, s, a, lc.idx);
  return hipGetLastError();
}
template hipError_t launch_linearize<float>(const LinArgs&, int, LongChunks, hipStream_t);
template hipError_t launch_linearize<double>(const LinArgs&, int, LongChunks, hipStream_t);

hipError_t launch_reduce_cost(const double* part, int n, DevScalars* dev, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_cost, dim3(1), dim3(1024), 0, s, part, n, dev);
  return hipGetLastError();
}

hipError_t launch_damp_points(const DampArgs& a, hipStream_t s) {
  const int n = a.np > MAX_BARRIER_GROUPS + 1 ? a.np : MAX_BARRIER_GROUPS + 1;
  hipLaunchKernelGGL(k_damp_points, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_point_q(const PointQArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_point_q<T>, dim3((unsigned)((a.no + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_point_q<float>(const PointQArgs&, hipStream_t);
template hipError_t launch_point_q<double>(const PointQArgs&, hipStream_t);

template <typename T>
hipError_t launch_schur_pairs(const SchurArgs& a, int nwg, hipStream_t s) {
  const int per = (nwg + 7) / 8;
  hipLaunchKernelGGL(k_schur_pairs<T>, dim3(8 * per), dim3(SCHUR_THREADS), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_schur_pairs<float>(const SchurArgs&, int, hipStream_t);
template hipError_t launch_schur_pairs<double>(const SchurArgs&, int, hipStream_t);

template <typename T>
hipError_t launch_camera_finish(const CamFinishArgs& a, int nc, hipStream_t s) {
  hipLaunchKernelGGL(k_camera_finish<T>, dim3(nc), dim3(64), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_camera_finish<float>(const CamFinishArgs&, int, hipStream_t);
template hipError_t launch_camera_finish<double>(const CamFinishArgs&, int, hipStream_t);

template <typename T>
hipError_t launch_backsub(const BackArgs& a, int nchunk, LongChunks lc, hipStream_t s) {
  hipLaunchKernelGGL(k_backsub<T>, dim3(nchunk), dim3(CHUNK), 0, s, a);
  if (lc.n > 0) hipLaunchKernelGGL(k_backsub_long<T>, dim3(lc.n), dim3(CHUNK), 0, s, a, lc.idx);
  return hipGetLastError();
}
template hipError_t launch_backsub<float>(const BackArgs&, int, LongChunks, hipStream_t);
template hipError_t launch_backsub<double>(const BackArgs&, int, LongChunks, hipStream_t);

hipError_t launch_retract_cameras(const RetractArgs& a, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_retract_cameras, dim3(nblk), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_candidate_cost(const CostArgs& a, int nchunk, hipStream_t s) {
  hipLaunchKernelGGL(k_candidate_cost, dim3(nchunk), dim3(CHUNK), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(FinalArgs a, hipStream_t s) {
  int g = (a.nchunk + 1023) / 1024;
  if (g < 1) g = 1;
  if (g > FINAL_STAGE_MAX) g = FINAL_STAGE_MAX;
  a.nstage = g;
  hipLaunchKernelGGL(k_final_stage, dim3(g), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_permute_rows(const PermArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_rows, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_set_observations(const ObsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_set_observations, dim3((unsigned)((a.no + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ba
