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
    for (int m = 0; m < 3; ++m) Jp[i][m] = (double)J[18 + i * 3 + m];
  }
}

__device__ __forceinline__ void load_sym3(const double* __restrict__ s, double M[3][3]) {
  M[0][0] = s[0]; M[0][1] = s[1]; M[0][2] = s[2];
  M[1][0] = s[1]; M[1][1] = s[3]; M[1][2] = s[4];
  M[2][0] = s[2]; M[2][1] = s[4]; M[2][2] = s[5];
}

// ---------------------------------------------------------------------------
// observation pass 1: residual, Jacobian blocks, robust weight, cost, and the
// point-keyed blocks V_j = sum w Jp^T Jp, gp_j = sum w Jp^T r
// (Alg. 1 first two lines; Sec. IV-A-2 batched Jacobian values).
// One workgroup per point-aligned chunk; segmented sums in LDS, fixed order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(CHUNK) void k_linearize(LinArgs a) {
  __shared__ double sh[9][CHUNK];
  __shared__ double red[CHUNK / 64];
  const int c = blockIdx.x;
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1];
  const int t = threadIdx.x;
  const int x = x0 + t;
  double cost = 0.0;
  if (x < x1) {
    const int ci = a.o_cam[x], pj = a.o_pt[x];
    const Camera cam = load_camera(a.cams + 10 * (size_t)ci);
    const double* P = a.pts + 3 * (size_t)pj;
    double Jc[2][9], Jp[2][3];
    const Proj pr = project_jac(cam, v3(P[0], P[1], P[2]), Jc, Jp);
    const double rx = pr.px - a.o_xy[2 * (size_t)x], ry = pr.py - a.o_xy[2 * (size_t)x + 1];
    double drho;
    const double rho = robust_rho(rx * rx + ry * ry, a.huber, &drho);
    const double om = a.o_w[x];
    const double w = om * drho;
    cost = 0.5 * om * rho;
    if (a.fixed[ci]) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int m = 0; m < 9; ++m) Jc[i][m] = 0.0;
    }
    a.r[2 * (size_t)x] = rx;
    a.r[2 * (size_t)x + 1] = ry;
    a.w[x] = w;
    T* J = reinterpret_cast<T*>(a.J) + (size_t)x * NJ;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int m = 0; m < 9; ++m) J[i * 9 + m] = (T)Jc[i][m];
#pragma unroll
      for (int m = 0; m < 3; ++m) J[18 + i * 3 + m] = (T)Jp[i][m];
    }
    sh[0][t] = w * (Jp[0][0] * Jp[0][0] + Jp[1][0] * Jp[1][0]);
    sh[1][t] = w * (Jp[0][0] * Jp[0][1] + Jp[1][0] * Jp[1][1]);
    sh[2][t] = w * (Jp[0][0] * Jp[0][2] + Jp[1][0] * Jp[1][2]);
    sh[3][t] = w * (Jp[0][1] * Jp[0][1] + Jp[1][1] * Jp[1][1]);
    sh[4][t] = w * (Jp[0][1] * Jp[0][2] + Jp[1][1] * Jp[1][2]);
    sh[5][t] = w * (Jp[0][2] * Jp[0][2] + Jp[1][2] * Jp[1][2]);
    sh[6][t] = w * (Jp[0][0] * rx + Jp[1][0] * ry);
    sh[7][t] = w * (Jp[0][1] * rx + Jp[1][1] * ry);
    sh[8][t] = w * (Jp[0][2] * rx + Jp[1][2] * ry);
  }
  __syncthreads();
  double gmax = 0.0;
  const int j0 = a.chunk_pt[c], j1 = a.chunk_pt[c + 1];
  for (int j = j0 + t; j < j1; j += blockDim.x) {
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
    gmax = fmax(gmax, fmax(fabs(s[6]), fmax(fabs(s[7]), fabs(s[8]))));
  }
  const double tot = block_sum(cost, red);
  const double gm = block_max(gmax, red);
  if (t == 0) {
    a.part_cost[c] = tot;
    a.part_gmax[c] = gm;
  }
}

// F = sum of the chunk partials (fixed order), and the gradient max over points.
__global__ __launch_bounds__(256) void k_reduce_cost(const double* __restrict__ part, int n,
                                                     DevScalars* dev) {
  __shared__ double red[4];
  const double F = block_sum_array(part, n, red);
  if (threadIdx.x == 0) dev->F = F;
}

// ---------------------------------------------------------------------------
// damping of the point blocks and their inverses (Eq. 2 with the clamp of
// Sec. IV-B-3): V*_j = V_j + lambda clamp(diag V_j), Vinv_j = V*_j^-1 by the
// adjugate, ep_j = Vinv_j gp_j.  One thread per point, FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_damp_points(DampArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j <= MAX_BARRIER_GROUPS) {  // the PCG grid barrier of this step starts from a clean state
    if (j == 0) {
      a.gs->count = 0u;
      a.gs->gen = 0u;
    } else {
      a.gs->group[j - 1].count = 0u;
    }
  }
  if (j >= a.np) return;
  const double lam = a.dev->lambda;
  const double* v = a.V + 6 * (size_t)j;
  const double m00 = v[0] + lam * fmin(fmax(v[0], a.dmin), a.dmax);
  const double m11 = v[3] + lam * fmin(fmax(v[3], a.dmin), a.dmax);
  const double m22 = v[5] + lam * fmin(fmax(v[5], a.dmin), a.dmax);
  const double m01 = v[1], m02 = v[2], m12 = v[4];
  const double c00 = m11 * m22 - m12 * m12;
  const double c01 = m02 * m12 - m01 * m22;
  const double c02 = m01 * m12 - m02 * m11;
  const double c11 = m00 * m22 - m02 * m02;
  const double c12 = m01 * m02 - m00 * m12;
  const double c22 = m00 * m11 - m01 * m01;
  const double det = m00 * c00 + m01 * c01 + m02 * c02;
  if (!(det > 0.0) || !isfinite(det)) atomicOr(&a.dev->error, (int)ERR_POINT_BLOCK);
  const double id = 1.0 / det;
  double* o = a.Vinv + 6 * (size_t)j;
  o[0] = c00 * id; o[1] = c01 * id; o[2] = c02 * id;
  o[3] = c11 * id; o[4] = c12 * id; o[5] = c22 * id;
  const double* g = a.gp + 3 * (size_t)j;
  double* e = a.ep + 3 * (size_t)j;
  e[0] = (c00 * g[0] + c01 * g[1] + c02 * g[2]) * id;
  e[1] = (c01 * g[0] + c11 * g[1] + c12 * g[2]) * id;
  e[2] = (c02 * g[0] + c12 * g[1] + c22 * g[2]) * id;
}

// ---------------------------------------------------------------------------
// per-observation factor of the Schur product: Q_x = w_x Jp_x Vinv_j (2x3),
// stored in the Jacobian precision (one thread per observation).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_point_q(PointQArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.no) return;
  const T* J = reinterpret_cast<const T*>(a.J) + (size_t)x * NJ + 18;
  double Vi[3][3];
  load_sym3(a.Vinv + 6 * (size_t)a.o_pt[x], Vi);
  const double w = a.w[x];
  T* Q = reinterpret_cast<T*>(a.Q) + (size_t)x * 6;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double j0 = (double)J[3 * i], j1 = (double)J[3 * i + 1], j2 = (double)J[3 * i + 2];
#pragma unroll
    for (int m = 0; m < 3; ++m) Q[3 * i + m] = (T)(w * (j0 * Vi[0][m] + j1 * Vi[1][m] + j2 * Vi[2][m]));
  }
}

// ---------------------------------------------------------------------------
// Schur blocks from the pair table (Sec. IV-B-1 numeric phase on the cached
// table): for block (a, b) and pairs (x, y) sharing a point, x in camera a,
// y in camera b,
//   S_ab  = -sum Jc_x^T (Q_x (w_y Jp_y)^T) Jc_y                  (a < b)
//   S_aa' = sum Jc_x^T ([x = y] w_x I - Q_x (w_y Jp_y)^T) Jc_y   (undamped)
// Each workgroup holds SCHUR_SLOTS chunk slots; SCHUR_LANES = 3 lanes share a
// chunk, lane k accumulating columns 3k..3k+2 of the block (27 values) over
// the chunk's pairs in registers, with the next pair's rows loaded while the
// current one is multiplied.  The chunks of one block sit in consecutive
// slots of one workgroup and are summed in slot order through LDS: no
// atomics, fixed summation order.  Off-diagonal blocks go to S (precision T);
// diagonal blocks, still to be damped, to the FP64 buffer Sdiag.  The self
// pairs (x, x) of a diagonal block visit every observation of its camera
// once, so the same lanes also form the camera vectors
//   gc_a = sum w Jc^T r,  diagU_a = diag(sum w Jc^T Jc),
//   bS_a + gc_a = sum w Jc^T Jp ep_j   (ep_j = Vinv_j gp_j),
// which saves a pass over the observations in camera order.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// the values of pair (x, y) one lane needs (columns c0..c0+2)
template <typename T> struct PairRows {
  T jx[18];  // Jc of x (both rows)
  T jy[6];   // Jc of y: row 0 then row 1 at columns c0..c0+2
  T py[6];   // Jp of y
  T q[6];    // Q of x
  double w;  // weight of y
};

__device__ __forceinline__ void load_rows(PairRows<float>& v, const float* J, const float* Q,
                                          const double* w, int x, int y, int c0) {
  const float* jx = J + (size_t)x * NJ;  // 96-byte rows: 16-byte aligned
  const float* jy = J + (size_t)y * NJ;
  const float* qx = Q + (size_t)x * 6;   // 24-byte rows: 8-byte aligned
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const f32x4 t = *reinterpret_cast<const f32x4*>(jx + 4 * k);
    v.jx[4 * k] = t.x;
    v.jx[4 * k + 1] = t.y;
    v.jx[4 * k + 2] = t.z;
    v.jx[4 * k + 3] = t.w;
  }
  {
    const f32x2 t = *reinterpret_cast<const f32x2*>(jx + 16);
    v.jx[16] = t.x;
    v.jx[17] = t.y;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const f32x2 t = *reinterpret_cast<const f32x2*>(jy + 18 + 2 * k);
    v.py[2 * k] = t.x;
    v.py[2 * k + 1] = t.y;
    const f32x2 u = *reinterpret_cast<const f32x2*>(qx + 2 * k);
    v.q[2 * k] = u.x;
    v.q[2 * k + 1] = u.y;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v.jy[k] = jy[c0 + k];
    v.jy[3 + k] = jy[9 + c0 + k];
  }
  v.w = w[y];
}

__device__ __forceinline__ void load_rows(PairRows<double>& v, const double* J, const double* Q,
                                          const double* w, int x, int y, int c0) {
  const double* jx = J + (size_t)x * NJ;  // 192-byte rows
  const double* jy = J + (size_t)y * NJ;
  const double* qx = Q + (size_t)x * 6;   // 48-byte rows
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const f64x2 t = *reinterpret_cast<const f64x2*>(jx + 2 * k);
    v.jx[2 * k] = t.x;
    v.jx[2 * k + 1] = t.y;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const f64x2 t = *reinterpret_cast<const f64x2*>(jy + 18 + 2 * k);
    v.py[2 * k] = t.x;
    v.py[2 * k + 1] = t.y;
    const f64x2 u = *reinterpret_cast<const f64x2*>(qx + 2 * k);
    v.q[2 * k] = u.x;
    v.q[2 * k + 1] = u.y;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v.jy[k] = jy[c0 + k];
    v.jy[3 + k] = jy[9 + c0 + k];
  }
  v.w = w[y];
}

// acc[r][c] += (Jc_x^T M Jc_y)[r][c0 + c],
// M = [x = y] w_y I - w_y Q_x Jp_y^T
template <typename T>
__device__ __forceinline__ void pair_update(double (&acc)[9][3], const PairRows<T>& v, bool self) {
  double M[2][2];
#pragma unroll
  for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2)
      M[i2][k2] = -v.w * ((double)v.q[3 * i2] * (double)v.py[3 * k2] +
                          (double)v.q[3 * i2 + 1] * (double)v.py[3 * k2 + 1] +
                          (double)v.q[3 * i2 + 2] * (double)v.py[3 * k2 + 2]);
  if (self) {
    M[0][0] += v.w;
    M[1][1] += v.w;
  }
  double g0[3], g1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double a0 = (double)v.jy[c], a1 = (double)v.jy[3 + c];
    g0[c] = M[0][0] * a0 + M[0][1] * a1;
    g1[c] = M[1][0] * a0 + M[1][1] * a1;
  }
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const double j0 = (double)v.jx[r], j1 = (double)v.jx[9 + r];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] += j0 * g0[c] + j1 * g1[c];
  }
}

template <typename T>
__global__ __launch_bounds__(SCHUR_THREADS) void k_schur_pairs(SchurArgs a) {
  // per slot: the 81 block values; afterwards (diagonal blocks) the camera
  // vectors gc, sum w Jc^T Jp ep and diag U of the slot's self pairs
  __shared__ double part[SCHUR_SLOTS][81];
  // workgroups are dispatched round-robin over the 8 XCDs: XCD k takes the
  // k-th contiguous range of slot workgroups, so that neighbouring rows (which
  // read the same observations) share that XCD's L2
  const int per = (a.nwg + 7) / 8;
  const int lw = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (lw >= a.nwg) return;
  const int slot = threadIdx.x / SCHUR_LANES;
  const int c0 = 3 * (threadIdx.x - SCHUR_LANES * slot);
  const size_t sbase = (size_t)lw * SCHUR_SLOTS;
  const T* __restrict__ Jall = reinterpret_cast<const T*>(a.J);
  const T* __restrict__ Qall = reinterpret_cast<const T*>(a.Q);
  double vg[3] = {0.0, 0.0, 0.0}, vb[3] = {0.0, 0.0, 0.0}, vu[3] = {0.0, 0.0, 0.0};
  bool diag_slot = false;
  if (slot < SCHUR_SLOTS) {
    const int e = a.slot_blk[sbase + slot];
    double acc[9][3];
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[r][c] = 0.0;
    const int pb = e >= 0 ? a.slot_pb[sbase + slot] : 0;
    const int pe = e >= 0 ? a.slot_pe[sbase + slot] : 0;
    // (a camera without observations has an empty diagonal block: zeros)
    diag_slot = e >= 0 && a.S_ptr[a.blk_row[e]] == e;
    if (pb < pe) {
      // software pipeline: rows of pair i + 1 and indices of pair i + 2 are
      // in flight while pair i is multiplied (indices clamped to the chunk)
      int x = a.pair_x[pb], y = a.pair_y[pb];
      PairRows<T> cur;
      load_rows(cur, Jall, Qall, a.w, x, y, c0);
      int xn = a.pair_x[min(pb + 1, pe - 1)], yn = a.pair_y[min(pb + 1, pe - 1)];
#pragma unroll 2
      for (int i = pb; i < pe; ++i) {
        PairRows<T> nxt;
        load_rows(nxt, Jall, Qall, a.w, xn, yn, c0);
        const int i2 = min(i + 2, pe - 1);
        const int xa = a.pair_x[i2], ya = a.pair_y[i2];
        pair_update(acc, cur, x == y);
        cur = nxt;
        x = xn;
        y = yn;
        xn = xa;
        yn = ya;
      }
      if (diag_slot) {
        // each observation of the camera is the self pair of exactly one
        // chunk of the diagonal block: the camera vectors of Alg. 1
        // (gradient J^T W r, the Schur right-hand side term, diag of U)
        for (int i = pb; i < pe; ++i) {
          const int xs = a.pair_x[i];
          if (a.pair_y[i] != xs) continue;
          const T* Jx = Jall + (size_t)xs * NJ;
          const double wx = a.w[xs];
          const double* ep = a.ep + 3 * (size_t)a.o_pt[xs];
          const double e0 = (double)Jx[18] * ep[0] + (double)Jx[19] * ep[1] + (double)Jx[20] * ep[2];
          const double e1 = (double)Jx[21] * ep[0] + (double)Jx[22] * ep[1] + (double)Jx[23] * ep[2];
          const double r0 = a.r[2 * (size_t)xs], r1 = a.r[2 * (size_t)xs + 1];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double j0 = (double)Jx[c0 + c], j1 = (double)Jx[9 + c0 + c];
            vg[c] += wx * (j0 * r0 + j1 * r1);
            vb[c] += wx * (j0 * e0 + j1 * e1);
            vu[c] += wx * (j0 * j0 + j1 * j1);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) part[slot][r * 9 + c0 + c] = acc[r][c];
  }
  __syncthreads();
  // every lead slot sums its block's chunk partials in slot order
  for (int t = threadIdx.x; t < SCHUR_SLOTS * 81; t += blockDim.x) {
    const int s = t / 81, q = t - 81 * (t / 81);
    const int n = a.slot_lead[sbase + s];
    if (n == 0) continue;
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += part[s + k][q];
    const int e = a.slot_blk[sbase + s];
    const int row = a.blk_row[e];
    if (a.S_ptr[row] == e) a.Sdiag[81 * (size_t)row + q] = v;
    else reinterpret_cast<T*>(a.S)[81 * (size_t)e + q] = (T)v;
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
    const int s = t / 27, q = t - 27 * (t / 27);
    const int n = a.slot_lead[sbase + s];
    if (n == 0) continue;
    const int e = a.slot_blk[sbase + s];
    const int row = a.blk_row[e];
    if (a.S_ptr[row] != e) continue;
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += part[s + k][q];
    if (q < 9) a.gc[9 * (size_t)row + q] = v;
    else if (q < 18) a.bS[9 * (size_t)row + (q - 9)] = v;  // - gc, added by the camera finish
    else a.diagU[9 * (size_t)row + (q - 18)] = v;
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
      for (int cc = 0; cc < 9; ++cc) {
        double s = 0.0;
        for (int k = (r > cc ? r : cc); k < 9; ++k) s += Li[k * 9 + r] * Li[k * 9 + cc];
        Mi[r * 9 + cc] = s;
      }
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
    if (a.fixed[cam]) {
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
  const int x = a.chunk_ptr[c] + threadIdx.x;
  double cost = 0.0;
  if (x < a.chunk_ptr[c + 1]) {
    const Camera cam = load_camera(a.cams + 10 * (size_t)a.o_cam[x]);
    const double* P = a.pts + 3 * (size_t)a.o_pt[x];
    const Proj pr = project(cam, v3(P[0], P[1], P[2]));
    const double rx = pr.px - a.o_xy[2 * (size_t)x], ry = pr.py - a.o_xy[2 * (size_t)x + 1];
    double drho;
    const double rho = robust_rho(rx * rx + ry * ry, a.huber, &drho);
    cost = 0.5 * a.o_w[x] * rho;
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
hipError_t launch_linearize(const LinArgs& a, int nchunk, hipStream_t s) {
  hipLaunchKernelGGL(k_linearize<T>, dim3(nchunk), dim3(CHUNK), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_linearize<float>(const LinArgs&, int, hipStream_t);
template hipError_t launch_linearize<double>(const LinArgs&, int, hipStream_t);

hipError_t launch_reduce_cost(const double* part, int n, DevScalars* dev, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_cost, dim3(1), dim3(256), 0, s, part, n, dev);
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
hipError_t launch_backsub(const BackArgs& a, int nchunk, hipStream_t s) {
  hipLaunchKernelGGL(k_backsub<T>, dim3(nchunk), dim3(CHUNK), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_backsub<float>(const BackArgs&, int, hipStream_t);
template hipError_t launch_backsub<double>(const BackArgs&, int, hipStream_t);

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

hipError_t launch_set_observations(const ObsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_set_observations, dim3((unsigned)((a.no + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ba
