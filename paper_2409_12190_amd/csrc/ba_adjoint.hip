// gfx950 kernels of the implicit-function adjoint of bundle adjustment.
//
// The paper runs the solver inside learning pipelines whose loss depends on
// the optimum (Sec. VI-D and App. A: bilevel use).  At a stationary point
// theta* the tangent gradient sum_k w_k J_k^T r_k vanishes (squared loss,
// weights w_k); differentiating that condition gives, for a loss L(theta*),
//   H v = dL/dtheta,   dL/dx_k = w_k J_k v,   dL/dw_k = -r_k . (J_k v),
// with H = sum_k w_k (J_k^T J_k + C_k) the exact Hessian of
// delta -> F(theta* (+) delta) at 0 and C_k = sum_m r_km Hess(pixel_km)
// (curvature12).  H has the block pattern of J^T J, so the same point
// elimination, pair table and PCG apply, with the per-observation
// camera-point block W_k = w_k (Jc^T Jp + C_k,cp) of H in place of
// w Jc^T Jp.  All arithmetic and storage are FP64.
//
// Per position x (observations sorted by point):
//   A[x][78]  w (J^T J + C) packed upper over [camera 9, point 3]
//   J[x][24]  Jc (2x9) then Jp (2x3), fixed cameras' columns zero
//   Y[x][27]  W_x V_j^-1 (9x3), V_j the exact point block.
#include "ba_adjoint.h"
#include "ba_reduce.h"
#include "ba_device.h"

namespace ba {

namespace {

// max(m, |v|), with a NaN v counted as infinity
__device__ __forceinline__ double absmax_inf(double m, double v) {
  return v == v ? fmax(m, fabs(v)) : INFINITY;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

// gradient with respect to the stored camera rows -> tangent gradient, by
// the derivative of the left retraction at zero:
//   t' = t + rho + phi x t,  q' = q + 1/2 (qw phi + phi x qv, -phi . qv)
//   d/drho = g_t,  d/dphi = t x g_t + 1/2 (qw g_qv + qv x g_qv - g_qw qv),
// intrinsics unchanged; fixed cameras get zero.
__global__ __launch_bounds__(256) void k_adj_tangent(AdjTangentArgs a) {
  const int cam = blockIdx.x * blockDim.x + threadIdx.x;
  if (cam >= a.nc) return;
  const double* c = a.cams + 10 * (size_t)cam;
  const double* g = a.gL_cams + 10 * (size_t)cam;
  double* o = a.gt + 9 * (size_t)cam;
  if (a.fixed[cam] & FIXED_CAMERA) {
    for (int i = 0; i < 9; ++i) o[i] = 0.0;
    return;
  }
  const V3 t = v3(c[0], c[1], c[2]), qv = v3(c[3], c[4], c[5]);
  const double qw = c[6];
  const V3 gt = v3(g[0], g[1], g[2]), gq = v3(g[3], g[4], g[5]);
  const double gw = g[6];
  const V3 gphi = cross(t, gt) + 0.5 * (qw * gq + cross(qv, gq) - gw * qv);
  o[0] = gt.x; o[1] = gt.y; o[2] = gt.z;
  o[3] = gphi.x; o[4] = gphi.y; o[5] = gphi.z;
  o[6] = g[7]; o[7] = g[8]; o[8] = g[9];
}

// per observation: residual, Jacobian, curvature, A = w (J^T J + C)
__global__ __launch_bounds__(128) void k_adj_obs(AdjObsArgs a) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= a.no) return;
  const int cam_i = a.o_cam[x];
  const Camera cam = load_camera(a.cams + 10 * (size_t)cam_i);
  const double* P = a.pts + 3 * (size_t)a.o_pt[x];
  const V3 X = v3(P[0], P[1], P[2]);
  double Jc[2][9], Jp[2][3];
  const Proj pr = project_jac(cam, X, Jc, Jp);
  const double r0 = pr.px - a.o_xy[2 * x], r1 = pr.py - a.o_xy[2 * x + 1];
  double C[78];
  curvature12(cam, X, r0, r1, C);
  const bool fx = (a.fixed[cam_i] & FIXED_CAMERA) != 0;
  double J[2][12];
  for (int m = 0; m < 2; ++m) {
    for (int i = 0; i < 9; ++i) J[m][i] = fx ? 0.0 : Jc[m][i];
    for (int i = 0; i < 3; ++i) J[m][9 + i] = Jp[m][i];
  }
  const double w = a.o_w[x];
  double* A = a.A + 78 * (size_t)x;
  for (int i = 0; i < 12; ++i)
    for (int j = i; j < 12; ++j) {
      const double c = (fx && i < 9) ? 0.0 : C[sym12(i, j)];
      A[sym12(i, j)] = w * (J[0][i] * J[0][j] + J[1][i] * J[1][j] + c);
    }
  double* Jo = a.J + 24 * (size_t)x;
  for (int m = 0; m < 2; ++m) {
    for (int i = 0; i < 9; ++i) Jo[9 * m + i] = J[m][i];
    for (int i = 0; i < 3; ++i) Jo[18 + 3 * m + i] = J[m][9 + i];
  }
  a.r[2 * x] = r0;
  a.r[2 * x + 1] = r1;
}

// Inverse of the 3x3 point block m (upper: 00 01 02 11 12 22) by the
// adjugate into o (same layout); a block that is not positive definite
// raises ERR_POINT_BLOCK.  An unobserved point (empty block) gets zeros.
__device__ __forceinline__ void point_block_inverse(const double (&m)[6], bool observed, double (&o)[6],
                                                    int* error) {
  for (int q = 0; q < 6; ++q) o[q] = 0.0;
  if (!observed) return;
  const double c00 = m[3] * m[5] - m[4] * m[4];
  const double c01 = m[2] * m[4] - m[1] * m[5];
  const double c02 = m[1] * m[4] - m[2] * m[3];
  const double c11 = m[0] * m[5] - m[2] * m[2];
  const double c12 = m[1] * m[2] - m[0] * m[4];
  const double c22 = m[0] * m[3] - m[1] * m[1];
  const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
  if (!(det > 0.0) || !isfinite(det) || !(m[0] > 0.0)) atomicOr(error, (int)ERR_POINT_BLOCK);
  const double id = 1.0 / det;
  o[0] = c00 * id; o[1] = c01 * id; o[2] = c02 * id;
  o[3] = c11 * id; o[4] = c12 * id; o[5] = c22 * id;
}

// Y_x = W_x V_j^-1 of position x (W_x: the camera-point coupling rows of A_x).
__device__ __forceinline__ void adj_y(const AdjPointArgs& a, int x, const double (&v)[6]) {
  const double Vm[3][3] = {{v[0], v[1], v[2]}, {v[1], v[3], v[4]}, {v[2], v[4], v[5]}};
  const double* A = a.A + 78 * (size_t)x;
  double* Y = a.Y + 27 * (size_t)x;
  for (int i = 0; i < 9; ++i) {
    const double w0 = A[sym12(i, 9)], w1 = A[sym12(i, 10)], w2 = A[sym12(i, 11)];
    for (int q = 0; q < 3; ++q) Y[3 * i + q] = w0 * Vm[0][q] + w1 * Vm[1][q] + w2 * Vm[2][q];
  }
}

// per chunk of points: exact point blocks V_j (segmented sums in LDS, fixed
// order), their inverses, and Y_x = W_x V_j^-1 for every position.  Also
// clears the PCG grid-barrier counters (first workgroup).
__global__ __launch_bounds__(CHUNK) void k_adj_points(AdjPointArgs a) {
  __shared__ double vs[6][CHUNK];
  __shared__ double vi[6][CHUNK];
  const int c = blockIdx.x;
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1];
  const int t = threadIdx.x, x = x0 + t;
  if (c == 0 && t <= MAX_BARRIER_GROUPS) {
    if (t == 0) {
      a.gs->count = 0u;
      a.gs->gen = 0u;
    } else {
      a.gs->group[t - 1].count = 0u;
    }
  }
  if (x1 - x0 > CHUNK) return;  // one long track: k_adj_points_long
  const int pidx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  if (x < x1) {
    const double* A = a.A + 78 * (size_t)x;
    for (int q = 0; q < 6; ++q) vs[q][t] = A[sym12(9 + pidx[q][0], 9 + pidx[q][1])];
  }
  __syncthreads();
  const int j0 = a.chunk_pt[c], j1 = a.chunk_pt[c + 1];
  for (int jj = j0 + t; jj < j1; jj += blockDim.x) {
    const int lo = a.pt_ptr[jj] - x0, hi = a.pt_ptr[jj + 1] - x0;
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (int y = lo; y < hi; ++y)
      for (int q = 0; q < 6; ++q) m[q] += vs[q][y];
    double o[6];
    point_block_inverse(m, hi > lo, o, a.error);
    double* Vg = a.Vinv + 6 * (size_t)jj;
    for (int q = 0; q < 6; ++q) {
      Vg[q] = o[q];
      vi[q][jj - j0] = o[q];
    }
  }
  __syncthreads();
  if (x < x1) {
    const int jl = a.o_pt[x] - j0;
    const double v[6] = {vi[0][jl], vi[1][jl], vi[2][jl], vi[3][jl], vi[4][jl], vi[5][jl]};
    adj_y(a, x, v);
  }
}

// The chunks of one point seen more than CHUNK times: each thread sums the
// point block over the observations t, t + CHUNK, ...; the threads' partials
// are added in a fixed order and thread 0 inverts.
__global__ __launch_bounds__(CHUNK) void k_adj_points_long(AdjPointArgs a, const int32_t* chunks) {
  __shared__ double lds[3 * (CHUNK / 64) + 6];
  const int c = chunks[blockIdx.x];
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1], j = a.chunk_pt[c], t = threadIdx.x;
  const int pidx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  double m[6] = {0, 0, 0, 0, 0, 0};
  for (int x = x0 + t; x < x1; x += CHUNK) {
    const double* A = a.A + 78 * (size_t)x;
    for (int q = 0; q < 6; ++q) m[q] += A[sym12(9 + pidx[q][0], 9 + pidx[q][1])];
  }
  block_sum3(m[0], m[1], m[2], lds);
  block_sum3(m[3], m[4], m[5], lds);
  double* const vb = lds + 3 * (CHUNK / 64);
  if (t == 0) {
    double o[6];
    point_block_inverse(m, true, o, a.error);
    for (int q = 0; q < 6; ++q) {
      a.Vinv[6 * (size_t)j + q] = o[q];
      vb[q] = o[q];
    }
  }
  __syncthreads();
  const double v[6] = {vb[0], vb[1], vb[2], vb[3], vb[4], vb[5]};
  for (int x = x0 + t; x < x1; x += CHUNK) adj_y(a, x, v);
}

// per camera: the exact camera block U_a = sum A_cc and the right-hand side
//   b_a = gL_a - sum_x Y_x gL_p(x)
// of the reduced system; fixed cameras and cameras without observations
// (nothing depends on them) get U = I, b = 0.
__global__ __launch_bounds__(CAM_THREADS) void k_adj_camera(AdjCameraArgs a) {
  __shared__ double red[CAM_THREADS / 64][54];
  const int cam = blockIdx.x;
  const int lo = a.cam_ptr[cam], hi = a.cam_ptr[cam + 1];
  double u[45], b[9];
  for (int q = 0; q < 45; ++q) u[q] = 0.0;
  for (int q = 0; q < 9; ++q) b[q] = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int x = a.cam_obs[i];
    const double* A = a.A + 78 * (size_t)x;
    int q = 0;
    for (int r = 0; r < 9; ++r)
      for (int cc = r; cc < 9; ++cc) u[q++] += A[sym12(r, cc)];
    const double* Y = a.Y + 27 * (size_t)x;
    const double* gp = a.gL_pts + 3 * (size_t)a.o_pt[x];
    for (int r = 0; r < 9; ++r) b[r] += Y[3 * r] * gp[0] + Y[3 * r + 1] * gp[1] + Y[3 * r + 2] * gp[2];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int q = 0; q < 45; ++q) {
    const double v = wsum(u[q]);
    if (lane == 0) red[wid][q] = v;
  }
  for (int q = 0; q < 9; ++q) {
    const double v = wsum(b[q]);
    if (lane == 0) red[wid][45 + q] = v;
  }
  __syncthreads();
  const bool fx = (a.fixed[cam] & FIXED_CAMERA) != 0 || hi == lo;
  if (threadIdx.x < 45) {
    double s = 0.0;
    for (int w2 = 0; w2 < CAM_THREADS / 64; ++w2) s += red[w2][threadIdx.x];
    int r = 0, q = threadIdx.x;
    while (q >= 9 - r) {
      q -= 9 - r;
      ++r;
    }
    const int cc = r + q;
    if (fx) s = (r == cc) ? 1.0 : 0.0;
    a.U[81 * (size_t)cam + 9 * r + cc] = s;
    a.U[81 * (size_t)cam + 9 * cc + r] = s;
  } else if (threadIdx.x < 54) {
    const int r = threadIdx.x - 45;
    double s = 0.0;
    for (int w2 = 0; w2 < CAM_THREADS / 64; ++w2) s += red[w2][threadIdx.x];
    a.b[9 * (size_t)cam + r] = fx ? 0.0 : a.gt[9 * (size_t)cam + r] - s;
  }
}

// reduced camera matrix of H from the pair table (the numeric phase of the
// same cached table as the forward step):
//   S_ab = [a = b] U_a - sum_{pairs (x, y)} Y_x W_y^T,
// SCHUR_LANES lanes per chunk of pairs, lane k owning output columns
// 3k..3k+2; chunks of one block summed in slot order through LDS.
__global__ __launch_bounds__(SCHUR_THREADS) void k_adj_schur(AdjSchurArgs a) {
  __shared__ double part[SCHUR_SLOTS][81];
  const int slot = threadIdx.x / SCHUR_LANES;
  const int c0 = 3 * (threadIdx.x - SCHUR_LANES * slot);
  const size_t sbase = (size_t)blockIdx.x * SCHUR_SLOTS;
  if (slot < SCHUR_SLOTS) {
    const int e = a.slot_blk[sbase + slot];
    double acc[9][3];
    for (int r = 0; r < 9; ++r)
      for (int c = 0; c < 3; ++c) acc[r][c] = 0.0;
    if (e >= 0) {
      const int pb = a.slot_pb[sbase + slot], pe = a.slot_pe[sbase + slot];
      for (int i = pb; i < pe; ++i) {
        const int x = a.pair_x[i], y = a.pair_y[i];
        const double* Y = a.Y + 27 * (size_t)x;
        const double* Ay = a.A + 78 * (size_t)y;
        double wv[3][3];
        for (int c = 0; c < 3; ++c)
          for (int t = 0; t < 3; ++t) wv[t][c] = Ay[sym12(c0 + c, 9 + t)];
        for (int r = 0; r < 9; ++r) {
          const double y0 = Y[3 * r], y1 = Y[3 * r + 1], y2 = Y[3 * r + 2];
          for (int c = 0; c < 3; ++c) acc[r][c] += y0 * wv[0][c] + y1 * wv[1][c] + y2 * wv[2][c];
        }
      }
    }
    for (int r = 0; r < 9; ++r)
      for (int c = 0; c < 3; ++c) part[slot][r * 9 + c0 + c] = acc[r][c];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SCHUR_SLOTS * 81; t += blockDim.x) {
    const int s = t / 81, q = t - 81 * (t / 81);
    const int n = a.slot_lead[sbase + s];
    if (n == 0) continue;
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += part[s + k][q];
    const int e = a.slot_blk[sbase + s];
    const int row = a.blk_row[e];
    if (a.S_ptr[row] == e) a.Sdiag[81 * (size_t)row + q] = a.U[81 * (size_t)row + q] - v;
    else a.S[81 * (size_t)e + q] = -v;
  }
}

// e_x = Jc v_c + Jp v_p of position x and its gradients dL/dx = w e_x,
// dL/dw = -r . e_x (written in creation order).
__device__ __forceinline__ void adj_gradients(const AdjBackArgs& a, int x, double v0, double v1, double v2) {
  const double* J = a.J + 24 * (size_t)x;
  const double* v = a.vc + 9 * (size_t)a.o_cam[x];
  const double vpp[3] = {v0, v1, v2};
  double e[2];
  for (int m = 0; m < 2; ++m) {
    double s = 0.0;
    for (int i = 0; i < 9; ++i) s += J[9 * m + i] * v[i];
    for (int i = 0; i < 3; ++i) s += J[18 + 3 * m + i] * vpp[i];
    e[m] = s;
  }
  const int64_t k = a.o_orig[x];
  const double w = a.o_w[x];
  a.dLdx[2 * k] = w * e[0];
  a.dLdx[2 * k + 1] = w * e[1];
  if (a.dLdw) a.dLdw[k] = -(a.r[2 * x] * e[0] + a.r[2 * x + 1] * e[1]);
}

// back-substitution of the point part of v and the gradients:
//   v_p = V_j^-1 (gL_p - sum_x W_x^T v_c(x)),  e_x = Jc v_c + Jp v_p,
//   dL/dx = w e_x,  dL/dw = -r . e_x   (written in creation order)
__global__ __launch_bounds__(CHUNK) void k_adj_backsub(AdjBackArgs a) {
  __shared__ double tk[3][CHUNK];
  __shared__ double vp[3][CHUNK];
  const int c = blockIdx.x;
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1];
  if (x1 - x0 > CHUNK) return;  // one long track: k_adj_backsub_long
  const int t = threadIdx.x, x = x0 + t;
  if (x < x1) {
    const double* A = a.A + 78 * (size_t)x;
    const double* v = a.vc + 9 * (size_t)a.o_cam[x];
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      for (int i = 0; i < 9; ++i) s += A[sym12(i, 9 + q)] * v[i];
      tk[q][t] = s;
    }
  }
  __syncthreads();
  const int j0 = a.chunk_pt[c], j1 = a.chunk_pt[c + 1];
  for (int jj = j0 + t; jj < j1; jj += blockDim.x) {
    const double* g = a.gL_pts + 3 * (size_t)jj;
    double s0 = g[0], s1 = g[1], s2 = g[2];
    const int lo = a.pt_ptr[jj] - x0, hi = a.pt_ptr[jj + 1] - x0;
    for (int y = lo; y < hi; ++y) {
      s0 -= tk[0][y];
      s1 -= tk[1][y];
      s2 -= tk[2][y];
    }
    const double* m = a.Vinv + 6 * (size_t)jj;
    const double d0 = m[0] * s0 + m[1] * s1 + m[2] * s2;
    const double d1 = m[1] * s0 + m[3] * s1 + m[4] * s2;
    const double d2 = m[2] * s0 + m[4] * s1 + m[5] * s2;
    vp[0][jj - j0] = d0;
    vp[1][jj - j0] = d1;
    vp[2][jj - j0] = d2;
    double* o = a.vp + 3 * (size_t)jj;
    o[0] = d0;
    o[1] = d1;
    o[2] = d2;
  }
  __syncthreads();
  if (x < x1) {
    const int jl = a.o_pt[x] - j0;
    adj_gradients(a, x, vp[0][jl], vp[1][jl], vp[2][jl]);
  }
}

// The chunks of one point seen more than CHUNK times: each thread sums
// W_x^T v_c over the observations t, t + CHUNK, ...; the threads' partials
// are added in a fixed order and thread 0 forms v_p.
__global__ __launch_bounds__(CHUNK) void k_adj_backsub_long(AdjBackArgs a, const int32_t* chunks) {
  __shared__ double lds[3 * (CHUNK / 64) + 3];
  const int c = chunks[blockIdx.x];
  const int x0 = a.chunk_ptr[c], x1 = a.chunk_ptr[c + 1], j = a.chunk_pt[c], t = threadIdx.x;
  double tk[3] = {0.0, 0.0, 0.0};
  for (int x = x0 + t; x < x1; x += CHUNK) {
    const double* A = a.A + 78 * (size_t)x;
    const double* v = a.vc + 9 * (size_t)a.o_cam[x];
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      for (int i = 0; i < 9; ++i) s += A[sym12(i, 9 + q)] * v[i];
      tk[q] += s;
    }
  }
  block_sum3(tk[0], tk[1], tk[2], lds);
  double* const vb = lds + 3 * (CHUNK / 64);
  if (t == 0) {
    const double* g = a.gL_pts + 3 * (size_t)j;
    const double s0 = g[0] - tk[0], s1 = g[1] - tk[1], s2 = g[2] - tk[2];
    const double* m = a.Vinv + 6 * (size_t)j;
    const double d0 = m[0] * s0 + m[1] * s1 + m[2] * s2;
    const double d1 = m[1] * s0 + m[3] * s1 + m[4] * s2;
    const double d2 = m[2] * s0 + m[4] * s1 + m[5] * s2;
    double* o = a.vp + 3 * (size_t)j;
    o[0] = d0; o[1] = d1; o[2] = d2;
    vb[0] = d0; vb[1] = d1; vb[2] = d2;
  }
  __syncthreads();
  for (int x = x0 + t; x < x1; x += CHUNK) adj_gradients(a, x, vb[0], vb[1], vb[2]);
}

// Stationarity of theta, the premise of the adjoint: per camera and per point
// the tangent gradient g = sum_k w_k J_k^T r_k (fixed cameras' columns are
// zero in J), and the largest single term |w_k (J_k^T r_k)_i| as its scale.
// stat[0] = max |g_i|, stat[1] = max term (maxima of non-negative doubles
// through their bit patterns, which order the same way; a non-finite
// gradient component counts as infinity and fails the test on the host).
__global__ __launch_bounds__(256) void k_adj_stationarity(AdjStatArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double gmax = 0.0, tmax = 0.0;
  if (t < a.nc) {
    double g[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = a.cam_ptr[t]; q < a.cam_ptr[t + 1]; ++q) {
      const int x = a.cam_obs[q];
      const double* J = a.J + 24 * (size_t)x;
      const double w = a.o_w[x], r0 = a.r[2 * x], r1 = a.r[2 * x + 1];
      for (int i = 0; i < 9; ++i) {
        const double term = w * (J[i] * r0 + J[9 + i] * r1);
        g[i] += term;
        tmax = fmax(tmax, fabs(term));
      }
    }
    for (int i = 0; i < 9; ++i) gmax = absmax_inf(gmax, g[i]);
  } else if (t < a.nc + a.np) {
    const int j = t - a.nc;
    double g[3] = {0, 0, 0};
    for (int x = a.pt_ptr[j]; x < a.pt_ptr[j + 1]; ++x) {
      const double* J = a.J + 24 * (size_t)x;
      const double w = a.o_w[x], r0 = a.r[2 * x], r1 = a.r[2 * x + 1];
      for (int i = 0; i < 3; ++i) {
        const double term = w * (J[18 + i] * r0 + J[21 + i] * r1);
        g[i] += term;
        tmax = fmax(tmax, fabs(term));
      }
    }
    for (int i = 0; i < 3; ++i) gmax = absmax_inf(gmax, g[i]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
    tmax = fmax(tmax, __shfl_xor(tmax, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(a.stat), (unsigned long long)__double_as_longlong(gmax));
    atomicMax(reinterpret_cast<unsigned long long*>(a.stat + 1), (unsigned long long)__double_as_longlong(tmax));
  }
}

hipError_t launch_adj_stationarity(const AdjStatArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_stationarity, dim3((a.nc + a.np + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_tangent(const AdjTangentArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_tangent, dim3((a.nc + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_obs(const AdjObsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_obs, dim3((unsigned)((a.no + 127) / 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_points(const AdjPointArgs& a, int nchunk, LongChunks lc, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_points, dim3(nchunk), dim3(CHUNK), 0, s, a);
  if (lc.n > 0) hipLaunchKernelGGL(k_adj_points_long, dim3(lc.n), dim3(CHUNK), 0, s, a, lc.idx);
  return hipGetLastError();
}

hipError_t launch_adj_camera(const AdjCameraArgs& a, int nc, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_camera, dim3(nc), dim3(CAM_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_schur(const AdjSchurArgs& a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_schur, dim3(nwg), dim3(SCHUR_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_backsub(const AdjBackArgs& a, int nchunk, LongChunks lc, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_backsub, dim3(nchunk), dim3(CHUNK), 0, s, a);
  if (lc.n > 0) hipLaunchKernelGGL(k_adj_backsub_long, dim3(lc.n), dim3(CHUNK), 0, s, a, lc.idx);
  return hipGetLastError();
}

}  // namespace ba
