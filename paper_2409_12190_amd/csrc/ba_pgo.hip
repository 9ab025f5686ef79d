// Pose graph optimisation kernels for gfx950 (Sec. IV-D, Eq. 4 and 5).
//
// Edge (i, j) with measurement T_ij and information Omega_ij has the residual
// r = Log(zeta_i^-1 zeta_j T_ij^-1) in se(3) = R^6 (translation part first)
// and, for the left update zeta <- Exp(delta) zeta,
//   d r / d delta_j =  Jl^-1(r) Ad(zeta_i^-1) =: J,   d r / d delta_i = -J,
// so the edge adds A = J^T Omega J to both diagonal blocks, -A to the block
// (i, j), and +-b, b = J^T Omega r, to the gradients of j and i.  The cost is
// F = 1/2 sum r^T Omega r.  All arithmetic is FP64.
//
// Rotations are handled as unit quaternions (scalar last): the error's
// rotation is q_i^* q_j q_T^* and Log takes its angle from atan2, which stays
// accurate near 0 and pi.  Jl^-1 of SE(3) is evaluated in closed form,
//   Jl^-1 = [[P, -P Q P], [0, P]],
// P = Jl^-1 of SO(3) = I - phi^/2 + a phi^2, a = (1 - (th/2) cot(th/2)) / th^2,
// and Q(rho, phi) the coupling block of the SE(3) left Jacobian in closed
// form (Barfoot and Furgale, "Associating Uncertainty with Three-Dimensional
// Poses for Use in Estimation Problems", 2014), with series for its
// coefficients at small angles.
#include <hip/hip_runtime.h>

#include "ba_device.h"
#include "ba_pgo.h"
#include "ba_reduce.h"

namespace ba {

namespace {

struct Quat {
  V3 v;
  double w;
};

__device__ __forceinline__ Quat qmul(Quat a, Quat b) {
  return Quat{a.w * b.v + b.w * a.v + cross(a.v, b.v), a.w * b.w - dot(a.v, b.v)};
}
__device__ __forceinline__ Quat qconj(Quat a) { return Quat{v3(-a.v.x, -a.v.y, -a.v.z), a.w}; }

struct Pose {
  V3 t;
  Quat q;
};

__device__ __forceinline__ Pose load_pose(const double* __restrict__ z) {
  return Pose{v3(z[0], z[1], z[2]), Quat{v3(z[3], z[4], z[5]), z[6]}};
}

// 3x3 matrices, row-major
struct M3 {
  double m[9];
};

__device__ __forceinline__ M3 hat(V3 a) {
  return M3{{0.0, -a.z, a.y, a.z, 0.0, -a.x, -a.y, a.x, 0.0}};
}
__device__ __forceinline__ M3 mul(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return C;
}
__device__ __forceinline__ M3 rotation(Quat q) {
  // columns are the images of the unit vectors
  const V3 c0 = quat_rotate(q.v, q.w, v3(1.0, 0.0, 0.0));
  const V3 c1 = quat_rotate(q.v, q.w, v3(0.0, 1.0, 0.0));
  const V3 c2 = quat_rotate(q.v, q.w, v3(0.0, 0.0, 1.0));
  return M3{{c0.x, c1.x, c2.x, c0.y, c1.y, c2.y, c0.z, c1.z, c2.z}};
}

// E = zeta_i^-1 zeta_j T^-1 and r = Log(E); optionally phi's angle theta
__device__ __forceinline__ void pgo_residual(const Pose& zi, const Pose& zj, const Pose& T, double r[6],
                                             double* th_out) {
  const Quat qa = qmul(qconj(zi.q), zj.q);
  const V3 ta = quat_rotate_inv(zi.q.v, zi.q.w, zj.t - zi.t);
  Quat qe = qmul(qa, qconj(T.q));
  const V3 te = ta - quat_rotate(qe.v, qe.w, T.t);
  if (qe.w < 0.0) qe = Quat{v3(-qe.v.x, -qe.v.y, -qe.v.z), -qe.w};
  const double n = sqrt(dot(qe.v, qe.v));
  // phi = theta v / |v|, theta = 2 atan2(|v|, w)
  double k;
  if (n < 1e-7) {
    const double iw = 1.0 / qe.w;
    k = 2.0 * iw * (1.0 - n * n * iw * iw * (1.0 / 3.0));
  } else {
    k = 2.0 * atan2(n, qe.w) / n;
  }
  const V3 phi = k * qe.v;
  const double th = k * n;
  // rho = P t with P = I - phi^/2 + a phi^2
  double a;
  if (th < 1e-2) {
    const double t2 = th * th;
    a = 1.0 / 12.0 + t2 * (1.0 / 720.0 + t2 * (1.0 / 30240.0));
  } else {
    double sh, ch;
    sincos(0.5 * th, &sh, &ch);
    a = (1.0 - 0.5 * th * ch / sh) / (th * th);
  }
  const V3 pt = cross(phi, te);
  const V3 rho = te - 0.5 * pt + a * cross(phi, pt);
  r[0] = rho.x; r[1] = rho.y; r[2] = rho.z;
  r[3] = phi.x; r[4] = phi.y; r[5] = phi.z;
  if (th_out) *th_out = th;
}

// J = Jl^-1(r) Ad(zeta_i^-1) as its two distinct 3x3 blocks: J = [[X, Y], [0, X]]
__device__ __forceinline__ void pgo_jacobian(const double r[6], double th, const Pose& zi, M3& X, M3& Y) {
  const V3 rho = v3(r[0], r[1], r[2]), phi = v3(r[3], r[4], r[5]);
  const double t2 = th * th;
  double a, c1, c2, c3;
  if (th < 1e-2) {
    a = 1.0 / 12.0 + t2 * (1.0 / 720.0 + t2 * (1.0 / 30240.0));
    c1 = 1.0 / 6.0 - t2 * (1.0 / 120.0 - t2 * (1.0 / 5040.0));
    c2 = 1.0 / 24.0 - t2 * (1.0 / 720.0 - t2 * (1.0 / 40320.0));
    c3 = 1.0 / 120.0 - t2 * (1.0 / 2520.0 - t2 * (1.0 / 120960.0));
  } else {
    double sn, cs, sh, ch;
    sincos(th, &sn, &cs);
    sincos(0.5 * th, &sh, &ch);
    a = (1.0 - 0.5 * th * ch / sh) / t2;
    c1 = (th - sn) / (t2 * th);
    c2 = (t2 + 2.0 * cs - 2.0) / (2.0 * t2 * t2);
    c3 = (2.0 * th - 3.0 * sn + th * cs) / (2.0 * t2 * t2 * th);
  }
  const M3 Ph = hat(phi), Rh = hat(rho);
  const M3 PR = mul(Ph, Rh), RP = mul(Rh, Ph);
  const M3 PRP = mul(PR, Ph);
  const M3 PP = mul(Ph, Ph);
  const M3 PPR = mul(Ph, PR), RPP = mul(RP, Ph);
  const M3 PRPP = mul(PRP, Ph), PPRP = mul(Ph, PRP);
  M3 Q, P;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    Q.m[q] = 0.5 * Rh.m[q] + c1 * (PR.m[q] + RP.m[q] + PRP.m[q]) +
             c2 * (PPR.m[q] + RPP.m[q] - 3.0 * PRP.m[q]) + c3 * (PRPP.m[q] + PPRP.m[q]);
    P.m[q] = (q % 4 == 0 ? 1.0 : 0.0) - 0.5 * Ph.m[q] + a * PP.m[q];
  }
  const M3 Mc = mul(mul(P, Q), P);  // Jl^-1's upper right block is -Mc
  // Ad(zeta_i^-1) = [[R, t^ R], [0, R]] with R = R_i^T, t = -R_i^T t_i
  M3 R = rotation(zi.q);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i + 1; j < 3; ++j) {
      const double s = R.m[3 * i + j];
      R.m[3 * i + j] = R.m[3 * j + i];
      R.m[3 * j + i] = s;
    }
  const V3 ti = quat_rotate_inv(zi.q.v, zi.q.w, zi.t);
  const M3 K = mul(hat(v3(-ti.x, -ti.y, -ti.z)), R);
  X = mul(P, R);
  const M3 PK = mul(P, K), MR = mul(Mc, R);
#pragma unroll
  for (int q = 0; q < 9; ++q) Y.m[q] = PK.m[q] - MR.m[q];
}

__device__ __forceinline__ double jel(const M3& X, const M3& Y, int a, int k) {
  // entry (a, k) of [[X, Y], [0, X]]
  if (a < 3) return k < 3 ? X.m[3 * a + k] : Y.m[3 * a + k - 3];
  return k < 3 ? 0.0 : X.m[3 * (a - 3) + k - 3];
}

__device__ __forceinline__ double omega_el(const double* __restrict__ om, int a, int b) { return om[6 * a + b]; }

// 1/2 r^T Omega r
__device__ __forceinline__ double edge_cost(const double* __restrict__ om, const double r[6]) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) t += omega_el(om, a, b) * r[b];
    s += r[a] * t;
  }
  return 0.5 * s;
}

}  // namespace

// Copies the measurements into the workspace with validation: finite values,
// unit quaternions (|q|^2 within 1e-10 of 1), symmetric information
// matrices with a positive diagonal.
__global__ __launch_bounds__(256) void k_pgo_set_edges(PgoEdgeArgs a) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= a.m) return;
  bool finite = true, bad = false;
  const double* T = a.T + 7 * e;
  double* dT = a.pg_T + 8 * e;
  for (int q = 0; q < 7; ++q) {
    dT[q] = T[q];
    finite = finite && isfinite(T[q]);
  }
  dT[7] = 0.0;
  const double qn = T[3] * T[3] + T[4] * T[4] + T[5] * T[5] + T[6] * T[6];
  if (!(fabs(qn - 1.0) <= 1e-10)) bad = true;
  double* dO = a.pg_om + 36 * e;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      const double v = a.omega ? a.omega[36 * e + 6 * i + j] : (i == j ? 1.0 : 0.0);
      dO[6 * i + j] = v;
      finite = finite && isfinite(v);
    }
  if (a.omega)
    for (int i = 0; i < 6; ++i) {
      if (!(a.omega[36 * e + 7 * i] > 0.0)) bad = true;
      for (int j = i + 1; j < 6; ++j)
        if (a.omega[36 * e + 6 * i + j] != a.omega[36 * e + 6 * j + i]) bad = true;
    }
  if (!finite) atomicOr(&a.dev->error, (int)ERR_NONFINITE_OBS);
  else if (bad) atomicOr(&a.dev->error, (int)ERR_BAD_WEIGHT);
}

// One thread per edge: r, J, the edge record (A, b) and the cost partials of
// its chunk of PGO_CHUNK edges.
__global__ __launch_bounds__(PGO_CHUNK) void k_pgo_linearize(PgoLinArgs a) {
  __shared__ double red[PGO_CHUNK / 64];
  const int64_t e = blockIdx.x * (int64_t)PGO_CHUNK + threadIdx.x;
  double cost = 0.0;
  if (e < a.m) {
    const Pose zi = load_pose(a.cams + 10 * (size_t)a.ei[e]);
    const Pose zj = load_pose(a.cams + 10 * (size_t)a.ej[e]);
    const Pose T = load_pose(a.T + 8 * e);
    const double* om = a.om + 36 * e;
    double r[6], th;
    pgo_residual(zi, zj, T, r, &th);
    M3 X, Y;
    pgo_jacobian(r, th, zi, X, Y);
    double orr[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b) t += omega_el(om, i, b) * r[b];
      orr[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) cost += r[i] * orr[i];
    cost *= 0.5;
    double* rec = a.rec + PGO_REC * e;
    // W = Omega J column by column, A = J^T W (upper triangle, mirrored)
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      double w[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < 6; ++b) t += omega_el(om, i, b) * jel(X, Y, b, l);
        w[i] = t;
      }
#pragma unroll
      for (int k = 0; k <= l; ++k) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) t += jel(X, Y, i, k) * w[i];
        rec[6 * k + l] = t;
        rec[6 * l + k] = t;
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) t += jel(X, Y, i, k) * orr[i];
      rec[36 + k] = t;
    }
  }
  const double s = block_sum(cost, red);
  if (threadIdx.x == 0) {
    a.part_cost[blockIdx.x] = s;
    a.part_gmax[blockIdx.x] = 0.0;  // the gradient maximum comes from gc
  }
}

// One workgroup per stored upper block: the block from its edges' records
// (fixed poses contribute nothing), written to Sdiag (diagonal, FP64, with
// the row's gradient, diag and a zero right-hand side) or to S (and its
// streamed copy) in the storage precision.  Rows and columns 6-8 of every
// 9x9 block are zero: a pose has no intrinsics.
template <typename T>
__global__ __launch_bounds__(PGO_ASM_THREADS) void k_pgo_assemble(PgoAsmArgs a) {
  const int64_t k = blockIdx.x;
  const int q = threadIdx.x;
  const int row = a.blk_row[k], col = a.S_col[k];
  const bool diag = row == col;
  const bool dead = (a.fixed[row] & FIXED_CAMERA) || (a.fixed[col] & FIXED_CAMERA);
  const int p0 = a.ptr[k], p1 = a.ptr[k + 1];
  if (q < 81) {
    const int i = q / 9, j = q - 9 * (q / 9);
    double v = 0.0;
    if (!dead && i < 6 && j < 6)
      for (int p = p0; p < p1; ++p) v += a.rec[PGO_REC * (size_t)(a.code[p] >> 1) + 6 * i + j];
    if (diag) {
      a.Sdiag[81 * (size_t)row + q] = v;
      if (i == j) a.diagU[9 * (size_t)row + i] = v;
    } else {
      v = -v;
      reinterpret_cast<T*>(a.S)[81 * (size_t)k + q] = (T)v;
      if (a.SI) {
        T* si = reinterpret_cast<T*>(a.SI) + (size_t)a.blk_pos[k] * SI_STRIDE;
        si[q] = (T)v;
        if (q < SI_STRIDE - 81) si[81 + q] = (T)0;
      }
    }
  } else if (diag && q < 90) {
    const int i = q - 81;
    double g = 0.0;
    if (!dead && i < 6)
      for (int p = p0; p < p1; ++p) {
        const int c = a.code[p];
        const double b = a.rec[PGO_REC * (size_t)(c >> 1) + 36 + i];
        g += (c & 1) ? -b : b;
      }
    a.gc[9 * (size_t)row + i] = g;
    a.bS[9 * (size_t)row + i] = 0.0;  // -gc, added by the camera finish
  }
}

// One thread per edge: the cost at the candidate poses and the model term
// (dx_j - dx_i)^T A (dx_j - dx_i) = |J_i dx_i + J_j dx_j|^2_Omega.
__global__ __launch_bounds__(PGO_CHUNK) void k_pgo_candidate(PgoCandArgs a) {
  __shared__ double red[PGO_CHUNK / 64];
  const int64_t e = blockIdx.x * (int64_t)PGO_CHUNK + threadIdx.x;
  double cost = 0.0, quad = 0.0;
  if (e < a.m) {
    const int32_t i = a.ei[e], j = a.ej[e];
    const Pose zi = load_pose(a.cams_new + 10 * (size_t)i);
    const Pose zj = load_pose(a.cams_new + 10 * (size_t)j);
    const Pose T = load_pose(a.T + 8 * e);
    double r[6];
    pgo_residual(zi, zj, T, r, nullptr);
    cost = edge_cost(a.om + 36 * e, r);
    double d[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) d[k] = a.dx[9 * (size_t)j + k] - a.dx[9 * (size_t)i + k];
    const double* A = a.rec + PGO_REC * e;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < 6; ++l) t += A[6 * k + l] * d[l];
      quad += d[k] * t;
    }
  }
  const double c = block_sum(cost, red);
  const double qd = block_sum(quad, red);
  if (threadIdx.x == 0) {
    a.part_cost_new[blockIdx.x] = c;
    a.part_pred[2 * (size_t)blockIdx.x] = qd;
    a.part_pred[2 * (size_t)blockIdx.x + 1] = 0.0;  // no point term
  }
}

hipError_t launch_pgo_set_edges(const PgoEdgeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pgo_set_edges, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pgo_linearize(const PgoLinArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pgo_linearize, dim3(pgo_chunks(a.m)), dim3(PGO_CHUNK), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pgo_assemble(const PgoAsmArgs& a, int64_t nnzb, hipStream_t s) {
  hipLaunchKernelGGL(k_pgo_assemble<T>, dim3((unsigned)nnzb), dim3(PGO_ASM_THREADS), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_pgo_assemble<float>(const PgoAsmArgs&, int64_t, hipStream_t);
template hipError_t launch_pgo_assemble<double>(const PgoAsmArgs&, int64_t, hipStream_t);

hipError_t launch_pgo_candidate(const PgoCandArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pgo_candidate, dim3(pgo_chunks(a.m)), dim3(PGO_CHUNK), 0, s, a);
  return hipGetLastError();
}

}  // namespace ba
