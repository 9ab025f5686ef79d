// Device-side arithmetic of one bundle-adjustment observation for gfx950.
//
// Camera row (10 doubles): [tx ty tz qx qy qz qw f k1 k2]; the pose maps world
// to camera (Y = R(q) X + t) and the pixel of a point in front (Y_z < 0) is
// f D(s) (u, v) with (u, v) = (-Y_x/Y_z, -Y_y/Y_z), s = u^2 + v^2 and
// D = 1 + k1 s + k2 s^2: the radially distorted pinhole of the paper's BAL
// benchmark, used as the projection of Eq. 1.
//
// Tangent of a camera (9): (rho, phi) of a left SE(3) update T <- Exp(rho, phi) T
// (Sec. III-C: the pose gradient space has 6 degrees of freedom), then
// additive f, k1, k2.  All arithmetic here is FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace ba {

struct V3 {
  double x, y, z;
};

__device__ __forceinline__ V3 v3(double x, double y, double z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Rotate v by the unit quaternion (qv, qw): v + 2 qw (qv x v) + 2 qv x (qv x v).
__device__ __forceinline__ V3 quat_rotate(V3 qv, double qw, V3 v) {
  const V3 c = cross(qv, v);
  return v + (2.0 * qw) * c + 2.0 * cross(qv, c);
}
// Rotate by the inverse (conjugate) quaternion.
__device__ __forceinline__ V3 quat_rotate_inv(V3 qv, double qw, V3 v) {
  const V3 c = cross(qv, v);
  return v - (2.0 * qw) * c + 2.0 * cross(qv, c);
}

struct Camera {
  V3 t, qv;
  double qw, f, k1, k2;
};

__device__ __forceinline__ Camera load_camera(const double* __restrict__ c) {
  Camera k;
  k.t = v3(c[0], c[1], c[2]);
  k.qv = v3(c[3], c[4], c[5]);
  k.qw = c[6];
  k.f = c[7];
  k.k1 = c[8];
  k.k2 = c[9];
  return k;
}

// Result of projecting one observation.
struct Proj {
  double px, py;  // pixel
  double Yz;      // depth coordinate (negative in front)
};

// Pixel of the camera-frame point Y (shared by the cost-only and the
// Jacobian paths so that both round identically).
__device__ __forceinline__ Proj pixel_of(const Camera& c, V3 Y, double* u_out, double* v_out,
                                         double* s_out, double* D_out, double* iz_out) {
  const double iz = 1.0 / Y.z;
  const double u = -Y.x * iz, v = -Y.y * iz;
  const double s = u * u + v * v;
  const double D = 1.0 + s * (c.k1 + c.k2 * s);
  *u_out = u;
  *v_out = v;
  *s_out = s;
  *D_out = D;
  *iz_out = iz;
  return Proj{c.f * D * u, c.f * D * v, Y.z};
}

__device__ __forceinline__ Proj project(const Camera& c, V3 X) {
  const V3 Y = quat_rotate(c.qv, c.qw, X) + c.t;
  double u, v, s, D, iz;
  return pixel_of(c, Y, &u, &v, &s, &D, &iz);
}

// Pixel plus its Jacobian rows.  Jc[i][0..8] is d pixel_i / d camera tangent,
// Jp[i][0..2] is d pixel_i / d point.
//
// With a = d pixel_i / dY (row i of (d pixel / d(u,v)) (d(u,v) / dY)):
//   translation part  a,
//   rotation part     d/dphi of a.(Exp(phi) Y) = a.(-[Y]x) = Y x a,
//   point part        a R = R^T a (rotate a by the inverse quaternion),
//   intrinsics        D (u,v), f s (u,v), f s^2 (u,v).
__device__ __forceinline__ Proj project_jac(const Camera& c, V3 X, double Jc[2][9], double Jp[2][3]) {
  const V3 Y = quat_rotate(c.qv, c.qw, X) + c.t;
  double u, v, s, D, iz;
  const Proj pr = pixel_of(c, Y, &u, &v, &s, &D, &iz);
  const double g = 2.0 * (c.k1 + 2.0 * c.k2 * s);  // 2 dD/ds
  // d pixel / d(u, v) = f (D I + g (u,v)(u,v)^T)
  const double A00 = c.f * (D + g * u * u), A01 = c.f * g * u * v, A11 = c.f * (D + g * v * v);
  // d(u, v)/dY: du/dYx = -1/Yz, du/dYz = Yx/Yz^2 = -u/Yz; likewise for v
  const double m = -iz;
  const V3 du = v3(m, 0.0, m * u);
  const V3 dv = v3(0.0, m, m * v);
  const V3 a0 = A00 * du + A01 * dv;
  const V3 a1 = A01 * du + A11 * dv;
  const V3 r0 = cross(Y, a0), r1 = cross(Y, a1);
  const V3 p0 = quat_rotate_inv(c.qv, c.qw, a0), p1 = quat_rotate_inv(c.qv, c.qw, a1);
  Jc[0][0] = a0.x; Jc[0][1] = a0.y; Jc[0][2] = a0.z;
  Jc[1][0] = a1.x; Jc[1][1] = a1.y; Jc[1][2] = a1.z;
  Jc[0][3] = r0.x; Jc[0][4] = r0.y; Jc[0][5] = r0.z;
  Jc[1][3] = r1.x; Jc[1][4] = r1.y; Jc[1][5] = r1.z;
  Jc[0][6] = D * u;        Jc[1][6] = D * v;
  Jc[0][7] = c.f * s * u;  Jc[1][7] = c.f * s * v;
  Jc[0][8] = c.f * s * s * u;  Jc[1][8] = c.f * s * s * v;
  Jp[0][0] = p0.x; Jp[0][1] = p0.y; Jp[0][2] = p0.z;
  Jp[1][0] = p1.x; Jp[1][1] = p1.y; Jp[1][2] = p1.z;
  return pr;
}

// Index of (i, j), i <= j, in the packed upper triangle of a 12 x 12 matrix.
__device__ __forceinline__ int sym12(int i, int j) { return i * 12 - (i * (i - 1)) / 2 + (j - i); }

// Curvature of one observation's pixel contracted with its residual r:
//   C = sum_m r_m Hess(pixel_m)
// over the 12-dimensional tangent z = [rho(3), phi(3), f, k1, k2, dX(3)] at
// z = 0, written packed upper (78 values).  To second order the camera-frame
// point is
//   Y = Y0 + R dX + rho + phi x Y0 + phi x (R dX) + 1/2 phi x (phi x Y0)
//       + 1/2 phi x rho
// (the SE(3) exponential acting on the moved point), and the pixel is
// q(Y, f, k1, k2) = f D(s) u with u = -(Y_x, Y_y)/Y_z.  With g = r . dq/dY,
// H_Y = r . d2q/dY2, H_Yk = r . d2q/dY dk and H_kk = r . d2q/dk2:
//   C = JY^T H_Y JY + sum_i g_i Hess(Y_i) + JY^T H_Yk + H_Yk^T JY + H_kk,
// JY = dY/dz = [I | -[Y0]x | 0 | R], and the second derivatives of Y are
//   phi-phi: 1/2 (g Y0^T + Y0 g^T) - (g . Y0) I,
//   phi-rho: -1/2 [g]x,   phi-dX: -[g]x R.
__device__ inline void curvature12(const Camera& c, V3 X, double r0, double r1, double* __restrict__ C) {
  const V3 Y = quat_rotate(c.qv, c.qw, X) + c.t;
  const double iz = 1.0 / Y.z;
  const double u[2] = {-Y.x * iz, -Y.y * iz};
  const double rr[2] = {r0, r1};
  const double s = u[0] * u[0] + u[1] * u[1];
  const double D = 1.0 + s * (c.k1 + c.k2 * s);
  const double D1 = c.k1 + 2.0 * c.k2 * s;  // dD/ds
  const double D2 = 2.0 * c.k2;              // d2D/ds2
  const double ru = r0 * u[0] + r1 * u[1];
  // derivatives of r . q with respect to u (2) and u-u (2 x 2)
  double gu[2], Hu[2][2];
  for (int n = 0; n < 2; ++n) {
    gu[n] = c.f * (D * rr[n] + 2.0 * D1 * ru * u[n]);
    for (int o = 0; o < 2; ++o)
      Hu[n][o] = c.f * (2.0 * D1 * (u[o] * rr[n] + u[n] * rr[o] + (n == o ? ru : 0.0)) +
                        4.0 * D2 * ru * u[n] * u[o]);
  }
  // du_n/dY = -iz (e_n + u_n e_z)
  double B[2][3] = {{-iz, 0.0, -iz * u[0]}, {0.0, -iz, -iz * u[1]}};
  double gY[3], HY[3][3];
  for (int j = 0; j < 3; ++j) gY[j] = gu[0] * B[0][j] + gu[1] * B[1][j];
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) {
      double h = 0.0;
      for (int n = 0; n < 2; ++n)
        for (int o = 0; o < 2; ++o) h += Hu[n][o] * B[n][j] * B[o][k];
      HY[j][k] = h;
    }
  // + sum_n gu_n d2u_n/dY2,  d2u_n/dY_j dY_k = iz^2 (d_jn d_kz + d_jz d_kn + 2 u_n d_jz d_kz)
  const double iz2 = iz * iz;
  HY[0][2] += gu[0] * iz2;
  HY[2][0] += gu[0] * iz2;
  HY[1][2] += gu[1] * iz2;
  HY[2][1] += gu[1] * iz2;
  HY[2][2] += 2.0 * iz2 * (gu[0] * u[0] + gu[1] * u[1]);
  // r . d2q / du dk for k = (f, k1, k2), then chained to Y
  double Huk[2][3];
  for (int n = 0; n < 2; ++n) {
    Huk[n][0] = D * rr[n] + 2.0 * D1 * ru * u[n];
    Huk[n][1] = c.f * (2.0 * ru * u[n] + s * rr[n]);
    Huk[n][2] = c.f * (4.0 * s * ru * u[n] + s * s * rr[n]);
  }
  double HYk[3][3];
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) HYk[j][k] = Huk[0][k] * B[0][j] + Huk[1][k] * B[1][j];
  // JY columns: rho -> e_b, phi -> -[Y0]x e_b = e_b x Y0, intrinsics -> 0,
  // dX -> R e_l (the rotated unit vectors)
  double JY[3][12];
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 12; ++i) JY[j][i] = 0.0;
  const double Yv[3] = {Y.x, Y.y, Y.z};
  for (int b = 0; b < 3; ++b) {
    JY[b][b] = 1.0;
    const V3 e = v3(b == 0, b == 1, b == 2);
    const V3 col = cross(e, Y);
    JY[0][3 + b] = col.x;
    JY[1][3 + b] = col.y;
    JY[2][3 + b] = col.z;
    const V3 Re = quat_rotate(c.qv, c.qw, e);
    JY[0][9 + b] = Re.x;
    JY[1][9 + b] = Re.y;
    JY[2][9 + b] = Re.z;
  }
  double T[3][12];  // HY JY, with H_Yk placed in the intrinsic columns
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 12; ++i)
      T[j][i] = (i >= 6 && i < 9) ? HYk[j][i - 6]
                                  : HY[j][0] * JY[0][i] + HY[j][1] * JY[1][i] + HY[j][2] * JY[2][i];
  for (int i = 0; i < 12; ++i)
    for (int j = i; j < 12; ++j) {
      double v;
      if (i >= 6 && i < 9 && j >= 6 && j < 9) {
        v = 0.0;  // H_kk: (f, k1) = s (r.u), (f, k2) = s^2 (r.u)
        if (i == 6 && j == 7) v = s * ru;
        if (i == 6 && j == 8) v = s * s * ru;
      } else if (i >= 6 && i < 9) {
        v = T[0][i] * JY[0][j] + T[1][i] * JY[1][j] + T[2][i] * JY[2][j];
      } else {
        v = JY[0][i] * T[0][j] + JY[1][i] * T[1][j] + JY[2][i] * T[2][j];
      }
      C[sym12(i, j)] = v;
    }
  // second derivatives of Y contracted with g
  const V3 g = v3(gY[0], gY[1], gY[2]);
  const double gdY = dot(g, Y);
  for (int a2 = 0; a2 < 3; ++a2)
    for (int b = a2; b < 3; ++b)
      C[sym12(3 + a2, 3 + b)] += 0.5 * (gY[a2] * Yv[b] + gY[b] * Yv[a2]) - (a2 == b ? gdY : 0.0);
  // [g]x entries: row a, column b
  const double gx[3][3] = {{0.0, -g.z, g.y}, {g.z, 0.0, -g.x}, {-g.y, g.x, 0.0}};
  for (int b = 0; b < 3; ++b)      // rho_b (row) - phi_a (column): (-1/2 [g]x)^T
    for (int a2 = 0; a2 < 3; ++a2) C[sym12(b, 3 + a2)] += -0.5 * gx[a2][b];
  for (int a2 = 0; a2 < 3; ++a2)   // phi_a (row) - dX_l (column): -[g]x R
    for (int l = 0; l < 3; ++l) {
      double v = 0.0;
      for (int k = 0; k < 3; ++k) v += gx[a2][k] * JY[k][9 + l];
      C[sym12(3 + a2, 9 + l)] -= v;
    }
}

// Robust loss on the squared residual norm s (Huber when delta > 0):
// returns rho(s) and writes rho'(s).
__device__ __forceinline__ double robust_rho(double s, double delta, double* drho) {
  if (delta > 0.0 && s > delta * delta) {
    const double rs = sqrt(s);
    *drho = delta / rs;
    return 2.0 * delta * rs - delta * delta;
  }
  *drho = 1.0;
  return s;
}

// Left SE(3) update of a camera row by the tangent (rho, phi, df, dk1, dk2):
// q' = normalise(q_phi * q), t' = q_phi(t) + V(phi) rho, with
// V(phi) rho = rho + b (phi x rho) + c phi x (phi x rho),
// b = (1 - cos th)/th^2, c = (th - sin th)/th^3 (second-order series below 1e-5).
__device__ __forceinline__ void retract_camera(const double* __restrict__ cam,
                                               const double* __restrict__ dlt,
                                               double* __restrict__ out) {
  const V3 rho = v3(dlt[0], dlt[1], dlt[2]);
  const V3 phi = v3(dlt[3], dlt[4], dlt[5]);
  const double th2 = dot(phi, phi);
  const double th = sqrt(th2);
  double b, c, hs, hc;
  if (th < 1e-5) {
    b = 0.5 - th2 * (1.0 / 24.0);
    c = (1.0 / 6.0) - th2 * (1.0 / 120.0);
    hs = 0.5 - th2 * (1.0 / 48.0);
    hc = 1.0 - th2 * 0.125;
  } else {
    double sn, cs;
    sincos(th, &sn, &cs);
    b = (1.0 - cs) / th2;
    c = (th - sn) / (th2 * th);
    double sh, ch;
    sincos(0.5 * th, &sh, &ch);
    hs = sh / th;
    hc = ch;
  }
  const V3 pv = hs * phi;  // quaternion of Exp(phi): (pv, hc)
  const V3 t = v3(cam[0], cam[1], cam[2]);
  const V3 pr = cross(phi, rho);
  const V3 tn = quat_rotate(pv, hc, t) + rho + b * pr + c * cross(phi, pr);
  const V3 qv = v3(cam[3], cam[4], cam[5]);
  const double qw = cam[6];
  // Hamilton product (pv, hc) * (qv, qw)
  const V3 nv = hc * qv + qw * pv + cross(pv, qv);
  const double nw = hc * qw - dot(pv, qv);
  const double inv = 1.0 / sqrt(dot(nv, nv) + nw * nw);
  out[0] = tn.x; out[1] = tn.y; out[2] = tn.z;
  out[3] = nv.x * inv; out[4] = nv.y * inv; out[5] = nv.z * inv; out[6] = nw * inv;
  out[7] = cam[7] + dlt[6];
  out[8] = cam[8] + dlt[7];
  out[9] = cam[9] + dlt[8];
}

// (Linv^T T)[r][c] = sum_{k >= r} Linv[k][r] T[k][c] for a lower-triangular
// 9x9 Linv (row-major): the block-Jacobi inverse Linv^T Linv with T = Linv,
// and the learned block Linv^T (Mh Linv) with T = Mh Linv.  One summation
// order for both, so a correction Mh of exactly the identity reproduces the
// block-Jacobi blocks bit for bit.
__device__ __forceinline__ double lt_times(const double* Li, const double* T, int r, int c) {
  double s = 0.0;
  for (int k = r; k < 9; ++k) s = fma(Li[9 * k + r], T[9 * k + c], s);
  return s;
}

}  // namespace ba
