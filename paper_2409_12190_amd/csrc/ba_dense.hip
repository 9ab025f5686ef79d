// gfx950 kernels of the direct solve of the reduced camera system: the
// paper's factorisation alternative to PCG (Sec. IV-C-1, Cholesky), applied
// to the Schur complement S (n = 9 n_c unknowns) assembled dense in FP64.
//
// Storage: lower triangle of S, row-major with leading dimension ld (a
// multiple of 64), followed by one extra row n holding b_S.  A right-looking
// blocked Cholesky with panels of DENSE_NB columns treats that row like any
// other row below the panel, so after the factorisation it holds y with
// L y = b_S (the forward substitution comes with the factorisation).  The
// back substitution L^T x = y runs panel by panel from the last one.
//
// Per panel k (columns k0 .. k0 + kb):
//   k_chol_diag    one workgroup: L11 = chol(A11) in LDS, and L11^-1;
//   k_chol_panel   L21 = A21 L11^-T for every row below the panel (and row n);
//   k_chol_update  A22 -= L21 L21^T on the lower triangle (64 x 64 tiles).
// Back substitution, per panel from the last:
//   k_back_partial partial sums of L21^T x over chunks of rows;
//   k_back_diag    x_k = L11^-T (y_k - sum of the partials, fixed order).
// All sums run in a fixed order: results are bitwise reproducible.
#include <algorithm>

#include "ba_dense.h"
#include "ba_device.h"

namespace ba {

namespace {

constexpr int NB = DENSE_NB;
constexpr int LDP = NB + 1;  // padded LDS row (doubles)

__device__ __forceinline__ double* row_ptr(double* A, int64_t ld, int64_t r) { return A + r * ld; }

}  // namespace

// zero the dense storage (rows 0 .. n, ld columns)
__global__ __launch_bounds__(256) void k_dense_zero(double* A, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    A[i] = 0.0;
}

// scatter S (upper blocks, diagonal blocks from Sdiag) into the lower
// triangle, and b_S into row n: one thread per stored value
template <typename T>
__global__ __launch_bounds__(256) void k_dense_scatter(DenseArgs a) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nblk = a.nnzb;
  const int n = 9 * a.nc;
  if (t < nblk * 81) {
    const int e = (int)(t / 81), q = (int)(t - 81 * (int64_t)(t / 81));
    const int i = q / 9, m = q - 9 * (q / 9);
    const int r = a.blk_row[e], c = a.S_col[e];
    if (r == c) {
      if (m <= i) row_ptr(a.A, a.ld, 9 * r + i)[9 * r + m] = a.Sdiag[81 * (size_t)r + q];
    } else {
      // S_rc[i][m] at (9r + i, 9c + m) with r < c: stored as (9c + m, 9r + i)
      row_ptr(a.A, a.ld, 9 * c + m)[9 * r + i] = (double)reinterpret_cast<const T*>(a.S)[81 * (size_t)e + q];
    }
  } else if (t < nblk * 81 + n) {
    const int j = (int)(t - nblk * 81);
    row_ptr(a.A, a.ld, n)[j] = a.b[j];
  }
}

// L11 = chol(A11) and its inverse, one workgroup of 256 threads
__global__ __launch_bounds__(256) void k_chol_diag(DenseArgs a, int k0, int kb) {
  __shared__ double L[NB][LDP];
  __shared__ double X[NB][LDP];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int q = t; q < NB * NB; q += blockDim.x) {
    const int i = q / NB, j = q - NB * (q / NB);
    L[i][j] = (i < kb && j <= i) ? row_ptr(a.A, a.ld, k0 + i)[k0 + j] : 0.0;
    X[i][j] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    // pivot, then column j below it, then the trailing lower triangle
    const double d = L[j][j];
    if (!(d > 0.0) || !isfinite(d)) {
      if (t == 0) bad = 1;
      break;  // uniform: every thread reads the same L[j][j]
    }
    const double piv = sqrt(d);
    __syncthreads();
    if (t == 0) L[j][j] = piv;
    for (int i = j + 1 + t; i < kb; i += blockDim.x) L[i][j] /= piv;
    __syncthreads();
    const int m = kb - j - 1;  // trailing size
    for (int q = t; q < m * m; q += blockDim.x) {
      const int i = j + 1 + q / m, c = j + 1 + (q - m * (q / m));
      if (c <= i) L[i][c] -= L[i][j] * L[c][j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (t == 0) atomicOr(a.error, (int)ERR_CAMERA_BLOCK);
    return;
  }
  // X = L11^-1 (lower): column c by one thread, forward substitution
  if (t < kb) {
    const int c = t;
    X[c][c] = 1.0 / L[c][c];
    for (int i = c + 1; i < kb; ++i) {
      double s = 0.0;
      for (int q = c; q < i; ++q) s += L[i][q] * X[q][c];
      X[i][c] = -s / L[i][i];
    }
  }
  __syncthreads();
  double* inv = a.Linv + (size_t)(k0 / NB) * NB * NB;
  for (int q = t; q < NB * NB; q += blockDim.x) {
    const int i = q / NB, j = q - NB * (q / NB);
    if (i < kb && j <= i) row_ptr(a.A, a.ld, k0 + i)[k0 + j] = L[i][j];
    inv[q] = X[i][j];
  }
}

// L21 = A21 L11^-T for rows k0 + kb .. n (row n: the right-hand side), 64
// rows per workgroup
__global__ __launch_bounds__(256) void k_chol_panel(DenseArgs a, int k0, int kb) {
  __shared__ double X[NB][LDP];
  __shared__ double R[NB][LDP];
  const int t = threadIdx.x;
  const int n = 9 * a.nc;
  const int r0 = k0 + kb + NB * blockIdx.x;
  const double* inv = a.Linv + (size_t)(k0 / NB) * NB * NB;
  for (int q = t; q < NB * NB; q += blockDim.x) {
    const int i = q / NB, j = q - NB * (q / NB);
    X[i][j] = inv[q];
    const int r = r0 + i;
    R[i][j] = (r <= n && j < kb) ? row_ptr(a.A, a.ld, r)[k0 + j] : 0.0;
  }
  __syncthreads();
  for (int q = t; q < NB * NB; q += blockDim.x) {
    const int i = q / NB, j = q - NB * (q / NB);
    const int r = r0 + i;
    if (r > n || j >= kb) continue;
    double s = 0.0;
    for (int p = 0; p <= j; ++p) s += R[i][p] * X[j][p];
    row_ptr(a.A, a.ld, r)[k0 + j] = s;
  }
}

// A22 -= L21 L21^T on the lower triangle of the trailing rows (and row n),
// one 64 x 64 tile per workgroup, 4 x 4 outputs per thread
__global__ __launch_bounds__(256) void k_chol_update(DenseArgs a, int k0, int kb) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (J > I) return;
  __shared__ double P[NB][LDP];
  __shared__ double Q[NB][LDP];
  const int t = threadIdx.x;
  const int n = 9 * a.nc;
  const int k1 = k0 + kb;
  const int ra = k1 + NB * I, ca = k1 + NB * J;
  for (int q = t; q < NB * NB; q += blockDim.x) {
    const int i = q / NB, p = q - NB * (q / NB);
    const int r = ra + i, c = ca + i;
    P[i][p] = (r <= n && p < kb) ? row_ptr(a.A, a.ld, r)[k0 + p] : 0.0;
    Q[i][p] = (c < n && p < kb) ? row_ptr(a.A, a.ld, c)[k0 + p] : 0.0;
  }
  __syncthreads();
  const int ti = t >> 4, tj = t & 15;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int p = 0; p < kb; ++p) {
    double x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = P[ti + 16 * u][p];
#pragma unroll
    for (int v = 0; v < 4; ++v) y[v] = Q[tj + 16 * v][p];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * y[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = ra + ti + 16 * u;
    if (r > n) continue;
    double* Ar = row_ptr(a.A, a.ld, r);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = ca + tj + 16 * v;
      if (c < n && c <= r) Ar[c] -= acc[u][v];
    }
  }
}

// partial sums of L21^T x over chunks of DENSE_BROWS rows below panel k:
// part[blk][j] = sum_r L[r][k0 + j] x_r (lane j of each wavefront owns
// column j; the four wavefronts' rows interleave and are summed in order)
__global__ __launch_bounds__(256) void k_back_partial(DenseArgs a, int k0, int kb) {
  __shared__ double red[4][NB];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int n = 9 * a.nc;
  const int r0 = k0 + kb + DENSE_BROWS * blockIdx.x;
  const int r1 = min(r0 + DENSE_BROWS, n);
  double s = 0.0;
  if (lane < kb)
    for (int r = r0 + w; r < r1; r += 4) s += row_ptr(a.A, a.ld, r)[k0 + lane] * a.x[r];
  red[w][lane] = s;
  __syncthreads();
  if (t < NB) a.part[(size_t)blockIdx.x * NB + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// x_k = L11^-T (y_k - sum_blk part[blk]) with y_k from row n
__global__ __launch_bounds__(64) void k_back_diag(DenseArgs a, int k0, int kb, int nparts) {
  __shared__ double tk[NB];
  const int j = threadIdx.x;
  const int n = 9 * a.nc;
  if (j < kb) {
    double s = row_ptr(a.A, a.ld, n)[k0 + j];
    for (int p = 0; p < nparts; ++p) s -= a.part[(size_t)p * NB + j];
    tk[j] = s;
  }
  __syncthreads();
  if (j < kb) {
    const double* inv = a.Linv + (size_t)(k0 / NB) * NB * NB;
    double s = 0.0;
    for (int i = j; i < kb; ++i) s += inv[i * NB + j] * tk[i];
    a.x[k0 + j] = s;
  }
}

// r = b_S - S x from the stored blocks (upper blocks of the row, their
// transposes from the column list, the FP64 diagonal block): per camera
// |r_a|^2 and |b_a|^2; then the relative residual into the step report
template <typename T>
__global__ __launch_bounds__(64) void k_dense_resid(DenseArgs a) {
  __shared__ double y[9];
  const int cam = blockIdx.x, t = threadIdx.x;
  if (t < 9) {
    const int i = t;
    double s = 0.0;
    const double* D = a.Sdiag + 81 * (size_t)cam;
    for (int m = 0; m < 9; ++m) s += D[9 * i + m] * a.x[9 * cam + m];
    for (int e = a.S_ptr[cam] + 1; e < a.S_ptr[cam + 1]; ++e) {
      const T* B = reinterpret_cast<const T*>(a.S) + 81 * (size_t)e;
      const int c = a.S_col[e];
      for (int m = 0; m < 9; ++m) s += (double)B[9 * i + m] * a.x[9 * c + m];
    }
    for (int q = a.T_ptr[cam]; q < a.T_ptr[cam + 1]; ++q) {
      const T* B = reinterpret_cast<const T*>(a.S) + 81 * (size_t)a.T_blk[q];
      const int r = a.T_src[q];
      for (int m = 0; m < 9; ++m) s += (double)B[9 * m + i] * a.x[9 * r + m];
    }
    y[i] = a.b[9 * cam + i] - s;
  }
  __syncthreads();
  if (t == 0) {
    double rr = 0.0, bb = 0.0;
    for (int i = 0; i < 9; ++i) {
      rr += y[i] * y[i];
      bb += a.b[9 * cam + i] * a.b[9 * cam + i];
    }
    a.resid[2 * (size_t)cam] = rr;
    a.resid[2 * (size_t)cam + 1] = bb;
  }
}

__global__ __launch_bounds__(256) void k_dense_resid_final(DenseArgs a) {
  __shared__ double sr[256], sb[256];
  const int t = threadIdx.x;
  double rr = 0.0, bb = 0.0;
  for (int c = t; c < a.nc; c += blockDim.x) {
    rr += a.resid[2 * (size_t)c];
    bb += a.resid[2 * (size_t)c + 1];
  }
  sr[t] = rr;
  sb[t] = bb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      sr[t] += sr[t + s];
      sb[t] += sb[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    a.info->cg_iters = 0;
    a.info->cg_breakdown = 0;
    a.info->cg_rel_resid = sb[0] > 0.0 ? sqrt(sr[0] / sb[0]) : 0.0;
  }
}

template <typename T>
hipError_t launch_dense_solve(const DenseArgs& a, hipStream_t s) {
  const int n = 9 * a.nc;
  const int64_t count = (int64_t)(n + 1) * a.ld;
  const int zb = (int)std::min<int64_t>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(k_dense_zero, dim3(zb), dim3(256), 0, s, a.A, count);
  const int64_t sc = a.nnzb * 81 + n;
  hipLaunchKernelGGL(k_dense_scatter<T>, dim3((unsigned)((sc + 255) / 256)), dim3(256), 0, s, a);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = std::min(NB, n - k0);
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, a, k0, kb);
    const int below = n - (k0 + kb) + 1;  // rows below the panel, with row n
    hipLaunchKernelGGL(k_chol_panel, dim3((below + NB - 1) / NB), dim3(256), 0, s, a, k0, kb);
    const int rows = below, cols = n - (k0 + kb);
    if (cols > 0) {
      const int tr = (rows + NB - 1) / NB, tc = (cols + NB - 1) / NB;
      hipLaunchKernelGGL(k_chol_update, dim3(tc, tr), dim3(256), 0, s, a, k0, kb);
    } else {
      // last panel: row n still takes the update of no trailing columns
    }
  }
  const int last = ((n - 1) / NB) * NB;
  for (int k0 = last; k0 >= 0; k0 -= NB) {
    const int kb = std::min(NB, n - k0);
    const int below = n - (k0 + kb);
    const int nparts = (below + DENSE_BROWS - 1) / DENSE_BROWS;
    if (nparts > 0)
      hipLaunchKernelGGL(k_back_partial, dim3(nparts), dim3(256), 0, s, a, k0, kb);
    hipLaunchKernelGGL(k_back_diag, dim3(1), dim3(64), 0, s, a, k0, kb, nparts);
  }
  hipLaunchKernelGGL(k_dense_resid<T>, dim3(a.nc), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_dense_resid_final, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_dense_solve<float>(const DenseArgs&, hipStream_t);
template hipError_t launch_dense_solve<double>(const DenseArgs&, hipStream_t);

}  // namespace ba
