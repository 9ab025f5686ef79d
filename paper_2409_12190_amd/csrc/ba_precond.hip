// gfx950 kernels of the learned correction of the block-Jacobi
// preconditioner of the reduced camera system.
//
// The paper preconditions its PCG with a diagonal (block) preconditioner
// (Sec. IV-C-2).  Here each 9x9 block of block-Jacobi is corrected from the
// camera co-visibility graph of the system:
//   S_ii = L_i L_i^T, S^_ij = L_i^-1 S_ij L_j^-T, E_i = sum_j S^_ij S^_ij^T,
//   a_ij = |S^_ij|_F, w_ij = a_ij / sum_j a_ij;
//   x_i = [upper(E_i), log(1 + tr E_i), log(1 + deg_i)]
//   h0 = relu(W_in x + b_in); three layers h = relu(W_s h + W_m (sum_j w_ij h_j) + b)
//   o = W_out h + b_out, C_i = strict lower(o) + diag(exp(o_diag)),
//   M_i = L_i^-T C_i C_i^T L_i^-1  (o = 0: block-Jacobi).
// Training loss of a system: (1/n) sum_i tr(Mh G Mh) - 2 tr(Mh) + 9 with
// Mh = C C^T, G = I + E (the squared Frobenius distance of the normalised
// preconditioned operator to I, block row by block row).
//
// All network arithmetic is FP32; every reduction runs in a fixed order
// (no atomics), so training is bitwise reproducible.
#include "ba_device.h"
#include "ba_precond.h"
#include "ba_reduce.h"

namespace ba {

namespace {

__device__ __forceinline__ int up9(int r, int c) { return r * 9 - (r * (r - 1)) / 2 + (c - r); }
__device__ __forceinline__ int lo9(int r, int c) { return (r * (r + 1)) / 2 + c; }

}  // namespace

// ---------------------------------------------------------------------------
// graph features of camera i (one workgroup of 64 per camera).  Each slot's
// normalised block is evaluated in the orientation of the stored upper block,
// T = Linv_row S_e Linv_col^T, by the same code from both endpoints, so the
// two endpoints see bit-identical weights.
// ---------------------------------------------------------------------------
// One workgroup of W wavefronts per camera i; wavefront v takes the
// camera's neighbour slots v, v + W, ...: the lanes share one block at a
// time through the wavefront's own LDS buffers (entry (r, c) of each 9x9
// product per lane; the wavefronts synchronise only within themselves), and
// the wavefronts' partial sums of E_i are added in wavefront order.  Small
// graphs take W = 16 (each camera's few rounds are the kernel's latency),
// large ones W = 4 (less LDS per workgroup: more cameras in flight).
constexpr int PC_FEAT_WMAX = 1024;  // slots whose weights wait in LDS for the normalisation
constexpr int PC_FEAT_SMALL = 1024;  // graphs up to this many cameras take 16 wavefronts

// Orders the LDS accesses of one wavefront's lanes (a wavefront-wide barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int PC_FEAT_WAVES, typename T>
__global__ __launch_bounds__(64 * PC_FEAT_WAVES) void k_pc_features(PcFeatureArgs a) {
  // block, the neighbour's Linv, products (rows of 128: every lane stores
  // entries lane and lane + 64 without a branch)
  __shared__ double sm[PC_FEAT_WAVES][4][128];
  __shared__ double Li[81];                    // this camera's Linv
  __shared__ double es[PC_FEAT_WAVES][45];
  __shared__ double as_[PC_FEAT_WAVES];
  __shared__ double etot[45];
  __shared__ float wl[PC_FEAT_WMAX];           // a_ij of the first PC_FEAT_WMAX slots
  const int i = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* Bv = sm[wave][0];
  double* Ln = sm[wave][1];
  double* Pm = sm[wave][2];
  double* Tm = sm[wave][3];
  for (int q = threadIdx.x; q < 81; q += blockDim.x) Li[q] = a.Linv[81 * (size_t)i + q];
  __syncthreads();
  const int s0 = a.nbr_ptr[i], s1 = a.nbr_ptr[i + 1];
  const T* __restrict__ Sv = reinterpret_cast<const T*>(a.S);
  // entry of E_i this lane accumulates (lanes < 45)
  int er = 0, ec = 0;
  if (lane < 45) {
    while (up9(er, 8) < lane) ++er;
    ec = er + (lane - up9(er, er));
  }
  double e_acc = 0.0, asum = 0.0;
  // this wavefront's slots: s0 + wave + PC_FEAT_WAVES * it, it < rounds
  const int rounds = s1 - s0 > wave ? (s1 - s0 - wave + PC_FEAT_WAVES - 1) / PC_FEAT_WAVES : 0;
  // the next round's block and neighbour factor are loaded into registers
  // while the current one is processed (entries lane and lane + 64)
  // (the neighbour of an upper block of row i has the larger index)
  int nblk = 0, nother = 0;
  double pb0 = 0.0, pb1 = 0.0, pl0 = 0.0, pl1 = 0.0;
  auto prefetch = [&](int it) {
    const int sl = min(s0 + it * PC_FEAT_WAVES + wave, s1 - 1);
    nblk = a.nbr_blk[sl];
    nother = a.nbr[sl];
    const int other = nother;
    pb0 = (double)Sv[81 * (size_t)nblk + lane];
    pl0 = a.Linv[81 * (size_t)other + lane];
    const int q1 = min(lane + 64, 80);
    pb1 = (double)Sv[81 * (size_t)nblk + q1];
    pl1 = a.Linv[81 * (size_t)other + q1];
  };
  if (rounds > 0) prefetch(0);
  for (int it = 0; it < rounds; ++it) {
    const int sl = s0 + it * PC_FEAT_WAVES + wave;
    const bool valid = sl < s1;
    const bool up = nother > i;  // camera i is the block's row (else its column)
    Bv[lane] = pb0;
    Ln[lane] = pl0;
    Bv[lane + 64] = pb1;
    Ln[lane + 64] = pl1;
    if (it + 1 < rounds) prefetch(it + 1);
    wave_sync();
    const double* La = up ? Li : Ln;  // Linv of the block's row camera
    const double* Lb = up ? Ln : Li;  // and of its column camera
    // P = Linv_row S_e (lower-triangular factor)
    for (int q = lane; q < 81; q += 64) {
      const int r = q / 9, c = q - 9 * r;
      double v = 0.0;
      for (int k = 0; k <= r; ++k) v += La[9 * r + k] * Bv[9 * k + c];
      Pm[q] = v;
    }
    wave_sync();
    // T = P Linv_col^T: the normalised block as stored
    double fro = 0.0;
    for (int q = lane; q < 81; q += 64) {
      const int r = q / 9, c = q - 9 * r;
      double v = 0.0;
      for (int k = 0; k <= c; ++k) v += Pm[9 * r + k] * Lb[9 * c + k];
      Tm[q] = v;
      fro += v * v;
    }
    wave_sync();
    fro = wave_sum(fro);
    if (valid) {
      // S^_ij = T (camera i is the block's row) or T^T: E_i += S^ S^^T
      if (lane < 45) {
        double v = 0.0;
        if (up)
          for (int k = 0; k < 9; ++k) v += Tm[9 * er + k] * Tm[9 * ec + k];
        else
          for (int k = 0; k < 9; ++k) v += Tm[9 * k + er] * Tm[9 * k + ec];
        e_acc += v;
      }
      const double aw = sqrt(fro);
      if (lane == 0) {  // normalised below
        if (sl - s0 < PC_FEAT_WMAX) wl[sl - s0] = (float)aw;
        else a.w[sl] = (float)aw;
      }
      asum += aw;
    }
    wave_sync();
  }
  if (lane < 45) es[wave][lane] = e_acc;
  if (lane == 0) as_[wave] = asum;
  __syncthreads();
  const int t = threadIdx.x;
  double tot = 0.0;
  for (int v = 0; v < PC_FEAT_WAVES; ++v) tot += as_[v];
  if (t < 45) {
    double e = 0.0;
    for (int v = 0; v < PC_FEAT_WAVES; ++v) e += es[v][t];
    etot[t] = e;
    a.E[45 * (size_t)i + t] = (float)e;
    a.X[GNN_F * (size_t)i + t] = (float)e;
  } else if (t == 46) {
    a.X[GNN_F * (size_t)i + 46] = (float)log1p((double)(s1 - s0));
  }
  // weights: a_ij / sum_j a_ij (each slot's a_ij stored above by its wavefront's lane 0)
  for (int sl = s0 + t; sl < s1; sl += blockDim.x) {
    const float aw = sl - s0 < PC_FEAT_WMAX ? wl[sl - s0] : a.w[sl];
    a.w[sl] = tot > 0.0 ? (float)((double)aw / tot) : 0.0f;
  }
  __syncthreads();
  double tr = 0.0;
  for (int r = 0; r < 9; ++r) tr += etot[up9(r, r)];
  const float xtr = (float)log1p(tr);
  if (t == 45) a.X[GNN_F * (size_t)i + 45] = xtr;
  if (a.H0 && t < GNN_H) {
    // input layer of the network for this camera, the training formula:
    // z = b_in + sum_k x_k W_in[t][k] in feature order, h0 = relu(z)
    const float* W = a.params + GNN_OFF_WIN + (size_t)t * GNN_F;
    float z = a.params[GNN_OFF_BIN + t];
    for (int k = 0; k < GNN_F; ++k) {
      const float xk = k < 45 ? (float)etot[k] : k == 45 ? xtr : (float)log1p((double)(s1 - s0));
      z = fmaf(xk, W[k], z);
    }
    a.H0[GNN_H * (size_t)i + t] = fmaxf(z, 0.0f);
  }
}

// ---------------------------------------------------------------------------
// dense layer: Z[n][o] = b[o] + sum_k X[n][k] W1[o][k] + sum_k M[n][k] W2[o][k],
// H = relu(Z); four rows x 64 outputs per workgroup
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gnn_dense(int n, const float* __restrict__ X, int K1,
                                                    const float* __restrict__ M, int K2,
                                                    const float* __restrict__ W1,
                                                    const float* __restrict__ W2,
                                                    const float* __restrict__ b, int nout,
                                                    float* __restrict__ Z, float* __restrict__ H) {
  const int o = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n || o >= nout) return;
  float z = b[o];
  const float* x = X + (size_t)row * K1;
  const float* w1 = W1 + (size_t)o * K1;
  for (int k = 0; k < K1; ++k) z = fmaf(x[k], w1[k], z);
  if (M) {
    const float* m = M + (size_t)row * K2;
    const float* w2 = W2 + (size_t)o * K2;
    for (int k = 0; k < K2; ++k) z = fmaf(m[k], w2[k], z);
  }
  Z[(size_t)row * nout + o] = z;
  if (H) H[(size_t)row * nout + o] = fmaxf(z, 0.0f);
}

// weighted mean of the neighbours' hidden states: M_i = sum_s w_s H_nbr(s)
__global__ __launch_bounds__(256) void k_gnn_aggregate(int n, const int32_t* __restrict__ nbr_ptr,
                                                        const int32_t* __restrict__ nbr,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ H,
                                                        float* __restrict__ M) {
  const int f = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  float m = 0.0f;
#pragma unroll 4
  for (int s = nbr_ptr[i]; s < nbr_ptr[i + 1]; ++s) m = fmaf(w[s], H[(size_t)nbr[s] * GNN_H + f], m);
  M[(size_t)i * GNN_H + f] = m;
}

// transpose of the aggregation: dH_j += sum_s w_rev(s) dM_nbr(s)
__global__ __launch_bounds__(256) void k_gnn_aggregate_t(int n, const int32_t* __restrict__ nbr_ptr,
                                                          const int32_t* __restrict__ nbr,
                                                          const int32_t* __restrict__ rev,
                                                          const float* __restrict__ w,
                                                          const float* __restrict__ dM,
                                                          float* __restrict__ dH) {
  const int f = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  float acc = dH[(size_t)j * GNN_H + f];
  for (int s = nbr_ptr[j]; s < nbr_ptr[j + 1]; ++s)
    acc = fmaf(w[rev[s]], dM[(size_t)nbr[s] * GNN_H + f], acc);
  dH[(size_t)j * GNN_H + f] = acc;
}

// ---------------------------------------------------------------------------
// output layer, loss and its gradient with respect to the outputs, or the
// preconditioner blocks (one workgroup of 64 per camera)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_gnn_output(GraphDev g, const float* __restrict__ P,
                                                    const double* __restrict__ Linv,
                                                    double* __restrict__ Minv, int with_loss) {
  __shared__ float o[45];
  __shared__ float C[81], Mh[81], Gm[81], Q[81], Gam[81];
  __shared__ double red[64];
  __shared__ double T[81];
  const int i = blockIdx.x, t = threadIdx.x;
  const float* h = g.H[GNN_L] + (size_t)i * GNN_H;
  if (t < GNN_O) {
    float v = P[GNN_OFF_BOUT + t];
    const float* wr = P + GNN_OFF_WOUT + (size_t)t * GNN_H;
    for (int k = 0; k < GNN_H; ++k) v = fmaf(wr[k], h[k], v);
    o[t] = v;
  }
  __syncthreads();
  for (int q = t; q < 81; q += 64) {
    const int r = q / 9, c = q - 9 * r;
    C[q] = c > r ? 0.0f : (c == r ? expf(o[lo9(r, r)]) : o[lo9(r, c)]);
  }
  __syncthreads();
  for (int q = t; q < 81; q += 64) {  // Mh = C C^T
    const int r = q / 9, c = q - 9 * r;
    float v = 0.0f;
    for (int k = 0; k < 9; ++k) v = fmaf(C[9 * r + k], C[9 * c + k], v);
    Mh[q] = v;
  }
  __syncthreads();
  if (Minv) {  // M_i = Linv^T (Mh Linv) in FP64
    const double* Li = Linv + 81 * (size_t)i;
    for (int q = t; q < 81; q += 64) {  // T = Mh Linv (exactly Linv for Mh = I)
      const int r = q / 9, c = q - 9 * r;
      double v = 0.0;
      for (int l = 0; l < 9; ++l) v = fma((double)Mh[9 * r + l], Li[9 * l + c], v);
      T[q] = v;
    }
    __syncthreads();
    for (int q = t; q < 81; q += 64) {
      const int r = q / 9, c = q - 9 * r;
      Minv[81 * (size_t)i + q] = lt_times(Li, T, r, c);
    }
  }
  if (!with_loss) return;
  const float* E = g.E + 45 * (size_t)i;
  for (int q = t; q < 81; q += 64) {
    const int r = q / 9, c = q - 9 * r;
    Gm[q] = E[r <= c ? up9(r, c) : up9(c, r)] + (r == c ? 1.0f : 0.0f);
  }
  __syncthreads();
  double part = 0.0;
  for (int q = t; q < 81; q += 64) {  // Q = Mh G, loss terms tr(Q Mh) and tr(Mh)
    const int r = q / 9, c = q - 9 * r;
    float v = 0.0f;
    for (int k = 0; k < 9; ++k) v = fmaf(Mh[9 * r + k], Gm[9 * k + c], v);
    Q[q] = v;
    part += (double)v * (double)Mh[9 * c + r] - (r == c ? 2.0 * (double)Mh[q] : 0.0);
  }
  red[t] = part;
  __syncthreads();
  if (t == 0) {
    double s = 9.0;
    for (int k = 0; k < 64; ++k) s += red[k];
    g.loss_part[i] = s / g.nc;
  }
  const float inv_n = 1.0f / (float)g.nc;
  for (int q = t; q < 81; q += 64) {  // Gam = (G Mh + Mh G - 2 I) / n = (Q^T + Q - 2 I) / n
    const int r = q / 9, c = q - 9 * r;
    Gam[q] = (Q[9 * c + r] + Q[q] - (r == c ? 2.0f : 0.0f)) * inv_n;
  }
  __syncthreads();
  if (t < GNN_O) {  // dC = 2 Gam C on the lower triangle; chain through exp on the diagonal
    int r = 0;
    while (lo9(r + 1, 0) <= t) ++r;
    const int c = t - lo9(r, 0);
    float v = 0.0f;
    for (int k = 0; k < 9; ++k) v = fmaf(Gam[9 * r + k], C[9 * k + c], v);
    v *= 2.0f;
    if (r == c) v *= C[9 * r + r];
    g.dO[(size_t)i * GNN_O + t] = v;
  }
}

__global__ __launch_bounds__(256) void k_sum_loss(const double* __restrict__ part, int n,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int k = 0; k < 256; ++k) tot += red[k];
    *out = tot;
  }
}

// ---------------------------------------------------------------------------
// backward of a dense layer Z = X W^T (+ b):
//   dW[o][k] += sum_n dZ[n][o] X[n][k], db[o] += sum_n dZ[n][o] (one thread
//   per weight, rows in order), and dX[n][k] = sum_o dZ[n][o] W[o][k]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gnn_dW(int n, int nout, int K, const float* __restrict__ dZ,
                                                 const float* __restrict__ X, float* __restrict__ dW,
                                                 float* __restrict__ db) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < nout * K) {
    const int o = idx / K, k = idx - K * (idx / K);
    float s = 0.0f;
    for (int r = 0; r < n; ++r) s = fmaf(dZ[(size_t)r * nout + o], X[(size_t)r * K + k], s);
    dW[idx] += s;
  } else if (db && idx < nout * K + nout) {
    const int o = idx - nout * K;
    float s = 0.0f;
    for (int r = 0; r < n; ++r) s += dZ[(size_t)r * nout + o];
    db[o] += s;
  }
}

__global__ __launch_bounds__(256) void k_gnn_dX(int n, int nout, int K, const float* __restrict__ dZ,
                                                 const float* __restrict__ W, float* __restrict__ dX,
                                                 const float* __restrict__ Zmask) {
  const int k = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n || k >= K) return;
  float s = 0.0f;
  for (int o = 0; o < nout; ++o) s = fmaf(dZ[(size_t)row * nout + o], W[(size_t)o * K + k], s);
  // with Zmask: the result is the gradient of the pre-activation of a relu layer
  if (Zmask && !(Zmask[(size_t)row * K + k] > 0.0f)) s = 0.0f;
  dX[(size_t)row * K + k] = s;
}

__global__ __launch_bounds__(256) void k_gnn_relu_mask(int n, const float* __restrict__ Z,
                                                       float* __restrict__ d) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < (int64_t)n * GNN_H && !(Z[q] > 0.0f)) d[q] = 0.0f;
}

__global__ __launch_bounds__(256) void k_gnn_adam(int64_t n, float* __restrict__ p,
                                                  const float* __restrict__ g, float* __restrict__ m,
                                                  float* __restrict__ v, float lr, float b1, float b2,
                                                  float eps, float c1, float c2, float gscale) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q] * gscale;
  const float mq = b1 * m[q] + (1.0f - b1) * gq;
  const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// ---------------------------------------------------------------------------
// inference of the message layers in BF16 on the matrix cores, FP32
// accumulate: the same layers as k_gnn_aggregate + k_gnn_dense with the
// dense inputs and weights rounded to bfloat16 (the input layer is formed in
// FP32 by the feature kernel).
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// weights of the message layers as BF16 rows: per layer [W_s | W_m] (64 x 128)
__global__ __launch_bounds__(256) void k_gnn_weights_bf16(const float* __restrict__ P,
                                                          short* __restrict__ Wb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= GNN_L * GNN_H * GNN_KHID) return;
  const int l = r / (GNN_H * GNN_KHID), rr = r - l * (GNN_H * GNN_KHID);
  const int o = rr / GNN_KHID, k = rr - GNN_KHID * (rr / GNN_KHID);
  const float* L0 = P + GNN_OFF_L0 + l * GNN_LAYER_SIZE;
  Wb[r] = to_bf16(k < GNN_H ? L0[o * GNN_H + k] : L0[GNN_H * GNN_H + o * GNN_H + (k - GNN_H)]);
}

// One message-passing layer of the inference, aggregation fused:
//   M = sum_s w_s H_nbr(s) for the workgroup's 16 rows (into LDS), then
//   Z = [H | M] [W_s | W_m]^T + b, H' = relu(Z) on the matrix cores (one
//   16x16 output tile per wavefront, v_mfma_f32_16x16x16_bf16; lane l: A row
//   l%16, k 4(l/16)..+3; B column l%16, same k; D rows 4(l/16)..+3 of column
//   l%16); the aggregated messages never go to memory.
__global__ __launch_bounds__(256) void k_gnn_layer_bf16(int n, const int32_t* __restrict__ nbr_ptr,
                                                         const int32_t* __restrict__ nbr,
                                                         const float* __restrict__ wgt,
                                                         const float* __restrict__ Hin,
                                                         const short* __restrict__ Wb,
                                                         const float* __restrict__ b,
                                                         float* __restrict__ Hout) {
  __shared__ float Ms[16][GNN_H + 4];
  const int r0 = blockIdx.x * 16;
  const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
  const int row = r0 + (lane & 15), kq = 4 * (lane >> 4);
  // this lane's matrix-core operands that do not depend on the messages (its
  // row's own features, the weights), requested before the aggregation
  constexpr int KB = GNN_KHID / 16;
  float hown[GNN_H / 16][4];
#pragma unroll
  for (int b4 = 0; b4 < GNN_H / 16; ++b4)
#pragma unroll
    for (int j = 0; j < 4; ++j) hown[b4][j] = row < n ? Hin[(size_t)row * GNN_H + 16 * b4 + kq + j] : 0.0f;
  bf16x4 wv4[KB];
  {
    const short* w = Wb + (size_t)(16 * t + (lane & 15)) * GNN_KHID + kq;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) wv4[kb] = *reinterpret_cast<const bf16x4*>(w + 16 * kb);
  }
  {
    // thread t: row t / 16 of the workgroup, features 4 (t % 16) .. + 3.
    // The row's 16 threads load 32 neighbour slots at once (two each) and
    // pass them round by shuffles, so the feature rows of 16 neighbours are
    // requested together; the sum still takes the neighbours in order.
    const int lr = threadIdx.x >> 4, j = threadIdx.x & 15, f = 4 * j;
    const int i = r0 + lr;
    float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f;
    const int s0 = i < n ? nbr_ptr[i] : 0, s1 = i < n ? nbr_ptr[i + 1] : 0;
    for (int sb = s0; sb < s1; sb += 32) {
      const int cnt = min(32, s1 - sb);
      const int my_n0 = j < cnt ? nbr[sb + j] : 0, my_n1 = j + 16 < cnt ? nbr[sb + j + 16] : 0;
      const float my_w0 = j < cnt ? wgt[sb + j] : 0.0f, my_w1 = j + 16 < cnt ? wgt[sb + j + 16] : 0.0f;
      for (int q0 = 0; q0 < cnt; q0 += 16) {
        const int my_n = q0 == 0 ? my_n0 : my_n1;
        const float my_w = q0 == 0 ? my_w0 : my_w1;
        float4 h[16];
        float wv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int src = __shfl(my_n, q, 16);
          wv[q] = __shfl(my_w, q, 16);
          h[q] = q0 + q < cnt ? *reinterpret_cast<const float4*>(Hin + (size_t)src * GNN_H + f)
                              : float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          if (q0 + q < cnt) {
            m0 = fmaf(wv[q], h[q].x, m0);
            m1 = fmaf(wv[q], h[q].y, m1);
            m2 = fmaf(wv[q], h[q].z, m2);
            m3 = fmaf(wv[q], h[q].w, m3);
          }
        }
      }
    }
    Ms[lr][f] = m0;
    Ms[lr][f + 1] = m1;
    Ms[lr][f + 2] = m2;
    Ms[lr][f + 3] = m3;
  }
  __syncthreads();
  f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    bf16x4 av;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 16 * kb + kq + j;
      float v = 0.0f;
      if (row < n) v = k < GNN_H ? hown[kb][j] : Ms[lane & 15][k - GNN_H];
      av[j] = to_bf16(v);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, wv4[kb], acc, 0, 0, 0);
  }
  const int col = 16 * t + (lane & 15);
  for (int j = 0; j < 4; ++j) {
    const int r = r0 + kq + j;
    if (r < n) Hout[(size_t)r * GNN_H + col] = fmaxf(acc[j] + b[col], 0.0f);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_gnn_weights_bf16(const float* P, short* Wb, hipStream_t s) {
  const int n = GNN_L * GNN_H * GNN_KHID;
  hipLaunchKernelGGL(k_gnn_weights_bf16, dim3((n + 255) / 256), dim3(256), 0, s, P, Wb);
  return hipGetLastError();
}

hipError_t launch_gnn_forward_bf16(const GraphDev& g, const float* P, const short* Wb, hipStream_t s) {
  const dim3 grid((g.nc + 15) / 16), blk(256);
  for (int l = 0; l < GNN_L; ++l) {
    const short* Wl = Wb + (size_t)l * GNN_H * GNN_KHID;
    const float* bl = P + GNN_OFF_L0 + l * GNN_LAYER_SIZE + 2 * GNN_H * GNN_H;
    hipLaunchKernelGGL(k_gnn_layer_bf16, grid, blk, 0, s, g.nc, g.nbr_ptr, g.nbr, g.w, g.H[l], Wl, bl,
                       g.H[l + 1]);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pc_features(const PcFeatureArgs& a, hipStream_t s) {
  if (a.nc <= PC_FEAT_SMALL)
    hipLaunchKernelGGL((k_pc_features<16, T>), dim3(a.nc), dim3(64 * 16), 0, s, a);
  else
    hipLaunchKernelGGL((k_pc_features<4, T>), dim3(a.nc), dim3(64 * 4), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_pc_features<float>(const PcFeatureArgs&, hipStream_t);
template hipError_t launch_pc_features<double>(const PcFeatureArgs&, hipStream_t);

hipError_t launch_gnn_forward(const GraphDev& g, const float* P, hipStream_t s) {
  const dim3 grid((g.nc + 3) / 4), blk(256);
  hipLaunchKernelGGL(k_gnn_dense, grid, blk, 0, s, g.nc, g.X, GNN_F, (const float*)nullptr, 0,
                     P + GNN_OFF_WIN, (const float*)nullptr, P + GNN_OFF_BIN, GNN_H, g.Z[0], g.H[0]);
  for (int l = 0; l < GNN_L; ++l) {
    const float* L0 = P + GNN_OFF_L0 + l * GNN_LAYER_SIZE;
    hipLaunchKernelGGL(k_gnn_aggregate, grid, blk, 0, s, g.nc, g.nbr_ptr, g.nbr, g.w, g.H[l], g.M[l]);
    hipLaunchKernelGGL(k_gnn_dense, grid, blk, 0, s, g.nc, g.H[l], GNN_H, g.M[l], GNN_H, L0,
                       L0 + GNN_H * GNN_H, L0 + 2 * GNN_H * GNN_H, GNN_H, g.Z[l + 1], g.H[l + 1]);
  }
  return hipGetLastError();
}

hipError_t launch_gnn_output(const GraphDev& g, const float* P, const double* Linv, double* Minv,
                             bool with_loss, hipStream_t s) {
  hipLaunchKernelGGL(k_gnn_output, dim3(g.nc), dim3(64), 0, s, g, P, Linv, Minv, with_loss ? 1 : 0);
  if (with_loss) hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, g.loss_part, g.nc, g.loss);
  return hipGetLastError();
}

hipError_t launch_gnn_backward(const GraphDev& gin, const float* P, float* G, hipStream_t s) {
  GraphDev g = gin;  // dZ / dH swap roles layer by layer
  const int n = g.nc;
  const dim3 rows((n + 3) / 4), blk(256);
  auto wgrid = [](int nout, int K) { return dim3((nout * K + nout + 255) / 256); };
  // output layer
  hipLaunchKernelGGL(k_gnn_dW, wgrid(GNN_O, GNN_H), blk, 0, s, n, GNN_O, GNN_H, g.dO, g.H[GNN_L],
                     G + GNN_OFF_WOUT, G + GNN_OFF_BOUT);
  // dZ_L = (dO W_out) masked by relu of Z_L
  hipLaunchKernelGGL(k_gnn_dX, rows, blk, 0, s, n, GNN_O, GNN_H, g.dO, P + GNN_OFF_WOUT, g.dZ,
                     g.Z[GNN_L]);
  for (int l = GNN_L - 1; l >= 0; --l) {
    const int64_t off = GNN_OFF_L0 + l * GNN_LAYER_SIZE;
    hipLaunchKernelGGL(k_gnn_dW, wgrid(GNN_H, GNN_H), blk, 0, s, n, GNN_H, GNN_H, g.dZ, g.H[l],
                       G + off, G + off + 2 * GNN_H * GNN_H);
    hipLaunchKernelGGL(k_gnn_dW, dim3((GNN_H * GNN_H + 255) / 256), blk, 0, s, n, GNN_H, GNN_H,
                       g.dZ, g.M[l], G + off + GNN_H * GNN_H, (float*)nullptr);
    // dM = dZ W_m, dH_l = dZ W_s + aggregation^T(dM), then the relu mask of Z_l
    hipLaunchKernelGGL(k_gnn_dX, rows, blk, 0, s, n, GNN_H, GNN_H, g.dZ, P + off + GNN_H * GNN_H,
                       g.dM, (const float*)nullptr);
    hipLaunchKernelGGL(k_gnn_dX, rows, blk, 0, s, n, GNN_H, GNN_H, g.dZ, P + off, g.dH,
                       (const float*)nullptr);
    hipLaunchKernelGGL(k_gnn_aggregate_t, rows, blk, 0, s, n, g.nbr_ptr, g.nbr, g.rev, g.w, g.dM, g.dH);
    hipLaunchKernelGGL(k_gnn_relu_mask, dim3((unsigned)(((int64_t)n * GNN_H + 255) / 256)), blk, 0, s,
                       n, g.Z[l], g.dH);
    // the masked dH_l is the next dZ
    float* tmp = g.dZ;
    g.dZ = g.dH;
    g.dH = tmp;
  }
  hipLaunchKernelGGL(k_gnn_dW, wgrid(GNN_H, GNN_F), blk, 0, s, n, GNN_H, GNN_F, g.dZ, g.X,
                     G + GNN_OFF_WIN, G + GNN_OFF_BIN);
  return hipGetLastError();
}

hipError_t launch_gnn_adam(int64_t n, float* p, const float* g, float* m, float* v, int step, float lr,
                           float b1, float b2, float eps, float gscale, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_gnn_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, g, m, v, lr,
                     b1, b2, eps, c1, c2, gscale);
  return hipGetLastError();
}

}  // namespace ba
