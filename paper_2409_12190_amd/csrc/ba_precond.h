// Learned correction of the block-Jacobi preconditioner: graph layout,
// argument blocks and launchers (device pointers only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ba_internal.h"

namespace ba {

constexpr int GNN_F = 47;    // node input features
constexpr int GNN_H = 64;    // hidden width
constexpr int GNN_O = 45;    // outputs: lower triangle of a 9x9 factor
constexpr int GNN_L = 3;     // message-passing layers

// offsets of the parameter blocks in the flat FP32 parameter vector:
// W_in [H][F], b_in [H], then per layer W_s [H][H], W_m [H][H], b [H],
// then W_out [O][H], b_out [O]
constexpr int64_t GNN_OFF_WIN = 0;
constexpr int64_t GNN_OFF_BIN = GNN_OFF_WIN + GNN_H * GNN_F;
constexpr int64_t GNN_OFF_L0 = GNN_OFF_BIN + GNN_H;
constexpr int64_t GNN_LAYER_SIZE = 2 * GNN_H * GNN_H + GNN_H;
constexpr int64_t GNN_OFF_WOUT = GNN_OFF_L0 + GNN_L * GNN_LAYER_SIZE;
constexpr int64_t GNN_OFF_BOUT = GNN_OFF_WOUT + GNN_O * GNN_H;
constexpr int64_t GNN_NPARAM = GNN_OFF_BOUT + GNN_O;
// BF16 copies of the message-layer weights, per layer [W_s | W_m] (64 x 128)
constexpr int GNN_KHID = 2 * GNN_H;
constexpr int64_t GNN_NBF16 = GNN_L * GNN_H * GNN_KHID;

// Device view of one camera graph and its activations.
struct GraphDev {
  int nc, ns;
  const int32_t *nbr_ptr, *nbr, *rev;
  float *X, *E, *w;            // [nc][F], [nc][45] upper of E, [ns] a_ij / A_i
  float *Z[GNN_L + 1], *H[GNN_L + 1], *M[GNN_L];  // [nc][GNN_H] each
  float *dO, *dH, *dZ, *dM;    // [nc][45], [nc][GNN_H] x 3
  double *loss_part, *loss;    // [nc], [1]
};

struct PcFeatureArgs {
  int nc;
  const int32_t *nbr_ptr, *nbr, *nbr_blk;
  const void* S;               // off-diagonal blocks, precision T
  const double* Linv;          // [nc][81] inverse Cholesky factors (lower)
  float *X, *E, *w;
  // inference: the input layer h0 = relu(W_in x + b_in) of each camera is
  // formed here too (FP32, as in training) into H0 [nc][GNN_H]; null: not
  const float* params;
  float* H0;
};

template <typename T> hipError_t launch_pc_features(const PcFeatureArgs&, hipStream_t);
hipError_t launch_gnn_forward(const GraphDev&, const float* params, hipStream_t);
// inference: BF16 matrix-core message layers from H[0] (formed by the feature
// kernel; weights converted once per parameter set)
hipError_t launch_gnn_weights_bf16(const float* params, short* Wb, hipStream_t);
hipError_t launch_gnn_forward_bf16(const GraphDev&, const float* params, const short* Wb, hipStream_t);
// loss, d loss / d outputs (training) or the preconditioner blocks
// M_i = Linv_i^T C_i C_i^T Linv_i (inference, Minv != nullptr)
hipError_t launch_gnn_output(const GraphDev&, const float* params, const double* Linv, double* Minv,
                             bool with_loss, hipStream_t);
hipError_t launch_gnn_backward(const GraphDev&, const float* params, float* grad, hipStream_t);
hipError_t launch_gnn_adam(int64_t n, float* params, const float* grad, float* m, float* v, int step,
                           float lr, float b1, float b2, float eps, float grad_scale, hipStream_t);

}  // namespace ba
