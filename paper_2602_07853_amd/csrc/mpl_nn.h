// Learned preconditioner network state (see mpl_nn.hip for the design).
//
// Parameter layout (FP32, flat): for each of the 21 layers in execution
// order (enc0a, enc0b, down0, enc1a, enc1b, down1, enc2a, enc2b, down2,
// bota, botb, up2, dec2a, dec2b, up1, dec1a, dec1b, up0, dec0a, dec0b, out)
// the weight W[tap][in channel][out channel] followed by the bias[out channel];
// taps of a k x k x k kernel are enumerated with the last axis fastest.
#pragma once
#include "mpl_internal.h"

#define NN_LAYERS 21
#define NN_WGRAD_CHUNK 4096

struct NNSampleStore;
struct NNState {
  DevBuf params, grad, adam_m, adam_v, wsw, act, gact, wpart, lpart, tmp;
  DevBuf csplit;  // FP32 partial sums of 3x3x3 layers split over input-channel chunks
  DevBuf dref;  // device scalar: mean diagonal over free nodes
  NNSampleStore* store = nullptr;
  // device flag: when nonzero the forward kernels return at once (set by the
  // solver once its iteration has converged or fallen back to Jacobi)
  const int32_t* skip = nullptr;
  size_t sw_fwd_off[NN_LAYERS] = {}, sw_bwd_off[NN_LAYERS] = {};
  // 3x3x3 layers: weights for the LDS-tiled kernel (forward, data gradient)
  size_t sw3_fwd_off[NN_LAYERS] = {}, sw3_bwd_off[NN_LAYERS] = {};
  // 3x3x3 layers with 16 output channels: weights for the register-blocked
  // kernel (forward when the layer has 16 outputs, data gradient when it has
  // 16 inputs; 0 = none)
  size_t sw3rr_fwd_off[NN_LAYERS] = {}, sw3rr_bwd_off[NN_LAYERS] = {};
  int box[3] = {0, 0, 0};
  size_t t_in = 0, t_out = 0, t_cat[3] = {0, 0, 0}, t_lay[NN_LAYERS] = {};
  size_t act_elems = 0;
  int64_t adam_t = 0;
  bool ready = false;
  bool lds_conv = true;  // 3x3x3 layers on the LDS-tiled kernel (MPL_NN_DIRECT_CONV=1: direct kernel)
  bool rr_conv = true;   // 16-output-channel 3x3x3 layers on the register-blocked kernel (MPL_NN_RR_CONV=0: off)
  int rr_grid = 0;       // workgroups of the register-blocked kernel (resident on the device at once)
  int lds_grid[4] = {0, 0, 0, 0};  // the same for the LDS-tiled kernel, CT = 1, 2, 4, 8
};

int64_t nn_param_count();
NNState* nn_state(mpl_ctx* c);
void nn_destroy(mpl_ctx* c);
mpl_status nn_forward(mpl_ctx* c, NNState& nn);
mpl_status nn_backward(mpl_ctx* c, NNState& nn);
mpl_status nn_backward_update(mpl_ctx* c, NNState& nn, float lr);

// ---- the network as a preconditioner on the solver grid ----
double nn_inv_free_dofs(mpl_ctx* c);
// The box covers all grid nodes (voxel (i,j,k) = node (i,j,k)), each axis
// padded to a multiple of 8.  Input channels: 0-2 = sqrt(Dinv) r / s,
// 3 = log(Dmean_i / Dref), 4 = 1 on free nodes; output channels 0-2 = o,
// and the preconditioner is z = Dinv r + s sqrt(Dinv) o on free nodes, with
// s^2 = sum_free Dinv r^2 / (free DOFs).
struct NNSampleStore {
  DevBuf feat;    // [n][voxels][16] bf16
  DevBuf target;  // [n][voxels][3] f32
  DevBuf mask;    // [n][voxels] f32
  int count = 0, capacity = 0;
  int64_t voxels = 0;
};
mpl_status nn_prepare_box(mpl_ctx* c, bool train);
mpl_status nn_set_dref(mpl_ctx* c, const double* Dinv);
// stage features of r into the network input; s2 = device scalar sum Dinv r^2
mpl_status nn_stage_features(mpl_ctx* c, const double* r, const double* Dinv, const double* s2);
// record a training pair from (r, e = xstar - x): features of r, target
// sqrt(D)(e - Dinv r)/s, mask of free nodes
mpl_status nn_record_sample(mpl_ctx* c, const double* r, const double* x, const double* xstar,
                            const double* Dinv, const double* s2);
NNSampleStore& nn_samples(mpl_ctx* c);
// stage the network's output gradient from a node vector (block layout)
mpl_status nn_stage_output_grad(mpl_ctx* c, const double* g);
// stage a caller-given network output (box layout [X][Y][Z][16], FP32,
// rounded to BF16) in place of the forward's output
mpl_status nn_stage_output_f32(mpl_ctx* c, const float* o_box);
// one Adam step with the parameter gradient in nn.grad, then the refresh
// of the BF16 weight copies
mpl_status nn_adam_update(mpl_ctx* c, NNState& nn, float lr);
