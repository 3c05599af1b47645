/*
 * phimvs_net.h — C ABI of the learned initial-plane proposal.
 *
 * The random initialisation of the depth-map search (paper Sec. III-B: random depth in
 * the depth range, random normal) can be replaced per pixel by a plane predicted by a
 * small convolutional network; the paper notes that a good initialisation speeds up
 * convergence (Sec. III-B) but proposes no network, so the network below is this
 * library's own addition.  The plain method's cost decides: a pixel keeps the
 * proposed plane only when its matching cost (Eq. 5) is not higher than that of its
 * random plane, and the random plane is kept otherwise.
 *
 * Network: 5 layers of 3x3 convolutions with zero padding, 5 -> 32 -> 32 -> 32 -> 32 -> 4
 * channels, ReLU after the first four; bfloat16 weights and activations, FP32
 * accumulation on the matrix cores.  It runs at 1/4 of the reference resolution
 * (h = ceil(H/4), w = ceil(W/4)).
 *   input  (h*w*5, float32, NHWC): channel 0 the mean of the 4x4 reference block,
 *          channels 1..4 the four sources closest to the reference camera sampled
 *          (bilinear) where the block centre (4X + 1.5, 4Y + 1.5) maps under the
 *          homography of the fronto-parallel plane at the middle of the depth range (0
 *          outside a source); grey values g enter as (g - 127.5) / 64.
 *   output (h*w*4, float32): o0 gives depth d_lo + (d_hi - d_lo) sigmoid(o0); (o1, o2, o3)
 *          normalised is the normal (turned to face the camera).
 *   Full-resolution planes are the bilinear interpolation of the four outputs at
 *   ((x - 1.5) / 4, (y - 1.5) / 4), clamped to the grid, then decoded as above.
 *
 * Parameters: a flat float32 vector, layer by layer, each layer's weights w[9][cin][cout]
 * (tap t = 3 (dy + 1) + (dx + 1) reads the input at (x + dx, y + dy)) followed by its
 * biases b[cout]; phimvs_net_param_count gives the length (30,372).
 *
 * Training: loss over the pixels with mask 1 of
 *   |log d - log d_target| + normal_weight (1 - n . n_target),
 * summed and divided by the number of pixels (masked or not); Adam on FP32 master
 * weights, bfloat16 copies for the matrix cores.
 *
 * Memory and errors follow phimvs.h: arrays marked "device" are device pointers on the
 * network's device; calls are issued on the network's stream and return PHIMVS_OK or a
 * negative PHIMVS_E_* code with a message readable by phimvs_net_last_error.
 */
#ifndef PHIMVS_NET_H
#define PHIMVS_NET_H

#include <stdint.h>

#include "phimvs.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PHIMVS_NET_IN 5
#define PHIMVS_NET_OUT 4
#define PHIMVS_NET_WIDTH 32
#define PHIMVS_NET_LAYERS 5

typedef struct phimvs_net phimvs_net;

/* Create a network with all parameters zero on HIP device `device_ordinal`, issuing
 * work on `hip_stream` (NULL = null stream). */
int phimvs_net_create(phimvs_net** out, int device_ordinal, void* hip_stream);
void phimvs_net_destroy(phimvs_net* net);
const char* phimvs_net_last_error(const phimvs_net* net);
int phimvs_net_set_stream(phimvs_net* net, void* hip_stream);
int64_t phimvs_net_param_count(void);

/* Replace / read the FP32 master parameters (layout above; host or device).  Setting
 * parameters resets the Adam state. */
int phimvs_net_set_params(phimvs_net* net, const float* params, int on_device);
int phimvs_net_get_params(phimvs_net* net, float* params, int on_device);

/* Forward pass of `batch` inputs of h x w (device, batch*h*w*5) into device outputs
 * (batch*h*w*4). */
int phimvs_net_forward(phimvs_net* net, int batch, int height, int width, const float* input, float* output);

/* Loss and its gradient with respect to every parameter, for device inputs
 * (batch*h*w*5), targets (batch*h*w*4: depth, normal), mask (batch*h*w) and depth
 * ranges (batch*2: d_lo, d_hi).  The gradient is kept for phimvs_net_adam; if `grad`
 * (device, param_count floats) is given it is copied there too.  If `loss` is given the
 * call waits for the result. */
int phimvs_net_loss_grad(phimvs_net* net, int batch, int height, int width, const float* input,
                         const float* target, const float* mask, const float* depth_range,
                         float normal_weight, double* loss, float* grad);

/* Test and inspection hook: copy a tensor the last pass stored on the device, bfloat16
 * widened to float32, padding channels dropped, into `out` (device, batch*h*w*C NHWC).
 * kind 0: the activation entering layer `layer` (0 .. PHIMVS_NET_LAYERS-1; layer 0's is
 * the bfloat16 input, C = PHIMVS_NET_IN, else C = 32), after phimvs_net_forward or
 * phimvs_net_loss_grad; kind 1: the gradient of the loss at the output of layer `layer`
 * (C = 32, or PHIMVS_NET_OUT for the last layer, whose gradient is the loss's own), after
 * phimvs_net_loss_grad.  PHIMVS_E_STATE before such a pass, PHIMVS_E_ARG for another kind
 * or layer. */
int phimvs_net_tensor(phimvs_net* net, int kind, int layer, float* out);

/* One Adam step (Kingma & Ba) with the gradient of the last phimvs_net_loss_grad. */
int phimvs_net_adam(phimvs_net* net, float lr, float beta1, float beta2, float eps);

/* Network input of reference `ref` (views of `ctx`, set by phimvs_set_views): the four
 * sources of `srcs` closest to the reference camera (fewer if n_srcs < 4; missing
 * channels are 0).  input: device, ceil(H/4)*ceil(W/4)*5. */
int phimvs_net_inputs(phimvs_ctx* ctx, phimvs_net* net, int ref, const int* srcs, int n_srcs, float* input);

/* Proposal planes of reference `ref`: input, forward pass, decode and upsampling into
 * `planes` (device, H*W*4 in the planes layout of phimvs.h). */
int phimvs_net_propose(phimvs_ctx* ctx, phimvs_net* net, int ref, const int* srcs, int n_srcs,
                       float* planes);

/* Decode a network output (device, ceil(H/4)*ceil(W/4)*4) of reference `ref` into
 * full-resolution planes (device, H*W*4). */
int phimvs_net_decode(phimvs_ctx* ctx, phimvs_net* net, int ref, const float* output, float* planes);

/* Training targets from a full-resolution depth-map result of size W x H (device:
 * depth H*W, normal H*W*3, cost H*W): block (X, Y) takes the 2 x 2 pixels around its
 * centre; mask 1 iff all four have depth > 0 and cost < max_cost; target depth is
 * their mean depth and target normal their normalised mean normal.  target: device
 * ceil(H/4)*ceil(W/4)*4, mask: device ceil(H/4)*ceil(W/4). */
int phimvs_net_targets(phimvs_net* net, int width, int height, const float* depth, const float* normal,
                       const float* cost, float max_cost, float* target, float* mask);

/* Depth-map estimation as phimvs_patchmatch, with the random initialisation gated by
 * proposal planes (planes layout, H*W*4; device if on_device): each pixel starts from
 * the proposal when its cost is not higher than its random plane's. */
int phimvs_patchmatch_proposal(phimvs_ctx* ctx, int ref, const int* srcs, int n_srcs, int window,
                               int dilation, int iters, const phimvs_params* p, const float* proposal,
                               float* depth, float* normal, float* cost, int on_device);

#ifdef __cplusplus
}
#endif

#endif /* PHIMVS_NET_H */
