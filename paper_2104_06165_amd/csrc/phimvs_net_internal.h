// Kernel-argument blocks and launchers of the learned-proposal network (not part of the
// public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace phimvs_net_internal {

constexpr int kMaxCO = 32;  // widest layer (output channels, padded)

// one 3x3 convolution (zero padding), NHWC bf16 activations
struct ConvArgs {
  int B, h, w;               // images, rows, columns
  int CI, CO;                // input / output channels (multiples of 16, CO <= kMaxCO)
  const uint16_t* x;         // B*h*w*CI bf16
  const uint16_t* wt;        // [9][CO][CI] bf16
  const float* bias;         // n_bias values or null (channels co >= n_bias get no bias)
  int n_bias;
  int relu;
  const uint16_t* mask16;    // B*h*w*CO bf16 or null: zero the output where mask <= 0
  uint16_t* y16;             // B*h*w*CO bf16 or null
  float* y32;                // B*h*w*co_keep fp32 or null
  int co_keep;
};

// weight gradient of one convolution, as per-image-row partial sums
struct WgradArgs {
  int B, h, w, CI, CO;
  const uint16_t* x;         // layer input, B*h*w*CI bf16
  const uint16_t* g;         // output gradient, B*h*w*CO bf16
  float* partial;            // [B*h][9][CI][CO]
  float* partial_bias;       // [B*h][CO] or null
};

struct LossArgs {
  int n_pix, h, w;           // n_pix = B*h*w
  const float* out;          // network output, n_pix*4
  const float* target;       // n_pix*4 (depth, normal)
  const float* mask;         // n_pix
  const float* drange;       // B*2
  float inv_count;           // loss normaliser (1 / n_pix)
  float lambda;              // normal-term weight
  uint16_t* grad16;          // n_pix*16 bf16 output gradient (channels >= 4 zero)
  float* loss_partial;       // one per 256-pixel block
};

struct ProposalInputs {
  int W, H, w, h;            // reference size and network input size (ceil(W/4), ceil(H/4))
  const __half* ref;         // reference grey values H*W
  const uint32_t* quad[4];   // source texel quads (null: channel stays 0)
  int sw[4], sh[4];          // source sizes
  float Hmid[36];            // per source: reference pixel -> source pixel, fronto-parallel plane at mid depth
  float* out;                // h*w*5
};

struct ProposalDecode {
  int W, H, w, h;
  const float* net_out;      // h*w*4
  float Kinv[9];
  float d_lo, d_hi;
  float* planes;             // H*W*4
};

struct TargetArgs {
  int W, H, w, h;
  const float* depth;        // H*W
  const float* normal;       // H*W*3
  const float* cost;         // H*W
  float max_cost;
  float* target;             // h*w*4
  float* mask;               // h*w
};

hipError_t launch_conv(const ConvArgs& a, hipStream_t st);
hipError_t launch_wgrad(const WgradArgs& a, hipStream_t st);
hipError_t launch_reduce_rows(const float* partial, int n_rows, int stride, int n, float* out, hipStream_t st);
hipError_t launch_to_bf16(const float* x, int n_pix, int C0, int CP, uint16_t* y, hipStream_t st);
// bf16 NHWC with CP channels -> float32 NHWC with the first C channels
hipError_t launch_bf16_unpad(const uint16_t* x, int n_pix, int CP, int C, float* y, hipStream_t st);
hipError_t launch_pack_weights(const float* w, int CIN, int COUT, int CIP, int COP, uint16_t* fwd, uint16_t* flip,
                               hipStream_t st);
// padded gradient gp [9][CIP][COP] (+ bias gb[COP]) -> flat [9][CIN][COUT] then [COUT]
hipError_t launch_unpad_grad(const float* gp, const float* gb, int CIN, int COUT, int CIP, int COP, float* g,
                             hipStream_t st);
hipError_t launch_loss(const LossArgs& a, hipStream_t st);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t st);
hipError_t launch_proposal_inputs(const ProposalInputs& a, hipStream_t st);
hipError_t launch_proposal_decode(const ProposalDecode& a, hipStream_t st);
hipError_t launch_targets(const TargetArgs& a, hipStream_t st);

}  // namespace phimvs_net_internal
