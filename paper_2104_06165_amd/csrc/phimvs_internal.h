// Internal kernel-argument blocks and launchers shared by the host library and the
// kernels of the PatchMatch library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "phimvs.h"

namespace phimvs_internal {

// one source view as the kernels see it
struct SrcDev {
  float M[9];           // K_j R_rel K_0^-1
  float e[3];           // K_j t_rel
  float Wm1, Hm1;       // last valid sample position
  int W, H;
  const uint32_t* quad; // W*H 8-bit texel quads
};

// problem block, passed by value (kernel arguments live in the constant path)
struct Args {
  int W, H, Wc;         // reference size, colour-plane width ceil(W/2)
  int R, s;             // tap radius (taps per side 2R+1) and dilation
  int n_src, top_k, bilateral;
  int TW, TH, n_taps;   // LDS tile width/height, (2R+1)^2
  float Kinv[9];
  double Kinv_d[9];
  float d_lo, d_hi, eps_v, eps_c;
  uint32_t seed_lo, seed_hi;
  const __half* ref;    // reference grey values, H*W
  const float* wcol;    // 256 colour weights
  const float* wsp;     // n_taps spatial weights
  float4* plane[2];     // colour planes (n.x, n.y, n.z, d), H*Wc each
  float* cost[2];
  SrcDev src[PHIMVS_MAX_SOURCES];
};

// per-launch step arguments
struct Step {
  int colour, iteration, ncand;
  float4* cand;             // candidate planes, slot-major (slot k at cand + k * H * Wc)
  const float* planes_in;   // init: optional proposal; evaluation: planes to evaluate (row-major H*W*4)
  float* cost_out;          // MODE 2
  float* per_view_out;      // MODE 2, optional H*W*n_src
  uint8_t* valid_out;       // MODE 2, optional H*W*n_src
  unsigned long long* count;  // optional: + number of (pixel, hypothesis) pairs scored
};

// mode 0: initialise, 1: update from candidates, 2: evaluate input planes
hipError_t launch_select(int mode, const Args& A, const Step& S, hipStream_t st);
// kind 0: random initialisation (+ proposal), 1: propagation, 2: refinement candidates
hipError_t launch_candidates(int kind, const Args& A, const Step& S, hipStream_t st);
hipError_t launch_build_view(const uint8_t* img, int64_t stride, int W, int H, __half* plain, uint32_t* quad,
                             hipStream_t st);
hipError_t launch_unpack(const Args& A, float* planes, float* depth, float* normal, float* cost, hipStream_t st);
hipError_t launch_pack(const Args& A, const float* planes, const float* cost, hipStream_t st);
hipError_t launch_rcp_check(uint32_t first, uint32_t count, unsigned long long* mism, uint32_t* example,
                            hipStream_t st);

}  // namespace phimvs_internal
