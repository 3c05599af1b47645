// Internal kernel-argument blocks and launchers shared by the host library and the
// kernels of the PatchMatch library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "phimvs.h"

namespace phimvs_internal {

constexpr int kBlock = 256;        // threads per evaluate workgroup
// evaluate kernel's compaction arrays in dynamic LDS, in floats: per pixel S_w, mu_a,
// var_a (3 kBlock), cost per (slot, pixel) (8 kBlock), the (pixel, slot) list as 16-bit
// entries (4 kBlock) and the waves' counts (8)
constexpr int kDepthBuckets = 256;  // inverse-depth buckets of the depth-ordered work list (one per thread)
static_assert(kDepthBuckets == kBlock, "the bucket scan gives each thread of the workgroup one bucket");
constexpr int kDepthBucketLds = 15 * kBlock + 8;  // their counters, after the wave totals
constexpr int kCompactLds = kDepthBucketLds + kDepthBuckets;
constexpr int kMaxTopK = PHIMVS_MAX_SOURCES;
constexpr int kMaxTaps1D = 31;     // taps per window side

// one source view as the kernels see it
struct SrcDev {
  float M[9];              // K_j R_rel K_0^-1
  float e[3];              // K_j t_rel
  float Wm1, Hm1;          // last valid sample position
  int W, H;
  const uint32_t* quad;    // W*H 8-bit texel quads
};

// one problem: a reference view, its sources and its solver state
struct Args {
  int W, H, Wc;            // reference size, colour-plane width ceil(W/2)
  int R, s;                // tap radius (taps per side 2R+1) and dilation
  int n_src, top_k, bilateral;
  int n_taps;              // (2R+1)^2
  int frac;                // window-resize scheme: interpolated reference taps at fractional offsets
  int rv;                  // validity radius: a pixel is valid when its window (x +- rv) is inside
  int halo;                // reference-tile halo in pixels
  int lanes;               // lanes sharing a pixel (1, or 2..16: split tap sums, single-job launches)
  int score_all;           // propagation candidates left out when they cannot win: 0 all such (equal
                           // to an earlier one, to the current plane, or to one the previous launch of
                           // the colour offered); 1 not the last kind; 2 none
  float off[kMaxTaps1D];   // tap offsets k = 0 .. 2R: s (k - R), in FP32
  float Kinv[9];
  double Kinv_d[9];
  float d_lo, d_hi, eps_v, eps_c;
  uint32_t seed_lo, seed_hi;
  const __half* ref;       // reference grey values, H*W
  const float* wcol;       // 256 colour weights
  const float* wsp;        // n_taps spatial weights
  float4* plane[2];        // colour planes (n.x, n.y, n.z, d), H*Wc each
  float* cost[2];
  SrcDev src[PHIMVS_MAX_SOURCES];
};

// a problem plus its place in the launch-wide work spaces
struct Job {
  Args A;
  float4* cand;            // candidate planes, slot-major: slot k at cand + k * H * Wc
  float4* hist[2];         // per colour: the 8 candidates the last propagation launch of that colour
                           // offered each pixel, slot-major like cand
  const float* planes_in;  // init: optional proposal; evaluation: planes to score (row-major H*W*4)
  float* cost_out;         // evaluation outputs (row-major)
  float* per_view_out;
  uint8_t* valid_out;
  float* depth_out;        // unpack outputs (row-major)
  float* normal_out;
  float* final_cost_out;
  float* planes_out;
  int tile0;               // first evaluate tile of this job
  int tiles_x, tiles_y;
  int xband[8];            // XCD k evaluates local tiles [xband[k], xband[k + 1]) (xband[8] = all tiles); whole tile rows
  int xoff[8];             // where that band starts in XCD k's list (bands of earlier jobs first)
  int cblk0;               // first candidate / unpack block of this job
  int cblk_x;              // blocks per row
};

// one launch over all jobs
struct Launch {
  int n_jobs;
  int colour, iteration, ncand, mode;  // mode 0: initialise, 1: update, 2: evaluate planes_in, 3: cost of
                                       // every candidate slot, written out
  int tile_rows;                       // rows of an evaluate tile (4, 2 or 1); 256 / tile_rows columns
  int total_tiles, total_cblk;
  int xcd_len[8];                      // evaluate tiles of each XCD's list
  int persistent;                      // evaluate: tiles pulled from per-XCD queues
  int order_by_depth;                  // evaluate: work items of launches with <= 3 candidates per
                                       // pixel handed out by the candidate's inverse depth
  int frac;                            // evaluate: some job uses the window-resize scheme
  int skip_current;                    // propagation candidates: drop those equal to the pixel's current
                                       // plane (only when every stored cost is its plane's own cost)
  int hist_mode;                       // propagation candidates: 0 none; 1 record the candidates offered;
                                       // 2 also drop those the previous launch of the colour offered
  unsigned int* queue;                 // 8 counters, zero at launch (persistent only)
  unsigned long long* count;           // optional: + (pixel, hypothesis) pairs scored
};

// launch-wide LDS need in bytes for the evaluate kernel
size_t eval_lds_bytes(int tile_rows, int max_radius_px, int max_taps);

// raise the evaluate kernel's dynamic-LDS limit on the current device (outside any stream
// capture); *max_dynamic receives the largest dynamic LDS a launch may then ask for
hipError_t eval_lds_setup(size_t* max_dynamic);
hipError_t launch_eval(const Job* d_jobs, const Launch& L, int grid, size_t lds, hipStream_t st);
// single-job evaluate launch with `lanes` (2, 4, 8, 16) lanes per pixel (job 0 of H rows,
// Wc compacted columns); its LDS need for a reference-tile halo and tap count
size_t eval_lanes_lds_bytes(int lanes, int radius_px, int n_taps);
hipError_t launch_eval_lanes(const Job* d_jobs, const Launch& L, int lanes, int H, int Wc, size_t lds,
                             hipStream_t st);
// kind 0: random initialisation (+ proposal), 1: propagation, 2: refinement candidates
hipError_t launch_candidates(int kind, const Job* d_jobs, const Launch& L, hipStream_t st);
// the 4 planar hypothesis maps hyp (4 W H) as candidate slots 0..L.ncand-1 of colour L.colour
hipError_t launch_hyp_candidates(const Job* d_jobs, const Launch& L, const float* hyp, hipStream_t st);
hipError_t launch_unpack(const Job* d_jobs, const Launch& L, hipStream_t st);
// row-major planes + cost -> the colour planes of job 0 (W x H)
hipError_t launch_pack(const Job* d_jobs, int W, int H, const float* planes, const float* cost, hipStream_t st);
hipError_t launch_zero(unsigned int* p, int n, hipStream_t st);
hipError_t launch_build_view(const uint8_t* img, int64_t stride, int W, int H, __half* plain, uint32_t* quad,
                             hipStream_t st);
hipError_t launch_rcp_check(uint32_t first, uint32_t count, unsigned long long* mism, uint32_t* example,
                            hipStream_t st);

// geometric-consistency filter: one neighbour view and the launch
struct FilterNbr {
  double K[9], Kinv[9], R[9], t[3];
  int W, H;
  const float* depth;
  const float* normal;
};
struct FilterArgs {
  int W, H;
  double K[9], Kinv[9], R[9], t[3];
  const float* depth;
  const float* normal;
  int n_nbrs;
  const FilterNbr* nbrs;  // device array of n_nbrs
  double tau_d, cos_n, tau_r;
  int min_consistent;
  float* depth_out;
  float* normal_out;
  uint8_t* count_out;
};
hipError_t launch_filter(const FilterArgs& a, hipStream_t st);

// depth-map fusion: one map's camera and depth, at offset `off` of the concatenated pixels
struct FuseMap {
  double K[9], Kinv[9], R[9], t[3];
  int W, H;
  int64_t off;
  const float* depth;
};
// the whole fusion of n_maps maps (h_maps on the host, d_maps its device copy); alive and
// claim: scratch over the concatenated pixels
hipError_t launch_fuse(const FuseMap* h_maps, const FuseMap* d_maps, int n_maps, double tau, uint8_t* alive,
                       int32_t* claim, float* points, int32_t* support, int64_t* owner, hipStream_t st);

// plane hypothesis inference
struct PhiCam {
  double Kinv[9];
};
// 64-bit words of the per-direction occupancy bitmaps of a W x H map (the fit's scratch)
size_t phi_bits_words(int W, int H);
// the allocation-free entry point's scratch: a static device array of kPhiScratchWords
// words per GPU; phi_scratch_setup looks up its device address on `device` (which must be
// current) once per device, phi_scratch_get returns it (no HIP call, no allocation)
constexpr size_t kPhiScratchWords = (size_t)1 << 20;
hipError_t phi_scratch_setup(int device);
hipError_t phi_scratch_get(int device, uint64_t** p);
hipError_t launch_phi_hypotheses(const float* depth, int W, int H, uint64_t* bits, float* hyp, hipStream_t st);
hipError_t launch_phi_mask_cost(const float* hyp, size_t n, float cmax, float* cost, hipStream_t st);
// node (X, Y) of the half-size graph from pixel (2X, 2Y): depth, 4 hypothesis planes, 4
// cost planes, one after the other in half (9 (W+1)/2 (H+1)/2 floats)
hipError_t launch_phi_half(const float* depth, const float* hyp, const float* cost, int W, int H, float* half,
                           hipStream_t st);
// dec: the decoded half-size depth ((W+1)/2 x (H+1)/2)
hipError_t launch_phi_select(const float* depth, const float* hyp, const float* dec, int W, int H, float* out,
                             hipStream_t st);
hipError_t launch_phi_normals(const float* depth, int W, int H, const PhiCam& cam, float* normal, hipStream_t st);

// a view of a context's scene, for the proposal network's host code
struct ViewInfo {
  int W, H;
  double K[9], R[9], t[3];
  double d_lo, d_hi;
  const __half* plain;     // grey values H*W
  const uint32_t* quad;    // texel quads H*W
};
int view_info(phimvs_ctx* c, int idx, ViewInfo* out);
int ctx_device(const phimvs_ctx* c);
hipStream_t ctx_stream(const phimvs_ctx* c);
int ctx_fail(phimvs_ctx* c, int code, const char* msg);

}  // namespace phimvs_internal
