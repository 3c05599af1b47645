/*
 * phimvs.h — C ABI of the MI355X (gfx950) PatchMatch multi-view stereo library.
 *
 * The library computes, for each pixel x of a reference image, a plane hypothesis
 * (depth d_x, normal n_x) from the reference image, a set of source images and their
 * cameras: the "depth map estimation" step of PHI-MVS (paper Sec. III intro, Sec.
 * III-B, Sec. III-C, Algorithm 1).  Hypotheses are scored by the weighted ZNCC of a
 * dilated support window (Eq. 4) warped into each source by the plane-induced
 * homography, aggregated over the best-K sources (Eq. 5), and searched by random
 * initialisation, red/black checkerboard propagation and random refinement.
 *
 * Conventions
 *   - Images are row-major, pixel (x, y) at column x, row y; pixel centres sit at
 *     integer coordinates.  8-bit grey values (PHIMVS_U8) are the supported input:
 *     every workload here is 8-bit imagery, whose values FP16 and FP32 hold exactly,
 *     so FP16 or FP32 input would add no precision; other dtypes fail with
 *     PHIMVS_E_UNSUPPORTED.
 *   - Cameras map world to camera: X_cam = R X_world + t.  K is 3x3 with last row
 *     (0, 0, 1).  All camera matrices are row-major doubles.
 *   - Depth is the reference camera's Z.  Normals are in the reference camera frame,
 *     facing the camera (n . K^-1 (x, y, 1) < 0).
 *   - Outputs are row-major: depth H*W, normal H*W*3, cost H*W (float32).  Pixels
 *     whose reference window leaves the image are invalid: depth 0, normal 0,
 *     cost PHIMVS_COST_MAX.
 *   - "planes" arrays are H*W*4 float32 (n.x, n.y, n.z, d) per pixel, row-major.
 *   - Limits (beyond them calls fail with PHIMVS_E_UNSUPPORTED): images below 2^28
 *     pixels; at most PHIMVS_MAX_SOURCES source views per reference; at most 31 taps
 *     per window side and a window radius (dilation x taps per side from the centre)
 *     of at most 30 px, 29 px with the window-resize scheme.
 *
 * Ownership and memory
 *   - The caller owns every buffer it passes.  phimvs_set_views copies the images
 *     (host or device) into library-owned device memory; the caller may free its
 *     copies on return.
 *   - Arguments with an "on_device" flag are device pointers (on the context's
 *     device) when the flag is non-zero, host pointers otherwise.  Device outputs are
 *     written asynchronously on the context's stream; host outputs are complete when
 *     the call returns.
 *
 * Errors and threading
 *   - Every int-returning call returns PHIMVS_OK (0) or a negative PHIMVS_E_* code and
 *     then sets a message readable with phimvs_last_error.  No exception crosses the
 *     ABI.  A context is not thread-safe: use one context per host thread / stream.
 */
#ifndef PHIMVS_H
#define PHIMVS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PHIMVS_COST_MAX 2.0f /* C_max = 1 - Z_min with Z_min = -1 (Sec. III-C, Eq. 5) */
#define PHIMVS_MAX_SOURCES 12

enum {
  PHIMVS_OK = 0,
  PHIMVS_E_ARG = -1,         /* invalid argument (message names it)                 */
  PHIMVS_E_STATE = -2,       /* call out of order (e.g. step before prepare)         */
  PHIMVS_E_DEVICE = -3,      /* HIP runtime error                                    */
  PHIMVS_E_OOM = -4,         /* device allocation failed                             */
  PHIMVS_E_UNSUPPORTED = -5  /* valid request the library does not implement         */
};

enum { PHIMVS_U8 = 0 };

typedef struct phimvs_ctx phimvs_ctx;

/* One input image.  stride_bytes = 0 means tightly packed rows. */
typedef struct {
  int32_t width, height;
  int64_t stride_bytes;
  int32_t dtype;       /* PHIMVS_U8 */
  const void* data;
  int32_t on_device;   /* non-zero: data is a device pointer */
} phimvs_image;

/* Solver parameters (Sec. III-C); phimvs_default_params fills the defaults. */
typedef struct {
  int32_t top_k;            /* Eq. 5 over the K lowest-cost valid sources; 0 = all (the paper's Eq. 5) */
  int32_t bilateral;        /* 0: weight 1 on every tap (Eq. 4 exactly); 1: bilateral weights           */
  double sigma_spatial_px;  /* bilateral spatial sigma in full-resolution px; <= 0: window radius        */
  double sigma_color;       /* bilateral colour sigma in grey levels (default 12)                      */
  double eps_var;           /* a patch with weighted variance below this is invalid (default 1e-4)     */
  double eps_cost;          /* per-source cost floor in the inverse weights of Eq. 5 (default 1e-4)    */
  uint64_t seed;            /* Philox4x32-10 key for the random draws (default 0x5EED)                 */
  int32_t tap_radius;       /* 0: taps x + s k, k = -r..r (integer dilation s).  > 0: the window-resize
                               scheme (Sec. III-C, Table III): r_now = tap_radius taps per side spread
                               over the window's radius r_orig = (window - 1) / 2 at spacing
                               r_orig / r_now (not necessarily an integer), reference values
                               interpolated bilinearly, the colour weight taken at the nearest integer
                               grey difference; needs dilation 1 and r_now <= r_orig (default 0)       */
  int32_t lanes;            /* 0 or 1: one lane scores a pixel's hypothesis, its taps summed in order.
                               2, 4, 8 or 16: G lanes share each pixel, lane g summing the taps
                               t = g, g + G, ... and the lanes' partial sums combined by an xor
                               butterfly (offsets G/2 .. 1).  For small references, whose pixels
                               alone do not fill the GPU; the order of the sums is part of the
                               result (it changes the FP32 rounding only).  Single-job calls only
                               (a batch job with lanes > 1, or combined with tap_radius > 0, fails
                               with PHIMVS_E_UNSUPPORTED) (default 0)                              */
  int32_t score_all;        /* 0: propagation candidates that cannot win are left out unscored: one
                               equal to an earlier candidate of the pixel, to its current plane, or to
                               a candidate the previous propagation of its colour offered it (each has
                               a cost no lower than the pixel's stored cost, and only a strictly lower
                               cost is taken, so no result changes).  1: all but the last kind are left
                               out.  2: every candidate is scored.  Results are bitwise the same under
                               every setting; only the work differs (default 0)                     */
} phimvs_params;

void phimvs_default_params(phimvs_params* p);

/* Create a context on HIP device `device_ordinal`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context.  Creation also
 * raises the evaluate kernel's dynamic-LDS limit on that device (so that no launch
 * changes a kernel attribute, which a stream capture could not record); it fails with
 * PHIMVS_E_DEVICE when the device does not report its LDS size. */
int phimvs_create(phimvs_ctx** out, int device_ordinal, void* hip_stream);
void phimvs_destroy(phimvs_ctx* ctx);
const char* phimvs_last_error(const phimvs_ctx* ctx);
/* Re-target the context's stream (e.g. the caller's current stream). */
int phimvs_set_stream(phimvs_ctx* ctx, void* hip_stream);
/* Block until all work issued on the context's stream has finished. */
int phimvs_sync(phimvs_ctx* ctx);

/* Upload the images and cameras of a scene (paper Sec. III: "images and camera
 * parameters" are the input).  K, R: n_views*9; t: n_views*3; depth_range:
 * n_views*2 (d_lo, d_hi per view, used when that view is the reference; requires
 * 0 < d_lo < d_hi).  Replaces any previous scene. */
int phimvs_set_views(phimvs_ctx* ctx, int n_views, const phimvs_image* images, const double* K,
                     const double* R, const double* t, const double* depth_range);

/* Full depth-map estimation of view `ref` against sources `srcs` (Algorithm 1
 * "depth map estimation": random initialisation, then `iters` x (red half-sweep,
 * black half-sweep), each half-sweep = propagation then random refinement).
 * window: odd side length in full-resolution px; dilation: tap stride s with
 * (window - 1) % (2 s) == 0, so taps are x + s k, k = -r..r, r = (window-1)/(2 s)
 * (Sec. III-C, dilated matching window).  p = NULL uses the defaults.  Outputs as
 * described above, on device if out_on_device. */
int phimvs_patchmatch(phimvs_ctx* ctx, int ref, const int* srcs, int n_srcs, int window, int dilation,
                      int iters, const phimvs_params* p, float* depth, float* normal, float* cost,
                      int out_on_device);

/* ---- step-wise interface (the same computation, one stage at a time) ---- */

/* Fix the problem for the calls below and allocate its state. */
int phimvs_prepare(phimvs_ctx* ctx, int ref, const int* srcs, int n_srcs, int window, int dilation,
                   const phimvs_params* p);
/* Random initialisation (Sec. III-B) of every valid pixel, with its cost.  If
 * `proposal` (planes layout) is given, each pixel keeps the proposal instead of its
 * random plane when the proposal's cost is not higher (learned-initialisation gate). */
int phimvs_init_planes(phimvs_ctx* ctx, const float* proposal, int on_device);
/* One half-sweep: propagation from the other colour then random refinement (Sec.
 * III-C) of colour `colour` (0: red, (x + y) even; 1: black) at iteration
 * `iteration` (>= 1; it keys the random draws).  do_propagate / do_refine select
 * the two stages (both 1 in the full method). */
int phimvs_step(phimvs_ctx* ctx, int iteration, int colour, int do_propagate, int do_refine);
/* Read / overwrite the current state (planes layout + cost H*W). */
int phimvs_get_state(phimvs_ctx* ctx, float* planes, float* cost, int on_device);
int phimvs_set_state(phimvs_ctx* ctx, const float* planes, const float* cost, int on_device);
/* Write depth / normal / cost of the current state (output layout). */
int phimvs_output(phimvs_ctx* ctx, float* depth, float* normal, float* cost, int on_device);
/* Cost (Eq. 5) of the given planes at every pixel; per_view (H*W*n_srcs, or NULL)
 * receives each source's 1 - Z (PHIMVS_COST_MAX when that source is invalid) and
 * valid (H*W*n_srcs bytes, or NULL) its validity flag.  A plane whose depth is NaN
 * fails the border rule in every source: cost PHIMVS_COST_MAX, every source invalid
 * (written without evaluating the window). */
int phimvs_eval_cost(phimvs_ctx* ctx, const float* planes, float* cost, float* per_view, uint8_t* valid,
                     int on_device);

/* ---- batches of reference views ---- */

/* One depth map of a batch: reference view, its sources, window / dilation as for
 * phimvs_patchmatch, and device outputs (depth H*W, normal H*W*3, cost H*W; any may be
 * NULL).  srcs is read during the call only. */
typedef struct {
  int32_t ref;
  const int32_t* srcs;
  int32_t n_srcs;
  int32_t window, dilation;
  phimvs_params params;
  float* depth;
  float* normal;
  float* cost;
} phimvs_job;

/* Depth-map estimation of every job of the batch in shared launches: each phase
 * (initialisation, a colour's propagation, a colour's refinement) is one launch over
 * the tiles of all jobs, so references of different sizes and source counts share the
 * GPU.  With use_graph != 0 the whole launch sequence is captured once into a hipGraph
 * (per batch geometry, iteration count and tuning) and replayed on later calls.  Work
 * is issued on the context's stream; outputs are complete when that stream is.  Each
 * job's result equals its own phimvs_patchmatch result. */
int phimvs_patchmatch_batch(phimvs_ctx* ctx, int n_jobs, const phimvs_job* jobs, int iters, int use_graph);

/* Launch configuration of the evaluate-and-select kernel: tile_rows (4, 2 or 1) rows of
 * 256 / tile_rows same-colour pixels per workgroup; persistent != 0 runs a fixed grid
 * of wgs_per_cu workgroups per compute unit pulling tiles from per-XCD queues, else
 * one workgroup per tile; order_by_depth, a mask of 1 (initialisation), 2 (propagation)
 * and 4 (refinement), hands those launches' (pixel, candidate) work items to the lanes in
 * order of the candidate's inverse depth instead of pixel order (results are the same
 * either way; it pays where the candidates' depths scatter the source gathers most, as
 * with converging cameras; the split-lane path of phimvs_params.lanes > 1 has no work list
 * and ignores it).  ms is the time measured by
 * phimvs_autotune.  A new context starts with tile_rows 4, persistent, 4 workgroups per
 * compute unit, pixel order. */
typedef struct {
  int32_t tile_rows;
  int32_t persistent;
  int32_t wgs_per_cu;
  int32_t order_by_depth;
  double ms;
} phimvs_tuning;

int phimvs_set_tuning(phimvs_ctx* ctx, const phimvs_tuning* t);
int phimvs_get_tuning(phimvs_ctx* ctx, phimvs_tuning* t);
/* Time every built-in configuration on the given batch (graph replays, `iters`
 * iterations: ten launch shapes in pixel order, then the fastest of them again with
 * order_by_depth = 7), keep the fastest in the context and report all of them in results
 * (capacity *n_results, updated to the number written).  A configuration that fails to
 * run is reported with ms = +inf and passed over (phimvs_last_error then names it); when
 * none runs, the previous configuration is restored and PHIMVS_E_DEVICE returned. */
int phimvs_autotune(phimvs_ctx* ctx, int n_jobs, const phimvs_job* jobs, int iters, phimvs_tuning* results,
                    int* n_results);

/* ---- geometric-consistency filter ---- */

/* A depth-map result of one view of the context's scene (device arrays of that view's
 * size: depth H*W, normal H*W*3; depth <= 0 marks a pixel without depth). */
typedef struct {
  int32_t view;
  const float* depth;
  const float* normal;
} phimvs_depth_map;

/* Thresholds of the consistency test (Sec. III-D): relative depth difference, normal
 * angle (degrees), re-projection error (pixels), and the number of consistent
 * neighbours a pixel needs to be kept (the paper: more than one).  Defaults 0.02, 30, 1, 2. */
typedef struct {
  double max_rel_depth;
  double max_angle_deg;
  double max_reproj_px;
  int32_t min_consistent;
} phimvs_filter_params;

void phimvs_default_filter_params(phimvs_filter_params* p);

/* Geometric-consistency filter of maps[ref_map] against the maps listed in nbrs (indices
 * into maps, at most PHIMVS_MAX_SOURCES, none equal to ref_map), Sec. III-D: each pixel
 * x with depth d is back-projected, projected into every neighbour view j and compared
 * with view j's map there: the depths agree when |z_j(X) - d'| < max_rel_depth d' (d' the
 * bilinear depth of view j, z_j(X) the point's depth in camera j), the normals when the
 * angle between them (world frame; view j's normal at the rounded position) is below
 * max_angle_deg, and view j's point at d' must re-project within max_reproj_px of x.  A
 * neighbour is not consistent when the projection leaves its image, lies behind it or
 * touches a texel without depth.  Outputs (device, reference size): depth and normal
 * kept or zeroed, and the count of consistent neighbours per pixel (uint8).  All
 * arithmetic is FP64.  p = NULL uses the defaults. */
int phimvs_filter(phimvs_ctx* ctx, int n_maps, const phimvs_depth_map* maps, int ref_map, const int32_t* nbrs,
                  int n_nbrs, const phimvs_filter_params* p, float* depth_out, float* normal_out,
                  uint8_t* count_out);

/* ---- depth-map fusion (Sec. III-F) ---- */

/* Merge threshold: a pixel of a later map joins a point when its back-projection lies
 * within max_rel_dist d of the point's first pixel's back-projection X (Euclidean
 * distance; d the depth of X in its own camera).  Default 0.01. */
typedef struct {
  double max_rel_dist;
} phimvs_fuse_params;

void phimvs_default_fuse_params(phimvs_fuse_params* p);

/* Depth-map fusion into a point cloud, Sec. III-F.  The maps are processed in the order
 * given (maps[k].normal is not used and may be NULL).  For map i, each pixel that still
 * has depth (> 0) is back-projected to X; in every later map j, X is projected and
 * rounded to the nearest pixel q (floor(u + 1/2), floor(v + 1/2)); if q is in the image,
 * still has depth and its back-projection is within the threshold of X, q is deleted from
 * map j and joins the point; among the pixels of map i that qualify for the same q, the
 * first in row-major order takes it.  The point is the mean of X and the back-projections
 * it took (summed in map order); then map i is deleted, and the next map is processed.
 * Outputs (device arrays over the concatenated pixels of the maps, map k starting after
 * the H*W pixels of maps 0..k-1; caller-owned):
 *   points  (3 floats per pixel): the world-frame point at the pixel it started from, else 0;
 *   support (int32 per pixel): the number of pixels merged into that point, else 0;
 *   owner   (int64 per pixel): the concatenated index of the point the pixel ended in,
 *           -1 for pixels without depth.
 * All arithmetic is FP64.  Work is queued on the context's stream; the library keeps
 * scratch of 5 bytes per concatenated pixel.  p = NULL uses the default threshold. */
int phimvs_fuse(phimvs_ctx* ctx, int n_maps, const phimvs_depth_map* maps, const phimvs_fuse_params* p,
                float* points, int32_t* support, int64_t* owner);

/* ---- plane hypothesis inference (Sec. III-E) ----
 * Depth hypotheses for the pixels a filtered depth map leaves empty, their matching
 * costs, the selection of one hypothesis per pixel through a pairwise graph model (the
 * part the paper runs on the CPU, here too), and normals for the filled pixels. */

/* Four hypotheses per pixel without depth (depth <= 0): for each direction (horizontal,
 * vertical, 45 degrees below (1, 1), 45 degrees above (1, -1)) the value at the pixel of
 * the straight line fitted by least squares (depth against step index) to the six
 * pixels with depth closest along that line (both sides, fewer if the image ends; none
 * below two points or when the fitted depth is not positive).  depth: device H*W;
 * hyp: device, planar 4*H*W (hypothesis k of pixel p at hyp[k * H * W + p]), 0 = none.
 * FP64 fit.  Work is queued on the context's stream; the library keeps scratch of one bit
 * per pixel and direction ((4 W + 2 H) H / 8 bytes, rounded up to 64-bit words). */
int phimvs_phi_hypotheses(phimvs_ctx* ctx, int width, int height, const float* depth, float* hyp);
/* The same hypotheses, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): this call makes
 * no allocation.  Its bitmaps live in a static device array of 2^20 64-bit words (8 MiB)
 * that every GPU the library runs on holds until the process ends; maps needing more
 * ((4 W + 2 H) H / 8 bytes, rounded up to words; e.g. 3200 x 2130 needs 4.5 MiB) fail with
 * PHIMVS_E_UNSUPPORTED.  All calls on one GPU share that GPU's array: calls that overlap
 * on one GPU (contexts on different streams, or host threads) race and must be ordered by
 * the caller.  Arguments, outputs and errors as phimvs_phi_hypotheses; the results are
 * identical to it. */
int phimvs_phi_hypotheses_noalloc(phimvs_ctx* ctx, int width, int height, const float* depth, float* hyp);

/* Matching cost (Eq. 5, the prepared problem's cost) of every hypothesis: the fronto-
 * parallel plane at the hypothesis depth, i.e. every window point back-projected at that
 * depth and projected into the sources.  Needs phimvs_prepare of the same reference; the
 * hypotheses pass through the prepared problem's candidate slots (so only the present ones
 * are scored), which the next step overwrites anyway.  hyp, cost: device planar 4*H*W;
 * cost of an empty hypothesis, or of a pixel whose window leaves the image, is
 * PHIMVS_COST_MAX. */
int phimvs_phi_costs(phimvs_ctx* ctx, const float* hyp, float* cost);

typedef struct {
  double k1, k2, k3;   /* potentials of Eq. 7 and Eq. 8 (defaults 1, 0.1, 2)              */
  int32_t iterations;  /* message-passing sweeps of the decoder (default 8)                */
} phimvs_phi_params;

void phimvs_default_phi_params(phimvs_phi_params* p);

/* Selection (Sec. III-E): the hypothesis maps are subsampled to half size (node (X, Y)
 * takes pixel (2X, 2Y)), the graph model (node states = hypotheses with potential
 * (C_max - C) / k1 + k2, pixels with depth = fixed states, 4-connected edges with
 * [k3 - min(1, relative depth difference)]^2) is decoded on the host by sequential
 * tree-reweighted message passing (as phimvs_phi_decode_host), the decoded half-size
 * depth is brought back to full
 * size (pixel (x, y) takes node (x / 2, y / 2)) as the reference map, and each pixel
 * without depth takes its hypothesis closest to the reference (lowest k on ties; stays
 * empty without hypothesis or reference).  Pixels with depth keep it.  depth, depth_out:
 * device H*W; hyp, cost: device planar 4*H*W.  The half-size inputs are gathered on the
 * device (9 (W+1)/2 (H+1)/2 floats of the context's scratch), copied to the host, decoded
 * there, and the decoded map goes back for the last step.  Synchronises the stream.
 * PHIMVS_E_ARG also for a cost above C_max + k1 k2 at a sampled hypothesis (no positive
 * potential). */
int phimvs_phi_select(phimvs_ctx* ctx, int width, int height, const float* depth, const float* hyp,
                      const float* cost, const phimvs_phi_params* p, float* depth_out);

/* The graph-model decoder of phimvs_phi_select on host arrays (CPU only): depth H*W
 * (> 0: fixed node), hyp and cost planar 4*H*W; label_out receives the chosen hypothesis
 * (-1: fixed or no state) and depth_out its depth (0: no state).  Sequential TRW-S
 * (Kolmogorov 2006) in raster order, `iterations` forward and backward sweeps, then
 * labelling in raster order; the result is that of the plain sequential schedule bit for
 * bit, computed as wavefronts of tiles on up to 16 host threads (one for graphs under
 * 8192 nodes).  Returns PHIMVS_OK; PHIMVS_E_ARG for a null array, a size below 1, k1 <= 0,
 * k2 <= 0, k3 <= 1, iterations < 0 or a hypothesis whose potential (C_max - C) / k1 + k2
 * is not positive; PHIMVS_E_UNSUPPORTED for graphs of 2^27 nodes or more; PHIMVS_E_OOM when
 * host memory runs out. */
int phimvs_phi_decode_host(int width, int height, const float* depth, const float* hyp, const float* cost,
                           double k1, double k2, double k3, double cost_max, int iterations, int32_t* label_out,
                           float* depth_out);

/* Normals of Eq. 10 (normalised by the norm): n = (X_up - X_down) x (X_left - X_right)
 * of the back-projected 4-connected neighbours, turned to face the camera; 0 where the
 * pixel or a neighbour has no depth or lies on the border.  view: the view whose K the
 * depth map belongs to; depth device H*W, normal_out device H*W*3.  FP64. */
int phimvs_phi_normals(phimvs_ctx* ctx, int view, const float* depth, float* normal_out);

/* ---- diagnostics ---- */

/* flags: PHIMVS_DIAG_COUNT counts the (pixel, hypothesis) pairs the evaluate-and-select
 * kernels score; PHIMVS_DIAG_TIME brackets every evaluate-and-select launch with HIP
 * events on the context's stream.  Enabling resets both; 0 disables. */
enum { PHIMVS_DIAG_COUNT = 1, PHIMVS_DIAG_TIME = 2 };
int phimvs_diag_enable(phimvs_ctx* ctx, int flags);
/* Synchronise the stream and read the diagnostics gathered since enabling: hypotheses
 * scored, number of evaluate-and-select launches timed and their summed duration (ms).
 * Any pointer may be NULL. */
int phimvs_diag_read(phimvs_ctx* ctx, uint64_t* hypotheses, uint64_t* launches, double* kernel_ms);

/* ---- self-test ---- */

/* The kernels divide by the third homogeneous coordinate w of every warped tap with a
 * fast reciprocal that must equal the correctly rounded 1/w on [2^-100, 2^100] (the
 * kernels fall back to IEEE division outside it).  This compares that reciprocal with
 * the correctly rounded one on the float bit patterns [first_bits, first_bits + count)
 * and returns the number of mismatches (and one mismatching pattern). */
int phimvs_check_reciprocal(phimvs_ctx* ctx, uint32_t first_bits, uint32_t count, uint64_t* mismatches,
                            uint32_t* example_bits);

#ifdef __cplusplus
}
#endif

#endif /* PHIMVS_H */
