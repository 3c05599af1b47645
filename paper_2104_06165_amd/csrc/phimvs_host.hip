// Host side of the PatchMatch library: the C ABI declared in phimvs.h.
//
// Responsibilities: argument validation, the FP64 per-problem constants (relative
// poses, M_j = K_j R_rel K_0^-1, e_j = K_j t_rel, K_0^-1, bilateral weight tables),
// device memory for views and solver state, the job table every kernel reads, and the
// launch sequence of the depth-map estimation step (Algorithm 1: initialisation, then
// per iteration a red and a black half-sweep, each propagation then refinement), issued
// eagerly or replayed from a captured hipGraph.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "phimvs.h"
#include "phimvs_internal.h"

using namespace phimvs_internal;

namespace {

struct ViewData {
  int W = 0, H = 0;
  double K[9], R[9], t[3];
  double d_lo = 0, d_hi = 0;
  __half* plain = nullptr;
  uint32_t* quad = nullptr;
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

// device state of one job
struct JobState {
  DevBuf<float4> plane[2];
  DevBuf<float> cost[2];
  DevBuf<float4> cand;
  DevBuf<float4> hist;           // 2 colours x 8 candidates per pixel
  DevBuf<float> wcol, wsp;
};

// a set of jobs with their table on the device and their launch geometry
struct Batch {
  std::vector<Job> jobs;         // host copy of the table
  std::vector<JobState> state;
  Job* d_jobs = nullptr;
  size_t d_cap = 0;
  int total_tiles = 0, total_cblk = 0, max_r = 0, max_taps = 0, tile_rows = 4;
  int xcd_len[8] = {};
  std::string layout_key;        // problems + tile shape the state was built for
  bool state_exact = false;      // every stored cost is the cost of its stored plane (the library's
                                 // own initialisation and steps keep this; phimvs_set_state does not)
  bool hist_valid[2] = {false, false};  // hist[c] holds the last propagation launch of colour c since the
                                        // state was initialised by the library (no phimvs_set_state since)
  // captured launch sequence
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string graph_key;
  DevBuf<unsigned int> queues;   // 8 counters per evaluate launch
  std::vector<unsigned char> uploaded;  // bytes of the table last copied to d_jobs
};

}  // namespace

struct phimvs_ctx {
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;  // private stream graphs are recorded on
  std::string err;
  std::vector<ViewData> views;
  bool prepared = false;
  Batch single;                   // the step-wise interface's job
  Batch multi;                    // phimvs_patchmatch_batch
  phimvs_tuning tuning{4, 1, 4, 0, 0.0};  // persistent, 4 workgroups per CU (the occupancy limit), pixel order
  size_t eval_lds_max = 0;                // largest dynamic LDS of an evaluate launch on this device
  DevBuf<float> io_a, io_b, io_c, io_d;  // staging for host inputs / outputs
  DevBuf<FilterNbr> filter_nbrs;          // neighbour table of the consistency filter
  std::vector<FilterNbr> filter_host;
  DevBuf<FuseMap> fuse_maps;              // fusion: map table, live flags and claims
  std::vector<FuseMap> fuse_host;
  DevBuf<uint8_t> fuse_alive;
  DevBuf<int32_t> fuse_claim;
  DevBuf<uint64_t> phi_bits;              // per-direction occupancy bitmaps of the hypothesis fits
  DevBuf<uint8_t> io_u8;
  // diagnostics
  int diag = 0;
  unsigned long long* diag_count = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> diag_events;
};

namespace {

int fail(phimvs_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHECK(ctx, call)                                                                        \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(ctx, e_ == hipErrorOutOfMemory ? PHIMVS_E_OOM : PHIMVS_E_DEVICE,                 \
                  std::string(#call) + ": " + hipGetErrorString(e_));                               \
  } while (0)

template <typename T>
int ensure(phimvs_ctx* c, DevBuf<T>& b, size_t n) {
  if (b.n >= n && b.p) return PHIMVS_OK;
  if (b.p) {
    HIPCHECK(c, hipFree(b.p));
    b.p = nullptr;
    b.n = 0;
  }
  HIPCHECK(c, hipMalloc((void**)&b.p, std::max<size_t>(n, 1) * sizeof(T)));
  b.n = n;
  return PHIMVS_OK;
}

template <typename T>
void release(DevBuf<T>& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.n = 0;
}

void release_graph(Batch& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.graph_key.clear();
}

void release_state(JobState& s) {
  for (int k = 0; k < 2; ++k) {
    release(s.plane[k]);
    release(s.cost[k]);
  }
  release(s.cand);
  release(s.hist);
  release(s.wcol);
  release(s.wsp);
}

// n job slots, freeing the device state of the slots dropped
void resize_jobs(Batch& b, size_t n) {
  for (size_t i = n; i < b.state.size(); ++i) release_state(b.state[i]);
  b.state.resize(n);
  b.jobs.resize(n);
}

void release_batch(Batch& b) {
  release_graph(b);
  resize_jobs(b, 0);
  b.layout_key.clear();
  if (b.d_jobs) (void)hipFree(b.d_jobs);
  b.d_jobs = nullptr;
  b.d_cap = 0;
  b.uploaded.clear();
  release(b.queues);
}

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// C = A B (3x3, row-major), summed left to right
void mul33(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i * 3 + 0] * B[0 * 3 + j] + A[i * 3 + 1] * B[1 * 3 + j] + A[i * 3 + 2] * B[2 * 3 + j];
}

void mulv3(const double* A, const double* v, double* o) {
  for (int i = 0; i < 3; ++i) o[i] = A[i * 3 + 0] * v[0] + A[i * 3 + 1] * v[1] + A[i * 3 + 2] * v[2];
}

// inverse through the adjugate (cofactors over the determinant)
bool inv33(const double* A, double* I) {
  const double c00 = A[4] * A[8] - A[5] * A[7];
  const double c01 = A[5] * A[6] - A[3] * A[8];
  const double c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  const double r = 1.0 / det;
  I[0] = c00 * r;
  I[1] = (A[2] * A[7] - A[1] * A[8]) * r;
  I[2] = (A[1] * A[5] - A[2] * A[4]) * r;
  I[3] = c01 * r;
  I[4] = (A[0] * A[8] - A[2] * A[6]) * r;
  I[5] = (A[2] * A[3] - A[0] * A[5]) * r;
  I[6] = c02 * r;
  I[7] = (A[1] * A[6] - A[0] * A[7]) * r;
  I[8] = (A[0] * A[4] - A[1] * A[3]) * r;
  return true;
}

bool orthonormal(const double* R) {
  double e = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += R[k * 3 + i] * R[k * 3 + j];
      e = std::max(e, std::fabs(s - (i == j ? 1.0 : 0.0)));
    }
  return e < 1e-4;
}

struct Problem {
  int ref;
  std::vector<int> srcs;
  int window, dilation;
  phimvs_params p;
};

std::string problem_key(const Problem& P) {
  std::string k = std::to_string(P.ref) + "," + std::to_string(P.window) + "," + std::to_string(P.dilation) + "," +
                  std::to_string(P.p.top_k) + "," + std::to_string(P.p.bilateral) + "," + std::to_string(P.p.seed) +
                  "," + std::to_string(P.p.sigma_color) + "," + std::to_string(P.p.sigma_spatial_px) + "," +
                  std::to_string(P.p.eps_var) + "," + std::to_string(P.p.eps_cost) + "," +
                  std::to_string(P.p.tap_radius) + "," + std::to_string(P.p.lanes) + "," +
                  std::to_string(P.p.score_all);
  for (int s : P.srcs) k += ";" + std::to_string(s);
  return k;
}

int validate_problem(phimvs_ctx* c, const Problem& P) {
  const int nv = (int)c->views.size();
  if (nv == 0) return fail(c, PHIMVS_E_STATE, "no views: call phimvs_set_views first");
  if (P.ref < 0 || P.ref >= nv) return fail(c, PHIMVS_E_ARG, "ref out of range");
  if (P.srcs.empty()) return fail(c, PHIMVS_E_ARG, "need at least one source view");
  if ((int)P.srcs.size() > PHIMVS_MAX_SOURCES)
    return fail(c, PHIMVS_E_UNSUPPORTED, "at most 12 source views per reference");
  for (size_t i = 0; i < P.srcs.size(); ++i) {
    if (P.srcs[i] < 0 || P.srcs[i] >= nv) return fail(c, PHIMVS_E_ARG, "source index out of range");
    if (P.srcs[i] == P.ref) return fail(c, PHIMVS_E_ARG, "the reference cannot be one of its sources");
    for (size_t k = 0; k < i; ++k)
      if (P.srcs[k] == P.srcs[i]) return fail(c, PHIMVS_E_ARG, "duplicate source view");
  }
  if (P.dilation < 1) return fail(c, PHIMVS_E_ARG, "dilation must be >= 1");
  if (P.window < 3 || P.window % 2 == 0 || (P.window - 1) % (2 * P.dilation) != 0)
    return fail(c, PHIMVS_E_ARG, "window must be odd with (window - 1) % (2 dilation) == 0");
  const int R = (P.window - 1) / (2 * P.dilation);
  if (R > 15) return fail(c, PHIMVS_E_UNSUPPORTED, "at most 31 taps per window side");
  if (P.dilation * R > 30) return fail(c, PHIMVS_E_UNSUPPORTED, "window radius above 30 px");
  const phimvs_params& p = P.p;
  if (p.tap_radius < 0) return fail(c, PHIMVS_E_ARG, "tap_radius must be >= 0");
  if (p.tap_radius > 0) {
    if (P.dilation != 1) return fail(c, PHIMVS_E_ARG, "the window-resize scheme (tap_radius > 0) needs dilation 1");
    if (p.tap_radius > (P.window - 1) / 2) return fail(c, PHIMVS_E_ARG, "tap_radius above the window radius");
    if (p.tap_radius > 15) return fail(c, PHIMVS_E_UNSUPPORTED, "at most 31 taps per window side");
    if ((P.window - 1) / 2 > 29) return fail(c, PHIMVS_E_UNSUPPORTED, "window radius above 29 px");
  }
  if (p.lanes < 0 || p.lanes > 16 || (p.lanes & (p.lanes - 1)))
    return fail(c, PHIMVS_E_ARG, "lanes must be 0, 1, 2, 4, 8 or 16");
  if (p.score_all < 0 || p.score_all > 2) return fail(c, PHIMVS_E_ARG, "score_all must be 0, 1 or 2");
  if (p.lanes > 1 && p.tap_radius > 0)
    return fail(c, PHIMVS_E_UNSUPPORTED, "lanes > 1 with the window-resize scheme");
  const int n = (int)P.srcs.size();
  if (p.top_k < 0 || p.top_k > n) return fail(c, PHIMVS_E_ARG, "top_k must be in [0, n_srcs]");
  if (!std::isfinite(p.sigma_spatial_px) || !(std::isfinite(p.sigma_color) && p.sigma_color > 0))
    return fail(c, PHIMVS_E_ARG, "bilateral sigmas must be finite, sigma_color > 0");
  if (!(p.eps_var >= 0 && std::isfinite(p.eps_var)) || !(p.eps_cost > 0 && std::isfinite(p.eps_cost)))
    return fail(c, PHIMVS_E_ARG, "eps_var must be >= 0 and eps_cost > 0");
  return PHIMVS_OK;
}

// fill the problem block of one job and allocate its state
int setup_job(phimvs_ctx* c, const Problem& P, Job& J, JobState& S) {
  const ViewData& V0 = c->views[P.ref];
  const phimvs_params& p = P.p;
  Args& A = J.A;
  A = Args{};
  const bool frac = p.tap_radius > 0;
  const int r_orig = (P.window - 1) / 2;
  const int R = frac ? p.tap_radius : (P.window - 1) / (2 * P.dilation);
  // spacing of the window-resize scheme, rounded to float once; offsets s k in FP32
  const double sf_d = frac ? (double)r_orig / (double)R : (double)P.dilation;
  const float sf = (float)sf_d;
  A.W = V0.W;
  A.H = V0.H;
  A.Wc = (V0.W + 1) / 2;
  A.R = R;
  A.s = frac ? 1 : P.dilation;
  A.frac = frac ? 1 : 0;
  for (int k = 0; k <= 2 * R; ++k) A.off[k] = frac ? sf * (float)(k - R) : (float)(P.dilation * (k - R));
  A.rv = frac ? r_orig : P.dilation * R;
  // interpolated taps read one texel beyond their offset
  A.halo = frac ? (int)std::ceil((double)A.off[2 * R]) + 1 : P.dilation * R;
  A.n_src = (int)P.srcs.size();
  A.top_k = p.top_k;
  A.bilateral = p.bilateral ? 1 : 0;
  A.n_taps = (2 * R + 1) * (2 * R + 1);
  A.lanes = p.lanes > 1 ? p.lanes : 1;
  A.score_all = p.score_all;
  double K0i[9];
  inv33(V0.K, K0i);
  for (int i = 0; i < 9; ++i) {
    A.Kinv[i] = (float)K0i[i];
    A.Kinv_d[i] = K0i[i];
  }
  A.d_lo = (float)V0.d_lo;
  A.d_hi = (float)V0.d_hi;
  A.eps_v = (float)p.eps_var;
  A.eps_c = (float)p.eps_cost;
  A.seed_lo = (uint32_t)(p.seed & 0xFFFFFFFFu);
  A.seed_hi = (uint32_t)(p.seed >> 32);
  A.ref = V0.plain;
  // relative poses and the plane-independent parts of the homographies (FP64)
  double R0t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R0t[i * 3 + j] = V0.R[j * 3 + i];
  for (int k = 0; k < A.n_src; ++k) {
    const ViewData& Vj = c->views[P.srcs[k]];
    double Rrel[9], Rt0[3], trel[3], KR[9], M[9], e[3];
    mul33(Vj.R, R0t, Rrel);
    mulv3(Rrel, V0.t, Rt0);
    for (int i = 0; i < 3; ++i) trel[i] = Vj.t[i] - Rt0[i];
    mul33(Vj.K, Rrel, KR);
    mul33(KR, K0i, M);
    mulv3(Vj.K, trel, e);
    SrcDev& D = A.src[k];
    for (int i = 0; i < 9; ++i) D.M[i] = (float)M[i];
    for (int i = 0; i < 3; ++i) D.e[i] = (float)e[i];
    D.W = Vj.W;
    D.H = Vj.H;
    D.Wm1 = (float)(Vj.W - 1);
    D.Hm1 = (float)(Vj.H - 1);
    D.quad = Vj.quad;
  }
  // bilateral weight factors: colour (|a - a_c| = 0..255) and space (tap offsets)
  const double sc = p.sigma_color;
  const double ss = p.sigma_spatial_px > 0 ? p.sigma_spatial_px : (double)((P.window - 1) / 2);
  std::vector<float> wc(256), ws(A.n_taps);
  for (int i = 0; i < 256; ++i) {
    const double d = (double)i;
    wc[i] = p.bilateral ? (float)std::exp(-(d * d) / (2.0 * sc * sc)) : 1.0f;
  }
  for (int k2 = -R, t = 0; k2 <= R; ++k2)
    for (int k1 = -R; k1 <= R; ++k1, ++t) {
      const double r2 = sf_d * sf_d * (double)(k1 * k1 + k2 * k2);
      ws[t] = p.bilateral ? (float)std::exp(-r2 / (2.0 * ss * ss)) : 1.0f;
    }
  int rc;
  if ((rc = ensure(c, S.wcol, 256)) || (rc = ensure(c, S.wsp, ws.size()))) return rc;
  HIPCHECK(c, hipMemcpyAsync(S.wcol.p, wc.data(), 256 * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHECK(c, hipMemcpyAsync(S.wsp.p, ws.data(), ws.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));  // the host vectors go out of scope
  A.wcol = S.wcol.p;
  A.wsp = S.wsp.p;
  const size_t ncol = (size_t)A.Wc * A.H;
  for (int k = 0; k < 2; ++k) {
    if ((rc = ensure(c, S.plane[k], ncol)) || (rc = ensure(c, S.cost[k], ncol))) return rc;
    A.plane[k] = S.plane[k].p;
    A.cost[k] = S.cost[k].p;
  }
  if ((rc = ensure(c, S.cand, 8 * ncol)) || (rc = ensure(c, S.hist, 16 * ncol))) return rc;
  J.cand = S.cand.p;
  J.hist[0] = S.hist.p;
  J.hist[1] = S.hist.p + 8 * ncol;
  J.planes_in = nullptr;
  J.cost_out = J.per_view_out = nullptr;
  J.valid_out = nullptr;
  J.depth_out = J.normal_out = J.final_cost_out = J.planes_out = nullptr;
  return PHIMVS_OK;
}

// tile / block offsets of every job for the current tile shape, and the launch-wide maxima
void layout(Batch& b, int tile_rows) {
  b.tile_rows = tile_rows;
  const int TC = kBlock / tile_rows;
  int t = 0, k = 0;
  b.max_r = 0;
  b.max_taps = 0;
  for (Job& J : b.jobs) {
    J.tile0 = t;
    J.tiles_x = (J.A.Wc + TC - 1) / TC;
    J.tiles_y = (J.A.H + tile_rows - 1) / tile_rows;
    t += J.tiles_x * J.tiles_y;
    J.cblk0 = k;
    J.cblk_x = (J.A.Wc + 127) / 128;
    k += J.cblk_x * J.A.H;
    b.max_r = std::max(b.max_r, J.A.halo);
    b.max_taps = std::max(b.max_taps, J.A.n_taps);
  }
  b.total_tiles = t;
  b.total_cblk = k;
  // XCD k takes the k-th of 8 bands (runs of whole tile rows) of every job, so every XCD
  // gets the same share of each job's work (jobs differ in source count and window) and a
  // compact band of each image
  for (int x = 0; x < 8; ++x) b.xcd_len[x] = 0;
  for (Job& J : b.jobs) {
    const int T = J.tiles_x * J.tiles_y;
    for (int x = 0; x < 8; ++x) {
      J.xband[x] = (int)((int64_t)J.tiles_y * x / 8) * J.tiles_x;
      J.xoff[x] = b.xcd_len[x];
    }
    for (int x = 0; x < 8; ++x) {
      const int end = x + 1 < 8 ? J.xband[x + 1] : T;
      b.xcd_len[x] += end - J.xband[x];
    }
  }
}

int upload_jobs(phimvs_ctx* c, Batch& b) {
  const size_t bytes = b.jobs.size() * sizeof(Job);
  const unsigned char* host = reinterpret_cast<const unsigned char*>(b.jobs.data());
  // the device already holds this table: nothing to copy and no queued work to wait for
  if (b.d_jobs && b.uploaded.size() == bytes && std::memcmp(b.uploaded.data(), host, bytes) == 0)
    return PHIMVS_OK;
  if (b.d_cap < bytes) {
    if (b.d_jobs) HIPCHECK(c, hipFree(b.d_jobs));
    b.d_jobs = nullptr;
    b.uploaded.clear();
    HIPCHECK(c, hipMalloc((void**)&b.d_jobs, bytes));
    b.d_cap = bytes;
  }
  // the table is read by work already queued: wait for it before overwriting
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  HIPCHECK(c, hipMemcpy(b.d_jobs, b.jobs.data(), bytes, hipMemcpyHostToDevice));
  b.uploaded.assign(host, host + bytes);
  return PHIMVS_OK;
}

Launch base_launch(const Batch& b) {
  Launch L{};
  L.n_jobs = (int)b.jobs.size();
  L.tile_rows = b.tile_rows;
  L.total_tiles = b.total_tiles;
  L.total_cblk = b.total_cblk;
  for (int x = 0; x < 8; ++x) L.xcd_len[x] = b.xcd_len[x];
  for (const Job& J : b.jobs) L.frac = L.frac || J.A.frac;
  return L;
}

int eval_grid(const phimvs_ctx* c, const Batch& b, bool persistent) {
  if (!persistent) return 8 * *std::max_element(b.xcd_len, b.xcd_len + 8);
  const int wgs = std::max(1, c->tuning.wgs_per_cu) * c->n_cu;
  return ((std::min(wgs, b.total_tiles) + 7) / 8) * 8;
}

// one evaluate-and-select launch (queue: 8 zeroed counters when persistent), with the
// optional diagnostics around it
int run_eval(phimvs_ctx* c, Batch& b, Launch L, unsigned int* queue) {
  const bool persistent = c->tuning.persistent != 0;
  L.persistent = persistent ? 1 : 0;
  // the depth-ordered instance for the launch kinds the tuning names (mask: 1 initialisation,
  // 2 propagation, 4 refinement)
  const int kind_bit = L.mode == 0 ? 1 : (L.ncand > 3 ? 2 : 4);
  L.order_by_depth = (c->tuning.order_by_depth & kind_bit) ? 1 : 0;
  L.queue = queue;
  if (c->diag & PHIMVS_DIAG_COUNT) L.count = c->diag_count;
  const bool split = b.jobs.size() == 1 && b.jobs[0].A.lanes > 1;
  const Args& A0 = b.jobs[0].A;
  const size_t lds = split ? eval_lanes_lds_bytes(A0.lanes, A0.halo, A0.n_taps)
                           : eval_lds_bytes(b.tile_rows, b.max_r, b.max_taps);
  if (lds > c->eval_lds_max)
    return fail(c, PHIMVS_E_UNSUPPORTED, "evaluate launch: " + std::to_string(b.tile_rows) + "-row tiles need " +
                                              std::to_string(lds) + " bytes of LDS, the device allows " +
                                              std::to_string(c->eval_lds_max));
  const int grid = eval_grid(c, b, persistent);
  const bool timed = (c->diag & PHIMVS_DIAG_TIME) != 0;
  if (timed) {
    hipEvent_t e0, e1;
    HIPCHECK(c, hipEventCreate(&e0));
    HIPCHECK(c, hipEventCreate(&e1));
    c->diag_events.emplace_back(e0, e1);
    HIPCHECK(c, hipEventRecord(e0, c->stream));
  }
  const hipError_t e = split ? launch_eval_lanes(b.d_jobs, L, A0.lanes, A0.H, A0.Wc, lds, c->stream)
                              : launch_eval(b.d_jobs, L, grid, lds, c->stream);
  if (e != hipSuccess)
    return fail(c, PHIMVS_E_DEVICE, "evaluate launch (" + std::to_string(grid) + " workgroups, " +
                                        std::to_string(lds) + " bytes of dynamic LDS): " + hipGetErrorString(e));
  if (timed) HIPCHECK(c, hipEventRecord(c->diag_events.back().second, c->stream));
  return PHIMVS_OK;
}

// the launch sequence of init + iters x (red, black) x (propagate, refine) (+ unpack);
// each evaluate launch gets its own 8 queue counters from b.queues, zeroed first by a
// kernel (no memset node, so the sequence replays correctly from a graph)
// with_proposal: the jobs carry proposal planes (planes_in) that compete with the random
// initial plane (kept when not costlier)
int issue_sequence(phimvs_ctx* c, Batch& b, int iters, bool do_unpack, bool with_proposal = false) {
  const int n_eval = 2 + 4 * iters;
  if (b.queues.n < (size_t)8 * n_eval) return fail(c, PHIMVS_E_STATE, "queue counters not allocated");
  HIPCHECK(c, launch_zero(b.queues.p, 8 * n_eval, c->stream));
  int q = 0, rc;
  Launch L = base_launch(b);
  b.hist_valid[0] = b.hist_valid[1] = false;
  for (int colour = 0; colour < 2; ++colour) {
    L.colour = colour;
    L.mode = 0;
    L.ncand = with_proposal ? 2 : 1;
    HIPCHECK(c, launch_candidates(0, b.d_jobs, L, c->stream));
    if ((rc = run_eval(c, b, L, b.queues.p + 8 * q++))) return rc;
  }
  b.state_exact = true;
  L.skip_current = 1;
  for (int it = 1; it <= iters; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      L.colour = colour;
      L.iteration = it;
      L.mode = 1;
      L.ncand = 8;
      L.hist_mode = it == 1 ? 1 : 2;
      HIPCHECK(c, launch_candidates(1, b.d_jobs, L, c->stream));
      if ((rc = run_eval(c, b, L, b.queues.p + 8 * q++))) return rc;
      L.ncand = 3;
      L.hist_mode = 0;
      HIPCHECK(c, launch_candidates(2, b.d_jobs, L, c->stream));
      if ((rc = run_eval(c, b, L, b.queues.p + 8 * q++))) return rc;
    }
  b.hist_valid[0] = b.hist_valid[1] = iters >= 1;
  if (do_unpack) HIPCHECK(c, launch_unpack(b.d_jobs, base_launch(b), c->stream));
  return PHIMVS_OK;
}

int need_prepared(phimvs_ctx* c) {
  if (!c) return PHIMVS_E_ARG;
  if (!c->prepared) return fail(c, PHIMVS_E_STATE, "call phimvs_prepare first");
  return PHIMVS_OK;
}

// device pointer for an input array: either the caller's, or a staging copy of host data
int input_ptr(phimvs_ctx* c, DevBuf<float>& stage, const float* p, size_t n, int on_device, const float** out) {
  if (on_device) {
    *out = p;
    return PHIMVS_OK;
  }
  int rc = ensure(c, stage, n);
  if (rc) return rc;
  HIPCHECK(c, hipMemcpyAsync(stage.p, p, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  *out = stage.p;
  return PHIMVS_OK;
}

// evaluate launch outside a sequence (its own queue)
int eval_once(phimvs_ctx* c, Batch& b, Launch L) {
  int rc = ensure(c, b.queues, 8);
  if (rc) return rc;
  HIPCHECK(c, launch_zero(b.queues.p, 8, c->stream));
  if ((rc = run_eval(c, b, L, b.queues.p))) return rc;
  return PHIMVS_OK;
}

Problem make_problem(int ref, const int* srcs, int n_srcs, int window, int dilation, const phimvs_params* pp) {
  Problem P;
  P.ref = ref;
  if (srcs && n_srcs > 0) P.srcs.assign(srcs, srcs + n_srcs);
  P.window = window;
  P.dilation = dilation;
  if (pp) P.p = *pp;
  else phimvs_default_params(&P.p);
  return P;
}

// the single-view problem: device state (kept when the problem is unchanged) and the job
// table with no outputs; upload: copy the table to the device now (else the caller does,
// after setting the outputs)
int prepare_single(phimvs_ctx* c, int ref, const int* srcs, int n_srcs, int window, int dilation,
                   const phimvs_params* pp, bool upload) {
  if (!c) return PHIMVS_E_ARG;
  c->prepared = false;
  if (n_srcs < 0 || (n_srcs > 0 && !srcs)) return fail(c, PHIMVS_E_ARG, "need at least one source view");
  Problem P = make_problem(ref, srcs, n_srcs, window, dilation, pp);
  int rc = validate_problem(c, P);
  if (rc) return rc;
  HIPCHECK(c, hipSetDevice(c->device));
  Batch& b = c->single;
  const std::string key = problem_key(P) + "@" + std::to_string(c->tuning.tile_rows);
  if (key != b.layout_key || b.jobs.size() != 1) {
    release_graph(b);
    resize_jobs(b, 1);
    if ((rc = setup_job(c, P, b.jobs[0], b.state[0]))) return rc;
    layout(b, c->tuning.tile_rows);
    b.layout_key = key;
  }
  Job& J = b.jobs[0];
  J.planes_in = nullptr;
  J.cost_out = J.per_view_out = nullptr;
  J.valid_out = nullptr;
  J.depth_out = J.normal_out = J.final_cost_out = J.planes_out = nullptr;
  if (upload && (rc = upload_jobs(c, b))) return rc;
  b.state_exact = false;
  b.hist_valid[0] = b.hist_valid[1] = false;
  c->prepared = true;
  return PHIMVS_OK;
}

// after the sequence has been issued (or its graph launched): what it leaves in the state
void sequence_done(Batch& b, int iters) {
  b.state_exact = true;
  b.hist_valid[0] = b.hist_valid[1] = iters >= 1;
}

// The iteration sequence through a hipGraph: recorded once per gkey (which names
// everything the recorded launches hold: geometry, iterations, launch configuration,
// buffers), replayed on later calls.  The job table is read at run time, so its outputs may
// change between replays.
int run_sequence_graph(phimvs_ctx* c, Batch& b, const std::string& gkey, int iters) {
  int rc;
  if (b.exec && b.graph_key == gkey) {
    HIPCHECK(c, hipGraphLaunch(b.exec, c->stream));
    sequence_done(b, iters);
    return PHIMVS_OK;
  }
  release_graph(b);
  // record on a private stream (the caller's may be the null stream, which cannot be
  // captured); the graph is then launched on the caller's stream, after its prior work
  if (!c->capture_stream) HIPCHECK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  c->stream = c->capture_stream;
  hipError_t eb = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) {
    c->stream = user;
    return fail(c, PHIMVS_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(eb));
  }
  rc = issue_sequence(c, b, iters, true);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->stream, &g);
  c->stream = user;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  HIPCHECK(c, ec);
  b.graph = g;
  HIPCHECK(c, hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
  b.graph_key = gkey;
  HIPCHECK(c, hipGraphLaunch(b.exec, c->stream));
  return PHIMVS_OK;
}

// one depth map through the single-job batch: prepare, then the whole launch sequence
// (replayed from a graph when there is no proposal); proposal (planes layout, optional)
// gates the random initialisation
int run_single(phimvs_ctx* c, int ref, const int* srcs, int n_srcs, int window, int dilation, int iters,
               const phimvs_params* p, const float* proposal, float* depth, float* normal, float* cost,
               int on_device) {
  if (!c) return PHIMVS_E_ARG;
  if (iters < 0) return fail(c, PHIMVS_E_ARG, "iters must be >= 0");
  int rc = prepare_single(c, ref, srcs, n_srcs, window, dilation, p, false);
  if (rc) return rc;
  Batch& b = c->single;
  Job& J = b.jobs[0];
  const size_t n = (size_t)J.A.W * J.A.H;
  const float* prop = nullptr;
  if (proposal) {
    if (on_device) {
      prop = proposal;
    } else {
      if ((rc = ensure(c, c->io_d, 4 * n))) return rc;
      HIPCHECK(c, hipMemcpyAsync(c->io_d.p, proposal, 4 * n * sizeof(float), hipMemcpyHostToDevice, c->stream));
      prop = c->io_d.p;
    }
  }
  if (on_device) {
    J.depth_out = depth;
    J.normal_out = normal;
    J.final_cost_out = cost;
  } else {
    if ((rc = ensure(c, c->io_a, 3 * n)) || (rc = ensure(c, c->io_b, n)) || (rc = ensure(c, c->io_c, n))) return rc;
    J.normal_out = normal ? c->io_a.p : nullptr;
    J.depth_out = depth ? c->io_b.p : nullptr;
    J.final_cost_out = cost ? c->io_c.p : nullptr;
  }
  J.planes_in = prop;
  // the table is complete before the sequence starts (unchanged from the last call: not
  // copied again, and nothing waited for)
  rc = upload_jobs(c, b);
  J.planes_in = nullptr;  // the next upload drops the caller's pointer
  if (rc) return rc;
  if ((rc = ensure(c, b.queues, (size_t)8 * (2 + 4 * iters)))) return rc;
  if (prop || c->diag) {
    rc = issue_sequence(c, b, iters, true, prop != nullptr);
  } else {
    char ptrs[64];
    std::snprintf(ptrs, sizeof ptrs, "#%p#%p", (void*)b.d_jobs, (void*)b.queues.p);
    const std::string gkey = b.layout_key + "#" + std::to_string(iters) + "#" +
                             std::to_string(c->tuning.persistent) + "#" + std::to_string(c->tuning.wgs_per_cu) +
                             "#" + std::to_string(c->tuning.order_by_depth) + ptrs;
    rc = run_sequence_graph(c, b, gkey, iters);
  }
  if (rc) return rc;
  if (!on_device) {
    if (normal) HIPCHECK(c, hipMemcpyAsync(normal, c->io_a.p, 3 * n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (depth) HIPCHECK(c, hipMemcpyAsync(depth, c->io_b.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (cost) HIPCHECK(c, hipMemcpyAsync(cost, c->io_c.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
  }
  return PHIMVS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------- internal accessors

namespace phimvs_internal {

int view_info(phimvs_ctx* c, int idx, ViewInfo* out) {
  if (!c) return PHIMVS_E_ARG;
  if (idx < 0 || idx >= (int)c->views.size()) return fail(c, PHIMVS_E_ARG, "view index out of range");
  const ViewData& v = c->views[idx];
  out->W = v.W;
  out->H = v.H;
  for (int i = 0; i < 9; ++i) out->K[i] = v.K[i], out->R[i] = v.R[i];
  for (int i = 0; i < 3; ++i) out->t[i] = v.t[i];
  out->d_lo = v.d_lo;
  out->d_hi = v.d_hi;
  out->plain = v.plain;
  out->quad = v.quad;
  return PHIMVS_OK;
}

int ctx_device(const phimvs_ctx* c) { return c->device; }
hipStream_t ctx_stream(const phimvs_ctx* c) { return c->stream; }
int ctx_fail(phimvs_ctx* c, int code, const char* msg) { return fail(c, code, msg); }

}  // namespace phimvs_internal

extern "C" {

void phimvs_default_params(phimvs_params* p) {
  if (!p) return;
  p->top_k = 0;
  p->bilateral = 1;
  p->sigma_spatial_px = 0.0;
  p->sigma_color = 12.0;
  p->eps_var = 1e-4;
  p->eps_cost = 1e-4;
  p->seed = 0x5EED;
  p->tap_radius = 0;
  p->lanes = 0;
  p->score_all = 0;
}

int phimvs_create(phimvs_ctx** out, int device_ordinal, void* hip_stream) {
  if (!out) return PHIMVS_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device_ordinal < 0 || device_ordinal >= n) return PHIMVS_E_DEVICE;
  if (hipSetDevice(device_ordinal) != hipSuccess) return PHIMVS_E_DEVICE;
  phimvs_ctx* c = new (std::nothrow) phimvs_ctx();
  if (!c) return PHIMVS_E_OOM;
  c->device = device_ordinal;
  c->stream = (hipStream_t)hip_stream;
  if (eval_lds_setup(&c->eval_lds_max) != hipSuccess) {
    delete c;
    return PHIMVS_E_DEVICE;
  }
  // the allocation-free entry point's scratch address on this device (looked up once per
  // device; a failure is kept and reported by that entry point alone)
  (void)phi_scratch_setup(device_ordinal);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device_ordinal) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  *out = c;
  return PHIMVS_OK;
}

static void free_views(phimvs_ctx* c) {
  for (auto& v : c->views) {
    if (v.plain) (void)hipFree(v.plain);
    if (v.quad) (void)hipFree(v.quad);
  }
  c->views.clear();
}

void phimvs_destroy(phimvs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_views(c);
  release_batch(c->single);
  release_batch(c->multi);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  release(c->io_a);
  release(c->io_b);
  release(c->io_c);
  release(c->io_d);
  release(c->filter_nbrs);
  release(c->fuse_maps);
  release(c->fuse_alive);
  release(c->fuse_claim);
  release(c->phi_bits);
  release(c->io_u8);
  if (c->diag_count) (void)hipFree(c->diag_count);
  for (auto& e : c->diag_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  delete c;
}

const char* phimvs_last_error(const phimvs_ctx* c) { return c ? c->err.c_str() : "null context"; }

int phimvs_set_stream(phimvs_ctx* c, void* hip_stream) {
  if (!c) return PHIMVS_E_ARG;
  c->stream = (hipStream_t)hip_stream;  // a captured graph replays on whatever stream launches it
  return PHIMVS_OK;
}

int phimvs_sync(phimvs_ctx* c) {
  if (!c) return PHIMVS_E_ARG;
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return PHIMVS_OK;
}

int phimvs_set_views(phimvs_ctx* c, int n_views, const phimvs_image* images, const double* K, const double* R,
                     const double* t, const double* depth_range) {
  if (!c) return PHIMVS_E_ARG;
  if (n_views < 2 || !images || !K || !R || !t || !depth_range)
    return fail(c, PHIMVS_E_ARG, "set_views needs n_views >= 2 and non-null images/K/R/t/depth_range");
  for (int i = 0; i < n_views; ++i) {
    const phimvs_image& im = images[i];
    if (im.dtype != PHIMVS_U8) return fail(c, PHIMVS_E_UNSUPPORTED, "only PHIMVS_U8 images are supported");
    if (im.width < 1 || im.height < 1 || !im.data) return fail(c, PHIMVS_E_ARG, "image " + std::to_string(i) + " is empty");
    if ((int64_t)im.width * im.height >= (int64_t)1 << 28)
      return fail(c, PHIMVS_E_UNSUPPORTED, "image " + std::to_string(i) + " exceeds 2^28 pixels");
    if (im.stride_bytes != 0 && im.stride_bytes < im.width)
      return fail(c, PHIMVS_E_ARG, "image " + std::to_string(i) + " stride smaller than its width");
    if (!finite_all(K + 9 * i, 9) || !finite_all(R + 9 * i, 9) || !finite_all(t + 3 * i, 3) ||
        !finite_all(depth_range + 2 * i, 2))
      return fail(c, PHIMVS_E_ARG, "camera " + std::to_string(i) + " has non-finite entries");
    double Ki[9];
    if (!inv33(K + 9 * i, Ki)) return fail(c, PHIMVS_E_ARG, "K of view " + std::to_string(i) + " is singular");
    if (!orthonormal(R + 9 * i)) return fail(c, PHIMVS_E_ARG, "R of view " + std::to_string(i) + " is not a rotation");
    if (!(depth_range[2 * i] > 0 && depth_range[2 * i] < depth_range[2 * i + 1]))
      return fail(c, PHIMVS_E_ARG, "depth range of view " + std::to_string(i) + " needs 0 < d_lo < d_hi");
  }
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  free_views(c);
  release_batch(c->single);
  release_batch(c->multi);
  c->prepared = false;
  c->views.resize(n_views);
  for (int i = 0; i < n_views; ++i) {
    const phimvs_image& im = images[i];
    ViewData& v = c->views[i];
    v.W = im.width;
    v.H = im.height;
    std::memcpy(v.K, K + 9 * i, sizeof v.K);
    std::memcpy(v.R, R + 9 * i, sizeof v.R);
    std::memcpy(v.t, t + 3 * i, sizeof v.t);
    v.d_lo = depth_range[2 * i];
    v.d_hi = depth_range[2 * i + 1];
    const size_t npx = (size_t)v.W * v.H;
    HIPCHECK(c, hipMalloc((void**)&v.plain, npx * sizeof(__half)));
    HIPCHECK(c, hipMalloc((void**)&v.quad, npx * sizeof(uint32_t)));
    const int64_t stride = im.stride_bytes ? im.stride_bytes : im.width;
    int rc = ensure(c, c->io_u8, npx);
    if (rc) return rc;
    HIPCHECK(c, hipMemcpy2DAsync(c->io_u8.p, v.W, im.data, stride, v.W, v.H,
                                 im.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, launch_build_view(c->io_u8.p, v.W, v.W, v.H, v.plain, v.quad, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
  }
  return PHIMVS_OK;
}

int phimvs_prepare(phimvs_ctx* c, int ref, const int* srcs, int n_srcs, int window, int dilation,
                   const phimvs_params* pp) {
  return prepare_single(c, ref, srcs, n_srcs, window, dilation, pp, true);
}

int phimvs_init_planes(phimvs_ctx* c, const float* proposal, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  HIPCHECK(c, hipSetDevice(c->device));
  Batch& b = c->single;
  const float* prop = nullptr;
  if (proposal) {
    if ((rc = input_ptr(c, c->io_a, proposal, (size_t)b.jobs[0].A.W * b.jobs[0].A.H * 4, on_device, &prop))) return rc;
  }
  if (b.jobs[0].planes_in != prop) {
    b.jobs[0].planes_in = prop;
    if ((rc = upload_jobs(c, b))) return rc;
  }
  Launch L = base_launch(b);
  L.mode = 0;
  L.ncand = prop ? 2 : 1;
  for (int colour = 0; colour < 2; ++colour) {
    L.colour = colour;
    HIPCHECK(c, launch_candidates(0, b.d_jobs, L, c->stream));
    if ((rc = eval_once(c, b, L))) return rc;
  }
  if (prop) {
    b.jobs[0].planes_in = nullptr;
    if ((rc = upload_jobs(c, b))) return rc;  // waits for the launches reading the proposal
  }
  b.state_exact = true;
  b.hist_valid[0] = b.hist_valid[1] = false;
  return PHIMVS_OK;
}

int phimvs_step(phimvs_ctx* c, int iteration, int colour, int do_propagate, int do_refine) {
  int rc = need_prepared(c);
  if (rc) return rc;
  if (colour != 0 && colour != 1) return fail(c, PHIMVS_E_ARG, "colour must be 0 or 1");
  if (iteration < 1) return fail(c, PHIMVS_E_ARG, "iteration must be >= 1");
  HIPCHECK(c, hipSetDevice(c->device));
  Batch& b = c->single;
  Launch L = base_launch(b);
  L.colour = colour;
  L.iteration = iteration;
  L.mode = 1;
  L.skip_current = b.state_exact ? 1 : 0;
  if (do_propagate) {
    L.ncand = 8;
    L.hist_mode = b.hist_valid[colour] ? 2 : 1;
    b.hist_valid[colour] = false;  // until the selection that the recorded candidates went through is done
    HIPCHECK(c, launch_candidates(1, b.d_jobs, L, c->stream));
    if ((rc = eval_once(c, b, L))) return rc;
    b.hist_valid[colour] = true;
    L.hist_mode = 0;
  }
  if (do_refine) {
    L.ncand = 3;
    HIPCHECK(c, launch_candidates(2, b.d_jobs, L, c->stream));
    if ((rc = eval_once(c, b, L))) return rc;
  }
  return PHIMVS_OK;
}

// unpack the single job's state into the given device outputs
static int unpack_single(phimvs_ctx* c, float* planes, float* depth, float* normal, float* cost) {
  Batch& b = c->single;
  Job& J = b.jobs[0];
  J.planes_out = planes;
  J.depth_out = depth;
  J.normal_out = normal;
  J.final_cost_out = cost;
  int rc = upload_jobs(c, b);
  if (rc) return rc;
  HIPCHECK(c, launch_unpack(b.d_jobs, base_launch(b), c->stream));
  return PHIMVS_OK;
}

int phimvs_get_state(phimvs_ctx* c, float* planes, float* cost, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  HIPCHECK(c, hipSetDevice(c->device));
  const size_t n = (size_t)c->single.jobs[0].A.W * c->single.jobs[0].A.H;
  float* dp = planes;
  float* dc = cost;
  if (!on_device) {
    if ((rc = ensure(c, c->io_a, 4 * n)) || (rc = ensure(c, c->io_b, n))) return rc;
    dp = planes ? c->io_a.p : nullptr;
    dc = cost ? c->io_b.p : nullptr;
  }
  if ((rc = unpack_single(c, dp, nullptr, nullptr, dc))) return rc;
  if (!on_device) {
    if (planes) HIPCHECK(c, hipMemcpyAsync(planes, c->io_a.p, 4 * n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (cost) HIPCHECK(c, hipMemcpyAsync(cost, c->io_b.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
  }
  return PHIMVS_OK;
}

int phimvs_set_state(phimvs_ctx* c, const float* planes, const float* cost, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  if (!planes || !cost) return fail(c, PHIMVS_E_ARG, "set_state needs planes and cost");
  HIPCHECK(c, hipSetDevice(c->device));
  const Job& J = c->single.jobs[0];
  const size_t n = (size_t)J.A.W * J.A.H;
  const float *dp, *dc;
  if ((rc = input_ptr(c, c->io_a, planes, 4 * n, on_device, &dp))) return rc;
  if ((rc = input_ptr(c, c->io_b, cost, n, on_device, &dc))) return rc;
  HIPCHECK(c, launch_pack(c->single.d_jobs, J.A.W, J.A.H, dp, dc, c->stream));
  if (!on_device) HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->single.state_exact = false;  // the caller's costs need not be its planes' costs
  // a cost the caller raised can make a candidate offered earlier win again
  c->single.hist_valid[0] = c->single.hist_valid[1] = false;
  return PHIMVS_OK;
}

int phimvs_output(phimvs_ctx* c, float* depth, float* normal, float* cost, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  HIPCHECK(c, hipSetDevice(c->device));
  const size_t n = (size_t)c->single.jobs[0].A.W * c->single.jobs[0].A.H;
  float *dd = depth, *dn = normal, *dc = cost;
  if (!on_device) {
    if ((rc = ensure(c, c->io_a, 3 * n)) || (rc = ensure(c, c->io_b, n)) || (rc = ensure(c, c->io_c, n))) return rc;
    dn = normal ? c->io_a.p : nullptr;
    dd = depth ? c->io_b.p : nullptr;
    dc = cost ? c->io_c.p : nullptr;
  }
  if ((rc = unpack_single(c, nullptr, dd, dn, dc))) return rc;
  if (!on_device) {
    if (normal) HIPCHECK(c, hipMemcpyAsync(normal, c->io_a.p, 3 * n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (depth) HIPCHECK(c, hipMemcpyAsync(depth, c->io_b.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (cost) HIPCHECK(c, hipMemcpyAsync(cost, c->io_c.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
  }
  return PHIMVS_OK;
}

int phimvs_eval_cost(phimvs_ctx* c, const float* planes, float* cost, float* per_view, uint8_t* valid, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  if (!planes || !cost) return fail(c, PHIMVS_E_ARG, "eval_cost needs planes and cost");
  HIPCHECK(c, hipSetDevice(c->device));
  Batch& b = c->single;
  Job& J = b.jobs[0];
  const size_t n = (size_t)J.A.W * J.A.H;
  const size_t nv = (size_t)J.A.n_src;
  const float* pin;
  if ((rc = input_ptr(c, c->io_a, planes, 4 * n, on_device, &pin))) return rc;
  J.planes_in = pin;
  J.cost_out = cost;
  J.per_view_out = per_view;
  J.valid_out = valid;
  if (!on_device) {
    if ((rc = ensure(c, c->io_b, n)) || (rc = ensure(c, c->io_c, per_view ? n * nv : 1)) ||
        (rc = ensure(c, c->io_u8, valid ? n * nv : 1)))
      return rc;
    J.cost_out = c->io_b.p;
    J.per_view_out = per_view ? c->io_c.p : nullptr;
    J.valid_out = valid ? c->io_u8.p : nullptr;
  }
  if ((rc = upload_jobs(c, b))) return rc;
  Launch L = base_launch(b);
  L.mode = 2;
  for (int colour = 0; colour < 2; ++colour) {
    L.colour = colour;
    if ((rc = eval_once(c, b, L))) return rc;
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  if (!on_device) {
    HIPCHECK(c, hipMemcpy(cost, c->io_b.p, n * sizeof(float), hipMemcpyDeviceToHost));
    if (per_view) HIPCHECK(c, hipMemcpy(per_view, c->io_c.p, n * nv * sizeof(float), hipMemcpyDeviceToHost));
    if (valid) HIPCHECK(c, hipMemcpy(valid, c->io_u8.p, n * nv, hipMemcpyDeviceToHost));
  }
  J.planes_in = nullptr;
  J.cost_out = J.per_view_out = nullptr;
  J.valid_out = nullptr;
  return upload_jobs(c, b);
}

int phimvs_patchmatch(phimvs_ctx* c, int ref, const int* srcs, int n_srcs, int window, int dilation, int iters,
                      const phimvs_params* p, float* depth, float* normal, float* cost, int out_on_device) {
  return run_single(c, ref, srcs, n_srcs, window, dilation, iters, p, nullptr, depth, normal, cost, out_on_device);
}

int phimvs_patchmatch_proposal(phimvs_ctx* c, int ref, const int* srcs, int n_srcs, int window, int dilation,
                               int iters, const phimvs_params* p, const float* proposal, float* depth, float* normal,
                               float* cost, int on_device) {
  if (!c) return PHIMVS_E_ARG;
  if (!proposal) return fail(c, PHIMVS_E_ARG, "proposal planes required");
  return run_single(c, ref, srcs, n_srcs, window, dilation, iters, p, proposal, depth, normal, cost, on_device);
}

// ---------------------------------------------------------------------------- consistency filter

void phimvs_default_filter_params(phimvs_filter_params* p) {
  if (!p) return;
  p->max_rel_depth = 0.02;
  p->max_angle_deg = 30.0;
  p->max_reproj_px = 1.0;
  p->min_consistent = 2;
}

int phimvs_filter(phimvs_ctx* c, int n_maps, const phimvs_depth_map* maps, int ref_map, const int32_t* nbrs,
                  int n_nbrs, const phimvs_filter_params* pp, float* depth_out, float* normal_out,
                  uint8_t* count_out) {
  if (!c) return PHIMVS_E_ARG;
  if (n_maps < 1 || !maps || ref_map < 0 || ref_map >= n_maps) return fail(c, PHIMVS_E_ARG, "invalid map list");
  if (n_nbrs < 0 || n_nbrs > PHIMVS_MAX_SOURCES || (n_nbrs > 0 && !nbrs))
    return fail(c, PHIMVS_E_ARG, "between 0 and PHIMVS_MAX_SOURCES neighbours");
  if (!depth_out || !normal_out || !count_out) return fail(c, PHIMVS_E_ARG, "null output");
  phimvs_filter_params p;
  phimvs_default_filter_params(&p);
  if (pp) p = *pp;
  if (!(p.max_rel_depth > 0) || !(p.max_angle_deg > 0 && p.max_angle_deg <= 180) || !(p.max_reproj_px > 0) ||
      p.min_consistent < 0)
    return fail(c, PHIMVS_E_ARG, "invalid filter thresholds");
  auto view_ok = [&](const phimvs_depth_map& m) {
    return m.view >= 0 && m.view < (int)c->views.size() && m.depth && m.normal;
  };
  const phimvs_depth_map& R0 = maps[ref_map];
  if (!view_ok(R0)) return fail(c, PHIMVS_E_ARG, "reference map: invalid view or null arrays");
  HIPCHECK(c, hipSetDevice(c->device));
  const ViewData& V0 = c->views[R0.view];
  FilterArgs a{};
  a.W = V0.W;
  a.H = V0.H;
  for (int i = 0; i < 9; ++i) a.K[i] = V0.K[i], a.R[i] = V0.R[i];
  for (int i = 0; i < 3; ++i) a.t[i] = V0.t[i];
  if (!inv33(V0.K, a.Kinv)) return fail(c, PHIMVS_E_ARG, "singular K");
  a.depth = R0.depth;
  a.normal = R0.normal;
  a.tau_d = p.max_rel_depth;
  a.cos_n = std::cos(p.max_angle_deg * 3.14159265358979323846 / 180.0);
  a.tau_r = p.max_reproj_px;
  a.min_consistent = p.min_consistent;
  a.depth_out = depth_out;
  a.normal_out = normal_out;
  a.count_out = count_out;
  // the previous call's table may still be in use by its launch
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->filter_host.assign(std::max(n_nbrs, 1), FilterNbr{});
  for (int k = 0; k < n_nbrs; ++k) {
    if (nbrs[k] < 0 || nbrs[k] >= n_maps || nbrs[k] == ref_map || !view_ok(maps[nbrs[k]]))
      return fail(c, PHIMVS_E_ARG, "neighbour " + std::to_string(k) + ": invalid map index, view or arrays");
    const phimvs_depth_map& M = maps[nbrs[k]];
    const ViewData& V = c->views[M.view];
    FilterNbr& nb = c->filter_host[k];
    for (int i = 0; i < 9; ++i) nb.K[i] = V.K[i], nb.R[i] = V.R[i];
    for (int i = 0; i < 3; ++i) nb.t[i] = V.t[i];
    if (!inv33(V.K, nb.Kinv)) return fail(c, PHIMVS_E_ARG, "singular K");
    nb.W = V.W;
    nb.H = V.H;
    nb.depth = M.depth;
    nb.normal = M.normal;
  }
  int rc;
  if ((rc = ensure(c, c->filter_nbrs, c->filter_host.size()))) return rc;
  HIPCHECK(c, hipMemcpyAsync(c->filter_nbrs.p, c->filter_host.data(), c->filter_host.size() * sizeof(FilterNbr),
                             hipMemcpyHostToDevice, c->stream));
  a.n_nbrs = n_nbrs;
  a.nbrs = c->filter_nbrs.p;
  HIPCHECK(c, launch_filter(a, c->stream));
  return PHIMVS_OK;
}

// ---------------------------------------------------------------------------- depth-map fusion

void phimvs_default_fuse_params(phimvs_fuse_params* p) {
  if (!p) return;
  p->max_rel_dist = 0.01;
}

int phimvs_fuse(phimvs_ctx* c, int n_maps, const phimvs_depth_map* maps, const phimvs_fuse_params* pp, float* points,
                int32_t* support, int64_t* owner) {
  if (!c) return PHIMVS_E_ARG;
  if (n_maps < 1 || !maps) return fail(c, PHIMVS_E_ARG, "invalid map list");
  if (!points || !support || !owner) return fail(c, PHIMVS_E_ARG, "null output");
  phimvs_fuse_params p;
  phimvs_default_fuse_params(&p);
  if (pp) p = *pp;
  if (!(p.max_rel_dist >= 0.0) || !std::isfinite(p.max_rel_dist))
    return fail(c, PHIMVS_E_ARG, "max_rel_dist must be finite and >= 0");
  HIPCHECK(c, hipSetDevice(c->device));
  // the previous call's table may still be in use by its launches
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->fuse_host.assign(n_maps, FuseMap{});
  int64_t total = 0;
  for (int k = 0; k < n_maps; ++k) {
    const phimvs_depth_map& M = maps[k];
    if (M.view < 0 || M.view >= (int)c->views.size() || !M.depth)
      return fail(c, PHIMVS_E_ARG, "map " + std::to_string(k) + ": invalid view or null depth");
    const ViewData& V = c->views[M.view];
    if ((int64_t)V.W * V.H >= INT32_MAX) return fail(c, PHIMVS_E_UNSUPPORTED, "map above 2^31 pixels");
    FuseMap& f = c->fuse_host[k];
    for (int i = 0; i < 9; ++i) f.K[i] = V.K[i], f.R[i] = V.R[i];
    for (int i = 0; i < 3; ++i) f.t[i] = V.t[i];
    if (!inv33(V.K, f.Kinv)) return fail(c, PHIMVS_E_ARG, "singular K");
    f.W = V.W;
    f.H = V.H;
    f.off = total;
    f.depth = M.depth;
    total += (int64_t)V.W * V.H;
  }
  int rc;
  if ((rc = ensure(c, c->fuse_maps, (size_t)n_maps))) return rc;
  if ((rc = ensure(c, c->fuse_alive, (size_t)total))) return rc;
  if ((rc = ensure(c, c->fuse_claim, (size_t)total))) return rc;
  HIPCHECK(c, hipMemcpyAsync(c->fuse_maps.p, c->fuse_host.data(), n_maps * sizeof(FuseMap), hipMemcpyHostToDevice,
                             c->stream));
  HIPCHECK(c, launch_fuse(c->fuse_host.data(), c->fuse_maps.p, n_maps, p.max_rel_dist, c->fuse_alive.p,
                          c->fuse_claim.p, points, support, owner, c->stream));
  return PHIMVS_OK;
}

// ---------------------------------------------------------------------------- plane hypothesis inference

int phimvs_phi_hypotheses(phimvs_ctx* c, int width, int height, const float* depth, float* hyp) {
  if (!c) return PHIMVS_E_ARG;
  if (width < 1 || height < 1 || !depth || !hyp) return fail(c, PHIMVS_E_ARG, "invalid size or null array");
  HIPCHECK(c, hipSetDevice(c->device));
  int rc = ensure(c, c->phi_bits, phi_bits_words(width, height));
  if (rc) return rc;
  HIPCHECK(c, launch_phi_hypotheses(depth, width, height, c->phi_bits.p, hyp, c->stream));
  return PHIMVS_OK;
}

int phimvs_phi_hypotheses_noalloc(phimvs_ctx* c, int width, int height, const float* depth, float* hyp) {
  if (!c) return PHIMVS_E_ARG;
  if (width < 1 || height < 1 || !depth || !hyp) return fail(c, PHIMVS_E_ARG, "invalid size or null array");
  const size_t need = phi_bits_words(width, height);
  if (need > kPhiScratchWords)
    return fail(c, PHIMVS_E_UNSUPPORTED, "a " + std::to_string(width) + "x" + std::to_string(height) +
                                             " map needs " + std::to_string(need) + " words of scratch; " +
                                             "the allocation-free entry point has " +
                                             std::to_string(kPhiScratchWords));
  uint64_t* bits = nullptr;
  const hipError_t e = phi_scratch_get(c->device, &bits);
  if (e != hipSuccess)
    return fail(c, PHIMVS_E_DEVICE, std::string("scratch of the allocation-free entry point: ") + hipGetErrorString(e));
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, launch_phi_hypotheses(depth, width, height, bits, hyp, c->stream));
  return PHIMVS_OK;
}

int phimvs_phi_costs(phimvs_ctx* c, const float* hyp, float* cost) {
  int rc = need_prepared(c);
  if (rc) return rc;
  if (!hyp || !cost) return fail(c, PHIMVS_E_ARG, "null array");
  HIPCHECK(c, hipSetDevice(c->device));
  // the hypotheses become the candidate slots of each colour in turn, and one evaluate
  // launch per colour scores the present ones through the compacted work list (pixels with
  // depth or without a hypothesis take no lane) and writes every slot's cost
  Batch& b = c->single;
  Job& J = b.jobs[0];
  const size_t n = (size_t)J.A.W * J.A.H;
  J.cost_out = cost;
  if ((rc = upload_jobs(c, b))) return rc;
  Launch L = base_launch(b);
  L.mode = 3;
  L.ncand = 4;
  for (int colour = 0; colour < 2 && !rc; ++colour) {
    L.colour = colour;
    const hipError_t e = launch_hyp_candidates(b.d_jobs, L, hyp, c->stream);
    if (e != hipSuccess) rc = fail(c, PHIMVS_E_DEVICE, std::string("hypothesis candidates: ") + hipGetErrorString(e));
    if (!rc) rc = eval_once(c, b, L);
  }
  J.cost_out = nullptr;
  const int rc2 = upload_jobs(c, b);  // the next upload drops the caller's pointer
  if (rc) return rc;
  if (rc2) return rc2;
  HIPCHECK(c, launch_phi_mask_cost(hyp, 4 * n, PHIMVS_COST_MAX, cost, c->stream));
  return PHIMVS_OK;
}

void phimvs_default_phi_params(phimvs_phi_params* p) {
  if (!p) return;
  p->k1 = 1.0;
  p->k2 = 0.1;
  p->k3 = 2.0;
  p->iterations = 8;
}

int phimvs_phi_select(phimvs_ctx* c, int width, int height, const float* depth, const float* hyp, const float* cost,
                      const phimvs_phi_params* pp, float* depth_out) {
  if (!c) return PHIMVS_E_ARG;
  if (width < 1 || height < 1 || !depth || !hyp || !cost || !depth_out)
    return fail(c, PHIMVS_E_ARG, "invalid size or null array");
  phimvs_phi_params p;
  phimvs_default_phi_params(&p);
  if (pp) p = *pp;
  HIPCHECK(c, hipSetDevice(c->device));
  const int W = width, H = height;
  // half size: node (X, Y) takes pixel (2X, 2Y); the GPU gathers the nodes' inputs (depth,
  // 4 hypotheses, 4 costs) and the host decodes
  const int W2 = (W + 1) / 2, H2 = (H + 1) / 2;
  const size_t n2 = (size_t)W2 * H2;
  int rc;
  if ((rc = ensure(c, c->io_a, 10 * n2))) return rc;
  float* half = c->io_a.p;
  float* dec_d = c->io_a.p + 9 * n2;
  HIPCHECK(c, launch_phi_half(depth, hyp, cost, W, H, half, c->stream));
  std::vector<float> h, dec;
  std::vector<int32_t> lab;
  try {
    h.resize(9 * n2);
    dec.resize(n2);
    lab.resize(n2);
  } catch (const std::bad_alloc&) {
    return fail(c, PHIMVS_E_OOM, "out of host memory for the graph model");
  }
  HIPCHECK(c, hipMemcpyAsync(h.data(), half, 9 * n2 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  rc = phimvs_phi_decode_host(W2, H2, h.data(), h.data() + n2, h.data() + 5 * n2, p.k1, p.k2, p.k3, PHIMVS_COST_MAX,
                              p.iterations, lab.data(), dec.data());
  if (rc == PHIMVS_E_OOM) return fail(c, rc, "out of host memory in the graph-model decoder");
  if (rc == PHIMVS_E_UNSUPPORTED) return fail(c, rc, "graph model too large for the decoder (2^27 nodes or more)");
  if (rc != PHIMVS_OK)
    return fail(c, PHIMVS_E_ARG,
                "invalid PHI parameters or costs (k1 > 0, k2 > 0, k3 > 1, iterations >= 0, cost <= C_max + k1 k2)");
  // back to full size in the kernel: pixel (x, y) reads node (x / 2, y / 2)
  HIPCHECK(c, hipMemcpyAsync(dec_d, dec.data(), n2 * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHECK(c, launch_phi_select(depth, hyp, dec_d, W, H, depth_out, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));  // the host copy of the decoded map goes out of scope
  return PHIMVS_OK;
}

int phimvs_phi_normals(phimvs_ctx* c, int view, const float* depth, float* normal_out) {
  if (!c) return PHIMVS_E_ARG;
  if (view < 0 || view >= (int)c->views.size()) return fail(c, PHIMVS_E_ARG, "view index out of range");
  if (!depth || !normal_out) return fail(c, PHIMVS_E_ARG, "null array");
  HIPCHECK(c, hipSetDevice(c->device));
  const ViewData& V = c->views[view];
  PhiCam cam{};
  if (!inv33(V.K, cam.Kinv)) return fail(c, PHIMVS_E_ARG, "singular K");
  HIPCHECK(c, launch_phi_normals(depth, V.W, V.H, cam, normal_out, c->stream));
  return PHIMVS_OK;
}

// ---------------------------------------------------------------------------- batches

int phimvs_patchmatch_batch(phimvs_ctx* c, int n_jobs, const phimvs_job* jobs, int iters, int use_graph) {
  if (!c) return PHIMVS_E_ARG;
  if (n_jobs < 1 || !jobs) return fail(c, PHIMVS_E_ARG, "need at least one job");
  if (iters < 0) return fail(c, PHIMVS_E_ARG, "iters must be >= 0");
  HIPCHECK(c, hipSetDevice(c->device));
  Batch& b = c->multi;
  std::vector<Problem> probs;
  std::string key = std::to_string(c->tuning.tile_rows);
  for (int i = 0; i < n_jobs; ++i) {
    const phimvs_job& j = jobs[i];
    if (j.n_srcs < 1 || !j.srcs) return fail(c, PHIMVS_E_ARG, "job " + std::to_string(i) + ": no source views");
    Problem P = make_problem(j.ref, j.srcs, j.n_srcs, j.window, j.dilation, &j.params);
    int rc = validate_problem(c, P);
    if (rc) return fail(c, rc, "job " + std::to_string(i) + ": " + c->err);
    if (P.p.lanes > 1)
      return fail(c, PHIMVS_E_UNSUPPORTED, "job " + std::to_string(i) + ": lanes > 1 is for single-job calls");
    probs.push_back(P);
    key += "|" + problem_key(P);
  }
  int rc;
  if (key != b.layout_key) {
    release_graph(b);
    resize_jobs(b, (size_t)n_jobs);
    for (int i = 0; i < n_jobs; ++i)
      if ((rc = setup_job(c, probs[i], b.jobs[i], b.state[i]))) return rc;
    layout(b, c->tuning.tile_rows);
    b.layout_key = key;
  }
  bool changed = false;
  for (int i = 0; i < n_jobs; ++i) {
    Job& J = b.jobs[i];
    changed = changed || J.depth_out != jobs[i].depth || J.normal_out != jobs[i].normal ||
              J.final_cost_out != jobs[i].cost;
    J.depth_out = jobs[i].depth;
    J.normal_out = jobs[i].normal;
    J.final_cost_out = jobs[i].cost;
  }
  if (changed || !b.exec) {
    if ((rc = upload_jobs(c, b))) return rc;  // the table is read at run time, also by the graph
  }
  if ((rc = ensure(c, b.queues, (size_t)8 * (2 + 4 * iters)))) return rc;
  const std::string gkey = key + "#" + std::to_string(iters) + "#" + std::to_string(c->tuning.persistent) + "#" +
                           std::to_string(c->tuning.wgs_per_cu) + "#" + std::to_string(c->tuning.order_by_depth);
  if (!use_graph || c->diag) return issue_sequence(c, b, iters, true);
  return run_sequence_graph(c, b, gkey, iters);
}

int phimvs_set_tuning(phimvs_ctx* c, const phimvs_tuning* t) {
  if (!c || !t) return PHIMVS_E_ARG;
  if (t->tile_rows != 1 && t->tile_rows != 2 && t->tile_rows != 4)
    return fail(c, PHIMVS_E_ARG, "tile_rows must be 1, 2 or 4");
  if (t->persistent && (t->wgs_per_cu < 1 || t->wgs_per_cu > 16))
    return fail(c, PHIMVS_E_ARG, "wgs_per_cu must be in [1, 16] for persistent launches");
  if (t->order_by_depth < 0 || t->order_by_depth > 7)
    return fail(c, PHIMVS_E_ARG, "order_by_depth is a mask of 1 (initialisation), 2 (propagation), 4 (refinement)");
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const bool shape = t->tile_rows != c->tuning.tile_rows;
  c->tuning = *t;
  c->tuning.ms = 0.0;
  if (shape) {
    // the tile shape changes the layout of every job: rebuild on next use
    c->prepared = false;
    c->single.layout_key.clear();
    c->multi.layout_key.clear();
  }
  release_graph(c->multi);
  return PHIMVS_OK;
}

int phimvs_get_tuning(phimvs_ctx* c, phimvs_tuning* t) {
  if (!c || !t) return PHIMVS_E_ARG;
  *t = c->tuning;
  return PHIMVS_OK;
}

int phimvs_autotune(phimvs_ctx* c, int n_jobs, const phimvs_job* jobs, int iters, phimvs_tuning* results,
                    int* n_results) {
  if (!c) return PHIMVS_E_ARG;
  HIPCHECK(c, hipSetDevice(c->device));
  // ten launch shapes in pixel order; the last trial is the fastest of them in depth order
  phimvs_tuning cands[] = {{4, 0, 0, 0, 0}, {2, 0, 0, 0, 0}, {1, 0, 0, 0, 0}, {4, 1, 2, 0, 0},
                           {4, 1, 3, 0, 0}, {4, 1, 4, 0, 0}, {4, 1, 6, 0, 0}, {2, 1, 3, 0, 0},
                           {2, 1, 4, 0, 0}, {1, 1, 4, 0, 0}, {4, 1, 4, 1, 0}};
  const int n = (int)(sizeof(cands) / sizeof(cands[0]));
  const phimvs_tuning prev = c->tuning;
  phimvs_tuning best{};
  double best_ms = HUGE_VAL;
  std::string failures;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto destroy = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    destroy();
    return fail(c, PHIMVS_E_DEVICE, "autotune: hipEventCreate failed");
  }
  // a configuration that fails (its launch refused, say) is reported with ms = +inf and
  // passed over; the others are still timed
  for (int i = 0; i < n; ++i) {
    if (i == n - 1 && best_ms < HUGE_VAL) {
      cands[i] = best;
      cands[i].order_by_depth = 7;
      cands[i].ms = 0.0;
    }
    phimvs_tuning r = cands[i];
    r.ms = HUGE_VAL;
    int rc = phimvs_set_tuning(c, &cands[i]);
    if (!rc) rc = phimvs_patchmatch_batch(c, n_jobs, jobs, iters, 1);  // capture + warm
    if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(c, PHIMVS_E_DEVICE, "hipEventRecord");
    if (!rc) rc = phimvs_patchmatch_batch(c, n_jobs, jobs, iters, 1);
    if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = fail(c, PHIMVS_E_DEVICE, "hipEventRecord");
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(c, PHIMVS_E_DEVICE, "hipEventSynchronize");
    float ms = 0.f;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(c, PHIMVS_E_DEVICE, "hipEventElapsedTime");
    if (rc) {
      failures += " [rows " + std::to_string(cands[i].tile_rows) + ", persistent " +
                  std::to_string(cands[i].persistent) + ", " + std::to_string(cands[i].wgs_per_cu) + "/CU, order " +
                  std::to_string(cands[i].order_by_depth) + ": " + c->err + "]";
    } else {
      r.ms = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = r;
      }
    }
    if (results && n_results && i < *n_results) results[i] = r;
  }
  destroy();
  if (n_results) *n_results = std::min(*n_results, n);
  if (!(best_ms < HUGE_VAL)) {
    (void)phimvs_set_tuning(c, &prev);
    return fail(c, PHIMVS_E_DEVICE, "autotune: no configuration ran:" + failures);
  }
  int rc = phimvs_set_tuning(c, &best);
  if (rc) return rc;
  c->tuning.ms = best_ms;
  c->err = failures.empty() ? std::string() : "autotune: configurations passed over:" + failures;
  return PHIMVS_OK;
}

// ---------------------------------------------------------------------------- diagnostics

int phimvs_diag_enable(phimvs_ctx* c, int flags) {
  if (!c) return PHIMVS_E_ARG;
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  for (auto& e : c->diag_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  c->diag_events.clear();
  if (!c->diag_count) HIPCHECK(c, hipMalloc((void**)&c->diag_count, sizeof(unsigned long long)));
  HIPCHECK(c, hipMemset(c->diag_count, 0, sizeof(unsigned long long)));
  c->diag = flags & (PHIMVS_DIAG_COUNT | PHIMVS_DIAG_TIME);
  return PHIMVS_OK;
}

int phimvs_diag_read(phimvs_ctx* c, uint64_t* hypotheses, uint64_t* launches, double* kernel_ms) {
  if (!c) return PHIMVS_E_ARG;
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  unsigned long long n = 0;
  if (c->diag_count) HIPCHECK(c, hipMemcpy(&n, c->diag_count, sizeof n, hipMemcpyDeviceToHost));
  double ms = 0.0;
  for (auto& e : c->diag_events) {
    float t = 0.f;
    HIPCHECK(c, hipEventElapsedTime(&t, e.first, e.second));
    ms += t;
  }
  if (hypotheses) *hypotheses = n;
  if (launches) *launches = c->diag_events.size();
  if (kernel_ms) *kernel_ms = ms;
  return PHIMVS_OK;
}

int phimvs_check_reciprocal(phimvs_ctx* c, uint32_t first_bits, uint32_t count, uint64_t* mismatches,
                            uint32_t* example_bits) {
  if (!c || !mismatches) return PHIMVS_E_ARG;
  HIPCHECK(c, hipSetDevice(c->device));
  unsigned long long* dm = nullptr;
  uint32_t* de = nullptr;
  HIPCHECK(c, hipMalloc((void**)&dm, sizeof(unsigned long long)));
  HIPCHECK(c, hipMalloc((void**)&de, sizeof(uint32_t)));
  HIPCHECK(c, hipMemsetAsync(dm, 0, sizeof(unsigned long long), c->stream));
  HIPCHECK(c, hipMemsetAsync(de, 0, sizeof(uint32_t), c->stream));
  HIPCHECK(c, launch_rcp_check(first_bits, count, dm, de, c->stream));
  unsigned long long hm = 0;
  uint32_t he = 0;
  HIPCHECK(c, hipMemcpyAsync(&hm, dm, sizeof hm, hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipMemcpyAsync(&he, de, sizeof he, hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  (void)hipFree(dm);
  (void)hipFree(de);
  *mismatches = hm;
  if (example_bits) *example_bits = he;
  return PHIMVS_OK;
}

}  // extern "C"
