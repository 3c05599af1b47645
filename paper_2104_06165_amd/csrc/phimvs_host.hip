// Host side of the PatchMatch library: the C ABI declared in phimvs.h.
//
// Responsibilities: argument validation, the FP64 per-problem constants (relative
// poses, M_j = K_j R_rel K_0^-1, e_j = K_j t_rel, K_0^-1, bilateral weight tables),
// device memory for views and state, and the launch sequence of the depth-map
// estimation step (Algorithm 1: initialisation, then per iteration a red and a
// black half-sweep).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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

}  // namespace

struct phimvs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<ViewData> views;
  bool prepared = false;
  Args args{};
  int ref = -1;
  std::vector<int> srcs;
  DevBuf<float4> plane[2];
  DevBuf<float> cost[2];
  DevBuf<float4> cand;  // up to 8 candidate planes per pixel of one colour
  DevBuf<float> wcol, wsp;
  std::vector<float> wcol_h, wsp_h;
  DevBuf<float> io_a, io_b, io_c;  // staging for host inputs / outputs
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

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// C = A B (3x3, row-major), summed left to right
void mul33(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i * 3 + 0] * B[0 * 3 + j] + A[i * 3 + 1] * B[1 * 3 + j] + A[i * 3 + 2] * B[2 * 3 + j];
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

int validate_params(phimvs_ctx* c, const phimvs_params& p, int n_srcs) {
  if (p.top_k < 0 || p.top_k > n_srcs) return fail(c, PHIMVS_E_ARG, "top_k must be in [0, n_srcs]");
  if (!std::isfinite(p.sigma_spatial_px) || !(std::isfinite(p.sigma_color) && p.sigma_color > 0))
    return fail(c, PHIMVS_E_ARG, "bilateral sigmas must be finite, sigma_color > 0");
  if (!(p.eps_var >= 0 && std::isfinite(p.eps_var)) || !(p.eps_cost > 0 && std::isfinite(p.eps_cost)))
    return fail(c, PHIMVS_E_ARG, "eps_var must be >= 0 and eps_cost > 0");
  return PHIMVS_OK;
}

}  // namespace

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
  for (int k = 0; k < 2; ++k) {
    release(c->plane[k]);
    release(c->cost[k]);
  }
  release(c->cand);
  release(c->wcol);
  release(c->wsp);
  release(c->io_a);
  release(c->io_b);
  release(c->io_c);
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
  c->stream = (hipStream_t)hip_stream;
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
  if (!c) return PHIMVS_E_ARG;
  c->prepared = false;
  const int nv = (int)c->views.size();
  if (nv == 0) return fail(c, PHIMVS_E_STATE, "no views: call phimvs_set_views first");
  if (ref < 0 || ref >= nv) return fail(c, PHIMVS_E_ARG, "ref out of range");
  if (n_srcs < 1 || !srcs) return fail(c, PHIMVS_E_ARG, "need at least one source view");
  if (n_srcs > 12) return fail(c, PHIMVS_E_UNSUPPORTED, "at most 12 source views per reference");
  for (int i = 0; i < n_srcs; ++i) {
    if (srcs[i] < 0 || srcs[i] >= nv) return fail(c, PHIMVS_E_ARG, "source index out of range");
    if (srcs[i] == ref) return fail(c, PHIMVS_E_ARG, "the reference cannot be one of its sources");
    for (int k = 0; k < i; ++k)
      if (srcs[k] == srcs[i]) return fail(c, PHIMVS_E_ARG, "duplicate source view");
  }
  if (dilation < 1) return fail(c, PHIMVS_E_ARG, "dilation must be >= 1");
  if (window < 3 || window % 2 == 0 || (window - 1) % (2 * dilation) != 0)
    return fail(c, PHIMVS_E_ARG, "window must be odd with (window - 1) % (2 dilation) == 0");
  const int R = (window - 1) / (2 * dilation);
  if (R > 15) return fail(c, PHIMVS_E_UNSUPPORTED, "at most 31 taps per window side");
  if (dilation * R > 30) return fail(c, PHIMVS_E_UNSUPPORTED, "window radius above 30 px");
  phimvs_params p;
  if (pp) p = *pp;
  else phimvs_default_params(&p);
  int rc = validate_params(c, p, n_srcs);
  if (rc) return rc;

  const ViewData& V0 = c->views[ref];
  Args& A = c->args;
  A = Args{};
  A.W = V0.W;
  A.H = V0.H;
  A.Wc = (V0.W + 1) / 2;
  A.R = R;
  A.s = dilation;
  A.n_src = n_srcs;
  A.top_k = p.top_k;
  A.bilateral = p.bilateral ? 1 : 0;
  A.TW = 128 + 2 * dilation * R;
  A.TH = 4 + 2 * dilation * R;
  A.n_taps = (2 * R + 1) * (2 * R + 1);
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
  for (int k = 0; k < n_srcs; ++k) {
    const ViewData& Vj = c->views[srcs[k]];
    double Rrel[9], Rt0[3], trel[3], KR[9], M[9], e[3];
    mul33(Vj.R, R0t, Rrel);
    mulv3(Rrel, V0.t, Rt0);
    for (int i = 0; i < 3; ++i) trel[i] = Vj.t[i] - Rt0[i];
    mul33(Vj.K, Rrel, KR);
    mul33(KR, K0i, M);
    mulv3(Vj.K, trel, e);
    SrcDev& S = A.src[k];
    for (int i = 0; i < 9; ++i) S.M[i] = (float)M[i];
    for (int i = 0; i < 3; ++i) S.e[i] = (float)e[i];
    S.W = Vj.W;
    S.H = Vj.H;
    S.Wm1 = (float)(Vj.W - 1);
    S.Hm1 = (float)(Vj.H - 1);
    S.quad = Vj.quad;
  }
  // bilateral weight factors: colour (|a - a_c| = 0..255) and space (tap offsets)
  const double sc = p.sigma_color;
  const double ss = p.sigma_spatial_px > 0 ? p.sigma_spatial_px : (double)((window - 1) / 2);
  std::vector<float> wc(256), ws(A.n_taps);
  for (int i = 0; i < 256; ++i) {
    const double d = (double)i;
    wc[i] = p.bilateral ? (float)std::exp(-(d * d) / (2.0 * sc * sc)) : 1.0f;
  }
  for (int k2 = -R, t = 0; k2 <= R; ++k2)
    for (int k1 = -R; k1 <= R; ++k1, ++t) {
      const double r2 = (double)(dilation * dilation) * (double)(k1 * k1 + k2 * k2);
      ws[t] = p.bilateral ? (float)std::exp(-r2 / (2.0 * ss * ss)) : 1.0f;
    }
  HIPCHECK(c, hipSetDevice(c->device));
  if (ws != c->wsp_h || wc != c->wcol_h || !c->wcol.p || !c->wsp.p) {
    if ((rc = ensure(c, c->wcol, 256))) return rc;
    if ((rc = ensure(c, c->wsp, ws.size()))) return rc;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(c->wcol.p, wc.data(), 256 * sizeof(float), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->wsp.p, ws.data(), ws.size() * sizeof(float), hipMemcpyHostToDevice));
    c->wcol_h = wc;
    c->wsp_h = ws;
  }
  A.wcol = c->wcol.p;
  A.wsp = c->wsp.p;
  const size_t ncol = (size_t)A.Wc * A.H;
  for (int k = 0; k < 2; ++k) {
    if ((rc = ensure(c, c->plane[k], ncol))) return rc;
    if ((rc = ensure(c, c->cost[k], ncol))) return rc;
    A.plane[k] = c->plane[k].p;
    A.cost[k] = c->cost[k].p;
  }
  if ((rc = ensure(c, c->cand, 8 * ncol))) return rc;
  c->ref = ref;
  c->srcs.assign(srcs, srcs + n_srcs);
  c->prepared = true;
  return PHIMVS_OK;
}

// evaluate-and-select launch with the optional diagnostics around it
static hipError_t run_select(phimvs_ctx* c, int mode, Step S) {
  hipError_t e;
  if (c->diag & PHIMVS_DIAG_COUNT) S.count = c->diag_count;
  if (c->diag & PHIMVS_DIAG_TIME) {
    hipEvent_t a, b;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return e;
    c->diag_events.emplace_back(a, b);
    if ((e = hipEventRecord(a, c->stream)) != hipSuccess) return e;
    if ((e = launch_select(mode, c->args, S, c->stream)) != hipSuccess) return e;
    return hipEventRecord(b, c->stream);
  }
  return launch_select(mode, c->args, S, c->stream);
}

static int need_prepared(phimvs_ctx* c) {
  if (!c) return PHIMVS_E_ARG;
  if (!c->prepared) return fail(c, PHIMVS_E_STATE, "call phimvs_prepare first");
  return PHIMVS_OK;
}

// device pointer for an input array: either the caller's, or a staging copy of host data
static int input_ptr(phimvs_ctx* c, DevBuf<float>& stage, const float* p, size_t n, int on_device,
                     const float** out) {
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

int phimvs_init_planes(phimvs_ctx* c, const float* proposal, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  HIPCHECK(c, hipSetDevice(c->device));
  Step S{};
  S.cand = c->cand.p;
  S.ncand = 1;
  if (proposal) {
    if ((rc = input_ptr(c, c->io_a, proposal, (size_t)c->args.W * c->args.H * 4, on_device, &S.planes_in))) return rc;
    S.ncand = 2;
  }
  for (int colour = 0; colour < 2; ++colour) {
    S.colour = colour;
    HIPCHECK(c, launch_candidates(0, c->args, S, c->stream));
    HIPCHECK(c, run_select(c, 0, S));
  }
  if (proposal && !on_device) HIPCHECK(c, hipStreamSynchronize(c->stream));
  return PHIMVS_OK;
}

int phimvs_step(phimvs_ctx* c, int iteration, int colour, int do_propagate, int do_refine) {
  int rc = need_prepared(c);
  if (rc) return rc;
  if (colour != 0 && colour != 1) return fail(c, PHIMVS_E_ARG, "colour must be 0 or 1");
  if (iteration < 1) return fail(c, PHIMVS_E_ARG, "iteration must be >= 1");
  HIPCHECK(c, hipSetDevice(c->device));
  Step S{};
  S.colour = colour;
  S.iteration = iteration;
  S.cand = c->cand.p;
  if (do_propagate) {
    S.ncand = 8;
    HIPCHECK(c, launch_candidates(1, c->args, S, c->stream));
    HIPCHECK(c, run_select(c, 1, S));
  }
  if (do_refine) {
    S.ncand = 3;
    HIPCHECK(c, launch_candidates(2, c->args, S, c->stream));
    HIPCHECK(c, run_select(c, 1, S));
  }
  return PHIMVS_OK;
}

static int finish_outputs(phimvs_ctx* c, int on_device, std::initializer_list<std::pair<float*, DevBuf<float>*>> outs,
                          std::initializer_list<size_t> sizes) {
  if (on_device) return PHIMVS_OK;
  auto sz = sizes.begin();
  for (auto& o : outs) {
    if (o.first) HIPCHECK(c, hipMemcpyAsync(o.first, o.second->p, *sz * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    ++sz;
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return PHIMVS_OK;
}

int phimvs_get_state(phimvs_ctx* c, float* planes, float* cost, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  HIPCHECK(c, hipSetDevice(c->device));
  const size_t n = (size_t)c->args.W * c->args.H;
  float* dp = planes;
  float* dc = cost;
  if (!on_device) {
    if ((rc = ensure(c, c->io_a, 4 * n)) || (rc = ensure(c, c->io_b, n))) return rc;
    dp = planes ? c->io_a.p : nullptr;
    dc = cost ? c->io_b.p : nullptr;
  }
  HIPCHECK(c, launch_unpack(c->args, dp, nullptr, nullptr, dc, c->stream));
  return finish_outputs(c, on_device, {{planes, &c->io_a}, {cost, &c->io_b}}, {4 * n, n});
}

int phimvs_set_state(phimvs_ctx* c, const float* planes, const float* cost, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  if (!planes || !cost) return fail(c, PHIMVS_E_ARG, "set_state needs planes and cost");
  HIPCHECK(c, hipSetDevice(c->device));
  const size_t n = (size_t)c->args.W * c->args.H;
  const float *dp, *dc;
  if ((rc = input_ptr(c, c->io_a, planes, 4 * n, on_device, &dp))) return rc;
  if ((rc = input_ptr(c, c->io_b, cost, n, on_device, &dc))) return rc;
  HIPCHECK(c, launch_pack(c->args, dp, dc, c->stream));
  if (!on_device) HIPCHECK(c, hipStreamSynchronize(c->stream));
  return PHIMVS_OK;
}

int phimvs_output(phimvs_ctx* c, float* depth, float* normal, float* cost, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  HIPCHECK(c, hipSetDevice(c->device));
  const size_t n = (size_t)c->args.W * c->args.H;
  float *dd = depth, *dn = normal, *dc = cost;
  if (!on_device) {
    if ((rc = ensure(c, c->io_a, 3 * n)) || (rc = ensure(c, c->io_b, n)) || (rc = ensure(c, c->io_c, n))) return rc;
    dn = normal ? c->io_a.p : nullptr;
    dd = depth ? c->io_b.p : nullptr;
    dc = cost ? c->io_c.p : nullptr;
  }
  HIPCHECK(c, launch_unpack(c->args, nullptr, dd, dn, dc, c->stream));
  return finish_outputs(c, on_device, {{normal, &c->io_a}, {depth, &c->io_b}, {cost, &c->io_c}}, {3 * n, n, n});
}

int phimvs_eval_cost(phimvs_ctx* c, const float* planes, float* cost, float* per_view, uint8_t* valid, int on_device) {
  int rc = need_prepared(c);
  if (rc) return rc;
  if (!planes || !cost) return fail(c, PHIMVS_E_ARG, "eval_cost needs planes and cost");
  HIPCHECK(c, hipSetDevice(c->device));
  const size_t n = (size_t)c->args.W * c->args.H;
  const size_t nv = (size_t)c->args.n_src;
  Step S{};
  if ((rc = input_ptr(c, c->io_a, planes, 4 * n, on_device, &S.planes_in))) return rc;
  S.cost_out = cost;
  S.per_view_out = per_view;
  S.valid_out = valid;
  if (!on_device) {
    if ((rc = ensure(c, c->io_b, n)) || (rc = ensure(c, c->io_c, per_view ? n * nv : 1)) ||
        (rc = ensure(c, c->io_u8, valid ? n * nv : 1)))
      return rc;
    S.cost_out = c->io_b.p;
    S.per_view_out = per_view ? c->io_c.p : nullptr;
    S.valid_out = valid ? c->io_u8.p : nullptr;
  }
  for (int colour = 0; colour < 2; ++colour) {
    S.colour = colour;
    HIPCHECK(c, run_select(c, 2, S));
  }
  if (!on_device) {
    HIPCHECK(c, hipMemcpyAsync(cost, c->io_b.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (per_view) HIPCHECK(c, hipMemcpyAsync(per_view, c->io_c.p, n * nv * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (valid) HIPCHECK(c, hipMemcpyAsync(valid, c->io_u8.p, n * nv, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
  }
  return PHIMVS_OK;
}

int phimvs_patchmatch(phimvs_ctx* c, int ref, const int* srcs, int n_srcs, int window, int dilation, int iters,
                      const phimvs_params* p, float* depth, float* normal, float* cost, int out_on_device) {
  if (!c) return PHIMVS_E_ARG;
  if (iters < 0) return fail(c, PHIMVS_E_ARG, "iters must be >= 0");
  int rc = phimvs_prepare(c, ref, srcs, n_srcs, window, dilation, p);
  if (rc) return rc;
  if ((rc = phimvs_init_planes(c, nullptr, 0))) return rc;
  for (int it = 1; it <= iters; ++it)
    for (int colour = 0; colour < 2; ++colour)
      if ((rc = phimvs_step(c, it, colour, 1, 1))) return rc;
  return phimvs_output(c, depth, normal, cost, out_on_device);
}

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
