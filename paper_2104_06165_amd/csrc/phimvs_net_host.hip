// Host side of the learned initial-plane proposal: parameters, Adam state, activation
// buffers, and the layer-by-layer forward and backward passes built from the kernels in
// phimvs_net.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "phimvs.h"
#include "phimvs_internal.h"
#include "phimvs_net.h"
#include "phimvs_net_internal.h"

using namespace phimvs_net_internal;

namespace {

constexpr int kLayers = PHIMVS_NET_LAYERS;
constexpr int kCin[kLayers] = {PHIMVS_NET_IN, 32, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 32, PHIMVS_NET_OUT};
constexpr int kCip[kLayers] = {16, 32, 32, 32, 32};   // padded to multiples of 16
constexpr int kCop[kLayers] = {32, 32, 32, 32, 16};

constexpr int64_t layer_params(int l) { return 9LL * kCin[l] * kCout[l] + kCout[l]; }
constexpr int64_t total_params() {
  int64_t n = 0;
  for (int l = 0; l < kLayers; ++l) n += layer_params(l);
  return n;
}
int64_t layer_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += layer_params(i);
  return o;
}

template <typename T>
struct Buf {
  T* p = nullptr;
  size_t n = 0;
};

}  // namespace

struct phimvs_net {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  float* params = nullptr;  // fp32 master parameters
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t adam_t = 0;
  bool have_grad = false;
  uint16_t* wfwd[kLayers] = {};   // [9][COP][CIP] bf16
  uint16_t* wflip[kLayers] = {};  // [9][CIP][COP] bf16, taps mirrored (data gradient)
  Buf<uint16_t> act[kLayers + 1];  // act[0]: input (16 ch); act[l]: output of layer l (32 ch)
  Buf<uint16_t> g16[kLayers];      // g16[l]: gradient at the output of layer l (kCop[l] ch)
  int last_B = 0, last_h = 0, last_w = 0;  // shape of the last forward pass
  bool have_act = false;   // act[] hold the last forward pass
  bool have_bwd = false;   // g16[] hold the backward pass of that forward pass
  Buf<float> out32, partial, partial_b, gpad, gbias, loss_partial, tmp_in, tmp_out;
};

namespace {

int fail(phimvs_net* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  return code;
}

#define NCHECK(net, call)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(net, e_ == hipErrorOutOfMemory ? PHIMVS_E_OOM : PHIMVS_E_DEVICE,                 \
                  std::string(#call) + ": " + hipGetErrorString(e_));                               \
  } while (0)

template <typename T>
int ensure(phimvs_net* n, Buf<T>& b, size_t count) {
  if (b.p && b.n >= count) return PHIMVS_OK;
  if (b.p) NCHECK(n, hipFree(b.p));
  b.p = nullptr;
  b.n = 0;
  NCHECK(n, hipMalloc(&b.p, std::max<size_t>(count, 1) * sizeof(T)));
  b.n = count;
  return PHIMVS_OK;
}

template <typename T>
void release(Buf<T>& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.n = 0;
}

int repack(phimvs_net* n) {
  for (int l = 0; l < kLayers; ++l)
    NCHECK(n, launch_pack_weights(n->params + layer_offset(l), kCin[l], kCout[l], kCip[l], kCop[l], n->wfwd[l],
                                  n->wflip[l], n->stream));
  return PHIMVS_OK;
}

int check_shape(phimvs_net* n, int batch, int h, int w) {
  if (batch < 1 || h < 1 || w < 1) return fail(n, PHIMVS_E_ARG, "batch, height and width must be >= 1");
  if ((int64_t)batch * h * w > (1LL << 28)) return fail(n, PHIMVS_E_ARG, "input too large");
  return PHIMVS_OK;
}

// forward pass; keeps every layer's bf16 output in act[] (training needs them)
int forward(phimvs_net* n, int B, int h, int w, const float* input, float* output) {
  const size_t np = (size_t)B * h * w;
  int rc;
  if ((rc = ensure(n, n->act[0], np * kCip[0]))) return rc;
  for (int l = 1; l < kLayers; ++l)
    if ((rc = ensure(n, n->act[l], np * kCop[l - 1]))) return rc;
  n->have_act = false;
  n->have_bwd = false;
  NCHECK(n, launch_to_bf16(input, (int)np, PHIMVS_NET_IN, kCip[0], n->act[0].p, n->stream));
  for (int l = 0; l < kLayers; ++l) {
    ConvArgs a{};
    a.B = B;
    a.h = h;
    a.w = w;
    a.CI = kCip[l];
    a.CO = kCop[l];
    a.x = n->act[l].p;
    a.wt = n->wfwd[l];
    a.bias = n->params + layer_offset(l) + 9LL * kCin[l] * kCout[l];
    a.n_bias = kCout[l];
    const bool last = l == kLayers - 1;
    a.relu = last ? 0 : 1;
    a.mask16 = nullptr;
    a.y16 = last ? nullptr : n->act[l + 1].p;
    a.y32 = last ? output : nullptr;
    a.co_keep = last ? PHIMVS_NET_OUT : 0;
    NCHECK(n, launch_conv(a, n->stream));
  }
  n->last_B = B;
  n->last_h = h;
  n->last_w = w;
  n->have_act = true;
  return PHIMVS_OK;
}

}  // namespace

extern "C" {

int64_t phimvs_net_param_count(void) { return total_params(); }

int phimvs_net_create(phimvs_net** out, int device_ordinal, void* hip_stream) {
  if (!out) return PHIMVS_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device_ordinal < 0 || device_ordinal >= count)
    return PHIMVS_E_DEVICE;
  phimvs_net* n = new phimvs_net;
  n->device = device_ordinal;
  n->stream = (hipStream_t)hip_stream;
  const size_t np = (size_t)total_params();
  bool ok = hipSetDevice(device_ordinal) == hipSuccess && hipMalloc(&n->params, np * sizeof(float)) == hipSuccess &&
            hipMalloc(&n->grad, np * sizeof(float)) == hipSuccess &&
            hipMalloc(&n->adam_m, np * sizeof(float)) == hipSuccess &&
            hipMalloc(&n->adam_v, np * sizeof(float)) == hipSuccess;
  for (int l = 0; ok && l < kLayers; ++l) {
    const size_t nw = 9 * (size_t)kCip[l] * kCop[l];
    ok = hipMalloc(&n->wfwd[l], nw * 2) == hipSuccess && hipMalloc(&n->wflip[l], nw * 2) == hipSuccess;
  }
  if (ok) {
    std::vector<float> zero(np, 0.f);
    ok = hipMemcpy(n->params, zero.data(), np * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(n->adam_m, zero.data(), np * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(n->adam_v, zero.data(), np * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         repack(n) == PHIMVS_OK && hipStreamSynchronize(n->stream) == hipSuccess;
  }
  if (!ok) {
    phimvs_net_destroy(n);
    return PHIMVS_E_DEVICE;
  }
  *out = n;
  return PHIMVS_OK;
}

void phimvs_net_destroy(phimvs_net* n) {
  if (!n) return;
  (void)hipSetDevice(n->device);
  (void)hipStreamSynchronize(n->stream);
  for (float* p : {n->params, n->grad, n->adam_m, n->adam_v})
    if (p) (void)hipFree(p);
  for (int l = 0; l < kLayers; ++l) {
    if (n->wfwd[l]) (void)hipFree(n->wfwd[l]);
    if (n->wflip[l]) (void)hipFree(n->wflip[l]);
  }
  for (auto& b : n->act) release(b);
  for (auto& b : n->g16) release(b);
  for (auto* b : {&n->out32, &n->partial, &n->partial_b, &n->gpad, &n->gbias, &n->loss_partial, &n->tmp_in, &n->tmp_out})
    release(*b);
  delete n;
}

const char* phimvs_net_last_error(const phimvs_net* n) { return n ? n->err.c_str() : "null network"; }

int phimvs_net_set_stream(phimvs_net* n, void* hip_stream) {
  if (!n) return PHIMVS_E_ARG;
  n->stream = (hipStream_t)hip_stream;
  return PHIMVS_OK;
}

int phimvs_net_set_params(phimvs_net* n, const float* params, int on_device) {
  if (!n || !params) return fail(n, PHIMVS_E_ARG, "null argument");
  NCHECK(n, hipSetDevice(n->device));
  const size_t bytes = (size_t)total_params() * sizeof(float);
  NCHECK(n, hipMemcpyAsync(n->params, params, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           n->stream));
  NCHECK(n, hipMemsetAsync(n->adam_m, 0, bytes, n->stream));
  NCHECK(n, hipMemsetAsync(n->adam_v, 0, bytes, n->stream));
  n->adam_t = 0;
  n->have_grad = false;
  int rc = repack(n);
  if (rc) return rc;
  if (!on_device) NCHECK(n, hipStreamSynchronize(n->stream));
  return PHIMVS_OK;
}

int phimvs_net_get_params(phimvs_net* n, float* params, int on_device) {
  if (!n || !params) return fail(n, PHIMVS_E_ARG, "null argument");
  NCHECK(n, hipSetDevice(n->device));
  const size_t bytes = (size_t)total_params() * sizeof(float);
  NCHECK(n, hipMemcpyAsync(params, n->params, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           n->stream));
  if (!on_device) NCHECK(n, hipStreamSynchronize(n->stream));
  return PHIMVS_OK;
}

int phimvs_net_forward(phimvs_net* n, int batch, int height, int width, const float* input, float* output) {
  if (!n || !input || !output) return fail(n, PHIMVS_E_ARG, "null argument");
  int rc = check_shape(n, batch, height, width);
  if (rc) return rc;
  NCHECK(n, hipSetDevice(n->device));
  return forward(n, batch, height, width, input, output);
}

int phimvs_net_loss_grad(phimvs_net* n, int batch, int height, int width, const float* input, const float* target,
                         const float* mask, const float* depth_range, float normal_weight, double* loss, float* grad) {
  if (!n || !input || !target || !mask || !depth_range) return fail(n, PHIMVS_E_ARG, "null argument");
  int rc = check_shape(n, batch, height, width);
  if (rc) return rc;
  if (!(normal_weight >= 0.f)) return fail(n, PHIMVS_E_ARG, "normal_weight must be >= 0");
  NCHECK(n, hipSetDevice(n->device));
  const int B = batch, h = height, w = width;
  const size_t np = (size_t)B * h * w;
  if ((rc = ensure(n, n->out32, np * PHIMVS_NET_OUT))) return rc;
  if ((rc = forward(n, B, h, w, input, n->out32.p))) return rc;

  const int n_blocks = (int)((np + 255) / 256);
  if ((rc = ensure(n, n->loss_partial, n_blocks))) return rc;
  for (int l = 0; l < kLayers; ++l)
    if ((rc = ensure(n, n->g16[l], np * kCop[l]))) return rc;
  LossArgs la{};
  la.n_pix = (int)np;
  la.h = h;
  la.w = w;
  la.out = n->out32.p;
  la.target = target;
  la.mask = mask;
  la.drange = depth_range;
  la.inv_count = 1.f / (float)np;
  la.lambda = normal_weight;
  la.grad16 = n->g16[kLayers - 1].p;
  la.loss_partial = n->loss_partial.p;
  NCHECK(n, launch_loss(la, n->stream));

  const int rows = B * h;
  const size_t max_w = 9 * 32 * 32;
  if ((rc = ensure(n, n->partial, (size_t)rows * max_w)) || (rc = ensure(n, n->partial_b, (size_t)rows * 32)) ||
      (rc = ensure(n, n->gpad, max_w)) || (rc = ensure(n, n->gbias, 32)))
    return rc;
  for (int l = kLayers - 1; l >= 0; --l) {
    WgradArgs wa{};
    wa.B = B;
    wa.h = h;
    wa.w = w;
    wa.CI = kCip[l];
    wa.CO = kCop[l];
    wa.x = n->act[l].p;
    wa.g = n->g16[l].p;
    wa.partial = n->partial.p;
    wa.partial_bias = n->partial_b.p;
    NCHECK(n, launch_wgrad(wa, n->stream));
    const int nwp = 9 * kCip[l] * kCop[l];
    NCHECK(n, launch_reduce_rows(n->partial.p, rows, nwp, nwp, n->gpad.p, n->stream));
    NCHECK(n, launch_reduce_rows(n->partial_b.p, rows, kCop[l], kCop[l], n->gbias.p, n->stream));
    NCHECK(n, launch_unpad_grad(n->gpad.p, n->gbias.p, kCin[l], kCout[l], kCip[l], kCop[l],
                                n->grad + layer_offset(l), n->stream));
    if (l == 0) break;
    // data gradient into the input of layer l, through the ReLU of layer l - 1
    ConvArgs a{};
    a.B = B;
    a.h = h;
    a.w = w;
    a.CI = kCop[l];
    a.CO = kCip[l];
    a.x = n->g16[l].p;
    a.wt = n->wflip[l];
    a.bias = nullptr;
    a.relu = 0;
    a.mask16 = n->act[l].p;
    a.y16 = n->g16[l - 1].p;
    a.y32 = nullptr;
    a.co_keep = 0;
    NCHECK(n, launch_conv(a, n->stream));
  }
  n->have_grad = true;
  n->have_bwd = true;
  if (grad)
    NCHECK(n, hipMemcpyAsync(grad, n->grad, (size_t)total_params() * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
  if (loss) {
    std::vector<float> part(n_blocks);
    NCHECK(n, hipMemcpyAsync(part.data(), n->loss_partial.p, n_blocks * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NCHECK(n, hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (float v : part) s += v;
    *loss = s;
  }
  return PHIMVS_OK;
}

int phimvs_net_tensor(phimvs_net* n, int kind, int layer, float* out) {
  if (!n || !out) return fail(n, PHIMVS_E_ARG, "null argument");
  if ((kind != 0 && kind != 1) || layer < 0 || layer >= kLayers)
    return fail(n, PHIMVS_E_ARG, "kind must be 0 or 1 and layer in [0, " + std::to_string(kLayers - 1) + "]");
  if (kind == 0 && !n->have_act) return fail(n, PHIMVS_E_STATE, "no forward pass yet");
  if (kind == 1 && !n->have_bwd) return fail(n, PHIMVS_E_STATE, "call phimvs_net_loss_grad first");
  NCHECK(n, hipSetDevice(n->device));
  const int np = n->last_B * n->last_h * n->last_w;
  if (kind == 0)
    NCHECK(n, launch_bf16_unpad(n->act[layer].p, np, kCip[layer], kCin[layer], out, n->stream));
  else
    NCHECK(n, launch_bf16_unpad(n->g16[layer].p, np, kCop[layer], kCout[layer], out, n->stream));
  return PHIMVS_OK;
}

int phimvs_net_adam(phimvs_net* n, float lr, float beta1, float beta2, float eps) {
  if (!n) return PHIMVS_E_ARG;
  if (!n->have_grad) return fail(n, PHIMVS_E_STATE, "call phimvs_net_loss_grad first");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(n, PHIMVS_E_ARG, "invalid Adam hyper-parameters");
  NCHECK(n, hipSetDevice(n->device));
  n->adam_t += 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)n->adam_t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)n->adam_t));
  NCHECK(n, launch_adam(n->params, n->grad, n->adam_m, n->adam_v, (int)total_params(), lr, beta1, beta2, eps, c1, c2,
                        n->stream));
  return repack(n);
}

int phimvs_net_targets(phimvs_net* n, int width, int height, const float* depth, const float* normal,
                       const float* cost, float max_cost, float* target, float* mask) {
  if (!n || !depth || !normal || !cost || !target || !mask) return fail(n, PHIMVS_E_ARG, "null argument");
  if (width < 1 || height < 1) return fail(n, PHIMVS_E_ARG, "width and height must be >= 1");
  NCHECK(n, hipSetDevice(n->device));
  TargetArgs a{};
  a.W = width;
  a.H = height;
  a.w = (width + 3) / 4;
  a.h = (height + 3) / 4;
  a.depth = depth;
  a.normal = normal;
  a.cost = cost;
  a.max_cost = max_cost;
  a.target = target;
  a.mask = mask;
  NCHECK(n, launch_targets(a, n->stream));
  return PHIMVS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------- proposal

namespace {

using phimvs_internal::ViewInfo;

void inv33(const double* A, double* I) {
  const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  I[0] = c00 / det;
  I[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  I[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  I[3] = c01 / det;
  I[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  I[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  I[6] = c02 / det;
  I[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  I[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

void mul33(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// camera centre -R^T t
void centre(const ViewInfo& v, double* c) {
  for (int i = 0; i < 3; ++i) c[i] = -(v.R[i] * v.t[0] + v.R[3 + i] * v.t[1] + v.R[6 + i] * v.t[2]);
}

int err_ctx(phimvs_ctx* c, int code, const std::string& m) { return phimvs_internal::ctx_fail(c, code, m.c_str()); }

int build_inputs(phimvs_ctx* c, phimvs_net* n, int ref, const int* srcs, int n_srcs, float* input) {
  if (!c || !n) return PHIMVS_E_ARG;
  if (!input) return err_ctx(c, PHIMVS_E_ARG, "null input buffer");
  if (n_srcs < 0 || (n_srcs > 0 && !srcs)) return err_ctx(c, PHIMVS_E_ARG, "invalid source list");
  ViewInfo r{};
  int rc = phimvs_internal::view_info(c, ref, &r);
  if (rc) return rc;
  if (n->device != phimvs_internal::ctx_device(c)) return err_ctx(c, PHIMVS_E_ARG, "network and context on different devices");
  // the (up to) four sources closest to the reference camera, ties by list order
  std::vector<std::pair<double, int>> by_dist;
  double c0[3];
  centre(r, c0);
  for (int i = 0; i < n_srcs; ++i) {
    ViewInfo s{};
    if ((rc = phimvs_internal::view_info(c, srcs[i], &s))) return rc;
    if (srcs[i] == ref) return err_ctx(c, PHIMVS_E_ARG, "reference listed among its sources");
    double cs[3];
    centre(s, cs);
    const double d2 = (cs[0] - c0[0]) * (cs[0] - c0[0]) + (cs[1] - c0[1]) * (cs[1] - c0[1]) + (cs[2] - c0[2]) * (cs[2] - c0[2]);
    by_dist.push_back({d2, i});
  }
  std::stable_sort(by_dist.begin(), by_dist.end(),
                   [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first < b.first; });
  ProposalInputs a{};
  a.W = r.W;
  a.H = r.H;
  a.w = (r.W + 3) / 4;
  a.h = (r.H + 3) / 4;
  a.ref = r.plain;
  a.out = input;
  double Kinv[9];
  inv33(r.K, Kinv);
  const double dmid = 0.5 * (r.d_lo + r.d_hi);
  for (int k = 0; k < 4; ++k) {
    a.quad[k] = nullptr;
    a.sw[k] = a.sh[k] = 1;
    for (int e = 0; e < 9; ++e) a.Hmid[9 * k + e] = 0.f;
    if (k >= (int)by_dist.size()) continue;
    ViewInfo s{};
    phimvs_internal::view_info(c, srcs[by_dist[k].second], &s);
    // X_s = R_rel X + t_rel with X on the plane z = dmid: X_s = (R_rel + t_rel (0, 0, 1) / dmid) X
    double Rrel[9], RrT[9], A[9], KA[9], Hm[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) RrT[3 * i + j] = r.R[3 * j + i];
    mul33(s.R, RrT, Rrel);
    double trel[3];
    for (int i = 0; i < 3; ++i) trel[i] = s.t[i] - (Rrel[3 * i] * r.t[0] + Rrel[3 * i + 1] * r.t[1] + Rrel[3 * i + 2] * r.t[2]);
    for (int i = 0; i < 9; ++i) A[i] = Rrel[i];
    for (int i = 0; i < 3; ++i) A[3 * i + 2] += trel[i] / dmid;
    mul33(s.K, A, KA);
    mul33(KA, Kinv, Hm);
    for (int e = 0; e < 9; ++e) a.Hmid[9 * k + e] = (float)Hm[e];
    a.quad[k] = s.quad;
    a.sw[k] = s.W;
    a.sh[k] = s.H;
  }
  hipError_t e = launch_proposal_inputs(a, phimvs_internal::ctx_stream(c));
  if (e != hipSuccess) return err_ctx(c, PHIMVS_E_DEVICE, std::string("proposal inputs: ") + hipGetErrorString(e));
  return PHIMVS_OK;
}

int decode(phimvs_ctx* c, const ViewInfo& r, const float* out, float* planes) {
  ProposalDecode a{};
  a.W = r.W;
  a.H = r.H;
  a.w = (r.W + 3) / 4;
  a.h = (r.H + 3) / 4;
  a.net_out = out;
  double Kinv[9];
  inv33(r.K, Kinv);
  for (int i = 0; i < 9; ++i) a.Kinv[i] = (float)Kinv[i];
  a.d_lo = (float)r.d_lo;
  a.d_hi = (float)r.d_hi;
  a.planes = planes;
  hipError_t e = launch_proposal_decode(a, phimvs_internal::ctx_stream(c));
  if (e != hipSuccess) return err_ctx(c, PHIMVS_E_DEVICE, std::string("proposal decode: ") + hipGetErrorString(e));
  return PHIMVS_OK;
}

}  // namespace

extern "C" {

int phimvs_net_inputs(phimvs_ctx* c, phimvs_net* n, int ref, const int* srcs, int n_srcs, float* input) {
  if (!c || !n) return PHIMVS_E_ARG;
  if (hipSetDevice(n->device) != hipSuccess) return PHIMVS_E_DEVICE;
  return build_inputs(c, n, ref, srcs, n_srcs, input);
}

int phimvs_net_decode(phimvs_ctx* c, phimvs_net* n, int ref, const float* output, float* planes) {
  if (!c || !n) return PHIMVS_E_ARG;
  if (!output || !planes) return err_ctx(c, PHIMVS_E_ARG, "null buffer");
  ViewInfo r{};
  int rc = phimvs_internal::view_info(c, ref, &r);
  if (rc) return rc;
  if (hipSetDevice(n->device) != hipSuccess) return PHIMVS_E_DEVICE;
  return decode(c, r, output, planes);
}

int phimvs_net_propose(phimvs_ctx* c, phimvs_net* n, int ref, const int* srcs, int n_srcs, float* planes) {
  if (!c || !n) return PHIMVS_E_ARG;
  if (!planes) return err_ctx(c, PHIMVS_E_ARG, "null planes buffer");
  ViewInfo r{};
  int rc = phimvs_internal::view_info(c, ref, &r);
  if (rc) return rc;
  if (hipSetDevice(n->device) != hipSuccess) return PHIMVS_E_DEVICE;
  const int w = (r.W + 3) / 4, h = (r.H + 3) / 4;
  if ((rc = ensure(n, n->tmp_in, (size_t)w * h * PHIMVS_NET_IN)) ||
      (rc = ensure(n, n->tmp_out, (size_t)w * h * PHIMVS_NET_OUT)))
    return err_ctx(c, rc, n->err);
  // the network works on the context's stream for this call
  hipStream_t saved = n->stream;
  n->stream = phimvs_internal::ctx_stream(c);
  rc = build_inputs(c, n, ref, srcs, n_srcs, n->tmp_in.p);
  if (!rc) {
    rc = forward(n, 1, h, w, n->tmp_in.p, n->tmp_out.p);
    if (rc) rc = err_ctx(c, rc, n->err);
  }
  if (!rc) rc = decode(c, r, n->tmp_out.p, planes);
  n->stream = saved;
  return rc;
}

}  // extern "C"
