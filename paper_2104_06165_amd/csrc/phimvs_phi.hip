// Data-parallel parts of plane hypothesis inference (PHI-MVS Sec. III-E): depth
// hypotheses by 1-D line fits in four directions, the fronto-parallel planes whose cost
// scores them, the choice of the hypothesis closest to the decoded reference map, and
// the normals of Eq. 10.  One thread per pixel; FP64 wherever a value decides something,
// written in the order stated so that results equal a sequential FP64 evaluation.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>
#include <mutex>

#include "phimvs_internal.h"

namespace pmp {

using namespace phimvs_internal;

// Each direction's pixels with depth are held as a bitmap along that direction's lines, so
// that a fit finds the next pixel with depth on either side with a word scan instead of a
// pixel-by-pixel walk (holes can span hundreds of pixels).  Direction k, its lines and
// the position of a pixel on its line:
//   0 (1, 0):  line y,             position x, W positions
//   1 (0, 1):  line x,             position y, H positions
//   2 (1, 1):  line x - y + H - 1, position y, H positions (W + H - 1 lines)
//   3 (1, -1): line x + y,         position y, H positions (W + H - 1 lines)
// Word w of line l is at bm[w * lines + l] (so neighbouring lines are neighbouring words);
// bit b is position 64 w + b; positions outside the image are 0.
struct PhiBits {
  uint64_t* bm[4];
  int lines[4], words[4];
};

__host__ __device__ inline PhiBits phi_bits_layout(uint64_t* base, int W, int H) {
  PhiBits B;
  const int wx = (W + 63) / 64, wy = (H + 63) / 64;
  B.lines[0] = H;
  B.words[0] = wx;
  B.lines[1] = W;
  B.words[1] = wy;
  B.lines[2] = B.lines[3] = W + H - 1;
  B.words[2] = B.words[3] = wy;
  size_t off = 0;
  for (int k = 0; k < 4; ++k) {
    B.bm[k] = base ? base + off : nullptr;
    off += (size_t)B.lines[k] * B.words[k];
  }
  return B;
}

__device__ __forceinline__ bool has_depth(const float* __restrict__ depth, int W, int x, int y) {
  return depth[(size_t)y * W + x] > 0.0f;  // the same test as (double)d > 0.0
}

// direction 0: one wave per 64 pixels of a row, the word is the wave's ballot
__global__ __launch_bounds__(256) void phi_bits_rows_kernel(const float* __restrict__ depth, int W, int H,
                                                            PhiBits B) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  const bool v = x < W && has_depth(depth, W, x, y);
  const uint64_t word = __ballot(v);
  const int x0 = x & ~63;
  if ((threadIdx.x & 63) == 0 && x0 < W) B.bm[0][(size_t)(x0 >> 6) * B.lines[0] + y] = word;
}

// directions 1-3 (blockIdx.z): one thread per (line, word), 64 rows; neighbouring threads
// take neighbouring lines, which read neighbouring pixels of a row
__global__ __launch_bounds__(256) void phi_bits_cols_kernel(const float* __restrict__ depth, int W, int H,
                                                            PhiBits B) {
  const int k = 1 + blockIdx.z;
  const int line = blockIdx.x * 256 + threadIdx.x, w = blockIdx.y;
  if (line >= B.lines[k]) return;
  uint64_t word = 0;
  for (int b = 0; b < 64; ++b) {
    const int y = w * 64 + b;
    if (y >= H) break;
    const int x = k == 1 ? line : (k == 2 ? line - (H - 1) + y : line - y);
    if (x >= 0 && x < W && has_depth(depth, W, x, y)) word |= 1ull << b;
  }
  B.bm[k][(size_t)w * B.lines[k] + line] = word;
}

// nearest position with depth above q on line l (q may be -1), or -1
__device__ __forceinline__ int bits_up(const uint64_t* __restrict__ bm, int lines, int words, int l, int q) {
  const int p = q + 1;
  int w = p >> 6;
  if (w >= words) return -1;
  uint64_t bits = bm[(size_t)w * lines + l] & (~0ull << (p & 63));
  while (bits == 0) {
    if (++w >= words) return -1;
    bits = bm[(size_t)w * lines + l];
  }
  return w * 64 + __builtin_ctzll(bits);
}

// nearest position with depth below q on line l, or -1
__device__ __forceinline__ int bits_down(const uint64_t* __restrict__ bm, int lines, int l, int q) {
  const int p = q - 1;
  if (p < 0) return -1;
  int w = p >> 6;
  uint64_t bits = bm[(size_t)w * lines + l] & (~0ull >> (63 - (p & 63)));
  while (bits == 0) {
    if (--w < 0) return -1;
    bits = bm[(size_t)w * lines + l];
  }
  return w * 64 + 63 - __builtin_clzll(bits);
}

// Least-squares line through the six pixels with depth closest to (x, y) along direction
// k, value at step 0.  Candidates are taken by increasing step s, the -s side before the
// +s side at equal s, until six are taken or both sides leave the image; the sums take
// them in that order.
__device__ double line_fit(const float* __restrict__ depth, int W, int H, const PhiBits& B, int k, int x, int y) {
  const uint64_t* bm = B.bm[k];
  const int lines = B.lines[k], words = B.words[k];
  const int l = k == 0 ? y : (k == 1 ? x : (k == 2 ? x - y + H - 1 : x + y));
  const int pos = k == 0 ? x : y;
  // along direction 3 a step of +1 lowers the position
  const bool rev = k == 3;
  int a = rev ? bits_up(bm, lines, words, l, pos) : bits_down(bm, lines, l, pos);  // side -1
  int b = rev ? bits_down(bm, lines, l, pos) : bits_up(bm, lines, words, l, pos);  // side +1
  double S0 = 0.0, S1 = 0.0, S2 = 0.0, T0 = 0.0, T1 = 0.0;
  int n = 0;
  while (n < 6 && (a >= 0 || b >= 0)) {
    const int sa = a >= 0 ? abs(a - pos) : INT_MAX, sb = b >= 0 ? abs(b - pos) : INT_MAX;
    int q, step;
    if (sa <= sb) {
      q = a;
      step = -sa;
      a = rev ? bits_up(bm, lines, words, l, a) : bits_down(bm, lines, l, a);
    } else {
      q = b;
      step = sb;
      b = rev ? bits_down(bm, lines, l, b) : bits_up(bm, lines, words, l, b);
    }
    const int xs = k == 0 ? q : (k == 1 ? x : (k == 2 ? x + (q - y) : x - (q - y)));
    const int ys = k == 0 ? y : q;
    const double d = depth[(size_t)ys * W + xs];
    const double si = (double)step;
    S0 = S0 + 1.0;
    S1 = S1 + si;
    S2 = S2 + si * si;
    T0 = T0 + d;
    T1 = T1 + si * d;
    ++n;
  }
  if (n < 2) return 0.0;
  const double det = S0 * S2 - S1 * S1;
  const double a0 = (S2 * T0 - S1 * T1) / det;
  return a0 > 0.0 ? a0 : 0.0;
}

__global__ __launch_bounds__(256) void phi_hyp_kernel(const float* __restrict__ depth, int W, int H, PhiBits B,
                                                      float* __restrict__ hyp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const size_t p = (size_t)y * W + x, plane = (size_t)W * H;
  const bool hole = !(depth[p] > 0.0f);
  for (int k = 0; k < 4; ++k) hyp[k * plane + p] = hole ? (float)line_fit(depth, W, H, B, k, x, y) : 0.0f;
}

// an empty hypothesis (h <= 0) costs C_max
__global__ void phi_mask_cost_kernel(const float* __restrict__ hyp, size_t n, float cmax, float* __restrict__ cost) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!(hyp[i] > 0.0f)) cost[i] = cmax;
}

// the graph model's inputs at half size, node (X, Y) from pixel (2X, 2Y), in one array:
// depth (W2 H2), then the 4 hypothesis planes, then the 4 cost planes
__global__ void phi_half_kernel(const float* __restrict__ depth, const float* __restrict__ hyp,
                                const float* __restrict__ cost, int W, int H, int W2, int H2,
                                float* __restrict__ half) {
  const int X = blockIdx.x * blockDim.x + threadIdx.x, Y = blockIdx.y;
  if (X >= W2 || Y >= H2) return;
  const size_t q = (size_t)Y * W2 + X, n2 = (size_t)W2 * H2;
  const size_t p = (size_t)(2 * Y) * W + 2 * X, plane = (size_t)W * H;
  half[q] = depth[p];
  for (int k = 0; k < 4; ++k) {
    half[(1 + k) * n2 + q] = hyp[k * plane + p];
    half[(5 + k) * n2 + q] = cost[k * plane + p];
  }
}

// each pixel without depth takes the hypothesis closest to the reference map: the decoded
// half-size depth dec, pixel (x, y) reading node (x / 2, y / 2)
__global__ void phi_select_kernel(const float* __restrict__ depth, const float* __restrict__ hyp,
                                  const float* __restrict__ dec, int W, int H, int W2, float* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const size_t p = (size_t)y * W + x, plane = (size_t)W * H;
  const float d = depth[p];
  if (d > 0.0f) {
    out[p] = d;
    return;
  }
  const double r = dec[(size_t)(y >> 1) * W2 + (x >> 1)];
  float best = 0.0f;
  double bd = 0.0;
  if (r > 0.0)
    for (int k = 0; k < 4; ++k) {
      const float h = hyp[k * plane + p];
      if (!(h > 0.0f)) continue;
      const double e = fabs((double)h - r);
      if (best == 0.0f || e < bd) {
        best = h;
        bd = e;
      }
    }
  out[p] = best;
}

__global__ void phi_normals_kernel(const float* __restrict__ depth, int W, int H, PhiCam cam,
                                   float* __restrict__ normal) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const size_t p = (size_t)y * W + x;
  float* n = normal + 3 * p;
  n[0] = n[1] = n[2] = 0.0f;
  if (x < 1 || y < 1 || x + 1 >= W || y + 1 >= H) return;
  if (!(depth[p] > 0.0f && depth[p - W] > 0.0f && depth[p + W] > 0.0f && depth[p - 1] > 0.0f && depth[p + 1] > 0.0f))
    return;
  auto back = [&](int xx, int yy, double* X) {
    const double px = (double)xx, py = (double)yy;
    const double d = depth[(size_t)yy * W + xx];
    for (int k = 0; k < 3; ++k) X[k] = d * (cam.Kinv[3 * k] * px + cam.Kinv[3 * k + 1] * py + cam.Kinv[3 * k + 2] * 1.0);
  };
  double Xu[3], Xd[3], Xl[3], Xr[3], C[3];
  back(x, y - 1, Xu);
  back(x, y + 1, Xd);
  back(x - 1, y, Xl);
  back(x + 1, y, Xr);
  back(x, y, C);
  const double a0 = Xu[0] - Xd[0], a1 = Xu[1] - Xd[1], a2 = Xu[2] - Xd[2];
  const double b0 = Xl[0] - Xr[0], b1 = Xl[1] - Xr[1], b2 = Xl[2] - Xr[2];
  double c0 = a1 * b2 - a2 * b1, c1 = a2 * b0 - a0 * b2, c2 = a0 * b1 - a1 * b0;
  const double len = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  if (!(len > 0.0)) return;
  if (c0 * C[0] + c1 * C[1] + c2 * C[2] > 0.0) {
    c0 = -c0;
    c1 = -c1;
    c2 = -c2;
  }
  n[0] = (float)(c0 / len);
  n[1] = (float)(c1 / len);
  n[2] = (float)(c2 / len);
}

}  // namespace pmp

// Scratch of the allocation-free hypothesis entry point: one call's occupancy bitmaps, at
// most kPhiScratchWords 64-bit words (8 MiB), one copy on every GPU the library runs on,
// held until the process ends.  Host code never passes `scratch` itself to a kernel (its
// host-side name is not a device address): it passes the device address that
// phi_scratch_setup looked up on each device.  Every call on one GPU shares that GPU's
// copy; every word of the layout is rewritten by each call, so nothing needs clearing.
static __device__ __align__(256) uint64_t scratch[phimvs_internal::kPhiScratchWords];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
bool g_scratch_done[kMaxScratchDevices] = {};
hipError_t g_scratch_err[kMaxScratchDevices] = {};
uint64_t* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

namespace phimvs_internal {

hipError_t phi_scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_done[device]) {
    // the caller has made `device` current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? static_cast<uint64_t*>(p) : nullptr;
    g_scratch_done[device] = true;
  }
  return g_scratch_err[device];
}

hipError_t phi_scratch_get(int device, uint64_t** p) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_done[device]) return hipErrorNotInitialized;
  if (g_scratch_err[device] != hipSuccess) return g_scratch_err[device];
  *p = g_scratch_ptr[device];
  return hipSuccess;
}

size_t phi_bits_words(int W, int H) {
  const pmp::PhiBits B = pmp::phi_bits_layout(nullptr, W, H);
  size_t n = 0;
  for (int k = 0; k < 4; ++k) n += (size_t)B.lines[k] * B.words[k];
  return n;
}

hipError_t launch_phi_hypotheses(const float* depth, int W, int H, uint64_t* bits, float* hyp, hipStream_t st) {
  const pmp::PhiBits B = pmp::phi_bits_layout(bits, W, H);
  hipLaunchKernelGGL(pmp::phi_bits_rows_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, W, H, B);
  hipLaunchKernelGGL(pmp::phi_bits_cols_kernel, dim3((W + H - 1 + 255) / 256, B.words[1], 3), dim3(256), 0, st,
                     depth, W, H, B);
  hipLaunchKernelGGL(pmp::phi_hyp_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, W, H, B, hyp);
  return hipGetLastError();
}

hipError_t launch_phi_mask_cost(const float* hyp, size_t n, float cmax, float* cost, hipStream_t st) {
  hipLaunchKernelGGL(pmp::phi_mask_cost_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, hyp, n, cmax,
                     cost);
  return hipGetLastError();
}

hipError_t launch_phi_half(const float* depth, const float* hyp, const float* cost, int W, int H, float* half,
                           hipStream_t st) {
  const int W2 = (W + 1) / 2, H2 = (H + 1) / 2;
  hipLaunchKernelGGL(pmp::phi_half_kernel, dim3((W2 + 255) / 256, H2), dim3(256), 0, st, depth, hyp, cost, W, H, W2,
                     H2, half);
  return hipGetLastError();
}

hipError_t launch_phi_select(const float* depth, const float* hyp, const float* dec, int W, int H, float* out,
                             hipStream_t st) {
  const int W2 = (W + 1) / 2;
  hipLaunchKernelGGL(pmp::phi_select_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, hyp, dec, W, H, W2,
                     out);
  return hipGetLastError();
}

hipError_t launch_phi_normals(const float* depth, int W, int H, const PhiCam& cam, float* normal, hipStream_t st) {
  hipLaunchKernelGGL(pmp::phi_normals_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, W, H, cam, normal);
  return hipGetLastError();
}

}  // namespace phimvs_internal
