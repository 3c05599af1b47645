// Learned initial-plane proposal: a 5-layer 3x3 convolutional network (5 -> 32 -> 32 ->
// 32 -> 32 -> 4 channels, ReLU between layers) over a 1/4-resolution input (the
// reference and four source views warped by the fronto-parallel plane at the middle of
// the depth range).  Its output seeds the random initialisation of Sec. III-B: each
// pixel keeps the proposed plane only when its matching cost is not higher than the
// random plane's (the gate lives in the initialisation kernel).
//
// Numerics: weights and activations are bfloat16, every convolution accumulates in FP32
// on the matrix cores (v_mfma_f32_16x16x16bf16_1k).  Activations are NHWC with the
// channel count padded to a multiple of 16.  A convolution is an implicit GEMM over
// K = 9 taps x input channels: one wave computes 16 pixels of one image row x 16
// output channels per matrix instruction; a workgroup of 16 waves stages the layer's
// weights in LDS once, so only the input patches go through the texture path.  Training runs on the same kernels: the data
// gradient is the forward convolution with flipped, transposed weights; the weight
// gradient accumulates (input patch)^T x (output gradient) over 16-pixel slices per
// image row, written as per-row partial sums and reduced in a fixed order (16
// interleaved groups of rows, then the groups in turn).

#include <hip/hip_runtime.h>
#include <hip/hip_bfloat16.h>
#include <stdint.h>

#include "phimvs_net_internal.h"

namespace pmn {

using namespace phimvs_net_internal;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even (NaN not expected)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------- convolution
// y[b, r, c, co] = bias[co] + sum_{t, ci} x[b, r + dy_t, c + dx_t, ci] * w[t][co][ci]
// (zero outside the image), optionally ReLU; x: bf16 NHWC with CI channels (multiple of 16);
// w: bf16 [9][CO][CI]; CO multiple of 16.  Output: bf16 (y16, CO channels) and / or fp32
// (y32, first co_keep channels).  If mask16 is given the result is multiplied by
// (mask16 > 0) (ReLU backward of the producing layer) before storing.
constexpr int kConvBlock = 1024;  // 16 waves, each 16 pixels of a row
constexpr int kMaxCI = 32;        // widest layer input (channels, padded)
constexpr int kConvPad = 4;       // bf16 padding of each LDS weight row (spreads the banks)
__global__ __launch_bounds__(kConvBlock) void conv3x3_kernel(ConvArgs a) {
  // the weights [9][CO][CI], staged once per workgroup; each (tap, output channel) row padded
  __shared__ uint2 wl[9 * kMaxCO * (kMaxCI + kConvPad) / 4];
  const int q = a.CI / 4, qp = (a.CI + kConvPad) / 4;
  {
    const uint2* __restrict__ wg = reinterpret_cast<const uint2*>(a.wt);
    for (int i = threadIdx.x; i < 9 * a.CO * q; i += kConvBlock) {
      const int row = i / q, k = i - row * q;
      wl[row * qp + k] = wg[i];
    }
  }
  __syncthreads();
  const uint16_t* ws = reinterpret_cast<const uint16_t*>(wl);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int segs = (a.w + 15) / 16;
  const int task = blockIdx.x * (kConvBlock / 64) + wave;  // (b, r, seg)
  if (task >= a.B * a.h * segs) return;
  const int seg = task % segs;
  const int br = task / segs;
  const int r = br % a.h, b = br / a.h;
  const int c0 = seg * 16;
  const int lr = lane & 15, lk = lane >> 4;  // row / column of the fragment, K group
  v4f acc[kMaxCO / 16];
#pragma unroll
  for (int i = 0; i < kMaxCO / 16; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  const int nco = a.CO / 16;
  for (int t = 0; t < 9; ++t) {
    const int rr = r + t / 3 - 1;
    const int cc = c0 + lr + t % 3 - 1;
    const bool inside = rr >= 0 && rr < a.h && cc >= 0 && cc < a.w;
    const size_t pix = ((size_t)b * a.h + (inside ? rr : 0)) * a.w + (inside ? cc : 0);
    for (int cib = 0; cib < a.CI / 16; ++cib) {
      const int ci = cib * 16 + lk * 4;
      v4s A = v4s{0, 0, 0, 0};
      if (inside) A = *reinterpret_cast<const v4s*>(a.x + pix * a.CI + ci);
#pragma unroll
      for (int i = 0; i < kMaxCO / 16; ++i) {
        if (i < nco) {
          const int co = i * 16 + lr;
          const v4s Bf = *reinterpret_cast<const v4s*>(ws + (t * a.CO + co) * (qp * 4) + ci);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bf, acc[i], 0, 0, 0);
        }
      }
    }
  }
  // acc[i][j]: pixel c0 + 4 lk + j, output channel 16 i + lr
#pragma unroll
  for (int i = 0; i < kMaxCO / 16; ++i) {
    if (i >= nco) continue;
    const int co = i * 16 + lr;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + lk * 4 + j;
      if (c >= a.w) continue;
      float v = acc[i][j] + ((a.bias && co < a.n_bias) ? a.bias[co] : 0.f);
      if (a.relu) v = fmaxf(v, 0.f);
      const size_t p = ((size_t)b * a.h + r) * a.w + c;
      if (a.mask16 && !(bf2f(a.mask16[p * a.CO + co]) > 0.f)) v = 0.f;
      if (a.y16) a.y16[p * a.CO + co] = f2bf(v);
      if (a.y32 && co < a.co_keep) a.y32[p * a.co_keep + co] = v;
    }
  }
}

// Weight gradient partials: for image row (b, r): P[b r][t][ci][co] = sum_c x[b, r+dy, c+dx, ci] *
// g[b, r, c, co]; bias partial Pb[b r][co] = sum_c g[b, r, c, co].  One workgroup per image row;
// wave k of 4 handles the taps t = k, k + 4, k + 8 for every (ci, co) block.  The row is
// walked in chunks of 64 pixels staged in LDS by coalesced loads (the three input rows
// and the output-gradient row); every accumulator takes its 16-pixel slices in row order.
constexpr int kWgChunk = 64;   // pixels staged per step (4 slices of 16)
constexpr int kWgStride = 36;  // bf16 per staged pixel: 32 channels + 4 of padding (spreads the banks)
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(WgradArgs a) {
  // rows r - 1 .. r + 1 of the input (pixels c_base - 1 .. c_base + 64) and row r of the
  // output gradient (pixels c_base .. c_base + 63), zero outside the image
  __shared__ uint2 xs2[3 * (kWgChunk + 2) * kWgStride / 4];
  __shared__ uint2 gs2[kWgChunk * kWgStride / 4];
  const int br = blockIdx.x;
  if (br >= a.B * a.h) return;
  const int r = br % a.h, b = br / a.h;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int nci = a.CI / 16, nco = a.CO / 16;
  const int qi = a.CI / 4, qo = a.CO / 4;
  const uint16_t* xs = reinterpret_cast<const uint16_t*>(xs2);
  const uint16_t* gs = reinterpret_cast<const uint16_t*>(gs2);
  const uint2* __restrict__ xg = reinterpret_cast<const uint2*>(a.x);
  const uint2* __restrict__ gg = reinterpret_cast<const uint2*>(a.g);
  v4f acc[3][kMaxCO / 16][kMaxCO / 16];  // taps wave, wave + 4, wave + 8 x input block x output block
#pragma unroll
  for (int ti = 0; ti < 3; ++ti)
#pragma unroll
    for (int u = 0; u < kMaxCO / 16; ++u)
#pragma unroll
      for (int v = 0; v < kMaxCO / 16; ++v) acc[ti][u][v] = v4f{0.f, 0.f, 0.f, 0.f};
  float bias = 0.f;
  for (int c_base = 0; c_base < a.w; c_base += kWgChunk) {
    __syncthreads();  // the previous chunk's reads are done
    for (int i = threadIdx.x; i < 3 * (kWgChunk + 2) * qi; i += 256) {
      const int row = i / ((kWgChunk + 2) * qi);
      const int rem = i - row * (kWgChunk + 2) * qi;
      const int px = rem / qi, k = rem - px * qi;
      const int rr = r + row - 1, cx = c_base + px - 1;
      uint2 v = make_uint2(0u, 0u);
      if (rr >= 0 && rr < a.h && cx >= 0 && cx < a.w) v = xg[(((size_t)b * a.h + rr) * a.w + cx) * qi + k];
      xs2[(row * (kWgChunk + 2) + px) * (kWgStride / 4) + k] = v;
    }
    for (int i = threadIdx.x; i < kWgChunk * qo; i += 256) {
      const int px = i / qo, k = i - px * qo;
      const int c = c_base + px;
      uint2 v = make_uint2(0u, 0u);
      if (c < a.w) v = gg[(((size_t)b * a.h + r) * a.w + c) * qo + k];
      gs2[px * (kWgStride / 4) + k] = v;
    }
    __syncthreads();
    for (int sl = 0; sl < kWgChunk / 16; ++sl) {
      const int lp = sl * 16;  // first pixel of the slice, relative to c_base
      if (c_base + lp >= a.w) break;
#pragma unroll
      for (int ti = 0; ti < 3; ++ti) {
        const int t = wave + 4 * ti;
        if (t >= 9) break;
        const int ty = t / 3, dx = t % 3 - 1;
#pragma unroll
        for (int cib = 0; cib < kMaxCO / 16; ++cib) {
          if (cib >= nci) break;
          // A (16 ci x 16 px): lane -> ci = 16 cib + lr, pixels c + 4 lk .. + 3 (zero past the row end)
          v4s A;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int p = lp + lk * 4 + j;
            A[j] = (c_base + p < a.w) ? (short)xs[(ty * (kWgChunk + 2) + p + dx + 1) * kWgStride + cib * 16 + lr] : 0;
          }
#pragma unroll
          for (int cob = 0; cob < kMaxCO / 16; ++cob) {
            if (cob >= nco) break;
            // B (16 px x 16 co): lane -> co = 16 cob + lr, pixels c + 4 lk .. + 3
            v4s Bf;
#pragma unroll
            for (int j = 0; j < 4; ++j) Bf[j] = (short)gs[(lp + lk * 4 + j) * kWgStride + cob * 16 + lr];
            acc[ti][cib][cob] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bf, acc[ti][cib][cob], 0, 0, 0);
          }
        }
      }
    }
    // bias partial: first wave, one lane per output channel, in pixel order
    if (a.partial_bias && wave == 0 && lane < a.CO) {
      const int n = min(kWgChunk, a.w - c_base);
      for (int p = 0; p < n; ++p) bias = bias + bf2f(gs[p * kWgStride + lane]);
    }
  }
  float* P = a.partial + (size_t)br * 9 * a.CI * a.CO;
#pragma unroll
  for (int ti = 0; ti < 3; ++ti) {
    const int t = wave + 4 * ti;
    if (t >= 9) break;
#pragma unroll
    for (int cib = 0; cib < kMaxCO / 16; ++cib) {
      if (cib >= nci) break;
#pragma unroll
      for (int cob = 0; cob < kMaxCO / 16; ++cob) {
        if (cob >= nco) break;
        // acc[j]: ci = 16 cib + 4 lk + j, co = 16 cob + lr
#pragma unroll
        for (int j = 0; j < 4; ++j)
          P[((size_t)t * a.CI + cib * 16 + lk * 4 + j) * a.CO + cob * 16 + lr] = acc[ti][cib][cob][j];
      }
    }
  }
  if (a.partial_bias && wave == 0 && lane < a.CO) a.partial_bias[(size_t)br * a.CO + lane] = bias;
}

// out[i] = sum_{k < n_rows} partial[k * stride + i] in a fixed order: a workgroup of 16
// waves takes 64 outputs, wave g sums rows g, g + 16, g + 32, ... in turn, and the 16
// sums are added in wave order, so the result does not depend on scheduling
constexpr int kReduceGroups = 16;
__global__ __launch_bounds__(kReduceGroups * 64) void reduce_rows_kernel(const float* __restrict__ partial,
                                                                         int n_rows, int stride, int n,
                                                                         float* __restrict__ out) {
  __shared__ float part[kReduceGroups][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (i < n) {
#pragma unroll 4
    for (int k = g; k < n_rows; k += kReduceGroups) s += partial[(size_t)k * stride + i];
  }
  part[g][lane] = s;
  __syncthreads();
  if (g == 0 && i < n) {
    float t = 0.f;
    for (int q = 0; q < kReduceGroups; ++q) t += part[q][lane];
    out[i] = t;
  }
}

// fp32 NHWC (C0 channels) -> bf16 NHWC (CP channels, zero padded)
__global__ void to_bf16_kernel(const float* __restrict__ x, int n_pix, int C0, int CP, uint16_t* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n_pix * CP) return;
  const size_t p = i / CP;
  const int c = (int)(i - p * CP);
  y[i] = c < C0 ? f2bf(x[p * C0 + c]) : (uint16_t)0;
}

// master fp32 weights [9][CIN][COUT] -> bf16 forward [9][COP][CIP] and flipped [9][CIP][COP]
__global__ void bf16_unpad_kernel(const uint16_t* __restrict__ x, int n_pix, int CP, int C, float* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n_pix * C) return;
  const size_t p = i / C, c = i - p * C;
  y[i] = bf2f(x[p * CP + c]);
}

__global__ void pack_weights_kernel(const float* __restrict__ w, int CIN, int COUT, int CIP, int COP,
                                    uint16_t* __restrict__ fwd, uint16_t* __restrict__ flip) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * CIP * COP) return;
  const int t = i / (CIP * COP);
  const int rem = i - t * CIP * COP;
  const int co = rem / CIP, ci = rem - co * CIP;
  const float v = (ci < CIN && co < COUT) ? w[((size_t)t * CIN + ci) * COUT + co] : 0.f;
  fwd[((size_t)t * COP + co) * CIP + ci] = f2bf(v);
  // data gradient: g_in[ci] = sum_{t, co} g[p - off_t][co] w[t][ci][co] = conv with w'[8 - t][ci][co]
  flip[((size_t)(8 - t) * CIP + ci) * COP + co] = f2bf(v);
}

// padded weight gradient [9][CIP][COP] (+ bias [COP]) -> flat [9][CIN][COUT] then [COUT]
__global__ void unpad_grad_kernel(const float* __restrict__ gp, const float* __restrict__ gb, int CIN, int COUT, int CIP,
                                  int COP, float* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = 9 * CIN * COUT;
  if (i < nw) {
    const int t = i / (CIN * COUT);
    const int rem = i - t * CIN * COUT;
    const int ci = rem / COUT, co = rem - ci * COUT;
    g[i] = gp[((size_t)t * CIP + ci) * COP + co];
  } else if (i < nw + COUT) {
    g[i] = gb[i - nw];
  }
}

// ---------------------------------------------------------------------------- loss
// out: B*h*w*4 fp32 (o0: depth logit, o1..o3: normal); target: B*h*w*4 (depth, normal);
// mask: B*h*w; drange: B*2.  Per pixel: depth = lo + (hi - lo) sigmoid(o0), n = o / |o|;
// loss = m (|log depth - log depth_t| + lambda (1 - n . n_t)) / sum(mask).
// Writes the output gradient (bf16, 16 channels) and per-block loss partials.
__global__ void loss_kernel(LossArgs a) {
  __shared__ float red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < a.n_pix) {
    const int b = i / (a.h * a.w);
    const float lo = a.drange[2 * b], hi = a.drange[2 * b + 1];
    const float* o = a.out + (size_t)i * 4;
    const float* tg = a.target + (size_t)i * 4;
    const float m = a.mask[i] * a.inv_count;
    float g[4] = {0.f, 0.f, 0.f, 0.f};
    if (m > 0.f) {
      const float s = 1.f / (1.f + expf(-o[0]));
      const float d = lo + (hi - lo) * s;
      const float diff = logf(d) - logf(tg[0]);
      const float nrm = sqrtf(o[1] * o[1] + o[2] * o[2] + o[3] * o[3]) + 1e-6f;
      const float nx = o[1] / nrm, ny = o[2] / nrm, nz = o[3] / nrm;
      const float dotp = nx * tg[1] + ny * tg[2] + nz * tg[3];
      l = m * (fabsf(diff) + a.lambda * (1.f - dotp));
      const float sg = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
      g[0] = m * sg * (hi - lo) * s * (1.f - s) / d;
      const float k = -m * a.lambda / nrm;
      g[1] = k * (tg[1] - dotp * nx);
      g[2] = k * (tg[2] - dotp * ny);
      g[3] = k * (tg[3] - dotp * nz);
    }
    for (int c = 0; c < 16; ++c) a.grad16[(size_t)i * 16 + c] = c < 4 ? f2bf(g[c]) : (uint16_t)0;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.loss_partial[blockIdx.x] = red[0];
}

// Adam on the fp32 master weights
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                            int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------- proposal
// 1/4-resolution network input for reference pixel block (X, Y): channel 0 = mean of the
// 4x4 reference block, channels 1..4 = source k sampled (bilinear) at the image of the block
// centre under H_k (fronto-parallel plane at the middle of the depth range); 0 outside the
// source.  Values are (I - 127.5) / 64.
__global__ void proposal_inputs_kernel(ProposalInputs a) {
  const int X = blockIdx.x * blockDim.x + threadIdx.x, Y = blockIdx.y;
  if (X >= a.w || Y >= a.h) return;
  float s = 0.f;
  for (int dy = 0; dy < 4; ++dy)
    for (int dx = 0; dx < 4; ++dx) {
      const int x = min(4 * X + dx, a.W - 1), y = min(4 * Y + dy, a.H - 1);
      s += __half2float(a.ref[(size_t)y * a.W + x]);
    }
  float* o = a.out + ((size_t)Y * a.w + X) * 5;
  o[0] = (s / 16.f - 127.5f) / 64.f;
  const float px = 4.f * X + 1.5f, py = 4.f * Y + 1.5f;
  for (int k = 0; k < 4; ++k) {
    const float* Hm = a.Hmid + 9 * k;
    const float u = Hm[0] * px + Hm[1] * py + Hm[2];
    const float v = Hm[3] * px + Hm[4] * py + Hm[5];
    const float w = Hm[6] * px + Hm[7] * py + Hm[8];
    float val = 0.f;
    if (a.quad[k] && w > 0.f) {
      const float up = u / w, vp = v / w;
      if (up >= 0.f && vp >= 0.f && up <= (float)(a.sw[k] - 1) && vp <= (float)(a.sh[k] - 1)) {
        const int x0 = (int)up, y0 = (int)vp;
        const float fx = up - x0, fy = vp - y0;
        const uint32_t q = a.quad[k][(size_t)y0 * a.sw[k] + x0];
        const float t00 = (float)(q & 0xFF), t01 = (float)((q >> 8) & 0xFF);
        const float t10 = (float)((q >> 16) & 0xFF), t11 = (float)(q >> 24);
        const float top = t00 + fx * (t01 - t00), bot = t10 + fx * (t11 - t10);
        val = ((top + fy * (bot - top)) - 127.5f) / 64.f;
      }
    }
    o[1 + k] = val;
  }
}

// full-resolution planes from the 1/4-resolution network output: bilinear upsampling of the
// four raw outputs, depth = lo + (hi - lo) sigmoid(o0), normal = o / |o| turned to face the camera
__global__ void proposal_decode_kernel(ProposalDecode a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.W || y >= a.H) return;
  const float X = fminf(fmaxf(((float)x - 1.5f) * 0.25f, 0.f), (float)(a.w - 1));
  const float Y = fminf(fmaxf(((float)y - 1.5f) * 0.25f, 0.f), (float)(a.h - 1));
  const int x0 = (int)X, y0 = (int)Y;
  const int x1 = min(x0 + 1, a.w - 1), y1 = min(y0 + 1, a.h - 1);
  const float fx = X - x0, fy = Y - y0;
  float o[4];
  for (int c = 0; c < 4; ++c) {
    const float v00 = a.net_out[((size_t)y0 * a.w + x0) * 4 + c], v01 = a.net_out[((size_t)y0 * a.w + x1) * 4 + c];
    const float v10 = a.net_out[((size_t)y1 * a.w + x0) * 4 + c], v11 = a.net_out[((size_t)y1 * a.w + x1) * 4 + c];
    const float top = v00 + fx * (v01 - v00), bot = v10 + fx * (v11 - v10);
    o[c] = top + fy * (bot - top);
  }
  const float d = a.d_lo + (a.d_hi - a.d_lo) / (1.f + expf(-o[0]));
  float nx = o[1], ny = o[2], nz = o[3];
  const float nrm = sqrtf(nx * nx + ny * ny + nz * nz);
  if (nrm > 1e-6f) {
    nx /= nrm;
    ny /= nrm;
    nz /= nrm;
  } else {
    nx = 0.f;
    ny = 0.f;
    nz = -1.f;
  }
  const float rx = a.Kinv[0] * x + a.Kinv[1] * y + a.Kinv[2];
  const float ry = a.Kinv[3] * x + a.Kinv[4] * y + a.Kinv[5];
  const float rz = a.Kinv[6] * x + a.Kinv[7] * y + a.Kinv[8];
  if (nx * rx + ny * ry + nz * rz > 0.f) {
    nx = -nx;
    ny = -ny;
    nz = -nz;
  }
  float* p = a.planes + ((size_t)y * a.W + x) * 4;
  p[0] = nx;
  p[1] = ny;
  p[2] = nz;
  p[3] = d;
}

// training targets at network resolution from a full-resolution plain PatchMatch result:
// block (X, Y) looks at the 2x2 full-resolution pixels around its centre (4X + 1.5, 4Y + 1.5);
// it is kept (mask 1) when all four are valid with cost below max_cost, with the mean depth
// and the normalised mean normal as target
__global__ void targets_kernel(TargetArgs a) {
  const int X = blockIdx.x * blockDim.x + threadIdx.x, Y = blockIdx.y;
  if (X >= a.w || Y >= a.h) return;
  float d = 0.f, nx = 0.f, ny = 0.f, nz = 0.f;
  bool ok = true;
  for (int dy = 1; dy <= 2; ++dy)
    for (int dx = 1; dx <= 2; ++dx) {
      const int x = min(4 * X + dx, a.W - 1), y = min(4 * Y + dy, a.H - 1);
      const size_t p = (size_t)y * a.W + x;
      const float c = a.cost[p], dd = a.depth[p];
      ok = ok && dd > 0.f && c < a.max_cost;
      d += dd;
      nx += a.normal[3 * p];
      ny += a.normal[3 * p + 1];
      nz += a.normal[3 * p + 2];
    }
  const float nrm = sqrtf(nx * nx + ny * ny + nz * nz);
  ok = ok && nrm > 1e-6f;
  float* t = a.target + ((size_t)Y * a.w + X) * 4;
  t[0] = ok ? 0.25f * d : 1.f;
  t[1] = ok ? nx / nrm : 0.f;
  t[2] = ok ? ny / nrm : 0.f;
  t[3] = ok ? nz / nrm : -1.f;
  a.mask[(size_t)Y * a.w + X] = ok ? 1.f : 0.f;
}

}  // namespace pmn

namespace phimvs_net_internal {

hipError_t launch_conv(const ConvArgs& a, hipStream_t st) {
  const int segs = (a.w + 15) / 16;
  const int tasks = a.B * a.h * segs;
  if (a.CI % 16 || a.CO % 16 || a.CI < 16 || a.CO < 16 || a.CI > pmn::kMaxCI || a.CO > kMaxCO)
    return hipErrorInvalidValue;
  constexpr int wpb = pmn::kConvBlock / 64;
  hipLaunchKernelGGL(pmn::conv3x3_kernel, dim3((tasks + wpb - 1) / wpb), dim3(pmn::kConvBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& a, hipStream_t st) {
  if (a.CI % 16 || a.CO % 16 || a.CI < 16 || a.CO < 16 || a.CI > kMaxCO || a.CO > kMaxCO) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pmn::conv3x3_wgrad_kernel, dim3(a.B * a.h), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_bf16_unpad(const uint16_t* x, int n_pix, int CP, int C, float* y, hipStream_t st) {
  const size_t n = (size_t)n_pix * C;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(pmn::bf16_unpad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n_pix, CP, C, y);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const float* partial, int n_rows, int stride, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(pmn::reduce_rows_kernel, dim3((n + 63) / 64), dim3(pmn::kReduceGroups * 64), 0, st, partial,
                     n_rows, stride, n, out);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, int n_pix, int C0, int CP, uint16_t* y, hipStream_t st) {
  const size_t n = (size_t)n_pix * CP;
  hipLaunchKernelGGL(pmn::to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n_pix, C0, CP, y);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float* w, int CIN, int COUT, int CIP, int COP, uint16_t* fwd, uint16_t* flip,
                               hipStream_t st) {
  const int n = 9 * CIP * COP;
  hipLaunchKernelGGL(pmn::pack_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, CIN, COUT, CIP, COP, fwd, flip);
  return hipGetLastError();
}

hipError_t launch_unpad_grad(const float* gp, const float* gb, int CIN, int COUT, int CIP, int COP, float* g,
                             hipStream_t st) {
  const int n = 9 * CIN * COUT + COUT;
  hipLaunchKernelGGL(pmn::unpad_grad_kernel, dim3((n + 255) / 256), dim3(256), 0, st, gp, gb, CIN, COUT, CIP, COP, g);
  return hipGetLastError();
}

hipError_t launch_loss(const LossArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(pmn::loss_kernel, dim3((a.n_pix + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(pmn::adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_proposal_inputs(const ProposalInputs& a, hipStream_t st) {
  hipLaunchKernelGGL(pmn::proposal_inputs_kernel, dim3((a.w + 127) / 128, a.h), dim3(128), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_proposal_decode(const ProposalDecode& a, hipStream_t st) {
  hipLaunchKernelGGL(pmn::proposal_decode_kernel, dim3((a.W + 255) / 256, a.H), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_targets(const TargetArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(pmn::targets_kernel, dim3((a.w + 127) / 128, a.h), dim3(128), 0, st, a);
  return hipGetLastError();
}

}  // namespace phimvs_net_internal
