// gfx950 kernels of the PatchMatch depth-map estimation step (PHI-MVS Sec. III-B,
// Sec. III-C, Eq. 4, Eq. 5, Algorithm 1 "depth map estimation").
//
// Work decomposition.  The per-pixel state lives in two checkerboard-compacted
// colour planes (red: (x + y) even, black: odd), each H x Wc with Wc = ceil(W / 2):
// pixel (x, y) of colour c sits at column x >> 1 of its colour plane.  A workgroup is
// 4 waves; wave w handles 64 consecutive compacted pixels of row (4 by + w), i.e. 128
// full-resolution columns.  One lane owns one pixel and evaluates its hypotheses one
// after the other; for each hypothesis it walks the window taps in row-major order
// and, per tap, every source view of the current view group, so the reference-side
// tap values (LDS) are read once per group and each view's sums are accumulated in
// plain tap order (the oracle's order: no cross-lane reduction is needed).
//
// Arithmetic.  Every float operation below is the one the method's canonical FP32
// statement performs, in the same order (explicit fmaf, correctly rounded division and
// square root, no contraction), so the results equal a sequential FP32 evaluation.
// The per-tap perspective division uses 1/w computed as one Newton step from
// v_rcp_f32, which is the correctly rounded reciprocal for w in [2^-100, 2^100]
// (checked exhaustively over every float in that range on the device); a sound
// per-(pixel, hypothesis, view) bound derived from the window corners selects the
// IEEE division instead whenever a tap's w could leave that range.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "phimvs_internal.h"

namespace pmk {

using namespace phimvs_internal;

constexpr float kCmax = 2.0f;
constexpr double kPiD = 3.14159265358979323846;

// ---------------------------------------------------------------------------- random numbers
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
// two 32x32->64 multiplies with key bumps by the golden-ratio Weyl constants.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ float u24(uint32_t v) { return (float)(v >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------- arithmetic helpers
__device__ __forceinline__ float dot3f(float ax, float ay, float az, float bx, float by, float bz) {
  return __builtin_fmaf(ax, bx, __builtin_fmaf(ay, by, az * bz));
}

// correctly rounded 1/w for w in [2^-100, 2^100] (one Newton step from the hardware estimate)
__device__ __forceinline__ float rcp_nr(float w) {
  const float r0 = __builtin_amdgcn_rcpf(w);
  const float e = __builtin_fmaf(-w, r0, 1.0f);
  return __builtin_fmaf(e, r0, r0);
}

// bilinear sample from a texel-quad image at a position already clamped into the image:
// the 32-bit quad at (x0, y0) holds the bytes I[y0][x0], I[y0][x1], I[y1][x0], I[y1][x1]
// (x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1)); lerp(a, b, t) = fma(t, b - a, a) with
// exact integer differences.  Four bytes per record (half of an fp16 quad) halve the L1
// lines each lane's window walks through, which is what bounds the gathers.
__device__ __forceinline__ float sample_quad(const uint32_t* __restrict__ quad, int W, float up, float vp) {
  // up, vp >= 0: fract(u) = u - floor(u) exactly
  const float fx = __builtin_amdgcn_fractf(up);
  const float fy = __builtin_amdgcn_fractf(vp);
  const uint32_t x0 = (uint32_t)up, y0 = (uint32_t)vp;
  const uint32_t q = quad[__umul24(y0, (uint32_t)W) + x0];
  const float t00 = (float)(q & 0xFFu), t01 = (float)((q >> 8) & 0xFFu);
  const float t10 = (float)((q >> 16) & 0xFFu), t11 = (float)(q >> 24);
  const float top = __builtin_fmaf(fx, t01 - t00, t00);
  const float bot = __builtin_fmaf(fx, t11 - t10, t10);
  return __builtin_fmaf(fy, bot - top, top);
}

// clamp into [0, hi]; equals fmin(fmax(v, 0), hi) for every non-NaN v (a NaN position only
// arises in a view already ruled invalid, and any result keeps the sample address in range)
__device__ __forceinline__ float clampf(float v, float hi) { return __builtin_amdgcn_fmed3f(v, 0.0f, hi); }

// ---------------------------------------------------------------------------- per-pixel reference data
struct RefPix {
  int x, y;
  float X0, Y0;
  float rx, ry, rz;       // K^-1 (x, y, 1)
  float a_c, S_w, mu_a, var_a;
  bool ok;                // pixel valid and reference patch variance >= eps_v
  int tbase;              // LDS index of the window's first tap
};

// ---------------------------------------------------------------------------- plane cost
// Per-hypothesis values shared by every view: the pixel and m = K^-T n / rho.
struct Hyp {
  float m[3];
  bool ok;  // the reference patch is usable and the plane faces the camera
};

// Sums of one view group over the window taps in row-major order.  Hm holds the G
// homographies of views J0 .. J0+G-1.  EXACT selects IEEE division for 1/w.
template <int G, int J0, bool EXACT>
__device__ __forceinline__ void tap_pass(const Args& A, const RefPix& rp, const float* __restrict__ tile,
                                         const float* __restrict__ wcol, const float* __restrict__ wsp,
                                         const float (&Hm)[G][9], const float (&bc)[G], float (&Sb)[G],
                                         float (&Sbb)[G], float (&Sab)[G]) {
  const int R = A.R, s = A.s, TW = A.TW;
  const float sf = (float)s;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    Sb[g] = 0.0f;
    Sbb[g] = 0.0f;
    Sab[g] = 0.0f;
  }
  int t = 0;
  for (int k2 = -R; k2 <= R; ++k2) {
    const float Y = (float)(rp.y + s * k2);
    float rbu[G], rbv[G], rbw[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      rbu[g] = __builtin_fmaf(Hm[g][1], Y, Hm[g][2]);
      rbv[g] = __builtin_fmaf(Hm[g][4], Y, Hm[g][5]);
      rbw[g] = __builtin_fmaf(Hm[g][7], Y, Hm[g][8]);
    }
    const float* trow = tile + rp.tbase + (k2 + R) * s * TW;
    float X = (float)(rp.x - s * R);
    for (int k1 = 0; k1 <= 2 * R; ++k1, ++t) {
      const float a = trow[k1 * s] - rp.a_c;
      float w = 1.0f;
      if (A.bilateral) w = wcol[(int)fabsf(a)] * wsp[t];
      const float wa = w * a;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const SrcDev& V = A.src[J0 + g];
        const float u = __builtin_fmaf(Hm[g][0], X, rbu[g]);
        const float v = __builtin_fmaf(Hm[g][3], X, rbv[g]);
        const float ww = __builtin_fmaf(Hm[g][6], X, rbw[g]);
        const float r = EXACT ? 1.0f / ww : rcp_nr(ww);
        const float up = clampf(u * r, V.Wm1);
        const float vp = clampf(v * r, V.Hm1);
        const float b = sample_quad(V.quad, V.W, up, vp) - bc[g];
        const float tb = w * b;
        Sb[g] = Sb[g] + tb;
        Sbb[g] = __builtin_fmaf(tb, b, Sbb[g]);
        Sab[g] = __builtin_fmaf(wa, b, Sab[g]);
      }
      X = X + sf;
    }
  }
}

// Views [J0, NV) in groups of G: per group, build the homographies H_j = M_j + e_j m^T,
// apply the border rule at the window corners, take the centre sample, run the tap
// pass and finish each view's ZNCC into cj / ok.
template <int NV, int G, int J0>
__device__ __forceinline__ void view_groups(const Args& A, const RefPix& rp, const Hyp& h,
                                            const float* __restrict__ tile, const float* __restrict__ wcol,
                                            const float* __restrict__ wsp, float (&cj)[NV], bool (&ok)[NV]) {
  if constexpr (J0 < NV) {
    constexpr int GG = (NV - J0 < G) ? (NV - J0) : G;
    float Hm[GG][9], bc[GG];
    bool fast[GG];
    const int r = A.s * A.R;
    const float Xmax = rp.X0 + (float)r, Ymax = rp.Y0 + (float)r;
    bool need_exact = false, any_ok = false;
#pragma unroll
    for (int g = 0; g < GG; ++g) {
      const SrcDev& V = A.src[J0 + g];
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
#pragma unroll
        for (int c = 0; c < 3; ++c) Hm[g][rr * 3 + c] = __builtin_fmaf(V.e[rr], h.m[c], V.M[rr * 3 + c]);
      // border rule at the four window corners (IEEE division)
      bool inside = h.ok;
      float wmin = 3.0e38f, wmax = -3.0e38f;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const float X = (float)(rp.x + ((cc & 1) ? r : -r));
        const float Y = (float)(rp.y + ((cc & 2) ? r : -r));
        const float u = __builtin_fmaf(Hm[g][0], X, __builtin_fmaf(Hm[g][1], Y, Hm[g][2]));
        const float v = __builtin_fmaf(Hm[g][3], X, __builtin_fmaf(Hm[g][4], Y, Hm[g][5]));
        const float w = __builtin_fmaf(Hm[g][6], X, __builtin_fmaf(Hm[g][7], Y, Hm[g][8]));
        const float rw = 1.0f / w;
        const float up = u * rw, vp = v * rw;
        inside = inside && (w > 0.0f) && (up >= 0.0f && up <= V.Wm1 && vp >= 0.0f && vp <= V.Hm1);
        wmin = fminf(wmin, w);
        wmax = fmaxf(wmax, w);
      }
      // every tap's computed w lies within 2^-22 S of the corner range (fma error bound)
      const float S = fabsf(Hm[g][6]) * Xmax + fabsf(Hm[g][7]) * Ymax + fabsf(Hm[g][8]);
      const float slack = S * 0x1p-22f;
      fast[g] = (wmin - slack >= 0x1p-100f) && (wmax + slack <= 0x1p100f);
      ok[J0 + g] = inside;
      need_exact = need_exact || (inside && !fast[g]);
      any_ok = any_ok || inside;
      {
        const float u = __builtin_fmaf(Hm[g][0], rp.X0, __builtin_fmaf(Hm[g][1], rp.Y0, Hm[g][2]));
        const float v = __builtin_fmaf(Hm[g][3], rp.X0, __builtin_fmaf(Hm[g][4], rp.Y0, Hm[g][5]));
        const float w = __builtin_fmaf(Hm[g][6], rp.X0, __builtin_fmaf(Hm[g][7], rp.Y0, Hm[g][8]));
        const float rw = 1.0f / w;
        bc[g] = sample_quad(V.quad, V.W, clampf(u * rw, V.Wm1), clampf(v * rw, V.Hm1));
      }
    }
    if (__ballot(any_ok) != 0) {
      float Sb[GG], Sbb[GG], Sab[GG];
      if (__ballot(need_exact) != 0)
        tap_pass<GG, J0, true>(A, rp, tile, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
      else
        tap_pass<GG, J0, false>(A, rp, tile, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
#pragma unroll
      for (int g = 0; g < GG; ++g) {
        if (ok[J0 + g]) {
          const float mu_b = Sb[g] / rp.S_w;
          const float var_b = Sbb[g] / rp.S_w - mu_b * mu_b;
          const float cov = Sab[g] / rp.S_w - rp.mu_a * mu_b;
          if (var_b >= A.eps_v) {
            float z = cov / __builtin_sqrtf(rp.var_a * var_b);
            z = fminf(fmaxf(z, -1.0f), 1.0f);
            cj[J0 + g] = 1.0f - z;
          } else {
            ok[J0 + g] = false;
          }
        }
      }
    }
    view_groups<NV, G, J0 + G>(A, rp, h, tile, wcol, wsp, cj, ok);
  }
}

// Cost (Eq. 5 over the best-K valid sources) of plane (n, d) at pixel rp; optionally the
// per-source costs and the validity mask.
template <int NV, int G, bool PERVIEW>
__device__ float plane_cost(const Args& A, const RefPix& rp, const float* __restrict__ tile,
                            const float* __restrict__ wcol, const float* __restrict__ wsp, float nx, float ny,
                            float nz, float d, float* pv_out, uint32_t* valid_out) {
  float cj[NV];
  bool ok[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    cj[j] = kCmax;
    ok[j] = false;
  }
  const float nr = dot3f(nx, ny, nz, rp.rx, rp.ry, rp.rz);
  Hyp h;
  h.ok = rp.ok && (nr < 0.0f);
  if (__ballot(h.ok) != 0) {
    const float rho = d * nr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float kn = __builtin_fmaf(A.Kinv[0 * 3 + c], nx, __builtin_fmaf(A.Kinv[1 * 3 + c], ny, A.Kinv[2 * 3 + c] * nz));
      h.m[c] = kn / rho;
    }
    view_groups<NV, G, 0>(A, rp, h, tile, wcol, wsp, cj, ok);
  }
  if (PERVIEW) {
    uint32_t vm = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      pv_out[j] = ok[j] ? cj[j] : kCmax;
      vm |= ok[j] ? (1u << j) : 0u;
    }
    *valid_out = vm;
  }
  // Eq. 5 over the K lowest (C_j, j) valid sources, summed in ascending order
  int nvalid = 0;
#pragma unroll
  for (int j = 0; j < NV; ++j) nvalid += ok[j] ? 1 : 0;
  const int K = A.top_k > 0 ? (A.top_k < nvalid ? A.top_k : nvalid) : nvalid;
  float sum = 0.0f;
  uint32_t used = 0;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < K) {
      float best = 0.0f;
      int bj = -1;
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        const bool cand = ok[j] && !((used >> j) & 1u);
        if (cand && (bj < 0 || cj[j] < best)) {
          best = cj[j];
          bj = j;
        }
      }
      used |= 1u << bj;
      sum = sum + 1.0f / fmaxf(best, A.eps_c);
    }
  }
  return K > 0 ? (float)K / sum : kCmax;
}

// ---------------------------------------------------------------------------- plane helpers
// viewing ray K^-1 (x, y, 1) in float
__device__ __forceinline__ void ray_f(const Args& A, int x, int y, float& rx, float& ry, float& rz) {
  const float X = (float)x, Y = (float)y;
  rx = __builtin_fmaf(A.Kinv[0], X, __builtin_fmaf(A.Kinv[1], Y, A.Kinv[2]));
  ry = __builtin_fmaf(A.Kinv[3], X, __builtin_fmaf(A.Kinv[4], Y, A.Kinv[5]));
  rz = __builtin_fmaf(A.Kinv[6], X, __builtin_fmaf(A.Kinv[7], Y, A.Kinv[8]));
}

// unit normal from spherical angles (FP64), facing the camera at pixel (x, y), rounded to float
__device__ __forceinline__ void facing_normal(const Args& A, int x, int y, double theta, double phi, float& nx,
                                              float& ny, float& nz) {
  double n0 = cos(theta) * sin(phi), n1 = sin(theta) * sin(phi), n2 = cos(phi);
  const double X = (double)x, Y = (double)y;
  const double r0 = __builtin_fma(A.Kinv_d[0], X, __builtin_fma(A.Kinv_d[1], Y, A.Kinv_d[2]));
  const double r1 = __builtin_fma(A.Kinv_d[3], X, __builtin_fma(A.Kinv_d[4], Y, A.Kinv_d[5]));
  const double r2 = __builtin_fma(A.Kinv_d[6], X, __builtin_fma(A.Kinv_d[7], Y, A.Kinv_d[8]));
  if (n0 * r0 + n1 * r1 + n2 * r2 > 0.0) {
    n0 = -n0;
    n1 = -n1;
    n2 = -n2;
  }
  nx = (float)n0;
  ny = (float)n1;
  nz = (float)n2;
}

__device__ __forceinline__ bool pixel_valid(const Args& A, int x, int y) {
  const int r = A.s * A.R;
  return x - r >= 0 && x + r <= A.W - 1 && y - r >= 0 && y + r <= A.H - 1;
}

// propagation offsets of the "up" direction (other colour: |dx| + |dy| odd); the other
// directions are rotations: down (dx, -dy), left (dy, dx), right (-dy, dx)
__constant__ int8_t kNearUp[9][2] = {{0, -1}, {-1, -2}, {1, -2}, {0, -3}, {-2, -3}, {2, -3}, {-1, -4}, {1, -4}, {0, -5}};

// ---------------------------------------------------------------------------- candidate generation
// Candidate planes live in S.cand: slot k of compacted pixel i at S.cand[k * A.H * A.Wc + i];
// d = NaN marks an empty slot.

__device__ __forceinline__ bool colour_pixel(const Args& A, int colour, int& x, int& y, int& ci) {
  y = blockIdx.y;
  ci = blockIdx.x * blockDim.x + threadIdx.x;
  x = 2 * ci + ((y + colour) & 1);
  return ci < A.Wc && y < A.H && x < A.W;
}

// random initialisation (Sec. III-B): d uniform in the depth range, theta in [0, 2 pi],
// phi in [-pi/2, pi/2], n = (cos theta sin phi, sin theta sin phi, cos phi) turned to face
// the camera; slot 1 carries the caller's proposal, if any
__global__ void cand_init_kernel(Args A, Step S) {
  int x, y, ci;
  if (!colour_pixel(A, S.colour, x, y, ci)) return;
  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  float4 c0 = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
  if (pixel_valid(A, x, y)) {
    const uint32_t plin = (uint32_t)((uint64_t)y * (uint64_t)A.W + (uint64_t)x);
    const uint4 rnd = philox10(make_uint4(plin, 0u, 0u, 0u), A.seed_lo, A.seed_hi);
    const float u0 = u24(rnd.x), u1 = u24(rnd.y), u2 = u24(rnd.z);
    const float d = __builtin_fmaf(u0, A.d_hi - A.d_lo, A.d_lo);
    const double theta = 2.0 * kPiD * (double)u1;
    const double phi = kPiD * ((double)u2 - 0.5);
    float nx, ny, nz;
    facing_normal(A, x, y, theta, phi, nx, ny, nz);
    c0 = make_float4(nx, ny, nz, d);
  }
  S.cand[cidx] = c0;
  if (S.planes_in) S.cand[plane_sz + cidx] = reinterpret_cast<const float4*>(S.planes_in)[(size_t)y * A.W + x];
}

// red/black propagation candidates: per region, the other colour's lowest-cost pixel q
// (first in enumeration order on ties), its plane re-expressed at p by ray-plane
// intersection; empty if the plane does not face p's ray or leaves the depth range
__global__ void cand_prop_kernel(Args A, Step S) {
  int x, y, ci;
  if (!colour_pixel(A, S.colour, x, y, ci)) return;
  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  const bool valid = pixel_valid(A, x, y);
  const int oc = 1 - S.colour;
  const float4* __restrict__ oplane = A.plane[oc];
  const float* __restrict__ ocost = A.cost[oc];
  float rx, ry, rz;
  ray_f(A, x, y, rx, ry, rz);
  for (int g = 0; g < 8; ++g) {
    float4 cand = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    if (valid) {
      const int dir = g & 3;
      const bool far = g >= 4;
      const int count = far ? 10 : 9;
      int qx = -1, qy = -1;
      float qc = 0.0f;
      for (int i = 0; i < count; ++i) {
        const int dx = far ? 0 : (int)kNearUp[i][0];
        const int dy = far ? -(2 * (i + 3) + 1) : (int)kNearUp[i][1];
        int ox, oy;
        if (dir == 0) { ox = dx; oy = dy; }
        else if (dir == 1) { ox = dx; oy = -dy; }
        else if (dir == 2) { ox = dy; oy = dx; }
        else { ox = -dy; oy = dx; }
        const int xq = x + ox, yq = y + oy;
        if (xq < 0 || xq >= A.W || yq < 0 || yq >= A.H || !pixel_valid(A, xq, yq)) continue;
        const float c = ocost[(size_t)yq * A.Wc + (xq >> 1)];
        if (qx < 0 || c < qc) { qx = xq; qy = yq; qc = c; }
      }
      if (qx >= 0) {
        const float4 q = oplane[(size_t)qy * A.Wc + (qx >> 1)];
        float rqx, rqy, rqz;
        ray_f(A, qx, qy, rqx, rqy, rqz);
        const float num = dot3f(q.x, q.y, q.z, q.w * rqx, q.w * rqy, q.w * rqz);
        const float den = dot3f(q.x, q.y, q.z, rx, ry, rz);
        const float dn = num / den;
        if ((den < 0.0f) && (dn >= A.d_lo && dn <= A.d_hi)) cand = make_float4(q.x, q.y, q.z, dn);
      }
    }
    S.cand[g * plane_sz + cidx] = cand;
  }
}

// random refinement candidates (Sec. III-C): Delta_d in [-d_hi/4, d_hi/4], Delta_theta in
// [-pi/2, pi/2], Delta_phi in [-pi/12, pi/12]; (d_new, n_old), (d_old, n_new), (d_new, n_new),
// the two using d_new empty when it leaves the depth range
__global__ void cand_refine_kernel(Args A, Step S) {
  int x, y, ci;
  if (!colour_pixel(A, S.colour, x, y, ci)) return;
  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  const float qnan = __int_as_float(0x7fc00000);
  float4 c0 = make_float4(0.f, 0.f, 0.f, qnan), c1 = c0, c2 = c0;
  if (pixel_valid(A, x, y)) {
    const float4 cur = A.plane[S.colour][cidx];
    const uint32_t plin = (uint32_t)((uint64_t)y * (uint64_t)A.W + (uint64_t)x);
    const uint4 rnd = philox10(make_uint4(plin, (uint32_t)S.iteration, 1u, 0u), A.seed_lo, A.seed_hi);
    const float u0 = u24(rnd.x), u1 = u24(rnd.y), u2 = u24(rnd.z);
    const float dd = (2.0f * u0 - 1.0f) * (A.d_hi * 0.25f);
    const float d_new = cur.w + dd;
    const bool d_ok = d_new >= A.d_lo && d_new <= A.d_hi;
    const double theta = atan2((double)cur.y, (double)cur.x);
    const double phi = acos(fmin(fmax((double)cur.z, -1.0), 1.0));
    const double dth = (2.0 * (double)u1 - 1.0) * (kPiD / 2.0);
    const double dph = (2.0 * (double)u2 - 1.0) * (kPiD / 12.0);
    float nx, ny, nz;
    facing_normal(A, x, y, theta + dth, phi + dph, nx, ny, nz);
    if (d_ok) c0 = make_float4(cur.x, cur.y, cur.z, d_new);
    c1 = make_float4(nx, ny, nz, cur.w);
    if (d_ok) c2 = make_float4(nx, ny, nz, d_new);
  }
  S.cand[cidx] = c0;
  S.cand[plane_sz + cidx] = c1;
  S.cand[2 * plane_sz + cidx] = c2;
}

// ---------------------------------------------------------------------------- evaluate and select
// MODE 0: initialisation: slot 0 (random plane) is taken, slot 1 (proposal) replaces it when
//         its cost is not higher.
// MODE 1: update: candidates 0..ncand-1 in order replace the current plane on a strictly
//         lower cost (the first of equal costs wins).
// MODE 2: cost of row-major input planes (teacher-forced evaluation), per source optional.
template <int NV, int G, int MODE>
__global__ __launch_bounds__(256) void select_kernel(Args A, Step S) {
  extern __shared__ float lds[];
  float* wcol = lds;                 // 256
  float* wsp = lds + 256;            // (2R+1)^2
  float* tile = wsp + A.n_taps;      // TH x TW
  const int colour = S.colour;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = A.s * A.R;
  const int x_org = blockIdx.x * 128 - r;
  const int y_org = blockIdx.y * 4 - r;

  // stage weights and the reference tile (fp16 -> fp32) in LDS
  for (int i = threadIdx.x; i < 256; i += 256) wcol[i] = A.wcol[i];
  for (int i = threadIdx.x; i < A.n_taps; i += 256) wsp[i] = A.wsp[i];
  const int tsize = A.TW * A.TH;
  for (int i = threadIdx.x; i < tsize; i += 256) {
    const int ty = i / A.TW, tx = i - ty * A.TW;
    const int gx = min(max(x_org + tx, 0), A.W - 1);
    const int gy = min(max(y_org + ty, 0), A.H - 1);
    tile[i] = __half2float(A.ref[(size_t)gy * A.W + gx]);
  }
  __syncthreads();

  const int y = blockIdx.y * 4 + wave;
  const int ci = blockIdx.x * 64 + lane;
  const int par = (y + colour) & 1;
  const int x = 2 * ci + par;
  const bool in_img = y < A.H && x < A.W && ci < A.Wc;
  const bool valid = in_img && pixel_valid(A, x, y);
  if (__ballot(in_img) == 0) return;

  RefPix rp;
  rp.x = x;
  rp.y = y;
  rp.X0 = (float)x;
  rp.Y0 = (float)y;
  rp.ok = false;
  rp.tbase = wave * A.TW + 2 * lane + par;  // tile position of the window's first tap (-R, -R)
  ray_f(A, x, y, rp.rx, rp.ry, rp.rz);
  rp.a_c = 0.0f;
  rp.S_w = 1.0f;
  rp.mu_a = 0.0f;
  rp.var_a = 0.0f;
  if (valid) {
    rp.a_c = tile[(wave + r) * A.TW + 2 * lane + par + r];
    float S_w = 0.0f, S_a = 0.0f, S_aa = 0.0f;
    int t = 0;
    for (int k2 = 0; k2 <= 2 * A.R; ++k2) {
      const float* trow = tile + rp.tbase + k2 * A.s * A.TW;
      for (int k1 = 0; k1 <= 2 * A.R; ++k1, ++t) {
        const float a = trow[k1 * A.s] - rp.a_c;
        float w = 1.0f;
        if (A.bilateral) w = wcol[(int)fabsf(a)] * wsp[t];
        const float wa = w * a;
        S_w = S_w + w;
        S_a = S_a + wa;
        S_aa = __builtin_fmaf(wa, a, S_aa);
      }
    }
    rp.S_w = S_w;
    rp.mu_a = S_a / S_w;
    rp.var_a = S_aa / S_w - rp.mu_a * rp.mu_a;
    rp.ok = rp.var_a >= A.eps_v;
  }
  if (!in_img) return;

  if (MODE == 2) {
    const size_t p = (size_t)y * A.W + x;
    float c = kCmax;
    float pv[NV];
    uint32_t vm = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) pv[j] = kCmax;
    if (S.count && lane == 0) atomicAdd(S.count, (unsigned long long)__popcll(__ballot(valid)));
    if (valid) {
      const float4 pl = reinterpret_cast<const float4*>(S.planes_in)[p];
      c = plane_cost<NV, G, true>(A, rp, tile, wcol, wsp, pl.x, pl.y, pl.z, pl.w, pv, &vm);
    }
    S.cost_out[p] = c;
    if (S.per_view_out)
      for (int j = 0; j < NV; ++j) S.per_view_out[p * NV + j] = pv[j];
    if (S.valid_out)
      for (int j = 0; j < NV; ++j) S.valid_out[p * NV + j] = (uint8_t)((vm >> j) & 1u);
    return;
  }

  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  float4 best = make_float4(0.f, 0.f, 0.f, 0.f);
  float bc = kCmax;
  if (MODE == 1 && valid) {
    best = A.plane[colour][cidx];
    bc = A.cost[colour][cidx];
  }
  for (int k = 0; k < S.ncand; ++k) {
    const float4 h = S.cand[k * plane_sz + cidx];
    const bool has = valid && !__builtin_isnan(h.w);
    const unsigned long long bal = __ballot(has);
    if (bal == 0) continue;
    if (S.count && lane == 0) atomicAdd(S.count, (unsigned long long)__popcll(bal));
    if (has) {
      const float c = plane_cost<NV, G, false>(A, rp, tile, wcol, wsp, h.x, h.y, h.z, h.w, nullptr, nullptr);
      const bool take = MODE == 0 ? (k == 0 || c <= bc) : (c < bc);
      if (take) {
        bc = c;
        best = h;
      }
    }
  }
  if (MODE == 1 && !valid) return;
  if (!valid) {
    best = make_float4(0.f, 0.f, 0.f, 0.f);
    bc = kCmax;
  }
  A.plane[colour][cidx] = best;
  A.cost[colour][cidx] = bc;
}

// ---------------------------------------------------------------------------- image preparation
// 8-bit image -> fp16 copy (reference tiles) and 8-bit texel quads (bilinear gathers)
__global__ void build_view_kernel(const uint8_t* __restrict__ img, int64_t stride, int W, int H,
                                  __half* __restrict__ plain, uint32_t* __restrict__ quad) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W || y >= H) return;
  const int x1 = min(x + 1, W - 1), y1 = min(y + 1, H - 1);
  const uint32_t i00 = img[(size_t)y * stride + x], i01 = img[(size_t)y * stride + x1];
  const uint32_t i10 = img[(size_t)y1 * stride + x], i11 = img[(size_t)y1 * stride + x1];
  plain[(size_t)y * W + x] = __float2half((float)i00);
  quad[(size_t)y * W + x] = i00 | (i01 << 8) | (i10 << 16) | (i11 << 24);
}

// colour planes -> row-major planes (n, d) + cost, or depth / normal / cost
__global__ void unpack_kernel(const float4* __restrict__ p0, const float4* __restrict__ p1, const float* __restrict__ c0,
                              const float* __restrict__ c1, int W, int H, int Wc, float* __restrict__ planes,
                              float* __restrict__ depth, float* __restrict__ normal, float* __restrict__ cost) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W || y >= H) return;
  const int colour = (x + y) & 1;
  const size_t ci = (size_t)y * Wc + (x >> 1);
  const float4 pl = colour ? p1[ci] : p0[ci];
  const float c = colour ? c1[ci] : c0[ci];
  const size_t p = (size_t)y * W + x;
  if (planes) reinterpret_cast<float4*>(planes)[p] = pl;
  if (depth) depth[p] = pl.w;
  if (normal) {
    normal[3 * p + 0] = pl.x;
    normal[3 * p + 1] = pl.y;
    normal[3 * p + 2] = pl.z;
  }
  if (cost) cost[p] = c;
}

__global__ void pack_kernel(const float* __restrict__ planes, const float* __restrict__ cost, int W, int H, int Wc,
                            float4* __restrict__ p0, float4* __restrict__ p1, float* __restrict__ c0,
                            float* __restrict__ c1) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W || y >= H) return;
  const int colour = (x + y) & 1;
  const size_t ci = (size_t)y * Wc + (x >> 1);
  const size_t p = (size_t)y * W + x;
  const float4 pl = reinterpret_cast<const float4*>(planes)[p];
  if (colour) { p1[ci] = pl; c1[ci] = cost[p]; }
  else { p0[ci] = pl; c0[ci] = cost[p]; }
}

// exhaustive check of rcp_nr against the correctly rounded reciprocal on a range of bit patterns
__global__ void rcp_check_kernel(uint32_t first, uint32_t count, unsigned long long* mismatches, uint32_t* example) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t bits = first + i;
  const float w = __uint_as_float(bits);
  const float fast = rcp_nr(w);
  const float ref = (float)(1.0 / (double)w);
  if (__float_as_uint(fast) != __float_as_uint(ref)) {
    atomicAdd(mismatches, 1ull);
    *example = bits;
  }
}

}  // namespace pmk

// ---------------------------------------------------------------------------- launchers
namespace phimvs_internal {

template <int NV>
static hipError_t launch_nv(int mode, const Args& A, const Step& S, dim3 grid, size_t lds, hipStream_t st) {
  constexpr int G = NV < 2 ? NV : 2;  // two views per pass over the taps (occupancy)
  if (mode == 0) hipLaunchKernelGGL((pmk::select_kernel<NV, G, 0>), grid, dim3(256), lds, st, A, S);
  else if (mode == 1) hipLaunchKernelGGL((pmk::select_kernel<NV, G, 1>), grid, dim3(256), lds, st, A, S);
  else hipLaunchKernelGGL((pmk::select_kernel<NV, G, 2>), grid, dim3(256), lds, st, A, S);
  return hipGetLastError();
}

hipError_t launch_select(int mode, const Args& A, const Step& S, hipStream_t st) {
  const dim3 grid((A.Wc + 63) / 64, (A.H + 3) / 4, 1);
  const size_t lds = sizeof(float) * (256 + A.n_taps + A.TW * A.TH);
  switch (A.n_src) {
    case 1: return launch_nv<1>(mode, A, S, grid, lds, st);
    case 2: return launch_nv<2>(mode, A, S, grid, lds, st);
    case 3: return launch_nv<3>(mode, A, S, grid, lds, st);
    case 4: return launch_nv<4>(mode, A, S, grid, lds, st);
    case 5: return launch_nv<5>(mode, A, S, grid, lds, st);
    case 6: return launch_nv<6>(mode, A, S, grid, lds, st);
    case 7: return launch_nv<7>(mode, A, S, grid, lds, st);
    case 8: return launch_nv<8>(mode, A, S, grid, lds, st);
    case 9: return launch_nv<9>(mode, A, S, grid, lds, st);
    case 10: return launch_nv<10>(mode, A, S, grid, lds, st);
    case 11: return launch_nv<11>(mode, A, S, grid, lds, st);
    case 12: return launch_nv<12>(mode, A, S, grid, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_candidates(int kind, const Args& A, const Step& S, hipStream_t st) {
  const dim3 grid((A.Wc + 127) / 128, A.H);
  if (kind == 0) hipLaunchKernelGGL(pmk::cand_init_kernel, grid, dim3(128), 0, st, A, S);
  else if (kind == 1) hipLaunchKernelGGL(pmk::cand_prop_kernel, grid, dim3(128), 0, st, A, S);
  else hipLaunchKernelGGL(pmk::cand_refine_kernel, grid, dim3(128), 0, st, A, S);
  return hipGetLastError();
}

hipError_t launch_build_view(const uint8_t* img, int64_t stride, int W, int H, __half* plain, uint32_t* quad,
                             hipStream_t st) {
  hipLaunchKernelGGL(pmk::build_view_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, img, stride, W, H, plain, quad);
  return hipGetLastError();
}

hipError_t launch_unpack(const Args& A, float* planes, float* depth, float* normal, float* cost, hipStream_t st) {
  hipLaunchKernelGGL(pmk::unpack_kernel, dim3((A.W + 255) / 256, A.H), dim3(256), 0, st, A.plane[0], A.plane[1],
                     A.cost[0], A.cost[1], A.W, A.H, A.Wc, planes, depth, normal, cost);
  return hipGetLastError();
}

hipError_t launch_pack(const Args& A, const float* planes, const float* cost, hipStream_t st) {
  hipLaunchKernelGGL(pmk::pack_kernel, dim3((A.W + 255) / 256, A.H), dim3(256), 0, st, planes, cost, A.W, A.H, A.Wc,
                     A.plane[0], A.plane[1], A.cost[0], A.cost[1]);
  return hipGetLastError();
}

hipError_t launch_rcp_check(uint32_t first, uint32_t count, unsigned long long* mism, uint32_t* example,
                            hipStream_t st) {
  hipLaunchKernelGGL(pmk::rcp_check_kernel, dim3((count + 255) / 256), dim3(256), 0, st, first, count, mism, example);
  return hipGetLastError();
}

}  // namespace phimvs_internal
