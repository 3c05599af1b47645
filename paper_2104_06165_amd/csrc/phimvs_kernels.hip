// gfx950 kernels of the PatchMatch depth-map estimation step (PHI-MVS Sec. III-B,
// Sec. III-C, Eq. 4, Eq. 5, Algorithm 1 "depth map estimation").
//
// Work decomposition.  The per-pixel state lives in two checkerboard-compacted
// colour planes (red: (x + y) even, black: odd), each H x Wc with Wc = ceil(W / 2):
// pixel (x, y) of colour c sits at column x >> 1 of its colour plane.  A launch covers a
// table of jobs (one reference view each, with its own sources, window and state).  The
// evaluate kernel works on tiles of tile_rows x (256 / tile_rows) compacted pixels of one
// colour; one lane owns one pixel and scores its hypotheses one after the other; for
// each hypothesis it walks the window taps in row-major order and, per tap, the two
// source views of the current pair, so the reference-side tap values (LDS) are read once
// per pair and each view's sums are accumulated in plain tap order (the oracle's order:
// no cross-lane reduction is needed).  Cheap candidate kernels (random initialisation,
// red/black propagation, random refinement) write candidate planes that the evaluate
// kernel scores and selects from.
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

// Pointers read from the job table are generic; naming the global address space keeps
// the accesses global loads/stores (flat ones would also hold the LDS wait counter).
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GLOBAL T* gl(const T* p) { return (const GLOBAL T*)p; }
template <typename T>
__device__ __forceinline__ GLOBAL T* gl(T* p) { return (GLOBAL T*)p; }
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4(const float4* p, size_t i) {
  const f4v v = ((const GLOBAL f4v*)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(float4* p, size_t i, float4 a) {
  f4v v;
  v.x = a.x;
  v.y = a.y;
  v.z = a.z;
  v.w = a.w;
  ((GLOBAL f4v*)p)[i] = v;
}

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

// 1/w correctly rounded (the IEEE quotient) for every w: the fast form when every lane's
// |w| lies in [2^-100, 2^100) (a wave-uniform test, so only one form runs), division else
__device__ __forceinline__ float rcp_ieee(float w) {
  const float a = fabsf(w);
  if (__ballot(!(a >= 0x1p-100f && a < 0x1p100f)) == 0) return rcp_nr(w);
  return 1.0f / w;
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
  const uint32_t q = gl(quad)[__umul24(y0, (uint32_t)W) + x0];
  const float t00 = (float)(q & 0xFFu), t01 = (float)((q >> 8) & 0xFFu);
  const float t10 = (float)((q >> 16) & 0xFFu), t11 = (float)(q >> 24);
  const float top = __builtin_fmaf(fx, t01 - t00, t00);
  const float bot = __builtin_fmaf(fx, t11 - t10, t10);
  return __builtin_fmaf(fy, bot - top, top);
}

// The tap loop's form of the same bilinear sample.  The quad's bytes become FP16
// subnormals k 2^-24 (one byte permute per pair; exact, FP16 denormals are kept):
// lo = (I00, I10), hi = (I01, I11), and one packed FP16 subtraction gives both exact
// differences.  The mixed-precision FMA reads them as FP32 without a conversion, so every
// lerp is the canonical one on values scaled by 2^-24: scaling by a power of two commutes
// with each rounding (all intermediate values are 0 or far above the FP32 normal range's
// lower end), and the caller undoes it exactly in its shift by the centre sample.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2v quad_lo(uint32_t q) {
  return __builtin_bit_cast(h2v, __builtin_amdgcn_perm(0u, q, 0x0c020c00u));
}
__device__ __forceinline__ h2v quad_hi(uint32_t q) {
  return __builtin_bit_cast(h2v, __builtin_amdgcn_perm(0u, q, 0x0c030c01u));
}
// 2^-24 times the bilinear sample of quad q at fractions (fx, fy)
__device__ __forceinline__ float bilerp_scaled(uint32_t q, float fx, float fy) {
  const h2v lo = quad_lo(q), hi = quad_hi(q);
  const h2v df = hi - lo;  // (I01 - I00, I11 - I10) 2^-24, exact
  const float top = __builtin_fmaf(fx, (float)df.x, (float)lo.x);
  const float bot = __builtin_fmaf(fx, (float)df.y, (float)lo.y);
  return __builtin_fmaf(fy, bot - top, top);
}

// Texel-quad gathers through a buffer resource with a 4-byte record stride: the hardware
// scales the record index (no 64-bit address arithmetic per tap) and range-checks it
// against the record count (an index past the end reads 0 instead of faulting).
typedef int v4i32 __attribute__((ext_vector_type(4)));
__device__ int struct_buffer_load_i32(v4i32 rsrc, int vindex, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.buffer.load.i32");
__device__ __forceinline__ v4i32 quad_rsrc(const uint32_t* p, uint32_t n_records) {
  const uint64_t a = (uint64_t)p;
  v4i32 r;
  r.x = (int)(uint32_t)a;                         // base address, low 32 bits
  r.y = (int)((uint32_t)(a >> 32) | (4u << 16));  // base address, high bits; stride 4 bytes
  r.z = (int)n_records;                           // records (range check)
  r.w = 0x00020000;                               // 32-bit data format
  return r;
}

// clamp into [0, hi]; equals fmin(fmax(v, 0), hi) for every non-NaN v (a NaN position only
// arises in a view already ruled invalid, and any result keeps the sample address in range)
__device__ __forceinline__ float clampf(float v, float hi) { return __builtin_amdgcn_fmed3f(v, 0.0f, hi); }

// ---------------------------------------------------------------------------- per-pixel reference data
struct RefPix {
  int x, y;
  float X0, Y0;
  float rx, ry, rz;       // K^-1 (x, y, 1)
  float a_c;              // 4x the centre's grey value (the tile's scale)
  float S_w, mu_a, var_a;
  bool ok;                // pixel valid and reference patch variance >= eps_v
  int tbase;              // LDS index of the window's first tap (integer spacing)
  int tox, toy;           // image position of the reference tile's first texel
};

// Reference value of tap (k1, k2) (0 .. 2R) from the LDS tile: a texel at integer
// spacing; with the window-resize scheme the bilinear value at (x + off[k1], y + off[k2]),
// lerp(a, b, t) = fma(t, b - a, a) as for the sources.  The tile replicates the image
// border, so a position a rounding error outside the image reads the border value.
template <bool FRAC>
__device__ __forceinline__ float ref_tap(const Args& A, const RefPix& rp, const float* __restrict__ tile, int TW,
                                         int k1, int k2) {
  if (!FRAC) return tile[rp.tbase + (k2 * TW + k1) * A.s];
  const float X = rp.X0 + A.off[k1], Y = rp.Y0 + A.off[k2];
  const float fx = __builtin_amdgcn_fractf(X), fy = __builtin_amdgcn_fractf(Y);
  const int ix = (int)floorf(X), iy = (int)floorf(Y);
  const float* q = tile + (iy - rp.toy) * TW + (ix - rp.tox);
  const float t00 = q[0], t01 = q[1], t10 = q[TW], t11 = q[TW + 1];
  const float top = __builtin_fmaf(fx, t01 - t00, t00);
  const float bot = __builtin_fmaf(fx, t11 - t10, t10);
  return __builtin_fmaf(fy, bot - top, top);
}

// Colour weight of a reference tap from its difference to the centre, given four times
// over (the LDS tile holds 4x the grey values, exactly, and every reference difference
// and sum below carries that factor until it is divided out).  A power-of-two factor
// commutes with every rounding in the normal range; a product that falls below it (a
// weight of a difference above 158 grey levels) can differ in bits that vanish in any
// sum with a normal term.  At integer spacing 4 |a - a_c| is the byte offset of the
// table entry, which sits at LDS address 0, so the lookup needs no index arithmetic;
// interpolated taps take the nearest grey level as before.
template <bool FRAC>
__device__ __forceinline__ float colour_weight(const float* __restrict__ wcol, float a4) {
  if (FRAC) return wcol[(int)__builtin_rintf(fabsf(a4) * 0.25f)];
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(wcol) + (uint32_t)fabsf(a4));
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
  const int r = A.rv;
  return x - r >= 0 && x + r <= A.W - 1 && y - r >= 0 && y + r <= A.H - 1;
}

// propagation offsets of the "up" direction (other colour: |dx| + |dy| odd); the other
// directions are rotations: down (dx, -dy), left (dy, dx), right (-dy, dx)
__constant__ int8_t kNearUp[9][2] = {{0, -1}, {-1, -2}, {1, -2}, {0, -3}, {-2, -3}, {2, -3}, {-1, -4}, {1, -4}, {0, -5}};

// ---------------------------------------------------------------------------- plane cost
// Per-hypothesis values shared by every view: m = K^-T n / rho.
struct Hyp {
  float m[3];
  bool ok;  // the reference patch is usable and the plane faces the camera
};

// Sums of a group of G views (J0, J0 + 1, ...) over the window taps in row-major order.
// EXACT selects IEEE division for 1/w; CLAMP clamps every sample position into the image
// (without it the caller has proved every position inside).  The loop is software-pipelined by one tap with
// two alternating register sets: the texel loads of tap t + 1 are issued before tap t's
// texels are interpolated and accumulated, so each gather's latency overlaps a tap of
// arithmetic.  Every tap's arithmetic and the order of accumulation are unchanged.  The
// weight tables hold 1.0 when the weights are off, so w = 1 exactly then.
template <int G, bool EXACT, bool CLAMP, bool FRAC>
__device__ __forceinline__ void tap_pass(const Args& A, int J0, const RefPix& rp, const float* __restrict__ tile,
                                         int TW, const float* __restrict__ wcol, const float* __restrict__ wsp,
                                         const float (&Hm)[G][9], const float (&bc)[G], float (&Sb)[G],
                                         float (&Sbb)[G], float (&Sab)[G]) {
  const int R = A.R, s = A.s;
  const int n = 2 * R + 1;
  const int T = n * n;
  uint32_t Wq[G];
  v4i32 rs[G];
  float Wm1[G], Hm1[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    Sb[g] = 0.0f;
    Sbb[g] = 0.0f;
    Sab[g] = 0.0f;
    Wq[g] = (uint32_t)A.src[J0 + g].W;
    rs[g] = quad_rsrc(A.src[J0 + g].quad, (uint32_t)A.src[J0 + g].W * (uint32_t)A.src[J0 + g].H);
    Wm1[g] = A.src[J0 + g].Wm1;
    Hm1[g] = A.src[J0 + g].Hm1;
  }

  // bases of the row being issued: (H[1] Y + H[2], H[4] Y + H[5], H[7] Y + H[8])
  float rbu[G], rbv[G], rbw[G];
  auto row_bases = [&](int k2) {
    // integer spacing: s (k - R) exactly (integers below 2^24), the table's value, without a load
    const float Y = rp.Y0 + (FRAC ? A.off[k2] : (float)(s * (k2 - R)));
#pragma unroll
    for (int g = 0; g < G; ++g) {
      rbu[g] = __builtin_fmaf(Hm[g][1], Y, Hm[g][2]);
      rbv[g] = __builtin_fmaf(Hm[g][4], Y, Hm[g][5]);
      rbw[g] = __builtin_fmaf(Hm[g][7], Y, Hm[g][8]);
    }
  };
  // warp column k1 of the row whose bases are loaded and issue its texel loads
  auto issue = [&](int k1, uint32_t (&qo)[G], float (&fxo)[G], float (&fyo)[G]) {
    const float X = rp.X0 + (FRAC ? A.off[k1] : (float)(s * (k1 - R)));
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const float u = __builtin_fmaf(Hm[g][0], X, rbu[g]);
      const float v = __builtin_fmaf(Hm[g][3], X, rbv[g]);
      const float ww = __builtin_fmaf(Hm[g][6], X, rbw[g]);
      const float r = EXACT ? 1.0f / ww : rcp_nr(ww);
      const float up = CLAMP ? clampf(u * r, Wm1[g]) : u * r;
      const float vp = CLAMP ? clampf(v * r, Hm1[g]) : v * r;
      // up, vp >= 0: fract(u) = u - floor(u) exactly
      fxo[g] = __builtin_amdgcn_fractf(up);
      fyo[g] = __builtin_amdgcn_fractf(vp);
      const uint32_t x0 = (uint32_t)up, y0 = (uint32_t)vp;
      qo[g] = (uint32_t)struct_buffer_load_i32(rs[g], (int)(__umul24(y0, Wq[g]) + x0), 0, 0, 0);
    }
  };
  // interpolate and accumulate tap (row k2 at trow, column k1, index t)
  auto process = [&](const float* trow, int k1, int k2, int t, const uint32_t (&qi)[G], const float (&fxi)[G],
                     const float (&fyi)[G]) {
    const float a4 = (FRAC ? ref_tap<true>(A, rp, tile, TW, k1, k2) : trow[k1 * s]) - rp.a_c;  // 4 (a - a_c)
    const float w = colour_weight<FRAC>(wcol, a4) * wsp[t];
    const float wa = w * a4;  // 4 w (a - a_c): the cross sum below is 4 S_ab
#pragma unroll
    for (int g = 0; g < G; ++g) {
      // b - b_c with the sample's 2^-24 scale undone inside one exact-product FMA
      const float b = __builtin_fmaf(bilerp_scaled(qi[g], fxi[g], fyi[g]), 0x1p24f, -bc[g]);
      const float tb = w * b;
      Sb[g] = Sb[g] + tb;
      Sbb[g] = __builtin_fmaf(tb, b, Sbb[g]);
      Sab[g] = __builtin_fmaf(wa, b, Sab[g]);
    }
  };
  // one row: column 0 is in flight in (QA); columns alternate between the two register
  // sets (n is odd, so the last column lands in QA again); the next row's column 0 is
  // issued into QB before the last column is processed
  auto row = [&](int k2, uint32_t (&qA)[G], float (&fxA)[G], float (&fyA)[G], uint32_t (&qB)[G], float (&fxB)[G],
                 float (&fyB)[G]) {
    const float* trow = tile + rp.tbase + k2 * s * TW;
    const int t0 = k2 * n;
    for (int c = 0; c + 1 < n; c += 2) {
      issue(c + 1, qB, fxB, fyB);
      process(trow, c, k2, t0 + c, qA, fxA, fyA);
      issue(c + 2, qA, fxA, fyA);
      process(trow, c + 1, k2, t0 + c + 1, qB, fxB, fyB);
    }
    if (k2 + 1 < n) {
      row_bases(k2 + 1);
      issue(0, qB, fxB, fyB);
    }
    process(trow, n - 1, k2, t0 + n - 1, qA, fxA, fyA);
  };

  uint32_t qa[G], qb[G];
  float fxa[G], fya[G], fxb[G], fyb[G];
  row_bases(0);
  issue(0, qa, fxa, fya);
  // rows alternate which register set holds their column 0 (n is odd)
  int k2 = 0;
  for (; k2 + 1 < n; k2 += 2) {
    row(k2, qa, fxa, fya, qb, fxb, fyb);
    row(k2 + 1, qb, fxb, fyb, qa, fxa, fya);
  }
  row(k2, qa, fxa, fya, qb, fxb, fyb);
}

// The same sums with LANES lanes sharing the pixel: lane g (its position within its aligned
// group of LANES lanes) sums the taps t = g, g + LANES, ... in order, every tap computed
// exactly as in tap_pass (the same fma chains; tap_pass only hoists the row's part), and the
// partial sums are then combined by an xor butterfly: at offset o = LANES/2, ..., 1 every
// lane adds the partial sum of lane g xor o to its own.  Addition commutes, so all lanes of
// the group end with the same, bitwise equal, totals.  Lanes of one group always share
// their pixel and candidate, so a butterfly partner is always active.
template <int G, bool EXACT, bool CLAMP, int LANES>
__device__ __forceinline__ void tap_pass_lanes(const Args& A, int J0, const RefPix& rp, const float* __restrict__ tile,
                                               int TW, const float* __restrict__ wcol, const float* __restrict__ wsp,
                                               const float (&Hm)[G][9], const float (&bc)[G], float (&Sb)[G],
                                               float (&Sbb)[G], float (&Sab)[G]) {
  const int R = A.R, s = A.s;
  const int n = 2 * R + 1;
  const int T = n * n;
  const int g = (int)(threadIdx.x % LANES);
  uint32_t Wq[G];
  v4i32 rs[G];
  float Wm1[G], Hm1[G];
#pragma unroll
  for (int v = 0; v < G; ++v) {
    Sb[v] = 0.0f;
    Sbb[v] = 0.0f;
    Sab[v] = 0.0f;
    Wq[v] = (uint32_t)A.src[J0 + v].W;
    rs[v] = quad_rsrc(A.src[J0 + v].quad, (uint32_t)A.src[J0 + v].W * (uint32_t)A.src[J0 + v].H);
    Wm1[v] = A.src[J0 + v].Wm1;
    Hm1[v] = A.src[J0 + v].Hm1;
  }
  for (int t = g; t < T; t += LANES) {
    const int k2 = t / n, k1 = t - k2 * n;
    const float X = rp.X0 + (float)(s * (k1 - R));
    const float Y = rp.Y0 + (float)(s * (k2 - R));
    const float a4 = tile[rp.tbase + (k2 * TW + k1) * s] - rp.a_c;  // 4 (a - a_c)
    const float w = colour_weight<false>(wcol, a4) * wsp[t];
    const float wa = w * a4;
    uint32_t q[G];
    float fx[G], fy[G];
#pragma unroll
    for (int v = 0; v < G; ++v) {
      const float u = __builtin_fmaf(Hm[v][0], X, __builtin_fmaf(Hm[v][1], Y, Hm[v][2]));
      const float vv = __builtin_fmaf(Hm[v][3], X, __builtin_fmaf(Hm[v][4], Y, Hm[v][5]));
      const float ww = __builtin_fmaf(Hm[v][6], X, __builtin_fmaf(Hm[v][7], Y, Hm[v][8]));
      const float r = EXACT ? 1.0f / ww : rcp_nr(ww);
      const float up = CLAMP ? clampf(u * r, Wm1[v]) : u * r;
      const float vp = CLAMP ? clampf(vv * r, Hm1[v]) : vv * r;
      fx[v] = __builtin_amdgcn_fractf(up);
      fy[v] = __builtin_amdgcn_fractf(vp);
      const uint32_t x0 = (uint32_t)up, y0 = (uint32_t)vp;
      q[v] = (uint32_t)struct_buffer_load_i32(rs[v], (int)(__umul24(y0, Wq[v]) + x0), 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < G; ++v) {
      const float b = __builtin_fmaf(bilerp_scaled(q[v], fx[v], fy[v]), 0x1p24f, -bc[v]);
      const float tb = w * b;
      Sb[v] = Sb[v] + tb;
      Sbb[v] = __builtin_fmaf(tb, b, Sbb[v]);
      Sab[v] = __builtin_fmaf(wa, b, Sab[v]);
    }
  }
#pragma unroll
  for (int o = LANES / 2; o >= 1; o >>= 1) {
#pragma unroll
    for (int v = 0; v < G; ++v) {
      Sb[v] = Sb[v] + __shfl_xor(Sb[v], o);
      Sbb[v] = Sbb[v] + __shfl_xor(Sbb[v], o);
      Sab[v] = Sab[v] + __shfl_xor(Sab[v], o);
    }
  }
}

// Views J0 .. J0+G-1: build H_j = M_j + e_j m^T, apply the border rule at the window
// corners, take the centre sample, run the tap pass and finish each view's ZNCC.
// c[g] / ok[g] receive 1 - Z and the validity.
template <int G, bool FR, int LANES>
__device__ __forceinline__ void view_group(const Args& A, int J0, const RefPix& rp, const Hyp& h,
                                           const float* __restrict__ tile, int TW, const float* __restrict__ wcol,
                                           const float* __restrict__ wsp, float (&c)[G], bool (&ok)[G]) {
  float Hm[G][9], bc[G];
  const float Xmax = rp.X0 + A.off[2 * A.R], Ymax = rp.Y0 + A.off[2 * A.R];
  bool need_exact = false, need_clamp = false, any_ok = false;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const SrcDev& V = A.src[J0 + g];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) Hm[g][rr * 3 + cc] = __builtin_fmaf(V.e[rr], h.m[cc], V.M[rr * 3 + cc]);
    // border rule at the four window corners (correctly rounded reciprocals)
    bool inside = h.ok;
    float wmin = 3.0e38f, wmax = -3.0e38f;
    float umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float X = rp.X0 + A.off[(k & 1) ? 2 * A.R : 0];
      const float Y = rp.Y0 + A.off[(k & 2) ? 2 * A.R : 0];
      const float u = __builtin_fmaf(Hm[g][0], X, __builtin_fmaf(Hm[g][1], Y, Hm[g][2]));
      const float v = __builtin_fmaf(Hm[g][3], X, __builtin_fmaf(Hm[g][4], Y, Hm[g][5]));
      const float w = __builtin_fmaf(Hm[g][6], X, __builtin_fmaf(Hm[g][7], Y, Hm[g][8]));
      const float rw = rcp_ieee(w);
      const float up = u * rw, vp = v * rw;
      inside = inside && (w > 0.0f) && (up >= 0.0f && up <= V.Wm1 && vp >= 0.0f && vp <= V.Hm1);
      wmin = fminf(wmin, w);
      wmax = fmaxf(wmax, w);
      umin = fminf(umin, up);
      umax = fmaxf(umax, up);
      vmin = fminf(vmin, vp);
      vmax = fmaxf(vmax, vp);
    }
    // every tap's computed w lies within 2^-22 S of the corner range (fma error bound), so
    // the fast reciprocal is exact for the whole window when this range stays in [2^-100, 2^100]
    const float S = fabsf(Hm[g][6]) * Xmax + fabsf(Hm[g][7]) * Ymax + fabsf(Hm[g][8]);
    const float slack = S * 0x1p-22f;
    const bool fast = (wmin - slack >= 0x1p-100f) && (wmax + slack <= 0x1p100f);
    // Clamp-free taps: a computed tap position differs from the exact one by at most
    // mu = (2^-23 S_u + W 2^-23 S) / w_low + 2^-22 W (two fma roundings in u and w, the
    // reciprocal and the product), doubled here for safety; exact tap positions lie in the
    // convex image of the window (w > 0), so corners at least 2 mu inside put every
    // computed tap inside, where the clamp changes nothing.
    if (inside && fast) {
      const float Su = fabsf(Hm[g][0]) * Xmax + fabsf(Hm[g][1]) * Ymax + fabsf(Hm[g][2]);
      const float Sv = fabsf(Hm[g][3]) * Xmax + fabsf(Hm[g][4]) * Ymax + fabsf(Hm[g][5]);
      // 1 / w_low in [2^-100, 2^100] here; the factor 2 covers a product's rounding
      const float rlow = rcp_nr(wmin - slack);
      const float Wf = V.Wm1 + 1.0f, Hf = V.Hm1 + 1.0f;
      const float mu_u = 2.0f * ((Su + Wf * S) * 0x1p-23f * rlow + Wf * 0x1p-22f);
      const float mu_v = 2.0f * ((Sv + Hf * S) * 0x1p-23f * rlow + Hf * 0x1p-22f);
      const bool safe = umin >= 2.0f * mu_u && umax <= V.Wm1 - 2.0f * mu_u && vmin >= 2.0f * mu_v &&
                        vmax <= V.Hm1 - 2.0f * mu_v;
      need_clamp = need_clamp || !safe;
    }
    ok[g] = inside;
    c[g] = kCmax;
    need_exact = need_exact || (inside && !fast);
    any_ok = any_ok || inside;
    {
      const float u = __builtin_fmaf(Hm[g][0], rp.X0, __builtin_fmaf(Hm[g][1], rp.Y0, Hm[g][2]));
      const float v = __builtin_fmaf(Hm[g][3], rp.X0, __builtin_fmaf(Hm[g][4], rp.Y0, Hm[g][5]));
      const float w = __builtin_fmaf(Hm[g][6], rp.X0, __builtin_fmaf(Hm[g][7], rp.Y0, Hm[g][8]));
      const float rw = rcp_ieee(w);
      bc[g] = sample_quad(V.quad, V.W, clampf(u * rw, V.Wm1), clampf(v * rw, V.Hm1));
    }
    // a lane whose view is invalid walks the constant map to texel (0, 0): its sums are
    // discarded, and its loads stay in bounds and in cache
    if (!inside) {
#pragma unroll
      for (int e = 0; e < 8; ++e) Hm[g][e] = 0.0f;
      Hm[g][8] = 1.0f;
    }
  }
  if (__ballot(any_ok) == 0) return;
  float Sb[G], Sbb[G], Sab[G];
  if constexpr (LANES > 1) {
    if (__ballot(need_exact) != 0)
      tap_pass_lanes<G, true, true, LANES>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
    else if (__ballot(need_clamp) != 0)
      tap_pass_lanes<G, false, true, LANES>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
    else
      tap_pass_lanes<G, false, false, LANES>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
  } else if (FR && A.frac) {
    // the window-resize scheme: computed tap positions X0 + off[k] are monotone in k, so they
    // stay between the corners' and the bounds above hold for them as for integer spacing
    if (__ballot(need_exact) != 0)
      tap_pass<G, true, true, true>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
    else if (__ballot(need_clamp) != 0)
      tap_pass<G, false, true, true>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
    else
      tap_pass<G, false, false, true>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
  } else if (__ballot(need_exact) != 0) {
    tap_pass<G, true, true, false>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
  } else if (__ballot(need_clamp) != 0) {
    tap_pass<G, false, true, false>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
  } else {
    tap_pass<G, false, false, false>(A, J0, rp, tile, TW, wcol, wsp, Hm, bc, Sb, Sbb, Sab);
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (ok[g]) {
      const float mu_b = Sb[g] / rp.S_w;
      const float var_b = Sbb[g] / rp.S_w - mu_b * mu_b;
      const float cov = (Sab[g] * 0.25f) / rp.S_w - rp.mu_a * mu_b;
      if (var_b >= A.eps_v) {
        float z = cov / __builtin_sqrtf(rp.var_a * var_b);
        z = fminf(fmaxf(z, -1.0f), 1.0f);
        c[g] = 1.0f - z;
      } else {
        ok[g] = false;
      }
    }
  }
}

// keep the valid per-source costs in ascending order (equal values keep arrival order)
__device__ __forceinline__ void topk_insert(float (&top)[kMaxTopK], float c) {
#pragma unroll
  for (int i = 0; i < kMaxTopK; ++i) {
    const float t = top[i];
    const bool lt = c < t;
    top[i] = lt ? c : t;
    c = lt ? t : c;
  }
}

// Cost (Eq. 5 over the best-K valid sources) of plane (n, d) at pixel rp.  Sources are
// scored two at a time; per_view / valid (global, optional) receive 1 - Z and the flag of
// each source.  FR: the job may use the window-resize scheme (A.frac decides).
template <bool FR, int LANES = 1>
__device__ __forceinline__ float plane_cost(const Args& A, const RefPix& rp, const float* __restrict__ tile, int TW,
                            const float* __restrict__ wcol, const float* __restrict__ wsp, float nx, float ny,
                            float nz, float d, float* per_view, uint8_t* valid) {
  float top[kMaxTopK];
#pragma unroll
  for (int i = 0; i < kMaxTopK; ++i) top[i] = __builtin_inff();
  int nvalid = 0;
  const int NV = A.n_src;
  const float nr = dot3f(nx, ny, nz, rp.rx, rp.ry, rp.rz);
  Hyp h;
  h.ok = rp.ok && (nr < 0.0f);
  const bool any = __ballot(h.ok) != 0;
  if (any) {
    const float rho = d * nr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float kn = __builtin_fmaf(A.Kinv[0 * 3 + c], nx, __builtin_fmaf(A.Kinv[1 * 3 + c], ny, A.Kinv[2 * 3 + c] * nz));
      h.m[c] = kn / rho;
    }
  }
  for (int j0 = 0; j0 < NV; j0 += 2) {
    float c[2] = {kCmax, kCmax};
    bool ok[2] = {false, false};
    const int gn = NV - j0 < 2 ? 1 : 2;
    if (any) {
      if (gn == 2) {
        view_group<2, FR, LANES>(A, j0, rp, h, tile, TW, wcol, wsp, c, ok);
      } else {
        float c1[1];
        bool ok1[1];
        view_group<1, FR, LANES>(A, j0, rp, h, tile, TW, wcol, wsp, c1, ok1);
        c[0] = c1[0];
        ok[0] = ok1[0];
      }
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      if (g < gn) {
        if (per_view) gl(per_view)[j0 + g] = ok[g] ? c[g] : kCmax;
        if (valid) gl(valid)[j0 + g] = ok[g] ? 1 : 0;
        if (ok[g]) {
          topk_insert(top, c[g]);
          ++nvalid;
        }
      }
    }
  }
  // Eq. 5 over the K lowest valid costs, summed in ascending order
  const int K = A.top_k > 0 ? (A.top_k < nvalid ? A.top_k : nvalid) : nvalid;
  float sum = 0.0f;
#pragma unroll
  for (int i = 0; i < kMaxTopK; ++i)
    if (i < K) sum = sum + 1.0f / fmaxf(top[i], A.eps_c);
  return K > 0 ? (float)K / sum : kCmax;
}

// ---------------------------------------------------------------------------- job lookup
// The job owning global index g of a work space whose jobs start at first(j) (ascending).
// The job owning position i of XCD x's tile list (its bands in job order; a job whose band
// is empty shares its start with the next job and is passed over).
__device__ __forceinline__ int job_of_xcd_tile(const Job* __restrict__ jobs, int n_jobs, int x, int i) {
  int j = 0;
  while (j + 1 < n_jobs && i >= jobs[j + 1].xoff[x]) ++j;
  return j;
}

// Tile (tx, ty) at position p of job J's band on XCD x.  A band is a run of whole tile
// rows; it is walked in columns of kTileBlockW tiles, row-major inside a column, so the
// tiles an XCD has in flight together form a compact block whose source footprint stays in
// that XCD's L2 (row-major order over the full image width would not fit).
constexpr int kTileBlockW = 16;
__device__ __forceinline__ void band_tile(const Job& J, int x, int p, int& tx, int& ty) {
  const int ry0 = J.xband[x] / J.tiles_x;
  const int ry1 = (x + 1 < 8 ? J.xband[x + 1] : J.tiles_x * J.tiles_y) / J.tiles_x;
  const int nrows = ry1 - ry0;  // > 0: the band holds position p
  const int nb = J.tiles_x / kTileBlockW, per = kTileBlockW * nrows;
  const int bc = p / per;
  if (bc < nb) {
    const int q = p - bc * per;
    ty = ry0 + q / kTileBlockW;
    tx = bc * kTileBlockW + q % kTileBlockW;
  } else {
    const int rem = J.tiles_x - nb * kTileBlockW, q = p - nb * per;
    ty = ry0 + q / rem;
    tx = nb * kTileBlockW + q % rem;
  }
}

__device__ __forceinline__ int job_of_cblk(const Job* __restrict__ jobs, int n_jobs, int g) {
  int j = 0;
  while (j + 1 < n_jobs && g >= jobs[j + 1].cblk0) ++j;
  return j;
}

// candidate / unpack blocks: 128 consecutive compacted pixels (or 256 pixels) of one row
__device__ __forceinline__ bool cblk_pixel(const Job* __restrict__ jobs, const Launch& L, int& jb, int& x, int& y,
                                           int& ci) {
  const int g = blockIdx.x;
  jb = job_of_cblk(jobs, L.n_jobs, g);
  const Job& J = jobs[jb];
  const int local = g - J.cblk0;
  y = local / J.cblk_x;
  ci = (local - y * J.cblk_x) * 128 + (int)threadIdx.x;
  x = 2 * ci + ((y + L.colour) & 1);
  return ci < J.A.Wc && y < J.A.H && x < J.A.W;
}

// ---------------------------------------------------------------------------- candidate generation
// Candidate planes live in J.cand: slot k of compacted pixel i at J.cand[k * H * Wc + i];
// d = NaN marks an empty slot.

// random initialisation (Sec. III-B): d uniform in the depth range, theta in [0, 2 pi],
// phi in [-pi/2, pi/2], n = (cos theta sin phi, sin theta sin phi, cos phi) turned to face
// the camera; slot 1 carries the caller's proposal, if any
__global__ __launch_bounds__(128) void cand_init_kernel(const Job* __restrict__ jobs, Launch L) {
  int jb, x, y, ci;
  if (!cblk_pixel(jobs, L, jb, x, y, ci)) return;
  const Job& J = jobs[jb];
  const Args& A = J.A;
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
  J.cand[cidx] = c0;
  if (J.planes_in) J.cand[plane_sz + cidx] = reinterpret_cast<const float4*>(J.planes_in)[(size_t)y * A.W + x];
}

__device__ __forceinline__ bool same4(float4 a, float4 b) {
  return __float_as_uint(a.x) == __float_as_uint(b.x) && __float_as_uint(a.y) == __float_as_uint(b.y) &&
         __float_as_uint(a.z) == __float_as_uint(b.z) && __float_as_uint(a.w) == __float_as_uint(b.w);
}

// red/black propagation candidates: per region, the other colour's lowest-cost pixel q
// (first in enumeration order on ties), its plane re-expressed at p by ray-plane
// intersection; empty if the plane does not face p's ray or leaves the depth range.
// A candidate bitwise equal to an earlier one, or (skip_current) to the pixel's current
// plane, has that plane's cost, so under the strict-improvement rule it can never be
// taken: it is left empty, which leaves the selection's result unchanged.  The same holds
// for a candidate that the previous propagation launch of this colour offered the pixel
// (hist_mode 2): that launch left the pixel's stored cost at or below the candidate's
// cost (it was either not taken, or taken and the pixel's cost is its cost or lower), and a
// stored cost only decreases afterwards, under the library's own steps.  hist_mode >= 1
// records this launch's candidates, as computed, for the next launch of the colour.
__global__ __launch_bounds__(128) void cand_prop_kernel(const Job* __restrict__ jobs, Launch L) {
  int jb, x, y, ci;
  if (!cblk_pixel(jobs, L, jb, x, y, ci)) return;
  const Job& J = jobs[jb];
  const Args& A = J.A;
  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  const bool valid = pixel_valid(A, x, y);
  const int oc = 1 - L.colour;
  const float4* __restrict__ oplane = A.plane[oc];
  const GLOBAL float* __restrict__ ocost = gl(A.cost[oc]);
  float rx, ry, rz;
  ray_f(A, x, y, rx, ry, rz);
  const bool skip_dup = A.score_all < 2;
  const bool skip_cur = skip_dup && L.skip_current;
  const int hist_mode = A.score_all == 0 ? L.hist_mode : 0;
  const float4 cur = valid && skip_cur ? ld4(A.plane[L.colour], cidx) : make_float4(0.f, 0.f, 0.f, 0.f);
  float4 prev[8], fresh[8];
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    float4 cand = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    if (valid) {
      const int dir = g & 3;
      const bool far = g >= 4;
      const int count = far ? 10 : 9;
      // every offset's cost is loaded first (at index 0 where the offset is unusable), so
      // that the region's loads are in flight together; then the usable ones are compared
      // in enumeration order
      int xs[10], ys[10];
      bool use[10];
      float cs_[10];
#pragma unroll
      for (int i = 0; i < count; ++i) {
        const int dx = far ? 0 : (int)kNearUp[i][0];
        const int dy = far ? -(2 * (i + 3) + 1) : (int)kNearUp[i][1];
        int ox, oy;
        if (dir == 0) { ox = dx; oy = dy; }
        else if (dir == 1) { ox = dx; oy = -dy; }
        else if (dir == 2) { ox = dy; oy = dx; }
        else { ox = -dy; oy = dx; }
        xs[i] = x + ox;
        ys[i] = y + oy;
        use[i] = !(xs[i] < 0 || xs[i] >= A.W || ys[i] < 0 || ys[i] >= A.H || !pixel_valid(A, xs[i], ys[i]));
        cs_[i] = ocost[use[i] ? (size_t)ys[i] * A.Wc + (xs[i] >> 1) : 0];
      }
      int qx = -1, qy = -1;
      float qc = 0.0f;
#pragma unroll
      for (int i = 0; i < count; ++i)
        if (use[i] && (qx < 0 || cs_[i] < qc)) { qx = xs[i]; qy = ys[i]; qc = cs_[i]; }
      if (qx >= 0) {
        const float4 q = ld4(oplane, (size_t)qy * A.Wc + (qx >> 1));
        float rqx, rqy, rqz;
        ray_f(A, qx, qy, rqx, rqy, rqz);
        const float num = dot3f(q.x, q.y, q.z, q.w * rqx, q.w * rqy, q.w * rqz);
        const float den = dot3f(q.x, q.y, q.z, rx, ry, rz);
        const float dn = num / den;
        if ((den < 0.0f) && (dn >= A.d_lo && dn <= A.d_hi)) cand = make_float4(q.x, q.y, q.z, dn);
      }
    }
    fresh[g] = cand;
    if (skip_dup && !__builtin_isnan(cand.w)) {
      bool dup = skip_cur && same4(cand, cur);
#pragma unroll
      for (int j = 0; j < g; ++j) dup = dup || same4(cand, prev[j]);
      if (dup) cand = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    }
    prev[g] = cand;
  }
  float4* hist = J.hist[L.colour];
  if (valid && hist_mode == 2) {
    float4 old[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) old[k] = ld4(hist, k * plane_sz + cidx);
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      if (__builtin_isnan(prev[g].w)) continue;
      bool seen = false;
#pragma unroll
      for (int k = 0; k < 8; ++k) seen = seen || same4(prev[g], old[k]);
      if (seen) prev[g] = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    }
  }
  if (valid && hist_mode >= 1) {
#pragma unroll
    for (int g = 0; g < 8; ++g) st4(hist, g * plane_sz + cidx, fresh[g]);
  }
#pragma unroll
  for (int g = 0; g < 8; ++g) st4(J.cand, g * plane_sz + cidx, prev[g]);
}

// random refinement candidates (Sec. III-C): Delta_d in [-d_hi/4, d_hi/4], Delta_theta in
// [-pi/2, pi/2], Delta_phi in [-pi/12, pi/12]; (d_new, n_old), (d_old, n_new), (d_new, n_new),
// the two using d_new empty when it leaves the depth range
__global__ __launch_bounds__(128) void cand_refine_kernel(const Job* __restrict__ jobs, Launch L) {
  int jb, x, y, ci;
  if (!cblk_pixel(jobs, L, jb, x, y, ci)) return;
  const Job& J = jobs[jb];
  const Args& A = J.A;
  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  const float qnan = __int_as_float(0x7fc00000);
  float4 c0 = make_float4(0.f, 0.f, 0.f, qnan), c1 = c0, c2 = c0;
  if (pixel_valid(A, x, y)) {
    const float4 cur = A.plane[L.colour][cidx];
    const uint32_t plin = (uint32_t)((uint64_t)y * (uint64_t)A.W + (uint64_t)x);
    const uint4 rnd = philox10(make_uint4(plin, (uint32_t)L.iteration, 1u, 0u), A.seed_lo, A.seed_hi);
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
  J.cand[cidx] = c0;
  J.cand[plane_sz + cidx] = c1;
  J.cand[2 * plane_sz + cidx] = c2;
}

// ---------------------------------------------------------------------------- evaluate and select
// A tile is tile_rows rows x (256 / tile_rows) compacted pixels of one colour of one job.
// mode 0: initialisation (slot 0, the random plane, is taken; slot 1, a proposal, replaces
// it when not more expensive).  mode 1: update (candidates 0..ncand-1 in order replace the
// current plane on a strictly lower cost; the first of equal costs wins).  In both, the
// tile's non-empty (pixel, slot) pairs form one list in LDS that every lane of the
// workgroup's waves draws from, whatever its pixel, so that empty slots, left-out
// duplicates and pixels outside the image take no lane; each pair's cost goes to LDS, and
// each pixel's own lane then makes the selection in slot order.  mode 2: cost of row-major
// input planes, one lane per pixel, optionally per source (a plane whose depth is NaN
// scores C_max with every source invalid).
//
// Dynamic LDS: the compaction's arrays (kCompactLds floats), the spatial weights, then the
// reference tile.
template <bool FR, bool DEPTH>
__device__ __forceinline__ void eval_tile(const Job& J, const Launch& L, int tile_x, int tile_y, float* wcol,
                                          float* lds) {
  const Args& A = J.A;
  const bool frac = FR && A.frac;
  const int TR = L.tile_rows;
  const int TC = kBlock / TR;  // compacted columns per tile
  const int r = A.halo;
  const int TW = 2 * TC + 2 * r, TH = TR + 2 * r;
  float* ref_lds = lds;                                     // S_w (-1: not usable), mu_a, var_a per pixel
  float* cost_lds = lds + 3 * kBlock;                       // cost of slot k of pixel p at [k][p]
  uint16_t* item_lds = reinterpret_cast<uint16_t*>(lds + 11 * kBlock);  // (pixel << 3 | slot)
  int* wave_total = reinterpret_cast<int*>(lds + 15 * kBlock);
  float* wsp = lds + kCompactLds;  // n_taps
  float* tile_lds = wsp + A.n_taps;
  const int x_org = tile_x * 2 * TC - r;
  const int y_org = tile_y * TR - r;
  for (int i = threadIdx.x; i < 256; i += kBlock) wcol[i] = gl(A.wcol)[i];
  for (int i = threadIdx.x; i < A.n_taps; i += kBlock) wsp[i] = gl(A.wsp)[i];
  for (int i = threadIdx.x; i < TW * TH; i += kBlock) {
    const int ty = i / TW, tx = i - ty * TW;
    const int gx = min(max(x_org + tx, 0), A.W - 1);
    const int gy = min(max(y_org + ty, 0), A.H - 1);
    const unsigned short hb = gl(reinterpret_cast<const unsigned short*>(A.ref))[(size_t)gy * A.W + gx];
    tile_lds[i] = 4.0f * __half2float(__ushort_as_half(hb));  // 4x the grey value, exact
  }
  __syncthreads();

  const int row = threadIdx.x / TC, col = threadIdx.x - row * TC;
  const int colour = L.colour;
  const int y = tile_y * TR + row;
  const int ci = tile_x * TC + col;
  const int par = (y + colour) & 1;
  const int x = 2 * ci + par;
  const bool in_img = y < A.H && ci < A.Wc && x < A.W;
  const bool valid = in_img && pixel_valid(A, x, y);

  RefPix rp;
  rp.x = x;
  rp.y = y;
  rp.X0 = (float)x;
  rp.Y0 = (float)y;
  rp.ok = false;
  rp.tbase = (row + r - A.s * A.R) * TW + 2 * col + par + r - A.s * A.R;  // first tap (-R, -R)
  rp.tox = x_org;
  rp.toy = y_org;
  ray_f(A, x, y, rp.rx, rp.ry, rp.rz);
  rp.a_c = 0.0f;
  rp.S_w = 1.0f;
  rp.mu_a = 0.0f;
  rp.var_a = 0.0f;
  if (valid) {
    rp.a_c = tile_lds[(row + r) * TW + 2 * col + par + r];
    float S_w = 0.0f, S_a4 = 0.0f, S_aa16 = 0.0f;  // S_a and S_aa, 4 and 16 times over
    int t = 0;
    for (int k2 = 0; k2 <= 2 * A.R; ++k2) {
      const float* trow = tile_lds + rp.tbase + k2 * A.s * TW;
      for (int k1 = 0; k1 <= 2 * A.R; ++k1, ++t) {
        const float a4 = (frac ? ref_tap<true>(A, rp, tile_lds, TW, k1, k2) : trow[k1 * A.s]) - rp.a_c;
        const float w = (frac ? colour_weight<true>(wcol, a4) : colour_weight<false>(wcol, a4)) * wsp[t];
        const float wa4 = w * a4;
        S_w = S_w + w;
        S_a4 = S_a4 + wa4;
        S_aa16 = __builtin_fmaf(wa4, a4, S_aa16);
      }
    }
    rp.S_w = S_w;
    rp.mu_a = (S_a4 * 0.25f) / S_w;
    rp.var_a = (S_aa16 * 0.0625f) / S_w - rp.mu_a * rp.mu_a;
    rp.ok = rp.var_a >= A.eps_v;
  }
  const int lane = threadIdx.x & 63;

  if (L.mode == 2) {
    if (in_img) {
      const size_t p = (size_t)y * A.W + x;
      float c = kCmax;
      float* pv = J.per_view_out ? J.per_view_out + p * A.n_src : nullptr;
      uint8_t* vm = J.valid_out ? J.valid_out + p * A.n_src : nullptr;
      float4 pl = make_float4(0.f, 0.f, 0.f, 0.f);
      if (valid) pl = ld4(reinterpret_cast<const float4*>(J.planes_in), p);
      // a plane whose depth is NaN fails the border rule in every source, so it scores
      // C_max with every source invalid: written without evaluating it (waves whose
      // planes are all such skip the tap passes)
      const bool score = valid && !__builtin_isnan(pl.w);
      const unsigned long long bal = __ballot(score);
      if (L.count && lane == 0) atomicAdd(L.count, (unsigned long long)__popcll(bal));
      if (score) {
        c = plane_cost<FR>(A, rp, tile_lds, TW, wcol, wsp, pl.x, pl.y, pl.z, pl.w, pv, vm);
      } else {
        for (int j = 0; j < A.n_src; ++j) {
          if (pv) gl(pv)[j] = kCmax;
          if (vm) gl(vm)[j] = 0;
        }
      }
      gl(J.cost_out)[p] = c;
    }
    return;
  }

  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  // this pixel's reference data for whichever lane scores its candidates
  ref_lds[threadIdx.x] = rp.ok ? rp.S_w : -1.0f;
  ref_lds[kBlock + threadIdx.x] = rp.mu_a;
  ref_lds[2 * kBlock + threadIdx.x] = rp.var_a;
  unsigned live = 0;  // non-empty slots
  if (valid)
    for (int k = 0; k < L.ncand; ++k)
      if (!__builtin_isnan(gl(J.cand)[k * plane_sz + cidx].w)) live |= 1u << k;
  // the list: pixel order, slot order within a pixel (exclusive prefix of the counts over
  // the workgroup: a scan within each wave, then the totals of the earlier waves); or, with
  // order_by_depth, by buckets of the candidate's inverse depth, so that a wave's lanes
  // sample nearby points of each source.  Each item's cost is computed on its own and the
  // selection below reads the costs in slot order, so the order of the list changes no
  // result.

  const int cnt = __popc(live);
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  const int wave = threadIdx.x >> 6;
  if (lane == 63) wave_total[wave] = incl;
  __syncthreads();
  int n_items = 0, off = incl - cnt;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    n_items += wave_total[w];
    if (w < wave) off += wave_total[w];
  }
  if constexpr (!DEPTH) {
    for (unsigned m = live; m; m &= m - 1) item_lds[off++] = (uint16_t)((threadIdx.x << 3) | (__ffs(m) - 1));
  } else {
    // counting sort into kDepthBuckets (= kBlock) buckets of 1/d over [1/d_hi, 1/d_lo]:
    // counts, an exclusive scan over the workgroup (one bucket per thread), then each item
    // takes the next place of its bucket (the order within a bucket is whichever the atomics
    // give).  A candidate's depth is read again from its slot where needed (a cache hit)
    // rather than kept in registers.
    int* bucket = reinterpret_cast<int*>(lds + kDepthBucketLds);
    bucket[threadIdx.x] = 0;
    __syncthreads();
    const float inv_lo = 1.0f / A.d_hi, scale = (float)kDepthBuckets / (1.0f / A.d_lo - 1.0f / A.d_hi);
    auto bucket_of = [&](int k) {
      const int b = (int)((1.0f / gl(J.cand)[k * plane_sz + cidx].w - inv_lo) * scale);
      return b < 0 ? 0 : (b >= kDepthBuckets ? kDepthBuckets - 1 : b);
    };
    for (unsigned m = live; m; m &= m - 1) atomicAdd(&bucket[bucket_of(__ffs(m) - 1)], 1);
    __syncthreads();
    {
      const int c0 = bucket[threadIdx.x];
      int inc = c0;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
      }
      if (lane == 63) wave_total[wave] = inc;  // the list's scan above has read its totals
      __syncthreads();
      int excl = inc - c0;
      for (int w = 0; w < wave; ++w) excl += wave_total[w];
      bucket[threadIdx.x] = excl;
    }
    __syncthreads();
    for (unsigned m = live; m; m &= m - 1) {
      const int k = __ffs(m) - 1;
      item_lds[atomicAdd(&bucket[bucket_of(k)], 1)] = (uint16_t)((threadIdx.x << 3) | k);
    }
  }
  if (L.count && threadIdx.x == 0) atomicAdd(L.count, (unsigned long long)n_items);
  __syncthreads();
  for (int base = wave * 64; base < n_items; base += kBlock) {
    const int i = base + lane;
    if (i < n_items) {
      const int item = item_lds[i];
      const int p = item >> 3, k = item & 7;
      const int prow = p / TC, pcol = p - prow * TC;
      const int py = tile_y * TR + prow;
      const int pci = tile_x * TC + pcol;
      const int ppar = (py + colour) & 1;
      const int px = 2 * pci + ppar;
      RefPix q;
      q.x = px;
      q.y = py;
      q.X0 = (float)px;
      q.Y0 = (float)py;
      q.tbase = (prow + r - A.s * A.R) * TW + 2 * pcol + ppar + r - A.s * A.R;
      q.tox = x_org;
      q.toy = y_org;
      ray_f(A, px, py, q.rx, q.ry, q.rz);
      q.a_c = tile_lds[(prow + r) * TW + 2 * pcol + ppar + r];
      const float sw = ref_lds[p];
      q.ok = sw > 0.0f;
      q.S_w = q.ok ? sw : 1.0f;
      q.mu_a = ref_lds[kBlock + p];
      q.var_a = ref_lds[2 * kBlock + p];
      const float4 h = ld4(J.cand, k * plane_sz + (size_t)py * A.Wc + pci);
      cost_lds[k * kBlock + p] =
          plane_cost<FR>(A, q, tile_lds, TW, wcol, wsp, h.x, h.y, h.z, h.w, nullptr, nullptr);
    }
  }
  __syncthreads();
  if (L.mode == 3) {
    // the cost of every slot, written out row-major (slot k of pixel (x, y) at k H W + y W +
    // x); an empty slot, or a pixel whose window leaves the image, costs C_max
    if (in_img) {
      const size_t n = (size_t)A.W * A.H, p = (size_t)y * A.W + x;
      for (int k = 0; k < L.ncand; ++k)
        gl(J.cost_out)[k * n + p] = ((live >> k) & 1u) ? cost_lds[k * kBlock + threadIdx.x] : kCmax;
    }
    return;
  }
  if (!in_img || (L.mode == 1 && !valid)) return;
  float4 best = make_float4(0.f, 0.f, 0.f, 0.f);
  float bc = kCmax;
  if (L.mode == 1) {
    best = ld4(A.plane[colour], cidx);
    bc = gl(A.cost[colour])[cidx];
  }
  int pick = -1;
  for (int k = 0; k < L.ncand; ++k) {
    if (!((live >> k) & 1u)) continue;
    const float c = cost_lds[k * kBlock + threadIdx.x];
    const bool take = L.mode == 0 ? (k == 0 || c <= bc) : (c < bc);
    if (take) {
      bc = c;
      pick = k;
    }
  }
  if (pick >= 0) best = ld4(J.cand, pick * plane_sz + cidx);
  if (!valid) {
    best = make_float4(0.f, 0.f, 0.f, 0.f);
    bc = kCmax;
  }
  st4(A.plane[colour], cidx, best);
  gl(A.cost[colour])[cidx] = bc;
}

// Each XCD has its own list of tiles: the k-th of 8 contiguous bands of every job, so each
// XCD's L2 serves a compact band of each image and every XCD gets the same share of every
// job.  Non-persistent: workgroup b runs on XCD b % 8 and takes position b / 8 of that
// XCD's list.  Persistent: a fixed grid; each workgroup pulls positions from its XCD's
// queue, so uneven tiles balance dynamically within an XCD.  FR: instantiated with the
// window-resize scheme's code (launches holding such a job), whose register needs then do
// not weigh on the integer-spacing instance; DEPTH likewise for the depth-ordered work
// list, so that the pixel-order instance carries none of its code.
template <bool FR, bool DEPTH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void eval_kernel(
    const Job* __restrict__ jobs, Launch L) {
  // the colour-weight table at the start of LDS: a reference difference (x4) is then its
  // entry's address
  __shared__ float wcol[256];
  extern __shared__ float lds[];
  __shared__ int next_tile;
  const int xcd = blockIdx.x & 7;
  const int len = L.xcd_len[xcd];
  if (!L.persistent) {
    const int i = (int)(blockIdx.x >> 3);
    if (i >= len) return;
    const Job& J = jobs[job_of_xcd_tile(jobs, L.n_jobs, xcd, i)];
    int tx, ty;
    band_tile(J, xcd, i - J.xoff[xcd], tx, ty);
    eval_tile<FR, DEPTH>(J, L, tx, ty, wcol, lds);
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) next_tile = (int)atomicAdd(&L.queue[xcd], 1u);
    __syncthreads();
    const int i = next_tile;
    __syncthreads();
    if (i >= len) return;
    const Job& J = jobs[job_of_xcd_tile(jobs, L.n_jobs, xcd, i)];
    int tx, ty;
    band_tile(J, xcd, i - J.xoff[xcd], tx, ty);
    eval_tile<FR, DEPTH>(J, L, tx, ty, wcol, lds);
    __syncthreads();  // the next tile re-stages LDS
  }
}

// Small references, whose pixels alone do not fill the GPU: LANES lanes share each pixel,
// its tap sums split as in tap_pass_lanes.  A workgroup covers 256 / LANES compacted pixels
// of one row of one colour of job 0 (single-job launches); every lane of a pixel's group
// scores the same hypotheses and reaches the same costs, and the group's first lane
// writes.  Modes as in eval_tile; the reference-side sums stay sequential per pixel.
template <int LANES>
__global__ __launch_bounds__(kBlock) void eval_lanes_kernel(const Job* __restrict__ jobs, Launch L) {
  __shared__ float wcol[256];
  extern __shared__ float lds[];
  const Job& J = jobs[0];
  const Args& A = J.A;
  constexpr int P = kBlock / LANES;
  const int tiles_x = (A.Wc + P - 1) / P;
  const int tile_y = (int)blockIdx.x / tiles_x, tile_x = (int)blockIdx.x - tile_y * tiles_x;
  const int r = A.halo;
  const int TW = 2 * P + 2 * r, TH = 1 + 2 * r;
  float* wsp = lds;
  float* tile_lds = wsp + A.n_taps;
  const int x_org = tile_x * 2 * P - r, y_org = tile_y - r;
  for (int i = threadIdx.x; i < 256; i += kBlock) wcol[i] = gl(A.wcol)[i];
  for (int i = threadIdx.x; i < A.n_taps; i += kBlock) wsp[i] = gl(A.wsp)[i];
  for (int i = threadIdx.x; i < TW * TH; i += kBlock) {
    const int ty = i / TW, tx = i - ty * TW;
    const int gx = min(max(x_org + tx, 0), A.W - 1);
    const int gy = min(max(y_org + ty, 0), A.H - 1);
    const unsigned short hb = gl(reinterpret_cast<const unsigned short*>(A.ref))[(size_t)gy * A.W + gx];
    tile_lds[i] = 4.0f * __half2float(__ushort_as_half(hb));  // 4x the grey value, exact
  }
  __syncthreads();

  const int slot = (int)threadIdx.x / LANES, g = (int)threadIdx.x % LANES;
  const int lane = threadIdx.x & 63;
  const int colour = L.colour;
  const int y = tile_y;
  const int ci = tile_x * P + slot;
  const int par = (y + colour) & 1;
  const int x = 2 * ci + par;
  const bool in_img = y < A.H && ci < A.Wc && x < A.W;
  const bool valid = in_img && pixel_valid(A, x, y);
  RefPix rp;
  rp.x = x;
  rp.y = y;
  rp.X0 = (float)x;
  rp.Y0 = (float)y;
  rp.ok = false;
  rp.tbase = (r - A.s * A.R) * TW + 2 * slot + par + r - A.s * A.R;  // first tap (-R, -R)
  rp.tox = x_org;
  rp.toy = y_org;
  ray_f(A, x, y, rp.rx, rp.ry, rp.rz);
  rp.a_c = 0.0f;
  rp.S_w = 1.0f;
  rp.mu_a = 0.0f;
  rp.var_a = 0.0f;
  if (valid) {
    rp.a_c = tile_lds[r * TW + 2 * slot + par + r];
    float S_w = 0.0f, S_a4 = 0.0f, S_aa16 = 0.0f;
    int t = 0;
    for (int k2 = 0; k2 <= 2 * A.R; ++k2) {
      const float* trow = tile_lds + rp.tbase + k2 * A.s * TW;
      for (int k1 = 0; k1 <= 2 * A.R; ++k1, ++t) {
        const float a4 = trow[k1 * A.s] - rp.a_c;
        const float w = colour_weight<false>(wcol, a4) * wsp[t];
        const float wa4 = w * a4;
        S_w = S_w + w;
        S_a4 = S_a4 + wa4;
        S_aa16 = __builtin_fmaf(wa4, a4, S_aa16);
      }
    }
    rp.S_w = S_w;
    rp.mu_a = (S_a4 * 0.25f) / S_w;
    rp.var_a = (S_aa16 * 0.0625f) / S_w - rp.mu_a * rp.mu_a;
    rp.ok = rp.var_a >= A.eps_v;
  }
  const bool writer = g == 0;

  if (L.mode == 2) {
    if (in_img) {
      const size_t p = (size_t)y * A.W + x;
      float c = kCmax;
      float* pv = J.per_view_out && writer ? J.per_view_out + p * A.n_src : nullptr;
      uint8_t* vm = J.valid_out && writer ? J.valid_out + p * A.n_src : nullptr;
      float4 pl = make_float4(0.f, 0.f, 0.f, 0.f);
      if (valid) pl = ld4(reinterpret_cast<const float4*>(J.planes_in), p);
      const bool score = valid && !__builtin_isnan(pl.w);
      const unsigned long long bal = __ballot(score && writer);
      if (L.count && lane == 0) atomicAdd(L.count, (unsigned long long)__popcll(bal));
      if (score) {
        c = plane_cost<false, LANES>(A, rp, tile_lds, TW, wcol, wsp, pl.x, pl.y, pl.z, pl.w, pv, vm);
      } else {
        for (int j = 0; j < A.n_src; ++j) {
          if (pv) gl(pv)[j] = kCmax;
          if (vm) gl(vm)[j] = 0;
        }
      }
      if (writer) gl(J.cost_out)[p] = c;
    }
    return;
  }

  const size_t cidx = (size_t)y * A.Wc + ci;
  const size_t plane_sz = (size_t)A.H * A.Wc;
  float4 best = make_float4(0.f, 0.f, 0.f, 0.f);
  float bc = kCmax;
  if (L.mode == 1 && valid) {
    best = ld4(A.plane[colour], cidx);
    bc = gl(A.cost[colour])[cidx];
  }
  for (int k = 0; k < L.ncand; ++k) {
    float4 h = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    if (valid) h = ld4(J.cand, k * plane_sz + cidx);
    const bool has = valid && !__builtin_isnan(h.w);
    if (__ballot(has) == 0) continue;
    // the ballot over the whole wave, before only its first lane goes on to count
    const unsigned long long scored = __ballot(has && writer);
    if (L.count && lane == 0) atomicAdd(L.count, (unsigned long long)__popcll(scored));
    if (has) {
      const float c = plane_cost<false, LANES>(A, rp, tile_lds, TW, wcol, wsp, h.x, h.y, h.z, h.w, nullptr, nullptr);
      const bool take = L.mode == 0 ? (k == 0 || c <= bc) : (c < bc);
      if (take) {
        bc = c;
        best = h;
      }
    }
  }
  if (!in_img || (L.mode == 1 && !valid) || !writer) return;
  if (!valid) {
    best = make_float4(0.f, 0.f, 0.f, 0.f);
    bc = kCmax;
  }
  st4(A.plane[colour], cidx, best);
  gl(A.cost[colour])[cidx] = bc;
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

// colour planes -> row-major outputs (planes and cost, or depth / normal / cost); blocks of
// 256 pixels of one row (cblk_x counts 128-wide compacted blocks = 256-wide pixel blocks)
// the depth hypotheses of plane hypothesis inference as candidate planes of the fronto-
// parallel kind (0, 0, -1, h) for the pixels of one colour: slot k from hypothesis map k
// (planar, k H W + y W + x); a missing hypothesis (h <= 0) is an empty slot
__global__ __launch_bounds__(128) void cand_hyp_kernel(const Job* __restrict__ jobs, Launch L,
                                                       const float* __restrict__ hyp) {
  int jb, x, y, ci;
  if (!cblk_pixel(jobs, L, jb, x, y, ci)) return;
  const Job& J = jobs[jb];
  const Args& A = J.A;
  const size_t cidx = (size_t)y * A.Wc + ci, plane_sz = (size_t)A.H * A.Wc, n = (size_t)A.W * A.H;
  for (int k = 0; k < L.ncand; ++k) {
    const float h = gl(hyp)[k * n + (size_t)y * A.W + x];
    st4(J.cand, k * plane_sz + cidx, make_float4(0.0f, 0.0f, -1.0f, h > 0.0f ? h : __int_as_float(0x7fc00000)));
  }
}

__global__ __launch_bounds__(256) void unpack_kernel(const Job* __restrict__ jobs, Launch L) {
  const int g = blockIdx.x;
  const int jb = job_of_cblk(jobs, L.n_jobs, g);
  const Job& J = jobs[jb];
  const Args& A = J.A;
  const int local = g - J.cblk0;
  const int y = local / J.cblk_x;
  const int x = (local - y * J.cblk_x) * 256 + (int)threadIdx.x;
  if (x >= A.W || y >= A.H) return;
  const int colour = (x + y) & 1;
  const size_t ci = (size_t)y * A.Wc + (x >> 1);
  const float4 pl = A.plane[colour][ci];
  const float c = A.cost[colour][ci];
  const size_t p = (size_t)y * A.W + x;
  if (J.planes_out) reinterpret_cast<float4*>(J.planes_out)[p] = pl;
  if (J.depth_out) J.depth_out[p] = pl.w;
  if (J.normal_out) {
    J.normal_out[3 * p + 0] = pl.x;
    J.normal_out[3 * p + 1] = pl.y;
    J.normal_out[3 * p + 2] = pl.z;
  }
  if (J.final_cost_out) J.final_cost_out[p] = c;
}

// row-major planes + cost -> the colour planes of job 0
__global__ __launch_bounds__(256) void pack_kernel(const Job* __restrict__ jobs, const float* __restrict__ planes,
                                                   const float* __restrict__ cost) {
  const Args& A = jobs[0].A;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.W || y >= A.H) return;
  const int colour = (x + y) & 1;
  const size_t ci = (size_t)y * A.Wc + (x >> 1);
  const size_t p = (size_t)y * A.W + x;
  A.plane[colour][ci] = reinterpret_cast<const float4*>(planes)[p];
  A.cost[colour][ci] = cost[p];
}

__global__ void zero_kernel(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
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

size_t eval_lds_bytes(int tile_rows, int max_radius_px, int max_taps) {
  const int TC = kBlock / tile_rows;
  const size_t tw = 2 * TC + 2 * max_radius_px, th = tile_rows + 2 * max_radius_px;
  // the colour-weight table is static
  return sizeof(float) * ((size_t)kCompactLds + (size_t)max_taps + tw * th);
}

hipError_t eval_lds_setup(size_t* max_dynamic) {
  // Tiles above 64 KiB of LDS (one-row tiles with wide windows) need the opt-in limit.  It
  // is raised here, once per device and context, for both kernel instances, to what a
  // workgroup may hold beside the instance's static LDS (the colour-weight table and the
  // queue slot): never in the middle of a stream capture, where the launches are recorded.
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int optin = 0, per_cu = 0;
  if ((e = hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev)) != hipSuccess)
    return e;
  const size_t per_wg = std::min<size_t>((size_t)std::max(optin, per_cu), 160 * 1024);
  size_t lim = per_wg;
  const void* fns[8] = {(const void*)pmk::eval_kernel<false, false>, (const void*)pmk::eval_kernel<true, false>,
                        (const void*)pmk::eval_kernel<false, true>,  (const void*)pmk::eval_kernel<true, true>,
                        (const void*)pmk::eval_lanes_kernel<2>,      (const void*)pmk::eval_lanes_kernel<4>,
                        (const void*)pmk::eval_lanes_kernel<8>,      (const void*)pmk::eval_lanes_kernel<16>};
  for (const void* fn : fns) {
    hipFuncAttributes a{};
    if ((e = hipFuncGetAttributes(&a, fn)) != hipSuccess) return e;
    if (a.sharedSizeBytes >= per_wg) return hipErrorInvalidValue;
    const size_t dyn = per_wg - a.sharedSizeBytes;
    if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn)) != hipSuccess) return e;
    lim = std::min(lim, dyn);
  }
  *max_dynamic = lim;
  return hipSuccess;
}

hipError_t launch_eval(const Job* d_jobs, const Launch& L, int grid, size_t lds, hipStream_t st) {
  // hipLaunchKernel returns this launch's own status (hipGetLastError would also report an
  // earlier call's error on this thread)
  Launch l = L;
  void* args[] = {(void*)&d_jobs, (void*)&l};
  const void* fn = L.order_by_depth
                       ? (L.frac ? (const void*)pmk::eval_kernel<true, true> : (const void*)pmk::eval_kernel<false, true>)
                       : (L.frac ? (const void*)pmk::eval_kernel<true, false> : (const void*)pmk::eval_kernel<false, false>);
  return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, lds, st);
}

size_t eval_lanes_lds_bytes(int lanes, int radius_px, int n_taps) {
  const int P = kBlock / lanes;
  return sizeof(float) * ((size_t)n_taps + (size_t)(2 * P + 2 * radius_px) * (size_t)(1 + 2 * radius_px));
}

hipError_t launch_eval_lanes(const Job* d_jobs, const Launch& L, int lanes, int H, int Wc, size_t lds,
                             hipStream_t st) {
  const int P = kBlock / lanes;
  const long long grid = (long long)H * ((Wc + P - 1) / P);
  if (grid < 1 || grid > 0x7fffffff) return hipErrorInvalidValue;
  Launch l = L;
  void* args[] = {(void*)&d_jobs, (void*)&l};
  const void* fn = lanes == 2 ? (const void*)pmk::eval_lanes_kernel<2>
                   : lanes == 4 ? (const void*)pmk::eval_lanes_kernel<4>
                   : lanes == 8 ? (const void*)pmk::eval_lanes_kernel<8>
                   : lanes == 16 ? (const void*)pmk::eval_lanes_kernel<16>
                                 : nullptr;
  if (!fn) return hipErrorInvalidValue;
  return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kBlock), args, lds, st);
}

hipError_t launch_candidates(int kind, const Job* d_jobs, const Launch& L, hipStream_t st) {
  const dim3 grid(L.total_cblk);
  if (kind == 0) hipLaunchKernelGGL(pmk::cand_init_kernel, grid, dim3(128), 0, st, d_jobs, L);
  else if (kind == 1) hipLaunchKernelGGL(pmk::cand_prop_kernel, grid, dim3(128), 0, st, d_jobs, L);
  else hipLaunchKernelGGL(pmk::cand_refine_kernel, grid, dim3(128), 0, st, d_jobs, L);
  return hipGetLastError();
}

hipError_t launch_hyp_candidates(const Job* d_jobs, const Launch& L, const float* hyp, hipStream_t st) {
  hipLaunchKernelGGL(pmk::cand_hyp_kernel, dim3(L.total_cblk), dim3(128), 0, st, d_jobs, L, hyp);
  return hipGetLastError();
}

hipError_t launch_unpack(const Job* d_jobs, const Launch& L, hipStream_t st) {
  hipLaunchKernelGGL(pmk::unpack_kernel, dim3(L.total_cblk), dim3(256), 0, st, d_jobs, L);
  return hipGetLastError();
}

hipError_t launch_pack(const Job* d_jobs, int W, int H, const float* planes, const float* cost, hipStream_t st) {
  hipLaunchKernelGGL(pmk::pack_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, d_jobs, planes, cost);
  return hipGetLastError();
}

hipError_t launch_zero(unsigned int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(pmk::zero_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_build_view(const uint8_t* img, int64_t stride, int W, int H, __half* plain, uint32_t* quad,
                             hipStream_t st) {
  hipLaunchKernelGGL(pmk::build_view_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, img, stride, W, H, plain, quad);
  return hipGetLastError();
}

hipError_t launch_rcp_check(uint32_t first, uint32_t count, unsigned long long* mism, uint32_t* example,
                            hipStream_t st) {
  hipLaunchKernelGGL(pmk::rcp_check_kernel, dim3((count + 255) / 256), dim3(256), 0, st, first, count, mism, example);
  return hipGetLastError();
}

}  // namespace phimvs_internal
