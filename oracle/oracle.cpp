// PatchMatch multi-view stereo oracle — TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU statement of what the PHI-MVS depth-map
// estimation step computes (paper Sec. III-B random initialisation, Sec. III-C
// depth map estimation with Eq. 4 and Eq. 5, Algorithm 1 "depth map estimation").
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may load it;
// the GPU library never does, and the two share no code.
//
// Every function is written for one pixel / one hypothesis / one view at a time in
// the order the paper states the method; there is no blocking, fusion or
// reordering.  The arithmetic type T is float ("FP32 canonical": every rounding
// step written out, fma only where written) or double (FP64, used to state the
// error of the FP32 results).  Points the paper leaves open follow these readings:
//
//  * Cost (Eq. 4): weighted ZNCC over the dilated window; weight 1 everywhere
//    reproduces Eq. 4 exactly; bilateral weights come from the reference patch
//    only: w = exp(-(a-a_c)^2 / (2 sc^2)) * exp(-s^2 (k1^2 + k2^2) / (2 ss^2)), each
//    factor evaluated in FP64 and, in FP32 mode, rounded to float.
//  * Sums are shifted by the centre samples (a - a_c, b - b_c) before squaring; NCC
//    is shift invariant, so this changes nothing but cancellation.
//  * Border rule: a view is invalid when any warped tap leaves
//    [0, W-1] x [0, H-1] or lies behind the source camera (w <= 0).  It is tested at
//    the four window corners: for w > 0 the plane-induced homography maps the window
//    rectangle onto the convex quadrilateral spanned by the corner images, so the
//    corner test is exactly the all-taps test.  Every tap's sample position is then
//    clamped into the image (a no-op in exact arithmetic) before bilinear sampling.
//  * C_max = 1 - Z_min with Z_min = -1, so C_max = 2; omega in Eq. 5 is 1; a view's
//    validity is an explicit flag instead of a float comparison with C_max; the
//    inverse cost weight uses max(C_j, eps_c); a view with weighted variance below
//    eps_v (either patch) is invalid; Eq. 5 is taken over the K lowest-cost valid
//    views (K = 0: all valid views, which is the paper's Eq. 5), summed in ascending
//    (cost, view) order.
//  * Depth is reference-camera Z; normals live in the reference camera frame and
//    face the camera (n . r_p < 0); initial normals are drawn as in Sec. III-B and
//    flipped to face the camera.
//  * Random refinement (Sec. III-C, last paragraph): Delta_d in [-d_hi/4, d_hi/4],
//    Delta_theta in [-pi/2, pi/2], Delta_phi in [-pi/12, pi/12] applied to
//    (theta, phi) = (atan2(n_y, n_x), acos(n_z)); candidates (d_new, n_old),
//    (d_old, n_new), (d_new, n_new) in that order, strict improvement, first listed
//    wins ties; an out-of-range d_new drops the two candidates that use it.  The
//    normals are formed in FP64 (then rounded to float in FP32 mode).
//  * Red/black propagation (Sec. III intro): each pixel of one colour looks at 8
//    regions of the other colour (4 near "V" regions of 9 offsets, 4 far strips of
//    10 offsets), takes the lowest-cost pixel of each region, re-expresses its plane
//    at the pixel by ray-plane intersection, and keeps the best candidate if it
//    strictly lowers the cost.  Refinement of a colour follows its propagation; one
//    iteration is red then black.
//  * Summation order: a view's source-side sums (S_b, S_bb, S_ab) run over the taps in
//    row-major order; with lanes = G > 1 they are formed as G lanes sharing the view form
//    them (lane g sums the taps t = g mod G in order, then an xor butterfly over offsets
//    G/2 .. 1), the order of the GPU's split sums.  The reference-side sums stay sequential.
//  * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = seed and counter
//    = (pixel index y*W + x, iteration, phase, 0); uniforms (x >> 8) * 2^-24.
//  * Pixels whose reference window leaves the image are invalid: never updated,
//    output depth 0, normal 0, cost C_max.
//
// Threads.  The same source is also built with OpenMP (liboracle_omp.so): the loops over
// the pixels of one colour within a half-sweep (and over the pixels of an initialisation
// or a cost evaluation) are then shared among threads.  Within a half-sweep a pixel reads
// only the other colour's state and its own, the random numbers are keyed by pixel, and
// each pixel's arithmetic is unchanged, so the results are bitwise those of one thread.
// Without OpenMP the pragmas are ignored and the build is the single-threaded one.

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;
const int kPhaseInit = 0;
const int kPhaseRefine = 1;

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11.
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// uniform in [0, 1) with 24 random bits (exact in float)
double unit24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

// ---------------------------------------------------------------- small FP64 linear algebra
void mat3_mul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}

void mat3_transpose(const double* A, double* T) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[i * 3 + j] = A[j * 3 + i];
}

void mat3_vec(const double* A, const double* v, double* o) {
  for (int i = 0; i < 3; ++i) o[i] = A[i * 3 + 0] * v[0] + A[i * 3 + 1] * v[1] + A[i * 3 + 2] * v[2];
}

// inverse by the adjugate; returns false when singular
bool mat3_inverse(const double* A, double* inv) {
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  double id = 1.0 / det;
  inv[0] = c00 * id;
  inv[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  inv[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  inv[3] = c01 * id;
  inv[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  inv[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  inv[6] = c02 * id;
  inv[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  inv[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  return true;
}

}  // namespace

extern "C" {

// The problem as plain arrays.  View 0 is the reference, views 1..n_views-1 the
// sources.  Cameras map world to camera: X_cam = R X_world + t; K has last row
// (0, 0, 1).  Images are grey values (0..255 for 8-bit input), row-major H x W.
typedef struct {
  int32_t n_views;
  const int32_t* width;
  const int32_t* height;
  const float* const* images;
  const double* K;  // n_views * 9
  const double* R;  // n_views * 9
  const double* t;  // n_views * 3
  double d_lo, d_hi;
  int32_t window, dilation, top_k, bilateral;
  double sigma_s, sigma_c, eps_v, eps_c;
  uint64_t seed;
  int32_t tap_radius;  // > 0: the window-resize scheme, r_now = tap_radius taps per side
  int32_t lanes;       // > 1 (a power of two): the source-side tap sums as G lanes form them
} oracle_problem;

}  // extern "C"

namespace {

template <typename T>
T fmaT(T a, T b, T c) { return std::fma(a, b, c); }

template <typename T>
struct V3 { T x, y, z; };

// Eq. 5 over the K lowest-cost valid views (K <= 0: all valid views):
// C = n_sel / sum_sel 1 / max(C_j, eps_c), summed in ascending (C_j, j) order; C_max when none is valid.
template <typename T>
T aggregate(const T* cj, const int* ok, int n, int top_k, T eps_c) {
  std::vector<int> order;
  for (int j = 0; j < n; ++j)
    if (ok[j]) order.push_back(j);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return cj[a] < cj[b] || (cj[a] == cj[b] && a < b); });
  int k = top_k > 0 ? std::min<int>(top_k, (int)order.size()) : (int)order.size();
  if (k == 0) return T(2);
  T sum = T(0);
  for (int i = 0; i < k; ++i) sum = sum + T(1) / std::fmax(cj[order[i]], eps_c);
  return (T)k / sum;
}

template <typename T>
T dot3(const V3<T>& a, const V3<T>& b) { return fmaT(a.x, b.x, fmaT(a.y, b.y, a.z * b.z)); }

template <typename T>
T lerp(T a, T b, T t) { return fmaT(t, b - a, a); }

// The solver's view of the problem in arithmetic type T.
template <typename T>
struct Solver {
  const oracle_problem* pb;
  int W, H, n_src, R_now, s;
  // window-resize scheme (Sec. III-C, Fig. 4, Table III): r_now taps per side spread over
  // the original radius r_orig, spacing s = r_orig / r_now (not necessarily an integer);
  // tap k sits at offset off[k] = s k (rounded to T), reference values are interpolated
  bool frac = false;
  int r_orig = 0;
  double sf_d = 0.0;
  std::vector<T> off;  // 2 R_now + 1 offsets, k = -R_now .. R_now
  double Kinv_d[9];     // reference K^-1 in FP64
  T Kinv[9];            // ... rounded to T
  std::vector<T> M;     // n_src * 9: K_j R_rel K_0^-1
  std::vector<T> e;     // n_src * 3: K_j t_rel
  T d_lo, d_hi, eps_v, eps_c;
  static constexpr double kCmax = 2.0;

  bool setup(const oracle_problem* p) {
    pb = p;
    if (p->lanes > 1 && (p->lanes & (p->lanes - 1))) return false;  // G must be a power of two
    W = p->width[0];
    H = p->height[0];
    n_src = p->n_views - 1;
    s = p->dilation;
    R_now = (p->window - 1) / (2 * p->dilation);
    frac = p->tap_radius > 0;
    if (frac) {
      r_orig = (p->window - 1) / 2;
      R_now = p->tap_radius;
      s = 1;
      sf_d = (double)r_orig / (double)R_now;
    }
    off.resize(2 * R_now + 1);
    for (int k = -R_now; k <= R_now; ++k) off[k + R_now] = frac ? (T)sf_d * (T)k : (T)(s * k);
    if (!mat3_inverse(p->K, Kinv_d)) return false;
    for (int i = 0; i < 9; ++i) Kinv[i] = (T)Kinv_d[i];
    M.assign(9 * n_src, T(0));
    e.assign(3 * n_src, T(0));
    double R0t[9];
    mat3_transpose(p->R, R0t);
    for (int j = 0; j < n_src; ++j) {
      const double* Kj = p->K + 9 * (j + 1);
      const double* Rj = p->R + 9 * (j + 1);
      const double* tj = p->t + 3 * (j + 1);
      double Rrel[9], Rt0[3], trel[3], KR[9], Mj[9], ej[3];
      mat3_mul(Rj, R0t, Rrel);              // R_rel = R_j R_0^T
      mat3_vec(Rrel, p->t, Rt0);            // R_rel t_0
      for (int i = 0; i < 3; ++i) trel[i] = tj[i] - Rt0[i];  // t_rel = t_j - R_rel t_0
      mat3_mul(Kj, Rrel, KR);
      mat3_mul(KR, Kinv_d, Mj);             // M_j = (K_j R_rel) K_0^-1
      mat3_vec(Kj, trel, ej);               // e_j = K_j t_rel
      for (int i = 0; i < 9; ++i) M[9 * j + i] = (T)Mj[i];
      for (int i = 0; i < 3; ++i) e[3 * j + i] = (T)ej[i];
    }
    d_lo = (T)p->d_lo;
    d_hi = (T)p->d_hi;
    eps_v = (T)p->eps_v;
    eps_c = (T)p->eps_c;
    return true;
  }

  bool pixel_valid(int x, int y) const {
    int r = frac ? r_orig : s * R_now;
    return x - r >= 0 && x + r <= W - 1 && y - r >= 0 && y + r <= H - 1;
  }

  // reference value of tap (k1, k2) (indices -R_now .. R_now) of pixel (x, y): a texel,
  // or in the window-resize scheme the bilinear value at (x + off[k1], y + off[k2])
  T ref_tap(int x, int y, int k1, int k2) const {
    if (!frac) return ref(x + s * k1, y + s * k2);
    return sample(0, (T)x + off[k1 + R_now], (T)y + off[k2 + R_now]);
  }

  T ref(int x, int y) const { return (T)pb->images[0][(size_t)y * W + x]; }

  // viewing ray of reference pixel (x, y): K_0^-1 (x, y, 1)
  V3<T> ray(int x, int y) const {
    T X = (T)x, Y = (T)y;
    return {fmaT(Kinv[0], X, fmaT(Kinv[1], Y, Kinv[2])),
            fmaT(Kinv[3], X, fmaT(Kinv[4], Y, Kinv[5])),
            fmaT(Kinv[6], X, fmaT(Kinv[7], Y, Kinv[8]))};
  }

  // the same ray in FP64 (used to orient drawn normals)
  void ray_d(int x, int y, double* r) const {
    double X = x, Y = y;
    r[0] = std::fma(Kinv_d[0], X, std::fma(Kinv_d[1], Y, Kinv_d[2]));
    r[1] = std::fma(Kinv_d[3], X, std::fma(Kinv_d[4], Y, Kinv_d[5]));
    r[2] = std::fma(Kinv_d[6], X, std::fma(Kinv_d[7], Y, Kinv_d[8]));
  }

  // bilateral weight factors
  T w_colour(T da) const {
    if (!pb->bilateral) return T(1);
    // an interpolated reference difference is taken at the nearest integer grey level
    double d = frac ? (double)std::nearbyint(std::fabs(da)) : (double)da;
    return (T)std::exp(-(d * d) / (2.0 * pb->sigma_c * pb->sigma_c));
  }
  T w_space(int k1, int k2) const {
    if (!pb->bilateral) return T(1);
    double r2 = (frac ? sf_d * sf_d : (double)(s * s)) * (double)(k1 * k1 + k2 * k2);
    return (T)std::exp(-r2 / (2.0 * pb->sigma_s * pb->sigma_s));
  }

  // bilinear sample of source view v (1-based view index) at (u, v), position clamped into the image
  T sample(int view, T u, T v) const {
    int Wj = pb->width[view], Hj = pb->height[view];
    const float* img = pb->images[view];
    u = std::fmin(std::fmax(u, T(0)), (T)(Wj - 1));
    v = std::fmin(std::fmax(v, T(0)), (T)(Hj - 1));
    T fx0 = std::floor(u), fy0 = std::floor(v);
    T fx = u - fx0, fy = v - fy0;
    int x0 = (int)fx0, y0 = (int)fy0;
    int x1 = std::min(x0 + 1, Wj - 1), y1 = std::min(y0 + 1, Hj - 1);
    T i00 = (T)img[(size_t)y0 * Wj + x0], i01 = (T)img[(size_t)y0 * Wj + x1];
    T i10 = (T)img[(size_t)y1 * Wj + x0], i11 = (T)img[(size_t)y1 * Wj + x1];
    T top = lerp(i00, i01, fx);
    T bot = lerp(i10, i11, fx);
    return lerp(top, bot, fy);
  }

  // homography of source j (0-based) induced by the plane (n, d) seen at reference pixel p
  // H_j = M_j + e_j m^T with m = K_0^-T n / rho, rho = d (n . r_p)
  void homography(int j, const V3<T>& n, T rho, T* Hm) const {
    T kn[3];
    for (int c = 0; c < 3; ++c)
      kn[c] = fmaT(Kinv[0 * 3 + c], n.x, fmaT(Kinv[1 * 3 + c], n.y, Kinv[2 * 3 + c] * n.z));
    T m[3] = {kn[0] / rho, kn[1] / rho, kn[2] / rho};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Hm[r * 3 + c] = fmaT(e[3 * j + r], m[c], M[9 * j + r * 3 + c]);
  }

  // warp reference position (X, Y) with H: returns w (third coordinate) and the divided position
  T warp(const T* Hm, T X, T Y, T* up, T* vp) const {
    T u = fmaT(Hm[0], X, fmaT(Hm[1], Y, Hm[2]));
    T v = fmaT(Hm[3], X, fmaT(Hm[4], Y, Hm[5]));
    T w = fmaT(Hm[6], X, fmaT(Hm[7], Y, Hm[8]));
    T r = T(1) / w;
    *up = u * r;
    *vp = v * r;
    return w;
  }

  // Aggregated cost (Eq. 5 over the best-K valid views) of plane (n, d) at pixel (x, y).
  // per_view / valid (optional, length n_src) receive each source's C_j and flag.
  T cost(int x, int y, const V3<T>& n, T d, T* per_view, int32_t* valid_out) const {
    std::vector<T> cj(n_src, (T)kCmax);
    std::vector<int> ok(n_src, 0);
    auto finish = [&]() -> T {
      if (per_view)
        for (int j = 0; j < n_src; ++j) per_view[j] = cj[j];
      if (valid_out)
        for (int j = 0; j < n_src; ++j) valid_out[j] = ok[j];
      return aggregate<T>(cj.data(), ok.data(), n_src, pb->top_k, eps_c);
    };

    V3<T> rp = ray(x, y);
    T nr = dot3(n, rp);
    if (!(nr < T(0))) return finish();
    T rho = d * nr;

    // reference side of the window (independent of the plane and the view)
    const int R = R_now;
    const int taps = (2 * R + 1) * (2 * R + 1);
    std::vector<T> wk(taps), wak(taps);
    T a_c = ref(x, y);
    T S_w = 0, S_a = 0, S_aa = 0;
    for (int k2 = -R, t = 0; k2 <= R; ++k2)
      for (int k1 = -R; k1 <= R; ++k1, ++t) {
        T a = ref_tap(x, y, k1, k2) - a_c;
        T w = w_colour(a) * w_space(k1, k2);
        T wa = w * a;
        S_w = S_w + w;
        S_a = S_a + wa;
        S_aa = fmaT(wa, a, S_aa);
        wk[t] = w;
        wak[t] = wa;
      }
    T mu_a = S_a / S_w;
    T var_a = S_aa / S_w - mu_a * mu_a;
    if (!(var_a >= eps_v)) return finish();

    for (int j = 0; j < n_src; ++j) {
      const int view = j + 1;
      const T Wm1 = (T)(pb->width[view] - 1), Hm1 = (T)(pb->height[view] - 1);
      T Hm[9];
      homography(j, n, rho, Hm);
      // border rule at the four window corners
      bool inside = true;
      const int cx[4] = {-R, R, -R, R}, cy[4] = {-R, -R, R, R};
      for (int c = 0; c < 4; ++c) {
        T up, vp;
        T w = warp(Hm, (T)x + off[cx[c] + R], (T)y + off[cy[c] + R], &up, &vp);
        if (!(w > T(0)) || !(up >= T(0) && up <= Wm1 && vp >= T(0) && vp <= Hm1)) inside = false;
      }
      if (!inside) continue;
      T up, vp;
      warp(Hm, (T)x, (T)y, &up, &vp);
      T b_c = sample(view, up, vp);
      T S_b = 0, S_bb = 0, S_ab = 0;
      if (pb->lanes <= 1) {
        for (int k2 = -R, t = 0; k2 <= R; ++k2)
          for (int k1 = -R; k1 <= R; ++k1, ++t) {
            warp(Hm, (T)x + off[k1 + R], (T)y + off[k2 + R], &up, &vp);
            T b = sample(view, up, vp) - b_c;
            T tb = wk[t] * b;
            S_b = S_b + tb;
            S_bb = fmaT(tb, b, S_bb);
            S_ab = fmaT(wak[t], b, S_ab);
          }
      } else {
        // G lanes share the view: lane g sums the taps t = g, g + G, g + 2G, ... (row-major
        // tap index, in that order); then at each offset o = G/2, G/4, ..., 1 every lane adds
        // the partial sum of lane g xor o to its own, after which all lanes hold the total
        const int G = pb->lanes;
        std::vector<T> pb_(G, T(0)), pbb(G, T(0)), pab(G, T(0));
        for (int k2 = -R, t = 0; k2 <= R; ++k2)
          for (int k1 = -R; k1 <= R; ++k1, ++t) {
            warp(Hm, (T)x + off[k1 + R], (T)y + off[k2 + R], &up, &vp);
            T b = sample(view, up, vp) - b_c;
            T tb = wk[t] * b;
            const int g = t % G;
            pb_[g] = pb_[g] + tb;
            pbb[g] = fmaT(tb, b, pbb[g]);
            pab[g] = fmaT(wak[t], b, pab[g]);
          }
        for (int o = G / 2; o >= 1; o /= 2) {
          std::vector<T> nb(G), nbb(G), nab(G);
          for (int g = 0; g < G; ++g) {
            nb[g] = pb_[g] + pb_[g ^ o];
            nbb[g] = pbb[g] + pbb[g ^ o];
            nab[g] = pab[g] + pab[g ^ o];
          }
          pb_.swap(nb);
          pbb.swap(nbb);
          pab.swap(nab);
        }
        S_b = pb_[0];
        S_bb = pbb[0];
        S_ab = pab[0];
      }
      T mu_b = S_b / S_w;
      T var_b = S_bb / S_w - mu_b * mu_b;
      T cov = S_ab / S_w - mu_a * mu_b;
      if (!(var_b >= eps_v)) continue;
      T z = cov / std::sqrt(var_a * var_b);
      z = std::fmin(std::fmax(z, T(-1)), T(1));
      cj[j] = T(1) - z;
      ok[j] = 1;
    }
    return finish();
  }

  void draw(int x, int y, int iteration, int phase, T u[4]) const {
    uint32_t ctr[4] = {(uint32_t)((uint64_t)y * (uint64_t)W + (uint64_t)x), (uint32_t)iteration,
                       (uint32_t)phase, 0u};
    uint32_t key[2] = {(uint32_t)(pb->seed & 0xFFFFFFFFu), (uint32_t)(pb->seed >> 32)};
    uint32_t o[4];
    philox4x32_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = (T)unit24(o[i]);
  }

  // normal from spherical angles (FP64), turned to face the camera at pixel (x, y)
  V3<T> facing_normal(int x, int y, double theta, double phi) const {
    double n[3] = {std::cos(theta) * std::sin(phi), std::sin(theta) * std::sin(phi), std::cos(phi)};
    double r[3];
    ray_d(x, y, r);
    if (n[0] * r[0] + n[1] * r[1] + n[2] * r[2] > 0.0) {
      n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2];
    }
    return {(T)n[0], (T)n[1], (T)n[2]};
  }

  // Sec. III-B: d uniform in the depth range, theta in [0, 2 pi], phi in [-pi/2, pi/2]
  void init_pixel(int x, int y, T* plane, T* c) const {
    T u[4];
    draw(x, y, 0, kPhaseInit, u);
    T d = fmaT(u[0], d_hi - d_lo, d_lo);
    double theta = 2.0 * kPi * (double)u[1];
    double phi = kPi * ((double)u[2] - 0.5);
    V3<T> n = facing_normal(x, y, theta, phi);
    plane[0] = n.x; plane[1] = n.y; plane[2] = n.z; plane[3] = d;
    *c = cost(x, y, n, d, nullptr, nullptr);
  }

  // red/black propagation of pixel (x, y): reads the other colour's state
  void propagate_pixel(int x, int y, const T* planes, const T* costs, T* plane_out, T* c_out) const {
    static const int up_near[9][2] = {{0, -1}, {-1, -2}, {1, -2}, {0, -3}, {-2, -3}, {2, -3}, {-1, -4}, {1, -4}, {0, -5}};
    const size_t p = (size_t)y * W + x;
    V3<T> rp = ray(x, y);
    T best_c = costs[p];
    int best_g = -1;
    V3<T> best_n{0, 0, 0};
    T best_d = 0;
    for (int g = 0; g < 8; ++g) {
      const int dir = g & 3;  // up, down, left, right
      const bool far = g >= 4;
      const int count = far ? 10 : 9;
      int qx = -1, qy = -1;
      T qc = 0;
      for (int i = 0; i < count; ++i) {
        int dx = far ? 0 : up_near[i][0];
        int dy = far ? -(2 * (i + 3) + 1) : up_near[i][1];
        int ox, oy;
        if (dir == 0) { ox = dx; oy = dy; }
        else if (dir == 1) { ox = dx; oy = -dy; }
        else if (dir == 2) { ox = dy; oy = dx; }
        else { ox = -dy; oy = dx; }
        int xq = x + ox, yq = y + oy;
        if (xq < 0 || xq >= W || yq < 0 || yq >= H || !pixel_valid(xq, yq)) continue;
        T c = costs[(size_t)yq * W + xq];
        if (qx < 0 || c < qc) { qx = xq; qy = yq; qc = c; }
      }
      if (qx < 0) continue;
      const T* pq = planes + 4 * ((size_t)qy * W + qx);
      V3<T> nq{pq[0], pq[1], pq[2]};
      T dq = pq[3];
      V3<T> rq = ray(qx, qy);
      V3<T> Xq{dq * rq.x, dq * rq.y, dq * rq.z};
      T num = dot3(nq, Xq);
      T den = dot3(nq, rp);
      if (!(den < T(0))) continue;
      T dn = num / den;
      if (!(dn >= d_lo && dn <= d_hi)) continue;
      T c = cost(x, y, nq, dn, nullptr, nullptr);
      if (c < best_c) { best_c = c; best_g = g; best_n = nq; best_d = dn; }
    }
    const T* cur = planes + 4 * p;
    if (best_g >= 0) {
      plane_out[0] = best_n.x; plane_out[1] = best_n.y; plane_out[2] = best_n.z; plane_out[3] = best_d;
      *c_out = best_c;
    } else {
      for (int i = 0; i < 4; ++i) plane_out[i] = cur[i];
      *c_out = costs[p];
    }
  }

  // random refinement of pixel (x, y) at the given iteration
  void refine_pixel(int x, int y, int iteration, T* plane, T* c) const {
    T u[4];
    draw(x, y, iteration, kPhaseRefine, u);
    V3<T> n_old{plane[0], plane[1], plane[2]};
    T d_old = plane[3];
    T dd = (T(2) * u[0] - T(1)) * (d_hi * T(0.25));
    T d_new = d_old + dd;
    bool d_ok = d_new >= d_lo && d_new <= d_hi;
    double theta = std::atan2((double)n_old.y, (double)n_old.x);
    double nz = std::fmin(std::fmax((double)n_old.z, -1.0), 1.0);
    double phi = std::acos(nz);
    double dtheta = (2.0 * (double)u[1] - 1.0) * (kPi / 2.0);
    double dphi = (2.0 * (double)u[2] - 1.0) * (kPi / 12.0);
    V3<T> n_new = facing_normal(x, y, theta + dtheta, phi + dphi);
    T best = *c;
    int pick = -1;
    T c1 = d_ok ? cost(x, y, n_old, d_new, nullptr, nullptr) : (T)kCmax;
    if (d_ok && c1 < best) { best = c1; pick = 0; }
    T c2 = cost(x, y, n_new, d_old, nullptr, nullptr);
    if (c2 < best) { best = c2; pick = 1; }
    T c3 = d_ok ? cost(x, y, n_new, d_new, nullptr, nullptr) : (T)kCmax;
    if (d_ok && c3 < best) { best = c3; pick = 2; }
    if (pick == 0) { plane[3] = d_new; }
    else if (pick == 1) { plane[0] = n_new.x; plane[1] = n_new.y; plane[2] = n_new.z; }
    else if (pick == 2) { plane[0] = n_new.x; plane[1] = n_new.y; plane[2] = n_new.z; plane[3] = d_new; }
    *c = best;
  }
};

template <typename T>
void load_state(const double* planes, const double* costs, size_t n, std::vector<T>& P, std::vector<T>& C) {
  P.resize(4 * n);
  C.resize(n);
  for (size_t i = 0; i < 4 * n; ++i) P[i] = (T)planes[i];
  for (size_t i = 0; i < n; ++i) C[i] = (T)costs[i];
}

template <typename T>
void store_state(const std::vector<T>& P, const std::vector<T>& C, double* planes, double* costs) {
  for (size_t i = 0; i < P.size(); ++i) planes[i] = (double)P[i];
  for (size_t i = 0; i < C.size(); ++i) costs[i] = (double)C[i];
}

template <typename T>
int run_init(const oracle_problem* pb, double* planes, double* costs) {
  Solver<T> S;
  if (!S.setup(pb)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < S.H; ++y)
    for (int x = 0; x < S.W; ++x) {
      size_t p = (size_t)y * S.W + x;
      T pl[4] = {0, 0, 0, 0}, c = (T)Solver<T>::kCmax;
      if (S.pixel_valid(x, y)) S.init_pixel(x, y, pl, &c);
      for (int i = 0; i < 4; ++i) planes[4 * p + i] = (double)pl[i];
      costs[p] = (double)c;
    }
  return 0;
}

// one half-sweep of one colour: propagation then refinement, on all pixels of the colour
// (or on the listed ones only; updates within a colour are independent)
template <typename T>
int run_halfsweep(const oracle_problem* pb, int iteration, int colour, double* planes, double* costs,
                  const int32_t* subset, int n_subset, int do_prop, int do_refine) {
  Solver<T> S;
  if (!S.setup(pb)) return -1;
  const size_t n = (size_t)S.W * S.H;
  std::vector<T> P, C;
  load_state<T>(planes, costs, n, P, C);
  std::vector<T> Pn = P, Cn = C;
  auto visit = [&](int x, int y) {
    if (((x + y) & 1) != colour || !S.pixel_valid(x, y)) return;
    size_t p = (size_t)y * S.W + x;
    T pl[4], c;
    if (do_prop) S.propagate_pixel(x, y, P.data(), C.data(), pl, &c);
    else { for (int i = 0; i < 4; ++i) pl[i] = P[4 * p + i]; c = C[p]; }
    if (do_refine) S.refine_pixel(x, y, iteration, pl, &c);
    for (int i = 0; i < 4; ++i) Pn[4 * p + i] = pl[i];
    Cn[p] = c;
  };
  if (subset) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n_subset; ++i) visit(subset[i] % S.W, subset[i] / S.W);
  } else {
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < S.H; ++y)
      for (int x = 0; x < S.W; ++x) visit(x, y);
  }
  store_state<T>(Pn, Cn, planes, costs);
  return 0;
}

template <typename T>
int run_patchmatch(const oracle_problem* pb, int iters, float* depth, float* normal, float* cost_out) {
  Solver<T> S;
  if (!S.setup(pb)) return -1;
  const size_t n = (size_t)S.W * S.H;
  std::vector<T> P(4 * n, T(0)), C(n, (T)Solver<T>::kCmax);
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < S.H; ++y)
    for (int x = 0; x < S.W; ++x)
      if (S.pixel_valid(x, y)) S.init_pixel(x, y, &P[4 * ((size_t)y * S.W + x)], &C[(size_t)y * S.W + x]);
  for (int it = 1; it <= iters; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      // the other colour is read-only during this half-sweep, so in-place updates are exact
#pragma omp parallel for schedule(dynamic, 1)
      for (int y = 0; y < S.H; ++y)
        for (int x = 0; x < S.W; ++x) {
          if (((x + y) & 1) != colour || !S.pixel_valid(x, y)) continue;
          size_t p = (size_t)y * S.W + x;
          T pl[4], c;
          S.propagate_pixel(x, y, P.data(), C.data(), pl, &c);
          S.refine_pixel(x, y, it, pl, &c);
          for (int i = 0; i < 4; ++i) P[4 * p + i] = pl[i];
          C[p] = c;
        }
    }
  for (size_t p = 0; p < n; ++p) {
    int x = (int)(p % S.W), y = (int)(p / S.W);
    bool v = S.pixel_valid(x, y);
    depth[p] = v ? (float)P[4 * p + 3] : 0.0f;
    for (int i = 0; i < 3; ++i) normal[3 * p + i] = v ? (float)P[4 * p + i] : 0.0f;
    cost_out[p] = v ? (float)C[p] : (float)Solver<T>::kCmax;
  }
  return 0;
}

template <typename T>
int run_eval(const oracle_problem* pb, const double* planes, double* cost_out, double* per_view,
             int32_t* valid, const int32_t* subset, int n_subset) {
  Solver<T> S;
  if (!S.setup(pb)) return -1;
  auto visit = [&](size_t p) {
    int x = (int)(p % S.W), y = (int)(p / S.W);
    T c = (T)Solver<T>::kCmax;
    std::vector<T> pv(S.n_src, (T)Solver<T>::kCmax);
    std::vector<int32_t> ok(S.n_src, 0);
    if (S.pixel_valid(x, y)) {
      const double* pl = planes + 4 * p;
      V3<T> n{(T)pl[0], (T)pl[1], (T)pl[2]};
      c = S.cost(x, y, n, (T)pl[3], pv.data(), ok.data());
    }
    cost_out[p] = (double)c;
    if (per_view)
      for (int j = 0; j < S.n_src; ++j) per_view[p * S.n_src + j] = (double)pv[j];
    if (valid)
      for (int j = 0; j < S.n_src; ++j) valid[p * S.n_src + j] = ok[j];
  };
  if (subset) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n_subset; ++i) visit((size_t)subset[i]);
  } else {
#pragma omp parallel for schedule(dynamic, 256)
    for (long long p = 0; p < (long long)S.W * S.H; ++p) visit((size_t)p);
  }
  return 0;
}

// ---------------------------------------------------------------- geometric-consistency filter
// Sec. III-D: pixel x of reference view i with depth d_x and normal n_x is projected into
// neighbour view j with its depth (X = d_x K_i^-1 (x, y, 1) in camera i, then world, then
// camera j, then K_j).  There d' is the bilinear interpolation of view j's depth map and n'
// view j's normal at the rounded position.  The pair is consistent when the depths agree
// (|z_j(X) - d'| < tau_d d', X's depth in camera j against d'), the normals agree (angle
// below tau_n, compared in world coordinates as n . n' > cos tau_n) and the point of view
// j at d' re-projects into view i within tau_r pixels of x.  A pixel is kept when it is
// consistent with at least min_consistent neighbours (the paper: more than one).
// Readings: relative depth difference in view j; the neighbour is unusable (not
// consistent) when the position leaves [0, W-1] x [0, H-1], lies behind camera j, or any
// of the four depth texels is not positive; rounding is floor(u + 1/2); the re-projected
// point must lie in front of camera i.  Everything is FP64, one step at a time.
struct CamD {
  double K[9], Kinv[9], R[9], t[3];
};

bool cam_setup(const double* K, const double* R, const double* t, CamD& c) {
  for (int i = 0; i < 9; ++i) c.K[i] = K[i], c.R[i] = R[i];
  for (int i = 0; i < 3; ++i) c.t[i] = t[i];
  return mat3_inverse(c.K, c.Kinv);
}

// camera frame -> world: R^T (X - t)
void cam_to_world(const CamD& c, const double* X, double* Xw) {
  const double d0 = X[0] - c.t[0], d1 = X[1] - c.t[1], d2 = X[2] - c.t[2];
  for (int i = 0; i < 3; ++i) Xw[i] = c.R[i] * d0 + c.R[3 + i] * d1 + c.R[6 + i] * d2;
}

// world -> camera frame: R Xw + t
void world_to_cam(const CamD& c, const double* Xw, double* X) {
  for (int i = 0; i < 3; ++i) X[i] = c.R[3 * i] * Xw[0] + c.R[3 * i + 1] * Xw[1] + c.R[3 * i + 2] * Xw[2] + c.t[i];
}

// world-frame normal: R^T n
void normal_to_world(const CamD& c, const float* n, double* nw) {
  for (int i = 0; i < 3; ++i) nw[i] = c.R[i] * (double)n[0] + c.R[3 + i] * (double)n[1] + c.R[6 + i] * (double)n[2];
}

bool consistent_with(const CamD& ci, const CamD& cj, int Wj, int Hj, const float* Dj, const float* Nj, int x, int y,
                     double d, const float* n, double tau_d, double cos_n, double tau_r) {
  const double pix[3] = {(double)x, (double)y, 1.0};
  double ray[3], Xi[3], Xw[3], Xj[3], p[3];
  mat3_vec(ci.Kinv, pix, ray);
  for (int k = 0; k < 3; ++k) Xi[k] = d * ray[k];
  cam_to_world(ci, Xi, Xw);
  world_to_cam(cj, Xw, Xj);
  mat3_vec(cj.K, Xj, p);
  if (!(p[2] > 0.0)) return false;
  const double u = p[0] / p[2], v = p[1] / p[2];
  if (!(u >= 0.0 && u <= (double)(Wj - 1) && v >= 0.0 && v <= (double)(Hj - 1))) return false;
  // bilinear depth of view j
  const int x0 = (int)std::floor(u), y0 = (int)std::floor(v);
  const int x1 = std::min(x0 + 1, Wj - 1), y1 = std::min(y0 + 1, Hj - 1);
  const double fx = u - x0, fy = v - y0;
  const double d00 = Dj[(size_t)y0 * Wj + x0], d01 = Dj[(size_t)y0 * Wj + x1];
  const double d10 = Dj[(size_t)y1 * Wj + x0], d11 = Dj[(size_t)y1 * Wj + x1];
  if (!(d00 > 0.0 && d01 > 0.0 && d10 > 0.0 && d11 > 0.0)) return false;
  const double top = d00 + fx * (d01 - d00), bot = d10 + fx * (d11 - d10);
  const double dj = top + fy * (bot - top);
  // depth test in camera j
  if (!(std::fabs(Xj[2] - dj) < tau_d * dj)) return false;
  // normal test at the rounded position, in world coordinates
  const int xr = std::min((int)std::floor(u + 0.5), Wj - 1), yr = std::min((int)std::floor(v + 0.5), Hj - 1);
  const float* nj = Nj + 3 * ((size_t)yr * Wj + xr);
  double ni_w[3], nj_w[3];
  normal_to_world(ci, n, ni_w);
  normal_to_world(cj, nj, nj_w);
  const double dot = ni_w[0] * nj_w[0] + ni_w[1] * nj_w[1] + ni_w[2] * nj_w[2];
  if (!(dot > cos_n)) return false;
  // re-projection of view j's point into view i
  const double pj[3] = {u, v, 1.0};
  double rj[3], Yj[3], Yw[3], Yi[3], q[3];
  mat3_vec(cj.Kinv, pj, rj);
  for (int k = 0; k < 3; ++k) Yj[k] = dj * rj[k];
  cam_to_world(cj, Yj, Yw);
  world_to_cam(ci, Yw, Yi);
  mat3_vec(ci.K, Yi, q);
  if (!(q[2] > 0.0)) return false;
  const double ex = q[0] / q[2] - (double)x, ey = q[1] / q[2] - (double)y;
  return std::sqrt(ex * ex + ey * ey) < tau_r;
}

// ---------------------------------------------------------------- plane hypothesis inference
// Sec. III-E.  Hypotheses: every pixel without depth gets one depth per direction
// (horizontal, vertical, 45 degrees below, 45 degrees above), the value at the pixel of
// the straight line fitted (least squares, depth against step index s) to the six
// closest pixels with depth along that direction (both sides; by |s|, the negative side
// first on ties; fewer if the line leaves the image; none below two points or when the
// fitted depth is not positive).  FP64, sums in collection order.
const int kPhiDir[4][2] = {{1, 0}, {0, 1}, {1, 1}, {1, -1}};

double phi_line_fit(const float* depth, int W, int H, int x, int y, int dx, int dy) {
  double S0 = 0, S1 = 0, S2 = 0, T0 = 0, T1 = 0;
  int n = 0;
  for (int s = 1; n < 6; ++s) {
    bool any_inside = false;
    for (int side = -1; side <= 1 && n < 6; side += 2) {
      const int xs = x + side * s * dx, ys = y + side * s * dy;
      if (xs < 0 || xs >= W || ys < 0 || ys >= H) continue;
      any_inside = true;
      const double d = depth[(size_t)ys * W + xs];
      if (!(d > 0.0)) continue;
      const double si = (double)(side * s);
      S0 = S0 + 1.0;
      S1 = S1 + si;
      S2 = S2 + si * si;
      T0 = T0 + d;
      T1 = T1 + si * d;
      ++n;
    }
    if (!any_inside) break;
  }
  if (n < 2) return 0.0;
  const double det = S0 * S2 - S1 * S1;
  const double a = (S2 * T0 - S1 * T1) / det;
  return a > 0.0 ? a : 0.0;
}

// MAP labelling of a 4-connected grid by exhaustive search (tiny grids only): node i has
// n_lab[i] states with unary potentials un[i * 4 + k] > 0; an edge between nodes i and j
// (right and down neighbours) multiplies by pw(h_i, h_j).  Maximises the product (sum of
// logs).  Returns the label per node.
double phi_pairwise(double h1, double h2, double k3) {
  const double rel = h1 > h2 ? (h1 - h2) / h2 : (h2 - h1) / h1;
  const double m = rel < 1.0 ? rel : 1.0;
  return (k3 - m) * (k3 - m);
}

}  // namespace

extern "C" {

// Philox4x32-10 block: counter ctr[4], key key[2] -> out[4]
// Threads used by the pixel loops of the OpenMP build (returns the count in effect); the
// single-threaded build ignores the request and returns 1.
int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

void oracle_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

// Full PatchMatch run (init + iters x (red, black)); outputs row-major H x W (x3 for normal).
int oracle_patchmatch(const oracle_problem* pb, int iters, int fp64, float* depth, float* normal, float* cost) {
  return fp64 ? run_patchmatch<double>(pb, iters, depth, normal, cost)
              : run_patchmatch<float>(pb, iters, depth, normal, cost);
}

// Random initialisation of every pixel: planes (H*W*4: n.x, n.y, n.z, d), costs (H*W).
int oracle_init(const oracle_problem* pb, int fp64, double* planes, double* costs) {
  return fp64 ? run_init<double>(pb, planes, costs) : run_init<float>(pb, planes, costs);
}

// One half-sweep (colour 0 = red (x+y even), 1 = black) in place on (planes, costs).
int oracle_halfsweep(const oracle_problem* pb, int iteration, int colour, int fp64, double* planes, double* costs,
                     const int32_t* subset, int n_subset, int do_prop, int do_refine) {
  return fp64 ? run_halfsweep<double>(pb, iteration, colour, planes, costs, subset, n_subset, do_prop, do_refine)
              : run_halfsweep<float>(pb, iteration, colour, planes, costs, subset, n_subset, do_prop, do_refine);
}

// Cost of given planes (H*W*4) at every pixel (or at the listed pixels only).
int oracle_eval_cost(const oracle_problem* pb, int fp64, const double* planes, double* cost, double* per_view,
                     int32_t* valid, const int32_t* subset, int n_subset) {
  return fp64 ? run_eval<double>(pb, planes, cost, per_view, valid, subset, n_subset)
              : run_eval<float>(pb, planes, cost, per_view, valid, subset, n_subset);
}

// FP64 homography of source j (0-based) for plane (n, d) seen at reference pixel (x, y).
int oracle_homography(const oracle_problem* pb, int j, const double* n, double d, int x, int y, double* Hout) {
  Solver<double> S;
  if (!S.setup(pb)) return -1;
  V3<double> nn{n[0], n[1], n[2]};
  double rho = d * dot3(nn, S.ray(x, y));
  S.homography(j, nn, rho, Hout);
  return 0;
}

// Bilinear sample (position clamped into the image) of a single image.
double oracle_bilinear(const float* img, int W, int H, double u, double v, int fp64) {
  int32_t w[2] = {W, W}, h[2] = {H, H};
  const float* ims[2] = {img, img};
  oracle_problem pb{};
  pb.n_views = 2;
  pb.width = w;
  pb.height = h;
  pb.images = ims;
  if (fp64) {
    Solver<double> S;
    S.pb = &pb;
    return S.sample(1, u, v);
  }
  Solver<float> S;
  S.pb = &pb;
  return (double)S.sample(1, (float)u, (float)v);
}

// Geometric-consistency filter of reference view `ref` against `n_nbrs` neighbour views
// (Sec. III-D).  Cameras: K, R (9 doubles each), t (3) per view; depth / normal maps per
// view (row-major H x W and H x W x 3 float; NULL for views without a map).  Outputs
// (reference size): depth and normal kept or zeroed, and the number of consistent
// neighbours per pixel (pixels with depth <= 0 get 0 and are zeroed).
int oracle_consistency(int n_views, const int32_t* width, const int32_t* height, const double* K, const double* R,
                       const double* t, const float* const* depth, const float* const* normal, int ref,
                       const int32_t* nbrs, int n_nbrs, double tau_d, double tau_n_deg, double tau_r,
                       int min_consistent, float* out_depth, float* out_normal, uint8_t* out_count) {
  if (ref < 0 || ref >= n_views || !depth[ref] || !normal[ref]) return -1;
  std::vector<CamD> cams(n_views);
  for (int v = 0; v < n_views; ++v)
    if (!cam_setup(K + 9 * v, R + 9 * v, t + 3 * v, cams[v])) return -1;
  for (int k = 0; k < n_nbrs; ++k)
    if (nbrs[k] < 0 || nbrs[k] >= n_views || nbrs[k] == ref || !depth[nbrs[k]] || !normal[nbrs[k]]) return -1;
  const double cos_n = std::cos(tau_n_deg * 3.14159265358979323846 / 180.0);
  const int W = width[ref], H = height[ref];
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const size_t p = (size_t)y * W + x;
      const double d = depth[ref][p];
      const float* n = normal[ref] + 3 * p;
      int count = 0;
      if (d > 0.0)
        for (int k = 0; k < n_nbrs; ++k) {
          const int j = nbrs[k];
          count += consistent_with(cams[ref], cams[j], width[j], height[j], depth[j], normal[j], x, y, d, n, tau_d,
                                   cos_n, tau_r);
        }
      const bool keep = d > 0.0 && count >= min_consistent;
      out_count[p] = (uint8_t)std::min(count, 255);
      out_depth[p] = keep ? depth[ref][p] : 0.0f;
      for (int c = 0; c < 3; ++c) out_normal[3 * p + c] = keep ? n[c] : 0.0f;
    }
  return 0;
}

// Depth-map fusion (Sec. III-F).  The maps are handled in the order given.  For map i,
// every pixel that still has depth, in row-major order, is back-projected to X_i; for
// every later map j (earlier maps are already deleted) X_i is projected into camera j and
// rounded to the nearest pixel q = (floor(u + 1/2), floor(v + 1/2)); when q lies in the
// image, still has depth and its back-projection X'_j is within max_rel_dist d_i of X_i
// (Euclidean distance, compared squared; d_i the depth of X_i in camera i), q is deleted from map j and X'_j
// joins the point.  The point is the mean of X_i and its joined X'_j (summed in j order),
// then map i is deleted.  Outputs over the concatenated maps (map i at the offset of the
// pixel counts of maps 0..i-1): points (3 floats, world frame) and support (pixels merged)
// at the pixel a point started from, zero elsewhere; owner = the concatenated index of
// the point a pixel ended in, -1 for pixels without depth.  FP64 throughout.
static void fuse_back_project(const CamD& c, int x, int y, double d, double* Xw) {
  const double pix[3] = {(double)x, (double)y, 1.0};
  double ray[3], X[3];
  mat3_vec(c.Kinv, pix, ray);
  for (int k = 0; k < 3; ++k) X[k] = d * ray[k];
  cam_to_world(c, X, Xw);
}

int oracle_fuse(int n_maps, const int32_t* width, const int32_t* height, const double* K, const double* R,
                const double* t, const float* const* depth, double max_rel_dist, float* points, int32_t* support,
                int64_t* owner) {
  std::vector<CamD> cams(n_maps);
  std::vector<size_t> off(n_maps + 1, 0);
  for (int v = 0; v < n_maps; ++v) {
    if (!cam_setup(K + 9 * v, R + 9 * v, t + 3 * v, cams[v]) || !depth[v] || width[v] <= 0 || height[v] <= 0)
      return -1;
    off[v + 1] = off[v] + (size_t)width[v] * height[v];
  }
  std::vector<uint8_t> alive(off[n_maps]);
  for (int v = 0; v < n_maps; ++v)
    for (size_t p = 0; p < off[v + 1] - off[v]; ++p) {
      alive[off[v] + p] = depth[v][p] > 0.0f;
      owner[off[v] + p] = -1;
      support[off[v] + p] = 0;
      for (int c = 0; c < 3; ++c) points[3 * (off[v] + p) + c] = 0.0f;
    }
  for (int i = 0; i < n_maps; ++i) {
    const int Wi = width[i], Hi = height[i];
    for (int y = 0; y < Hi; ++y)
      for (int x = 0; x < Wi; ++x) {
        const size_t gi = off[i] + (size_t)y * Wi + x;
        if (!alive[gi]) continue;
        const double d = depth[i][(size_t)y * Wi + x];
        double Xi[3];
        fuse_back_project(cams[i], x, y, d, Xi);
        double sum[3] = {Xi[0], Xi[1], Xi[2]};
        int count = 1;
        owner[gi] = (int64_t)gi;
        for (int j = i + 1; j < n_maps; ++j) {
          double Xj[3], p[3];
          world_to_cam(cams[j], Xi, Xj);
          mat3_vec(cams[j].K, Xj, p);
          if (!(p[2] > 0.0)) continue;
          const double xr = std::floor(p[0] / p[2] + 0.5), yr = std::floor(p[1] / p[2] + 0.5);
          if (!(xr >= 0.0 && xr <= (double)(width[j] - 1) && yr >= 0.0 && yr <= (double)(height[j] - 1))) continue;
          const int qx = (int)xr, qy = (int)yr;
          const size_t q = (size_t)qy * width[j] + qx;
          if (!alive[off[j] + q]) continue;
          double Yw[3];
          fuse_back_project(cams[j], qx, qy, (double)depth[j][q], Yw);
          const double e0 = Yw[0] - Xi[0], e1 = Yw[1] - Xi[1], e2 = Yw[2] - Xi[2];
          const double lim = max_rel_dist * d;
          if (!(e0 * e0 + e1 * e1 + e2 * e2 < lim * lim)) continue;  // distance below lim, squared
          alive[off[j] + q] = 0;
          owner[off[j] + q] = (int64_t)gi;
          for (int k = 0; k < 3; ++k) sum[k] = sum[k] + Yw[k];
          ++count;
        }
        alive[gi] = 0;
        support[gi] = count;
        for (int k = 0; k < 3; ++k) points[3 * gi + k] = (float)(sum[k] / (double)count);
      }
  }
  return 0;
}

// Plane-hypothesis depths (Sec. III-E) of every pixel without depth: hyp (H*W*4), 0 = none.
void oracle_phi_hypotheses(const float* depth, int W, int H, float* hyp) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const size_t p = (size_t)y * W + x;
      for (int k = 0; k < 4; ++k)
        hyp[4 * p + k] = depth[p] > 0.0f ? 0.0f : (float)phi_line_fit(depth, W, H, x, y, kPhiDir[k][0], kPhiDir[k][1]);
    }
}

// Exact MAP of the pairwise model of Sec. III-E on a tiny grid (W*H nodes, at most 4
// states each, brute force over all labellings).  depth[i] > 0 makes node i a fixed
// single-state node with that depth and potential 1; otherwise its states are the
// non-zero hyp[4 i + k] with unary (C_max - cost[4 i + k]) / k1 + k2.  Edge potential
// [k3 - min(1, relative difference)]^2 (Eq. 8).  label[i] receives the chosen k (or -1
// for fixed nodes / nodes without a state); returns the maximal log-potential.  Labellings
// are enumerated with node 0 varying fastest and each node's states in order of k; of
// equal maxima the first one is kept.
double oracle_phi_map_bruteforce(const float* depth, const float* hyp, const float* cost, int W, int H, double k1,
                                 double k2, double k3, double cmax, int32_t* label) {
  const int N = W * H;
  std::vector<std::vector<int>> states(N);
  std::vector<std::vector<double>> val(N), logu(N);
  for (int i = 0; i < N; ++i) {
    if (depth[i] > 0.0f) {
      states[i].push_back(-1);
      val[i].push_back(depth[i]);
      logu[i].push_back(0.0);
      continue;
    }
    for (int k = 0; k < 4; ++k)
      if (hyp[4 * i + k] > 0.0f) {
        states[i].push_back(k);
        val[i].push_back(hyp[4 * i + k]);
        logu[i].push_back(std::log((cmax - (double)cost[4 * i + k]) / k1 + k2));
      }
    if (states[i].empty()) {  // no state: isolated from the model
      states[i].push_back(-1);
      val[i].push_back(0.0);
      logu[i].push_back(0.0);
    }
  }
  std::vector<int> cur(N, 0), best(N, 0);
  double best_e = -1e300;
  for (;;) {
    double e = 0.0;
    for (int i = 0; i < N; ++i) e += logu[i][cur[i]];
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const int i = y * W + x;
        const double hi = val[i][cur[i]];
        if (!(hi > 0.0)) continue;
        if (x + 1 < W && val[i + 1][cur[i + 1]] > 0.0) e += std::log(phi_pairwise(hi, val[i + 1][cur[i + 1]], k3));
        if (y + 1 < H && val[i + W][cur[i + W]] > 0.0) e += std::log(phi_pairwise(hi, val[i + W][cur[i + W]], k3));
      }
    if (e > best_e) {
      best_e = e;
      best = cur;
    }
    int i = 0;
    while (i < N && ++cur[i] == (int)states[i].size()) cur[i++] = 0;
    if (i == N) break;
  }
  for (int i = 0; i < N; ++i) label[i] = states[i][best[i]];
  return best_e;
}

// Approximate MAP of the same model by sequential tree-reweighted message passing (the
// paper decodes its graph model with TRW, Sec. III-E; TRW-S as published by Kolmogorov,
// 2006, on the 4-connected grid with the nodes in raster order), minimising the sum of
// -log potentials.  Nodes with a state: a fixed node has its depth as its only state,
// with cost 0; a node without depth has its non-zero hypotheses, in order of k, with cost
// -log((C_max - cost) / k1 + k2).  An edge between two nodes with states costs
// -log([k3 - min(1, relative difference)]^2).  Messages start at 0.  One iteration is a
// forward pass over the nodes in raster order, then a backward pass in reverse order.  At
// each node the belief is its cost plus the incoming messages, added in the order up, left,
// right, down; the node then sends to each of its later neighbours (right, down; in the
// backward pass its earlier ones, up and left) the message
//   m(s_j) = min over s of [gamma b(s) - m_{j->i}(s) + E(s, s_j)]
// (evaluated left to right), minus its smallest value, where gamma = 1 / max(number of
// earlier, number of later neighbours with states).  Then the nodes are labelled in raster
// order: the state with the lowest cost plus edge costs to the labels already chosen for
// the up and left neighbours plus the messages from the right and down neighbours (these
// terms added in the order up, left, right, down), the first such state on ties.
// label[i] receives k (-1 for a fixed node or one without states), value[i] its depth (0
// without states).  Parity unpinned in part: on a forest TRW is exact and the tests hold
// it to the enumerated MAP; the weights gamma and the exact sweep schedule act on graphs
// with loops alone, where the tests hold the decoder to the exact minimum only for binary
// submodular energies (where TRW reaches the global minimum, Kolmogorov and Wainwright
// 2005; the enumerated MAP on small grids, a minimum s-t cut on larger ones: over-counting
// and smaller weights fail there, a message also sent against the sweep direction does
// not) and otherwise to near-optimality.
void oracle_phi_trws(const float* depth, const float* hyp, const float* cost, int W, int H, double k1, double k2,
                     double k3, double cmax, int iterations, int32_t* label, float* value) {
  const int N = W * H;
  std::vector<std::vector<int>> states(N);
  std::vector<std::vector<double>> val(N), unary(N);
  for (int i = 0; i < N; ++i) {
    if (depth[i] > 0.0f) {
      states[i].push_back(-1);
      val[i].push_back(depth[i]);
      unary[i].push_back(0.0);
      continue;
    }
    for (int k = 0; k < 4; ++k)
      if (hyp[4 * i + k] > 0.0f) {
        states[i].push_back(k);
        val[i].push_back(hyp[4 * i + k]);
        unary[i].push_back(-std::log((cmax - (double)cost[4 * i + k]) / k1 + k2));
      }
  }
  // neighbour of node i in direction d (0 up, 1 left, 2 right, 3 down) with states, or -1
  auto nb = [&](int i, int d) {
    const int x = i % W, y = i / W;
    int j = -1;
    if (d == 0 && y > 0) j = i - W;
    if (d == 1 && x > 0) j = i - 1;
    if (d == 2 && x + 1 < W) j = i + 1;
    if (d == 3 && y + 1 < H) j = i + W;
    return j >= 0 && !states[j].empty() ? j : -1;
  };
  auto E = [&](double a, double b) { return -std::log(phi_pairwise(a, b, k3)); };
  // msg[i][d]: the message node i received from its neighbour in direction d
  std::vector<std::vector<std::vector<double>>> msg(N, std::vector<std::vector<double>>(4));
  std::vector<double> gamma(N, 1.0);
  for (int i = 0; i < N; ++i) {
    for (int d = 0; d < 4; ++d) msg[i][d].assign(states[i].size(), 0.0);
    int earlier = 0, later = 0;
    for (int d = 0; d < 4; ++d)
      if (nb(i, d) >= 0) (d < 2 ? earlier : later)++;
    const int m = std::max(earlier, later);
    if (m > 0) gamma[i] = 1.0 / m;
  }
  auto visit = [&](int i, int d_first) {
    const size_t n = states[i].size();
    if (n == 0) return;
    std::vector<double> b(unary[i]);
    for (int d = 0; d < 4; ++d)
      if (nb(i, d) >= 0)
        for (size_t s = 0; s < n; ++s) b[s] += msg[i][d][s];
    for (int d = d_first; d < d_first + 2; ++d) {
      const int j = nb(i, d);
      if (j < 0) continue;
      std::vector<double>& out = msg[j][3 - d];
      double lo = std::numeric_limits<double>::infinity();
      for (size_t t = 0; t < states[j].size(); ++t) {
        double best = std::numeric_limits<double>::infinity();
        for (size_t s = 0; s < n; ++s) {
          const double v = gamma[i] * b[s] - msg[i][d][s] + E(val[i][s], val[j][t]);
          if (v < best) best = v;
        }
        out[t] = best;
        if (best < lo) lo = best;
      }
      for (double& v : out) v -= lo;
    }
  };
  for (int it = 0; it < iterations; ++it) {
    for (int i = 0; i < N; ++i) visit(i, 2);
    for (int i = N - 1; i >= 0; --i) visit(i, 0);
  }
  std::vector<int> pick(N, -1);
  for (int i = 0; i < N; ++i) {
    label[i] = -1;
    value[i] = 0.0f;
    if (states[i].empty()) continue;
    double best = std::numeric_limits<double>::infinity();
    for (size_t s = 0; s < states[i].size(); ++s) {
      double e = unary[i][s];
      for (int d = 0; d < 4; ++d) {
        const int j = nb(i, d);
        if (j < 0) continue;
        e += d < 2 ? E(val[j][pick[j]], val[i][s]) : msg[i][d][s];
      }
      if (e < best) {
        best = e;
        pick[i] = (int)s;
      }
    }
    if (pick[i] < 0) pick[i] = 0;
    label[i] = states[i][pick[i]];
    value[i] = (float)val[i][pick[i]];
  }
}

// Normals of Eq. 10 (with the norm, not its square): n = (X_u - X_d) x (X_l - X_r),
// normalised and turned to face the camera, X the back-projection d K^-1 (x, y, 1) of the
// 4-connected neighbours (up = y - 1, left = x - 1).  Pixels without depth, or with a
// neighbour without depth or outside the image, get 0.  FP64.
int oracle_phi_normals(const float* depth, int W, int H, const double* K, float* normal) {
  double Ki[9];
  if (!mat3_inverse(K, Ki)) return -1;
  auto back = [&](int x, int y, double* X) {
    const double pix[3] = {(double)x, (double)y, 1.0};
    double r[3];
    mat3_vec(Ki, pix, r);
    const double d = depth[(size_t)y * W + x];
    for (int k = 0; k < 3; ++k) X[k] = d * r[k];
  };
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      float* n = normal + 3 * ((size_t)y * W + x);
      n[0] = n[1] = n[2] = 0.0f;
      if (x < 1 || y < 1 || x + 1 >= W || y + 1 >= H) continue;
      const size_t p = (size_t)y * W + x;
      if (!(depth[p] > 0.0f && depth[p - W] > 0.0f && depth[p + W] > 0.0f && depth[p - 1] > 0.0f &&
            depth[p + 1] > 0.0f))
        continue;
      double Xu[3], Xd[3], Xl[3], Xr[3], C[3];
      back(x, y - 1, Xu);
      back(x, y + 1, Xd);
      back(x - 1, y, Xl);
      back(x + 1, y, Xr);
      back(x, y, C);
      const double a[3] = {Xu[0] - Xd[0], Xu[1] - Xd[1], Xu[2] - Xd[2]};
      const double b[3] = {Xl[0] - Xr[0], Xl[1] - Xr[1], Xl[2] - Xr[2]};
      double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
      const double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      if (!(len > 0.0)) continue;
      if (c[0] * C[0] + c[1] * C[1] + c[2] * C[2] > 0.0) c[0] = -c[0], c[1] = -c[1], c[2] = -c[2];
      for (int k = 0; k < 3; ++k) n[k] = (float)(c[k] / len);
    }
  return 0;
}

// Eq. 5 over the best-K valid views, for hand-set per-view costs.
double oracle_aggregate(const double* cj, const int32_t* valid, int n, int top_k, double eps_c, int fp64) {
  std::vector<int> ok(valid, valid + n);
  if (fp64) return aggregate<double>(cj, ok.data(), n, top_k, eps_c);
  std::vector<float> cf(cj, cj + n);
  return (double)aggregate<float>(cf.data(), ok.data(), n, top_k, (float)eps_c);
}

}  // extern "C"
