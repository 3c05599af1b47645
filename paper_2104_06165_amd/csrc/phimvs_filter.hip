// Geometric-consistency filter of a depth map against its neighbours' maps (PHI-MVS
// Sec. III-D).  One thread per reference pixel; per neighbour the point is carried from
// the reference camera to the world and into the neighbour camera, compared with the
// neighbour's bilinear depth and its normal at the rounded position, and the neighbour's
// point is carried back to test the re-projection error.  FP64 throughout, each step
// written out in the order stated (no contraction), so the keep / drop decision of every
// pixel is the one a sequential FP64 evaluation takes.  The work is about 250 FP64
// instructions (the camera chain, four divisions, a square root) and about 30 bytes of
// gathers per pixel and neighbour: the FP64 instruction stream is the tighter limit
// (the vector ALU about 80% busy), the memory system about half.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phimvs_internal.h"

namespace pmf {

using namespace phimvs_internal;

__device__ __forceinline__ void mat_vec(const double* M, const double* v, double* o) {
#pragma unroll
  for (int i = 0; i < 3; ++i) o[i] = M[3 * i] * v[0] + M[3 * i + 1] * v[1] + M[3 * i + 2] * v[2];
}

// camera -> world: R^T (X - t)
__device__ __forceinline__ void to_world(const double* R, const double* t, const double* X, double* Xw) {
  const double d0 = X[0] - t[0], d1 = X[1] - t[1], d2 = X[2] - t[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) Xw[i] = R[i] * d0 + R[3 + i] * d1 + R[6 + i] * d2;
}

// world -> camera: R Xw + t
__device__ __forceinline__ void to_cam(const double* R, const double* t, const double* Xw, double* X) {
#pragma unroll
  for (int i = 0; i < 3; ++i) X[i] = R[3 * i] * Xw[0] + R[3 * i + 1] * Xw[1] + R[3 * i + 2] * Xw[2] + t[i];
}

// R^T n
__device__ __forceinline__ void normal_world(const double* R, float n0, float n1, float n2, double* nw) {
#pragma unroll
  for (int i = 0; i < 3; ++i) nw[i] = R[i] * (double)n0 + R[3 + i] * (double)n1 + R[6 + i] * (double)n2;
}

__device__ bool consistent(const FilterArgs& a, const FilterNbr& nb, int x, int y, double d, float n0, float n1,
                           float n2) {
  const double pix[3] = {(double)x, (double)y, 1.0};
  double ray[3], Xi[3], Xw[3], Xj[3], p[3];
  mat_vec(a.Kinv, pix, ray);
#pragma unroll
  for (int k = 0; k < 3; ++k) Xi[k] = d * ray[k];
  to_world(a.R, a.t, Xi, Xw);
  to_cam(nb.R, nb.t, Xw, Xj);
  mat_vec(nb.K, Xj, p);
  if (!(p[2] > 0.0)) return false;
  const double u = p[0] / p[2], v = p[1] / p[2];
  if (!(u >= 0.0 && u <= (double)(nb.W - 1) && v >= 0.0 && v <= (double)(nb.H - 1))) return false;
  const int x0 = (int)floor(u), y0 = (int)floor(v);
  const int x1 = min(x0 + 1, nb.W - 1), y1 = min(y0 + 1, nb.H - 1);
  const double fx = u - (double)x0, fy = v - (double)y0;
  const double d00 = nb.depth[(size_t)y0 * nb.W + x0], d01 = nb.depth[(size_t)y0 * nb.W + x1];
  const double d10 = nb.depth[(size_t)y1 * nb.W + x0], d11 = nb.depth[(size_t)y1 * nb.W + x1];
  if (!(d00 > 0.0 && d01 > 0.0 && d10 > 0.0 && d11 > 0.0)) return false;
  const double top = d00 + fx * (d01 - d00), bot = d10 + fx * (d11 - d10);
  const double dj = top + fy * (bot - top);
  if (!(fabs(Xj[2] - dj) < a.tau_d * dj)) return false;
  const int xr = min((int)floor(u + 0.5), nb.W - 1), yr = min((int)floor(v + 0.5), nb.H - 1);
  const float* nj = nb.normal + 3 * ((size_t)yr * nb.W + xr);
  double niw[3], njw[3];
  normal_world(a.R, n0, n1, n2, niw);
  normal_world(nb.R, nj[0], nj[1], nj[2], njw);
  const double dot = niw[0] * njw[0] + niw[1] * njw[1] + niw[2] * njw[2];
  if (!(dot > a.cos_n)) return false;
  const double pj[3] = {u, v, 1.0};
  double rj[3], Yj[3], Yw[3], Yi[3], q[3];
  mat_vec(nb.Kinv, pj, rj);
#pragma unroll
  for (int k = 0; k < 3; ++k) Yj[k] = dj * rj[k];
  to_world(nb.R, nb.t, Yj, Yw);
  to_cam(a.R, a.t, Yw, Yi);
  mat_vec(a.K, Yi, q);
  if (!(q[2] > 0.0)) return false;
  const double ex = q[0] / q[2] - (double)x, ey = q[1] / q[2] - (double)y;
  return sqrt(ex * ex + ey * ey) < a.tau_r;
}

__global__ __launch_bounds__(256) void filter_kernel(FilterArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.W || y >= a.H) return;
  const size_t p = (size_t)y * a.W + x;
  const float df = a.depth[p];
  const float n0 = a.normal[3 * p], n1 = a.normal[3 * p + 1], n2 = a.normal[3 * p + 2];
  const double d = (double)df;
  int count = 0;
  if (d > 0.0)
    for (int k = 0; k < a.n_nbrs; ++k) count += consistent(a, a.nbrs[k], x, y, d, n0, n1, n2) ? 1 : 0;
  const bool keep = d > 0.0 && count >= a.min_consistent;
  a.count_out[p] = (uint8_t)min(count, 255);
  a.depth_out[p] = keep ? df : 0.0f;
  a.normal_out[3 * p] = keep ? n0 : 0.0f;
  a.normal_out[3 * p + 1] = keep ? n1 : 0.0f;
  a.normal_out[3 * p + 2] = keep ? n2 : 0.0f;
}

}  // namespace pmf

namespace phimvs_internal {

hipError_t launch_filter(const FilterArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(pmf::filter_kernel, dim3((a.W + 255) / 256, a.H), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace phimvs_internal
