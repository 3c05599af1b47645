// Data-parallel parts of plane hypothesis inference (PHI-MVS Sec. III-E): depth
// hypotheses by 1-D line fits in four directions, the fronto-parallel planes whose cost
// scores them, the choice of the hypothesis closest to the decoded reference map, and
// the normals of Eq. 10.  One thread per pixel; FP64 wherever a value decides something,
// written in the order stated so that results equal a sequential FP64 evaluation.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phimvs_internal.h"

namespace pmp {

using namespace phimvs_internal;

__constant__ int kDir[4][2] = {{1, 0}, {0, 1}, {1, 1}, {1, -1}};

// least-squares line through the six closest pixels with depth along (dx, dy), value at s = 0
__device__ double line_fit(const float* __restrict__ depth, int W, int H, int x, int y, int dx, int dy) {
  double S0 = 0.0, S1 = 0.0, S2 = 0.0, T0 = 0.0, T1 = 0.0;
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

__global__ __launch_bounds__(256) void phi_hyp_kernel(const float* __restrict__ depth, int W, int H,
                                                      float* __restrict__ hyp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const size_t p = (size_t)y * W + x, plane = (size_t)W * H;
  const bool hole = !(depth[p] > 0.0f);
  for (int k = 0; k < 4; ++k)
    hyp[k * plane + p] = hole ? (float)line_fit(depth, W, H, x, y, kDir[k][0], kDir[k][1]) : 0.0f;
}

// hypothesis k -> fronto-parallel plane (n = (0, 0, -1), d = h); an empty one gets d = 1
// (finite arithmetic; its cost is replaced afterwards)
__global__ void phi_planes_kernel(const float* __restrict__ hyp, size_t n, float* __restrict__ planes) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float h = hyp[i];
  planes[4 * i] = 0.0f;
  planes[4 * i + 1] = 0.0f;
  planes[4 * i + 2] = -1.0f;
  planes[4 * i + 3] = h > 0.0f ? h : 1.0f;
}

__global__ void phi_mask_cost_kernel(const float* __restrict__ hyp, size_t n, float cmax, float* __restrict__ cost) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!(hyp[i] > 0.0f)) cost[i] = cmax;
}

// each pixel without depth takes the hypothesis closest to the reference map
__global__ void phi_select_kernel(const float* __restrict__ depth, const float* __restrict__ hyp,
                                  const float* __restrict__ ref, int W, int H, float* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const size_t p = (size_t)y * W + x, plane = (size_t)W * H;
  const float d = depth[p];
  if (d > 0.0f) {
    out[p] = d;
    return;
  }
  const double r = ref[p];
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

namespace phimvs_internal {

hipError_t launch_phi_hypotheses(const float* depth, int W, int H, float* hyp, hipStream_t st) {
  hipLaunchKernelGGL(pmp::phi_hyp_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, W, H, hyp);
  return hipGetLastError();
}

hipError_t launch_phi_planes(const float* hyp, size_t n, float* planes, hipStream_t st) {
  hipLaunchKernelGGL(pmp::phi_planes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, hyp, n, planes);
  return hipGetLastError();
}

hipError_t launch_phi_mask_cost(const float* hyp, size_t n, float cmax, float* cost, hipStream_t st) {
  hipLaunchKernelGGL(pmp::phi_mask_cost_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, hyp, n, cmax,
                     cost);
  return hipGetLastError();
}

hipError_t launch_phi_select(const float* depth, const float* hyp, const float* ref, int W, int H, float* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(pmp::phi_select_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, hyp, ref, W, H, out);
  return hipGetLastError();
}

hipError_t launch_phi_normals(const float* depth, int W, int H, const PhiCam& cam, float* normal, hipStream_t st) {
  hipLaunchKernelGGL(pmp::phi_normals_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, W, H, cam, normal);
  return hipGetLastError();
}

}  // namespace phimvs_internal
