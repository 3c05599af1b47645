// Depth-map fusion (PHI-MVS Sec. III-F) as a sequence of data-parallel steps.  The paper
// walks the maps in order and, within a map, its pixels one by one; a later pixel only
// sees what earlier ones deleted.  Within one map's step the only state that changes is
// the deletion of pixels of later maps, and a pixel of map j is deleted by the first pixel
// (row-major) of map i that passes the test against it.  So each step is two launches:
// every pixel of map i tests its candidate in each later map and claims it with an atomic
// minimum of its own index; then every pixel merges exactly the candidates it won.  The
// result equals the sequential walk.  All arithmetic is FP64, each expression in the order
// written, so both launches compute the same candidate for a pixel.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phimvs_internal.h"

namespace pmu {

using namespace phimvs_internal;

constexpr int kBlock = 256;

// pixel (x, y) at depth d of a map's camera -> world point: R^T (d K^-1 (x, y, 1) - t)
__device__ __forceinline__ void back_project(const FuseMap& m, int x, int y, double d, double* Xw) {
  const double px = (double)x, py = (double)y;
  double X[3];
  for (int k = 0; k < 3; ++k) X[k] = d * (m.Kinv[3 * k] * px + m.Kinv[3 * k + 1] * py + m.Kinv[3 * k + 2] * 1.0);
  const double d0 = X[0] - m.t[0], d1 = X[1] - m.t[1], d2 = X[2] - m.t[2];
  for (int k = 0; k < 3; ++k) Xw[k] = m.R[k] * d0 + m.R[3 + k] * d1 + m.R[6 + k] * d2;
}

// nearest pixel of map m that world point Xw projects to; false when behind the camera
// or outside the image
__device__ __forceinline__ bool project_round(const FuseMap& m, const double* Xw, int& qx, int& qy) {
  double X[3], p[3];
  for (int k = 0; k < 3; ++k) X[k] = m.R[3 * k] * Xw[0] + m.R[3 * k + 1] * Xw[1] + m.R[3 * k + 2] * Xw[2] + m.t[k];
  for (int k = 0; k < 3; ++k) p[k] = m.K[3 * k] * X[0] + m.K[3 * k + 1] * X[1] + m.K[3 * k + 2] * X[2];
  if (!(p[2] > 0.0)) return false;
  const double xr = floor(p[0] / p[2] + 0.5), yr = floor(p[1] / p[2] + 0.5);
  if (!(xr >= 0.0 && xr <= (double)(m.W - 1) && yr >= 0.0 && yr <= (double)(m.H - 1))) return false;
  qx = (int)xr;
  qy = (int)yr;
  return true;
}

__global__ __launch_bounds__(kBlock) void fuse_init_kernel(FuseMap m, uint8_t* __restrict__ alive,
                                                           float* __restrict__ points, int32_t* __restrict__ support,
                                                           int64_t* __restrict__ owner) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t n = (int64_t)m.W * m.H;
  if (p >= n) return;
  const int64_t g = m.off + p;
  alive[g] = m.depth[p] > 0.0f ? 1 : 0;
  support[g] = 0;
  owner[g] = -1;
  points[3 * g] = 0.0f;
  points[3 * g + 1] = 0.0f;
  points[3 * g + 2] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void fuse_fill_kernel(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] = v;
}

// every live pixel of map i claims, in each later map, the candidate that passes the test
__global__ __launch_bounds__(kBlock) void fuse_claim_kernel(const FuseMap* __restrict__ maps, int n_maps, int i,
                                                            double tau, const uint8_t* __restrict__ alive,
                                                            int32_t* __restrict__ claim) {
  const FuseMap& mi = maps[i];
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= mi.W * mi.H || !alive[mi.off + p]) return;
  const int y = p / mi.W, x = p - y * mi.W;
  const double d = mi.depth[p];
  double Xi[3];
  back_project(mi, x, y, d, Xi);
  const double lim = tau * d;
  for (int j = i + 1; j < n_maps; ++j) {
    const FuseMap& mj = maps[j];
    int qx, qy;
    if (!project_round(mj, Xi, qx, qy)) continue;
    const int64_t q = (int64_t)qy * mj.W + qx;
    if (!alive[mj.off + q]) continue;
    double Yw[3];
    back_project(mj, qx, qy, (double)mj.depth[q], Yw);
    const double e0 = Yw[0] - Xi[0], e1 = Yw[1] - Xi[1], e2 = Yw[2] - Xi[2];
    if (!(e0 * e0 + e1 * e1 + e2 * e2 < lim * lim)) continue;
    atomicMin(&claim[mj.off + q], p);
  }
}

// every live pixel of map i becomes a point with the candidates it won, which are deleted
__global__ __launch_bounds__(kBlock) void fuse_merge_kernel(const FuseMap* __restrict__ maps, int n_maps, int i,
                                                            uint8_t* __restrict__ alive,
                                                            const int32_t* __restrict__ claim,
                                                            float* __restrict__ points, int32_t* __restrict__ support,
                                                            int64_t* __restrict__ owner) {
  const FuseMap& mi = maps[i];
  const int p = blockIdx.x * kBlock + threadIdx.x;
  const int64_t g = mi.off + p;
  // a pixel of map i is only read and written by its own thread here
  if (p >= mi.W * mi.H || !alive[g]) return;
  const int y = p / mi.W, x = p - y * mi.W;
  const double d = mi.depth[p];
  double Xi[3];
  back_project(mi, x, y, d, Xi);
  double sum[3] = {Xi[0], Xi[1], Xi[2]};
  int count = 1;
  for (int j = i + 1; j < n_maps; ++j) {
    const FuseMap& mj = maps[j];
    int qx, qy;
    if (!project_round(mj, Xi, qx, qy)) continue;
    const int64_t q = (int64_t)qy * mj.W + qx;
    // a claim by p means q was live and passed the test in the claim launch
    if (claim[mj.off + q] != p) continue;
    double Yw[3];
    back_project(mj, qx, qy, (double)mj.depth[q], Yw);
    alive[mj.off + q] = 0;
    owner[mj.off + q] = g;
    for (int k = 0; k < 3; ++k) sum[k] = sum[k] + Yw[k];
    ++count;
  }
  alive[g] = 0;
  owner[g] = g;
  support[g] = count;
  for (int k = 0; k < 3; ++k) points[3 * g + k] = (float)(sum[k] / (double)count);
}

}  // namespace pmu

namespace phimvs_internal {

hipError_t launch_fuse(const FuseMap* h_maps, const FuseMap* d_maps, int n_maps, double tau, uint8_t* alive,
                       int32_t* claim, float* points, int32_t* support, int64_t* owner, hipStream_t st) {
  const int64_t total = h_maps[n_maps - 1].off + (int64_t)h_maps[n_maps - 1].W * h_maps[n_maps - 1].H;
  for (int v = 0; v < n_maps; ++v) {
    const int64_t n = (int64_t)h_maps[v].W * h_maps[v].H;
    hipLaunchKernelGGL(pmu::fuse_init_kernel, dim3((unsigned)((n + pmu::kBlock - 1) / pmu::kBlock)),
                       dim3(pmu::kBlock), 0, st, h_maps[v], alive, points, support, owner);
  }
  for (int i = 0; i < n_maps; ++i) {
    const int64_t n = (int64_t)h_maps[i].W * h_maps[i].H;
    const unsigned blocks = (unsigned)((n + pmu::kBlock - 1) / pmu::kBlock);
    if (i + 1 < n_maps) {
      const int64_t rest = total - h_maps[i + 1].off;
      hipLaunchKernelGGL(pmu::fuse_fill_kernel, dim3((unsigned)((rest + pmu::kBlock - 1) / pmu::kBlock)),
                         dim3(pmu::kBlock), 0, st, claim + h_maps[i + 1].off, rest, INT32_MAX);
      hipLaunchKernelGGL(pmu::fuse_claim_kernel, dim3(blocks), dim3(pmu::kBlock), 0, st, d_maps, n_maps, i, tau,
                         (const uint8_t*)alive, claim);
    }
    hipLaunchKernelGGL(pmu::fuse_merge_kernel, dim3(blocks), dim3(pmu::kBlock), 0, st, d_maps, n_maps, i, alive,
                       (const int32_t*)claim, points, support, owner);
  }
  return hipGetLastError();
}

}  // namespace phimvs_internal
