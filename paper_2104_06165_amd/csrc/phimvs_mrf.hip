// Host-side selection step of plane hypothesis inference (PHI-MVS Sec. III-E): the
// pairwise undirected graph model over a 4-connected pixel grid, decoded by sequential
// tree-reweighted message passing (TRW-S, Kolmogorov 2006).  The paper runs this part on
// the CPU; so does the library.  Potentials: node states are a pixel's depth hypotheses
// with phi_n = (C_max - C) / k1 + k2 (Eq. 7), pixels that already have depth are fixed
// single-state nodes (phi = 1), edges carry phi_e = [k3 - min(1, relative difference)]^2
// (Eq. 8); decoding maximises the product, i.e. minimises the sum of -log potentials.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

#include "phimvs.h"

namespace {

constexpr int kMaxLab = 4;

struct Node {
  int n = 0;                 // number of states (0: not part of the model)
  int label[kMaxLab];        // hypothesis index of each state (-1: the fixed depth)
  double value[kMaxLab];     // depth of each state
  double unary[kMaxLab];     // -log phi_n
};

double edge_energy(double h1, double h2, double k3) {
  const double rel = h1 > h2 ? (h1 - h2) / h2 : (h2 - h1) / h1;
  const double m = rel < 1.0 ? rel : 1.0;
  return -std::log((k3 - m) * (k3 - m));
}

}  // namespace

extern "C" int phimvs_phi_decode_host(int width, int height, const float* depth, const float* hyp, const float* cost,
                                      double k1, double k2, double k3, double cost_max, int iterations,
                                      int32_t* label_out, float* depth_out) {
  if (width < 1 || height < 1 || !depth || !hyp || !cost || !label_out || !depth_out) return PHIMVS_E_ARG;
  if (!(k1 > 0) || !(k2 > 0) || !(k3 > 1) || iterations < 0) return PHIMVS_E_ARG;
  const int W = width, H = height, N = W * H;
  const size_t plane = (size_t)N;
  std::vector<Node> nodes(N);
  for (int i = 0; i < N; ++i) {
    Node& nd = nodes[i];
    if (depth[i] > 0.0f) {
      nd.n = 1;
      nd.label[0] = -1;
      nd.value[0] = depth[i];
      nd.unary[0] = 0.0;
      continue;
    }
    for (int k = 0; k < kMaxLab; ++k) {
      const float h = hyp[k * plane + i];
      if (!(h > 0.0f)) continue;
      const double phi = (cost_max - (double)cost[k * plane + i]) / k1 + k2;
      nd.label[nd.n] = k;
      nd.value[nd.n] = h;
      nd.unary[nd.n] = -std::log(phi);
      ++nd.n;
    }
  }
  // messages into node i from its neighbour in direction d (0 up, 1 left, 2 right, 3 down)
  std::vector<double> msg((size_t)N * 4 * kMaxLab, 0.0);
  auto nbr = [&](int i, int d) -> int {
    const int x = i % W, y = i / W;
    switch (d) {
      case 0: return y > 0 ? i - W : -1;
      case 1: return x > 0 ? i - 1 : -1;
      case 2: return x + 1 < W ? i + 1 : -1;
      default: return y + 1 < H ? i + W : -1;
    }
  };
  auto opposite = [](int d) { return 3 - d; };
  auto M = [&](int i, int d) -> double* { return &msg[((size_t)i * 4 + d) * kMaxLab]; };
  // a neighbour takes part when it has states; gamma = 1 / max(#earlier, #later) neighbours
  std::vector<double> gamma(N, 1.0);
  for (int i = 0; i < N; ++i) {
    if (!nodes[i].n) continue;
    int before = 0, after = 0;
    for (int d = 0; d < 4; ++d) {
      const int j = nbr(i, d);
      if (j < 0 || !nodes[j].n) continue;
      (d < 2 ? before : after)++;
    }
    const int m = std::max(before, after);
    gamma[i] = m > 0 ? 1.0 / m : 1.0;
  }
  auto belief = [&](int i, double* b) {
    const Node& nd = nodes[i];
    for (int l = 0; l < nd.n; ++l) b[l] = nd.unary[l];
    for (int d = 0; d < 4; ++d) {
      const int j = nbr(i, d);
      if (j < 0 || !nodes[j].n) continue;
      const double* m = M(i, d);
      for (int l = 0; l < nd.n; ++l) b[l] += m[l];
    }
  };
  // send the message i -> j (j is neighbour d of i)
  auto send = [&](int i, int d, const double* b) {
    const int j = nbr(i, d);
    const Node& ni = nodes[i];
    const Node& nj = nodes[j];
    const double* back = M(i, d);  // message j -> i
    double* out = M(j, opposite(d));
    double lo = std::numeric_limits<double>::infinity();
    for (int m = 0; m < nj.n; ++m) {
      double best = std::numeric_limits<double>::infinity();
      for (int l = 0; l < ni.n; ++l) {
        const double v = gamma[i] * b[l] - back[l] + edge_energy(ni.value[l], nj.value[m], k3);
        best = std::min(best, v);
      }
      out[m] = best;
      lo = std::min(lo, best);
    }
    for (int m = 0; m < nj.n; ++m) out[m] -= lo;
  };
  double b[kMaxLab];
  for (int it = 0; it < iterations; ++it) {
    for (int i = 0; i < N; ++i) {  // forward: to the right and down neighbours
      if (!nodes[i].n) continue;
      belief(i, b);
      for (int d = 2; d < 4; ++d) {
        const int j = nbr(i, d);
        if (j >= 0 && nodes[j].n) send(i, d, b);
      }
    }
    for (int i = N - 1; i >= 0; --i) {  // backward: to the up and left neighbours
      if (!nodes[i].n) continue;
      belief(i, b);
      for (int d = 0; d < 2; ++d) {
        const int j = nbr(i, d);
        if (j >= 0 && nodes[j].n) send(i, d, b);
      }
    }
  }
  // decode in order: earlier neighbours contribute their chosen state, later ones their messages
  std::vector<int> pick(N, -1);
  for (int i = 0; i < N; ++i) {
    const Node& nd = nodes[i];
    label_out[i] = -1;
    depth_out[i] = 0.0f;
    if (!nd.n) continue;
    double best = std::numeric_limits<double>::infinity();
    int arg = 0;
    for (int l = 0; l < nd.n; ++l) {
      double e = nd.unary[l];
      for (int d = 0; d < 4; ++d) {
        const int j = nbr(i, d);
        if (j < 0 || !nodes[j].n) continue;
        if (d < 2)
          e += edge_energy(nodes[j].value[pick[j]], nd.value[l], k3);
        else
          e += M(i, d)[l];
      }
      if (e < best) {
        best = e;
        arg = l;
      }
    }
    pick[i] = arg;
    label_out[i] = nd.label[arg];
    depth_out[i] = (float)nd.value[arg];
  }
  return PHIMVS_OK;
}
