// Host-side selection step of plane hypothesis inference (PHI-MVS Sec. III-E): the
// pairwise undirected graph model over a 4-connected pixel grid, decoded by sequential
// tree-reweighted message passing (TRW-S, Kolmogorov 2006).  The paper runs this part on
// the CPU; so does the library.  Potentials: node states are a pixel's depth hypotheses
// with phi_n = (C_max - C) / k1 + k2 (Eq. 7), pixels that already have depth are fixed
// single-state nodes (phi = 1), edges carry phi_e = [k3 - min(1, relative difference)]^2
// (Eq. 8); decoding maximises the product, i.e. minimises the sum of -log potentials.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <functional>
#include <limits>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "phimvs.h"

namespace {

constexpr int kMaxLab = 4;
constexpr unsigned kMaxThreads = 16;

// symmetric in its arguments, bit for bit: (h1, h2) and (h2, h1) take the same branch values
double edge_energy(double h1, double h2, double k3) {
  const double rel = h1 > h2 ? (h1 - h2) / h2 : (h2 - h1) / h1;
  const double m = rel < 1.0 ? rel : 1.0;
  return -std::log((k3 - m) * (k3 - m));
}

unsigned worker_count(size_t nodes) {
  if (nodes < 8192) return 1;
  const unsigned hw = std::thread::hardware_concurrency();
  return std::max(1u, std::min(hw, kMaxThreads));
}

// Host threads kept for one decoding: run(f) runs f on every member, the calling thread
// included, and returns once all have finished it.  Members wait for the next job by
// yielding.  If a thread cannot be started the team is smaller; every job below shares its
// work through counters, so any team size gives the same result.
class Team {
 public:
  explicit Team(unsigned want) {
    for (unsigned t = 1; t < want; ++t) {
      try {
        th_.emplace_back([this] { member(); });
      } catch (...) {
        break;
      }
    }
    n_ = (unsigned)th_.size() + 1;
    ready_.store(true, std::memory_order_release);
  }
  ~Team() {
    stop_ = true;
    gen_.fetch_add(1, std::memory_order_release);
    for (auto& x : th_) x.join();
  }
  Team(const Team&) = delete;
  Team& operator=(const Team&) = delete;
  unsigned size() const { return n_; }
  void run(const std::function<void()>& f) {
    job_ = &f;
    done_.store(0, std::memory_order_relaxed);
    gen_.fetch_add(1, std::memory_order_release);
    f();
    while (done_.load(std::memory_order_acquire) != n_ - 1) std::this_thread::yield();
  }

 private:
  void member() {
    while (!ready_.load(std::memory_order_acquire)) std::this_thread::yield();
    unsigned seen = 0;
    for (;;) {
      unsigned g;
      while ((g = gen_.load(std::memory_order_acquire)) == seen) std::this_thread::yield();
      seen = g;
      if (stop_) return;
      (*job_)();
      done_.fetch_add(1, std::memory_order_acq_rel);
    }
  }
  std::vector<std::thread> th_;
  unsigned n_ = 1;
  std::atomic<bool> ready_{false};
  std::atomic<unsigned> gen_{0}, done_{0};
  bool stop_ = false;
  const std::function<void()>* job_ = nullptr;
};

// f(y0, y1) over blocks of rows
template <class F>
void parallel_rows(Team& team, int H, F&& f) {
  std::atomic<int> next{0};
  team.run([&] {
    for (;;) {
      const int y = next.fetch_add(16);
      if (y >= H) break;
      f(y, std::min(H, y + 16));
    }
  });
}

// The tiles of the sweep schedule: 32 x 64 nodes, halved (down to 8 x 16) until each
// anti-diagonal of tiles can hold two per thread
struct Tiling {
  int th = 32, tw = 64, nx = 0, ny = 0;
  std::vector<int> order;  // tiles by anti-diagonal
  Tiling(int W, int H, unsigned T) {
    for (;;) {
      nx = (W + tw - 1) / tw;
      ny = (H + th - 1) / th;
      if (th <= 8 || (unsigned)std::min(nx, ny) >= 2 * T) break;
      th /= 2;
      tw /= 2;
    }
    order.reserve((size_t)nx * ny);
    for (int s = 0; s < nx + ny - 1; ++s)
      for (int ty = 0; ty < ny; ++ty)
        if (s - ty >= 0 && s - ty < nx) order.push_back(ty * nx + (s - ty));
  }
};

// visit(i) for every node of a W x H grid, each after its left and upper neighbours
// (forward) or after its right and lower neighbours (backward): tiles are handed out by
// anti-diagonal, a tile starts once the tiles it borders in that direction are done, and
// inside a tile the nodes go in raster (reverse raster) order
template <class F>
void wavefront(Team& team, const Tiling& tl, int W, int H, bool forward, F&& visit) {
  const int n_tiles = tl.nx * tl.ny;
  std::unique_ptr<std::atomic<int>[]> done(new std::atomic<int>[n_tiles]);
  for (int t = 0; t < n_tiles; ++t) done[t].store(0, std::memory_order_relaxed);
  std::atomic<int> next{0};
  const int dir = forward ? -1 : 1;
  team.run([&] {
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n_tiles) break;
      const int t = forward ? tl.order[k] : tl.order[n_tiles - 1 - k];
      const int tx = t % tl.nx, ty = t / tl.nx;
      // those tiles come earlier in the hand-out order, so someone already holds them
      if (tx + dir >= 0 && tx + dir < tl.nx)
        while (!done[ty * tl.nx + tx + dir].load(std::memory_order_acquire)) std::this_thread::yield();
      if (ty + dir >= 0 && ty + dir < tl.ny)
        while (!done[(ty + dir) * tl.nx + tx].load(std::memory_order_acquire)) std::this_thread::yield();
      const int x0 = tx * tl.tw, x1 = std::min(W, x0 + tl.tw);
      const int y0 = ty * tl.th, y1 = std::min(H, y0 + tl.th);
      if (forward) {
        for (int y = y0; y < y1; ++y)
          for (int x = x0; x < x1; ++x) visit(y * W + x);
      } else {
        for (int y = y1 - 1; y >= y0; --y)
          for (int x = x1 - 1; x >= x0; --x) visit(y * W + x);
      }
      done[t].store(1, std::memory_order_release);
    }
  });
}

}  // namespace

// Sequential TRW-S visits the nodes in raster order (forward sweep: each node sends to its
// right and lower neighbours) and then in reverse raster order (backward sweep: to its upper
// and left neighbours).  In a forward sweep a node reads the messages its left and upper
// neighbours sent in the same sweep and those its right and lower neighbours sent in the
// previous backward sweep, which nothing in between rewrites; so any order that visits a
// node after its left and upper neighbours computes the same messages, bit for bit, as the
// raster order (likewise for the backward sweep and for the final decoding, which reads the
// choices of the left and upper neighbours).  These passes run as wavefronts of tiles on
// several threads.  The edge energies are computed once per edge (they do not change), and a
// message into a node with a single state is 0 after its normalisation, whatever was sent.
extern "C" int phimvs_phi_decode_host(int width, int height, const float* depth, const float* hyp, const float* cost,
                                      double k1, double k2, double k3, double cost_max, int iterations,
                                      int32_t* label_out, float* depth_out) {
  if (width < 1 || height < 1 || !depth || !hyp || !cost || !label_out || !depth_out) return PHIMVS_E_ARG;
  if (!(k1 > 0) || !(k2 > 0) || !(k3 > 1) || iterations < 0) return PHIMVS_E_ARG;
  if ((int64_t)width * height > INT32_MAX / 16) return PHIMVS_E_UNSUPPORTED;
  try {
    const int W = width, H = height, N = W * H;
    const size_t plane = (size_t)N;
    Team team(worker_count(plane));
    const Tiling tiling(W, H, team.size());
    // node i: ns[i] states (0: not part of the model); state l: hypothesis lab (-1: the
    // fixed depth), depth val, unary -log phi_n
    std::vector<uint8_t> ns(N, 0), live(N, 0);
    std::vector<int8_t> lab((size_t)N * kMaxLab);
    std::vector<double> val((size_t)N * kMaxLab), un((size_t)N * kMaxLab);
    std::atomic<bool> bad{false};
    parallel_rows(team, H, [&](int y0, int y1) {
      for (int i = y0 * W; i < y1 * W; ++i) {
        const size_t q = (size_t)i * kMaxLab;
        if (depth[i] > 0.0f) {
          ns[i] = 1;
          lab[q] = -1;
          val[q] = depth[i];
          un[q] = 0.0;
          continue;
        }
        int n = 0;
        for (int k = 0; k < kMaxLab; ++k) {
          const float h = hyp[k * plane + i];
          if (!(h > 0.0f)) continue;
          const double phi = (cost_max - (double)cost[k * plane + i]) / k1 + k2;
          if (!(phi > 0.0)) bad.store(true, std::memory_order_relaxed);
          lab[q + n] = (int8_t)k;
          val[q + n] = h;
          un[q + n] = -std::log(phi);
          ++n;
        }
        ns[i] = (uint8_t)n;
      }
    });
    if (bad.load()) return PHIMVS_E_ARG;  // a node potential that is not positive
    // live[i] bit d: neighbour d (0 up, 1 left, 2 right, 3 down) exists and has states;
    // gamma = 1 / max(#earlier, #later) such neighbours; the energies of the edge to the
    // right (er) and the one below (ed) of node i, indexed [state of i][state of the
    // neighbour], laid out row after row
    const int step[4] = {-W, -1, 1, W};
    std::vector<double> gamma(N, 1.0);
    std::vector<int64_t> er(N, -1), ed(N, -1), row_start(H + 1, 0);
    parallel_rows(team, H, [&](int y0, int y1) {
      for (int y = y0; y < y1; ++y) {
        int64_t count = 0;
        for (int x = 0, i = y * W; x < W; ++x, ++i) {
          if (!ns[i]) continue;
          const bool has[4] = {y > 0 && ns[i - W], x > 0 && ns[i - 1], x + 1 < W && ns[i + 1],
                               y + 1 < H && ns[i + W]};
          int before = 0, after = 0;
          for (int d = 0; d < 4; ++d) {
            if (!has[d]) continue;
            live[i] |= (uint8_t)(1 << d);
            (d < 2 ? before : after)++;
          }
          // no energy is needed between two single-state nodes: no message goes into one,
          // and one decodes to its only state
          if (has[2] && ns[i] * ns[i + 1] > 1) er[i] = count, count += ns[i] * ns[i + 1];
          if (has[3] && ns[i] * ns[i + W] > 1) ed[i] = count, count += ns[i] * ns[i + W];
          const int m = std::max(before, after);
          gamma[i] = m > 0 ? 1.0 / m : 1.0;
        }
        row_start[y + 1] = count;
      }
    });
    for (int y = 0; y < H; ++y) row_start[y + 1] += row_start[y];
    std::unique_ptr<double[]> energy(new double[(size_t)row_start[H]]);
    parallel_rows(team, H, [&](int y0, int y1) {
      for (int y = y0; y < y1; ++y)
        for (int i = y * W; i < (y + 1) * W; ++i)
          for (int d = 2; d < 4; ++d) {
            int64_t& o = d == 2 ? er[i] : ed[i];
            if (o < 0) continue;
            o += row_start[y];
            const int j = i + step[d];
            for (int l = 0; l < ns[i]; ++l)
              for (int m = 0; m < ns[j]; ++m)
                energy[o + l * ns[j] + m] = edge_energy(val[(size_t)i * kMaxLab + l], val[(size_t)j * kMaxLab + m], k3);
          }
    });
    // E(i in state l, j in state m) for the edge from i to its neighbour j in direction d:
    // e[l * sl + m * sm]
    auto edge = [&](int i, int j, int d, const double*& e, int& sl, int& sm) {
      if (d >= 2) {
        e = &energy[d == 2 ? er[i] : ed[i]];
        sl = ns[j];
        sm = 1;
      } else {
        e = &energy[d == 1 ? er[j] : ed[j]];
        sl = 1;
        sm = ns[i];
      }
    };
    // messages into node i from its neighbour in direction d; those into a single-state
    // node are never written (they stay 0)
    std::unique_ptr<double[]> msg(new double[(size_t)N * 4 * kMaxLab]);
    parallel_rows(team, H, [&](int y0, int y1) {
      std::fill(&msg[(size_t)y0 * W * 4 * kMaxLab], &msg[(size_t)y1 * W * 4 * kMaxLab], 0.0);
    });
    auto M = [&](int i, int d) -> double* { return &msg[((size_t)i * 4 + d) * kMaxLab]; };
    // the belief of node i, then its messages to the neighbours in directions d0, d0 + 1.
    // A single-state node's belief is its unary term plus zeros, and what it sends depends
    // on nothing else: its messages are the same in every sweep, so it only sends in the
    // first sweep of each direction.
    auto update = [&](int i, int d0, bool first) {
      const int n = ns[i];
      if (!n || (n == 1 && !first)) return;
      double b[kMaxLab];
      for (int l = 0; l < n; ++l) b[l] = un[(size_t)i * kMaxLab + l];
      for (int d = 0; d < 4; ++d) {
        if (!(live[i] >> d & 1)) continue;
        if (n == 1) {
          b[0] += 0.0;
          continue;
        }
        const double* m = M(i, d);
        for (int l = 0; l < n; ++l) b[l] += m[l];
      }
      for (int d = d0; d < d0 + 2; ++d) {
        if (!(live[i] >> d & 1)) continue;
        const int j = i + step[d], nj = ns[j];
        if (nj == 1) continue;
        double* out = M(j, 3 - d);
        const double* back = M(i, d);  // message j -> i
        const double* e;
        int sl, sm;
        edge(i, j, d, e, sl, sm);
        double a[kMaxLab];
        for (int l = 0; l < n; ++l) a[l] = gamma[i] * b[l] - back[l];
        double lo = std::numeric_limits<double>::infinity();
        for (int m = 0; m < nj; ++m) {
          double best = std::numeric_limits<double>::infinity();
          for (int l = 0; l < n; ++l) best = std::min(best, a[l] + e[l * sl + m * sm]);
          out[m] = best;
          lo = std::min(lo, best);
        }
        for (int m = 0; m < nj; ++m) out[m] -= lo;
      }
    };
    for (int it = 0; it < iterations; ++it) {
      wavefront(team, tiling, W, H, true, [&](int i) { update(i, 2, it == 0); });
      wavefront(team, tiling, W, H, false, [&](int i) { update(i, 0, it == 0); });
    }
    // decode in order: earlier neighbours contribute their chosen state, later ones their messages
    std::vector<int8_t> pick(N, -1);
    wavefront(team, tiling, W, H, true, [&](int i) {
      label_out[i] = -1;
      depth_out[i] = 0.0f;
      const int n = ns[i];
      if (!n) return;
      if (n == 1) {
        pick[i] = 0;
        label_out[i] = lab[(size_t)i * kMaxLab];
        depth_out[i] = (float)val[(size_t)i * kMaxLab];
        return;
      }
      double best = std::numeric_limits<double>::infinity();
      int arg = 0;
      for (int l = 0; l < n; ++l) {
        double e = un[(size_t)i * kMaxLab + l];
        for (int d = 0; d < 4; ++d) {
          if (!(live[i] >> d & 1)) continue;
          if (d < 2) {
            const int j = i + step[d];
            const double* ee;
            int sl, sm;
            edge(i, j, d, ee, sl, sm);
            e += ee[l * sl + pick[j] * sm];
          } else {
            e += M(i, d)[l];
          }
        }
        if (e < best) {
          best = e;
          arg = l;
        }
      }
      pick[i] = (int8_t)arg;
      label_out[i] = lab[(size_t)i * kMaxLab + arg];
      depth_out[i] = (float)val[(size_t)i * kMaxLab + arg];
    });
  } catch (const std::bad_alloc&) {
    return PHIMVS_E_OOM;
  } catch (...) {
    return PHIMVS_E_UNSUPPORTED;
  }
  return PHIMVS_OK;
}
