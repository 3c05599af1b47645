"""Exact minimum of the plane-hypothesis graph model (Sec. III-E) when every node without a
fixed depth holds exactly two hypotheses (k = 0 and 1) and every edge between two such
nodes is submodular: a minimum s-t cut of the graph of Kolmogorov and Zabih (PAMI 2004),
computed by scipy's maximum flow on capacities scaled to integers.  Test code, independent
of the oracle."""
import math

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import breadth_first_order, maximum_flow


def energy_terms(depth, hyp, cost, k1, k2, k3, cmax=2.0):
    """-log potentials: unary U[node] = [E(k=0), E(k=1)] for the free nodes (fixed
    neighbours folded in), pairwise V[(p, q)] 2 x 2 between free nodes, and the constant
    of the fixed-fixed edges."""
    H, W = depth.shape

    def e_pair(a, b):
        rel = (a - b) / b if a > b else (b - a) / a
        return -math.log((k3 - min(1.0, rel)) ** 2)

    U = {(y, x): [-math.log((cmax - float(cost[y, x, s])) / k1 + k2) for s in (0, 1)]
         for y in range(H) for x in range(W) if depth[y, x] <= 0}
    V, const = {}, 0.0
    for y in range(H):
        for x in range(W):
            for yy, xx in ((y, x + 1), (y + 1, x)):
                if yy >= H or xx >= W:
                    continue
                p, q = (y, x), (yy, xx)
                if p in U and q in U:
                    V[(p, q)] = [[e_pair(float(hyp[y, x, s]), float(hyp[yy, xx, t])) for t in (0, 1)] for s in (0, 1)]
                elif p in U:
                    for s in (0, 1):
                        U[p][s] += e_pair(float(hyp[y, x, s]), float(depth[yy, xx]))
                elif q in U:
                    for t in (0, 1):
                        U[q][t] += e_pair(float(depth[y, x]), float(hyp[yy, xx, t]))
                else:
                    const += e_pair(float(depth[y, x]), float(depth[yy, xx]))
    return U, V, const


def energy(terms, labels):
    """Energy of a labelling (labels[y, x] in {0, 1} at the free nodes)."""
    U, V, const = terms
    e = const + sum(U[n][int(labels[n])] for n in U)
    return e + sum(V[(p, q)][int(labels[p])][int(labels[q])] for (p, q) in V)


def min_cut_labels(terms, shape, scale=1e7):
    """Labels (H, W) of a minimum cut (-1 at fixed nodes): the source side takes k = 0.
    A pairwise term A, B, C, D (A + D <= B + C) is A + (C - A) x_p + (D - C) x_q +
    (B + C - A - D)(1 - x_p) x_q, the last one an edge p -> q."""
    U, V, _ = terms
    nodes = list(U)
    idx = {n: i + 2 for i, n in enumerate(nodes)}  # 0 source, 1 sink
    a = {n: list(U[n]) for n in nodes}
    cap = {}

    def add(u, v, c):
        if c > 0:
            cap[(u, v)] = cap.get((u, v), 0) + int(round(c * scale))

    for (p, q), M in V.items():
        A, B, C, D = M[0][0], M[0][1], M[1][0], M[1][1]
        assert A + D <= B + C + 1e-12, "not submodular"
        a[p][1] += C - A
        a[q][1] += D - C
        add(idx[p], idx[q], B + C - A - D)
    for n in nodes:
        if a[n][1] > a[n][0]:
            add(0, idx[n], a[n][1] - a[n][0])
        else:
            add(idx[n], 1, a[n][0] - a[n][1])
    N = len(nodes) + 2
    rows, cols, vals = zip(*[(u, v, c) for (u, v), c in cap.items()])
    G = csr_matrix((np.array(vals, np.int32), (rows, cols)), shape=(N, N))
    F = maximum_flow(G, 0, 1).flow
    R = (G.astype(np.int64) - F.astype(np.int64)).tocsr()  # the flow is skew-symmetric
    R.data[R.data < 0] = 0
    R.eliminate_zeros()
    seen = np.zeros(N, bool)
    seen[breadth_first_order(R, 0, directed=True, return_predecessors=False)] = True
    lab = np.full(shape, -1, np.int32)
    for n in nodes:
        lab[n] = 0 if seen[idx[n]] else 1
    return lab


def two_cluster_problem(rng, H, W, fixed=0.1):
    """Free nodes with one hypothesis near 2.1 and one near 3.9 (every free-free edge is
    then submodular), 10% fixed nodes, random costs."""
    depth = np.where(rng.random((H, W)) < fixed, rng.uniform(1.5, 4.5, (H, W)), 0.0).astype(np.float32)
    hyp = np.zeros((H, W, 4), np.float32)
    hyp[..., 0] = rng.uniform(2.0, 2.3, (H, W))
    hyp[..., 1] = rng.uniform(3.6, 4.2, (H, W))
    hyp[depth > 0] = 0
    cost = rng.uniform(0, 2, (H, W, 4)).astype(np.float32)
    return depth, hyp, cost
