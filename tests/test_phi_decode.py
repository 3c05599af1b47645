"""The library's host-side graph-model decoder of plane hypothesis inference (Sec. III-E;
the paper runs it on the CPU, so does the library) against the oracle's exact MAP on
tiny grids: exact on chains (a tree, where sequential tree-reweighted message passing
is exact), on loopy grids with binary submodular energies (where TRW is exact too), and
on other small loopy grids equal to the optimum or within a small margin of it;
and against the oracle's plain sequential TRW decoder bit for bit on grids large enough
for the library's threaded tile schedule, with fixed and single-state nodes, ragged tile
edges and several iteration counts.  No GPU needed: the decoder takes host arrays."""
import numpy as np
import pytest

import binary_mincut
import oracle
import paper_2104_06165_amd as pm


def log_potential(depth, hyp, cost, labels, k1, k2, k3, cmax=2.0):
    """Sum of log potentials of a labelling (-1: the fixed depth)."""
    H, W = depth.shape

    def value(y, x):
        l = labels[y, x]
        if depth[y, x] > 0:
            return float(depth[y, x])
        return float(hyp[y, x, l]) if l >= 0 else 0.0

    e = 0.0
    for y in range(H):
        for x in range(W):
            l = labels[y, x]
            if depth[y, x] <= 0 and l >= 0:
                e += np.log((cmax - float(cost[y, x, l])) / k1 + k2)
            v = value(y, x)
            for yy, xx in ((y, x + 1), (y + 1, x)):
                if yy < H and xx < W:
                    u = value(yy, xx)
                    if v > 0 and u > 0:
                        rel = (v - u) / u if v > u else (u - v) / v
                        e += np.log((k3 - min(1.0, rel)) ** 2)
    return e


def random_problem(r, H, W, fixed_frac=0.2, missing_frac=0.15):
    depth = np.where(r.uniform(size=(H, W)) < fixed_frac, r.uniform(2, 5, (H, W)), 0.0).astype(np.float32)
    hyp = r.uniform(2, 5, (H, W, 4)).astype(np.float32)
    hyp[r.uniform(size=(H, W, 4)) < missing_frac] = 0.0
    hyp[depth > 0] = 0.0
    cost = r.uniform(0, 2, (H, W, 4)).astype(np.float32)
    return depth, hyp, cost


@pytest.mark.parametrize("W", [2, 4, 7])
def test_decoder_is_exact_on_chains(W):
    r = np.random.default_rng(W)
    k1, k2, k3 = 1.0, 0.1, 2.0
    for _ in range(15):
        depth, hyp, cost = random_problem(r, 1, W)
        lab_o, e_o = oracle.phi_map_bruteforce(depth, hyp, cost, k1, k2, k3)
        lab, dep = pm.phi_decode_host(depth, hyp.transpose(2, 0, 1), cost.transpose(2, 0, 1),
                                      pm.PhiParams(k1, k2, k3, 10))
        e = log_potential(depth, hyp, cost, lab, k1, k2, k3)
        assert np.isclose(e, e_o, rtol=1e-9, atol=1e-12), (e, e_o)
        # depths follow the labels
        exp = np.where(depth > 0, depth, np.take_along_axis(hyp, np.maximum(lab, 0)[..., None], 2)[..., 0])
        exp = np.where((depth <= 0) & (lab < 0), 0.0, exp)
        assert np.allclose(dep, exp)


def test_decoder_on_small_loopy_grids():
    r = np.random.default_rng(7)
    k1, k2, k3 = 1.0, 0.1, 2.0
    gaps = []
    for _ in range(25):
        depth, hyp, cost = random_problem(r, 3, 3)
        _, e_o = oracle.phi_map_bruteforce(depth, hyp, cost, k1, k2, k3)
        lab, _ = pm.phi_decode_host(depth, hyp.transpose(2, 0, 1), cost.transpose(2, 0, 1), pm.PhiParams(k1, k2, k3, 20))
        e = log_potential(depth, hyp, cost, lab, k1, k2, k3)
        assert e <= e_o + 1e-9  # never above the exact optimum (sanity of both)
        gaps.append((e_o - e) / abs(e_o))
    gaps = np.array(gaps)
    assert (gaps < 1e-9).mean() >= 0.8  # the optimum itself in most cases
    assert gaps.max() < 0.05


@pytest.mark.parametrize("shape", [(100, 100), (120, 160)])
def test_decoder_reaches_the_min_cut_minimum_on_large_binary_submodular_grids(shape):
    """Sizes that run the decoder's threaded tile schedule, two hypotheses per free node
    (every free-free edge submodular): 100 sweeps reach the exact minimum, a minimum s-t
    cut computed in the tests (Kolmogorov and Zabih 2004, scipy's maximum flow)."""
    r = np.random.default_rng(shape[1])
    k1, k2, k3 = 0.5, 0.1, 2.5
    d, hyp, cost = binary_mincut.two_cluster_problem(r, *shape)
    terms = binary_mincut.energy_terms(d, hyp, cost, k1, k2, k3)
    e_mc = binary_mincut.energy(terms, binary_mincut.min_cut_labels(terms, shape))
    lab, _ = pm.phi_decode_host(d, hyp.transpose(2, 0, 1), cost.transpose(2, 0, 1), pm.PhiParams(k1, k2, k3, 100))
    e = binary_mincut.energy(terms, lab)
    assert e_mc - 1e-3 <= e <= e_mc + 1e-6, (e, e_mc)


def test_decoder_is_exact_on_binary_submodular_loopy_grids():
    """Loopy grids whose free nodes hold one hypothesis near each of two depths (every edge
    between two of them submodular): there TRW reaches the global minimum (Kolmogorov and
    Wainwright, UAI 2005), so the decoder must give the enumerated optimum."""
    r = np.random.default_rng(22)
    for trial in range(40):
        H, W = [(3, 4), (4, 4), (4, 3), (2, 6)][trial % 4]
        k1, k2, k3 = (0.5, 1.0, 2.0)[trial % 3], 0.1, (2.5, 2.0)[trial % 2]
        depth = np.where(r.uniform(size=(H, W)) < 0.1, r.uniform(1.5, 4.5, (H, W)), 0.0).astype(np.float32)
        hyp = np.zeros((H, W, 4), np.float32)
        hyp[..., 0] = r.uniform(2.0, 2.3, (H, W))
        hyp[..., 1] = r.uniform(3.6, 4.2, (H, W))
        hyp[depth > 0] = 0.0
        cost = r.uniform(0, 2, (H, W, 4)).astype(np.float32)
        _, e_o = oracle.phi_map_bruteforce(depth, hyp, cost, k1, k2, k3)
        lab, _ = pm.phi_decode_host(depth, hyp.transpose(2, 0, 1), cost.transpose(2, 0, 1), pm.PhiParams(k1, k2, k3, 30))
        assert np.isclose(log_potential(depth, hyp, cost, lab, k1, k2, k3), e_o, rtol=1e-9, atol=1e-12), trial


def test_decoder_arguments():
    d = np.zeros((2, 2), np.float32)
    h = np.zeros((4, 2, 2), np.float32)
    with pytest.raises(pm.PhimvsError):
        pm.phi_decode_host(d, h, h, pm.PhiParams(k1=0.0))
    with pytest.raises(ValueError):
        pm.phi_decode_host(d, h[:3], h)
    lab, dep = pm.phi_decode_host(d, h, h)  # no states anywhere
    assert np.all(lab == -1) and np.all(dep == 0)


@pytest.mark.parametrize("H,W,fixed,k1,k3,iters", [
    (150, 260, 0.25, 1.0, 2.0, 8),   # several threads, ragged tiles at both edges
    (150, 260, 0.6, 0.5, 2.5, 3),    # mostly fixed nodes, as in filtered maps
    (33, 1000, 0.3, 1.0, 2.0, 1),    # one and a bit tile rows
    (1000, 9, 0.3, 2.0, 1.5, 2),     # a single tile column
    (129, 193, 0.0, 1.0, 2.0, 0),    # no message passing: the greedy raster decoding
    (520, 1030, 0.6, 1.0, 2.0, 2),   # large enough for the largest tiles on 8 threads
])
def test_decoder_equals_the_oracle_trws(H, W, fixed, k1, k3, iters):
    r = np.random.default_rng(H * 7 + W)
    depth = np.where(r.uniform(size=(H, W)) < fixed, r.uniform(2, 5, (H, W)), 0.0).astype(np.float32)
    hyp = r.uniform(2, 5, (H, W, 4)).astype(np.float32)
    hyp[r.uniform(size=(H, W, 4)) < 0.3] = 0.0
    hyp[depth > 0] = 0.0
    single = r.uniform(size=(H, W)) < 0.05  # nodes left with one hypothesis
    hyp[single, 1:] = 0.0
    cost = r.uniform(0, 2, (H, W, 4)).astype(np.float32)
    lab_o, dep_o = oracle.phi_trws(depth, hyp, cost, k1, 0.1, k3, iterations=iters)
    lab, dep = pm.phi_decode_host(depth, hyp.transpose(2, 0, 1), cost.transpose(2, 0, 1),
                                  pm.PhiParams(k1, 0.1, k3, iters))
    assert np.array_equal(lab, lab_o), f"{(lab != lab_o).sum()} labels differ"
    assert np.array_equal(dep, dep_o)


def test_decoder_rejects_a_potential_that_is_not_positive():
    """A cost above C_max + k1 k2 makes (C_max - C) / k1 + k2 negative: no valid potential."""
    d = np.zeros((2, 2), np.float32)
    h = np.full((4, 2, 2), 3.0, np.float32)
    c = np.zeros((4, 2, 2), np.float32)
    c[2, 1, 1] = 2.5
    with pytest.raises(pm.PhimvsError):
        pm.phi_decode_host(d, h, c)
