"""Pins of the plane-hypothesis-inference oracle (Sec. III-E): the line fits reproduce
affine depth exactly in all four directions and equal numpy's least-squares fit on the
six closest samples; the exact MAP agrees with hand-worked chains; the TRW decoder is
exact on chains, forests and loopy grids with binary submodular energies, reduces to
closed forms where its messages are fixed or absent, and is near the exact MAP on other
small loopy grids; the normals of Eq. 10 equal the normal of the
plane a depth map was rendered from."""
import itertools
import math

import numpy as np
import pytest

import binary_mincut
import oracle

DIRS = [(1, 0), (0, 1), (1, 1), (1, -1)]


@pytest.mark.parametrize("k", range(4))
def test_affine_depth_is_reproduced_in_its_direction(k):
    H, W = 21, 23
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    dx, dy = DIRS[k]
    # depth affine along direction k (constant across it): the fit is exact
    d = (3.0 + 0.05 * (xx * dx + yy * dy)).astype(np.float32)
    holes = np.zeros((H, W), bool)
    holes[8:13, 6:15] = True
    dm = d.copy()
    dm[holes] = 0.0
    hyp = oracle.phi_hypotheses(dm)
    got = hyp[..., k][holes]
    np.testing.assert_allclose(got, d[holes].astype(np.float64), rtol=1e-6)
    assert np.all(hyp[~holes] == 0)  # pixels with depth get no hypotheses


def test_six_closest_samples_and_numpy_fit():
    W = 40
    d = np.zeros((1, W), np.float32)
    r = np.random.default_rng(0)
    valid = [2, 5, 11, 13, 17, 18, 30, 33]
    d[0, valid] = r.uniform(2, 6, len(valid)).astype(np.float32)
    x = 15
    hyp = oracle.phi_hypotheses(d)
    # closest valid samples to x = 15 by |s| (negative side first on ties): 13 (2), 17 (2), 18 (3), 11 (4), 5 (10), 2 (13)
    pts = [13, 17, 18, 11, 5, 2]
    s = np.array(pts, np.float64) - x
    coef = np.polyfit(s, d[0, pts].astype(np.float64), 1)
    assert np.isclose(hyp[0, x, 0], np.polyval(coef, 0.0), rtol=1e-6)
    # the vertical and diagonal lines of a single row see nothing
    assert np.all(hyp[0, :, 1:] == 0)


@pytest.mark.parametrize("k", range(4))
def test_tie_at_the_sixth_sample_takes_the_negative_side(k):
    """Samples at steps -1, +1, -2, +2, -3, -4, +4 along direction k: the six closest
    are those up to |s| = 3 and then -4 (the negative side first on the tie at 4), so
    the fit equals numpy's on exactly those six; step +s is (x + s dx, y + s dy)."""
    dx, dy = DIRS[k]
    H = W = 21
    x0 = y0 = 10
    steps = [-1, 1, -2, 2, -3, -4, 4]
    r = np.random.default_rng(k)
    vals = r.uniform(2.0, 6.0, len(steps)).astype(np.float32)
    d = np.zeros((H, W), np.float32)
    for st, v in zip(steps, vals):
        d[y0 + st * dy, x0 + st * dx] = v
    hyp = oracle.phi_hypotheses(d)
    take = steps[:6]
    coef = np.polyfit(np.array(take, np.float64), vals[:6].astype(np.float64), 1)
    assert np.isclose(hyp[y0, x0, k], np.polyval(coef, 0.0), rtol=1e-6)
    # with +4 instead of -4 the value differs, so the tie order is what decides it
    alt = np.polyfit(np.array(steps[:5] + [4], np.float64), np.r_[vals[:5], vals[6]].astype(np.float64), 1)
    assert not np.isclose(np.polyval(alt, 0.0), np.polyval(coef, 0.0), rtol=1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_line_fits_match_brute_force_up_to_the_borders(seed):
    """Every hypothesis of small maps with half the pixels empty, where most lines reach an
    image border (row 0 and column 0 included): walk steps -1, +1, -2, +2, ... along the
    direction, keep the samples inside the image with depth, take the first six, and fit
    a straight line with numpy (no hypothesis below two samples or for a fit <= 0)."""
    r = np.random.default_rng(100 + seed)
    H, W = 9, 11
    d = r.uniform(1.0, 9.0, (H, W)).astype(np.float32)
    d[r.random((H, W)) < 0.5] = 0.0
    hyp = oracle.phi_hypotheses(d)
    for y in range(H):
        for x in range(W):
            for k, (dx, dy) in enumerate(DIRS):
                if d[y, x] > 0:
                    assert hyp[y, x, k] == 0
                    continue
                take = []
                for step in itertools.chain.from_iterable((-m, m) for m in range(1, max(H, W) + 1)):
                    xs, ys = x + step * dx, y + step * dy
                    if 0 <= xs < W and 0 <= ys < H and d[ys, xs] > 0 and len(take) < 6:
                        take.append((step, float(d[ys, xs])))
                if len(take) < 2:
                    assert hyp[y, x, k] == 0
                    continue
                st, dv = np.array(take).T
                v = np.polyval(np.polyfit(st, dv, 1), 0.0)
                if v <= 0:
                    assert hyp[y, x, k] == 0
                else:
                    assert np.isclose(hyp[y, x, k], v, rtol=1e-6), (y, x, k, take)


def test_negative_and_nan_depths_are_holes():
    r = np.random.default_rng(4)
    d = r.uniform(1.0, 9.0, (15, 17)).astype(np.float32)
    d[r.uniform(size=d.shape) < 0.5] = 0.0
    bad = d.copy()
    neg = r.uniform(size=d.shape) < 0.1
    nan = (r.uniform(size=d.shape) < 0.1) & ~neg
    bad[neg & (d == 0)] = -2.0
    bad[nan & (d == 0)] = np.nan
    assert np.array_equal(oracle.phi_hypotheses(bad), oracle.phi_hypotheses(d))


def test_too_few_samples_or_negative_fit_give_no_hypothesis():
    d = np.zeros((1, 20), np.float32)
    d[0, 3] = 4.0
    assert np.all(oracle.phi_hypotheses(d)[0, :, 0] == 0)  # one sample only
    d[0, 4] = 1.0  # the line through (3, 4) and (4, 1): 13 - 3 x, zero at x = 13/3
    h = oracle.phi_hypotheses(d)[0, :, 0]
    assert np.isclose(h[0], 13.0, rtol=1e-6) and np.isclose(h[2], 7.0, rtol=1e-6)
    assert np.all(h[5:] == 0)  # not positive there


def test_map_on_chains_matches_enumeration():
    """Exact MAP on 1 x 3 chains against an enumeration written out here."""
    r = np.random.default_rng(1)
    k1, k2, k3 = 1.0, 0.1, 2.0
    for trial in range(20):
        d = np.zeros((1, 3), np.float32)
        if trial % 3 == 0:
            d[0, 0] = 3.0  # a fixed node
        hyp = r.uniform(2, 5, (1, 3, 4)).astype(np.float32)
        hyp[d > 0] = 0
        hyp[0, 1, 3] = 0  # a missing state
        cost = r.uniform(0, 2, (1, 3, 4)).astype(np.float32)
        lab, e = oracle.phi_map_bruteforce(d, hyp, cost, k1, k2, k3)

        def states(i):
            if d[0, i] > 0:
                return [(-1, float(d[0, i]), 0.0)]
            return [(k, float(hyp[0, i, k]), np.log((2.0 - float(cost[0, i, k])) / k1 + k2)) for k in range(4)
                    if hyp[0, i, k] > 0]

        def pw(a, b):
            rel = (a - b) / b if a > b else (b - a) / a
            return np.log((k3 - min(1.0, rel)) ** 2)

        best = max(itertools.product(states(0), states(1), states(2)),
                   key=lambda c: c[0][2] + c[1][2] + c[2][2] + pw(c[0][1], c[1][1]) + pw(c[1][1], c[2][1]))
        val = best[0][2] + best[1][2] + best[2][2] + pw(best[0][1], best[1][1]) + pw(best[1][1], best[2][1])
        assert np.isclose(e, val, rtol=1e-12)
        assert list(lab[0]) == [c[0] for c in best]


def test_map_ties_take_the_first_labelling_in_enumeration_order():
    """Two hypotheses of a node with the same depth and cost tie under every labelling of
    the others: the enumeration (node 0 varying fastest, states in order of k) keeps the
    first maximal labelling, so the lower k."""
    d = np.zeros((1, 3), np.float32)
    d[0, 0] = 3.0
    hyp = np.zeros((1, 3, 4), np.float32)
    hyp[0, 1] = [0.0, 3.5, 2.0, 3.5]
    hyp[0, 2] = [2.5, 0.0, 0.0, 4.0]
    cost = np.full((1, 3, 4), 0.4, np.float32)
    lab, _ = oracle.phi_map_bruteforce(d, hyp, cost, 1.0, 0.1, 2.0)
    assert lab[0, 0] == -1 and lab[0, 1] == 1


def test_map_on_a_grid_matches_enumeration():
    """Exact MAP on 2 x 3 grids (right and down edges) against an enumeration written out
    here; hypotheses over [1, 6] so that relative differences above 1 (the truncation of
    Eq. 8) occur; k3 = 2 and 2.5; some grids with a node that has no hypothesis (isolated)."""
    r = np.random.default_rng(2)
    k1, k2 = 1.0, 0.1
    H, W = 2, 3
    for trial in range(16):
        k3 = 2.0 if trial % 2 == 0 else 2.5
        d = np.zeros((H, W), np.float32)
        if trial % 4 == 0:
            d[1, 2] = 2.5  # a fixed node
        hyp = r.uniform(1, 6, (H, W, 4)).astype(np.float32)
        hyp[r.random((H, W, 4)) < 0.4] = 0  # missing states
        hyp[d > 0] = 0
        hyp[0, 0, 0] = 1.2
        if trial % 3 == 1:
            hyp[1, 0] = 0  # a free node without any hypothesis: isolated from the model
        cost = r.uniform(0, 2, (H, W, 4)).astype(np.float32)
        lab, e = oracle.phi_map_bruteforce(d, hyp, cost, k1, k2, k3)

        def states(y, x):
            if d[y, x] > 0:
                return [(-1, float(d[y, x]), 0.0)]
            s_ = [(k, float(hyp[y, x, k]), np.log((2.0 - float(cost[y, x, k])) / k1 + k2)) for k in range(4)
                  if hyp[y, x, k] > 0]
            return s_ or [(-1, 0.0, 0.0)]

        def pw(a, b):
            if a <= 0 or b <= 0:
                return 0.0  # an edge to an isolated node carries nothing
            rel = (a - b) / b if a > b else (b - a) / a
            return np.log((k3 - min(1.0, rel)) ** 2)

        nodes = [(y, x) for y in range(H) for x in range(W)]
        edges = [(i, j) for i, (y, x) in enumerate(nodes) for j, (y2, x2) in enumerate(nodes)
                 if (y2 == y and x2 == x + 1) or (x2 == x and y2 == y + 1)]

        def energy(c):
            return sum(s[2] for s in c) + sum(pw(c[i][1], c[j][1]) for i, j in edges)

        best = max(itertools.product(*[states(y, x) for y, x in nodes]), key=energy)
        assert np.isclose(e, energy(best), rtol=1e-12)
        assert list(lab.ravel()) == [s[0] for s in best]


def _log_potential(d, hyp, cost, lab, k1, k2, k3, cmax=2.0):
    """Sum of log potentials of a labelling (-1: the fixed depth, or no state)."""
    H, W = d.shape

    def value(y, x):
        if d[y, x] > 0:
            return float(d[y, x])
        return float(hyp[y, x, lab[y, x]]) if lab[y, x] >= 0 else 0.0

    e = 0.0
    for y in range(H):
        for x in range(W):
            if d[y, x] <= 0 and lab[y, x] >= 0:
                e += math.log((cmax - float(cost[y, x, lab[y, x]])) / k1 + k2)
            for yy, xx in ((y, x + 1), (y + 1, x)):
                if yy < H and xx < W and value(y, x) > 0 and value(yy, xx) > 0:
                    a, b = value(y, x), value(yy, xx)
                    rel = (a - b) / b if a > b else (b - a) / a
                    e += math.log((k3 - min(1.0, rel)) * (k3 - min(1.0, rel)))
    return e


def _random_model(r, H, W, fixed=0.25, missing=0.3, lo=1.0, hi=6.0):
    d = np.where(r.random((H, W)) < fixed, r.uniform(lo, hi, (H, W)), 0.0).astype(np.float32)
    hyp = r.uniform(lo, hi, (H, W, 4)).astype(np.float32)
    hyp[r.random((H, W, 4)) < missing] = 0
    hyp[d > 0] = 0
    cost = r.uniform(0, 2, (H, W, 4)).astype(np.float32)
    return d, hyp, cost


@pytest.mark.parametrize("shape", [(1, 2), (1, 5), (1, 8), (6, 1)])
def test_trws_is_exact_on_chains(shape):
    """A chain is a tree, on which sequential TRW decodes the exact MAP (Kolmogorov 2006):
    its labelling reaches the enumerated optimum's log potential; depths follow the labels."""
    r = np.random.default_rng(shape[1] * 10 + shape[0])
    k2 = 0.1
    for trial in range(15):
        k3 = 2.0 if trial % 2 else 2.5
        k1 = (0.5, 1.0, 2.0)[trial % 3]
        d, hyp, cost = _random_model(r, *shape)
        lab, val = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=10)
        _, e_opt = oracle.phi_map_bruteforce(d, hyp, cost, k1, k2, k3)
        assert np.isclose(_log_potential(d, hyp, cost, lab, k1, k2, k3), e_opt, rtol=1e-9, atol=1e-12)
        picked = np.take_along_axis(hyp, np.maximum(lab, 0)[..., None], 2)[..., 0]
        expect = np.where(d > 0, d, np.where(lab >= 0, picked, 0.0))
        assert np.array_equal(val, expect.astype(np.float32))
        assert np.all(lab[d > 0] == -1)


def _is_forest(alive):
    """The 4-connected graph of the True cells has no cycle."""
    H, W = alive.shape
    parent = {c: c for c in zip(*np.nonzero(alive))}

    def root(c):
        while parent[c] != c:
            c = parent[c]
        return c

    for y, x in list(parent):
        for c2 in ((y, x + 1), (y + 1, x)):
            if c2 in parent:
                a, b = root((y, x)), root(c2)
                if a == b:
                    return False
                parent[a] = b
    return True


def test_trws_is_exact_on_forests_in_any_raster_order():
    """Grids whose nodes with states form a forest (the others have neither depth nor
    hypotheses): TRW decodes the exact MAP there too.  Unlike chains, such trees bend back
    against the raster order (a node can have both its upper and its left neighbour in the
    model), so messages in both sweeps and both directions are needed; k1 varies."""
    r = np.random.default_rng(14)
    k2, k3 = 0.1, 2.0
    tested = 0
    for trial in range(300):
        alive = r.random((3, 4)) < 0.7
        if alive.sum() < 5 or not _is_forest(alive):
            continue
        k1 = (0.5, 1.0, 2.0)[trial % 3]
        d = np.where((r.random((3, 4)) < 0.2) & alive, r.uniform(1, 6, (3, 4)), 0.0).astype(np.float32)
        hyp = r.uniform(1, 6, (3, 4, 4)).astype(np.float32)
        hyp[r.random((3, 4, 4)) < 0.4] = 0
        hyp[(d > 0) | ~alive] = 0
        cost = r.uniform(0, 2, (3, 4, 4)).astype(np.float32)
        lab, _ = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=10)
        _, e_opt = oracle.phi_map_bruteforce(d, hyp, cost, k1, k2, k3)
        assert np.isclose(_log_potential(d, hyp, cost, lab, k1, k2, k3), e_opt, rtol=1e-9, atol=1e-12)
        tested += 1
    assert tested >= 60


def test_trws_ties_go_to_the_first_state():
    """Two hypotheses of a node with the same depth and cost score the same under every
    message: the lower k is taken, with and without message passing."""
    r = np.random.default_rng(15)
    for iters in (0, 1, 4):
        d, hyp, cost = _random_model(r, 5, 6, fixed=0.3, missing=0.0)
        free = np.argwhere(d <= 0)
        for y, x in free:
            hyp[y, x, 3] = hyp[y, x, 1]
            cost[y, x, 3] = cost[y, x, 1]
            hyp[y, x, 0] = 0.0  # state order: 1, 2, 3
        lab, _ = oracle.phi_trws(d, hyp, cost, 0.7, 0.1, 2.0, iterations=iters)
        assert not (lab == 3).any()
        assert ((lab == 1) | (lab == 2))[d <= 0].all()


def test_trws_free_nodes_between_fixed_ones():
    """Free nodes whose neighbours all have a fixed depth (or no state) are independent:
    after any number of iterations each takes the state with the highest product of its
    potential and its edge potentials to the fixed neighbours."""
    r = np.random.default_rng(11)
    k1, k2, k3 = 1.7, 0.1, 2.0
    H, W = 7, 9
    for trial in range(6):
        yy, xx = np.mgrid[0:H, 0:W]
        d = np.where((yy + xx) % 2 == 0, r.uniform(1, 6, (H, W)), 0.0).astype(np.float32)
        hyp = r.uniform(1, 6, (H, W, 4)).astype(np.float32)
        hyp[r.random((H, W, 4)) < 0.3] = 0
        hyp[d > 0] = 0
        if trial % 2:
            d[3, 4] = 0.0  # a node with neither depth nor hypotheses: no state
            hyp[3, 4] = 0
        cost = r.uniform(0, 2, (H, W, 4)).astype(np.float32)
        for iters in (1, 3):
            lab, _ = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=iters)
            for y in range(H):
                for x in range(W):
                    if d[y, x] > 0 or not (hyp[y, x] > 0).any():
                        continue
                    score = {}
                    for k in np.nonzero(hyp[y, x] > 0)[0]:
                        h = float(hyp[y, x, k])
                        e = math.log((2.0 - float(cost[y, x, k])) / k1 + k2)
                        for y2, x2 in ((y - 1, x), (y, x - 1), (y, x + 1), (y + 1, x)):
                            if 0 <= y2 < H and 0 <= x2 < W and d[y2, x2] > 0:
                                a = float(d[y2, x2])
                                rel = (a - h) / h if a > h else (h - a) / a
                                e += math.log((k3 - min(1.0, rel)) ** 2)
                        score[k] = e
                    best = max(score.values())
                    assert np.isclose(score[lab[y, x]], best, rtol=1e-12), (y, x, score, lab[y, x])


def test_trws_without_iterations_labels_greedily():
    """With no message passing the decoding is greedy in raster order: each node takes the
    state with the highest product of its potential and the edge potentials to the states
    already chosen for its upper and left neighbours (first state on ties)."""
    r = np.random.default_rng(12)
    k1, k2, k3 = 0.6, 0.1, 2.5
    H, W = 6, 7
    for _ in range(5):
        d, hyp, cost = _random_model(r, H, W)
        lab, val = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=0)
        chosen = np.zeros((H, W))
        for y in range(H):
            for x in range(W):
                if d[y, x] > 0:
                    chosen[y, x] = d[y, x]
                    assert lab[y, x] == -1
                    continue
                ks = [k for k in range(4) if hyp[y, x, k] > 0]
                if not ks:
                    assert lab[y, x] == -1 and val[y, x] == 0
                    continue
                best_k, best_e = None, None
                for k in ks:
                    h = float(hyp[y, x, k])
                    e = math.log((2.0 - float(cost[y, x, k])) / k1 + k2)
                    for y2, x2 in ((y - 1, x), (y, x - 1)):
                        if y2 >= 0 and x2 >= 0 and chosen[y2, x2] > 0:
                            a = chosen[y2, x2]
                            rel = (a - h) / h if a > h else (h - a) / a
                            e += math.log((k3 - min(1.0, rel)) ** 2)
                    if best_e is None or e > best_e:
                        best_k, best_e = k, e
                assert lab[y, x] == best_k
                chosen[y, x] = hyp[y, x, best_k]


def test_trws_on_small_loopy_grids():
    """On 3 x 3 grids (loops) TRW is an approximation: its labelling never beats the
    enumerated optimum, reaches it in most cases and stays close otherwise."""
    r = np.random.default_rng(13)
    k1, k2, k3 = 1.0, 0.1, 2.0
    gaps = []
    for _ in range(25):
        d, hyp, cost = _random_model(r, 3, 3, fixed=0.2, missing=0.15, lo=2.0, hi=5.0)
        lab, _ = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=20)
        _, e_opt = oracle.phi_map_bruteforce(d, hyp, cost, k1, k2, k3)
        e = _log_potential(d, hyp, cost, lab, k1, k2, k3)
        assert e <= e_opt + 1e-9
        gaps.append((e_opt - e) / abs(e_opt))
    gaps = np.array(gaps)
    assert (gaps < 1e-9).mean() >= 0.8
    assert gaps.max() < 0.05


def test_trws_is_exact_on_binary_submodular_loopy_grids():
    """Loopy grids whose free nodes hold two hypotheses, one near 2.1 and one near 3.9 in
    depth, so that every edge between two such nodes is submodular (the two same-side pairs
    cost no more together than the two mixed pairs): for such binary energies TRW reaches
    the global minimum (Kolmogorov and Wainwright, UAI 2005), so the decoding must equal the
    enumerated optimum although the graph has cycles.  Greedy decoding misses it on most of
    these instances; decoders that over-count beliefs (gamma = 1, plain max-product, or
    gamma = m instead of 1/m) miss it on some."""
    r = np.random.default_rng(21)
    greedy_misses = 0
    n = 120
    for trial in range(n):
        H, W = [(3, 4), (4, 4), (4, 3), (2, 6)][trial % 4]
        k1, k2, k3 = (0.5, 1.0, 2.0)[trial % 3], 0.1, (2.5, 2.0)[trial % 2]
        d = np.where(r.random((H, W)) < 0.1, r.uniform(1.5, 4.5, (H, W)), 0.0).astype(np.float32)
        hyp = np.zeros((H, W, 4), np.float32)
        hyp[..., 0] = r.uniform(2.0, 2.3, (H, W))
        hyp[..., 1] = r.uniform(3.6, 4.2, (H, W))
        hyp[d > 0] = 0
        cost = r.uniform(0, 2, (H, W, 4)).astype(np.float32)

        def e_pair(a, b):
            rel = (a - b) / b if a > b else (b - a) / a
            return -math.log((k3 - min(1.0, rel)) ** 2)

        for y in range(H):
            for x in range(W):
                for yy, xx in ((y, x + 1), (y + 1, x)):
                    if yy < H and xx < W and d[y, x] <= 0 and d[yy, xx] <= 0:
                        a, b = hyp[y, x].astype(float), hyp[yy, xx].astype(float)
                        assert e_pair(a[0], b[0]) + e_pair(a[1], b[1]) <= e_pair(a[0], b[1]) + e_pair(a[1], b[0])
        _, e_opt = oracle.phi_map_bruteforce(d, hyp, cost, k1, k2, k3)
        lab, _ = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=30)
        assert np.isclose(_log_potential(d, hyp, cost, lab, k1, k2, k3), e_opt, rtol=1e-9, atol=1e-12), trial
        lab0, _ = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=0)
        greedy_misses += not np.isclose(_log_potential(d, hyp, cost, lab0, k1, k2, k3), e_opt, rtol=1e-9, atol=1e-12)
    assert greedy_misses >= n // 3


@pytest.mark.parametrize("shape,iters", [((20, 20), 30), ((16, 24), 30), ((12, 30), 30), ((30, 30), 30),
                                         ((100, 100), 100)])
def test_trws_reaches_the_min_cut_minimum_on_larger_binary_submodular_grids(shape, iters):
    """Grids too large to enumerate, with the two-cluster hypotheses of the test above: the
    exact minimum is a minimum s-t cut (Kolmogorov and Zabih 2004, computed with scipy's
    maximum flow, written in the tests), and TRW reaches it within the given sweeps.  A
    decoder with smaller weights (the right neighbour counted as earlier) falls short here
    within these sweeps."""
    r = np.random.default_rng(shape[0] * 100 + shape[1])
    for trial in range(2):
        k1, k2, k3 = (0.5, 1.0, 2.0)[trial % 3], 0.1, (2.5, 2.0)[trial % 2]
        d, hyp, cost = binary_mincut.two_cluster_problem(r, *shape)
        terms = binary_mincut.energy_terms(d, hyp, cost, k1, k2, k3)
        e_mc = binary_mincut.energy(terms, binary_mincut.min_cut_labels(terms, shape))
        lab, _ = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=iters)
        e = binary_mincut.energy(terms, lab)
        assert e_mc - 1e-3 <= e <= e_mc + 1e-6, (e, e_mc)
        lab0, _ = oracle.phi_trws(d, hyp, cost, k1, k2, k3, iterations=0)
        assert binary_mincut.energy(terms, lab0) > e_mc + 1.0  # greedy decoding is far from it


def test_normals_of_a_rendered_plane():
    H, W, f = 30, 40, 50.0
    K = np.array([[f, 0, (W - 1) / 2], [0, f, (H - 1) / 2], [0, 0, 1.0]])
    n = np.array([0.3, -0.2, -1.0])
    n /= np.linalg.norm(n)
    c = 5.0  # plane n . X = -c  (points in front of the camera)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    rays = np.stack([xx, yy, np.ones_like(xx)], -1) @ np.linalg.inv(K).T
    depth = (-c / (rays @ n)) * rays[..., 2]  # Z of the ray-plane intersection
    dm = depth.astype(np.float32)
    dm[10, 10] = 0.0
    out = oracle.phi_normals(dm, K)
    inner = np.zeros((H, W), bool)
    inner[1:-1, 1:-1] = True
    inner[9:12, 9:12] = False  # the hole and its 4-neighbours
    inner[10, 10] = False
    np.testing.assert_allclose(out[inner], np.broadcast_to(n, (inner.sum(), 3)), atol=2e-5)
    assert np.all(out[10, 10] == 0) and np.all(out[0] == 0) and np.all(out[10, 11] == 0)
    # the hole's 4-neighbours and the image's border rows and columns get no normal
    for yy_, xx_ in ((9, 10), (11, 10), (10, 9), (10, 11)):
        assert np.all(out[yy_, xx_] == 0)
    assert np.all(out[-1] == 0) and np.all(out[:, 0] == 0) and np.all(out[:, -1] == 0)
