"""Pins of the plane-hypothesis-inference oracle (Sec. III-E): the line fits reproduce
affine depth exactly in all four directions and equal numpy's least-squares fit on the
six closest samples; the exact MAP agrees with hand-worked chains; the normals of Eq. 10
equal the normal of the plane a depth map was rendered from."""
import itertools

import numpy as np
import pytest

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
