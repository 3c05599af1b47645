"""Pins of the depth-map fusion oracle (Sec. III-F) against closed forms and invariants:
a lone map is its own back-projection; two identical maps merge pixel for pixel into the
first; a half-resolution copy from the same camera centre maps 2x2 pixels onto one, so
the first of them in row-major order takes it and the Euclidean threshold decides at a
distance known in closed form (half a pixel diagonally); and on random multi-view maps
every pixel with depth ends in exactly one point (support is conserved), each merged
pixel within the threshold of its point's first pixel."""
import numpy as np
import pytest

import oracle


def cam(f, W, H, centre=(0.0, 0.0, 0.0), yaw=0.0):
    K = np.array([[f, 0.0, (W - 1) / 2.0], [0.0, f, (H - 1) / 2.0], [0.0, 0.0, 1.0]])
    c, s = np.cos(yaw), np.sin(yaw)
    R = np.array([[c, 0.0, -s], [0.0, 1.0, 0.0], [s, 0.0, c]])
    t = -R @ np.asarray(centre, np.float64)
    return K, R, t


def stack(cams):
    return (np.stack([c[0] for c in cams]), np.stack([c[1] for c in cams]), np.stack([c[2] for c in cams]))


def back_project(K, R, t, depth):
    """World points of every pixel, closed form: X_c = d ((x - cx)/f, (y - cy)/f, 1), X_w = R^T (X_c - t)."""
    H, W = depth.shape
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    d = depth.astype(np.float64)
    Xc = np.stack([d * (x - K[0, 2]) / K[0, 0], d * (y - K[1, 2]) / K[1, 1], d], -1)
    return (Xc - t) @ R  # row vectors: (R^T v)^T = v^T R


def random_depth(r, H, W, lo=3.0, hi=5.0, holes=0.2):
    d = r.uniform(lo, hi, (H, W)).astype(np.float32)
    d[r.uniform(size=(H, W)) < holes] = 0.0
    return d


@pytest.mark.parametrize("yaw,centre", [(0.0, (0.0, 0.0, 0.0)), (0.3, (1.0, -2.0, 0.5))])
def test_single_map_is_its_back_projection(yaw, centre):
    r = np.random.default_rng(1)
    W, H = 23, 17
    K, R, t = cam(40.0, W, H, centre, yaw)
    d = random_depth(r, H, W)
    pts, sup, own = oracle.fuse([d], K[None], R[None], t[None])
    has = d.ravel() > 0
    exp = back_project(K, R, t, d).reshape(-1, 3)
    assert np.allclose(pts[has], exp[has], rtol=1e-6, atol=1e-6)
    assert np.all(pts[~has] == 0)
    assert np.array_equal(sup, has.astype(np.int32))
    assert np.array_equal(own, np.where(has, np.arange(W * H), -1))


def test_identical_maps_merge_into_the_first():
    r = np.random.default_rng(2)
    W, H = 31, 19
    K, R, t = stack([cam(50.0, W, H, (0.2, 0.1, -0.3), 0.1)] * 2)
    d = random_depth(r, H, W)
    pts, sup, own = oracle.fuse([d, d], K, R, t)
    has = d.ravel() > 0
    n = W * H
    # the mean of a point with itself is the point: the first map's back-projections exactly
    alone, _, _ = oracle.fuse([d], K[:1], R[:1], t[:1])
    assert np.array_equal(pts[:n], alone)
    assert np.array_equal(sup[:n], 2 * has.astype(np.int32))
    assert np.all(sup[n:] == 0) and np.all(pts[n:] == 0)
    idx = np.arange(n)
    assert np.array_equal(own[:n], np.where(has, idx, -1))
    assert np.array_equal(own[n:], np.where(has, idx, -1))
    # the order of the maps decides which one keeps the points
    _, sup2, _ = oracle.fuse([d, d], K[::-1], R[::-1], t[::-1])
    assert np.array_equal(sup2[:n], 2 * has.astype(np.int32))


@pytest.mark.parametrize("tau,merged", [(0.01, True), (0.0071, True), (0.0070, False), (0.004, False)])
def test_half_resolution_copy_first_in_row_major_order_wins(tau, merged):
    """Map 1 is the same camera at half resolution (f/2, same centre); a fronto-parallel
    plane at Z on both.  Map 0's pixel (x, y) lands at ((x - 1/2)/2, (y - 1/2)/2) in map 1,
    so pixels (2k..2k+1, 2m..2m+1) all round to (k, m), and (2k, 2m) comes first.  Map 1's
    pixel (k, m) is map 0's position (2k + 1/2, 2m + 1/2): half a pixel away on both axes,
    a distance of Z sqrt(1/2) / f = 0.00707 Z at f = 100."""
    W, H, f, Z = 40, 24, 100.0, 4.0
    K0, R0, t0 = cam(f, W, H)
    K1, R1, t1 = cam(f / 2, W // 2, H // 2)
    d0 = np.full((H, W), Z, np.float32)
    d1 = np.full((H // 2, W // 2), Z, np.float32)
    pts, sup, own = oracle.fuse([d0, d1], np.stack([K0, K1]), np.stack([R0, R1]), np.stack([t0, t1]), tau)
    n0 = W * H
    assert (np.sqrt(0.5) / f < tau) == merged
    s0 = sup[:n0].reshape(H, W)
    if merged:
        exp = np.ones((H, W), np.int32)
        exp[0::2, 0::2] = 2
        assert np.array_equal(s0, exp)
        assert np.all(sup[n0:] == 0)
        k, m = np.meshgrid(np.arange(W // 2), np.arange(H // 2))
        assert np.array_equal(own[n0:].reshape(H // 2, W // 2), (2 * m) * W + 2 * k)
        # the merged point is the midpoint of the two back-projections
        a = back_project(K0, R0, t0, d0)[0::2, 0::2].reshape(-1, 3)
        b = back_project(K1, R1, t1, d1).reshape(-1, 3)
        assert np.allclose(pts[:n0].reshape(H, W, 3)[0::2, 0::2].reshape(-1, 3), (a + b) / 2, rtol=1e-6, atol=1e-6)
    else:
        assert np.all(s0 == 1) and np.all(sup[n0:] == 1)


@pytest.mark.parametrize("shape", [(0, 5), (5, 0)])
def test_a_map_without_pixels_is_refused(shape):
    K, R, t = stack([cam(40.0, 5, 5), cam(40.0, 5, 5)])
    with pytest.raises(ValueError):
        oracle.fuse([np.ones((5, 5), np.float32), np.ones(shape, np.float32)], K, R, t)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_support_is_conserved_on_random_views(seed):
    """Five cameras on an arc looking at a noisy plane, maps with holes: every pixel with
    depth ends in exactly one point, each point's support counts the pixels that name it
    as owner, a pixel is only ever merged into a point of an earlier map (or its own
    pixel), and each merged pixel lies within the threshold of the point's first pixel."""
    r = np.random.default_rng(seed)
    W, H, f, tau = 36, 28, 40.0, 0.01
    cams, depths = [], []
    for v in range(5):
        a = 0.06 * (v - 2)
        centre = (4.0 * np.sin(a), 0.05 * v, 4.0 - 4.0 * np.cos(a))
        K, R, t = cam(f, W, H, centre, a)
        # a plane z = 4 in the world, seen by each camera, with 0.3% depth noise
        y, x = np.mgrid[0:H, 0:W].astype(np.float64)
        ray = np.stack([(x - K[0, 2]) / f, (y - K[1, 2]) / f, np.ones_like(x)], -1) @ R  # world direction
        C = -R.T @ t
        lam = (4.0 - C[2]) / ray[..., 2]
        d = (lam * (1 + 0.003 * r.standard_normal((H, W)))).astype(np.float32)
        d[r.uniform(size=(H, W)) < 0.15] = 0.0
        cams.append((K, R, t))
        depths.append(d)
    K, R, t = stack(cams)
    pts, sup, own = oracle.fuse(depths, K, R, t, tau)
    has = np.concatenate([d.ravel() > 0 for d in depths])
    assert sup.sum() == has.sum()
    assert np.all(own[~has] == -1) and np.all(own[has] >= 0)
    counts = np.bincount(own[has], minlength=len(own))
    assert np.array_equal(counts, sup)
    idx = np.arange(len(own))
    assert np.all(own[has] <= idx[has])
    assert np.all(sup[own[has]] >= 1)
    X = np.concatenate([back_project(*cams[v], depths[v]).reshape(-1, 3) for v in range(5)])
    dep = np.concatenate([d.ravel() for d in depths]).astype(np.float64)
    m = has & (own != idx)
    dist = np.linalg.norm(X[m] - X[own[m]], axis=1)
    assert np.all(dist < tau * dep[own[m]] * (1 + 1e-9))
    assert m.sum() > 0.2 * has.sum()  # the views overlap: many pixels merge
    # each point is the mean of the pixels it holds
    for g in np.flatnonzero(sup > 1)[:50]:
        assert np.allclose(pts[g], X[own == g].mean(0), rtol=1e-6, atol=1e-6)
