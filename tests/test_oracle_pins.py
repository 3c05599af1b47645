"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each check is a closed form, an
invariant, a library routine on a special case, a published known-answer vector, or
brute force on a tiny input.
"""
import math
import os

import numpy as np
import pytest
import scipy.stats

import oracle
import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- helpers
def _K(w, h, f=None, dcx=0.0, dcy=0.0):
    f = 0.9 * w if f is None else f
    return np.array([[f, 0, (w - 1) / 2 + dcx], [0, f, (h - 1) / 2 + dcy], [0, 0, 1.0]])


def _textured(h, w, seed):
    rng = np.random.default_rng(seed)
    base = rng.integers(20, 236, size=(h, w)).astype(np.float32)
    # mild smoothing keeps it band-limited but textured; round to integers (8-bit data)
    sm = (base + np.roll(base, 1, 0) + np.roll(base, 1, 1) + np.roll(base, (1, 1), (0, 1))) / 4
    return np.round(sm).astype(np.float32)


def _pose_problem(images, Ks, Rs=None, ts=None, window=7, dilation=1, top_k=0, bilateral=False, **kw):
    n = len(images)
    Rs = [np.eye(3)] * n if Rs is None else Rs
    ts = [np.zeros(3)] * n if ts is None else ts
    return oracle.Problem(images, np.stack(Ks), np.stack(Rs), np.stack(ts), (1.0, 10.0), window, dilation,
                          top_k, bilateral=bilateral, **kw)


def _fronto(h, w, d=4.0):
    planes = np.zeros((h, w, 4))
    planes[..., 2] = -1.0
    planes[..., 3] = d
    return planes


def _rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


# ----------------------------------------------------------------------------- Philox
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# ----------------------------------------------------------------------------- ZNCC (Eq. 4)
@pytest.mark.parametrize("bilateral", [False, True])
def test_identical_patches_give_zero_cost(bilateral):
    h, w = 24, 28
    A = _textured(h, w, 1)
    K = _K(w, h)
    pb = _pose_problem([A, A, A], [K, K, K], window=7, bilateral=bilateral, top_k=0)
    cost, pv, ok = oracle.eval_cost(pb, _fronto(h, w), fp64=False)
    m = pb.valid_mask()
    assert ok[m].all()
    assert np.all(pv[m] == 0.0)  # Z = 1 exactly
    # Eq. 5 with C_j floored at eps_c: n / (n / eps_c) = eps_c
    assert np.all(cost[m] == np.float32(1e-4))
    assert np.all(cost[~m] == oracle.CMAX)


@pytest.mark.parametrize("alpha,beta,z", [(2.0, -40.0, 1.0), (0.37, 11.5, 1.0), (-1.5, 300.0, -1.0)])
@pytest.mark.parametrize("bilateral", [False, True])
def test_source_affine_invariance(alpha, beta, z, bilateral):
    h, w = 20, 22
    A = _textured(h, w, 2)
    B = (alpha * A + beta).astype(np.float32)
    K = _K(w, h)
    pb = _pose_problem([A, B], [K, K], window=7, bilateral=bilateral)
    _, pv, ok = oracle.eval_cost(pb, _fronto(h, w), fp64=True)
    m = pb.valid_mask()
    assert ok[m].all()
    np.testing.assert_allclose(1.0 - pv[m][:, 0], z, atol=1e-12)


def test_reference_offset_invariance_with_bilateral_weights():
    h, w = 20, 22
    A = _textured(h, w, 3)
    B = _textured(h, w, 4)
    K = _K(w, h)
    c0 = oracle.eval_cost(_pose_problem([A, B], [K, K], bilateral=True), _fronto(h, w), fp64=True)[1]
    c1 = oracle.eval_cost(_pose_problem([A + 17.0, B], [K, K], bilateral=True), _fronto(h, w), fp64=True)[1]
    np.testing.assert_allclose(c0, c1, atol=1e-12)


def test_zncc_bounded_and_symmetric():
    h, w = 22, 26
    A = _textured(h, w, 5)
    B = _textured(h, w, 6)
    K = _K(w, h)
    # one pixel of margin: windows that touch the image edge exactly may round outside it
    m = _pose_problem([A, B], [K, K]).valid_mask()
    m[[3, -4], :] = False
    m[:, [3, -4]] = False
    _, ab, okab = oracle.eval_cost(_pose_problem([A, B], [K, K]), _fronto(h, w), fp64=True)
    _, ba, okba = oracle.eval_cost(_pose_problem([B, A], [K, K]), _fronto(h, w), fp64=True)
    assert okab[m].all() and okba[m].all()
    assert np.all((ab[m] >= 0) & (ab[m] <= 2))  # |Z| <= 1 (Cauchy-Schwarz)
    np.testing.assert_allclose(ab[m], ba[m], atol=1e-12)  # w = 1: Z(a, b) = Z(b, a)


@pytest.mark.parametrize("dilation,window", [(1, 7), (2, 9), (3, 7)])
@pytest.mark.parametrize("bilateral", [False, True])
@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_zncc_matches_library_correlation(dilation, window, bilateral, lanes):
    """Integer-translation homography: the warped window is a shifted dilated window of the
    source, so 1 - C_j must be numpy's (weighted) Pearson correlation of the two patches,
    however the source-side tap sums are split over lanes."""
    h, w = 40, 44
    A = _textured(h, w, 7)
    B = _textured(h, w, 8)
    D = 3
    K0 = _K(w, h)
    Kj = _K(w, h, dcx=D)
    sig_s, sig_c = 4.0, 12.0
    pb = _pose_problem([A, B], [K0, Kj], window=window, dilation=dilation, bilateral=bilateral,
                       sigma_s=sig_s, sigma_c=sig_c, lanes=lanes)
    _, pv, ok = oracle.eval_cost(pb, _fronto(h, w), fp64=True)
    R = (window - 1) // (2 * dilation)
    ks = np.arange(-R, R + 1) * dilation
    rng = np.random.default_rng(0)
    r = dilation * R
    checked = 0
    for _ in range(40):
        x = int(rng.integers(r, w - r - D))
        y = int(rng.integers(r, h - r))
        a = A[np.ix_(y + ks, x + ks)].astype(np.float64).ravel()
        b = B[np.ix_(y + ks, x + D + ks)].astype(np.float64).ravel()
        if bilateral:
            k2, k1 = np.meshgrid(ks, ks, indexing="ij")
            wt = np.exp(-((a - A[y, x]) ** 2) / (2 * sig_c ** 2)) * np.exp(-(k1.ravel() ** 2 + k2.ravel() ** 2) / (2 * sig_s ** 2))
            cv = np.cov(np.stack([a, b]), aweights=wt, bias=True)
            z = cv[0, 1] / math.sqrt(cv[0, 0] * cv[1, 1])
        else:
            z = np.corrcoef(a, b)[0, 1]
        assert ok[y, x, 0]
        assert abs((1 - pv[y, x, 0]) - z) < 1e-10
        checked += 1
    assert checked == 40


@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
def test_lane_split_sums_differ_from_one_sum_by_rounding_only(small_scene, lanes):
    """Splitting each view's tap sums over G lanes changes only the FP32 rounding: costs of
    random and ground-truth planes within 1e-5 of the single-sum costs (FP32), within 1e-12
    in FP64; identical patches still give C = 0 exactly; G not a power of two is refused."""
    sc = small_scene
    one = oracle.Problem.from_scene(sc, 7, 1, top_k=0)
    many = oracle.Problem.from_scene(sc, 7, 1, top_k=0, lanes=lanes)
    P, _ = oracle.init(one)
    gt = np.zeros(P.shape)
    gt[..., :3] = sc.gt_normal
    gt[..., 3] = sc.gt_depth
    m = one.valid_mask()
    differ = 0
    for planes in (P, gt):
        a = oracle.eval_cost(one, planes)[0][m]
        b = oracle.eval_cost(many, planes)[0][m]
        assert np.abs(a - b).max() <= 1e-5
        differ += int((a != b).sum())
        a64 = oracle.eval_cost(one, planes, fp64=True)[0][m]
        b64 = oracle.eval_cost(many, planes, fp64=True)[0][m]
        assert np.abs(a64 - b64).max() <= 1e-12
    # the split order is really taken: its FP32 rounding shows on some pixels
    assert differ > 0
    A = _textured(24, 28, 1)
    K = _K(28, 24)
    same = _pose_problem([A, A], [K, K], window=7, lanes=lanes)
    _, pv, ok = oracle.eval_cost(same, _fronto(24, 28))
    assert np.all(pv[same.valid_mask()] == 0.0)
    with pytest.raises(ValueError):
        oracle.eval_cost(oracle.Problem.from_scene(sc, 7, 1, lanes=lanes + 1 if lanes > 2 else 3), P)


def test_dilation_equals_dense_window_on_decimated_images():
    """Dilation s=2 over a (4R+1)-wide window on full-res images equals the dense
    (2R+1) window on 2x-decimated images (translation-only homography, even disparity)."""
    h, w = 48, 52
    A = _textured(h, w, 9)
    B = _textured(h, w, 10)
    D = 4
    full = _pose_problem([A, B], [_K(w, h, f=40.0), _K(w, h, f=40.0, dcx=D)], window=13, dilation=2,
                         bilateral=True, sigma_s=5.0)
    A2, B2 = A[::2, ::2].copy(), B[::2, ::2].copy()
    h2, w2 = A2.shape
    half = _pose_problem([A2, B2], [_K(w2, h2, f=20.0), _K(w2, h2, f=20.0, dcx=D // 2)], window=7, dilation=1,
                         bilateral=True, sigma_s=2.5)
    _, pv_full, ok_full = oracle.eval_cost(full, _fronto(h, w), fp64=True)
    _, pv_half, ok_half = oracle.eval_cost(half, _fronto(h2, w2), fp64=True)
    m = half.valid_mask()
    ys, xs = np.nonzero(m)
    n = 0
    for y2, x2 in zip(ys, xs):
        y, x = 2 * y2, 2 * x2
        # skip windows touching an image edge exactly (rounding may put them outside)
        if not (6 < x and x + D + 6 < w - 1 and 6 < y < h - 7):
            continue
        assert ok_full[y, x, 0] == ok_half[y2, x2, 0]
        if ok_full[y, x, 0]:
            assert abs(pv_full[y, x, 0] - pv_half[y2, x2, 0]) < 1e-9
            n += 1
    assert n > 50


@pytest.mark.parametrize("dcx,dcy", [(6, 0), (6.5, 0), (-6.5, 0), (0, 6.5), (0, -6.5), (4.5, -3.5)])
def test_border_rule_invalidates_view(dcx, dcy):
    """A window warped by a translation (dcx, dcy) partly past the source border gives
    C_max for that view only, at exactly the pixels where a corner of the 7 x 7 window
    leaves [0, W - 1] x [0, H - 1] (each side of the image in turn), and C_max overall
    when no view is valid (paper: C_max = 1 - Z_min)."""
    h, w = 30, 40
    A = _textured(h, w, 11)
    K0 = _K(w, h)
    pb = _pose_problem([A, A, A], [K0, _K(w, h, dcx=dcx, dcy=dcy), _K(w, h, dcx=-500)], window=7)
    c, pv, ok = oracle.eval_cost(pb, _fronto(h, w), fp64=True)
    m = pb.valid_mask()
    ys, xs = np.nonzero(m)
    r = 3
    inside = (xs + dcx - r >= 0) & (xs + dcx + r <= w - 1) & (ys + dcy - r >= 0) & (ys + dcy + r <= h - 1)
    assert np.array_equal(ok[ys, xs, 0], inside)
    assert not ok[ys, xs, 1].any() and np.all(pv[ys, xs, 1] == 2.0)
    assert inside.any() and (~inside).any()
    assert np.all(c[ys[~inside], xs[~inside]] == 2.0)


# ----------------------------------------------------------------------------- homography
@pytest.mark.parametrize("kind", ["pinhole", "skew", "general"])
def test_homography_maps_plane_points_exactly(kind):
    """Points of a plane through a reference pixel's ray: the homography maps each one's
    reference projection onto its source projection.  Besides pinhole matrices, a K with
    skew and non-square pixels, and general invertible 3 x 3 matrices (every entry
    non-zero: the mapping is a projective one for any invertible K), so that every
    cofactor of the inverse matters."""
    rng = np.random.default_rng(3)
    w, h = 200, 150
    K0 = _K(w, h)
    Kj = _K(w, h, f=170.0, dcx=3.5, dcy=-2.0)
    if kind == "skew":
        K0[0, 1], K0[1, 1] = 4.3, 0.93 * K0[1, 1]
        Kj[0, 1], Kj[0, 0] = -2.1, 1.07 * Kj[0, 0]
    elif kind == "general":
        K0 = K0 + rng.normal(size=(3, 3)) * np.array([[3.0, 3.0, 3.0], [3.0, 3.0, 3.0], [1e-3, 1e-3, 0.05]])
        Kj = Kj + rng.normal(size=(3, 3)) * np.array([[3.0, 3.0, 3.0], [3.0, 3.0, 3.0], [1e-3, 1e-3, 0.05]])
        assert np.all(K0 != 0) and np.all(Kj != 0)
    R0, Rj = _rand_rot(rng), _rand_rot(rng)
    t0, tj = rng.normal(size=3), rng.normal(size=3)
    img = np.zeros((h, w), np.float32)
    pb = oracle.Problem([img, img], np.stack([K0, Kj]), np.stack([R0, Rj]), np.stack([t0, tj]), (1, 10), 7, 1)
    for _ in range(20):
        x, y = int(rng.integers(0, w)), int(rng.integers(0, h))
        n = rng.normal(size=3)
        rp = np.linalg.solve(K0, [x, y, 1.0])
        if n @ rp > 0:
            n = -n
        d = rng.uniform(2, 8)
        H = oracle.homography(pb, 0, n, d, x, y)
        Xp = d * rp  # the plane passes through this reference-camera point
        for _ in range(10):
            q = np.array([rng.uniform(0, w), rng.uniform(0, h), 1.0])
            rq = np.linalg.solve(K0, q)
            X = rq * (n @ Xp) / (n @ rq)  # ray-plane intersection, reference camera frame
            Xw = R0.T @ (X - t0)
            xj = Kj @ (Rj @ Xw + tj)
            hq = H @ q
            np.testing.assert_allclose(hq[:2] / hq[2], xj[:2] / xj[2], atol=1e-9)


def test_homography_rectified_disparity_and_identity():
    w, h = 120, 90
    f = 100.0
    K = _K(w, h, f=f)
    b, Z = 0.3, 5.0
    img = np.zeros((h, w), np.float32)
    pb = oracle.Problem([img, img], np.stack([K, K]), np.stack([np.eye(3)] * 2),
                        np.stack([np.zeros(3), np.array([-b, 0, 0])]), (1, 10), 7, 1)
    H = oracle.homography(pb, 0, np.array([0, 0, -1.0]), Z, 60, 45)
    for u, v in [(10, 20), (60, 45), (100, 80)]:
        p = H @ np.array([u, v, 1.0])
        assert abs(p[0] / p[2] - (u - f * b / Z)) < 1e-9 and abs(p[1] / p[2] - v) < 1e-9
    pb0 = oracle.Problem([img, img], np.stack([K, K]), np.stack([np.eye(3)] * 2), np.zeros((2, 3)), (1, 10), 7, 1)
    H0 = oracle.homography(pb0, 0, np.array([0.3, -0.2, -0.9]), 3.0, 10, 10)
    np.testing.assert_allclose(H0, np.eye(3), atol=1e-12)


# ----------------------------------------------------------------------------- bilinear
def test_bilinear_exact_at_integers_and_on_bilinear_functions():
    h, w = 17, 23
    img = _textured(h, w, 12)
    for y in range(h):
        for x in range(w):
            assert oracle.bilinear(img, x, y, fp64=False) == img[y, x]
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    c0, c1, c2, c3 = 7.0, 3.0, -2.0, 0.5
    f = (c0 + c1 * xx + c2 * yy + c3 * xx * yy).astype(np.float32)
    rng = np.random.default_rng(1)
    for _ in range(200):
        u, v = rng.uniform(0, w - 1), rng.uniform(0, h - 1)
        assert abs(oracle.bilinear(f, u, v, fp64=True) - (c0 + c1 * u + c2 * v + c3 * u * v)) < 1e-9


# ----------------------------------------------------------------------------- Eq. 5
def test_aggregate_closed_form():
    c = [0.2, 0.5, 0.1, 1.7]
    v = [1, 1, 1, 0]
    assert abs(oracle.aggregate(c, v, top_k=0) - scipy.stats.hmean([0.2, 0.5, 0.1])) < 1e-15
    assert abs(oracle.aggregate(c, v, top_k=2) - scipy.stats.hmean([0.1, 0.2])) < 1e-15
    assert abs(oracle.aggregate(c, [1, 1, 1, 1], top_k=1) - 0.1) < 1e-15
    assert oracle.aggregate(c, [0, 0, 0, 0]) == 2.0
    assert abs(oracle.aggregate([0.0, 0.3], [1, 1], eps_c=1e-4) - 2 / (1e4 + 1 / 0.3)) < 1e-15
    assert abs(oracle.aggregate([0.3, 0.3, 0.9], [1, 1, 1], top_k=2) - 0.3) < 1e-15
    # the FP32 form: the same values within FP32 rounding
    assert abs(oracle.aggregate(c, v, top_k=0, fp64=False) - scipy.stats.hmean([0.2, 0.5, 0.1])) < 1e-6
    assert abs(oracle.aggregate(c, v, top_k=2, fp64=False) - scipy.stats.hmean([0.1, 0.2])) < 1e-6
    assert oracle.aggregate(c, [0, 0, 0, 0], fp64=False) == 2.0


# ----------------------------------------------------------------------------- search behaviour
@pytest.fixture(scope="module")
def small_scene():
    return sg.make_scene(11, sg.tiny_config(64, 48, n_src=2, n_planes=2, n_textureless=0), device="cpu")


def test_scene_photo_consistency(small_scene):
    """Renderer pin: reference pixels re-projected through GT depth see the same intensity
    in every source (up to noise, occlusion and interpolation)."""
    sc = small_scene
    H, W = sc.gt_depth.shape
    ys, xs = np.mgrid[0:H, 0:W]
    K0 = sc.cams[0].K
    rays = np.linalg.solve(K0, np.stack([xs.ravel(), ys.ravel(), np.ones(H * W)]))
    Xc = rays * sc.gt_depth.ravel()
    Xw = sc.cams[0].R.T @ (Xc - sc.cams[0].t[:, None])
    ref = sc.images[0].ravel().astype(np.float64)
    for j in range(1, len(sc.images)):
        cj = sc.cams[j]
        p = cj.K @ (cj.R @ Xw + cj.t[:, None])
        u, v = p[0] / p[2], p[1] / p[2]
        inb = (u >= 0) & (u <= W - 1) & (v >= 0) & (v <= H - 1)
        vals = np.array([oracle.bilinear(sc.images[j], uu, vv) for uu, vv in zip(u[inb], v[inb])])
        diff = np.abs(vals - ref[inb])
        assert inb.mean() > 0.7
        assert np.median(diff) < 4.0


def test_init_distribution(small_scene):
    sc = small_scene
    pb = oracle.Problem.from_scene(sc, 7, 1)
    planes, cost = oracle.init(pb)
    m = pb.valid_mask()
    d = planes[..., 3][m]
    lo, hi = sc.depth_range
    assert d.min() >= np.float32(lo) and d.max() <= np.float32(hi)
    assert scipy.stats.kstest((d - lo) / (hi - lo), "uniform").pvalue > 1e-3
    n = planes[..., :3][m]
    ys, xs = np.nonzero(m)
    rays = np.linalg.solve(sc.cams[0].K, np.stack([xs, ys, np.ones_like(xs)]).astype(np.float64)).T
    assert np.all((n * rays).sum(1) <= 0)  # facing the camera
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-6)
    # phi uniform on [-pi/2, pi/2] => the angle to the optical axis, acos|n_z|, is uniform on [0, pi/2]
    ang = np.arccos(np.clip(np.abs(n[:, 2]), 0, 1))
    assert scipy.stats.kstest(ang / (np.pi / 2), "uniform").pvalue > 1e-3
    # theta uniform on [0, 2 pi] => the azimuth, taken modulo pi (the camera-facing flip
    # adds pi), is uniform on [0, pi)
    az = np.mod(np.arctan2(n[:, 1], n[:, 0]), np.pi)
    assert scipy.stats.kstest(az / np.pi, "uniform").pvalue > 1e-3
    c = cost[m]
    assert np.all((c >= 0) & (c <= 2))


def _uniforms(seed, x, y, W, iteration, phase):
    """The four uniforms of pixel (x, y) (reading s27), from the KAT-pinned Philox block."""
    o = oracle.philox4x32_10([y * W + x, iteration, phase, 0], [seed & 0xFFFFFFFF, seed >> 32])
    return [(int(v) >> 8) * 2.0 ** -24 for v in o]


def _facing(theta, phi, ray):
    n = np.array([math.cos(theta) * math.sin(phi), math.sin(theta) * math.sin(phi), math.cos(phi)])
    return -n if n @ ray > 0 else n


def test_draws_map_to_the_documented_initial_planes(small_scene):
    """Initialisation (Sec. III-B, readings s18 and s27), FP64: pixel (x, y) draws its four
    uniforms from counter (y W + x, 0, 0, 0); d = d_lo + u0 (d_hi - d_lo), theta = 2 pi u1,
    phi = pi (u2 - 1/2), the normal turned to face the camera."""
    pb = oracle.Problem.from_scene(small_scene, 7, 1)
    P, _ = oracle.init(pb, fp64=True)
    lo, hi = small_scene.depth_range
    Kinv = np.linalg.inv(small_scene.cams[0].K)
    seed = pb.s.seed
    ys, xs = np.nonzero(pb.valid_mask())
    for i in np.random.default_rng(4).choice(len(xs), 50, replace=False):
        x, y = int(xs[i]), int(ys[i])
        u = _uniforms(seed, x, y, pb.W, 0, 0)
        assert abs(P[y, x, 3] - (lo + u[0] * (hi - lo))) <= 1e-12 * hi
        n = _facing(2 * math.pi * u[1], math.pi * (u[2] - 0.5), Kinv @ [x, y, 1.0])
        np.testing.assert_allclose(P[y, x, :3], n, atol=1e-12)


def test_draws_map_to_the_documented_refinement_candidates(small_scene):
    """Random refinement (Sec. III-C, readings s12, s13, s15, s27), FP64: at iteration it
    pixel (x, y) draws from counter (y W + x, it, 1, 0); d_new = d + (2 u0 - 1) d_hi / 4,
    theta_new = atan2(n_y, n_x) + (2 u1 - 1) pi / 2, phi_new = acos(n_z) + (2 u2 - 1) pi / 12;
    the candidates (d_new, n), (d, n_new), (d_new, n_new), the first two using d_new only
    inside the depth range, are scored here through the oracle's cost of a single plane,
    and the pixel must end with the first strictly best of them (or keep its plane)."""
    pb = oracle.Problem.from_scene(small_scene, 7, 1, top_k=1)
    P, C = oracle.init(pb, fp64=True)
    it = 3
    P2, C2 = oracle.halfsweep(pb, P, C, it, 0, fp64=True, propagate=False, refine=True)
    lo, hi = small_scene.depth_range
    Kinv = np.linalg.inv(small_scene.cams[0].K)
    seed = pb.s.seed
    m = pb.valid_mask() & _colour_mask(pb.H, pb.W, 0)
    ys, xs = np.nonzero(m)
    changed = 0
    for i in np.random.default_rng(5).choice(len(xs), 40, replace=False):
        x, y = int(xs[i]), int(ys[i])
        u = _uniforms(seed, x, y, pb.W, it, 1)
        n_old, d_old = P[y, x, :3], P[y, x, 3]
        d_new = d_old + (2 * u[0] - 1) * (hi * 0.25)
        d_ok = lo <= d_new <= hi
        theta = math.atan2(n_old[1], n_old[0]) + (2 * u[1] - 1) * (math.pi / 2)
        phi = math.acos(min(max(n_old[2], -1.0), 1.0)) + (2 * u[2] - 1) * (math.pi / 12)
        n_new = _facing(theta, phi, Kinv @ [x, y, 1.0])
        cands = [(n_old, d_new, d_ok), (n_new, d_old, True), (n_new, d_new, d_ok)]
        best_c, best = C[y, x], (n_old, d_old)
        for n, d, ok in cands:
            if not ok:
                continue
            Q = P.copy()
            Q[y, x, :3], Q[y, x, 3] = n, d
            c = oracle.eval_cost(pb, Q, fp64=True, subset=[y * pb.W + x])[0][y, x]
            if c < best_c:
                best_c, best = c, (n, d)
        np.testing.assert_allclose(P2[y, x, :3], best[0], atol=1e-12)
        assert abs(P2[y, x, 3] - best[1]) <= 1e-12 * hi
        assert C2[y, x] == best_c
        changed += int(best_c < C[y, x])
    assert changed > 5


def test_halfsweeps_never_raise_cost_and_leave_other_colour(small_scene):
    pb = oracle.Problem.from_scene(small_scene, 7, 1, top_k=0)
    P, C = oracle.init(pb)
    m = pb.valid_mask()
    H, W = pb.H, pb.W
    colour_of = (np.add.outer(np.arange(H), np.arange(W)) & 1)
    for it in (1, 2):
        for col in (0, 1):
            P2, C2 = oracle.halfsweep(pb, P, C, it, col)
            assert np.all(C2[m] <= C[m])
            other = colour_of != col
            assert np.array_equal(P2[other], P[other]) and np.array_equal(C2[other], C[other])
            assert np.array_equal(P2[~m], P[~m])
            P, C = P2, C2


def test_refinement_ranges(small_scene):
    pb = oracle.Problem.from_scene(small_scene, 7, 1)
    P, C = oracle.init(pb)
    P2, C2 = oracle.halfsweep(pb, P, C, 1, 0, propagate=False, refine=True)
    ch = np.any(P2 != P, axis=-1)
    assert ch.sum() > 10
    d_hi = small_scene.depth_range[1]
    dd = np.abs(P2[..., 3] - P[..., 3])[ch]
    assert np.all(dd <= d_hi / 4 * (1 + 1e-6))
    n0 = P[..., :3][ch]
    n1 = P2[..., :3][ch]
    dphi = np.abs(np.arccos(np.clip(n1[:, 2], -1, 1)) - np.arccos(np.clip(n0[:, 2], -1, 1)))
    # |delta phi| <= pi/12 unless the camera-facing flip moved the normal (phi -> pi - phi)
    same_side = np.sign(n1[:, 2]) == np.sign(n0[:, 2])
    assert np.all(dphi[same_side] <= np.pi / 12 + 1e-5)


def _zero_baseline_problem(h, w, f, depth_range, window=5, seed=31):
    """A reference and one source with the same camera and the same image: every plane
    that faces the camera scores eps_c (Z = 1 in the one view), so under the strict-
    improvement rule a pixel whose stored cost is C_max takes the first candidate it is
    offered, whatever that candidate's plane.  This exposes the candidates themselves."""
    img = _textured(h, w, seed)
    K = _K(w, h, f=f)
    return oracle.Problem([img, img], np.stack([K, K]), np.stack([np.eye(3)] * 2), np.stack([np.zeros(3)] * 2),
                          depth_range, window, 1, top_k=0, bilateral=True)


def _colour_mask(h, w, colour):
    return (np.add.outer(np.arange(h), np.arange(w)) & 1) == colour


def _inner(pb):
    """Valid pixels whose window stays at least one pixel inside the image: with H = I up
    to rounding, a window touching the edge exactly can be placed a rounding error outside."""
    m = pb.valid_mask()
    return m & np.roll(m, 1, 0) & np.roll(m, -1, 0) & np.roll(m, 1, 1) & np.roll(m, -1, 1)


@pytest.mark.parametrize("fp64", [False, True])
def test_propagation_re_expresses_a_slanted_plane(fp64):
    """Sec. III-C propagation hands a neighbour's plane to the pixel (reading s17: the plane
    itself, so the depth is where the pixel's own ray meets it).  Every black pixel holds
    the same strongly slanted plane; after one red propagation half-sweep every red pixel
    must hold that plane too, its depth being the intersection of its ray with the plane,
    found here by solving the parametric form X0 + a u1 + b u2 = lam r (not the oracle's
    formula).  A copied neighbour depth would be off by > 0.5% per pixel of offset."""
    h, w = 56, 72
    pb = _zero_baseline_problem(h, w, f=0.9 * w, depth_range=(1.0, 20.0))
    n = np.array([0.6, -0.6, -1.0])
    n /= np.linalg.norm(n)
    X0 = np.array([0.2, -0.1, 6.0])
    u1 = np.cross(n, [0.0, 0.0, 1.0])
    u1 /= np.linalg.norm(u1)
    u2 = np.cross(n, u1)
    Kinv = np.linalg.inv(pb.K[0].reshape(3, 3))
    ys, xs = np.mgrid[0:h, 0:w]
    rays = np.einsum("ij,jhw->hwi", Kinv, np.stack([xs, ys, np.ones_like(xs)]).astype(np.float64))
    depth = np.empty((h, w))
    for y in range(h):
        for x in range(w):
            lam, _, _ = np.linalg.solve(np.stack([rays[y, x], -u1, -u2], axis=1), X0)
            depth[y, x] = lam * rays[y, x, 2]
    assert depth.min() > 2.0 and depth.max() < 19.0
    # the plane is steep: one pixel step along either axis changes the depth by > 0.5%
    assert (np.abs(np.diff(depth, axis=1)) / depth[:, 1:]).min() > 0.005
    assert (np.abs(np.diff(depth, axis=0)) / depth[1:, :]).min() > 0.005
    P = np.zeros((h, w, 4))
    C = np.full((h, w), 2.0)
    black = _colour_mask(h, w, 1)
    P[..., :3] = n
    P[..., 3] = np.where(black, depth, 9.0)
    P[~black, :3] = [0.0, 0.0, -1.0]
    C[black] = 0.5
    P2, C2 = oracle.halfsweep(pb, P, C, 1, 0, fp64=fp64, propagate=True, refine=False)
    red = _inner(pb) & ~black
    assert red.sum() > 1500
    assert np.all(C2[red] < 2.0)  # every red pixel took a candidate
    stored_n = n if fp64 else n.astype(np.float32).astype(np.float64)
    assert np.array_equal(P2[red][:, :3], np.broadcast_to(stored_n, (red.sum(), 3)))
    rel = np.abs(P2[..., 3][red] - depth[red]) / depth[red]
    assert rel.max() <= (1e-12 if fp64 else 1e-5), rel.max()


@pytest.mark.parametrize("fp64", [False, True])
def test_refinement_depth_perturbation_covers_its_range(fp64):
    """Sec. III-C random refinement: Delta_d is drawn from [-d_max/4, d_max/4] (reading s12:
    d_max = d_hi).  Each red pixel holds depth 5.5 in the range [1, 10], so d_new always
    stays in range and the first listed candidate (d_new, n_old) is the one taken; the
    observed Delta_d must then be uniform on [-2.5, 2.5], reach within 5% of both ends, and
    leave the normal untouched."""
    h, w = 96, 80
    pb = _zero_baseline_problem(h, w, f=0.9 * w, depth_range=(1.0, 10.0))
    P = np.zeros((h, w, 4))
    P[..., :3] = [0.1, -0.2, -0.97467943448]
    P[..., 3] = 5.5
    C = np.full((h, w), 2.0)
    P2, C2 = oracle.halfsweep(pb, P, C, 1, 0, fp64=fp64, propagate=False, refine=True)
    red = _inner(pb) & _colour_mask(h, w, 0)
    assert red.sum() > 3000
    assert np.all(C2[red] < 2.0)
    n0 = P[..., :3][red] if fp64 else P[..., :3][red].astype(np.float32).astype(np.float64)
    assert np.array_equal(P2[..., :3][red], n0)
    dd = P2[..., 3][red] - 5.5
    half = 10.0 / 4
    assert np.all(np.abs(dd) <= half * (1 + 1e-6))
    assert dd.min() <= -0.95 * half and dd.max() >= 0.95 * half
    assert scipy.stats.kstest((dd + half) / (2 * half), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("fp64", [False, True])
def test_refinement_normal_perturbation_covers_its_ranges(fp64):
    """Sec. III-C random refinement: the normal's angles are perturbed by Delta_theta in
    [-pi/2, pi/2] and Delta_phi in [-pi/12, pi/12] (reading s13: on theta = atan2(n_y, n_x),
    phi = acos(n_z)).  Every red pixel sits at d_hi with a range of width 0.01, so d_new
    leaves the range on all but ~0.2% of pixels and the candidate (d_old, n_new) is taken;
    with phi = 3 pi/4 and a narrow field of view (f = 3 W) no perturbed normal needs the
    camera-facing flip, so the angles of the new normal, less the old ones, are the draws:
    uniform on their ranges and reaching within 5% of every end."""
    h, w = 96, 80
    pb = _zero_baseline_problem(h, w, f=3.0 * w, depth_range=(9.99, 10.0))
    th0, ph0 = 0.3, 3 * np.pi / 4
    n0 = np.array([np.cos(th0) * np.sin(ph0), np.sin(th0) * np.sin(ph0), np.cos(ph0)])
    P = np.zeros((h, w, 4))
    P[..., :3] = n0
    P[..., 3] = 10.0
    C = np.full((h, w), 2.0)
    P2, C2 = oracle.halfsweep(pb, P, C, 2, 0, fp64=fp64, propagate=False, refine=True)
    red = _inner(pb) & _colour_mask(h, w, 0)
    took_n = red & (P2[..., 3] == 10.0)
    assert took_n.sum() > 0.99 * red.sum() > 3000
    assert np.all(C2[red] < 2.0)
    ns = n0 if fp64 else n0.astype(np.float32).astype(np.float64)
    th_old, ph_old = np.arctan2(ns[1], ns[0]), np.arccos(ns[2])
    n1 = P2[..., :3][took_n]
    dth = np.angle(np.exp(1j * (np.arctan2(n1[:, 1], n1[:, 0]) - th_old)))
    dph = np.arccos(np.clip(n1[:, 2], -1, 1)) - ph_old
    for d, half in ((dth, np.pi / 2), (dph, np.pi / 12)):
        assert np.all(np.abs(d) <= half + 1e-5)
        assert d.min() <= -0.95 * half and d.max() >= 0.95 * half
        assert scipy.stats.kstest((d + half) / (2 * half), "uniform").pvalue > 1e-3


def test_resume_equals_uninterrupted_run(small_scene):
    pb = oracle.Problem.from_scene(small_scene, 7, 1, top_k=1)
    d, n, c = oracle.patchmatch(pb, 2)
    P, C = oracle.init(pb)
    for it in (1, 2):
        for col in (0, 1):
            P, C = oracle.halfsweep(pb, P, C, it, col)
    m = pb.valid_mask()
    assert np.array_equal(P[..., 3][m].astype(np.float32), d[m])
    assert np.array_equal(C[m].astype(np.float32), c[m])


def test_zero_baseline_keeps_init():
    """A source identical to the reference (same camera, same image): every plane scores
    eps_c, so no strict improvement exists and the state stays the initial one."""
    sc = sg.make_scene(12, sg.tiny_config(48, 40, n_src=1, n_planes=2), device="cpu")
    pb = oracle.Problem([sc.images[0], sc.images[0]], np.stack([sc.cams[0].K] * 2), np.stack([sc.cams[0].R] * 2),
                        np.stack([sc.cams[0].t] * 2), sc.depth_range, 7, 1)
    P, C = oracle.init(pb)
    d, n, c = oracle.patchmatch(pb, 2)
    m = pb.valid_mask()
    assert np.all(c[m] == np.float32(1e-4))
    # pixels that scored eps_c at init (all but windows touching the image edge exactly,
    # which rounding may place outside) can never change
    keep = m & (C == np.float32(1e-4))
    assert keep.sum() > 0.9 * m.sum()
    assert np.array_equal(d[keep], P[..., 3][keep].astype(np.float32))
    assert np.array_equal(n[keep], P[..., :3][keep].astype(np.float32))


def _propagation_offsets():
    """The neighbourhood of the red/black propagation as read from the cited sampling
    scheme (reading s16), written as geometry: per axis direction e, a near "V" region of
    the other colour's pixels o with o . e > 0, |o x e| < o . e and |o|_1 odd and <= 5, and
    a far strip of the pixels k e, k = 7, 9, ..., 25."""
    regions = []
    for e in ((0, -1), (0, 1), (-1, 0), (1, 0)):
        near = []
        for dx in range(-6, 7):
            for dy in range(-6, 7):
                along = dx * e[0] + dy * e[1]
                across = abs(dx * e[1] - dy * e[0])
                l1 = abs(dx) + abs(dy)
                if along > 0 and across < along and l1 % 2 == 1 and l1 <= 5:
                    near.append((dx, dy))
        regions.append(near)
    for e in ((0, -1), (0, 1), (-1, 0), (1, 0)):
        regions.append([(k * e[0], k * e[1]) for k in range(7, 26, 2)])
    return regions


def _probe_problem():
    """Zero-baseline 64x64 problem (every camera-facing plane in range scores eps_c), a
    probe pixel at its centre, and a state in which no neighbour offers a usable plane: the
    other colour holds planes whose re-expression at any pixel lies far beyond the depth
    range."""
    h = w = 64
    pb = _zero_baseline_problem(h, w, f=0.9 * w, depth_range=(1.0, 20.0))
    P = np.zeros((h, w, 4))
    P[..., 2] = -1.0
    P[..., 3] = 200.0
    C = np.full((h, w), 1.0)
    px, py = 32, 32
    C[py, px] = 2.0
    return pb, P, C, px, py


def test_propagation_neighbourhood_geometry():
    """Sec. III-C propagation (reading s16): a pixel is offered a neighbour's plane exactly
    when that neighbour lies in one of its 8 regions.  Black-box probe: one usable plane at
    a single offset, everything else unusable; the probe pixel (stored cost C_max) must take
    it for the 76 offsets of the regions and for no other offset of the other colour within
    27 pixels."""
    pb, P, C, px, py = _probe_problem()
    regions = _propagation_offsets()
    expected = {o for r in regions for o in r}
    assert len(expected) == 76
    sub = [py * pb.W + px]
    taken = set()
    for dy in range(-27, 28):
        for dx in range(-27, 28):
            if (abs(dx) + abs(dy)) % 2 == 0:
                continue
            P2, C2 = P.copy(), C.copy()
            P2[py + dy, px + dx] = (0.0, 0.0, -1.0, 5.0)
            C2[py + dy, px + dx] = 0.0
            Po, Co = oracle.halfsweep(pb, P2, C2, 1, 0, subset=sub, propagate=True, refine=False)
            if Co[py, px] < 2.0:
                taken.add((dx, dy))
                assert Po[py, px, 2] == -1.0 and 4.0 < Po[py, px, 3] < 6.0
    assert taken == expected


def test_propagation_takes_each_regions_lowest_cost_neighbour():
    """Per region the neighbour offered is the other colour's lowest-cost pixel: with two
    pixels of one region holding planes, the usable plane is taken only when its holder has
    the lower stored cost (the other holds an unusable plane)."""
    pb, P, C, px, py = _probe_problem()
    sub = [py * pb.W + px]
    for region in _propagation_offsets():
        (ax, ay), (bx, by) = region[0], region[-1]
        for good_cost, other_cost, expect in ((0.3, 0.6, True), (0.6, 0.3, False)):
            P2, C2 = P.copy(), C.copy()
            P2[py + ay, px + ax] = (0.0, 0.0, -1.0, 5.0)
            C2[py + ay, px + ax] = good_cost
            C2[py + by, px + bx] = other_cost
            _, Co = oracle.halfsweep(pb, P2, C2, 1, 0, subset=sub, propagate=True, refine=False)
            assert (Co[py, px] < 2.0) == expect


def test_subset_evaluation_equals_the_full_pass(small_scene):
    """Evaluating or half-sweeping a list of pixels gives at those pixels what the pass over
    the whole image gives, and leaves every other pixel as it was."""
    pb = oracle.Problem.from_scene(small_scene, 7, 1, top_k=1)
    P, C = oracle.init(pb)
    m = pb.valid_mask()
    ys, xs = np.nonzero(m & _colour_mask(pb.H, pb.W, 1))
    pick = np.random.default_rng(3).choice(len(xs), 60, replace=False)
    sub = (ys[pick] * pb.W + xs[pick]).astype(np.int32)
    full_c = oracle.eval_cost(pb, P)[0]
    sub_c = oracle.eval_cost(pb, P, subset=sub)[0]
    at = (ys[pick], xs[pick])
    assert np.array_equal(sub_c[at], full_c[at])
    Pf, Cf = oracle.halfsweep(pb, P, C, 1, 1)
    Ps, Cs = oracle.halfsweep(pb, P, C, 1, 1, subset=sub)
    assert np.array_equal(Ps[at], Pf[at]) and np.array_equal(Cs[at], Cf[at])
    rest = np.ones((pb.H, pb.W), bool)
    rest[at] = False
    assert np.array_equal(Ps[rest], P[rest]) and np.array_equal(Cs[rest], C[rest])


@pytest.mark.parametrize("fp64", [False, True])
def test_stored_costs_are_the_stored_planes_costs(small_scene, fp64):
    """After initialisation and after every half-sweep (propagation and refinement) each
    pixel's stored cost is the cost of its stored plane, evaluated afresh."""
    pb = oracle.Problem.from_scene(small_scene, 7, 1, top_k=1)
    P, C = oracle.init(pb, fp64=fp64)
    m = pb.valid_mask()
    for it in (1, 2):
        for col in (0, 1):
            P, C = oracle.halfsweep(pb, P, C, it, col, fp64=fp64)
            assert np.array_equal(oracle.eval_cost(pb, P, fp64=fp64)[0][m], C[m])


def test_propagation_floods_a_seeded_plane():
    """Rectified pair of white-noise images related by a fronto-parallel plane (integer
    disparity): the true plane is the unique good hypothesis.  Seeded at one pixel, it must
    reach every valid pixel by propagation alone (no refinement)."""
    h, w = 40, 56
    rng = np.random.default_rng(21)
    A = rng.integers(0, 256, size=(h, w + 20)).astype(np.float32)
    f, Z, b = 50.0, 4.0, 0.4
    D = int(round(f * b / Z))  # 5 px
    K = _K(w, h, f=f)
    ref = np.ascontiguousarray(A[:, 10:10 + w])
    left = np.ascontiguousarray(A[:, 10 + D:10 + D + w])   # camera moved by +b: u_j = u - D
    right = np.ascontiguousarray(A[:, 10 - D:10 - D + w])  # camera moved by -b: u_j = u + D
    pb = oracle.Problem([ref, left, right], np.stack([K] * 3), np.stack([np.eye(3)] * 3),
                        np.stack([np.zeros(3), np.array([-b, 0, 0]), np.array([b, 0, 0])]), (2.0, 8.0), 7, 1,
                        top_k=0, bilateral=True)
    P, C = oracle.init(pb)
    y0, x0 = h // 2, w // 2
    P[y0, x0] = [0.0, 0.0, -1.0, Z]
    C[y0, x0] = oracle.eval_cost(pb, P, subset=[y0 * w + x0])[0][y0, x0]
    for it in range(1, 5):
        for col in (0, 1):
            P, C = oracle.halfsweep(pb, P, C, it, col, propagate=True, refine=False)
    m = pb.valid_mask()
    assert np.all(np.abs(P[..., 3][m] - Z) < 1e-4)
    assert np.all(np.abs(P[..., :3][m] - [0, 0, -1]) < 1e-6)


def test_brute_force_search_recovers_ground_truth():
    """Exhaustive search over a discretised plane set (depth grid x {GT normals, random
    normals}) recovers GT depth to the grid step on unoccluded pixels, and PatchMatch ends at
    or below the brute-force minimum cost, at the right depth, on nearly all of them."""
    sc = sg.crop_reference(sg.make_scene(14, sg.tiny_config(160, 120, n_src=4, n_planes=2), device="cpu"), 48, 36)
    pb = oracle.Problem.from_scene(sc, 7, 1, top_k=0)
    H, W = pb.H, pb.W
    gt = np.zeros((H, W, 4))
    gt[..., :3] = sc.gt_normal
    gt[..., 3] = sc.gt_depth
    # pixels whose true plane matches well in the sources (not occluded, not at the border)
    sel = pb.valid_mask() & (oracle.eval_cost(pb, gt)[0] < 0.1)
    assert sel.sum() > 300
    lo, hi = sc.depth_range
    depths = np.linspace(lo, hi, 24)
    rng = np.random.default_rng(0)
    normals = [sc.gt_normal[sc.gt_plane == k][0] for k in np.unique(sc.gt_plane)]
    for _ in range(6):
        v = rng.normal(size=3)
        v[2] = -abs(v[2]) - 1.0
        normals.append(v / np.linalg.norm(v))
    best = np.full((H, W), np.inf)
    best_d = np.zeros((H, W))
    for nrm in normals:
        for dep in depths:
            planes = np.zeros((H, W, 4))
            planes[..., :3] = nrm
            planes[..., 3] = dep
            c, _, _ = oracle.eval_cost(pb, planes)
            better = c < best
            best[better] = c[better]
            best_d[better] = dep
    step = depths[1] - depths[0]
    assert (np.abs(best_d - sc.gt_depth) <= step)[sel].mean() > 0.95
    d, n, c = oracle.patchmatch(pb, 4)
    assert (c[sel] <= best[sel] + 1e-3).mean() > 0.95
    assert (np.abs(d - sc.gt_depth)[sel] <= step).mean() > 0.95
