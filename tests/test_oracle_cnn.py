"""Pins of the proposal-network oracle against things other than itself: library
routines (scipy's correlation and bilinear interpolation, torch's bfloat16 conversion),
adjoint identities, central finite differences, closed forms and projective geometry."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import cnn

torch = pytest.importorskip("torch")


def rng(seed=0):
    return np.random.default_rng(seed)


def small_params(seed=0, scale=0.25):
    r = rng(seed)
    layers = []
    for ci, co in cnn.SHAPES:
        layers.append((r.normal(0, scale / np.sqrt(9 * ci), (9, ci, co)), r.normal(0, 0.05, co)))
    return cnn.pack(layers)


def test_param_count_matches_the_architecture():
    assert cnn.param_count() == 30372
    p = small_params()
    assert p.size == 30372
    assert np.array_equal(cnn.pack(cnn.unpack(p)), p)


def test_bf16_rounding_matches_torch():
    r = rng(1)
    x = np.concatenate([r.normal(0, 1, 5000), r.normal(0, 1e-3, 1000), r.normal(0, 1e4, 1000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(x), ref)
    # ties go to even: 1 + 2^-8 is half-way between 1 and 1 + 2^-7
    assert cnn.bf16(np.float32(1.0 + 2 ** -8)) == 1.0


@pytest.mark.parametrize("shape", [(1, 7, 9), (2, 5, 4), (1, 1, 1), (1, 3, 17)])
def test_conv_equals_scipy_correlation(shape):
    B, h, w = shape
    r = rng(2)
    x = r.normal(size=(B, h, w, 3))
    wt = r.normal(size=(9, 3, 2))
    b = r.normal(size=2)
    y = cnn.conv3x3(x, wt, b)
    for bi in range(B):
        for co in range(2):
            ref = np.full((h, w), b[co])
            for ci in range(3):
                k = wt[:, ci, co].reshape(3, 3)  # k[dy + 1, dx + 1]
                ref += ndi.correlate(x[bi, :, :, ci], k, mode="constant", cval=0.0)
            np.testing.assert_allclose(y[bi, :, :, co], ref, rtol=1e-12, atol=1e-12)


def test_conv_gradients_are_adjoint():
    """<conv(x, w), g> = <x, dgrad(g, w)> = <w, wgrad(x, g)> (convolution is bilinear)."""
    r = rng(3)
    x = r.normal(size=(2, 6, 7, 4))
    w = r.normal(size=(9, 4, 5))
    g = r.normal(size=(2, 6, 7, 5))
    lhs = (cnn.conv3x3(x, w) * g).sum()
    assert np.isclose(lhs, (x * cnn.conv3x3_dgrad(g, w)).sum(), rtol=1e-12)
    assert np.isclose(lhs, (w * cnn.conv3x3_wgrad(x, g)).sum(), rtol=1e-12)


def _problem(seed=4, B=2, h=6, w=7):
    r = rng(seed)
    x = r.normal(size=(B, h, w, 5))
    drange = np.array([[1.0, 9.0], [2.0, 5.0]])[:B]
    lo = drange[:, 0][:, None, None]
    hi = drange[:, 1][:, None, None]
    tgt = np.zeros((B, h, w, 4))
    tgt[..., 0] = lo + (hi - lo) * r.uniform(0.05, 0.95, (B, h, w))
    n = r.normal(size=(B, h, w, 3))
    tgt[..., 1:] = n / np.linalg.norm(n, axis=-1, keepdims=True)
    mask = (r.uniform(size=(B, h, w)) < 0.8).astype(np.float64)
    return x, tgt, mask, drange


def test_loss_output_gradient_matches_finite_differences():
    x, tgt, mask, drange = _problem()
    r = rng(5)
    out = r.normal(size=tgt.shape)
    g = cnn.loss_output_grad(out, tgt, mask, drange, 0.7)
    eps = 1e-6
    idx = [tuple(r.integers(0, s) for s in out.shape) for _ in range(60)]
    for i in idx:
        op, om = out.copy(), out.copy()
        op[i] += eps
        om[i] -= eps
        fd = (cnn.loss(op, tgt, mask, drange, 0.7) - cnn.loss(om, tgt, mask, drange, 0.7)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_parameter_gradient_matches_finite_differences():
    x, tgt, mask, drange = _problem()
    p = small_params(6, scale=1.0)
    L, g = cnn.loss_grad(p, x, tgt, mask, drange, 0.5)
    r = rng(7)
    # coordinates in every layer, weights and biases
    offs = np.cumsum([0] + [9 * ci * co + co for ci, co in cnn.SHAPES])
    idx = []
    for l in range(5):
        idx += list(r.integers(offs[l], offs[l + 1], 8))
        idx.append(offs[l + 1] - 1)  # a bias
    eps = 1e-6
    checked = 0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (cnn.loss(cnn.forward(pp, x)[0], tgt, mask, drange, 0.5)
              - cnn.loss(cnn.forward(pm, x)[0], tgt, mask, drange, 0.5)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-8 + 1e-4 * abs(fd), (i, fd, g[i])
        checked += abs(g[i]) > 1e-9
    assert checked >= 20  # most checked coordinates carry a non-zero gradient


def test_input_gradient_chain_matches_finite_differences():
    """The backward pass carried one layer further, to the network input, against finite
    differences of the loss in the input."""
    x, tgt, mask, drange = _problem(8, B=1, h=5, w=5)
    p = small_params(9, scale=1.0)
    layers = cnn.unpack(p)
    out, acts = cnn.forward(p, x)
    g = cnn.loss_output_grad(out, tgt, mask, drange, 1.0)
    for i in range(4, -1, -1):
        gx = cnn.conv3x3_dgrad(g, layers[i][0])
        if i == 0:
            break
        g = gx * (acts[i] > 0)
    eps = 1e-6
    r = rng(10)
    for _ in range(20):
        j = tuple(r.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[j] += eps
        xm[j] -= eps
        fd = (cnn.loss(cnn.forward(p, xp)[0], tgt, mask, drange) - cnn.loss(cnn.forward(p, xm)[0], tgt, mask, drange)) / (2 * eps)
        assert abs(fd - gx[j]) <= 1e-8 + 1e-4 * abs(fd)


def test_adam_first_step_closed_form():
    """With bias correction the first step moves every weight by lr * g / (|g| + eps')."""
    r = rng(11)
    p = r.normal(size=50)
    g = r.normal(size=50)
    p1, m, v = cnn.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def _cam(f, W, H, yaw, pos):
    K = np.array([[f, 0, (W - 1) / 2], [0, f, (H - 1) / 2], [0, 0, 1.0]])
    c, s = np.cos(yaw), np.sin(yaw)
    R = np.array([[c, 0, -s], [0, 1, 0], [s, 0, c]])
    t = -R @ np.asarray(pos, dtype=np.float64)
    return K, R, t


def test_plane_homography_maps_points_of_the_plane():
    K0, R0, t0 = _cam(100, 64, 48, 0.0, [0, 0, 0])
    K1, R1, t1 = _cam(120, 80, 60, 0.2, [0.5, 0.1, -0.2])
    Hm = cnn.plane_homography(K0, R0, t0, K1, R1, t1, 4.0)
    r = rng(12)
    for _ in range(20):
        u, v = r.uniform(0, 63), r.uniform(0, 47)
        X = 4.0 * np.linalg.inv(K0) @ np.array([u, v, 1.0])  # reference camera frame, Z = 4
        Xw = R0.T @ (X - t0)
        p = K1 @ (R1 @ Xw + t1)
        q = Hm @ np.array([u, v, 1.0])
        np.testing.assert_allclose(q[:2] / q[2], p[:2] / p[2], atol=1e-9)


def test_plane_homography_with_a_moved_reference():
    """The same with the reference camera itself moved and turned (its pose enters the
    relative transform)."""
    K0, R0, t0 = _cam(100, 64, 48, 0.15, [0.3, -0.2, 0.5])
    K1, R1, t1 = _cam(120, 80, 60, -0.25, [1.1, 0.3, 0.2])
    Hm = cnn.plane_homography(K0, R0, t0, K1, R1, t1, 5.5)
    r = rng(14)
    for _ in range(20):
        u, v = r.uniform(0, 63), r.uniform(0, 47)
        X = 5.5 * np.linalg.inv(K0) @ np.array([u, v, 1.0])
        Xw = R0.T @ (X - t0)
        p = K1 @ (R1 @ Xw + t1)
        q = Hm @ np.array([u, v, 1.0])
        np.testing.assert_allclose(q[:2] / q[2], p[:2] / p[2], atol=1e-9)


def test_nearest_sources_by_camera_centre():
    Rs, ts = [], []
    for x in [0.0, 3.0, -1.0, 0.5, 2.0, -0.2]:
        K, R, t = _cam(100, 64, 48, 0.0, [x, 0, 0])
        Rs.append(R)
        ts.append(t)
    assert cnn.nearest_sources(Rs, ts, 0, [1, 2, 3, 4, 5]) == [5, 3, 2, 4]
    # the reference away from the origin: distances are to its centre
    Rs, ts = [], []
    for x in [5.0, 8.0, 4.0, 5.5, 7.0, 4.8]:
        K, R, t = _cam(100, 64, 48, 0.1, [x, 1.0, -2.0])
        Rs.append(R)
        ts.append(t)
    assert cnn.nearest_sources(Rs, ts, 0, [1, 2, 3, 4, 5]) == [5, 3, 2, 4]


@pytest.mark.parametrize("H,W", [(36, 44), (37, 45)])
def test_proposal_inputs_warp_general_poses(H, W):
    """Reference moved and turned, six sources around it: channels 1-4 hold the four
    nearest sources (by camera centre, in that order), each sampled where the point of the
    reference plane Z = (d_lo + d_hi) / 2 behind block centre (4X + 1.5, 4Y + 1.5)
    projects, computed here through world coordinates; the sources are affine ramps in
    their pixel coordinates, so bilinear sampling is exact; outside a source: 0."""
    f = 50.0
    K0, R0, t0 = _cam(f, W, H, 0.1, [0.4, -0.3, 0.2])
    poses = [(-0.05, [0.9, -0.3, 0.2]), (0.2, [0.1, -0.1, 0.1]), (0.15, [0.4, 0.5, 0.2]), (0.0, [2.5, -0.3, 0.2]),
             (0.12, [0.4, -0.3, -0.5]), (0.3, [-0.9, -0.3, 0.2])]
    Ks, Rs, ts, images = [K0], [R0], [t0], [np.full((H, W), 100.0)]
    coef = []
    for j, (yaw, pos) in enumerate(poses):
        Ws, Hs = W + 3 * j, H + 2 * j
        Kj, Rj, tj = _cam(f * (1 + 0.1 * j), Ws, Hs, yaw, pos)
        a, b, c = 20.0 + 10 * j, 1.5 + 0.2 * j, -0.8 + 0.3 * j
        yy, xx = np.mgrid[0:Hs, 0:Ws].astype(np.float64)
        Ks.append(Kj)
        Rs.append(Rj)
        ts.append(tj)
        images.append(a + b * xx + c * yy)
        coef.append((a, b, c))
    lo, hi = 1.5, 9.5
    out = cnn.proposal_inputs(images, Ks, Rs, ts, (lo, hi), 0, [1, 2, 3, 4, 5, 6])
    h, w = -(-H // 4), -(-W // 4)
    assert out.shape == (h, w, 5)
    c0 = -R0.T @ t0
    dist = [np.sum((-Rs[s].T @ ts[s] - c0) ** 2) for s in range(1, 7)]
    order = [1 + int(i) for i in np.argsort(dist, kind="stable")[:4]]
    dmid = 0.5 * (lo + hi)
    checked = 0
    for k, s in enumerate(order):
        a, b, c = coef[s - 1]
        Hs, Ws = images[s].shape
        for Y in range(h):
            for X in range(w):
                x = np.array([4 * X + 1.5, 4 * Y + 1.5, 1.0])
                Xw = R0.T @ (dmid * (np.linalg.inv(K0) @ x) - t0)
                p = Ks[s] @ (Rs[s] @ Xw + ts[s])
                u, v = p[0] / p[2], p[1] / p[2]
                inside = p[2] > 0 and 0 <= u <= Ws - 1 and 0 <= v <= Hs - 1
                want = (a + b * u + c * v - 127.5) / 64.0 if inside else 0.0
                assert abs(out[Y, X, 1 + k] - want) < 1e-9
                checked += inside
    assert checked > 2 * h * w


def test_decode_upsamples_random_outputs_bilinearly():
    """Random raw outputs (normals of any length): each output channel is interpolated
    linearly at ((y - 1.5) / 4, (x - 1.5) / 4) clamped to the grid (scipy's order-1
    map_coordinates), depth through the scaled sigmoid, the normal normalised and turned
    to face the camera."""
    H, W = 19, 26
    h, w = 5, 7
    K, _, _ = _cam(30, W, H, 0.0, [0, 0, 0])
    r = rng(21)
    out = r.normal(size=(h, w, 4)) * np.array([1.5, 2.0, 2.0, 2.0])
    planes = cnn.decode(out, K, (2.0, 10.0), H, W)
    Y, X = np.meshgrid(np.clip((np.arange(H) - 1.5) / 4, 0, h - 1), np.clip((np.arange(W) - 1.5) / 4, 0, w - 1),
                       indexing="ij")
    o = np.stack([ndi.map_coordinates(out[..., c], [Y.ravel(), X.ravel()], order=1).reshape(H, W)
                  for c in range(4)], -1)
    np.testing.assert_allclose(planes[..., 3], 2.0 + 8.0 / (1 + np.exp(-o[..., 0])), rtol=1e-12)
    n = o[..., 1:] / np.linalg.norm(o[..., 1:], axis=-1, keepdims=True)
    rays = np.stack(list(np.meshgrid(np.arange(W), np.arange(H))) + [np.ones((H, W))], -1) @ np.linalg.inv(K).T
    n[(n * rays).sum(-1) > 0] *= -1
    np.testing.assert_allclose(planes[..., :3], n, atol=1e-12)


def test_targets_of_ramps():
    """Depth and normals varying per pixel: block (X, Y) averages the depths of pixels
    4X + 1 .. 4X + 2, 4Y + 1 .. 4Y + 2 (clamped) and normalises the sum of their normals."""
    H, W = 14, 17
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    depth = 2.0 + 0.1 * xx + 0.05 * yy + 0.01 * xx * yy
    normal = np.stack([0.02 * xx, -0.03 * yy, -np.ones_like(xx)], -1)
    cost = np.full((H, W), 0.2)
    tgt, mask = cnn.targets(depth, normal, cost, 0.5)
    h, w = 4, 5
    assert np.all(mask == 1)
    for Y in range(h):
        for X in range(w):
            ys = np.minimum([4 * Y + 1, 4 * Y + 2], H - 1)
            xs = np.minimum([4 * X + 1, 4 * X + 2], W - 1)
            blk = np.ix_(ys, xs)
            assert np.isclose(tgt[Y, X, 0], depth[blk].mean(), rtol=1e-14)
            ns = normal[blk].reshape(-1, 3).sum(0)
            np.testing.assert_allclose(tgt[Y, X, 1:], ns / np.linalg.norm(ns), atol=1e-14)


def test_proposal_inputs_identity_source_and_ramp():
    """A source identical to the reference samples the reference at the block centres
    (scipy's linear interpolation); a linear ramp averages to its value at the block centre."""
    H, W = 22, 30  # ragged: 30 = 4 * 7 + 2, 22 = 4 * 5 + 2
    K, R, t = _cam(40, W, H, 0.0, [0, 0, 0])
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = 3.0 * xx + 2.0 * yy + 10.0
    r = rng(13)
    noise = r.uniform(0, 255, (H, W))
    images = [img, noise, img]
    Ks = [K, K, K]
    Rs = [R, R, R]
    ts = [t, t + np.array([5.0, 0, 0]), t]
    out = cnn.proposal_inputs(images, Ks, Rs, ts, (2.0, 6.0), 0, [2])
    h, w = 6, 8
    assert out.shape == (h, w, 5)
    # channel 0 on interior blocks: ramp value at (4X + 1.5, 4Y + 1.5)
    for Y in range(h - 1):
        for X in range(w - 1):
            assert np.isclose(out[Y, X, 0] * 64 + 127.5, 3.0 * (4 * X + 1.5) + 2.0 * (4 * Y + 1.5) + 10.0)
    # edge blocks repeat the last column / row: mean over clamped coordinates
    xs = np.minimum(np.arange(4 * (w - 1), 4 * w), W - 1)
    assert np.isclose(out[0, w - 1, 0] * 64 + 127.5, (3.0 * xs.mean() + 2.0 * 1.5 + 10.0))
    ys = np.minimum(np.arange(4 * (h - 1), 4 * h), H - 1)
    assert np.isclose(out[h - 1, 0, 0] * 64 + 127.5, (3.0 * 1.5 + 2.0 * ys.mean() + 10.0))
    # identity homography for the identical source: channel 1 = reference bilinear at block centres
    cy, cx = np.mgrid[0:h, 0:w].astype(np.float64) * 4 + 1.5
    inside = (cx <= W - 1) & (cy <= H - 1)
    ref = ndi.map_coordinates(img, [cy.ravel(), cx.ravel()], order=1).reshape(h, w)
    np.testing.assert_allclose(out[..., 1][inside] * 64 + 127.5, ref[inside], atol=1e-9)
    assert np.all(out[..., 1][~inside] == 0)
    assert np.all(out[..., 2:] == 0)  # only one source given


def test_decode_closed_forms():
    H, W = 13, 18
    K, _, _ = _cam(20, W, H, 0.0, [0, 0, 0])
    h, w = 4, 5
    out = np.zeros((h, w, 4))
    # depth logit linear in X: o0 = 0.3 X - 0.5 ; normal (0, 0, -1)
    X = np.arange(w, dtype=np.float64)
    out[..., 0] = 0.3 * X[None, :] - 0.5
    out[..., 3] = -1.0
    planes = cnn.decode(out, K, (2.0, 10.0), H, W)
    xs = np.clip((np.arange(W) - 1.5) / 4, 0, w - 1)
    d = 2.0 + 8.0 / (1 + np.exp(-(0.3 * xs - 0.5)))
    np.testing.assert_allclose(planes[..., 3], np.broadcast_to(d, (H, W)), rtol=1e-12)
    np.testing.assert_allclose(planes[..., :3], np.broadcast_to([0, 0, -1.0], (H, W, 3)))
    # a normal pointing away from the camera is turned around; zero vector -> (0, 0, -1)
    out[..., 1:] = [0.0, 0.0, 2.0]
    out[0, 0, 1:] = 0.0
    planes = cnn.decode(out, K, (2.0, 10.0), H, W)
    rays = np.stack(list(np.meshgrid(np.arange(W), np.arange(H))) + [np.ones((H, W))], -1) @ np.linalg.inv(K).T
    assert np.all((planes[..., :3] * rays).sum(-1) < 0)
    np.testing.assert_allclose(planes[0, 0, :3], [0, 0, -1.0])


def test_targets_of_a_constant_plane_and_masking():
    H, W = 10, 13
    depth = np.full((H, W), 3.0)
    normal = np.broadcast_to(np.array([0.0, 0.6, -0.8]), (H, W, 3)).copy()
    cost = np.full((H, W), 0.1)
    cost[5, 6] = 0.9  # block (X=1, Y=1) looks at (5..6, 5..6)
    depth[9, 12] = 0.0  # invalid pixel: last block column/row (clamped)
    tgt, mask = cnn.targets(depth, normal, cost, 0.5)
    assert tgt.shape == (3, 4, 4)
    assert mask[1, 1] == 0 and mask[2, 3] == 0
    keep = mask > 0
    assert keep.sum() == 10
    np.testing.assert_allclose(tgt[keep][:, 0], 3.0)
    np.testing.assert_allclose(tgt[keep][:, 1:], np.broadcast_to([0.0, 0.6, -0.8], (10, 3)), atol=1e-15)
