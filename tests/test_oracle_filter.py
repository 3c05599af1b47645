"""Pins of the geometric-consistency filter oracle (Sec. III-D) against closed forms on
analytic scenes: a neighbour that is the reference camera itself (depth ratio, normal
angle and counting thresholds exactly), a rectified pair looking at a fronto-parallel
plane (re-projection error f b (1/Z' - 1/Z) in closed form, rounding of the normal
lookup), and the cases that make a neighbour unusable."""
import numpy as np
import pytest

import oracle


def cam(f, W, H, tx=0.0, yaw=0.0):
    K = np.array([[f, 0.0, (W - 1) / 2.0], [0.0, f, (H - 1) / 2.0], [0.0, 0.0, 1.0]])
    c, s = np.cos(yaw), np.sin(yaw)
    R = np.array([[c, 0.0, -s], [0.0, 1.0, 0.0], [s, 0.0, c]])
    t = -R @ np.array([tx, 0.0, 0.0])
    return K, R, t


def stack(cams):
    return (np.stack([c[0] for c in cams]), np.stack([c[1] for c in cams]), np.stack([c[2] for c in cams]))


def plane_maps(W, H, Z):
    return np.full((H, W), Z, np.float32), np.broadcast_to(np.array([0.0, 0.0, -1.0], np.float32), (H, W, 3)).copy()


W, H, F = 64, 48, 100.0


def test_identical_neighbours_are_consistent():
    K, R, t = stack([cam(F, W, H)] * 3)
    d, n = plane_maps(W, H, 4.0)
    od, on, oc = oracle.consistency({0: d, 1: d, 2: d}, {0: n, 1: n, 2: n}, K, R, t, 0, [1, 2])
    assert np.all(oc == 2)
    assert np.array_equal(od, d) and np.array_equal(on, n)


@pytest.mark.parametrize("eps,ok", [(0.0200, True), (0.0203, True), (0.0206, False), (0.05, False), (-0.0195, True),
                                    (-0.0205, False)])
def test_depth_ratio_threshold(eps, ok):
    """Same camera, neighbour depth (1 + eps) d: consistent iff |eps| / (1 + eps) < 0.02."""
    K, R, t = stack([cam(F, W, H)] * 2)
    d, n = plane_maps(W, H, 4.0)
    dn = (d.astype(np.float64) * (1 + eps)).astype(np.float32)
    _, _, oc = oracle.consistency({0: d, 1: dn}, {0: n, 1: n}, K, R, t, 0, [1], min_consistent=1)
    assert np.all(oc == (1 if ok else 0))
    assert (abs(eps) / (1 + eps) < 0.02) == ok


@pytest.mark.parametrize("deg,ok", [(29.0, True), (29.9, True), (30.1, False), (45.0, False)])
def test_normal_angle_threshold(deg, ok):
    K, R, t = stack([cam(F, W, H)] * 2)
    d, n = plane_maps(W, H, 4.0)
    a = np.radians(deg)
    nr = np.broadcast_to(np.array([np.sin(a), 0.0, -np.cos(a)], np.float32), (H, W, 3)).copy()
    _, _, oc = oracle.consistency({0: d, 1: d}, {0: n, 1: nr}, K, R, t, 0, [1], min_consistent=1)
    assert np.all(oc == (1 if ok else 0))


@pytest.mark.parametrize("b,ok", [(3.9, True), (4.03, True), (4.15, False), (6.0, False)])
def test_reprojection_error_closed_form(b, ok):
    """Rectified pair, baseline b, plane at Z on the reference and Z' = 1.01 Z on the
    neighbour: depth and normal tests pass; the neighbour's point re-projects
    f b (1/Z - 1/Z') pixels away from x."""
    Wb = 400
    K, R, t = stack([cam(F, Wb, H), cam(F, Wb, H, tx=b)])
    Z = 4.0
    d, n = plane_maps(Wb, H, Z)
    d2, _ = plane_maps(Wb, H, Z * 1.01)
    _, _, oc = oracle.consistency({0: d, 1: d2}, {0: n, 1: n}, K, R, t, 0, [1], min_consistent=1)
    err = F * b * (1 / Z - 1 / (Z * 1.01))
    assert (err < 1.0) == ok
    disp = F * b / Z
    xs = np.arange(Wb)
    seen = (xs - disp >= 0) & (xs - disp <= Wb - 2)  # the bilinear cell stays inside
    assert np.all(oc[:, seen] == (1 if ok else 0))
    assert np.all(oc[:, xs - disp < 0] == 0)  # projects left of the neighbour's image


@pytest.mark.parametrize("disp,parity", [(2.4, 0), (2.6, 1), (-2.4, 0), (-2.6, 1)])
def test_normal_taken_at_the_rounded_position(disp, parity):
    """The neighbour's normal is read at floor(u + 1/2): with disparity 2.4 the rounded
    column has x's parity, with 2.6 the other one.  Negative disparities move the points
    right, so that u within half a pixel of the last column reads that column (odd)."""
    Wb = 80
    Z = 4.0
    b = disp * Z / F
    K, R, t = stack([cam(F, Wb, H), cam(F, Wb, H, tx=b)])
    d, n = plane_maps(Wb, H, Z)
    nb = n.copy()
    a = np.radians(40.0)
    nb[:, 1::2] = [np.sin(a), 0.0, -np.cos(a)]  # odd columns fail the normal test
    _, _, oc = oracle.consistency({0: d, 1: d}, {0: n, 1: nb}, K, R, t, 0, [1], min_consistent=1)
    xs = np.arange(Wb)
    u = xs - disp
    inside = (u >= 0) & (u <= Wb - 1)
    rounded_even = (np.floor(u + 0.5).astype(int) % 2) == 0
    assert np.all(oc[:, inside & rounded_even] == 1)
    assert np.all(oc[:, inside & ~rounded_even] == 0)
    # the rounded column keeps x's parity for 2.4 (x - 2) and flips it for 2.6 (x - 3)
    assert np.all(rounded_even[inside] == ((xs[inside] + parity) % 2 == 0))


def test_unusable_neighbours_and_minimum_count():
    K0, R0, t0 = cam(F, W, H)
    K1, R1, t1 = cam(F, W, H, yaw=np.pi)  # looks the other way: everything behind it
    K, R, t = stack([(K0, R0, t0), (K0, R0, t0), (K1, R1, t1), (K0, R0, t0)])
    d, n = plane_maps(W, H, 4.0)
    holes = d.copy()
    holes[10:20, 10:20] = 0.0  # invalid texels
    maps = {0: d, 1: d, 2: d, 3: holes}
    norms = {0: n, 1: n, 2: n, 3: n}
    od, on, oc = oracle.consistency(maps, norms, K, R, t, 0, [1, 2, 3])
    # view 1 always consistent, view 2 never (behind), view 3 except where its texels are holes
    near_hole = np.zeros((H, W), bool)
    near_hole[9:20, 9:20] = True  # a bilinear cell touching the hole
    assert np.all(oc[~near_hole] == 2) and np.all(oc[10:20, 10:20] == 1)
    # min 2: the pixels with a single consistent neighbour are dropped
    assert np.all(od[10:20, 10:20] == 0) and np.all(on[10:20, 10:20] == 0)
    assert np.all(od[~near_hole] == 4.0)
    # a reference pixel without depth is never kept and counts nothing
    d0 = d.copy()
    d0[0, 0] = 0.0
    od2, _, oc2 = oracle.consistency({0: d0, 1: d, 3: d}, {0: n, 1: n, 3: n}, K, R, t, 0, [1, 3])
    assert oc2[0, 0] == 0 and od2[0, 0] == 0 and oc2[1, 1] == 2


@pytest.mark.parametrize("eps,ok", [(0.019, True), (-0.019, True), (0.021, False), (-0.021, False)])
def test_depth_sampled_bilinearly_at_subpixel_positions(eps, ok):
    """Same pose, the neighbour's principal point shifted by (0.3, 0.6): reference pixel x
    lands on (x + 0.3, y + 0.6) of the neighbour, whose depth map is a bilinear function of
    the pixel coordinates, so its bilinear interpolation there is exact.  With the
    reference depth (1 + eps) times that value the depth test passes iff |eps| < 0.02 (the
    re-projection comes back to x exactly and the normals agree)."""
    K0, R0, t0 = cam(F, W, H)
    K1 = K0.copy()
    K1[0, 2] += 0.3
    K1[1, 2] += 0.6
    K, R, t = stack([(K0, R0, t0), (K1, R0, t0)])
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)

    def dj(u, v):
        return 4.0 + 0.05 * u + 0.2 * v + 0.003 * u * v

    d1 = dj(xx, yy).astype(np.float32)
    d0 = (dj(xx + 0.3, yy + 0.6) * (1 + eps)).astype(np.float32)
    _, n = plane_maps(W, H, 4.0)
    _, _, oc = oracle.consistency({0: d0, 1: d1}, {0: n, 1: n}, K, R, t, 0, [1], min_consistent=1)
    inner = np.zeros((H, W), bool)
    inner[:H - 1, :W - 1] = True  # the bilinear cell lies inside
    assert np.all(oc[inner] == (1 if ok else 0))
    assert np.all(oc[~inner] == 0)


def _rot(yaw, pitch):
    cy, sy, cp, sp = np.cos(yaw), np.sin(yaw), np.cos(pitch), np.sin(pitch)
    Ry = np.array([[cy, 0.0, -sy], [0.0, 1.0, 0.0], [sy, 0.0, cy]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, cp, -sp], [0.0, sp, cp]])
    return Rx @ Ry


@pytest.mark.parametrize("frame,ok", [("own", True), ("reference", False)])
def test_normals_compared_in_world_coordinates(frame, ok):
    """A slanted plane seen from two cameras at the same centre, the second turned by 12
    degrees of yaw and 35 of pitch.  Each view's depth is the plane's exact depth on its
    rays; its normal is the plane normal in its own camera frame.  Compared in world
    coordinates the normals agree and every pixel whose re-projection lands inside is
    consistent; the second view's normals left in the reference frame (off by the 37
    degree rotation) fail the 30 degree test everywhere."""
    Wb, Hb, f = 64, 48, 60.0
    K0, _, _ = cam(f, Wb, Hb)
    R1 = _rot(np.radians(12.0), np.radians(35.0))
    K, R, t = stack([(K0, np.eye(3), np.zeros(3)), (K0, R1, np.zeros(3))])
    n0 = np.array([0.35, -0.45, -1.0])
    n0 /= np.linalg.norm(n0)
    c = 5.0  # plane n0 . X = -c in the reference (world) frame
    yy, xx = np.mgrid[0:Hb, 0:Wb].astype(np.float64)
    rays = np.stack([xx, yy, np.ones_like(xx)], -1) @ np.linalg.inv(K0).T

    def depth_in(Rj):
        nj = Rj @ n0  # the plane in camera j's frame: nj . X = -c (no translation)
        return ((-c / (rays @ nj)) * rays[..., 2]).astype(np.float32), nj.astype(np.float32)

    d0, nn0 = depth_in(np.eye(3))
    d1, nn1 = depth_in(R1)
    assert np.all(d0 > 0) and np.all(d1 > 0)
    N0 = np.broadcast_to(nn0, (Hb, Wb, 3)).copy()
    N1 = np.broadcast_to(nn1 if frame == "own" else nn0, (Hb, Wb, 3)).copy()
    _, _, oc = oracle.consistency({0: d0, 1: d1}, {0: N0, 1: N1}, K, R, t, 0, [1], min_consistent=1,
                                  tau_d=0.02, tau_r=1.0)
    X = rays * d0[..., None].astype(np.float64) / rays[..., 2:3]
    p = (X @ R1.T) @ K0.T
    u, v = p[..., 0] / p[..., 2], p[..., 1] / p[..., 2]
    inside = (u >= 0) & (u <= Wb - 2) & (v >= 0) & (v <= Hb - 2)
    assert inside.sum() > 200
    if ok:
        assert np.all(oc[inside] == 1)
    else:
        assert np.all(oc == 0)
    assert np.degrees(np.arccos(np.clip(nn0 @ nn1, -1, 1))) > 30.0


@pytest.mark.parametrize("disp,parity", [(2.4, 0), (2.6, 1), (-2.4, 0), (-2.6, 1)])
def test_normal_taken_at_the_rounded_row(disp, parity):
    """The same as for columns, with a vertical baseline: the neighbour's normal is read in
    row floor(v + 1/2); odd rows hold a normal that fails the test.  Negative disparities
    reach the last row (odd)."""
    Hb = 60
    Z = 4.0
    b = disp * Z / F
    K0, R0, _ = cam(F, W, Hb)
    t1 = -R0 @ np.array([0.0, b, 0.0])
    K, R, t = stack([(K0, R0, np.zeros(3)), (K0, R0, t1)])
    d, n = plane_maps(W, Hb, Z)
    nb = n.copy()
    a = np.radians(40.0)
    nb[1::2, :] = [0.0, np.sin(a), -np.cos(a)]  # odd rows fail the normal test
    _, _, oc = oracle.consistency({0: d, 1: d}, {0: n, 1: nb}, K, R, t, 0, [1], min_consistent=1)
    ys = np.arange(Hb)
    v = ys - disp
    inside = (v >= 0) & (v <= Hb - 1)
    rounded_even = (np.floor(v + 0.5).astype(int) % 2) == 0
    assert np.all(oc[inside & rounded_even, :] == 1)
    assert np.all(oc[inside & ~rounded_even, :] == 0)
    assert np.all(rounded_even[inside] == ((ys[inside] + parity) % 2 == 0))


@pytest.mark.parametrize("deg", [20.0, 37.0])
def test_normals_tilted_out_of_the_horizontal_plane(deg):
    """Same camera, both views holding the normal (0, sin a, -cos a): the normals are equal,
    so every pixel is consistent whatever the tilt (the dot product takes x with x, y with
    y and z with z)."""
    K, R, t = stack([cam(F, W, H)] * 2)
    d, _ = plane_maps(W, H, 4.0)
    a = np.radians(deg)
    n = np.broadcast_to(np.array([0.0, np.sin(a), -np.cos(a)], np.float32), (H, W, 3)).copy()
    _, _, oc = oracle.consistency({0: d, 1: d}, {0: n, 1: n}, K, R, t, 0, [1], min_consistent=1)
    assert np.all(oc == 1)


@pytest.mark.parametrize("sx,sy", [(0.5, 0.5), (0.5, 1e-6), (1e-6, 0.5), (1 - 1e-6, 0.5), (0.5, 1 - 1e-6)])
def test_a_hole_texel_voids_the_four_cells_that_hold_it(sx, sy):
    """The neighbour's principal point shifted by (sx, sy): pixel (x, y) interpolates the
    cell of texels x..x+1, y..y+1.  A single hole texel (depth 0) at (hx, hy) makes the
    neighbour unusable at exactly the four pixels whose cells hold it, one for each corner
    of the cell.  With a shift of 1e-6 along one axis the far corners weigh almost nothing,
    so the interpolated depth would pass the depth test: there the corner check alone
    decides; with 1 - 1e-6 the near corners weigh almost nothing instead."""
    K0, R0, t0 = cam(F, W, H)
    K1 = K0.copy()
    K1[0, 2] += sx
    K1[1, 2] += sy
    K, R, t = stack([(K0, R0, t0), (K1, R0, t0)])
    d, n = plane_maps(W, H, 4.0)
    hy, hx = 20, 30
    d1 = d.copy()
    d1[hy, hx] = 0.0
    _, _, oc = oracle.consistency({0: d, 1: d1}, {0: n, 1: n}, K, R, t, 0, [1], min_consistent=1)
    expect = np.zeros((H, W), np.uint8)
    expect[:H - 1, :W - 1] = 1  # cells inside the image
    expect[hy - 1:hy + 1, hx - 1:hx + 1] = 0
    assert np.array_equal(oc, expect)
