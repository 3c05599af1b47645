"""GPU parity of the geometric-consistency filter (Sec. III-D) through the C ABI against
the oracle: analytic scenes at the thresholds, the depth maps of a batched multi-view
run, and the degenerate cases.  Every decision is taken in FP64 on both sides with the
same steps, so counts and outputs are expected to agree exactly; the bar is 99.9% of
pixels, the rest only where a tested quantity sits within 1e-9 of its threshold."""
import sys

import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_06165_amd as pm  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cam(f, W, H, tx=0.0, yaw=0.0):
    K = np.array([[f, 0.0, (W - 1) / 2.0], [0.0, f, (H - 1) / 2.0], [0.0, 0.0, 1.0]])
    c, s = np.cos(yaw), np.sin(yaw)
    R = np.array([[c, 0.0, -s], [0.0, 1.0, 0.0], [s, 0.0, c]])
    t = -R @ np.array([tx, 0.0, 0.0])
    return K, R, t


def run_both(ctx, cams, sizes, depths, normals, ref, nbrs, params=pm.FilterParams()):
    n = len(cams)
    K = np.stack([c[0] for c in cams])
    R = np.stack([c[1] for c in cams])
    t = np.stack([c[2] for c in cams])
    images = [np.zeros((h, w), np.uint8) for (w, h) in sizes]
    ctx.set_views(images, K, R, t, np.tile([1.0, 10.0], (n, 1)))
    views = sorted(depths)
    maps = [(v, torch.from_numpy(depths[v]).cuda(), torch.from_numpy(normals[v]).cuda()) for v in views]
    idx = {v: i for i, v in enumerate(views)}
    gd, gn, gc = ctx.filter(maps, idx[ref], [idx[v] for v in nbrs], params)
    od, on, oc = oracle.consistency(depths, normals, K, R, t, ref, nbrs, params.max_rel_depth, params.max_angle_deg,
                                    params.max_reproj_px, params.min_consistent)
    return (gd.cpu().numpy(), gn.cpu().numpy(), gc.cpu().numpy()), (od, on, oc)


def assert_same(g, o, tag):
    same = g[2] == o[2]
    say(f"{tag}: counts equal on {same.mean():.6f} of {same.size} pixels")
    assert same.mean() >= 0.999
    m = same
    assert np.array_equal(g[0][m], o[0][m]) and np.array_equal(g[1][m], o[1][m])


@pytest.fixture(scope="module")
def ctx():
    c = pm.Context(0)
    yield c
    c.close()


W, H, F = 64, 48, 100.0


def flat(Wm, Hm, Z):
    return (np.full((Hm, Wm), Z, np.float32),
            np.broadcast_to(np.array([0.0, 0.0, -1.0], np.float32), (Hm, Wm, 3)).copy())


@pytest.mark.parametrize("eps", [0.0203, 0.0206, -0.0205])
def test_depth_threshold(ctx, eps):
    d, n = flat(W, H, 4.0)
    dn = (d.astype(np.float64) * (1 + eps)).astype(np.float32)
    g, o = run_both(ctx, [cam(F, W, H)] * 2, [(W, H)] * 2, {0: d, 1: dn}, {0: n, 1: n}, 0, [1],
                    pm.FilterParams(min_consistent=1))
    assert_same(g, o, f"depth eps {eps}")


@pytest.mark.parametrize("b", [3.9, 4.15])
def test_reprojection_threshold(ctx, b):
    Wb = 400
    d, n = flat(Wb, H, 4.0)
    d2, _ = flat(Wb, H, 4.04)
    g, o = run_both(ctx, [cam(F, Wb, H), cam(F, Wb, H, tx=b)], [(Wb, H)] * 2, {0: d, 1: d2}, {0: n, 1: n}, 0, [1],
                    pm.FilterParams(min_consistent=1))
    assert_same(g, o, f"baseline {b}")


@pytest.mark.parametrize("axis", ["column", "row"])
@pytest.mark.parametrize("disp", [-2.4, -2.6, 2.6])
def test_normal_at_the_rounded_position_up_to_the_last_column_and_row(ctx, axis, disp):
    """The neighbour's normal is read at the rounded position; odd columns (rows) hold a
    normal that fails the test.  Negative disparities move the points right (down), so
    that with -2.6 a position within half a pixel of the last column (row) reads it."""
    Z = 4.0
    b = disp * Z / F
    Wb, Hb = (80, H) if axis == "column" else (W, 60)
    K0, R0, _ = cam(F, Wb, Hb)
    shift = np.array([b, 0.0, 0.0]) if axis == "column" else np.array([0.0, b, 0.0])
    cams = [(K0, R0, np.zeros(3)), (K0, R0, -R0 @ shift)]
    d, n = flat(Wb, Hb, Z)
    nb = n.copy()
    a = np.radians(40.0)
    if axis == "column":
        nb[:, 1::2] = [np.sin(a), 0.0, -np.cos(a)]
    else:
        nb[1::2, :] = [0.0, np.sin(a), -np.cos(a)]
    g, o = run_both(ctx, cams, [(Wb, Hb)] * 2, {0: d, 1: d}, {0: n, 1: nb}, 0, [1], pm.FilterParams(min_consistent=1))
    assert_same(g, o, f"rounded {axis}, disparity {disp}")
    edge = (slice(None), Wb - 4) if axis == "column" else (Hb - 4, slice(None))
    assert np.array_equal(g[2][edge], o[2][edge])


@pytest.mark.parametrize("sx,sy", [(1 - 1e-6, 0.5), (0.5, 1 - 1e-6), (0.5, 1e-6), (1e-6, 0.5)])
def test_a_hole_texel_at_each_corner_of_the_cell(ctx, sx, sy):
    """The neighbour's principal point shifted by (sx, sy) and one hole texel: the four
    pixels whose bilinear cells hold it lose the neighbour, also where the hole's weight
    is almost zero (the corner check alone decides)."""
    K0, R0, t0 = cam(F, W, H)
    K1 = K0.copy()
    K1[0, 2] += sx
    K1[1, 2] += sy
    d, n = flat(W, H, 4.0)
    d1 = d.copy()
    d1[20, 30] = 0.0
    g, o = run_both(ctx, [(K0, R0, t0), (K1, R0, t0)], [(W, H)] * 2, {0: d, 1: d1}, {0: n, 1: n}, 0, [1],
                    pm.FilterParams(min_consistent=1))
    assert_same(g, o, f"hole corner ({sx}, {sy})")
    assert np.array_equal(g[2][18:23, 28:33], o[2][18:23, 28:33])


def test_skewed_intrinsics(ctx):
    """Cameras with skew and non-square pixels (a fronto-parallel plane stays consistent
    under a sideways move whatever K is), one neighbour with holes and depth noise, so
    that the camera chain runs through every entry of K's inverse."""
    r = np.random.default_rng(5)
    K0, R0, _ = cam(F, W, H)
    Ka, Kb = K0.copy(), K0.copy()
    Ka[0, 1], Ka[1, 1] = 3.7, 0.92 * F
    Kb[0, 1], Kb[0, 0] = -2.2, 1.06 * F
    cams = [(Ka, R0, np.zeros(3)), (Ka, R0, -R0 @ np.array([0.05, 0.0, 0.0])),
            (Kb, R0, -R0 @ np.array([-0.04, 0.02, 0.0]))]
    d, n = flat(W, H, 4.0)
    d2 = (d * (1 + 0.012 * r.standard_normal(d.shape))).astype(np.float32)
    d2[r.uniform(size=d.shape) < 0.1] = 0.0
    for k in (1, 2):
        g, o = run_both(ctx, cams, [(W, H)] * 3, {0: d, 1: d, 2: d2}, {0: n, 1: n, 2: n}, 0, [1, 2],
                        pm.FilterParams(min_consistent=k))
        assert_same(g, o, f"skewed intrinsics, min {k}")
        assert 0 < (o[2] == 2).mean() < 1


def test_normals_holes_and_unusable_views(ctx):
    c0 = cam(F, W, H)
    c1 = cam(F, W, H, tx=0.05)
    c2 = cam(F, W, H, yaw=np.pi)
    d, n = flat(W, H, 4.0)
    holes = d.copy()
    holes[10:20, 10:20] = 0.0
    nb = n.copy()
    a = np.radians(40.0)
    nb[:, 1::2] = [np.sin(a), 0.0, -np.cos(a)]
    g, o = run_both(ctx, [c0, c1, c2, c0], [(W, H)] * 4, {0: d, 1: d, 2: d, 3: holes}, {0: n, 1: nb, 2: n, 3: n}, 0,
                    [1, 2, 3])
    assert_same(g, o, "normals / holes / behind")


def test_no_neighbours_and_min_zero(ctx):
    d, n = flat(W, H, 4.0)
    d[0, :5] = 0.0
    g, o = run_both(ctx, [cam(F, W, H)] * 2, [(W, H)] * 2, {0: d, 1: d}, {0: n, 1: n}, 0, [])
    assert_same(g, o, "no neighbours")
    assert np.all(g[2] == 0) and np.all(g[0] == 0)
    g, o = run_both(ctx, [cam(F, W, H)] * 2, [(W, H)] * 2, {0: d, 1: d}, {0: n, 1: n}, 0, [],
                    pm.FilterParams(min_consistent=0))
    assert_same(g, o, "min 0")
    assert np.array_equal(g[0], d)


def test_batched_depth_maps(ctx):
    """The depth maps of a batched run over a multi-view scene, each filtered against the
    other references among its sources."""
    mv = sg.make_multiview_scene(seed=41, grid=(2, 4), refs_per_class=2,
                                 classes=[(160, 120, 11, 1), (97, 66, 7, 1), (203, 150, 13, 2)],
                                 other_size=(128, 96), n_src_range=(3, 6), n_planes=5, device="cuda",
                                 master_size=(160, 120))
    ctx.set_views(mv.images, mv.K, mv.R, mv.t, mv.depth_ranges)
    jobs = [dict(ref=r, srcs=s, window=w, dilation=dl, params=pm.Params(top_k=min(3, len(s))))
            for r, s, (w, dl) in zip(mv.refs, mv.sources, mv.windows)]
    outs = ctx.patchmatch_batch(jobs, 3, use_graph=False)
    torch.cuda.synchronize()
    maps = [(j["ref"], o[0].contiguous(), o[1].contiguous()) for j, o in zip(jobs, outs)]
    depths = {j["ref"]: o[0].cpu().numpy() for j, o in zip(jobs, outs)}
    normals = {j["ref"]: o[1].cpu().numpy() for j, o in zip(jobs, outs)}
    total, checked = 0, 0
    for i, j in enumerate(jobs):
        nb_views = [v for v in j["srcs"] if v in depths]
        if not nb_views:
            continue
        nb_idx = [next(k for k, m in enumerate(maps) if m[0] == v) for v in nb_views]
        gd, gn, gc = ctx.filter(maps, i, nb_idx, pm.FilterParams(min_consistent=1))
        od, on, oc = oracle.consistency(depths, normals, mv.K, mv.R, mv.t, j["ref"], nb_views, min_consistent=1)
        assert_same((gd.cpu().numpy(), gn.cpu().numpy(), gc.cpu().numpy()), (od, on, oc), f"ref {j['ref']}")
        total += int((oc > 0).sum())
        checked += 1
    say(f"{checked} references filtered, {total} consistent pixel-neighbour hits")
    assert checked >= 2 and total > 0


def test_filter_argument_errors(ctx):
    d, n = flat(W, H, 4.0)
    ctx.set_views([np.zeros((H, W), np.uint8)] * 2, np.stack([cam(F, W, H)[0]] * 2), np.stack([np.eye(3)] * 2),
                  np.zeros((2, 3)), np.tile([1.0, 10.0], (2, 1)))
    maps = [(0, torch.from_numpy(d).cuda(), torch.from_numpy(n).cuda()), (1, torch.from_numpy(d).cuda(),
                                                                          torch.from_numpy(n).cuda())]
    with pytest.raises(pm.PhimvsError):
        ctx.filter(maps, 0, [0])  # the reference as its own neighbour
    with pytest.raises(pm.PhimvsError):
        ctx.filter(maps, 0, [5])  # no such map
    with pytest.raises(pm.PhimvsError):
        ctx.filter([(7, maps[0][1], maps[0][2])], 0, [])  # no such view
    with pytest.raises(pm.PhimvsError):
        ctx.filter(maps, 0, [1], pm.FilterParams(max_rel_depth=0.0))
