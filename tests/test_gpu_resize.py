"""GPU parity of the window-resize scheme (Sec. III-C, Fig. 4, Table III; `tap_radius`):
integer spacings are bitwise the integer dilation on the GPU itself, fractional spacings
match the oracle teacher-forced and end to end (same bar as the other parity tests), also
under skewed intrinsics with windows leaving the sources."""
import dataclasses
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


@pytest.fixture(scope="module")
def tiny():
    return sg.workload_scene("tiny", device="cuda")


@pytest.fixture(scope="module")
def ctx(tiny):
    c = pm.Context(0)
    c.set_scene(tiny)
    yield c
    c.close()


def run(ctx, tiny, window, dilation, tap_radius, iters=2):
    srcs = list(range(1, len(tiny.images)))
    p = pm.Params(top_k=3, sigma_spatial_px=(window - 1) / 2.0, tap_radius=tap_radius)
    d, n, c = ctx.patchmatch(0, srcs, window, dilation, iters, p)
    return d.cpu().numpy(), n.cpu().numpy(), c.cpu().numpy()


@pytest.mark.parametrize("window,tap_radius,dilation", [(11, 5, 1), (21, 5, 2), (13, 3, 2)])
def test_integer_spacing_is_the_integer_dilation(ctx, tiny, window, tap_radius, dilation):
    a = run(ctx, tiny, window, 1, tap_radius)
    b = run(ctx, tiny, window, dilation, 0)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("window,tap_radius", [(13, 5), (17, 5), (19, 5), (15, 4)])
def test_fractional_spacing_parity(ctx, tiny, window, tap_radius):
    srcs = list(range(1, len(tiny.images)))
    sig = (window - 1) / 2.0
    pb = oracle.Problem.from_scene(tiny, window, 1, top_k=3, bilateral=True, sigma_s=sig, sigma_c=12.0,
                                   tap_radius=tap_radius)
    m = pb.valid_mask()
    # teacher-forced: the cost of the ground-truth planes
    planes = np.concatenate([tiny.gt_normal, tiny.gt_depth[..., None]], -1)
    ctx.prepare(0, srcs, window, 1, pm.Params(top_k=3, sigma_spatial_px=sig, tap_radius=tap_radius))
    gc, gpv, gok = [t.cpu().numpy() for t in ctx.eval_cost(torch.from_numpy(planes.astype(np.float32)).cuda(),
                                                          per_view=True)]
    oc, opv, ook = oracle.eval_cost(pb, planes.astype(np.float32).astype(np.float64))
    bit = (gc[m] == oc[m].astype(np.float32)).mean()
    say(f"window {window} / {tap_radius} taps per side: teacher-forced cost bitwise {bit:.6f}")
    assert bit >= 0.999
    # end to end, 2 iterations
    gd, _, gcost = run(ctx, tiny, window, 1, tap_radius)
    od, _, ocost = oracle.patchmatch(pb, 2)
    ok = (np.abs(gcost - ocost) <= 1e-4) & (np.abs(gd - od) <= 1e-3 * np.abs(od))
    say(f"  end to end: {ok[m].mean():.6f} within tolerance, cost bitwise {(gcost[m] == ocost[m]).mean():.6f}")
    assert ok[m].mean() >= 0.999


@pytest.mark.parametrize("window,tap_radius", [(17, 5), (15, 4)])
def test_fractional_spacing_parity_with_skewed_shifted_intrinsics(tiny, window, tap_radius):
    """Fractional spacing under intrinsics the images were not rendered with: skew and
    non-square pixels on every view, the sources' principal points moved 6.5 pixels so
    that windows leave each side of a source image.  Teacher-forced bitwise, end to end
    within the tolerances."""
    cams = []
    for i, c in enumerate(tiny.cams):
        K = c.K.copy()
        K[0, 1] = 3.9 if i % 2 else -2.4
        K[1, 1] *= 0.95 if i % 2 else 1.04
        if i > 0:
            dx, dy = [(6.5, 0.0), (-6.5, 0.0), (0.0, 6.5), (0.0, -6.5)][(i - 1) % 4]
            K[0, 2] += dx
            K[1, 2] += dy
        cams.append(dataclasses.replace(c, K=K))
    sc = dataclasses.replace(tiny, cams=cams)
    srcs = list(range(1, len(sc.images)))
    sig = (window - 1) / 2.0
    pb = oracle.Problem.from_scene(sc, window, 1, top_k=3, bilateral=True, sigma_s=sig, sigma_c=12.0,
                                   tap_radius=tap_radius)
    m = pb.valid_mask()
    planes = np.concatenate([sc.gt_normal, sc.gt_depth[..., None]], -1)
    c = pm.Context(0)
    try:
        c.set_scene(sc)
        c.prepare(0, srcs, window, 1, pm.Params(top_k=3, sigma_spatial_px=sig, tap_radius=tap_radius))
        gc, _, gok = [t.cpu().numpy() for t in c.eval_cost(torch.from_numpy(planes.astype(np.float32)).cuda(),
                                                           per_view=True)]
        gd, _, gcost = run(c, sc, window, 1, tap_radius)
    finally:
        c.close()
    oc, _, ook = oracle.eval_cost(pb, planes.astype(np.float32).astype(np.float64))
    bit = (gc[m] == oc[m].astype(np.float32)).mean()
    say(f"skewed, shifted; window {window} / {tap_radius} taps per side: teacher-forced cost bitwise {bit:.6f}, "
        f"valid views {ook[m].mean():.3f}")
    assert bit >= 0.999 and (gok.astype(bool) == ook).mean() >= 0.999
    assert ook[m].mean() < 0.99  # windows do leave the sources
    od, _, ocost = oracle.patchmatch(pb, 2)
    ok = (np.abs(gcost - ocost) <= 1e-4) & (np.abs(gd - od) <= 1e-3 * np.abs(od))
    say(f"  end to end: {ok[m].mean():.6f} within tolerance, cost bitwise {(gcost[m] == ocost[m]).mean():.6f}")
    assert ok[m].mean() >= 0.999


def test_resize_argument_errors(ctx, tiny):
    srcs = [1, 2]
    with pytest.raises(pm.PhimvsError):
        ctx.patchmatch(0, srcs, 21, 2, 1, pm.Params(tap_radius=5))  # needs dilation 1
    with pytest.raises(pm.PhimvsError):
        ctx.patchmatch(0, srcs, 11, 1, 1, pm.Params(tap_radius=6))  # above the window radius
    with pytest.raises(pm.PhimvsError):
        ctx.patchmatch(0, srcs, 11, 1, 1, pm.Params(tap_radius=-1))
