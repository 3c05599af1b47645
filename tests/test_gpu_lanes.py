"""The evaluate kernel with G lanes sharing each pixel (phimvs_params.lanes = G), for small
references that do not fill the GPU, against the oracle summing in the same lane-split
order (oracle.Problem(lanes=G)): teacher-forced costs per source, initialisation, one
half-sweep and whole tiny runs bitwise (>= 99.9%, measured 100%), ragged and limit
cases, and the argument rules."""
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

FRAC = 0.999


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = pm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def tiny():
    return sg.workload_scene("tiny", device="cuda"), sg.SOLVER["tiny"]


def params(window, top_k, lanes, bilateral=True):
    return pm.Params(top_k=top_k, bilateral=bilateral, sigma_spatial_px=(window - 1) / 2.0, seed=sg.PM_SEED,
                     lanes=lanes)


def problem(scene, window, dilation, top_k, lanes, bilateral=True):
    return oracle.Problem.from_scene(scene, window, dilation, top_k=top_k, bilateral=bilateral,
                                     sigma_s=(window - 1) / 2.0, sigma_c=12.0, seed=sg.PM_SEED, lanes=lanes)


@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
def test_teacher_forced_stages(ctx, tiny, lanes):
    scene, cfg = tiny
    win, dil, K = cfg["window"], cfg["dilation"], cfg["top_k"]
    ctx.set_scene(scene)
    n = len(scene.images) - 1
    ctx.prepare(0, list(range(1, n + 1)), win, dil, params(win, K, lanes))
    pb = problem(scene, win, dil, K, lanes)
    m = pb.valid_mask()
    P, _ = oracle.init(pb)
    gc, gpv, gvm = ctx.eval_cost(torch.tensor(P, dtype=torch.float32, device="cuda"), per_view=True)
    oc, opv, ovm = oracle.eval_cost(pb, P)
    bit = (gc.cpu().numpy() == oc.astype(np.float32)).mean()
    pv_bit = (gpv.cpu().numpy() == opv.astype(np.float32))[m].mean()
    vm = (gvm.cpu().numpy().astype(bool) == ovm)[m].mean()
    say(f"G={lanes}: cost bitwise {bit:.6f}, per-view bitwise {pv_bit:.6f}, validity agree {vm:.6f}")
    assert bit >= FRAC and pv_bit >= FRAC and vm >= FRAC
    ctx.init_planes()
    gp, gci = ctx.get_state()
    op, oci = oracle.init(pb)
    assert (np.all(gp.cpu().numpy() == op.astype(np.float32), -1)[m]).mean() >= FRAC
    assert (gci.cpu().numpy() == oci.astype(np.float32))[m].mean() >= FRAC
    ctx.set_state(torch.tensor(op, dtype=torch.float32, device="cuda"),
                  torch.tensor(oci, dtype=torch.float32, device="cuda"))
    ctx.step(1, 0)
    gp, gc2 = ctx.get_state()
    P2, C2 = oracle.halfsweep(pb, op, oci, 1, 0)
    pb_ = np.all(gp.cpu().numpy() == P2.astype(np.float32), -1)[m].mean()
    cb = (gc2.cpu().numpy() == C2.astype(np.float32))[m].mean()
    say(f"G={lanes}: half-sweep planes bitwise {pb_:.6f}, costs bitwise {cb:.6f}")
    assert pb_ >= FRAC and cb >= FRAC


@pytest.mark.parametrize("lanes", [2, 16])
def test_hypothesis_count_matches_one_lane(ctx, tiny, lanes):
    """The diagnostic count of scored (pixel, hypothesis) pairs is the same whether one
    lane or G lanes score each pixel: from the same state the candidate kernels offer the
    same candidates (an initialisation, then a half-sweep from the oracle's state)."""
    scene, cfg = tiny
    win, dil, K = cfg["window"], cfg["dilation"], cfg["top_k"]
    ctx.set_scene(scene)
    srcs = list(range(1, len(scene.images)))
    pb = problem(scene, win, dil, K, 0)
    P, C = oracle.init(pb)
    counts = {}
    for g in (0, lanes):
        ctx.prepare(0, srcs, win, dil, params(win, K, g))
        ctx.diag_enable(pm.DIAG_COUNT)
        ctx.init_planes()
        n_init, _, _ = ctx.diag_read()
        ctx.set_state(torch.tensor(P, dtype=torch.float32, device="cuda"),
                      torch.tensor(C, dtype=torch.float32, device="cuda"))
        ctx.diag_enable(pm.DIAG_COUNT)
        ctx.step(1, 0)
        n_step, _, _ = ctx.diag_read()
        ctx.diag_enable(0)
        counts[g] = (n_init, n_step)
    say(f"G={lanes}: scored pairs (initialisation, half-sweep) {counts[lanes]}, one lane {counts[0]}")
    assert counts[lanes] == counts[0] and counts[0][1] > counts[0][0] > 0


@pytest.mark.parametrize("lanes", [4, 16])
def test_tiny_run(ctx, tiny, lanes):
    scene, cfg = tiny
    win, dil, K, iters = cfg["window"], cfg["dilation"], cfg["top_k"], cfg["iters"]
    ctx.set_scene(scene)
    n = len(scene.images) - 1
    d, nrm, c = ctx.patchmatch(0, list(range(1, n + 1)), win, dil, iters, params(win, K, lanes))
    torch.cuda.synchronize()
    pb = problem(scene, win, dil, K, lanes)
    od, on, oc = oracle.patchmatch(pb, iters)
    m = pb.valid_mask()
    gd, gc = d.cpu().numpy(), c.cpu().numpy()
    bit_c = (gc == oc)[m].mean()
    bit_d = (gd == od)[m].mean()
    say(f"G={lanes}: tiny run cost bitwise {bit_c:.6f}, depth bitwise {bit_d:.6f}")
    assert bit_c >= FRAC and bit_d >= FRAC
    # against the one-lane order: only the FP32 rounding of the sums differs
    d1, _, c1 = oracle.patchmatch(problem(scene, win, dil, K, 1), iters)
    same = (np.abs(gd - d1) <= 1e-3 * np.abs(d1))[m].mean()
    say(f"G={lanes}: depth within 1e-3 of the one-lane order on {same:.5f} of the pixels")
    assert same >= 0.99


@pytest.mark.parametrize("W,H,n_src,window,dilation,top_k,lanes", [
    (133, 67, 2, 7, 1, 0, 16),     # ragged width and height
    (130, 61, 3, 9, 2, 1, 8),      # dilation 2, best-1
    (97, 50, 1, 7, 3, 0, 2),       # one source, dilation 3
    (100, 72, 2, 61, 2, 0, 4),     # the largest window: 31 x 31 taps over a 30-pixel radius
    (96, 64, 12, 7, 1, 5, 16),     # the most sources
])
def test_edge_cases(ctx, W, H, n_src, window, dilation, top_k, lanes):
    scene = sg.make_scene(100 + W + H, sg.tiny_config(W, H, n_src=n_src, n_planes=3, n_textureless=1), device="cuda")
    ctx.set_scene(scene)
    srcs = list(range(1, n_src + 1))
    d, nrm, c = ctx.patchmatch(0, srcs, window, dilation, 2, params(window, top_k, lanes))
    torch.cuda.synchronize()
    pb = problem(scene, window, dilation, top_k, lanes)
    od, on, oc = oracle.patchmatch(pb, 2)
    m = pb.valid_mask()
    gd, gc = d.cpu().numpy(), c.cpu().numpy()
    ok = ((np.abs(gc - oc) <= 1e-4) & (np.abs(gd - od) <= 1e-3 * np.abs(od)))[m].mean()
    say(f"edge {W}x{H} n={n_src} win={window} s={dilation} K={top_k} G={lanes}: within tolerance {ok:.6f}, "
        f"cost bitwise {(gc == oc)[m].mean():.6f}")
    assert ok >= FRAC
    assert np.all(gd[~m] == 0) and np.all(gc[~m] == 2.0)


def test_lane_arguments(ctx, tiny):
    scene, cfg = tiny
    ctx.set_scene(scene)
    with pytest.raises(pm.PhimvsError) as e:
        ctx.patchmatch(0, [1, 2], 11, 1, 1, pm.Params(lanes=3))
    assert e.value.code == -1
    with pytest.raises(pm.PhimvsError) as e:
        ctx.patchmatch(0, [1, 2], 11, 1, 1, pm.Params(lanes=32))
    assert e.value.code == -1
    with pytest.raises(pm.PhimvsError) as e:
        ctx.patchmatch(0, [1, 2], 11, 1, 1, pm.Params(lanes=4, tap_radius=3))
    assert e.value.code == -5
    H, W = scene.images[0].shape
    job = dict(ref=0, srcs=[1, 2], window=11, dilation=1, params=pm.Params(lanes=4),
               depth=torch.empty((H, W), device="cuda"), normal=torch.empty((H, W, 3), device="cuda"),
               cost=torch.empty((H, W), device="cuda"))
    with pytest.raises(pm.PhimvsError) as e:
        ctx.patchmatch_batch([job], 1)
    assert e.value.code == -5
