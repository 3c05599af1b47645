"""Leaving out propagation candidates that cannot win (phimvs_params.score_all) changes
no result.  A candidate equal to an earlier candidate of the pixel, to the pixel's
current plane, or to a candidate that the previous propagation of the pixel's colour
offered it has a cost no lower than the pixel's stored cost; only a strictly lower cost
is taken.  On the 3200x2130 workload (10 sources, 11x11 taps, 8 iterations) the three
settings give bitwise the same depth, normal and cost at every pixel, while the number
of hypotheses scored falls (reported, and asserted to fall at each step); so do they on
the 160x120 workload, with one lane per pixel and with 16 lanes sharing each pixel.

Likewise, handing a tile's (pixel, candidate) work items to the lanes in order
of the candidates' inverse depth (phimvs_tuning.order_by_depth) instead of pixel order
gives bitwise the same maps: each item's cost is computed on its own, and the selection
reads the costs in slot order."""
import sys

import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_06165_amd as pm  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("workload,lanes", [("tiny", 0), ("tiny", 16), ("highres", 0)])
def test_skipping_changes_no_result(workload, lanes):
    scene = sg.workload_scene(workload, device="cuda")
    sol = sg.SOLVER[workload]
    ctx = pm.Context(0)
    try:
        ctx.set_scene(scene)
        srcs = list(range(1, len(scene.images)))
        res, hyps = [], []
        for level in (2, 1, 0):
            p = pm.Params(top_k=sol["top_k"], sigma_spatial_px=(sol["window"] - 1) / 2.0, seed=sg.PM_SEED,
                          score_all=level, lanes=lanes)
            ctx.diag_enable(pm.DIAG_COUNT)
            d, n, c = ctx.patchmatch(0, srcs, sol["window"], sol["dilation"], sol["iters"], p)
            n_hyp, _, _ = ctx.diag_read()
            ctx.diag_enable(0)
            res.append((d.clone(), n.clone(), c.clone()))
            hyps.append(n_hyp)
        say(f"{workload} (lanes {lanes}): hypotheses scored per depth map: every candidate {hyps[0]}, without duplicates and "
            f"current planes {hyps[1]} ({hyps[1] / hyps[0]:.3f}), also without candidates offered before "
            f"{hyps[2]} ({hyps[2] / hyps[0]:.3f})")
        for level, (d, n, c) in zip((1, 0), res[1:]):
            assert torch.equal(d, res[0][0]) and torch.equal(n, res[0][1]) and torch.equal(c, res[0][2]), level
        assert hyps[0] > hyps[1] > hyps[2]
    finally:
        ctx.close()


def test_score_all_is_validated():
    ctx = pm.Context(0)
    try:
        scene = sg.workload_scene("tiny", device="cuda")
        ctx.set_scene(scene)
        with pytest.raises(RuntimeError, match="score_all"):
            ctx.patchmatch(0, [1, 2], 11, 1, 1, pm.Params(score_all=3))
    finally:
        ctx.close()


@pytest.mark.parametrize("workload", ["tiny", "highres"])
def test_depth_ordered_work_lists_change_no_result(workload):
    scene = sg.workload_scene(workload, device="cuda")
    sol = sg.SOLVER[workload]
    ctx = pm.Context(0)
    try:
        ctx.set_scene(scene)
        srcs = list(range(1, len(scene.images)))
        p = pm.Params(top_k=sol["top_k"], sigma_spatial_px=(sol["window"] - 1) / 2.0, seed=sg.PM_SEED)
        res = []
        for order in (False, True):
            ctx.set_tuning(pm.Tuning(4, True, 4, order_by_depth=order))
            d, n, c = ctx.patchmatch(0, srcs, sol["window"], sol["dilation"], sol["iters"], p)
            res.append((d.clone(), n.clone(), c.clone()))
        (d0, n0, c0), (d1, n1, c1) = res
        same = torch.equal(d0, d1) and torch.equal(n0, n1) and torch.equal(c0, c1)
        say(f"{workload}: depth-ordered work lists give the pixel-order maps bitwise: {same}")
        assert same
    finally:
        ctx.close()
