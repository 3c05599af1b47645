"""The steps after estimation on the batched workload's full-size depth maps (24
references from the 40-camera scene, 8 iterations): the consistency filter of three
references, one of each size, against the oracle (whole maps, bitwise), plane
hypotheses and Eq. 10 normals of a filtered 960x640 and a filtered 3200x2130 map
(whole maps, bitwise), fusion of the eight 960x640 maps and of all 24 maps (73 M
pixels) against the oracle's sequential walk (bitwise), and the invariants any fusion
must keep on all 24."""
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
def run():
    mv = sg.make_multiview_scene(seed=sg.SCENE_SEEDS["batched"], device="cuda")
    ctx = pm.Context(0)
    ctx.set_views(mv.images, mv.K, mv.R, mv.t, mv.depth_ranges)
    jobs = []
    for i, (ref, srcs, (win, dil)) in enumerate(zip(mv.refs, mv.sources, mv.windows)):
        H, W = mv.images[ref].shape
        jobs.append(dict(ref=ref, srcs=srcs, window=win, dilation=dil,
                         params=pm.Params(top_k=min(5, len(srcs)), seed=sg.PM_SEED + i),
                         depth=torch.empty((H, W), device="cuda"), normal=torch.empty((H, W, 3), device="cuda"),
                         cost=torch.empty((H, W), device="cuda")))
    ctx.patchmatch_batch(jobs, 8, use_graph=True)
    maps = [(j["ref"], j["depth"], j["normal"]) for j in jobs]
    index = {j["ref"]: i for i, j in enumerate(jobs)}
    filtered = []
    for i, j in enumerate(jobs):
        nb = [index[v] for v in j["srcs"] if v in index]
        d, n, c = ctx.filter(maps, i, nb)
        filtered.append((d.clone(), n.clone(), c.clone(), nb))
    torch.cuda.synchronize()
    yield mv, ctx, jobs, filtered
    ctx.close()


def test_filter_full_size(run):
    mv, ctx, jobs, filtered = run
    depths = {j["ref"]: j["depth"].cpu().numpy() for j in jobs}
    normals = {j["ref"]: j["normal"].cpu().numpy() for j in jobs}
    for i in (2, 1, 0):  # a 960x640, a 1600x1066 and a 3200x2130 reference
        nb = filtered[i][3]
        od, on, oc = oracle.consistency(depths, normals, mv.K, mv.R, mv.t, jobs[i]["ref"],
                                        [jobs[k]["ref"] for k in nb])
        gd, gn, gc = [t.cpu().numpy() for t in filtered[i][:3]]
        say(f"filter of job {i} ({gd.shape[1]}x{gd.shape[0]}, {len(nb)} neighbour maps): kept {(gd > 0).mean():.3f}, "
            f"bitwise depth {np.array_equal(gd, od)}, normal {np.array_equal(gn, on)}, count {np.array_equal(gc, oc)}")
        assert np.array_equal(gc, oc) and np.array_equal(gd, od) and np.array_equal(gn, on)


@pytest.mark.parametrize("i", [2, 0], ids=["960x640", "3200x2130"])
def test_phi_steps_full_size(run, i):
    mv, ctx, jobs, filtered = run
    d = filtered[i][0]
    hyp = ctx.phi_hypotheses(d).cpu().numpy().transpose(1, 2, 0)
    dn = d.cpu().numpy()
    o = oracle.phi_hypotheses(dn)
    say(f"hypotheses of job {i} ({dn.shape[1]}x{dn.shape[0]}): {(dn <= 0).mean():.3f} of pixels empty, "
        f"bitwise {np.array_equal(hyp, o)}")
    assert np.array_equal(hyp, o)
    nrm = ctx.phi_normals(jobs[i]["ref"], d).cpu().numpy()
    assert np.array_equal(nrm, oracle.phi_normals(dn, mv.K[jobs[i]["ref"]]))


def test_fusion_small_maps_against_oracle(run):
    mv, ctx, jobs, filtered = run
    sel = [i for i, j in enumerate(jobs) if mv.images[j["ref"]].shape == (640, 960)]
    maps = [(jobs[i]["ref"], filtered[i][0]) for i in sel]
    pts, sup, own = [t.cpu().numpy() for t in ctx.fuse(maps)]
    views = [jobs[i]["ref"] for i in sel]
    o = oracle.fuse([filtered[i][0].cpu().numpy() for i in sel], mv.K[views], mv.R[views], mv.t[views])
    say(f"fusion of {len(sel)} 960x640 maps: {(o[1] > 0).sum()} points, mean support {o[1][o[1] > 0].mean():.2f}; "
        f"bitwise points {np.array_equal(pts, o[0])}, support {np.array_equal(sup, o[1])}, owner {np.array_equal(own, o[2])}")
    assert np.array_equal(sup, o[1]) and np.array_equal(own, o[2]) and np.array_equal(pts, o[0])


def test_fusion_all_maps_against_oracle(run):
    """All 24 filtered maps (three sizes, 73 M pixels) against the oracle's sequential walk."""
    mv, ctx, jobs, filtered = run
    maps = [(j["ref"], filtered[i][0]) for i, j in enumerate(jobs)]
    pts, sup, own = [t.cpu().numpy() for t in ctx.fuse(maps)]
    views = [j["ref"] for j in jobs]
    o = oracle.fuse([filtered[i][0].cpu().numpy() for i in range(len(jobs))], mv.K[views], mv.R[views],
                    mv.t[views])
    say(f"fusion of all {len(jobs)} maps: {(o[1] > 0).sum()} points; bitwise points {np.array_equal(pts, o[0])}, "
        f"support {np.array_equal(sup, o[1])}, owner {np.array_equal(own, o[2])}")
    assert np.array_equal(sup, o[1]) and np.array_equal(own, o[2]) and np.array_equal(pts, o[0])


def test_fusion_all_maps_invariants(run):
    mv, ctx, jobs, filtered = run
    maps = [(j["ref"], filtered[i][0]) for i, j in enumerate(jobs)]
    pts, sup, own = ctx.fuse(maps)
    has = torch.cat([d.reshape(-1) > 0 for _, d in maps])
    assert int(sup.sum()) == int(has.sum())  # every pixel with depth ends in exactly one point
    assert bool((own[~has] == -1).all()) and bool((own[has] >= 0).all())
    counts = torch.bincount(own[has], minlength=own.numel())
    assert torch.equal(counts.to(torch.int32), sup)  # a point's support = the pixels naming it
    idx = torch.arange(own.numel(), device=own.device)
    assert bool((own[has] <= idx[has]).all())  # merged only into earlier pixels (or itself)
    assert bool(torch.isfinite(pts[sup > 0]).all()) and bool((pts[sup == 0] == 0).all())
    say(f"fusion of all {len(maps)} maps: {int(has.sum())} pixels with depth -> {int((sup > 0).sum())} points")
