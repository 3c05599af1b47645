"""Batched execution: every job of a batch (references of different sizes, source
counts and dilations, in shared launches, eager or replayed from a hipGraph, under
every launch configuration) gives bitwise the result of its own single-view run, which
the parity tests tie to the oracle."""
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
def mv():
    return sg.make_multiview_scene(seed=41, grid=(2, 4), refs_per_class=2,
                                   classes=[(160, 120, 11, 1), (97, 66, 7, 1), (203, 150, 13, 2)],
                                   other_size=(128, 96), n_src_range=(2, 5), n_planes=5, device="cuda",
                                   master_size=(160, 120))


@pytest.fixture(scope="module")
def ctx(mv):
    c = pm.Context(0)
    c.set_views(mv.images, mv.K, mv.R, mv.t, mv.depth_ranges)
    yield c
    c.close()


def jobs_of(mv):
    jobs = []
    for i, (ref, srcs, (win, dil)) in enumerate(zip(mv.refs, mv.sources, mv.windows)):
        jobs.append(dict(ref=ref, srcs=srcs, window=win, dilation=dil,
                         params=pm.Params(top_k=min(3, len(srcs)), seed=1000 + i)))
    return jobs


def single_runs(ctx, jobs, iters):
    outs = []
    for j in jobs:
        d, n, c = ctx.patchmatch(j["ref"], j["srcs"], j["window"], j["dilation"], iters, j["params"])
        outs.append((d.clone(), n.clone(), c.clone()))
    torch.cuda.synchronize()
    return outs


TUNINGS = [pm.Tuning(4, False, 0), pm.Tuning(4, True, 3), pm.Tuning(2, True, 4), pm.Tuning(1, False, 0),
           pm.Tuning(2, False, 0), pm.Tuning(4, True, 4, order_by_depth=True),
           pm.Tuning(1, False, 0, order_by_depth=True)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: f"rows{t.tile_rows}-p{int(t.persistent)}-{t.wgs_per_cu}"
                                                          f"{'-depth' if t.order_by_depth else ''}")
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_runs(ctx, mv, tuning, use_graph):
    iters = 2
    jobs = jobs_of(mv)
    ctx.set_tuning(tuning)
    ref = single_runs(ctx, jobs, iters)
    outs = ctx.patchmatch_batch(jobs, iters, use_graph=use_graph)
    torch.cuda.synchronize()
    for k, ((d, n, c), (rd, rn, rc)) in enumerate(zip(outs, ref)):
        assert torch.equal(d, rd) and torch.equal(n, rn) and torch.equal(c, rc), f"job {k}"
    say(f"batch of {len(jobs)} jobs == single runs ({tuning}, graph={use_graph})")


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_with_per_job_cost_parameters(ctx, mv, use_graph):
    """Every job with its own colour and spatial sigmas, variance and cost floors, top-K,
    bilateral switch and seed: the batch equals the single runs bitwise, so each job's
    parameters reach its own tiles only."""
    jobs = jobs_of(mv)
    for i, j in enumerate(jobs):
        j["params"] = pm.Params(top_k=i % (len(j["srcs"]) + 1), bilateral=i % 5 != 3, sigma_spatial_px=1.5 + 0.7 * i,
                                sigma_color=4.0 + 3.5 * i, eps_var=10.0 ** -(3 + i % 4), eps_cost=10.0 ** -(1 + i % 5),
                                seed=(i + 1) * 0x9E3779B97F4A7C15 % (1 << 64))
    ctx.set_tuning(pm.Tuning(4, True, 4))
    ref = single_runs(ctx, jobs, 2)
    outs = ctx.patchmatch_batch(jobs, 2, use_graph=use_graph)
    torch.cuda.synchronize()
    for k, ((d, n, c), (rd, rn, rc)) in enumerate(zip(outs, ref)):
        assert torch.equal(d, rd) and torch.equal(n, rn) and torch.equal(c, rc), f"job {k}"
    say(f"batch of {len(jobs)} jobs with per-job parameters == single runs (graph={use_graph})")
    if use_graph:
        return
    for k in (3, 4):  # job 3 without the bilateral weights
        j, (d, n, c) = jobs[k], outs[k]
        p = j["params"]
        views = [j["ref"]] + list(j["srcs"])
        pb = oracle.Problem([mv.images[v] for v in views], mv.K[views], mv.R[views], mv.t[views],
                            mv.depth_ranges[j["ref"]], j["window"], j["dilation"], top_k=p.top_k,
                            bilateral=p.bilateral, sigma_s=p.sigma_spatial_px, sigma_c=p.sigma_color,
                            eps_v=p.eps_var, eps_c=p.eps_cost, seed=p.seed)
        od, on, oc = oracle.patchmatch(pb, 2)
        m = pb.valid_mask()
        gc, gd = c.cpu().numpy(), d.cpu().numpy()
        ok = (np.abs(gc - oc) <= 1e-4) & (np.abs(gd - od) <= 1e-3 * np.abs(od))
        say(f"  job {k} vs oracle: {ok[m].mean():.6f} within tolerance, bitwise {(gc[m] == oc[m]).mean():.6f}")
        assert ok[m].mean() >= 0.999


@pytest.mark.parametrize("use_graph", [False, True])
def test_depth_ordered_batch_equals_pixel_order_singles(ctx, mv, use_graph):
    """The batch in depth order equals the single runs in pixel order, job by job."""
    iters = 2
    jobs = jobs_of(mv)
    ctx.set_tuning(pm.Tuning(4, True, 4))
    ref = single_runs(ctx, jobs, iters)
    ctx.set_tuning(pm.Tuning(4, True, 4, order_by_depth=True))
    outs = ctx.patchmatch_batch(jobs, iters, use_graph=use_graph)
    torch.cuda.synchronize()
    for k, ((d, n, c), (rd, rn, rc)) in enumerate(zip(outs, ref)):
        assert torch.equal(d, rd) and torch.equal(n, rn) and torch.equal(c, rc), f"job {k}"
    say(f"depth-ordered batch of {len(jobs)} jobs == pixel-order single runs (graph={use_graph})")


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("order_by_depth", [False, True])
def test_batch_mixing_window_resize_and_integer_jobs(ctx, mv, use_graph, order_by_depth):
    """A launch that holds a window-resize job runs the fractional-spacing kernel instance
    for every job in it: each job, resize or integer spacing, still equals its single run
    bitwise (the single runs in pixel order; the batch in either order)."""
    iters = 2
    jobs = jobs_of(mv)
    j0 = jobs[0]  # radius 6 sampled by 5 taps per side (spacing 6/5)
    jobs[0] = dict(j0, window=13, dilation=1,
                   params=pm.Params(top_k=j0["params"].top_k, seed=j0["params"].seed, tap_radius=5))
    ctx.set_tuning(pm.Tuning(4, False, 0))
    ref = single_runs(ctx, jobs, iters)
    ctx.set_tuning(pm.Tuning(4, False, 0, order_by_depth=order_by_depth))
    outs = ctx.patchmatch_batch(jobs, iters, use_graph=use_graph)
    torch.cuda.synchronize()
    for k, ((d, n, c), (rd, rn, rc)) in enumerate(zip(outs, ref)):
        assert torch.equal(d, rd) and torch.equal(n, rn) and torch.equal(c, rc), f"job {k}"
    say(f"mixed batch ({len(jobs)} jobs, one window-resize) == single runs (graph={use_graph}, "
        f"depth order {order_by_depth})")


def test_graph_replays_with_eager_work_between(ctx, mv):
    iters = 2
    jobs = jobs_of(mv)
    ctx.set_tuning(pm.Tuning(4, True, 2))
    first = [tuple(t.clone() for t in o) for o in ctx.patchmatch_batch(jobs, iters, use_graph=False)]
    torch.cuda.synchronize()
    outs = [dict(depth=torch.empty_like(o[0]), normal=torch.empty_like(o[1]), cost=torch.empty_like(o[2]))
            for o in first]
    gjobs = [dict(j, **o) for j, o in zip(jobs, outs)]
    for rep in range(3):
        for o in outs:
            o["depth"].fill_(-1.0)
            o["cost"].fill_(-1.0)
        junk = torch.randn(1 << 20, device="cuda").sum()  # the program's own eager work
        ctx.patchmatch_batch(gjobs, iters, use_graph=True)
        torch.cuda.synchronize()
        float(junk)
        for k, (o, f) in enumerate(zip(outs, first)):
            assert torch.equal(o["depth"], f[0]) and torch.equal(o["cost"], f[2]), f"replay {rep} job {k}"
    say("graph replays x3 equal the eager run")


def test_batch_job_against_oracle(ctx, mv):
    """One job of the batch checked directly against the CPU oracle (end to end)."""
    jobs = jobs_of(mv)
    j = jobs[1]
    ctx.set_tuning(pm.Tuning(4, True, 3))
    outs = ctx.patchmatch_batch(jobs, 2, use_graph=True)
    torch.cuda.synchronize()
    d, n, c = outs[1]
    views = [j["ref"]] + list(j["srcs"])
    pb = oracle.Problem([mv.images[v] for v in views], mv.K[views], mv.R[views], mv.t[views],
                        mv.depth_ranges[j["ref"]], j["window"], j["dilation"], top_k=j["params"].top_k,
                        bilateral=True, sigma_s=(j["window"] - 1) / 2.0, seed=j["params"].seed)
    od, on, oc = oracle.patchmatch(pb, 2)
    m = pb.valid_mask()
    gc = c.cpu().numpy()
    gd = d.cpu().numpy()
    ok = (np.abs(gc - oc) <= 1e-4) & (np.abs(gd - od) <= 1e-3 * np.abs(od))
    say(f"batch job vs oracle: {ok[m].mean():.6f} within tolerance, bitwise {(gc[m] == oc[m]).mean():.6f}")
    assert ok[m].mean() >= 0.999


def test_autotune_picks_a_measured_configuration(ctx, mv):
    jobs = jobs_of(mv)
    best, allr = ctx.autotune(jobs, iters=1)
    assert len(allr) >= 5 and all(r.ms > 0 for r in allr)
    assert best.ms == min(r.ms for r in allr)
    say("autotune: " + ", ".join(f"rows{r.tile_rows}/p{int(r.persistent)}/{r.wgs_per_cu}: {r.ms:.3f} ms" for r in allr))
    # the chosen configuration still reproduces the single-view results
    ref = single_runs(ctx, jobs, 1)
    outs = ctx.patchmatch_batch(jobs, 1, use_graph=True)
    torch.cuda.synchronize()
    for (d, n, c), (rd, rn, rc) in zip(outs, ref):
        assert torch.equal(d, rd) and torch.equal(c, rc)


def test_batch_argument_errors(ctx, mv):
    jobs = jobs_of(mv)
    bad = dict(jobs[0], srcs=[jobs[0]["ref"]])
    with pytest.raises(pm.PhimvsError):
        ctx.patchmatch_batch([jobs[1], bad], 1)
    with pytest.raises(pm.PhimvsError):
        ctx.set_tuning(pm.Tuning(3, False, 0))
    with pytest.raises(pm.PhimvsError):
        ctx.set_tuning(pm.Tuning(4, True, 0))


def test_batch_with_mixed_candidate_skipping(ctx, mv):
    """Jobs of one batch may leave out different kinds of candidates that cannot win
    (phimvs_params.score_all 0, 1, 2): each job's result is still bitwise its single run
    with every such candidate left out."""
    iters = 3
    jobs = jobs_of(mv)
    ctx.set_tuning(pm.Tuning(4, False, 0))
    ref = single_runs(ctx, jobs, iters)
    mixed = []
    for i, j in enumerate(jobs):
        p = j["params"]
        mixed.append(dict(j, params=pm.Params(top_k=p.top_k, seed=p.seed, score_all=i % 3)))
    outs = ctx.patchmatch_batch(mixed, iters, use_graph=False)
    torch.cuda.synchronize()
    for i, ((d, n, c), (rd, rn, rc)) in enumerate(zip(outs, ref)):
        assert torch.equal(d, rd) and torch.equal(n, rn) and torch.equal(c, rc), f"job {i} (score_all {i % 3})"
    say(f"{len(jobs)} jobs with score_all 0/1/2 mixed: bitwise equal to their single runs")
