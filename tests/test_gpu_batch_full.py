"""The batched workload at its full size (24 references: 8 x 3200x2130, 8 x 1600x1066,
8 x 960x640 from a 40-camera scene, 6-12 sources each, 8 iterations, shared launches
replayed from a hipGraph): the final cost of every job re-evaluated by the oracle at
sampled pixels (teacher-forced on the GPU's own output planes), and the properties every
output pixel must have checked on all 73 M pixels."""
import sys

import numpy as np
import pytest

import oracle
import scenegen as sg
from fp64_error import report as fp64_report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_06165_amd as pm  # noqa: E402

SAMPLES_PER_JOB = 250
THREADS = oracle.default_threads()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_full_batched_workload_sampled():
    mv = sg.make_multiview_scene(seed=sg.SCENE_SEEDS["batched"], device="cuda")
    ctx = pm.Context(0)
    try:
        ctx.set_views(mv.images, mv.K, mv.R, mv.t, mv.depth_ranges)
        jobs = []
        for i, (ref, srcs, (win, dil)) in enumerate(zip(mv.refs, mv.sources, mv.windows)):
            H, W = mv.images[ref].shape
            jobs.append(dict(ref=ref, srcs=srcs, window=win, dilation=dil,
                             params=pm.Params(top_k=min(5, len(srcs)), seed=sg.PM_SEED + i),
                             depth=torch.empty((H, W), device="cuda"), normal=torch.empty((H, W, 3), device="cuda"),
                             cost=torch.empty((H, W), device="cuda")))
        ctx.set_tuning(pm.Tuning(4, False, 0))
        ctx.patchmatch_batch(jobs, 8, use_graph=True)
        torch.cuda.synchronize()
        say(f"batch of {len(jobs)} done")
        rng = np.random.default_rng(7)
        n_ok = n_all = 0
        g_all, o64_all = [], []
        for i, j in enumerate(jobs):
            d = j["depth"].cpu().numpy()
            nm = j["normal"].cpu().numpy()
            c = j["cost"].cpu().numpy()
            views = [j["ref"]] + list(j["srcs"])
            pb = oracle.Problem([mv.images[v] for v in views], mv.K[views], mv.R[views], mv.t[views],
                                mv.depth_ranges[j["ref"]], j["window"], j["dilation"], top_k=j["params"].top_k,
                                bilateral=True, sigma_s=(j["window"] - 1) / 2.0, seed=j["params"].seed)
            m = pb.valid_mask()
            # properties of every pixel
            assert np.all((c >= 0) & (c <= pm.COST_MAX))
            assert np.all(d[~m] == 0) and np.all(c[~m] == pm.COST_MAX) and np.all(nm[~m] == 0)
            lo, hi = mv.depth_ranges[j["ref"]]
            assert np.all((d[m] >= np.float32(lo)) & (d[m] <= np.float32(hi)))
            assert np.allclose(np.linalg.norm(nm[m], axis=-1), 1.0, atol=1e-5)
            # teacher-forced: the oracle's cost of the output plane at sampled pixels
            idx = np.flatnonzero(m.ravel())
            sub = rng.choice(idx, size=SAMPLES_PER_JOB, replace=False).astype(np.int32)
            planes = np.concatenate([nm, d[..., None]], -1).astype(np.float64)
            oc, _, _ = oracle.eval_cost(pb, planes, subset=sub, threads=THREADS)
            o64, _, _ = oracle.eval_cost(pb, planes, fp64=True, subset=sub, threads=THREADS)
            g = c.ravel()[sub]
            o = oc.ravel()[sub]
            ok = np.abs(g - o) <= 1e-4
            n_ok += int(ok.sum())
            n_all += len(sub)
            g_all.append(g)
            o64_all.append(o64.ravel()[sub])
            say(f"job {i} ({d.shape[1]}x{d.shape[0]}, {len(j['srcs'])} sources, s={j['dilation']}): "
                f"{ok.mean():.4f} of {len(sub)} sampled costs within 1e-4, bitwise {(g == o.astype(np.float32)).mean():.4f}")
        say(f"all jobs: {n_ok} of {n_all} sampled costs within 1e-4")
        fp64_report("all jobs: teacher-forced cost at the sampled pixels", np.concatenate(g_all),
                    np.concatenate(o64_all))
        assert n_ok >= 0.999 * n_all
    finally:
        ctx.close()
