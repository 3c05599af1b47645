"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same
seeded inputs.  Bar (per result): |cost_gpu - cost_oracle| <= 1e-4 and
|depth_gpu - depth_oracle| <= 1e-3 depth_oracle on >= 99.9% of valid pixels; the
teacher-forced stages are expected to agree bitwise and are held to that on >= 99.9%.
The FP64 oracle's distance to each FP32 result is printed."""
import dataclasses
import os
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

COST_TOL = 1e-4
DEPTH_TOL = 1e-3
FRAC = 0.999
THREADS = oracle.default_threads()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = pm.Context(0)
    yield c
    c.close()


def params_for(window, top_k, bilateral=True, seed=0x5EED):
    return pm.Params(top_k=top_k, bilateral=bilateral, sigma_spatial_px=(window - 1) / 2.0, seed=seed)


def oracle_problem(scene, window, dilation, top_k, bilateral=True, seed=0x5EED):
    return oracle.Problem.from_scene(scene, window, dilation, top_k=top_k, bilateral=bilateral,
                                     sigma_s=(window - 1) / 2.0, sigma_c=12.0, seed=seed)


def compare(tag, gpu_cost, orc_cost, mask, gpu_depth=None, orc_depth=None):
    gc, oc = gpu_cost[mask], orc_cost[mask]
    ok = np.abs(gc - oc) <= COST_TOL
    bit = (gc.astype(np.float32) == oc.astype(np.float32)).mean() if gc.size else 1.0
    msg = f"{tag}: n={gc.size} cost within tol {ok.mean() if gc.size else 1:.6f} bitwise {bit:.6f}"
    if gpu_depth is not None:
        gd, od = gpu_depth[mask], orc_depth[mask]
        okd = np.abs(gd - od) <= DEPTH_TOL * np.abs(od)
        msg += f" depth within tol {okd.mean() if gd.size else 1:.6f}"
        ok = ok & okd
    say(msg)
    return ok.mean() if gc.size else 1.0, bit


# ----------------------------------------------------------------------------- fast reciprocal
def test_fast_reciprocal_is_correctly_rounded(ctx):
    """Every float w with |w| in [2^-100, 2^100]: the kernels' 1/w equals the correctly
    rounded reciprocal."""
    lo = (127 - 100) << 23
    hi = (127 + 100) << 23
    total = 0
    for sign in (0, 0x80000000):
        first = lo
        while first < hi:
            count = min(1 << 28, hi - first)
            mism, ex = ctx.check_reciprocal(sign | first, count)
            assert mism == 0, f"mismatch at bits {ex:#x}"
            total += count
            first += count
    say(f"reciprocal checked on {total} floats")


# ----------------------------------------------------------------------------- tiny workload
@pytest.fixture(scope="module")
def tiny():
    scene = sg.workload_scene("tiny", device="cuda")
    cfg = sg.SOLVER["tiny"]
    return scene, cfg


def _prep(ctx, scene, cfg, bilateral=True, seed=0x5EED):
    ctx.set_scene(scene)
    n = len(scene.images) - 1
    ctx.prepare(0, list(range(1, n + 1)), cfg["window"], cfg["dilation"],
                params_for(cfg["window"], cfg["top_k"], bilateral, seed))
    return oracle_problem(scene, cfg["window"], cfg["dilation"], cfg["top_k"], bilateral, seed)


def _test_planes(scene, pb, rng):
    H, W = pb.H, pb.W
    init_p, _ = oracle.init(pb)
    gt = np.zeros((H, W, 4))
    gt[..., :3] = scene.gt_normal
    gt[..., 3] = scene.gt_depth
    rnd = np.zeros((H, W, 4))
    n = rng.normal(size=(H, W, 3))
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    rnd[..., :3] = n  # about half of them face away (cost C_max expected)
    lo, hi = scene.depth_range
    rnd[..., 3] = rng.uniform(lo, hi, size=(H, W))
    # planes without a depth (NaN): whole rows (entire waves) and 30% of the other pixels
    gtn = gt.astype(np.float32).astype(np.float64)
    gtn[20:60, :, 3] = np.nan
    gtn[..., 3][rng.uniform(size=(H, W)) < 0.3] = np.nan
    return {"init": init_p, "gt": gt.astype(np.float32).astype(np.float64),
            "random": rnd.astype(np.float32).astype(np.float64), "gt_nan_depths": gtn}


def test_eval_cost_parity_tiny(ctx, tiny):
    scene, cfg = tiny
    pb = _prep(ctx, scene, cfg)
    m = pb.valid_mask()
    for name, planes in _test_planes(scene, pb, np.random.default_rng(0)).items():
        gc, gpv, gvm = ctx.eval_cost(torch.tensor(planes, dtype=torch.float32, device="cuda"), per_view=True)
        oc, opv, ovm = oracle.eval_cost(pb, planes)
        frac, bit = compare(f"eval[{name}]", gc.cpu().numpy(), oc, np.ones_like(m))
        assert frac >= FRAC and bit >= FRAC
        vm_agree = (gvm.cpu().numpy().astype(bool) == ovm).mean()
        pv_ok = (np.abs(gpv.cpu().numpy() - opv) <= COST_TOL).mean()
        say(f"  per-view validity agree {vm_agree:.6f}, per-view cost within tol {pv_ok:.6f}")
        assert vm_agree >= FRAC and pv_ok >= FRAC
        # the FP64 oracle's distance to the FP32 cost (teacher-forced)
        o64, _, _ = oracle.eval_cost(pb, planes, fp64=True)
        fp64_report(f"  eval[{name}]", gc.cpu().numpy(), o64, m)


def _with_intrinsics(scene, kind):
    """The scene with other intrinsics than its images were rendered with: "skew" (skew and
    non-square pixels on every view), "shifted" (the sources' principal points moved 6.5
    pixels right, left, down and up), "general" (every entry of every K perturbed)."""
    rng = np.random.default_rng(7)
    cams = []
    for i, c in enumerate(scene.cams):
        K = c.K.copy()
        if kind == "skew":
            K[0, 1] = 4.3 if i % 2 else -2.1
            K[1, 1] *= 0.93 if i % 2 else 1.07
        elif kind == "shifted" and i > 0:
            dx, dy = [(6.5, 0.0), (-6.5, 0.0), (0.0, 6.5), (0.0, -6.5)][(i - 1) % 4]
            K[0, 2] += dx
            K[1, 2] += dy
        elif kind == "general":
            K = K + rng.normal(size=(3, 3)) * np.array([[2.0, 2.0, 2.0], [2.0, 2.0, 2.0], [1e-4, 1e-4, 0.02]])
        cams.append(dataclasses.replace(c, K=K))
    return dataclasses.replace(scene, cams=cams)


@pytest.mark.parametrize("kind", ["skew", "shifted", "general"])
def test_eval_cost_parity_with_other_intrinsics(ctx, tiny, kind):
    """Teacher-forced costs under intrinsics the images were not rendered with (both sides
    take K as given, so they must still agree): a skewed K with non-square pixels on every
    view; the sources' principal points moved 6.5 pixels right, left, down and up, so that
    windows leave each side of a source image; general invertible matrices (every entry
    non-zero), so that every cofactor of K's inverse matters."""
    scene, cfg = tiny
    sc = _with_intrinsics(scene, kind)
    pb = _prep(ctx, sc, cfg)
    m = pb.valid_mask()
    for name, planes in _test_planes(sc, pb, np.random.default_rng(1)).items():
        say(f"intrinsics {kind}, planes {name}")
        gc, gpv, gvm = ctx.eval_cost(torch.tensor(planes, dtype=torch.float32, device="cuda"), per_view=True)
        oc, opv, ovm = oracle.eval_cost(pb, planes)
        frac, bit = compare(f"eval[{kind}/{name}]", gc.cpu().numpy(), oc, np.ones_like(m))
        assert frac >= FRAC and bit >= FRAC
        vm = ovm[m]
        say(f"  valid views {vm.mean():.3f} of {vm.size}")
        assert (gvm.cpu().numpy().astype(bool) == ovm).mean() >= FRAC
        assert (np.abs(gpv.cpu().numpy() - opv) <= COST_TOL).mean() >= FRAC
        if kind == "shifted" and name == "gt":
            assert 0.3 < vm.mean() < 0.99  # windows do leave the sources


@pytest.mark.parametrize("sc,ss,ev,ec,k", [(5.5, 2.3, 2e-3, 0.05, 2), (30.0, 7.5, 1e-6, 1e-6, 0)])
def test_parity_with_other_cost_parameters(ctx, tiny, sc, ss, ev, ec, k):
    """Colour and spatial sigmas, the variance floor, the cost floor of Eq. 5 and top-K
    away from their defaults: teacher-forced costs on every plane set and the whole tiny
    run against the oracle with the same parameters."""
    scene, cfg = tiny
    n = len(scene.images) - 1
    p = pm.Params(top_k=k, sigma_spatial_px=ss, sigma_color=sc, eps_var=ev, eps_cost=ec, seed=0x5EED)
    ctx.set_scene(scene)
    ctx.prepare(0, list(range(1, n + 1)), cfg["window"], cfg["dilation"], p)
    pb = oracle.Problem.from_scene(scene, cfg["window"], cfg["dilation"], top_k=k, bilateral=True, sigma_s=ss,
                                   sigma_c=sc, eps_v=ev, eps_c=ec, seed=0x5EED)
    m = pb.valid_mask()
    for name, planes in _test_planes(scene, pb, np.random.default_rng(2)).items():
        gc, gpv, gvm = ctx.eval_cost(torch.tensor(planes, dtype=torch.float32, device="cuda"), per_view=True)
        oc, opv, ovm = oracle.eval_cost(pb, planes)
        frac, bit = compare(f"eval[{name}] sigma_c {sc} sigma_s {ss} eps_v {ev} eps_c {ec} top-{k}", gc.cpu().numpy(),
                            oc, np.ones_like(m))
        assert frac >= FRAC and bit >= FRAC
        assert (gvm.cpu().numpy().astype(bool) == ovm).mean() >= FRAC
    d, nrm, c = ctx.patchmatch(0, list(range(1, n + 1)), cfg["window"], cfg["dilation"], cfg["iters"], p)
    torch.cuda.synchronize()
    od, on, oc = oracle.patchmatch(pb, cfg["iters"])
    frac, bit = compare(f"patchmatch tiny, sigma_c {sc} top-{k}", c.cpu().numpy(), oc, m, d.cpu().numpy(), od)
    assert frac >= FRAC


def test_init_parity_tiny(ctx, tiny):
    scene, cfg = tiny
    pb = _prep(ctx, scene, cfg)
    ctx.init_planes()
    gp, gc = ctx.get_state()
    op, oc = oracle.init(pb)
    m = pb.valid_mask()
    gp = gp.cpu().numpy()
    plane_bit = np.all(gp == op.astype(np.float32), axis=-1)[m].mean()
    say(f"init planes bitwise {plane_bit:.6f}")
    frac, bit = compare("init", gc.cpu().numpy(), oc, m, gp[..., 3], op[..., 3])
    assert plane_bit >= FRAC and frac >= FRAC


@pytest.mark.parametrize("seed", [0x9E3779B97F4A7C15, 0xFFFFFFFF00000001])
def test_init_and_refinement_parity_with_64_bit_seeds(ctx, tiny, seed):
    """Seeds whose high 32 bits are set (the second word of the Philox key): the random
    initial planes bitwise, and one teacher-forced half-sweep (its refinement draws)."""
    scene, cfg = tiny
    pb = _prep(ctx, scene, cfg, seed=seed)
    ctx.init_planes()
    gp, gc = ctx.get_state()
    op, oc = oracle.init(pb)
    m = pb.valid_mask()
    gp = gp.cpu().numpy()
    plane_bit = np.all(gp == op.astype(np.float32), axis=-1)[m].mean()
    say(f"seed {seed:#x}: init planes bitwise {plane_bit:.6f}")
    frac, _ = compare(f"init seed {seed:#x}", gc.cpu().numpy(), oc, m, gp[..., 3], op[..., 3])
    assert plane_bit >= FRAC and frac >= FRAC
    ctx.set_state(torch.tensor(op, dtype=torch.float32, device="cuda"), torch.tensor(oc, dtype=torch.float32, device="cuda"))
    ctx.step(1, 0)
    gp, gc = ctx.get_state()
    P2, C2 = oracle.halfsweep(pb, op, oc, 1, 0)
    gp = gp.cpu().numpy()
    plane_bit = np.all(gp == P2.astype(np.float32), axis=-1)[m].mean()
    say(f"  half-sweep: planes bitwise {plane_bit:.6f}")
    frac, _ = compare(f"half-sweep seed {seed:#x}", gc.cpu().numpy(), C2, m, gp[..., 3], P2[..., 3])
    assert frac >= FRAC and plane_bit >= FRAC
    # the high word matters: the initial planes differ from those of the low word alone
    op_lo, _ = oracle.init(oracle_problem(scene, cfg["window"], cfg["dilation"], cfg["top_k"], seed=seed & 0xFFFFFFFF))
    assert not np.array_equal(op_lo[m], op[m])


def test_halfsweep_parity_tiny(ctx, tiny):
    """Teacher-forced: both sides start each half-sweep from the oracle's state."""
    scene, cfg = tiny
    pb = _prep(ctx, scene, cfg)
    P, Cst = oracle.init(pb)
    m = pb.valid_mask()
    for it, col in [(1, 0), (1, 1), (2, 0), (2, 1)]:
        ctx.set_state(torch.tensor(P, dtype=torch.float32, device="cuda"),
                      torch.tensor(Cst, dtype=torch.float32, device="cuda"))
        ctx.step(it, col)
        gp, gc = ctx.get_state()
        P2, C2 = oracle.halfsweep(pb, P, Cst, it, col)
        gp = gp.cpu().numpy()
        plane_bit = np.all(gp == P2.astype(np.float32), axis=-1)[m].mean()
        say(f"half-sweep it={it} colour={col}: planes bitwise {plane_bit:.6f}")
        frac, bit = compare(f"half-sweep {it}/{col}", gc.cpu().numpy(), C2, m, gp[..., 3], P2[..., 3])
        assert frac >= FRAC and plane_bit >= FRAC
        P, Cst = P2, C2


def test_halfsweep_after_a_state_whose_costs_are_not_its_planes(ctx, tiny):
    """A propagation candidate equal to the pixel's current plane, or to one that the
    previous propagation of its colour offered, is left out only while every stored cost
    is its plane's own cost and no candidate offered earlier can beat it (the library's
    own initialisation and steps).  After set_state with every cost at C_max neither
    holds: such candidates must be scored and taken, as the oracle does.  The library's
    own steps run first, so that both colours have a record of offered candidates that
    set_state has to discard."""
    scene, cfg = tiny
    pb = _prep(ctx, scene, cfg)
    ctx.init_planes()
    ctx.step(1, 0)
    ctx.step(1, 1)
    P, _ = oracle.init(pb)
    P, C = oracle.halfsweep(pb, P, oracle.eval_cost(pb, P)[0], 1, 0)
    P, C = oracle.halfsweep(pb, P, C, 1, 1)
    Cmax = np.full_like(C, 2.0)
    m = pb.valid_mask()
    for it, col in [(2, 0), (2, 1)]:
        ctx.set_state(torch.tensor(P, dtype=torch.float32, device="cuda"),
                      torch.tensor(Cmax, dtype=torch.float32, device="cuda"))
        ctx.step(it, col, refine=False)
        gp, gc = ctx.get_state()
        P2, C2 = oracle.halfsweep(pb, P, Cmax, it, col, refine=False)
        gp = gp.cpu().numpy()
        same = np.all(gp == P2.astype(np.float32), axis=-1)[m]
        say(f"propagation {it}/{col} from costs at C_max: planes bitwise {same.mean():.6f}")
        frac, bit = compare(f"propagation {it}/{col} (costs at C_max)", gc.cpu().numpy(), C2, m, gp[..., 3], P2[..., 3])
        assert same.mean() >= FRAC and bit >= FRAC
        # pixels whose current plane came back as a candidate were updated to its cost
        colour = (np.add.outer(np.arange(pb.H), np.arange(pb.W)) & 1) == col
        assert (C2[m & colour] < 2.0).mean() > 0.99


def test_steps_match_the_whole_run(ctx, tiny):
    """The library's own steps after init_planes, with a set_state of the library's own
    state between two of them, give bitwise the whole run's result (the run issues the
    same launches; set_state only switches off the exact skipping of candidates that
    cannot win, which does not change any result)."""
    scene, cfg = tiny
    iters = 3
    pb = _prep(ctx, scene, cfg)
    d_run, _, c_run = ctx.patchmatch(0, list(range(1, len(scene.images))), cfg["window"], cfg["dilation"],
                                     iters, params_for(cfg["window"], cfg["top_k"]))
    d_run, c_run = d_run.clone(), c_run.clone()
    _prep(ctx, scene, cfg)
    ctx.init_planes()
    for it in range(1, iters + 1):
        for col in (0, 1):
            ctx.step(it, col)
            if (it, col) == (2, 0):
                ctx.set_state(*ctx.get_state())
    gp, gc = ctx.get_state()
    m = torch.from_numpy(pb.valid_mask()).cuda()
    same_d = (gp[..., 3] == d_run)[m].float().mean().item()
    same_c = (gc == c_run)[m].float().mean().item()
    say(f"steps vs whole run ({iters} iterations): depth bitwise {same_d:.6f}, cost bitwise {same_c:.6f}")
    assert same_d == 1.0 and same_c == 1.0


def test_repeated_runs_replay_the_eager_result(ctx, tiny):
    """A single-view run is recorded into a hipGraph on its first call and replayed on
    later ones (the job table, which holds the outputs, is read at run time).  Each replay,
    with other eager work and synchronisations between them and with new output tensors on
    one of them, gives bitwise the result of the eager sequence (diagnostics on: eager)."""
    scene, cfg = tiny
    _prep(ctx, scene, cfg)  # also gives the binding the reference's size for eval_cost
    srcs = list(range(1, len(scene.images)))
    prm = params_for(cfg["window"], cfg["top_k"])
    ctx.diag_enable(pm.DIAG_COUNT)
    ref = [t.clone() for t in ctx.patchmatch(0, srcs, cfg["window"], cfg["dilation"], cfg["iters"], prm)]
    ctx.diag_enable(0)
    out = tuple(torch.full_like(t, -1.0) for t in ref)
    for rep in range(4):
        if rep == 2:
            out = tuple(torch.full_like(t, -1.0) for t in ref)  # outputs move: the table is copied again
        got = ctx.patchmatch(0, srcs, cfg["window"], cfg["dilation"], cfg["iters"], prm, out=out)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(got, ref))
        say(f"run {rep + 1} after the eager one: bitwise {same}")
        assert same
        # eager work of the program's own between the replays
        ctx.eval_cost(torch.zeros((scene.images[0].shape[0], scene.images[0].shape[1], 4), device="cuda"))
        for t in out:
            t.fill_(-1.0)
        torch.cuda.synchronize()
    # the state a replay leaves behind serves the next steps as the eager run's does
    _prep(ctx, scene, cfg)
    ctx.patchmatch(0, srcs, cfg["window"], cfg["dilation"], cfg["iters"], prm, out=out)
    ctx.step(cfg["iters"] + 1, 0)
    gp, gc = ctx.get_state()
    ctx.diag_enable(pm.DIAG_COUNT)
    ctx.patchmatch(0, srcs, cfg["window"], cfg["dilation"], cfg["iters"], prm, out=out)
    ctx.diag_enable(0)
    ctx.step(cfg["iters"] + 1, 0)
    ep, ec = ctx.get_state()
    assert torch.equal(gp, ep) and torch.equal(gc, ec)


def test_host_outputs_equal_device_outputs(ctx, tiny):
    """phimvs_patchmatch with host output arrays (staged through the library's device
    buffers, the sequence replayed from its graph on the second call) gives bitwise the
    device-output result."""
    import ctypes
    scene, cfg = tiny
    ctx.set_scene(scene)
    srcs = list(range(1, len(scene.images)))
    prm = params_for(cfg["window"], cfg["top_k"])
    d, n, c = (t.cpu().numpy() for t in ctx.patchmatch(0, srcs, cfg["window"], cfg["dilation"], cfg["iters"], prm))
    H, W = d.shape
    L = pm.lib()
    sa = (ctypes.c_int * len(srcs))(*srcs)
    p = prm._c()
    for call in range(2):
        hd = np.full((H, W), -1.0, np.float32)
        hn = np.full((H, W, 3), -1.0, np.float32)
        hc = np.full((H, W), -1.0, np.float32)
        rc = L.phimvs_patchmatch(ctx.h, 0, sa, len(srcs), cfg["window"], cfg["dilation"], cfg["iters"],
                                 ctypes.byref(p), hd.ctypes.data, hn.ctypes.data, hc.ctypes.data, 0)
        assert rc == 0, L.phimvs_last_error(ctx.h)
        same = np.array_equal(hd, d) and np.array_equal(hn, n) and np.array_equal(hc, c)
        say(f"host outputs, call {call + 1}: bitwise {same}")
        assert same


def test_patchmatch_parity_tiny(ctx, tiny):
    scene, cfg = tiny
    pb = _prep(ctx, scene, cfg)
    n = len(scene.images) - 1
    d, nrm, c = ctx.patchmatch(0, list(range(1, n + 1)), cfg["window"], cfg["dilation"], cfg["iters"],
                               params_for(cfg["window"], cfg["top_k"]))
    torch.cuda.synchronize()
    od, on, oc = oracle.patchmatch(pb, cfg["iters"])
    m = pb.valid_mask()
    frac, bit = compare("patchmatch tiny", c.cpu().numpy(), oc, m, d.cpu().numpy(), od)
    assert frac >= FRAC
    od64, _, oc64 = oracle.patchmatch(pb, cfg["iters"], fp64=True)
    gd = d.cpu().numpy()
    planes = np.concatenate([nrm.cpu().numpy(), gd[..., None]], -1).astype(np.float64)
    tf64, _, _ = oracle.eval_cost(pb, planes, fp64=True)
    fp64_report("  tiny: teacher-forced cost of the output planes", c.cpu().numpy(), tf64, m)
    fp64_report("  tiny: free-running depth", gpu_depth=gd, fp64_depth=od64, mask=m)
    # invalid pixels: depth 0, normal 0, cost C_max
    assert np.all(gd[~m] == 0) and np.all(c.cpu().numpy()[~m] == 2.0) and np.all(nrm.cpu().numpy()[~m] == 0)


@pytest.mark.parametrize("kind", ["skew", "general"])
def test_patchmatch_parity_tiny_with_other_intrinsics(ctx, tiny, kind):
    """The whole tiny run (initialisation, propagation with its ray-plane re-expression,
    refinement) under skewed or general invertible intrinsics: within the tolerances, as
    for the rendered cameras."""
    scene, cfg = tiny
    sc = _with_intrinsics(scene, kind)
    pb = _prep(ctx, sc, cfg)
    n = len(sc.images) - 1
    d, nrm, c = ctx.patchmatch(0, list(range(1, n + 1)), cfg["window"], cfg["dilation"], cfg["iters"],
                               params_for(cfg["window"], cfg["top_k"]))
    torch.cuda.synchronize()
    od, on, oc = oracle.patchmatch(pb, cfg["iters"])
    m = pb.valid_mask()
    frac, bit = compare(f"patchmatch tiny, {kind} intrinsics", c.cpu().numpy(), oc, m, d.cpu().numpy(), od)
    assert frac >= FRAC


def test_patchmatch_parity_tiny_depth_ordered(ctx, tiny):
    """The whole tiny run with its work items handed out in order of
    the candidates' inverse depth, against the oracle to the same bar as in pixel order."""
    scene, cfg = tiny
    pb = _prep(ctx, scene, cfg)
    n = len(scene.images) - 1
    prev = ctx.get_tuning()
    ctx.set_tuning(pm.Tuning(prev.tile_rows, prev.persistent, prev.wgs_per_cu, order_by_depth=True))
    try:
        d, nrm, c = ctx.patchmatch(0, list(range(1, n + 1)), cfg["window"], cfg["dilation"], cfg["iters"],
                                   params_for(cfg["window"], cfg["top_k"]))
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning(prev)
    od, on, oc = oracle.patchmatch(pb, cfg["iters"])
    m = pb.valid_mask()
    frac, bit = compare("patchmatch tiny, depth-ordered work", c.cpu().numpy(), oc, m, d.cpu().numpy(), od)
    assert frac >= FRAC


# ----------------------------------------------------------------------------- edge cases
@pytest.mark.parametrize("W,H,n_src,window,dilation,top_k,bilateral", [
    (133, 67, 2, 7, 1, 0, True),     # ragged width/height (not multiples of 128 / 4)
    (130, 61, 3, 9, 2, 1, True),     # dilation 2, best-1
    (97, 50, 1, 7, 3, 0, False),     # one source, dilation 3, plain Eq. 4 weights
    (200, 9, 2, 7, 1, 2, True),      # 1 valid row band
    (64, 40, 6, 5, 1, 3, True),      # six sources
    (100, 72, 2, 61, 2, 0, True),    # the largest window: 31 taps per side over a 30-pixel radius
    (96, 64, 12, 7, 1, 5, True),     # the most sources (12)
])
def test_edge_case_parity(ctx, W, H, n_src, window, dilation, top_k, bilateral):
    scene = sg.make_scene(100 + W + H, sg.tiny_config(W, H, n_src=n_src, n_planes=3, n_textureless=1), device="cuda")
    ctx.set_scene(scene)
    srcs = list(range(1, n_src + 1))
    p = params_for(window, top_k, bilateral)
    d, nrm, c = ctx.patchmatch(0, srcs, window, dilation, 2, p)
    torch.cuda.synchronize()
    pb = oracle_problem(scene, window, dilation, top_k, bilateral)
    od, on, oc = oracle.patchmatch(pb, 2)
    m = pb.valid_mask()
    frac, _ = compare(f"edge {W}x{H} n={n_src} win={window} s={dilation} K={top_k} bil={bilateral}",
                      c.cpu().numpy(), oc, m, d.cpu().numpy(), od)
    assert frac >= FRAC
    assert np.all(d.cpu().numpy()[~m] == 0) and np.all(c.cpu().numpy()[~m] == 2.0)


def test_no_valid_pixel(ctx):
    """A reference smaller than the window: every pixel is invalid."""
    scene = sg.make_scene(7, sg.tiny_config(12, 10, n_src=2, n_planes=1), device="cuda")
    ctx.set_scene(scene)
    d, nrm, c = ctx.patchmatch(0, [1, 2], 11, 1, 1, params_for(11, 0))
    torch.cuda.synchronize()
    assert torch.all(d == 0) and torch.all(c == 2.0) and torch.all(nrm == 0)


def test_argument_errors(ctx, tiny):
    scene, cfg = tiny
    ctx.set_scene(scene)
    bad = [
        dict(ref=0, srcs=[0, 1], window=11, dilation=1),      # ref among sources
        dict(ref=0, srcs=[1, 1], window=11, dilation=1),      # duplicate source
        dict(ref=0, srcs=[1], window=10, dilation=1),         # even window
        dict(ref=0, srcs=[1], window=11, dilation=3),         # (window-1) % (2 s) != 0
        dict(ref=9, srcs=[1], window=11, dilation=1),         # ref out of range
        dict(ref=0, srcs=[], window=11, dilation=1),          # no source
    ]
    for b in bad:
        with pytest.raises(pm.PhimvsError) as e:
            ctx.patchmatch(b["ref"], b["srcs"], b["window"], b["dilation"], 1)
        assert e.value.code == -1
    with pytest.raises(pm.PhimvsError):
        ctx.patchmatch(0, [1, 2], 11, 1, 1, pm.Params(top_k=3))  # top_k > n_srcs
    with pytest.raises(pm.PhimvsError):
        ctx.prepare(0, [1], 11, 1, pm.Params(sigma_color=-1.0))


def test_size_limits(ctx, tiny):
    """Requests beyond the documented limits fail with PHIMVS_E_UNSUPPORTED (-5)."""
    scene, cfg = tiny
    ctx.set_scene(scene)
    for window, dilation in [(63, 1), (67, 3)]:  # 32 taps per side; a 33-pixel radius
        with pytest.raises(pm.PhimvsError) as e:
            ctx.patchmatch(0, [1], window, dilation, 1)
        assert e.value.code == -5
    many = sg.make_scene(11, sg.tiny_config(40, 30, n_src=13, n_planes=1), device="cuda")
    ctx.set_scene(many)
    with pytest.raises(pm.PhimvsError) as e:  # 13 sources
        ctx.patchmatch(0, list(range(1, 14)), 5, 1, 1)
    assert e.value.code == -5
    K = np.array([[100.0, 0.0, 8.0], [0.0, 100.0, 8.0], [0.0, 0.0, 1.0]])
    big = np.zeros((1 << 14, 1 << 14), np.uint8)  # 2^28 pixels
    with pytest.raises(pm.PhimvsError) as e:
        ctx.set_views([big, np.zeros((16, 16), np.uint8)], np.stack([K, K]), np.stack([np.eye(3)] * 2),
                      np.zeros((2, 3)), np.tile([1.0, 10.0], (2, 1)))
    assert e.value.code == -5
    ctx.set_scene(scene)


# ----------------------------------------------------------------------------- high-resolution workload
@pytest.fixture(scope="module")
def highres():
    say("rendering the 3200x2130 scene (10 sources, 25 planes)")
    return sg.workload_scene("highres", device="cuda")


def test_highres_crop_parity(ctx, highres):
    """The 320x213 centre crop of the reference (sources whole) as its own problem, end to
    end at the workload's 8 iterations, against the FP32 oracle (the bar) and the FP64 one
    (stated): free-running depth, and the cost of the GPU's output planes re-evaluated."""
    cfg = sg.SOLVER["highres"]
    scene = sg.crop_reference(highres, 320, 213)
    iters = cfg["iters"]
    ctx.set_scene(scene)
    n = len(scene.images) - 1
    d, nrm, c = ctx.patchmatch(0, list(range(1, n + 1)), cfg["window"], cfg["dilation"], iters,
                               params_for(cfg["window"], cfg["top_k"]))
    torch.cuda.synchronize()
    pb = oracle_problem(scene, cfg["window"], cfg["dilation"], cfg["top_k"])
    say(f"highres crop: oracle, {iters} iterations on {THREADS} threads")
    od, on, oc = oracle.patchmatch(pb, iters, threads=THREADS)
    m = pb.valid_mask()
    gd, gc = d.cpu().numpy(), c.cpu().numpy()
    frac, _ = compare(f"highres crop ({iters} iterations)", gc, oc, m, gd, od)
    assert frac >= FRAC
    od64, _, _ = oracle.patchmatch(pb, iters, fp64=True, threads=THREADS)
    planes = np.concatenate([nrm.cpu().numpy(), gd[..., None]], -1).astype(np.float64)
    tf64, _, _ = oracle.eval_cost(pb, planes, fp64=True, threads=THREADS)
    fp64_report("highres crop: teacher-forced cost of the output planes", gc, tf64, m)
    fp64_report("highres crop: free-running depth", gpu_depth=gd, fp64_depth=od64, mask=m)


def test_highres_full_frame_sampled(ctx, highres):
    """Full 3200x2130, 10 sources, 31x31 at dilation 3, top-5, 8 iterations (the benchmark's
    launch configuration): final costs re-evaluated by the oracle at sampled pixels, and one
    further half-sweep checked pixel by pixel on a sample."""
    cfg = sg.SOLVER["highres"]
    scene = highres
    ctx.set_scene(scene)
    n = len(scene.images) - 1
    srcs = list(range(1, n + 1))
    p = params_for(cfg["window"], cfg["top_k"])
    ctx.prepare(0, srcs, cfg["window"], cfg["dilation"], p)
    ctx.init_planes()
    for it in range(1, cfg["iters"] + 1):
        for col in (0, 1):
            ctx.step(it, col)
    planes, cost = ctx.get_state()
    torch.cuda.synchronize()
    pb = oracle_problem(scene, cfg["window"], cfg["dilation"], cfg["top_k"])
    m = pb.valid_mask()
    rng = np.random.default_rng(1)
    idx = np.flatnonzero(m.ravel())
    sub = rng.choice(idx, size=5000, replace=False).astype(np.int32)
    P = planes.cpu().numpy().astype(np.float64)
    oc, _, _ = oracle.eval_cost(pb, P, subset=sub, threads=THREADS)
    g = cost.cpu().numpy().ravel()[sub]
    o = oc.ravel()[sub]
    ok = np.abs(g - o) <= COST_TOL
    say(f"full frame: final cost re-evaluated at {len(sub)} pixels: within tol {ok.mean():.5f}, "
        f"bitwise {(g == o.astype(np.float32)).mean():.5f}")
    assert ok.mean() >= FRAC
    o64, _, _ = oracle.eval_cost(pb, P, fp64=True, subset=sub, threads=THREADS)
    fp64_report("full frame: teacher-forced cost at the sampled pixels", g, o64.ravel()[sub])
    # one more half-sweep, GPU vs oracle on a sample of red pixels
    Cst = cost.cpu().numpy().astype(np.float64)
    ctx.step(cfg["iters"] + 1, 0)
    gp2, gc2 = ctx.get_state()
    torch.cuda.synchronize()
    ys, xs = np.divmod(idx, pb.W)
    red = idx[((xs + ys) & 1) == 0]
    sub2 = rng.choice(red, size=3000, replace=False).astype(np.int32)
    P2, C2 = oracle.halfsweep(pb, P, Cst, cfg["iters"] + 1, 0, subset=sub2, threads=THREADS)
    g2 = gc2.cpu().numpy().ravel()[sub2]
    o2 = C2.ravel()[sub2]
    gd2 = gp2.cpu().numpy()[..., 3].ravel()[sub2]
    od2 = P2[..., 3].ravel()[sub2]
    ok2 = (np.abs(g2 - o2) <= COST_TOL) & (np.abs(gd2 - od2) <= DEPTH_TOL * np.abs(od2))
    say(f"full frame: half-sweep at {len(sub2)} pixels: within tol {ok2.mean():.5f}")
    assert ok2.mean() >= FRAC
    P64, _ = oracle.halfsweep(pb, P, Cst, cfg["iters"] + 1, 0, fp64=True, subset=sub2, threads=THREADS)
    fp64_report("full frame: depth after the half-sweep at the sampled pixels", gpu_depth=gd2,
                fp64_depth=P64[..., 3].ravel()[sub2])
