"""The allocation-free hypothesis entry point (phimvs_phi_hypotheses_noalloc) through the
C ABI against phimvs_phi_hypotheses: bitwise equal outputs on two calls in a row (the
second on a smaller map, so the shared scratch still holds the first call's larger
bitmaps), free device memory unchanged by a call, and a map beyond its scratch refused."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_06165_amd as pm  # noqa: E402


def depth_map(H, W, seed):
    """Planar depth with holes: scattered pixels, a wide band and a block, plus negative and
    NaN depths (no depth too)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    ys = torch.arange(H, device="cuda", dtype=torch.float32)[:, None]
    xs = torch.arange(W, device="cuda", dtype=torch.float32)[None, :]
    d = 4.0 + 0.001 * xs - 0.0007 * ys
    keep = torch.rand((H, W), generator=g, device="cuda") < 0.6
    d = torch.where(keep, d, torch.zeros_like(d))
    d[H // 3:H // 3 + max(1, H // 10), :] = 0.0
    d[:, W // 2:W // 2 + max(1, W // 7)] = 0.0
    d[5 % H, 7 % W] = -1.0
    d[(H // 2) % H, (W // 3) % W] = float("nan")
    return d.contiguous()


def test_noalloc_hypotheses_equal_the_allocating_entry_point():
    ctx = pm.Context(0)
    try:
        for i, (H, W) in enumerate([(2130, 3200), (301, 517)]):
            d = depth_map(H, W, 100 + i)
            out = torch.full((4, H, W), -7.0, device="cuda")
            torch.cuda.synchronize()
            ctx.phi_hypotheses_noalloc(d, out)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            ctx.phi_hypotheses_noalloc(d, out)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            ref = ctx.phi_hypotheses(d)
            torch.cuda.synchronize()
            print(f"{W}x{H}: hypotheses {(ref > 0).sum().item()}, free memory change {free0 - free1} B", flush=True)
            assert free1 == free0
            assert torch.equal(out, ref)
            assert (ref > 0).sum().item() > 0.2 * H * W
    finally:
        ctx.close()


def test_noalloc_refuses_a_map_beyond_its_scratch():
    ctx = pm.Context(0)
    try:
        d = torch.ones((4000, 6000), device="cuda")  # (4 W + 2 H) H / 8 = 16 MB of bitmaps
        out = torch.empty((4, 4000, 6000), device="cuda")
        with pytest.raises(pm.PhimvsError) as e:
            ctx.phi_hypotheses_noalloc(d, out)
        assert e.value.code == -5
    finally:
        ctx.close()
