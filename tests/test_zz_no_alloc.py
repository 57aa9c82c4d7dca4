"""grt_render_mis_noalloc: the MIS render with its scratch in the library's
fixed per-device array instead of a workspace argument.  Two calls in a row
(the second smaller, over what the first left in the array) against
grt_render_mis with a workspace, bit for bit, and a size past the array's
limit refused with a clear error."""
import numpy as np
import pytest
import torch

from paper_2607_22780_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(grt, ctx, H, Wd, split, seed):
    from gpu_util import t, scene_tensors
    s = W.scene1(n=20000, seed=seed, s_lo=0.01, s_hi=0.06)
    gb = W.gbuffer1(H, Wd, seed=seed)
    env = W.envmap(64, 128, seed=seed)
    scene = grt.Scene(ctx, *scene_tensors(s))
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, torch.device("cuda", 0))
    return scene, E, G


def _noalloc(grt, scene, E, G, split, seed, k):
    dev = G.x.device
    spp = sum(split)
    out = torch.full((G.npix, 3), float("nan"), device=dev)
    saved = torch.full((grt.grt_render_saved_bytes(G.npix, spp) // 4,), float("nan"), device=dev)
    opts = grt.make_mis_opts(split, seed, 0, 1e-3, 1e-3, k)
    grt.grt_render_mis_noalloc(scene.handle, E.handle, G.struct(), opts, out, saved)
    return out, saved


def test_noalloc_matches_workspace_render_twice():
    from paper_2607_22780_amd import grt
    ctx = grt.Context(0)
    for H, Wd, split, seed, k in [(48, 40, (16, 8, 8), 3, 12), (20, 17, (4, 2, 2), 4, 8)]:
        scene, E, G = _case(grt, ctx, H, Wd, split, seed)
        spp = sum(split)
        want = grt.render_mis(scene, E, G, split=split, seed=seed, k=k, save=True, dump=True)
        got, saved = _noalloc(grt, scene, E, G, split, seed, k)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), want["rgb"].cpu().numpy())
        traced = want["dump"][..., 3].reshape(-1).cpu().numpy() > 0
        nray = G.npix * spp
        s_ct = saved[: 4 * nray].view(nray, 4).cpu().numpy()[traced]
        s_st = saved[4 * nray: 5 * nray].cpu().numpy()[traced]
        np.testing.assert_array_equal(s_ct, want["saved_ct"].cpu().numpy()[traced])
        np.testing.assert_array_equal(s_st, want["saved_stop"].cpu().numpy()[traced])
        assert traced.sum() > 0.2 * nray


def test_noalloc_refuses_more_than_its_scratch():
    from paper_2607_22780_amd import grt
    ctx = grt.Context(0)
    scene, E, G = _case(grt, ctx, 8, 8, (1, 1, 1), 5)
    big = grt.GBuffer(512, 512, G.x, G.n, G.wo, G.albedo, G.rough, G.metal, G.valid)  # never launched
    opts = grt.make_mis_opts((16, 8, 8), 1, 0, 1e-3, 1e-3, 8)
    with pytest.raises(grt.GrtError) as ei:
        grt.grt_render_mis_noalloc(scene.handle, E.handle, big.struct(), opts, G.x, None)
    assert ei.value.code == grt.ERR_INVALID and "scratch" in str(ei.value)
