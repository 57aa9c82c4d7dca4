"""GPU parity of the cross-bilateral denoiser (Sec. 3.4.2, "Denoising")
against the oracle's written-out definition: within 1e-4 relative / 1e-5
absolute, over radii, bandwidths, ragged image sizes (partial tiles), invalid
pixels and a real low-sample render."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grt_ctx():
    from paper_2607_22780_amd import grt
    return grt, grt.Context(0)


def run(grt, ctx, rgb, gb, **kw):
    from gpu_util import t
    out = grt.denoise(ctx, t(rgb.astype(np.float32)), t(gb.depth), t(gb.n), t(gb.valid), gb.H, gb.W, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("H,Wd", [(64, 61), (1, 1), (17, 33), (5, 300)])
@pytest.mark.parametrize("kw", [dict(), dict(radius=1, sigma_s=0.8), dict(radius=8, sigma_s=4.0, sigma_n=16.0),
                                dict(radius=2, sigma_d=0.0, eps_d=0.5)])
def test_denoise_parity(grt_ctx, H, Wd, kw):
    grt, ctx = grt_ctx
    gb = W.gbuffer1(H, Wd, seed=1)
    g = np.random.default_rng(H * 1000 + Wd)
    rgb = g.uniform(0, 2, (gb.npix, 3)).astype(np.float32)
    got = run(grt, ctx, rgb, gb, **kw)
    ref = O.denoise(rgb, gb.depth, gb.n, gb.valid, gb.H, gb.W, **kw)
    np.testing.assert_allclose(got, ref, rtol=1e-4, atol=1e-5)
    inv = gb.valid == 0
    np.testing.assert_array_equal(got[inv], rgb[inv])


def test_denoise_low_sample_render(grt_ctx):
    """A 4-spp MIS render of the sphere/torus scene, denoised on the GPU and
    by the oracle from the same noisy image.  With uniform materials (the
    workload draws them per pixel, which the filter, averaging colour, would
    blur as if it were noise) the filter lowers the error against a 64-spp
    render."""
    import dataclasses
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene1(n=20000, seed=0, s_lo=0.01, s_hi=0.06)
    gb = W.gbuffer1(96, 96, seed=0)
    v8 = gb.valid.astype(np.float32)
    gb = dataclasses.replace(gb, albedo=np.ascontiguousarray(np.outer(v8, [0.6, 0.5, 0.4]).astype(np.float32)),
                             rough=np.ascontiguousarray(0.5 * v8), metal=np.zeros_like(v8))
    env = W.envmap(64, 128, seed=0)
    scene = grt.Scene(ctx, *scene_tensors(s))
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, torch.device("cuda", 0))
    noisy = grt.render_mis(scene, E, G, split=(2, 1, 1), seed=5)["rgb"].cpu().numpy()
    ref_img = grt.render_mis(scene, E, G, split=(32, 16, 16), seed=6)["rgb"].cpu().numpy()
    got = run(grt, ctx, noisy, gb)
    want = O.denoise(noisy, gb.depth, gb.n, gb.valid, gb.H, gb.W)
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-5)
    v = gb.valid.astype(bool)
    assert np.mean((got[v] - ref_img[v]) ** 2) < np.mean((noisy[v] - ref_img[v]) ** 2)


def test_denoise_rejects_bad_arguments(grt_ctx):
    grt, ctx = grt_ctx
    from gpu_util import t
    gb = W.gbuffer1(8, 8, seed=1)
    rgb = t(np.ones((gb.npix, 3), np.float32))
    for kw in (dict(radius=0), dict(radius=9), dict(sigma_s=0.0), dict(eps_d=0.0)):
        with pytest.raises(grt.GrtError) as e:
            grt.denoise(ctx, rgb, t(gb.depth), t(gb.n), t(gb.valid), gb.H, gb.W, **kw)
        assert e.value.code == grt.ERR_INVALID
