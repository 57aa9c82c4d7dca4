"""GPU parity of the backward passes (Sec. 3.2: gradients backpropagate
through the secondary-ray queries) against the oracle's gradients, which are
themselves pinned by autograd and finite differences.

Tolerance per parameter block: |g - g_ref| <= 1e-3 max(|g_ref|, 1e-2
max|g_ref|_block) element-wise (the floor absorbs single-precision sums of
many signed terms) and relative L2 error <= 1e-3."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W

pytestmark = pytest.mark.gpu

BLOCKS = dict(means=(0, 3), scales=(3, 5), quats=(5, 9), opacity=(9, 10), rgb=(10, 13))


@pytest.fixture(scope="module")
def grt_ctx():
    from paper_2607_22780_amd import grt
    return grt, grt.Context(0)


def check_grads(g, ref13, ref13_abs=None, rel=1e-3, floor=1e-2):
    """Every block of the 13 gradient columns to the bar of grad_close."""
    from gpu_util import grad_close
    if isinstance(ref13, tuple):
        ref13, ref13_abs = ref13
    for name, (a, b) in BLOCKS.items():
        grad_close(g[name].reshape(len(ref13), -1), ref13[:, a:b], name,
                   None if ref13_abs is None else ref13_abs[:, a:b], rel=rel, floor=floor)


@pytest.mark.parametrize("bounded", [False, True])
def test_trace_backward_config0(grt_ctx, bounded):
    """Re-traversal over the whole ray range, or bounded by the forward's
    saved stop depth: the same gradients."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene0(); r = W.rays0()
    g = np.random.default_rng(0)
    ref_f = O.trace(s, r.origins, r.dirs, cap=64)
    keep = ref_f["margins"][:, 3] >= 1e-5  # cutoff knife edges carry no gradient in either side
    gC = (g.normal(0, 1, (r.n, 3)) * keep[:, None]).astype(np.float32)
    gT = (g.normal(0, 1, r.n) * keep).astype(np.float32)
    ref = O.trace_backward(s, r.origins, r.dirs, gC, gT, with_abs=True)
    scene = grt.Scene(ctx, *scene_tensors(s))
    o, d = t(r.origins), t(r.dirs)
    fwd = grt.trace(scene, o, d, save_stop=bounded)
    gg = grt.trace_backward(scene, o, d, fwd["rgb"], fwd["T"], t(gC), t(gT), stop=fwd.get("stop"))
    torch.cuda.synchronize()
    check_grads({k: v.cpu().numpy() for k, v in gg.items()}, ref)
    if bounded:  # the stop depth is the depth of the last composited hit
        nh = ref_f["nhit"]
        last = np.where(nh > 0, ref_f["tau"][np.arange(r.n), np.maximum(nh - 1, 0)], 0.0)
        stop = fwd["stop"].cpu().numpy()
        ok = keep & (nh <= 64)
        np.testing.assert_allclose(stop[ok], last[ok], rtol=1e-5, atol=1e-6)


def test_trace_autograd_function(grt_ctx):
    """TraceFn: torch.autograd drives the same kernels."""
    grt, ctx = grt_ctx
    from gpu_util import t
    s = W.scene0(n=1500, seed=3); r = W.rays0(res=20, per=4, seed=3)
    params = [t(a).requires_grad_(True) for a in s.arrays()]
    rgb, T = grt.TraceFn.apply(*params, t(r.origins), t(r.dirs), ctx, 0.0, 16, 1e-3, 1.0 / 255.0)
    g = np.random.default_rng(1)
    gC = g.normal(0, 1, (r.n, 3)).astype(np.float32); gT = g.normal(0, 1, r.n).astype(np.float32)
    ref_f = O.trace(s, r.origins, r.dirs)
    keep = ref_f["margins"][:, 3] >= 1e-5
    gC *= keep[:, None]; gT *= keep
    ((rgb * t(gC)).sum() + (T * t(gT)).sum()).backward()
    ref = O.trace_backward(s, r.origins, r.dirs, gC, gT, with_abs=True)
    got = dict(zip(("means", "scales", "quats", "opacity", "rgb"), (p.grad.cpu().numpy() for p in params)))
    check_grads(got, ref)


@pytest.mark.parametrize("k_bwd", [16, 13])
def test_render_backward_small_scene(grt_ctx, k_bwd):
    """Retrace backward of the MIS render on pixels whose every sample is
    clear of knife edges (the rest get zero upstream gradient); 13 is the
    benchmarked backward's hit-buffer size (its own kernel)."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene1(n=20000, seed=0, s_lo=0.01, s_hi=0.06)
    gb = W.gbuffer1(40, 37, seed=0)
    env = W.envmap(64, 128, seed=0)
    split = (16, 8, 8)
    ref_f = O.render_mis(s, gb, env, split, 3, dump=True)
    m = ref_f["margins"]
    edge = ((m[..., 3] < 1e-5) | (m[..., 4] < 1e-9)).any(axis=1)
    g = np.random.default_rng(4)
    grad = (g.normal(0, 1, (gb.npix, 3)) * (~edge)[:, None]).astype(np.float32)
    ref = O.render_mis_backward(s, gb, env, split, 3, grad, with_abs=True)
    scene = grt.Scene(ctx, *scene_tensors(s))
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, torch.device("cuda", 0))
    fwd = grt.render_mis(scene, E, G, split=split, seed=3, save=True)
    gg = grt.render_mis_backward(scene, E, G, t(grad), fwd["saved"], split=split, seed=3, k=k_bwd)
    torch.cuda.synchronize()
    check_grads({k: v.cpu().numpy() for k, v in gg.items()}, ref)


def test_render_autograd_matches_direct(grt_ctx):
    """RenderMISFn.backward == grt_render_mis_backward on the same inputs."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene1(n=8000, seed=5, s_lo=0.01, s_hi=0.05)
    gb = W.gbuffer1(16, 16, seed=5)
    env = W.envmap(32, 64, seed=5)
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, torch.device("cuda", 0))
    params = [t(a).requires_grad_(True) for a in s.arrays()]
    img = grt.RenderMISFn.apply(*params, ctx, E, G, (4, 2, 2), 11, 16, 1.0 / 255.0)
    w = torch.randn_like(img)
    (img * w).sum().backward()
    scene = grt.Scene(ctx, *scene_tensors(s))
    fwd = grt.render_mis(scene, E, G, split=(4, 2, 2), seed=11, save=True)
    np.testing.assert_array_equal(fwd["rgb"].cpu().numpy(), img.detach().cpu().numpy())
    gg = grt.render_mis_backward(scene, E, G, w, fwd["saved"], split=(4, 2, 2), seed=11)
    for p, name in zip(params, ("means", "scales", "quats", "opacity", "rgb")):
        np.testing.assert_allclose(p.grad.cpu().numpy(), gg[name].cpu().numpy(), rtol=1e-4, atol=1e-6)


def _small_render_case(grt, ctx):
    from gpu_util import t, scene_tensors
    s = W.scene1(n=20000, seed=0, s_lo=0.01, s_hi=0.06)
    gb = W.gbuffer1(40, 37, seed=0)
    env = W.envmap(64, 128, seed=0)
    split = (16, 8, 8)
    ref_f = O.render_mis(s, gb, env, split, 3, dump=True)
    m = ref_f["margins"]
    edge = ((m[..., 3] < 1e-5) | (m[..., 4] < 1e-9)).any(axis=1)
    g = np.random.default_rng(4)
    grad = (g.normal(0, 1, (gb.npix, 3)) * (~edge)[:, None]).astype(np.float32)
    scene = grt.Scene(ctx, *scene_tensors(s))
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, torch.device("cuda", 0))
    return s, gb, env, split, grad, scene, E, G


@pytest.mark.parametrize("cap", [2, 256])
def test_render_backward_stored_lists(grt_ctx, cap):
    """Stored-hit-list backward (the forward records each sample's hits):
    equal to the oracle's gradient as the re-traversal backward is.  With a
    capacity of 2 most samples overflow and are re-traversed; with 256 none
    do.  The stored counts are the number of hits each sample composited."""
    grt, ctx = grt_ctx
    from gpu_util import t
    s, gb, env, split, grad, scene, E, G = _small_render_case(grt, ctx)
    ref = O.render_mis_backward(s, gb, env, split, 3, grad, with_abs=True)
    spp = sum(split)
    hits = grt.make_hit_list(gb.npix, spp, cap, torch.device("cuda", 0))
    fwd = grt.render_mis(scene, E, G, split=split, seed=3, save=True, dump=True, hits=hits, hit_cap=cap)
    plain = grt.render_mis(scene, E, G, split=split, seed=3)
    np.testing.assert_array_equal(fwd["rgb"].cpu().numpy(), plain["rgb"].cpu().numpy())
    gg = grt.render_mis_backward(scene, E, G, t(grad), fwd["saved"], split=split, seed=3, hits=hits, hit_cap=cap)
    torch.cuda.synchronize()
    check_grads({k: v.cpu().numpy() for k, v in gg.items()}, ref)
    counts = hits[: gb.npix * spp].cpu().numpy().astype(np.int64)
    traced = fwd["dump"].reshape(-1, 10)[:, 3].cpu().numpy() > 0  # q > 0: the sample was traced
    T = fwd["saved_ct"][:, 3].cpu().numpy()
    stop = fwd["saved_stop"].cpu().numpy()
    assert np.all(counts[~traced] == 0)
    assert np.all((counts[traced] > 0) == (T[traced] < 1.0))  # a hit iff transmittance dropped
    # the saved stop depth of a traced sample: 0 without a composited hit,
    # past t_min with one (untraced samples save nothing)
    assert np.all((stop[traced] > 1e-3) == (counts[traced] > 0))
    assert np.all(stop[traced & (counts == 0)] == 0)
    if cap == 2:
        assert np.mean(counts > cap) > 0.2  # the overflow path is exercised
    else:
        assert counts.max() <= cap


def test_stored_lists_hold_the_composited_hits(grt_ctx):
    """The stored list of a sample names the surfels the plain trace
    composites along the same ray, in the same order."""
    grt, ctx = grt_ctx
    from gpu_util import t
    s, gb, env, split, grad, scene, E, G = _small_render_case(grt, ctx)
    spp = sum(split)
    cap = 128
    hits = grt.make_hit_list(gb.npix, spp, cap, torch.device("cuda", 0))
    res = grt.render_mis(scene, E, G, split=split, seed=3, save=True, dump=True, hits=hits, hit_cap=cap)
    dump = res["dump"].reshape(-1, 10).cpu().numpy()
    counts = hits[: gb.npix * spp].cpu().numpy()
    lists = hits[gb.npix * spp:].reshape(-1, cap).cpu().numpy()
    rec_ids = scene.arrays()["records"][:, 11].contiguous().view(torch.int32).cpu().numpy()
    g = np.random.default_rng(9)
    traced = np.nonzero(dump[:, 3] > 0)[0]
    pick = np.sort(g.choice(traced, 256, replace=False))
    pix = pick // spp
    o = t(np.ascontiguousarray(gb.x[pix])); d = t(np.ascontiguousarray(dump[pick, 0:3]))
    tr = grt.trace(scene, o, d, t_min=1e-3, dump_cap=cap)
    ids = tr["ids"].cpu().numpy(); nh = tr["nhit"].cpu().numpy()
    for k, r in enumerate(pick):
        assert counts[r] == nh[k]
        n = min(int(nh[k]), cap)
        np.testing.assert_array_equal(rec_ids[lists[r, :n]], ids[k, :n])


def test_render_autograd_stored_matches_retrace(grt_ctx):
    """RenderMISFn with stored hit lists gives the re-traversal gradients."""
    grt, ctx = grt_ctx
    from gpu_util import t
    s = W.scene1(n=8000, seed=5, s_lo=0.01, s_hi=0.05)
    gb = W.gbuffer1(16, 16, seed=5)
    env = W.envmap(32, 64, seed=5)
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, torch.device("cuda", 0))
    grads = []
    for cap in (0, 64):
        params = [t(a).requires_grad_(True) for a in s.arrays()]
        img = grt.RenderMISFn.apply(*params, ctx, E, G, (4, 2, 2), 11, 16, 1.0 / 255.0, cap)
        w = torch.from_numpy(np.random.default_rng(2).normal(0, 1, tuple(img.shape)).astype(np.float32)).cuda()
        (img * w).sum().backward()
        grads.append([p.grad.cpu().numpy() for p in params])
    for a, b in zip(*grads):
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("cap", [0, 64])
def test_differentiable_step_full_scene_sampled(grt_ctx, cap):
    """The differentiable step at full size: 300k surfels, 800x800, 16/8/8,
    L2 loss against a target rendered from perturbed radiance and opacity.
    The upstream gradient 2 (c - target) is kept on 48 seeded valid pixels
    (clear of knife edges) and the whole backward runs on the GPU, by
    re-traversal (cap 0) and from stored hit lists (cap 64); the oracle
    differentiates the same 48 pixels."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene1()
    tgt = W.perturbed(s)
    gb = W.gbuffer1()
    env = W.envmap()
    split, seed = (16, 8, 8), 5
    dev = torch.device("cuda", 0)
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, dev)
    scene_t = grt.Scene(ctx, *scene_tensors(tgt))
    target = grt.render_mis(scene_t, E, G, split=split, seed=seed)["rgb"]
    del scene_t
    scene = grt.Scene(ctx, *scene_tensors(s))
    hits = grt.make_hit_list(gb.npix, sum(split), cap, dev) if cap else None
    fwd = grt.render_mis(scene, E, G, split=split, seed=seed, save=True, hits=hits, hit_cap=cap)
    valid = np.nonzero(gb.valid)[0]
    pix = np.sort(np.random.default_rng(7).choice(valid, 64, replace=False))
    ref_f = O.render_mis(s, gb, env, split, seed, pix=pix, dump=True)
    m = ref_f["margins"]
    clear = ~((m[..., 3] < 1e-5) | (m[..., 4] < 1e-9)).any(axis=1)
    pix = pix[clear][:48]
    assert len(pix) == 48
    up = torch.zeros(gb.npix, 3, device=dev)
    idx = torch.from_numpy(pix).to(dev)
    up[idx] = 2.0 * (fwd["rgb"][idx] - target[idx])
    gg = grt.render_mis_backward(scene, E, G, up, fwd["saved"], split=split, seed=seed, hits=hits, hit_cap=cap)
    torch.cuda.synchronize()
    ref = O.render_mis_backward(s, gb, env, split, seed, up[idx].cpu().numpy().astype(np.float64), pix=pix, with_abs=True)
    check_grads({k: v.cpu().numpy() for k, v in gg.items()}, ref)
    assert np.count_nonzero(ref[0][:, 10]) >= 64  # at least 64 surfels carry gradient
