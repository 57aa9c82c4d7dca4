"""GPU parity of the backward of the primary-ray G-buffer (Eq. deferred_maps
on traced camera rays; Sec. 3.3) against the oracle's gradients, which are
pinned by a closed form, float64 autograd and finite differences.

Tolerance per parameter block (surfel parameters and attributes):
|g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 max|g_ref|_block) element-wise on all
but 0.1% of the entries, and relative L2 error <= 1e-3.  Upstream gradients
are kept off the knife edges that a float32 forward may take the other way
(coverage within 1e-5 of its threshold, the cutoff's stop margin) and off
pixels whose averaged normal nearly vanishes (|N| / W < 0.05, where the
normal map's derivative is ill-conditioned)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W

pytestmark = pytest.mark.gpu

BLOCKS = dict(means=(0, 3), scales=(3, 5), quats=(5, 9), opacity=(9, 10), rgb=(10, 13))
ABLOCKS = dict(albedo=(0, 3), rough=(3, 4), metal=(4, 5))
DIM = dict(x=3, n=3, albedo=3, rgb=3, rough=1, metal=1, depth=1)


@pytest.fixture(scope="module")
def grt_ctx():
    from paper_2607_22780_amd import grt
    return grt, grt.Context(0)


def close(got, want, name, rel=1e-3, floor=1e-2, want_abs=None):
    from gpu_util import grad_close
    grad_close(got, want, name, want_abs, rel=rel, floor=floor)


def check(gg, ga, ref13, refa, ref13_abs=None, refa_abs=None, **kw):
    for name, (a, b) in BLOCKS.items():
        close(gg[name].cpu().numpy(), ref13[:, a:b], name,
              want_abs=None if ref13_abs is None else ref13_abs[:, a:b], **kw)
    for name, (a, b) in ABLOCKS.items():
        close(ga[name].cpu().numpy(), refa[:, a:b], name,
              want_abs=None if refa_abs is None else refa_abs[:, a:b], **kw)


def camera(H, Wd, seed=0):
    g = np.random.default_rng(seed)
    v = g.standard_normal(3); v[1] = 0.3 * abs(v[1]); v /= np.linalg.norm(v)
    o, d = W.pinhole(3.5 * v, (0.0, 0.0, 0.0), 40.0, H, Wd)
    return o.astype(np.float32), d.astype(np.float32)


def upstream(s, at, o, d, thr, seed, keys=tuple(DIM)):
    """Seeded upstream gradients, zero off the knife edges and where the
    averaged normal nearly vanishes."""
    tr = O.trace(s, o, d)
    nb = np.linalg.norm(O.trace_attr(s, at, o, d)["normal"], axis=1)
    keep = ~((np.abs((1 - tr["T"]) - thr) < 1e-5) | (tr["margins"][:, 3] < 1e-5) | (nb < 0.05))
    g = np.random.default_rng(seed)
    up = {}
    for k in keys:
        v = g.normal(0, 1, (len(o), DIM[k])) * keep[:, None]
        up[k] = (v[:, 0] if DIM[k] == 1 else v).astype(np.float32)
    return up, keep


def run_gpu(grt, ctx, s, at, o, d, H, Wd, up, thr, k=12, scene=None):
    from gpu_util import t, scene_tensors
    if scene is None:
        scene = grt.Scene(ctx, *scene_tensors(s))
    mats = [t(a) for a in at]
    fwd = grt.trace_gbuffer(scene, *mats, t(o), t(d), H, Wd, min_opacity=thr, k=k)
    gg, ga = grt.trace_gbuffer_backward(scene, *mats, t(o), t(d), fwd, {kk: t(v) for kk, v in up.items()}, k=k)
    torch.cuda.synchronize()
    return gg, ga, fwd, scene


@pytest.mark.parametrize("H,Wd,thr", [(48, 40, 0.5), (33, 17, 0.2)])
def test_gbuffer_backward_parity(grt_ctx, H, Wd, thr):
    grt, ctx = grt_ctx
    s = W.scene1(n=20000, seed=0, s_lo=0.01, s_hi=0.06)
    at = W.surfel_materials(s.n, seed=7)
    o, d = camera(H, Wd, seed=H)
    up, keep = upstream(s, at, o, d, thr, seed=H + 1)
    gg, ga, fwd, _ = run_gpu(grt, ctx, s, at, o, d, H, Wd, up, thr)
    assert fwd["valid"].float().mean().item() > 0.1
    ref13, refa, ref13_abs, refa_abs = O.trace_gbuffer_backward(s, at, o, d, {k: v.astype(np.float64) for k, v in up.items()},
                                           min_opacity=thr, with_abs=True)
    assert np.count_nonzero(ref13[:, 0]) >= 100
    check(gg, ga, ref13, refa, ref13_abs, refa_abs)


@pytest.mark.parametrize("keys", [("n",), ("depth", "x"), ("albedo", "rough", "metal"), ("rgb",)])
def test_gbuffer_backward_each_map(grt_ctx, keys):
    """One map at a time, so that no term hides behind another's scale."""
    grt, ctx = grt_ctx
    s = W.scene1(n=10000, seed=2, s_lo=0.01, s_hi=0.06)
    at = W.surfel_materials(s.n, seed=3)
    o, d = camera(24, 24, seed=5)
    up, _ = upstream(s, at, o, d, 0.5, seed=11, keys=keys)
    gg, ga, _, _ = run_gpu(grt, ctx, s, at, o, d, 24, 24, up, 0.5)
    ref13, refa, ref13_abs, refa_abs = O.trace_gbuffer_backward(s, at, o, d, {k: v.astype(np.float64) for k, v in up.items()},
                                           min_opacity=0.5, with_abs=True)
    check(gg, ga, ref13, refa, ref13_abs, refa_abs)


def test_gbuffer_backward_k_and_nothing_upstream(grt_ctx):
    """K, and bounding the re-traversal by the saved stop depth, only change
    the order of float atomics; zero upstream gradients, or gradients only on
    uncovered pixels, add exactly nothing; attribute gradients may be left
    out."""
    grt, ctx = grt_ctx
    from gpu_util import t, DEV
    s = W.scene1(n=10000, seed=1, s_lo=0.01, s_hi=0.06)
    at = W.surfel_materials(s.n, seed=8)
    o, d = camera(32, 24, seed=2)
    up, _ = upstream(s, at, o, d, 0.5, seed=4)
    gg12, ga12, fwd, scene = run_gpu(grt, ctx, s, at, o, d, 32, 24, up, 0.5, k=12)
    mats = [t(a) for a in at]
    # unbounded re-traversal (no saved stop depth) gives the same gradients
    fwd_nostop = {kk: v for kk, v in fwd.items() if kk != "stop"}
    gu, gau = grt.trace_gbuffer_backward(scene, *mats, t(o), t(d), fwd_nostop, {kk: t(v) for kk, v in up.items()})
    for name in BLOCKS:
        close(gu[name].cpu().numpy(), gg12[name].cpu().numpy().astype(np.float64), f"{name} unbounded", rel=1e-4)
    for name in ABLOCKS:
        close(gau[name].cpu().numpy(), ga12[name].cpu().numpy().astype(np.float64), f"{name} unbounded", rel=1e-4)
    for k in (1, 32):
        gk, gak, _, _ = run_gpu(grt, ctx, s, at, o, d, 32, 24, up, 0.5, k=k, scene=scene)
        for name in BLOCKS:
            close(gk[name].cpu().numpy(), gg12[name].cpu().numpy().astype(np.float64), f"{name} k={k}", rel=1e-4)
        for name in ABLOCKS:
            close(gak[name].cpu().numpy(), ga12[name].cpu().numpy().astype(np.float64), f"{name} k={k}", rel=1e-4)
    zero = {kk: torch.zeros_like(t(v)) for kk, v in up.items()}
    g0, a0 = grt.trace_gbuffer_backward(scene, *mats, t(o), t(d), fwd, zero)
    unc = (fwd["valid"] == 0)
    assert unc.any()
    only_unc = {kk: t(v) * (unc[:, None] if t(v).dim() == 2 else unc).float() for kk, v in up.items()}
    g1, a1 = grt.trace_gbuffer_backward(scene, *mats, t(o), t(d), fwd, only_unc)
    part = {"albedo": torch.zeros(s.n, 3, device=DEV), "rough": None, "metal": None}
    g2, a2 = grt.trace_gbuffer_backward(scene, *mats, t(o), t(d), fwd, {kk: t(v) for kk, v in up.items()},
                                        attr_grads=part)
    torch.cuda.synchronize()
    for gset in (g0, a0, g1, a1):
        for v in gset.values():
            assert not v.any()
    np.testing.assert_allclose(a2["albedo"].cpu().numpy(), ga12["albedo"].cpu().numpy(), rtol=1e-4, atol=1e-6)
    for name in BLOCKS:
        np.testing.assert_allclose(g2[name].cpu().numpy(), gg12[name].cpu().numpy(), rtol=1e-3,
                                   atol=1e-5 * max(1.0, float(gg12[name].abs().max())))


def test_gbuffer_backward_room_1024_sampled(grt_ctx):
    """At full size: the room (1M surfels), a 1024^2 camera inside it, the
    launch the bench times.  Upstream gradients sit on 48 seeded covered
    pixels clear of the knife edges; the oracle differentiates those pixels."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors, log
    s = W.scene3()
    at = W.surfel_materials(s.n, seed=0)
    H = Wd = 1024
    cam_o, cam_d = W.pinhole(*W.camera3(W.rng(3, 2)), 60.0, H, Wd)
    o, d = cam_o.astype(np.float32), cam_d.astype(np.float32)
    scene = grt.Scene(ctx, *scene_tensors(s))
    mats = [t(a) for a in at]
    fwd = grt.trace_gbuffer(scene, *mats, t(o), t(d), H, Wd)
    torch.cuda.synchronize()
    valid = np.nonzero(fwd["valid"].cpu().numpy())[0]
    pix = np.sort(np.random.default_rng(3).choice(valid, 96, replace=False))
    up_s, keep = upstream(s, at, o[pix], d[pix], 0.5, seed=6)
    sel = np.nonzero(keep)[0][:48]
    assert len(sel) == 48
    pix, up_s = pix[sel], {k: v[sel] for k, v in up_s.items()}
    log(f"room 1024^2 G-buffer backward, pixels {pix[:4]}...")
    up = {}
    for k, v in up_s.items():
        full = np.zeros((H * Wd,) + v.shape[1:], np.float32)
        full[pix] = v
        up[k] = t(full)
    gg, ga = grt.trace_gbuffer_backward(scene, *mats, t(o), t(d), fwd, up)
    torch.cuda.synchronize()
    ref13, refa, ref13_abs, refa_abs = O.trace_gbuffer_backward(s, at, o[pix], d[pix], {k: v.astype(np.float64) for k, v in up_s.items()}, with_abs=True)
    assert np.count_nonzero(ref13[:, 0]) >= 64
    check(gg, ga, ref13, refa, ref13_abs, refa_abs)


def test_gbuffer_backward_edge_cases(grt_ctx):
    """An empty scene covers nothing and gets no gradient; no rays is a
    no-op; a single pixel matches the oracle; a forward without its saved
    weight is refused."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors, DEV
    z = lambda *sh: np.zeros(sh, np.float32)
    scene0 = grt.Scene(ctx, *scene_tensors(W.Surfels(z(0, 3), z(0, 2), z(0, 4), z(0), z(0, 3))))
    mats0 = [t(z(0, 3)), t(z(0)), t(z(0))]
    o, d = camera(4, 3, seed=1)
    fwd = grt.trace_gbuffer(scene0, *mats0, t(o), t(d), 4, 3)
    assert not fwd["valid"].any()
    up = {k: torch.ones_like(fwd[k]) for k in DIM}
    gg, ga = grt.trace_gbuffer_backward(scene0, *mats0, t(o), t(d), fwd, up)
    torch.cuda.synchronize()
    assert all(v.numel() == 0 for v in gg.values()) and all(v.numel() == 0 for v in ga.values())
    s = W.scene1(n=20000, seed=0, s_lo=0.01, s_hi=0.06)
    at = W.surfel_materials(s.n, seed=7)
    scene = grt.Scene(ctx, *scene_tensors(s))
    mats = [t(a) for a in at]
    e3 = torch.empty(0, 3, device=DEV)
    f0 = grt.trace_gbuffer(scene, *mats, e3, e3.clone(), 0, 0)
    g0, a0 = grt.trace_gbuffer_backward(scene, *mats, e3, e3.clone(), f0, {})
    torch.cuda.synchronize()
    assert not any(v.any() for v in g0.values()) and not any(v.any() for v in a0.values())
    o1, d1 = camera(1, 1, seed=1)
    up1, keep = upstream(s, at, o1, d1, 0.5, seed=3)
    assert keep.all()
    gg1, ga1, fw1, _ = run_gpu(grt, ctx, s, at, o1, d1, 1, 1, up1, 0.5, scene=scene)
    ref13, refa, ref13_abs, refa_abs = O.trace_gbuffer_backward(s, at, o1, d1, {k: v.astype(np.float64) for k, v in up1.items()},
                                           min_opacity=0.5, with_abs=True)
    assert np.count_nonzero(ref13[:, 0]) >= 10
    check(gg1, ga1, ref13, refa, ref13_abs, refa_abs)
    bad = {k: v for k, v in fw1.items() if k != "weight"}
    with pytest.raises(grt.GrtError):
        grt.trace_gbuffer_backward(scene, *mats, t(o1), t(d1), bad, {k: t(v) for k, v in up1.items()})


def test_gbuffer_autograd_function(grt_ctx):
    """GBufferFn: torch.autograd drives the same forward and backward kernels
    (maps, then grads of sum_k g_k . map_k for surfels and attributes)."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene1(n=10000, seed=4, s_lo=0.01, s_hi=0.06)
    at = W.surfel_materials(s.n, seed=5)
    o, d = camera(24, 20, seed=3)
    up, _ = upstream(s, at, o, d, 0.5, seed=8)
    params = [t(a).requires_grad_(True) for a in s.arrays()]
    mats = [t(a).requires_grad_(True) for a in at]
    outs = grt.GBufferFn.apply(*params, *mats, ctx, t(o), t(d), 24, 20)
    maps = dict(zip(("x", "n", "albedo", "rough", "metal", "depth", "rgb"), outs[:7]))
    assert outs[7].dtype == torch.uint8 and not outs[7].requires_grad
    loss = sum((maps[k] * t(v).reshape(maps[k].shape)).sum() for k, v in up.items())
    loss.backward()
    torch.cuda.synchronize()
    scene = grt.Scene(ctx, *scene_tensors(s))
    mt = [t(a) for a in at]
    fwd = grt.trace_gbuffer(scene, *mt, t(o), t(d), 24, 20)
    gg, ga = grt.trace_gbuffer_backward(scene, *mt, t(o), t(d), fwd, {k: t(v) for k, v in up.items()})
    torch.cuda.synchronize()
    for p, name in zip(params, BLOCKS):
        close(p.grad.cpu().numpy(), gg[name].cpu().numpy().astype(np.float64), name, rel=1e-4)
    for m, name in zip(mats, ABLOCKS):
        close(m.grad.cpu().numpy(), ga[name].cpu().numpy().astype(np.float64), name, rel=1e-4)
    for k in ("x", "n", "albedo", "depth", "rgb"):
        np.testing.assert_array_equal(maps[k].detach().cpu().numpy(), fwd[k].cpu().numpy())
