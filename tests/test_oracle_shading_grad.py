"""Pins of the oracle's gradient of the MIS estimator (Sec. 3.4.1 Eq. mis)
with respect to each pixel's shading state (Sec. 3.3 "Shading state",
Eq. deferred_maps): the position x the secondary rays leave from, the
normal, the view direction, albedo, roughness and metallic.  Reading 36 holds
each sample's direction and mixture pdf fixed, as the radiance backward
holds the hit set fixed.

- x, albedo, metallic: neither the sampled directions nor the pdfs depend on
  them, so central differences of the oracle's own forward pin them.
- n, wo, roughness (and albedo, metallic again): float64 torch autograd of an
  independent formulation of sum_j f(wo, w_j) (w_j . n) / q_j L_j, with the
  samples' directions, pdfs and incident radiance from the oracle's dump.
- The BRDF partials are also checked against central differences of the
  BRDF itself at fixed directions."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W


def cube_scene():
    """Two nested cubes of six large surfels each (half sizes 1 and 1.3,
    scale 3): every ray from near the centre crosses one wall of each at
    rho^2 well inside the support, so everything is smooth in the origin."""
    means, quats = [], []
    for hs in (1.0, 1.3):
        for ax in range(3):
            for sgn in (-1.0, 1.0):
                m = [0.0, 0.0, 0.0]
                m[ax] = sgn * hs
                means.append(m)
                # frame whose normal is the axis: rotate +z onto it
                q = {0: (math.cos(math.pi / 4), 0.0, math.sin(math.pi / 4), 0.0),
                     1: (math.cos(math.pi / 4), -math.sin(math.pi / 4), 0.0, 0.0),
                     2: (1.0, 0.0, 0.0, 0.0)}[ax]
                quats.append(q)
    n = len(means)
    g = np.random.default_rng(0)
    return W.Surfels(np.float32(means), np.full((n, 2), 3.0, np.float32), np.float32(quats),
                     g.uniform(0.4, 0.7, n).astype(np.float32), g.uniform(0.1, 0.9, (n, 3)).astype(np.float32))


def shading_buffer(npx, seed):
    g = np.random.default_rng(seed)
    x = g.uniform(-0.3, 0.3, (npx, 3))
    n = g.standard_normal((npx, 3)); n /= np.linalg.norm(n, axis=1, keepdims=True)
    t = np.cross(n, g.standard_normal((npx, 3))); t /= np.linalg.norm(t, axis=1, keepdims=True)
    ang = g.uniform(0.2, 1.2, (npx, 1))
    wo = np.cos(ang) * n + np.sin(ang) * t
    # stored vectors slightly off unit length, so the normalisation is exercised
    n *= g.uniform(0.9, 1.1, (npx, 1)); wo *= g.uniform(0.9, 1.1, (npx, 1))
    f = lambda a: np.ascontiguousarray(a, np.float32)
    return W.GBuffer(1, npx, f(x), f(n), f(wo), f(g.uniform(0.1, 0.9, (npx, 3))), f(g.uniform(0.3, 0.9, npx)),
                     f(g.uniform(0.0, 1.0, npx)), np.ones(npx, np.uint8))


SPLIT = (8, 4, 4)


def loss(s, gb, env, G, seed=5):
    return float((O.render_mis(s, gb, env, SPLIT, seed) * G).sum())


def test_position_albedo_metallic_against_central_differences():
    s = cube_scene()
    gb = shading_buffer(6, 1)
    env = W.envmap(32, 64, seed=2)
    G = np.random.default_rng(3).normal(0, 1, (gb.npix, 3))
    _, shade = O.render_mis_backward(s, gb, env, SPLIT, 5, G, shading=True)
    h = 2.0 ** -12
    for p in range(gb.npix):
        for c in range(3):
            vals = []
            for sgn in (1, -1):
                g2 = W.GBuffer(*(np.array(a, copy=True) if isinstance(a, np.ndarray) else a
                                 for a in (gb.H, gb.W) + gb.arrays()))
                g2.x[p, c] = gb.x[p, c] + sgn * h
                vals.append(loss(s, g2, env, G))
            fd = (vals[0] - vals[1]) / (2 * h)
            np.testing.assert_allclose(shade[p, c], fd, rtol=2e-5, atol=1e-9, err_msg=f"x[{p},{c}]")
        for key, col in (("albedo", 9), ("metal", 12 + 1)):
            for c in (range(3) if key == "albedo" else [None]):
                vals = []
                for sgn in (1, -1):
                    g2 = W.GBuffer(*(np.array(a, copy=True) if isinstance(a, np.ndarray) else a
                                     for a in (gb.H, gb.W) + gb.arrays()))
                    arr = getattr(g2, key)
                    if c is None:
                        arr[p] += sgn * 0.01
                    else:
                        arr[p, c] += sgn * 0.01
                    vals.append(loss(s, g2, env, G))
                fd = (vals[0] - vals[1]) / (2 * 0.01)
                want = shade[p, col + (c or 0)] if c is not None else shade[p, col]
                np.testing.assert_allclose(want, fd, rtol=1e-6, atol=1e-10, err_msg=f"{key}[{p},{c}]")
    assert np.abs(shade[:, 0:3]).max() > 1e-3  # the position term is exercised


def torch_estimator(gb, d, G, spp):
    """sum over pixels and samples of G . f(wo, w) (w . n) / q * L, in float64
    torch from the formulas (GGX D with alpha = r^2, Smith G1, Schlick F on
    w.h, F0 = 0.04 (1 - m) + m a; n and wo normalised inside)."""
    import torch
    dt = torch.float64
    n = torch.tensor(gb.n, dtype=dt, requires_grad=True)
    wo = torch.tensor(gb.wo, dtype=dt, requires_grad=True)
    a = torch.tensor(gb.albedo, dtype=dt, requires_grad=True)
    r = torch.tensor(gb.rough, dtype=dt, requires_grad=True)
    m = torch.tensor(gb.metal, dtype=dt, requires_grad=True)
    w = torch.tensor(d["dir"], dtype=dt)
    q = torch.tensor(d["q"], dtype=dt)
    L = torch.tensor(d["Li"], dtype=dt)
    tr = torch.tensor(d["traced"].astype(bool) & (d["q"] > 0))
    nh = n / n.norm(dim=1, keepdim=True)
    oh = wo / wo.norm(dim=1, keepdim=True)
    nn, oo = nh[:, None, :], oh[:, None, :]
    ni = (w * nn).sum(-1)
    no = (oo * nn).sum(-1).expand_as(ni)
    hv = w + oo
    hv = hv / hv.norm(dim=-1, keepdim=True)
    ndh = (hv * nn).sum(-1)
    idh = (w * hv).sum(-1)
    a2 = (r ** 4)[:, None]
    Dg = a2 / (math.pi * (ndh ** 2 * (a2 - 1) + 1) ** 2)
    g1 = lambda v: 2 * v / (v + torch.sqrt(a2 + (1 - a2) * v * v))
    Gs = g1(ni) * g1(no)
    x5 = torch.clamp(1 - idh, min=0) ** 5
    F0 = 0.04 * (1 - m)[:, None, None] + m[:, None, None] * a[:, None, :]
    F = F0 + (1 - F0) * x5[..., None]
    f = (1 - m)[:, None, None] * a[:, None, :] / math.pi + (Dg * Gs / (4 * ni * no))[..., None] * F
    gt = f * ni[..., None] / torch.where(tr, q, torch.ones_like(q))[..., None] * L
    gt = torch.where(tr[..., None], gt, torch.zeros_like(gt))
    total = (torch.tensor(G, dtype=dt)[:, None, :] * gt).sum() / spp
    total.backward()
    return {k: v.grad.numpy() for k, v in dict(n=n, wo=wo, albedo=a, rough=r, metal=m).items()}


@pytest.mark.parametrize("seed", [1, 2])
def test_direction_and_roughness_terms_against_autograd(seed):
    s = cube_scene()
    gb = shading_buffer(8, 10 + seed)
    env = W.envmap(32, 64, seed=4)
    G = np.random.default_rng(seed).normal(0, 1, (gb.npix, 3))
    d = O.render_mis(s, gb, env, SPLIT, 5, dump=True)
    _, shade = O.render_mis_backward(s, gb, env, SPLIT, 5, G, shading=True)
    want = torch_estimator(gb, d, G, sum(SPLIT))
    # sample directions reach the torch side rounded to float32 (the dump)
    np.testing.assert_allclose(shade[:, 3:6], want["n"], rtol=2e-4, atol=1e-7)
    np.testing.assert_allclose(shade[:, 6:9], want["wo"], rtol=2e-4, atol=1e-7)
    np.testing.assert_allclose(shade[:, 9:12], want["albedo"], rtol=2e-4, atol=1e-7)
    np.testing.assert_allclose(shade[:, 12], want["rough"], rtol=2e-4, atol=1e-7)
    np.testing.assert_allclose(shade[:, 13], want["metal"], rtol=2e-4, atol=1e-7)
    assert np.abs(want["n"]).max() > 1e-3 and np.abs(want["rough"]).max() > 1e-3


def test_invalid_and_backfacing_pixels_get_nothing():
    s = cube_scene()
    gb = shading_buffer(4, 3)
    gb.valid[1] = 0
    gb.wo[2] = -gb.n[2]  # the view direction below the surface
    env = W.envmap(16, 32, seed=1)
    _, shade = O.render_mis_backward(s, gb, env, SPLIT, 5, np.ones((4, 3)), shading=True)
    assert np.all(shade[1] == 0) and np.all(shade[2] == 0)
    assert np.abs(shade[0]).max() > 0 and np.abs(shade[3]).max() > 0
