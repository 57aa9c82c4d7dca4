"""Pins of the oracle's primary-ray G-buffer by 2DGRT (Eq. deferred_maps on
traced primary rays): closed forms at single and stacked surfels, the
telescoping identity sum_k T_k a_k = 1 - T that ties the colour map to the
radiance trace, and coverage by accumulated opacity."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W


def frame_of(q):
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    return R[:, 0], R[:, 1], R[:, 2]


def surfels(mus, scales, quats, ops, rgbs):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
    return W.Surfels(f(mus), f(scales), f(quats), f(ops), f(rgbs))


@pytest.mark.parametrize("seed", range(4))
def test_single_surfel(seed):
    """Depth = z, x = the crossing point, the surfel's own materials and
    colour, the normal facing the camera; covered iff alpha >= 1/2."""
    g = np.random.default_rng(seed)
    q = g.standard_normal(4); q /= np.linalg.norm(q)
    tu, tv, n = frame_of(q)
    mu = g.uniform(-1, 1, 3); su, sv = g.uniform(0.1, 0.3, 2)
    op = [0.95, 0.45, 0.9, 0.4][seed]
    u0, v0 = g.uniform(-0.6, 0.6, 2); z = g.uniform(0.5, 2.0)
    side = 1.0 if seed % 2 == 0 else -1.0
    o = mu + u0 * su * tu + v0 * sv * tv + side * z * n
    c = g.uniform(0, 1, 3)
    s = surfels([mu], [(su, sv)], [q], [op], [c])
    at = (g.uniform(0, 1, (1, 3)).astype(np.float32), np.float32([0.3]), np.float32([1.0]))
    out = O.trace_gbuffer(s, at, o[None], (-side * n)[None])
    alpha = op * np.exp(-0.5 * (u0 ** 2 + v0 ** 2))
    if alpha < 0.5:
        assert out["valid"][0] == 0 and not out["x"].any() and not out["rgb"].any()
        return
    assert out["valid"][0] == 1
    np.testing.assert_allclose(out["depth"][0], z, rtol=1e-5)
    np.testing.assert_allclose(out["x"][0], mu + u0 * su * tu + v0 * sv * tv, atol=1e-5)
    np.testing.assert_allclose(out["n"][0], side * n, atol=1e-6)
    np.testing.assert_allclose(out["wo"][0], side * n, atol=1e-6)
    np.testing.assert_allclose(out["albedo"][0], at[0][0], rtol=1e-6)
    np.testing.assert_allclose(out["rgb"][0], c.astype(np.float32), rtol=1e-6)


def test_two_stacked_surfels_depth():
    """Parallel disks at depths z1 < z2 along the ray: depth is the
    normalized-weight mean (w1 z1 + w2 z2) / (w1 + w2)."""
    q = np.array([1.0, 0, 0, 0])
    z1, z2 = 0.5, 1.25
    ops = np.array([0.6, 0.8])
    s = surfels([(0, 0, -z1), (0, 0, -z2)], [(0.3, 0.3), (0.3, 0.3)], [q, q], ops, [(1, 0, 0), (0, 1, 0)])
    at = (np.float32([[0.2, 0.2, 0.2], [0.8, 0.8, 0.8]]), np.float32([0.1, 0.9]), np.float32([0, 1]))
    out = O.trace_gbuffer(s, at, np.float32([[0, 0, 0]]), np.float32([[0, 0, -1]]))
    w1, w2 = ops[0], (1 - ops[0]) * ops[1]
    np.testing.assert_allclose(out["depth"][0], (w1 * z1 + w2 * z2) / (w1 + w2), rtol=1e-6)
    np.testing.assert_allclose(out["rgb"][0], [w1 / (w1 + w2), w2 / (w1 + w2), 0], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(out["rough"][0], (0.1 * w1 + 0.9 * w2) / (w1 + w2), rtol=1e-5)
    np.testing.assert_allclose(out["n"][0], [0, 0, 1], atol=1e-12)


@pytest.mark.parametrize("seed", range(2))
def test_colour_map_is_the_trace_over_its_opacity(seed):
    """Telescoping: sum_k T_k a_k = 1 - T_fin, so the colour map equals the
    radiance trace's c_rt / (1 - T) on every covered pixel, and coverage is
    exactly 1 - T >= the threshold."""
    g = np.random.default_rng(seed)
    s = W.scene0(n=4096, seed=seed)
    at = W.surfel_materials(s.n, seed=seed)
    o = g.uniform(-1, 1, (400, 3)).astype(np.float32)
    d = g.standard_normal((400, 3)); d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    for thr in (0.5, 0.2):
        out = O.trace_gbuffer(s, at, o, d, min_opacity=thr)
        tr = O.trace(s, o, d)
        cov = (1 - tr["T"]) >= thr
        np.testing.assert_array_equal(out["valid"].astype(bool), cov & (tr["nhit"] > 0))
        v = out["valid"].astype(bool)
        assert v.sum() > 10
        np.testing.assert_allclose(out["rgb"][v], tr["C"][v] / (1 - tr["T"][v])[:, None], rtol=1e-9)
        np.testing.assert_allclose(np.linalg.norm(out["n"][v], axis=1), 1.0, rtol=1e-12)
        np.testing.assert_allclose(out["x"][v], o[v] + out["depth"][v][:, None] * d[v], rtol=1e-12, atol=1e-12)


def test_miss_is_uncovered():
    s = surfels([(0, 0, 0)], [(0.1, 0.1)], [(1, 0, 0, 0)], [0.9], [(1, 1, 1)])
    at = (np.float32([[1, 1, 1]]), np.float32([0.5]), np.float32([0.0]))
    out = O.trace_gbuffer(s, at, np.float32([[3, 3, 1]]), np.float32([[0, 0, -1]]))
    assert out["valid"][0] == 0 and not out["depth"].any() and not out["n"].any()
