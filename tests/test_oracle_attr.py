"""Pins of the oracle's attribute query (Sec. 3.5.1, Eq. trace_attr, the
Gaussian backend: material attributes of the ordered hits averaged with the
normalized blending weights of Eq. deferred_maps, and V from the accumulated
opacity) against closed forms, invariants and special cases."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W


def frame_of(quat_wxyz):
    """(t_u, t_v, n) from scipy's rotation matrix (an independent route)."""
    q = np.asarray(quat_wxyz, dtype=np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    return R[:, 0], R[:, 1], R[:, 2]


def surfels(mus, scales, quats, ops):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
    n = len(mus)
    return W.Surfels(f(mus), f(scales), f(quats), f(ops), f(np.zeros((n, 3))))


def attrs_of(g, n):
    return (g.uniform(0, 1, (n, 3)).astype(np.float32), g.uniform(0.05, 1, n).astype(np.float32),
            (g.uniform(0, 1, n) < 0.5).astype(np.float32))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("side", [1.0, -1.0])
def test_single_surfel_returns_its_attributes(seed, side):
    """One hit: its weight normalizes to 1, so the query returns the surfel's
    albedo, roughness and metallic exactly, its normal turned to face the ray
    origin, and V = 1 - alpha with alpha = o exp(-(u0^2+v0^2)/2)."""
    g = np.random.default_rng(seed)
    q = g.standard_normal(4); q /= np.linalg.norm(q)
    tu, tv, n = frame_of(q)
    mu = g.uniform(-1, 1, 3); su, sv = g.uniform(0.05, 0.3, 2); op = g.uniform(0.4, 0.99)
    u0, v0 = g.uniform(-1.5, 1.5, 2); z = g.uniform(0.5, 2.0)
    o = mu + u0 * su * tu + v0 * sv * tv + side * z * n   # from either side of the disk
    s = surfels([mu], [(su, sv)], [q], [op])
    at = attrs_of(g, 1)
    out = O.trace_attr(s, at, o[None], (-side * n)[None])
    alpha = op * np.exp(-0.5 * (u0 ** 2 + v0 ** 2))
    np.testing.assert_allclose(out["V"][0], 1 - alpha, rtol=1e-5)
    np.testing.assert_allclose(out["albedo"][0], at[0][0], rtol=1e-6)
    np.testing.assert_allclose(out["rough"][0], at[1][0], rtol=1e-6)
    np.testing.assert_allclose(out["metal"][0], at[2][0], atol=1e-7)
    np.testing.assert_allclose(out["normal"][0], side * n, atol=1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_two_stacked_surfels_closed_form(seed):
    """Two parallel disks on the ray at depths z1 < z2: weights
    a1 / (a1 + (1-a1) a2) and (1-a1) a2 / (a1 + (1-a1) a2), and
    V = (1-a1)(1-a2); opposite normals both come back facing the origin."""
    g = np.random.default_rng(10 + seed)
    q = g.standard_normal(4); q /= np.linalg.norm(q)
    # the same plane with its normal flipped: a half turn about the local t_u
    r2 = Rotation.from_quat([q[1], q[2], q[3], q[0]]) * Rotation.from_rotvec([np.pi, 0, 0])
    x2 = r2.as_quat()
    q2 = np.array([x2[3], x2[0], x2[1], x2[2]])
    tu, tv, n = frame_of(q)
    n2 = frame_of(q2)[2]
    assert np.allclose(n2, -n, atol=1e-12)
    base = g.uniform(-1, 1, 3)
    z1, z2 = 0.4, 1.1
    ops = g.uniform(0.3, 0.9, 2)
    mus = [base - z1 * n, base - z2 * n]
    s = surfels(mus, [(0.2, 0.3), (0.25, 0.15)], [q, q2], ops)
    at = attrs_of(g, 2)
    o = base + 0.05 * tu
    d = -n
    out = O.trace_attr(s, at, o[None], d[None])
    uu = np.array([0.05 / 0.2, 0.05 / 0.25])
    a = ops * np.exp(-0.5 * uu ** 2)
    w1, w2 = a[0], (1 - a[0]) * a[1]
    W_ = w1 + w2
    np.testing.assert_allclose(out["V"][0], (1 - a[0]) * (1 - a[1]), rtol=1e-5)
    np.testing.assert_allclose(out["albedo"][0], (w1 * at[0][0] + w2 * at[0][1]) / W_, rtol=1e-5)
    np.testing.assert_allclose(out["rough"][0], (w1 * at[1][0] + w2 * at[1][1]) / W_, rtol=1e-5)
    np.testing.assert_allclose(out["metal"][0], (w1 * at[2][0] + w2 * at[2][1]) / W_, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(out["normal"][0], n, atol=1e-5)  # both face the origin (+n)


def test_miss_and_empty_scene():
    """No composited hit: V = 1 and all attributes 0."""
    g = np.random.default_rng(5)
    s = surfels([(0, 0, 0)], [(0.1, 0.1)], [(1, 0, 0, 0)], [0.8])
    at = attrs_of(g, 1)
    out = O.trace_attr(s, at, np.float32([[5, 5, 1]]), np.float32([[0, 0, -1]]))
    assert out["V"][0] == 1.0
    assert not out["albedo"].any() and not out["rough"].any() and not out["metal"].any() and not out["normal"].any()
    e = surfels(np.zeros((0, 3)), np.zeros((0, 2)), np.zeros((0, 4)), np.zeros(0))
    out = O.trace_attr(e, (np.zeros((0, 3), np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32)),
                       np.float32([[0, 0, 1]]), np.float32([[0, 0, -1]]))
    assert out["V"][0] == 1.0 and not out["albedo"].any()


def _random_case(seed, nr=300):
    g = np.random.default_rng(seed)
    s = W.scene0(n=400, seed=seed)
    at = attrs_of(g, s.n)
    o = g.uniform(-1, 1, (nr, 3)).astype(np.float32)
    d = g.standard_normal((nr, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    return s, at, o, d.astype(np.float32)


@pytest.mark.parametrize("seed", range(3))
def test_constant_attributes_pass_through(seed):
    """The weights are normalized: with equal attributes on every surfel, every
    ray with a hit returns exactly those attributes."""
    s, at, o, d = _random_case(seed)
    n = s.n
    const = (np.tile(np.float32([0.3, 0.6, 0.9]), (n, 1)), np.full(n, 0.42, np.float32), np.full(n, 0.7, np.float32))
    out = O.trace_attr(s, const, o, d)
    hit = out["V"] < 1.0
    assert hit.sum() > 20
    np.testing.assert_allclose(out["albedo"][hit], np.tile([0.3, 0.6, 0.9], (hit.sum(), 1)), rtol=1e-6)
    np.testing.assert_allclose(out["rough"][hit], 0.42, rtol=1e-6)
    np.testing.assert_allclose(out["metal"][hit], 0.7, rtol=1e-6)
    # averaged unit normals: length at most 1, and facing the ray origin
    nn = np.linalg.norm(out["normal"][hit], axis=1)
    assert np.all(nn <= 1 + 1e-9)
    assert np.all(np.einsum("ij,ij->i", out["normal"][hit], d[hit].astype(np.float64)) <= 1e-9)


@pytest.mark.parametrize("seed", range(2))
def test_visibility_equals_trace_transmittance_and_permutation(seed):
    """V is the transmittance the radiance trace ends with (1 - o_rt), and the
    query does not depend on the order the surfels are given in."""
    s, at, o, d = _random_case(20 + seed)
    out = O.trace_attr(s, at, o, d)
    tr = O.trace(s, o, d)
    np.testing.assert_allclose(out["V"], tr["T"], rtol=1e-12, atol=0)
    perm = np.random.default_rng(seed).permutation(s.n)
    sp = W.Surfels(*(np.ascontiguousarray(a[perm]) for a in (s.means, s.scales, s.quats, s.opacity, s.rgb)))
    atp = tuple(np.ascontiguousarray(a[perm]) for a in at)
    outp = O.trace_attr(sp, atp, o, d)
    # ids change with the permutation, so only pairs of equal depth could reorder
    for k in ("V", "albedo", "rough", "metal", "normal"):
        np.testing.assert_allclose(outp[k], out[k], rtol=1e-9, atol=1e-12)
