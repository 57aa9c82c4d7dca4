"""Pins of the oracle's mesh backend of the attribute query (Sec. 3.5.2,
closest-hit ray-triangle query with barycentric attributes) against closed
forms, an independent linear solve and invariants."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W


def tri_mesh(tris_xyz, attrs=None, normals=None, seed=0):
    g = np.random.default_rng(seed)
    v = np.asarray(tris_xyz, np.float32).reshape(-1, 3)
    n = v.shape[0]
    f = np.arange(n, dtype=np.int32).reshape(-1, 3)
    if normals is None:
        normals = np.tile([0.0, 0.0, 1.0], (n, 1))
    a = attrs if attrs is not None else (g.uniform(0, 1, (n, 3)), g.uniform(0.05, 1, n), g.uniform(0, 1, n))
    return W.Mesh(v, f, *(np.asarray(x, np.float32) for x in a), np.asarray(normals, np.float32))


@pytest.mark.parametrize("seed", range(6))
def test_hit_point_and_barycentric_attributes(seed):
    """A ray aimed at the point (1-u-v) a + u b + v c of a random triangle:
    t = the distance, and every attribute is that barycentric mix (solved
    independently with numpy.linalg)."""
    g = np.random.default_rng(seed)
    tri = g.uniform(-1, 1, (3, 3))
    u, v = g.uniform(0.05, 0.45, 2)
    P = (1 - u - v) * tri[0] + u * tri[1] + v * tri[2]
    o = P + g.uniform(0.5, 2.0) * np.array([0.2, 0.3, 1.0]) / np.linalg.norm([0.2, 0.3, 1.0])
    d = (P - o) / np.linalg.norm(P - o)
    nrm = g.standard_normal((3, 3)); nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    m = tri_mesh(tri, normals=nrm, seed=seed)
    out = O.mesh_trace_attr(m, o[None].astype(np.float32), d[None].astype(np.float32))
    # the same barycentrics by a linear solve o + t d = a + u' (b-a) + v' (c-a)
    of, df, tf = o.astype(np.float32).astype(float), d.astype(np.float32).astype(float), m.verts.astype(float)
    M = np.stack([-df, tf[1] - tf[0], tf[2] - tf[0]], 1)
    t, uu, vv = np.linalg.solve(M, of - tf[0])
    w = np.array([1 - uu - vv, uu, vv])
    assert out["V"][0] == 0.0
    np.testing.assert_allclose(out["albedo"][0], w @ m.albedo.astype(float), rtol=1e-9)
    np.testing.assert_allclose(out["rough"][0], w @ m.rough.astype(float), rtol=1e-9)
    np.testing.assert_allclose(out["metal"][0], w @ m.metal.astype(float), rtol=1e-9, atol=1e-12)
    n = w @ m.normal.astype(float)
    n = n if n @ df <= 0 else -n
    np.testing.assert_allclose(out["normal"][0], n, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(out["margins"][0, 0], min(w), rtol=1e-8)


def test_closest_of_stacked_triangles_and_t_range():
    """Three parallel triangles at z = 0, -1, -2 under a ray going down: the
    first is returned; with t_min past it, the second; t_max before it: miss."""
    base = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], float)
    tris = np.concatenate([base + [0, 0, -k] for k in range(3)])
    albedo = np.repeat(np.eye(3), 3, axis=0)  # triangle k is coloured e_k
    m = tri_mesh(tris, attrs=(albedo, np.full(9, 0.5), np.zeros(9)))
    o = np.float32([[0, 0, 1]]); d = np.float32([[0, 0, -1]])
    np.testing.assert_allclose(O.mesh_trace_attr(m, o, d)["albedo"][0], [1, 0, 0])
    np.testing.assert_allclose(O.mesh_trace_attr(m, o, d, t_min=1.5)["albedo"][0], [0, 1, 0])
    out = O.mesh_trace_attr(m, o, d, t_max=0.9)
    assert out["V"][0] == 1.0 and not out["albedo"].any()
    np.testing.assert_allclose(O.mesh_trace_attr(m, o, d)["margins"][0, 1], 1.0)  # (2 - 1) / 1


def test_two_sided_and_miss():
    """Back faces count (the normal still faces the origin); rays beside the
    triangle or parallel to it miss."""
    tri = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], float)
    m = tri_mesh(tri)
    up = O.mesh_trace_attr(m, np.float32([[0, 0, -1]]), np.float32([[0, 0, 1]]))
    assert up["V"][0] == 0.0
    np.testing.assert_allclose(up["normal"][0], [0, 0, -1])
    side = O.mesh_trace_attr(m, np.float32([[3, 3, 1], [0, 0, 0.5]]), np.float32([[0, 0, -1], [1, 0, 0]]))
    assert (side["V"] == 1.0).all()


def test_triangle_order_does_not_matter():
    """Shuffling the triangles changes nothing (no ties in a random soup)."""
    m = W.tri_soup(400, seed=1)
    g = np.random.default_rng(2)
    o = g.uniform(-1, 1, (300, 3)).astype(np.float32)
    d = g.standard_normal((300, 3)); d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    a = O.mesh_trace_attr(m, o, d)
    perm = g.permutation(m.nf)
    mp = W.Mesh(m.verts, np.ascontiguousarray(m.tris[perm]), m.albedo, m.rough, m.metal, m.normal)
    b = O.mesh_trace_attr(mp, o, d)
    assert (a["V"] < 1).sum() > 30
    for k in ("V", "albedo", "rough", "metal", "normal"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-12, atol=1e-15)


def test_relight_through_an_empty_mesh_is_the_radiance_estimator():
    """No triangles: every secondary ray sees the environment (V = 1), so the
    mesh-backed relit image equals the radiance render with no geometry."""
    gb = W.gbuffer1(16, 16, seed=2)
    env = W.envmap(32, 64, seed=4)
    z = np.zeros
    m = W.Mesh(z((3, 3), np.float32), z((0, 3), np.int32), z((3, 3), np.float32), z(3, np.float32),
               z(3, np.float32), z((3, 3), np.float32))
    s = W.Surfels(z((0, 3), np.float32), z((0, 2), np.float32), z((0, 4), np.float32), z(0, np.float32),
                  z((0, 3), np.float32))
    np.testing.assert_array_equal(O.render_relight_mesh(m, gb, env, (4, 2, 2), seed=5),
                                  O.render_mis(s, gb, env, (4, 2, 2), seed=5))


def test_relight_under_a_mesh_ceiling():
    """A pixel under a large two-triangle ceiling that every upward ray hits
    (V = 0): with a constant environment L0 and metallic 1, L_i = L0 (a A + B)
    for the interpolated albedo a, within the DFG table's range."""
    L0 = 0.6
    env = np.full((32, 64, 3), L0, np.float32)
    v = np.float32([[-50, -50, 1], [50, -50, 1], [50, 50, 1], [-50, 50, 1]])
    f = np.int32([[0, 1, 2], [0, 2, 3]])
    m = W.Mesh(v, f, np.full((4, 3), 0.7, np.float32), np.full(4, 0.4, np.float32), np.ones(4, np.float32),
               np.tile(np.float32([0, 0, -1]), (4, 1)))
    gb = W.GBuffer(1, 1, np.float32([[0, 0, 0]]), np.float32([[0, 0, 1]]), np.float32([[0, 0.6, 0.8]]),
                   np.float32([[0.5, 0.5, 0.5]]), np.float32([0.5]), np.float32([0.0]), np.uint8([1]))
    d = O.render_relight_mesh(m, gb, env, (8, 4, 4), seed=3, dump=True)
    lut = O.dfg_lut()
    tr = d["traced"][0].astype(bool)
    Li = d["Li"][0][tr]
    assert tr.sum() > 8
    lo, hi = L0 * (0.7 * lut[..., 0] + lut[..., 1]).min(), L0 * (0.7 * lut[..., 0] + lut[..., 1]).max()
    assert (Li >= lo - 1e-9).all() and (Li <= hi + 1e-9).all()
    assert np.allclose(Li[:, 0], Li[:, 1]) and np.allclose(Li[:, 1], Li[:, 2])  # grey albedo, grey light
