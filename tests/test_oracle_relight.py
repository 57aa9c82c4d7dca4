"""Pins of the oracle's split-sum relighting (Sec. 3.5.1, Eq.
relight_splitsum): the prefiltered environment E, the DFG table, and the
relit MIS estimator, against closed forms, special cases, an independent
adaptive quadrature and the radiance estimator it reduces to."""
import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W


def grid_dirs(H, Wd):
    th = np.pi * (np.arange(H) + 0.5) / H
    ph = 2 * np.pi * (np.arange(Wd) + 0.5) / Wd
    T, P = np.meshgrid(th, ph, indexing="ij")
    return np.stack([np.sin(T) * np.cos(P), np.cos(T), np.sin(T) * np.sin(P)], -1)


def test_constant_environment_is_reproduced():
    """A constant environment L gives E_d = E_s = L at every direction and level."""
    e = np.full((64, 128, 3), 0.37, np.float32)
    Ed, Es = O.env_prefilter(e)
    L = float(np.float32(0.37))  # the environment is stored in single precision
    np.testing.assert_allclose(Ed, L, rtol=1e-12)
    np.testing.assert_allclose(Es, L, rtol=1e-12)


def test_linear_gradient_closed_form():
    """L(l) = 1 + l_y (and the same in every channel): the cosine lobe's mean
    direction is (2/3) n, so E_d(n) = 1 + (2/3) n_y; a GGX lobe about R gives
    1 + kappa(r) R_y with 2/3 <= kappa < 1, kappa growing as r falls."""
    H, Wd = 128, 256
    d = grid_dirs(H, Wd)
    e = np.repeat((1.0 + d[..., 1:2]), 3, -1).astype(np.float32)
    Ed, Es = O.env_prefilter(e)
    n = grid_dirs(O.PF_H, O.PF_W)
    np.testing.assert_allclose(Ed[..., 0], 1.0 + (2.0 / 3.0) * n[..., 1], atol=2e-3)
    sel = np.abs(n[..., 1]) > 0.3
    kappas = []
    for lvl in range(O.PF_L - 1):
        k = (Es[lvl, ..., 0] - 1.0)[sel] / n[..., 1][sel]
        assert k.std() < 0.01 * abs(k.mean()) + 2e-3, (lvl, k.std())
        kappas.append(k.mean())
    assert all(a > b for a, b in zip(kappas, kappas[1:]))  # sharper lobes follow R more closely
    assert kappas[-1] == pytest.approx(2.0 / 3.0, abs=2e-3) and kappas[0] < 1.0


def test_roughest_level_equals_the_diffuse_table():
    """At r = 1 (alpha = 1) the GGX distribution is the constant 1/pi, so the
    specular weights are the cosine weights: E_s(., 1) = E_d."""
    e = W.envmap(64, 128, seed=4)
    Ed, Es = O.env_prefilter(e)
    np.testing.assert_allclose(Es[-1], Ed, rtol=1e-10)


def test_single_texel_weighting():
    """One bright texel l* of solid angle dW: E_d(n) = L max(0, n.l*) dW / S(n)
    with S(n) the cosine integral, pi up to the texel quadrature."""
    H, Wd = 64, 128
    e = np.zeros((H, Wd, 3), np.float32)
    i, j = 20, 40
    e[i, j] = (5.0, 2.0, 1.0)
    Ed, Es = O.env_prefilter(e)
    ls = grid_dirs(H, Wd)[i, j]
    dW = 2 * np.pi / Wd * (np.cos(np.pi * i / H) - np.cos(np.pi * (i + 1) / H))
    n = grid_dirs(O.PF_H, O.PF_W)
    c = np.clip(n @ ls, 0, None)
    want = c[..., None] * dW / np.pi * np.float64([5.0, 2.0, 1.0])
    np.testing.assert_allclose(Ed, want, rtol=2e-2, atol=1e-9)
    # linearity in the environment
    e2 = np.zeros_like(e); e2[50, 100] = (1.0, 1.0, 1.0)
    a, _ = O.env_prefilter(e2)
    b, _ = O.env_prefilter(e + 3 * e2)
    np.testing.assert_allclose(b, Ed + 3 * a, rtol=1e-10, atol=1e-14)


def _dfg_reference(mu, r):
    """A and B by scipy's adaptive quadrature over incident directions l
    (spherical coordinates about n), from the GGX / Smith / Schlick BRDF."""
    a2 = (r * r) ** 2
    v = np.array([np.sqrt(1 - mu * mu), 0.0, mu])
    G1 = lambda x: 2 * x / (x + np.sqrt(a2 + (1 - a2) * x * x))

    def f(ph, th, part):
        l = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        nl = l[2]
        h = l + v; h /= np.linalg.norm(h)
        D = a2 / (np.pi * (h[2] ** 2 * (a2 - 1) + 1) ** 2)
        fs = D * G1(nl) * G1(mu) / (4 * nl * mu)
        fc = (1 - max(h @ v, 0)) ** 5
        return fs * (1 - fc if part == 0 else fc) * nl * np.sin(th)
    out = []
    for part in (0, 1):
        val, _ = integrate.dblquad(f, 0, np.pi / 2, 0, 2 * np.pi, args=(part,), epsabs=1e-7, epsrel=1e-5)
        out.append(val)
    return out


@pytest.mark.parametrize("i,j", [(10, 15), (20, 20), (28, 25), (5, 31), (16, 12)])
def test_dfg_table_against_adaptive_quadrature(i, j):
    """Cells of moderate and high roughness, where an adaptive quadrature over
    incident directions converges: A and B to 2e-3 (the table's 256 x 256
    midpoint rule meets the horizon cut n.l > 0 within a node's width)."""
    lut = O.dfg_lut()
    mu, r = (i + 0.5) / O.LUT_N, (j + 0.5) / O.LUT_N
    A, B = _dfg_reference(mu, r)
    np.testing.assert_allclose(lut[i, j], [A, B], atol=2e-3)


def test_dfg_table_bounds():
    """0 <= A, B and A + B <= 1 (the specular lobe loses energy, never gains);
    near-mirror cells reflect everything."""
    lut = O.dfg_lut()
    assert (lut >= 0).all()
    assert (lut.sum(-1) <= 1 + 1e-9).all()
    assert lut[16:, 0].sum(-1).min() > 0.99


def test_relight_without_geometry_is_the_radiance_estimator():
    """With no surfels every secondary ray sees the environment (V = 1), so
    the relit image equals the radiance render under the same environment."""
    gb = W.gbuffer1(24, 24, seed=3)
    env = W.envmap(32, 64, seed=2)
    z = np.zeros
    s = W.Surfels(z((0, 3), np.float32), z((0, 2), np.float32), z((0, 4), np.float32), z(0, np.float32),
                  z((0, 3), np.float32))
    at = (z((0, 3), np.float32), z(0, np.float32), z(0, np.float32))
    a = O.render_relight(s, at, gb, env, (4, 2, 2), seed=9)
    b = O.render_mis(s, gb, env, (4, 2, 2), seed=9)
    np.testing.assert_array_equal(a, b)
    assert a.max() > 0


def test_relight_behind_an_opaque_wall():
    """Every secondary ray of a pixel under a stack of wide opaque layers sees
    no environment (V ~ 0): with a constant environment L0 and layers of
    albedo a, metallic 1 (no diffuse, F0 = a), L_i = L0 (a A + B) <= L0;
    with metallic 0 and albedo 0, L_i = L0 (0.04 A + B)."""
    L0 = 0.8
    env = np.full((32, 64, 3), L0, np.float32)
    n_layers = 12
    mus = np.array([[0.0, 0.0, 0.1 + 0.05 * k] for k in range(n_layers)], np.float32)
    s = W.Surfels(mus, np.full((n_layers, 2), 50.0, np.float32), np.tile(np.float32([1, 0, 0, 0]), (n_layers, 1)),
                  np.full(n_layers, 0.99, np.float32), np.zeros((n_layers, 3), np.float32))
    gb = W.GBuffer(1, 1, np.float32([[0, 0, 0]]), np.float32([[0, 0, 1]]), np.float32([[0, 0.6, 0.8]]),
                   np.float32([[0.5, 0.5, 0.5]]), np.float32([0.5]), np.float32([0.0]), np.uint8([1]))
    for metal, alb in ((1.0, 0.6), (0.0, 0.0)):
        at = (np.full((n_layers, 3), alb, np.float32), np.full(n_layers, 0.5, np.float32),
              np.full(n_layers, metal, np.float32))
        d = O.render_relight(s, at, gb, env, (8, 4, 4), seed=3, dump=True)
        lut = O.dfg_lut()
        tr = d["traced"][0].astype(bool)
        assert tr.sum() > 8
        Li = d["Li"][0][tr]
        F0 = 0.04 * (1 - metal) + metal * alb
        lo = L0 * (F0 * lut[..., 0] + lut[..., 1]).min()
        hi = L0 * (F0 * lut[..., 0] + lut[..., 1]).max()
        assert (Li >= lo - 1e-6).all() and (Li <= hi + 1e-6).all()
        assert (Li <= L0 + 1e-9).all()


# --------------------------------------------------------------------------
# SplitSum's table lookups, on tables of known content.  A direction table
# filled with a function that is bilinear in its texel coordinates
# (x = phi / 2pi * 32 - 1/2, v = theta / pi * 16 - 1/2, integers at texel
# centres) is reproduced exactly by bilinear interpolation between centres,
# at any direction away from the azimuth seam and the poles; likewise a DFG
# table bilinear in (mu * 32 - 1/2, r * 32 - 1/2).  So the relit radiance at
# any query has a closed form:
#   (1 - m) a Ed(n) + [(1 - t) Es_l(R) + t Es_{l+1}(R)] (F0 A(mu, r) + B(mu, r))
# with n the renormalized query normal, v = -w, R = 2 (n.v) n - v, mu = n.v,
# r * 5 = l + t, F0 = 0.04 (1 - m) + m a (reading of Eq. relight_splitsum);
# level 0 is the environment at R's nearest texel.
# --------------------------------------------------------------------------

def _tex_coords(w):
    th = np.arccos(np.clip(w[:, 1], -1, 1))
    ph = np.mod(np.arctan2(w[:, 2], w[:, 0]), 2 * np.pi)
    return ph / (2 * np.pi) * O.PF_W - 0.5, th / np.pi * O.PF_H - 0.5


def _bilinear_table(c):
    """[16, 32, 3] table with T[i, j] = c0 + c1 j + c2 i + c3 i j per channel."""
    i, j = np.meshgrid(np.arange(O.PF_H), np.arange(O.PF_W), indexing="ij")
    return np.stack([c[k, 0] + c[k, 1] * j + c[k, 2] * i + c[k, 3] * i * j for k in range(3)], -1)


def _eval_bilinear(c, x, v):
    return np.stack([c[k, 0] + c[k, 1] * x + c[k, 2] * v + c[k, 3] * x * v for k in range(3)], -1)


def _tables(g):
    cd = g.uniform(0.2, 1.0, (3, 4)) * np.float64([1, 0.05, 0.07, 0.01])
    cs = [g.uniform(0.2, 1.0, (3, 4)) * np.float64([1, 0.05, 0.07, 0.01]) + 3.0 * lv for lv in range(5)]
    Ed = _bilinear_table(cd)
    Es = np.stack([_bilinear_table(c) for c in cs])
    ca = np.float64([0.5, 0.011, -0.007, 0.0003])
    cb = np.float64([0.1, -0.002, 0.004, 0.0001])
    i, j = np.meshgrid(np.arange(O.LUT_N), np.arange(O.LUT_N), indexing="ij")
    lut = np.stack([ca[0] + ca[1] * i + ca[2] * j + ca[3] * i * j, cb[0] + cb[1] * i + cb[2] * j + cb[3] * i * j], -1)
    return cd, cs, Ed, Es, ca, cb, lut


def _interior_dirs(g, m):
    """Unit directions with theta in [0.2, pi - 0.2] and phi in [0.4, 2pi - 0.4]."""
    th = g.uniform(0.2, np.pi - 0.2, m)
    ph = g.uniform(0.4, 2 * np.pi - 0.4, m)
    return np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], -1)


def _queries(g, m):
    """Normals n and mirror directions R, both interior, with n.R in [0.1, 0.95];
    the ray direction is w = -v with v = 2 (n.R) n - R (so R mirrors v)."""
    ns, Rs = [], []
    while len(ns) < m:
        n = _interior_dirs(g, 1)[0]
        R = _interior_dirs(g, 1)[0]
        c = n @ R
        if 0.1 < c < 0.95:
            ns.append(n); Rs.append(R)
    n, R = np.array(ns), np.array(Rs)
    v = 2 * (n * R).sum(1, keepdims=True) * n - R
    return n, R, -v


@pytest.mark.parametrize("metal", [0.0, 1.0, 0.35])
def test_split_sum_lookups_closed_form(metal):
    """Diffuse (m = 0, a > 0), specular (m = 1) and mixed queries at rough-
    ness between the prefiltered levels: E_d is read at n (not R), E_s at R
    between the two levels around r, and the DFG terms at (n.v, r)."""
    g = np.random.default_rng(int(metal * 100) + 1)
    cd, cs, Ed, Es, ca, cb, lut = _tables(g)
    m = 64
    n, R, w = _queries(g, m)
    a = g.uniform(0.1, 1.0, (m, 3))
    r = g.uniform(0.21, 0.98, m)  # DFG cells span r in [1/64, 63/64]
    nsum = n * g.uniform(0.3, 2.0, (m, 1))  # the query's summed normal, renormalized inside
    env = np.ones((8, 16, 3), np.float32)
    got = O.split_sum(env, Ed, Es, lut, a, r, np.full(m, metal), nsum, w)
    xn, vn = _tex_coords(n)
    xr, vr = _tex_coords(R)
    Ld = _eval_bilinear(cd, xn, vn)
    lv = r * 5
    l0 = np.floor(lv).astype(int)
    t = (lv - l0)[:, None]
    Ls = np.stack([(1 - t[k]) * _eval_bilinear(cs[l0[k] - 1], xr[k:k + 1], vr[k:k + 1])[0] +
                   t[k] * _eval_bilinear(cs[l0[k]], xr[k:k + 1], vr[k:k + 1])[0] for k in range(m)])
    mu = (n * -w).sum(1)
    xi, yj = mu * O.LUT_N - 0.5, r * O.LUT_N - 0.5
    A = ca[0] + ca[1] * xi + ca[2] * yj + ca[3] * xi * yj
    B = cb[0] + cb[1] * xi + cb[2] * yj + cb[3] * xi * yj
    F0 = 0.04 * (1 - metal) + metal * a
    want = (1 - metal) * a * Ld + Ls * (F0 * A[:, None] + B[:, None])
    np.testing.assert_allclose(got, want, rtol=1e-10)


def test_split_sum_level_zero_reads_the_environment():
    """Below the first prefiltered roughness the specular lookup blends the
    environment itself at R's nearest texel with the first table."""
    g = np.random.default_rng(21)
    cd, cs, Ed, Es, ca, cb, lut = _tables(g)
    H, Wd = 8, 16
    env = g.uniform(0.5, 4.0, (H, Wd, 3)).astype(np.float32)
    m = 48
    n, R, w = _queries(g, m)
    a = g.uniform(0.1, 1.0, (m, 3))
    r = g.uniform(0.05, 0.19, m)
    got = O.split_sum(env, Ed, Es, lut, a, r, np.ones(m), n, w)
    th = np.arccos(np.clip(R[:, 1], -1, 1))
    ph = np.mod(np.arctan2(R[:, 2], R[:, 0]), 2 * np.pi)
    texel = env[np.minimum((th / np.pi * H).astype(int), H - 1), np.minimum((ph / (2 * np.pi) * Wd).astype(int), Wd - 1)]
    t = (r * 5)[:, None]
    xr, vr = _tex_coords(R)
    Ls = (1 - t) * texel + t * _eval_bilinear(cs[0], xr, vr)
    mu = (n * -w).sum(1)
    xi, yj = mu * O.LUT_N - 0.5, r * O.LUT_N - 0.5
    A = ca[0] + ca[1] * xi + ca[2] * yj + ca[3] * xi * yj
    B = cb[0] + cb[1] * xi + cb[2] * yj + cb[3] * xi * yj
    want = Ls * (a * A[:, None] + B[:, None])
    np.testing.assert_allclose(got, want, rtol=1e-10)
