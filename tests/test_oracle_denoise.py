"""Pins of the oracle's cross-bilateral denoiser (Sec. 3.4.2, "Denoising":
the bilateral weight B(p, p') and the normalized weighted average) against
special cases that reduce to library routines and closed forms."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import oracle as O


def flat(H, W, depth=2.0):
    n = np.tile([0.0, 0.0, 1.0], (H * W, 1))
    return np.full(H * W, depth), n, np.ones(H * W, np.uint8)


def test_constant_image_is_unchanged():
    H, W = 17, 23
    g = np.random.default_rng(0)
    D = g.uniform(1, 3, H * W); n = g.standard_normal((H * W, 3)); v = np.ones(H * W, np.uint8)
    c = np.tile([0.2, 0.5, 0.7], (H * W, 1))
    np.testing.assert_allclose(O.denoise(c, D, n, v, H, W), c, rtol=1e-13)


@pytest.mark.parametrize("radius,sigma_s", [(2, 1.0), (4, 2.5)])
def test_flat_plane_is_a_normalized_gaussian_blur(radius, sigma_s):
    """Equal depths and normals: B is the spatial Gaussian alone, so the
    output is the truncated Gaussian blur renormalized at the image border --
    scipy's convolution of the image and of the ones image, divided."""
    H, W = 31, 29
    g = np.random.default_rng(1)
    c = g.uniform(0, 1, (H * W, 3))
    D, n, v = flat(H, W)
    out = O.denoise(c, D, n, v, H, W, radius=radius, sigma_s=sigma_s)
    ax = np.arange(-radius, radius + 1)
    k = np.exp(-(ax[:, None] ** 2 + ax[None, :] ** 2) / (2 * sigma_s ** 2))
    img = c.reshape(H, W, 3)
    num = np.stack([ndimage.convolve(img[..., ch], k, mode="constant") for ch in range(3)], -1)
    den = ndimage.convolve(np.ones((H, W)), k, mode="constant")
    np.testing.assert_allclose(out.reshape(H, W, 3), num / den[..., None], rtol=1e-12)


def test_orthogonal_normals_do_not_mix():
    """Two halves with perpendicular normals: max(0, n.n')^sigma_n = 0 across
    the edge, so each half is blurred on its own (no leak)."""
    H, W = 12, 16
    g = np.random.default_rng(2)
    c = g.uniform(0, 1, (H * W, 3))
    D, n, v = flat(H, W)
    n = n.reshape(H, W, 3).copy(); n[:, W // 2:] = [1.0, 0.0, 0.0]
    out = O.denoise(c, D, n.reshape(-1, 3), v, H, W).reshape(H, W, 3)
    left = O.denoise(c.reshape(H, W, 3)[:, :W // 2].reshape(-1, 3), *flat(H, W // 2), H, W // 2).reshape(H, W // 2, 3)
    np.testing.assert_allclose(out[:, :W // 2], left, rtol=1e-12)


def test_depth_edge_is_preserved():
    """A large depth step on a plane of zero gradient: across the step
    exp(-|dD| / eps_d) underflows to 0, so the two sides do not mix."""
    H, W = 10, 14
    g = np.random.default_rng(3)
    c = g.uniform(0, 1, (H * W, 3))
    D, n, v = flat(H, W)
    D = D.reshape(H, W).copy(); D[:, W // 2:] = 50.0
    out = O.denoise(c, D.reshape(-1), n, v, H, W).reshape(H, W, 3)
    left = O.denoise(c.reshape(H, W, 3)[:, :W // 2].reshape(-1, 3), *flat(H, W // 2), H, W // 2).reshape(H, W // 2, 3)
    # the step makes the one-sided gradient large only in the two columns at the edge
    np.testing.assert_allclose(out[:, :W // 2 - 1], left[:, :W // 2 - 1], rtol=1e-9)


def test_single_pair_weight_closed_form():
    """A 1x2 image: out(0) = (c0 + B c1) / (1 + B) with B written out, for a
    depth gradient (one-sided) and tilted normals."""
    c = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.5]])
    D = np.array([2.0, 2.3])
    n = np.array([[0.0, 0.0, 1.0], [0.0, 0.6, 0.8]])
    v = np.ones(2, np.uint8)
    s_s, s_d, s_n, e_d = 1.5, 0.7, 8.0, 0.01
    out = O.denoise(c, D, n, v, 1, 2, radius=1, sigma_s=s_s, sigma_d=s_d, sigma_n=s_n, eps_d=e_d)
    g0 = D[1] - D[0]
    B = np.exp(-1 / (2 * s_s ** 2)) * np.exp(-abs(D[0] - D[1]) / (s_d * abs(g0 * 1) + e_d)) * 0.8 ** s_n
    np.testing.assert_allclose(out[0], (c[0] + B * c[1]) / (1 + B), rtol=1e-13)


def test_invalid_pixels_pass_through_and_never_contribute():
    H, W = 9, 9
    g = np.random.default_rng(4)
    c = g.uniform(0, 1, (H * W, 3))
    D, n, v = flat(H, W)
    v = v.copy(); v[40] = 0
    out = O.denoise(c, D, n, v, H, W)
    np.testing.assert_array_equal(out[40], c[40])
    c2 = c.copy(); c2[40] = 1e6  # an invalid pixel's colour must not leak
    out2 = O.denoise(c2, D, n, v, H, W)
    np.testing.assert_allclose(np.delete(out2, 40, 0), np.delete(out, 40, 0), rtol=1e-13)


def _brute(c, D, n, v, H, W, R, ss, sd, sn, ed):
    """Pixel by pixel, neighbour by neighbour, in plain Python."""
    c = c.reshape(H, W, 3); D = D.reshape(H, W); n = n.reshape(H, W, 3); v = v.reshape(H, W)
    nn = [[n[y, x] / np.linalg.norm(n[y, x]) for x in range(W)] for y in range(H)]

    def g(y, x, oy, ox):
        yp, xp, ym, xm = y + oy, x + ox, y - oy, x - ox
        hp = 0 <= yp < H and 0 <= xp < W and v[yp, xp]
        hm = 0 <= ym < H and 0 <= xm < W and v[ym, xm]
        if hp and hm:
            return (D[yp, xp] - D[ym, xm]) / 2
        if hp:
            return D[yp, xp] - D[y, x]
        if hm:
            return D[y, x] - D[ym, xm]
        return 0.0
    out = c.copy()
    for y in range(H):
        for x in range(W):
            if not v[y, x]:
                continue
            gx, gy = g(y, x, 0, 1), g(y, x, 1, 0)
            num = np.zeros(3); den = 0.0
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    qy, qx = y + dy, x + dx
                    if not (0 <= qy < H and 0 <= qx < W and v[qy, qx]):
                        continue
                    B = (np.exp(-(dx * dx + dy * dy) / (2 * ss * ss))
                         * np.exp(-abs(D[y, x] - D[qy, qx]) / (sd * abs(gx * dx + gy * dy) + ed))
                         * max(0.0, float(nn[y][x] @ nn[qy][qx])) ** sn)
                    num += B * c[qy, qx]; den += B
            out[y, x] = num / den
    return out.reshape(H * W, 3)


@pytest.mark.parametrize("H,W,R", [(2, 9, 3), (5, 4, 8), (1, 1, 2), (7, 6, 2)])
def test_brute_force_on_tiny_images(H, W, R):
    """Against a per-pixel loop, including windows larger than the image."""
    g = np.random.default_rng(H * 100 + W)
    c = g.uniform(0, 1, (H * W, 3)); D = g.uniform(1, 2, H * W)
    n = g.standard_normal((H * W, 3)); n[:, 2] = np.abs(n[:, 2]) + 1.0
    v = (g.uniform(0, 1, H * W) < 0.85).astype(np.uint8); v[0] = 1
    kw = dict(radius=R, sigma_s=1.3, sigma_d=0.9, sigma_n=4.0, eps_d=0.05)
    got = O.denoise(c, D, n, v, H, W, **kw)
    want = _brute(c, D, n, v, H, W, R, 1.3, 0.9, 4.0, 0.05)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)
