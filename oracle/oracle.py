"""Python face of the CPU oracle (``liboracle.so``, plain C, OpenMP).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline leg import this module.  It never touches the GPU library and the
GPU library never touches it.

Every function takes numpy arrays (the seeded inputs) and returns numpy
arrays in double precision.  See ``oracle.c`` for the equations each part
follows and for the fixed single-precision decision order.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

P = C.c_void_p
I64 = C.c_int64
F = C.c_float


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            import importlib.util
            spec = importlib.util.spec_from_file_location("oracle_build", os.path.join(HERE, "build.py"))
            m = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(m)
            m.build()
        L = C.CDLL(path)
        L.orc_trace.restype = C.c_int
        L.orc_trace.argtypes = [I64, P, P, P, P, P, F, I64, P, P, P, P, F, F, F, P, P, P, P, P, I64, P, P, P]
        L.orc_trace_backward.restype = C.c_int
        L.orc_trace_backward.argtypes = [I64, P, P, P, P, P, F, I64, P, P, P, P, F, F, F, P, P, P, P]
        L.orc_env_cdf.restype = C.c_int
        L.orc_env_cdf.argtypes = [C.c_int, C.c_int, P, P, P]
        L.orc_philox.restype = None
        L.orc_philox.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, P]
        L.orc_render_mis.restype = C.c_int
        L.orc_render_mis.argtypes = ([I64, P, P, P, P, P, F] + [P] * 7 + [C.c_int, C.c_int, P, P, P] +
                                     [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32, F, F, I64, P, P] + [P] * 6)
        L.orc_render_mis_backward.restype = C.c_int
        L.orc_render_mis_backward.argtypes = ([I64, P, P, P, P, P, F] + [P] * 7 + [C.c_int, C.c_int, P, P, P] +
                                              [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32, F, F, I64, P, P, P, P, P,
                                               P])
        L.orc_env_prefilter.restype = C.c_int
        L.orc_env_prefilter.argtypes = [C.c_int, C.c_int, P, P, P]
        L.orc_dfg_lut.restype = C.c_int
        L.orc_dfg_lut.argtypes = [P]
        L.orc_render_relight.restype = C.c_int
        L.orc_render_relight.argtypes = ([I64, P, P, P, P, F, P, P, P] + [P] * 7 + [C.c_int, C.c_int, P, P, P] +
                                         [P, P, P] +
                                         [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32, F, F, I64, P, P] +
                                         [P] * 6)
        L.orc_mesh_trace_attr.restype = C.c_int
        L.orc_mesh_trace_attr.argtypes = [I64, P, I64, P, P, P, P, P, I64, P, P, F, F, P, P, P, P, P, P]
        L.orc_render_relight_mesh.restype = C.c_int
        L.orc_render_relight_mesh.argtypes = ([I64, P, I64, P, P, P, P, P] + [P] * 7 + [C.c_int, C.c_int, P, P, P] +
                                              [P, P, P] + [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32, F,
                                                           I64, P, P] + [P] * 6)
        L.orc_trace_gbuffer.restype = C.c_int
        L.orc_trace_gbuffer.argtypes = ([I64, P, P, P, P, P, F, P, P, P, I64, P, P, F, F, F, C.c_double] + [P] * 9)
        L.orc_trace_gbuffer_backward.restype = C.c_int
        L.orc_trace_gbuffer_backward.argtypes = ([I64, P, P, P, P, P, F, P, P, P, I64, P, P, F, F, F, C.c_double]
                                                 + [P] * 11)
        L.orc_trace_attr.restype = C.c_int
        L.orc_trace_attr.argtypes = [I64, P, P, P, P, F, P, P, P, I64, P, P, F, F, F, P, P, P, P, P]
        if hasattr(L, "orc_count_work"):
            L.orc_count_work.restype = C.c_int
            L.orc_count_work.argtypes = [I64, P, P, P, P, P, F, F, I64, P, P, F, F, F, P, P, P]
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt=np.float32):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


def _scene(s):
    return [_c(s.means), _c(s.scales), _c(s.quats), _c(s.opacity), _c(s.rgb)]


ALPHA_MIN = 1.0 / 255.0
T_CUT = 1e-3

# padding of the surfel bounding boxes used for the work counts (scene units)
AABB_PAD = 1e-5


def trace(s, origins, dirs, t_min=0.0, t_max=np.inf, t_cut=T_CUT, alpha_min=ALPHA_MIN, sky=(0.5, 0.5, 0.5),
          cap=0):
    """Brute-force Trace(r_o, r_d) for every ray.

    Returns dict: C [R,3] (c_rt), T [R] (1 - o_rt), L [R,3] = C + T sky,
    nhit [R] composited hits, margins [R,5] (support margin in radians of
    ray direction, grazing margin, depth margin, relative cutoff margin,
    environment texel margin), and with ``cap`` > 0 the
    composited ids/depths ``ids``/``tau`` [R,cap] (-1 padded).
    """
    arrs = _scene(s)
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    tmin_a = _c(t_min) if np.ndim(t_min) else None
    tmax_a = _c(t_max) if np.ndim(t_max) else None
    sky_a = _c(sky)
    out = dict(C=np.zeros((R, 3)), T=np.zeros(R), L=np.zeros((R, 3)), nhit=np.zeros(R, np.int32),
               margins=np.zeros((R, 5), np.float32))
    ids = np.zeros((R, max(cap, 1)), np.int32) if cap else None
    tau = np.zeros((R, max(cap, 1)), np.float32) if cap else None
    rc = lib().orc_trace(s.n, *map(_p, arrs), alpha_min, R, _p(o), _p(d), _p(tmin_a), _p(tmax_a),
                         float(0.0 if tmin_a is not None else t_min), float(np.inf if tmax_a is not None else t_max),
                         t_cut, _p(sky_a), _p(out["C"]), _p(out["T"]), _p(out["L"]), _p(out["nhit"]),
                         cap, _p(ids), _p(tau), _p(out["margins"]))
    assert rc == 0
    if cap:
        out["ids"] = ids; out["tau"] = tau
    return out


def trace_env(s, origins, dirs, env_rgb, t_min=0.0, t_max=np.inf, t_cut=T_CUT, alpha_min=ALPHA_MIN):
    """L [R,3] = c_rt + T_fin L_env(d) of every ray under an environment map
    (nearest texel of the ray direction) instead of a constant sky."""
    L = lib()
    L.orc_trace_env.restype = C.c_int
    L.orc_trace_env.argtypes = [I64, P, P, P, P, P, F, I64, P, P, F, F, F, C.c_int, C.c_int, P, P]
    arrs = _scene(s)
    o = _c(origins); d = _c(dirs); e = _c(env_rgb)
    R = o.shape[0]
    out = np.zeros((R, 3))
    rc = L.orc_trace_env(s.n, *map(_p, arrs), alpha_min, R, _p(o), _p(d), float(t_min), float(t_max), t_cut,
                         e.shape[0], e.shape[1], _p(e), _p(out))
    assert rc == 0
    return out


def trace_attr(s, attrs, origins, dirs, t_min=0.0, t_max=np.inf, t_cut=T_CUT, alpha_min=ALPHA_MIN):
    """Brute-force attribute query Trace_attr(x, w) for every ray (the
    Gaussian backend): attrs = (albedo [n,3], rough [n], metal [n]).

    Returns dict: V [R] (final transmittance), albedo [R,3], rough [R],
    metal [R], normal [R,3]: normalized-blending-weight averages over the
    composited hits (normals facing the ray origin; all 0 when nothing is hit).
    """
    means, scales, quats, opacity, _ = _scene(s)
    alb, rough, metal = (_c(a) for a in attrs)
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    out = dict(V=np.zeros(R), albedo=np.zeros((R, 3)), rough=np.zeros(R), metal=np.zeros(R), normal=np.zeros((R, 3)))
    rc = lib().orc_trace_attr(s.n, _p(means), _p(scales), _p(quats), _p(opacity), alpha_min, _p(alb), _p(rough),
                              _p(metal), R, _p(o), _p(d), float(t_min), float(t_max), t_cut, _p(out["V"]),
                              _p(out["albedo"]), _p(out["rough"]), _p(out["metal"]), _p(out["normal"]))
    assert rc == 0
    return out


def mesh_trace_attr(m, origins, dirs, t_min=0.0, t_max=np.inf):
    """Mesh backend of Trace_attr: closest-hit V [R], albedo [R,3], rough,
    metal [R], normal [R,3] (barycentric, facing the origin) and margins
    [R,2] (barycentric margin, relative t gap to the next triangle)."""
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    out = dict(V=np.zeros(R), albedo=np.zeros((R, 3)), rough=np.zeros(R), metal=np.zeros(R), normal=np.zeros((R, 3)),
               margins=np.zeros((R, 2)))
    tris = _c(m.tris, np.int32)
    rc = lib().orc_mesh_trace_attr(m.nv, _p(_c(m.verts)), m.nf, _p(tris), _p(_c(m.albedo)), _p(_c(m.rough)),
                                   _p(_c(m.metal)), _p(_c(m.normal)), R, _p(o), _p(d), float(t_min), float(t_max),
                                   *(_p(out[k]) for k in ("V", "albedo", "rough", "metal", "normal", "margins")))
    assert rc == 0
    return out


def trace_gbuffer(s, attrs, origins, dirs, t_min=0.0, t_max=np.inf, t_cut=T_CUT, alpha_min=ALPHA_MIN,
                  min_opacity=0.5):
    """Primary-ray G-buffer by 2DGRT (Eq. deferred_maps on traced primary
    rays): dict of x, n, wo, albedo [R,3], rough, metal, depth [R], rgb [R,3]
    and valid [R] (uint8: accumulated opacity >= min_opacity)."""
    arrs = _scene(s)
    alb, rough, metal = (_c(a) for a in attrs)
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    out = dict(x=np.zeros((R, 3)), n=np.zeros((R, 3)), wo=np.zeros((R, 3)), albedo=np.zeros((R, 3)),
               rough=np.zeros(R), metal=np.zeros(R), depth=np.zeros(R), rgb=np.zeros((R, 3)),
               valid=np.zeros(R, np.uint8))
    rc = lib().orc_trace_gbuffer(s.n, *map(_p, arrs), alpha_min, _p(alb), _p(rough), _p(metal), R, _p(o), _p(d),
                                 float(t_min), float(t_max), t_cut, float(min_opacity),
                                 *(_p(out[k]) for k in ("x", "n", "wo", "albedo", "rough", "metal", "depth", "rgb",
                                                        "valid")))
    assert rc == 0
    return out


GBUF_GRAD_KEYS = ("x", "n", "albedo", "rough", "metal", "depth", "rgb")


def trace_gbuffer_backward(s, attrs, origins, dirs, grads, t_min=0.0, t_max=np.inf, t_cut=T_CUT,
                           alpha_min=ALPHA_MIN, min_opacity=0.5, with_abs=False):
    """d/d(surfels, attributes) of the sum over covered pixels of
    grads[k] . map_k for the maps of trace_gbuffer (keys x, n, albedo, rough,
    metal, depth, rgb; missing keys are zero).  Returns (g13 [N,13] as
    trace_backward, gattr [N,5] = albedo 3, roughness, metallic); with
    ``with_abs`` also each element's error scale (g13_abs, gattr_abs): the
    magnitudes of its per-hit terms plus the chain rule applied to the
    magnitudes of what each hit's dL/dalpha sums (see orc_trace_gbuffer_backward)."""
    arrs = _scene(s)
    alb, rough, metal = (_c(a) for a in attrs)
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    shape = dict(x=(R, 3), n=(R, 3), albedo=(R, 3), rgb=(R, 3), rough=(R,), metal=(R,), depth=(R,))
    gp = {k: (_c(grads[k], np.float64).reshape(shape[k]) if grads.get(k) is not None else None)
          for k in GBUF_GRAD_KEYS}
    g13 = np.zeros((s.n, 13)); ga = np.zeros((s.n, 5))
    g13a = np.zeros((s.n, 13)) if with_abs else None
    gaa = np.zeros((s.n, 5)) if with_abs else None
    rc = lib().orc_trace_gbuffer_backward(s.n, *map(_p, arrs), alpha_min, _p(alb), _p(rough), _p(metal), R, _p(o),
                                          _p(d), float(t_min), float(t_max), t_cut, float(min_opacity),
                                          *(_p(gp[k]) for k in ("x", "n", "albedo", "rough", "metal", "depth",
                                                                "rgb")), _p(g13), _p(ga), _p(g13a), _p(gaa))
    assert rc == 0
    return (g13, ga, g13a, gaa) if with_abs else (g13, ga)


def trace_backward(s, origins, dirs, gC, gT, t_min=0.0, t_max=np.inf, t_cut=T_CUT, alpha_min=ALPHA_MIN,
                   with_abs=False):
    """d/d(surfels) of sum_r gC_r . c_rt + gT_r T_fin; returns [N,13] double
    (mean 3, scale 2, quat 4, opacity 1, rgb 3); with ``with_abs`` also each
    element's error scale: the magnitudes of its per-hit terms plus the chain
    rule applied to the magnitudes of what each hit's dL/dalpha sums."""
    arrs = _scene(s)
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    tmin_a = _c(t_min) if np.ndim(t_min) else None
    tmax_a = _c(t_max) if np.ndim(t_max) else None
    gC = _c(gC, np.float64).reshape(R, 3); gT = _c(gT, np.float64).reshape(R)
    g = np.zeros((s.n, 13))
    ga = np.zeros((s.n, 13)) if with_abs else None
    rc = lib().orc_trace_backward(s.n, *map(_p, arrs), alpha_min, R, _p(o), _p(d), _p(tmin_a), _p(tmax_a),
                                  float(0.0 if tmin_a is not None else t_min),
                                  float(np.inf if tmax_a is not None else t_max), t_cut, _p(gC), _p(gT), _p(g),
                                  _p(ga))
    assert rc == 0
    return (g, ga) if with_abs else g


def env_cdf(env_rgb):
    """Marginal [H+1] and conditional [H,W+1] float32 tables of an [H,W,3] map."""
    e = _c(env_rgb)
    H, W = e.shape[:2]
    marg = np.zeros(H + 1, np.float32)
    cond = np.zeros((H, W + 1), np.float32)
    lib().orc_env_cdf(H, W, _p(e), _p(marg), _p(cond))
    return marg, cond


def philox(seed, c0, c1, c2, c3):
    out = np.zeros(4, np.uint32)
    lib().orc_philox(seed, c0, c1, c2, c3, _p(out))
    return out


def _gb(gb):
    return [_c(gb.x), _c(gb.n), _c(gb.wo), _c(gb.albedo), _c(gb.rough), _c(gb.metal), _c(gb.valid, np.uint8)]


def render_mis(s, gb, env_rgb, split, seed, pix=None, job=0, t_min=1e-3, t_cut=T_CUT, alpha_min=ALPHA_MIN,
               dump=False):
    """c_pbr of the G-buffer pixels ``pix`` (default all).  With ``dump``,
    also per-sample dir/q/wt/Li/traced/margins."""
    nc, ng, ne = split
    spp = nc + ng + ne
    arrs = _scene(s)
    g = _gb(gb)
    e = _c(env_rgb)
    marg, cond = env_cdf(e)
    pix = np.arange(gb.npix, dtype=np.int64) if pix is None else _c(pix, np.int64)
    npx = len(pix)
    out = np.zeros((npx, 3))
    d = {}
    if dump:
        d = dict(dir=np.zeros((npx, spp, 3), np.float32), q=np.zeros((npx, spp)), wt=np.zeros((npx, spp, 3)),
                 Li=np.zeros((npx, spp, 3)), traced=np.zeros((npx, spp), np.uint8),
                 margins=np.zeros((npx, spp, 5), np.float32))
    rc = lib().orc_render_mis(s.n, *map(_p, arrs), alpha_min, *map(_p, g), e.shape[0], e.shape[1], _p(e), _p(marg),
                              _p(cond), nc, ng, ne, seed, job, t_min, t_cut, npx, _p(pix), _p(out),
                              _p(d.get("dir")), _p(d.get("q")), _p(d.get("wt")), _p(d.get("Li")),
                              _p(d.get("traced")), _p(d.get("margins")))
    assert rc == 0
    if dump:
        d["rgb"] = out
        return d
    return out


PF_H, PF_W, PF_L, LUT_N = 16, 32, 6, 32


def env_prefilter(env_rgb):
    """The prefiltered representation E of an environment (Eq.
    relight_splitsum): diffuse Ed [16,32,3] and specular Es [5,16,32,3] at
    roughness 0.2, 0.4, ..., 1.0 (level 0 is the environment itself)."""
    e = _c(env_rgb)
    Ed = np.zeros((PF_H, PF_W, 3)); Es = np.zeros((PF_L - 1, PF_H, PF_W, 3))
    assert lib().orc_env_prefilter(e.shape[0], e.shape[1], _p(e), _p(Ed), _p(Es)) == 0
    return Ed, Es


def dfg_lut():
    """The split-sum DFG table [32 (n.v), 32 (roughness), 2 (A, B)] at cell centres."""
    lut = np.zeros((LUT_N, LUT_N, 2))
    assert lib().orc_dfg_lut(_p(lut)) == 0
    return lut


def render_relight(s, attrs, gb, env_rgb, split, seed, pix=None, job=0, t_min=1e-3, t_cut=T_CUT,
                   alpha_min=ALPHA_MIN, dump=False, tables=None):
    """Relit c_pbr of the G-buffer pixels ``pix`` under env_rgb (Sec. 3.5.1):
    the MIS estimator with L_i = V L_env + (1 - V) SplitSum(attributes the
    query returns, prefiltered env).  attrs = (albedo [n,3], rough [n], metal
    [n]); ``tables`` = (Ed, Es, lut) to reuse, else computed here."""
    nc, ng, ne = split
    spp = nc + ng + ne
    means, scales, quats, opacity, _ = _scene(s)
    alb, rough, metal = (_c(a) for a in attrs)
    g = _gb(gb)
    e = _c(env_rgb)
    marg, cond = env_cdf(e)
    if tables is None:
        Ed, Es = env_prefilter(e)
        lut = dfg_lut()
    else:
        Ed, Es, lut = (np.ascontiguousarray(a, np.float64) for a in tables)
    pix = np.arange(gb.npix, dtype=np.int64) if pix is None else _c(pix, np.int64)
    npx = len(pix)
    out = np.zeros((npx, 3))
    d = {}
    if dump:
        d = dict(dir=np.zeros((npx, spp, 3), np.float32), q=np.zeros((npx, spp)), wt=np.zeros((npx, spp, 3)),
                 Li=np.zeros((npx, spp, 3)), traced=np.zeros((npx, spp), np.uint8),
                 margins=np.zeros((npx, spp, 5), np.float32))
    rc = lib().orc_render_relight(s.n, _p(means), _p(scales), _p(quats), _p(opacity), alpha_min, _p(alb), _p(rough),
                                  _p(metal), *map(_p, g), e.shape[0], e.shape[1], _p(e), _p(marg), _p(cond),
                                  _p(Ed), _p(Es), _p(lut), nc, ng, ne, seed, job, t_min, t_cut, npx, _p(pix),
                                  _p(out), _p(d.get("dir")), _p(d.get("q")), _p(d.get("wt")), _p(d.get("Li")),
                                  _p(d.get("traced")), _p(d.get("margins")))
    assert rc == 0
    if dump:
        d["rgb"] = out
        return d
    return out


def denoise(rgb, depth, normal, valid, H, W, radius=3, sigma_s=2.0, sigma_d=1.0, sigma_n=128.0, eps_d=1e-2):
    """Cross-bilateral denoiser (Sec. 3.4.2, "Denoising"), written out in
    double: for each valid pixel p, over the valid pixels p' of the
    (2 radius + 1)^2 window around it (inside the image),
        B = exp(-|p - p'|^2 / (2 sigma_s^2))
            * exp(-|D(p) - D(p')| / (sigma_d |grad D(p) . (p - p')| + eps_d))
            * max(0, N(p) . N(p'))^sigma_n,
        out(p) = sum B c(p') / sum B,
    with N normalized per pixel and grad D(p) the screen-space depth gradient
    by central differences (one-sided where a neighbour is outside the image
    or invalid, 0 where both are).  Invalid pixels pass through unchanged.
    rgb [H*W,3], depth [H*W], normal [H*W,3], valid [H*W]; returns [H*W,3]."""
    c = np.asarray(rgb, np.float64).reshape(H, W, 3)
    D = np.asarray(depth, np.float64).reshape(H, W)
    n = np.asarray(normal, np.float64).reshape(H, W, 3)
    v = np.asarray(valid).reshape(H, W).astype(bool)
    ln = np.linalg.norm(n, axis=-1, keepdims=True)
    n = np.where(ln > 0, n / np.where(ln > 0, ln, 1.0), 0.0)

    def grad(axis):
        g = np.zeros((H, W))
        Dp = np.full((H, W), np.nan); Dm = np.full((H, W), np.nan)
        if axis == 1:
            Dp[:, :-1] = np.where(v[:, 1:], D[:, 1:], np.nan)
            Dm[:, 1:] = np.where(v[:, :-1], D[:, :-1], np.nan)
        else:
            Dp[:-1, :] = np.where(v[1:, :], D[1:, :], np.nan)
            Dm[1:, :] = np.where(v[:-1, :], D[:-1, :], np.nan)
        hp, hm = ~np.isnan(Dp), ~np.isnan(Dm)
        both = hp & hm
        g[both] = (Dp[both] - Dm[both]) / 2.0
        only_p = hp & ~hm
        g[only_p] = Dp[only_p] - D[only_p]
        only_m = hm & ~hp
        g[only_m] = D[only_m] - Dm[only_m]
        return g
    gx, gy = grad(1), grad(0)
    num = np.zeros((H, W, 3)); den = np.zeros((H, W))
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            # neighbour q = p + (dx, dy): shifted arrays, zero weight outside
            if abs(dy) >= H or abs(dx) >= W:
                continue  # every neighbour at this offset lies outside the image
            ys = slice(max(0, -dy), H - max(0, dy)); xs = slice(max(0, -dx), W - max(0, dx))
            yq = slice(max(0, dy), H - max(0, -dy)); xq = slice(max(0, dx), W - max(0, -dx))
            ok = v[ys, xs] & v[yq, xq]
            ws = np.exp(-(dx * dx + dy * dy) / (2.0 * sigma_s ** 2))
            wd = np.exp(-np.abs(D[ys, xs] - D[yq, xq]) / (sigma_d * np.abs(gx[ys, xs] * dx + gy[ys, xs] * dy) + eps_d))
            wn = np.maximum(0.0, np.einsum("ijk,ijk->ij", n[ys, xs], n[yq, xq])) ** sigma_n
            B = np.where(ok, ws * wd * wn, 0.0)
            num[ys, xs] += B[..., None] * c[yq, xq]
            den[ys, xs] += B
    out = np.where(v[..., None], num / np.where(den > 0, den, 1.0)[..., None], c)
    return out.reshape(H * W, 3)


def render_relight_mesh(m, gb, env_rgb, split, seed, pix=None, job=0, t_min=1e-3, dump=False, tables=None):
    """Relit c_pbr with the mesh backend answering the attribute query
    (mesh m with per-vertex attributes; otherwise as render_relight).  With
    ``dump`` the margins carry the mesh query's barycentric margin [..., 0]
    and depth gap [..., 1]."""
    nc, ng, ne = split
    spp = nc + ng + ne
    g = _gb(gb)
    e = _c(env_rgb)
    marg, cond = env_cdf(e)
    if tables is None:
        Ed, Es = env_prefilter(e)
        lut = dfg_lut()
    else:
        Ed, Es, lut = (np.ascontiguousarray(a, np.float64) for a in tables)
    pix = np.arange(gb.npix, dtype=np.int64) if pix is None else _c(pix, np.int64)
    npx = len(pix)
    out = np.zeros((npx, 3))
    d = {}
    if dump:
        d = dict(dir=np.zeros((npx, spp, 3), np.float32), q=np.zeros((npx, spp)), wt=np.zeros((npx, spp, 3)),
                 Li=np.zeros((npx, spp, 3)), traced=np.zeros((npx, spp), np.uint8),
                 margins=np.zeros((npx, spp, 5), np.float32))
    tris = _c(m.tris, np.int32)
    rc = lib().orc_render_relight_mesh(m.nv, _p(_c(m.verts)), m.nf, _p(tris), _p(_c(m.albedo)), _p(_c(m.rough)),
                                       _p(_c(m.metal)), _p(_c(m.normal)), *map(_p, g), e.shape[0], e.shape[1], _p(e),
                                       _p(marg), _p(cond), _p(Ed), _p(Es), _p(lut), nc, ng, ne, seed, job, t_min, npx,
                                       _p(pix), _p(out), _p(d.get("dir")), _p(d.get("q")), _p(d.get("wt")),
                                       _p(d.get("Li")), _p(d.get("traced")), _p(d.get("margins")))
    assert rc == 0
    if dump:
        d["rgb"] = out
        return d
    return out


def render_mis_backward(s, gb, env_rgb, split, seed, grad, pix=None, job=0, t_min=1e-3, t_cut=T_CUT,
                        alpha_min=ALPHA_MIN, with_abs=False, shading=False):
    """d/d(surfels) of sum_k grad[k] . c_pbr(pix[k]); returns [N,13] double
    (with ``with_abs`` also each element's error scale, as trace_backward).
    With ``shading`` also d/d(shading state) of the listed pixels, with every
    sample's direction and pdf held fixed: [len(pix), 14] = x 3, n 3, wo 3
    (the stored, unnormalised vectors), albedo 3, roughness, metallic;
    returned last (with ``with_abs`` followed by its error scales, the same
    shape: the terms' magnitudes, and for x the mean terms' error scales)."""
    nc, ng, ne = split
    arrs = _scene(s)
    g = _gb(gb)
    e = _c(env_rgb)
    marg, cond = env_cdf(e)
    pix = np.arange(gb.npix, dtype=np.int64) if pix is None else _c(pix, np.int64)
    grad = _c(grad, np.float64).reshape(len(pix), 3)
    out = np.zeros((s.n, 13))
    oabs = np.zeros((s.n, 13)) if with_abs else None
    shade = np.zeros((len(pix), 14)) if shading else None
    sabs = np.zeros((len(pix), 14)) if shading and with_abs else None
    rc = lib().orc_render_mis_backward(s.n, *map(_p, arrs), alpha_min, *map(_p, g), e.shape[0], e.shape[1], _p(e),
                                       _p(marg), _p(cond), nc, ng, ne, seed, job, t_min, t_cut, len(pix), _p(pix),
                                       _p(grad), _p(out), _p(oabs), _p(shade), _p(sabs))
    assert rc == 0
    res = (out,) + ((oabs,) if with_abs else ()) + ((shade,) if shading else ()) + \
        ((sabs,) if sabs is not None else ())
    return res if len(res) > 1 else out


def split_grads(g13):
    """[N,13] -> dict of per-parameter gradient blocks."""
    return dict(means=g13[:, 0:3], scales=g13[:, 3:5], quats=g13[:, 5:9], opacity=g13[:, 9], rgb=g13[:, 10:13])


def count_work(s, origins, dirs, t_min=0.0, t_max=np.inf, t_cut=T_CUT, alpha_min=ALPHA_MIN, pad=AABB_PAD):
    """Per-ray (N_cand, N_node, N_hit) on the reference LBVH (see workcount.c)."""
    arrs = _scene(s)
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    nc = np.zeros(R, np.int64); nn = np.zeros(R, np.int64); nh = np.zeros(R, np.int64)
    rc = lib().orc_count_work(s.n, *map(_p, arrs), alpha_min, pad, R, _p(o), _p(d), float(t_min), float(t_max),
                              t_cut, _p(nc), _p(nn), _p(nh))
    assert rc == 0
    return nc, nn, nh


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _env_args(env_rgb):
    if env_rgb is None:
        return 0, 0, None, None, None
    e = _c(env_rgb)
    marg, cond = env_cdf(e)
    return e.shape[0], e.shape[1], e, marg, cond


def sample_dirs(tech, n, wo, rough, u, env_rgb=None):
    """Directions from technique 0 (cosine), 1 (GGX visible normals), 2 (env) for uniforms u [m,2]."""
    L = lib()
    L.orc_sample_dirs.restype = None
    L.orc_sample_dirs.argtypes = [C.c_int, P, P, C.c_double, C.c_int, C.c_int, P, P, P, I64, P, P]
    eH, eW, e, marg, cond = _env_args(env_rgb)
    u = _d(u).reshape(-1, 2)
    w = np.zeros((len(u), 3))
    L.orc_sample_dirs(tech, _p(_d(n)), _p(_d(wo)), rough, eH, eW, _p(e), _p(marg), _p(cond), len(u), _p(u), _p(w))
    return w


def pdfs(n, wo, rough, w, env_rgb=None, split=(1, 1, 1)):
    """(p_c, p_g, p_e) [m,3] and the mixture q [m] at directions w [m,3]."""
    L = lib()
    L.orc_pdfs.restype = None
    L.orc_pdfs.argtypes = [P, P, C.c_double, C.c_int, C.c_int, P, P, P, C.c_int, C.c_int, C.c_int, I64, P, P, P]
    eH, eW, e, marg, cond = _env_args(env_rgb)
    w = _d(w).reshape(-1, 3)
    p3 = np.zeros((len(w), 3)); q = np.zeros(len(w))
    if eH == 0:
        split = (split[0], split[1], 0)
    L.orc_pdfs(_p(_d(n)), _p(_d(wo)), rough, eH, eW, _p(e), _p(marg), _p(cond), split[0], split[1], split[2],
               len(w), _p(w), _p(p3), _p(q))
    return p3, q


def brdf(n, wo, albedo, rough, metal, wi):
    L = lib()
    L.orc_brdf.restype = None
    L.orc_brdf.argtypes = [P, P, P, C.c_double, C.c_double, I64, P, P]
    wi = _d(wi).reshape(-1, 3)
    f = np.zeros((len(wi), 3))
    L.orc_brdf(_p(_d(n)), _p(_d(wo)), _p(_d(albedo)), rough, metal, len(wi), _p(wi), _p(f))
    return f


def env_lookup(env_rgb, w):
    L = lib()
    L.orc_env_lookup.restype = None
    L.orc_env_lookup.argtypes = [C.c_int, C.c_int, P, I64, P, P]
    e = _c(env_rgb)
    w = _d(w).reshape(-1, 3)
    out = np.zeros((len(w), 3))
    L.orc_env_lookup(e.shape[0], e.shape[1], _p(e), len(w), _p(w), _p(out))
    return out


def trace_extent(s, origins, dirs, t_min=0.0, t_max=np.inf, t_cut=T_CUT, alpha_min=ALPHA_MIN):
    """Per ray: the depth where compositing ended (the last composited hit's
    depth if the ray was cut off, else t_max) and the composited hit count,
    the segment the work counter prices."""
    L = lib()
    L.orc_trace_extent.restype = C.c_int
    L.orc_trace_extent.argtypes = [I64, P, P, P, P, F, I64, P, P, F, F, F, P, P]
    means, scales, quats, opacity, _ = _scene(s)
    o = _c(origins); d = _c(dirs)
    R = o.shape[0]
    t_term = np.zeros(R, np.float32); nhit = np.zeros(R, np.int64)
    rc = L.orc_trace_extent(s.n, _p(means), _p(scales), _p(quats), _p(opacity), alpha_min, R, _p(o), _p(d),
                            float(t_min), float(t_max), t_cut, _p(t_term), _p(nhit))
    assert rc == 0
    return t_term, nhit


def split_sum(env_rgb, Ed, Es, lut, albedo, rough, metal, nsum, w):
    """SplitSum of Eq. relight_splitsum for query results (albedo [m,3],
    rough [m], metal [m], summed normal nsum [m,3]) of secondary rays w [m,3],
    with the given tables Ed [16,32,3], Es [5,16,32,3], lut [32,32,2] and the
    environment env_rgb [H,W,3] (level 0 of the specular lookup)."""
    L = lib()
    L.orc_split_sum.restype = None
    L.orc_split_sum.argtypes = [C.c_int, C.c_int, P, P, P, P, I64, P, P, P, P, P, P]
    e = _c(env_rgb)
    albedo = _d(albedo).reshape(-1, 3)
    m = len(albedo)
    out = np.zeros((m, 3))
    L.orc_split_sum(e.shape[0], e.shape[1], _p(e), _p(_d(Ed)), _p(_d(Es)), _p(_d(lut)), m, _p(albedo),
                    _p(_d(rough).reshape(m)), _p(_d(metal).reshape(m)), _p(_d(nsum).reshape(m, 3)),
                    _p(_d(w).reshape(m, 3)), _p(out))
    return out
