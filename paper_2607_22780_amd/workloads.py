"""Seeded synthetic inputs for 2D Gaussian ray tracing workloads.

This module only *draws inputs*: surfel parameters, rays, G-buffers (primary
hits of a pinhole camera on analytic shapes), environment maps, loss targets
and request streams.  It holds none of the method's arithmetic (no ray-surfel
intersection, compositing, sampling or shading), so both the CPU oracle's
tests and the GPU path can take their inputs from here.

Every array is drawn from numpy's PCG64 seeded with ``[config_id, stream_id]``
and returned as contiguous float32 (uint8 for masks).  The recipes follow the
five synthetic workloads the path is measured on:

* ``scene0`` / ``rays0``: 4,096 surfels scattered in [-1,1]^3 and 64x64x8
  secondary rays from random points with random normals.
* ``scene1`` + ``gbuffer1`` + ``envmap``: 300k surfels on the union of three
  spheres and two tori, an 800x800 G-buffer and a 256x512 environment map.
* ``perturbed``: the loss target's surfel radiance/opacity perturbation.
* ``scene3`` + ``gbuffer3``: 1M surfels in a 4x3x4 room with 20 objects and a
  1024x1024 G-buffer from a camera inside the room.
* ``requests4``: a Poisson stream of relighting requests.

Surfel quaternions are (w, x, y, z); a surfel's normal is its rotation applied
to +z, its tangents the rotation applied to +x and +y.  Scales are the
standard deviations (s_u, s_v) of the 2D Gaussian in its tangent plane.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32 = np.float32


def rng(config_id: int, stream_id: int) -> np.random.Generator:
    """Generator for one (workload, stream) pair; streams never overlap."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([config_id, stream_id])))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _normalize(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def random_unit_vectors(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.standard_normal((n, 3))
    return _normalize(v)


def random_quats(g: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed unit quaternions (normalised 4D Gaussian)."""
    return _normalize(g.standard_normal((n, 4)))


def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of (w,x,y,z) quaternion arrays."""
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def quats_aligned_to(normals: np.ndarray, angles: np.ndarray) -> np.ndarray:
    """Quaternions rotating +z onto ``normals``, spun by ``angles`` about it.

    The spin is applied first (about +z), then the shortest-arc rotation
    from +z to the normal, so the surfel's third axis is the given normal.
    """
    n = _normalize(np.asarray(normals, dtype=np.float64))
    nz = n[:, 2]
    # shortest arc from e3 to n: q = (1 + nz, e3 x n) normalised
    q_arc = np.stack([1.0 + nz, -n[:, 1], n[:, 0], np.zeros_like(nz)], axis=-1)
    flip = nz < -0.999999
    q_arc[flip] = np.array([0.0, 1.0, 0.0, 0.0])  # 180 degrees about x
    q_arc = _normalize(q_arc)
    half = 0.5 * np.asarray(angles, dtype=np.float64)
    q_spin = np.stack([np.cos(half), np.zeros_like(half), np.zeros_like(half), np.sin(half)], axis=-1)
    return _normalize(_qmul(q_arc, q_spin))


def log_uniform(g: np.random.Generator, lo: float, hi: float, size) -> np.ndarray:
    return np.exp(g.uniform(math.log(lo), math.log(hi), size))


# --------------------------------------------------------------------------
# Surfel sets
# --------------------------------------------------------------------------

@dataclass
class Surfels:
    """Surfel parameters in the layout the library takes (SoA, float32)."""
    means: np.ndarray    # [N,3]
    scales: np.ndarray   # [N,2]  (s_u, s_v), linear standard deviations
    quats: np.ndarray    # [N,4]  (w,x,y,z), not necessarily unit
    opacity: np.ndarray  # [N]    in [0,1]
    rgb: np.ndarray      # [N,3]  outgoing radiance

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def arrays(self):
        return self.means, self.scales, self.quats, self.opacity, self.rgb

    def subset(self, idx) -> "Surfels":
        idx = np.asarray(idx)
        return Surfels(*(_f32(a[idx]) for a in self.arrays()))


def _attributes(g: np.random.Generator, n: int):
    opacity = g.uniform(0.2, 0.99, n)
    rgb = g.uniform(0.0, 1.0, (n, 3))
    return opacity, rgb


def scene0(n: int = 4096, seed: int = 0) -> Surfels:
    """Surfels scattered uniformly in [-1,1]^3 with random orientation."""
    g = rng(0 + 100 * seed, 0)
    means = g.uniform(-1.0, 1.0, (n, 3))
    scales = log_uniform(g, 0.01, 0.05, (n, 2))
    quats = random_quats(g, n)
    opacity, rgb = _attributes(g, n)
    return Surfels(_f32(means), _f32(scales), _f32(quats), _f32(opacity), _f32(rgb))


@dataclass
class Rays:
    origins: np.ndarray  # [R,3]
    dirs: np.ndarray     # [R,3] unit
    t_min: float = 0.0
    t_max: float = float("inf")

    @property
    def n(self) -> int:
        return int(self.origins.shape[0])


def hemisphere_dirs(g: np.random.Generator, normals: np.ndarray, per: int) -> np.ndarray:
    """``per`` uniform directions on the hemisphere of each normal, pixel-major."""
    n = np.repeat(normals, per, axis=0)
    d = random_unit_vectors(g, n.shape[0])
    s = np.sign(np.sum(d * n, axis=1, keepdims=True))
    s[s == 0] = 1.0
    return d * s


def rays0(res: int = 64, per: int = 8, seed: int = 0) -> Rays:
    """res x res random points with random normals, ``per`` hemisphere rays each."""
    g = rng(0 + 100 * seed, 1)
    npx = res * res
    origins = g.uniform(-1.0, 1.0, (npx, 3))
    normals = random_unit_vectors(g, npx)
    dirs = hemisphere_dirs(g, normals, per)
    return Rays(_f32(np.repeat(origins, per, axis=0)), _f32(dirs), 0.0, float("inf"))


# --- analytic shapes ---------------------------------------------------------

@dataclass
class Sphere:
    c: np.ndarray
    r: float

    def area(self):
        return 4.0 * math.pi * self.r ** 2

    def sample(self, g, m):
        nrm = random_unit_vectors(g, m)
        return self.c + self.r * nrm, nrm

    def sdf(self, p):
        return np.linalg.norm(p - self.c, axis=-1) - self.r

    def normal(self, p):
        return _normalize(p - self.c)


def _frame_from_axis(axis: np.ndarray):
    a = axis / np.linalg.norm(axis)
    h = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(a, h)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    # local axes: x=e1, y=a (torus symmetry axis), z=e2
    return np.stack([e1, a, e2], axis=0)  # rows are local axes


@dataclass
class Torus:
    c: np.ndarray
    axis: np.ndarray
    R: float
    r: float
    frame: np.ndarray = field(init=False)

    def __post_init__(self):
        self.frame = _frame_from_axis(self.axis)

    def area(self):
        return 4.0 * math.pi ** 2 * self.R * self.r

    def _local(self, p):
        return (p - self.c) @ self.frame.T

    def sample(self, g, m):
        # rejection on the area element (R + r cos theta)
        th_all, ph_all = [], []
        need = m
        while need > 0:
            k = int(need * 1.6) + 16
            th = g.uniform(0, 2 * math.pi, k)
            ph = g.uniform(0, 2 * math.pi, k)
            acc = g.uniform(0, self.R + self.r, k) < self.R + self.r * np.cos(th)
            th_all.append(th[acc]); ph_all.append(ph[acc])
            need -= int(acc.sum())
        th = np.concatenate(th_all)[:m]; ph = np.concatenate(ph_all)[:m]
        ring = np.stack([np.cos(ph), np.zeros_like(ph), np.sin(ph)], axis=-1)
        nl = np.cos(th)[:, None] * ring + np.sin(th)[:, None] * np.array([0.0, 1.0, 0.0])
        pl = self.R * ring + self.r * nl
        return self.c + pl @ self.frame, nl @ self.frame

    def sdf(self, p):
        q = self._local(p)
        rad = np.sqrt(q[..., 0] ** 2 + q[..., 2] ** 2) - self.R
        return np.sqrt(rad ** 2 + q[..., 1] ** 2) - self.r

    def normal(self, p):
        q = self._local(p)
        rxz = np.sqrt(q[..., 0] ** 2 + q[..., 2] ** 2)
        ring = np.stack([q[..., 0] / rxz, np.zeros_like(rxz), q[..., 2] / rxz], axis=-1)
        nl = _normalize(q - self.R * ring)
        return nl @ self.frame


@dataclass
class Box:
    c: np.ndarray
    half: np.ndarray
    yaw: float

    @property
    def rot(self):
        cy, sy = math.cos(self.yaw), math.sin(self.yaw)
        # rows: local x, y, z axes in world coordinates
        return np.array([[cy, 0.0, -sy], [0.0, 1.0, 0.0], [sy, 0.0, cy]])

    def area(self):
        hx, hy, hz = self.half
        return 8.0 * (hx * hy + hy * hz + hx * hz)

    def sample(self, g, m):
        hx, hy, hz = self.half
        areas = np.array([hy * hz, hy * hz, hx * hz, hx * hz, hx * hy, hx * hy])
        face = g.choice(6, size=m, p=areas / areas.sum())
        uv = g.uniform(-1.0, 1.0, (m, 2))
        pl = np.zeros((m, 3)); nl = np.zeros((m, 3))
        axis = face // 2
        sgn = np.where(face % 2 == 0, -1.0, 1.0)
        for a in range(3):
            sel = axis == a
            o1, o2 = [b for b in range(3) if b != a]
            pl[sel, a] = sgn[sel] * self.half[a]
            pl[sel, o1] = uv[sel, 0] * self.half[o1]
            pl[sel, o2] = uv[sel, 1] * self.half[o2]
            nl[sel, a] = sgn[sel]
        R = self.rot
        return self.c + pl @ R, nl @ R

    def inside(self, p):
        q = (p - self.c) @ self.rot.T
        return np.all(np.abs(q) < self.half, axis=-1)

    def intersect(self, o, d):
        """Entry distance and world normal of rays o + t d (inf where missed)."""
        R = self.rot
        ol = (o - self.c) @ R.T
        dl = d @ R.T
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / dl
            t0 = (-self.half - ol) * inv
            t1 = (self.half - ol) * inv
        tn = np.minimum(t0, t1); tf = np.maximum(t0, t1)
        tn = np.nan_to_num(tn, nan=-np.inf); tf = np.nan_to_num(tf, nan=np.inf)
        tnear = tn.max(axis=1); tfar = tf.min(axis=1)
        ax = tn.argmax(axis=1)
        hit = (tnear <= tfar) & (tnear > 1e-9)
        t = np.where(hit, tnear, np.inf)
        nl = np.zeros_like(ol)
        nl[np.arange(len(ax)), ax] = -np.sign(dl[np.arange(len(ax)), ax])
        return t, nl @ R


def _sphere_intersect(o, d, c, r):
    oc = o - c
    b = np.sum(oc * d, axis=1)
    cc = np.sum(oc * oc, axis=1) - r * r
    disc = b * b - cc
    sq = np.sqrt(np.maximum(disc, 0.0))
    t0 = -b - sq
    t1 = -b + sq
    t = np.where(t0 > 1e-9, t0, np.where(t1 > 1e-9, t1, np.inf))
    return np.where(disc >= 0, t, np.inf)


def _place_on_union(g, shapes, n, inside_fns):
    """Area-proportional points on the exterior of a union of shapes."""
    areas = np.array([s.area() for s in shapes])
    pts, nrm = [], []
    have = 0
    while have < n:
        m = int((n - have) * 1.3) + 64
        counts = g.multinomial(m, areas / areas.sum())
        for si, (s, cnt) in enumerate(zip(shapes, counts)):
            if cnt == 0:
                continue
            p, nl = s.sample(g, int(cnt))
            keep = np.ones(len(p), dtype=bool)
            for sj, fn in enumerate(inside_fns):
                if sj != si:
                    keep &= ~fn(p)
            pts.append(p[keep]); nrm.append(nl[keep])
            have += int(keep.sum())
    p = np.concatenate(pts); nl = np.concatenate(nrm)
    order = g.permutation(len(p))[:n]
    return p[order], nl[order]


def _surfels_on(g, pts, nrm, s_lo, s_hi) -> Surfels:
    n = len(pts)
    angles = g.uniform(0.0, 2.0 * math.pi, n)
    quats = quats_aligned_to(nrm, angles)
    scales = log_uniform(g, s_lo, s_hi, (n, 2))
    opacity, rgb = _attributes(g, n)
    return Surfels(_f32(pts), _f32(scales), _f32(quats), _f32(opacity), _f32(rgb))


def shapes1(seed: int = 0):
    g = rng(1 + 100 * seed, 0)
    spheres = [Sphere(g.uniform(-0.8, 0.8, 3), float(g.uniform(0.3, 0.6))) for _ in range(3)]
    tori = [Torus(g.uniform(-0.8, 0.8, 3), random_unit_vectors(g, 1)[0], 0.5, 0.15) for _ in range(2)]
    return spheres + tori


def scene1(n: int = 300_000, seed: int = 0, s_lo: float = 0.003, s_hi: float = 0.02) -> Surfels:
    """Normal-aligned surfels on the union of 3 spheres and 2 tori."""
    shapes = shapes1(seed)
    g = rng(1 + 100 * seed, 1)
    inside = [(lambda p, s=s: s.sdf(p) < 0.0) for s in shapes]
    pts, nrm = _place_on_union(g, shapes, n, inside)
    return _surfels_on(g, pts, nrm, s_lo, s_hi)


# --- G-buffers --------------------------------------------------------------

@dataclass
class GBuffer:
    """Per-pixel shading state; invalid pixels carry zeros and valid == 0."""
    H: int
    W: int
    x: np.ndarray       # [H*W,3] surface point
    n: np.ndarray       # [H*W,3] unit normal
    wo: np.ndarray      # [H*W,3] unit direction towards the camera
    albedo: np.ndarray  # [H*W,3]
    rough: np.ndarray   # [H*W]
    metal: np.ndarray   # [H*W]
    valid: np.ndarray   # [H*W] uint8
    depth: np.ndarray = None  # [H*W] distance from the camera (0 where invalid), when known

    @property
    def npix(self):
        return self.H * self.W

    def arrays(self):
        return self.x, self.n, self.wo, self.albedo, self.rough, self.metal, self.valid

    def subset(self, idx) -> "GBuffer":
        idx = np.asarray(idx)
        a = [np.ascontiguousarray(v[idx]) for v in self.arrays()]
        return GBuffer(1, len(idx), *a)


def pinhole(eye, target, vfov_deg, H, W, up=(0.0, 1.0, 0.0)):
    eye = np.asarray(eye, dtype=np.float64); target = np.asarray(target, dtype=np.float64)
    fwd = _normalize(target - eye)
    right = _normalize(np.cross(fwd, np.asarray(up, dtype=np.float64)))
    upv = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) * 0.5)
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    sx = ((jj + 0.5) / W * 2.0 - 1.0) * th * (W / H)
    sy = (1.0 - (ii + 0.5) / H * 2.0) * th
    d = fwd[None, :] + sx.reshape(-1, 1) * right[None, :] + sy.reshape(-1, 1) * upv[None, :]
    d = _normalize(d)
    return np.broadcast_to(eye, d.shape).copy(), d


def _materials(g, npx, valid):
    albedo = g.uniform(0.0, 1.0, (npx, 3))
    rough = g.uniform(0.05, 1.0, npx)
    metal = (g.uniform(0.0, 1.0, npx) < 0.3).astype(np.float64)
    return albedo * valid[:, None], rough * valid, metal * valid


def _finish_gbuffer(H, W, x, nrm, d, valid, g, o=None):
    valid = valid.astype(bool)
    depth = None
    if o is not None:
        depth = _f32(np.where(valid, np.einsum("ij,ij->i", x - o, d), 0.0))
    x = np.where(valid[:, None], x, 0.0)
    nrm = np.where(valid[:, None], nrm, 0.0)
    wo = np.where(valid[:, None], -d, 0.0)
    albedo, rough, metal = _materials(g, H * W, valid)
    return GBuffer(H, W, _f32(x), _f32(nrm), _f32(wo), _f32(albedo), _f32(rough), _f32(metal),
                   np.ascontiguousarray(valid.astype(np.uint8)), depth)


def _sphere_trace(shapes, o, d, t_far=10.0, eps=1e-10, iters=2000):
    t = np.zeros(len(o))
    active = np.ones(len(o), dtype=bool)
    hit = np.zeros(len(o), dtype=bool)
    for _ in range(iters):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        p = o[idx] + t[idx, None] * d[idx]
        dist = np.min(np.stack([s.sdf(p) for s in shapes], axis=0), axis=0)
        done = dist < eps
        hit[idx[done]] = True
        active[idx[done]] = False
        t[idx[~done]] += dist[~done]
        far = t[idx] > t_far
        active[idx[far & ~done]] = False
    p = o + t[:, None] * d
    sd = np.stack([s.sdf(p) for s in shapes], axis=0)
    which = np.argmin(sd, axis=0)
    nrm = np.zeros_like(p)
    for si, s in enumerate(shapes):
        sel = hit & (which == si)
        if sel.any():
            nrm[sel] = s.normal(p[sel])
    return p, nrm, hit


def gbuffer1(H: int = 800, W: int = 800, seed: int = 0, cam_stream: int = 2) -> GBuffer:
    """Pinhole view of the sphere/torus union from a radius-3.5 orbit."""
    shapes = shapes1(seed)
    g = rng(1 + 100 * seed, cam_stream)
    while True:
        v = random_unit_vectors(g, 1)[0]
        if abs(v[1]) < 0.9:
            break
    o, d = pinhole(3.5 * v, (0.0, 0.0, 0.0), 40.0, H, W)
    x, nrm, hit = _sphere_trace(shapes, o, d)
    return _finish_gbuffer(H, W, x, nrm, d, hit, g, o)


# --- the room scene ----------------------------------------------------------

ROOM_LO = np.array([-2.0, 0.0, -2.0])
ROOM_HI = np.array([2.0, 3.0, 2.0])


def objects3(seed: int = 0):
    g = rng(3 + 100 * seed, 0)
    spheres, boxes = [], []
    for _ in range(10):
        r = float(g.uniform(0.15, 0.45))
        c = np.array([g.uniform(-1.3, 1.3), g.uniform(0.6, 2.2), g.uniform(-1.3, 1.3)])
        spheres.append(Sphere(c, r))
    for _ in range(10):
        half = g.uniform(0.1, 0.4, 3)
        c = np.array([g.uniform(-1.3, 1.3), g.uniform(0.6, 2.2), g.uniform(-1.3, 1.3)])
        boxes.append(Box(c, half, float(g.uniform(0.0, 2.0 * math.pi))))
    return spheres, boxes


def _room_walls_sample(g, m):
    """Area-proportional points on floor + 4 walls, inward normals."""
    # faces: floor (y=0), x=-2, x=+2, z=-2, z=+2
    areas = np.array([16.0, 12.0, 12.0, 12.0, 12.0])
    face = g.choice(5, size=m, p=areas / areas.sum())
    a = g.uniform(0.0, 1.0, m); b = g.uniform(0.0, 1.0, m)
    p = np.zeros((m, 3)); nl = np.zeros((m, 3))
    f = face == 0
    p[f] = np.stack([-2 + 4 * a[f], np.zeros(f.sum()), -2 + 4 * b[f]], axis=-1); nl[f] = (0, 1, 0)
    for k, (axis, val, sgn) in enumerate([(0, -2.0, 1.0), (0, 2.0, -1.0), (2, -2.0, 1.0), (2, 2.0, -1.0)], start=1):
        f = face == k
        q = np.zeros((f.sum(), 3))
        other = 2 if axis == 0 else 0
        q[:, axis] = val
        q[:, 1] = 3.0 * a[f]
        q[:, other] = -2 + 4 * b[f]
        p[f] = q
        nv = np.zeros(3); nv[axis] = sgn
        nl[f] = nv
    return p, nl


def scene3(n_walls: int = 700_000, n_objects: int = 300_000, seed: int = 0,
           s_lo: float = 0.002, s_hi: float = 0.03) -> Surfels:
    """Surfels on the walls and floor of a 4x3x4 room plus 10 spheres and 10 boxes."""
    spheres, boxes = objects3(seed)
    g = rng(3 + 100 * seed, 1)
    pw, nw = _room_walls_sample(g, n_walls)
    shapes = spheres + boxes
    inside = [(lambda p, s=s: np.linalg.norm(p - s.c, axis=-1) < s.r) for s in spheres] + \
             [(lambda p, b=b: b.inside(p)) for b in boxes]
    po, no = _place_on_union(g, shapes, n_objects, inside)
    pts = np.concatenate([pw, po]); nrm = np.concatenate([nw, no])
    perm = g.permutation(len(pts))
    return _surfels_on(g, pts[perm], nrm[perm], s_lo, s_hi)


def _room_intersect(o, d, spheres, boxes):
    nray = len(o)
    best = np.full(nray, np.inf)
    nrm = np.zeros((nray, 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        for (axis, val, nv) in [(1, 0.0, (0, 1, 0)), (0, -2.0, (1, 0, 0)), (0, 2.0, (-1, 0, 0)),
                                (2, -2.0, (0, 0, 1)), (2, 2.0, (0, 0, -1))]:
            t = (val - o[:, axis]) / d[:, axis]
            t = np.where(np.isfinite(t) & (t > 1e-9), t, np.inf)
            p = o + np.where(np.isfinite(t), t, 0.0)[:, None] * d
            inb = np.all((p >= ROOM_LO - 1e-9) & (p <= ROOM_HI + 1e-9), axis=1)
            t = np.where(inb, t, np.inf)
            upd = t < best
            best[upd] = t[upd]; nrm[upd] = nv
    for s in spheres:
        t = _sphere_intersect(o, d, s.c, s.r)
        upd = t < best
        best[upd] = t[upd]
        nrm[upd] = _normalize(o[upd] + t[upd, None] * d[upd] - s.c)
    for b in boxes:
        t, nb = b.intersect(o, d)
        upd = t < best
        best[upd] = t[upd]; nrm[upd] = nb[upd]
    hit = np.isfinite(best)
    x = o + np.where(hit, best, 0.0)[:, None] * d
    return x, nrm, hit


def camera3(g):
    eye = (g.uniform(-1.0, 1.0), g.uniform(1.2, 2.0), 1.95)
    target = (g.uniform(-0.5, 0.5), g.uniform(0.5, 1.5), -2.0)
    return eye, target


def gbuffer3(H: int = 1024, W: int = 1024, seed: int = 0, cam_stream: int = 2) -> GBuffer:
    """View from a camera inside the room (60 degree vertical field of view)."""
    spheres, boxes = objects3(seed)
    g = rng(3 + 100 * seed, cam_stream)
    eye, target = camera3(g)
    o, d = pinhole(eye, target, 60.0, H, W)
    x, nrm, hit = _room_intersect(o, d, spheres, boxes)
    return _finish_gbuffer(H, W, x, nrm, d, hit, g, o)


# --- triangle meshes (the mesh backend's input) ----------------------------

@dataclass
class Mesh:
    """A triangle mesh with per-vertex material attributes and normals."""
    verts: np.ndarray   # [V,3]
    tris: np.ndarray    # [F,3] int32 vertex indices
    albedo: np.ndarray  # [V,3]
    rough: np.ndarray   # [V]
    metal: np.ndarray   # [V]
    normal: np.ndarray  # [V,3] unit

    @property
    def nv(self):
        return self.verts.shape[0]

    @property
    def nf(self):
        return self.tris.shape[0]


def _grid(p0, eu, ev, res):
    """(res+1)^2 vertices over the parallelogram p0 + s eu + t ev, 2 res^2 triangles."""
    s, t = np.meshgrid(np.linspace(0.0, 1.0, res + 1), np.linspace(0.0, 1.0, res + 1), indexing="ij")
    v = p0[None, :] + s.reshape(-1, 1) * eu[None, :] + t.reshape(-1, 1) * ev[None, :]
    i, j = np.meshgrid(np.arange(res), np.arange(res), indexing="ij")
    a = (i * (res + 1) + j).reshape(-1)
    b, c, d = a + (res + 1), a + 1, a + res + 2
    return v, np.concatenate([np.stack([a, b, d], 1), np.stack([a, d, c], 1)])


def _with_materials(g, parts):
    verts, tris, nrm, base = [], [], [], 0
    for v, f, n in parts:
        verts.append(v); tris.append(f + base); nrm.append(n); base += v.shape[0]
    verts = np.concatenate(verts); tris = np.concatenate(tris); nrm = _normalize(np.concatenate(nrm))
    nv = verts.shape[0]
    albedo = g.uniform(0.0, 1.0, (nv, 3)); rough = g.uniform(0.05, 1.0, nv)
    metal = (g.uniform(0.0, 1.0, nv) < 0.3).astype(np.float64)
    return Mesh(_f32(verts), np.ascontiguousarray(tris.astype(np.int32)), _f32(albedo), _f32(rough), _f32(metal),
                _f32(nrm))


def mesh3(seed: int = 0, wall_res: int = 48, segments: int = 48) -> Mesh:
    """The room as triangles: floor and four walls (normals inward, open
    ceiling) as grids, the 10 spheres as UV spheres and the 10 boxes with
    their yaw -- stand-ins for a mesh extracted from optimized surfels."""
    spheres, boxes = objects3(seed)
    g = rng(6 + 100 * seed, 0)
    parts = []
    lo, hi = ROOM_LO, ROOM_HI
    ext = hi - lo
    X, Y, Z = np.eye(3)
    for p0, eu, ev, n in ((lo, ext[0] * X, ext[2] * Z, Y),
                          (lo, ext[1] * Y, ext[2] * Z, X), (np.array([hi[0], lo[1], lo[2]]), ext[1] * Y, ext[2] * Z, -X),
                          (lo, ext[0] * X, ext[1] * Y, Z), (np.array([lo[0], lo[1], hi[2]]), ext[0] * X, ext[1] * Y, -Z)):
        v, f = _grid(p0, eu, ev, wall_res)
        parts.append((v, f, np.tile(n, (v.shape[0], 1))))
    for sp in spheres:
        th, ph = np.meshgrid(np.linspace(0.0, math.pi, segments // 2 + 1), np.linspace(0.0, 2 * math.pi, segments + 1),
                             indexing="ij")
        n = np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], -1).reshape(-1, 3)
        rows, cols = segments // 2, segments
        i, j = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
        a = (i * (cols + 1) + j).reshape(-1)
        b, c, d = a + (cols + 1), a + 1, a + cols + 2
        f = np.concatenate([np.stack([a, b, d], 1), np.stack([a, d, c], 1)])
        parts.append((sp.c + sp.r * n, f, n))
    for bx in boxes:
        R = bx.rot
        for axis in range(3):
            o1, o2 = [b for b in range(3) if b != axis]
            for sgn in (-1.0, 1.0):
                nl = np.zeros(3); nl[axis] = sgn
                corners = []
                for s1, s2 in ((-1, -1), (1, -1), (1, 1), (-1, 1)):
                    pl = np.zeros(3); pl[axis] = sgn * bx.half[axis]
                    pl[o1] = s1 * bx.half[o1]; pl[o2] = s2 * bx.half[o2]
                    corners.append(bx.c + pl @ R)
                v = np.array(corners)
                f = np.array([[0, 1, 2], [0, 2, 3]])
                parts.append((v, f, np.tile(nl @ R, (4, 1))))
    return _with_materials(g, parts)


def tri_soup(n: int = 2000, seed: int = 0) -> Mesh:
    """n random triangles in [-1,1]^3 (edges 0.05..0.3), per-vertex attributes
    and random unit normals."""
    g = rng(7 + 100 * seed, 0)
    c = g.uniform(-1.0, 1.0, (n, 3))
    e1 = random_unit_vectors(g, n) * g.uniform(0.05, 0.3, (n, 1))
    e2 = random_unit_vectors(g, n) * g.uniform(0.05, 0.3, (n, 1))
    v = np.stack([c, c + e1, c + e2], 1).reshape(-1, 3)
    f = np.arange(3 * n).reshape(n, 3)
    return _with_materials(g, [(v, f, random_unit_vectors(g, 3 * n))])


# --- environment maps ------------------------------------------------------

def envmap(H: int = 256, W: int = 512, seed: int = 0, stream: int = 3, config_id: int = 1) -> np.ndarray:
    """Equirectangular RGB radiance [H,W,3]: log-normal texels plus 3 bright lobes.

    Row 0 is the zenith (+y); texel (i,j) centre has polar angle pi(i+.5)/H
    and azimuth 2pi(j+.5)/W measured from +x towards +z.
    """
    g = rng(config_id + 100 * seed, stream)
    L = np.exp(g.normal(-1.0, 0.75, (H, W, 3)))
    th = math.pi * (np.arange(H) + 0.5) / H
    ph = 2.0 * math.pi * (np.arange(W) + 0.5) / W
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    dirs = np.stack([st * np.cos(ph)[None, :], np.broadcast_to(ct, (H, W)), st * np.sin(ph)[None, :]], axis=-1)
    for _ in range(3):
        c = random_unit_vectors(g, 1)[0]
        sigma = g.uniform(0.05, 0.15)
        peak = g.uniform(20.0, 100.0)
        ang = np.arccos(np.clip(dirs @ c, -1.0, 1.0))
        L += peak * np.exp(-0.5 * (ang / sigma) ** 2)[..., None]
    return _f32(L)


# --- loss target -------------------------------------------------------------

def surfel_materials(n: int, seed: int = 0, config_id: int = 5):
    """Per-surfel material attributes for the attribute query: albedo
    U[0,1]^3, roughness U[0.05, 1], metallic Bernoulli(0.3) -- the G-buffer
    material distribution.  Returns (albedo [n,3], rough [n], metal [n])."""
    g = rng(config_id, 10 + seed)
    albedo = g.uniform(0.0, 1.0, (n, 3))
    rough = g.uniform(0.05, 1.0, n)
    metal = (g.uniform(0.0, 1.0, n) < 0.3).astype(np.float64)
    return _f32(albedo), _f32(rough), _f32(metal)


def perturbed(s: Surfels, seed: int = 0, sigma: float = 0.05) -> Surfels:
    """Surfels with radiance and opacity perturbed by N(0, sigma^2) noise."""
    g = rng(2 + 100 * seed, 0)
    rgb = np.maximum(0.0, s.rgb + g.normal(0.0, sigma, s.rgb.shape))
    op = np.clip(s.opacity + g.normal(0.0, sigma, s.opacity.shape), 0.01, 0.99)
    return Surfels(s.means, s.scales, s.quats, _f32(op), _f32(rgb))


# --- sample allocations ----------------------------------------------------

def mis_split(spp: int):
    """Cosine / GGX / environment sample counts: 2:1:1 (32 -> 16/8/8)."""
    n_c = spp // 2
    n_g = (spp - n_c) // 2
    n_e = spp - n_c - n_g
    return n_c, n_g, n_e


# --- relighting request stream --------------------------------------------

@dataclass
class Request:
    rid: int
    arrival_s: float
    res: int
    spp: int
    seed: int
    cam: int          # index into a pool of pre-rendered G-buffers at this res
    env_seed: int


def requests4(n: int, rate_hz: float, seed: int = 0, n_cams: int = 4):
    """Poisson arrivals; resolution and spp drawn uniformly from the fixed sets."""
    g = rng(4 + 100 * seed, 0)
    gaps = g.exponential(1.0 / rate_hz, n)
    t = np.cumsum(gaps) - gaps[0]
    res = g.choice([256, 512, 768, 1024], n)
    spp = g.choice([4, 8, 16, 32, 64], n)
    cams = g.integers(0, n_cams, n)
    return [Request(i, float(t[i]), int(res[i]), int(spp[i]), 1000 + i, int(cams[i]), 5000 + i)
            for i in range(n)]
