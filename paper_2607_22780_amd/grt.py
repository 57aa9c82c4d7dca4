"""Python binding of libgrt (ctypes over the C ABI in ``include/grt.h``).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libgrt.so``.  The functions named ``grt_*`` mirror the C entry points one to
one and take torch tensors (device memory) plus the current HIP stream; the
classes below them only own workspaces and keep borrowed tensors alive.  If
the library is missing or no GPU is present, calls raise ``GrtError``: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrt.so")
# the same sources compiled with -DGRT_STATS (walk statistics; slower kernels)
STATS_LIB_PATH = os.path.join(HERE, "libgrt_stats.so")

OK = 0
ERR_INVALID = -1
ERR_OOM = -2
ERR_NOT_BUILT = -3
ERR_DEVICE = -4
ERR_ADMISSION = -5
ERR_BUSY = -6
ERR_CANCELLED = -7
ERR_TIMEOUT = -8


class GrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


VP = C.c_void_p


class grt_surfels(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", VP), ("scales", VP), ("quats", VP), ("opacity", VP), ("rgb", VP)]


class grt_scene_view(C.Structure):
    _fields_ = [("n", C.c_int64), ("records", VP), ("nodes", VP), ("order", VP), ("leaf_boxes", VP),
                ("colours", VP), ("quats", VP), ("nodes4", VP), ("nodes4_count", VP)]


class grt_rays(C.Structure):
    _fields_ = [("n", C.c_int64), ("origins", VP), ("dirs", VP), ("t_min", VP), ("t_max", VP),
                ("t_min_all", C.c_float), ("t_max_all", C.c_float)]


class grt_trace_opts(C.Structure):
    _fields_ = [("k", C.c_int), ("t_cut", C.c_float), ("sky", C.c_float * 3), ("hit_ids", VP), ("hit_tau", VP),
                ("hit_cap", C.c_int), ("stop_depth", VP), ("env", VP)]


class grt_surfel_grads(C.Structure):
    _fields_ = [("means", VP), ("scales", VP), ("quats", VP), ("opacity", VP), ("rgb", VP)]


class grt_gbuffer_out(C.Structure):
    _fields_ = [("x", VP), ("n", VP), ("wo", VP), ("albedo", VP), ("rough", VP), ("metal", VP), ("depth", VP),
                ("rgb", VP), ("valid", VP), ("weight", VP), ("nlen", VP)]


class grt_gbuffer_grad(C.Structure):
    _fields_ = [("x", VP), ("n", VP), ("albedo", VP), ("rough", VP), ("metal", VP), ("depth", VP), ("rgb", VP)]


class grt_shading_grads(C.Structure):
    _fields_ = [("x", VP), ("n", VP), ("wo", VP), ("albedo", VP), ("rough", VP), ("metal", VP)]


class grt_attr_grads(C.Structure):
    _fields_ = [("albedo", VP), ("rough", VP), ("metal", VP)]


class grt_mesh_desc(C.Structure):
    _fields_ = [("nv", C.c_int64), ("verts", VP), ("nf", C.c_int64), ("tris", VP)]


class grt_vertex_attrs(C.Structure):
    _fields_ = [("albedo", VP), ("rough", VP), ("metal", VP), ("normal", VP)]


class grt_denoise_opts(C.Structure):
    _fields_ = [("radius", C.c_int), ("sigma_s", C.c_float), ("sigma_d", C.c_float), ("sigma_n", C.c_float),
                ("eps_d", C.c_float)]


class grt_surfel_attrs(C.Structure):
    _fields_ = [("albedo", VP), ("rough", VP), ("metal", VP)]


class grt_gbuffer(C.Structure):
    _fields_ = [("H", C.c_int), ("W", C.c_int), ("x", VP), ("n", VP), ("wo", VP), ("albedo", VP), ("rough", VP),
                ("metal", VP), ("valid", VP)]


class grt_mis_opts(C.Structure):
    _fields_ = [("n_cos", C.c_int), ("n_ggx", C.c_int), ("n_env", C.c_int), ("seed", C.c_uint64),
                ("job", C.c_uint32), ("t_min", C.c_float), ("t_cut", C.c_float), ("k", C.c_int),
                ("sample_dump", VP), ("hit_list", VP), ("hit_cap", C.c_int), ("timer", VP)]


class grt_server_opts(C.Structure):
    _fields_ = [("mem_budget", C.c_size_t), ("max_jobs", C.c_int), ("epoch_rays", C.c_int64), ("k", C.c_int),
                ("t_min", C.c_float), ("t_cut", C.c_float), ("slack_per_ray", C.c_double),
                ("preempt_share", C.c_double), ("attrs", grt_surfel_attrs), ("workspace", VP),
                ("ws_bytes", C.c_size_t), ("co_trace", C.c_int), ("k_relight", C.c_int)]


class grt_camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3), ("vfov_deg", C.c_double)]


def make_camera(eye, target, vfov_deg, up=(0.0, 1.0, 0.0)) -> grt_camera:
    c = grt_camera()
    for i in range(3):
        c.eye[i], c.target[i], c.up[i] = float(eye[i]), float(target[i]), float(up[i])
    c.vfov_deg = float(vfov_deg)
    return c


class grt_job(C.Structure):
    _fields_ = [("H", C.c_int), ("W", C.c_int), ("x", VP), ("n", VP), ("wo", VP), ("albedo", VP), ("rough", VP),
                ("metal", VP), ("valid", VP), ("env_rgb", VP), ("env_H", C.c_int), ("env_W", C.c_int),
                ("n_cos", C.c_int), ("n_ggx", C.c_int), ("n_env", C.c_int), ("seed", C.c_uint64),
                ("job", C.c_uint32), ("out_rgb", VP), ("camera_request", C.c_int), ("camera", grt_camera),
                ("min_opacity", C.c_float), ("relight", C.c_int)]


# every symbol include/grt.h declares, with (restype, argtypes)
P = C.POINTER
SIGNATURES = {
    "grt_last_error": (C.c_char_p, []),
    "grt_status_str": (C.c_char_p, [C.c_int]),
    "grt_version": (C.c_int, []),
    "grt_ctx_create": (C.c_int, [C.c_int, P(VP)]),
    "grt_ctx_destroy": (C.c_int, [VP]),
    "grt_scene_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "grt_scene_create": (C.c_int, [VP, P(grt_surfels), C.c_float, VP, C.c_size_t, P(VP)]),
    "grt_scene_build": (C.c_int, [VP, VP]),
    "grt_scene_set_surfels": (C.c_int, [VP, P(grt_surfels)]),
    "grt_scene_destroy": (C.c_int, [VP]),
    "grt_scene_view_get": (C.c_int, [VP, P(grt_scene_view)]),
    "grt_trace_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "grt_trace": (C.c_int, [VP, P(grt_rays), P(grt_trace_opts), VP, VP, VP, VP, VP, C.c_size_t, VP]),
    "grt_trace_backward": (C.c_int, [VP, P(grt_rays), P(grt_trace_opts), VP, VP, VP, VP, P(grt_surfel_grads), VP,
                                     C.c_size_t, VP]),
    "grt_trace_attr": (C.c_int, [VP, P(grt_rays), P(grt_trace_opts), P(grt_surfel_attrs), VP, VP, VP, VP, VP, VP,
                                 C.c_size_t, VP]),
    "grt_trace_gbuffer": (C.c_int, [VP, P(grt_rays), P(grt_trace_opts), P(grt_surfel_attrs), C.c_float,
                                    P(grt_gbuffer_out), VP, C.c_size_t, VP]),
    "grt_camera_rays": (C.c_int, [VP, P(grt_camera), C.c_int, C.c_int, VP, VP, VP]),
    "grt_trace_gbuffer_backward": (C.c_int, [VP, P(grt_rays), P(grt_trace_opts), P(grt_surfel_attrs),
                                             P(grt_gbuffer_out), P(grt_gbuffer_grad), P(grt_surfel_grads),
                                             P(grt_attr_grads), VP, C.c_size_t, VP]),
    "grt_env_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int]),
    "grt_env_create": (C.c_int, [VP, VP, C.c_int, C.c_int, VP, C.c_size_t, P(VP)]),
    "grt_env_build": (C.c_int, [VP, VP]),
    "grt_env_tables": (C.c_int, [VP, P(VP), P(VP)]),
    "grt_env_prefilter": (C.c_int, [VP, VP]),
    "grt_mesh_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "grt_mesh_create": (C.c_int, [VP, P(grt_mesh_desc), VP, C.c_size_t, P(VP)]),
    "grt_mesh_build": (C.c_int, [VP, VP]),
    "grt_mesh_destroy": (C.c_int, [VP]),
    "grt_mesh_trace_attr": (C.c_int, [VP, P(grt_rays), P(grt_vertex_attrs), VP, VP, VP, VP, VP, VP]),
    "grt_render_relight_mesh": (C.c_int, [VP, VP, P(grt_vertex_attrs), P(grt_gbuffer), P(grt_mis_opts), VP, VP,
                                          C.c_size_t, VP]),
    "grt_denoise": (C.c_int, [VP, C.c_int, C.c_int, VP, VP, VP, VP, P(grt_denoise_opts), VP, VP]),
    "grt_env_relight_tables": (C.c_int, [VP, P(VP), P(VP), P(VP)]),
    "grt_render_relight": (C.c_int, [VP, VP, P(grt_surfel_attrs), P(grt_gbuffer), P(grt_mis_opts), VP, VP,
                                     C.c_size_t, VP]),
    "grt_env_destroy": (C.c_int, [VP]),
    "grt_render_saved_bytes": (C.c_size_t, [C.c_int64, C.c_int]),
    "grt_render_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int]),
    "grt_render_mis": (C.c_int, [VP, VP, P(grt_gbuffer), P(grt_mis_opts), VP, VP, VP, C.c_size_t, VP]),
    "grt_render_mis_noalloc": (C.c_int, [VP, VP, P(grt_gbuffer), P(grt_mis_opts), VP, VP, VP]),
    "grt_render_mis_backward": (C.c_int, [VP, VP, P(grt_gbuffer), P(grt_mis_opts), VP, VP, P(grt_surfel_grads),
                                          VP, C.c_size_t, VP]),
    "grt_render_mis_backward_shading": (C.c_int, [VP, VP, P(grt_gbuffer), P(grt_mis_opts), VP, VP,
                                                  P(grt_surfel_grads), P(grt_shading_grads), VP, C.c_size_t, VP]),
    "grt_render_hit_list_bytes": (C.c_size_t, [C.c_int64, C.c_int, C.c_int]),
    "grt_timer_create": (C.c_int, [VP, P(VP)]),
    "grt_timer_ms": (C.c_int, [VP, P(C.c_float)]),
    "grt_timer_destroy": (C.c_int, [VP]),
    "grt_walk_stats": (C.c_int, [VP, P(C.c_uint64), C.c_int]),
    "grt_server_job_bytes": (C.c_size_t, [P(grt_job)]),
    "grt_server_workspace_bytes": (C.c_size_t, [P(grt_server_opts)]),
    "grt_server_create": (C.c_int, [VP, VP, P(grt_server_opts), P(VP)]),
    "grt_server_submit": (C.c_int, [VP, P(grt_job), P(C.c_uint64)]),
    "grt_server_poll": (C.c_int, [VP, C.c_uint64, P(C.c_int)]),
    "grt_server_wait": (C.c_int, [VP, C.c_uint64, C.c_double]),
    "grt_server_cancel": (C.c_int, [VP, C.c_uint64]),
    "grt_server_job_times": (C.c_int, [VP, C.c_uint64, P(C.c_double), P(C.c_double), P(C.c_double)]),
    "grt_server_stats": (C.c_int, [VP, P(C.c_uint64), P(C.c_uint64), P(C.c_int64), P(C.c_size_t)]),
    "grt_server_destroy": (C.c_int, [VP]),
}
OPTIONAL = {}

_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libgrt.so and declare every signature; raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise GrtError(ERR_DEVICE, f"libgrt.so not built at {path}: run __graft_entry__.build()")
    lib = C.CDLL(path)
    for name, (res, args) in {**SIGNATURES, **OPTIONAL}.items():
        if not hasattr(lib, name):
            if name in OPTIONAL:
                continue
            raise GrtError(ERR_INVALID, f"libgrt.so lacks {name}")
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load_library()
        raise GrtError(rc, f"{lib.grt_status_str(rc).decode()}: {lib.grt_last_error().decode()}")


def _ptr(t):
    if t is None:
        return None
    return VP(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return VP(stream.cuda_stream)


def _dev_f32(t, shape_tail, name, device):
    if not isinstance(t, torch.Tensor):
        raise GrtError(ERR_INVALID, f"{name} must be a tensor")
    if t.dtype != torch.float32 or t.device != device or not t.is_contiguous():
        raise GrtError(ERR_INVALID, f"{name} must be contiguous float32 on {device}")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise GrtError(ERR_INVALID, f"{name} has shape {tuple(t.shape)}, want [n,{shape_tail}]")
    return t


# --------------------------------------------------------------------------
# One-to-one wrappers of the C entry points
# --------------------------------------------------------------------------

def grt_version() -> int:
    return load_library().grt_version()


def grt_ctx_create(device: int = 0):
    out = VP()
    _check(load_library().grt_ctx_create(device, C.byref(out)))
    return out


def grt_ctx_destroy(ctx):
    _check(load_library().grt_ctx_destroy(ctx))


def grt_scene_workspace_bytes(n: int) -> int:
    return int(load_library().grt_scene_workspace_bytes(n))


def _surfels_struct(means, scales, quats, opacity, rgb):
    dev = means.device
    n = means.shape[0]
    _dev_f32(means, (3,), "means", dev); _dev_f32(scales, (2,), "scales", dev); _dev_f32(quats, (4,), "quats", dev)
    _dev_f32(rgb, (3,), "rgb", dev)
    if opacity.dtype != torch.float32 or opacity.device != dev or not opacity.is_contiguous() or opacity.dim() != 1:
        raise GrtError(ERR_INVALID, "opacity must be contiguous float32 [n]")
    for t in (scales, quats, opacity, rgb):
        if t.shape[0] != n:
            raise GrtError(ERR_INVALID, "surfel arrays disagree in length")
    return grt_surfels(n, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opacity), _ptr(rgb))


def grt_scene_create(ctx, surfels: grt_surfels, alpha_min: float, workspace: torch.Tensor):
    out = VP()
    _check(load_library().grt_scene_create(ctx, C.byref(surfels), alpha_min, _ptr(workspace), workspace.numel(),
                                           C.byref(out)))
    return out


def grt_scene_build(scene, stream=None):
    _check(load_library().grt_scene_build(scene, _stream(stream)))


def grt_scene_set_surfels(scene, surfels: grt_surfels):
    _check(load_library().grt_scene_set_surfels(scene, C.byref(surfels)))


def grt_scene_destroy(scene):
    _check(load_library().grt_scene_destroy(scene))


def grt_scene_view_get(scene) -> grt_scene_view:
    v = grt_scene_view()
    _check(load_library().grt_scene_view_get(scene, C.byref(v)))
    return v


def grt_trace_workspace_bytes(n: int) -> int:
    return int(load_library().grt_trace_workspace_bytes(n))


def grt_trace(scene, rays: grt_rays, opts: grt_trace_opts, out_rgb, out_T, out_L, out_nhit, workspace, stream=None):
    _check(load_library().grt_trace(scene, C.byref(rays), C.byref(opts), _ptr(out_rgb), _ptr(out_T), _ptr(out_L),
                                    _ptr(out_nhit), _ptr(workspace), workspace.numel(), _stream(stream)))


def grt_trace_attr(scene, rays: grt_rays, opts: grt_trace_opts, attrs: grt_surfel_attrs, out_V, out_albedo, out_rough,
                   out_metal, out_normal, workspace, stream=None):
    _check(load_library().grt_trace_attr(scene, C.byref(rays), C.byref(opts), C.byref(attrs), _ptr(out_V),
                                         _ptr(out_albedo), _ptr(out_rough), _ptr(out_metal), _ptr(out_normal),
                                         _ptr(workspace), workspace.numel(), _stream(stream)))


def grt_trace_backward(scene, rays, opts, fwd_rgb, fwd_T, grad_rgb, grad_T, grads: grt_surfel_grads, workspace,
                       stream=None):
    _check(load_library().grt_trace_backward(scene, C.byref(rays), C.byref(opts), _ptr(fwd_rgb), _ptr(fwd_T),
                                             _ptr(grad_rgb), _ptr(grad_T), C.byref(grads), _ptr(workspace),
                                             workspace.numel(), _stream(stream)))


def grt_env_workspace_bytes(H: int, W: int) -> int:
    return int(load_library().grt_env_workspace_bytes(H, W))


def grt_env_create(ctx, rgb, H, W, workspace):
    out = VP()
    _check(load_library().grt_env_create(ctx, _ptr(rgb), H, W, _ptr(workspace), workspace.numel(), C.byref(out)))
    return out


def grt_env_build(env, stream=None):
    _check(load_library().grt_env_build(env, _stream(stream)))


def grt_env_tables(env):
    m, c = VP(), VP()
    _check(load_library().grt_env_tables(env, C.byref(m), C.byref(c)))
    return m.value, c.value


def grt_env_prefilter(env, stream=None):
    _check(load_library().grt_env_prefilter(env, _stream(stream)))


def grt_env_relight_tables(env):
    a, b, c = VP(), VP(), VP()
    _check(load_library().grt_env_relight_tables(env, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def grt_render_relight(scene, env, attrs: grt_surfel_attrs, gbuf: grt_gbuffer, opts: grt_mis_opts, out_rgb,
                       workspace, stream=None):
    _check(load_library().grt_render_relight(scene, env, C.byref(attrs), C.byref(gbuf), C.byref(opts),
                                             _ptr(out_rgb), _ptr(workspace), workspace.numel(), _stream(stream)))


def grt_env_destroy(env):
    _check(load_library().grt_env_destroy(env))


def grt_render_saved_bytes(npix: int, spp: int) -> int:
    return int(load_library().grt_render_saved_bytes(npix, spp))


def grt_render_workspace_bytes(npix: int, spp: int) -> int:
    return int(load_library().grt_render_workspace_bytes(npix, spp))


def grt_render_mis(scene, env, gbuf: grt_gbuffer, opts: grt_mis_opts, out_rgb, saved, workspace, stream=None):
    _check(load_library().grt_render_mis(scene, env, C.byref(gbuf), C.byref(opts), _ptr(out_rgb), _ptr(saved),
                                         _ptr(workspace), workspace.numel(), _stream(stream)))


def grt_render_mis_noalloc(scene, env, gbuf: grt_gbuffer, opts: grt_mis_opts, out_rgb, saved, stream=None):
    _check(load_library().grt_render_mis_noalloc(scene, env, C.byref(gbuf), C.byref(opts), _ptr(out_rgb),
                                                 _ptr(saved), _stream(stream)))


def grt_render_mis_backward(scene, env, gbuf, opts, grad_rgb, saved, grads: grt_surfel_grads, workspace,
                            stream=None):
    _check(load_library().grt_render_mis_backward(scene, env, C.byref(gbuf), C.byref(opts), _ptr(grad_rgb),
                                                  _ptr(saved), C.byref(grads), _ptr(workspace), workspace.numel(),
                                                  _stream(stream)))


# --------------------------------------------------------------------------
# Owners of handles and workspaces
# --------------------------------------------------------------------------

def grt_render_mis_backward_shading(scene, env, gbuf, opts, grad_rgb, saved, grads: grt_surfel_grads,
                                    shade: grt_shading_grads, workspace, stream=None):
    _check(load_library().grt_render_mis_backward_shading(scene, env, C.byref(gbuf), C.byref(opts), _ptr(grad_rgb),
                                                          _ptr(saved), C.byref(grads), C.byref(shade),
                                                          _ptr(workspace), workspace.numel(), _stream(stream)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Context:
    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self.handle = grt_ctx_create(device)

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.grt_ctx_destroy(self.handle)
            self.handle = None


class Scene:
    """A built LBVH over borrowed surfel tensors (kept alive here)."""

    def __init__(self, ctx: Context, means, scales, quats, opacity, rgb, alpha_min: float = 1.0 / 255.0,
                 build: bool = True, stream=None):
        self.ctx = ctx
        self.n = int(means.shape[0])
        self.tensors = (means, scales, quats, opacity, rgb)
        st = _surfels_struct(*self.tensors)
        self.workspace = _workspace(grt_scene_workspace_bytes(self.n), ctx.device)
        self.handle = grt_scene_create(ctx.handle, st, alpha_min, self.workspace)
        self.alpha_min = alpha_min
        if build:
            self.build(stream)

    def set_surfels(self, means, scales, quats, opacity, rgb):
        self.tensors = (means, scales, quats, opacity, rgb)
        grt_scene_set_surfels(self.handle, _surfels_struct(*self.tensors))

    def build(self, stream=None):
        grt_scene_build(self.handle, stream)

    def view(self):
        return grt_scene_view_get(self.handle)

    def arrays(self):
        """Torch views into the built scene: records [n,16], nodes [n-1,16]
        (float32; children as int32 in words 12-13), leaf boxes [n,6], order [n],
        colours [n,4] (rgb, s_v) and stored quaternions [n,4], all in sorted order;
        nodes4 [n-1,32] (the 4-wide hierarchy: boxes as structure of arrays in
        words 0-23, children as int32 in words 24-27) and nodes4_count [1]."""
        v = self.view()
        base = self.workspace.data_ptr()

        def sl(ptr, count, dtype):
            off = ptr - base
            return self.workspace[off:off + 4 * count].view(dtype)

        n = self.n
        return dict(records=sl(v.records, 16 * n, torch.float32).view(n, 16),
                    nodes=sl(v.nodes, 16 * max(n - 1, 0), torch.float32).view(max(n - 1, 0), 16),
                    leaf_boxes=sl(v.leaf_boxes, 6 * n, torch.float32).view(n, 6),
                    order=sl(v.order, n, torch.int32),
                    colours=sl(v.colours, 4 * n, torch.float32).view(n, 4),
                    quats=sl(v.quats, 4 * n, torch.float32).view(n, 4),
                    nodes4=sl(v.nodes4, 32 * max(n - 1, 0), torch.float32).view(max(n - 1, 0), 32),
                    nodes4_count=sl(v.nodes4_count, 1, torch.int32))

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.grt_scene_destroy(self.handle)
            self.handle = None


class Env:
    """Environment map [H,W,3] with its sampling tables."""

    def __init__(self, ctx: Context, rgb: torch.Tensor, stream=None):
        if rgb.dim() != 3 or rgb.shape[2] != 3 or rgb.dtype != torch.float32 or not rgb.is_contiguous():
            raise GrtError(ERR_INVALID, "env must be contiguous float32 [H,W,3]")
        self.ctx = ctx
        self.rgb = rgb
        self.H, self.W = int(rgb.shape[0]), int(rgb.shape[1])
        self.workspace = _workspace(grt_env_workspace_bytes(self.H, self.W), ctx.device)
        self.handle = grt_env_create(ctx.handle, rgb, self.H, self.W, self.workspace)
        grt_env_build(self.handle, stream)

    def tables(self):
        """(marg [H+1], cond [H,W+1]) as tensors viewing the workspace."""
        m, c = grt_env_tables(self.handle)
        base = self.workspace.data_ptr()
        ws = self.workspace
        mo, co = (m - base), (c - base)
        marg = ws[mo:mo + 4 * (self.H + 1)].view(torch.float32)
        cond = ws[co:co + 4 * self.H * (self.W + 1)].view(torch.float32).view(self.H, self.W + 1)
        return marg, cond

    def prefilter(self, stream=None):
        """Build the prefiltered tables split-sum relighting reads."""
        grt_env_prefilter(self.handle, stream)
        return self

    def relight_tables(self):
        """(Ed [16,32,3], Es [5,16,32,3], lut [32,32,2]) viewing the workspace."""
        base = self.workspace.data_ptr()
        ws = self.workspace
        out = []
        for ptr, shape in zip(grt_env_relight_tables(self.handle), ((16, 32, 3), (5, 16, 32, 3), (32, 32, 2))):
            n = 1
            for x in shape:
                n *= x
            o = ptr - base
            out.append(ws[o:o + 4 * n].view(torch.float32).view(*shape))
        return tuple(out)

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.grt_env_destroy(self.handle)
            self.handle = None


def make_rays(origins, dirs, t_min=0.0, t_max=float("inf")):
    dev = origins.device
    _dev_f32(origins, (3,), "origins", dev); _dev_f32(dirs, (3,), "dirs", dev)
    r = grt_rays(origins.shape[0], _ptr(origins), _ptr(dirs), None, None, 0.0, 0.0)
    if isinstance(t_min, torch.Tensor):
        r.t_min = _ptr(t_min)
    else:
        r.t_min_all = float(t_min)
    if isinstance(t_max, torch.Tensor):
        r.t_max = _ptr(t_max)
    else:
        r.t_max_all = float(t_max)
    return r


def make_trace_opts(k=16, t_cut=1e-3, sky=(0.5, 0.5, 0.5), hit_ids=None, hit_tau=None, stop=None, env=None):
    o = grt_trace_opts()
    o.env = env.handle if env is not None else None
    o.k = k
    o.t_cut = t_cut
    for i in range(3):
        o.sky[i] = sky[i]
    o.hit_ids = _ptr(hit_ids)
    o.hit_tau = _ptr(hit_tau)
    o.hit_cap = int(hit_ids.shape[1]) if hit_ids is not None else 0
    o.stop_depth = _ptr(stop)
    return o


def trace(scene: Scene, origins, dirs, t_min=0.0, t_max=float("inf"), k=16, t_cut=1e-3, sky=(0.5, 0.5, 0.5),
          dump_cap=0, save_stop=False, stream=None, env=None):
    """Trace every ray; returns dict of rgb [R,3], T [R], L [R,3], nhit [R]
    (L = rgb + T sky, or rgb + T L_env(d) under a built Env ``env``)
    (and ids/tau [R,dump_cap] when dump_cap > 0; with ``save_stop`` also
    stop [R], the depth of each ray's last composited hit, which
    trace_backward takes to bound its re-traversal)."""
    dev = origins.device
    R = origins.shape[0]
    out = dict(rgb=torch.empty(R, 3, device=dev), T=torch.empty(R, device=dev), L=torch.empty(R, 3, device=dev),
               nhit=torch.empty(R, dtype=torch.int32, device=dev))
    ids = tau = None
    if dump_cap:
        ids = torch.empty(R, dump_cap, dtype=torch.int32, device=dev)
        tau = torch.empty(R, dump_cap, dtype=torch.float32, device=dev)
        out["ids"], out["tau"] = ids, tau
    if save_stop:
        out["stop"] = torch.empty(R, device=dev)
    rays = make_rays(origins, dirs, t_min, t_max)
    opts = make_trace_opts(k, t_cut, sky, ids, tau, out.get("stop"), env)
    ws = _workspace(grt_trace_workspace_bytes(R), dev)
    grt_trace(scene.handle, rays, opts, out["rgb"], out["T"], out["L"], out["nhit"], ws, stream)
    return out


def trace_attr(scene: Scene, albedo, rough, metal, origins, dirs, t_min=0.0, t_max=float("inf"), k=12, t_cut=1e-3,
               stream=None):
    """Attribute query (Eq. trace_attr, Gaussian backend) of every ray: dict
    of V [R] (environment visibility), albedo [R,3], rough [R], metal [R],
    normal [R,3] (normalized-weight averages over the composited hits)."""
    dev = origins.device
    R = origins.shape[0]
    for a in (albedo, rough, metal):
        assert a.is_contiguous() and a.dtype == torch.float32 and a.device == dev
    out = dict(V=torch.empty(R, device=dev), albedo=torch.empty(R, 3, device=dev), rough=torch.empty(R, device=dev),
               metal=torch.empty(R, device=dev), normal=torch.empty(R, 3, device=dev))
    rays = make_rays(origins, dirs, t_min, t_max)
    opts = make_trace_opts(k, t_cut, (0.0, 0.0, 0.0), None, None)
    attrs = grt_surfel_attrs(_ptr(albedo), _ptr(rough), _ptr(metal))
    ws = _workspace(grt_trace_workspace_bytes(R), dev)
    grt_trace_attr(scene.handle, rays, opts, attrs, out["V"], out["albedo"], out["rough"], out["metal"],
                   out["normal"], ws, stream)
    return out


GBUFFER_OUT_KEYS = ("x", "n", "wo", "albedo", "rough", "metal", "depth", "rgb", "valid", "weight", "nlen")
GBUFFER_GRAD_KEYS = ("x", "n", "albedo", "rough", "metal", "depth", "rgb")


def _gbuffer_out_struct(o):
    return grt_gbuffer_out(*(_ptr(o[k_]) if o.get(k_) is not None else None for k_ in GBUFFER_OUT_KEYS))


def camera_rays(ctx: Context, camera: grt_camera, H: int, W: int, stream=None):
    """Primary rays of an H x W pinhole camera (row-major, row 0 at the top):
    (origins [H*W,3], dirs [H*W,3]) on the context's device."""
    dev = ctx.device
    o = torch.empty(H * W, 3, device=dev)
    d = torch.empty(H * W, 3, device=dev)
    _check(load_library().grt_camera_rays(ctx.handle, C.byref(camera), int(H), int(W), _ptr(o), _ptr(d),
                                          _stream(stream)))
    return o, d


def trace_gbuffer(scene: Scene, albedo, rough, metal, origins, dirs, H: int, W: int, min_opacity=0.5, k=12,
                  t_cut=1e-3, stream=None):
    """Primary-ray G-buffer by 2DGRT of H x W camera rays (row-major): dict
    with a GBuffer ("gbuffer", usable by render_mis / render_relight), the
    depth [H*W] and colour [H*W,3] maps, and what the backward needs besides
    the maps (weight = the sum of the blending weights, nlen = the averaged
    normal's length before renormalization, stop = the depth of the last
    composited hit)."""
    dev = origins.device
    R = origins.shape[0]
    assert R == H * W
    for a in (albedo, rough, metal):
        assert a.is_contiguous() and a.dtype == torch.float32 and a.device == dev
    e3 = lambda: torch.empty(R, 3, device=dev)
    e1 = lambda: torch.empty(R, device=dev)
    o = dict(x=e3(), n=e3(), wo=e3(), albedo=e3(), rough=e1(), metal=e1(), depth=e1(), rgb=e3(),
             valid=torch.empty(R, dtype=torch.uint8, device=dev), weight=e1(), nlen=e1(), stop=e1())
    st = _gbuffer_out_struct(o)
    rays = make_rays(origins, dirs, 0.0, float("inf"))
    opts = make_trace_opts(k, t_cut, (0.0, 0.0, 0.0), None, None, o["stop"])
    attrs = grt_surfel_attrs(_ptr(albedo), _ptr(rough), _ptr(metal))
    ws = _workspace(grt_trace_workspace_bytes(R), dev)
    _check(load_library().grt_trace_gbuffer(scene.handle, C.byref(rays), C.byref(opts), C.byref(attrs),
                                            float(min_opacity), C.byref(st), _ptr(ws), ws.numel(), _stream(stream)))
    o["gbuffer"] = GBuffer(H, W, o["x"], o["n"], o["wo"], o["albedo"], o["rough"], o["metal"], o["valid"])
    return o


def trace_gbuffer_backward(scene: Scene, albedo, rough, metal, origins, dirs, fwd, grad, k=12, t_cut=1e-3,
                           grads=None, attr_grads=None, stream=None):
    """Backward of trace_gbuffer (same scene, rays, attributes, k and t_cut;
    ``fwd`` is its output dict): accumulates d/d(surfels) and d/d(albedo,
    rough, metal) of the sum over covered pixels of grad[key] . map[key]
    (keys x, n, albedo, rough, metal, depth, rgb; missing keys are zero).
    Returns (grads, attr_grads)."""
    dev = origins.device
    R = origins.shape[0]
    for a in (albedo, rough, metal):
        assert a.is_contiguous() and a.dtype == torch.float32 and a.device == dev
    if grads is None:
        grads = zero_grads(scene.n, dev)
    if attr_grads is None:
        attr_grads = dict(albedo=torch.zeros(scene.n, 3, device=dev), rough=torch.zeros(scene.n, device=dev),
                          metal=torch.zeros(scene.n, device=dev))
    gin = {}
    for key in GBUFFER_GRAD_KEYS:
        g = grad.get(key)
        if g is not None:
            g = g.contiguous()
            assert g.dtype == torch.float32 and g.device == dev and g.numel() == R * (3 if fwd[key].dim() == 2 else 1)
        gin[key] = g
    gst = grt_gbuffer_grad(*(_ptr(gin[key]) if gin[key] is not None else None for key in GBUFFER_GRAD_KEYS))
    ast = grt_attr_grads(*(_ptr(attr_grads[key]) if attr_grads.get(key) is not None else None
                           for key in ("albedo", "rough", "metal")))
    rays = make_rays(origins, dirs, 0.0, float("inf"))
    opts = make_trace_opts(k, t_cut, (0.0, 0.0, 0.0), None, None, fwd.get("stop"))
    attrs = grt_surfel_attrs(_ptr(albedo), _ptr(rough), _ptr(metal))
    ws = _workspace(grt_trace_workspace_bytes(R), dev)
    _check(load_library().grt_trace_gbuffer_backward(scene.handle, C.byref(rays), C.byref(opts), C.byref(attrs),
                                                     C.byref(_gbuffer_out_struct(fwd)), C.byref(gst),
                                                     C.byref(_grads_struct(grads)), C.byref(ast), _ptr(ws),
                                                     ws.numel(), _stream(stream)))
    return grads, attr_grads


def zero_grads(n: int, device):
    return dict(means=torch.zeros(n, 3, device=device), scales=torch.zeros(n, 2, device=device),
                quats=torch.zeros(n, 4, device=device), opacity=torch.zeros(n, device=device),
                rgb=torch.zeros(n, 3, device=device))


def _grads_struct(g):
    return grt_surfel_grads(_ptr(g["means"]), _ptr(g["scales"]), _ptr(g["quats"]), _ptr(g["opacity"]),
                            _ptr(g["rgb"]))


def trace_backward(scene: Scene, origins, dirs, fwd_rgb, fwd_T, grad_rgb, grad_T=None, t_min=0.0,
                   t_max=float("inf"), k=16, t_cut=1e-3, grads=None, stop=None, stream=None):
    """Accumulate d/d(surfels) of sum grad_rgb . c_rt + grad_T . T into
    ``grads``; ``stop`` (the forward's, from trace(save_stop=True)) bounds the
    re-traversal."""
    if grads is None:
        grads = zero_grads(scene.n, origins.device)
    rays = make_rays(origins, dirs, t_min, t_max)
    opts = make_trace_opts(k, t_cut, stop=stop)
    ws = _workspace(grt_trace_workspace_bytes(origins.shape[0]), origins.device)
    grt_trace_backward(scene.handle, rays, opts, fwd_rgb, fwd_T, grad_rgb.contiguous(),
                       None if grad_T is None else grad_T.contiguous(), _grads_struct(grads), ws, stream)
    return grads


class GBuffer:
    """Device copy of a shading-state buffer (x, n, wo, albedo, rough, metal, valid)."""

    def __init__(self, H, W, x, n, wo, albedo, rough, metal, valid):
        self.H, self.W = int(H), int(W)
        self.x, self.n, self.wo, self.albedo, self.rough, self.metal, self.valid = x, n, wo, albedo, rough, metal, valid

    @staticmethod
    def from_numpy(gb, device):
        t = lambda a: torch.from_numpy(a).to(device).contiguous()
        return GBuffer(gb.H, gb.W, t(gb.x), t(gb.n), t(gb.wo), t(gb.albedo), t(gb.rough), t(gb.metal), t(gb.valid))

    @property
    def npix(self):
        return self.H * self.W

    def struct(self):
        return grt_gbuffer(self.H, self.W, _ptr(self.x), _ptr(self.n), _ptr(self.wo), _ptr(self.albedo),
                           _ptr(self.rough), _ptr(self.metal), _ptr(self.valid))


class Timer:
    """Kernel timer (grt_timer): pass as ``timer=`` to render_mis /
    render_mis_backward; ``ms()`` is the last recorded trace kernel's time."""

    def __init__(self, ctx: Context):
        self._ctx = ctx
        h = VP()
        _check(load_library().grt_timer_create(ctx.handle, C.byref(h)))
        self.handle = h

    def ms(self) -> float:
        v = C.c_float()
        _check(load_library().grt_timer_ms(self.handle, C.byref(v)))
        return float(v.value)

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.grt_timer_destroy(self.handle)
            self.handle = None


WALK_STATS = ("rays", "node_visits", "leaf_tests", "composites", "rounds", "restarts", "deferred", "wave_steps",
              "active_lanes")


def walk_stats(ctx: Context, reset: bool = True) -> dict:
    """The walk statistics (grt_walk_stats) of a library built with
    -DGRT_STATS: {"forward": {...}, "backward": {...}} of WALK_STATS sums."""
    out = (C.c_uint64 * (2 * len(WALK_STATS)))()
    _check(load_library().grt_walk_stats(ctx.handle, out, int(reset)))
    v = list(out)
    n = len(WALK_STATS)
    return {kind: dict(zip(WALK_STATS, v[i * n:(i + 1) * n])) for i, kind in enumerate(("forward", "backward"))}


def make_mis_opts(split=(16, 8, 8), seed=0, job=0, t_min=1e-3, t_cut=1e-3, k=16, dump=None, hits=None, hit_cap=0,
                  timer=None):
    o = grt_mis_opts()
    o.n_cos, o.n_ggx, o.n_env = split
    o.seed = seed
    o.job = job
    o.t_min = t_min
    o.t_cut = t_cut
    o.k = k
    o.sample_dump = _ptr(dump)
    o.hit_list = _ptr(hits)
    o.hit_cap = int(hit_cap) if hits is not None else 0
    o.timer = timer.handle if timer is not None else None
    return o


def grt_render_hit_list_bytes(npix: int, spp: int, hit_cap: int) -> int:
    return int(load_library().grt_render_hit_list_bytes(npix, spp, hit_cap))


def make_hit_list(npix: int, spp: int, hit_cap: int, device):
    """Device buffer for stored hit lists: counts [nray] then [nray, hit_cap]."""
    n = grt_render_hit_list_bytes(npix, spp, hit_cap) // 4
    return torch.empty(n, dtype=torch.int32, device=device)


def render_mis(scene: Scene, env: Env, gb: GBuffer, split=(16, 8, 8), seed=0, job=0, t_min=1e-3, t_cut=1e-3, k=16,
               save=False, dump=False, workspace=None, stream=None, hits=None, hit_cap=0, timer=None):
    """c_pbr [npix,3]; with ``save`` also the per-sample state for the
    backward ("saved", flat; views "saved_ct" [nray,4] = (c_rt, T) and
    "saved_stop" [nray] = the depth of the last composited hit, 0 if none),
    with ``dump`` the per-sample record [npix, spp, 10]."""
    dev = gb.x.device
    spp = sum(split)
    out = torch.empty(gb.npix, 3, device=dev)
    saved = torch.empty(grt_render_saved_bytes(gb.npix, spp) // 4, device=dev) if save else None
    dmp = torch.zeros(gb.npix, spp, 10, device=dev) if dump else None
    opts = make_mis_opts(split, seed, job, t_min, t_cut, k, dmp, hits, hit_cap, timer)
    need = grt_render_workspace_bytes(gb.npix, spp)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    grt_render_mis(scene.handle, env.handle, gb.struct(), opts, out, saved, workspace, stream)
    res = dict(rgb=out)
    if save:
        nray = gb.npix * spp
        res["saved"] = saved
        res["saved_ct"] = saved[: 4 * nray].view(nray, 4)
        res["saved_stop"] = saved[4 * nray: 5 * nray]
    if dump:
        res["dump"] = dmp
    return res


def render_relight(scene: Scene, env: Env, albedo, rough, metal, gb: GBuffer, split=(16, 8, 8), seed=0, job=0,
                   t_min=1e-3, t_cut=1e-3, k=12, dump=False, workspace=None, stream=None):
    """Relit c_pbr [npix,3] under the prefiltered `env` (Sec. 3.5.1, Eq.
    relight_splitsum), surfel attributes albedo [n,3], rough [n], metal [n]."""
    dev = gb.x.device
    spp = sum(split)
    out = torch.empty(gb.npix, 3, device=dev)
    dmp = torch.zeros(gb.npix, spp, 10, device=dev) if dump else None
    opts = make_mis_opts(split, seed, job, t_min, t_cut, k, dmp)
    attrs = grt_surfel_attrs(_ptr(albedo), _ptr(rough), _ptr(metal))
    need = grt_render_workspace_bytes(gb.npix, spp)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    grt_render_relight(scene.handle, env.handle, attrs, gb.struct(), opts, out, workspace, stream)
    res = dict(rgb=out)
    if dump:
        res["dump"] = dmp
    return res


class Mesh:
    """A triangle mesh (verts [V,3] float32, tris [F,3] int32, device) with its
    LBVH, for the mesh backend of the attribute query."""

    def __init__(self, ctx: Context, verts: torch.Tensor, tris: torch.Tensor, stream=None):
        assert verts.is_contiguous() and verts.dtype == torch.float32
        assert tris.is_contiguous() and tris.dtype == torch.int32
        self.ctx, self.verts, self.tris = ctx, verts, tris
        self.nv, self.nf = int(verts.shape[0]), int(tris.shape[0])
        self.workspace = _workspace(int(load_library().grt_mesh_workspace_bytes(self.nf)), verts.device)
        self.desc = grt_mesh_desc(self.nv, _ptr(verts), self.nf, _ptr(tris))
        h = VP()
        _check(load_library().grt_mesh_create(ctx.handle, C.byref(self.desc), _ptr(self.workspace),
                                              self.workspace.numel(), C.byref(h)))
        self.handle = h.value
        _check(load_library().grt_mesh_build(self.handle, _stream(stream)))

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.grt_mesh_destroy(self.handle)
            self.handle = None


def mesh_trace_attr(mesh: Mesh, albedo, rough, metal, normal, origins, dirs, t_min=0.0, t_max=float("inf"),
                    stream=None):
    """Mesh backend of Trace_attr: dict of V [R], albedo [R,3], rough [R],
    metal [R], normal [R,3] (barycentric, facing the ray origin)."""
    dev = origins.device
    R = origins.shape[0]
    for a in (albedo, rough, metal, normal):
        assert a.is_contiguous() and a.dtype == torch.float32 and a.device == dev
    out = dict(V=torch.empty(R, device=dev), albedo=torch.empty(R, 3, device=dev), rough=torch.empty(R, device=dev),
               metal=torch.empty(R, device=dev), normal=torch.empty(R, 3, device=dev))
    rays = make_rays(origins, dirs, t_min, t_max)
    va = grt_vertex_attrs(_ptr(albedo), _ptr(rough), _ptr(metal), _ptr(normal))
    _check(load_library().grt_mesh_trace_attr(mesh.handle, C.byref(rays), C.byref(va), _ptr(out["V"]),
                                              _ptr(out["albedo"]), _ptr(out["rough"]), _ptr(out["metal"]),
                                              _ptr(out["normal"]), _stream(stream)))
    return out


def render_relight_mesh(mesh: Mesh, env: Env, albedo, rough, metal, normal, gb, split=(16, 8, 8), seed=0, job=0,
                        t_min=1e-3, dump=False, workspace=None, stream=None):
    """Relit c_pbr [npix,3] under the prefiltered `env` with the mesh backend
    answering the attribute query (per-vertex albedo, rough, metal, normal)."""
    dev = gb.x.device
    spp = sum(split)
    out = torch.empty(gb.npix, 3, device=dev)
    dmp = torch.zeros(gb.npix, spp, 10, device=dev) if dump else None
    opts = make_mis_opts(split, seed, job, t_min, 1e-3, 12, dmp)
    va = grt_vertex_attrs(_ptr(albedo), _ptr(rough), _ptr(metal), _ptr(normal))
    need = grt_render_workspace_bytes(gb.npix, spp)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    _check(load_library().grt_render_relight_mesh(mesh.handle, env.handle, C.byref(va), C.byref(gb.struct()),
                                                  C.byref(opts), _ptr(out), _ptr(workspace), workspace.numel(),
                                                  _stream(stream)))
    res = dict(rgb=out)
    if dump:
        res["dump"] = dmp
    return res


def denoise(ctx: Context, rgb, depth, normal, valid, H: int, W: int, radius=3, sigma_s=2.0, sigma_d=1.0,
            sigma_n=128.0, eps_d=1e-2, stream=None):
    """Cross-bilateral denoiser (Sec. 3.4.2): rgb [H*W,3] guided by depth
    [H*W], normal [H*W,3] and valid [H*W] (uint8); returns the filtered image."""
    dev = rgb.device
    for a in (rgb, depth, normal, valid):
        assert a.is_contiguous() and a.device == dev
    out = torch.empty(H * W, 3, device=dev)
    o = grt_denoise_opts(int(radius), float(sigma_s), float(sigma_d), float(sigma_n), float(eps_d))
    _check(load_library().grt_denoise(ctx.handle, H, W, _ptr(rgb), _ptr(depth), _ptr(normal), _ptr(valid),
                                      C.byref(o), _ptr(out), _stream(stream)))
    return out


def render_mis_backward(scene: Scene, env: Env, gb: GBuffer, grad_rgb, saved, split=(16, 8, 8), seed=0, job=0,
                        t_min=1e-3, t_cut=1e-3, k=16, grads=None, stream=None, hits=None, hit_cap=0, timer=None):
    """Gradients into `grads` (+=).  With `hits` (the forward's stored hit
    lists) the backward works from the lists instead of re-traversing."""
    if grads is None:
        grads = zero_grads(scene.n, gb.x.device)
    opts = make_mis_opts(split, seed, job, t_min, t_cut, k, None, hits, hit_cap, timer)
    ws = _workspace(grt_render_workspace_bytes(gb.npix, sum(split)), gb.x.device)
    grt_render_mis_backward(scene.handle, env.handle, gb.struct(), opts, grad_rgb.contiguous(), saved,
                            _grads_struct(grads), ws, stream)
    return grads


SHADING_KEYS = ("x", "n", "wo", "albedo", "rough", "metal")


def render_mis_backward_shading(scene: Scene, env: Env, gb: GBuffer, grad_rgb, saved, split=(16, 8, 8), seed=0,
                                job=0, t_min=1e-3, t_cut=1e-3, k=16, grads=None, stream=None, hits=None, hit_cap=0):
    """render_mis_backward plus the gradients with respect to the shading
    state (each sample's direction and pdf held fixed): returns (grads,
    shade) with shade = {x, n, wo, albedo [npix,3], rough, metal [npix]}."""
    dev = gb.x.device
    if grads is None:
        grads = zero_grads(scene.n, dev)
    shade = {key: torch.empty((gb.npix, 3) if key not in ("rough", "metal") else (gb.npix,), device=dev)
             for key in SHADING_KEYS}
    opts = make_mis_opts(split, seed, job, t_min, t_cut, k, None, hits, hit_cap)
    ws = _workspace(grt_render_workspace_bytes(gb.npix, sum(split)), dev)
    grt_render_mis_backward_shading(scene.handle, env.handle, gb.struct(), opts, grad_rgb.contiguous(), saved,
                                    _grads_struct(grads), grt_shading_grads(*(_ptr(shade[key]) for key in SHADING_KEYS)),
                                    ws, stream)
    return grads, shade


# --------------------------------------------------------------------------
# Autograd (Sec. 3.2: gradients backpropagate through the secondary rays)
# --------------------------------------------------------------------------

class TraceFn(torch.autograd.Function):
    """(c_rt, T) = Trace(origins, dirs) as a function of the surfel parameters."""

    @staticmethod
    def forward(ctx_, means, scales, quats, opacity, rgb, origins, dirs, gctx, t_min, k, t_cut, alpha_min):
        scene = Scene(gctx, means.detach().contiguous(), scales.detach().contiguous(), quats.detach().contiguous(),
                      opacity.detach().contiguous(), rgb.detach().contiguous(), alpha_min)
        out = trace(scene, origins, dirs, t_min=t_min, k=k, t_cut=t_cut, save_stop=True)
        ctx_.scene = scene
        ctx_.cfg = (t_min, k, t_cut)
        ctx_.save_for_backward(origins, dirs, out["rgb"], out["T"], out["stop"])
        return out["rgb"], out["T"]

    @staticmethod
    def backward(ctx_, g_rgb, g_T):
        origins, dirs, rgb, T, stop = ctx_.saved_tensors
        t_min, k, t_cut = ctx_.cfg
        g = trace_backward(ctx_.scene, origins, dirs, rgb, T,
                           torch.zeros_like(rgb) if g_rgb is None else g_rgb,
                           None if g_T is None else g_T, t_min=t_min, k=k, t_cut=t_cut, stop=stop)
        return g["means"], g["scales"], g["quats"], g["opacity"], g["rgb"], None, None, None, None, None, None, None


class RenderMISFn(torch.autograd.Function):
    """c_pbr image as a function of the surfel parameters (Eq. mis)."""

    @staticmethod
    def forward(ctx_, means, scales, quats, opacity, rgb, gctx, env, gb, split, seed, k, alpha_min, hit_cap=0,
                k_bwd=None, timers=None):
        """hit_cap > 0: store up to hit_cap hits per sample in the forward and
        differentiate from the stored lists; 0: re-traverse in the backward.
        k_bwd: k-buffer size of the backward (default k, at most 13: the
        backward's register budget; results do not depend on either).
        timers: optional (forward, backward) Timer pair that records the
        trace kernels of the two passes."""
        scene = Scene(gctx, means.detach().contiguous(), scales.detach().contiguous(), quats.detach().contiguous(),
                      opacity.detach().contiguous(), rgb.detach().contiguous(), alpha_min)
        hits = make_hit_list(gb.npix, sum(split), hit_cap, gb.x.device) if hit_cap > 0 else None
        tf, tb = timers if timers is not None else (None, None)
        res = render_mis(scene, env, gb, split=split, seed=seed, k=k, save=True, hits=hits, hit_cap=hit_cap, timer=tf)
        if k_bwd is None:
            k_bwd = min(k, 13)
        ctx_.scene, ctx_.env, ctx_.gb, ctx_.cfg = scene, env, gb, (split, seed, k_bwd, hit_cap)
        ctx_.saved_state, ctx_.hits, ctx_.timer = res["saved"], hits, tb
        return res["rgb"]

    @staticmethod
    def backward(ctx_, g_rgb):
        split, seed, k, hit_cap = ctx_.cfg
        g = render_mis_backward(ctx_.scene, ctx_.env, ctx_.gb, g_rgb, ctx_.saved_state, split=split, seed=seed, k=k,
                                hits=ctx_.hits, hit_cap=hit_cap, timer=ctx_.timer)
        return (g["means"], g["scales"], g["quats"], g["opacity"], g["rgb"], None, None, None, None, None, None, None,
                None, None, None)


class RenderMISShadedFn(torch.autograd.Function):
    """c_pbr image as a function of the surfel parameters and of the shading
    state (x, n, wo, albedo, rough, metal), e.g. the maps GBufferFn returns,
    so that a loss on the render reaches the surfels both through the
    secondary rays and through the primary G-buffer.  Each sample's direction
    and mixture pdf are held fixed in the backward."""

    @staticmethod
    def forward(ctx_, means, scales, quats, opacity, rgb, x, n, wo, albedo, rough, metal, valid, gctx, env, H, W,
                split, seed, k, alpha_min, hit_cap=0):
        scene = Scene(gctx, means.detach().contiguous(), scales.detach().contiguous(), quats.detach().contiguous(),
                      opacity.detach().contiguous(), rgb.detach().contiguous(), alpha_min)
        gb = GBuffer(H, W, *(t.detach().contiguous() for t in (x, n, wo, albedo, rough, metal)), valid.contiguous())
        hits = make_hit_list(gb.npix, sum(split), hit_cap, gb.x.device) if hit_cap > 0 else None
        res = render_mis(scene, env, gb, split=split, seed=seed, k=k, save=True, hits=hits, hit_cap=hit_cap)
        # the backward's k: at most 12 (its register budget)
        ctx_.scene, ctx_.env, ctx_.gb, ctx_.cfg = scene, env, gb, (split, seed, min(k, 12), hit_cap)
        ctx_.saved_state, ctx_.hits = res["saved"], hits
        return res["rgb"]

    @staticmethod
    def backward(ctx_, g_rgb):
        split, seed, k, hit_cap = ctx_.cfg
        kw = dict(split=split, seed=seed, k=k, hits=ctx_.hits, hit_cap=hit_cap)
        if any(ctx_.needs_input_grad[5:11]):
            g, sh = render_mis_backward_shading(ctx_.scene, ctx_.env, ctx_.gb, g_rgb, ctx_.saved_state, **kw)
            gs = tuple(sh[key] for key in SHADING_KEYS)
        else:
            g = render_mis_backward(ctx_.scene, ctx_.env, ctx_.gb, g_rgb, ctx_.saved_state, **kw)
            gs = (None,) * 6
        return (g["means"], g["scales"], g["quats"], g["opacity"], g["rgb"]) + gs + (None,) * 10


class GBufferFn(torch.autograd.Function):
    """The primary-ray G-buffer's deferred maps (Eq. deferred_maps on traced
    camera rays) as functions of the surfel parameters and their attributes:
    returns (x, n, albedo, rough, metal, depth, rgb, valid); valid is not
    differentiable, and wo (= -d) is left out."""

    @staticmethod
    def forward(ctx_, means, scales, quats, opacity, rgb, albedo, rough, metal, gctx, origins, dirs, H, W,
                min_opacity=0.5, k=12, alpha_min=1.0 / 255.0):
        scene = Scene(gctx, means.detach().contiguous(), scales.detach().contiguous(), quats.detach().contiguous(),
                      opacity.detach().contiguous(), rgb.detach().contiguous(), alpha_min)
        mats = [a.detach().contiguous() for a in (albedo, rough, metal)]
        fwd = trace_gbuffer(scene, *mats, origins, dirs, H, W, min_opacity=min_opacity, k=k)
        ctx_.scene, ctx_.mats, ctx_.fwd, ctx_.rays, ctx_.k = scene, mats, fwd, (origins, dirs), k
        ctx_.mark_non_differentiable(fwd["valid"])
        ctx_.set_materialize_grads(False)
        return tuple(fwd[key] for key in GBUFFER_GRAD_KEYS) + (fwd["valid"],)

    @staticmethod
    def backward(ctx_, *grads):
        grad = {key: g for key, g in zip(GBUFFER_GRAD_KEYS, grads[:len(GBUFFER_GRAD_KEYS)])}
        gs, ga = trace_gbuffer_backward(ctx_.scene, *ctx_.mats, *ctx_.rays, ctx_.fwd, grad, k=ctx_.k)
        return ((gs["means"], gs["scales"], gs["quats"], gs["opacity"], gs["rgb"], ga["albedo"], ga["rough"],
                 ga["metal"]) + (None,) * 8)


# --------------------------------------------------------------------------
# Relighting server
# --------------------------------------------------------------------------

def grt_server_create(ctx, scene, opts: grt_server_opts):
    out = VP()
    _check(load_library().grt_server_create(ctx, scene, C.byref(opts), C.byref(out)))
    return out


def grt_server_submit(server, job: grt_job) -> int:
    jid = C.c_uint64()
    _check(load_library().grt_server_submit(server, C.byref(job), C.byref(jid)))
    return jid.value


def grt_server_poll(server, jid: int) -> int:
    st = C.c_int()
    _check(load_library().grt_server_poll(server, jid, C.byref(st)))
    return st.value


def grt_server_wait(server, jid: int, timeout_s: float) -> int:
    return load_library().grt_server_wait(server, jid, timeout_s)


def grt_server_cancel(server, jid: int):
    _check(load_library().grt_server_cancel(server, jid))


def grt_server_job_times(server, jid: int):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(load_library().grt_server_job_times(server, jid, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def grt_server_stats(server):
    e, st, r, f = C.c_uint64(), C.c_uint64(), C.c_int64(), C.c_size_t()
    _check(load_library().grt_server_stats(server, C.byref(e), C.byref(st), C.byref(r), C.byref(f)))
    return dict(epochs=e.value, stopped=st.value, rays=r.value, pool_free=f.value)


def grt_server_destroy(server):
    _check(load_library().grt_server_destroy(server))


def grt_server_job_bytes(job: grt_job) -> int:
    return int(load_library().grt_server_job_bytes(C.byref(job)))


def grt_server_workspace_bytes(opts: grt_server_opts) -> int:
    return int(load_library().grt_server_workspace_bytes(C.byref(opts)))


class Request:
    """A relighting request, kept alive until the server is done with it.
    Inputs are host tensors (pinned when ``pin``) or, given as device
    tensors, used in place.  ``gb`` is a G-buffer, or ``camera`` (a
    grt_camera, with H and W) asks the server to trace the G-buffer itself,
    coverage at ``min_opacity``.  ``relight``: split-sum relighting of the
    server's surfel materials (Eq. relight_splitsum) instead of the radiance
    estimator.  ``out_device``: the image is written to a device tensor."""

    def __init__(self, gb, env_rgb, split=(16, 8, 8), seed=0, job=0, pin=True, camera=None, H=None, W=None,
                 min_opacity=0.5, relight=False, out_device=None):
        def host(a):
            t = torch.from_numpy(a) if not isinstance(a, torch.Tensor) else a
            t = t.contiguous()
            return t.pin_memory() if pin and not t.is_cuda else t
        self.env = host(env_rgb)
        if camera is None:
            self.arrays = [host(a) for a in (gb.x, gb.n, gb.wo, gb.albedo, gb.rough, gb.metal, gb.valid)]
            self.H, self.W = int(gb.H), int(gb.W)
        else:
            self.arrays = [None] * 7
            self.H, self.W = int(H), int(W)
        if out_device is not None:
            self.out = torch.zeros(self.H * self.W, 3, device=out_device)
        else:
            self.out = torch.zeros(self.H * self.W, 3)
            if pin:
                self.out = self.out.pin_memory()
        x, n, wo, alb, rough, metal, valid = self.arrays
        self.struct = grt_job(self.H, self.W, _ptr(x), _ptr(n), _ptr(wo), _ptr(alb), _ptr(rough), _ptr(metal),
                              _ptr(valid), _ptr(self.env), int(self.env.shape[0]), int(self.env.shape[1]),
                              split[0], split[1], split[2], seed, job, _ptr(self.out))
        if camera is not None:
            self.struct.camera_request = 1
            self.struct.camera = camera
            self.struct.min_opacity = float(min_opacity)
        self.struct.relight = 1 if relight else 0
        self.rays = self.H * self.W * sum(split)


class Server:
    """Owns a grt_server over a built scene; submit Requests, wait, read times."""

    def __init__(self, ctx: Context, scene: Scene, mem_budget: int, max_jobs: int = 16, epoch_rays: int = 0, k=8,
                 t_min=1e-3, t_cut=1e-3, slack_per_ray=-1.0, preempt_share=-1.0, attrs=None, co_trace=False,
                 k_relight=12):
        """attrs: (albedo, rough, metal) device tensors for camera and
        relighting requests, kept alive with the server.  The server's device
        memory (pool and tables) is a torch tensor owned here.  co_trace:
        trace waiting requests that share a G-buffer in one joint order (off
        by default: it holds the earliest request until the whole group is
        done, and did not raise throughput on the relighting mix).
        k_relight: k-buffer size of relighting epochs (k for radiance)."""
        self.ctx, self.scene = ctx, scene
        self.attrs = attrs
        at = grt_surfel_attrs(*(_ptr(a) for a in attrs)) if attrs is not None else grt_surfel_attrs()
        self.opts = grt_server_opts(int(mem_budget), int(max_jobs), int(epoch_rays), int(k), float(t_min),
                                    float(t_cut), float(slack_per_ray), float(preempt_share), at)
        need = grt_server_workspace_bytes(self.opts)
        if need == 0:
            raise GrtError(ERR_INVALID, "bad server options")
        self.workspace = _workspace(need, ctx.device)
        self.opts.workspace = _ptr(self.workspace)
        self.opts.ws_bytes = self.workspace.numel()
        self.opts.co_trace = 1 if co_trace else 0
        self.opts.k_relight = int(k_relight)
        self.handle = grt_server_create(ctx.handle, scene.handle, self.opts)
        self.requests = {}

    def submit(self, req: Request) -> int:
        jid = grt_server_submit(self.handle, req.struct)
        self.requests[jid] = req
        return jid

    def wait(self, jid: int, timeout_s: float = 120.0) -> int:
        return grt_server_wait(self.handle, jid, timeout_s)

    def poll(self, jid: int) -> int:
        return grt_server_poll(self.handle, jid)

    def cancel(self, jid: int):
        grt_server_cancel(self.handle, jid)

    def times(self, jid: int):
        return grt_server_job_times(self.handle, jid)

    def stats(self):
        return grt_server_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            grt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.grt_server_destroy(self.handle)
            self.handle = None
