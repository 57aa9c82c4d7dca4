// api.hip -- the extern "C" entry points of libgrt: argument checks, handle
// bookkeeping and kernel dispatch.  No exception or abort crosses the ABI.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "grt_internal.h"

// Scratch of grt_render_mis_noalloc (ray-fetch counters, per-sample ray
// records, contributions and sort buffers): a file-scope device array, so
// that call allocates nothing.  Every device the library runs on holds its
// own copy until the process ends.  Host code never uses this name as a
// device address: grt_ctx_create looks each device's copy up once with
// hipGetSymbolAddress and keeps that address in the context.
static __device__ __align__(256) unsigned char scratch[GRT_NOALLOC_SCRATCH_BYTES];

namespace {
// device address of `scratch` per device, looked up once per device
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};
}  // namespace

// A kernel timer: events recorded around a call's persistent trace kernels.
struct grt_timer {
    grt_ctx *ctx;
    grt::KernelTimer ev;
    bool recorded = false;
};

static const grt::KernelTimer *use_timer(const grt_mis_opts *o)
{
    if (!o || !o->timer) return nullptr;
    o->timer->recorded = true;
    return &o->timer->ev;
}

struct grt_scene {
    grt_ctx *ctx;
    grt_surfels s;
    float alpha_min;
    void *ws;
    size_t ws_bytes;
    grt::SceneWS w;
    bool built;
};

struct grt_mesh {
    grt_ctx *ctx;
    grt_mesh_desc m;
    grt::MeshWS w;
    bool built;
};

struct grt_env {
    grt_ctx *ctx;
    const float *rgb;
    int H, W;
    grt::EnvWS w;
    bool built;
    bool prefiltered;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(GRT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

grt::SceneDev scene_dev(const grt_scene *s)
{
    grt::SceneDev d;
    d.rec = s->w.rec;
    d.col = s->w.col;
    d.nodes = s->w.nodes;
    d.quat = s->w.quat;
    d.nodes4 = s->w.nodes4;
    d.n = (int32_t)s->s.n;
    return d;
}

int check_rays(const grt_rays *r)
{
    if (!r) return fail(GRT_ERR_INVALID, "rays is NULL");
    if (r->n < 0 || r->n > (int64_t)1 << 40) return fail(GRT_ERR_INVALID, "ray count %lld out of range", (long long)r->n);
    if (r->n > 0 && (!r->origins || !r->dirs)) return fail(GRT_ERR_INVALID, "ray origins/dirs NULL");
    if (!r->t_min && !(r->t_min_all >= 0.0f)) return fail(GRT_ERR_INVALID, "t_min must be >= 0");
    if (!r->t_min && !r->t_max && !(r->t_max_all > r->t_min_all))
        return fail(GRT_ERR_INVALID, "t_max must exceed t_min");
    return GRT_OK;
}

// backward: the MIS backward also takes 13 (the size that fits its register
// budget at 3 wavefronts per SIMD)
static int check_k(int k, bool backward = false)
{
    if (k == 1 || k == 2 || k == 4 || k == 8 || k == 12 || k == 16 || k == 32) return GRT_OK;
    if (backward && k == 13) return GRT_OK;
    return fail(GRT_ERR_INVALID, "k = %d is not one of 1,2,4,8,12,16,32%s", k, backward ? " (or 13)" : "");
}

int check_scene(const grt_scene *s)
{
    if (!s) return fail(GRT_ERR_INVALID, "scene is NULL");
    if (!s->built) return fail(GRT_ERR_NOT_BUILT, "scene used before grt_scene_build");
    return GRT_OK;
}

int check_grads(const grt_surfel_grads *g, int64_t n)
{
    if (!g) return fail(GRT_ERR_INVALID, "grads is NULL");
    if (n > 0 && (!g->means || !g->scales || !g->quats || !g->opacity || !g->rgb))
        return fail(GRT_ERR_INVALID, "a gradient accumulator is NULL");
    return GRT_OK;
}

grt::GradPtrs grad_ptrs(const grt_scene *s, const grt_surfel_grads *g)
{
    grt::GradPtrs p;
    p.means = g->means; p.scales = g->scales; p.quats = g->quats; p.opacity = g->opacity; p.rgb = g->rgb;
    p.order = nullptr;
    p.acc = s->w.acc;
    return p;
}

}  // namespace

namespace grt {
int scene_dev_of(const grt_scene *scene, SceneDev *out, const char **why)
{
    if (!scene->built) {
        *why = "scene used before grt_scene_build";
        return GRT_ERR_NOT_BUILT;
    }
    *out = scene_dev(scene);
    return GRT_OK;
}

int set_error(int code, const char *msg)
{
    return fail(code, "%s", msg);
}
}  // namespace grt

namespace {

int set_device(grt_ctx *c)
{
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return GRT_OK;
}

}  // namespace

extern "C" {

const char *grt_last_error(void) { return g_err; }

const char *grt_status_str(int status)
{
    switch (status) {
    case GRT_OK: return "GRT_OK";
    case GRT_ERR_INVALID: return "GRT_ERR_INVALID";
    case GRT_ERR_OOM: return "GRT_ERR_OOM";
    case GRT_ERR_NOT_BUILT: return "GRT_ERR_NOT_BUILT";
    case GRT_ERR_DEVICE: return "GRT_ERR_DEVICE";
    case GRT_ERR_ADMISSION: return "GRT_ERR_ADMISSION";
    case GRT_ERR_BUSY: return "GRT_ERR_BUSY";
    case GRT_ERR_CANCELLED: return "GRT_ERR_CANCELLED";
    case GRT_ERR_TIMEOUT: return "GRT_ERR_TIMEOUT";
    default: return "GRT_ERR_UNKNOWN";
    }
}

int grt_version(void) { return (1 << 16) | 0; }

int grt_ctx_create(int device, grt_ctx **out)
{
    if (!out) return fail(GRT_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(GRT_ERR_DEVICE, "device %d not present (%d devices)", device, count);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    void *scr = nullptr;
    if (device < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[device]) {
            int prev = 0;
            if ((e = hipGetDevice(&prev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
            if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            const hipError_t e2 = hipSetDevice(prev);
            if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
            if (e2 != hipSuccess) return hip_fail(e2, "hipSetDevice");
            g_scratch_dev[device] = p;
        }
        scr = g_scratch_dev[device];
    }
    grt_ctx *c = new (std::nothrow) grt_ctx;
    if (!c) return fail(GRT_ERR_OOM, "host allocation failed");
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->scratch = scr;
    *out = c;
    return GRT_OK;
}

int grt_ctx_destroy(grt_ctx *ctx)
{
    delete ctx;
    return GRT_OK;
}

int grt_timer_create(grt_ctx *ctx, grt_timer **out)
{
    if (!ctx || !out) return fail(GRT_ERR_INVALID, "ctx/out is NULL");
    *out = nullptr;
    int rc = set_device(ctx);
    if (rc) return rc;
    grt_timer *t = new (std::nothrow) grt_timer();
    if (!t) return fail(GRT_ERR_OOM, "timer");
    t->ctx = ctx;
    hipError_t e = hipEventCreate(&t->ev.begin);
    if (e == hipSuccess) {
        e = hipEventCreate(&t->ev.end);
        if (e != hipSuccess) (void)hipEventDestroy(t->ev.begin);
    }
    if (e != hipSuccess) {
        delete t;
        return hip_fail(e, "hipEventCreate");
    }
    *out = t;
    return GRT_OK;
}

int grt_timer_ms(grt_timer *t, float *ms)
{
    if (!t || !ms) return fail(GRT_ERR_INVALID, "timer/ms is NULL");
    if (!t->recorded) return fail(GRT_ERR_INVALID, "the timer has recorded nothing yet");
    int rc = set_device(t->ctx);
    if (rc) return rc;
    hipError_t e = hipEventSynchronize(t->ev.end);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, t->ev.begin, t->ev.end);
    if (e != hipSuccess) return hip_fail(e, "timer read");
    return GRT_OK;
}

int grt_timer_destroy(grt_timer *t)
{
    if (!t) return GRT_OK;
    (void)set_device(t->ctx);
    (void)hipEventDestroy(t->ev.begin);
    (void)hipEventDestroy(t->ev.end);
    delete t;
    return GRT_OK;
}

int grt_walk_stats(grt_ctx *ctx, uint64_t *out, int reset)
{
    if (!ctx || !out) return fail(GRT_ERR_INVALID, "ctx/out is NULL");
    if (!grt::walk_stats_built()) return fail(GRT_ERR_INVALID, "the library was built without walk statistics");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    static_assert(sizeof(uint64_t) == sizeof(unsigned long long), "64-bit sums");
    e = grt::walk_stats_read(reinterpret_cast<unsigned long long *>(out), reset != 0);
    if (e != hipSuccess) return hip_fail(e, "walk statistics");
    return GRT_OK;
}

size_t grt_scene_workspace_bytes(int64_t n)
{
    if (n < 0) return 0;
    return grt::carve_scene(nullptr, n).bytes;
}

static int check_surfels(const grt_surfels *s)
{
    if (!s) return fail(GRT_ERR_INVALID, "surfels is NULL");
    if (s->n < 0 || s->n > 0x7fffffff) return fail(GRT_ERR_INVALID, "surfel count %lld out of range", (long long)s->n);
    if (s->n > 0 && (!s->means || !s->scales || !s->quats || !s->opacity || !s->rgb))
        return fail(GRT_ERR_INVALID, "a surfel array is NULL");
    if (s->quats && !aligned(s->quats, 16)) return fail(GRT_ERR_INVALID, "quats must be 16-byte aligned");
    return GRT_OK;
}

int grt_scene_create(grt_ctx *ctx, const grt_surfels *surfels, float alpha_min, void *workspace, size_t ws_bytes,
                     grt_scene **out)
{
    if (!ctx || !out) return fail(GRT_ERR_INVALID, "ctx/out is NULL");
    *out = nullptr;
    int rc = check_surfels(surfels);
    if (rc) return rc;
    if (!(alpha_min >= 0.0f && alpha_min < 1.0f)) return fail(GRT_ERR_INVALID, "alpha_min must be in [0,1)");
    size_t need = grt_scene_workspace_bytes(surfels->n);
    if (!workspace || ws_bytes < need)
        return fail(GRT_ERR_OOM, "scene workspace of %zu bytes < %zu needed", ws_bytes, need);
    if (!aligned(workspace, 256)) return fail(GRT_ERR_INVALID, "workspace must be 256-byte aligned");
    grt_scene *s = new (std::nothrow) grt_scene;
    if (!s) return fail(GRT_ERR_OOM, "host allocation failed");
    s->ctx = ctx;
    s->s = *surfels;
    s->alpha_min = alpha_min;
    s->ws = workspace;
    s->ws_bytes = ws_bytes;
    s->w = grt::carve_scene(workspace, surfels->n);
    s->built = false;
    *out = s;
    return GRT_OK;
}

int grt_scene_set_surfels(grt_scene *scene, const grt_surfels *surfels)
{
    if (!scene) return fail(GRT_ERR_INVALID, "scene is NULL");
    int rc = check_surfels(surfels);
    if (rc) return rc;
    if (surfels->n != scene->s.n) return fail(GRT_ERR_INVALID, "surfel count changed (%lld -> %lld)",
                                              (long long)scene->s.n, (long long)surfels->n);
    scene->s = *surfels;
    scene->built = false;
    return GRT_OK;
}

int grt_scene_build(grt_scene *scene, void *stream)
{
    if (!scene) return fail(GRT_ERR_INVALID, "scene is NULL");
    int rc = set_device(scene->ctx);
    if (rc) return rc;
    hipError_t e = grt::launch_scene_build(scene->s, scene->alpha_min, scene->w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "scene build launch");
    scene->built = true;
    return GRT_OK;
}

int grt_scene_destroy(grt_scene *scene)
{
    delete scene;
    return GRT_OK;
}

int grt_scene_view_get(const grt_scene *scene, grt_scene_view *out)
{
    if (!scene || !out) return fail(GRT_ERR_INVALID, "scene/out is NULL");
    out->n = scene->s.n;
    out->records = reinterpret_cast<const float *>(scene->w.rec);
    out->nodes = reinterpret_cast<const float *>(scene->w.nodes);
    out->order = reinterpret_cast<const int32_t *>(scene->w.vals0);
    out->leaf_boxes = scene->w.leaf_box;
    out->colours = reinterpret_cast<const float *>(scene->w.col);
    out->quats = reinterpret_cast<const float *>(scene->w.quat);
    out->nodes4 = reinterpret_cast<const float *>(scene->w.nodes4);
    out->nodes4_count = scene->w.ctl4 + 2;
    return GRT_OK;
}

static int fill_trace_args(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                           grt::TraceArgs &a)
{
    int rc = check_scene(scene);
    if (rc) return rc;
    if ((rc = check_rays(rays))) return rc;
    if (!opts) return fail(GRT_ERR_INVALID, "opts is NULL");
    if ((rc = check_k(opts->k))) return rc;
    if (!(opts->t_cut >= 0.0f && opts->t_cut < 1.0f)) return fail(GRT_ERR_INVALID, "t_cut must be in [0,1)");
    memset(&a, 0, sizeof(a));
    a.S = scene_dev(scene);
    a.n = rays->n;
    a.o = rays->origins; a.d = rays->dirs;
    a.tmin_a = rays->t_min; a.tmax_a = rays->t_max;
    a.tmin = rays->t_min_all; a.tmax = rays->t_max_all;
    a.tcut = opts->t_cut;
    for (int c = 0; c < 3; ++c) a.sky[c] = opts->sky[c];
    a.stop_depth = opts->stop_depth;
    if (opts->env) {
        if (!opts->env->built) return fail(GRT_ERR_NOT_BUILT, "trace environment used before grt_env_build");
        a.env_rgb = opts->env->rgb;
        a.env_H = opts->env->H;
        a.env_W = opts->env->W;
    }
    return GRT_OK;
}

size_t grt_trace_workspace_bytes(int64_t nrays)
{
    (void)nrays;
    return grt::kCounterBytes;
}

static int check_ws(void *ws, size_t bytes, size_t need, const char *what)
{
    if (!ws || bytes < need) return fail(GRT_ERR_OOM, "%s workspace of %zu bytes < %zu needed", what, bytes, need);
    if (!aligned(ws, 256)) return fail(GRT_ERR_INVALID, "%s workspace must be 256-byte aligned", what);
    return GRT_OK;
}

int grt_trace(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts, float *out_rgb, float *out_T,
              float *out_L, int32_t *out_nhit, void *workspace, size_t ws_bytes, void *stream)
{
    grt::TraceArgs a;
    int rc = fill_trace_args(scene, rays, opts, a);
    if (rc) return rc;
    if (rays->n > 0 && (!out_rgb || !out_T)) return fail(GRT_ERR_INVALID, "out_rgb/out_T is NULL");
    if (opts->hit_ids && (!opts->hit_tau || opts->hit_cap <= 0))
        return fail(GRT_ERR_INVALID, "hit dump needs hit_tau and hit_cap > 0");
    a.out_rgb = out_rgb; a.out_T = out_T; a.out_L = out_L; a.out_nhit = out_nhit;
    a.dump_id = opts->hit_ids; a.dump_tau = opts->hit_tau; a.cap = opts->hit_ids ? opts->hit_cap : 0;
    if ((rc = check_ws(workspace, ws_bytes, grt_trace_workspace_bytes(rays->n), "trace"))) return rc;
    a.counters = (unsigned long long *)workspace;
    if ((rc = set_device(scene->ctx))) return rc;
    hipError_t e = grt::launch_trace(a, opts->k, scene->ctx->num_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "trace launch");
    return GRT_OK;
}

int grt_trace_attr(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                   const grt_surfel_attrs *attrs, float *out_V, float *out_albedo, float *out_rough, float *out_metal,
                   float *out_normal, void *workspace, size_t ws_bytes, void *stream)
{
    grt::TraceAttrArgs b;
    int rc = fill_trace_args(scene, rays, opts, b.f);
    if (rc) return rc;
    if (!attrs) return fail(GRT_ERR_INVALID, "attrs is NULL");
    if (scene->s.n > 0 && (!attrs->albedo || !attrs->rough || !attrs->metal))
        return fail(GRT_ERR_INVALID, "an attribute array is NULL");
    if (rays->n > 0 && (!out_V || !out_albedo || !out_rough || !out_metal || !out_normal))
        return fail(GRT_ERR_INVALID, "an output array is NULL");
    b.albedo = attrs->albedo; b.rough = attrs->rough; b.metal = attrs->metal;
    b.out_V = out_V; b.out_albedo = out_albedo; b.out_rough = out_rough; b.out_metal = out_metal;
    b.out_normal = out_normal;
    if ((rc = check_ws(workspace, ws_bytes, grt_trace_workspace_bytes(rays->n), "trace_attr"))) return rc;
    b.f.counters = (unsigned long long *)workspace;
    if ((rc = set_device(scene->ctx))) return rc;
    hipError_t e = grt::launch_trace_attr(b, opts->k, scene->ctx->num_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "trace_attr launch");
    return GRT_OK;
}

int grt_trace_gbuffer(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                      const grt_surfel_attrs *attrs, float min_opacity, grt_gbuffer_out *out, void *workspace,
                      size_t ws_bytes, void *stream)
{
    grt::TraceGBufArgs b;
    int rc = fill_trace_args(scene, rays, opts, b.f);
    if (rc) return rc;
    if (!attrs || !out) return fail(GRT_ERR_INVALID, "attrs/out is NULL");
    if (scene->s.n > 0 && (!attrs->albedo || !attrs->rough || !attrs->metal))
        return fail(GRT_ERR_INVALID, "an attribute array is NULL");
    if (rays->n > 0 && (!out->x || !out->n || !out->wo || !out->albedo || !out->rough || !out->metal ||
                        !out->depth || !out->rgb || !out->valid))
        return fail(GRT_ERR_INVALID, "an output array is NULL");
    if (!(min_opacity > 0.0f && min_opacity <= 1.0f)) return fail(GRT_ERR_INVALID, "min_opacity must be in (0,1]");
    b.albedo = attrs->albedo; b.rough = attrs->rough; b.metal = attrs->metal;
    b.min_opacity = min_opacity;
    b.x = out->x; b.n = out->n; b.wo = out->wo; b.out_albedo = out->albedo; b.out_rough = out->rough;
    b.out_metal = out->metal; b.depth = out->depth; b.rgb = out->rgb; b.valid = out->valid;
    b.weight = out->weight; b.nlen = out->nlen;
    if ((rc = check_ws(workspace, ws_bytes, grt_trace_workspace_bytes(rays->n), "trace_gbuffer"))) return rc;
    b.f.counters = (unsigned long long *)workspace;
    if ((rc = set_device(scene->ctx))) return rc;
    hipError_t e = grt::launch_trace_gbuffer(b, opts->k, scene->ctx->num_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "trace_gbuffer launch");
    return GRT_OK;
}

int grt_trace_gbuffer_backward(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                               const grt_surfel_attrs *attrs, const grt_gbuffer_out *fwd,
                               const grt_gbuffer_grad *grad, grt_surfel_grads *grads, grt_attr_grads *agrads,
                               void *workspace, size_t ws_bytes, void *stream)
{
    grt::TraceGBufBwdArgs b;
    int rc = fill_trace_args(scene, rays, opts, b.f);
    if (rc) return rc;
    if (!attrs || !fwd || !grad) return fail(GRT_ERR_INVALID, "attrs/fwd/grad is NULL");
    if (scene->s.n > 0 && (!attrs->albedo || !attrs->rough || !attrs->metal))
        return fail(GRT_ERR_INVALID, "an attribute array is NULL");
    if (rays->n > 0 && (!fwd->n || !fwd->albedo || !fwd->rough || !fwd->metal || !fwd->depth || !fwd->rgb ||
                        !fwd->valid || !fwd->weight || !fwd->nlen))
        return fail(GRT_ERR_INVALID, "a forward map (n, albedo, rough, metal, depth, rgb, valid, weight, nlen) is NULL");
    if ((rc = check_grads(grads, scene->s.n))) return rc;
    b.albedo = attrs->albedo; b.rough = attrs->rough; b.metal = attrs->metal;
    b.fwd_n = fwd->n; b.fwd_albedo = fwd->albedo; b.fwd_rough = fwd->rough; b.fwd_metal = fwd->metal;
    b.fwd_depth = fwd->depth; b.fwd_rgb = fwd->rgb; b.fwd_weight = fwd->weight; b.fwd_nlen = fwd->nlen;
    b.fwd_valid = fwd->valid;
    b.g_x = grad->x; b.g_n = grad->n; b.g_albedo = grad->albedo; b.g_rough = grad->rough; b.g_metal = grad->metal;
    b.g_depth = grad->depth; b.g_rgb = grad->rgb;
    b.g = grad_ptrs(scene, grads);
    b.ga_albedo = agrads ? agrads->albedo : nullptr;
    b.ga_rough = agrads ? agrads->rough : nullptr;
    b.ga_metal = agrads ? agrads->metal : nullptr;
    if ((rc = check_ws(workspace, ws_bytes, grt_trace_workspace_bytes(rays->n), "trace_gbuffer backward"))) return rc;
    b.f.counters = (unsigned long long *)workspace;
    if ((rc = set_device(scene->ctx))) return rc;
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = grt::launch_grad_lines_zero(b.g.acc, scene->s.n, st);
    if (e == hipSuccess) e = grt::launch_trace_gbuffer_backward(b, opts->k, scene->ctx->num_cu, st);
    if (e == hipSuccess) e = grt::launch_grad_lines_apply(b.g, scene->s.n, st);
    if (e != hipSuccess) return hip_fail(e, "trace_gbuffer backward launch");
    return GRT_OK;
}

int grt_trace_backward(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts, const float *fwd_rgb,
                       const float *fwd_T, const float *grad_rgb, const float *grad_T, grt_surfel_grads *grads,
                       void *workspace, size_t ws_bytes, void *stream)
{
    grt::TraceBwdArgs b;
    int rc = fill_trace_args(scene, rays, opts, b.f);
    if (rc) return rc;
    if (rays->n > 0 && (!fwd_rgb || !fwd_T || !grad_rgb)) return fail(GRT_ERR_INVALID, "fwd_rgb/fwd_T/grad_rgb NULL");
    if ((rc = check_grads(grads, scene->s.n))) return rc;
    b.fwd_rgb = fwd_rgb; b.fwd_T = fwd_T; b.grad_rgb = grad_rgb; b.grad_T = grad_T;
    b.g = grad_ptrs(scene, grads);
    if ((rc = check_ws(workspace, ws_bytes, grt_trace_workspace_bytes(rays->n), "trace backward"))) return rc;
    b.f.counters = (unsigned long long *)workspace;
    if ((rc = set_device(scene->ctx))) return rc;
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = grt::launch_grad_lines_zero(b.g.acc, scene->s.n, st);
    if (e == hipSuccess) e = grt::launch_trace_backward(b, opts->k, scene->ctx->num_cu, st);
    if (e == hipSuccess) e = grt::launch_grad_lines_apply(b.g, scene->s.n, st);
    if (e != hipSuccess) return hip_fail(e, "trace backward launch");
    return GRT_OK;
}

size_t grt_env_workspace_bytes(int H, int W)
{
    if (H <= 0 || W <= 0) return 0;
    return grt::carve_env(nullptr, H, W).bytes;
}

int grt_env_create(grt_ctx *ctx, const float *rgb, int H, int W, void *workspace, size_t ws_bytes, grt_env **out)
{
    if (!ctx || !out) return fail(GRT_ERR_INVALID, "ctx/out is NULL");
    *out = nullptr;
    if (H <= 0 || W <= 0 || (int64_t)H * W > ((int64_t)1 << 28)) return fail(GRT_ERR_INVALID, "bad env size %dx%d", H, W);
    if (!rgb) return fail(GRT_ERR_INVALID, "env rgb is NULL");
    size_t need = grt_env_workspace_bytes(H, W);
    if (!workspace || ws_bytes < need) return fail(GRT_ERR_OOM, "env workspace of %zu bytes < %zu needed", ws_bytes, need);
    if (!aligned(workspace, 256)) return fail(GRT_ERR_INVALID, "workspace must be 256-byte aligned");
    grt_env *e = new (std::nothrow) grt_env;
    if (!e) return fail(GRT_ERR_OOM, "host allocation failed");
    e->ctx = ctx;
    e->rgb = rgb;
    e->H = H; e->W = W;
    e->w = grt::carve_env(workspace, H, W);
    e->built = false;
    e->prefiltered = false;
    *out = e;
    return GRT_OK;
}

int grt_env_build(grt_env *env, void *stream)
{
    if (!env) return fail(GRT_ERR_INVALID, "env is NULL");
    int rc = set_device(env->ctx);
    if (rc) return rc;
    hipError_t e = grt::launch_env_build(env->rgb, env->H, env->W, env->w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "env build launch");
    env->built = true;
    return GRT_OK;
}

int grt_env_prefilter(grt_env *env, void *stream)
{
    if (!env) return fail(GRT_ERR_INVALID, "env is NULL");
    int rc = set_device(env->ctx);
    if (rc) return rc;
    hipError_t e = grt::launch_env_prefilter(env->rgb, env->H, env->W, env->w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "env prefilter launch");
    env->prefiltered = true;
    return GRT_OK;
}

int grt_env_relight_tables(const grt_env *env, const float **Ed, const float **Es, const float **lut)
{
    if (!env || !Ed || !Es || !lut) return fail(GRT_ERR_INVALID, "NULL argument");
    if (!env->prefiltered) return fail(GRT_ERR_NOT_BUILT, "environment not prefiltered");
    *Ed = env->w.Ed;
    *Es = env->w.Es;
    *lut = env->w.lut;
    return GRT_OK;
}

int grt_env_tables(const grt_env *env, const float **marg, const float **cond)
{
    if (!env || !marg || !cond) return fail(GRT_ERR_INVALID, "NULL argument");
    *marg = env->w.marg;
    *cond = env->w.cond;
    return GRT_OK;
}

int grt_env_destroy(grt_env *env)
{
    delete env;
    return GRT_OK;
}

size_t grt_render_saved_bytes(int64_t npix, int spp)
{
    if (npix < 0 || spp <= 0) return 0;
    return (size_t)npix * (size_t)spp * 20u;
}

size_t grt_render_hit_list_bytes(int64_t npix, int spp, int hit_cap)
{
    if (npix < 0 || spp <= 0 || hit_cap < 0) return 0;
    return (size_t)npix * (size_t)spp * 4u * (1u + (size_t)hit_cap);
}

size_t grt_render_workspace_bytes(int64_t npix, int spp)
{
    if (npix < 0 || spp <= 0) return 0;
    return grt::carve_render(nullptr, npix * spp).bytes;
}

static int fill_render_common(const grt_env *env, const grt_gbuffer *g, const grt_mis_opts *o, grt::RenderArgs &a,
                              bool backward = false);

static int fill_render_args(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g, const grt_mis_opts *o,
                            grt::RenderArgs &a, bool backward = false)
{
    int rc = check_scene(scene);
    if (rc) return rc;
    if ((rc = fill_render_common(env, g, o, a, backward))) return rc;
    a.S = scene_dev(scene);
    return GRT_OK;
}

// everything of a render but the scene (a.S left empty)
static int fill_render_common(const grt_env *env, const grt_gbuffer *g, const grt_mis_opts *o, grt::RenderArgs &a,
                              bool backward)
{
    int rc;
    if (!env) return fail(GRT_ERR_INVALID, "env is NULL");
    if (!env->built) return fail(GRT_ERR_NOT_BUILT, "environment used before grt_env_build");
    if (!g || !o) return fail(GRT_ERR_INVALID, "gbuffer/opts is NULL");
    if (g->H < 0 || g->W < 0 || (int64_t)g->H * g->W > 0x7fffffff) return fail(GRT_ERR_INVALID, "bad G-buffer size");
    if (o && (int64_t)g->H * g->W * ((int64_t)o->n_cos + o->n_ggx + o->n_env) > 0x7fffffff)
        return fail(GRT_ERR_INVALID, "more than 2^31 - 1 samples");
    if ((int64_t)g->H * g->W > 0 && (!g->x || !g->n || !g->wo || !g->albedo || !g->rough || !g->metal || !g->valid))
        return fail(GRT_ERR_INVALID, "a G-buffer array is NULL");
    if (o->n_cos < 0 || o->n_ggx < 0 || o->n_env < 0 || o->n_cos + o->n_ggx + o->n_env <= 0 ||
        o->n_cos + o->n_ggx + o->n_env > 65536)
        return fail(GRT_ERR_INVALID, "bad sample allocation %d/%d/%d", o->n_cos, o->n_ggx, o->n_env);
    if ((rc = check_k(o->k, backward))) return rc;
    if (!(o->t_min >= 0.0f)) return fail(GRT_ERR_INVALID, "t_min must be >= 0");
    if (!(o->t_cut >= 0.0f && o->t_cut < 1.0f)) return fail(GRT_ERR_INVALID, "t_cut must be in [0,1)");
    memset(&a, 0, sizeof(a));
    a.E.H = env->H; a.E.W = env->W; a.E.rgb = env->rgb; a.E.marg = env->w.marg; a.E.cond = env->w.cond;
    a.H = g->H; a.W = g->W;
    a.x = g->x; a.n = g->n; a.wo = g->wo; a.alb = g->albedo; a.rough = g->rough; a.metal = g->metal; a.valid = g->valid;
    a.nc = o->n_cos; a.ng = o->n_ggx; a.ne = o->n_env;
    a.seed = o->seed; a.job = o->job;
    a.tmin = o->t_min; a.tcut = o->t_cut;
    if (o->hit_list) {
        if (o->hit_cap < 0 || o->hit_cap > 65536) return fail(GRT_ERR_INVALID, "hit_cap must be in 0..65536");
        if (!aligned(o->hit_list, 4)) return fail(GRT_ERR_INVALID, "hit_list must be 4-byte aligned");
        a.hits = o->hit_list;
        a.hcap = o->hit_cap;
    }
    return GRT_OK;
}

size_t grt_mesh_workspace_bytes(int64_t nf)
{
    if (nf < 0) return 0;
    return grt::carve_mesh(nullptr, nf).bytes;
}

int grt_mesh_create(grt_ctx *ctx, const grt_mesh_desc *m, void *workspace, size_t ws_bytes, grt_mesh **out)
{
    if (!ctx || !m || !out) return fail(GRT_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (m->nv < 0 || m->nv > 0x7fffffff || m->nf < 0 || m->nf > (1 << 29))
        return fail(GRT_ERR_INVALID, "mesh size out of range (nv %lld, nf %lld)", (long long)m->nv, (long long)m->nf);
    if (m->nf > 0 && (!m->verts || !m->tris)) return fail(GRT_ERR_INVALID, "verts/tris is NULL");
    const size_t need = grt_mesh_workspace_bytes(m->nf);
    if (!workspace || ws_bytes < need) return fail(GRT_ERR_OOM, "mesh workspace of %zu bytes < %zu needed", ws_bytes, need);
    if (!aligned(workspace, 256)) return fail(GRT_ERR_INVALID, "workspace must be 256-byte aligned");
    grt_mesh *h = new (std::nothrow) grt_mesh;
    if (!h) return fail(GRT_ERR_OOM, "host allocation failed");
    h->ctx = ctx;
    h->m = *m;
    h->w = grt::carve_mesh(workspace, m->nf);
    h->built = false;
    *out = h;
    return GRT_OK;
}

int grt_mesh_build(grt_mesh *mesh, void *stream)
{
    if (!mesh) return fail(GRT_ERR_INVALID, "mesh is NULL");
    int rc = set_device(mesh->ctx);
    if (rc) return rc;
    hipError_t e = grt::launch_mesh_build((int)mesh->m.nv, mesh->m.verts, (int)mesh->m.nf, mesh->m.tris, mesh->w,
                                         (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mesh build launch");
    mesh->built = true;
    return GRT_OK;
}

int grt_mesh_trace_attr(const grt_mesh *mesh, const grt_rays *rays, const grt_vertex_attrs *attrs, float *out_V,
                        float *out_albedo, float *out_rough, float *out_metal, float *out_normal, void *stream)
{
    if (!mesh || !rays || !attrs) return fail(GRT_ERR_INVALID, "NULL argument");
    if (!mesh->built) return fail(GRT_ERR_NOT_BUILT, "mesh used before grt_mesh_build");
    int rc = check_rays(rays);
    if (rc) return rc;
    if (rays->t_min || rays->t_max) return fail(GRT_ERR_INVALID, "the mesh query takes scalar t_min/t_max only");
    if (mesh->m.nf > 0 && (!attrs->albedo || !attrs->rough || !attrs->metal || !attrs->normal))
        return fail(GRT_ERR_INVALID, "a vertex attribute array is NULL");
    if (rays->n > 0 && (!out_V || !out_albedo || !out_rough || !out_metal || !out_normal))
        return fail(GRT_ERR_INVALID, "an output array is NULL");
    grt::MeshTraceArgs a;
    a.n = rays->n;
    a.nv = (int)mesh->m.nv; a.nf = (int)mesh->m.nf;
    a.rec = mesh->w.rec; a.nodes = mesh->w.nodes; a.tris = mesh->m.tris;
    a.o = rays->origins; a.d = rays->dirs; a.tmin = rays->t_min_all; a.tmax = rays->t_max_all;
    a.albedo = attrs->albedo; a.rough = attrs->rough; a.metal = attrs->metal; a.vnormal = attrs->normal;
    a.out_V = out_V; a.out_albedo = out_albedo; a.out_rough = out_rough; a.out_metal = out_metal;
    a.out_normal = out_normal;
    if ((rc = set_device(mesh->ctx))) return rc;
    hipError_t e = grt::launch_mesh_trace_attr(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mesh trace launch");
    return GRT_OK;
}

int grt_mesh_destroy(grt_mesh *mesh)
{
    delete mesh;
    return GRT_OK;
}

int grt_camera_rays(grt_ctx *ctx, const grt_camera *cam, int H, int W, float *out_o, float *out_d, void *stream)
{
    if (!ctx || !cam || !out_o || !out_d) return fail(GRT_ERR_INVALID, "NULL argument");
    if (H <= 0 || W <= 0 || (int64_t)H * W > 0x7fffffff) return fail(GRT_ERR_INVALID, "bad image size %dx%d", H, W);
    grt::PinholeDev c;
    if (!grt::make_pinhole(cam->eye, cam->target, cam->up, cam->vfov_deg, H, W, c))
        return fail(GRT_ERR_INVALID, "degenerate camera");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipError_t e = grt::launch_camera_rays(c, H, W, out_o, out_d, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "camera rays launch");
    return GRT_OK;
}

int grt_denoise(grt_ctx *ctx, int H, int W, const float *rgb, const float *depth, const float *normal,
                const uint8_t *valid, const grt_denoise_opts *opts, float *out_rgb, void *stream)
{
    if (!ctx || !opts) return fail(GRT_ERR_INVALID, "ctx/opts is NULL");
    if (H < 0 || W < 0 || (int64_t)H * W > 0x7fffffff) return fail(GRT_ERR_INVALID, "bad image size %dx%d", H, W);
    if ((int64_t)H * W > 0 && (!rgb || !depth || !normal || !valid || !out_rgb))
        return fail(GRT_ERR_INVALID, "an image array is NULL");
    if (out_rgb && out_rgb == rgb) return fail(GRT_ERR_INVALID, "out_rgb must not alias rgb");
    if (opts->radius < 1 || opts->radius > grt::kDenoiseMaxRadius)
        return fail(GRT_ERR_INVALID, "radius must be in 1..%d", grt::kDenoiseMaxRadius);
    if (!(opts->sigma_s > 0.0f) || !(opts->sigma_d >= 0.0f) || !(opts->sigma_n >= 0.0f) || !(opts->eps_d > 0.0f))
        return fail(GRT_ERR_INVALID, "need sigma_s > 0, sigma_d >= 0, sigma_n >= 0, eps_d > 0");
    grt::DenoiseArgs a;
    a.H = H; a.W = W; a.radius = opts->radius;
    a.sigma_s = opts->sigma_s; a.sigma_d = opts->sigma_d; a.sigma_n = opts->sigma_n; a.eps_d = opts->eps_d;
    a.rgb = rgb; a.depth = depth; a.normal = normal; a.valid = valid; a.out = out_rgb;
    int rc = set_device(ctx);
    if (rc) return rc;
    hipError_t e = grt::launch_denoise(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "denoise launch");
    return GRT_OK;
}

int grt_render_relight(const grt_scene *scene, const grt_env *env, const grt_surfel_attrs *attrs,
                       const grt_gbuffer *g, const grt_mis_opts *opts, float *out_rgb, void *workspace, size_t ws_bytes,
                       void *stream)
{
    grt::RenderArgs a;
    int rc = fill_render_args(scene, env, g, opts, a);
    if (rc) return rc;
    if (!env->prefiltered) return fail(GRT_ERR_NOT_BUILT, "relighting needs grt_env_prefilter first");
    if (!attrs) return fail(GRT_ERR_INVALID, "attrs is NULL");
    if (scene->s.n > 0 && (!attrs->albedo || !attrs->rough || !attrs->metal))
        return fail(GRT_ERR_INVALID, "an attribute array is NULL");
    if ((int64_t)g->H * g->W > 0 && !out_rgb) return fail(GRT_ERR_INVALID, "out_rgb is NULL");
    if (opts->hit_list) return fail(GRT_ERR_INVALID, "relighting stores no hit lists");
    a.E.Ed = env->w.Ed; a.E.Es = env->w.Es; a.E.lut = env->w.lut;
    a.sa_albedo = attrs->albedo; a.sa_rough = attrs->rough; a.sa_metal = attrs->metal;
    a.out = out_rgb;
    a.dump = opts->sample_dump;
    const int spp = opts->n_cos + opts->n_ggx + opts->n_env;
    if ((rc = check_ws(workspace, ws_bytes, grt_render_workspace_bytes((int64_t)g->H * g->W, spp), "relight")))
        return rc;
    const grt::RenderWS w = grt::carve_render(workspace, (int64_t)g->H * g->W * spp);
    a.counters = w.counters;
    a.contrib = w.contrib;
    a.rays = w.rays;
    a.order = a.S.n >= 2 ? w.v1 : nullptr;
    // the sort's other buffers are dead once the order is built: the trace
    // parks each sample's averaged normal there for the shading pass
    a.rl_nx = reinterpret_cast<float *>(w.k0);
    a.rl_ny = reinterpret_cast<float *>(w.v0);
    a.rl_nz = reinterpret_cast<float *>(w.k1);
    if ((rc = set_device(scene->ctx))) return rc;
    hipError_t e = grt::launch_render_relight(a, w, opts->k, scene->ctx->num_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "relight launch");
    return GRT_OK;
}

int grt_render_relight_mesh(const grt_mesh *mesh, const grt_env *env, const grt_vertex_attrs *attrs,
                            const grt_gbuffer *g, const grt_mis_opts *opts, float *out_rgb, void *workspace,
                            size_t ws_bytes, void *stream)
{
    if (!mesh || !attrs) return fail(GRT_ERR_INVALID, "mesh/attrs is NULL");
    if (!mesh->built) return fail(GRT_ERR_NOT_BUILT, "mesh used before grt_mesh_build");
    grt::RenderArgs a;
    int rc = fill_render_common(env, g, opts, a);
    if (rc) return rc;
    if (!env->prefiltered) return fail(GRT_ERR_NOT_BUILT, "relighting needs grt_env_prefilter first");
    if (mesh->m.nf > 0 && (!attrs->albedo || !attrs->rough || !attrs->metal || !attrs->normal))
        return fail(GRT_ERR_INVALID, "a vertex attribute array is NULL");
    if ((int64_t)g->H * g->W > 0 && !out_rgb) return fail(GRT_ERR_INVALID, "out_rgb is NULL");
    if (opts->hit_list) return fail(GRT_ERR_INVALID, "relighting stores no hit lists");
    a.E.Ed = env->w.Ed; a.E.Es = env->w.Es; a.E.lut = env->w.lut;
    a.out = out_rgb;
    a.dump = opts->sample_dump;
    const int spp = opts->n_cos + opts->n_ggx + opts->n_env;
    if ((rc = check_ws(workspace, ws_bytes, grt_render_workspace_bytes((int64_t)g->H * g->W, spp), "relight")))
        return rc;
    const grt::RenderWS w = grt::carve_render(workspace, (int64_t)g->H * g->W * spp);
    a.counters = w.counters;
    a.contrib = w.contrib;
    a.rays = w.rays;
    a.order = nullptr;
    a.rl_nx = reinterpret_cast<float *>(w.k0);
    a.rl_ny = reinterpret_cast<float *>(w.v0);
    a.rl_nz = reinterpret_cast<float *>(w.k1);
    grt::MeshTraceArgs m{};
    m.nv = (int)mesh->m.nv; m.nf = (int)mesh->m.nf;
    m.rec = mesh->w.rec; m.nodes = mesh->w.nodes; m.tris = mesh->m.tris;
    m.albedo = attrs->albedo; m.rough = attrs->rough; m.metal = attrs->metal; m.vnormal = attrs->normal;
    if ((rc = set_device(mesh->ctx))) return rc;
    hipError_t e = grt::launch_render_relight_mesh(a, m, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mesh relight launch");
    return GRT_OK;
}

int grt_render_mis(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g, const grt_mis_opts *opts,
                   float *out_rgb, void *saved, void *workspace, size_t ws_bytes, void *stream)
{
    grt::RenderArgs a;
    int rc = fill_render_args(scene, env, g, opts, a);
    if (rc) return rc;
    if ((int64_t)g->H * g->W > 0 && !out_rgb) return fail(GRT_ERR_INVALID, "out_rgb is NULL");
    if (saved && !aligned(saved, 16)) return fail(GRT_ERR_INVALID, "saved must be 16-byte aligned");
    a.out = out_rgb;
    a.saved = reinterpret_cast<float4 *>(saved);
    a.saved_t = saved ? reinterpret_cast<float *>(a.saved + (int64_t)g->H * g->W * (opts->n_cos + opts->n_ggx + opts->n_env))
                      : nullptr;
    a.dump = opts->sample_dump;
    const int spp = opts->n_cos + opts->n_ggx + opts->n_env;
    if ((rc = check_ws(workspace, ws_bytes, grt_render_workspace_bytes((int64_t)g->H * g->W, spp), "render")))
        return rc;
    const grt::RenderWS w = grt::carve_render(workspace, (int64_t)g->H * g->W * spp);
    a.counters = w.counters;
    a.contrib = w.contrib;
    a.rays = w.rays;
    a.order = a.S.n >= 2 ? w.v1 : nullptr;
    if ((rc = set_device(scene->ctx))) return rc;
    if (opts->timer && opts->timer->ctx->device != scene->ctx->device)
        return fail(GRT_ERR_INVALID, "the timer belongs to another device");
    hipError_t e = grt::launch_render(a, w, opts->k, scene->ctx->num_cu, (hipStream_t)stream, use_timer(opts));
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return GRT_OK;
}

int grt_render_mis_noalloc(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g, const grt_mis_opts *opts,
                           float *out_rgb, void *saved, void *stream)
{
    if (!scene) return fail(GRT_ERR_INVALID, "scene is NULL");
    if (!g || !opts) return fail(GRT_ERR_INVALID, "gbuffer/opts is NULL");
    if (g->H < 0 || g->W < 0) return fail(GRT_ERR_INVALID, "G-buffer size %d x %d", g->H, g->W);
    const int spp = opts->n_cos + opts->n_ggx + opts->n_env;
    if (opts->n_cos < 0 || opts->n_ggx < 0 || opts->n_env < 0 || spp <= 0)
        return fail(GRT_ERR_INVALID, "sample allocation %d/%d/%d", opts->n_cos, opts->n_ggx, opts->n_env);
    const size_t need = grt_render_workspace_bytes((int64_t)g->H * g->W, spp);
    if (need > GRT_NOALLOC_SCRATCH_BYTES)
        return fail(GRT_ERR_INVALID,
                    "grt_render_mis_noalloc: %d x %d pixels x %d spp need %zu bytes of scratch, more than its "
                    "fixed %zu (about %zu samples); use grt_render_mis with a workspace",
                    g->H, g->W, spp, need, (size_t)GRT_NOALLOC_SCRATCH_BYTES,
                    (size_t)GRT_NOALLOC_SCRATCH_BYTES / 81u);
    if (!scene->ctx->scratch) return fail(GRT_ERR_DEVICE, "no scratch on device %d", scene->ctx->device);
    return grt_render_mis(scene, env, g, opts, out_rgb, saved, scene->ctx->scratch, GRT_NOALLOC_SCRATCH_BYTES,
                          stream);
}

static int render_backward(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g,
                           const grt_mis_opts *opts, const float *grad_rgb, const void *saved,
                           grt_surfel_grads *grads, const grt_shading_grads *shade, void *workspace,
                           size_t ws_bytes, void *stream)
{
    grt::RenderArgs a;
    int rc = fill_render_args(scene, env, g, opts, a, true);
    if (rc) return rc;
    if ((int64_t)g->H * g->W > 0 && (!grad_rgb || !saved)) return fail(GRT_ERR_INVALID, "grad_rgb/saved is NULL");
    if (saved && !aligned(saved, 16)) return fail(GRT_ERR_INVALID, "saved must be 16-byte aligned");
    if ((rc = check_grads(grads, scene->s.n))) return rc;
    a.grad = grad_rgb;
    a.saved = const_cast<float4 *>(reinterpret_cast<const float4 *>(saved));
    a.saved_t = reinterpret_cast<float *>(a.saved + (int64_t)g->H * g->W * (opts->n_cos + opts->n_ggx + opts->n_env));
    a.g = grad_ptrs(scene, grads);
    const int spp = opts->n_cos + opts->n_ggx + opts->n_env;
    if ((rc = check_ws(workspace, ws_bytes, grt_render_workspace_bytes((int64_t)g->H * g->W, spp),
                       "render backward")))
        return rc;
    const grt::RenderWS w = grt::carve_render(workspace, (int64_t)g->H * g->W * spp);
    a.counters = w.counters;
    a.rays = w.rays;
    a.order = a.S.n >= 2 ? w.v1 : nullptr;
    // the backward does not use the contribution slots: they hold the
    // per-sample origin gradients when the shading state is differentiated
    a.gorig = shade ? w.contrib : nullptr;
    if (opts->timer && opts->timer->ctx->device != scene->ctx->device)
        return fail(GRT_ERR_INVALID, "the timer belongs to another device");
    if ((rc = set_device(scene->ctx))) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const grt::KernelTimer *tm = use_timer(opts);
    hipError_t e = grt::launch_grad_lines_zero(a.g.acc, scene->s.n, st);
    if (e == hipSuccess)
        e = a.hits ? grt::launch_render_backward_stored(a, w, opts->k, scene->ctx->num_cu, st, tm)
                   : grt::launch_render_backward(a, w, opts->k, scene->ctx->num_cu, st, tm);
    if (e == hipSuccess) e = grt::launch_grad_lines_apply(a.g, scene->s.n, st);
    if (e == hipSuccess && shade) {
        const grt::ShadeGradOut o{shade->x, shade->n, shade->wo, shade->albedo, shade->rough, shade->metal};
        e = grt::launch_render_shade_grad(a, o, st);
    }
    if (e != hipSuccess) return hip_fail(e, "render backward launch");
    return GRT_OK;
}

int grt_render_mis_backward(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g, const grt_mis_opts *opts,
                            const float *grad_rgb, const void *saved, grt_surfel_grads *grads, void *workspace,
                            size_t ws_bytes, void *stream)
{
    return render_backward(scene, env, g, opts, grad_rgb, saved, grads, nullptr, workspace, ws_bytes, stream);
}

int grt_render_mis_backward_shading(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g,
                                    const grt_mis_opts *opts, const float *grad_rgb, const void *saved,
                                    grt_surfel_grads *grads, const grt_shading_grads *shade, void *workspace,
                                    size_t ws_bytes, void *stream)
{
    if (!shade) return fail(GRT_ERR_INVALID, "shade is NULL");
    return render_backward(scene, env, g, opts, grad_rgb, saved, grads, shade, workspace, ws_bytes, stream);
}

}  // extern "C"
