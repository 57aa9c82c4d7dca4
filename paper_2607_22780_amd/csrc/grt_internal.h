// grt_internal.h -- host-side structures shared by the translation units of
// libgrt (workspace carving and kernel launchers).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "grt.h"
#include "grt_device.h"

struct grt_ctx {
    int device;
    int num_cu;
    void *scratch;  // this device's copy of grt_render_mis_noalloc's scratch (device address)
};


namespace grt {

// bytes of per-launch counters at the head of every kernel workspace
constexpr size_t kCounterBytes = 256;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

inline int64_t sort_blocks(int64_t n) { return (n + kSortTile - 1) / kSortTile; }
// Words of sort histogram for n keys: 256 per sort block, then the chunk
// sums of the multi-block scan (one per 4096 histogram words).
inline size_t sort_hist_words(int64_t n)
{
    const size_t total = 256 * (size_t)(sort_blocks(n) > 0 ? sort_blocks(n) : 1);
    return total + (total + 4095) / 4096;
}

// Carving of a scene workspace; the same function sizes and places.
struct SceneWS {
    float4 *rec;
    float4 *col;
    Node *nodes;
    float *leaf_box;   // [n,6] sorted order
    float *box_tmp;    // [n,6] surfel order
    uint32_t *keys0, *keys1, *vals0, *vals1;
    int32_t *parent_int;   // [n-1]
    int32_t *parent_leaf;  // [n]
    uint32_t *flags;       // [n-1]
    uint32_t *hist;        // [256 * blocks]
    int32_t *bounds;       // [8]
    float *acc;            // [n,16] gradient lines of the backward passes
    float4 *quat;          // [n] stored quaternions in record order
    Node4 *nodes4;         // [n-1] the 4-wide hierarchy (node 0 the root)
    int32_t *f4;           // [n-1] binary node each 4-wide node was collapsed from
    int32_t *ctl4;         // [4] collapse state: level range [lo, hi), node count
    size_t bytes;
};

inline SceneWS carve_scene(void *base, int64_t n)
{
    SceneWS w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? (char *)base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    size_t nn = (size_t)(n > 0 ? n : 1);
    size_t ni = (size_t)(n > 1 ? n - 1 : 1);
    w.rec = (float4 *)take(64 * nn);
    w.col = (float4 *)take(16 * nn);
    w.nodes = (Node *)take(sizeof(Node) * ni);
    w.leaf_box = (float *)take(24 * nn);
    w.box_tmp = (float *)take(24 * nn);
    w.keys0 = (uint32_t *)take(4 * nn);
    w.keys1 = (uint32_t *)take(4 * nn);
    w.vals0 = (uint32_t *)take(4 * nn);
    w.vals1 = (uint32_t *)take(4 * nn);
    w.parent_int = (int32_t *)take(4 * ni);
    w.parent_leaf = (int32_t *)take(4 * nn);
    w.flags = (uint32_t *)take(4 * ni);
    w.hist = (uint32_t *)take(4 * sort_hist_words(n));
    w.bounds = (int32_t *)take(4 * 8);
    w.acc = (float *)take(64 * nn);
    w.quat = (float4 *)take(16 * nn);
    w.nodes4 = (Node4 *)take(sizeof(Node4) * ni);
    w.f4 = (int32_t *)take(4 * ni);
    w.ctl4 = (int32_t *)take(16);
    w.bytes = off;
    return w;
}

// Prefiltered representation of an environment for split-sum relighting:
// kPfH x kPfW direction tables (texel centres, the environment's convention)
// of the diffuse and of the specular average at roughness l / (kPfL - 1),
// l = 1 .. kPfL - 1 (level 0 is the environment itself), and the DFG table
// [kLutN (n.v)][kLutN (roughness)][A, B] integrated on kLutQ x kLutQ nodes.
constexpr int kPfH = 16, kPfW = 32, kPfL = 6, kLutN = 32, kLutQ = 256;

struct EnvWS {
    float *marg;   // [H+1]
    float *cond;   // [H,W+1]
    double *rows;  // [H]
    float *Ed;     // [kPfH, kPfW, 3]
    float *Es;     // [kPfL - 1, kPfH, kPfW, 3]
    float *lut;    // [kLutN, kLutN, 2]
    size_t bytes;
};

inline EnvWS carve_env(void *base, int H, int W)
{
    EnvWS w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? (char *)base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    w.marg = (float *)take(4 * (size_t)(H + 1));
    w.cond = (float *)take(4 * (size_t)H * (size_t)(W + 1));
    w.rows = (double *)take(8 * (size_t)H);
    w.Ed = (float *)take(4 * (size_t)kPfH * kPfW * 3);
    w.Es = (float *)take(4 * (size_t)(kPfL - 1) * kPfH * kPfW * 3);
    w.lut = (float *)take(4 * (size_t)kLutN * kLutN * 2);
    w.bytes = off;
    return w;
}

// Scene build (scene.hip)
hipError_t launch_scene_build(const grt_surfels &s, float alpha_min, const SceneWS &w, hipStream_t st);
// Stable LSD radix sort of n (key, value) pairs over the low 8*passes bits of
// the keys; the result is in (k1, v1) after an odd number of passes, in
// (k0, v0) after an even number.  hist holds 256 * sort_blocks(n) words.
void launch_radix_sort(int n, int passes, uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, uint32_t *hist,
                       hipStream_t st);

// Trace forward/backward (trace.hip)
struct TraceArgs {
    SceneDev S;
    int64_t n;
    const float *o, *d, *tmin_a, *tmax_a;
    float tmin, tmax, tcut;
    float sky[3];
    float *out_rgb, *out_T, *out_L;
    int32_t *out_nhit;
    int32_t *dump_id;
    float *dump_tau;
    int cap;
    float *stop_depth;  // written by the forwards, read by the backwards (NULL: unused)
    unsigned long long *counters;
    const float *env_rgb;  // environment [env_H, env_W, 3] for L, or NULL: the constant sky
    int env_H, env_W;
};
hipError_t launch_trace(const TraceArgs &a, int k, int num_cu, hipStream_t st);

// Attribute query over the rays of `f` (its radiance outputs unused).
struct TraceAttrArgs {
    TraceArgs f;
    const float *albedo, *rough, *metal;
    float *out_V, *out_albedo, *out_rough, *out_metal, *out_normal;
};
hipError_t launch_trace_attr(const TraceAttrArgs &a, int k, int num_cu, hipStream_t st);

// Primary-ray G-buffer over the rays of `f`: a full G-buffer (x, n, wo,
// albedo, rough, metal, valid) plus the depth and colour maps.
struct TraceGBufArgs {
    TraceArgs f;
    const float *albedo, *rough, *metal;
    float min_opacity;
    float *x, *n, *wo, *out_albedo, *out_rough, *out_metal, *depth, *rgb;
    uint8_t *valid;
    float *weight, *nlen;  // saved for the backward (NULL: not written)
};
hipError_t launch_trace_gbuffer(const TraceGBufArgs &a, int k, int num_cu, hipStream_t st);

struct GradPtrs {
    float *means, *scales, *quats, *opacity, *rgb;
    float *acc;  // [n,16] per-surfel lines the kernels accumulate into
    const int32_t *order;  // unused by kernels (ids travel in records)
};
struct TraceBwdArgs {
    TraceArgs f;
    const float *fwd_rgb, *fwd_T, *grad_rgb, *grad_T;
    GradPtrs g;
};
hipError_t launch_trace_backward(const TraceBwdArgs &a, int k, int num_cu, hipStream_t st);
// Pinhole camera rays (grt_camera_rays): the camera frame in double, set up
// on the host, and one ray per pixel centre.
struct PinholeDev {
    double eye[3], f[3], r[3], u[3];
    double t, aspect;
};
bool make_pinhole(const double eye[3], const double target[3], const double up[3], double vfov_deg, int H, int W,
                  PinholeDev &c);
hipError_t launch_camera_rays(const PinholeDev &c, int H, int W, float *o, float *d, hipStream_t st);

// Backward of the primary-ray G-buffer: the forward's maps (fwd_*), upstream
// gradients (g_*, NULL = zero) and attribute gradients (ga_*, NULL = skipped).
struct TraceGBufBwdArgs {
    TraceArgs f;
    const float *albedo, *rough, *metal;
    const float *fwd_n, *fwd_albedo, *fwd_rough, *fwd_metal, *fwd_depth, *fwd_rgb, *fwd_weight, *fwd_nlen;
    const uint8_t *fwd_valid;
    const float *g_x, *g_n, *g_albedo, *g_rough, *g_metal, *g_depth, *g_rgb;
    GradPtrs g;
    float *ga_albedo, *ga_rough, *ga_metal;
};
hipError_t launch_trace_gbuffer_backward(const TraceGBufBwdArgs &a, int k, int num_cu, hipStream_t st);
// Clear the scene's gradient lines (before a backward pass) and add them to
// the caller's gradient arrays (after it).
hipError_t launch_grad_lines_zero(float *acc, int64_t n, hipStream_t st);
hipError_t launch_grad_lines_apply(const GradPtrs &g, int64_t n, hipStream_t st);

// Environment and MIS (render.hip)
struct EnvDev {
    int H, W;
    const float *rgb;
    const float *marg;
    const float *cond;
    const float *Ed, *Es, *lut;  // prefiltered tables (relighting), or null
};
hipError_t launch_env_build(const float *rgb, int H, int W, const EnvWS &w, hipStream_t st);

// LBVH pieces shared by the surfel scene and the triangle mesh (scene.hip)
hipError_t launch_bounds_reset(int32_t *bounds, hipStream_t st);
hipError_t launch_morton_sort(int n, const float *centres, const int32_t *bounds, uint32_t *keys0, uint32_t *vals0,
                              uint32_t *keys1, uint32_t *vals1, uint32_t *hist, hipStream_t st);
hipError_t launch_hierarchy_refit(int n, const uint32_t *keys, const float *leaf_box, Node *nodes, int32_t *parent_int,
                                  int32_t *parent_leaf, uint32_t *flags, hipStream_t st);

// Triangle mesh for the mesh backend of the attribute query (mesh.hip):
// records in Morton order, 48 B each: (v0, triangle id bits), (e1, 0), (e2, 0).
struct MeshWS {
    float4 *rec;
    Node *nodes;
    float *leaf_box;  // [nf,6] sorted order
    float *box_tmp;   // [nf,6] triangle order
    float *centre;    // [nf,3]
    uint32_t *keys0, *keys1, *vals0, *vals1;
    int32_t *parent_int, *parent_leaf;
    uint32_t *flags, *hist;
    int32_t *bounds;
    size_t bytes;
};

inline MeshWS carve_mesh(void *base, int64_t nf)
{
    MeshWS w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? (char *)base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    size_t n = (size_t)(nf > 0 ? nf : 1), ni = (size_t)(nf > 1 ? nf - 1 : 1);
    w.rec = (float4 *)take(48 * n);
    w.nodes = (Node *)take(sizeof(Node) * ni);
    w.leaf_box = (float *)take(24 * n);
    w.box_tmp = (float *)take(24 * n);
    w.centre = (float *)take(12 * n);
    w.keys0 = (uint32_t *)take(4 * n);
    w.keys1 = (uint32_t *)take(4 * n);
    w.vals0 = (uint32_t *)take(4 * n);
    w.vals1 = (uint32_t *)take(4 * n);
    w.parent_int = (int32_t *)take(4 * ni);
    w.parent_leaf = (int32_t *)take(4 * n);
    w.flags = (uint32_t *)take(4 * ni);
    w.hist = (uint32_t *)take(4 * sort_hist_words((int64_t)n));
    w.bounds = (int32_t *)take(4 * 8);
    w.bytes = off;
    return w;
}

struct MeshTraceArgs {
    int64_t n;                       // rays
    int nv, nf;
    const float4 *rec;
    const Node *nodes;
    const int32_t *tris;             // [nf,3]
    const float *o, *d;
    float tmin, tmax;
    const float *albedo, *rough, *metal, *vnormal;  // per vertex
    float *out_V, *out_albedo, *out_rough, *out_metal, *out_normal;
};
hipError_t launch_mesh_build(int nv, const float *verts, int nf, const int32_t *tris, const MeshWS &w, hipStream_t st);
hipError_t launch_mesh_trace_attr(const MeshTraceArgs &a, hipStream_t st);

// Cross-bilateral denoiser (denoise.hip)
constexpr int kDenoiseMaxRadius = 8;
struct DenoiseArgs {
    int H, W, radius;
    float sigma_s, sigma_d, sigma_n, eps_d;
    const float *rgb, *depth, *normal;
    const uint8_t *valid;
    float *out;
};
hipError_t launch_denoise(const DenoiseArgs &a, hipStream_t st);
// The prefiltered direction tables of an environment, and (lut) the DFG
// table, which depends on nothing but its resolution.
hipError_t launch_env_prefilter(const float *rgb, int H, int W, const EnvWS &w, hipStream_t st, bool lut = true);
hipError_t launch_dfg_lut(float *lut, hipStream_t st);

// Walk statistics of the instrumented build (compiled with GRT_STATS): 2 x 9
// sums of the render kernels' walks; reset zeroes them after the read.  The
// caller synchronises the device first.
bool walk_stats_built();
hipError_t walk_stats_read(unsigned long long *out, bool reset);

struct RenderArgs {
    SceneDev S;
    EnvDev E;
    int H, W;
    const float *x, *n, *wo, *alb, *rough, *metal;
    const uint8_t *valid;
    int nc, ng, ne;
    uint64_t seed;
    uint32_t job;
    float tmin, tcut;
    float *out;
    float4 *saved;
    float *saved_t;  // the forward's stop depth per sample (after the saved (C, T) records)
    float *dump;
    float4 *contrib;  // per sample f L_i cos / q, reduced per pixel afterwards
    float4 *rays;     // per sample record written by the generation kernel (3 x float4)
    const uint32_t *order;  // samples in traversal order (null: index order)
    uint32_t *hits;         // stored hit lists: counts [nray], then [nray][hcap] (null: none)
    int hcap;
    unsigned long long *counters;
    // relighting: per-surfel attributes (by id), and where the trace parks
    // each sample's averaged normal for the shading pass (three float arrays)
    const float *sa_albedo, *sa_rough, *sa_metal;
    float *rl_nx, *rl_ny, *rl_nz;
    // backward
    const float *grad;
    GradPtrs g;
    // backward with the shading state: per sample, the loss's gradient with
    // respect to its ray's origin (xyz; null: not formed)
    float4 *gorig;
};
// Render workspace: counters | contributions (16 B/sample) | ray records
// (48 B/sample) | sort keys and values (2 x 2 x 4 B/sample) | sort histogram.
struct RenderWS {
    unsigned long long *counters;
    float4 *contrib;
    float4 *rays;
    uint32_t *k0, *v0, *k1, *v1, *hist;
    size_t bytes;
};

inline RenderWS carve_render(void *base, int64_t nray)
{
    RenderWS w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? (char *)base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t n = (size_t)(nray > 0 ? nray : 1);
    w.counters = (unsigned long long *)take(kCounterBytes);
    w.contrib = (float4 *)take(16 * n);
    w.rays = (float4 *)take(48 * n);
    w.k0 = (uint32_t *)take(4 * n);
    w.v0 = (uint32_t *)take(4 * n);
    w.k1 = (uint32_t *)take(4 * n);
    w.v1 = (uint32_t *)take(4 * n);
    w.hist = (uint32_t *)take(4 * sort_hist_words((int64_t)n));
    w.bytes = off;
    return w;
}

// one ray record per sample of the whole G-buffer (sampling only, no trace)
hipError_t launch_render_gen(const RenderArgs &a, hipStream_t st);
// The coherent-order sort key of each of a's first n samples (direction bin,
// then origin cell; untraced samples last), with value tag | sample index.
hipError_t launch_ray_keys(const RenderArgs &a, int n, uint32_t *keys, uint32_t *vals, uint32_t tag, hipStream_t st);
// Split-sum relighting (needs a.E's prefiltered tables and a.sa_*): the
// forward render with the attribute query and Eq. relight_splitsum.
hipError_t launch_render_relight(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st);
// Relighting's shading pass alone, over every sample of a.H x a.W x spp whose
// attribute query has run (the server runs it once a request's rays are done).
hipError_t launch_relight_shade(const RenderArgs &a, hipStream_t st);
// relighting through the mesh: the query pass over a render's ray records
// (m's ray fields unused), then the surfel relight's shading pass
hipError_t launch_mesh_relight_query(const RenderArgs &a, const MeshTraceArgs &m, hipStream_t st);
hipError_t launch_render_relight_mesh(const RenderArgs &a, const MeshTraceArgs &m, hipStream_t st);
// Order the traced samples for coherent traversal: by direction bin, then by
// the Morton code of the origin in the scene's root box (untraced last).
// Sets nothing on the host; a.order must point at w.v1 afterwards.
hipError_t launch_ray_order(const RenderArgs &a, const RenderWS &w, hipStream_t st);
// Events recorded around the persistent trace kernel(s) of a launch (null: none).
struct KernelTimer {
    hipEvent_t begin, end;
};
hipError_t launch_render(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st,
                         const KernelTimer *tm = nullptr);
hipError_t launch_render_backward(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st,
                                  const KernelTimer *tm = nullptr);
// Backward from stored hit lists (a.hits); re-traverses overflowing samples.
hipError_t launch_render_backward_stored(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st,
                                         const KernelTimer *tm = nullptr);
// After a backward with a.gorig set: the gradients with respect to each
// pixel's shading state (null outputs are not written).
struct ShadeGradOut {
    float *x, *n, *wo, *alb, *rough, *metal;
};
hipError_t launch_render_shade_grad(const RenderArgs &a, const ShadeGradOut &o, hipStream_t st);

// Zero the per-launch counters; persistent grid size for a kernel.
hipError_t launch_zero_counters(unsigned long long *c, hipStream_t st);
template <class Kern>
inline int persistent_blocks(Kern kernel, int num_cu, int64_t work_items)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    int64_t want = (work_items + 255) / 256;
    int64_t cap = (int64_t)per_cu * num_cu;
    int64_t nb = want < cap ? want : cap;
    return (int)(nb < 1 ? 1 : nb);
}

}  // namespace grt
