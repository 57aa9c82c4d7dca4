/*
 * grt.h -- C ABI of libgrt: differentiable 2D Gaussian ray tracing (2DGRT) of
 * secondary rays with multiple-importance-sampled (MIS) shading, for AMD
 * Instinct MI355X (gfx950).
 *
 * The operations follow "Inter-Reflective Gaussian Splatting for Robust and
 * Efficient Inverse Rendering" (IRGS++):
 *   - a surfel is a 2D Gaussian disk (centre, tangents t_u, t_v, scales s_u,
 *     s_v, opacity o, outgoing radiance c)            -- Sec. 3.1, "2D Gaussian splatting";
 *   - Trace(r_o, r_d) -> (c_rt, o_rt) composites the ray's intersected
 *     surfels front to back                           -- Sec. 3.2, Eq. raytracing_intersection, Eq. trace;
 *   - L_i = V L_dir + L_ind with V = 1 - o_rt, L_ind = c_rt
 *                                                      -- Sec. 3.3, Eqs. lighting_decompose, incident_trace;
 *   - c_pbr = (1/N_r) sum g(w)/q(w) with the deterministic mixture q of a
 *     cosine, a GGX and an environment proposal       -- Sec. 3.3 Eq. montecarlo, Sec. 3.4.1 Eq. mis;
 *   - gradients flow back through the secondary-ray queries (Sec. 3.2).
 *
 * Conventions (every entry point):
 *   - Return value: GRT_OK (0) or a negative GRT_ERR_* code; nothing throws or
 *     aborts across the ABI.  grt_last_error() gives the message of the last
 *     failure on the calling thread.
 *   - Array arguments are DEVICE pointers to contiguous row-major float32
 *     (uint8 for masks) unless stated, owned by the caller and borrowed only
 *     until the work queued on `stream` has finished.  `stream` is a
 *     hipStream_t passed as void* (NULL = the null stream).
 *   - Calls are asynchronous on `stream`; a kernel fault surfaces as
 *     GRT_ERR_DEVICE from a later call that synchronises.
 *   - Device scratch is caller-allocated ("workspace"); the library allocates
 *     device memory only inside the relighting server (from its budget).
 *   - Surfel quaternions are (w, x, y, z) and need not be unit; t_u, t_v and
 *     the normal n are the columns of the rotation matrix of q/|q|.
 *   - A surfel is hit where the ray crosses its plane at t_min < tau <= t_max,
 *     |n . d| >= 1e-6, and rho^2 = u^2 + v^2 <= min(9, 2 ln(o / alpha_min))
 *     (three standard deviations and the minimum influence alpha_min).  Hits
 *     are composited in ascending (tau, surfel id); compositing includes the
 *     hit that takes the transmittance below t_cut and then stops.
 */
#ifndef GRT_H
#define GRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRT_OK 0
#define GRT_ERR_INVALID (-1)    /* bad argument, size or state */
#define GRT_ERR_OOM (-2)        /* workspace too small / budget exhausted */
#define GRT_ERR_NOT_BUILT (-3)  /* scene or environment used before its build call */
#define GRT_ERR_DEVICE (-4)     /* a HIP runtime call failed */
#define GRT_ERR_ADMISSION (-5)  /* server: job can never fit the memory budget */
#define GRT_ERR_BUSY (-6)       /* server: queue full, retry later */
#define GRT_ERR_CANCELLED (-7)  /* server: job was cancelled */
#define GRT_ERR_TIMEOUT (-8)    /* server: wait timed out */

typedef struct grt_ctx grt_ctx;
typedef struct grt_scene grt_scene;
typedef struct grt_env grt_env;
typedef struct grt_server grt_server;

/* Message of the last failing call on this thread ("" if none). */
const char *grt_last_error(void);
/* Static name of a status code. */
const char *grt_status_str(int status);
/* Library version, (major << 16) | minor. */
int grt_version(void);

/* ---------------------------------------------------------------- context */

/* Bind to HIP device `device`.  *out receives a handle freed by
 * grt_ctx_destroy.  Fails with GRT_ERR_DEVICE if the device is absent. */
int grt_ctx_create(int device, grt_ctx **out);
int grt_ctx_destroy(grt_ctx *ctx);

/* ------------------------------------------------------------------ scene */

/* Surfel parameters, device pointers, SoA (Sec. 3.1 "2D Gaussian splatting";
 * Sec. 3.2 "Bounding proxy and ray-splat intersection"):
 *   means [n,3], scales [n,2] (s_u, s_v > 0, linear standard deviations),
 *   quats [n,4] (w,x,y,z), opacity [n] in [0,1], rgb [n,3] outgoing radiance. */
typedef struct {
    int64_t n;
    const float *means;
    const float *scales;
    const float *quats;
    const float *opacity;
    const float *rgb;
} grt_surfels;

/* Bytes of device workspace a scene of n surfels needs (records and stored
 * quaternions in LBVH order, bounding boxes, LBVH nodes, sort buffers, and 64
 * bytes per surfel in which the backward passes sum gradients).  256-byte aligned pointer required. */
size_t grt_scene_workspace_bytes(int64_t n);

/* Create a scene over borrowed surfel arrays and a caller-owned workspace of
 * `ws_bytes` >= grt_scene_workspace_bytes(n).  alpha_min is the minimum
 * influence (1/255 in the workloads; 0 keeps only the 3-sigma bound).  The
 * scene is not usable until grt_scene_build.  n may be 0 (empty scene). */
int grt_scene_create(grt_ctx *ctx, const grt_surfels *surfels, float alpha_min, void *workspace, size_t ws_bytes,
                     grt_scene **out);

/* Build the acceleration structure on `stream`: per-surfel frames and
 * 3-sigma bounding boxes (the paper's adaptive bounding proxy, Eq.
 * icosahedron_transform, as an axis-aligned box), then an LBVH (Morton codes
 * of box centres, LSD radix sort, Karras hierarchy, bottom-up refit) -- the
 * BVH the paper builds over its proxies (Sec. 3.2).  Reads the surfel arrays;
 * call again after any parameter change. */
int grt_scene_build(grt_scene *scene, void *stream);

/* Re-point the scene at new surfel arrays of the same count (no build). */
int grt_scene_set_surfels(grt_scene *scene, const grt_surfels *surfels);
int grt_scene_destroy(grt_scene *scene);

/* Device pointers into the built scene, for inspection by tests:
 * records [n,16] float (sorted order; word 11 holds the surfel id as bits,
 * word 15 the stored scale s_u), nodes [max(n-1,0),16] (child boxes lo/hi as
 * floats 0..11, children as int32 words 12,13: >= 0 internal node, < 0 leaf
 * -(pos+1)), order [n] int32 (sorted position -> surfel id). */
typedef struct {
    int64_t n;
    const float *records;
    const float *nodes;
    const int32_t *order;
    const float *leaf_boxes; /* [n,6] lo.xyz, hi.xyz in sorted order */
    const float *colours;    /* [n,4] rgb and the stored scale s_v, sorted order */
    const float *quats;      /* [n,4] the stored quaternion (w first), sorted order */
    /* The 4-wide hierarchy the traversal walks, collapsed from `nodes`:
     * nodes4 [max(n-1,0),32] (floats 0..23 the four child boxes as lo.x[4],
     * lo.y[4], lo.z[4], hi.x[4], hi.y[4], hi.z[4]; int32 words 24..27 the
     * children: >= 0 a 4-wide node, < 0 leaf -(pos+1), 0x7fffffff unused;
     * word 28 the child count), of which the first *nodes4_count are used
     * (node 0 the root; device int32, valid once the build has run). */
    const float *nodes4;
    const int32_t *nodes4_count;
} grt_scene_view;
int grt_scene_view_get(const grt_scene *scene, grt_scene_view *out);

/* ------------------------------------------------------------------ trace */

/* Rays (Sec. 3.2, r_o + tau r_d).  origins/dirs [n,3]; dirs unit length.
 * t_min/t_max per ray [n] or NULL to use the scalars; 0 <= t_min < t_max.
 * The scalar t_min_all must be >= 0 (GRT_ERR_INVALID otherwise); a negative
 * or NaN per-ray t_min is read as 0 (a ray starts at its origin, and depth
 * keys order depths by their bit patterns, which is monotone for tau >= 0
 * only), so hits behind the origin are never admitted. */
typedef struct {
    int64_t n;
    const float *origins;
    const float *dirs;
    const float *t_min;
    const float *t_max;
    float t_min_all;
    float t_max_all;
} grt_rays;

/* k: k-nearest hit buffer size per traversal round, one of 1,2,4,8,12,16,32
 *    (results do not depend on k).
 * t_cut: transmittance cutoff (1e-3 in the workloads).
 * sky: radiance of escaped rays, L = c_rt + T sky (when env is NULL).
 * env: optional built environment (grt_env_build); then L = c_rt + T L_env(d)
 *    with the environment at the nearest texel of the ray direction, as the
 *    MIS render looks it up (Sec. 3.3 Eq. lighting_decompose).  It must stay
 *    alive until the trace has run on its stream.
 * hit_ids/hit_tau: optional [n, hit_cap] dump of the composited hits in
 *    order (surfel id, depth), -1 / 0 padded; NULL to skip.
 * stop_depth: optional [n] (device, float32).  grt_trace and
 *    grt_trace_gbuffer write the depth of each ray's last composited hit
 *    (0 when none); grt_trace_backward and grt_trace_gbuffer_backward, given
 *    the opts of that forward, end their re-traversal there (every hit they
 *    composite lies at or before it), which saves the walk beyond.  It must
 *    then hold that forward's values for the same rays; NULL: the backward
 *    walks the whole ray range. */
typedef struct {
    int k;
    float t_cut;
    float sky[3];
    int32_t *hit_ids;
    float *hit_tau;
    int hit_cap;
    float *stop_depth;
    const grt_env *env;
} grt_trace_opts;

/* Bytes of device workspace grt_trace / grt_trace_backward need (the
 * dynamic ray-fetch counters of the launch).  256-byte aligned. */
size_t grt_trace_workspace_bytes(int64_t nrays);

/* Trace(r_o, r_d) for every ray (Eq. trace):
 *   out_rgb [n,3] = c_rt, out_T [n] = 1 - o_rt (transmittance after the last
 *   composited hit), out_L [n,3] = c_rt + T sky (NULL to skip),
 *   out_nhit [n] int32 composited hits (NULL to skip).
 * workspace: >= grt_trace_workspace_bytes(n), not shared by launches that
 * may overlap. */
int grt_trace(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts, float *out_rgb,
              float *out_T, float *out_L, int32_t *out_nhit, void *workspace, size_t ws_bytes, void *stream);

/* Gradient accumulators (device, float32, ADDED to): means [n,3], scales
 * [n,2], quats [n,4], opacity [n], rgb [n,3].  Gradients are w.r.t. the
 * stored parameters (unnormalised quaternion, linear scales, opacity). */
typedef struct {
    float *means;
    float *scales;
    float *quats;
    float *opacity;
    float *rgb;
} grt_surfel_grads;

/* Per-surfel material attributes (device, float32, borrowed): albedo [n,3],
 * roughness [n], metallic [n] -- the attributes a_i, r_i, m_i that the
 * deferred maps blend (Sec. 3.3, Eq. deferred_maps). */
typedef struct {
    const float *albedo;
    const float *rough;
    const float *metal;
} grt_surfel_attrs;

/* Attribute query (Sec. 3.5.1, Eq. trace_attr; the Gaussian backend): for
 * every ray, the same ordered hits and cut-off as grt_trace, returning
 *   out_V [n]          visibility of the environment = the final
 *                      transmittance (grt_trace's out_T, 1 - o_rt);
 *   out_albedo [n,3], out_rough [n], out_metal [n], out_normal [n,3]
 *                      the composited surfels' attributes averaged with the
 *                      normalized blending weights T_k alpha_k / sum_j T_j
 *                      alpha_j (as in Eq. deferred_maps); each surfel normal
 *                      n = t_u x t_v enters turned toward the ray origin,
 *                      and the averaged normal is not renormalized.
 * A ray with no composited hit returns V = 1 and zero attributes.  Same
 * rays/opts as grt_trace (sky and the dump fields are ignored); same
 * workspace (grt_trace_workspace_bytes). */
int grt_trace_attr(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                   const grt_surfel_attrs *attrs, float *out_V, float *out_albedo, float *out_rough, float *out_metal,
                   float *out_normal, void *workspace, size_t ws_bytes, void *stream);

/* Primary-ray G-buffer by 2DGRT (Sec. 3.3, Eq. deferred_maps with the
 * camera rays traced instead of rasterized).  For every ray (camera origin o,
 * unit direction d), the same ordered hits and cut-off as grt_trace; the
 * deferred maps are the averages over the composited hits with normalized
 * weights T_k alpha_k / sum_j T_j alpha_j of the hit depth tau_k, the surfel
 * normal (turned toward the camera), colour and attributes.  A pixel is
 * covered when its accumulated opacity 1 - T reaches min_opacity (0, 1] and
 * the averaged normal N does not vanish; then
 *   x = o + D d, n = N/|N|, wo = -d, albedo, rough, metal = the maps,
 *   depth = D, rgb = the colour map, valid = 1,
 * and every entry is 0 otherwise.  The arrays (device, [n,3] or [n]) form a
 * grt_gbuffer that grt_render_mis and grt_render_relight take as is.  Same
 * rays/opts/workspace as grt_trace (sky and dump ignored).
 * weight and nlen are optional (NULL: not written) and are what
 * grt_trace_gbuffer_backward needs besides the maps: weight [n] = W, the sum
 * of the blending weights sum_k T_k alpha_k, and nlen [n] = |N| of the
 * averaged normal before renormalization; both 0 on uncovered pixels. */
typedef struct {
    float *x;
    float *n;
    float *wo;
    float *albedo;
    float *rough;
    float *metal;
    float *depth;
    float *rgb;
    uint8_t *valid;
    float *weight;
    float *nlen;
} grt_gbuffer_out;
int grt_trace_gbuffer(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                      const grt_surfel_attrs *attrs, float min_opacity, grt_gbuffer_out *out, void *workspace,
                      size_t ws_bytes, void *stream);

/* A pinhole camera (double): the eye, a point it looks at, the up direction
 * and the vertical field of view in degrees. */
typedef struct {
    double eye[3];
    double target[3];
    double up[3];
    double vfov_deg;
} grt_camera;

/* Primary rays of an H x W image, one through each pixel centre, row-major
 * with row 0 at the top (the camera rays grt_trace_gbuffer takes):
 *   f = normalize(target - eye), r = normalize(f x up), u = r x f,
 *   t = tan(vfov_deg * pi/180 * 0.5),
 *   sx = ((j + 0.5) / W * 2 - 1) * t * (W / H), sy = (1 - (i + 0.5) / H * 2) * t,
 *   d(i, j) = normalize(f + sx r + sy u),  o = eye,
 * each evaluated in double, left to right as written, with no fused
 * multiply-add, then rounded to float.  out_o, out_d [H*W, 3] device float32.
 * GRT_ERR_INVALID for a degenerate camera (eye = target, up parallel to the
 * view direction, vfov outside (0, 180)) or an empty image. */
int grt_camera_rays(grt_ctx *ctx, const grt_camera *cam, int H, int W, float *out_o, float *out_d, void *stream);

/* Upstream gradients of the primary-ray G-buffer's maps (device, float32,
 * borrowed; x, n, albedo, rgb [n,3], rough, metal, depth [n]; any NULL =
 * zero).  wo and valid have none. */
typedef struct {
    const float *x;
    const float *n;
    const float *albedo;
    const float *rough;
    const float *metal;
    const float *depth;
    const float *rgb;
} grt_gbuffer_grad;

/* Gradient accumulators of the per-surfel attributes (device, float32, ADDED
 * to, by surfel id: albedo [n,3], rough [n], metal [n]; any NULL = not
 * computed). */
typedef struct {
    float *albedo;
    float *rough;
    float *metal;
} grt_attr_grads;

/* Backward of grt_trace_gbuffer by re-traversal (Sec. 3.3, Eq. deferred_maps:
 * gradients reach the surfels through the deferred maps of the primary
 * rays): accumulates d/d(surfels) into `grads` and d/d(attributes) into
 * `agrads` (NULL: none) of
 *   L = sum over covered pixels of grad.x . x + grad.n . n + ... + grad.rgb . rgb.
 * Every map is a ratio of blended sums over W = sum_k T_k alpha_k, and
 * n = N/|N|; x = o + depth d, so grad.x reaches the surfels through the depth.
 * Uncovered pixels contribute nothing (their maps are constant) and the
 * coverage test is not differentiated.  `fwd` holds the forward's outputs
 * with the same scene, rays, opts and attributes, including weight and nlen
 * (x and wo are not read).  The surfel terms are summed in the scene's
 * workspace, so backward passes over one scene must not overlap in time; the
 * attribute terms are float32 atomics in no fixed order.  Same workspace as
 * grt_trace. */
int grt_trace_gbuffer_backward(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                               const grt_surfel_attrs *attrs, const grt_gbuffer_out *fwd,
                               const grt_gbuffer_grad *grad, grt_surfel_grads *grads, grt_attr_grads *agrads,
                               void *workspace, size_t ws_bytes, void *stream);

/* Backward of grt_trace by re-traversal (Sec. 3.2: gradients backpropagate
 * through the traced radiance): accumulates d/d(surfels) of
 *   sum_r grad_rgb[r] . c_rt(r) + grad_T[r] T(r)
 * given the forward's fwd_rgb/fwd_T.  grad_T may be NULL (zero).  Same
 * rays/opts as the forward (the dump fields are ignored).  The terms are
 * summed in the scene's workspace (float32 atomics, order not fixed) and then
 * added to `grads`, so backward passes over one scene must not overlap in
 * time (queue them on one stream). */
int grt_trace_backward(const grt_scene *scene, const grt_rays *rays, const grt_trace_opts *opts,
                       const float *fwd_rgb, const float *fwd_T, const float *grad_rgb, const float *grad_T,
                       grt_surfel_grads *grads, void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ environment */

/* Equirectangular environment L_dir (Sec. 3.3 "Light parametrization"):
 * rgb [H,W,3] device; row 0 is the zenith (+y), texel (i,j) spans polar
 * angle [pi i/H, pi (i+1)/H) and azimuth [2pi j/W, 2pi (j+1)/W), azimuth
 * measured from +x towards +z.  Radiance lookups take the nearest texel. */
size_t grt_env_workspace_bytes(int H, int W);
int grt_env_create(grt_ctx *ctx, const float *rgb, int H, int W, void *workspace, size_t ws_bytes, grt_env **out);

/* Build the environment proposal's tables (Sec. 3.4.1: drawn from the
 * intensity distribution of the map, with the texel's solid angle): texel
 * weight = Rec.709 luminance x sin(theta at the texel centre); per-row
 * cumulative sums and the row marginal accumulated left to right in double,
 * divided by the total and rounded to float; last entries exactly 1. */
int grt_env_build(grt_env *env, void *stream);
/* Device pointers to the built tables: marg [H+1], cond [H, W+1]. */
int grt_env_tables(const grt_env *env, const float **marg, const float **cond);

/* Build the prefiltered representation E of the environment that split-sum
 * relighting reads (Sec. 3.5.1, Eq. relight_splitsum), in the environment's
 * workspace.  The map is taken as constant over each texel; every entry is a
 * ratio of sums over all texels (centre direction l, exact solid angle dW),
 * accumulated in double and stored as float:
 *   Ed [16,32,3]   E_d(n) = sum L max(0,n.l) dW / sum max(0,n.l) dW
 *   Es [5,16,32,3] E_s(R,r) = sum L D(h) max(0,R.l) dW / sum D(h) max(0,R.l) dW,
 *                  h = normalize(R + l), GGX D with alpha = r^2, at
 *                  r = 0.2, 0.4, ..., 1.0 (r = 0 is the map itself)
 * on 16 x 32 direction grids (texel centres, the map's convention), and the
 * DFG table lut [32 (n.v), 32 (r), 2] at cell centres: the Schlick split
 *   A = int f_s/F (1 - (1 - v.h)^5) n.l dl,  B = int f_s/F (1 - v.h)^5 n.l dl
 * of the specular directional albedo, integrated over half vectors drawn as
 * D(h) n.h on a 256 x 256 midpoint grid.  Needs no grt_env_build. */
int grt_env_prefilter(grt_env *env, void *stream);
/* Device pointers to the prefiltered tables (layouts above);
 * GRT_ERR_NOT_BUILT before grt_env_prefilter. */
int grt_env_relight_tables(const grt_env *env, const float **Ed, const float **Es, const float **lut);
int grt_env_destroy(grt_env *env);

/* ------------------------------------------------------------ MIS render */

/* Deferred shading state per pixel (Sec. 3.3 "Shading state", Eq.
 * deferred_maps): npix = H*W; x [npix,3] surface point, n [npix,3] unit
 * normal, wo [npix,3] unit direction to the viewer, albedo [npix,3],
 * rough [npix], metal [npix], valid [npix] uint8 (0 = background, shaded 0). */
typedef struct {
    int H, W;
    const float *x;
    const float *n;
    const float *wo;
    const float *albedo;
    const float *rough;
    const float *metal;
    const uint8_t *valid;
} grt_gbuffer;

/* n_cos/n_ggx/n_env: the allocations N_c, N_g, N_e (Sec. 3.4.1; the paper's
 * efficient setting is 16/8/8).  Sample j of pixel p uses the first two
 * words of Philox-4x32-10 with key `seed` and counter (p, j, job, 0), as
 * u = (word >> 8) 2^-24; j < N_c is cosine, then N_g GGX (visible normals,
 * alpha = roughness^2), then N_e environment samples.
 * t_min: self-intersection offset along the secondary ray (1e-3).
 * k: k-nearest hit buffer size per traversal round, one of 1,2,4,8,12,16,32;
 *   grt_render_mis_backward(_shading) also takes 13 (results do not depend
 *   on k; the room workload runs 16 forward, 13 backward, 12 relighting).
 * sample_dump: optional [npix, spp, 10] floats per sample: direction (3),
 *   mixture pdf q, weight f cos/q (3), incident radiance L_i (3); zeros for
 *   samples below the horizon or invalid pixels.
 * hit_list, hit_cap: optional stored hit lists (device memory of
 *   grt_render_hit_list_bytes).  Layout: nray = npix * spp uint32 counts (the
 *   number of hits sample r composited; 0 if not traced), then [nray][hit_cap]
 *   uint32 record positions in compositing order (positions past hit_cap are
 *   not stored).  grt_render_mis writes them; grt_render_mis_backward given
 *   them differentiates from the stored lists instead of re-traversing, and
 *   re-traverses only samples whose count exceeds hit_cap.  NULL: not used.
 * timer: optional kernel timer (grt_timer_create), NULL: none. */
typedef struct grt_timer grt_timer;
typedef struct {
    int n_cos, n_ggx, n_env;
    uint64_t seed;
    uint32_t job;
    float t_min;
    float t_cut;
    int k;
    float *sample_dump;
    uint32_t *hit_list;
    int hit_cap;
    grt_timer *timer;
} grt_mis_opts;

/* Kernel timer: two HIP events that grt_render_mis, grt_render_mis_noalloc
 * and grt_render_mis_backward(_shading) record on their stream around the
 * persistent trace kernel(s) alone (after the sample generation and the
 * coherent-order sort, before the per-pixel reduction or the gradient
 * application), when opts->timer is set; NULL: nothing recorded.  A timer
 * belongs to the context's device; one call at a time may use it.
 * grt_timer_ms waits for the last recording to complete and returns its
 * elapsed milliseconds (GRT_ERR_INVALID if nothing was recorded yet). */
int grt_timer_create(grt_ctx *ctx, grt_timer **out);
int grt_timer_ms(grt_timer *timer, float *ms);
int grt_timer_destroy(grt_timer *timer);

/* Walk statistics (Sec. 3.1 traversal, counted per ray): only a library
 * compiled with -DGRT_STATS keeps them (the default build returns
 * GRT_ERR_INVALID); the counting slows its kernels.  Sums since the last reset,
 * over the context's device, per kernel kind: row 0 the forward radiance trace
 * of grt_render_mis (and _noalloc), row 1 the backward re-traversal of
 * grt_render_mis_backward(_shading).  Columns (GRT_WALK_STATS): rays traced,
 * 4-wide node visits, leaf tests, composited hits, k-buffer rounds, rounds
 * restarted at the root (deferred list dropped), deferred items, wavefront
 * steps, active lanes summed over those steps.  out: host array
 * [2][GRT_WALK_STATS] (caller-owned); reset != 0 zeroes the sums after the
 * read.  Synchronises the device. */
#define GRT_WALK_STATS 9
int grt_walk_stats(grt_ctx *ctx, uint64_t *out, int reset);

/* Bytes of a stored hit list for npix * spp samples (4 * nray * (1 + hit_cap)),
 * 0 on bad arguments. */
size_t grt_render_hit_list_bytes(int64_t npix, int spp, int hit_cap);

/* Bytes of per-sample state the forward saves for grt_render_mis_backward:
 * the composite (c_rt, T) of every sample, then the depth of its last
 * composited hit (the backward's re-traversal stops there). */
size_t grt_render_saved_bytes(int64_t npix, int spp);

/* Bytes of device workspace grt_render_mis and grt_render_mis_backward need:
 * the launch's ray-fetch counters, a 48-byte record per sample (direction,
 * weight f cos/q, environment radiance, written by a generation kernel), a
 * 16-byte contribution per sample, summed per pixel in sample order by a
 * reduction kernel, and 16 bytes per sample plus a histogram for sorting the
 * samples into a coherent traversal order (about 80 bytes per sample).
 * At most 2^31 - 1 samples (H * W * spp) per call. */
size_t grt_render_workspace_bytes(int64_t npix, int spp);

/* c_pbr for every pixel (Eq. mis): out_rgb [npix,3] = (1/N_r) sum_j
 * f(wo, w_j) L_i(w_j) (w_j . n) / q(w_j), L_i = c_rt + T L_env(w_j) from one
 * secondary trace per sample above the horizon.  Per-pixel sums use a fixed
 * order (results are reproducible run to run and independent of scheduling).
 * `saved` (device, >=
 * grt_render_saved_bytes) receives what the backward needs, or NULL. */
int grt_render_mis(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g, const grt_mis_opts *opts,
                   float *out_rgb, void *saved, void *workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * render as grt_render_mis, with its scratch (ray-fetch counters, ray
 * records, contributions, sort buffers: grt_render_workspace_bytes) taken
 * from a fixed device array of GRT_NOALLOC_SCRATCH_BYTES that the library
 * holds per device until the process ends, instead of a workspace argument.
 * It calls no hipMalloc, hipFree or allocating routine.  The caller still
 * passes out_rgb [npix,3] and `saved` (or NULL) as for grt_render_mis; the
 * result is the same bit for bit.  GRT_ERR_INVALID (with the sizes in
 * grt_last_error) when grt_render_workspace_bytes(npix, spp) exceeds the
 * array, i.e. above about 1.6M samples (H * W * spp).  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialized by the caller.  The
 * counters that must start at zero are cleared by the call itself. */
#define GRT_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int grt_render_mis_noalloc(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g,
                           const grt_mis_opts *opts, float *out_rgb, void *saved, void *stream);

/* Backward of grt_render_mis by re-traversal: regenerates every sample from
 * its counter, retraces, and accumulates d/d(surfels) of
 * sum_p grad_rgb[p] . c_pbr(p) into `grads`.  As for grt_trace_backward,
 * the terms are summed in the scene's workspace (atomic adds in no fixed
 * order) and backward passes over one scene must not overlap in time.
 * `saved` must come from the forward with the same scene build,
 * environment, G-buffer and opts. */
int grt_render_mis_backward(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g,
                            const grt_mis_opts *opts, const float *grad_rgb, const void *saved,
                            grt_surfel_grads *grads, void *workspace, size_t ws_bytes, void *stream);

/* Gradients of a loss on the MIS render with respect to the shading state
 * of each pixel (Sec. 3.3, Eq. deferred_maps), so that they can flow on into
 * the G-buffer's own backward (grt_trace_gbuffer_backward).  Each sample's
 * direction and mixture pdf are held fixed, as its hit set is: the estimator
 * is differentiated through the weights f(wo, w) (w . n) / q and through the
 * secondary rays' common origin x, not through the proposals.  Device
 * float32 arrays, [npix,3] or [npix]; every pixel is written (0 where the
 * pixel is invalid or wo . n <= 0); a NULL member is not written.
 *   x:      d/dx of the secondary rays' origin (the hits' geometry moves
 *           with mu - x: minus the sum of their mean gradients)
 *   n, wo:  d/d the stored vectors (they are normalised before use, so the
 *           gradient is orthogonal to them and scales with 1/|n|, 1/|wo|)
 *   albedo, rough, metal: d/d the material maps */
typedef struct {
    float *x;
    float *n;
    float *wo;
    float *albedo;
    float *rough;
    float *metal;
} grt_shading_grads;

/* grt_render_mis_backward (the surfel gradients, accumulated into `grads`
 * exactly as there) plus the shading-state gradients `shade` (overwritten).
 * Same arguments and workspace otherwise; GRT_ERR_INVALID if shade is NULL.
 * With stored hit lists (opts->hit_list) the origin gradients come from the
 * lists, and from the re-traversal for samples whose list overflowed. */
int grt_render_mis_backward_shading(const grt_scene *scene, const grt_env *env, const grt_gbuffer *g,
                                    const grt_mis_opts *opts, const float *grad_rgb, const void *saved,
                                    grt_surfel_grads *grads, const grt_shading_grads *shade, void *workspace,
                                    size_t ws_bytes, void *stream);

/* Relighting under the environment `env` (Sec. 3.5.1): the MIS estimator of
 * grt_render_mis (same samples, same proposals and pdfs from env's tables),
 * with the incident radiance of every traced sample replaced by
 *   L_i = V L_env(w) + (1 - V) SplitSum(a, r, m, n, E)     (Eq. relight_splitsum)
 * where (V, a, r, m, n) is the attribute query of the sample's ray (as
 * grt_trace_attr, surfel attributes `attrs`) and, with v = -w, n the
 * renormalized averaged normal (v if it vanished), R = 2 (n.v) n - v,
 * mu = clamp(n.v, 0, 1), r clamped to [0, 1]:
 *   SplitSum = (1 - m) a E_d(n) + E_s(R, r) (F0 A(mu, r) + B(mu, r)),
 *   F0 = 0.04 (1 - m) + m a,
 * E_d, E_s bilinear in direction over texel centres (wrapping in azimuth,
 * clamped in the polar angle), linear between roughness levels, and A, B
 * bilinear over the DFG table's cell centres (clamped).  env must be built
 * and prefiltered.  opts as for grt_render_mis (no hit lists, no saved state:
 * relighting has no backward).  Same workspace as grt_render_mis. */
int grt_render_relight(const grt_scene *scene, const grt_env *env, const grt_surfel_attrs *attrs,
                       const grt_gbuffer *g, const grt_mis_opts *opts, float *out_rgb, void *workspace,
                       size_t ws_bytes, void *stream);

/* Mesh backend of the attribute query (Sec. 3.5.2, "Mesh-based ray
 * tracing"): a triangle mesh answers Eq. trace_attr by a closest-hit query.
 *   verts [nv,3], tris [nf,3] int32 vertex indices (device, borrowed, not to
 *   change after grt_mesh_build; a triangle with an index outside [0, nv) is
 *   ignored).  0 <= nf <= 2^29.  Workspace: grt_mesh_workspace_bytes(nf),
 *   256-byte aligned (LBVH over the triangles' boxes). */
typedef struct {
    int64_t nv;
    const float *verts;
    int64_t nf;
    const int32_t *tris;
} grt_mesh_desc;
typedef struct grt_mesh grt_mesh;
size_t grt_mesh_workspace_bytes(int64_t nf);
int grt_mesh_create(grt_ctx *ctx, const grt_mesh_desc *mesh, void *workspace, size_t ws_bytes, grt_mesh **out);
int grt_mesh_build(grt_mesh *mesh, void *stream);
int grt_mesh_destroy(grt_mesh *mesh);

/* Per-vertex attributes (device, float32): albedo [nv,3], rough [nv],
 * metal [nv], normal [nv,3]. */
typedef struct {
    const float *albedo;
    const float *rough;
    const float *metal;
    const float *normal;
} grt_vertex_attrs;

/* For every ray (scalar t_min/t_max only), the closest triangle hit with
 * t_min < t <= t_max (two-sided, Moller-Trumbore in float; equal t: the
 * lower triangle index).  A miss: out_V = 1 and zero attributes.  A hit:
 * out_V = 0 and the vertex attributes interpolated with the hit's
 * barycentric weights (1 - u - v, u, v), the normal turned toward the ray
 * origin (not renormalized).  Same outputs as grt_trace_attr, so either
 * backend can answer the query. */
int grt_mesh_trace_attr(const grt_mesh *mesh, const grt_rays *rays, const grt_vertex_attrs *attrs, float *out_V,
                        float *out_albedo, float *out_rough, float *out_metal, float *out_normal, void *stream);

/* Relighting with the mesh backend answering the attribute query (Sec.
 * 3.5.2: Eq. relight_splitsum unchanged, only the query's backend differs):
 * as grt_render_relight, each traced sample's (V, a, r, m, n) coming from
 * grt_mesh_trace_attr's closest-hit query of its ray (t > t_min) against
 * `mesh` with per-vertex `attrs`.  Same opts, workspace and env needs. */
int grt_render_relight_mesh(const grt_mesh *mesh, const grt_env *env, const grt_vertex_attrs *attrs,
                            const grt_gbuffer *g, const grt_mis_opts *opts, float *out_rgb, void *workspace,
                            size_t ws_bytes, void *stream);

/* Cross-bilateral denoiser for low-sample renders (Sec. 3.4.2,
 * "Denoising"), on an H x W image with its guides (device arrays, row-major
 * pixels): rgb [H*W,3] noisy colour, depth [H*W] distance from the camera,
 * normal [H*W,3] (normalized here), valid [H*W] (uint8).  For each valid
 * pixel p, over the valid pixels p' of the (2 radius + 1)^2 window inside the
 * image,
 *   B = exp(-|p-p'|^2 / (2 sigma_s^2))
 *     * exp(-|D(p)-D(p')| / (sigma_d |grad D(p).(p-p')| + eps_d))
 *     * max(0, N(p).N(p'))^sigma_n,
 *   out(p) = sum B c(p') / sum B   (0 if the sum vanishes),
 * with grad D the screen-space depth gradient by central differences
 * (one-sided next to the border or an invalid pixel, 0 with neither
 * neighbour).  Invalid pixels are copied unchanged.  radius 1..8 (pixels);
 * sigma_s > 0 (pixels), sigma_d >= 0, sigma_n >= 0, eps_d > 0 (depth units).
 * Workloads use radius 3, sigma_s 2, sigma_d 1, sigma_n 128, eps_d 0.01.
 * out_rgb [H*W,3] must not overlap the inputs. */
typedef struct {
    int radius;
    float sigma_s;
    float sigma_d;
    float sigma_n;
    float eps_d;
} grt_denoise_opts;
int grt_denoise(grt_ctx *ctx, int H, int W, const float *rgb, const float *depth, const float *normal,
                const uint8_t *valid, const grt_denoise_opts *opts, float *out_rgb, void *stream);

/* ------------------------------------------------------- relighting server */

/* A continuously batched relighting server over a resident built scene
 * (Sec. 3.5.1: relighting evaluates the rendering equation with the MIS
 * density for every pixel of a view under a new environment map).  One
 * scheduler thread runs in epochs: it admits queued requests in arrival order
 * while a slot and room in the device pool are free (uploads, sampling
 * tables and every sample's ray record on a copy stream, overlapping the
 * trace), hands each epoch's ray budget to resident requests in order of
 * deadline (arrival time plus slack_per_ray times the request's ray count,
 * so small requests pass large ones while a large one is never starved), and
 * traces the rays of all of them in one persistent trace launch.  Two
 * epochs are in flight at once on two streams, so the waves of the next
 * epoch fill the tail of the current one.  An epoch of one request's rays
 * (at least 2,097,152) is stopped early when requests with earlier deadlines
 * wait, if the work they add ahead of it stays within preempt_share of its
 * own rays: its waves claim no more rays, and the rest runs after them.
 * Requests that complete are
 * reduced per pixel and copied back.  A request's image equals
 * grt_render_mis with the same inputs and opts (seed, job) whatever it was
 * mixed with.  The scene must not be rebuilt or destroyed while the server
 * exists.
 *
 * mem_budget:    device bytes of the request pool (inside the workspace).
 * max_jobs:      requests resident at once (1..256).
 * epoch_rays:    at most this many rays per epoch (0 = 134,217,728); an epoch
 *                takes the rest of the earliest-deadline request, plus the
 *                next requests while the epoch stays within 4,194,304 rays.
 *                One epoch runs at a time (the next starts once the one in
 *                flight is done, or stopped).
 * k:             k-buffer size, 4, 8, 12 or 16.  t_min, t_cut as in grt_mis_opts.
 * k_relight:     k-buffer size of relighting epochs, 4, 8, 12 or 16 (0 = k).
 * slack_per_ray: seconds of deadline per ray (0 = arrival order only;
 *                negative = 4e-8, about twice a request's time alone).
 * preempt_share: rays that more urgent requests may run ahead of a started
 *                request by stopping its epochs, as a share of its own rays
 *                (0 or negative = never stop an epoch).  Stopping lowers the
 *                mean latency under load and raises the largest ones.
 * attrs:         per-surfel materials (device, borrowed for the server's
 *                life) for camera and relighting requests; all NULL = such
 *                requests are refused.
 * workspace:     device memory the caller owns (e.g. a torch tensor), 256-byte
 *                aligned, at least grt_server_workspace_bytes(opts) bytes,
 *                borrowed until grt_server_destroy returns: the request pool,
 *                the epochs' job and chunk tables and their claim counters,
 *                and the DFG table that every relighting request shares (it
 *                depends on nothing but its resolution, so the server builds
 *                it once) all live there (the server allocates no device
 *                memory; it holds a few pinned host buffers of tables and
 *                flags).
 * co_trace:      nonzero: when the earliest-deadline request has not started,
 *                the requests of the same kind waiting with the very same
 *                G-buffer (the same arrays and size) are traced with it in
 *                one epoch, all their samples in one joint coherent order
 *                (direction bin, then origin cell): up to 16 requests, at
 *                most 2^26 samples in all (and within epoch_rays), while the
 *                epoch's buffers fit the pool (the joint order and its sort,
 *                and a copy of the samples' records in that order: 104
 *                bytes a sample for relighting, 92 for radiance).  Each
 *                image is the same as traced alone.  Every member finishes
 *                with the group, so the earliest request waits for the
 *                others: 0 keeps requests in deadline order. */
typedef struct {
    size_t mem_budget;
    int max_jobs;
    int64_t epoch_rays;
    int k;
    float t_min;
    float t_cut;
    double slack_per_ray;
    double preempt_share;
    grt_surfel_attrs attrs;
    void *workspace;
    size_t ws_bytes;
    int co_trace;
    int k_relight;
} grt_server_opts;

/* Device bytes grt_server_create needs in opts->workspace for these opts
 * (mem_budget plus the epoch tables); 0 if max_jobs or mem_budget is out of
 * range. */
size_t grt_server_workspace_bytes(const grt_server_opts *opts);

/* A request.  Pointers may be host or device memory, borrowed until the
 * request is done (pinned host memory lets uploads overlap compute).
 * G-buffer arrays as in grt_gbuffer; env_rgb [env_H, env_W, 3] as in
 * grt_env_create; sample allocation and random identity as in grt_mis_opts;
 * out_rgb [H*W*3] (host or device) receives c_pbr.
 * relight = 0: the radiance estimator of grt_render_mis under the request's
 * environment (the surfels' stored radiance, L_i = c_rt + T L_env).
 * relight != 0: relighting under the request's environment (Sec. 3.5.1):
 * the attribute query of the server's surfel materials and the split-sum
 * shading of Eq. relight_splitsum, as grt_render_relight; the image equals
 * grt_render_relight with the same inputs and opts whatever it was mixed
 * with.  An epoch holds requests of one kind, and relighting epochs are never
 * stopped early.
 * Camera request (camera_request != 0): the G-buffer pointers are ignored
 * (may be NULL).  The server traces the request's G-buffer from `camera` on
 * its upload stream, as grt_camera_rays followed by grt_trace_gbuffer (the
 * server's attrs, k and t_cut, coverage at min_opacity in (0, 1]), and then
 * renders it like an uploaded one: the image equals grt_render_mis on that
 * traced G-buffer. */
typedef struct {
    int H, W;
    const float *x;
    const float *n;
    const float *wo;
    const float *albedo;
    const float *rough;
    const float *metal;
    const uint8_t *valid;
    const float *env_rgb;
    int env_H, env_W;
    int n_cos, n_ggx, n_env;
    uint64_t seed;
    uint32_t job;
    float *out_rgb;
    int camera_request;
    grt_camera camera;
    float min_opacity;
    int relight;
} grt_job;

/* Pool bytes a request occupies while resident (0 if malformed). */
size_t grt_server_job_bytes(const grt_job *job);

int grt_server_create(grt_ctx *ctx, const grt_scene *scene, const grt_server_opts *opts, grt_server **out);

/* Queue a request; *id identifies it.  GRT_ERR_ADMISSION if it can never fit
 * the memory budget, GRT_ERR_INVALID if malformed, GRT_ERR_BUSY if 4,096
 * requests are already queued. */
int grt_server_submit(grt_server *server, const grt_job *job, uint64_t *id);

/* *state: 0 queued, 1 uploading, 2 running, 3 done, or the failing status
 * (GRT_ERR_CANCELLED, GRT_ERR_DEVICE). */
int grt_server_poll(grt_server *server, uint64_t id, int *state);

/* Block until the request is done (returns its status) or timeout_s seconds
 * pass (GRT_ERR_TIMEOUT).  The server remembers the last 65,536 finished
 * requests; older ids are unknown (GRT_ERR_INVALID) to poll, wait and
 * job_times. */
int grt_server_wait(grt_server *server, uint64_t id, double timeout_s);

/* Cancel a request: removed if queued, dropped at the next epoch boundary if
 * resident (its pool memory is freed then). */
int grt_server_cancel(grt_server *server, uint64_t id);

/* Seconds since the server was created at which the request was submitted,
 * started running (-1 if not yet) and finished (-1 if not yet). */
int grt_server_job_times(grt_server *server, uint64_t id, double *submit_s, double *start_s, double *done_s);

/* Epochs run, epochs stopped early for a more urgent request (their
 * unclaimed rays ran in later epochs), rays traced, and free pool bytes.
 * Any pointer may be NULL. */
int grt_server_stats(grt_server *server, uint64_t *epochs, uint64_t *stopped, int64_t *rays, size_t *pool_free);

/* Stop the scheduler (after its current epoch), cancel what is left, free
 * the pool. */
int grt_server_destroy(grt_server *server);

#ifdef __cplusplus
}
#endif

#endif /* GRT_H */
