// trace.hip -- Trace(r_o, r_d) forward and its backward by re-traversal.
//
// Forward (Sec. 3.2, Eq. trace): the hits of a ray arrive from the ordered
// traversal in ascending (tau, id); each one composites
//   C += T alpha c,  T <- T (1 - alpha),  alpha = o exp(-rho^2 / 2)
// until T < t_cut (that hit included).  Returns c_rt = C and T = 1 - o_rt.
//
// Backward: with the forward's C and T_fin known, the same traversal
// replays the hits in the same order and, per hit k,
//   dL/dc_k     = T_k alpha_k g_C
//   dL/dalpha_k = T_k (g_C . c_k) - [g_C . (C - P_k) + g_T T_fin] / (1 - alpha_k)
// (P_k = colour composited through hit k), then chains alpha -> (o, u, v)
// -> (s_u, s_v, mu, t_u, t_v, n) -> q, and adds the 13 parameter gradients of
// the surfel to its line of the scene's gradient buffer (device atomics,
// staged per wavefront so that one instruction updates whole lines).
//
// Both kernels run persistent wavefronts that fetch rays dynamically.
#include <cmath>

#include "grt_internal.h"
#include "grt_kernels.h"
#include "grt_render.h"

namespace grt {

__global__ void k_zero_counters(unsigned long long *c)
{
    if (threadIdx.x < kCounterBytes / sizeof(unsigned long long)) c[threadIdx.x] = 0ull;
}

hipError_t launch_zero_counters(unsigned long long *c, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, c);
    return hipGetLastError();
}

template <int K>
struct TraceJob {
    const TraceArgs &a;
    SceneDev S;
    Walker<K> w;
    CompositeVisit<false> v;

    __device__ TraceJob(const TraceArgs &a_) : a(a_), S(a_.S), v(a_.S, a_.tcut) {}
    __device__ __forceinline__ Walker<K> &walker() { return w; }
    __device__ __forceinline__ CompositeVisit<false> &visit() { return v; }

    __device__ __forceinline__ bool begin(int64_t r)
    {
        const float3 o = make_float3(a.o[3 * r], a.o[3 * r + 1], a.o[3 * r + 2]);
        const float3 d = make_float3(a.d[3 * r], a.d[3 * r + 1], a.d[3 * r + 2]);
        const float tmin = a.tmin_a ? fmaxf(a.tmin_a[r], 0.0f) : a.tmin;  // negative: 0
        const float tmax = a.tmax_a ? a.tmax_a[r] : a.tmax;
        v.reset();
        if (a.dump_id) { v.did = a.dump_id + r * a.cap; v.dtau = a.dump_tau + r * a.cap; v.cap = a.cap; }
        w.start(S, o, d, tmin, tmax);
        if (S.n <= 0) {
            finish(r);
            return false;
        }
        return true;
    }

    __device__ __forceinline__ void finish(int64_t r)
    {
        a.out_rgb[3 * r] = v.C.x; a.out_rgb[3 * r + 1] = v.C.y; a.out_rgb[3 * r + 2] = v.C.z;
        a.out_T[r] = v.T;
        if (a.out_L) {
            float3 Le = make_float3(a.sky[0], a.sky[1], a.sky[2]);
            if (a.env_rgb) {  // L_env at the nearest texel of the direction (Eq. lighting_decompose)
                EnvDev E{};
                E.H = a.env_H; E.W = a.env_W; E.rgb = a.env_rgb;
                Le = env_radiance(E, v3(a.d[3 * r], a.d[3 * r + 1], a.d[3 * r + 2]));
            }
            a.out_L[3 * r] = v.C.x + v.T * Le.x;
            a.out_L[3 * r + 1] = v.C.y + v.T * Le.y;
            a.out_L[3 * r + 2] = v.C.z + v.T * Le.z;
        }
        if (a.out_nhit) a.out_nhit[r] = v.cnt;
        if (a.stop_depth) a.stop_depth[r] = w.stop_depth();
        if (a.dump_id)
            for (int i = v.cnt; i < a.cap; ++i) { v.did[i] = -1; v.dtau[i] = 0.0f; }
    }
    __device__ __forceinline__ void after_step() {}
    __device__ __forceinline__ void drain() {}
};

template <int K>
struct TraceBwdJob {
    const TraceBwdArgs &a;
    SceneDev S;
    BwdWalker<K> w;
    GradVisit v;

    __device__ TraceBwdJob(const TraceBwdArgs &a_, WaveStage *t) : a(a_), S(a_.f.S), v(a_.f.S, a_.f.tcut, a_.g)
    {
        v.stage = t;
        stage_init(t);
    }
    __device__ __forceinline__ BwdWalker<K> &walker() { return w; }
    __device__ __forceinline__ GradVisit &visit() { return v; }

    __device__ __forceinline__ bool begin(int64_t r)
    {
        if (S.n <= 0) return false;
        const float3 gC = make_float3(a.grad_rgb[3 * r], a.grad_rgb[3 * r + 1], a.grad_rgb[3 * r + 2]);
        const float gT = a.grad_T ? a.grad_T[r] : 0.0f;
        if (gC.x == 0.0f && gC.y == 0.0f && gC.z == 0.0f && gT == 0.0f) return false;
        const float3 o = make_float3(a.f.o[3 * r], a.f.o[3 * r + 1], a.f.o[3 * r + 2]);
        const float3 d = make_float3(a.f.d[3 * r], a.f.d[3 * r + 1], a.f.d[3 * r + 2]);
        const float tmin = a.f.tmin_a ? fmaxf(a.f.tmin_a[r], 0.0f) : a.f.tmin;  // negative: 0
        const float tmax = a.f.tmax_a ? a.f.tmax_a[r] : a.f.tmax;
        const float3 C = make_float3(a.fwd_rgb[3 * r], a.fwd_rgb[3 * r + 1], a.fwd_rgb[3 * r + 2]);
        v.reset(gC, gT, C, a.fwd_T[r]);
        w.start(S, o, d, tmin, stop_bound(a.f.stop_depth, r, tmax));
        return true;
    }

    __device__ __forceinline__ void finish(int64_t) {}
    __device__ __forceinline__ void after_step() { stage_sync(a.g.acc, v.stage, false); }
    __device__ __forceinline__ void drain() { stage_sync(a.g.acc, v.stage, true); }
};

template <int K>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_trace(TraceArgs a)
{
    TraceJob<K> job(a);
    run_persistent<K>(job, a.counters, a.n);
}

// Attribute query (Eq. trace_attr): the trace's traversal with the attribute
// payload; outputs the visibility and the normalized-weight attributes.
template <int K>
struct TraceAttrJob {
    const TraceAttrArgs &a;
    SceneDev S;
    Walker<K> w;
    AttrVisit v;

    __device__ TraceAttrJob(const TraceAttrArgs &a_)
        : a(a_), S(a_.f.S), v(a_.f.S, a_.f.tcut, a_.albedo, a_.rough, a_.metal) {}
    __device__ __forceinline__ Walker<K> &walker() { return w; }
    __device__ __forceinline__ AttrVisit &visit() { return v; }

    __device__ __forceinline__ bool begin(int64_t r)
    {
        const float3 o = make_float3(a.f.o[3 * r], a.f.o[3 * r + 1], a.f.o[3 * r + 2]);
        const float3 d = make_float3(a.f.d[3 * r], a.f.d[3 * r + 1], a.f.d[3 * r + 2]);
        const float tmin = a.f.tmin_a ? fmaxf(a.f.tmin_a[r], 0.0f) : a.f.tmin;  // negative: 0
        const float tmax = a.f.tmax_a ? a.f.tmax_a[r] : a.f.tmax;
        v.reset();
        w.start(S, o, d, tmin, tmax);
        if (S.n <= 0) {
            finish(r);
            return false;
        }
        return true;
    }

    __device__ __forceinline__ void finish(int64_t r)
    {
        const float inv = v.W > 0.0f ? 1.0f / v.W : 0.0f;
        a.out_V[r] = v.T;
        a.out_albedo[3 * r] = v.A.x * inv; a.out_albedo[3 * r + 1] = v.A.y * inv; a.out_albedo[3 * r + 2] = v.A.z * inv;
        a.out_rough[r] = v.R * inv;
        a.out_metal[r] = v.M * inv;
        a.out_normal[3 * r] = v.N.x * inv; a.out_normal[3 * r + 1] = v.N.y * inv; a.out_normal[3 * r + 2] = v.N.z * inv;
    }
    __device__ __forceinline__ void after_step() {}
    __device__ __forceinline__ void drain() {}
};

// Primary-ray G-buffer (Eq. deferred_maps by 2DGRT): the attribute query
// with the depth and colour maps; a pixel is covered when its accumulated
// opacity reaches min_opacity (and its averaged normal does not vanish).
template <int K>
struct TraceGBufJob {
    const TraceGBufArgs &a;
    SceneDev S;
    Walker<K> w;
    GBufVisit v;

    __device__ TraceGBufJob(const TraceGBufArgs &a_)
        : a(a_), S(a_.f.S), v(a_.f.S, a_.f.tcut, a_.albedo, a_.rough, a_.metal) {}
    __device__ __forceinline__ Walker<K> &walker() { return w; }
    __device__ __forceinline__ GBufVisit &visit() { return v; }

    __device__ __forceinline__ bool begin(int64_t r)
    {
        const float3 o = make_float3(a.f.o[3 * r], a.f.o[3 * r + 1], a.f.o[3 * r + 2]);
        const float3 d = make_float3(a.f.d[3 * r], a.f.d[3 * r + 1], a.f.d[3 * r + 2]);
        const float tmin = a.f.tmin_a ? fmaxf(a.f.tmin_a[r], 0.0f) : a.f.tmin;  // negative: 0
        const float tmax = a.f.tmax_a ? a.f.tmax_a[r] : a.f.tmax;
        v.reset();
        w.start(S, o, d, tmin, tmax);
        if (S.n <= 0) {
            finish(r);
            return false;
        }
        return true;
    }

    __device__ __forceinline__ void finish(int64_t r)
    {
        const float inv = v.W > 0.0f ? 1.0f / v.W : 0.0f;
        const float3 N = make_float3(v.N.x * inv, v.N.y * inv, v.N.z * inv);
        const float nl = sqrtf(N.x * N.x + N.y * N.y + N.z * N.z);
        const bool ok = v.W > 0.0f && 1.0f - v.T >= a.min_opacity && nl > 0.0f;
        const float in = ok ? 1.0f / nl : 0.0f, D = ok ? v.Dsum * inv : 0.0f, m = ok ? inv : 0.0f;
        a.x[3 * r] = ok ? w.o.x + D * w.d.x : 0.0f;  // the walker holds the ray
        a.x[3 * r + 1] = ok ? w.o.y + D * w.d.y : 0.0f;
        a.x[3 * r + 2] = ok ? w.o.z + D * w.d.z : 0.0f;
        a.n[3 * r] = N.x * in; a.n[3 * r + 1] = N.y * in; a.n[3 * r + 2] = N.z * in;
        a.wo[3 * r] = ok ? -w.d.x : 0.0f; a.wo[3 * r + 1] = ok ? -w.d.y : 0.0f; a.wo[3 * r + 2] = ok ? -w.d.z : 0.0f;
        a.out_albedo[3 * r] = v.A.x * m; a.out_albedo[3 * r + 1] = v.A.y * m; a.out_albedo[3 * r + 2] = v.A.z * m;
        a.out_rough[r] = v.R * m;
        a.out_metal[r] = v.M * m;
        a.depth[r] = D;
        a.rgb[3 * r] = v.Csum.x * m; a.rgb[3 * r + 1] = v.Csum.y * m; a.rgb[3 * r + 2] = v.Csum.z * m;
        a.valid[r] = ok ? 1 : 0;
        if (a.weight) a.weight[r] = ok ? v.W : 0.0f;
        if (a.nlen) a.nlen[r] = ok ? nl : 0.0f;
        if (a.f.stop_depth) a.f.stop_depth[r] = w.stop_depth();
    }
    __device__ __forceinline__ void after_step() {}
    __device__ __forceinline__ void drain() {}
};

template <int K>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_trace_gbuffer(TraceGBufArgs a)
{
    TraceGBufJob<K> job(a);
    run_persistent<K>(job, a.f.counters, a.f.n);
}

template <int K>
static hipError_t go_trace_gbuffer(const TraceGBufArgs &a, int num_cu, hipStream_t st)
{
    const int nb = persistent_blocks(k_trace_gbuffer<K>, num_cu, a.f.n);
    hipLaunchKernelGGL(k_trace_gbuffer<K>, dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_trace_gbuffer(const TraceGBufArgs &a, int k, int num_cu, hipStream_t st)
{
    if (a.f.n <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.f.counters, st);
    if (e != hipSuccess) return e;
    switch (k) {
    case 1: return go_trace_gbuffer<1>(a, num_cu, st);
    case 2: return go_trace_gbuffer<2>(a, num_cu, st);
    case 4: return go_trace_gbuffer<4>(a, num_cu, st);
    case 8: return go_trace_gbuffer<8>(a, num_cu, st);
    case 12: return go_trace_gbuffer<12>(a, num_cu, st);
    case 16: return go_trace_gbuffer<16>(a, num_cu, st);
    case 32: return go_trace_gbuffer<32>(a, num_cu, st);
    default: return hipErrorInvalidValue;
    }
}

// ---- pinhole camera rays ----------------------------------------------------
// Every quantity is formed in double in the order the ABI states, with
// contraction off, so the rays equal that formula evaluated on any IEEE
// machine and rounded to float.

static bool normalize3(const double v[3], double out[3])
{
#pragma clang fp contract(off)
    const double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!(l > 0.0) || !std::isfinite(l)) return false;
    for (int c = 0; c < 3; ++c) out[c] = v[c] / l;
    return true;
}

static void cross3(const double a[3], const double b[3], double out[3])
{
#pragma clang fp contract(off)
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

bool make_pinhole(const double eye[3], const double target[3], const double up[3], double vfov_deg, int H, int W,
                  PinholeDev &c)
{
#pragma clang fp contract(off)
    if (H <= 0 || W <= 0 || !(vfov_deg > 0.0 && vfov_deg < 180.0)) return false;
    const double v[3] = {target[0] - eye[0], target[1] - eye[1], target[2] - eye[2]};
    double rr[3];
    if (!normalize3(v, c.f)) return false;
    cross3(c.f, up, rr);
    if (!normalize3(rr, c.r)) return false;
    cross3(c.r, c.f, c.u);
    for (int k = 0; k < 3; ++k) c.eye[k] = eye[k];
    c.t = tan(vfov_deg * (M_PI / 180.0) * 0.5);
    c.aspect = (double)W / (double)H;
    return true;
}

__global__ void k_camera_rays(PinholeDev c, int H, int W, float *o, float *d)
{
#pragma clang fp contract(off)
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p % W);
    const double sx = (((double)j + 0.5) / (double)W * 2.0 - 1.0) * c.t * c.aspect;
    const double sy = (1.0 - ((double)i + 0.5) / (double)H * 2.0) * c.t;
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = c.f[k] + sx * c.r[k] + sy * c.u[k];
    const double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; ++k) {
        d[3 * p + k] = (float)(v[k] / l);
        o[3 * p + k] = (float)c.eye[k];
    }
}

hipError_t launch_camera_rays(const PinholeDev &c, int H, int W, float *o, float *d, hipStream_t st)
{
    const int64_t n = (int64_t)H * W;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_camera_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, c, H, W, o, d);
    return hipGetLastError();
}

// Backward of the primary-ray G-buffer by re-traversal: the same hits as the
// forward, with the per-ray constants of GBufGradVisit from the forward's
// maps; uncovered pixels (constant maps) are skipped.
template <int K>
struct TraceGBufBwdJob {
    const TraceGBufBwdArgs &a;
    SceneDev S;
    BwdWalker<K> w;
    GBufGradVisit v;

    __device__ TraceGBufBwdJob(const TraceGBufBwdArgs &a_, WaveStage *t) : a(a_), S(a_.f.S), v(a_.f.S, a_.f.tcut, a_.g)
    {
        v.albedo = a.albedo; v.rough = a.rough; v.metal = a.metal;
        v.ga_albedo = a.ga_albedo; v.ga_rough = a.ga_rough; v.ga_metal = a.ga_metal;
        v.stage = t;
        stage_init(t);
    }
    __device__ __forceinline__ BwdWalker<K> &walker() { return w; }
    __device__ __forceinline__ GBufGradVisit &visit() { return v; }

    static __device__ __forceinline__ float3 ld3(const float *p, int64_t r)
    {
        return p ? make_float3(p[3 * r], p[3 * r + 1], p[3 * r + 2]) : make_float3(0.f, 0.f, 0.f);
    }

    __device__ __forceinline__ bool begin(int64_t r)
    {
        if (S.n <= 0 || !a.fwd_valid[r]) return false;
        const float Wt = a.fwd_weight[r], nl = a.fwd_nlen[r];
        if (!(Wt > 0.0f) || !(nl > 0.0f)) return false;
        const float3 o = make_float3(a.f.o[3 * r], a.f.o[3 * r + 1], a.f.o[3 * r + 2]);
        const float3 d = make_float3(a.f.d[3 * r], a.f.d[3 * r + 1], a.f.d[3 * r + 2]);
        const float3 gx = ld3(a.g_x, r), gn = ld3(a.g_n, r), gA = ld3(a.g_albedo, r), gC = ld3(a.g_rgb, r);
        const float gR = a.g_rough ? a.g_rough[r] : 0.0f, gM = a.g_metal ? a.g_metal[r] : 0.0f;
        // x = o + D d: the hit-point map moves with the depth only
        const float gD = (a.g_depth ? a.g_depth[r] : 0.0f) + dot3(gx, d);
        if (gD == 0.0f && gR == 0.0f && gM == 0.0f && gn.x == 0.0f && gn.y == 0.0f && gn.z == 0.0f &&
            gA.x == 0.0f && gA.y == 0.0f && gA.z == 0.0f && gC.x == 0.0f && gC.y == 0.0f && gC.z == 0.0f)
            return false;
        const float iW = 1.0f / Wt;
        v.kD = gD * iW; v.kR = gR * iW; v.kM = gM * iW;
        v.kA = make_float3(gA.x * iW, gA.y * iW, gA.z * iW);
        v.kC = make_float3(gC.x * iW, gC.y * iW, gC.z * iW);
        const float3 A = ld3(a.fwd_albedo, r), C = ld3(a.fwd_rgb, r), nh = ld3(a.fwd_n, r);
        v.e0 = v.kD * a.fwd_depth[r] + dot3(v.kA, A) + v.kR * a.fwd_rough[r] + v.kM * a.fwd_metal[r] + dot3(v.kC, C);
        // d(N/|N|)/dN applied to g_n, with |N| = W |N / W|
        const float ndg = dot3(nh, gn), iN = iW / nl;
        v.kN = make_float3((gn.x - nh.x * ndg) * iN, (gn.y - nh.y * ndg) * iN, (gn.z - nh.z * ndg) * iN);
        const float tmin = a.f.tmin_a ? fmaxf(a.f.tmin_a[r], 0.0f) : a.f.tmin;  // negative: 0
        const float tmax = a.f.tmax_a ? a.f.tmax_a[r] : a.f.tmax;
        v.reset();
        w.start(S, o, d, tmin, stop_bound(a.f.stop_depth, r, tmax));
        return true;
    }

    __device__ __forceinline__ void finish(int64_t) {}
    __device__ __forceinline__ void after_step() { stage_sync(a.g.acc, v.stage, false); }
    __device__ __forceinline__ void drain() { stage_sync(a.g.acc, v.stage, true); }
};

template <int K>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_trace_gbuffer_bwd(TraceGBufBwdArgs a)
{
    __shared__ WaveStage stages[4];
    TraceGBufBwdJob<K> job(a, &stages[(threadIdx.x >> 6) & 3]);
    run_persistent<K>(job, a.f.counters, a.f.n);
}

template <int K>
static hipError_t go_trace_gbuffer_bwd(const TraceGBufBwdArgs &a, int num_cu, hipStream_t st)
{
    const int nb = persistent_blocks(k_trace_gbuffer_bwd<K>, num_cu, a.f.n);
    hipLaunchKernelGGL(k_trace_gbuffer_bwd<K>, dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_trace_gbuffer_backward(const TraceGBufBwdArgs &a, int k, int num_cu, hipStream_t st)
{
    if (a.f.n <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.f.counters, st);
    if (e != hipSuccess) return e;
    switch (k) {
    case 1: return go_trace_gbuffer_bwd<1>(a, num_cu, st);
    case 2: return go_trace_gbuffer_bwd<2>(a, num_cu, st);
    case 4: return go_trace_gbuffer_bwd<4>(a, num_cu, st);
    case 8: return go_trace_gbuffer_bwd<8>(a, num_cu, st);
    case 12: return go_trace_gbuffer_bwd<12>(a, num_cu, st);
    case 16: return go_trace_gbuffer_bwd<16>(a, num_cu, st);
    case 32: return go_trace_gbuffer_bwd<32>(a, num_cu, st);
    default: return hipErrorInvalidValue;
    }
}

template <int K>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_trace_attr(TraceAttrArgs a)
{
    TraceAttrJob<K> job(a);
    run_persistent<K>(job, a.f.counters, a.f.n);
}

template <int K>
static hipError_t go_trace_attr(const TraceAttrArgs &a, int num_cu, hipStream_t st)
{
    const int nb = persistent_blocks(k_trace_attr<K>, num_cu, a.f.n);
    hipLaunchKernelGGL(k_trace_attr<K>, dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_trace_attr(const TraceAttrArgs &a, int k, int num_cu, hipStream_t st)
{
    if (a.f.n <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.f.counters, st);
    if (e != hipSuccess) return e;
    switch (k) {
    case 1: return go_trace_attr<1>(a, num_cu, st);
    case 2: return go_trace_attr<2>(a, num_cu, st);
    case 4: return go_trace_attr<4>(a, num_cu, st);
    case 8: return go_trace_attr<8>(a, num_cu, st);
    case 12: return go_trace_attr<12>(a, num_cu, st);
    case 16: return go_trace_attr<16>(a, num_cu, st);
    case 32: return go_trace_attr<32>(a, num_cu, st);
    default: return hipErrorInvalidValue;
    }
}

template <int K>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_trace_bwd(TraceBwdArgs a)
{
    __shared__ WaveStage stages[4];
    TraceBwdJob<K> job(a, &stages[(threadIdx.x >> 6) & 3]);
    run_persistent<K>(job, a.f.counters, a.f.n);
}

template <int K>
static hipError_t go_trace(const TraceArgs &a, int num_cu, hipStream_t st)
{
    const int nb = persistent_blocks(k_trace<K>, num_cu, a.n);
    hipLaunchKernelGGL(k_trace<K>, dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int K>
static hipError_t go_trace_bwd(const TraceBwdArgs &a, int num_cu, hipStream_t st)
{
    const int nb = persistent_blocks(k_trace_bwd<K>, num_cu, a.f.n);
    hipLaunchKernelGGL(k_trace_bwd<K>, dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs &a, int k, int num_cu, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.counters, st);
    if (e != hipSuccess) return e;
    switch (k) {
    case 1: return go_trace<1>(a, num_cu, st);
    case 2: return go_trace<2>(a, num_cu, st);
    case 4: return go_trace<4>(a, num_cu, st);
    case 8: return go_trace<8>(a, num_cu, st);
    case 12: return go_trace<12>(a, num_cu, st);
    case 16: return go_trace<16>(a, num_cu, st);
    case 32: return go_trace<32>(a, num_cu, st);
    default: return hipErrorInvalidValue;
    }
}

// Gradient lines: 16 floats per surfel, terms in the order
// (mu xyz, s_u, s_v, q wxyz, opacity, rgb).
__global__ void k_grad_lines_zero(float4 *acc, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_grad_lines_apply(GradPtrs g, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 *l = reinterpret_cast<const float4 *>(g.acc) + 4 * i;
    const float4 a0 = l[0], a1 = l[1], a2 = l[2], a3 = l[3];
    g.means[3 * i] += a0.x;
    g.means[3 * i + 1] += a0.y;
    g.means[3 * i + 2] += a0.z;
    g.scales[2 * i] += a0.w;
    g.scales[2 * i + 1] += a1.x;
    g.quats[4 * i] += a1.y;
    g.quats[4 * i + 1] += a1.z;
    g.quats[4 * i + 2] += a1.w;
    g.quats[4 * i + 3] += a2.x;
    g.opacity[i] += a2.y;
    g.rgb[3 * i] += a2.z;
    g.rgb[3 * i + 1] += a2.w;
    g.rgb[3 * i + 2] += a3.x;
}

hipError_t launch_grad_lines_zero(float *acc, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t n4 = 4 * n;
    hipLaunchKernelGGL(k_grad_lines_zero, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<float4 *>(acc), n4);
    return hipGetLastError();
}

hipError_t launch_grad_lines_apply(const GradPtrs &g, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_lines_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, n);
    return hipGetLastError();
}

hipError_t launch_trace_backward(const TraceBwdArgs &a, int k, int num_cu, hipStream_t st)
{
    if (a.f.n <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.f.counters, st);
    if (e != hipSuccess) return e;
    switch (k) {
    case 1: return go_trace_bwd<1>(a, num_cu, st);
    case 2: return go_trace_bwd<2>(a, num_cu, st);
    case 4: return go_trace_bwd<4>(a, num_cu, st);
    case 8: return go_trace_bwd<8>(a, num_cu, st);
    case 12: return go_trace_bwd<12>(a, num_cu, st);
    case 16: return go_trace_bwd<16>(a, num_cu, st);
    case 32: return go_trace_bwd<32>(a, num_cu, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace grt
