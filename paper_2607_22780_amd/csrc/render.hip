// render.hip -- environment tables and the fused MIS render (forward and
// backward by re-traversal).
//
// One ray per (pixel, sample): a generation kernel draws every sample and
// writes its ray record, persistent wavefronts trace them (fetching rays
// dynamically), and a reduction sums each pixel.  Per sample (Sec. 3.3 Eq.
// montecarlo, Sec. 3.4.1 Eq. mis):
//   u1,u2  <- Philox-4x32-10(key = seed, counter = (pixel, j, job, 0))
//   w      <- cosine (j < N_c) | GGX visible normal (j < N_c+N_g) | env texel
//   q      =  (N_c p_c + N_g p_g + N_e p_e) / N_r          (balance heuristic)
//   if w.n > 0:  (C, T) <- Trace(x, w);  L_i = C + T L_env(w)   (Eqs. incident_trace, lighting_decompose)
//                g/q = f(wo, w) L_i (w.n) / q              (Eqs. brdf_decompose, brdf_specular)
// is written per sample; a second kernel sums each pixel's samples in sample
// order, so the estimate (1/N_r) sum g/q is reproducible run to run and does
// not depend on other pixels or on the scheduling.
#include "grt_render.h"

namespace grt {

constexpr float kPi = 3.14159265358979323846f;

// ---------------------------------------------------------------------------
// Environment proposal tables: texel weight = luminance x sin(theta_centre);
// cumulative sums in double, left to right, rounded to float at the end.
// ---------------------------------------------------------------------------
__global__ void k_env_rows(int H, int W, const float *__restrict__ rgb, float *__restrict__ cond,
                           double *__restrict__ rows)
{
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= H) return;
    const double st = sin(3.14159265358979323846 * (i + 0.5) / H);
    double acc = 0.0;
    for (int j = 0; j < W; ++j) {
        const float *p = rgb + ((size_t)i * W + j) * 3;
        double lum = 0.2126 * (double)p[0] + 0.7152 * (double)p[1] + 0.0722 * (double)p[2];
        acc += lum * st;
    }
    rows[i] = acc;
    float *cr = cond + (size_t)i * (W + 1);
    cr[0] = 0.0f;
    double run = 0.0;
    for (int j = 0; j < W; ++j) {
        const float *p = rgb + ((size_t)i * W + j) * 3;
        double lum = 0.2126 * (double)p[0] + 0.7152 * (double)p[1] + 0.0722 * (double)p[2];
        run += lum * st;
        cr[j + 1] = acc > 0.0 ? (float)(run / acc) : (float)((double)(j + 1) / W);
    }
    cr[W] = 1.0f;
}

__global__ void k_env_marginal(int H, const double *__restrict__ rows, float *__restrict__ marg)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double tot = 0.0;
    for (int i = 0; i < H; ++i) tot += rows[i];
    double acc = 0.0;
    marg[0] = 0.0f;
    for (int i = 0; i < H; ++i) {
        acc += rows[i];
        marg[i + 1] = tot > 0.0 ? (float)(acc / tot) : (float)((double)(i + 1) / H);
    }
    marg[H] = 1.0f;
}

hipError_t launch_env_build(const float *rgb, int H, int W, const EnvWS &w, hipStream_t st)
{
    hipLaunchKernelGGL(k_env_rows, dim3((H + 63) / 64), dim3(64), 0, st, H, W, rgb, w.cond, w.rows);
    hipLaunchKernelGGL(k_env_marginal, dim3(1), dim3(64), 0, st, H, w.rows, w.marg);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Prefiltered environment for split-sum relighting (Eq. relight_splitsum).
// The environment is piecewise constant over its texels; each table entry is
// a ratio of sums over all texels (centre direction l, exact solid angle dW)
// accumulated in double:
//   E_d(n)    = sum L max(0, n.l) dW / sum max(0, n.l) dW
//   E_s(R, r) = sum L D(h) max(0, R.l) dW / sum D(h) max(0, R.l) dW,
//               h = normalize(R + l), GGX D with alpha = r^2.
// One wavefront per table texel: lanes split the environment's texels, then
// a fixed-order tree in LDS sums the lanes.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_env_prefilter(int H, int W, const float *__restrict__ rgb,
                                                      float *__restrict__ Ed, float *__restrict__ Es)
{
#pragma clang fp contract(off)
    constexpr int kAcc = 4 + 4 * (kPfL - 1);  // diffuse (L, weight), then each level
    __shared__ double part[kAcc][64];
    const int t = blockIdx.x, lane = threadIdx.x;
    const double tth = kPiD * ((t / kPfW) + 0.5) / kPfH, tph = 2.0 * kPiD * ((t % kPfW) + 0.5) / kPfW;
    const V3 nt = v3(sin(tth) * cos(tph), cos(tth), sin(tth) * sin(tph));
    double acc[kAcc];
#pragma unroll
    for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;
    for (int k = lane; k < H * W; k += 64) {
        const int i = k / W, j = k - i * W;
        const double th = kPiD * (i + 0.5) / H, ph = 2.0 * kPiD * (j + 0.5) / W;
        const V3 l = v3(sin(th) * cos(ph), cos(th), sin(th) * sin(ph));
        const double c = dot(nt, l);
        if (!(c > 0.0)) continue;
        const double om = 2.0 * kPiD / W * (cos(kPiD * i / H) - cos(kPiD * (i + 1) / H));
        const float *L = rgb + (size_t)k * 3;
        const double w = c * om;
        acc[0] += w * L[0]; acc[1] += w * L[1]; acc[2] += w * L[2]; acc[3] += w;
        const double ndh = dot(nt, normalized(v3(nt.x + l.x, nt.y + l.y, nt.z + l.z)));
#pragma unroll
        for (int lv = 1; lv < kPfL; ++lv) {
            const double r = (double)lv / (kPfL - 1), al = r * r;
            const double wl = ggx_D(ndh, al * al) * w;
            double *s = acc + 4 * lv;
            s[0] += wl * L[0]; s[1] += wl * L[1]; s[2] += wl * L[2]; s[3] += wl;
        }
    }
#pragma unroll
    for (int q = 0; q < kAcc; ++q) part[q][lane] = acc[q];
    __syncthreads();
    for (int half = 32; half > 0; half >>= 1) {
        if (lane < half)
            for (int q = 0; q < kAcc; ++q) part[q][lane] += part[q][lane + half];
        __syncthreads();
    }
    if (lane < 3) {
        Ed[t * 3 + lane] = part[3][0] > 0.0 ? (float)(part[lane][0] / part[3][0]) : 0.0f;
        for (int lv = 1; lv < kPfL; ++lv) {
            const double wsum = part[4 * lv + 3][0];
            Es[((size_t)(lv - 1) * kPfH * kPfW + t) * 3 + lane] = wsum > 0.0 ? (float)(part[4 * lv + lane][0] / wsum) : 0.0f;
        }
    }
}

// DFG table: per cell (n.v = mu, roughness r at cell centres), the Schlick
// split of the specular directional albedo (F = 1),
//   A = E[g (1 - (1 - v.h)^5)],  B = E[g (1 - v.h)^5],  g = G (v.h) / (mu n.h),
// over half vectors h distributed as D(h) n.h (the inverse GGX distribution
// on a kLutQ x kLutQ midpoint grid of (xi, azimuth)), l = reflect(v, h) above
// the horizon.  One workgroup per cell, one azimuth row per thread, a
// fixed-order tree over the rows.
__global__ void __launch_bounds__(256) k_dfg_lut(float *__restrict__ lut)
{
#pragma clang fp contract(off)
    static_assert(kLutQ == 256, "one thread per quadrature row");
    __shared__ double pa[256], pb[256];
    const int cell = blockIdx.x, i = cell / kLutN, j = cell % kLutN, s = threadIdx.x;
    const double mu = (i + 0.5) / kLutN, r = (j + 0.5) / kLutN, al = r * r, a2 = al * al;
    const V3 v = v3(sqrt(1.0 - mu * mu), 0.0, mu);
    const double xi = (s + 0.5) / kLutQ;
    const double c2 = (1.0 - xi) / (1.0 + (a2 - 1.0) * xi);
    const double ct = sqrt(c2), st = sqrt(1.0 - c2 > 0.0 ? 1.0 - c2 : 0.0);
    const double g1v = smith_G1(mu, a2);
    double A = 0.0, B = 0.0;
    for (int t = 0; t < kLutQ; ++t) {
        const double ph = 2.0 * kPiD * (t + 0.5) / kLutQ;
        const V3 h = v3(st * cos(ph), st * sin(ph), ct);
        const double vh = dot(v, h);
        if (!(vh > 0.0)) continue;
        const double nl = 2.0 * vh * h.z - v.z;
        if (!(nl > 0.0)) continue;
        const double g = smith_G1(nl, a2) * g1v * vh / (mu * ct);
        const double x = 1.0 - vh, fc = x * x * x * x * x;
        A += g * (1.0 - fc);
        B += g * fc;
    }
    pa[s] = A;
    pb[s] = B;
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if (s < half) { pa[s] += pa[s + half]; pb[s] += pb[s + half]; }
        __syncthreads();
    }
    if (s == 0) {
        lut[2 * cell] = (float)(pa[0] / ((double)kLutQ * kLutQ));
        lut[2 * cell + 1] = (float)(pb[0] / ((double)kLutQ * kLutQ));
    }
}

hipError_t launch_env_prefilter(const float *rgb, int H, int W, const EnvWS &w, hipStream_t st, bool lut)
{
    hipLaunchKernelGGL(k_env_prefilter, dim3(kPfH * kPfW), dim3(64), 0, st, H, W, rgb, w.Ed, w.Es);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !lut) return e;
    return launch_dfg_lut(w.lut, st);
}

hipError_t launch_dfg_lut(float *lut, hipStream_t st)
{
    hipLaunchKernelGGL(k_dfg_lut, dim3(kLutN * kLutN), dim3(256), 0, st, lut);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_render_gen(RenderArgs a)
{
    const int64_t total = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= total) return;
    gen_ray(a, r);
}

// ---------------------------------------------------------------------------
// Jobs for the persistent loop.  Ray index order keeps a wavefront's chunk on
// neighbouring pixels (shared origins, nearby surfaces).
// ---------------------------------------------------------------------------
template <int K, bool kHitList>
struct RenderJob {
    static constexpr int kStatSlot = 0;  // walk statistics (instrumented build)
    const RenderArgs &a;
    SceneDev S;
    ShadeTrace<K, kHitList> t;
    int64_t r;  // sample index of the lane's ray

    __device__ RenderJob(const RenderArgs &a_) : a(a_), S(a_.S), r(0) { t.bind(a, S); }
    __device__ __forceinline__ Walker<K> &walker() { return t.w; }
    __device__ __forceinline__ decltype(t.v) &visit() { return t.v; }
    __device__ __forceinline__ bool begin(int64_t g)
    {
        r = a.order ? (int64_t)a.order[g] : g;
        return t.begin(a, S, r);
    }
    __device__ __forceinline__ void finish(int64_t) { t.finish(a, r); }
    __device__ __forceinline__ void after_step() {}
    __device__ __forceinline__ void drain() {}
};

// Relighting (Sec. 3.5.1), first pass: the forward render's job with the
// attribute query instead of the radiance trace (RelightTrace parks each
// traced sample's query result for the shading pass).
template <int K>
struct RelightJob {
    const RenderArgs &a;
    SceneDev S;
    RelightTrace<K> t;
    int64_t r;

    __device__ RelightJob(const RenderArgs &a_) : a(a_), S(a_.S), r(0) { t.bind(a, S); }
    __device__ __forceinline__ Walker<K> &walker() { return t.w; }
    __device__ __forceinline__ AttrVisit &visit() { return t.v; }
    __device__ __forceinline__ bool begin(int64_t g)
    {
        r = a.order ? (int64_t)a.order[g] : g;
        return t.begin(a, S, r);
    }
    __device__ __forceinline__ void finish(int64_t) { t.finish(a, r); }
    __device__ __forceinline__ void after_step() {}
    __device__ __forceinline__ void drain() {}
};

// Relighting, second pass (one thread per sample): the incident radiance
// V L_env(w) + (1 - V) SplitSum(a, r, m, n, E) (Eq. relight_splitsum) of each
// traced sample from its parked query, weighted by f cos / q.
__global__ void __launch_bounds__(256) k_relight_shade(RenderArgs a, int64_t total)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= total) return;
    const float4 r0 = a.rays[3 * r];
    if (r0.w == 0.0f) return;  // untraced: its contribution is already 0
    const float4 r1 = a.rays[3 * r + 1], r2 = a.rays[3 * r + 2], q = a.contrib[r];
    const double V = q.x;
    V3 L = v3((double)r1.w * V, (double)r2.x * V, (double)r2.y * V);
    if (V < 1.0) {
        const V3 ss = split_sum(a.E, v3(q.y, q.z, q.w), r2.z, r2.w, v3(a.rl_nx[r], a.rl_ny[r], a.rl_nz[r]),
                                v3(r0.x, r0.y, r0.z));
        L = v3(L.x + (1.0 - V) * ss.x, L.y + (1.0 - V) * ss.y, L.z + (1.0 - V) * ss.z);
    }
    a.contrib[r] = make_float4((float)(r1.x * L.x), (float)(r1.y * L.y), (float)(r1.z * L.z), 0.0f);
    if (a.dump) {
        float *dp = a.dump + r * 10;
        dp[7] = (float)L.x; dp[8] = (float)L.y; dp[9] = (float)L.z;
    }
}

// kOrigin: also write each sample's origin gradient to a.gorig (zero for a
// sample that contributes nothing; samples done from stored hit lists are
// left to that kernel).
template <int K, bool kOrigin>
struct RenderBwdJob {
    static constexpr int kStatSlot = 1;  // walk statistics (instrumented build)
    const RenderArgs &a;
    SceneDev S;
    BwdWalker<K> w;
    GradVisitT<kOrigin> v;
    int spp;

    __device__ RenderBwdJob(const RenderArgs &a_, WaveStage *t)
        : a(a_), S(a_.S), v(a_.S, a_.tcut, a_.g), spp(a_.nc + a_.ng + a_.ne)
    {
        v.stage = t;
        stage_init(t);
    }
    __device__ __forceinline__ BwdWalker<K> &walker() { return w; }
    __device__ __forceinline__ GradVisitT<kOrigin> &visit() { return v; }

    __device__ __forceinline__ bool skip(int64_t r)
    {
        if constexpr (kOrigin) a.gorig[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        return false;
    }

    __device__ __forceinline__ bool begin(int64_t g)
    {
        const int64_t r = a.order ? (int64_t)a.order[g] : g;
        if (S.n <= 0) return skip(r);
        const float4 r0 = a.rays[3 * r];
        if (r0.w == 0.0f) return skip(r);
        if (a.hits && a.hits[r] <= (uint32_t)a.hcap) return false;  // done from its stored list
        const int64_t p = r / spp;
        const float inv = 1.0f / (float)spp;
        const float3 gp = make_float3(a.grad[3 * p] * inv, a.grad[3 * p + 1] * inv, a.grad[3 * p + 2] * inv);
        if (gp.x == 0.0f && gp.y == 0.0f && gp.z == 0.0f) return skip(r);
        const float4 r1 = a.rays[3 * r + 1], r2 = a.rays[3 * r + 2];
        const float3 gC = make_float3(r1.x * gp.x, r1.y * gp.y, r1.z * gp.z);
        const float gT = gC.x * r1.w + gC.y * r2.x + gC.z * r2.y;
        const float4 sv = a.saved[r];
        const float3 x = make_float3(a.x[3 * p], a.x[3 * p + 1], a.x[3 * p + 2]);
        const float3 d = make_float3(r0.x, r0.y, r0.z);
        v.reset(gC, gT, make_float3(sv.x, sv.y, sv.z), sv.w);
        w.start(S, x, d, a.tmin, stop_bound(a.saved_t, r, INFINITY));
        if constexpr (kOrigin) cur = r;
        return true;
    }

    __device__ __forceinline__ void finish(int64_t)
    {
        if constexpr (kOrigin) a.gorig[cur] = make_float4(-v.gmu.x, -v.gmu.y, -v.gmu.z, 0.0f);
    }
    __device__ __forceinline__ void after_step() { stage_sync(a.g.acc, v.stage, false); }
    __device__ __forceinline__ void drain() { stage_sync(a.g.acc, v.stage, true); }

    int64_t cur = 0;  // the lane's sample (kOrigin)
};

// kHitList: the launch stores hit lists (a.hits set); a separate kernel, so
// that the plain forward carries no list pointer in its registers.
template <int K, bool kHitList>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_render(RenderArgs a)
{
    RenderJob<K, kHitList> job(a);
    run_persistent<K>(job, a.counters, (int64_t)a.H * a.W * (a.nc + a.ng + a.ne));
}

// The forward with a 12-hit buffer fits 3 wavefronts per SIMD (168 VGPRs)
// when the compiler is held to it; it then beats K = 8 (fewer rounds).
#ifndef GRT_FWD12_WAVES
#define GRT_FWD12_WAVES 3
#endif
template <int K, bool kHitList>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GRT_FWD12_WAVES))) k_render_w3(RenderArgs a)
{
    RenderJob<K, kHitList> job(a);
    run_persistent<K>(job, a.counters, (int64_t)a.H * a.W * (a.nc + a.ng + a.ne));
}

template <int K>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_render_relight(RenderArgs a)
{
    RelightJob<K> job(a);
    run_persistent<K>(job, a.counters, (int64_t)a.H * a.W * (a.nc + a.ng + a.ne));
}

template <int K>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_render_relight_w3(RenderArgs a)
{
    RelightJob<K> job(a);
    run_persistent<K>(job, a.counters, (int64_t)a.H * a.W * (a.nc + a.ng + a.ne));
}

template <int K, bool kOrigin>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_render_bwd(RenderArgs a)
{
    __shared__ WaveStage stages[4];
    RenderBwdJob<K, kOrigin> job(a, &stages[(threadIdx.x >> 6) & 3]);
    run_persistent<K>(job, a.counters, (int64_t)a.H * a.W * (a.nc + a.ng + a.ne));
}

// The re-traversal with a 13-hit buffer fits 3 wavefronts per SIMD (168
// VGPRs) when the compiler is held to it, and then beats K = 12.
template <int K, bool kOrigin>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_render_bwd_w3(RenderArgs a)
{
    __shared__ WaveStage stages[4];
    RenderBwdJob<K, kOrigin> job(a, &stages[(threadIdx.x >> 6) & 3]);
    run_persistent<K>(job, a.counters, (int64_t)a.H * a.W * (a.nc + a.ng + a.ne));
}

// Backward from stored hit lists: one thread per sample runs the gradient of
// its composited hits in order (no traversal).  Samples whose list
// overflowed are left to the re-traversal kernel.  The wavefront steps
// through the lists together, one hit per lane per step, so that its staged
// terms are flushed at wavefront-uniform points.  kOrigin: also writes each
// sample's origin gradient (overflowed samples: by the re-traversal).
template <bool kOrigin>
__global__ void __launch_bounds__(256) k_render_bwd_stored(RenderArgs a)
{
    __shared__ WaveStage stages[4];
    WaveStage *stage = &stages[(threadIdx.x >> 6) & 3];
    stage_init(stage);
    const int spp = a.nc + a.ng + a.ne;
    const int64_t nray = (int64_t)a.H * a.W * spp;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // samples in traversal order: a wavefront's rays are neighbours and share surfels
    const int64_t r = g < nray ? (a.order ? (int64_t)a.order[g] : g) : 0;
    const uint32_t nh = g < nray && a.S.n > 0 ? a.hits[r] : 0u;
    const float4 r0 = nh ? a.rays[3 * r] : make_float4(0.f, 0.f, 0.f, 0.f);
    GradVisitT<kOrigin> v(a.S, a.tcut, a.g);
    v.stage = stage;
    v.gmu = make_float3(0.f, 0.f, 0.f);
    uint32_t cnt = 0;
    float3 x = make_float3(0.f, 0.f, 0.f), d = x;
    const uint32_t *list = a.hits + nray + r * a.hcap;
    if (nh > 0u && nh <= (uint32_t)a.hcap && r0.w != 0.0f) {
        const int64_t p = r / spp;
        const float inv = 1.0f / (float)spp;
        const float3 gp = make_float3(a.grad[3 * p] * inv, a.grad[3 * p + 1] * inv, a.grad[3 * p + 2] * inv);
        if (gp.x != 0.0f || gp.y != 0.0f || gp.z != 0.0f) {
            const float4 r1 = a.rays[3 * r + 1], r2 = a.rays[3 * r + 2];
            const float3 gC = make_float3(r1.x * gp.x, r1.y * gp.y, r1.z * gp.z);
            const float gT = gC.x * r1.w + gC.y * r2.x + gC.z * r2.y;
            const float4 sv = a.saved[r];
            x = make_float3(a.x[3 * p], a.x[3 * p + 1], a.x[3 * p + 2]);
            d = make_float3(r0.x, r0.y, r0.z);
            v.reset(gC, gT, make_float3(sv.x, sv.y, sv.z), sv.w);
            cnt = nh;
        }
    }
    for (uint32_t i = 0; __ballot(i < cnt); ++i) {
        if (i < cnt) visit_hit(v, a.S.rec, list[i], x, d);
        stage_sync(a.g.acc, stage, false);
    }
    stage_sync(a.g.acc, stage, true);
    if constexpr (kOrigin) {
        if (g < nray && !(nh > (uint32_t)a.hcap && r0.w != 0.0f))
            a.gorig[r] = make_float4(-v.gmu.x, -v.gmu.y, -v.gmu.z, 0.0f);
    }
}

// Gradients of the loss with respect to each pixel's shading state (x, the
// stored normal and view direction, albedo, roughness, metallic), each
// sample's direction and mixture pdf held fixed; one thread per pixel, its
// samples in order.  The sample's weight f (n.w) / q is differentiated from
// the regenerated direction and pdf (in double), its incident radiance L_i =
// c_rt + T L_env comes from the forward's saved state, and x moves every
// secondary ray's origin (the per-sample origin gradients of the backward
// pass, a.gorig).  Unit n and wo are the stored vectors over their lengths,
// so their gradients are projected off the unit vector and divided by them.
__global__ void __launch_bounds__(256) k_render_shade_grad(RenderArgs a, ShadeGradOut o)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)a.H * a.W) return;
    const int spp = a.nc + a.ng + a.ne;
    ShadeGrad g{};
    double gx[3] = {0.0, 0.0, 0.0};
    Shade s;
    const bool lit = load_pixel(a, p, s);
    if (lit) {
        const double gp[3] = {a.grad[3 * p], a.grad[3 * p + 1], a.grad[3 * p + 2]};
        for (int j = 0; j < spp; ++j) {
            const int64_t r = p * spp + j;
            if (a.rays[3 * r].w == 0.0f) continue;  // below the horizon: not traced
            const float4 go = a.gorig[r];
            gx[0] += go.x; gx[1] += go.y; gx[2] += go.z;
            V3 w;
            float3 wf, wt;
            double q;
            draw(a, s, p, j, w, wf, q, wt);
            if (!(q > 0.0)) continue;
            const float4 sv = a.saved[r], r1 = a.rays[3 * r + 1], r2 = a.rays[3 * r + 2];
            const float Li[3] = {sv.x + sv.w * r1.w, sv.y + sv.w * r2.x, sv.z + sv.w * r2.y};
            double u[3];
            for (int c = 0; c < 3; ++c) u[c] = gp[c] * (double)Li[c] / ((double)spp * q);
            brdf_cos_backward(s.n, s.wo, w, s.alb, s.rough, s.metal, u, g);
        }
    }
    V3 gn = v3(0.0, 0.0, 0.0), gw = gn;
    if (lit) {
        const double ln = sqrt((double)a.n[3 * p] * a.n[3 * p] + (double)a.n[3 * p + 1] * a.n[3 * p + 1] +
                               (double)a.n[3 * p + 2] * a.n[3 * p + 2]);
        const double lo = sqrt((double)a.wo[3 * p] * a.wo[3 * p] + (double)a.wo[3 * p + 1] * a.wo[3 * p + 1] +
                               (double)a.wo[3 * p + 2] * a.wo[3 * p + 2]);
        const double pn = dot(s.n, g.n), po = dot(s.wo, g.wo);
        gn = v3((g.n.x - s.n.x * pn) / ln, (g.n.y - s.n.y * pn) / ln, (g.n.z - s.n.z * pn) / ln);
        gw = v3((g.wo.x - s.wo.x * po) / lo, (g.wo.y - s.wo.y * po) / lo, (g.wo.z - s.wo.z * po) / lo);
    }
    auto put3 = [&](float *dst, double x, double y, double z) {
        if (dst) { dst[3 * p] = (float)x; dst[3 * p + 1] = (float)y; dst[3 * p + 2] = (float)z; }
    };
    put3(o.x, gx[0], gx[1], gx[2]);
    put3(o.n, gn.x, gn.y, gn.z);
    put3(o.wo, gw.x, gw.y, gw.z);
    put3(o.alb, g.alb.x, g.alb.y, g.alb.z);
    if (o.rough) o.rough[p] = (float)g.rough;
    if (o.metal) o.metal[p] = (float)g.metal;
}

hipError_t launch_render_shade_grad(const RenderArgs &a, const ShadeGradOut &o, hipStream_t st)
{
    const int64_t npix = (int64_t)a.H * a.W;
    if (npix <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_render_shade_grad, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, a, o);
    return hipGetLastError();
}

__global__ void k_render_reduce(int64_t npix, int spp, const float4 *__restrict__ contrib, float *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    reduce_pixel(p, spp, contrib, out);
}

template <int K, bool kHitList>
static hipError_t go_render_as(const RenderArgs &a, int num_cu, hipStream_t st)
{
    const int64_t total = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    if constexpr (K == 12 || K == 16) {
        const int nb = persistent_blocks(k_render_w3<K, kHitList>, num_cu, total);
        hipLaunchKernelGGL((k_render_w3<K, kHitList>), dim3(nb), dim3(256), 0, st, a);
    } else {
        const int nb = persistent_blocks(k_render<K, kHitList>, num_cu, total);
        hipLaunchKernelGGL((k_render<K, kHitList>), dim3(nb), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

template <int K>
static hipError_t go_render(const RenderArgs &a, int num_cu, hipStream_t st)
{
    return a.hits ? go_render_as<K, true>(a, num_cu, st) : go_render_as<K, false>(a, num_cu, st);
}

// (the shading-state variant, kOrigin, keeps the plain kernel: it carries
// the origin gradient too and would spill at 3 wavefronts per SIMD)
template <int K, bool kOrigin>
static hipError_t go_render_bwd_as(const RenderArgs &a, int num_cu, hipStream_t st)
{
    const int64_t total = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    if constexpr (K == 13 && !kOrigin) {
        const int nb = persistent_blocks(k_render_bwd_w3<K, kOrigin>, num_cu, total);
        hipLaunchKernelGGL((k_render_bwd_w3<K, kOrigin>), dim3(nb), dim3(256), 0, st, a);
    } else {
        const int nb = persistent_blocks(k_render_bwd<K, kOrigin>, num_cu, total);
        hipLaunchKernelGGL((k_render_bwd<K, kOrigin>), dim3(nb), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

template <int K>
static hipError_t go_render_bwd(const RenderArgs &a, int num_cu, hipStream_t st)
{
    return a.gorig ? go_render_bwd_as<K, true>(a, num_cu, st) : go_render_bwd_as<K, false>(a, num_cu, st);
}

static hipError_t timer_mark(const KernelTimer *tm, bool end, hipStream_t st)
{
    return tm ? hipEventRecord(end ? tm->end : tm->begin, st) : hipSuccess;
}

hipError_t launch_render_backward_stored(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st,
                                         const KernelTimer *tm)
{
    const int64_t nray = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    if (nray <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.counters, st);
    if (e != hipSuccess) return e;
    if ((e = launch_render_gen(a, st)) != hipSuccess) return e;
    if (a.order && (e = launch_ray_order(a, w, st)) != hipSuccess) return e;
    if ((e = timer_mark(tm, false, st)) != hipSuccess) return e;
    if (a.gorig)
        hipLaunchKernelGGL(k_render_bwd_stored<true>, dim3((unsigned)((nray + 255) / 256)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_render_bwd_stored<false>, dim3((unsigned)((nray + 255) / 256)), dim3(256), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // samples whose list overflowed: re-traverse (the others return at once)
    RenderArgs b = a;
    b.order = nullptr;
    switch (k) {
    case 1: e = go_render_bwd<1>(b, num_cu, st); break;
    case 2: e = go_render_bwd<2>(b, num_cu, st); break;
    case 4: e = go_render_bwd<4>(b, num_cu, st); break;
    case 8: e = go_render_bwd<8>(b, num_cu, st); break;
    case 12: e = go_render_bwd<12>(b, num_cu, st); break;
    case 13: e = go_render_bwd<13>(b, num_cu, st); break;
    case 16: e = go_render_bwd<16>(b, num_cu, st); break;
    case 32: e = go_render_bwd<32>(b, num_cu, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return timer_mark(tm, true, st);
}

hipError_t launch_render_gen(const RenderArgs &a, hipStream_t st)
{
    const int64_t total = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    hipLaunchKernelGGL(k_render_gen, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---- coherent traversal order ------------------------------------------------
// Samples of one pixel leave in all directions, so index order hands a
// wavefront 64 unrelated rays.  Sorting by (direction bin, origin cell) gives
// each wavefront rays that walk nearly the same nodes, which the per-XCD L2
// then serves.  The order changes only which lane traces which ray: every
// result is written at its sample index.

__device__ __forceinline__ uint32_t spread3(uint32_t x)  // 6 bits -> every third bit
{
    x &= 63u;
    x = (x | (x << 8)) & 0x0000F00Fu;
    x = (x | (x << 4)) & 0x000C30C3u;
    x = (x | (x << 2)) & 0x00249249u;
    return x;
}

__global__ void __launch_bounds__(256) k_ray_keys(RenderArgs a, int n, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals, uint32_t tag)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float4 r0 = a.rays[3 * (int64_t)r];
    uint32_t key = 0xFFFFFFu;  // untraced samples go last
    if (r0.w != 0.0f) {
        // scene root box from the two child boxes of node 0
        const Node nd = a.S.nodes[0];
        const float lx = fminf(nd.a.x, nd.b.z), ly = fminf(nd.a.y, nd.b.w), lz = fminf(nd.a.z, nd.c.x);
        const float hx = fmaxf(nd.a.w, nd.c.y), hy = fmaxf(nd.b.x, nd.c.z), hz = fmaxf(nd.b.y, nd.c.w);
        const int spp = a.nc + a.ng + a.ne;
        const int64_t p = (int64_t)r / spp;
        auto cell = [](float v, float lo, float hi) -> uint32_t {
            const float t = (v - lo) / fmaxf(hi - lo, 1e-20f) * 64.0f;
            return (uint32_t)fminf(fmaxf(t, 0.0f), 63.0f);
        };
        const uint32_t m = (spread3(cell(a.x[3 * p], lx, hx)) << 2) | (spread3(cell(a.x[3 * p + 1], ly, hy)) << 1) |
                           spread3(cell(a.x[3 * p + 2], lz, hz));
        // octahedral direction bin, 8 x 8
        const float s = fabsf(r0.x) + fabsf(r0.y) + fabsf(r0.z);
        float u = r0.x / s, v = r0.z / s;
        if (r0.y < 0.0f) {
            const float uu = (1.0f - fabsf(v)) * (u >= 0.0f ? 1.0f : -1.0f);
            const float vv = (1.0f - fabsf(u)) * (v >= 0.0f ? 1.0f : -1.0f);
            u = uu;
            v = vv;
        }
        const uint32_t iu = (uint32_t)fminf(fmaxf((u * 0.5f + 0.5f) * 8.0f, 0.0f), 7.0f);
        const uint32_t iv = (uint32_t)fminf(fmaxf((v * 0.5f + 0.5f) * 8.0f, 0.0f), 7.0f);
        key = ((iv * 8u + iu) << 18) | m;
    }
    keys[r] = key;
    vals[r] = tag | (uint32_t)r;
}

hipError_t launch_ray_keys(const RenderArgs &a, int n, uint32_t *keys, uint32_t *vals, uint32_t tag, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ray_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, keys, vals, tag);
    return hipGetLastError();
}

hipError_t launch_ray_order(const RenderArgs &a, const RenderWS &w, hipStream_t st)
{
    const int64_t n = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    if (n <= 0 || a.S.n < 2) return hipSuccess;
    hipLaunchKernelGGL(k_ray_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, (int)n, w.k0, w.v0, 0u);
    // 24-bit keys: three passes leave the order in (k1, v1)
    launch_radix_sort((int)n, 3, w.k0, w.v0, w.k1, w.v1, w.hist, st);
    return hipGetLastError();
}

hipError_t launch_render(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st,
                         const KernelTimer *tm)
{
    const int64_t npix = (int64_t)a.H * a.W;
    if (npix <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.counters, st);
    if (e != hipSuccess) return e;
    if ((e = launch_render_gen(a, st)) != hipSuccess) return e;
    if (a.order && (e = launch_ray_order(a, w, st)) != hipSuccess) return e;
    if ((e = timer_mark(tm, false, st)) != hipSuccess) return e;
    switch (k) {
    case 1: e = go_render<1>(a, num_cu, st); break;
    case 2: e = go_render<2>(a, num_cu, st); break;
    case 4: e = go_render<4>(a, num_cu, st); break;
    case 8: e = go_render<8>(a, num_cu, st); break;
    case 12: e = go_render<12>(a, num_cu, st); break;
    case 16: e = go_render<16>(a, num_cu, st); break;
    case 32: e = go_render<32>(a, num_cu, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if ((e = timer_mark(tm, true, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_render_reduce, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, npix,
                       a.nc + a.ng + a.ne, a.contrib, a.out);
    return hipGetLastError();
}

template <int K>
static hipError_t go_relight(const RenderArgs &a, int num_cu, hipStream_t st)
{
    const int64_t total = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    if constexpr (K == 12) {
        const int nb = persistent_blocks(k_render_relight_w3<K>, num_cu, total);
        hipLaunchKernelGGL(k_render_relight_w3<K>, dim3(nb), dim3(256), 0, st, a);
    } else {
        const int nb = persistent_blocks(k_render_relight<K>, num_cu, total);
        hipLaunchKernelGGL(k_render_relight<K>, dim3(nb), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_render_relight(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st)
{
    const int64_t npix = (int64_t)a.H * a.W;
    if (npix <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.counters, st);
    if (e != hipSuccess) return e;
    if ((e = launch_render_gen(a, st)) != hipSuccess) return e;
    if (a.order && (e = launch_ray_order(a, w, st)) != hipSuccess) return e;
    switch (k) {
    case 1: e = go_relight<1>(a, num_cu, st); break;
    case 2: e = go_relight<2>(a, num_cu, st); break;
    case 4: e = go_relight<4>(a, num_cu, st); break;
    case 8: e = go_relight<8>(a, num_cu, st); break;
    case 12: e = go_relight<12>(a, num_cu, st); break;
    case 16: e = go_relight<16>(a, num_cu, st); break;
    case 32: e = go_relight<32>(a, num_cu, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const int64_t total = npix * (a.nc + a.ng + a.ne);
    hipLaunchKernelGGL(k_relight_shade, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, total);
    hipLaunchKernelGGL(k_render_reduce, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, npix,
                       a.nc + a.ng + a.ne, a.contrib, a.out);
    return hipGetLastError();
}

hipError_t launch_relight_shade(const RenderArgs &a, hipStream_t st)
{
    const int64_t total = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_relight_shade, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, total);
    return hipGetLastError();
}

hipError_t launch_render_relight_mesh(const RenderArgs &a, const MeshTraceArgs &m, hipStream_t st)
{
    const int64_t npix = (int64_t)a.H * a.W;
    if (npix <= 0) return hipSuccess;
    hipError_t e = launch_render_gen(a, st);
    if (e != hipSuccess) return e;
    if ((e = launch_mesh_relight_query(a, m, st)) != hipSuccess) return e;
    const int64_t total = npix * (a.nc + a.ng + a.ne);
    hipLaunchKernelGGL(k_relight_shade, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, total);
    hipLaunchKernelGGL(k_render_reduce, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, npix,
                       a.nc + a.ng + a.ne, a.contrib, a.out);
    return hipGetLastError();
}

hipError_t launch_render_backward(const RenderArgs &a, const RenderWS &w, int k, int num_cu, hipStream_t st,
                                  const KernelTimer *tm)
{
    if ((int64_t)a.H * a.W <= 0) return hipSuccess;
    hipError_t e = launch_zero_counters(a.counters, st);
    if (e != hipSuccess) return e;
    if ((e = launch_render_gen(a, st)) != hipSuccess) return e;
    if (a.order && (e = launch_ray_order(a, w, st)) != hipSuccess) return e;
    if ((e = timer_mark(tm, false, st)) != hipSuccess) return e;
    switch (k) {
    case 1: e = go_render_bwd<1>(a, num_cu, st); break;
    case 2: e = go_render_bwd<2>(a, num_cu, st); break;
    case 4: e = go_render_bwd<4>(a, num_cu, st); break;
    case 8: e = go_render_bwd<8>(a, num_cu, st); break;
    case 12: e = go_render_bwd<12>(a, num_cu, st); break;
    case 13: e = go_render_bwd<13>(a, num_cu, st); break;
    case 16: e = go_render_bwd<16>(a, num_cu, st); break;
    case 32: e = go_render_bwd<32>(a, num_cu, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return timer_mark(tm, true, st);
}

bool walk_stats_built()
{
#ifdef GRT_STATS
    return true;
#else
    return false;
#endif
}

hipError_t walk_stats_read(unsigned long long *out, bool reset)
{
#ifdef GRT_STATS
    hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_walk_stats), sizeof(g_walk_stats));
    if (e == hipSuccess && reset) {
        unsigned long long zero[2][kNumWalkStats] = {};
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_walk_stats), zero, sizeof(zero));
    }
    return e;
#else
    (void)out;
    (void)reset;
    return hipErrorNotSupported;
#endif
}

}  // namespace grt
