// grt_kernels.h -- per-hit work shared by the trace and render kernels:
// front-to-back compositing (forward) and its gradient (backward).
#pragma once

#include "grt_internal.h"

namespace grt {

// Forward compositing (Sec. 3.2, Eq. trace; Eq. alpha_blending along the ray).
// Where to stop is decided on the transmittance of the canonical
// single-precision alphas (Td); the composited values use alphas from the
// double-precision crossing.  kHitList: the visitor also records the record
// positions of the composited hits in the ray's stored hit list (hl); the
// plain forward carries no list pointer at all.
template <bool kHitList>
struct CompositeVisit {
    const float4 *rec;
    const float4 *col;
    float tcut;
    float3 C;
    float T, Td;
    int cnt;
    int32_t *did = nullptr;
    float *dtau = nullptr;
    int cap = 0;
    uint32_t *hl = nullptr;  // stored hit list of the ray (record positions)
    int hcap = 0;

    __device__ CompositeVisit() {}
    __device__ CompositeVisit(const SceneDev &S, float t_cut) : rec(S.rec), col(S.col), tcut(t_cut) {}

    __device__ __forceinline__ void reset()
    {
        C = make_float3(0.f, 0.f, 0.f);
        T = 1.0f;
        Td = 1.0f;
        cnt = 0;
    }

    // Hit p (record r0..r3, canonical rho^2 crho2) of the ray, in order;
    // true when compositing stops after it.
    __device__ __forceinline__ bool operator()(uint32_t p, uint32_t id, float tau, const float4 r0, const float4 r1,
                                               const float4 r2, const float4 r3, float crho2, const float3 o,
                                               const float3 d)
    {
        const float4 c = col[p];
        HitGeo g;
        value_geo(r0, r1, r2, r3, o, d, g);
        const float a = r1.w * expf(-0.5f * g.rho2);
        const float w = T * a;
        C.x += w * c.x; C.y += w * c.y; C.z += w * c.z;
        if (did && cnt < cap) { did[cnt] = (int32_t)id; dtau[cnt] = tau; }
        if (kHitList && hl && cnt < hcap) hl[cnt] = p;
        ++cnt;
        T = T * (1.0f - a);
        Td = trans_step(Td, hit_alpha(r1.w, crho2));
        return Td < tcut;
    }
};

__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Attribute query of a ray (Eq. trace_attr, Gaussian backend): along the same
// ordered hits and cut-off as the radiance trace, the material attributes of
// the composited surfels summed with blending weights w = T alpha (Eq.
// deferred_maps), each normal turned to face the ray origin; the caller
// normalizes by the summed weight.  T ends as the visibility V of the
// environment.
struct AttrVisit {
    const float4 *rec;
    const float *albedo, *rough, *metal;  // per surfel id
    float tcut;
    float T, Td, W, R, M;
    float3 A, N;

    __device__ AttrVisit() {}
    __device__ AttrVisit(const SceneDev &S, float t_cut, const float *al, const float *ro, const float *me)
        : rec(S.rec), albedo(al), rough(ro), metal(me), tcut(t_cut) {}

    __device__ __forceinline__ void reset()
    {
        T = 1.0f;
        Td = 1.0f;
        W = 0.0f; R = 0.0f; M = 0.0f;
        A = make_float3(0.f, 0.f, 0.f);
        N = make_float3(0.f, 0.f, 0.f);
    }

    __device__ __forceinline__ bool operator()(uint32_t p, uint32_t id, float tau, const float4 r0, const float4 r1,
                                               const float4 r2, const float4 r3, float crho2, const float3 o,
                                               const float3 d)
    {
        HitGeo g;
        value_geo(r0, r1, r2, r3, o, d, g);
        const float a = r1.w * expf(-0.5f * g.rho2);
        const float w = T * a;
        const float wn = g.den > 0.0f ? -w : w;  // normal toward the ray origin
        const size_t i = id;
        W += w;
        A.x += w * albedo[3 * i]; A.y += w * albedo[3 * i + 1]; A.z += w * albedo[3 * i + 2];
        R += w * rough[i];
        M += w * metal[i];
        N.x += wn * r1.x; N.y += wn * r1.y; N.z += wn * r1.z;
        T = T * (1.0f - a);
        Td = trans_step(Td, hit_alpha(r1.w, crho2));
        return Td < tcut;
    }
};

// Primary-ray G-buffer (Eq. deferred_maps on traced camera rays): the
// attribute sums plus the depth tau and the colour of each composited hit,
// with the same weights.
struct GBufVisit : AttrVisit {
    const float4 *col;
    float Dsum;
    float3 Csum;

    __device__ GBufVisit() {}
    __device__ GBufVisit(const SceneDev &S, float t_cut, const float *al, const float *ro, const float *me)
        : AttrVisit(S, t_cut, al, ro, me), col(S.col) {}

    __device__ __forceinline__ void reset()
    {
        AttrVisit::reset();
        Dsum = 0.0f;
        Csum = make_float3(0.f, 0.f, 0.f);
    }

    __device__ __forceinline__ bool operator()(uint32_t p, uint32_t id, float tau, const float4 r0, const float4 r1,
                                               const float4 r2, const float4 r3, float crho2, const float3 o,
                                               const float3 d)
    {
        HitGeo g;
        value_geo(r0, r1, r2, r3, o, d, g);
        const float a = r1.w * expf(-0.5f * g.rho2);
        const float w = T * a;
        const float4 c = col[p];
        Dsum += w * tau;
        Csum.x += w * c.x; Csum.y += w * c.y; Csum.z += w * c.z;
        return AttrVisit::operator()(p, id, tau, r0, r1, r2, r3, crho2, o, d);
    }
};

// Gradient terms reach global memory through per-wavefront LDS staging.
// Device FP32 atomics are limited by the cache lines they touch (one line per
// lane-atomic when lanes update unrelated surfels), not by the dwords: 16
// lanes adding to the 16 floats of one line cost what one lane does.  So each
// surfel owns a 16-float line of a scratch buffer (13 terms used), a hit's
// terms are staged in LDS where it is composited (any subset of lanes), and a
// flush has 16 lanes add one staged hit to its line in one instruction, four
// hits per instruction.  Flushes run at wavefront-uniform points; a step
// stages at most one hit per lane, so flushing whenever the list could not
// take another full step keeps it from overflowing.
constexpr int kStageStride = 16;  // 13 terms, then the surfel id (16-byte aligned entries)
template <int Cap>
struct WaveStageN {
    static constexpr int kCap = Cap;
    alignas(16) float v[Cap * kStageStride];
    int count;
};
// 80 entries of 64 bytes: with the backward's 16-deep stacks, 52 KB of LDS
// per workgroup, three workgroups per CU
#ifndef GRT_STAGE_CAP
#define GRT_STAGE_CAP 80
#endif
using WaveStage = WaveStageN<GRT_STAGE_CAP>;

// Active lanes: stage one hit each (13 terms of surfel id).
template <class Stage>
__device__ __forceinline__ void stage_add(Stage *s, uint32_t id, const float (&t)[13])
{
    const uint64_t m = __ballot(1);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    volatile int *cnt = &s->count;
    const int base = __builtin_amdgcn_readfirstlane(*cnt);
    // four 16-byte stores per entry; stage_sync's fences order them
    float4 *e = reinterpret_cast<float4 *>(&s->v[(base + rank) * kStageStride]);
    e[0] = make_float4(t[0], t[1], t[2], t[3]);
    e[1] = make_float4(t[4], t[5], t[6], t[7]);
    e[2] = make_float4(t[8], t[9], t[10], t[11]);
    e[3] = make_float4(t[12], __uint_as_float(id), 0.0f, 0.0f);
    if (rank == 0) *cnt = base + __popcll(m);
}

// All 64 lanes of the wavefront: start with an empty list.
template <class Stage>
__device__ __forceinline__ void stage_init(Stage *s)
{
    if ((threadIdx.x & 63) == 0) *(volatile int *)&s->count = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// All 64 lanes of the wavefront, at a wavefront-uniform point: add the staged
// hits to their surfels' lines once the list is past half full (all of it
// when `all`), then empty it.
template <class Stage>
__device__ __forceinline__ void stage_sync(float *acc, Stage *s, bool all)
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int n = __builtin_amdgcn_readfirstlane(*(volatile int *)&s->count);
    if (n == 0 || (!all && n <= Stage::kCap - 64)) return;
    const int lane = threadIdx.x & 63, c = lane & 15;
    const volatile float *v = s->v;
    if (c < 13)
        for (int e = lane >> 4; e < n; e += 4) {
            const uint32_t id = reinterpret_cast<const volatile uint32_t *>(v)[e * kStageStride + 13];
            unsafeAtomicAdd(&acc[16 * (size_t)id + c], v[e * kStageStride + c]);
        }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane == 0) *(volatile int *)&s->count = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Backward of g_C . C + g_T . T_fin through every composited hit, with the
// hit set, order and stop index of the forward.
// Chain rule of one composited hit: from dL/dalpha (dA) -- and, for callers
// that also read the hit's depth tau and normal n, a direct dL/dtau (dtau)
// and dL/dn (dnx) -- to the surfel's stored parameters, out[0..9] = (mu xyz,
// s_u, s_v, q wxyz, opacity).  alpha = o G(u, v) at the tangent-plane
// crossing x = o + tau d, tau = n.(mu - o) / n.d, so tau moves with mu and n.
template <bool kDirect>
__device__ __forceinline__ void hit_param_grads(const HitGeo &hg, const float4 r1, const float4 r2, const float4 r3,
                                                float3 d, float a, float G, float dA, float dtau, float3 dnx,
                                                float4 q, float su, float sv, float out[10])
{
    const float3 n = make_float3(r1.x, r1.y, r1.z);
    const float den = hg.den;
    const float3 D = hg.D;
    const float3 au = make_float3(r2.x, r2.y, r2.z), av = make_float3(r3.x, r3.y, r3.z);
    const float u = hg.u, v = hg.v;
    const float gamma = -0.5f * a * dA;  // dL/d(rho^2)
    const float du = 2.0f * u * gamma, dv = 2.0f * v * gamma;
    // parameters of the surfel in its stored form (q, su, sv from the record order)
    const float ql = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    const float iq = 1.0f / ql;
    const float qw = q.x * iq, qx = q.y * iq, qy = q.z * iq, qz = q.w * iq;
    const float dsu = -(u / su) * du, dsv = -(v / sv) * dv;
    const float3 gD = make_float3(du * au.x + dv * av.x, du * au.y + dv * av.y, du * au.z + dv * av.z);
    const float gDd = kDirect ? (dot3(gD, d) + dtau) / den : dot3(gD, d) / den;
    const float3 dmu = make_float3(gDd * n.x - gD.x, gDd * n.y - gD.y, gDd * n.z - gD.z);
    const float ku = du / su, kv = dv / sv;
    const float3 dtu = make_float3(ku * D.x, ku * D.y, ku * D.z);
    const float3 dtv = make_float3(kv * D.x, kv * D.y, kv * D.z);
    float3 dn = make_float3(-gDd * D.x, -gDd * D.y, -gDd * D.z);
    if (kDirect) { dn.x += dnx.x; dn.y += dnx.y; dn.z += dnx.z; }
    // d(columns of R)/d(unit quaternion)
    float dqw = 2.f * (dtu.y * qz - dtu.z * qy - dtv.x * qz + dtv.z * qx + dn.x * qy - dn.y * qx);
    float dqx = 2.f * (dtu.y * qy + dtu.z * qz + dtv.x * qy - 2.f * dtv.y * qx + dtv.z * qw + dn.x * qz - dn.y * qw -
                       2.f * dn.z * qx);
    float dqy = 2.f * (-2.f * dtu.x * qy + dtu.y * qx - dtu.z * qw + dtv.x * qx + dtv.z * qz + dn.x * qw +
                       dn.y * qz - 2.f * dn.z * qy);
    float dqz = 2.f * (-2.f * dtu.x * qz + dtu.y * qw + dtu.z * qx - dtv.x * qw - 2.f * dtv.y * qz + dtv.z * qy +
                       dn.x * qx + dn.y * qy);
    const float proj = qw * dqw + qx * dqx + qy * dqy + qz * dqz;
    dqw = (dqw - qw * proj) * iq; dqx = (dqx - qx * proj) * iq;
    dqy = (dqy - qy * proj) * iq; dqz = (dqz - qz * proj) * iq;
    out[0] = dmu.x; out[1] = dmu.y; out[2] = dmu.z;
    out[3] = dsu; out[4] = dsv;
    out[5] = dqw; out[6] = dqx; out[7] = dqy; out[8] = dqz;
    out[9] = G * dA;
}

// kOrigin: also sum the hits' mean terms per ray.  Every hit's geometry is a
// function of mu - o, so the loss's gradient with respect to the ray origin
// is minus that sum (kept in `gmu`).
template <bool kOrigin = false>
struct GradVisitT {
    const float4 *rec;
    const float4 *col;
    float tcut;
    GradPtrs g;
    WaveStage *stage = nullptr;  // the wavefront's staging list
    float3 gC;
    float3 R;     // colour still ahead: the saved c_rt minus the hits composited so far
    float gTf;    // dL/dT times the saved transmittance
    float T, Td;
    float3 gmu;

    __device__ GradVisitT() {}
    const float4 *quat;
    __device__ GradVisitT(const SceneDev &S, float t_cut, const GradPtrs &gp)
        : rec(S.rec), col(S.col), tcut(t_cut), g(gp), quat(S.quat) {}

    __device__ __forceinline__ void reset(float3 gC_, float gT_, float3 Cf_, float Tf_)
    {
        gC = gC_;
        R = Cf_;
        gTf = gT_ * Tf_;
        T = 1.0f;
        Td = 1.0f;
        gmu = make_float3(0.f, 0.f, 0.f);
    }

    __device__ __forceinline__ bool operator()(uint32_t p, uint32_t id, float tau, const float4 r0, const float4 r1,
                                               const float4 r2, const float4 r3, float crho2, const float3 o,
                                               const float3 d)
    {
        const float4 c = col[p];
        const float op = r1.w;
        HitGeo hg;
        value_geo(r0, r1, r2, r3, o, d, hg);
        const float G = expf(-0.5f * hg.rho2);
        const float a = op * G;
        const float w = T * a;
        R.x -= w * c.x; R.y -= w * c.y; R.z -= w * c.z;
        float dA = T * (gC.x * c.x + gC.y * c.y + gC.z * c.z);
        const float om = 1.0f - a;
        if (om >= 1e-6f) {
            float behind = gC.x * R.x + gC.y * R.y + gC.z * R.z + gTf;
            dA -= behind / om;
        }
        float terms[13];
        hit_param_grads<false>(hg, r1, r2, r3, d, a, G, dA, 0.0f, make_float3(0.f, 0.f, 0.f), quat[p], r3.w, c.w,
                               terms);
        terms[10] = w * gC.x; terms[11] = w * gC.y; terms[12] = w * gC.z;
        stage_add(stage, id, terms);
        if constexpr (kOrigin) {
            gmu.x += terms[0]; gmu.y += terms[1]; gmu.z += terms[2];
        }

        T = T * (1.0f - a);
        Td = trans_step(Td, hit_alpha(op, crho2));
        return Td < tcut;
    }
};

using GradVisit = GradVisitT<false>;

// Backward of the primary-ray G-buffer (Eq. deferred_maps on traced camera
// rays).  Every map is a ratio S_f / W of blended sums S_f = sum_k w_k f_k,
// W = sum_k w_k, w_k = T_k alpha_k, and the normal map is N / |N| with
// N = sum_k w_k s_k n_k.  Holding the hits' values fixed, dL/dw_k is
//   e_k = sum_f g_f (f_k - F_f) / W + s_k n_k . (I - n n^T) g_n / |N|,
// and sum_k w_k e_k = 0 (every map is invariant to a common scale of the
// weights), so the part of the loss behind hit k is -(e_1 w_1 + ... + e_k w_k).
// The per-ray constants come from the forward's maps, W and |N| / W.
struct GBufGradVisit {
    const float4 *rec;
    const float4 *col;
    const float *albedo, *rough, *metal;  // per surfel id
    float *ga_albedo, *ga_rough, *ga_metal;  // attribute gradients (NULL: skipped)
    float tcut;
    GradPtrs g;
    WaveStage *stage = nullptr;
    float kD, kR, kM, e0;  // upstream gradients over W, and sum_f g_f F_f / W
    float3 kA, kC, kN;
    float T, Td, P;

    __device__ GBufGradVisit() {}
    const float4 *quat;
    __device__ GBufGradVisit(const SceneDev &S, float t_cut, const GradPtrs &gp)
        : rec(S.rec), col(S.col), tcut(t_cut), g(gp), quat(S.quat) {}

    __device__ __forceinline__ void reset()
    {
        T = 1.0f;
        Td = 1.0f;
        P = 0.0f;
    }

    __device__ __forceinline__ bool operator()(uint32_t p, uint32_t id, float tau, const float4 r0, const float4 r1,
                                               const float4 r2, const float4 r3, float crho2, const float3 o,
                                               const float3 d)
    {
        const float4 c = col[p];
        const float op = r1.w;
        HitGeo hg;
        value_geo(r0, r1, r2, r3, o, d, hg);
        const float G = expf(-0.5f * hg.rho2);
        const float a = op * G;
        const float w = T * a;
        const float side = hg.den > 0.0f ? -1.0f : 1.0f;  // normal toward the camera
        const size_t i = id;
        const float3 al = make_float3(albedo[3 * i], albedo[3 * i + 1], albedo[3 * i + 2]);
        const float e = kD * tau + kA.x * al.x + kA.y * al.y + kA.z * al.z + kR * rough[i] + kM * metal[i] +
                        kC.x * c.x + kC.y * c.y + kC.z * c.z - e0 + side * (r1.x * kN.x + r1.y * kN.y + r1.z * kN.z);
        P += w * e;
        float dA = T * e;
        const float om = 1.0f - a;
        if (om >= 1e-6f) dA += P / om;
        const float sw = side * w;
        float terms[13];
        hit_param_grads<true>(hg, r1, r2, r3, d, a, G, dA, w * kD, make_float3(sw * kN.x, sw * kN.y, sw * kN.z),
                              quat[p], r3.w, c.w, terms);
        terms[10] = w * kC.x; terms[11] = w * kC.y; terms[12] = w * kC.z;
        stage_add(stage, id, terms);
        if (ga_albedo) {
            atomicAdd(ga_albedo + 3 * i, w * kA.x);
            atomicAdd(ga_albedo + 3 * i + 1, w * kA.y);
            atomicAdd(ga_albedo + 3 * i + 2, w * kA.z);
        }
        if (ga_rough) atomicAdd(ga_rough + i, w * kR);
        if (ga_metal) atomicAdd(ga_metal + i, w * kM);

        T = T * (1.0f - a);
        Td = trans_step(Td, hit_alpha(op, crho2));
        return Td < tcut;
    }
};

// Hand hit p of the visit's ray to `visit` (record loaded, canonical rho^2
// computed here): for callers that hold only the record position.
template <class Visit>
__device__ __forceinline__ bool visit_hit(Visit &visit, const float4 *rec, uint32_t p, float3 o, float3 d)
{
    const float4 *r = rec + 4 * (size_t)p;
    const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
    float den, tau, rho2;
    canon_geo(r0, r1, r2, r3, o, d, den, tau, rho2);
    return visit(p, __float_as_uint(r2.w), tau, r0, r1, r2, r3, rho2, o, d);
}

}  // namespace grt
