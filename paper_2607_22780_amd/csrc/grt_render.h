// grt_render.h -- per-sample device code shared by the MIS render and the
// relighting server: random numbers, proposals and pdfs, the BRDF, and the
// generation of one sample's ray record.
#pragma once

#include "grt_internal.h"
#include "grt_kernels.h"

namespace grt {

// ---------------------------------------------------------------------------
// Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void uniforms(uint64_t seed, uint32_t pix, uint32_t j, uint32_t job, float &u1, float &u2)
{
    uint32_t c0 = pix, c1 = j, c2 = job, c3 = 0u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    u1 = (float)(c0 >> 8) * (1.0f / 16777216.0f);
    u2 = (float)(c1 >> 8) * (1.0f / 16777216.0f);
}

// ---------------------------------------------------------------------------
// Proposals, pdfs and the BRDF, per sample in double precision with a fixed
// operation order (a few hundred flops per sample against thousands of bytes
// of traversal): the sampled direction, rounded once to single precision, is
// then reproducible to the last bit, and so is every hit decision downstream.
// ---------------------------------------------------------------------------
constexpr double kPiD = 3.14159265358979323846;

struct V3 {
    double x, y, z;
};

__device__ __forceinline__ V3 v3(double x, double y, double z) { return V3{x, y, z}; }
__device__ __forceinline__ double dot(V3 a, V3 b)
{
#pragma clang fp contract(off)
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ V3 normalized(V3 a)
{
#pragma clang fp contract(off)
    double l = sqrt(dot(a, a));
    return v3(a.x / l, a.y / l, a.z / l);
}
// x b1 + y b2 + z n, summed left to right
__device__ __forceinline__ V3 combine(double x, V3 b1, double y, V3 b2, double z, V3 n)
{
#pragma clang fp contract(off)
    return v3(x * b1.x + y * b2.x + z * n.x, x * b1.y + y * b2.y + z * n.y, x * b1.z + y * b2.z + z * n.z);
}

// orthonormal basis around n (Duff et al., JCGT 2017)
__device__ __forceinline__ void onb(V3 n, V3 &b1, V3 &b2)
{
#pragma clang fp contract(off)
    double sign = copysign(1.0, n.z);
    double a = -1.0 / (sign + n.z);
    double b = n.x * n.y * a;
    b1 = v3(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
    b2 = v3(b, sign + n.y * n.y * a, -n.y);
}

__device__ __forceinline__ double ggx_D(double ndh, double a2)
{
#pragma clang fp contract(off)
    double t = ndh * ndh * (a2 - 1.0) + 1.0;
    return a2 / (kPiD * t * t);
}

__device__ __forceinline__ double smith_G1(double ndv, double a2)
{
#pragma clang fp contract(off)
    return 2.0 * ndv / (ndv + sqrt(a2 + (1.0 - a2) * ndv * ndv));
}

// cosine-weighted direction (Malley: uniform disk lifted to the hemisphere)
__device__ __forceinline__ V3 sample_cos(V3 n, double u1, double u2)
{
#pragma clang fp contract(off)
    V3 b1, b2;
    onb(n, b1, b2);
    double r = sqrt(u1), ph = 2.0 * kPiD * u2;
    double x = r * cos(ph), y = r * sin(ph), z = sqrt(1.0 - u1 > 0.0 ? 1.0 - u1 : 0.0);
    return combine(x, b1, y, b2, z, n);
}

// visible-normal sampling of GGX (Heitz, JCGT 2018), then reflect wo about h
__device__ __forceinline__ V3 sample_ggx(V3 n, V3 wo, double rough, double u1, double u2)
{
#pragma clang fp contract(off)
    V3 b1, b2;
    onb(n, b1, b2);
    double a = rough * rough;
    V3 Vh = normalized(v3(a * dot(wo, b1), a * dot(wo, b2), dot(wo, n)));
    double lensq = Vh.x * Vh.x + Vh.y * Vh.y;
    V3 T1 = v3(1.0, 0.0, 0.0);
    if (lensq > 0.0) {
        double il = 1.0 / sqrt(lensq);
        T1 = v3(-Vh.y * il, Vh.x * il, 0.0);
    }
    V3 T2 = v3(Vh.y * T1.z - Vh.z * T1.y, Vh.z * T1.x - Vh.x * T1.z, Vh.x * T1.y - Vh.y * T1.x);
    double r = sqrt(u1), ph = 2.0 * kPiD * u2;
    double t1 = r * cos(ph), t2 = r * sin(ph);
    double s = 0.5 * (1.0 + Vh.z);
    t2 = (1.0 - s) * sqrt(1.0 - t1 * t1) + s * t2;
    double t3 = 1.0 - t1 * t1 - t2 * t2;
    t3 = sqrt(t3 > 0.0 ? t3 : 0.0);
    V3 Nh = v3(t1 * T1.x + t2 * T2.x + t3 * Vh.x, t1 * T1.y + t2 * T2.y + t3 * Vh.y, t1 * T1.z + t2 * T2.z + t3 * Vh.z);
    V3 Ne = normalized(v3(a * Nh.x, a * Nh.y, Nh.z > 0.0 ? Nh.z : 0.0));
    V3 h = combine(Ne.x, b1, Ne.y, b2, Ne.z, n);
    double oh = dot(wo, h);
    return v3(2.0 * oh * h.x - wo.x, 2.0 * oh * h.y - wo.y, 2.0 * oh * h.z - wo.z);
}

// first k in [0, n) with cdf[k+1] > u (cdf[n] == 1 > u)
__device__ __forceinline__ int cdf_find(const float *__restrict__ cdf, int n, double u)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((double)cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ V3 sample_env(const EnvDev &E, double u1, double u2)
{
#pragma clang fp contract(off)
    int i = cdf_find(E.marg, E.H, u1);
    double dv = (u1 - (double)E.marg[i]) / ((double)E.marg[i + 1] - (double)E.marg[i]);
    const float *cr = E.cond + (size_t)i * (E.W + 1);
    int j = cdf_find(cr, E.W, u2);
    double du = (u2 - (double)cr[j]) / ((double)cr[j + 1] - (double)cr[j]);
    double th = kPiD * (i + dv) / E.H, ph = 2.0 * kPiD * (j + du) / E.W;
    return v3(sin(th) * cos(ph), cos(th), sin(th) * sin(ph));
}

// nearest texel of a direction; sin(theta) for the pdf
__device__ __forceinline__ void env_index(const EnvDev &E, V3 w, int &i, int &j, double &sin_t)
{
#pragma clang fp contract(off)
    double y = w.y < -1.0 ? -1.0 : (w.y > 1.0 ? 1.0 : w.y);
    double th = acos(y);
    double ph = atan2(w.z, w.x);
    if (ph < 0.0) ph += 2.0 * kPiD;
    int ii = (int)(th / kPiD * E.H), jj = (int)(ph / (2.0 * kPiD) * E.W);
    i = ii < E.H - 1 ? ii : E.H - 1;
    j = jj < E.W - 1 ? jj : E.W - 1;
    if (i < 0) i = 0;
    if (j < 0) j = 0;
    sin_t = sqrt(1.0 - y * y > 0.0 ? 1.0 - y * y : 0.0);
}

__device__ __forceinline__ float3 env_radiance(const EnvDev &E, V3 w)
{
    int i, j;
    double st;
    env_index(E, w, i, j, st);
    const float *p = E.rgb + ((size_t)i * E.W + j) * 3;
    return make_float3(p[0], p[1], p[2]);
}

__device__ __forceinline__ double env_pdf(const EnvDev &E, V3 w)
{
#pragma clang fp contract(off)
    int i, j;
    double st;
    env_index(E, w, i, j, st);
    if (st <= 0.0) return 0.0;
    const float *cr = E.cond + (size_t)i * (E.W + 1);
    double pij = ((double)E.marg[i + 1] - (double)E.marg[i]) * ((double)cr[j + 1] - (double)cr[j]);
    return pij * E.H * E.W / (2.0 * kPiD * kPiD * st);
}

// q = (N_c p_c + N_g p_g + N_e p_e) / N_r (Sec. 3.4.1, deterministic mixture)
__device__ __forceinline__ double mixture_pdf(const EnvDev &E, V3 n, V3 wo, double rough, V3 w, int nc, int ng,
                                              int ne)
{
#pragma clang fp contract(off)
    double ndi = dot(n, w), ndo = dot(n, wo);
    double pc = ndi > 0.0 ? ndi / kPiD : 0.0;
    double pg = 0.0;
    V3 h = v3(w.x + wo.x, w.y + wo.y, w.z + wo.z);
    double hl = sqrt(dot(h, h));
    if (hl > 0.0) {
        h = v3(h.x / hl, h.y / hl, h.z / hl);
        double ndh = dot(n, h);
        if (ndh > 0.0 && dot(wo, h) > 0.0) {
            double a = rough * rough, a2 = a * a;
            pg = smith_G1(ndo, a2) * ggx_D(ndh, a2) / (4.0 * ndo);
        }
    }
    double pe = ne > 0 ? env_pdf(E, w) : 0.0;
    return ((double)nc * pc + (double)ng * pg + (double)ne * pe) / (double)(nc + ng + ne);
}

// f(wo, wi) for wi.n > 0, wo.n > 0 (Eqs. brdf_decompose, brdf_specular;
// F0 = 0.04 (1 - m) + m a; D GGX, G separable Smith, F Schlick on wi.h)
__device__ __forceinline__ V3 brdf(V3 n, V3 wo, V3 wi, V3 alb, double rough, double metal)
{
#pragma clang fp contract(off)
    double ndi = dot(n, wi), ndo = dot(n, wo);
    V3 h = normalized(v3(wi.x + wo.x, wi.y + wo.y, wi.z + wo.z));
    double ndh = dot(n, h), idh = dot(wi, h);
    double a = rough * rough, a2 = a * a;
    double D = ggx_D(ndh, a2);
    double G = smith_G1(ndi, a2) * smith_G1(ndo, a2);
    double x = 1.0 - idh;
    if (x < 0.0) x = 0.0;
    double x5 = x * x * x * x * x;
    double al[3] = {alb.x, alb.y, alb.z}, f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double F0 = 0.04 * (1.0 - metal) + metal * al[c];
        double F = F0 + (1.0 - F0) * x5;
        f[c] = (1.0 - metal) * al[c] / kPiD + D * F * G / (4.0 * ndi * ndo);
    }
    return v3(f[0], f[1], f[2]);
}

// Backward of the BRDF times the cosine, sum_c u_c f_c(wo, wi) (n.wi), with
// wi held fixed: accumulates the derivatives with respect to the unit normal
// n, the unit view direction wo, albedo, roughness and metallic.  The
// specular part of f_c is K F_c, K = D G1(n.wi) G1(n.wo) / (4 (n.wi)(n.wo)),
// and everything that moves K enters through its logarithm:
//   d ln K / d(n.wi) = -(1 + s'(n.wi)) / (n.wi + s(n.wi))  (G1's 1/v and the
//     denominator's cancel; s(v) = sqrt(a2 + (1 - a2) v^2), s' = ds/dv),
//   the same in n.wo,  d ln K / d(n.h) = -4 (n.h)(a2 - 1) / t,
//   t = (n.h)^2 (a2 - 1) + 1,  with h = (wi + wo) / |wi + wo|;
// the roughness (a2 = r^4) enters D directly and G1 through s:
//   dD/da2 = (1 - 2 a2 (n.h)^2 / t) / (pi t^2),  d ln G1 / da2 = -(ds/da2) / (v + s).
// F_c = F0_c + (1 - F0_c) x^5, x = max(0, 1 - wi.h), F0_c = 0.04 (1 - m) + m a_c.
struct ShadeGrad {
    V3 n, wo, alb;
    double rough, metal;
};

__device__ __forceinline__ void brdf_cos_backward(V3 n, V3 wo, V3 wi, V3 alb, double rough, double metal,
                                                  const double u[3], ShadeGrad &g)
{
#pragma clang fp contract(off)
    const double ndi = dot(n, wi), ndo = dot(n, wo);
    const V3 hs = v3(wi.x + wo.x, wi.y + wo.y, wi.z + wo.z);
    const double hl = sqrt(dot(hs, hs));
    const V3 h = v3(hs.x / hl, hs.y / hl, hs.z / hl);
    const double ndh = dot(n, h), idh = dot(wi, h);
    const double r2 = rough * rough, a2 = r2 * r2;
    const double t = ndh * ndh * (a2 - 1.0) + 1.0;
    const double D = a2 / (kPiD * t * t);
    const double si = sqrt(a2 + (1.0 - a2) * ndi * ndi), so = sqrt(a2 + (1.0 - a2) * ndo * ndo);
    const double G1i = 2.0 * ndi / (ndi + si), G1o = 2.0 * ndo / (ndo + so);
    const double den = 4.0 * ndi * ndo;
    const double K = D * G1i * G1o / den;
    double x = 1.0 - idh;
    if (x < 0.0) x = 0.0;
    const double x4 = x * x * x * x, x5 = x4 * x;
    const double al[3] = {alb.x, alb.y, alb.z};
    // channel sums: sum u f, sum u F, sum u dF/d(wi.h), and the albedo/metal terms
    double uf = 0.0, uF = 0.0, udF = 0.0, um = 0.0, ga[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double F0 = 0.04 * (1.0 - metal) + metal * al[c];
        const double F = F0 + (1.0 - F0) * x5;
        uf += u[c] * ((1.0 - metal) * al[c] / kPiD + K * F);
        uF += u[c] * F;
        udF += u[c] * (x > 0.0 ? -5.0 * (1.0 - F0) * x4 : 0.0);
        ga[c] = u[c] * ndi * ((1.0 - metal) / kPiD + K * metal * (1.0 - x5));
        um += u[c] * (-al[c] / kPiD + K * (al[c] - 0.04) * (1.0 - x5));
    }
    const double KuF = K * uF;
    const double Li = -(1.0 + (1.0 - a2) * ndi / si) / (ndi + si);
    const double Lo = -(1.0 + (1.0 - a2) * ndo / so) / (ndo + so);
    const double Lh = -4.0 * ndh * (a2 - 1.0) / t;
    // d/dn of (n.wi), (n.wo), (n.h); d/dwo of (n.wo), (n.h), (wi.h)
    const double cn_i = ndi * KuF * Li + uf, cn_o = ndi * KuF * Lo, cn_h = ndi * KuF * Lh;
    g.n = v3(g.n.x + cn_i * wi.x + cn_o * wo.x + cn_h * h.x, g.n.y + cn_i * wi.y + cn_o * wo.y + cn_h * h.y,
             g.n.z + cn_i * wi.z + cn_o * wo.z + cn_h * h.z);
    const double cw_h = cn_h / hl, cw_i = ndi * K * udF / hl;
    g.wo = v3(g.wo.x + cn_o * n.x + cw_h * (n.x - h.x * ndh) + cw_i * (wi.x - h.x * idh),
              g.wo.y + cn_o * n.y + cw_h * (n.y - h.y * ndh) + cw_i * (wi.y - h.y * idh),
              g.wo.z + cn_o * n.z + cw_h * (n.z - h.z * ndh) + cw_i * (wi.z - h.z * idh));
    g.alb = v3(g.alb.x + ga[0], g.alb.y + ga[1], g.alb.z + ga[2]);
    g.metal += ndi * um;
    const double dD = (1.0 - 2.0 * a2 * ndh * ndh / t) / (kPiD * t * t);
    const double dlnG = -(1.0 - ndi * ndi) / (2.0 * si * (ndi + si)) - (1.0 - ndo * ndo) / (2.0 * so * (ndo + so));
    const double dK = dD * G1i * G1o / den + K * dlnG;
    g.rough += ndi * uF * dK * 4.0 * r2 * rough;
}

// ---------------------------------------------------------------------------
// Split-sum relighting (Eq. relight_splitsum), in double: lookups of the
// prefiltered tables and SplitSum(a, r, m, n, E) of a surface seen along -w.
// ---------------------------------------------------------------------------
// bilinear over texel centres; wraps in the azimuth, clamps in the polar angle
__device__ __forceinline__ V3 table_lookup(const float *__restrict__ T, V3 w)
{
#pragma clang fp contract(off)
    double y = w.y < -1.0 ? -1.0 : (w.y > 1.0 ? 1.0 : w.y);
    double th = acos(y), ph = atan2(w.z, w.x);
    if (ph < 0.0) ph += 2.0 * kPiD;
    // clamps written so that a NaN lands on the lower bound (indices stay in range)
    double x = ph / (2.0 * kPiD) * kPfW - 0.5, v = th / kPiD * kPfH - 0.5;
    x = x > -1.0 ? (x < (double)kPfW ? x : (double)kPfW) : -1.0;
    double fx0 = floor(x);
    double fx = x - fx0;
    int j0 = (int)fx0;
    j0 = ((j0 % kPfW) + kPfW) % kPfW;
    int j1 = (j0 + 1) % kPfW;
    v = v > 0.0 ? (v < (double)(kPfH - 1) ? v : (double)(kPfH - 1)) : 0.0;
    int i0 = (int)floor(v);
    if (i0 > kPfH - 2) i0 = kPfH - 2;
    double fy = v - i0;
    double o[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double a = T[(i0 * kPfW + j0) * 3 + k], b = T[(i0 * kPfW + j1) * 3 + k];
        double c = T[((i0 + 1) * kPfW + j0) * 3 + k], d = T[((i0 + 1) * kPfW + j1) * 3 + k];
        o[k] = (1.0 - fy) * ((1.0 - fx) * a + fx * b) + fy * ((1.0 - fx) * c + fx * d);
    }
    return v3(o[0], o[1], o[2]);
}

// diffuse (1 - m) a E_d(n) plus specular E_s(R, r) (F0 A + B), F0 = 0.04 (1 - m)
// + m a; n the query's averaged normal (renormalized; -w if it vanished), v = -w
__device__ __forceinline__ V3 split_sum(const EnvDev &E, V3 alb, double rough, double metal, V3 nsum, V3 w)
{
#pragma clang fp contract(off)
    V3 v = v3(-w.x, -w.y, -w.z);
    double nl = sqrt(dot(nsum, nsum));
    V3 n = nl > 0.0 ? v3(nsum.x / nl, nsum.y / nl, nsum.z / nl) : v;
    double ndv = dot(n, v);
    V3 R = v3(2.0 * ndv * n.x - v.x, 2.0 * ndv * n.y - v.y, 2.0 * ndv * n.z - v.z);
    double mu = ndv > 0.0 ? (ndv < 1.0 ? ndv : 1.0) : 0.0;
    double r = rough > 0.0 ? (rough < 1.0 ? rough : 1.0) : 0.0;
    V3 Ld = table_lookup(E.Ed, n);
    double xl = r * (kPfL - 1);
    int l0 = (int)floor(xl);
    if (l0 > kPfL - 2) l0 = kPfL - 2;
    double tl = xl - l0;
    V3 L0;
    if (l0 == 0) {
        float3 e = env_radiance(E, R);
        L0 = v3(e.x, e.y, e.z);
    } else {
        L0 = table_lookup(E.Es + (size_t)(l0 - 1) * kPfH * kPfW * 3, R);
    }
    V3 L1 = table_lookup(E.Es + (size_t)l0 * kPfH * kPfW * 3, R);
    V3 Ls = v3((1.0 - tl) * L0.x + tl * L1.x, (1.0 - tl) * L0.y + tl * L1.y, (1.0 - tl) * L0.z + tl * L1.z);
    double xi = mu * kLutN - 0.5, yj = r * kLutN - 0.5;
    if (xi < 0.0) xi = 0.0;
    if (xi > kLutN - 1) xi = kLutN - 1;
    if (yj < 0.0) yj = 0.0;
    if (yj > kLutN - 1) yj = kLutN - 1;
    int i0 = (int)floor(xi), j0 = (int)floor(yj);
    if (i0 > kLutN - 2) i0 = kLutN - 2;
    if (j0 > kLutN - 2) j0 = kLutN - 2;
    double fi = xi - i0, fj = yj - j0, AB[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double a = E.lut[2 * (i0 * kLutN + j0) + k], b = E.lut[2 * (i0 * kLutN + j0 + 1) + k];
        double c = E.lut[2 * ((i0 + 1) * kLutN + j0) + k], d = E.lut[2 * ((i0 + 1) * kLutN + j0 + 1) + k];
        AB[k] = (1.0 - fi) * ((1.0 - fj) * a + fj * b) + fi * ((1.0 - fj) * c + fj * d);
    }
    double al[3] = {alb.x, alb.y, alb.z}, Lds[3] = {Ld.x, Ld.y, Ld.z}, Lss[3] = {Ls.x, Ls.y, Ls.z}, o[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double F0 = 0.04 * (1.0 - metal) + metal * al[k];
        o[k] = (1.0 - metal) * al[k] * Lds[k] + Lss[k] * (F0 * AB[0] + AB[1]);
    }
    return v3(o[0], o[1], o[2]);
}

struct Shade {
    V3 n, wo, alb;
    float3 x;
    double rough, metal;
};

// the normal and the view direction are directions: normalised in double
__device__ __forceinline__ bool load_pixel(const RenderArgs &a, int64_t p, Shade &s)
{
    if (p >= (int64_t)a.H * a.W || !a.valid[p]) return false;
    s.x = make_float3(a.x[3 * p], a.x[3 * p + 1], a.x[3 * p + 2]);
    V3 n = v3(a.n[3 * p], a.n[3 * p + 1], a.n[3 * p + 2]);
    V3 wo = v3(a.wo[3 * p], a.wo[3 * p + 1], a.wo[3 * p + 2]);
    s.n = dot(n, n) > 0.0 ? normalized(n) : n;
    s.wo = dot(wo, wo) > 0.0 ? normalized(wo) : wo;
    s.alb = v3(a.alb[3 * p], a.alb[3 * p + 1], a.alb[3 * p + 2]);
    s.rough = a.rough[p];
    s.metal = a.metal[p];
    return dot(s.n, s.wo) > 0.0;
}

// Sample j of pixel p: direction w (double, and its single-precision ray
// direction wf), mixture pdf q and weight f cos / q; false below the horizon.
__device__ __forceinline__ bool draw(const RenderArgs &a, const Shade &s, int64_t p, int j, V3 &w, float3 &wf,
                                     double &q, float3 &wt)
{
    uint32_t c0 = (uint32_t)p, c1 = (uint32_t)j;
    float u1f, u2f;
    uniforms(a.seed, c0, c1, a.job, u1f, u2f);
    const double u1 = u1f, u2 = u2f;  // exact: 24-bit integers times 2^-24
    if (j < a.nc) w = sample_cos(s.n, u1, u2);
    else if (j < a.nc + a.ng) w = sample_ggx(s.n, s.wo, s.rough, u1, u2);
    else w = sample_env(a.E, u1, u2);
    wf = make_float3((float)w.x, (float)w.y, (float)w.z);
    double ndi = dot(s.n, w);
    q = 0.0;
    wt = make_float3(0.f, 0.f, 0.f);
    if (!(ndi > 0.0)) return false;
    q = mixture_pdf(a.E, s.n, s.wo, s.rough, w, a.nc, a.ng, a.ne);
    if (q > 0.0) {
        V3 f = brdf(s.n, s.wo, w, s.alb, s.rough, s.metal);
        wt = make_float3((float)(f.x * ndi / q), (float)(f.y * ndi / q), (float)(f.z * ndi / q));
    }
    return true;
}

// ---------------------------------------------------------------------------
// Sample generation of ray r = pixel * spp + j.  Writes the ray record the
// trace kernels read (48 B): (direction, traced flag), (f cos / q, L_env.x),
// (L_env.y, L_env.z, -, -).  Samples below the horizon and invalid pixels are
// flagged 0 and never traced.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gen_ray(const RenderArgs &a, int64_t r)
{
    const int spp = a.nc + a.ng + a.ne;
    const int64_t p = r / spp;
    const int j = (int)(r - p * spp);
    Shade s;
    float3 wf = make_float3(0.f, 0.f, 0.f), wt = wf, Le = wf;
    double q = 0.0;
    bool traced = false;
    if (load_pixel(a, p, s)) {
        V3 dir;
        traced = draw(a, s, p, j, dir, wf, q, wt);
        if (traced) Le = env_radiance(a.E, dir);
    }
    float4 *rr = a.rays + 3 * r;
    rr[0] = make_float4(wf.x, wf.y, wf.z, traced ? 1.0f : 0.0f);
    rr[1] = make_float4(wt.x, wt.y, wt.z, Le.x);
    rr[2] = make_float4(Le.y, Le.z, 0.0f, 0.0f);
    if (a.dump) {
        float *dp = a.dump + r * 10;
        dp[0] = wf.x; dp[1] = wf.y; dp[2] = wf.z; dp[3] = (float)q;
        dp[4] = wt.x; dp[5] = wt.y; dp[6] = wt.z;
        dp[7] = 0.0f; dp[8] = 0.0f; dp[9] = 0.0f;
    }
}

// The persistent-loop job of the forward render: begin loads the ray record
// (skipping untraced samples), finish writes f L_i cos / q and the saved
// (C, T).  kHitList: the launch stores hit lists (a.hits); only then does the
// visitor carry one.  kPerRayArgs: lanes may trace for different requests
// (the server's mixed epochs), so the visitor's tables are set with each
// ray; otherwise the job sets them once (bind) and they stay
// wavefront-uniform (at K = 12 that removed the kernel's 2 spilled registers
// and 3% of its time).
template <int K, bool kHitList = false, bool kPerRayArgs = false>
struct ShadeTrace {
    Walker<K> w;
    CompositeVisit<kHitList> v;

    __device__ __forceinline__ void bind(const RenderArgs &a, const SceneDev &S)
    {
        v.rec = S.rec;
        v.col = S.col;
        v.tcut = a.tcut;
    }

    __device__ __forceinline__ bool begin(const RenderArgs &a, const SceneDev &S, int64_t r)
    {
        const float4 r0 = a.rays[3 * r];
        if (r0.w == 0.0f) {
            a.contrib[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (a.hits) a.hits[r] = 0u;
            return false;
        }
        const int spp = a.nc + a.ng + a.ne;
        const int64_t p = r / spp;
        if (kHitList && a.hits) {
            const int64_t nray = (int64_t)a.H * a.W * spp;
            v.hl = a.hits + nray + r * a.hcap;
            v.hcap = a.hcap;
        }
        const float3 x = make_float3(a.x[3 * p], a.x[3 * p + 1], a.x[3 * p + 2]);
        const float3 d = make_float3(r0.x, r0.y, r0.z);
        if constexpr (kPerRayArgs) bind(a, S);
        v.reset();
        w.start(S, x, d, a.tmin, INFINITY);
        if (S.n <= 0) {
            finish(a, r);
            return false;
        }
        return true;
    }

    __device__ __forceinline__ void finish(const RenderArgs &a, int64_t r)
    {
        const float4 r1 = a.rays[3 * r + 1], r2 = a.rays[3 * r + 2];
        const float3 Li = make_float3(v.C.x + v.T * r1.w, v.C.y + v.T * r2.x, v.C.z + v.T * r2.y);
        a.contrib[r] = make_float4(r1.x * Li.x, r1.y * Li.y, r1.z * Li.z, 0.0f);
        if (a.saved) {
            a.saved[r] = make_float4(v.C.x, v.C.y, v.C.z, v.T);
            a.saved_t[r] = w.stop_depth();
        }
        if (a.hits) a.hits[r] = (uint32_t)v.cnt;
        if (a.dump) {
            float *dp = a.dump + r * 10;
            dp[7] = Li.x; dp[8] = Li.y; dp[9] = Li.z;
        }
    }
};

// The persistent-loop job of the relighting trace (Sec. 3.5.1, Eq.
// trace_attr): begin loads the ray record (skipping untraced samples), and
// finish parks the attribute query's result for the shading pass: (V,
// albedo) in the sample's contribution slot, (roughness, metallic) in the
// spare words of its ray record, the averaged normal in rl_n*.  `a` may
// differ per lane (the server mixes requests).
//
// kPerRayArgs: lanes may trace for different requests (the server's mixed
// epochs), so the query's tables are set with each ray.  Otherwise the job
// sets them once (bind) and they stay wavefront-uniform: held per lane, the
// five values pushed the K = 12 kernel to 23 spilled registers.
template <int K, bool kPerRayArgs = false>
struct RelightTrace {
    Walker<K> w;
    AttrVisit v;

    __device__ __forceinline__ void bind(const RenderArgs &a, const SceneDev &S)
    {
        v.rec = S.rec;
        v.albedo = a.sa_albedo;
        v.rough = a.sa_rough;
        v.metal = a.sa_metal;
        v.tcut = a.tcut;
    }

    __device__ __forceinline__ bool begin(const RenderArgs &a, const SceneDev &S, int64_t r)
    {
        const float4 r0 = a.rays[3 * r];
        if (r0.w == 0.0f) {
            a.contrib[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            return false;
        }
        const int64_t p = r / (a.nc + a.ng + a.ne);
        const float3 x = make_float3(a.x[3 * p], a.x[3 * p + 1], a.x[3 * p + 2]);
        const float3 d = make_float3(r0.x, r0.y, r0.z);
        if constexpr (kPerRayArgs) bind(a, S);
        v.reset();
        w.start(S, x, d, a.tmin, INFINITY);
        if (S.n <= 0) {
            finish(a, r);
            return false;
        }
        return true;
    }

    __device__ __forceinline__ void finish(const RenderArgs &a, int64_t r)
    {
        const float inv = v.W > 0.0f ? 1.0f / v.W : 0.0f;
        a.contrib[r] = make_float4(v.T, v.A.x * inv, v.A.y * inv, v.A.z * inv);
        float4 *r2 = a.rays + 3 * r + 2;
        r2->z = v.R * inv;
        r2->w = v.M * inv;
        a.rl_nx[r] = v.N.x * inv;
        a.rl_ny[r] = v.N.y * inv;
        a.rl_nz[r] = v.N.z * inv;
    }
};

// Once per job, for jobs whose lanes all trace for one request: the trace's
// tables (a per-ray trace takes them in begin).
template <int K, bool kHitList>
__device__ __forceinline__ void bind_trace(ShadeTrace<K, kHitList, false> &t, const RenderArgs &a, const SceneDev &S)
{
    t.bind(a, S);
}
template <int K>
__device__ __forceinline__ void bind_trace(RelightTrace<K, false> &t, const RenderArgs &a, const SceneDev &S)
{
    t.bind(a, S);
}

// c_pbr = (1/N_r) sum_j contrib[p, j], summed in sample order
__device__ __forceinline__ void reduce_pixel(int64_t p, int spp, const float4 *__restrict__ contrib,
                                             float *__restrict__ out)
{
    const float4 *c = contrib + p * spp;
    float x = 0.f, y = 0.f, z = 0.f;
    for (int j = 0; j < spp; ++j) {
        const float4 v = c[j];
        x += v.x; y += v.y; z += v.z;
    }
    const float inv = 1.0f / (float)spp;
    out[3 * p] = x * inv;
    out[3 * p + 1] = y * inv;
    out[3 * p + 2] = z * inv;
}

}  // namespace grt
