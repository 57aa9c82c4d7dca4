/*
 * oracle.c -- plain, slow CPU reference for differentiable 2D Gaussian ray
 * tracing (2DGRT) of secondary rays with multiple-importance-sampled shading,
 * after "Inter-Reflective Gaussian Splatting for Robust and Efficient Inverse
 * Rendering" (IRGS++).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * What it computes, by brute force (every ray against every surfel, no
 * acceleration structure):
 *   - ray/surfel intersection and 2D Gaussian weight   (Sec. 3.2, Eq. raytracing_intersection and the influence G(p))
 *   - exact front-to-back order and compositing         (Sec. 3.2, Eq. trace; Eq. alpha_blending)
 *   - incident radiance L_i = c_rt + (1 - o_rt) L_env   (Sec. 3.3, Eqs. lighting_decompose, incident_trace)
 *   - the metallic microfacet BRDF                      (Sec. 3.1, Eqs. brdf_decompose, brdf_specular)
 *   - the MIS estimator with cosine/GGX/env proposals   (Sec. 3.4.1, Eqs. montecarlo, mis)
 *   - gradients of a loss through all of the above      (Sec. 3.2 "gradients can backpropagate through the secondary-ray queries")
 *
 * Precision.  Values (weights, radiance, pdfs, gradients) are computed in
 * double.  Decisions that turn floating point into integers -- whether a
 * surfel is hit, the depth order, and where compositing stops -- are taken
 * in single precision with a fixed operation order (this file is compiled
 * with -ffp-contract=off), because that is the precision the GPU kernels
 * decide in.  The fixed order is:
 *   frame:  l = sqrtf(((w*w + x*x) + y*y) + z*z); q <- q / l (four divisions)
 *           t_u = (1-2(yy+zz), 2(xy+wz), 2(xz-wy)), t_v = (2(xy-wz), 1-2(xx+zz), 2(yz+wx)),
 *           n = (2(xz+wy), 2(yz-wx), 1-2(xx+yy)),  a_u = t_u / s_u,  a_v = t_v / s_v
 *   bound:  r2max = (float) min(9, 2 ln(o / alpha_min))   evaluated in double
 *   test:   m = mu - o;  den = (n.x d.x + n.y d.y) + n.z d.z;  skip if |den| < 1e-6
 *           tau = ((n.x m.x + n.y m.y) + n.z m.z) / den;  keep if t_min < tau <= t_max
 *           D = tau d - m;  u = a_u.D;  v = a_v.D;  hit iff u*u + v*v <= r2max
 *   order:  ascending (bits(tau), id)  -- tau > 0, so the bit pattern is monotone
 *   stop:   T32 <- T32 * (1 - o*expf(-0.5*r2)); stop after the hit that makes T32 < T_cut
 *
 * Readings of the paper taken here (where it is silent):
 *   - support: 3 sigma (rho^2 <= 9) and the minimum influence alpha >= alpha_min,
 *     i.e. rho^2 <= 2 ln(o/alpha_min), the radius the paper's adaptive bounding
 *     proxy uses (Eq. icosahedron_transform);
 *   - rotations are (w,x,y,z) quaternions normalised inside; t_u, t_v, n are the
 *     columns of the rotation matrix; gradients are taken w.r.t. the stored
 *     (unnormalised) quaternion, the linear scales and the activated opacity;
 *   - compositing includes the hit that makes T < T_cut, then stops;
 *   - the GGX proposal samples visible normals (Heitz 2018) with alpha = r^2;
 *     D is GGX, G the separable Smith form, F Schlick on (omega_i . h);
 *   - proposals are normalised over the sphere; samples below the horizon
 *     count in N_k and contribute zero;
 *   - the environment proposal is piecewise constant over texels weighted by
 *     luminance times sin(theta) at the texel centre; radiance is looked up at
 *     the nearest texel; +y is up, row 0 is the zenith, phi = atan2(z, x);
 *   - random numbers: Philox-4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (pixel, sample, job, 0); u = (word >> 8) * 2^-24.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Surfels                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    /* single precision: the hit decision and the depth key */
    float mu[3], n[3], au[3], av[3], r2max, op;
} Surf32;

typedef struct {
    /* double precision: everything that is a value */
    double mu[3], tu[3], tv[3], n[3], su, sv, op, c[3];
    double qhat[4], qlen;
} Surf64;

typedef struct {
    int64_t n;
    Surf32 *s32;
    Surf64 *s64;
} Scene;

/* Frame of a 2D Gaussian from its quaternion and scales (Sec. 3.2, the
 * primitive's centre, tangents t_u, t_v, scales and opacity; n = t_u x t_v). */
static void prep_one32(const float *mu, const float *sc, const float *q, float op, float alpha_min, Surf32 *o)
{
    float w = q[0], x = q[1], y = q[2], z = q[3];
    float l = sqrtf(w * w + x * x + y * y + z * z);
    w = w / l; x = x / l; y = y / l; z = z / l;
    float xx = x * x, yy = y * y, zz = z * z;
    float xy = x * y, xz = x * z, yz = y * z;
    float wx = w * x, wy = w * y, wz = w * z;
    float tu[3] = {1.0f - 2.0f * (yy + zz), 2.0f * (xy + wz), 2.0f * (xz - wy)};
    float tv[3] = {2.0f * (xy - wz), 1.0f - 2.0f * (xx + zz), 2.0f * (yz + wx)};
    float nn[3] = {2.0f * (xz + wy), 2.0f * (yz - wx), 1.0f - 2.0f * (xx + yy)};
    for (int i = 0; i < 3; ++i) {
        o->mu[i] = mu[i];
        o->n[i] = nn[i];
        o->au[i] = tu[i] / sc[0];
        o->av[i] = tv[i] / sc[1];
    }
    o->op = op;
    if (alpha_min > 0.0f) {
        double b = 2.0 * log((double)op / (double)alpha_min);
        o->r2max = (float)(b < 9.0 ? b : 9.0);
    } else {
        o->r2max = 9.0f;
    }
}

static void prep_one64(const float *mu, const float *sc, const float *q, float op, const float *rgb, Surf64 *o)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double l = sqrt(w * w + x * x + y * y + z * z);
    o->qlen = l;
    w /= l; x /= l; y /= l; z /= l;
    o->qhat[0] = w; o->qhat[1] = x; o->qhat[2] = y; o->qhat[3] = z;
    /* rotation matrix of a unit Hamilton quaternion; columns are t_u, t_v, n */
    o->tu[0] = 1.0 - 2.0 * (y * y + z * z); o->tu[1] = 2.0 * (x * y + w * z); o->tu[2] = 2.0 * (x * z - w * y);
    o->tv[0] = 2.0 * (x * y - w * z); o->tv[1] = 1.0 - 2.0 * (x * x + z * z); o->tv[2] = 2.0 * (y * z + w * x);
    o->n[0] = 2.0 * (x * z + w * y); o->n[1] = 2.0 * (y * z - w * x); o->n[2] = 1.0 - 2.0 * (x * x + y * y);
    for (int i = 0; i < 3; ++i) { o->mu[i] = mu[i]; o->c[i] = rgb ? rgb[i] : 0.0; }
    o->su = sc[0]; o->sv = sc[1]; o->op = op;
}

static int scene_init(Scene *S, int64_t n, const float *means, const float *scales, const float *quats,
                      const float *opacity, const float *rgb, float alpha_min)
{
    S->n = n;
    S->s32 = (Surf32 *)malloc(sizeof(Surf32) * (size_t)(n > 0 ? n : 1));
    S->s64 = (Surf64 *)malloc(sizeof(Surf64) * (size_t)(n > 0 ? n : 1));
    if (!S->s32 || !S->s64) { free(S->s32); free(S->s64); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        prep_one32(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], alpha_min, &S->s32[i]);
        prep_one64(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], rgb ? rgb + 3 * i : NULL, &S->s64[i]);
    }
    return 0;
}

static void scene_free(Scene *S) { free(S->s32); free(S->s64); }

/* ------------------------------------------------------------------------ */
/* One ray against one surfel                                                */
/* ------------------------------------------------------------------------ */

/* Decision in single precision (Eq. raytracing_intersection, then the 2D
 * Gaussian's local coordinates u, v).  Returns 1 on a hit and the depth; the
 * margins record how close each test came to its threshold. */
typedef struct { float r2, den, tau, texel; } Margin;

static int hit32(const Surf32 *s, const float o[3], const float d[3], float tmin, float tmax,
                 float *tau_out, float *r2_out, Margin *mg)
{
    float m0 = s->mu[0] - o[0], m1 = s->mu[1] - o[1], m2 = s->mu[2] - o[2];
    float den = s->n[0] * d[0] + s->n[1] * d[1] + s->n[2] * d[2];
    if (mg) { float a = fabsf(fabsf(den) - 1e-6f); if (a < mg->den) mg->den = a; }
    if (fabsf(den) < 1e-6f) return 0;
    float num = s->n[0] * m0 + s->n[1] * m1 + s->n[2] * m2;
    float tau = num / den;
    int in_range = tau > tmin && tau <= tmax;
    if (!in_range && !mg) return 0;
    float dx = tau * d[0] - m0, dy = tau * d[1] - m1, dz = tau * d[2] - m2;
    float u = s->au[0] * dx + s->au[1] * dy + s->au[2] * dz;
    float v = s->av[0] * dx + s->av[1] * dy + s->av[2] * dz;
    float r2 = u * u + v * v;
    if (mg && s->r2max >= 0.0f && r2 < 4.0f * s->r2max + 1.0f && tau > 0.0f) {
        /* How far each decision is from flipping, expressed as the change of
         * ray direction (radians, to first order) that would flip it.  Only
         * crossings near the support count: far ones cannot flip. */
        float amax = fmaxf(fmaxf(fabsf(s->au[0]), fabsf(s->au[1])), fmaxf(fabsf(s->au[2]),
                     fmaxf(fmaxf(fabsf(s->av[0]), fabsf(s->av[1])), fabsf(s->av[2]))));
        float ad = fabsf(den);
        float sens = 2.0f * sqrtf(r2) * 1.7320508f * amax * tau * (1.0f + 1.0f / ad) + 1e-30f;
        if (in_range) {
            float a = fabsf(r2 - s->r2max) / sens;
            if (a < mg->r2) mg->r2 = a;
        }
        if (r2 <= s->r2max) {
            float b = fabsf(tau - tmin) * ad / tau;
            if (b < mg->tau) mg->tau = b;
        }
    }
    if (!in_range) return 0;
    if (!(r2 <= s->r2max)) return 0;
    *tau_out = tau;
    *r2_out = r2;
    return 1;
}

/* Values in double along the same (single-precision) ray. */
typedef struct { double tau, den, D[3], u, v, r2, G, alpha; } Geo64;

static void geo64(const Surf64 *s, const float of[3], const float df[3], Geo64 *g)
{
    double o[3] = {of[0], of[1], of[2]}, d[3] = {df[0], df[1], df[2]};
    double m[3] = {s->mu[0] - o[0], s->mu[1] - o[1], s->mu[2] - o[2]};
    g->den = s->n[0] * d[0] + s->n[1] * d[1] + s->n[2] * d[2];
    g->tau = (s->n[0] * m[0] + s->n[1] * m[1] + s->n[2] * m[2]) / g->den;
    for (int i = 0; i < 3; ++i) g->D[i] = o[i] + g->tau * d[i] - s->mu[i];  /* p - mu */
    g->u = (s->tu[0] * g->D[0] + s->tu[1] * g->D[1] + s->tu[2] * g->D[2]) / s->su;
    g->v = (s->tv[0] * g->D[0] + s->tv[1] * g->D[1] + s->tv[2] * g->D[2]) / s->sv;
    g->r2 = g->u * g->u + g->v * g->v;
    g->G = exp(-0.5 * g->r2);
    g->alpha = s->op * g->G;
}

/* ------------------------------------------------------------------------ */
/* Ordered hit list and compositing of one ray (Eq. trace)                    */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t key; int64_t id; float r2; } Hit;

static int hit_cmp(const void *a, const void *b)
{
    const Hit *x = (const Hit *)a, *y = (const Hit *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

static uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float bitsf(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

typedef struct {
    Hit *h;          /* all hits, sorted */
    int64_t nh;      /* number of hits on the ray */
    int64_t K;       /* number composited (the stop index) */
    double C[3], T;  /* c_rt and the final transmittance 1 - o_rt */
    Margin mg;       /* closest approach of any decision to its threshold */
    float tstop;     /* |T32 - T_cut| / T_cut at the closest step */
} RayResult;

static void trace_ray(const Scene *S, const float o[3], const float d[3], float tmin, float tmax,
                      float t_cut, RayResult *R)
{
    int64_t cap = 64, nh = 0;
    Hit *h = (Hit *)malloc(sizeof(Hit) * (size_t)cap);
    R->mg.r2 = INFINITY; R->mg.den = INFINITY; R->mg.tau = INFINITY; R->mg.texel = INFINITY;
    for (int64_t i = 0; i < S->n; ++i) {
        float tau, r2;
        if (hit32(&S->s32[i], o, d, tmin, tmax, &tau, &r2, &R->mg)) {
            if (nh == cap) { cap *= 2; h = (Hit *)realloc(h, sizeof(Hit) * (size_t)cap); }
            h[nh].key = ((uint64_t)fbits(tau) << 32) | (uint64_t)(uint32_t)i;
            h[nh].id = i;
            h[nh].r2 = r2;
            ++nh;
        }
    }
    qsort(h, (size_t)nh, sizeof(Hit), hit_cmp);
    /* front to back: C += T alpha c, T *= 1 - alpha; stop after T < T_cut */
    double C[3] = {0, 0, 0}, T = 1.0;
    float T32 = 1.0f;
    float tstop = INFINITY;
    int64_t K = 0;
    for (int64_t k = 0; k < nh; ++k) {
        const Surf64 *s = &S->s64[h[k].id];
        Geo64 g;
        geo64(s, o, d, &g);
        for (int c = 0; c < 3; ++c) C[c] += T * g.alpha * s->c[c];
        T *= 1.0 - g.alpha;
        float a32 = S->s32[h[k].id].op * expf(-0.5f * h[k].r2);
        T32 = T32 * (1.0f - a32);
        K = k + 1;
        float rel = fabsf(T32 - t_cut) / t_cut;
        if (rel < tstop) tstop = rel;
        if (T32 < t_cut) break;
    }
    R->h = h; R->nh = nh; R->K = K;
    R->C[0] = C[0]; R->C[1] = C[1]; R->C[2] = C[2]; R->T = T;
    R->tstop = tstop;
}

/* Gradient of g_C . c_rt + g_T . T_fin w.r.t. every composited surfel, with
 * the hit set, order and stop index held fixed.  Derived from Eq. trace:
 *   dC/dc_k = T_k a_k,  dC/da_k = T_k c_k - (C - P_k)/(1 - a_k),  dT/da_k = -T/(1 - a_k)
 * with P_k the colour composited up to and including hit k; then through
 * a = o G, G = exp(-(u^2+v^2)/2), u = t_u.(p-mu)/s_u, v = t_v.(p-mu)/s_v,
 * p = r_o + tau r_d, tau = n.(mu - r_o)/(n.r_d), and the quaternion frame.
 * Gradients are accumulated into g (13 doubles per surfel:
 * mean 3, scale 2, quat 4, opacity 1, rgb 3). */
/* Chain rule of one composited hit (the hit's alpha through rho^2 = u^2 + v^2
 * of the tangent-plane crossing, Sec. 3.1): from dL/dalpha (dA), dL/dtau
 * (dtau, the hit's depth along the ray) and a direct dL/dn (dnx, NULL = none)
 * to the stored parameters, out[10] = (mean 3, scale 2, quaternion 4,
 * opacity).  The crossing point is x = o + tau d with
 * tau = n.(mu - o) / n.d, so tau moves with mu and n. */
static void hit_chain(const Surf64 *s, const float d[3], const Geo64 *g, double dA, double dtau,
                      const double dnx[3], double out[10])
{
    double a = g->alpha;
    double gamma = -0.5 * a * dA;            /* dL/d(rho^2) */
    double du = 2.0 * g->u * gamma, dv = 2.0 * g->v * gamma;
    double dsu = -(g->u / s->su) * du, dsv = -(g->v / s->sv) * dv;
    double gD[3], dtu[3], dtv[3], dn[3], dmu[3];
    for (int i = 0; i < 3; ++i) gD[i] = du * s->tu[i] / s->su + dv * s->tv[i] / s->sv;
    /* total dL/dtau: through the crossing point, plus the direct term */
    double gDd = (gD[0] * d[0] + gD[1] * d[1] + gD[2] * d[2] + dtau) / g->den;
    for (int i = 0; i < 3; ++i) {
        dmu[i] = gDd * s->n[i] - gD[i];
        dtu[i] = du * g->D[i] / s->su;
        dtv[i] = dv * g->D[i] / s->sv;
        dn[i] = -gDd * g->D[i] + (dnx ? dnx[i] : 0.0);
    }
    /* columns of R(q) -> unit quaternion (w,x,y,z) */
    double qw = s->qhat[0], qx = s->qhat[1], qy = s->qhat[2], qz = s->qhat[3];
    double dq[4];
    dq[0] = dtu[1] * (2 * qz) + dtu[2] * (-2 * qy)
          + dtv[0] * (-2 * qz) + dtv[2] * (2 * qx)
          + dn[0] * (2 * qy) + dn[1] * (-2 * qx);
    dq[1] = dtu[1] * (2 * qy) + dtu[2] * (2 * qz)
          + dtv[0] * (2 * qy) + dtv[1] * (-4 * qx) + dtv[2] * (2 * qw)
          + dn[0] * (2 * qz) + dn[1] * (-2 * qw) + dn[2] * (-4 * qx);
    dq[2] = dtu[0] * (-4 * qy) + dtu[1] * (2 * qx) + dtu[2] * (-2 * qw)
          + dtv[0] * (2 * qx) + dtv[2] * (2 * qz)
          + dn[0] * (2 * qw) + dn[1] * (2 * qz) + dn[2] * (-4 * qy);
    dq[3] = dtu[0] * (-4 * qz) + dtu[1] * (2 * qw) + dtu[2] * (2 * qx)
          + dtv[0] * (-2 * qw) + dtv[1] * (-4 * qz) + dtv[2] * (2 * qy)
          + dn[0] * (2 * qx) + dn[1] * (2 * qy);
    /* unit quaternion -> stored quaternion: (I - qhat qhat^T) / |q| */
    double proj = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
    out[0] = dmu[0]; out[1] = dmu[1]; out[2] = dmu[2];
    out[3] = dsu; out[4] = dsv;
    for (int i = 0; i < 4; ++i) out[5 + i] = (dq[i] - s->qhat[i] * proj) / s->qlen;
    out[9] = g->G * dA;
}

/* dst += src; with dst_abs (may be NULL) also dst_abs += |src|. */
static void add_grads(double *dst, double *dst_abs, const double *src, int m)
{
    for (int i = 0; i < m; ++i) {
#ifdef _OPENMP
#pragma omp atomic
#endif
        dst[i] += src[i];
        if (dst_abs) {
#ifdef _OPENMP
#pragma omp atomic
#endif
            dst_abs[i] += fabs(src[i]);
        }
    }
}

static void backward_ray(const Scene *S, const float o[3], const float d[3], const RayResult *R,
                         const double gC[3], double gT, double *g13, double *g13_abs, double *dmu_sum,
                         double *dmu_abs)
{
    double T = 1.0, P[3] = {0, 0, 0};
    for (int64_t k = 0; k < R->K; ++k) {
        int64_t id = R->h[k].id;
        const Surf64 *s = &S->s64[id];
        Geo64 g;
        geo64(s, o, d, &g);
        double a = g.alpha;
        double w = T * a;
        for (int c = 0; c < 3; ++c) P[c] += w * s->c[c];
        double dA = T * (gC[0] * s->c[0] + gC[1] * s->c[1] + gC[2] * s->c[2]);
        if (1.0 - a >= 1e-6) {
            double behind = gC[0] * (R->C[0] - P[0]) + gC[1] * (R->C[1] - P[1]) + gC[2] * (R->C[2] - P[2]) + gT * R->T;
            dA -= behind / (1.0 - a);
        }
        double add[13];
        hit_chain(s, d, &g, dA, 0.0, NULL, add);
        for (int c = 0; c < 3; ++c) add[10 + c] = w * gC[c];
        add_grads(g13 + 13 * id, NULL, add, 13);
        if (dmu_sum)
            for (int c = 0; c < 3; ++c) dmu_sum[c] += add[c];
        if (g13_abs) {
            /* error scale: each term's own magnitude, plus the chain applied
             * to the magnitudes dL/dalpha is formed from (a single-precision
             * path forms C - P_k as a difference of running sums) */
            double dAs = T * (fabs(gC[0] * s->c[0]) + fabs(gC[1] * s->c[1]) + fabs(gC[2] * s->c[2]));
            if (1.0 - a >= 1e-6) {
                double m = fabs(gT * R->T);
                for (int c = 0; c < 3; ++c) m += fabs(gC[c]) * (fabs(R->C[c]) + fabs(P[c]));
                dAs += m / (1.0 - a);
            }
            double sc[13];
            hit_chain(s, d, &g, dAs, 0.0, NULL, sc);
            for (int i = 0; i < 13; ++i) sc[i] = fabs(add[i]) + (i < 10 ? fabs(sc[i]) : 0.0);
            add_grads(g13_abs + 13 * id, NULL, sc, 13);
            if (dmu_abs)
                for (int c = 0; c < 3; ++c) dmu_abs[c] += sc[c];
        }
        T *= 1.0 - a;
    }
}

/* ------------------------------------------------------------------------ */
/* Exported: trace (Eq. trace with L_i = c_rt + T sky, Eq. lighting_decompose) */
/* ------------------------------------------------------------------------ */

/*
 * rays: origins/dirs [R,3] float; t_min/t_max per ray (or NULL: scalars).
 * outputs (any may be NULL): C [R,3], T [R], L [R,3], nhit [R] composited,
 * dump_id/dump_tau [R,cap] of composited hits in order, margins [R,5] =
 * (support margin in radians of ray direction, |den| margin, tau margin,
 * relative stop margin, environment texel margin (infinite here)).
 */
int orc_trace(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
              const float *rgb, float alpha_min,
              int64_t nr, const float *orig, const float *dirs, const float *tmin_a, const float *tmax_a,
              float tmin_s, float tmax_s, float t_cut, const float *sky,
              double *outC, double *outT, double *outL, int32_t *nhit,
              int64_t cap, int32_t *dump_id, float *dump_tau, float *margins)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, rgb, alpha_min)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        float tmin = tmin_a ? tmin_a[r] : tmin_s, tmax = tmax_a ? tmax_a[r] : tmax_s;
        if (!(tmin >= 0.0f)) tmin = 0.0f; /* a ray starts at its origin: negative t_min is 0 */
        RayResult R;
        trace_ray(&S, orig + 3 * r, dirs + 3 * r, tmin, tmax, t_cut, &R);
        for (int c = 0; c < 3; ++c) {
            if (outC) outC[3 * r + c] = R.C[c];
            if (outL) outL[3 * r + c] = R.C[c] + R.T * (double)sky[c];
        }
        if (outT) outT[r] = R.T;
        if (nhit) nhit[r] = (int32_t)R.K;
        if (dump_id) {
            for (int64_t k = 0; k < cap; ++k) {
                dump_id[r * cap + k] = k < R.K ? (int32_t)R.h[k].id : -1;
                dump_tau[r * cap + k] = k < R.K ? bitsf((uint32_t)(R.h[k].key >> 32)) : 0.0f;
            }
        }
        if (margins) {
            margins[5 * r + 0] = R.mg.r2; margins[5 * r + 1] = R.mg.den;
            margins[5 * r + 2] = R.mg.tau; margins[5 * r + 3] = R.tstop; margins[5 * r + 4] = R.mg.texel;
        }
        free(R.h);
    }
    scene_free(&S);
    return 0;
}

/* Attribute query of one ray per ray (Sec. 3.5.1, Eq. trace_attr, the
 * Gaussian backend): along the same ordered, cut-off hit list as orc_trace,
 * the material attributes of the composited surfels averaged with the
 * normalized blending weights w_k = T_k a_k / sum_j T_j a_j (the weights of
 * Eq. deferred_maps), and V = the final transmittance (visibility of the
 * environment, 1 - o_rt).  A surfel's normal n = t_u x t_v enters facing the
 * ray origin (negated when n . d > 0).  With no composited hit: V = 1 and
 * every attribute 0.  Outputs (double): V [nr], albedo [nr,3], rough [nr],
 * metal [nr], normal [nr,3] (the weighted average, not renormalized). */
typedef struct { const float *albedo, *rough, *metal; } Attrs;
typedef struct { double V, a[3], r, m, n[3]; } AttrOut;

static void attr_of_ray(const Scene *S, const Attrs *at, const float o[3], const float d[3], const RayResult *R,
                        AttrOut *out)
{
    double T = 1.0, W = 0.0, A[3] = {0, 0, 0}, Rg = 0.0, M = 0.0, N[3] = {0, 0, 0};
    for (int64_t k = 0; k < R->K; ++k) {
        int64_t id = R->h[k].id;
        const Surf64 *sf = &S->s64[id];
        Geo64 g;
        geo64(sf, o, d, &g);
        double w = T * g.alpha;
        double sgn = g.den > 0.0 ? -1.0 : 1.0;
        W += w;
        for (int c = 0; c < 3; ++c) {
            A[c] += w * (double)at->albedo[3 * id + c];
            N[c] += w * sgn * sf->n[c];
        }
        Rg += w * (double)at->rough[id];
        M += w * (double)at->metal[id];
        T *= 1.0 - g.alpha;
    }
    double inv = W > 0.0 ? 1.0 / W : 0.0;
    out->V = R->T;
    for (int c = 0; c < 3; ++c) {
        out->a[c] = A[c] * inv;
        out->n[c] = N[c] * inv;
    }
    out->r = Rg * inv;
    out->m = M * inv;
}

int orc_trace_attr(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                   float alpha_min, const float *albedo, const float *rough, const float *metal,
                   int64_t nr, const float *orig, const float *dirs, float tmin_s, float tmax_s, float t_cut,
                   double *outV, double *outA, double *outR, double *outM, double *outN)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, NULL, alpha_min)) return -1;
    Attrs at = {albedo, rough, metal};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        const float *o = orig + 3 * r, *d = dirs + 3 * r;
        RayResult R;
        trace_ray(&S, o, d, tmin_s, tmax_s, t_cut, &R);
        AttrOut q;
        attr_of_ray(&S, &at, o, d, &R, &q);
        outV[r] = q.V;
        for (int c = 0; c < 3; ++c) {
            outA[3 * r + c] = q.a[c];
            outN[3 * r + c] = q.n[c];
        }
        outR[r] = q.r;
        outM[r] = q.m;
        free(R.h);
    }
    scene_free(&S);
    return 0;
}

/* Primary-ray G-buffer by 2DGRT (Sec. 3.3, Eq. deferred_maps, with the
 * primary rays traced instead of rasterized): along each camera ray's
 * ordered, cut-off hits, the deferred maps are the normalized-weight
 * averages sum w_k {c_k, d_k, n_k, a_k, r_k, m_k}, w_k = T_k a_k / sum_j T_j a_j,
 * d_k the depth tau_k of the hit, n_k facing the camera.  The pixel is
 * covered (valid) when its accumulated opacity 1 - T reaches min_opacity;
 * then the G-buffer holds x = o + D d, the unit normal N / |N|, wo = -d and
 * the material maps; otherwise every entry is 0.  Outputs (double):
 * x, n, wo, albedo [nr,3], rough, metal, depth [nr], rgb [nr,3] (C, the
 * normalized radiance map, 0 where not covered), valid [nr] (uint8). */
int orc_trace_gbuffer(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                      const float *rgb, float alpha_min, const float *albedo, const float *rough, const float *metal,
                      int64_t nr, const float *orig, const float *dirs, float tmin_s, float tmax_s, float t_cut,
                      double min_opacity, double *ox, double *on, double *owo, double *oa, double *orough,
                      double *ometal, double *odepth, double *orgb, uint8_t *ovalid)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, rgb, alpha_min)) return -1;
    Attrs at = {albedo, rough, metal};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        const float *o = orig + 3 * r, *d = dirs + 3 * r;
        RayResult R;
        trace_ray(&S, o, d, tmin_s, tmax_s, t_cut, &R);
        AttrOut q;
        attr_of_ray(&S, &at, o, d, &R, &q);
        /* depth and colour maps with the same weights */
        double T = 1.0, W = 0.0, Dm = 0.0, C[3] = {0, 0, 0};
        for (int64_t k = 0; k < R.K; ++k) {
            const Surf64 *sf = &S.s64[R.h[k].id];
            Geo64 g;
            geo64(sf, o, d, &g);
            double w = T * g.alpha;
            W += w;
            Dm += w * g.tau;
            for (int c = 0; c < 3; ++c) C[c] += w * sf->c[c];
            T *= 1.0 - g.alpha;
        }
        double inv = W > 0.0 ? 1.0 / W : 0.0;
        int valid = 1.0 - q.V >= min_opacity && W > 0.0;
        double nl = sqrt(q.n[0] * q.n[0] + q.n[1] * q.n[1] + q.n[2] * q.n[2]);
        if (!(nl > 0.0)) valid = 0;
        double D = Dm * inv;
        for (int c = 0; c < 3; ++c) {
            ox[3 * r + c] = valid ? (double)o[c] + D * (double)d[c] : 0.0;
            on[3 * r + c] = valid ? q.n[c] / nl : 0.0;
            owo[3 * r + c] = valid ? -(double)d[c] : 0.0;
            oa[3 * r + c] = valid ? q.a[c] : 0.0;
            orgb[3 * r + c] = valid ? C[c] * inv : 0.0;
        }
        orough[r] = valid ? q.r : 0.0;
        ometal[r] = valid ? q.m : 0.0;
        odepth[r] = valid ? D : 0.0;
        ovalid[r] = (uint8_t)valid;
        free(R.h);
    }
    scene_free(&S);
    return 0;
}

/* Gradient of the primary-ray G-buffer of orc_trace_gbuffer (Eq.
 * deferred_maps on traced camera rays):
 *   L = sum over covered pixels of gx.x + gn.n + ga.albedo + gr rough
 *       + gm metal + gd depth + gc.rgb
 * with upstream gradients gx, gn, ga, gc [R,3] and gr, gm, gd [R] (double,
 * NULL = zero).  An uncovered pixel's maps are constant zeros, and the
 * coverage test itself is not differentiated.  g13 [n,13] (as
 * orc_trace_backward) and gattr [n,5] (albedo 3, roughness, metallic) are
 * overwritten.
 * Written from the definitions: every map is a ratio S_f / W of blended sums
 * S_f = sum_k w_k f_k, W = sum_k w_k, w_k = T_k alpha_k, and
 * n = N / |N| with N = sum_k w_k s_k n_k (s_k turns the surfel normal toward
 * the camera).  With the hits' values held fixed, dL/dw_k = e_k, and
 * w_i depends on alpha_k through T_i for i > k:
 *   dw_k/dalpha_k = T_k,  dw_i/dalpha_k = -alpha_i prod_{j<i, j!=k} (1 - alpha_j).
 * The hit's depth tau_k, normal n_k, colour and attributes get their direct
 * terms w_k dL/dS_f. */
int orc_trace_gbuffer_backward(int64_t n, const float *means, const float *scales, const float *quats,
                               const float *opacity, const float *rgb, float alpha_min, const float *albedo,
                               const float *rough, const float *metal, int64_t nr, const float *orig,
                               const float *dirs, float tmin_s, float tmax_s, float t_cut, double min_opacity,
                               const double *gx, const double *gn, const double *ga, const double *gr,
                               const double *gm, const double *gd, const double *gc, double *g13, double *gattr,
                               double *g13_abs, double *gattr_abs)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, rgb, alpha_min)) return -1;
    memset(g13, 0, sizeof(double) * 13 * (size_t)n);
    memset(gattr, 0, sizeof(double) * 5 * (size_t)n);
    if (g13_abs) memset(g13_abs, 0, sizeof(double) * 13 * (size_t)n);
    if (gattr_abs) memset(gattr_abs, 0, sizeof(double) * 5 * (size_t)n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        const float *o = orig + 3 * r, *d = dirs + 3 * r;
        RayResult R;
        trace_ray(&S, o, d, tmin_s, tmax_s, t_cut, &R);
        int64_t K = R.K;
        Geo64 *geo = (Geo64 *)malloc(sizeof(Geo64) * (size_t)(K > 0 ? K : 1));
        double *Tk = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
        double *e = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
        double *es = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
        /* forward sums */
        double T = 1.0, W = 0.0, SD = 0.0, SA[3] = {0, 0, 0}, SR = 0.0, SM = 0.0, SC[3] = {0, 0, 0};
        double N[3] = {0, 0, 0};
        for (int64_t k = 0; k < K; ++k) {
            int64_t id = R.h[k].id;
            const Surf64 *sf = &S.s64[id];
            geo64(sf, o, d, &geo[k]);
            Tk[k] = T;
            double w = T * geo[k].alpha;
            double sgn = geo[k].den > 0.0 ? -1.0 : 1.0;
            W += w;
            SD += w * geo[k].tau;
            for (int c = 0; c < 3; ++c) {
                SA[c] += w * (double)albedo[3 * id + c];
                SC[c] += w * sf->c[c];
                N[c] += w * sgn * sf->n[c];
            }
            SR += w * (double)rough[id];
            SM += w * (double)metal[id];
            T *= 1.0 - geo[k].alpha;
        }
        double nbar = W > 0.0 ? sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]) / W : 0.0;
        int valid = 1.0 - R.T >= min_opacity && W > 0.0 && nbar > 0.0;
        if (valid) {
            double D = SD / W, A[3], C[3], Rm = SR / W, Mm = SM / W;
            double nl = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]), nh[3];
            for (int c = 0; c < 3; ++c) {
                A[c] = SA[c] / W;
                C[c] = SC[c] / W;
                nh[c] = N[c] / nl;
            }
            const double zero3[3] = {0, 0, 0};
            const double *pgx = gx ? gx + 3 * r : zero3, *pgn = gn ? gn + 3 * r : zero3;
            const double *pga = ga ? ga + 3 * r : zero3, *pgc = gc ? gc + 3 * r : zero3;
            double grr = gr ? gr[r] : 0.0, gmm = gm ? gm[r] : 0.0;
            /* x = o + D d: the hit-point map moves with the depth only */
            double gD = (gd ? gd[r] : 0.0) + pgx[0] * d[0] + pgx[1] * d[1] + pgx[2] * d[2];
            /* d(N/|N|)/dN applied to gn */
            double ndg = nh[0] * pgn[0] + nh[1] * pgn[1] + nh[2] * pgn[2], gN[3];
            for (int c = 0; c < 3; ++c) gN[c] = (pgn[c] - nh[c] * ndg) / nl;
            for (int64_t k = 0; k < K; ++k) {
                int64_t id = R.h[k].id;
                const Surf64 *sf = &S.s64[id];
                double sgn = geo[k].den > 0.0 ? -1.0 : 1.0, ek = gD * (geo[k].tau - D);
                for (int c = 0; c < 3; ++c)
                    ek += pga[c] * ((double)albedo[3 * id + c] - A[c]) + pgc[c] * (sf->c[c] - C[c]);
                ek += grr * ((double)rough[id] - Rm) + gmm * ((double)metal[id] - Mm);
                e[k] = ek / W + sgn * (sf->n[0] * gN[0] + sf->n[1] * gN[1] + sf->n[2] * gN[2]);
                /* magnitudes of the summands of e_k (the error scale of a
                 * single-precision e_k) */
                double m = fabs(gD * geo[k].tau) + fabs(gD * D) + fabs(grr * (double)rough[id]) + fabs(grr * Rm) +
                           fabs(gmm * (double)metal[id]) + fabs(gmm * Mm);
                for (int c = 0; c < 3; ++c)
                    m += fabs(pga[c] * (double)albedo[3 * id + c]) + fabs(pga[c] * A[c]) + fabs(pgc[c] * sf->c[c]) +
                         fabs(pgc[c] * C[c]);
                es[k] = m / W + fabs(sf->n[0] * gN[0]) + fabs(sf->n[1] * gN[1]) + fabs(sf->n[2] * gN[2]);
            }
            double Ps = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                int64_t id = R.h[k].id;
                const Surf64 *sf = &S.s64[id];
                double dA = e[k] * Tk[k], prod = Tk[k];
                for (int64_t i = k + 1; i < K; ++i) {
                    dA -= e[i] * geo[i].alpha * prod;
                    prod *= 1.0 - geo[i].alpha;
                }
                double w = Tk[k] * geo[k].alpha, sgn = geo[k].den > 0.0 ? -1.0 : 1.0;
                double dnx[3] = {w * sgn * gN[0], w * sgn * gN[1], w * sgn * gN[2]};
                double add[13], at[5];
                hit_chain(sf, d, &geo[k], dA, w * gD / W, dnx, add);
                for (int c = 0; c < 3; ++c) {
                    add[10 + c] = w * pgc[c] / W;
                    at[c] = w * pga[c] / W;
                }
                at[3] = w * grr / W;
                at[4] = w * gmm / W;
                add_grads(g13 + 13 * id, NULL, add, 13);
                add_grads(gattr + 5 * id, gattr_abs ? gattr_abs + 5 * id : NULL, at, 5);
                if (g13_abs) {
                    /* error scale: the terms' magnitudes, plus the chain
                     * applied to the magnitudes dL/dalpha_k is formed from
                     * (a single-precision path forms the part behind hit k
                     * as minus the running sum of w_i e_i in front of it) */
                    Ps += w * es[k];
                    double dAs = Tk[k] * es[k] + (1.0 - geo[k].alpha >= 1e-6 ? Ps / (1.0 - geo[k].alpha) : 0.0);
                    double sc[13];
                    hit_chain(sf, d, &geo[k], dAs, 0.0, NULL, sc);
                    for (int i = 0; i < 13; ++i) sc[i] = fabs(add[i]) + (i < 10 ? fabs(sc[i]) : 0.0);
                    add_grads(g13_abs + 13 * id, NULL, sc, 13);
                }
            }
        }
        free(geo);
        free(Tk);
        free(e);
        free(es);
        free(R.h);
    }
    scene_free(&S);
    return 0;
}

/* Gradient of sum_r (gC_r . c_rt(r) + gT_r T_fin(r)) w.r.t. the surfels.
 * g13 [n,13] is overwritten (mean 3, scale 2, quat 4, opacity 1, rgb 3). */
int orc_trace_backward(int64_t n, const float *means, const float *scales, const float *quats,
                       const float *opacity, const float *rgb, float alpha_min,
                       int64_t nr, const float *orig, const float *dirs, const float *tmin_a, const float *tmax_a,
                       float tmin_s, float tmax_s, float t_cut,
                       const double *gC, const double *gT, double *g13, double *g13_abs)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, rgb, alpha_min)) return -1;
    memset(g13, 0, sizeof(double) * 13 * (size_t)n);
    if (g13_abs) memset(g13_abs, 0, sizeof(double) * 13 * (size_t)n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        float tmin = tmin_a ? tmin_a[r] : tmin_s, tmax = tmax_a ? tmax_a[r] : tmax_s;
        if (!(tmin >= 0.0f)) tmin = 0.0f; /* a ray starts at its origin: negative t_min is 0 */
        RayResult R;
        trace_ray(&S, orig + 3 * r, dirs + 3 * r, tmin, tmax, t_cut, &R);
        backward_ray(&S, orig + 3 * r, dirs + 3 * r, &R, gC + 3 * r, gT[r], g13, g13_abs, NULL, NULL);
        free(R.h);
    }
    scene_free(&S);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Environment map: luminance x sin(theta) distribution (Sec. 3.4.1, the      */
/* environment-light proposal; piecewise-constant 2D sampling after Pharr)    */
/* ------------------------------------------------------------------------ */

/* marg [H+1] and cond [H, W+1]: cumulative sums in double, one row at a
 * time from the left, divided by the total, rounded to float; the last entry
 * of each table is exactly 1.  A row of zero weight gets a uniform table. */
int orc_env_cdf(int H, int W, const float *rgb, float *marg, float *cond)
{
    double *rows = (double *)malloc(sizeof(double) * (size_t)H);
    for (int i = 0; i < H; ++i) {
        double st = sin(ORC_PI * (i + 0.5) / H);
        double acc = 0.0;
        float *cr = cond + (size_t)i * (W + 1);
        double *tmp = (double *)malloc(sizeof(double) * (size_t)(W + 1));
        tmp[0] = 0.0;
        for (int j = 0; j < W; ++j) {
            const float *p = rgb + ((size_t)i * W + j) * 3;
            double lum = 0.2126 * (double)p[0] + 0.7152 * (double)p[1] + 0.0722 * (double)p[2];
            acc += lum * st;
            tmp[j + 1] = acc;
        }
        rows[i] = acc;
        cr[0] = 0.0f;
        for (int j = 1; j <= W; ++j)
            cr[j] = acc > 0.0 ? (float)(tmp[j] / acc) : (float)((double)j / W);
        cr[W] = 1.0f;
        free(tmp);
    }
    double tot = 0.0;
    for (int i = 0; i < H; ++i) tot += rows[i];
    double acc = 0.0;
    marg[0] = 0.0f;
    for (int i = 0; i < H; ++i) {
        acc += rows[i];
        marg[i + 1] = tot > 0.0 ? (float)(acc / tot) : (float)((double)(i + 1) / H);
    }
    marg[H] = 1.0f;
    free(rows);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                         */
/* ------------------------------------------------------------------------ */

static void philox(uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* the two uniforms of sample j of pixel p in job `job` */
static void uniforms(uint64_t seed, uint32_t pix, uint32_t j, uint32_t job, double *u1, double *u2)
{
    uint32_t ctr[4] = {pix, j, job, 0}, out[4];
    philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
    *u1 = (double)(out[0] >> 8) * (1.0 / 16777216.0);
    *u2 = (double)(out[1] >> 8) * (1.0 / 16777216.0);
}

/* exported for the generator's statistical tests */
void orc_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t *out)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

/* ------------------------------------------------------------------------ */
/* BRDF and proposals (Sec. 3.1 Eqs. brdf_decompose/brdf_specular; Sec. 3.4.1) */
/* ------------------------------------------------------------------------ */

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void normalize3(double a[3])
{
    double l = sqrt(dot3(a, a));
    a[0] /= l; a[1] /= l; a[2] /= l;
}

/* orthonormal basis around n (Duff et al., JCGT 2017) */
static void onb(const double n[3], double b1[3], double b2[3])
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a; b1[1] = sign * b; b1[2] = -sign * n[0];
    b2[0] = b; b2[1] = sign + n[1] * n[1] * a; b2[2] = -n[1];
}

static double ggx_D(double ndh, double a2)
{
    double t = ndh * ndh * (a2 - 1.0) + 1.0;
    return a2 / (ORC_PI * t * t);
}

static double smith_G1(double ndv, double a2)
{
    return 2.0 * ndv / (ndv + sqrt(a2 + (1.0 - a2) * ndv * ndv));
}

/* f(wo, wi) for ndi > 0, ndo > 0 (per channel) */
static void brdf(const double n[3], const double wo[3], const double wi[3], const double alb[3], double rough,
                 double metal, double f[3])
{
    double ndi = dot3(n, wi), ndo = dot3(n, wo);
    double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    normalize3(h);
    double ndh = dot3(n, h), idh = dot3(wi, h);
    double a = rough * rough, a2 = a * a;
    double D = ggx_D(ndh, a2);
    double G = smith_G1(ndi, a2) * smith_G1(ndo, a2);
    double x = 1.0 - idh;
    if (x < 0.0) x = 0.0;
    double x5 = x * x * x * x * x;
    for (int c = 0; c < 3; ++c) {
        double F0 = 0.04 * (1.0 - metal) + metal * alb[c];
        double F = F0 + (1.0 - F0) * x5;
        f[c] = (1.0 - metal) * alb[c] / ORC_PI + D * F * G / (4.0 * ndi * ndo);
    }
}

/* f(wo, wi) of brdf() and its partial derivatives with respect to its
 * arguments taken as free vectors and scalars (Sec. 3.1 Eq. brdf_specular,
 * differentiated by hand): dn[c][i] = df_c/dn_i, dwo[c][i] = df_c/dwo_i,
 * da[c] = df_c/da_c, dr[c] = df_c/d(roughness), dm[c] = df_c/d(metallic).
 * With h = (wi + wo)/|wi + wo|, a2 = r^4, t = (n.h)^2 (a2 - 1) + 1,
 * S = D F G1(n.wi) G1(n.wo) / (4 n.wi n.wo):
 *   dD/d(n.h) = -4 a2 (n.h)(a2 - 1) / (pi t^3),  dD/da2 = 1/(pi t^2) - 2 a2 (n.h)^2/(pi t^3)
 *   G1(v) = 2v/(v + s), s = sqrt(a2 + (1 - a2) v^2): dG1/dv = 2 (s - v ds/dv)/(v + s)^2,
 *   ds/dv = (1 - a2) v / s, dG1/da2 = -2 v (ds/da2)/(v + s)^2, ds/da2 = (1 - v^2)/(2 s)
 *   dF/d(wi.h) = -5 (1 - F0) (1 - wi.h)^4,  dh/dwo = (I - h h^T)/|wi + wo|. */
static void brdf_partials(const double n[3], const double wo[3], const double wi[3], const double alb[3],
                          double rough, double metal, double f[3], double dn[3][3], double dwo[3][3], double da[3],
                          double dr[3], double dm[3])
{
    double ndi = dot3(n, wi), ndo = dot3(n, wo);
    double hs[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    double hl = sqrt(dot3(hs, hs));
    double h[3] = {hs[0] / hl, hs[1] / hl, hs[2] / hl};
    double ndh = dot3(n, h), idh = dot3(wi, h);
    double a = rough * rough, a2 = a * a;
    double t = ndh * ndh * (a2 - 1.0) + 1.0;
    double D = a2 / (ORC_PI * t * t);
    double dD_dnh = -4.0 * a2 * ndh * (a2 - 1.0) / (ORC_PI * t * t * t);
    double dD_da2 = 1.0 / (ORC_PI * t * t) - 2.0 * a2 * ndh * ndh / (ORC_PI * t * t * t);
    double vs[2] = {ndi, ndo}, G1[2], dG1[2], dG1a[2];
    for (int k = 0; k < 2; ++k) {
        double v = vs[k], sq = sqrt(a2 + (1.0 - a2) * v * v);
        double ds_dv = (1.0 - a2) * v / sq, ds_da = (1.0 - v * v) / (2.0 * sq);
        G1[k] = 2.0 * v / (v + sq);
        dG1[k] = 2.0 * (sq - v * ds_dv) / ((v + sq) * (v + sq));
        dG1a[k] = -2.0 * v * ds_da / ((v + sq) * (v + sq));
    }
    double G = G1[0] * G1[1];
    double x = 1.0 - idh;
    if (x < 0.0) x = 0.0;
    double x4 = x * x * x * x, x5 = x4 * x;
    double den = 4.0 * ndi * ndo;
    double dnh_dwo[3], dih_dwo[3];
    for (int i = 0; i < 3; ++i) {
        dnh_dwo[i] = (n[i] - h[i] * ndh) / hl;
        dih_dwo[i] = (wi[i] - h[i] * idh) / hl;
    }
    for (int c = 0; c < 3; ++c) {
        double F0 = 0.04 * (1.0 - metal) + metal * alb[c];
        double F = F0 + (1.0 - F0) * x5;
        double S = D * F * G / den;
        f[c] = (1.0 - metal) * alb[c] / ORC_PI + S;
        double dF_dih = x > 0.0 ? -5.0 * (1.0 - F0) * x4 : 0.0;
        /* S through n.wi and n.wo (numerator G1 and the denominator) */
        double dS_dni = D * F * G1[1] / (4.0 * ndo) * (dG1[0] * ndi - G1[0]) / (ndi * ndi);
        double dS_dno = D * F * G1[0] / (4.0 * ndi) * (dG1[1] * ndo - G1[1]) / (ndo * ndo);
        double dS_dnh = dD_dnh * F * G / den;
        double dS_dih = D * dF_dih * G / den;
        for (int i = 0; i < 3; ++i) {
            dn[c][i] = dS_dni * wi[i] + dS_dno * wo[i] + dS_dnh * h[i];
            dwo[c][i] = dS_dno * n[i] + dS_dnh * dnh_dwo[i] + dS_dih * dih_dwo[i];
        }
        double dG_da2 = dG1a[0] * G1[1] + G1[0] * dG1a[1];
        dr[c] = (dD_da2 * F * G + D * F * dG_da2) / den * 4.0 * rough * rough * rough;
        da[c] = (1.0 - metal) / ORC_PI + D * G / den * (1.0 - x5) * metal;
        dm[c] = -alb[c] / ORC_PI + D * G / den * (1.0 - x5) * (alb[c] - 0.04);
    }
}

typedef struct {
    int H, W;
    const float *rgb;
    const float *marg, *cond;
} Env;

static void env_index(const Env *E, const double w[3], int *i, int *j, double *sin_t)
{
    double y = w[1] < -1.0 ? -1.0 : (w[1] > 1.0 ? 1.0 : w[1]);
    double th = acos(y);
    double ph = atan2(w[2], w[0]);
    if (ph < 0.0) ph += 2.0 * ORC_PI;
    int ii = (int)(th / ORC_PI * E->H), jj = (int)(ph / (2.0 * ORC_PI) * E->W);
    *i = ii < E->H - 1 ? ii : E->H - 1;
    *j = jj < E->W - 1 ? jj : E->W - 1;
    if (*i < 0) *i = 0;
    if (*j < 0) *j = 0;
    *sin_t = sqrt(1.0 - y * y > 0.0 ? 1.0 - y * y : 0.0);
}

static double env_pdf(const Env *E, const double w[3])
{
    int i, j;
    double st;
    env_index(E, w, &i, &j, &st);
    if (st <= 0.0) return 0.0;
    const float *cr = E->cond + (size_t)i * (E->W + 1);
    double pij = ((double)E->marg[i + 1] - (double)E->marg[i]) * ((double)cr[j + 1] - (double)cr[j]);
    return pij * E->H * E->W / (2.0 * ORC_PI * ORC_PI * st);
}

static void env_radiance(const Env *E, const double w[3], double L[3])
{
    int i, j;
    double st;
    env_index(E, w, &i, &j, &st);
    const float *p = E->rgb + ((size_t)i * E->W + j) * 3;
    L[0] = p[0]; L[1] = p[1]; L[2] = p[2];
}

/* first k in [0,n) with cdf[k+1] > u (cdf[n] == 1 > u) */
static int cdf_find(const float *cdf, int n, double u)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if ((double)cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static void sample_env(const Env *E, double u1, double u2, double w[3])
{
    int i = cdf_find(E->marg, E->H, u1);
    double dv = (u1 - E->marg[i]) / ((double)E->marg[i + 1] - (double)E->marg[i]);
    const float *cr = E->cond + (size_t)i * (E->W + 1);
    int j = cdf_find(cr, E->W, u2);
    double du = (u2 - cr[j]) / ((double)cr[j + 1] - (double)cr[j]);
    double th = ORC_PI * (i + dv) / E->H, ph = 2.0 * ORC_PI * (j + du) / E->W;
    w[0] = sin(th) * cos(ph); w[1] = cos(th); w[2] = sin(th) * sin(ph);
}

/* cosine-weighted direction (Malley: uniform disk lifted to the hemisphere) */
static void sample_cos(const double n[3], double u1, double u2, double w[3])
{
    double b1[3], b2[3];
    onb(n, b1, b2);
    double r = sqrt(u1), ph = 2.0 * ORC_PI * u2;
    double x = r * cos(ph), y = r * sin(ph), z = sqrt(1.0 - u1 > 0.0 ? 1.0 - u1 : 0.0);
    for (int i = 0; i < 3; ++i) w[i] = x * b1[i] + y * b2[i] + z * n[i];
}

/* visible-normal GGX sample (Heitz, JCGT 2018), then mirror wo about h */
static void sample_ggx(const double n[3], const double wo[3], double rough, double u1, double u2, double w[3])
{
    double b1[3], b2[3];
    onb(n, b1, b2);
    double a = rough * rough;
    double vl[3] = {dot3(wo, b1), dot3(wo, b2), dot3(wo, n)};
    double Vh[3] = {a * vl[0], a * vl[1], vl[2]};
    normalize3(Vh);
    double lensq = Vh[0] * Vh[0] + Vh[1] * Vh[1];
    double T1[3] = {1.0, 0.0, 0.0};
    if (lensq > 0.0) { double il = 1.0 / sqrt(lensq); T1[0] = -Vh[1] * il; T1[1] = Vh[0] * il; T1[2] = 0.0; }
    double T2[3] = {Vh[1] * T1[2] - Vh[2] * T1[1], Vh[2] * T1[0] - Vh[0] * T1[2], Vh[0] * T1[1] - Vh[1] * T1[0]};
    double r = sqrt(u1), ph = 2.0 * ORC_PI * u2;
    double t1 = r * cos(ph), t2 = r * sin(ph);
    double s = 0.5 * (1.0 + Vh[2]);
    t2 = (1.0 - s) * sqrt(1.0 - t1 * t1) + s * t2;
    double t3 = 1.0 - t1 * t1 - t2 * t2;
    t3 = sqrt(t3 > 0.0 ? t3 : 0.0);
    double Nh[3];
    for (int i = 0; i < 3; ++i) Nh[i] = t1 * T1[i] + t2 * T2[i] + t3 * Vh[i];
    double Ne[3] = {a * Nh[0], a * Nh[1], Nh[2] > 0.0 ? Nh[2] : 0.0};
    normalize3(Ne);
    double h[3];
    for (int i = 0; i < 3; ++i) h[i] = Ne[0] * b1[i] + Ne[1] * b2[i] + Ne[2] * n[i];
    double oh = dot3(wo, h);
    for (int i = 0; i < 3; ++i) w[i] = 2.0 * oh * h[i] - wo[i];
}

/* mixture density q = (N_c p_c + N_g p_g + N_e p_e) / N_r at w (Sec. 3.4.1) */
static double mixture_pdf(const Env *E, const double n[3], const double wo[3], double rough, const double w[3],
                          int nc, int ng, int ne)
{
    double ndi = dot3(n, w), ndo = dot3(n, wo);
    double pc = ndi > 0.0 ? ndi / ORC_PI : 0.0;
    double pg = 0.0;
    double h[3] = {w[0] + wo[0], w[1] + wo[1], w[2] + wo[2]};
    double hl = sqrt(dot3(h, h));
    if (hl > 0.0) {
        h[0] /= hl; h[1] /= hl; h[2] /= hl;
        double ndh = dot3(n, h);
        if (ndh > 0.0 && dot3(wo, h) > 0.0) {
            double a = rough * rough, a2 = a * a;
            pg = smith_G1(ndo, a2) * ggx_D(ndh, a2) / (4.0 * ndo);
        }
    }
    double pe = ne > 0 ? env_pdf(E, w) : 0.0;
    return ((double)nc * pc + (double)ng * pg + (double)ne * pe) / (double)(nc + ng + ne);
}

/* ------------------------------------------------------------------------ */
/* Exported: MIS shading of G-buffer pixels (Eqs. montecarlo, mis)           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nc, ng, ne;
    uint64_t seed;
    uint32_t job;
    float tmin, tcut;
} MisOpts;

/* Sample j of pixel p: direction, weight f cos / q, incident radiance; and,
 * when traced, the ray's hit list (caller frees R->h). Returns 1 if traced. */
/* ------------------------------------------------------------------------ */
/* Split-sum relighting (Sec. 3.5.1, Eq. relight_splitsum)                   */
/* ------------------------------------------------------------------------ */

/* The prefiltered representation E of an environment (piecewise constant over
 * its texels; integrals are sums over texel centres weighted by each texel's
 * exact solid angle), on a coarse equirectangular grid of PF_H x PF_W texel
 * centres (same direction convention as the environment):
 *   E_d(n)    = sum L(l) max(0, n.l) dW / sum max(0, n.l) dW       (diffuse)
 *   E_s(R, r) = sum L(l) D(h) max(0, R.l) dW / sum D(h) max(0, R.l) dW,
 *               h = normalize(R + l), D GGX with alpha = r^2       (specular)
 * at roughness levels r = l / (PF_L - 1), l = 1 .. PF_L - 1; level 0 is the
 * environment itself.  The DFG table holds, for n.v = mu and roughness r at
 * LUT_N x LUT_N cell centres, the Schlick split of the specular lobe's
 * directional albedo (F = 1):
 *   A = int f_s/F (1 - (1 - v.h)^5) n.l dl,  B = int f_s/F (1 - v.h)^5 n.l dl
 * integrated over half vectors h distributed as D(h) n.h (midpoint rule on
 * LUT_Q x LUT_Q points of the inverse GGX distribution and the azimuth). */
#define PF_H 16
#define PF_W 32
#define PF_L 6
#define LUT_N 32
#define LUT_Q 256

static void texel_dir(int H, int W, int i, int j, double w[3])
{
    double th = ORC_PI * (i + 0.5) / H, ph = 2.0 * ORC_PI * (j + 0.5) / W;
    w[0] = sin(th) * cos(ph); w[1] = cos(th); w[2] = sin(th) * sin(ph);
}

static double texel_omega(int H, int W, int i)
{
    return 2.0 * ORC_PI / W * (cos(ORC_PI * i / H) - cos(ORC_PI * (i + 1) / H));
}

int orc_env_prefilter(int H, int W, const float *rgb, double *Ed, double *Es)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < PF_H * PF_W; ++t) {
        double nt[3];
        texel_dir(PF_H, PF_W, t / PF_W, t % PF_W, nt);
        double sd[3] = {0, 0, 0}, wd = 0.0, ss[PF_L][3], ws[PF_L];
        for (int l = 0; l < PF_L; ++l) { ss[l][0] = ss[l][1] = ss[l][2] = 0.0; ws[l] = 0.0; }
        for (int i = 0; i < H; ++i) {
            double om = texel_omega(H, W, i);
            for (int j = 0; j < W; ++j) {
                double lk[3];
                texel_dir(H, W, i, j, lk);
                double c = dot3(nt, lk);
                if (!(c > 0.0)) continue;
                const float *L = rgb + ((size_t)i * W + j) * 3;
                double w = c * om;
                for (int k = 0; k < 3; ++k) sd[k] += w * L[k];
                wd += w;
                double h[3] = {nt[0] + lk[0], nt[1] + lk[1], nt[2] + lk[2]};
                normalize3(h);
                double ndh = dot3(nt, h);
                for (int l = 1; l < PF_L; ++l) {
                    double r = (double)l / (PF_L - 1), a = r * r;
                    double wl = ggx_D(ndh, a * a) * w;
                    for (int k = 0; k < 3; ++k) ss[l][k] += wl * L[k];
                    ws[l] += wl;
                }
            }
        }
        for (int k = 0; k < 3; ++k) Ed[3 * t + k] = wd > 0.0 ? sd[k] / wd : 0.0;
        for (int l = 1; l < PF_L; ++l)
            for (int k = 0; k < 3; ++k)
                Es[((size_t)(l - 1) * PF_H * PF_W + t) * 3 + k] = ws[l] > 0.0 ? ss[l][k] / ws[l] : 0.0;
    }
    return 0;
}

int orc_dfg_lut(double *lut)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < LUT_N; ++i)
        for (int j = 0; j < LUT_N; ++j) {
            double mu = (i + 0.5) / LUT_N, r = (j + 0.5) / LUT_N, a = r * r, a2 = a * a;
            double v[3] = {sqrt(1.0 - mu * mu), 0.0, mu};
            double A = 0.0, B = 0.0;
            for (int s = 0; s < LUT_Q; ++s) {
                double xi = (s + 0.5) / LUT_Q;
                double c2 = (1.0 - xi) / (1.0 + (a2 - 1.0) * xi);
                double ct = sqrt(c2), st = sqrt(1.0 - c2 > 0.0 ? 1.0 - c2 : 0.0);
                for (int t = 0; t < LUT_Q; ++t) {
                    double ph = 2.0 * ORC_PI * (t + 0.5) / LUT_Q;
                    double h[3] = {st * cos(ph), st * sin(ph), ct};
                    double vh = dot3(v, h);
                    if (!(vh > 0.0)) continue;
                    double nl = 2.0 * vh * h[2] - v[2];
                    if (!(nl > 0.0)) continue;
                    double g = smith_G1(nl, a2) * smith_G1(mu, a2) * vh / (mu * ct);
                    double x = 1.0 - vh, fc = x * x * x * x * x;
                    A += g * (1.0 - fc);
                    B += g * fc;
                }
            }
            lut[2 * (i * LUT_N + j)] = A / (LUT_Q * LUT_Q);
            lut[2 * (i * LUT_N + j) + 1] = B / (LUT_Q * LUT_Q);
        }
    return 0;
}

/* Bilinear lookup of a PF_H x PF_W direction table (texel centres; wraps in
 * the azimuth, clamps in the polar angle). */
static void table_lookup(const double *T, const double w[3], double out[3])
{
    double y = w[1] < -1.0 ? -1.0 : (w[1] > 1.0 ? 1.0 : w[1]);
    double th = acos(y), ph = atan2(w[2], w[0]);
    if (ph < 0.0) ph += 2.0 * ORC_PI;
    double x = ph / (2.0 * ORC_PI) * PF_W - 0.5, v = th / ORC_PI * PF_H - 0.5;
    x = x > -1.0 ? (x < (double)PF_W ? x : (double)PF_W) : -1.0;
    double fx0 = floor(x);
    double fx = x - fx0;
    int j0 = (int)fx0;
    j0 = ((j0 % PF_W) + PF_W) % PF_W;
    int j1 = (j0 + 1) % PF_W;
    v = v > 0.0 ? (v < (double)(PF_H - 1) ? v : (double)(PF_H - 1)) : 0.0;
    int i0 = (int)floor(v);
    if (i0 > PF_H - 2) i0 = PF_H - 2;
    double fy = v - i0;
    for (int k = 0; k < 3; ++k) {
        double a = T[((size_t)i0 * PF_W + j0) * 3 + k], b = T[((size_t)i0 * PF_W + j1) * 3 + k];
        double c = T[((size_t)(i0 + 1) * PF_W + j0) * 3 + k], d = T[((size_t)(i0 + 1) * PF_W + j1) * 3 + k];
        out[k] = (1.0 - fy) * ((1.0 - fx) * a + fx * b) + fy * ((1.0 - fx) * c + fx * d);
    }
}

struct MeshRefS;
static void mesh_query(const struct MeshRefS *m, const double o[3], const double d[3], double tmin, double tmax,
                       AttrOut *q, double mg[2]);
typedef struct {
    Attrs at;
    const double *Ed, *Es, *lut;
    const struct MeshRefS *mesh;  /* the mesh backend answers the query, or NULL: the surfels */
} Relight;

/* SplitSum(a, r, m, n, E) of the surface a secondary ray met, seen along -w
 * (Eq. relight_splitsum: diffuse (1 - m) a E_d(n) plus specular
 * E_s(R, r) (F0 A + B), F0 = 0.04 (1 - m) + m a, R the mirror of -w). */
static void split_sum(const Env *E, const Relight *rl, const AttrOut *q, const double w[3], double out[3])
{
    double nr[3] = {q->n[0], q->n[1], q->n[2]};
    double nl = sqrt(dot3(nr, nr));
    double v[3] = {-w[0], -w[1], -w[2]};
    if (nl > 0.0) { nr[0] /= nl; nr[1] /= nl; nr[2] /= nl; }
    else { nr[0] = v[0]; nr[1] = v[1]; nr[2] = v[2]; }
    double ndv = dot3(nr, v);
    double R[3] = {2.0 * ndv * nr[0] - v[0], 2.0 * ndv * nr[1] - v[1], 2.0 * ndv * nr[2] - v[2]};
    double mu = ndv > 0.0 ? (ndv < 1.0 ? ndv : 1.0) : 0.0;
    double r = q->r > 0.0 ? (q->r < 1.0 ? q->r : 1.0) : 0.0;
    double Ld[3], Ls[3], L0[3], L1[3];
    table_lookup(rl->Ed, nr, Ld);
    double xl = r * (PF_L - 1);
    int l0 = (int)floor(xl);
    if (l0 > PF_L - 2) l0 = PF_L - 2;
    double tl = xl - l0;
    if (l0 == 0) env_radiance(E, R, L0);
    else table_lookup(rl->Es + (size_t)(l0 - 1) * PF_H * PF_W * 3, R, L0);
    table_lookup(rl->Es + (size_t)l0 * PF_H * PF_W * 3, R, L1);
    for (int k = 0; k < 3; ++k) Ls[k] = (1.0 - tl) * L0[k] + tl * L1[k];
    /* DFG: bilinear over cell centres in (mu, r), clamped */
    double xi = mu * LUT_N - 0.5, yj = r * LUT_N - 0.5;
    if (xi < 0.0) xi = 0.0;
    if (xi > LUT_N - 1) xi = LUT_N - 1;
    if (yj < 0.0) yj = 0.0;
    if (yj > LUT_N - 1) yj = LUT_N - 1;
    int i0 = (int)floor(xi), j0 = (int)floor(yj);
    if (i0 > LUT_N - 2) i0 = LUT_N - 2;
    if (j0 > LUT_N - 2) j0 = LUT_N - 2;
    double fi = xi - i0, fj = yj - j0, AB[2];
    for (int k = 0; k < 2; ++k) {
        double a = rl->lut[2 * (i0 * LUT_N + j0) + k], b = rl->lut[2 * (i0 * LUT_N + j0 + 1) + k];
        double c = rl->lut[2 * ((i0 + 1) * LUT_N + j0) + k], d = rl->lut[2 * ((i0 + 1) * LUT_N + j0 + 1) + k];
        AB[k] = (1.0 - fi) * ((1.0 - fj) * a + fj * b) + fi * ((1.0 - fj) * c + fj * d);
    }
    for (int k = 0; k < 3; ++k) {
        double F0 = 0.04 * (1.0 - q->m) + q->m * q->a[k];
        out[k] = (1.0 - q->m) * q->a[k] * Ld[k] + Ls[k] * (F0 * AB[0] + AB[1]);
    }
}

/* One MIS sample of a pixel; with `rl`, the incident radiance is the
 * relighting one (Eq. relight_splitsum) instead of c_rt + T L_env. */
static int mis_sample(const Scene *S, const Env *E, const MisOpts *op, const Relight *rl, uint32_t pix, int j,
                      const double x[3], const double n[3], const double wo[3], const double alb[3],
                      double rough, double metal,
                      double w_out[3], double wt[3], double Li[3], double *q_out, RayResult *R, float df_out[3])
{
    double u1, u2;
    uniforms(op->seed, pix, (uint32_t)j, op->job, &u1, &u2);
    double w[3];
    if (j < op->nc) sample_cos(n, u1, u2, w);
    else if (j < op->nc + op->ng) sample_ggx(n, wo, rough, u1, u2, w);
    else sample_env(E, u1, u2, w);
    for (int i = 0; i < 3; ++i) w_out[i] = w[i];
    double ndi = dot3(n, w);
    double texel = INFINITY;
    {
        double y = w[1] < -1.0 ? -1.0 : (w[1] > 1.0 ? 1.0 : w[1]);
        double th = acos(y), ph = atan2(w[2], w[0]);
        if (ph < 0.0) ph += 2.0 * ORC_PI;
        double ft = th / ORC_PI * E->H, fp = ph / (2.0 * ORC_PI) * E->W;
        double dt = fabs(ft - floor(ft + 0.5)) * ORC_PI / E->H;
        double dp = fabs(fp - floor(fp + 0.5)) * 2.0 * ORC_PI / E->W * sin(th);
        texel = dt < dp ? dt : dp;
    }
    wt[0] = wt[1] = wt[2] = 0.0; Li[0] = Li[1] = Li[2] = 0.0; *q_out = 0.0;
    if (!(ndi > 0.0)) return 0;
    double q = mixture_pdf(E, n, wo, rough, w, op->nc, op->ng, op->ne);
    *q_out = q;
    float of[3] = {(float)x[0], (float)x[1], (float)x[2]};
    float df[3] = {(float)w[0], (float)w[1], (float)w[2]};
    for (int i = 0; i < 3; ++i) df_out[i] = df[i];
    trace_ray(S, of, df, op->tmin, INFINITY, op->tcut, R);
    R->mg.texel = (float)texel;
    double Le[3];
    env_radiance(E, w, Le);
    if (rl) {
        AttrOut a;
        if (rl->mesh) {
            double od[3] = {of[0], of[1], of[2]}, dd[3] = {df[0], df[1], df[2]}, mg[2];
            mesh_query(rl->mesh, od, dd, op->tmin, INFINITY, &a, mg);
            R->mg.r2 = (float)mg[0];
            R->mg.den = (float)mg[1];
        } else {
            attr_of_ray(S, &rl->at, of, df, R, &a);
        }
        double ss[3] = {0, 0, 0};
        if (a.V < 1.0) split_sum(E, rl, &a, w, ss);
        for (int c = 0; c < 3; ++c) Li[c] = a.V * Le[c] + (1.0 - a.V) * ss[c];
    } else {
        for (int c = 0; c < 3; ++c) Li[c] = R->C[c] + R->T * Le[c];
    }
    if (q > 0.0) {
        double f[3];
        brdf(n, wo, w, alb, rough, metal, f);
        for (int c = 0; c < 3; ++c) wt[c] = f[c] * ndi / q;
    }
    return 1;
}

/* The normal and the view direction are directions (Sec. 3.3, "Shading
 * state": N sets the hemisphere and the cosine); they are normalised here, as
 * single-precision storage leaves |n| = 1 +- 1e-7, which sharp GGX lobes
 * (alpha^2 ~ 1e-5) would otherwise feel through 1 - (n.h)^2. */
static void load_pixel(const float *gx, const float *gn, const float *gwo, const float *galb, int64_t p,
                       double x[3], double n[3], double wo[3], double alb[3])
{
    for (int i = 0; i < 3; ++i) {
        x[i] = gx[3 * p + i]; n[i] = gn[3 * p + i]; wo[i] = gwo[3 * p + i]; alb[i] = galb[3 * p + i];
    }
    if (dot3(n, n) > 0.0) normalize3(n);
    if (dot3(wo, wo) > 0.0) normalize3(wo);
}

/*
 * Shade the pixels listed in pix [np] (indices into the G-buffer, which also
 * seed the random counters).  out [np,3] = c_pbr.  Optional per-sample dump
 * (spp = nc+ng+ne): dir [np,spp,3], q [np,spp], wt [np,spp,3] = f cos/q,
 * Li [np,spp,3], traced [np,spp], margins [np,spp,5] (as in orc_trace, the
 * texel margin being the angle from the sampled direction to the nearest
 * environment texel edge).
 */
static void shade_pixels(const Scene *S, const Env *E, const MisOpts *op, const Relight *rl,
                         const float *gx, const float *gn, const float *gwo, const float *galb, const float *grough,
                         const float *gmetal, const uint8_t *gvalid, int64_t np, const int64_t *pix, double *out,
                         float *s_dir, double *s_q, double *s_wt, double *s_Li, uint8_t *s_traced, float *s_margin)
{
    int spp = op->nc + op->ng + op->ne;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < np; ++k) {
        int64_t p = pix[k];
        double acc[3] = {0, 0, 0};
        double x[3], nn[3], wo[3], alb[3];
        load_pixel(gx, gn, gwo, galb, p, x, nn, wo, alb);
        int ok = gvalid[p] && dot3(nn, wo) > 0.0;
        for (int j = 0; j < spp; ++j) {
            size_t si = (size_t)k * spp + j;
            double w[3] = {0, 0, 0}, wt[3] = {0, 0, 0}, Li[3] = {0, 0, 0}, q = 0.0;
            float df[3] = {0, 0, 0};
            RayResult R;
            R.h = NULL;
            R.mg.r2 = R.mg.den = R.mg.tau = R.mg.texel = INFINITY;
            R.tstop = INFINITY;
            int traced = 0;
            if (ok) {
                traced = mis_sample(S, E, op, rl, (uint32_t)p, j, x, nn, wo, alb, grough[p], gmetal[p], w, wt, Li, &q,
                                    &R, df);
                for (int c = 0; c < 3; ++c) acc[c] += wt[c] * Li[c];
            }
            if (s_dir) for (int c = 0; c < 3; ++c) s_dir[3 * si + c] = (float)w[c];
            if (s_q) s_q[si] = q;
            if (s_wt) for (int c = 0; c < 3; ++c) s_wt[3 * si + c] = wt[c];
            if (s_Li) for (int c = 0; c < 3; ++c) s_Li[3 * si + c] = Li[c];
            if (s_traced) s_traced[si] = (uint8_t)traced;
            if (s_margin) {
                s_margin[5 * si + 0] = R.mg.r2; s_margin[5 * si + 1] = R.mg.den;
                s_margin[5 * si + 2] = R.mg.tau; s_margin[5 * si + 3] = R.tstop; s_margin[5 * si + 4] = R.mg.texel;
            }
            free(R.h);
        }
        for (int c = 0; c < 3; ++c) out[3 * k + c] = acc[c] / (double)spp;
    }
}

int orc_render_mis(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                   const float *rgb, float alpha_min,
                   const float *gx, const float *gn, const float *gwo, const float *galb, const float *grough,
                   const float *gmetal, const uint8_t *gvalid,
                   int eH, int eW, const float *env_rgb, const float *marg, const float *cond,
                   int nc, int ng, int ne, uint64_t seed, uint32_t job, float tmin, float tcut,
                   int64_t np, const int64_t *pix, double *out,
                   float *s_dir, double *s_q, double *s_wt, double *s_Li, uint8_t *s_traced, float *s_margin)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, rgb, alpha_min)) return -1;
    Env E = {eH, eW, env_rgb, marg, cond};
    MisOpts op = {nc, ng, ne, seed, job, tmin, tcut};
    shade_pixels(&S, &E, &op, NULL, gx, gn, gwo, galb, grough, gmetal, gvalid, np, pix, out, s_dir, s_q, s_wt, s_Li,
                 s_traced, s_margin);
    scene_free(&S);
    return 0;
}

/* Relighting (Sec. 3.5.1): the same MIS estimator, with the incident
 * radiance of Eq. relight_splitsum -- V L_env(w) + (1 - V) SplitSum of the
 * attributes the ray's query returns -- from the environment's prefiltered
 * tables Ed, Es (orc_env_prefilter) and the DFG table lut (orc_dfg_lut).
 * Arguments as orc_render_mis, plus the per-surfel attributes. */
int orc_render_relight(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                       float alpha_min, const float *s_albedo, const float *s_rough, const float *s_metal,
                       const float *gx, const float *gn, const float *gwo, const float *galb, const float *grough,
                       const float *gmetal, const uint8_t *gvalid,
                       int eH, int eW, const float *env_rgb, const float *marg, const float *cond,
                       const double *Ed, const double *Es, const double *lut,
                       int nc, int ng, int ne, uint64_t seed, uint32_t job, float tmin, float tcut,
                       int64_t np, const int64_t *pix, double *out,
                       float *s_dir, double *s_q, double *s_wt, double *s_Li, uint8_t *s_traced, float *s_margin)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, NULL, alpha_min)) return -1;
    Env E = {eH, eW, env_rgb, marg, cond};
    MisOpts op = {nc, ng, ne, seed, job, tmin, tcut};
    Relight rl = {{s_albedo, s_rough, s_metal}, Ed, Es, lut, NULL};
    shade_pixels(&S, &E, &op, &rl, gx, gn, gwo, galb, grough, gmetal, gvalid, np, pix, out, s_dir, s_q, s_wt, s_Li,
                 s_traced, s_margin);
    scene_free(&S);
    return 0;
}

/* Gradient of sum_k grad[k] . c_pbr(pix[k]) w.r.t. the surfels; g13 [n,13]
 * overwritten.  The samples are regenerated from the same counters. */
int orc_render_mis_backward(int64_t n, const float *means, const float *scales, const float *quats,
                            const float *opacity, const float *rgb, float alpha_min,
                            const float *gx, const float *gn, const float *gwo, const float *galb,
                            const float *grough, const float *gmetal, const uint8_t *gvalid,
                            int eH, int eW, const float *env_rgb, const float *marg, const float *cond,
                            int nc, int ng, int ne, uint64_t seed, uint32_t job, float tmin, float tcut,
                            int64_t np, const int64_t *pix, const double *grad, double *g13, double *g13_abs,
                            double *g_shade, double *g_shade_abs)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, rgb, alpha_min)) return -1;
    memset(g13, 0, sizeof(double) * 13 * (size_t)n);
    if (g13_abs) memset(g13_abs, 0, sizeof(double) * 13 * (size_t)n);
    if (g_shade) memset(g_shade, 0, sizeof(double) * 14 * (size_t)np);
    if (!(g_shade && g13_abs)) g_shade_abs = NULL;
    if (g_shade_abs) memset(g_shade_abs, 0, sizeof(double) * 14 * (size_t)np);
    Env E = {eH, eW, env_rgb, marg, cond};
    MisOpts op = {nc, ng, ne, seed, job, tmin, tcut};
    int spp = nc + ng + ne;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < np; ++k) {
        int64_t p = pix[k];
        double x[3], nn[3], wo[3], alb[3];
        load_pixel(gx, gn, gwo, galb, p, x, nn, wo, alb);
        if (!(gvalid[p] && dot3(nn, wo) > 0.0)) continue;
        /* d/d(shading state) with each sample's direction and pdf held fixed
         * (reading 36): x (through the secondary rays' origin), the unit
         * normal and view direction, albedo, roughness, metallic */
        double Gx[3] = {0, 0, 0}, Gn[3] = {0, 0, 0}, Go[3] = {0, 0, 0}, Ga[3] = {0, 0, 0}, Gr = 0.0, Gm = 0.0;
        /* error scales: the terms' magnitudes (x: with the chain of magnitudes
         * of the surfel gradients' error scale) */
        double Ax[3] = {0, 0, 0}, An[3] = {0, 0, 0}, Ao[3] = {0, 0, 0}, Aa[3] = {0, 0, 0}, Ar = 0.0, Am = 0.0;
        for (int j = 0; j < spp; ++j) {
            double w[3], wt[3], Li[3], q;
            float df[3];
            RayResult R;
            R.h = NULL;
            if (mis_sample(&S, &E, &op, NULL, (uint32_t)p, j, x, nn, wo, alb, grough[p], gmetal[p], w, wt, Li, &q, &R, df)) {
                /* c_pbr += wt * (C + T L_env) / spp */
                double gC[3], Le[3];
                env_radiance(&E, w, Le);
                double gT = 0.0;
                for (int c = 0; c < 3; ++c) {
                    gC[c] = grad[3 * k + c] * wt[c] / (double)spp;
                    gT += gC[c] * Le[c];
                }
                float of[3] = {(float)x[0], (float)x[1], (float)x[2]};
                double dmu[3] = {0, 0, 0};
                backward_ray(&S, of, df, &R, gC, gT, g13, g13_abs, g_shade ? dmu : NULL, g_shade_abs ? Ax : NULL);
                if (g_shade && q > 0.0) {
                    /* the secondary ray leaves from x: every hit's geometry
                     * depends on (mu - x), so d/dx = -d/dmu summed over hits */
                    for (int c = 0; c < 3; ++c) Gx[c] -= dmu[c];
                    double f[3], dn[3][3], dwo[3][3], da[3], dr[3], dm[3];
                    brdf_partials(nn, wo, w, alb, grough[p], gmetal[p], f, dn, dwo, da, dr, dm);
                    double ndi = dot3(nn, w);
                    for (int c = 0; c < 3; ++c) {
                        /* g_c = f_c (n.w) / q; its weight in the loss */
                        double u = grad[3 * k + c] * Li[c] / (double)spp / q;
                        for (int i = 0; i < 3; ++i) {
                            Gn[i] += u * (dn[c][i] * ndi + f[c] * w[i]);
                            Go[i] += u * dwo[c][i] * ndi;
                        }
                        Ga[c] += u * da[c] * ndi;
                        Gr += u * dr[c] * ndi;
                        Gm += u * dm[c] * ndi;
                        if (g_shade_abs) {
                            double ua = fabs(u) * ndi;
                            for (int i = 0; i < 3; ++i) {
                                An[i] += ua * fabs(dn[c][i]) + fabs(u * f[c] * w[i]);
                                Ao[i] += ua * fabs(dwo[c][i]);
                            }
                            Aa[c] += ua * fabs(da[c]);
                            Ar += ua * fabs(dr[c]);
                            Am += ua * fabs(dm[c]);
                        }
                    }
                }
            }
            free(R.h);
        }
        if (g_shade) {
            /* through the normalisations n / |n| and wo / |wo| of the stored values */
            double nr[3] = {gn[3 * p], gn[3 * p + 1], gn[3 * p + 2]}, orw[3] = {gwo[3 * p], gwo[3 * p + 1], gwo[3 * p + 2]};
            double ln = sqrt(dot3(nr, nr)), lo = sqrt(dot3(orw, orw));
            double pn = dot3(nn, Gn), po = dot3(wo, Go);
            double *o = g_shade + 14 * k;
            for (int i = 0; i < 3; ++i) {
                o[i] = Gx[i];
                o[3 + i] = (Gn[i] - nn[i] * pn) / ln;
                o[6 + i] = (Go[i] - wo[i] * po) / lo;
                o[9 + i] = Ga[i];
            }
            o[12] = Gr;
            o[13] = Gm;
            if (g_shade_abs) {
                double *oa = g_shade_abs + 14 * k;
                double sn = fabs(nn[0]) * An[0] + fabs(nn[1]) * An[1] + fabs(nn[2]) * An[2];
                double so = fabs(wo[0]) * Ao[0] + fabs(wo[1]) * Ao[1] + fabs(wo[2]) * Ao[2];
                for (int i = 0; i < 3; ++i) {
                    oa[i] = Ax[i];
                    oa[3 + i] = (An[i] + fabs(nn[i]) * sn) / ln;
                    oa[6 + i] = (Ao[i] + fabs(wo[i]) * so) / lo;
                    oa[9 + i] = Aa[i];
                }
                oa[12] = Ar;
                oa[13] = Am;
            }
        }
    }
    scene_free(&S);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exported pieces of the shading, for pinning them one by one               */
/* ------------------------------------------------------------------------ */

/* technique 0 = cosine, 1 = GGX (visible normals), 2 = environment;
 * m directions from the uniforms u [m,2] at one shading point. */
void orc_sample_dirs(int tech, const double *n, const double *wo, double rough, int eH, int eW,
                     const float *env_rgb, const float *marg, const float *cond, int64_t m, const double *u,
                     double *w)
{
    Env E = {eH, eW, env_rgb, marg, cond};
    for (int64_t k = 0; k < m; ++k) {
        if (tech == 0) sample_cos(n, u[2 * k], u[2 * k + 1], w + 3 * k);
        else if (tech == 1) sample_ggx(n, wo, rough, u[2 * k], u[2 * k + 1], w + 3 * k);
        else sample_env(&E, u[2 * k], u[2 * k + 1], w + 3 * k);
    }
}

/* pdfs [m,3] = (p_c, p_g, p_e) at directions w [m,3], and the mixture
 * q [m] for the allocation (nc, ng, ne). */
void orc_pdfs(const double *n, const double *wo, double rough, int eH, int eW, const float *env_rgb,
              const float *marg, const float *cond, int nc, int ng, int ne, int64_t m, const double *w,
              double *p3, double *q)
{
    Env E = {eH, eW, env_rgb, marg, cond};
    for (int64_t k = 0; k < m; ++k) {
        const double *x = w + 3 * k;
        if (p3) {
            p3[3 * k + 0] = mixture_pdf(&E, n, wo, rough, x, 1, 0, 0);
            p3[3 * k + 1] = mixture_pdf(&E, n, wo, rough, x, 0, 1, 0);
            p3[3 * k + 2] = eH > 0 ? mixture_pdf(&E, n, wo, rough, x, 0, 0, 1) : 0.0;
        }
        if (q) q[k] = mixture_pdf(&E, n, wo, rough, x, nc, ng, ne);
    }
}

/* f(wo, wi) [m,3] for directions wi [m,3] (zero below either horizon) */
void orc_brdf(const double *n, const double *wo, const double *alb, double rough, double metal, int64_t m,
              const double *wi, double *f)
{
    for (int64_t k = 0; k < m; ++k) {
        const double *x = wi + 3 * k;
        if (dot3(n, x) > 0.0 && dot3(n, wo) > 0.0) brdf(n, wo, x, alb, rough, metal, f + 3 * k);
        else f[3 * k] = f[3 * k + 1] = f[3 * k + 2] = 0.0;
    }
}

/* nearest-texel radiance [m,3] at directions w [m,3] */
void orc_env_lookup(int eH, int eW, const float *env_rgb, int64_t m, const double *w, double *L)
{
    Env E = {eH, eW, env_rgb, NULL, NULL};
    for (int64_t k = 0; k < m; ++k) env_radiance(&E, w + 3 * k, L + 3 * k);
}

/* Per ray: the depth where compositing ended (the last composited hit's
 * depth if the ray stopped at T < T_cut, else t_max) and the number of
 * composited hits.  Used by the work counter. */
int orc_trace_extent(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                     float alpha_min, int64_t nr, const float *orig, const float *dirs, float tmin, float tmax,
                     float t_cut, float *t_term, int64_t *nhit)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, NULL, alpha_min)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        RayResult R;
        trace_ray(&S, orig + 3 * r, dirs + 3 * r, tmin, tmax, t_cut, &R);
        float T32 = 1.0f;
        for (int64_t k = 0; k < R.K; ++k) T32 = T32 * (1.0f - S.s32[R.h[k].id].op * expf(-0.5f * R.h[k].r2));
        int stopped = R.K > 0 && T32 < t_cut;
        t_term[r] = stopped ? bitsf((uint32_t)(R.h[R.K - 1].key >> 32)) : tmax;
        nhit[r] = R.K;
        free(R.h);
    }
    scene_free(&S);
    return 0;
}

/* Mesh backend of the attribute query (Sec. 3.5.2, "Mesh-based ray
 * tracing"): the closest triangle hit by the ray with t_min < t <= t_max
 * (two-sided, Moller-Trumbore, in double; equal t: the lower triangle id).
 * A miss returns V = 1 and zero attributes; a hit V = 0 and the per-vertex
 * albedo, roughness, metallic and normal interpolated with the barycentric
 * weights (1 - u - v, u, v) of the hit, the normal turned toward the ray
 * origin (not renormalized).  Margins: [0] the hit's barycentric margin
 * min(u, v, 1 - u - v), [1] the relative gap in t to the next triangle met
 * (inf if none). */
typedef struct MeshRefS {
    int64_t nf;
    const float *verts;
    const int32_t *tris;
    const float *albedo, *rough, *metal, *normal;
} MeshRef;

static void mesh_query(const struct MeshRefS *m, const double o[3], const double d[3], double tmin, double tmax,
                       AttrOut *q, double mg[2])
{
    double best = INFINITY, second = INFINITY, bu = 0.0, bv = 0.0;
    int64_t bf = -1;
    for (int64_t f = 0; f < m->nf; ++f) {
        const float *a = m->verts + 3 * (int64_t)m->tris[3 * f], *b = m->verts + 3 * (int64_t)m->tris[3 * f + 1],
                    *c = m->verts + 3 * (int64_t)m->tris[3 * f + 2];
        double v0[3] = {a[0], a[1], a[2]};
        double e1[3] = {b[0] - v0[0], b[1] - v0[1], b[2] - v0[2]}, e2[3] = {c[0] - v0[0], c[1] - v0[1], c[2] - v0[2]};
        double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
        double det = dot3(e1, p);
        if (fabs(det) < 1e-12) continue;
        double inv = 1.0 / det;
        double sv[3] = {o[0] - v0[0], o[1] - v0[1], o[2] - v0[2]};
        double u = dot3(sv, p) * inv;
        if (u < 0.0 || u > 1.0) continue;
        double qq[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2], sv[0] * e1[1] - sv[1] * e1[0]};
        double v = dot3(d, qq) * inv;
        if (v < 0.0 || u + v > 1.0) continue;
        double t = dot3(e2, qq) * inv;
        if (!(t > tmin && t <= tmax)) continue;
        if (t < best) { second = best; best = t; bf = f; bu = u; bv = v; }
        else if (t < second) second = t;
    }
    double A[3] = {0, 0, 0}, Rg = 0.0, M = 0.0, N[3] = {0, 0, 0};
    if (bf >= 0) {
        double w[3] = {1.0 - bu - bv, bu, bv};
        for (int k = 0; k < 3; ++k) {
            int64_t vi = m->tris[3 * bf + k];
            for (int c = 0; c < 3; ++c) {
                A[c] += w[k] * (double)m->albedo[3 * vi + c];
                N[c] += w[k] * (double)m->normal[3 * vi + c];
            }
            Rg += w[k] * (double)m->rough[vi];
            M += w[k] * (double)m->metal[vi];
        }
        if (dot3(N, d) > 0.0) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; }
    }
    q->V = bf >= 0 ? 0.0 : 1.0;
    for (int c = 0; c < 3; ++c) { q->a[c] = A[c]; q->n[c] = N[c]; }
    q->r = Rg;
    q->m = M;
    if (mg) {
        double bm = 1.0 - bu - bv;
        if (bu < bm) bm = bu;
        if (bv < bm) bm = bv;
        mg[0] = bf >= 0 ? bm : INFINITY;
        mg[1] = bf >= 0 && second < INFINITY ? (second - best) / best : INFINITY;
    }
}

int orc_mesh_trace_attr(int64_t nv, const float *verts, int64_t nf, const int32_t *tris, const float *albedo,
                        const float *rough, const float *metal, const float *vnormal, int64_t nr, const float *orig,
                        const float *dirs, float tmin_s, float tmax_s, double *outV, double *outA, double *outR,
                        double *outM, double *outN, double *margins)
{
    (void)nv;
    MeshRef m = {nf, verts, tris, albedo, rough, metal, vnormal};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        double o[3] = {orig[3 * r], orig[3 * r + 1], orig[3 * r + 2]};
        double d[3] = {dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2]};
        AttrOut q;
        double mg[2];
        mesh_query(&m, o, d, tmin_s, tmax_s, &q, mg);
        outV[r] = q.V;
        for (int c = 0; c < 3; ++c) { outA[3 * r + c] = q.a[c]; outN[3 * r + c] = q.n[c]; }
        outR[r] = q.r;
        outM[r] = q.m;
        if (margins) { margins[2 * r] = mg[0]; margins[2 * r + 1] = mg[1]; }
    }
    return 0;
}

/* Relighting with the mesh backend answering the attribute query (Sec.
 * 3.5.2 leaves Eq. relight_splitsum unchanged): as orc_render_relight, the
 * secondary rays queried against the triangle mesh instead of the surfels.
 * Sample margins [np,spp,5] carry the mesh query's barycentric margin and
 * depth gap in [0] and [1], the texel margin in [4]. */
int orc_render_relight_mesh(int64_t nv, const float *verts, int64_t nf, const int32_t *tris, const float *v_albedo,
                            const float *v_rough, const float *v_metal, const float *v_normal,
                            const float *gx, const float *gn, const float *gwo, const float *galb, const float *grough,
                            const float *gmetal, const uint8_t *gvalid,
                            int eH, int eW, const float *env_rgb, const float *marg, const float *cond,
                            const double *Ed, const double *Es, const double *lut,
                            int nc, int ng, int ne, uint64_t seed, uint32_t job, float tmin,
                            int64_t np, const int64_t *pix, double *out,
                            float *s_dir, double *s_q, double *s_wt, double *s_Li, uint8_t *s_traced, float *s_margin)
{
    (void)nv;
    Scene S = {0, NULL, NULL};
    Env E = {eH, eW, env_rgb, marg, cond};
    MisOpts op = {nc, ng, ne, seed, job, tmin, 1e-3f};
    MeshRef m = {nf, verts, tris, v_albedo, v_rough, v_metal, v_normal};
    Relight rl = {{NULL, NULL, NULL}, Ed, Es, lut, &m};
    shade_pixels(&S, &E, &op, &rl, gx, gn, gwo, galb, grough, gmetal, gvalid, np, pix, out, s_dir, s_q, s_wt, s_Li,
                 s_traced, s_margin);
    return 0;
}

/* SplitSum(a, r, m, n, E) (Eq. relight_splitsum) of m query results with
 * caller-supplied prefiltered tables (Ed [PF_H,PF_W,3], Es [PF_L-1,PF_H,PF_W,3],
 * lut [LUT_N,LUT_N,2]) and environment (level 0 of the specular lookup):
 * the same function the relit estimator calls, exposed so that its table
 * lookups can be checked against tables of known content. */
void orc_split_sum(int eH, int eW, const float *env_rgb, const double *Ed, const double *Es, const double *lut,
                   int64_t m, const double *albedo, const double *rough, const double *metal, const double *nsum,
                   const double *w, double *out)
{
    Env E = {eH, eW, env_rgb, NULL, NULL};
    Relight rl = {{NULL, NULL, NULL}, Ed, Es, lut, NULL};
    for (int64_t k = 0; k < m; ++k) {
        AttrOut q;
        q.V = 0.0;
        for (int c = 0; c < 3; ++c) { q.a[c] = albedo[3 * k + c]; q.n[c] = nsum[3 * k + c]; }
        q.r = rough[k];
        q.m = metal[k];
        split_sum(&E, &rl, &q, w + 3 * k, out + 3 * k);
    }
}

/* Trace with an environment map instead of a constant sky (Sec. 3.3 Eq.
 * lighting_decompose): L = c_rt + T_fin L_env(d), the environment looked up
 * at the nearest texel of the ray direction (the render's lookup).  Rays as
 * in orc_trace with scalar t_min/t_max; outL [nr,3]. */
int orc_trace_env(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                  const float *rgb, float alpha_min, int64_t nr, const float *orig, const float *dirs, float tmin,
                  float tmax, float t_cut, int eH, int eW, const float *env_rgb, double *outL)
{
    Scene S;
    if (scene_init(&S, n, means, scales, quats, opacity, rgb, alpha_min)) return -1;
    Env E = {eH, eW, env_rgb, NULL, NULL};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        RayResult R;
        trace_ray(&S, orig + 3 * r, dirs + 3 * r, tmin, tmax, t_cut, &R);
        double w[3] = {dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2]}, Le[3];
        env_radiance(&E, w, Le);
        for (int c = 0; c < 3; ++c) outL[3 * r + c] = R.C[c] + R.T * Le[c];
        free(R.h);
    }
    scene_free(&S);
    return 0;
}
