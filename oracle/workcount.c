/*
 * workcount.c -- the algorithmic work of each ray on a reference LBVH.
 *
 * MEASUREMENT INFRASTRUCTURE (test/benchmark side only).  Gives, per ray,
 *   N_cand: surfels whose padded bounding box the segment [t_min, t_term]
 *           pierces, where t_term is where compositing ended;
 *   N_node: internal nodes of a reference LBVH whose box that segment pierces;
 *   N_hit:  composited hits.
 * These counts do not depend on how the GPU traverses, so they define the
 * bytes a ray must move at least once (node and surfel records), against
 * which the measured time is priced.
 *
 * The reference LBVH: 30-bit Morton codes of box centres in the scene bounds,
 * sorted by (code, index), hierarchy by Karras (HPG 2012) with the index
 * breaking ties between equal codes, one surfel per leaf, boxes as unions.
 * A surfel's box bounds its ellipse of support rho^2 <= r2max (the radius of
 * the paper's adaptive bounding proxy, Eq. icosahedron_transform) plus `pad`.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int orc_trace_extent(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                     float alpha_min, int64_t nr, const float *orig, const float *dirs, float tmin, float tmax,
                     float t_cut, float *t_term, int64_t *nhit);

typedef struct { double lo[3], hi[3]; } Box;

static void surfel_box(const float *mu, const float *sc, const float *q, float op, float alpha_min, double pad, Box *b)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double l = sqrt(w * w + x * x + y * y + z * z);
    w /= l; x /= l; y /= l; z /= l;
    double tu[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
    double tv[3] = {2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x)};
    double r2 = 9.0;
    if (alpha_min > 0.0f) { double bnd = 2.0 * log((double)op / (double)alpha_min); if (bnd < r2) r2 = bnd; }
    double r = r2 > 0.0 ? sqrt(r2) : 0.0;
    for (int i = 0; i < 3; ++i) {
        double a = sc[0] * tu[i], c = sc[1] * tv[i];
        double e = r * sqrt(a * a + c * c) + pad;
        b->lo[i] = mu[i] - e; b->hi[i] = mu[i] + e;
    }
}

static uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

static const uint32_t *g_codes;
static int cmp_idx(const void *a, const void *b)
{
    uint32_t i = *(const uint32_t *)a, j = *(const uint32_t *)b;
    if (g_codes[i] != g_codes[j]) return g_codes[i] < g_codes[j] ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

static int clz32(uint32_t v) { return v ? __builtin_clz(v) : 32; }

/* length of the common prefix of sorted keys i and j (code, then position) */
static int delta(const uint32_t *sc, int64_t n, int64_t i, int64_t j)
{
    if (j < 0 || j >= n) return -1;
    if (sc[i] != sc[j]) return clz32(sc[i] ^ sc[j]);
    return 32 + clz32((uint32_t)i ^ (uint32_t)j);
}

/* children of internal node i: >= 0 internal index, < 0 leaf -(pos+1) */
static void karras_node(const uint32_t *sc, int64_t n, int64_t i, int64_t *left, int64_t *right)
{
    int d = delta(sc, n, i, i + 1) - delta(sc, n, i, i - 1) > 0 ? 1 : -1;
    int dmin = delta(sc, n, i, i - d);
    int64_t lmax = 2;
    while (delta(sc, n, i, i + lmax * d) > dmin) lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (delta(sc, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = delta(sc, n, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) / 2;
        if (delta(sc, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t gamma = i + s * d + (d < 0 ? d : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    *left = (lo == gamma) ? -(gamma + 1) : gamma;
    *right = (hi == gamma + 1) ? -(gamma + 2) : gamma + 1;
}

static int seg_box(const Box *b, const double o[3], const double d[3], double t0, double t1)
{
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < b->lo[a] || o[a] > b->hi[a]) return 0;
            continue;
        }
        double ta = (b->lo[a] - o[a]) / d[a], tb = (b->hi[a] - o[a]) / d[a];
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

int orc_count_work(int64_t n, const float *means, const float *scales, const float *quats, const float *opacity,
                   const float *rgb, float alpha_min, float pad, int64_t nr, const float *orig, const float *dirs,
                   float tmin, float tmax, float t_cut, int64_t *n_cand, int64_t *n_node, int64_t *n_hit)
{
    (void)rgb;
    float *t_term = (float *)malloc(sizeof(float) * (size_t)(nr > 0 ? nr : 1));
    orc_trace_extent(n, means, scales, quats, opacity, alpha_min, nr, orig, dirs, tmin, tmax, t_cut, t_term, n_hit);
    Box *leaf = (Box *)malloc(sizeof(Box) * (size_t)n);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i) {
        surfel_box(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], alpha_min, pad, &leaf[i]);
        for (int a = 0; a < 3; ++a) {
            double c = 0.5 * (leaf[i].lo[a] + leaf[i].hi[a]);
            if (c < lo[a]) lo[a] = c;
            if (c > hi[a]) hi[a] = c;
        }
    }
    uint32_t *codes = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            double ext = hi[a] - lo[a];
            double c = 0.5 * (leaf[i].lo[a] + leaf[i].hi[a]);
            double f = ext > 0.0 ? (c - lo[a]) / ext : 0.0;
            double v = floor(f * 1024.0);
            q[a] = (uint32_t)(v < 0 ? 0 : (v > 1023 ? 1023 : v));
        }
        codes[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
        order[i] = (uint32_t)i;
    }
    g_codes = codes;
    qsort(order, (size_t)n, sizeof(uint32_t), cmp_idx);
    uint32_t *sc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) sc[i] = codes[order[i]];
    int64_t ni = n > 1 ? n - 1 : 0;
    int64_t *lc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ni + 1));
    int64_t *rc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ni + 1));
    Box *nb = (Box *)malloc(sizeof(Box) * (size_t)(ni + 1));
    for (int64_t i = 0; i < ni; ++i) karras_node(sc, n, i, &lc[i], &rc[i]);
    /* boxes bottom-up: post-order walk from the root */
    if (ni > 0) {
        int64_t *st = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n + 2));
        uint8_t *seen = (uint8_t *)calloc((size_t)ni, 1);
        int64_t sp = 0;
        st[sp++] = 0;
        while (sp) {
            int64_t v = st[sp - 1];
            if (!seen[v]) {
                seen[v] = 1;
                if (lc[v] >= 0) st[sp++] = lc[v];
                if (rc[v] >= 0) st[sp++] = rc[v];
                continue;
            }
            --sp;
            Box b;
            for (int a = 0; a < 3; ++a) { b.lo[a] = INFINITY; b.hi[a] = -INFINITY; }
            int64_t ch[2] = {lc[v], rc[v]};
            for (int k = 0; k < 2; ++k) {
                const Box *c = ch[k] >= 0 ? &nb[ch[k]] : &leaf[order[-ch[k] - 1]];
                for (int a = 0; a < 3; ++a) {
                    if (c->lo[a] < b.lo[a]) b.lo[a] = c->lo[a];
                    if (c->hi[a] > b.hi[a]) b.hi[a] = c->hi[a];
                }
            }
            nb[v] = b;
        }
        free(st); free(seen);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nr; ++r) {
        double o[3] = {orig[3 * r], orig[3 * r + 1], orig[3 * r + 2]};
        double d[3] = {dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2]};
        double t0 = tmin, t1 = t_term[r];
        int64_t cand = 0, nodes = 0;
        if (ni == 0) {
            for (int64_t i = 0; i < n; ++i) cand += seg_box(&leaf[i], o, d, t0, t1);
        } else if (seg_box(&nb[0], o, d, t0, t1)) {
            int64_t stack[128];
            int sp = 0;
            stack[sp++] = 0;
            while (sp) {
                int64_t v = stack[--sp];
                ++nodes;
                int64_t ch[2] = {lc[v], rc[v]};
                for (int k = 0; k < 2; ++k) {
                    if (ch[k] >= 0) {
                        if (seg_box(&nb[ch[k]], o, d, t0, t1)) stack[sp++] = ch[k];
                    } else {
                        cand += seg_box(&leaf[order[-ch[k] - 1]], o, d, t0, t1);
                    }
                }
            }
        }
        n_cand[r] = cand;
        n_node[r] = nodes;
    }
    free(t_term); free(leaf); free(codes); free(order); free(sc); free(lc); free(rc); free(nb);
    return 0;
}
