// mesh.hip -- mesh backend of the attribute query (Sec. 3.5.2, "Mesh-based
// ray tracing"): a triangle mesh with per-vertex albedo, roughness, metallic
// and normal answers Trace_attr by one closest-hit ray-triangle query per ray
// instead of ordered ray-splat evaluation.  A miss sets V = 1 (the ray sees
// the environment); a hit sets V = 0 and interpolates the vertex attributes
// with the hit's barycentric weights.
//
// MI355X has no ray-tracing units, so the query is software: an LBVH over the
// triangles' boxes, built with the surfel scene's Morton / radix-sort /
// Karras / refit kernels, and a closest-hit traversal, one thread per ray,
// nearer child first, pruned by the closest hit so far.
#include "grt_internal.h"

namespace grt {

// Box (exact, padded by kPad) and centre of each triangle; the centres'
// bounds by block reduction and one atomic per block and axis.  A triangle
// with a vertex index outside [0, nv) is made degenerate: an empty box that
// no ray enters.
__global__ void k_tri_boxes(int nv, const float *__restrict__ verts, int nf, const int32_t *__restrict__ tris,
                            float *__restrict__ box, float *__restrict__ centre, int32_t *__restrict__ bounds)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float c[3] = {INFINITY, INFINITY, INFINITY}, C[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (i < nf) {
        const int ia = tris[3 * i], ib = tris[3 * i + 1], ic = tris[3 * i + 2];
        const bool ok = ia >= 0 && ia < nv && ib >= 0 && ib < nv && ic >= 0 && ic < nv;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float lo = INFINITY, hi = -INFINITY, m = 0.0f;
            if (ok) {
                const float x = verts[3 * ia + a], y = verts[3 * ib + a], z = verts[3 * ic + a];
                lo = fminf(fminf(x, y), z) - kPad;
                hi = fmaxf(fmaxf(x, y), z) + kPad;
                m = (x + y + z) * (1.0f / 3.0f);
                c[a] = C[a] = m;
            }
            box[6 * (size_t)i + a] = lo;
            box[6 * (size_t)i + 3 + a] = hi;
            centre[3 * (size_t)i + a] = m;
        }
    }
    __shared__ float red[6][256];
#pragma unroll
    for (int a = 0; a < 3; ++a) { red[a][threadIdx.x] = c[a]; red[3 + a][threadIdx.x] = C[a]; }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 3 && red[threadIdx.x][0] <= red[3 + threadIdx.x][0]) {
        atomicMin(&bounds[threadIdx.x], f2o(red[threadIdx.x][0]));
        atomicMax(&bounds[3 + threadIdx.x], f2o(red[3 + threadIdx.x][0]));
    }
}

// Records and leaf boxes in Morton order.
__global__ void k_tri_records(int nv, const float *__restrict__ verts, int nf, const int32_t *__restrict__ tris,
                              const uint32_t *__restrict__ order, const float *__restrict__ box_tmp,
                              float4 *__restrict__ rec, float *__restrict__ leaf_box)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nf) return;
    const uint32_t id = order[p];
    const int ia = tris[3 * id], ib = tris[3 * id + 1], ic = tris[3 * id + 2];
    const bool ok = ia >= 0 && ia < nv && ib >= 0 && ib < nv && ic >= 0 && ic < nv;
    float3 v0 = make_float3(0.f, 0.f, 0.f), e1 = v0, e2 = v0;
    if (ok) {
        v0 = make_float3(verts[3 * ia], verts[3 * ia + 1], verts[3 * ia + 2]);
        e1 = make_float3(verts[3 * ib] - v0.x, verts[3 * ib + 1] - v0.y, verts[3 * ib + 2] - v0.z);
        e2 = make_float3(verts[3 * ic] - v0.x, verts[3 * ic + 1] - v0.y, verts[3 * ic + 2] - v0.z);
    }
    rec[3 * (size_t)p] = make_float4(v0.x, v0.y, v0.z, __uint_as_float(id));
    rec[3 * (size_t)p + 1] = make_float4(e1.x, e1.y, e1.z, 0.0f);
    rec[3 * (size_t)p + 2] = make_float4(e2.x, e2.y, e2.z, 0.0f);
#pragma unroll
    for (int a = 0; a < 6; ++a) leaf_box[6 * (size_t)p + a] = box_tmp[6 * (size_t)id + a];
}

hipError_t launch_mesh_build(int nv, const float *verts, int nf, const int32_t *tris, const MeshWS &w, hipStream_t st)
{
    if (nf <= 0) return hipSuccess;
    const int tb = 256, gb = (nf + tb - 1) / tb;
    hipError_t e = launch_bounds_reset(w.bounds, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tri_boxes, dim3(gb), dim3(tb), 0, st, nv, verts, nf, tris, w.box_tmp, w.centre, w.bounds);
    if ((e = launch_morton_sort(nf, w.centre, w.bounds, w.keys0, w.vals0, w.keys1, w.vals1, w.hist, st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_tri_records, dim3(gb), dim3(tb), 0, st, nv, verts, nf, tris, w.vals0, w.box_tmp, w.rec,
                       w.leaf_box);
    return launch_hierarchy_refit(nf, w.keys0, w.leaf_box, w.nodes, w.parent_int, w.parent_leaf, w.flags, st);
}

// Moller-Trumbore (two-sided) with a fixed operation order; true on a hit
// with t in (tmin, tbest], or at t == tbest with a lower triangle id.
__device__ __forceinline__ bool tri_hit(const float4 r0, const float4 r1, const float4 r2, float3 o, float3 d,
                                        float tmin, float tbest, uint32_t best_id, float &t, float &u, float &v)
{
#pragma clang fp contract(off)
    const float3 e1 = make_float3(r1.x, r1.y, r1.z), e2 = make_float3(r2.x, r2.y, r2.z);
    const float px = d.y * e2.z - d.z * e2.y, py = d.z * e2.x - d.x * e2.z, pz = d.x * e2.y - d.y * e2.x;
    const float det = e1.x * px + e1.y * py + e1.z * pz;
    if (fabsf(det) < 1e-20f) return false;
    const float inv = 1.0f / det;
    const float sx = o.x - r0.x, sy = o.y - r0.y, sz = o.z - r0.z;
    u = (sx * px + sy * py + sz * pz) * inv;
    if (u < 0.0f || u > 1.0f) return false;
    const float qx = sy * e1.z - sz * e1.y, qy = sz * e1.x - sx * e1.z, qz = sx * e1.y - sy * e1.x;
    v = (d.x * qx + d.y * qy + d.z * qz) * inv;
    if (v < 0.0f || u + v > 1.0f) return false;
    t = (e2.x * qx + e2.y * qy + e2.z * qz) * inv;
    if (!(t > tmin && t <= tbest)) return false;
    return t < tbest || __float_as_uint(r0.w) < best_id;
}

constexpr int kMeshStack = 64;  // LBVH depth <= 63: one far child per level

// Closest hit of one ray: triangle id (0xffffffff: miss) and barycentrics.
__device__ __forceinline__ void mesh_closest(const float4 *__restrict__ rec, const Node *__restrict__ nodes, int nf,
                                             float3 o, float3 d, float tmin, float tmax, uint32_t &bid, float &bu,
                                             float &bv)
{
    const float3 inv = make_float3(safe_inv(d.x), safe_inv(d.y), safe_inv(d.z));
    float best = tmax;
    bu = 0.0f; bv = 0.0f;
    bid = 0xffffffffu;
    int stack[kMeshStack];
    int sp = 0;
    int cur = nf <= 0 ? kNone : (nf == 1 ? -1 : 0);
    while (cur != kNone) {
        if (cur < 0) {  // leaf: triangle record -(cur + 1)
            const float4 *rr = rec + 3 * (size_t)(-cur - 1);
            const float4 r0 = rr[0], r1 = rr[1], r2 = rr[2];
            float t, u, v;
            if (tri_hit(r0, r1, r2, o, d, tmin, best, bid, t, u, v)) {
                best = t; bu = u; bv = v; bid = __float_as_uint(r0.w);
            }
            cur = sp > 0 ? stack[--sp] : kNone;
            continue;
        }
        const Node nd = nodes[cur];
        float tl, tr;
        const bool hl = slab(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, o, inv, tmin, best, tl);
        const bool hr = slab(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, o, inv, tmin, best, tr);
        if (hl && hr) {
            const bool lf = tl <= tr;
            if (sp < kMeshStack) stack[sp++] = lf ? nd.d.y : nd.d.x;
            cur = lf ? nd.d.x : nd.d.y;
        } else if (hl) {
            cur = nd.d.x;
        } else if (hr) {
            cur = nd.d.y;
        } else {
            cur = sp > 0 ? stack[--sp] : kNone;
        }
    }
}

// Barycentric vertex attributes of the hit (the normal facing the ray
// origin); V = 1 and zeros on a miss.
struct MeshHitAttrs {
    float V, A[3], R, M, N[3];
};
__device__ __forceinline__ MeshHitAttrs mesh_attrs(const int32_t *__restrict__ tris, int nf, const float *albedo,
                                                   const float *rough, const float *metal, const float *vnormal,
                                                   uint32_t bid, float bu, float bv, float3 d)
{
    MeshHitAttrs h = {1.0f, {0.f, 0.f, 0.f}, 0.0f, 0.0f, {0.f, 0.f, 0.f}};
    if (bid == 0xffffffffu || bid >= (uint32_t)nf) return h;
    h.V = 0.0f;
    const float w[3] = {1.0f - bu - bv, bu, bv};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int vi = tris[3 * (size_t)bid + k];  // valid: degenerate triangles are never hit
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h.A[c] += w[k] * albedo[3 * (size_t)vi + c];
            h.N[c] += w[k] * vnormal[3 * (size_t)vi + c];
        }
        h.R += w[k] * rough[vi];
        h.M += w[k] * metal[vi];
    }
    if (h.N[0] * d.x + h.N[1] * d.y + h.N[2] * d.z > 0.0f) { h.N[0] = -h.N[0]; h.N[1] = -h.N[1]; h.N[2] = -h.N[2]; }
    return h;
}

__global__ void __launch_bounds__(256) k_mesh_trace_attr(MeshTraceArgs a)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    const float3 o = make_float3(a.o[3 * r], a.o[3 * r + 1], a.o[3 * r + 2]);
    const float3 d = make_float3(a.d[3 * r], a.d[3 * r + 1], a.d[3 * r + 2]);
    uint32_t bid;
    float bu, bv;
    mesh_closest(a.rec, a.nodes, a.nf, o, d, a.tmin, a.tmax, bid, bu, bv);
    const MeshHitAttrs h = mesh_attrs(a.tris, a.nf, a.albedo, a.rough, a.metal, a.vnormal, bid, bu, bv, d);
    a.out_V[r] = h.V;
#pragma unroll
    for (int c = 0; c < 3; ++c) { a.out_albedo[3 * r + c] = h.A[c]; a.out_normal[3 * r + c] = h.N[c]; }
    a.out_rough[r] = h.R;
    a.out_metal[r] = h.M;
}

// Relighting through the mesh, query pass: for every traced sample of the
// render's ray records, the mesh query parked for the shading pass as the
// surfel relight parks it ((V, albedo) in the contribution slot, (r, m) in
// the ray record's spare words, the normal in rl_n*).
__global__ void __launch_bounds__(256) k_mesh_relight_query(RenderArgs a, MeshTraceArgs m, int64_t total)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= total) return;
    const float4 r0 = a.rays[3 * r];
    if (r0.w == 0.0f) {
        a.contrib[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const int64_t p = r / (a.nc + a.ng + a.ne);
    const float3 x = make_float3(a.x[3 * p], a.x[3 * p + 1], a.x[3 * p + 2]);
    const float3 d = make_float3(r0.x, r0.y, r0.z);
    uint32_t bid;
    float bu, bv;
    mesh_closest(m.rec, m.nodes, m.nf, x, d, a.tmin, INFINITY, bid, bu, bv);
    const MeshHitAttrs h = mesh_attrs(m.tris, m.nf, m.albedo, m.rough, m.metal, m.vnormal, bid, bu, bv, d);
    a.contrib[r] = make_float4(h.V, h.A[0], h.A[1], h.A[2]);
    float4 *r2 = a.rays + 3 * r + 2;
    r2->z = h.R;
    r2->w = h.M;
    a.rl_nx[r] = h.N[0];
    a.rl_ny[r] = h.N[1];
    a.rl_nz[r] = h.N[2];
}

hipError_t launch_mesh_relight_query(const RenderArgs &a, const MeshTraceArgs &m, hipStream_t st)
{
    const int64_t total = (int64_t)a.H * a.W * (a.nc + a.ng + a.ne);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mesh_relight_query, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, m, total);
    return hipGetLastError();
}

hipError_t launch_mesh_trace_attr(const MeshTraceArgs &a, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mesh_trace_attr, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace grt
