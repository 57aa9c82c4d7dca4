// scene.hip -- surfel records and LBVH construction on the GPU.
//
// The paper bounds each 2D Gaussian by an adaptive icosahedron whose radius
// sqrt(2 ln(o / alpha_min)) shrinks with opacity, and indexes the proxies with
// a BVH (Sec. 3.2, Eq. icosahedron_transform).  Here the proxy is the
// axis-aligned box of the ellipse rho <= min(3, sqrt(2 ln(o / alpha_min))), and
// the BVH is an LBVH built in five steps, all on the caller's stream:
//   1. boxes + scene bounds of box centres     (k_boxes, ordered-int atomics)
//   2. 30-bit Morton codes of the centres      (k_morton)
//   3. stable LSD radix sort, 4 passes x 8 bit (k_radix_hist/scan/scatter)
//   4. records in sorted order                 (k_records)
//   5. Karras hierarchy, then bottom-up refit  (k_hierarchy, k_refit)
#include <algorithm>

#include "grt_internal.h"

namespace grt {


// support bound rho^2 <= min(9, 2 ln(o / alpha_min)), evaluated in double and
// rounded once, so it does not depend on the math library's last ulp
__device__ __forceinline__ float support_r2(float op, float alpha_min)
{
    if (!(alpha_min > 0.0f)) return 9.0f;
    double b = 2.0 * log((double)op / (double)alpha_min);
    return (float)(b < 9.0 ? b : 9.0);
}

__global__ void k_init(int32_t *bounds)
{
    if (threadIdx.x < 3) bounds[threadIdx.x] = 0x7fffffff;            // min of centres
    else if (threadIdx.x < 6) bounds[threadIdx.x] = (int32_t)0x80000000;  // max of centres
}

__global__ void k_boxes(int n, const float *__restrict__ means, const float *__restrict__ scales,
                        const float *__restrict__ quats, const float *__restrict__ opacity, float alpha_min,
                        float *__restrict__ box, int32_t *__restrict__ bounds)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    float c[3] = {INFINITY, INFINITY, INFINITY}, C[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (i < n) {
        float3 tu, tv, nn;
        frame32(quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3], tu, tv, nn);
        float su = scales[2 * i], sv = scales[2 * i + 1];
        float r2 = support_r2(opacity[i], alpha_min);
        float r = r2 > 0.0f ? sqrtf(r2) * 1.00001f : 0.0f;
        float tuv[3][2] = {{tu.x, tv.x}, {tu.y, tv.y}, {tu.z, tv.z}};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float x = su * tuv[a][0], y = sv * tuv[a][1];
            float e = r * sqrtf(x * x + y * y) + kPad;
            float mu = means[3 * i + a];
            box[6 * (size_t)i + a] = mu - e;
            box[6 * (size_t)i + 3 + a] = mu + e;
            c[a] = C[a] = mu;
        }
    }
    // block reduction of the centre bounds, then one atomic per block and axis
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
    if (threadIdx.x < 3) atomicMin(&bounds[threadIdx.x], f2o(red[threadIdx.x][0]));
    else if (threadIdx.x < 6) atomicMax(&bounds[threadIdx.x], f2o(red[threadIdx.x][0]));
}

__device__ __forceinline__ uint32_t spread_bits(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton(int n, const float *__restrict__ means, const int32_t *__restrict__ bounds,
                         uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float lo = o2f(bounds[a]), hi = o2f(bounds[3 + a]);
        float ext = hi - lo;
        float f = ext > 0.0f ? (means[3 * i + a] - lo) / ext : 0.0f;
        int v = (int)floorf(f * 1024.0f);
        q[a] = (uint32_t)min(max(v, 0), 1023);
    }
    keys[i] = (spread_bits(q[0]) << 2) | (spread_bits(q[1]) << 1) | spread_bits(q[2]);
    vals[i] = (uint32_t)i;
}

// ---- stable LSD radix sort, 8-bit digits -----------------------------------

// Per-tile digit counts, stored digit-major: hist[digit * blocks + tile].
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(int n, const uint32_t *__restrict__ keys, int shift,
                                                             uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortItems; ++r) {
        int i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix sum over the digit-major histogram (one block).
__global__ void __launch_bounds__(1024) k_radix_scan(int total, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t part[1024];
    int per = (total + 1023) / 1024;
    int beg = threadIdx.x * per, end = min(beg + per, total);
    uint32_t s = 0;
    for (int i = beg; i < end; ++i) s += hist[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (int i = beg; i < end; ++i) {
        uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

// The same exclusive prefix sum for long histograms (the sort of a frame's
// samples): per-chunk sums, a scan of the sums, then each chunk rescanned
// from its offset.  kScanChunk entries per block, 16 per thread.
constexpr int kScanChunk = 4096;

__global__ void __launch_bounds__(256) k_scan_sums(int total, const uint32_t *__restrict__ hist,
                                                   uint32_t *__restrict__ sums)
{
    __shared__ uint32_t part[256];
    const int base = blockIdx.x * kScanChunk + threadIdx.x * 16;
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (base + i < total) acc += hist[base + i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = part[0];
}

__global__ void __launch_bounds__(256) k_scan_apply(int total, uint32_t *__restrict__ hist,
                                                    const uint32_t *__restrict__ sums)
{
    __shared__ uint32_t part[256];
    const int base = blockIdx.x * kScanChunk + threadIdx.x * 16;
    uint32_t v[16], acc = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        v[i] = base + i < total ? hist[base + i] : 0u;
        acc += v[i];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the thread sums
        const uint32_t x = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    uint32_t run = sums[blockIdx.x] + part[threadIdx.x] - acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (base + i < total) hist[base + i] = run;
        run += v[i];
    }
}

// Scatter with ranks that follow the input order inside the tile: each round
// of 256 keys is ranked per wavefront by matching digits bit by bit with
// ballots, then across the four wavefronts of the block through LDS.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(int n, const uint32_t *__restrict__ kin,
                                                                const uint32_t *__restrict__ vin,
                                                                uint32_t *__restrict__ kout,
                                                                uint32_t *__restrict__ vout, int shift,
                                                                const uint32_t *__restrict__ hist)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    run[tid] = hist[tid * gridDim.x + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int base = blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        int i = base + r * kSortThreads + tid;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        uint32_t val = valid ? vin[i] : 0u;
        uint32_t dig = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (dig >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0u;
        __syncthreads();
        if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t p = run[dig] + rank;
            for (int w = 0; w < wave; ++w) p += wcnt[w][dig];
            kout[p] = key;
            vout[p] = val;
        }
        __syncthreads();
        run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

// ---- records in sorted order ---------------------------------------------------

__global__ void k_records(int n, const uint32_t *__restrict__ order, const float *__restrict__ means,
                          const float *__restrict__ scales, const float *__restrict__ quats,
                          const float *__restrict__ opacity, const float *__restrict__ rgb, float alpha_min,
                          const float *__restrict__ box_tmp, float4 *__restrict__ rec, float4 *__restrict__ col,
                          float *__restrict__ leaf_box, float4 *__restrict__ qrec)
{
#pragma clang fp contract(off)
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t id = order[p];
    float3 tu, tv, nn;
    frame32(quats[4 * id], quats[4 * id + 1], quats[4 * id + 2], quats[4 * id + 3], tu, tv, nn);
    float su = scales[2 * id], sv = scales[2 * id + 1];
    float op = opacity[id];
    rec[4 * (size_t)p + 0] = make_float4(means[3 * id], means[3 * id + 1], means[3 * id + 2], support_r2(op, alpha_min));
    rec[4 * (size_t)p + 1] = make_float4(nn.x, nn.y, nn.z, op);
    rec[4 * (size_t)p + 2] = make_float4(tu.x / su, tu.y / su, tu.z / su, __uint_as_float(id));
    rec[4 * (size_t)p + 3] = make_float4(tv.x / sv, tv.y / sv, tv.z / sv, su);
    col[p] = make_float4(rgb[3 * id], rgb[3 * id + 1], rgb[3 * id + 2], sv);
    qrec[p] = make_float4(quats[4 * id], quats[4 * id + 1], quats[4 * id + 2], quats[4 * id + 3]);
#pragma unroll
    for (int a = 0; a < 6; ++a) leaf_box[6 * (size_t)p + a] = box_tmp[6 * (size_t)id + a];
}

// ---- Karras (HPG 2012) hierarchy ---------------------------------------------

// common prefix length of sorted keys i, j; equal codes continue into the
// positions, so all keys are distinct
__device__ __forceinline__ int prefix(const uint32_t *__restrict__ codes, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    uint32_t a = codes[i], b = codes[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

__global__ void k_hierarchy(int n, const uint32_t *__restrict__ codes, Node *__restrict__ nodes,
                            int32_t *__restrict__ parent_int, int32_t *__restrict__ parent_leaf,
                            uint32_t *__restrict__ flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (prefix(codes, n, i, i + 1) - prefix(codes, n, i, i - 1)) > 0 ? 1 : -1;
    int dmin = prefix(codes, n, i, i - d);
    int lmax = 2;
    while (prefix(codes, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix(codes, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = prefix(codes, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix(codes, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + min(d, 0);
    int lo = min(i, j), hi = max(i, j);
    int left = (lo == gamma) ? -(gamma + 1) : gamma;
    int right = (hi == gamma + 1) ? -(gamma + 2) : gamma + 1;
    nodes[i].d = make_int4(left, right, 0, 0);
    if (left < 0) parent_leaf[gamma] = (i << 1) | 0; else parent_int[gamma] = (i << 1) | 0;
    if (right < 0) parent_leaf[gamma + 1] = (i << 1) | 1; else parent_int[gamma + 1] = (i << 1) | 1;
    if (i == 0) parent_int[0] = -1;
    flags[i] = 0u;
}

__device__ __forceinline__ void put_box(Node *nd, int side, const float b[6])
{
    float *w = reinterpret_cast<float *>(nd);
    int o = side ? 6 : 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) w[o + a] = b[a];
}

// Bottom-up: each leaf writes its box into its parent's slot; the second of
// two children to arrive at a node (atomic counter) merges both slots and
// carries the union upwards.  Slot reads go to the coherent level with
// device-scope atomic loads.
__global__ void k_refit(int n, const float *__restrict__ leaf_box, Node *nodes, const int32_t *__restrict__ parent_int,
                        const int32_t *__restrict__ parent_leaf, uint32_t *flags)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float b[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) b[a] = leaf_box[6 * (size_t)p + a];
    int link = parent_leaf[p];
    while (link >= 0) {
        int node = link >> 1, side = link & 1;
        put_box(&nodes[node], side, b);
        __threadfence();
        uint32_t old = atomicAdd(&flags[node], 1u);
        if (old == 0u) return;
        __threadfence();
        const float *w = reinterpret_cast<const float *>(&nodes[node]);
        float v[12];
#pragma unroll
        for (int a = 0; a < 12; ++a) v[a] = __hip_atomic_load(w + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b[a] = fminf(v[a], v[6 + a]);
            b[3 + a] = fmaxf(v[3 + a], v[9 + a]);
        }
        link = parent_int[node];
    }
}

// ---------------------------------------------------------------------------
// The 4-wide hierarchy the traversal walks, collapsed top down from the
// binary LBVH, one level of 4-wide nodes per launch.  A 4-wide node starts
// from a binary node's two children and twice opens the internal child of
// largest surface area (replacing it by its two children), so it has 2..4
// children.  Its internal children become the 4-wide nodes of the next level:
// each takes the next index from a counter and records which binary node it
// collapses.  Level ranges and the counter live in device memory, so the
// host launches a fixed number of levels without reading anything back.
// ---------------------------------------------------------------------------
constexpr int kCollapseLevels = 64;  // >= the LBVH's depth bound (63) + 1

__device__ __forceinline__ float box_area(const float *b)
{
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
}

__global__ void k_collapse_init(int32_t *__restrict__ ctl, int32_t *__restrict__ f4)
{
    if (threadIdx.x == 0) {
        ctl[0] = 0;  // level range [lo, hi)
        ctl[1] = 1;
        ctl[2] = 1;  // nodes allocated
        f4[0] = 0;   // the root collapses binary node 0
    }
}

__global__ void k_collapse_next(int32_t *__restrict__ ctl)
{
    if (threadIdx.x == 0) {
        ctl[0] = ctl[1];
        ctl[1] = ctl[2];
    }
}

__global__ void __launch_bounds__(256) k_collapse(const Node *__restrict__ bin, Node4 *__restrict__ out,
                                                   int32_t *__restrict__ f4, int32_t *ctl)
{
    const int lo = ctl[0], hi = ctl[1];
    for (int i = lo + (int)(blockIdx.x * blockDim.x + threadIdx.x); i < hi; i += (int)(gridDim.x * blockDim.x)) {
        float box[4][6];
        int ref[4];
        const float *w = reinterpret_cast<const float *>(&bin[f4[i]]);
        const int4 c = bin[f4[i]].d;
#pragma unroll
        for (int a = 0; a < 6; ++a) { box[0][a] = w[a]; box[1][a] = w[6 + a]; }
        ref[0] = c.x;
        ref[1] = c.y;
        int m = 2;
        for (int e = 0; e < 2; ++e) {
            int best = -1;
            float ba = -1.0f;
            for (int j = 0; j < m; ++j)
                if (ref[j] >= 0) {
                    const float ar = box_area(box[j]);
                    if (ar > ba) { ba = ar; best = j; }
                }
            if (best < 0) break;
            const Node &nd = bin[ref[best]];
            const float *v = reinterpret_cast<const float *>(&nd);
            const int4 d = nd.d;
#pragma unroll
            for (int a = 0; a < 6; ++a) { box[best][a] = v[a]; box[m][a] = v[6 + a]; }
            ref[best] = d.x;
            ref[m] = d.y;
            ++m;
        }
        Node4 o;
        float *lo4 = reinterpret_cast<float *>(&o.lx);  // lx, ly, lz, hx, hy, hz: 6 x 4 floats
        int *ch = reinterpret_cast<int *>(&o.ch);
        for (int j = 0; j < 4; ++j) {
            int r = kNoChild;
            if (j < m) {
                r = ref[j];
                if (r >= 0) {
                    const int k = atomicAdd(&ctl[2], 1);
                    f4[k] = r;
                    r = k;
                }
            }
            ch[j] = r;
#pragma unroll
            for (int a = 0; a < 6; ++a) lo4[4 * a + j] = j < m ? box[j][a] : 0.0f;
        }
        o.pad = make_int4(m, 0, 0, 0);
        out[i] = o;
    }
}

hipError_t launch_collapse4(int n, const Node *nodes, Node4 *nodes4, int32_t *f4, int32_t *ctl, hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(1024, ((int64_t)n / 2 + 255) / 256);
    hipLaunchKernelGGL(k_collapse_init, dim3(1), dim3(64), 0, st, ctl, f4);
    for (int l = 0; l < kCollapseLevels; ++l) {
        hipLaunchKernelGGL(k_collapse, dim3(blocks), dim3(256), 0, st, nodes, nodes4, f4, ctl);
        hipLaunchKernelGGL(k_collapse_next, dim3(1), dim3(64), 0, st, ctl);
    }
    return hipGetLastError();
}

void launch_radix_sort(int n, int passes, uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, uint32_t *hist,
                       hipStream_t st)
{
    const int sb = (int)sort_blocks(n);
    const int total = 256 * sb;
    // long histograms: chunk sums live after the histogram (scan_sum_words)
    const int chunks = (total + kScanChunk - 1) / kScanChunk;
    uint32_t *sums = hist + total;
    uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3(sb), dim3(kSortThreads), 0, st, n, ki, shift, hist);
        if (chunks > 16) {
            hipLaunchKernelGGL(k_scan_sums, dim3(chunks), dim3(256), 0, st, total, hist, sums);
            hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, chunks, sums);
            hipLaunchKernelGGL(k_scan_apply, dim3(chunks), dim3(256), 0, st, total, hist, sums);
        } else {
            hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, total, hist);
        }
        hipLaunchKernelGGL(k_radix_scatter, dim3(sb), dim3(kSortThreads), 0, st, n, ki, vi, ko, vo, shift, hist);
        uint32_t *t0 = ki, *t1 = vi;
        ki = ko; vi = vo; ko = t0; vo = t1;
    }
}

// Pieces of the LBVH build shared with the triangle mesh: reset the centre
// bounds; Morton codes of centres [n,3] within the bounds and their sort
// (sorted codes / original indices back in keys0 / vals0); the hierarchy over
// the sorted codes and the refit from leaf boxes in sorted order.
hipError_t launch_bounds_reset(int32_t *bounds, hipStream_t st)
{
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, bounds);
    return hipGetLastError();
}

hipError_t launch_morton_sort(int n, const float *centres, const int32_t *bounds, uint32_t *keys0, uint32_t *vals0,
                              uint32_t *keys1, uint32_t *vals1, uint32_t *hist, hipStream_t st)
{
    const int tb = 256, gb = (n + tb - 1) / tb;
    hipLaunchKernelGGL(k_morton, dim3(gb), dim3(tb), 0, st, n, centres, bounds, keys0, vals0);
    launch_radix_sort(n, 4, keys0, vals0, keys1, vals1, hist, st);
    return hipGetLastError();
}

hipError_t launch_hierarchy_refit(int n, const uint32_t *keys, const float *leaf_box, Node *nodes, int32_t *parent_int,
                                  int32_t *parent_leaf, uint32_t *flags, hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    const int tb = 256, gb = (n + tb - 1) / tb, gi = (n - 1 + tb - 1) / tb;
    hipLaunchKernelGGL(k_hierarchy, dim3(gi), dim3(tb), 0, st, n, keys, nodes, parent_int, parent_leaf, flags);
    hipLaunchKernelGGL(k_refit, dim3(gb), dim3(tb), 0, st, n, leaf_box, nodes, parent_int, parent_leaf, flags);
    return hipGetLastError();
}

hipError_t launch_scene_build(const grt_surfels &s, float alpha_min, const SceneWS &w, hipStream_t st)
{
    const int n = (int)s.n;
    if (n <= 0) return hipSuccess;
    const int tb = 256, gb = (n + tb - 1) / tb;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, w.bounds);
    hipLaunchKernelGGL(k_boxes, dim3(gb), dim3(tb), 0, st, n, s.means, s.scales, s.quats, s.opacity, alpha_min,
                       w.box_tmp, w.bounds);
    hipLaunchKernelGGL(k_morton, dim3(gb), dim3(tb), 0, st, n, s.means, w.bounds, w.keys0, w.vals0);
    // four passes: sorted codes/ids are back in keys0/vals0
    launch_radix_sort(n, 4, w.keys0, w.vals0, w.keys1, w.vals1, w.hist, st);
    hipLaunchKernelGGL(k_records, dim3(gb), dim3(tb), 0, st, n, w.vals0, s.means, s.scales, s.quats, s.opacity, s.rgb,
                       alpha_min, w.box_tmp, w.rec, w.col, w.leaf_box, w.quat);
    if (n > 1) {
        int gi = (n - 1 + tb - 1) / tb;
        hipLaunchKernelGGL(k_hierarchy, dim3(gi), dim3(tb), 0, st, n, w.keys0, w.nodes, w.parent_int, w.parent_leaf,
                           w.flags);
        hipLaunchKernelGGL(k_refit, dim3(gb), dim3(tb), 0, st, n, w.leaf_box, w.nodes, w.parent_int, w.parent_leaf,
                           w.flags);
        return launch_collapse4(n, w.nodes, w.nodes4, w.f4, w.ctl4, st);
    }
    return hipGetLastError();
}

}  // namespace grt
