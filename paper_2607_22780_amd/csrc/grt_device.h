// grt_device.h -- device-side data layout and the shared traversal of libgrt.
//
// Scene layout in the caller's workspace (all in Morton order of the surfel
// bounding-box centres, so neighbouring surfels sit in neighbouring lines):
//   rec  [n][4] float4   r0 = (mu.xyz, r2max)      r1 = (n.xyz, opacity)
//                        r2 = (a_u.xyz, id bits)   r3 = (a_v.xyz, s_u)
//                        with a_u = t_u / s_u, a_v = t_v / s_v      (64 B)
//   col  [n]    float4   (rgb, s_v)                                  (16 B)
//   quat [n]    float4   the stored quaternion (w, x, y, z)          (16 B)
// The backward's chain rule reads the stored scales and quaternion of each
// composited hit from these, by record position, not from the caller's arrays
// by surfel id, which would cost a random line per hit.
//   node [n-1]  Node     both child boxes + child references        (64 B)
// A child reference >= 0 is an internal node, < 0 is leaf -(pos+1).
//   node4 [<= n-1] Node4 the same hierarchy collapsed to 4 children per
//                        node (boxes as structure of arrays, references as
//                        above, >= 0 now a 4-wide node)           (128 B)
// The traversal walks the 4-wide nodes: half the node steps of the binary
// tree, each testing up to four boxes from one 128-byte line.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

// Minimum waves per SIMD requested for the persistent trace kernels (caps
// their register budget); 0 leaves the choice to the compiler.
#ifndef GRT_WAVES_PER_EU
#define GRT_WAVES_PER_EU 0
#endif
#if GRT_WAVES_PER_EU > 0
#define GRT_OCCUPANCY __attribute__((amdgpu_waves_per_eu(GRT_WAVES_PER_EU)))
#else
#define GRT_OCCUPANCY
#endif

namespace grt {

constexpr float kGrazing = 1e-6f; // |n . d| below this is no intersection
constexpr float kPad = 1e-5f;     // absolute padding of surfel boxes (scene units)

struct alignas(16) Node {
    float4 a;  // L.lo.x L.lo.y L.lo.z L.hi.x
    float4 b;  // L.hi.y L.hi.z R.lo.x R.lo.y
    float4 c;  // R.lo.z R.hi.x R.hi.y R.hi.z
    int4 d;    // left, right, unused, unused
};

// Unused child slots of a 4-wide node hold this reference (and a zero box).
constexpr int kNoChild = 0x7fffffff;

struct alignas(16) Node4 {
    float4 lx, ly, lz;  // lower corners of the four child boxes
    float4 hx, hy, hz;  // upper corners
    int4 ch;            // child references (kNoChild: unused slot)
    int4 pad;
};

struct SceneDev {
    const float4 *rec;
    const float4 *col;
    const Node *nodes;
    const float4 *quat;  // stored quaternions in record order
    const Node4 *nodes4;
    int32_t n;
};

// ---------------------------------------------------------------------------
// Canonical single-precision arithmetic of the hit decision.  The operation
// order is fixed and contraction is off, so the decision, the depth and the
// (depth, id) order are reproducible bit for bit by any IEEE implementation
// of the same sequence.
// ---------------------------------------------------------------------------

// Frame of a surfel: t_u, t_v, n are the columns of R(q/|q|) (Hamilton, w first).
__device__ __forceinline__ void frame32(float w, float x, float y, float z, float3 &tu, float3 &tv, float3 &n)
{
#pragma clang fp contract(off)
    float l = sqrtf(w * w + x * x + y * y + z * z);
    w = w / l; x = x / l; y = y / l; z = z / l;
    float xx = x * x, yy = y * y, zz = z * z;
    float xy = x * y, xz = x * z, yz = y * z;
    float wx = w * x, wy = w * y, wz = w * z;
    tu = make_float3(1.0f - 2.0f * (yy + zz), 2.0f * (xy + wz), 2.0f * (xz - wy));
    tv = make_float3(2.0f * (xy - wz), 1.0f - 2.0f * (xx + zz), 2.0f * (yz + wx));
    n = make_float3(2.0f * (xz + wy), 2.0f * (yz - wx), 1.0f - 2.0f * (xx + yy));
}

// Canonical crossing: m = mu - o, den = n.d, tau = n.m / den, D = tau d - m,
// u = a_u.D, v = a_v.D, rho^2 = u^2 + v^2 (fixed order, no contraction).
__device__ __forceinline__ void canon_geo(const float4 r0, const float4 r1, const float4 r2, const float4 r3,
                                          const float3 o, const float3 d, float &den, float &tau, float &rho2)
{
#pragma clang fp contract(off)
    float m0 = r0.x - o.x, m1 = r0.y - o.y, m2 = r0.z - o.z;
    den = r1.x * d.x + r1.y * d.y + r1.z * d.z;
    float num = r1.x * m0 + r1.y * m1 + r1.z * m2;
    tau = num / den;
    float dx = tau * d.x - m0, dy = tau * d.y - m1, dz = tau * d.z - m2;
    float u = r2.x * dx + r2.y * dy + r2.z * dz;
    float v = r3.x * dx + r3.y * dy + r3.z * dz;
    rho2 = u * u + v * v;
}

// Value geometry of a hit: the same crossing evaluated in double from the
// single-precision record (the in-plane offset D = tau d - m cancels badly in
// single precision for small surfels seen from afar).
struct HitGeo {
    float u, v, rho2, den;
    float3 D;
};

__device__ __forceinline__ void value_geo(const float4 r0, const float4 r1, const float4 r2, const float4 r3,
                                          const float3 o, const float3 d, HitGeo &g)
{
    // with num = n.m and den = n.d:  den * u = num (a_u.d) - den (a_u.m), the
    // cancelling terms taken in double; one single-precision reciprocal
    const double mx = (double)r0.x - (double)o.x, my = (double)r0.y - (double)o.y, mz = (double)r0.z - (double)o.z;
    const double dx = d.x, dy = d.y, dz = d.z;
    const double nx = r1.x, ny = r1.y, nz = r1.z;
    const double den = nx * dx + ny * dy + nz * dz;
    const double num = nx * mx + ny * my + nz * mz;
    const double U = num * ((double)r2.x * dx + (double)r2.y * dy + (double)r2.z * dz) -
                     den * ((double)r2.x * mx + (double)r2.y * my + (double)r2.z * mz);
    const double V = num * ((double)r3.x * dx + (double)r3.y * dy + (double)r3.z * dz) -
                     den * ((double)r3.x * mx + (double)r3.y * my + (double)r3.z * mz);
    const float fden = (float)den;
    const float rden = 1.0f / fden;
    g.u = (float)U * rden;
    g.v = (float)V * rden;
    g.rho2 = g.u * g.u + g.v * g.v;
    g.den = fden;
    g.D = make_float3((float)(num * dx - den * mx) * rden, (float)(num * dy - den * my) * rden,
                      (float)(num * dz - den * mz) * rden);
}

// Opacity contribution of a hit, alpha = o exp(-rho^2 / 2), and the
// single-precision transmittance step that decides where compositing stops.
__device__ __forceinline__ float hit_alpha(float op, float rho2)
{
#pragma clang fp contract(off)
    return op * expf(-0.5f * rho2);
}

__device__ __forceinline__ float trans_step(float T, float a)
{
#pragma clang fp contract(off)
    return T * (1.0f - a);
}

// ---------------------------------------------------------------------------
// Slab test against one box, clipped to [t0, t1]; conservative by a few ulps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool slab(float lx, float ly, float lz, float hx, float hy, float hz, const float3 o,
                                     const float3 inv, float t0, float t1, float &tnear)
{
    float ax = (lx - o.x) * inv.x, bx = (hx - o.x) * inv.x;
    float ay = (ly - o.y) * inv.y, by = (hy - o.y) * inv.y;
    float az = (lz - o.z) * inv.z, bz = (hz - o.z) * inv.z;
    float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t0));
    float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), t1));
    tnear = tn;
    return tn <= tf * 1.0000005f + 1e-30f;
}

// The same test with each plane's entry depth as one fused multiply-add,
// l inv + (-o inv), noi = -o inv formed once per node: within an ulp of the
// subtract-then-multiply form, far inside the boxes' 1e-5 padding and the
// test's relative slack, so it still never rejects a box the ray enters.
__device__ __forceinline__ bool slab_fma(float lx, float ly, float lz, float hx, float hy, float hz, const float3 inv,
                                         const float3 noi, float t0, float t1, float &tnear)
{
    float ax = fmaf(lx, inv.x, noi.x), bx = fmaf(hx, inv.x, noi.x);
    float ay = fmaf(ly, inv.y, noi.y), by = fmaf(hy, inv.y, noi.y);
    float az = fmaf(lz, inv.z, noi.z), bz = fmaf(hz, inv.z, noi.z);
    float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t0));
    float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), t1));
    tnear = tn;
    return tn <= tf * 1.0000005f + 1e-30f;
}

// order-preserving float <-> int maps (atomic min/max of floats)
__device__ __forceinline__ int f2o(float f)
{
    int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float o2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff); }

__device__ __forceinline__ float safe_inv(float d)
{
    return 1.0f / (fabsf(d) > 1e-30f ? d : copysignf(1e-30f, d));
}

// The walk's inverse direction, formed at each node step rather than held (3
// registers): the hardware reciprocal (1 ulp) is far inside the slab test's
// slack and the boxes' padding, so the test still rejects no box the ray
// enters.
__device__ __forceinline__ float fast_inv(float d)
{
    return __builtin_amdgcn_rcpf(fabsf(d) > 1e-30f ? d : copysignf(1e-30f, d));
}

__device__ __forceinline__ uint64_t make_key(float tau, uint32_t id)
{
    return ((uint64_t)__float_as_uint(tau) << 32) | (uint64_t)id;
}

// ---------------------------------------------------------------------------
// Ordered traversal with a k-nearest hit buffer, in rounds that resume from a
// deferred frontier, as a per-lane state machine.
//
// A round walks the LBVH keeping the K smallest keys (bits(tau), id) strictly
// greater than the last key composited in the previous round (registers,
// sorted by unrolled insertion).  Once the buffer is full its largest depth
// thi bounds the walk.  Everything the bound excludes is not dropped but
// deferred to the next round: subtrees whose box is entered beyond thi, hits
// rejected by the full buffer and hits evicted from it.  The buffered hits
// are then handed to `visit` (record position, surfel id, depth) in order;
// `visit` returns true to stop (transmittance cutoff).  The next round starts
// from the deferred items instead of the root, so a ray's hits cost about one
// walk whatever K is; a round that defers nothing ends the ray.  Keys are
// unique, so hits of equal depth are neither lost nor repeated, and results
// do not depend on K.
//
// The walk stack and the deferred list share one private array, growing from
// opposite ends; their roles swap every round.  If they would collide, the
// deferred list is dropped and the next round restarts from the root, which
// re-finds every hit beyond the last composited key.
//
// advance() does one node or one hit, so a wavefront can hold rays at
// different rounds and refill lanes whose ray has finished (run_persistent).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// A lane's stack: the top kLdsDepth entries live in LDS (lane-interleaved, so
// a wavefront's accesses are conflict-free), deeper ones spill to a private
// array.  Position p sits in LDS slot p % kLdsDepth; a push that reuses the
// slot of position p - kLdsDepth first copies that entry out (entries never
// change once pushed), and a pop reads the private copy for positions below
// `spilled`.  Positions [0, spilled) always have valid private copies.
// ---------------------------------------------------------------------------
#ifndef GRT_LDS_DEPTH
#define GRT_LDS_DEPTH 24
#endif
constexpr int kLdsDepth = GRT_LDS_DEPTH;  // LDS entries per lane and stack
#ifndef GRT_BWD_LDS_DEPTH
#define GRT_BWD_LDS_DEPTH 16
#endif
constexpr int kBwdLdsDepth = GRT_BWD_LDS_DEPTH;  // backward kernels: their LDS also holds gradient tables
// Backward kernels composite a hit (running the gradient chain) only in
// surfel steps where at least kBwdCompShare16/16 of the wavefront's active
// lanes have one to composite, or no lane is still walking, and run surfel
// steps once kBwdSiteShare8/8 of the active lanes wait for one.
#ifndef GRT_BWD_COMP_SHARE16
#define GRT_BWD_COMP_SHARE16 3
#endif
#ifndef GRT_BWD_SITE_SHARE8
#define GRT_BWD_SITE_SHARE8 3
#endif
constexpr int kBwdCompShare16 = GRT_BWD_COMP_SHARE16;
constexpr int kBwdSiteShare8 = GRT_BWD_SITE_SHARE8;
// Surfel steps run when at least kSurfelShare4 / 4 of a wavefront's active
// lanes wait for one.
#ifndef GRT_SURFEL_SHARE4
#define GRT_SURFEL_SHARE4 2
#endif
constexpr int kSurfelShare4 = GRT_SURFEL_SHARE4;
constexpr int kStackCap = 384;  // logical capacity of a stack
constexpr int kNone = 0x7fffffff;

template <int D>
struct SpillStack {
    int sp, spilled;

    __device__ __forceinline__ void reset() { sp = 0; spilled = 0; }

    // lds: this lane's slot 0 of the stack (slot i at lds[64 * i]); mem:
    // its private overflow array [kStackCap]
    __device__ __forceinline__ void push(int x, int *lds, int *mem)
    {
        const int slot = sp % D;
        if (sp >= D && sp - D >= spilled) {
            mem[sp - D] = lds[64 * slot];
            spilled = sp - D + 1;
        }
        lds[64 * slot] = x;
        ++sp;
    }

    __device__ __forceinline__ int pop(int *lds, int *mem)
    {
        --sp;
        if (sp < spilled) {
            spilled = sp;
            return mem[sp];
        }
        return lds[64 * (sp % D)];
    }
};

// The walk stack and the deferred list of a lane; their roles swap each
// round (the deferred list becomes the next round's walk stack).  A round's
// stack starts with at most kMaxDeferred items; below them, a node step pops
// one item and pushes at most three, so the stack holds at most three
// siblings for each 4-wide level of the current path.  The 4-wide tree is no
// deeper than the binary LBVH (each of its edges spans at least one binary
// edge), whose depth is at most 63 (30-bit codes, then the position breaking
// ties), so the stack stays within kMaxDeferred + 3 * 63 <= kStackCap.
constexpr int kMaxDeferred = 192;
static_assert(kMaxDeferred + 3 * 63 <= kStackCap, "walk stack bound");

template <int D>
struct Frontier {
    SpillStack<D> walk;  // the current round's walk stack
    SpillStack<D> def;   // deferrals for the next round
    int *lds;            // this lane's slot 0 of stack 0; stack 1 starts D slots on
    int *mem0, *mem1;    // the two stacks' private overflow arrays
    int role;            // the stack that holds the walk (the other one defers)

    __device__ __forceinline__ int *lds_of(int which) const { return lds + 64 * D * which; }
    __device__ __forceinline__ int *mem_of(int which) const { return which ? mem1 : mem0; }
    __device__ __forceinline__ void push_walk(int x) { walk.push(x, lds_of(role), mem_of(role)); }
    __device__ __forceinline__ int pop_walk() { return walk.pop(lds_of(role), mem_of(role)); }
    __device__ __forceinline__ void push_def(int x) { def.push(x, lds_of(role ^ 1), mem_of(role ^ 1)); }

    // the deferred list becomes the walk stack (positions swapped, no copy)
    __device__ __forceinline__ void swap_roles()
    {
        const SpillStack<D> t = walk;
        walk = def;
        def = t;
        role ^= 1;
    }
};

// kCompShare16 > 0: lanes with buffered hits join a surfel step only when at
// least kCompShare16/16 of the active lanes have one, or when no lane is still
// walking, so an expensive visitor runs with more lanes at once.  Each lane's
// own sequence of steps is unchanged, and every call either walks some lane
// or runs the step for all of them.  0: they join every surfel step.
// kSiteShare8 > 0: surfel steps run once kSiteShare8/8 of the active lanes
// wait for one (0: kSurfelShare4/4).
#ifndef GRT_FWD_COMP_SHARE16
#define GRT_FWD_COMP_SHARE16 0
#endif
template <int K, int D = kLdsDepth, int kCompShare16 = GRT_FWD_COMP_SHARE16, int kSiteShare8 = 0>
struct Walker {
    static constexpr int kDepth = D;  // LDS entries per lane and stack
    float3 o, d;
    float tmin, tmax;
    uint64_t last;        // start key of the round; while compositing, the last composited hit
    uint64_t key[K];
    uint32_t pos[K];
    int cnt;
    int cur;              // item in hand: node >= 0, leaf -(pos+1), or kNone
    bool lost;            // deferred list dropped: next round restarts at the root
    Frontier<D> F;        // walk stack and deferred list (LDS + private spill)
    int ncomp;            // buffered hits still to composite (0 while walking)
    int pend;             // leaf waiting for the next surfel step (record position), or kNone
#ifdef GRT_STATS
    int st_nodes, st_leaves, st_comps, st_rounds, st_lost, st_deferred;
#endif

    __device__ __forceinline__ void clear_buffer()
    {
#pragma unroll
        for (int i = 0; i < K; ++i) { key[i] = ~0ull; pos[i] = 0; }
        cnt = 0;
    }

    // The round's walk covers [lo_bound, hi_bound]: from the last composited
    // key's depth (tmin in the first round) to the full buffer's largest
    // depth (tmax while it is not full).  Derived when needed rather than
    // held, to keep two registers free.
    __device__ __forceinline__ float lo_bound() const
    {
        return fmaxf(tmin, __uint_as_float((uint32_t)(last >> 32)));
    }
    __device__ __forceinline__ float hi_bound() const
    {
        return cnt >= K ? __uint_as_float((uint32_t)(key[K - 1] >> 32)) : tmax;
    }

    __device__ __forceinline__ void start(const SceneDev &S, float3 o_, float3 d_, float tmin_, float tmax_)
    {
        o = o_;
        d = d_;
        tmin = tmin_;
        tmax = tmax_;
        last = 0;
        ncomp = 0;
        pend = kNone;
        F.walk.reset();
        F.def.reset();
        lost = false;
        cur = S.n == 1 ? -1 : 0;
        clear_buffer();
#ifdef GRT_STATS
        st_nodes = st_leaves = st_comps = st_lost = st_deferred = 0;
        st_rounds = 1;
#endif
    }

    __device__ __forceinline__ void defer(int x)
    {
        if (lost) return;
        if (F.def.sp >= kMaxDeferred) {  // too many: drop the list, restart the next round at the root
            lost = true;
            F.def.reset();
            return;
        }
        F.push_def(x);
#ifdef GRT_STATS
        ++st_deferred;
#endif
    }

    // Leaf test from the canonical crossing of surfel record p (den, tau,
    // rho^2 as canon_geo computes them; r0.w is the bound r2max, r2.w the id):
    // a hit goes into the k-buffer, or is deferred when beyond it.
    __device__ __forceinline__ void test_leaf(uint32_t p, float den, float tau, float rho2, float r2max, float idbits)
    {
#ifdef GRT_STATS
        ++st_leaves;
#endif
        if (fabsf(den) < kGrazing || !(tau > tmin && tau <= tmax) || !(rho2 <= r2max)) return;
        uint64_t k = make_key(tau, __float_as_uint(idbits));
        if (k <= last) return;
        if (k >= key[K - 1]) {  // beyond the full buffer: next round
            defer(-(int)p - 1);
            return;
        }
        if (cnt >= K) defer(-(int)pos[K - 1] - 1);  // evicted
        // sorted insertion, the largest key drops out
        bool placed = false;
#pragma unroll
        for (int i = K - 1; i > 0; --i) {
            bool shift = key[i - 1] > k;
            uint64_t nk = shift ? key[i - 1] : (placed ? key[i] : k);
            uint32_t np = shift ? pos[i - 1] : (placed ? pos[i] : p);
            placed = placed || !shift;
            key[i] = nk;
            pos[i] = np;
        }
        if (!placed) { key[0] = k; pos[0] = p; }
        ++cnt;
    }

    // A child box met by the ray in [tlo, tmax]: process now if it starts
    // within thi, else defer it.
    __device__ __forceinline__ bool keep_child(int c, bool hit, float tn, float thi)
    {
        if (!hit) return false;
        if (tn > thi) {
            defer(c);
            return false;
        }
        return true;
    }

    // One item of the current round; true when the round's walk is complete.
    // One item of the current round's walk; `leaf` receives at most one leaf
    // to test.  True when the round's walk is complete.
    __device__ __forceinline__ bool step(const SceneDev &S, int &leaf)
    {
        if (cur == kNone) {
            if (F.walk.sp == 0) return true;
            cur = F.pop_walk();
        }
        if (cur < 0) {
            leaf = cur;
            cur = kNone;
        } else {
            walk_node(S, leaf);
        }
        return false;
    }

    // Test the children of 4-wide node `cur`; sets the next item and at most
    // one leaf to test.  Kept children (met within thi) are taken nearest
    // entry first: a leaf among them goes to the single surfel site in
    // advance() (a wavefront then runs it once per step however its lanes'
    // children are mixed), the nearest other child becomes the item in hand,
    // and the rest go on the walk stack, farthest first.
    __device__ __forceinline__ void walk_node(const SceneDev &S, int &leaf)
    {
#ifdef GRT_STATS
        ++st_nodes;
#endif
        const Node4 *nd = S.nodes4 + cur;
        const float tlo = lo_bound(), thi = hi_bound();
        const float3 inv = make_float3(fast_inv(d.x), fast_inv(d.y), fast_inv(d.z));
        const float4 lx = nd->lx, ly = nd->ly, lz = nd->lz, hx = nd->hx, hy = nd->hy, hz = nd->hz;
        const int4 ch = nd->ch;
        // all four boxes tested without branches (an unused slot's zero box
        // is masked by its reference)
        float t0, t1, t2, t3;
#ifdef GRT_SLAB_FMA
        const float3 noi = make_float3(-o.x * inv.x, -o.y * inv.y, -o.z * inv.z);
        bool k0 = slab_fma(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, inv, noi, tlo, tmax, t0);
        bool k1 = slab_fma(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, inv, noi, tlo, tmax, t1);
        bool k2 = slab_fma(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, inv, noi, tlo, tmax, t2);
        bool k3 = slab_fma(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, inv, noi, tlo, tmax, t3);
#else
        bool k0 = slab(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, o, inv, tlo, tmax, t0);
        bool k1 = slab(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, o, inv, tlo, tmax, t1);
        bool k2 = slab(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, o, inv, tlo, tmax, t2);
        bool k3 = slab(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, o, inv, tlo, tmax, t3);
#endif
        k0 = k0 & (ch.x != kNoChild);
        k1 = k1 & (ch.y != kNoChild);
        k2 = k2 & (ch.z != kNoChild);
        k3 = k3 & (ch.w != kNoChild);
        k0 = keep_child(ch.x, k0, t0, thi);
        k1 = keep_child(ch.y, k1, t1, thi);
        k2 = keep_child(ch.z, k2, t2, thi);
        k3 = keep_child(ch.w, k3, t3, thi);
        const int m = (int)k0 + (int)k1 + (int)k2 + (int)k3;
        // kept children first, by entry depth (a five-exchange sorting network)
        float s0 = k0 ? t0 : INFINITY, s1 = k1 ? t1 : INFINITY, s2 = k2 ? t2 : INFINITY, s3 = k3 ? t3 : INFINITY;
        int c0 = k0 ? ch.x : kNone, c1 = k1 ? ch.y : kNone, c2 = k2 ? ch.z : kNone, c3 = k3 ? ch.w : kNone;
        auto xch = [](float &sa, int &ca, float &sb, int &cb) {
            const bool sw = sb < sa;
            const float ts = sw ? sb : sa;
            const int tc = sw ? cb : ca;
            sb = sw ? sa : sb;
            cb = sw ? ca : cb;
            sa = ts;
            ca = tc;
        };
        xch(s0, c0, s1, c1);
        xch(s2, c2, s3, c3);
        xch(s0, c0, s2, c2);
        xch(s1, c1, s3, c3);
        xch(s1, c1, s2, c2);
        // the nearest kept leaf, if any, is the step's leaf; the others in order
        const int li = (m > 0 && c0 < 0) ? 0 : (m > 1 && c1 < 0) ? 1 : (m > 2 && c2 < 0) ? 2 : (m > 3 && c3 < 0) ? 3 : -1;
        int o0 = c0, o1 = c1, o2 = c2, o3 = c3, no = m;
        if (li >= 0) {
            leaf = li == 0 ? c0 : li == 1 ? c1 : li == 2 ? c2 : c3;
            o0 = li == 0 ? c1 : c0;
            o1 = li <= 1 ? c2 : c1;
            o2 = li <= 2 ? c3 : c2;
            no = m - 1;
        }
        cur = no >= 1 ? o0 : kNone;
        if (no >= 4) F.push_walk(o3);
        if (no >= 3) F.push_walk(o2);
        if (no >= 2) F.push_walk(o1);
    }

    // Set up the next round from the deferred frontier (or the root).  A next
    // round follows only a full buffer whose K hits were all composited, so
    // `last` already holds the round's largest key, where the next one starts.
    __device__ __forceinline__ void next_round(const SceneDev &S)
    {
        // The buffer is empty already (every composite shifted an empty key in
        // at its end, and the round composited all its hits), so only the
        // count is reset: rewriting the keys would give the registers a
        // second version to reconcile at every exit of the surfel step.
        cnt = 0;
#ifdef GRT_STATS
        ++st_rounds;
        st_lost += lost ? 1 : 0;
#endif
        F.walk.reset();  // empty: the walk is complete
        if (lost) {
            F.def.reset();
            lost = false;
            cur = S.n == 1 ? -1 : 0;
        } else {
            F.swap_roles();
            cur = kNone;
        }
    }

    // Depth of the last composited hit once the ray is finished (0 when none
    // was): a re-traversal bounded there meets the same composited hits.
    __device__ __forceinline__ float stop_depth() const { return __uint_as_float((uint32_t)(last >> 32)); }

    __device__ __forceinline__ bool deferred_empty() const
    {
        return !lost && F.def.sp == 0;
    }

    // One unit of work: an item of the walk, or, once the round's walk is
    // complete, one buffered hit handed to `visit` (front of the buffer, which
    // then shifts down).  Compositing a hit per call keeps a lane that ends
    // its round from holding the wavefront for K hits.  Returns true when the
    // ray is finished.
    // One step of the lane.  Walking lanes step a node every call; a leaf they
    // find waits (pend) for a surfel step, and so do buffered hits to
    // composite.  Surfel steps -- the record, its canonical crossing, then the
    // k-buffer insertion or the visitor -- run for the whole wavefront at
    // once, when enough of its active lanes wait for one (or all do),
    // so that block runs with many lanes (leaf tests postponed as in
    // speculative while-while traversal).  Returns true when the ray is
    // finished.  Every active lane of the wavefront calls it in the same step
    // (the decision is a ballot over them).
    template <class Visit>
    __device__ __forceinline__ bool advance(const SceneDev &S, Visit &visit)
    {
        if (ncomp == 0 && pend == kNone) {
            int leaf = kNone;
            if (step(S, leaf)) {  // the round's walk is complete
                const int m = cnt < K ? cnt : K;
                if (m == 0) return true;
                ncomp = m;
            } else if (leaf != kNone) {
                pend = -leaf - 1;
            }
        }
        const bool wl = pend != kNone, wc = ncomp > 0;
        bool want = wl || wc;
        int nwant, nact;
        bool all;
        if (kCompShare16 == 0) {
            nwant = __popcll(__ballot(want));
            nact = __popcll(__ballot(1));
            all = nwant == nact;
        } else {
            const int nl = __popcll(__ballot(wl)), nc = __popcll(__ballot(wc));
            nact = __popcll(__ballot(1));
            all = nl + nc == nact;
            const bool comp_ok = 16 * nc >= kCompShare16 * nact || all;
            want = wl || (wc && comp_ok);
            nwant = nl + (comp_ok ? nc : 0);
        }
        const bool few = kSiteShare8 ? 8 * nwant < kSiteShare8 * nact : 4 * nwant < kSurfelShare4 * nact;
        if (!want || (few && !all)) return false;
        const bool comp = ncomp > 0;
        const uint32_t sp = comp ? pos[0] : (uint32_t)pend;
        // One surfel site for leaf tests and composites: the record and its
        // canonical crossing are shared by both kinds of lanes.
        const float4 *r = S.rec + 4 * (size_t)sp;
        const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
        float den, tau, rho2;
        canon_geo(r0, r1, r2, r3, o, d, den, tau, rho2);
        if (!comp) {
            test_leaf(sp, den, tau, rho2, r0.w, r2.w);
            pend = kNone;
            return false;
        }
        const bool stop = visit(sp, (uint32_t)(key[0] & 0xffffffffu), __uint_as_float((uint32_t)(key[0] >> 32)), r0,
                                r1, r2, r3, rho2, o, d);
#ifdef GRT_STATS
        ++st_comps;
#endif
        last = key[0];  // the last composited hit (next_round resets it)
#pragma unroll
        for (int i = 0; i < K - 1; ++i) { key[i] = key[i + 1]; pos[i] = pos[i + 1]; }
        key[K - 1] = ~0ull;
        --ncomp;
        if (stop) return true;
        if (ncomp == 0) {
            if (cnt < K || deferred_empty()) return true;
            next_round(S);
        }
        return false;
    }

};

// The walker of the backward kernels (see kBwdCompShare16, kBwdSiteShare8).
template <int K>
using BwdWalker = Walker<K, kBwdLdsDepth, kBwdCompShare16, kBwdSiteShare8>;

// Upper end of a backward's re-traversal: the depth of the forward's last
// composited hit when it was saved (every hit the backward composites lies at
// or before it, and ties there come after the hit that ended the forward),
// with a margin that keeps node culling clear of rounding.
__device__ __forceinline__ float stop_bound(const float *stop_depth, int64_t r, float tmax)
{
    if (!stop_depth) return tmax;
    const float ts = stop_depth[r];
    return fminf(tmax, ts + 1e-6f * ts + 1e-6f);
}

// ---------------------------------------------------------------------------
// Persistent wavefronts with dynamic ray fetching.
//
// Rays 0..total-1 are split into 8 contiguous partitions, one per XCD (the
// hardware deals workgroups to XCDs round robin), each with its own counter;
// a wavefront claims chunks of kChunk consecutive rays from its XCD's
// partition, then from the others once that one is drained.  Lanes whose ray
// has finished take the next ray of the wavefront's chunk at once, so a
// wavefront never waits for its slowest ray.  Every wavefront leaves the loop
// once all partitions are drained and its lanes are idle.
//
// Job: bool begin(int64_t ray)  -- set up the ray; false if it needs no trace
//      (then it must already have written its result)
//      Walker<K, D> &walker(), Visit &visit(), void finish(int64_t ray),
//      void after_step() and void drain() -- run by every lane of the
//      wavefront after each step and before it leaves
// ---------------------------------------------------------------------------
constexpr int kParts = 8;
constexpr int kChunk = 64;

__host__ __device__ __forceinline__ int64_t part_begin(int64_t total, int q) { return total * q / kParts; }

#ifdef GRT_STATS
// Walk statistics of the instrumented build.  Per kernel kind (a Job with
// kStatSlot 0: the forward radiance trace, 1: the backward re-traversal;
// other jobs are not counted), sums over the rays each kind traced and over
// its wavefront steps; each TU holds its own copy (render kernels: render.hip).
enum { kStRays, kStNodes, kStLeaves, kStComps, kStRounds, kStRestarts, kStDeferred, kStSteps, kStActive, kNumWalkStats };
static __device__ unsigned long long g_walk_stats[2][kNumWalkStats];

template <class J, class = void>
struct StatSlot { static constexpr int value = -1; };
template <class J>
struct StatSlot<J, std::void_t<decltype(J::kStatSlot)>> { static constexpr int value = J::kStatSlot; };

// The lane's sums of a finished ray's walk counters.
template <class W>
__device__ __forceinline__ void walk_tally(uint32_t (&t)[kNumWalkStats], const W &w)
{
    ++t[kStRays];
    t[kStNodes] += w.st_nodes;
    t[kStLeaves] += w.st_leaves;
    t[kStComps] += w.st_comps;
    t[kStRounds] += w.st_rounds;
    t[kStRestarts] += w.st_lost;
    t[kStDeferred] += w.st_deferred;
}

// Adds the wavefront's sums to the kind's totals (all lanes, wavefront-uniform point).
template <int kSlot>
__device__ __forceinline__ void walk_flush(const uint32_t (&t)[kNumWalkStats])
{
    if constexpr (kSlot >= 0) {
#pragma unroll
        for (int i = 0; i < kNumWalkStats; ++i) {
            unsigned long long v = t[i];
            for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
            if ((threadIdx.x & 63) == 0) atomicAdd(&g_walk_stats[kSlot][i], v);
        }
    }
}
#endif

// stop: optional flag in host memory; once it reads non-zero, wavefronts
// claim no further chunks, finish the rays they hold and leave, so the claim
// counters then say exactly which rays were traced (a prefix of each
// partition).
template <int K, class Job>
__device__ __forceinline__ void run_persistent(Job &job, unsigned long long *counters, int64_t total,
                                               const int *stop = nullptr)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int part = blockIdx.x % kParts;
    int tried = 0;
    int64_t pool_next = 0, pool_end = 0;  // wavefront-uniform
    bool exhausted = false;               // wavefront-uniform
    bool active = false;
    int64_t ray = -1;
    using WalkerT = typename std::remove_reference<decltype(job.walker())>::type;
    constexpr int D = WalkerT::kDepth;
    __shared__ int lds_stacks[4][2][D][64];  // [wave][stack][slot][lane]
    int spill0[kStackCap], spill1[kStackCap];
    const int wave = (threadIdx.x >> 6) & 3;
    {
        auto &F = job.walker().F;
        F.lds = &lds_stacks[wave][0][0][lane];
        F.mem0 = spill0;
        F.mem1 = spill1;
        F.role = 0;
        F.walk.reset();
        F.def.reset();
    }
#ifdef GRT_STATS
    uint32_t tally[kNumWalkStats] = {};
#endif
    for (;;) {
        const uint64_t idle = __ballot(!active);
        if (idle && !exhausted) {
            if (pool_next >= pool_end) {
                // claim a chunk (leader lane), moving on to other partitions when drained
                for (;;) {
                    const int64_t pb = part_begin(total, part), pe = part_begin(total, part + 1);
                    unsigned long long got = 0;
                    int halt = 0;
                    const int leader = __ffsll((long long)idle) - 1;
                    if (lane == leader) {
                        if (stop) halt = __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        if (!halt) got = atomicAdd(&counters[part], (unsigned long long)kChunk);
                    }
                    if (__shfl(halt, leader, 64)) { exhausted = true; break; }
                    got = __shfl(got, leader, 64);
                    if (pb + (int64_t)got < pe) {
                        pool_next = pb + (int64_t)got;
                        pool_end = min(pe, pool_next + kChunk);
                        break;
                    }
                    if (++tried >= kParts) { exhausted = true; break; }
                    part = (part + 1) % kParts;
                }
            }
            if (!exhausted) {
                const int64_t avail = pool_end - pool_next;
                const int rank = __popcll(idle & lt);
                if (!active && rank < avail) {
                    ray = pool_next + rank;
                    active = job.begin(ray);
                }
                const int nidle = __popcll(idle);
                pool_next += (int64_t)(nidle < avail ? nidle : avail);
            }
        }
        const uint64_t busy = __ballot(active);
        if (!busy) {
            if (exhausted) {
#ifdef GRT_STATS
                walk_flush<StatSlot<Job>::value>(tally);
#endif
                job.drain();
                break;
            }
            continue;
        }
#ifdef GRT_STATS
        if (lane == 0) {
            ++tally[kStSteps];
            tally[kStActive] += (uint32_t)__popcll(busy);
        }
#endif
        if (active) {
            if (job.walker().advance(job.S, job.visit())) {
#ifdef GRT_STATS
                walk_tally(tally, job.walker());
#endif
                job.finish(ray);
                active = false;
            }
        }
        job.after_step();  // wavefront-uniform point
    }
}

}  // namespace grt
