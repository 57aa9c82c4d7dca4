// server.hip -- continuously batched relighting server over a resident scene.
//
// Relighting requests (a G-buffer, an environment map, a sample budget) are
// served by one scheduler thread that runs in short epochs.  Each epoch it
//   1. admits queued requests in arrival order while a slot and room in the
//      device pool are free: the request's G-buffer and environment are
//      uploaded, its sampling tables built and all its sample rays generated
//      on a copy stream, overlapping the trace;
//   2. hands the epoch's ray budget to running requests in order of deadline
//      (arrival plus a slack proportional to the request's size, so small
//      requests pass large ones and no request starves);
//   3. launches one persistent trace kernel over the rays of all requests of
//      the epoch together (the mix), then, for the requests that complete,
//      the per-pixel reduction and the copy back.
// Two epochs are in flight on two streams: the next epoch's waves take the
// CUs that the current epoch's tail leaves idle.
// Every sample's random counter carries its request id and every pixel is
// summed in sample order, so a request's image is the same alone or in any
// mix.  Scene and LBVH stay resident; each epoch launch ends when its rays
// are done, so no kernel outlives the epoch.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "grt_render.h"

namespace grt {
// defined in api.hip (the scene handle is opaque here)
int scene_dev_of(const grt_scene *scene, SceneDev *out, const char **why);
int set_error(int code, const char *msg);

struct ServeChunk {
    int slot;       // job slot in the epoch's job table
    int pad;
    int64_t begin;  // first ray of the job in this chunk
    int64_t offset; // position of the chunk in the epoch's ray range
};

struct ServeEpoch {
    const RenderArgs *jobs;
    const ServeChunk *chunks;
    int nchunks;
    int64_t total;
    unsigned long long *counters;
    const int *stop;  // preemption flag (host memory) or null
    SceneDev S;
};

// A co-traced epoch: the joint order (entry g = member << kJointShift | the
// member's sample index, mslot[member] its job slot) and the epoch's own
// copies of its rays in that order -- ray records, origins, and what the
// trace writes back (contributions; relighting: the query's record words and
// averaged normals) -- so that the trace runs the uniform-argument kernel of
// a single request over them.
constexpr int kMaxMembers = 16;
constexpr int kJointShift = 27;
struct JointEpoch {
    const RenderArgs *jobs;
    int mslot[kMaxMembers];
    const uint32_t *joint;
    int64_t n;
    float4 *rays;     // [3n]
    float *x;         // [3n]
    float4 *contrib;  // [n]
    float *nrm;       // [3][n] (relighting: x, y, z planes)
    int relight;
};

// Gather the joint order's ray records and origins.
__global__ void k_joint_gather(JointEpoch je)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= je.n) return;
    const uint32_t v = je.joint[g];
    const RenderArgs &a = je.jobs[je.mslot[v >> kJointShift]];
    const int64_t r = (int64_t)(v & ((1u << kJointShift) - 1u));
    const int64_t p = r / (a.nc + a.ng + a.ne);
    je.rays[3 * g] = a.rays[3 * r];
    je.rays[3 * g + 1] = a.rays[3 * r + 1];
    je.rays[3 * g + 2] = a.rays[3 * r + 2];
    je.x[3 * g] = a.x[3 * p];
    je.x[3 * g + 1] = a.x[3 * p + 1];
    je.x[3 * g + 2] = a.x[3 * p + 2];
}

// Scatter what the trace wrote back to each member's buffers.
__global__ void k_joint_scatter(JointEpoch je)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= je.n) return;
    const uint32_t v = je.joint[g];
    const RenderArgs &a = je.jobs[je.mslot[v >> kJointShift]];
    const int64_t r = (int64_t)(v & ((1u << kJointShift) - 1u));
    a.contrib[r] = je.contrib[g];
    if (je.relight) {
        a.rays[3 * r + 2] = je.rays[3 * g + 2];  // the query's roughness and metallic (z, w)
        a.rl_nx[r] = je.nrm[g];
        a.rl_ny[r] = je.nrm[je.n + g];
        a.rl_nz[r] = je.nrm[2 * je.n + g];
    }
}

__device__ __forceinline__ int find_chunk(const ServeChunk *chunks, int nchunks, int64_t g)
{
    int lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunks[mid].offset <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Trace: ShadeTrace<K, false, true> (the radiance trace of Eq. mis) or
// RelightTrace<K, true> (the attribute query of relighting, Eq.
// trace_attr), both taking their request's tables with each ray; an epoch
// holds requests of one kind.
template <int K, class Trace>
struct ServeJob {
    const ServeEpoch &e;
    SceneDev S;
    Trace t;
    const RenderArgs *a;
    int64_t r;

    __device__ ServeJob(const ServeEpoch &e_) : e(e_), S(e_.S), a(nullptr), r(0) {}
    __device__ __forceinline__ Walker<K> &walker() { return t.w; }
    __device__ __forceinline__ decltype(t.v) &visit() { return t.v; }

    __device__ __forceinline__ bool begin(int64_t g)
    {
        const ServeChunk ch = e.chunks[find_chunk(e.chunks, e.nchunks, g)];
        a = &e.jobs[ch.slot];
        r = ch.begin + (g - ch.offset);
        if (a->order) r = (int64_t)a->order[r];
        return t.begin(*a, S, r);
    }

    __device__ __forceinline__ void finish(int64_t) { t.finish(*a, r); }
    __device__ __forceinline__ void after_step() {}
    __device__ __forceinline__ void drain() {}
};

// kStop: the epoch may be stopped (e.stop set).  Without it the persistent
// loop carries no stop test, as a direct render's does.
template <int K, class Trace, bool kStop>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY k_serve(ServeEpoch e)
{
    ServeJob<K, Trace> job(e);
    if (kStop)
        run_persistent<K>(job, e.counters, e.total, e.stop);
    else
        run_persistent<K>(job, e.counters, e.total);
}

template <int K, class Trace, bool kStop>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_serve_w3(ServeEpoch e)
{
    ServeJob<K, Trace> job(e);
    if (kStop)
        run_persistent<K>(job, e.counters, e.total, e.stop);
    else
        run_persistent<K>(job, e.counters, e.total);
}

// An epoch holding rays of one request only: its arguments travel by value
// (uniform across the grid, as in a direct render); its rays are one range
// of the request's sample order, or a few once a stopped epoch handed some
// back (then each ray finds its range in the chunk table).
template <int K, class Trace, bool kPlain>
struct ServeOneJob {
    const RenderArgs &a;
    SceneDev S;
    Trace t;
    const ServeChunk *chunks;
    int nchunks;
    int64_t r0;

    int64_t r;

    __device__ ServeOneJob(const RenderArgs &a_, const ServeChunk *c, int nc, int64_t r0_)
        : a(a_), S(a_.S), chunks(c), nchunks(nc), r0(r0_), r(0)
    {
        bind_trace(t, a, S);
    }
    __device__ __forceinline__ Walker<K> &walker() { return t.w; }
    __device__ __forceinline__ decltype(t.v) &visit() { return t.v; }
    __device__ __forceinline__ bool begin(int64_t g)
    {
        int64_t q = r0 + g;
        if (!kPlain && nchunks > 1) {
            const ServeChunk ch = chunks[find_chunk(chunks, nchunks, g)];
            q = ch.begin + (g - ch.offset);
        }
        r = a.order ? (int64_t)a.order[q] : q;
        return t.begin(a, S, r);
    }
    __device__ __forceinline__ void finish(int64_t) { t.finish(a, r); }
    __device__ __forceinline__ void after_step() {}
    __device__ __forceinline__ void drain() {}
};

// kPlain: one range of rays and no stop flag (every epoch while preemption
// is off, and every relighting epoch), so the kernel is the direct render's
// loop with the request's arguments; otherwise it handles a range table and
// a stop flag.
template <int K, class Trace, bool kPlain>
__global__ void __launch_bounds__(256) GRT_OCCUPANCY
    k_serve_one(RenderArgs a, const ServeChunk *chunks, int nchunks, int64_t r0, int64_t n,
                unsigned long long *counters, const int *stop)
{
    ServeOneJob<K, Trace, kPlain> job(a, chunks, nchunks, r0);
    if (kPlain)
        run_persistent<K>(job, counters, n);
    else
        run_persistent<K>(job, counters, n, stop);
}

// K = 12 held to 3 wavefronts per SIMD, as the direct render's forward
template <int K, class Trace, bool kPlain>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
    k_serve_one_w3(RenderArgs a, const ServeChunk *chunks, int nchunks, int64_t r0, int64_t n,
                   unsigned long long *counters, const int *stop)
{
    ServeOneJob<K, Trace, kPlain> job(a, chunks, nchunks, r0);
    if (kPlain)
        run_persistent<K>(job, counters, n);
    else
        run_persistent<K>(job, counters, n, stop);
}

// counters/total: the claim counters of a preemptible epoch that held the
// request's last rays; if the epoch was stopped before claiming them all, the
// request is not complete and the reduction does nothing.
__global__ void k_serve_reduce(const RenderArgs *a, int64_t npix, const unsigned long long *counters, int64_t total)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    if (counters)
        for (int q = 0; q < kParts; ++q)
            if ((int64_t)counters[q] < part_begin(total, q + 1) - part_begin(total, q)) return;
    reduce_pixel(p, a->nc + a->ng + a->ne, a->contrib, a->out);
}

// K = 12 held to 3 wavefronts per SIMD, as in a direct render
template <int K, class Trace, bool kStop>
static hipError_t go_serve_as(const ServeEpoch &e, int num_cu, hipStream_t st)
{
    if constexpr (K == 12) {
        const int nb = persistent_blocks(k_serve_w3<K, Trace, kStop>, num_cu, e.total);
        hipLaunchKernelGGL((k_serve_w3<K, Trace, kStop>), dim3(nb), dim3(256), 0, st, e);
    } else {
        const int nb = persistent_blocks(k_serve<K, Trace, kStop>, num_cu, e.total);
        hipLaunchKernelGGL((k_serve<K, Trace, kStop>), dim3(nb), dim3(256), 0, st, e);
    }
    return hipGetLastError();
}

template <int K, class Trace, bool kPlain>
static hipError_t go_serve_one_as(const RenderArgs &a, const ServeEpoch &e, int64_t r0, int num_cu, hipStream_t st)
{
    if constexpr (K == 12) {
        const int nb = persistent_blocks(k_serve_one_w3<K, Trace, kPlain>, num_cu, e.total);
        hipLaunchKernelGGL((k_serve_one_w3<K, Trace, kPlain>), dim3(nb), dim3(256), 0, st, a, e.chunks, e.nchunks,
                           r0, e.total, e.counters, e.stop);
    } else {
        const int nb = persistent_blocks(k_serve_one<K, Trace, kPlain>, num_cu, e.total);
        hipLaunchKernelGGL((k_serve_one<K, Trace, kPlain>), dim3(nb), dim3(256), 0, st, a, e.chunks, e.nchunks, r0,
                           e.total, e.counters, e.stop);
    }
    return hipGetLastError();
}

// Radiance epochs may be stopped; relighting epochs never are.  A mixed
// epoch's lanes trace for different requests, so its relighting query takes
// its tables with each ray.
template <int K>
static hipError_t go_relight_epoch(const ServeEpoch &e, const RenderArgs *one, int64_t r0, int num_cu,
                                   hipStream_t st)
{
    return one ? go_serve_one_as<K, RelightTrace<K>, true>(*one, e, r0, num_cu, st)
               : go_serve_as<K, RelightTrace<K, true>, false>(e, num_cu, st);
}

template <int K>
static hipError_t go_epoch(const ServeEpoch &e, const RenderArgs *one, int64_t r0, bool relight, int num_cu,
                           hipStream_t st)
{
    if (relight) return go_relight_epoch<K>(e, one, r0, num_cu, st);
    if (one)
        return (!e.stop && e.nchunks <= 1) ? go_serve_one_as<K, ShadeTrace<K>, true>(*one, e, r0, num_cu, st)
                                           : go_serve_one_as<K, ShadeTrace<K>, false>(*one, e, r0, num_cu, st);
    return e.stop ? go_serve_as<K, ShadeTrace<K, false, true>, true>(e, num_cu, st)
                  : go_serve_as<K, ShadeTrace<K, false, true>, false>(e, num_cu, st);
}

// one: the request when every chunk of the epoch is of that one request, else
// null; r0: the first ray of chunk 0; relight: the epoch's requests are
// relighting requests (the attribute query)
static hipError_t launch_epoch(const ServeEpoch &e, const RenderArgs *one, int64_t r0, bool relight, int k, int num_cu,
                               hipStream_t st)
{
    const hipError_t err = launch_zero_counters(e.counters, st);
    if (err != hipSuccess) return err;
    switch (k) {
    case 4: return go_epoch<4>(e, one, r0, relight, num_cu, st);
    case 8: return go_epoch<8>(e, one, r0, relight, num_cu, st);
    case 12: return go_epoch<12>(e, one, r0, relight, num_cu, st);
    case 16: return go_epoch<16>(e, one, r0, relight, num_cu, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
using Clock = std::chrono::steady_clock;

enum JobState { kQueued = 0, kUploading = 1, kRunning = 2, kDone = 3 };

struct ServerJob {
    uint64_t id = 0;
    grt_job spec{};
    int state = kQueued;
    int status = GRT_OK;  // error code once failed or cancelled
    bool cancel = false;
    bool pooled = false;  // holds [off, off + bytes) of the pool
    size_t bytes = 0, off = 0;
    int slot = -1;
    RenderArgs args{};
    EnvWS env{};
    RenderWS sort{};  // sort keys/values and histogram (counters, rays, contrib unused)
    int64_t npix = 0, total = 0;
    bool relight = false;  // a relighting request (Eq. relight_splitsum), else radiance (Eq. mis)
    bool out_device = false;  // out_rgb is device memory (else host)
    // rays not yet handed to an epoch: ranges of the request's sample order
    // (one range, until a stopped epoch hands back what it did not claim)
    std::deque<std::pair<int64_t, int64_t>> left;
    int64_t nleft = 0;
    // with preemption on: rays other requests may still run ahead of it once
    // it has started; at zero it goes first and its epochs are not stopped
    int64_t passable = 0;
    bool started = false;
    int inflight = 0;      // epochs in flight that hold rays of this job
    double deadline = 0;   // scheduling key
    hipEvent_t ready = nullptr;
    double t_submit = 0, t_start = -1, t_done = -1;
};

// First-fit allocator over the device pool (offsets, 256-byte granules).
struct PoolAlloc {
    std::map<size_t, size_t> free_;  // offset -> size
    void init(size_t bytes) { free_.clear(); free_[0] = bytes; }
    bool alloc(size_t bytes, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// bytes a job needs in the pool and where each array goes
static size_t carve_job(ServerJob &j, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const int spp = j.spec.n_cos + j.spec.n_ggx + j.spec.n_env;
    const size_t npix = (size_t)j.spec.H * (size_t)j.spec.W, nray = npix * (size_t)spp;
    RenderArgs &a = j.args;
    a.x = (const float *)take(12 * npix);
    a.n = (const float *)take(12 * npix);
    a.wo = (const float *)take(12 * npix);
    a.alb = (const float *)take(12 * npix);
    a.rough = (const float *)take(4 * npix);
    a.metal = (const float *)take(4 * npix);
    a.valid = (const uint8_t *)take(npix);
    a.E.rgb = (const float *)take(12 * (size_t)j.spec.env_H * j.spec.env_W);
    char *envws = take(carve_env(nullptr, j.spec.env_H, j.spec.env_W).bytes);
    j.env = carve_env(envws, j.spec.env_H, j.spec.env_W);
    a.rays = (float4 *)take(48 * nray);
    a.contrib = (float4 *)take(16 * nray);
    a.out = (float *)take(12 * npix);
    if (j.spec.relight) {  // where the attribute query parks each sample's averaged normal
        a.rl_nx = (float *)take(4 * nray);
        a.rl_ny = (float *)take(4 * nray);
        a.rl_nz = (float *)take(4 * nray);
    }
    // coherent traversal order of the request's samples, and its sort scratch
    j.sort.k0 = (uint32_t *)take(4 * nray);
    j.sort.v0 = (uint32_t *)take(4 * nray);
    j.sort.k1 = (uint32_t *)take(4 * nray);
    j.sort.v1 = (uint32_t *)take(4 * nray);
    j.sort.hist = (uint32_t *)take(4 * sort_hist_words((int64_t)nray));
    a.order = base ? j.sort.v1 : nullptr;
    return off;
}

// One of the two epochs that can be in flight: its tables, stream and the
// jobs it touches.
struct EpochSlot {
    RenderArgs *d_jobs = nullptr, *h_jobs = nullptr;
    ServeChunk *d_chunks = nullptr, *h_chunks = nullptr;
    unsigned long long *counters = nullptr;
    unsigned long long *h_counters = nullptr;  // the claim counters, copied back
    int *stop_h = nullptr;                     // preemption flag (host memory) ...
    int *stop_d = nullptr;                     // ... and its device address
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool inflight = false;
    bool preemptible = false;  // one request's rays: may be stopped early
    bool relight = false;      // an epoch of relighting requests
    bool stopped = false;      // the stop flag was raised
    int nch = 0;
    int64_t rays = 0;       // rays of the epoch in flight
    double t_launch = 0.0;  // when it was launched (server clock)
    std::vector<uint64_t> members, finishing;
    size_t joint_off = 0, joint_bytes = 0;  // a co-traced epoch's sort buffers in the pool (0: none)
};

}  // namespace grt

using grt::ServerJob;
using grt::kQueued;
using grt::kUploading;
using grt::kRunning;
using grt::kDone;

struct grt_server {
    grt_ctx *ctx = nullptr;
    grt::SceneDev S{};
    grt_server_opts opts{};
    double slack = 0;
    double share = 0;  // preempt_share in effect
    char *pool = nullptr;
    grt::PoolAlloc alloc;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    int error = GRT_OK;
    std::deque<uint64_t> pending;
    std::map<uint64_t, ServerJob> jobs;
    std::deque<uint64_t> history;  // finished requests, oldest first (bounded)
    std::vector<uint64_t> resident;  // uploading or running, in admission order
    std::vector<int> free_slots;
    hipStream_t copy = nullptr;
    unsigned long long *copy_counters = nullptr;  // ray fetch of G-buffer traces on the copy stream
    float *lut = nullptr;                          // the shared DFG table (workspace)
    grt::EpochSlot ep[2];
    int chunk_cap = 0;  // chunk table entries per epoch
    double rate = 5e7;  // traced rays per second, running estimate (launch gate)
    uint64_t next_id = 1;
    grt::Clock::time_point t0;
    // statistics
    uint64_t epochs = 0;
    uint64_t stopped = 0;  // epochs stopped before claiming all their rays
    int64_t rays_done = 0;

    double now() const { return std::chrono::duration<double>(grt::Clock::now() - t0).count(); }
};

namespace {

int sfail(int code, const char *msg) { return grt::set_error(code, msg); }

// Finished requests the server keeps for poll, wait and job_times.
constexpr size_t kHistory = 65536;

size_t job_bytes(const grt_job &spec)
{
    ServerJob j;
    j.spec = spec;
    return grt::carve_job(j, nullptr);
}

int check_job(const grt_job *j)
{
    if (!j) return GRT_ERR_INVALID;
    if (j->H <= 0 || j->W <= 0 || (int64_t)j->H * j->W > (1 << 26)) return GRT_ERR_INVALID;
    if (j->env_H <= 0 || j->env_W <= 0 || (int64_t)j->env_H * j->env_W > (1 << 24)) return GRT_ERR_INVALID;
    const int spp = j->n_cos + j->n_ggx + j->n_env;
    if (j->n_cos < 0 || j->n_ggx < 0 || j->n_env < 0 || spp <= 0 || spp > 4096) return GRT_ERR_INVALID;
    if (!j->env_rgb || !j->out_rgb) return GRT_ERR_INVALID;
    if (j->camera_request) {
        grt::PinholeDev c;
        if (!(j->min_opacity > 0.0f && j->min_opacity <= 1.0f)) return GRT_ERR_INVALID;
        if (!grt::make_pinhole(j->camera.eye, j->camera.target, j->camera.up, j->camera.vfov_deg, j->H, j->W, c))
            return GRT_ERR_INVALID;
    } else if (!j->x || !j->n || !j->wo || !j->albedo || !j->rough || !j->metal || !j->valid) {
        return GRT_ERR_INVALID;
    }
    return GRT_OK;
}

// The G-buffer of a camera request, traced on the copy stream into the
// request's G-buffer area (as grt_camera_rays + grt_trace_gbuffer).  The
// camera rays borrow the request's ray-record area (24 of its >= 48 bytes per
// pixel) and the depth and colour maps its contribution area (16 of >= 16
// bytes per pixel); both are written only later, on the same stream.
hipError_t trace_request_gbuffer(grt_server *s, ServerJob &j)
{
    const grt_job &q = j.spec;
    const int64_t npix = (int64_t)q.H * q.W;
    grt::RenderArgs &a = j.args;
    grt::PinholeDev c;
    if (!grt::make_pinhole(q.camera.eye, q.camera.target, q.camera.up, q.camera.vfov_deg, q.H, q.W, c))
        return hipErrorInvalidValue;  // checked at submission
    float *o = reinterpret_cast<float *>(a.rays), *d = o + 3 * npix;
    hipError_t e = grt::launch_camera_rays(c, q.H, q.W, o, d, s->copy);
    if (e != hipSuccess) return e;
    grt::TraceGBufArgs b;
    memset(&b, 0, sizeof(b));
    b.f.S = s->S;
    b.f.n = npix;
    b.f.o = o;
    b.f.d = d;
    b.f.tmin = 0.0f;
    b.f.tmax = INFINITY;
    b.f.tcut = s->opts.t_cut;
    b.f.counters = s->copy_counters;
    b.albedo = s->opts.attrs.albedo;
    b.rough = s->opts.attrs.rough;
    b.metal = s->opts.attrs.metal;
    b.min_opacity = q.min_opacity;
    b.x = const_cast<float *>(a.x);
    b.n = const_cast<float *>(a.n);
    b.wo = const_cast<float *>(a.wo);
    b.out_albedo = const_cast<float *>(a.alb);
    b.out_rough = const_cast<float *>(a.rough);
    b.out_metal = const_cast<float *>(a.metal);
    b.valid = const_cast<uint8_t *>(a.valid);
    b.depth = reinterpret_cast<float *>(a.contrib);
    b.rgb = b.depth + npix;
    return grt::launch_trace_gbuffer(b, s->opts.k, s->ctx->num_cu, s->copy);
}

// The copy kind for a host-or-device pointer: a host source or destination
// takes the DMA engines (H2D / D2H), not a copy kernel that would wait for
// compute units behind a running epoch.
static bool on_device(const void *p)
{
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // plain host memory the runtime does not know
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// Upload a job's inputs and build its tables on the copy stream.
hipError_t upload(grt_server *s, ServerJob &j)
{
    hipError_t e;
    const size_t npix = (size_t)j.spec.H * j.spec.W;
    const grt_job &q = j.spec;
    grt::RenderArgs &a = j.args;
    struct Cp {
        const void *dst;
        const void *src;
        size_t n;
    } cps[] = {{a.E.rgb, q.env_rgb, 12 * (size_t)q.env_H * q.env_W}, {a.x, q.x, 12 * npix},
               {a.n, q.n, 12 * npix},         {a.wo, q.wo, 12 * npix},    {a.alb, q.albedo, 12 * npix},
               {a.rough, q.rough, 4 * npix},  {a.metal, q.metal, 4 * npix}, {a.valid, q.valid, npix}};
    // a camera request uploads only its environment and traces its G-buffer
    const int ncp = q.camera_request ? 1 : (int)(sizeof(cps) / sizeof(cps[0]));
    for (int i = 0; i < ncp; ++i)
        if ((e = hipMemcpyAsync((void *)cps[i].dst, cps[i].src, cps[i].n,
                                on_device(cps[i].src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                s->copy)) !=
            hipSuccess)
            return e;
    if (q.camera_request && (e = trace_request_gbuffer(s, j)) != hipSuccess) return e;
    if ((e = grt::launch_env_build(a.E.rgb, q.env_H, q.env_W, j.env, s->copy)) != hipSuccess) return e;
    // relighting: the prefiltered environment and the DFG table (Eq. relight_splitsum)
    if (j.relight && (e = grt::launch_env_prefilter(a.E.rgb, q.env_H, q.env_W, j.env, s->copy, false)) != hipSuccess)
        return e;
    // every sample's ray record up front, so epochs only trace, and the
    // samples' coherent traversal order
    if ((e = grt::launch_render_gen(a, s->copy)) != hipSuccess) return e;
    if ((e = grt::launch_ray_order(a, j.sort, s->copy)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&j.ready, hipEventDisableTiming)) != hipSuccess) return e;
    return hipEventRecord(j.ready, s->copy);
}

void setup_args(grt_server *s, ServerJob &j)
{
    grt::RenderArgs &a = j.args;
    a.S = s->S;
    if (a.S.n < 2) a.order = nullptr;  // no hierarchy to order by: index order
    a.E.H = j.spec.env_H;
    a.E.W = j.spec.env_W;
    a.E.marg = j.env.marg;
    a.E.cond = j.env.cond;
    a.H = j.spec.H;
    a.W = j.spec.W;
    a.nc = j.spec.n_cos;
    a.ng = j.spec.n_ggx;
    a.ne = j.spec.n_env;
    a.seed = j.spec.seed;
    a.job = j.spec.job;
    a.tmin = s->opts.t_min;
    a.tcut = s->opts.t_cut;
    a.saved = nullptr;
    a.saved_t = nullptr;
    a.dump = nullptr;
    a.grad = nullptr;
    a.hits = nullptr;
    if (j.relight) {
        a.E.Ed = j.env.Ed;
        a.E.Es = j.env.Es;
        a.E.lut = s->lut;
        a.sa_albedo = s->opts.attrs.albedo;
        a.sa_rough = s->opts.attrs.rough;
        a.sa_metal = s->opts.attrs.metal;
    }
}

void finish_job(grt_server *s, ServerJob &j, int status)
{
    if (j.state == kDone) return;
    if (j.ready) { (void)hipEventDestroy(j.ready); j.ready = nullptr; }
    if (j.pooled) s->alloc.release(j.off, j.bytes);
    j.pooled = false;
    if (j.slot >= 0) s->free_slots.push_back(j.slot);
    j.slot = -1;
    j.state = kDone;
    j.status = status;
    j.t_done = s->now();
    // remember a bounded number of finished requests (j itself is the newest)
    s->history.push_back(j.id);
    while (s->history.size() > kHistory) {
        s->jobs.erase(s->history.front());
        s->history.pop_front();
    }
}

// Called with no epoch in flight (or after a device error, when nothing
// more will be waited for).
void fail_all(grt_server *s, int status)
{
    for (uint64_t id : s->resident) finish_job(s, s->jobs[id], status);
    s->resident.clear();
    for (uint64_t id : s->pending) finish_job(s, s->jobs[id], status);
    s->pending.clear();
}

void device_failed(grt_server *s)
{
    s->error = GRT_ERR_DEVICE;
    fail_all(s, GRT_ERR_DEVICE);
    s->cv.notify_all();
}

// Admit queued jobs in arrival order while a slot and pool room are free.
void admit(grt_server *s, std::vector<uint64_t> &to_upload)
{
    while (!s->pending.empty() && !s->free_slots.empty()) {
        ServerJob &j = s->jobs[s->pending.front()];
        size_t off;
        if (!s->alloc.alloc(j.bytes, off)) break;
        j.off = off;
        j.pooled = true;
        j.slot = s->free_slots.back();
        s->free_slots.pop_back();
        grt::carve_job(j, s->pool + off);
        setup_args(s, j);
        j.state = kUploading;
        s->pending.pop_front();
        s->resident.push_back(j.id);
        to_upload.push_back(j.id);
    }
}

// A stopped epoch has ended: the rays it did not claim (a suffix of each of
// its partitions) go back, in order, to the front of its request's ranges,
// and the request is not finishing after all.
void give_back(grt_server *s, grt::EpochSlot &E)
{
    ServerJob &j = s->jobs[E.members[0]];
    std::vector<std::pair<int64_t, int64_t>> back;
    for (int q = 0; q < grt::kParts; ++q) {
        const int64_t pb = grt::part_begin(E.rays, q), pe = grt::part_begin(E.rays, q + 1);
        const int64_t a = pb + std::min((int64_t)E.h_counters[q], pe - pb);
        for (int c = 0; c < E.nch && a < pe; ++c) {
            const int64_t co = E.h_chunks[c].offset, ce = c + 1 < E.nch ? E.h_chunks[c + 1].offset : E.rays;
            const int64_t lo = std::max(a, co), hi = std::min(pe, ce);
            if (lo >= hi) continue;
            const int64_t b0 = E.h_chunks[c].begin + (lo - co), b1 = E.h_chunks[c].begin + (hi - co);
            if (!back.empty() && back.back().second == b0) back.back().second = b1;
            else back.push_back({b0, b1});
        }
    }
    if (back.empty()) return;
    int64_t n = 0;
    for (auto it = back.rbegin(); it != back.rend(); ++it) {
        if (!j.left.empty() && j.left.front().first == it->second) j.left.front().first = it->first;
        else j.left.push_front(*it);
        n += it->second - it->first;
    }
    j.nleft += n;
    s->rays_done -= n;
    ++s->stopped;
    E.finishing.clear();
}

// An epoch has completed on the device: its finishing jobs are done,
// cancelled jobs with no epoch left in flight are dropped.
void retire(grt_server *s, grt::EpochSlot &E)
{
    if (E.inflight && E.stopped) give_back(s, E);
    if (E.inflight && !E.stopped && E.rays >= (1 << 20)) {
        const double dt = s->now() - E.t_launch;
        if (dt > 1e-4) s->rate = 0.7 * s->rate + 0.3 * (double)E.rays / dt;
    }
    for (uint64_t id : E.members) --s->jobs[id].inflight;
    for (uint64_t id : E.finishing) {
        ServerJob &j = s->jobs[id];
        if (!j.cancel) finish_job(s, j, GRT_OK);
    }
    if (E.joint_bytes) s->alloc.release(E.joint_off, E.joint_bytes);
    E.joint_bytes = 0;
    E.members.clear();
    E.finishing.clear();
    E.inflight = false;
}

// Drop cancelled jobs that no epoch references; promote uploaded jobs.
void sweep(grt_server *s)
{
    std::vector<uint64_t> keep;
    for (uint64_t id : s->resident) {
        ServerJob &j = s->jobs[id];
        if (j.state == kDone) continue;
        if (j.cancel && j.inflight == 0) {
            if (j.ready) (void)hipEventSynchronize(j.ready);
            finish_job(s, j, GRT_ERR_CANCELLED);
            continue;
        }
        if (j.state == kUploading && hipEventQuery(j.ready) == hipSuccess) {
            j.state = kRunning;
            j.t_start = s->now();
        }
        keep.push_back(id);
    }
    s->resident.swap(keep);
}

// Requests are batched into one epoch only while it stays within this many
// rays.  A lone launch of a few hundred thousand rays is bound by its slowest
// rays; on a stream of 256x256 requests at 4 or 8 spp, epochs of up to 4M
// rays traced 59 Mrays/s, 1M-ray epochs 43, one launch per request 26.
#ifndef GRT_SERVE_FILL_RAYS
#define GRT_SERVE_FILL_RAYS (1 << 22)
#endif
constexpr int64_t kFillRays = GRT_SERVE_FILL_RAYS;
// A single-request epoch of at least this many rays can be stopped when a
// request with an earlier deadline arrives, unless it is estimated to end
// within kStopSeconds anyway.
constexpr int64_t kPreemptRays = 1 << 21;
constexpr double kStopSeconds = 0.015;
// Launch gate: the estimated time left of the epoch in flight below which the
// next epoch starts, and the share of its remaining rays below which a next
// epoch counts as small and starts at once.  Both are off: an epoch started
// while another is in flight takes the CUs as the other's waves leave, so the
// other's shading and per-pixel sum, queued behind it, wait for it to end.
// Starting a large epoch in the tail of another measured slower on
// relighting bursts (38.4 s against 38.0 s for 220 requests: the two ray
// streams share the caches), and letting small epochs pass made the
// replay's tail latencies vary by 10% from run to run and rise on average.
#ifndef GRT_SERVE_TAIL_S
#define GRT_SERVE_TAIL_S 0.0
#endif
#ifndef GRT_SERVE_SMALL_SHARE
#define GRT_SERVE_SMALL_SHARE 0.0
#endif
constexpr double kTailSeconds = GRT_SERVE_TAIL_S;
constexpr double kSmallShare = GRT_SERVE_SMALL_SHARE;

// Requests that share a G-buffer: the same arrays of the same size (a
// camera request's G-buffer is the server's own, never shared).
static bool same_gbuffer(const ServerJob &a, const ServerJob &b)
{
    const grt_job &p = a.spec, &q = b.spec;
    return !p.camera_request && !q.camera_request && p.H == q.H && p.W == q.W && p.x == q.x && p.n == q.n &&
           p.wo == q.wo && p.albedo == q.albedo && p.rough == q.rough && p.metal == q.metal && p.valid == q.valid;
}

// Not started: every ray still to hand out, in one range (and few enough to
// index in a joint order entry).
static bool whole(const ServerJob &j)
{
    return !j.started && j.inflight == 0 && j.nleft == j.total && j.left.size() == 1 &&
           j.total < ((int64_t)1 << grt::kJointShift);
}

// Co-tracing: the head request and the waiting requests of its kind that
// share its G-buffer, traced in one epoch in one joint coherent order (the
// samples of all of them sorted together by direction bin, then origin
// cell), so that a batch of requests of a few samples per pixel each walks
// the scene as coherently as one request of their summed samples.  The
// samples are gathered into the epoch's own buffers in that order and traced
// by the single-request kernel (uniform arguments: the mixed kernel, which
// finds each ray's request per lane, holds more registers), then the results
// are scattered back.  False (nothing launched) when fewer than two requests
// qualify or the epoch's buffers do not fit the pool.
// k of an epoch's trace: relighting epochs take k_relight when it is set
static int epoch_k(const grt_server *s, bool relight)
{
    return relight && s->opts.k_relight ? s->opts.k_relight : s->opts.k;
}

static bool launch_cotrace(grt_server *s, grt::EpochSlot &E, grt::EpochSlot &other,
                           const std::vector<ServerJob *> &run, int64_t budget, hipError_t &err)
{
    if (!s->opts.co_trace || run.empty() || !whole(*run[0])) return false;
    // at most 2^26 samples per co-traced epoch: its buffers take 104 bytes a sample
    const int64_t cap = std::min(budget, (int64_t)1 << 26);
    std::vector<ServerJob *> mem{run[0]};
    int64_t n = run[0]->total;
    for (size_t i = 1; i < run.size() && (int)mem.size() < grt::kMaxMembers; ++i) {
        ServerJob *j = run[i];
        if (whole(*j) && same_gbuffer(*j, *run[0]) && n + j->total <= cap) {
            mem.push_back(j);
            n += j->total;
        }
    }
    if (mem.size() < 2) return false;
    const bool relight = mem[0]->relight;
    const size_t q4 = grt::align256(4 * (size_t)n), q12 = grt::align256(12 * (size_t)n);
    const size_t bytes = 4 * q4 + grt::align256(4 * grt::sort_hist_words(n)) + grt::align256(48 * (size_t)n) + q12 +
                         grt::align256(16 * (size_t)n) + (relight ? q12 : 0);
    size_t off = 0;
    if (!s->alloc.alloc(bytes, off)) return false;
    char *p = s->pool + off;
    auto take = [&p](size_t b) { char *r = p; p += b; return r; };
    uint32_t *k0 = (uint32_t *)take(q4), *v0 = (uint32_t *)take(q4), *k1 = (uint32_t *)take(q4),
             *v1 = (uint32_t *)take(q4);
    uint32_t *hist = (uint32_t *)take(grt::align256(4 * grt::sort_hist_words(n)));
    grt::JointEpoch je{};
    je.rays = (float4 *)take(grt::align256(48 * (size_t)n));
    je.x = (float *)take(q12);
    je.contrib = (float4 *)take(grt::align256(16 * (size_t)n));
    je.nrm = relight ? (float *)take(q12) : nullptr;
    je.jobs = E.d_jobs;
    je.joint = v1;
    je.n = n;
    je.relight = relight ? 1 : 0;
    for (size_t m = 0; m < mem.size(); ++m) {
        ServerJob *j = mem[m];
        E.h_jobs[j->slot] = j->args;
        je.mslot[m] = j->slot;
        j->nleft = 0;
        j->left.clear();
        ++j->inflight;
        j->started = true;
        E.members.push_back(j->id);
        E.finishing.push_back(j->id);
    }
    for (ServerJob *j : run)
        if (j->started && j->nleft > 0 && std::find(E.members.begin(), E.members.end(), j->id) == E.members.end())
            j->passable -= n;
    E.relight = relight;
    E.preemptible = false;
    E.stopped = false;
    E.nch = 0;
    E.joint_off = off;
    E.joint_bytes = bytes;
    __atomic_store_n(E.stop_h, 0, __ATOMIC_RELEASE);
    // the trace sees one request: the members' shared G-buffer has become a
    // per-sample origin array, one sample per "pixel"
    grt::RenderArgs J = mem[0]->args;
    J.H = 1;
    J.W = (int)n;
    J.nc = 1;
    J.ng = 0;
    J.ne = 0;
    J.x = je.x;
    J.rays = je.rays;
    J.contrib = je.contrib;
    J.order = nullptr;
    J.out = nullptr;
    J.saved = nullptr;
    J.saved_t = nullptr;
    J.dump = nullptr;
    J.hits = nullptr;
    if (relight) {
        J.rl_nx = je.nrm;
        J.rl_ny = je.nrm + n;
        J.rl_nz = je.nrm + 2 * n;
    }
    grt::ServeEpoch e{};
    e.jobs = E.d_jobs;
    e.chunks = E.d_chunks;
    e.nchunks = 0;
    e.total = n;
    e.counters = E.counters;
    e.stop = nullptr;
    e.S = s->S;
    err = hipMemcpyAsync(E.d_jobs, E.h_jobs, sizeof(grt::RenderArgs) * s->opts.max_jobs, hipMemcpyHostToDevice,
                         E.stream);
    // the joint order: every member's sort keys tagged with its member index,
    // then one sort (24-bit keys: three passes leave it in (k1, v1))
    int64_t at = 0;
    for (size_t m = 0; m < mem.size() && err == hipSuccess; ++m) {
        err = grt::launch_ray_keys(mem[m]->args, (int)mem[m]->total, k0 + at, v0 + at,
                                   (uint32_t)m << grt::kJointShift, E.stream);
        at += mem[m]->total;
    }
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (err == hipSuccess) {
        grt::launch_radix_sort((int)n, 3, k0, v0, k1, v1, hist, E.stream);
        hipLaunchKernelGGL(grt::k_joint_gather, dim3(nb), dim3(256), 0, E.stream, je);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = grt::launch_epoch(e, &J, 0, relight, epoch_k(s, relight), s->ctx->num_cu, E.stream);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(grt::k_joint_scatter, dim3(nb), dim3(256), 0, E.stream, je);
        err = hipGetLastError();
    }
    for (ServerJob *j : mem) {
        if (err != hipSuccess) break;
        if (j->relight && (err = grt::launch_relight_shade(j->args, E.stream)) != hipSuccess) break;
        hipLaunchKernelGGL(grt::k_serve_reduce, dim3((unsigned)((j->npix + 255) / 256)), dim3(256), 0, E.stream,
                           E.d_jobs + j->slot, j->npix, nullptr, n);
        err = hipGetLastError();
        if (err == hipSuccess)
            err = hipMemcpyAsync(j->spec.out_rgb, j->args.out, 12 * (size_t)j->npix,
                                 j->out_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, E.stream);
    }
    if (err == hipSuccess) err = hipEventRecord(E.done, E.stream);
    (void)other;
    E.inflight = true;
    E.rays = n;
    E.t_launch = s->now();
    s->rays_done += n;
    ++s->epochs;
    return true;
}

// Plan an epoch into slot E and launch it; false if no ray is left to trace.
bool launch(grt_server *s, grt::EpochSlot &E, grt::EpochSlot &other, int64_t budget, hipError_t &err)
{
    // A request whose rays are in the other epoch while that one may still be
    // stopped waits for it: a stop hands unclaimed rays back to the request,
    // which must then not be finishing in this epoch already.
    const uint64_t held = other.inflight && other.preemptible && !other.members.empty() ? other.members[0] : 0;
    std::vector<ServerJob *> run;
    for (uint64_t id : s->resident) {
        ServerJob &j = s->jobs[id];
        if (j.state == kRunning && !j.cancel && j.nleft > 0 && j.id != held) run.push_back(&j);
    }
    if (run.empty()) return false;
    // earliest deadline first (protected requests before all others); the
    // budget goes down the list
    const bool budgets = s->share > 0.0;
    auto guarded = [budgets](const ServerJob *j) { return budgets && j->started && j->passable <= 0; };
    std::stable_sort(run.begin(), run.end(), [&](const ServerJob *a, const ServerJob *b) {
        const bool pa = guarded(a), pb = guarded(b);
        return pa != pb ? pa : a->deadline < b->deadline;
    });
    // an epoch holds requests of the head request's kind (one trace per kernel)
    const bool relight = run[0]->relight;
    run.erase(std::remove_if(run.begin(), run.end(), [relight](const ServerJob *j) { return j->relight != relight; }),
              run.end());
    // With preemption on, an earlier-deadline request still uploading needs
    // the CUs for its sampling and sort kernels first: a persistent epoch
    // would hold them (without it, that request passes at the next epoch).
    if (budgets && !guarded(run[0]))
        for (uint64_t id : s->resident) {
            const ServerJob &u = s->jobs[id];
            if (u.state == kUploading && !u.cancel && u.deadline < run[0]->deadline) return false;
        }
    // Launch gate: while the other epoch is in flight, the next one starts
    // only once that one is estimated to be within kTailSeconds of its end,
    // or at once when it is small next to what the other epoch has left (both
    // off as built: the next epoch waits for the one in flight).
    if (other.inflight && !other.stopped) {
        int64_t want = 0;
        for (ServerJob *j : run) {
            const int64_t take = std::min(j->nleft, budget - want);
            if (want > 0 && want + take > kFillRays) break;
            want += take;
            if (want >= budget) break;
        }
        // (kTailSeconds 0: never on the estimate alone.  The rate is a mean
        // and an epoch's end is its slowest rays, so an estimate that says
        // the other epoch is over comes early; a large epoch started then held
        // the CUs that the other's shading and per-pixel sum still needed,
        // and a 4M-ray request waited 0.47 s for a 38M-ray one.)
        const double left = (double)other.rays - s->rate * (s->now() - other.t_launch);
        const bool tail = kTailSeconds > 0.0 && left <= s->rate * kTailSeconds;
        const bool small = kSmallShare > 0.0 && (double)want <= kSmallShare * left;
        if (!tail && !small) return false;
    }
    if (launch_cotrace(s, E, other, run, budget, err)) return true;
    if (err != hipSuccess) return true;
    int nch = 0;
    int64_t off = 0;
    for (ServerJob *j : run) {
        // an epoch is the head request's rest, topped up with the next
        // requests while the whole stays small (a small request is never
        // held back by a large one sharing its epoch)
        if (off >= budget || nch >= s->chunk_cap) break;
        int64_t take = std::min(j->nleft, budget - off);
        if (nch > 0 && off + take > kFillRays) break;
        E.h_jobs[j->slot] = j->args;
        while (take > 0 && nch < s->chunk_cap) {
            std::pair<int64_t, int64_t> &rg = j->left.front();
            const int64_t n = std::min(take, rg.second - rg.first);
            E.h_chunks[nch].slot = j->slot;
            E.h_chunks[nch].pad = 0;
            E.h_chunks[nch].begin = rg.first;
            E.h_chunks[nch].offset = off;
            ++nch;
            off += n;
            take -= n;
            j->nleft -= n;
            rg.first += n;
            if (rg.first == rg.second) j->left.pop_front();
        }
        ++j->inflight;
        j->started = true;
        E.members.push_back(j->id);
        if (j->nleft == 0) E.finishing.push_back(j->id);
    }
    // started requests this epoch passes are charged for its rays
    for (ServerJob *j : run)
        if (j->started && j->nleft > 0 && std::find(E.members.begin(), E.members.end(), j->id) == E.members.end())
            j->passable -= off;
    // an epoch of one request's radiance rays may be stopped for a more
    // urgent one (relighting epochs run to their end)
    E.relight = relight;
    E.preemptible = !relight && s->share > 0.0 && E.members.size() == 1 && off >= kPreemptRays;
    E.stopped = false;
    E.nch = nch;
    __atomic_store_n(E.stop_h, 0, __ATOMIC_RELEASE);
    grt::ServeEpoch e{};
    e.jobs = E.d_jobs;
    e.chunks = E.d_chunks;
    e.nchunks = nch;
    e.total = off;
    e.counters = E.counters;
    e.stop = E.preemptible ? E.stop_d : nullptr;
    e.S = s->S;
    err = hipMemcpyAsync(E.d_jobs, E.h_jobs, sizeof(grt::RenderArgs) * s->opts.max_jobs, hipMemcpyHostToDevice,
                         E.stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(E.d_chunks, E.h_chunks, sizeof(grt::ServeChunk) * nch, hipMemcpyHostToDevice, E.stream);
    const grt::RenderArgs *one = E.members.size() == 1 ? &E.h_jobs[E.h_chunks[0].slot] : nullptr;
    if (err == hipSuccess)
        err = grt::launch_epoch(e, one, E.h_chunks[0].begin, relight, epoch_k(s, relight), s->ctx->num_cu, E.stream);
    if (err == hipSuccess && E.preemptible)
        err = hipMemcpyAsync(E.h_counters, E.counters, grt::kParts * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             E.stream);
    // a finishing job may still have rays in the other epoch
    if (err == hipSuccess && !E.finishing.empty() && other.inflight)
        err = hipStreamWaitEvent(E.stream, other.done, 0);
    for (uint64_t id : E.finishing) {
        if (err != hipSuccess) break;
        ServerJob &j = s->jobs[id];
        // relighting: the shading pass over the request's parked query results
        if (j.relight && (err = grt::launch_relight_shade(j.args, E.stream)) != hipSuccess) break;
        hipLaunchKernelGGL(grt::k_serve_reduce, dim3((unsigned)((j.npix + 255) / 256)), dim3(256), 0, E.stream,
                           E.d_jobs + j.slot, j.npix, E.preemptible ? E.counters : nullptr, off);
        err = hipGetLastError();
        if (err == hipSuccess)
            err = hipMemcpyAsync(j.spec.out_rgb, j.args.out, 12 * (size_t)j.npix,
                                 j.out_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, E.stream);
    }
    if (err == hipSuccess) err = hipEventRecord(E.done, E.stream);
    E.inflight = true;
    E.rays = off;
    E.t_launch = s->now();
    s->rays_done += off;
    ++s->epochs;
    return true;
}

// Raise the stop flag of a preemptible epoch in flight when resident
// requests with earlier deadlines wait (uploading, or ready with rays left),
// the epoch is not about to end by itself, and the rays they would run ahead
// of its request fit what that request still lets pass.  The request then
// is charged for them when they launch.
void preempt(grt_server *s)
{
    for (grt::EpochSlot &E : s->ep) {
        if (!E.inflight || !E.preemptible || E.stopped) continue;
        const double left = ((double)E.rays - s->rate * (s->now() - E.t_launch)) / s->rate;
        if (left < kStopSeconds) continue;
        ServerJob &J = s->jobs[E.members[0]];
        int64_t ahead = 0;
        for (uint64_t id : s->resident) {
            const ServerJob &j = s->jobs[id];
            if (j.cancel || j.id == J.id || j.nleft == 0 || j.deadline >= J.deadline) continue;
            if (j.state != kUploading && j.state != kRunning) continue;
            ahead += j.nleft;
        }
        if (ahead == 0 || ahead > J.passable) continue;
        __atomic_store_n(E.stop_h, 1, __ATOMIC_RELEASE);
        E.stopped = true;
    }
}

void scheduler(grt_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    const int64_t budget = s->opts.epoch_rays > 0 ? s->opts.epoch_rays : (int64_t)1 << 27;
    std::vector<uint64_t> to_upload;
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        bool progressed = false;
        admit(s, to_upload);
        if (!to_upload.empty()) {
            std::vector<uint64_t> ids;
            ids.swap(to_upload);
            for (uint64_t id : ids) {
                ServerJob *j = &s->jobs[id];
                lk.unlock();
                const hipError_t e = upload(s, *j);
                lk.lock();
                if (e != hipSuccess) {
                    device_failed(s);
                    return;
                }
            }
            progressed = true;
        }
        // retire epochs that have completed (never block: arrivals keep
        // being admitted and uploaded while epochs run)
        for (grt::EpochSlot &E : s->ep) {
            if (!E.inflight) continue;
            const hipError_t e = hipEventQuery(E.done);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) {
                device_failed(s);
                return;
            }
            retire(s, E);
            progressed = true;
        }
        sweep(s);
        preempt(s);
        // fill free epoch slots
        for (int b = 0; b < 2; ++b) {
            grt::EpochSlot &E = s->ep[b];
            if (E.inflight) continue;
            hipError_t err = hipSuccess;
            if (!launch(s, E, s->ep[b ^ 1], budget, err)) break;
            if (err != hipSuccess) {
                device_failed(s);
                return;
            }
            progressed = true;
        }
        if (progressed) {
            s->cv.notify_all();
            continue;
        }
        if (s->resident.empty() && s->pending.empty() && !s->ep[0].inflight && !s->ep[1].inflight)
            s->cv.wait(lk, [s] { return s->stop || !s->pending.empty(); });
        else
            s->cv.wait_for(lk, std::chrono::microseconds(50));
    }
    lk.unlock();
    for (grt::EpochSlot &E : s->ep)
        if (E.stream) (void)hipStreamSynchronize(E.stream);
    (void)hipStreamSynchronize(s->copy);
    lk.lock();
    for (grt::EpochSlot &E : s->ep) retire(s, E);
    fail_all(s, GRT_ERR_CANCELLED);
    s->cv.notify_all();
}

void destroy_resources(grt_server *s)
{
    for (grt::EpochSlot &E : s->ep) {
        if (E.stream) (void)hipStreamSynchronize(E.stream);
        if (E.h_jobs) (void)hipHostFree(E.h_jobs);
        if (E.h_chunks) (void)hipHostFree(E.h_chunks);
        if (E.h_counters) (void)hipHostFree(E.h_counters);
        if (E.stop_h) (void)hipHostFree(E.stop_h);
        if (E.done) (void)hipEventDestroy(E.done);
        if (E.stream) (void)hipStreamDestroy(E.stream);
    }
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    if (s->copy) (void)hipStreamDestroy(s->copy);
}

// The server's device memory, all in the caller's workspace: per epoch slot
// the job table, the chunk table and the claim counters, the copy stream's
// counters, then the request pool.
struct ServerWS {
    grt::RenderArgs *d_jobs[2];
    grt::ServeChunk *d_chunks[2];
    unsigned long long *counters[2];
    unsigned long long *copy_counters;
    float *lut;  // the DFG table every relighting request shares
    char *pool;
    size_t pool_bytes;
    size_t bytes;
};

ServerWS carve_server(void *base, const grt_server_opts &o)
{
    ServerWS w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? (char *)base + off : nullptr;
        off += grt::align256(bytes);
        return p;
    };
    const int chunk_cap = o.max_jobs + 64;
    for (int b = 0; b < 2; ++b) {
        w.d_jobs[b] = (grt::RenderArgs *)take(sizeof(grt::RenderArgs) * (size_t)o.max_jobs);
        w.d_chunks[b] = (grt::ServeChunk *)take(sizeof(grt::ServeChunk) * (size_t)chunk_cap);
        w.counters[b] = (unsigned long long *)take(grt::kCounterBytes);
    }
    w.copy_counters = (unsigned long long *)take(grt::kCounterBytes);
    w.lut = (float *)take(sizeof(float) * 2 * grt::kLutN * grt::kLutN);
    w.pool_bytes = o.mem_budget & ~(size_t)255;
    w.pool = take(w.pool_bytes);
    w.bytes = off;
    return w;
}

int check_opts(const grt_server_opts *opts)
{
    if (opts->max_jobs <= 0 || opts->max_jobs > 256) return sfail(GRT_ERR_INVALID, "max_jobs must be in 1..256");
    if (opts->mem_budget < ((size_t)1 << 20)) return sfail(GRT_ERR_INVALID, "mem_budget below 1 MiB");
    return GRT_OK;
}

}  // namespace

extern "C" {

size_t grt_server_workspace_bytes(const grt_server_opts *opts)
{
    if (!opts || opts->max_jobs <= 0 || opts->max_jobs > 256 || opts->mem_budget < ((size_t)1 << 20)) return 0;
    return carve_server(nullptr, *opts).bytes;
}

size_t grt_server_job_bytes(const grt_job *job)
{
    if (check_job(job) != GRT_OK) return 0;
    return job_bytes(*job);
}

int grt_server_create(grt_ctx *ctx, const grt_scene *scene, const grt_server_opts *opts, grt_server **out)
{
    if (!ctx || !scene || !opts || !out) return sfail(GRT_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (int rc = check_opts(opts)) return rc;
    const ServerWS need = carve_server(nullptr, *opts);
    if (!opts->workspace || opts->ws_bytes < need.bytes)
        return sfail(GRT_ERR_OOM, "server workspace missing or below grt_server_workspace_bytes");
    if (((uintptr_t)opts->workspace & 255u) != 0) return sfail(GRT_ERR_INVALID, "server workspace must be 256-byte aligned");
    if (!(opts->k == 4 || opts->k == 8 || opts->k == 12 || opts->k == 16))
        return sfail(GRT_ERR_INVALID, "server k must be 4, 8, 12 or 16");
    if (!(opts->k_relight == 0 || opts->k_relight == 4 || opts->k_relight == 8 || opts->k_relight == 12 ||
          opts->k_relight == 16))
        return sfail(GRT_ERR_INVALID, "server k_relight must be 0, 4, 8, 12 or 16");
    if (!(opts->t_min >= 0.0f) || !(opts->t_cut >= 0.0f && opts->t_cut < 1.0f))
        return sfail(GRT_ERR_INVALID, "bad t_min / t_cut");
    grt_server *s = new (std::nothrow) grt_server;
    if (!s) return sfail(GRT_ERR_OOM, "host allocation failed");
    const char *why = nullptr;
    if (grt::scene_dev_of(scene, &s->S, &why) != GRT_OK) {
        delete s;
        return sfail(GRT_ERR_NOT_BUILT, why ? why : "scene not built");
    }
    s->ctx = ctx;
    s->opts = *opts;
    s->t0 = grt::Clock::now();
    s->slack = opts->slack_per_ray < 0.0 ? 4e-8 : opts->slack_per_ray;
    s->share = opts->preempt_share < 0.0 ? 0.0 : opts->preempt_share;
    // a request's rays may come back from stopped epochs in up to 8 ranges
    // per stop; an epoch takes as many as its table holds, the rest wait
    s->chunk_cap = opts->max_jobs + 64;
    const ServerWS w = carve_server(opts->workspace, *opts);
    s->pool = w.pool;
    s->copy_counters = w.copy_counters;
    s->lut = w.lut;
    bool ok = hipSetDevice(ctx->device) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) == hipSuccess;
    // the DFG table once, ahead of every upload on the copy stream (relighting
    // epochs wait for their request's upload)
    ok = ok && grt::launch_dfg_lut(s->lut, s->copy) == hipSuccess;
    for (int b = 0; b < 2; ++b) {
        grt::EpochSlot &E = s->ep[b];
        E.d_jobs = w.d_jobs[b];
        E.d_chunks = w.d_chunks[b];
        E.counters = w.counters[b];
        ok = ok && hipHostMalloc((void **)&E.h_jobs, sizeof(grt::RenderArgs) * opts->max_jobs) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&E.h_chunks, sizeof(grt::ServeChunk) * s->chunk_cap) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&E.h_counters, grt::kCounterBytes) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&E.stop_h, 64, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
        ok = ok && hipHostGetDevicePointer((void **)&E.stop_d, E.stop_h, 0) == hipSuccess;
        ok = ok && hipStreamCreateWithFlags(&E.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&E.done, hipEventDisableTiming) == hipSuccess;
        if (ok) memset(E.h_jobs, 0, sizeof(grt::RenderArgs) * opts->max_jobs);
    }
    if (!ok) {
        destroy_resources(s);
        delete s;
        return sfail(GRT_ERR_OOM, "host allocation for the server failed");
    }
    s->alloc.init(w.pool_bytes);
    for (int i = opts->max_jobs - 1; i >= 0; --i) s->free_slots.push_back(i);
    try {
        s->th = std::thread(scheduler, s);
    } catch (...) {
        destroy_resources(s);
        delete s;
        return sfail(GRT_ERR_DEVICE, "could not start the scheduler thread");
    }
    *out = s;
    return GRT_OK;
}

int grt_server_submit(grt_server *s, const grt_job *job, uint64_t *id)
{
    if (!s || !id) return sfail(GRT_ERR_INVALID, "NULL argument");
    if (check_job(job) != GRT_OK) return sfail(GRT_ERR_INVALID, "malformed job");
    if ((job->camera_request || job->relight) && s->S.n > 0 &&
        (!s->opts.attrs.albedo || !s->opts.attrs.rough || !s->opts.attrs.metal))
        return sfail(GRT_ERR_INVALID, "camera and relighting requests need the server's surfel attributes");
    const size_t bytes = job_bytes(*job);
    if (bytes > (s->opts.mem_budget & ~(size_t)255)) return sfail(GRT_ERR_ADMISSION, "job exceeds the memory budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error) return sfail(s->error, "server failed");
    if (s->pending.size() >= 4096) return sfail(GRT_ERR_BUSY, "queue full");
    ServerJob &j = s->jobs[s->next_id];
    j.id = s->next_id++;
    j.spec = *job;
    j.relight = job->relight != 0;
    j.out_device = on_device(job->out_rgb);
    j.bytes = bytes;
    j.npix = (int64_t)job->H * job->W;
    j.total = j.npix * (job->n_cos + job->n_ggx + job->n_env);
    j.left.assign(1, {0, j.total});
    j.nleft = j.total;
    j.passable = (int64_t)(s->share * (double)j.total);
    j.t_submit = s->now();
    j.deadline = j.t_submit + s->slack * (double)j.total;
    s->pending.push_back(j.id);
    *id = j.id;
    s->cv.notify_all();
    return GRT_OK;
}

int grt_server_poll(grt_server *s, uint64_t id, int *state)
{
    if (!s || !state) return sfail(GRT_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return sfail(GRT_ERR_INVALID, "unknown job id");
    *state = it->second.state == kDone && it->second.status != GRT_OK ? it->second.status : it->second.state;
    return GRT_OK;
}

int grt_server_wait(grt_server *s, uint64_t id, double timeout_s)
{
    if (!s) return sfail(GRT_ERR_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = grt::Clock::now() + std::chrono::duration<double>(timeout_s);
    for (;;) {
        // looked up after every wake: entries of old finished requests are dropped
        auto it = s->jobs.find(id);
        if (it == s->jobs.end()) return sfail(GRT_ERR_INVALID, "unknown job id");
        if (it->second.state == kDone) return it->second.status;
        if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout) {
            it = s->jobs.find(id);
            if (it != s->jobs.end() && it->second.state == kDone) return it->second.status;
            return sfail(GRT_ERR_TIMEOUT, "wait timed out");
        }
    }
}

int grt_server_cancel(grt_server *s, uint64_t id)
{
    if (!s) return sfail(GRT_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return sfail(GRT_ERR_INVALID, "unknown job id");
    ServerJob &j = it->second;
    if (j.state == kDone) return GRT_OK;
    if (j.state == kQueued) {
        for (auto p = s->pending.begin(); p != s->pending.end(); ++p)
            if (*p == id) { s->pending.erase(p); break; }
        finish_job(s, j, GRT_ERR_CANCELLED);
        s->cv.notify_all();
        return GRT_OK;
    }
    j.cancel = true;  // dropped at the next epoch boundary
    return GRT_OK;
}

int grt_server_job_times(grt_server *s, uint64_t id, double *submit_s, double *start_s, double *done_s)
{
    if (!s) return sfail(GRT_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return sfail(GRT_ERR_INVALID, "unknown job id");
    if (submit_s) *submit_s = it->second.t_submit;
    if (start_s) *start_s = it->second.t_start;
    if (done_s) *done_s = it->second.t_done;
    return GRT_OK;
}

int grt_server_stats(grt_server *s, uint64_t *epochs, uint64_t *stopped, int64_t *rays, size_t *pool_free)
{
    if (!s) return sfail(GRT_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (epochs) *epochs = s->epochs;
    if (stopped) *stopped = s->stopped;
    if (rays) *rays = s->rays_done;
    if (pool_free) {
        size_t f = 0;
        for (auto &kv : s->alloc.free_) f += kv.second;
        *pool_free = f;
    }
    return GRT_OK;
}

int grt_server_destroy(grt_server *s)
{
    if (!s) return GRT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    destroy_resources(s);
    delete s;
    return GRT_OK;
}

}  // extern "C"
