"""Benchmark: differentiable 2D Gaussian ray tracing of secondary rays with
MIS shading, one training step on the 1M-surfel room scene.

One step = the whole hot path over one synthetic batch, inputs resident in
HBM: surfel frames + LBVH build, the fused MIS render (sample, trace with a
k-nearest buffer, shade, per-pixel reduction) and its backward by
re-traversal (gradients for every surfel parameter), driven through the
torch.autograd.Function.  Workload: 1,000,000 surfels (700k on the walls and
floor of a 4x3x4 room, 300k on 10 spheres and 10 boxes), a 1024x1024
G-buffer from a camera inside the room, 32 samples per pixel split 16/8/8
(cosine / GGX / environment) against a 256x512 environment map.

Beside the headline the line carries the other measured workloads: the plain
trace of 4,096 surfels, the 300k-surfel forward and its differentiable step
(re-traversal against stored hit lists), split-sum relighting of the room,
and the relighting server against one launch per request.

Prints ONE JSON line.  Mrays/s counts rays as valid pixels x spp (or rays,
for the plain trace).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PROFILES = os.path.join(ROOT, "profiles")
WORKCOUNT = {name: os.path.join(PROFILES, f"workcount_{name}.json")
             for name in ("room1m_1024px_32spp", "shapes300k_800px_32spp", "plain4k_32768rays")}
TRAFFIC = os.path.join(PROFILES, "traffic_room1m_1024px_32spp.json")
CSRC = os.path.join(ROOT, "paper_2607_22780_amd", "csrc")

# the sources the render kernels are built from
KERNEL_SOURCES = ("render.hip", "grt_device.h", "grt_kernels.h", "grt_render.h", "grt_internal.h")


def source_hash():
    """Hash of the render kernels' sources: traffic counters are only valid
    for the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


SPLIT = (16, 8, 8)
SEED = 7
HBM_PEAK_GBS = 8000.0
RES = 1024
WORK_RAYS = 65536  # sampled rays per work count (2,048 pixels x 32 spp)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs():
    from paper_2607_22780_amd import workloads as W
    s = W.scene3()
    gb = W.gbuffer3(RES, RES)
    env = W.envmap(256, 512, seed=0, stream=3, config_id=1)
    return s, gb, env


def shapes_inputs():
    from paper_2607_22780_amd import workloads as W
    return W.scene1(), W.gbuffer1(), W.envmap()


# --------------------------------------------------------------------------
# Algorithmic work per ray (the oracle's reference LBVH), for the rooflines
# --------------------------------------------------------------------------

def _count_render(name, s, gb, env, npx):
    from oracle import oracle as O
    valid = np.nonzero(gb.valid)[0]
    pix = np.sort(np.random.default_rng(1).choice(valid, npx, replace=False))
    t0 = time.time()
    d = O.render_mis(s, gb, env, SPLIT, SEED, pix=pix, dump=True)
    tr = d["traced"].astype(bool)
    org = np.repeat(gb.x[pix][:, None, :], sum(SPLIT), axis=1)[tr]
    nc, nn, nh = O.count_work(s, org.astype(np.float32), d["dir"][tr].astype(np.float32), t_min=1e-3)
    return dict(sample_pixels=int(npx), sample_rays=int(npx * sum(SPLIT)), traced_rays=int(tr.sum()),
                traced_fraction=float(tr.mean()), mean_n_node=float(nn.mean()), mean_n_cand=float(nc.mean()),
                mean_n_hit=float(nh.mean()), seconds=round(time.time() - t0, 1))


def count_work():
    """Per-ray algorithmic work (N_node, N_cand, N_hit) of each workload,
    counted by the oracle on its reference LBVH over 65,536 seeded sample
    rays (all 32,768 rays of the plain trace), written to profiles/
    (measurement infrastructure)."""
    from oracle import oracle as O
    from paper_2607_22780_amd import workloads as W
    out = {}
    s0, r0 = W.scene0(), W.rays0()
    t0 = time.time()
    nc, nn, nh = O.count_work(s0, r0.origins, r0.dirs, t_min=0.0)
    out["plain4k_32768rays"] = dict(workload="plain trace, 4,096 surfels, 32,768 rays", sample_rays=int(r0.n),
                                    traced_rays=int(r0.n), traced_fraction=1.0, mean_n_node=float(nn.mean()),
                                    mean_n_cand=float(nc.mean()), mean_n_hit=float(nh.mean()),
                                    seconds=round(time.time() - t0, 1))
    npx = WORK_RAYS // sum(SPLIT)
    s1, g1, e1 = shapes_inputs()
    out["shapes300k_800px_32spp"] = dict(workload="shapes, 300k surfels, 800x800 G-buffer, 32 spp (16/8/8), "
                                                  "256x512 env", **_count_render("shapes", s1, g1, e1, npx))
    s3, g3, e3 = make_inputs()
    out["room1m_1024px_32spp"] = dict(workload="room 1M surfels, 1024x1024 G-buffer, 32 spp (16/8/8), 256x512 env",
                                      **_count_render("room", s3, g3, e3, npx))
    os.makedirs(PROFILES, exist_ok=True)
    for name, d in out.items():
        with open(WORKCOUNT[name], "w") as f:
            json.dump(d, f, indent=1)
    return out


def load_work(name):
    p = WORKCOUNT[name]
    return json.load(open(p)) if os.path.exists(p) else None


def trace_bytes(wc):
    """Algorithmic bytes of one traced ray: the ray (32), its output (16), one
    64-byte line per reference-LBVH node and per candidate surfel."""
    return 32 + 16 + 64 * wc["mean_n_node"] + 64 * wc["mean_n_cand"]


def bytes_per_ray(wc, env_hw=(256, 512)):
    """Algorithmic bytes per sample ray (forward and backward), from the counts."""
    spp = sum(SPLIT)
    tf = wc["traced_fraction"]
    env_lookup = 12 + (SPLIT[2] / spp) * 4 * (math.log2(env_hw[0]) + math.log2(env_hw[1]))
    shade = (56 + 12) / spp + env_lookup
    fwd = shade + tf * (trace_bytes(wc) + 16)            # + 16 B saved per traced ray
    bwd = shade + 12 / spp + tf * (trace_bytes(wc) + 16 + 52 * wc["mean_n_hit"])
    return fwd, bwd


def trace_kernel(kind, k):
    """Base name of the kernel the library launches for the MIS forward
    ("fwd") or its re-traversal backward ("bwd") at k-buffer size k (the
    sizes held to 3 wavefronts per SIMD have their own kernels)."""
    if kind == "bwd":
        return "k_render_bwd_w3" if k == 13 else "k_render_bwd"
    return "k_render_w3" if k in (12, 16) else "k_render"


def roofline(bytes_per, units, ms):
    achieved = bytes_per * units / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), bytes_per_unit=round(bytes_per, 1), kernel_ms=round(ms, 3))


# --------------------------------------------------------------------------
# The oracle on the host
# --------------------------------------------------------------------------

def cpu_model():
    """The host CPU as lscpu reports it: the model name (a virtual machine
    may shorten it) with the family/model/stepping, the logical CPUs and the
    clock, so that the identification does not rest on the name alone."""
    keys = {"Model name": "model_name", "Vendor ID": "vendor", "CPU family": "family", "Model": "model",
            "Stepping": "stepping", "CPU(s)": "cpus", "Thread(s) per core": "threads_per_core",
            "Socket(s)": "sockets", "CPU max MHz": "max_mhz", "L3 cache": "l3"}
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in keys and v.strip():
                info[keys[k.strip()]] = v.strip()
    except Exception:
        pass
    if "model_name" not in info:
        try:
            with open("/proc/cpuinfo") as f:
                name = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
            if name:
                info["model_name"] = name
        except OSError:
            pass
    return info or None


def cpu_baseline(s, gb, env, npx: int = 192, runs: int = 3):
    """The oracle (brute force, OpenMP) on a bounded sample of the same step,
    forward + backward, median of `runs` runs."""
    from oracle import oracle as O
    valid = np.nonzero(gb.valid)[0]
    pix = np.sort(np.random.default_rng(2).choice(valid, npx, replace=False))
    grad = np.random.default_rng(3).normal(0, 1, (npx, 3))
    O.lib()
    fw, bw = [], []
    for _ in range(runs):
        t0 = time.time()
        O.render_mis(s, gb, env, SPLIT, SEED, pix=pix)
        t1 = time.time()
        O.render_mis_backward(s, gb, env, SPLIT, SEED, grad, pix=pix)
        t2 = time.time()
        fw.append(t1 - t0)
        bw.append(t2 - t1)
    f, b = float(np.median(fw)), float(np.median(bw))
    rays = npx * sum(SPLIT)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=round(rays / (f + b) / 1e6, 6), unit="Mrays/s", cores=cores, kind="oracle", cpu=cpu_model(),
                sample=f"{npx} valid pixels x {sum(SPLIT)} spp ({rays} rays) of the same step, forward + backward, "
                       f"median of {runs} runs (forward {f:.2f}s, backward {b:.2f}s), scene/G-buffer generation "
                       f"excluded")


# --------------------------------------------------------------------------
# Further workloads
# --------------------------------------------------------------------------

def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def _median_ms(fn, reps):
    import torch
    st = torch.cuda.current_stream()
    e0, e1 = _events(2)
    ts = []
    for _ in range(reps):
        e0.record(st)
        fn()
        e1.record(st)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def leg_plain(ctx, k, oracle=True):
    """The plain trace: 4,096 surfels, 32,768 rays (grt_trace); with `oracle`
    also the oracle on all of them (one run)."""
    import torch
    from paper_2607_22780_amd import grt
    from paper_2607_22780_amd import workloads as W
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    s, r = W.scene0(), W.rays0()
    scene = grt.Scene(ctx, *(t(a) for a in s.arrays()))
    o, d = t(r.origins), t(r.dirs)
    grt.trace(scene, o, d, k=k)
    build_ms = _median_ms(scene.build, 5)
    ms = _median_ms(lambda: grt.trace(scene, o, d, k=k), 10)
    out = dict(workload="4,096 surfels, 32,768 rays from 64x64 points, 8 hemisphere rays each",
               build_ms=round(build_ms, 3), trace_ms=round(ms, 4), mrays_s=round(r.n / (ms * 1e-3) / 1e6, 1))
    wc = load_work("plain4k_32768rays")
    if wc:
        out["roofline"] = roofline(trace_bytes(wc), r.n, ms)
    if oracle:
        from oracle import oracle as O
        t0 = time.time()
        O.trace(s, r.origins, r.dirs)
        sec = time.time() - t0
        out["oracle"] = dict(mrays_s=round(r.n / sec / 1e6, 4), seconds=round(sec, 3), rays=r.n,
                             cores=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), runs=1)
    return out


def leg_shapes(ctx, k, k_bwd, hit_cap, oracle_px=256):
    """The 300k-surfel scene at 800x800, 32 spp: the MIS forward, and the
    differentiable step (loss against a target from perturbed radiance and
    opacity) by re-traversal and from stored hit lists; with oracle_px > 0
    also the oracle's forward and backward on that many seeded valid pixels
    (one run)."""
    import torch
    from paper_2607_22780_amd import grt
    from paper_2607_22780_amd import workloads as W
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    s, gb, env = shapes_inputs()
    rays = int(gb.valid.sum()) * sum(SPLIT)
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, dev)
    tgt_scene = grt.Scene(ctx, *(t(a) for a in W.perturbed(s).arrays()))
    target = grt.render_mis(tgt_scene, E, G, split=SPLIT, seed=SEED, k=k)["rgb"]
    del tgt_scene
    scene = grt.Scene(ctx, *(t(a) for a in s.arrays()))
    build_ms = _median_ms(scene.build, 5)
    state = {}

    def fwd():
        state["f"] = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=k, save=True)

    def bwd():
        up = 2.0 * (state["f"]["rgb"] - target)
        grt.render_mis_backward(scene, E, G, up, state["f"]["saved"], split=SPLIT, seed=SEED, k=k_bwd)

    fwd()
    fwd_ms = _median_ms(fwd, 5)
    bwd_ms = _median_ms(bwd, 5)
    hits = grt.make_hit_list(gb.npix, sum(SPLIT), hit_cap, dev)

    # the list-writing forward carries the list pointer: at most K = 12 fits
    # its register budget without spills
    def fwd_s():
        state["f"] = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=min(k, 12), save=True, hits=hits,
                                    hit_cap=hit_cap)

    def bwd_s():
        up = 2.0 * (state["f"]["rgb"] - target)
        grt.render_mis_backward(scene, E, G, up, state["f"]["saved"], split=SPLIT, seed=SEED, k=k_bwd, hits=hits,
                                hit_cap=hit_cap)

    fwd_s()
    sf_ms = _median_ms(fwd_s, 3)
    sb_ms = _median_ms(bwd_s, 3)
    cnt = hits[:gb.npix * sum(SPLIT)].cpu().numpy()
    out = dict(workload="300k surfels on 3 spheres + 2 tori, 800x800 G-buffer, 32 spp (16/8/8), 256x512 env",
               rays=rays, build_ms=round(build_ms, 3), fwd_ms=round(fwd_ms, 3),
               fwd_mrays_s=round(rays / (fwd_ms * 1e-3) / 1e6, 1),
               step={"loss": "L2 against perturbed radiance and opacity (sigma 0.05)",
                     "retrace": {"fwd_ms": round(fwd_ms, 3), "bwd_ms": round(bwd_ms, 3),
                                 "mrays_s": round(rays / ((fwd_ms + bwd_ms) * 1e-3) / 1e6, 1)},
                     "stored": {"hit_cap": hit_cap, "list_gb": round(hits.numel() * 4 / 1e9, 3),
                                "overflow_frac": round(float((cnt > hit_cap).mean()), 5),
                                "fwd_ms": round(sf_ms, 3), "bwd_ms": round(sb_ms, 3),
                                "mrays_s": round(rays / ((sf_ms + sb_ms) * 1e-3) / 1e6, 1)},
                     "saved_state_gb": round(grt.grt_render_saved_bytes(gb.npix, sum(SPLIT)) / 1e9, 3)})
    wc = load_work("shapes300k_800px_32spp")
    if wc:
        bf, bb = bytes_per_ray(wc)
        out["roofline_fwd"] = roofline(bf, rays, fwd_ms)
        out["roofline_bwd"] = roofline(bb, rays, bwd_ms)
    del hits, state
    if oracle_px > 0:
        from oracle import oracle as O
        pix = np.sort(np.random.default_rng(2).choice(np.nonzero(gb.valid)[0], oracle_px, replace=False))
        grad = np.random.default_rng(3).normal(0, 1, (oracle_px, 3))
        t0 = time.time()
        O.render_mis(s, gb, env, SPLIT, SEED, pix=pix)
        t1 = time.time()
        O.render_mis_backward(s, gb, env, SPLIT, SEED, grad, pix=pix)
        t2 = time.time()
        n = oracle_px * sum(SPLIT)
        out["oracle"] = dict(rays=n, fwd_mrays_s=round(n / (t1 - t0) / 1e6, 6),
                             step_mrays_s=round(n / (t2 - t0) / 1e6, 6), fwd_s=round(t1 - t0, 2),
                             bwd_s=round(t2 - t1, 2), runs=1,
                             cores=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    return out


def _gbuffer_task(key):
    from paper_2607_22780_amd import workloads as W
    res, cam = key
    return key, W.gbuffer3(res, res, cam_stream=10 + cam)


def serve_inputs(n, rate):
    """Relighting requests over the room scene: Poisson arrivals; resolution,
    spp, camera and a 128x256 environment map per request."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_2607_22780_amd import workloads as W
    reqs = W.requests4(n, rate)
    keys = sorted({(q.res, q.cam) for q in reqs}, key=lambda k: -k[0])
    with ProcessPoolExecutor(max_workers=min(8, len(keys))) as ex:
        gbs = dict(ex.map(_gbuffer_task, keys))
    envs = [W.envmap(128, 256, seed=q.env_seed, stream=3, config_id=1) for q in reqs]
    return reqs, gbs, envs


def serve_leg(ctx, scene, k, reqs, gbs, envs, warm, slack=-1.0, epoch=0, extra=False, load=0.0, slack_alt=-1.0,
              small=0, replays=3):
    """The persistent batched server against one launch per request (upload,
    tables, render, copy back, in arrival order), on the same relighting
    requests (the attribute query and split-sum shading under each request's
    own environment) all at once and then replayed at their arrival times.
    The first `warm` requests of each run warm the system and are left out of
    the latency statistics.  load > 0: the Poisson arrival times are scaled so
    that the offered load is `load` of one launch per request's measured
    capacity (its mean service time in the all-at-once run).  slack_alt >= 0:
    the server's replay once more at that slack.  small > 0: a stream of that
    many small requests (256x256, 4 or 8 spp) submitted at once, where one
    launch per request is bound by each launch's slowest rays and the server
    batches requests into epochs of up to 4M rays.  k: the relighting query's
    k-buffer size, on both sides.  replays: runs of each replay (alternating);
    the medians are reported, and each run beside them."""
    import torch
    from paper_2607_22780_amd import grt
    from paper_2607_22780_amd import workloads as W
    from types import SimpleNamespace
    dev = torch.device("cuda", 0)
    splits = [W.mis_split(q.spp) for q in reqs]
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    pinned = {key: SimpleNamespace(H=g.H, W=g.W, x=pin(g.x), n=pin(g.n), wo=pin(g.wo), albedo=pin(g.albedo),
                                   rough=pin(g.rough), metal=pin(g.metal), valid=pin(g.valid))
              for key, g in gbs.items()}
    mats = [torch.from_numpy(a).to(dev) for a in W.surfel_materials(scene.n, seed=0)]
    mk = lambda: [grt.Request(pinned[(q.res, q.cam)], pin(envs[i]), splits[i], q.seed, q.rid, relight=True)
                  for i, q in enumerate(reqs)]
    req_srv, req_one = mk(), mk()
    measured = slice(warm, len(reqs))
    rays_m = sum(r.rays for r in req_srv[measured])
    arrivals = [q.arrival_s for q in reqs]

    def run_server(replay, share=-1.0, rlist=None, sl=None, arr=None, meas=None):
        rlist = req_srv if rlist is None else rlist
        arr = arrivals if arr is None else arr
        meas = measured if meas is None else meas
        srv = grt.Server(ctx, scene, mem_budget=48 << 30, max_jobs=16, k=12, k_relight=k,
                         slack_per_ray=slack if sl is None else sl, epoch_rays=epoch, preempt_share=share, attrs=mats)
        t0 = time.perf_counter()
        ids = []
        for q, r in zip(arr, rlist):
            if replay:
                dt = t0 + q - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            ids.append(srv.submit(r))
        for j in ids:
            st = srv.wait(j, 600.0)
            if st != 0:
                raise grt.GrtError(st, "server request failed")
        times = [srv.times(j) for j in ids]
        srv.close()
        lat = [d - s for s, _, d in times][meas]
        tm = times[meas]
        span = max(d for _, _, d in tm) - min(s for s, _, _ in tm)
        return lat, span

    def run_one(replay, rlist=None, arr=None, meas=None):
        rlist = req_one if rlist is None else rlist
        arr = arrivals if arr is None else arr
        meas = measured if meas is None else meas
        stream = torch.cuda.current_stream()
        t0 = time.perf_counter()
        lat, marks = [], []
        for q, r in zip(arr, rlist):
            if replay:
                dt = t0 + q - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            arrive = t0 + q if replay else t0
            x, n, wo, alb, rough, metal, valid = (a.to(dev, non_blocking=True) for a in r.arrays)
            G = grt.GBuffer(r.H, r.W, x, n, wo, alb, rough, metal, valid)
            E = grt.Env(ctx, r.env.to(dev, non_blocking=True)).prefilter()
            sp = (r.struct.n_cos, r.struct.n_ggx, r.struct.n_env)
            out = grt.render_relight(scene, E, *mats, G, split=sp, seed=r.struct.seed, job=r.struct.job, k=k)["rgb"]
            r.out.copy_(out, non_blocking=True)
            stream.synchronize()
            done = time.perf_counter()
            lat.append(done - arrive)
            marks.append((arrive, done))
            del E
        tm = marks[meas]
        return lat[meas], max(d for _, d in tm) - min(a for a, _ in tm)

    pct = lambda a, p: float(np.percentile(np.asarray(a), p))
    summary = lambda lat, span: {"p50_s": round(pct(lat, 50), 4), "p99_s": round(pct(lat, 99), 4),
                                 "mean_s": round(float(np.mean(lat)), 4), "mrays_s": round(rays_m / span / 1e6, 2)}
    log("bench: per-request leg (all at once)")
    o_bur = run_one(False)
    log("bench: server leg (all at once)")
    s_bur = run_server(False)
    same = all(torch.equal(a.out, b.out) for a, b in zip(req_srv, req_one))
    service_s = o_bur[1] / (len(reqs) - warm)  # one launch per request's mean time per request
    if load > 0.0:
        gap0 = arrivals[-1] / max(len(arrivals) - 1, 1)
        arrivals = [a * (service_s / load) / gap0 for a in arrivals]
    # the replay, server and one launch per request alternating, `replays`
    # times each: single replays' tail latencies vary from run to run (p99
    # over 200 requests is their second-largest latency)
    s_runs, o_runs = [], []
    for i in range(max(replays, 1)):
        log(f"bench: server leg (replayed arrivals, run {i + 1})")
        s_runs.append(summary(*run_server(True)))
        log(f"bench: per-request leg (replayed arrivals, run {i + 1})")
        o_runs.append(summary(*run_one(True)))
    s_alt = None
    if slack_alt >= 0.0:
        log(f"bench: server leg (replayed arrivals, slack {slack_alt:g} s/ray)")
        s_alt = run_server(True, sl=slack_alt)
    med = lambda runs: {key: round(float(np.median([r[key] for r in runs])), 4) for key in runs[0]}
    gap = arrivals[-1] / max(len(arrivals) - 1, 1)
    res = {
        "workload": f"room scene resident; relighting (attribute query + split-sum) of {len(reqs)} requests, "
                    f"the first {warm} as warm-up, {len(reqs) - warm} measured; Poisson {gap:.3f} s mean gap; "
                    f"res in {{256,512,768,1024}}^2, spp in {{4..64}}, 128x256 env each",
        "measured_rays": rays_m,
        "server_slack_per_ray_s": slack,
        "one_launch_mean_service_s": round(service_s, 4),
        "arrival_rate_hz": round(1.0 / gap, 4),
        "offered_load": round(service_s / gap, 3),
        "replay_runs": len(s_runs),
        "server": {"replay": med(s_runs), "replay_each": s_runs, "burst": summary(*s_bur)},
        "one_launch_per_request": {"replay": med(o_runs), "replay_each": o_runs, "burst": summary(*o_bur)},
        "images_identical": bool(same),
    }
    if s_alt is not None:
        res[f"server_replay_slack_{slack_alt:g}"] = summary(*s_alt)
    if small > 0:
        # small requests only: 256x256 at 4 or 8 spp over the four cameras,
        # all submitted at once (no warm-up left out)
        g = np.random.default_rng(17)
        cams = sorted(c for r, c in pinned if r == 256)
        sm = [(int(g.choice(cams)), int(g.choice([4, 8]))) for _ in range(small)]
        env_of = lambda i: envs[i % len(envs)]
        mk_small = lambda: [grt.Request(pinned[(256, cam)], pin(env_of(i)), W.mis_split(spp), 7000 + i, 9000 + i,
                                        relight=True) for i, (cam, spp) in enumerate(sm)]
        zero, allm = [0.0] * small, slice(0, small)
        sm_rays = sum(256 * 256 * spp for _, spp in sm)
        log(f"bench: small-request stream ({small} requests, all at once)")
        ro, rs = mk_small(), mk_small()
        o_sm = run_one(False, rlist=ro, arr=zero, meas=allm)
        s_sm = run_server(False, rlist=rs, arr=zero, meas=allm)
        same_sm = all(torch.equal(a.out, b.out) for a, b in zip(rs, ro))
        summ = lambda lat, span: {"p50_s": round(pct(lat, 50), 4), "p99_s": round(pct(lat, 99), 4),
                                  "mean_s": round(float(np.mean(lat)), 4), "mrays_s": round(sm_rays / span / 1e6, 2)}
        res["small_request_stream"] = {"requests": small, "rays": sm_rays, "res": 256, "spp": [4, 8],
                                       "server": summ(*s_sm), "one_launch_per_request": summ(*o_sm),
                                       "images_identical": bool(same_sm)}
    if extra:
        log("bench: server leg with preemption (radiance requests, replayed arrivals)")
        rad = [grt.Request(pinned[(q.res, q.cam)], pin(envs[i]), splits[i], q.seed, q.rid) for i, q in enumerate(reqs)]
        res["server_radiance_preempt_share_0.25"] = summary(*run_server(True, share=0.25, rlist=rad))
        log("bench: server leg with camera requests (replayed arrivals)")
        cams = {q.cam: grt.make_camera(*W.camera3(W.rng(3, 10 + q.cam)), 60.0) for q in reqs}
        rc = [grt.Request(None, pin(envs[i]), splits[i], q.seed, q.rid, camera=cams[q.cam], H=q.res, W=q.res,
                          relight=True) for i, q in enumerate(reqs)]
        res["server_camera_requests"] = summary(*run_server(True, rlist=rc))
    return res


def calib_copy():
    """A plain 1 GiB device copy (2 GiB moved): the achieved bandwidth beside
    the 8 TB/s peak, and the kernel the byte counters are scaled by."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = _median_ms(lambda: b.copy_(a), 10)
    gbs = 2 * a.numel() * 4 / (ms * 1e-3) / 1e9
    del a, b
    return {"bytes_moved": 2 << 30, "ms": round(ms, 3), "achieved_gbs": round(gbs, 1), "peak_gbs": HBM_PEAK_GBS,
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 3)}


def walk_stats_run(k, k_bwd):
    """Walk counters of one differentiable step of the room workload, from
    the library compiled with -DGRT_STATS (its kernels run slower; the
    per-ray counts do not depend on timing, the per-step lane counts only
    through the order in which wavefronts claim rays)."""
    import torch
    from paper_2607_22780_amd import grt
    grt.load_library(grt.STATS_LIB_PATH)
    dev = torch.device("cuda", 0)
    s, gb, env = make_inputs()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = grt.Context(0)
    scene = grt.Scene(ctx, *(t(a) for a in s.arrays()))
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, dev)
    upstream = t(np.random.default_rng(0).normal(0, 1, (gb.npix, 3)).astype(np.float32))
    grt.walk_stats(ctx, reset=True)
    res = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=k, save=True)
    grt.render_mis_backward(scene, E, G, upstream, res["saved"], split=SPLIT, seed=SEED, k=k_bwd)
    st = grt.walk_stats(ctx, reset=True)
    out = {}
    for kind, d in st.items():
        n = max(d["rays"], 1)
        row = {"rays": d["rays"]}
        for key in ("node_visits", "leaf_tests", "composites", "rounds", "restarts", "deferred"):
            row[key + "_per_ray"] = round(d[key] / n, 3)
        row["lane_steps_per_ray"] = round(d["active_lanes"] / n, 3)
        row["wave_steps_x64_per_ray"] = round(64 * d["wave_steps"] / n, 3)
        row["active_lanes_per_step"] = round(d["active_lanes"] / max(d["wave_steps"], 1), 3)
        out[kind] = row
    return {"walk_stats": out, "k": k, "k_bwd": k_bwd,
            "config": {"workload": f"room 1M surfels, {RES}x{RES} G-buffer, 32 spp (16/8/8)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=16, help="k-buffer size of the forward")
    ap.add_argument("--k-bwd", type=int, default=13, help="k-buffer size of the backward")
    ap.add_argument("--k-relight", type=int, default=12, help="k-buffer size of the relighting query")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=192, help="pixels of the step the oracle times per run")
    ap.add_argument("--no-serve", action="store_true", help="skip the relighting-server leg")
    ap.add_argument("--serve-extra", action="store_true",
                    help="also replay the server with preemption and with camera requests")
    ap.add_argument("--no-legs", action="store_true", help="skip the plain-trace and 300k-surfel legs")
    ap.add_argument("--room-stored", action="store_true", help="also time stored hit lists on the room")
    ap.add_argument("--no-relight", action="store_true", help="skip the split-sum relighting leg")
    ap.add_argument("--hit-cap", type=int, default=64, help="hits stored per sample in the stored-list legs")
    ap.add_argument("--serve-requests", type=int, default=220)
    ap.add_argument("--serve-warm", type=int, default=20)
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate, requests/s (0: --serve-load of one launch per request's capacity)")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load when the rate is derived: arrivals are spaced so that one launch per request "
                         "(its mean service time measured in the all-at-once run) is busy this share of the time")
    ap.add_argument("--serve-slack", type=float, default=0.0,
                    help="server deadline seconds per ray (-1: the server's default, 4e-8); 0 is arrival order, "
                         "which gives the lowest p99 on one GPU")
    ap.add_argument("--serve-slack-alt", type=float, default=2e-8,
                    help="a second replay of the server at this slack (lower mean latency; negative: skip)")
    ap.add_argument("--serve-replays", type=int, default=3,
                    help="runs of each replay (server and one launch per request alternating; medians reported)")
    ap.add_argument("--serve-small", type=int, default=200,
                    help="requests of the small-request stream (256x256, 4 or 8 spp, all at once; 0: skip)")
    ap.add_argument("--serve-epoch", type=int, default=0, help="server rays per epoch (0: default)")
    ap.add_argument("--count-work", action="store_true", help="recount per-ray work with the oracle and exit")
    ap.add_argument("--calib-copy", action="store_true", help="only time a plain 1 GiB device copy and exit")
    ap.add_argument("--walk-stats", action="store_true",
                    help="only count the walk of one step with the instrumented library (libgrt_stats.so) and exit")
    args = ap.parse_args()

    if args.count_work:
        print(json.dumps(count_work()))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_22780_amd import grt

    if args.calib_copy:
        print(json.dumps(calib_copy()))
        return
    if args.walk_stats:
        print(json.dumps(walk_stats_run(args.k, args.k_bwd)))
        return

    dev = torch.device("cuda", 0)
    log("bench: generating inputs")
    s, gb, env = make_inputs()
    npx_valid = int(gb.valid.sum())
    spp = sum(SPLIT)
    rays = npx_valid * spp
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = grt.Context(0)
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, dev)
    params = [t(a).requires_grad_(True) for a in s.arrays()]
    upstream = t(np.random.default_rng(0).normal(0, 1, (gb.npix, 3)).astype(np.float32))

    def step(timers=None):
        for p in params:
            p.grad = None
        img = grt.RenderMISFn.apply(*params, ctx, E, G, SPLIT, SEED, args.k, 1.0 / 255.0, 0, args.k_bwd, timers)
        loss = (img * upstream).sum()
        loss.backward()
        return img

    log("bench: warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the trace kernels of every timed step, timed by the library with HIP
    # events on their launch stream (a timer pair per step: no sync inside)
    timers = [(grt.Timer(ctx), grt.Timer(ctx)) for _ in range(args.steps)]
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(timers[i])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    kern_fwd_ms = float(np.mean([a.ms() for a, _ in timers])) if timers else None
    kern_bwd_ms = float(np.mean([b.ms() for _, b in timers])) if timers else None
    del timers

    # per-kernel timing with events on the launch stream (torch's current one)
    st = torch.cuda.current_stream()
    scene = grt.Scene(ctx, *(p.detach() for p in params))
    eb0, eb1, ef0, ef1, eg0, eg1 = _events(6)
    build_ms, fwd_ms, bwd_ms = [], [], []
    for _ in range(max(args.steps, 1)):
        eb0.record(st); scene.build(); eb1.record(st)
        ef0.record(st)
        res = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=args.k, save=True)
        ef1.record(st)
        eg0.record(st)
        grt.render_mis_backward(scene, E, G, upstream, res["saved"], split=SPLIT, seed=SEED, k=args.k_bwd)
        eg1.record(st)
        torch.cuda.synchronize()
        build_ms.append(eb0.elapsed_time(eb1)); fwd_ms.append(ef0.elapsed_time(ef1)); bwd_ms.append(eg0.elapsed_time(eg1))
    build_ms, fwd_ms, bwd_ms = (float(np.median(x)) for x in (build_ms, fwd_ms, bwd_ms))
    del res

    stored = None
    if args.room_stored:
        # the same step differentiated from stored hit lists instead of re-traversal
        hits = grt.make_hit_list(gb.npix, spp, args.hit_cap, dev)
        sf, sb = [], []
        for _ in range(max(args.steps // 2, 2)):
            ef0.record(st)
            res = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=min(args.k, 12), save=True, hits=hits,
                                 hit_cap=args.hit_cap)
            ef1.record(st)
            eg0.record(st)
            grt.render_mis_backward(scene, E, G, upstream, res["saved"], split=SPLIT, seed=SEED, k=args.k_bwd,
                                    hits=hits, hit_cap=args.hit_cap)
            eg1.record(st)
            torch.cuda.synchronize()
            sf.append(ef0.elapsed_time(ef1)); sb.append(eg0.elapsed_time(eg1))
        cnt = hits[:gb.npix * spp].cpu().numpy()
        stored = {"hit_cap": args.hit_cap, "list_gb": round(hits.numel() * 4 / 1e9, 3),
                  "overflow_frac": round(float((cnt > args.hit_cap).mean()), 5),
                  "mean_hits_per_sample": round(float(cnt.mean()), 3),
                  "render_fwd_ms": round(float(np.median(sf)), 3), "render_bwd_ms": round(float(np.median(sb)), 3),
                  "retrace_bwd_ms": round(bwd_ms, 3)}
        del hits, res

    legs = None
    if not args.no_legs:
        log("bench: plain-trace leg (4,096 surfels)")
        legs = {"plain_trace_4k": leg_plain(ctx, 16, oracle=not args.no_cpu_baseline)}
        log("bench: 300k-surfel leg (forward; differentiable step, re-traversal and stored lists)")
        legs["shapes_300k"] = leg_shapes(ctx, args.k, args.k_bwd, args.hit_cap,
                                         oracle_px=0 if args.no_cpu_baseline else 256)

    relight = None
    if not args.no_relight:
        # novel illumination: a fresh 128x256 map, prefiltered; the surfels
        # carry seeded materials; the same G-buffer and samples per pixel
        from paper_2607_22780_amd import workloads as W
        log("bench: relighting leg")
        env_new = W.envmap(128, 256, seed=11, stream=3, config_id=1)
        mats = [t(a) for a in W.surfel_materials(s.n, seed=0)]
        E2 = grt.Env(ctx, t(env_new))
        pf, rf = [], []
        for _ in range(3):
            ef0.record(st); E2.prefilter(); ef1.record(st)
            eg0.record(st)
            out = grt.render_relight(scene, E2, *mats, G, split=SPLIT, seed=SEED, k=args.k_relight)
            eg1.record(st)
            torch.cuda.synchronize()
            pf.append(ef0.elapsed_time(ef1)); rf.append(eg0.elapsed_time(eg1))
        frame = float(np.median(rf))
        # cross-bilateral denoise of the relit frame (radius 3: 7x7 window)
        dgb = [t(gb.depth), G.n, G.valid]
        dn_ms = _median_ms(lambda: grt.denoise(ctx, out["rgb"], *dgb, gb.H, gb.W), 5)
        # primary-ray G-buffer by 2DGRT of a 1024^2 camera inside the room
        cam_o, cam_d = W.pinhole(*W.camera3(W.rng(3, 2)), 60.0, gb.H, gb.W)
        co, cd = t(cam_o.astype(np.float32)), t(cam_d.astype(np.float32))
        holder = {}

        def gtrace():
            holder["g"] = grt.trace_gbuffer(scene, *mats, co, cd, gb.H, gb.W, k=12)

        gt_ms = _median_ms(gtrace, 5)
        gbt = holder.pop("g")
        covered = float(gbt["valid"].float().mean().item())
        # its backward by re-traversal, seeded upstream gradients on every map
        gen = torch.Generator(device=dev).manual_seed(SEED)
        gup = {kk: torch.randn(gbt[kk].shape, generator=gen, device=dev)
               for kk in ("x", "n", "albedo", "rough", "metal", "depth", "rgb")}
        gzs = grt.zero_grads(scene.n, dev)
        gza = dict(albedo=torch.zeros(scene.n, 3, device=dev), rough=torch.zeros(scene.n, device=dev),
                   metal=torch.zeros(scene.n, device=dev))
        gbw_ms = _median_ms(lambda: grt.trace_gbuffer_backward(scene, *mats, co, cd, gbt, gup, k=12, grads=gzs,
                                                               attr_grads=gza), 3)
        del gbt, gup, gzs, gza
        # the same relit frame with the mesh backend answering the query
        # (the room as 46k triangles with per-vertex materials)
        mesh3 = W.mesh3()
        mt = [t(a) for a in (mesh3.verts, mesh3.tris)]
        ma = [t(a) for a in (mesh3.albedo, mesh3.rough, mesh3.metal, mesh3.normal)]
        em0, em1 = _events(2)
        em0.record(st)
        M = grt.Mesh(ctx, *mt)
        em1.record(st)
        torch.cuda.synchronize()
        mesh_build_ms = em0.elapsed_time(em1)
        mesh_frame = _median_ms(lambda: grt.render_relight_mesh(M, E2, *ma, G, split=SPLIT, seed=SEED), 3)
        del M
        relight = {"env": "128x256, prefiltered to 16x32 tables at 6 roughness levels + 32x32 DFG",
                   "mesh_backend": {"triangles": int(mesh3.nf), "build_ms": round(mesh_build_ms, 3),
                                    "frame_ms": round(mesh_frame, 3),
                                    "mrays_s": round(rays / (mesh_frame * 1e-3) / 1e6, 2)},
                   "gbuffer_trace_ms": round(gt_ms, 3), "gbuffer_covered": round(covered, 4),
                   "gbuffer_backward_ms": round(gbw_ms, 3),
                   "prefilter_ms": round(float(np.median(pf)), 3), "frame_ms": round(frame, 3),
                   "mrays_s": round(rays / (frame * 1e-3) / 1e6, 2),
                   "radiance_fwd_ms": round(fwd_ms, 3),
                   "denoise_ms": round(dn_ms, 4),
                   "denoise_gb_s": round(gb.npix * 41 / (dn_ms * 1e-3) / 1e9, 1)}
        del out, E2

    roof = None
    wc = load_work("room1m_1024px_32spp")
    if wc:
        bf, bb = bytes_per_ray(wc)
        # the trace kernels alone, averaged over the timed steps
        kf, kb = kern_fwd_ms, kern_bwd_ms
        dominant = "bwd" if kb >= kf else "fwd"
        ms = kb if dominant == "bwd" else kf
        per_ray = bb if dominant == "bwd" else bf
        kname = trace_kernel(dominant, args.k_bwd if dominant == "bwd" else args.k)
        traffic = l2_hit = None
        if os.path.exists(TRAFFIC):
            tr = json.load(open(TRAFFIC))
            if tr.get("source_hash") == source_hash() and kname in tr.get("kernels", {}):
                traffic = tr["kernels"][kname]["hbm_bytes"]
                l2_hit = tr["kernels"][kname].get("l2_hit")
        r = roofline(per_ray, rays, ms)
        roof = dict(bound="hbm", achieved=r["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=r["frac"],
                    traffic=traffic, l2_hit=l2_hit, kernel=kname, bytes_per_ray=round(per_ray, 1),
                    kernel_ms=round(ms, 3), traffic_gbs=round(traffic / (ms * 1e-3) / 1e9, 1) if traffic else None,
                    traced_fraction=round(wc["traced_fraction"], 4), work_sample_rays=wc.get("sample_rays"),
                    kernel_timing=f"library HIP events around the trace kernel on its stream, mean of the "
                                  f"{args.steps} timed steps",
                    fwd_kernel_ms=round(kf, 3), fwd_frac=roofline(bf, rays, kf)["frac"])

    log("bench: device copy (achieved bandwidth)")
    copy = calib_copy()

    serve = None
    if not args.no_serve:
        log("bench: generating relighting requests")
        derived = args.serve_rate <= 0.0
        reqs, gbs, envs = serve_inputs(args.serve_requests, 1.0 if derived else args.serve_rate)
        serve = serve_leg(ctx, scene, args.k_relight, reqs, gbs, envs, args.serve_warm, args.serve_slack, args.serve_epoch,
                          extra=args.serve_extra, load=args.serve_load if derived else 0.0,
                          slack_alt=args.serve_slack_alt, small=args.serve_small, replays=args.serve_replays)
        del reqs, gbs, envs

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(s, gb, env, args.cpu_pixels)

    out = {
        "metric": "Mrays/s fwd & fwd+bwd (1M surfels, 32 spp); relight p50/p99 latency",
        "value": round(rays / dt / 1e6, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "room scene, 1M surfels, 1024x1024 G-buffer, 32 spp (16/8/8 MIS), 256x512 env; "
                               "fwd+bwd training step", "surfels": s.n, "valid_pixels": npx_valid, "spp": spp,
                   "rays_per_step": rays, "k": args.k, "k_bwd": args.k_bwd},
        "fwd_mrays_s": round(rays / (fwd_ms * 1e-3) / 1e6, 2),
        "phase_ms": {"build": round(build_ms, 3), "render_fwd": round(fwd_ms, 3), "render_bwd": round(bwd_ms, 3)},
        "roofline": roof,
        "copy_bandwidth": copy,
        "legs": legs,
        "stored_hit_lists_room": stored,
        "relight_split_sum": relight,
        "relight_server": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
