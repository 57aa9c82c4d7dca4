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

Prints ONE JSON line.  Mrays/s counts rays as valid pixels x spp.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKCOUNT = os.path.join(ROOT, "profiles", "workcount_room1m_1024px_32spp.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_room1m_1024px_32spp.json")
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs():
    from paper_2607_22780_amd import workloads as W
    s = W.scene3()
    gb = W.gbuffer3(RES, RES)
    env = W.envmap(256, 512, seed=0, stream=3, config_id=1)
    return s, gb, env


def count_work(nsample_px: int = 256):
    """Per-ray algorithmic work (N_node, N_cand, N_hit) of the room workload,
    counted by the oracle on a reference LBVH over a seeded pixel sample,
    written to profiles/ for the roofline (measurement infrastructure)."""
    from oracle import oracle as O
    s, gb, env = make_inputs()
    valid = np.nonzero(gb.valid)[0]
    pix = np.sort(np.random.default_rng(1).choice(valid, nsample_px, replace=False))
    t0 = time.time()
    d = O.render_mis(s, gb, env, SPLIT, SEED, pix=pix, dump=True)
    tr = d["traced"].astype(bool)
    org = np.repeat(gb.x[pix][:, None, :], sum(SPLIT), axis=1)[tr]
    dirs = d["dir"][tr]
    nc, nn, nh = O.count_work(s, org.astype(np.float32), dirs.astype(np.float32), t_min=1e-3)
    spp = sum(SPLIT)
    out = dict(workload="room 1M surfels, 1024x1024 G-buffer, 32 spp (16/8/8), 256x512 env",
               sample_pixels=int(nsample_px), sample_rays=int(nsample_px * spp), traced_rays=int(tr.sum()),
               traced_fraction=float(tr.mean()), mean_n_node=float(nn.mean()), mean_n_cand=float(nc.mean()),
               mean_n_hit=float(nh.mean()), seconds=time.time() - t0)
    os.makedirs(os.path.dirname(WORKCOUNT), exist_ok=True)
    with open(WORKCOUNT, "w") as f:
        json.dump(out, f, indent=1)
    return out


def bytes_per_ray(wc, env_hw=(256, 512)):
    """Algorithmic bytes per sample ray (forward and backward), from the counts."""
    spp = sum(SPLIT)
    tf = wc["traced_fraction"]
    trace_fwd = 32 + 16 + 64 * wc["mean_n_node"] + 64 * wc["mean_n_cand"]
    env_lookup = 12 + (SPLIT[2] / spp) * 4 * (math.log2(env_hw[0]) + math.log2(env_hw[1]))
    shade = (56 + 12) / spp + env_lookup
    fwd = shade + tf * (trace_fwd + 16)            # + 16 B saved per traced ray
    bwd = shade + 12 / spp + tf * (trace_fwd + 16 + 52 * wc["mean_n_hit"])
    return fwd, bwd


def cpu_baseline(s, gb, env, npx: int = 384):
    """The oracle (brute force, OpenMP) on a bounded sample of the same step."""
    from oracle import oracle as O
    valid = np.nonzero(gb.valid)[0]
    pix = np.sort(np.random.default_rng(2).choice(valid, npx, replace=False))
    grad = np.random.default_rng(3).normal(0, 1, (npx, 3))
    O.lib()
    t0 = time.time()
    O.render_mis(s, gb, env, SPLIT, SEED, pix=pix)
    t1 = time.time()
    O.render_mis_backward(s, gb, env, SPLIT, SEED, grad, pix=pix)
    t2 = time.time()
    rays = npx * sum(SPLIT)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=rays / (t2 - t0) / 1e6, unit="Mrays/s", cores=cores, kind="oracle", cpu=model,
                sample=f"{npx} valid pixels x {sum(SPLIT)} spp ({rays} rays) of the same step, forward "
                       f"{t1 - t0:.2f}s + backward {t2 - t1:.2f}s, scene/G-buffer generation excluded")


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


def serve_leg(ctx, scene, k, reqs, gbs, envs, slack=-1.0, epoch=0, detail=False, share=-1.0):
    """The persistent batched server versus one launch per request (upload,
    table build, render, copy back, in arrival order), on the same requests
    replayed at their arrival times and then all at once."""
    import torch
    from paper_2607_22780_amd import grt
    from paper_2607_22780_amd import workloads as W
    dev = torch.device("cuda", 0)
    from types import SimpleNamespace
    splits = [W.mis_split(q.spp) for q in reqs]
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    pinned = {key: SimpleNamespace(H=g.H, W=g.W, x=pin(g.x), n=pin(g.n), wo=pin(g.wo), albedo=pin(g.albedo),
                                   rough=pin(g.rough), metal=pin(g.metal), valid=pin(g.valid))
              for key, g in gbs.items()}
    mk = lambda: [grt.Request(pinned[(q.res, q.cam)], pin(envs[i]), splits[i], q.seed, q.rid)
                  for i, q in enumerate(reqs)]
    req_srv, req_one = mk(), mk()
    rays = sum(r.rays for r in req_srv)
    # the same requests as cameras: the server traces each G-buffer itself
    # (2DGRT primary rays with the surfels' materials) and uploads only the
    # environment
    cams = {q.cam: grt.make_camera(*W.camera3(W.rng(3, 10 + q.cam)), 60.0) for q in reqs}
    mats = [torch.from_numpy(a).to(dev) for a in W.surfel_materials(scene.n, seed=0)]
    req_cam = [grt.Request(None, pin(envs[i]), splits[i], q.seed, q.rid, camera=cams[q.cam], H=q.res, W=q.res)
               for i, q in enumerate(reqs)]

    def run_server(replay, share=share, rlist=None):
        rlist = req_srv if rlist is None else rlist
        srv = grt.Server(ctx, scene, mem_budget=48 << 30, max_jobs=16, k=k, slack_per_ray=slack, epoch_rays=epoch,
                         preempt_share=share, attrs=mats)
        warm = grt.Request(pinned[(reqs[0].res, reqs[0].cam)], pin(envs[0]), (1, 1, 1), 1, 1)
        srv.wait(srv.submit(warm))
        t0 = time.perf_counter()
        ids = []
        for q, r in zip(reqs, rlist):
            if replay:
                dt = t0 + q.arrival_s - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            ids.append(srv.submit(r))
        for j in ids:
            st = srv.wait(j, 600.0)
            if st != 0:
                raise grt.GrtError(st, "server request failed")
        times = [srv.times(j) for j in ids]
        lat = [d - s for s, _, d in times]
        span = max(d for _, _, d in times) - min(s for s, _, _ in times)
        stats = srv.stats()
        srv.close()
        return lat, span, stats

    def run_one(replay):
        stream = torch.cuda.current_stream()
        t0 = time.perf_counter()
        lat = []
        for q, r in zip(reqs, req_one):
            if replay:
                dt = t0 + q.arrival_s - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            arrive = t0 + q.arrival_s if replay else t0
            x, n, wo, alb, rough, metal, valid = (a.to(dev, non_blocking=True) for a in r.arrays)
            G = grt.GBuffer(r.H, r.W, x, n, wo, alb, rough, metal, valid)
            E = grt.Env(ctx, r.env.to(dev, non_blocking=True))
            sp = (r.struct.n_cos, r.struct.n_ggx, r.struct.n_env)
            out = grt.render_mis(scene, E, G, split=sp, seed=r.struct.seed, job=r.struct.job, k=k)["rgb"]
            r.out.copy_(out, non_blocking=True)
            stream.synchronize()
            lat.append(time.perf_counter() - arrive)
            del E
        return lat, time.perf_counter() - t0

    pct = lambda a, p: float(np.percentile(np.asarray(a), p))
    res = {}
    log("bench: server leg (replayed arrivals)")
    lat_s, span_s, st = run_server(True)
    log("bench: per-request leg (replayed arrivals)")
    lat_o, span_o = run_one(True)
    same = all(torch.equal(a.out, b.out) for a, b in zip(req_srv, req_one))
    log("bench: server leg (all at once)")
    blat_s, burst_s, bst = run_server(False)
    log("bench: per-request leg (all at once)")
    blat_o, burst_o = run_one(False)
    log("bench: server leg with preemption (replayed arrivals)")
    plat_s, pspan_s, pst = run_server(True, share=0.25)
    log("bench: server leg with camera requests (replayed arrivals)")
    clat_s, cspan_s, _ = run_server(True, rlist=req_cam)
    res = {
        "workload": f"room scene resident; {len(reqs)} requests, Poisson {reqs[-1].arrival_s / max(len(reqs) - 1, 1):.3f}"
                    f" s mean gap, res in {{256,512,768,1024}}^2, spp in {{4..64}}, 128x256 env each",
        "rays": rays,
        "server": {"p50_s": round(pct(lat_s, 50), 4), "p99_s": round(pct(lat_s, 99), 4),
                   "mean_s": round(float(np.mean(lat_s)), 4),
                   "mrays_s_replay": round(rays / span_s / 1e6, 2), "mrays_s_burst": round(rays / burst_s / 1e6, 2),
                   "burst_p50_s": round(pct(blat_s, 50), 4), "burst_p99_s": round(pct(blat_s, 99), 4),
                   "epochs": st["epochs"], "stopped_epochs": st["stopped"]},
        "one_launch_per_request": {"p50_s": round(pct(lat_o, 50), 4), "p99_s": round(pct(lat_o, 99), 4),
                                   "mean_s": round(float(np.mean(lat_o)), 4),
                                   "mrays_s_replay": round(rays / span_o / 1e6, 2),
                                   "mrays_s_burst": round(rays / burst_o / 1e6, 2),
                                   "burst_p50_s": round(pct(blat_o, 50), 4), "burst_p99_s": round(pct(blat_o, 99), 4)},
        "server_preempt_share_0.25": {"p50_s": round(pct(plat_s, 50), 4), "p99_s": round(pct(plat_s, 99), 4),
                                      "mean_s": round(float(np.mean(plat_s)), 4),
                                      "mrays_s_replay": round(rays / pspan_s / 1e6, 2),
                                      "stopped_epochs": pst["stopped"]},
        "server_camera_requests": {"p50_s": round(pct(clat_s, 50), 4), "p99_s": round(pct(clat_s, 99), 4),
                                   "mean_s": round(float(np.mean(clat_s)), 4),
                                   "mrays_s_replay": round(rays / cspan_s / 1e6, 2),
                                   "upload_per_request": "environment only (G-buffer traced by the server)"},
        "images_identical": bool(same),
    }
    if detail:
        res["latency_s"] = [dict(res=q.res, spp=q.spp, arrival=round(q.arrival_s, 3), server=round(a, 4),
                                 one_launch=round(b, 4)) for q, a, b in zip(reqs, lat_s, lat_o)]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=12, help="k-buffer size of the forward")
    ap.add_argument("--k-bwd", type=int, default=8, help="k-buffer size of the backward")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=384, help="pixels of the step the oracle times")
    ap.add_argument("--no-serve", action="store_true", help="skip the relighting-server leg")
    ap.add_argument("--no-stored", action="store_true", help="skip the stored-hit-list backward leg")
    ap.add_argument("--no-relight", action="store_true", help="skip the split-sum relighting leg")
    ap.add_argument("--hit-cap", type=int, default=64, help="hits stored per sample in the stored-list leg")
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-rate", type=float, default=5.9,
                    help="Poisson arrival rate, requests/s (5.9: 70%% load, 0.7 over the 0.119 s mean service time of one launch per request)")
    ap.add_argument("--serve-slack", type=float, default=-1.0, help="server deadline seconds per ray (-1: default)")
    ap.add_argument("--serve-epoch", type=int, default=0, help="server rays per epoch (0: default)")
    ap.add_argument("--count-work", action="store_true", help="recount per-ray work with the oracle and exit")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates the HBM byte counters)")
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

    ev = {}

    def step(record=False):
        for p in params:
            p.grad = None
        img = grt.RenderMISFn.apply(*params, ctx, E, G, SPLIT, SEED, args.k, 1.0 / 255.0, 0, args.k_bwd)
        loss = (img * upstream).sum()
        loss.backward()
        return img

    log("bench: warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)

    # per-kernel timing with events on the launch stream (torch's current one)
    st = torch.cuda.current_stream()
    scene = grt.Scene(ctx, *(p.detach() for p in params))
    eb0, eb1, ef0, ef1, eg0, eg1 = (torch.cuda.Event(enable_timing=True) for _ in range(6))
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

    stored = None
    if not args.no_stored:
        # the same step differentiated from stored hit lists instead of re-traversal
        hits = grt.make_hit_list(gb.npix, spp, args.hit_cap, dev)
        sf, sb = [], []
        for _ in range(max(args.steps // 2, 2)):
            ef0.record(st)
            res = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=args.k, save=True, hits=hits,
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
        ws = None
        for _ in range(max(args.steps // 2, 3)):
            ef0.record(st); E2.prefilter(); ef1.record(st)
            eg0.record(st)
            out = grt.render_relight(scene, E2, *mats, G, split=SPLIT, seed=SEED, k=args.k, workspace=ws)
            eg1.record(st)
            torch.cuda.synchronize()
            pf.append(ef0.elapsed_time(ef1)); rf.append(eg0.elapsed_time(eg1))
        frame = float(np.median(rf))
        # cross-bilateral denoise of the relit frame (radius 3: 7x7 window)
        dgb = [t(gb.depth), G.n, G.valid]
        dn = []
        for _ in range(5):
            ef0.record(st)
            grt.denoise(ctx, out["rgb"], *dgb, gb.H, gb.W)
            ef1.record(st)
            torch.cuda.synchronize()
            dn.append(ef0.elapsed_time(ef1))
        dn_ms = float(np.median(dn))
        # primary-ray G-buffer by 2DGRT of a 1024^2 camera inside the room
        cam_o, cam_d = W.pinhole(*W.camera3(W.rng(3, 2)), 60.0, gb.H, gb.W)
        co, cd = t(cam_o.astype(np.float32)), t(cam_d.astype(np.float32))
        gt = []
        for _ in range(5):
            ef0.record(st)
            gbt = grt.trace_gbuffer(scene, *mats, co, cd, gb.H, gb.W, k=args.k)
            ef1.record(st)
            torch.cuda.synchronize()
            gt.append(ef0.elapsed_time(ef1))
        covered = float(gbt["valid"].float().mean().item())
        # its backward by re-traversal, seeded upstream gradients on every map
        gen = torch.Generator(device=dev).manual_seed(SEED)
        gup = {kk: torch.randn(gbt[kk].shape, generator=gen, device=dev)
               for kk in ("x", "n", "albedo", "rough", "metal", "depth", "rgb")}
        gzs = grt.zero_grads(scene.n, dev)
        gza = dict(albedo=torch.zeros(scene.n, 3, device=dev), rough=torch.zeros(scene.n, device=dev),
                   metal=torch.zeros(scene.n, device=dev))
        gbw = []
        for _ in range(3):
            ef0.record(st)
            grt.trace_gbuffer_backward(scene, *mats, co, cd, gbt, gup, k=args.k, grads=gzs, attr_grads=gza)
            ef1.record(st)
            torch.cuda.synchronize()
            gbw.append(ef0.elapsed_time(ef1))
        del gbt, gup, gzs, gza
        # the same relit frame with the mesh backend answering the query
        # (the room as 46k triangles with per-vertex materials)
        mesh3 = W.mesh3()
        mt = [t(a) for a in (mesh3.verts, mesh3.tris)]
        ma = [t(a) for a in (mesh3.albedo, mesh3.rough, mesh3.metal, mesh3.normal)]
        em0, em1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        em0.record(st)
        M = grt.Mesh(ctx, *mt)
        em1.record(st)
        torch.cuda.synchronize()
        mesh_build_ms = em0.elapsed_time(em1)
        mf = []
        for _ in range(3):
            em0.record(st)
            grt.render_relight_mesh(M, E2, *ma, G, split=SPLIT, seed=SEED)
            em1.record(st)
            torch.cuda.synchronize()
            mf.append(em0.elapsed_time(em1))
        mesh_frame = float(np.median(mf))
        del M
        relight = {"env": "128x256, prefiltered to 16x32 tables at 6 roughness levels + 32x32 DFG",
                   "mesh_backend": {"triangles": int(mesh3.nf), "build_ms": round(mesh_build_ms, 3),
                                    "frame_ms": round(mesh_frame, 3),
                                    "mrays_s": round(rays / (mesh_frame * 1e-3) / 1e6, 2)},
                   "gbuffer_trace_ms": round(float(np.median(gt)), 3), "gbuffer_covered": round(covered, 4),
                   "gbuffer_backward_ms": round(float(np.median(gbw)), 3),
                   "prefilter_ms": round(float(np.median(pf)), 3), "frame_ms": round(frame, 3),
                   "mrays_s": round(rays / (frame * 1e-3) / 1e6, 2),
                   "radiance_fwd_ms": round(fwd_ms, 3),
                   "denoise_ms": round(dn_ms, 4),
                   "denoise_gb_s": round(gb.npix * 41 / (dn_ms * 1e-3) / 1e9, 1)}
        del out, E2

    roofline = None
    if os.path.exists(WORKCOUNT):
        wc = json.load(open(WORKCOUNT))
        bf, bb = bytes_per_ray(wc)
        dominant = "bwd" if bwd_ms >= fwd_ms else "fwd"
        ms = bwd_ms if dominant == "bwd" else fwd_ms
        per_ray = bb if dominant == "bwd" else bf
        achieved = per_ray * rays / (ms * 1e-3) / 1e9
        kname = "k_render_bwd" if dominant == "bwd" else "k_render"
        traffic = l2_hit = None
        if os.path.exists(TRAFFIC):
            tr = json.load(open(TRAFFIC))
            if tr.get("source_hash") == source_hash() and kname in tr.get("kernels", {}):
                traffic = tr["kernels"][kname]["hbm_bytes"]
                l2_hit = tr["kernels"][kname].get("l2_hit")
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, l2_hit=l2_hit, kernel=kname,
                        bytes_per_ray=round(per_ray, 1), kernel_ms=round(ms, 3),
                        traffic_gbs=round(traffic / (ms * 1e-3) / 1e9, 1) if traffic else None,
                        traced_fraction=round(wc["traced_fraction"], 4))

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    serve = None
    if not args.no_serve:
        log("bench: generating relighting requests")
        reqs, gbs, envs = serve_inputs(args.serve_requests, args.serve_rate)
        serve = serve_leg(ctx, scene, args.k, reqs, gbs, envs, args.serve_slack, args.serve_epoch)
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
        "roofline": roofline,
        "stored_hit_lists": stored,
        "relight_split_sum": relight,
        "relight_server": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
