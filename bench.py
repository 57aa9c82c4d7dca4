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


def source_hash():
    """Hash of the HIP sources: traffic counters are only valid for the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
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


def cpu_baseline(npx: int = 48):
    """The oracle (brute force, OpenMP) on a bounded sample of the same step."""
    from oracle import oracle as O
    s, gb, env = make_inputs()
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
    return dict(value=rays / (t2 - t0) / 1e6, unit="Mrays/s", cores=cores, kind="oracle",
                sample=f"{npx} valid pixels x {sum(SPLIT)} spp ({rays} rays) of the same step, forward "
                       f"{t1 - t0:.2f}s + backward {t2 - t1:.2f}s, scene/G-buffer generation excluded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
        img = grt.RenderMISFn.apply(*params, ctx, E, G, SPLIT, SEED, args.k, 1.0 / 255.0)
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
        grt.render_mis_backward(scene, E, G, upstream, res["saved"], split=SPLIT, seed=SEED, k=args.k)
        eg1.record(st)
        torch.cuda.synchronize()
        build_ms.append(eb0.elapsed_time(eb1)); fwd_ms.append(ef0.elapsed_time(ef1)); bwd_ms.append(eg0.elapsed_time(eg1))
    build_ms, fwd_ms, bwd_ms = (float(np.median(x)) for x in (build_ms, fwd_ms, bwd_ms))

    roofline = None
    if os.path.exists(WORKCOUNT):
        wc = json.load(open(WORKCOUNT))
        bf, bb = bytes_per_ray(wc)
        dominant = "bwd" if bwd_ms >= fwd_ms else "fwd"
        ms = bwd_ms if dominant == "bwd" else fwd_ms
        per_ray = bb if dominant == "bwd" else bf
        achieved = per_ray * rays / (ms * 1e-3) / 1e9
        kname = "k_render_bwd" if dominant == "bwd" else "k_render"
        traffic = None
        if os.path.exists(TRAFFIC):
            tr = json.load(open(TRAFFIC))
            if tr.get("source_hash") == source_hash() and kname in tr.get("kernels", {}):
                traffic = tr["kernels"][kname]["hbm_bytes"]
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=kname,
                        bytes_per_ray=round(per_ray, 1), kernel_ms=round(ms, 3))

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline()

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
                   "rays_per_step": rays, "k": args.k},
        "fwd_mrays_s": round(rays / (fwd_ms * 1e-3) / 1e6, 2),
        "phase_ms": {"build": round(build_ms, 3), "render_fwd": round(fwd_ms, 3), "render_bwd": round(bwd_ms, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
