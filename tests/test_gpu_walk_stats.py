"""Walk statistics (grt_walk_stats) of the instrumented library
(libgrt_stats.so: the same sources compiled with -DGRT_STATS) on the MIS
render and its re-traversal backward (Sec. 3.1 traversal, Sec. 3.4.1 Eq.
mis).  The counts are checked against what fixes them: the rays traced are
the samples with a nonzero mixture pdf, the composited hits sum to the
stored hit counts, the backward re-traversal composites exactly the
forward's hits, the stored-list forward walks as the plain one does, and the
lane counts bound the per-ray counts.  The instrumented kernels give the
product library's images and hit counts.  The product library reports that
it keeps no statistics."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_2607_22780_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SPLIT, SEED, CAP = (4, 2, 2), 7, 512


def case():
    s = W.scene1(n=6000, seed=0, s_lo=0.01, s_hi=0.05)
    gb = W.gbuffer1(64, 48, seed=0)
    env = W.envmap(32, 64, seed=0)
    return s, gb, env


def run(grt, out_dir=None):
    """Forward with stored hit lists and the sample dump, the plain forward,
    and the re-traversal backward with a unit upstream gradient; with the
    instrumented library also the walk statistics after each."""
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    s, gb, env = case()
    ctx = grt.Context(0)
    scene = grt.Scene(ctx, *(t(a) for a in s.arrays()))
    E = grt.Env(ctx, t(env))
    G = grt.GBuffer.from_numpy(gb, dev)
    spp = sum(SPLIT)
    hits = grt.make_hit_list(gb.npix, spp, CAP, dev)
    stats = out_dir is not None
    if stats:
        grt.walk_stats(ctx, reset=True)
    a = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=12, save=True, dump=True, hits=hits, hit_cap=CAP)
    st_list = grt.walk_stats(ctx, reset=True)["forward"] if stats else None
    b = grt.render_mis(scene, E, G, split=SPLIT, seed=SEED, k=12, save=True)
    st_fwd = grt.walk_stats(ctx, reset=True)["forward"] if stats else None
    grt.render_mis_backward(scene, E, G, torch.ones(gb.npix, 3, device=dev), b["saved"], split=SPLIT, seed=SEED,
                            k=8)
    st_bwd = grt.walk_stats(ctx, reset=True)["backward"] if stats else None
    torch.cuda.synchronize()
    res = dict(rgb_list=a["rgb"].cpu().numpy(), rgb=b["rgb"].cpu().numpy(),
               counts=hits[:gb.npix * spp].cpu().numpy(), q=a["dump"][..., 3].reshape(-1).cpu().numpy())
    if stats:
        np.savez(os.path.join(out_dir, "stats_run.npz"), **res)
        return dict(list=st_list, fwd=st_fwd, bwd=st_bwd)
    return res


CHILD = """
import json, sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
from paper_2607_22780_amd import grt
grt.load_library(grt.STATS_LIB_PATH)
import test_gpu_walk_stats as T
print(json.dumps(T.run(grt, {out!r})), flush=True)
"""


@pytest.fixture(scope="module")
def instrumented(tmp_path_factory):
    from paper_2607_22780_amd import grt
    assert os.path.exists(grt.STATS_LIB_PATH), "libgrt_stats.so is built by __graft_entry__.build()"
    out = str(tmp_path_factory.mktemp("walk"))
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), out=out)
    print("walk stats: instrumented library in a child process", flush=True)
    p = subprocess.run([sys.executable, "-u", "-c", code], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr[-4000:]
    st = json.loads(p.stdout.strip().splitlines()[-1])
    res = dict(np.load(os.path.join(out, "stats_run.npz")))
    return st, res


def test_product_library_keeps_no_statistics():
    from paper_2607_22780_amd import grt
    ctx = grt.Context(0)
    with pytest.raises(grt.GrtError) as e:
        grt.walk_stats(ctx)
    assert e.value.code == grt.ERR_INVALID


def test_instrumented_kernels_give_the_product_results(instrumented):
    from paper_2607_22780_amd import grt
    _, got = instrumented
    want = run(grt)
    np.testing.assert_array_equal(got["counts"], want["counts"])
    np.testing.assert_array_equal(got["q"], want["q"])
    for key in ("rgb_list", "rgb"):
        np.testing.assert_allclose(got[key], want[key], rtol=1e-5, atol=1e-6, err_msg=key)


def test_walk_counts(instrumented):
    st, res = instrumented
    traced = int((res["q"] != 0).sum())
    comps = int(res["counts"].astype(np.int64).sum())
    assert traced > 0 and comps > 0 and res["counts"].max() <= CAP
    fwd, lst, bwd = st["fwd"], st["list"], st["bwd"]
    for d in (fwd, lst, bwd):
        assert d["rays"] == traced
        assert d["composites"] == comps
        assert d["rounds"] >= d["rays"] and d["leaf_tests"] >= d["composites"]
        assert d["restarts"] <= d["rounds"] - d["rays"]
        # a lane walks at most one node, and runs at most one surfel step, per step
        assert d["node_visits"] <= d["active_lanes"]
        assert d["leaf_tests"] + d["composites"] <= d["active_lanes"]
        assert d["active_lanes"] <= 64 * d["wave_steps"]
    # storing the hit lists does not change the walk
    for key in ("node_visits", "leaf_tests", "rounds", "restarts", "deferred"):
        assert lst[key] == fwd[key], key
    # rays with more hits than the 12-entry buffer take further rounds
    assert fwd["rounds"] > fwd["rays"] and int((res["counts"] > 12).sum()) > 0
