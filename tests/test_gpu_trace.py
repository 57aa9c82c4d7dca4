"""GPU parity of the scene build and Trace against the CPU oracle (Sec. 3.2:
Eq. raytracing_intersection, the Gaussian influence, Eq. trace).

Hit sets, order and depths are compared bit for bit (both sides decide in the
same single-precision operation order); radiance and transmittance within
1e-4 relative / 1e-5 absolute.  A ray is excused only where the oracle's
single-precision transmittance came within 1e-5 (relative) of the cutoff,
since the two exp implementations may differ in the last ulp there."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2607_22780_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-4, 1e-5


@pytest.fixture(scope="module")
def grt_ctx():
    from paper_2607_22780_amd import grt
    return grt, grt.Context(0)


def run_gpu(grt, ctx, s, origins, dirs, t_min=0.0, t_max=np.inf, k=16, cap=64, sky=(0.5, 0.5, 0.5)):
    from gpu_util import t, scene_tensors
    scene = grt.Scene(ctx, *scene_tensors(s))
    out = grt.trace(scene, t(origins), t(dirs), t_min=t_min, t_max=t_max, k=k, dump_cap=cap, sky=sky)
    torch.cuda.synchronize()
    return {kk: v.cpu().numpy() for kk, v in out.items()}, scene


def compare(gpu, ref, cap, excuse_margin=1e-5, max_excused=0.001):
    nr = len(ref["T"])
    stop_edge = ref["margins"][:, 3] < excuse_margin
    ok = ~stop_edge
    # hit lists: ids and depths bit-exact
    kk = min(cap, ref["ids"].shape[1])
    np.testing.assert_array_equal(gpu["ids"][ok, :kk], ref["ids"][ok, :kk])
    np.testing.assert_array_equal(gpu["tau"][ok, :kk].view(np.uint32), ref["tau"][ok, :kk].view(np.uint32))
    np.testing.assert_array_equal(gpu["nhit"][ok], ref["nhit"][ok])
    np.testing.assert_allclose(gpu["rgb"][ok], ref["C"][ok], rtol=RTOL, atol=ATOL)
    np.testing.assert_allclose(gpu["T"][ok], ref["T"][ok], rtol=RTOL, atol=ATOL)
    np.testing.assert_allclose(gpu["L"][ok], ref["L"][ok], rtol=RTOL, atol=ATOL)
    assert stop_edge.sum() <= max(1, max_excused * nr), stop_edge.sum()
    # excused rays: still a valid prefix of the same ordered hit list
    for r in np.nonzero(stop_edge)[0]:
        m = min(gpu["nhit"][r], ref["nhit"][r], kk)
        np.testing.assert_array_equal(gpu["ids"][r, :m], ref["ids"][r, :m])


def test_config0_trace_parity(grt_ctx):
    """The 4,096-surfel workload, all 32,768 rays."""
    grt, ctx = grt_ctx
    s = W.scene0(); r = W.rays0()
    ref = O.trace(s, r.origins, r.dirs, cap=64)
    gpu, _ = run_gpu(grt, ctx, s, r.origins, r.dirs, cap=64)
    compare(gpu, ref, 64)


@pytest.mark.parametrize("k", [1, 2, 4, 8, 12, 32])
def test_results_do_not_depend_on_k(grt_ctx, k):
    """k-buffer size changes rounds, not results: bitwise equal to k = 16."""
    grt, ctx = grt_ctx
    s = W.scene0(n=2000, seed=1); r = W.rays0(res=24, per=8, seed=1)
    a, _ = run_gpu(grt, ctx, s, r.origins, r.dirs, k=16, cap=48)
    b, _ = run_gpu(grt, ctx, s, r.origins, r.dirs, k=k, cap=48)
    for key in ("rgb", "T", "nhit", "ids", "tau"):
        np.testing.assert_array_equal(a[key], b[key])


@pytest.mark.parametrize("n,res,per", [(1, 7, 3), (2, 9, 5), (3, 11, 7), (257, 13, 9), (5000, 37, 7)])
def test_small_and_ragged(grt_ctx, n, res, per):
    """Tiny trees (1-3 leaves), ray counts that are not multiples of the block."""
    grt, ctx = grt_ctx
    s = W.scene0(n=n, seed=2)
    s = W.Surfels(s.means * 0.3, s.scales * 5, s.quats, s.opacity, s.rgb)
    s = W.Surfels(*(np.ascontiguousarray(a, dtype=np.float32) for a in s.arrays()))
    r = W.rays0(res=res, per=per, seed=2)
    ref = O.trace(s, r.origins * 0.5, r.dirs, cap=32)
    gpu, _ = run_gpu(grt, ctx, s, (r.origins * 0.5).astype(np.float32), r.dirs, cap=32)
    compare(gpu, ref, 32)
    assert ref["nhit"].sum() > 0


def test_empty_scene(grt_ctx):
    grt, ctx = grt_ctx
    z = lambda *sh: np.zeros(sh, np.float32)
    s = W.Surfels(z(0, 3), z(0, 2), z(0, 4), z(0), z(0, 3))
    r = W.rays0(res=5, per=3)
    gpu, _ = run_gpu(grt, ctx, s, r.origins, r.dirs, cap=4, sky=(0.1, 0.2, 0.3))
    assert np.all(gpu["T"] == 1.0) and np.all(gpu["rgb"] == 0.0) and np.all(gpu["nhit"] == 0)
    np.testing.assert_allclose(gpu["L"], np.broadcast_to(np.float32([0.1, 0.2, 0.3]), gpu["L"].shape))


def test_stacked_and_occluded(grt_ctx):
    """Closed forms on the GPU: 40 stacked equal-alpha surfels; an opaque
    surfel hit at its centre gives T = 0 exactly and hides what is behind."""
    grt, ctx = grt_ctx
    nsurf, alpha = 40, 0.3
    c = np.float32([0.2, 0.6, 0.9])
    s = W.Surfels(np.float32([(0, 0, -(k + 1.0)) for k in range(nsurf)]), np.full((nsurf, 2), 0.2, np.float32),
                  np.tile(np.float32([1, 0, 0, 0]), (nsurf, 1)), np.full(nsurf, alpha, np.float32),
                  np.tile(c, (nsurf, 1)))
    o = np.zeros((3, 3), np.float32); d = np.tile(np.float32([0, 0, -1]), (3, 1))
    gpu, _ = run_gpu(grt, ctx, s, o, d, cap=nsurf, sky=(0, 0, 0))
    T = (1 - alpha) ** 20
    np.testing.assert_allclose(gpu["T"], T, rtol=1e-5)
    np.testing.assert_allclose(gpu["rgb"], np.tile(c * (1 - T), (3, 1)), rtol=1e-5)
    assert np.all(gpu["nhit"] == 20)
    s2 = W.Surfels(np.float32([(0, 0, -3.0), (0, 0, -1.0)]), np.full((2, 2), 0.2, np.float32),
                   np.tile(np.float32([1, 0, 0, 0]), (2, 1)), np.float32([0.6, 1.0]),
                   np.float32([(1, 1, 1), (0.3, 0.4, 0.5)]))
    gpu2, _ = run_gpu(grt, ctx, s2, o[:1], d[:1], cap=4)
    assert gpu2["T"][0] == 0.0 and gpu2["nhit"][0] == 1 and gpu2["ids"][0, 0] == 1
    np.testing.assert_array_equal(gpu2["rgb"][0], np.float32([0.3, 0.4, 0.5]))


def test_bvh_structure(grt_ctx):
    """The LBVH is a binary tree over all leaves; every node's child boxes
    contain their subtrees' leaf boxes; records hold a permutation of ids, and
    the stored parameters the backward reads by record position (centre,
    opacity, s_u, s_v, quaternion, colour) are the caller's, bit for bit."""
    grt, ctx = grt_ctx
    from gpu_util import scene_tensors
    s = W.scene1(n=20000, seed=0)
    scene = grt.Scene(ctx, *scene_tensors(s))
    torch.cuda.synchronize()
    arr = {k: v.cpu().numpy() for k, v in scene.arrays().items()}
    n = s.n
    rec, nd, lb = arr["records"], arr["nodes"], arr["leaf_boxes"]
    ids = rec[:, 11].view(np.uint32)
    assert np.array_equal(np.sort(ids), np.arange(n, dtype=np.uint32))
    assert np.array_equal(arr["order"].view(np.uint32), ids)
    means, scales, quats, opac, rgb = (np.asarray(a, np.float32) for a in s.arrays())
    np.testing.assert_array_equal(rec[:, 0:3], means[ids])
    np.testing.assert_array_equal(rec[:, 7], opac.reshape(-1)[ids])
    np.testing.assert_array_equal(rec[:, 15], scales[ids, 0])
    np.testing.assert_array_equal(arr["colours"][:, 3], scales[ids, 1])
    np.testing.assert_array_equal(arr["colours"][:, 0:3], rgb[ids])
    np.testing.assert_array_equal(arr["quats"], quats[ids])
    ch = nd[:, 12:14].view(np.int32)
    seen_leaf = np.zeros(n, bool)
    seen_node = np.zeros(n - 1, bool)
    stack = [(0, None)]
    while stack:
        i, _ = stack.pop()
        assert not seen_node[i]
        seen_node[i] = True
        for side in range(2):
            c = ch[i, side]
            box = nd[i, 6 * side:6 * side + 6]
            if c < 0:
                p = -c - 1
                assert not seen_leaf[p]
                seen_leaf[p] = True
                assert np.all(box[:3] <= lb[p, :3]) and np.all(box[3:] >= lb[p, 3:])
            else:
                sub = nd[c]
                lo = np.minimum(sub[0:3], sub[6:9]); hi = np.maximum(sub[3:6], sub[9:12])
                assert np.all(box[:3] <= lo) and np.all(box[3:] >= hi)
                stack.append((c, i))
    assert seen_leaf.all() and seen_node.all()


@pytest.mark.parametrize("which", ["scene1", "scene3"])
def test_full_scene_trace_parity_sampled(grt_ctx, which):
    """The 300k / 1M-surfel scenes: all G-buffer hemisphere rays traced on the
    GPU, a seeded sample of 1,024 of them brute-forced by the oracle."""
    grt, ctx = grt_ctx
    if which == "scene1":
        s = W.scene1(); gb = W.gbuffer1(200, 200)
    else:
        s = W.scene3(); gb = W.gbuffer3(256, 256)
    valid = np.nonzero(gb.valid)[0]
    g = np.random.default_rng(11)
    org = np.repeat(gb.x[valid], 4, axis=0)
    dirs = W.hemisphere_dirs(g, gb.n[valid], 4).astype(np.float32)
    gpu, _ = run_gpu(grt, ctx, s, org, dirs, t_min=1e-3, cap=64)
    pick = np.sort(g.choice(len(org), 1024, replace=False))
    ref = O.trace(s, org[pick], dirs[pick], t_min=1e-3, cap=64)
    sub = {k: v[pick] for k, v in gpu.items()}
    compare(sub, ref, 64, max_excused=0.001)
    assert ref["nhit"].mean() > 1.0


def test_negative_per_ray_t_min_is_zero(grt_ctx):
    """Per-ray t_min below zero (or NaN) is read as 0, as the oracle does."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene0(n=1500, seed=8)
    r = W.rays0(res=10, per=4, seed=8)
    tm = np.random.default_rng(0).uniform(-2.0, -1e-3, r.n).astype(np.float32)
    tm[::7] = np.nan
    scene = grt.Scene(ctx, *scene_tensors(s))
    a = grt.trace(scene, t(r.origins), t(r.dirs), t_min=0.0, dump_cap=32)
    b = grt.trace(scene, t(r.origins), t(r.dirs), t_min=t(tm), t_max=t(np.full(r.n, np.inf, np.float32)), dump_cap=32)
    torch.cuda.synchronize()
    for k in ("rgb", "T", "nhit", "ids", "tau"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy())
    ref = O.trace(s, r.origins, r.dirs, t_min=tm, t_max=np.full(r.n, np.inf, np.float32), cap=32)
    compare({kk: v.cpu().numpy() for kk, v in b.items()}, ref, 32)


def test_trace_under_an_environment(grt_ctx):
    """grt_trace_opts.env: L = c_rt + T L_env(d) against the oracle."""
    grt, ctx = grt_ctx
    from gpu_util import t, scene_tensors
    s = W.scene0(); r = W.rays0()
    env = W.envmap(64, 128, seed=6)
    scene = grt.Scene(ctx, *scene_tensors(s))
    E = grt.Env(ctx, t(env))
    out = grt.trace(scene, t(r.origins), t(r.dirs), env=E)
    torch.cuda.synchronize()
    ref = O.trace(s, r.origins, r.dirs)
    L = O.trace_env(s, r.origins, r.dirs, env)
    ok = ref["margins"][:, 3] >= 1e-5
    np.testing.assert_allclose(out["L"].cpu().numpy()[ok], L[ok], rtol=RTOL, atol=ATOL)
    np.testing.assert_allclose(out["T"].cpu().numpy()[ok], ref["T"][ok], rtol=RTOL, atol=ATOL)
    assert ok.mean() > 0.999


@pytest.mark.parametrize("n", [2, 3, 5, 257, 20000])
def test_wide_bvh_structure(grt_ctx, n):
    """The 4-wide hierarchy the traversal walks: every node has 2..4
    children, every leaf is reached exactly once, every node is used once,
    and each child box is exactly the union of its subtree's leaf boxes (the
    binary LBVH's boxes, regrouped)."""
    grt, ctx = grt_ctx
    from gpu_util import scene_tensors
    s = W.scene1(n=max(n, 2), seed=1).subset(np.arange(n))
    scene = grt.Scene(ctx, *scene_tensors(s))
    torch.cuda.synchronize()
    arr = {k: v.cpu().numpy() for k, v in scene.arrays().items()}
    lb, n4 = arr["leaf_boxes"], int(arr["nodes4_count"][0])
    nd4 = arr["nodes4"][:n4]
    assert 1 <= n4 <= n - 1
    boxes = nd4[:, :24].reshape(n4, 6, 4)  # [node, lo.x..hi.z, child]
    ch = nd4[:, 24:28].view(np.int32)
    cnt = nd4[:, 28].view(np.int32)
    seen_leaf = np.zeros(n, bool)
    seen_node = np.zeros(n4, bool)

    def walk(i):
        assert not seen_node[i]
        seen_node[i] = True
        assert 2 <= cnt[i] <= 4
        lo = np.full(3, np.inf, np.float32); hi = np.full(3, -np.inf, np.float32)
        for j in range(4):
            c = ch[i, j]
            if j >= cnt[i]:
                assert c == 0x7fffffff
                continue
            if c < 0:
                p = -c - 1
                assert not seen_leaf[p]
                seen_leaf[p] = True
                sub_lo, sub_hi = lb[p, :3], lb[p, 3:]
            else:
                sub_lo, sub_hi = walk(c)
            np.testing.assert_array_equal(boxes[i, :3, j], sub_lo)
            np.testing.assert_array_equal(boxes[i, 3:, j], sub_hi)
            lo = np.minimum(lo, sub_lo); hi = np.maximum(hi, sub_hi)
        return lo, hi

    import sys
    sys.setrecursionlimit(10000)
    walk(0)
    assert seen_leaf.all() and seen_node.all()
