"""The GPU tree builder (Morton keys, radix sort, level-by-level splitting and
pair-frontier lists as HIP kernels) against the host reference builder, bit
for bit: frame, sorted keys, permutation, boxes, level offsets and the four
pair lists, at the N = 10^6 three-layer workload, on every geometry of the
batched workload and on edge cases; the same errors for invalid point sets;
and the lists' completeness (every source point reaches every target leaf
exactly once through the lists of the leaf and its ancestors).
"""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
K3 = (2 * math.pi * 80, 2 * math.pi * 120, 2 * math.pi * 100)
FIELDS = ("frame", "keys", "perm", "boxes", "lev_begin", "fv", "iv", "fu", "iu")


def _both(hf, k, ifs, xy, **opts):
    import torch
    pts = torch.tensor(np.asarray(xy, float), dtype=torch.float64, device="cuda:0")
    g = hf.build_tree(k, ifs, pts, builder=hf.HFMM_TREE_GPU, **opts)
    h = hf.build_tree(k, ifs, pts, builder=hf.HFMM_TREE_HOST, **opts)
    return g, h


def _assert_same(g, h, label):
    for key in ("levels", "top", "boxes_count"):
        assert g[key] == h[key], "%s: %s %s vs %s" % (label, key, g[key], h[key])
    for f in FIELDS:
        assert g[f].shape == h[f].shape, "%s: %s shape %s vs %s" % (label, f, g[f].shape, h[f].shape)
        assert np.array_equal(g[f], h[f]), "%s: %s differs" % (label, f)


def _complete(t, lists):
    """Every target leaf reaches every point exactly once through the pairs
    (A, s) of `lists` whose target A is the leaf or one of its ancestors (the
    sources contribute their points [begin, end))."""
    boxes, n = t["boxes"], t["n"]
    by_t = {}
    for name in lists:
        for a, s in t[name]:
            by_t.setdefault(int(a), []).append(int(s))
    for b in np.nonzero(boxes[:, 11])[0]:
        cover = np.zeros(n, np.int32)
        a = int(b)
        while a >= 0:
            for s in by_t.get(a, []):
                cover[boxes[s, 3]:boxes[s, 4]] += 1
            a = int(boxes[a, 5])
        assert cover.min() == 1 and cover.max() == 1, "leaf %d: points covered %d..%d times" % (
            b, cover.min(), cover.max())


def test_tree_n1e6_matches_host(gpu_lib):
    w = workloads.three_layer_ellipses(n=1_000_000)
    g, h = _both(gpu_lib, w.k, w.interfaces, w.xy, leaf_size=w.leaf)
    print("N=1e6: %d boxes, %d levels, top %d, |fv| %d |iv| %d |fu| %d |iu| %d" % (
        g["boxes_count"], g["levels"], g["top"], len(g["fv"]), len(g["iv"]), len(g["fu"]), len(g["iu"])))
    _assert_same(g, h, "N=1e6")
    assert np.all(np.diff(g["keys"].astype(np.uint64)) >= 0)
    assert np.array_equal(np.sort(g["perm"]), np.arange(w.n))


def test_tree_batched_geometries_match_host(gpu_lib):
    for gi in range(32):
        w = workloads.batched_geometry(gi, nrhs=1)
        g, h = _both(gpu_lib, w.k, w.interfaces, w.xy, leaf_size=w.leaf)
        _assert_same(g, h, "geometry %d" % gi)


@pytest.mark.parametrize("case", ["uniform", "line", "tiny1", "tiny2", "close_pair", "deep_leaf1",
                                  "no_refine", "max_level3", "top2", "two_layer_config"])
def test_tree_edge_cases_match_host_and_are_complete(gpu_lib, case):
    rng = workloads.rng_for(1703, 9136, 61, len(case))
    k, ifs = (8 * math.pi, 12 * math.pi), (0.0,)
    opts = dict(leaf_size=32)
    if case == "uniform":
        xy = workloads.uniform_box(rng, 3000, 0.0, 1.0, 0.05, 1.05)
    elif case == "line":  # every x equal: the root side comes from y
        xy = np.stack([np.full(500, 0.3), rng.uniform(0.1, 0.9, 500)], 1)
    elif case == "tiny1":
        xy = np.array([[0.25, 0.5]])
    elif case == "tiny2":
        xy = np.array([[0.25, 0.5], [0.75, 0.6]])
    elif case == "close_pair":  # two points in one key cell, not coincident
        xy = workloads.uniform_box(rng, 200, 0.0, 1.0, 0.05, 1.05)
        xy = np.vstack([xy, xy[:1] + np.array([[1e-13, 0.0]])])
    elif case == "deep_leaf1":
        xy = workloads.uniform_box(rng, 400, 0.0, 1.0, 0.05, 1.05)
        opts = dict(leaf_size=1)
    elif case == "no_refine":
        xy = workloads.uniform_box(rng, 2000, 0.0, 1.0, 0.01, 1.01)
        opts = dict(leaf_size=16, interface_refine=0, leaf_kb=0.0)
    elif case == "max_level3":
        xy = workloads.uniform_box(rng, 2000, 0.0, 1.0, 0.05, 1.05)
        opts = dict(leaf_size=8, max_level=3)
    elif case == "top2":
        xy = workloads.ellipse_points(rng, 5000, 8, (0.55, 0.9), 0.51)
        k, ifs = K3, (0.5, 0.0)
        opts = dict(leaf_size=32, top_level=2)
    else:
        w = workloads.two_layer_uniform(n=1024, seed=1)
        xy, k, ifs = w.xy, w.k, w.interfaces
    g, h = _both(gpu_lib, k, ifs, xy, **opts)
    _assert_same(g, h, case)
    if g["n"] <= 5000:
        _complete(g, ("fv", "fu"))
        _complete(g, ("iv", "iu"))


@pytest.mark.parametrize("bad", ["nan", "below", "coincident"])
def test_tree_domain_errors_agree(gpu_lib, bad):
    import torch
    rng = workloads.rng_for(1703, 9136, 62)
    xy = workloads.uniform_box(rng, 300, 0.0, 1.0, 0.05, 1.05)
    if bad == "nan":
        xy[17, 0] = float("nan")
    elif bad == "below":
        xy[23, 1] = -0.01
        xy[40, 1] = float("inf")
    else:
        xy[200] = xy[31]
    pts = torch.tensor(xy, dtype=torch.float64, device="cuda:0")
    msgs = []
    for builder in (gpu_lib.HFMM_TREE_GPU, gpu_lib.HFMM_TREE_HOST):
        with pytest.raises(gpu_lib.HFMMError) as ei:
            gpu_lib.build_tree((8 * math.pi,), (0.0,), pts, builder=builder)
        msgs.append(str(ei.value))
    print(bad, msgs[0])
    assert "DOMAIN" in msgs[0] and msgs[0] == msgs[1]
