"""GPU parity at full size, in the configuration bench.py times (pair levels
in two alternating arrays, capacity grown on overflow).

Checked against the oracle: every key, the whole sorted order and every node
(the oracle does those in seconds); every traversal counter, the level-1
pairs of every top-level sub-tree (SHA-256 per sub-tree, in order) and the
closest hit of every ray (SHA-256 of the triangle ids and of the t, u, v
bits), against the values that tests/golden/make_fullsize.py wrote by
running the oracle over the whole frame; the closest hits of a random ray
sample against naive N x M ray tracing.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from conftest import workload
from oracle import oracle as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bits(a):
    a = np.asarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def _sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a))
    return h.hexdigest()


def check_against_golden(g, gold, F):
    """Counters, per-sub-tree level-1 pair digests and hit digests of a GPU
    frame against the oracle's full-frame values."""
    nl = gold["levels"]
    assert g["n"] == gold["rays"] and g["n_levels"] == nl
    assert [g["tests"][lv] for lv in range(1, nl + 1)] == gold["tests"]
    assert [g["hits"][lv] for lv in range(1, nl + 1)] == gold["hits"]
    for k in ("mesh_tests", "mesh_hits", "final_tests"):
        assert g[k] == gold[k], k
    assert (int(g["meta"].final_u_pass), int(g["meta"].final_uv_pass)) == (gold["u_pass"], gold["uv_pass"])
    t1, n1 = g["pairs"][1]
    assert len(t1) == gold["hits"][0]
    span = F ** (nl - 1)
    top = n1 // np.uint32(span)
    assert bool((top[1:] >= top[:-1]).all()), "level-1 pairs not grouped by top-level sub-tree"
    bounds = np.searchsorted(top, np.arange(gold["top_nodes"] + 1, dtype=np.uint32))
    del top
    for i, p in enumerate(gold["per_top"]):
        b, e = int(bounds[i]), int(bounds[i + 1])
        assert e - b == p["n1"], ("level-1 pair count of sub-tree", i)
        assert _sha(t1[b:e], n1[b:e]) == p["sha"], ("level-1 pairs of sub-tree", i)
    tri, t, u, v = g["hit"]
    assert int((tri >= 0).sum()) == gold["hit_count"]
    assert _sha(tri.astype("<i4")) == gold["hit_tri_sha256"]
    # t, u, v: the kernels repeat the oracle's operations in its order, so the
    # bits agree (a stricter bar than the 1e-5 relative tolerance)
    for a, k in ((t, "t"), (u, "u"), (v, "v")):
        assert _sha(_bits(a).astype("<u4")) == gold[f"hit_{k}_sha256"], k


@pytest.mark.parametrize("name,n_brute", [("refl_1024", 512), ("mixed_1080p", 192)])
def test_full_size_frame(name, n_brute):
    import gpu_util as gu
    gold = json.load(open(os.path.join(GOLDEN, f"fullsize_{name}.json")))
    print(f"[fullsize] {name}: building workload", flush=True)
    wl = workload(name)
    print(f"[fullsize] {name}: GPU frame", flush=True)
    g = gu.run_pipeline(wl, pair_capacity=1 << 26, keep_levels=False)
    print(f"[fullsize] {name}: oracle hash/sort/build", flush=True)
    h = O.hash_rays(wl)
    assert g["n"] == h["n"]
    assert np.array_equal(g["keys"], h["keys"])
    for k in O.RAY_FIELDS:
        assert np.array_equal(_bits(g["rays"][k]), _bits(h["rays"][k])), k
    ks, ids = O.sort_rays(h["keys"], h["ids"])
    assert np.array_equal(g["sorted_ids"], ids)
    tree = O.build_tree(h["rays"], ids, wl.B, wl.F, wl.n)
    assert g["n_levels"] == tree["n_levels"]
    for k in O.NODE_FIELDS:
        assert np.array_equal(_bits(g["nodes"][k]), _bits(tree["nodes"][k])), k
    nl = tree["n_levels"]
    assert int(tree["level_cnt"][nl - 1]) == gold["top_nodes"]
    print(f"[fullsize] {name}: counters, level-1 pairs and hits against the oracle's full frame", flush=True)
    check_against_golden(g, gold, wl.F)
    # a random ray sample against naive ray tracing
    print(f"[fullsize] {name}: brute force on {n_brute} rays", flush=True)
    rs = np.random.default_rng(3).choice(h["n"], n_brute, replace=False)
    b = O.brute_closest_hit(h["rays"], rs, wl.scene, wl.t_min)
    assert np.array_equal(g["hit"][0][rs], b[0])
    for a, c in zip(g["hit"][1:], b[1:]):
        assert np.allclose(a[rs], c, rtol=1e-5, atol=0)
    print(f"[fullsize] {name}: ok ({g['n']} rays, {len(g['pairs'][1][0])} level-1 pairs)", flush=True)
    # the last level fused with the final tests (crsh_leaf_hit): the same
    # closest hits and counters as the stored-pair path above
    print(f"[fullsize] {name}: fused last level", flush=True)
    del g["pairs"]
    f = gu.run_pipeline(wl, pair_capacity=1 << 26, keep_levels=False, leaf_hit=True)
    for a, b in zip(f["hit"], g["hit"]):
        assert np.array_equal(_bits(a), _bits(b))
    for k in ("final_tests", "mesh_tests", "mesh_hits"):
        assert f[k] == g[k], k
    for lv in range(1, nl + 1):
        assert f["tests"][lv] == g["tests"][lv] and f["hits"][lv] == g["hits"][lv], lv


def test_batch_64_full_size():
    """The batched form at full size (64 frames, ~14 M rays, ~3.2 M
    triangles) in the configuration bench.py times (B=16, F=4, n=5,
    hit_block=256): keys, sorted order, nodes and closest hits of the three
    smallest frames against the oracle, and in every frame the closest hits
    of a random ray sample against naive ray tracing."""
    import dataclasses
    from workloads.scenes import make_batch
    from paper_2312_06538_amd.batch import DeviceBatch
    print("[batch fullsize] building 64 frames", flush=True)
    wls = [dataclasses.replace(w, B=16, F=4, n=5) for w in make_batch(0, 64)]
    db = DeviceBatch(wls, 16, 4, 5, 256, pair_capacity=1 << 24)
    m = db.run_with_retry()
    print(f"[batch fullsize] {int(m.n_rays)} rays", flush=True)
    res = db.frame_results(m, with_pairs=False)
    order = sorted(range(len(wls)), key=lambda f: res[f]["n"] * wls[f].scene.m)
    for f in order[:3]:
        wl, r = wls[f], res[f]
        print(f"[batch fullsize] frame {f}: {r['n']} rays, {wl.scene.m} triangles, oracle", flush=True)
        o = O.run_pipeline(wl)
        assert r["n"] == o["hash"]["n"]
        assert np.array_equal(r["keys"], o["hash"]["keys"])
        assert np.array_equal(r["sorted_ids"], o["sorted_ids"])
        for k in O.NODE_FIELDS:
            assert np.array_equal(_bits(r["nodes"][k]), _bits(o["tree"]["nodes"][k])), k
        assert np.array_equal(r["hit"][0], o["hits"][0])
        for a, b in zip(r["hit"][1:], o["hits"][1:]):
            assert np.array_equal(_bits(a), _bits(b))
    rng = np.random.default_rng(5)
    for f, (wl, r) in enumerate(zip(wls, res)):
        if r["n"] == 0:
            continue
        rs = rng.choice(r["n"], min(16, r["n"]), replace=False)
        b = O.brute_closest_hit(r["rays"], rs, wl.scene, wl.t_min)
        assert np.array_equal(r["hit"][0][rs], b[0]), f
        for a, c in zip(r["hit"][1:], b[1:]):
            assert np.allclose(a[rs], c, rtol=1e-5, atol=0), f
    print("[batch fullsize] ok", flush=True)
