"""GPU parity at full size, in the configuration bench.py times (pair levels
in two alternating arrays, capacity grown on overflow).

Checked against the oracle: every key, the whole sorted order and every node
(the oracle does those in seconds); level-1 pairs and counters restricted to
an evenly spread sample of top-level sub-trees (sub-trees are independent);
closest hits of every ray under the sampled sub-trees, and of a random ray
sample against naive N x M ray tracing.
"""
import numpy as np
import pytest

from conftest import workload
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bits(a):
    a = np.asarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


@pytest.mark.parametrize("name,n_top,n_brute", [("refl_1024", 6, 512), ("mixed_1080p", 4, 192)])
def test_full_size_frame(name, n_top, n_brute):
    import gpu_util as gu
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
    ntop = int(tree["level_cnt"][nl - 1])
    assert g["mesh_tests"] == ntop * wl.scene.n_mesh
    # sampled sub-trees: level-1 pairs, in order
    sub = np.unique(np.linspace(0, ntop - 1, n_top).astype(np.uint32))
    print(f"[fullsize] {name}: oracle traversal of top nodes {sub.tolist()}", flush=True)
    tr = O.traverse(tree, wl.scene, top_subset=sub)
    span = wl.F ** (nl - 1)
    t1, n1 = g["pairs"][1]
    keep = np.isin(n1.astype(np.int64) // span, sub.astype(np.int64))
    assert np.array_equal(t1[keep], tr["pairs"][1][0])
    assert np.array_equal(n1[keep], tr["pairs"][1][1])
    # closest hits of every ray under the sampled sub-trees
    hits = O.closest_hit(h["rays"], ids, wl.B, tr["pairs"][1], wl.scene, wl.t_min)
    ray_span = wl.B * span
    pos = np.concatenate([np.arange(int(s) * ray_span, min((int(s) + 1) * ray_span, h["n"])) for s in sub])
    rid = ids[pos].astype(np.int64)
    assert np.array_equal(g["hit"][0][rid], hits[0][rid])
    for a, b in zip(g["hit"][1:], hits[1:]):
        assert np.allclose(a[rid], b[rid], rtol=1e-5, atol=0)
    # a random ray sample against naive ray tracing
    print(f"[fullsize] {name}: brute force on {n_brute} rays", flush=True)
    rs = np.random.default_rng(3).choice(h["n"], n_brute, replace=False)
    b = O.brute_closest_hit(h["rays"], rs, wl.scene, wl.t_min)
    assert np.array_equal(g["hit"][0][rs], b[0])
    for a, c in zip(g["hit"][1:], b[1:]):
        assert np.allclose(a[rs], c, rtol=1e-5, atol=0)
    print(f"[fullsize] {name}: ok ({g['n']} rays, {len(t1)} level-1 pairs)", flush=True)
    # the last level fused with the final tests (crsh_leaf_hit): the same
    # closest hits and counters as the stored-pair path above
    print(f"[fullsize] {name}: fused last level", flush=True)
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
