"""GPU parity: every HIP stage against the oracle, through the C-ABI.

Bar: bit-exact keys, ids, rays, sorted order, node arrays and pair levels
(in order), exact counters, exact closest-hit triangle ids; t, u, v within
1e-5 relative (they come out bit-equal, since both sides do the same
binary32 operations).  Sizes: the 128x128 shadow workload, and reduced
versions of the 1024x1024 and 1920x1080 workloads that span many tiles and
leave ragged tails.
"""
import numpy as np
import pytest

from conftest import small, oracle_run, workload
from oracle import oracle as O

pytestmark = pytest.mark.gpu

CASES = ["shadow_128", "refl_96", "mixed_128x72"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06538_amd import crsh
    crsh.lib()


def _gu():
    import gpu_util
    return gpu_util


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint32) if a.dtype == np.float32 else a,
                                                 b.view(np.uint32) if b.dtype == np.float32 else b)


@pytest.mark.parametrize("name", CASES)
def test_hash_bit_exact(name):
    base, kw = small(name)
    print(f"[hash] {name}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)["hash"]
    g = _gu().gpu_hash(wl)
    assert g["status"] == 0
    assert g["n"] == o["n"]
    assert _same(g["keys"], o["keys"])
    assert _same(g["ids"], o["ids"])
    for k in O.RAY_FIELDS:
        assert _same(g["rays"][k], o["rays"][k]), k
    assert _same(g["rays"]["pix"], o["rays"]["pix"])


@pytest.mark.parametrize("n,span,cap", [(0, 7, None), (1, 7, None), (4095, 1 << 32, None), (4096, 3, None),
                                        (4097, 1 << 20, None), (8191, 1 << 32, None), (8192, 5, None),
                                        (8193, 1 << 20, None), (50000, 1 << 32, None), (123457, 97, None),
                                        (300001, 1 << 16, None),
                                        # several million keys; capacity well above the keys
                                        ((1 << 22) + 4097, 1 << 32, None), (5000001, 193, None),
                                        (100000, 1 << 32, 1 << 22), (0, 7, 1 << 22)])
def test_sort_bit_exact(n, span, cap):
    print(f"[sort] n={n} span={span} cap={cap}", flush=True)
    rng = np.random.default_rng(n + span % 1000)
    keys = rng.integers(0, span, size=n, dtype=np.uint64).astype(np.uint32)
    ids = np.arange(n, dtype=np.uint32)
    ok, oi = O.sort_rays(keys, ids)
    gk, gi = _gu().gpu_sort(keys, ids, capacity=cap if cap is not None else n + 1000)
    assert _same(gk, ok) and _same(gi, oi)


def test_sort_digit_skipping_and_values():
    gu = _gu()
    rng = np.random.default_rng(5)
    # every key equal: all passes skipped, plain copy
    keys = np.full(10000, 0xDEADBEEF, np.uint32)
    ids = rng.permutation(10000).astype(np.uint32)
    gk, gi = gu.gpu_sort(keys, ids)
    assert _same(gi, ids) and _same(gk, keys)
    # only the top byte varies: three passes skipped
    keys = (rng.integers(0, 256, 20000).astype(np.uint32) << 24) | 0x00123456
    ok, oi = O.sort_rays(keys, ids[:0].tolist() or np.arange(20000, dtype=np.uint32))
    gk, gi = gu.gpu_sort(keys, np.arange(20000, dtype=np.uint32))
    assert _same(gk, ok) and _same(gi, oi)
    # arbitrary values travel with their keys, equal keys keep input order
    keys = rng.integers(0, 40, 30000).astype(np.uint32)
    vals = rng.permutation(30000).astype(np.uint32)
    ok, oi = O.sort_rays(keys, vals)
    gk, gi = gu.gpu_sort(keys, vals)
    assert _same(gk, ok) and _same(gi, oi)


@pytest.mark.parametrize("name", CASES)
def test_sort_of_workload_keys(name):
    base, kw = small(name)
    o = oracle_run(base, **kw)
    gk, gi = _gu().gpu_sort(o["hash"]["keys"], o["hash"]["ids"])
    assert _same(gk, o["sorted_keys"]) and _same(gi, o["sorted_ids"])


@pytest.mark.parametrize("n,span", [(0, 7), (1, 7), (4096, 3), (4097, 1 << 20), (50000, 1 << 32),
                                    (300001, 1 << 16)])
def test_sort_chunked_bit_exact(n, span):
    """Compression -> chunk sort -> decompression gives the stable order."""
    print(f"[sort chunked] n={n} span={span}", flush=True)
    rng = np.random.default_rng(n + span % 997)
    keys = rng.integers(0, span, size=n, dtype=np.uint64).astype(np.uint32)
    # long runs of equal keys, as coherent rays give
    keys = np.repeat(keys, rng.integers(1, 40, size=n))[:n] if n else keys
    ids = rng.permutation(n).astype(np.uint32)
    ok, oi = O.sort_rays(keys, ids)
    gk, gi = _gu().gpu_sort(keys, ids, capacity=n + 777, chunked=True)
    assert _same(gk, ok) and _same(gi, oi)


@pytest.mark.parametrize("name", CASES)
def test_sort_chunked_of_workload_keys(name):
    base, kw = small(name)
    o = oracle_run(base, **kw)
    gk, gi = _gu().gpu_sort(o["hash"]["keys"], o["hash"]["ids"], chunked=True)
    assert _same(gk, o["sorted_keys"]) and _same(gi, o["sorted_ids"])


def _check_tree(g, o):
    assert g["n_levels"] == o["n_levels"]
    assert _same(g["level_cnt"], o["level_cnt"])
    assert _same(g["level_off"], o["level_off"])
    for k in O.NODE_FIELDS:
        assert _same(g["nodes"][k], o["nodes"][k]), k


@pytest.mark.parametrize("name", CASES)
def test_build_bit_exact(name):
    base, kw = small(name)
    print(f"[build] {name}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    g = _gu().gpu_build(o["hash"]["rays"], o["sorted_ids"], wl.B, wl.F, wl.n)
    _check_tree(g, o["tree"])
    sid = o["sorted_ids"].astype(np.int64)
    for k in O.RAY_FIELDS:
        assert _same(g["sorted"][k], o["hash"]["rays"][k][sid]), k


@pytest.mark.parametrize("B,F,n", [(1, 2, 3), (4, 2, 6), (5, 7, 4), (8, 8, 2), (32, 3, 3), (16, 16, 2),
                                   (16, 4, 1)])
def test_build_shapes(B, F, n):
    base, kw = small("refl_96")
    print(f"[build-shape] B={B} F={F} n={n}", flush=True)
    o = oracle_run(base, **kw)
    ot = O.build_tree(o["hash"]["rays"], o["sorted_ids"], B, F, n)
    g = _gu().gpu_build(o["hash"]["rays"], o["sorted_ids"], B, F, n)
    _check_tree(g, ot)


def test_build_empty_and_tiny():
    gu = _gu()
    r = {k: np.zeros(3, np.float32) for k in O.RAY_FIELDS}
    r["dz"][:] = 1.0
    r["pix"] = np.zeros(3, np.uint32)
    g = gu.gpu_build(r, np.arange(3, dtype=np.uint32), 8, 4, 4, n_rays=0)
    assert g["n_levels"] == 0
    g = gu.gpu_build(r, np.arange(3, dtype=np.uint32), 8, 4, 4, n_rays=3)
    o = O.build_tree(r, np.arange(3, dtype=np.uint32), 8, 4, 4)
    _check_tree(g, o)


@pytest.mark.parametrize("name", CASES)
def test_traverse_bit_exact(name):
    base, kw = small(name)
    print(f"[traverse] {name}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    cap = max(len(t) for t, _ in o["trav"]["pairs"].values()) + 4096
    g = _gu().gpu_traverse(o["tree"], wl.scene, wl.B, wl.F, capacity=cap)
    assert g["status"] == 0
    tr = o["trav"]
    for lv in tr["pairs"]:
        assert _same(g["pairs"][lv][0], tr["pairs"][lv][0]), lv
        assert _same(g["pairs"][lv][1], tr["pairs"][lv][1]), lv
        assert g["tests"][lv] == tr["tests"][lv]
        assert g["hits"][lv] == tr["hits"][lv]
    assert g["mesh_tests"] == tr["mesh_tests"]
    assert g["mesh_hits"] == tr["mesh_hits"]


@pytest.mark.parametrize("B,F,n", [(16, 2, 4), (16, 3, 3), (16, 8, 3), (32, 16, 2), (24, 4, 4), (8, 4, 4),
                                   (8, 8, 2), (4, 4, 7), (2, 16, 4)])
def test_traverse_shapes(B, F, n):
    """Traversal pairs, node tests and survivors of every level for merge
    factors 2..16 and bundles on both sides of 16 rays (one (parent, child)
    test per lane, NF = the merge factor rounded up to a power of two lanes
    per parent).  The count passes copy the run of child nodes below one
    top-level node to LDS when it has at most 1024 nodes: (4, 4, 7) has runs
    of 4^6 = 4096 nodes on level 1 (read from the node arrays) and of exactly
    1024 on level 2; (2, 16, 4) has runs of 16^3 = 4096 on level 1."""
    base, kw = small("refl_96")
    print(f"[traverse-shape] B={B} F={F} n={n}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    tree = O.build_tree(o["hash"]["rays"], o["sorted_ids"], B, F, n)
    ot = O.traverse(tree, wl.scene, 0, wl.scene.m)
    cap = max([len(t) for t, _ in ot["pairs"].values()] + [1]) + 4096
    g = _gu().gpu_traverse(tree, wl.scene, B, F, capacity=cap)
    assert g["status"] == 0
    for lv in ot["pairs"]:
        assert _same(g["pairs"][lv][0], ot["pairs"][lv][0]), lv
        assert _same(g["pairs"][lv][1], ot["pairs"][lv][1]), lv
        assert g["tests"][lv] == ot["tests"][lv], lv
        assert g["hits"][lv] == ot["hits"][lv], lv


def test_traverse_triangle_batches():
    base, kw = small("refl_96")
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    m = wl.scene.m
    cuts = [(0, 777), (777, m // 2), (m // 2, m)]
    g = _gu().gpu_traverse(o["tree"], wl.scene, wl.B, wl.F, batches=cuts, capacity=1 << 24)
    for run, (b, e) in zip(g["runs"], cuts):
        ot = O.traverse(o["tree"], wl.scene, b, e)
        for lv in ot["pairs"]:
            assert _same(run["pairs"][lv][0], ot["pairs"][lv][0])
            assert _same(run["pairs"][lv][1], ot["pairs"][lv][1])
    # counters sum over batches
    for lv in o["trav"]["tests"]:
        assert g["tests"][lv] == o["trav"]["tests"][lv]
        assert g["hits"][lv] == o["trav"]["hits"][lv]


def test_traverse_capacity_overflow_reports_required_size():
    base, kw = small("shadow_128")
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    need = max(len(t) for t, _ in o["trav"]["pairs"].values())
    g = _gu().gpu_traverse(o["tree"], wl.scene, wl.B, wl.F, capacity=need // 3)
    assert g["status"] == 2    # CRSH_ERR_CAPACITY
    top = o["tree"]["n_levels"]
    assert g["meta"].pairs[top - 1] == len(o["trav"]["pairs"][top][0])


@pytest.mark.parametrize("name", CASES)
def test_closest_hit_matches_oracle(name):
    base, kw = small(name)
    print(f"[hit] {name}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    g, m = _gu().gpu_closest_hit(o["hash"]["rays"], o["sorted_ids"], wl.B, o["trav"]["pairs"][1], wl.scene,
                                 wl.t_min)
    assert np.array_equal(g[0], o["hits"][0])
    for a, b in zip(g[1:], o["hits"][1:]):
        assert np.allclose(a, b, rtol=1e-5, atol=0)
    assert int(m.final_tests) == o["trav"]["final_tests"]
    # how far the tests got: u passed, u and v passed
    assert (int(m.final_u_pass), int(m.final_uv_pass)) == (o["stages"]["u"], o["stages"]["uv"])


@pytest.mark.parametrize("t_min", [-1.0, -1e-3, 0.0])
def test_closest_hit_with_an_interval_start_at_or_below_zero(t_min):
    """Intervals that admit t <= 0: every bounce ray meets its own surface
    at t of about -1e-3 (origins sit 1e-3 off the surface), so with t_min
    = -1 the closest hit has a negative t, and several negative hits
    compete; the keys must order negative distances as floats do (and
    -0 like +0).  Same level-1 pairs as the oracle's."""
    base, kw = small("refl_96")
    print(f"[hit] t_min {t_min}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    ref = O.closest_hit(o["hash"]["rays"], o["sorted_ids"], wl.B, o["trav"]["pairs"][1], wl.scene, t_min)
    g, m = _gu().gpu_closest_hit(o["hash"]["rays"], o["sorted_ids"], wl.B, o["trav"]["pairs"][1], wl.scene, t_min)
    assert np.array_equal(g[0], ref[0])
    for a, b in zip(g[1:], ref[1:]):
        assert np.allclose(a, b, rtol=1e-5, atol=0)
    if t_min < -1e-2:
        assert int(((ref[0] >= 0) & (ref[1] < 0)).sum()) > 1000


@pytest.mark.parametrize("name", CASES)
def test_pipeline_end_to_end(name):
    base, kw = small(name)
    print(f"[pipeline] {name}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    g = _gu().run_pipeline(wl, pair_capacity=1 << 16)
    assert g["n"] == o["hash"]["n"]
    assert _same(g["keys"], o["hash"]["keys"])
    assert _same(g["sorted_ids"], o["sorted_ids"])
    _check_tree(g, o["tree"])
    for lv, (t, n) in o["trav"]["pairs"].items():
        assert _same(g["pairs"][lv][0], t) and _same(g["pairs"][lv][1], n)
    assert g["final_tests"] == o["trav"]["final_tests"]
    assert (int(g["meta"].final_u_pass), int(g["meta"].final_uv_pass)) == (o["stages"]["u"], o["stages"]["uv"])
    assert np.array_equal(g["hit"][0], o["hits"][0])
    for a, b in zip(g["hit"][1:], o["hits"][1:]):
        assert np.allclose(a, b, rtol=1e-5, atol=0)


@pytest.mark.parametrize("name,shape,levels", [("mixed_128x72", {}, 16), ("mixed_128x72", {}, None),
                                               ("refl_96", dict(B=8, F=8, n=2), None)])
def test_unsorted_comparison_mode_bit_exact(name, shape, levels):
    """The comparison configuration (keys of type and light only, one
    always-passing mesh): every product -- built to a single top node, at
    the workload's own shape, and at the paper's evaluation setting
    (hierarchy depth 2, node subdivision 8, Sec. 4.1)."""
    from workloads import unsorted_variant
    base, kw = small(name)
    wl = unsorted_variant(workload(base, **kw, **shape), levels=levels)
    o = O.run_pipeline(wl)
    print(f"[unsorted] {o['hash']['n']} rays, {o['tree']['n_levels']} levels", flush=True)
    g = _gu().run_pipeline(wl, pair_capacity=1 << 20)
    assert _same(g["keys"], o["hash"]["keys"]) and _same(g["sorted_ids"], o["sorted_ids"])
    _check_tree(g, o["tree"])
    for lv, (t, n) in o["trav"]["pairs"].items():
        assert _same(g["pairs"][lv][0], t) and _same(g["pairs"][lv][1], n), lv
    assert np.array_equal(g["hit"][0], o["hits"][0])
    f = _gu().run_pipeline(wl, pair_capacity=1 << 20, keep_levels=False, leaf_hit=True)
    _check_fused(f, o)


@pytest.mark.parametrize("name", ["refl_96", "mixed_128x72"])
def test_bounce_generations_bit_exact(name):
    """Three generations (Sec. 3.3.8): each next generation's rays come from
    the previous closest hits; every product of every generation, with
    stored pairs and with the fused last level."""
    base, kw = small(name)
    wl = workload(base, **kw)
    print(f"[bounce] {name}: oracle", flush=True)
    og = O.run_generations(wl, 3)
    gg = _gu().run_generations(wl, 3, pair_capacity=1 << 20, keep_levels=True, leaf_hit=False)
    fg = _gu().run_generations(wl, 3, pair_capacity=1 << 20, keep_levels=False, leaf_hit=True)
    for gen, (o, g, f) in enumerate(zip(og, gg, fg)):
        print(f"[bounce] {name} generation {gen}: {o['hash']['n']} rays", flush=True)
        assert g["n"] == o["hash"]["n"]
        assert _same(g["keys"], o["hash"]["keys"])
        for k in O.RAY_FIELDS:
            assert _same(g["rays"][k], o["hash"]["rays"][k]), k
        assert _same(g["rays"]["pix"], o["hash"]["rays"]["pix"])
        assert _same(g["sorted_ids"], o["sorted_ids"])
        _check_tree(g, o["tree"])
        for lv, (t, n) in o["trav"]["pairs"].items():
            assert _same(g["pairs"][lv][0], t) and _same(g["pairs"][lv][1], n), lv
        assert np.array_equal(g["hit"][0], o["hits"][0])
        for a, b in zip(g["hit"][1:], o["hits"][1:]):
            assert _same(a, b)
        _check_fused(f, o)


def test_spherical_keys_bit_exact():
    """Spherical-coordinate direction codes: keys and the whole path."""
    import dataclasses
    from workloads import KEY_SPHERICAL
    base, kw = small("mixed_128x72")
    wl0 = workload(base, **kw)
    wl = dataclasses.replace(wl0, ray_types=wl0.ray_types | KEY_SPHERICAL)
    o = O.run_pipeline(wl)
    g = _gu().run_pipeline(wl, pair_capacity=1 << 20)
    assert _same(g["keys"], o["hash"]["keys"]) and _same(g["sorted_ids"], o["sorted_ids"])
    _check_tree(g, o["tree"])
    for lv, (t, n) in o["trav"]["pairs"].items():
        assert _same(g["pairs"][lv][0], t) and _same(g["pairs"][lv][1], n), lv
    assert np.array_equal(g["hit"][0], o["hits"][0])


LEAF_SHAPES = [(16, 4, 5), (8, 2, 3), (32, 8, 4), (5, 3, 4), (1, 16, 3), (12, 4, 2), (16, 4, 1), (4, 4, 7)]


def _check_fused(g, o):
    """The fused last level: closest hits and every counter of the stage
    order (level-1 tests and pairs formed, ray-triangle tests)."""
    tr = o["trav"]
    assert g["final_tests"] == tr["final_tests"]
    if "stages" in o:
        assert (int(g["meta"].final_u_pass), int(g["meta"].final_uv_pass)) == (o["stages"]["u"], o["stages"]["uv"])
    nl = o["tree"]["n_levels"]
    for lv in range(1, nl + 1):
        assert g["tests"][lv] == tr["tests"][lv], lv
        assert g["hits"][lv] == len(tr["pairs"][lv][0]), lv
    assert g["mesh_tests"] == tr["mesh_tests"] and g["mesh_hits"] == tr["mesh_hits"]
    assert np.array_equal(g["hit"][0], o["hits"][0])
    for a, b in zip(g["hit"][1:], o["hits"][1:]):
        assert _same(a, b)


@pytest.mark.parametrize("name", CASES)
def test_leaf_hit_matches_oracle(name):
    base, kw = small(name)
    print(f"[leaf_hit] {name}", flush=True)
    wl = workload(base, **kw)
    o = oracle_run(base, **kw)
    g = _gu().run_pipeline(wl, pair_capacity=1 << 16, keep_levels=False, leaf_hit=True)
    _check_fused(g, o)


@pytest.mark.parametrize("B,F,n", LEAF_SHAPES)
def test_leaf_hit_shapes(B, F, n):
    """Bundles that do not fill a lane group, merge factors that do not fill
    a power of two, single-level hierarchies (only the stored path), and
    level-1 runs of 4096 nodes, too long for the count's LDS copy."""
    import dataclasses
    base, kw = small("refl_96")
    wl = dataclasses.replace(workload(base, **kw), B=B, F=F, n=n)
    print(f"[leaf_hit] B={B} F={F} n={n}", flush=True)
    o = O.run_pipeline(wl)
    g = _gu().run_pipeline(wl, pair_capacity=1 << 16, keep_levels=False, leaf_hit=True)
    _check_fused(g, o)


def test_leaf_hit_single_leaf_and_no_rays():
    """A hierarchy that is one leaf (its level-1 pairs come from the top-level
    pass) and a frame without any ray."""
    import dataclasses
    for wl in (workload("shadow_128", W=3, H=3),
               dataclasses.replace(workload("shadow_128", W=8, H=8),
                                   gbuf=dict(workload("shadow_128", W=8, H=8).gbuf,
                                             mat=np.full(64, -1, np.int32)))):
        o = O.run_pipeline(wl)
        print(f"[leaf_hit] {o['hash']['n']} rays, {o['tree']['n_levels']} levels", flush=True)
        g = _gu().run_pipeline(wl, pair_capacity=1 << 12, keep_levels=False, leaf_hit=True)
        assert g["n"] == o["hash"]["n"]
        if g["n"]:
            _check_fused(g, o)


def test_leaf_hit_triangle_batches():
    base, kw = small("mixed_128x72")
    wl = workload(base, **kw)
    m = wl.scene.m
    batches = [(0, m // 3), (m // 3, m // 3), (m // 3, 2 * m // 3 + 5), (2 * m // 3 + 5, m)]
    o = O.run_pipeline(wl, tri_batches=batches)
    g = _gu().run_pipeline(wl, pair_capacity=1 << 16, keep_levels=False, tri_batches=batches, leaf_hit=True)
    assert g["final_tests"] == sum(t["final_tests"] for t in o["trav"])
    assert np.array_equal(g["hit"][0], o["hits"][0])
    for a, b in zip(g["hit"][1:], o["hits"][1:]):
        assert _same(a, b)


def test_packed_pairs_bit_exact_per_triangle_batch():
    """Pairs packed one 32-bit word each (node above 14 bits of triangle
    offset, Sec. 3.3.7) over triangle batches of at most 2^14 triangles:
    every level of every batch decodes to the oracle's pairs of that batch,
    in order, with the same counters; over all batches the closest hits are
    the oracle's."""
    from paper_2312_06538_amd import pipeline as P
    gu = _gu()
    base, kw = small("refl_96")
    wl = workload(base, **kw)
    batches = P.packed_batches(wl.scene.m)
    assert len(batches) > 1 and all(e - b <= 1 << 14 for b, e in batches)
    o = O.run_pipeline(wl, tri_batches=batches)
    for i, (b, e) in enumerate(batches):
        print(f"[packed] batch [{b}, {e})", flush=True)
        g = gu.run_pipeline(wl, pair_capacity=1 << 20, keep_levels=True, tri_batches=[(b, e)], packed=True)
        tr = o["trav"][i]
        for lv, (t, nd) in tr["pairs"].items():
            pt, pn = gu.decode_packed(g["pairs"][lv][0], b)
            assert np.array_equal(pt, t) and np.array_equal(pn, nd), (b, lv)
        assert g["tests"] == {lv: int(v) for lv, v in tr["tests"].items()}
        assert g["final_tests"] == tr["final_tests"] and g["mesh_tests"] == tr["mesh_tests"]
    g = gu.run_pipeline(wl, pair_capacity=1 << 20, keep_levels=False, packed=True)
    assert g["final_tests"] == sum(t["final_tests"] for t in o["trav"])
    assert np.array_equal(g["hit"][0], o["hits"][0])
    for a, b in zip(g["hit"][1:], o["hits"][1:]):
        assert _same(a, b)


def test_packed_pairs_reject_levels_over_2_18_nodes():
    """A level of more than 2^18 nodes cannot be packed: the traversal flags
    it on the device (the pairs of that call are not valid)."""
    import dataclasses
    from paper_2312_06538_amd import crsh as X
    from paper_2312_06538_amd import pipeline as P
    wl = dataclasses.replace(workload("refl_1024", W=400, H=400), B=1, F=4, n=2)
    fr = P.DeviceFrame(wl)
    bf = P.Buffers(fr, 1 << 22, keep_levels=False)
    P.run_frame(fr, bf, tri_batches=[(0, 1 << 14)], packed=True)
    m, st = P.read_meta(bf)
    assert int(m.level_cnt[0]) > X.PACKED_MAX_NODES
    assert st != X.OK and m.status & X.OVERFLOW_PACKED
    # within the limit (one level of at most 2^18 nodes) the flag stays clear
    wl = dataclasses.replace(workload("refl_1024", W=96, H=96), B=1, F=4, n=2)
    fr = P.DeviceFrame(wl)
    bf = P.Buffers(fr, 1 << 22, keep_levels=False)
    P.run_frame(fr, bf, tri_batches=[(0, 1 << 14)], packed=True)
    m, st = P.read_meta(bf)
    assert not m.status & X.OVERFLOW_PACKED


def test_pipeline_is_deterministic():
    base, kw = small("refl_96")
    wl = workload(base, **kw)
    a = _gu().run_pipeline(wl, pair_capacity=1 << 22)
    b = _gu().run_pipeline(wl, pair_capacity=1 << 22)
    for lv in a["pairs"]:
        assert _same(a["pairs"][lv][0], b["pairs"][lv][0]) and _same(a["pairs"][lv][1], b["pairs"][lv][1])
    for x, y in zip(a["hit"], b["hit"]):
        assert _same(x, y)
