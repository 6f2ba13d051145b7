"""Pins of the oracle's hierarchy traversal (Sec. 3.3.7, Eq. 9) and of its
intersection counters (Sec. 4.3.1, Tables 1-4).

Eq. 9 is pinned by geometry: with a zero-spread, zero-radius node it is the
textbook point-to-line distance test; for any node it must pass every sphere
that some ray of the node actually meets (sampled in float64) and reject
spheres far outside the node.  The traversal is pinned by the fact that
culling is conservative (every brute-force hit survives to level 1) and by
the counting identities that the paper's own tables satisfy.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from conftest import small, oracle_run, workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table_counts.json")


def node11(C, r, a, phi):
    a = np.asarray(a, np.float64)
    a = a / np.linalg.norm(a)
    c, s = np.float32(np.cos(phi)), np.float32(np.sin(phi))
    tan = np.float32(s / c) if c > 0 else np.float32(0)
    sec = np.float32(np.float32(1) / c) if c > 0 else np.float32(0)
    return np.array([C[0], C[1], C[2], r, a[0], a[1], a[2], c, s, tan, sec], np.float32)


def test_eq9_zero_spread_is_point_to_line_distance(rng):
    for _ in range(3000):
        C = rng.uniform(-5, 5, 3)
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        P = rng.uniform(-5, 5, 3)
        d = rng.uniform(0, 3)
        nd = node11(C, 0.0, a, 0.0)
        a32 = nd[4:7].astype(np.float64)
        v = P - C
        dist = np.linalg.norm(v - (v @ a32) / (a32 @ a32) * a32)
        if abs(dist - d) < 1e-4 * (1 + d):
            continue
        assert O.node_sphere_test(nd, np.r_[P, d]) == (dist <= d)


def _sample_node_rays(rng, C, r, a, phi, k):
    """Origins uniform in the ball, directions uniform in the cone (float64)."""
    u = rng.normal(size=(k, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    o = C + u * (r * rng.uniform(0, 1, (k, 1)) ** (1 / 3))
    a = a / np.linalg.norm(a)
    t1 = np.cross(a, [1, 0, 0] if abs(a[0]) < 0.9 else [0, 1, 0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(a, t1)
    cz = rng.uniform(np.cos(phi), 1, k)
    sz = np.sqrt(1 - cz * cz)
    az = rng.uniform(0, 2 * np.pi, k)
    d = cz[:, None] * a + sz[:, None] * (np.cos(az)[:, None] * t1 + np.sin(az)[:, None] * t2)
    return o, d


def _ray_meets_sphere(o, d, P, rad):
    v = P - o
    t = np.maximum((v * d).sum(1), 0.0)
    return np.linalg.norm(o + t[:, None] * d - P, axis=1) <= rad


def test_eq9_passes_every_sphere_a_node_ray_meets(rng):
    checked = 0
    for _ in range(1500):
        C = rng.uniform(-5, 5, 3)
        r = rng.uniform(0, 1.0)
        a = rng.normal(size=3)
        phi = rng.uniform(0, 1.2)
        o, d = _sample_node_rays(rng, C, r, a, phi, 256)
        # a sphere placed near a random point of a random sampled ray
        i = rng.integers(0, 256)
        P = o[i] + d[i] * rng.uniform(-2, 20) + rng.normal(size=3) * rng.uniform(0, 2)
        rad = rng.uniform(0.01, 1.0)
        if _ray_meets_sphere(o, d, P, rad).any():
            checked += 1
            assert O.node_sphere_test(node11(C, r, a, phi), np.r_[P, rad])
    assert checked > 300


def test_eq9_rejects_spheres_far_outside(rng):
    for _ in range(1000):
        C = rng.uniform(-5, 5, 3)
        r = rng.uniform(0, 1.0)
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        phi = rng.uniform(0, 1.0)
        rad = rng.uniform(0.01, 1.0)
        t = rng.uniform(-10, 10)
        perp = np.cross(a, rng.normal(size=3))
        perp /= np.linalg.norm(perp)
        bound = abs(t) * np.tan(phi) + (rad + r) / np.cos(phi)
        P = C + t * a + perp * bound * rng.uniform(1.01, 3)
        assert not O.node_sphere_test(node11(C, r, a, phi), np.r_[P, rad])


def test_eq9_full_node_never_culls():
    nd = node11([0, 0, 0], 0.1, [0, 0, 1], 0.0)
    nd[7], nd[8], nd[9], nd[10] = -1, 0, 0, 0
    assert O.node_sphere_test(nd, np.array([1e6, 1e6, -1e6, 1e-3], np.float32))


def _leaf_of(sorted_ids, B):
    leaf = np.empty(len(sorted_ids), np.int64)
    leaf[sorted_ids.astype(np.int64)] = np.arange(len(sorted_ids)) // B
    return leaf


@pytest.mark.parametrize("name,nsample", [("shadow_128", None), ("refl_96", 600), ("mixed_128x72", 300)])
def test_every_brute_force_hit_survives_to_level1(name, nsample):
    """Culling is conservative: any ray-triangle hit, closest or not, keeps
    its (triangle, leaf) pair up to the final tests."""
    base, kw = small(name)
    wl = workload(base, **kw)
    r = oracle_run(base, **kw)
    h = r["hash"]
    rays = np.arange(h["n"]) if nsample is None else \
        np.random.default_rng(7).choice(h["n"], nsample, replace=False)
    hr, ht = O.brute_all_hits(h["rays"], rays, wl.scene, wl.t_min)
    assert len(hr) > 0
    leaf = _leaf_of(r["sorted_ids"], wl.B)
    t1, n1 = r["trav"]["pairs"][1]
    have = np.sort((n1.astype(np.int64) << 32) | t1)
    need = (leaf[hr] << 32) | ht.astype(np.int64)
    pos = np.minimum(np.searchsorted(have, need), len(have) - 1)
    assert np.all(have[pos] == need)


@pytest.mark.parametrize("name", ["shadow_128", "refl_96", "mixed_128x72"])
def test_pairs_descend_from_parent_pairs(name):
    base, kw = small(name)
    r = oracle_run(base, **kw)
    tree, tr = r["tree"], r["trav"]
    F = tree["F"]
    nl = tree["n_levels"]
    for lv in range(1, nl):
        t, n = tr["pairs"][lv]
        tu, nu = tr["pairs"][lv + 1]
        up = np.sort((nu.astype(np.int64) << 32) | tu)
        key = ((n.astype(np.int64) // F) << 32) | t
        pos = np.minimum(np.searchsorted(up, key), len(up) - 1)
        assert np.all(up[pos] == key)
        # no pair twice
        own = np.sort((n.astype(np.int64) << 32) | t)
        assert np.all(own[1:] != own[:-1])


@pytest.mark.parametrize("name", ["shadow_128", "refl_96", "mixed_128x72"])
def test_counter_identities(name):
    base, kw = small(name)
    wl = workload(base, **kw)
    r = oracle_run(base, **kw)
    tree, tr = r["tree"], r["trav"]
    F, B, N = tree["F"], tree["B"], tree["n_rays"]
    cnt = tree["level_cnt"]
    nl = tree["n_levels"]
    assert tr["mesh_tests"] == int(cnt[nl - 1]) * wl.scene.n_mesh
    for lv in range(1, nl):
        t, p = tr["pairs"][lv + 1]
        children = np.minimum(F, cnt[lv - 1].astype(np.int64) - p.astype(np.int64) * F)
        assert tr["tests"][lv] == int(children.sum())
        assert tr["hits"][lv] == len(tr["pairs"][lv][0])
    t, j = tr["pairs"][1]
    rays_in = np.minimum(B, N - j.astype(np.int64) * B)
    assert tr["final_tests"] == int(rays_in.sum())


def test_paper_tables_obey_the_counting_convention():
    """Tables 1-3 and the totals of Table 4 satisfy: level-1 tests are 8x the
    level-2 hits, and the total is the node tests of both levels plus 8 rays
    per level-1 hit (node subdivision 8, Sec. 4.1)."""
    g = json.load(open(GOLDEN))
    k = g["subdivision"]
    for name, row in g["rows"].items():
        total = 0
        for typ, c in row["types"].items():
            assert c["l2_misses"] + c["l2_hits"] == c["l2_tests"], name
            assert c["l1_misses"] + c["l1_hits"] == c["l1_tests"], name
            assert c["l1_tests"] == k * c["l2_hits"], name
            total += c["l2_tests"] + c["l1_tests"] + k * c["l1_hits"]
        assert total == row["total"], name
    bf = g["brute_force"]
    assert bf["office"] == g["rays"]["office"] * 36308
    assert bf["sponza"] == g["rays"]["sponza"] * 66450


def test_oracle_counters_follow_the_paper_convention():
    """With every node full, the oracle's counters reduce to the paper's:
    tests(k) = F * hits(k+1) and final tests = B * hits(1)."""
    wl = workload("shadow_128")
    r = oracle_run("shadow_128")
    B, F = 8, 4
    ids = r["sorted_ids"][:B * F ** 3 * 16]
    tree = O.build_tree(r["hash"]["rays"], ids, B, F, 4)
    assert list(tree["level_cnt"]) == [1024, 256, 64, 16]
    tr = O.traverse(tree, wl.scene)
    for lv in range(1, 4):
        assert tr["tests"][lv] == F * tr["hits"][lv + 1]
    assert tr["final_tests"] == B * tr["hits"][1]


def test_triangle_batches_partition_the_pairs():
    base, kw = small("refl_96")
    wl = workload(base, **kw)
    r = oracle_run(base, **kw)
    m = wl.scene.m
    cuts = [0, 1000, 30000, 30001, m]
    full = r["trav"]
    got = {lv: [] for lv in full["pairs"]}
    tests = {lv: 0 for lv in full["pairs"]}
    final = 0
    for b, e in zip(cuts[:-1], cuts[1:]):
        tr = O.traverse(r["tree"], wl.scene, b, e)
        for lv, (t, n) in tr["pairs"].items():
            assert np.all((t >= b) & (t < e))
            got[lv].append((n.astype(np.int64) << 32) | t)
            tests[lv] += tr["tests"][lv]
        final += tr["final_tests"]
    for lv, (t, n) in full["pairs"].items():
        a = np.sort(np.concatenate(got[lv]))
        assert np.array_equal(a, np.sort((n.astype(np.int64) << 32) | t))
        assert tests[lv] == full["tests"][lv]
    assert final == full["final_tests"]


def test_top_subset_restricts_to_subtrees():
    base, kw = small("refl_96")
    wl = workload(base, **kw)
    r = oracle_run(base, **kw)
    tree = r["tree"]
    nl = tree["n_levels"]
    sub = np.array([0, 3, 4], np.uint32)
    tr = O.traverse(tree, wl.scene, top_subset=sub)
    F = tree["F"]
    for lv, (t, n) in r["trav"]["pairs"].items():
        top = n.astype(np.int64) // F ** (nl - lv)
        keep = np.isin(top, sub)
        want = np.sort((n[keep].astype(np.int64) << 32) | t[keep])
        ts, ns = tr["pairs"][lv]
        assert np.array_equal(np.sort((ns.astype(np.int64) << 32) | ts), want)


@pytest.mark.parametrize("name", ["refl_1024", "mixed_1080p"])
def test_fullsize_golden_is_self_consistent(name):
    """The full-frame values written by tests/golden/make_fullsize.py (oracle
    only) hang together: per-sub-tree level-1 pair counts sum to the level-1
    count, the chained digest is that of the per-sub-tree digests, level k's
    tests are the children of level k+1's pairs (R14 with full nodes except
    ragged tails: at most F per parent pair), and the final tests are at most
    B per level-1 pair."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"fullsize_{name}.json")
    g = json.load(open(path))
    assert g["written_by"].startswith("tests/golden/make_fullsize.py")
    assert len(g["per_top"]) == g["top_nodes"]
    assert sum(p["n1"] for p in g["per_top"]) == g["hits"][0]
    chain = hashlib.sha256("".join(p["sha"] for p in g["per_top"]).encode()).hexdigest()
    assert chain == g["pairs1_sha256"]
    nl = g["levels"]
    for k in range(nl - 1):
        assert g["tests"][k] <= g["F"] * g["hits"][k + 1]
        assert g["tests"][k] >= g["hits"][k]
    assert g["final_tests"] <= g["B"] * g["hits"][0]
    assert g["tests"][nl - 1] >= g["hits"][nl - 1]
    assert g["mesh_hits"] <= g["mesh_tests"]
    assert 0 < g["hit_count"] <= g["rays"]
