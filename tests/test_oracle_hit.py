"""Pins of the oracle's final intersection tests and closest hit (Sec. 3.3.8).

Moller-Trumbore is pinned by an exactly representable closed form and by an
independent float64 geometric test (ray-plane intersection plus barycentric
coordinates from signed areas).  The whole pipeline is pinned by naive ray
tracing (Sec. 1): the closest hit through the hierarchy must equal the
brute-force N x M closest hit exactly, for any bundle size, merge factor and
level count.
"""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import Scene
from conftest import small, oracle_run, workload


def test_mt_closed_form():
    tri = np.array([0, 0, 0, 1, 0, 0, 0, 1, 0], np.float32)
    hit, tuv = O.mt([0.25, 0.5, 1.0], [0, 0, -1], 1e-4, 10.0, tri)
    assert hit and tuple(tuv) == (1.0, 0.25, 0.5)
    # from behind (two-sided)
    hit, tuv = O.mt([0.25, 0.5, -2.0], [0, 0, 1], 1e-4, 10.0, tri)
    assert hit and tuple(tuv) == (2.0, 0.25, 0.5)
    # just outside each edge, beyond tmax, before t_min, parallel
    assert not O.mt([-0.01, 0.5, 1.0], [0, 0, -1], 1e-4, 10.0, tri)[0]
    assert not O.mt([0.5, -0.01, 1.0], [0, 0, -1], 1e-4, 10.0, tri)[0]
    assert not O.mt([0.6, 0.6, 1.0], [0, 0, -1], 1e-4, 10.0, tri)[0]
    assert not O.mt([0.25, 0.5, 1.0], [0, 0, -1], 1e-4, 0.5, tri)[0]
    assert not O.mt([0.25, 0.5, 1.0], [0, 0, 1], 1e-4, 10.0, tri)[0]
    assert not O.mt([0.25, 0.5, 1.0], [1, 0, 0], 1e-4, 10.0, tri)[0]
    # degenerate triangle
    deg = np.array([0, 0, 0, 1, 0, 0, 2, 0, 0], np.float32)
    assert not O.mt([0.5, 0.0, 1.0], [0, 0, -1], 1e-4, 10.0, deg)[0]


def _geom64(o, d, tri):
    """Ray-plane intersection and signed-area barycentrics, float64."""
    v0, v1, v2 = tri[:3], tri[3:6], tri[6:]
    n = np.cross(v1 - v0, v2 - v0)
    den = d @ n
    if den == 0:
        return None
    t = ((v0 - o) @ n) / den
    p = o + t * d
    nn = n @ n
    u = np.cross(v2 - v0, p - v0) @ n / nn * -1.0
    w = np.cross(v1 - v0, p - v0) @ n / nn
    # p = v0 + u (v1 - v0) + w (v2 - v0)
    return t, u, w


def test_mt_matches_float64_geometry(rng):
    agree = 0
    for _ in range(4000):
        tri = rng.normal(size=9) * 3
        o = rng.normal(size=3) * 5
        target = tri[:3] + rng.uniform(-0.2, 1.2) * (tri[3:6] - tri[:3]) + \
            rng.uniform(-0.2, 1.2) * (tri[6:] - tri[:3])
        d = target - o
        d /= np.linalg.norm(d)
        o32, d32, tri32 = o.astype(np.float32), d.astype(np.float32), tri.astype(np.float32)
        g = _geom64(o32.astype(np.float64), d32.astype(np.float64), tri32.astype(np.float64))
        if g is None:
            continue
        t, u, w = g
        margin = min(u, w, 1 - u - w)
        n = np.cross(tri[3:6] - tri[:3], tri[6:] - tri[:3])
        grazing = abs(d @ n) / np.linalg.norm(n) < 0.1     # ill-conditioned in float32
        if abs(margin) < 1e-4 or abs(t) < 1e-3 or grazing:
            continue
        inside = margin > 0 and t > 1e-4
        hit, tuv = O.mt(o32, d32, 1e-4, np.float32(np.finfo(np.float32).max), tri32)
        assert hit == inside
        if hit:
            agree += 1
            assert np.allclose(tuv, [t, u, w], rtol=1e-4, atol=1e-4)
    assert agree > 500


@pytest.mark.parametrize("name,nsample", [("shadow_128", None), ("refl_96", 1200), ("mixed_128x72", 500)])
def test_closest_hit_equals_brute_force(name, nsample):
    base, kw = small(name)
    wl = workload(base, **kw)
    r = oracle_run(base, **kw)
    h = r["hash"]
    rays = np.arange(h["n"]) if nsample is None else \
        np.random.default_rng(11).choice(h["n"], nsample, replace=False)
    b = O.brute_closest_hit(h["rays"], rays, wl.scene, wl.t_min)
    got = [a[rays] for a in r["hits"]]
    assert (b[0] >= 0).sum() > len(rays) // 20
    for x, y in zip(got, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("B,F,n", [(1, 2, 3), (4, 2, 6), (8, 8, 2), (32, 3, 3), (16, 4, 1)])
def test_closest_hit_independent_of_hierarchy_shape(B, F, n):
    wl = workload("shadow_128")
    r = oracle_run("shadow_128")
    h = r["hash"]
    tree = O.build_tree(h["rays"], r["sorted_ids"], B, F, n)
    tr = O.traverse(tree, wl.scene)
    hits = O.closest_hit(h["rays"], r["sorted_ids"], B, tr["pairs"][1], wl.scene, wl.t_min)
    for x, y in zip(hits, r["hits"]):
        assert np.array_equal(x, y)


def test_closest_hit_over_triangle_batches():
    base, kw = small("refl_96")
    wl = workload(base, **kw)
    r = oracle_run(base, **kw)
    m = wl.scene.m
    res = O.run_pipeline(wl, tri_batches=[(0, 777), (777, m // 2), (m // 2, m)])
    for x, y in zip(res["hits"], r["hits"]):
        assert np.array_equal(x, y)


def test_tie_breaks_to_lower_triangle_and_tmax_respected():
    tri = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]] * 3, np.float32)
    tri[0, :, 2] = -1.0       # farther copy
    sc = Scene(tris=tri, mesh_first=np.array([0], np.uint32), mesh_count=np.array([3], np.uint32),
               mesh_sphere=np.array([[0.5, 0.5, -0.5, 2.0]], np.float32),
               mesh_mat=np.zeros(1, np.int32), mat_flags=np.zeros(1, np.uint32),
               mat_ior=np.ones(1, np.float32))
    rays = {"ox": np.array([0.2, 0.2], np.float32), "oy": np.array([0.2, 0.2], np.float32),
            "oz": np.array([1.0, 1.0], np.float32), "dx": np.zeros(2, np.float32),
            "dy": np.zeros(2, np.float32), "dz": np.full(2, -1.0, np.float32),
            "tmax": np.array([5.0, 0.5], np.float32), "pix": np.zeros(2, np.uint32)}
    b = O.brute_closest_hit(rays, np.arange(2), sc, 1e-4)
    assert list(b[0]) == [1, -1]     # triangles 1 and 2 coincide: lower id wins
    assert b[1][0] == 1.0
    tree = O.build_tree(rays, np.arange(2, dtype=np.uint32), 2, 2, 2)
    tr = O.traverse(tree, sc)
    hits = O.closest_hit(rays, np.arange(2, dtype=np.uint32), 2, tr["pairs"][1], sc, 1e-4)
    assert list(hits[0]) == [1, -1]


def test_mt64_closed_form_and_derivatives():
    """The float64 fixed-triangle solve used for finite differences: exact on
    an axis-aligned case, and its derivatives there are the textbook ones
    (t grows with the origin's height, u and v follow the origin's x, y)."""
    tri = np.array([0, 0, 0, 1, 0, 0, 0, 1, 0], np.float64)
    o = np.array([0.25, 0.5, 1.0])
    d = np.array([0.0, 0.0, -1.0])
    ok, tuv = O.mt64(o, d, tri)
    assert ok and np.array_equal(tuv, [1.0, 0.25, 0.5])
    h = 1e-4
    def fd(vec, k):
        a, b = vec.copy(), vec.copy()
        a[k] += h
        b[k] -= h
        return a, b
    for k, want in ((0, [0, 1, 0]), (1, [0, 0, 1]), (2, [1, 0, 0])):
        a, b = fd(o, k)
        g = (O.mt64(a, d, tri)[1] - O.mt64(b, d, tri)[1]) / (2 * h)
        assert np.allclose(g, want, atol=1e-9)
    # moving v1 along x by h stretches u: u = 0.25 / (1 + h)
    a, b = fd(tri, 3)
    g = (O.mt64(o, d, a)[1] - O.mt64(o, d, b)[1]) / (2 * h)
    assert np.allclose(g, [0, -0.25, 0], atol=1e-7)


def test_mt64_agrees_with_float32_test(rng):
    n = 0
    for _ in range(500):
        tri = rng.normal(size=9) * 3
        o = rng.normal(size=3) * 5
        target = tri[:3] + 0.3 * (tri[3:6] - tri[:3]) + 0.3 * (tri[6:] - tri[:3])
        d = (target - o) / np.linalg.norm(target - o)
        hit, tuv = O.mt(o.astype(np.float32), d.astype(np.float32), 1e-4,
                        np.float32(np.finfo(np.float32).max), tri.astype(np.float32))
        ok, t64 = O.mt64(o.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64),
                         tri.astype(np.float32).astype(np.float64))
        nrm = np.cross(tri[3:6] - tri[:3], tri[6:] - tri[:3])
        if not hit or abs(d @ nrm) / np.linalg.norm(nrm) < 0.1:
            continue
        n += 1
        assert np.allclose(tuv, t64, rtol=1e-4, atol=1e-4)
    assert n > 100


def test_adjoint64_matches_finite_differences(rng):
    """The float64 adjoint (implicit-function form) against central
    differences of the float64 Moller-Trumbore solve, on random rays through
    random triangles, and its closed form for an axis-aligned triangle."""
    h = 1e-6
    done = 0
    while done < 40:
        tri = rng.normal(size=9)
        bary = rng.dirichlet([2.0, 2.0, 2.0])
        hit = bary[0] * tri[0:3] + bary[1] * tri[3:6] + bary[2] * tri[6:9]
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        o = hit - rng.uniform(0.5, 3.0) * d
        g = rng.normal(size=3)
        dv0, dv1, dv2, do, dd, cond = O.adjoint64(o, d, tri, g)
        if cond > 50:
            continue
        f = lambda o_, d_, t_: float(np.dot(g, O.mt64(o_, d_, t_)[1]))
        for vec, grad, which in ((o, do, "o"), (d, dd, "d")):
            for k in range(3):
                p, m = vec.copy(), vec.copy()
                p[k] += h
                m[k] -= h
                fd = (f(p, d, tri) - f(m, d, tri)) / (2 * h) if which == "o" else \
                    (f(o, p, tri) - f(o, m, tri)) / (2 * h)
                assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)), (which, k, fd, grad[k])
        for j, grad in enumerate((dv0, dv1, dv2)):
            for k in range(3):
                p, m = tri.copy(), tri.copy()
                p[3 * j + k] += h
                m[3 * j + k] -= h
                fd = (f(o, d, p) - f(o, d, m)) / (2 * h)
                assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)), (j, k, fd, grad[k])
        done += 1
    # axis-aligned triangle in z = 0, ray straight down from (0.25, 0.5, 1)
    dv0, dv1, dv2, do, dd, _ = O.adjoint64([0.25, 0.5, 1.0], [0, 0, -1.0], [0, 0, 0, 1, 0, 0, 0, 1, 0], [1, 0, 0])
    assert np.allclose(do, [0, 0, 1]) and np.allclose(dd, [0, 0, 1])
    assert np.allclose([dv0[2], dv1[2], dv2[2]], [-0.25, -0.25, -0.5])


def test_stage_counts_follow_the_test_order():
    """How far each final test got (Sec. 3.3.8): one triangle (0,0,0),
    (1,0,0), (0,1,0) in the z = 0 plane, rays straight down from z = 1 in one
    leaf: a ray parallel to the plane (determinant check fails), one with
    u < 0, one with u in range but u + v > 1, one inside but beyond tmax,
    and two hits.  u passes: 4; u and v pass: 3; closest hits: 2."""
    tri = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32)
    sc = Scene(tris=tri, mesh_first=np.array([0], np.uint32), mesh_count=np.array([1], np.uint32),
               mesh_sphere=np.array([[0.5, 0.5, 0.0, 2.0]], np.float32),
               mesh_mat=np.zeros(1, np.int32), mat_flags=np.zeros(1, np.uint32),
               mat_ior=np.ones(1, np.float32))
    #           parallel  u<0   u+v>1  tmax   hit    hit
    ox = np.array([0.2, -0.3, 0.6, 0.2, 0.2, 0.1], np.float32)
    oy = np.array([0.2, 0.2, 0.6, 0.2, 0.3, 0.1], np.float32)
    dz = np.array([0.0, -1, -1, -1, -1, -1], np.float32)
    dx = np.array([1.0, 0, 0, 0, 0, 0], np.float32)
    rays = {"ox": ox, "oy": oy, "oz": np.ones(6, np.float32), "dx": dx, "dy": np.zeros(6, np.float32),
            "dz": dz, "tmax": np.array([9, 9, 9, 0.5, 9, 9], np.float32), "pix": np.zeros(6, np.uint32)}
    ids = np.arange(6, dtype=np.uint32)
    st = {}
    hits = O.closest_hit(rays, ids, 8, (np.zeros(1, np.uint32), np.zeros(1, np.uint32)), sc, 1e-4, stages=st)
    assert (st["u"], st["uv"]) == (4, 3)
    assert list(hits[0]) == [-1, -1, -1, -1, 0, 0]
    # on a workload: final tests >= u passes >= u-and-v passes >= hit rays,
    # and the counts add up over calls
    base, kw = small("refl_96")
    o = oracle_run(base, **kw)
    assert o["trav"]["final_tests"] >= o["stages"]["u"] >= o["stages"]["uv"] >= int((o["hits"][0] >= 0).sum())
    st2 = {}
    O.closest_hit(o["hash"]["rays"], o["sorted_ids"], workload(base, **kw).B, o["trav"]["pairs"][1],
                  workload(base, **kw).scene, workload(base, **kw).t_min, stages=st2)
    O.closest_hit(o["hash"]["rays"], o["sorted_ids"], workload(base, **kw).B, o["trav"]["pairs"][1],
                  workload(base, **kw).scene, workload(base, **kw).t_min, stages=st2)
    assert st2 == {"u": 2 * o["stages"]["u"], "uv": 2 * o["stages"]["uv"]}
