"""Pins of the oracle's hierarchy creation (Sec. 3.3.6, Eq. 1-8).

The node sphere must contain the ray origins and the node cone the ray
directions (Sec. 3.3.6), and upper nodes must contain their children
(Sec. 3.3.7); both are checked in float64 on every node of every level.
Exact special cases (shared origin, identical rays, two-ray cones, two
spheres) pin the formulas themselves.
"""
import numpy as np
import pytest

from oracle import oracle as O
from conftest import small, oracle_run, workload

PAD = 2.0 ** -20        # sphere pad (relative)
CONE_PAD = 2.0 ** -16   # cone pad (radians)


def _ang(a, b):
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), (a * b).sum(-1))


def _nodes64(tree, lv):
    nd = tree["nodes"]
    o, c = int(tree["level_off"][lv - 1]), int(tree["level_cnt"][lv - 1])
    sl = slice(o, o + c)
    C = np.stack([nd["cx"][sl], nd["cy"][sl], nd["cz"][sl]], 1).astype(np.float64)
    A = np.stack([nd["ax"][sl], nd["ay"][sl], nd["az"][sl]], 1).astype(np.float64)
    return C, nd["r"][sl].astype(np.float64), A, nd["c"][sl].astype(np.float64), nd["s"][sl].astype(np.float64)


def check_containment(rays, sorted_ids, tree):
    """Every ray inside its leaf, every child inside its parent (float64)."""
    B, F, N = tree["B"], tree["F"], tree["n_rays"]
    if tree["n_levels"] == 0:
        return
    Cn, R, A, c, s = _nodes64(tree, 1)
    pos = np.arange(N)
    leaf = pos // B
    ids = sorted_ids.astype(np.int64)
    o = np.stack([rays["ox"][ids], rays["oy"][ids], rays["oz"][ids]], 1).astype(np.float64)
    d = np.stack([rays["dx"][ids], rays["dy"][ids], rays["dz"][ids]], 1).astype(np.float64)
    dist = np.linalg.norm(o - Cn[leaf], axis=1)
    assert np.all(dist <= R[leaf]), "origin outside its leaf sphere"
    full = c[leaf] <= 0
    phi = np.arctan2(s, c)
    ang = _ang(d, A[leaf])
    assert np.all(full | (ang <= phi[leaf] + 1e-12)), "direction outside its leaf cone"
    for lv in range(2, tree["n_levels"] + 1):
        Cp, Rp, Ap, cp, sp = _nodes64(tree, lv)
        Cc, Rc, Ac, cc, sc = _nodes64(tree, lv - 1)
        par = np.arange(len(Rc)) // F
        assert np.all(np.linalg.norm(Cc - Cp[par], axis=1) + Rc <= Rp[par]), "child sphere escapes"
        pfull = cp[par] <= 0
        assert np.all(pfull | (cc > 0)), "full child under a non-full parent"
        phic = np.arctan2(sc, cc)
        phip = np.arctan2(sp, cp)
        ok = pfull | (_ang(Ac, Ap[par]) + phic <= phip[par] + 1e-12)
        assert np.all(ok), "child cone escapes its parent"


@pytest.mark.parametrize("name", ["shadow_128", "refl_96", "mixed_128x72"])
def test_containment_every_node(name):
    base, kw = small(name)
    r = oracle_run(base, **kw)
    check_containment(r["hash"]["rays"], r["sorted_ids"], r["tree"])


@pytest.mark.parametrize("B,F,n", [(4, 2, 6), (8, 8, 2), (16, 4, 5), (32, 3, 3), (5, 7, 4)])
def test_containment_other_shapes(B, F, n):
    base, kw = small("refl_96")
    wl = workload(base, **kw)
    r = oracle_run(base, **kw)
    tree = O.build_tree(r["hash"]["rays"], r["sorted_ids"], B, F, n)
    check_containment(r["hash"]["rays"], r["sorted_ids"], tree)


def test_level_counts():
    assert list(O.level_counts(0, 8, 4, 4)) == []
    assert list(O.level_counts(5, 8, 4, 4)) == [1]
    assert list(O.level_counts(16384, 8, 4, 4)) == [2048, 512, 128, 32]
    assert list(O.level_counts(16385, 8, 4, 4)) == [2049, 513, 129, 33]
    # stops at the first level with a single node
    assert list(O.level_counts(100, 8, 4, 9)) == [13, 4, 1]
    assert list(O.level_counts(10836, 8, 4, 4)) == [1355, 339, 85, 22]


def test_shared_origin_stays_exact(rng):
    """Shadow rays of one light share their origin: every node centre is the
    light, bit for bit, and the radius is only accumulated padding."""
    L = np.array([5.0, 10.0, 5.0], np.float32)
    n = 1000
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = {"ox": np.full(n, L[0], np.float32), "oy": np.full(n, L[1], np.float32),
            "oz": np.full(n, L[2], np.float32), "dx": d[:, 0].astype(np.float32),
            "dy": d[:, 1].astype(np.float32), "dz": d[:, 2].astype(np.float32),
            "tmax": np.ones(n, np.float32), "pix": np.arange(n, dtype=np.uint32)}
    tree = O.build_tree(rays, np.arange(n, dtype=np.uint32), 8, 4, 4)
    nd = tree["nodes"]
    assert np.all(nd["cx"] == L[0]) and np.all(nd["cy"] == L[1]) and np.all(nd["cz"] == L[2])
    # depth of unions: 3 inside a leaf of 8, 2 per level of 4 -> at most 9 pads
    assert np.all(nd["r"] <= 9 * 1.01 * PAD * 10.0)
    assert np.all(nd["r"] > 0)


def test_identical_rays_leave_cone_untouched():
    x = np.array([0.6, 0.0, 0.8], np.float32)
    out = O.cone_add_ray(x, 1.0, 0.0, x)
    assert np.array_equal(out, np.array([0.6, 0.0, 0.8, 1.0, 0.0], np.float32))


def test_ray_inside_cone_leaves_it_untouched():
    x = np.array([0.0, 0.0, 1.0], np.float32)
    c, s = np.float32(np.cos(0.3)), np.float32(np.sin(0.3))
    r = np.array([np.sin(0.2), 0.0, np.cos(0.2)], np.float32)
    out = O.cone_add_ray(x, c, s, r)
    assert np.array_equal(out, np.array([0, 0, 1, c, s], np.float32))


@pytest.mark.parametrize("theta", [0.01, 0.3, 1.0, 2.0, 2.5])
def test_two_ray_cone_is_half_angle(theta):
    """Adding a ray at angle theta to a zero-spread cone gives the bisector
    axis and half-angle theta/2 (plus the CONE_PAD widening)."""
    a = np.array([1.0, 0.0, 0.0])
    b = np.array([np.cos(theta), np.sin(theta), 0.0])
    out = O.cone_add_ray(a.astype(np.float32), 1.0, 0.0, b.astype(np.float32)).astype(np.float64)
    bis = (a + b) / np.linalg.norm(a + b)
    assert _ang(out[:3], bis) < 1e-6
    phi = np.arctan2(out[4], out[3])
    assert abs(phi - (theta / 2 + CONE_PAD)) < 2e-6


def test_fold_two_rays_far_edge():
    """A cone of half-angle phi around +z plus a ray at angle theta > phi
    in the xz plane: the new half-angle is (phi + theta)/2 and the axis sits
    at (theta - phi)/2 from +z towards the ray (Eq. 1-4)."""
    phi, theta = 0.2, 0.9
    x = np.array([0, 0, 1], np.float32)
    r = np.array([np.sin(theta), 0, np.cos(theta)], np.float32)
    out = O.cone_add_ray(x, np.float32(np.cos(phi)), np.float32(np.sin(phi)), r).astype(np.float64)
    ax = np.array([np.sin((theta - phi) / 2), 0, np.cos((theta - phi) / 2)])
    assert _ang(out[:3], ax) < 1e-6
    assert abs(np.arctan2(out[4], out[3]) - ((phi + theta) / 2 + CONE_PAD)) < 2e-6


def test_fold_antiparallel_and_wide_become_full():
    x = np.array([0, 0, 1], np.float32)
    out = O.cone_add_ray(x, 1.0, 0.0, -x)
    assert out[3] == -1.0 and out[4] == 0.0
    # two rays 172 degrees apart: the bisector is too ill-conditioned, full
    r = np.array([np.sin(3.0), 0, np.cos(3.0)], np.float32)
    out = O.cone_add_ray(x, 1.0, 0.0, r)
    assert out[3] == -1.0 and out[4] == 0.0
    # cone of 60 deg + ray at 150 deg: new half-angle 105 deg -> full
    r = np.array([np.sin(2.618), 0, np.cos(2.618)], np.float32)
    out = O.cone_add_ray(x, np.float32(0.5), np.float32(np.sqrt(0.75)), r)
    assert out[3] == -1.0 and out[4] == 0.0


def test_cone_union_closed_forms():
    # equal axes: the larger child's angle, widened by PAD
    x = np.array([0, 1, 0], np.float32)
    a = np.array([0, 1, 0, np.cos(0.1), np.sin(0.1)], np.float32)
    b = np.array([0, 1, 0, np.cos(0.3), np.sin(0.3)], np.float32)
    out = O.cone_union(a, b).astype(np.float64)
    assert np.array_equal(out[:3], x)
    assert abs(np.arctan2(out[4], out[3]) - (0.3 + CONE_PAD)) < 1e-6
    # axes 0.8 rad apart, spreads 0.1 and 0.2: half the axis angle + the larger spread
    a = np.array([1, 0, 0, np.cos(0.1), np.sin(0.1)], np.float32)
    b = np.array([np.cos(0.8), np.sin(0.8), 0, np.cos(0.2), np.sin(0.2)], np.float32)
    out = O.cone_union(a, b).astype(np.float64)
    assert _ang(out[:3], np.array([np.cos(0.4), np.sin(0.4), 0])) < 1e-6
    assert abs(np.arctan2(out[4], out[3]) - (0.4 + 0.2 + CONE_PAD)) < 2e-6
    # a full child makes a full parent; opposite axes make a full parent
    f = np.array([1, 0, 0, -1, 0], np.float32)
    assert O.cone_union(a, f)[3] == -1
    opp = np.array([-1, 0, 0, 1, 0], np.float32)
    assert O.cone_union(np.array([1, 0, 0, 1, 0], np.float32), opp)[3] == -1
    # union wider than 90 degrees is full (45 deg + 0.9 rad)
    w1 = np.array([1, 0, 0, np.cos(0.9), np.sin(0.9)], np.float32)
    w2 = np.array([0, 1, 0, np.cos(0.2), np.sin(0.2)], np.float32)
    assert O.cone_union(w1, w2)[3] == -1


def test_sphere_union_closed_form():
    a = np.array([0, 0, 0, 1], np.float32)
    b = np.array([4, 0, 0, 1], np.float32)
    out = O.sphere_union(a, b)
    r = np.float32(3.0)
    r = np.float32(r + np.float32(PAD) * np.float32(r + np.float32(2.0)))
    assert np.array_equal(out, np.array([2, 0, 0, r], np.float32))
    # nested spheres: the union still contains both
    a = np.array([1, 2, 3, 5], np.float32)
    b = np.array([1.5, 2, 3, 0.5], np.float32)
    out = O.sphere_union(a, b).astype(np.float64)
    for q in (a, b):
        q = q.astype(np.float64)
        assert np.linalg.norm(q[:3] - out[:3]) + q[3] <= out[3]


def test_random_unions_contain_children(rng):
    for _ in range(2000):
        ca = rng.normal(size=3) * 10
        cb = ca + rng.normal(size=3) * rng.choice([1e-4, 1e-2, 1, 10])
        ra, rb = rng.uniform(0, 2, size=2)
        a = np.r_[ca, ra].astype(np.float32)
        b = np.r_[cb, rb].astype(np.float32)
        u = O.sphere_union(a, b).astype(np.float64)
        for q in (a, b):
            q = q.astype(np.float64)
            assert np.linalg.norm(q[:3] - u[:3]) + q[3] <= u[3]
        xa = rng.normal(size=3)
        xa /= np.linalg.norm(xa)
        xb = xa + rng.normal(size=3) * rng.choice([1e-5, 1e-3, 0.1, 1])
        xb /= np.linalg.norm(xb)
        pa, pb = rng.uniform(0, 0.7, size=2)
        A = np.r_[xa, np.cos(pa), np.sin(pa)].astype(np.float32)
        Bc = np.r_[xb, np.cos(pb), np.sin(pb)].astype(np.float32)
        k = O.cone_union(A, Bc).astype(np.float64)
        if k[3] <= 0:
            continue
        phi = np.arctan2(k[4], k[3])
        for q in (A, Bc):
            q = q.astype(np.float64)
            assert _ang(q[:3], k[:3]) + np.arctan2(q[4], q[3]) <= phi + 1e-12


def test_random_folds_contain_rays(rng):
    for _ in range(300):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        spread = rng.choice([1e-6, 1e-4, 1e-2, 0.3])
        d = axis + rng.normal(size=(16, 3)) * spread
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        d32 = d.astype(np.float32)
        x, c, s = d32[0], np.float32(1), np.float32(0)
        for r in d32[1:]:
            out = O.cone_add_ray(x, c, s, r)
            x, c, s = out[:3], out[3], out[4]
        if c <= 0:
            continue
        phi = np.arctan2(np.float64(s), np.float64(c))
        assert np.all(_ang(d32.astype(np.float64), x.astype(np.float64)) <= phi + 1e-12)


def _tri_scene(tris):
    from workloads.scenes import Scene
    tris = np.ascontiguousarray(tris, np.float32)
    m = len(tris)
    return Scene(tris=tris, mesh_first=np.zeros(1, np.uint32), mesh_count=np.array([m], np.uint32),
                 mesh_sphere=np.zeros((1, 4), np.float32), mesh_mat=np.zeros(1, np.int32),
                 mat_flags=np.zeros(1, np.uint32), mat_ior=np.ones(1, np.float32))


def test_triangle_spheres_closed_forms():
    """Triangle bounding spheres (the spheres of Eq. 9's coarse tests):
    centroid and largest centroid-vertex distance.  A right triangle with
    legs 3 on the axes has centroid (1, 1, 0) and farthest vertices at
    sqrt(5); an equilateral triangle of circumradius 2 centred at c has its
    centroid at c and every vertex at 2; a degenerate triangle (one point)
    has radius (nearly) zero.  The padding widens by at most 2^-20 of
    (radius + largest centre coordinate)."""
    s3 = np.sqrt(3.0)
    c = np.array([5.0, -7.0, 11.0])
    tris = np.array([
        [[0, 0, 0], [3, 0, 0], [0, 3, 0]],
        [c + [2, 0, 0], c + [-1, s3, 0], c + [-1, -s3, 0]],
        [[1.5, 2.5, -4], [1.5, 2.5, -4], [1.5, 2.5, -4]],
    ], np.float64)
    cx, cy, cz, r = (x.astype(np.float64) for x in O.tri_spheres(_tri_scene(tris)))
    want_c = [[1, 1, 0], c, [1.5, 2.5, -4]]
    want_r = [np.sqrt(5.0), 2.0, 0.0]
    for i in range(3):
        got_c = np.array([cx[i], cy[i], cz[i]])
        assert np.allclose(got_c, want_c[i], rtol=0, atol=4e-6 * (1 + np.abs(want_c[i]).max())), i
        slack = 2.0 ** -20 * (want_r[i] + np.abs(want_c[i]).max()) + 1e-5 * want_r[i] + 1e-6
        assert want_r[i] - 1e-6 <= r[i] <= want_r[i] + slack, (i, r[i])


@pytest.mark.parametrize("name", ["shadow_128", "refl_96", "mixed_128x72"])
def test_triangle_spheres_contain_every_vertex(name):
    """Every vertex of every triangle of the workload lies inside its
    triangle's sphere in float64, and no sphere is looser than its float64
    centroid-vertex distance by more than the padding."""
    base, kw = small(name)
    sc = workload(base, **kw).scene
    cx, cy, cz, r = (x.astype(np.float64) for x in O.tri_spheres(sc))
    ctr = np.stack([cx, cy, cz], 1)
    d = np.linalg.norm(sc.tris.astype(np.float64) - ctr[:, None, :], axis=2).max(axis=1)
    assert np.all(d <= r)
    m = np.abs(ctr).max(axis=1)
    assert np.all(r <= d * (1 + 2.0 ** -18) + 2.0 ** -18 * m + 1e-30)
