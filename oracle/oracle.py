"""ctypes front end of the plain C oracle (``oracle/crsh_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  numpy arrays in,
numpy arrays out; every step runs in the C file, written in binary32 with a
fixed operation order.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "crsh_oracle.c")
LIB = os.path.join(HERE, "libcrsh_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared"]
MAX_LEVELS = 16

f32p = C.POINTER(C.c_float)
u32p = C.POINTER(C.c_uint32)
i32p = C.POINTER(C.c_int32)
u64p = C.POINTER(C.c_uint64)
f64p = C.POINTER(C.c_double)


def compile_lib():
    """Compile the oracle with gcc (always; the checker must match its source)."""
    subprocess.check_call(["gcc", *CFLAGS, "-o", LIB, SRC, "-lm"])


class Gbuf(C.Structure):
    _fields_ = [("w", C.c_int32), ("h", C.c_int32),
                ("px", f32p), ("py", f32p), ("pz", f32p),
                ("nx", f32p), ("ny", f32p), ("nz", f32p), ("mat", i32p)]


class Raygen(C.Structure):
    _fields_ = [("n_lights", C.c_int32), ("lights", (C.c_float * 3) * 4), ("eye", C.c_float * 3),
                ("mat_flags", u32p), ("mat_ior", f32p), ("n_mats", C.c_int32),
                ("ray_types", C.c_uint32), ("eps_off", C.c_float), ("eps_shadow", C.c_float),
                ("lo", C.c_float * 3), ("inv_ext", C.c_float * 3)]


class Rays(C.Structure):
    _fields_ = [(k, f32p) for k in ("ox", "oy", "oz", "dx", "dy", "dz", "tmax")] + [("pix", u32p)]


class Nodes(C.Structure):
    _fields_ = [(k, f32p) for k in ("cx", "cy", "cz", "r", "ax", "ay", "az", "c", "s", "tan", "sec")]


RAY_FIELDS = ("ox", "oy", "oz", "dx", "dy", "dz", "tmax")
NODE_FIELDS = ("cx", "cy", "cz", "r", "ax", "ay", "az", "c", "s", "tan", "sec")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            compile_lib()
        L = C.CDLL(LIB)
        L.orc_hash.restype = C.c_int64
        L.orc_hash.argtypes = [C.POINTER(Gbuf), C.POINTER(Raygen), C.POINTER(Rays), u32p, u32p, C.c_uint32]
        L.orc_sort.argtypes = [u32p, u32p, C.c_uint32, u32p, u32p]
        L.orc_bounce.restype = C.c_int64
        L.orc_bounce.argtypes = [C.POINTER(Rays), u32p, C.c_uint32, i32p, f32p, f32p * 9, C.c_uint32, i32p,
                                 C.POINTER(Raygen), C.POINTER(Rays), u32p, u32p, C.c_uint32]
        L.orc_level_counts.restype = C.c_int
        L.orc_level_counts.argtypes = [C.c_uint32, C.c_int, C.c_int, C.c_int, u32p]
        L.orc_build.restype = C.c_int
        L.orc_build.argtypes = [C.POINTER(Rays), u32p, C.c_uint32, C.c_int, C.c_int, C.c_int,
                                C.POINTER(Nodes), u32p, u32p]
        L.orc_tri_spheres.argtypes = [f32p * 9, C.c_uint32, f32p, f32p, f32p, f32p]
        L.orc_traverse.restype = C.c_void_p
        L.orc_traverse.argtypes = [C.POINTER(Nodes), u32p, u32p, C.c_int, C.c_uint32, C.c_int, C.c_int,
                                   f32p, f32p, f32p, f32p, u32p, u32p, C.c_uint32, f32p,
                                   C.c_uint32, C.c_uint32, u32p, C.c_uint32]
        L.orc_trav_count.restype = C.c_uint64
        L.orc_trav_count.argtypes = [C.c_void_p, C.c_int]
        L.orc_trav_copy.argtypes = [C.c_void_p, C.c_int, u32p, u32p]
        L.orc_trav_counters.argtypes = [C.c_void_p, u64p, u64p]
        L.orc_trav_free.argtypes = [C.c_void_p]
        L.orc_closest_hit.argtypes = [C.POINTER(Rays), u32p, C.c_uint32, C.c_int, u32p, u32p, C.c_uint64,
                                      f32p * 9, C.c_float, i32p, f32p, f32p, f32p, u64p]
        L.orc_brute_closest_hit.argtypes = [C.POINTER(Rays), u32p, C.c_uint32, f32p * 9, C.c_uint32,
                                            C.c_float, i32p, f32p, f32p, f32p]
        L.orc_brute_all_hits.restype = C.c_uint64
        L.orc_brute_all_hits.argtypes = [C.POINTER(Rays), u32p, C.c_uint32, f32p * 9, C.c_uint32,
                                         C.c_float, u32p, u32p, C.c_uint64]
        L.orc_mt.restype = C.c_int
        L.orc_mt.argtypes = [f32p, f32p, C.c_float, C.c_float, f32p, f32p]
        L.orc_mt64.restype = C.c_int
        L.orc_mt64.argtypes = [f64p, f64p, f64p, f64p]
        L.orc_shadow_key.restype = C.c_uint32
        L.orc_shadow_key.argtypes = [C.c_int, f32p]
        L.orc_bounce_key.restype = C.c_uint32
        L.orc_bounce_key.argtypes = [C.c_uint32, f32p, f32p, C.POINTER(Raygen)]
        L.orc_oct_code.argtypes = [f32p, C.c_int, u32p, u32p]
        L.orc_sph_code.argtypes = [f32p, C.c_int, u32p, u32p]
        L.orc_cone_add_ray.argtypes = [f32p, C.c_float, C.c_float, f32p, f32p]
        L.orc_cone_union.argtypes = [f32p, f32p, f32p]
        L.orc_sphere_union.argtypes = [f32p, f32p, f32p]
        L.orc_node_sphere_test.restype = C.c_int
        L.orc_node_sphere_test.argtypes = [f32p, f32p]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def make_raygen(wl):
    g = Raygen()
    L = len(wl.lights)
    g.n_lights = L
    for i in range(L):
        for k in range(3):
            g.lights[i][k] = float(wl.lights[i][k])
    for k in range(3):
        g.eye[k] = float(wl.eye[k])
        g.lo[k] = float(wl.lo[k])
        g.inv_ext[k] = float(wl.inv_ext[k])
    sc = wl.scene
    g._keep = (_u32(sc.mat_flags), _f32(sc.mat_ior))
    g.mat_flags = _p(g._keep[0], u32p)
    g.mat_ior = _p(g._keep[1], f32p)
    g.n_mats = len(sc.mat_flags)
    g.ray_types = wl.ray_types
    g.eps_off = wl.eps_off
    g.eps_shadow = wl.eps_shadow
    return g


def _rays_struct(r):
    s = Rays()
    for k in RAY_FIELDS:
        setattr(s, k, _p(r[k], f32p))
    s.pix = _p(r["pix"], u32p)
    return s


def hash_rays(wl):
    """Stage 1.  Returns dict: rays (ox..tmax float32, pix uint32), keys, ids, n."""
    gbuf = {k: _f32(wl.gbuf[k]) for k in ("px", "py", "pz", "nx", "ny", "nz")}
    mat = np.ascontiguousarray(wl.gbuf["mat"], dtype=np.int32)
    gb = Gbuf(wl.W, wl.H, *[_p(gbuf[k], f32p) for k in ("px", "py", "pz", "nx", "ny", "nz")],
              _p(mat, i32p))
    g = make_raygen(wl)
    cap = wl.n_slots
    r = {k: np.zeros(cap, np.float32) for k in RAY_FIELDS}
    r["pix"] = np.zeros(cap, np.uint32)
    keys = np.zeros(cap, np.uint32)
    ids = np.zeros(cap, np.uint32)
    rs = _rays_struct(r)
    n = lib().orc_hash(C.byref(gb), C.byref(g), C.byref(rs), _p(keys, u32p), _p(ids, u32p), cap)
    assert n >= 0
    out = {k: v[:n].copy() for k, v in r.items()}
    return {"rays": out, "keys": keys[:n].copy(), "ids": ids[:n].copy(), "n": int(n)}


def sort_rays(keys, ids):
    """Stage 2: (keys, ids) ordered by key, ties by id."""
    keys = _u32(keys)
    ids = _u32(ids)
    n = len(keys)
    ko = np.zeros(n, np.uint32)
    io = np.zeros(n, np.uint32)
    lib().orc_sort(_p(keys, u32p), _p(ids, u32p), n, _p(ko, u32p), _p(io, u32p))
    return ko, io


def level_counts(n_rays, B, F, levels):
    cnt = np.zeros(MAX_LEVELS, np.uint32)
    nl = lib().orc_level_counts(n_rays, B, F, levels, _p(cnt, u32p))
    return cnt[:nl].copy()


def build_tree(rays, sorted_ids, B, F, levels):
    """Stage 3.  Returns dict: node arrays (all levels concatenated, level 1
    first), level_off, level_cnt, n_levels."""
    rays = {k: _f32(rays[k]) for k in RAY_FIELDS} | {"pix": _u32(rays["pix"])}
    sorted_ids = _u32(sorted_ids)
    n = len(sorted_ids)
    cnt = level_counts(n, B, F, levels)
    total = int(cnt.sum())
    nodes = {k: np.zeros(max(total, 1), np.float32) for k in NODE_FIELDS}
    ns = Nodes(*[_p(nodes[k], f32p) for k in NODE_FIELDS])
    off = np.zeros(MAX_LEVELS, np.uint32)
    cn = np.zeros(MAX_LEVELS, np.uint32)
    rs = _rays_struct(rays)
    nl = lib().orc_build(C.byref(rs), _p(sorted_ids, u32p), n, B, F, levels, C.byref(ns),
                         _p(off, u32p), _p(cn, u32p))
    nodes = {k: v[:total].copy() for k, v in nodes.items()}
    return {"nodes": nodes, "level_off": off[:nl].copy(), "level_cnt": cn[:nl].copy(),
            "n_levels": int(nl), "n_rays": n, "B": B, "F": F}


def tri_spheres(scene):
    v = [_f32(a) for a in scene.soa()]
    m = scene.m
    out = [np.zeros(m, np.float32) for _ in range(4)]
    arr = (f32p * 9)(*[_p(a, f32p) for a in v])
    lib().orc_tri_spheres(arr, m, *[_p(a, f32p) for a in out])
    return out


def traverse(tree, scene, tri_begin=0, tri_end=None, top_subset=None, tsph=None):
    """Stage 4.  Returns dict: pairs {level: (tri, node)}, tests[level],
    hits[level], mesh_tests, mesh_hits, final_tests."""
    if tri_end is None:
        tri_end = scene.m
    if tsph is None:
        tsph = tri_spheres(scene)
    nodes = {k: _f32(tree["nodes"][k]) for k in NODE_FIELDS}
    ns = Nodes(*[_p(nodes[k], f32p) for k in NODE_FIELDS])
    off = _u32(np.resize(tree["level_off"], MAX_LEVELS) if len(tree["level_off"]) else np.zeros(MAX_LEVELS))
    cnt = _u32(np.resize(tree["level_cnt"], MAX_LEVELS) if len(tree["level_cnt"]) else np.zeros(MAX_LEVELS))
    msph = _f32(scene.mesh_sphere.reshape(-1))
    mf = _u32(scene.mesh_first)
    mc = _u32(scene.mesh_count)
    if top_subset is not None:
        sub = _u32(top_subset)
        subp, nsub = _p(sub, u32p), len(sub)
    else:
        subp, nsub = None, 0
    L = lib()
    T = L.orc_traverse(C.byref(ns), _p(off, u32p), _p(cnt, u32p), tree["n_levels"], tree["n_rays"],
                       tree["B"], tree["F"], *[_p(a, f32p) for a in tsph], _p(mf, u32p), _p(mc, u32p),
                       scene.n_mesh, _p(msph, f32p), tri_begin, tri_end, subp, nsub)
    try:
        pairs = {}
        for lv in range(1, tree["n_levels"] + 1):
            n = L.orc_trav_count(T, lv)
            tri = np.zeros(n, np.uint32)
            nd = np.zeros(n, np.uint32)
            if n:
                L.orc_trav_copy(T, lv, _p(tri, u32p), _p(nd, u32p))
            pairs[lv] = (tri, nd)
        tests = np.zeros(MAX_LEVELS, np.uint64)
        misc = np.zeros(3, np.uint64)
        L.orc_trav_counters(T, _p(tests, u64p), _p(misc, u64p))
    finally:
        L.orc_trav_free(T)
    nl = tree["n_levels"]
    return {"pairs": pairs,
            "tests": {lv: int(tests[lv - 1]) for lv in range(1, nl + 1)},
            "hits": {lv: len(pairs[lv][0]) for lv in range(1, nl + 1)},
            "mesh_tests": int(misc[0]), "mesh_hits": int(misc[1]), "final_tests": int(misc[2])}


def _tri_arr(scene):
    v = [_f32(a) for a in scene.soa()]
    return v, (f32p * 9)(*[_p(a, f32p) for a in v])


def closest_hit(rays, sorted_ids, B, pairs1, scene, t_min, init=None, stages=None):
    """Stage 5 over the level-1 pairs.  Returns (tri int32, t, u, v) by ray id.
    With `stages` (a dict), adds to stages["u"] / stages["uv"] the tests whose
    u passed / whose u and v passed."""
    rays = {k: _f32(rays[k]) for k in RAY_FIELDS} | {"pix": _u32(rays["pix"])}
    sorted_ids = _u32(sorted_ids)
    n = len(sorted_ids)
    if init is None:
        tri = np.full(n, -1, np.int32)
        t, u, v = (np.zeros(n, np.float32) for _ in range(3))
    else:
        tri, t, u, v = (a.copy() for a in init)
    ptri, pnode = _u32(pairs1[0]), _u32(pairs1[1])
    keep, arr = _tri_arr(scene)
    rs = _rays_struct(rays)
    cnt = np.zeros(2, np.uint64)
    lib().orc_closest_hit(C.byref(rs), _p(sorted_ids, u32p), n, B, _p(ptri, u32p), _p(pnode, u32p),
                          len(ptri), arr, t_min, _p(tri, i32p), _p(t, f32p), _p(u, f32p), _p(v, f32p),
                          _p(cnt, u64p))
    if stages is not None:
        stages["u"] = stages.get("u", 0) + int(cnt[0])
        stages["uv"] = stages.get("uv", 0) + int(cnt[1])
    return tri, t, u, v


def bounce(rays, keys, hits, wl):
    """The next generation of secondary rays from the closest hits of the
    reflection / refraction rays (Sec. 3.3.8), with the ray-generation
    parameters of the workload (lights, materials, key box).  Returns the
    same dict as hash_rays."""
    rays = {k: _f32(rays[k]) for k in RAY_FIELDS} | {"pix": _u32(rays["pix"])}
    keys = _u32(keys)
    n_par = len(keys)
    tri = np.ascontiguousarray(hits[0], np.int32)
    t = _f32(hits[1])
    tri_mat = np.ascontiguousarray(wl.scene.tri_mat(), np.int32)
    g = make_raygen(wl)
    cap = max(n_par * (len(wl.lights) + 2), 1)
    r = {k: np.zeros(cap, np.float32) for k in RAY_FIELDS}
    r["pix"] = np.zeros(cap, np.uint32)
    out_keys = np.zeros(cap, np.uint32)
    ids = np.zeros(cap, np.uint32)
    keep, arr = _tri_arr(wl.scene)
    ps, rs = _rays_struct(rays), _rays_struct(r)
    n = lib().orc_bounce(C.byref(ps), _p(keys, u32p), n_par, _p(tri, i32p), _p(t, f32p), arr, wl.scene.m,
                         _p(tri_mat, i32p), C.byref(g), C.byref(rs), _p(out_keys, u32p), _p(ids, u32p), cap)
    assert n >= 0
    return {"rays": {k: v[:n].copy() for k, v in r.items()}, "keys": out_keys[:n].copy(), "ids": ids[:n].copy(),
            "n": int(n)}


def run_generations(wl, depth, leaf_top_subset=None):
    """`depth` generations of the whole path: the first from the primary-hit
    buffer, each next one from the closest hits of the previous (bounce).
    Returns the list of per-generation dicts (as run_pipeline, plus the
    generation's rays under "hash")."""
    out = []
    h = hash_rays(wl)
    for gen in range(depth):
        ks, ids = sort_rays(h["keys"], h["ids"])
        tree = build_tree(h["rays"], ids, wl.B, wl.F, wl.n)
        tr = traverse(tree, wl.scene)
        if tree["n_levels"]:
            hits = closest_hit(h["rays"], ids, wl.B, tr["pairs"][1], wl.scene, wl.t_min)
        else:
            n = h["n"]
            hits = (np.full(n, -1, np.int32), np.zeros(n, np.float32), np.zeros(n, np.float32),
                    np.zeros(n, np.float32))
        out.append({"hash": h, "sorted_keys": ks, "sorted_ids": ids, "tree": tree, "trav": tr, "hits": hits})
        if gen + 1 < depth:
            h = bounce(h["rays"], h["keys"], hits, wl)
    return out


def brute_closest_hit(rays, ray_list, scene, t_min):
    """Naive N x M closest hit of the listed rays (by ray id)."""
    rays = {k: _f32(rays[k]) for k in RAY_FIELDS} | {"pix": _u32(rays["pix"])}
    rl = _u32(ray_list)
    n = len(rl)
    tri = np.full(n, -1, np.int32)
    t, u, v = (np.zeros(n, np.float32) for _ in range(3))
    keep, arr = _tri_arr(scene)
    rs = _rays_struct(rays)
    lib().orc_brute_closest_hit(C.byref(rs), _p(rl, u32p), n, arr, scene.m, t_min,
                                _p(tri, i32p), _p(t, f32p), _p(u, f32p), _p(v, f32p))
    return tri, t, u, v


def brute_all_hits(rays, ray_list, scene, t_min, cap=1 << 24):
    rays = {k: _f32(rays[k]) for k in RAY_FIELDS} | {"pix": _u32(rays["pix"])}
    rl = _u32(ray_list)
    o_r = np.zeros(cap, np.uint32)
    o_t = np.zeros(cap, np.uint32)
    keep, arr = _tri_arr(scene)
    rs = _rays_struct(rays)
    n = lib().orc_brute_all_hits(C.byref(rs), _p(rl, u32p), len(rl), arr, scene.m, t_min,
                                 _p(o_r, u32p), _p(o_t, u32p), cap)
    assert n <= cap
    return o_r[:n].copy(), o_t[:n].copy()


def mt(o, d, t_min, tmax, tri9):
    o, d, tri9 = _f32(o), _f32(d), _f32(tri9)
    out = np.zeros(3, np.float32)
    hit = lib().orc_mt(_p(o, f32p), _p(d, f32p), t_min, tmax, _p(tri9, f32p), _p(out, f32p))
    return bool(hit), out


def mt64(o, d, tri9):
    o = np.ascontiguousarray(o, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    tri9 = np.ascontiguousarray(tri9, np.float64)
    out = np.zeros(3, np.float64)
    ok = lib().orc_mt64(_p(o, f64p), _p(d, f64p), _p(tri9, f64p), _p(out, f64p))
    return bool(ok), out


def adjoint64(o, d, tri9, g):
    """Gradient of g . (t, u, v) of the float64 Moller-Trumbore solution
    (Sec. 3.3.8) with respect to v0, v1, v2, O and D, the hit triangle held
    fixed.  Plain definition: (t, u, v) solves [D | -e1 | -e2] (t, u, v)^T =
    v0 - O with e1 = v1 - v0, e2 = v2 - v0; by the implicit function theorem
    the gradient is lam^T times the derivative of the residual, where
    [D | -e1 | -e2]^T lam = g.  Returns (dv0, dv1, dv2, dO, dD, cond) in
    float64; cond is the 2-norm condition number of the matrix."""
    o, d, tri9, g = (np.asarray(x, np.float64) for x in (o, d, tri9, g))
    v0, v1, v2 = tri9[0:3], tri9[3:6], tri9[6:9]
    e1, e2 = v1 - v0, v2 - v0
    M = np.stack([d, -e1, -e2], axis=1)
    t, u, v = np.linalg.solve(M, v0 - o)
    lam = np.linalg.solve(M.T, g)
    # residual r = O + t D - (1-u-v) v0 - u v1 - v v2 = 0
    return ((1.0 - u - v) * lam, u * lam, v * lam, -lam, -t * lam, float(np.linalg.cond(M)))


def shadow_key(light, d):
    d = _f32(d)
    return int(lib().orc_shadow_key(light, _p(d, f32p)))


def bounce_key(typ, o, d, wl):
    o, d = _f32(o), _f32(d)
    g = make_raygen(wl)
    return int(lib().orc_bounce_key(typ, _p(o, f32p), _p(d, f32p), C.byref(g)))


def sph_code(d, k):
    d = _f32(d)
    u = np.zeros(1, np.uint32)
    v = np.zeros(1, np.uint32)
    lib().orc_sph_code(_p(d, f32p), k, _p(u, u32p), _p(v, u32p))
    return int(u[0]), int(v[0])


def oct_code(d, k):
    d = _f32(d)
    u = np.zeros(1, np.uint32)
    v = np.zeros(1, np.uint32)
    lib().orc_oct_code(_p(d, f32p), k, _p(u, u32p), _p(v, u32p))
    return int(u[0]), int(v[0])


def cone_add_ray(x, c, s, r):
    x, r = _f32(x), _f32(r)
    out = np.zeros(5, np.float32)
    lib().orc_cone_add_ray(_p(x, f32p), c, s, _p(r, f32p), _p(out, f32p))
    return out


def cone_union(a5, b5):
    a5, b5 = _f32(a5), _f32(b5)
    out = np.zeros(5, np.float32)
    lib().orc_cone_union(_p(a5, f32p), _p(b5, f32p), _p(out, f32p))
    return out


def sphere_union(a4, b4):
    a4, b4 = _f32(a4), _f32(b4)
    out = np.zeros(4, np.float32)
    lib().orc_sphere_union(_p(a4, f32p), _p(b4, f32p), _p(out, f32p))
    return out


def node_sphere_test(node11, sph4):
    node11, sph4 = _f32(node11), _f32(sph4)
    return bool(lib().orc_node_sphere_test(_p(node11, f32p), _p(sph4, f32p)))


def run_pipeline(wl, top_subset=None, tri_batches=None):
    """All five stages on one workload; returns a dict of every product."""
    h = hash_rays(wl)
    ks, ids = sort_rays(h["keys"], h["ids"])
    tree = build_tree(h["rays"], ids, wl.B, wl.F, wl.n)
    tsph = tri_spheres(wl.scene)
    batches = tri_batches or [(0, wl.scene.m)]
    hits = None
    travs = []
    stages = {"u": 0, "uv": 0}
    for (b, e) in batches:
        tr = traverse(tree, wl.scene, b, e, top_subset=top_subset, tsph=tsph)
        travs.append(tr)
        if tree["n_levels"]:
            hits = closest_hit(h["rays"], ids, wl.B, tr["pairs"][1], wl.scene, wl.t_min, init=hits, stages=stages)
    if hits is None:
        n = h["n"]
        hits = (np.full(n, -1, np.int32), np.zeros(n, np.float32), np.zeros(n, np.float32),
                np.zeros(n, np.float32))
    return {"hash": h, "sorted_keys": ks, "sorted_ids": ids, "tree": tree, "tsph": tsph,
            "trav": travs[0] if len(travs) == 1 else travs, "hits": hits, "stages": stages}
