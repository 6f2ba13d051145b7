"""Seeded synthetic workloads standing in for the paper's scenes.

The paper measures on OFFICE, CORNELL and SPONZA (Sec. 4.2), which are not
available; these procedural scenes replace them.  A workload bundles:

* the scene: float32 triangles grouped into meshes, one enclosing sphere per
  mesh (Sec. 3.3.1 precomputes a minimum ball per mesh; any enclosing sphere
  is valid, here Ritter's construction refined by a few Badoiu-Clarkson
  steps, in float64, rounded outwards to float32), a material per mesh;
* the primary-hit buffer from ``workloads.caster`` (Sec. 3.2);
* the ray-generation inputs (lights, eye, material table) and the hierarchy
  parameters (bundle size B, merge factor F, level count n, Sec. 3.3.6).

Input generation only: no step of the secondary-ray path lives here.
"""
from dataclasses import dataclass, field, replace

import numpy as np

from . import meshes as _m
from .caster import cast_primary

SHADOW, REFLECT, REFRACT = 1, 2, 4
KEY_TYPE_ONLY = 0x100           # keys of ray type and light only (comparison mode)
KEY_SPHERICAL = 0x200           # spherical-coordinate direction codes
MAT_REFLECT, MAT_REFRACT = 1, 2


@dataclass
class Scene:
    tris: np.ndarray          # float32 [M, 3, 3]
    mesh_first: np.ndarray    # uint32 [n_mesh]
    mesh_count: np.ndarray    # uint32 [n_mesh]
    mesh_sphere: np.ndarray   # float32 [n_mesh, 4]  (cx, cy, cz, r)
    mesh_mat: np.ndarray      # int32 [n_mesh]
    mat_flags: np.ndarray     # uint32 [n_mat]   bit0 reflective, bit1 refractive
    mat_ior: np.ndarray       # float32 [n_mat]
    verts: np.ndarray = None  # float32 [V, 3] (indexed form, when requested)
    faces: np.ndarray = None  # int32 [M, 3]

    @property
    def m(self):
        return int(self.tris.shape[0])

    @property
    def n_mesh(self):
        return int(self.mesh_first.shape[0])

    def tri_mat(self):
        return np.repeat(self.mesh_mat, self.mesh_count.astype(np.int64))

    def soa(self):
        """Nine float32 arrays v0x, v0y, v0z, v1x, ..., v2z."""
        return [np.ascontiguousarray(self.tris[:, k // 3, k % 3]) for k in range(9)]


@dataclass
class Workload:
    name: str
    seed: int
    scene: Scene
    W: int
    H: int
    eye: np.ndarray           # float32 [3]
    look: np.ndarray
    vfov: float
    lights: np.ndarray        # float32 [L, 3]
    gbuf: dict                # px..nz float32, mat int32, tri int32 (length W*H)
    B: int
    F: int
    n: int
    ray_types: int
    eps_off: float = 1e-3
    eps_shadow: float = 1e-3
    t_min: float = 1e-4
    lo: np.ndarray = None     # float32 [3] origin-quantisation box
    inv_ext: np.ndarray = None
    extra: dict = field(default_factory=dict)

    @property
    def n_slots(self):
        return self.W * self.H * (len(self.lights) + 2)


def enclosing_sphere(v):
    """Conservative float32 sphere around float64 points v [V,3]."""
    x = v[0]
    y = v[np.argmax(((v - x) ** 2).sum(1))]
    z = v[np.argmax(((v - y) ** 2).sum(1))]
    c = 0.5 * (y + z)
    r = 0.5 * np.linalg.norm(z - y)
    for _ in range(len(v)):  # Ritter growth, farthest outside point first
        dist = np.sqrt(((v - c) ** 2).sum(1))
        k = int(np.argmax(dist))
        d = dist[k]
        if d <= r:
            break
        nr = 0.5 * (r + d)
        c = c + (v[k] - c) * ((nr - r) / d)
        r = nr
    cb = v.mean(0)
    for i in range(1, 65):  # Badoiu-Clarkson refinement from the centroid
        far = v[np.argmax(((v - cb) ** 2).sum(1))]
        cb = cb + (far - cb) / (i + 1)
    rb = np.sqrt(((v - cb) ** 2).sum(1).max())
    if rb < r:
        c, r = cb, rb
    c32 = c.astype(np.float32)
    r64 = np.sqrt(((v - c32.astype(np.float64)) ** 2).sum(1).max())
    r64 = r64 * (1.0 + 2.0 ** -20) + 2.0 ** -20 * float(np.abs(c32).max())
    r32 = np.nextafter(np.float32(r64), np.float32(np.inf))
    return np.array([c32[0], c32[1], c32[2], r32], dtype=np.float32)


def _assemble(mesh_list, mats, mat_flags, mat_ior, indexed=False):
    tris, first, count, sph, vlist, flist = [], [], [], [], [], []
    off = 0
    voff = 0
    for (v, f) in mesh_list:
        v32 = v.astype(np.float32)
        t = v32[f]
        tris.append(t)
        first.append(off)
        count.append(len(f))
        off += len(f)
        sph.append(enclosing_sphere(v32.astype(np.float64)[np.unique(f)]))
        if indexed:
            vlist.append(v32)
            flist.append(f + voff)
            voff += len(v32)
    sc = Scene(
        tris=np.ascontiguousarray(np.concatenate(tris).astype(np.float32)),
        mesh_first=np.array(first, dtype=np.uint32),
        mesh_count=np.array(count, dtype=np.uint32),
        mesh_sphere=np.array(sph, dtype=np.float32),
        mesh_mat=np.array(mats, dtype=np.int32),
        mat_flags=np.array(mat_flags, dtype=np.uint32),
        mat_ior=np.array(mat_ior, dtype=np.float32),
    )
    if indexed:
        sc.verts = np.ascontiguousarray(np.concatenate(vlist).astype(np.float32))
        sc.faces = np.ascontiguousarray(np.concatenate(flist).astype(np.int32))
    return sc


def _place(v, rng, center, scale):
    R = _m.random_rotation(rng)
    return (v @ R.T) * scale + center


def _proc_mesh(rng, family, res):
    if family == 0:
        v, f = _ico(res["ico"])
    elif family == 1:
        v, f = _m.torus(*res["torus"])
    else:
        v, f = _m.displaced_grid(res["grid"], rng)
    return v, f


def _box(tris, pad=1e-3):
    lo = tris.reshape(-1, 3).min(0).astype(np.float64) - pad
    hi = tris.reshape(-1, 3).max(0).astype(np.float64) + pad
    lo32 = lo.astype(np.float32)
    hi32 = hi.astype(np.float32)
    inv = (np.float32(1.0) / (hi32 - lo32)).astype(np.float32)
    return lo32, inv


_ICO = {2: None, 3: None, 4: None}


def _ico(sub):
    if _ICO.get(sub) is None:
        _ICO[sub] = _m.icosphere(sub)
    return _ICO[sub]


def make_shadow_128(seed=0, W=128, H=128, B=8, F=4, n=4):
    """4 icospheres (subdivision 2) + ground quad; 128x128; one light; shadow rays."""
    rng = np.random.default_rng(seed)
    vs, fs = _ico(2)
    mesh_list = []
    for _ in range(4):
        r = rng.uniform(0.5, 1.5)
        c = rng.uniform(-3.0, 3.0, size=3)
        mesh_list.append((vs * r + c, fs))
    g = np.array([[-50, -4, -50], [50, -4, -50], [50, -4, 50], [-50, -4, 50]], dtype=np.float64)
    mesh_list.append((g, np.array([[0, 2, 1], [0, 3, 2]])))
    sc = _assemble(mesh_list, [0] * 5, [0], [1.0])
    eye = np.array([0, 2, 12], np.float32)
    look = np.array([0, 0, 0], np.float32)
    lights = np.array([[5, 10, 5]], np.float32)
    return _finish("shadow_128", seed, sc, W, H, eye, look, 45.0, lights, B, F, n, SHADOW)


def _room(lo, hi, sub=8):
    return _m.room_walls(lo, hi, sub)


def make_refl_1024(seed=0, W=1024, H=1024, n_meshes=64, B=16, F=4, n=5, with_room=True):
    """64 mixed procedural meshes in U[-10,10]^3, 1024^2, shadow + reflection."""
    rng = np.random.default_rng(seed)
    res = {"ico": 3, "torus": (32, 16), "grid": 32}
    mesh_list = []
    for _ in range(n_meshes):
        fam = int(rng.integers(0, 3))
        v, f = _proc_mesh(rng, fam, res)
        v = _place(v, rng, rng.uniform(-10.0, 10.0, size=3), rng.lognormal(0.0, 0.5))
        mesh_list.append((v, f))
    if with_room:
        mesh_list += _room([-30, -16, -30], [30, 30, 42])
    sc = _assemble(mesh_list, [0] * len(mesh_list), [MAT_REFLECT], [1.0])
    eye = np.array([0, 8, 38], np.float32)
    look = np.array([0, 0, 0], np.float32)
    lights = np.array([[15, 25, 15]], np.float32)
    return _finish("refl_1024", seed, sc, W, H, eye, look, 45.0, lights, B, F, n, SHADOW | REFLECT)


def make_mixed_1080p(seed=0, W=1920, H=1080, n_meshes=256, B=16, F=4, n=6, with_room=True):
    """256 meshes in 8 Gaussian clusters, 25 % refractive; 1920x1080; 2 lights."""
    rng = np.random.default_rng(seed)
    res = {"ico": 3, "torus": (48, 24), "grid": 32}
    means = rng.uniform(-10.0, 10.0, size=(8, 3))
    mesh_list, mats = [], []
    for _ in range(n_meshes):
        fam = int(rng.integers(0, 3))
        v, f = _proc_mesh(rng, fam, res)
        c = means[int(rng.integers(0, 8))] + rng.normal(0.0, 3.0, size=3)
        v = _place(v, rng, c, rng.lognormal(0.0, 0.5))
        mesh_list.append((v, f))
        mats.append(1 if rng.uniform() < 0.25 else 0)
    if with_room:
        walls = _room([-35, -18, -35], [35, 32, 50])
        mesh_list += walls
        mats += [0] * len(walls)
    sc = _assemble(mesh_list, mats, [MAT_REFLECT, MAT_REFRACT], [1.0, 1.5])
    eye = np.array([0, 10, 45], np.float32)
    look = np.array([0, 0, 0], np.float32)
    lights = np.array([[15, 25, 15], [-20, 22, -10]], np.float32)
    return _finish("mixed_1080p", seed, sc, W, H, eye, look, 45.0, lights, B, F, n,
                   SHADOW | REFLECT | REFRACT)


def make_adjoint_512(seed=0, W=512, H=512, B=16, F=4, n=5):
    """16 displaced icospheres (subdivision 3, indexed), 512^2 reflection rays."""
    rng = np.random.default_rng(seed)
    vs, fs = _ico(3)
    mesh_list = []
    for _ in range(16):
        noise = _m.value_noise3(rng, freq=2.0)
        v = vs * (1.0 + 0.1 * noise(vs))[:, None]
        r = rng.uniform(0.5, 1.5)
        c = rng.uniform(-6.0, 6.0, size=3)
        mesh_list.append((v * r + c, fs))
    sc = _assemble(mesh_list, [0] * 16, [MAT_REFLECT], [1.0], indexed=True)
    eye = np.array([0, 2, 18], np.float32)
    look = np.array([0, 0, 0], np.float32)
    lights = np.zeros((0, 3), np.float32)
    return _finish("adjoint_512", seed, sc, W, H, eye, look, 45.0, lights, B, F, n, REFLECT)


def make_frame(seed, target_rays, target_tris, B=16, F=4, n=5):
    """One frame of the batched workload: about target_rays shadow + reflection
    rays (square resolution) over about target_tris procedural triangles."""
    rng = np.random.default_rng(seed)
    Wd = max(8, int(np.ceil(np.sqrt(target_rays / 2.0))))
    res = {"ico": 3, "torus": (32, 16), "grid": 32}
    mesh_list = _room([-30, -16, -30], [30, 30, 42], sub=4)
    total = sum(len(f) for _, f in mesh_list)
    while total < target_tris:
        fam = int(rng.integers(0, 3))
        v, f = _proc_mesh(rng, fam, res)
        v = _place(v, rng, rng.uniform(-10.0, 10.0, size=3), rng.lognormal(0.0, 0.5))
        mesh_list.append((v, f))
        total += len(f)
    sc = _assemble(mesh_list, [0] * len(mesh_list), [MAT_REFLECT], [1.0])
    eye = np.array([0, 8, 38], np.float32)
    look = np.array([0, 0, 0], np.float32)
    lights = np.array([[15, 25, 15]], np.float32)
    return _finish("frame", seed, sc, Wd, Wd, eye, look, 45.0, lights, B, F, n, SHADOW | REFLECT)


def _batch_frame(job):
    fseed, tr, tt, path = job
    import os
    if path and os.path.exists(path):
        return _load(path)
    wl = make_frame(fseed, tr, tt)
    if path:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        _save(wl, path)
    return wl


def make_batch(seed=0, frames=64, cache_dir=None, jobs=1):
    """Frame list of the batched workload: rays per frame log-uniform in
    [4096, 1M], triangles per frame log-uniform in [1000, 200000].  With
    `cache_dir` (or CRSH_WORKLOAD_CACHE) every frame is kept there as an
    .npz and reloaded by later calls; `jobs` > 1 builds the frames in a
    forked process pool (call it before the process uses the GPU)."""
    import os
    cache_dir = cache_dir or os.environ.get("CRSH_WORKLOAD_CACHE")
    rng = np.random.default_rng(seed)
    work = []
    for i in range(frames):
        tr = float(np.exp(rng.uniform(np.log(4096), np.log(1 << 20))))
        tt = float(np.exp(rng.uniform(np.log(1000), np.log(200000))))
        fseed = seed * 1000 + i + 1
        path = os.path.join(cache_dir, f"frame_seed{fseed}_{tr:.6g}_{tt:.6g}.npz") if cache_dir else None
        work.append((fseed, tr, tt, path))
    if jobs <= 1 or frames <= 1:
        return [_batch_frame(w) for w in work]
    import multiprocessing as mp
    # largest frames first, so that the pool's tail is short
    order = sorted(range(frames), key=lambda k: -work[k][1] * work[k][2])
    with mp.get_context("fork").Pool(min(jobs, frames)) as pool:
        built = pool.map(_batch_frame, [work[k] for k in order], chunksize=1)
    out = [None] * frames
    for k, wl in zip(order, built):
        out[k] = wl
    return out


def _finish(name, seed, sc, W, H, eye, look, vfov, lights, B, F, n, types):
    g = cast_primary(sc.tris, sc.tri_mat(), W, H, eye, look, vfov)
    lo, inv = _box(sc.tris)
    return Workload(name=name, seed=seed, scene=sc, W=W, H=H, eye=eye, look=look,
                    vfov=vfov, lights=lights, gbuf=g, B=B, F=F, n=n, ray_types=types,
                    lo=lo, inv_ext=inv)


def unsorted_variant(wl, levels=None):
    """The comparison configuration of the same inputs: the ray-space
    hierarchy without ray sorting and without whole-mesh culling (Sec. 2) --
    keys of ray type and light only, every triangle in one mesh whose sphere
    always passes -- with the same hierarchy shape (B, F and the level count,
    as the paper compares both hierarchies at one depth, Sec. 4.1), or
    `levels` levels when given."""
    sc = wl.scene
    one = Scene(tris=sc.tris, mesh_first=np.zeros(1, np.uint32), mesh_count=np.array([sc.m], np.uint32),
                mesh_sphere=np.array([[0.0, 0.0, 0.0, 1e30]], np.float32), mesh_mat=np.zeros(1, np.int32),
                mat_flags=sc.mat_flags, mat_ior=sc.mat_ior, verts=sc.verts, faces=sc.faces)
    return replace(wl, name=wl.name + "_unsorted", scene=one, ray_types=wl.ray_types | KEY_TYPE_ONLY,
                   n=wl.n if levels is None else levels)


MAKERS = {"shadow_128": make_shadow_128, "refl_1024": make_refl_1024, "mixed_1080p": make_mixed_1080p, "adjoint_512": make_adjoint_512}


def _save(wl, path):
    """Every array of a workload into one .npz (no pickled objects)."""
    sc = wl.scene
    a = {f"scene_{k}": getattr(sc, k) for k in ("tris", "mesh_first", "mesh_count", "mesh_sphere", "mesh_mat",
                                                 "mat_flags", "mat_ior", "verts", "faces")
         if getattr(sc, k) is not None}
    a.update({f"gbuf_{k}": v for k, v in wl.gbuf.items()})
    for k in ("eye", "look", "lights", "lo", "inv_ext"):
        a[k] = getattr(wl, k)
    a["ints"] = np.array([wl.seed, wl.W, wl.H, wl.B, wl.F, wl.n, wl.ray_types], np.int64)
    a["floats"] = np.array([wl.vfov, wl.eps_off, wl.eps_shadow, wl.t_min], np.float64)
    a["name"] = np.array(wl.name)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **a)
    import os
    os.replace(tmp, path)


def _load(path):
    with np.load(path, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    sc = Scene(**{k[6:]: v for k, v in g.items() if k.startswith("scene_")})
    seed, W, H, B, F, n, types = (int(x) for x in g["ints"])
    vfov, eps_off, eps_shadow, t_min = (float(x) for x in g["floats"])
    return Workload(name=str(g["name"]), seed=seed, scene=sc, W=W, H=H, eye=g["eye"], look=g["look"], vfov=vfov,
                    lights=g["lights"], gbuf={k[5:]: v for k, v in g.items() if k.startswith("gbuf_")}, B=B, F=F,
                    n=n, ray_types=types, eps_off=eps_off, eps_shadow=eps_shadow, t_min=t_min, lo=g["lo"],
                    inv_ext=g["inv_ext"])


def make_workload(name, seed=0, cache_dir=None, **kw):
    """Build a named workload.  With `cache_dir` (or the CRSH_WORKLOAD_CACHE
    environment variable) the default-sized workload is kept there as an
    .npz and reloaded by later calls with the same name and seed."""
    import os
    cache_dir = cache_dir or os.environ.get("CRSH_WORKLOAD_CACHE")
    if not cache_dir or kw:
        return MAKERS[name](seed=seed, **kw)
    path = os.path.join(cache_dir, f"{name}_seed{seed}.npz")
    if os.path.exists(path):
        return _load(path)
    wl = MAKERS[name](seed=seed)
    os.makedirs(cache_dir, exist_ok=True)
    _save(wl, path)
    return wl
