"""Pins of the oracle's ray generation, trimming and hashing (Sec. 3.3.2).

Each check is tied to geometry or to a closed form, not to the oracle's own
formulas: reflection obeys the law of reflection, refraction obeys Snell's
law, trimming keeps exactly the real rays in order, and the octahedral key of
a direction decodes (with an independent float64 inverse map) to a direction
within one cell of it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import Workload, Scene, SHADOW, REFLECT, REFRACT
from conftest import workload


def tiny_workload(P, N, mat, lights, eye, flags, ior, types, W=None, H=1):
    P = np.asarray(P, np.float32).reshape(-1, 3)
    N = np.asarray(N, np.float32).reshape(-1, 3)
    W = W or len(P)
    sc = Scene(tris=np.zeros((1, 3, 3), np.float32), mesh_first=np.zeros(1, np.uint32),
               mesh_count=np.ones(1, np.uint32), mesh_sphere=np.zeros((1, 4), np.float32),
               mesh_mat=np.zeros(1, np.int32), mat_flags=np.asarray(flags, np.uint32),
               mat_ior=np.asarray(ior, np.float32))
    g = {"px": P[:, 0].copy(), "py": P[:, 1].copy(), "pz": P[:, 2].copy(),
         "nx": N[:, 0].copy(), "ny": N[:, 1].copy(), "nz": N[:, 2].copy(),
         "mat": np.asarray(mat, np.int32)}
    return Workload(name="tiny", seed=0, scene=sc, W=W, H=H, eye=np.asarray(eye, np.float32),
                    look=np.zeros(3, np.float32), vfov=45.0,
                    lights=np.asarray(lights, np.float32).reshape(-1, 3), gbuf=g,
                    B=4, F=2, n=3, ray_types=types,
                    lo=np.array([-8, -8, -8], np.float32),
                    inv_ext=np.full(3, np.float32(1.0) / np.float32(16.0), np.float32))


def test_shadow_ray_axis_aligned_closed_form():
    wl = tiny_workload([[1, -2, 3]], [[0, 1, 0]], [0], [[1, 1, 3]], [0, 0, 10], [0], [1.0], SHADOW)
    h = O.hash_rays(wl)
    r = h["rays"]
    assert h["n"] == 1
    # origin moved to the light, direction exactly -y, extent |P-L| - eps
    assert (r["ox"][0], r["oy"][0], r["oz"][0]) == (1.0, 1.0, 3.0)
    assert (r["dx"][0], r["dy"][0], r["dz"][0]) == (0.0, -1.0, 0.0)
    assert r["tmax"][0] == np.float32(3.0) - np.float32(1e-3)


def test_shadow_ray_too_close_to_light_is_dropped():
    wl = tiny_workload([[0, 0, 0]], [[0, 1, 0]], [0], [[0, 0.0005, 0]], [0, 0, 10], [0], [1.0], SHADOW)
    assert O.hash_rays(wl)["n"] == 0


def _reflect_case(rng, n=200):
    P = rng.uniform(-3, 3, size=(n, 3))
    N = rng.normal(size=(n, 3))
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    eye = np.array([0.5, 1.0, 12.0])
    v = P - eye
    # the primary-hit buffer always stores a normal facing the camera
    flip = (v * N).sum(1) > 0
    N[flip] = -N[flip]
    return P.astype(np.float32), N.astype(np.float32), eye.astype(np.float32)


def test_reflection_obeys_law_of_reflection(rng):
    P, N, eye = _reflect_case(rng)
    wl = tiny_workload(P, N, [0] * len(P), np.zeros((0, 3)), eye, [1], [1.0], REFLECT)
    h = O.hash_rays(wl)
    assert h["n"] == len(P)
    r = h["rays"]
    D = np.stack([r["dx"], r["dy"], r["dz"]], 1).astype(np.float64)
    v = P.astype(np.float64) - eye.astype(np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    n = N.astype(np.float64)
    assert np.allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-6)
    # equal angles on both sides of the normal
    assert np.allclose((D * n).sum(1), -(v * n).sum(1), atol=2e-6)
    # reflected ray lies in the plane of incidence
    assert np.allclose(np.einsum("ij,ij->i", np.cross(v, n), D), 0.0, atol=2e-6)
    # origin offset along the normal, unbounded extent
    O64 = np.stack([r["ox"], r["oy"], r["oz"]], 1).astype(np.float64)
    assert np.allclose(O64, P + 1e-3 * n, atol=1e-6)
    assert np.all(r["tmax"] == np.finfo(np.float32).max)


def test_refraction_obeys_snell(rng):
    P, N, eye = _reflect_case(rng)
    wl = tiny_workload(P, N, [0] * len(P), np.zeros((0, 3)), eye, [2], [1.5], REFRACT)
    h = O.hash_rays(wl)
    assert h["n"] == len(P)   # entering a denser medium: never total internal reflection
    r = h["rays"]
    T = np.stack([r["dx"], r["dy"], r["dz"]], 1).astype(np.float64)
    v = P.astype(np.float64) - eye.astype(np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    n = N.astype(np.float64)
    sin_i = np.linalg.norm(np.cross(v, n), axis=1)
    sin_t = np.linalg.norm(np.cross(T, n), axis=1)
    assert np.allclose(sin_t, sin_i / 1.5, atol=3e-6)
    assert np.all((T * n).sum(1) < 0)                 # transmitted into the surface
    assert np.allclose(np.einsum("ij,ij->i", np.cross(v, n), T), 0.0, atol=3e-6)
    O64 = np.stack([r["ox"], r["oy"], r["oz"]], 1).astype(np.float64)
    assert np.allclose(O64, P - 1e-3 * n, atol=1e-6)


def test_refraction_total_internal_reflection():
    # leaving a medium (relative index 2): beyond the critical angle (30 deg) no ray
    eye = np.array([0, 0, 10], np.float32)
    P = []
    N = []
    for ang in (10.0, 25.0, 35.0, 60.0):
        a = np.radians(ang)
        v = np.array([np.sin(a), 0, -np.cos(a)])
        P.append(eye + 10 * v)
        N.append([0, 0, 1])
    wl = tiny_workload(P, N, [0] * 4, np.zeros((0, 3)), eye, [2], [0.5], REFRACT)
    h = O.hash_rays(wl)
    assert h["n"] == 2
    assert list(h["rays"]["pix"]) == [0, 1]


def test_trimming_keeps_real_rays_in_slot_order():
    # 6 pixels: sky, diffuse, reflective, refractive, both, sky; 2 lights
    P = [[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0], [4, 0, 0], [5, 0, 0]]
    N = [[0, 0, 1]] * 6
    mat = [-1, 0, 1, 2, 3, -1]
    flags = [0, 1, 2, 3]
    wl = tiny_workload(P, N, mat, [[0, 5, 5], [5, 5, 5]], [0, 0, 10], flags, [1, 1, 1.5, 1.5],
                       SHADOW | REFLECT | REFRACT)
    h = O.hash_rays(wl)
    # pixel 1: 2 shadow; 2: 2 shadow + refl; 3: 2 shadow + refr; 4: 2 shadow + refl + refr
    assert list(h["rays"]["pix"]) == [1, 1, 2, 2, 2, 3, 3, 3, 4, 4, 4, 4]
    assert list(h["ids"]) == list(range(12))
    typ = h["keys"] >> 30
    assert list(typ) == [0, 0, 0, 0, 1, 0, 0, 2, 0, 0, 1, 2]
    light = (h["keys"] >> 28) & 3
    assert list(light[typ == 0]) == [0, 1] * 4
    # a ray type that is switched off is never made
    wl.ray_types = SHADOW
    assert O.hash_rays(wl)["n"] == 8


@pytest.mark.parametrize("k", [6, 14])
def test_octahedral_code_axes(k):
    half, top = 1 << (k - 1), (1 << k) - 1
    assert O.oct_code([1, 0, 0], k) == (top, half)
    assert O.oct_code([-1, 0, 0], k) == (0, half)
    assert O.oct_code([0, 1, 0], k) == (half, top)
    assert O.oct_code([0, -1, 0], k) == (half, 0)
    assert O.oct_code([0, 0, 1], k) == (half, half)
    assert O.oct_code([0, 0, -1], k) == (top, top)


def _oct_decode64(u, v, k):
    """Inverse octahedral map (float64) of the centre of cell (u, v)."""
    px = (u + 0.5) / 2 ** (k - 1) - 1.0
    py = (v + 0.5) / 2 ** (k - 1) - 1.0
    z = 1.0 - abs(px) - abs(py)
    if z < 0:
        px, py = (1.0 - abs(py)) * np.sign(px), (1.0 - abs(px)) * np.sign(py)
    d = np.array([px, py, z])
    return d / np.linalg.norm(d)


@pytest.mark.parametrize("k", [6, 14])
def test_octahedral_code_decodes_near_direction(rng, k):
    worst = 0.0
    for _ in range(400):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        u, v = O.oct_code(d.astype(np.float32), k)
        e = _oct_decode64(u, v, k)
        worst = max(worst, np.arccos(np.clip(d @ e, -1, 1)))
    # an octahedral cell of side 2/2^k spans at most ~pi * 2^-k radians
    assert worst < np.pi * 2.0 ** -k * 1.5


def _deinterleave2(m):
    u = v = 0
    for i in range(16):
        u |= ((m >> (2 * i)) & 1) << i
        v |= ((m >> (2 * i + 1)) & 1) << i
    return u, v


def test_shadow_key_layout(rng):
    for light in range(4):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        key = O.shadow_key(light, d.astype(np.float32))
        assert key >> 30 == 0
        assert (key >> 28) & 3 == light
        assert _deinterleave2(key & ((1 << 28) - 1)) == O.oct_code(d.astype(np.float32), 14)


def test_bounce_key_layout_and_corner_cells():
    wl = tiny_workload([[0, 0, 0]], [[0, 0, 1]], [0], np.zeros((0, 3)), [0, 0, 10], [1], [1.0], REFLECT)
    lo = wl.lo.astype(np.float64)
    hi = lo + 16.0
    d = np.array([0, 0, 1], np.float32)
    for typ in (1, 2):
        k_lo = O.bounce_key(typ, lo.astype(np.float32), d, wl)
        k_hi = O.bounce_key(typ, (hi - 1e-3).astype(np.float32), d, wl)
        k_out = O.bounce_key(typ, (hi + 5).astype(np.float32), d, wl)
        assert k_lo >> 30 == typ
        assert (k_lo >> 12) & ((1 << 18) - 1) == 0                  # cell (0,0,0)
        assert (k_hi >> 12) & ((1 << 18) - 1) == (1 << 18) - 1      # cell (63,63,63)
        assert k_out == k_hi                                          # clamped
        assert k_lo & 0xFFF == _interleave2(*O.oct_code(d, 6))
    # cell (1, 0, 0) -> bit 0; (0, 1, 0) -> bit 1; (0, 0, 1) -> bit 2 of the cell field
    step = 16.0 / 64
    for axis, bit in ((0, 0), (1, 1), (2, 2)):
        o = lo + 0.5 * step
        o[axis] += step
        key = O.bounce_key(1, o.astype(np.float32), d, wl)
        assert (key >> 12) & ((1 << 18) - 1) == 1 << bit


def _interleave2(u, v):
    m = 0
    for i in range(16):
        m |= ((u >> i) & 1) << (2 * i) | ((v >> i) & 1) << (2 * i + 1)
    return m


@pytest.mark.parametrize("name", ["shadow_128", "refl_96", "mixed_128x72"])
def test_workload_ray_counts(name):
    from conftest import small, oracle_run
    base, kw = small(name)
    wl = workload(base, **kw)
    h = oracle_run(base, **kw)["hash"]
    hit = wl.gbuf["mat"] >= 0
    if name == "shadow_128":
        assert h["n"] == hit.sum()                     # one shadow ray per hit pixel
    if name == "refl_96":
        assert h["n"] == 2 * hit.sum()                 # shadow + reflection everywhere
    if name == "mixed_128x72":
        assert h["n"] == 3 * hit.sum()                 # 2 shadow + reflection or refraction
    assert np.all(np.diff(h["rays"]["pix"].astype(np.int64)) >= 0)


def test_unsorted_comparison_keys_keep_type_and_light():
    """Comparison mode (the hierarchy without ray sorting, Sec. 2): the same
    rays, keys reduced to the type and light bits, so the sort only groups
    the rays per type and light and keeps their generation order."""
    from workloads import unsorted_variant
    wl = workload("mixed_1080p", W=48, H=32, n_meshes=24)
    a = O.hash_rays(wl)
    b = O.hash_rays(unsorted_variant(wl))
    assert b["n"] == a["n"]
    for k in O.RAY_FIELDS:
        assert np.array_equal(a["rays"][k], b["rays"][k])
    assert np.array_equal(b["keys"], a["keys"] & np.uint32(0xF0000000))
    ks, ids = O.sort_rays(b["keys"], b["ids"])
    assert np.array_equal(ids, np.argsort(a["keys"] >> np.uint32(28), kind="stable").astype(np.uint32))
    assert len(np.unique(b["keys"] >> np.uint32(28))) >= 3     # two shadow lights and a bounce type


def test_spherical_codes_follow_float64_spherical_coordinates(rng):
    """Spherical direction codes (theta = acos dz, phi = atan2(dy, dx), each
    in 2^k bins): within one bin of the float64 bins everywhere (the
    polynomial acos / atan err by < 7e-5 rad, 0.37 of a 14-bit theta bin),
    equal away from bin edges, and the poles and axes land where they must."""
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = d.astype(np.float32)
    for k in (6, 14):
        n = 1 << k
        for x in d:
            u, v = O.sph_code(x, k)
            x64 = x.astype(np.float64)
            th = np.arccos(np.clip(x64[2], -1, 1)) / np.pi * n
            ph = (np.arctan2(x64[1], x64[0]) + np.pi) / (2 * np.pi) * n
            eu, ev = min(int(np.floor(th)), n - 1), min(int(np.floor(ph)), n - 1)
            assert abs(u - eu) <= 1 and abs(v - ev) <= 1, (x, k, u, eu, v, ev)
            # away from a bin edge by more than the approximation error plus
            # the binary32 evaluation error (a few ulps of pi, and of the bin
            # index), both in bins, the bin is the exact one
            mt = (6.7e-5 + 4e-6) * n / np.pi + 8 * n * 2.0 ** -24
            mp = (1e-5 + 4e-6) * n / (2 * np.pi) + 8 * n * 2.0 ** -24
            if mt < th % 1 < 1 - mt:
                assert u == eu, (x, k, u, th)
            if mp < ph % 1 < 1 - mp:
                assert v == ev, (x, k, v, ph)
    assert O.sph_code([0, 0, 1], 14)[0] == 0                      # north pole
    assert O.sph_code([0, 0, -1], 14)[0] == (1 << 14) - 1          # south pole, clamped
    assert O.sph_code([1, 0, 0], 6) == (31, 32)                   # theta pi/2 (just below), phi 0
    assert O.sph_code([-1, 0, 0], 6)[1] == 63                      # phi = pi, clamped
    assert O.sph_code([0, -1, 0], 6)[1] == 16                      # phi = -pi/2


def test_spherical_keys_replace_only_the_direction_bits():
    wl = workload("mixed_1080p", W=48, H=32, n_meshes=24)
    import dataclasses
    from workloads import KEY_SPHERICAL
    a = O.hash_rays(wl)
    b = O.hash_rays(dataclasses.replace(wl, ray_types=wl.ray_types | KEY_SPHERICAL))
    assert b["n"] == a["n"]
    for k in O.RAY_FIELDS:
        assert np.array_equal(a["rays"][k], b["rays"][k])
    shadow = (a["keys"] >> np.uint32(30)) == 0
    # type, light and origin cell bits unchanged
    assert np.array_equal(a["keys"][shadow] >> np.uint32(28), b["keys"][shadow] >> np.uint32(28))
    assert np.array_equal(a["keys"][~shadow] >> np.uint32(12), b["keys"][~shadow] >> np.uint32(12))
    assert not np.array_equal(a["keys"], b["keys"])
    for i in np.nonzero(shadow)[0][:200]:
        d = np.array([b["rays"]["dx"][i], b["rays"]["dy"][i], b["rays"]["dz"][i]])
        u, v = O.sph_code(d, 14)
        m = 0
        for j in range(14):
            m |= ((u >> j) & 1) << (2 * j) | ((v >> j) & 1) << (2 * j + 1)
        assert int(b["keys"][i]) & ((1 << 28) - 1) == m
