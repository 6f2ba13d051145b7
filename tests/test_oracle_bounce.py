"""Pins of the oracle's next-bounce generation (Sec. 3.3.8): children come
only from reflection / refraction parents with a closest hit, in parent
order; their rays obey the same laws as the first generation's, at the hit
point and with the hit triangle's normal and material."""
import numpy as np

from conftest import oracle_run, workload
from oracle import oracle as O


def _gen2(name, **kw):
    wl = workload(name, **kw)
    o = oracle_run(name, **kw)
    h = o["hash"]
    return wl, h, o["hits"], O.bounce(h["rays"], h["keys"], o["hits"], wl)


def _vec(r, pre, i):
    return np.array([r[pre + "x"][i], r[pre + "y"][i], r[pre + "z"][i]], np.float64)


def test_children_come_from_bounce_parents_with_hits():
    wl, h, hits, b = _gen2("mixed_1080p", W=96, H=54, n_meshes=32)
    parents = np.nonzero((hits[0] >= 0) & ((h["keys"] >> np.uint32(30)) != 0))[0]
    assert b["n"] > 0 and len(parents) > 0
    # children keep their parent's pixel, in parent order (pixels ascend)
    pix = b["rays"]["pix"]
    assert np.all(np.diff(pix.astype(np.int64)) >= 0)
    assert set(np.unique(pix)) <= set(h["rays"]["pix"][parents])
    # every parent yields at most n_lights + 2 children
    L = len(wl.lights)
    assert b["n"] <= len(parents) * (L + 2)
    # shadow-only frames have no bounce parents
    wl_s = workload("shadow_128", W=32, H=32)
    o_s = O.run_pipeline(wl_s)
    assert O.bounce(o_s["hash"]["rays"], o_s["hash"]["keys"], o_s["hits"], wl_s)["n"] == 0


def test_children_obey_the_ray_laws_at_the_hit_point():
    wl, h, hits, b = _gen2("mixed_1080p", W=96, H=54, n_meshes=32)
    tri = wl.scene.tris.astype(np.float64)
    tmat = wl.scene.tri_mat()
    parents = [i for i in range(h["n"]) if hits[0][i] >= 0 and (h["keys"][i] >> 30) != 0]
    # one bounce parent per pixel here (a material reflects or refracts), so a
    # child's pixel names its parent
    assert len({int(h["rays"]["pix"][i]) for i in parents}) == len(parents)
    rr = b["rays"]
    j = 0
    checked = {"shadow": 0, "reflect": 0, "refract": 0}
    for i in parents:
        O_ = _vec(h["rays"], "o", i)
        D = _vec(h["rays"], "d", i)
        P = O_ + hits[1][i] * D
        v0, v1, v2 = tri[hits[0][i]]
        n = np.cross(v1 - v0, v2 - v0)
        n /= np.linalg.norm(n)
        if n @ D > 0:
            n = -n
        # P on the triangle's plane
        assert abs((P - v0) @ n) <= 1e-4 * (1 + np.abs(P).max())
        flags = wl.scene.mat_flags[tmat[hits[0][i]]]
        while j < b["n"] and rr["pix"][j] == h["rays"]["pix"][i]:
            key = int(b["keys"][j])
            d = _vec(rr, "d", j)
            o = _vec(rr, "o", j)
            assert abs(np.linalg.norm(d) - 1) < 1e-5
            if key >> 30 == 0:          # shadow ray from light (key bits 29-28) to P
                lt = wl.lights[(key >> 28) & 3].astype(np.float64)
                assert np.allclose(o, lt)
                assert np.allclose(o + (rr["tmax"][j] + wl.eps_shadow) * d, P, atol=1e-3)
                checked["shadow"] += 1
            elif key >> 30 == 1:        # mirror reflection about n, off the surface
                assert flags & 1
                assert np.allclose(d, D - 2 * (D @ n) * n, atol=1e-4)
                assert np.allclose(o, P + wl.eps_off * n, atol=1e-4)
                checked["reflect"] += 1
            else:                       # Snell: sin ratio 1/ior, across the surface
                assert flags & 2
                ior = float(wl.scene.mat_ior[tmat[hits[0][i]]])
                si = np.linalg.norm(np.cross(D, n))
                st = np.linalg.norm(np.cross(d, n))
                assert abs(st - si / ior) < 1e-4
                assert d @ n < 0 and np.allclose(o, P - wl.eps_off * n, atol=1e-4)
                checked["refract"] += 1
            j += 1
    assert j == b["n"]
    assert checked["shadow"] > 100 and checked["reflect"] > 100 and checked["refract"] > 10


def test_first_generation_of_the_chain_is_the_plain_frame():
    wl = workload("refl_1024", W=48, H=48)
    g = O.run_generations(wl, 2)
    o = O.run_pipeline(wl)
    assert np.array_equal(g[0]["hash"]["keys"], o["hash"]["keys"])
    assert np.array_equal(g[0]["hits"][0], o["hits"][0])
    assert g[1]["hash"]["n"] > 0
    # second generation: every ray's pixel is a pixel of a hit reflection ray
    h = o["hash"]
    par = set(h["rays"]["pix"][(o["hits"][0] >= 0) & ((h["keys"] >> np.uint32(30)) == 1)])
    assert set(np.unique(g[1]["hash"]["rays"]["pix"])) <= par
