"""GPU adjoint of the closest hit (Sec. 3.3.8) behind torch.autograd.

Forward: caller-given rays through the whole path equal the oracle's closest
hits.  Backward: checked against float64 central finite differences (h=1e-4)
of the oracle's fixed-triangle Moller-Trumbore solve, on rays whose
barycentric margin exceeds 1e-3, for a sample of vertex coordinates and ray
parameters; against the translation-invariance identity (moving every vertex
and every ray origin together changes no t, u, v, so the gradients sum to
zero); and against a closed form.
"""
import numpy as np
import pytest

from conftest import workload, oracle_run
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _scene(wl, **kw):
    from paper_2312_06538_amd.autograd import RayScene
    sc = wl.scene
    return RayScene(sc.faces, sc.mesh_first, sc.mesh_count, wl.lo, wl.inv_ext, B=wl.B, F=wl.F,
                    levels=wl.n, t_min=wl.t_min, ray_type=1, **kw)


@pytest.fixture(scope="module")
def adjoint_case():
    import torch
    from paper_2312_06538_amd.autograd import ClosestHit
    print("[adjoint] building workload", flush=True)
    wl = workload("adjoint_512")
    o_run = oracle_run("adjoint_512")
    h = o_run["hash"]
    r = h["rays"]
    o = np.stack([r["ox"], r["oy"], r["oz"]], 1)
    d = np.stack([r["dx"], r["dy"], r["dz"]], 1)
    verts = torch.tensor(wl.scene.verts, device="cuda", requires_grad=True)
    ot = torch.tensor(o, device="cuda", requires_grad=True)
    dt = torch.tensor(d, device="cuda", requires_grad=True)
    scene = _scene(wl, pair_capacity=1 << 20)
    tri, t, u, v = ClosestHit.apply(verts, ot, dt, scene)
    rng = np.random.default_rng(0)
    n = len(o)
    w, a, b = (rng.normal(size=n).astype(np.float32) for _ in range(3))
    tri_np, u_np, v_np = tri.cpu().numpy(), u.detach().cpu().numpy(), v.detach().cpu().numpy()
    margin = np.minimum(np.minimum(u_np, v_np), 1 - u_np - v_np)
    keep = (tri_np >= 0) & (margin > 1e-3)
    w, a, b = (np.where(keep, x, 0).astype(np.float32) for x in (w, a, b))
    W, A, Bw = (torch.tensor(x, device="cuda") for x in (w, a, b))
    loss = (W * t).sum() + (A * u).sum() + (Bw * v).sum()
    loss.backward()
    return dict(wl=wl, oracle=o_run, o=o, d=d, tri=tri_np, t=t.detach().cpu().numpy(), u=u_np, v=v_np,
                w=w, a=a, b=b, keep=keep, g_verts=verts.grad.cpu().numpy(), g_o=ot.grad.cpu().numpy(),
                g_d=dt.grad.cpu().numpy())


def test_forward_matches_oracle(adjoint_case):
    c = adjoint_case
    o = c["oracle"]["hits"]
    assert np.array_equal(c["tri"], o[0])
    for x, y in zip((c["t"], c["u"], c["v"]), o[1:]):
        assert np.allclose(x, y, rtol=1e-5, atol=0)
    # enough hit rays away from triangle edges for the samples below (2,048
    # vertex coordinates, 342 rays x 6 parameters)
    assert c["keep"].sum() > 2000


def _loss_terms(c, ray, o, d, tri9):
    ok, tuv = O.mt64(o, d, tri9)
    assert ok
    return c["w"][ray] * tuv[0] + c["a"][ray] * tuv[1] + c["b"][ray] * tuv[2]


U32 = 2.0 ** -24


def _f32_scale(o, tri9):
    """First-order error scale of a float32 Moller-Trumbore solve and its
    adjoint on float32 inputs: the matrix [D | -e1 | -e2] carries relative
    error ~u * max|v| / min|e| from the float32 edge subtractions, amplified
    by its condition number."""
    v = np.asarray(tri9, np.float64).reshape(3, 3)
    e = min(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[0]))
    return max(1.0, np.abs(v).max() / e, np.abs(o).max() / e)


def _check(g, g_fd, bound):
    """Global: relative 2-norm error <= 1e-3.  Per component: within 1e-3 of
    max(|g_fd|, 1e-3 max|g_fd|), plus the float32 error bound of the terms
    that make up the component (8 u cond * scale * |term|, summed)."""
    g, g_fd, bound = np.asarray(g), np.asarray(g_fd), np.asarray(bound)
    rel = np.linalg.norm(g - g_fd) / np.linalg.norm(g_fd)
    assert rel <= 1e-3, rel
    base = 1e-3 * np.maximum(np.abs(g_fd), 1e-3 * np.abs(g_fd).max())
    tol = base + bound
    err = np.abs(g - g_fd)
    # how close the components come to their tolerances, and to the part of
    # it that is not the float32 error bound
    worst = int(np.argmax(err / tol))
    print(f"[adjoint] {len(g)} components: relative 2-norm error {rel:.2e}; worst component "
          f"error / tolerance {err[worst] / tol[worst]:.3f} (error / 1e-3-relative part "
          f"{err[worst] / base[worst]:.3f}); components over the 1e-3-relative part alone: "
          f"{int((err > base).sum())}", flush=True)
    bad = err > tol
    assert not bad.any(), (np.nonzero(bad)[0][:10], g[bad][:5], g_fd[bad][:5], bound[bad][:5])


def test_vertex_gradients_match_finite_differences(adjoint_case):
    c = adjoint_case
    sc = c["wl"].scene
    faces = sc.faces.astype(np.int64)
    verts = sc.verts.astype(np.float64)
    hit_rays = np.nonzero(c["keep"])[0]
    by_vertex = {}
    for ray in hit_rays:
        for k in range(3):
            by_vertex.setdefault(int(faces[c["tri"][ray], k]), []).append(ray)
    rng = np.random.default_rng(1)
    cand = np.array(sorted(by_vertex))
    pick = rng.choice(len(cand) * 3, size=min(2048, len(cand) * 3), replace=False)
    h = 1e-4
    g, g_fd, bound = [], [], []
    for p in pick:
        vj, comp = int(cand[p // 3]), int(p % 3)
        acc = 0.0
        err = 0.0
        for ray in by_vertex[vj]:
            f = faces[c["tri"][ray]]
            tri9 = verts[f].reshape(-1).copy()
            o = c["o"][ray].astype(np.float64)
            d = c["d"][ray].astype(np.float64)
            for sgn in (1, -1):
                t9 = tri9.copy()
                for k in range(3):
                    if f[k] == vj:
                        t9[3 * k + comp] += sgn * h
                acc += sgn * _loss_terms(c, ray, o, d, t9)
            *dv, _, _, cond = O.adjoint64(o, d, tri9, [c["w"][ray], c["a"][ray], c["b"][ray]])
            term = sum(abs(dv[k][comp]) for k in range(3) if f[k] == vj)
            err += 8 * U32 * cond * _f32_scale(o, tri9) * term
        g_fd.append(acc / (2 * h))
        g.append(c["g_verts"][vj, comp])
        bound.append(err)
    _check(g, g_fd, bound)


def test_ray_gradients_match_finite_differences(adjoint_case):
    c = adjoint_case
    sc = c["wl"].scene
    faces = sc.faces.astype(np.int64)
    verts = sc.verts.astype(np.float64)
    rays = np.random.default_rng(2).choice(np.nonzero(c["keep"])[0], 342, replace=False)
    h = 1e-4
    g, g_fd, bound = [], [], []
    for ray in rays:
        tri9 = verts[faces[c["tri"][ray]]].reshape(-1)
        o = c["o"][ray].astype(np.float64)
        d = c["d"][ray].astype(np.float64)
        _, _, _, do, dd, cond = O.adjoint64(o, d, tri9, [c["w"][ray], c["a"][ray], c["b"][ray]])
        scale = 8 * U32 * cond * _f32_scale(o, tri9)
        for which, vec in (("o", o), ("d", d)):
            for comp in range(3):
                p, m = vec.copy(), vec.copy()
                p[comp] += h
                m[comp] -= h
                if which == "o":
                    lp, lm = _loss_terms(c, ray, p, d, tri9), _loss_terms(c, ray, m, d, tri9)
                else:
                    lp, lm = _loss_terms(c, ray, o, p, tri9), _loss_terms(c, ray, o, m, tri9)
                g_fd.append((lp - lm) / (2 * h))
                g.append(c["g_o" if which == "o" else "g_d"][ray, comp])
                bound.append(scale * abs((do if which == "o" else dd)[comp]))
    _check(g, g_fd, bound)


def test_gradients_are_translation_invariant(adjoint_case):
    c = adjoint_case
    s = c["g_verts"].astype(np.float64).sum(0) + c["g_o"].astype(np.float64).sum(0)
    scale = np.abs(c["g_verts"]).sum() + np.abs(c["g_o"]).sum()
    assert np.all(np.abs(s) <= 1e-4 * scale), (s, scale)
    # misses and masked rays get no gradient
    assert np.all(c["g_o"][c["tri"] < 0] == 0) and np.all(c["g_d"][c["tri"] < 0] == 0)


def test_closed_form_axis_aligned_triangle():
    import torch
    from paper_2312_06538_amd.autograd import RayScene, ClosestHit
    verts = torch.tensor([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=torch.float32, device="cuda",
                         requires_grad=True)
    o = torch.tensor([[0.25, 0.5, 1.0]], device="cuda", requires_grad=True)
    d = torch.tensor([[0.0, 0.0, -1.0]], device="cuda", requires_grad=True)
    scene = RayScene(np.array([[0, 1, 2]]), [0], [1], [-2, -2, -2], [0.25, 0.25, 0.25], B=1, F=2, levels=1)
    tri, t, u, v = ClosestHit.apply(verts, o, d, scene)
    assert tri.item() == 0 and (t.item(), u.item(), v.item()) == (1.0, 0.25, 0.5)
    t.sum().backward(retain_graph=True)
    # t = o_z / (-d_z): dt/do = (0,0,1), dt/dd = (0,0,1); raising the plane lowers t
    assert np.allclose(o.grad.cpu().numpy(), [[0, 0, 1]])
    assert np.allclose(d.grad.cpu().numpy(), [[0, 0, 1]])
    assert np.allclose(verts.grad.cpu().numpy()[:, 2], [-0.25, -0.25, -0.5])
    for x in (verts, o, d):
        x.grad = None
    u.sum().backward()
    # u follows the origin's x; stretching v1 along x shrinks it
    assert np.allclose(o.grad.cpu().numpy(), [[1, 0, 0]])
    assert np.allclose(verts.grad.cpu().numpy()[1], [-0.25, 0, 0])


def test_forward_after_vertices_move():
    """A second forward pass after the vertices moved: the mesh spheres are
    recomputed from the moved triangles, so the closest hits equal the
    oracle's for the moved scene (and naive ray tracing on a sample).  Mesh
    0 is shifted by three of its radii, so hits land on triangles that lie
    wholly outside its original sphere."""
    import dataclasses
    import torch
    from paper_2312_06538_amd.autograd import ClosestHit
    from workloads.scenes import Scene, enclosing_sphere
    wl = workload("adjoint_512")
    sc = wl.scene
    h = oracle_run("adjoint_512")["hash"]
    r = h["rays"]
    o = torch.tensor(np.stack([r["ox"], r["oy"], r["oz"]], 1), device="cuda")
    d = torch.tensor(np.stack([r["dx"], r["dy"], r["dz"]], 1), device="cuda")
    scene = _scene(wl, pair_capacity=1 << 20)
    ClosestHit.apply(torch.tensor(sc.verts, device="cuda"), o, d, scene)      # at the original vertices
    # move mesh 0 towards the camera by 3 radii
    c0, r0 = sc.mesh_sphere[0, :3].astype(np.float64), float(sc.mesh_sphere[0, 3])
    shift = (wl.eye.astype(np.float64) - c0)
    shift = (3.0 * r0 * shift / np.linalg.norm(shift)).astype(np.float32)
    f0, n0 = int(sc.mesh_first[0]), int(sc.mesh_count[0])
    vids = np.unique(sc.faces[f0:f0 + n0])
    verts = sc.verts.copy()
    verts[vids] += shift
    tri, t, u, v = ClosestHit.apply(torch.tensor(verts, device="cuda"), o, d, scene)
    tri = tri.cpu().numpy()
    # the oracle on the moved scene (its own enclosing spheres)
    tris = verts[sc.faces]
    spheres = np.array([enclosing_sphere(tris[int(a):int(a) + int(b)].reshape(-1, 3).astype(np.float64))
                        for a, b in zip(sc.mesh_first, sc.mesh_count)], np.float32)
    moved = Scene(tris=np.ascontiguousarray(tris), mesh_first=sc.mesh_first, mesh_count=sc.mesh_count,
                  mesh_sphere=spheres, mesh_mat=sc.mesh_mat, mat_flags=sc.mat_flags, mat_ior=sc.mat_ior)
    o_run = O.run_pipeline(dataclasses.replace(wl, scene=moved))
    assert np.array_equal(tri, o_run["hits"][0])
    for x, y in zip((t, u, v), o_run["hits"][1:]):
        assert np.allclose(x.cpu().numpy(), y, rtol=1e-5, atol=0)
    # hits on moved triangles that lie wholly outside mesh 0's original sphere
    out = np.linalg.norm(tris[f0:f0 + n0].astype(np.float64) - c0, axis=2).min(axis=1) > r0
    hit0 = tri[(tri >= f0) & (tri < f0 + n0)]
    assert int(out[hit0 - f0].sum()) > 100
    rs = np.random.default_rng(11).choice(len(tri), 256, replace=False)
    b = O.brute_closest_hit(r, rs, moved, wl.t_min)
    assert np.array_equal(tri[rs], b[0])


def test_mesh_spheres_contain_every_vertex():
    """crsh_mesh_spheres on a scene of many meshes (plus an empty mesh and
    one clamped at the end of the triangle arrays): every vertex lies inside
    its mesh's sphere in float64, and no radius exceeds the half diagonal of
    the mesh's bounding box by more than the 2^-20 widening and rounding."""
    import torch
    import gpu_util as gu
    from paper_2312_06538_amd import crsh as X
    base, kw = ("mixed_1080p", dict(W=128, H=72, n_meshes=48))
    sc = workload(base, **kw).scene
    first = np.concatenate([sc.mesh_first, [sc.m, sc.m - 5]]).astype(np.uint32)
    count = np.concatenate([sc.mesh_count, [0, 100]]).astype(np.uint32)
    v9 = [gu.dev_f32(a) for a in sc.soa()]
    mf, mc = gu.dev_u32(first), gu.dev_u32(count)
    out = torch.full((4 * len(first),), -1.0, dtype=torch.float32, device="cuda")
    X.crsh_mesh_spheres([a.data_ptr() for a in v9], sc.m, mf.data_ptr(), mc.data_ptr(), len(first),
                        out.data_ptr(), gu.s())
    sph = out.cpu().numpy().reshape(-1, 4).astype(np.float64)
    for i, (a, n) in enumerate(zip(first, count)):
        a, e = int(a), min(int(a) + int(n), sc.m)
        if e <= a:
            assert np.array_equal(sph[i], [0, 0, 0, 0]), i
            continue
        p = sc.tris[a:e].reshape(-1, 3).astype(np.float64)
        dist = np.linalg.norm(p - sph[i, :3], axis=1)
        assert dist.max() <= sph[i, 3], i
        half = 0.5 * np.linalg.norm(p.max(0) - p.min(0))
        assert sph[i, 3] <= half * (1 + 2.0 ** -18) + 1e-6, i
