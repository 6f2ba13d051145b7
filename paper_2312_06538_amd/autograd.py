"""Differentiable closest hit: the CRSH path as a torch.autograd.Function.

Forward: caller-given rays (origin, direction) against an indexed triangle
mesh -- crsh_hash_rays, crsh_sort, crsh_build, crsh_traverse,
crsh_closest_hit -- returning per ray the hit triangle (-1 on a miss) and
t, u, v.  Backward: crsh_closest_hit_backward, the adjoint with each ray's hit
triangle held fixed, giving dL/d(vertices), dL/d(origins), dL/d(directions);
vertex gradients accumulate with float32 atomics.  Nothing but the C-ABI
computes; torch provides memory and the stream.
"""
import numpy as np
import torch

from . import crsh as X
from .pipeline import NODE_KEYS, RAY_KEYS, node_capacity, stream_handle


def _p(t):
    return t.data_ptr()


class RayScene:
    """An indexed mesh with its mesh ranges, and the hierarchy parameters,
    for closest hits of caller-given rays.  The vertices come with every
    call; each call gathers the triangles and recomputes every mesh's
    enclosing sphere from them (crsh_mesh_spheres), so whole-mesh culling
    stays conservative while the vertices move."""

    def __init__(self, faces, mesh_first, mesh_count, lo, inv_ext, B=16, F=4, levels=5,
                 t_min=1e-4, ray_type=1, pair_capacity=1 << 22):
        dev = torch.device("cuda")
        self.faces = torch.as_tensor(np.ascontiguousarray(faces, np.int32)).to(dev)
        self.m = int(self.faces.shape[0])
        self.mesh_first = torch.as_tensor(np.asarray(mesh_first, np.uint32).view(np.int32)).to(dev)
        self.mesh_count = torch.as_tensor(np.asarray(mesh_count, np.uint32).view(np.int32)).to(dev)
        self.n_mesh = int(self.mesh_first.shape[0])
        self.msph = torch.empty(4 * max(self.n_mesh, 1), dtype=torch.float32, device=dev)
        self.lo = [float(x) for x in lo]
        self.inv_ext = [float(x) for x in inv_ext]
        self.B, self.F, self.levels, self.t_min, self.ray_type = B, F, levels, float(t_min), ray_type
        self.pair_capacity = int(pair_capacity)
        self.v9 = [torch.empty(self.m, dtype=torch.float32, device=dev) for _ in range(9)]
        self._cap = 0

    def _alloc(self, n):
        dev = torch.device("cuda")
        cap = max(n, 1)
        e = lambda k, dt: torch.empty(max(int(k), 1), dtype=dt, device=dev)
        self.rays = {k: e(cap, torch.float32) for k in RAY_KEYS}
        self.srays = {k: e(cap, torch.float32) for k in RAY_KEYS}
        self.keys, self.ids = e(cap, torch.int32), e(cap, torch.int32)
        self.skeys, self.sids = e(cap, torch.int32), e(cap, torch.int32)
        self.node_cap = node_capacity(cap, self.B, self.F, self.levels)
        self.nodes = {k: e(self.node_cap, torch.float32) for k in NODE_KEYS}
        self.meta = torch.zeros(X.ctypes_sizeof_meta(), dtype=torch.uint8, device=dev)
        self._cap = cap
        self._alloc_pairs()

    def _alloc_pairs(self):
        dev = torch.device("cuda")
        e = lambda k, dt: torch.empty(max(int(k), 1), dtype=dt, device=dev)
        nbuf = min(2, self.levels)
        self.pbuf = [(e(self.pair_capacity, torch.int32), e(self.pair_capacity, torch.int32)) for _ in range(nbuf)]
        self.table = X.PairTable()
        for lv in range(1, self.levels + 1):
            b = self.pbuf[lv % nbuf]
            self.table[lv - 1] = X.Pairs(_p(b[0]), _p(b[1]), self.pair_capacity)
        self.ws_bytes = X.crsh_workspace_size(self._cap, self.m, self.n_mesh, self.node_cap, self.pair_capacity)
        self.ws = e(self.ws_bytes, torch.uint8)

    def closest_hit(self, verts, o, d):
        """verts [V,3], o/d [N,3] float32 cuda -> (tri int32, t, u, v) per ray."""
        n = int(o.shape[0])
        if n > self._cap:
            self._alloc(n)
        s = stream_handle()
        X.crsh_gather_triangles(_p(verts), int(verts.shape[0]), _p(self.faces), self.m,
                                [_p(a) for a in self.v9], s)
        X.crsh_mesh_spheres([_p(a) for a in self.v9], self.m, _p(self.mesh_first), _p(self.mesh_count),
                            self.n_mesh, _p(self.msph), s)
        for i, k in enumerate(("ox", "oy", "oz")):
            self.rays[k][:n].copy_(o[:, i])
        for i, k in enumerate(("dx", "dy", "dz")):
            self.rays[k][:n].copy_(d[:, i])
        self.rays["tmax"][:n].fill_(float(np.finfo(np.float32).max))
        c_rays = X.Rays(*[_p(self.rays[k]) for k in RAY_KEYS], None, self._cap)
        c_srays = X.Rays(*[_p(self.srays[k]) for k in RAY_KEYS], None, self._cap)
        c_nodes = X.Nodes(*[_p(self.nodes[k]) for k in NODE_KEYS], self.node_cap)
        scene = X.Scene((X.vp * 9)(*[_p(a) for a in self.v9]), self.m, _p(self.mesh_first), _p(self.mesh_count),
                        _p(self.msph), self.n_mesh)
        dev = verts.device
        tkey = torch.empty(self._cap, dtype=torch.int64, device=dev)
        tri = torch.empty(self._cap, dtype=torch.int32, device=dev)
        t, u, v = (torch.empty(self._cap, dtype=torch.float32, device=dev) for _ in range(3))
        hits = X.Hits(_p(tkey), _p(tri), _p(t), _p(u), _p(v), self._cap)
        for _ in range(12):
            meta = _p(self.meta)
            X.crsh_meta_reset(meta, s)
            X.crsh_hash_rays(c_rays, n, self.ray_type, 0, self.lo, self.inv_ext, _p(self.keys), _p(self.ids),
                             meta, s)
            X.crsh_sort(_p(self.keys), _p(self.ids), _p(self.skeys), _p(self.sids), self._cap, meta, _p(self.ws),
                        self.ws_bytes, s)
            X.crsh_build(c_rays, _p(self.sids), self.B, self.F, self.levels, c_nodes, c_srays, meta, s)
            X.crsh_hits_reset(hits, s)
            X.crsh_traverse(c_nodes, scene, 0, self.m, self.B, self.F, self.table, meta, _p(self.ws), self.ws_bytes,
                            s)
            X.crsh_closest_hit(c_srays, _p(self.sids), self.B, self.table[0], scene, self.t_min, hits, meta,
                               _p(self.ws), self.ws_bytes, s)
            m, st = X.crsh_read_meta(meta, s)
            if st == X.OK:
                break
            if m.status & ~X.OVERFLOW_PAIRS:
                raise X.CrshError(st, X.last_error())
            need = max(int(m.pairs[k]) for k in range(X.MAX_LEVELS))
            self.pair_capacity = max(int(need * 1.25) + 1024, 2 * self.pair_capacity)
            self._alloc_pairs()
        else:
            raise X.CrshError(X.ERR_CAPACITY, "pair capacity still too small")
        self.last_meta = m
        return tri[:n], t[:n], u[:n], v[:n]

    def backward(self, verts, o, d, tri, t, u, v, g_t, g_u, g_v):
        n = int(o.shape[0])
        dev = verts.device
        rays = {k: torch.empty(max(n, 1), dtype=torch.float32, device=dev) for k in RAY_KEYS}
        for i, k in enumerate(("ox", "oy", "oz")):
            rays[k][:n].copy_(o[:, i])
        for i, k in enumerate(("dx", "dy", "dz")):
            rays[k][:n].copy_(d[:, i])
        c_rays = X.Rays(*[_p(rays[k]) for k in RAY_KEYS], None, max(n, 1))
        tri, t, u, v = (x.contiguous() for x in (tri, t, u, v))
        hits = X.Hits(None, _p(tri), _p(t), _p(u), _p(v), max(n, 1))
        g_verts = torch.zeros_like(verts)
        g_o = torch.empty((n, 3), dtype=torch.float32, device=dev)
        g_d = torch.empty((n, 3), dtype=torch.float32, device=dev)
        keep = [g.contiguous() if g is not None else None for g in (g_t, g_u, g_v)]
        gp = [None if g is None else _p(g) for g in keep]
        X.crsh_closest_hit_backward(c_rays, n, hits, gp[0], gp[1], gp[2], _p(verts), int(verts.shape[0]),
                                    _p(self.faces), self.m, _p(g_verts), _p(g_o), _p(g_d), stream_handle())
        return g_verts, g_o, g_d


class ClosestHit(torch.autograd.Function):
    """tri, t, u, v = ClosestHit.apply(verts, o, d, scene); t, u, v are
    differentiable with respect to verts, o and d (hit triangles held fixed)."""

    @staticmethod
    def forward(ctx, verts, o, d, scene):
        verts = verts.contiguous()
        o = o.contiguous()
        d = d.contiguous()
        tri, t, u, v = scene.closest_hit(verts, o, d)
        tri, t, u, v = tri.clone(), t.clone(), u.clone(), v.clone()
        ctx.scene = scene
        ctx.save_for_backward(verts, o, d, tri, t, u, v)
        ctx.mark_non_differentiable(tri)
        return tri, t, u, v

    @staticmethod
    def backward(ctx, g_tri, g_t, g_u, g_v):
        verts, o, d, tri, t, u, v = ctx.saved_tensors
        g_verts, g_o, g_d = ctx.scene.backward(verts, o, d, tri, t, u, v, g_t, g_u, g_v)
        return g_verts, g_o, g_d, None


def closest_hit(verts, o, d, scene):
    return ClosestHit.apply(verts, o, d, scene)
