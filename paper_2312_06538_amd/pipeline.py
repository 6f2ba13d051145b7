"""The five CRSH stages chained on one stream, with torch tensors as the
device memory.  This module allocates and marshals; the C-ABI calls in
``paper_2312_06538_amd.crsh`` do the work.
"""
import ctypes

import numpy as np
import torch

from . import crsh as X

F32, I32, I64, U8 = torch.float32, torch.int32, torch.int64, torch.uint8
C_META_BYTES = ctypes.sizeof(X.Meta)
RAY_KEYS = ("ox", "oy", "oz", "dx", "dy", "dz", "tmax")
NODE_KEYS = ("cx", "cy", "cz", "r", "ax", "ay", "az", "c", "s", "tan", "sec")


def _p(t):
    return None if t is None else t.data_ptr()


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def u32(t):
    """Device int32 tensor -> host uint32 numpy array."""
    return t.cpu().numpy().view(np.uint32)


def node_capacity(max_rays, B, F, levels):
    c = (max_rays + B - 1) // B
    tot = c
    for _ in range(levels - 1):
        if c <= 1:
            break
        c = (c + F - 1) // F
        tot += c
    return max(tot, 1)


class DeviceFrame:
    """One frame's inputs, uploaded once: primary-hit buffer, ray-generation
    tables, scene."""

    def __init__(self, wl, device="cuda"):
        dev = torch.device(device)
        g = wl.gbuf
        self.wl = wl
        self.W, self.H = wl.W, wl.H
        self.B, self.F, self.n = wl.B, wl.F, wl.n
        self.t_min = wl.t_min
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
        self.g = {k: t(g[k], F32) for k in ("px", "py", "pz", "nx", "ny", "nz")}
        self.g["mat"] = t(g["mat"], I32)
        sc = wl.scene
        self.v = [t(a, F32) for a in sc.soa()]
        self.mesh_first = t(sc.mesh_first.view(np.int32), I32)
        self.mesh_count = t(sc.mesh_count.view(np.int32), I32)
        self.msph = t(sc.mesh_sphere.reshape(-1), F32)
        self.tri_mat = t(np.ascontiguousarray(sc.tri_mat(), np.int32), I32)
        self.mat_flags = t(sc.mat_flags.view(np.int32), I32)
        self.mat_ior = t(sc.mat_ior, F32)
        self.m, self.n_mesh = sc.m, sc.n_mesh
        self.gbuf = X.Gbuf(*[_p(self.g[k]) for k in ("px", "py", "pz", "nx", "ny", "nz", "mat")], wl.W, wl.H)
        rg = X.Raygen()
        rg.n_lights = len(wl.lights)
        for i, L in enumerate(wl.lights):
            for k in range(3):
                rg.lights[i][k] = float(L[k])
        for k in range(3):
            rg.eye[k] = float(wl.eye[k])
            rg.lo[k] = float(wl.lo[k])
            rg.inv_ext[k] = float(wl.inv_ext[k])
        rg.mat_flags, rg.mat_ior, rg.n_mats = _p(self.mat_flags), _p(self.mat_ior), len(sc.mat_flags)
        rg.ray_types, rg.eps_off, rg.eps_shadow = wl.ray_types, wl.eps_off, wl.eps_shadow
        self.raygen = rg
        self.scene = X.Scene((X.vp * 9)(*[_p(a) for a in self.v]), self.m, _p(self.mesh_first),
                             _p(self.mesh_count), _p(self.msph), self.n_mesh)
        self.max_rays = wl.W * wl.H * (len(wl.lights) + 2)


class Buffers:
    """Every device array of one frame.  keep_levels=True keeps all pair
    levels (for inspection); otherwise two arrays alternate between levels."""

    def __init__(self, fr, pair_capacity, keep_levels=False, device="cuda", ray_capacity=None):
        dev = torch.device(device)
        cap = int(ray_capacity or fr.max_rays)
        self.cap = cap
        e = lambda n, dt: torch.empty(max(int(n), 1), dtype=dt, device=dev)
        self.rays = {k: e(cap, F32) for k in RAY_KEYS}
        self.rays["pix"] = e(cap, I32)
        self.keys, self.ids = e(cap, I32), e(cap, I32)
        self.skeys, self.sids = e(cap, I32), e(cap, I32)
        self.srays = {k: e(cap, F32) for k in RAY_KEYS}
        self.srays["pix"] = e(cap, I32)
        self.node_cap = node_capacity(cap, fr.B, fr.F, fr.n)
        self.nodes = {k: e(self.node_cap, F32) for k in NODE_KEYS}
        self.keep_levels = keep_levels
        self.pair_capacity = int(pair_capacity)
        nbuf = fr.n if keep_levels else min(2, fr.n)
        self.pair_bufs = [(e(self.pair_capacity, I32), e(self.pair_capacity, I32)) for _ in range(nbuf)]
        self.tkey = e(cap, I64)
        self.hit_tri, self.hit_t, self.hit_u, self.hit_v = e(cap, I32), e(cap, F32), e(cap, F32), e(cap, F32)
        self.meta = torch.zeros(C_META_BYTES, dtype=U8, device=dev)
        self.ray_capacity = cap
        self.ws_bytes = X.crsh_workspace_size(cap, fr.m, fr.n_mesh, self.node_cap, self.pair_capacity)
        self.ws = e(self.ws_bytes, U8)
        r = self.rays
        self.c_rays = X.Rays(*[_p(r[k]) for k in RAY_KEYS], _p(r["pix"]), cap)
        s = self.srays
        self.c_srays = X.Rays(*[_p(s[k]) for k in RAY_KEYS], _p(s["pix"]), cap)
        self.c_nodes = X.Nodes(*[_p(self.nodes[k]) for k in NODE_KEYS], self.node_cap)
        self.c_pairs = X.PairTable()
        for lv in range(1, fr.n + 1):
            b = self.level_buf(lv)
            self.c_pairs[lv - 1] = X.Pairs(_p(b[0]), _p(b[1]), self.pair_capacity)
        self.c_hits = X.Hits(_p(self.tkey), _p(self.hit_tri), _p(self.hit_t), _p(self.hit_u), _p(self.hit_v), cap)
        # packed pairs (one word each) reuse the triangle array of every level
        self.c_packed = X.PackedPairTable()
        for lv in range(1, fr.n + 1):
            self.c_packed[lv - 1] = X.PackedPairs(_p(self.level_buf(lv)[0]), self.pair_capacity)

    def level_buf(self, lv):
        return self.pair_bufs[lv - 1] if self.keep_levels else self.pair_bufs[lv % len(self.pair_bufs)]


def packed_batches(m):
    """Triangle batches of at most PACKED_MAX_TRIS triangles covering [0, m)."""
    return [(b, min(b + X.PACKED_MAX_TRIS, m)) for b in range(0, max(m, 1), X.PACKED_MAX_TRIS)]


def run_frame(fr, bf, stream=None, tri_batches=None, leaf_hit=False, parent=None, packed=False):
    """Chain hash -> sort -> build -> traverse -> closest hit on one stream.
    leaf_hit: the last traversal level runs fused with the final tests
    (crsh_traverse_upper + crsh_leaf_hit); otherwise every level-1 pair is
    stored (crsh_traverse + crsh_closest_hit).  packed: pairs stored one
    32-bit word each (crsh_traverse_packed + crsh_closest_hit_packed), over
    triangle batches of at most PACKED_MAX_TRIS.  parent: the Buffers of the
    previous generation; the rays then come from its closest hits
    (crsh_bounce) instead of the primary-hit buffer."""
    s = stream_handle(stream)
    meta, ws, wsb = _p(bf.meta), _p(bf.ws), bf.ws_bytes
    X.crsh_meta_reset(meta, s)
    if parent is None:
        X.crsh_hash(fr.gbuf, fr.raygen, bf.c_rays, _p(bf.keys), _p(bf.ids), meta, ws, wsb, s)
    else:
        X.crsh_bounce(parent.c_rays, _p(parent.keys), parent.c_hits, _p(parent.meta), fr.scene, _p(fr.tri_mat),
                      fr.raygen, bf.c_rays, _p(bf.keys), _p(bf.ids), meta, ws, wsb, s)
    X.crsh_sort(_p(bf.keys), _p(bf.ids), _p(bf.skeys), _p(bf.sids), bf.cap, meta, ws, wsb, s)
    X.crsh_build(bf.c_rays, _p(bf.sids), fr.B, fr.F, fr.n, bf.c_nodes, bf.c_srays, meta, s)
    X.crsh_hits_reset(bf.c_hits, s)
    fuse = leaf_hit and fr.n >= 2
    if packed and tri_batches is None:
        tri_batches = packed_batches(fr.m)
    for (b, e) in (tri_batches or [(0, fr.m)]):
        if packed:
            X.crsh_traverse_packed(bf.c_nodes, fr.scene, b, e, fr.B, fr.F, bf.c_packed, meta, ws, wsb, s)
            X.crsh_closest_hit_packed(bf.c_srays, _p(bf.sids), fr.B, bf.c_packed[0], b, fr.scene, fr.t_min,
                                      bf.c_hits, meta, ws, wsb, s)
        elif fuse:
            X.crsh_traverse_upper(bf.c_nodes, fr.scene, b, e, fr.B, fr.F, bf.c_pairs, meta, ws, wsb, s)
            X.crsh_leaf_hit(bf.c_srays, _p(bf.sids), fr.B, fr.F, bf.c_nodes, bf.c_pairs, fr.scene, fr.t_min,
                            bf.c_hits, meta, ws, wsb, s)
        else:
            X.crsh_traverse(bf.c_nodes, fr.scene, b, e, fr.B, fr.F, bf.c_pairs, meta, ws, wsb, s)
            X.crsh_closest_hit(bf.c_srays, _p(bf.sids), fr.B, bf.c_pairs[0], fr.scene, fr.t_min, bf.c_hits, meta,
                               ws, wsb, s)


def read_meta(bf, stream=None):
    m, st = X.crsh_read_meta(_p(bf.meta), stream_handle(stream))
    return m, st


def run_with_retry(fr, bf, stream=None, tri_batches=None, grow=1.25, max_tries=12, leaf_hit=False, parent=None,
                   packed=False):
    """Run a frame; if a pair level overflowed, regrow the pair arrays and run
    again (the ray arrays likewise for a bounce generation that outgrew
    them).  An overflowing level truncates the levels below it, so their
    reported sizes are lower bounds: grow to at least twice the capacity.
    Returns (buffers, meta)."""
    for _ in range(max_tries):
        run_frame(fr, bf, stream, tri_batches, leaf_hit=leaf_hit, parent=parent, packed=packed)
        m, st = read_meta(bf, stream)
        if st == X.OK:
            return bf, m
        if m.status & ~(X.OVERFLOW_PAIRS | X.OVERFLOW_RAYS):
            raise X.CrshError(st, X.last_error())
        need = max(int(m.pairs[k]) for k in range(X.MAX_LEVELS))
        cap = max(int(need * grow) + 1024, 2 * bf.pair_capacity) if m.status & X.OVERFLOW_PAIRS else \
            bf.pair_capacity
        rays = max(int(m.rays_required), bf.ray_capacity)
        bf = Buffers(fr, cap, keep_levels=bf.keep_levels, ray_capacity=rays)
    raise X.CrshError(X.ERR_CAPACITY, "capacity still too small after regrowing")


def run_generations(fr, depth, pair_capacity=1 << 22, keep_levels=False, leaf_hit=False, stream=None):
    """`depth` generations of the path (Sec. 3.3.8): the first from the
    primary-hit buffer, each next one from the closest hits of the previous
    (crsh_bounce), every one through sort, build, traversal and final tests.
    Returns [(buffers, meta)] per generation."""
    out = []
    parent = None
    for _ in range(depth):
        bf = Buffers(fr, pair_capacity, keep_levels=keep_levels,
                     ray_capacity=None if parent is None else parent[0].ray_capacity)
        bf, m = run_with_retry(fr, bf, stream, leaf_hit=leaf_hit, parent=None if parent is None else parent[0])
        out.append((bf, m))
        parent = (bf, m)
    return out


def results(fr, bf, m):
    """Host copies of every product of a frame (for tests and inspection)."""
    n = int(m.n_rays)
    out = {"n": n, "meta": m}
    out["rays"] = {k: bf.rays[k][:n].cpu().numpy() for k in RAY_KEYS}
    out["rays"]["pix"] = u32(bf.rays["pix"][:n])
    out["keys"], out["ids"] = u32(bf.keys[:n]), u32(bf.ids[:n])
    out["sorted_keys"], out["sorted_ids"] = u32(bf.skeys[:n]), u32(bf.sids[:n])
    nl = int(m.n_levels)
    tot = int(sum(m.level_cnt[k] for k in range(nl)))
    out["nodes"] = {k: bf.nodes[k][:tot].cpu().numpy() for k in NODE_KEYS}
    out["level_off"] = np.array([m.level_off[k] for k in range(nl)], np.uint32)
    out["level_cnt"] = np.array([m.level_cnt[k] for k in range(nl)], np.uint32)
    out["n_levels"] = nl
    pairs = {}
    for lv in range(1, nl + 1):
        if bf.keep_levels or lv == 1:
            c = int(min(m.pairs[lv - 1], bf.pair_capacity))
            t, nd = bf.level_buf(lv)
            pairs[lv] = (u32(t[:c]), u32(nd[:c]))
    out["pairs"] = pairs
    out["tests"] = {lv: int(m.tests[lv - 1]) for lv in range(1, nl + 1)}
    out["hits"] = {lv: int(m.hits[lv - 1]) for lv in range(1, nl + 1)}
    out["mesh_tests"], out["mesh_hits"], out["final_tests"] = int(m.mesh_tests), int(m.mesh_hits), int(m.final_tests)
    out["hit"] = (bf.hit_tri[:n].cpu().numpy(), bf.hit_t[:n].cpu().numpy(), bf.hit_u[:n].cpu().numpy(),
                  bf.hit_v[:n].cpu().numpy())
    return out
