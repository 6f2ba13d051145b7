"""Batched form: many independent frames through one launch sequence of the
CRSH stages (crsh_batch_enqueue), optionally replayed as one hipGraph.

This module concatenates the frames' inputs into device arrays, fills the
crsh_batch descriptor and slices the products back per frame.  It allocates
and marshals; the C-ABI does the work.
"""
import ctypes

import numpy as np
import torch

from . import crsh as X
from .pipeline import F32, I32, I64, NODE_KEYS, RAY_KEYS, U8, node_capacity, stream_handle, u32


def _p(t):
    return None if t is None else t.data_ptr()


def top_nodes_bound(max_rays, B, F, levels):
    """Most top-level nodes a frame of at most max_rays rays can have."""
    c = max((max_rays + B - 1) // B, 1)
    for _ in range(levels - 1):
        if c <= 1:
            break
        c = (c + F - 1) // F
    return c


class DeviceBatch:
    """The frames (workloads) of one batch, uploaded once, with every device
    array the batched pipeline writes.  All frames use the hierarchy shape
    (B, F, levels); hit_block is the workgroup size of the final tests."""

    def __init__(self, wls, B, F, levels, hit_block=256, pair_capacity=1 << 22, keep_levels=False,
                 leaf_hit=False, ray_capacity=None, device="cuda"):
        if not 1 <= len(wls) <= X.MAX_FRAMES:
            raise ValueError(f"a batch holds 1..{X.MAX_FRAMES} frames")
        dev = torch.device(device)
        self.dev = dev
        self.wls = list(wls)
        self.B, self.F, self.levels, self.hit_block = int(B), int(F), int(levels), int(hit_block)
        self.keep_levels = keep_levels
        self.leaf_hit = bool(leaf_hit)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
        frames = (X.Frame * len(wls))()
        gb = {k: [] for k in ("px", "py", "pz", "nx", "ny", "nz", "mat")}
        soa = [[] for _ in range(9)]
        mesh_first, mesh_count, msph, mat_flags, mat_ior = [], [], [], [], []
        pix = tri = mesh = mat = 0
        self.cap = 0
        self.pair_capacity = int(pair_capacity)
        for f, wl in enumerate(wls):
            sc = wl.scene
            npx = wl.W * wl.H
            if npx < 1 or sc.n_mesh < 1:
                raise ValueError("every frame needs at least one pixel and one mesh")
            if len(wl.lights) > X.MAX_LIGHTS:
                raise ValueError("too many lights")
            for k in gb:
                gb[k].append(np.asarray(wl.gbuf[k]))
            for k, a in enumerate(sc.soa()):
                soa[k].append(a)
            mesh_first.append(sc.mesh_first.astype(np.int64) + tri)
            mesh_count.append(sc.mesh_count.astype(np.int64))
            msph.append(sc.mesh_sphere.reshape(-1))
            mat_flags.append(sc.mat_flags)
            mat_ior.append(sc.mat_ior)
            fr = frames[f]
            fr.pix_begin, fr.pix_count = pix, npx
            fr.mesh_begin, fr.mesh_count = mesh, sc.n_mesh
            fr.mat_begin, fr.n_mats = mat, len(sc.mat_flags)
            fr.n_lights, fr.ray_types = len(wl.lights), wl.ray_types
            for i, L in enumerate(wl.lights):
                for k in range(3):
                    fr.lights[i][k] = float(L[k])
            for k in range(3):
                fr.eye[k] = float(wl.eye[k])
                fr.lo[k] = float(wl.lo[k])
                fr.inv_ext[k] = float(wl.inv_ext[k])
            fr.eps_off, fr.eps_shadow, fr.t_min = wl.eps_off, wl.eps_shadow, wl.t_min
            self.cap += npx * (len(wl.lights) + 2)
            pix += npx
            tri += sc.m
            mesh += sc.n_mesh
            mat += len(sc.mat_flags)
        if ray_capacity is not None:     # room beyond the frames' most rays
            self.cap = max(self.cap, int(ray_capacity))
        if self.cap >= 1 << 30 or tri >= 1 << 32:
            raise ValueError("batch too large")
        self.n_frames, self.n_pix, self.m, self.n_mesh = len(wls), pix, tri, mesh
        self.slots = [wl.W * wl.H * (len(wl.lights) + 2) for wl in wls]
        self.frames_host = frames
        self.frames = t(np.frombuffer(bytes(frames), np.uint8), U8)
        self.frame_meta = torch.zeros(len(wls) * ctypes.sizeof(X.FrameMeta), dtype=U8, device=dev)
        self.g = {k: t(np.concatenate(v), I32 if k == "mat" else F32) for k, v in gb.items()}
        self.v = [t(np.concatenate(a), F32) for a in soa]
        self.mesh_first = t(np.concatenate(mesh_first).astype(np.uint32).view(np.int32), I32)
        self.mesh_count = t(np.concatenate(mesh_count).astype(np.uint32).view(np.int32), I32)
        self.msph = t(np.concatenate(msph).astype(np.float32), F32)
        self.mat_flags = t(np.concatenate(mat_flags).astype(np.uint32).view(np.int32), I32)
        self.mat_ior = t(np.concatenate(mat_ior).astype(np.float32), F32)
        e = lambda n, dt: torch.empty(max(int(n), 1), dtype=dt, device=dev)
        cap = self.cap
        self.rays = {k: e(cap, F32) for k in RAY_KEYS}
        self.rays["pix"] = e(cap, I32)
        self.srays = {k: e(cap, F32) for k in RAY_KEYS}
        self.srays["pix"] = e(cap, I32)
        self.keys, self.ids, self.skeys, self.sids = (e(cap, I32) for _ in range(4))
        self.ray_frame = e(cap, I32)
        self.tkey = e(cap, I64)
        self.hit_tri, self.hit_t, self.hit_u, self.hit_v = e(cap, I32), e(cap, F32), e(cap, F32), e(cap, F32)
        self.meta = torch.zeros(ctypes.sizeof(X.Meta), dtype=U8, device=dev)
        self.reshape(self.B, self.F, self.levels, self.hit_block, pair_capacity)

    def reshape(self, B, F, levels, hit_block=None, pair_capacity=None):
        """Change the hierarchy shape (and workgroup size of the final tests)
        keeping the uploaded frames; node and pair storage are resized."""
        self.B, self.F, self.levels = int(B), int(F), int(levels)
        if hit_block is not None:
            self.hit_block = int(hit_block)
        e = lambda n, dt: torch.empty(max(int(n), 1), dtype=dt, device=self.dev)
        self.node_cap = sum(node_capacity(s, self.B, self.F, self.levels) for s in self.slots)
        self.top_cap = sum(top_nodes_bound(s, self.B, self.F, self.levels) * wl.scene.n_mesh
                           for s, wl in zip(self.slots, self.wls))
        self.nodes = {k: e(self.node_cap, F32) for k in NODE_KEYS}
        self._alloc(pair_capacity if pair_capacity is not None else self.pair_capacity)

    def _alloc(self, pair_capacity):
        e = lambda n, dt: torch.empty(max(int(n), 1), dtype=dt, device=self.dev)
        cap = self.cap
        self.pair_capacity = int(pair_capacity)
        self.pair_bufs = None
        self.ws = None
        nbuf = self.levels if self.keep_levels else min(2, self.levels)
        self.pair_bufs = [(e(self.pair_capacity, I32), e(self.pair_capacity, I32)) for _ in range(nbuf)]
        self.ws_bytes = X.crsh_batch_ws_size(cap, self.m, self.node_cap, self.pair_capacity, self.top_cap)
        self.ws = e(self.ws_bytes, U8)
        self.c = self._descriptor()

    def level_buf(self, lv):
        return self.pair_bufs[lv - 1] if self.keep_levels else self.pair_bufs[lv % len(self.pair_bufs)]

    def _descriptor(self):
        b = X.Batch()
        b.n_frames, b.frames, b.frame_meta = self.n_frames, _p(self.frames), _p(self.frame_meta)
        b.gbuf = X.Gbuf(*[_p(self.g[k]) for k in ("px", "py", "pz", "nx", "ny", "nz", "mat")], self.n_pix, 1)
        b.mat_flags, b.mat_ior = _p(self.mat_flags), _p(self.mat_ior)
        b.scene = X.Scene((X.vp * 9)(*[_p(a) for a in self.v]), self.m, _p(self.mesh_first), _p(self.mesh_count),
                          _p(self.msph), self.n_mesh)
        r, s = self.rays, self.srays
        b.rays = X.Rays(*[_p(r[k]) for k in RAY_KEYS], _p(r["pix"]), self.cap)
        b.sorted = X.Rays(*[_p(s[k]) for k in RAY_KEYS], _p(s["pix"]), self.cap)
        b.keys, b.ids, b.skeys, b.sids = _p(self.keys), _p(self.ids), _p(self.skeys), _p(self.sids)
        b.ray_frame = _p(self.ray_frame)
        b.nodes = X.Nodes(*[_p(self.nodes[k]) for k in NODE_KEYS], self.node_cap)
        for lv in range(1, self.levels + 1):
            t, nd = self.level_buf(lv)
            b.pairs[lv - 1] = X.Pairs(_p(t), _p(nd), self.pair_capacity)
        b.hits = X.Hits(_p(self.tkey), _p(self.hit_tri), _p(self.hit_t), _p(self.hit_u), _p(self.hit_v), self.cap)
        b.meta = _p(self.meta)
        b.top_item_capacity = self.top_cap
        b.ws, b.ws_bytes = _p(self.ws), self.ws_bytes
        b.bundle, b.merge, b.levels, b.hit_block = self.B, self.F, self.levels, self.hit_block
        b.leaf_hit = 1 if self.leaf_hit else 0
        return b

    # ------------------------------------------------------------- running
    def enqueue(self, stream=None):
        X.crsh_batch_enqueue(self.c, stream_handle(stream))

    def read_meta(self, stream=None):
        return X.crsh_read_meta(_p(self.meta), stream_handle(stream))

    def run_with_retry(self, stream=None, grow=1.25, max_tries=12):
        """Enqueue; if a pair level overflowed, regrow the pair arrays (at
        least doubling) and run again.  Returns the batch meta."""
        for _ in range(max_tries):
            self.enqueue(stream)
            m, st = self.read_meta(stream)
            if st == X.OK:
                return m
            if m.status & ~X.OVERFLOW_PAIRS:
                raise X.CrshError(st, X.last_error())
            need = max(int(m.pairs[k]) for k in range(X.MAX_LEVELS))
            self._alloc(max(int(need * grow) + 1024, 2 * self.pair_capacity))
        raise X.CrshError(X.ERR_CAPACITY, "pair capacity still too small after regrowing")

    def graph(self, stream):
        """Capture the batch on `stream` (a torch.cuda.Stream, not the default
        stream) into a hipGraph; returns a BatchGraph."""
        return BatchGraph(self, stream)

    # ------------------------------------------------------------ products
    def frame_meta_host(self):
        raw = self.frame_meta.cpu().numpy().tobytes()
        return (X.FrameMeta * self.n_frames).from_buffer_copy(raw)

    def frame_results(self, m, with_pairs=True):
        """Per-frame host copies of every product, in the frame's own ids and
        node numbering (comparable with a plain run of the frame); without
        the pair levels when with_pairs is False."""
        fm = self.frame_meta_host()
        n = int(m.n_rays)
        host = {
            "rays": {k: self.rays[k][:n].cpu().numpy() for k in RAY_KEYS},
            "keys": u32(self.keys[:n]), "ids": u32(self.ids[:n]),
            "skeys": u32(self.skeys[:n]), "sids": u32(self.sids[:n]),
            "frame": u32(self.ray_frame[:n]),
            "hit": (self.hit_tri[:n].cpu().numpy(), self.hit_t[:n].cpu().numpy(), self.hit_u[:n].cpu().numpy(),
                    self.hit_v[:n].cpu().numpy()),
        }
        host["rays"]["pix"] = u32(self.rays["pix"][:n])
        nl = int(m.n_levels)
        tot = int(sum(m.level_cnt[k] for k in range(nl)))
        nodes = {k: self.nodes[k][:tot].cpu().numpy() for k in NODE_KEYS}
        pairs = {}
        for lv in range(1, nl + 1 if with_pairs else 1):
            if self.keep_levels or lv == 1:
                c = int(min(m.pairs[lv - 1], self.pair_capacity))
                t, nd = self.level_buf(lv)
                pairs[lv] = (u32(t[:c]), u32(nd[:c]))
        out = []
        tri_base = 0
        for f in range(self.n_frames):
            F_ = fm[f]
            rb, nr = int(F_.ray_begin), int(F_.n_rays)
            sl = slice(rb, rb + nr)
            pix0 = int(self.frames_host[f].pix_begin)
            r = {"n": nr, "ray_begin": rb, "n_levels": int(F_.n_levels)}
            r["rays"] = {k: v[sl] for k, v in host["rays"].items()}
            r["rays"]["pix"] = r["rays"]["pix"] - np.uint32(pix0)
            r["keys"] = host["keys"][sl]
            r["ids"] = host["ids"][sl] - np.uint32(rb)
            r["sorted_keys"] = host["skeys"][sl]
            r["sorted_ids"] = host["sids"][sl] - np.uint32(rb)
            r["ray_frame"] = host["frame"][sl]
            tri_hit = host["hit"][0][sl].copy()
            tri_hit[tri_hit >= 0] -= tri_base
            r["hit"] = (tri_hit, host["hit"][1][sl], host["hit"][2][sl], host["hit"][3][sl])
            nlf = int(F_.n_levels)
            r["level_cnt"] = np.array([F_.level_cnt[k] for k in range(nlf)], np.uint32)
            idx = np.concatenate([int(m.level_off[k]) + int(F_.level_base[k]) + np.arange(int(F_.level_cnt[k]))
                                  for k in range(nlf)]) if nlf else np.zeros(0, np.int64)
            r["nodes"] = {k: v[idx] for k, v in nodes.items()}
            r["pairs"] = {}
            for lv, (t, nd) in pairs.items():
                if lv > nlf:
                    continue
                base, cnt = int(F_.level_base[lv - 1]), int(F_.level_cnt[lv - 1])
                keep = (nd >= base) & (nd < base + cnt)
                r["pairs"][lv] = (t[keep] - np.uint32(tri_base), nd[keep] - np.uint32(base))
            out.append(r)
            tri_base += self.wls[f].scene.m
        return out


class BatchGraph:
    """One captured batch: launch() replays every stage of every frame."""

    def __init__(self, batch, stream):
        if stream is None or stream.cuda_stream == 0:
            raise ValueError("capture needs a non-default stream")
        self.batch = batch
        self.stream = stream
        self.g = X.crsh_batch_graph_create(batch.c, stream.cuda_stream)

    def launch(self):
        X.crsh_graph_launch(self.g, self.stream.cuda_stream)

    def close(self):
        if self.g is not None:
            X.crsh_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
