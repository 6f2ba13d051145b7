"""Stage-by-stage calls of the HIP library through its C-ABI, for parity
tests.  Inputs may come from the oracle (so a stage is tested on exactly the
oracle's input); expected values always come from the oracle."""
import ctypes

import numpy as np
import torch

from paper_2312_06538_amd import crsh as X
from paper_2312_06538_amd import pipeline as P

RAY_KEYS = P.RAY_KEYS
NODE_KEYS = P.NODE_KEYS


def dev_f32(a, n=None):
    a = np.ascontiguousarray(a, np.float32)
    t = torch.zeros(max(n or len(a), 1), dtype=torch.float32, device="cuda")
    if len(a):
        t[:len(a)] = torch.from_numpy(a).cuda()
    return t


def dev_u32(a, n=None):
    a = np.ascontiguousarray(a, np.uint32).view(np.int32)
    t = torch.zeros(max(n or len(a), 1), dtype=torch.int32, device="cuda")
    if len(a):
        t[:len(a)] = torch.from_numpy(a).cuda()
    return t


def s():
    return P.stream_handle()


def new_meta(**fields):
    """A device crsh_meta with the given host fields set."""
    m = X.Meta()
    for k, v in fields.items():
        if isinstance(v, (list, tuple, np.ndarray)):
            arr = getattr(m, k)
            for i, x in enumerate(v):
                arr[i] = int(x)
        else:
            setattr(m, k, int(v))
    raw = np.frombuffer(bytes(m), dtype=np.uint8).copy()
    return torch.from_numpy(raw).cuda()


def read_meta(meta_t):
    m, st = X.crsh_read_meta(meta_t.data_ptr(), s())
    return m, st


def ws_tensor(nbytes):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def gpu_hash(wl):
    fr = P.DeviceFrame(wl)
    cap = fr.max_rays
    rays = {k: torch.zeros(cap, dtype=torch.float32, device="cuda") for k in RAY_KEYS}
    rays["pix"] = torch.zeros(cap, dtype=torch.int32, device="cuda")
    keys = torch.zeros(cap, dtype=torch.int32, device="cuda")
    ids = torch.zeros(cap, dtype=torch.int32, device="cuda")
    c_rays = X.Rays(*[rays[k].data_ptr() for k in RAY_KEYS], rays["pix"].data_ptr(), cap)
    meta = new_meta()
    wsb = X.crsh_workspace_size(cap, 1, 1, 1, 1)
    ws = ws_tensor(wsb)
    X.crsh_hash(fr.gbuf, fr.raygen, c_rays, keys.data_ptr(), ids.data_ptr(), meta.data_ptr(), ws.data_ptr(), wsb,
                s())
    m, st = read_meta(meta)
    n = int(m.n_rays)
    out = {k: rays[k][:n].cpu().numpy() for k in RAY_KEYS}
    out["pix"] = P.u32(rays["pix"][:n])
    return {"rays": out, "keys": P.u32(keys[:n]), "ids": P.u32(ids[:n]), "n": n, "meta": m, "status": st}


def gpu_sort(keys, ids, capacity=None, chunked=False):
    n = len(keys)
    cap = max(capacity or n, 1)
    kin, vin = dev_u32(keys, cap), dev_u32(ids, cap)
    kout = torch.zeros(cap, dtype=torch.int32, device="cuda")
    vout = torch.zeros(cap, dtype=torch.int32, device="cuda")
    meta = new_meta(n_rays=n)
    wsb = X.crsh_workspace_size(cap, 1, 1, 1, 1)
    ws = ws_tensor(wsb)
    fn = X.crsh_sort_chunked if chunked else X.crsh_sort
    fn(kin.data_ptr(), vin.data_ptr(), kout.data_ptr(), vout.data_ptr(), cap, meta.data_ptr(), ws.data_ptr(), wsb,
       s())
    read_meta(meta)
    return P.u32(kout[:n]), P.u32(vout[:n])


def gpu_build(rays, sorted_ids, B, F, levels, n_rays=None):
    n = len(sorted_ids) if n_rays is None else n_rays
    cap = max(len(sorted_ids), 1)
    r = {k: dev_f32(rays[k], max(len(rays[k]), 1)) for k in RAY_KEYS}
    sid = dev_u32(sorted_ids, cap)
    sr = {k: torch.zeros(cap, dtype=torch.float32, device="cuda") for k in RAY_KEYS}
    spix = torch.zeros(cap, dtype=torch.int32, device="cuda")
    pix = dev_u32(rays["pix"], max(len(rays["pix"]), 1))
    c_rays = X.Rays(*[r[k].data_ptr() for k in RAY_KEYS], pix.data_ptr(), cap)
    c_sr = X.Rays(*[sr[k].data_ptr() for k in RAY_KEYS], spix.data_ptr(), cap)
    ncap = P.node_capacity(cap, B, F, levels)
    nodes = {k: torch.zeros(ncap, dtype=torch.float32, device="cuda") for k in NODE_KEYS}
    c_nodes = X.Nodes(*[nodes[k].data_ptr() for k in NODE_KEYS], ncap)
    meta = new_meta(n_rays=n)
    X.crsh_build(c_rays, sid.data_ptr(), B, F, levels, c_nodes, c_sr, meta.data_ptr(), s())
    m, st = read_meta(meta)
    nl = int(m.n_levels)
    tot = int(sum(m.level_cnt[k] for k in range(nl)))
    return {"nodes": {k: nodes[k][:tot].cpu().numpy() for k in NODE_KEYS},
            "level_off": np.array([m.level_off[k] for k in range(nl)], np.uint32),
            "level_cnt": np.array([m.level_cnt[k] for k in range(nl)], np.uint32),
            "n_levels": nl, "sorted": {k: sr[k][:n].cpu().numpy() for k in RAY_KEYS},
            "sorted_pix": P.u32(spix[:n]), "meta": m, "status": st}


def _scene(sc):
    keep = [dev_f32(a) for a in sc.soa()]
    mf, mc = dev_u32(sc.mesh_first), dev_u32(sc.mesh_count)
    ms = dev_f32(sc.mesh_sphere.reshape(-1))
    keep += [mf, mc, ms]
    c = X.Scene((X.vp * 9)(*[keep[k].data_ptr() for k in range(9)]), sc.m, mf.data_ptr(), mc.data_ptr(),
                ms.data_ptr(), sc.n_mesh)
    return c, keep


def gpu_traverse(tree, sc, B, F, batches=None, capacity=None, n_levels_alloc=None):
    """tree: oracle-format dict (nodes, level_off, level_cnt, n_levels, n_rays)."""
    nl = tree["n_levels"]
    total = int(sum(tree["level_cnt"])) if nl else 0
    ncap = max(total, 1)
    nodes = {k: dev_f32(tree["nodes"][k], ncap) for k in NODE_KEYS}
    c_nodes = X.Nodes(*[nodes[k].data_ptr() for k in NODE_KEYS], ncap)
    c_sc, keep = _scene(sc)
    cap = capacity or 1 << 20
    nalloc = n_levels_alloc or max(nl, 1)
    bufs = [(torch.zeros(cap, dtype=torch.int32, device="cuda"), torch.zeros(cap, dtype=torch.int32, device="cuda"))
            for _ in range(nalloc)]
    table = X.PairTable()
    for k in range(nalloc):
        table[k] = X.Pairs(bufs[k][0].data_ptr(), bufs[k][1].data_ptr(), cap)
    meta = new_meta(n_rays=tree["n_rays"], n_levels=nl, level_off=list(tree["level_off"]),
                    level_cnt=list(tree["level_cnt"]))
    wsb = X.crsh_workspace_size(1, sc.m, sc.n_mesh, ncap, cap)
    ws = ws_tensor(wsb)
    runs = []
    for (b, e) in (batches or [(0, sc.m)]):
        X.crsh_traverse(c_nodes, c_sc, b, e, B, F, table, meta.data_ptr(), ws.data_ptr(), wsb, s())
        m, st = read_meta(meta)
        pairs = {}
        for lv in range(1, nl + 1):
            c = int(min(m.pairs[lv - 1], cap))
            pairs[lv] = (P.u32(bufs[lv - 1][0][:c]), P.u32(bufs[lv - 1][1][:c]))
        runs.append({"pairs": pairs, "meta": m, "status": st})
    m = runs[-1]["meta"]
    return {"runs": runs, "pairs": runs[-1]["pairs"],
            "tests": {lv: int(m.tests[lv - 1]) for lv in range(1, nl + 1)},
            "hits": {lv: int(m.hits[lv - 1]) for lv in range(1, nl + 1)},
            "mesh_tests": int(m.mesh_tests), "mesh_hits": int(m.mesh_hits), "status": runs[-1]["status"],
            "meta": m}


def gpu_closest_hit(rays, sorted_ids, B, pairs1, sc, t_min):
    """rays by id (oracle format), level-1 pairs (tri, node)."""
    n = len(sorted_ids)
    cap = max(n, 1)
    sid = sorted_ids.astype(np.int64)
    sr = {k: dev_f32(np.asarray(rays[k])[sid], cap) for k in RAY_KEYS}
    c_sr = X.Rays(*[sr[k].data_ptr() for k in RAY_KEYS], None, cap)
    d_sid = dev_u32(sorted_ids, cap)
    pt, pn = dev_u32(pairs1[0]), dev_u32(pairs1[1])
    lvl1 = X.Pairs(pt.data_ptr(), pn.data_ptr(), max(len(pairs1[0]), 1))
    c_sc, keep = _scene(sc)
    tkey = torch.zeros(cap, dtype=torch.int64, device="cuda")
    tri = torch.zeros(cap, dtype=torch.int32, device="cuda")
    tt, uu, vv = (torch.zeros(cap, dtype=torch.float32, device="cuda") for _ in range(3))
    hits = X.Hits(tkey.data_ptr(), tri.data_ptr(), tt.data_ptr(), uu.data_ptr(), vv.data_ptr(), cap)
    meta = new_meta(n_rays=n, n_levels=1, pairs=[len(pairs1[0])])
    wsb = X.crsh_workspace_size(cap, sc.m, 1, 1, 1)
    ws = ws_tensor(wsb)
    X.crsh_hits_reset(hits, s())
    X.crsh_closest_hit(c_sr, d_sid.data_ptr(), B, lvl1, c_sc, t_min, hits, meta.data_ptr(), ws.data_ptr(),
                       wsb, s())
    m, st = read_meta(meta)
    return (tri[:n].cpu().numpy(), tt[:n].cpu().numpy(), uu[:n].cpu().numpy(), vv[:n].cpu().numpy()), m


def run_pipeline(wl, pair_capacity=1 << 20, keep_levels=True, tri_batches=None, leaf_hit=False, packed=False):
    """The whole path; leaf_hit=False stores every pair level (for
    inspection), True runs the last level fused with the final tests.
    packed: pairs as packed words (results' pairs hold the words in place of
    the triangle ids; decode with decode_packed)."""
    fr = P.DeviceFrame(wl)
    bf = P.Buffers(fr, pair_capacity, keep_levels=keep_levels)
    bf, m = P.run_with_retry(fr, bf, tri_batches=tri_batches, leaf_hit=leaf_hit, packed=packed)
    return P.results(fr, bf, m)


def decode_packed(words, tri_begin):
    """(triangle ids, node ids) of packed pairs of the batch starting at tri_begin."""
    w = np.asarray(words).astype(np.uint32)
    low = w & np.uint32(X.PACKED_MAX_TRIS - 1)
    return (low + np.uint32(tri_begin)).astype(np.uint32), (w >> np.uint32(X.PACKED_TRI_BITS)).astype(np.uint32)


def pair_keys(t, n):
    return (np.asarray(n, np.uint64) << np.uint64(32)) | np.asarray(t, np.uint64)


def run_generations(wl, depth, pair_capacity=1 << 20, keep_levels=True, leaf_hit=False):
    fr = P.DeviceFrame(wl)
    return [P.results(fr, bf, m) for bf, m in P.run_generations(fr, depth, pair_capacity, keep_levels, leaf_hit)]
