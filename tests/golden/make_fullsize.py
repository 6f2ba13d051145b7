"""Write the full-frame expected values of the two large workloads.

Calls only the oracle (``oracle/``) and the seeded input generators
(``workloads/``).  The oracle is sequential; the frame is split over its
top-level sub-trees, which are independent (Sec. 3.3.7: every pair below the
top descends from one top node, and a top node's rays are a contiguous run of
the sorted order), and the sub-trees are run in a process pool.  Because the
oracle writes the top level node by node and every lower level in the order
of its parents, each level of the whole frame is the concatenation of the
sub-trees' levels in top-node order.

Written per workload, to ``fullsize_<name>.json``:

* every traversal counter of the frame: node tests and surviving pairs per
  level, mesh tests and hits, final ray-triangle tests, and how many of
  those passed the u check and the u and v checks;
* per top node: its level-1 pair count and the SHA-256 of its level-1 pairs
  (the triangle ids, then the node ids, as little-endian uint32);
* ``pairs1_sha256``: SHA-256 of the concatenated per-top-node digests;
* the closest hits by ray id: SHA-256 of the triangle ids (int32) and of the
  bit patterns of t, u and v (float32), plus the hit count.

Usage: python tests/golden/make_fullsize.py [refl_1024] [mixed_1080p] [--jobs N]
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O            # noqa: E402
from workloads import make_workload       # noqa: E402

_G = {}


def _subtree(i):
    """Traversal and closest hits of top node i (runs in a worker)."""
    wl, h, ids, tree, tsph = _G["wl"], _G["h"], _G["ids"], _G["tree"], _G["tsph"]
    t0 = time.perf_counter()
    tr = O.traverse(tree, wl.scene, top_subset=np.array([i], np.uint32), tsph=tsph)
    t1 = time.perf_counter()
    stages = {}
    hits = O.closest_hit(h["rays"], ids, wl.B, tr["pairs"][1], wl.scene, wl.t_min, stages=stages)
    t2 = time.perf_counter()
    nl = tree["n_levels"]
    span = wl.B * wl.F ** (nl - 1)
    pos = np.arange(i * span, min((i + 1) * span, h["n"]))
    rid = ids[pos]
    p1t, p1n = tr["pairs"][1]
    dig = hashlib.sha256(np.ascontiguousarray(p1t, "<u4").tobytes() + np.ascontiguousarray(p1n, "<u4").tobytes())
    return {"i": i, "tests": tr["tests"], "hits": tr["hits"], "mesh_tests": tr["mesh_tests"],
            "mesh_hits": tr["mesh_hits"], "final_tests": tr["final_tests"], "u_pass": stages["u"],
            "uv_pass": stages["uv"], "n1": int(len(p1t)),
            "sha": dig.hexdigest(), "rid": rid, "hit": [a[rid] for a in hits],
            "sec_traverse": t1 - t0, "sec_hit": t2 - t1}


def digest(a, dt):
    return hashlib.sha256(np.ascontiguousarray(a).view(dt).astype(dt.newbyteorder("<")).tobytes()).hexdigest()


def make(name, jobs, out_dir):
    t0 = time.perf_counter()
    wl = make_workload(name)
    h = O.hash_rays(wl)
    ks, ids = O.sort_rays(h["keys"], h["ids"])
    tree = O.build_tree(h["rays"], ids, wl.B, wl.F, wl.n)
    tsph = O.tri_spheres(wl.scene)
    nl = tree["n_levels"]
    ntop = int(tree["level_cnt"][nl - 1])
    print(f"[golden] {name}: {h['n']} rays, {nl} levels, {ntop} top nodes ({time.perf_counter() - t0:.1f} s)",
          flush=True)
    _G.update(wl=wl, h=h, ids=ids, tree=tree, tsph=tsph)
    n = h["n"]
    tri = np.full(n, -1, np.int32)
    t, u, v = (np.zeros(n, np.float32) for _ in range(3))
    tests = {lv: 0 for lv in range(1, nl + 1)}
    hits = {lv: 0 for lv in range(1, nl + 1)}
    tot = {"mesh_tests": 0, "mesh_hits": 0, "final_tests": 0, "u_pass": 0, "uv_pass": 0}
    per_top = []
    secs = []
    ctx = mp.get_context("fork")
    with ctx.Pool(jobs) as pool:
        for r in pool.imap(_subtree, range(ntop), chunksize=1):
            for lv in tests:
                tests[lv] += r["tests"][lv]
                hits[lv] += r["hits"][lv]
            for k in tot:
                tot[k] += r[k]
            tri[r["rid"]], t[r["rid"]], u[r["rid"]], v[r["rid"]] = r["hit"]
            per_top.append({"n1": r["n1"], "sha": r["sha"]})
            secs.append((r["sec_traverse"], r["sec_hit"]))
            if r["i"] % 32 == 0:
                print(f"[golden] {name}: top node {r['i']} of {ntop}", flush=True)
    chain = hashlib.sha256("".join(p["sha"] for p in per_top).encode()).hexdigest()
    out = {
        "workload": name, "seed": 0, "rays": n, "triangles": wl.scene.m, "B": wl.B, "F": wl.F,
        "levels": nl, "top_nodes": ntop,
        "tests": [tests[lv] for lv in range(1, nl + 1)],
        "hits": [hits[lv] for lv in range(1, nl + 1)],
        **tot,
        "pairs1_sha256": chain,
        "per_top": per_top,
        "hit_count": int((tri >= 0).sum()),
        "hit_tri_sha256": digest(tri, np.dtype(np.int32)),
        "hit_t_sha256": digest(t, np.dtype(np.uint32)),
        "hit_u_sha256": digest(u, np.dtype(np.uint32)),
        "hit_v_sha256": digest(v, np.dtype(np.uint32)),
        "oracle_seconds": {"traverse": round(sum(s[0] for s in secs), 1), "hit": round(sum(s[1] for s in secs), 1)},
        "written_by": "tests/golden/make_fullsize.py (oracle only)",
    }
    path = os.path.join(out_dir, f"fullsize_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"[golden] {name}: wrote {path} in {time.perf_counter() - t0:.1f} s", flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("names", nargs="*", default=["refl_1024", "mixed_1080p"])
    ap.add_argument("--jobs", type=int, default=min(len(os.sched_getaffinity(0)), 16))
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args()
    for name in a.names:
        make(name, a.jobs, a.out)


if __name__ == "__main__":
    main()
