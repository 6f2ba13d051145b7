#!/usr/bin/env python3
"""Benchmark of the CRSH secondary-ray path on one MI355X.

A step is one whole frame of the path -- hash, sort, build, traverse,
closest hit -- by default over the 1920x1080 workload with two lights and
shadow, reflection and refraction rays (256 procedural meshes in 8 clusters
plus the room, 482,048 triangles, 6.2M secondary rays, B=16 F=4 n=6), with
every input resident in HBM before timing starts.  Prints one JSON line:
secondary rays/s, the ray-triangle test counts against brute force N x M,
the roofline of the dominant kernel (timed with HIP events on its own
launches) and the plain CPU oracle timed on a bounded sample of the same
frame.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak of the dominant kernel's bound.  The final ray-triangle test is plain
# float32 VALU arithmetic without fused multiply-add or packed math: one
# operation per lane per cycle, 64 lanes per CU (4 SIMD x 16), 256 CUs,
# 2.4 GHz -> 39.3 T operations/s.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic float32 operations of the Moller-Trumbore test as written
# (Sec. 3.3.8), with its early exits: every test computes p = D x e2 (9),
# det = e1 . p (5), checks |det| (1), 1 / det (1), T = O - v0 (3), u (a dot
# product 5 and the scaling 1) and checks its two bounds (2): 27 operations;
# a test whose u passes adds q = T x e1 (9), v (6) and its checks (v >= 0,
# u + v, <= 1: 3): 18 more; a test whose u and v pass adds t (6) and its two
# bounds (2): 8 more.  The kernels count the tests that pass u and those that
# pass u and v (crsh_meta.final_u_pass / final_uv_pass).  e1 and e2 are
# per-triangle precomputation, not per-test work; a test failing the
# determinant check (a ray parallel to the plane, a vanishing share) is
# counted as if it reached the u check.
MT_OPS_ALL, MT_OPS_U, MT_OPS_UV = 27, 18, 8
# float32 operations of one node-sphere test (Eq. 9) as written: P - C (3),
# t = (P-C).a (5), (P-C) x a (9), its squared length (5),
# |t| tan + (d + r) sec (4: two products, two sums), squaring (1),
# comparison (1), the full-cone check (1).
NODE_OPS = 29
HBM_PEAK_GBS = 8000.0
# MI355X's published float32 vector peak, which counts a fused multiply-add
# as two operations and packed float32 as two lanes
PUBLISHED_FP32_TFLOPS = 157.3


# HBM traffic of the dominant kernel per launch, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE; calibrated against a copy of known size).
# The summary records a hash of the kernel's source files; a figure taken
# before the sources changed is not reported.
TRAFFIC_PROFILES = "profiles/*_hbm_traffic_*.md"
TRAFFIC_SOURCES = {"k_hit": ["paper_2312_06538_amd/csrc/hit.hip", "paper_2312_06538_amd/csrc/intersect.hpp",
                             "paper_2312_06538_amd/csrc/batch.hpp", "paper_2312_06538_amd/csrc/common.hpp",
                             "include/crsh.h"]}


def sources_sha256(kernel):
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """(bytes per launch, note) from a traffic summary, or (None, why)."""
    import glob
    stale = False
    for path in sorted(glob.glob(os.path.join(ROOT, TRAFFIC_PROFILES))):
        for ln in open(path).read().splitlines():
            if not ln.startswith("bench-traffic:"):
                continue
            kv = dict(f.split("=", 1) for f in ln.split()[1:])
            if kv.get("kernel") != kernel or kv.get("workload") != workload:
                continue
            if kv.get("sources") != sources_sha256(kernel):
                stale = True
                continue
            return int(kv["bytes"]), f"rocprofv3 FETCH_SIZE + WRITE_SIZE, {os.path.basename(path)}"
    return None, ("counters predate the kernel's current sources" if stale
                  else "no counters for this kernel and workload")


def hip():
    return ctypes.CDLL("libamdhip64.so.7")


class HipEvents:
    def __init__(self, n):
        self.h = hip()
        self.ev = []
        for _ in range(2 * n):
            e = ctypes.c_void_p()
            assert self.h.hipEventCreate(ctypes.byref(e)) == 0
            self.ev.append(e)

    def pair(self, i):
        return self.ev[2 * i], self.ev[2 * i + 1]

    def ms(self, i):
        a, b = self.pair(i)
        out = ctypes.c_float()
        assert self.h.hipEventSynchronize(b) == 0
        if self.h.hipEventElapsedTime(ctypes.byref(out), a, b) != 0:
            return None
        return out.value


_CPU = {}


def _cpu_subtrees(top_nodes):
    """Oracle traversal + final tests of the listed top-level sub-trees (one
    task).  Runs in a forked worker or in the calling process; returns the
    seconds it took."""
    from oracle import oracle as O
    import numpy as np
    wl, h, ids, tree, tsph = (_CPU[k] for k in ("wl", "h", "ids", "tree", "tsph"))
    t0 = time.perf_counter()
    for i in top_nodes:
        tr = O.traverse(tree, wl.scene, top_subset=np.array([i], np.uint32), tsph=tsph)
        O.closest_hit(h["rays"], ids, wl.B, tr["pairs"][1], wl.scene, wl.t_min)
    return time.perf_counter() - t0


def host_cores(max_cores=16):
    """Host threads for process pools: the affinity mask, at most the share
    of the host that one GPU gets."""
    return max(1, min(len(os.sched_getaffinity(0)), max_cores))


def cpu_baseline(wl, n_sample_top=64, n_sample_one=4, max_cores=16):
    """The oracle as it stands (sequential C, never tuned) on the host's
    cores.  Hash, sort and build run over the whole frame in one process.
    Traversal and final tests -- by far the larger part -- run over an evenly
    spread sample of top-level sub-trees, which are independent, one
    sub-tree per task in a pool of one forked process per core (at most
    `max_cores`, the share of the host a single GPU gets); the pool's wall
    time, scaled to the whole frame by the share of rays under the sample,
    gives the multi-core rate.  The one-core rate adds up the sample's
    per-task times instead, corrected by how much slower a few of its
    sub-trees ran in the pool than alone in this process afterwards.  Must
    run before this process initialises the GPU (the pool forks)."""
    import multiprocessing as mp
    import numpy as np
    from oracle import oracle as O
    t = {}
    t0 = time.perf_counter()
    h = O.hash_rays(wl)
    t["hash"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ks, ids = O.sort_rays(h["keys"], h["ids"])
    t["sort"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    tree = O.build_tree(h["rays"], ids, wl.B, wl.F, wl.n)
    t["build"] = time.perf_counter() - t0
    tsph = O.tri_spheres(wl.scene)
    _CPU.update(wl=wl, h=h, ids=ids, tree=tree, tsph=tsph)
    nl = tree["n_levels"]
    ntop = int(tree["level_cnt"][nl - 1])
    span = wl.B * wl.F ** (nl - 1)
    rays_under = lambda sub: int(sum(min(span, h["n"] - int(i) * span) for i in sub))
    hsb = t["hash"] + t["sort"] + t["build"]
    cores = host_cores(max_cores)
    sub = [int(i) for i in np.unique(np.linspace(0, ntop - 1, min(n_sample_top, ntop)).astype(np.int64))]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        # one sub-tree per task, handed out as workers free up (sub-trees
        # differ in cost by two orders of magnitude)
        task_s = pool.map(_cpu_subtrees, [[i] for i in sub], chunksize=1)
    t["pool_sample"] = time.perf_counter() - t0
    scale = h["n"] / max(rays_under(sub), 1)
    frame_pool = hsb + t["pool_sample"] * scale
    # one core: the same sample's task times, with the pool's slowdown
    # measured on a few of its sub-trees (spread over the sample) run alone
    pick = sorted(set(int(k) for k in np.linspace(0, len(sub) - 1, min(n_sample_one, len(sub))).astype(np.int64)))
    alone = sum(_cpu_subtrees([sub[k]]) for k in pick)
    in_pool = sum(task_s[k] for k in pick)
    slowdown = in_pool / alone if alone > 0 else 1.0
    t["one_sample"] = alone
    t["sample_cpu"] = sum(task_s)
    frame_one = hsb + sum(task_s) / slowdown * scale
    _CPU.clear()
    return {"value": round(h["n"] / frame_pool, 1), "unit": "secondary rays/s", "cores": cores, "kind": "oracle",
            "sample": (f"hash+sort+build of the whole frame ({h['n']} rays, one process), then traversal and final "
                       f"tests of {len(sub)} of {ntop} top-level sub-trees ({rays_under(sub)} rays) on {cores} "
                       f"forked processes, scaled by {scale:.2f} to the frame"),
            "one_core": {"value": round(h["n"] / frame_one, 1),
                         "sample": (f"the same {len(sub)} sub-trees' task times in the pool divided by the pool's "
                                    f"slowdown {slowdown:.2f} (measured on {len(pick)} of them run alone)")},
            "seconds": {k: round(v, 3) for k, v in t.items()},
            "est_frame_s": round(frame_pool, 2), "est_frame_s_one_core": round(frame_one, 2)}


def ray_label(wl):
    """The workload's ray types as generated: shadow rays per light, then
    reflection and refraction rays."""
    from workloads import SHADOW, REFLECT, REFRACT
    parts = []
    if wl.ray_types & SHADOW:
        nl = len(wl.lights)
        parts.append("shadow" if nl == 1 else f"shadow x{nl} lights")
    if wl.ray_types & REFLECT:
        parts.append("reflection")
    if wl.ray_types & REFRACT:
        parts.append("refraction")
    return "+".join(parts) or "no rays"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed_1080p",
                    choices=["shadow_128", "refl_1024", "mixed_1080p", "adjoint_512", "batch_64"])
    ap.add_argument("--pairs", default="arrays", choices=["arrays", "packed"],
                    help="pair storage: two uint32 arrays, or one packed word per pair over triangle batches of "
                         "at most 2^14 triangles (crsh_traverse_packed)")
    ap.add_argument("--last-level", default="stored", choices=["stored", "fused"],
                    help="fused: the level-1 node tests and the final tests in crsh_leaf_hit, the level-1 pairs "
                         "never stored (crsh_traverse_upper + crsh_leaf_hit)")
    ap.add_argument("--variant", default="crsh", choices=["crsh", "unsorted"],
                    help="unsorted: the comparison hierarchy without ray sorting or whole-mesh culling, on the "
                         "same inputs and with the same hierarchy shape")
    ap.add_argument("--size", default=None, help="WxH: the workload's scene and camera at another resolution")
    ap.add_argument("--bundle", type=int, default=None, help="rays per leaf (B) instead of the workload's")
    ap.add_argument("--merge", type=int, default=None, help="children per node (F) instead of the workload's")
    ap.add_argument("--levels", type=int, default=None, help="hierarchy levels (n) instead of the workload's")
    ap.add_argument("--frames", type=int, default=64, help="batch_64: number of frames")
    ap.add_argument("--sort-sweep", action="store_true",
                    help="instead of a frame: crsh_sort on 2^20..2^27 random keys, GB/s per radix pass")
    ap.add_argument("--tune", action="store_true",
                    help="batch_64: tune (B, levels, hit_block) by timing the captured batch")
    ap.add_argument("--tune-cache", default=None, help="batch_64: JSON cache of tuned points")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched form's figures (64 frames as one captured batch against the same frames "
                         "through the plain calls) that follow the measurement of the frame (taken only with the "
                         "workload's own shape and the crsh variant)")
    ap.add_argument("--cpu-sample-top", type=int, default=128,
                    help="top-level sub-trees the oracle traverses in the process pool")
    ap.add_argument("--cpu-sample-one", type=int, default=4,
                    help="sub-trees of the sample the oracle also traverses alone, for the one-core rate")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, one device copy of this size: calibrates HBM counters under rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the split of the path over several "
              "GPUs (rays sharded by image band or frame, scene replicated) is not built", file=sys.stderr)
        return 2

    if args.sort_sweep:
        return bench_sort_sweep(args)
    if args.workload == "batch_64":
        return bench_batch(args)

    from workloads import make_workload

    t0 = time.perf_counter()
    kw = {}
    if args.size:
        kw["W"], kw["H"] = (int(x) for x in args.size.lower().split("x"))
    for k, v in (("B", args.bundle), ("F", args.merge), ("n", args.levels)):
        if v is not None:
            kw[k] = v
    wl = make_workload(args.workload, seed=args.seed, **kw)
    if args.variant == "unsorted":
        from workloads import unsorted_variant
        wl = unsorted_variant(wl)
    print(f"[bench] workload {args.workload}: {wl.W}x{wl.H}, M={wl.scene.m}, built in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    # the oracle's leg first: its process pool forks, which must happen
    # before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(wl, args.cpu_sample_top, args.cpu_sample_one)
        print(f"[bench] oracle baseline in {time.perf_counter() - t0:.1f}s: {cpu['value']:.0f} rays/s on "
              f"{cpu['cores']} cores", file=sys.stderr, flush=True)

    # the batched form's frames, built in a process pool, also before the GPU
    wls = None
    reshaped = args.size or args.variant != "crsh" or any(v is not None for v in (args.bundle, args.merge, args.levels))
    if not args.no_batch and not reshaped:
        from workloads.scenes import make_batch
        t0 = time.perf_counter()
        wls = make_batch(args.seed, args.frames, jobs=host_cores())
        print(f"[bench] batch of {len(wls)} frames built in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
              flush=True)

    import torch
    from paper_2312_06538_amd import crsh as X
    from paper_2312_06538_amd import pipeline as P

    fr = P.DeviceFrame(wl)
    bf = P.Buffers(fr, 1 << 24, keep_levels=False)
    packed = args.pairs == "packed"
    fused = args.last_level == "fused"
    bf, m = P.run_with_retry(fr, bf, packed=packed, leaf_hit=fused)
    print(f"[bench] sized: N={m.n_rays} levels={m.n_levels} pair capacity={bf.pair_capacity}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        P.run_frame(fr, bf, packed=packed, leaf_hit=fused)
    torch.cuda.synchronize()
    ev = HipEvents(args.steps)
    # kernels timed on alternate steps: the two heaviest (the final tests and
    # the level pass that forms level 1, the last k_level launch of a frame)
    # and the sort and compaction kernels measured against HBM bandwidth (the
    # second radix pass, the emit that writes level 1)
    nl = int(m.n_levels)
    # (fused last level: the first k_hit launch tests the level-1 pairs a
    # top-level pass stored, none here; the second is the fused one, and no
    # emit writes level 1)
    probes = [("k_hit", 1 if fused else 0), ("k_level", max(nl - 2, 0)), ("k_sort_pass", 1)]
    if not fused:
        probes.append(("k_level_emit", max(nl - 2, 0)))
    t0 = time.perf_counter()
    for k in range(args.steps):
        a, b = ev.pair(k)
        name, occ = probes[k % len(probes)]
        if not packed:           # packed: one launch per triangle batch, no single kernel to time
            X.crsh_profile_next(name, occ, a, b)
        P.run_frame(fr, bf, packed=packed, leaf_hit=fused)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m, st = P.read_meta(bf)
    assert st == X.OK, X.last_error()
    durs = {}
    for k in range(0 if packed else args.steps):
        v = ev.ms(k)
        if v is not None:
            durs.setdefault(probes[k % len(probes)][0], []).append(v)
    ms_step = (t1 - t0) / args.steps * 1e3
    n = int(m.n_rays)
    nl = int(m.n_levels)
    node_tests = sum(int(m.tests[k]) for k in range(nl))
    final = int(m.final_tests)
    brute = n * wl.scene.m
    kern = {}
    u_pass, uv_pass = int(m.final_u_pass), int(m.final_uv_pass)
    work = {"k_hit": final * MT_OPS_ALL + u_pass * MT_OPS_U + uv_pass * MT_OPS_UV,
            "k_level": int(m.tests[0]) * NODE_OPS}
    for name in work:
        if durs.get(name):
            avg = sum(durs[name]) / len(durs[name])
            tops = work[name] / (avg * 1e-3) / 1e12
            kern[name] = {"bound": "alu", "achieved": round(tops, 3), "peak": round(ALU_PEAK_TOPS, 1),
                          "unit": "TOP/s", "frac": round(tops / ALU_PEAK_TOPS, 4), "traffic": None,
                          "frac_of_published_fp32": round(tops / PUBLISHED_FP32_TFLOPS, 4),
                          "kernel": name, "kernel_ms": round(avg, 4), "ops_per_launch": work[name],
                          "launches_timed": len(durs[name])}
    dom = max(kern, key=lambda k: kern[k]["kernel_ms"]) if kern else None
    roof = kern.get(dom)
    if roof is not None and dom in TRAFFIC_SOURCES:
        roof["traffic"], roof["traffic_source"] = measured_traffic(dom, args.workload + ("" if args.variant == "crsh"
                                                                                           else "_" + args.variant))
    other = {k: v for k, v in kern.items() if k != dom}
    # HBM kernels: algorithmic bytes per launch.  Sort pass: key + id read
    # and written (16 B per key).  Level emit: the pass bits of every parent
    # pair (one per child slot: the merge factor rounded up to a power of
    # two), each parent pair with a survivor read (8 B, at most min(in, out)
    # of them) and every output pair written (8 B).
    n_in = int(m.hits[1]) if nl >= 2 else 0
    n_out = int(m.hits[0])
    nf = 1 << (wl.F - 1).bit_length()
    hbm_bytes = {"k_sort_pass": 16 * n, "k_level_emit": n_in * nf // 8 + 8 * min(n_in, n_out) + 8 * n_out}
    hbm = {}
    for name, nbytes in hbm_bytes.items():
        if durs.get(name) and nbytes:
            avg = sum(durs[name]) / len(durs[name])
            gbs = nbytes / (avg * 1e-3) / 1e9
            hbm[name] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "kernel_ms": round(avg, 4), "bytes_per_launch": nbytes,
                         "launches_timed": len(durs[name])}
    out = {
        "metric": "secondary rays/sec (hash+sort+build+traverse+hit); ray-tri tests vs brute N×M",
        "value": round(n / (ms_step * 1e-3), 1),
        "unit": "secondary rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.W}x{wl.H} {ray_label(wl)}, "
                               f"{wl.scene.n_mesh} meshes, {wl.scene.m} triangles, B={wl.B} F={wl.F} n={wl.n}",
                   "rays": n, "triangles": wl.scene.m, "seed": args.seed, "variant": args.variant,
                   "pairs": args.pairs, "last_level": args.last_level},
        "tests": {"node_tests": node_tests, "final_ray_tri_tests": final, "final_u_pass": u_pass,
                  "final_uv_pass": uv_pass, "total": node_tests + final,
                  "brute_force": brute, "frac_of_brute": round((node_tests + final) / brute, 5),
                  "mesh_tests": int(m.mesh_tests), "levels": nl},
        "roofline": roof,
        "other_kernels": other,
        "hbm_kernels": hbm,
    }
    if args.copy_probe_mib:
        n4 = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 4 * n4
    if cpu is not None:
        out["cpu_baseline"] = cpu
    rc = 0
    if wls is not None:
        # the batched form, after the headline frame's buffers are released
        del bf, fr
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        bt = measure_batch(args, wls)
        out["batch_64"] = {"value": bt["value"], "unit": bt["unit"], "ms_per_batch": bt["ms_per_step"],
                           "per_frame_plain": bt["per_frame_plain"], "config": bt["config"], "tests": bt["tests"]}
        if not bt["per_frame_plain"]["same_closest_hits"]:
            rc = 1
    print(json.dumps(out), flush=True)
    return rc


def bench_sort_sweep(args):
    """crsh_sort alone on uniformly random 32-bit keys (no digit pass
    skipped) from 2^20 to 2^27 keys: the sizes past the 256 MiB last-level
    cache show the HBM rate.  Bytes per radix pass: key and id read and
    written (16 B per key)."""
    import torch
    from paper_2312_06538_amd import crsh as X
    from paper_2312_06538_amd import pipeline as P

    rows = []
    ev = HipEvents(2)
    h = ev.h
    for lg in range(20, 28):
        n = 1 << lg
        g = torch.Generator(device="cuda").manual_seed(args.seed + lg)
        keys = torch.randint(-(1 << 31), (1 << 31) - 1, (n,), dtype=torch.int32, device="cuda", generator=g)
        ids = torch.arange(n, dtype=torch.int32, device="cuda")
        ko, io = torch.empty_like(keys), torch.empty_like(ids)
        meta = torch.zeros(ctypes.sizeof(X.Meta), dtype=torch.uint8, device="cuda")
        meta[:4] = torch.tensor([n], dtype=torch.int32).view(torch.uint8).cuda()
        wsb = X.crsh_workspace_size(n, 1, 1, 1, 1)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        s = P.stream_handle()
        call = lambda: X.crsh_sort(keys.data_ptr(), ids.data_ptr(), ko.data_ptr(), io.data_ptr(), n,
                                   meta.data_ptr(), ws.data_ptr(), wsb, s)
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        pass_ms = []
        whole = []
        for k in range(args.steps):
            a, b = ev.pair(0)
            X.crsh_profile_next("k_sort_pass", k % 4, a, b)
            c, d = ev.pair(1)
            h.hipEventRecord(c, ctypes.c_void_p(s))
            call()
            h.hipEventRecord(d, ctypes.c_void_p(s))
            torch.cuda.synchronize()
            pass_ms.append(ev.ms(0))
            whole.append(ev.ms(1))
        pm = sum(pass_ms) / len(pass_ms)
        wm = sorted(whole)[len(whole) // 2]
        # whole sort per pass: every kernel of the sort (digit histograms,
        # plan, and per pass the upsweep and digit scan where used) charged
        # to the four passes
        sp = wm / 4
        rows.append({"keys": n, "pass_ms": round(pm, 4), "pass_GBs": round(16 * n / (pm * 1e-3) / 1e9, 1),
                     "pass_frac": round(16 * n / (pm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "sort_ms": round(wm, 4),
                     "sort_Mkeys_s": round(n / (wm * 1e-3) / 1e6, 1),
                     "sort_per_pass_GBs": round(16 * n / (sp * 1e-3) / 1e9, 1),
                     "sort_per_pass_frac": round(16 * n / (sp * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        print(f"[bench] sort 2^{lg}: pass kernel {pm:.4f} ms, {rows[-1]['pass_GBs']} GB/s; whole sort {wm:.4f} ms, "
              f"{rows[-1]['sort_per_pass_GBs']} GB/s per pass", file=sys.stderr, flush=True)
        del keys, ids, ko, io, ws
    print(json.dumps({"metric": "crsh_sort radix pass bandwidth (16 B per key per pass)", "unit": "GB/s",
                      "peak": HBM_PEAK_GBS, "steps": args.steps, "rows": rows}), flush=True)
    return 0


def measure_batch(args, wls=None):
    """Batched form: `frames` independent frames (log-uniform sizes) as one
    captured batch, against the same frames one after the other through the
    plain calls with the same hierarchy shape.  Returns the JSON record; its
    `per_frame_plain.same_closest_hits` says whether the two forms found the
    same closest hits (bits of t, u, v included)."""
    import dataclasses

    import torch
    from workloads.scenes import make_batch
    from paper_2312_06538_amd import crsh as X
    from paper_2312_06538_amd import pipeline as P
    from paper_2312_06538_amd import tune as T
    from paper_2312_06538_amd.batch import DeviceBatch

    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    if wls is None:
        t0 = time.perf_counter()
        wls = make_batch(args.seed, args.frames, jobs=host_cores())
        log(f"[bench] batch of {len(wls)} frames built in {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.Stream()
    p = dict(T.START)
    db = DeviceBatch(wls, p["B"], 4, p["levels"], p["hit_block"], pair_capacity=1 << 24)
    tuned = "default"
    if args.tune or args.tune_cache:
        cache = T.TuneCache(args.tune_cache) if args.tune_cache else None
        best, ms, seen = T.tune_batch(db, stream, cache=cache, log=log)
        p = best
        tuned = f"tuned over {len(seen)} points" if seen else "from cache"
    m = db.run_with_retry()
    n = int(m.n_rays)
    g = db.graph(stream)
    for _ in range(args.warmup):
        g.launch()
    stream.synchronize()
    ev = HipEvents(1)
    a, b = ev.pair(0)
    h = ev.h
    t0 = time.perf_counter()
    h.hipEventRecord(a, ctypes.c_void_p(stream.cuda_stream))
    for _ in range(args.steps):
        g.launch()
    h.hipEventRecord(b, ctypes.c_void_p(stream.cuda_stream))
    stream.synchronize()
    t1 = time.perf_counter()
    ms_batch = ev.ms(0) / args.steps
    m2, st = db.read_meta(stream)
    assert st == X.OK, X.last_error()
    g.close()
    log(f"[bench] batch: {n} rays, {ms_batch:.3f} ms per batch ({p})")
    # the same frames one by one through the plain calls (pre-sized, no host
    # synchronisation between frames), the same B / F / levels
    plain = []
    for wl in wls:
        w2 = dataclasses.replace(wl, B=p["B"], F=4, n=p["levels"])
        fr = P.DeviceFrame(w2)
        bf = P.Buffers(fr, 1 << 20)
        bf, _ = P.run_with_retry(fr, bf)
        plain.append((fr, bf))
    for _ in range(args.warmup):
        for fr, bf in plain:
            P.run_frame(fr, bf)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream().cuda_stream
    h.hipEventRecord(a, ctypes.c_void_p(cur))
    for _ in range(args.steps):
        for fr, bf in plain:
            P.run_frame(fr, bf)
    h.hipEventRecord(b, ctypes.c_void_p(cur))
    torch.cuda.synchronize()
    ms_plain = ev.ms(0) / args.steps
    n_plain = sum(int(P.read_meta(bf)[0].n_rays) for _, bf in plain)
    assert n_plain == n
    # the two forms must find the same closest hits: triangle ids and the
    # bits of t, u, v, frame by frame
    import numpy as np
    batch_res = db.frame_results(m2, with_pairs=False)
    same = True
    for f, ((fr, bf), r) in enumerate(zip(plain, batch_res)):
        pm, _ = P.read_meta(bf)
        res = P.results(fr, bf, pm)
        for x, y in zip(res["hit"], r["hit"]):
            if not np.array_equal(np.asarray(x).view(np.uint32), np.asarray(y).view(np.uint32)):
                same = False
                log(f"[bench] frame {f}: batched and plain closest hits differ")
                break
    tris = sum(wl.scene.m for wl in wls)
    out = {
        "metric": "secondary rays/sec (hash+sort+build+traverse+hit), batched frames",
        "value": round(n / (ms_batch * 1e-3), 1),
        "unit": "secondary rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_batch, 4),
        "host_ms_per_step": round((t1 - t0) / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch_64: {len(wls)} frames, rays per frame log-uniform in [4096, 1M], "
                               f"triangles per frame log-uniform in [1000, 200000], shadow+reflection",
                   "rays": n, "triangles": tris, "B": p["B"], "F": 4, "levels": p["levels"],
                   "hit_block": p["hit_block"], "params": tuned, "seed": args.seed},
        "per_frame_plain": {"ms_per_batch": round(ms_plain, 4), "value": round(n / (ms_plain * 1e-3), 1),
                            "speedup_of_batch": round(ms_plain / ms_batch, 3), "same_closest_hits": same},
        "tests": {"final_ray_tri_tests": int(m2.final_tests),
                  "node_tests": sum(int(m2.tests[k]) for k in range(int(m2.n_levels)))},
    }
    return out


def bench_batch(args):
    out = measure_batch(args)
    print(json.dumps(out), flush=True)
    return 0 if out["per_frame_plain"]["same_closest_hits"] else 1


if __name__ == "__main__":
    sys.exit(main())
