"""GPU parity of the batched form: every frame of a batch gets exactly the
oracle's products for that frame alone (keys, sorted order, nodes, every
pair level, closest hits) and the batch counters are the sums of the
frames' counters.  The batch mixes frames of different sizes (so their
hierarchies have different top levels, down to a single leaf), light
counts, ray types and materials, and a frame whose pixels all missed.
A captured hipGraph replays to the same products as the eager launch."""
import dataclasses

import numpy as np
import pytest

from conftest import workload
from oracle import oracle as O

pytestmark = pytest.mark.gpu

B, F, N = 16, 4, 5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _shape(wl, **kw):
    return dataclasses.replace(wl, B=kw.get("B", B), F=kw.get("F", F), n=kw.get("n", N))


def _missed(wl):
    g = dict(wl.gbuf)
    g["mat"] = np.full_like(np.asarray(g["mat"]), -1)
    return dataclasses.replace(wl, gbuf=g)


_FRAMES = {}


def frames(**kw):
    key = tuple(sorted(kw.items()))
    if key not in _FRAMES:
        _FRAMES[key] = _make_frames(**kw)
    return _FRAMES[key]


def _make_frames(**kw):
    from workloads.scenes import make_frame
    f0 = make_frame(11, 6000, 3000)
    return [_shape(f0, **kw),
            _shape(workload("shadow_128", W=40, H=40), **kw),
            _shape(make_frame(12, 80, 1200), **kw),                 # a few leaves: low top level
            _shape(workload("mixed_1080p", W=64, H=40, n_meshes=24), **kw),
            _shape(_missed(f0), **kw),                              # no rays at all
            _shape(make_frame(13, 20000, 5000), **kw),
            _shape(workload("shadow_128", W=3, H=3), **kw)]          # one leaf: top is level 1


_ORC = {}


def oracle_of(wl):
    key = id(wl)
    if key not in _ORC:
        _ORC[key] = (wl, O.run_pipeline(wl, tri_batches=None))
    return _ORC[key][1]


def _bits(a):
    a = np.asarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def check_frame(got, wl, orc, all_levels):
    h = orc["hash"]
    n = h["n"]
    assert got["n"] == n
    assert np.array_equal(got["keys"], h["keys"])
    assert np.array_equal(got["ids"], h["ids"])
    for k in O.RAY_FIELDS:
        assert np.array_equal(_bits(got["rays"][k]), _bits(h["rays"][k])), k
    assert np.array_equal(got["sorted_keys"], orc["sorted_keys"])
    assert np.array_equal(got["sorted_ids"], orc["sorted_ids"])
    tree = orc["tree"]
    assert got["n_levels"] == tree["n_levels"]
    assert np.array_equal(got["level_cnt"], tree["level_cnt"][:tree["n_levels"]])
    for k in O.NODE_FIELDS:
        assert np.array_equal(_bits(got["nodes"][k]), _bits(tree["nodes"][k])), k
    tr = orc["trav"]
    levels = range(1, tree["n_levels"] + 1) if all_levels else [1] if tree["n_levels"] else []
    for lv in levels:
        t, nd = got["pairs"][lv]
        assert np.array_equal(t, tr["pairs"][lv][0]), lv
        assert np.array_equal(nd, tr["pairs"][lv][1]), lv
    hits = orc["hits"]
    assert np.array_equal(got["hit"][0], hits[0])
    for a, b in zip(got["hit"][1:], hits[1:]):
        assert np.array_equal(_bits(a), _bits(b))


def _counters(orcs):
    tot = {"mesh_tests": 0, "mesh_hits": 0, "final_tests": 0, "tests": {}, "hits": {}, "u": 0, "uv": 0}
    for o in orcs:
        tr = o["trav"]
        tot["mesh_tests"] += tr["mesh_tests"]
        tot["mesh_hits"] += tr["mesh_hits"]
        tot["final_tests"] += tr["final_tests"]
        tot["u"] += o.get("stages", {}).get("u", 0)
        tot["uv"] += o.get("stages", {}).get("uv", 0)
        for lv, v in tr["tests"].items():
            tot["tests"][lv] = tot["tests"].get(lv, 0) + v
        for lv, (t, _) in tr["pairs"].items():
            tot["hits"][lv] = tot["hits"].get(lv, 0) + len(t)
    return tot


@pytest.mark.parametrize("hit_block", [64, 256])
def test_batch_matches_oracle_per_frame(hit_block):
    from paper_2312_06538_amd.batch import DeviceBatch
    wls = frames()
    print(f"[batch] {len(wls)} frames, hit_block {hit_block}", flush=True)
    db = DeviceBatch(wls, B, F, N, hit_block=hit_block, pair_capacity=1 << 20, keep_levels=True, leaf_hit=False)
    m = db.run_with_retry()
    orcs = [oracle_of(wl) for wl in wls]
    res = db.frame_results(m)
    assert int(m.n_rays) == sum(o["hash"]["n"] for o in orcs)
    assert res[4]["n"] == 0 and res[4]["n_levels"] == 0
    assert sorted({r["n_levels"] for r in res}) == [0, 1, 3, N]   # every kind of top level
    for f, (r, wl, o) in enumerate(zip(res, wls, orcs)):
        print(f"[batch] frame {f}: {r['n']} rays, {r['n_levels']} levels", flush=True)
        check_frame(r, wl, o, all_levels=True)
    tot = _counters(orcs)
    assert int(m.mesh_tests) == tot["mesh_tests"]
    assert int(m.mesh_hits) == tot["mesh_hits"]
    assert int(m.final_tests) == tot["final_tests"]
    assert (int(m.final_u_pass), int(m.final_uv_pass)) == (tot["u"], tot["uv"])
    for lv, v in tot["tests"].items():
        assert int(m.tests[lv - 1]) == v, lv
    for lv, v in tot["hits"].items():
        assert int(m.hits[lv - 1]) == v, lv


def test_batch_large_ray_capacity_matches_oracle():
    """A ray capacity of several million slots: every launch (the sort's
    frame-digit pass included) is sized for the capacity while the frames
    stay small."""
    from paper_2312_06538_amd.batch import DeviceBatch
    wls = frames()
    db = DeviceBatch(wls, B, F, N, pair_capacity=1 << 20, leaf_hit=False, ray_capacity=(1 << 22) + 777)
    m = db.run_with_retry()
    for f, (r, wl) in enumerate(zip(db.frame_results(m), wls)):
        print(f"[batch large capacity] frame {f}: {r['n']} rays", flush=True)
        check_frame(r, wl, oracle_of(wl), all_levels=False)


def test_batch_fused_last_level_matches_oracle():
    """The batch with the last level fused with the final tests: closest
    hits per frame and the counters summed over frames."""
    from paper_2312_06538_amd.batch import DeviceBatch
    wls = frames()
    db = DeviceBatch(wls, B, F, N, pair_capacity=1 << 20, leaf_hit=True)
    m = db.run_with_retry()
    orcs = [oracle_of(wl) for wl in wls]
    for f, (r, o) in enumerate(zip(db.frame_results(m), orcs)):
        print(f"[batch fused] frame {f}: {r['n']} rays", flush=True)
        assert r["n"] == o["hash"]["n"]
        assert np.array_equal(r["hit"][0], o["hits"][0])
        for a, b in zip(r["hit"][1:], o["hits"][1:]):
            assert np.array_equal(_bits(a), _bits(b))
    tot = _counters(orcs)
    assert int(m.final_tests) == tot["final_tests"]
    for lv, v in tot["tests"].items():
        assert int(m.tests[lv - 1]) == v, lv
    for lv, v in tot["hits"].items():
        assert int(m.hits[lv - 1]) == v, lv


def test_batch_shapes_and_single_frame():
    """Other hierarchy shapes (bundle 8 / merge 2 / 3 levels, bundle 32 /
    merge 8 / 7 levels) and a batch of one frame."""
    from paper_2312_06538_amd.batch import DeviceBatch
    for (b, f, n) in ((8, 2, 3), (32, 8, 7)):
        wls = frames(B=b, F=f, n=n)[:4]
        print(f"[batch] shape B={b} F={f} n={n}", flush=True)
        db = DeviceBatch(wls, b, f, n, pair_capacity=1 << 20, leaf_hit=False)
        m = db.run_with_retry()
        for r, wl in zip(db.frame_results(m), wls):
            check_frame(r, wl, oracle_of(wl), all_levels=False)
    wl = frames()[5]
    db = DeviceBatch([wl], B, F, N, pair_capacity=1 << 20, leaf_hit=False)
    m = db.run_with_retry()
    check_frame(db.frame_results(m)[0], wl, oracle_of(wl), all_levels=False)


def test_batch_pair_overflow_regrows():
    from paper_2312_06538_amd.batch import DeviceBatch
    wls = frames()[:3]
    db = DeviceBatch(wls, B, F, N, pair_capacity=64, leaf_hit=False)
    m = db.run_with_retry()
    assert db.pair_capacity > 64
    for r, wl in zip(db.frame_results(m), wls):
        check_frame(r, wl, oracle_of(wl), all_levels=False)


def test_batch_graph_replays_match_eager():
    import torch
    from paper_2312_06538_amd.batch import DeviceBatch
    wls = frames()
    db = DeviceBatch(wls, B, F, N, pair_capacity=1 << 20)
    m = db.run_with_retry()            # sizes the pair arrays
    want = db.frame_results(m)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = db.graph(s)
    for rep in range(3):
        # the program's own eager work between replays
        db.hit_t.fill_(-1.0)
        db.sids.fill_(0)
        torch.cuda.synchronize()
        g.launch()
        m2, st = db.read_meta(s)
        assert st == 0
        got = db.frame_results(m2)
        print(f"[batch] graph replay {rep}", flush=True)
        for a, b in zip(got, want):
            assert a["n"] == b["n"]
            assert np.array_equal(a["sorted_ids"], b["sorted_ids"])
            for k in ("cx", "r", "c", "s"):
                assert np.array_equal(_bits(a["nodes"][k]), _bits(b["nodes"][k]))
            assert np.array_equal(a["pairs"][1][0], b["pairs"][1][0]) if 1 in b["pairs"] else True
            for x, y in zip(a["hit"], b["hit"]):
                assert np.array_equal(_bits(x), _bits(y))
    g.close()
