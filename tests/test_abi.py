"""The C-ABI library without a GPU: it loads, exports every entry point that
include/crsh.h declares, its ctypes mirrors match the C layouts, and
argument errors are reported on the host before anything is launched."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2312_06538_amd import crsh as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crsh.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(crsh_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = X.lib()
    names = declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.check_output(["nm", "-D", "--defined-only", X.LIB_PATH]).decode()
    exported = set(re.findall(r" T (crsh_\w+)", out))
    assert set(names) <= exported


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "crsh.h"
#define S(t) printf(#t " %zu\n", sizeof(t));
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f));
int main(void) {
  S(crsh_meta) O(crsh_meta, status) O(crsh_meta, pairs) O(crsh_meta, hits) O(crsh_meta, tests)
  O(crsh_meta, final_tests) O(crsh_meta, nodes_required) O(crsh_meta, final_u_pass) O(crsh_meta, final_uv_pass)
  S(crsh_gbuf) O(crsh_gbuf, mat) O(crsh_gbuf, w)
  S(crsh_raygen) O(crsh_raygen, mat_flags) O(crsh_raygen, ray_types) O(crsh_raygen, inv_ext)
  S(crsh_rays) O(crsh_rays, pix) O(crsh_rays, capacity)
  S(crsh_nodes) O(crsh_nodes, sec) O(crsh_nodes, capacity)
  S(crsh_scene) O(crsh_scene, m) O(crsh_scene, msph) O(crsh_scene, n_mesh)
  S(crsh_pairs) O(crsh_pairs, capacity)
  S(crsh_packed_pairs) O(crsh_packed_pairs, capacity)
  S(crsh_hits) O(crsh_hits, v) O(crsh_hits, capacity)
  S(crsh_frame) O(crsh_frame, n_lights) O(crsh_frame, lights) O(crsh_frame, eye) O(crsh_frame, t_min)
  O(crsh_frame, inv_ext)
  S(crsh_frame_meta) O(crsh_frame_meta, level_base) O(crsh_frame_meta, level_cnt) O(crsh_frame_meta, item_base)
  S(crsh_batch) O(crsh_batch, gbuf) O(crsh_batch, scene) O(crsh_batch, rays) O(crsh_batch, sorted)
  O(crsh_batch, ray_frame) O(crsh_batch, nodes) O(crsh_batch, pairs) O(crsh_batch, hits) O(crsh_batch, meta)
  O(crsh_batch, top_item_capacity) O(crsh_batch, ws_bytes) O(crsh_batch, hit_block)
  return 0;
}
"""


def test_ctypes_layouts_match_header(tmp_path):
    c = tmp_path / "layout.c"
    c.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(c), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    mirror = {"crsh_meta": X.Meta, "crsh_gbuf": X.Gbuf, "crsh_raygen": X.Raygen, "crsh_rays": X.Rays,
              "crsh_nodes": X.Nodes, "crsh_scene": X.Scene, "crsh_pairs": X.Pairs,
              "crsh_packed_pairs": X.PackedPairs, "crsh_hits": X.Hits,
              "crsh_frame": X.Frame, "crsh_frame_meta": X.FrameMeta, "crsh_batch": X.Batch}
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(mirror[t], f).offset == int(val), key
        else:
            assert ctypes.sizeof(mirror[key]) == int(val), key


def test_invalid_arguments_are_rejected_on_the_host():
    L = X.lib()
    assert L.crsh_meta_reset(None, None) == X.ERR_INVALID
    assert "NULL" in X.last_error()
    r = X.Rays(*([1] * 8), 100)
    n = X.Nodes(*([1] * 11), 100)
    # bundle 0 / merge 1 / levels 0
    for B, F, lv in ((0, 4, 4), (8, 1, 4), (8, 4, 0), (33, 4, 4), (8, 17, 4), (8, 4, 17)):
        st = L.crsh_build(ctypes.byref(r), 1, B, F, lv, ctypes.byref(n), ctypes.byref(r), 1, None)
        assert st == X.ERR_INVALID, (B, F, lv)
    assert "bundle" in X.last_error()
    # sort: aliasing, oversized capacity, small workspace
    assert L.crsh_sort(8, 16, 8, 24, 10, 1, 1, 1 << 30, None) == X.ERR_INVALID
    assert L.crsh_sort(8, 16, 32, 24, 1 << 30, 1, 1, 1 << 40, None) == X.ERR_INVALID
    assert L.crsh_sort(8, 16, 32, 24, 1000, 1, 1, 10, None) == X.ERR_INVALID
    assert "workspace" in X.last_error()
    # hash: empty primary-hit buffer
    g = X.Gbuf(*([1] * 7), 0, 4)
    rg = X.Raygen()
    assert L.crsh_hash(ctypes.byref(g), ctypes.byref(rg), ctypes.byref(r), 1, 1, 1, 1, 1 << 20, None) == \
        X.ERR_INVALID
    # traverse: triangle batch outside the scene
    sc = X.Scene((X.vp * 9)(*([1] * 9)), 10, 1, 1, 1, 1)
    pt = X.PairTable()
    pt[0] = X.Pairs(1, 1, 10)
    assert L.crsh_traverse(ctypes.byref(n), ctypes.byref(sc), 5, 11, 8, 4, pt, 1, 1, 1 << 30, None) == \
        X.ERR_INVALID
    assert "batch" in X.last_error()
    # packed pairs: a triangle batch over 2^14 triangles, a batch outside the scene
    big = X.Scene((X.vp * 9)(*([1] * 9)), 1 << 20, 1, 1, 1, 1)
    pp = X.PackedPairTable()
    pp[0] = X.PackedPairs(1, 10)
    assert L.crsh_traverse_packed(ctypes.byref(n), ctypes.byref(big), 0, X.PACKED_MAX_TRIS + 1, 8, 4, pp, 1, 1,
                                  1 << 30, None) == X.ERR_INVALID
    assert "at most" in X.last_error()
    assert L.crsh_traverse_packed(ctypes.byref(n), ctypes.byref(sc), 5, 11, 8, 4, pp, 1, 1, 1 << 30, None) == \
        X.ERR_INVALID
    assert "batch" in X.last_error()
    assert L.crsh_closest_hit_packed(ctypes.byref(r), 1, 8, None, 0, ctypes.byref(sc), ctypes.c_float(1e-4),
                                     None, 1, 1, 1 << 30, None) == X.ERR_INVALID
    # closest hit: bundle out of range
    h = X.Hits(1, 1, 1, 1, 1, 100)
    assert L.crsh_closest_hit(ctypes.byref(r), 1, 0, ctypes.byref(pt[0]), ctypes.byref(sc), ctypes.c_float(1e-4),
                              ctypes.byref(h), 1, 1, 1 << 30, None) == X.ERR_INVALID
    # fused last level: level-1 storage without capacity, merge factor 1, no level-2 table, small workspace
    lt = X.PairTable()
    lt[0] = X.Pairs(1, 1, 0)
    lt[1] = X.Pairs(1, 1, 10)
    assert L.crsh_leaf_hit(ctypes.byref(r), 1, 8, 4, ctypes.byref(n), lt, ctypes.byref(sc), ctypes.c_float(1e-4),
                           ctypes.byref(h), 1, 1, 1 << 30, None) == X.ERR_INVALID
    assert "level-1" in X.last_error()
    lt[0] = X.Pairs(1, 1, 10)
    assert L.crsh_leaf_hit(ctypes.byref(r), 1, 8, 1, ctypes.byref(n), lt, ctypes.byref(sc), ctypes.c_float(1e-4),
                           ctypes.byref(h), 1, 1, 1 << 30, None) == X.ERR_INVALID
    assert "merge" in X.last_error()
    assert L.crsh_leaf_hit(ctypes.byref(r), 1, 8, 4, ctypes.byref(n), lt, ctypes.byref(sc), ctypes.c_float(1e-4),
                           ctypes.byref(h), 1, 1, 16, None) == X.ERR_INVALID
    assert "workspace" in X.last_error()
    lt[1] = X.Pairs(0, 0, 0)
    assert L.crsh_leaf_hit(ctypes.byref(r), 1, 8, 4, ctypes.byref(n), lt, ctypes.byref(sc), ctypes.c_float(1e-4),
                           ctypes.byref(h), 1, 1, 1 << 30, None) == X.ERR_INVALID
    assert "level-2" in X.last_error()
    assert L.crsh_profile_next(None, 0, 1, 1) == X.ERR_INVALID


def _dummy_batch(**kw):
    b = X.Batch()
    b.n_frames, b.frames, b.frame_meta = 2, 1, 1
    b.gbuf = X.Gbuf(*([1] * 7), 64, 1)
    b.mat_flags = b.mat_ior = b.keys = b.ids = b.skeys = b.sids = b.ray_frame = b.meta = b.ws = 1
    b.rays = X.Rays(*([1] * 8), 100)
    b.sorted = X.Rays(*([1] * 8), 100)
    b.nodes = X.Nodes(*([1] * 11), 100)
    b.scene = X.Scene((X.vp * 9)(*([1] * 9)), 10, 1, 1, 1, 1)
    for k in range(4):
        b.pairs[k] = X.Pairs(1, 1, 100)
    b.hits = X.Hits(1, 1, 1, 1, 1, 100)
    b.top_item_capacity = 100
    b.ws_bytes = 1 << 30
    b.bundle, b.merge, b.levels, b.hit_block = 8, 4, 4, 256
    for k, v in kw.items():
        setattr(b, k, v)
    return b


def test_invalid_batches_are_rejected_on_the_host():
    L = X.lib()
    bad = [dict(n_frames=0), dict(n_frames=X.MAX_FRAMES + 1), dict(frames=None), dict(ray_frame=None),
           dict(levels=5), dict(levels=0), dict(levels=17), dict(hit_block=32), dict(bundle=0), dict(merge=1),
           dict(ws_bytes=1000)]
    for kw in bad:
        b = _dummy_batch(**kw)
        assert L.crsh_batch_enqueue(ctypes.byref(b), None) == X.ERR_INVALID, kw
    assert "workspace" in X.last_error()
    g = X.vp()
    b = _dummy_batch(levels=5)
    assert L.crsh_batch_graph_create(ctypes.byref(b), None, ctypes.byref(g)) == X.ERR_INVALID
    assert not g.value
    assert L.crsh_graph_launch(None, None) == X.ERR_INVALID
    L.crsh_graph_destroy(None)


def test_batch_workspace_grows_with_every_bound():
    base = X.crsh_batch_ws_size(1 << 16, 1000, 1 << 12, 1 << 16, 1 << 12)
    for args in ((1 << 17, 1000, 1 << 12, 1 << 16, 1 << 12), (1 << 16, 100000, 1 << 12, 1 << 16, 1 << 12),
                 (1 << 16, 1000, 1 << 16, 1 << 16, 1 << 12), (1 << 16, 1000, 1 << 12, 1 << 20, 1 << 12),
                 (1 << 16, 1000, 1 << 12, 1 << 16, 1 << 22)):
        assert X.crsh_batch_ws_size(*args) > base, args


def test_workspace_size_covers_every_stage():
    a = X.crsh_workspace_size(1 << 20, 1000, 10, 1 << 16, 1 << 20)
    b = X.crsh_workspace_size(1 << 21, 1000, 10, 1 << 16, 1 << 20)
    assert b > a > (1 << 20) * 8


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(X, "_lib", None)
    monkeypatch.setattr(X, "LIB_PATH", "/nonexistent/libcrsh.so")
    with pytest.raises(RuntimeError, match="missing"):
        X.lib()
