"""ctypes binding of libcrsh.so: the C-ABI of ``include/crsh.h`` under the same
names.  Argument marshalling only -- every step runs in the HIP kernels.

Device memory comes from torch tensors (``tensor.data_ptr()``) and streams
from ``torch.cuda.current_stream().cuda_stream``; nothing here computes.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# CRSH_LIBRARY may name another build of the same library (e.g. a variant
# built with different compile-time tile sizes); the default is in-tree.
LIB_PATH = os.environ.get("CRSH_LIBRARY") or os.path.join(HERE, "libcrsh.so")

MAX_LEVELS = 16
MAX_LIGHTS = 4
MAX_BUNDLE = 32
MAX_MERGE = 16
MAX_FRAMES = 256

OK, ERR_INVALID, ERR_CAPACITY, ERR_HIP = 0, 1, 2, 3
OVERFLOW_RAYS, OVERFLOW_NODES, OVERFLOW_PAIRS, OVERFLOW_ITEMS, OVERFLOW_PACKED = 1, 2, 4, 8, 16
PACKED_TRI_BITS = 14
PACKED_MAX_TRIS = 1 << PACKED_TRI_BITS
PACKED_MAX_NODES = 1 << (32 - PACKED_TRI_BITS)
RAY_SHADOW, RAY_REFLECT, RAY_REFRACT = 1, 2, 4
KEY_TYPE_ONLY = 0x100
KEY_SPHERICAL = 0x200

vp = C.c_void_p


class CrshError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"crsh status {status}: {msg}")
        self.status = status


class Meta(C.Structure):
    _fields_ = [("n_rays", C.c_uint32), ("n_levels", C.c_uint32),
                ("level_off", C.c_uint32 * MAX_LEVELS), ("level_cnt", C.c_uint32 * MAX_LEVELS),
                ("status", C.c_uint32), ("reserved", C.c_uint32),
                ("pairs", C.c_uint64 * MAX_LEVELS), ("hits", C.c_uint64 * MAX_LEVELS),
                ("tests", C.c_uint64 * MAX_LEVELS),
                ("mesh_tests", C.c_uint64), ("mesh_hits", C.c_uint64), ("final_tests", C.c_uint64),
                ("rays_required", C.c_uint64), ("nodes_required", C.c_uint64),
                ("final_u_pass", C.c_uint64), ("final_uv_pass", C.c_uint64)]


class Gbuf(C.Structure):
    _fields_ = [("px", vp), ("py", vp), ("pz", vp), ("nx", vp), ("ny", vp), ("nz", vp), ("mat", vp),
                ("w", C.c_int32), ("h", C.c_int32)]


class Raygen(C.Structure):
    _fields_ = [("n_lights", C.c_int32), ("lights", (C.c_float * 3) * MAX_LIGHTS), ("eye", C.c_float * 3),
                ("mat_flags", vp), ("mat_ior", vp), ("n_mats", C.c_int32), ("ray_types", C.c_uint32),
                ("eps_off", C.c_float), ("eps_shadow", C.c_float),
                ("lo", C.c_float * 3), ("inv_ext", C.c_float * 3)]


class Rays(C.Structure):
    _fields_ = [("ox", vp), ("oy", vp), ("oz", vp), ("dx", vp), ("dy", vp), ("dz", vp), ("tmax", vp),
                ("pix", vp), ("capacity", C.c_uint32)]


class Nodes(C.Structure):
    _fields_ = [(k, vp) for k in ("cx", "cy", "cz", "r", "ax", "ay", "az", "c", "s", "tan", "sec")] + \
               [("capacity", C.c_uint32)]


class Scene(C.Structure):
    _fields_ = [("v", vp * 9), ("m", C.c_uint32), ("mesh_first", vp), ("mesh_count", vp), ("msph", vp),
                ("n_mesh", C.c_uint32)]


class Pairs(C.Structure):
    _fields_ = [("tri", vp), ("node", vp), ("capacity", C.c_uint64)]


class PackedPairs(C.Structure):
    _fields_ = [("pair", vp), ("capacity", C.c_uint64)]


class Hits(C.Structure):
    _fields_ = [("tkey", vp), ("tri", vp), ("t", vp), ("u", vp), ("v", vp), ("capacity", C.c_uint32)]


PairTable = Pairs * MAX_LEVELS
PackedPairTable = PackedPairs * MAX_LEVELS


class Frame(C.Structure):
    _fields_ = [("pix_begin", C.c_uint32), ("pix_count", C.c_uint32),
                ("mesh_begin", C.c_uint32), ("mesh_count", C.c_uint32),
                ("mat_begin", C.c_uint32), ("n_mats", C.c_uint32),
                ("n_lights", C.c_int32), ("ray_types", C.c_uint32),
                ("lights", (C.c_float * 3) * MAX_LIGHTS), ("eye", C.c_float * 3),
                ("eps_off", C.c_float), ("eps_shadow", C.c_float), ("t_min", C.c_float),
                ("lo", C.c_float * 3), ("inv_ext", C.c_float * 3)]


class FrameMeta(C.Structure):
    _fields_ = [("ray_begin", C.c_uint32), ("n_rays", C.c_uint32), ("n_levels", C.c_uint32),
                ("reserved", C.c_uint32),
                ("level_base", C.c_uint32 * MAX_LEVELS), ("level_cnt", C.c_uint32 * MAX_LEVELS),
                ("item_base", C.c_uint64)]


class Batch(C.Structure):
    _fields_ = [("n_frames", C.c_uint32), ("frames", vp), ("frame_meta", vp), ("gbuf", Gbuf),
                ("mat_flags", vp), ("mat_ior", vp), ("scene", Scene), ("rays", Rays), ("sorted", Rays),
                ("keys", vp), ("ids", vp), ("skeys", vp), ("sids", vp), ("ray_frame", vp),
                ("nodes", Nodes), ("pairs", PairTable), ("hits", Hits), ("meta", vp),
                ("top_item_capacity", C.c_uint64), ("ws", vp), ("ws_bytes", C.c_size_t),
                ("bundle", C.c_int32), ("merge", C.c_int32), ("levels", C.c_int32), ("hit_block", C.c_int32),
                ("leaf_hit", C.c_int32)]

_lib = None


def lib():
    """The loaded library; raises if it was not built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2312_06538_amd/build.py "
                               "(the CRSH path runs only in its HIP kernels)")
        # torch ships its own HIP runtime under the same soname; load it first so
        # that libcrsh.so binds to that one runtime (one set of streams and memory)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        L.crsh_last_error.restype = C.c_char_p
        L.crsh_last_error.argtypes = []
        L.crsh_workspace_size.restype = C.c_size_t
        L.crsh_workspace_size.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]
        L.crsh_meta_reset.restype = st
        L.crsh_meta_reset.argtypes = [vp, vp]
        L.crsh_read_meta.restype = st
        L.crsh_read_meta.argtypes = [vp, C.POINTER(Meta), vp]
        L.crsh_hash.restype = st
        L.crsh_hash.argtypes = [C.POINTER(Gbuf), C.POINTER(Raygen), C.POINTER(Rays), vp, vp, vp, vp,
                                C.c_size_t, vp]
        L.crsh_hash_static.restype = st
        L.crsh_hash_static.argtypes = [C.POINTER(Gbuf), C.POINTER(Raygen), C.POINTER(Rays), vp, vp, vp, vp]
        L.crsh_bounce.restype = st
        L.crsh_bounce.argtypes = [C.POINTER(Rays), vp, C.POINTER(Hits), vp, C.POINTER(Scene), vp, C.POINTER(Raygen),
                                  C.POINTER(Rays), vp, vp, vp, vp, C.c_size_t, vp]
        L.crsh_sort.restype = st
        L.crsh_sort.argtypes = [vp, vp, vp, vp, C.c_uint32, vp, vp, C.c_size_t, vp]
        L.crsh_sort_chunked.restype = st
        L.crsh_sort_chunked.argtypes = [vp, vp, vp, vp, C.c_uint32, vp, vp, C.c_size_t, vp]
        L.crsh_build.restype = st
        L.crsh_build.argtypes = [C.POINTER(Rays), vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Nodes),
                                 C.POINTER(Rays), vp, vp]
        L.crsh_traverse.restype = st
        L.crsh_traverse.argtypes = [C.POINTER(Nodes), C.POINTER(Scene), C.c_uint32, C.c_uint32, C.c_int32,
                                    C.c_int32, PairTable, vp, vp, C.c_size_t, vp]
        L.crsh_traverse_packed.restype = st
        L.crsh_traverse_packed.argtypes = [C.POINTER(Nodes), C.POINTER(Scene), C.c_uint32, C.c_uint32, C.c_int32,
                                           C.c_int32, PackedPairTable, vp, vp, C.c_size_t, vp]
        L.crsh_closest_hit_packed.restype = st
        L.crsh_closest_hit_packed.argtypes = [C.POINTER(Rays), vp, C.c_int32, C.POINTER(PackedPairs), C.c_uint32,
                                              C.POINTER(Scene), C.c_float, C.POINTER(Hits), vp, vp, C.c_size_t, vp]
        L.crsh_traverse_upper.restype = st
        L.crsh_traverse_upper.argtypes = [C.POINTER(Nodes), C.POINTER(Scene), C.c_uint32, C.c_uint32, C.c_int32,
                                          C.c_int32, PairTable, vp, vp, C.c_size_t, vp]
        L.crsh_leaf_hit.restype = st
        L.crsh_leaf_hit.argtypes = [C.POINTER(Rays), vp, C.c_int32, C.c_int32, C.POINTER(Nodes), PairTable,
                                    C.POINTER(Scene), C.c_float, C.POINTER(Hits), vp, vp, C.c_size_t, vp]
        L.crsh_hits_reset.restype = st
        L.crsh_hits_reset.argtypes = [C.POINTER(Hits), vp]
        L.crsh_hash_rays.restype = st
        L.crsh_hash_rays.argtypes = [C.POINTER(Rays), C.c_uint32, C.c_uint32, C.c_uint32, C.c_float * 3,
                                     C.c_float * 3, vp, vp, vp, vp]
        L.crsh_gather_triangles.restype = st
        L.crsh_gather_triangles.argtypes = [vp, C.c_uint32, vp, C.c_uint32, vp * 9, vp]
        L.crsh_mesh_spheres.restype = st
        L.crsh_mesh_spheres.argtypes = [vp * 9, C.c_uint32, vp, vp, C.c_uint32, vp, vp]
        L.crsh_closest_hit_backward.restype = st
        L.crsh_closest_hit_backward.argtypes = [C.POINTER(Rays), C.c_uint32, C.POINTER(Hits), vp, vp, vp, vp,
                                                C.c_uint32, vp, C.c_uint32, vp, vp, vp, vp]
        L.crsh_profile_next.restype = st
        L.crsh_profile_next.argtypes = [C.c_char_p, C.c_int32, vp, vp]
        L.crsh_batch_ws_size.restype = C.c_size_t
        L.crsh_batch_ws_size.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64]
        L.crsh_batch_enqueue.restype = st
        L.crsh_batch_enqueue.argtypes = [C.POINTER(Batch), vp]
        L.crsh_batch_graph_create.restype = st
        L.crsh_batch_graph_create.argtypes = [C.POINTER(Batch), vp, C.POINTER(vp)]
        L.crsh_graph_launch.restype = st
        L.crsh_graph_launch.argtypes = [vp, vp]
        L.crsh_graph_destroy.restype = None
        L.crsh_graph_destroy.argtypes = [vp]
        L.crsh_closest_hit.restype = st
        L.crsh_closest_hit.argtypes = [C.POINTER(Rays), vp, C.c_int32, C.POINTER(Pairs), C.POINTER(Scene),
                                       C.c_float, C.POINTER(Hits), vp, vp, C.c_size_t, vp]
        _lib = L
    return _lib


def last_error():
    return lib().crsh_last_error().decode()


def _check(status, allow_capacity=False):
    if status == OK or (allow_capacity and status == ERR_CAPACITY):
        return status
    raise CrshError(status, last_error())


def crsh_workspace_size(max_rays, max_tris, max_meshes, max_nodes, max_pairs):
    return int(lib().crsh_workspace_size(max_rays, max_tris, max_meshes, max_nodes, max_pairs))


def crsh_meta_reset(meta, stream):
    return _check(lib().crsh_meta_reset(meta, stream))


def crsh_read_meta(meta, stream, allow_capacity=True):
    out = Meta()
    st = lib().crsh_read_meta(meta, C.byref(out), stream)
    _check(st, allow_capacity=allow_capacity)
    return out, st


def crsh_hash(gbuf, raygen, rays, keys, ids, meta, ws, ws_bytes, stream):
    return _check(lib().crsh_hash(C.byref(gbuf), C.byref(raygen), C.byref(rays), keys, ids, meta, ws, ws_bytes,
                                  stream))


def crsh_hash_static(gbuf, raygen, rays, keys, ids, meta, stream):
    return _check(lib().crsh_hash_static(C.byref(gbuf), C.byref(raygen), C.byref(rays), keys, ids, meta, stream))


def crsh_bounce(parents, parent_keys, hits, parent_meta, scene, tri_mat, raygen, out, keys, ids, meta, ws, ws_bytes,
                stream):
    return _check(lib().crsh_bounce(C.byref(parents), parent_keys, C.byref(hits), parent_meta, C.byref(scene),
                                    tri_mat, C.byref(raygen), C.byref(out), keys, ids, meta, ws, ws_bytes, stream))


def crsh_sort(keys_in, ids_in, keys_out, ids_out, capacity, meta, ws, ws_bytes, stream):
    return _check(lib().crsh_sort(keys_in, ids_in, keys_out, ids_out, capacity, meta, ws, ws_bytes, stream))


def crsh_sort_chunked(keys_in, ids_in, keys_out, ids_out, capacity, meta, ws, ws_bytes, stream):
    return _check(lib().crsh_sort_chunked(keys_in, ids_in, keys_out, ids_out, capacity, meta, ws, ws_bytes,
                                          stream))


def crsh_build(rays, sorted_ids, bundle, merge, levels, nodes, sorted_rays, meta, stream):
    return _check(lib().crsh_build(C.byref(rays), sorted_ids, bundle, merge, levels, C.byref(nodes),
                                   C.byref(sorted_rays), meta, stream))


def crsh_traverse(nodes, scene, tri_begin, tri_end, bundle, merge, pairs, meta, ws, ws_bytes, stream):
    return _check(lib().crsh_traverse(C.byref(nodes), C.byref(scene), tri_begin, tri_end, bundle, merge, pairs,
                                      meta, ws, ws_bytes, stream))


def crsh_traverse_packed(nodes, scene, tri_begin, tri_end, bundle, merge, pairs, meta, ws, ws_bytes, stream):
    return _check(lib().crsh_traverse_packed(C.byref(nodes), C.byref(scene), tri_begin, tri_end, bundle, merge,
                                             pairs, meta, ws, ws_bytes, stream))


def crsh_closest_hit_packed(sorted_rays, sorted_ids, bundle, level1, tri_begin, scene, t_min, hits, meta, ws,
                            ws_bytes, stream):
    return _check(lib().crsh_closest_hit_packed(C.byref(sorted_rays), sorted_ids, bundle, C.byref(level1),
                                                tri_begin, C.byref(scene), t_min, C.byref(hits), meta, ws,
                                                ws_bytes, stream))


def crsh_traverse_upper(nodes, scene, tri_begin, tri_end, bundle, merge, pairs, meta, ws, ws_bytes, stream):
    return _check(lib().crsh_traverse_upper(C.byref(nodes), C.byref(scene), tri_begin, tri_end, bundle, merge,
                                            pairs, meta, ws, ws_bytes, stream))


def crsh_leaf_hit(sorted_rays, sorted_ids, bundle, merge, nodes, pairs, scene, t_min, hits, meta, ws, ws_bytes,
                  stream):
    return _check(lib().crsh_leaf_hit(C.byref(sorted_rays), sorted_ids, bundle, merge, C.byref(nodes), pairs,
                                      C.byref(scene), t_min, C.byref(hits), meta, ws, ws_bytes, stream))


def crsh_hits_reset(hits, stream):
    return _check(lib().crsh_hits_reset(C.byref(hits), stream))


def crsh_closest_hit(sorted_rays, sorted_ids, bundle, level1, scene, t_min, hits, meta, ws, ws_bytes, stream):
    return _check(lib().crsh_closest_hit(C.byref(sorted_rays), sorted_ids, bundle, C.byref(level1),
                                         C.byref(scene), t_min, C.byref(hits), meta, ws, ws_bytes, stream))


def crsh_profile_next(kernel, occurrence, start_event, stop_event):
    """Arm the one-shot timer; events are hipEvent_t handles (torch.cuda.Event.cuda_event)."""
    return _check(lib().crsh_profile_next(kernel.encode(), occurrence, start_event, stop_event))


def crsh_hash_rays(rays, n, typ, light, lo, inv_ext, keys, ids, meta, stream):
    lo3 = (C.c_float * 3)(*[float(x) for x in lo])
    inv3 = (C.c_float * 3)(*[float(x) for x in inv_ext])
    return _check(lib().crsh_hash_rays(C.byref(rays), n, typ, light, lo3, inv3, keys, ids, meta, stream))


def crsh_gather_triangles(verts, n_verts, faces, m, v9, stream):
    return _check(lib().crsh_gather_triangles(verts, n_verts, faces, m, (vp * 9)(*v9), stream))


def crsh_mesh_spheres(v9, m, mesh_first, mesh_count, n_mesh, msph, stream):
    return _check(lib().crsh_mesh_spheres((vp * 9)(*v9), m, mesh_first, mesh_count, n_mesh, msph, stream))


def crsh_closest_hit_backward(rays, n, hits, g_t, g_u, g_v, verts, n_verts, faces, m, g_verts, g_o, g_d, stream):
    return _check(lib().crsh_closest_hit_backward(C.byref(rays), n, C.byref(hits), g_t, g_u, g_v, verts, n_verts,
                                                  faces, m, g_verts, g_o, g_d, stream))


def crsh_batch_ws_size(max_rays, max_tris, max_nodes, max_pairs, max_top_items):
    return int(lib().crsh_batch_ws_size(max_rays, max_tris, max_nodes, max_pairs, max_top_items))


def crsh_batch_enqueue(batch, stream):
    return _check(lib().crsh_batch_enqueue(C.byref(batch), stream))


def crsh_batch_graph_create(batch, stream):
    g = vp()
    _check(lib().crsh_batch_graph_create(C.byref(batch), stream, C.byref(g)))
    return g


def crsh_graph_launch(graph, stream):
    return _check(lib().crsh_graph_launch(graph, stream))


def crsh_graph_destroy(graph):
    lib().crsh_graph_destroy(graph)


def ctypes_sizeof_meta():
    return C.sizeof(Meta)
