// Batched form: many independent frames through the five stages as one
// launch sequence (one launch per kernel for the whole batch), optionally
// captured into a hipGraph.
//
// The stage launchers are those of the plain entry points with the batch's
// device view: frame-aware kernels find their frame from per-frame bases
// (pixels, rays, nodes of each level, top-level items) and otherwise do what
// the plain kernels do, so every frame gets exactly its plain result.  The
// sort takes one more, most significant, digit: the ray's frame, which keeps
// each frame's rays together in the stable order of their keys.
//
// Workspace: per-node first ray / first child and count + frame (written by
// the build, read by the traversal and the final tests) and the top-level
// pass scalars stay for the whole batch; the stages share the rest, one after
// the other, as in the plain calls.
#include <algorithm>

#include "batch.hpp"

struct crsh_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace crsh {

struct batch_layout {
    size_t first, info, top, stage, total;
};

static batch_layout layout(uint32_t ray_cap, uint64_t pixels, uint32_t m, uint32_t node_cap, uint64_t max_pairs,
                           uint64_t top_items)
{
    batch_layout L;
    L.first = 0;
    L.info = L.first + align256((size_t)node_cap * 4 + 4);
    L.top = L.info + align256((size_t)node_cap * 4 + 4);
    L.stage = L.top + align256(2 * sizeof(uint64_t));
    size_t st = std::max(sort_ws_bytes(ray_cap), hash_ws_bytes(pixels));
    st = std::max(st, trav_ws_bytes(m, node_cap, top_items, max_pairs));
    const uint32_t slots = hit_slots(ray_cap, true);
    st = std::max(st, std::max(hit_ws_bytes(m, slots), leaf_hit_ws_bytes(m, node_cap, max_pairs, slots)));
    L.total = L.stage + st;
    return L;
}

__global__ void k_batch_clear(uint32_t *meta, uint32_t meta_words, uint32_t *fm, uint32_t fm_words,
                              unsigned long long *tkey, uint32_t n_tkey)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_tkey || i < meta_words || i < fm_words;
         i += stride) {
        if (i < meta_words) meta[i] = 0;
        if (i < fm_words) fm[i] = 0;
        if (i < n_tkey) tkey[i] = ~0ull;
    }
}

static crsh_status check_batch(const crsh_batch *b, batch_layout &L)
{
    if (!b) {
        set_error("crsh_batch: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (b->n_frames < 1 || b->n_frames > CRSH_MAX_FRAMES || !b->frames || !b->frame_meta) {
        set_error("crsh_batch: need 1..%d frames and their device tables", CRSH_MAX_FRAMES);
        return CRSH_ERR_INVALID;
    }
    if (!b->mat_flags || !b->mat_ior || !b->keys || !b->ids || !b->skeys || !b->sids || !b->ray_frame ||
        !b->meta || !b->ws || !b->hits.tkey) {
        set_error("crsh_batch: NULL array");
        return CRSH_ERR_INVALID;
    }
    if (b->levels < 1 || b->levels > CRSH_MAX_LEVELS || b->bundle < 1 || b->bundle > CRSH_MAX_BUNDLE ||
        b->merge < 2 || b->merge > CRSH_MAX_MERGE) {
        set_error("crsh_batch: bundle must be in [1, %d], merge in [2, %d], levels in [1, %d]", CRSH_MAX_BUNDLE,
                  CRSH_MAX_MERGE, CRSH_MAX_LEVELS);
        return CRSH_ERR_INVALID;
    }
    if (b->hit_block != 64 && b->hit_block != 128 && b->hit_block != 256) {
        set_error("crsh_batch: hit_block must be 64, 128 or 256");
        return CRSH_ERR_INVALID;
    }
    const crsh_gbuf &g = b->gbuf;
    const crsh_rays &r = b->rays, &s = b->sorted;
    const crsh_nodes &n = b->nodes;
    const crsh_scene &sc = b->scene;
    const crsh_hits &h = b->hits;
    bool arrays = g.px && g.py && g.pz && g.nx && g.ny && g.nz && g.mat;
    arrays = arrays && r.ox && r.oy && r.oz && r.dx && r.dy && r.dz && r.tmax && r.pix;
    arrays = arrays && s.ox && s.oy && s.oz && s.dx && s.dy && s.dz && s.tmax;
    arrays = arrays && n.cx && n.cy && n.cz && n.r && n.ax && n.ay && n.az && n.c && n.s && n.tan && n.sec;
    arrays = arrays && sc.mesh_first && sc.mesh_count && sc.msph && sc.n_mesh > 0;
    for (int k = 0; k < 9; ++k) arrays = arrays && (sc.v[k] || sc.m == 0);
    arrays = arrays && h.tri && h.t && h.u && h.v;
    if (!arrays) {
        set_error("crsh_batch: incomplete primary-hit, ray, node, scene or hit arrays");
        return CRSH_ERR_INVALID;
    }
    if (r.capacity >= (1u << 30)) {
        set_error("crsh_batch: ray capacity must stay below 2^30");
        return CRSH_ERR_INVALID;
    }
    if (b->hits.capacity < b->rays.capacity || b->sorted.capacity < b->rays.capacity) {
        set_error("crsh_batch: sorted-ray or hit capacity below the ray capacity");
        return CRSH_ERR_INVALID;
    }
    if (b->gbuf.w <= 0 || b->gbuf.h <= 0 || (uint64_t)b->gbuf.w * (uint64_t)b->gbuf.h >= (1ull << 31)) {
        set_error("crsh_batch: empty or oversized primary-hit buffer");
        return CRSH_ERR_INVALID;
    }
    uint64_t max_pairs = 0;
    for (int k = 0; k < b->levels; ++k) {
        if (!b->pairs[k].tri || !b->pairs[k].node) {
            set_error("crsh_batch: no pair storage for level %d", k + 1);
            return CRSH_ERR_INVALID;
        }
        max_pairs = std::max(max_pairs, b->pairs[k].capacity);
    }
    const uint64_t pixels = (uint64_t)b->gbuf.w * (uint64_t)b->gbuf.h;
    L = layout(b->rays.capacity, pixels, b->scene.m, b->nodes.capacity, max_pairs, b->top_item_capacity);
    if (b->ws_bytes < L.total) {
        set_error("crsh_batch: workspace too small (%zu < %zu)", b->ws_bytes, L.total);
        return CRSH_ERR_INVALID;
    }
    return CRSH_OK;
}

}  // namespace crsh

using namespace crsh;

extern "C" size_t crsh_batch_ws_size(uint32_t max_rays, uint32_t max_tris, uint32_t max_nodes, uint64_t max_pairs,
                                     uint64_t max_top_items)
{
    return layout(max_rays, max_rays, max_tris, max_nodes, max_pairs, max_top_items).total;
}

extern "C" crsh_status crsh_batch_enqueue(const crsh_batch *b, hipStream_t stream)
{
    batch_layout L;
    crsh_status st = check_batch(b, L);
    if (st != CRSH_OK) return st;
    char *ws = (char *)b->ws;
    batch_dev bd;
    bd.frames = b->frames;
    bd.fm = b->frame_meta;
    bd.n_frames = b->n_frames;
    bd.node_first = (uint32_t *)(ws + L.first);
    bd.node_info = (uint32_t *)(ws + L.info);
    bd.ray_frame = b->ray_frame;
    bd.top = (uint64_t *)(ws + L.top);
    bd.top_cap = b->top_item_capacity;
    bd.mat_flags = b->mat_flags;
    bd.mat_ior = b->mat_ior;
    void *stage = ws + L.stage;
    const size_t stage_bytes = b->ws_bytes - L.stage;

    const uint32_t meta_words = sizeof(crsh_meta) / 4;
    const uint32_t fm_words = b->n_frames * (uint32_t)(sizeof(crsh_frame_meta) / 4);
    const uint32_t n_clear = std::max(std::max(meta_words, fm_words), b->hits.capacity);
    k_batch_clear<<<std::max<uint32_t>(std::min<uint32_t>((n_clear + 255) / 256, 4096), 1), 256, 0, stream>>>(
        (uint32_t *)b->meta, meta_words, (uint32_t *)b->frame_meta, fm_words, b->hits.tkey, b->hits.capacity);
    if ((st = hip_check(hipGetLastError(), "crsh_batch clear")) != CRSH_OK) return st;

    crsh_rays rays = b->rays, sorted = b->sorted;
    st = hash_launch(&b->gbuf, nullptr, &bd, &rays, b->keys, b->ids, b->ray_frame, b->meta, stage, stage_bytes,
                     stream);
    if (st != CRSH_OK) return st;
    st = sort_launch(b->keys, b->ids, b->ray_frame, b->skeys, b->sids, b->rays.capacity, b->meta, stage,
                     stage_bytes, stream);
    if (st != CRSH_OK) return st;
    crsh_nodes nodes = b->nodes;
    st = build_launch(&rays, b->sids, b->bundle, b->merge, b->levels, &nodes, &sorted, b->meta, &bd, stream);
    if (st != CRSH_OK) return st;
    const int32_t lowest = b->leaf_hit ? 2 : 1;
    st = traverse_launch(&nodes, &b->scene, 0, b->scene.m, b->bundle, b->merge, b->pairs, b->meta, stage,
                         stage_bytes, &bd, b->levels, b->top_item_capacity, lowest, stream);
    if (st != CRSH_OK) return st;
    crsh_hits hits = b->hits;
    if (b->leaf_hit && b->levels >= 2)
        return leaf_hit_launch(&sorted, b->sids, b->bundle, b->merge, &nodes, &b->pairs[0], &b->pairs[1],
                               &b->scene, 0.0f, &hits, b->meta, stage, stage_bytes, &bd, b->hit_block,
                               (uint32_t)b->levels, stream);
    return hit_launch(&sorted, b->sids, b->bundle, &b->pairs[0], &b->scene, 0.0f, &hits, b->meta, stage,
                      stage_bytes, &bd, b->hit_block, stream);
}

extern "C" crsh_status crsh_batch_graph_create(const crsh_batch *b, hipStream_t stream, crsh_graph **out)
{
    if (!out) {
        set_error("crsh_batch_graph_create: NULL argument");
        return CRSH_ERR_INVALID;
    }
    *out = nullptr;
    batch_layout L;
    crsh_status st = check_batch(b, L);
    if (st != CRSH_OK) return st;
    if ((st = hip_check(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture")) !=
        CRSH_OK)
        return st;
    crsh_status enq = crsh_batch_enqueue(b, stream);
    hipGraph_t graph = nullptr;
    st = hip_check(hipStreamEndCapture(stream, &graph), "end capture");
    if (enq != CRSH_OK || st != CRSH_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return enq != CRSH_OK ? enq : st;
    }
    hipGraphExec_t exec = nullptr;
    if ((st = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate")) != CRSH_OK) {
        (void)hipGraphDestroy(graph);
        return st;
    }
    crsh_graph *g = new (std::nothrow) crsh_graph{graph, exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        set_error("crsh_batch_graph_create: out of host memory");
        return CRSH_ERR_INVALID;
    }
    *out = g;
    return CRSH_OK;
}

extern "C" crsh_status crsh_graph_launch(crsh_graph *g, hipStream_t stream)
{
    if (!g) {
        set_error("crsh_graph_launch: NULL graph");
        return CRSH_ERR_INVALID;
    }
    return hip_check(hipGraphLaunch(g->exec, stream), "graph launch");
}

extern "C" void crsh_graph_destroy(crsh_graph *g)
{
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}
