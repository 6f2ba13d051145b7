// The last traversal level fused with the final tests (Sec. 3.3.7 at level 1,
// Sec. 3.3.8).
//
// In stage order the level-2 pairs become level-1 pairs (triangle, leaf),
// which are written out, read back and tested ray by ray.  Here the level-1
// count pass of the traversal runs on the level-2 pairs (its pass bits, one
// per (parent pair, child), land in the workspace) and the final-test kernel
// reads the level-2 pairs with their pass bits instead of level-1 pairs,
// listing each run's (pair, child) items in LDS: the level-1 pairs are never
// stored, and neither the scan nor the emit of level 1 runs.  The counters
// are those of the stage order (level-1 node tests, level-1 pairs formed,
// ray-triangle tests and how far they got) and so are the closest hits (the
// same tests, the same minimum).  Level-1 pairs that a top-level pass wrote (a
// hierarchy whose top is level 1) go through the plain final-test kernel
// first.
#include "traverse.hpp"

namespace crsh {

struct lh_ws {
    float4 *tri;         // packed triangles (v0, e1, e2)
    hit_slots_ws hs;     // packed ray slots and their keys
    float4 *tsph;        // triangle bounding spheres
    float4 *na, *nb;     // packed nodes for the level-1 count
    float *ns;
    trav_scratch S;      // level-1 count: survivors per tile, pass bits
};

// tiles of the level-1 count over at most cap2 level-2 pairs
static uint64_t lh_tiles(uint64_t cap2) { return (cap2 + LEVEL_TILE - 1) / LEVEL_TILE; }

static lh_ws carve(void *ws, uint32_t m, uint32_t node_cap, uint64_t cap2, uint32_t slots)
{
    const uint64_t tiles = lh_tiles(cap2) + 1;
    char *w = (char *)ws;
    lh_ws L;
    L.tri = (float4 *)w;
    w += align256((size_t)m * 48);
    L.hs = carve_hit_slots(w, slots);
    w += hit_slots_bytes(slots);
    L.tsph = (float4 *)w;
    w += align256((size_t)m * 16);
    L.na = (float4 *)w;
    w += align256((size_t)node_cap * 16);
    L.nb = (float4 *)w;
    w += align256((size_t)node_cap * 16);
    L.ns = (float *)w;
    w += align256((size_t)node_cap * 4);
    L.S.cnt = (uint32_t *)w;
    w += align256(tiles * 4);
    L.S.off = nullptr;
    L.S.mask = (uint32_t *)w;
    w += align256(tiles * LEVEL_THREADS * 4 + 4);
    L.S.scan_flags = (uint64_t *)w;
    w += align256((tiles / SCAN_TILE + 2) * 8);
    L.S.scan_ctr = (uint32_t *)w;
    return L;
}

size_t leaf_hit_ws_bytes(uint32_t m, uint32_t node_cap, uint64_t cap2, uint32_t slots)
{
    const uint64_t tiles = lh_tiles(cap2) + 1;
    return align256((size_t)m * 48) + hit_slots_bytes(slots) + align256((size_t)m * 16) +
           align256((size_t)node_cap * 16) * 2 + align256((size_t)node_cap * 4) + align256(tiles * 4) +
           align256(tiles * LEVEL_THREADS * 4 + 4) + align256((tiles / SCAN_TILE + 2) * 8) + align256(4);
}

// level-1 pairs formed: the survivors of every tile of the level-1 count
__global__ void k_lh_survivors(trav_scratch S, crsh_meta *meta, uint64_t cap2)
{
    __shared__ uint64_t s_red[256 / WAVE];
    uint64_t nin = meta->n_levels >= 2 ? meta->pairs[1] : 0u;
    nin = nin < cap2 ? nin : cap2;
    const uint64_t ntiles = (nin + LEVEL_TILE - 1) / LEVEL_TILE;
    uint64_t sum = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntiles;
         i += (uint64_t)gridDim.x * blockDim.x)
        sum += S.cnt[i];
    sum = wave_sum(sum);
    if (lane_id() == 0) s_red[threadIdx.x / WAVE] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (uint32_t w = 0; w < blockDim.x / WAVE; ++w) t += s_red[w];
        if (t) atomicAdd((unsigned long long *)&meta->hits[0], (unsigned long long)t);
    }
}

crsh_status leaf_hit_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle, int32_t merge,
                            const crsh_nodes *nodes, const crsh_pairs *level1, const crsh_pairs *level2,
                            const crsh_scene *scene, float t_min, crsh_hits *hits, crsh_meta *meta, void *ws,
                            size_t ws_bytes, const batch_dev *bd, int32_t hit_block, uint32_t top_levels,
                            hipStream_t stream)
{
    crsh_status st = hit_check(sorted, sorted_ids, bundle, level1, scene, hits, meta, ws, hit_block,
                               "crsh_leaf_hit");
    if (st != CRSH_OK) return st;
    if (merge < 2 || merge > CRSH_MAX_MERGE || !nodes || !level2 || !level2->tri || !level2->node) {
        set_error("crsh_leaf_hit: bad merge factor or missing node / level-2 arrays");
        return CRSH_ERR_INVALID;
    }
    if (!nodes->cx || !nodes->cy || !nodes->cz || !nodes->r || !nodes->ax || !nodes->ay || !nodes->az ||
        !nodes->c || !nodes->tan || !nodes->sec) {
        set_error("crsh_leaf_hit: incomplete node arrays");
        return CRSH_ERR_INVALID;
    }
    if (!level1->tri || !level1->capacity) {
        set_error("crsh_leaf_hit: level-1 pair storage missing");
        return CRSH_ERR_INVALID;
    }
    const uint32_t slots = hit_slots(sorted->capacity, bd != nullptr);
    const size_t need = leaf_hit_ws_bytes(scene->m, nodes->capacity, level2->capacity, slots);
    if (ws_bytes < need) {
        set_error("crsh_leaf_hit: workspace too small (%zu < %zu)", ws_bytes, need);
        return CRSH_ERR_INVALID;
    }
    const lh_ws L = carve(ws, scene->m, nodes->capacity, level2->capacity, slots);
    hit_prep_launch(scene, L.tri, stream);
    tri_spheres_launch(scene, 0, scene->m, L.tsph, stream);
    node_pack_launch(nodes, meta, L.na, L.nb, L.ns, false, stream);
    // level-1 pairs stored by a top-level pass at level 1 (this also packs
    // the ray slots)
    hit_pairs_launch(sorted, L.tri, L.hs, level1, bundle, scene, t_min, hits, meta, bd, hit_block, stream);
    // the level-1 node tests: pass bits and survivors per tile, node tests
    // added to meta
    pair_levels P{};
    P.p[0] = pairs_dev{level1->tri, level1->node, level1->capacity, 0u, 0u};
    P.p[1] = pairs_dev{level2->tri, level2->node, level2->capacity, 0u, 0u};
    level_count_launch(2, merge, L.na, L.nb, L.ns, L.tsph, scene->m, P, L.S, meta, bd, lh_tiles(level2->capacity),
                       top_levels, stream, false);
    const uint32_t gs = (uint32_t)std::max<uint64_t>(std::min<uint64_t>((lh_tiles(level2->capacity) + 255) / 256,
                                                                        1024), 1);
    k_lh_survivors<<<gs, 256, 0, stream>>>(L.S, meta, level2->capacity);
    hit_masked_launch(sorted, L.tri, L.hs, level2, L.S.mask, merge, bundle, scene, t_min, hits, meta, bd,
                      hit_block, stream);
    hit_final_launch(sorted, sorted_ids, L.tri, L.hs, bundle, scene, t_min, hits, meta, bd, stream);
    return hip_check(hipGetLastError(), "crsh_leaf_hit launch");
}

}  // namespace crsh

using namespace crsh;

extern "C" crsh_status crsh_leaf_hit(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle,
                                     int32_t merge, const crsh_nodes *nodes,
                                     const crsh_pairs pairs[CRSH_MAX_LEVELS], const crsh_scene *scene, float t_min,
                                     crsh_hits *hits, crsh_meta *meta, void *ws, size_t ws_bytes,
                                     hipStream_t stream)
{
    if (!pairs) {
        set_error("crsh_leaf_hit: NULL argument");
        return CRSH_ERR_INVALID;
    }
    // levels present in the pair table: consecutive entries with storage
    uint32_t levels = 0;
    while (levels < CRSH_MAX_LEVELS && pairs[levels].tri && pairs[levels].node) ++levels;
    return leaf_hit_launch(sorted, sorted_ids, bundle, merge, nodes, &pairs[0], &pairs[1], scene, t_min, hits, meta,
                           ws, ws_bytes, nullptr, 256, levels, stream);
}
