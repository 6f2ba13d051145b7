// Device types and launchers of the traversal shared with the fused last
// level (crsh_leaf_hit).
#pragma once

#include "batch.hpp"

namespace crsh {

struct pairs_dev {
    uint32_t *tri, *node;
    uint64_t cap;
};
struct pair_levels {
    pairs_dev p[CRSH_MAX_LEVELS];
};
struct node_arrays {
    const float *cx, *cy, *cz, *r, *ax, *ay, *az, *c, *tan, *sec;
};

// per-level scratch carved from the workspace
struct trav_scratch {
    uint32_t *cnt;         // survivors per work item
    uint64_t *off;         // exclusive offsets of the work items
    uint32_t *mask;        // pass masks of the lower-level count pass
    uint64_t *scan_flags;  // look-back words of the scan
    uint32_t *scan_ctr;    // tile counter of the scan
};

constexpr uint32_t SCAN_THREADS = 256;
constexpr uint32_t SCAN_ITEMS = 16;
constexpr uint32_t SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
static_assert(SCAN_TILE == SCAN_TILE_ITEMS, "workspace sizing");

void node_pack_launch(const crsh_nodes *nodes, crsh_meta *meta, float4 *na, float4 *nb, float *ns, bool clear_pairs,
                      hipStream_t stream);
// count pass of one level (pass masks and per-tile survivor counts in S,
// node tests added to meta)
void level_count_launch(int32_t parent_level, int32_t merge, const float4 *na, const float4 *nb, const float *ns,
                        const float4 *tsph, uint32_t m, const pair_levels &P, const trav_scratch &S, crsh_meta *meta,
                        const batch_dev *bd, uint64_t tiles_cap, hipStream_t stream);

}  // namespace crsh
