// Device types and launchers of the traversal shared with the fused last
// level (crsh_leaf_hit).
#pragma once

#include "batch.hpp"

namespace crsh {

// One level's pairs: two arrays (triangle, node), or one packed word per
// pair -- node in the high bits, triangle minus tri_base in the low
// CRSH_PACKED_TRI_BITS (Sec. 3.3.7's 32-bit pair encoding; node == nullptr).
struct pairs_dev {
    uint32_t *tri, *node;
    uint64_t cap;
    uint32_t packed;       // 1: packed words in `tri`
    uint32_t tri_base;     // first triangle of the batch (packed form)
};

// PACKED is a compile-time choice so that the two-array kernels are the
// same code as without packed support.
template <bool PACKED>
__device__ __forceinline__ void pair_get(const pairs_dev &p, uint64_t q, uint32_t &tri, uint32_t &node)
{
    if constexpr (PACKED) {
        const uint32_t w = p.tri[q];
        tri = p.tri_base + (w & ((1u << CRSH_PACKED_TRI_BITS) - 1u));
        node = w >> CRSH_PACKED_TRI_BITS;
    } else {
        tri = p.tri[q];
        node = p.node[q];
    }
}

template <bool PACKED>
__device__ __forceinline__ void pair_put(const pairs_dev &p, uint64_t at, uint32_t tri, uint32_t node)
{
    if constexpr (PACKED) {
        p.tri[at] = (node << CRSH_PACKED_TRI_BITS) | (tri - p.tri_base);
    } else {
        p.tri[at] = tri;
        p.node[at] = node;
    }
}

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
                        const batch_dev *bd, uint64_t tiles_cap, uint32_t top_levels, hipStream_t stream,
                        bool packed = false);

}  // namespace crsh
