// Device view of a batch of independent frames and the lookups that map a
// batch-wide index (pixel, node, top-level item) to its frame.
//
// A batch concatenates its frames: pixels, rays and the nodes of each level
// are laid out frame by frame, so a frame owns one contiguous range of each,
// starting at a per-frame base that is non-decreasing in the frame index.
// The frame of an index x is the last frame whose base is <= x; a frame with
// an empty range shares its base with the next frame and is never returned
// for an index inside that next frame's range.
#pragma once

#include "common.hpp"

namespace crsh {

struct batch_dev {
    const crsh_frame *frames;
    crsh_frame_meta *fm;
    uint32_t n_frames;
    uint32_t *node_first;        // per packed node: first sorted ray (level 1) or first child (level-local)
    uint32_t *node_info;         // per packed node: count in bits 0-7, frame in bits 8-15
    const uint32_t *ray_frame;   // frame of every ray id
    uint64_t *top;               // [0] items of the current top-level pass, [1] its append base
    uint64_t top_cap;            // capacity for top-level items
    const uint32_t *mat_flags;
    const float *mat_ior;
};

constexpr uint32_t INFO_COUNT_MASK = 255u;
constexpr uint32_t INFO_FRAME_SHIFT = 8;

// last f in [0, n) with base(f) <= x, for a non-decreasing base with base(0) <= x
template <typename Base>
__device__ __forceinline__ uint32_t last_at_most(uint32_t n, uint64_t x, Base base)
{
    uint32_t lo = 1, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)base(mid) <= x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo - 1;
}

__device__ __forceinline__ uint32_t frame_of_pixel(const batch_dev &b, uint32_t p)
{
    return last_at_most(b.n_frames, p, [&](uint32_t f) { return b.frames[f].pix_begin; });
}

// frame of a node with level-local index j on level lv (0-based)
__device__ __forceinline__ uint32_t frame_of_node(const batch_dev &b, uint32_t lv, uint32_t j)
{
    return last_at_most(b.n_frames, j, [&](uint32_t f) { return b.fm[f].level_base[lv]; });
}

__device__ __forceinline__ uint32_t frame_of_item(const batch_dev &b, uint64_t it)
{
    return last_at_most(b.n_frames, it, [&](uint32_t f) { return b.fm[f].item_base; });
}

}  // namespace crsh
