// Shared device helpers of the CRSH HIP library (gfx950, wave64).
//
// Floating point: every kernel is compiled with -ffp-contract=off and
// correctly rounded float32 division and square root, so each written
// operation rounds once (IEEE binary32, nearest-even) and sums of three terms
// are evaluated as (a + b) + c.  That fixed order is what makes keys, nodes
// and pairs reproducible bit for bit by any other conforming implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crsh.h"

namespace crsh {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ float3
struct f3 {
    float x, y, z;
};

__device__ __forceinline__ f3 mk(float x, float y, float z)
{
    f3 r;
    r.x = x;
    r.y = y;
    r.z = z;
    return r;
}
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ f3 operator/(f3 a, float s) { return mk(a.x / s, a.y / s, a.z / s); }
__device__ __forceinline__ f3 operator-(f3 a) { return mk(-a.x, -a.y, -a.z); }
__device__ __forceinline__ float dot(f3 a, f3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float len(f3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ float fmax2(float a, float b) { return a > b ? a : b; }

// Conservativeness margins (see the hierarchy build): spheres grow by
// SPHERE_PAD * (r + max|c|) per union, cones by CONE_PAD radians per change.
// Bisectors of sums shorter than BISECT_MIN are too inaccurate: full cone.
constexpr float SPHERE_PAD = 0x1p-20f;
constexpr float CONE_PAD = 0x1p-16f;
constexpr float BISECT_MIN = 0.25f;
constexpr float INSIDE_MARGIN = 0x1p-20f;
constexpr float NEAR_PARALLEL = 0x1p-10f;
constexpr float DET_EPS = 1e-12f;

// --------------------------------------------------------------- wave ops
__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// wave mask of the lanes where p holds (inactive lanes: 0); lowers to the
// compare result itself, with no per-lane select
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Raw buffer resource over `bytes` bytes at p (bytes clamped to 2^32 - 1):
// loads through it take a 32-bit byte offset, and a load past the end
// returns zeros instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint64_t bytes)
{
    const int n = (int)(bytes < 0xFFFFFFFFull ? bytes : 0xFFFFFFFFull);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, n, 0x00020000);
}

__device__ __forceinline__ float4 buf_load4(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float buf_load1(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// inclusive prefix sum over the 64 lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T o = __shfl_up(v, d, WAVE);
        if (l >= (uint32_t)d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// Exclusive block scan of one value per thread; returns the exclusive prefix
// and the block total.  scratch: NWAVES entries of LDS.
template <typename T, int NWAVES>
__device__ __forceinline__ T block_excl_scan(T v, T *scratch, T &total)
{
    const uint32_t l = lane_id();
    const uint32_t w = threadIdx.x / WAVE;
    T inc = wave_incl_scan(v);
    if (l == WAVE - 1) scratch[w] = inc;
    __syncthreads();
    T before = 0;
    T tot = 0;
#pragma unroll
    for (int i = 0; i < NWAVES; ++i) {
        T s = scratch[i];
        if ((uint32_t)i < w) before += s;
        tot += s;
    }
    total = tot;
    __syncthreads();
    return before + inc - v;
}

// ------------------------------------------------ decoupled look-back scan
// Tiles publish their own count first (flag 1), then the inclusive prefix
// once known (flag 2); a tile walks back over its predecessors until it meets
// an inclusive prefix.  Tiles take their index from an atomic counter in
// launch order, so every tile waited on has already started and publishes
// its count without waiting itself: the walk always ends.
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr uint64_t LB_MASK = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by a whole wave (all 64 lanes); returns the exclusive prefix of
// `count` to every lane.  The wave reads 64 predecessors' words at once
// (lane i looks at tile - 1 - i), so a walk over many tiles that have only
// published their own count costs one round trip per 64 tiles.
__device__ __forceinline__ uint64_t lookback_wave(uint64_t *flags, uint32_t tile, uint64_t count)
{
    const uint32_t l = lane_id();
    if (tile == 0) {
        if (l == 0) lb_store(&flags[0], LB_INC | count);
        return 0;
    }
    if (l == 0) lb_store(&flags[tile], LB_AGG | count);
    uint64_t excl = 0;
    int64_t top = (int64_t)tile - 1;
    for (;;) {
        const int64_t idx = top - (int64_t)l;
        const uint64_t f = idx >= 0 ? lb_load(&flags[idx]) : LB_INC;   // before tile 0: prefix 0
        const uint64_t kind = f & ~LB_MASK;
        const uint64_t inc = ballot(kind == LB_INC);
        const uint64_t none = ballot(kind == 0);
        const uint32_t first = inc ? (uint32_t)__builtin_ctzll(inc) : 64u;
        const uint64_t upto = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
        if (none & upto) {                 // a tile we need has not published yet
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum((uint64_t)(l <= first ? (f & LB_MASK) : 0ull));
        if (first < 64) break;
        top -= WAVE;
    }
    if (l == 0) lb_store(&flags[tile], LB_INC | (excl + count));
    return excl;
}

// Called by one thread of the tile; returns the exclusive prefix of `count`.
__device__ __forceinline__ uint64_t lookback(uint64_t *flags, uint32_t tile, uint64_t count)
{
    if (tile == 0) {
        lb_store(&flags[0], LB_INC | count);
        return 0;
    }
    lb_store(&flags[tile], LB_AGG | count);
    uint64_t excl = 0;
    int64_t j = (int64_t)tile - 1;
    while (j >= 0) {
        uint64_t f = lb_load(&flags[j]);
        if ((f & ~LB_MASK) == 0) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += f & LB_MASK;
        if ((f & ~LB_MASK) == LB_INC) break;
        --j;
    }
    lb_store(&flags[tile], LB_INC | (excl + count));
    return excl;
}

// ------------------------------------------------------------- workspace
// Every stage carves its scratch from the start of the caller's workspace;
// these are the byte counts each stage needs.
constexpr uint32_t SORT_TILE = 4096;      // keys per sort tile
constexpr uint32_t SORT_PASSES = 4;       // 8-bit digits of a 32-bit key
constexpr uint32_t HASH_BLOCK = 256;      // pixels per hash block
constexpr uint64_t HASH_STATIC_MAX_PIXELS = CRSH_HASH_STATIC_MAX_PIXELS;  // crsh_hash_static
constexpr uint32_t LEVEL_THREADS = 256;   // threads of a traversal tile
#ifndef CRSH_EMIT_PPT
#define CRSH_EMIT_PPT 2
#endif
constexpr uint32_t LEVEL_PPT = 1;   // parent pairs per thread of the count pass
constexpr uint32_t LEVEL_TILE = LEVEL_THREADS * LEVEL_PPT;   // parent pairs per count tile
constexpr uint32_t COUNT_THREADS = 512;    // threads of a count block: COUNT_TPS tiles per step
constexpr uint32_t COUNT_TPS = COUNT_THREADS / LEVEL_THREADS;
constexpr uint32_t COUNT_WINDOW = 1024;    // child nodes a count block keeps in LDS (36 B each)
#define COUNT_WAVES_PER_SIMD 6             // 3 count blocks per compute unit (LDS: 48 KiB each)
constexpr uint32_t EMIT_PPT = CRSH_EMIT_PPT;     // parent pairs per thread of the emit pass
constexpr uint32_t EMIT_TILE = LEVEL_THREADS * EMIT_PPT;     // parent pairs per emit tile
static_assert(EMIT_PPT % LEVEL_PPT == 0, "an emit tile covers whole count tiles");
// parent pairs per emit thread for NF children per parent: the thread's pass
// bits (NF per pair) must fit one 32-bit mask word
constexpr int emit_ppt(int nf) { return (int)EMIT_PPT * nf <= 32 ? (int)EMIT_PPT : 32 / nf; }
constexpr uint32_t SCAN_TILE_ITEMS = 4096;                 // counts per scan tile

__host__ __device__ constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t sort_ws_bytes(uint32_t cap);
size_t hash_ws_bytes(uint64_t pixels);
size_t trav_ws_bytes(uint32_t m, uint32_t node_cap, uint64_t top_items, uint64_t max_pairs);
// Final-test workspace: packed triangles (48 B each), then per ray slot the
// packed ray (32 B: origin and direction in two arrays of 16 B per slot) and
// a closest-hit key (8 B).  Slots: one per sorted ray in
// the plain form; in the batched form B per level-1 node, at most the rays
// plus B - 1 per frame.
size_t hit_ws_bytes(uint32_t m, uint32_t slots);
// bounds of the final tests' 32-bit byte offsets (16 B per ray slot in each
// of two arrays, 48 B per triangle)
#define CRSH_HIT_MAX_SLOTS (1u << 27)
#define CRSH_HIT_MAX_TRIS (1u << 26)
constexpr uint32_t hit_slots(uint32_t rays, bool batch)
{
    return batch ? rays + CRSH_MAX_FRAMES * (CRSH_MAX_BUNDLE - 1) : rays;
}
struct hit_slots_ws {
    float4 *org;                 // per slot: origin, tmax
    float *dir;                  // per slot: direction (12 bytes)
    unsigned long long *keys;    // per slot (batched form)
    uint32_t slots;
};
inline hit_slots_ws carve_hit_slots(void *at, uint32_t slots)
{
    hit_slots_ws h;
    h.org = (float4 *)at;
    h.dir = (float *)((char *)at + align256((size_t)slots * 16));
    h.keys = (unsigned long long *)((char *)h.dir + align256((size_t)slots * 16));
    h.slots = slots;
    return h;
}
inline size_t hit_slots_bytes(uint32_t slots) { return 2 * align256((size_t)slots * 16) + align256((size_t)slots * 8); }

// Stage launchers shared by the plain entry points (bd == nullptr) and the
// batched form (bd: the batch's device view, frame-aware kernels).
struct batch_dev;
crsh_status hash_launch(const crsh_gbuf *gbuf, const crsh_raygen *rg, const batch_dev *bd, crsh_rays *out,
                        uint32_t *keys, uint32_t *ids, uint32_t *ray_frame, crsh_meta *meta, void *ws,
                        size_t ws_bytes, hipStream_t stream);
crsh_status sort_launch(const uint32_t *keys_in, const uint32_t *ids_in, const uint32_t *frame_of,
                        uint32_t *keys_out, uint32_t *ids_out, uint32_t capacity, crsh_meta *meta, void *ws,
                        size_t ws_bytes, hipStream_t stream);
crsh_status build_launch(const crsh_rays *rays, const uint32_t *sorted_ids, int32_t bundle, int32_t merge,
                         int32_t levels, crsh_nodes *nodes, crsh_rays *sorted, crsh_meta *meta,
                         const batch_dev *bd, hipStream_t stream);
crsh_status traverse_launch(const crsh_nodes *nodes, const crsh_scene *scene, uint32_t tri_begin, uint32_t tri_end,
                            int32_t bundle, int32_t merge, const crsh_pairs pairs[CRSH_MAX_LEVELS],
                            crsh_meta *meta, void *ws, size_t ws_bytes, const batch_dev *bd, int32_t levels,
                            uint64_t top_items, int32_t lowest, hipStream_t stream);
crsh_status hit_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle,
                       const crsh_pairs *level1, const crsh_scene *scene, float t_min, crsh_hits *hits,
                       crsh_meta *meta, void *ws, size_t ws_bytes, const batch_dev *bd, int32_t hit_block,
                       hipStream_t stream, bool packed = false, uint32_t tri_base = 0);
crsh_status leaf_hit_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle, int32_t merge,
                            const crsh_nodes *nodes, const crsh_pairs *level1, const crsh_pairs *level2,
                            const crsh_scene *scene, float t_min, crsh_hits *hits, crsh_meta *meta, void *ws,
                            size_t ws_bytes, const batch_dev *bd, int32_t hit_block, uint32_t top_levels,
                            hipStream_t stream);
// pieces of the final tests shared by crsh_closest_hit and crsh_leaf_hit
crsh_status hit_check(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle, const crsh_pairs *level1,
                      const crsh_scene *scene, crsh_hits *hits, crsh_meta *meta, void *ws, int32_t hit_block,
                      const char *who);
void hit_prep_launch(const crsh_scene *scene, float4 *tri, hipStream_t stream);
void hit_pairs_launch(const crsh_rays *sorted, const float4 *tri, const hit_slots_ws &hs, const crsh_pairs *level1,
                      int32_t bundle, const crsh_scene *scene, float t_min, crsh_hits *hits, crsh_meta *meta,
                      const batch_dev *bd, int32_t hit_block, hipStream_t stream, bool packed = false,
                      uint32_t tri_base = 0);
// final tests of the level-1 pairs given as level-2 pairs and level-1 pass
// masks (the fused last level); rays packed by hit_pairs_launch first
void hit_masked_launch(const crsh_rays *sorted, const float4 *tri, const hit_slots_ws &hs, const crsh_pairs *level2,
                       const uint32_t *mask, int32_t merge, int32_t bundle, const crsh_scene *scene, float t_min,
                       crsh_hits *hits, crsh_meta *meta, const batch_dev *bd, int32_t hit_block, hipStream_t stream);
void hit_final_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, const float4 *tri,
                      const hit_slots_ws &hs, int32_t bundle, const crsh_scene *scene, float t_min,
                      crsh_hits *hits, crsh_meta *meta, const batch_dev *bd, hipStream_t stream);
void tri_spheres_launch(const crsh_scene *scene, uint32_t b, uint32_t e, float4 *out, hipStream_t stream);
size_t leaf_hit_ws_bytes(uint32_t m, uint32_t node_cap, uint64_t level2_cap, uint32_t rays);
size_t sort_chunked_ws_bytes(uint32_t cap);

// launch helpers
void set_error(const char *fmt, ...);
crsh_status hip_check(hipError_t e, const char *what);

// Largest grid of `threads`-thread blocks of kernel f that the current device
// keeps resident at once (occupancy x compute units), capped at `want`.
uint32_t resident_grid(const void *f, int threads, uint64_t want);

// One-shot kernel timer (crsh_profile_next): prof_begin returns true when
// this launch is the armed one and has recorded the start event.
bool prof_begin(const char *kernel, hipStream_t s);
void prof_end(bool armed, hipStream_t s);

struct prof_scope {
    bool on;
    hipStream_t s;
    prof_scope(const char *k, hipStream_t st) : on(prof_begin(k, st)), s(st) {}
    ~prof_scope() { prof_end(on, s); }
};

}  // namespace crsh
