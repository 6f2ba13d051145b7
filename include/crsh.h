/*
 * crsh.h -- C-ABI of the Coherent Ray-Space Hierarchy (CRSH) secondary-ray
 * path on AMD Instinct MI355X (gfx950).
 *
 * Method: Reis, Costa, Pereira, "Ray-Tracing With a Coherent Ray-Space
 * Hierarchy".  A frame's primary hits (position, normal, material per pixel,
 * Sec. 3.2) become secondary rays that are hashed (Sec. 3.3.2), sorted by key
 * (Sec. 3.3.3-3.3.5), bundled into an n-level hierarchy of sphere-cone nodes
 * (Sec. 3.3.6, Eq. 1-8), traversed top-down against whole-mesh and per-
 * triangle bounding spheres (Sec. 3.3.7, Eq. 9), and finally tested ray by
 * ray against the surviving triangles for the closest hit (Sec. 3.3.8).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array pointer is a DEVICE pointer owned by the caller.  The library
 *   allocates nothing inside a stage call and frees nothing it did not make.
 * - Every stage call is asynchronous on the given HIP stream.  Counts that the
 *   GPU discovers (number of rays, node and pair counts, counters, overflow
 *   flags) live in a caller-owned device block `crsh_meta`; the host reads it
 *   with crsh_read_meta(), which synchronises the stream.
 * - Argument errors are detected on the host before anything is launched and
 *   return CRSH_ERR_INVALID; a failed launch returns CRSH_ERR_HIP.  Running out
 *   of a capacity is detected on the device: the stage writes what fits, sets
 *   a bit in meta->status and keeps counting, so meta holds the size that would
 *   have been needed.  crsh_read_meta() then returns CRSH_ERR_CAPACITY.
 * - crsh_last_error() returns a short text for the last failure of the
 *   calling thread.  No C++ exception crosses this interface.
 * - Layouts are structure-of-arrays, float32 for geometry, uint32 for keys,
 *   ids and pair members.  Rays are indexed by ray id (the order in which
 *   crsh_hash emits them) except where a function says "sorted order".
 */
#ifndef CRSH_H
#define CRSH_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CRSH_MAX_LEVELS 16
#define CRSH_MAX_LIGHTS 4
#define CRSH_MAX_BUNDLE 32
#define CRSH_MAX_MERGE 16

typedef enum crsh_status {
    CRSH_OK = 0,
    CRSH_ERR_INVALID = 1,   /* bad argument; nothing was launched */
    CRSH_ERR_CAPACITY = 2,  /* a device buffer was too small (see meta) */
    CRSH_ERR_HIP = 3        /* a HIP call failed */
} crsh_status;

/* bits of crsh_meta.status */
#define CRSH_OVERFLOW_RAYS 1u    /* more secondary rays than crsh_rays.capacity */
#define CRSH_OVERFLOW_NODES 2u   /* more nodes than crsh_nodes.capacity */
#define CRSH_OVERFLOW_PAIRS 4u   /* a pair level exceeded its crsh_pairs.capacity */

/* ray-type bits of crsh_raygen.ray_types */
#define CRSH_RAY_SHADOW 1u
#define CRSH_RAY_REFLECT 2u
#define CRSH_RAY_REFRACT 4u
/* material bits of crsh_raygen.mat_flags[] */
#define CRSH_MAT_REFLECTIVE 1u
#define CRSH_MAT_REFRACTIVE 2u

/* Device-resident bookkeeping shared by the stages of one frame.  The caller
 * allocates sizeof(crsh_meta) bytes of device memory and clears it with
 * crsh_meta_reset() before a frame. */
typedef struct crsh_meta {
    uint32_t n_rays;                        /* written by crsh_hash (or the caller) */
    uint32_t n_levels;                      /* written by crsh_build */
    uint32_t level_off[CRSH_MAX_LEVELS];    /* first node of level k+1 in crsh_nodes */
    uint32_t level_cnt[CRSH_MAX_LEVELS];    /* nodes on level k+1 */
    uint32_t status;                        /* CRSH_OVERFLOW_* bits */
    uint32_t reserved;
    uint64_t pairs[CRSH_MAX_LEVELS];        /* pairs of level k+1 from the last crsh_traverse
                                               call (may exceed the capacity) */
    uint64_t hits[CRSH_MAX_LEVELS];         /* the same, summed over triangle batches */
    uint64_t tests[CRSH_MAX_LEVELS];        /* node-triangle tests on level k+1 (Tables 1-3) */
    uint64_t mesh_tests, mesh_hits;         /* top nodes x mesh spheres (Sec. 3.3.7) */
    uint64_t final_tests;                   /* ray-triangle tests of Sec. 3.3.8 */
    uint64_t rays_required;                 /* rays that crsh_hash wanted to write */
    uint64_t nodes_required;                /* nodes that crsh_build wanted to write */
} crsh_meta;

/* Primary-hit buffer (Sec. 3.2), W*H pixels in row-major order: hit position,
 * unit normal facing the camera, material index (-1: nothing was hit). */
typedef struct crsh_gbuf {
    const float *px, *py, *pz;
    const float *nx, *ny, *nz;
    const int32_t *mat;
    int32_t w, h;
} crsh_gbuf;

/* Secondary-ray generation and hashing parameters (Sec. 3.3.2).
 * Shadow rays start AT the light and end eps_shadow before the surface point.
 * Reflection / refraction rays start eps_off off the surface along the normal.
 * [lo, lo + 1/inv_ext] is the box whose 64^3 cells quantise bounce-ray
 * origins in their keys; inv_ext is given (float32) so that every
 * implementation quantises identically.  mat_flags / mat_ior are device
 * arrays of n_mats entries. */
typedef struct crsh_raygen {
    int32_t n_lights;
    float lights[CRSH_MAX_LIGHTS][3];
    float eye[3];
    const uint32_t *mat_flags;
    const float *mat_ior;
    int32_t n_mats;
    uint32_t ray_types;
    float eps_off, eps_shadow;
    float lo[3], inv_ext[3];
} crsh_raygen;

/* A ray array: origin, unit direction, extent (t < tmax), source pixel. */
typedef struct crsh_rays {
    float *ox, *oy, *oz;
    float *dx, *dy, *dz;
    float *tmax;
    uint32_t *pix;          /* may be NULL where a function says so */
    uint32_t capacity;      /* elements available in every array */
} crsh_rays;

/* Sphere-cone nodes of all levels, level 1 first, packed (Sec. 3.3.6): the
 * node sphere (cx, cy, cz, r) holds the ray origins, the cone (axis ax, ay,
 * az with cos c and sin s of the half-angle) holds the directions; c <= 0
 * marks a cone of 90 degrees or more, never culled.  tan = s/c, sec = 1/c for
 * the traversal test (0 when c <= 0). */
typedef struct crsh_nodes {
    float *cx, *cy, *cz, *r;
    float *ax, *ay, *az, *c, *s;
    float *tan, *sec;
    uint32_t capacity;
} crsh_nodes;

/* Scene: M triangles as nine arrays v[0..8] = v0x, v0y, v0z, v1x, ..., v2z;
 * meshes are contiguous triangle ranges [mesh_first[i], +mesh_count[i]) with
 * an enclosing sphere msph[4*i .. 4*i+3] = (cx, cy, cz, r) each (Sec. 3.3.1). */
typedef struct crsh_scene {
    const float *v[9];
    uint32_t m;
    const uint32_t *mesh_first, *mesh_count;
    const float *msph;
    uint32_t n_mesh;
} crsh_scene;

/* Candidate (triangle id, node id) pairs of one level (Sec. 3.3.7); node ids
 * are local to their level. */
typedef struct crsh_pairs {
    uint32_t *tri, *node;
    uint64_t capacity;
} crsh_pairs;

/* Closest hits.  tkey is scratch in SORTED order (one 64-bit word per sorted
 * ray: float bits of t above the triangle id); tri/t/u/v are the results by
 * ray id: triangle (-1 on a miss), distance and barycentrics (0 on a miss). */
typedef struct crsh_hits {
    unsigned long long *tkey;
    int32_t *tri;
    float *t, *u, *v;
    uint32_t capacity;
} crsh_hits;

/* Last failure text of the calling thread ("" if none). */
const char *crsh_last_error(void);

/* Size in bytes of the scratch workspace that every stage needs for up to
 * max_rays rays (and pixels), max_tris triangles, max_meshes meshes,
 * max_nodes nodes (crsh_nodes.capacity) and max_pairs pairs per level.  Each
 * stage uses the workspace only during its own call, so one workspace serves
 * all stages of a frame on one stream. */
size_t crsh_workspace_size(uint32_t max_rays, uint32_t max_tris, uint32_t max_meshes,
                           uint32_t max_nodes, uint64_t max_pairs);

/* Clear a device crsh_meta (stream ordered, no memset node). */
crsh_status crsh_meta_reset(crsh_meta *meta, hipStream_t stream);

/* Copy meta to host_out after synchronising the stream.  Returns
 * CRSH_ERR_CAPACITY if any overflow bit is set, CRSH_OK otherwise. */
crsh_status crsh_read_meta(const crsh_meta *meta, crsh_meta *host_out, hipStream_t stream);

/* Stage 1 -- secondary-ray generation, trimming and hashing (Sec. 3.3.2).
 * Per pixel with a hit, in slot order: one shadow ray per light, then a
 * reflection ray (reflective material), then a refraction ray (refractive
 * material, no total internal reflection); only enabled types.  Holes are
 * trimmed (Fig. 4): ray ids are consecutive in (pixel, slot) order.
 * keys[id] = 32-bit hash (bits 31-30 type; shadow: light in 29-28, 28-bit
 * octahedral direction code; bounce: 18-bit origin cell over a 12-bit
 * direction code), ids[id] = id.  Writes meta->n_rays.  out, keys and ids
 * need out->capacity >= W*H*(n_lights+2) entries to never overflow.
 * ws: crsh_workspace_size() bytes. */
crsh_status crsh_hash(const crsh_gbuf *gbuf, const crsh_raygen *rg, crsh_rays *out,
                      uint32_t *keys, uint32_t *ids, crsh_meta *meta,
                      void *ws, size_t ws_bytes, hipStream_t stream);

/* Stage 2 -- ray sorting (Sec. 3.3.3-3.3.5).  Stable LSD radix sort of the
 * meta->n_rays (key, id) pairs by the 32-bit key; equal keys keep their input
 * order.  Inputs are not modified; outputs hold `capacity` entries.  Digit
 * passes in which every key has the same digit are skipped on the device. */
crsh_status crsh_sort(const uint32_t *keys_in, const uint32_t *ids_in,
                      uint32_t *keys_out, uint32_t *ids_out, uint32_t capacity,
                      crsh_meta *meta, void *ws, size_t ws_bytes, hipStream_t stream);

/* Stage 3 -- hierarchy creation (Sec. 3.3.6, Eq. 1-8).  Level 1 node j bounds
 * the rays at sorted positions [j*bundle, (j+1)*bundle); level k node j bounds
 * level k-1 nodes [j*merge, (j+1)*merge).  Building stops after `levels`
 * levels or at the first level with one node.  Writes nodes (packed, level 1
 * first), meta->n_levels / level_off / level_cnt, and the rays in sorted
 * order into `sorted` (origin, direction, tmax; sorted->pix may be NULL).
 * bundle in [1, CRSH_MAX_BUNDLE], merge in [2, CRSH_MAX_MERGE], levels in
 * [1, CRSH_MAX_LEVELS]. */
crsh_status crsh_build(const crsh_rays *rays, const uint32_t *sorted_ids,
                       int32_t bundle, int32_t merge, int32_t levels,
                       crsh_nodes *nodes, crsh_rays *sorted, crsh_meta *meta,
                       hipStream_t stream);

/* Stage 4 -- hierarchy traversal (Sec. 3.3.7, Eq. 9).  Top level: every top
 * node against every mesh sphere, then against the bounding sphere of every
 * triangle of each passing mesh that lies in [tri_begin, tri_end) (triangle
 * batches).  Each lower level tests every surviving (triangle, node) pair
 * against the node's children.  pairs[k] receives level k+1's surviving
 * pairs, in the order (parent pair, child) -- for the top level (node, mesh,
 * triangle) -- so every level is trimmed and deterministic.  pairs[k] and
 * pairs[k+2] may share storage (ping-pong); level 1 must not alias level 2.
 * Counters (tests, hits, mesh tests, final ray-triangle tests) accumulate in
 * meta.  `merge` and `bundle` must be those given to crsh_build. */
crsh_status crsh_traverse(const crsh_nodes *nodes, const crsh_scene *scene,
                          uint32_t tri_begin, uint32_t tri_end,
                          int32_t bundle, int32_t merge,
                          const crsh_pairs pairs[CRSH_MAX_LEVELS], crsh_meta *meta,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* Clear the closest-hit scratch before a frame (tkey = all ones). */
crsh_status crsh_hits_reset(crsh_hits *hits, hipStream_t stream);

/* Stage 5 -- final intersection tests (Sec. 3.3.8).  For every level-1 pair
 * (triangle, leaf) of `level1` and every ray of the leaf: two-sided
 * Moller-Trumbore, accepted for t_min < t < tmax; each ray keeps the smallest
 * (t, triangle id).  `sorted` and `sorted_ids` are the outputs of crsh_build /
 * crsh_sort.  Results merge with earlier calls (triangle batches) through
 * hits->tkey and are written by ray id into hits->tri/t/u/v. */
crsh_status crsh_closest_hit(const crsh_rays *sorted, const uint32_t *sorted_ids,
                             int32_t bundle, const crsh_pairs *level1,
                             const crsh_scene *scene, float t_min,
                             crsh_hits *hits, crsh_meta *meta,
                             void *ws, size_t ws_bytes, hipStream_t stream);

/* Instrumentation.  Arms a one-shot timer: the `occurrence`-th launch
 * (0-based, counted from this call, in the calling thread) of the library
 * kernel named `kernel` (e.g. "k_hit", "k_level", "k_sort_pass") is
 * bracketed by hipEventRecord(start) and hipEventRecord(stop) on the stream
 * it is launched on.  The events are owned by the caller.  Returns
 * CRSH_ERR_INVALID for a NULL name or event. */
crsh_status crsh_profile_next(const char *kernel, int32_t occurrence, hipEvent_t start, hipEvent_t stop);

#ifdef __cplusplus
}
#endif
#endif /* CRSH_H */
