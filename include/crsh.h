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
#define CRSH_OVERFLOW_ITEMS 8u   /* batched form: more top-level (node, mesh) items than
                                    crsh_batch.top_item_capacity */
#define CRSH_OVERFLOW_PACKED 16u /* packed pairs: a level has more nodes than
                                    CRSH_PACKED_MAX_NODES (its pairs are not valid) */

/* ray-type bits of crsh_raygen.ray_types */
#define CRSH_RAY_SHADOW 1u
#define CRSH_RAY_REFLECT 2u
#define CRSH_RAY_REFRACT 4u
/* Comparison mode (the ray-space hierarchy without ray sorting, Sec. 2):
 * keys keep only the type and light bits (31-28), so crsh_sort only groups
 * the rays per type and light and keeps their generation order. */
#define CRSH_KEY_TYPE_ONLY 0x100u
/* Direction codes from spherical coordinates (theta = acos dz, phi =
 * atan2(dy, dx), Sec. 3.3.2) instead of the octahedral map; acos / atan are
 * the Abramowitz & Stegun 4.4.45 / 4.4.47 polynomials in binary32. */
#define CRSH_KEY_SPHERICAL 0x200u
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
    uint64_t final_u_pass;                  /* final tests whose u passed (Moller-Trumbore, Sec. 3.3.8) */
    uint64_t final_uv_pass;                 /* final tests whose u and v passed */
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

/* The same pairs packed into one 32-bit word each, as Sec. 3.3.7 stores them:
 * node id (local to its level) in bits 31-14, triangle id minus the first
 * triangle of the batch in bits 13-0.  A triangle batch therefore holds at
 * most 2^14 triangles and a level at most 2^18 nodes. */
#define CRSH_PACKED_TRI_BITS 14
#define CRSH_PACKED_MAX_TRIS (1u << CRSH_PACKED_TRI_BITS)
#define CRSH_PACKED_MAX_NODES (1u << (32 - CRSH_PACKED_TRI_BITS))
typedef struct crsh_packed_pairs {
    uint32_t *pair;
    uint64_t capacity;
} crsh_packed_pairs;

/* Closest hits.  tkey is scratch in SORTED order (one 64-bit word per sorted
 * ray: the bits of t mapped to an order-preserving unsigned form -- negative
 * values complemented, others with the sign bit set -- above the triangle
 * id; all ones = no hit); tri/t/u/v are the results by ray id: triangle (-1
 * on a miss), distance and barycentrics (0 on a miss). */
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

/* crsh_hash without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments (less ws / ws_bytes), kernels and results
 * as crsh_hash.  Its scratch -- one 32-bit ray count per block of 256 pixels,
 * 512.25 KiB -- is a static device array that each GPU holds from the first
 * call on that GPU until the process ends; the call allocates nothing.
 * Every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU (concurrent streams or threads) race: serialise them.  The array needs
 * no clearing between calls.  The stream must belong to the current device.
 * Errors: CRSH_ERR_INVALID for more than CRSH_HASH_STATIC_MAX_PIXELS pixels
 * (nothing launched) and for crsh_hash's argument errors; CRSH_ERR_HIP if the
 * array's device address cannot be obtained. */
#define CRSH_HASH_STATIC_MAX_PIXELS (1ull << 25)
crsh_status crsh_hash_static(const crsh_gbuf *gbuf, const crsh_raygen *rg, crsh_rays *out,
                             uint32_t *keys, uint32_t *ids, crsh_meta *meta, hipStream_t stream);

/* Stage 2 -- ray sorting (Sec. 3.3.3-3.3.5).  Stable LSD radix sort of the
 * meta->n_rays (key, id) pairs by the 32-bit key; equal keys keep their input
 * order.  Inputs are not modified; outputs hold `capacity` entries.  Digit
 * passes in which every key has the same digit are skipped on the device. */
crsh_status crsh_sort(const uint32_t *keys_in, const uint32_t *ids_in,
                      uint32_t *keys_out, uint32_t *ids_out, uint32_t capacity,
                      crsh_meta *meta, void *ws, size_t ws_bytes, hipStream_t stream);

/* Stage 2 in the paper's layout (Sec. 3.3.3-3.3.5): compression of the
 * pairs into chunks of equal consecutive keys (head flags + scan), a radix
 * sort of the chunks by key, decompression (scan of the sorted chunk sizes,
 * then every output position takes its chunk's element).  Same contract and
 * result as crsh_sort; it moves one sort entry per chunk, which pays when
 * runs of equal keys are long.  ws: crsh_workspace_size() bytes. */
crsh_status crsh_sort_chunked(const uint32_t *keys_in, const uint32_t *ids_in,
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

/* Stage 4 with packed pairs (Sec. 3.3.7's encoding) for one triangle batch
 * [tri_begin, tri_end) of at most CRSH_PACKED_MAX_TRIS triangles: the same
 * tests, counters and pair order as crsh_traverse over the same batch, every
 * pair stored as one crsh_packed_pairs word (4 bytes instead of 8).
 * Errors: CRSH_ERR_INVALID for a batch over CRSH_PACKED_MAX_TRIS triangles
 * (nothing launched); a hierarchy level with more than CRSH_PACKED_MAX_NODES
 * nodes sets CRSH_OVERFLOW_PACKED in meta->status on the device, and the
 * pairs of that call are then not valid.  Workspace: crsh_workspace_size. */
crsh_status crsh_traverse_packed(const crsh_nodes *nodes, const crsh_scene *scene,
                                 uint32_t tri_begin, uint32_t tri_end,
                                 int32_t bundle, int32_t merge,
                                 const crsh_packed_pairs pairs[CRSH_MAX_LEVELS], crsh_meta *meta,
                                 void *ws, size_t ws_bytes, hipStream_t stream);

/* Stage 4 without its last level pass: as crsh_traverse, but the level-1
 * pairs that descend from level 2 are not formed; crsh_leaf_hit forms and
 * consumes them on chip.  pairs[0] still needs storage: a hierarchy whose top
 * is level 1 gets its level-1 pairs from the top-level pass. */
crsh_status crsh_traverse_upper(const crsh_nodes *nodes, const crsh_scene *scene,
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

/* Stage 5 on the packed level-1 pairs of crsh_traverse_packed: tri_begin is
 * that call's first triangle.  Same results as crsh_closest_hit on the
 * unpacked pairs; results merge across triangle batches through hits->tkey
 * (clear it with crsh_hits_reset before the first batch). */
crsh_status crsh_closest_hit_packed(const crsh_rays *sorted, const uint32_t *sorted_ids,
                                    int32_t bundle, const crsh_packed_pairs *level1, uint32_t tri_begin,
                                    const crsh_scene *scene, float t_min,
                                    crsh_hits *hits, crsh_meta *meta,
                                    void *ws, size_t ws_bytes, hipStream_t stream);

/* Stages 4 (level 1, Eq. 9) and 5 (Sec. 3.3.8) fused, after
 * crsh_traverse_upper: every level-2 pair of pairs[1] is tested against the
 * children (leaves) of its node (Eq. 9), the pass bits kept in the
 * workspace, and every passing (triangle, leaf) is tested against the
 * leaf's rays (Moller-Trumbore) straight from the level-2 pairs and those
 * bits.  Level-1 pairs stored in pairs[0] (top level 1) are tested as in
 * crsh_closest_hit.  Results and counters equal crsh_traverse followed by
 * crsh_closest_hit: meta->tests[0], hits[0] (level-1 pairs formed),
 * final_tests, final_u_pass and final_uv_pass accumulate; the level-1 pairs
 * are not stored (pairs[0] still needs storage, with a nonzero capacity:
 * CRSH_ERR_INVALID otherwise).  `sorted`, `sorted_ids`, `nodes`, bundle and
 * merge as given to crsh_build.  ws: crsh_workspace_size() bytes. */
crsh_status crsh_leaf_hit(const crsh_rays *sorted, const uint32_t *sorted_ids,
                          int32_t bundle, int32_t merge, const crsh_nodes *nodes,
                          const crsh_pairs pairs[CRSH_MAX_LEVELS], const crsh_scene *scene,
                          float t_min, crsh_hits *hits, crsh_meta *meta,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* The next bounce (Sec. 3.3.8: the algorithm goes on with a new set of
 * secondary rays from the sorting step).  Every reflection or refraction
 * parent ray (key type 01 or 10) with a closest hit spawns, in parent-id
 * order, the secondary rays of its hit point exactly as crsh_hash does for a
 * primary hit: P = O + t D, the unit geometric normal of the hit triangle
 * (e1 x e2 normalised) turned against D, the triangle's material
 * tri_mat[tri] (index into rg->mat_flags / mat_ior), and D itself instead of
 * the view direction (rg->eye is not used).  Shadow parents and misses spawn
 * nothing; children keep their parent's pix.  Parents are by ray id with
 * their keys and hits (crsh_closest_hit's tri and t); their count is
 * parent_meta->n_rays.  Writes out / keys / ids and meta->n_rays like
 * crsh_hash (meta cleared by the caller, distinct from parent_meta; out and
 * keys distinct from the parents').  ws: crsh_workspace_size() bytes. */
crsh_status crsh_bounce(const crsh_rays *parents, const uint32_t *parent_keys, const crsh_hits *hits,
                        const crsh_meta *parent_meta, const crsh_scene *scene, const int32_t *tri_mat,
                        const crsh_raygen *rg, crsh_rays *out, uint32_t *keys, uint32_t *ids,
                        crsh_meta *meta, void *ws, size_t ws_bytes, hipStream_t stream);

/* Stage 1 for rays the caller already has (e.g. a differentiable renderer):
 * keys[i] = the hash of ray i under the same layout as crsh_hash -- `type`
 * 0 shadow (bits 29-28 = `light`), 1 reflection, 2 refraction (origin cell
 * in the box [lo, lo + 1/inv_ext]) -- and ids[i] = i, for i < n.  Writes
 * meta->n_rays = n.  rays->capacity must be >= n. */
crsh_status crsh_hash_rays(const crsh_rays *rays, uint32_t n, uint32_t type, uint32_t light,
                           const float lo[3], const float inv_ext[3], uint32_t *keys, uint32_t *ids,
                           crsh_meta *meta, hipStream_t stream);

/* Layout helper for indexed meshes: v[k][i] = verts[3 * faces[3 * i + k / 3] + k % 3]
 * (the nine triangle arrays of crsh_scene) for the m triangles; faces index
 * the n_verts vertices (xyz interleaved).  A triangle with an index outside
 * [0, n_verts) is written as all zeros (degenerate: never hit). */
crsh_status crsh_gather_triangles(const float *verts, uint32_t n_verts, const int32_t *faces, uint32_t m,
                                  float *const v[9], hipStream_t stream);

/* Enclosing sphere of every mesh (Sec. 3.3.1) from the current triangle
 * arrays v[0..8] (crsh_scene layout): msph[4*i .. 4*i+3] = (cx, cy, cz, r)
 * with the centre at the midpoint of the bounding box of mesh i's vertices
 * and r the largest vertex distance from it, widened by 2^-20 of itself so
 * that float32 rounding never leaves a vertex outside.  Meshes are the
 * triangle ranges [mesh_first[i], +mesh_count[i]) (clamped to m); an empty
 * mesh gets (0, 0, 0, 0).  For geometry that moves between frames (e.g.
 * vertices being optimised): the traversal's whole-mesh culling is only
 * conservative with spheres that hold the current vertices.  All pointers
 * are device pointers. */
crsh_status crsh_mesh_spheres(const float *const v[9], uint32_t m, const uint32_t *mesh_first,
                              const uint32_t *mesh_count, uint32_t n_mesh, float *msph, hipStream_t stream);

/* Adjoint of the closest hit (Sec. 3.3.8) with respect to the triangle
 * vertices and the ray, holding each ray's hit triangle fixed.  For ray i
 * with hit triangle tri[i] >= 0 (t, u, v from crsh_closest_hit), the
 * Moller-Trumbore solution satisfies O + t D = (1-u-v) v0 + u v1 + v v2; with
 * upstream gradients (g_t, g_u, g_v) and lambda solving
 * [D | -e1 | -e2]^T lambda = (g_t, g_u, g_v) (recomputed per hit from cross
 * products, nothing stored by the forward pass):
 *   dL/dO = -lambda, dL/dD = -t lambda,
 *   dL/dv0 += (1-u-v) lambda, dL/dv1 += u lambda, dL/dv2 += v lambda.
 * Rays are by ray id (origin, direction), n of them; hits->tri/t/u/v by ray
 * id; faces index verts (xyz interleaved).  g_verts (3 floats per vertex) is
 * ACCUMULATED with float32 atomics -- the caller zeroes it; g_o, g_d
 * (3 floats per ray, xyz interleaved) are written, zero for misses.  Any of
 * g_t, g_u, g_v may be NULL (zero). */
crsh_status crsh_closest_hit_backward(const crsh_rays *rays, uint32_t n, const crsh_hits *hits,
                                      const float *g_t, const float *g_u, const float *g_v,
                                      const float *verts, uint32_t n_verts, const int32_t *faces, uint32_t m,
                                      float *g_verts, float *g_o, float *g_d, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent frames (each its own primary-hit buffer,
 * lights, camera, materials and meshes) run as ONE pipeline.  Arrays are the
 * concatenation of the frames' arrays; every stage is one launch sequence
 * for the whole batch, each kernel finding its frame from per-frame offsets
 * on the device, so frames of a few thousand rays do not leave the chip
 * idle.  Per frame the results are exactly those of the plain calls with the
 * same bundle / merge / levels: a frame's rays, keys, sorted order, nodes,
 * pairs and closest hits do not depend on the other frames (node ids and
 * sorted positions are offset by the frame's bases).  The sequence allocates
 * nothing, synchronises nothing and records no memset, so it can be captured
 * into one hipGraph (crsh_batch_graph_create).
 *
 * Layout.  Frame f's pixels, rays, sorted rays and hits are the ranges that
 * start at crsh_frame.pix_begin and crsh_frame_meta.ray_begin.  Level k+1 of
 * the node arrays holds every frame's nodes of that level, frame by frame
 * (frame f's at crsh_frame_meta.level_base[k] within the level), and levels
 * are packed as in crsh_build (meta->level_off).  A frame's hierarchy stops
 * after `levels` levels or at its first level with one node, so frames have
 * different top levels; pairs[k] holds level k+1 pairs of all frames: first
 * those that descend from level k+2, in parent order, then the top-level
 * pairs of frames whose top is level k+1, frame by frame.  Each frame's
 * subsequence is exactly its plain pair list with node ids offset by
 * level_base[k].
 * ------------------------------------------------------------------------ */

#define CRSH_MAX_FRAMES 256

/* One frame of a batch (an array of these lives in device memory).  Frames
 * must cover the primary-hit buffer in order: frame 0 starts at pixel 0 and
 * frame f+1 at pix_begin + pix_count of frame f. */
typedef struct crsh_frame {
    uint32_t pix_begin, pix_count;      /* this frame's pixels in the batch's primary-hit buffer */
    uint32_t mesh_begin, mesh_count;    /* this frame's meshes in the batch's scene (their triangle
                                           ranges index the batch's triangle arrays) */
    uint32_t mat_begin, n_mats;         /* this frame's materials in the batch's material tables */
    int32_t n_lights;
    uint32_t ray_types;
    float lights[CRSH_MAX_LIGHTS][3];
    float eye[3];
    float eps_off, eps_shadow, t_min;
    float lo[3], inv_ext[3];            /* bounce-ray origin box, as in crsh_raygen */
} crsh_frame;

/* Per-frame results written on the device by the batched stages. */
typedef struct crsh_frame_meta {
    uint32_t ray_begin, n_rays;         /* the frame's rays in the batch's ray arrays */
    uint32_t n_levels;                  /* levels of the frame's hierarchy (top = n_levels) */
    uint32_t reserved;
    uint32_t level_base[CRSH_MAX_LEVELS];   /* first node of the frame within level k+1 */
    uint32_t level_cnt[CRSH_MAX_LEVELS];    /* nodes of the frame on level k+1 */
    uint64_t item_base;                 /* scratch of the top-level traversal pass */
} crsh_frame_meta;

/* Everything a batch reads and writes; all pointers are device pointers.
 * gbuf covers all frames' pixels (w = total pixels, h = 1); material indices
 * in gbuf.mat are frame-local.  rays, sorted and keys/ids/skeys/sids/
 * ray_frame hold rays.capacity entries (enough for every pixel's
 * n_lights + 2 slots never overflows); ray_frame receives each ray's frame.
 * meta receives batch totals (n_rays, per-level node offsets and totals,
 * pair counts, counters summed over frames).  nodes, pairs and hits as in
 * the plain calls.  top_item_capacity bounds the (top node, mesh) items of
 * one top-level pass: the sum over the frames that share a top level of
 * top nodes x meshes.  bundle / merge / levels shape every frame's
 * hierarchy; hit_block (64, 128 or 256) is the workgroup size of the final
 * tests.  ws: crsh_batch_ws_size() bytes. */
typedef struct crsh_batch {
    uint32_t n_frames;                  /* 1 .. CRSH_MAX_FRAMES */
    const crsh_frame *frames;
    crsh_frame_meta *frame_meta;
    crsh_gbuf gbuf;
    const uint32_t *mat_flags;
    const float *mat_ior;
    crsh_scene scene;
    crsh_rays rays, sorted;
    uint32_t *keys, *ids, *skeys, *sids, *ray_frame;
    crsh_nodes nodes;
    crsh_pairs pairs[CRSH_MAX_LEVELS];
    crsh_hits hits;
    crsh_meta *meta;
    uint64_t top_item_capacity;
    void *ws;
    size_t ws_bytes;
    int32_t bundle, merge, levels, hit_block;
    int32_t leaf_hit;                   /* nonzero: last level fused with the final tests (crsh_leaf_hit);
                                           pairs[0] then holds only top-level-1 pairs */
} crsh_batch;

typedef struct crsh_graph crsh_graph;

/* Workspace of a batch: max_rays rays (and at most as many pixels),
 * max_tris triangles, max_nodes nodes, max_pairs pairs per level and
 * max_top_items top-level items. */
size_t crsh_batch_ws_size(uint32_t max_rays, uint32_t max_tris, uint32_t max_nodes, uint64_t max_pairs,
                          uint64_t max_top_items);

/* Enqueue the whole batched pipeline (clear, hash, sort, build, traverse,
 * closest hit) on a stream.  Overflow is reported through meta as for the
 * plain calls (crsh_read_meta after the stream completes); the caller then
 * grows the named buffer and runs the batch again.  Argument errors return
 * CRSH_ERR_INVALID before anything is enqueued. */
crsh_status crsh_batch_enqueue(const crsh_batch *b, hipStream_t stream);

/* Capture crsh_batch_enqueue on `stream` (not the legacy default stream) into
 * a hipGraph and instantiate it; crsh_graph_launch replays the whole batch
 * with one launch.  The graph keeps the pointers and sizes of `b`: replays
 * read the device arrays' current contents.  No kernel timer may be armed
 * (crsh_profile_next) while capturing. */
crsh_status crsh_batch_graph_create(const crsh_batch *b, hipStream_t stream, crsh_graph **out);
crsh_status crsh_graph_launch(crsh_graph *g, hipStream_t stream);
void crsh_graph_destroy(crsh_graph *g);

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
