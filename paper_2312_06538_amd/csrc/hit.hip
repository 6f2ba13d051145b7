// Stage 5: final intersection tests and closest hit (Sec. 3.3.8).
//
// k_hit_prep   triangles repacked as 3 x float4 (v0, e1 = v1 - v0,
//              e2 = v2 - v0): one 48-byte fetch per test instead of nine
//              scattered loads; e1, e2 are the same single roundings the
//              test would make.
// k_hit        persistent waves over the level-1 pairs; a group of G lanes
//              (G = bundle rounded up to a power of two) takes one pair, one
//              lane per ray of its leaf, so a leaf's rays are read
//              contiguously from the sorted ray arrays.  A hit lowers the
//              ray's 64-bit (t bits, triangle) key with an atomic minimum:
//              positive floats order like their bit patterns, so the minimum
//              is the closest hit with ties to the lower triangle id.
// k_hit_final  one thread per sorted ray: decode the key, recompute u, v with
//              the same test, write the result at the ray id.
// Batched form: a leaf's rays are the range the build recorded with it (first
// sorted ray, count) and the accepted interval starts at its frame's t_min.
#include "batch.hpp"
#include "intersect.hpp"

namespace crsh {

__global__ void k_hit_prep(const float *__restrict__ v0x, const float *__restrict__ v0y,
                           const float *__restrict__ v0z, const float *__restrict__ v1x,
                           const float *__restrict__ v1y, const float *__restrict__ v1z,
                           const float *__restrict__ v2x, const float *__restrict__ v2y,
                           const float *__restrict__ v2z, uint32_t m, float4 *tri)
{
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        float ax = v0x[t], ay = v0y[t], az = v0z[t];
        float e1x = v1x[t] - ax, e1y = v1y[t] - ay, e1z = v1z[t] - az;
        float e2x = v2x[t] - ax, e2y = v2y[t] - ay, e2z = v2z[t] - az;
        tri[3 * t + 0] = make_float4(ax, ay, az, e1x);
        tri[3 * t + 1] = make_float4(e1y, e1z, e2x, e2y);
        tri[3 * t + 2] = make_float4(e2z, 0.0f, 0.0f, 0.0f);
    }
}

struct sorted_rays {
    const float *ox, *oy, *oz, *dx, *dy, *dz, *tmax;
};

#ifndef CRSH_HIT_UNROLL
#define CRSH_HIT_UNROLL 2
#endif
constexpr int HIT_UNROLL = CRSH_HIT_UNROLL;    // pairs per lane group in flight at once

// Sorted rays repacked as 2 x float4 (origin, tmax), (direction, 0): two
// 16-byte loads per test instead of seven scattered ones.
__global__ void k_hit_rays(sorted_rays R, const crsh_meta *meta, uint32_t cap, float4 *rays)
{
    const uint32_t n = min(meta->n_rays, cap);
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        rays[2 * s] = make_float4(R.ox[s], R.oy[s], R.oz[s], R.tmax[s]);
        rays[2 * s + 1] = make_float4(R.dx[s], R.dy[s], R.dz[s], 0.0f);
    }
}

template <bool BATCH>
__global__ __launch_bounds__(256) void k_hit(const float4 *__restrict__ R, const float4 *__restrict__ tri,
                                             const uint32_t *__restrict__ ptri, const uint32_t *__restrict__ pnode,
                                             uint64_t cap1, uint32_t B, uint32_t log2G, float t_min0,
                                             unsigned long long *tkey, crsh_meta *meta, uint32_t ray_cap, uint32_t m,
                                             batch_dev bd)
{
    __shared__ uint64_t s_red[256 / WAVE];
    const uint32_t n = min(meta->n_rays, ray_cap);
    const uint32_t n_leaf = meta->level_cnt[0];
    uint64_t np = meta->n_levels ? meta->pairs[0] : 0;
    np = np < cap1 ? np : cap1;
    const uint32_t l = lane_id();
    const uint32_t G = 1u << log2G;
    const uint32_t slot = l >> log2G;        // pair slot of this lane in the wave
    const uint32_t j = l & (G - 1);          // ray of the leaf
    const uint32_t per_wave = WAVE >> log2G;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
    uint64_t tests = 0;
    // Each lane group takes HIT_UNROLL pairs per iteration, a grid stride
    // apart, and issues all their loads before any test: the pair, triangle
    // and ray loads of the pairs overlap instead of forming one dependent
    // chain per pair.
    const uint64_t step = nwaves * per_wave;
    const bool lane_ok = j < B;
    for (uint64_t q0 = wave * per_wave; q0 < np; q0 += HIT_UNROLL * step) {
        uint32_t t[HIT_UNROLL], s[HIT_UNROLL];
        bool ok[HIT_UNROLL];
        float t_min[HIT_UNROLL];
#pragma unroll
        for (int k = 0; k < HIT_UNROLL; ++k) {
            const uint64_t q = q0 + slot + k * step;
            ok[k] = lane_ok && q < np;
            t[k] = ok[k] ? ptri[q] : 0u;
            const uint32_t leaf = ok[k] ? pnode[q] : 0u;
            t_min[k] = t_min0;
            if constexpr (BATCH) {
                ok[k] = ok[k] && leaf < n_leaf;
                const uint32_t info = ok[k] ? bd.node_info[leaf] : 0u;
                ok[k] = ok[k] && j < (info & INFO_COUNT_MASK);
                s[k] = ok[k] ? bd.node_first[leaf] + j : 0u;
                if (ok[k]) t_min[k] = bd.frames[info >> INFO_FRAME_SHIFT].t_min;
            } else {
                s[k] = leaf * B + j;
            }
            ok[k] = ok[k] && s[k] < n && t[k] < m;
        }
        tri_t tr[HIT_UNROLL];
        float4 ro[HIT_UNROLL], rd[HIT_UNROLL];
#pragma unroll
        for (int k = 0; k < HIT_UNROLL; ++k) {
            tr[k] = load_tri(tri, ok[k] ? t[k] : 0u);
            ro[k] = R[2 * (ok[k] ? s[k] : 0u)];
            rd[k] = R[2 * (ok[k] ? s[k] : 0u) + 1];
        }
#pragma unroll
        for (int k = 0; k < HIT_UNROLL; ++k) {
            if (!ok[k]) continue;
            ++tests;
            float th;
            if (moller_trumbore_t(mk(ro[k].x, ro[k].y, ro[k].z), mk(rd[k].x, rd[k].y, rd[k].z), t_min[k], ro[k].w,
                                  tr[k], th)) {
                unsigned long long key = ((unsigned long long)__float_as_uint(th) << 32) | t[k];
                atomicMin(&tkey[s[k]], key);
            }
        }
    }
    tests = wave_sum(tests);
    if (l == 0) s_red[threadIdx.x / WAVE] = tests;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot = 0;
        for (uint32_t i = 0; i < blockDim.x / WAVE; ++i) tot += s_red[i];
        if (tot) atomicAdd((unsigned long long *)&meta->final_tests, (unsigned long long)tot);
    }
}

struct hit_out {
    int32_t *tri;
    float *t, *u, *v;
};

template <bool BATCH>
__global__ void k_hit_final(sorted_rays R, const float4 *__restrict__ tri, const uint32_t *__restrict__ sorted_ids,
                            float t_min0, const unsigned long long *tkey, hit_out out, const crsh_meta *meta,
                            uint32_t ray_cap, uint32_t m, batch_dev bd)
{
    const uint32_t n = min(meta->n_rays, ray_cap);
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        const unsigned long long key = tkey[s];
        const uint32_t id = sorted_ids[s];
        if (id >= ray_cap) continue;    // ids come from the sort: never taken
        float t_min = t_min0;
        if constexpr (BATCH) t_min = bd.frames[min(bd.ray_frame[id], bd.n_frames - 1)].t_min;
        int32_t best = -1;
        float th = 0.0f, uh = 0.0f, vh = 0.0f;
        if (key != ~0ull && (uint32_t)(key & 0xFFFFFFFFull) < m) {
            const uint32_t t = (uint32_t)(key & 0xFFFFFFFFull);
            const f3 O = mk(R.ox[s], R.oy[s], R.oz[s]);
            const f3 D = mk(R.dx[s], R.dy[s], R.dz[s]);
            if (moller_trumbore(O, D, t_min, R.tmax[s], load_tri(tri, t), th, uh, vh)) {
                best = (int32_t)t;
            } else {                     // cannot happen: same inputs, same operations
                best = (int32_t)t;
                th = __uint_as_float((uint32_t)(key >> 32));
            }
        }
        out.tri[id] = best;
        out.t[id] = th;
        out.u[id] = uh;
        out.v[id] = vh;
    }
}

__global__ void k_tkey_fill(unsigned long long *tkey, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) tkey[i] = ~0ull;
}

}  // namespace crsh

using namespace crsh;

extern "C" crsh_status crsh_hits_reset(crsh_hits *hits, hipStream_t stream)
{
    if (!hits || !hits->tkey) {
        set_error("crsh_hits_reset: NULL argument");
        return CRSH_ERR_INVALID;
    }
    uint32_t g = std::min<uint32_t>((hits->capacity + 255) / 256, 4096);
    if (g == 0) g = 1;
    k_tkey_fill<<<g, 256, 0, stream>>>(hits->tkey, hits->capacity);
    return hip_check(hipGetLastError(), "crsh_hits_reset launch");
}

namespace crsh {

void hit_prep_launch(const crsh_scene *scene, float4 *tri, hipStream_t stream)
{
    const float *const *v = scene->v;
    if (scene->m) {
        uint32_t g = std::min<uint32_t>((scene->m + 255) / 256, 2048);
        k_hit_prep<<<g, 256, 0, stream>>>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], scene->m, tri);
    }
}

void hit_pairs_launch(const crsh_rays *sorted, const float4 *tri, float4 *rays4, const crsh_pairs *level1,
                      int32_t bundle, const crsh_scene *scene, float t_min, crsh_hits *hits, crsh_meta *meta,
                      const batch_dev *bd, int32_t hit_block, hipStream_t stream)
{
    if (!level1->capacity) return;
    uint32_t log2G = 0;
    while ((1u << log2G) < (uint32_t)bundle) ++log2G;
    {
        sorted_rays S{sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, sorted->tmax};
        uint32_t g = std::max<uint32_t>(std::min<uint32_t>((sorted->capacity + 255) / 256, 4096), 1);
        k_hit_rays<<<g, 256, 0, stream>>>(S, meta, sorted->capacity, rays4);
    }
    const float4 *R = rays4;
    const batch_dev b = bd ? *bd : batch_dev{};
    const uint32_t grid = 2048u * 256u / (uint32_t)hit_block;   // the same number of waves
    prof_scope ps("k_hit", stream);
    if (bd)
        k_hit<true><<<grid, hit_block, 0, stream>>>(R, tri, level1->tri, level1->node, level1->capacity,
                                                    (uint32_t)bundle, log2G, t_min, hits->tkey, meta,
                                                    sorted->capacity, scene->m, b);
    else
        k_hit<false><<<grid, hit_block, 0, stream>>>(R, tri, level1->tri, level1->node, level1->capacity,
                                                     (uint32_t)bundle, log2G, t_min, hits->tkey, meta,
                                                     sorted->capacity, scene->m, b);
}

void hit_final_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, const float4 *tri,
                      const crsh_scene *scene, float t_min, crsh_hits *hits, crsh_meta *meta, const batch_dev *bd,
                      hipStream_t stream)
{
    sorted_rays R{sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, sorted->tmax};
    const batch_dev b = bd ? *bd : batch_dev{};
    uint32_t g = std::min<uint32_t>((sorted->capacity + 255) / 256, 4096);
    if (g == 0) g = 1;
    hit_out o{hits->tri, hits->t, hits->u, hits->v};
    prof_scope ps("k_hit_final", stream);
    if (bd)
        k_hit_final<true><<<g, 256, 0, stream>>>(R, tri, sorted_ids, t_min, hits->tkey, o, meta, sorted->capacity,
                                                 scene->m, b);
    else
        k_hit_final<false><<<g, 256, 0, stream>>>(R, tri, sorted_ids, t_min, hits->tkey, o, meta,
                                                  sorted->capacity, scene->m, b);
}

crsh_status hit_check(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle, const crsh_pairs *level1,
                      const crsh_scene *scene, crsh_hits *hits, crsh_meta *meta, void *ws, int32_t hit_block,
                      const char *who)
{
    if (!sorted || !sorted_ids || !level1 || !scene || !hits || !meta || !ws) {
        set_error("%s: NULL argument", who);
        return CRSH_ERR_INVALID;
    }
    if (bundle < 1 || bundle > CRSH_MAX_BUNDLE) {
        set_error("%s: bundle must be in [1, %d]", who, CRSH_MAX_BUNDLE);
        return CRSH_ERR_INVALID;
    }
    if (hit_block != 64 && hit_block != 128 && hit_block != 256) {
        set_error("%s: workgroup size must be 64, 128 or 256", who);
        return CRSH_ERR_INVALID;
    }
    if (!sorted->ox || !sorted->oy || !sorted->oz || !sorted->dx || !sorted->dy || !sorted->dz ||
        !sorted->tmax || !hits->tkey || !hits->tri || !hits->t || !hits->u || !hits->v ||
        (level1->capacity && (!level1->tri || !level1->node))) {
        set_error("%s: incomplete arrays", who);
        return CRSH_ERR_INVALID;
    }
    for (int k = 0; k < 9; ++k)
        if (!scene->v[k] && scene->m) {
            set_error("%s: missing vertex array", who);
            return CRSH_ERR_INVALID;
        }
    if (hits->capacity < sorted->capacity) {
        set_error("%s: hit capacity below the ray capacity", who);
        return CRSH_ERR_INVALID;
    }
    return CRSH_OK;
}

crsh_status hit_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle,
                       const crsh_pairs *level1, const crsh_scene *scene, float t_min, crsh_hits *hits,
                       crsh_meta *meta, void *ws, size_t ws_bytes, const batch_dev *bd, int32_t hit_block,
                       hipStream_t stream)
{
    crsh_status st = hit_check(sorted, sorted_ids, bundle, level1, scene, hits, meta, ws, hit_block,
                               "crsh_closest_hit");
    if (st != CRSH_OK) return st;
    if (ws_bytes < hit_ws_bytes(scene->m, sorted->capacity)) {
        set_error("crsh_closest_hit: workspace too small (%zu < %zu)", ws_bytes,
                  hit_ws_bytes(scene->m, sorted->capacity));
        return CRSH_ERR_INVALID;
    }
    float4 *tri = (float4 *)ws;
    float4 *rays4 = (float4 *)((char *)ws + align256((size_t)scene->m * 48));
    hit_prep_launch(scene, tri, stream);
    hit_pairs_launch(sorted, tri, rays4, level1, bundle, scene, t_min, hits, meta, bd, hit_block, stream);
    hit_final_launch(sorted, sorted_ids, tri, scene, t_min, hits, meta, bd, stream);
    return hip_check(hipGetLastError(), "crsh_closest_hit launch");
}

}  // namespace crsh

extern "C" crsh_status crsh_closest_hit(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle,
                                        const crsh_pairs *level1, const crsh_scene *scene, float t_min,
                                        crsh_hits *hits, crsh_meta *meta, void *ws, size_t ws_bytes,
                                        hipStream_t stream)
{
    return hit_launch(sorted, sorted_ids, bundle, level1, scene, t_min, hits, meta, ws, ws_bytes, nullptr, 256,
                      stream);
}
