// Stage 4: hierarchy traversal (Sec. 3.3.7, Eq. 9).
//
// k_tri_sph    bounding sphere of every triangle (centroid, farthest vertex).
// k_top        persistent waves; one (top node, mesh) item per wave in item
//              order: mesh-sphere test, then the mesh's triangles (in the
//              current triangle batch) against the node, 64 per step.  The
//              item's survivors are counted, its offset found by decoupled
//              look-back over items, and the survivors written in triangle
//              order.
// k_level      persistent 256-thread blocks; one parent pair per thread, its
//              F children tested in order; block scan + look-back over tiles
//              give every survivor its place, so the child level comes out
//              trimmed (Fig. 4) and in (parent pair, child) order.
// Both orders equal a sequential traversal's, so each pair level is
// deterministic.
#include "common.hpp"

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
struct trav_ctl {
    uint32_t top_ctr;
    uint32_t lvl_ctr[CRSH_MAX_LEVELS];
};

__global__ void k_tri_sph(const float *__restrict__ v0x, const float *__restrict__ v0y,
                          const float *__restrict__ v0z, const float *__restrict__ v1x,
                          const float *__restrict__ v1y, const float *__restrict__ v1z,
                          const float *__restrict__ v2x, const float *__restrict__ v2y,
                          const float *__restrict__ v2z, uint32_t b, uint32_t e, float4 *out)
{
    const float third = 1.0f / 3.0f;
    for (uint32_t t = b + blockIdx.x * blockDim.x + threadIdx.x; t < e; t += gridDim.x * blockDim.x) {
        f3 a = mk(v0x[t], v0y[t], v0z[t]);
        f3 bb = mk(v1x[t], v1y[t], v1z[t]);
        f3 c = mk(v2x[t], v2y[t], v2z[t]);
        f3 ctr = ((a + bb) + c) * third;
        float r = fmax2(fmax2(len(a - ctr), len(bb - ctr)), len(c - ctr));
        float m = fmax2(fmax2(fabsf(ctr.x), fabsf(ctr.y)), fabsf(ctr.z));
        r = r + SPHERE_PAD * (r + m);
        out[t] = make_float4(ctr.x, ctr.y, ctr.z, r);
    }
}

// Eq. 9 with H the projection of P on the node axis: |P-H| = |(P-C) x a|,
// |C-H| = |(P-C).a|; pass iff |P-H|^2 <= (|C-H| tan + (d + r) sec)^2.
struct node_t {
    f3 C, a;
    float r, c, tan, sec;
};

__device__ __forceinline__ node_t load_node(const node_arrays &nd, uint32_t i)
{
    node_t n;
    n.C = mk(nd.cx[i], nd.cy[i], nd.cz[i]);
    n.r = nd.r[i];
    n.a = mk(nd.ax[i], nd.ay[i], nd.az[i]);
    n.c = nd.c[i];
    n.tan = nd.tan[i];
    n.sec = nd.sec[i];
    return n;
}

__device__ __forceinline__ bool node_meets(const node_t &n, f3 P, float d)
{
    if (!(n.c > 0.0f)) return true;
    f3 v = P - n.C;
    float t = dot(v, n.a);
    f3 w = cross(v, n.a);
    float lhs2 = dot(w, w);
    float rhs = fabsf(t) * n.tan + (d + n.r) * n.sec;
    return lhs2 <= rhs * rhs;
}

// Zero the look-back words that the next traversal kernel will use.
__global__ void k_trav_prep(uint64_t *flags, trav_ctl *ctl, crsh_meta *meta, int32_t parent_level,
                            uint32_t n_mesh, pair_levels P, int32_t first)
{
    const uint32_t nl = meta->n_levels;
    uint64_t need = 0;
    if (parent_level == 0) {
        if (nl > 0) need = (uint64_t)meta->level_cnt[nl - 1] * n_mesh;
    } else if ((uint32_t)parent_level <= nl && parent_level >= 2) {
        uint64_t nin = meta->pairs[parent_level - 1];
        uint64_t cap = P.p[parent_level - 1].cap;
        nin = nin < cap ? nin : cap;
        need = (nin + LEVEL_TILE - 1) / LEVEL_TILE;
    }
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < need;
         i += (uint64_t)gridDim.x * blockDim.x)
        flags[i] = 0;
    if (first && blockIdx.x == 0 && threadIdx.x < CRSH_MAX_LEVELS) {
        meta->pairs[threadIdx.x] = 0;
        ctl->lvl_ctr[threadIdx.x] = 0;
        if (threadIdx.x == 0) ctl->top_ctr = 0;
    }
}

__global__ __launch_bounds__(WAVE) void k_top(node_arrays nd, const float4 *__restrict__ tsph,
                                              const uint32_t *__restrict__ mesh_first,
                                              const uint32_t *__restrict__ mesh_count,
                                              const float *__restrict__ msph, uint32_t n_mesh, uint32_t tri_begin,
                                              uint32_t tri_end, pair_levels P, uint64_t *flags, trav_ctl *ctl,
                                              crsh_meta *meta)
{
    const uint32_t nl = meta->n_levels;
    if (nl == 0) return;
    const uint32_t top = nl - 1;
    const uint32_t ntop = meta->level_cnt[top];
    const uint32_t off = meta->level_off[top];
    const uint64_t n_items = (uint64_t)ntop * n_mesh;
    const pairs_dev out = P.p[top];
    const uint32_t l = lane_id();
    if (out.tri == nullptr) {       // no storage for this many levels
        if (blockIdx.x == 0 && l == 0) atomicOr(&meta->status, CRSH_OVERFLOW_PAIRS);
        return;
    }
    uint64_t tests = 0, mhits = 0, items = 0;
    for (;;) {
        uint32_t item = 0;
        if (l == 0) item = atomicAdd(&ctl->top_ctr, 1u);
        item = __shfl(item, 0, WAVE);
        if (item >= n_items) break;
        ++items;
        const uint32_t i = item / n_mesh;
        const uint32_t m = item - i * n_mesh;
        const node_t node = load_node(nd, off + i);
        const bool pass = node_meets(node, mk(msph[4 * m], msph[4 * m + 1], msph[4 * m + 2]), msph[4 * m + 3]);
        uint32_t b = 0, e = 0;
        if (pass) {
            ++mhits;
            b = max(mesh_first[m], tri_begin);
            e = min(mesh_first[m] + mesh_count[m], tri_end);
            if (e < b) e = b;
            tests += e - b;
        }
        uint32_t cnt = 0;
        for (uint32_t t0 = b; t0 < e; t0 += WAVE) {
            uint32_t t = t0 + l;
            bool ok = false;
            if (t < e) {
                float4 s = tsph[t];
                ok = node_meets(node, mk(s.x, s.y, s.z), s.w);
            }
            cnt += (uint32_t)__popcll(ballot(ok));
        }
        uint64_t excl = 0;
        if (l == 0) excl = lookback(flags, item, cnt);
        excl = __shfl(excl, 0, WAVE);
        uint64_t pos = excl;
        if (cnt) {
            for (uint32_t t0 = b; t0 < e; t0 += WAVE) {
                uint32_t t = t0 + l;
                bool ok = false;
                if (t < e) {
                    float4 s = tsph[t];
                    ok = node_meets(node, mk(s.x, s.y, s.z), s.w);
                }
                uint64_t mask = ballot(ok);
                uint64_t at = pos + rank_below(mask);
                if (ok && at < out.cap) {
                    out.tri[at] = t;
                    out.node[at] = i;
                }
                pos += (uint32_t)__popcll(mask);
            }
        }
        if (item == n_items - 1 && l == 0) {
            uint64_t total = excl + cnt;
            meta->pairs[top] = total;
            atomicAdd((unsigned long long *)&meta->hits[top], (unsigned long long)total);
            if (total > out.cap) atomicOr(&meta->status, CRSH_OVERFLOW_PAIRS);
        }
    }
    if (l == 0) {
        if (tests) atomicAdd((unsigned long long *)&meta->tests[top], (unsigned long long)tests);
        if (mhits) atomicAdd((unsigned long long *)&meta->mesh_hits, (unsigned long long)mhits);
        if (items) atomicAdd((unsigned long long *)&meta->mesh_tests, (unsigned long long)items);
    }
}

__global__ __launch_bounds__(LEVEL_TILE) void k_level(int32_t parent_level, uint32_t F, node_arrays nd,
                                                      const float4 *__restrict__ tsph, uint32_t m, pair_levels P,
                                                      uint64_t *flags, trav_ctl *ctl, crsh_meta *meta)
{
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_scan[LEVEL_TILE / WAVE];
    __shared__ uint64_t s_red[LEVEL_TILE / WAVE];
    const uint32_t nl = meta->n_levels;
    if ((uint32_t)parent_level > nl) return;
    const pairs_dev in = P.p[parent_level - 1];
    const pairs_dev out = P.p[parent_level - 2];
    if (in.tri == nullptr || out.tri == nullptr) return;
    uint64_t nin = meta->pairs[parent_level - 1];
    nin = nin < in.cap ? nin : in.cap;
    const uint64_t ntiles = (nin + LEVEL_TILE - 1) / LEVEL_TILE;
    const uint32_t nk = meta->level_cnt[parent_level - 2];
    const uint32_t offk = meta->level_off[parent_level - 2];
    uint64_t tests = 0;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&ctl->lvl_ctr[parent_level - 1], 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint64_t q = (uint64_t)tile * LEVEL_TILE + threadIdx.x;
        uint32_t mask = 0, tri = 0, p = 0;
        if (q < nin) {
            tri = in.tri[q];
            p = in.node[q];
            const float4 s = tsph[tri < m ? tri : 0];
            const f3 Pc = mk(s.x, s.y, s.z);
            for (uint32_t j = 0; j < F; ++j) {
                const uint32_t ch = p * F + j;
                if (ch >= nk) break;
                ++tests;
                if (node_meets(load_node(nd, offk + ch), Pc, s.w)) mask |= 1u << j;
            }
        }
        const uint32_t c = (uint32_t)__popc(mask);
        uint32_t total;
        const uint32_t ex = block_excl_scan<uint32_t, LEVEL_TILE / WAVE>(c, s_scan, total);
        if (threadIdx.x == 0) s_excl = lookback(flags, tile, total);
        __syncthreads();
        uint64_t at = s_excl + ex;
        while (mask) {
            const uint32_t j = (uint32_t)__builtin_ctz(mask);
            mask &= mask - 1;
            if (at < out.cap) {
                out.tri[at] = tri;
                out.node[at] = p * F + j;
            }
            ++at;
        }
        if (tile == ntiles - 1 && threadIdx.x == 0) {
            const uint64_t all = s_excl + total;
            meta->pairs[parent_level - 2] = all;
            atomicAdd((unsigned long long *)&meta->hits[parent_level - 2], (unsigned long long)all);
            if (all > out.cap) atomicOr(&meta->status, CRSH_OVERFLOW_PAIRS);
        }
        __syncthreads();
    }
    tests = wave_sum(tests);
    if (lane_id() == 0) s_red[threadIdx.x / WAVE] = tests;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < LEVEL_TILE / WAVE; ++i) t += s_red[i];
        if (t) atomicAdd((unsigned long long *)&meta->tests[parent_level - 2], (unsigned long long)t);
    }
}

}  // namespace crsh

using namespace crsh;

extern "C" crsh_status crsh_traverse(const crsh_nodes *nodes, const crsh_scene *scene, uint32_t tri_begin,
                                     uint32_t tri_end, int32_t bundle, int32_t merge,
                                     const crsh_pairs pairs[CRSH_MAX_LEVELS], crsh_meta *meta, void *ws,
                                     size_t ws_bytes, hipStream_t stream)
{
    if (!nodes || !scene || !pairs || !meta || !ws) {
        set_error("crsh_traverse: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (bundle < 1 || bundle > CRSH_MAX_BUNDLE || merge < 2 || merge > CRSH_MAX_MERGE) {
        set_error("crsh_traverse: bad bundle or merge factor");
        return CRSH_ERR_INVALID;
    }
    for (int k = 0; k < 9; ++k)
        if (!scene->v[k] && scene->m) {
            set_error("crsh_traverse: missing vertex array");
            return CRSH_ERR_INVALID;
        }
    if (scene->n_mesh == 0 || !scene->mesh_first || !scene->mesh_count || !scene->msph) {
        set_error("crsh_traverse: scene has no meshes");
        return CRSH_ERR_INVALID;
    }
    if (tri_end > scene->m || tri_begin > tri_end) {
        set_error("crsh_traverse: triangle batch [%u, %u) outside [0, %u)", tri_begin, tri_end, scene->m);
        return CRSH_ERR_INVALID;
    }
    // levels present in the pair table: consecutive entries with storage
    int levels = 0;
    uint64_t max_pairs = 0;
    while (levels < CRSH_MAX_LEVELS && pairs[levels].tri && pairs[levels].node) {
        max_pairs = std::max(max_pairs, pairs[levels].capacity);
        ++levels;
    }
    if (levels == 0) {
        set_error("crsh_traverse: no pair storage");
        return CRSH_ERR_INVALID;
    }
    size_t need = trav_ws_bytes(scene->m, (uint64_t)nodes->capacity * scene->n_mesh, max_pairs);
    if (ws_bytes < need) {
        set_error("crsh_traverse: workspace too small (%zu < %zu)", ws_bytes, need);
        return CRSH_ERR_INVALID;
    }
    char *w = (char *)ws;
    float4 *tsph = (float4 *)w;
    w += align256((size_t)scene->m * 16);
    trav_ctl *ctl = (trav_ctl *)w;
    w += align256(64 * 8);
    uint64_t *flags = (uint64_t *)w;

    node_arrays nd{nodes->cx, nodes->cy, nodes->cz, nodes->r, nodes->ax, nodes->ay, nodes->az,
                   nodes->c, nodes->tan, nodes->sec};
    pair_levels P;
    for (int k = 0; k < CRSH_MAX_LEVELS; ++k) {
        P.p[k].tri = k < levels ? pairs[k].tri : nullptr;
        P.p[k].node = k < levels ? pairs[k].node : nullptr;
        P.p[k].cap = k < levels ? pairs[k].capacity : 0;
    }
    const float *const *v = scene->v;
    if (tri_end > tri_begin) {
        uint32_t g = std::min<uint32_t>((tri_end - tri_begin + 255) / 256, 2048);
        k_tri_sph<<<g, 256, 0, stream>>>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], tri_begin,
                                         tri_end, tsph);
    }
    k_trav_prep<<<1024, 256, 0, stream>>>(flags, ctl, meta, 0, scene->n_mesh, P, 1);
    {
        prof_scope ps("k_top", stream);
        k_top<<<2048, WAVE, 0, stream>>>(nd, tsph, scene->mesh_first, scene->mesh_count, scene->msph, scene->n_mesh,
                                     tri_begin, tri_end, P, flags, ctl, meta);
    }
    for (int L = levels; L >= 2; --L) {
        uint64_t tiles = (pairs[L - 1].capacity + LEVEL_TILE - 1) / LEVEL_TILE;
        uint32_t g = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(tiles, 1), 2048);
        k_trav_prep<<<1024, 256, 0, stream>>>(flags, ctl, meta, L, scene->n_mesh, P, 0);
        {
            prof_scope ps("k_level", stream);
            k_level<<<g, LEVEL_TILE, 0, stream>>>(L, (uint32_t)merge, nd, tsph, scene->m, P, flags, ctl, meta);
        }
    }
    return hip_check(hipGetLastError(), "crsh_traverse launch");
}
