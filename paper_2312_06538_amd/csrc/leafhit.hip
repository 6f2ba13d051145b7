// The last traversal level fused with the final tests (Sec. 3.3.7 at level 1,
// Sec. 3.3.8).
//
// In stage order the level-2 pairs become level-1 pairs (triangle, leaf) and
// then every ray of each leaf is tested; every child test reloads its node
// and every ray test reloads its ray.  Here the level-2 pairs are grouped by
// their node first (counting sort of the triangle ids: histogram, scan,
// scatter), then a workgroup takes one node and a chunk of its triangles:
//   - the node's children (leaves) and their rays are read once, the rays
//     into LDS, each lane keeping one child for the Eq. 9 tests;
//   - a wave tests 64 / NF triangles against the NF children at once (one
//     lane per (triangle, child)), and the passing pairs are handed out to
//     groups of G lanes (G = bundle rounded up to a power of two), one lane
//     per ray of the leaf, for the Moller-Trumbore tests;
//   - each ray's closest (t, triangle) is kept in LDS with an atomic minimum
//     and merged into the global per-ray key once per chunk.
// The counters are those of the stage order (level-1 node tests, level-1
// pairs, ray-triangle tests) and so are the closest hits (the minimum does
// not depend on the order of the tests); the level-1 pairs are not stored.
// Level-1 pairs that a top-level pass wrote (a hierarchy whose top is level
// 1) go through the plain final-test kernel first.
#include "batch.hpp"
#include "bounds.hpp"
#include "intersect.hpp"

namespace crsh {

constexpr uint32_t LH_THREADS = 256;
constexpr uint32_t LH_WAVES = LH_THREADS / WAVE;
constexpr uint32_t LH_CHUNK = 256;                                  // triangles per work item
constexpr uint32_t LH_MAX_RAYS = CRSH_MAX_BUNDLE * CRSH_MAX_MERGE;  // rays under one level-2 node
constexpr uint32_t LH_TILE = 4096;                                  // nodes per scan tile
constexpr uint32_t LH_PER_THREAD = LH_TILE / LH_THREADS;

struct lh_ws {
    float4 *tri;         // packed triangles (v0, e1, e2)
    hit_slots_ws hs;     // packed ray slots and their keys, for level-1 pairs of a top-level pass
    float4 *tsph;        // triangle bounding spheres
    uint32_t *cnt;       // level-2 pairs per node
    uint32_t *cursor;    // scatter cursors
    uint64_t *off;       // first bucket slot of each node
    uint32_t *ib;        // first work item of each node
    uint64_t *tsum;      // per scan tile: (pairs, items)
    uint32_t *n_items;   // work items in total
    uint32_t *bucket;    // triangle ids grouped by node
};

static lh_ws carve(void *ws, uint32_t m, uint32_t node_cap, uint64_t cap2, uint32_t slots)
{
    const uint32_t tiles = (node_cap + LH_TILE - 1) / LH_TILE + 1;
    char *w = (char *)ws;
    lh_ws L;
    L.tri = (float4 *)w;
    w += align256((size_t)m * 48);
    L.hs = carve_hit_slots(w, slots);
    w += hit_slots_bytes(slots);
    L.tsph = (float4 *)w;
    w += align256((size_t)m * 16);
    L.cnt = (uint32_t *)w;
    w += align256((size_t)node_cap * 4 + 4);
    L.cursor = (uint32_t *)w;
    w += align256((size_t)node_cap * 4 + 4);
    L.off = (uint64_t *)w;
    w += align256((size_t)node_cap * 8 + 8);
    L.ib = (uint32_t *)w;
    w += align256((size_t)node_cap * 4 + 4);
    L.tsum = (uint64_t *)w;
    w += align256((size_t)tiles * 16);
    L.n_items = (uint32_t *)w;
    w += align256(16);
    L.bucket = (uint32_t *)w;
    (void)cap2;
    return L;
}

size_t leaf_hit_ws_bytes(uint32_t m, uint32_t node_cap, uint64_t cap2, uint32_t slots)
{
    const uint32_t tiles = (node_cap + LH_TILE - 1) / LH_TILE + 1;
    return align256((size_t)m * 48) + hit_slots_bytes(slots) + align256((size_t)m * 16) +
           align256((size_t)node_cap * 4 + 4) * 2 + align256((size_t)node_cap * 8 + 8) +
           align256((size_t)node_cap * 4 + 4) + align256((size_t)tiles * 16) + align256(16) +
           align256((size_t)cap2 * 4 + 4);
}

// level-2 node count and the number of stored level-2 pairs
__device__ __forceinline__ void level2_sizes(const crsh_meta *meta, uint64_t cap2, uint32_t node_cap, uint32_t &n2,
                                             uint64_t &nin)
{
    const bool two = meta->n_levels >= 2;
    n2 = two ? min(meta->level_cnt[1], node_cap) : 0u;
    nin = two ? meta->pairs[1] : 0u;
    nin = nin < cap2 ? nin : cap2;
}

__global__ void k_lh_clear(lh_ws L, const crsh_meta *meta, uint64_t cap2, uint32_t node_cap)
{
    uint32_t n2;
    uint64_t nin;
    level2_sizes(meta, cap2, node_cap, n2, nin);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) {
        L.cnt[i] = 0;
        L.cursor[i] = 0;
    }
}

__global__ void k_lh_hist(const uint32_t *__restrict__ pnode, lh_ws L, const crsh_meta *meta, uint64_t cap2,
                          uint32_t node_cap)
{
    uint32_t n2;
    uint64_t nin;
    level2_sizes(meta, cap2, node_cap, n2, nin);
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nin;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t P = pnode[q];
        if (P < n2) atomicAdd(&L.cnt[P], 1u);
    }
}

__device__ __forceinline__ uint32_t chunks(uint32_t c) { return (c + LH_CHUNK - 1) / LH_CHUNK; }

// per tile of LH_TILE nodes: total pairs and total work items
__global__ __launch_bounds__(LH_THREADS) void k_lh_tiles(lh_ws L, const crsh_meta *meta, uint64_t cap2,
                                                         uint32_t node_cap)
{
    __shared__ uint64_t s_a[LH_WAVES], s_b[LH_WAVES];
    uint32_t n2;
    uint64_t nin;
    level2_sizes(meta, cap2, node_cap, n2, nin);
    const uint32_t base = blockIdx.x * LH_TILE;
    if (base >= n2) return;
    uint64_t a = 0, b = 0;
    for (uint32_t k = 0; k < LH_PER_THREAD; ++k) {
        const uint32_t P = base + threadIdx.x * LH_PER_THREAD + k;
        const uint32_t c = P < n2 ? L.cnt[P] : 0u;
        a += c;
        b += chunks(c);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane_id() == 0) {
        s_a[threadIdx.x / WAVE] = a;
        s_b[threadIdx.x / WAVE] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t ta = 0, tb = 0;
        for (uint32_t i = 0; i < LH_WAVES; ++i) {
            ta += s_a[i];
            tb += s_b[i];
        }
        L.tsum[2 * blockIdx.x] = ta;
        L.tsum[2 * blockIdx.x + 1] = tb;
    }
}

// exclusive scan of the tile sums in place (one block)
__global__ __launch_bounds__(1024) void k_lh_tilescan(lh_ws L, const crsh_meta *meta, uint64_t cap2,
                                                      uint32_t node_cap)
{
    __shared__ uint64_t s_scan[1024 / WAVE];
    __shared__ uint64_t s_ca, s_cb;
    uint32_t n2;
    uint64_t nin;
    level2_sizes(meta, cap2, node_cap, n2, nin);
    const uint32_t tiles = (n2 + LH_TILE - 1) / LH_TILE;
    if (threadIdx.x == 0) {
        s_ca = 0;
        s_cb = 0;
    }
    __syncthreads();
    for (uint32_t base = 0; base < tiles; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t a = i < tiles ? L.tsum[2 * i] : 0u;
        const uint64_t b = i < tiles ? L.tsum[2 * i + 1] : 0u;
        uint64_t ta, tb;
        const uint64_t ea = block_excl_scan<uint64_t, 1024 / WAVE>(a, s_scan, ta);
        const uint64_t eb = block_excl_scan<uint64_t, 1024 / WAVE>(b, s_scan, tb);
        const uint64_t ca = s_ca, cb = s_cb;
        if (i < tiles) {
            L.tsum[2 * i] = ca + ea;
            L.tsum[2 * i + 1] = cb + eb;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_ca = ca + ta;
            s_cb = cb + tb;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) L.n_items[0] = (uint32_t)min(s_cb, (uint64_t)0xFFFFFFFFu);
}

__global__ __launch_bounds__(LH_THREADS) void k_lh_apply(lh_ws L, const crsh_meta *meta, uint64_t cap2,
                                                         uint32_t node_cap)
{
    __shared__ uint64_t s_scan[LH_WAVES];
    uint32_t n2;
    uint64_t nin;
    level2_sizes(meta, cap2, node_cap, n2, nin);
    const uint32_t base = blockIdx.x * LH_TILE;
    if (base >= n2) return;
    const uint32_t first = base + threadIdx.x * LH_PER_THREAD;
    uint32_t c[LH_PER_THREAD];
    uint64_t a = 0, b = 0;
    for (uint32_t k = 0; k < LH_PER_THREAD; ++k) {
        c[k] = first + k < n2 ? L.cnt[first + k] : 0u;
        a += c[k];
        b += chunks(c[k]);
    }
    uint64_t ta, tb;
    uint64_t ea = block_excl_scan<uint64_t, LH_WAVES>(a, s_scan, ta);
    uint64_t eb = block_excl_scan<uint64_t, LH_WAVES>(b, s_scan, tb);
    ea += L.tsum[2 * blockIdx.x];
    eb += L.tsum[2 * blockIdx.x + 1];
    for (uint32_t k = 0; k < LH_PER_THREAD; ++k) {
        if (first + k < n2) {
            L.off[first + k] = ea;
            L.ib[first + k] = (uint32_t)eb;
        }
        ea += c[k];
        eb += chunks(c[k]);
    }
}

__global__ void k_lh_scatter(const uint32_t *__restrict__ ptri, const uint32_t *__restrict__ pnode, lh_ws L,
                             const crsh_meta *meta, uint64_t cap2, uint32_t node_cap)
{
    uint32_t n2;
    uint64_t nin;
    level2_sizes(meta, cap2, node_cap, n2, nin);
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nin;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t P = pnode[q];
        if (P < n2) {
            const uint64_t pos = L.off[P] + atomicAdd(&L.cursor[P], 1u);
            if (pos < cap2) L.bucket[pos] = ptri[q];
        }
    }
}

struct lh_args {
    const float *ox, *oy, *oz, *dx, *dy, *dz, *tmax;                        // sorted rays
    const float *ncx, *ncy, *ncz, *nr, *nax, *nay, *naz, *nc, *ntan, *nsec;  // nodes (level 1 first)
    unsigned long long *tkey;
    uint32_t B, F, log2G, ray_cap, m, node_cap;
    uint64_t cap2;
    float t_min;
};

template <int NF, bool BATCH>
__global__ __launch_bounds__(LH_THREADS) void k_leaf_hit(lh_args a, lh_ws L, crsh_meta *meta, batch_dev bd)
{
    constexpr uint32_t TB = WAVE / NF;   // triangles per Eq. 9 round of a wave
    __shared__ float4 s_o[LH_MAX_RAYS];
    __shared__ float4 s_d[LH_MAX_RAYS];
    __shared__ unsigned long long s_best[LH_MAX_RAYS];
    __shared__ uint32_t s_first[NF], s_count[NF];
    __shared__ uint64_t s_red[5][LH_WAVES];
    uint32_t n2;
    uint64_t nin;
    level2_sizes(meta, a.cap2, a.node_cap, n2, nin);
    const uint32_t items = n2 ? L.n_items[0] : 0u;
    const uint32_t n = min(meta->n_rays, a.ray_cap);
    const uint32_t n1 = meta->level_cnt[0];
    const uint32_t off2 = meta->level_off[1];
    const uint32_t l = lane_id();
    const uint32_t w = threadIdx.x / WAVE;
    const uint32_t NG = WAVE >> a.log2G;
    const uint32_t grp = l >> a.log2G;
    const uint32_t j = l & ((1u << a.log2G) - 1u);
    const uint32_t tk = l / NF;          // Eq. 9 slot of this lane: triangle tk of a round ...
    const uint32_t tc = l % NF;          // ... against child tc
    uint64_t tests = 0, hits = 0, finals = 0, upass = 0, uvpass = 0;
    for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
        const uint32_t P = last_at_most(n2, item, [&](uint32_t q) { return L.ib[q]; });
        const uint64_t pstart = L.off[P];
        const uint64_t pbeg = pstart + (uint64_t)(item - L.ib[P]) * LH_CHUNK;
        uint64_t pend = pstart + L.cnt[P];
        pend = pend < pbeg + LH_CHUNK ? pend : pbeg + LH_CHUNK;
        pend = pend < nin ? pend : nin;
        uint32_t c0, nc;
        float t_min = a.t_min;
        if constexpr (BATCH) {
            const uint32_t info = bd.node_info[off2 + P];
            c0 = bd.node_first[off2 + P];
            nc = info & INFO_COUNT_MASK;
            t_min = bd.frames[info >> INFO_FRAME_SHIFT].t_min;
        } else {
            c0 = P * a.F;
            nc = c0 < n1 ? min(a.F, n1 - c0) : 0u;
        }
        nc = min(nc, (uint32_t)NF);
        if (threadIdx.x < NF) {
            uint32_t first = 0, count = 0;
            const uint32_t leaf = c0 + threadIdx.x;
            if (threadIdx.x < nc && leaf < n1) {
                if constexpr (BATCH) {
                    first = bd.node_first[leaf];
                    count = bd.node_info[leaf] & INFO_COUNT_MASK;
                } else {
                    first = leaf * a.B;
                    count = first < n ? min(a.B, n - first) : 0u;
                }
            }
            s_first[threadIdx.x] = first;
            s_count[threadIdx.x] = min(count, a.B);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nc * a.B; i += LH_THREADS) {
            const uint32_t c = i / a.B, r = i - c * a.B;
            float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f), d = o;
            const uint32_t s = s_first[c] + r;
            if (r < s_count[c] && s < n) {
                o = make_float4(a.ox[s], a.oy[s], a.oz[s], a.tmax[s]);
                d = make_float4(a.dx[s], a.dy[s], a.dz[s], 0.0f);
            }
            s_o[i] = o;
            s_d[i] = d;
            s_best[i] = ~0ull;
        }
        float4 A = make_float4(0.0f, 0.0f, 0.0f, 0.0f), Bv = A;
        float S = -1.0f;
        const bool child = tc < nc && c0 + tc < n1;
        if (child) {
            const uint32_t q = c0 + tc;          // level 1 is first in the node arrays
            A = make_float4(a.ncx[q], a.ncy[q], a.ncz[q], a.nr[q]);
            Bv = make_float4(a.nax[q], a.nay[q], a.naz[q], a.ntan[q]);
            S = a.nc[q] > 0.0f ? a.nsec[q] : -1.0f;
        }
        __syncthreads();
        for (uint64_t b0 = pbeg + (uint64_t)w * TB; b0 < pend; b0 += (uint64_t)LH_WAVES * TB) {
            const uint64_t qi = b0 + tk;
            const bool valid = child && qi < pend;
            bool pass = false;
            if (valid) {
                const uint32_t t = L.bucket[qi];
                if (t < a.m) {
                    const float4 sp = L.tsph[t];
                    pass = packed_meets(A, Bv, S, mk(sp.x, sp.y, sp.z), sp.w);
                }
            }
            tests += valid ? 1u : 0u;
            hits += pass ? 1u : 0u;
            uint64_t mask = ballot(pass);
            while (mask) {
                // the next NG passing (triangle, child) pairs, one per lane group
                uint32_t mine = WAVE;
                for (uint32_t g = 0; g < NG && mask; ++g) {
                    const uint32_t bit = (uint32_t)__builtin_ctzll(mask);
                    mask &= mask - 1;
                    if (grp == g) mine = bit;
                }
                if (mine < WAVE) {
                    const uint32_t kk = mine / NF, cc = mine % NF;
                    if (j < s_count[cc]) {
                        ++finals;
                        const uint32_t tt = L.bucket[b0 + kk];
                        const tri_t tr = load_tri(L.tri, tt);
                        const uint32_t ri = cc * a.B + j;
                        const float4 o = s_o[ri], d = s_d[ri];
                        float th, uh, vh;
                        uint32_t checks;
                        if (moller_trumbore(mk(o.x, o.y, o.z), mk(d.x, d.y, d.z), t_min, o.w, tr, th, uh, vh,
                                            &checks))
                            atomicMin(&s_best[ri], hit_key(th, tt));
                        upass += (checks & MT_U) ? 1u : 0u;
                        uvpass += (checks & MT_UV) ? 1u : 0u;
                    }
                }
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nc * a.B; i += LH_THREADS) {
            const unsigned long long k = s_best[i];
            if (k != ~0ull) {
                const uint32_t c = i / a.B, r = i - c * a.B;
                atomicMin(&a.tkey[s_first[c] + r], k);
            }
        }
        __syncthreads();
    }
    tests = wave_sum(tests);
    hits = wave_sum(hits);
    finals = wave_sum(finals);
    upass = wave_sum(upass);
    uvpass = wave_sum(uvpass);
    if (l == 0) {
        s_red[0][w] = tests;
        s_red[1][w] = hits;
        s_red[2][w] = finals;
        s_red[3][w] = upass;
        s_red[4][w] = uvpass;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t[5] = {0, 0, 0, 0, 0};
        for (uint32_t i = 0; i < LH_WAVES; ++i)
            for (int k = 0; k < 5; ++k) t[k] += s_red[k][i];
        unsigned long long *dst[5] = {(unsigned long long *)&meta->tests[0], (unsigned long long *)&meta->hits[0],
                                      (unsigned long long *)&meta->final_tests,
                                      (unsigned long long *)&meta->final_u_pass,
                                      (unsigned long long *)&meta->final_uv_pass};
        for (int k = 0; k < 5; ++k)
            if (t[k]) atomicAdd(dst[k], (unsigned long long)t[k]);
    }
}

crsh_status leaf_hit_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle, int32_t merge,
                            const crsh_nodes *nodes, const crsh_pairs *level1, const crsh_pairs *level2,
                            const crsh_scene *scene, float t_min, crsh_hits *hits, crsh_meta *meta, void *ws,
                            size_t ws_bytes, const batch_dev *bd, int32_t hit_block, hipStream_t stream)
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
    const uint32_t slots = hit_slots(sorted->capacity, bd != nullptr);
    const size_t need = leaf_hit_ws_bytes(scene->m, nodes->capacity, level2->capacity, slots);
    if (ws_bytes < need) {
        set_error("crsh_leaf_hit: workspace too small (%zu < %zu)", ws_bytes, need);
        return CRSH_ERR_INVALID;
    }
    const lh_ws L = carve(ws, scene->m, nodes->capacity, level2->capacity, slots);
    const batch_dev b = bd ? *bd : batch_dev{};
    hit_prep_launch(scene, L.tri, stream);
    tri_spheres_launch(scene, 0, scene->m, L.tsph, stream);
    // level-1 pairs stored by a top-level pass at level 1
    hit_pairs_launch(sorted, L.tri, L.hs, level1, bundle, scene, t_min, hits, meta, bd, hit_block, stream);

    const uint64_t cap2 = level2->capacity;
    const uint32_t ncap = nodes->capacity;
    const uint32_t gn = std::max<uint32_t>(std::min<uint32_t>((ncap + 255) / 256, 2048), 1);
    const uint32_t gp = (uint32_t)std::max<uint64_t>(std::min<uint64_t>((cap2 + 255) / 256, 4096), 1);
    const uint32_t tiles = std::max<uint32_t>((ncap + LH_TILE - 1) / LH_TILE, 1);
    k_lh_clear<<<gn, 256, 0, stream>>>(L, meta, cap2, ncap);
    {
        prof_scope ps("k_lh_hist", stream);
        k_lh_hist<<<gp, 256, 0, stream>>>(level2->node, L, meta, cap2, ncap);
    }
    k_lh_tiles<<<tiles, LH_THREADS, 0, stream>>>(L, meta, cap2, ncap);
    k_lh_tilescan<<<1, 1024, 0, stream>>>(L, meta, cap2, ncap);
    k_lh_apply<<<tiles, LH_THREADS, 0, stream>>>(L, meta, cap2, ncap);
    {
        prof_scope ps("k_lh_scatter", stream);
        k_lh_scatter<<<gp, 256, 0, stream>>>(level2->tri, level2->node, L, meta, cap2, ncap);
    }
    uint32_t log2G = 0;
    while ((1u << log2G) < (uint32_t)bundle) ++log2G;
    lh_args a{sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, sorted->tmax,
              nodes->cx, nodes->cy, nodes->cz, nodes->r, nodes->ax, nodes->ay, nodes->az, nodes->c, nodes->tan,
              nodes->sec, hits->tkey, (uint32_t)bundle, (uint32_t)merge, log2G, sorted->capacity, scene->m,
              ncap, cap2, t_min};
    const uint32_t grid = 4096;
    {
        prof_scope ps("k_leaf_hit", stream);
        int nf = 2;
        while (nf < merge) nf *= 2;
#define CRSH_LH(NF)                                                                                   \
    (bd ? k_leaf_hit<NF, true><<<grid, LH_THREADS, 0, stream>>>(a, L, meta, b)                        \
        : k_leaf_hit<NF, false><<<grid, LH_THREADS, 0, stream>>>(a, L, meta, b))
        switch (nf) {
        case 2: CRSH_LH(2); break;
        case 4: CRSH_LH(4); break;
        case 8: CRSH_LH(8); break;
        default: CRSH_LH(16); break;
        }
#undef CRSH_LH
    }
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
    return leaf_hit_launch(sorted, sorted_ids, bundle, merge, nodes, &pairs[0], &pairs[1], scene, t_min, hits, meta,
                           ws, ws_bytes, nullptr, 256, stream);
}
