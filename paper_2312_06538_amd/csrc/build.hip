// Stage 3: hierarchy creation (Sec. 3.3.6, Eq. 1-8).
//
// k_build_info  node counts of every level from the ray count (device side,
//               so the frame needs no host round trip);
// k_permute     rays gathered into sorted order (coalesced writes); the leaf
//               kernel and the final tests then read them contiguously;
// k_build_leaf  one thread per level-1 node: the compact cone of its B rays
//               added one at a time in sorted order (Eq. 1-4) and the sphere
//               of their origins as a balanced pairwise tree (Eq. 7-8);
// k_build_up    one thread per upper node: balanced pairwise trees of its F
//               children's spheres (Eq. 7-8) and cones (Eq. 5-6).
// Trees are unrolled over a power-of-two slot count, so every slot index is a
// compile-time constant and the nodes stay in registers.
//
// Batched form: k_batch_levels sizes every frame's levels (the same rule as
// k_build_info, per frame) and lays each level out frame by frame; the leaf
// and upper kernels find their frame and take their rays / children from the
// frame's ranges, and record each node's first ray or child and its count
// (with the frame) for the traversal and the final tests.
#include "batch.hpp"
#include "bounds.hpp"

namespace crsh {

struct nodes_dev {
    float *cx, *cy, *cz, *r, *ax, *ay, *az, *c, *s, *tan, *sec;
    uint32_t cap;
};

__device__ __forceinline__ void put_node(const nodes_dev &nd, uint32_t i, const sph &sp, const cone &k)
{
    nd.cx[i] = sp.c.x;
    nd.cy[i] = sp.c.y;
    nd.cz[i] = sp.c.z;
    nd.r[i] = sp.r;
    nd.ax[i] = k.x.x;
    nd.ay[i] = k.x.y;
    nd.az[i] = k.x.z;
    nd.c[i] = k.c;
    nd.s[i] = k.s;
    bool open = k.c > 0.0f;
    nd.tan[i] = open ? k.s / k.c : 0.0f;
    nd.sec[i] = open ? 1.0f / k.c : 0.0f;
}

__global__ void k_build_info(crsh_meta *meta, uint32_t B, uint32_t F, uint32_t levels, uint32_t node_cap,
                             uint32_t ray_cap)
{
    uint32_t n = min(meta->n_rays, ray_cap);
    meta->n_rays = n;
    uint32_t nl = 0, total = 0;
    if (n > 0) {
        uint32_t c = (n + B - 1) / B;
        meta->level_cnt[0] = c;
        meta->level_off[0] = 0;
        total = c;
        nl = 1;
        while (nl < levels && c > 1) {
            c = (c + F - 1) / F;
            meta->level_off[nl] = total;
            meta->level_cnt[nl] = c;
            total += c;
            ++nl;
        }
    }
    for (uint32_t k = nl; k < CRSH_MAX_LEVELS; ++k) {
        meta->level_cnt[k] = 0;
        meta->level_off[k] = total;
    }
    meta->nodes_required = total;
    if (total > node_cap) {
        atomicOr(&meta->status, CRSH_OVERFLOW_NODES);
        nl = 0;                      // nothing is built; the host regrows
    }
    meta->n_levels = nl;
}

// One thread per frame (at most CRSH_MAX_FRAMES frames, one block).
__global__ __launch_bounds__(256) void k_batch_levels(batch_dev bd, crsh_meta *meta, uint32_t B, uint32_t F,
                                                      uint32_t levels, uint32_t node_cap, uint32_t ray_cap)
{
    __shared__ uint32_t scratch[256 / WAVE];
    __shared__ uint32_t s_total[CRSH_MAX_LEVELS];
    __shared__ uint32_t s_nl;
    const uint32_t f = threadIdx.x;
    const bool live = f < bd.n_frames;
    const uint32_t n = min(meta->n_rays, ray_cap);
    if (f == 0) s_nl = 0;
    uint32_t rb = live ? min(bd.fm[f].ray_begin, n) : n;
    uint32_t re = (f + 1 < bd.n_frames) ? min(bd.fm[f + 1].ray_begin, n) : n;
    const uint32_t nr = (live && re > rb) ? re - rb : 0u;
    __syncthreads();
    uint32_t nl = 0, c = 0;
    for (uint32_t k = 0; k < CRSH_MAX_LEVELS; ++k) {
        // the plain rule per frame: ceil(n / B) leaves, then ceil(c / F) while
        // under `levels` levels and more than one node
        if (k == 0) {
            c = (nr + B - 1) / B;
            nl = nr ? 1u : 0u;
        } else if (nl == k && k < levels && c > 1) {
            c = (c + F - 1) / F;
            nl = k + 1;
        }
        const uint32_t ck = k < nl ? c : 0u;
        uint32_t total;
        const uint32_t base = block_excl_scan<uint32_t, 256 / WAVE>(ck, scratch, total);
        if (live) {
            bd.fm[f].level_base[k] = base;
            bd.fm[f].level_cnt[k] = ck;
        }
        if (f == 0) s_total[k] = total;
    }
    if (live) atomicMax(&s_nl, nl);
    __syncthreads();
    uint32_t total = 0;
    for (uint32_t k = 0; k < CRSH_MAX_LEVELS; ++k) total += s_total[k];
    const bool over = total > node_cap;
    if (live) {
        bd.fm[f].ray_begin = rb;
        bd.fm[f].n_rays = nr;
        bd.fm[f].n_levels = over ? 0u : nl;
    }
    if (f == 0) {
        uint32_t off = 0;
        for (uint32_t k = 0; k < CRSH_MAX_LEVELS; ++k) {
            meta->level_off[k] = off;
            meta->level_cnt[k] = s_total[k];
            off += s_total[k];
        }
        meta->n_rays = n;
        meta->nodes_required = total;
        if (over) atomicOr(&meta->status, CRSH_OVERFLOW_NODES);
        meta->n_levels = over ? 0u : s_nl;
    }
}

struct rays_in {
    const float *ox, *oy, *oz, *dx, *dy, *dz, *tmax;
    const uint32_t *pix;
};
struct rays_out {
    float *ox, *oy, *oz, *dx, *dy, *dz, *tmax;
    uint32_t *pix;
};

__global__ void k_permute(rays_in in, const uint32_t *sorted_ids, rays_out out, const crsh_meta *meta,
                          uint32_t cap)
{
    uint32_t n = meta->n_rays;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        uint32_t id = sorted_ids[s];
        if (id >= cap) id = 0;      // ids come from the sort: never taken
        out.ox[s] = in.ox[id];
        out.oy[s] = in.oy[id];
        out.oz[s] = in.oz[id];
        out.dx[s] = in.dx[id];
        out.dy[s] = in.dy[id];
        out.dz[s] = in.dz[id];
        out.tmax[s] = in.tmax[id];
        if (out.pix) out.pix[s] = in.pix ? in.pix[id] : 0u;
    }
}

template <int NB, bool BATCH>
__global__ __launch_bounds__(256) void k_build_leaf(const float *__restrict__ ox, const float *__restrict__ oy,
                                                    const float *__restrict__ oz, const float *__restrict__ dx,
                                                    const float *__restrict__ dy, const float *__restrict__ dz,
                                                    uint32_t B, nodes_dev nd, const crsh_meta *meta, batch_dev bd)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (meta->n_levels == 0 || j >= meta->level_cnt[0]) return;
    uint32_t b, k;
    if constexpr (BATCH) {
        const uint32_t f = frame_of_node(bd, 0, j);
        const uint32_t local = (j - bd.fm[f].level_base[0]) * B;
        b = bd.fm[f].ray_begin + local;
        k = min(B, bd.fm[f].n_rays - local);
        bd.node_first[j] = b;
        bd.node_info[j] = k | (f << INFO_FRAME_SHIFT);
    } else {
        b = j * B;
        k = min(B, meta->n_rays - b);
    }
    sph sp[NB];
    cone kc;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if ((uint32_t)i < k) {
            uint32_t s = b + i;
            sp[i].c = mk(ox[s], oy[s], oz[s]);
            sp[i].r = 0.0f;
            f3 d = mk(dx[s], dy[s], dz[s]);
            if (i == 0) {
                kc.x = d;
                kc.c = 1.0f;
                kc.s = 0.0f;
            } else {
                kc = cone_take(kc, d);
            }
        }
    }
#pragma unroll
    for (int w = 1; w < NB; w *= 2) {
#pragma unroll
        for (int i = 0; i + w < NB; i += 2 * w)
            if ((uint32_t)(i + w) < k) sp[i] = merge_spheres(sp[i], sp[i + w]);
    }
    put_node(nd, j, sp[0], kc);
}

template <int NF, bool BATCH>
__global__ __launch_bounds__(256) void k_build_up(uint32_t lv, uint32_t F, nodes_dev nd, const crsh_meta *meta,
                                                  batch_dev bd)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (lv >= meta->n_levels || j >= meta->level_cnt[lv]) return;
    const uint32_t below = meta->level_off[lv - 1];
    uint32_t b, k;
    if constexpr (BATCH) {
        const uint32_t f = frame_of_node(bd, lv, j);
        const uint32_t local = (j - bd.fm[f].level_base[lv]) * F;
        b = bd.fm[f].level_base[lv - 1] + local;
        k = min(F, bd.fm[f].level_cnt[lv - 1] - local);
        bd.node_first[meta->level_off[lv] + j] = b;
        bd.node_info[meta->level_off[lv] + j] = k | (f << INFO_FRAME_SHIFT);
    } else {
        b = j * F;
        k = min(F, meta->level_cnt[lv - 1] - b);
    }
    sph sp[NF];
    cone kc[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        if ((uint32_t)i < k) {
            uint32_t q = below + b + i;
            sp[i].c = mk(nd.cx[q], nd.cy[q], nd.cz[q]);
            sp[i].r = nd.r[q];
            kc[i].x = mk(nd.ax[q], nd.ay[q], nd.az[q]);
            kc[i].c = nd.c[q];
            kc[i].s = nd.s[q];
        }
    }
#pragma unroll
    for (int w = 1; w < NF; w *= 2) {
#pragma unroll
        for (int i = 0; i + w < NF; i += 2 * w) {
            if ((uint32_t)(i + w) < k) {
                sp[i] = merge_spheres(sp[i], sp[i + w]);
                kc[i] = merge_cones(kc[i], kc[i + w]);
            }
        }
    }
    put_node(nd, meta->level_off[lv] + j, sp[0], kc[0]);
}

static int pow2_at_least(int x)
{
    int p = 1;
    while (p < x) p *= 2;
    return p;
}

}  // namespace crsh

using namespace crsh;

namespace crsh {

crsh_status build_launch(const crsh_rays *rays, const uint32_t *sorted_ids, int32_t bundle, int32_t merge,
                         int32_t levels, crsh_nodes *nodes, crsh_rays *sorted, crsh_meta *meta,
                         const batch_dev *bd, hipStream_t stream)
{
    if (!rays || !sorted_ids || !nodes || !sorted || !meta) {
        set_error("crsh_build: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (bundle < 1 || bundle > 32 || merge < 2 || merge > CRSH_MAX_MERGE || levels < 1 ||
        levels > CRSH_MAX_LEVELS) {
        set_error("crsh_build: bundle must be in [1,32], merge in [2,%d], levels in [1,%d]", CRSH_MAX_MERGE,
                  CRSH_MAX_LEVELS);
        return CRSH_ERR_INVALID;
    }
    if (!rays->ox || !rays->oy || !rays->oz || !rays->dx || !rays->dy || !rays->dz || !rays->tmax ||
        !sorted->ox || !sorted->oy || !sorted->oz || !sorted->dx || !sorted->dy || !sorted->dz || !sorted->tmax) {
        set_error("crsh_build: incomplete ray arrays");
        return CRSH_ERR_INVALID;
    }
    if (sorted->capacity < rays->capacity) {
        set_error("crsh_build: sorted-ray capacity below the ray capacity");
        return CRSH_ERR_INVALID;
    }
    if (!nodes->cx || !nodes->cy || !nodes->cz || !nodes->r || !nodes->ax || !nodes->ay || !nodes->az ||
        !nodes->c || !nodes->s || !nodes->tan || !nodes->sec) {
        set_error("crsh_build: incomplete node arrays");
        return CRSH_ERR_INVALID;
    }
    const batch_dev b = bd ? *bd : batch_dev{};
    if (bd)
        k_batch_levels<<<1, 256, 0, stream>>>(b, meta, (uint32_t)bundle, (uint32_t)merge, (uint32_t)levels,
                                               nodes->capacity, rays->capacity);
    else
        k_build_info<<<1, 1, 0, stream>>>(meta, (uint32_t)bundle, (uint32_t)merge, (uint32_t)levels,
                                          nodes->capacity, rays->capacity);
    rays_in ri{rays->ox, rays->oy, rays->oz, rays->dx, rays->dy, rays->dz, rays->tmax, rays->pix};
    rays_out ro{sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, sorted->tmax, sorted->pix};
    uint32_t cap = rays->capacity;
    uint32_t pb = std::min<uint32_t>((cap + 255) / 256, 4096);
    if (pb == 0) pb = 1;
    {
        prof_scope ps("k_permute", stream);
        k_permute<<<pb, 256, 0, stream>>>(ri, sorted_ids, ro, meta, cap);
    }
    nodes_dev nd{nodes->cx, nodes->cy, nodes->cz, nodes->r, nodes->ax, nodes->ay, nodes->az,
                 nodes->c, nodes->s, nodes->tan, nodes->sec, nodes->capacity};
    // launch bounds from the capacity (every frame may add one partial node
    // per level); kernels read the real counts from meta
    const uint64_t extra = bd ? bd->n_frames : 0;
    uint64_t cnt = ((uint64_t)cap + bundle - 1) / bundle + extra;
    uint32_t g = (uint32_t)std::min<uint64_t>((cnt + 255) / 256, 1u << 22);
    if (g == 0) g = 1;
    const float *sx = sorted->ox, *sy = sorted->oy, *sz = sorted->oz;
    const float *tx = sorted->dx, *ty = sorted->dy, *tz = sorted->dz;
#define CRSH_LEAF(NB)                                                                                      \
    (bd ? k_build_leaf<NB, true><<<g, 256, 0, stream>>>(sx, sy, sz, tx, ty, tz, bundle, nd, meta, b)       \
        : k_build_leaf<NB, false><<<g, 256, 0, stream>>>(sx, sy, sz, tx, ty, tz, bundle, nd, meta, b))
    switch (pow2_at_least(bundle)) {
    case 1: CRSH_LEAF(1); break;
    case 2: CRSH_LEAF(2); break;
    case 4: CRSH_LEAF(4); break;
    case 8: CRSH_LEAF(8); break;
    case 16: CRSH_LEAF(16); break;
    default: CRSH_LEAF(32); break;
    }
#undef CRSH_LEAF
    int nf = pow2_at_least(merge);
#define CRSH_UP(NF)                                                                                        \
    (bd ? k_build_up<NF, true><<<g, 256, 0, stream>>>(lv, merge, nd, meta, b)                             \
        : k_build_up<NF, false><<<g, 256, 0, stream>>>(lv, merge, nd, meta, b))
    for (int lv = 1; lv < levels; ++lv) {
        cnt = (cnt + merge - 1) / merge + extra;
        g = (uint32_t)std::min<uint64_t>((cnt + 255) / 256, 1u << 22);
        if (g == 0) g = 1;
        switch (nf) {
        case 2: CRSH_UP(2); break;
        case 4: CRSH_UP(4); break;
        case 8: CRSH_UP(8); break;
        default: CRSH_UP(16); break;
        }
        if (!bd && cnt <= 1) break;
    }
#undef CRSH_UP
    return hip_check(hipGetLastError(), "crsh_build launch");
}

}  // namespace crsh

extern "C" crsh_status crsh_build(const crsh_rays *rays, const uint32_t *sorted_ids, int32_t bundle, int32_t merge,
                                  int32_t levels, crsh_nodes *nodes, crsh_rays *sorted, crsh_meta *meta,
                                  hipStream_t stream)
{
    return build_launch(rays, sorted_ids, bundle, merge, levels, nodes, sorted, meta, nullptr, stream);
}
