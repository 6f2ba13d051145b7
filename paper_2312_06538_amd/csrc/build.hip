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
#include "common.hpp"

namespace crsh {

struct cone {
    f3 x;
    float c, s;
};
struct sph {
    f3 c;
    float r;
};

__device__ __forceinline__ cone full_cone(f3 x)
{
    cone k;
    k.x = x;
    k.c = -1.0f;
    k.s = 0.0f;
    return k;
}

__device__ __forceinline__ bool is_full(const cone &k) { return !(k.c > 0.0f); }

// Widen by CONE_PAD radians (a first-order rotation of (c, s)); cones of 90
// degrees or more become the canonical full cone.
__device__ __forceinline__ cone widen(cone k)
{
    if (!(k.c > 0.0f)) return full_cone(k.x);
    cone o = k;
    o.c = k.c - CONE_PAD * k.s;
    o.s = k.s + CONE_PAD * k.c;
    if (!(o.c > 0.0f)) return full_cone(k.x);
    return o;
}

// Eq. 5-6: bisector axis; half-angle = half the axis angle + larger spread,
// by the angle-addition formulas on (cos, sin).
__device__ __forceinline__ cone merge_cones(const cone &a, const cone &b)
{
    if (is_full(a) || is_full(b)) return full_cone(a.x);
    f3 sum = a.x + b.x;
    float h = len(sum);
    if (!(h >= BISECT_MIN)) return full_cone(a.x);
    cone o;
    o.x = sum / h;
    float ch = h * 0.5f;
    float sh = len(a.x - b.x) * 0.5f;
    float cm = a.c, sm = a.s;
    if (b.s > a.s) {
        cm = b.c;
        sm = b.s;
    }
    o.c = ch * cm - sh * sm;
    o.s = sh * cm + ch * sm;
    return widen(o);
}

// Eq. 1-4: grow a cone to take in ray direction r.
__device__ __forceinline__ cone cone_take(const cone &k, f3 r)
{
    if (is_full(k)) return k;
    f3 nv = cross(k.x, r);
    float st = len(nv);
    float ct = dot(k.x, r);
    if (ct > 0.0f && (st == 0.0f || k.s * ct - k.c * st >= INSIDE_MARGIN)) return k;
    if (st == 0.0f || k.s * ct + k.c * st <= 0.0f) return full_cone(k.x);
    if (st < NEAR_PARALLEL) {
        cone rr;
        rr.x = r;
        rr.c = 1.0f;
        rr.s = 0.0f;
        return merge_cones(k, rr);
    }
    f3 q = -(cross(nv, k.x) / st);         // Eq. 1: away from r, orthogonal to x
    f3 e = k.x * k.c + q * k.s;            // Eq. 2: far edge
    f3 er = e + r;
    float h = len(er);
    if (!(h >= BISECT_MIN)) return full_cone(k.x);
    cone o;
    o.x = er / h;                          // Eq. 3
    o.c = dot(o.x, r);                     // Eq. 4
    o.s = len(e - r) * 0.5f;
    return widen(o);
}

__device__ __forceinline__ float grow_radius(f3 c, float r)
{
    float m = fmax2(fmax2(fabsf(c.x), fabsf(c.y)), fabsf(c.z));
    return r + SPHERE_PAD * (r + m);
}

// Eq. 7-8
__device__ __forceinline__ sph merge_spheres(const sph &a, const sph &b)
{
    sph o;
    o.c = (a.c + b.c) * 0.5f;
    float e = len(b.c - a.c) * 0.5f;
    o.r = grow_radius(o.c, e + fmax2(a.r, b.r));
    return o;
}

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

template <int NB>
__global__ __launch_bounds__(256) void k_build_leaf(const float *__restrict__ ox, const float *__restrict__ oy,
                                                    const float *__restrict__ oz, const float *__restrict__ dx,
                                                    const float *__restrict__ dy, const float *__restrict__ dz,
                                                    uint32_t B, nodes_dev nd, const crsh_meta *meta)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (meta->n_levels == 0 || j >= meta->level_cnt[0]) return;
    const uint32_t n = meta->n_rays;
    const uint32_t b = j * B;
    const uint32_t k = min(B, n - b);
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

template <int NF>
__global__ __launch_bounds__(256) void k_build_up(uint32_t lv, uint32_t F, nodes_dev nd, const crsh_meta *meta)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (lv >= meta->n_levels || j >= meta->level_cnt[lv]) return;
    const uint32_t below = meta->level_off[lv - 1];
    const uint32_t nb = meta->level_cnt[lv - 1];
    const uint32_t b = j * F;
    const uint32_t k = min(F, nb - b);
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

extern "C" crsh_status crsh_build(const crsh_rays *rays, const uint32_t *sorted_ids, int32_t bundle, int32_t merge,
                                  int32_t levels, crsh_nodes *nodes, crsh_rays *sorted, crsh_meta *meta,
                                  hipStream_t stream)
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
    k_build_info<<<1, 1, 0, stream>>>(meta, (uint32_t)bundle, (uint32_t)merge, (uint32_t)levels, nodes->capacity,
                                      rays->capacity);
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
    // launch bounds from the capacity; kernels read the real counts from meta
    uint64_t cnt = ((uint64_t)cap + bundle - 1) / bundle;
    uint32_t g = (uint32_t)((cnt + 255) / 256);
    if (g == 0) g = 1;
    switch (pow2_at_least(bundle)) {
    case 1: k_build_leaf<1><<<g, 256, 0, stream>>>(sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, bundle, nd, meta); break;
    case 2: k_build_leaf<2><<<g, 256, 0, stream>>>(sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, bundle, nd, meta); break;
    case 4: k_build_leaf<4><<<g, 256, 0, stream>>>(sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, bundle, nd, meta); break;
    case 8: k_build_leaf<8><<<g, 256, 0, stream>>>(sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, bundle, nd, meta); break;
    case 16: k_build_leaf<16><<<g, 256, 0, stream>>>(sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, bundle, nd, meta); break;
    default: k_build_leaf<32><<<g, 256, 0, stream>>>(sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, bundle, nd, meta); break;
    }
    int nf = pow2_at_least(merge);
    for (int lv = 1; lv < levels; ++lv) {
        cnt = (cnt + merge - 1) / merge;
        g = (uint32_t)((cnt + 255) / 256);
        if (g == 0) g = 1;
        switch (nf) {
        case 2: k_build_up<2><<<g, 256, 0, stream>>>(lv, merge, nd, meta); break;
        case 4: k_build_up<4><<<g, 256, 0, stream>>>(lv, merge, nd, meta); break;
        case 8: k_build_up<8><<<g, 256, 0, stream>>>(lv, merge, nd, meta); break;
        default: k_build_up<16><<<g, 256, 0, stream>>>(lv, merge, nd, meta); break;
        }
        if (cnt <= 1) break;
    }
    return hip_check(hipGetLastError(), "crsh_build launch");
}
