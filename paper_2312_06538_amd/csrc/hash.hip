// Stage 1: secondary-ray generation, trimming and hashing (Sec. 3.3.2).
//
// One thread per pixel.  Pass 1 counts the real rays of every pixel and sums
// them per block; a single-block scan turns block sums into block offsets;
// pass 2 regenerates the rays and writes them at block offset + the
// exclusive prefix inside the block, so ray ids are consecutive in (pixel,
// slot) order -- the trimmed arrays of Fig. 4 without a head-flag array.
#include <float.h>

#include "common.hpp"

namespace crsh {

struct raygen_dev {
    int32_t n_lights;
    float lx[CRSH_MAX_LIGHTS], ly[CRSH_MAX_LIGHTS], lz[CRSH_MAX_LIGHTS];
    float ex, ey, ez;
    const uint32_t *mat_flags;
    const float *mat_ior;
    int32_t n_mats;
    uint32_t types;
    float eps_off, eps_shadow;
    float lo[3], inv[3];
};

struct gbuf_dev {
    const float *px, *py, *pz, *nx, *ny, *nz;
    const int32_t *mat;
    uint32_t npix;
};

struct ray_t {
    f3 o, d;
    float tmax;
    uint32_t key;
};

// Octahedral map of a unit direction to a 2^k x 2^k grid.
__device__ __forceinline__ void octahedral(f3 d, int k, uint32_t &u, uint32_t &v)
{
    float a = (fabsf(d.x) + fabsf(d.y)) + fabsf(d.z);
    float px = d.x / a;
    float py = d.y / a;
    if (d.z < 0.0f) {
        float sx = px >= 0.0f ? 1.0f : -1.0f;
        float sy = py >= 0.0f ? 1.0f : -1.0f;
        float fx = (1.0f - fabsf(py)) * sx;
        float fy = (1.0f - fabsf(px)) * sy;
        px = fx;
        py = fy;
    }
    const float half = (float)(1u << (k - 1));
    const float top = (float)((1u << k) - 1u);
    float fu = floorf((px + 1.0f) * half);
    float fv = floorf((py + 1.0f) * half);
    fu = fu >= 0.0f ? fu : 0.0f;
    fv = fv >= 0.0f ? fv : 0.0f;
    fu = fu > top ? top : fu;
    fv = fv > top ? top : fv;
    u = (uint32_t)fu;
    v = (uint32_t)fv;
}

// Spread the low 16 bits of x to the even bit positions.
__device__ __forceinline__ uint32_t spread2(uint32_t x)
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Spread the low 10 bits of x to every third bit position.
__device__ __forceinline__ uint32_t spread3(uint32_t x)
{
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t cell64(float o, float lo, float inv)
{
    float f = floorf(((o - lo) * inv) * 64.0f);
    f = f >= 0.0f ? f : 0.0f;
    f = f > 63.0f ? 63.0f : f;
    return (uint32_t)f;
}

// Shadow: 00 | light:2 | octahedral(14+14).  Bounce: type:2 | cell:18 | octahedral(6+6).
__device__ __forceinline__ uint32_t key_shadow(uint32_t light, f3 d)
{
    uint32_t u, v;
    octahedral(d, 14, u, v);
    return (light << 28) | spread2(u) | (spread2(v) << 1);
}

__device__ __forceinline__ uint32_t key_bounce(uint32_t type, f3 o, f3 d, const raygen_dev &g)
{
    uint32_t cx = cell64(o.x, g.lo[0], g.inv[0]);
    uint32_t cy = cell64(o.y, g.lo[1], g.inv[1]);
    uint32_t cz = cell64(o.z, g.lo[2], g.inv[2]);
    uint32_t u, v;
    octahedral(d, 6, u, v);
    uint32_t cell = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
    return (type << 30) | (cell << 12) | spread2(u) | (spread2(v) << 1);
}

// Generates slot s of a pixel (shadow rays of lights 0..L-1, reflection,
// refraction); returns false for a hole.
__device__ __forceinline__ bool make_slot(int s, f3 P, f3 N, uint32_t flags, float ior, const raygen_dev &g,
                                          ray_t &r)
{
    if (s < g.n_lights) {
        if (!(g.types & CRSH_RAY_SHADOW)) return false;
        f3 L = mk(g.lx[s], g.ly[s], g.lz[s]);
        f3 d0 = P - L;
        float l = len(d0);
        if (!(l > g.eps_shadow)) return false;
        r.o = L;                  // origin moved to the light
        r.d = d0 / l;
        r.tmax = l - g.eps_shadow;
        r.key = key_shadow((uint32_t)s, r.d);
        return true;
    }
    f3 E = mk(g.ex, g.ey, g.ez);
    f3 v0 = P - E;
    f3 v = v0 / len(v0);
    float k = dot(v, N);
    if (s == g.n_lights) {
        if (!(g.types & CRSH_RAY_REFLECT) || !(flags & CRSH_MAT_REFLECTIVE)) return false;
        f3 rr = v - N * (2.0f * k);
        r.d = rr / len(rr);
        r.o = P + N * g.eps_off;
        r.tmax = FLT_MAX;
        r.key = key_bounce(1u, r.o, r.d, g);
        return true;
    }
    if (!(g.types & CRSH_RAY_REFRACT) || !(flags & CRSH_MAT_REFRACTIVE)) return false;
    float eta = 1.0f / ior;
    float ci = -k;
    float k2 = 1.0f - (eta * eta) * (1.0f - ci * ci);
    if (k2 < 0.0f) return false;    // total internal reflection
    float b = eta * ci - sqrtf(k2);
    f3 t = v * eta + N * b;
    r.d = t / len(t);
    r.o = P - N * g.eps_off;
    r.tmax = FLT_MAX;
    r.key = key_bounce(2u, r.o, r.d, g);
    return true;
}

struct pixel_t {
    f3 P, N;
    uint32_t flags;
    float ior;
    bool hit;
};

__device__ __forceinline__ pixel_t load_pixel(const gbuf_dev &gb, const raygen_dev &g, uint32_t p)
{
    pixel_t px;
    px.hit = false;
    if (p >= gb.npix) return px;
    int32_t m = gb.mat[p];
    if (m < 0) return px;
    px.hit = true;
    px.P = mk(gb.px[p], gb.py[p], gb.pz[p]);
    px.N = mk(gb.nx[p], gb.ny[p], gb.nz[p]);
    px.flags = m < g.n_mats ? g.mat_flags[m] : 0u;
    px.ior = m < g.n_mats ? g.mat_ior[m] : 1.0f;
    return px;
}

__global__ __launch_bounds__(HASH_BLOCK) void k_hash_count(gbuf_dev gb, raygen_dev g, uint32_t *block_sums)
{
    __shared__ uint32_t red[HASH_BLOCK / WAVE];
    uint32_t p = blockIdx.x * HASH_BLOCK + threadIdx.x;
    pixel_t px = load_pixel(gb, g, p);
    uint32_t c = 0;
    if (px.hit) {
        for (int s = 0; s < g.n_lights + 2; ++s) {
            ray_t r;
            c += make_slot(s, px.P, px.N, px.flags, px.ior, g, r) ? 1u : 0u;
        }
    }
    c = wave_sum(c);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < HASH_BLOCK / WAVE; ++i) t += red[i];
        block_sums[blockIdx.x] = t;
    }
}

// Exclusive scan of nb block sums in place (one block of 1024 threads).
__global__ __launch_bounds__(1024) void k_hash_scan(uint32_t *block_sums, uint32_t nb, crsh_meta *meta,
                                                    uint32_t capacity)
{
    __shared__ uint32_t scratch[1024 / WAVE];
    __shared__ uint32_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += 1024) {
        uint32_t i = base + threadIdx.x;
        uint32_t v = i < nb ? block_sums[i] : 0u;
        uint32_t total;
        uint32_t ex = block_excl_scan<uint32_t, 1024 / WAVE>(v, scratch, total);
        uint32_t carry = carry_s;
        if (i < nb) block_sums[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint32_t n = carry_s;
        meta->rays_required = n;
        if (n > capacity) {
            atomicOr(&meta->status, CRSH_OVERFLOW_RAYS);
            n = capacity;
        }
        meta->n_rays = n;
    }
}

struct rays_dev {
    float *ox, *oy, *oz, *dx, *dy, *dz, *tmax;
    uint32_t *pix;
    uint32_t cap;
};

__global__ __launch_bounds__(HASH_BLOCK) void k_hash_emit(gbuf_dev gb, raygen_dev g, const uint32_t *block_off,
                                                          rays_dev out, uint32_t *keys, uint32_t *ids)
{
    __shared__ uint32_t scratch[HASH_BLOCK / WAVE];
    uint32_t p = blockIdx.x * HASH_BLOCK + threadIdx.x;
    pixel_t px = load_pixel(gb, g, p);
    uint32_t c = 0;
    if (px.hit) {
        for (int s = 0; s < g.n_lights + 2; ++s) {
            ray_t r;
            c += make_slot(s, px.P, px.N, px.flags, px.ior, g, r) ? 1u : 0u;
        }
    }
    uint32_t total;
    uint32_t id = block_off[blockIdx.x] + block_excl_scan<uint32_t, HASH_BLOCK / WAVE>(c, scratch, total);
    if (!px.hit || c == 0) return;
    for (int s = 0; s < g.n_lights + 2; ++s) {
        ray_t r;
        if (!make_slot(s, px.P, px.N, px.flags, px.ior, g, r)) continue;
        if (id < out.cap) {
            out.ox[id] = r.o.x;
            out.oy[id] = r.o.y;
            out.oz[id] = r.o.z;
            out.dx[id] = r.d.x;
            out.dy[id] = r.d.y;
            out.dz[id] = r.d.z;
            out.tmax[id] = r.tmax;
            out.pix[id] = p;
            keys[id] = r.key;
            ids[id] = id;
        }
        ++id;
    }
}

}  // namespace crsh

using namespace crsh;

extern "C" crsh_status crsh_hash(const crsh_gbuf *gbuf, const crsh_raygen *rg, crsh_rays *out, uint32_t *keys,
                                 uint32_t *ids, crsh_meta *meta, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!gbuf || !rg || !out || !keys || !ids || !meta || !ws) {
        set_error("crsh_hash: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (gbuf->w <= 0 || gbuf->h <= 0 || !gbuf->px || !gbuf->py || !gbuf->pz || !gbuf->nx || !gbuf->ny ||
        !gbuf->nz || !gbuf->mat) {
        set_error("crsh_hash: empty or incomplete primary-hit buffer");
        return CRSH_ERR_INVALID;
    }
    if (rg->n_lights < 0 || rg->n_lights > CRSH_MAX_LIGHTS || rg->n_mats < 0 ||
        (rg->n_mats > 0 && (!rg->mat_flags || !rg->mat_ior))) {
        set_error("crsh_hash: bad ray-generation parameters");
        return CRSH_ERR_INVALID;
    }
    if (!out->ox || !out->oy || !out->oz || !out->dx || !out->dy || !out->dz || !out->tmax || !out->pix) {
        set_error("crsh_hash: incomplete ray arrays");
        return CRSH_ERR_INVALID;
    }
    uint64_t npix = (uint64_t)gbuf->w * (uint64_t)gbuf->h;
    if (npix >= (1ull << 31)) {
        set_error("crsh_hash: too many pixels");
        return CRSH_ERR_INVALID;
    }
    if (ws_bytes < hash_ws_bytes(npix)) {
        set_error("crsh_hash: workspace too small (%zu < %zu)", ws_bytes, hash_ws_bytes(npix));
        return CRSH_ERR_INVALID;
    }
    gbuf_dev gb{gbuf->px, gbuf->py, gbuf->pz, gbuf->nx, gbuf->ny, gbuf->nz, gbuf->mat, (uint32_t)npix};
    raygen_dev g;
    g.n_lights = rg->n_lights;
    for (int i = 0; i < CRSH_MAX_LIGHTS; ++i) {
        g.lx[i] = rg->lights[i][0];
        g.ly[i] = rg->lights[i][1];
        g.lz[i] = rg->lights[i][2];
    }
    g.ex = rg->eye[0];
    g.ey = rg->eye[1];
    g.ez = rg->eye[2];
    g.mat_flags = rg->mat_flags;
    g.mat_ior = rg->mat_ior;
    g.n_mats = rg->n_mats;
    g.types = rg->ray_types;
    g.eps_off = rg->eps_off;
    g.eps_shadow = rg->eps_shadow;
    for (int i = 0; i < 3; ++i) {
        g.lo[i] = rg->lo[i];
        g.inv[i] = rg->inv_ext[i];
    }
    uint32_t nb = (uint32_t)((npix + HASH_BLOCK - 1) / HASH_BLOCK);
    uint32_t *blocks = (uint32_t *)ws;
    {
        prof_scope ps("k_hash_count", stream);
        k_hash_count<<<nb, HASH_BLOCK, 0, stream>>>(gb, g, blocks);
    }
    k_hash_scan<<<1, 1024, 0, stream>>>(blocks, nb, meta, out->capacity);
    rays_dev rd{out->ox, out->oy, out->oz, out->dx, out->dy, out->dz, out->tmax, out->pix, out->capacity};
    {
        prof_scope ps("k_hash_emit", stream);
        k_hash_emit<<<nb, HASH_BLOCK, 0, stream>>>(gb, g, blocks, rd, keys, ids);
    }
    return hip_check(hipGetLastError(), "crsh_hash launch");
}
