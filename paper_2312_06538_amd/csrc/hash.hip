// Stage 1: secondary-ray generation, trimming and hashing (Sec. 3.3.2).
//
// One thread per pixel.  Pass 1 counts the real rays of every pixel and sums
// them per block; a single-block scan turns block sums into block offsets;
// pass 2 regenerates the rays and writes them at block offset + the
// exclusive prefix inside the block, so ray ids are consecutive in (pixel,
// slot) order -- the trimmed arrays of Fig. 4 without a head-flag array.
// In a batch every pixel takes the ray-generation parameters of its frame;
// frames are consecutive pixel ranges, so each frame's rays are consecutive
// ids and the thread of a frame's first pixel records where they start.
#include <float.h>

#include <mutex>

#include "batch.hpp"
#include "raygen.hpp"

namespace crsh {

__device__ __forceinline__ raygen_dev frame_raygen(const batch_dev &b, uint32_t f)
{
    const crsh_frame &fr = b.frames[f];
    raygen_dev g;
    g.n_lights = min(max(fr.n_lights, 0), CRSH_MAX_LIGHTS);
    for (int i = 0; i < CRSH_MAX_LIGHTS; ++i) {
        g.lx[i] = fr.lights[i][0];
        g.ly[i] = fr.lights[i][1];
        g.lz[i] = fr.lights[i][2];
    }
    g.ex = fr.eye[0];
    g.ey = fr.eye[1];
    g.ez = fr.eye[2];
    g.mat_flags = b.mat_flags + fr.mat_begin;
    g.mat_ior = b.mat_ior + fr.mat_begin;
    g.n_mats = (int32_t)fr.n_mats;
    g.types = fr.ray_types;
    g.eps_off = fr.eps_off;
    g.eps_shadow = fr.eps_shadow;
    for (int i = 0; i < 3; ++i) {
        g.lo[i] = fr.lo[i];
        g.inv[i] = fr.inv_ext[i];
    }
    return g;
}

// Where a thread's surface point comes from.
enum : int { SRC_GBUF = 0, SRC_BATCH = 1, SRC_BOUNCE = 2 };

struct src_dev {
    gbuf_dev gb;
    batch_dev bd;
    bounce_dev bo;
    uint32_t n;        // threads to cover (pixels, or parent-ray capacity)
};

template <int SRC>
__device__ __forceinline__ pixel_t load_point(const src_dev &src, const raygen_dev &g0, uint32_t p, raygen_dev &g,
                                              uint32_t &f)
{
    f = 0;
    g = g0;
    if constexpr (SRC == SRC_BATCH) {
        if (p < src.gb.npix) {
            f = frame_of_pixel(src.bd, p);
            g = frame_raygen(src.bd, f);
        }
    }
    if constexpr (SRC == SRC_BOUNCE)
        return load_bounce(src.bo, g, p);
    else
        return load_pixel(src.gb, g, p);
}

template <int SRC>
__global__ __launch_bounds__(HASH_BLOCK) void k_hash_count(src_dev src, raygen_dev g0, uint32_t *block_sums)
{
    __shared__ uint32_t red[HASH_BLOCK / WAVE];
    uint32_t p = blockIdx.x * HASH_BLOCK + threadIdx.x;
    uint32_t f;
    raygen_dev g;
    const pixel_t px = load_point<SRC>(src, g0, p, g, f);
    uint32_t c = 0;
    if (px.hit) {
        for (int s = 0; s < g.n_lights + 2; ++s) {
            ray_t r;
            c += make_slot(s, px.P, px.N, px.v, px.flags, px.ior, g, r) ? 1u : 0u;
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
    uint32_t *frame;
    uint32_t cap;
};

template <int SRC>
__global__ __launch_bounds__(HASH_BLOCK) void k_hash_emit(src_dev src, raygen_dev g0, const uint32_t *block_off,
                                                          rays_dev out, uint32_t *keys, uint32_t *ids)
{
    __shared__ uint32_t scratch[HASH_BLOCK / WAVE];
    uint32_t p = blockIdx.x * HASH_BLOCK + threadIdx.x;
    uint32_t f;
    raygen_dev g;
    const pixel_t px = load_point<SRC>(src, g0, p, g, f);
    uint32_t c = 0;
    if (px.hit) {
        for (int s = 0; s < g.n_lights + 2; ++s) {
            ray_t r;
            c += make_slot(s, px.P, px.N, px.v, px.flags, px.ior, g, r) ? 1u : 0u;
        }
    }
    uint32_t total;
    uint32_t id = block_off[blockIdx.x] + block_excl_scan<uint32_t, HASH_BLOCK / WAVE>(c, scratch, total);
    if constexpr (SRC == SRC_BATCH) {
        if (p < src.gb.npix && p == src.bd.frames[f].pix_begin) src.bd.fm[f].ray_begin = id;
    }
    if (!px.hit || c == 0) return;
    for (int s = 0; s < g.n_lights + 2; ++s) {
        ray_t r;
        if (!make_slot(s, px.P, px.N, px.v, px.flags, px.ior, g, r)) continue;
        if (id < out.cap) {
            out.ox[id] = r.o.x;
            out.oy[id] = r.o.y;
            out.oz[id] = r.o.z;
            out.dx[id] = r.d.x;
            out.dy[id] = r.d.y;
            out.dz[id] = r.d.z;
            out.tmax[id] = r.tmax;
            out.pix[id] = px.pix;
            keys[id] = r.key;
            ids[id] = id;
            if constexpr (SRC == SRC_BATCH) out.frame[id] = f;
        }
        ++id;
    }
}

static raygen_dev to_device(const crsh_raygen *rg)
{
    raygen_dev g{};
    if (!rg) return g;
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
    return g;
}

static crsh_status check_raygen(const crsh_raygen *rg, const char *who)
{
    if (rg->n_lights < 0 || rg->n_lights > CRSH_MAX_LIGHTS || rg->n_mats < 0 ||
        (rg->n_mats > 0 && (!rg->mat_flags || !rg->mat_ior))) {
        set_error("%s: bad ray-generation parameters", who);
        return CRSH_ERR_INVALID;
    }
    return CRSH_OK;
}

static crsh_status check_out(const crsh_rays *out, const char *who)
{
    if (!out->ox || !out->oy || !out->oz || !out->dx || !out->dy || !out->dz || !out->tmax || !out->pix) {
        set_error("%s: incomplete ray arrays", who);
        return CRSH_ERR_INVALID;
    }
    return CRSH_OK;
}

template <int SRC>
static crsh_status hash_kernels(const src_dev &src, const raygen_dev &g, crsh_rays *out, uint32_t *keys,
                                uint32_t *ids, uint32_t *ray_frame, crsh_meta *meta, void *ws, hipStream_t stream)
{
    const uint32_t nb = (uint32_t)(((uint64_t)src.n + HASH_BLOCK - 1) / HASH_BLOCK);
    uint32_t *blocks = (uint32_t *)ws;
    if (nb) {
        prof_scope ps("k_hash_count", stream);
        k_hash_count<SRC><<<nb, HASH_BLOCK, 0, stream>>>(src, g, blocks);
    }
    k_hash_scan<<<1, 1024, 0, stream>>>(blocks, nb, meta, out->capacity);
    rays_dev rd{out->ox, out->oy, out->oz, out->dx, out->dy, out->dz, out->tmax, out->pix, ray_frame, out->capacity};
    if (nb) {
        prof_scope ps("k_hash_emit", stream);
        k_hash_emit<SRC><<<nb, HASH_BLOCK, 0, stream>>>(src, g, blocks, rd, keys, ids);
    }
    return hip_check(hipGetLastError(), "crsh_hash launch");
}

}  // namespace crsh

using namespace crsh;

namespace crsh {

crsh_status hash_launch(const crsh_gbuf *gbuf, const crsh_raygen *rg, const batch_dev *bd, crsh_rays *out,
                        uint32_t *keys, uint32_t *ids, uint32_t *ray_frame, crsh_meta *meta, void *ws,
                        size_t ws_bytes, hipStream_t stream)
{
    if (!gbuf || (!rg && !bd) || !out || !keys || !ids || !meta || !ws || (bd && !ray_frame)) {
        set_error("crsh_hash: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (gbuf->w <= 0 || gbuf->h <= 0 || !gbuf->px || !gbuf->py || !gbuf->pz || !gbuf->nx || !gbuf->ny ||
        !gbuf->nz || !gbuf->mat) {
        set_error("crsh_hash: empty or incomplete primary-hit buffer");
        return CRSH_ERR_INVALID;
    }
    if (rg && check_raygen(rg, "crsh_hash") != CRSH_OK) return CRSH_ERR_INVALID;
    if (check_out(out, "crsh_hash") != CRSH_OK) return CRSH_ERR_INVALID;
    uint64_t npix = (uint64_t)gbuf->w * (uint64_t)gbuf->h;
    if (npix >= (1ull << 31)) {
        set_error("crsh_hash: too many pixels");
        return CRSH_ERR_INVALID;
    }
    if (ws_bytes < hash_ws_bytes(npix)) {
        set_error("crsh_hash: workspace too small (%zu < %zu)", ws_bytes, hash_ws_bytes(npix));
        return CRSH_ERR_INVALID;
    }
    src_dev src{};
    src.gb = gbuf_dev{gbuf->px, gbuf->py, gbuf->pz, gbuf->nx, gbuf->ny, gbuf->nz, gbuf->mat, (uint32_t)npix};
    src.n = (uint32_t)npix;
    if (bd) src.bd = *bd;
    const raygen_dev g = to_device(rg);
    return bd ? hash_kernels<SRC_BATCH>(src, g, out, keys, ids, ray_frame, meta, ws, stream)
              : hash_kernels<SRC_GBUF>(src, g, out, keys, ids, nullptr, meta, ws, stream);
}

}  // namespace crsh

extern "C" crsh_status crsh_hash(const crsh_gbuf *gbuf, const crsh_raygen *rg, crsh_rays *out, uint32_t *keys,
                                 uint32_t *ids, crsh_meta *meta, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!rg) {
        set_error("crsh_hash: NULL argument");
        return CRSH_ERR_INVALID;
    }
    return hash_launch(gbuf, rg, nullptr, out, keys, ids, nullptr, meta, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// crsh_hash_static: crsh_hash with its scratch (the per-block ray counts that
// k_hash_count writes, k_hash_scan turns into offsets and k_hash_emit reads)
// in a fixed device array instead of a caller workspace, for callers that
// cannot allocate.  Every block's count is written before it is read, so the
// array needs no clearing between calls.  In host code `scratch` names a
// host-side shadow, not device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept.
namespace crsh {

// one count per block of HASH_BLOCK pixels plus the scan's total, rounded up
// to whole 256-byte lines as the workspace sizing rounds it
static __device__ __align__(256) uint32_t scratch[(HASH_STATIC_MAX_PIXELS / HASH_BLOCK + 1 + 63) / 64 * 64];

constexpr int STATIC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[STATIC_MAX_DEVICES];

static crsh_status static_scratch(void **out, const char *who)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES) {
        set_error("%s: no usable current device", who);
        return CRSH_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("%s: hipGetSymbolAddress of the static scratch failed on device %d: %s", who, dev,
                      hipGetErrorString(e));
            return CRSH_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CRSH_OK;
}

}  // namespace crsh

extern "C" crsh_status crsh_hash_static(const crsh_gbuf *gbuf, const crsh_raygen *rg, crsh_rays *out,
                                        uint32_t *keys, uint32_t *ids, crsh_meta *meta, hipStream_t stream)
{
    if (!rg || !gbuf) {
        set_error("crsh_hash_static: NULL argument");
        return CRSH_ERR_INVALID;
    }
    const uint64_t npix = (uint64_t)(gbuf->w > 0 ? gbuf->w : 0) * (uint64_t)(gbuf->h > 0 ? gbuf->h : 0);
    if (npix > HASH_STATIC_MAX_PIXELS) {
        set_error("crsh_hash_static: %llu pixels exceed the static scratch's maximum of %llu",
                  (unsigned long long)npix, (unsigned long long)HASH_STATIC_MAX_PIXELS);
        return CRSH_ERR_INVALID;
    }
    if (stream) {   // the stream must belong to the current device, whose scratch the kernels get
        hipDevice_t sd = -1;
        int cur = -1;
        if (hipStreamGetDevice(stream, &sd) != hipSuccess || hipGetDevice(&cur) != hipSuccess || sd != cur) {
            set_error("crsh_hash_static: the stream does not belong to the current device");
            return CRSH_ERR_INVALID;
        }
    }
    void *ws = nullptr;
    const crsh_status st = static_scratch(&ws, "crsh_hash_static");
    if (st != CRSH_OK) return st;
    return hash_launch(gbuf, rg, nullptr, out, keys, ids, nullptr, meta, ws, sizeof(scratch), stream);
}

namespace crsh {

struct given_rays {
    const float *ox, *oy, *oz, *dx, *dy, *dz;
};

__global__ void k_hash_rays(given_rays r, uint32_t n, uint32_t type, uint32_t light, raygen_dev g, uint32_t *keys,
                            uint32_t *ids)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const f3 d = mk(r.dx[i], r.dy[i], r.dz[i]);
        keys[i] = type == 0 ? key_shadow(light, d) : key_bounce(type, mk(r.ox[i], r.oy[i], r.oz[i]), d, g);
        ids[i] = i;
    }
}

__global__ void k_set_rays(crsh_meta *meta, uint32_t n)
{
    meta->n_rays = n;
    meta->rays_required = n;
}

}  // namespace crsh

extern "C" crsh_status crsh_hash_rays(const crsh_rays *rays, uint32_t n, uint32_t type, uint32_t light,
                                      const float lo[3], const float inv_ext[3], uint32_t *keys, uint32_t *ids,
                                      crsh_meta *meta, hipStream_t stream)
{
    if (!rays || !keys || !ids || !meta || !lo || !inv_ext) {
        set_error("crsh_hash_rays: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (type > 2 || light >= CRSH_MAX_LIGHTS || n > rays->capacity || !rays->ox || !rays->oy || !rays->oz ||
        !rays->dx || !rays->dy || !rays->dz) {
        set_error("crsh_hash_rays: bad type, light, count or ray arrays");
        return CRSH_ERR_INVALID;
    }
    raygen_dev g{};
    for (int i = 0; i < 3; ++i) {
        g.lo[i] = lo[i];
        g.inv[i] = inv_ext[i];
    }
    given_rays r{rays->ox, rays->oy, rays->oz, rays->dx, rays->dy, rays->dz};
    k_set_rays<<<1, 1, 0, stream>>>(meta, n);
    if (n) {
        uint32_t grid = std::min<uint32_t>((n + 255) / 256, 4096);
        k_hash_rays<<<grid, 256, 0, stream>>>(r, n, type, light, g, keys, ids);
    }
    return hip_check(hipGetLastError(), "crsh_hash_rays launch");
}

extern "C" crsh_status crsh_bounce(const crsh_rays *parents, const uint32_t *parent_keys, const crsh_hits *hits,
                                   const crsh_meta *parent_meta, const crsh_scene *scene, const int32_t *tri_mat,
                                   const crsh_raygen *rg, crsh_rays *out, uint32_t *keys, uint32_t *ids,
                                   crsh_meta *meta, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!parents || !parent_keys || !hits || !parent_meta || !scene || !tri_mat || !rg || !out || !keys || !ids ||
        !meta || !ws) {
        set_error("crsh_bounce: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (!parents->ox || !parents->oy || !parents->oz || !parents->dx || !parents->dy || !parents->dz ||
        !hits->tri || !hits->t || hits->capacity < parents->capacity) {
        set_error("crsh_bounce: incomplete parent rays or hits");
        return CRSH_ERR_INVALID;
    }
    for (int k = 0; k < 9; ++k)
        if (!scene->v[k] && scene->m) {
            set_error("crsh_bounce: missing vertex array");
            return CRSH_ERR_INVALID;
        }
    if (check_raygen(rg, "crsh_bounce") != CRSH_OK || check_out(out, "crsh_bounce") != CRSH_OK)
        return CRSH_ERR_INVALID;
    if (ws_bytes < hash_ws_bytes(parents->capacity)) {
        set_error("crsh_bounce: workspace too small (%zu < %zu)", ws_bytes, hash_ws_bytes(parents->capacity));
        return CRSH_ERR_INVALID;
    }
    if (out->ox == parents->ox || keys == parent_keys || meta == parent_meta) {
        set_error("crsh_bounce: the new generation must not overwrite its parents");
        return CRSH_ERR_INVALID;
    }
    src_dev src{};
    bounce_dev &b = src.bo;
    b.ox = parents->ox;
    b.oy = parents->oy;
    b.oz = parents->oz;
    b.dx = parents->dx;
    b.dy = parents->dy;
    b.dz = parents->dz;
    b.pix = parents->pix;
    b.keys = parent_keys;
    b.tri = hits->tri;
    b.t = hits->t;
    for (int k = 0; k < 9; ++k) b.v[k] = scene->v[k];
    b.tri_mat = tri_mat;
    b.parent_meta = parent_meta;
    b.cap = parents->capacity;
    b.m = scene->m;
    src.n = parents->capacity;
    return hash_kernels<SRC_BOUNCE>(src, to_device(rg), out, keys, ids, nullptr, meta, ws, stream);
}
