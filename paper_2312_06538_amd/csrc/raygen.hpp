// Secondary-ray generation and ray keys (Sec. 3.3.2): per-slot rays of a
// primary hit and their 32-bit hash keys.
#pragma once

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

// Spherical coordinates of a unit direction, theta = acos(dz) and
// phi = atan2(dy, dx), each quantised to 2^k bins (the direction layout of
// Sec. 3.3.2).  acos and atan: Abramowitz & Stegun 4.4.45 and 4.4.47
// polynomials in binary32, operation by operation, so the codes are
// reproducible.
constexpr float SPH_PI = 3.14159265f;
constexpr float SPH_HALF_PI = 1.57079633f;
constexpr float SPH_INV_PI = 0.318309886f;
constexpr float SPH_INV_TWO_PI = 0.159154943f;

__device__ __forceinline__ float sph_acos(float x)
{
    const float ax = fabsf(x);
    const float p = ((-0.0187293f * ax + 0.0742610f) * ax - 0.2121144f) * ax + 1.5707288f;
    const float r = sqrtf(1.0f - ax) * p;
    return x < 0.0f ? SPH_PI - r : r;
}

__device__ __forceinline__ float sph_atan2(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float hi = ax > ay ? ax : ay;
    const float lo = ax > ay ? ay : ax;
    if (!(hi > 0.0f)) return 0.0f;
    const float a = lo / hi;
    const float s = a * a;
    float r = a * ((((0.0208351f * s - 0.0851330f) * s + 0.1801410f) * s - 0.3302995f) * s + 0.9998660f);
    if (ay > ax) r = SPH_HALF_PI - r;
    if (x < 0.0f) r = SPH_PI - r;
    if (y < 0.0f) r = -r;
    return r;
}

__device__ __forceinline__ void spherical(f3 d, int k, uint32_t &u, uint32_t &v)
{
    const float scale = (float)(1u << k);
    const float top = (float)((1u << k) - 1u);
    float fu = floorf((sph_acos(d.z) * SPH_INV_PI) * scale);
    float fv = floorf(((sph_atan2(d.y, d.x) + SPH_PI) * SPH_INV_TWO_PI) * scale);
    fu = fu >= 0.0f ? fu : 0.0f;
    fv = fv >= 0.0f ? fv : 0.0f;
    fu = fu > top ? top : fu;
    fv = fv > top ? top : fv;
    u = (uint32_t)fu;
    v = (uint32_t)fv;
}

__device__ __forceinline__ void dir_code(f3 d, int k, uint32_t types, uint32_t &u, uint32_t &v)
{
    if (types & CRSH_KEY_SPHERICAL)
        spherical(d, k, u, v);
    else
        octahedral(d, k, u, v);
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
__device__ __forceinline__ uint32_t key_shadow(uint32_t light, f3 d, uint32_t types = 0u)
{
    uint32_t u, v;
    dir_code(d, 14, types, u, v);
    return (light << 28) | spread2(u) | (spread2(v) << 1);
}

__device__ __forceinline__ uint32_t key_bounce(uint32_t type, f3 o, f3 d, const raygen_dev &g)
{
    uint32_t cx = cell64(o.x, g.lo[0], g.inv[0]);
    uint32_t cy = cell64(o.y, g.lo[1], g.inv[1]);
    uint32_t cz = cell64(o.z, g.lo[2], g.inv[2]);
    uint32_t u, v;
    dir_code(d, 6, g.types, u, v);
    uint32_t cell = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
    return (type << 30) | (cell << 12) | spread2(u) | (spread2(v) << 1);
}

// Slot s of a surface point P with normal N facing against the unit incoming
// direction v (shadow rays of lights 0..L-1, reflection, refraction);
// returns false for a hole.  With CRSH_KEY_TYPE_ONLY the key keeps only the
// ray type and light: the comparison hierarchy without ray sorting (Sec. 2).
__device__ __forceinline__ bool make_slot(int s, f3 P, f3 N, f3 v, uint32_t flags, float ior, const raygen_dev &g,
                                          ray_t &r)
{
    bool ok = false;
    if (s < g.n_lights) {
        if (g.types & CRSH_RAY_SHADOW) {
            f3 L = mk(g.lx[s], g.ly[s], g.lz[s]);
            f3 d0 = P - L;
            float l = len(d0);
            if (l > g.eps_shadow) {
                r.o = L;                  // origin moved to the light
                r.d = d0 / l;
                r.tmax = l - g.eps_shadow;
                r.key = key_shadow((uint32_t)s, r.d, g.types);
                ok = true;
            }
        }
    } else if (s == g.n_lights) {
        if ((g.types & CRSH_RAY_REFLECT) && (flags & CRSH_MAT_REFLECTIVE)) {
            float k = dot(v, N);
            f3 rr = v - N * (2.0f * k);
            r.d = rr / len(rr);
            r.o = P + N * g.eps_off;
            r.tmax = FLT_MAX;
            r.key = key_bounce(1u, r.o, r.d, g);
            ok = true;
        }
    } else if ((g.types & CRSH_RAY_REFRACT) && (flags & CRSH_MAT_REFRACTIVE)) {
        float k = dot(v, N);
        float eta = 1.0f / ior;
        float ci = -k;
        float k2 = 1.0f - (eta * eta) * (1.0f - ci * ci);
        if (k2 >= 0.0f) {                 // otherwise total internal reflection
            float b = eta * ci - sqrtf(k2);
            f3 t = v * eta + N * b;
            r.d = t / len(t);
            r.o = P - N * g.eps_off;
            r.tmax = FLT_MAX;
            r.key = key_bounce(2u, r.o, r.d, g);
            ok = true;
        }
    }
    if (ok && (g.types & CRSH_KEY_TYPE_ONLY)) r.key &= 0xF0000000u;
    return ok;
}

// A surface point that emits secondary rays: a primary hit (pixel) or the
// closest hit of a previous bounce ray.
struct pixel_t {
    f3 P, N, v;       // point, normal facing against v, unit incoming direction
    uint32_t flags;
    float ior;
    uint32_t pix;     // source pixel of the rays
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
    const f3 v0 = px.P - mk(g.ex, g.ey, g.ez);
    px.v = v0 / len(v0);
    px.flags = m < g.n_mats ? g.mat_flags[m] : 0u;
    px.ior = m < g.n_mats ? g.mat_ior[m] : 1.0f;
    px.pix = p;
    return px;
}

// Closest hits of a previous generation (Sec. 3.3.8): reflection and
// refraction rays with a hit spawn the secondary rays of their hit point.
struct bounce_dev {
    const float *ox, *oy, *oz, *dx, *dy, *dz;
    const uint32_t *pix, *keys;
    const int32_t *tri;
    const float *t;
    const float *v[9];
    const int32_t *tri_mat;
    const crsh_meta *parent_meta;
    uint32_t cap, m;
};

__device__ __forceinline__ pixel_t load_bounce(const bounce_dev &b, const raygen_dev &g, uint32_t i)
{
    pixel_t px;
    px.hit = false;
    if (i >= min(b.parent_meta->n_rays, b.cap)) return px;
    const int32_t tri = b.tri[i];
    if (tri < 0 || (uint32_t)tri >= b.m || (b.keys[i] >> 30) == 0u) return px;
    const f3 O = mk(b.ox[i], b.oy[i], b.oz[i]);
    const f3 D = mk(b.dx[i], b.dy[i], b.dz[i]);
    const f3 a = mk(b.v[0][tri], b.v[1][tri], b.v[2][tri]);
    const f3 bb = mk(b.v[3][tri], b.v[4][tri], b.v[5][tri]);
    const f3 c = mk(b.v[6][tri], b.v[7][tri], b.v[8][tri]);
    const f3 nn = cross(bb - a, c - a);
    const float l = len(nn);
    if (!(l > 0.0f)) return px;
    f3 N = nn / l;
    if (dot(N, D) > 0.0f) N = -N;
    px.hit = true;
    px.P = O + D * b.t[i];
    px.N = N;
    px.v = D;
    const int32_t mt = b.tri_mat[tri];
    px.flags = (mt >= 0 && mt < g.n_mats) ? g.mat_flags[mt] : 0u;
    px.ior = (mt >= 0 && mt < g.n_mats) ? g.mat_ior[mt] : 1.0f;
    px.pix = b.pix ? b.pix[i] : i;
    return px;
}

}  // namespace crsh
