/*
 * Plain CPU oracle of the Coherent Ray-Space Hierarchy (CRSH) secondary-ray
 * path: ray generation + hashing, ray sort, hierarchy build, hierarchy
 * traversal and final closest-hit tests (Reis, Costa, Pereira, "Ray-Tracing
 * With a Coherent Ray-Space Hierarchy", Sec. 3.3.2-3.3.8).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path is
 * the HIP library; the two share no code.
 *
 * Arithmetic: IEEE binary32, round to nearest even, one rounding per written
 * operation, no contraction into fused multiply-add (build with
 * -ffp-contract=off, no fast-math, SSE scalar math).  Every expression is
 * written in the order it is evaluated; sums of three terms are (a + b) + c.
 * The paper keeps its buffers in 32-bit floats (Sec. 3.2); the parity
 * contract of the path fixes binary32 for every stage, so this oracle follows
 * it.  Independent float64 checks live in the tests.
 *
 * Deliberately slow and sequential: loops follow the text of the paper in
 * order, one ray / node / pair at a time.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define ORC_MAX_LEVELS 16

/* ---------------------------------------------------------------- vectors */
typedef struct { float x, y, z; } v3;

static v3 mk(float x, float y, float z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vmul(v3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
static v3 vdiv(v3 a, float s) { return mk(a.x / s, a.y / s, a.z / s); }
static v3 vneg(v3 a) { return mk(-a.x, -a.y, -a.z); }
static float vdot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 vcross(v3 a, v3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static float vnorm(v3 a) { return sqrtf(vdot(a, a)); }
static float maxf(float a, float b) { return a > b ? a : b; }

/* Float32 rounding must never let a sphere or a cone lose a ray, so every
 * union is widened: spheres by PAD relative to (radius + largest |centre|
 * coordinate), cones by CONE_PAD radians.  A normalised sum shorter than
 * H_MIN (two directions more than ~151 degrees apart) cannot give an accurate
 * bisector; such cones are made full.  A ray counts as already inside a cone
 * only with INSIDE_MARGIN to spare (the sine of the angle left over). */
static const float PAD = 0x1p-20f;
static const float CONE_PAD = 0x1p-16f;
static const float H_MIN = 0.25f;
static const float INSIDE_MARGIN = 0x1p-20f;

/* ======================================================================
 * Stage 1: secondary-ray generation, trimming and hashing (Sec. 3.3.2)
 * ====================================================================== */

typedef struct {
    int32_t w, h;
    const float *px, *py, *pz, *nx, *ny, *nz;
    const int32_t *mat;
} orc_gbuf;

typedef struct {
    int32_t n_lights;
    float lights[4][3];
    float eye[3];
    const uint32_t *mat_flags;   /* bit0 reflective, bit1 refractive */
    const float *mat_ior;
    int32_t n_mats;
    uint32_t ray_types;          /* bit0 shadow, bit1 reflection, bit2 refraction;
                                    bit8: keys of type and light only (unsorted comparison);
                                    bit9: spherical-coordinate direction codes */
    float eps_off, eps_shadow;
    float lo[3], inv_ext[3];     /* origin quantisation box for keys */
} orc_raygen;

typedef struct {
    float *ox, *oy, *oz, *dx, *dy, *dz, *tmax;
    uint32_t *pix;
} orc_rays;

/* Shadow ray: the origin is moved to the light (Sec. 3.3.2) so that all rays
 * of one light share their origin; it runs from the light to the surface
 * point and stops eps_shadow before it. */
static int shadow_ray(v3 P, v3 L, float eps_shadow, v3 *O, v3 *D, float *tmax)
{
    v3 d0 = vsub(P, L);
    float len = vnorm(d0);
    if (!(len > eps_shadow)) return 0;
    *O = L;
    *D = vdiv(d0, len);
    *tmax = len - eps_shadow;
    return 1;
}

/* Unit view direction from the eye to a primary hit. */
static v3 view_dir(v3 P, v3 E)
{
    v3 v0 = vsub(P, E);
    return vdiv(v0, vnorm(v0));
}

/* Mirror reflection of the unit incoming direction v about the normal N
 * (which faces against v). */
static void reflect_ray(v3 P, v3 N, v3 v, float eps_off, v3 *O, v3 *D, float *tmax)
{
    float k = vdot(v, N);
    v3 r = vsub(v, vmul(N, 2.0f * k));
    *D = vdiv(r, vnorm(r));
    *O = vadd(P, vmul(N, eps_off));
    *tmax = FLT_MAX;
}

/* Snell refraction of the unit incoming direction v into the surface,
 * relative index 1/ior; returns 0 on total internal reflection. */
static int refract_ray(v3 P, v3 N, v3 v, float ior, float eps_off, v3 *O, v3 *D, float *tmax)
{
    float k = vdot(v, N);
    float eta = 1.0f / ior;
    float ci = -k;
    float k2 = 1.0f - (eta * eta) * (1.0f - ci * ci);
    if (k2 < 0.0f) return 0;
    float b = eta * ci - sqrtf(k2);
    v3 t = vadd(vmul(v, eta), vmul(N, b));
    *D = vdiv(t, vnorm(t));
    *O = vsub(P, vmul(N, eps_off));
    *tmax = FLT_MAX;
    return 1;
}

/* Octahedral direction code: k bits per axis. */
static void oct_code(v3 D, int k, uint32_t *u, uint32_t *v)
{
    float a = (fabsf(D.x) + fabsf(D.y)) + fabsf(D.z);
    float px = D.x / a;
    float py = D.y / a;
    if (D.z < 0.0f) {
        float sx = px >= 0.0f ? 1.0f : -1.0f;
        float sy = py >= 0.0f ? 1.0f : -1.0f;
        float qx = (1.0f - fabsf(py)) * sx;
        float qy = (1.0f - fabsf(px)) * sy;
        px = qx;
        py = qy;
    }
    float scale = ldexpf(1.0f, k - 1);
    float top = (float)((1u << k) - 1u);
    float fu = floorf((px + 1.0f) * scale);
    float fv = floorf((py + 1.0f) * scale);
    if (!(fu >= 0.0f)) fu = 0.0f;
    if (fu > top) fu = top;
    if (!(fv >= 0.0f)) fv = 0.0f;
    if (fv > top) fv = top;
    *u = (uint32_t)fu;
    *v = (uint32_t)fv;
}

/* Spherical-coordinate direction code, the layout of Sec. 3.3.2 (directions
 * converted to spherical coordinates): theta = acos(dz) in [0, pi] and
 * phi = atan2(dy, dx) in [-pi, pi], each quantised to k bits.  acos and
 * atan are the polynomial approximations of Abramowitz & Stegun 4.4.45
 * (|error| <= 6.7e-5) and 4.4.47 (|error| <= 1e-5), evaluated in binary32 in
 * the written order, so any implementation reproduces the same codes. */
static const float SPH_PI = 3.14159265f;
static const float SPH_HALF_PI = 1.57079633f;
static const float SPH_INV_PI = 0.318309886f;
static const float SPH_INV_TWO_PI = 0.159154943f;

static float sph_acos(float x)
{
    float ax = fabsf(x);
    float p = ((-0.0187293f * ax + 0.0742610f) * ax - 0.2121144f) * ax + 1.5707288f;
    float r = sqrtf(1.0f - ax) * p;
    return x < 0.0f ? SPH_PI - r : r;
}

static float sph_atan2(float y, float x)
{
    float ax = fabsf(x), ay = fabsf(y);
    float hi = ax > ay ? ax : ay;
    float lo = ax > ay ? ay : ax;
    if (!(hi > 0.0f)) return 0.0f;
    float a = lo / hi;
    float s = a * a;
    float r = a * ((((0.0208351f * s - 0.0851330f) * s + 0.1801410f) * s - 0.3302995f) * s + 0.9998660f);
    if (ay > ax) r = SPH_HALF_PI - r;
    if (x < 0.0f) r = SPH_PI - r;
    if (y < 0.0f) r = -r;
    return r;
}

static void sph_code(v3 D, int k, uint32_t *u, uint32_t *v)
{
    float scale = ldexpf(1.0f, k);
    float top = (float)((1u << k) - 1u);
    float fu = floorf((sph_acos(D.z) * SPH_INV_PI) * scale);
    float fv = floorf(((sph_atan2(D.y, D.x) + SPH_PI) * SPH_INV_TWO_PI) * scale);
    if (!(fu >= 0.0f)) fu = 0.0f;
    if (fu > top) fu = top;
    if (!(fv >= 0.0f)) fv = 0.0f;
    if (fv > top) fv = top;
    *u = (uint32_t)fu;
    *v = (uint32_t)fv;
}

/* Direction code of a key: octahedral, or spherical with ray_types bit 9. */
static void dir_code(v3 D, int k, uint32_t types, uint32_t *u, uint32_t *v)
{
    if (types & 0x200u)
        sph_code(D, k, u, v);
    else
        oct_code(D, k, u, v);
}

/* Interleave: bit i of u -> bit 2i, bit i of v -> bit 2i+1. */
static uint32_t morton2(uint32_t u, uint32_t v, int k)
{
    uint32_t m = 0;
    for (int i = 0; i < k; ++i) {
        m |= ((u >> i) & 1u) << (2 * i);
        m |= ((v >> i) & 1u) << (2 * i + 1);
    }
    return m;
}

/* Interleave: bit i of x -> 3i, y -> 3i+1, z -> 3i+2. */
static uint32_t morton3(uint32_t x, uint32_t y, uint32_t z, int k)
{
    uint32_t m = 0;
    for (int i = 0; i < k; ++i) {
        m |= ((x >> i) & 1u) << (3 * i);
        m |= ((y >> i) & 1u) << (3 * i + 1);
        m |= ((z >> i) & 1u) << (3 * i + 2);
    }
    return m;
}

/* 64 cells per axis of the quantisation box. */
static uint32_t cell64(float o, float lo, float inv_ext)
{
    float f = floorf(((o - lo) * inv_ext) * 64.0f);
    if (!(f >= 0.0f)) f = 0.0f;
    if (f > 63.0f) f = 63.0f;
    return (uint32_t)f;
}

/* Shadow key: type 00 | light (2 bits) | 28-bit octahedral direction code.
 * The light index sits above the direction so that rays of one light sort
 * together (Sec. 3.3.2). */
static uint32_t shadow_key(int light, v3 D, uint32_t types)
{
    uint32_t u, v;
    dir_code(D, 14, types, &u, &v);
    return ((uint32_t)light << 28) | morton2(u, v, 14);
}

/* Reflection / refraction key: type (2 bits) | 18-bit origin cell |
 * 12-bit octahedral direction code; origins matter because these rays do not
 * share them (Sec. 3.3.2). */
static uint32_t bounce_key(uint32_t type, v3 O, v3 D, const orc_raygen *g)
{
    uint32_t cx = cell64(O.x, g->lo[0], g->inv_ext[0]);
    uint32_t cy = cell64(O.y, g->lo[1], g->inv_ext[1]);
    uint32_t cz = cell64(O.z, g->lo[2], g->inv_ext[2]);
    uint32_t u, v;
    dir_code(D, 6, g->ray_types, &u, &v);
    return (type << 30) | (morton3(cx, cy, cz, 6) << 12) | morton2(u, v, 6);
}

/* The secondary rays of one surface point P with normal N (facing against
 * the unit incoming direction v) and material flags / index of refraction,
 * in slot order: shadow rays of lights 0..L-1, then reflection, then
 * refraction.  Appends the real ones (holes trimmed, Sec. 3.3.2) at n with
 * source index `pix`; returns the new count, or -1 past `capacity`. */
static int64_t emit_slots(v3 P, v3 N, v3 v, uint32_t flags, float ior, uint32_t pix, const orc_raygen *g,
                          orc_rays *out, uint32_t *keys, uint32_t *ids, uint32_t n, uint32_t capacity)
{
    for (int s = 0; s < g->n_lights + 2; ++s) {
        v3 O, D;
        float tmax;
        uint32_t key;
        int ok = 0;
        if (s < g->n_lights) {
            if (g->ray_types & 1u) {
                v3 L = mk(g->lights[s][0], g->lights[s][1], g->lights[s][2]);
                ok = shadow_ray(P, L, g->eps_shadow, &O, &D, &tmax);
                if (ok) key = shadow_key(s, D, g->ray_types);
            }
        } else if (s == g->n_lights) {
            if ((g->ray_types & 2u) && (flags & 1u)) {
                reflect_ray(P, N, v, g->eps_off, &O, &D, &tmax);
                ok = 1;
                key = bounce_key(1u, O, D, g);
            }
        } else {
            if ((g->ray_types & 4u) && (flags & 2u)) {
                ok = refract_ray(P, N, v, ior, g->eps_off, &O, &D, &tmax);
                if (ok) key = bounce_key(2u, O, D, g);
            }
        }
        if (!ok) continue;
        /* Comparison hierarchy without ray sorting (the RSH of Sec. 2):
         * the key keeps only the ray type and light, so the sort groups
         * rays per type and light and keeps their generation order. */
        if (g->ray_types & 0x100u) key &= 0xF0000000u;
        if (n >= capacity) return -1;
        out->ox[n] = O.x; out->oy[n] = O.y; out->oz[n] = O.z;
        out->dx[n] = D.x; out->dy[n] = D.y; out->dz[n] = D.z;
        out->tmax[n] = tmax;
        out->pix[n] = pix;
        keys[n] = key;
        ids[n] = n;
        ++n;
    }
    return n;
}

/* Generates every secondary ray of every pixel, in pixel order and, within a
 * pixel, shadow rays of lights 0..L-1, then reflection, then refraction.
 * Holes are trimmed away (Sec. 3.3.2): a ray's id is the number of real rays
 * before it.  Returns N, or -1 if more than `capacity` rays would be made. */
int64_t orc_hash(const orc_gbuf *gb, const orc_raygen *g, orc_rays *out,
                 uint32_t *keys, uint32_t *ids, uint32_t capacity)
{
    int64_t n = 0;
    v3 E = mk(g->eye[0], g->eye[1], g->eye[2]);
    int64_t npx = (int64_t)gb->w * gb->h;
    for (int64_t p = 0; p < npx; ++p) {
        int32_t m = gb->mat[p];
        if (m < 0) continue;
        v3 P = mk(gb->px[p], gb->py[p], gb->pz[p]);
        v3 N = mk(gb->nx[p], gb->ny[p], gb->nz[p]);
        uint32_t flags = (m < g->n_mats) ? g->mat_flags[m] : 0u;
        float ior = (m < g->n_mats) ? g->mat_ior[m] : 1.0f;
        n = emit_slots(P, N, view_dir(P, E), flags, ior, (uint32_t)p, g, out, keys, ids, (uint32_t)n, capacity);
        if (n < 0) return -1;
    }
    return n;
}

/* The next bounce (Sec. 3.3.8: the algorithm continues with a new set of
 * secondary rays from the sorting step).  Every reflection or refraction
 * ray (key type 01 or 10) with a closest hit spawns the secondary rays of
 * its hit point, in parent-id order: P = O + t D, the unit geometric normal
 * of the hit triangle (e1 x e2 normalised) turned against D, the material
 * of the triangle (tri_mat), and D itself as the incoming direction.  Shadow
 * rays and misses spawn nothing.  Children keep their parent's source pixel.
 * Returns the new count, or -1 past `capacity`. */
int64_t orc_bounce(const orc_rays *par, const uint32_t *par_keys, uint32_t n_par, const int32_t *hit_tri,
                   const float *hit_t, const float *const v[9], uint32_t m, const int32_t *tri_mat,
                   const orc_raygen *g, orc_rays *out, uint32_t *keys, uint32_t *ids, uint32_t capacity)
{
    int64_t n = 0;
    for (uint32_t i = 0; i < n_par; ++i) {
        int32_t tri = hit_tri[i];
        if (tri < 0 || (uint32_t)tri >= m || (par_keys[i] >> 30) == 0u) continue;
        v3 O = mk(par->ox[i], par->oy[i], par->oz[i]);
        v3 D = mk(par->dx[i], par->dy[i], par->dz[i]);
        v3 P = vadd(O, vmul(D, hit_t[i]));
        v3 a = mk(v[0][tri], v[1][tri], v[2][tri]);
        v3 b = mk(v[3][tri], v[4][tri], v[5][tri]);
        v3 c = mk(v[6][tri], v[7][tri], v[8][tri]);
        v3 nn = vcross(vsub(b, a), vsub(c, a));
        float len = vnorm(nn);
        if (!(len > 0.0f)) continue;
        v3 N = vdiv(nn, len);
        if (vdot(N, D) > 0.0f) N = vneg(N);
        int32_t mt = tri_mat[tri];
        uint32_t flags = (mt >= 0 && mt < g->n_mats) ? g->mat_flags[mt] : 0u;
        float ior = (mt >= 0 && mt < g->n_mats) ? g->mat_ior[mt] : 1.0f;
        n = emit_slots(P, N, D, flags, ior, par->pix[i], g, out, keys, ids, (uint32_t)n, capacity);
        if (n < 0) return -1;
    }
    return n;
}

/* Exposed for closed-form key checks. */
uint32_t orc_shadow_key(int light, const float d[3]) { return shadow_key(light, mk(d[0], d[1], d[2]), 0u); }
void orc_sph_code(const float d[3], int k, uint32_t *u, uint32_t *v) { sph_code(mk(d[0], d[1], d[2]), k, u, v); }
uint32_t orc_bounce_key(uint32_t type, const float o[3], const float d[3], const orc_raygen *g)
{
    return bounce_key(type, mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]), g);
}
void orc_oct_code(const float d[3], int k, uint32_t *u, uint32_t *v) { oct_code(mk(d[0], d[1], d[2]), k, u, v); }

/* ======================================================================
 * Stage 2: ray sorting (Sec. 3.3.3-3.3.5)
 *
 * Compression into chunks of equal consecutive keys, a sort of the chunks by
 * key, and decompression give the (key, id) pairs stably ordered by key:
 * equal keys keep their input order.  The oracle states that result
 * directly, with a library sort on (key, input position).
 * ====================================================================== */
typedef struct { uint32_t key, id, pos; } kv;

static int kv_cmp(const void *a, const void *b)
{
    const kv *x = (const kv *)a, *y = (const kv *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return 0;
}

void orc_sort(const uint32_t *keys, const uint32_t *ids, uint32_t n,
              uint32_t *keys_out, uint32_t *ids_out)
{
    kv *a = (kv *)malloc(sizeof(kv) * (n ? n : 1));
    for (uint32_t i = 0; i < n; ++i) { a[i].key = keys[i]; a[i].id = ids[i]; a[i].pos = i; }
    qsort(a, n, sizeof(kv), kv_cmp);
    for (uint32_t i = 0; i < n; ++i) { keys_out[i] = a[i].key; ids_out[i] = a[i].id; }
    free(a);
}

/* ======================================================================
 * Stage 3: hierarchy creation (Sec. 3.3.6, Eq. 1-8)
 * ====================================================================== */

/* A cone is kept as unit-ish axis x with (cos, sin) of its half-angle, so no
 * inverse trigonometric function is needed; c <= 0 means "90 degrees or
 * more", which the traversal never culls. */
typedef struct { v3 x; float c, s; } cone;
typedef struct { v3 c; float r; } sphere;

static int cone_full(cone k) { return !(k.c > 0.0f); }

static cone cone_fullify(v3 x)
{
    cone o;
    o.x = x;
    o.c = -1.0f;
    o.s = 0.0f;
    return o;
}

/* Every cone that a union produces is either canonical full (c = -1, s = 0)
 * or has c > 0 and is widened by CONE_PAD radians, i.e. (c, s) rotated by
 * CONE_PAD (first order). */
static cone cone_finish(cone k)
{
    if (!(k.c > 0.0f)) return cone_fullify(k.x);
    cone o = k;
    o.c = k.c - CONE_PAD * k.s;
    o.s = k.s + CONE_PAD * k.c;
    if (!(o.c > 0.0f)) return cone_fullify(k.x);
    return o;
}

/* Union of two cones (Eq. 5-6): the axis is the normalised sum of the axes;
 * the half-angle is half the angle between the axes plus the larger child
 * half-angle, applied with the angle-addition formulas. */
static cone cone_union(cone a, cone b)
{
    if (cone_full(a) || cone_full(b)) return cone_fullify(a.x);
    v3 sum = vadd(a.x, b.x);
    float h = vnorm(sum);
    if (!(h >= H_MIN)) return cone_fullify(a.x);
    v3 x = vdiv(sum, h);
    float ch = h * 0.5f;                       /* cos of half the axis angle */
    float sh = vnorm(vsub(a.x, b.x)) * 0.5f;   /* sin of half the axis angle */
    float cm = a.c, sm = a.s;
    if (b.s > a.s) { cm = b.c; sm = b.s; }
    cone o;
    o.x = x;
    o.c = ch * cm - sh * sm;
    o.s = sh * cm + ch * sm;
    return cone_finish(o);
}

/* Add one ray direction r to a cone (Eq. 1-4, compact cones). */
static cone cone_add_ray(cone k, v3 r)
{
    if (cone_full(k)) return k;
    v3 nv = vcross(k.x, r);
    float st = vnorm(nv);            /* |x||r| sin(theta) */
    float ct = vdot(k.x, r);         /* |x||r| cos(theta) */
    /* inside: parallel, or sin(phi - theta) at least INSIDE_MARGIN */
    if (ct > 0.0f && (st == 0.0f || k.s * ct - k.c * st >= INSIDE_MARGIN)) return k;
    /* antiparallel, or the new half-angle (phi + theta)/2 reaches 90 degrees */
    if (st == 0.0f || k.s * ct + k.c * st <= 0.0f) return cone_fullify(k.x);
    if (st < 0x1p-10f) {
        /* nearly parallel: the plane of x and r is ill-defined, use Eq. 5-6 */
        cone rr;
        rr.x = r; rr.c = 1.0f; rr.s = 0.0f;
        return cone_union(k, rr);
    }
    /* Eq. 1: unit vector orthogonal to x in the plane of x and r, on the far
     * side of the axis from r. */
    v3 q = vneg(vdiv(vcross(nv, k.x), st));
    /* Eq. 2: far edge of the current cone. */
    v3 e = vadd(vmul(k.x, k.c), vmul(q, k.s));
    /* Eq. 3: new axis bisects the far edge and the ray. */
    v3 er = vadd(e, r);
    float h = vnorm(er);
    if (!(h >= H_MIN)) return cone_fullify(k.x);
    cone o;
    o.x = vdiv(er, h);
    /* Eq. 4: new half-angle is the angle between the new axis and the ray;
     * its sine is half the chord between the far edge and the ray. */
    o.c = vdot(o.x, r);
    o.s = vnorm(vsub(e, r)) * 0.5f;
    return cone_finish(o);
}

static float pad_radius(v3 c, float r)
{
    float m = maxf(maxf(fabsf(c.x), fabsf(c.y)), fabsf(c.z));
    return r + PAD * (r + m);
}

/* Union of two spheres (Eq. 7-8): midpoint centre, radius half the centre
 * distance plus the larger radius. */
static sphere sphere_union(sphere a, sphere b)
{
    sphere o;
    o.c = vmul(vadd(a.c, b.c), 0.5f);
    float e = vnorm(vsub(b.c, a.c)) * 0.5f;
    o.r = pad_radius(o.c, e + maxf(a.r, b.r));
    return o;
}

/* Balanced pairwise reduction in index order: (0,1), (2,3), ...; an odd last
 * element passes to the next round unchanged. */
static sphere sphere_reduce(sphere *t, int k)
{
    while (k > 1) {
        int h = 0;
        for (int i = 0; i + 1 < k; i += 2) t[h++] = sphere_union(t[i], t[i + 1]);
        if (k & 1) t[h++] = t[k - 1];
        k = h;
    }
    return t[0];
}

static cone cone_reduce(cone *t, int k)
{
    while (k > 1) {
        int h = 0;
        for (int i = 0; i + 1 < k; i += 2) t[h++] = cone_union(t[i], t[i + 1]);
        if (k & 1) t[h++] = t[k - 1];
        k = h;
    }
    return t[0];
}

/* Node storage, structure of arrays; level k (1-based) occupies
 * [level_off[k-1], level_off[k-1] + level_cnt[k-1]). */
typedef struct {
    float *cx, *cy, *cz, *r, *ax, *ay, *az, *c, *s, *tan, *sec;
} orc_nodes;

static void store_node(orc_nodes *nd, uint32_t i, sphere sp, cone k)
{
    nd->cx[i] = sp.c.x; nd->cy[i] = sp.c.y; nd->cz[i] = sp.c.z; nd->r[i] = sp.r;
    nd->ax[i] = k.x.x; nd->ay[i] = k.x.y; nd->az[i] = k.x.z;
    nd->c[i] = k.c; nd->s[i] = k.s;
    if (k.c > 0.0f) {
        nd->tan[i] = k.s / k.c;
        nd->sec[i] = 1.0f / k.c;
    } else {
        nd->tan[i] = 0.0f;
        nd->sec[i] = 0.0f;
    }
}

/* Number of levels built and the node count of each: level 1 has
 * ceil(N/B) nodes, level k has ceil(n_{k-1}/F); building stops at `levels`
 * or at the first level with a single node (Sec. 3.3.6 limits the depth). */
int orc_level_counts(uint32_t n_rays, int B, int F, int levels, uint32_t *cnt)
{
    if (n_rays == 0) return 0;
    uint32_t c = (n_rays + (uint32_t)B - 1) / (uint32_t)B;
    int k = 0;
    cnt[k++] = c;
    while (k < levels && c > 1) {
        c = (c + (uint32_t)F - 1) / (uint32_t)F;
        cnt[k++] = c;
    }
    return k;
}

/* Builds every level bottom-up.  Rays are read through the sorted id list;
 * leaves start as radius-0 spheres at the origins and zero-spread cones
 * (Sec. 3.3.6).  Returns the number of levels. */
int orc_build(const orc_rays *rays, const uint32_t *sorted_ids, uint32_t n_rays,
              int B, int F, int levels, orc_nodes *nd, uint32_t *level_off, uint32_t *level_cnt)
{
    int nl = orc_level_counts(n_rays, B, F, levels, level_cnt);
    uint32_t off = 0;
    for (int k = 0; k < nl; ++k) { level_off[k] = off; off += level_cnt[k]; }
    int tmpn = B > F ? B : F;
    sphere *ts = (sphere *)malloc(sizeof(sphere) * (size_t)tmpn);
    cone *tc = (cone *)malloc(sizeof(cone) * (size_t)tmpn);
    if (nl > 0) {
        for (uint32_t j = 0; j < level_cnt[0]; ++j) {
            uint32_t b = j * (uint32_t)B;
            uint32_t e = b + (uint32_t)B;
            if (e > n_rays) e = n_rays;
            cone k;
            for (uint32_t s = b; s < e; ++s) {
                uint32_t id = sorted_ids[s];
                v3 o = mk(rays->ox[id], rays->oy[id], rays->oz[id]);
                v3 d = mk(rays->dx[id], rays->dy[id], rays->dz[id]);
                ts[s - b].c = o;
                ts[s - b].r = 0.0f;
                if (s == b) {
                    k.x = d; k.c = 1.0f; k.s = 0.0f;
                } else {
                    k = cone_add_ray(k, d);
                }
            }
            sphere sp = sphere_reduce(ts, (int)(e - b));
            store_node(nd, level_off[0] + j, sp, k);
        }
    }
    for (int lv = 1; lv < nl; ++lv) {
        uint32_t below = level_off[lv - 1], nb = level_cnt[lv - 1];
        for (uint32_t j = 0; j < level_cnt[lv]; ++j) {
            uint32_t b = j * (uint32_t)F;
            uint32_t e = b + (uint32_t)F;
            if (e > nb) e = nb;
            for (uint32_t ch = b; ch < e; ++ch) {
                uint32_t i = below + ch;
                ts[ch - b].c = mk(nd->cx[i], nd->cy[i], nd->cz[i]);
                ts[ch - b].r = nd->r[i];
                tc[ch - b].x = mk(nd->ax[i], nd->ay[i], nd->az[i]);
                tc[ch - b].c = nd->c[i];
                tc[ch - b].s = nd->s[i];
            }
            sphere sp = sphere_reduce(ts, (int)(e - b));
            cone k = cone_reduce(tc, (int)(e - b));
            store_node(nd, level_off[lv] + j, sp, k);
        }
    }
    free(ts);
    free(tc);
    return nl;
}

/* Exposed single steps, for closed-form checks. */
void orc_cone_add_ray(const float x[3], float c, float s, const float r[3], float out[5])
{
    cone k; k.x = mk(x[0], x[1], x[2]); k.c = c; k.s = s;
    cone o = cone_add_ray(k, mk(r[0], r[1], r[2]));
    out[0] = o.x.x; out[1] = o.x.y; out[2] = o.x.z; out[3] = o.c; out[4] = o.s;
}
void orc_cone_union(const float a[5], const float b[5], float out[5])
{
    cone x, y;
    x.x = mk(a[0], a[1], a[2]); x.c = a[3]; x.s = a[4];
    y.x = mk(b[0], b[1], b[2]); y.c = b[3]; y.s = b[4];
    cone o = cone_union(x, y);
    out[0] = o.x.x; out[1] = o.x.y; out[2] = o.x.z; out[3] = o.c; out[4] = o.s;
}
void orc_sphere_union(const float a[4], const float b[4], float out[4])
{
    sphere x, y;
    x.c = mk(a[0], a[1], a[2]); x.r = a[3];
    y.c = mk(b[0], b[1], b[2]); y.r = b[3];
    sphere o = sphere_union(x, y);
    out[0] = o.c.x; out[1] = o.c.y; out[2] = o.c.z; out[3] = o.r;
}

/* ======================================================================
 * Stage 4: hierarchy traversal (Sec. 3.3.7, Eq. 9)
 * ====================================================================== */

/* Triangle bounding spheres used by the coarse tests: centroid and the
 * largest centroid-vertex distance, padded outwards. */
void orc_tri_spheres(const float *const v[9], uint32_t m, float *tcx, float *tcy, float *tcz, float *tr)
{
    const float third = 1.0f / 3.0f;
    for (uint32_t i = 0; i < m; ++i) {
        v3 a = mk(v[0][i], v[1][i], v[2][i]);
        v3 b = mk(v[3][i], v[4][i], v[5][i]);
        v3 c = mk(v[6][i], v[7][i], v[8][i]);
        v3 ctr = vmul(vadd(vadd(a, b), c), third);
        float r = maxf(maxf(vnorm(vsub(a, ctr)), vnorm(vsub(b, ctr))), vnorm(vsub(c, ctr)));
        tcx[i] = ctr.x; tcy[i] = ctr.y; tcz[i] = ctr.z;
        tr[i] = pad_radius(ctr, r);
    }
}

/* Eq. 9: a sphere (P, d) may meet a ray of a node (centre C, radius r, axis
 * a, half-angle alpha) iff |P-H| <= |C-H| tan(alpha) + (d + r)/cos(alpha),
 * H being the projection of P on the axis.  |P-H| is |(P-C) x a| and |C-H| is
 * |(P-C).a|; both sides are compared squared.  Nodes of 90 degrees or more
 * are never culled. */
static int node_sphere_test(const orc_nodes *nd, uint32_t i, v3 P, float d)
{
    if (!(nd->c[i] > 0.0f)) return 1;
    v3 C = mk(nd->cx[i], nd->cy[i], nd->cz[i]);
    v3 a = mk(nd->ax[i], nd->ay[i], nd->az[i]);
    v3 v = vsub(P, C);
    float t = vdot(v, a);
    v3 w = vcross(v, a);
    float lhs2 = vdot(w, w);
    float rhs = fabsf(t) * nd->tan[i] + (d + nd->r[i]) * nd->sec[i];
    return lhs2 <= rhs * rhs;
}

int orc_node_sphere_test(const float node[11], const float sph[4])
{
    orc_nodes nd;
    float *p = (float *)node;
    nd.cx = p + 0; nd.cy = p + 1; nd.cz = p + 2; nd.r = p + 3;
    nd.ax = p + 4; nd.ay = p + 5; nd.az = p + 6; nd.c = p + 7; nd.s = p + 8;
    nd.tan = p + 9; nd.sec = p + 10;
    return node_sphere_test(&nd, 0, mk(sph[0], sph[1], sph[2]), sph[3]);
}

typedef struct {
    uint32_t *tri, *node;   /* node ids are local to their level */
    uint64_t n, cap;
} orc_pairvec;

static void pv_push(orc_pairvec *v, uint32_t t, uint32_t nd)
{
    if (v->n == v->cap) {
        v->cap = v->cap ? v->cap * 2 : 1024;
        v->tri = (uint32_t *)realloc(v->tri, sizeof(uint32_t) * v->cap);
        v->node = (uint32_t *)realloc(v->node, sizeof(uint32_t) * v->cap);
    }
    v->tri[v->n] = t;
    v->node[v->n] = nd;
    v->n++;
}

typedef struct {
    int n_levels;
    orc_pairvec pairs[ORC_MAX_LEVELS];      /* pairs[k-1] = level k */
    uint64_t tests[ORC_MAX_LEVELS];
    uint64_t mesh_tests, mesh_hits, final_tests;
} orc_trav;

/* Top-down traversal.  Top level: every top node against every mesh sphere,
 * then, for the (node, mesh) pairs that pass, against the bounding sphere of
 * every triangle of the mesh that lies in [tri_begin, tri_end).  Lower
 * levels: every (triangle, node) pair that passed is tested against each child
 * of the node.  Surviving pairs form the trimmed array of the next level.
 * If top_subset is non-null only those top nodes are traversed (their
 * sub-trees are independent).  Counters follow the paper's tables: tests and
 * hits per level, plus the final ray-triangle tests (rays of every leaf that
 * reaches level 1). */
orc_trav *orc_traverse(const orc_nodes *nd, const uint32_t *level_off, const uint32_t *level_cnt,
                       int n_levels, uint32_t n_rays, int B, int F,
                       const float *tcx, const float *tcy, const float *tcz, const float *tr,
                       const uint32_t *mesh_first, const uint32_t *mesh_count, uint32_t n_mesh,
                       const float *msph /* [n_mesh][4] */,
                       uint32_t tri_begin, uint32_t tri_end,
                       const uint32_t *top_subset, uint32_t n_subset)
{
    orc_trav *T = (orc_trav *)calloc(1, sizeof(orc_trav));
    T->n_levels = n_levels;
    if (n_levels == 0) return T;
    int top = n_levels - 1;
    orc_pairvec *pt = &T->pairs[top];
    uint32_t ntop = top_subset ? n_subset : level_cnt[top];
    for (uint32_t ii = 0; ii < ntop; ++ii) {
        uint32_t i = top_subset ? top_subset[ii] : ii;
        if (i >= level_cnt[top]) continue;
        uint32_t gi = level_off[top] + i;
        for (uint32_t m = 0; m < n_mesh; ++m) {
            T->mesh_tests++;
            v3 P = mk(msph[4 * m + 0], msph[4 * m + 1], msph[4 * m + 2]);
            if (!node_sphere_test(nd, gi, P, msph[4 * m + 3])) continue;
            T->mesh_hits++;
            uint32_t b = mesh_first[m], e = mesh_first[m] + mesh_count[m];
            if (b < tri_begin) b = tri_begin;
            if (e > tri_end) e = tri_end;
            for (uint32_t t = b; t < e; ++t) {
                T->tests[top]++;
                if (node_sphere_test(nd, gi, mk(tcx[t], tcy[t], tcz[t]), tr[t])) pv_push(pt, t, i);
            }
        }
    }
    for (int lv = top - 1; lv >= 0; --lv) {
        orc_pairvec *up = &T->pairs[lv + 1];
        orc_pairvec *dn = &T->pairs[lv];
        for (uint64_t q = 0; q < up->n; ++q) {
            uint32_t t = up->tri[q], p = up->node[q];
            v3 P = mk(tcx[t], tcy[t], tcz[t]);
            for (int j = 0; j < F; ++j) {
                uint32_t ch = p * (uint32_t)F + (uint32_t)j;
                if (ch >= level_cnt[lv]) break;
                T->tests[lv]++;
                if (node_sphere_test(nd, level_off[lv] + ch, P, tr[t])) pv_push(dn, t, ch);
            }
        }
    }
    for (uint64_t q = 0; q < T->pairs[0].n; ++q) {
        uint32_t j = T->pairs[0].node[q];
        uint32_t b = j * (uint32_t)B, e = b + (uint32_t)B;
        if (e > n_rays) e = n_rays;
        T->final_tests += e - b;
    }
    return T;
}

uint64_t orc_trav_count(const orc_trav *T, int level) { return T->pairs[level - 1].n; }
void orc_trav_copy(const orc_trav *T, int level, uint32_t *tri, uint32_t *node)
{
    const orc_pairvec *v = &T->pairs[level - 1];
    memcpy(tri, v->tri, sizeof(uint32_t) * v->n);
    memcpy(node, v->node, sizeof(uint32_t) * v->n);
}
void orc_trav_counters(const orc_trav *T, uint64_t *tests, uint64_t *misc)
{
    for (int k = 0; k < ORC_MAX_LEVELS; ++k) tests[k] = T->tests[k];
    misc[0] = T->mesh_tests;
    misc[1] = T->mesh_hits;
    misc[2] = T->final_tests;
}
void orc_trav_free(orc_trav *T)
{
    for (int k = 0; k < ORC_MAX_LEVELS; ++k) { free(T->pairs[k].tri); free(T->pairs[k].node); }
    free(T);
}

/* ======================================================================
 * Stage 5: final intersection tests and closest hit (Sec. 3.3.8)
 * ====================================================================== */

/* Moller-Trumbore ray-triangle test, two-sided, accepting t in (t_min, tmax).
 * Returns how far the test got: 0 the determinant is too small, 1 u failed,
 * 2 v (or u + v) failed, 3 t is outside the interval, 4 accepted (then t, u,
 * v are written). */
static int mt_stage(v3 O, v3 D, float t_min, float tmax, v3 v0, v3 v1, v3 v2,
                    float *pt, float *pu, float *pv)
{
    v3 e1 = vsub(v1, v0);
    v3 e2 = vsub(v2, v0);
    v3 p = vcross(D, e2);
    float det = vdot(e1, p);
    if (!(fabsf(det) >= 1e-12f)) return 0;
    float inv = 1.0f / det;
    v3 T = vsub(O, v0);
    float u = vdot(T, p) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return 1;
    v3 q = vcross(T, e1);
    float v = vdot(D, q) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return 2;
    float t = vdot(e2, q) * inv;
    if (!(t > t_min && t < tmax)) return 3;
    *pt = t; *pu = u; *pv = v;
    return 4;
}

static int mt_test(v3 O, v3 D, float t_min, float tmax, v3 v0, v3 v1, v3 v2,
                   float *pt, float *pu, float *pv)
{
    return mt_stage(O, D, t_min, tmax, v0, v1, v2, pt, pu, pv) == 4;
}

int orc_mt(const float o[3], const float d[3], float t_min, float tmax, const float tri[9], float out[3])
{
    return mt_test(mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]), t_min, tmax,
                   mk(tri[0], tri[1], tri[2]), mk(tri[3], tri[4], tri[5]), mk(tri[6], tri[7], tri[8]),
                   &out[0], &out[1], &out[2]);
}

static void keep_closest(int32_t *best_tri, float *bt, float *bu, float *bv, uint32_t id,
                         uint32_t tri, float t, float u, float v)
{
    if (best_tri[id] < 0 || t < bt[id] || (t == bt[id] && (int32_t)tri < best_tri[id])) {
        best_tri[id] = (int32_t)tri; bt[id] = t; bu[id] = u; bv[id] = v;
    }
}

/* For every (triangle, leaf) pair of level 1, every ray of the leaf is
 * tested against the triangle; each ray keeps its closest hit, ties broken by
 * the lower triangle id.  Results are indexed by ray id; misses keep tri -1.
 * Outputs must be initialised by the caller (tri = -1) so that several
 * triangle batches merge. */
void orc_closest_hit(const orc_rays *rays, const uint32_t *sorted_ids, uint32_t n_rays, int B,
                     const uint32_t *pair_tri, const uint32_t *pair_node, uint64_t n_pairs,
                     const float *const v[9], float t_min,
                     int32_t *hit_tri, float *ht, float *hu, float *hv, uint64_t *stage_counts)
{
    /* stage_counts (may be NULL) accumulates [tests whose u passed, tests
     * whose u and v passed] */
    for (uint64_t q = 0; q < n_pairs; ++q) {
        uint32_t t = pair_tri[q], j = pair_node[q];
        v3 a = mk(v[0][t], v[1][t], v[2][t]);
        v3 b = mk(v[3][t], v[4][t], v[5][t]);
        v3 c = mk(v[6][t], v[7][t], v[8][t]);
        uint32_t s0 = j * (uint32_t)B, s1 = s0 + (uint32_t)B;
        if (s1 > n_rays) s1 = n_rays;
        for (uint32_t s = s0; s < s1; ++s) {
            uint32_t id = sorted_ids[s];
            float tt, uu, vv;
            const int st = mt_stage(mk(rays->ox[id], rays->oy[id], rays->oz[id]),
                                    mk(rays->dx[id], rays->dy[id], rays->dz[id]),
                                    t_min, rays->tmax[id], a, b, c, &tt, &uu, &vv);
            if (stage_counts) {
                stage_counts[0] += st >= 2;
                stage_counts[1] += st >= 3;
            }
            if (st == 4) keep_closest(hit_tri, ht, hu, hv, id, t, tt, uu, vv);
        }
    }
}

/* Naive ray tracing (Sec. 1): every listed ray against every triangle. */
void orc_brute_closest_hit(const orc_rays *rays, const uint32_t *ray_list, uint32_t n_list,
                           const float *const v[9], uint32_t m, float t_min,
                           int32_t *hit_tri, float *ht, float *hu, float *hv)
{
    for (uint32_t i = 0; i < n_list; ++i) {
        uint32_t id = ray_list[i];
        v3 O = mk(rays->ox[id], rays->oy[id], rays->oz[id]);
        v3 D = mk(rays->dx[id], rays->dy[id], rays->dz[id]);
        int32_t bt_ = -1;
        float btt = 0.0f, bu = 0.0f, bv = 0.0f;
        for (uint32_t t = 0; t < m; ++t) {
            float tt, uu, vv;
            if (!mt_test(O, D, t_min, rays->tmax[id], mk(v[0][t], v[1][t], v[2][t]),
                         mk(v[3][t], v[4][t], v[5][t]), mk(v[6][t], v[7][t], v[8][t]), &tt, &uu, &vv))
                continue;
            if (bt_ < 0 || tt < btt) { bt_ = (int32_t)t; btt = tt; bu = uu; bv = vv; }
        }
        hit_tri[i] = bt_; ht[i] = btt; hu[i] = bu; hv[i] = bv;
    }
}

/* Every listed ray against every triangle: all hits (ray index, triangle),
 * written while they fit in `cap`; returns the total number. */
uint64_t orc_brute_all_hits(const orc_rays *rays, const uint32_t *ray_list, uint32_t n_list,
                            const float *const v[9], uint32_t m, float t_min,
                            uint32_t *out_ray, uint32_t *out_tri, uint64_t cap)
{
    uint64_t n = 0;
    for (uint32_t i = 0; i < n_list; ++i) {
        uint32_t id = ray_list[i];
        v3 O = mk(rays->ox[id], rays->oy[id], rays->oz[id]);
        v3 D = mk(rays->dx[id], rays->dy[id], rays->dz[id]);
        for (uint32_t t = 0; t < m; ++t) {
            float tt, uu, vv;
            if (!mt_test(O, D, t_min, rays->tmax[id], mk(v[0][t], v[1][t], v[2][t]),
                         mk(v[3][t], v[4][t], v[5][t]), mk(v[6][t], v[7][t], v[8][t]), &tt, &uu, &vv))
                continue;
            if (n < cap) { out_ray[n] = id; out_tri[n] = t; }
            ++n;
        }
    }
    return n;
}

/* ======================================================================
 * Float64 references for the closest-hit adjoint
 * ====================================================================== */

/* Moller-Trumbore in float64 with the triangle fixed (no accept/reject):
 * solves O + t D = (1-u-v) v0 + u v1 + v v2.  Used for central finite
 * differences of (t, u, v). */
int orc_mt64(const double o[3], const double d[3], const double tri[9], double out[3])
{
    double e1[3], e2[3], T[3], p[3], q[3];
    for (int i = 0; i < 3; ++i) {
        e1[i] = tri[3 + i] - tri[i];
        e2[i] = tri[6 + i] - tri[i];
        T[i] = o[i] - tri[i];
    }
    p[0] = d[1] * e2[2] - d[2] * e2[1];
    p[1] = d[2] * e2[0] - d[0] * e2[2];
    p[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0.0) return 0;
    q[0] = T[1] * e1[2] - T[2] * e1[1];
    q[1] = T[2] * e1[0] - T[0] * e1[2];
    q[2] = T[0] * e1[1] - T[1] * e1[0];
    out[1] = (T[0] * p[0] + T[1] * p[1] + T[2] * p[2]) / det;
    out[2] = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) / det;
    out[0] = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) / det;
    return 1;
}
