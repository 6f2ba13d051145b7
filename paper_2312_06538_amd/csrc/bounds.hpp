// Bounding volumes of the hierarchy (Sec. 3.3.6, Eq. 1-8) and the
// node-sphere test of the traversal (Sec. 3.3.7, Eq. 9).
#pragma once

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

// Eq. 9 with H the projection of P on the node axis: |P-H| = |(P-C) x a|,
// |C-H| = |(P-C).a|; pass iff |P-H|^2 <= (|C-H| tan + (d + r) sec)^2.
__device__ __forceinline__ bool packed_meets(float4 A, float4 Bv, float sec, f3 P, float d)
{
    if (!(sec > 0.0f)) return true;
    f3 v = P - mk(A.x, A.y, A.z);
    f3 a = mk(Bv.x, Bv.y, Bv.z);
    float t = dot(v, a);
    f3 w = cross(v, a);
    float lhs2 = dot(w, w);
    float rhs = fabsf(t) * Bv.w + (d + A.w) * sec;
    return lhs2 <= rhs * rhs;
}

// packed_meets with every operation performed and the outcome selected at
// the end: the same values and the same decision, with no branch for the
// compiler to sink a caller's loads of A, Bv and sec into.
__device__ __forceinline__ bool packed_meets_flat(float4 A, float4 Bv, float sec, f3 P, float d)
{
    const f3 v = P - mk(A.x, A.y, A.z);
    const f3 a = mk(Bv.x, Bv.y, Bv.z);
    const float t = dot(v, a);
    const f3 w = cross(v, a);
    const float lhs2 = dot(w, w);
    const float rhs = fabsf(t) * Bv.w + (d + A.w) * sec;
    return !(sec > 0.0f) || lhs2 <= rhs * rhs;
}

// packed_meets_flat over a wave: the mask of the lanes whose pair passes,
// each condition taken as a mask of its own (a compare's result is already
// a mask; their combination is then one scalar operation).  Called by every
// lane of the wave.
__device__ __forceinline__ uint64_t packed_meets_mask(float4 A, float4 Bv, float sec, f3 P, float d)
{
    const f3 v = P - mk(A.x, A.y, A.z);
    const f3 a = mk(Bv.x, Bv.y, Bv.z);
    const float t = dot(v, a);
    const f3 w = cross(v, a);
    const float lhs2 = dot(w, w);
    const float rhs = fabsf(t) * Bv.w + (d + A.w) * sec;
    return ballot(!(sec > 0.0f)) | ballot(lhs2 <= rhs * rhs);
}


}  // namespace crsh
