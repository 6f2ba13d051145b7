// Final ray-triangle test (Sec. 3.3.8): Moller-Trumbore on triangles packed
// as (v0, e1, e2).
#pragma once

#include "common.hpp"

namespace crsh {

// Closest-hit key: the bits of t mapped to an unsigned order that follows
// the float order for either sign (negative values complemented, others with
// the sign bit set; -0 taken as +0, so equal distances tie) above the
// triangle id.  The 64-bit minimum is the smallest t, ties to the lower
// triangle; all ones (the bits of a NaN) means no hit.
__device__ __forceinline__ unsigned long long hit_key(float t, uint32_t tri)
{
    uint32_t b = __float_as_uint(t == 0.0f ? 0.0f : t);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((unsigned long long)b << 32) | tri;
}

__device__ __forceinline__ float hit_key_t(unsigned long long key)
{
    const uint32_t b = (uint32_t)(key >> 32);
    return __uint_as_float((b & 0x80000000u) ? (b & 0x7FFFFFFFu) : ~b);
}

struct tri_t {
    f3 v0, e1, e2;
};

__device__ __forceinline__ tri_t load_tri(const float4 *__restrict__ tri, uint32_t t)
{
    float4 a = tri[3 * t + 0];
    float4 b = tri[3 * t + 1];
    float4 c = tri[3 * t + 2];
    tri_t r;
    r.v0 = mk(a.x, a.y, a.z);
    r.e1 = mk(a.w, b.x, b.y);
    r.e2 = mk(b.z, b.w, c.x);
    return r;
}

// Checks of the test a ray passed: MT_U (u in [0, 1]), MT_UV (and v >= 0,
// u + v <= 1), MT_HIT (and t_min < t < tmax), each implying the ones before.
constexpr uint32_t MT_U = 1u, MT_UV = 2u, MT_HIT = 4u;

// Two-sided Moller-Trumbore, accepted for t_min < t < tmax; the checks passed
// go to *checks when given.
//
// u = a * (1/det) is first decided without the division where its sign or
// size settles the test exactly as the rounded quotient would: with
// |det| <= 2^60 the rounded reciprocal has magnitude >= 2^-60, so opposite
// signs and |a| >= 2^-60 give u <= -2^-120 < 0; and |a| above the rounded
// |det| (1 + 2^-19) with equal signs gives a quotient above 1 + 2^-20, which
// two roundings cannot bring down to 1.  Other cases divide as written.
__device__ __forceinline__ bool moller_trumbore(f3 O, f3 D, float t_min, float tmax, const tri_t &tr, float &tt,
                                                float &uu, float &vv, uint32_t *checks = nullptr)
{
    if (checks) *checks = 0u;
    f3 p = cross(D, tr.e2);
    float det = dot(tr.e1, p);
    const float adet = fabsf(det);
    if (!(adet >= DET_EPS)) return false;
    f3 T = O - tr.v0;
    const float a = dot(T, p);
    if (adet <= 0x1p60f) {
        const bool opposite = (a < 0.0f) != (det < 0.0f);
        if (opposite && fabsf(a) >= 0x1p-60f) return false;
        if (!opposite && fabsf(a) > adet * (1.0f + 0x1p-19f)) return false;
    }
    float inv = 1.0f / det;
    float u = a * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    if (checks) *checks = MT_U;
    f3 q = cross(T, tr.e1);
    float v = dot(D, q) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    if (checks) *checks = MT_U | MT_UV;
    float t = dot(tr.e2, q) * inv;
    if (!(t > t_min && t < tmax)) return false;
    if (checks) *checks = MT_U | MT_UV | MT_HIT;
    tt = t;
    uu = u;
    vv = v;
    return true;
}


// The first half of the test, for the final-test kernel: p = D x e2,
// det = e1 . p, T = O - v0 and a = T . p (u = a / det before rounding), and
// the wave mask of the lanes whose ray can still pass -- clear exactly where
// moller_trumbore's determinant check or its division-free decision on u
// rejects it.  Called by every lane of the wave.
struct mt_head {
    f3 p, T;
    float det, a;
};

__device__ __forceinline__ uint64_t mt_first_half(f3 O, f3 D, const tri_t &tr, mt_head &h)
{
    h.p = cross(D, tr.e2);
    h.det = dot(tr.e1, h.p);
    h.T = O - tr.v0;
    h.a = dot(h.T, h.p);
    // moller_trumbore's early checks, combined without branches.  With
    // s = a carrying det's sign (|s| = |a|; s < 0 iff a and det have
    // opposite signs, a = -0 counting as 0), its two rejections are
    // s <= -2^-60 and s > |det| (1 + 2^-19) while |det| <= 2^60; a NaN s
    // fails both comparisons and is rejected here, as the division would
    // reject it (u NaN).
    const float adet = fabsf(h.det);
    const float sg = __uint_as_float(__float_as_uint(h.a) ^ (__float_as_uint(h.det) & 0x80000000u));
    // each comparison is a wave mask as it stands; they combine in scalar
    // operations
    return ballot(adet >= DET_EPS) &
           (ballot(adet > 0x1p60f) | (ballot(sg > -0x1p-60f) & ballot(sg <= adet * (1.0f + 0x1p-19f))));
}

// The rest of the test for a ray that mt_first_half let through: the same
// operations, in the same order, as moller_trumbore after its early checks.
// The checks passed, as wave masks: pu (u in [0, 1]), puv (and v >= 0,
// u + v <= 1), hit (and t_min < t < tmax), each implying the ones before; all
// comparisons are made and combined without short-circuit.
__device__ __forceinline__ void mt_second_half(f3 D, float t_min, float tmax, const tri_t &tr, const mt_head &h,
                                               float &tt, uint64_t &pu, uint64_t &puv, uint64_t &hit)
{
    const float inv = 1.0f / h.det;
    const float u = h.a * inv;
    const f3 q = cross(h.T, tr.e1);
    const float v = dot(D, q) * inv;
    const float t = dot(tr.e2, q) * inv;
    tt = t;
    pu = ballot(u >= 0.0f) & ballot(u <= 1.0f);
    puv = pu & ballot(v >= 0.0f) & ballot(u + v <= 1.0f);
    hit = puv & ballot(t > t_min) & ballot(t < tmax);
}

// The same test for the final-test kernel, without early exits: every
// quantity of the test is computed and the acceptance conditions are combined
// at the end, so the whole wave runs one straight sequence (the division
// included) instead of branching on each condition.  Values and the accept
// decision are those of moller_trumbore.
__device__ __forceinline__ bool moller_trumbore_t(f3 O, f3 D, float t_min, float tmax, const tri_t &tr, float &tt)
{
    const f3 p = cross(D, tr.e2);
    const float det = dot(tr.e1, p);
    const float inv = 1.0f / det;
    const f3 T = O - tr.v0;
    const float u = dot(T, p) * inv;
    const f3 q = cross(T, tr.e1);
    const float v = dot(D, q) * inv;
    const float t = dot(tr.e2, q) * inv;
    tt = t;
    return fabsf(det) >= DET_EPS && (u >= 0.0f && u <= 1.0f) && (v >= 0.0f && u + v <= 1.0f) &&
           (t > t_min && t < tmax);
}

}  // namespace crsh
