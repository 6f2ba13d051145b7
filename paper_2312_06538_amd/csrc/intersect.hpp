// Final ray-triangle test (Sec. 3.3.8): Moller-Trumbore on triangles packed
// as (v0, e1, e2).
#pragma once

#include "common.hpp"

namespace crsh {

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

// Two-sided Moller-Trumbore, accepted for t_min < t < tmax.
//
// u = a * (1/det) is first decided without the division where its sign or
// size settles the test exactly as the rounded quotient would: with
// |det| <= 2^60 the rounded reciprocal has magnitude >= 2^-60, so opposite
// signs and |a| >= 2^-60 give u <= -2^-120 < 0; and |a| above the rounded
// |det| (1 + 2^-19) with equal signs gives a quotient above 1 + 2^-20, which
// two roundings cannot bring down to 1.  Other cases divide as written.
__device__ __forceinline__ bool moller_trumbore(f3 O, f3 D, float t_min, float tmax, const tri_t &tr, float &tt,
                                                float &uu, float &vv)
{
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
    f3 q = cross(T, tr.e1);
    float v = dot(D, q) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    float t = dot(tr.e2, q) * inv;
    if (!(t > t_min && t < tmax)) return false;
    tt = t;
    uu = u;
    vv = v;
    return true;
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
