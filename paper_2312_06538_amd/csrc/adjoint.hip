// Adjoint of the closest hit (Sec. 3.3.8) and the indexed-mesh layout helper.
//
// k_gather_tris    indexed mesh -> the nine triangle arrays of a scene.
// k_hit_backward   one thread per ray.  The hit triangle is held fixed: the
//                  Moller-Trumbore solution (t, u, v) satisfies
//                  O + t D = (1-u-v) v0 + u v1 + v v2, so
//                  [D | -e1 | -e2] d(t, u, v) = -dO - t dD + (1-u-v) dv0
//                  + u dv1 + v dv2, and the gradient needs lambda with
//                  [D | -e1 | -e2]^T lambda = (g_t, g_u, g_v).  By Cramer's
//                  rule on the columns, lambda = (g_t (e1 x e2) + g_u (D x e2)
//                  + g_v (e1 x D)) / det[D | -e1 | -e2], and that determinant
//                  is minus the Moller-Trumbore det = e1 . (D x e2).  Every
//                  quantity is recomputed from the inputs; vertex gradients
//                  accumulate with float32 atomics (vertices are shared).
#include "common.hpp"

namespace crsh {

__global__ void k_gather_tris(const float *__restrict__ verts, uint32_t n_verts, const int32_t *__restrict__ faces,
                              uint32_t m, float *v0x, float *v0y, float *v0z, float *v1x, float *v1y, float *v1z,
                              float *v2x, float *v2y, float *v2z)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const int32_t a = faces[3 * i], b = faces[3 * i + 1], c = faces[3 * i + 2];
        const bool ok = a >= 0 && b >= 0 && c >= 0 && (uint32_t)a < n_verts && (uint32_t)b < n_verts &&
                        (uint32_t)c < n_verts;
        const uint32_t ia = ok ? (uint32_t)a : 0u, ib = ok ? (uint32_t)b : 0u, ic = ok ? (uint32_t)c : 0u;
        v0x[i] = ok ? verts[3 * ia] : 0.0f;
        v0y[i] = ok ? verts[3 * ia + 1] : 0.0f;
        v0z[i] = ok ? verts[3 * ia + 2] : 0.0f;
        v1x[i] = ok ? verts[3 * ib] : 0.0f;
        v1y[i] = ok ? verts[3 * ib + 1] : 0.0f;
        v1z[i] = ok ? verts[3 * ib + 2] : 0.0f;
        v2x[i] = ok ? verts[3 * ic] : 0.0f;
        v2y[i] = ok ? verts[3 * ic + 1] : 0.0f;
        v2z[i] = ok ? verts[3 * ic + 2] : 0.0f;
    }
}

struct tri9 {
    const float *v[9];
};

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d, WAVE));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, WAVE));
    return v;
}

// Enclosing sphere of every mesh from its triangles' vertices (Sec. 3.3.1
// asks for a bounding sphere per mesh; any enclosing one keeps the culling
// conservative).  One workgroup per mesh: the centre is the midpoint of the
// vertices' bounding box, the radius the largest float32 vertex distance
// from it widened by 2^-20 of itself.  Each float32 difference, square and
// sum is off by at most a few units in the last place relative to the
// exact value (all terms are non-negative), so the widened radius is at
// least the exact largest distance.  An empty mesh gets (0, 0, 0, 0).
__global__ __launch_bounds__(256) void k_mesh_spheres(tri9 T, uint32_t m, const uint32_t *__restrict__ mesh_first,
                                                      const uint32_t *__restrict__ mesh_count, uint32_t n_mesh,
                                                      float *__restrict__ msph)
{
    __shared__ float s_lo[3][256 / WAVE], s_hi[3][256 / WAVE], s_d[256 / WAVE];
    const uint32_t w = threadIdx.x / WAVE;
    for (uint32_t i = blockIdx.x; i < n_mesh; i += gridDim.x) {
        const uint32_t b = min(mesh_first[i], m);
        const uint32_t e = (uint32_t)min((uint64_t)b + mesh_count[i], (uint64_t)m);
        f3 lo = mk(INFINITY, INFINITY, INFINITY), hi = mk(-INFINITY, -INFINITY, -INFINITY);
        for (uint32_t t = b + threadIdx.x; t < e; t += blockDim.x) {
            for (int k = 0; k < 3; ++k) {
                const f3 p = mk(T.v[3 * k][t], T.v[3 * k + 1][t], T.v[3 * k + 2][t]);
                lo = mk(fminf(lo.x, p.x), fminf(lo.y, p.y), fminf(lo.z, p.z));
                hi = mk(fmaxf(hi.x, p.x), fmaxf(hi.y, p.y), fmaxf(hi.z, p.z));
            }
        }
        lo = mk(wave_min(lo.x), wave_min(lo.y), wave_min(lo.z));
        hi = mk(wave_max(hi.x), wave_max(hi.y), wave_max(hi.z));
        if (lane_id() == 0) {
            s_lo[0][w] = lo.x, s_lo[1][w] = lo.y, s_lo[2][w] = lo.z;
            s_hi[0][w] = hi.x, s_hi[1][w] = hi.y, s_hi[2][w] = hi.z;
        }
        __syncthreads();
        for (uint32_t k = 0; k < blockDim.x / WAVE; ++k) {
            lo = mk(fminf(lo.x, s_lo[0][k]), fminf(lo.y, s_lo[1][k]), fminf(lo.z, s_lo[2][k]));
            hi = mk(fmaxf(hi.x, s_hi[0][k]), fmaxf(hi.y, s_hi[1][k]), fmaxf(hi.z, s_hi[2][k]));
        }
        const f3 c = e > b ? lo * 0.5f + hi * 0.5f : mk(0.0f, 0.0f, 0.0f);
        float d2 = 0.0f;
        for (uint32_t t = b + threadIdx.x; t < e; t += blockDim.x) {
            for (int k = 0; k < 3; ++k) {
                const f3 q = mk(T.v[3 * k][t], T.v[3 * k + 1][t], T.v[3 * k + 2][t]) - c;
                d2 = fmaxf(d2, dot(q, q));
            }
        }
        d2 = wave_max(d2);
        if (lane_id() == 0) s_d[w] = d2;
        __syncthreads();
        for (uint32_t k = 0; k < blockDim.x / WAVE; ++k) d2 = fmaxf(d2, s_d[k]);
        if (threadIdx.x == 0) {
            const float r = sqrtf(d2);
            msph[4 * i] = c.x;
            msph[4 * i + 1] = c.y;
            msph[4 * i + 2] = c.z;
            msph[4 * i + 3] = r + r * 0x1p-20f;
        }
        __syncthreads();    // the LDS slots are reused by the next mesh
    }
}

struct adj_in {
    const float *ox, *oy, *oz, *dx, *dy, *dz;
    const int32_t *tri;
    const float *t, *u, *v;
    const float *gt, *gu, *gv;
    const float *verts;
    const int32_t *faces;
    uint32_t n, n_verts, m;
};

__device__ __forceinline__ f3 vload(const float *p, uint32_t i) { return mk(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }

__device__ __forceinline__ void vatomic(float *p, uint32_t i, f3 g)
{
    atomicAdd(&p[3 * i], g.x);
    atomicAdd(&p[3 * i + 1], g.y);
    atomicAdd(&p[3 * i + 2], g.z);
}

__device__ __forceinline__ void vstore(float *p, uint32_t i, f3 g)
{
    p[3 * i] = g.x;
    p[3 * i + 1] = g.y;
    p[3 * i + 2] = g.z;
}

__global__ __launch_bounds__(256) void k_hit_backward(adj_in a, float *g_verts, float *g_o, float *g_d)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
        const int32_t tri = a.tri[i];
        f3 go = mk(0.0f, 0.0f, 0.0f), gd = go;
        bool ok = tri >= 0 && (uint32_t)tri < a.m;
        uint32_t i0 = 0, i1 = 0, i2 = 0;
        if (ok) {
            const int32_t f0 = a.faces[3 * tri], f1 = a.faces[3 * tri + 1], f2 = a.faces[3 * tri + 2];
            ok = f0 >= 0 && f1 >= 0 && f2 >= 0 && (uint32_t)f0 < a.n_verts && (uint32_t)f1 < a.n_verts &&
                 (uint32_t)f2 < a.n_verts;
            i0 = (uint32_t)f0;
            i1 = (uint32_t)f1;
            i2 = (uint32_t)f2;
        }
        if (ok) {
            const f3 v0 = vload(a.verts, i0), v1 = vload(a.verts, i1), v2 = vload(a.verts, i2);
            const f3 e1 = v1 - v0, e2 = v2 - v0;
            const f3 D = mk(a.dx[i], a.dy[i], a.dz[i]);
            const f3 p = cross(D, e2);
            const float det = dot(e1, p);
            if (fabsf(det) >= DET_EPS) {
                const float gt = a.gt ? a.gt[i] : 0.0f;
                const float gu = a.gu ? a.gu[i] : 0.0f;
                const float gv = a.gv ? a.gv[i] : 0.0f;
                const f3 c1 = cross(e1, e2), c3 = cross(e1, D);
                const float s = -1.0f / det;
                const f3 lam = ((c1 * gt + p * gu) + c3 * gv) * s;
                const float t = a.t[i], u = a.u[i], v = a.v[i];
                go = -lam;
                gd = lam * (-t);
                vatomic(g_verts, i0, lam * ((1.0f - u) - v));
                vatomic(g_verts, i1, lam * u);
                vatomic(g_verts, i2, lam * v);
            }
        }
        vstore(g_o, i, go);
        vstore(g_d, i, gd);
    }
}

}  // namespace crsh

using namespace crsh;

extern "C" crsh_status crsh_gather_triangles(const float *verts, uint32_t n_verts, const int32_t *faces, uint32_t m,
                                             float *const v[9], hipStream_t stream)
{
    if (!verts || !faces || !v) {
        set_error("crsh_gather_triangles: NULL argument");
        return CRSH_ERR_INVALID;
    }
    for (int k = 0; k < 9; ++k)
        if (!v[k]) {
            set_error("crsh_gather_triangles: missing output array");
            return CRSH_ERR_INVALID;
        }
    if (m) {
        uint32_t g = std::min<uint32_t>((m + 255) / 256, 4096);
        k_gather_tris<<<g, 256, 0, stream>>>(verts, n_verts, faces, m, v[0], v[1], v[2], v[3], v[4], v[5], v[6],
                                             v[7], v[8]);
    }
    return hip_check(hipGetLastError(), "crsh_gather_triangles launch");
}

extern "C" crsh_status crsh_mesh_spheres(const float *const v[9], uint32_t m, const uint32_t *mesh_first,
                                         const uint32_t *mesh_count, uint32_t n_mesh, float *msph,
                                         hipStream_t stream)
{
    if (!v || (n_mesh && (!mesh_first || !mesh_count || !msph))) {
        set_error("crsh_mesh_spheres: NULL argument");
        return CRSH_ERR_INVALID;
    }
    tri9 T{};
    for (int k = 0; k < 9; ++k) {
        if (!v[k] && m) {
            set_error("crsh_mesh_spheres: missing vertex array");
            return CRSH_ERR_INVALID;
        }
        T.v[k] = v[k];
    }
    if (n_mesh) k_mesh_spheres<<<std::min<uint32_t>(n_mesh, 4096), 256, 0, stream>>>(T, m, mesh_first, mesh_count,
                                                                                       n_mesh, msph);
    return hip_check(hipGetLastError(), "crsh_mesh_spheres launch");
}

extern "C" crsh_status crsh_closest_hit_backward(const crsh_rays *rays, uint32_t n, const crsh_hits *hits,
                                                 const float *g_t, const float *g_u, const float *g_v,
                                                 const float *verts, uint32_t n_verts, const int32_t *faces,
                                                 uint32_t m, float *g_verts, float *g_o, float *g_d,
                                                 hipStream_t stream)
{
    if (!rays || !hits || !verts || !faces || !g_verts || !g_o || !g_d) {
        set_error("crsh_closest_hit_backward: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (!rays->ox || !rays->oy || !rays->oz || !rays->dx || !rays->dy || !rays->dz || !hits->tri || !hits->t ||
        !hits->u || !hits->v || n > rays->capacity || n > hits->capacity) {
        set_error("crsh_closest_hit_backward: incomplete arrays or count above capacity");
        return CRSH_ERR_INVALID;
    }
    adj_in a{rays->ox, rays->oy, rays->oz, rays->dx, rays->dy, rays->dz, hits->tri, hits->t, hits->u, hits->v,
             g_t, g_u, g_v, verts, faces, n, n_verts, m};
    if (n) {
        uint32_t g = std::min<uint32_t>((n + 255) / 256, 4096);
        prof_scope ps("k_hit_backward", stream);
        k_hit_backward<<<g, 256, 0, stream>>>(a, g_verts, g_o, g_d);
    }
    return hip_check(hipGetLastError(), "crsh_closest_hit_backward launch");
}
