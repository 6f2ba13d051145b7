// Stage 5: final intersection tests and closest hit (Sec. 3.3.8).
//
// k_hit_prep   triangles repacked as 3 x float4 (v0, e1 = v1 - v0,
//              e2 = v2 - v0): one 48-byte fetch per test instead of nine
//              scattered loads; e1, e2 are the same single roundings the
//              test would make.
// k_hit        persistent waves over the level-1 pairs; a group of G lanes
//              (G = bundle rounded up to a power of two) takes one pair, one
//              lane per ray of its leaf, so a leaf's rays are read
//              contiguously from the sorted ray arrays.  A hit lowers the
//              ray's 64-bit (order-mapped t, triangle) key with an atomic
//              minimum: the closest hit, ties to the lower triangle id.
// k_hit_final  one thread per sorted ray: decode the key, recompute u, v with
//              the same test, write the result at the ray id.
// Ray slots: k_hit reads the rays of leaf l at slots l * B + j, j < B, of two
// packed arrays: (origin, tmax), 16 bytes a slot, and the direction, 12
// bytes a slot; the interval start t_min is the frame's.  In the plain form
// slot s is sorted ray s.  In the batched form a frame's rays are bundled B
// at a time from its own first ray, so only a frame's last leaf can hold
// fewer than B rays; its slots are padded (zeros, a marker in place of tmax)
// and the closest-hit keys are kept by slot, so the pair loop finds a ray
// with no per-leaf lookup.  k_hit_final maps each sorted ray back to its
// slot through its frame's first leaf and first ray.
#include "batch.hpp"
#include "intersect.hpp"

namespace crsh {

__global__ void k_hit_prep(const float *__restrict__ v0x, const float *__restrict__ v0y,
                           const float *__restrict__ v0z, const float *__restrict__ v1x,
                           const float *__restrict__ v1y, const float *__restrict__ v1z,
                           const float *__restrict__ v2x, const float *__restrict__ v2y,
                           const float *__restrict__ v2z, uint32_t m, float4 *tri)
{
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        float ax = v0x[t], ay = v0y[t], az = v0z[t];
        float e1x = v1x[t] - ax, e1y = v1y[t] - ay, e1z = v1z[t] - az;
        float e2x = v2x[t] - ax, e2y = v2y[t] - ay, e2z = v2z[t] - az;
        tri[3 * t + 0] = make_float4(ax, ay, az, e1x);
        tri[3 * t + 1] = make_float4(e1y, e1z, e2x, e2y);
        tri[3 * t + 2] = make_float4(e2z, 0.0f, 0.0f, 0.0f);
    }
}

struct sorted_rays {
    const float *ox, *oy, *oz, *dx, *dy, *dz, *tmax;
};

// tmax word of a padded slot (a NaN); a NaN tmax of a real ray is stored as
// the default quiet NaN, which accepts no hit either
constexpr uint32_t PAD_SLOT = 0x7FC0DEADu;
__device__ __forceinline__ float slot_tmax(float tmax) { return tmax != tmax ? __uint_as_float(0x7FC00000u) : tmax; }

// slots of the batched form in use: B per level-1 node
__device__ __forceinline__ uint32_t batch_slots(const crsh_meta *meta, uint32_t B, uint32_t slot_cap)
{
    const uint64_t ns = meta->n_levels ? (uint64_t)meta->level_cnt[0] * B : 0u;
    return (uint32_t)(ns < slot_cap ? ns : slot_cap);
}

// Plain form: sorted rays repacked as (origin, tmax), 16 bytes a slot, and
// the direction, 12 bytes a slot (the interval start is the frame's, a
// kernel argument): a 16-byte and a 12-byte load per test instead of seven
// scattered ones, and the 16 rays of a leaf are 256 and 192 contiguous
// bytes.
__global__ void k_hit_rays(sorted_rays R, const crsh_meta *meta, uint32_t cap, float4 *org, float *dir3)
{
    const uint32_t n = min(meta->n_rays, cap);
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        org[s] = make_float4(R.ox[s], R.oy[s], R.oz[s], R.tmax[s]);
        dir3[3 * (size_t)s + 0] = R.dx[s];
        dir3[3 * (size_t)s + 1] = R.dy[s];
        dir3[3 * (size_t)s + 2] = R.dz[s];
    }
}

__device__ __forceinline__ f3 buf_load3(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    typedef float v3f __attribute__((ext_vector_type(3)));
    const v3f v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
    return mk(v.x, v.y, v.z);
}

// Batched form: slot p = leaf * B + j holds ray j of level-1 node `leaf`
// (first ray and count as the build recorded them), or zeros and the padding
// marker; every slot's closest-hit key starts at all ones.
__global__ void k_hit_rays_batch(sorted_rays R, const crsh_meta *meta, uint32_t ray_cap, uint32_t B,
                                 uint32_t slot_cap, batch_dev bd, float4 *org, float *dir3,
                                 unsigned long long *keys)
{
    const uint32_t n = min(meta->n_rays, ray_cap);
    const uint32_t ns = batch_slots(meta, B, slot_cap);
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < ns; p += gridDim.x * blockDim.x) {
        const uint32_t leaf = p / B;
        const uint32_t j = p - leaf * B;
        const uint32_t info = bd.node_info[leaf];
        const uint32_t f = info >> INFO_FRAME_SHIFT;
        const uint32_t s = bd.node_first[leaf] + j;
        float dx = 0.0f, dy = 0.0f, dz = 0.0f;
        if (j < (info & INFO_COUNT_MASK) && s < n && f < bd.n_frames) {
            org[p] = make_float4(R.ox[s], R.oy[s], R.oz[s], slot_tmax(R.tmax[s]));
            dx = R.dx[s];
            dy = R.dy[s];
            dz = R.dz[s];
        } else {
            org[p] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(PAD_SLOT));
        }
        dir3[3 * (size_t)p + 0] = dx;
        dir3[3 * (size_t)p + 1] = dy;
        dir3[3 * (size_t)p + 2] = dz;
        keys[p] = ~0ull;
    }
}

// One step of the final tests for a wave: each lane group holds a pair --
// its triangle (a, b, c: v0, e1, e2 packed), the triangle id, the byte
// offsets of the leaf's first ray slot and first direction, and the interval
// start of the pair's frame -- and lane j of the group tests ray j of the
// leaf.  `live` is the wave mask of the lanes whose test is one of the
// pair's.  A lane outside it may still read a ray: that of a slot past the
// leaf's rays, or a zero ray (a padded slot, or an offset past the arrays'
// ends, which reads zeros); a zero ray has a zero determinant and fails the
// first half, so only the lanes j >= B of a group wider than the bundle need
// the mask.  COUNT: the step counts its tests (the lanes of `live`, less the
// padded slots of the batched form); without it the caller counts them.
// Hits go to the slot keys.  Called by every lane of the wave.
template <bool BATCH, bool COUNT>
__device__ __forceinline__ void hit_step(const __amdgpu_buffer_rsrc_t &org_r, const __amdgpu_buffer_rsrc_t &dir_r,
                                         const float4 &a, const float4 &b, float tc, uint32_t tri_id,
                                         uint32_t ray_off, uint32_t dir_off, float t_min, uint64_t live, uint32_t j,
                                         unsigned long long *keys, uint64_t &tests, uint64_t &upass,
                                         uint64_t &uvpass)
{
    const uint32_t ro = ray_off + j * 16u;
    const float4 ro4 = buf_load4(org_r, ro);
    const f3 D = buf_load3(dir_r, dir_off + j * 12u);
    tri_t tr;
    tr.v0 = mk(a.x, a.y, a.z);
    tr.e1 = mk(a.w, b.x, b.y);
    tr.e2 = mk(b.z, b.w, tc);
    if constexpr (COUNT) {
        // a padded slot's NaN t_min accepts nothing; it only must not count
        // as a test
        if (BATCH) live &= ballot(__float_as_uint(ro4.w) != PAD_SLOT);
        tests += (uint64_t)__popcll(live);
    }
    mt_head h;
    const uint64_t mm = mt_first_half(mk(ro4.x, ro4.y, ro4.z), D, tr, h) & live;
    // a wave-uniform branch: the wave runs the second half only if one of
    // its lanes needs it (every lane computes it; the masks keep the lanes
    // that needed it)
    if (mm != 0) {
        float th;
        uint64_t pu, puv, hit;
        mt_second_half(D, t_min, ro4.w, tr, h, th, pu, puv, hit);
        upass += (uint64_t)__popcll(pu & mm);
        uvpass += (uint64_t)__popcll(puv & mm);
        if (__builtin_amdgcn_inverse_ballot_w64(hit & mm)) atomicMin(&keys[ro >> 4], hit_key(th, tri_id));
    }
}

// The wave totals of a final-test kernel added to meta (s_red: [3][waves]).
__device__ __forceinline__ void hit_counts(uint64_t (*s_red)[256 / WAVE], uint32_t wib, uint32_t l, uint64_t tests,
                                           uint64_t upass, uint64_t uvpass, crsh_meta *meta)
{
    if (l == 0) {
        s_red[0][wib] = tests;
        s_red[1][wib] = upass;
        s_red[2][wib] = uvpass;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint64_t tot = 0;
        for (uint32_t i = 0; i < blockDim.x / WAVE; ++i) tot += s_red[threadIdx.x][i];
        unsigned long long *dst = threadIdx.x == 0 ? (unsigned long long *)&meta->final_tests
                                : threadIdx.x == 1 ? (unsigned long long *)&meta->final_u_pass
                                                   : (unsigned long long *)&meta->final_uv_pass;
        if (tot) atomicAdd(dst, (unsigned long long)tot);
    }
}

// Slots in use: the plain form's sorted rays, or B per level-1 node.  PACKED:
// the level-1 pairs are packed words in ptri (node above the low
// CRSH_PACKED_TRI_BITS, triangle minus tri_base below; pnode unused).
// Batched form: the build's per-node record of a leaf (bd.node_info) holds
// its ray count and frame, and the frame its interval start.
//
// A wave takes runs of 64 consecutive pairs before the grid stride
// (neighbouring level-1 pairs share their triangle -- siblings of one
// parent pair -- or their leaves, so a run finds its rays in the vector L1
// cache).  Each lane reads one pair of the run, its triangle, and writes a
// record to the wave's LDS slice: the triangle (v0, e1, e2), the triangle
// id, the byte offsets of the leaf's first ray slot and first direction
// (past the arrays for a pair out of range, so that its rays read as
// zeros) and, batched form, the interval start of the leaf's frame.  The
// run is then tested 64 / G pairs at a time, each lane group reading its
// pair's record from LDS (the 16 lanes of a group read the same address), so
// the vector memory path carries only the rays.  The tests are counted per
// pair when the record is written (the leaf's rays), not per step.  Rays are
// read with buffer loads on 32-bit byte offsets (the host bounds them; a read
// past the end returns zeros), origins and directions from their own
// arrays, so each of the two loads of a step covers contiguous bytes per
// pair (256 and 192).  The test is split where most of its cost lies: every lane computes
// the division-free first half, and the wave runs the rest (the division
// included) only when one of its lanes can still pass.
constexpr uint32_t RAY_OFF_NONE = 0xFFFF0000u;   // above every slot array (2^31 bytes at most)
template <bool BATCH, bool PACKED>
__global__ __launch_bounds__(256) void k_hit(const float4 *__restrict__ RO, const float *__restrict__ RD,
                                             const float4 *__restrict__ tri,
                                             const uint32_t *__restrict__ ptri, const uint32_t *__restrict__ pnode,
                                             uint64_t cap1, uint32_t B, uint32_t log2G, unsigned long long *keys,
                                             crsh_meta *meta, uint32_t slot_cap, uint32_t m, uint32_t tri_base,
                                             batch_dev bd, float t_min)
{
    constexpr uint32_t RW = BATCH ? 4 : 3;           // record words
    __shared__ uint64_t s_red[3][256 / WAVE];
    __shared__ float4 s_rec[256 / WAVE][RW][WAVE];   // [wave][record word][pair of the run]
    const uint32_t ns = BATCH ? batch_slots(meta, B, slot_cap) : min(meta->n_rays, slot_cap);
    uint64_t np = meta->n_levels ? meta->pairs[0] : 0;
    np = np < cap1 ? np : cap1;
    const uint32_t l = lane_id();
    const uint32_t G = 1u << log2G;
    const uint32_t slot = l >> log2G;        // pair of this lane within a step
    const uint32_t j = l & (G - 1);          // ray of the leaf
    const uint32_t per_wave = WAVE >> log2G;
    const uint64_t live = ballot(j < B);     // the lanes of a group that test a ray of the leaf
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // scalar: so is the run arithmetic
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + wib;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
    const __amdgpu_buffer_rsrc_t org_r = make_rsrc(RO, (uint64_t)ns * 16u);
    const __amdgpu_buffer_rsrc_t dir_r = make_rsrc(RD, (uint64_t)ns * 12u);
    const __amdgpu_buffer_rsrc_t tris_r = make_rsrc(tri, (uint64_t)m * 48u);
    float4(*rec)[WAVE] = s_rec[wib];
    uint32_t my_tests = 0;                   // this lane's pairs: rays of their leaves
    uint64_t tests = 0, upass = 0, uvpass = 0;   // wave-wide counts
    for (uint64_t c0 = wave * WAVE; c0 < np; c0 += nwaves * WAVE) {
        const uint32_t cn = __builtin_amdgcn_readfirstlane((uint32_t)min(np - c0, (uint64_t)WAVE));
        uint32_t my_t = 0u, my_rb = RAY_OFF_NONE, my_db = RAY_OFF_NONE, leaf = 0u;
        bool valid = false;
        if (l < cn) {
            if constexpr (PACKED) {
                const uint32_t w = ptri[c0 + l];
                my_t = tri_base + (w & ((1u << CRSH_PACKED_TRI_BITS) - 1u));
                leaf = w >> CRSH_PACKED_TRI_BITS;
            } else {
                my_t = ptri[c0 + l];
                leaf = pnode[c0 + l];
            }
            // rays of the leaf present in the slot array (none for a pair out
            // of range)
            const uint64_t first = (uint64_t)leaf * B;
            if (my_t < m && first < ns) {
                valid = true;
                my_rb = (uint32_t)first * 16u;
                my_db = (uint32_t)first * 12u;
            }
        }
        const uint32_t tb = valid ? my_t * 48u : 0u;
        const float4 ta = buf_load4(tris_r, tb);
        const float4 tbv = buf_load4(tris_r, tb + 16u);
        const float tc = buf_load1(tris_r, tb + 32u);
        uint32_t cnt = valid ? min(B, ns - leaf * B) : 0u;
        float my_tmin = 0.0f;
        if constexpr (BATCH) {
            const uint32_t info = valid ? bd.node_info[leaf] : 0u;
            cnt = min(cnt, info & INFO_COUNT_MASK);
            const uint32_t f = info >> INFO_FRAME_SHIFT;
            my_tmin = cnt && f < bd.n_frames ? bd.frames[f].t_min : 0.0f;
        }
        my_tests += cnt;
        __builtin_amdgcn_wave_barrier();          // the previous run's reads come first
        rec[0][l] = ta;
        rec[1][l] = tbv;
        rec[2][l] = make_float4(tc, __uint_as_float(my_t), __uint_as_float(my_rb), __uint_as_float(my_db));
        if constexpr (BATCH) ((float *)rec[3])[l] = my_tmin;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t k = 0; k < cn; k += per_wave) {
            const uint32_t src = k + slot;
            const float4 a = rec[0][src];
            const float4 b = rec[1][src];
            const float4 c = rec[2][src];
            const float tm = BATCH ? ((const float *)rec[3])[src] : t_min;
            hit_step<BATCH, false>(org_r, dir_r, a, b, c.x, __float_as_uint(c.y), __float_as_uint(c.z),
                                   __float_as_uint(c.w), tm, live, j, keys, tests, upass, uvpass);
        }
    }
    tests = wave_sum((uint64_t)my_tests);
    hit_counts(s_red, wib, l, tests, upass, uvpass, meta);
}

// Final tests of the level-1 pairs that the level-2 pairs and the level-1
// pass masks describe (the fused last level: the level-1 pairs are never
// stored).  Level-2 pair q keeps child j (leaf first(q) + j, first = node * F
// or the build's record) when bit q * nf + j of `mask` is set (nf: F rounded
// up to a power of two), the layout the level count writes.  A wave takes
// runs of 64 level-2 pairs: each lane reads one pair, its pass bits and its
// triangle into the wave's LDS records, the run's (pair, child) items are
// listed in LDS in (pair, child) order -- the order of the level-1 pairs the
// emit would have written -- and tested 64 / G items at a time as k_hit
// tests pairs, up to MASKED_ITEMS items per round.
// (240 items keep a 256-thread block under 20 KiB of LDS: eight blocks per
// compute unit, the one round of blocks the launch assumes)
constexpr uint32_t MASKED_ITEMS = 240;
template <bool BATCH>
__global__ __launch_bounds__(256) void k_hit_masked(const float4 *__restrict__ RO, const float *__restrict__ RD,
                                                    const float4 *__restrict__ tri,
                                                    const uint32_t *__restrict__ ptri2,
                                                    const uint32_t *__restrict__ pnode2, uint64_t cap2,
                                                    const uint32_t *__restrict__ mask, uint32_t nf, uint32_t F,
                                                    uint32_t B, uint32_t log2G, unsigned long long *keys,
                                                    crsh_meta *meta, uint32_t slot_cap, uint32_t m, batch_dev bd,
                                                    float t_min)
{
    __shared__ uint64_t s_red[3][256 / WAVE];
    __shared__ float4 s_rec[256 / WAVE][3][WAVE];           // [wave][record word][pair of the run]
    __shared__ uint2 s_item[256 / WAVE][MASKED_ITEMS];     // [wave][item]: pair of the run, leaf
    const uint32_t ns = BATCH ? batch_slots(meta, B, slot_cap) : min(meta->n_rays, slot_cap);
    uint64_t n2 = meta->n_levels >= 2 ? meta->pairs[1] : 0;
    n2 = n2 < cap2 ? n2 : cap2;
    const uint32_t n1 = meta->level_cnt[0];
    const uint32_t off2 = meta->level_off[1];
    const uint32_t np2 = meta->level_cnt[1];
    const uint32_t l = lane_id();
    const uint32_t G = 1u << log2G;
    const uint32_t slot = l >> log2G;        // item of this lane within a step
    const uint32_t j = l & (G - 1);          // ray of the leaf
    const uint32_t per_wave = WAVE >> log2G;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + wib;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
    const __amdgpu_buffer_rsrc_t org_r = make_rsrc(RO, (uint64_t)ns * 16u);
    const __amdgpu_buffer_rsrc_t dir_r = make_rsrc(RD, (uint64_t)ns * 12u);
    const __amdgpu_buffer_rsrc_t tris_r = make_rsrc(tri, (uint64_t)m * 48u);
    const uint32_t nfm = nf >= 32 ? ~0u : (1u << nf) - 1u;
    float4(*rec)[WAVE] = s_rec[wib];
    uint2 *items = s_item[wib];
    uint64_t tests = 0, upass = 0, uvpass = 0;   // wave-wide counts
    for (uint64_t c0 = wave * WAVE; c0 < n2; c0 += nwaves * WAVE) {
        const uint32_t cn = __builtin_amdgcn_readfirstlane((uint32_t)min(n2 - c0, (uint64_t)WAVE));
        uint32_t my_t = 0u, bits = 0u, first = 0u;
        float my_tmin = t_min;                    // batched form: the pair's frame's
        if (l < cn) {
            const uint64_t q = c0 + l;
            my_t = ptri2[q];
            const uint32_t node = pnode2[q];
            const uint64_t bit = q * nf;          // nf divides 32: the bits lie in one word
            bits = (mask[bit >> 5] >> (uint32_t)(bit & 31u)) & nfm;
            if constexpr (BATCH) {
                first = node < np2 ? bd.node_first[off2 + node] : 0u;
                const uint32_t f = node < np2 ? bd.node_info[off2 + node] >> INFO_FRAME_SHIFT : bd.n_frames;
                my_tmin = f < bd.n_frames ? bd.frames[f].t_min : 0.0f;
                if (node >= np2) bits = 0u;
            } else {
                first = node * F;
            }
            if (my_t >= m) bits = 0u;
        }
        const uint32_t tb = bits ? my_t * 48u : 0u;
        const float4 ta = buf_load4(tris_r, tb);
        const float4 tbv = buf_load4(tris_r, tb + 16u);
        const float tc = buf_load1(tris_r, tb + 32u);
        const uint32_t cnt = (uint32_t)__popc(bits);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t excl = incl - cnt;
        const uint32_t total = __builtin_amdgcn_readlane(incl, WAVE - 1);
        __builtin_amdgcn_wave_barrier();          // the previous run's reads come first
        rec[0][l] = ta;
        rec[1][l] = tbv;
        rec[2][l] = make_float4(tc, __uint_as_float(my_t), my_tmin, 0.0f);
        for (uint32_t rb = 0; rb < total; rb += MASKED_ITEMS) {
            // this round's items: the lane's (pair, child) items with index
            // in [rb, rb + MASKED_ITEMS), in (pair, child) order
            __builtin_amdgcn_wave_barrier();      // the previous round's reads come first
            // an item holds the pair's lane and the leaf's ray count (bits 8
            // and up), and the byte offset of the leaf's first ray slot (slots
            // below 2^27: 32-bit arithmetic)
            uint32_t bl = bits, idx = excl;
            while (bl) {
                const uint32_t leaf = first + (uint32_t)__builtin_ctz(bl);
                bl &= bl - 1u;
                const uint32_t fs = leaf * B;
                const uint32_t rc = leaf < n1 && fs < ns ? min(B, ns - fs) : 0u;
                if (idx - rb < MASKED_ITEMS) items[idx - rb] = make_uint2(l | (rc << 8), rc ? fs * 16u : 0u);
                ++idx;
            }
            __builtin_amdgcn_wave_barrier();
            const uint32_t nit = min(MASKED_ITEMS, total - rb);
            for (uint32_t k = 0; k < nit; k += per_wave) {
                const uint32_t src = k + slot;
                const uint2 it = items[src < nit ? src : 0u];
                const uint32_t p = it.x & 63u;
                const float4 a = rec[0][p];
                const float4 b = rec[1][p];
                const float4 c = rec[2][p];
                const uint32_t cnt = src < nit ? it.x >> 8 : 0u;
                hit_step<BATCH, true>(org_r, dir_r, a, b, c.x, __float_as_uint(c.y), it.y, (it.y >> 2) * 3u, c.z,
                                      ballot(j < cnt), j, keys, tests, upass, uvpass);
            }
        }
    }
    hit_counts(s_red, wib, l, tests, upass, uvpass, meta);
}

struct hit_out {
    int32_t *tri;
    float *t, *u, *v;
};

// Batched form: the key of sorted ray s is the smaller of its slot's key and
// tkey[s] (the level-1 pairs of the fused path test by sorted ray), and is
// left in tkey[s] as in the plain form.
template <bool BATCH>
__global__ void k_hit_final(sorted_rays R, const float4 *__restrict__ tri, const uint32_t *__restrict__ sorted_ids,
                            float t_min0, unsigned long long *tkey, const unsigned long long *__restrict__ keys,
                            uint32_t B, uint32_t slot_cap, hit_out out, const crsh_meta *meta, uint32_t ray_cap,
                            uint32_t m, batch_dev bd)
{
    const uint32_t n = min(meta->n_rays, ray_cap);
    const uint32_t ns = BATCH ? batch_slots(meta, B, slot_cap) : 0u;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        unsigned long long key = tkey[s];
        const uint32_t id = sorted_ids[s];
        if (id >= ray_cap) continue;    // ids come from the sort: never taken
        float t_min = t_min0;
        if constexpr (BATCH) {
            const uint32_t f = min(bd.ray_frame[id], bd.n_frames - 1);
            t_min = bd.frames[f].t_min;
            const uint32_t rb = bd.fm[f].ray_begin;
            const uint64_t p = (uint64_t)bd.fm[f].level_base[0] * B + (s - rb);
            if (s >= rb && p < ns) key = min(key, keys[p]);
            tkey[s] = key;
        }
        int32_t best = -1;
        float th = 0.0f, uh = 0.0f, vh = 0.0f;
        if (key != ~0ull && (uint32_t)(key & 0xFFFFFFFFull) < m) {
            const uint32_t t = (uint32_t)(key & 0xFFFFFFFFull);
            const f3 O = mk(R.ox[s], R.oy[s], R.oz[s]);
            const f3 D = mk(R.dx[s], R.dy[s], R.dz[s]);
            if (moller_trumbore(O, D, t_min, R.tmax[s], load_tri(tri, t), th, uh, vh)) {
                best = (int32_t)t;
            } else {                     // cannot happen: same inputs, same operations
                best = (int32_t)t;
                th = hit_key_t(key);
            }
        }
        out.tri[id] = best;
        out.t[id] = th;
        out.u[id] = uh;
        out.v[id] = vh;
    }
}

__global__ void k_tkey_fill(unsigned long long *tkey, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) tkey[i] = ~0ull;
}

}  // namespace crsh

using namespace crsh;

extern "C" crsh_status crsh_hits_reset(crsh_hits *hits, hipStream_t stream)
{
    if (!hits || !hits->tkey) {
        set_error("crsh_hits_reset: NULL argument");
        return CRSH_ERR_INVALID;
    }
    uint32_t g = std::min<uint32_t>((hits->capacity + 255) / 256, 4096);
    if (g == 0) g = 1;
    k_tkey_fill<<<g, 256, 0, stream>>>(hits->tkey, hits->capacity);
    return hip_check(hipGetLastError(), "crsh_hits_reset launch");
}

namespace crsh {

void hit_prep_launch(const crsh_scene *scene, float4 *tri, hipStream_t stream)
{
    const float *const *v = scene->v;
    if (scene->m) {
        uint32_t g = std::min<uint32_t>((scene->m + 255) / 256, 2048);
        k_hit_prep<<<g, 256, 0, stream>>>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], scene->m, tri);
    }
}

void hit_pairs_launch(const crsh_rays *sorted, const float4 *tri, const hit_slots_ws &hs, const crsh_pairs *level1,
                      int32_t bundle, const crsh_scene *scene, float t_min, crsh_hits *hits, crsh_meta *meta,
                      const batch_dev *bd, int32_t hit_block, hipStream_t stream, bool packed, uint32_t tri_base)
{
    const uint32_t g = std::max<uint32_t>(std::min<uint32_t>((hs.slots + 255) / 256, 4096), 1);
    sorted_rays S{sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, sorted->tmax};
    if (bd)     // also the start value of every slot key, read by k_hit_final
        k_hit_rays_batch<<<g, 256, 0, stream>>>(S, meta, sorted->capacity, (uint32_t)bundle, hs.slots, *bd,
                                                hs.org, hs.dir, hs.keys);
    if (!level1->capacity) return;
    if (!bd) k_hit_rays<<<g, 256, 0, stream>>>(S, meta, sorted->capacity, hs.org, hs.dir);
    uint32_t log2G = 0;
    while ((1u << log2G) < (uint32_t)bundle) ++log2G;
    const uint32_t grid = 2048u * 256u / (uint32_t)hit_block;   // the same number of waves
    prof_scope ps("k_hit", stream);
    if (bd)
        k_hit<true, false><<<grid, hit_block, 0, stream>>>(hs.org, hs.dir, tri, level1->tri, level1->node,
                                                           level1->capacity, (uint32_t)bundle, log2G, hs.keys, meta,
                                                           hs.slots, scene->m, 0u, *bd, 0.0f);
    else if (packed)
        k_hit<false, true><<<grid, hit_block, 0, stream>>>(hs.org, hs.dir, tri, level1->tri, nullptr, level1->capacity,
                                                           (uint32_t)bundle, log2G, hits->tkey, meta, hs.slots,
                                                           scene->m, tri_base, batch_dev{}, t_min);
    else
        k_hit<false, false><<<grid, hit_block, 0, stream>>>(hs.org, hs.dir, tri, level1->tri, level1->node,
                                                            level1->capacity, (uint32_t)bundle, log2G, hits->tkey,
                                                            meta, hs.slots, scene->m, 0u, batch_dev{}, t_min);
}

void hit_masked_launch(const crsh_rays *sorted, const float4 *tri, const hit_slots_ws &hs, const crsh_pairs *level2,
                       const uint32_t *mask, int32_t merge, int32_t bundle, const crsh_scene *scene, float t_min,
                       crsh_hits *hits, crsh_meta *meta, const batch_dev *bd, int32_t hit_block, hipStream_t stream)
{
    (void)sorted;
    uint32_t nf = 2;
    while (nf < (uint32_t)merge) nf *= 2;
    uint32_t log2G = 0;
    while ((1u << log2G) < (uint32_t)bundle) ++log2G;
    const uint32_t grid = 2048u * 256u / (uint32_t)hit_block;
    const batch_dev b = bd ? *bd : batch_dev{};
    prof_scope ps("k_hit", stream);
    if (bd)
        k_hit_masked<true><<<grid, hit_block, 0, stream>>>(hs.org, hs.dir, tri, level2->tri, level2->node,
                                                           level2->capacity, mask, nf, (uint32_t)merge,
                                                           (uint32_t)bundle, log2G, hs.keys, meta, hs.slots,
                                                           scene->m, b, 0.0f);
    else
        k_hit_masked<false><<<grid, hit_block, 0, stream>>>(hs.org, hs.dir, tri, level2->tri, level2->node,
                                                            level2->capacity, mask, nf, (uint32_t)merge,
                                                            (uint32_t)bundle, log2G, hits->tkey, meta, hs.slots,
                                                            scene->m, b, t_min);
}

void hit_final_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, const float4 *tri,
                      const hit_slots_ws &hs, int32_t bundle, const crsh_scene *scene, float t_min,
                      crsh_hits *hits, crsh_meta *meta, const batch_dev *bd, hipStream_t stream)
{
    sorted_rays R{sorted->ox, sorted->oy, sorted->oz, sorted->dx, sorted->dy, sorted->dz, sorted->tmax};
    const batch_dev b = bd ? *bd : batch_dev{};
    uint32_t g = std::min<uint32_t>((sorted->capacity + 255) / 256, 4096);
    if (g == 0) g = 1;
    hit_out o{hits->tri, hits->t, hits->u, hits->v};
    prof_scope ps("k_hit_final", stream);
    if (bd)
        k_hit_final<true><<<g, 256, 0, stream>>>(R, tri, sorted_ids, t_min, hits->tkey, hs.keys, (uint32_t)bundle,
                                                 hs.slots, o, meta, sorted->capacity, scene->m, b);
    else
        k_hit_final<false><<<g, 256, 0, stream>>>(R, tri, sorted_ids, t_min, hits->tkey, nullptr, (uint32_t)bundle,
                                                  0u, o, meta, sorted->capacity, scene->m, b);
}

crsh_status hit_check(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle, const crsh_pairs *level1,
                      const crsh_scene *scene, crsh_hits *hits, crsh_meta *meta, void *ws, int32_t hit_block,
                      const char *who)
{
    if (!sorted || !sorted_ids || !level1 || !scene || !hits || !meta || !ws) {
        set_error("%s: NULL argument", who);
        return CRSH_ERR_INVALID;
    }
    if (bundle < 1 || bundle > CRSH_MAX_BUNDLE) {
        set_error("%s: bundle must be in [1, %d]", who, CRSH_MAX_BUNDLE);
        return CRSH_ERR_INVALID;
    }
    if (hit_block != 64 && hit_block != 128 && hit_block != 256) {
        set_error("%s: workgroup size must be 64, 128 or 256", who);
        return CRSH_ERR_INVALID;
    }
    if (!sorted->ox || !sorted->oy || !sorted->oz || !sorted->dx || !sorted->dy || !sorted->dz ||
        !sorted->tmax || !hits->tkey || !hits->tri || !hits->t || !hits->u || !hits->v ||
        (level1->capacity && (!level1->tri || !level1->node))) {
        set_error("%s: incomplete arrays", who);
        return CRSH_ERR_INVALID;
    }
    for (int k = 0; k < 9; ++k)
        if (!scene->v[k] && scene->m) {
            set_error("%s: missing vertex array", who);
            return CRSH_ERR_INVALID;
        }
    if (hits->capacity < sorted->capacity) {
        set_error("%s: hit capacity below the ray capacity", who);
        return CRSH_ERR_INVALID;
    }
    // the final tests address ray slots (16 B in each of two arrays) and
    // triangles (48 B) by 32-bit byte offsets
    if ((uint64_t)sorted->capacity + (uint64_t)CRSH_MAX_FRAMES * (CRSH_MAX_BUNDLE - 1) > CRSH_HIT_MAX_SLOTS ||
        scene->m > CRSH_HIT_MAX_TRIS) {
        set_error("%s: at most %u ray slots and %u triangles", who, (unsigned)CRSH_HIT_MAX_SLOTS,
                  (unsigned)CRSH_HIT_MAX_TRIS);
        return CRSH_ERR_INVALID;
    }
    return CRSH_OK;
}

crsh_status hit_launch(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle,
                       const crsh_pairs *level1, const crsh_scene *scene, float t_min, crsh_hits *hits,
                       crsh_meta *meta, void *ws, size_t ws_bytes, const batch_dev *bd, int32_t hit_block,
                       hipStream_t stream, bool packed, uint32_t tri_base)
{
    crsh_status st = hit_check(sorted, sorted_ids, bundle, level1, scene, hits, meta, ws, hit_block,
                               "crsh_closest_hit");
    if (st != CRSH_OK) return st;
    const uint32_t slots = hit_slots(sorted->capacity, bd != nullptr);
    if (ws_bytes < hit_ws_bytes(scene->m, slots)) {
        set_error("crsh_closest_hit: workspace too small (%zu < %zu)", ws_bytes, hit_ws_bytes(scene->m, slots));
        return CRSH_ERR_INVALID;
    }
    float4 *tri = (float4 *)ws;
    const hit_slots_ws hs = carve_hit_slots((char *)ws + align256((size_t)scene->m * 48), slots);
    hit_prep_launch(scene, tri, stream);
    hit_pairs_launch(sorted, tri, hs, level1, bundle, scene, t_min, hits, meta, bd, hit_block, stream, packed,
                     tri_base);
    hit_final_launch(sorted, sorted_ids, tri, hs, bundle, scene, t_min, hits, meta, bd, stream);
    return hip_check(hipGetLastError(), "crsh_closest_hit launch");
}

}  // namespace crsh

extern "C" crsh_status crsh_closest_hit(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle,
                                        const crsh_pairs *level1, const crsh_scene *scene, float t_min,
                                        crsh_hits *hits, crsh_meta *meta, void *ws, size_t ws_bytes,
                                        hipStream_t stream)
{
    return hit_launch(sorted, sorted_ids, bundle, level1, scene, t_min, hits, meta, ws, ws_bytes, nullptr, 256,
                      stream, false, 0u);
}

extern "C" crsh_status crsh_closest_hit_packed(const crsh_rays *sorted, const uint32_t *sorted_ids, int32_t bundle,
                                               const crsh_packed_pairs *level1, uint32_t tri_begin,
                                               const crsh_scene *scene, float t_min, crsh_hits *hits,
                                               crsh_meta *meta, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!level1) {
        set_error("crsh_closest_hit_packed: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (level1->capacity && !level1->pair) {
        set_error("crsh_closest_hit_packed: incomplete arrays");
        return CRSH_ERR_INVALID;
    }
    // the packed words travel in the triangle array; no node array
    crsh_pairs p{level1->pair, level1->pair, level1->capacity};
    return hit_launch(sorted, sorted_ids, bundle, &p, scene, t_min, hits, meta, ws, ws_bytes, nullptr, 256, stream,
                      true, tri_begin);
}
