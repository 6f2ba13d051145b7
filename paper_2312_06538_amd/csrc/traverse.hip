// Stage 4: hierarchy traversal (Sec. 3.3.7, Eq. 9).
//
// Every level is produced in three launches with no wait between blocks:
//   count  each work item (top level: one (top node, mesh) pair per wave;
//          lower levels: a tile of 256 parent pairs, one (parent, child)
//          test per lane, child nodes read from a run of them copied to
//          LDS) runs its Eq. 9 tests and records how many pass
//          (lower levels also keep the pass bits, one per child slot,
//          packed in 32-bit words);
//   scan   exclusive scan of the counts -> output offset of every item;
//   emit   each item writes its survivors at its offset, in (parent pair,
//          child) order -- at the top level (node, mesh, triangle) order;
//          lower levels in tiles of two count tiles, staged through LDS.
// The pair arrays therefore come out trimmed (Fig. 4) and in the order of a
// sequential traversal, so they are deterministic.  Work is spread with
// grid-stride loops; nothing depends on which blocks are resident.  Pairs are
// two arrays (triangle, node) or, for crsh_traverse_packed, one 32-bit word
// each (Sec. 3.3.7's encoding), a compile-time choice of every kernel.
//
// Batched form: frames have their own top levels, so levels are produced from
// the highest down; on each level the pairs that descend from the level above
// come first, then a top-level pass appends the (node, mesh, triangle) pairs
// of the frames whose top is this level.  A top-level item is (frame, top
// node, mesh of the frame); a parent's children are the range recorded with
// it by the build (first child, count), so below the top a frame is looked
// up only when a count block copies a new run of child nodes to LDS.
#include "bounds.hpp"
#include "traverse.hpp"


namespace crsh {

__global__ void k_tri_sph(const float *__restrict__ v0x, const float *__restrict__ v0y,
                          const float *__restrict__ v0z, const float *__restrict__ v1x,
                          const float *__restrict__ v1y, const float *__restrict__ v1z,
                          const float *__restrict__ v2x, const float *__restrict__ v2y,
                          const float *__restrict__ v2z, uint32_t b, uint32_t e, float4 *out)
{
    const float third = 1.0f / 3.0f;
    for (uint32_t t = b + blockIdx.x * blockDim.x + threadIdx.x; t < e; t += gridDim.x * blockDim.x) {
        f3 a = mk(v0x[t], v0y[t], v0z[t]);
        f3 bb = mk(v1x[t], v1y[t], v1z[t]);
        f3 c = mk(v2x[t], v2y[t], v2z[t]);
        f3 ctr = ((a + bb) + c) * third;
        float r = fmax2(fmax2(len(a - ctr), len(bb - ctr)), len(c - ctr));
        float m = fmax2(fmax2(fabsf(ctr.x), fabsf(ctr.y)), fabsf(ctr.z));
        r = r + SPHERE_PAD * (r + m);
        out[t] = make_float4(ctr.x, ctr.y, ctr.z, r);
    }
}

// Traversal copy of the nodes: (cx, cy, cz, r), (ax, ay, az, tan) and sec,
// with sec = -1 marking a cone of 90 degrees or more (c <= 0 gives no
// positive sec, c > 0 always does), so one test reads 36 bytes in 3 loads.
// Also clears the per-call pair counts.
__global__ void k_node_pack(node_arrays nd, crsh_meta *meta, float4 *na, float4 *nb, float *ns, bool clear_pairs)
{
    const uint32_t nl = meta->n_levels;
    const uint32_t total = nl ? meta->level_off[nl - 1] + meta->level_cnt[nl - 1] : 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        na[i] = make_float4(nd.cx[i], nd.cy[i], nd.cz[i], nd.r[i]);
        nb[i] = make_float4(nd.ax[i], nd.ay[i], nd.az[i], nd.tan[i]);
        ns[i] = nd.c[i] > 0.0f ? nd.sec[i] : -1.0f;
    }
    if (clear_pairs && blockIdx.x == 0 && threadIdx.x < CRSH_MAX_LEVELS) meta->pairs[threadIdx.x] = 0;
}

// number of work items of a level: top level (parent_level 0) = top nodes x
// meshes, lower levels = tiles of LEVEL_TILE parent pairs
__device__ __forceinline__ uint64_t level_items(const crsh_meta *meta, int32_t parent_level, uint32_t n_mesh,
                                                const pair_levels &P)
{
    const uint32_t nl = meta->n_levels;
    if (parent_level == 0) return nl ? (uint64_t)meta->level_cnt[nl - 1] * n_mesh : 0;
    if ((uint32_t)parent_level > nl || parent_level < 2) return 0;
    uint64_t nin = meta->pairs[parent_level - 1];
    const uint64_t cap = P.p[parent_level - 1].cap;
    nin = nin < cap ? nin : cap;
    return (nin + LEVEL_TILE - 1) / LEVEL_TILE;
}

__device__ __forceinline__ void clear_scan(const trav_scratch &S, uint64_t items)
{
    const uint64_t nt = (items + SCAN_TILE - 1) / SCAN_TILE;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = gid; i < nt; i += (uint64_t)gridDim.x * blockDim.x) S.scan_flags[i] = 0;
    if (gid == 0) *S.scan_ctr = 0;
}

// ------------------------------------------------------------- top level
// Item -> (node i within the level, mesh m).  Plain: item = i * n_mesh + m.
// Batch: the item's frame, then (top node, mesh) within the frame.
template <bool BATCH>
__device__ __forceinline__ void top_item(uint64_t item, uint32_t n_mesh, uint32_t top, uint32_t off,
                                         const batch_dev &bd, const float4 *na, const float4 *nb, const float *ns,
                                         const float *msph, const uint32_t *mesh_first, const uint32_t *mesh_count,
                                         uint32_t tri_begin, uint32_t tri_end, float4 &A, float4 &Bv, float &S,
                                         uint32_t &i, uint32_t &b, uint32_t &e, bool &pass)
{
    uint32_t m;
    if constexpr (BATCH) {
        const uint32_t f = frame_of_item(bd, item);
        const uint64_t local = item - bd.fm[f].item_base;
        const uint32_t mc = bd.frames[f].mesh_count;
        const uint32_t li = (uint32_t)(local / mc);
        i = bd.fm[f].level_base[top] + li;
        m = bd.frames[f].mesh_begin + (uint32_t)(local - (uint64_t)li * mc);
    } else {
        i = (uint32_t)item / n_mesh;
        m = (uint32_t)item - i * n_mesh;
    }
    A = na[off + i];
    Bv = nb[off + i];
    S = ns[off + i];
    const bool real = !BATCH || m < n_mesh;    // frames name meshes of the batch's scene
    if (!real) m = 0;
    pass = real && packed_meets(A, Bv, S, mk(msph[4 * m], msph[4 * m + 1], msph[4 * m + 2]), msph[4 * m + 3]);
    b = e = 0;
    if (pass) {
        b = max(mesh_first[m], tri_begin);
        e = min(mesh_first[m] + mesh_count[m], tri_end);
        if (e < b) e = b;
    }
}

// top level of this pass (0-based) and its number of items
template <bool BATCH>
__device__ __forceinline__ bool top_pass(const crsh_meta *meta, const batch_dev &bd, uint32_t L, uint32_t n_mesh,
                                         const pair_levels &P, uint32_t &top, uint64_t &n_items)
{
    const uint32_t nl = meta->n_levels;
    if (nl == 0) return false;
    if constexpr (BATCH) {
        if (L > nl) return false;
        top = L - 1;
        n_items = bd.top[0];
    } else {
        top = nl - 1;
        n_items = level_items(meta, 0, n_mesh, P);
    }
    return true;
}

template <bool BATCH>
__global__ __launch_bounds__(256) void k_top_count(const float4 *__restrict__ na, const float4 *__restrict__ nb,
                                                   const float *__restrict__ ns, const float4 *__restrict__ tsph,
                                                   const uint32_t *__restrict__ mesh_first,
                                                   const uint32_t *__restrict__ mesh_count,
                                                   const float *__restrict__ msph, uint32_t n_mesh,
                                                   uint32_t tri_begin, uint32_t tri_end, pair_levels P,
                                                   trav_scratch S, crsh_meta *meta, batch_dev bd, uint32_t L)
{
    __shared__ uint64_t s_red[3][256 / WAVE];
    uint32_t top;
    uint64_t n_items;
    if (!top_pass<BATCH>(meta, bd, L, n_mesh, P, top, n_items)) return;
    clear_scan(S, n_items);
    const uint32_t off = meta->level_off[top];
    const uint32_t l = lane_id();
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
    uint64_t tests = 0, mhits = 0, items = 0;
    for (uint64_t it = wave; it < n_items; it += nwaves) {
        float4 A, Bv;
        float Sg;
        uint32_t i, b, e;
        bool pass;
        top_item<BATCH>(it, n_mesh, top, off, bd, na, nb, ns, msph, mesh_first, mesh_count, tri_begin, tri_end,
                        A, Bv, Sg, i, b, e, pass);
        ++items;
        mhits += pass ? 1 : 0;
        tests += e - b;
        uint32_t cnt = 0;
        for (uint32_t t0 = b; t0 < e; t0 += WAVE) {
            const uint32_t t = t0 + l;
            bool ok = false;
            if (t < e) {
                const float4 s = tsph[t];
                ok = packed_meets(A, Bv, Sg, mk(s.x, s.y, s.z), s.w);
            }
            cnt += (uint32_t)__popcll(ballot(ok));
        }
        if (l == 0) S.cnt[it] = cnt;
    }
    if (l == 0) {
        s_red[0][threadIdx.x / WAVE] = tests;
        s_red[1][threadIdx.x / WAVE] = mhits;
        s_red[2][threadIdx.x / WAVE] = items;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, bq = 0, c = 0;
        for (int w = 0; w < 256 / WAVE; ++w) {
            a += s_red[0][w];
            bq += s_red[1][w];
            c += s_red[2][w];
        }
        if (a) atomicAdd((unsigned long long *)&meta->tests[top], (unsigned long long)a);
        if (bq) atomicAdd((unsigned long long *)&meta->mesh_hits, (unsigned long long)bq);
        if (c) atomicAdd((unsigned long long *)&meta->mesh_tests, (unsigned long long)c);
    }
}

template <bool BATCH, bool PACKED = false>
__global__ __launch_bounds__(256) void k_top_emit(const float4 *__restrict__ na, const float4 *__restrict__ nb,
                                                  const float *__restrict__ ns, const float4 *__restrict__ tsph,
                                                  const uint32_t *__restrict__ mesh_first,
                                                  const uint32_t *__restrict__ mesh_count,
                                                  const float *__restrict__ msph, uint32_t n_mesh,
                                                  uint32_t tri_begin, uint32_t tri_end, pair_levels P,
                                                  trav_scratch S, const crsh_meta *meta, batch_dev bd, uint32_t L)
{
    uint32_t top;
    uint64_t n_items;
    if (!top_pass<BATCH>(meta, bd, L, n_mesh, P, top, n_items)) return;
    const pairs_dev out = P.p[top];
    if (out.tri == nullptr) return;
    const uint32_t off = meta->level_off[top];
    const uint32_t l = lane_id();
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
    for (uint64_t it = wave; it < n_items; it += nwaves) {
        if (S.cnt[it] == 0) continue;
        float4 A, Bv;
        float Sg;
        uint32_t i, b, e;
        bool pass;
        top_item<BATCH>(it, n_mesh, top, off, bd, na, nb, ns, msph, mesh_first, mesh_count, tri_begin, tri_end,
                        A, Bv, Sg, i, b, e, pass);
        uint64_t pos = S.off[it];
        for (uint32_t t0 = b; t0 < e; t0 += WAVE) {
            const uint32_t t = t0 + l;
            bool ok = false;
            if (t < e) {
                const float4 s = tsph[t];
                ok = packed_meets(A, Bv, Sg, mk(s.x, s.y, s.z), s.w);
            }
            const uint64_t mask = ballot(ok);
            const uint64_t at = pos + rank_below(mask);
            if (ok && at < out.cap) {
                pair_put<PACKED>(out, at, t, i);
            }
            pos += (uint32_t)__popcll(mask);
        }
    }
}

// ----------------------------------------------------------- lower levels
// Lane i of each quad of four lanes gets the value of lane (i / NF) * NF + r
// of its quad (NF <= 4: the NF lanes of a group share one source lane).  r
// is a constant once the slice loop is unrolled; the switch folds away.
template <uint32_t NF>
__device__ __forceinline__ uint32_t quad_pick(uint32_t v, uint32_t r)
{
    static_assert(NF == 2 || NF == 4, "groups within a quad");
#define CRSH_QP(R) ((((0 / NF) * NF + (R)) & 3) | ((((1 / NF) * NF + (R)) & 3) << 2) | \
                    ((((2 / NF) * NF + (R)) & 3) << 4) | ((((3 / NF) * NF + (R)) & 3) << 6))
    switch (r) {
    case 0: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CRSH_QP(0), 0xF, 0xF, true);
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CRSH_QP(1), 0xF, 0xF, true);
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CRSH_QP(2), 0xF, 0xF, true);
    default: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CRSH_QP(3), 0xF, 0xF, true);
    }
#undef CRSH_QP
}
template <uint32_t NF>
__device__ __forceinline__ float quad_pick(float v, uint32_t r)
{
    return __uint_as_float(quad_pick<NF>(__float_as_uint(v), r));
}
// The same through the other DPP builtin: a second, separate copy of a value
// quad_pick already took (the compiler folds a DPP move into the one
// instruction that uses it, and would merge two identical moves).
template <uint32_t NF>
__device__ __forceinline__ float quad_pick_again(float v, uint32_t r)
{
#define CRSH_QP(R) ((((0 / NF) * NF + (R)) & 3) | ((((1 / NF) * NF + (R)) & 3) << 2) | \
                    ((((2 / NF) * NF + (R)) & 3) << 4) | ((((3 / NF) * NF + (R)) & 3) << 6))
    const int x = (int)__float_as_uint(v);
    switch (r) {
    case 0: return __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(0, x, CRSH_QP(0), 0xF, 0xF, true));
    case 1: return __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(0, x, CRSH_QP(1), 0xF, 0xF, true));
    case 2: return __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(0, x, CRSH_QP(2), 0xF, 0xF, true));
    default: return __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(0, x, CRSH_QP(3), 0xF, 0xF, true));
    }
#undef CRSH_QP
}

// Count pass with one (parent pair, child) test per lane.
// A tile of LEVEL_TILE parent pairs is tested in NF slices of LEVEL_TILE /
// NF parents; in a slice the NF lanes of a parent test its NF consecutive
// children, and the wave's ballot is directly the pass bits of its 64 / NF
// parents in the mask layout of the count pass (NF bits per parent,
// parent-major).  A block of COUNT_THREADS takes COUNT_TPS tiles per step.
// What the NF lanes of a parent share -- the parent's children and the
// triangle sphere -- is read once: each lane reads the pair and sphere of
// one of the wave's 64 parents of the tile.  For NF <= 4 that lane is one
// of the parent's NF lanes (lane NF * p + r holds parent p of slice r), and
// in slice r the others take the values from it within their quad of lanes
// (a DPP broadcast, no LDS); for larger NF the lanes put them in a
// wave-private LDS record and the lanes of a slice read their parent's
// record from there.  The next step's pairs and spheres are requested
// before a step is tested (pairs two steps ahead, since the sphere read
// depends on them).
//
// Child nodes (36 bytes a test) come from LDS where they can: the
// descendants of one top-level node on the child level are a contiguous
// run of F^(levels above the child level) nodes, aligned to that length
// from the frame's first node of the level, and the pairs of a level are
// ordered by top-level node first, so a block's consecutive steps keep
// testing children from the same run.  When the run fits COUNT_WINDOW
// nodes, the block copies the run holding its step's first child, and the
// runs after it as far as the window reaches within the frame, into LDS
// (once per window it enters; the batched form looks the frame up only
// then) and its waves read the children there; a group of slices with a
// child outside the window reads the node arrays directly.  In the batched form a
// parent's children are the range the build recorded with it (first,
// count); the lane that reads a parent's pair reads that record too, in the
// same stage as the sphere, and puts it in the parent's LDS record.
template <int NF, bool BATCH, bool PACKED, bool STAGED>
__global__ __launch_bounds__(COUNT_THREADS) void k_level_count_lanes(int32_t parent_level, uint32_t F,
                                                                     const float4 *__restrict__ na,
                                                                     const float4 *__restrict__ nb,
                                                                     const float *__restrict__ ns,
                                                                     const float4 *__restrict__ tsph, uint32_t m,
                                                                     pair_levels P, trav_scratch S, crsh_meta *meta,
                                                                     batch_dev bd)
{
    static_assert(LEVEL_PPT == 1 && WAVE % NF == 0, "whole parents per wave");
    constexpr uint32_t PR = LEVEL_THREADS / NF;   // parents per slice; NF slices make a tile
    constexpr uint32_t PW = WAVE / NF;            // parents of a wave per slice
    constexpr uint32_t WPT = LEVEL_THREADS / WAVE;   // waves per tile
    constexpr uint32_t NW = COUNT_THREADS / WAVE;    // waves per block
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    constexpr uint32_t WN = STAGED ? COUNT_WINDOW : 1u;
    constexpr bool QB = NF <= 4;             // parent values by quad broadcast
    constexpr uint32_t NR = QB ? 1u : NW;    // wave records in LDS
    __shared__ uint32_t s_red32[2][NW];
    __shared__ uint64_t s_red[NW];
    __shared__ uint32_t s_head[2];          // the step's first pair: 16 x (first child, children)
    __shared__ float4 s_sph[NR][WAVE];      // [wave][record]
    __shared__ uint32_t s_first[NR][WAVE];  // 16 x first child (level-local)
    __shared__ uint32_t s_n[NR][WAVE];      // 16 x children below nk (0: none)
    __shared__ float4 s_wa[WN], s_wb[WN];   // the staged run of child nodes
    __shared__ float s_ws[WN];
    const uint32_t nl = meta->n_levels;
    if ((uint32_t)parent_level > nl || parent_level < 2) return;
    const uint64_t ntiles = level_items(meta, parent_level, 0, P);
    clear_scan(S, ntiles);                  // the scan that follows reads these
    const pairs_dev in = P.p[parent_level - 1];
    if (in.tri == nullptr || P.p[parent_level - 2].tri == nullptr) return;
    uint64_t nin = meta->pairs[parent_level - 1];
    nin = nin < in.cap ? nin : in.cap;
    const uint64_t nsteps = (ntiles + COUNT_TPS - 1) / COUNT_TPS;
    const uint32_t nk = meta->level_cnt[parent_level - 2];
    const uint32_t offk = meta->level_off[parent_level - 2];
    const uint32_t offp = meta->level_off[parent_level - 1];
    const uint32_t np = meta->level_cnt[parent_level - 1];
    const uint32_t F16 = F * 16u, nk16 = nk * 16u;
    const uint32_t l = lane_id();
    // wave indices, made scalar so that the addresses built from them are
    // scalar arithmetic
    const uint32_t wb = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wave of the block
    const uint32_t half = wb / WPT;                   // tile of the step
    const uint32_t tw = wb % WPT;                     // wave of the tile
    const uint32_t j = l % NF;              // child of this lane in every slice
    const uint32_t j16 = j * 16u;
    const uint32_t mlane = l == 0 ? 0u : 0x80000000u;   // mask stores: past the range but for lane 0
    const uint32_t pi = l / NF;             // parent of this lane within the wave's slice
    // the parent whose pair and sphere this lane reads: quad broadcast,
    // slice j, parent pi of the wave's share of it; else slice l / PW,
    // parent l % PW
    const uint32_t own = QB ? j * PR + tw * PW + pi : (l / PW) * PR + tw * PW + l % PW;
    // nodes from offk + ch for ch < nk, by 32-bit byte offsets
    const uint64_t nodes = (uint64_t)offk + nk;
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(na, nodes * 16u);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(nb, nodes * 16u);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(ns, nodes * 4u);
    // descendants of one top-level node on the child level of a hierarchy
    // with `levels` levels: F^(levels - L + 1) (above WN: more than the
    // window holds)
    auto run_of = [&](uint32_t levels) {
        uint32_t run = 1;
        for (uint32_t e = 0; e < levels - (uint32_t)parent_level + 1 && run <= WN; ++e) run *= F;
        return run;
    };
    // STAGED: the host's bound on the runs of this level fits the window
    const bool staged = STAGED && (BATCH || run_of(nl) <= WN);
    uint32_t wlo = NONE, wlen = 0;          // staged run (block-uniform)
    uint32_t wlo16 = 0u, wlen16 = 0u;       // the same, x 16
    uint32_t ulo = NONE, ulen = 0;          // batch: a frame's nodes whose runs do not fit
    // the pair this lane reads for a step, by buffer loads over the tile's
    // pairs (a step past the end reads nothing): no branch, so that the
    // loads of every step count alike where the compiler places its waits
    auto load_pair = [&](uint64_t step, uint32_t &tri, uint32_t &par) {
        const uint64_t q0 = (step * COUNT_TPS + half) * LEVEL_TILE;
        // pairs of the tile: min(nin - q0, LEVEL_TILE), 0 past the end, in
        // 32-bit scalar operations (both below 2^63)
        const uint64_t left = nin - q0;
        const uint32_t lhi = (uint32_t)(left >> 32), llo = (uint32_t)left;
        const uint32_t nq = lhi == 0u ? min(llo, (uint32_t)LEVEL_TILE) : (lhi >> 31 ? 0u : (uint32_t)LEVEL_TILE);
        const __amdgpu_buffer_rsrc_t rt = make_rsrc(in.tri + q0, (uint64_t)nq * 4u);
        const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rt, own * 4u, 0, 0);
        if constexpr (PACKED) {
            tri = in.tri_base + (w & ((1u << CRSH_PACKED_TRI_BITS) - 1u));
            par = own < nq ? w >> CRSH_PACKED_TRI_BITS : NONE;
        } else {
            const __amdgpu_buffer_rsrc_t rn = make_rsrc(in.node + q0, (uint64_t)nq * 4u);
            tri = w;
            par = own < nq ? __builtin_amdgcn_raw_buffer_load_b32(rn, own * 4u, 0, 0) : NONE;
        }
    };
    uint64_t tests = 0;                     // wave-wide
    uint32_t parity = 0;
    // a parent's children: plain, par * F + [0, F); batch, the build's
    // record (level-local first child, count); as 16 x (first, number below
    // nk), byte offsets into the staged run (node indices stay below 2^28:
    // 32-bit byte offsets into the node arrays)
    auto children = [&](uint32_t par, uint32_t &first16, uint32_t &n16) {
        if constexpr (BATCH) {
            const bool ok = par < np;
            const uint32_t first = ok ? bd.node_first[offp + par] : 0u;
            const uint32_t cnt = ok ? bd.node_info[offp + par] & INFO_COUNT_MASK : 0u;
            first16 = first < nk ? first * 16u : 0u;
            n16 = first < nk ? (min(first + cnt, nk) - first) * 16u : 0u;
        } else {
            // a parent below np has its first child below nk; F16, nk16:
            // F and nk times 16 (scalar); first16 of no parent is never read
            first16 = par * F16;
            n16 = par < np ? min(F16, nk16 - first16) : 0u;
        }
    };
    // two-stage prefetch: the sphere (and batch: the child range) of the
    // next step and the pair of the step after it are in flight while a
    // step is tested
    uint32_t first_n = 0u, n_n = 0u, tri_nn = 0u, par_nn = NONE;
    float4 sp_n = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (blockIdx.x < nsteps) {
        uint32_t tri0, par0;
        load_pair(blockIdx.x, tri0, par0);
        sp_n = tsph[tri0 < m ? tri0 : 0u];
        children(par0, first_n, n_n);
        load_pair(blockIdx.x + gridDim.x, tri_nn, par_nn);
    }
    // the prologue's loads are in before the loop: the waits the compiler
    // places in the loop then count only the loop's own memory operations
    // (not every store of the previous step)
    __builtin_amdgcn_s_waitcnt(0x0F70);     // vmcnt(0)
    // a 32-bit step index (steps stay far below 2^31: 512 pairs a step), so
    // the loop's bookkeeping is scalar arithmetic
    const uint32_t nsteps32 = (uint32_t)min(nsteps, (uint64_t)0x7FFFFFFFu);
    for (uint32_t step = blockIdx.x; step < nsteps32; step += gridDim.x, parity ^= 1u) {
        const uint64_t tile = step * COUNT_TPS + half;
        // this wave's slice-0 word of the tile's pass masks (scalar)
        uint2 *const mrow = (uint2 *)S.mask + (tile * LEVEL_TILE + tw * PW) * NF / 64;
        const __amdgpu_buffer_rsrc_t mrs = make_rsrc(mrow, tile < ntiles ? (NF - 1) * (PR * NF / 64) * 8u + 8u : 0u);
        // this step's parent values: kept in registers (quad broadcast) or
        // put in the wave's records (the wave's previous reads of them are
        // done: program order within the wave); the step's first pair is
        // lane 0's of wave 0
        const float4 sp_c = sp_n;
        const uint32_t first_c = first_n, n_c = n_n;
        if constexpr (!QB) {
            __builtin_amdgcn_wave_barrier();
            s_sph[wb][l] = sp_n;
            s_first[wb][l] = first_n;
            s_n[wb][l] = n_n;
            __builtin_amdgcn_wave_barrier();
        }
        if (staged && wb == 0 && l == 0) {
            s_head[0] = first_n;
            s_head[1] = n_n;
        }
        if (staged) {
            // every wave has finished its reads of the staged run (they
            // precede the previous step's count barrier)
            __syncthreads();
            const uint32_t c0 = s_head[0] / 16u;
            if (s_head[1] != 0u && c0 - wlo >= wlen && c0 - ulo >= ulen) {
                // the frame's nodes on the child level and its levels
                uint32_t base = 0u, cntf = nk, levels = nl;
                if constexpr (BATCH) {
                    const uint32_t f = frame_of_node(bd, (uint32_t)parent_level - 2, c0);
                    base = bd.fm[f].level_base[parent_level - 2];
                    cntf = bd.fm[f].level_cnt[parent_level - 2];
                    levels = bd.fm[f].n_levels;
                }
                const uint32_t run = run_of(levels);
                if (run <= WN && c0 >= base && c0 - base < cntf) {
                    // as many whole runs as the window holds, from the one
                    // holding c0 (later steps move on to the next runs)
                    const uint32_t lo = base + (c0 - base) / run * run;
                    const uint32_t len = min(WN / run * run, base + cntf - lo);
                    for (uint32_t i = threadIdx.x; i < len; i += COUNT_THREADS) {
                        s_wa[i] = na[offk + lo + i];
                        s_wb[i] = nb[offk + lo + i];
                        s_ws[i] = ns[offk + lo + i];
                    }
                    __syncthreads();
                    wlo = lo;
                    wlen = len;
                    wlo16 = lo * 16u;
                    wlen16 = len * 16u;
                } else {
                    ulo = base;
                    ulen = cntf;
                }
            }
        }
        sp_n = tsph[tri_nn < m ? tri_nn : 0u];
        children(par_nn, first_n, n_n);
        load_pair(step + 2u * gridDim.x, tri_nn, par_nn);
        uint32_t c = 0;
        // slices in groups of K: every node read of a group is issued before
        // its first test, and the test has no branch to sink them into.
        // Which lanes test a child, and which of those find it outside the
        // staged run, are wave masks (scalar registers), and so are the
        // results; children outside the run are read from the node arrays
        // afterwards, in a branch of their own, so the reads from LDS never
        // wait behind memory loads.
        constexpr uint32_t KG = 2;
        constexpr uint32_t K = NF < KG ? NF : KG;
#pragma unroll
        for (uint32_t r0 = 0; r0 < NF; r0 += K) {
            uint64_t okm[K], outm[K], bal[K];
            uint32_t ch16[K], idx16[K];
            f3 pc[K];                       // the parent's triangle sphere (records)
            float pr[K];
            // the same by quad broadcast, taken where it is used (each copy
            // has one use: the compiler folds it into that instruction)
            auto sph_c = [&](uint32_t k) {
                if constexpr (QB)
                    return mk(quad_pick<NF>(sp_c.x, r0 + k), quad_pick<NF>(sp_c.y, r0 + k), quad_pick<NF>(sp_c.z, r0 + k));
                else
                    return pc[k];
            };
            auto sph_r = [&](uint32_t k) {
                if constexpr (QB)
                    return quad_pick<NF>(sp_c.w, r0 + k);
                else
                    return pr[k];
            };
#pragma unroll
            for (uint32_t k = 0; k < K; ++k) {
                const uint32_t r = r0 + k;
                uint32_t f16, n16;
                if constexpr (QB) {
                    f16 = quad_pick<NF>(first_c, r);
                    n16 = quad_pick<NF>(n_c, r);
                } else {
                    const uint32_t rec = r * PW + pi;
                    f16 = s_first[wb][rec];
                    n16 = s_n[wb][rec];
                    const float4 sp = s_sph[wb][rec];
                    pc[k] = mk(sp.x, sp.y, sp.z);
                    pr[k] = sp.w;
                }
                ch16[k] = f16 + j16;
                okm[k] = ballot(j16 < n16);
                const uint32_t i16 = ch16[k] - wlo16;
                outm[k] = okm[k] & ~ballot(i16 < wlen16);
                // any slot of the window for a lane that tests nothing here
                idx16[k] = min(i16, (WN - 1u) * 16u);
            }
            if constexpr (STAGED) {
                float4 A[K], Bv[K];
                float Sg[K];
#pragma unroll
                for (uint32_t k = 0; k < K; ++k) {
                    A[k] = *(const float4 *)((const char *)s_wa + idx16[k]);
                    Bv[k] = *(const float4 *)((const char *)s_wb + idx16[k]);
                    Sg[k] = *(const float *)((const char *)s_ws + idx16[k] / 4u);
                }
#pragma unroll
                for (uint32_t k = 0; k < K; ++k)
                    bal[k] = packed_meets_mask(A[k], Bv[k], Sg[k], sph_c(k), sph_r(k)) & okm[k] & ~outm[k];
                // rare: a slice with children outside the run, one at a time
                uint64_t any_out = 0;
#pragma unroll
                for (uint32_t k = 0; k < K; ++k) any_out |= outm[k];
                if (any_out != 0) {
#pragma unroll
                    for (uint32_t k = 0; k < K; ++k) {
                        if (outm[k] == 0) continue;
                        const uint32_t g = offk + (((outm[k] >> l) & 1u) ? ch16[k] / 16u : 0u);
                        const float4 Ag = buf_load4(ra, g * 16u);
                        const float4 Bg = buf_load4(rb, g * 16u);
                        const float Sgg = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, g * 4u, 0, 0));
                        f3 c = pc[k];
                        float d = pr[k];
                        if constexpr (QB) {     // copies of its own (see sph_c)
                            c = mk(quad_pick_again<NF>(sp_c.x, r0 + k), quad_pick_again<NF>(sp_c.y, r0 + k),
                                   quad_pick_again<NF>(sp_c.z, r0 + k));
                            d = quad_pick_again<NF>(sp_c.w, r0 + k);
                        }
                        bal[k] |= packed_meets_mask(Ag, Bg, Sgg, c, d) & outm[k];
                    }
                }
            } else {
                // runs longer than the window: every child from the node
                // arrays, the group's loads issued together (outm == okm)
                float4 A[K], Bv[K];
                float Sg[K];
#pragma unroll
                for (uint32_t k = 0; k < K; ++k) {
                    const uint32_t g = offk + (((okm[k] >> l) & 1u) ? ch16[k] / 16u : 0u);
                    A[k] = buf_load4(ra, g * 16u);
                    Bv[k] = buf_load4(rb, g * 16u);
                    Sg[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, g * 4u, 0, 0));
                }
#pragma unroll
                for (uint32_t k = 0; k < K; ++k)
                    bal[k] = packed_meets_mask(A[k], Bv[k], Sg[k], sph_c(k), sph_r(k)) & okm[k];
            }
#pragma unroll
            for (uint32_t k = 0; k < K; ++k) {
                const uint32_t r = r0 + k;
                tests += (uint64_t)__popcll(okm[k]);
                // the wave's pass bits of slice r: bit (tile * LEVEL_TILE +
                // r * PR + tw * PW) * NF of the level's masks, a multiple of 64
                // (r * PR * NF = 64 r words' worth of 4 bits: uint2 4 r).
                // Every lane stores, lane 0 in range: no branch around it
                typedef uint32_t v2u __attribute__((ext_vector_type(2)));
                const v2u w = {(uint32_t)bal[k], (uint32_t)(bal[k] >> 32)};
                __builtin_amdgcn_raw_buffer_store_b64(w, mrs, mlane + r * (PR * NF / 64) * 8u, 0, 0);
                c += (uint32_t)__popcll(bal[k]);
            }
        }
        // survivors of each tile: wave sums in alternating LDS slots (one
        // barrier per step)
        if (l == 0) s_red32[parity][wb] = c;
        __syncthreads();
        if (threadIdx.x % LEVEL_THREADS == 0 && tile < ntiles) {
            uint32_t t = 0;
            for (uint32_t ww = 0; ww < WPT; ++ww) t += s_red32[parity][half * WPT + ww];
            S.cnt[tile] = t;
        }
    }
    if (l == 0) s_red[wb] = tests;          // a wave-wide count: the same in every lane
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tt = 0;
        for (uint32_t ww = 0; ww < NW; ++ww) tt += s_red[ww];
        if (tt) atomicAdd((unsigned long long *)&meta->tests[parent_level - 2], (unsigned long long)tt);
    }
}

// Survivors of a tile are first placed in LDS at their tile-local offsets
// and then copied out with consecutive lanes writing consecutive pairs, so
// the stores are coalesced whatever the pass masks.
// Emit pass: PPT parent pairs per thread, EMIT_TILE per block iteration,
// covering EMIT_PPT / LEVEL_PPT count tiles (their masks, survivor counts and
// the first one's output offset).
template <int NF, int PPT, bool BATCH, bool PACKED = false>
__global__ __launch_bounds__(LEVEL_THREADS) void k_level_emit(int32_t parent_level, uint32_t F, pair_levels P,
                                                              trav_scratch S, const crsh_meta *meta, batch_dev bd)
{
    static_assert(PPT * NF <= 32, "one bit per child");
    constexpr uint32_t TILE = LEVEL_THREADS * PPT;
    constexpr uint32_t TILE_OUT = TILE * NF;
    constexpr uint32_t R = PPT / LEVEL_PPT;    // count tiles per emit tile
    static_assert(PPT % LEVEL_PPT == 0, "whole count tiles");
    __shared__ uint32_t s_scan[LEVEL_THREADS / WAVE];
    __shared__ uint32_t s_tri[TILE_OUT];
    __shared__ uint32_t s_node[TILE_OUT];
    const uint32_t nl = meta->n_levels;
    if ((uint32_t)parent_level > nl) return;
    const pairs_dev in = P.p[parent_level - 1];
    const pairs_dev out = P.p[parent_level - 2];
    if (in.tri == nullptr || out.tri == nullptr) return;
    uint64_t nin = meta->pairs[parent_level - 1];
    nin = nin < in.cap ? nin : in.cap;
    const uint64_t ctiles = (nin + LEVEL_TILE - 1) / LEVEL_TILE;
    const uint64_t ntiles = (nin + TILE - 1) / TILE;
    const uint32_t offp = meta->level_off[parent_level - 1];
    const uint32_t np = meta->level_cnt[parent_level - 1];
    // pass mask (NF bits per parent pair, PPT pairs: bits of one packed
    // word), survivor count and output offset of emit tile T
    auto tile_head = [&](uint64_t T, uint32_t &mask, uint32_t &cnt, uint64_t &off) {
        constexpr uint32_t BITS = PPT * NF;
        const uint64_t p0 = T * TILE + (uint64_t)threadIdx.x * PPT;
        mask = 0;
        if (p0 < nin) {
            const uint64_t bit = p0 * NF;
            const uint32_t w = S.mask[bit / 32];
            mask = BITS == 32 ? w : (w >> (uint32_t)(bit % 32)) & ((1u << (BITS % 32)) - 1u);
        }
        cnt = 0;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r)
            if (T * R + r < ctiles) cnt += S.cnt[T * R + r];
        off = S.off[T * R];
    };
    // Software pipeline over the block's tiles: the pass mask, survivor
    // count and output offset of the next tile are loaded while the current
    // tile is compacted, and a tile's parent pairs are requested before its
    // scan, so no tile waits for two dependent round trips to memory.
    uint32_t mask_n = 0, cnt_n = 0;
    uint64_t off_n = 0;
    if (blockIdx.x < ntiles) tile_head(blockIdx.x, mask_n, cnt_n, off_n);
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t mask = mask_n, cnt = cnt_n;
        const uint64_t base = off_n;
        const uint64_t q0 = tile * TILE + (uint64_t)threadIdx.x * PPT;
        uint32_t tri[PPT], par[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const bool live = ((mask >> (k * NF)) & ((1u << NF) - 1u)) != 0u && q0 + k < nin;
            tri[k] = 0u;
            par[k] = 0u;
            if (live) pair_get<PACKED>(in, q0 + k, tri[k], par[k]);
        }
        // first child of each parent: p * F, or (batched form) the build's
        // record, requested here so that its latency overlaps the scan
        uint32_t first[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            first[k] = par[k] * F;
            if constexpr (BATCH) {
                const bool live = ((mask >> (k * NF)) & ((1u << NF) - 1u)) != 0u && par[k] < np;
                first[k] = live ? bd.node_first[offp + par[k]] : 0u;
            }
        }
        const uint64_t nt = tile + gridDim.x;
        if (nt < ntiles) tile_head(nt, mask_n, cnt_n, off_n);
        if (cnt == 0) continue;                  // uniform over the block
        uint32_t total;
        const uint32_t ex = block_excl_scan<uint32_t, LEVEL_THREADS / WAVE>((uint32_t)__popc(mask), s_scan, total);
        if (mask) {
            uint32_t at = ex;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (((mask >> (k * NF)) & ((1u << NF) - 1u)) == 0u) continue;
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    if (!((mask >> (k * NF + j)) & 1u)) continue;
                    if (at < TILE_OUT) {
                        s_tri[at] = tri[k];
                        s_node[at] = first[k] + (uint32_t)j;
                    }
                    ++at;
                }
            }
        }
        __syncthreads();
        const uint32_t n_out = min(total, TILE_OUT);
        for (uint32_t i = threadIdx.x; i < n_out; i += LEVEL_THREADS) {
            const uint64_t at = base + i;
            if (at < out.cap) pair_put<PACKED>(out, at, s_tri[i], s_node[i]);
        }
        __syncthreads();                         // LDS is reused by the next tile
    }
}

// ------------------------------------------------------------------ scan
// Exclusive scan of the item counts into 64-bit offsets; the total becomes
// the pair count of the output level.  Tiles take their index from an atomic
// counter in launch order, so every tile waited on in the look-back has
// started and publishes its sum without waiting: the look-back always ends.
// There are few tiles (SCAN_TILE items each).
// A batch's top-level pass (batch_top = its level, 1-based) scans bd_top[0]
// items and appends after the bd_top[1] pairs already on that level.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_items(int32_t parent_level, uint32_t n_mesh, pair_levels P,
                                                             trav_scratch S, crsh_meta *meta, uint32_t batch_top,
                                                             const uint64_t *bd_top)
{
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    __shared__ uint64_t s_scan[SCAN_THREADS / WAVE];
    const uint32_t nl = meta->n_levels;
    if (nl == 0) return;
    if (batch_top > nl) return;
    const uint64_t n = batch_top ? bd_top[0] : level_items(meta, parent_level, n_mesh, P);
    const uint64_t base = batch_top ? bd_top[1] : 0u;
    const uint32_t out_level = batch_top ? batch_top - 1 : (parent_level == 0 ? nl - 1 : (uint32_t)parent_level - 2);
    const uint64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (blockIdx.x >= ntiles) return;       // only ntiles blocks take a tile
    if (threadIdx.x == 0) s_tile = atomicAdd(S.scan_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) return;
    const uint64_t first = (uint64_t)tile * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t v[SCAN_ITEMS];
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = first + k < n ? S.cnt[first + k] : 0u;
        sum += v[k];
    }
    uint64_t total;
    const uint64_t ex = block_excl_scan<uint64_t, SCAN_THREADS / WAVE>(sum, s_scan, total);
    if (threadIdx.x < WAVE) {
        const uint64_t e = lookback_wave(S.scan_flags, tile, total);
        if (threadIdx.x == 0) s_excl = e;
    }
    __syncthreads();
    uint64_t run = s_excl + ex;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
        if (first + k < n) S.off[first + k] = base + run;
        run += v[k];
    }
    if (tile == ntiles - 1 && threadIdx.x == SCAN_THREADS - 1) {
        meta->pairs[out_level] = base + run;
        atomicAdd((unsigned long long *)&meta->hits[out_level], (unsigned long long)run);
        if (base + run > P.p[out_level].cap) atomicOr(&meta->status, CRSH_OVERFLOW_PAIRS);
    }
}

// Batch, before the top-level pass of level L: item ranges of the frames
// whose top is L (one thread per frame), their total, and the pairs already
// on that level (the append base).  Too many items: flagged, pass skipped.
__global__ __launch_bounds__(256) void k_batch_top_plan(batch_dev bd, crsh_meta *meta, uint32_t L)
{
    __shared__ uint64_t scratch[256 / WAVE];
    const uint32_t f = threadIdx.x;
    const bool live = f < bd.n_frames;
    uint64_t items = 0;
    if (live && bd.fm[f].n_levels == L && L >= 1)
        items = (uint64_t)bd.fm[f].level_cnt[L - 1] * bd.frames[f].mesh_count;
    uint64_t total;
    const uint64_t ex = block_excl_scan<uint64_t, 256 / WAVE>(items, scratch, total);
    if (live) bd.fm[f].item_base = ex;
    if (f == 0) {
        if (total > bd.top_cap) {
            atomicOr(&meta->status, CRSH_OVERFLOW_ITEMS);
            total = 0;
        }
        bd.top[0] = total;
        bd.top[1] = L >= 1 ? meta->pairs[L - 1] : 0u;
    }
}

__global__ void k_no_storage(crsh_meta *meta, uint32_t levels_given)
{
    if (meta->n_levels > levels_given) atomicOr(&meta->status, CRSH_OVERFLOW_PAIRS);
}

}  // namespace crsh

using namespace crsh;

namespace crsh {

void node_pack_launch(const crsh_nodes *nodes, crsh_meta *meta, float4 *na, float4 *nb, float *ns, bool clear_pairs,
                      hipStream_t stream)
{
    node_arrays nd{nodes->cx, nodes->cy, nodes->cz, nodes->r, nodes->ax, nodes->ay, nodes->az,
                   nodes->c, nodes->tan, nodes->sec};
    uint32_t g = std::min<uint32_t>((nodes->capacity + 255) / 256, 2048);
    if (g == 0) g = 1;
    k_node_pack<<<g, 256, 0, stream>>>(nd, meta, na, nb, ns, clear_pairs);
}

// Blocks of a persistent grid-stride kernel that fit the device at once.  Its
// blocks get equal shares of the tiles, so they finish in rounds of this many;
// a grid of whole rounds leaves no round partly empty.  0 if unknown.
template <typename K>
static uint32_t resident_blocks(K kernel, uint32_t threads)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)threads, 0) != hipSuccess || cus < 1 ||
        per_cu < 1)
        return 0;
    return (uint32_t)cus * (uint32_t)per_cu;
}

void level_count_launch(int32_t parent_level, int32_t merge, const float4 *na, const float4 *nb, const float *ns,
                        const float4 *tsph, uint32_t m, const pair_levels &P, const trav_scratch &S, crsh_meta *meta,
                        const batch_dev *bd, uint64_t tiles_cap, uint32_t top_levels, hipStream_t stream, bool packed)
{
    const batch_dev b = bd ? *bd : batch_dev{};
    const uint32_t Fu = (uint32_t)merge;
    const int L = parent_level;
    int nf = 2;
    while (nf < merge) nf *= 2;
    // descendants of a top-level node on the child level, for a hierarchy
    // of at most top_levels levels: the staged kernel if they fit the window
    uint64_t run = 1;
    for (int e = 0; e < (int)top_levels - L + 1 && run <= COUNT_WINDOW; ++e) run *= Fu;
    const bool st = run <= COUNT_WINDOW;
    prof_scope ps("k_level", stream);
    // a persistent grid of one round of resident blocks (at most one block
    // per step of COUNT_TPS tiles)
#define CRSH_COUNT_ONE(NF, BT, PK, ST)                                                                       \
    {                                                                                                        \
        const uint32_t rb = resident_blocks(k_level_count_lanes<NF, BT, PK, ST>, COUNT_THREADS);             \
        const uint64_t want = std::max<uint64_t>((tiles_cap + COUNT_TPS - 1) / COUNT_TPS, 1);                \
        const uint32_t gl = (uint32_t)std::min<uint64_t>(want, rb ? rb : 2048);                              \
        k_level_count_lanes<NF, BT, PK, ST><<<gl, COUNT_THREADS, 0, stream>>>(L, Fu, na, nb, ns, tsph, m, P, S, \
                                                                            meta, b);                       \
    }
#define CRSH_COUNT_ST(NF, BT, PK)                                                                            \
    if (st)                                                                                                  \
        CRSH_COUNT_ONE(NF, BT, PK, true)                                                                     \
    else                                                                                                     \
        CRSH_COUNT_ONE(NF, BT, PK, false)
#define CRSH_COUNT_NF(BT, PK)                                                                                \
    switch (nf) {                                                                                            \
    case 2: CRSH_COUNT_ST(2, BT, PK) break;                                                                  \
    case 4: CRSH_COUNT_ST(4, BT, PK) break;                                                                  \
    case 8: CRSH_COUNT_ST(8, BT, PK) break;                                                                  \
    default: CRSH_COUNT_ST(16, BT, PK) break;                                                                \
    }
    if (bd) {
        CRSH_COUNT_NF(true, false)
    } else if (packed) {
        CRSH_COUNT_NF(false, true)
    } else {
        CRSH_COUNT_NF(false, false)
    }
#undef CRSH_COUNT_NF
#undef CRSH_COUNT_ST
#undef CRSH_COUNT_ONE
}

void tri_spheres_launch(const crsh_scene *scene, uint32_t b, uint32_t e, float4 *out, hipStream_t stream)
{
    const float *const *v = scene->v;
    if (e > b) {
        uint32_t g = std::min<uint32_t>((e - b + 255) / 256, 2048);
        k_tri_sph<<<g, 256, 0, stream>>>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], b, e, out);
    }
}

// lowest: the lowest level produced (1, or 2 when crsh_leaf_hit forms the
// level-1 pairs itself); a top-level pass always writes its own level.
// P: the pair storage of `levels` consecutive levels (largest capacity
// max_pairs), unpacked or packed.
static crsh_status traverse_run(const crsh_nodes *nodes, const crsh_scene *scene, uint32_t tri_begin,
                                uint32_t tri_end, int32_t bundle, int32_t merge, const pair_levels &P, int levels,
                                uint64_t max_pairs, crsh_meta *meta, void *ws, size_t ws_bytes, const batch_dev *bd,
                                int32_t batch_levels, uint64_t batch_top_items, int32_t lowest, hipStream_t stream)
{
    if (!nodes || !scene || !meta || !ws) {
        set_error("crsh_traverse: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (bundle < 1 || bundle > CRSH_MAX_BUNDLE || merge < 2 || merge > CRSH_MAX_MERGE) {
        set_error("crsh_traverse: bad bundle or merge factor");
        return CRSH_ERR_INVALID;
    }
    for (int k = 0; k < 9; ++k)
        if (!scene->v[k] && scene->m) {
            set_error("crsh_traverse: missing vertex array");
            return CRSH_ERR_INVALID;
        }
    if (scene->n_mesh == 0 || !scene->mesh_first || !scene->mesh_count || !scene->msph) {
        set_error("crsh_traverse: scene has no meshes");
        return CRSH_ERR_INVALID;
    }
    if (tri_end > scene->m || tri_begin > tri_end) {
        set_error("crsh_traverse: triangle batch [%u, %u) outside [0, %u)", tri_begin, tri_end, scene->m);
        return CRSH_ERR_INVALID;
    }
    if (lowest < 1 || lowest > 2) {
        set_error("crsh_traverse: lowest level must be 1 or 2");
        return CRSH_ERR_INVALID;
    }
    if (levels == 0) {
        set_error("crsh_traverse: no pair storage");
        return CRSH_ERR_INVALID;
    }
    if (bd && levels < batch_levels) {
        set_error("crsh_batch: pair storage for %d levels, %d needed", levels, batch_levels);
        return CRSH_ERR_INVALID;
    }
    const bool packed = P.p[0].packed != 0;
    if (packed && bd) {
        set_error("crsh_batch: packed pairs are not supported in the batched form");
        return CRSH_ERR_INVALID;
    }
    const uint64_t top_items = bd ? batch_top_items : (uint64_t)nodes->capacity * scene->n_mesh;
    size_t need = trav_ws_bytes(scene->m, nodes->capacity, top_items, max_pairs);
    if (ws_bytes < need) {
        set_error("crsh_traverse: workspace too small (%zu < %zu)", ws_bytes, need);
        return CRSH_ERR_INVALID;
    }
    const uint64_t level_tiles = (max_pairs + LEVEL_TILE - 1) / LEVEL_TILE;
    const uint64_t items = std::max(top_items, level_tiles) + 1;
    char *w = (char *)ws;
    float4 *tsph = (float4 *)w;
    w += align256((size_t)scene->m * 16);
    float4 *na = (float4 *)w;
    w += align256((size_t)nodes->capacity * 16);
    float4 *nb = (float4 *)w;
    w += align256((size_t)nodes->capacity * 16);
    float *ns = (float *)w;
    w += align256((size_t)nodes->capacity * 4);
    trav_scratch S;
    S.cnt = (uint32_t *)w;
    w += align256(items * 4);
    S.off = (uint64_t *)w;
    w += align256(items * 8);
    S.mask = (uint32_t *)w;
    w += align256(level_tiles * LEVEL_THREADS * 4 + 4);
    S.scan_flags = (uint64_t *)w;
    w += align256((items / SCAN_TILE + 2) * 8);
    S.scan_ctr = (uint32_t *)w;

    int nf = 2;
    while (nf < merge) nf *= 2;
    const batch_dev b = bd ? *bd : batch_dev{};
    tri_spheres_launch(scene, tri_begin, tri_end, tsph, stream);
    node_pack_launch(nodes, meta, na, nb, ns, true, stream);
    k_no_storage<<<1, 1, 0, stream>>>(meta, (uint32_t)levels);
    const uint32_t scan_grid = (uint32_t)std::min<uint64_t>((items + SCAN_TILE - 1) / SCAN_TILE, 1u << 20);
    const uint32_t top_grid = (uint32_t)std::max<uint64_t>(std::min<uint64_t>((top_items + 3) / 4, 2048), 1);
    const uint32_t Fu = (uint32_t)merge;

    // top-level pass: plain (L = 0, the one top level) or a batch level L
    auto top_pass_launch = [&](uint32_t L) {
        if (bd) {
            k_batch_top_plan<<<1, 256, 0, stream>>>(b, meta, L);
            {
                prof_scope ps("k_top_count", stream);
                k_top_count<true><<<top_grid, 256, 0, stream>>>(na, nb, ns, tsph, scene->mesh_first,
                                                                scene->mesh_count, scene->msph, scene->n_mesh,
                                                                tri_begin, tri_end, P, S, meta, b, L);
            }
            k_scan_items<<<scan_grid, SCAN_THREADS, 0, stream>>>(0, scene->n_mesh, P, S, meta, L, b.top);
            {
                prof_scope ps("k_top_emit", stream);
                k_top_emit<true><<<top_grid, 256, 0, stream>>>(na, nb, ns, tsph, scene->mesh_first,
                                                               scene->mesh_count, scene->msph, scene->n_mesh,
                                                               tri_begin, tri_end, P, S, meta, b, L);
            }
        } else {
            {
                prof_scope ps("k_top_count", stream);
                k_top_count<false><<<top_grid, 256, 0, stream>>>(na, nb, ns, tsph, scene->mesh_first,
                                                                 scene->mesh_count, scene->msph, scene->n_mesh,
                                                                 tri_begin, tri_end, P, S, meta, b, 0);
            }
            k_scan_items<<<scan_grid, SCAN_THREADS, 0, stream>>>(0, scene->n_mesh, P, S, meta, 0, nullptr);
            {
                prof_scope ps("k_top_emit", stream);
                if (packed)
                    k_top_emit<false, true><<<top_grid, 256, 0, stream>>>(na, nb, ns, tsph, scene->mesh_first,
                                                                          scene->mesh_count, scene->msph,
                                                                          scene->n_mesh, tri_begin, tri_end, P, S,
                                                                          meta, b, 0);
                else
                    k_top_emit<false><<<top_grid, 256, 0, stream>>>(na, nb, ns, tsph, scene->mesh_first,
                                                                    scene->mesh_count, scene->msph, scene->n_mesh,
                                                                    tri_begin, tri_end, P, S, meta, b, 0);
            }
        }
    };
    // one level pass: pairs of level L (1-based parent) -> level L - 1
    auto level_pass_launch = [&](int L) {
        const uint64_t tiles = (P.p[L - 1].cap + LEVEL_TILE - 1) / LEVEL_TILE;
        uint32_t g = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(tiles, 1), 4096);
#define CRSH_EMIT(NF, BT, PK)                                                                              \
    k_level_emit<NF, emit_ppt(NF), BT, PK><<<g, LEVEL_THREADS, 0, stream>>>(L, Fu, P, S, meta, b)
#define CRSH_EMIT_NF(BT, PK)                                                                               \
    switch (nf) {                                                                                          \
    case 2: CRSH_EMIT(2, BT, PK); break;                                                                   \
    case 4: CRSH_EMIT(4, BT, PK); break;                                                                   \
    case 8: CRSH_EMIT(8, BT, PK); break;                                                                   \
    default: CRSH_EMIT(16, BT, PK); break;                                                                 \
    }
        level_count_launch(L, merge, na, nb, ns, tsph, scene->m, P, S, meta, bd, tiles,
                           (uint32_t)(bd ? batch_levels : levels), stream, packed);
        k_scan_items<<<scan_grid, SCAN_THREADS, 0, stream>>>(L, scene->n_mesh, P, S, meta, 0, nullptr);
        {
            prof_scope ps("k_level_emit", stream);
            if (bd) {
                CRSH_EMIT_NF(true, false)
            } else if (packed) {
                CRSH_EMIT_NF(false, true)
            } else {
                CRSH_EMIT_NF(false, false)
            }
        }
#undef CRSH_EMIT_NF
#undef CRSH_EMIT
    };
    if (bd) {
        for (int L = batch_levels; L >= 1; --L) {
            if (L < batch_levels && L >= lowest) level_pass_launch(L + 1);
            top_pass_launch((uint32_t)L);
        }
    } else {
        top_pass_launch(0);
        for (int L = levels; L >= lowest + 1; --L) level_pass_launch(L);
    }
    return hip_check(hipGetLastError(), "crsh_traverse launch");
}

crsh_status traverse_launch(const crsh_nodes *nodes, const crsh_scene *scene, uint32_t tri_begin, uint32_t tri_end,
                            int32_t bundle, int32_t merge, const crsh_pairs pairs[CRSH_MAX_LEVELS],
                            crsh_meta *meta, void *ws, size_t ws_bytes, const batch_dev *bd, int32_t batch_levels,
                            uint64_t batch_top_items, int32_t lowest, hipStream_t stream)
{
    if (!pairs) {
        set_error("crsh_traverse: NULL argument");
        return CRSH_ERR_INVALID;
    }
    // levels present in the pair table: consecutive entries with storage
    pair_levels P{};
    int levels = 0;
    uint64_t max_pairs = 0;
    while (levels < CRSH_MAX_LEVELS && pairs[levels].tri && pairs[levels].node) {
        P.p[levels].tri = pairs[levels].tri;
        P.p[levels].node = pairs[levels].node;
        P.p[levels].cap = pairs[levels].capacity;
        max_pairs = std::max(max_pairs, pairs[levels].capacity);
        ++levels;
    }
    return traverse_run(nodes, scene, tri_begin, tri_end, bundle, merge, P, levels, max_pairs, meta, ws, ws_bytes,
                        bd, batch_levels, batch_top_items, lowest, stream);
}

// packed pairs need every level's node ids below 2^(32 - CRSH_PACKED_TRI_BITS)
__global__ void k_packed_check(crsh_meta *meta)
{
    const uint32_t nl = min(meta->n_levels, (uint32_t)CRSH_MAX_LEVELS);
    for (uint32_t k = 0; k < nl; ++k)
        if (meta->level_cnt[k] > CRSH_PACKED_MAX_NODES) atomicOr(&meta->status, CRSH_OVERFLOW_PACKED);
}

}  // namespace crsh

extern "C" crsh_status crsh_traverse_packed(const crsh_nodes *nodes, const crsh_scene *scene, uint32_t tri_begin,
                                            uint32_t tri_end, int32_t bundle, int32_t merge,
                                            const crsh_packed_pairs pairs[CRSH_MAX_LEVELS], crsh_meta *meta,
                                            void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!pairs || !meta) {
        set_error("crsh_traverse_packed: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (tri_begin > tri_end || tri_end - tri_begin > CRSH_PACKED_MAX_TRIS) {
        set_error("crsh_traverse_packed: a triangle batch holds at most %u triangles (got [%u, %u))",
                  CRSH_PACKED_MAX_TRIS, tri_begin, tri_end);
        return CRSH_ERR_INVALID;
    }
    pair_levels P{};
    int levels = 0;
    uint64_t max_pairs = 0;
    while (levels < CRSH_MAX_LEVELS && pairs[levels].pair) {
        P.p[levels].tri = pairs[levels].pair;
        P.p[levels].node = nullptr;
        P.p[levels].cap = pairs[levels].capacity;
        P.p[levels].packed = 1;
        P.p[levels].tri_base = tri_begin;
        max_pairs = std::max(max_pairs, pairs[levels].capacity);
        ++levels;
    }
    crsh_status st = traverse_run(nodes, scene, tri_begin, tri_end, bundle, merge, P, levels, max_pairs, meta, ws,
                                  ws_bytes, nullptr, 0, 0, 1, stream);
    if (st != CRSH_OK) return st;
    k_packed_check<<<1, 1, 0, stream>>>(meta);
    return hip_check(hipGetLastError(), "crsh_traverse_packed launch");
}

extern "C" crsh_status crsh_traverse(const crsh_nodes *nodes, const crsh_scene *scene, uint32_t tri_begin,
                                     uint32_t tri_end, int32_t bundle, int32_t merge,
                                     const crsh_pairs pairs[CRSH_MAX_LEVELS], crsh_meta *meta, void *ws,
                                     size_t ws_bytes, hipStream_t stream)
{
    return traverse_launch(nodes, scene, tri_begin, tri_end, bundle, merge, pairs, meta, ws, ws_bytes, nullptr, 0,
                           0, 1, stream);
}

extern "C" crsh_status crsh_traverse_upper(const crsh_nodes *nodes, const crsh_scene *scene, uint32_t tri_begin,
                                           uint32_t tri_end, int32_t bundle, int32_t merge,
                                           const crsh_pairs pairs[CRSH_MAX_LEVELS], crsh_meta *meta, void *ws,
                                           size_t ws_bytes, hipStream_t stream)
{
    return traverse_launch(nodes, scene, tri_begin, tri_end, bundle, merge, pairs, meta, ws, ws_bytes, nullptr, 0,
                           0, 2, stream);
}
