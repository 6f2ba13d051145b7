// Stage 2: ray sorting (Sec. 3.3.3-3.3.5) as a stable LSD radix sort of
// (key, id) by the 32-bit key, 8-bit digits, one pass per digit.
//
// The paper compresses runs of equal keys into chunks, sorts the chunks and
// decompresses; the result is the stable order of the pairs by key, which a
// stable radix sort produces directly.  Layout on the GPU:
//   k_sort_hist   one read of the keys builds the 4 digit histograms;
//   k_sort_plan   scans them into digit offsets and skips passes whose digit
//                 is the same for every key; it also routes the remaining
//                 passes through the output / alternate buffers so that the
//                 last pass writes the output;
//   k_sort_pass   one launch per digit: 4096-key tiles ranked in LDS with
//                 wave ballots (stable), a decoupled look-back across tiles
//                 per digit, then a coalesced scatter staged through LDS.
#include "common.hpp"

namespace crsh {

constexpr uint32_t SORT_THREADS = 256;
constexpr uint32_t SORT_WAVES = SORT_THREADS / WAVE;
constexpr uint32_t SORT_ITEMS = SORT_TILE / SORT_THREADS;   // 16 keys per thread
constexpr uint32_t SORT_ROUNDS = SORT_ITEMS;                 // 64 keys per wave round

// look-back words: flag in bits 31-30 (1 tile count, 2 inclusive prefix)
constexpr uint32_t SLB_AGG = 1u << 30;
constexpr uint32_t SLB_INC = 2u << 30;
constexpr uint32_t SLB_MASK = (1u << 30) - 1;

// The batched form adds a fifth, most significant digit: the frame of the
// ray, read through the value (ray id) from a per-ray frame table.
constexpr uint32_t MAX_PASSES = SORT_PASSES + 1;

// plan codes for the source / destination of each pass
enum : uint32_t { BUF_IN = 0, BUF_OUT = 1, BUF_ALT = 2, BUF_SKIP = 3 };

struct sort_ctl {
    uint32_t src[MAX_PASSES], dst[MAX_PASSES];
    uint32_t tile_ctr[MAX_PASSES];
    uint32_t copy_through;   // every pass skipped: copy input to output
    uint32_t n;
};

__global__ void k_sort_clear(uint32_t *hist, sort_ctl *ctl, uint32_t *flags, const crsh_meta *meta,
                             uint32_t tiles_cap, uint32_t cap)
{
    uint32_t n = min(meta->n_rays, cap);
    uint32_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    uint64_t nflag = (uint64_t)MAX_PASSES * tiles_cap * 256;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nflag;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t tile = (uint32_t)((i / 256) % tiles_cap);
        if (tile < tiles) flags[i] = 0;
    }
    uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < MAX_PASSES * 256) hist[g] = 0;
    if (g < sizeof(sort_ctl) / 4) ((uint32_t *)ctl)[g] = 0;
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const uint32_t *keys, const uint32_t *vals,
                                                            const uint32_t *frame_of, const crsh_meta *meta,
                                                            uint32_t *hist, uint32_t cap)
{
    __shared__ uint32_t h[MAX_PASSES * 256];
    uint32_t n = min(meta->n_rays, cap);
    uint32_t base = blockIdx.x * SORT_TILE;
    if (base >= n) return;
    for (uint32_t i = threadIdx.x; i < MAX_PASSES * 256; i += SORT_THREADS) h[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < SORT_TILE; i += SORT_THREADS) {
        uint32_t g = base + i;
        if (g < n) {
            uint32_t k = keys[g];
#pragma unroll
            for (uint32_t p = 0; p < SORT_PASSES; ++p) atomicAdd(&h[p * 256 + ((k >> (8 * p)) & 255u)], 1u);
            if (frame_of) atomicAdd(&h[SORT_PASSES * 256 + (frame_of[vals[g]] & 255u)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < MAX_PASSES * 256; i += SORT_THREADS)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ __launch_bounds__(256) void k_sort_plan(uint32_t *hist, sort_ctl *ctl, const crsh_meta *meta,
                                                  uint32_t cap, uint32_t passes)
{
    __shared__ uint32_t scratch[256 / WAVE];
    __shared__ uint32_t skip[MAX_PASSES];
    uint32_t n = min(meta->n_rays, cap);
    uint32_t d = threadIdx.x;
    if (d < MAX_PASSES) skip[d] = (n == 0) || d >= passes;
    __syncthreads();
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t c = hist[p * 256 + d];
        if (c == n) skip[p] = 1;    // one digit value holds every key
        uint32_t total;
        uint32_t ex = block_excl_scan<uint32_t, 256 / WAVE>(c, scratch, total);
        hist[p * 256 + d] = ex;
    }
    __syncthreads();
    if (d == 0) {
        // walk the kept passes backwards: the last writes OUT, the one before ALT, ...
        uint32_t target = BUF_OUT;
        int first = -1;
        for (int p = MAX_PASSES - 1; p >= 0; --p) {
            if (skip[p]) {
                ctl->src[p] = BUF_SKIP;
                ctl->dst[p] = BUF_SKIP;
                continue;
            }
            ctl->dst[p] = target;
            target = (target == BUF_OUT) ? BUF_ALT : BUF_OUT;
            first = p;
        }
        for (int p = 0; p < (int)MAX_PASSES; ++p) {
            if (skip[p]) continue;
            ctl->src[p] = (p == first) ? BUF_IN : (ctl->dst[p] == BUF_OUT ? BUF_ALT : BUF_OUT);
        }
        ctl->copy_through = (first < 0) ? 1u : 0u;
        ctl->n = n;
    }
}

struct sort_bufs {
    const uint32_t *kin, *vin;
    uint32_t *kout, *vout, *kalt, *valt;
};

__device__ __forceinline__ const uint32_t *pick_src(const sort_bufs &b, uint32_t code, bool key)
{
    if (code == BUF_IN) return key ? b.kin : b.vin;
    if (code == BUF_OUT) return key ? b.kout : b.vout;
    return key ? b.kalt : b.valt;
}

__device__ __forceinline__ uint32_t *pick_dst(const sort_bufs &b, uint32_t code, bool key)
{
    if (code == BUF_OUT) return key ? b.kout : b.vout;
    return key ? b.kalt : b.valt;
}

template <bool FRAME>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_pass(sort_bufs bufs, const uint32_t *offsets,
                                                            sort_ctl *ctl, uint32_t *flags, uint32_t pass,
                                                            uint32_t tiles_cap, const uint32_t *frame_of)
{
    __shared__ uint32_t s_keys[SORT_TILE];
    __shared__ uint32_t s_vals[SORT_TILE];
    __shared__ uint32_t s_wcnt[SORT_WAVES * 256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_start[256];
    __shared__ uint32_t s_scan[SORT_WAVES];
    __shared__ uint32_t s_tile;

    const uint32_t src = ctl->src[pass];
    if (src == BUF_SKIP) return;
    const uint32_t dst = ctl->dst[pass];
    const uint32_t n = ctl->n;
    const uint32_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    if (threadIdx.x == 0) s_tile = atomicAdd(&ctl->tile_ctr[pass], 1u);
    for (uint32_t i = threadIdx.x; i < SORT_WAVES * 256; i += SORT_THREADS) s_wcnt[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) return;

    const uint32_t *kin = pick_src(bufs, src, true);
    const uint32_t *vin = pick_src(bufs, src, false);
    const uint32_t w = threadIdx.x / WAVE;
    const uint32_t l = lane_id();
    const uint32_t shift = 8 * (pass & 3u);
    const uint32_t base = tile * SORT_TILE + w * (WAVE * SORT_ROUNDS);

    uint32_t key[SORT_ROUNDS], val[SORT_ROUNDS], rank[SORT_ROUNDS];
#pragma unroll
    for (uint32_t r = 0; r < SORT_ROUNDS; ++r) {
        uint32_t g = base + r * WAVE + l;
        bool ok = g < n;
        key[r] = ok ? kin[g] : 0xFFFFFFFFu;
        val[r] = ok ? vin[g] : 0u;
    }
    // stable rank inside the wave: rounds in order, lanes in order
#pragma unroll
    for (uint32_t r = 0; r < SORT_ROUNDS; ++r) {
        uint32_t g = base + r * WAVE + l;
        bool ok = g < n;
        uint32_t d = FRAME ? (ok ? frame_of[val[r]] & 255u : 0u) : (key[r] >> shift) & 255u;
        uint64_t peers = ballot(ok);
#pragma unroll
        for (uint32_t b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t before = rank_below(peers);
        uint32_t cnt = (uint32_t)__popcll(peers);
        uint32_t leader = (uint32_t)__builtin_ctzll(peers | (1ull << 63));
        uint32_t wbase = ok ? s_wcnt[w * 256 + d] : 0u;
        rank[r] = wbase + before;
        if (ok && l == leader) s_wcnt[w * 256 + d] = wbase + cnt;
    }
    __syncthreads();
    // per digit: offsets of the waves, tile count, tile-local digit start
    const uint32_t d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (uint32_t ww = 0; ww < SORT_WAVES; ++ww) {
        uint32_t c = s_wcnt[ww * 256 + d];
        s_wcnt[ww * 256 + d] = run;
        run += c;
    }
    uint32_t total;
    uint32_t start = block_excl_scan<uint32_t, SORT_WAVES>(run, s_scan, total);
    // look-back over the tiles for digit d
    uint32_t *fl = flags + ((size_t)pass * tiles_cap) * 256;
    uint32_t excl = 0;
    if (tile == 0) {
        __hip_atomic_store(&fl[d], SLB_INC | run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(&fl[(size_t)tile * 256 + d], SLB_AGG | run, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        int32_t j = (int32_t)tile - 1;
        while (j >= 0) {
            uint32_t f = __hip_atomic_load(&fl[(size_t)j * 256 + d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t fl2 = f & ~SLB_MASK;
            if (fl2 == 0) {
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += f & SLB_MASK;
            if (fl2 == SLB_INC) break;
            --j;
        }
        __hip_atomic_store(&fl[(size_t)tile * 256 + d], SLB_INC | (excl + run), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // global position of tile-local sorted slot q of digit d is s_base[d] + q
    s_base[d] = offsets[pass * 256 + d] + excl - start;
    s_start[d] = start;
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < SORT_ROUNDS; ++r) {
        uint32_t g = base + r * WAVE + l;
        if (g < n) {
            uint32_t dd = FRAME ? frame_of[val[r]] & 255u : (key[r] >> shift) & 255u;
            uint32_t q = s_start[dd] + s_wcnt[w * 256 + dd] + rank[r];
            if (q < SORT_TILE) {
                s_keys[q] = key[r];
                s_vals[q] = val[r];
            }
        }
    }
    __syncthreads();
    uint32_t *kout = pick_dst(bufs, dst, true);
    uint32_t *vout = pick_dst(bufs, dst, false);
    const uint32_t tile_n = min(SORT_TILE, n - tile * SORT_TILE);
    for (uint32_t q = threadIdx.x; q < tile_n; q += SORT_THREADS) {
        uint32_t k = s_keys[q];
        uint32_t vq = s_vals[q];
        uint32_t pos = s_base[FRAME ? frame_of[vq] & 255u : (k >> shift) & 255u] + q;
        if (pos < n) {
            kout[pos] = k;
            vout[pos] = vq;
        }
    }
}

__global__ void k_sort_copy(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                            const sort_ctl *ctl)
{
    if (!ctl->copy_through) return;
    uint32_t n = ctl->n;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        kout[i] = kin[i];
        vout[i] = vin[i];
    }
}

}  // namespace crsh

using namespace crsh;

namespace crsh {

crsh_status sort_launch(const uint32_t *keys_in, const uint32_t *ids_in, const uint32_t *frame_of,
                        uint32_t *keys_out, uint32_t *ids_out, uint32_t capacity, crsh_meta *meta, void *ws,
                        size_t ws_bytes, hipStream_t stream)
{
    if (!keys_in || !ids_in || !keys_out || !ids_out || !meta || !ws) {
        set_error("crsh_sort: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (capacity >= (1u << 30)) {
        set_error("crsh_sort: capacity must stay below 2^30");
        return CRSH_ERR_INVALID;
    }
    if (ws_bytes < sort_ws_bytes(capacity)) {
        set_error("crsh_sort: workspace too small (%zu < %zu)", ws_bytes, sort_ws_bytes(capacity));
        return CRSH_ERR_INVALID;
    }
    if (keys_in == keys_out || ids_in == ids_out) {
        set_error("crsh_sort: input and output must not alias");
        return CRSH_ERR_INVALID;
    }
    uint32_t tiles_cap = (capacity + SORT_TILE - 1) / SORT_TILE;
    if (tiles_cap == 0) tiles_cap = 1;
    char *w = (char *)ws;
    uint32_t *kalt = (uint32_t *)w;
    w += align256((size_t)capacity * 4);
    uint32_t *valt = (uint32_t *)w;
    w += align256((size_t)capacity * 4);
    uint32_t *hist = (uint32_t *)w;
    w += align256(MAX_PASSES * 256 * 4);
    sort_ctl *ctl = (sort_ctl *)w;
    w += align256(64 * 4);
    uint32_t *flags = (uint32_t *)w;
    const uint32_t passes = frame_of ? MAX_PASSES : SORT_PASSES;

    k_sort_clear<<<1024, 256, 0, stream>>>(hist, ctl, flags, meta, tiles_cap, capacity);
    {
        prof_scope ps("k_sort_hist", stream);
        k_sort_hist<<<tiles_cap, SORT_THREADS, 0, stream>>>(keys_in, ids_in, frame_of, meta, hist, capacity);
    }
    k_sort_plan<<<1, 256, 0, stream>>>(hist, ctl, meta, capacity, passes);
    sort_bufs b{keys_in, ids_in, keys_out, ids_out, kalt, valt};
    for (uint32_t p = 0; p < passes; ++p) {
        prof_scope ps("k_sort_pass", stream);
        if (p < SORT_PASSES)
            k_sort_pass<false><<<tiles_cap, SORT_THREADS, 0, stream>>>(b, hist, ctl, flags, p, tiles_cap, nullptr);
        else
            k_sort_pass<true><<<tiles_cap, SORT_THREADS, 0, stream>>>(b, hist, ctl, flags, p, tiles_cap, frame_of);
    }
    k_sort_copy<<<256, 256, 0, stream>>>(keys_in, ids_in, keys_out, ids_out, ctl);
    return hip_check(hipGetLastError(), "crsh_sort launch");
}

}  // namespace crsh

extern "C" crsh_status crsh_sort(const uint32_t *keys_in, const uint32_t *ids_in, uint32_t *keys_out,
                                 uint32_t *ids_out, uint32_t capacity, crsh_meta *meta, void *ws, size_t ws_bytes,
                                 hipStream_t stream)
{
    return sort_launch(keys_in, ids_in, nullptr, keys_out, ids_out, capacity, meta, ws, ws_bytes, stream);
}
