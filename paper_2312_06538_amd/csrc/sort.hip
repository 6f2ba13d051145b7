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
//   k_sort_pass   one launch per digit: 8192-key tiles ranked in LDS with
//                 wave ballots (stable), a decoupled look-back across tiles
//                 per digit, then a coalesced scatter staged through LDS.
#include "common.hpp"

namespace crsh {

constexpr uint32_t SORT_THREADS = 256;
#ifndef CRSH_SORT_PASS_THREADS
#define CRSH_SORT_PASS_THREADS 512
#endif
#ifndef CRSH_SORT_PASS_ITEMS
#define CRSH_SORT_PASS_ITEMS 16
#endif
constexpr uint32_t PASS_THREADS = CRSH_SORT_PASS_THREADS;  // threads of a pass tile
constexpr uint32_t PASS_ITEMS = CRSH_SORT_PASS_ITEMS;      // keys per thread
constexpr uint32_t PASS_TILE = PASS_THREADS * PASS_ITEMS;  // keys per pass tile (8192)
#ifndef CRSH_SORT_HIST_BLOCKS
#define CRSH_SORT_HIST_BLOCKS 1024
#endif
constexpr uint32_t SORT_HIST_BLOCKS = CRSH_SORT_HIST_BLOCKS;  // most blocks of the histogram kernel

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

// The digit histograms of every pass in one read of the keys.  Blocks walk
// tiles of SORT_TILE keys (grid-stride), counting in LDS, and add their
// counts to the global histograms once at the end: one global atomic per
// bin per block, not per tile (every block's atomics go to the same few
// cache lines).  A tile's keys are all loaded before any is counted.
__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const uint32_t *keys, const uint32_t *vals,
                                                            const uint32_t *frame_of, const crsh_meta *meta,
                                                            uint32_t *hist, uint32_t cap)
{
    constexpr uint32_t PER = SORT_TILE / SORT_THREADS;
    __shared__ uint32_t h[MAX_PASSES * 256];
    const uint32_t n = min(meta->n_rays, cap);
    const uint32_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    if (blockIdx.x >= ntiles) return;
    for (uint32_t i = threadIdx.x; i < MAX_PASSES * 256; i += SORT_THREADS) h[i] = 0;
    __syncthreads();
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t base = tile * SORT_TILE;
        uint32_t k[PER], f[PER];
#pragma unroll
        for (uint32_t r = 0; r < PER; ++r) {
            const uint32_t g = base + r * SORT_THREADS + threadIdx.x;
            k[r] = g < n ? keys[g] : 0u;
            f[r] = (frame_of && g < n) ? vals[g] : 0u;
        }
        if (frame_of) {
#pragma unroll
            for (uint32_t r = 0; r < PER; ++r)
                f[r] = base + r * SORT_THREADS + threadIdx.x < n ? frame_of[f[r]] : 0u;
        }
#pragma unroll
        for (uint32_t r = 0; r < PER; ++r) {
            if (base + r * SORT_THREADS + threadIdx.x >= n) continue;
#pragma unroll
            for (uint32_t p = 0; p < SORT_PASSES; ++p) atomicAdd(&h[p * 256 + ((k[r] >> (8 * p)) & 255u)], 1u);
            if (frame_of) atomicAdd(&h[SORT_PASSES * 256 + (f[r] & 255u)], 1u);
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

// Digit of element r of a thread for this pass: a key byte, or the frame of
// the ray (read through the value) for the frame pass.
template <bool FRAME>
__device__ __forceinline__ uint32_t pass_digit(uint32_t key, uint32_t val, bool ok, uint32_t shift,
                                               const uint32_t *frame_of)
{
    return FRAME ? (ok ? frame_of[val] & 255u : 0u) : (key >> shift) & 255u;
}

// Stable rank of a tile inside each wave: rounds in order, lanes in order.
// Element r of the thread gets its rank among the wave's elements of equal
// digit, with the digit in the high half (slot[r] = d << 16 | rank);
// s_wcnt[w * 256 + d] ends as wave w's count of digit d.  Peers of equal
// digit are found with one ballot per digit bit: a lane keeps the ballot
// where its own bit is set and the complement where it is clear: the lanes
// whose bit is clear, XOR the lane's bit spread over a word, folded into the
// running AND as one three-input bit operation (every lane of the wave is
// active here).  The last peer adds the group's count.
template <bool FRAME, uint32_t ITEMS>
__device__ __forceinline__ void rank_tile(const uint32_t *key, const uint32_t *val, uint32_t base, uint32_t n,
                                          uint32_t shift, const uint32_t *frame_of, uint32_t *s_wcnt,
                                          uint32_t *slot)
{
    // truth table of a & (b ^ c) over the operand patterns 0xF0, 0xCC, 0xAA
    constexpr uint32_t AND_XOR = 0xF0u & (0xCCu ^ 0xAAu);
    const uint32_t w = threadIdx.x / WAVE;
    const uint32_t l = lane_id();
#pragma unroll
    for (uint32_t r = 0; r < ITEMS; ++r) {
        const bool ok = base + r * WAVE + l < n;
        const uint32_t d = pass_digit<FRAME>(key[r], val[r], ok, shift, frame_of);
        const uint64_t live = ballot(ok);
        uint32_t plo = (uint32_t)live, phi = (uint32_t)(live >> 32);
#pragma unroll
        for (uint32_t b = 0; b < 8; ++b) {
            const uint32_t sb = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1u);    // 0 or ~0
            const uint64_t nm = __builtin_amdgcn_uicmp(sb, 0u, 32);    // lanes whose bit b is clear (32: equal)
            plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)nm, sb, AND_XOR);
            phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(nm >> 32), sb, AND_XOR);
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t before = rank_below(peers);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        const uint32_t wbase = ok ? s_wcnt[w * 256 + d] : 0u;
        slot[r] = (d << 16) | (wbase + before);
        if (ok && before + 1u == cnt) s_wcnt[w * 256 + d] = wbase + cnt;
    }
}

// LDS of one pass tile.
template <uint32_t THREADS, uint32_t ITEMS>
struct pass_lds {
    uint32_t buf[THREADS * ITEMS];         // the tile, at its sorted slots
    uint32_t wcnt[THREADS / WAVE * 256];   // per wave and digit: count, then tile-local start
    uint32_t hist[256];
    uint32_t base[256];
    uint32_t scan[256 / WAVE];
    uint32_t tile;
};

// One radix pass over tiles of THREADS * ITEMS keys.  A tile counts its
// digits and publishes the counts for the decoupled look-back first, then
// ranks its keys stably in registers and LDS (while its predecessors publish
// theirs), reads its global digit offsets from the look-back, and writes out
// through one LDS buffer in two phases (the array the digit comes from first,
// then the other), so each phase's stores are runs of consecutive positions
// per digit.  The run length per digit grows with the tile, and with it the
// efficiency of the scattered writes.
template <bool FRAME, uint32_t THREADS, uint32_t ITEMS>
__device__ __forceinline__ void sort_tile(pass_lds<THREADS, ITEMS> &S, const uint32_t *kin, const uint32_t *vin,
                                          uint32_t *kout, uint32_t *vout, const uint32_t *offsets, uint32_t *fl,
                                          uint32_t pass, uint32_t n, uint32_t tile, const uint32_t *frame_of)
{
    constexpr uint32_t TILE = THREADS * ITEMS;
    constexpr uint32_t WAVES = THREADS / WAVE;
    const uint32_t w = threadIdx.x / WAVE;
    const uint32_t l = lane_id();
    const uint32_t shift = 8 * (pass & 3u);
    const uint32_t base = tile * TILE + w * (WAVE * ITEMS);
    const uint32_t d = threadIdx.x;

    uint32_t key[ITEMS], val[ITEMS], slot[ITEMS];
#pragma unroll
    for (uint32_t r = 0; r < ITEMS; ++r) {
        const uint32_t g = base + r * WAVE + l;
        const bool ok = g < n;
        key[r] = ok ? kin[g] : 0xFFFFFFFFu;
        val[r] = ok ? vin[g] : 0u;
    }
    // the tile's digit counts, published before the ranking: the ranking
    // then overlaps the wait for the predecessors' counts
#pragma unroll
    for (uint32_t r = 0; r < ITEMS; ++r)
        if (base + r * WAVE + l < n)
            atomicAdd(&S.hist[pass_digit<FRAME>(key[r], val[r], true, shift, frame_of)], 1u);
    __syncthreads();
    uint32_t run = 0;
    if (d < 256) {
        run = S.hist[d];
        __hip_atomic_store(&fl[(size_t)tile * 256 + d], (tile == 0 ? SLB_INC : SLB_AGG) | run, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    rank_tile<FRAME, ITEMS>(key, val, base, n, shift, frame_of, S.wcnt, slot);
    // tile-local start of each digit (scan of the tile's counts)
    if (d < 256) {
        const uint32_t inc = wave_incl_scan(run);
        if (l == WAVE - 1) S.scan[w] = inc;
    }
    __syncthreads();
    // per digit (threads 0..255): the tile-local start of the digit's slots
    // of each wave, and the look-back for the tile's global digit offset
    if (d < 256) {
        uint32_t before = 0;
#pragma unroll
        for (uint32_t i = 0; i < 256 / WAVE; ++i)
            if (i < w) before += S.scan[i];
        const uint32_t start = before + wave_incl_scan(run) - run;
        uint32_t acc = start;
#pragma unroll
        for (uint32_t ww = 0; ww < WAVES; ++ww) {
            const uint32_t c = S.wcnt[ww * 256 + d];
            S.wcnt[ww * 256 + d] = acc;
            acc += c;
        }
        uint32_t excl = 0;
        if (tile > 0) {
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
        // global position of tile-local sorted slot q of digit d is base[d] + q
        S.base[d] = offsets[pass * 256 + d] + excl - start;
    }
    __syncthreads();
    // phase 1: the array the digit is read from (keys; values for the frame
    // digit) into LDS at its tile-local sorted slot, then out; each slot's
    // global position is kept for phase 2
#pragma unroll
    for (uint32_t r = 0; r < ITEMS; ++r) {
        if (base + r * WAVE + l < n) {
            slot[r] = (slot[r] & 0xFFFFu) + S.wcnt[w * 256 + (slot[r] >> 16)];
            if (slot[r] < TILE) S.buf[slot[r]] = FRAME ? val[r] : key[r];
        }
    }
    __syncthreads();
    uint32_t *out1 = FRAME ? vout : kout;
    uint32_t *out2 = FRAME ? kout : vout;
    const uint32_t tile_n = min(TILE, n - tile * TILE);
    uint32_t pos[ITEMS];
#pragma unroll
    for (uint32_t j = 0; j < ITEMS; ++j) {
        const uint32_t q = threadIdx.x + j * THREADS;
        pos[j] = 0xFFFFFFFFu;
        if (q < tile_n) {
            const uint32_t x = S.buf[q];
            pos[j] = S.base[FRAME ? frame_of[x] & 255u : (x >> shift) & 255u] + q;
            if (pos[j] < n) out1[pos[j]] = x;
        }
    }
    __syncthreads();
    // phase 2: the other array through the same slots
#pragma unroll
    for (uint32_t r = 0; r < ITEMS; ++r)
        if (base + r * WAVE + l < n && slot[r] < TILE) S.buf[slot[r]] = FRAME ? key[r] : val[r];
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < ITEMS; ++j) {
        const uint32_t q = threadIdx.x + j * THREADS;
        if (q < tile_n && pos[j] < n) out2[pos[j]] = S.buf[q];
    }
}

template <bool FRAME, uint32_t THREADS, uint32_t ITEMS>
__global__ __launch_bounds__(THREADS) void k_sort_pass(sort_bufs bufs, const uint32_t *offsets, sort_ctl *ctl,
                                                       uint32_t *flags, uint32_t pass, uint32_t tiles_cap,
                                                       const uint32_t *frame_of)
{
    constexpr uint32_t TILE = THREADS * ITEMS;
    static_assert(THREADS >= 256 && THREADS % 256 == 0, "one thread per digit");
    static_assert(TILE % SORT_TILE == 0, "look-back words are sized for SORT_TILE tiles");
    __shared__ pass_lds<THREADS, ITEMS> S;

    const uint32_t src = ctl->src[pass];
    if (src == BUF_SKIP) return;
    const uint32_t dst = ctl->dst[pass];
    const uint32_t n = ctl->n;
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    if (threadIdx.x == 0) S.tile = atomicAdd(&ctl->tile_ctr[pass], 1u);
    for (uint32_t i = threadIdx.x; i < THREADS / WAVE * 256; i += THREADS) S.wcnt[i] = 0;
    if (threadIdx.x < 256) S.hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t tile = S.tile;
    if (tile >= ntiles) return;
    const uint32_t *kin = pick_src(bufs, src, true);
    const uint32_t *vin = pick_src(bufs, src, false);
    uint32_t *kout = pick_dst(bufs, dst, true);
    uint32_t *vout = pick_dst(bufs, dst, false);
    uint32_t *fl = flags + ((size_t)pass * tiles_cap) * 256;
    sort_tile<FRAME, THREADS, ITEMS>(S, kin, vin, kout, vout, offsets, fl, pass, n, tile, frame_of);
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
        k_sort_hist<<<std::min<uint32_t>(tiles_cap, SORT_HIST_BLOCKS), SORT_THREADS, 0, stream>>>(
            keys_in, ids_in, frame_of, meta, hist, capacity);
    }
    k_sort_plan<<<1, 256, 0, stream>>>(hist, ctl, meta, capacity, passes);
    sort_bufs b{keys_in, ids_in, keys_out, ids_out, kalt, valt};
    const uint32_t pass_tiles = (capacity + PASS_TILE - 1) / PASS_TILE;
    for (uint32_t p = 0; p < passes; ++p) {
        prof_scope ps("k_sort_pass", stream);
        if (p < SORT_PASSES)
            k_sort_pass<false, PASS_THREADS, PASS_ITEMS><<<pass_tiles, PASS_THREADS, 0, stream>>>(
                b, hist, ctl, flags, p, tiles_cap, nullptr);
        else
            k_sort_pass<true, PASS_THREADS, PASS_ITEMS><<<pass_tiles, PASS_THREADS, 0, stream>>>(
                b, hist, ctl, flags, p, tiles_cap, frame_of);
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
