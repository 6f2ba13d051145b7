// Stage 2 in the paper's own layout (Sec. 3.3.3-3.3.5): compression of the
// (key, id) pairs into chunks of equal consecutive keys, a radix sort of the
// chunks by key, and decompression.
//
//   heads    flag[i] = 1 where key[i] differs from key[i-1] (and at i = 0);
//   scan     exclusive scan of the flags -> chunk index of every head;
//   emit     chunk key, first element and own index for every head;
//   sort     the chunks by key (the stable LSD radix sort of crsh_sort,
//            on its own device count);
//   sizes    sizes of the chunks in sorted order, scanned into offsets;
//   expand   output position p belongs to the last sorted chunk whose offset
//            is <= p; it takes that chunk's element p - offset.
// Chunks keep their input order among equal keys and elements keep theirs
// inside a chunk, so the result is the stable order of crsh_sort.  The
// radix sort then moves one entry per chunk instead of one per ray, which
// pays where runs of equal keys are long (coherent shadow rays).
#include <algorithm>

#include "batch.hpp"

namespace crsh {

constexpr uint32_t CS_THREADS = 256;
constexpr uint32_t CS_TILE = 4096;
constexpr uint32_t CS_PT = CS_TILE / CS_THREADS;

struct cs_ws {
    uint32_t *flag;     // head flags, then chunk index of every head
    uint32_t *ckey;     // chunk keys
    uint32_t *cfirst;   // first element of each chunk
    uint32_t *cval;     // chunk index (the sorted value)
    uint32_t *skey;     // sorted chunk keys
    uint32_t *sval;     // sorted chunk indices
    uint32_t *size;     // sizes of the sorted chunks, then their offsets
    uint32_t *tiles;    // per scan tile sums, then their exclusive bases
    uint32_t *total;    // [0] heads total
    crsh_meta *cmeta;   // device count of the chunk sort (n_rays = chunks)
    void *sort_ws;
    size_t sort_bytes;
};

static size_t cs_bytes(uint32_t cap, cs_ws *L, void *ws)
{
    const size_t tiles = (cap + CS_TILE - 1) / CS_TILE + 1;
    const size_t a = align256((size_t)cap * 4 + 4);
    size_t off = 0;
    char *w = (char *)ws;
    uint32_t **arr[7];
    if (L) {
        arr[0] = &L->flag;
        arr[1] = &L->ckey;
        arr[2] = &L->cfirst;
        arr[3] = &L->cval;
        arr[4] = &L->skey;
        arr[5] = &L->sval;
        arr[6] = &L->size;
    }
    for (int k = 0; k < 7; ++k) {
        if (L) *arr[k] = (uint32_t *)(w + off);
        off += a;
    }
    if (L) L->tiles = (uint32_t *)(w + off);
    off += align256(tiles * 4);
    if (L) L->total = (uint32_t *)(w + off);
    off += align256(16);
    if (L) L->cmeta = (crsh_meta *)(w + off);
    off += align256(sizeof(crsh_meta));
    if (L) {
        L->sort_ws = w + off;
        L->sort_bytes = sort_ws_bytes(cap);
    }
    off += sort_ws_bytes(cap);
    return off;
}

size_t sort_chunked_ws_bytes(uint32_t cap) { return cs_bytes(cap, nullptr, nullptr); }

__device__ __forceinline__ uint32_t count_of(const uint32_t *n_dev, uint32_t cap)
{
    return min(*n_dev, cap);
}

// ---------------------------------------------- exclusive scan of u32 counts
__global__ __launch_bounds__(CS_THREADS) void k_cs_tiles(const uint32_t *in, const uint32_t *n_dev, uint32_t cap,
                                                         uint32_t *tiles)
{
    __shared__ uint32_t s_red[CS_THREADS / WAVE];
    const uint32_t n = count_of(n_dev, cap);
    const uint32_t base = blockIdx.x * CS_TILE;
    if (base >= n) return;
    uint32_t sum = 0;
    for (uint32_t k = 0; k < CS_PT; ++k) {
        const uint32_t i = base + k * CS_THREADS + threadIdx.x;
        sum += i < n ? in[i] : 0u;
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_red[threadIdx.x / WAVE] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < CS_THREADS / WAVE; ++w) t += s_red[w];
        tiles[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_cs_top(uint32_t *tiles, const uint32_t *n_dev, uint32_t cap,
                                                 uint32_t *total)
{
    __shared__ uint32_t s_scan[1024 / WAVE];
    __shared__ uint32_t s_carry;
    const uint32_t n = count_of(n_dev, cap);
    const uint32_t nt = (n + CS_TILE - 1) / CS_TILE;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t b = 0; b < nt; b += 1024) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < nt ? tiles[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<uint32_t, 1024 / WAVE>(v, s_scan, tot);
        const uint32_t carry = s_carry;
        if (i < nt) tiles[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) total[0] = s_carry;
}

// out[i] = exclusive prefix of in[i]; tile-major so that a thread's 16
// elements are consecutive
__global__ __launch_bounds__(CS_THREADS) void k_cs_apply(const uint32_t *in, uint32_t *out, const uint32_t *n_dev,
                                                         uint32_t cap, const uint32_t *tiles)
{
    __shared__ uint32_t s_scan[CS_THREADS / WAVE];
    const uint32_t n = count_of(n_dev, cap);
    const uint32_t base = blockIdx.x * CS_TILE;
    if (base >= n) return;
    const uint32_t first = base + threadIdx.x * CS_PT;
    uint32_t v[CS_PT];
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < CS_PT; ++k) {
        v[k] = first + k < n ? in[first + k] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = tiles[blockIdx.x] + block_excl_scan<uint32_t, CS_THREADS / WAVE>(sum, s_scan, tot);
#pragma unroll
    for (uint32_t k = 0; k < CS_PT; ++k) {
        if (first + k < n) out[first + k] = run;
        run += v[k];
    }
}

static void scan_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint32_t cap, uint32_t *tiles,
                     uint32_t *total, hipStream_t stream)
{
    const uint32_t g = std::max<uint32_t>((cap + CS_TILE - 1) / CS_TILE, 1);
    k_cs_tiles<<<g, CS_THREADS, 0, stream>>>(in, n_dev, cap, tiles);
    k_cs_top<<<1, 1024, 0, stream>>>(tiles, n_dev, cap, total);
    k_cs_apply<<<g, CS_THREADS, 0, stream>>>(in, out, n_dev, cap, tiles);
}

// ------------------------------------------------------------------ stages
__global__ void k_cs_clear(crsh_meta *cmeta)
{
    uint32_t *p = (uint32_t *)cmeta;
    for (uint32_t i = threadIdx.x; i < sizeof(crsh_meta) / 4; i += blockDim.x) p[i] = 0;
}

__global__ void k_cs_heads(const uint32_t *keys, const crsh_meta *meta, uint32_t cap, uint32_t *flag)
{
    const uint32_t n = min(meta->n_rays, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// flag[] holds the chunk index of every element's run start after the scan
// only at heads; a head is recognised again from the keys
__global__ void k_cs_emit(const uint32_t *keys, const crsh_meta *meta, uint32_t cap, cs_ws L)
{
    const uint32_t n = min(meta->n_rays, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (i == 0 || keys[i] != keys[i - 1]) {
            const uint32_t c = L.flag[i];
            if (c < cap) {
                L.ckey[c] = keys[i];
                L.cfirst[c] = i;
                L.cval[c] = c;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) L.cmeta->n_rays = min(L.total[0], cap);
}

__global__ void k_cs_sizes(const crsh_meta *meta, uint32_t cap, cs_ws L)
{
    const uint32_t n = min(meta->n_rays, cap);
    const uint32_t nc = min(L.cmeta->n_rays, cap);
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nc; j += gridDim.x * blockDim.x) {
        const uint32_t c = min(L.sval[j], nc - 1);
        const uint32_t end = c + 1 < nc ? L.cfirst[c + 1] : n;
        L.flag[j] = end - L.cfirst[c];          // reuse: sizes in sorted order
    }
}

__global__ void k_cs_expand(const uint32_t *keys_in, const uint32_t *ids_in, uint32_t *keys_out, uint32_t *ids_out,
                            const crsh_meta *meta, uint32_t cap, cs_ws L)
{
    const uint32_t n = min(meta->n_rays, cap);
    const uint32_t nc = min(L.cmeta->n_rays, cap);
    if (nc == 0) return;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const uint32_t j = last_at_most(nc, p, [&](uint32_t q) { return L.size[q]; });
        const uint32_t c = min(L.sval[j], nc - 1);
        const uint32_t i = min(L.cfirst[c] + (p - L.size[j]), n - 1);
        keys_out[p] = keys_in[i];
        ids_out[p] = ids_in[i];
    }
}

}  // namespace crsh

using namespace crsh;

extern "C" crsh_status crsh_sort_chunked(const uint32_t *keys_in, const uint32_t *ids_in, uint32_t *keys_out,
                                         uint32_t *ids_out, uint32_t capacity, crsh_meta *meta, void *ws,
                                         size_t ws_bytes, hipStream_t stream)
{
    if (!keys_in || !ids_in || !keys_out || !ids_out || !meta || !ws) {
        set_error("crsh_sort_chunked: NULL argument");
        return CRSH_ERR_INVALID;
    }
    if (capacity >= (1u << 30)) {
        set_error("crsh_sort_chunked: capacity must stay below 2^30");
        return CRSH_ERR_INVALID;
    }
    if (keys_in == keys_out || ids_in == ids_out) {
        set_error("crsh_sort_chunked: input and output must not alias");
        return CRSH_ERR_INVALID;
    }
    const size_t need = sort_chunked_ws_bytes(capacity);
    if (ws_bytes < need) {
        set_error("crsh_sort_chunked: workspace too small (%zu < %zu)", ws_bytes, need);
        return CRSH_ERR_INVALID;
    }
    cs_ws L;
    cs_bytes(capacity, &L, ws);
    const uint32_t g = std::max<uint32_t>(std::min<uint32_t>((capacity + 255) / 256, 4096), 1);
    k_cs_clear<<<1, 256, 0, stream>>>(L.cmeta);
    {
        prof_scope ps("k_cs_heads", stream);
        k_cs_heads<<<g, 256, 0, stream>>>(keys_in, meta, capacity, L.flag);
    }
    scan_u32(L.flag, L.flag, &meta->n_rays, capacity, L.tiles, L.total, stream);
    k_cs_emit<<<g, 256, 0, stream>>>(keys_in, meta, capacity, L);
    crsh_status st = sort_launch(L.ckey, L.cval, nullptr, L.skey, L.sval, capacity, L.cmeta, L.sort_ws,
                                 L.sort_bytes, stream);
    if (st != CRSH_OK) return st;
    k_cs_sizes<<<g, 256, 0, stream>>>(meta, capacity, L);
    scan_u32(L.flag, L.size, &L.cmeta->n_rays, capacity, L.tiles, L.total, stream);
    {
        prof_scope ps("k_cs_expand", stream);
        k_cs_expand<<<g, 256, 0, stream>>>(keys_in, ids_in, keys_out, ids_out, meta, capacity, L);
    }
    return hip_check(hipGetLastError(), "crsh_sort_chunked launch");
}
