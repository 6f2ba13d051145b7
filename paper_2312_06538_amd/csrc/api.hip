// Host-side plumbing of the CRSH library: error text, workspace sizing and
// the device bookkeeping block (crsh_meta).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "common.hpp"

namespace crsh {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

crsh_status hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return CRSH_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return CRSH_ERR_HIP;
}

struct prof_state {
    char name[64];
    int32_t remaining;
    hipEvent_t start, stop;
    bool armed;
};
static thread_local prof_state g_prof = {"", 0, nullptr, nullptr, false};

bool prof_begin(const char *kernel, hipStream_t s)
{
    if (!g_prof.armed || strcmp(kernel, g_prof.name) != 0) return false;
    if (g_prof.remaining-- > 0) return false;
    (void)hipEventRecord(g_prof.start, s);
    return true;
}

void prof_end(bool armed, hipStream_t s)
{
    if (!armed) return;
    (void)hipEventRecord(g_prof.stop, s);
    g_prof.armed = false;
}

uint32_t resident_grid(const void *f, int threads, uint64_t want)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, threads, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    uint64_t g = (uint64_t)per_cu * (uint64_t)cus;
    if (want < g) g = want;
    return g ? (uint32_t)g : 1u;
}

size_t sort_ws_bytes(uint32_t cap)
{
    size_t tiles = (cap + SORT_TILE - 1) / SORT_TILE;
    return align256((size_t)cap * 4) * 2                   // alternate keys, ids
           + align256((SORT_PASSES + 1) * 256 * 4)         // digit histograms (+ frame digit)
           + align256(64 * 4)                              // pass plan + tile counters
           + align256((SORT_PASSES + 1) * tiles * 256 * 4);   // look-back words
}

size_t hash_ws_bytes(uint64_t pixels)
{
    return align256(((pixels + HASH_BLOCK - 1) / HASH_BLOCK + 1) * 4);
}

size_t trav_ws_bytes(uint32_t m, uint32_t node_cap, uint64_t top_items, uint64_t max_pairs)
{
    uint64_t level_tiles = (max_pairs + LEVEL_TILE - 1) / LEVEL_TILE;
    uint64_t items = std::max<uint64_t>(top_items, level_tiles) + 1;
    return align256((size_t)m * 16)                            // triangle spheres
           + align256((size_t)node_cap * 16) * 2               // packed nodes
           + align256((size_t)node_cap * 4)
           + align256(items * 4) + align256(items * 8)         // counts, offsets
           + align256(level_tiles * LEVEL_THREADS * 4 + 4)     // pass masks
           + align256((items / SCAN_TILE_ITEMS + 2) * 8)       // scan look-back words
           + align256(4);                                      // scan tile counter
}

size_t hit_ws_bytes(uint32_t m, uint32_t slots) { return align256((size_t)m * 48) + hit_slots_bytes(slots); }

__global__ void k_meta_clear(uint32_t *p, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace crsh

using namespace crsh;

extern "C" const char *crsh_last_error(void) { return g_err; }

extern "C" size_t crsh_workspace_size(uint32_t max_rays, uint32_t max_tris, uint32_t max_meshes,
                                      uint32_t max_nodes, uint64_t max_pairs)
{
    size_t a = std::max(sort_ws_bytes(max_rays), sort_chunked_ws_bytes(max_rays));
    size_t b = hash_ws_bytes(max_rays);
    size_t c = trav_ws_bytes(max_tris, max_nodes, (uint64_t)max_nodes * max_meshes, max_pairs);
    size_t d = std::max(hit_ws_bytes(max_tris, max_rays),
                        leaf_hit_ws_bytes(max_tris, max_nodes, max_pairs, max_rays));
    return std::max(std::max(a, b), std::max(c, d));
}

extern "C" crsh_status crsh_meta_reset(crsh_meta *meta, hipStream_t stream)
{
    if (!meta) {
        set_error("crsh_meta_reset: meta is NULL");
        return CRSH_ERR_INVALID;
    }
    const uint32_t n = sizeof(crsh_meta) / 4;
    k_meta_clear<<<(n + 255) / 256, 256, 0, stream>>>((uint32_t *)meta, n);
    return hip_check(hipGetLastError(), "crsh_meta_reset");
}

extern "C" crsh_status crsh_read_meta(const crsh_meta *meta, crsh_meta *host_out, hipStream_t stream)
{
    if (!meta || !host_out) {
        set_error("crsh_read_meta: NULL argument");
        return CRSH_ERR_INVALID;
    }
    crsh_status st = hip_check(hipMemcpyAsync(host_out, meta, sizeof(crsh_meta), hipMemcpyDeviceToHost, stream),
                               "crsh_read_meta copy");
    if (st != CRSH_OK) return st;
    st = hip_check(hipStreamSynchronize(stream), "crsh_read_meta sync");
    if (st != CRSH_OK) return st;
    if (host_out->status) {
        set_error("capacity exceeded (status 0x%x): rays needed %llu, nodes needed %llu", host_out->status,
                  (unsigned long long)host_out->rays_required, (unsigned long long)host_out->nodes_required);
        return CRSH_ERR_CAPACITY;
    }
    return CRSH_OK;
}

extern "C" crsh_status crsh_profile_next(const char *kernel, int32_t occurrence, hipEvent_t start, hipEvent_t stop)
{
    if (!kernel || !start || !stop || occurrence < 0 || strlen(kernel) >= sizeof(g_prof.name)) {
        set_error("crsh_profile_next: bad argument");
        return CRSH_ERR_INVALID;
    }
    strcpy(g_prof.name, kernel);
    g_prof.remaining = occurrence;
    g_prof.start = start;
    g_prof.stop = stop;
    g_prof.armed = true;
    return CRSH_OK;
}
