// Device memory of the library.  Every device buffer of a plan (tables,
// factors, boundary maps, work buffers, Krylov workspaces) comes from here.
// Blocks a plan gives back can be kept in a per-device cache and handed out
// again to later requests of about the same size instead of going back to the
// driver: a driver free of a large block takes milliseconds per gigabyte and
// waits for the whole device, which a serving loop that factors, trims and
// destroys plans on several streams would otherwise pay on every batch.  The
// cache holds at most asp_set_cache_limit bytes (0 by default: every block
// goes straight back to the driver).  Every free in the library follows a
// synchronization of the owning plan's stream, so a cached block has no work
// pending on it and may go to a plan on another stream.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>

#include "asp_internal.h"

namespace {

constexpr int MAX_DEVICES = 64;
constexpr size_t MIB = (size_t)1 << 20;

struct Block {
    int dev;
    size_t bytes;   // rounded size
};

struct DeviceCache {
    std::multimap<size_t, void*> free;   // rounded size -> cached block
    size_t cached = 0;
};

std::mutex g_mu;
DeviceCache g_cache[MAX_DEVICES];
std::unordered_map<void*, Block> g_blocks;   // blocks handed out
size_t g_limit = 0;

// sizes rounded so that requests of one shape map to one size: 512 bytes
// below 1 MiB, 2 MiB above
size_t rounded(size_t bytes) {
    if (bytes < 16) bytes = 16;
    const size_t q = bytes < MIB ? 512 : 2 * MIB;
    return (bytes + q - 1) / q * q;
}

// a cached block for `r` bytes: the smallest of at least r and at most
// r + max(r / 8, 2 MiB); its size goes to *got (the caller holds g_mu)
void* take_cached(DeviceCache& c, size_t r, size_t* got) {
    auto it = c.free.lower_bound(r);
    if (it == c.free.end() || it->first > r + std::max(r / 8, 2 * MIB)) return nullptr;
    void* p = it->second;
    *got = it->first;
    c.cached -= it->first;
    c.free.erase(it);
    return p;
}

// return cached blocks of `dev` to the driver until at most `keep` bytes stay
void trim_device(int dev, size_t keep) {
    DeviceCache& c = g_cache[dev];
    while (c.cached > keep && !c.free.empty()) {   // largest first
        auto it = std::prev(c.free.end());
        (void)hipFree(it->second);
        c.cached -= it->first;
        c.free.erase(it);
    }
}

}  // namespace

hipError_t devmem_alloc(void** p, size_t bytes) {
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    const size_t r = rounded(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    size_t got = r;
    void* q = take_cached(g_cache[dev], r, &got);
    if (!q) {
        e = hipMalloc(&q, r);
        if (e != hipSuccess) {
            // give the cache back to the driver and try once more
            (void)hipGetLastError();
            trim_device(dev, 0);
            e = hipMalloc(&q, r);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return e;
            }
        }
    }
    g_blocks[q] = Block{dev, got};
    *p = q;
    return hipSuccess;
}

void devmem_free(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_blocks.find(p);
    if (it == g_blocks.end()) {   // not ours: nothing to do but hand it back
        (void)hipFree(p);
        return;
    }
    const Block b = it->second;
    g_blocks.erase(it);
    DeviceCache& c = g_cache[b.dev];
    if (c.cached + b.bytes > g_limit) {
        (void)hipFree(p);
        return;
    }
    c.free.emplace(b.bytes, p);
    c.cached += b.bytes;
}

extern "C" size_t asp_set_cache_limit(size_t bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    const size_t old = g_limit;
    g_limit = bytes;
    for (int d = 0; d < MAX_DEVICES; ++d) trim_device(d, bytes);
    return old;
}

extern "C" size_t asp_cached_bytes(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    size_t s = 0;
    for (const DeviceCache& c : g_cache) s += c.cached;
    return s;
}
