// Device memory for the library's buffers: blocks are kept per device after release and
// handed out again for a later request that fits (the smallest idle block of at least the
// request's size class and at most twice it), so that graph builds and solves in a loop do
// not pay hipMalloc / hipFree (tens of microseconds each, and hipFree waits for the whole
// device) for every buffer, also when their sizes vary from one graph to the next.
//
// Reuse is safe because every release happens when no queued work can still use the
// block: temporaries are released after their stream has been synchronised, a buffer that
// is reallocated waits for the device first, and graphs (with their solve plans) are freed
// only after a device synchronisation.  At most a quarter of the device's memory (and no
// more than kCacheCapMax) stays cached per device, enough for the graphs of a large batch to
// be recycled into the next one; a failed hipMalloc releases the device's cached blocks and
// tries once more, and release_cached() hands every cached block back to the device.
//
// That argument holds within one stream.  Host threads that work on streams of their own
// (the many-graph build) therefore get pools of their own: a thread with a pool tag
// returns blocks only there, takes them from there first and else from the shared pool
// (which the many-graph build only opens to its threads after a device synchronisation,
// with its caller waiting), and its pool joins the shared one once its stream has been
// synchronised.
#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>

#include "internal.h"

namespace qh {

namespace {

constexpr size_t kCacheCapMax = (size_t)64 << 30;
constexpr size_t kCacheCapDefault = (size_t)4 << 30;   // until the device's size is known

struct DeviceCache {
    std::map<uintptr_t, std::multimap<size_t, void *>> idle;   // pool tag -> size class -> block
    size_t idle_bytes = 0;
    size_t cap = 0;                                            // 0: not yet set
};

thread_local uintptr_t t_pool = 0;   // 0: the shared pool

struct Block {
    int device;
    size_t cls;
};

std::mutex g_mu;
std::map<int, DeviceCache> g_cache;
std::unordered_map<void *, Block> g_live;

size_t size_class(size_t bytes) {
    const size_t q = bytes <= ((size_t)1 << 20) ? 4096 : ((size_t)2 << 20);
    return (bytes + q - 1) / q * q;
}

void trim(int device) {   // caller holds g_mu (hipFree waits for the device's work)
    DeviceCache &c = g_cache[device];
    for (auto &pool : c.idle)
        for (auto &kv : pool.second) (void)hipFree(kv.second);
    c.idle.clear();
    c.idle_bytes = 0;
}

}  // namespace

void *device_alloc(size_t bytes) {
    int dev = 0;
    QH_HIP(hipGetDevice(&dev));
    const size_t cls = size_class(bytes == 0 ? 1 : bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[dev];
    if (!c.cap) {           // the device is current here
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && total_b)
            c.cap = std::min(total_b / 4, kCacheCapMax);
        else
            (void)hipGetLastError();
        if (!c.cap) c.cap = kCacheCapDefault;
    }
    for (uintptr_t tag : {t_pool, (uintptr_t)0}) {
        auto &pool = c.idle[tag];
        auto it = pool.lower_bound(cls);
        if (it != pool.end() && it->first <= 2 * cls) {
            void *p = it->second;
            const size_t have = it->first;     // the block keeps its own size class
            pool.erase(it);
            c.idle_bytes -= have;
            g_live[p] = Block{dev, have};
            return p;
        }
        if (tag == 0) break;
    }
    void *p = nullptr;
    if (hipMalloc(&p, cls) != hipSuccess) {
        (void)hipGetLastError();
        trim(dev);
        if (hipMalloc(&p, cls) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    g_live[p] = Block{dev, cls};
    return p;
}

void device_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    const Block b = it->second;
    g_live.erase(it);
    DeviceCache &c = g_cache[b.device];
    if (c.idle_bytes + b.cls > (c.cap ? c.cap : kCacheCapDefault)) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != b.device) (void)hipSetDevice(b.device);
        (void)hipFree(p);
        if (cur != b.device) (void)hipSetDevice(cur);
        return;
    }
    c.idle[t_pool].emplace(b.cls, p);
    c.idle_bytes += b.cls;
}

void set_pool(uintptr_t tag) { t_pool = tag; }

size_t release_cached() {
    std::lock_guard<std::mutex> lk(g_mu);
    size_t released = 0;
    int cur = -1;
    for (auto &kv : g_cache) {
        if (kv.second.idle.empty()) continue;   // no device call when nothing is cached
        if (cur < 0) (void)hipGetDevice(&cur);
        released += kv.second.idle_bytes;
        if (kv.first != cur) (void)hipSetDevice(kv.first);
        trim(kv.first);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    return released;
}

void merge_pool(int device, uintptr_t tag) {
    if (tag == 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[device];
    auto it = c.idle.find(tag);
    if (it == c.idle.end()) return;
    auto &shared = c.idle[0];
    for (auto &kv : it->second) shared.emplace(kv.first, kv.second);
    c.idle.erase(it);
}

}  // namespace qh
