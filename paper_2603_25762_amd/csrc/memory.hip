// Device memory for the library's buffers: blocks are kept per device after release and
// handed out again for a later request of the same size class, so that graph builds and
// solves in a loop do not pay hipMalloc / hipFree (tens of microseconds each, and hipFree
// waits for the whole device) for every buffer.
//
// Reuse is safe because every release happens when no queued work can still use the
// block: temporaries are released after their stream has been synchronised, a buffer that
// is reallocated waits for the device first, and graphs (with their solve plans) are freed
// only after a device synchronisation.  At most kCacheCap bytes per device stay cached;
// a failed hipMalloc releases the device's cached blocks and tries once more.
#include <map>
#include <mutex>
#include <unordered_map>

#include "internal.h"

namespace qh {

namespace {

constexpr size_t kCacheCap = (size_t)4 << 30;

struct DeviceCache {
    std::multimap<size_t, void *> idle;   // size class -> block
    size_t idle_bytes = 0;
};

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

void trim(int device) {   // caller holds g_mu
    DeviceCache &c = g_cache[device];
    for (auto &kv : c.idle) (void)hipFree(kv.second);
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
    auto it = c.idle.find(cls);
    if (it != c.idle.end()) {
        void *p = it->second;
        c.idle.erase(it);
        c.idle_bytes -= cls;
        g_live[p] = Block{dev, cls};
        return p;
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
    if (c.idle_bytes + b.cls > kCacheCap) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != b.device) (void)hipSetDevice(b.device);
        (void)hipFree(p);
        if (cur != b.device) (void)hipSetDevice(cur);
        return;
    }
    c.idle.emplace(b.cls, p);
    c.idle_bytes += b.cls;
}

}  // namespace qh
