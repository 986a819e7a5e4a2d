// Device workspace cache.  The library's scratch buffers (candidate lists,
// node tables, chunk sums, ...) are the same sizes from one call to the next;
// allocating and freeing them every call cost several milliseconds per C2
// build on MI355X (freeing a few hundred MB blocks in hipFreeAsync).  Blocks
// are therefore kept per device after use and handed out again: ws_malloc
// takes a cached block of at least the requested size (and at most twice
// it), else allocates with hipMalloc; ws_free returns the block to the cache.
// A block returned in a call may be reused later in the same call only on
// the same stream (stream order keeps that safe); the calls that allocate
// hold the device's lock (DeviceLock) until they have synchronised their
// stream, so another call never receives a block still in use.
//
// A caller that must not allocate sets an arena for its thread (ArenaScope):
// ws_malloc then hands out consecutive 256-byte aligned blocks of that
// memory and fails with hipErrorOutOfMemory when it is exhausted.
#include "knng_internal.hpp"

#include <map>
#include <mutex>
#include <new>
#include <unordered_map>

namespace knng {
namespace {

constexpr int kMaxDevices = 64;

// Arena of the calling thread (ArenaScope): while set, ws_malloc carves
// blocks from it and never calls hipMalloc; ws_free of an arena block is a
// no-op (the whole arena is released when the scope ends).
struct Arena {
    uint8_t* base;
    size_t cap;
    size_t used;
};
thread_local Arena* t_arena = nullptr;

struct Cache {
    std::mutex mu;                                // guards the maps
    std::multimap<size_t, void*> free_blocks;     // size class -> block
    std::unordered_map<void*, size_t> live;       // block -> size class
};

Cache& cache(int dev) {
    static Cache caches[kMaxDevices];
    return caches[dev];
}

std::mutex& device_mutex(int dev) {
    static std::mutex mus[kMaxDevices];
    return mus[dev];
}

int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
    return dev;
}

size_t size_class(size_t bytes) {
    const size_t g = bytes <= (size_t{1} << 20) ? 4096 : (size_t{1} << 20);
    return (bytes + g - 1) / g * g;
}

}  // namespace

size_t ws_arena_block(size_t bytes) {
    return (bytes == 0 ? size_t{1} : bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

ArenaScope::ArenaScope(void* base, size_t cap) {
    static_assert(sizeof(Arena) <= sizeof(storage_), "arena record fits the scope's storage");
    Arena* a = new (storage_) Arena{static_cast<uint8_t*>(base), cap, 0};
    t_arena = a;
}

ArenaScope::~ArenaScope() { t_arena = nullptr; }

hipError_t ws_malloc(void** p, size_t bytes, hipStream_t /*s*/) {
    *p = nullptr;
    if (t_arena != nullptr) {
        const size_t b = ws_arena_block(bytes);
        if (b > t_arena->cap - t_arena->used) return hipErrorOutOfMemory;
        *p = t_arena->base + t_arena->used;
        t_arena->used += b;
        return hipSuccess;
    }
    const int dev = current_device();
    if (dev < 0) return hipErrorInvalidDevice;
    const size_t sc = size_class(bytes == 0 ? 1 : bytes);
    Cache& c = cache(dev);
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.free_blocks.lower_bound(sc);
        if (it != c.free_blocks.end() && it->first <= 2 * sc) {
            *p = it->second;
            c.live[it->second] = it->first;
            c.free_blocks.erase(it);
            return hipSuccess;
        }
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sc);
    if (e == hipErrorOutOfMemory) {
        // give the cached blocks back and try once more
        ws_release_device(dev);
        e = hipMalloc(&q, sc);
    }
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(c.mu);
    c.live[q] = sc;
    *p = q;
    return hipSuccess;
}

void ws_free(void* p, hipStream_t /*s*/) {
    if (p == nullptr) return;
    if (t_arena != nullptr) {
        const uint8_t* q = static_cast<const uint8_t*>(p);
        if (q >= t_arena->base && q < t_arena->base + t_arena->cap) return;
    }
    const int dev = current_device();
    if (dev < 0) return;
    Cache& c = cache(dev);
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    c.free_blocks.emplace(it->second, p);
    c.live.erase(it);
}

void ws_release_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    Cache& c = cache(dev);
    std::lock_guard<std::mutex> g(c.mu);
    for (auto& kv : c.free_blocks) (void)hipFree(kv.second);
    c.free_blocks.clear();
}

DeviceLock::DeviceLock() : dev_(current_device()) {
    if (dev_ >= 0) device_mutex(dev_).lock();
}

DeviceLock::~DeviceLock() {
    if (dev_ >= 0) device_mutex(dev_).unlock();
}

int DeviceLock::device() const { return dev_; }

}  // namespace knng
