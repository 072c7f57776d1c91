// Caching device allocator of one context.  Blocks come from hipMalloc once
// and are kept: a freed block goes back to a size-ordered free list tagged with
// the stream it was freed on and an event recorded there, so a later request
// of about the same size reuses it (at once on the same stream; behind a wait
// on that event on another).  Steady-state layer calls therefore make no
// runtime allocation at all, and blocks are never returned to the runtime
// while the context lives.  Near the device's capacity (a new block would take
// the held total past 90 % of its memory) a larger cached block is reused
// instead, or else the largest cached blocks are released (after a device
// synchronisation) until the new one fits; a failed hipMalloc releases the
// whole cache and retries.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace vr {

class DeviceArena {
public:
    explicit DeviceArena(int device);
    ~DeviceArena();
    DeviceArena(const DeviceArena&) = delete;
    DeviceArena& operator=(const DeviceArena&) = delete;

    // Memory usable by work queued on s after this call; nullptr when the
    // device is out of memory even with the cache released.
    void* alloc(size_t bytes, hipStream_t s);
    // A block straight from the runtime, bypassing the cache (for memory a
    // captured graph will own: no stream dependency may be recorded then).
    void* alloc_fresh(size_t bytes);
    // Stream-ordered free: the block may be reused once the work queued on s
    // before this call has finished.
    void release(void* p, hipStream_t s);
    // Synchronises the device and returns every cached free block.
    void trim();
    void usage(size_t* reserved, size_t* in_use);

    static size_t round_size(size_t bytes);

private:
    struct Block {
        void* p;
        size_t size;
        hipStream_t stream;
        hipEvent_t ev;
    };
    hipEvent_t take_event();
    void* take(std::multimap<size_t, Block>::iterator it, hipStream_t s);
    void trim_locked();

    int device_;
    std::mutex mu_;
    std::multimap<size_t, Block> free_;
    std::unordered_map<void*, size_t> live_;
    std::vector<hipEvent_t> events_;
    size_t reserved_ = 0, in_use_ = 0, soft_limit_ = 0;
};

}  // namespace vr
