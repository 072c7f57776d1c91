#include "alloc.h"

namespace vr {

size_t DeviceArena::round_size(size_t bytes)
{
    const size_t small = 4096, large = 2u << 20;
    if (bytes == 0) bytes = 1;
    if (bytes < (1u << 20)) return (bytes + small - 1) / small * small;
    return (bytes + large - 1) / large * large;
}

DeviceArena::DeviceArena(int device) : device_(device)
{
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) soft_limit_ = total_b / 10 * 9;
    (void)hipGetLastError();
}

DeviceArena::~DeviceArena()
{
    std::lock_guard<std::mutex> g(mu_);
    trim_locked();
    for (hipEvent_t e : events_) (void)hipEventDestroy(e);
}

hipEvent_t DeviceArena::take_event()
{
    if (!events_.empty()) {
        hipEvent_t e = events_.back();
        events_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void* DeviceArena::take(std::multimap<size_t, Block>::iterator it, hipStream_t s)
{
    Block b = it->second;
    free_.erase(it);
    if (b.ev) {
        if (b.stream != s) (void)hipStreamWaitEvent(s, b.ev, 0);
        events_.push_back(b.ev);
    }
    live_[b.p] = b.size;
    in_use_ += b.size;
    return b.p;
}

void* DeviceArena::alloc(size_t bytes, hipStream_t s)
{
    const size_t want = round_size(bytes);
    const size_t limit = want + want / 4 + 4096;   // bound on the waste of a reused block
    std::lock_guard<std::mutex> g(mu_);
    auto best = free_.end();
    for (auto it = free_.lower_bound(want); it != free_.end() && it->first <= limit; ++it) {
        if (it->second.stream == s) {
            best = it;
            break;
        }
        if (best == free_.end()) best = it;
    }
    if (best != free_.end()) return take(best, s);
    const bool over = soft_limit_ && reserved_ + want > soft_limit_;
    if (over) {
        // near the device's capacity: any larger cached block beats a new one
        auto it = free_.lower_bound(want);
        if (it != free_.end()) return take(it, s);
        // else return the largest cached blocks until the new one fits
        (void)hipDeviceSynchronize();
        while (!free_.empty() && reserved_ + want > soft_limit_) {
            auto last = std::prev(free_.end());
            (void)hipFree(last->second.p);
            reserved_ -= last->second.size;
            if (last->second.ev) events_.push_back(last->second.ev);
            free_.erase(last);
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        trim_locked();
        p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    reserved_ += want;
    in_use_ += want;
    live_[p] = want;
    return p;
}

void* DeviceArena::alloc_fresh(size_t bytes)
{
    const size_t want = round_size(bytes);
    std::lock_guard<std::mutex> g(mu_);
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    reserved_ += want;
    in_use_ += want;
    live_[p] = want;
    return p;
}

void DeviceArena::release(void* p, hipStream_t s)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    const size_t size = it->second;
    live_.erase(it);
    in_use_ -= size;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) != hipSuccess) {
        (void)hipGetLastError();
        events_.push_back(e);
        e = nullptr;
        // no event: make the block safe for any stream before caching it
        (void)hipStreamSynchronize(s);
    }
    free_.insert({size, Block{p, size, s, e}});
}

void DeviceArena::trim_locked()
{
    if (free_.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& kv : free_) {
        (void)hipFree(kv.second.p);
        reserved_ -= kv.second.size;
        if (kv.second.ev) events_.push_back(kv.second.ev);
    }
    free_.clear();
}

void DeviceArena::trim()
{
    std::lock_guard<std::mutex> g(mu_);
    trim_locked();
}

void DeviceArena::usage(size_t* reserved, size_t* in_use)
{
    std::lock_guard<std::mutex> g(mu_);
    if (reserved) *reserved = reserved_;
    if (in_use) *in_use = in_use_;
}

}  // namespace vr
