// Host-side bookkeeping of the serving loop's device memory (see
// ih_admission.h).  Plain C++, no HIP.
#include "ih_admission.h"

#include <algorithm>
#include <iterator>

namespace ih {

size_t Arena::rounded(size_t bytes) const
{
    bytes = std::max<size_t>(bytes, 1);
    return (bytes + align_ - 1) / align_ * align_;
}

void Arena::reset(size_t size)
{
    std::lock_guard<std::mutex> lock(mu_);
    size_ = size / align_ * align_;
    free_.clear();
    if (size_) free_[0] = size_;
    used_ = 0;
    peak_ = 0;
}

bool Arena::alloc(size_t bytes, size_t* off)
{
    std::lock_guard<std::mutex> lock(mu_);
    bytes = rounded(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < bytes) continue;
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
    }
    return false;
}

void Arena::release(size_t off, size_t bytes)
{
    std::lock_guard<std::mutex> lock(mu_);
    bytes = rounded(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
        it->second += next->second;
        free_.erase(next);
    }
    if (it != free_.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            free_.erase(it);
        }
    }
}

size_t Arena::used() const
{
    std::lock_guard<std::mutex> lock(mu_);
    return used_;
}

size_t Arena::size() const
{
    std::lock_guard<std::mutex> lock(mu_);
    return size_;
}

size_t Arena::peak() const
{
    std::lock_guard<std::mutex> lock(mu_);
    return peak_;
}

size_t Arena::largest_free() const
{
    std::lock_guard<std::mutex> lock(mu_);
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
}

bool Residency::any_in_use() const
{
    if (!orphans_.empty()) return true;
    for (auto& kv : latest_)
        if (kv.second.users > 0) return true;
    return false;
}

bool Residency::evict_one(int32_t keep_stream)
{
    for (auto it = lru_.begin(); it != lru_.end(); ++it) {
        if (*it == keep_stream) continue;
        auto e = latest_.find(*it);
        if (e == latest_.end() || e->second.users > 0) continue;
        arena_.release(e->second.off, e->second.bytes);
        latest_.erase(e);
        lru_.erase(it);
        return true;
    }
    return false;
}

Admit Residency::reserve(size_t ih_bytes, size_t work_bytes, bool in_flight, size_t* ih_off, size_t* work_off)
{
    for (;;) {
        size_t a = 0, b = 0;
        if (arena_.alloc(ih_bytes, &a)) {
            if (arena_.alloc(work_bytes, &b)) {
                *ih_off = a;
                *work_off = b;
                return Admit::kOk;
            }
            arena_.release(a, ih_bytes);
        }
        if (!evict_one()) break;
    }
    return in_flight || any_in_use() ? Admit::kWait : Admit::kNever;
}

Admit Residency::reserve_one(size_t bytes, bool in_flight, int32_t keep_stream, size_t* off)
{
    for (;;) {
        if (arena_.alloc(bytes, off)) return Admit::kOk;
        if (!evict_one(keep_stream)) break;
    }
    return in_flight || any_in_use() ? Admit::kWait : Admit::kNever;
}

void Residency::retain(int32_t stream_id, const Retained& r)
{
    auto old = latest_.find(stream_id);
    if (old != latest_.end()) {
        if (old->second.users > 0) orphans_.push_back(old->second);
        else arena_.release(old->second.off, old->second.bytes);
        lru_.remove(stream_id);
        latest_.erase(old);
    }
    Retained e = r;
    e.users = 0;
    latest_[stream_id] = e;
    lru_.push_back(stream_id);
}

std::map<int32_t, uint64_t> Residency::tickets() const
{
    std::map<int32_t, uint64_t> t;
    for (auto& kv : latest_) t[kv.first] = kv.second.ticket;
    return t;
}

bool Residency::acquire(int32_t stream_id, Retained* out)
{
    auto it = latest_.find(stream_id);
    if (it == latest_.end()) return false;
    it->second.users += 1;
    *out = it->second;
    return true;
}

void Residency::release_reader(int32_t stream_id, uint64_t ticket)
{
    auto it = latest_.find(stream_id);
    if (it != latest_.end() && it->second.ticket == ticket) {
        it->second.users -= 1;
        return;
    }
    for (auto o = orphans_.begin(); o != orphans_.end(); ++o) {
        if (o->ticket != ticket) continue;
        if (--o->users == 0) {
            arena_.release(o->off, o->bytes);
            orphans_.erase(o);
        }
        return;
    }
}

}  // namespace ih
