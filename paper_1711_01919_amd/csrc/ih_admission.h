// Host-side bookkeeping of the serving loop's device memory: a first-fit
// allocator over one block of device addresses (offsets only) and the
// retention of each video stream's latest integral histogram, with the
// admission decision built on them.  No HIP calls: this file compiles and is
// tested on a machine without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <list>
#include <map>
#include <mutex>

namespace ih {

// First-fit allocator over [0, size): offsets only, neighbours merged on
// free, sizes rounded up to `align`.  Thread-safe.
class Arena {
public:
    explicit Arena(size_t align = 256) : align_(align) {}
    void reset(size_t size);
    bool alloc(size_t bytes, size_t* off);
    void release(size_t off, size_t bytes);
    size_t used() const;
    size_t size() const;
    size_t peak() const;
    size_t largest_free() const;
    size_t rounded(size_t bytes) const;

private:
    mutable std::mutex mu_;
    size_t align_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;       // offset -> bytes
};

// The latest integral histogram of a video stream kept on the device after
// its request finished, in least-recently-retained order.  An entry that a
// query is reading (users > 0) is never evicted; replacing it only marks it,
// and its memory goes back when its last reader is done.
struct Retained {
    uint64_t ticket = 0;
    int32_t H = 0, W = 0, B = 0;
    size_t off = 0, bytes = 0;
    int32_t users = 0;
};

enum class Admit {
    kOk,       // both blocks reserved
    kWait,     // not now: memory held by work in flight or by retained
               // histograms being read may free up
    kNever     // nothing holds memory that could free up, and it still does
               // not fit: the request can never be admitted
};

// Device memory of the serving loop: the arena plus the retained histograms
// in it.  Not thread-safe: the scheduler thread owns it (the server guards
// reads of its counters with its own lock).
class Residency {
public:
    void reset(size_t budget) { arena_.reset(budget); }
    Arena& arena() { return arena_; }
    const Arena& arena() const { return arena_; }

    // Reserve a request's integral-histogram block and work block.  When
    // either does not fit, the least recently retained histogram that nobody
    // is reading is evicted and both are tried again, until they fit or
    // nothing evictable is left.  in_flight: whether admitted work still
    // holds memory that it will release.
    Admit reserve(size_t ih_bytes, size_t work_bytes, bool in_flight, size_t* ih_off, size_t* work_off);
    // Reserve one block the same way (evicting as needed), keeping the
    // retained entry of `keep_stream` (being read by the caller).
    Admit reserve_one(size_t bytes, bool in_flight, int32_t keep_stream, size_t* off);
    void release(size_t off, size_t bytes) { arena_.release(off, bytes); }

    // A finished request's histogram becomes its stream's latest; the
    // stream's previous one is released (or, while being read, released by
    // its last reader).
    void retain(int32_t stream_id, const Retained& r);
    // The latest histogram of a stream, marked as being read (users + 1).
    bool acquire(int32_t stream_id, Retained* out);
    // A reader of (stream_id, ticket) is done.
    void release_reader(int32_t stream_id, uint64_t ticket);
    size_t retained_count() const { return latest_.size(); }
    // stream -> ticket of its latest resident histogram
    std::map<int32_t, uint64_t> tickets() const;
    // Evict the least recently retained histogram nobody is reading (other
    // than keep_stream's).  False when there is none.
    bool evict_one(int32_t keep_stream = -1);

private:
    bool any_in_use() const;
    Arena arena_;
    std::map<int32_t, Retained> latest_;             // stream -> its latest histogram
    std::list<int32_t> lru_;                         // streams, least recently retained first
    std::list<Retained> orphans_;                    // replaced while being read
};

}  // namespace ih
