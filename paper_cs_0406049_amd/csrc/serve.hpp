// serve.hpp -- host-side pieces of the request server that tests can reach:
// the first-fit arena allocator for output buffers.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>

namespace mi355 {

// First-fit allocator over [0, capacity) with `align`-byte granules; freed
// ranges coalesce with their neighbours.  Not thread-safe (the scheduler
// thread owns it).
class Arena {
public:
    explicit Arena(uint64_t capacity = 0, uint64_t align = 256) { reset(capacity, align); }

    void reset(uint64_t capacity, uint64_t align)
    {
        align_ = align;
        capacity_ = capacity / align * align;
        free_.clear();
        if (capacity_ > 0)
            free_[0] = capacity_;
        used_ = 0;
    }

    // Offset of a block of at least `bytes`, or -1.
    int64_t alloc(uint64_t bytes)
    {
        const uint64_t need = (bytes + align_ - 1) / align_ * align_;
        if (need == 0)
            return -1;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const uint64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > need)
                    free_[off + need] = len - need;
                used_ += need;
                return (int64_t)off;
            }
        }
        return -1;
    }

    void release(uint64_t off, uint64_t bytes)
    {
        const uint64_t len = (bytes + align_ - 1) / align_ * align_;
        used_ -= len;
        auto next = free_.lower_bound(off);
        uint64_t start = off, size = len;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + len == next->first) {
            size += next->second;
            free_.erase(next);
        }
        free_[start] = size;
    }

    uint64_t used() const { return used_; }
    uint64_t capacity() const { return capacity_; }
    size_t fragments() const { return free_.size(); }
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (auto &kv : free_)
            m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    uint64_t align_ = 256, capacity_ = 0, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

}  // namespace mi355
