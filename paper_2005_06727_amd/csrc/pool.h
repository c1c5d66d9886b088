// First-fit allocator over one fixed region of `cap` bytes (offsets only; the
// memory itself is owned by the caller).  The server carves every in-flight
// batch's workspace out of one device allocation of its HBM budget with it,
// so admission is byte accounting against the whole budget rather than a
// fixed share per stream.  Pure host code: no HIP, no locking (the caller
// holds its own lock).
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace wmd {

class RegionPool {
  public:
    static constexpr size_t kAlign = 256;

    explicit RegionPool(size_t cap = 0) { reset(cap); }

    // Forget every allocation; the whole region is free again.
    void reset(size_t cap) {
        cap_ = cap / kAlign * kAlign;
        used_ = 0;
        free_.clear();
        if (cap_ > 0) free_[0] = cap_;
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }

    // Bytes actually reserved for a request of `bytes` (a multiple of kAlign,
    // at least kAlign).
    static size_t rounded(size_t bytes) {
        const size_t r = (bytes + kAlign - 1) / kAlign * kAlign;
        return r == 0 ? kAlign : r;
    }

    // Largest request that alloc() would grant right now.
    size_t largest_free() const {
        size_t best = 0;
        for (const auto& f : free_)
            if (f.second > best) best = f.second;
        return best;
    }

    // Reserve rounded(bytes) at the lowest offset that has room; false (and
    // *off untouched) when no free range is large enough.
    bool alloc(size_t bytes, size_t* off) {
        const size_t need = rounded(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t o = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[o + need] = len - need;
            used_ += need;
            *off = o;
            return true;
        }
        return false;
    }

    // Return a range handed out by alloc(off, bytes) with the same `bytes`;
    // adjacent free ranges merge.
    void release(size_t off, size_t bytes) {
        const size_t len = rounded(bytes);
        used_ -= len;
        auto next = free_.lower_bound(off);
        size_t start = off, size = len;
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

    // Free ranges in offset order (offset, length), for checks.
    const std::map<size_t, size_t>& free_ranges() const { return free_; }

  private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length, disjoint, never adjacent
};

}  // namespace wmd
