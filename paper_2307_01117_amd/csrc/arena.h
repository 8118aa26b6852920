// arena.h -- first-fit bookkeeping of one contiguous device block, used by
// the server to admit requests by their HBM footprint.  Pure host code (no
// HIP calls), so it is unit-tested on the CPU.
#pragma once

#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace heat {

class ArenaBook {
  public:
    static constexpr size_t ALIGN = 256;
    static size_t round(size_t b) { return (b + ALIGN - 1) & ~(ALIGN - 1); }

    void reset(size_t cap) {
        cap_ = cap & ~(ALIGN - 1);
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = peak_ = 0;
    }
    // First fit; returns false (and leaves the book unchanged) if no free
    // range is large enough.
    bool alloc(size_t bytes, size_t *off) {
        bytes = round(bytes);
        if (bytes == 0) bytes = ALIGN;
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
    // Return a block obtained from alloc (same size); merges with neighbours.
    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        if (bytes == 0) bytes = ALIGN;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t cap() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t free_ranges() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;   // offset -> size, coalesced, non-adjacent
};

}  // namespace heat
