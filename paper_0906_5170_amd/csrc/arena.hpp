// Host-side bookkeeping of the serving scheduler's device memory budget and
// its admission order.  No device code: the scheduler maps arena offsets to
// device addresses itself.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace cfi {

// First-fit allocator over the offsets [0, size) in 256-byte granules;
// freed ranges merge with free neighbours.
class Arena {
   public:
    static size_t granule(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) / 256 * 256; }

    void reset(size_t size) {
        size_ = size / 256 * 256;
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    // Lowest-offset free range that holds `bytes`; false when none does.
    bool alloc(size_t bytes, size_t* off) {
        bytes = granule(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = granule(bytes);
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
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
    size_t n_free_ranges() const { return free_.size(); }

   private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

// One admission pass: walk the queue in arrival order and admit every
// request whose bytes fit now (a later request may pass an earlier one that
// does not fit yet).  Returns the queue positions admitted, in order, with
// their offsets.
inline std::vector<std::pair<size_t, size_t>> admit_pass(Arena& a, const std::vector<size_t>& queue_bytes) {
    std::vector<std::pair<size_t, size_t>> out;
    for (size_t k = 0; k < queue_bytes.size(); ++k) {
        size_t off;
        if (a.alloc(queue_bytes[k], &off)) out.emplace_back(k, off);
    }
    return out;
}

}  // namespace cfi
