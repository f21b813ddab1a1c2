// First-fit sub-allocator over one caller-owned block of device memory.
//
// Host-only bookkeeping (no device calls): it hands out 256-byte aligned
// offsets into [0, capacity) and merges neighbouring free ranges on release,
// so that lattices of very different sizes can come and go without the
// block fragmenting into unusable pieces.  The serving loop uses it to admit
// lattices by their device-memory footprint.
#ifndef LBM_ARENA_H
#define LBM_ARENA_H

#include <cstddef>
#include <iterator>
#include <map>

namespace lbm_arena {

class Arena {
  public:
    static constexpr size_t kAlign = 256;

    explicit Arena(size_t capacity = 0) { reset(capacity); }

    void reset(size_t capacity)
    {
        capacity_ = capacity / kAlign * kAlign;
        free_.clear();
        if (capacity_) free_[0] = capacity_;
        used_ = peak_ = 0;
    }

    static size_t rounded(size_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

    // Reserve `bytes` (rounded up to kAlign); false if no free range fits.
    bool alloc(size_t bytes, size_t *offset)
    {
        const size_t need = rounded(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            *offset = off;
            used_ += need;
            if (used_ > peak_) peak_ = used_;
            return true;
        }
        return false;
    }

    // Return a range obtained from alloc (same size argument).
    void release(size_t offset, size_t bytes)
    {
        size_t off = offset, len = rounded(bytes == 0 ? 1 : bytes);
        used_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return;
            }
        }
        free_[off] = len;
    }

    // Could a request of `bytes` ever be satisfied (by an empty arena)?
    bool could_fit(size_t bytes) const { return rounded(bytes == 0 ? 1 : bytes) <= capacity_; }

    size_t capacity() const { return capacity_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t free_ranges() const { return free_.size(); }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &kv : free_)
            if (kv.second > m) m = kv.second;
        return m;
    }

  private:
    size_t capacity_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length, disjoint, never adjacent
};

}  // namespace lbm_arena

#endif
