// sw_pool.h -- bookkeeping of a device memory pool: first-fit allocation of
// byte ranges inside one fixed-size device buffer, with coalescing on free.
// Pure host code (no HIP), so it can be unit-tested on a machine without a
// GPU.  Not thread-safe: the caller serialises access.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace sw {

class PoolAllocator {
public:
    static constexpr int64_t kAlign = 256;

    explicit PoolAllocator(int64_t capacity = 0) { reset(capacity); }

    void reset(int64_t capacity) {
        cap_ = capacity < 0 ? 0 : capacity - capacity % kAlign;
        free_.clear();
        used_.clear();
        in_use_ = 0;
        peak_ = 0;
        if (cap_ > 0) free_[0] = cap_;
    }

    static int64_t round_up(int64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    // Offset of a block of at least n bytes, or -1 if no free range is large
    // enough.  n == 0 allocates one alignment unit.
    int64_t alloc(int64_t n) {
        if (n < 0) return -1;
        const int64_t need = round_up(n > 0 ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const int64_t off = it->first;
            const int64_t rest = it->second - need;
            free_.erase(it);
            if (rest > 0) free_[off + need] = rest;
            used_[off] = need;
            in_use_ += need;
            if (in_use_ > peak_) peak_ = in_use_;
            return off;
        }
        return -1;
    }

    // Release a block returned by alloc; returns false for an unknown offset.
    bool release(int64_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        int64_t start = off, len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
        return true;
    }

    int64_t capacity() const { return cap_; }
    int64_t in_use() const { return in_use_; }
    int64_t peak() const { return peak_; }
    int64_t largest_free() const {
        int64_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    size_t free_ranges() const { return free_.size(); }
    size_t live_blocks() const { return used_.size(); }

private:
    int64_t cap_ = 0;
    int64_t in_use_ = 0;
    int64_t peak_ = 0;
    std::map<int64_t, int64_t> free_;   // offset -> length
    std::map<int64_t, int64_t> used_;   // offset -> length
};

}  // namespace sw
