// Randomised test of the device-pool bookkeeping (sw_pool.h) on the host:
// blocks never overlap, stay inside the pool, accounting is exact, freeing
// everything coalesces back to one range, and the peak never exceeds capacity.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "sw_pool.h"

#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); return 1; } } while (0)

int main() {
    std::mt19937_64 rng(2208);
    for (int round = 0; round < 50; ++round) {
        const int64_t cap = (int64_t)(rng() % 4096 + 1) * sw::PoolAllocator::kAlign;
        sw::PoolAllocator p(cap);
        CHECK(p.capacity() == cap);
        std::map<int64_t, int64_t> live;  // off -> rounded size
        int64_t used = 0;
        for (int step = 0; step < 5000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                const int64_t n = (int64_t)(rng() % (cap / 4 + 1));
                const int64_t off = p.alloc(n);
                if (off < 0) {
                    CHECK(p.largest_free() < sw::PoolAllocator::round_up(n > 0 ? n : 1));
                    continue;
                }
                const int64_t len = sw::PoolAllocator::round_up(n > 0 ? n : 1);
                CHECK(off % sw::PoolAllocator::kAlign == 0);
                CHECK(off >= 0 && off + len <= cap);
                auto nx = live.lower_bound(off);
                if (nx != live.end()) CHECK(off + len <= nx->first);
                if (nx != live.begin()) { auto pv = std::prev(nx); CHECK(pv->first + pv->second <= off); }
                live[off] = len;
                used += len;
            } else {
                auto it = live.begin();
                std::advance(it, (long)(rng() % live.size()));
                CHECK(p.release(it->first));
                used -= it->second;
                live.erase(it);
            }
            CHECK(p.in_use() == used);
            CHECK(p.peak() <= cap);
            CHECK(p.live_blocks() == live.size());
        }
        CHECK(!p.release(cap + 1));
        for (auto& kv : live) CHECK(p.release(kv.first));
        CHECK(p.in_use() == 0);
        CHECK(p.free_ranges() == 1 && p.largest_free() == cap);
    }
    std::printf("pool ok\n");
    return 0;
}
