// Host check of the server's pool allocator, built with the address and
// undefined-behaviour sanitizers by tests/test_host_sanitized.py.  A seeded
// random sequence of allocations and releases is checked against the
// allocator's contract: blocks are 256-byte aligned, lie inside the pool and
// never overlap; an allocation fails only when no free range is large enough
// (a first-fit scan over an independent interval model); releasing every block
// restores one free range of the whole pool.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "pool_allocator.h"

namespace {

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// Independent model: the set of live blocks; the largest free gap follows.
size_t largest_gap(const std::map<size_t, size_t> &live, size_t pool) {
    size_t best = 0, pos = 0;
    for (const auto &kv : live) {
        if (kv.first > pos) best = std::max(best, kv.first - pos);
        pos = kv.first + kv.second;
    }
    if (pool > pos) best = std::max(best, pool - pos);
    return best;
}

int check(uint64_t seed, size_t pool, int steps) {
    grav::PoolAllocator a(pool);
    std::map<size_t, size_t> live;   // offset -> rounded size
    std::mt19937_64 rng(seed);
    for (int s = 0; s < steps; ++s) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t want = 1 + rng() % (pool / 6);
            size_t off = 0;
            const bool ok = a.alloc(want, &off);
            const size_t need = round256(want);
            if (!ok) {
                if (largest_gap(live, pool) >= need) {
                    std::printf("seed %llu step %d: refused %zu with a large enough gap\n",
                                (unsigned long long)seed, s, need);
                    return 1;
                }
                continue;
            }
            if (off % 256 != 0 || off + need > pool) {
                std::printf("seed %llu step %d: block [%zu, +%zu) misplaced\n",
                            (unsigned long long)seed, s, off, need);
                return 1;
            }
            auto nx = live.lower_bound(off);
            if (nx != live.end() && nx->first < off + need) return 2;
            if (nx != live.begin()) {
                auto pv = std::prev(nx);
                if (pv->first + pv->second > off) return 3;
            }
            live[off] = need;
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            a.release(it->first, it->second);
            live.erase(it);
        }
    }
    for (const auto &kv : live) a.release(kv.first, kv.second);
    size_t off = 0;
    if (!a.alloc(pool, &off) || off != 0) {
        std::printf("seed %llu: pool not whole after releasing every block\n",
                    (unsigned long long)seed);
        return 4;
    }
    return 0;
}

}  // namespace

int main() {
    for (uint64_t seed = 1; seed <= 40; ++seed) {
        const int rc = check(seed, (size_t)(1 + seed % 7) << 20, 4000);
        if (rc) return rc;
    }
    std::printf("ok\n");
    return 0;
}
