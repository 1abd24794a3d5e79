// Host bookkeeping of the server's device memory pool: first-fit allocation
// over [0, size) in 256-byte units, with coalescing of neighbouring free
// ranges on release.  Plain C++ (no HIP), so it is also checked on the host
// under the address and undefined-behaviour sanitizers.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace grav {

class PoolAllocator {
  public:
    explicit PoolAllocator(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, base = it->first + bytes;
                free_.erase(it);
                if (rest) free_[base] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
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
  private:
    std::map<size_t, size_t> free_;
};

}  // namespace grav
