// Host-side admission of the serving loop: a first-fit allocator over the
// request pool and the in-order admission rule.  Pure host code (no HIP), so
// it is tested on the CPU against a reference model.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace heston {
namespace rt {

// First-fit allocator over one device buffer, in 256-byte units.
class Pool {
  public:
    void init(unsigned char *base, uint64_t bytes)
    {
        base_ = base;
        free_.clear();
        used_.clear();
        if (bytes >= 256)
            free_[0] = bytes & ~uint64_t(255);
    }
    uint64_t free_bytes() const
    {
        uint64_t t = 0;
        for (auto &f : free_)
            t += f.second;
        return t;
    }
    unsigned char *alloc(uint64_t bytes)
    {
        bytes = (bytes + 255) & ~uint64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const uint64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest)
                    free_[off + bytes] = rest;
                used_[off] = bytes;
                return base_ + off;
            }
        }
        return nullptr;
    }
    void release(unsigned char *p)
    {
        const uint64_t off = (uint64_t)(p - base_);
        auto u = used_.find(off);
        if (u == used_.end())
            return;
        uint64_t bytes = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(off);
        uint64_t start = off;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                bytes += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.find(off + (bytes - (off - start)));
        if (next != free_.end()) {
            bytes += next->second;
            free_.erase(next);
        }
        free_[start] = bytes;
    }

  private:
    unsigned char *base_ = nullptr;
    std::map<uint64_t, uint64_t> free_, used_;
};

// Moves queued requests to the active set in arrival order while fewer than
// `max_active` are active and the pool holds the head's bytes(q); the first
// request that does not fit stops admission (no overtaking, so no request
// waits forever behind later, smaller ones).  place(q, mem) records the
// allocation.  Returns the number admitted.
template <class Queue, class Active, class Bytes, class Place>
size_t admit_in_order(Queue &queue, Active &active, size_t max_active, Pool &pool, Bytes bytes,
                      Place place)
{
    size_t n = 0;
    while (!queue.empty() && active.size() < max_active) {
        auto q = queue.front();
        unsigned char *m = pool.alloc(bytes(q));
        if (!m)
            break;
        place(q, m);
        queue.pop_front();
        active.push_back(q);
        ++n;
    }
    return n;
}

} // namespace rt
} // namespace heston
