// rc_sched.hpp -- host-side admission logic of the request server (internal).
//
// Pure C++ with no HIP dependency, so that the same code the server runs can
// be exercised on the CPU by a simulated executor (and built with the
// address and undefined-behaviour sanitizers).
//
//   Arena      first-fit allocator over one device slab, by byte offset;
//              blocks are freed in any order and neighbours coalesce.
//   admit()    one admission round: requests are taken in arrival order,
//              later requests fill in (backfill) while earlier ones do not
//              fit, as long as the bytes in flight stay within the budget,
//              the round stays under a ray cap, and every request whose
//              outputs the library allocates gets an arena block.  The
//              oldest waiting request can be passed over only max_bypass
//              times; after that nothing behind it is admitted until it is,
//              so a large request cannot be starved by a stream of small ones.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace rc {
namespace sched {

constexpr size_t kArenaAlign = 256;

inline size_t align_up(size_t n) { return (n + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

class Arena {
public:
    Arena() = default;
    explicit Arena(size_t cap) { reset(cap); }

    void reset(size_t cap)
    {
        cap_ = cap / kArenaAlign * kArenaAlign;
        free_.clear();
        used_ = 0;
        if (cap_)
            free_[0] = cap_;
    }

    // First fit.  Returns false (and leaves the arena unchanged) when no free
    // block holds n bytes; a zero-byte request takes no space and succeeds.
    bool alloc(size_t n, size_t *off)
    {
        n = align_up(n);
        if (n == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n)
                continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest)
                free_[at] = rest;
            used_ += n;
            return true;
        }
        return false;
    }

    // Return a block taken by alloc (same size argument).
    void release(size_t off, size_t n)
    {
        n = align_up(n);
        if (n == 0)
            return;
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {  // merge with the block after
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {  // merge with the block before
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &kv : free_)
            m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t free_blocks() const { return free_.size(); }

private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length, disjoint, non-adjacent
};

// What admission needs to know of a queued request.
struct Pending {
    size_t bytes = 0;        // charged against the budget while in flight
    size_t arena_bytes = 0;  // outputs the library allocates (part of bytes), 0 for caller buffers
    int64_t rays = 0;
    size_t arena_off = 0;    // set by admit() when arena_bytes > 0
    int bypassed = 0;        // times later requests were admitted while this one waited at the head
};

struct RoundLimits {
    size_t budget = 0;       // bytes in flight allowed
    int64_t max_rays = 0;    // ray cap of one round (a single larger request is admitted alone)
    int lookahead = 256;     // requests scanned per round
    bool fifo_only = false;  // plain mode: at most one request, strictly the oldest
    int max_bypass = 8;      // rounds the oldest request may be passed over
};

// Whether a request could ever be admitted (alone, with nothing in flight).
inline bool fits_alone(const Pending &p, const RoundLimits &lim) { return p.bytes <= lim.budget; }

// One admission round over `queue` (arrival order).  Removes the admitted
// requests from the queue and returns them in admission order; in_use is
// raised by their bytes.  Arena blocks are taken for requests that need
// them; a request that does not fit (budget, ray cap or arena) stays queued.
template <class R>
std::vector<R *> admit(std::deque<R *> &queue, size_t &in_use, Arena &arena, const RoundLimits &lim)
{
    std::vector<R *> batch;
    size_t bytes = 0;
    int64_t rays = 0;
    int scanned = 0;
    R *oldest_left = nullptr;  // the oldest request that stays queued this round
    bool overtaken = false;    // a later request was admitted after it was skipped
    for (auto it = queue.begin(); it != queue.end() && scanned < lim.lookahead; ++scanned) {
        Pending &p = (*it)->pending;
        bool fits = in_use + bytes + p.bytes <= lim.budget && (batch.empty() || rays + p.rays <= lim.max_rays);
        if (fits && p.arena_bytes)
            fits = arena.alloc(p.arena_bytes, &p.arena_off);
        if (fits) {
            batch.push_back(*it);
            bytes += p.bytes;
            rays += p.rays;
            overtaken = overtaken || oldest_left;
            it = queue.erase(it);
            if (lim.fifo_only)
                break;
        } else {
            if (lim.fifo_only)
                break;
            if (!oldest_left) {
                oldest_left = *it;
                if (p.bypassed >= lim.max_bypass)
                    break;  // the oldest request goes next: nothing overtakes it any more
            }
            ++it;
        }
    }
    if (overtaken)
        oldest_left->pending.bypassed += 1;
    in_use += bytes;
    return batch;
}

}  // namespace sched
}  // namespace rc
