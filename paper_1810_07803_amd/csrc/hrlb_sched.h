// hrlb_sched.h -- device-memory arena and admission policy of the request server (host only, no
// HIP dependency, so that the policy can be exercised on a CPU).
#pragma once

#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace hrlb {

// First-fit allocator over one caller-provided device region [0, capacity).  Offsets and sizes are
// multiples of 256 bytes (the alignment a case workspace needs); a released block merges with its
// free neighbours, so a fully released arena is one free range again.
class Arena {
public:
    static constexpr size_t kAlign = 256;

    explicit Arena(size_t capacity = 0) { reset(capacity); }

    void reset(size_t capacity)
    {
        cap_ = capacity & ~(kAlign - 1);
        free_.clear();
        used_.clear();
        if (cap_) free_[0] = cap_;
    }

    static size_t round_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

    // offset of a new block of at least `bytes` (lowest address that fits), or -1
    long long alloc(size_t bytes)
    {
        const size_t need = round_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > need) free_[off + need] = sz - need;
            used_[off] = need;
            return (long long)off;
        }
        return -1;
    }

    // false if off is not the start of a live block (nothing changes then)
    bool release(size_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t start = off, size = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + size) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = size;
        return true;
    }

    size_t capacity() const { return cap_; }
    size_t used_bytes() const
    {
        size_t s = 0;
        for (const auto& kv : used_) s += kv.second;
        return s;
    }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t live_blocks() const { return used_.size(); }

    // free and used ranges tile [0, capacity) exactly, and no two free ranges touch
    bool consistent() const
    {
        std::map<size_t, std::pair<size_t, bool>> all;
        for (const auto& kv : free_) all[kv.first] = {kv.second, true};
        for (const auto& kv : used_) {
            if (all.count(kv.first)) return false;
            all[kv.first] = {kv.second, false};
        }
        size_t pos = 0;
        bool prev_free = false;
        for (const auto& kv : all) {
            if (kv.first != pos || kv.second.first == 0 || kv.second.first % kAlign) return false;
            if (prev_free && kv.second.second) return false;
            prev_free = kv.second.second;
            pos += kv.second.first;
        }
        return pos == cap_;
    }

private:
    size_t cap_ = 0;
    std::map<size_t, size_t> free_, used_;
};

// Admission in arrival order with bounded backfill.  q holds the waiting requests oldest first.
// try_place(i) tries to reserve what request i needs and returns true if it did.  A request that
// does not fit may be passed by later ones (each admission passing it counts one bypass) until it
// has been passed max_bypass times; from then on nothing behind it is admitted before it is.
// Returns the indices admitted, in order.
struct Waiting {
    int bypassed;
};

template <class TryPlace>
std::vector<int> admit_in_order(std::vector<Waiting>& q, int free_slots, int max_bypass, TryPlace try_place)
{
    std::vector<int> admitted, skipped;
    for (int i = 0; i < (int)q.size() && free_slots > 0; ++i) {
        bool starved = false;
        for (int k : skipped) starved = starved || q[k].bypassed >= max_bypass;
        if (starved) break;
        if (try_place(i)) {
            admitted.push_back(i);
            --free_slots;
            for (int k : skipped) ++q[k].bypassed;
        } else {
            skipped.push_back(i);
        }
    }
    return admitted;
}

}  // namespace hrlb
