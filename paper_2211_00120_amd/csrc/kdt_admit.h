// kdt_admit.h -- memory pool and admission policy of the build server (plain
// C++, no HIP, so the policy is testable on any host).
//
// The server owns one device allocation of the configured HBM budget and
// carves it with ArenaAllocator.  A batch of requests holds two blocks: its
// points and outputs (kept until every request of the batch is released) and
// its build workspace (freed as soon as the batch has run).  choose_batch
// decides which queued requests start next.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "kdt_plan.h"

namespace kdt {

// First-fit allocator over [0, capacity) with WS_ALIGN granularity; free
// blocks are coalesced with their neighbours.
class ArenaAllocator {
public:
    static constexpr size_t NPOS = ~(size_t)0;

    explicit ArenaAllocator(size_t capacity = 0) { reset(capacity); }

    void reset(size_t capacity)
    {
        cap_ = capacity & ~(WS_ALIGN - 1);
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = 0;
    }

    size_t alloc(size_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            return off;
        }
        return NPOS;
    }

    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
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

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t largest_free() const
    {
        size_t b = 0;
        for (const auto& kv : free_) b = std::max(b, kv.second);
        return b;
    }
    size_t free_blocks() const { return free_.size(); }

private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
};

// Device bytes of a batch's points and outputs: points, tree (n*k float32
// each), perm (n uint32), dim (n uint8) of all its requests back to back,
// and a status word.
inline size_t batch_output_bytes(uint64_t ntotal, uint32_t k)
{
    return align_up(ntotal * k * 4) * 2 + align_up(ntotal * 4) + align_up(ntotal) + WS_ALIGN;
}

struct QueuedShape {
    uint32_t n, k;
    int mode;
};

struct BatchChoice {
    std::vector<size_t> picks;   // queue positions, in queue order
    size_t out_bytes = 0, ws_bytes = 0;
};

// The batch to start now: the oldest request and, after it, the queued
// requests of the same k and split rule (at most max_requests, at most
// max_points points), as many as let both blocks fit the pool.  Requests of
// another shape stay queued in order.  An empty choice means the oldest
// request does not fit yet.
inline BatchChoice choose_batch(const std::vector<QueuedShape>& queue, const ArenaAllocator& pool,
                                uint32_t max_requests, uint64_t max_points)
{
    BatchChoice best;
    if (queue.empty()) return best;
    const QueuedShape& h = queue[0];
    std::vector<size_t> cand;
    uint64_t pts = 0;
    for (size_t i = 0; i < queue.size() && cand.size() < max_requests; ++i) {
        const QueuedShape& q = queue[i];
        if (q.k != h.k || q.mode != h.mode) continue;
        if (!cand.empty() && pts + q.n > max_points) break;
        cand.push_back(i);
        pts += q.n;
    }
    // the two blocks must fit in two separate free blocks; take the largest
    // prefix of the candidates that does (binary search on its length)
    auto fits = [&](size_t m, BatchChoice& c) {
        std::vector<uint32_t> n(m);
        uint64_t tot = 0;
        for (size_t j = 0; j < m; ++j) {
            n[j] = queue[cand[j]].n;
            tot += n[j];
        }
        c.out_bytes = batch_output_bytes(tot, h.k);
        c.ws_bytes = workspace_bytes_any(n, h.k, h.mode == 1);
        ArenaAllocator trial = pool;
        if (trial.alloc(c.out_bytes) == ArenaAllocator::NPOS) return false;
        return trial.alloc(c.ws_bytes) != ArenaAllocator::NPOS;
    };
    size_t lo = 0, hi = cand.size();
    while (lo < hi) {
        const size_t mid = (lo + hi + 1) / 2;
        BatchChoice c;
        if (fits(mid, c)) lo = mid;
        else hi = mid - 1;
    }
    if (lo == 0) return best;
    fits(lo, best);
    best.picks.assign(cand.begin(), cand.begin() + lo);
    return best;
}

// Bytes a single request needs in an otherwise empty pool (both blocks).
inline size_t request_footprint(uint32_t n, uint32_t k, int mode)
{
    return batch_output_bytes(n, k) + workspace_bytes_any(std::vector<uint32_t>{n}, k, mode == 1);
}

}  // namespace kdt
