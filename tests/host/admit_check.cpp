// Host check of the build server's memory pool and admission policy
// (kdt_admit.h): the allocator against a byte-map model under random
// alloc/free sequences, and choose_batch's picks (oldest first, one shape,
// limits honoured, both blocks fit, no further candidate would fit).
// Prints "ok" and exits 0 on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "kdt_admit.h"

using namespace kdt;

static int g_fail = 0;
#define CHECK(cond, ...)                                \
    do {                                                \
        if (!(cond)) {                                  \
            std::printf("FAIL %s: ", #cond);            \
            std::printf(__VA_ARGS__);                   \
            std::printf("\n");                          \
            if (++g_fail > 20) std::exit(1);            \
        }                                               \
    } while (0)

static void check_arena(std::mt19937_64& rng)
{
    const size_t units = 4096;                    // capacity in WS_ALIGN units
    ArenaAllocator a(units * WS_ALIGN);
    std::vector<int> owner(units, -1);            // model: which block holds each unit
    struct Blk { size_t off, bytes; int id; };
    std::vector<Blk> live;
    int next_id = 0;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t bytes = 1 + rng() % (64 * WS_ALIGN);
            const size_t off = a.alloc(bytes);
            const size_t u = (bytes + WS_ALIGN - 1) / WS_ALIGN;
            // the model says whether some gap of u free units exists
            bool any = false;
            for (size_t s = 0, run = 0; s < units && !any; ++s) {
                run = owner[s] < 0 ? run + 1 : 0;
                any = run >= u;
            }
            if (off == ArenaAllocator::NPOS) {
                CHECK(!any, "alloc of %zu units failed although a gap exists", u);
                continue;
            }
            CHECK(off % WS_ALIGN == 0 && off / WS_ALIGN + u <= units, "block in range");
            for (size_t s = off / WS_ALIGN; s < off / WS_ALIGN + u && s < units; ++s) {
                CHECK(owner[s] < 0, "unit %zu handed out twice", s);
                owner[s] = next_id;
            }
            live.push_back({off, bytes, next_id++});
        } else {
            const size_t i = rng() % live.size();
            const Blk b = live[i];
            live.erase(live.begin() + (long)i);
            a.release(b.off, b.bytes);
            for (size_t s = b.off / WS_ALIGN; s < b.off / WS_ALIGN + (b.bytes + WS_ALIGN - 1) / WS_ALIGN; ++s)
                owner[s] = -1;
        }
        size_t used = 0;
        for (int o : owner) used += o >= 0;
        CHECK(a.used() == used * WS_ALIGN, "used bytes %zu vs %zu", a.used(), used * WS_ALIGN);
    }
    for (const Blk& b : live) a.release(b.off, b.bytes);
    CHECK(a.used() == 0 && a.free_blocks() == 1 && a.largest_free() == units * WS_ALIGN, "coalesced when empty");
}

static void check_choose(std::mt19937_64& rng)
{
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int rep = 0; rep < 300; ++rep) {
        std::vector<QueuedShape> q(1 + rng() % 30);
        for (auto& s : q) {
            s.k = 2 + (uint32_t)(rng() % 3);
            s.mode = (int)(rng() % 2);
            s.n = (uint32_t)std::exp(u(rng) * std::log(400000.0));
        }
        if (rep % 3 == 0)
            for (auto& s : q) { s.k = q[0].k; s.mode = q[0].mode; }
        const size_t cap = (size_t)(request_footprint(q[0].n, q[0].k, q[0].mode) * (0.8 + 6.0 * u(rng)));
        ArenaAllocator pool(cap + WS_ALIGN);
        // some resident blocks
        std::vector<std::pair<size_t, size_t>> held;
        for (int j = 0; j < (int)(rng() % 4); ++j) {
            const size_t b = 1 + rng() % (cap / 8 + 1);
            const size_t off = pool.alloc(b);
            if (off != ArenaAllocator::NPOS) held.push_back({off, b});
        }
        const uint32_t maxr = 1 + (uint32_t)(rng() % 12);
        const uint64_t maxp = 1 + rng() % 2000000;
        const BatchChoice c = choose_batch(q, pool, maxr, maxp);
        if (c.picks.empty()) {
            ArenaAllocator t = pool;
            const bool out_ok = t.alloc(batch_output_bytes(q[0].n, q[0].k)) != ArenaAllocator::NPOS;
            const bool ws_ok = out_ok && t.alloc(workspace_bytes_any({q[0].n}, q[0].k, q[0].mode == 1)) !=
                                             ArenaAllocator::NPOS;
            CHECK(!ws_ok, "the oldest request fits but nothing was chosen");
            continue;
        }
        CHECK(c.picks[0] == 0, "the oldest request comes first");
        CHECK(c.picks.size() <= maxr, "request limit");
        uint64_t pts = 0;
        std::vector<uint32_t> n;
        for (size_t j = 0; j < c.picks.size(); ++j) {
            const QueuedShape& s = q[c.picks[j]];
            CHECK(s.k == q[0].k && s.mode == q[0].mode, "one shape per batch");
            if (j) CHECK(c.picks[j] > c.picks[j - 1], "queue order");
            pts += s.n;
            n.push_back(s.n);
        }
        CHECK(c.picks.size() == 1 || pts <= maxp, "point limit");
        CHECK(c.out_bytes == batch_output_bytes(pts, q[0].k), "output block size");
        CHECK(c.ws_bytes == workspace_bytes_any(n, q[0].k, q[0].mode == 1), "workspace size");
        ArenaAllocator t = pool;
        CHECK(t.alloc(c.out_bytes) != ArenaAllocator::NPOS && t.alloc(c.ws_bytes) != ArenaAllocator::NPOS,
              "chosen blocks fit");
        // skipped same-shape requests come only after the last pick, and the
        // next candidate would break a limit or not fit
        size_t next = q.size();
        for (size_t i = 0; i < q.size(); ++i) {
            bool picked = false;
            for (size_t p : c.picks) picked |= p == i;
            if (picked || q[i].k != q[0].k || q[i].mode != q[0].mode) continue;
            CHECK(i > c.picks.back(), "same-shape request %zu skipped before the last pick", i);
            if (next == q.size()) next = i;
        }
        if (next < q.size() && c.picks.size() < maxr && pts + q[next].n <= maxp) {
            std::vector<uint32_t> n2 = n;
            n2.push_back(q[next].n);
            ArenaAllocator t2 = pool;
            const bool fit2 = t2.alloc(batch_output_bytes(pts + q[next].n, q[0].k)) != ArenaAllocator::NPOS &&
                              t2.alloc(workspace_bytes_any(n2, q[0].k, q[0].mode == 1)) != ArenaAllocator::NPOS;
            CHECK(!fit2, "one more request would have fitted");
        }
    }
    // a pool of exactly one request's footprint admits that request alone
    for (uint32_t n : {1u, 100u, 2048u, 2049u, 100000u, 3000000u}) {
        ArenaAllocator pool(request_footprint(n, 3, 0));
        const BatchChoice c = choose_batch({{n, 3, 0}, {n, 3, 0}}, pool, 8, 1ull << 40);
        CHECK(c.picks.size() == 1, "footprint of n=%u admits it alone", n);
    }
}

int main()
{
    std::mt19937_64 rng(7);
    check_arena(rng);
    check_choose(rng);
    if (g_fail) return 1;
    std::printf("ok\n");
    return 0;
}
