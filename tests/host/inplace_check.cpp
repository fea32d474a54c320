// Host check of the in-place build's arithmetic (kdt_inplace.h) against
// direct enumeration of the level-order tree:
//   - io_begin / io_pivot / seg_size against an in-order traversal of the tree;
//   - inorder_to_level against the same traversal;
//   - the swap-only op list of plan_to_level_order, replayed on the host,
//     takes the in-order sequence of node indices to 0, 1, ..., n-1;
//   - the bitonic pass schedule of plan_level_sort, with the pair and group
//     index helpers, sorts random keys of every length up to a few blocks,
//     padding never stored;
//   - the group index helpers enumerate every position exactly once.
// Prints "ok" and exits 0 on success.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "kdt_inplace.h"

using namespace kdt;
using namespace kdt::ip;

static int fails = 0;
#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            std::printf("FAIL " __VA_ARGS__); \
            std::printf("\n");                \
            if (++fails > 20) std::exit(1);   \
        }                                     \
    } while (0)

// In-order traversal of the level-order tree of n nodes: order[p] = node at
// in-order position p; first[s] = in-order position of the leftmost node of
// s's subtree; size[s] = nodes under s.
struct Traversal {
    std::vector<uint32_t> order, pos, first, size;
};

static Traversal traverse(uint32_t n)
{
    Traversal t;
    t.pos.assign(n, 0);
    t.first.assign(n, 0);
    t.size.assign(n, 0);
    // iterative in-order walk
    std::vector<uint32_t> st;
    uint32_t x = 0;
    while ((x < n) || !st.empty()) {
        while (x < n) {
            st.push_back(x);
            x = 2 * x + 1;
        }
        x = st.back();
        st.pop_back();
        t.pos[x] = (uint32_t)t.order.size();
        t.order.push_back(x);
        x = 2 * x + 2;
    }
    for (int64_t s = (int64_t)n - 1; s >= 0; --s) {
        uint32_t sz = 1, f = t.pos[s];
        const uint64_t a = 2 * (uint64_t)s + 1, b = a + 1;
        if (a < n) {
            sz += t.size[a];
            f = t.first[a];
        }
        if (b < n) sz += t.size[b];
        t.size[s] = sz;
        t.first[s] = f;
    }
    return t;
}

static void check_layout(uint32_t n)
{
    const Traversal t = traverse(n);
    const uint32_t L = num_levels(n);
    for (uint32_t l = 0; l < L; ++l) {
        const Level v = make_level(n, l);
        for (uint32_t i = 0; i < v.nseg; ++i) {
            const uint64_t s = (uint64_t)v.Fl + i;
            if (s >= n) break;
            CHECK(io_begin(v, i) == t.first[s], "io_begin n=%u l=%u i=%u", n, l, i);
            CHECK(seg_size(v, i) == t.size[s], "seg_size n=%u l=%u i=%u", n, l, i);
            if (l + 2 <= L) CHECK(io_pivot(v, i) == t.pos[s], "io_pivot n=%u l=%u i=%u", n, l, i);
        }
        if (l + 2 <= L) {
            // io_seg_of inverts io_begin: every position of a subtree's range maps to it,
            // the nodes of the levels above to 0xFFFFFFFF
            std::vector<uint32_t> want(n, 0xFFFFFFFFu);
            for (uint32_t i = 0; i < v.nseg; ++i)
                for (uint32_t p = io_begin(v, i); p < io_begin(v, i) + seg_size(v, i); ++p) want[p] = i;
            for (uint32_t p = 0; p < n; ++p) CHECK(io_seg_of(v, p) == want[p], "io_seg_of n=%u l=%u p=%u", n, l, p);
        }
        if (l + 2 <= L) {
            uint32_t mx = 0;
            for (uint32_t i = 0; i < v.nseg; ++i) mx = std::max(mx, seg_size(v, i));
            CHECK(mx == seg_size(v, 0), "largest subtree is subtree 0, n=%u l=%u", n, l);
            CHECK(net_len(v) >= mx && net_len(v) < 2 * mx + 1, "net_len n=%u l=%u", n, l);
        }
    }
    const uint32_t lg = deep_level(L);
    if (lg + 1 <= L) {
        const Level v = make_level(n, lg);
        for (uint32_t i = 0; i < v.nseg && (uint64_t)v.Fl + i < n; ++i)
            CHECK(seg_size(v, i) < BLK, "deep subtree fits a block n=%u i=%u", n, i);
    }
    for (uint32_t p = 0; p < n; ++p) CHECK(inorder_to_level(p, n) == t.order[p], "inorder_to_level n=%u p=%u", n, p);
}

// Replay the op list of plan_to_level_order on the in-order sequence.
static void check_ops(uint32_t n)
{
    const Traversal t = traverse(n);
    std::vector<uint32_t> a = t.order;
    std::vector<uint32_t> tmp;
    plan_to_level_order(n, [&](const Op& o) {
        switch (o.kind) {
        case OP_UNSHUF_LDS:
            CHECK((uint64_t)o.a + o.n <= n, "unshuffle range n=%u", n);
            for (uint32_t b = 0; b < op_work(o); ++b) {
                const uint32_t b0 = o.a + b * BLK, cnt = std::min(BLK, o.n - b * BLK);
                tmp.assign(cnt, 0);
                for (uint32_t j = 0; j < cnt; ++j) tmp[(j & 1) ? (j >> 1) : (cnt >> 1) + (j >> 1)] = a[b0 + j];
                std::copy(tmp.begin(), tmp.end(), a.begin() + b0);
            }
            break;
        case OP_SWAP_LEVEL: {
            const uint32_t Q = 1u << (o.j - 2);
            for (uint32_t g = 0; g < op_work(o); ++g) {
                const uint32_t x = o.a + ((g >> (o.j - 2)) << o.j) + Q + (g & (Q - 1));
                CHECK((uint64_t)x + Q < n && x + Q < o.a + o.n, "swap level in range n=%u", n);
                std::swap(a[x], a[x + Q]);
            }
            break;
        }
        case OP_REVERSE:
            CHECK((uint64_t)o.a + o.n <= n, "reverse range n=%u", n);
            for (uint32_t g = 0; g < op_work(o); ++g) std::swap(a[o.a + g], a[o.a + o.n - 1 - g]);
            break;
        default:
            CHECK(o.a == 0 && o.n <= BLK && o.n <= n, "lds tree op n=%u", n);
            tmp.assign(o.n, 0);
            for (uint32_t j = 0; j < o.n; ++j) tmp[inorder_to_level(j, o.n)] = a[j];
            std::copy(tmp.begin(), tmp.end(), a.begin());
            break;
        }
    });
    for (uint32_t s = 0; s < n; ++s) CHECK(a[s] == s, "level order after ops n=%u s=%u got %u", n, s, a[s]);
}

// The pass schedule of one iteration's sort on one subtree of `len`
// entries, network length P = 2^logP >= len.
static void cmpx(std::vector<uint64_t>& k, uint32_t lo, uint32_t hi)
{
    if (k[lo] > k[hi]) std::swap(k[lo], k[hi]);
}

static void block_pass(std::vector<uint64_t>& k, uint32_t len, bool sort)
{
    for (uint32_t u = 0; u * SBLK < len; ++u) {
        const uint32_t base = u * SBLK, cnt = std::min(SBLK, len - base);
        for (uint32_t e = sort ? 1u : SBLK_LOG; e <= SBLK_LOG; ++e)
            for (int ls = (int)e - 1; ls >= 0; --ls)
                for (uint32_t q = 0; q < SBLK / 2; ++q) {
                    uint32_t lo, hi;
                    if (sort && ls == (int)e - 1)
                        mirror_pair(q, e, lo, hi);
                    else
                        half_pair(q, (uint32_t)ls, lo, hi);
                    if (hi < cnt) cmpx(k, base + lo, base + hi);
                }
    }
}

static void check_sort(uint32_t len, uint32_t logP, std::mt19937_64& rng)
{
    std::vector<uint64_t> k(len);
    for (uint32_t i = 0; i < len; ++i) k[i] = ((rng() % 7) << 32) | i;   // heavy key ties, unique ids
    std::shuffle(k.begin(), k.end(), rng);
    plan_level_sort(logP, [&](const Step& x) {
        switch (x.kind) {
        case ST_BLOCK_SORT: block_pass(k, len, true); break;
        case ST_BLOCK_MERGE: block_pass(k, len, false); break;
        case ST_MGROUP: {
            // the mirrored stride on two groups per thread, then half-cleaners inside each
            CHECK(x.c >= 1 && x.c <= MGROUP_MAX && x.e0 == x.e - x.c && x.e0 >= SBLK_LOG, "mgroup step e=%u", x.e);
            const uint32_t G = 1u << x.c;
            for (uint32_t h = 0; h < (1u << (logP - x.c - 1)); ++h) {
                const uint32_t ba = mgroup_base(h, x.e0, x.c), bb = ba ^ ((1u << x.e0) - 1u);
                if (ba >= len) continue;
                auto pos = [&](uint32_t j) { return group_pos(j < G ? ba : bb, j & (G - 1), x.e0); };
                auto cx = [&](uint32_t a, uint32_t b) {
                    if (pos(b) < len) cmpx(k, pos(a), pos(b));
                };
                for (uint32_t xx = 0; xx < G; ++xx) {
                    const uint32_t a = xx, b = G + (G - 1 - xx);
                    CHECK(pos(a) + pos(b) + 1 == 2 * ((pos(a) >> x.e) << x.e) + (1u << x.e), "mirror pair e=%u", x.e);
                    if (xx >> (x.c - 1)) cx(b, a);
                    else cx(a, b);
                }
                for (int sb = (int)x.c - 2; sb >= 0; --sb)
                    for (uint32_t half = 0; half < 2 * G; half += G)
                        for (uint32_t p = 0; p < G / 2; ++p) {
                            const uint32_t xx = ((p >> sb) << (sb + 1)) | (p & ((1u << sb) - 1));
                            cx(half + xx, half + (xx | (1u << sb)));
                        }
            }
            break;
        }
        default: {
            CHECK(x.c >= 1 && x.c <= GROUP_MAX && x.e0 >= SBLK_LOG && x.e0 + x.c <= x.e - 1, "group step e=%u", x.e);
            for (uint32_t h = 0; h < (1u << (logP - x.c)); ++h) {
                const uint32_t gb = group_base(h, x.e0, x.c);
                if (gb >= len) continue;
                for (int sb = (int)x.c - 1; sb >= 0; --sb)
                    for (uint32_t p = 0; p < (1u << (x.c - 1)); ++p) {
                        const uint32_t xx = ((p >> sb) << (sb + 1)) | (p & ((1u << sb) - 1));
                        const uint32_t lo = group_pos(gb, xx, x.e0), hi = group_pos(gb, xx | (1u << sb), x.e0);
                        if (hi < len) cmpx(k, lo, hi);
                    }
            }
        }
        }
    });
    CHECK(std::is_sorted(k.begin(), k.end()), "sort schedule len=%u logP=%u", len, logP);
}

static void check_groups()
{
    // mirrored group pairs: every position exactly once over both groups of every pair
    for (uint32_t logP = 3; logP <= 16; ++logP)
        for (uint32_t c = 1; c <= MGROUP_MAX; ++c)
            for (uint32_t e0 = 1; e0 + c <= logP; ++e0) {
                std::vector<uint8_t> seen(1u << logP, 0);
                for (uint32_t h = 0; h < (1u << (logP - c - 1)); ++h) {
                    const uint32_t ba = mgroup_base(h, e0, c), bb = ba ^ ((1u << e0) - 1u);
                    for (uint32_t x = 0; x < (1u << c); ++x)
                        for (uint32_t b : {ba, bb}) {
                            const uint32_t r = group_pos(b, x, e0);
                            CHECK(r < (1u << logP) && !seen[r], "mgroup positions logP=%u c=%u e0=%u", logP, c, e0);
                            if (r < (1u << logP)) seen[r] = 1;
                        }
                }
            }
    for (uint32_t logP = 2; logP <= 16; ++logP)
        for (uint32_t c = 1; c <= GROUP_MAX && c <= logP; ++c)
            for (uint32_t e0 = 0; e0 + c <= logP; ++e0) {
                std::vector<uint8_t> seen(1u << logP, 0);
                for (uint32_t h = 0; h < (1u << (logP - c)); ++h)
                    for (uint32_t x = 0; x < (1u << c); ++x) {
                        const uint32_t r = group_pos(group_base(h, e0, c), x, e0);
                        CHECK(r < (1u << logP) && !seen[r], "group positions logP=%u c=%u e0=%u", logP, c, e0);
                        if (r < (1u << logP)) seen[r] = 1;
                    }
            }
}

int main()
{
    for (uint32_t n = 1; n <= 5000; ++n) {
        check_layout(n);
        check_ops(n);
    }
    std::mt19937_64 rng(12345);
    for (int it = 0; it < 40; ++it) {
        const uint32_t n = 5000 + (uint32_t)(rng() % 300000);
        check_layout(n);
        check_ops(n);
    }
    for (uint32_t n : {8191u, 8192u, 8193u, 16383u, 16384u, 65535u, 65536u, 65537u, 262143u, 262144u, 1048575u,
                       1048576u, 1048577u}) {
        check_layout(n);
        check_ops(n);
    }
    check_groups();
    for (uint32_t q = 0; q < (1u << 16); q += 7)
        for (uint32_t ls = 0; ls < 12; ++ls) {
            uint32_t lo, hi;
            half_pair(q, ls, lo, hi);
            const uint32_t st = 1u << ls;
            CHECK(lo == (q / st) * 2 * st + q % st && hi == lo + st, "half_pair q=%u ls=%u", q, ls);
        }
    for (uint32_t len : {1u, 2u, 3u, 100u, 2047u, 2048u, 2049u, 3000u, 4095u, 4096u, 4097u, 8191u, 8192u, 8193u,
                         9000u, 16384u, 20000u, 40000u, 65536u, 70001u, 131073u})
        check_sort(len, log2_exact(ceil_pow2(len)), rng);
    for (int it = 0; it < 10; ++it) {
        const uint32_t len = 1 + (uint32_t)(rng() % 100000);
        check_sort(len, log2_exact(ceil_pow2(len)), rng);
        check_sort(len, log2_exact(ceil_pow2(len)) + 1, rng);      // a longer network than needed
    }
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
