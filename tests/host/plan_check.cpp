// Host check of the build planner (kdt_plan.cpp) on random batches: every
// launch's shares tile exactly the work of the trees that take part, the
// histogram, domain-table and workspace ranges never overlap, and the tail
// groups fit one workgroup.  Subtree sizes are counted by walking the
// level-order tree, not taken from the closed forms.
// Prints "ok" and exits 0 on success.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "kdt_layout.h"
#include "kdt_plan.h"

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

// largest subtree among the nodes of level l of an n-node level-order tree
static uint64_t biggest_subtree(uint64_t n, uint32_t l)
{
    uint64_t best = 0;
    const uint64_t first = (1ull << l) - 1;
    for (uint64_t s = first; s < 2 * first + 1 && s < n; ++s) {
        uint64_t c = 0;
        for (uint64_t lo = s, w = 1; lo < n; lo = 2 * lo + 1, w *= 2) {
            const uint64_t hi = lo + w;
            c += (hi < n ? hi : n) - lo;
        }
        if (c > best) best = c;
    }
    return best;
}

// sizes of the subtrees of level l, in level order
static std::vector<uint64_t> subtree_sizes(uint64_t n, uint32_t l)
{
    std::vector<uint64_t> out;
    const uint64_t first = (1ull << l) - 1;
    for (uint64_t s = first; s < 2 * first + 1 && s < n; ++s) {
        uint64_t c = 0;
        for (uint64_t lo = s, w = 1; lo < n; lo = 2 * lo + 1, w *= 2) {
            const uint64_t hi = lo + w;
            c += (hi < n ? hi : n) - lo;
        }
        out.push_back(c);
    }
    return out;
}

static bool disjoint(std::vector<std::pair<uint64_t, uint64_t>> r)
{
    std::sort(r.begin(), r.end());
    for (size_t i = 1; i < r.size(); ++i)
        if (r[i].first < r[i - 1].second) return false;
    return true;
}

static void check_steps_tile(const std::vector<TreeStep>& steps, uint32_t total, const char* what)
{
    uint32_t expect = 0;
    for (size_t i = 0; i < steps.size(); ++i) {
        CHECK(steps[i].tile0 == expect || (i > 0 && steps[i].tile0 >= steps[i - 1].tile0), "%s share %zu", what, i);
        expect = steps[i].tile0;
    }
    CHECK(steps.empty() || steps.back().tile0 < total, "%s last share starts inside", what);
}

static void check_plan(const std::vector<uint32_t>& n, uint32_t k, bool widest, const PlanOptions& opt)
{
    const Plan p = make_plan(n, k, widest, opt);
    const uint32_t T = (uint32_t)n.size();
    // trees back to back
    uint64_t off = 0;
    for (uint32_t t = 0; t < T; ++t) {
        CHECK(p.trees[t].off == off && p.trees[t].n == n[t], "tree %u", t);
        off += n[t];
    }
    CHECK(p.ntotal == off, "ntotal");
    // small / large split
    std::vector<int> role(T, 0);
    for (size_t i = 0; i < p.small.size(); ++i) {
        const TreeStep& s = p.small[i];
        CHECK(s.tile0 == i && s.pair0 == 1 && n[s.tree] >= 1 && n[s.tree] <= TAIL_CAP, "small %zu", i);
        role[s.tree] |= 1;
    }
    for (size_t i = 0; i < p.large.size(); ++i) {
        const uint32_t t = p.large[i];
        CHECK(n[t] > TAIL_CAP && p.trees[t].idx == i, "large %zu", i);
        role[t] |= 2;
    }
    for (uint32_t t = 0; t < T; ++t) CHECK((n[t] == 0) == (role[t] == 0) && role[t] != 3, "role of tree %u", t);
    if (p.large.empty()) {
        CHECK(p.levels.empty() && p.tail.empty() && p.pass_words.empty(), "no passes without large trees");
    } else {
        CHECK(p.P >= 2 && p.RB >= 8 && p.RB <= 10 && p.P * p.RB >= p.B, "digits B=%u RB=%u P=%u", p.B, p.RB, p.P);
        if (opt.radix_bits) CHECK(p.RB == opt.radix_bits, "radix option");
    }
    const uint32_t NB = 1u << p.RB;
    // whole-array steps: contiguous tiles in tree order
    uint32_t pt = 0, st = 0;
    for (size_t i = 0; i < p.large.size(); ++i) {
        const uint32_t t = p.large[i];
        CHECK(p.prep[i].tree == t && p.prep[i].tile0 == pt, "prep %zu", i);
        CHECK(p.level0[i].tree == t && p.level0[i].tile0 == pt, "level0 %zu", i);
        CHECK(p.presort[i].tree == t && p.presort[i].tile0 == st, "presort %zu", i);
        pt += (n[t] + PREP_TILE - 1) / PREP_TILE;
        st += (n[t] + PRESORT_TILE - 1) / PRESORT_TILE;
    }
    CHECK(pt == p.prep_tiles && st == p.presort_tiles, "whole-array tile totals");
    // first tail level against counted subtree sizes
    std::vector<uint32_t> l0(T, 0);
    for (uint32_t t : p.large) {
        const uint32_t L = num_levels(n[t]);
        uint32_t want = 1;
        while (want + 2 <= L && biggest_subtree(n[t], want) > TAIL_CAP) ++want;
        l0[t] = first_tail_level(n[t]);
        CHECK(l0[t] == want && l0[t] >= 1 && l0[t] + 2 <= L, "tail level of n=%u: %u vs %u", n[t], l0[t], want);
    }
    // domain tables
    std::vector<std::pair<uint64_t, uint64_t>> box;
    for (uint32_t t : p.large) {
        const uint32_t b = p.trees[t].box_off;
        CHECK(b + (1u << l0[t]) <= p.box_entries, "box range of tree %u", t);
        box.push_back({b, b + (1ull << l0[t])});
    }
    CHECK(disjoint(box), "box ranges overlap");
    // iterations run as passes
    uint32_t maxl = 0;
    for (uint32_t t : p.large) maxl = l0[t] > maxl ? l0[t] : maxl;
    CHECK(p.levels.size() == (maxl ? maxl - 1 : 0), "level launches %zu", p.levels.size());
    for (size_t li = 0; li < p.levels.size(); ++li) {
        const LevelLaunch& ll = p.levels[li];
        const uint32_t l = (uint32_t)li + 1;
        CHECK(ll.level == l && (ll.items == 4 || ll.items == (uint32_t)PART_ITEMS), "level %u", l);
        CHECK(ll.sorted == (!widest && l % k == 0), "level %u sorted flag", l);
        CHECK(ll.items == 4u || ll.items == (uint32_t)PART_ITEMS, "split tile size");
        if (opt.max_items == 4) CHECK(ll.items == 4u, "small split tiles only");
        std::vector<std::pair<uint64_t, uint64_t>> hist;
        uint32_t tiles = 0, htiles = 0, ptiles = 0, pwords = 0;
        size_t si = 0;
        for (uint32_t t : p.large) {
            if (l >= l0[t]) continue;
            CHECK(si < ll.steps.size(), "level %u misses tree %u", l, t);
            if (si >= ll.steps.size()) break;
            const TreeStep& s = ll.steps[si];
            const TreeStep& h = ll.ssteps[si];
            ++si;
            const Level v = make_level(n[t], l);
            CHECK(s.tree == t && s.level == l && s.tile0 == tiles, "level %u share of tree %u", l, t);
            CHECK(h.tree == t && h.tile0 == htiles && h.hist == s.hist, "select share of tree %u", t);
            const TreeStep& pv = ll.psteps[si - 1];
            CHECK(pv.tree == t && pv.tile0 == ptiles && pv.hist == s.hist && pv.piv == s.piv && s.piv == pwords,
                  "pivot share of tree %u", t);
            ptiles += (v.nseg + PIVOT_SEGS - 1) / PIVOT_SEGS;
            pwords += 2 * v.nseg;
            tiles += tiles_level(v, (uint32_t)SWEEP_THREADS * ll.items).tiles;
            htiles += tiles_level(v, HIST_TILE).tiles;
            const uint64_t lo = (l % 3u) * (uint64_t)p.hist_words, hi = lo + p.hist_words;
            const uint64_t words = (uint64_t)v.nseg * p.P * NB;
            CHECK(s.hist >= lo && s.hist + words <= hi, "hist range of tree %u at level %u", t, l);
            hist.push_back({s.hist, s.hist + words});
            // next iteration's histograms
            if (l + 1 < l0[t]) {
                const LevelLaunch& nx = p.levels[li + 1];
                uint32_t want = NO_HIST;
                for (const TreeStep& s2 : nx.steps)
                    if (s2.tree == t) want = s2.hist;
                CHECK(want != NO_HIST && s.hist_next == want, "hist_next of tree %u at level %u", t, l);
            } else {
                CHECK(s.hist_next == NO_HIST, "no hist_next for tree %u at its last pass level", t);
            }
        }
        CHECK(disjoint(hist), "histogram ranges overlap at level %u", l);
        CHECK(si == ll.steps.size() && ll.ssteps.size() == si, "level %u share count", l);
        CHECK(tiles == ll.tiles && htiles == ll.select_tiles && ptiles == ll.pivot_tiles, "level %u tile totals", l);
        CHECK(pwords == ll.piv_words && pwords <= p.piv_words && ll.psteps.size() == ll.steps.size(),
              "level %u pivot words", l);
        uint32_t hw = 0;
        for (const TreeStep& s : ll.steps) hw += make_level(n[s.tree], l).nseg * p.P * NB;
        CHECK(hw == ll.hist_words && hw <= p.hist_words, "level %u hist words", l);
    }
    for (size_t i = 0; i < p.level0.size(); ++i) {
        const uint32_t t = p.level0[i].tree;
        uint32_t want = NO_HIST;
        if (!p.levels.empty())
            for (const TreeStep& s2 : p.levels[0].steps)
                if (s2.tree == t) want = s2.hist;
        CHECK(p.level0[i].hist_next == want, "level0 hist_next of tree %u", t);
    }
    // tail
    uint32_t groups = 0;
    CHECK(p.tail.size() == p.large.size(), "tail shares");
    for (size_t i = 0; i < p.tail.size() && i < p.large.size(); ++i) {
        const TreeStep& s = p.tail[i];
        const uint32_t t = p.large[i];
        const Level v = make_level(n[t], l0[t]);
        CHECK(s.tree == t && s.level == l0[t] && s.tile0 == groups, "tail share of tree %u", t);
        CHECK(s.pair0 <= v.nseg, "tail pair0 of %u", t);
        CHECK(s.buf == ((l0[t] - 1u) & 1u), "tail buffer of tree %u", t);
        // every workgroup's subtrees fit TAIL_CAP (sizes counted on the
        // tree), every subtree is in exactly one group, and no lone subtree
        // before pair0 could have shared a workgroup
        const uint32_t ng = tail_group_count(v.nseg, s.pair0);
        std::vector<uint64_t> sizes = subtree_sizes(n[t], l0[t]);
        uint32_t covered = 0;
        for (uint32_t gi = 0; gi < ng; ++gi) {
            uint32_t i0, i1;
            tail_group_range(gi, s.pair0, v.nseg, i0, i1);
            CHECK(i0 == covered && i1 > i0 && i1 - i0 <= 2, "tail group %u of tree %u", gi, t);
            uint64_t pts = 0;
            for (uint32_t i = i0; i < i1 && i < sizes.size(); ++i) pts += sizes[i];
            CHECK(pts <= TAIL_CAP, "tail group %u of tree %u holds %llu points", gi, t, (unsigned long long)pts);
            covered = i1;
        }
        CHECK(covered == v.nseg, "tail groups of tree %u cover its subtrees", t);
        for (uint32_t i = 0; i < s.pair0 && i < sizes.size(); ++i)
            CHECK(sizes[i] > TAIL_CAP / 2, "subtree %u of tree %u could pair", i, t);
        groups += ng;
    }
    CHECK(groups == p.tail_groups, "tail groups");
    // look-back words
    // presort: roles in groups of presort_group, each of the 4 passes of a
    // group one launch; with per-role rank arrays the root's role runs alone
    // first and every other role's passes come after all of the root's
    const uint32_t G = p.presort_group;
    CHECK(G == std::min(k, opt.presort_dims ? std::min(opt.presort_dims, PRESORT_GROUP) : PRESORT_GROUP),
          "presort group %u (option %u)", G, opt.presort_dims);
    std::vector<Plan::PresortLaunch> want;
    if (!p.large.empty()) {
        if (p.rank_dm)
            for (uint32_t q = 0; q < 4u; ++q) want.push_back({0u, 1u, q});
        for (uint32_t r0 = p.rank_dm ? 1u : 0u; r0 < k; r0 += G) {
            const uint32_t nd = std::min(G, k - r0);
            for (uint32_t q = 0; q < 4u; ++q) want.push_back({r0, nd, q});
        }
    }
    CHECK(want.size() == p.presort_launches.size(), "presort launch count");
    uint32_t sorted_passes[4] = {0, 0, 0, 0};
    for (size_t i = 0; i < want.size() && i < p.presort_launches.size(); ++i) {
        const Plan::PresortLaunch& a = p.presort_launches[i];
        CHECK(a.role0 == want[i].role0 && a.ndims == want[i].ndims && a.pass == want[i].pass, "presort launch %zu", i);
        CHECK(a.ndims >= 1 && a.ndims <= G && a.role0 + a.ndims <= k, "presort launch shape");
        if (a.role0 > 0 && p.rank_dm) CHECK(sorted_passes[0] == 0xFu, "role %u before the root's passes", a.role0);
        for (uint32_t r = a.role0; r < a.role0 + a.ndims && r < 4; ++r) sorted_passes[r] |= 1u << a.pass;
    }
    for (uint32_t r = 0; r < k && !p.large.empty(); ++r) CHECK(sorted_passes[r] == 0xFu, "role %u passes", r);
    // roles <-> dimensions: a bijection for every root dimension
    for (uint32_t d0 = 0; d0 < k; ++d0) {
        uint32_t seen = 0;
        for (uint32_t r = 0; r < k; ++r) {
            const uint32_t d = role_dim(r, d0);
            CHECK(d < k && dim_role(d, d0) == r, "role %u of root dimension %u", r, d0);
            seen |= 1u << d;
        }
        CHECK(seen == (1u << k) - 1u && role_dim(0, d0) == d0, "roles of root dimension %u", d0);
    }
    // per-XCD presort queues (many trees): every presort tile in exactly one
    // queue, a tree's tiles all in one queue and in order
    CHECK(p.xq == (p.large.size() >= XQ_MIN_TREES && p.presort_launches.size() <= XQ_LAUNCHES), "xq choice");
    if (p.xq) {
        CHECK(p.xq_table.size() == 16 + (size_t)p.presort_tiles, "xq table size");
        std::vector<int> seen(p.presort_tiles, 0);
        std::vector<int> queue_of(p.large.size(), -1);
        std::vector<int64_t> last(p.large.size(), -1);
        for (uint32_t x = 0; x < 8 && p.xq_table.size() >= 16; ++x) {
            const uint32_t off = p.xq_table[x], len = p.xq_table[8 + x];
            CHECK(16 + (size_t)off + len <= p.xq_table.size(), "queue %u bounds", x);
            for (uint32_t i = 0; i < len && 16 + (size_t)off + i < p.xq_table.size(); ++i) {
                const uint32_t g = p.xq_table[16 + off + i];
                if (g >= p.presort_tiles) { CHECK(false, "queue %u tile %u out of range", x, g); continue; }
                seen[g]++;
                size_t tr = 0;
                while (tr + 1 < p.large.size() && p.presort[tr + 1].tile0 <= g) ++tr;
                CHECK(queue_of[tr] < 0 || queue_of[tr] == (int)x, "tree %zu in two queues", tr);
                queue_of[tr] = (int)x;
                CHECK((int64_t)g > last[tr], "tree %zu tiles out of order", tr);
                last[tr] = g;
            }
        }
        for (uint32_t g = 0; g < p.presort_tiles; ++g) CHECK(seen[g] == 1, "tile %u queued %d times", g, seen[g]);
        // iteration 0's XCD map: every prep tile once; workgroup b holds a
        // tile of a tree whose presort queue is b mod 8
        CHECK(p.xmap0.size() % 8 == 0, "xmap0 size");
        std::vector<int> once(p.prep_tiles, 0);
        for (size_t b = 0; b < p.xmap0.size(); ++b) {
            const uint32_t g = p.xmap0[b];
            if (g == 0xFFFFFFFFu) continue;
            if (g >= p.prep_tiles) { CHECK(false, "xmap0 tile %u out of range", g); continue; }
            once[g]++;
            size_t tr = 0;
            while (tr + 1 < p.large.size() && p.level0[tr + 1].tile0 <= g) ++tr;
            CHECK(queue_of[tr] == (int)(b % 8), "xmap0: tree %zu off its XCD", tr);
        }
        for (uint32_t g = 0; g < p.prep_tiles; ++g) CHECK(once[g] == 1, "prep tile %u mapped %d times", g, once[g]);
        // the tail's XCD map: every group once, on its tree's XCD
        CHECK(p.xmapt.size() % 8 == 0, "xmapt size");
        std::vector<int> gonce(p.tail_groups, 0);
        for (size_t b = 0; b < p.xmapt.size(); ++b) {
            const uint32_t g = p.xmapt[b];
            if (g == 0xFFFFFFFFu) continue;
            if (g >= p.tail_groups) { CHECK(false, "xmapt group %u out of range", g); continue; }
            gonce[g]++;
            size_t tr = 0;
            while (tr + 1 < p.tail.size() && p.tail[tr + 1].tile0 <= g) ++tr;
            CHECK(queue_of[tr] == (int)(b % 8), "xmapt: tree %zu off its XCD", tr);
        }
        for (uint32_t g = 0; g < p.tail_groups; ++g) CHECK(gonce[g] == 1, "tail group %u mapped %d times", g, gonce[g]);
    } else {
        CHECK(p.xmap0.empty() && p.xmapt.empty(), "XCD maps without queues");
    }
    const size_t npass = p.presort_launches.size() + p.levels.size();
    CHECK(p.pass_words.size() == npass && npass <= MAX_PASSES, "pass count");
    for (size_t i = 0; i < p.presort_launches.size() && p.pass_words.size() == npass; ++i)
        CHECK(p.pass_words[i] == p.presort_launches[i].ndims * p.presort_tiles * RADIX_HOST, "presort look-back words");
    for (size_t li = 0; li < p.levels.size() && p.pass_words.size() == npass; ++li)
        CHECK(p.pass_words[p.presort_launches.size() + li] == p.levels[li].tiles * PART_BINS,
              "split look-back words of level %zu", li);
    for (uint32_t w : p.pass_words) CHECK(w <= p.lb_words, "look-back words");
    // workspace regions: aligned, in order, disjoint
    const size_t N = p.ntotal;
    struct R { size_t off, bytes; const char* name; } regs[] = {
        {p.o_status, 64, "status"}, {p.o_counters, MAX_COUNTERS * 4, "counters"},
        {p.o_hist_rank, p.large.size() * k * 4 * RADIX_HOST * 4, "hist_rank"},
        {p.o_hist, (size_t)p.hist_words * 12, "hist"}, {p.o_lb[0], (size_t)p.lb_words * 4, "lb0"},
        {p.o_lb[1], (size_t)p.lb_words * 4, "lb1"}, {p.o_keys, N * k * 4, "keys"}, {p.o_perms, N * k * 4, "perms"},
        {p.o_ranks, N * k * 4, "ranks"}, {p.o_rec, std::max(p.rec_words * 2, (size_t)4 * G * N) * 4, "rec"}, {p.o_nodeperm, N * 4, "nodeperm"},
        {p.o_dimnode, N, "dimnode"}, {p.o_box[0], (size_t)p.box_entries * 32, "box0"},
        {p.o_box[1], (size_t)p.box_entries * 32, "box1"}, {p.o_bbox, p.large.size() * KEYSUM_WORDS * 4, "keysum"}, {p.o_piv, (size_t)p.piv_words * 4, "piv"},
        {p.o_tables, p.tables ? p.blob.size() : 0, "tables"}, {p.o_wcount, (size_t)k * RANK_MAX_WIN * 4, "wcount"},
        {p.o_tstatus, p.trees.size() * 4, "tstatus"}};
    size_t end = 0;
    for (const R& r : regs) {
        CHECK(r.off % WS_ALIGN == 0 && r.off >= end, "region %s at %zu (previous end %zu)", r.name, r.off, end);
        end = r.off + r.bytes;
    }
    CHECK(end <= p.total && p.total % WS_ALIGN == 0, "total");
    CHECK(p.rec_words >= N * k && p.rec_words >= 2 * N, "record words");
    // rank layout: per-dimension arrays (in the ranks region) packed into the
    // second record buffer, for k >= 2 only, when forced or when the largest
    // tree's point-major table would exceed RANK_DM_BYTES
    {
        uint64_t nmax = 0;
        for (uint32_t t : p.large) nmax = std::max<uint64_t>(nmax, n[t]);
        const bool want = k >= 2 && !p.large.empty() &&
                          (opt.rank_layout == 2 || (opt.rank_layout == 0 && nmax * k * 4 > RANK_DM_BYTES));
        CHECK(p.rank_dm == want, "rank layout (k %u, layout %u, N %zu)", k, opt.rank_layout, N);
        // windowed scatter: at most RANK_MAX_WIN windows covering every
        // index, each of at most N indices, and the buckets (2 words per
        // pair, 2^wbits pairs per window) inside one dimension's ping-pong
        if (p.rank_dm) {
            const uint64_t W = 1ull << p.rank_wbits;
            CHECK(p.rank_nwin >= 1 && p.rank_nwin <= RANK_MAX_WIN, "window count %u", p.rank_nwin);
            CHECK(W * p.rank_nwin >= N && W * (p.rank_nwin - 1) < N, "windows cover the indices");
            CHECK(W <= N && 2 * W * p.rank_nwin <= 4 * (uint64_t)N, "buckets fit a ping-pong");
        }
    }
    // the uploaded tables hold the host lists
    auto same = [&](size_t at, const void* v, size_t bytes) {
        return at + bytes <= p.blob.size() && (bytes == 0 || std::memcmp(p.blob.data() + at, v, bytes) == 0);
    };
    CHECK(same(p.t_trees, p.trees.data(), p.trees.size() * sizeof(TreeInfo)), "trees table");
    CHECK(same(p.t_small, p.small.data(), p.small.size() * sizeof(TreeStep)), "small table");
    CHECK(same(p.t_tail, p.tail.data(), p.tail.size() * sizeof(TreeStep)), "tail table");
    for (size_t li = 0; li < p.levels.size(); ++li) {
        CHECK(same(p.t_level[li], p.levels[li].steps.data(), p.levels[li].steps.size() * sizeof(TreeStep)),
              "level table %zu", li);
        CHECK(same(p.t_select[li], p.levels[li].ssteps.data(), p.levels[li].ssteps.size() * sizeof(TreeStep)),
              "select table %zu", li);
        CHECK(same(p.t_pivot[li], p.levels[li].psteps.data(), p.levels[li].psteps.size() * sizeof(TreeStep)),
              "pivot table %zu", li);
    }
    CHECK(p.tables == (p.small.size() > 1 || p.large.size() > 1), "table flag");
    check_steps_tile(p.small, (uint32_t)p.small.size(), "small");
}

int main()
{
    std::mt19937_64 rng(12345);
    // single trees around every tail boundary
    for (uint32_t n : {0u, 1u, 2u, 3u, 2047u, 2048u, 2049u, 4095u, 4096u, 4097u, 8191u, 65537u, 1000000u,
                       10000000u, 100000000u}) {
        for (uint32_t k = 1; k <= 4; ++k) {
            check_plan({n}, k, false, PlanOptions());
            check_plan({n}, k, true, PlanOptions());
        }
    }
    // random batches with log-uniform sizes, empty and tiny clouds mixed in
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int rep = 0; rep < 60; ++rep) {
        const uint32_t C = 1 + (uint32_t)(u(rng) * (rep < 50 ? 40 : 600));
        const double hi = rep % 3 == 0 ? 2.0e6 : 3.0e5;
        std::vector<uint32_t> n(C);
        for (uint32_t c = 0; c < C; ++c) {
            const double r = u(rng);
            n[c] = r < 0.05 ? 0u : (uint32_t)std::exp(std::log(1.0) + u(rng) * std::log(hi));
        }
        PlanOptions opt;
        if (rep % 4 == 1) opt.radix_bits = 8 + (uint32_t)(u(rng) * 3);
        if (rep % 5 == 2) opt.max_items = 4;
        opt.rank_layout = rep % 3;
        opt.presort_dims = rep % 5;
        check_plan(n, 1 + rep % 4, rep % 2 == 1, opt);
    }
    if (g_fail) return 1;
    std::printf("ok\n");
    return 0;
}
