// kdt_plan.cpp -- host planner of a build call (see kdt_plan.h).
#include "kdt_plan.h"

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "kdt_layout.h"

namespace kdt {

namespace {

// Records per thread of an iteration's split tiles (tile = SWEEP_THREADS * items): the
// largest tile, up to `cap` records per thread, that the iteration's biggest
// subtree still fills.
uint32_t level_items(uint32_t big, uint32_t cap)
{
    const uint32_t large = cap == (uint32_t)PART_ITEMS ? (uint32_t)PART_ITEMS : 4u;
    return big >= (uint32_t)SWEEP_THREADS * large ? large : 4u;
}

TreeStep step(uint32_t tree, uint32_t level, uint32_t tile0)
{
    TreeStep s{};
    s.tree = tree;
    s.level = level;
    s.tile0 = tile0;
    s.hist = 0;
    s.hist_next = NO_HIST;
    s.pair0 = 0;
    s.buf = 0;
    s.piv = 0;
    return s;
}

size_t push_table(std::vector<uint8_t>& blob, const void* p, size_t bytes)
{
    const size_t at = blob.size();
    blob.resize(align_up(at + bytes));
    if (bytes) memcpy(blob.data() + at, p, bytes);
    return at;
}

std::mutex g_tune_mu;
std::map<std::tuple<uint32_t, bool, uint32_t>, PlanOptions> g_tune;

}  // namespace

std::vector<PlanOptions> tuning_candidates()
{
    std::vector<PlanOptions> c;
    for (uint32_t rb : {8u, 9u, 10u})
        for (uint32_t items : {4u, (uint32_t)PART_ITEMS})
            for (uint32_t dims : {1u, PRESORT_GROUP}) {
                PlanOptions o;
                o.radix_bits = rb;
                o.max_items = items;
                o.presort_dims = dims;
                c.push_back(o);
            }
    return c;
}

PlanOptions tuned_options(uint32_t k, bool widest, uint32_t bits)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(k, widest, bits));
    return it == g_tune.end() ? PlanOptions() : it->second;
}

void set_tuned_options(uint32_t k, bool widest, uint32_t bits, const PlanOptions& o)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(k, widest, bits)] = o;
}

void clear_tuning()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

// One line per entry: "k widest bits radix_bits max_items rank_layout presort_dims".
bool save_tuning(const char* path)
{
    FILE* f = fopen(path, "w");
    if (!f) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune)
        fprintf(f, "%u %d %u %u %u %u %u\n", std::get<0>(kv.first), std::get<1>(kv.first) ? 1 : 0,
                std::get<2>(kv.first), kv.second.radix_bits, kv.second.max_items, kv.second.rank_layout,
                kv.second.presort_dims);
    return fclose(f) == 0;
}

bool load_tuning(const char* path)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    std::map<std::tuple<uint32_t, bool, uint32_t>, PlanOptions> t;
    unsigned k, w, bits, rb, items, layout, dims;
    int r;
    bool ok = true;
    while ((r = fscanf(f, "%u %u %u %u %u %u %u", &k, &w, &bits, &rb, &items, &layout, &dims)) == 7) {
        if (k < 1 || k > 4 || w > 1 || bits > 32 || (rb && (rb < 8 || rb > 10)) || (items && items != 4 && items != (unsigned)PART_ITEMS) ||
            layout > 2 || dims > 4) {
            ok = false;
            break;
        }
        PlanOptions o;
        o.radix_bits = rb;
        o.max_items = items;
        o.rank_layout = layout;
        o.presort_dims = dims;
        t[std::make_tuple((uint32_t)k, w == 1u, (uint32_t)bits)] = o;
    }
    if (r != EOF) ok = false;
    fclose(f);
    if (!ok) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : t) g_tune[kv.first] = kv.second;
    return true;
}

uint32_t plan_rank_bits(const std::vector<uint32_t>& n)
{
    uint32_t b = 0;
    for (uint32_t x : n)
        if (x > TAIL_CAP) b = std::max(b, rank_bits(x));
    return b;
}

size_t workspace_bytes_any(const std::vector<uint32_t>& n, uint32_t k, bool widest)
{
    size_t b = 0;
    PlanOptions automatic;
    automatic.radix_bits = 0;
    automatic.max_items = 0;
    for (const PlanOptions& o : tuning_candidates()) b = std::max(b, make_plan(n, k, widest, o).total);
    return std::max(b, make_plan(n, k, widest, automatic).total);
}

uint32_t first_tail_level(uint32_t n)
{
    // the first subtree of a level is its largest; subtrees of level L-2
    // hold at most 3 points, so for n > TAIL_CAP the result is in 1 .. L-2
    const uint32_t L = num_levels(n);
    uint32_t l = 1;
    while (l + 2 <= L && seg_size(make_level(n, l), 0) > TAIL_CAP) ++l;
    return l;
}

Plan make_plan(const std::vector<uint32_t>& n, uint32_t k, bool widest, const PlanOptions& given)
{
    const PlanOptions opt =
        (given.radix_bits || given.max_items || given.rank_layout || given.presort_dims)
            ? given
            : tuned_options(k, widest, plan_rank_bits(n));
    Plan p;
    p.k = k;
    p.widest = widest;
    const uint32_t T = (uint32_t)n.size();
    p.trees.resize(T);
    uint64_t off = 0;
    for (uint32_t t = 0; t < T; ++t) {
        p.trees[t] = TreeInfo{(uint32_t)off, n[t], 0u, 0u};
        off += n[t];
    }
    p.ntotal = off;

    for (uint32_t t = 0; t < T; ++t) {
        if (n[t] == 0) continue;
        if (n[t] <= TAIL_CAP) {
            TreeStep s = step(t, 0u, (uint32_t)p.small.size());
            s.pair0 = 1;
            p.small.push_back(s);
        } else {
            p.trees[t].idx = (uint32_t)p.large.size();
            p.large.push_back(t);
        }
    }

    // digit width of the pivot selects: fewest digits over the largest rank
    // with 8..10-bit digits, then the narrowest digit that keeps that count
    // (a tree of more than TAIL_CAP points has ranks of >= 12 bits, so P >= 2)
    for (uint32_t t : p.large) p.B = std::max(p.B, rank_bits(n[t]));
    if (p.B) {
        const uint32_t pmin = (p.B + 9u) / 10u;
        p.RB = 10;
        for (uint32_t rb = 8; rb <= 10; ++rb)
            if ((p.B + rb - 1u) / rb == pmin) {
                p.RB = rb;
                break;
            }
        if (opt.radix_bits >= 8 && opt.radix_bits <= 10) p.RB = opt.radix_bits;
        p.P = (p.B + p.RB - 1u) / p.RB;
    }
    const uint32_t items_cap = opt.max_items == 4u ? 4u : (uint32_t)PART_ITEMS;
    // rank table layout (k = 1 scatters nothing: the only dimension is the
    // root's); the tiles of one tree run together, so the largest tree's
    // table is what the scatters of a pass spread over
    uint32_t nmax = 0;
    for (uint32_t t : p.large) nmax = std::max(nmax, n[t]);
    p.rank_dm = k >= 2 && !p.large.empty() &&
                (opt.rank_layout == 2 || (opt.rank_layout == 0 && (uint64_t)nmax * k * 4 > RANK_DM_BYTES));
    if (p.rank_dm) {
        // windows of 2^RANK_WIN_BITS indices (2^wbits: at most RANK_MAX_WIN of them,
        // and at most ntotal indices each, so that the buckets fit the
        // 4 * ntotal words of a dimension's ping-pong)
        uint32_t lg = 0, fl = 0;
        while ((1ull << lg) < p.ntotal) ++lg;
        while ((2ull << fl) <= p.ntotal) ++fl;
        uint32_t wb = std::max<uint32_t>(RANK_WIN_BITS, lg > 11u ? lg - 11u : 0u);
        wb = std::min(wb, fl);
        p.rank_wbits = wb;
        p.rank_nwin = (uint32_t)((p.ntotal + (1ull << wb) - 1) >> wb);
    }
    const uint32_t NB = 1u << p.RB;

    // per-tree shares of the whole-array steps
    std::vector<uint32_t> l0(T, 0);
    uint32_t maxl = 0;
    for (uint32_t t : p.large) {
        TreeInfo& ti = p.trees[t];
        l0[t] = first_tail_level(ti.n);
        maxl = std::max(maxl, l0[t]);
        ti.box_off = p.box_entries;
        p.box_entries += 1u << l0[t];     // subtrees of the deepest iteration with a domain table
        p.prep.push_back(step(t, 0u, p.prep_tiles));
        p.level0.push_back(step(t, 0u, p.prep_tiles));
        p.prep_tiles += ceil_div(ti.n, PREP_TILE);
        p.presort.push_back(step(t, 0u, p.presort_tiles));
        p.presort_tiles += ceil_div(ti.n, PRESORT_TILE);
        p.roots.push_back(step(t, 0u, 0u));
    }

    // iterations 1 .. run as digit passes (tree t takes part while l < l0[t]);
    // every segment stays in the root dimension's order, which for round
    // robin is dimension 0
    for (uint32_t l = 1; l < maxl; ++l) {
        LevelLaunch ll;
        ll.level = l;
        ll.sorted = !widest && l % k == 0;
        uint32_t big = 0;
        for (uint32_t t : p.large)
            if (l < l0[t]) big = std::max(big, seg_size(make_level(n[t], l), 0));
        ll.items = level_items(big, items_cap);
        for (uint32_t t : p.large) {
            if (l >= l0[t]) continue;
            const Level v = make_level(n[t], l);
            TreeStep s = step(t, l, ll.tiles);
            s.hist = ll.hist_words;
            s.piv = ll.piv_words;
            ll.tiles += tiles_level(v, (uint32_t)SWEEP_THREADS * ll.items).tiles;
            ll.hist_words += v.nseg * p.P * NB;
            ll.steps.push_back(s);
            TreeStep h = step(t, l, ll.select_tiles);
            ll.select_tiles += tiles_level(v, HIST_TILE).tiles;
            ll.ssteps.push_back(h);
            TreeStep pv = step(t, l, ll.pivot_tiles);
            pv.piv = ll.piv_words;
            ll.pivot_tiles += ceil_div(v.nseg, PIVOT_SEGS);
            ll.piv_words += 2u * v.nseg;
            ll.psteps.push_back(pv);
        }
        p.hist_words = std::max(p.hist_words, ll.hist_words);
        p.levels.push_back(std::move(ll));
    }
    // iteration l's histograms live in third (l mod 3) of the histogram region
    for (LevelLaunch& ll : p.levels) {
        const uint32_t base = (ll.level % 3u) * p.hist_words;
        for (size_t i = 0; i < ll.steps.size(); ++i) {
            ll.steps[i].hist += base;
            ll.ssteps[i].hist = ll.steps[i].hist;
            ll.psteps[i].hist = ll.steps[i].hist;
        }
        p.piv_words = std::max(p.piv_words, ll.piv_words);
    }
    // each share's histogram offset for the next iteration
    auto next_hist = [&](size_t li, uint32_t tree) {
        if (li >= p.levels.size()) return NO_HIST;
        for (const TreeStep& s : p.levels[li].steps)
            if (s.tree == tree) return s.hist;
        return NO_HIST;
    };
    for (size_t li = 0; li < p.levels.size(); ++li)
        for (TreeStep& s : p.levels[li].steps) s.hist_next = next_hist(li + 1, s.tree);
    for (TreeStep& s : p.level0) s.hist_next = next_hist(0, s.tree);

    // the tail of every large tree from its own first tail iteration; each
    // iteration's split flips the record buffer
    // (subtree sizes never grow with the index, so the subtrees that fit
    // two to a workgroup are a suffix)
    for (uint32_t t : p.large) {
        const Level v = make_level(n[t], l0[t]);
        // sizes: 2W-1 below a = R/W, then one of W-1 + R%W, then W-1
        const uint32_t half = TAIL_CAP / 2u, a = v.R / v.W;
        uint32_t pair0 = v.nseg;
        if (seg_size(v, 0) <= half) pair0 = 0;
        else if (a < v.nseg && seg_size(v, a) <= half) pair0 = a;
        else if (a + 1u < v.nseg && seg_size(v, a + 1u) <= half) pair0 = a + 1u;
        TreeStep s = step(t, l0[t], p.tail_groups);
        s.pair0 = pair0;
        s.buf = (l0[t] - 1u) & 1u;
        p.tail.push_back(s);
        p.tail_groups += tail_group_count(v.nseg, pair0);
    }

    // look-back words per pass, in the order the passes run
    // presort launches: roles in groups whose 4 passes share a launch each;
    // with per-role rank arrays the root's role runs alone first (the other
    // roles read its ranks as payloads), and each group's last pass is
    // followed by the windowed scatter of its ranks
    p.presort_group = std::min(k, opt.presort_dims ? std::min(opt.presort_dims, PRESORT_GROUP) : PRESORT_GROUP);
    if (!p.large.empty()) {
        if (p.rank_dm)
            for (uint32_t q = 0; q < 4u; ++q) p.presort_launches.push_back({0u, 1u, q});
        for (uint32_t r0 = p.rank_dm ? 1u : 0u; r0 < k; r0 += p.presort_group) {
            const uint32_t nd = std::min(p.presort_group, k - r0);
            for (uint32_t q = 0; q < 4u; ++q) p.presort_launches.push_back({r0, nd, q});
        }
    }
    for (const Plan::PresortLaunch& pl : p.presort_launches)
        p.pass_words.push_back(pl.ndims * p.presort_tiles * RADIX_HOST);

    // per-XCD presort tile queues: trees to the queue with the fewest tiles
    // so far, largest first; each queue lists its trees' tiles in tree order
    p.xq = p.large.size() >= XQ_MIN_TREES && p.presort_launches.size() <= XQ_LAUNCHES;
    if (p.xq) {
        std::vector<uint32_t> order(p.large.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (uint32_t)i;
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t x, uint32_t y) { return n[p.large[x]] > n[p.large[y]]; });
        std::vector<std::vector<uint32_t>> qs(8);
        uint64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        std::vector<uint32_t> owner(p.large.size());
        for (uint32_t i : order) {
            const uint32_t x = (uint32_t)(std::min_element(load, load + 8) - load);
            owner[i] = x;
            load[x] += ceil_div(n[p.large[i]], PRESORT_TILE);
        }
        for (size_t i = 0; i < p.large.size(); ++i) {
            const TreeStep& s = p.presort[i];
            const uint32_t nt = ceil_div(n[p.large[i]], PRESORT_TILE);
            for (uint32_t g = 0; g < nt; ++g) qs[owner[i]].push_back(s.tile0 + g);
        }
        p.xq_table.assign(16, 0u);
        for (uint32_t x = 0; x < 8; ++x) {
            p.xq_table[x] = (uint32_t)(p.xq_table.size() - 16);
            p.xq_table[8 + x] = (uint32_t)qs[x].size();
            p.xq_table.insert(p.xq_table.end(), qs[x].begin(), qs[x].end());
        }
        // static launches (iteration 0, tail): workgroup b runs on XCD b mod
        // 8 and takes the (b / 8)-th tile of that XCD's trees; tree i owns
        // tiles first[i] .. first[i] + count[i] - 1; padding entries are empty
        auto xcd_map = [&](const std::vector<uint32_t>& first, const std::vector<uint32_t>& count) {
            std::vector<std::vector<uint32_t>> ls(8);
            for (size_t i = 0; i < p.large.size(); ++i)
                for (uint32_t g = 0; g < count[i]; ++g) ls[owner[i]].push_back(first[i] + g);
            size_t longest = 0;
            for (const auto& l : ls) longest = std::max(longest, l.size());
            std::vector<uint32_t> m(8 * longest, 0xFFFFFFFFu);
            for (uint32_t x = 0; x < 8; ++x)
                for (size_t j = 0; j < ls[x].size(); ++j) m[8 * j + x] = ls[x][j];
            return m;
        };
        std::vector<uint32_t> first(p.large.size()), count(p.large.size());
        for (size_t i = 0; i < p.large.size(); ++i) {
            first[i] = p.level0[i].tile0;
            count[i] = ceil_div(n[p.large[i]], PREP_TILE);
        }
        p.xmap0 = xcd_map(first, count);
        for (size_t i = 0; i < p.large.size(); ++i) {
            first[i] = p.tail[i].tile0;
            count[i] = tail_group_count(make_level(n[p.large[i]], p.tail[i].level).nseg, p.tail[i].pair0);
        }
        p.xmapt = xcd_map(first, count);
    }
    for (const LevelLaunch& ll : p.levels) p.pass_words.push_back(ll.tiles * PART_BINS);
    for (uint32_t w : p.pass_words) p.lb_words = std::max(p.lb_words, w);

    // share tables
    p.t_trees = push_table(p.blob, p.trees.data(), p.trees.size() * sizeof(TreeInfo));
    p.t_small = push_table(p.blob, p.small.data(), p.small.size() * sizeof(TreeStep));
    p.t_prep = push_table(p.blob, p.prep.data(), p.prep.size() * sizeof(TreeStep));
    p.t_presort = push_table(p.blob, p.presort.data(), p.presort.size() * sizeof(TreeStep));
    p.t_xq = push_table(p.blob, p.xq_table.data(), p.xq_table.size() * 4);
    p.t_xmap0 = push_table(p.blob, p.xmap0.data(), p.xmap0.size() * 4);
    p.t_xmapt = push_table(p.blob, p.xmapt.data(), p.xmapt.size() * 4);
    p.t_level0 = push_table(p.blob, p.level0.data(), p.level0.size() * sizeof(TreeStep));
    p.t_tail = push_table(p.blob, p.tail.data(), p.tail.size() * sizeof(TreeStep));
    p.t_roots = push_table(p.blob, p.roots.data(), p.roots.size() * sizeof(TreeStep));
    p.tables = p.small.size() > 1 || p.large.size() > 1;
    for (const LevelLaunch& ll : p.levels) {
        p.t_level.push_back(push_table(p.blob, ll.steps.data(), ll.steps.size() * sizeof(TreeStep)));
        p.t_select.push_back(push_table(p.blob, ll.ssteps.data(), ll.ssteps.size() * sizeof(TreeStep)));
        p.t_pivot.push_back(push_table(p.blob, ll.psteps.data(), ll.psteps.size() * sizeof(TreeStep)));
    }

    // workspace
    const size_t N = p.ntotal;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + bytes);
        return r;
    };
    p.o_status = take(64);
    p.o_counters = take(MAX_COUNTERS * 4);
    p.o_hist_rank = take((size_t)p.large.size() * k * 4 * RADIX_HOST * 4);
    p.o_hist = take((size_t)p.hist_words * 3 * 4);
    p.o_lb[0] = take((size_t)p.lb_words * 4);
    p.o_lb[1] = take((size_t)p.lb_words * 4);
    p.o_keys = take(N * k * 4);
    p.o_perms = take(N * k * 4);
    p.o_ranks = take(N * k * 4);
    // the record buffers also hold the presort's (key, index) ping-pongs
    p.rec_words = std::max(N * k, 2 * N);
    // (a launch of g roles takes slots 0 .. g-1 of 4N words each)
    p.o_rec = take(std::max(p.rec_words * 2, (size_t)4 * p.presort_group * N) * 4);
    p.o_nodeperm = take(N * 4);
    p.o_dimnode = take(N);
    p.o_box[0] = take((size_t)p.box_entries * 8 * 4);
    p.o_box[1] = take((size_t)p.box_entries * 8 * 4);
    p.o_bbox = take((size_t)p.large.size() * KEYSUM_WORDS * 4);
    p.o_piv = take((size_t)p.piv_words * 4);
    p.o_tables = take(p.tables ? p.blob.size() : 0);
    p.o_wcount = take((size_t)k * RANK_MAX_WIN * 4);
    p.o_tstatus = take((size_t)T * 4);        // a status word per tree
    p.total = o;
    return p;
}

}  // namespace kdt
