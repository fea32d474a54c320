// kdt_plan.h -- host planner of a build call (plain C++, no HIP).
//
// A call builds a list of independent trees.  The plan fixes, from the tree
// sizes, k and the split rule alone: which trees are built whole by one
// workgroup, the launch sequence of the others (prep, presorts, iteration
// 0, the iterations run as pivot selects and splits, the tail), every
// launch's share table, the digit width of the pivot selects and the
// workspace layout.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "kdt_shares.h"

namespace kdt {

constexpr size_t WS_ALIGN = 256;
inline size_t align_up(size_t x) { return (x + WS_ALIGN - 1) & ~(WS_ALIGN - 1); }
constexpr uint32_t NO_HIST = 0xFFFFFFFFu;

// Choices the planner otherwise makes itself (0 = automatic).
struct PlanOptions {
    uint32_t radix_bits = 0;   // digit width of the pivot selects: 8, 9 or 10
    uint32_t max_items = 0;    // records per thread of the split tiles: 4 (512 x 4 only) or PART_ITEMS (also 512 x PART_ITEMS)
    uint32_t rank_layout = 0;  // 1: point-major rank table, 2: per-role rank arrays (windowed scatter)
    uint32_t presort_dims = 0; // non-root presort roles whose digit passes share a launch: 1..4 (clamped)
};

// A tree whose rank table is larger than this has its ranks scattered into
// per-role arrays through payload windows (random 4-byte writes that leave a
// line partly written cost about twice as much as ones that, over the pass,
// fill it); smaller tables stay in the last-level cache while their tree's
// tiles run and are written point-major.
constexpr uint64_t RANK_DM_BYTES = 128ull << 20;

// One iteration run as digit passes over every tree that still has subtrees
// larger than TAIL_CAP: P-1 pivot-select launches (none when `sorted`), the
// pivot launch, then the split.
struct LevelLaunch {
    uint32_t level = 0;
    uint32_t items = 4;              // records per thread of its split tiles
    uint32_t tiles = 0;              // split tiles
    uint32_t select_tiles = 0;       // pivot-select tiles
    uint32_t pivot_tiles = 0;        // pivot workgroups (PIVOT_SEGS subtrees each)
    uint32_t piv_words = 0;          // words of its pivot entries
    uint32_t hist_words = 0;         // words of its digit histograms
    bool sorted = false;             // round robin at the root's dimension: segments are in key order
    std::vector<TreeStep> steps;     // split shares
    std::vector<TreeStep> ssteps;    // pivot-select shares (tiles of HIST_TILE)
    std::vector<TreeStep> psteps;    // pivot shares (workgroups of PIVOT_SEGS subtrees)
};

// Everything about one call that depends only on the tree sizes, k and mode.
// Iteration l's digit histograms live in third (l mod 3) of the histogram
// region, so that the split of iteration l can clear the third of l + 2.
struct Plan {
    uint32_t k = 0;
    bool widest = false;
    uint64_t ntotal = 0;
    std::vector<TreeInfo> trees;     // every tree of the call
    std::vector<uint32_t> large;     // trees built by digit passes
    std::vector<TreeStep> small;     // whole-tree shares (one workgroup each)
    uint32_t B = 0, RB = 8, P = 0;   // rank bits / digit bits / digits of the pivot selects
    bool rank_dm = false;            // per-role rank arrays (windowed scatter) instead of a point-major table
    uint32_t rank_wbits = 0, rank_nwin = 0;  // payload windows of the windowed scatter
    uint32_t presort_group = 1;      // presort roles sharing a launch (the root's role runs alone, first)
    struct PresortLaunch {
        uint32_t role0, ndims, pass;  // digit pass `pass` of presort roles role0 .. role0+ndims-1
    };
    std::vector<PresortLaunch> presort_launches;  // in order
    bool xq = false;                 // presort tiles from per-XCD queues (many trees)
    std::vector<uint32_t> xq_table;  // off[8], len[8], then each queue's presort tile indices
    std::vector<uint32_t> xmap0;     // iteration 0: per workgroup its prep-tile (same trees per XCD as xq)
    std::vector<uint32_t> xmapt;     // tail: per workgroup its group (same trees per XCD as xq)
    std::vector<TreeStep> prep, presort, level0, tail, roots;
    uint32_t prep_tiles = 0, presort_tiles = 0, tail_groups = 0;
    std::vector<LevelLaunch> levels; // iterations 1.. run as passes
    uint32_t hist_words = 0;         // per third of the histogram region
    uint32_t lb_words = 0;           // per look-back buffer
    uint32_t piv_words = 0;          // pivot entries of the largest iteration
    uint32_t box_entries = 0;        // per split-widest domain buffer
    std::vector<uint32_t> pass_words;// look-back words of every onesweep pass, in order
    bool tables = false;             // some launch reads a device share table
    std::vector<uint8_t> blob;       // the share tables, as uploaded
    size_t t_trees = 0, t_small = 0, t_prep = 0, t_presort = 0, t_level0 = 0, t_tail = 0, t_roots = 0, t_xq = 0,
           t_xmap0 = 0, t_xmapt = 0;
    std::vector<size_t> t_level, t_select, t_pivot;
    // workspace offsets (bytes)
    size_t o_status = 0, o_counters = 0, o_hist_rank = 0, o_hist = 0, o_lb[2] = {0, 0}, o_keys = 0, o_perms = 0,
           o_ranks = 0, o_rec = 0, o_nodeperm = 0, o_dimnode = 0, o_box[2] = {0, 0}, o_bbox = 0, o_piv = 0, o_tables = 0,
           o_wcount = 0, o_tstatus = 0, total = 0;
    size_t rec_words = 0;            // words per record buffer
};

// Plan of a call over trees of n[t] points (in that order, back to back).
// Default options take the tuned choice for (k, rule, rank bits), if any.
Plan make_plan(const std::vector<uint32_t>& n, uint32_t k, bool widest, const PlanOptions& opt = PlanOptions());

// Rank bits of the largest tree built by digit passes (0 if none).
uint32_t plan_rank_bits(const std::vector<uint32_t>& n);

// Workspace bytes that hold the plan under every tuning choice.
size_t workspace_bytes_any(const std::vector<uint32_t>& n, uint32_t k, bool widest);

// The autotuner's table: one choice per (k, split rule, rank bits).
std::vector<PlanOptions> tuning_candidates();
PlanOptions tuned_options(uint32_t k, bool widest, uint32_t bits);
void set_tuned_options(uint32_t k, bool widest, uint32_t bits, const PlanOptions& o);
void clear_tuning();
bool save_tuning(const char* path);
bool load_tuning(const char* path);

// First iteration at which every subtree of an n-point tree holds at most
// TAIL_CAP points (n > TAIL_CAP).
uint32_t first_tail_level(uint32_t n);

}  // namespace kdt
