// kdt_shares.h -- constants and launch-table records shared by the host
// planner and the kernels (plain C++: the planner also builds without HIP).
#pragma once

#include <stdint.h>

namespace kdt {

constexpr uint32_t KDT_STATUS_NONFINITE = 4;    // == KDT_ENONFINITE
constexpr uint32_t KDT_STATUS_INTERNAL = 0x100; // an internal bound or wait check failed

constexpr uint32_t RADIX_HOST = 256;
constexpr uint32_t MAX_PASSES = 256;       // onesweep passes per build (tile counters)
constexpr uint32_t XQ_LAUNCHES = 16;       // presort launches that can take tiles from per-XCD queues
constexpr uint32_t MAX_COUNTERS = MAX_PASSES + 8 * XQ_LAUNCHES;   // pass counters, then 8 queue counters each
constexpr uint32_t XQ_MIN_TREES = 16;      // trees from which presorts use per-XCD tile queues
constexpr uint32_t MAX_LEVEL_PASSES = 3;   // digits of a rank of at most 30 bits (8..10-bit digits)
constexpr uint32_t MAX_BINS = 1024;        // 2^10 digit values
constexpr uint32_t PART_BINS = 4;          // digit values of the split passes (smaller, pivot, larger)
constexpr uint32_t PREP_TILE = 4096;       // points per workgroup of prep / iteration 0
// Per-tree key summary, as orderable keys: [0..3] per-dimension minimum,
// [4..7] maximum, [8..11] bitwise AND, [12..15] bitwise OR, kept in
// KEYSUM_COPIES copies on lines of their own (prep workgroup b updates copy
// b mod KEYSUM_COPIES: one line taking every tile's atomics serialises them)
// that k_root_dim combines into the first copy.
constexpr uint32_t KEYSUM_COPIES = 8;
constexpr uint32_t KEYSUM_COPY_WORDS = 32;                          // 128 bytes
constexpr uint32_t KEYSUM_WORDS = KEYSUM_COPIES * KEYSUM_COPY_WORDS; // per tree

// Threads of the onesweep workgroups (presort and level passes).
#ifndef KDT_SWEEP_THREADS
#define KDT_SWEEP_THREADS 512
#endif
constexpr int SWEEP_THREADS = KDT_SWEEP_THREADS;

// Tile shapes (items per thread of a SWEEP_THREADS workgroup); tuning knobs.
#ifndef KDT_PRESORT_ITEMS
#define KDT_PRESORT_ITEMS 14
#endif
constexpr int PRESORT_ITEMS = KDT_PRESORT_ITEMS;
constexpr uint32_t PRESORT_TILE = (uint32_t)SWEEP_THREADS * PRESORT_ITEMS;
// Dimensions whose presort digit passes share a launch (each needs its own
// (key, index) ping-pong of 4 words per point).
#ifndef KDT_PRESORT_GROUP
#define KDT_PRESORT_GROUP 4
#endif
constexpr uint32_t PRESORT_GROUP = KDT_PRESORT_GROUP;
// Records per thread of the large split tiles (the small ones take 4).
#ifndef KDT_PART_ITEMS
#define KDT_PART_ITEMS 10
#endif
constexpr int PART_ITEMS = KDT_PART_ITEMS;
constexpr uint32_t RANK_MAX_WIN = 2048;      // index windows of the windowed rank scatter
#ifndef KDT_RANK_WIN_BITS
#define KDT_RANK_WIN_BITS 18
#endif
constexpr uint32_t RANK_WIN_BITS = KDT_RANK_WIN_BITS;  // log2 of the indices per window (at least)
#ifndef KDT_RANK_WIN_CHUNK
#define KDT_RANK_WIN_CHUNK 8192
#endif
constexpr uint32_t RANK_WIN_CHUNK = KDT_RANK_WIN_CHUNK;  // pairs per k_rank_window workgroup
#ifndef KDT_HIST_TILE
#define KDT_HIST_TILE 8192
#endif
constexpr uint32_t HIST_TILE = KDT_HIST_TILE;  // keys per workgroup of the pivot selects
constexpr uint32_t PIVOT_SEGS = 4;         // subtrees per pivot workgroup (one wave each)
constexpr int TAIL_THREADS = 512;          // subtree tail: 512 threads x 4 slots = up to 2048 points
constexpr int TAIL_ITEMS = 4;
constexpr uint32_t TAIL_CAP = (uint32_t)TAIL_THREADS * TAIL_ITEMS;

// One tree of a call.
struct TreeInfo {
    uint32_t off;        // first entry of the tree in every per-point array
    uint32_t n;          // points
    uint32_t box_off;    // first entry of its split-widest domain tables
    uint32_t idx;        // position in the call's tree list (histogram / box slots)
};

// One tree's share of a launch.
struct TreeStep {
    uint32_t tree;       // index into the TreeInfo table
    uint32_t level;      // iteration processed (tail: first iteration it runs)
    uint32_t tile0;      // first tile (tail: first workgroup) of this share
    uint32_t hist;       // word offset of the share's digit histograms for this iteration
    uint32_t hist_next;  // word offset of its histograms for the next iteration (~0u: none)
    uint32_t pair0;      // tail: level-l0 subtrees [0, pair0) take one workgroup each, the later ones two
    uint32_t buf;        // tail: record buffer (0/1) that holds the tree's level-l0 records
    uint32_t piv;        // word offset of the share's per-subtree pivot entries (2 words each)
};

}  // namespace kdt
