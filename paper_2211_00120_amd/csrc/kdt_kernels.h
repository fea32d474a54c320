// kdt_kernels.h -- interface between the host driver and the gfx950 kernels.
//
// Every kernel works on a set of independent trees (one for kdt_build_ws,
// many for kdt_build_batched).  All per-point arrays of a call -- points,
// outputs, keys, ranks, records, node tables -- hold the trees back to back:
// tree t occupies entries [off_t, off_t + n_t).  A launch covers a list of
// (tree, level) shares; a workgroup finds its share by binary search on the
// share's first tile.  With a single share the list is passed inline in the
// kernel arguments, so a single build needs no table in device memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_layout.h"
#include "kdt_shares.h"

namespace kdt {

// The shares of one launch: a device table, or (steps == nullptr) the single
// share held inline.
struct Shares {
    const TreeInfo* trees;
    const TreeStep* steps;
    uint32_t nsteps;
    TreeInfo tree0;
    TreeStep step0;
};

// Per-call outputs and per-point tables (indexed by off_t + local index).
struct Outs {
    const float* pts;
    float* tree;            // nullable
    uint8_t* dim;           // nullable (round robin)
    uint32_t* nodeperm;     // original (local) index per node (the caller's perm or workspace)
    uint8_t* dimnode;       // split dim per node (split-widest; caller's dim or workspace)
    uint32_t* status;       // device status word
    uint32_t* tstatus;      // per tree of the call (TreeStep::tree): its own status word (non-finite input)
    uint32_t* box[2];       // split-widest domains of live subtrees as keys of their bounds,
                            // [level & 1][(box_off + i)*8 + (0..3 lo, 4..7 hi)]
    uint32_t* bbox;         // per tree: key summary [idx*KEYSUM_WORDS + ...] (scene box, bits that vary)
    uint32_t i32;           // coordinates are int32 (pts, tree: 32-bit words of int32 values), else float32
};

struct PrepArgs {
    Shares sh;              // one share per tree, tiles of PREP_TILE points
    uint32_t* keys;         // [d*ntotal + off + i]
    uint32_t* hist;         // per tree: [(idx*k + d)*4 + pass][256]
    uint32_t ntotal;
    Outs o;
};

// Pass `pass` (digit 8*pass) of one dimension's presort.  A pass whose
// digit is the same in every key of a tree (from the key summary) is skipped
// for that tree; each tree's passes read the output of its last pass that
// ran (or prep's keys, before any) and write the other (key, index) buffer.
// The last pass always runs.
struct PresortArgs {
    Shares sh;              // one share per tree, tiles of PRESORT_TILE points
    const uint32_t* keys;   // prep's keys, [d*ntotal + off + i] (value = local index)
    uint32_t* kv;           // (key, local index) pairs, interleaved: dimension slot j ping-pongs between
                            // kv + (2j)*kv_words and kv + (2j+1)*kv_words
    size_t kv_words;
    const uint32_t* keysum; // per tree key summaries
    uint32_t pass;
    uint32_t role0, ndims;  // the launch sorts roles role0 .. role0+ndims-1 (role_dim), tiles interleaved
    const uint32_t* hist;   // per tree digit histograms: hist + idx*hist_stride + (d*4 + pass)*RADIX
    uint32_t hist_stride;
    uint32_t* lb;           // look-back words of this pass, dimension slot j at lb + j*lb_dim_words
    uint32_t lb_dim_words;
    uint32_t* lb_zero;      // look-back words to clear for the next pass
    uint32_t lb_zero_n;
    uint32_t* counter;      // dynamic tile counter of this pass
    const uint32_t* xq;     // per-XCD tile queues (null: take tiles from `counter`)
    uint32_t* xq_cnt;       // the 8 queue counters of this launch
    uint32_t* perms;        // last pass: per tree and role the sorted payloads, [role*ntotal + off + rank]
    // Payloads: each point's local index; or, with root_ranks, for every
    // role but the root's the point's root rank (its position in the root
    // dimension's order, read in the role's first pass from root_ranks), so
    // that the role's ranks land at root positions.
    uint32_t* rank_table;   // point-major layout: last pass writes [(off + index)*k + dim] = rank for every
                            // role but the root's; null in the per-role layout (k_rank_bucket / k_rank_window
                            // write the ranks)
    const uint32_t* root_ranks;   // per-role layout: role 0's array, root rank by local index [off + i]; else null
    const uint8_t* dimnode; // split-widest: node dims (the root's is tree's first entry); null: root dimension 0
    uint32_t k;
    uint32_t ntotal;
    uint32_t* status;
    // k = 1: the last pass places every tree (its sorted order is the tree's
    // in-order sequence), with o's outputs; no iteration follows
    uint32_t place1;
    Outs o;
};

struct Level0Args {
    Shares sh;              // one share per tree, tiles of PREP_TILE ranks
    const uint32_t* xmap;   // null, or per workgroup its tile (0xFFFFFFFF: none), trees grouped by XCD
    const uint32_t* perms;  // presort outputs, [role*ntotal + off + rank]; role 0: root order -> local index
    const uint32_t* rank_table;   // point-major layout: records by local index, [(off + i)*k + d] (gathered)
    const uint32_t* role_ranks;   // per-role layout: rank of the point at root position r in role j's dimension,
                                  // [j*ntotal + off + r] (j >= 1, streamed); null in the point-major layout
    uint32_t* rout;         // iteration-1 records
    uint32_t* kout;         // iteration-1 split keys (share.hist_next != NO_HIST and keys_next)
    uint32_t* hist;         // base of the iteration-1 histograms (share.hist_next offsets)
    uint32_t keys_next;     // iteration 1 selects its pivots from keys and histograms
    uint32_t ntotal;
    uint32_t passes;
    uint32_t radix_bits;
    Outs o;
};

// Pivot selection of iteration l, one digit: the digit histogram, per
// subtree, of the split keys whose higher digits equal the pivot's (known
// from the histograms of the higher digits).
struct LevelSelectArgs {
    Shares sh;              // shares of one iteration, tiles of HIST_TILE
    const uint32_t* kin;    // split key (rank in the subtree's split dimension) per live position
    uint32_t* hist;         // histogram region; share.hist word offsets
    uint32_t passes;        // digits per key (the top one is counted when the keys are written)
    uint32_t digit;         // digit counted by this launch (0 = lowest)
    uint32_t radix_bits;
    uint32_t* status;
    const uint8_t* dimnode; // split-widest: node dims; subtrees split in the root's dimension are skipped
                            // (their pivot is the point at position ss(2s+1))
};

// The pivot of every subtree of iteration l, one wave per subtree: its key
// (from the digit histograms, or, in the root's dimension, its position),
// its node's point (placed here) and, for split-widest, its children's
// dimensions and domains.  Writes piv[share.piv + 2*seg] = key and
// piv[share.piv + 2*seg + 1] = child dimensions (left | right << 8).
struct LevelPivotArgs {
    Shares sh;              // shares of one iteration, workgroups of PIVOT_SEGS subtrees
    const uint32_t* rin;    // records (the pivot record of segments split in the root's dimension)
    const uint32_t* hist;   // histogram region; share.hist word offsets
    uint32_t* piv;
    const uint32_t* perms;  // presort outputs, [role*ntotal + off + rank] (see PresortArgs)
    uint32_t root_payload;  // the roles but the root's carry root ranks (per-role layout): two lookups
    uint32_t ntotal;
    uint32_t passes, radix_bits;
    uint32_t sorted;
    uint32_t k;
    Outs o;
};

// The update of iteration l: a stable three-way split of every subtree's
// segment around its pivot (smaller key, the pivot, larger key), which is
// the sorted order of Sec. 3.1 restricted to what the tag update reads.
struct LevelPartArgs {
    Shares sh;              // shares of one iteration, tiles of 512*items
    const uint32_t* rin;
    uint32_t* rout;         // next iteration's records
    uint32_t* kout;         // next iteration's split keys (keys_next)
    uint32_t* hist;         // histogram region; share.hist_next word offsets (next iteration's top digit)
    const uint32_t* piv;    // pivot entries of this iteration (LevelPivotArgs)
    uint32_t passes, radix_bits;
    uint32_t items;         // records per thread in this launch's tiles (tile = SWEEP_THREADS * items)
    uint32_t keys_next;     // write the next iteration's split keys and top-digit histograms
    uint32_t* lb;
    uint32_t* lb_zero;
    uint32_t lb_zero_n;
    uint32_t* zero2;        // buffer to clear (histograms of the iteration after next)
    uint32_t zero2_n;
    uint32_t* counter;
    uint32_t k;             // dimension count (round robin split dimension = level mod k)
    Outs o;
};

struct TailArgs {
    Shares sh;              // tail shares: workgroup ranges, level = first tail iteration
    const uint32_t* xmap;   // null, or per workgroup its group (0xFFFFFFFF: none), trees grouped by XCD
    const uint32_t* rin[2]; // the two record buffers (share.buf selects; from_points: unused)
    uint32_t from_points;   // whole trees of at most TAIL_CAP points, built from the points
    uint32_t init_status;   // a single workgroup that first zeroes o.status itself (no init launch)
    Outs o;
};

void launch_set_word(uint32_t* dst, uint32_t value, hipStream_t st);
// out record s = in record perm[s], records of `stride` bytes, s < n.
void launch_permute(const uint32_t* perm, uint32_t n, const void* in, void* out, uint32_t stride, uint32_t* status,
                    hipStream_t st);
void launch_copy_word(uint32_t* dst, const uint32_t* src, hipStream_t st);
void launch_init(uint32_t* status, uint32_t* counters, uint32_t* z1, uint32_t n1, uint32_t* z2, uint32_t n2,
                 uint32_t* z3, uint32_t n3, uint32_t* z4, uint32_t n4, uint32_t* z5, uint32_t n5, uint32_t* bbox,
                 uint32_t nbox, hipStream_t st);
void launch_prep(int k, const PrepArgs& a, uint32_t tiles, bool widest, hipStream_t st);
void launch_root_dim(int k, const Shares& sh, const Outs& o, uint32_t ntrees, bool widest, hipStream_t st);
void launch_presort_pass(const PresortArgs& a, bool last, uint32_t tiles, hipStream_t st);
// Windowed scatter of one dimension's ranks into its per-dimension array
// (see k_rank_bucket).  Windows of 2^wbits global indices, at most
// RANK_MAX_WIN of them; each bucket holds up to 2^wbits (index, rank) pairs.

struct RankBucketArgs {
    Shares sh;              // presort shares: tiles of PRESORT_TILE ranks per tree
    const uint32_t* perm;   // this role's rank -> payload (local index or root position), [off + rank]
    uint32_t* pairs;        // bucket w: uint2 (global payload, rank) at [(w << wbits) + e]
    uint32_t* wcount;       // pairs in each bucket (zero before the launch)
    uint32_t wbits, nwin;
    uint32_t* status;
};

struct RankWindowArgs {
    const uint32_t* pairs;
    const uint32_t* wcount;
    uint32_t* dm;           // this role's rank array, [global payload]
    uint32_t wbits, nwin, chunks;   // chunks = 2^wbits / RANK_WIN_CHUNK (at least 1)
    uint32_t ntotal;
};

void launch_rank_bucket(const RankBucketArgs& a, uint32_t tiles, hipStream_t st);
void launch_rank_window(const RankWindowArgs& a, hipStream_t st);

// Per-dimension rank arrays dm[d*ntotal + i] -> point-major records
// pm[i*k + d], i < ntotal.
void launch_level0(int k, const Level0Args& a, uint32_t tiles, bool widest, hipStream_t st);
void launch_level_select(const LevelSelectArgs& a, uint32_t tiles, hipStream_t st);
void launch_level_pivot(int k, const LevelPivotArgs& a, uint32_t tiles, bool widest, hipStream_t st);
void launch_level_part(int k, const LevelPartArgs& a, uint32_t tiles, bool widest, hipStream_t st);
void launch_tail(int k, const TailArgs& a, uint32_t groups, bool widest, hipStream_t st);

}  // namespace kdt
