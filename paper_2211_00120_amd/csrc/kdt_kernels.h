// kdt_kernels.h -- interface between the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_layout.h"

namespace kdt {

// Control words at the start of the workspace.
constexpr uint32_t CTL_STATUS = 0;      // 0 or KDT_STATUS_NONFINITE
constexpr uint32_t CTL_DIM0 = 1;        // split dimension of the root
constexpr uint32_t CTL_BOX_LO = 4;      // 4 words: scene box minimum (orderable keys)
constexpr uint32_t CTL_BOX_HI = 8;      // 4 words: scene box maximum (orderable keys)
constexpr uint32_t CTL_SCENE_LO = 12;   // 4 words: scene box minimum (float bits)
constexpr uint32_t CTL_SCENE_HI = 16;   // 4 words: scene box maximum (float bits)
constexpr uint32_t CTL_WORDS = 64;
constexpr uint32_t KDT_STATUS_NONFINITE = 4;   // == KDT_ENONFINITE
constexpr uint32_t KDT_STATUS_INTERNAL = 0x100; // an internal bound or wait check failed

constexpr uint32_t RADIX_HOST = 256;
constexpr uint32_t DIGIT_BITS_HOST = 8;
constexpr uint32_t MAX_PASSES = 256;       // onesweep passes per build (tile counters)
constexpr uint32_t MAX_LEVEL_PASSES = 3;   // digit passes over a rank of at most 30 bits (8..10-bit digits)
constexpr uint32_t MAX_BINS = 1024;        // 2^10 digit values
// Tile shapes (items per thread of a 256-thread workgroup); tuning knobs.
// (512-thread workgroups for the onesweep passes.)
#ifndef KDT_PRESORT_ITEMS
#define KDT_PRESORT_ITEMS 8
#endif
constexpr int PRESORT_ITEMS = KDT_PRESORT_ITEMS;   // presort tile: 512 x this many (key, index) pairs
constexpr uint32_t PRESORT_TILE = 512u * PRESORT_ITEMS;
constexpr uint32_t HIST_TILE = 16384;               // chunk of the split-widest histogram kernel
constexpr int TAIL_ITEMS = 8;                     // subtree tail: up to 2048 points per workgroup
constexpr uint32_t TAIL_CAP = 256u * TAIL_ITEMS;   // chunk of the split-widest histogram kernel

struct Outs {
    const float* pts;
    float* tree;            // nullable
    uint8_t* dim;           // nullable (round robin)
    uint32_t* nodeperm;     // original index per node (the caller's perm or workspace)
    uint8_t* dimnode;       // split dim per node (split-widest; caller's dim or workspace)
    const uint32_t* perm0;  // rank in dimension 0 -> original index
    const uint32_t* ctl;    // control words (scene box)
    uint32_t* status;       // device status word (ctl + CTL_STATUS)
    float* box[2];          // split-widest: domain of every live subtree, [level & 1][i*8 + (0..3 lo, 4..7 hi)]
    uint32_t n;
};

struct PresortArgs {
    const uint32_t* kin;    // first pass: prep's keys of this dimension (value = index)
    const uint32_t* kvin;   // later passes: (key, index) pairs, interleaved
    uint32_t* kvout;
    const uint32_t* hist;   // 256 counts of this pass's digit
    uint32_t* lb;           // look-back words of this pass
    uint32_t* lb_zero;      // look-back words to clear for the next pass
    uint32_t lb_zero_n;
    uint32_t* counter;      // dynamic tile counter of this pass
    uint32_t n;
    uint32_t shift;
    uint32_t* perm_out;     // last pass: rank -> index of this dimension
    uint32_t* rank_table;   // last pass: point-major ranks, [index*k + dim]
    uint32_t k;
    uint32_t dim;
    uint32_t* status;
};

struct Level0Args {
    const uint32_t* perms;       // presort outputs, [d*n + rank]
    const uint32_t* rank_table;  // point-major ranks
    uint32_t* rout;              // iteration-1 records
    uint32_t* hist_next;         // nullable: iteration-1 digit histograms (2 segments)
    uint32_t next_passes;
    uint32_t radix_bits;
    Outs o;
};

struct LevelHistArgs {
    const uint32_t* rin;
    const uint8_t* dimnode;
    uint32_t* hist;              // [seg][pass][2^radix_bits]
    uint32_t passes;
    uint32_t radix_bits;
    Level v;
    SegTiles tl;                 // tiling with HIST_TILE capacity
    uint32_t* status;
};

struct LevelPassArgs {
    const uint32_t* rin;
    uint32_t* rout;              // next pass's input, or (last pass) next iteration's records
    const uint32_t* hist;        // [seg][pass][2^radix_bits] of this iteration
    uint32_t passes, pass, shift, radix_bits;
    uint32_t items;              // records per thread in this launch's tiles (tile = 512 * items)
    uint32_t* lb;
    uint32_t* lb_zero;
    uint32_t lb_zero_n;
    uint32_t* zero2;             // buffer to clear (next iteration's histograms)
    uint32_t zero2_n;
    uint32_t* counter;
    Level v;
    SegTiles tl;                 // LEVEL_TILE tiling of iteration l
    uint32_t dim_rr;             // round robin split dimension l mod k
    uint32_t* hist_next;         // last pass, nullable: next iteration's histograms
    uint32_t next_passes;
    uint32_t dim_next_rr;
    Outs o;
};


struct TailArgs {
    const uint32_t* rin;         // records of iteration v0.l
    Level v0;                    // first iteration handled by the tail
    uint32_t G;                  // level-l0 subtrees per workgroup (1 or 2)
    uint32_t rank_bits;
    Outs o;
};

void launch_tail(int k, const TailArgs& a, bool widest, hipStream_t st);
void launch_set_word(uint32_t* dst, uint32_t value, hipStream_t st);
void launch_copy_word(uint32_t* dst, const uint32_t* src, hipStream_t st);
void launch_init(uint32_t* ctl, uint32_t* counters, uint32_t* z1, uint32_t n1, uint32_t* z2, uint32_t n2,
                 uint32_t* z3, uint32_t n3, hipStream_t st);
void launch_prep(int k, const float* pts, uint32_t n, uint32_t* keys, uint32_t* hist, uint32_t* ctl, bool widest,
                 hipStream_t st);
void launch_root_dim(int k, uint32_t* ctl, uint8_t* dimnode, float* box0, hipStream_t st);
void launch_presort_pass(const PresortArgs& a, bool first, bool last, uint32_t tiles, hipStream_t st);
void launch_level0(int k, const Level0Args& a, bool widest, hipStream_t st);
void launch_level_hist(int k, const LevelHistArgs& a, hipStream_t st);
void launch_level_pass(int k, const LevelPassArgs& a, bool last, bool widest, hipStream_t st);

}  // namespace kdt
