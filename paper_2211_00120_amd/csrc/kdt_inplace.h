// kdt_inplace.h -- arithmetic of the low-memory in-place build (host and
// device; the host check tests/host/inplace_check.cpp runs it on the CPU).
//
// Sec. 7 (Discussion) observes that the method itself needs one int per node
// of temporary storage, and that a sort built only from swaps (bitonic sort)
// would need nothing more.  The in-place build takes that literally: the
// points are permuted where they lie, the one int per node is the caller's
// perm array (the original index, which is also the tie-break of the order
// (coordinate, index)), and every data movement is a compare-exchange or a
// swap.  The workspace holds only the status word, the scene box and one
// byte (split-widest: plus one box) per subtree of the first LDS level.
//
// Layout during the build: IN-ORDER.  The subtrees of one level occupy
// disjoint ranges of the array and the pivots of the levels above lie
// between them, exactly as in an in-order traversal; the tag of a point is
// therefore implied by its position and is never stored.  Iteration l sorts
// every level-l subtree's range along its split dimension (Sec. 3.1's sort,
// restricted to one subtree as the tag order makes it); the update of
// Sec. 3.2 then needs no work: the point at offset ss(2s+1) of the range is
// the pivot and stays there, the points before it form the left child's
// range, the points after it the right child's.  Between two consecutive
// subtrees of a level lies exactly one node of the levels above (their
// lowest common ancestor), so the i-th subtree of level l starts at
//     io_begin(i) = sb(s,l) - F(l) + i      (s = F(l) + i)
// with sb the segment begin of Sec. 4.2.  After the last iteration the array
// is the in-order sequence of the tree, and a swap-only permutation turns it
// into level order (the array layout of Sec. 2).
//
// In-order to level order.  With U = F(L-1) nodes above the last level and
// m = N - U leaves, the in-order sequence is l0 u0 l1 u1 ... l(m-1) u(m-1)
// u(m) ... u(U-1), where u is the in-order sequence of the perfect tree of
// the upper L-1 levels and l the leaves left to right (leaf j is the left or
// right child of bottom node floor(j/2) and directly precedes u(j)).  So an
// unshuffle of the first 2m entries (odd positions first, then even ones,
// each in order) followed by a rotation that moves the m leaves to the end
// leaves [u in order | leaves in order]; the leaves are then in level order,
// and the perfect tree u is handled the same way (its bottom level sits at
// the even positions) until it fits in one LDS block.
//
// An unshuffle of a range is done bottom up: LDS blocks of BLK entries are
// unshuffled whole; then for block sizes S = 2 BLK, 4 BLK, ... each block is
// [O1 E1 | O2 E2] (its two halves already unshuffled) and swapping the
// equal-sized E1 and O2 unshuffles it.  A last, shorter block needs the
// rotation [E1 O2] -> [O2 E1] of unequal parts: three reversals.
#pragma once

#include "kdt_layout.h"

namespace kdt {
namespace ip {

constexpr uint32_t BLK_LOG = 11;
constexpr uint32_t BLK = 1u << BLK_LOG;   // records of one LDS block (2048 x (k+1) words)
constexpr uint32_t THREADS = 256;         // threads of the LDS kernels
constexpr uint32_t GROUP_MAX = 4;         // strides one global compare-exchange pass applies
constexpr uint32_t SBLK_LOG = 12;
constexpr uint32_t SBLK = 1u << SBLK_LOG; // entries of one LDS block of an iteration's sort
constexpr uint32_t MGROUP_MAX = 3;        // first strides of a stage (the mirrored one first) in one pass

// In-order begin of the i-th subtree of level l (levels 0..L-1; on level
// L-1 only the R existing leaves, i < R).
KDT_HD uint32_t io_begin(const Level& v, uint32_t i) { return seg_offset(v, i) + i; }
// In-order position of that subtree's pivot (levels 0..L-2).
KDT_HD uint32_t io_pivot(const Level& v, uint32_t i) { return io_begin(v, i) + seg_left_size(v, i); }

// Subtree of level l (l <= L-2) whose in-order range holds position P (the
// inverse of io_begin): its index, or 0xFFFFFFFF for a position holding a
// node of the levels above.  The subtrees come in the three sizes of
// kdt_layout.h, each followed by one such node.
KDT_HD uint32_t io_seg_of(const Level& v, uint32_t P)
{
    const uint32_t a = v.R / v.W;                  // subtrees of the larger size (levels <= L-2: W >= 2)
    const uint32_t big = 2u * v.W - 1u, small = v.W - 1u;
    if (a >= v.nseg) {
        const uint32_t i = P / (big + 1u);
        return P - i * (big + 1u) < big ? i : 0xFFFFFFFFu;
    }
    const uint32_t head = a * (big + 1u);
    if (P < head) {
        const uint32_t i = P / (big + 1u);
        return P - i * (big + 1u) < big ? i : 0xFFFFFFFFu;
    }
    const uint32_t mid = (v.W - 1u) + (v.R - a * v.W);
    const uint32_t q = P - head;
    if (q < mid) return a;
    if (q == mid) return 0xFFFFFFFFu;
    const uint32_t r = q - mid - 1u;
    const uint32_t i = r / (small + 1u);
    return r - i * (small + 1u) < small ? a + 1u + i : 0xFFFFFFFFu;
}

// First level whose subtrees (at most 2^(L-l) - 1 nodes) fit one LDS block.
KDT_HD uint32_t deep_level(uint32_t L) { return L > BLK_LOG ? L - BLK_LOG : 0u; }

// Smallest power of two >= x (x >= 1, x <= 2^31).
KDT_HD uint32_t ceil_pow2(uint32_t x) { return x <= 1u ? 1u : 1u << (32u - (uint32_t)__builtin_clz(x - 1u)); }
KDT_HD uint32_t log2_exact(uint32_t p) { return 31u - (uint32_t)__builtin_clz(p); }

// Padded length of the bitonic network of level l: every subtree of the
// level is sorted as if it had P entries, the missing ones +infinity.
// Subtree 0 is the level's largest.
KDT_HD uint32_t net_len(const Level& v) { return ceil_pow2(seg_size(v, 0)); }

// One step of the in-order -> level-order permutation.
enum OpKind : uint32_t {
    OP_UNSHUF_LDS = 0,   // blocks of BLK entries of [a, a+n): odd offsets first, then even ones
    OP_SWAP_LEVEL = 1,   // blocks of 2^j of [a, a+n) with a full second half: swap E1 <-> O2
    OP_REVERSE = 2,      // reverse [a, a+n)
    OP_LDS_TREE = 3,     // [0, n), n <= BLK: in-order -> level order of an n-node tree, in LDS
};
struct Op {
    uint32_t kind, a, n, j;
};

// Threads (or workgroups, for the LDS kinds) an op needs.
KDT_HD uint32_t op_work(const Op& o)
{
    switch (o.kind) {
    case OP_UNSHUF_LDS: return ceil_div(o.n, BLK);
    case OP_SWAP_LEVEL: {
        const uint32_t S = 1u << o.j;
        return (o.n / S) * (S >> 2);           // full blocks x quarter-block swaps
    }
    case OP_REVERSE: return o.n >> 1;
    default: return 1u;
    }
}

// Emit the ops of an unshuffle of [a, a+n) through `emit(Op)`.
template <class F>
KDT_HD void plan_unshuffle(uint32_t a, uint32_t n, F&& emit)
{
    if (n < 2u) return;
    emit(Op{OP_UNSHUF_LDS, a, n, 0u});
    for (uint32_t j = BLK_LOG + 1u; j < 32u && (1u << (j - 1u)) < n; ++j) {
        const uint32_t S = 1u << j, H = S >> 1, Q = H >> 1;
        if (n / S) emit(Op{OP_SWAP_LEVEL, a, n, j});
        const uint32_t bs = (n / S) * S;                  // last, partial block
        if (bs + H < n) {
            const uint32_t r = n - bs - H;                // length of its second half (< H)
            const uint32_t o2 = r >> 1;                   // odd offsets of that half
            if (o2) {
                emit(Op{OP_REVERSE, a + bs + Q, Q, 0u});
                emit(Op{OP_REVERSE, a + bs + H, o2, 0u});
                emit(Op{OP_REVERSE, a + bs + Q, Q + o2, 0u});
            }
        }
    }
}

// Emit every op that takes the in-order array of an n-node tree to level order.
template <class F>
KDT_HD void plan_to_level_order(uint32_t n, F&& emit)
{
    if (n < 2u) return;
    if (n <= BLK) {
        emit(Op{OP_LDS_TREE, 0u, n, 0u});
        return;
    }
    const uint32_t L = num_levels(n);
    const uint32_t U = full_nodes(L - 1u);
    const uint32_t m = n - U;
    if (m == U + 1u) {
        plan_unshuffle(0u, n, emit);                      // perfect: [upper | leaves]
    } else {
        plan_unshuffle(0u, 2u * m, emit);                 // [u0..u(m-1) | leaves | u(m)..]
        // rotate [m, n) left by m: leaves after the rest of u
        emit(Op{OP_REVERSE, m, m, 0u});
        emit(Op{OP_REVERSE, 2u * m, n - 2u * m, 0u});
        emit(Op{OP_REVERSE, m, n - m, 0u});
    }
    // perfect upper trees: [0, u) holds one in order; unshuffle until it fits a block
    uint32_t u = U;
    while (u > BLK) {
        plan_unshuffle(0u, u, emit);
        u >>= 1;                                          // 2^(h-1) - 1
    }
    if (u >= 2u) emit(Op{OP_LDS_TREE, 0u, u, 0u});
}

// Bitonic sort of a sequence padded to P = 2^logP entries, the padding
// +infinity, ascending, without direction flips: stage e (blocks of 2^e)
// first compares entry w of every block with entry 2^e - 1 - w (mirrored
// pairs), then runs half-cleaners of strides 2^(e-2) .. 1 (entry i against
// i + stride inside every block of twice the stride; stride 2^ls).  A compare-exchange
// whose upper entry lies in the padding does nothing, so padding is never
// stored.  Pair q of a step:
KDT_HD void mirror_pair(uint32_t q, uint32_t e, uint32_t& lo, uint32_t& hi)
{
    const uint32_t S = 1u << e;
    const uint32_t w = q & ((S >> 1) - 1u);
    const uint32_t b0 = (q >> (e - 1u)) << e;
    lo = b0 + w;
    hi = b0 + S - 1u - w;
}
KDT_HD void half_pair(uint32_t q, uint32_t ls, uint32_t& lo, uint32_t& hi)   // stride 2^ls
{
    lo = ((q >> ls) << (ls + 1u)) | (q & ((1u << ls) - 1u));
    hi = lo + (1u << ls);
}

// The passes of one iteration's sort over subtrees longer than one block:
// stages up to SBLK inside LDS blocks, then per larger stage e one pass of
// its first strides (the mirrored one, 2^(e-1), and half-cleaners down to
// 2^(e-c)), the remaining half-cleaner strides down to SBLK in groups of up
// to GROUP_MAX per pass (largest first), and the strides below SBLK in LDS.
enum StepKind : uint32_t { ST_BLOCK_SORT = 0, ST_MGROUP = 1, ST_GROUP = 2, ST_BLOCK_MERGE = 3 };
struct Step {
    uint32_t kind, e, e0, c;   // ST_MGROUP: stage e, strides 2^(e-1) .. 2^(e-c); ST_GROUP: strides 2^e0 .. 2^(e0+c-1)
};
template <class F>
KDT_HD void plan_level_sort(uint32_t logP, F&& emit)
{
    emit(Step{ST_BLOCK_SORT, 0u, 0u, 0u});
    for (uint32_t e = SBLK_LOG + 1u; e <= logP; ++e) {
        const uint32_t cm = umin(MGROUP_MAX, e - SBLK_LOG);
        emit(Step{ST_MGROUP, e, e - cm, cm});
        uint32_t top = e - 1u - cm;                       // largest half-cleaner stride exponent left
        while (top + 1u > SBLK_LOG) {
            const uint32_t c = umin(GROUP_MAX, top - SBLK_LOG + 1u);
            emit(Step{ST_GROUP, e, top - c + 1u, c});
            top -= c;
        }
        emit(Step{ST_BLOCK_MERGE, e, 0u, 0u});
    }
}

// A mirrored group pass over stage e with c strides takes two groups of 2^c
// entries per thread: A with base b, B with base b ^ (2^e0 - 1) (e0 = e - c),
// entries b | x << e0; entry x of A and entry 2^c - 1 - x of B are mirrored
// in their 2^e-block.  Pair h of a network of length 2^logP has zeros in bits
// [e0 - 1, e0 + c) of its A base (e0 >= 1).
KDT_HD uint32_t mgroup_base(uint32_t h, uint32_t e0, uint32_t c)
{
    return ((h >> (e0 - 1u)) << (e0 + c)) | (h & ((1u << (e0 - 1u)) - 1u));
}

// Position (relative to the range start) of element e of a compare-exchange
// group: the group's base with e written into bits [e0, e0 + c).
KDT_HD uint32_t group_pos(uint32_t base, uint32_t e, uint32_t e0) { return base | (e << e0); }
// Base of group h of a network of length P when groups span bits [e0, e0+c).
KDT_HD uint32_t group_base(uint32_t h, uint32_t e0, uint32_t c)
{
    const uint32_t lowmask = (1u << e0) - 1u;
    return ((h >> e0) << (e0 + c)) | (h & lowmask);
}

}  // namespace ip
}  // namespace kdt
