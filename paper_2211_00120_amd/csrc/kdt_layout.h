// kdt_layout.h -- implicit-tree arithmetic of the build, host and device.
//
// Level-order indexing (Sec. 2): node s has children 2s+1, 2s+2, level(s) =
// 31 - clz(s+1), a tree of N nodes has L = 32 - clz(N) levels (Sec. 4.2 with
// the revision-3 erratum), F(l) = 2^l - 1 nodes live above level l.
//
// Sec. 4 gives O(1) forms for the subtree size ss(s) and the segment begin
// sb(s,l).  With W = 2^(L-l-1) and R = N - F(L-1) (nodes on the last level),
// the i-th subtree of level l (s = F(l) + i) has
//     ss(s)  = (W - 1) + clamp(R - i*W, 0, W)
//     sb(s,l) - F(l) = i*(W - 1) + min(i*W, R)
// which is the paper's pair of formulas with the first-lowest-level-child
// term written as (s+1)*W - 1 = F(L-1) + i*W, and the inner-node term read as
// 2^(L-l-1) - 1 (the mathematical reading, not C operator precedence).
// Consequently the subtrees of a level come in at most three sizes: the first
// a = R / W are full (2W - 1), subtree a holds W - 1 + R % W, the rest W - 1.
//
// The pivot of subtree s in iteration l sits at sb(s,l) + ss(2s+1)
// (Sec. 3.2); for the i-th subtree, relative to F(l):
//     pivot_i = i*(W - 1) + min(i*W, R) + (W/2 - 1) + clamp(R - i*W, 0, W/2).
//
// All positions here are "live" positions: the array of one iteration holds
// only the N - F(l) points whose node is not fixed yet, so position p is the
// paper's array index F(l) + p (Sec. 7.1: the first F(l) entries need neither
// sorting nor updating).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define KDT_HD __host__ __device__ inline
#else
#define KDT_HD inline
#endif

namespace kdt {

// Every shift count below 32 and every clz argument non-zero, for every
// argument value: the edges (n = 0, l >= L - 1, s = 2^32 - 1, l >= 32) get
// defined results instead of undefined behaviour.
KDT_HD uint32_t num_levels(uint32_t n) { return n ? 32u - (uint32_t)__builtin_clz(n) : 0u; }
KDT_HD uint32_t level_of(uint32_t s)                                         // 32 for s = 2^32 - 1
{
    return s == 0xFFFFFFFFu ? 32u : 31u - (uint32_t)__builtin_clz(s + 1u);
}
KDT_HD uint32_t full_nodes(uint32_t l) { return l >= 32u ? 0xFFFFFFFFu : (1u << l) - 1u; }   // F(l)
KDT_HD uint32_t pow2(uint32_t e) { return e >= 32u ? 0u : 1u << e; }       // 2^e, 0 once it overflows
KDT_HD uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
// clamp(r - x, 0, cap), written without a branch: the guarded form
// `r > x ? min(r - x, cap) : 0` let the gfx950 compiler (ROCm 7.2 LLVM)
// hoist the min out of its branch with the no-wrap facts of the guarded
// subtraction still attached, and then fold an unrelated min(x, r) that
// follows (the one in seg_offset) to x.
KDT_HD uint32_t clamp_sub(uint32_t r, uint32_t x, uint32_t cap)
{
    return umin(r - umin(r, x), cap);
}
// Bits needed to write every rank 0..n-1.
KDT_HD uint32_t rank_bits(uint32_t n) { return n > 1 ? 32u - (uint32_t)__builtin_clz(n - 1u) : 0u; }

// Subtree arithmetic for iteration l of a build over n points.
struct Level {
    uint32_t n;     // N
    uint32_t l;     // iteration / level being split
    uint32_t L;     // levels of the tree
    uint32_t W;     // 2^(L-l-1): width of a level-l subtree on the last level
    uint32_t R;     // N - F(L-1): nodes on the last level
    uint32_t nseg;  // 2^l subtrees on level l
    uint32_t Fl;    // F(l)
};

KDT_HD Level make_level(uint32_t n, uint32_t l)
{
    Level v;
    v.n = n;
    v.l = l;
    v.L = num_levels(n);
    // levels l >= L have no subtrees: W = 0 (only l <= L - 2 is ever split)
    v.W = l < v.L ? pow2(v.L - l - 1u) : 0u;
    v.R = v.L ? n - full_nodes(v.L - 1u) : 0u;
    v.nseg = pow2(l);
    v.Fl = full_nodes(l);
    return v;
}

KDT_HD uint32_t seg_offset(const Level& v, uint32_t i) { return i * (v.W - 1u) + umin(i * v.W, v.R); }
KDT_HD uint32_t seg_size(const Level& v, uint32_t i) { return (v.W - 1u) + clamp_sub(v.R, i * v.W, v.W); }
KDT_HD uint32_t seg_left_size(const Level& v, uint32_t i)                   // ss(2s+1)
{
    uint32_t h = v.W >> 1;
    return (h - 1u) + clamp_sub(v.R, i * v.W, h);
}
KDT_HD uint32_t seg_pivot(const Level& v, uint32_t i) { return seg_offset(v, i) + seg_left_size(v, i); }

// Live position -> subtree index on level l (inverse of seg_offset).  On
// levels 0..L-2 (W >= 2) every subtree is non-empty; on level L-1 (W = 1)
// the subtrees are single nodes and position p is subtree p; a level below
// the tree (W = 0) has none, and 0 is returned.
KDT_HD uint32_t seg_of_pos(const Level& v, uint32_t p)
{
    if (v.W < 2u) return v.W ? p : 0u;
    uint32_t big = 2u * v.W - 1u;
    uint32_t a = v.R / v.W;                // number of full subtrees
    if (a >= v.nseg) return p / big;
    uint32_t head = a * big;
    if (p < head) return p / big;
    uint32_t mid = (v.W - 1u) + (v.R - a * v.W);
    uint32_t q = p - head;
    if (q < mid) return a;
    return a + 1u + (q - mid) / (v.W - 1u);
}

// In-order position -> level-order node of a left-balanced complete tree of
// n nodes (n >= 1).  With U = F(L-1) nodes above the last level and m = n - U
// leaves, the in-order sequence interleaves the first m in-order nodes of the
// upper perfect tree with the leaves (leaf j directly precedes upper node j),
// then lists the remaining upper nodes; an upper node's level and index follow
// from the trailing zeros of its in-order index plus one.
KDT_HD uint32_t inorder_to_level(uint32_t p, uint32_t n)
{
    const uint32_t L = num_levels(n);
    const uint32_t U = full_nodes(L - 1u);        // nodes above the last level
    const uint32_t m = n - U;                      // leaves on the last level
    uint32_t u;                                    // in-order index inside the upper perfect tree
    if (p < 2u * m) {
        if ((p & 1u) == 0u) return U + (p >> 1);
        u = p >> 1;
    } else {
        u = p - m;
    }
    // perfect tree of L-1 levels: in-order index u -> level order
    const uint32_t z = (uint32_t)__builtin_ctz(u + 1u);    // height above the bottom
    const uint32_t lev = (L - 2u) - z;
    return full_nodes(lev) + ((u + 1u) >> (z + 1u));
}

// Presort roles of a tree whose root splits in dimension d0 (k dimensions):
// role 0 is d0, roles 1 .. k-1 are the other dimensions in increasing order.
KDT_HD uint32_t role_dim(uint32_t role, uint32_t d0) { return role == 0u ? d0 : (role <= d0 ? role - 1u : role); }
KDT_HD uint32_t dim_role(uint32_t d, uint32_t d0) { return d == d0 ? 0u : (d < d0 ? d + 1u : d); }

// Subtrees of a level come in three sizes (see the header comment); a
// segment-aligned tiling cuts each one into tiles of at most `tile` points.
struct SegTiles {
    uint32_t nseg;      // number of segments
    uint32_t a;         // segments [0,a) have size `big`
    uint32_t big, mid, small;  // segment a has size `mid`, segments > a size `small`
    uint32_t tb, tm, ts;       // tiles per big / mid / small segment
    uint32_t tiles;     // total tiles
    uint32_t tile;      // tile capacity
};

KDT_HD uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1u) / b; }

KDT_HD SegTiles make_tiles(uint32_t nseg, uint32_t a, uint32_t big, uint32_t mid, uint32_t small, uint32_t tile)
{
    SegTiles t;
    t.nseg = nseg;
    t.a = a < nseg ? a : nseg;
    t.big = big;
    t.mid = mid;
    t.small = small;
    t.tile = tile;
    t.tb = ceil_div(big, tile);
    t.tm = ceil_div(mid, tile);
    t.ts = ceil_div(small, tile);
    t.tiles = t.a * t.tb;
    if (t.a < nseg) t.tiles += t.tm + (nseg - t.a - 1u) * t.ts;
    return t;
}

// One segment of n points (the presorts that compute the per-dimension ranks).
KDT_HD SegTiles tiles_single(uint32_t n, uint32_t tile) { return make_tiles(1u, 0u, 0u, n, 0u, tile); }

// The subtrees of iteration l.
KDT_HD SegTiles tiles_level(const Level& v, uint32_t tile)
{
    uint32_t a = v.W ? v.R / v.W : 0u;
    uint32_t mid = (v.W - 1u) + (a < v.nseg ? v.R - a * v.W : 0u);
    return make_tiles(v.nseg, a, 2u * v.W - 1u, mid, v.W - 1u, tile);
}

KDT_HD uint32_t tiles_seg_offset(const SegTiles& t, uint32_t i)
{
    if (i <= t.a) return i * t.big;
    return t.a * t.big + t.mid + (i - t.a - 1u) * t.small;
}
KDT_HD uint32_t tiles_seg_size(const SegTiles& t, uint32_t i)
{
    // operands as values: a conditional over the members themselves selects
    // between their addresses, which keeps the struct out of registers
    const uint32_t big = t.big, mid = t.mid, small = t.small;
    return i < t.a ? big : (i == t.a ? mid : small);
}

// Tile g -> (segment, tile index inside the segment).
KDT_HD void tile_locate(const SegTiles& t, uint32_t g, uint32_t& seg, uint32_t& u)
{
    uint32_t head = t.a * t.tb;
    if (g < head) { seg = g / t.tb; u = g - seg * t.tb; return; }
    uint32_t q = g - head;
    if (q < t.tm) { seg = t.a; u = q; return; }
    q -= t.tm;
    uint32_t j = q / t.ts;
    seg = t.a + 1u + j;
    u = q - j * t.ts;
}

// Workgroups of the tail over the nseg subtrees of one tree's first tail
// iteration: subtrees [0, pair0) one each, the later ones two each.
KDT_HD uint32_t tail_group_count(uint32_t nseg, uint32_t pair0) { return pair0 + (nseg - pair0 + 1u) / 2u; }
KDT_HD void tail_group_range(uint32_t gi, uint32_t pair0, uint32_t nseg, uint32_t& i0, uint32_t& i1)
{
    i0 = gi < pair0 ? gi : pair0 + 2u * (gi - pair0);
    i1 = umin(i0 + (gi < pair0 ? 1u : 2u), nseg);
}

}  // namespace kdt
