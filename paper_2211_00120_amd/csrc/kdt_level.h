// kdt_level.h -- the update of one iteration run as digit passes: a stable
// three-way split of every subtree segment around its pivot, with the tag
// update of Sec. 3.2 fused into its scatter.  Instantiated per dimension
// count in kdt_level_k{1,2,3,4}.hip (compiled in parallel).
//
// The tag update reads only where each point lands relative to its
// subtree's pivot ss(2s+1): before it (new tag 2s+1), at it (node s is
// fixed), after it (2s+2).  Once the pivot's key is known, that is one
// comparison per point, and a stable split by it leaves the two children in
// their parent's order -- so every segment keeps the order of iteration 0,
// the root dimension's sorted order.  The pivot's key is the key of rank
// ss(2s+1) in the segment; k_level_select counts it digit by digit into
// per-segment digit histograms (radix select) and k_level_pivot reads it off
// them, one wave per segment -- or, where the segment is already in
// split-key order (round robin, split dimension = the root's), takes the key
// at that position.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_common.h"
#include "kdt_device.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"
#include "kdt_sweep.h"

namespace kdt {

// Digit of the split pass: 0 smaller key, 1 the pivot, 2 larger key.
constexpr int PART_RB = 2;

template <int K, bool WIDEST, bool I32>
__global__ void __launch_bounds__(64 * PIVOT_SEGS) k_level_pivot(LevelPivotArgs a)
{
    TreeStep st;
    TreeInfo ti;
    find_share(a.sh, blockIdx.x, st, ti);
    const Level v = make_level(ti.n, st.level);
    const uint32_t seg = (blockIdx.x - st.tile0) * PIVOT_SEGS + (threadIdx.x >> 6);
    if (seg >= v.nseg) return;
    const size_t off = ti.off;
    const uint32_t d = WIDEST ? (uint32_t)a.o.dimnode[off + v.Fl + seg] : st.level % a.k;
    const uint32_t ls = seg_left_size(v, seg);
    const uint32_t s = v.Fl + seg;
    // the root's dimension: every segment is in its order, so the pivot is
    // the record at position ls, which carries the point's index in that
    // dimension's slot; its key for the split is that live position
    const uint32_t d0 = WIDEST ? (uint32_t)a.o.dimnode[off] : 0u;
    uint32_t p = 0;
    uint32_t idx = 0;
    if (d == d0) {
        p = seg_offset(v, seg) + ls;
        idx = pick4(load_rec4<K>(a.rin, off + p), d0);
    } else {
        const uint32_t RBv = a.radix_bits;
        const uint32_t NB = 1u << RBv;
        const uint32_t* h = a.hist + st.hist + (size_t)seg * a.passes * NB;
        uint32_t kk = ls;
        for (int jj = (int)a.passes - 1; jj >= 0; --jj)
            p = (p << RBv) | wave_find_bucket(h + (size_t)jj * NB, NB, kk, a.o.status);
    }
    if (lane_id() != 0) return;
    // rank p in dimension d -> that role's payload: the local index, or
    // the point's root position, whose root-role payload is the index
    if (d != d0 && in_bounds(p, ti.n, a.o.status)) {
        idx = a.perms[(size_t)dim_role(d, d0) * a.ntotal + off + p];
        if (a.root_payload && in_bounds(idx, ti.n, a.o.status)) idx = a.perms[off + idx];
    }
    if (!in_bounds(idx, ti.n, a.o.status)) idx = 0;
    place<K, WIDEST>(a.o, ti, s, idx);
    uint32_t c0 = (st.level + 1u) % a.k, c1 = c0;
    if (WIDEST) {
        const uint32_t plane = plane_key<I32>(a.o, ti, idx, d, K);
        const uint32_t* bc = a.o.box[st.level & 1u] + ((size_t)ti.box_off + seg) * 8;
        c0 = child_dim<K, I32>(bc, plane, d, 0u);
        c1 = child_dim<K, I32>(bc, plane, d, 1u);
        widest_children<K, I32>(a.o, ti, s, seg, plane, d, a.o.box[st.level & 1u], a.o.box[(st.level + 1u) & 1u]);
    }
    a.piv[st.piv + 2u * seg] = p;
    a.piv[st.piv + 2u * seg + 1u] = c0 | (c1 << 8);
}

template <int K, bool WIDEST, int ITEMS>
__global__ void __launch_bounds__(SWEEP_THREADS) k_level_part(LevelPartArgs a)
{
    constexpr uint32_t T = SWEEP_THREADS * (uint32_t)ITEMS;
    __shared__ SweepSmem<PART_RB, K, false> sm;
    __shared__ uint32_t nh[2 * MAX_BINS];   // top-digit histograms of the two children
    __shared__ uint32_t segc[4];            // the segment's count of each split digit

    if (threadIdx.x == 0) sm.tile = atomicAdd(a.counter, 1u);
    __syncthreads();
    const uint32_t g = uniform(sm.tile);
    TreeStep st;
    TreeInfo ti;
    find_share(a.sh, g, st, ti);
    const Level v = make_level(ti.n, st.level);
    const SegTiles tl = tiles_level(v, T);
    uint32_t seg, u;
    tile_locate(tl, g - st.tile0, seg, u);
    const uint32_t soff = tiles_seg_offset(tl, seg);
    const uint32_t ssz = tiles_seg_size(tl, seg);
    const uint32_t start = u * T;
    const uint32_t cnt = min(T, ssz - start);
    const size_t off = ti.off;
    const uint32_t d = WIDEST ? (uint32_t)a.o.dimnode[off + v.Fl + seg] : st.level % a.k;
    const uint32_t d0 = WIDEST ? (uint32_t)a.o.dimnode[off] : 0u;   // the root's dimension
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint32_t live = v.n - v.Fl;
    const uint32_t RBv = a.radix_bits;
    const uint32_t NB = 1u << RBv;
    const uint32_t P = a.passes;
    const uint32_t top = RBv * (P - 1u);
    const uint32_t ls = seg_left_size(v, seg);        // ss(2s+1): rank of the pivot in the segment
    const bool keys = a.keys_next != 0u && st.hist_next != 0xFFFFFFFFu;
    if (keys) {
        for (uint32_t x = threadIdx.x; x < 2u * NB; x += SWEEP_THREADS) nh[x] = 0u;
    }

    // the tile's records
    uint4 rec[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = w * 64u * ITEMS + (uint32_t)i * 64u + lane;
        ok[i] = j < cnt;
        rec[i] = ok[i] ? load_rec4<K>(a.rin, off + soff + start + j) : make_uint4(0u, 0u, 0u, 0u);
    }

    // the pivot's key and the children's dimensions (k_level_pivot)
    const uint32_t p = uniform(a.piv[st.piv + 2u * seg]);
    const uint32_t cdw = uniform(a.piv[st.piv + 2u * seg + 1u]);
    const uint32_t cd0 = cdw & 0xFFu, cd1 = cdw >> 8;
    if (threadIdx.x == 0) {
        // sweep_tile's barriers publish these before they are read
        segc[0] = ls;
        segc[1] = 1u;
        segc[2] = ssz - ls - 1u;
        segc[3] = 0u;
    }

    // the comparison with the pivot: by key, or in the root's dimension (the
    // segment's own order, whose slot holds the index) by position
    const bool bypos = d == d0;
    uint32_t dig[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = w * 64u * ITEMS + (uint32_t)i * 64u + lane;
        const uint32_t x = bypos ? start + j : pick4(rec[i], d);
        const uint32_t y = bypos ? ls : p;
        dig[i] = x < y ? 0u : (x == y ? 1u : 2u);
    }
    // (the split pass stores from registers: sweep_tile never re-derives a
    // digit from a record, which for the root's dimension it could not)
    auto digit_of = [&](const uint4& r) {
        const uint32_t x = pick4(r, d);
        return x < p ? 0u : (x == p ? 1u : 2u);
    };
    const uint32_t piv = soff + ls;
    auto store = [&](uint32_t, uint32_t pos, const uint4& r) {
        if (pos == piv) return;                 // node s, placed above
        const uint32_t side = pos > piv ? 1u : 0u;
        const uint32_t nxt = pos - seg - side;  // live position in iteration l+1
        if (!in_bounds(pos, live, a.o.status) || !in_bounds(nxt, live - v.nseg, a.o.status)) return;
        store_rec4<K>(a.rout, off + nxt, r);
        if (keys) {
            // no split key for a child split in the root's dimension: its
            // pivot is found by position
            const uint32_t cd = side ? cd1 : cd0;
            if (cd != d0) {
                const uint32_t kv = pick4(r, cd);
                a.kout[off + nxt] = kv;
                atomicAdd(&nh[side * NB + ((kv >> top) & (NB - 1u))], 1u);
            }
        }
    };
    sweep_tile<PART_RB, ITEMS, K, decltype(digit_of), decltype(store), false>(
        sm, rec, ok, dig, ITEMS, cnt, segc, soff, a.lb, g, g - u, a.o.status, digit_of, store);

    if (keys) {
        // sweep_tile ends with a barrier, so nh is complete; children 2seg
        // and 2seg+1 are segments of iteration l+1
        for (uint32_t x = threadIdx.x; x < 2u * NB; x += SWEEP_THREADS) {
            const uint32_t c = x / NB;
            if (nh[x])
                atomicAdd(&a.hist[st.hist_next + ((size_t)(2u * seg + c) * P + P - 1u) * NB + (x - c * NB)], nh[x]);
        }
    }
    zero_range(a.lb_zero, a.lb_zero_n);
    zero_range(a.zero2, a.zero2_n);
}

template <int K>
void launch_level_pivot_k(const LevelPivotArgs& a, uint32_t tiles, bool widest, hipStream_t st)
{
    // round robin never reads a coordinate here: one instantiation
    if (!widest) k_level_pivot<K, false, false><<<tiles, 64 * PIVOT_SEGS, 0, st>>>(a);
    else if (a.o.i32) k_level_pivot<K, true, true><<<tiles, 64 * PIVOT_SEGS, 0, st>>>(a);
    else k_level_pivot<K, true, false><<<tiles, 64 * PIVOT_SEGS, 0, st>>>(a);
}

template <int K, int ITEMS>
static void level_part_ki(const LevelPartArgs& a, uint32_t tiles, bool widest, hipStream_t st)
{
    if (widest) k_level_part<K, true, ITEMS><<<tiles, SWEEP_THREADS, 0, st>>>(a);
    else k_level_part<K, false, ITEMS><<<tiles, SWEEP_THREADS, 0, st>>>(a);
}

template <int K>
void launch_level_part_k(const LevelPartArgs& a, uint32_t tiles, bool widest, hipStream_t st)
{
    switch (a.items) {
    case 4: level_part_ki<K, 4>(a, tiles, widest, st); break;
    default: level_part_ki<K, PART_ITEMS>(a, tiles, widest, st); break;
    }
}

}  // namespace kdt
