// kdt_level.h -- the segmented digit pass of one iteration's sort, with the
// tag update fused into its last pass.  Instantiated per dimension count in
// kdt_level_k{1,2,3,4}.hip (compiled in parallel).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_common.h"
#include "kdt_device.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"
#include "kdt_sweep.h"

namespace kdt {

// One stable digit pass of the per-segment sort of iteration l, ordering each
// subtree's points by the rank of its split dimension (RB-bit digits).  Tiles
// never straddle a segment; global offsets are segment offset + digit prefix
// inside the segment (from the histogram) + look-back over the segment's
// earlier tiles.  LAST fuses the tag update of Sec. 3.2 into the scatter and,
// for round robin, accumulates the next iteration's digit histograms.
template <int K, bool LAST, bool WIDEST, int RB, int ITEMS>
__global__ void __launch_bounds__(SWEEP_THREADS) k_level_pass(LevelPassArgs a)
{
    constexpr uint32_t NB = 1u << RB;
    constexpr uint32_t MASK = NB - 1u;
    constexpr uint32_t T = SWEEP_THREADS * (uint32_t)ITEMS;
    __shared__ SweepSmem<RB, K> sm;
    __shared__ uint32_t nh[LAST ? 2 * MAX_LEVEL_PASSES * NB : 1];

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
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint32_t live = v.n - v.Fl;
    const uint32_t shift = a.shift;
    const uint32_t* seg_hist = a.hist + st.hist + ((size_t)seg * a.passes + a.pass) * NB;
    const uint32_t NP = a.passes;
    const bool acc = LAST && a.acc_next && st.hist_next != 0xFFFFFFFFu;
    if (acc) {
        for (uint32_t x = threadIdx.x; x < 2u * NP * NB; x += SWEEP_THREADS) nh[x] = 0u;
    }

    uint4 rec[ITEMS];
    uint32_t dig[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = w * 64u * ITEMS + (uint32_t)i * 64u + lane;
        ok[i] = j < cnt;
        rec[i] = ok[i] ? load_rec4<K>(a.rin, off + soff + start + j) : make_uint4(0u, 0u, 0u, 0u);
        dig[i] = (pick4(rec[i], d) >> shift) & MASK;
    }
    auto digit_of = [&](const uint4& r) { return (pick4(r, d) >> shift) & MASK; };
    if (!LAST) {
        sweep_tile<RB, ITEMS, K>(sm, rec, ok, dig, ITEMS, cnt, seg_hist, soff, a.lb, g, g - u, a.o.status, digit_of,
                                 [&](uint32_t, uint32_t pos, const uint4& r) {
                                     if (in_bounds(pos, live, a.o.status)) store_rec4<K>(a.rout, off + pos, r);
                                 });
        zero_range(a.lb_zero, a.lb_zero_n);
        zero_range(a.zero2, a.zero2_n);
        return;
    }
    // tag update (Sec. 3.2) for subtree s = F(l) + seg: the sorted segment is
    // [soff, soff + ssz); the pivot is the entry at soff + ss(2s+1).
    const uint32_t piv = seg_pivot(v, seg);
    const uint32_t s = v.Fl + seg;
    const uint32_t dn = (st.level + 1u) % a.k;
    sweep_tile<RB, ITEMS, K>(
        sm, rec, ok, dig, ITEMS, cnt, seg_hist, soff, a.lb, g, g - u, a.o.status, digit_of,
        [&](uint32_t, uint32_t pos, const uint4& r) {
            if (pos == piv) {
                if (!in_bounds(r.x, ti.n, a.o.status)) return;
                const uint32_t idx = a.o.perm0[off + r.x];
                place<K, WIDEST>(a.o, ti, s, idx);
                if (WIDEST)
                    widest_children<K>(a.o, ti, s, seg, a.o.pts[(off + idx) * K + d], d, a.o.box[st.level & 1u],
                                       a.o.box[(st.level + 1u) & 1u]);
                return;
            }
            const uint32_t side = pos > piv ? 1u : 0u;
            const uint32_t nxt = pos - seg - side;
            if (!in_bounds(pos, live, a.o.status) || !in_bounds(nxt, live - v.nseg, a.o.status)) return;
            store_rec4<K>(a.rout, off + nxt, r);
            if (acc) {
                const uint32_t vv = pick4(r, dn);
                for (uint32_t p = 0; p < NP; ++p)
                    atomicAdd(&nh[(side * NP + p) * NB + ((vv >> (RB * p)) & MASK)], 1u);
            }
        });
    if (acc) {
        // sweep_tile ends with a barrier, so nh is complete; children 2seg and
        // 2seg+1 of the next iteration are adjacent
        uint32_t* dst = a.hist + st.hist_next + (size_t)(2u * seg) * NP * NB;
        for (uint32_t x = threadIdx.x; x < 2u * NP * NB; x += SWEEP_THREADS)
            if (nh[x]) atomicAdd(&dst[x], nh[x]);
    }
    zero_range(a.lb_zero, a.lb_zero_n);
    zero_range(a.zero2, a.zero2_n);
}

template <int K, int RB, int ITEMS>
static void level_pass_kri(const LevelPassArgs& a, uint32_t tiles, bool last, bool widest, hipStream_t st)
{
    if (last) {
        if (widest) k_level_pass<K, true, true, RB, ITEMS><<<tiles, SWEEP_THREADS, 0, st>>>(a);
        else k_level_pass<K, true, false, RB, ITEMS><<<tiles, SWEEP_THREADS, 0, st>>>(a);
    } else {
        if (widest) k_level_pass<K, false, true, RB, ITEMS><<<tiles, SWEEP_THREADS, 0, st>>>(a);
        else k_level_pass<K, false, false, RB, ITEMS><<<tiles, SWEEP_THREADS, 0, st>>>(a);
    }
}

template <int K, int RB>
static void level_pass_kr(const LevelPassArgs& a, uint32_t tiles, bool last, bool widest, hipStream_t st)
{
    switch (a.items) {
    case 4: level_pass_kri<K, RB, 4>(a, tiles, last, widest, st); break;
    default: level_pass_kri<K, RB, 8>(a, tiles, last, widest, st); break;
    }
}

template <int K>
void launch_level_pass_k(const LevelPassArgs& a, uint32_t tiles, bool last, bool widest, hipStream_t st)
{
    switch (a.radix_bits) {
    case 8: level_pass_kr<K, 8>(a, tiles, last, widest, st); break;
    case 9: level_pass_kr<K, 9>(a, tiles, last, widest, st); break;
    default: level_pass_kr<K, 10>(a, tiles, last, widest, st); break;
    }
}

}  // namespace kdt
