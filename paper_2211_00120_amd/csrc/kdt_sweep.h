// kdt_sweep.h -- one stable LSD digit pass of a segmented onesweep radix sort.
//
// A tile is up to BLOCK*ITEMS consecutive elements of ONE segment.  Its
// elements are held in registers in wave-striped order (item i of lane j of
// wave w is tile element w*64*ITEMS + i*64 + j), ranked by digit with wave64
// ballots (stable), counted per digit, and scattered through LDS so that the
// global writes of one digit are contiguous.  The global position of a digit
// run is: segment offset + count of smaller digits in the segment (from the
// segment's digit histogram) + count of the same digit in the segment's
// earlier tiles (decoupled look-back that stops at the segment's first tile).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_device.h"

namespace kdt {

template <int RB, int ITEMS, int RW>
struct SweepSmem {
    static constexpr uint32_t NB = 1u << RB;
    static constexpr uint32_t T = BLOCK * ITEMS;
    uint32_t wh[NWAVE * NB];     // per-wave digit counters, then per-wave exclusive offsets
    uint32_t dstart[NB];         // tile-local start of each digit run
    uint32_t gbase[NB];          // global position of the run minus dstart
    uint32_t sh[NWAVE];
    uint32_t tile;
    uint32_t stage[RW][T];       // records in sorted tile order
};

// Stable wave multisplit over RB-bit digits (see wave_multisplit).
template <int RB, int ITEMS>
__device__ __forceinline__ void wave_multisplit_rb(const uint32_t (&digit)[ITEMS], const bool (&valid)[ITEMS],
                                                   uint32_t (&rank)[ITEMS], uint32_t* wh)
{
    constexpr uint32_t NB = 1u << RB;
    for (uint32_t j = lane_id(); j < NB; j += 64) wh[j] = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        uint64_t peers = __ballot(valid[i]);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const bool bit = (digit[i] >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = count_below(peers);
        uint32_t base = 0;
        if (valid[i]) base = wh[digit[i]];
        if (valid[i] && below == 0) wh[digit[i]] = base + (uint32_t)__popcll(peers);
        rank[i] = base + below;
    }
}

// Number of predecessor tiles whose look-back words are fetched at once.
#ifndef KDT_LB_WINDOW
#define KDT_LB_WINDOW 16
#endif
constexpr int LB_WINDOW = KDT_LB_WINDOW;

// Decoupled look-back of digit `bin` for tile g (g > g0): sums the published
// counts of tiles g-1, g-2, ... until one with an inclusive prefix (the
// segment's first tile g0 always publishes one).  The words of LB_WINDOW
// predecessors are requested together, so a long chain of aggregates costs
// one memory round trip per window instead of one per tile; a word that is not
// published yet is polled alone (bounded, see LB_MAX_POLLS).
__device__ __forceinline__ uint32_t lookback_window(const uint32_t* lb, uint32_t NB, uint32_t g, uint32_t g0,
                                                    uint32_t bin, uint32_t* status)
{
    uint32_t excl = 0;
    uint32_t gg = g - 1u;          // next predecessor to consume
    for (;;) {
        uint32_t v[LB_WINDOW];
#pragma unroll
        for (int j = 0; j < LB_WINDOW; ++j)
            v[j] = (gg >= g0 + (uint32_t)j) ? lb_load(&lb[(size_t)(gg - j) * NB + bin]) : 0u;
#pragma unroll
        for (int j = 0; j < LB_WINDOW; ++j) {
            uint32_t s = v[j];
            uint32_t polls = 0;
            while ((s & ~LB_VAL) == 0u) {
                if (++polls > LB_MAX_POLLS) {
                    atomicOr(status, 0x100u);
                    return excl;
                }
                __builtin_amdgcn_s_sleep(1);
                s = lb_load(&lb[(size_t)(gg - j) * NB + bin]);
            }
            excl += s & LB_VAL;
            if ((s & ~LB_VAL) == LB_INC || gg - j == g0) return excl;
        }
        gg -= LB_WINDOW;
    }
}

// The digit pass proper, after the caller has loaded the tile into rec/ok
// and computed dig.  seg_hist: NB digit counts of the whole segment for this
// pass; seg_off: segment start; lb: look-back words of this pass, tile g of a
// segment whose first tile is g0.  Calls store(j, pos, r) for every element,
// j being its tile-local sorted index (consecutive threads get consecutive j)
// and pos its global position.
template <int RB, int ITEMS, int RW, class Digit, class Store>
__device__ __forceinline__ void sweep_tile(SweepSmem<RB, ITEMS, RW>& sm, const uint4 (&rec)[ITEMS],
                                           const bool (&ok)[ITEMS], const uint32_t (&dig)[ITEMS], uint32_t cnt,
                                           const uint32_t* __restrict__ seg_hist, uint32_t seg_off, uint32_t* lb,
                                           uint32_t g, uint32_t g0, uint32_t* status, Digit digit_of, Store store)
{
    constexpr uint32_t NB = 1u << RB;
    constexpr uint32_t BPT = NB / BLOCK;      // bins per thread (contiguous)
    static_assert(NB % BLOCK == 0, "digit bins must be a multiple of the block size");
    const uint32_t w = threadIdx.x >> 6;
    uint32_t rnk[ITEMS];
    wave_multisplit_rb<RB, ITEMS>(dig, ok, rnk, sm.wh + w * NB);
    __syncthreads();

    // per-digit tile counts and per-wave exclusive offsets
    const uint32_t t0 = threadIdx.x * BPT;
    uint32_t c[BPT], h[BPT];
    uint32_t csum = 0, hsum = 0;
#pragma unroll
    for (uint32_t b = 0; b < BPT; ++b) {
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < NWAVE; ++ww) {
            const uint32_t x = sm.wh[ww * NB + t0 + b];
            sm.wh[ww * NB + t0 + b] = run;
            run += x;
        }
        c[b] = run;
        csum += run;
        h[b] = seg_hist[t0 + b];
        hsum += h[b];
    }
    // publish this tile's counts before anything else, so successors can go on
    const bool first = (g == g0);
#pragma unroll
    for (uint32_t b = 0; b < BPT; ++b) lb_store(&lb[(size_t)g * NB + t0 + b], (first ? LB_INC : LB_AGG) | c[b]);
    uint32_t cex = block_excl_scan(csum, sm.sh);
    uint32_t hex = block_excl_scan(hsum, sm.sh);
#pragma unroll
    for (uint32_t b = 0; b < BPT; ++b) {
        const uint32_t bin = t0 + b;
        const uint32_t excl = first ? 0u : lookback_window(lb, NB, g, g0, bin, status);
        if (!first) lb_store(&lb[(size_t)g * NB + bin], LB_INC | (excl + c[b]));
        sm.dstart[bin] = cex;
        sm.gbase[bin] = seg_off + hex + excl - cex;
        cex += c[b];
        hex += h[b];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (ok[i]) {
            const uint32_t dst = sm.dstart[dig[i]] + sm.wh[w * NB + dig[i]] + rnk[i];
            sm.stage[0][dst] = rec[i].x;
            if constexpr (RW > 1) sm.stage[1][dst] = rec[i].y;
            if constexpr (RW > 2) sm.stage[2][dst] = rec[i].z;
            if constexpr (RW > 3) sm.stage[3][dst] = rec[i].w;
        }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += BLOCK) {
        uint4 r = make_uint4(sm.stage[0][j], 0u, 0u, 0u);
        if constexpr (RW > 1) r.y = sm.stage[1][j];
        if constexpr (RW > 2) r.z = sm.stage[2][j];
        if constexpr (RW > 3) r.w = sm.stage[3][j];
        const uint32_t d = digit_of(r);
        store(j, sm.gbase[d] + j, r);
    }
}

}  // namespace kdt
