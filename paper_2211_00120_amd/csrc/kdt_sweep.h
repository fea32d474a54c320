// kdt_sweep.h -- one stable LSD digit pass of a segmented onesweep radix sort.
//
// A tile is up to SWEEP_THREADS*active consecutive elements of ONE segment
// (active <= ITEMS items per thread, chosen per launch).  Its elements are
// held in registers in wave-striped order (item i of lane j of wave w is tile
// element w*64*active + i*64 + j), ranked by digit with wave64 ballots
// (stable), counted per digit, and written out through an LDS stage in
// rounds of SWEEP_STAGE elements so that the global writes of one digit are
// contiguous.  The global position of a digit run is: segment offset + count
// of smaller digits in the segment (from the segment's digit histogram) +
// count of the same digit in the segment's earlier tiles (decoupled
// look-back that stops at the segment's first tile).
//
// Large tiles matter on this part: the look-back reads every digit's status
// word of each predecessor still in flight with device-coherent (uncached)
// loads, and the number of predecessors in flight grows with the tile rate,
// so the status traffic per byte of data falls with the square of the tile
// size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_device.h"
#include "kdt_shares.h"

namespace kdt {

constexpr int SWEEP_WAVES = SWEEP_THREADS / 64;
#ifndef KDT_SWEEP_STAGE
#define KDT_SWEEP_STAGE 8192
#endif
constexpr uint32_t SWEEP_STAGE = KDT_SWEEP_STAGE;

// Predecessor windows of the look-back: a short first window (the common
// case is a nearby inclusive prefix), then wider ones.
#ifndef KDT_LB_FIRST
#define KDT_LB_FIRST 2
#endif
constexpr int LB_FIRST = KDT_LB_FIRST;
#ifndef KDT_LB_WINDOW
#define KDT_LB_WINDOW 2
#endif
constexpr int LB_WINDOW = KDT_LB_WINDOW;

// Element type of the write-out stage for records of RW words: one LDS
// access per record (uint4 also for 3 words).
template <int RW> struct StageOf { using T = uint4; };
template <> struct StageOf<2> { using T = uint2; };
template <> struct StageOf<1> { using T = uint32_t; };

__device__ __forceinline__ void stage_put(uint4& s, const uint4& r) { s = r; }
__device__ __forceinline__ void stage_put(uint2& s, const uint4& r) { s = make_uint2(r.x, r.y); }
__device__ __forceinline__ void stage_put(uint32_t& s, const uint4& r) { s = r.x; }
__device__ __forceinline__ uint4 stage_get(const uint4& s) { return s; }
__device__ __forceinline__ uint4 stage_get(const uint2& s) { return make_uint4(s.x, s.y, 0u, 0u); }
__device__ __forceinline__ uint4 stage_get(const uint32_t& s) { return make_uint4(s, 0u, 0u, 0u); }

template <int RB, int RW, bool STAGE = true>
struct SweepSmem {
    static constexpr uint32_t NB = 1u << RB;
    uint16_t wh[SWEEP_WAVES * NB];   // per-wave digit counters, then per-wave exclusive offsets
    uint32_t dstart[NB];             // tile-local start of each digit run
    uint32_t gbase[NB];              // global position of the run minus dstart
    uint32_t sh[2 * SWEEP_WAVES];
    uint32_t tile;
    typename StageOf<RW>::T stage[STAGE ? SWEEP_STAGE : 1];   // one round of records in sorted tile order
};

// Exclusive scan of one value per thread over a workgroup of NWV waves
// (sh: NWV words of LDS).
template <int NWV = SWEEP_WAVES>
__device__ __forceinline__ uint32_t sweep_excl_scan(uint32_t v, uint32_t* sh)
{
    const int lane = (int)lane_id();
    const int w = (int)(threadIdx.x >> 6);
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint32_t base = 0;
#pragma unroll
    for (int i = 0; i < NWV; ++i)
        if (i < w) base += sh[i];
    __syncthreads();
    return base + inc - v;
}

// Exclusive scans of two values per thread at once (same two barriers).
__device__ __forceinline__ void sweep_excl_scan2(uint32_t a, uint32_t b, uint32_t* sh, uint32_t& ea, uint32_t& eb)
{
    const int lane = (int)lane_id();
    const int w = (int)(threadIdx.x >> 6);
    const uint32_t ia = wave_incl_scan(a);
    const uint32_t ib = wave_incl_scan(b);
    if (lane == 63) {
        sh[w] = ia;
        sh[SWEEP_WAVES + w] = ib;
    }
    __syncthreads();
    uint32_t ba = 0, bb = 0;
#pragma unroll
    for (int i = 0; i < SWEEP_WAVES; ++i)
        if (i < w) {
            ba += sh[i];
            bb += sh[SWEEP_WAVES + i];
        }
    __syncthreads();
    ea = ba + ia - a;
    eb = bb + ib - b;
}

// Pivot search in one digit histogram of a segment (NB counts): the digit
// value whose run holds the key of rank kk (0-based) among the counted keys;
// kk becomes its rank inside that run.  Each thread passes its FIND_BPT
// consecutive counts (load_bins), so that the loads of several digits can be
// issued before the first search.  Workgroup-wide: every thread passes the
// same kk and gets the same result.  sh: 2*SWEEP_WAVES words and sel: 2
// words of LDS.  A histogram that holds fewer than kk + 1 keys flags an
// internal error and yields digit 0.  Contains barriers; ends with one.
constexpr uint32_t FIND_BPT = (MAX_BINS + SWEEP_THREADS - 1) / SWEEP_THREADS;

__device__ __forceinline__ void load_bins(const uint32_t* h, uint32_t NB, uint32_t (&c)[FIND_BPT])
{
    const uint32_t bpt = (NB + SWEEP_THREADS - 1u) / SWEEP_THREADS;
    const uint32_t t0 = threadIdx.x * bpt;
#pragma unroll
    for (uint32_t b = 0; b < FIND_BPT; ++b) c[b] = (b < bpt && t0 + b < NB) ? h[t0 + b] : 0u;
}

__device__ __forceinline__ uint32_t find_bucket(const uint32_t (&c)[FIND_BPT], uint32_t NB, uint32_t& kk,
                                                uint32_t* sh, uint32_t* sel, uint32_t* status)
{
    const uint32_t bpt = (NB + SWEEP_THREADS - 1u) / SWEEP_THREADS;
    const uint32_t t0 = threadIdx.x * bpt;
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t b = 0; b < FIND_BPT; ++b) sum += c[b];
    if (threadIdx.x == 0) sel[0] = 0xFFFFFFFFu;
    // the scan's barriers order the sentinel before the hit's write below
    const uint32_t ex = sweep_excl_scan(sum, sh);
    if (kk >= ex && kk - ex < sum) {
        uint32_t run = ex;
#pragma unroll
        for (uint32_t b = 0; b < FIND_BPT; ++b) {
            if (kk - run < c[b]) {
                sel[0] = t0 + b;
                sel[1] = kk - run;
                break;
            }
            run += c[b];
        }
    }
    __syncthreads();
    uint32_t bk = sel[0];
    uint32_t rest = sel[1];
    __syncthreads();
    if (bk == 0xFFFFFFFFu) {
        if (threadIdx.x == 0) atomicOr(status, KDT_STATUS_INTERNAL);
        bk = 0u;
        rest = 0u;
    }
    kk = uniform(rest);
    return uniform(bk);
}

// find_bucket for one wave on its own (no barriers): each lane takes NB/64
// consecutive counts of h.
__device__ __forceinline__ uint32_t wave_find_bucket(const uint32_t* h, uint32_t NB, uint32_t& kk,
                                                     uint32_t* status)
{
    constexpr uint32_t MAXB = MAX_BINS / 64u;
    const uint32_t lane = lane_id();
    const uint32_t bpl = NB / 64u;
    uint32_t c[MAXB];
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t b = 0; b < MAXB; ++b) {
        c[b] = b < bpl ? h[lane * bpl + b] : 0u;
        sum += c[b];
    }
    const uint32_t ex = wave_incl_scan(sum) - sum;
    const uint64_t hit = __ballot(kk >= ex && kk - ex < sum);
    if (hit == 0u) {
        if (lane == 0) atomicOr(status, KDT_STATUS_INTERNAL);
        kk = 0u;
        return 0u;
    }
    const int src = __builtin_ctzll(hit);
    uint32_t bsel = 0, rest = 0;
    if ((int)lane == src) {
        uint32_t run = ex;
#pragma unroll
        for (uint32_t b = 0; b < MAXB; ++b) {
            if (b < bpl && kk - run < c[b]) {
                bsel = lane * bpl + b;
                rest = kk - run;
                break;
            }
            run += c[b];
        }
    }
    kk = uniform((uint32_t)__shfl((int)rest, src, 64));
    return uniform((uint32_t)__shfl((int)bsel, src, 64));
}

// Stable wave multisplit over RB-bit digits of the first `active` items.
template <int RB, int ITEMS>
__device__ __forceinline__ void wave_multisplit16(const uint32_t (&digit)[ITEMS], const bool (&valid)[ITEMS],
                                                  uint32_t (&rank)[ITEMS], uint16_t* wh, int active)
{
    constexpr uint32_t NB = 1u << RB;
    for (uint32_t j = lane_id(); j < NB; j += 64) wh[j] = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (i >= active) break;
        const uint64_t v = __ballot(valid[i]);
        uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
        for (int b = 0; b < RB; ++b) match_bit(~digit[i], (uint32_t)b, lo, hi);
        const uint64_t peers = ((uint64_t)hi << 32) | lo;
        const uint32_t below = count_below(peers);
        uint32_t base = 0;
        if (valid[i]) base = wh[digit[i]];
        if (valid[i] && below == 0) wh[digit[i]] = (uint16_t)(base + (uint32_t)__popcll(peers));
        rank[i] = base + below;
    }
}

// Decoupled look-back of digit `bin` for tile g (g > g0): sums the published
// counts of tiles g-1, g-2, ... until one with an inclusive prefix (the
// segment's first tile g0 always publishes one).  Predecessor words are
// requested a window at a time; a word that is not published yet is polled
// alone (bounded, see LB_MAX_POLLS).
template <int W>
__device__ __forceinline__ bool lookback_round(const uint32_t* lb, uint32_t NB, uint32_t& gg, uint32_t g0,
                                               uint32_t bin, uint32_t& excl, uint32_t* status)
{
    uint32_t v[W];
#pragma unroll
    for (int j = 0; j < W; ++j) v[j] = (gg >= g0 + (uint32_t)j) ? lb_load(&lb[(size_t)(gg - j) * NB + bin]) : 0u;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        uint32_t s = v[j];
        uint32_t polls = 0;
        while ((s & ~LB_VAL) == 0u) {
            if (++polls > LB_MAX_POLLS) {
                atomicOr(status, KDT_STATUS_INTERNAL);
                return true;
            }
            __builtin_amdgcn_s_sleep(1);
            s = lb_load(&lb[(size_t)(gg - j) * NB + bin]);
        }
        excl += s & LB_VAL;
        if ((s & ~LB_VAL) == LB_INC || gg - j == g0) return true;
    }
    gg -= W;
    return false;
}

__device__ __forceinline__ uint32_t lookback_bin(const uint32_t* lb, uint32_t NB, uint32_t g, uint32_t g0,
                                                 uint32_t bin, uint32_t* status)
{
    uint32_t excl = 0, gg = g - 1u;
    if (lookback_round<LB_FIRST>(lb, NB, gg, g0, bin, excl, status)) return excl;
    while (!lookback_round<LB_WINDOW>(lb, NB, gg, g0, bin, excl, status)) {
    }
    return excl;
}

// The digit pass proper, after the caller has loaded the tile into rec/ok
// (first `active` items per thread) and computed dig.  seg_hist: NB digit
// counts of the whole segment for this pass; seg_off: segment start; lb:
// look-back words of this pass, tile g of a segment whose first tile is g0.
// Calls store(j, pos, r) for every element, j being its tile-local sorted
// index and pos its global position.  With STAGE (many digit values) the
// records go out through LDS in sorted order, consecutive threads taking
// consecutive j; without, each thread stores its own items.  Ends with a
// barrier.
template <int RB, int ITEMS, int RW, class Digit, class Store, bool STAGE = true>
__device__ __forceinline__ void sweep_tile(SweepSmem<RB, RW, STAGE>& sm, const uint4 (&rec)[ITEMS], const bool (&ok)[ITEMS],
                                           const uint32_t (&dig)[ITEMS], int active, uint32_t cnt,
                                           const uint32_t* __restrict__ seg_hist, uint32_t seg_off, uint32_t* lb,
                                           uint32_t g, uint32_t g0, uint32_t* status, Digit digit_of, Store store)
{
    constexpr uint32_t NB = 1u << RB;
    constexpr uint32_t BPT = NB > SWEEP_THREADS ? NB / SWEEP_THREADS : 1u;   // bins per thread (contiguous)
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t t0 = threadIdx.x * BPT;
    const bool has = t0 < NB;
    // the segment's digit counts: from global memory (the staged passes),
    // loaded before the multisplit so that their latency hides behind it;
    // from LDS (the split passes, whose caller writes them just before the
    // call) after its barrier
    uint32_t h[BPT];
#pragma unroll
    for (uint32_t b = 0; b < BPT; ++b) h[b] = (STAGE && has) ? seg_hist[t0 + b] : 0u;
    uint32_t rnk[ITEMS];
    wave_multisplit16<RB, ITEMS>(dig, ok, rnk, sm.wh + w * NB, active);
    __syncthreads();

    // per-digit tile counts and per-wave exclusive offsets
    uint32_t c[BPT];
    uint32_t csum = 0, hsum = 0;
#pragma unroll
    for (uint32_t b = 0; b < BPT; ++b) {
        c[b] = 0;
        if (!has) continue;
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < SWEEP_WAVES; ++ww) {
            const uint32_t x = sm.wh[ww * NB + t0 + b];
            sm.wh[ww * NB + t0 + b] = (uint16_t)run;
            run += x;
        }
        c[b] = run;
        csum += run;
        if (!STAGE) h[b] = seg_hist[t0 + b];
        hsum += h[b];
    }
    // publish this tile's counts first, so successors can go on
    const bool first = (g == g0);
    if (has) {
#pragma unroll
        for (uint32_t b = 0; b < BPT; ++b) lb_store(&lb[(size_t)g * NB + t0 + b], (first ? LB_INC : LB_AGG) | c[b]);
    }
    uint32_t cex, hex;
    sweep_excl_scan2(csum, hsum, sm.sh, cex, hex);
    if (STAGE && cnt <= SWEEP_STAGE) {
        // one staging round: the tile-local digit starts first, then the
        // look-back of the waves that own digits while every wave stages its
        // items (those without digits at once, instead of idling through
        // the look-back), then the write-out
        if (has) {
            uint32_t x = cex;
#pragma unroll
            for (uint32_t b = 0; b < BPT; ++b) {
                sm.dstart[t0 + b] = x;
                x += c[b];
            }
        }
        __syncthreads();
        if (has) {
#pragma unroll
            for (uint32_t b = 0; b < BPT; ++b) {
                const uint32_t bin = t0 + b;
                const uint32_t excl = first ? 0u : lookback_bin(lb, NB, g, g0, bin, status);
                if (!first) lb_store(&lb[(size_t)g * NB + bin], LB_INC | (excl + c[b]));
                sm.gbase[bin] = seg_off + hex + excl - cex;
                cex += c[b];
                hex += h[b];
            }
        }
        // every item's staging position first (the counter reads need no
        // guard: digits are in range), so the reads are in flight together
        uint32_t spos[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = dig[i] & (NB - 1u);
            spos[i] = sm.dstart[d] + sm.wh[w * NB + d] + (i < active ? rnk[i] : 0u);
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (i >= active) break;
            if (ok[i]) stage_put(sm.stage[spos[i]], rec[i]);
        }
        __syncthreads();
        // four sorted positions per thread and round: their staged records
        // and run bases are read before any of them is stored
        constexpr uint32_t U = 4;
        for (uint32_t j0 = threadIdx.x; j0 < cnt; j0 += U * SWEEP_THREADS) {
            uint4 r[U];
            uint32_t gbv[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t j = j0 + u * SWEEP_THREADS;
                r[u] = j < cnt ? stage_get(sm.stage[j]) : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) gbv[u] = sm.gbase[digit_of(r[u]) & (NB - 1u)];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t j = j0 + u * SWEEP_THREADS;
                if (j < cnt) store(j, gbv[u] + j, r[u]);
            }
        }
        __syncthreads();
        return;
    }
    if (has) {
#pragma unroll
        for (uint32_t b = 0; b < BPT; ++b) {
            const uint32_t bin = t0 + b;
            const uint32_t excl = first ? 0u : lookback_bin(lb, NB, g, g0, bin, status);
            if (!first) lb_store(&lb[(size_t)g * NB + bin], LB_INC | (excl + c[b]));
            sm.dstart[bin] = cex;
            sm.gbase[bin] = seg_off + hex + excl - cex;
            cex += c[b];
            hex += h[b];
        }
    }
    __syncthreads();
    uint32_t dst[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t d = dig[i] & (NB - 1u);
        const uint32_t at = sm.dstart[d] + sm.wh[w * NB + d] + (i < active ? rnk[i] : 0u);
        dst[i] = (i < active && ok[i]) ? at : 0xFFFFFFFFu;
    }
    if (!STAGE) {
        // few digit values: each wave's stores of one item already form a
        // few contiguous runs, so they go out straight from the registers
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (i >= active) break;
            if (ok[i]) store(dst[i], sm.gbase[dig[i]] + dst[i], rec[i]);
        }
        __syncthreads();
        return;
    }
    // write-out in rounds of SWEEP_STAGE sorted positions
    for (uint32_t base = 0; base < cnt; base += SWEEP_STAGE) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (i >= active) break;
            const uint32_t o = dst[i] - base;
            if (o < SWEEP_STAGE) stage_put(sm.stage[o], rec[i]);
        }
        __syncthreads();
        const uint32_t m = min(SWEEP_STAGE, cnt - base);
        for (uint32_t j = threadIdx.x; j < m; j += SWEEP_THREADS) {
            const uint4 r = stage_get(sm.stage[j]);
            const uint32_t d = digit_of(r);
            store(base + j, sm.gbase[d] + base + j, r);
        }
        __syncthreads();
    }
}

}  // namespace kdt
