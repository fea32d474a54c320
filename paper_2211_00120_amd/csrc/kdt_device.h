// kdt_device.h -- wave64 building blocks shared by the gfx950 kernels.
//
// Everything here is written for CDNA wavefronts of 64 lanes and 256-thread
// workgroups (4 waves).  The radix digit is 8 bits (256 buckets, one per
// thread of the workgroup).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_shares.h"

namespace kdt {

constexpr int BLOCK = 256;
constexpr int NWAVE = BLOCK / 64;
constexpr uint32_t RADIX = 256;
constexpr uint32_t DIGIT_BITS = 8;

// Decoupled look-back status word: 2 flag bits over a 30-bit count.
constexpr uint32_t LB_AGG = 1u << 30;       // tile's own count published
constexpr uint32_t LB_INC = 2u << 30;       // inclusive prefix published
constexpr uint32_t LB_VAL = (1u << 30) - 1u;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// A value every lane of the wave holds alike, moved to a scalar register.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// One bit of a lane-set match: keeps in (lo, hi) -- the two halves of a
// wave64 lane mask -- the lanes whose bit b of v equals this lane's; nv is
// ~v.  With nm = (this lane's bit ? 0 : ~0) the kept set is (ballot ^ nm),
// so a bit costs a shift, a compare and two three-input logic operations
// (no per-lane select between the ballot and its complement).
__device__ __forceinline__ void match_bit(uint32_t nv, uint32_t b, uint32_t& lo, uint32_t& hi)
{
    const uint32_t nm = (uint32_t)((int32_t)(nv << (31u - b)) >> 31);
    const uint64_t bal = __ballot(nm == 0u);
    lo &= (uint32_t)bal ^ nm;
    hi &= (uint32_t)(bal >> 32) ^ nm;
}

// Lanes of this wave whose (valid, digit) equal this lane's: 8 ballots.
__device__ __forceinline__ uint64_t match_digit(uint32_t digit, bool valid)
{
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < (int)DIGIT_BITS; ++b) match_bit(~digit, (uint32_t)b, lo, hi);
    return ((uint64_t)hi << 32) | lo;
}

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t count_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = (int)lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over the 256-thread block.
// `sh` is NWAVE words of LDS.  Contains two barriers.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total = nullptr)
{
    const int lane = (int)lane_id();
    const int w = (int)(threadIdx.x >> 6);
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) {
        const uint32_t t = sh[i];
        if (i < w) base += t;
        tot += t;
    }
    __syncthreads();
    if (total) *total = tot;
    return base + inc - v;
}

// Stable wave-level multisplit of ITEMS items per lane.  Items are in
// "wave-striped" order: item i of lane j is element i*64 + j of the wave's
// chunk, so walking i outer / lanes inner visits the chunk in order and the
// resulting ranks are stable.  wh: this wave's 256 LDS counters, zeroed here.
// On return rank[i] is the item's position among the wave's items with the
// same digit and wh[d] holds the wave's count of digit d.
template <int ITEMS>
__device__ __forceinline__ void wave_multisplit(const uint32_t (&digit)[ITEMS], const bool (&valid)[ITEMS],
                                                uint32_t (&rank)[ITEMS], uint32_t* wh)
{
    for (int j = (int)lane_id(); j < (int)RADIX; j += 64) wh[j] = 0;
    // LDS accesses of one wave complete in issue order, so the counter reads
    // and the leader's update below need no barrier.
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t peers = match_digit(digit[i], valid[i]);
        const uint32_t below = count_below(peers);
        uint32_t base = 0;
        if (valid[i]) base = wh[digit[i]];
        if (valid[i] && below == 0) wh[digit[i]] = base + (uint32_t)__popcll(peers);
        rank[i] = base + below;
    }
}

// Block-level ranking of a tile after wave_multisplit: converts the wave
// counters `wh_all[NWAVE][256]` into exclusive per-wave offsets (in place) and
// returns, for digit t = threadIdx.x, the tile count of that digit; writes the
// exclusive scan over digits into digit_start[t].  Contains barriers.
__device__ __forceinline__ uint32_t tile_digit_counts(uint32_t* wh_all, uint32_t* digit_start, uint32_t* sh)
{
    __syncthreads();
    const uint32_t t = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) {
        const uint32_t c = wh_all[w * RADIX + t];
        wh_all[w * RADIX + t] = run;
        run += c;
    }
    digit_start[t] = block_excl_scan(run, sh);
    return run;
}

__device__ __forceinline__ uint32_t lb_load(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Upper bound on the polls of one look-back wait (each poll sleeps ~64
// clocks plus a device-scope load, so around a second); exceeding it flags an internal error
// instead of spinning forever.
constexpr uint32_t LB_MAX_POLLS = 1u << 20;

// Decoupled look-back for digit t of tile g whose segment starts at tile g0:
// publishes the tile count, walks back to the segment's first tile and
// returns the exclusive prefix of the digit over the segment's earlier tiles.
__device__ __forceinline__ uint32_t lookback(uint32_t* lb, uint32_t g, uint32_t g0, uint32_t t, uint32_t count,
                                             uint32_t* status)
{
    if (g == g0) {
        lb_store(&lb[(size_t)g * RADIX + t], LB_INC | count);
        return 0;
    }
    lb_store(&lb[(size_t)g * RADIX + t], LB_AGG | count);
    uint32_t excl = 0;
    uint32_t gg = g - 1u;
    uint32_t polls = 0;
    for (;;) {
        const uint32_t s = lb_load(&lb[(size_t)gg * RADIX + t]);
        const uint32_t f = s & ~LB_VAL;
        if (f == 0u) {
            if (++polls > LB_MAX_POLLS) {
                atomicOr(status, KDT_STATUS_INTERNAL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += s & LB_VAL;
        if (f == LB_INC || gg == g0) break;
        --gg;
    }
    lb_store(&lb[(size_t)g * RADIX + t], LB_INC | (excl + count));
    return excl;
}

// Order-preserving map of float32 bits to uint32 (-0 folded onto +0, so the
// two compare equal as IEEE says).
__device__ __forceinline__ uint32_t orderable(uint32_t b)
{
    if (b == 0x80000000u) b = 0u;
    return b ^ ((b >> 31) ? 0xFFFFFFFFu : 0x80000000u);
}
__device__ __forceinline__ float from_orderable(uint32_t u)
{
    const uint32_t b = (u & 0x80000000u) ? (u ^ 0x80000000u) : ~u;
    return __uint_as_float(b);
}
__device__ __forceinline__ bool nonfinite(uint32_t b) { return (b & 0x7F800000u) == 0x7F800000u; }

// Order-preserving uint32 key of a coordinate's 32 bits: float32 (orderable
// above) or int32 (sign bit flipped).  Only float32 can be non-finite.
template <bool I32>
__device__ __forceinline__ uint32_t coord_key(uint32_t b)
{
    return I32 ? (b ^ 0x80000000u) : orderable(b);
}
template <bool I32>
__device__ __forceinline__ bool coord_bad(uint32_t b)
{
    return !I32 && nonfinite(b);
}

// Split-widest boxes hold the keys of their bounds, so clipping is unsigned
// min / max for both coordinate types.  The extent hi - lo of one dimension
// is compared as the input type defines it: float32 subtraction of the two
// bounds (round to nearest, no flush to zero, may overflow to +inf) or, for
// int32, the exact difference, which the difference of the keys is.
// Widest extent of a box; lowest dimension on ties.
template <int K, bool I32>
__device__ __forceinline__ uint32_t widest_dim(const uint32_t (&lo)[K], const uint32_t (&hi)[K])
{
    uint32_t best = 0;
    if (I32) {
        uint32_t be = hi[0] - lo[0];
#pragma unroll
        for (int d = 1; d < K; ++d) {
            const uint32_t e = hi[d] - lo[d];
            if (e > be) { be = e; best = (uint32_t)d; }
        }
    } else {
        float be = __fsub_rn(from_orderable(hi[0]), from_orderable(lo[0]));
#pragma unroll
        for (int d = 1; d < K; ++d) {
            const float e = __fsub_rn(from_orderable(hi[d]), from_orderable(lo[d]));
            if (e > be) { be = e; best = (uint32_t)d; }
        }
    }
    return best;
}

}  // namespace kdt
