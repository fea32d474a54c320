// kdt_tail.hip -- the deep iterations of the build, one subtree per workgroup.
//
// Once every subtree of iteration l0 holds at most TAIL_CAP points, the
// remaining iterations l0 .. L-2 only ever compare points of the same
// subtree.  Each workgroup therefore takes one (or two) whole level-l0
// subtrees, reads their records from HBM once and runs the rest of the
// paper's loop on them in LDS:
//
//   * once per dimension d, the subtree's points are sorted by rank_d (LDS
//     radix sort of (rank, slot)), giving the list ord_d.  Any subset of the
//     points keeps its relative order in ord_d, so ord_d restricted to a
//     deeper subtree is that subtree's sorted order in dimension d;
//   * iteration l: a point's position inside its subtree segment after the
//     sort of Sec. 3.1 is the number of points of the same segment that
//     precede it in ord_d (d = the segment's split dimension).  Waves walk
//     ord_d with one counter per (wave, segment), ranking lanes of equal
//     segment with ballots;
//   * the tag update of Sec. 3.2 then compares that position with the pivot
//     position ss(2s+1): the pivot is placed at node s, the others move to
//     segment 2q or 2q+1 of the next iteration; at l = L-2 the children are
//     leaves and are placed directly.
//
// The iterations before l0 split every segment stably, so a subtree's input
// is in the root dimension's order, and that dimension needs no sort.
//
// A whole tree of at most TAIL_CAP points is built the same way straight
// from its points (from_points): the per-dimension orders come from a stable
// radix sort of the order-preserving coordinate keys (float32 or int32)
// starting in index order, so equal coordinates keep index order, and the
// loop starts at iteration 0.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_common.h"
#include "kdt_device.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"
#include "kdt_sweep.h"

namespace kdt {

constexpr uint32_t DONE = 0xFFFFu;

// Domain of local node (t, q) for split-widest: the box of its ancestor on
// local level t0 <= t (box0, indexed by that ancestor's position: the group
// roots' boxes for t0 = 0) clipped by the planes of its ancestors below
// (stored per local node); all bounds and planes are coordinate keys (see
// widest_dim).
template <int K>
__device__ __forceinline__ void local_box(uint32_t t, uint32_t q, uint32_t gc, uint32_t t0, const uint32_t (*box0)[8],
                                          const uint8_t* ndim, const uint32_t* nplane, uint32_t (&lo)[K],
                                          uint32_t (&hi)[K])
{
    const uint32_t r = q >> (t - t0);
#pragma unroll
    for (int d = 0; d < K; ++d) {
        lo[d] = box0[r][d];
        hi[d] = box0[r][4 + d];
    }
    uint32_t qq = q;
    // the steps' LDS reads do not depend on each other: unrolled, they are
    // issued together instead of one round trip per ancestor
#pragma unroll 4
    for (uint32_t tt = t; tt > t0; --tt) {
        const uint32_t pq = qq >> 1;
        const uint32_t idx = gc * ((1u << (tt - 1u)) - 1u) + pq;
        const uint32_t da = ndim[idx];
        const uint32_t plane = nplane[idx];
#pragma unroll
        for (int d = 0; d < K; ++d) {
            if ((uint32_t)d == da) {
                if ((qq & 1u) == 0u) hi[d] = min(hi[d], plane);
                else lo[d] = max(lo[d], plane);
            }
        }
        qq = pq;
    }
}

constexpr uint32_t TAIL_SORT_BINS = 512;       // LDS sort digits of up to 9 bits

// Digit offsets of one LDS sort pass over NB digit values: wh[w*NB + digit]
// holds wave w's count of each digit; it becomes wave w's exclusive offset
// inside the digit's run, and dstart[digit] the run's start.  Contains
// barriers.
template <uint32_t NB>
__device__ __forceinline__ void tail_digit_offsets(uint16_t* wh, uint32_t* dstart, uint32_t* sh)
{
    const uint32_t t = threadIdx.x;
    uint32_t run = 0;
    if (t < NB) {
#pragma unroll
        for (int ww = 0; ww < TAIL_THREADS / 64; ++ww) {
            const uint32_t x = wh[ww * NB + t];
            wh[ww * NB + t] = (uint16_t)run;
            run += x;
        }
    }
    const uint32_t ex = sweep_excl_scan<TAIL_THREADS / 64>(run, sh);
    if (t < NB) dstart[t] = ex;
}

// One stable LSD pass of the group's LDS sort: it[] (key above bit 12, slot
// below) ordered by the digit (it >> sft) & mask, mask < TAIL_SORT_BINS.
template <int ITEMS>
__device__ __forceinline__ void tail_sort_pass(uint64_t (&it)[ITEMS], const bool (&ok)[ITEMS], uint32_t sft,
                                               uint32_t mask, uint64_t* x, uint16_t* wh, uint32_t* dstart,
                                               uint32_t* sh)
{
    constexpr uint32_t NB = TAIL_SORT_BINS;
    constexpr uint32_t CW = 64u * ITEMS;
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    uint32_t dig[ITEMS], rnk[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) dig[i] = (uint32_t)(it[i] >> sft) & mask;
    wave_multisplit16<9, ITEMS>(dig, ok, rnk, wh + w * NB, ITEMS);
    __syncthreads();
    tail_digit_offsets<NB>(wh, dstart, sh);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (ok[i]) x[dstart[dig[i]] + wh[w * NB + dig[i]] + rnk[i]] = it[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * CW + (uint32_t)i * 64u + lane;
        if (ok[i]) it[i] = x[p];
    }
    __syncthreads();
}

// Bucket sort of one dimension's keys of the group, for keys spread over
// their range (ranks of a subtree's points are): bucket = (key - min) >>
// shift, with at most TB_BUCKETS buckets; a key's slot inside its bucket
// comes from an LDS atomic, and its place inside the bucket from counting
// the bucket's smaller keys (equal keys by slot, i.e. input order).  Gives
// up, leaving ord untouched, when a bucket holds more than TB_FILL keys.
// All threads call it; it starts and ends with a barrier.
constexpr uint32_t TB_BITS = 11;
constexpr uint32_t TB_BUCKETS = 1u << TB_BITS;
constexpr uint32_t TB_FILL = 32;

template <int ITEMS>
__device__ __forceinline__ bool tail_bucket_sort(const uint32_t (&key)[ITEMS], const bool (&ok)[ITEMS],
                                                 uint16_t* ordd, uint32_t* bc, uint32_t* tk, uint16_t* ts,
                                                 uint32_t* red, uint32_t* sh)
{
    constexpr int NW = TAIL_THREADS / 64;
    constexpr uint32_t CW = 64u * ITEMS;
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (!ok[i]) continue;
        lo = min(lo, key[i]);
        hi = max(hi, key[i]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        red[0] = 0xFFFFFFFFu;
        red[1] = 0u;
        red[2] = 0u;
    }
    for (uint32_t x = threadIdx.x; x <= TB_BUCKETS; x += TAIL_THREADS) bc[x] = 0u;
    __syncthreads();
    if (lane == 0) {
        atomicMin(&red[0], lo);
        atomicMax(&red[1], hi);
    }
    __syncthreads();
    const uint32_t kmin = red[0];
    const uint32_t range = red[1] - kmin;
    const uint32_t rbits = range ? 32u - (uint32_t)__builtin_clz(range) : 0u;
    const uint32_t shift = rbits > TB_BITS ? rbits - TB_BITS : 0u;
    uint32_t b[ITEMS], at[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        b[i] = ok[i] ? (key[i] - kmin) >> shift : 0u;
        at[i] = ok[i] ? atomicAdd(&bc[b[i]], 1u) : 0u;
    }
    __syncthreads();
    // bucket starts (exclusive scan, 4 buckets per thread) and the fullest bucket
    constexpr uint32_t BPT = TB_BUCKETS / TAIL_THREADS;
    const uint32_t t0 = threadIdx.x * BPT;
    uint32_t c[BPT];
    uint32_t sum = 0, mx = 0;
#pragma unroll
    for (uint32_t j = 0; j < BPT; ++j) {
        c[j] = bc[t0 + j];
        sum += c[j];
        mx = max(mx, c[j]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if (lane == 0) atomicMax(&red[2], mx);
    const uint32_t ex = sweep_excl_scan<NW>(sum, sh);
    uint32_t run = ex;
#pragma unroll
    for (uint32_t j = 0; j < BPT; ++j) {
        bc[t0 + j] = run;
        run += c[j];
    }
    if (threadIdx.x == TAIL_THREADS - 1) bc[TB_BUCKETS] = run;
    __syncthreads();
    if (red[2] > TB_FILL) {
        __syncthreads();
        return false;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
        if (!ok[i]) continue;
        const uint32_t j = bc[b[i]] + at[i];
        tk[j] = key[i];
        ts[j] = (uint16_t)e;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
        if (!ok[i]) continue;
        const uint32_t st = bc[b[i]], en = bc[b[i] + 1u];
        uint32_t r = 0;
        for (uint32_t j = st; j < en; ++j) {
            const uint32_t k2 = tk[j];
            r += (k2 < key[i] || (k2 == key[i] && (uint32_t)ts[j] < e)) ? 1u : 0u;
        }
        ordd[st + r] = (uint16_t)e;
    }
    __syncthreads();
    return true;
}

// The group's rank keys of ND dimensions bucket-sorted together.  As
// tail_bucket_sort, but for ranks: they are unique, so a bucket's keys need
// no tie-break and only their low 16 bits (the bucket fixes the rest when the
// bucket shift is at most 16); bucket counters and starts are 16-bit.  The ND
// sorts then fit the LDS of one and share its barriers.  rec holds the keys
// (dimension dims[j] of record i), bcp ND * TB_BUCKETS / 2 words, tk ND *
// TAIL_CAP halves, red 3 * ND words, sh ND * (TAIL_THREADS / 64) words.
// Returns the dimensions it sorted (bit d for dimension d): one whose shift
// exceeds 16 or whose fullest bucket holds more than TB_FILL keys is left to
// the caller.  All threads call it; it starts and ends with a barrier.
template <int ITEMS, int ND>
__device__ __forceinline__ uint32_t tail_bucket_sort_ranks(const uint4 (&rec)[ITEMS], const bool (&ok)[ITEMS],
                                                           uint16_t (*ord)[TAIL_CAP], const uint32_t (&dims)[ND],
                                                           uint32_t m, uint32_t* bcp, uint16_t* tk, uint32_t* red,
                                                           uint32_t* sh)
{
    constexpr int NW = TAIL_THREADS / 64;
    constexpr uint32_t CW = 64u * ITEMS;
    constexpr uint32_t HB = TB_BUCKETS / 2u;                 // counter words of one dimension
    static_assert(TB_BUCKETS == 4u * TAIL_THREADS, "four buckets per thread");
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    uint32_t lo[ND], hi[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        lo[j] = 0xFFFFFFFFu;
        hi[j] = 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (!ok[i]) continue;
            const uint32_t k = pick4(rec[i], dims[j]);
            lo[j] = min(lo[j], k);
            hi[j] = max(hi[j], k);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            lo[j] = min(lo[j], (uint32_t)__shfl_xor((int)lo[j], o, 64));
            hi[j] = max(hi[j], (uint32_t)__shfl_xor((int)hi[j], o, 64));
        }
    __syncthreads();
    if (threadIdx.x < (uint32_t)ND) {
        red[3 * threadIdx.x] = 0xFFFFFFFFu;
        red[3 * threadIdx.x + 1] = 0u;
        red[3 * threadIdx.x + 2] = 0u;
    }
    for (uint32_t x = threadIdx.x; x < ND * HB; x += TAIL_THREADS) bcp[x] = 0u;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            atomicMin(&red[3 * j], lo[j]);
            atomicMax(&red[3 * j + 1], hi[j]);
        }
    __syncthreads();
    uint32_t kmin[ND], shift[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        kmin[j] = red[3 * j];
        const uint32_t range = red[3 * j + 1] - kmin[j];
        const uint32_t rbits = range ? 32u - (uint32_t)__builtin_clz(range) : 0u;
        shift[j] = rbits > TB_BITS ? rbits - TB_BITS : 0u;
    }
    // each key's place in its bucket's arrival order (two 16-bit places a
    // word: items 2h and 2h+1); the bucket is recomputed from the key
    auto bucket = [&](int j, int i) { return (pick4(rec[i], dims[j]) - kmin[j]) >> shift[j]; };
    uint32_t pl[ND][(ITEMS + 1) / 2];
#pragma unroll
    for (int j = 0; j < ND; ++j)
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if ((i & 1) == 0) pl[j][i / 2] = 0u;
            if (!ok[i]) continue;
            const uint32_t b = bucket(j, i);
            const uint32_t half = 16u * (b & 1u);
            const uint32_t old = atomicAdd(&bcp[j * HB + (b >> 1)], 1u << half);
            pl[j][i / 2] |= ((old >> half) & 0xFFFFu) << (16 * (i & 1));
        }
    __syncthreads();
    // bucket starts: four consecutive buckets per thread and dimension (the
    // counts are read again after the barrier rather than kept live)
    uint32_t ex[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        const uint32_t w0 = bcp[j * HB + 2u * threadIdx.x], w1 = bcp[j * HB + 2u * threadIdx.x + 1u];
        const uint32_t sum = (w0 & 0xFFFFu) + (w0 >> 16) + (w1 & 0xFFFFu) + (w1 >> 16);
        uint32_t mx = max(max(w0 & 0xFFFFu, w0 >> 16), max(w1 & 0xFFFFu, w1 >> 16));
        const uint32_t inc = wave_incl_scan(sum);
        ex[j] = inc - sum;
        if (lane == 63) sh[j * NW + w] = inc;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        if (lane == 0) atomicMax(&red[3 * j + 2], mx);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        uint32_t s0 = ex[j];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww)
            if (ww < (int)w) s0 += sh[j * NW + ww];
        const uint32_t w0 = bcp[j * HB + 2u * threadIdx.x], w1 = bcp[j * HB + 2u * threadIdx.x + 1u];
        const uint32_t s1 = s0 + (w0 & 0xFFFFu), s2 = s1 + (w0 >> 16), s3 = s2 + (w1 & 0xFFFFu);
        bcp[j * HB + 2u * threadIdx.x] = s0 | (s1 << 16);
        bcp[j * HB + 2u * threadIdx.x + 1u] = s2 | (s3 << 16);
    }
    __syncthreads();
    uint32_t done = 0;
#pragma unroll
    for (int j = 0; j < ND; ++j)
        if (shift[j] <= 16u && red[3 * j + 2] <= TB_FILL) done |= 1u << dims[j];
    auto start_of = [&](int j, uint32_t b) { return (bcp[j * HB + (b >> 1)] >> (16u * (b & 1u))) & 0xFFFFu; };
    // the keys' low 16 bits (relative to the minimum) by bucket; each
    // dimension's bucket starts are read for all items before any store
    // (the stores might otherwise alias the next item's read and wait)
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        if (!((done >> dims[j]) & 1u)) continue;
        uint32_t at[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) at[i] = start_of(j, bucket(j, i) & (TB_BUCKETS - 1u));
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (!ok[i]) continue;
            const uint32_t place = (pl[j][i / 2] >> (16 * (i & 1))) & 0xFFFFu;
            tk[j * TAIL_CAP + at[i] + place] = (uint16_t)(pick4(rec[i], dims[j]) - kmin[j]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        if (!((done >> dims[j]) & 1u)) continue;
        uint32_t st[ITEMS], en[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t b = bucket(j, i) & (TB_BUCKETS - 1u);
            st[i] = start_of(j, b);
            en[i] = b + 1u < TB_BUCKETS ? start_of(j, b + 1u) : m;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (!ok[i]) continue;
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            const uint32_t mine = (pick4(rec[i], dims[j]) - kmin[j]) & 0xFFFFu;
            uint32_t r = 0;
            for (uint32_t x = st[i]; x < en[i]; ++x) r += (uint32_t)tk[j * TAIL_CAP + x] < mine ? 1u : 0u;
            ord[dims[j]][st[i] + r] = (uint16_t)e;
        }
    }
    __syncthreads();
    return done;
}

template <int K, bool WIDEST, bool I32>
__global__ void __launch_bounds__(TAIL_THREADS, 4) k_tail(TailArgs a)
{
    constexpr int ITEMS = TAIL_ITEMS;
    constexpr int NW = TAIL_THREADS / 64;
    constexpr uint32_t C = TAIL_CAP;
    constexpr uint32_t CW = 64u * ITEMS;           // slots (and list positions) per wave
    // local nodes: every segment of every tail iteration is non-empty, so a
    // group fixes at most C of them
    constexpr uint32_t NODES = WIDEST ? C : 1u;
    __shared__ uint16_t ord[K][C];
    __shared__ uint16_t seg[C];
    __shared__ uint16_t tmp[C];
    __shared__ union __attribute__((aligned(16))) {
        struct {
            uint64_t x[C];                         // sort exchange
            uint16_t wh[NW * TAIL_SORT_BINS];      // per-wave digit counters
            uint32_t dstart[TAIL_SORT_BINS];
        } sort;
        struct {
            uint32_t bc[TB_BUCKETS + 1];           // bucket counts, then starts
            uint32_t tk[C];                        // keys in bucket order
            uint16_t ts[C];                        // their slots
        } bsort;
        struct {
            uint32_t bcp[(K > 1 ? K - 1 : 1) * TB_BUCKETS / 2];   // packed 16-bit bucket counts, then starts
            uint16_t tk[(K > 1 ? K - 1 : 1) * C];                  // low key bits in bucket order
        } rsort;
        uint16_t cnt[NW][C];                       // per-(wave, segment) counters of an iteration
        uint32_t stage[4 * C];                     // write-out: coordinates by local node
    } ub;
    __shared__ uint32_t sh[(K > 1 ? K - 1 : 1) * NW];
    __shared__ uint32_t red[3 * (K > 1 ? K - 1 : 1)];
    __shared__ uint8_t segdim[2][WIDEST ? C : 1];
    __shared__ uint16_t wl[WIDEST ? C : 1];        // split-widest: the iteration's walk list
    __shared__ __attribute__((aligned(16))) uint32_t lcnt[WIDEST ? K : 1][NW];   // split-widest: walk-list slots per (dimension, wave)
    __shared__ uint32_t dmask[2];                  // split-widest: bit d set if some segment splits in d
    __shared__ uint8_t ndim[NODES];
    __shared__ uint32_t nplane[NODES];             // keys of the fixed local nodes' planes
    __shared__ uint32_t rootbox[2][8];             // keys of the group roots' domains
    // split-widest: the domains of the TBOX nodes of local level log2(TBOX /
    // gc), so that deeper domains clip from there, not from the roots
    constexpr uint32_t TBOX = 128;
    __shared__ uint32_t tbox[WIDEST ? TBOX : 1][8];
    __shared__ uint32_t bxk[8];                    // from_points split-widest: scene box keys

    const Outs& o = a.o;
    if (a.init_status) {                           // one workgroup, one tree: it clears its status words itself
        if (threadIdx.x == 0) {
            *o.status = 0u;
            o.tstatus[0] = 0u;
        }
        __syncthreads();
    }
    // with an XCD map, workgroup b (on XCD b mod 8) takes the group the map
    // gives it: a tree's groups all on one XCD, whose L2 then holds the
    // tree's index list and points for the gathers; padding takes none
    const uint32_t grp = a.xmap ? a.xmap[blockIdx.x] : blockIdx.x;
    if (grp == 0xFFFFFFFFu) return;
    TreeStep stp;
    TreeInfo ti;
    find_share(a.sh, grp, stp, ti);
    const bool FP = a.from_points != 0u;
    const size_t off = ti.off;
    const Level v0 = make_level(ti.n, FP ? 0u : stp.level);
    const uint32_t l0 = v0.l;
    const uint32_t L = v0.L;
    uint32_t i0, i1;
    tail_group_range(grp - stp.tile0, stp.pair0, v0.nseg, i0, i1);
    const uint32_t gc = i1 - i0;
    const uint32_t live0 = v0.n - v0.Fl;
    const uint32_t off0 = FP ? 0u : seg_offset(v0, i0);
    const uint32_t m = FP ? ti.n : ((i1 == v0.nseg) ? live0 : seg_offset(v0, i1)) - off0;
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint32_t B = FP ? 32u : rank_bits(ti.n);    // ranks of this tree are < n
    if (m > C) {                                   // the host sizes groups to fit
        if (threadIdx.x == 0) atomicOr(o.status, KDT_STATUS_INTERNAL);
        return;
    }

    // ---- load the group (slot e = its position in the input) ----
    uint4 rec[ITEMS];                              // per-dimension sort keys of each slot
    uint32_t idx[ITEMS];                           // original (local) index of each slot
    float4 pc[ITEMS];                              // coordinates of each slot's point
    uint32_t lid[ITEMS];                           // local node of each slot, once placed (see the write-out)
    uint32_t sq[ITEMS];                            // each slot's segment (its owner's copy of seg)
    bool ok[ITEMS];
    bool bad = false;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) ok[i] = w * CW + (uint32_t)i * 64u + lane < m;
    if (FP) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            idx[i] = e;
            pc[i] = ok[i] ? load_point<K>(o.pts, off + e) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            const float cf[4] = {pc[i].x, pc[i].y, pc[i].z, pc[i].w};
            uint32_t kk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int d = 0; d < K; ++d) {
                const uint32_t bits = __float_as_uint(cf[d]);
                bad |= ok[i] && coord_bad<I32>(bits);
                kk[d] = coord_key<I32>(bits);
            }
            rec[i] = ok[i] ? make_uint4(kk[0], kk[1], kk[2], kk[3]) : make_uint4(0u, 0u, 0u, 0u);
            sq[i] = ok[i] ? 0u : DONE;
            seg[e] = (uint16_t)sq[i];
        }
    } else {
        // the records (the root dimension's slot holds the point's index:
        // the segments are in that dimension's order), then the segment of
        // every slot (the points follow after the sorts)
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            rec[i] = ok[i] ? load_rec4<K>(a.rin[stp.buf & 1u], off + off0 + e) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            sq[i] = ok[i] ? seg_of_pos(v0, off0 + e) - i0 : DONE;
            seg[e] = (uint16_t)sq[i];
        }
    }
    if (FP) {
        if (__any(bad) && lane == 0) {
            atomicOr(o.status, KDT_STATUS_NONFINITE);
            atomicOr(&o.tstatus[stp.tree], KDT_STATUS_NONFINITE);
        }
        if (WIDEST) {
            // scene box of the tree (keys)
            if (threadIdx.x < 8) bxk[threadIdx.x] = threadIdx.x < 4 ? 0xFFFFFFFFu : 0u;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                if (!ok[i]) continue;
#pragma unroll
                for (int d = 0; d < K; ++d) {
                    atomicMin(&bxk[d], pick4(rec[i], (uint32_t)d));
                    atomicMax(&bxk[4 + d], pick4(rec[i], (uint32_t)d));
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t lo[K], hi[K];
#pragma unroll
                for (int d = 0; d < K; ++d) {
                    lo[d] = bxk[d];
                    hi[d] = bxk[4 + d];
                    rootbox[0][d] = lo[d];
                    rootbox[0][4 + d] = hi[d];
                }
                const uint32_t d0 = widest_dim<K, I32>(lo, hi);
                segdim[0][0] = (uint8_t)d0;
                dmask[0] = 1u << d0;
                dmask[1] = 0u;
                o.dimnode[off] = (uint8_t)d0;
            }
        }
        // a single point is the root
        if (L < 2u && ok[0] && threadIdx.x == 0) place_pt<K, WIDEST>(o, ti, 0u, idx[0], pc[0]);
    }
    if (!FP && WIDEST && threadIdx.x < gc) {
        // domain of each group root, written by its parent's pivot
        const uint32_t q = threadIdx.x;
        const uint32_t* bx = o.box[l0 & 1u] + ((size_t)ti.box_off + i0 + q) * 8;
#pragma unroll
        for (int d = 0; d < 8; ++d) rootbox[q][d] = bx[d];
        segdim[0][q] = o.dimnode[off + v0.Fl + i0 + q];
        if (q == 0) {
            uint32_t dm = 0;
            for (uint32_t r = 0; r < gc; ++r) dm |= 1u << o.dimnode[off + v0.Fl + i0 + r];
            dmask[0] = dm;
            dmask[1] = 0u;
        }
    }
    // dimension whose order the input already has (within every segment):
    // the root's
    uint32_t free_dim = 0xFFFFFFFFu;
    if (!FP) free_dim = WIDEST ? (uint32_t)o.dimnode[off] : 0u;
    __syncthreads();

    // ---- ord_d: the group sorted by rank_d: bucket sort, or where the keys
    // bunch, stable LSD radix in LDS with the fewest passes over the B key
    // bits (digits of at most 9 bits) ----
    const uint32_t nsb = ((B + 7u) / 8u == (B + 8u) / 9u) ? 8u : 9u;
    // ranks (unique keys): the dimensions but the free one in one bucket sort
    uint32_t sorted = 0;
    if constexpr (K > 1) {
        if (!FP) {
            uint32_t dims[K - 1];
#pragma unroll
            for (int j = 0; j < K - 1; ++j) dims[j] = (uint32_t)j + ((uint32_t)j >= free_dim ? 1u : 0u);
            sorted = tail_bucket_sort_ranks<ITEMS, K - 1>(rec, ok, ord, dims, m, ub.rsort.bcp, ub.rsort.tk, red, sh);
        }
    }
    for (uint32_t d = 0; d < (uint32_t)K; ++d) {
        if (d == free_dim) {
            for (uint32_t p = threadIdx.x; p < m; p += TAIL_THREADS) ord[d][p] = (uint16_t)p;
            continue;
        }
        if ((sorted >> d) & 1u) continue;
        uint32_t key[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) key[i] = pick4(rec[i], d);
        if (tail_bucket_sort<ITEMS>(key, ok, ord[d], ub.bsort.bc, ub.bsort.tk, ub.bsort.ts, red, sh)) continue;
        uint64_t it[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            it[i] = ((uint64_t)key[i] << 12) | e;
        }
        for (uint32_t sft = 12; sft < 12 + B; sft += nsb)
            tail_sort_pass<ITEMS>(it, ok, sft, (1u << nsb) - 1u, ub.sort.x, ub.sort.wh, ub.sort.dstart, sh);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = w * CW + (uint32_t)i * 64u + lane;
            if (ok[i]) ord[d][p] = (uint16_t)(it[i] & 0xFFFu);
        }
    }
    __syncthreads();

    if (!FP) {
        // the points of the slots, by the index in the root dimension's slot
        // of each record (taken only now: not live across the sorts); an
        // index out of range -- a corrupt input record -- is flagged and its
        // slot reads point 0
        bool oob = false;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            idx[i] = ok[i] ? pick4(rec[i], free_dim) : 0xFFFFFFFFu;
            const bool in = idx[i] < ti.n;
            oob |= ok[i] && !in;
            if (!in) idx[i] = 0u;
            pc[i] = ok[i] ? load_point<K>(o.pts, off + idx[i]) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (__any(oob) && lane == 0) atomicOr(o.status, KDT_STATUS_INTERNAL);
    }
    // split-widest, while the segments split in several dimensions: seg[e]
    // of a live slot holds, beside its segment (below 2048), the segment's
    // split dimension in bits 12-13, which the walk list reads
    auto pack_dims = [&](uint32_t cs) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            if (sq[i] != DONE) seg[e] = (uint16_t)(sq[i] | ((uint32_t)segdim[cs][sq[i]] << 12));
        }
    };
    if (WIDEST) {
        const uint32_t dm = dmask[0];
        if (dm & (dm - 1u)) pack_dims(0u);
    }

    // ---- iterations l0 .. L-2 ----
    uint32_t cur = 0;
    for (uint32_t l = l0; l + 2u <= L; ++l) {
        const uint32_t t = l - l0;
        const Level vl = make_level(ti.n, l);
        const uint32_t S = gc << t;                       // group segments on this level
        const uint32_t gbits = rank_bits(S);
        const bool last = (l + 2u == L);
        {
            // the counters of the S segments, eight to a 16-byte store (C
            // is a multiple of 8, so rounding S up stays inside each row)
            const uint32_t per = (S + 7u) >> 3;
            uint4* z = reinterpret_cast<uint4*>(&ub.cnt[0][0]);
            for (uint32_t x = threadIdx.x; x < NW * per; x += TAIL_THREADS) {
                const uint32_t ww = x / per;
                z[ww * (C / 8u) + (x - ww * per)] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
        __syncthreads();
        // split-widest: do all segments of this iteration split in one
        // dimension (then the walk list is that dimension's order itself)?
        // The previous domain step (or the set-up) collected their dimensions
        uint32_t dall = 0;
        bool uni = false;
        if (WIDEST) {
            const uint32_t dm = dmask[cur];
            dall = dm ? (uint32_t)__builtin_ctz(dm) : 0u;
            uni = (dm & (dm - 1u)) == 0u;
            if (threadIdx.x == 0) dmask[cur ^ 1u] = 0u;   // filled by this iteration's domain step
        }
        // position of each point inside its segment in the order of the
        // segment's split dimension: a walk over a list in which each
        // segment's points appear in that order -- ord_d itself for round
        // robin and for split-widest iterations whose segments all split in
        // one dimension; otherwise the concatenation over d of the slots of
        // the segments split in d, each part in ord_d order
        uint32_t M = m;
        if (WIDEST && !uni) {
            // one read of every (dimension, slot), kept for the write-out
            uint32_t le[K][ITEMS];
            uint64_t lb[K][ITEMS];
#pragma unroll
            for (int d = 0; d < K; ++d) {
                uint32_t c = 0;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t p = w * CW + (uint32_t)i * 64u + lane;
                    const uint32_t e = p < m ? (uint32_t)ord[d][p] : 0u;
                    const uint32_t v = p < m ? (uint32_t)seg[e] : DONE;
                    le[d][i] = e;
                    lb[d][i] = __ballot(v != DONE && (v >> 12) == (uint32_t)d);
                    c += (uint32_t)__popcll(lb[d][i]);
                }
                if (lane == 0) lcnt[d][w] = c;
            }
            __syncthreads();
            uint32_t base = 0;
            static_assert(NW % 4 == 0, "walk-list counts are read four at a time");
#pragma unroll
            for (int d = 0; d < K; ++d) {
                uint32_t b = base;
#pragma unroll
                for (int w4 = 0; w4 < NW / 4; ++w4) {
                    const uint4 c4 = reinterpret_cast<const uint4*>(&lcnt[d][0])[w4];
                    const uint32_t cc[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        b += (uint32_t)(4 * w4 + j) < w ? cc[j] : 0u;
                        base += cc[j];
                    }
                }
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    if ((lb[d][i] >> lane) & 1u) wl[b + count_below(lb[d][i])] = (uint16_t)le[d][i];
                    b += (uint32_t)__popcll(lb[d][i]);
                }
            }
            M = base;
            __syncthreads();
        }
        {
            const uint32_t d = WIDEST ? dall : l % (uint32_t)K;     // the split dimension of every segment
            uint32_t e[ITEMS], q[ITEMS];
            bool valid[ITEMS];
            uint32_t plo[ITEMS], phi[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t p = w * CW + (uint32_t)i * 64u + lane;
                e[i] = p < M ? (uint32_t)((WIDEST && !uni) ? wl[p] : ord[d][p]) : 0u;
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t p = w * CW + (uint32_t)i * 64u + lane;
                const uint32_t v = p < M ? (uint32_t)seg[e[i]] : DONE;
                q[i] = v == DONE ? DONE : (v & 0xFFFu);
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                valid[i] = q[i] != DONE;
                const uint64_t v = __ballot(valid[i]);
                plo[i] = (uint32_t)v;
                phi[i] = (uint32_t)(v >> 32);
            }
            for (uint32_t b = 0; b < gbits; ++b) {
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) match_bit(~q[i], b, plo[i], phi[i]);
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint64_t peers = ((uint64_t)phi[i] << 32) | plo[i];
                const uint32_t below = count_below(peers);
                uint32_t base = 0;
                if (valid[i]) base = ub.cnt[w][q[i]];
                if (valid[i] && below == 0) ub.cnt[w][q[i]] = (uint16_t)(base + (uint32_t)__popcll(peers));
                if (valid[i]) tmp[e[i]] = (uint16_t)((w << 12) | (base + below));
            }
        }
        __syncthreads();
        // two segments' counters to a 32-bit word (an odd S scans one
        // zeroed counter past the end, which nothing reads)
        for (uint32_t q2 = threadIdx.x; 2u * q2 < S; q2 += TAIL_THREADS) {
            uint32_t run0 = 0, run1 = 0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                uint32_t* c2 = reinterpret_cast<uint32_t*>(&ub.cnt[ww][2u * q2]);
                const uint32_t c = *c2;
                *c2 = run0 | (run1 << 16);
                run0 += c & 0xFFFFu;
                run1 += c >> 16;
            }
        }
        __syncthreads();
        // tag update (Sec. 3.2): each slot's owner learns its node or child
        // segment.  All loads first: a store to seg may alias a later
        // slot's load, which would otherwise wait for it
        uint32_t tv[ITEMS], cw[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            tv[i] = sq[i] != DONE ? (uint32_t)tmp[e] : 0u;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) cw[i] = sq[i] != DONE ? (uint32_t)ub.cnt[tv[i] >> 12][sq[i]] : 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = w * CW + (uint32_t)i * 64u + lane;
            const uint32_t q = sq[i];
            if (q == DONE) continue;
            const uint32_t wr = (tv[i] & 0xFFFu) + cw[i];
            const uint32_t gq = (i0 << t) + q;
            const uint32_t ls = seg_left_size(vl, gq);
            if (wr == ls) {
                lid[i] = gc * ((1u << t) - 1u) + q;
                if (WIDEST) {
                    // the node's dimension and plane; its children follow
                    // below, one thread per segment
                    const uint32_t ds = segdim[cur][q];
                    const uint32_t nidx = gc * ((1u << t) - 1u) + q;
                    ndim[nidx] = (uint8_t)ds;
                    nplane[nidx] = coord_key<I32>(__float_as_uint(pickf(pc[i], ds)));
                }
                sq[i] = DONE;
            } else {
                const uint32_t side = wr > ls ? 1u : 0u;
                if (last) {
                    lid[i] = gc * ((2u << t) - 1u) + 2u * q + side;
                    sq[i] = DONE;
                } else {
                    sq[i] = 2u * q + side;
                }
            }
            seg[e] = (uint16_t)sq[i];
        }
        __syncthreads();
        if (WIDEST) {
            // each segment's children: domain = the segment's domain (root
            // box clipped by its ancestors' planes) clipped by its own plane;
            // while the segments are at most half the threads, one thread per
            // child (both walk the segment's ancestors), else one per segment
            uint32_t used = 0;                     // dimensions of the children this thread set
            const uint32_t ts = 31u - (uint32_t)__builtin_clz(TBOX / gc);   // local level of the tbox nodes
            auto children = [&](uint32_t q, uint32_t c0, uint32_t c1) {
                const uint32_t gq = (i0 << t) + q;
                const uint32_t sn = vl.Fl + gq;
                const uint32_t nidx = gc * ((1u << t) - 1u) + q;
                const uint32_t ds = ndim[nidx];
                const uint32_t plane = nplane[nidx];
                uint32_t lo[K], hi[K];
                const bool deep = t >= ts;
                local_box<K>(t, q, gc, deep ? ts : 0u, deep ? tbox : rootbox, ndim, nplane, lo, hi);
                for (uint32_t c = c0; c < c1; ++c) {
                    const uint32_t child = 2u * sn + 1u + c;
                    if (child >= ti.n) continue;
                    uint32_t l2[K], h2[K];
#pragma unroll
                    for (int dd = 0; dd < K; ++dd) {
                        l2[dd] = lo[dd];
                        h2[dd] = hi[dd];
                        if ((uint32_t)dd == ds) {
                            if (c == 0u) h2[dd] = min(hi[dd], plane);
                            else l2[dd] = max(lo[dd], plane);
                        }
                    }
                    const uint32_t cd = widest_dim<K, I32>(l2, h2);
                    o.dimnode[off + child] = (uint8_t)cd;
                    if (!last) {
                        segdim[cur ^ 1u][2u * q + c] = (uint8_t)cd;
                        used |= 1u << cd;
                        if (t + 1u == ts) {
#pragma unroll
                            for (int dd = 0; dd < K; ++dd) {
                                tbox[2u * q + c][dd] = l2[dd];
                                tbox[2u * q + c][4 + dd] = h2[dd];
                            }
                        }
                    }
                }
            };
            if (2u * S <= TAIL_THREADS) {
                if (threadIdx.x < 2u * S) children(threadIdx.x >> 1, threadIdx.x & 1u, (threadIdx.x & 1u) + 1u);
            } else {
                for (uint32_t q = threadIdx.x; q < S; q += TAIL_THREADS) children(q, 0u, 2u);
            }
            if (!last) {
                uint32_t wm = 0;
#pragma unroll
                for (int d = 0; d < K; ++d)
                    if (__any((used >> d) & 1u)) wm |= 1u << d;
                if (lane == 0 && wm) atomicOr(&dmask[cur ^ 1u], wm);
            }
            // the next iteration reads segdim and dmask after its first barrier
            if (!last) {
                __syncthreads();
                const uint32_t dm = dmask[cur ^ 1u];
                if (dm & (dm - 1u)) pack_dims(cur ^ 1u);
            }
        }
        cur ^= 1u;
    }

    // ---- write-out (Sec. 3.2's placement, made coalesced): local node id
    // p numbers the group's nodes level by level, gc * (2^t - 1) + j for the
    // j-th node of local level t, whose global node is F(l0 + t) + i0 * 2^t
    // + j; the last level holds only its existing nodes, so the ids of the m
    // slots are exactly 0 .. m-1.  The slots' points and indices go to LDS
    // by id, then every thread writes consecutive nodes of each level ----
    if (l0 + 2u <= L) {
        // ub and tmp/seg were last read before the final iteration's update
        // barrier; the domain step after it touches neither
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (!ok[i]) continue;
            const uint32_t q = lid[i];
            const float cf[4] = {pc[i].x, pc[i].y, pc[i].z, pc[i].w};
#pragma unroll
            for (int d = 0; d < K; ++d) ub.stage[(uint32_t)d * C + q] = __float_as_uint(cf[d]);
            tmp[q] = (uint16_t)(idx[i] & 0xFFFFu);
            seg[q] = (uint16_t)(idx[i] >> 16);
        }
        __syncthreads();
        // every thread's (at most C / TAIL_THREADS) nodes read from LDS
        // before the first store
        constexpr int R = (int)(C / TAIL_THREADS);
        uint32_t cv[R][K], ix[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const uint32_t p = threadIdx.x + (uint32_t)u * TAIL_THREADS;
            const uint32_t pp = p < m ? p : 0u;
#pragma unroll
            for (int d = 0; d < K; ++d) cv[u][d] = ub.stage[(uint32_t)d * C + pp];
            ix[u] = (uint32_t)tmp[pp] | ((uint32_t)seg[pp] << 16);
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const uint32_t p = threadIdx.x + (uint32_t)u * TAIL_THREADS;
            if (p >= m) continue;
            const uint32_t t = 31u - (uint32_t)__builtin_clz(p / gc + 1u);
            const uint32_t node = full_nodes(l0 + t) + (i0 << t) + (p - gc * ((1u << t) - 1u));
            if (!in_bounds(node, ti.n, o.status)) continue;
            const size_t at = off + node;
            if (o.tree) {
                float* tp = o.tree + at * K;
                if constexpr (K == 4)
                    *reinterpret_cast<float4*>(tp) = make_float4(__uint_as_float(cv[u][0]), __uint_as_float(cv[u][1]),
                                                                 __uint_as_float(cv[u][2]), __uint_as_float(cv[u][3]));
                else
#pragma unroll
                    for (int d = 0; d < K; ++d) tp[d] = __uint_as_float(cv[u][d]);
            }
            o.nodeperm[at] = ix[u];
            if (!WIDEST && o.dim) o.dim[at] = (uint8_t)((l0 + t) % (uint32_t)K);
        }
    }
}

template <int K>
static void tail_k(const TailArgs& a, uint32_t groups, bool widest, hipStream_t st)
{
    // a coordinate is read as a key only by whole trees and split-widest
    const bool i32 = a.o.i32 && (widest || a.from_points);
    if (i32) {
        if (widest) k_tail<K, true, true><<<groups, TAIL_THREADS, 0, st>>>(a);
        else k_tail<K, false, true><<<groups, TAIL_THREADS, 0, st>>>(a);
    } else {
        if (widest) k_tail<K, true, false><<<groups, TAIL_THREADS, 0, st>>>(a);
        else k_tail<K, false, false><<<groups, TAIL_THREADS, 0, st>>>(a);
    }
}

void launch_tail(int k, const TailArgs& a, uint32_t groups, bool widest, hipStream_t st)
{
    switch (k) {
    case 1: tail_k<1>(a, groups, widest, st); break;
    case 2: tail_k<2>(a, groups, widest, st); break;
    case 3: tail_k<3>(a, groups, widest, st); break;
    default: tail_k<4>(a, groups, widest, st); break;
    }
}

}  // namespace kdt
