// kdt_kernels.hip -- gfx950 kernels of the left-balanced k-d tree build.
//
// Data flow of one build (all device-resident):
//
//  prep        one read of the points: order-preserving uint32 key per
//              coordinate (SoA), non-finite flag, scene box (split-widest) and
//              the digit histograms of every presort pass.
//  presort     for each dimension d a stable LSD radix sort (4 onesweep passes
//              over 8-bit digits) of (key_d, index); its output gives the
//              dense rank of every point in the order (coordinate, index).
//              Comparing ranks is comparing (coordinate, index), the total
//              order the build sorts by (Sec. 3.1 plus the index tie-break).
//  level 0     the presort of the root's dimension already is the iteration-0
//              sort (all tags are 0), so iteration 0 is only the tag update:
//              place the root at the pivot ss(1), write the rest compacted.
//  level l     the live points are grouped by subtree (Obs. 3.2), so the sort
//              by (tag, coordinate) only has to order each subtree's segment
//              by the rank of its split dimension: segmented onesweep passes
//              over the rank digits, with tiles that never straddle a segment
//              and look-back that stops at the segment's first tile.  The last
//              pass is fused with the tag update (Sec. 3.2): each point's
//              sorted position decides pivot / left / right, pivots are placed
//              at their node, the others are written compacted for the next
//              iteration (position p - i - [p > pivot]).
//  deep levels once a whole subtree segment fits in one workgroup, each
//              workgroup sorts whole segments in LDS and applies the update in
//              the same kernel (one read and one write per iteration).
//
// Records carried through the iterations are the k per-dimension ranks of a
// point (k uint32, array of structs); the float points are only read by prep,
// by the placement of fixed nodes and by the split-widest plane lookups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_common.h"
#include "kdt_device.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"
#include "kdt_sweep.h"

namespace kdt {

// --------------------------------------------------------------------- init

__global__ void __launch_bounds__(BLOCK) k_init(uint32_t* ctl, uint32_t* counters, uint32_t* z1, uint32_t n1,
                                                uint32_t* z2, uint32_t n2, uint32_t* z3, uint32_t n3)
{
    const uint32_t gid = blockIdx.x * BLOCK + threadIdx.x;
    if (gid < CTL_WORDS) {
        uint32_t v = 0u;
        if (gid >= CTL_BOX_LO && gid < CTL_BOX_LO + 4) v = 0xFFFFFFFFu;   // running minimum
        ctl[gid] = v;
    }
    if (gid < MAX_PASSES) counters[gid] = 0u;
    zero_range(z1, n1);
    zero_range(z2, n2);
    zero_range(z3, n3);
}

// --------------------------------------------------------------------- prep

// One read of the points: uint32 keys (SoA, keys[d*n + i]), non-finite flag,
// scene box (as orderable keys) and the 4 digit histograms of every
// dimension's presort (hist[(d*4 + pass)*256 + digit]).
template <int K, bool WIDEST>
__global__ void __launch_bounds__(BLOCK) k_prep(const float* __restrict__ pts, uint32_t n, uint32_t* __restrict__ keys,
                                                uint32_t* __restrict__ hist, uint32_t* __restrict__ ctl)
{
    __shared__ uint32_t sh[K * 4 * RADIX];
    __shared__ uint32_t s_lo[K], s_hi[K];
    for (uint32_t x = threadIdx.x; x < K * 4 * RADIX; x += BLOCK) sh[x] = 0u;
    if (threadIdx.x < K) { s_lo[threadIdx.x] = 0xFFFFFFFFu; s_hi[threadIdx.x] = 0u; }
    __syncthreads();
    uint32_t lo[K], hi[K];
#pragma unroll
    for (int d = 0; d < K; ++d) { lo[d] = 0xFFFFFFFFu; hi[d] = 0u; }
    bool bad = false;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
#pragma unroll
        for (int d = 0; d < K; ++d) {
            const uint32_t b = __float_as_uint(pts[(size_t)i * K + d]);
            bad |= nonfinite(b);
            const uint32_t u = orderable(b);
            keys[(size_t)d * n + i] = u;
            if (WIDEST) { lo[d] = min(lo[d], u); hi[d] = max(hi[d], u); }
#pragma unroll
            for (int p = 0; p < 4; ++p) atomicAdd(&sh[(d * 4 + p) * RADIX + ((u >> (8 * p)) & 0xFFu)], 1u);
        }
    }
    if (__any(bad) && lane_id() == 0) atomicOr(&ctl[CTL_STATUS], (uint32_t)KDT_STATUS_NONFINITE);
    if (WIDEST) {
#pragma unroll
        for (int d = 0; d < K; ++d) {
            atomicMin(&s_lo[d], lo[d]);
            atomicMax(&s_hi[d], hi[d]);
        }
    }
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < K * 4 * RADIX; x += BLOCK)
        if (sh[x]) atomicAdd(&hist[x], sh[x]);
    if (WIDEST && threadIdx.x < K) {
        atomicMin(&ctl[CTL_BOX_LO + threadIdx.x], s_lo[threadIdx.x]);
        atomicMax(&ctl[CTL_BOX_HI + threadIdx.x], s_hi[threadIdx.x]);
    }
}

// Split-widest: scene box back to floats, root dimension (Sec. 6).
template <int K>
__global__ void k_root_dim(uint32_t* ctl, uint8_t* dimnode, float* box0)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float lo[K], hi[K];
#pragma unroll
    for (int d = 0; d < K; ++d) {
        lo[d] = from_orderable(ctl[CTL_BOX_LO + d]);
        hi[d] = from_orderable(ctl[CTL_BOX_HI + d]);
        ctl[CTL_SCENE_LO + d] = __float_as_uint(lo[d]);
        ctl[CTL_SCENE_HI + d] = __float_as_uint(hi[d]);
    }
    const uint32_t d0 = widest_dim<K>(lo, hi);
    ctl[CTL_DIM0] = d0;
    dimnode[0] = (uint8_t)d0;
#pragma unroll
    for (int d = 0; d < K; ++d) {
        box0[d] = lo[d];
        box0[4 + d] = hi[d];
    }
}

// ------------------------------------------------------------ presort passes

// One stable LSD digit pass of the (key, index) sort of one dimension.
// FIRST reads the keys of prep and takes the index as value; LAST writes the
// sorted indices (rank -> index) and scatters each index's rank into the
// point-major rank table.  Pairs are stored interleaved (uint2).
template <bool FIRST, bool LAST>
__global__ void __launch_bounds__(SWEEP_THREADS) k_presort_pass(PresortArgs a)
{
    constexpr int ITEMS = PRESORT_ITEMS;
    constexpr int RB = 8;
    constexpr uint32_t T = SWEEP_THREADS * ITEMS;
    __shared__ SweepSmem<RB, 2> sm;

    if (threadIdx.x == 0) sm.tile = atomicAdd(a.counter, 1u);
    __syncthreads();
    const uint32_t g = sm.tile;
    const uint32_t start = g * T;
    const uint32_t cnt = min(T, a.n - start);
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint32_t shift = a.shift;

    uint4 rec[ITEMS];
    uint32_t dig[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = w * 64u * ITEMS + (uint32_t)i * 64u + lane;
        ok[i] = j < cnt;
        rec[i] = make_uint4(0u, 0u, 0u, 0u);
        if (ok[i]) {
            if (FIRST) {
                rec[i].x = a.kin[start + j];
                rec[i].y = start + j;
            } else {
                const uint2 kv = reinterpret_cast<const uint2*>(a.kvin)[start + j];
                rec[i].x = kv.x;
                rec[i].y = kv.y;
            }
        }
        dig[i] = (rec[i].x >> shift) & 0xFFu;
    }
    const uint32_t n = a.n;
    sweep_tile<RB, ITEMS, 2>(
        sm, rec, ok, dig, ITEMS, cnt, a.hist, 0u, a.lb, g, 0u, a.status,
        [&](const uint4& r) { return (r.x >> shift) & 0xFFu; },
        [&](uint32_t, uint32_t pos, const uint4& r) {
            if (!in_bounds(pos, n, a.status) || !in_bounds(r.y, n, a.status)) return;
            if (LAST) {
                a.perm_out[pos] = r.y;
                a.rank_table[(size_t)r.y * a.k + a.dim] = pos;
            } else {
                reinterpret_cast<uint2*>(a.kvout)[pos] = make_uint2(r.x, r.y);
            }
        });
    // clear the next pass's look-back words (nothing waits on these stores)
    zero_range(a.lb_zero, a.lb_zero_n);
}

// ------------------------------------------------------------------ level 0

// Iteration 0: every tag is 0 and the presort of the root's dimension is the
// sorted order, so array position r holds the point of rank r.  The pivot is
// ss(1) (Sec. 3.2, Sec. 5); the root is placed, the others keep their order
// and are written compacted (left subtree then right subtree).  With N <= 3
// the children are leaves and are placed directly.  Optionally accumulates
// the digit histograms of iteration 1 (round robin).
template <int K, bool WIDEST>
__global__ void __launch_bounds__(BLOCK) k_level0(Level0Args a)
{
    __shared__ uint32_t nh[2 * MAX_LEVEL_PASSES * MAX_BINS];
    const uint32_t P = a.next_passes;
    const uint32_t RBv = a.radix_bits;
    const uint32_t NB = 1u << RBv;
    const bool acc = a.hist_next != nullptr;
    if (acc)
        for (uint32_t x = threadIdx.x; x < 2u * P * NB; x += BLOCK) nh[x] = 0u;
    __syncthreads();
    const uint32_t n = a.o.n;
    const uint32_t L = num_levels(n);
    const uint32_t d0 = WIDEST ? a.o.ctl[CTL_DIM0] : 0u;
    const uint32_t* perm_d0 = a.perms + (size_t)d0 * n;
    const uint32_t piv = (L >= 2) ? seg_pivot(make_level(n, 0), 0) : 0u;
    const uint32_t dn = (K == 1) ? 0u : 1u % (uint32_t)K;
    for (uint32_t r = blockIdx.x * BLOCK + threadIdx.x; r < n; r += gridDim.x * BLOCK) {
        const uint32_t idx = perm_d0[r];
        if (r == piv) {
            place<K, WIDEST>(a.o, 0u, idx);
            if (WIDEST && L >= 2) widest_children<K>(a.o, 0u, 0u, idx, d0, a.o.box[0], L > 2 ? a.o.box[1] : nullptr);
            continue;
        }
        if (L == 2) {                       // N = 2 or 3: children are leaves
            place<K, WIDEST>(a.o, r < piv ? 1u : 2u, idx);
            continue;
        }
        uint32_t rec[K];
        load_rec<K>(a.rank_table, idx, rec);
        const uint32_t side = r > piv ? 1u : 0u;
        store_rec<K>(a.rout, r - side, rec);
        if (acc) {
            const uint32_t u = pick<K>(rec, dn);
            for (uint32_t p = 0; p < P; ++p)
                atomicAdd(&nh[(side * P + p) * NB + ((u >> (RBv * p)) & (NB - 1u))], 1u);
        }
    }
    if (acc) {
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < 2u * P * NB; x += BLOCK)
            if (nh[x]) atomicAdd(&a.hist_next[x], nh[x]);
    }
}

// ------------------------------------------------------ segmented level pass

// Digit histograms of iteration l for split-widest (the split dimension of a
// subtree is only known once its parent's pivot is fixed).  Blocks cover
// segment-aligned chunks of the live array.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_level_hist(LevelHistArgs a)
{
    __shared__ uint32_t h[MAX_LEVEL_PASSES * MAX_BINS];
    const uint32_t P = a.passes;
    const uint32_t RBv = a.radix_bits;
    const uint32_t NB = 1u << RBv;
    for (uint32_t x = threadIdx.x; x < P * NB; x += BLOCK) h[x] = 0u;
    __syncthreads();
    uint32_t seg, u;
    tile_locate(a.tl, blockIdx.x, seg, u);
    const uint32_t off = tiles_seg_offset(a.tl, seg);
    const uint32_t sz = tiles_seg_size(a.tl, seg);
    const uint32_t start = u * a.tl.tile;
    const uint32_t cnt = min(a.tl.tile, sz - start);
    const uint32_t d = a.dimnode[a.v.Fl + seg];
    for (uint32_t j = threadIdx.x; j < cnt; j += BLOCK) {
        const uint32_t r = a.rin[(size_t)(off + start + j) * K + d];
        for (uint32_t p = 0; p < P; ++p) atomicAdd(&h[p * NB + ((r >> (RBv * p)) & (NB - 1u))], 1u);
    }
    __syncthreads();
    uint32_t* dst = a.hist + (size_t)seg * P * NB;
    for (uint32_t x = threadIdx.x; x < P * NB; x += BLOCK)
        if (h[x]) atomicAdd(&dst[x], h[x]);
}

template <int K>
void launch_level_pass_k(const LevelPassArgs& a, bool last, bool widest, hipStream_t st);

void launch_level_pass(int k, const LevelPassArgs& a, bool last, bool widest, hipStream_t st)
{
    switch (k) {
    case 1: launch_level_pass_k<1>(a, last, widest, st); break;
    case 2: launch_level_pass_k<2>(a, last, widest, st); break;
    case 3: launch_level_pass_k<3>(a, last, widest, st); break;
    default: launch_level_pass_k<4>(a, last, widest, st); break;
    }
}

__global__ void k_set_word(uint32_t* dst, uint32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}
__global__ void k_copy_word(uint32_t* dst, const uint32_t* src)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

// ------------------------------------------------------------- launchers

void launch_set_word(uint32_t* dst, uint32_t value, hipStream_t st) { k_set_word<<<1, 64, 0, st>>>(dst, value); }
void launch_copy_word(uint32_t* dst, const uint32_t* src, hipStream_t st) { k_copy_word<<<1, 64, 0, st>>>(dst, src); }

template <int K>
static void launch_prep_k(const float* pts, uint32_t n, uint32_t* keys, uint32_t* hist, uint32_t* ctl, bool widest,
                          uint32_t grid, hipStream_t st)
{
    if (widest) k_prep<K, true><<<grid, BLOCK, 0, st>>>(pts, n, keys, hist, ctl);
    else k_prep<K, false><<<grid, BLOCK, 0, st>>>(pts, n, keys, hist, ctl);
}

void launch_init(uint32_t* ctl, uint32_t* counters, uint32_t* z1, uint32_t n1, uint32_t* z2, uint32_t n2,
                 uint32_t* z3, uint32_t n3, hipStream_t st)
{
    uint32_t m = CTL_WORDS > MAX_PASSES ? CTL_WORDS : MAX_PASSES;
    uint32_t big = n1 > n2 ? n1 : n2;
    big = big > n3 ? big : n3;
    uint32_t grid = ceil_div(m > big ? m : big, BLOCK);
    if (grid > 2048) grid = 2048;
    if (grid == 0) grid = 1;
    k_init<<<grid, BLOCK, 0, st>>>(ctl, counters, z1, n1, z2, n2, z3, n3);
}

void launch_prep(int k, const float* pts, uint32_t n, uint32_t* keys, uint32_t* hist, uint32_t* ctl, bool widest,
                 hipStream_t st)
{
    uint32_t grid = ceil_div(n, BLOCK * 16u);
    if (grid > 4096) grid = 4096;
    if (grid == 0) grid = 1;
    switch (k) {
    case 1: launch_prep_k<1>(pts, n, keys, hist, ctl, widest, grid, st); break;
    case 2: launch_prep_k<2>(pts, n, keys, hist, ctl, widest, grid, st); break;
    case 3: launch_prep_k<3>(pts, n, keys, hist, ctl, widest, grid, st); break;
    default: launch_prep_k<4>(pts, n, keys, hist, ctl, widest, grid, st); break;
    }
}

void launch_root_dim(int k, uint32_t* ctl, uint8_t* dimnode, float* box0, hipStream_t st)
{
    switch (k) {
    case 1: k_root_dim<1><<<1, 64, 0, st>>>(ctl, dimnode, box0); break;
    case 2: k_root_dim<2><<<1, 64, 0, st>>>(ctl, dimnode, box0); break;
    case 3: k_root_dim<3><<<1, 64, 0, st>>>(ctl, dimnode, box0); break;
    default: k_root_dim<4><<<1, 64, 0, st>>>(ctl, dimnode, box0); break;
    }
}

void launch_presort_pass(const PresortArgs& a, bool first, bool last, uint32_t tiles, hipStream_t st)
{
    if (first && last) k_presort_pass<true, true><<<tiles, SWEEP_THREADS, 0, st>>>(a);
    else if (first) k_presort_pass<true, false><<<tiles, SWEEP_THREADS, 0, st>>>(a);
    else if (last) k_presort_pass<false, true><<<tiles, SWEEP_THREADS, 0, st>>>(a);
    else k_presort_pass<false, false><<<tiles, SWEEP_THREADS, 0, st>>>(a);
}

template <int K>
static void level0_k(const Level0Args& a, bool widest, uint32_t grid, hipStream_t st)
{
    if (widest) k_level0<K, true><<<grid, BLOCK, 0, st>>>(a);
    else k_level0<K, false><<<grid, BLOCK, 0, st>>>(a);
}

void launch_level0(int k, const Level0Args& a, bool widest, hipStream_t st)
{
    uint32_t grid = ceil_div(a.o.n, BLOCK * 8u);
    if (grid > 2048) grid = 2048;
    if (grid == 0) grid = 1;
    switch (k) {
    case 1: level0_k<1>(a, widest, grid, st); break;
    case 2: level0_k<2>(a, widest, grid, st); break;
    case 3: level0_k<3>(a, widest, grid, st); break;
    default: level0_k<4>(a, widest, grid, st); break;
    }
}

void launch_level_hist(int k, const LevelHistArgs& a, hipStream_t st)
{
    const uint32_t grid = a.tl.tiles;
    switch (k) {
    case 1: k_level_hist<1><<<grid, BLOCK, 0, st>>>(a); break;
    case 2: k_level_hist<2><<<grid, BLOCK, 0, st>>>(a); break;
    case 3: k_level_hist<3><<<grid, BLOCK, 0, st>>>(a); break;
    default: k_level_hist<4><<<grid, BLOCK, 0, st>>>(a); break;
    }
}

}  // namespace kdt
