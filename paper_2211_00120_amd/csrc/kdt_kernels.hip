// kdt_kernels.hip -- gfx950 kernels of the left-balanced k-d tree build
// (everything but the level passes, kdt_level*.hip, and the tail,
// kdt_tail.hip).
//
// Data flow of one build (all device-resident, per tree of the call):
//
//  prep        one read of the points: order-preserving uint32 key per
//              coordinate (SoA), non-finite flag, scene box (split-widest) and
//              the digit histograms of every presort pass.
//  presort     for each dimension d a stable LSD radix sort (4 onesweep passes
//              over 8-bit digits) of (key_d, local index); its output gives
//              the dense rank of every point in the order (coordinate, index).
//              Comparing ranks is comparing (coordinate, index), the total
//              order the build sorts by (Sec. 3.1 plus the index tie-break).
//  level 0     the presort of the root's dimension already is the iteration-0
//              sort (all tags are 0), so iteration 0 is only the tag update:
//              place the root at the pivot ss(1), write the rest compacted.
//  level l     the live points are grouped by subtree (Obs. 3.2) and every
//              subtree's segment is still in the root dimension's order.  The
//              tag update only asks where each point falls relative to its
//              subtree's pivot, so the sort by (tag, coordinate) reduces to a
//              radix select of the pivot's key (k_level_select, digit
//              histograms per subtree) and one stable three-way split around
//              it that applies the update (kdt_level.h).
//  tail        once every subtree fits one workgroup, the remaining
//              iterations run in LDS (kdt_tail.hip).
//
// Records carried through the iterations are the k per-dimension ranks of a
// point (k uint32, array of structs); the float points are only read by prep,
// by the placement of fixed nodes and by the split-widest plane lookups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kdt_common.h"
#include "kdt_device.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"
#include "kdt_sweep.h"

namespace kdt {

// --------------------------------------------------------------------- init

__global__ void __launch_bounds__(BLOCK) k_init(uint32_t* status, uint32_t* counters, uint32_t* z1, uint32_t n1,
                                                uint32_t* z2, uint32_t n2, uint32_t* z3, uint32_t n3,
                                                uint32_t* z4, uint32_t n4, uint32_t* z5, uint32_t n5,
                                                uint32_t* bbox, uint32_t nbox)
{
    const uint32_t gid = blockIdx.x * BLOCK + threadIdx.x;
    if (gid == 0) *status = 0u;
    if (gid < MAX_COUNTERS) counters[gid] = 0u;
    zero_range(z1, n1);
    zero_range(z2, n2);
    zero_range(z3, n3);
    zero_range(z4, n4);
    zero_range(z5, n5);
    // per-tree scene boxes as running (min, max) of orderable keys
    // per-tree key summaries: running minima and ANDs start all ones, maxima
    // and ORs all zeros
    for (uint32_t x = gid; x < nbox * KEYSUM_WORDS; x += gridDim.x * BLOCK) bbox[x] = (x & 4u) ? 0u : 0xFFFFFFFFu;
}

// --------------------------------------------------------------------- prep

// One tile of one tree: uint32 keys (SoA), non-finite flag, the tree's key
// summary (scene box for split-widest; the bits that are not the same in
// every key) and the 4 digit histograms of every dimension's presort.
// I32: the coordinates are int32 (order-preserving key: sign bit flipped).
#ifndef KDT_PREP_COPIES
#define KDT_PREP_COPIES 2
#endif
template <int K, bool WIDEST, bool I32>
__global__ void __launch_bounds__(BLOCK) k_prep(PrepArgs a)
{
    // digit counters in PREP_COPIES copies, lane-interleaved: the high key
    // bytes of typical data take few values, and lanes adding to one LDS
    // word in one instruction are serialised.  A tile counts at most
    // PREP_TILE < 2^16 keys, so two 16-bit counters share a word.
    static_assert(PREP_TILE < 65536u, "16-bit digit counters");
    constexpr uint32_t COPIES = KDT_PREP_COPIES;
    constexpr uint32_t HW = K * 4 * RADIX;          // counters per copy
    __shared__ uint32_t sh[COPIES * HW / 2];
    __shared__ uint32_t s_sum[KEYSUM_WORDS];
    for (uint32_t x = threadIdx.x; x < COPIES * HW / 2; x += BLOCK) sh[x] = 0u;
    if (threadIdx.x < KEYSUM_WORDS) s_sum[threadIdx.x] = (threadIdx.x & 4u) ? 0u : 0xFFFFFFFFu;
    __syncthreads();
    TreeStep st;
    TreeInfo ti;
    find_share(a.sh, blockIdx.x, st, ti);
    const uint32_t start = (blockIdx.x - st.tile0) * PREP_TILE;
    const uint32_t end = min(start + PREP_TILE, ti.n);
    uint32_t lo[K], hi[K], kand[K], kor[K];
#pragma unroll
    for (int d = 0; d < K; ++d) {
        lo[d] = 0xFFFFFFFFu;
        hi[d] = 0u;
        kand[d] = 0xFFFFFFFFu;
        kor[d] = 0u;
    }
    bool bad = false;
    for (uint32_t i = start + threadIdx.x; i < end; i += BLOCK) {
        const size_t gi = (size_t)ti.off + i;
#pragma unroll
        for (int d = 0; d < K; ++d) {
            const uint32_t b = __float_as_uint(a.o.pts[gi * K + d]);
            bad |= coord_bad<I32>(b);
            const uint32_t u = coord_key<I32>(b);
            a.keys[(size_t)d * a.ntotal + gi] = u;
            if (WIDEST) { lo[d] = min(lo[d], u); hi[d] = max(hi[d], u); }
            kand[d] &= u;
            kor[d] |= u;
            uint32_t* shc = sh + (lane_id() & (COPIES - 1u)) * (HW / 2);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t c = (d * 4 + p) * RADIX + ((u >> (8 * p)) & 0xFFu);
                atomicAdd(&shc[c >> 1], 1u << (16u * (c & 1u)));
            }
        }
    }
    if (__any(bad) && lane_id() == 0) {
        atomicOr(a.o.status, KDT_STATUS_NONFINITE);
        atomicOr(&a.o.tstatus[st.tree], KDT_STATUS_NONFINITE);
    }
    // the summaries reduced across the wave first: every lane adding to the
    // same LDS word would be serialised
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int d = 0; d < K; ++d) {
            if (WIDEST) {
                lo[d] = min(lo[d], (uint32_t)__shfl_xor((int)lo[d], o, 64));
                hi[d] = max(hi[d], (uint32_t)__shfl_xor((int)hi[d], o, 64));
            }
            kand[d] &= (uint32_t)__shfl_xor((int)kand[d], o, 64);
            kor[d] |= (uint32_t)__shfl_xor((int)kor[d], o, 64);
        }
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int d = 0; d < K; ++d) {
            if (WIDEST) {
                atomicMin(&s_sum[d], lo[d]);
                atomicMax(&s_sum[4 + d], hi[d]);
            }
            atomicAnd(&s_sum[8 + d], kand[d]);
            atomicOr(&s_sum[12 + d], kor[d]);
        }
    }
    __syncthreads();
    uint32_t* hist = a.hist + (size_t)ti.idx * K * 4 * RADIX;
    for (uint32_t x = threadIdx.x; x < HW; x += BLOCK) {
        uint32_t c = 0;
#pragma unroll
        for (uint32_t cp = 0; cp < COPIES; ++cp) c += (sh[cp * (HW / 2) + (x >> 1)] >> (16u * (x & 1u))) & 0xFFFFu;
        if (c) atomicAdd(&hist[x], c);
    }
    if (threadIdx.x < (uint32_t)K) {
        uint32_t* sum = a.o.bbox + (size_t)ti.idx * KEYSUM_WORDS + (blockIdx.x % KEYSUM_COPIES) * KEYSUM_COPY_WORDS;
        const uint32_t d = threadIdx.x;
        if (WIDEST) {
            atomicMin(&sum[d], s_sum[d]);
            atomicMax(&sum[4 + d], s_sum[4 + d]);
        }
        atomicAnd(&sum[8 + d], s_sum[8 + d]);
        atomicOr(&sum[12 + d], s_sum[12 + d]);
    }
}

// Each tree's key summary combined into its first copy (which the presorts
// read); split-widest: the tree's scene box (the keys of its minima and
// maxima, the root's domain) and the root's dimension (Sec. 6).  One thread
// per share (one share per tree).
template <int K, bool I32, bool WIDEST>
__global__ void k_root_dim(Shares sh, Outs o, uint32_t ntrees)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntrees) return;
    const TreeInfo ti = sh.steps ? sh.trees[sh.steps[t].tree] : sh.tree0;
    uint32_t* sum = o.bbox + (size_t)ti.idx * KEYSUM_WORDS;
    uint32_t lo[K], hi[K];
#pragma unroll
    for (int d = 0; d < K; ++d) {
        keysum_box(sum, (uint32_t)d, lo[d], hi[d]);
        uint32_t kand = 0xFFFFFFFFu, kor = 0u;
#pragma unroll
        for (uint32_t c = 0; c < KEYSUM_COPIES; ++c) {
            kand &= sum[c * KEYSUM_COPY_WORDS + 8u + d];
            kor |= sum[c * KEYSUM_COPY_WORDS + 12u + d];
        }
        sum[d] = lo[d];
        sum[4 + d] = hi[d];
        sum[8 + d] = kand;
        sum[12 + d] = kor;
        if (WIDEST) {
            o.box[0][(size_t)ti.box_off * 8 + d] = lo[d];
            o.box[0][(size_t)ti.box_off * 8 + 4 + d] = hi[d];
        }
    }
    if (WIDEST) o.dimnode[ti.off] = (uint8_t)widest_dim<K, I32>(lo, hi);
}

// ------------------------------------------------------------ presort passes

// Tile of a launch over ndims dimensions taken from per-XCD queues (xq:
// off[8], len[8], then each queue's presort tile indices, a tree's tiles in
// order inside one queue): first from the queue of the XCD this workgroup
// runs on, so that a tree's tiles share that XCD's L2, then from the others.
// The launch has one workgroup per tile, so every tile is taken exactly once,
// and the tiles of a tree are taken in order (its look-back waits only on
// tiles taken before it).
__device__ uint32_t xq_take(const uint32_t* xq, uint32_t* cnt, uint32_t ndims, uint32_t* status)
{
    const uint32_t x0 = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;   // HW_REG_XCC_ID[3:0]
    for (uint32_t kk = 0; kk < 8u; ++kk) {
        const uint32_t x = (x0 + kk) & 7u;
        const uint32_t t = atomicAdd(&cnt[x], 1u);
        if (t < xq[8 + x] * ndims) return xq[16 + xq[x] + t / ndims] * ndims + t % ndims;
    }
    atomicOr(status, KDT_STATUS_INTERNAL);
    return 0xFFFFFFFFu;
}

// One stable LSD digit pass of the (key, payload) sorts of a group of
// presort roles, every tree a segment of its own (role r sorts dimension
// role_dim(r, d0) of a tree whose root splits in d0).  The roles' tiles are
// interleaved (tile t of the launch is tile t / ndims of role slot
// t % ndims), so the look-back chains of the group advance side by side.
// A tree's first pass that runs reads the keys of prep with the payload:
// the local index, or, in the per-role layout, for every role but the
// root's the point's root rank (written by the root's sort and windowed
// scatter, which run first).  LAST writes the sorted payloads (rank ->
// payload) and, in the point-major layout, scatters each rank into the rank
// table row of its index.  Ties keep the input order (local index order): a
// stable sort of keys read in index order, whatever the payload.  Pairs are stored interleaved (uint2).
// Passes whose digit is the same in every key of the tree are skipped (see
// PresortArgs).
template <bool LAST>
__global__ void __launch_bounds__(SWEEP_THREADS) k_presort_pass(PresortArgs a)
{
    constexpr int ITEMS = PRESORT_ITEMS;
    constexpr int RB = 8;
    constexpr uint32_t T = SWEEP_THREADS * ITEMS;
    __shared__ SweepSmem<RB, 2> sm;

    if (!LAST && a.sh.nsteps == 1) {
        // one tree: when its keys share this digit in every dimension of the
        // launch, no tile runs, and the workgroup leaves without taking a
        // tile (the whole launch would otherwise queue on the tile counter)
        const uint32_t* sum = a.keysum + (size_t)a.sh.tree0.idx * KEYSUM_WORDS;
        const uint32_t r0 = a.dimnode ? (uint32_t)a.dimnode[a.sh.tree0.off] : 0u;
        uint32_t runs = 0u;
        for (uint32_t j = 0; j < a.ndims; ++j) {
            const uint32_t d = role_dim(a.role0 + j, r0);
            runs |= ((sum[8 + d] ^ sum[12 + d]) >> (8u * a.pass)) & 0xFFu;
        }
        if (uniform(runs) == 0u) {
            zero_range(a.lb_zero, a.lb_zero_n);
            return;
        }
    }
    if (threadIdx.x == 0) sm.tile = a.xq ? xq_take(a.xq, a.xq_cnt, a.ndims, a.status) : atomicAdd(a.counter, 1u);
    __syncthreads();
    const uint32_t tt = uniform(sm.tile);
    if (tt == 0xFFFFFFFFu) {
        zero_range(a.lb_zero, a.lb_zero_n);
        return;
    }
    const uint32_t slot = tt % a.ndims, g = tt / a.ndims;
    const uint32_t role = a.role0 + slot;
    TreeStep st;
    TreeInfo ti;
    find_share(a.sh, g, st, ti);
    const uint32_t d0 = a.dimnode ? (uint32_t)a.dimnode[ti.off] : 0u;
    const uint32_t dim = role_dim(role, d0);
    // digits of this dimension that are not the same in every key of the tree
    const uint32_t* sum = a.keysum + (size_t)ti.idx * KEYSUM_WORDS;
    const uint32_t vary = uniform(sum[8 + dim] ^ sum[12 + dim]);
    const uint32_t q = a.pass;
    if (!LAST && ((vary >> (8u * q)) & 0xFFu) == 0u) {
        zero_range(a.lb_zero, a.lb_zero_n);
        return;
    }
    uint32_t ran = 0;                       // passes of this tree that ran before this one
    for (uint32_t qq = 0; qq < q; ++qq) ran += ((vary >> (8u * qq)) & 0xFFu) != 0u;
    const bool first = ran == 0u;
    uint32_t* kvs = a.kv + (size_t)(2u * slot) * a.kv_words;
    const uint32_t* kvin = kvs + (size_t)((ran + 1u) & 1u) * a.kv_words;
    uint32_t* kvout = kvs + (size_t)(ran & 1u) * a.kv_words;
    const uint32_t* kin = a.keys + (size_t)dim * a.ntotal;
    uint32_t* perm_out = a.perms + (size_t)role * a.ntotal;
    const uint32_t start = (g - st.tile0) * T;
    const uint32_t cnt = min(T, ti.n - start);
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint32_t shift = 8u * q;
    const size_t off = ti.off;

    uint4 rec[ITEMS];
    uint32_t dig[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        ok[i] = w * 64u * ITEMS + (uint32_t)i * 64u + lane < cnt;
        rec[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    // the two load forms as separate loops under the tile-uniform branch:
    // chosen per item inside a per-lane branch, both forms' loads shared
    // registers, and the waits between them kept one item's loads in
    // flight at a time
    if (first) {
        // the key, and the local index or, for the other roles, the root rank
        const bool by_index = role == 0u || !a.root_ranks;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = w * 64u * ITEMS + (uint32_t)i * 64u + lane;
            if (ok[i]) rec[i].x = kin[off + start + j];
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = w * 64u * ITEMS + (uint32_t)i * 64u + lane;
            if (ok[i]) rec[i].y = by_index ? start + j : a.root_ranks[off + start + j];
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = w * 64u * ITEMS + (uint32_t)i * 64u + lane;
            if (ok[i]) {
                const uint2 kv = reinterpret_cast<const uint2*>(kvin)[off + start + j];
                rec[i].x = kv.x;
                rec[i].y = kv.y;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) dig[i] = (rec[i].x >> shift) & 0xFFu;
    const uint32_t n = ti.n;
    sweep_tile<RB, ITEMS, 2>(
        sm, rec, ok, dig, ITEMS, cnt, a.hist + (size_t)ti.idx * a.hist_stride + (dim * 4u + q) * RADIX, 0u,
        a.lb + (size_t)slot * a.lb_dim_words, g, st.tile0, a.status,
        [&](const uint4& r) { return (r.x >> shift) & 0xFFu; },
        [&](uint32_t, uint32_t pos, const uint4& r) {
            if (!in_bounds(pos, n, a.status) || !in_bounds(r.y, n, a.status)) return;
            if (LAST && a.place1) {
                // k = 1: with one dimension every iteration after the first
                // finds its subtrees already sorted, and the update only
                // renumbers tags, so the point of rank pos ends at the node
                // the in-order position pos has in the tree
                const size_t at = off + inorder_to_level(pos, n);
                if (a.o.tree) {
                    uint32_t b;
                    if (a.o.i32) b = r.x ^ 0x80000000u;                     // int32 key: sign flip
                    else if (r.x == 0x80000000u) b = ((const uint32_t*)a.o.pts)[off + r.y];   // +-0: the point's own bits
                    else b = (r.x & 0x80000000u) ? (r.x ^ 0x80000000u) : ~r.x;
                    ((uint32_t*)a.o.tree)[at] = b;
                }
                a.o.nodeperm[at] = r.y;
                if (a.o.dim) a.o.dim[at] = 0u;
                if (a.o.dimnode) a.o.dimnode[at] = 0u;
                return;
            }
            if (LAST) {
                perm_out[off + pos] = r.y;
                // iteration 0 reads the root's ranks as positions
                if (a.rank_table && role != 0u) a.rank_table[(off + r.y) * a.k + dim] = pos;
            } else {
                reinterpret_cast<uint2*>(kvout)[off + pos] = make_uint2(r.x, r.y);
            }
        });
    // clear the next pass's look-back words (nothing waits on these stores)
    zero_range(a.lb_zero, a.lb_zero_n);
}

// ------------------------------------------------------ windowed rank scatter

// The per-role rank arrays of a large tree are written in two steps instead
// of one random scatter: k_rank_bucket reads a role's rank -> payload list
// and appends each (global payload, rank) pair to the bucket of its payload
// window (2^wbits payloads; a tile counts its pairs per window in LDS and
// reserves room with one atomic per window), then k_rank_window writes the
// ranks one window at a time, so that the lines it writes stay in cache
// until they are full.  The order of pairs inside a bucket is immaterial.
// The root's role gives each local index its root rank; the other roles
// give each root position the rank of its point in their dimension.
__global__ void __launch_bounds__(SWEEP_THREADS) k_rank_bucket(RankBucketArgs a)
{
    constexpr int ITEMS = PRESORT_ITEMS;
    __shared__ uint32_t cnt[RANK_MAX_WIN];
    __shared__ uint32_t base[RANK_MAX_WIN];
    TreeStep st;
    TreeInfo ti;
    find_share(a.sh, blockIdx.x, st, ti);
    const size_t off = ti.off;
    for (uint32_t x = threadIdx.x; x < a.nwin; x += SWEEP_THREADS) cnt[x] = 0u;
    __syncthreads();
    const uint32_t start = (blockIdx.x - st.tile0) * PRESORT_TILE;
    const uint32_t m = min(PRESORT_TILE, ti.n - start);
    uint32_t gi[ITEMS], slot[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = (uint32_t)i * SWEEP_THREADS + threadIdx.x;
        gi[i] = 0xFFFFFFFFu;
        slot[i] = 0u;
        if (j < m) {
            const uint32_t idx = __builtin_nontemporal_load(a.perm + off + start + j);   // read once
            if (in_bounds(idx, ti.n, a.status)) {
                gi[i] = (uint32_t)off + idx;
                slot[i] = atomicAdd(&cnt[gi[i] >> a.wbits], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < a.nwin; x += SWEEP_THREADS) {
        const uint32_t c = cnt[x];
        base[x] = c ? atomicAdd(&a.wcount[x], c) : 0u;
    }
    __syncthreads();
    const uint32_t W = 1u << a.wbits;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (gi[i] == 0xFFFFFFFFu) continue;
        const uint32_t w = gi[i] >> a.wbits;
        const uint32_t e = base[w] + slot[i];
        if (!in_bounds(e, W, a.status)) continue;
        const uint32_t j = (uint32_t)i * SWEEP_THREADS + threadIdx.x;
        reinterpret_cast<uint2*>(a.pairs)[((size_t)w << a.wbits) + e] = make_uint2(gi[i], start + j);
    }
}

// One chunk of RANK_WIN_CHUNK pairs of one window's bucket per workgroup.
// Workgroups are dispatched to the 8 XCDs round-robin, so workgroup b takes
// a window w = b mod 8 (mod 8): the lines of a window are then all written
// through one XCD's L2, which holds them until they are full.
__global__ void __launch_bounds__(BLOCK) k_rank_window(RankWindowArgs a)
{
    constexpr uint32_t PER = RANK_WIN_CHUNK / BLOCK;
    const uint32_t x = blockIdx.x & 7u, j = blockIdx.x >> 3;
    const uint32_t w = x + 8u * (j / a.chunks), c = j % a.chunks;
    if (w >= a.nwin) return;
    const uint32_t n = min(a.wcount[w], 1u << a.wbits);
    const uint2* pr = reinterpret_cast<const uint2*>(a.pairs) + ((size_t)w << a.wbits);
    uint2 v[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        const uint32_t e = c * RANK_WIN_CHUNK + j * BLOCK + threadIdx.x;
        // streamed once: non-temporal, so that the L2 keeps the window's
        // partly written rank lines (2.21 -> 2.10 ms per 100M build)
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        if (e < n) {
            const u32x2 x = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(pr) + e);
            v[j] = make_uint2(x.x, x.y);
        } else {
            v[j] = make_uint2(0xFFFFFFFFu, 0u);
        }
    }
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j)
        if (v[j].x < a.ntotal) a.dm[v[j].x] = v[j].y;
}

void launch_rank_bucket(const RankBucketArgs& a, uint32_t tiles, hipStream_t st)
{
    if (tiles) k_rank_bucket<<<tiles, SWEEP_THREADS, 0, st>>>(a);
}

// LDS the window launch reserves without using it: it caps the workgroups
// a CU holds at four (seven otherwise), so that fewer windows are written at
// once on each XCD and more of their lines can stay in its L2 until full:
// 2.20 against 2.31 ms of window writes per 100M-point build, and 2.38 ms
// with two workgroups per CU, whose reads have fewer loads in flight
constexpr uint32_t RANK_WIN_LDS = 40960;

void launch_rank_window(const RankWindowArgs& a, hipStream_t st)
{
    const uint32_t grid = ((a.nwin + 7u) / 8u) * 8u * a.chunks;
    if (grid) k_rank_window<<<grid, BLOCK, RANK_WIN_LDS, st>>>(a);
}

// ------------------------------------------------------------------ level 0

// Iteration 0 of one tile of one tree: every tag is 0 and the presort of the
// root's dimension is the sorted order, so array position r holds the point
// of rank r.  The pivot is ss(1) (Sec. 3.2, Sec. 5); the root is placed, the
// others keep their order and are written compacted (left subtree then right
// subtree).  With N <= 3 the children are leaves and are placed directly.
// With keys_next, also writes each survivor's split key of iteration 1 (its
// rank in its subtree's split dimension) and the top-digit histogram of
// every iteration-1 subtree.
template <int K, bool WIDEST, bool I32>
__global__ void __launch_bounds__(BLOCK) k_level0(Level0Args a)
{
    __shared__ uint32_t nh[2 * MAX_BINS];
    __shared__ uint32_t cdim[2];
    // with an XCD map, workgroup b (on XCD b mod 8) takes the tile the map
    // gives it: a tree's tiles all on one XCD, as the tail's groups later;
    // padding entries take none
    const uint32_t tile = a.xmap ? a.xmap[blockIdx.x] : blockIdx.x;
    if (tile == 0xFFFFFFFFu) return;
    TreeStep st;
    TreeInfo ti;
    find_share(a.sh, tile, st, ti);
    const uint32_t P = a.passes;
    const uint32_t RBv = a.radix_bits;
    const uint32_t NB = 1u << RBv;
    const uint32_t top = RBv * (P - 1u);
    const bool acc = a.keys_next != 0u && st.hist_next != 0xFFFFFFFFu;
    if (acc)
        for (uint32_t x = threadIdx.x; x < 2u * NB; x += BLOCK) nh[x] = 0u;
    const uint32_t n = ti.n;
    const size_t off = ti.off;
    const uint32_t L = num_levels(n);
    const uint32_t d0 = WIDEST ? (uint32_t)a.o.dimnode[off] : 0u;
    const uint32_t* perm_d0 = a.perms + off;                 // the root's role: root order -> local index
    const uint32_t piv = (L >= 2) ? seg_pivot(make_level(n, 0), 0) : 0u;
    if (threadIdx.x == 0) {
        // split dimensions of the root's children
        uint32_t c0 = (K == 1) ? 0u : 1u % (uint32_t)K, c1 = c0;
        if (WIDEST && acc) {
            uint32_t idx = perm_d0[piv];
            if (!in_bounds(idx, n, a.o.status)) idx = 0;
            const uint32_t plane = plane_key<I32>(a.o, ti, idx, d0, K);
            const uint32_t* bc = a.o.box[0] + (size_t)ti.box_off * 8;
            c0 = child_dim<K, I32>(bc, plane, d0, 0u);
            c1 = child_dim<K, I32>(bc, plane, d0, 1u);
        }
        cdim[0] = c0;
        cdim[1] = c1;
    }
    __syncthreads();
    const uint32_t cd0 = uniform(cdim[0]), cd1 = uniform(cdim[1]);
    const uint32_t start = (tile - st.tile0) * PREP_TILE;
    const uint32_t end = min(start + PREP_TILE, n);
    // four points per thread and round, all their loads issued before the
    // first point is processed
    constexpr uint32_t U = 4;
    for (uint32_t r0 = start + threadIdx.x; r0 < end; r0 += U * BLOCK) {
        uint32_t idxv[U];
        uint4 recv[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t r = r0 + u * BLOCK;
            idxv[u] = r < end ? perm_d0[r] : 0xFFFFFFFFu;
            recv[u] = make_uint4(0u, 0u, 0u, 0u);
        }
        // per-role arrays hold the ranks by root position (r's streams in);
        // the point-major table holds them by index (gathered)
        if (a.role_ranks) {
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t r = r0 + u * BLOCK;
                if (r >= end) continue;
#pragma unroll
                for (int d = 0; d < K; ++d)
                    if ((uint32_t)d != d0)
                        set4(recv[u], (uint32_t)d, a.role_ranks[(size_t)dim_role((uint32_t)d, d0) * a.ntotal + off + r]);
            }
        } else {
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (idxv[u] < n) recv[u] = load_rec4<K>(a.rank_table, off + idxv[u]);
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t r = r0 + u * BLOCK;
            if (r >= end) continue;
            const uint32_t idx = idxv[u];
            if (!in_bounds(idx, n, a.o.status)) continue;
            if (r == piv) {
                place<K, WIDEST>(a.o, ti, 0u, idx);
                if (WIDEST && L >= 2)
                    widest_children<K, I32>(a.o, ti, 0u, 0u, plane_key<I32>(a.o, ti, idx, d0, K), d0, a.o.box[0],
                                            L > 2 ? a.o.box[1] : nullptr);
                continue;
            }
            if (L == 2) {                       // N = 2 or 3: children are leaves
                place<K, WIDEST>(a.o, ti, r < piv ? 1u : 2u, idx);
                continue;
            }
            uint4 rec = recv[u];
            // the root dimension's rank is the position (every later segment
            // keeps the root dimension's order), so its slot carries the index
            set4(rec, d0, idx);
            const uint32_t side = r > piv ? 1u : 0u;
            store_rec4<K>(a.rout, off + r - side, rec);
            if (acc) {
                // no split key for a child split in the root's dimension: its
                // pivot is found by position
                const uint32_t cd = side ? cd1 : cd0;
                if (cd != d0) {
                    const uint32_t kv = pick4(rec, cd);
                    a.kout[off + r - side] = kv;
                    atomicAdd(&nh[side * NB + ((kv >> top) & (NB - 1u))], 1u);
                }
            }
        }
    }
    if (acc) {
        __syncthreads();
        // iteration-1 subtrees 0 and 1, top digit
        for (uint32_t x = threadIdx.x; x < 2u * NB; x += BLOCK) {
            const uint32_t c = x / NB;
            if (nh[x]) atomicAdd(&a.hist[st.hist_next + ((size_t)c * P + P - 1u) * NB + (x - c * NB)], nh[x]);
        }
    }
}

// --------------------------------------------------------- pivot selection

// One digit of the radix select of every subtree's pivot key in iteration l
// (see LevelSelectArgs).  Workgroups take segment-aligned chunks of HIST_TILE
// keys.  The pivot of the i-th subtree is its key of rank ss(2s+1) (its left
// size); the digits above `digit` are read off the histograms of the
// earlier launches, and this launch counts the `digit` values of the keys
// that agree with them.
__global__ void __launch_bounds__(SWEEP_THREADS) k_level_select(LevelSelectArgs a)
{
    __shared__ uint32_t lh[MAX_BINS];
    __shared__ uint32_t sh[2 * SWEEP_WAVES];
    __shared__ uint32_t sel[2];
    const uint32_t RBv = a.radix_bits;
    const uint32_t NB = 1u << RBv;
    const uint32_t P = a.passes;
    const uint32_t j = a.digit;
    for (uint32_t x = threadIdx.x; x < NB; x += SWEEP_THREADS) lh[x] = 0u;
    TreeStep st;
    TreeInfo ti;
    find_share(a.sh, blockIdx.x, st, ti);
    const Level v = make_level(ti.n, st.level);
    const SegTiles tl = tiles_level(v, HIST_TILE);
    uint32_t seg, u;
    tile_locate(tl, blockIdx.x - st.tile0, seg, u);
    // a subtree split in the root's dimension needs no select (its keys are
    // positions, and its pivot the point at position ss(2s+1))
    if (a.dimnode && a.dimnode[ti.off + v.Fl + seg] == a.dimnode[ti.off]) return;
    const uint32_t soff = tiles_seg_offset(tl, seg);
    const uint32_t sz = tiles_seg_size(tl, seg);
    const uint32_t start = u * HIST_TILE;
    const uint32_t cnt = min(HIST_TILE, sz - start);
    // the chunk's keys first, so that their loads overlap the digit search
    constexpr uint32_t KPT = HIST_TILE / SWEEP_THREADS;
    const uint32_t* kin = a.kin + (size_t)ti.off + soff + start;
    uint32_t key[KPT];
#pragma unroll
    for (uint32_t i = 0; i < KPT; ++i) {
        const uint32_t x = i * SWEEP_THREADS + threadIdx.x;
        key[i] = x < cnt ? kin[x] : 0u;
    }
    uint32_t* h = a.hist + st.hist + (size_t)seg * P * NB;
    uint32_t kk = seg_left_size(v, seg);
    uint32_t prefix = 0;
    // digits above j (P >= 2 and j <= P-2: at least one; each search ends
    // with a barrier, which also orders the clearing of lh)
    uint32_t c[MAX_LEVEL_PASSES][FIND_BPT];
#pragma unroll
    for (uint32_t jj = 0; jj < MAX_LEVEL_PASSES; ++jj)
        if (jj > j && jj < P) load_bins(h + (size_t)jj * NB, NB, c[jj]);
#pragma unroll
    for (int jj = (int)MAX_LEVEL_PASSES - 1; jj >= 0; --jj)
        if ((uint32_t)jj > j && (uint32_t)jj < P) prefix = (prefix << RBv) | find_bucket(c[jj], NB, kk, sh, sel, a.status);
    const uint32_t hs = RBv * (j + 1u), lo = RBv * j;
#pragma unroll
    for (uint32_t i = 0; i < KPT; ++i) {
        const uint32_t x = i * SWEEP_THREADS + threadIdx.x;
        if (x < cnt && (key[i] >> hs) == prefix) atomicAdd(&lh[(key[i] >> lo) & (NB - 1u)], 1u);
    }
    __syncthreads();
    uint32_t* dst = h + (size_t)j * NB;
    for (uint32_t x = threadIdx.x; x < NB; x += SWEEP_THREADS)
        if (lh[x]) atomicAdd(&dst[x], lh[x]);
}

// ------------------------------------------------------------ payload

// Per-point payload in tree order: record s of out is record perm[s] of in,
// each record `words` units of W.  An index outside [0, n) flags an internal
// error and leaves its record unwritten.
template <typename W>
__global__ void __launch_bounds__(BLOCK) k_permute(const uint32_t* __restrict__ perm, uint32_t n,
                                                  const W* __restrict__ in, W* __restrict__ out, uint32_t words,
                                                  uint32_t* status)
{
    const uint64_t total = (uint64_t)n * words;
    for (uint64_t x = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; x < total; x += (uint64_t)gridDim.x * BLOCK) {
        const uint64_t s = x / words, w = x - s * words;
        const uint32_t i = perm[s];
        if (i >= n) {
            if (status) atomicOr(status, KDT_STATUS_INTERNAL);
            continue;
        }
        out[s * words + w] = in[(uint64_t)i * words + w];
    }
}

void launch_permute(const uint32_t* perm, uint32_t n, const void* in, void* out, uint32_t stride, uint32_t* status,
                    hipStream_t st)
{
    const uintptr_t align = (uintptr_t)in | (uintptr_t)out | stride;
    uint32_t unit = (align % 16u) == 0u ? 16u : ((align % 4u) == 0u ? 4u : 1u);
    const uint32_t words = stride / unit;
    const uint64_t total = (uint64_t)n * words;
    if (total == 0) return;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((total + BLOCK - 1) / BLOCK, 1u << 16);
    if (unit == 16u)
        k_permute<uint4><<<grid, BLOCK, 0, st>>>(perm, n, (const uint4*)in, (uint4*)out, words, status);
    else if (unit == 4u)
        k_permute<uint32_t><<<grid, BLOCK, 0, st>>>(perm, n, (const uint32_t*)in, (uint32_t*)out, words, status);
    else
        k_permute<uint8_t><<<grid, BLOCK, 0, st>>>(perm, n, (const uint8_t*)in, (uint8_t*)out, words, status);
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

void launch_init(uint32_t* status, uint32_t* counters, uint32_t* z1, uint32_t n1, uint32_t* z2, uint32_t n2,
                 uint32_t* z3, uint32_t n3, uint32_t* z4, uint32_t n4, uint32_t* z5, uint32_t n5, uint32_t* bbox,
                 uint32_t nbox, hipStream_t st)
{
    uint32_t big = n1 > n2 ? n1 : n2;
    big = big > n3 ? big : n3;
    big = big > n4 ? big : n4;
    big = big > n5 ? big : n5;
    big = big > MAX_COUNTERS ? big : MAX_COUNTERS;
    big = big > nbox * KEYSUM_WORDS ? big : nbox * KEYSUM_WORDS;
    uint32_t grid = ceil_div(big, BLOCK);
    if (grid > 2048) grid = 2048;
    if (grid == 0) grid = 1;
    k_init<<<grid, BLOCK, 0, st>>>(status, counters, z1, n1, z2, n2, z3, n3, z4, n4, z5, n5, bbox, nbox);
}

template <int K>
static void prep_k(const PrepArgs& a, uint32_t tiles, bool widest, hipStream_t st)
{
    if (a.o.i32) {
        if (widest) k_prep<K, true, true><<<tiles, BLOCK, 0, st>>>(a);
        else k_prep<K, false, true><<<tiles, BLOCK, 0, st>>>(a);
    } else {
        if (widest) k_prep<K, true, false><<<tiles, BLOCK, 0, st>>>(a);
        else k_prep<K, false, false><<<tiles, BLOCK, 0, st>>>(a);
    }
}

void launch_prep(int k, const PrepArgs& a, uint32_t tiles, bool widest, hipStream_t st)
{
    switch (k) {
    case 1: prep_k<1>(a, tiles, widest, st); break;
    case 2: prep_k<2>(a, tiles, widest, st); break;
    case 3: prep_k<3>(a, tiles, widest, st); break;
    default: prep_k<4>(a, tiles, widest, st); break;
    }
}

template <int K>
static void root_dim_k(const Shares& sh, const Outs& o, uint32_t ntrees, bool widest, hipStream_t st)
{
    const uint32_t grid = ceil_div(ntrees, 64u);
    if (!widest) k_root_dim<K, false, false><<<grid, 64, 0, st>>>(sh, o, ntrees);
    else if (o.i32) k_root_dim<K, true, true><<<grid, 64, 0, st>>>(sh, o, ntrees);
    else k_root_dim<K, false, true><<<grid, 64, 0, st>>>(sh, o, ntrees);
}

void launch_root_dim(int k, const Shares& sh, const Outs& o, uint32_t ntrees, bool widest, hipStream_t st)
{
    switch (k) {
    case 1: root_dim_k<1>(sh, o, ntrees, widest, st); break;
    case 2: root_dim_k<2>(sh, o, ntrees, widest, st); break;
    case 3: root_dim_k<3>(sh, o, ntrees, widest, st); break;
    default: root_dim_k<4>(sh, o, ntrees, widest, st); break;
    }
}

void launch_presort_pass(const PresortArgs& a, bool last, uint32_t tiles, hipStream_t st)
{
    if (last) k_presort_pass<true><<<tiles, SWEEP_THREADS, 0, st>>>(a);
    else k_presort_pass<false><<<tiles, SWEEP_THREADS, 0, st>>>(a);
}

template <int K>
static void level0_k(const Level0Args& a, uint32_t tiles, bool widest, hipStream_t st)
{
    // round robin never reads a coordinate here: one instantiation
    if (!widest) k_level0<K, false, false><<<tiles, BLOCK, 0, st>>>(a);
    else if (a.o.i32) k_level0<K, true, true><<<tiles, BLOCK, 0, st>>>(a);
    else k_level0<K, true, false><<<tiles, BLOCK, 0, st>>>(a);
}

void launch_level0(int k, const Level0Args& a, uint32_t tiles, bool widest, hipStream_t st)
{
    switch (k) {
    case 1: level0_k<1>(a, tiles, widest, st); break;
    case 2: level0_k<2>(a, tiles, widest, st); break;
    case 3: level0_k<3>(a, tiles, widest, st); break;
    default: level0_k<4>(a, tiles, widest, st); break;
    }
}

void launch_level_select(const LevelSelectArgs& a, uint32_t tiles, hipStream_t st)
{
    k_level_select<<<tiles, SWEEP_THREADS, 0, st>>>(a);
}

template <int K>
void launch_level_pivot_k(const LevelPivotArgs& a, uint32_t tiles, bool widest, hipStream_t st);

void launch_level_pivot(int k, const LevelPivotArgs& a, uint32_t tiles, bool widest, hipStream_t st)
{
    switch (k) {
    case 1: launch_level_pivot_k<1>(a, tiles, widest, st); break;
    case 2: launch_level_pivot_k<2>(a, tiles, widest, st); break;
    case 3: launch_level_pivot_k<3>(a, tiles, widest, st); break;
    default: launch_level_pivot_k<4>(a, tiles, widest, st); break;
    }
}

template <int K>
void launch_level_part_k(const LevelPartArgs& a, uint32_t tiles, bool widest, hipStream_t st);

void launch_level_part(int k, const LevelPartArgs& a, uint32_t tiles, bool widest, hipStream_t st)
{
    switch (k) {
    case 1: launch_level_part_k<1>(a, tiles, widest, st); break;
    case 2: launch_level_part_k<2>(a, tiles, widest, st); break;
    case 3: launch_level_part_k<3>(a, tiles, widest, st); break;
    default: launch_level_part_k<4>(a, tiles, widest, st); break;
    }
}

}  // namespace kdt
