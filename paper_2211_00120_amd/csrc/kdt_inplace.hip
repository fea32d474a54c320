// kdt_inplace.hip -- the low-memory in-place build (kdt_build_inplace).
//
// The points are permuted where they lie; the only per-point storage is the
// caller's perm array, which holds each point's original index (the
// tie-break of the order (coordinate, index)) and, at the end, the tree's
// permutation.  Every data movement is a compare-exchange or a swap
// (Sec. 7: a swap-only sort such as bitonic sort needs no storage beyond
// the one int per node).  Arithmetic and layout: kdt_inplace.h.
//
// Launch sequence for n points, L = 32 - clz(n) levels, lg = deep_level(L):
//   k_ip_clear, k_ip_init             perm = identity, non-finite flag, scene box
//   iterations l = 0 .. lg-1          (subtrees larger than one LDS block)
//     [k_ip_setup]                    split-widest: every subtree's domain and dim
//     k_ip_block<SORT>                bitonic sort of every SBLK-block of every subtree
//     per stage S = 2 SBLK .. P:      k_ip_mgroup (the mirrored stride S/2 and the
//                                     next up to two, two mirrored groups per thread),
//                                     k_ip_group (strides down to SBLK, up to 4 per pass),
//                                     k_ip_block<MERGE> (strides SBLK/2 .. 1 in LDS)
//   [k_ip_setup]                      split-widest: domains of the level-lg subtrees
//   k_ip_deep                         one workgroup per level-lg subtree: its
//                                     remaining iterations in LDS
//   k_ip_unshuf / k_ip_swaplevel /    in-order -> level order (swap-only)
//   k_ip_reverse / k_ip_ldstree
//   [k_ip_rrdims], k_ip_finish        round-robin dims, status word
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../include/kdt.h"
#include "kdt_device.h"
#include "kdt_host.h"
#include "kdt_inplace.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"

namespace kdt {
namespace ip {

// Workspace: a 256-byte header (status word, scene box keys), then one byte
// per subtree of the iterations before lg (its split dimension), then, for
// split-widest, the domain box of every level-lg subtree (8 words each).
constexpr uint32_t HDR_WORDS = 64;
constexpr uint32_t HDR_STATUS = 0, HDR_LO = 8, HDR_HI = 16;
constexpr size_t WS_ALIGN_IP = 256;

__host__ __device__ inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct WsLayout {
    size_t segdim, boxes, total;
};

inline WsLayout ws_layout(uint32_t n, bool wide)
{
    const uint32_t lg = deep_level(num_levels(n));
    const size_t nsub = (size_t)1 << lg;
    WsLayout w;
    w.segdim = HDR_WORDS * 4;
    w.boxes = w.segdim + round_up(nsub, WS_ALIGN_IP);
    w.total = w.boxes + (wide ? round_up(nsub * 8 * 4, WS_ALIGN_IP) : 0);
    return w;
}

// ------------------------------------------------------------ device helpers

template <int K>
__device__ __forceinline__ void ld_pt(const uint32_t* __restrict__ pts, uint32_t p, uint32_t (&c)[K])
{
    const uint32_t* q = pts + (size_t)p * K;
    if constexpr (K == 4) {
        const uint4 v = *(const uint4*)q;
        c[0] = v.x;
        c[1] = v.y;
        c[2] = v.z;
        c[3] = v.w;
    } else if constexpr (K == 2) {
        const uint2 v = *(const uint2*)q;
        c[0] = v.x;
        c[1] = v.y;
    } else {
#pragma unroll
        for (int d = 0; d < K; ++d) c[d] = q[d];
    }
}

template <int K>
__device__ __forceinline__ void st_pt(uint32_t* __restrict__ pts, uint32_t p, const uint32_t (&c)[K])
{
    uint32_t* q = pts + (size_t)p * K;
    if constexpr (K == 4) {
        *(uint4*)q = make_uint4(c[0], c[1], c[2], c[3]);
    } else if constexpr (K == 2) {
        *(uint2*)q = make_uint2(c[0], c[1]);
    } else {
#pragma unroll
        for (int d = 0; d < K; ++d) q[d] = c[d];
    }
}

// Coordinate d of a register point, d a runtime value (a select chain, so
// the point stays in registers).
template <int K>
__device__ __forceinline__ uint32_t pick(const uint32_t (&c)[K], uint32_t d)
{
    uint32_t v = c[0];
#pragma unroll
    for (int j = 1; j < K; ++j) v = d == (uint32_t)j ? c[j] : v;
    return v;
}

template <int K>
__device__ __forceinline__ void set_at(uint32_t (&c)[K], uint32_t d, uint32_t v)
{
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (d == (uint32_t)j) c[j] = v;
}

// Sort key of a point in dimension d: (coordinate key, original index).
template <bool I32>
__device__ __forceinline__ uint64_t rkey(uint32_t cbits, uint32_t id)
{
    return ((uint64_t)coord_key<I32>(cbits) << 32) | id;
}

// Split dimension of segment `seg` of the current iteration.
__device__ __forceinline__ uint32_t seg_dim(const uint8_t* segdim, uint32_t dimrr, uint32_t seg)
{
    return segdim ? (uint32_t)segdim[seg] : dimrr;
}

// LDS record block: coordinates as structure of arrays, then the indices.
template <int K>
struct Lds {
    uint32_t c[K][BLK];
    uint32_t id[BLK];
};

template <int K, bool I32>
__device__ __forceinline__ void lds_cmpx(Lds<K>& s, uint32_t a, uint32_t b, uint32_t d)
{
    const uint64_t ka = rkey<I32>(s.c[d][a], s.id[a]);
    const uint64_t kb = rkey<I32>(s.c[d][b], s.id[b]);
    if (ka > kb) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t t = s.c[j][a];
            s.c[j][a] = s.c[j][b];
            s.c[j][b] = t;
        }
        const uint32_t t = s.id[a];
        s.id[a] = s.id[b];
        s.id[b] = t;
    }
}

template <int K>
__device__ __forceinline__ void lds_load(Lds<K>& s, const uint32_t* pts, const uint32_t* perm, uint32_t base,
                                         uint32_t cnt)
{
    for (uint32_t j = threadIdx.x; j < cnt; j += THREADS) {
        uint32_t c[K];
        ld_pt<K>(pts, base + j, c);
#pragma unroll
        for (int d = 0; d < K; ++d) s.c[d][j] = c[d];
        s.id[j] = perm[base + j];
    }
}

template <int K>
__device__ __forceinline__ void lds_store(const Lds<K>& s, uint32_t* pts, uint32_t* perm, uint32_t base,
                                          uint32_t cnt)
{
    for (uint32_t j = threadIdx.x; j < cnt; j += THREADS) {
        uint32_t c[K];
#pragma unroll
        for (int d = 0; d < K; ++d) c[d] = s.c[d][j];
        st_pt<K>(pts, base + j, c);
        perm[base + j] = s.id[j];
    }
}

// Swap two whole records in global memory.
template <int K>
__device__ __forceinline__ void swap_rec(uint32_t* pts, uint32_t* perm, uint32_t x, uint32_t y)
{
    uint32_t a[K], b[K];
    ld_pt<K>(pts, x, a);
    ld_pt<K>(pts, y, b);
    const uint32_t ia = perm[x], ib = perm[y];
    st_pt<K>(pts, x, b);
    st_pt<K>(pts, y, a);
    perm[x] = ib;
    perm[y] = ia;
}

// ------------------------------------------------------------ kernels

__global__ void k_ip_clear(uint32_t* hdr)
{
    const uint32_t t = threadIdx.x;
    if (t < HDR_WORDS) hdr[t] = (t >= HDR_LO && t < HDR_LO + 4u) ? 0xFFFFFFFFu : 0u;
}

// perm[i] = i, the non-finite flag and (split-widest) the scene box.
template <int K, bool I32, bool WIDE>
__global__ __launch_bounds__(256) void k_ip_init(const uint32_t* __restrict__ pts, uint32_t* __restrict__ perm,
                                                 uint32_t n, uint32_t* hdr)
{
    uint32_t lo[K], hi[K];
#pragma unroll
    for (int d = 0; d < K; ++d) {
        lo[d] = 0xFFFFFFFFu;
        hi[d] = 0u;
    }
    bool bad = false;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        perm[i] = i;
        if (WIDE || !I32) {
            uint32_t c[K];
            ld_pt<K>(pts, i, c);
#pragma unroll
            for (int d = 0; d < K; ++d) {
                bad |= coord_bad<I32>(c[d]);
                const uint32_t key = coord_key<I32>(c[d]);
                lo[d] = key < lo[d] ? key : lo[d];
                hi[d] = key > hi[d] ? key : hi[d];
            }
        }
    }
    if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&hdr[HDR_STATUS], KDT_STATUS_NONFINITE);
    if (WIDE) {
#pragma unroll
        for (int d = 0; d < K; ++d) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const uint32_t a = __shfl_xor(lo[d], off, 64);
                const uint32_t b = __shfl_xor(hi[d], off, 64);
                lo[d] = a < lo[d] ? a : lo[d];
                hi[d] = b > hi[d] ? b : hi[d];
            }
        }
        if (lane_id() == 0) {
#pragma unroll
            for (int d = 0; d < K; ++d) {
                atomicMin(&hdr[HDR_LO + d], lo[d]);
                atomicMax(&hdr[HDR_HI + d], hi[d]);
            }
        }
    }
}

// Split-widest: the domain of every subtree of level l, clipped by its
// ancestors' planes (Sec. 6), whose pivots already sit at their in-order
// positions.  boxes == nullptr: write the split dimension (segdim, dim);
// otherwise write the domain box (for the LDS iterations).
template <int K, bool I32>
__global__ __launch_bounds__(256) void k_ip_setup(const uint32_t* __restrict__ pts, uint32_t n, uint32_t l,
                                                  const uint32_t* hdr, uint8_t* segdim, uint32_t* boxes,
                                                  uint8_t* dim)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (1u << l)) return;
    uint32_t lo[K], hi[K];
#pragma unroll
    for (int d = 0; d < K; ++d) {
        lo[d] = hdr[HDR_LO + d];
        hi[d] = hdr[HDR_HI + d];
    }
    for (uint32_t a = 0; a < l; ++a) {
        const Level va = make_level(n, a);
        const uint32_t ia = i >> (l - a);
        const uint32_t d = widest_dim<K, I32>(lo, hi);
        const uint32_t key = coord_key<I32>(pts[(size_t)io_pivot(va, ia) * K + d]);
        if ((i >> (l - a - 1u)) & 1u)
            set_at<K>(lo, d, key);
        else
            set_at<K>(hi, d, key);
    }
    if (boxes) {
#pragma unroll
        for (int d = 0; d < K; ++d) {
            boxes[(size_t)i * 8 + d] = lo[d];
            boxes[(size_t)i * 8 + 4 + d] = hi[d];
        }
    } else {
        const uint32_t d = widest_dim<K, I32>(lo, hi);
        segdim[i] = (uint8_t)d;
        if (dim) dim[full_nodes(l) + i] = (uint8_t)d;
    }
}

// One LDS block (SBLK entries) of one subtree of iteration l: SORT runs the
// whole bitonic network of the block, MERGE the strides SBLK/2 .. 1 of the
// current stage.  The network runs on (key, slot) pairs in LDS; then every
// thread reads the records its output positions receive (all reads before
// any write) and stores them.
template <int K, bool I32, bool SORT>
__global__ __launch_bounds__(256) void k_ip_block(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm, uint32_t n,
                                                  uint32_t l, uint32_t dimrr, const uint8_t* segdim, uint32_t* hdr)
{
    constexpr uint32_t E = SBLK / THREADS;
    __shared__ uint64_t key[SBLK];
    __shared__ uint16_t slot[SBLK];
    const Level v = make_level(n, l);
    const SegTiles t = tiles_level(v, SBLK);
    uint32_t seg, u;
    tile_locate(t, blockIdx.x, seg, u);
    const uint32_t size = seg_size(v, seg);
    const uint32_t base = io_begin(v, seg) + u * SBLK;
    const uint32_t cnt = umin(SBLK, size - u * SBLK);
    if (u * SBLK >= size || base + cnt > n) {
        if (threadIdx.x == 0) atomicOr(&hdr[HDR_STATUS], KDT_STATUS_INTERNAL);
        return;
    }
    const uint32_t d = seg_dim(segdim, dimrr, seg);
    for (uint32_t p = threadIdx.x; p < cnt; p += THREADS) {
        key[p] = rkey<I32>(pts[(size_t)(base + p) * K + d], perm[base + p]);
        slot[p] = (uint16_t)p;
    }
    __syncthreads();
    for (uint32_t e = SORT ? 1u : SBLK_LOG; e <= SBLK_LOG; ++e) {
        for (int ls = (int)e - 1; ls >= 0; --ls) {
            const bool mirrored = SORT && ls == (int)e - 1;
            for (uint32_t q = threadIdx.x; q < SBLK / 2; q += THREADS) {
                uint32_t lo, hi;
                if (mirrored)
                    mirror_pair(q, e, lo, hi);
                else
                    half_pair(q, (uint32_t)ls, lo, hi);
                if (hi < cnt) {
                    const uint64_t a = key[lo], b = key[hi];
                    if (a > b) {
                        key[lo] = b;
                        key[hi] = a;
                        const uint16_t ts = slot[lo];
                        slot[lo] = slot[hi];
                        slot[hi] = ts;
                    }
                }
            }
            __syncthreads();
        }
    }
    uint32_t rc[E][K];
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
        const uint32_t p = threadIdx.x + j * THREADS;
        if (p < cnt && slot[p] != p) ld_pt<K>(pts, base + slot[p], rc[j]);
    }
    __syncthreads();                        // every read of the block done before any write
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
        const uint32_t p = threadIdx.x + j * THREADS;
        if (p < cnt && slot[p] != p) {
            st_pt<K>(pts, base + p, rc[j]);
            perm[base + p] = (uint32_t)key[p];
        }
    }
}

// The first c steps of stage e of iteration l over global memory: the
// mirrored step (entry w of every 2^e-block against entry 2^e - 1 - w), then
// half-cleaners of strides 2^(e-2) .. 2^(e-c), on two mirrored groups of 2^c
// entries per thread (see mgroup_base).  The network runs on keys and slots;
// the moved records are read, then written.
template <int K, bool I32, int C>
__global__ __launch_bounds__(256) void k_ip_mgroup(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm, uint32_t n,
                                                   uint32_t l, uint32_t logP, uint32_t e, uint32_t dimrr,
                                                   const uint8_t* segdim)
{
    constexpr int G = 1 << C;
    const uint32_t e0 = e - C;
    const Level v = make_level(n, l);
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (v.nseg << (logP - C - 1))) return;
    const uint32_t seg = g >> (logP - C - 1);
    const uint32_t ba = mgroup_base(g & ((1u << (logP - C - 1)) - 1u), e0, C);
    const uint32_t bb = ba ^ ((1u << e0) - 1u);
    const uint32_t size = seg_size(v, seg);
    if (ba >= size) return;                 // both groups lie past the subtree's end
    const uint32_t base = io_begin(v, seg);
    const uint32_t d = seg_dim(segdim, dimrr, seg);
    uint64_t key[2 * G];
    uint32_t slot[2 * G];
#pragma unroll
    for (int j = 0; j < 2 * G; ++j) {
        const uint32_t r = group_pos(j < G ? ba : bb, (uint32_t)(j & (G - 1)), e0);
        slot[j] = (uint32_t)j;
        key[j] = ~0ull;                     // past the subtree's end: +infinity
        if (r < size) key[j] = rkey<I32>(pts[(size_t)(base + r) * K + d], perm[base + r]);
    }
    auto cmpx = [&](int lo, int hi) {
        if (key[lo] > key[hi]) {
            const uint64_t tk = key[lo];
            key[lo] = key[hi];
            key[hi] = tk;
            const uint32_t ts = slot[lo];
            slot[lo] = slot[hi];
            slot[hi] = ts;
        }
    };
    // mirrored step: A[x] against B[G-1-x], the lower position first
#pragma unroll
    for (int x = 0; x < G; ++x) {
        const int a = x, b = G + (G - 1 - x);
        if (x >> (C - 1)) cmpx(b, a);
        else cmpx(a, b);
    }
    // half-cleaners inside each group
#pragma unroll
    for (int sb = C - 2; sb >= 0; --sb) {
#pragma unroll
        for (int half = 0; half < 2 * G; half += G) {
#pragma unroll
            for (int p = 0; p < G / 2; ++p) {
                const int x = ((p >> sb) << (sb + 1)) | (p & ((1 << sb) - 1));
                cmpx(half + x, half + (x | (1 << sb)));
            }
        }
    }
    uint32_t rc[2 * G][K];
#pragma unroll
    for (int j = 0; j < 2 * G; ++j)
        if (slot[j] != (uint32_t)j)
            ld_pt<K>(pts, base + group_pos(slot[j] < (uint32_t)G ? ba : bb, slot[j] & (uint32_t)(G - 1), e0), rc[j]);
#pragma unroll
    for (int j = 0; j < 2 * G; ++j) {
        if (slot[j] != (uint32_t)j) {
            const uint32_t r = group_pos(j < G ? ba : bb, (uint32_t)(j & (G - 1)), e0);
            st_pt<K>(pts, base + r, rc[j]);
            perm[base + r] = (uint32_t)key[j];
        }
    }
}

// C consecutive half-cleaner steps of iteration l over global memory:
// strides 2^(e0+C-1) .. 2^e0, applied by one thread to a group of 2^C
// entries (the group's base with bits [e0, e0+C) enumerated).  The network
// runs on the keys and their slots; the records that move are then read
// (all of them before any is written) and stored at their new slots.
template <int K, bool I32, int C>
__global__ __launch_bounds__(256) void k_ip_group(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm, uint32_t n,
                                                  uint32_t l, uint32_t logP, uint32_t e0, uint32_t dimrr,
                                                  const uint8_t* segdim)
{
    constexpr int G = 1 << C;
    const Level v = make_level(n, l);
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (v.nseg << (logP - C))) return;
    const uint32_t seg = g >> (logP - C);
    const uint32_t h = g & ((1u << (logP - C)) - 1u);
    const uint32_t gb = group_base(h, e0, C);
    const uint32_t size = seg_size(v, seg);
    if (gb >= size) return;
    const uint32_t base = io_begin(v, seg);
    const uint32_t d = seg_dim(segdim, dimrr, seg);
    uint64_t key[G];
    uint32_t slot[G];
#pragma unroll
    for (int x = 0; x < G; ++x) {
        const uint32_t r = group_pos(gb, (uint32_t)x, e0);
        slot[x] = (uint32_t)x;
        key[x] = ~0ull;     // past the subtree's end: +infinity
        if (r < size) key[x] = rkey<I32>(pts[(size_t)(base + r) * K + d], perm[base + r]);
    }
#pragma unroll
    for (int sb = C - 1; sb >= 0; --sb) {
#pragma unroll
        for (int p = 0; p < G / 2; ++p) {
            const int x = ((p >> sb) << (sb + 1)) | (p & ((1 << sb) - 1));
            const int y = x | (1 << sb);
            if (key[x] > key[y]) {
                const uint64_t tk = key[x];
                key[x] = key[y];
                key[y] = tk;
                const uint32_t ts = slot[x];
                slot[x] = slot[y];
                slot[y] = ts;
            }
        }
    }
    uint32_t rc[G][K];
#pragma unroll
    for (int x = 0; x < G; ++x)
        if (slot[x] != (uint32_t)x) ld_pt<K>(pts, base + group_pos(gb, slot[x], e0), rc[x]);
#pragma unroll
    for (int x = 0; x < G; ++x) {
        if (slot[x] != (uint32_t)x) {
            const uint32_t r = group_pos(gb, (uint32_t)x, e0);
            st_pt<K>(pts, base + r, rc[x]);
            perm[base + r] = (uint32_t)key[x];
        }
    }
}

// The iterations lg .. L-2 of one level-lg subtree (at most BLK - 1 nodes)
// in LDS, and the split dimensions of its nodes (levels lg .. L-1).  Each
// iteration sorts (key, slot) pairs of every sub-segment with the bitonic
// network, then moves the records to their new slots.
template <int K, bool I32, bool WIDE>
__global__ __launch_bounds__(256) void k_ip_deep(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm, uint32_t n,
                                                 uint32_t lg, const uint32_t* hdr, const uint32_t* boxes,
                                                 uint8_t* dim, uint32_t* hdr_w)
{
    constexpr uint32_t E = BLK / THREADS;
    __shared__ Lds<K> s;
    __shared__ uint64_t key[BLK];
    __shared__ uint16_t slot[BLK];
    __shared__ uint8_t sdim[BLK / 2];
    const uint32_t L = num_levels(n);
    const uint32_t i0 = blockIdx.x;
    const Level v0 = make_level(n, lg);
    const uint32_t base0 = io_begin(v0, i0);
    const uint32_t cnt = seg_size(v0, i0);
    if (cnt >= BLK || base0 + cnt > n) {
        if (threadIdx.x == 0) atomicOr(&hdr_w[HDR_STATUS], KDT_STATUS_INTERNAL);
        return;
    }
    uint32_t rlo[K], rhi[K];
    if (WIDE) {
#pragma unroll
        for (int d = 0; d < K; ++d) {
            rlo[d] = lg ? boxes[(size_t)i0 * 8 + d] : hdr[HDR_LO + d];
            rhi[d] = lg ? boxes[(size_t)i0 * 8 + 4 + d] : hdr[HDR_HI + d];
        }
    }
    lds_load<K>(s, pts, perm, base0, cnt);
    __syncthreads();
    for (uint32_t lp = lg; lp < L; ++lp) {
        const Level v = make_level(n, lp);
        const uint32_t rel = lp - lg;
        const uint32_t nsub = 1u << rel;
        const bool last = lp + 1u == L;
        for (uint32_t j = threadIdx.x; j < nsub; j += THREADS) {
            const uint32_t ig = (i0 << rel) | j;
            if (last && ig >= v.R) continue;                // no such leaf
            uint32_t dd;
            if (WIDE) {
                uint32_t lo[K], hi[K];
#pragma unroll
                for (int d = 0; d < K; ++d) {
                    lo[d] = rlo[d];
                    hi[d] = rhi[d];
                }
                for (uint32_t a = lg; a < lp; ++a) {
                    const Level va = make_level(n, a);
                    const uint32_t ia = ig >> (lp - a);
                    const uint32_t d = widest_dim<K, I32>(lo, hi);
                    const uint32_t kk = coord_key<I32>(s.c[d][io_pivot(va, ia) - base0]);
                    if ((ig >> (lp - a - 1u)) & 1u)
                        set_at<K>(lo, d, kk);
                    else
                        set_at<K>(hi, d, kk);
                }
                dd = widest_dim<K, I32>(lo, hi);
            } else {
                dd = lp % (uint32_t)K;
            }
            sdim[j] = (uint8_t)dd;
            if (dim && WIDE) dim[full_nodes(lp) + ig] = (uint8_t)dd;
        }
        if (last) break;
        __syncthreads();
        // keys of this iteration: (coordinate in the sub-segment's dimension, index)
        for (uint32_t p = threadIdx.x; p < cnt; p += THREADS) {
            const uint32_t sg = io_seg_of(v, base0 + p);
            const uint32_t dd = sg == 0xFFFFFFFFu ? 0u : (uint32_t)sdim[sg - (i0 << rel)];
            key[p] = rkey<I32>(s.c[dd][p], s.id[p]);
            slot[p] = (uint16_t)p;
        }
        __syncthreads();
        const uint32_t P = net_len(v);
        const uint32_t logP = log2_exact(P);
        const uint32_t pairs = nsub << (logP - 1u);
        for (uint32_t e = 1; e <= logP; ++e) {
            for (int ls = (int)e - 1; ls >= 0; --ls) {
                for (uint32_t g = threadIdx.x; g < pairs; g += THREADS) {
                    const uint32_t j = g >> (logP - 1u);
                    const uint32_t q = g & ((P >> 1) - 1u);
                    const uint32_t ig = (i0 << rel) | j;
                    const uint32_t size = seg_size(v, ig);
                    uint32_t lo, hi;
                    if (ls == (int)e - 1)
                        mirror_pair(q, e, lo, hi);
                    else
                        half_pair(q, (uint32_t)ls, lo, hi);
                    if (hi < size) {
                        const uint32_t pb = io_begin(v, ig) - base0;
                        const uint64_t a = key[pb + lo], b = key[pb + hi];
                        if (a > b) {
                            key[pb + lo] = b;
                            key[pb + hi] = a;
                            const uint16_t ts = slot[pb + lo];
                            slot[pb + lo] = slot[pb + hi];
                            slot[pb + hi] = ts;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // records to their new slots: read every moved record, then write
        uint32_t rc[E][K];
        uint32_t rid[E];
#pragma unroll
        for (uint32_t j = 0; j < E; ++j) {
            const uint32_t p = threadIdx.x + j * THREADS;
            if (p < cnt && slot[p] != p) {
                const uint32_t src = slot[p];
#pragma unroll
                for (int d = 0; d < K; ++d) rc[j][d] = s.c[d][src];
                rid[j] = s.id[src];
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < E; ++j) {
            const uint32_t p = threadIdx.x + j * THREADS;
            if (p < cnt && slot[p] != p) {
#pragma unroll
                for (int d = 0; d < K; ++d) s.c[d][p] = rc[j][d];
                s.id[p] = rid[j];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    lds_store<K>(s, pts, perm, base0, cnt);
}

// In-order -> level order, op OP_UNSHUF_LDS: block b of [a, a+n) becomes
// its odd offsets, then its even offsets.
template <int K>
__global__ __launch_bounds__(256) void k_ip_unshuf(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm, uint32_t a,
                                                   uint32_t n)
{
    __shared__ Lds<K> s;
    const uint32_t b0 = blockIdx.x * BLK;
    const uint32_t cnt = umin(BLK, n - b0);
    const uint32_t nodd = cnt >> 1;
    for (uint32_t j = threadIdx.x; j < cnt; j += THREADS) {
        const uint32_t dst = (j & 1u) ? (j >> 1) : nodd + (j >> 1);
        uint32_t c[K];
        ld_pt<K>(pts, a + b0 + j, c);
#pragma unroll
        for (int d = 0; d < K; ++d) s.c[d][dst] = c[d];
        s.id[dst] = perm[a + b0 + j];
    }
    __syncthreads();
    lds_store<K>(s, pts, perm, a + b0, cnt);
}

// OP_SWAP_LEVEL: in every full 2^j-block of [a, a+n), swap its second
// quarter with its third.
template <int K>
__global__ __launch_bounds__(256) void k_ip_swaplevel(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm,
                                                      uint32_t a, uint32_t j, uint32_t total)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const uint32_t Q = 1u << (j - 2u);
    const uint32_t x = a + ((g >> (j - 2u)) << j) + Q + (g & (Q - 1u));
    swap_rec<K>(pts, perm, x, x + Q);
}

// OP_REVERSE: reverse [a, a+n).
template <int K>
__global__ __launch_bounds__(256) void k_ip_reverse(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm,
                                                    uint32_t a, uint32_t n)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (n >> 1)) return;
    swap_rec<K>(pts, perm, a + g, a + n - 1u - g);
}

// OP_LDS_TREE: [0, n) from in-order to level order, n <= BLK.
template <int K>
__global__ __launch_bounds__(256) void k_ip_ldstree(uint32_t* __restrict__ pts, uint32_t* __restrict__ perm,
                                                    uint32_t n)
{
    __shared__ Lds<K> s;
    for (uint32_t j = threadIdx.x; j < n; j += THREADS) {
        const uint32_t dst = inorder_to_level(j, n);
        uint32_t c[K];
        ld_pt<K>(pts, j, c);
#pragma unroll
        for (int d = 0; d < K; ++d) s.c[d][dst] = c[d];
        s.id[dst] = perm[j];
    }
    __syncthreads();
    lds_store<K>(s, pts, perm, 0u, n);
}

__global__ void k_ip_rrdims(uint8_t* dim, uint32_t n, uint32_t k)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dim[s] = (uint8_t)(level_of(s) % k);
}

__global__ void k_ip_finish(const uint32_t* hdr, uint32_t* status)
{
    if (threadIdx.x == 0) *status = hdr[HDR_STATUS];
}

// ------------------------------------------------------------ host driver

inline uint32_t blocks_for(size_t threads) { return (uint32_t)((threads + 255) / 256); }

struct Call {
    uint32_t* pts;
    uint32_t* perm;
    uint8_t* dim;
    uint32_t* status;
    char* ws;
    uint32_t n, k;
    bool wide;
    hipStream_t st;
};

template <int K, bool I32>
struct Driver {
    static constexpr double REC = 4.0 * (K + 1);   // bytes of one record (point + index)

    static kdt_status run(const Call& c)
    {
        const WsLayout w = ws_layout(c.n, c.wide);
        uint32_t* hdr = (uint32_t*)c.ws;
        uint8_t* segdim = (uint8_t*)(c.ws + w.segdim);
        uint32_t* boxes = (uint32_t*)(c.ws + w.boxes);
        const uint32_t n = c.n;
        const uint32_t L = num_levels(n);
        const uint32_t lg = deep_level(L);
        hipStream_t st = c.st;

        if (kdt_status s = launch_profiled(st, KIND_IP_INIT, 0.0, 0.0, [&] { k_ip_clear<<<1, 64, 0, st>>>(hdr); }))
            return s;
        {
            const uint32_t nb = umin(blocks_for(n), 2048u);
            const double bytes = 4.0 * n + ((c.wide || !I32) ? 4.0 * K * n : 0.0);
            kdt_status s = launch_profiled(st, KIND_IP_INIT, bytes, 0.0, [&] {
                if (c.wide)
                    k_ip_init<K, I32, true><<<nb, 256, 0, st>>>(c.pts, c.perm, n, hdr);
                else
                    k_ip_init<K, I32, false><<<nb, 256, 0, st>>>(c.pts, c.perm, n, hdr);
            });
            if (s) return s;
        }
        for (uint32_t l = 0; l < lg; ++l) {
            const Level v = make_level(n, l);
            const uint32_t live = n - v.Fl;               // points of the level's subtrees
            const double pass = 2.0 * REC * live;         // read + write every record once
            const double method = 8.0 * (K + 1.0) * live; // the paper's iteration: each live point read + written
            const uint8_t* sd = c.wide ? segdim : nullptr;
            const uint32_t dimrr = l % K;
            if (c.wide) {
                kdt_status s = launch_profiled(st, KIND_IP_SETUP, 0.0, 0.0, [&] {
                    k_ip_setup<K, I32><<<blocks_for(v.nseg), 256, 0, st>>>(c.pts, n, l, hdr, segdim, nullptr,
                                                                            c.dim);
                });
                if (s) return s;
            }
            const uint32_t nblk = tiles_level(v, SBLK).tiles;
            const uint32_t logP = log2_exact(net_len(v));
            std::vector<Step> steps;
            plan_level_sort(logP, [&](const Step& x) { steps.push_back(x); });
            for (const Step& x : steps) {
                kdt_status s = KDT_OK;
                switch (x.kind) {
                case ST_BLOCK_SORT:
                    s = launch_profiled(st, KIND_IP_BLOCK, pass, method, [&] {
                        k_ip_block<K, I32, true><<<nblk, THREADS, 0, st>>>(c.pts, c.perm, n, l, dimrr, sd, hdr);
                    });
                    break;
                case ST_MGROUP: {
                    const uint32_t nb = blocks_for((size_t)v.nseg << (logP - x.c - 1u));
                    s = launch_profiled(st, KIND_IP_MIRROR, pass, 0.0, [&] {
                        switch (x.c) {
                        case 1: k_ip_mgroup<K, I32, 1><<<nb, 256, 0, st>>>(c.pts, c.perm, n, l, logP, x.e, dimrr, sd); break;
                        case 2: k_ip_mgroup<K, I32, 2><<<nb, 256, 0, st>>>(c.pts, c.perm, n, l, logP, x.e, dimrr, sd); break;
                        default: k_ip_mgroup<K, I32, 3><<<nb, 256, 0, st>>>(c.pts, c.perm, n, l, logP, x.e, dimrr, sd); break;
                        }
                    });
                    break;
                }
                case ST_GROUP: {
                    const uint32_t nb = blocks_for((size_t)v.nseg << (logP - x.c));
                    s = launch_profiled(st, KIND_IP_GROUP, pass, 0.0, [&] {
                        switch (x.c) {
                        case 1: k_ip_group<K, I32, 1><<<nb, 256, 0, st>>>(c.pts, c.perm, n, l, logP, x.e0, dimrr, sd); break;
                        case 2: k_ip_group<K, I32, 2><<<nb, 256, 0, st>>>(c.pts, c.perm, n, l, logP, x.e0, dimrr, sd); break;
                        case 3: k_ip_group<K, I32, 3><<<nb, 256, 0, st>>>(c.pts, c.perm, n, l, logP, x.e0, dimrr, sd); break;
                        default: k_ip_group<K, I32, 4><<<nb, 256, 0, st>>>(c.pts, c.perm, n, l, logP, x.e0, dimrr, sd); break;
                        }
                    });
                    break;
                }
                default:
                    s = launch_profiled(st, KIND_IP_BLOCK, pass, 0.0, [&] {
                        k_ip_block<K, I32, false><<<nblk, THREADS, 0, st>>>(c.pts, c.perm, n, l, dimrr, sd, hdr);
                    });
                    break;
                }
                if (s) return s;
            }
        }
        if (c.wide && lg > 0) {
            kdt_status s = launch_profiled(st, KIND_IP_SETUP, 0.0, 0.0, [&] {
                k_ip_setup<K, I32><<<blocks_for((size_t)1 << lg), 256, 0, st>>>(c.pts, n, lg, hdr, nullptr, boxes,
                                                                                 nullptr);
            });
            if (s) return s;
        }
        {
            double method = 0.0;
            for (uint32_t l = lg; l + 2u <= L; ++l) method += 8.0 * (K + 1.0) * (n - full_nodes(l));
            kdt_status s = launch_profiled(st, KIND_IP_DEEP, 2.0 * REC * n, method, [&] {
                if (c.wide)
                    k_ip_deep<K, I32, true><<<1u << lg, THREADS, 0, st>>>(c.pts, c.perm, n, lg, hdr, boxes, c.dim, hdr);
                else
                    k_ip_deep<K, I32, false><<<1u << lg, THREADS, 0, st>>>(c.pts, c.perm, n, lg, hdr, boxes, c.dim, hdr);
            });
            if (s) return s;
        }
        // in-order -> level order; the final placement of Sec. 5 (8k bytes per point)
        // is charged to the first op
        std::vector<Op> ops;
        plan_to_level_order(n, [&](const Op& o) { ops.push_back(o); });
        double place = 8.0 * K * n;
        for (const Op& o : ops) {
            kdt_status s = KDT_OK;
            const uint32_t work = op_work(o);
            switch (o.kind) {
            case OP_UNSHUF_LDS:
                s = launch_profiled(st, KIND_IP_PERM, 2.0 * REC * o.n, place, [&] {
                    k_ip_unshuf<K><<<work, THREADS, 0, st>>>(c.pts, c.perm, o.a, o.n);
                });
                break;
            case OP_SWAP_LEVEL:
                s = launch_profiled(st, KIND_IP_PERM, 4.0 * REC * work, place, [&] {
                    k_ip_swaplevel<K><<<blocks_for(work), 256, 0, st>>>(c.pts, c.perm, o.a, o.j, work);
                });
                break;
            case OP_REVERSE:
                if (!work) continue;
                s = launch_profiled(st, KIND_IP_PERM, 4.0 * REC * work, place, [&] {
                    k_ip_reverse<K><<<blocks_for(work), 256, 0, st>>>(c.pts, c.perm, o.a, o.n);
                });
                break;
            default:
                s = launch_profiled(st, KIND_IP_PERM, 2.0 * REC * o.n, place, [&] {
                    k_ip_ldstree<K><<<1, THREADS, 0, st>>>(c.pts, c.perm, o.n);
                });
                break;
            }
            if (s) return s;
            place = 0.0;
        }
        if (!c.wide && c.dim) {
            kdt_status s = launch_profiled(st, KIND_IP_INIT, (double)n, 0.0, [&] {
                k_ip_rrdims<<<blocks_for(n), 256, 0, st>>>(c.dim, n, K);
            });
            if (s) return s;
        }
        if (c.status) {
            kdt_status s = launch_profiled(st, KIND_IP_INIT, 0.0, 0.0, [&] { k_ip_finish<<<1, 64, 0, st>>>(hdr, c.status); });
            if (s) return s;
        }
        return KDT_OK;
    }
};

template <bool I32>
kdt_status dispatch(const Call& c)
{
    switch (c.k) {
    case 1: return Driver<1, I32>::run(c);
    case 2: return Driver<2, I32>::run(c);
    case 3: return Driver<3, I32>::run(c);
    default: return Driver<4, I32>::run(c);
    }
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    if (!a || !b || !na || !nb) return false;
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

kdt_status build_inplace_any(void* d_points, uint32_t n, uint32_t k, int mode, uint32_t* d_perm, uint8_t* d_dim,
                             uint32_t* d_status, void* d_ws, size_t ws_bytes, hipStream_t stream, bool i32)
{
    if (k < 1 || k > 4 || (mode != KDT_DIM_ROUND_ROBIN && mode != KDT_DIM_WIDEST)) {
        set_last_error("k must be in 1..4 and dim_mode a kdt_dim_mode (got k = %u, mode %d)", k, mode);
        return KDT_EINVAL;
    }
    if (n > KDT_MAX_POINTS) {
        set_last_error("n = %u exceeds KDT_MAX_POINTS", n);
        return KDT_EINVAL;
    }
    const bool wide = mode == KDT_DIM_WIDEST;
    const WsLayout w = ws_layout(n, wide);
    if (n > 0 && (!d_points || !d_perm)) {
        set_last_error("points and perm must not be null");
        return KDT_EINVAL;
    }
    if (!d_ws || ws_bytes < w.total) {
        set_last_error("workspace of %zu bytes needed (got %zu)", w.total, d_ws ? ws_bytes : (size_t)0);
        return KDT_EINVAL;
    }
    if (((uintptr_t)d_ws) % WS_ALIGN_IP) {
        set_last_error("workspace must be %zu-byte aligned", WS_ALIGN_IP);
        return KDT_EINVAL;
    }
    if (((uintptr_t)d_points) % (k == 4 ? 16 : k == 2 ? 8 : 4) || ((uintptr_t)d_perm) % 4) {
        set_last_error("points must be aligned to their point size (4, 8 or 16 bytes), perm to 4 bytes");
        return KDT_EINVAL;
    }
    const size_t pb = (size_t)n * k * 4;
    if (overlaps(d_points, pb, d_perm, (size_t)n * 4) || overlaps(d_points, pb, d_dim, n) ||
        overlaps(d_points, pb, d_ws, ws_bytes) || overlaps(d_perm, (size_t)n * 4, d_dim, n) ||
        overlaps(d_perm, (size_t)n * 4, d_ws, ws_bytes) || overlaps(d_dim, n, d_ws, ws_bytes) ||
        overlaps(d_status, 4, d_ws, ws_bytes) || overlaps(d_status, 4, d_points, pb) ||
        overlaps(d_status, 4, d_perm, (size_t)n * 4)) {
        set_last_error("points, perm, dim, status and workspace must not overlap");
        return KDT_EINVAL;
    }
    if (n == 0) {
        if (!d_status) return KDT_OK;
        launch_set_word(d_status, 0u, stream);
        return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
    }
    const Call c{(uint32_t*)d_points, d_perm, d_dim, d_status, (char*)d_ws, n, k, wide, stream};
    return i32 ? dispatch<true>(c) : dispatch<false>(c);
}

}  // namespace ip
}  // namespace kdt

extern "C" {

size_t kdt_inplace_workspace_bytes(uint32_t n, uint32_t k, int dim_mode)
{
    if (k < 1 || k > 4 || n > KDT_MAX_POINTS || (dim_mode != KDT_DIM_ROUND_ROBIN && dim_mode != KDT_DIM_WIDEST))
        return 0;
    return kdt::ip::ws_layout(n, dim_mode == KDT_DIM_WIDEST).total;
}

kdt_status kdt_build_inplace(float* d_points, uint32_t n, uint32_t k, int dim_mode, uint32_t* d_perm,
                             uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes, hipStream_t stream)
{
    return kdt::ip::build_inplace_any(d_points, n, k, dim_mode, d_perm, d_dim, d_status, d_ws, ws_bytes, stream,
                                      false);
}

kdt_status kdt_build_inplace_i32(int32_t* d_points, uint32_t n, uint32_t k, int dim_mode, uint32_t* d_perm,
                                 uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream)
{
    return kdt::ip::build_inplace_any(d_points, n, k, dim_mode, d_perm, d_dim, d_status, d_ws, ws_bytes, stream,
                                      true);
}

}  // extern "C"
