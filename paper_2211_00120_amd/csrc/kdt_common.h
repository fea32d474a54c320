// kdt_common.h -- device helpers shared by the build kernels: share lookup,
// placement of fixed nodes, split-widest child dimensions, record I/O.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdt_device.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"

namespace kdt {

// Bounds guard of every scatter: a position outside its buffer flags an
// internal error in the status word instead of writing.
__device__ __forceinline__ bool in_bounds(uint32_t pos, uint32_t limit, uint32_t* status)
{
    if (pos < limit) return true;
    atomicOr(status, KDT_STATUS_INTERNAL);
    return false;
}

// The share that tile (or workgroup) g belongs to; g is the same in every
// lane.  The result is made wave-uniform field by field, so that it and all
// the segment arithmetic derived from it live in scalar registers.
__device__ __forceinline__ void uniform_step(TreeStep& st, const TreeStep& s)
{
    st.tree = uniform(s.tree);
    st.level = uniform(s.level);
    st.tile0 = uniform(s.tile0);
    st.hist = uniform(s.hist);
    st.hist_next = uniform(s.hist_next);
    st.pair0 = uniform(s.pair0);
    st.buf = uniform(s.buf);
    st.piv = uniform(s.piv);
}

__device__ __forceinline__ void uniform_tree(TreeInfo& ti, const TreeInfo& t)
{
    ti.off = uniform(t.off);
    ti.n = uniform(t.n);
    ti.box_off = uniform(t.box_off);
    ti.idx = uniform(t.idx);
}

// (fields are read one by one in each branch: a copy of the whole struct
// through a select between the kernel argument and the table can leave a
// private-memory frame behind)
__device__ __forceinline__ void find_share(const Shares& sh, uint32_t g, TreeStep& st, TreeInfo& ti)
{
    if (sh.steps == nullptr) {
        uniform_step(st, sh.step0);
        uniform_tree(ti, sh.tree0);
        return;
    }
    uint32_t lo = 0, hi = sh.nsteps - 1u;
    while (lo < hi) {                   // largest i with steps[i].tile0 <= g
        const uint32_t mid = (lo + hi + 1u) >> 1;
        if (sh.steps[mid].tile0 <= g) lo = mid;
        else hi = mid - 1u;
    }
    uniform_step(st, sh.steps[lo]);
    uniform_tree(ti, sh.trees[st.tree]);
}

// Node `node` of tree ti holds its point of local index idx.
template <int K, bool WIDEST>
__device__ __forceinline__ void place(const Outs& o, const TreeInfo& ti, uint32_t node, uint32_t idx)
{
    if (!in_bounds(node, ti.n, o.status) || !in_bounds(idx, ti.n, o.status)) return;
    const size_t at = (size_t)ti.off + node;
    if (o.tree) {
#pragma unroll
        for (int d = 0; d < K; ++d) o.tree[at * K + d] = o.pts[((size_t)ti.off + idx) * K + d];
    }
    o.nodeperm[at] = idx;
    if (!WIDEST && o.dim) o.dim[at] = (uint8_t)(level_of(node) % (uint32_t)K);
}

// place() with the point's coordinates already loaded.
template <int K, bool WIDEST>
__device__ __forceinline__ void place_pt(const Outs& o, const TreeInfo& ti, uint32_t node, uint32_t idx,
                                         const float4& p)
{
    if (!in_bounds(node, ti.n, o.status)) return;
    const size_t at = (size_t)ti.off + node;
    if (o.tree) {
        float* t = o.tree + at * K;
        t[0] = p.x;
        if (K > 1) t[1] = p.y;
        if (K > 2) t[2] = p.z;
        if (K > 3) t[3] = p.w;
    }
    o.nodeperm[at] = idx;
    if (!WIDEST && o.dim) o.dim[at] = (uint8_t)(level_of(node) % (uint32_t)K);
}

template <int K>
__device__ __forceinline__ float4 load_point(const float* __restrict__ pts, size_t i)
{
    const float* p = pts + i * K;
    if constexpr (K == 4) return *reinterpret_cast<const float4*>(p);
    else if constexpr (K == 3) return make_float4(p[0], p[1], p[2], 0.f);
    else if constexpr (K == 2) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        return make_float4(v.x, v.y, 0.f, 0.f);
    } else return make_float4(p[0], 0.f, 0.f, 0.f);
}

__device__ __forceinline__ float pickf(const float4& p, uint32_t d)
{
    const float x = p.x, y = p.y, z = p.z, w = p.w;
    return d == 0u ? x : (d == 1u ? y : (d == 2u ? z : w));
}

// Key of coordinate d of local point idx of tree ti (the split plane of the
// node that point is placed at).
template <bool I32>
__device__ __forceinline__ uint32_t plane_key(const Outs& o, const TreeInfo& ti, uint32_t idx, uint32_t d, uint32_t k)
{
    const uint32_t* bits = reinterpret_cast<const uint32_t*>(o.pts);
    return coord_key<I32>(bits[((size_t)ti.off + idx) * k + d]);
}

// Split-widest (Sec. 6): the domain of a child of subtree s is s's domain
// bc (keys of lo[0..3], hi[4..7]) clipped by s's plane (left child c = 0:
// hi = plane, right child c = 1: lo = plane); the child's split dimension is
// its domain's widest extent.  plane is the key of the pivot's coordinate in
// s's split dimension ds.
template <int K>
__device__ __forceinline__ void split_box(const uint32_t* bc, uint32_t plane, uint32_t ds, uint32_t c,
                                          uint32_t (&l2)[K], uint32_t (&h2)[K])
{
#pragma unroll
    for (int d = 0; d < K; ++d) {
        l2[d] = bc[d];
        h2[d] = bc[4 + d];
        if ((uint32_t)d == ds) {
            if (c == 0u) h2[d] = min(h2[d], plane);
            else l2[d] = max(l2[d], plane);
        }
    }
}

template <int K, bool I32>
__device__ __forceinline__ uint32_t child_dim(const uint32_t* bc, uint32_t plane, uint32_t ds, uint32_t c)
{
    uint32_t l2[K], h2[K];
    split_box<K>(bc, plane, ds, c, l2, h2);
    return widest_dim<K, I32>(l2, h2);
}

// Writes the children's dimensions of subtree s (the i-th of its level in
// tree ti, domain box_cur[box_off + i]) to dimnode and, when box_next is
// set, their domains to box_next[box_off + 2i (+1)].
template <int K, bool I32>
__device__ void widest_children(const Outs& o, const TreeInfo& ti, uint32_t s, uint32_t i, uint32_t plane,
                                uint32_t ds, const uint32_t* box_cur, uint32_t* box_next)
{
    const uint32_t* bc = box_cur + ((size_t)ti.box_off + i) * 8;
#pragma unroll
    for (uint32_t c = 0; c < 2u; ++c) {
        const uint32_t child = 2u * s + 1u + c;
        if (child >= ti.n) continue;
        uint32_t l2[K], h2[K];
        split_box<K>(bc, plane, ds, c, l2, h2);
        o.dimnode[(size_t)ti.off + child] = (uint8_t)widest_dim<K, I32>(l2, h2);
        if (box_next) {
            uint32_t* bn = box_next + ((size_t)ti.box_off + 2u * i + c) * 8;
#pragma unroll
            for (int d = 0; d < K; ++d) {
                bn[d] = l2[d];
                bn[4 + d] = h2[d];
            }
        }
    }
}

// Records held in registers as uint4 (k <= 4 ranks; unused words are 0).
template <int K>
__device__ __forceinline__ uint4 load_rec4(const uint32_t* __restrict__ p, size_t i)
{
    if constexpr (K == 4) {
        return reinterpret_cast<const uint4*>(p)[i];
    } else if constexpr (K == 2) {
        const uint2 v = reinterpret_cast<const uint2*>(p)[i];
        return make_uint4(v.x, v.y, 0u, 0u);
    } else if constexpr (K == 3) {
        return make_uint4(p[i * 3], p[i * 3 + 1], p[i * 3 + 2], 0u);
    } else {
        return make_uint4(p[i], 0u, 0u, 0u);
    }
}
// Records are written with non-temporal stores: the next pass reads them
// once, much later, while the split keys written beside them are read by the
// pivot selects right away and should keep the last-level cache (2.45 ->
// 2.21 ms of selects per 100M-point build).
template <int K>
__device__ __forceinline__ void store_rec4(uint32_t* __restrict__ p, size_t i, uint4 r)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    if constexpr (K == 4) {
        const u32x4 v = {r.x, r.y, r.z, r.w};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(p) + i);
    } else if constexpr (K == 2) {
        const u32x2 v = {r.x, r.y};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x2*>(p) + i);
    } else if constexpr (K == 3) {
        __builtin_nontemporal_store(r.x, p + i * 3);
        __builtin_nontemporal_store(r.y, p + i * 3 + 1);
        __builtin_nontemporal_store(r.z, p + i * 3 + 2);
    } else {
        __builtin_nontemporal_store(r.x, p + i);
    }
}
__device__ __forceinline__ uint32_t pick4(uint4 r, uint32_t d)
{
    const uint32_t x = r.x, y = r.y, z = r.z, w = r.w;
    return d == 0u ? x : (d == 1u ? y : (d == 2u ? z : w));
}

__device__ __forceinline__ void set4(uint4& r, uint32_t d, uint32_t v)
{
    r.x = d == 0u ? v : r.x;
    r.y = d == 1u ? v : r.y;
    r.z = d == 2u ? v : r.z;
    r.w = d == 3u ? v : r.w;
}

// Lanes of this wave whose (valid, value) agree with this lane's on the low
// `bits` bits of value (bits <= 16; one ballot per bit).
__device__ __forceinline__ uint64_t match_bits(uint32_t value, uint32_t bits, bool valid)
{
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    for (uint32_t b = 0; b < bits; ++b) match_bit(~value, b, lo, hi);
    return ((uint64_t)hi << 32) | lo;
}

// Key summaries of a tree (its KEYSUM_WORDS words), combined over the
// copies: the least and greatest key of dimension d.
__device__ __forceinline__ void keysum_box(const uint32_t* sum, uint32_t d, uint32_t& lo, uint32_t& hi)
{
    lo = 0xFFFFFFFFu;
    hi = 0u;
#pragma unroll
    for (uint32_t c = 0; c < KEYSUM_COPIES; ++c) {
        lo = min(lo, sum[c * KEYSUM_COPY_WORDS + d]);
        hi = max(hi, sum[c * KEYSUM_COPY_WORDS + 4u + d]);
    }
}

__device__ __forceinline__ void zero_range(uint32_t* p, uint32_t n)
{
    if (!p) return;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) p[x] = 0u;
}

}  // namespace kdt
