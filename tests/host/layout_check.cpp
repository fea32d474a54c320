// Host check of the implicit-tree arithmetic in kdt_layout.h against direct
// enumeration of the level-order tree (no closed forms on this side).
// Usage: layout_check            -> exhaustive for N <= 3000, sampled above
// Prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "kdt_layout.h"

using namespace kdt;

static uint64_t count_subtree(uint64_t s, uint64_t n)
{
    // explicit stack walk over existing nodes
    uint64_t c = 0;
    std::vector<uint64_t> st{s};
    while (!st.empty()) {
        uint64_t x = st.back();
        st.pop_back();
        if (x >= n) continue;
        ++c;
        st.push_back(2 * x + 1);
        st.push_back(2 * x + 2);
    }
    return c;
}

static int fail(const char* what, uint32_t n, uint32_t l, uint32_t i, uint64_t got, uint64_t want)
{
    std::printf("FAIL %s n=%u l=%u i=%u got=%llu want=%llu\n", what, n, l, i, (unsigned long long)got,
                (unsigned long long)want);
    return 1;
}

static int check_n(uint32_t n, bool full)
{
    const uint32_t L = num_levels(n);
    uint32_t depth = 0;
    while ((2ull << depth) - 1 < n) ++depth;     // levels by counting
    if (L != depth + 1) return fail("num_levels", n, 0, 0, L, depth + 1);
    for (uint32_t l = 0; l + 2 <= L; ++l) {
        const Level v = make_level(n, l);
        std::vector<uint64_t> sizes(v.nseg), offs(v.nseg);
        uint64_t acc = 0;
        for (uint32_t i = 0; i < v.nseg; ++i) {
            const uint64_t s = (1ull << l) - 1 + i;
            sizes[i] = count_subtree(s, n);
            offs[i] = acc;
            acc += sizes[i];
        }
        if (acc != n - v.Fl) return fail("live", n, l, 0, acc, n - v.Fl);
        const uint32_t step = full ? 1 : (v.nseg > 64 ? v.nseg / 61 : 1);
        for (uint32_t i = 0; i < v.nseg; i += step) {
            const uint64_t s = (1ull << l) - 1 + i;
            if (seg_size(v, i) != sizes[i]) return fail("seg_size", n, l, i, seg_size(v, i), sizes[i]);
            if (seg_offset(v, i) != offs[i]) return fail("seg_offset", n, l, i, seg_offset(v, i), offs[i]);
            const uint64_t left = count_subtree(2 * s + 1, n);
            if (seg_left_size(v, i) != left) return fail("seg_left_size", n, l, i, seg_left_size(v, i), left);
            if (seg_pivot(v, i) != offs[i] + left) return fail("seg_pivot", n, l, i, seg_pivot(v, i), offs[i] + left);
            // inverse map at the segment's first, pivot and last positions
            const uint64_t probes[3] = {offs[i], offs[i] + left, offs[i] + sizes[i] - 1};
            for (uint64_t p : probes)
                if (seg_of_pos(v, (uint32_t)p) != i) return fail("seg_of_pos", n, l, i, seg_of_pos(v, (uint32_t)p), i);
        }
        // tiling: every live position covered exactly once, tiles never straddle
        for (uint32_t tile : {1u, 3u, 64u, 2048u}) {
            const SegTiles t = tiles_level(v, tile);
            if (!full && t.tiles > 200000) continue;
            std::vector<uint8_t> hit(n - v.Fl, 0);
            for (uint32_t g = 0; g < t.tiles; ++g) {
                uint32_t seg, u;
                tile_locate(t, g, seg, u);
                if (seg >= v.nseg) return fail("tile seg", n, l, g, seg, v.nseg);
                if (tiles_seg_offset(t, seg) != offs[seg]) return fail("tile off", n, l, seg, tiles_seg_offset(t, seg), offs[seg]);
                if (tiles_seg_size(t, seg) != sizes[seg]) return fail("tile size", n, l, seg, tiles_seg_size(t, seg), sizes[seg]);
                const uint64_t a = offs[seg] + (uint64_t)u * tile;
                if (a >= offs[seg] + sizes[seg]) return fail("tile empty", n, l, g, a, offs[seg] + sizes[seg]);
                const uint64_t b = std::min<uint64_t>(a + tile, offs[seg] + sizes[seg]);
                for (uint64_t p = a; p < b; ++p) {
                    if (hit[p]) return fail("tile overlap", n, l, g, p, 0);
                    hit[p] = 1;
                }
                if (u > 0) {   // previous tile belongs to the same segment
                    uint32_t s2, u2;
                    tile_locate(t, g - 1, s2, u2);
                    if (s2 != seg || u2 + 1 != u) return fail("tile order", n, l, g, s2, seg);
                }
            }
            for (uint64_t p = 0; p < hit.size(); ++p)
                if (!hit[p]) return fail("tile gap", n, l, tile, p, 0);
        }
    }
    return 0;
}

// Arguments at and beyond the edges of the arithmetic: every function must
// return a defined value (the sanitizer build of this file traps on an
// undefined shift, a clz of 0 or a division by zero).
static int check_edges()
{
    if (num_levels(0) != 0) return fail("num_levels(0)", 0, 0, 0, num_levels(0), 0);
    if (level_of(0xFFFFFFFFu) != 32) return fail("level_of(2^32-1)", 0, 0, 0, level_of(0xFFFFFFFFu), 32);
    if (level_of(0xFFFFFFFEu) != 31) return fail("level_of(2^32-2)", 0, 0, 0, level_of(0xFFFFFFFEu), 31);
    if (full_nodes(32) != 0xFFFFFFFFu || full_nodes(40) != 0xFFFFFFFFu || full_nodes(31) != 0x7FFFFFFFu)
        return fail("full_nodes", 0, 32, 0, full_nodes(32), 0xFFFFFFFFu);
    if (rank_bits(0) != 0 || rank_bits(1) != 0 || rank_bits(2) != 1 || rank_bits(0xFFFFFFFFu) != 32)
        return fail("rank_bits", 0, 0, 0, rank_bits(0xFFFFFFFFu), 32);
    // n = 0: no levels, no subtrees
    for (uint32_t l : {0u, 1u, 31u, 32u, 33u}) {
        const Level v = make_level(0, l);
        if (v.L != 0 || v.W != 0 || v.R != 0) return fail("make_level(0)", 0, l, 0, v.W, 0);
        (void)seg_of_pos(v, 0);
        (void)tiles_level(v, 64);
    }
    const uint32_t ns[] = {1u, 2u, 3u, 7u, 8u, 1000u, 0x3FFFFFFFu, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFFFu};
    for (uint32_t n : ns) {
        const uint32_t L = num_levels(n);
        for (uint32_t l = (L >= 2 ? L - 2 : 0); l <= L + 2 && l < 40; ++l) {
            const Level v = make_level(n, l);
            if (l + 1 == L) {
                // the last level: single-node subtrees, position p is subtree p
                if (v.W != 1 || v.R != n - full_nodes(L - 1)) return fail("last level", n, l, 0, v.W, 1);
                for (uint32_t p : {0u, v.R > 0 ? v.R - 1 : 0u})
                    if (seg_of_pos(v, p) != p) return fail("seg_of_pos last level", n, l, p, seg_of_pos(v, p), p);
                if (seg_size(v, 0) != 1) return fail("seg_size last level", n, l, 0, seg_size(v, 0), 1);
            }
            if (l >= L && v.W != 0) return fail("below the tree", n, l, 0, v.W, 0);
            (void)seg_of_pos(v, 0);
            (void)tiles_level(v, 4096);
            (void)seg_offset(v, v.nseg ? v.nseg - 1 : 0);
            (void)seg_left_size(v, 0);
        }
    }
    // clamp_sub at the wrap edges
    if (clamp_sub(5, 7, 3) != 0 || clamp_sub(7, 5, 3) != 2 || clamp_sub(0xFFFFFFFFu, 0, 9) != 9 ||
        clamp_sub(0, 0xFFFFFFFFu, 9) != 0)
        return fail("clamp_sub", 0, 0, 0, clamp_sub(5, 7, 3), 0);
    return 0;
}

int main()
{
    if (check_edges()) return 1;
    for (uint32_t n = 1; n <= 3000; ++n)
        if (check_n(n, true)) return 1;
    const uint32_t big[] = {4095, 4096, 4097, 65535, 65536, 65537, 100003, 1000000, 1048575, 1048576, 3333333};
    for (uint32_t n : big)
        if (check_n(n, false)) return 1;
    std::printf("ok\n");
    return 0;
}
