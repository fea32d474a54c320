/*
 * kdt_oracle.c -- CPU oracle for the left-balanced k-d tree build.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * library never does, and the two share no code (no headers, no helpers, no
 * tables).
 *
 * What it computes (Wald, "GPU-friendly, Parallel, and (Almost-)In-Place
 * Construction of Left-Balanced k-d Trees", arXiv 2211.00120):
 *
 *  - The tree is stored in level order: node s has children 2s+1 and 2s+2
 *    (Sec. 2).  It is left-balanced and complete, so the number of nodes in
 *    the subtree under s depends only on s and N (Sec. 2.1).  Here that size
 *    is obtained by directly counting the subtree's nodes level by level, NOT
 *    by the O(1) closed form of Sec. 4 (the GPU path uses the closed form; the
 *    oracle must not).
 *
 *  - Build is the "usual" recursive list build the introduction describes:
 *    sort the subtree's points along its split dimension, split at the
 *    balance position, recurse.  The balance position is the size of the left
 *    child's subtree (Observation 2.1): the point at that position of the
 *    sorted list becomes node s, lower positions form the left subtree, higher
 *    positions the right subtree.
 *
 *  - Sort order along dimension d is the total order
 *        i < j  <=>  P[i][d] < P[j][d]  or  (P[i][d] == P[j][d] and i < j)
 *    i.e. coordinate first, original index as tie-break.  The paper's less()
 *    (Sec. 3.1) has no tie-break; the original index is the reading adopted
 *    here, which makes the tree unique.  Comparison is IEEE float compare, so
 *    -0 == +0.
 *
 *  - Split dimension: round robin uses level(s) mod k (Sec. 2).  Split-widest
 *    (Sec. 6) uses the subtree's domain: the scene bounding box clipped by
 *    every ancestor's split plane (left child: hi[d] = plane, right child:
 *    lo[d] = plane), and picks the dimension with the largest extent
 *    hi[d]-lo[d] computed in float32; ties go to the lowest dimension.
 *    Every node gets a dimension, leaves included.
 *
 * Outputs: perm[s] = original index of the point stored at node s, and
 * dim[s] = split dimension of node s.  The tree's points are P[perm[s]].
 *
 * The checker (kdt_oracle_check) verifies a candidate (perm, dim) without
 * building: perm must be a permutation of [0,N); every node must be ordered
 * against each ancestor on the correct side in that ancestor's dimension
 * (the k-d condition of Sec. 1 under the total order above); and every dim
 * must match the rule above.  Because the left subtree of the root has a
 * fixed size, the root is the unique point with exactly that many
 * predecessors in the root's order, and by induction the whole tree is
 * unique; so passing the checker is equivalent to equality with
 * kdt_oracle_build.
 *
 * Pins: see tests/test_oracle_pins.py (paper walkthrough of Sec. 5, the
 * 6-point set of Fig. 1, special cases with textbook answers, brute force on
 * small inputs, cross-check against an independent model of the paper's
 * tag/sort loop).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_RR = 0, ORACLE_WIDEST = 1 };

/* ---------------------------------------------------------------- helpers */

/* Depth of node s in level order: floor(log2(s+1)), by repeated halving. */
static uint32_t node_level(uint64_t s)
{
    uint32_t l = 0;
    uint64_t v = s + 1;
    while (v > 1) { v >>= 1; l++; }
    return l;
}

/* Number of nodes of the subtree rooted at s in a level-order tree of N
 * nodes, by direct count: at depth m below s the subtree occupies the index
 * range [(s+1)*2^m - 1, (s+2)*2^m - 1); count how much of each such range is
 * below N. */
static uint64_t subtree_size(uint64_t s, uint64_t N)
{
    uint64_t lo = s, hi = s + 1, total = 0;
    while (lo < N) {
        total += (hi < N ? hi : N) - lo;
        lo = 2 * lo + 1;
        hi = 2 * hi + 1;
    }
    return total;
}

typedef struct { float v; uint32_t i; } item_t;

/* (coordinate, original index) total order; IEEE compare so -0 == +0. */
static int item_cmp(const void* a, const void* b)
{
    const item_t* x = (const item_t*)a;
    const item_t* y = (const item_t*)b;
    if (x->v < y->v) return -1;
    if (y->v < x->v) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

/* Dimension of largest float32 extent hi[d]-lo[d]; lowest d wins ties. */
static uint32_t widest_dim(const float* lo, const float* hi, uint32_t k)
{
    uint32_t best = 0;
    float best_e = hi[0] - lo[0];
    for (uint32_t d = 1; d < k; d++) {
        float e = hi[d] - lo[d];
        if (e > best_e) { best_e = e; best = d; }
    }
    return best;
}

static void scene_box(const float* P, uint64_t N, uint32_t k, float* lo, float* hi)
{
    for (uint32_t d = 0; d < k; d++) { lo[d] = P[d]; hi[d] = P[d]; }
    for (uint64_t i = 1; i < N; i++)
        for (uint32_t d = 0; d < k; d++) {
            float v = P[i * k + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
}

/* ------------------------------------------------------------------ build */

typedef struct {
    const float* P;
    uint64_t N;
    uint32_t k;
    int mode;
    uint32_t* perm;
    uint8_t* dim;
    item_t* scratch;   /* N items, reused by every call on its own range */
} build_ctx;

/* idx[0..n) holds the original indices of the points of subtree s. */
static void build(build_ctx* c, uint64_t s, uint32_t* idx, uint64_t n,
                  const float* lo, const float* hi)
{
    if (n == 0) return;
    const uint32_t k = c->k;
    uint32_t d = (c->mode == ORACLE_RR) ? node_level(s) % k : widest_dim(lo, hi, k);

    /* sort the subtree's points along d (Observation 2.1) */
    item_t* it = c->scratch;   /* ranges of sibling calls never overlap in time */
    for (uint64_t j = 0; j < n; j++) { it[j].v = c->P[(uint64_t)idx[j] * k + d]; it[j].i = idx[j]; }
    qsort(it, n, sizeof(item_t), item_cmp);
    for (uint64_t j = 0; j < n; j++) idx[j] = it[j].i;

    /* pivot position = size of the left child's subtree */
    uint64_t m = subtree_size(2 * s + 1, c->N);
    uint32_t p = idx[m];
    c->perm[s] = p;
    c->dim[s] = (uint8_t)d;
    float plane = c->P[(uint64_t)p * k + d];

    float lo2[4], hi2[4];
    memcpy(lo2, lo, k * sizeof(float));
    memcpy(hi2, hi, k * sizeof(float));
    hi2[d] = plane;                                   /* left child's domain */
    build(c, 2 * s + 1, idx, m, lo, hi2);
    lo2[d] = plane;                                   /* right child's domain */
    build(c, 2 * s + 2, idx + m + 1, n - m - 1, lo2, hi);
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 * points: N*k float32, row-major (point-major).  perm: N uint32.  dim: N u8.
 * k in [1,4]. */
int kdt_oracle_build(const float* points, uint64_t N, uint32_t k, int mode,
                     uint32_t* perm, uint8_t* dim)
{
    if (k < 1 || k > 4 || (mode != ORACLE_RR && mode != ORACLE_WIDEST)) return -1;
    if (N == 0) return 0;
    if (!points || !perm || !dim) return -1;
    uint32_t* idx = (uint32_t*)malloc(N * sizeof(uint32_t));
    item_t* scratch = (item_t*)malloc(N * sizeof(item_t));
    if (!idx || !scratch) { free(idx); free(scratch); return -2; }
    for (uint64_t i = 0; i < N; i++) idx[i] = (uint32_t)i;
    float lo[4], hi[4];
    scene_box(points, N, k, lo, hi);
    build_ctx c = { points, N, k, mode, perm, dim, scratch };
    build(&c, 0, idx, N, lo, hi);
    free(idx);
    free(scratch);
    return 0;
}

/* ---------------------------------------------------------------- checker */

/* Is point a before point b in the total order along d? */
static int before(const float* P, uint32_t k, uint32_t d, uint32_t a, uint32_t b)
{
    float x = P[(uint64_t)a * k + d], y = P[(uint64_t)b * k + d];
    if (x < y) return 1;
    if (y < x) return 0;
    return a < b;
}

/* Returns 0 if (perm, dim) is the tree of `points`, otherwise a positive code
 * naming the first failed property:
 *   1 perm is not a permutation of [0,N)
 *   2 k-d order violated between a node and one of its ancestors
 *   3 a node's dim differs from the split rule
 *  -1 bad arguments, -2 allocation failure.
 * *bad_node (nullable) receives the offending node index. */
int kdt_oracle_check(const float* points, uint64_t N, uint32_t k, int mode,
                     const uint32_t* perm, const uint8_t* dim, uint64_t* bad_node)
{
    if (k < 1 || k > 4 || (mode != ORACLE_RR && mode != ORACLE_WIDEST)) return -1;
    if (N == 0) return 0;
    if (!points || !perm || !dim) return -1;
    uint8_t* seen = (uint8_t*)calloc(N, 1);
    if (!seen) return -2;
    for (uint64_t s = 0; s < N; s++) {
        if (perm[s] >= N || seen[perm[s]]) {
            free(seen);
            if (bad_node) *bad_node = s;
            return 1;
        }
        seen[perm[s]] = 1;
    }
    free(seen);

    float slo[4], shi[4];
    scene_box(points, N, k, slo, shi);
    for (uint64_t s = 0; s < N; s++) {
        /* k-d order against every ancestor */
        uint64_t c = s;
        while (c > 0) {
            uint64_t a = (c - 1) / 2;
            int left = (c == 2 * a + 1);
            uint32_t da = dim[a];
            if (da >= k) { if (bad_node) *bad_node = a; return 3; }
            int ok = left ? before(points, k, da, perm[s], perm[a])
                          : before(points, k, da, perm[a], perm[s]);
            if (!ok) { if (bad_node) *bad_node = s; return 2; }
            c = a;
        }
        /* split dimension rule */
        uint32_t want;
        if (mode == ORACLE_RR) {
            want = node_level(s) % k;
        } else {
            float lo[4], hi[4];
            memcpy(lo, slo, sizeof lo);
            memcpy(hi, shi, sizeof hi);
            c = s;
            while (c > 0) {   /* clip by each ancestor's plane (intersection) */
                uint64_t a = (c - 1) / 2;
                uint32_t da = dim[a];
                float plane = points[(uint64_t)perm[a] * k + da];
                if (c == 2 * a + 1) { if (plane < hi[da]) hi[da] = plane; }
                else                { if (plane > lo[da]) lo[da] = plane; }
                c = a;
            }
            want = widest_dim(lo, hi, k);
        }
        if (dim[s] != want) { if (bad_node) *bad_node = s; return 3; }
    }
    return 0;
}

/* Exposed for the oracle's own pins (direct-count subtree size). */
uint64_t kdt_oracle_subtree_size(uint64_t s, uint64_t N) { return subtree_size(s, N); }
