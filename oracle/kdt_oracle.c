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
 *  - Build is the conventional recursive list build the introduction describes:
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
 * Coordinate types: float32 (the paper's float3/float4 points) and int32
 * (Table 1's int1 rows; Sec. 7.2 templates the builder over the point type).
 * Every coordinate is read into a double, which holds every float32 and every
 * int32 value exactly, so all comparisons are those of the input type.  The
 * split-widest extent of a float32 box is the float32 subtraction of its two
 * (exact) bounds; that of an int32 box is the exact difference hi - lo (the
 * paper does not say how an integer extent is formed; this is the reading
 * adopted here: an int32 subtraction could overflow).
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
enum { ORACLE_F32 = 0, ORACLE_I32 = 1 };

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

/* The points: N*k coordinates of one type, row-major. */
typedef struct {
    const void* P;
    int type;          /* ORACLE_F32 or ORACLE_I32 */
    uint64_t N;
    uint32_t k;
} pts_t;

/* Coordinate d of point i, exactly. */
static double coord(const pts_t* p, uint64_t i, uint32_t d)
{
    if (p->type == ORACLE_I32) return (double)((const int32_t*)p->P)[i * p->k + d];
    return (double)((const float*)p->P)[i * p->k + d];
}

typedef struct { double v; uint32_t i; } item_t;

/* (coordinate, original index) total order; IEEE compare so -0 == +0. */
static int item_cmp(const void* a, const void* b)
{
    const item_t* x = (const item_t*)a;
    const item_t* y = (const item_t*)b;
    if (x->v < y->v) return -1;
    if (y->v < x->v) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

/* Dimension of largest extent hi[d]-lo[d] (float32: computed in float32;
 * int32: exact); lowest d wins ties. */
static uint32_t widest_dim(int type, const double* lo, const double* hi, uint32_t k)
{
    uint32_t best = 0;
    if (type == ORACLE_F32) {
        float best_e = (float)hi[0] - (float)lo[0];
        for (uint32_t d = 1; d < k; d++) {
            float e = (float)hi[d] - (float)lo[d];
            if (e > best_e) { best_e = e; best = d; }
        }
    } else {
        double best_e = hi[0] - lo[0];
        for (uint32_t d = 1; d < k; d++) {
            double e = hi[d] - lo[d];
            if (e > best_e) { best_e = e; best = d; }
        }
    }
    return best;
}

static void scene_box(const pts_t* p, double* lo, double* hi)
{
    for (uint32_t d = 0; d < p->k; d++) { lo[d] = coord(p, 0, d); hi[d] = lo[d]; }
    for (uint64_t i = 1; i < p->N; i++)
        for (uint32_t d = 0; d < p->k; d++) {
            double v = coord(p, i, d);
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
}

/* ------------------------------------------------------------------ build */

typedef struct {
    pts_t pts;
    int mode;
    uint32_t* perm;
    uint8_t* dim;
    uint32_t* idx0;    /* the index array every call's idx points into */
    item_t* scratch;   /* N items: a call on idx[0..n) uses the same range of scratch */
    uint64_t task_min; /* parallel build: subtrees of at least this many points
                          run their two child calls as separate tasks (0: never) */
} build_ctx;

/* idx[0..n) holds the original indices of the points of subtree s. */
static void build(build_ctx* c, uint64_t s, uint32_t* idx, uint64_t n,
                  const double* lo, const double* hi)
{
    if (n == 0) return;
    const uint32_t k = c->pts.k;
    uint32_t d = (c->mode == ORACLE_RR) ? node_level(s) % k : widest_dim(c->pts.type, lo, hi, k);

    /* sort the subtree's points along d (Observation 2.1); the scratch range
       is this call's own (the ranges of two subtrees never overlap) */
    item_t* it = c->scratch + (idx - c->idx0);
    for (uint64_t j = 0; j < n; j++) { it[j].v = coord(&c->pts, idx[j], d); it[j].i = idx[j]; }
    qsort(it, n, sizeof(item_t), item_cmp);
    for (uint64_t j = 0; j < n; j++) idx[j] = it[j].i;

    /* pivot position = size of the left child's subtree */
    uint64_t m = subtree_size(2 * s + 1, c->pts.N);
    uint32_t p = idx[m];
    c->perm[s] = p;
    c->dim[s] = (uint8_t)d;
    double plane = coord(&c->pts, p, d);

    double lo2[4], hi2[4];
    memcpy(lo2, lo, k * sizeof(double));
    memcpy(hi2, hi, k * sizeof(double));
    hi2[d] = plane;                                   /* left child's domain */
    lo2[d] = plane;                                   /* right child's domain */
    if (c->task_min && n >= c->task_min) {
        /* the two subtrees touch disjoint ranges of idx, scratch, perm and
           dim, so they can run at the same time (same results) */
#pragma omp task default(shared) firstprivate(hi2)
        build(c, 2 * s + 1, idx, m, lo, hi2);
#pragma omp task default(shared) firstprivate(lo2)
        build(c, 2 * s + 2, idx + m + 1, n - m - 1, lo2, hi);
#pragma omp taskwait
    } else {
        build(c, 2 * s + 1, idx, m, lo, hi2);
        build(c, 2 * s + 2, idx + m + 1, n - m - 1, lo2, hi);
    }
}

static int build_any(const void* points, int type, uint64_t N, uint32_t k, int mode,
                     uint32_t* perm, uint8_t* dim, int threads)
{
    if (k < 1 || k > 4 || (mode != ORACLE_RR && mode != ORACLE_WIDEST)) return -1;
    if (N == 0) return 0;
    if (!points || !perm || !dim) return -1;
    uint32_t* idx = (uint32_t*)malloc(N * sizeof(uint32_t));
    item_t* scratch = (item_t*)malloc(N * sizeof(item_t));
    if (!idx || !scratch) { free(idx); free(scratch); return -2; }
    for (uint64_t i = 0; i < N; i++) idx[i] = (uint32_t)i;
    build_ctx c = { { points, type, N, k }, mode, perm, dim, idx, scratch, 0 };
    double lo[4], hi[4];
    scene_box(&c.pts, lo, hi);
    if (threads > 1) {
        c.task_min = 1u << 14;
#pragma omp parallel num_threads(threads)
#pragma omp single
        build(&c, 0, idx, N, lo, hi);
    } else {
        build(&c, 0, idx, N, lo, hi);
    }
    free(idx);
    free(scratch);
    return 0;
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 * points: N*k float32, row-major (point-major).  perm: N uint32.  dim: N u8.
 * k in [1,4]. */
int kdt_oracle_build(const float* points, uint64_t N, uint32_t k, int mode,
                     uint32_t* perm, uint8_t* dim)
{
    return build_any(points, ORACLE_F32, N, k, mode, perm, dim, 1);
}

/* The same recursion with the two child calls of every subtree of at least
 * 2^14 points run as OpenMP tasks on `threads` threads; the output is the
 * same as kdt_oracle_build's (every call writes only its own subtree's
 * entries).  Used to time the CPU on all host cores. */
int kdt_oracle_build_par(const float* points, uint64_t N, uint32_t k, int mode,
                         uint32_t* perm, uint8_t* dim, int threads)
{
    return build_any(points, ORACLE_F32, N, k, mode, perm, dim, threads < 1 ? 1 : threads);
}

/* kdt_oracle_build and kdt_oracle_build_par for int32 coordinates. */
int kdt_oracle_build_i32(const int32_t* points, uint64_t N, uint32_t k, int mode,
                         uint32_t* perm, uint8_t* dim)
{
    return build_any(points, ORACLE_I32, N, k, mode, perm, dim, 1);
}

int kdt_oracle_build_par_i32(const int32_t* points, uint64_t N, uint32_t k, int mode,
                             uint32_t* perm, uint8_t* dim, int threads)
{
    return build_any(points, ORACLE_I32, N, k, mode, perm, dim, threads < 1 ? 1 : threads);
}

/* ---------------------------------------------------------------- checker */

/* Is point a before point b in the total order along d? */
static int before(const pts_t* p, uint32_t d, uint32_t a, uint32_t b)
{
    double x = coord(p, a, d), y = coord(p, b, d);
    if (x < y) return 1;
    if (y < x) return 0;
    return a < b;
}

/* The checks of one node s: k-d order against every ancestor, then the split
 * rule.  Returns 0, 2 or 3 as kdt_oracle_check does; *at receives the node
 * the failure names. */
static int check_node(const pts_t* p, int mode, const uint32_t* perm, const uint8_t* dim,
                      const double* slo, const double* shi, uint64_t s, uint64_t* at)
{
    const uint32_t k = p->k;
    /* k-d order against every ancestor */
    uint64_t c = s;
    while (c > 0) {
        uint64_t a = (c - 1) / 2;
        int left = (c == 2 * a + 1);
        uint32_t da = dim[a];
        if (da >= k) { *at = a; return 3; }
        int ok = left ? before(p, da, perm[s], perm[a]) : before(p, da, perm[a], perm[s]);
        if (!ok) { *at = s; return 2; }
        c = a;
    }
    /* split dimension rule */
    uint32_t want;
    if (mode == ORACLE_RR) {
        want = node_level(s) % k;
    } else {
        double lo[4], hi[4];
        memcpy(lo, slo, sizeof lo);
        memcpy(hi, shi, sizeof hi);
        c = s;
        while (c > 0) {   /* clip by each ancestor's plane (intersection) */
            uint64_t a = (c - 1) / 2;
            uint32_t da = dim[a];
            double plane = coord(p, perm[a], da);
            if (c == 2 * a + 1) { if (plane < hi[da]) hi[da] = plane; }
            else                { if (plane > lo[da]) lo[da] = plane; }
            c = a;
        }
        want = widest_dim(p->type, lo, hi, k);
    }
    if (dim[s] != want) { *at = s; return 3; }
    return 0;
}

static int check_any(const void* points, int type, uint64_t N, uint32_t k, int mode,
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

    const pts_t p = { points, type, N, k };
    double slo[4], shi[4];
    scene_box(&p, slo, shi);
    /* nodes are independent: check them in parallel, and report the first
       failing node in index order (what a sequential loop would report) */
    uint64_t first = N;
    int code = 0;
#pragma omp parallel for schedule(dynamic, 65536) if (N >= (1u << 20))
    for (uint64_t s = 0; s < N; s++) {
        uint64_t at = s;
        int r = check_node(&p, mode, perm, dim, slo, shi, s, &at);
        if (r) {
#pragma omp critical
            if (s < first) { first = s; code = r; if (bad_node) *bad_node = at; }
        }
    }
    return code;
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
    return check_any(points, ORACLE_F32, N, k, mode, perm, dim, bad_node);
}

/* kdt_oracle_check for int32 coordinates. */
int kdt_oracle_check_i32(const int32_t* points, uint64_t N, uint32_t k, int mode,
                         const uint32_t* perm, const uint8_t* dim, uint64_t* bad_node)
{
    return check_any(points, ORACLE_I32, N, k, mode, perm, dim, bad_node);
}

/* Exposed for the oracle's own pins (direct-count subtree size). */
uint64_t kdt_oracle_subtree_size(uint64_t s, uint64_t N) { return subtree_size(s, N); }
