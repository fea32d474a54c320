/* Drives the CPU oracle (oracle/kdt_oracle.c) on random tie-heavy inputs of
 * both coordinate types, both split rules and k = 1..4, for the sanitizer
 * build of the tests: every build must pass the oracle's own checker, the
 * parallel build must equal the sequential one, a planted swap of two nodes
 * must be rejected, and the edges N = 0, 1, 2 must work.  Prints "ok". */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int kdt_oracle_build(const float*, uint64_t, uint32_t, int, uint32_t*, uint8_t*);
int kdt_oracle_build_par(const float*, uint64_t, uint32_t, int, uint32_t*, uint8_t*, int);
int kdt_oracle_build_i32(const int32_t*, uint64_t, uint32_t, int, uint32_t*, uint8_t*);
int kdt_oracle_build_par_i32(const int32_t*, uint64_t, uint32_t, int, uint32_t*, uint8_t*, int);
int kdt_oracle_check(const float*, uint64_t, uint32_t, int, const uint32_t*, const uint8_t*, uint64_t*);
int kdt_oracle_check_i32(const int32_t*, uint64_t, uint32_t, int, const uint32_t*, const uint8_t*, uint64_t*);

static uint64_t rng = 88172645463325252ull;
static uint32_t next(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)(rng >> 16);
}

static int one(uint64_t n, uint32_t k, int mode, int type)
{
    void* pts = malloc((n ? n : 1) * k * 4);
    uint32_t* perm = malloc((n ? n : 1) * 4);
    uint32_t* perm2 = malloc((n ? n : 1) * 4);
    uint8_t* dim = malloc(n ? n : 1);
    uint8_t* dim2 = malloc(n ? n : 1);
    const uint32_t levels = 1 + next() % 9;   /* few distinct values: ties */
    for (uint64_t i = 0; i < n * k; i++) {
        int32_t v = (int32_t)(next() % levels) - 3;
        /* int32: now and then a value anywhere in the 32-bit range */
        if (type) ((int32_t*)pts)[i] = (next() % 7 == 0) ? (int32_t)(next() ^ (next() << 16)) : v;
        else ((float*)pts)[i] = (next() % 11 == 0) ? -0.0f : (float)v * 0.25f;
    }
    int rc = type ? kdt_oracle_build_i32(pts, n, k, mode, perm, dim) : kdt_oracle_build(pts, n, k, mode, perm, dim);
    int rc2 = type ? kdt_oracle_build_par_i32(pts, n, k, mode, perm2, dim2, 4)
                   : kdt_oracle_build_par(pts, n, k, mode, perm2, dim2, 4);
    uint64_t bad = 0;
    int ok = rc == 0 && rc2 == 0;
    if (ok && n) ok = memcmp(perm, perm2, n * 4) == 0 && memcmp(dim, dim2, n) == 0;
    if (ok) ok = (type ? kdt_oracle_check_i32(pts, n, k, mode, perm, dim, &bad)
                       : kdt_oracle_check(pts, n, k, mode, perm, dim, &bad)) == 0;
    if (ok && n >= 2) {
        /* the tree is unique under the (coordinate, index) order, so any
           other permutation -- here the root swapped with the last node --
           must be rejected */
        uint32_t t = perm[0];
        perm[0] = perm[n - 1];
        perm[n - 1] = t;
        int c = type ? kdt_oracle_check_i32(pts, n, k, mode, perm, dim, &bad)
                     : kdt_oracle_check(pts, n, k, mode, perm, dim, &bad);
        ok = c != 0;
    }
    if (!ok) printf("FAIL n=%llu k=%u mode=%d type=%d rc=%d/%d\n", (unsigned long long)n, k, mode, type, rc, rc2);
    free(pts);
    free(perm);
    free(perm2);
    free(dim);
    free(dim2);
    return !ok;
}

int main(void)
{
    for (int type = 0; type < 2; type++)
        for (int mode = 0; mode < 2; mode++)
            for (uint32_t k = 1; k <= 4; k++) {
                for (uint64_t n = 0; n <= 40; n++)
                    if (one(n, k, mode, type)) return 1;
                for (int r = 0; r < 6; r++)
                    if (one(41 + next() % 3000, k, mode, type)) return 1;
                if (one(40000, k, mode, type)) return 1;   /* parallel subtrees */
            }
    printf("ok\n");
    return 0;
}
