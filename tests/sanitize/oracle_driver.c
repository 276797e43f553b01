/* Sanitizer driver for the oracle (oracle/oracle.c): walks of several
 * formats with every step enabled (flips, reductions, expands, restarts, the
 * additions objective, Z2), the meta operators, Resize and lifting.  Built
 * with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitize.py; exits 0 when every emitted scheme passes the Brent
 * equations (sanitizer findings abort the program). */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/oracle.h"

static int failures = 0;
#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond);    \
            ++failures;                                                               \
        }                                                                             \
    } while (0)

static void walk_format(int m, int n, int p, int z2, int objective)
{
    or_scheme *start = malloc(sizeof *start);
    or_walk *w = malloc(sizeof *w);
    or_standard(start, m, n, p, z2);
    or_walk_init(w, start);
    or_params prm = {0};
    prm.seed = 1234u + (uint64_t)(m * 100 + n * 10 + p);
    prm.max_iters = 3000;
    prm.plateau = 700;
    prm.target_rank = 0;
    prm.r_cap = m * n * p + 6;
    prm.flip_tries = 3;
    prm.restart_from_best = (m + n + p) & 1;
    prm.t_eq = 42949673u;
    prm.t_reduce = (3ull << 30);
    prm.t_expand = objective ? 0 : (1ull << 29);
    prm.objective = objective;
    or_walk_run(w, &prm, 1500);
    or_walk_run(w, &prm, 1500);
    CHECK(or_brent_violations(&w->cur) == 0);
    CHECK(or_brent_violations(&w->best) == 0);
    CHECK(w->t == 3000);
    free(start);
    free(w);
}

int main(void)
{
    const int fmts[][3] = {{2, 2, 2}, {2, 2, 3}, {2, 3, 3}, {3, 3, 3}, {3, 4, 5}, {4, 5, 12}};
    for (int q = 0; q < 6; ++q)
        for (int z2 = 0; z2 < 2; ++z2) walk_format(fmts[q][0], fmts[q][1], fmts[q][2], z2, 0);
    walk_format(3, 3, 3, 0, 1);
    walk_format(2, 3, 3, 1, 1);

    or_scheme *a = malloc(sizeof *a), *b = malloc(sizeof *b), *c = malloc(sizeof *c);
    or_standard(a, 2, 3, 4, 0);
    for (int axis = 0; axis < 3; ++axis) {
        CHECK(or_project(a, axis, 1, b) >= 0);
        CHECK(or_brent_violations(b) == 0);
        CHECK(or_extend(b, axis, c) >= 0);
        CHECK(or_brent_violations(c) == 0);
    }
    CHECK(or_swap_sizes(a, b) >= 0);
    CHECK(or_brent_violations(b) == 0);
    or_standard(b, 2, 3, 1, 0);
    CHECK(or_merge(a, b, 2, c) >= 0);
    CHECK(or_brent_violations(c) == 0);
    or_standard(b, 1, 1, 2, 0);
    CHECK(or_product(a, b, c) >= 0);
    CHECK(or_brent_violations(c) == 0);
    or_full_reduce(c);
    CHECK(or_brent_violations(c) == 0);

    /* Resize of a scheme against a table of two best schemes, many rounds */
    or_scheme *best = malloc(2 * sizeof *best);
    or_standard(&best[0], 2, 2, 2, 0);
    or_standard(&best[1], 2, 3, 4, 0);
    for (int round = 0; round < 40; ++round) {
        or_standard(a, 2, 2, 3, 0);
        or_resize(a, best, 2, 99u, round, 1ull << 32, 200, b);
        CHECK(or_brent_violations(b) == 0);
    }

    /* lifting of the standard (2,2,2) scheme read over Z2 */
    or_scheme *z = malloc(sizeof *z);
    or_standard(z, 2, 2, 2, 1);
    int64_t nodes = 0;
    CHECK(or_lift(z, 100000, c, &nodes) == 1);
    CHECK(or_brent_violations(c) == 0);

    free(a); free(b); free(c); free(best); free(z);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
