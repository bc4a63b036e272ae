/* Exercises the host side of the library (include/msg.h) without a GPU,
 * built with the library's host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py): the layout, the
 * solve planner behind msg_workspace_size over uniform and ragged batches
 * and every plan option, the planners of the plain cycles and of the Matern
 * fields, argument checking, and handle creation where no device is
 * present.  Any out-of-bounds access or undefined operation aborts the run.
 * Prints "host driver ok" at the end. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "msg.h"

static int failures = 0;
#define EXPECT(cond, what)                                                     \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "FAILED: %s (%s)\n", what, msg_last_error());      \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static uint64_t rng_state = 0x2545F4914F6CDD1Dull;
static uint32_t draw(uint32_t n)
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 2685821657736338717ull) >> 33) % n;
}

static void plan_batch(int c, int S, const int32_t *P, const int32_t *Q)
{
    const msg_batch_desc b = {S, c, P, Q};
    int64_t *cell = malloc(sizeof(int64_t) * (S + 1)), *xf = malloc(sizeof(int64_t) * (S + 1));
    int64_t *yf = malloc(sizeof(int64_t) * (S + 1)), *grid = malloc(sizeof(int64_t) * (S + 1));
    EXPECT(msg_layout(&b, cell, xf, yf, grid) == MSG_OK, "layout");
    EXPECT(msg_layout(&b, NULL, NULL, NULL, grid) == MSG_OK, "layout with null outputs");
    free(cell); free(xf); free(yf); free(grid);

    msg_solve_opts o;
    msg_default_opts(&o);
    size_t bytes = 0;
    EXPECT(msg_workspace_size(NULL, &b, &o, &bytes) == MSG_OK && bytes > 0, "workspace default");
    static const int32_t budgets[] = {0, 1024, 8192, 20480, 40960, 65536, 153600};
    for (int prec = 0; prec < 2; ++prec)
        for (int ov = -1; ov <= 2; ++ov)
            for (size_t t = 0; t < sizeof budgets / sizeof budgets[0]; ++t) {
                msg_default_opts(&o);
                o.precision = prec;
                o.overlap = ov;
                o.tail_budget = budgets[t];
                o.tile_width = (int32_t)(4 << draw(7));
                o.tile_cells = (int32_t)(64 << draw(7));
                o.tile_lds = (int32_t)(256 << draw(6));
                o.graphs = (int32_t)draw(2);
                o.handoff = (int32_t)draw(5) - 1;
                o.tail_levels = (int32_t)draw(10) - 1;
                const msg_status st = msg_workspace_size(NULL, &b, &o, &bytes);
                EXPECT(st == MSG_OK || st == MSG_ERR_UNSUPPORTED || st == MSG_ERR_ARG, "workspace options");
            }
    for (int kind = 0; kind < 2; ++kind) {
        msg_default_opts(&o);
        const msg_status st = msg_cycles_workspace_size(NULL, &b, &o, kind, &bytes);
        EXPECT(st == MSG_OK || st == MSG_ERR_UNSUPPORTED, "cycles workspace");
    }
    double *eta = malloc(sizeof(double) * S), *theta = malloc(sizeof(double) * S);
    for (int s = 0; s < S; ++s) {
        eta[s] = 0.0625 + 0.01 * s;
        theta[s] = 0.1 * s;
    }
    const msg_matern_spec m = {0.25, 0.5, eta, theta, NULL, 7, 0, 0};
    const msg_status st = msg_matern_workspace_size(&b, &m, &bytes);
    EXPECT(st == MSG_OK || st == MSG_ERR_UNSUPPORTED, "matern workspace");
    free(eta); free(theta);
}

int main(void)
{
    /* uniform batches at the corners of the supported range */
    static const int shapes[][4] = {{1, 1, 0, 0}, {2, 16, 7, 7}, {4, 8, 8, 4}, {4, 3, 3, 3}, {8, 2, 0, 9},
                                    {2, 1, 14, 0}, {4, 5, 9, 9}, {1, 7, 5, 2}};
    for (size_t k = 0; k < sizeof shapes / sizeof shapes[0]; ++k) {
        const int c = shapes[k][0], S = shapes[k][1];
        int32_t *P = malloc(sizeof(int32_t) * S), *Q = malloc(sizeof(int32_t) * S);
        for (int s = 0; s < S; ++s) {
            P[s] = shapes[k][2];
            Q[s] = shapes[k][3];
        }
        plan_batch(c, S, P, Q);
        free(P); free(Q);
    }
    /* ragged batches: every rectangle with l1 + l2 <= 8, and random mixes */
    {
        int32_t P[45], Q[45];
        int S = 0;
        for (int a = 0; a <= 8; ++a)
            for (int b = 0; a + b <= 8; ++b) {
                P[S] = a;
                Q[S] = b;
                ++S;
            }
        plan_batch(4, S, P, Q);
    }
    for (int trial = 0; trial < 20; ++trial) {
        const int S = 1 + (int)draw(300), c = 1 + (int)draw(8);
        int32_t *P = malloc(sizeof(int32_t) * S), *Q = malloc(sizeof(int32_t) * S);
        for (int s = 0; s < S; ++s) {
            P[s] = (int32_t)draw(8);
            Q[s] = (int32_t)draw(8);
        }
        plan_batch(c, S, P, Q);
        free(P); free(Q);
    }

    /* argument checking */
    int32_t P1 = 3, Q1 = 3, bad = 15;
    const msg_batch_desc ok = {1, 4, &P1, &Q1}, empty = {0, 4, &P1, &Q1}, big = {1, 4, &bad, &Q1};
    const msg_batch_desc badc = {1, 9, &P1, &Q1}, nullp = {1, 4, NULL, &Q1};
    size_t bytes;
    msg_solve_opts o;
    msg_default_opts(&o);
    EXPECT(msg_layout(&empty, NULL, NULL, NULL, NULL) != MSG_OK, "empty batch rejected");
    EXPECT(msg_layout(&big, NULL, NULL, NULL, NULL) != MSG_OK, "index 15 rejected");
    EXPECT(msg_layout(&badc, NULL, NULL, NULL, NULL) != MSG_OK, "c = 9 rejected");
    EXPECT(msg_layout(&nullp, NULL, NULL, NULL, NULL) != MSG_OK, "null P rejected");
    EXPECT(msg_workspace_size(NULL, &ok, NULL, &bytes) != MSG_OK, "null options rejected");
    o.mu = 0;
    EXPECT(msg_workspace_size(NULL, &ok, &o, &bytes) != MSG_OK, "mu = 0 rejected");
    msg_default_opts(&o);
    o.tail_budget = 160000;
    EXPECT(msg_workspace_size(NULL, &ok, &o, &bytes) != MSG_OK, "tail budget above the LDS rejected");
    EXPECT(msg_solve_batch(NULL, &ok, &o, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL) != MSG_OK,
           "null handle rejected");
    const msg_field_spec f = {0};
    EXPECT(msg_sample_field(NULL, &f, &ok, NULL, NULL, NULL, NULL, NULL, NULL) != MSG_OK, "null handle (field)");
    EXPECT(msg_sample_field_noalloc(NULL, &f, &ok, NULL, NULL, NULL, NULL, NULL, NULL) != MSG_OK,
           "null handle (field, no allocation)");

    /* a handle on a host without a device reports the HIP error */
    msg_handle h = NULL;
    const msg_status st = msg_create(&h, 0);
    if (st == MSG_OK)
        msg_destroy(h);
    else
        EXPECT(st == MSG_ERR_HIP && msg_last_error() != NULL, "create without a device");
    EXPECT(msg_create(&h, -1) != MSG_OK, "negative device rejected");

    if (failures) return 1;
    printf("host driver ok\n");
    return 0;
}
