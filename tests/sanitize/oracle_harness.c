/*
 * AddressSanitizer / UBSan harness for the oracle (oracle/vor_oracle.c), built and run by
 * tests/test_sanitizers.py: small sets in a box and in a convex polygon, sites on the boundary
 * of X, the entry bound of Euler's formula, the capacity answer, and every input error path.
 * Test infrastructure: it links the oracle only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int vor_oracle_validate(int32_t n, const int32_t *x, const int32_t *y, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1);
int vor_oracle_validate_poly(int32_t n, const int32_t *x, const int32_t *y, int32_t K,
                             const int32_t *vx, const int32_t *vy);
int64_t vor_oracle_cells(int32_t n, const int32_t *x, const int32_t *y, int32_t x0, int32_t y0,
                         int32_t x1, int32_t y1, int32_t m, const int32_t *cells, int32_t nthreads,
                         int32_t *counts, int64_t cap, int32_t *lines, int64_t *needed);
int64_t vor_oracle_cells_poly(int32_t n, const int32_t *x, const int32_t *y, int32_t K,
                              const int32_t *vx, const int32_t *vy, int32_t m,
                              const int32_t *cells, int32_t nthreads, int32_t *counts,
                              int64_t cap, int32_t *lines, int64_t *needed);
int vor_oracle_vertices(int32_t n, const int32_t *x, const int32_t *y, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, int32_t m, const int32_t *cells,
                        const int32_t *counts, const int32_t *lines, uint64_t *X2, uint64_t *Y2,
                        int64_t *D);
int vor_oracle_vertices_poly(int32_t n, const int32_t *x, const int32_t *y, int32_t K,
                             const int32_t *vx, const int32_t *vy, int32_t m,
                             const int32_t *cells, const int32_t *counts, const int32_t *lines,
                             uint64_t *X2, uint64_t *Y2, int64_t *D);

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);    \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

/* xorshift64 (Marsaglia 2003) */
static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(uint32_t mod) {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (uint32_t)((rs >> 11) % mod);
}

static int taken(int n, const int32_t *x, const int32_t *y, int32_t a, int32_t b) {
    for (int i = 0; i < n; ++i)
        if (x[i] == a && y[i] == b) return 1;
    return 0;
}

/* the octagon X used below, counter-clockwise */
static const int32_t OX[8] = {200, 400, 600, 800, 800, 600, 400, 200};
static const int32_t OY[8] = {400, 200, 200, 400, 600, 800, 800, 600};
static int in_octagon(int32_t x, int32_t y) {
    for (int e = 0; e < 8; ++e) {
        const int64_t ax = OX[e], ay = OY[e], bx = OX[(e + 1) % 8], by = OY[(e + 1) % 8];
        if ((bx - ax) * (y - ay) - (by - ay) * (x - ax) < 0) return 0;
    }
    return 1;
}

/* every cell of a set: entry count within [3n, 6n + K - 6], vertices with D > 0, and the
 * capacity answer one entry short */
static void all_cells(int n, const int32_t *x, const int32_t *y, int K, int box, int threads) {
    int32_t *cells = malloc(sizeof(int32_t) * n), *counts = malloc(sizeof(int32_t) * n);
    const int64_t cap = 6 * (int64_t)n + K + 16;
    int32_t *lines = malloc(sizeof(int32_t) * cap);
    uint64_t *X2 = malloc(sizeof(uint64_t) * 2 * cap), *Y2 = malloc(sizeof(uint64_t) * 2 * cap);
    int64_t *D = malloc(sizeof(int64_t) * cap), needed = 0;
    for (int i = 0; i < n; ++i) cells[i] = i;
    const int64_t r = box ? vor_oracle_cells(n, x, y, 0, 0, 1000, 1000, n, cells, threads, counts,
                                             cap, lines, &needed)
                          : vor_oracle_cells_poly(n, x, y, 8, OX, OY, n, cells, threads, counts,
                                                  cap, lines, &needed);
    CHECK(r >= 3 * (int64_t)n && r <= 6 * (int64_t)n + K - 6 && needed == r);
    const int v = box ? vor_oracle_vertices(n, x, y, 0, 0, 1000, 1000, n, cells, counts, lines,
                                            X2, Y2, D)
                      : vor_oracle_vertices_poly(n, x, y, 8, OX, OY, n, cells, counts, lines, X2,
                                                 Y2, D);
    CHECK(v == 0);
    for (int64_t e = 0; e < r; ++e) CHECK(D[e] > 0);
    needed = 0;
    const int64_t r2 = box ? vor_oracle_cells(n, x, y, 0, 0, 1000, 1000, n, cells, threads, counts,
                                              r - 1, lines, &needed)
                           : vor_oracle_cells_poly(n, x, y, 8, OX, OY, n, cells, threads, counts,
                                                   r - 1, lines, &needed);
    CHECK(r2 == -4 && needed == r);
    free(cells);
    free(counts);
    free(lines);
    free(X2);
    free(Y2);
    free(D);
}

int main(void) {
    int32_t x[400], y[400];
    for (int trial = 0; trial < 12; ++trial) {
        /* box [0, 1000]^2, the first sites on its sides and corners */
        const int n = 3 + 31 * trial, nb = trial % 5;
        int k = 0;
        static const int32_t BX[5] = {0, 1000, 500, 0, 1000}, BY[5] = {0, 0, 1000, 300, 1000};
        for (; k < nb && k < n; ++k) {
            x[k] = BX[k];
            y[k] = BY[k];
        }
        while (k < n) {
            const int32_t a = 1 + (int32_t)rnd(999), b = 1 + (int32_t)rnd(999);
            if (taken(k, x, y, a, b)) continue;
            x[k] = a;
            y[k] = b;
            ++k;
        }
        CHECK(vor_oracle_validate(n, x, y, 0, 0, 1000, 1000) == 0);
        all_cells(n, x, y, 4, 1, 1 + trial % 3);
        /* the octagon, one site on a side */
        k = 0;
        x[k] = 300;
        y[k] = 300;   /* on the side (200,400)-(400,200) */
        ++k;
        while (k < n) {
            const int32_t a = 200 + (int32_t)rnd(601), b = 200 + (int32_t)rnd(601);
            if (!in_octagon(a, b) || taken(k, x, y, a, b)) continue;
            x[k] = a;
            y[k] = b;
            ++k;
        }
        CHECK(vor_oracle_validate_poly(n, x, y, 8, OX, OY) == 0);
        all_cells(n, x, y, 8, 0, 2);
    }
    /* errors: equal sites, a site outside, a clockwise polygon, bad arguments */
    int32_t ex[4] = {10, 20, 10, 30}, ey[4] = {10, 20, 10, 40};
    CHECK(vor_oracle_validate(4, ex, ey, 0, 0, 100, 100) == -3);
    ex[2] = 101;
    CHECK(vor_oracle_validate(4, ex, ey, 0, 0, 100, 100) == -2);
    int32_t cw_x[8], cw_y[8];
    for (int e = 0; e < 8; ++e) {
        cw_x[e] = OX[7 - e];
        cw_y[e] = OY[7 - e];
    }
    int32_t px[1] = {500}, py[1] = {500};
    CHECK(vor_oracle_validate_poly(1, px, py, 8, cw_x, cw_y) == -1);
    CHECK(vor_oracle_validate(0, px, py, 0, 0, 100, 100) == -1);
    int32_t cell0[1] = {5}, cnt[1];
    CHECK(vor_oracle_cells(1, px, py, 0, 0, 1000, 1000, 1, cell0, 1, cnt, 8, NULL, NULL) == -1);
    puts("oracle harness ok");
    return 0;
}
