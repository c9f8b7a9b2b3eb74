/*
 * vor_oracle.c -- plain, slow, exact CPU oracle for the Voronoi diagram of integer point
 * sites restricted to an axis-aligned box.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code with the GPU path.
 *
 * What it computes (the plain definition, not the projector method):
 *   Section 2, Definition of the Voronoi diagram: the cell of p_k is the set of points of
 *   X at least as close to p_k as to every other site.  That set is X intersected with the
 *   n-1 closed half-planes H_kj = { x : 2 (p_j - p_k) . x <= |p_j|^2 - |p_k|^2 }.
 *   The oracle starts from X and intersects the half-planes one after another, exactly,
 *   in 128-bit integer arithmetic.  The intersection does not depend on the order.
 *
 * Output per cell (Section 6, storing the data; Section 7, the Delaunay graph):
 *   the counter-clockwise cyclic list of the lines that carry an edge of positive length,
 *   each line named by the index of the neighbouring site (0..n-1) or by a box-side code
 *       -1 : y = y0 (bottom)   -2 : x = x1 (right)   -3 : y = y1 (top)   -4 : x = x0 (left)
 *   For a convex polygon X with vertices v_0..v_{K-1} (counter-clockwise; Remark 11.1 on a
 *   general convex X), side e runs from v_e to v_{e+1} and is named -(e+1); its line is
 *   N.x <= N.v_e with N = (dy, -dx) / gcd(|dx|, |dy|), (dx, dy) = v_{e+1} - v_e, the primitive
 *   outward normal.  The box is the polygon (x0,y0), (x1,y0), (x1,y1), (x0,y1): the same codes
 *   and lines.
 *   rotated so that the entry that is smallest when read as uint32 comes first.
 *   Vertex i of the cell is line(i) ∩ line(i+1 mod m), written in pair form
 *       D = N1x N2y - N1y N2x,   X = c1 N2y - c2 N1y,   Y = N1x c2 - N2x c1,
 *   for rows N.x <= c of the two lines in absolute coordinates: site lines use
 *   N = 2 (p_j - p_k), c = |p_j|^2 - |p_k|^2, the sides use the unit outward normal.
 *
 * Arithmetic bounds (box extent <= 2^24, |coordinate| <= 2^30): |N| < 2^25, |c| < 2^56 for
 * site lines, so D < 2^51, |X|, |Y| < 2^82, and the clip test c_j D - N_j.(X, Y) < 2^110:
 * every quantity fits __int128 exactly.
 *
 * Error codes: 0 ok, -1 invalid argument, -2 site outside the closed X or box too large,
 * -3 two equal sites, -4 output capacity too small, -5 out of memory.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

typedef struct {
    int64_t nx, ny, c; /* N.x <= c, absolute coordinates */
    int32_t id;        /* site index, or -1..-4 for a box side */
} oline;

#define MAX_SIDES 256

typedef struct {
    int32_t n;
    const int32_t *x, *y;
    int32_t ns;                 /* sides of X */
    oline sides[MAX_SIDES];     /* side e (code -(e+1)), counter-clockwise */
} oset;

static oline make_line(const oset *S, int32_t k, int32_t id) {
    if (id < 0) return S->sides[-id - 1];
    oline L;
    L.id = id;
    int64_t px = S->x[k], py = S->y[k], qx = S->x[id], qy = S->y[id];
    L.nx = 2 * (qx - px);
    L.ny = 2 * (qy - py);
    L.c = (qx * qx + qy * qy) - (px * px + py * py);
    return L;
}

static int64_t gcd64(int64_t a, int64_t b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

/* Side lines of the convex polygon (vx, vy)[0..K-1]; the caller has validated it. */
static void polygon_sides(oset *S, int32_t K, const int32_t *vx, const int32_t *vy) {
    S->ns = K;
    for (int32_t e = 0; e < K; ++e) {
        const int64_t ax = vx[e], ay = vy[e], bx = vx[(e + 1) % K], by = vy[(e + 1) % K];
        const int64_t dx = bx - ax, dy = by - ay, g = gcd64(dx, dy);
        oline L;
        L.id = -(e + 1);
        L.nx = dy / g;
        L.ny = -dx / g;
        L.c = L.nx * ax + L.ny * ay;
        S->sides[e] = L;
    }
}

static void box_sides(oset *S, int32_t x0, int32_t y0, int32_t x1, int32_t y1) {
    const int32_t vx[4] = {x0, x1, x1, x0}, vy[4] = {y0, y0, y1, y1};
    polygon_sides(S, 4, vx, vy);
}

/* Intersection of two non-parallel lines, pair form (X/D, Y/D). */
static void meet(const oline *a, const oline *b, i128 *X, i128 *Y, int64_t *D) {
    *D = a->nx * b->ny - a->ny * b->nx;
    *X = (i128)a->c * b->ny - (i128)b->c * a->ny;
    *Y = (i128)a->nx * b->c - (i128)b->nx * a->c;
}

/* sign of c - N.v for v = (X/D, Y/D), D > 0: +1 strictly inside, 0 on the line, -1 outside */
static int side_of(const oline *L, i128 X, i128 Y, int64_t D) {
    i128 s = (i128)L->c * D - ((i128)L->nx * X + (i128)L->ny * Y);
    return (s > 0) - (s < 0);
}

static i128 iabs128(i128 v) { return v < 0 ? -v : v; }

/* Integer upper bound on max_i |v_i - p| (L1 bound of each vertex, rounded up). */
static int64_t radius_bound(const oline *P, int m, int64_t px, int64_t py) {
    int64_t r = 0;
    for (int i = 0; i < m; ++i) {
        i128 X, Y;
        int64_t D;
        meet(&P[i], &P[(i + 1) % m], &X, &Y, &D);
        i128 num = iabs128(X - (i128)px * D) + iabs128(Y - (i128)py * D);
        i128 q = (num + D - 1) / D;
        if (q > r) r = (int64_t)q;
    }
    return r;
}

/*
 * Intersect the convex polygon P (m lines, CCW) with the half-plane H.  Writes the result to
 * Q and returns its size.  Edge i lies on P[i] and runs from vertex i-1 to vertex i.
 */
static int clip(const oline *P, int m, const oline *H, oline *Q, int *s) {
    int any_out = 0;
    for (int i = 0; i < m; ++i) {
        i128 X, Y;
        int64_t D;
        meet(&P[i], &P[(i + 1) % m], &X, &Y, &D);
        s[i] = side_of(H, X, Y, D);
        if (s[i] < 0) any_out = 1;
    }
    if (!any_out) return -1; /* H contains P: touching at a vertex adds no edge */
    int q = 0;
    for (int i = 0; i < m; ++i) {
        int sp = s[(i + m - 1) % m], se = s[i];
        int keep = (sp > 0) || (se > 0);
        if (!keep) continue;
        Q[q++] = P[i];
        int next = (i + 1) % m;
        int keep_next = (se > 0) || (s[next] > 0);
        if (se < 0 || (se == 0 && !keep_next)) Q[q++] = *H;
    }
    return q;
}

/* One cell: returns the number of lines written to out (CCW, not yet rotated), or < 0. */
static int cell_lines(const oset *S, int32_t k, oline **bufA, oline **bufB, int **sbuf, int *cap,
                      int32_t *out_ids, int out_cap) {
    oline *P = *bufA, *Q = *bufB;
    int m = S->ns;
    for (int e = 0; e < m; ++e) P[e] = S->sides[e];
    int64_t px = S->x[k], py = S->y[k];
    int64_t R = radius_bound(P, m, px, py);
    for (int32_t j = 0; j < S->n; ++j) {
        if (j == k) continue;
        int64_t dx = (int64_t)S->x[j] - px, dy = (int64_t)S->y[j] - py;
        int64_t q2 = dx * dx + dy * dy;
        /* |z - p| <= R on P and |p_j - p| >= 2R  =>  P lies in H_kj (exact prune) */
        if (q2 >= 4 * R * R) continue;
        if (m + 1 > *cap) {
            int nc = *cap * 2;
            oline *a = (oline *)realloc(P, sizeof(oline) * nc);
            if (!a) { *bufA = P; *bufB = Q; return -5; }
            P = a;
            oline *b = (oline *)realloc(Q, sizeof(oline) * nc);
            if (!b) { *bufA = P; *bufB = Q; return -5; }
            Q = b;
            int *sb = (int *)realloc(*sbuf, sizeof(int) * nc);
            if (!sb) { *bufA = P; *bufB = Q; return -5; }
            *sbuf = sb;
            *cap = nc;
        }
        oline H = make_line(S, k, j);
        int r = clip(P, m, &H, Q, *sbuf);
        if (r < 0) continue;
        oline *t = P;
        P = Q;
        Q = t;
        m = r;
        R = radius_bound(P, m, px, py);
    }
    /* keep the buffers the caller owns in sync with the swapped pointers */
    *bufA = P;
    *bufB = Q;
    if (m > out_cap) return -4;
    for (int i = 0; i < m; ++i) out_ids[i] = P[i].id;
    return m;
}

static void rotate_canonical(int32_t *ids, int m) {
    int best = 0;
    for (int i = 1; i < m; ++i)
        if ((uint32_t)ids[i] < (uint32_t)ids[best]) best = i;
    if (best == 0) return;
    int32_t tmp[64];
    int32_t *t = m <= 64 ? tmp : (int32_t *)malloc(sizeof(int32_t) * m);
    for (int i = 0; i < m; ++i) t[i] = ids[(best + i) % m];
    memcpy(ids, t, sizeof(int32_t) * m);
    if (t != tmp) free(t);
}

typedef struct {
    const oset *S;
    const int32_t *cells;
    int32_t m;
    int32_t **res;   /* per requested cell: malloc'd id list */
    int32_t *counts; /* per requested cell */
    volatile int64_t *next;
    pthread_mutex_t *mu;
    int err;
} job_t;

static void *worker(void *arg) {
    job_t *J = (job_t *)arg;
    int cap = MAX_SIDES + 64;
    oline *A = (oline *)malloc(sizeof(oline) * cap);
    oline *B = (oline *)malloc(sizeof(oline) * cap);
    int *sb = (int *)malloc(sizeof(int) * cap);
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)J->S->n + MAX_SIDES + 8));
    if (!A || !B || !sb || !tmp) {
        J->err = -5;
        free(A); free(B); free(sb); free(tmp);
        return NULL;
    }
    for (;;) {
        int64_t i;
        pthread_mutex_lock(J->mu);
        i = (*J->next)++;
        pthread_mutex_unlock(J->mu);
        if (i >= J->m) break;
        int32_t k = J->cells[i];
        int r = cell_lines(J->S, k, &A, &B, &sb, &cap, tmp, J->S->n + MAX_SIDES + 8);
        if (r < 0) {
            J->err = r;
            break;
        }
        rotate_canonical(tmp, r);
        int32_t *o = (int32_t *)malloc(sizeof(int32_t) * r);
        if (!o) {
            J->err = -5;
            break;
        }
        memcpy(o, tmp, sizeof(int32_t) * r);
        J->res[i] = o;
        J->counts[i] = r;
    }
    free(A); free(B); free(sb); free(tmp);
    return NULL;
}

static int cmp_pt(const void *a, const void *b) {
    const int64_t *p = (const int64_t *)a, *q = (const int64_t *)b;
    return (*p > *q) - (*p < *q);
}

/* Distinctness by a lexicographic sort and an adjacent compare (the remark on checking that
 * the sites are distinct). */
static int check_distinct(int32_t n, const int32_t *x, const int32_t *y) {
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * n);
    if (!key) return -5;
    for (int32_t i = 0; i < n; ++i)
        key[i] = (int64_t)(((uint64_t)(uint32_t)x[i] << 32) | (uint64_t)(uint32_t)y[i]);
    qsort(key, n, sizeof(int64_t), cmp_pt);
    int dup = 0;
    for (int32_t i = 1; i < n; ++i)
        if (key[i] == key[i - 1]) { dup = 1; break; }
    free(key);
    return dup ? -3 : 0;
}

/*
 * Input check: distinct sites in the closed X.  The problem statement of Section 2 takes the
 * sites in the interior of X and notes that the definition of the cells extends to sites on the
 * boundary of X unchanged (a cell is X intersected with the half-planes of the other sites);
 * sites on the boundary are accepted, sites outside X are not.
 */
int vor_oracle_validate(int32_t n, const int32_t *x, const int32_t *y, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1) {
    if (n < 1 || !x || !y) return -1;
    if (!(x0 < x1 && y0 < y1)) return -1;
    if ((int64_t)x1 - x0 > (1 << 24) || (int64_t)y1 - y0 > (1 << 24)) return -2;
    const int64_t lim = (int64_t)1 << 30;
    if (x0 < -lim || y0 < -lim || x1 > lim || y1 > lim) return -2;
    for (int32_t i = 0; i < n; ++i)
        if (!(x[i] >= x0 && x[i] <= x1 && y[i] >= y0 && y[i] <= y1)) return -2;
    return check_distinct(n, x, y);
}

/*
 * X a convex polygon (Remark 11.1): 3 <= K <= 256 vertices, |coordinate| <= 2^30, bounding box
 * extent <= 2^24, counter-clockwise and strictly convex (every turn strictly left) and simple
 * (the edge directions go round once: they change between the upper and the lower half-plane
 * exactly twice).  Sites inside or on every side (the closed X).  -1 for a bad polygon, -2
 * for a site outside or an extent too large, -3 for equal sites.
 */
int vor_oracle_validate_poly(int32_t n, const int32_t *x, const int32_t *y, int32_t K,
                             const int32_t *vx, const int32_t *vy) {
    if (n < 1 || !x || !y || !vx || !vy || K < 3 || K > MAX_SIDES) return -1;
    const int64_t lim = (int64_t)1 << 30;
    int64_t mnx = vx[0], mxx = vx[0], mny = vy[0], mxy = vy[0];
    for (int32_t e = 0; e < K; ++e) {
        if (vx[e] < -lim || vx[e] > lim || vy[e] < -lim || vy[e] > lim) return -2;
        if (vx[e] < mnx) mnx = vx[e];
        if (vx[e] > mxx) mxx = vx[e];
        if (vy[e] < mny) mny = vy[e];
        if (vy[e] > mxy) mxy = vy[e];
    }
    if (mxx - mnx > (1 << 24) || mxy - mny > (1 << 24)) return -2;
    int changes = 0;
    for (int32_t e = 0; e < K; ++e) {
        const int32_t f = (e + 1) % K, g = (e + 2) % K;
        const int64_t ax = (int64_t)vx[f] - vx[e], ay = (int64_t)vy[f] - vy[e];
        const int64_t bx = (int64_t)vx[g] - vx[f], by = (int64_t)vy[g] - vy[f];
        if (ax * by - ay * bx <= 0) return -1;
        const int ua = ay > 0 || (ay == 0 && ax > 0), ub = by > 0 || (by == 0 && bx > 0);
        changes += ua != ub;
    }
    if (changes != 2) return -1;
    oset *S = (oset *)malloc(sizeof(oset));
    if (!S) return -5;
    polygon_sides(S, K, vx, vy);
    int out = 0;
    for (int32_t i = 0; i < n && !out; ++i)
        for (int32_t e = 0; e < K; ++e)
            if (S->sides[e].nx * x[i] + S->sides[e].ny * y[i] > S->sides[e].c) {
                out = 1;
                break;
            }
    free(S);
    return out ? -2 : check_distinct(n, x, y);
}

static int64_t cells_impl(const oset *S, int32_t m, const int32_t *cells, int32_t nthreads,
                          int32_t *counts, int64_t cap, int32_t *lines, int64_t *needed) {
    const int32_t n = S->n;
    if (m < 0 || (m > 0 && (!cells || !counts))) return -1;
    for (int32_t i = 0; i < m; ++i)
        if (cells[i] < 0 || cells[i] >= n) return -1;
    int32_t **res = (int32_t **)calloc(m > 0 ? m : 1, sizeof(int32_t *));
    if (!res) return -5;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    volatile int64_t next = 0;
    pthread_mutex_t mu;
    pthread_mutex_init(&mu, NULL);
    job_t J = {S, cells, m, res, counts, &next, &mu, 0};
    job_t jobs[256];
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = J;
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    int err = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].err) err = jobs[t].err;
    }
    pthread_mutex_destroy(&mu);
    int64_t total = 0;
    if (!err) {
        for (int32_t i = 0; i < m; ++i) total += counts[i];
        if (needed) *needed = total;
        if (total > cap || !lines) {
            err = -4;
        } else {
            int64_t o = 0;
            for (int32_t i = 0; i < m; ++i) {
                memcpy(lines + o, res[i], sizeof(int32_t) * counts[i]);
                o += counts[i];
            }
        }
    }
    for (int32_t i = 0; i < m; ++i) free(res[i]);
    free(res);
    return err ? err : total;
}

/*
 * Cells of the sites listed in cells[0..m-1].  counts[i] receives the size of cell cells[i];
 * the lists are written one after another to lines[0..cap-1].  Returns the total number of
 * entries, or a negative error code (-4 if cap is too small: *needed receives the size).
 */
int64_t vor_oracle_cells(int32_t n, const int32_t *x, const int32_t *y, int32_t x0, int32_t y0,
                         int32_t x1, int32_t y1, int32_t m, const int32_t *cells, int32_t nthreads,
                         int32_t *counts, int64_t cap, int32_t *lines, int64_t *needed) {
    int v = vor_oracle_validate(n, x, y, x0, y0, x1, y1);
    if (v) return v;
    oset *S = (oset *)malloc(sizeof(oset));
    if (!S) return -5;
    S->n = n;
    S->x = x;
    S->y = y;
    box_sides(S, x0, y0, x1, y1);
    const int64_t r = cells_impl(S, m, cells, nthreads, counts, cap, lines, needed);
    free(S);
    return r;
}

/* Same for a convex polygon X (vertices vx, vy, counter-clockwise). */
int64_t vor_oracle_cells_poly(int32_t n, const int32_t *x, const int32_t *y, int32_t K,
                              const int32_t *vx, const int32_t *vy, int32_t m,
                              const int32_t *cells, int32_t nthreads, int32_t *counts,
                              int64_t cap, int32_t *lines, int64_t *needed) {
    int v = vor_oracle_validate_poly(n, x, y, K, vx, vy);
    if (v) return v;
    oset *S = (oset *)malloc(sizeof(oset));
    if (!S) return -5;
    S->n = n;
    S->x = x;
    S->y = y;
    polygon_sides(S, K, vx, vy);
    const int64_t r = cells_impl(S, m, cells, nthreads, counts, cap, lines, needed);
    free(S);
    return r;
}

static int vertices_impl(const oset *S, int32_t m, const int32_t *cells, const int32_t *counts,
                         const int32_t *lines, uint64_t *X2, uint64_t *Y2, int64_t *D) {
    int64_t o = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t k = cells[i], c = counts[i];
        for (int32_t t = 0; t < c; ++t) {
            oline a = make_line(S, k, lines[o + t]);
            oline b = make_line(S, k, lines[o + (t + 1) % c]);
            i128 XX, YY;
            int64_t DD;
            meet(&a, &b, &XX, &YY, &DD);
            if (DD == 0) return -1;
            X2[2 * (o + t)] = (uint64_t)XX;
            X2[2 * (o + t) + 1] = (uint64_t)(XX >> 64);
            Y2[2 * (o + t)] = (uint64_t)YY;
            Y2[2 * (o + t) + 1] = (uint64_t)(YY >> 64);
            D[o + t] = DD;
        }
        o += c;
    }
    return 0;
}

/*
 * Pair-form vertices of given cells: for cell cells[i] with list l_0..l_{c-1} (as written by
 * vor_oracle_cells), vertex t = line(l_t) ∩ line(l_{t+1 mod c}).  X and Y are written as
 * (low 64 bits, high 64 bits) pairs.  Returns 0, or -1 for a parallel pair (never happens for
 * a valid cell).
 */
int vor_oracle_vertices(int32_t n, const int32_t *x, const int32_t *y, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, int32_t m, const int32_t *cells,
                        const int32_t *counts, const int32_t *lines, uint64_t *X2, uint64_t *Y2,
                        int64_t *D) {
    oset *S = (oset *)malloc(sizeof(oset));
    if (!S) return -5;
    S->n = n;
    S->x = x;
    S->y = y;
    box_sides(S, x0, y0, x1, y1);
    const int r = vertices_impl(S, m, cells, counts, lines, X2, Y2, D);
    free(S);
    return r;
}

int vor_oracle_vertices_poly(int32_t n, const int32_t *x, const int32_t *y, int32_t K,
                             const int32_t *vx, const int32_t *vy, int32_t m,
                             const int32_t *cells, const int32_t *counts, const int32_t *lines,
                             uint64_t *X2, uint64_t *Y2, int64_t *D) {
    if (K < 3 || K > MAX_SIDES || !vx || !vy) return -1;
    oset *S = (oset *)malloc(sizeof(oset));
    if (!S) return -5;
    S->n = n;
    S->x = x;
    S->y = y;
    polygon_sides(S, K, vx, vy);
    const int r = vertices_impl(S, m, cells, counts, lines, X2, Y2, D);
    free(S);
    return r;
}

/* Number of worker threads this library would use by default (all online CPUs). */
#include <unistd.h>
int32_t vor_oracle_default_threads(void) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c < 1 ? 1 : (int32_t)c;
}
