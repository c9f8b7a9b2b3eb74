/*
 * filter_exact.c -- exact checker of FP32 endpoint keys, and the seeded instance families it
 * is run on.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests may load this library.  It shares no code with the
 * GPU path: it never computes a key, it only decides, in exact integer arithmetic, whether
 * floating-point keys produced elsewhere bracket the exact value.
 *
 * The quantity (eq. Tdef of Theorem 2.2): a ray from p in direction d meets the line
 * N.w <= c (p-relative, doubled frame) at t = c / (N.d) when N.d > 0.  The keys under test are
 * in units of d 2^-sigma, so the exact key is K = c 2^sigma / (N.d).  A sound filter has
 *   lower key (certified)  <= K <= upper key (certified),
 * an upper key that is finite only when N.d > 0, a lower key that is finite whenever N.d > 0
 * and K is inside FP32's range (K <= 2^127), and a bound for an exactly decided winner >= K.
 *
 * Domain of the instances: |N| <= 2^24 componentwise, 0 < c <= 2^50, |d| < 2^78 (the walk's
 * vertex directions stay below 2^77), so N.d < 2^103 and every product below fits 128 bits.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

/* ---- counter-based generator (splitmix64 finaliser of a 64-bit counter) ----------------- */
static uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
typedef struct { uint64_t key, ctr; } gen_t;
static uint64_t next64(gen_t *g) { return mix64(g->key ^ mix64(g->ctr++)); }
/* uniform in [lo, hi] (hi - lo < 2^63; the tiny modulo bias is irrelevant here) */
static int64_t urange(gen_t *g, int64_t lo, int64_t hi) {
    return lo + (int64_t)(next64(g) % (uint64_t)(hi - lo + 1));
}
/* signed value with |v| < 2^bits, bits in [1, 99] */
static i128 sbits(gen_t *g, int bits) {
    u128 v = ((u128)next64(g) << 64) | next64(g);
    v >>= (128 - bits);
    return (next64(g) & 1) ? -(i128)v : (i128)v;
}

static void put_dir(int64_t *dir, i128 x, i128 y) {
    dir[0] = (int64_t)(x >> 64);
    dir[1] = (int64_t)(uint64_t)x;
    dir[2] = (int64_t)(y >> 64);
    dir[3] = (int64_t)(uint64_t)y;
}

/*
 * Instance families (seeded; instance i of a call depends only on (family, seed, first + i)):
 *   0  site candidate, delta of 4..24 bits, direction of 2..77 bits
 *   1  general line (unit side normals a quarter of the time), c up to 2^50, same directions
 *   2  ray nearly perpendicular to the normal: d = M N_perp + j N + r, |j| <= 1, |r| <= 3
 *   3  vertex directions of two site lines (the walk's Z), tested against either line (an
 *      exact tie) or a site one unit away from either (a near-tie)
 *   4  cocircular lattice sites: p and the sites o + v, v one of the 8 symmetries of o, lie on
 *      one circle about o; the ray towards o ties all of them exactly; half are moved a unit
 * Returns 0, or -1 for an unknown family.
 */
int fx_generate(int family, uint64_t seed, int64_t first, int64_t n, int32_t *kind, int32_t *nx,
                int32_t *ny, int64_t *c, int64_t *dir) {
    if (family < 0 || family > 4) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        gen_t g = {mix64(seed * 8 + (uint64_t)family), (uint64_t)(first + i) << 8};
        int32_t k = 0, a = 0, b = 0;
        int64_t cc = 0;
        i128 dx = 0, dy = 0;
        for (;;) {
            if (family == 0 || family == 1) {
                const int bits = (int)urange(&g, 2, 77);
                dx = sbits(&g, bits);
                dy = sbits(&g, bits);
                if (family == 0) {
                    const int sc = 4 << urange(&g, 0, 2);   /* 4, 8, 16 */
                    const int e = urange(&g, 0, 3) == 0 ? 24 : sc;
                    a = (int32_t)urange(&g, -(1 << e) + 1, (1 << e) - 1);
                    b = (int32_t)urange(&g, -(1 << e) + 1, (1 << e) - 1);
                } else {
                    k = 1;
                    if (urange(&g, 0, 3) == 0) {
                        const int s = (int)urange(&g, 0, 3);
                        a = s == 0 ? 1 : s == 2 ? -1 : 0;
                        b = s == 1 ? 1 : s == 3 ? -1 : 0;
                        cc = urange(&g, 1, (int64_t)1 << 25);
                    } else {
                        a = (int32_t)urange(&g, -(1 << 24), 1 << 24);
                        b = (int32_t)urange(&g, -(1 << 24), 1 << 24);
                        cc = urange(&g, 1, (int64_t)1 << 50);
                    }
                }
            } else if (family == 2) {
                const int e = (int)urange(&g, 1, 24);
                a = (int32_t)urange(&g, -(1 << e) + 1, (1 << e) - 1);
                b = (int32_t)urange(&g, -(1 << e) + 1, (1 << e) - 1);
                if (urange(&g, 0, 1)) {
                    k = 1;
                    cc = urange(&g, 1, (int64_t)1 << 50);
                }
                const i128 M = sbits(&g, (int)urange(&g, 1, 76 - e));
                const int j = (int)urange(&g, -1, 1);
                dx = -M * b + (i128)j * a + urange(&g, -3, 3);
                dy = M * a + (i128)j * b + urange(&g, -3, 3);
            } else if (family == 3) {
                const int e = (int)urange(&g, 2, 24);
                const int64_t a1 = urange(&g, -(1 << e) + 1, (1 << e) - 1);
                const int64_t b1 = urange(&g, -(1 << e) + 1, (1 << e) - 1);
                const int64_t a2 = urange(&g, -(1 << e) + 1, (1 << e) - 1);
                const int64_t b2 = urange(&g, -(1 << e) + 1, (1 << e) - 1);
                const i128 cr = (i128)a1 * b2 - (i128)b1 * a2;
                if (cr == 0) continue;
                const i128 c1 = (i128)a1 * a1 + (i128)b1 * b1, c2 = (i128)a2 * a2 + (i128)b2 * b2;
                dx = c1 * b2 - c2 * b1;
                dy = (i128)a1 * c2 - (i128)a2 * c1;
                if (cr < 0) {
                    dx = -dx;
                    dy = -dy;
                }
                const int w = (int)urange(&g, 0, 5);
                a = (int32_t)(w & 1 ? a2 : a1);
                b = (int32_t)(w & 1 ? b2 : b1);
                if (w >= 2) {   /* a site one unit away */
                    const int s = (int)urange(&g, 0, 3);
                    a += s == 0 ? 1 : s == 2 ? -1 : 0;
                    b += s == 1 ? 1 : s == 3 ? -1 : 0;
                }
            } else {
                const int e = (int)urange(&g, 1, 22);
                const int32_t ox = (int32_t)urange(&g, -(1 << e), 1 << e);
                const int32_t oy = (int32_t)urange(&g, -(1 << e), 1 << e);
                const int s = (int)urange(&g, 0, 6);   /* the 8 symmetries of o except -o */
                const int32_t vx[7] = {ox, -ox, ox, oy, -oy, oy, -oy};
                const int32_t vy[7] = {oy, oy, -oy, ox, ox, -ox, -ox};
                a = ox + vx[s];
                b = oy + vy[s];
                if (urange(&g, 0, 1)) {
                    const int u = (int)urange(&g, 0, 3);
                    a += u == 0 ? 1 : u == 2 ? -1 : 0;
                    b += u == 1 ? 1 : u == 3 ? -1 : 0;
                }
                const i128 f = urange(&g, 1, (int64_t)1 << urange(&g, 0, 40));
                dx = f * ox;
                dy = f * oy;
            }
            if (a == 0 && b == 0) continue;
            if (dx == 0 && dy == 0) continue;
            break;
        }
        kind[i] = k;
        nx[i] = a;
        ny[i] = b;
        c[i] = cc;
        put_dir(dir + 4 * i, dx, dy);
    }
    return 0;
}

/* ---- exact comparisons ------------------------------------------------------------------ */
static int bitlen(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    return hi ? 128 - __builtin_clzll(hi) : lo ? 64 - __builtin_clzll(lo) : 0;
}
/* sign(A 2^k - B), A, B < 2^128, k >= 0 */
static int cmp_shl(u128 A, int k, u128 B) {
    if (A == 0) return B ? -1 : 0;
    const int la = bitlen(A), lb = bitlen(B);
    if (la + k != lb) return la + k > lb ? 1 : -1;
    const u128 hi = B >> k;   /* k < 128 here */
    if (A != hi) return A > hi ? 1 : -1;
    const u128 rem = k ? (B & (((u128)1 << k) - 1)) : 0;
    return rem ? -1 : 0;
}
/* sign(A 2^ea - B 2^eb) */
static int cmp_pow(u128 A, int ea, u128 B, int eb) {
    return ea >= eb ? cmp_shl(A, ea - eb, B) : -cmp_shl(B, eb - ea, A);
}
/* sign(f - K) for finite f >= 0 and K = num 2^s / den (den > 0), with an extra factor
 * (fnum / 2^24) on K when fnum != 0 */
static int cmp_key(float f, u128 num, int s, u128 den) {
    if (f == 0.0f) return num ? -1 : 0;
    int ex;
    const float fr = frexpf(f, &ex);             /* f = fr 2^ex, fr in [0.5, 1) */
    const u128 m = (u128)(uint32_t)ldexpf(fr, 24); /* f = m 2^(ex - 24), m < 2^24 */
    return cmp_pow(m * den, ex - 24, num, s);
}

enum {
    FX_TOTAL = 0, FX_POS, FX_LO_FINITE, FX_HI_FINITE, FX_TIGHT,
    FX_BAD_SIGN, FX_BAD_LO_INF, FX_BAD_LO, FX_BAD_HI, FX_BAD_XUP, FX_BAD_TIGHT, FX_FIRST_BAD,
    FX_NCOUNTS
};

/*
 * Checks n instances (layout of the diagnostic entry: out[8i..8i+4] = key_lo, key_hi,
 * certified key_lo, certified key_hi, exact-winner bound) and adds to counts[FX_NCOUNTS]:
 * instances, N.d > 0, finite lower / upper keys, well-conditioned instances (2 N.d >= S,
 * S = |N_x d_x| + |N_y d_y|), and failures by kind; counts[FX_FIRST_BAD] (start it at -1)
 * gets the index of the first failing instance of this call unless already set.  Returns the
 * number of failing instances.  Threads: OpenMP over the instances.
 */
int64_t fx_check(int64_t n, const int32_t *kind, const int32_t *nx, const int32_t *ny,
                 const int64_t *c, const int64_t *dir, const float *out, const int32_t *sigma,
                 int64_t *counts) {
    int64_t bad_total = 0, first = -1;
#pragma omp parallel reduction(+ : bad_total)
    {
    int64_t cnt[FX_NCOUNTS] = {0};
    int64_t my_first = -1;
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const i128 dx = ((i128)dir[4 * i] << 64) | (uint64_t)dir[4 * i + 1];
        const i128 dy = ((i128)dir[4 * i + 2] << 64) | (uint64_t)dir[4 * i + 3];
        const i128 a = nx[i], b = ny[i];
        const u128 cc = kind[i] == 0 ? (u128)(a * a + b * b) : (u128)c[i];
        const i128 den = a * dx + b * dy;
        const float *o = out + 8 * i;
        const float klo = o[0], khi = o[1], klo_c = o[2], khi_c = o[3], xup = o[4];
        const int s = sigma[i];
        int bad = isnan(klo) || isnan(khi) || isnan(klo_c) || isnan(khi_c) || isnan(xup) ||
                  klo < 0.0f || khi < 0.0f || xup < 0.0f;
        if (bad) cnt[FX_BAD_SIGN]++;
        cnt[FX_TOTAL]++;
        if (!isinf(khi)) cnt[FX_HI_FINITE]++;
        if (den <= 0) {
            if (!isinf(khi) || !isinf(khi_c) || !isinf(xup)) {
                cnt[FX_BAD_SIGN]++;
                bad = 1;
            }
        } else {
            const u128 D = (u128)den;
            cnt[FX_POS]++;
            /* K > 2^127 <=> c 2^s > D 2^127 */
            const int huge = cmp_pow(cc, s, D, 127) > 0;
            if (isinf(klo)) {
                if (!huge) {
                    cnt[FX_BAD_LO_INF]++;
                    bad = 1;
                }
            } else {
                cnt[FX_LO_FINITE]++;
                if (cmp_key(klo_c, cc, s, D) > 0) {
                    cnt[FX_BAD_LO]++;
                    bad = 1;
                }
            }
            if (!isinf(khi_c) && cmp_key(khi_c, cc, s, D) < 0) {
                cnt[FX_BAD_HI]++;
                bad = 1;
            }
            if (isinf(xup) ? !huge : cmp_key(xup, cc, s, D) < 0) {
                cnt[FX_BAD_XUP]++;
                bad = 1;
            }
            const i128 ax = a * dx, by = b * dy;
            const u128 S = (u128)(ax < 0 ? -ax : ax) + (u128)(by < 0 ? -by : by);
            if ((u128)2 * D >= S) {
                /* well conditioned: both keys within 32u of K, i.e.
                 * K (2^24 - 32) <= key 2^24 <= K (2^24 + 32) */
                cnt[FX_TIGHT]++;
                int t = isinf(klo) || isinf(khi);
                const float ks[2] = {klo, khi};
                for (int q = 0; q < 2 && !t; ++q) {
                    int ex;
                    const float fr = frexpf(ks[q], &ex);
                    const u128 m = (u128)(uint32_t)ldexpf(fr, 24);
                    if (ks[q] == 0.0f ||
                        cmp_pow(m * D, ex, cc * (((u128)1 << 24) - 32), s) < 0 ||
                        cmp_pow(m * D, ex, cc * (((u128)1 << 24) + 32), s) > 0)
                        t = 1;
                }
                if (t) {
                    cnt[FX_BAD_TIGHT]++;
                    bad = 1;
                }
            }
        }
        if (bad) {
            if (my_first < 0) my_first = i;
            ++bad_total;
        }
    }
#pragma omp critical
    {
        for (int q = 0; q < FX_FIRST_BAD; ++q) counts[q] += cnt[q];
        if (my_first >= 0 && (first < 0 || my_first < first)) first = my_first;
    }
    }
    if (first >= 0 && counts[FX_FIRST_BAD] < 0) counts[FX_FIRST_BAD] = first;
    return bad_total;
}
