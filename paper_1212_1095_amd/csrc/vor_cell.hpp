// vor_cell.hpp -- one Voronoi cell by the projector algorithm (Section 4, Algorithm 1).
//
// The projector starts with three corner rays whose consecutive directions are less than pi
// apart; every subedge {d1, d2} (a wedge spanned by two shot rays, d1 -> d2 counter-clockwise)
// holds the lines L1, L2 the two endpoints lie on.  A subedge is resolved as follows:
//
//  * L1 = L2 (same line id): no vertex in the wedge, the subedge is dropped (line SameLines).
//  * Otherwise with Den = cross(N1, N2) the system B lambda = H of eq. (B_lambda) has
//    det B = Den cross(d1, d2) (Binet-Cauchy) and, because both endpoints lie in the cell,
//    lambda = ((1 - a) / (1 - ab), (1 - b) / (1 - ab)) with a, b <= 1, so the sign of Den alone
//    decides the branch:
//      Den = 0 : L1 and L2 are antiparallel (line ParallelLines); the split direction is the
//                line direction rot90(N1), which lies strictly inside the wedge;
//      Den < 0 : lambda < 0, u = L1 ∩ L2 is behind p (line OutsideWedge); split along p - u;
//      Den > 0 : u is in the wedge; a ray towards u decides whether u is in the cell (line
//                Vertex: store the vertex) or not (line OutsideCell: split along u - p).
//    With u = Z / Den, Z = (c1 N2y - c2 N1y, N1x c2 - N2x c1), both split directions are the
//    integer vector Z itself.
//  * Splits push the new corner; the subedges are processed depth-first counter-clockwise, so
//    the finished corners come out in counter-clockwise order and their lines, with repeats
//    removed, are the cell's edges in cyclic order (Section 6: order recovered by labelling the
//    rays; prime subedges partition the projector).
//
// Exact ties at an endpoint (Remark 11.3): among the lines through the endpoint the one whose
// outward normal is the most clockwise carries an edge of the cell; it is the one chosen.
//
// Lane policies.  Solo: one lane computes one cell (the filtered pass over all cells).
// Coop: the 64 lanes of a wave compute one cell together -- every lane runs the same control
// flow, the candidates of a row are split across the lanes and the per-lane results are merged
// by a butterfly (the exact passes and small sets, where latency matters).
#pragma once
#include "vor_device.hpp"
#include "vor_tree.hpp"

namespace vor {

struct Counters {
    uint32_t rays, nodes, evals, exact, shells;
    // vertex tests (rays towards a candidate vertex that confirmed it) in the low 16 bits, and
    // all vertex rays (towards u = L1 ∩ L2, confirming or not) in the high 16 bits: one
    // register for both (a lane's counts stay far below 2^16)
    uint32_t vt;
    uint32_t xinc;   // exact decisions of vertex rays (the vertex-in-cell / incircle test)
};
constexpr uint32_t VT_VRAY = 1u << 16;

// ------------------------------------------------------------------------------ exact argmin
struct XBest {
    int id;
    int nx, ny;
    uint64_t c;
    u128 den;
    bool have;
};

// true when candidate (c, den, n) beats the current exact best: nearer hit, or at an exact tie
// the more clockwise normal (the smaller id if the normals were parallel, never for valid input)
__device__ __forceinline__ bool x_better(const XBest &b, int id, int nx, int ny, uint64_t c,
                                         u128 den) {
    if (!b.have) return true;
    const int s = cmp_t(c, den, b.c, b.den);
    if (s != 0) return s < 0;
    const int64_t cr = (int64_t)b.nx * ny - (int64_t)b.ny * nx;
    if (cr != 0) return cr < 0;
    return id < b.id;
}

__device__ __forceinline__ void x_consider(XBest &b, int id, int nx, int ny, int64_t c,
                                           const Dir &d) {
    const i128 den = (i128)nx * d.x + (i128)ny * d.y;
    if (den <= 0) return;
    if (!x_better(b, id, nx, ny, (uint64_t)c, (u128)den)) return;
    b.id = id;
    b.nx = nx;
    b.ny = ny;
    b.c = (uint64_t)c;
    b.den = (u128)den;
    b.have = true;
}

// Upper bound (FP32 key, scaled frame) of the exact winner's t = c / den.
__device__ __forceinline__ float x_upper(const XBest &b, const Dir &d) {
    if (!b.have) return FINF;
    const double t = (double)b.c / u128_to_double(b.den);
    return (float)ldexp(t, d.sigma) * CERT_UP;
}

// ------------------------------------------------------------------------------ lane policies
struct Solo {
    static constexpr int W = 1;
    __device__ static __forceinline__ int lane() { return 0; }
    __device__ static __forceinline__ void reduce(Best &) {}
    __device__ static __forceinline__ void reduce(XBest &) {}
};

struct Coop {
    static constexpr int W = 64;
    __device__ static __forceinline__ int lane() { return threadIdx.x & 63; }
    // Merge of two (smallest, second smallest, argmin) summaries; a candidate held by both
    // halves (the winner carried over from an earlier pass) counts once.
    __device__ static __forceinline__ void reduce(Best &b) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float o1 = __shfl_xor(b.k1, off, 64);
            const float o2 = __shfl_xor(b.k2, off, 64);
            const int ow = __shfl_xor(b.w, off, 64);
            if (ow == b.w) {
                b.k2 = fminf(b.k2, o2);
            } else if (o1 < b.k1 || (o1 == b.k1 && ow < b.w)) {
                b.k2 = fminf(b.k1, o2);
                b.k1 = o1;
                b.w = ow;
            } else {
                b.k2 = fminf(b.k2, o1);
            }
        }
    }
    __device__ static __forceinline__ void reduce(XBest &b) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            XBest o;
            o.id = __shfl_xor(b.id, off, 64);
            o.nx = __shfl_xor(b.nx, off, 64);
            o.ny = __shfl_xor(b.ny, off, 64);
            const uint32_t c0 = __shfl_xor((uint32_t)b.c, off, 64);
            const uint32_t c1 = __shfl_xor((uint32_t)(b.c >> 32), off, 64);
            o.c = ((uint64_t)c1 << 32) | c0;
            uint32_t dd[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) dd[q] = __shfl_xor((uint32_t)(b.den >> (32 * q)), off, 64);
            o.den = ((u128)dd[3] << 96) | ((u128)dd[2] << 64) | ((u128)dd[1] << 32) | dd[0];
            o.have = __shfl_xor((int)b.have, off, 64) != 0;
            if (o.have && (!b.have || o.id != b.id) && x_better(b, o.id, o.nx, o.ny, o.c, o.den))
                b = o;
        }
    }
};

// The projector's corner ray i (0, 1, 2): (7, -4), (0, 1), (-7, -4), counter-clockwise, gaps < pi.
__device__ __forceinline__ Dir corner_dir(int i) {
    return make_dir(i == 1 ? 0 : (i == 0 ? 7 : -7), i == 1 ? 1 : -4);
}

// ------------------------------------------------------------------------------ FP32 scan
struct ScanOut {
    Best b;
    float Uw;   // upper bound key of the final winner
    float U;    // smallest upper bound seen
    float Tr;   // the bound whose S_I the scanned region contains
    Rect A;     // the scanned rectangle (it contains S_I of the endpoint)
};

// Upper bound key of candidate w (sorted position or side code).
__device__ __forceinline__ float upper_of(const Cell &C, const float2 *__restrict__ sxy, int w,
                                          float dx, float dy) {
    if (w == NO_TAG) return FINF;
    if (w >= 0) {
        const float2 a = sxy[w];
        const float ex = a.x - C.pxf, ey = a.y - C.pyf;
        return key_hi_line(site_q(ex, ey), ex, ey, dx, dy);
    }
    const Line L = side_line(C, w);
    return key_hi_line((float)L.c, (float)L.nx, (float)L.ny, dx, dy);
}

// The side of a convex polygon X through which the ray p + t d leaves, by binary search over
// the vertex directions w_e = v_e - p (counter-clockwise around p, p inside): the side e with
// w_e <= d < w_{e+1} in angle measured from w_0.  FP32 cross products with w exact (|w| <=
// 2^24) and d_s rounded: the computed cross differs from the exact one by at most 3.05u S,
// S = |w_x d_y| + |w_y d_x|; any decision closer than 8u S returns -1 (the caller takes every
// side).  A robust answer is exact: that side is hit first, and strictly before the others.
__device__ __forceinline__ int exit_side(const Cell &C, float dx, float dy) {
    const float tol = 8.0f * 5.9604644775390625e-8f;
    const SideRel s0 = C.sides[0];
    const int64_t w0x = (int64_t)s0.vx - C.px, w0y = (int64_t)s0.vy - C.py;
    // half-plane of d relative to w_0: 0 for angles in [0, pi), 1 for [pi, 2 pi)
    const float a0 = (float)w0x * dy, b0 = (float)w0y * dx;
    const float c0 = a0 - b0;
    if (!(fabsf(c0) > tol * (fabsf(a0) + fabsf(b0)))) return -1;
    const int hd = c0 > 0.0f ? 0 : 1;
    int lo = 1, hi = C.ns;   // smallest k in [1, ns] with angle(d) < angle(w_k); ns: none
    while (lo < hi) {
        const int k = (lo + hi) >> 1;
        const SideRel s = C.sides[k];
        const int64_t wx = (int64_t)s.vx - C.px, wy = (int64_t)s.vy - C.py;
        const int64_t cw = w0x * wy - w0y * wx;   // exact
        const int hw = (cw > 0 || (cw == 0 && w0x * wx + w0y * wy > 0)) ? 0 : 1;
        bool before;
        if (hd != hw) {
            before = hd < hw;
        } else {
            const float a = dx * (float)wy, bb = dy * (float)wx;
            const float cr = a - bb;   // cross(d, w_k)
            if (!(fabsf(cr) > tol * (fabsf(a) + fabsf(bb)))) return -1;
            before = cr > 0.0f;
        }
        if (before) hi = k; else lo = k + 1;
    }
    return lo - 1;
}

// Sides the ray can leave through: for the box at most one horizontal and one vertical side;
// for a polygon the exit side (every side with N.d > 0 when the search is not robust).
__device__ __forceinline__ void consider_sides(const Cell &C, float dx, float dy, int ex1, int ex2,
                                               Best &b) {
    if (C.ns > 0) {
        const int e = exit_side(C, dx, dy);
        if (e >= 0) {
            const int code = -e - 1;
            const Line L = side_line(C, code);
            float k = key_lo_line((float)L.c, (float)L.nx, (float)L.ny, dx, dy);
            k = (code == ex1 || code == ex2) ? FINF : k;
            consider(k, code, b);
            return;
        }
        for (int code = -1; code >= -C.ns; --code) {
            const Line L = side_line(C, code);
            float k = key_lo_line((float)L.c, (float)L.nx, (float)L.ny, dx, dy);
            k = (code == ex1 || code == ex2) ? FINF : k;
            consider(k, code, b);
        }
        return;
    }
    const int sv = dy > 0.0f ? -3 : -1, sh = dx > 0.0f ? -2 : -4;
    const Line Lv = side_line(C, sv), Lh = side_line(C, sh);
    float kv = key_lo_line((float)Lv.c, (float)Lv.nx, (float)Lv.ny, dx, dy);
    float kh = key_lo_line((float)Lh.c, (float)Lh.nx, (float)Lh.ny, dx, dy);
    kv = (sv == ex1 || sv == ex2) ? FINF : kv;
    kh = (sh == ex1 || sh == ex2) ? FINF : kh;
    consider(kv, sv, b);
    consider(kh, sh, b);
}

__device__ __forceinline__ void eval_at(const Cell &C, float2 a, int pos, float dx, float dy,
                                        int ex1, int ex2, Best &b) {
    const float ex = a.x - C.pxf, ey = a.y - C.pyf;
    float key = key_lo_scan(ex, ey, dx, dy);
    key = (pos == ex1 || pos == ex2) ? FINF : key;
    consider(key, pos, b);
}
__device__ __forceinline__ void eval_site(const Cell &C, const float2 *__restrict__ sxy, int pos,
                                          float dx, float dy, int ex1, int ex2, Best &b) {
    eval_at(C, sxy[pos], pos, dx, dy, ex1, ex2, b);
}

// Candidates [pos, end) with stride W, two per step so that their loads overlap.
template <int W>
__device__ __forceinline__ void eval_range(const Cell &C, const float2 *__restrict__ sxy, int pos,
                                           int end, float dx, float dy, int ex1, int ex2, Best &b,
                                           Counters &K) {
    if (pos < end) K.evals += (uint32_t)((end - pos + W - 1) / W);
    const float2 *q = sxy + pos;   // one pointer for both loads of a trip
    for (; pos + W < end; pos += 2 * W, q += 2 * W) {
        const float2 a0 = q[0], a1 = q[W];
        eval_at(C, a0, pos, dx, dy, ex1, ex2, b);
        eval_at(C, a1, pos + W, dx, dy, ex1, ex2, b);
    }
    if (pos < end) eval_at(C, q[0], pos, dx, dy, ex1, ex2, b);
}

// Row ranges of the cell's warm-start block (up to MAXROWS rows, h <= 2), loaded once per
// cell.  LdsRows keeps them in a per-thread column of LDS (the filtered pass);
// GlobalRows reads them from the bucket starts each time.  load() returns the longest row.
constexpr int MAXROWS = 5;

template <int BLOCK>
struct LdsRows {
    int (*lo)[BLOCK];
    int (*hi)[BLOCK];
    int nrows;
    __device__ __forceinline__ int load(const Cell &C, const int *__restrict__ bstart) {
        const Rect A = block_rect(C);
        nrows = A.y1 - A.y0 + 1;
        if (nrows > MAXROWS) return 0;
        int longest = 0;
        for (int i = 0; i < nrows; ++i) {
            const int base = C.boff + (A.y0 + i) * C.gx;
            const int a = bstart[base + A.x0], b = bstart[base + A.x1 + 1];
            lo[i][threadIdx.x] = a;
            hi[i][threadIdx.x] = b;
            longest = max(longest, b - a);
        }
        return longest;
    }
    __device__ __forceinline__ void get(const Cell &, const int *__restrict__, int r, int &a,
                                        int &b) const {
        a = lo[r][threadIdx.x];
        b = hi[r][threadIdx.x];
    }
};

struct GlobalRows {
    int nrows;
    __device__ __forceinline__ int load(const Cell &C, const int *__restrict__) {
        const Rect A = block_rect(C);
        nrows = A.y1 - A.y0 + 1;
        return 0;
    }
    __device__ __forceinline__ void get(const Cell &C, const int *__restrict__ bstart, int r,
                                        int &a, int &b) const {
        const Rect A = block_rect(C);
        const int base = C.boff + (A.y0 + r) * C.gx;
        a = bstart[base + A.x0];
        b = bstart[base + A.x1 + 1];
    }
};

// Candidates of rectangle O \ I, one flat loop per lane (a lane pays only for its own
// candidates); with the Coop policy lane i takes every 64th candidate of each row.  With
// DETECT a row segment longer than SEG_HEAVY stops the walk and sets `heavy`.
// With the Coop policy the rows are spread over lane groups: segment s of O \ I is the left
// (s even) or right (s odd) part of row O.y0 + s/2 (a row that misses I is whole in its left
// part); COOP_G lanes share a segment, so a pass costs one round of row loads and one of site
// loads instead of one per row.  A round that holds a long segment (a crowded bucket) is
// scanned segment by segment with all lanes instead.
constexpr int COOP_G = 8;
constexpr int COOP_LONG = 4 * COOP_G;
__device__ __forceinline__ void coop_segment(const Cell &C, const int *__restrict__ bstart,
                                             const Rect &O, const Rect &I, int s, int &a,
                                             int &e) {
    a = e = 0;
    const int row = O.y0 + (s >> 1);
    if (row > O.y1) return;
    int xa = O.x0, xb = O.x1;
    if (row >= I.y0 && row <= I.y1) {
        if (s & 1) xa = max(O.x0, I.x1 + 1);
        else xb = min(O.x1, I.x0 - 1);
    } else if (s & 1) {
        return;
    }
    if (xa > xb) return;
    const int base = C.boff + row * C.gx;
    a = bstart[base + xa];
    e = bstart[base + xb + 1];
}

template <class P, bool DETECT>
__device__ __forceinline__ void scan_rect_f32(const Cell &C, const float2 *__restrict__ sxy,
                                              const int *__restrict__ bstart, Rect O, Rect I,
                                              float dx, float dy, int ex1, int ex2, Best &b,
                                              Counters &K, bool &heavy) {
    if constexpr (P::W > 1) {
        const int grp = P::lane() / COOP_G, sub = P::lane() % COOP_G;
        const int nseg = 2 * (O.y1 - O.y0 + 1);
        for (int s0 = 0; s0 < nseg; s0 += P::W / COOP_G) {
            int a, e;
            coop_segment(C, bstart, O, I, s0 + grp, a, e);
            if (__any(e - a > COOP_LONG)) {
                for (int g = 0; g < P::W / COOP_G; ++g) {
                    const int ga = __shfl(a, g * COOP_G, 64), ge = __shfl(e, g * COOP_G, 64);
                    eval_range<P::W>(C, sxy, ga + P::lane(), ge, dx, dy, ex1, ex2, b, K);
                }
            } else {
                eval_range<COOP_G>(C, sxy, a + sub, e, dx, dy, ex1, ex2, b, K);
            }
        }
        return;
    }
    RowWalk wk;
    wk.start(O, I);
    while (wk.next(C, bstart)) {
        if (DETECT && wk.end - wk.pos > SEG_HEAVY) {
            heavy = true;
            break;
        }
        eval_range<P::W>(C, sxy, wk.pos + P::lane(), wk.end, dx, dy, ex1, ex2, b, K);
    }
}

// Exact argmin over rectangle O \ I.  With FILTER only candidates whose FP32 lower bound is
// <= Tlim count.
template <bool FILTER, class P>
__device__ __forceinline__ void exact_site(const Cell &C, float2 a, int q, const Dir &d,
                                           float lim, XBest &b, Counters &K) {
    const float ex = a.x - C.pxf, ey = a.y - C.pyf;
    if (FILTER && !(key_lo_line(site_q(ex, ey), ex, ey, d.fx, d.fy) * CERT_DN <= lim)) return;
    if (!FILTER) ++K.evals;
    const int nx = (int)a.x - C.px, ny = (int)a.y - C.py;
    if ((nx | ny) == 0) return;   // p itself
    x_consider(b, q, nx, ny, (int64_t)nx * nx + (int64_t)ny * ny, d);
}

template <bool FILTER, class P>
__device__ __forceinline__ void exact_rect(const Cell &C, const float2 *__restrict__ sxy,
                                           const int *__restrict__ bstart, const Dir &d, Rect O,
                                           Rect I, float Tlim, int ex1, int ex2, XBest &b,
                                           Counters &K) {
    const float lim = Tlim * CERT_UP;
    if constexpr (P::W > 1) {
        const int grp = P::lane() / COOP_G, sub = P::lane() % COOP_G;
        const int nseg = 2 * (O.y1 - O.y0 + 1);
        for (int s0 = 0; s0 < nseg; s0 += P::W / COOP_G) {
            int a, e;
            coop_segment(C, bstart, O, I, s0 + grp, a, e);
            if (__any(e - a > COOP_LONG)) {
                for (int g = 0; g < P::W / COOP_G; ++g) {
                    const int ga = __shfl(a, g * COOP_G, 64), ge = __shfl(e, g * COOP_G, 64);
                    for (int q = ga + P::lane(); q < ge; q += P::W) {
                        if (q == ex1 || q == ex2) continue;
                        exact_site<FILTER, P>(C, sxy[q], q, d, lim, b, K);
                    }
                }
            } else {
                for (int q = a + sub; q < e; q += COOP_G) {
                    if (q == ex1 || q == ex2) continue;
                    exact_site<FILTER, P>(C, sxy[q], q, d, lim, b, K);
                }
            }
        }
        return;
    }
    RowWalk wk;
    wk.start(O, I);
    int pos = 0, end = 0;
    for (;;) {
        if (pos < end) {
            const int q = pos;
            pos += P::W;
            if (q == ex1 || q == ex2) continue;
            exact_site<FILTER, P>(C, sxy[q], q, d, lim, b, K);
            continue;
        }
        if (!wk.next(C, bstart)) break;
        pos = wk.pos + P::lane();
        end = wk.end;
    }
}

__device__ __forceinline__ void exact_sides(const Cell &C, const Dir &d, float Tlim, bool filter,
                                            int ex1, int ex2, XBest &b) {
    const float lim = Tlim * CERT_UP;
    const int ns = C.ns > 0 ? C.ns : 4;
    for (int code = -1; code >= -ns; --code) {
        if (code == ex1 || code == ex2) continue;
        const Line L = side_line(C, code);
        if (filter &&
            !(key_lo_line((float)L.c, (float)L.nx, (float)L.ny, d.fx, d.fy) * CERT_DN <= lim))
            continue;
        x_consider(b, code, L.nx, L.ny, L.c, d);
    }
}

// ------------------------------------------------------------------------------ scanners
// A scanner answers the three questions a ray asks: the FP32 argmin over a certified region
// (scan), the exact argmin over the region a scan certified (exact), and the exact argmin with
// its own certification (exact_all, every decision exact).

// The first-pass summaries of the three corner rays (one lane per cell): the rays have fixed
// directions and scan the same block, so one pass over the block evaluates every candidate for
// all three (sharing its load, offset and q).  LdsCorners keeps the summaries in nine LDS
// columns that are free during the corner phase -- the top of the cell's stack, which stays
// empty until the third corner ray has returned; NoCorners: every ray scans on its own.
struct NoCorners {
    static constexpr bool ON = false;
    __device__ __forceinline__ void put(int, const Best &) {}
    __device__ __forceinline__ Best get(int) const { return Best{FINF, FINF, NO_TAG}; }
};
template <int BLOCK>
struct LdsCorners {
    static constexpr bool ON = true;
    int (*s)[BLOCK];   // nine rows
    __device__ __forceinline__ void put(int c, const Best &b) {
        s[3 * c][threadIdx.x] = __float_as_int(b.k1);
        s[3 * c + 1][threadIdx.x] = __float_as_int(b.k2);
        s[3 * c + 2][threadIdx.x] = b.w;
    }
    __device__ __forceinline__ Best get(int c) const {
        return Best{__int_as_float(s[3 * c][threadIdx.x]), __int_as_float(s[3 * c + 1][threadIdx.x]),
                    s[3 * c + 2][threadIdx.x]};
    }
};

// Uniform bucket grid: regions are rectangles of buckets, rows are contiguous ranges.
template <class P, class Rows, bool DETECT, class CS = NoCorners>
struct GridScan {
    Rows BR;
    const int *bstart;
    bool heavy;
    CS cs;
    int pre_n = -1;   // candidates of the corner pass (-1: none)

    __device__ __forceinline__ void load(const Cell &C, const float2 *__restrict__ sxy) {
        const int longest = BR.load(C, bstart);
        heavy = DETECT && longest > SEG_HEAVY;
        if (CS::ON && P::W == 1 && !heavy && BR.nrows <= MAXROWS) corners(C, sxy);
    }

    // The corner rays' pass over the block (no lines are excluded for them).
    __device__ __forceinline__ void corners(const Cell &C, const float2 *__restrict__ sxy) {
        const Dir d0 = corner_dir(0), d1 = corner_dir(1), d2 = corner_dir(2);
        Best b0{FINF, FINF, NO_TAG}, b1 = b0, b2 = b0;
        int n = 0;
        for (int r = 0; r < BR.nrows; ++r) {
            int pos, end;
            BR.get(C, bstart, r, pos, end);
            n += end - pos;
            for (; pos < end; ++pos) {
                const float2 a = sxy[pos];
                const float ex = a.x - C.pxf, ey = a.y - C.pyf;
                const float q = site_q_scan(ex, ey);
                consider(key_lo_scan_q(q, ex, ey, d0.fx, d0.fy), pos, b0);
                consider(key_lo_scan_q(q, ex, ey, d1.fx, d1.fy), pos, b1);
                consider(key_lo_scan_q(q, ex, ey, d2.fx, d2.fy), pos, b2);
            }
        }
        cs.put(0, b0);
        cs.put(1, b1);
        cs.put(2, b2);
        pre_n = n;
    }

    // FP32 argmin (Method 11.6): the cell's block of shells 0..h (a warm start that bounds the
    // endpoint by y), then while the integer rectangle S_I[y, |y - p|] of the bound is not
    // inside the scanned rectangle, grow the scanned rectangle towards it (at most doubling per
    // step); the rectangles of later, nearer bounds nest inside the earlier ones, so the final
    // scanned rectangle certifies the endpoint.
    // corner: the corner ray's index (0..2) in the walk's first three steps, else -1.
    __device__ __forceinline__ ScanOut scan(const Cell &C, const float2 *__restrict__ sxy,
                                            float dx, float dy, int ex1, int ex2, float tcap,
                                            Counters &K, int corner = -1) {
        Best b{FINF, FINF, NO_TAG};
        const Rect A = block_rect(C);
        // A vertex ray (tcap bounds its endpoint) starts from its own rectangle S_I when that
        // lies in the block: the rectangles of smaller bounds nest inside it, so the scan
        // never grows, and the block's other sites are farther from the target than p.
        const Rect O0 = first_rect(C, A, tcap, dx, dy);
        if (CS::ON && corner >= 0 && pre_n >= 0) {
            b = cs.get(corner);   // the block, from the corner pass (O0 = A: no bound)
            K.evals += (uint32_t)pre_n;
        } else if (P::W == 1 && BR.nrows <= MAXROWS) {
            for (int y = O0.y0; y <= O0.y1; ++y) {
                int pos, end;
                BR.get(C, bstart, y - A.y0, pos, end);
                const int base = C.boff + y * C.gx;
                if (O0.x0 != A.x0) pos = bstart[base + O0.x0];
                if (O0.x1 != A.x1) end = bstart[base + O0.x1 + 1];
                eval_range<P::W>(C, sxy, pos + P::lane(), end, dx, dy, ex1, ex2, b, K);
            }
        } else {
            scan_rect_f32<P, DETECT>(C, sxy, bstart, O0, Rect{1, 0, 1, 0}, dx, dy, ex1, ex2, b,
                                     K, heavy);
        }
        P::reduce(b);
        consider_sides(C, dx, dy, ex1, ex2, b);
        K.shells++;
        float U = upper_of(C, sxy, b.w, dx, dy);
        float Uw = U;
        Rect R = need_rect(C, fminf(U, tcap), dx, dy);
        Rect O = O0;
        while (!(DETECT && heavy) && !rect_inside(R, O)) {
            const Rect N = grow_rect(O, R);
            scan_rect_f32<P, DETECT>(C, sxy, bstart, N, O, dx, dy, ex1, ex2, b, K, heavy);
            P::reduce(b);
            O = N;
            K.shells++;
            Uw = upper_of(C, sxy, b.w, dx, dy);
            U = fminf(U, Uw);
            R = need_rect(C, fminf(U, tcap), dx, dy);
        }
        ScanOut o;
        o.b = b;
        o.Uw = Uw;
        o.U = U;
        o.Tr = fminf(U, tcap);
        o.A = O;
        return o;
    }

    __device__ __forceinline__ void exact(const Cell &C, const float2 *__restrict__ sxy,
                                          const Dir &d, const ScanOut &s, float Tlim, int ex1,
                                          int ex2, XBest &xb, Counters &K) {
        exact_rect<true, P>(C, sxy, bstart, d, s.A, Rect{1, 0, 1, 0}, Tlim, ex1, ex2, xb, K);
        P::reduce(xb);
        exact_sides(C, d, Tlim, true, ex1, ex2, xb);
    }

    __device__ __forceinline__ void exact_all(const Cell &C, const float2 *__restrict__ sxy,
                                              const Dir &d, float tu_hi, int ex1, int ex2,
                                              XBest &xb, Counters &K) {
        const Rect A = first_rect(C, block_rect(C), tu_hi, d.fx, d.fy);
        exact_rect<false, P>(C, sxy, bstart, d, A, Rect{1, 0, 1, 0}, FINF, ex1, ex2, xb, K);
        P::reduce(xb);
        exact_sides(C, d, FINF, false, ex1, ex2, xb);
        Rect O = A;
        K.shells++;
        Rect R = need_rect(C, fminf(x_upper(xb, d), tu_hi), d.fx, d.fy);
        while (!rect_inside(R, O)) {
            const Rect N = grow_rect(O, R);
            exact_rect<false, P>(C, sxy, bstart, d, N, O, FINF, ex1, ex2, xb, K);
            P::reduce(xb);
            O = N;
            K.shells++;
            R = need_rect(C, fminf(x_upper(xb, d), tu_hi), d.fx, d.fy);
        }
    }
};

// Per-cell candidate cache of the coordinate-rectangle scan: the sorted positions of every site
// in a region G around p, gathered once and grown on demand, so that a ray whose S_I square
// fits in G is answered by one flat pass over the list instead of a walk of the tree.
struct NoList {
    static constexpr int K = 0;
    __device__ __forceinline__ void put(int, int) {}
    __device__ __forceinline__ int get(int) const { return 0; }
};
template <int BLOCK, int KC>
struct LdsList {
    static constexpr int K = KC;
    int (*l)[BLOCK];
    __device__ __forceinline__ void put(int i, int v) { l[i][threadIdx.x] = v; }
    __device__ __forceinline__ int get(int i) const { return l[i][threadIdx.x]; }
};
// The same list in global memory, one column per thread (entry i at base[i * stride]): the
// adaptive pass keeps its LDS for the stack and the walk frames, so more waves fit on a CU.
template <int KC>
struct GlobalList {
    static constexpr int K = KC;
    int *base;
    int stride;
    __device__ __forceinline__ void put(int i, int v) { base[i * stride] = v; }
    __device__ __forceinline__ int get(int i) const { return base[i * stride]; }
};

// Adaptive buckets: regions are rectangles in coordinates; a pass over N \ O visits the leaves
// that meet it (and the disk of the current bound) and evaluates exactly the sites inside N and
// outside O.  With a list (LS::K > 0, one lane per cell) the sites of the growing region G are
// kept and later rays start from them.
template <class P, class FS, class LS = NoList>
struct TreeScan {
    Tree T;
    FS fs;
    LS ls;
    Rect Q0;
    bool heavy;
    Rect G;      // region whose sites are all in the list (while cached)
    int nl;      // sites in the list (may exceed LS::K: overflow)
    bool cached;
    int work;    // sub-buckets visited + evaluations for this cell (lane-per-cell scans)
    unsigned long long t0;   // when the lane started the cell (100 MHz clock)
    const int *done = nullptr;   // workgroups of the pass that have finished their cells
    int tail = 0;                // from this many on, the pass is in its tail

    // In the pass's tail, a lane that has spent TREE_TICKS on its cell hands it on: the walk's
    // steps are chains of dependent loads, so a cell near a cluster can hold its lane for
    // milliseconds within its work budget while the rest of the GPU idles.  Before the tail the
    // lanes share the GPU and their clocks say little.  The cell's result does not depend on
    // which pass computes it.
    __device__ __forceinline__ bool over_time() const {
        return done && wall_clock64() - t0 > TREE_TICKS &&
               __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= tail;
    }

    // Appends the sites of N \ O to the list; false (and the list as before) on overflow.
    __device__ __forceinline__ bool gather(const Cell &C, const float2 *__restrict__ sxy, Rect N,
                                           Rect O) {
        const int n0 = nl;
        TreeWalk wk;
        const Disk all{0.0f, 0.0f, FINF};
        wk.start(C, T, N, O, all);
        while (wk.next(C, T, fs)) {
            if (wk.full) {
                if (nl + (wk.end - wk.pos) > LS::K) {
                    nl = n0;
                    return false;
                }
                for (int q = wk.pos; q < wk.end; ++q) ls.put(nl++, q);
                continue;
            }
            for (int q0 = wk.pos; q0 < wk.end; q0 += TREE_BATCH) {
                float2 a[TREE_BATCH];
#pragma unroll
                for (int u = 0; u < TREE_BATCH; ++u)
                    a[u] = q0 + u < wk.end ? sxy[q0 + u] : make_float2(-1.0f, -1.0f);
#pragma unroll
                for (int u = 0; u < TREE_BATCH; ++u) {
                    if (q0 + u >= wk.end) break;
                    if (!(in_rect(N, a[u].x, a[u].y) && !in_rect(O, a[u].x, a[u].y))) continue;
                    if (nl >= LS::K) {
                        nl = n0;
                        return false;
                    }
                    ls.put(nl++, q0 + u);
                }
            }
        }
        return true;
    }

    // The list starts with p's leaf and grows by one leaf side per step while it holds fewer
    // than TREE_LIST_FILL sites and the next ring fits.
    __device__ __forceinline__ void load(const Cell &C, const float2 *__restrict__ sxy) {
        Q0 = tree_block(C, T, C.ht);
        heavy = false;
        work = 0;
        if (LS::K > 0) t0 = wall_clock64();
        if (LS::K > 0) {
            G = tree_block(C, T, 0);
            nl = 0;
            cached = gather(C, sxy, G, NO_RECT);
            const int side = G.x1 - G.x0 + 1;
            for (int ring = 0; cached && nl < TREE_LIST_FILL && ring < 4; ++ring) {
                const Rect N{max(G.x0 - side, 0), min(G.x1 + side, C.W), max(G.y0 - side, 0),
                             min(G.y1 + side, C.H)};
                if (rect_inside(N, G) || !gather(C, sxy, N, G)) break;
                G = N;
            }
        }
    }

    // Sites of N \ O.  CACHE: every such site is evaluated and appended to the list (no disk
    // pruning, the list must hold the whole region) until it is full (then nl > LS::K).
    // Otherwise sites and leaves outside the disk of the bound Tr are skipped, and the disk
    // shrinks whenever a new winner lowers the bound (Tr = min(Tr, its upper key), capped by
    // tcap): a site outside the disk of an evaluated site's upper bound is strictly worse.
    template <bool CACHE>
    __device__ __forceinline__ void visit_f32(const Cell &C, const float2 *__restrict__ sxy,
                                              Rect N, Rect O, float &Tr, float tcap, float dx,
                                              float dy, int ex1, int ex2, Best &b, Counters &K) {
        TreeWalk wk;
        const Disk all{0.0f, 0.0f, FINF};
        wk.start(C, T, N, O, CACHE ? all : need_disk(C, Tr, dx, dy));
        int pos = 0, end = 0, ev = 0;
        bool full = true;
        for (;;) {
            if (LS::K > 0 && work + wk.steps + ev > TREE_BUDGET) {
                heavy = true;   // the lane gives the cell to the one-wave-per-cell pass
                break;
            }
            if (pos < end) {
                float2 a[TREE_BATCH];
#pragma unroll
                for (int u = 0; u < TREE_BATCH; ++u) {
                    const int q = pos + u * P::W;
                    a[u] = q < end ? sxy[q] : make_float2(-1.0f, -1.0f);
                }
#pragma unroll
                for (int u = 0; u < TREE_BATCH; ++u) {
                    const int q = pos + u * P::W;
                    if (q >= end) break;
                    ++ev;
                    if (!full && !(in_rect(N, a[u].x, a[u].y) && !in_rect(O, a[u].x, a[u].y)))
                        continue;
                    const float ex = a[u].x - C.pxf, ey = a[u].y - C.pyf;
                    if (CACHE) {
                        if (nl < LS::K) ls.put(nl, q);
                        ++nl;
                    } else if (!in_disk(wk.D, ex, ey)) {
                        continue;
                    }
                    const float qq = site_q(ex, ey);
                    float key = key_lo_line(qq, ex, ey, dx, dy);
                    key = (q == ex1 || q == ex2) ? FINF : key;
                    const bool win = key < b.k1;
                    consider_once(key, q, b);
                    ++K.evals;
                    if (!CACHE && P::W == 1 && win) {
                        const float t = fminf(key_hi_line(qq, ex, ey, dx, dy), tcap);
                        if (t < Tr) {
                            Tr = t;
                            wk.D = need_disk(C, Tr, dx, dy);
                        }
                    }
                }
                pos += TREE_BATCH * P::W;
                continue;
            }
            if (LS::K > 0 && over_time()) {
                heavy = true;
                break;
            }
            if (!wk.next(C, T, fs)) break;
            pos = wk.pos + P::lane();
            end = wk.end;
            full = wk.full;
        }
        work += wk.steps + ev;
    }

    // Probes the leaves at the points p + (Tr 2^-k / 2) d_s, k = 1..TREE_PROBES, of the ray: a
    // bound found far out along a ray that enters a denser region tightens quickly, so the
    // region pass that follows prunes most of that region.  Any candidates are valid here.
    __device__ __forceinline__ void probe(const Cell &C, const float2 *__restrict__ sxy,
                                          float dx, float dy, int ex1, int ex2, float Tr,
                                          Best &b, Counters &K) {
        if (!(Tr < 1.0e30f)) return;
        float t = Tr;
        for (int k = 0; k < TREE_PROBES; ++k) {
            t *= 0.5f;
            const int x = C.px + (int)fminf(fmaxf(0.5f * t * dx, -(float)C.W), (float)C.W);
            const int y = C.py + (int)fminf(fmaxf(0.5f * t * dy, -(float)C.H), (float)C.H);
            if (x < 0 || x >= C.W || y < 0 || y >= C.H) continue;
            int lo, hi;
            leaf_at(C, T, x, y, lo, hi);
            for (int q0 = lo + P::lane(); q0 < hi; q0 += TREE_BATCH * P::W) {
                float2 a[TREE_BATCH];
#pragma unroll
                for (int u = 0; u < TREE_BATCH; ++u) {
                    const int q = q0 + u * P::W;
                    a[u] = q < hi ? sxy[q] : make_float2(-1.0f, -1.0f);
                }
#pragma unroll
                for (int u = 0; u < TREE_BATCH; ++u) {
                    const int q = q0 + u * P::W;
                    if (q >= hi) break;
                    const float ex = a[u].x - C.pxf, ey = a[u].y - C.pyf;
                    float key = key_lo_line(site_q(ex, ey), ex, ey, dx, dy);
                    key = (q == ex1 || q == ex2 || (ex == 0.0f && ey == 0.0f)) ? FINF : key;
                    consider_once(key, q, b);
                    ++K.evals;
                }
            }
            work += hi - lo + 4;
        }
        P::reduce(b);
    }

    // FP32 argmin starting from the cached list: its region G replaces the warm start.
    __device__ __forceinline__ ScanOut scan_cached(const Cell &C, const float2 *__restrict__ sxy,
                                                   float dx, float dy, int ex1, int ex2,
                                                   float tcap, Counters &K) {
        Best b{FINF, FINF, NO_TAG};
        for (int i0 = 0; i0 < nl; i0 += TREE_BATCH) {
            int q[TREE_BATCH];
            float2 a[TREE_BATCH];
#pragma unroll
            for (int u = 0; u < TREE_BATCH; ++u) q[u] = i0 + u < nl ? ls.get(i0 + u) : -1;
#pragma unroll
            for (int u = 0; u < TREE_BATCH; ++u)
                a[u] = q[u] >= 0 ? sxy[q[u]] : make_float2(-1.0f, -1.0f);
#pragma unroll
            for (int u = 0; u < TREE_BATCH; ++u) {
                if (q[u] < 0) break;
                const float ex = a[u].x - C.pxf, ey = a[u].y - C.pyf;
                float key = key_lo_line(site_q(ex, ey), ex, ey, dx, dy);
                key = (q[u] == ex1 || q[u] == ex2) ? FINF : key;
                consider(key, q[u], b);
            }
        }
        K.evals += nl;
        work += nl;
        consider_sides(C, dx, dy, ex1, ex2, b);
        K.shells++;
        float U = upper_of(C, sxy, b.w, dx, dy);
        float Uw = U;
        float Tr = fminf(U, tcap);
        Rect R = need_crect(C, Tr, dx, dy);
        Rect O = G;
        bool grow = true;   // O is still the list's region: the list may follow it
        if (!rect_inside(R, O)) {
            probe(C, sxy, dx, dy, ex1, ex2, Tr, b, K);
            Uw = upper_of(C, sxy, b.w, dx, dy);
            U = fminf(U, Uw);
            Tr = fminf(U, tcap);
            R = need_crect(C, Tr, dx, dy);
        }
        while (!heavy && !rect_inside(R, O)) {
            const Rect N = grow_crect(O, R);
            if (grow) {
                const int n0 = nl;
                float Tn = FINF;
                visit_f32<true>(C, sxy, N, O, Tn, tcap, dx, dy, ex1, ex2, b, K);
                if (nl <= LS::K) {
                    G = N;
                } else {
                    nl = n0;   // full: the list keeps region G, this ray goes on without it
                    grow = false;
                }
            } else {
                float Tv = Tr;
                visit_f32<false>(C, sxy, N, O, Tv, tcap, dx, dy, ex1, ex2, b, K);
            }
            O = N;
            K.shells++;
            Uw = upper_of(C, sxy, b.w, dx, dy);
            U = fminf(U, Uw);
            Tr = fminf(U, tcap);
            R = need_crect(C, Tr, dx, dy);
        }
        ScanOut o;
        o.b = b;
        o.Uw = Uw;
        o.U = U;
        o.Tr = Tr;
        o.A = O;
        return o;
    }

    __device__ __forceinline__ ScanOut scan(const Cell &C, const float2 *__restrict__ sxy,
                                            float dx, float dy, int ex1, int ex2, float tcap,
                                            Counters &K, int = -1) {
        if (LS::K > 0 && cached) return scan_cached(C, sxy, dx, dy, ex1, ex2, tcap, K);
        Best b{FINF, FINF, NO_TAG};
        float T0 = tcap;   // a vertex ray skips the sites outside the disk of its bound
        visit_f32<false>(C, sxy, Q0, NO_RECT, T0, tcap, dx, dy, ex1, ex2, b, K);
        P::reduce(b);
        consider_sides(C, dx, dy, ex1, ex2, b);
        K.shells++;
        float U = upper_of(C, sxy, b.w, dx, dy);
        float Uw = U;
        float Tr = fminf(U, tcap);
        Rect R = need_crect(C, Tr, dx, dy);
        Rect O = Q0;
        if (!rect_inside(R, O)) {
            probe(C, sxy, dx, dy, ex1, ex2, Tr, b, K);
            Uw = upper_of(C, sxy, b.w, dx, dy);
            U = fminf(U, Uw);
            Tr = fminf(U, tcap);
            R = need_crect(C, Tr, dx, dy);
        }
        while (!heavy && !rect_inside(R, O)) {
            const Rect N = grow_crect(O, R);
            float Tv = Tr;
            visit_f32<false>(C, sxy, N, O, Tv, tcap, dx, dy, ex1, ex2, b, K);
            P::reduce(b);
            O = N;
            K.shells++;
            Uw = upper_of(C, sxy, b.w, dx, dy);
            U = fminf(U, Uw);
            Tr = fminf(U, tcap);
            R = need_crect(C, Tr, dx, dy);
        }
        ScanOut o;
        o.b = b;
        o.Uw = Uw;
        o.U = U;
        o.Tr = Tr;
        o.A = O;
        return o;
    }

    template <bool FILTER>
    __device__ __forceinline__ void visit_exact(const Cell &C, const float2 *__restrict__ sxy,
                                                const Dir &d, Rect N, Rect O, const Disk &Dk,
                                                float Tlim, int ex1, int ex2, XBest &xb,
                                                Counters &K) {
        const float lim = Tlim * CERT_UP;
        TreeWalk wk;
        wk.start(C, T, N, O, Dk);
        int pos = 0, end = 0, ev = 0;
        bool full = true;
        for (;;) {
            // the lane-per-cell scans keep to the cell's work budget here too: a disk that
            // holds a cluster would keep one lane busy long after the others
            if (LS::K > 0 && work + wk.steps + ev > TREE_BUDGET) {
                heavy = true;
                break;
            }
            if (pos < end) {
                const int q = pos;
                pos += P::W;
                ++ev;
                if (q == ex1 || q == ex2) continue;
                const float2 a = sxy[q];
                if (!full && !(in_rect(N, a.x, a.y) && !in_rect(O, a.x, a.y))) continue;
                if (!in_disk(Dk, a.x - C.pxf, a.y - C.pyf)) continue;
                exact_site<FILTER, P>(C, a, q, d, lim, xb, K);
                continue;
            }
            if (LS::K > 0 && over_time()) {
                heavy = true;
                break;
            }
            if (!wk.next(C, T, fs)) break;
            pos = wk.pos + P::lane();
            end = wk.end;
            full = wk.full;
        }
        work += wk.steps + ev;
    }

    __device__ __forceinline__ void exact(const Cell &C, const float2 *__restrict__ sxy,
                                          const Dir &d, const ScanOut &s, float Tlim, int ex1,
                                          int ex2, XBest &xb, Counters &K) {
        visit_exact<true>(C, sxy, d, s.A, NO_RECT, need_disk(C, s.Tr, d.fx, d.fy), Tlim, ex1,
                          ex2, xb, K);
        P::reduce(xb);
        exact_sides(C, d, Tlim, true, ex1, ex2, xb);
    }

    __device__ __forceinline__ void exact_all(const Cell &C, const float2 *__restrict__ sxy,
                                              const Dir &d, float tu_hi, int ex1, int ex2,
                                              XBest &xb, Counters &K) {
        visit_exact<false>(C, sxy, d, Q0, NO_RECT, need_disk(C, tu_hi, d.fx, d.fy), FINF, ex1,
                           ex2, xb, K);
        P::reduce(xb);
        exact_sides(C, d, FINF, false, ex1, ex2, xb);
        Rect O = Q0;
        K.shells++;
        float Tr = fminf(x_upper(xb, d), tu_hi);
        Rect R = need_crect(C, Tr, d.fx, d.fy);
        while (!rect_inside(R, O)) {
            const Rect N = grow_crect(O, R);
            visit_exact<false>(C, sxy, d, N, O, need_disk(C, Tr, d.fx, d.fy), FINF, ex1, ex2, xb,
                               K);
            P::reduce(xb);
            O = N;
            K.shells++;
            Tr = fminf(x_upper(xb, d), tu_hi);
            R = need_crect(C, Tr, d.fx, d.fy);
        }
    }
};

// ------------------------------------------------------------------------------ stacks / outputs
template <int BLOCK>
struct LdsStack {
    int (*s)[BLOCK];
    int depth;
    __device__ __forceinline__ void push(int v) { s[depth++][threadIdx.x] = v; }
    __device__ __forceinline__ int top() const { return s[depth - 1][threadIdx.x]; }
    __device__ __forceinline__ int pop() { return s[--depth][threadIdx.x]; }
};

// Stack shared by the lanes of a wave (LDS or global memory); with the Coop policy every lane
// writes the same value to the same address.
struct GStack {
    int *s;
    int depth;
    __device__ __forceinline__ void push(int v) { s[depth++] = v; }
    __device__ __forceinline__ int top() const { return s[depth - 1]; }
    __device__ __forceinline__ int pop() { return s[--depth]; }
};

// Output of a cell walk: the lines as sorted positions (side codes unchanged), entry m at
// dst[m * stride] (the filtered passes store entry-major by the cell's own sorted position, so
// that the rows a wavefront writes are complete in L2 before they are written back), plus the
// count of neighbours with a larger id than the cell's own (k), i.e. the cell's Delaunay edges
// (i, j), i < j (Section 7).
struct Sink {
    int *dst;
    long long stride;
    const int *sid;
    int k;
    int up = 0;
    int lastup = 0;
    __device__ __forceinline__ void put(int m, int id) {
        dst[m * stride] = id;
        const int v = id >= 0 ? sid[id] : id;
        lastup = v > k;
        up += lastup;
    }
    // the last line closed the cycle (it is the first line again): not a new neighbour
    __device__ __forceinline__ void drop_last() { up -= lastup; }
};

// Output of a cell walk as sorted positions and side codes (the lines' own names, for a pass
// that still works on the lines before converting them).
struct PosSink {
    int *dst;
    __device__ __forceinline__ void put(int m, int id) { dst[m] = id; }
    __device__ __forceinline__ void drop_last() {}
};

// ------------------------------------------------------------------------------ ray shots
// MODE 0: FP32 filter, give up (defer the cell) when a decision is not certified.
// MODE 1: FP32 filter, exact decision when not certified.
// MODE 2: exact arithmetic for every decision.
//
// Plain ray (Den == 0): out = the line the endpoint lies on; returns 0.
// Vertex ray (Den > 0, d = Z, u = Z / Den; lines ex1, ex2 through u skipped): returns 1 when u
// is in the cell (a vertex), 0 when a line crosses [p, u) first (that line in out).
// Returns -1 when undecided (MODE 0), -4 when the scanner met a heavy bucket.
template <int MODE, class P, class Sc>
__device__ __forceinline__ int ray(const Cell &C, Sc &sc, const float2 *__restrict__ sxy,
                                   const Dir &d, int64_t Den, int ex1, int ex2, Line &out,
                                   Counters &K, int corner = -1) {
    const bool vmode = Den > 0;
    float tu_hi = FINF, tu_lo = FINF;
    if (vmode) {
        // t_u = 2^sigma / Den: Den rounds to FP32 with relative error <= u and v_rcp_f32 adds
        // <= 2 ulp, both far inside the 2^-19 margins
        const float tu = ldexpf(__builtin_amdgcn_rcpf((float)Den), d.sigma);
        tu_hi = tu * CERT_UP;
        tu_lo = tu * CERT_DN;
    }
    XBest xb;
    xb.have = false;
    if (MODE == 2) {
        sc.exact_all(C, sxy, d, tu_hi, ex1, ex2, xb, K);
    } else {
        // one scan variant for both kinds of rays (lanes of a wave may differ in kind)
        const ScanOut s = sc.scan(C, sxy, d.fx, d.fy, ex1, ex2, vmode ? tu_hi : FINF, K, corner);
        if (sc.heavy) return -4;
        if (vmode && s.b.k1 * CERT_DN > tu_hi) return 1;
        const float uw = s.Uw * CERT_UP;
        if (uw < s.b.k2 * CERT_DN && (!vmode || uw < tu_lo)) {
            out = make_line(C, sxy, s.b.w);
            return 0;
        }
        if (MODE == 0) return -1;
        K.exact++;
        K.xinc += vmode;
        // exact decision over the certified region, FP32-plausible candidates only
        sc.exact(C, sxy, d, s, vmode ? tu_hi : s.U, ex1, ex2, xb, K);
        if (sc.heavy) return -4;   // over the lane's work budget (tree scans)
    }
    // no line other than the two through u is crossed: u is the endpoint (a vertex)
    if (!xb.have) return vmode ? 1 : -1;
    // u is outside the cell iff some line is crossed before it: c_b / den_b < 1 / Den
    if (!vmode || (u128)xb.c * (u128)Den < xb.den) {
        out.id = xb.id;
        out.nx = xb.nx;
        out.ny = xb.ny;
        out.c = (int64_t)xb.c;
        return 0;
    }
    return 1;
}

// ------------------------------------------------------------------------------ one subedge
// The ray that resolves the subedge from the corner on line L1 to the next corner (counter-
// clockwise) on line L2, L1 != L2 (Algorithm 1): Den = cross(N1, N2); Den = 0: the lines are
// antiparallel and the ray runs along them (ParallelLines); otherwise u = L1 ∩ L2 = Z / Den and
// the ray runs along Z (towards u for Den > 0, the Vertex / OutsideCell test, which skips the
// two lines through u; away from it for Den < 0, OutsideWedge).
__device__ __forceinline__ void split_dir(const Line &L1, const Line &L2, Dir &d, int64_t &Den,
                                          int &ex1, int &ex2) {
    Den = (int64_t)L1.nx * L2.ny - (int64_t)L1.ny * L2.nx;
    if (Den == 0) {
        d = make_dir(-(i128)L1.ny, (i128)L1.nx);
    } else {
        const i128 Zx = (i128)L1.c * L2.ny - (i128)L2.c * L1.ny;
        const i128 Zy = (i128)L1.nx * L2.c - (i128)L2.nx * L1.c;
        d = make_dir(Zx, Zy);
        ex1 = L1.id;
        ex2 = L2.id;
    }
}


// ------------------------------------------------------------------------------ one cell
// The walk over a cell's subedges as a resumable state: cell_begin, then cell_step until it
// returns non-zero.  Phases 0..2 shoot the projector's corner rays (7,-4), (0,1), (-7,-4)
// (counter-clockwise, consecutive gaps < pi); every later step resolves the subedge on top of
// the stack.
struct CellWalk {
    Line cur, B;
    int m, first, last, nodes, phase;
};

// Returns 0, or -4 when the scanner met a heavy bucket (the cell belongs to the adaptive pass).
template <class Stack, class Sc>
__device__ __forceinline__ int cell_begin(const Cell &C, const float2 *__restrict__ sxy, Sc &sc,
                                          Stack &st, CellWalk &w) {
    w.cur = Line{};
    w.B = Line{};
    w.m = w.first = w.last = w.nodes = w.phase = 0;
    st.depth = 0;
    sc.load(C, sxy);
    return sc.heavy ? -4 : 0;
}

// One step.  Returns 0 (more steps), 1 (done: w.m lines in the sink), or
//   -1 undecided in MODE 0, -2 stack / output capacity, -3 node limit (never expected),
//   -4 the scanner met a heavy bucket.
template <int MODE, class P, class Stack, class Sc, class Snk>
__device__ __forceinline__ int cell_step(const Cell &C, const float2 *__restrict__ sxy, Sc &sc,
                                         Stack &st, int scap, Snk &sink, int ocap, Counters &K,
                                         CellWalk &w) {
    const int phase = w.phase++;
    Dir d;
    int64_t Den = 0;
    int ex1 = INT32_MIN, ex2 = INT32_MIN;
    bool leaf = false;
    Line R{}, L3{};
    if (phase < 3) {
        d = corner_dir(phase);
    } else {
        if (st.depth == 0) {
            if (w.m > 1 && w.last == w.first) {
                --w.m;
                sink.drop_last();
            }
            return 1;
        }
        if (++w.nodes > NODE_LIMIT_FACTOR * (scap + ocap) + 64) return -3;
        K.nodes++;
        R = make_line(C, sxy, st.top());
        const Line &cur = w.cur;
        if (cur.id == R.id) leaf = true;   // SameLines
        else split_dir(cur, R, d, Den, ex1, ex2);
    }
    if (!leaf) {
        const int r = ray<MODE, P, Sc>(C, sc, sxy, d, Den, ex1, ex2, L3, K, phase < 3 ? phase : -1);
        if (r < 0) return r == -4 ? -4 : -1;
        leaf = (r == 1);
        // a shot ray (Lemma on shot rays) yields a corner; a ray that confirms a vertex is the
        // in-cell test of the vertex
        if (leaf) K.vt++; else K.rays++;
        K.vt += Den > 0 ? VT_VRAY : 0u;
    }
    if (phase < 3) {
        if (phase == 0) {
            w.cur = L3;
            w.first = w.last = L3.id;
            sink.put(w.m++, L3.id);
        } else if (phase == 1) {
            w.B = L3;
        } else {
            st.push(w.first);   // closes the cycle
            st.push(L3.id);
            st.push(w.B.id);
        }
        return 0;
    }
    if (leaf) {
        const int id = st.pop();
        w.cur = R;
        if (id != w.last) {
            if (w.m >= ocap) return -2;
            sink.put(w.m++, id);
            w.last = id;
        }
    } else {
        if (st.depth >= scap) return -2;
        st.push(L3.id);
    }
    return 0;
}

// A whole cell.  Returns the number of lines written to the sink (>= 3), or the negative codes
// of cell_step.
template <int MODE, class P, class Stack, class Sc, class Snk>
__device__ __forceinline__ int run_cell(const Cell &C, const float2 *__restrict__ sxy, Sc &sc,
                                        Stack &st, int scap, Snk &sink, int ocap, Counters &K) {
    CellWalk w;
    if (cell_begin(C, sxy, sc, st, w) < 0) return -4;
    for (;;) {
        const int r = cell_step<MODE, P>(C, sxy, sc, st, scap, sink, ocap, K, w);
        if (r != 0) return r > 0 ? w.m : r;
    }
}

}  // namespace vor
