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
#pragma once
#include "vor_device.hpp"

namespace vor {

struct Counters {
    uint32_t rays, nodes, evals, exact, shells, vtests;
};

struct ScanOut {
    Best b;
    float Uw;   // upper bound key of the final winner
    float U;    // smallest upper bound seen
    Rect A;     // the scanned rectangle (it contains S_I of the endpoint)
};

// Upper bound key of candidate w (sorted position or side code).
__device__ __forceinline__ float upper_of(const Cell &C, const float2 *__restrict__ sxy, int w,
                                          float dx, float dy) {
    if (w >= 0) {
        const float2 a = sxy[w];
        const float ex = a.x - C.pxf, ey = a.y - C.pyf;
        return key_hi_line(site_q(ex, ey), ex, ey, dx, dy);
    }
    const Line L = side_line(C, w);
    return key_hi_line((float)L.c, (float)L.nx, (float)L.ny, dx, dy);
}

// FP32 scan of the rays's candidates, shell by shell, until the block certifies the endpoint
// (or the point at tcap, whichever is nearer).  Candidates ex1 / ex2 are skipped when EXCL.
// Box sides the ray can leave through: at most one horizontal and one vertical side.
template <bool EXCL>
__device__ __forceinline__ void consider_sides(const Cell &C, float dx, float dy, int ex1, int ex2,
                                               Best &b) {
    const int sv = dy > 0.0f ? -3 : -1, sh = dx > 0.0f ? -2 : -4;
    const Line Lv = side_line(C, sv), Lh = side_line(C, sh);
    float kv = key_lo_line((float)Lv.c, (float)Lv.nx, (float)Lv.ny, dx, dy);
    float kh = key_lo_line((float)Lh.c, (float)Lh.nx, (float)Lh.ny, dx, dy);
    if (EXCL) {
        kv = (sv == ex1 || sv == ex2) ? FINF : kv;
        kh = (sh == ex1 || sh == ex2) ? FINF : kh;
    }
    consider(kv, sv, b);
    consider(kh, sh, b);
}

template <bool EXCL>
__device__ __forceinline__ void eval_site(const Cell &C, const float2 *__restrict__ sxy, int pos,
                                          float dx, float dy, int ex1, int ex2, Best &b) {
    const float2 a = sxy[pos];
    const float ex = a.x - C.pxf, ey = a.y - C.pyf;
    float key = key_lo_line(site_q(ex, ey), ex, ey, dx, dy);
    if (EXCL) key = (pos == ex1 || pos == ex2) ? FINF : key;
    consider(key, pos, b);
}

// Row ranges of the cell's warm-start block (up to MAXROWS rows, h <= 2), loaded once per
// cell.  LdsRows keeps them in a per-thread column of LDS (the filtered pass);
// GlobalRows reads them from the bucket starts each time (the exact passes).
constexpr int MAXROWS = 5;

template <int BLOCK>
struct LdsRows {
    int (*lo)[BLOCK];
    int (*hi)[BLOCK];
    int nrows;
    __device__ __forceinline__ void load(const Cell &C, const int *__restrict__ bstart) {
        const Rect A = block_rect(C);
        nrows = A.y1 - A.y0 + 1;
        if (nrows > MAXROWS) return;
        for (int i = 0; i < nrows; ++i) {
            const int base = C.boff + (A.y0 + i) * C.gx;
            lo[i][threadIdx.x] = bstart[base + A.x0];
            hi[i][threadIdx.x] = bstart[base + A.x1 + 1];
        }
    }
    __device__ __forceinline__ void get(const Cell &, const int *__restrict__, int r, int &a,
                                        int &b) const {
        a = lo[r][threadIdx.x];
        b = hi[r][threadIdx.x];
    }
};

struct GlobalRows {
    int nrows;
    __device__ __forceinline__ void load(const Cell &C, const int *__restrict__) {
        const Rect A = block_rect(C);
        nrows = A.y1 - A.y0 + 1;
    }
    __device__ __forceinline__ void get(const Cell &C, const int *__restrict__ bstart, int r,
                                        int &a, int &b) const {
        const Rect A = block_rect(C);
        const int base = C.boff + (A.y0 + r) * C.gx;
        a = bstart[base + A.x0];
        b = bstart[base + A.x1 + 1];
    }
};

template <bool EXCL, class Rows>
__device__ __forceinline__ ScanOut scan_f32(const Cell &C, const Rows &BR,
                                            const float2 *__restrict__ sxy,
                                            const int *__restrict__ bstart, float dx, float dy,
                                            int ex1, int ex2, float tcap, Counters &K) {
    Best b{FINF, FINF, 0};
    consider_sides<EXCL>(C, dx, dy, ex1, ex2, b);
    // Method 11.6.  Pass A: the cell's block of shells 0..h (a warm start that bounds the
    // endpoint by y), one flat loop per lane over its rows; the row ranges are in registers,
    // so a lane pays only for its own candidates plus a select per row.
    const Rect A = block_rect(C);
    if (BR.nrows <= MAXROWS) {
        int r = 0, pos, end;
        BR.get(C, bstart, 0, pos, end);
        for (;;) {
            if (pos < end) {
                eval_site<EXCL>(C, sxy, pos, dx, dy, ex1, ex2, b);
                ++pos;
                ++K.evals;
                continue;
            }
            if (++r >= BR.nrows) break;
            BR.get(C, bstart, r, pos, end);
        }
    } else {
        RowWalk wk;
        wk.start(A, Rect{1, 0, 1, 0});
        for (;;) {
            if (wk.pos < wk.end) {
                eval_site<EXCL>(C, sxy, wk.pos, dx, dy, ex1, ex2, b);
                ++wk.pos;
                ++K.evals;
                continue;
            }
            if (!wk.next(C, bstart)) break;
        }
    }
    // One transition for all lanes: the integer rectangle S_I[y, |y - p|] of the bound.
    K.shells++;
    float U = upper_of(C, sxy, b.w, dx, dy);
    Rect R = need_rect(C, fminf(U, tcap), dx, dy);
    Rect O = A;
    if (!rect_inside(R, A)) {
        // Pass B (lanes whose rectangle sticks out of the block): grow the scanned rectangle
        // towards S_I, at most doubling per step; the rectangles of later, nearer bounds nest
        // inside the earlier ones, so the final scanned rectangle certifies the endpoint.
        RowWalk wk;
        wk.start(grow_rect(A, R), A);
        for (;;) {
            if (wk.pos < wk.end) {
                eval_site<EXCL>(C, sxy, wk.pos, dx, dy, ex1, ex2, b);
                ++wk.pos;
                ++K.evals;
                continue;
            }
            if (wk.next(C, bstart)) continue;
            K.shells++;
            U = fminf(U, upper_of(C, sxy, b.w, dx, dy));
            R = need_rect(C, fminf(U, tcap), dx, dy);
            if (rect_inside(R, wk.O)) break;
            const Rect prev = wk.O;
            wk.start(grow_rect(prev, R), prev);
        }
        O = wk.O;
    }
    const float Uw = upper_of(C, sxy, b.w, dx, dy);
    ScanOut o;
    o.b = b;
    o.Uw = Uw;
    o.U = fminf(U, Uw);
    o.A = O;
    return o;
}

// ------------------------------------------------------------------------------ exact argmin
struct XBest {
    int id;
    int nx, ny;
    uint64_t c;
    u128 den;
    bool have;
};

__device__ __forceinline__ void x_consider(XBest &b, int id, int nx, int ny, int64_t c,
                                           const Dir &d) {
    const i128 den = (i128)nx * d.x + (i128)ny * d.y;
    if (den <= 0) return;
    if (b.have) {
        const int s = cmp_t((uint64_t)c, (u128)den, b.c, b.den);
        if (s > 0) return;
        if (s == 0) {
            // tie at the endpoint: keep the most clockwise normal
            const int64_t cr = (int64_t)b.nx * ny - (int64_t)b.ny * nx;
            if (cr >= 0) return;
        }
    }
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

// Exact argmin over the rectangle an FP32 scan certified (prev), or over a block grown
// towards the certified rectangle of the exact winner (prev == null: exact-only precision).  With FILTER only candidates whose FP32 lower bound is <= Tlim count.
template <bool FILTER>
__device__ __forceinline__ void exact_scan(const Cell &C, const float2 *__restrict__ sxy,
                                           const int *__restrict__ bstart, const Dir &d,
                                           const ScanOut *prev, float Tlim, float tcap, int ex1,
                                           int ex2, XBest &b, Counters &K) {
    b.have = false;
    const float lim = Tlim * CERT_UP;
    for (int code = -1; code >= -4; --code) {
        if (code == ex1 || code == ex2) continue;
        const Line L = side_line(C, code);
        if (FILTER &&
            !(key_lo_line((float)L.c, (float)L.nx, (float)L.ny, d.fx, d.fy) * CERT_DN <= lim))
            continue;
        x_consider(b, code, L.nx, L.ny, L.c, d);
    }
    RowWalk wk;
    wk.start(prev ? prev->A : block_rect(C), Rect{1, 0, 1, 0});
    for (;;) {
        if (wk.pos < wk.end) {
            const int pos = wk.pos++;
            if (pos == ex1 || pos == ex2) continue;
            const float2 a = sxy[pos];
            const float ex = a.x - C.pxf, ey = a.y - C.pyf;
            if (FILTER && !(key_lo_line(site_q(ex, ey), ex, ey, d.fx, d.fy) * CERT_DN <= lim))
                continue;
            if (!FILTER) ++K.evals;
            const int nx = (int)a.x - C.px, ny = (int)a.y - C.py;
            if ((nx | ny) == 0) continue;   // p itself
            x_consider(b, pos, nx, ny, (int64_t)nx * nx + (int64_t)ny * ny, d);
            continue;
        }
        if (wk.next(C, bstart)) continue;
        if (prev) break;   // the FP32 scan's rectangle already certifies the endpoint
        K.shells++;
        const Rect R = need_rect(C, fminf(x_upper(b, d), tcap), d.fx, d.fy);
        if (rect_inside(R, wk.O)) break;
        wk.start(grow_rect(wk.O, R), wk.O);
    }
}

// ------------------------------------------------------------------------------ stacks / outputs
template <int BLOCK>
struct LdsStack {
    int (*s)[BLOCK];
    int depth;
    __device__ __forceinline__ void push(int v) { s[depth++][threadIdx.x] = v; }
    __device__ __forceinline__ int top() const { return s[depth - 1][threadIdx.x]; }
    __device__ __forceinline__ int pop() { return s[--depth][threadIdx.x]; }
};

struct GStack {
    int *s;
    int depth;
    __device__ __forceinline__ void push(int v) { s[depth++] = v; }
    __device__ __forceinline__ int top() const { return s[depth - 1]; }
    __device__ __forceinline__ int pop() { return s[--depth]; }
};

// Output sink: stores the line's label (local site index or side code).
struct Sink {
    int *dst;
    const int *sid;
    __device__ __forceinline__ void put(int m, int id) { dst[m] = id >= 0 ? sid[id] : id; }
};

// ------------------------------------------------------------------------------ ray shots
// MODE 0: FP32 filter, give up (defer the cell) when a decision is not certified.
// MODE 1: FP32 filter, exact decision when not certified.
// MODE 2: exact arithmetic for every decision.
//
// Plain ray (Den == 0): out = the line the endpoint lies on; returns 0.
// Vertex ray (Den > 0, d = Z, u = Z / Den; lines ex1, ex2 through u skipped): returns 1 when u
// is in the cell (a vertex), 0 when a line crosses [p, u) first (that line in out).
// Returns -1 when undecided (MODE 0).
template <int MODE, class Rows>
__device__ __forceinline__ int ray(const Cell &C, const Rows &BR, const float2 *__restrict__ sxy,
                                   const int *__restrict__ bstart, const Dir &d, int64_t Den,
                                   int ex1, int ex2, Line &out, Counters &K) {
    const bool vmode = Den > 0;
    float tu_hi = FINF, tu_lo = FINF;
    if (vmode) {
        const float tu = (float)ldexp(1.0 / (double)Den, d.sigma);
        tu_hi = tu * CERT_UP;
        tu_lo = tu * CERT_DN;
    }
    XBest xb;
    if (MODE == 2) {
        exact_scan<false>(C, sxy, bstart, d, nullptr, FINF, tu_hi, ex1, ex2, xb, K);
    } else {
        const ScanOut s =
            vmode ? scan_f32<true, Rows>(C, BR, sxy, bstart, d.fx, d.fy, ex1, ex2, tu_hi, K)
                  : scan_f32<false, Rows>(C, BR, sxy, bstart, d.fx, d.fy, ex1, ex2, FINF, K);
        if (vmode && s.b.k1 * CERT_DN > tu_hi) return 1;
        const float uw = s.Uw * CERT_UP;
        if (uw < s.b.k2 * CERT_DN && (!vmode || uw < tu_lo)) {
            out = make_line(C, sxy, s.b.w);
            return 0;
        }
        if (MODE == 0) return -1;
        K.exact++;
        exact_scan<true>(C, sxy, bstart, d, &s, vmode ? tu_hi : s.U, tu_hi, ex1, ex2, xb, K);
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

// ------------------------------------------------------------------------------ one cell
// Returns the number of lines written to the sink (>= 3), or
//   -1 undecided in MODE 0, -2 stack / output capacity, -3 node limit (never expected).
template <int MODE, class Stack, class Rows>
__device__ __forceinline__ int run_cell(const Cell &C, const float2 *__restrict__ sxy,
                                        const int *__restrict__ bstart, Stack &st, int scap,
                                        Rows &BR, Sink &sink, int ocap, Counters &K) {
    Line cur{}, B{}, L3{};
    int m = 0, first = 0, last = 0;
    const int node_limit = NODE_LIMIT_FACTOR * (scap + ocap) + 64;
    int nodes = 0;
    st.depth = 0;
    BR.load(C, bstart);
    // phases 0..2: the projector's corner rays (7,-4), (0,1), (-7,-4): counter-clockwise,
    // consecutive gaps < pi.  Then the subedge loop.
    for (int phase = 0;; ++phase) {
        Dir d;
        int64_t Den = 0;
        int ex1 = INT32_MIN, ex2 = INT32_MIN;
        bool leaf = false;
        Line R{};
        if (phase < 3) {
            d = make_dir(phase == 1 ? 0 : (phase == 0 ? 7 : -7), phase == 1 ? 1 : -4);
        } else {
            if (st.depth == 0) break;
            if (++nodes > node_limit) return -3;
            K.nodes++;
            R = make_line(C, sxy, st.top());
            if (cur.id == R.id) {
                leaf = true;   // SameLines
            } else {
                Den = (int64_t)cur.nx * R.ny - (int64_t)cur.ny * R.nx;
                if (Den == 0) {   // ParallelLines: direction of the lines, inside the wedge
                    d = make_dir(-(i128)cur.ny, (i128)cur.nx);
                } else {          // OutsideWedge (Den < 0) or Vertex / OutsideCell (Den > 0)
                    const i128 Zx = (i128)cur.c * R.ny - (i128)R.c * cur.ny;
                    const i128 Zy = (i128)cur.nx * R.c - (i128)R.nx * cur.c;
                    d = make_dir(Zx, Zy);
                    ex1 = cur.id;
                    ex2 = R.id;
                }
            }
        }
        if (!leaf) {
            const int r = ray<MODE, Rows>(C, BR, sxy, bstart, d, Den, ex1, ex2, L3, K);
            if (r < 0) return -1;
            leaf = (r == 1);
            // a shot ray (Lemma on shot rays) yields a corner; a ray that confirms a vertex
            // is the in-cell test of the vertex
            if (leaf) K.vtests++; else K.rays++;
        }
        if (phase < 3) {
            if (phase == 0) {
                cur = L3;
                first = last = L3.id;
                sink.put(m++, L3.id);
            } else if (phase == 1) {
                B = L3;
            } else {
                st.push(first);   // closes the cycle
                st.push(L3.id);
                st.push(B.id);
            }
            continue;
        }
        if (leaf) {
            const int id = st.pop();
            cur = R;
            if (id != last) {
                if (m >= ocap) return -2;
                sink.put(m++, id);
                last = id;
            }
        } else {
            if (st.depth >= scap) return -2;
            st.push(L3.id);
        }
    }
    if (m > 1 && last == first) --m;
    return m;
}

}  // namespace vor
