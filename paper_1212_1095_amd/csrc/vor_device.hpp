// vor_device.hpp -- device-side building blocks of the projector algorithm on gfx950.
//
// Coordinates.  Every cell is computed in the frame of its own site p, doubled:
// w = 2 (x - p).  In that frame the bisector of p and a site a is the line delta.w <= q with
// delta = a - p and q = |delta|^2 (the closed half-plane of the cell, Section 2), and a side of
// the box X is N.w <= 2 dist(p, side) with N the unit outward normal.  Every line is thus
// (N, c) with integer N, |N| < 2^24, and 0 < c < 2^49.
//
// Ray endpoint (eq. Tdef of Theorem 2.2).  A ray from p in direction d leaves the cell at
// T = min over lines with N.d > 0 of c / (N.d): the point p + t d stays in the half-plane of a
// line exactly while t N.d <= c.  The minimising line is the line the endpoint lies on
// (Method 5.1 reaches the same point: its temporary endpoints decrease monotonically, Lemma
// on z closer than y, and stop at the first line crossed).
//
// Candidates (Method 11.5 buckets, Method 11.6 with Remark 11.7(ii) shell order, Lemma on
// sites in the large square): buckets are scanned in Chebyshev shells around p's bucket.  Once
// the square S[y, |y - p|] around an upper bound y of the endpoint lies inside the scanned
// block, no unscanned site can be closer to y than p, so the scanned minimum is the endpoint
// and every line through it has been seen (the squares of points of [p, y] nest, Lemma
// B(y,y') / S(y,y')).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vor {

typedef __int128 i128;
typedef unsigned __int128 u128;

constexpr int KOUT = 24;     // lines per cell kept by the filtered pass (more: deferred)
constexpr int SCAP = 16;     // LDS stack entries per thread in the filtered pass
constexpr int DCAP1 = 128;   // stack / output entries per worker in the exact pass
constexpr int NODE_LIMIT_FACTOR = 4;

// status bits (device status word)
enum : int { ST_DOMAIN = 1, ST_DUP = 2, ST_CAPACITY = 4, ST_INTERNAL = 8 };

// stats slots
enum : int {
    SL_RAYS = 0, SL_NODES, SL_EVALS, SL_EXACT, SL_DEFERRED, SL_ASYM, SL_SHELLS, SL_EDGES,
    SL_VTESTS, SL_TREE, SL_TEVALS, SL_XINC, SL_VRAYS, SL_COUNT
};

struct SetDesc {
    int32_t W, H;        // box extent: relative box [0, W] x [0, H]
    int32_t x0, y0;      // absolute origin of the box
    int32_t n;           // number of sites
    int32_t site_off;    // first global index of the set (input, by-id and sorted arrays)
    int32_t gx, gy;      // bucket grid
    int32_t s;           // bucket side
    int32_t bucket_off;  // first global bucket of the set
    int32_t h;           // block half-width in buckets (shells 0..h scanned first)
    int32_t ht;          // leaf sides around p's leaf scanned first (coordinate scans)
    int32_t ns;          // 0: X is the box [0, W] x [0, H]; else the sides of a convex polygon X
    int32_t side_off;    // its first entry in the side table
};

// Side e of a convex polygon X (code -(e+1)): N.x <= c with the primitive outward normal N,
// x relative to the set's box origin (Remark 11.1: any convex polygon X); side e starts at
// vertex (vx, vy).
struct SideRel {
    int32_t nx, ny;
    int64_t c;
    int32_t vx, vy;
};

// ------------------------------------------------------------------------------ FP32 filter
// u = 2^-24.  With d rounded componentwise to FP32 (relative error <= 1.01u) and the products
// and sums rounded to nearest, |den_hat - den| <= 3.03 u S_hat; the upper / lower bounds
// den_hat +- 5u S_hat (one more rounding) bracket the exact scaled N.d.  q_hat has relative
// error <= 2.0001u, v_rcp_f32 is taken as <= 2 ulp (the ISA states 1 ulp), so
//   t >= key_lo (1 - 7.01u)   and   t <= key_hi / (1 - 7.01u).
// Certification multiplies by (1 +- 2^-19) = (1 +- 32u), which covers both factors and the
// rounding of the product itself.
constexpr float GAMMA = 5.0f * 5.9604644775390625e-8f;
constexpr float CERT_UP = 1.0f + 1.9073486328125e-6f;   // 1 + 2^-19
constexpr float CERT_DN = 1.0f - 1.9073486328125e-6f;   // 1 - 2^-19
constexpr float FINF = __builtin_huge_valf();

struct Best {
    float k1, k2;   // smallest and second smallest lower bound
    int w;          // sorted position (>= 0) or side code (-1..-4) of the smallest, or NO_TAG
};
constexpr int NO_TAG = INT32_MIN;   // no candidate yet

__device__ __forceinline__ void consider(float key, int tag, Best &b) {
    const bool better = key < b.k1;
    b.k2 = fminf(b.k2, fmaxf(b.k1, key));
    b.w = better ? tag : b.w;
    b.k1 = fminf(b.k1, key);
}

// For scans that may meet a candidate twice: a second evaluation of the current winner is
// ignored (it would pose as its own runner-up); a second evaluation of any other candidate
// leaves the summary unchanged anyway.
__device__ __forceinline__ void consider_once(float key, int tag, Best &b) {
    if (tag != b.w) consider(key, tag, b);
}

#pragma clang fp contract(off)
// Lower bound key of t = c / (N.d) for a line (nx, ny, c) (floats, exact), or +inf when N.d
// is certainly <= 0.
__device__ __forceinline__ float key_lo_line(float c, float nx, float ny, float dx, float dy) {
    const float mx = nx * dx, my = ny * dy;
    const float den = mx + my;
    const float S = fabsf(mx) + fabsf(my);
    const float up = fmaf(GAMMA, S, den);
    const float key = c * __builtin_amdgcn_rcpf(up);
    return up > 0.0f ? key : FINF;
}
// The same bound for a site in the argmin scans, without the test: up = max(., 0) is never -0
// (the fma adds +0 or more to den), so a line with up <= 0 gets c / +0 = +inf, and q carries an
// added 2^-100 so that the site p itself (delta = 0, den = 0) gets 2^-100 / +0 = +inf rather than
// NaN.  For every other site q >= 1, where 2^-100 is far below half an ulp: q still rounds to a
// neighbour of the exact |delta|^2 within half an ulp (only an exact tie may round the other
// way), so the error bounds above hold unchanged.
constexpr float Q_TINY = 0x1p-100f;
__device__ __forceinline__ float site_q_scan(float ex, float ey) {
    return fmaf(ex, ex, fmaf(ey, ey, Q_TINY));
}
__device__ __forceinline__ float key_lo_scan_q(float q, float ex, float ey, float dx, float dy) {
    const float mx = ex * dx, my = ey * dy;
    const float den = mx + my;
    const float S = fabsf(mx) + fabsf(my);
    const float up = fmaxf(fmaf(GAMMA, S, den), 0.0f);
    return q * __builtin_amdgcn_rcpf(up);
}
__device__ __forceinline__ float key_lo_scan(float ex, float ey, float dx, float dy) {
    return key_lo_scan_q(site_q_scan(ex, ey), ex, ey, dx, dy);
}
// Upper bound key (+inf unless N.d is certainly > 0).
__device__ __forceinline__ float key_hi_line(float c, float nx, float ny, float dx, float dy) {
    const float mx = nx * dx, my = ny * dy;
    const float den = mx + my;
    const float S = fabsf(mx) + fabsf(my);
    const float lo = fmaf(-GAMMA, S, den);
    const float key = c * __builtin_amdgcn_rcpf(lo);
    return lo > 0.0f ? key : FINF;
}
// Site candidate: delta = a - p exact in FP32 (|delta| < 2^24), q = |delta|^2 rounded.
__device__ __forceinline__ float site_q(float ex, float ey) { return fmaf(ex, ex, ey * ey); }
#pragma clang fp contract(fast)

// ------------------------------------------------------------------------------ workgroup scan
// Exclusive prefix sum of one value per thread over a workgroup of B threads; `total` gets
// the sum.  Every thread calls it (two barriers); wsum: B / 64 ints of LDS.
template <int B>
__device__ __forceinline__ int block_exscan(int v, int *wsum, int &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int before = incl - v;
    total = 0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) {
        before += w < wv ? wsum[w] : 0;
        total += wsum[w];
    }
    __syncthreads();
    return before;
}

// ------------------------------------------------------------------------------ exact helpers
__device__ __forceinline__ double u128_to_double(u128 m) {
    return (double)(uint64_t)(m >> 64) * 18446744073709551616.0 + (double)(uint64_t)m;
}
__device__ __forceinline__ double i128_to_double(i128 v) {
    const bool neg = v < 0;
    const double r = u128_to_double(neg ? (u128)(-v) : (u128)v);
    return neg ? -r : r;
}

// 64 x 128 -> 192-bit unsigned product, limbs little-endian.
__device__ __forceinline__ void mul_u64_u128(uint64_t a, u128 b, uint64_t r[3]) {
    const u128 lo = (u128)a * (uint64_t)b;
    const u128 hi = (u128)a * (uint64_t)(b >> 64);
    const u128 mid = (lo >> 64) + (u128)(uint64_t)hi;
    r[0] = (uint64_t)lo;
    r[1] = (uint64_t)mid;
    r[2] = (uint64_t)(mid >> 64) + (uint64_t)(hi >> 64);
}
__device__ __forceinline__ int cmp192(const uint64_t a[3], const uint64_t b[3]) {
    if (a[2] != b[2]) return a[2] < b[2] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    return 0;
}
// sign(t_i - t_j) for t = c / den with c > 0, den > 0:  sign(c_i den_j - c_j den_i).
__device__ __forceinline__ int cmp_t(uint64_t ci, u128 di, uint64_t cj, u128 dj) {
    uint64_t a[3], b[3];
    mul_u64_u128(ci, dj, a);
    mul_u64_u128(cj, di, b);
    return cmp192(a, b);
}

// ------------------------------------------------------------------------------ lines
struct Line {
    int id;         // sorted position (>= 0) or side code (-1 .. -4)
    int nx, ny;     // normal (doubled frame)
    int64_t c;      // right-hand side, > 0
};

struct Cell {       // per-cell constants
    int gx, gy, s, boff;  // the set's bucket grid
    int h;                // half-width (in buckets) of the block scanned first
    int ht;               // leaf sides around p's leaf scanned first (coordinate scans)
    float pxf, pyf; // p, relative to the box origin (exact floats)
    int px, py;
    int bx, by;     // p's bucket
    int W, H;       // box extent (relative box [0, W] x [0, H])
    int ns;         // 0: X is the box; else X is the convex polygon of `sides`
    const SideRel *sides;
    int grow;       // box sides pushed out by this many units (1: the enlarged box that holds a
                    // site on the boundary of X strictly inside; 0 otherwise)
};

// Side code -> line in p's doubled frame: N.w <= 2 (c - N.p).  Box sides (k = -code - 1: 0
// bottom, 1 right, 2 top, 3 left) are written with arithmetic selects so that no lookup table
// is materialised; polygon sides come from the side table.
__device__ __forceinline__ Line side_line(const Cell &C, int code) {
    if (C.ns > 0) {
        const SideRel s = C.sides[-code - 1];
        Line L;
        L.id = code;
        L.nx = s.nx;
        L.ny = s.ny;
        L.c = 2 * (s.c - (int64_t)s.nx * C.px - (int64_t)s.ny * C.py);
        return L;
    }
    const int k = -code - 1;
    const bool vert = (k & 1) == 0;            // bottom / top: normal along y
    const bool far = ((k + 1) >> 1) & 1;       // right / top: outward normal positive
    const int v = vert ? C.py : C.px;
    const int ext = vert ? C.H : C.W;
    const int sgn = far ? 1 : -1;
    Line L;
    L.id = code;
    L.nx = vert ? 0 : sgn;
    L.ny = vert ? sgn : 0;
    L.c = 2 * ((int64_t)(far ? ext - v : v) + C.grow);
    return L;
}
__device__ __forceinline__ Line site_line(const Cell &C, const float2 *sxy, int pos) {
    const float2 a = sxy[pos];
    Line L;
    L.id = pos;
    L.nx = (int)a.x - C.px;
    L.ny = (int)a.y - C.py;
    L.c = (int64_t)L.nx * L.nx + (int64_t)L.ny * L.ny;
    return L;
}
__device__ __forceinline__ Line make_line(const Cell &C, const float2 *sxy, int id) {
    return id >= 0 ? site_line(C, sxy, id) : side_line(C, id);
}

// Direction d (exact, 128-bit components) and its FP32 image d_s = d 2^-sigma rounded, with
// max |component| of d_s in [1, 2).
struct Dir {
    i128 x, y;
    float fx, fy;
    int sigma;
};
__device__ __forceinline__ Dir make_dir(i128 x, i128 y) {
    Dir d;
    d.x = x;
    d.y = y;
    const double ax = i128_to_double(x), ay = i128_to_double(y);
    const double m = fmax(fabs(ax), fabs(ay));
    int e;
    (void)frexp(m, &e);          // m = f 2^e, f in [0.5, 1)
    d.sigma = e - 1;             // m 2^-sigma in [1, 2)
    d.fx = (float)ldexp(ax, -d.sigma);
    d.fy = (float)ldexp(ay, -d.sigma);
    return d;
}

// ------------------------------------------------------------------------------ shells
// Calls f(lo, hi) for every sorted-position range of shell k around bucket (bx, by).
template <class F>
__device__ __forceinline__ void for_shell(const Cell &S, const int *__restrict__ bstart, int bx,
                                          int by, int k, F &&f) {
    const int base = S.boff;
    if (k == 0) {
        const int b = base + by * S.gx + bx;
        f(bstart[b], bstart[b + 1]);
        return;
    }
    const int xa = max(bx - k, 0), xb = min(bx + k, S.gx - 1);
    if (by - k >= 0) {
        const int r = base + (by - k) * S.gx;
        f(bstart[r + xa], bstart[r + xb + 1]);
    }
    if (by + k < S.gy) {
        const int r = base + (by + k) * S.gx;
        f(bstart[r + xa], bstart[r + xb + 1]);
    }
    const int ya = max(by - k + 1, 0), yb = min(by + k - 1, S.gy - 1);
    if (bx - k >= 0)
        for (int y = ya; y <= yb; ++y) {
            const int b = base + y * S.gx + bx - k;
            f(bstart[b], bstart[b + 1]);
        }
    if (bx + k < S.gx)
        for (int y = ya; y <= yb; ++y) {
            const int b = base + y * S.gx + bx + k;
            f(bstart[b], bstart[b + 1]);
        }
}

// Segment `seg` of shell k as a sorted-position range [lo, hi): shell 0 is p's bucket; shell
// k >= 1 has 4k segments: the bottom and top rows (2k+1 buckets, contiguous in row-major
// bucket order), then the 2k-1 buckets of the left column and of the right column.  Parts
// outside the grid are empty.
__device__ __forceinline__ void seg_range(const Cell &C, const int *__restrict__ bstart, int k,
                                          int seg, int &lo, int &hi) {
    int row, xa, xb;
    if (k == 0) {
        row = C.by;
        xa = xb = C.bx;
    } else if (seg < 2) {
        row = seg == 0 ? C.by - k : C.by + k;
        xa = max(C.bx - k, 0);
        xb = min(C.bx + k, C.gx - 1);
    } else {
        const int t = seg - 2;                 // 0 .. 4k-3
        const bool right = t >= 2 * k - 1;
        row = C.by - k + 1 + (right ? t - (2 * k - 1) : t);
        xa = xb = right ? C.bx + k : C.bx - k;
    }
    if (row < 0 || row >= C.gy || xa < 0 || xb >= C.gx || xa > xb) {
        lo = hi = 0;
        return;
    }
    const int r = C.boff + row * C.gx;
    lo = bstart[r + xa];
    hi = bstart[r + xb + 1];
}

// Bucket rectangle [x0, x1] x [y0, y1] (inclusive; empty when x0 > x1 or y0 > y1).
struct Rect {
    int x0, x1, y0, y1;
};

__device__ __forceinline__ bool rect_inside(const Rect &a, const Rect &b) {
    return a.x0 >= b.x0 && a.x1 <= b.x1 && a.y0 >= b.y0 && a.y1 <= b.y1;
}

// The point y = p + (T/2) d_s and its distance r from p, in p's frame (so that rounding errors
// scale with r, not with the coordinates), and the margin M that covers them: the products
// and the square root round with relative error below 4e-7 and d_s is within 1.01 u of the
// scaled direction, so M = 1e-5 r + 2 (>= 2 coordinate units) keeps every test conservative.
// Returns false for an infinite or undefined T.
__device__ __forceinline__ bool bound_point(float T, float dx, float dy, float &hx, float &hy,
                                            float &r, float &M) {
    const float Tu = T * CERT_UP;
    hx = 0.5f * Tu * dx;
    hy = 0.5f * Tu * dy;
    r = sqrtf(hx * hx + hy * hy);
    M = r * 1.0e-5f + 2.0f;
    return r < 1.0e30f;
}

// The integer rectangle S_I[y, |y - p|] of eq. (S_I), in buckets and clipped to the grid, for
// y = p + (T/2) d_s with T an upper bound of the endpoint parameter: by the lemma on sites in
// the large square every site that is not farther from y than p lies in it, and the rectangles
// of the points of [p, y] nest inside it.  The square is widened by the margin M of
// bound_point; an infinite or undefined T gives the whole grid.
__device__ __forceinline__ Rect need_rect(const Cell &C, float T, float dx, float dy) {
    float hx, hy, r, M;
    Rect R{0, C.gx - 1, 0, C.gy - 1};
    if (!bound_point(T, dx, dy, hx, hy, r, M)) return R;
    const float ext = (float)C.W + (float)C.H + 2.0f;   // clamp before converting
    const int lx = C.px + (int)fminf(fmaxf(floorf(hx - r - M), -ext), ext);
    const int ux = C.px + (int)fminf(fmaxf(ceilf(hx + r + M), -ext), ext);
    const int ly = C.py + (int)fminf(fmaxf(floorf(hy - r - M), -ext), ext);
    const int uy = C.py + (int)fminf(fmaxf(ceilf(hy + r + M), -ext), ext);
    R.x0 = min(max(lx, 0) / C.s, C.gx - 1);
    R.x1 = min(max(ux, 0) / C.s, C.gx - 1);
    R.y0 = min(max(ly, 0) / C.s, C.gy - 1);
    R.y1 = min(max(uy, 0) / C.s, C.gy - 1);
    return R;
}

// The cell's first block: shells 0..h around p's bucket, clipped to the grid.
__device__ __forceinline__ Rect block_rect(const Cell &C) {
    return Rect{max(C.bx - C.h, 0), min(C.bx + C.h, C.gx - 1), max(C.by - C.h, 0),
                min(C.by + C.h, C.gy - 1)};
}

// The first rectangle a scan covers: the block A, or, when tcap bounds the endpoint parameter
// (a vertex ray), the rectangle S_I of that bound if it lies inside A.
__device__ __forceinline__ Rect first_rect(const Cell &C, const Rect &A, float tcap, float dx,
                                           float dy) {
    if (!(tcap < FINF)) return A;
    const Rect R0 = need_rect(C, tcap, dx, dy);
    return rect_inside(R0, A) ? R0 : A;
}

// The next scanned rectangle: the bounding box of the scanned rectangle A and the needed
// rectangle R, but at most A widened by its own size on each side (a poor first bound gives
// a huge R; the region then grows geometrically and the bound tightens on the way).
__device__ __forceinline__ Rect grow_rect(const Rect &A, const Rect &R) {
    const int wx = A.x1 - A.x0 + 1, wy = A.y1 - A.y0 + 1;
    return Rect{max(min(A.x0, R.x0), A.x0 - wx), min(max(A.x1, R.x1), A.x1 + wx),
                max(min(A.y0, R.y0), A.y0 - wy), min(max(A.y1, R.y1), A.y1 + wy)};
}

// Walks the bucket rows of rectangle O minus rectangle I (I inside O, or empty) as
// sorted-position segments: a row of O is one contiguous segment (row-major bucket order),
// a row that crosses I splits into its parts left and right of I.  next() loads the next
// segment into [pos, end) and returns false when O \ I is exhausted.
struct RowWalk {
    Rect O, I;
    int row, part;
    int pos, end;

    __device__ __forceinline__ void start(Rect o, Rect i) {
        O = o;
        I = i;
        row = o.y0;
        part = 0;
        pos = end = 0;
    }
    __device__ __forceinline__ bool next(const Cell &C, const int *__restrict__ bstart) {
        if (row > O.y1) return false;
        int xa, xb;
        const int r = row;
        if (row >= I.y0 && row <= I.y1) {
            if (part == 0) {
                xa = O.x0;
                xb = min(O.x1, I.x0 - 1);
                part = 1;
            } else {
                xa = max(O.x0, I.x1 + 1);
                xb = O.x1;
                part = 0;
                ++row;
            }
        } else {
            xa = O.x0;
            xb = O.x1;
            ++row;
        }
        int a = 0, b = 0;
        if (xa <= xb) {
            const int base = C.boff + r * C.gx;
            a = bstart[base + xa];
            b = bstart[base + xb + 1];
        }
        pos = a;
        end = b;
        return true;
    }
};

}  // namespace vor
