// vor_tree.hpp -- adaptive bucketing for clustered sites.
//
// The uniform grid of Method 11.5 sizes its buckets for the mean density; in a cluster a bucket
// can hold thousands of sites and every ray that touches it scans all of them.  Buckets with
// more than TREE_C0 sites are therefore refined, recursively, up to TREE_LEVELS levels: the
// bounding square of the bucket's sites gets an m x m grid of sub-buckets (m a power of two
// chosen from the count), so that the grid follows the occupied part only.  Sites stay in one sorted array; the sites of a (sub-)bucket remain one contiguous
// range, and a refined bucket's range is the concatenation of its sub-buckets' ranges in
// row-major order.
//
// The certificate of Method 11.6 does not depend on the bucket shapes (the lemma on sites in
// the large square bounds the sites closer to y than p by the square S[y, |y - p|] itself), so
// the tree scan keeps the same warm-start-then-grow scheme with rectangles in coordinates
// instead of whole buckets: a pass visits the leaves that meet the new region and evaluates
// exactly the sites inside the new region and outside the region scanned before, so every
// site is evaluated at most once per ray.
#pragma once
#include "vor_device.hpp"

namespace vor {

constexpr int TREE_C0 = 16;       // a grid bucket with more sites is refined
constexpr int TREE_C1 = 6;        // a sub-bucket with more sites is refined
constexpr int TREE_LEVELS = 6;    // refinement levels below the bucket grid
constexpr int TREE_MMAX = 8;      // sub-buckets per axis at most (empty parts stay coarse)
constexpr int SEG_HEAVY = 96;     // the filtered pass hands a cell on at a longer row segment
constexpr int TFRAMES = TREE_LEVELS + 1;
constexpr int TREE_LIST = 48;     // cached candidate positions per cell (adaptive pass)
constexpr int TREE_LIST_FILL = 20;// the cached region grows until it holds this many sites
constexpr int TREE_PROBES = 6;    // leaves probed along the ray before a region pass
constexpr int TREE_BUDGET = 640;  // sub-buckets + evaluations a lane spends on one cell before
                                  // handing it to the one-wave-per-cell pass
constexpr unsigned long long TREE_TICKS = 30000;   // 300 us at the 100 MHz clock: a lane's
                                                 // time on one cell before it hands the cell on
                                                 // in the tree scans' tail
constexpr int TREE_BATCH = 4;     // candidate loads issued together (one lane walks one cell, so
                                  // the loads of a leaf or of the list overlap instead of queueing)

struct TNode {
    int ox, oy;   // origin of the bounding square of the node's sites (relative coordinates)
    int size;     // side of that square (set by the refinement)
    int a, cnt;   // sorted-position range [a, a + cnt) of its sites
    int pk;       // table slot of the parent that points to this node
    int ss, m;    // sub-bucket side, sub-buckets per axis (set by the refinement)
    int tab;      // first of the m*m + 1 sub-bucket starts in the table
    int lv;       // refinement level (1 for a refined grid bucket)
};

// Table of bucket starts: the grid's gtot + 1 starts first, then the nodes' sub-bucket starts;
// tchild[k] is the node that refines slot k, or -1 for a leaf; tref[b] counts the refined grid
// buckets before grid bucket b (so that a row range without refined buckets is one
// contiguous range of sites).
struct Tree {
    const int *tstart;
    const int *tchild;
    const TNode *nodes;
    const int *tref;
};

// The empty region: contains no point, meets no rectangle, contains no rectangle.
constexpr Rect NO_RECT{1 << 30, -(1 << 30), 1 << 30, -(1 << 30)};

__device__ __forceinline__ bool rect_meets(const Rect &a, const Rect &b) {
    return a.x0 <= b.x1 && b.x0 <= a.x1 && a.y0 <= b.y1 && b.y0 <= a.y1;
}

// The square S[y, |y - p|] widened by M, in coordinates (inclusive integer bounds) clipped to
// the box; the whole box for an infinite or undefined T.
__device__ __forceinline__ Rect need_crect(const Cell &C, float T, float dx, float dy) {
    float hx, hy, r, M;
    Rect R{0, C.W, 0, C.H};
    if (!bound_point(T, dx, dy, hx, hy, r, M)) return R;
    const float ext = (float)C.W + (float)C.H + 2.0f;   // clamp before converting
    const float lx = fminf(fmaxf(floorf(hx - r - M), -ext), ext);
    const float ux = fminf(fmaxf(ceilf(hx + r + M), -ext), ext);
    const float ly = fminf(fmaxf(floorf(hy - r - M), -ext), ext);
    const float uy = fminf(fmaxf(ceilf(hy + r + M), -ext), ext);
    R.x0 = min(max(C.px + (int)lx, 0), C.W);
    R.x1 = min(max(C.px + (int)ux, 0), C.W);
    R.y0 = min(max(C.py + (int)ly, 0), C.H);
    R.y1 = min(max(C.py + (int)uy, 0), C.H);
    return R;
}

// The closed disk D(y, |y - p| + M) of the same bound (the whole plane for an infinite or
// undefined T), centre in p's frame: by the lemma on sites in the large square every site not
// farther than p from y lies in D(y, |y - p|), so a leaf or site outside this disk can hold
// neither the endpoint's line nor a tie.  The squared radius carries a relative slack that
// covers the rounding of the distance tests.
struct Disk {
    float cx, cy, r2;
};
__device__ __forceinline__ Disk need_disk(const Cell &C, float T, float dx, float dy) {
    float hx, hy, r, M;
    Disk D{0.0f, 0.0f, FINF};
    if (!bound_point(T, dx, dy, hx, hy, r, M)) return D;
    const float rr = r + M;
    D.cx = hx;
    D.cy = hy;
    D.r2 = rr * rr * 1.0001f + 4.0f;
    return D;
}
// Rectangle and point tests in p's frame (integer differences below 2^25 are exact floats).
__device__ __forceinline__ bool disk_meets(const Cell &C, const Disk &D, const Rect &r) {
    const float x0 = (float)(r.x0 - C.px), x1 = (float)(r.x1 - C.px);
    const float y0 = (float)(r.y0 - C.py), y1 = (float)(r.y1 - C.py);
    const float ex = fmaxf(fmaxf(x0 - D.cx, D.cx - x1), 0.0f);
    const float ey = fmaxf(fmaxf(y0 - D.cy, D.cy - y1), 0.0f);
    return ex * ex + ey * ey <= D.r2;
}
__device__ __forceinline__ bool in_disk(const Disk &D, float ex, float ey) {
    const float fx = ex - D.cx, fy = ey - D.cy;
    return fx * fx + fy * fy <= D.r2;
}

// The leaf (sub-)bucket that contains p, widened by h leaf sides on each side: the warm-start
// region of every ray of the cell.
__device__ __forceinline__ Rect tree_block(const Cell &C, const Tree &T, int h) {
    int ox = C.bx * C.s, oy = C.by * C.s, side = C.s;
    int c = T.tchild[C.boff + C.by * C.gx + C.bx];
    for (int lv = 0; c >= 0 && lv < TREE_LEVELS; ++lv) {
        const TNode nd = T.nodes[c];
        const int i = min((C.px - nd.ox) / nd.ss, nd.m - 1);
        const int j = min((C.py - nd.oy) / nd.ss, nd.m - 1);
        ox = nd.ox + i * nd.ss;
        oy = nd.oy + j * nd.ss;
        side = nd.ss;
        c = T.tchild[nd.tab + j * nd.m + i];
    }
    const int w = h * side;
    return Rect{max(ox - w, 0), min(ox + side - 1 + w, C.W), max(oy - w, 0),
                min(oy + side - 1 + w, C.H)};
}

// Sorted-position range of the leaf (sub-)bucket that contains the point (x, y) of the box.
__device__ __forceinline__ void leaf_at(const Cell &C, const Tree &T, int x, int y, int &lo,
                                        int &hi) {
    const int bx = min(x / C.s, C.gx - 1), by = min(y / C.s, C.gy - 1);
    int k = C.boff + by * C.gx + bx;
    int c = T.tchild[k];
    for (int lv = 0; c >= 0 && lv < TREE_LEVELS; ++lv) {
        const TNode nd = T.nodes[c];
        const int i = (x - nd.ox) / nd.ss, j = (y - nd.oy) / nd.ss;
        if (x < nd.ox || y < nd.oy || i >= nd.m || j >= nd.m) {   // outside the sites' square
            lo = hi = 0;
            return;
        }
        k = nd.tab + j * nd.m + i;
        c = T.tchild[k];
    }
    lo = T.tstart[k];
    hi = T.tstart[k + 1];
}

// Next scanned region: bounding box of A and R, at most A widened by its own size per side.
__device__ __forceinline__ Rect grow_crect(const Rect &A, const Rect &R) {
    const int wx = A.x1 - A.x0 + 1, wy = A.y1 - A.y0 + 1;
    return Rect{max(min(A.x0, R.x0), A.x0 - wx), min(max(A.x1, R.x1), A.x1 + wx),
                max(min(A.y0, R.y0), A.y0 - wy), min(max(A.y1, R.y1), A.y1 + wy)};
}

// Frame stack of the depth-first leaf walk: a column per thread in LDS (one lane per cell).
template <int BLOCK>
struct LdsFrames {
    int (*f)[3][BLOCK];
    __device__ __forceinline__ void put(int d, int node, int i, int j) {
        f[d][0][threadIdx.x] = node;
        f[d][1][threadIdx.x] = i;
        f[d][2][threadIdx.x] = j;
    }
    __device__ __forceinline__ void get(int d, int &node, int &i, int &j) const {
        node = f[d][0][threadIdx.x];
        i = f[d][1][threadIdx.x];
        j = f[d][2][threadIdx.x];
    }
};

// Visits the leaves that meet region N and disk D and are not inside region O (O inside N, or
// empty), depth first; next() loads the next non-empty leaf's range into [pos, end) and sets
// `full` when every site of the leaf lies in N \ O (no per-site rectangle test needed).
struct TreeWalk {
    Rect N, O;
    Disk D;
    int node, ox, oy, ss, mx, my, tab;
    int i0, i1, j0, j1, i, j;
    int sp;
    int pos, end;
    int steps;   // sub-buckets visited so far
    bool full;

    __device__ __forceinline__ void frame(const Cell &C, const Tree &T, int nd) {
        node = nd;
        if (nd < 0) {
            ox = 0; oy = 0; ss = C.s; mx = C.gx; my = C.gy; tab = C.boff;
        } else {
            const TNode t = T.nodes[nd];
            ox = t.ox; oy = t.oy; ss = t.ss; mx = t.m; my = t.m; tab = t.tab;
        }
        // the part of N inside the disk's bounding square (whole coordinate units, widened by
        // one unit against rounding)
        int x0 = N.x0, x1 = N.x1, y0 = N.y0, y1 = N.y1;
        if (D.r2 < 1.0e30f) {
            const float r = sqrtf(D.r2) + 1.0f;
            x0 = max(x0, C.px + (int)fmaxf(floorf(D.cx - r), -(float)C.W - 2.0f));
            x1 = min(x1, C.px + (int)fminf(ceilf(D.cx + r), (float)C.W + 2.0f));
            y0 = max(y0, C.py + (int)fmaxf(floorf(D.cy - r), -(float)C.H - 2.0f));
            y1 = min(y1, C.py + (int)fminf(ceilf(D.cy + r), (float)C.H + 2.0f));
        }
        i0 = max(x0 - ox, 0) / ss;
        j0 = max(y0 - oy, 0) / ss;
        i1 = x1 < ox ? -1 : min((x1 - ox) / ss, mx - 1);
        j1 = y1 < oy ? -1 : min((y1 - oy) / ss, my - 1);
        if (x0 > x1 || y0 > y1 || i0 > i1 || j0 > j1) {
            i0 = 0; i1 = -1; j0 = 0; j1 = -1;
        }
    }
    __device__ __forceinline__ void start(const Cell &C, const Tree &T, Rect n, Rect o, Disk d) {
        N = n;
        O = o;
        D = d;
        sp = 0;
        steps = 0;
        frame(C, T, -1);
        i = i0 - 1;
        j = j0;
    }
    template <class FS>
    __device__ __forceinline__ bool next(const Cell &C, const Tree &T, FS &fs) {
        for (;;) {
            ++steps;
            if (++i > i1) {
                i = i0;
                if (++j > j1) {
                    if (sp == 0) return false;
                    int nd, ii, jj;
                    fs.get(--sp, nd, ii, jj);
                    frame(C, T, nd);
                    i = ii;
                    j = jj;
                    continue;
                }
            }
            if (node < 0 && i == i0) {
                // a grid row range without refined buckets: one contiguous range of sites
                const int k0 = tab + j * mx + i0, k1 = tab + j * mx + i1;
                if (T.tref[k1 + 1] == T.tref[k0]) {
                    i = i1;
                    const Rect cr{ox + i0 * ss, ox + i1 * ss + ss - 1, oy + j * ss,
                                  oy + j * ss + ss - 1};
                    if (rect_inside(cr, O) || !disk_meets(C, D, cr)) continue;
                    pos = T.tstart[k0];
                    end = T.tstart[k1 + 1];
                    if (pos >= end) continue;
                    full = rect_inside(cr, N) && !rect_meets(cr, O);
                    return true;
                }
            }
            const Rect cr{ox + i * ss, ox + i * ss + ss - 1, oy + j * ss, oy + j * ss + ss - 1};
            if (rect_inside(cr, O) || !disk_meets(C, D, cr)) continue;
            const int k = tab + j * mx + i;
            const int c = T.tchild[k];
            if (c >= 0) {
                fs.put(sp++, node, i, j);
                frame(C, T, c);
                i = i0 - 1;
                j = j0;
                continue;
            }
            pos = T.tstart[k];
            end = T.tstart[k + 1];
            if (pos >= end) continue;
            full = rect_inside(cr, N) && !rect_meets(cr, O);
            return true;
        }
    }
};

__device__ __forceinline__ bool in_rect(const Rect &r, float x, float y) {
    return x >= (float)r.x0 && x <= (float)r.x1 && y >= (float)r.y0 && y <= (float)r.y1;
}

}  // namespace vor
