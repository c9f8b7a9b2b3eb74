// vor_local.hpp -- local uniform grids for the cells of crowded regions.
//
// The bucket grid of Method 11.5 is sized for the mean density, so inside a cluster one bucket
// holds thousands of sites.  The refinement tree (vor_tree.hpp) follows the density, but its
// walks differ from lane to lane and a wavefront runs their union.  Here a chunk of consecutive
// sorted cells -- a compact patch, since the sorted order follows the tree -- copies every site
// of its own region (the bounding box of its cells widened by a few local spacings) into LDS
// and buckets them uniformly at the patch's own density (the better bucketing the paper's
// closing remarks call for).  Each cell then runs the same warm-block scans as the filtered
// pass, on that local grid.  The certificate of Method 11.6 is unchanged as long as the square
// S_I of a ray's bound lies inside the region, where every site of the set is present (the
// lemma on sites in the large square); a ray whose square leaves the region hands the cell on
// to the tree scans.
#pragma once
#include "vor_cell.hpp"

namespace vor {

constexpr int LOC_BLOCK = 256;      // cells per chunk (threads of a workgroup)
constexpr int LOC_CAP = 1280;       // sites of a chunk's region at most
constexpr int LOC_BCAP = 1024;      // local buckets at most (= 4 per thread, see the scan)
constexpr int LOC_RCAP = 768;       // leaf ranges of the region at most
constexpr float LOC_SPB = 1.5f;     // sites per local bucket
constexpr float LOC_MARGIN = 2.5f;  // region margin in local spacings
constexpr int LOC_GRID_MAX = 4096;  // workgroups at most (then each takes several chunks)
constexpr int LOC_NF = 2 * LOC_BLOCK;   // refined nodes per level of a region's gather at most
constexpr int LOC_GBMAX = 4096;     // grid buckets of a region at most
constexpr int LOC_MINGROUP = 64;    // a region that overflows is split down to this many cells
static_assert(LOC_BCAP == 4 * LOC_BLOCK, "the bucket scan gives each thread four buckets");
static_assert(2 * LOC_RCAP >= LOC_BCAP, "the fill counters reuse the range table");

// The local grid of a chunk.  Coordinates stay relative to the set's box origin.
struct LocalGrid {
    const float2 *xy;   // the region's sites, by local bucket (LDS)
    const int *start;   // local bucket starts, gx * gy + 1 (LDS)
    Rect RW;            // the region (inclusive): every site of the set inside it is in xy
    int ox, oy;         // corner of local bucket (0, 0) (= RW.x0, RW.y0)
    int s, gx, gy;      // bucket side, buckets per axis (gx s, gy s cover RW)
};

// Local buckets covering S_I of bound T (the coordinate square of need_crect), and whether that
// square leaves the region (then the local sites cannot certify the bound).
__device__ __forceinline__ Rect need_rect_local(const Cell &C, const LocalGrid &G, float T,
                                                float dx, float dy, bool &out) {
    const Rect Q = need_crect(C, T, dx, dy);
    out = !rect_inside(Q, G.RW);
    Rect R;
    R.x0 = min(max(Q.x0 - G.ox, 0) / G.s, G.gx - 1);
    R.x1 = min(max(Q.x1 - G.ox, 0) / G.s, G.gx - 1);
    R.y0 = min(max(Q.y0 - G.oy, 0) / G.s, G.gy - 1);
    R.y1 = min(max(Q.y1 - G.oy, 0) / G.s, G.gy - 1);
    return R;
}

// The cell as seen by its chunk's local grid: the same site and box, the local buckets.
__device__ __forceinline__ Cell local_cell(const Cell &C, const LocalGrid &G) {
    Cell L = C;
    L.s = G.s;
    L.gx = G.gx;
    L.gy = G.gy;
    L.boff = 0;
    L.h = 2;
    L.bx = min((C.px - G.ox) / G.s, G.gx - 1);
    L.by = min((C.py - G.oy) / G.s, G.gy - 1);
    return L;
}

// FP32 scans over the local grid (one lane per cell), the scheme of GridScan::scan: the block
// of shells 0..2 (or a vertex ray's own S_I rectangle inside it), then growth until the
// rectangle of the bound is covered.  Line ids are local site indices.  The pass decides in
// FP32 only (MODE 0): an uncertified ray, or a bound whose square leaves the region (heavy),
// hands the cell on, so the exact members are never called.
template <int BLOCK>
struct LocalScan {
    LocalGrid G;
    LdsRows<BLOCK> BR;
    bool heavy;
    LdsCorners<BLOCK> cs;   // the corner rays' summaries (the stack's top rows, as GridScan)
    int pre_n = -1;

    __device__ __forceinline__ void load(const Cell &C, const float2 *__restrict__ sxy) {
        BR.load(C, G.start);   // at most 5 rows (h = 2)
        heavy = false;
        corners(C, sxy);
    }

    // The corner rays' pass over the block (as GridScan::corners).
    __device__ __forceinline__ void corners(const Cell &C, const float2 *__restrict__ sxy) {
        const Dir d0 = corner_dir(0), d1 = corner_dir(1), d2 = corner_dir(2);
        Best b0{FINF, FINF, NO_TAG}, b1 = b0, b2 = b0;
        int n = 0;
        for (int r = 0; r < BR.nrows; ++r) {
            int pos, end;
            BR.get(C, G.start, r, pos, end);
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

    __device__ __forceinline__ ScanOut scan(const Cell &C, const float2 *__restrict__ sxy,
                                            float dx, float dy, int ex1, int ex2, float tcap,
                                            Counters &K, int corner = -1) {
        Best b{FINF, FINF, NO_TAG};
        const Rect A = block_rect(C);
        Rect O0 = A;
        if (tcap < FINF) {
            bool out0;
            const Rect R0 = need_rect_local(C, G, tcap, dx, dy, out0);
            if (!out0 && rect_inside(R0, A)) O0 = R0;
        }
        if (corner >= 0 && pre_n >= 0) {
            b = cs.get(corner);   // the block, from the corner pass (no bound: O0 = A)
            K.evals += (uint32_t)pre_n;
        } else {
            for (int y = O0.y0; y <= O0.y1; ++y) {
                int pos, end;
                BR.get(C, G.start, y - A.y0, pos, end);
                const int base = y * C.gx;
                if (O0.x0 != A.x0) pos = G.start[base + O0.x0];
                if (O0.x1 != A.x1) end = G.start[base + O0.x1 + 1];
                eval_range<1>(C, sxy, pos, end, dx, dy, ex1, ex2, b, K);
            }
        }
        consider_sides(C, dx, dy, ex1, ex2, b);
        K.shells++;
        float U = upper_of(C, sxy, b.w, dx, dy);
        float Uw = U;
        bool out;
        Rect R = need_rect_local(C, G, fminf(U, tcap), dx, dy, out);
        Rect O = O0;
        while (!out && !rect_inside(R, O)) {
            const Rect N = grow_rect(O, R);
            bool unused = false;
            scan_rect_f32<Solo, false>(C, sxy, G.start, N, O, dx, dy, ex1, ex2, b, K, unused);
            O = N;
            K.shells++;
            Uw = upper_of(C, sxy, b.w, dx, dy);
            U = fminf(U, Uw);
            R = need_rect_local(C, G, fminf(U, tcap), dx, dy, out);
        }
        heavy = out;
        ScanOut o;
        o.b = b;
        o.Uw = Uw;
        o.U = U;
        o.Tr = fminf(U, tcap);
        o.A = O;
        return o;
    }

    __device__ __forceinline__ void exact(const Cell &, const float2 *__restrict__, const Dir &,
                                          const ScanOut &, float, int, int, XBest &, Counters &) {}
    __device__ __forceinline__ void exact_all(const Cell &, const float2 *__restrict__,
                                              const Dir &, float, int, int, XBest &, Counters &) {}
};

// Output of a walk over local ids: the lines as sorted positions (through the chunk's table),
// entry m at dst[m * stride] as in Sink, and the count of neighbours with a larger id than the
// cell's own (its Delaunay edges).
struct LocalSink {
    int *dst;
    long long stride;
    const int *sid;
    const int *lpos;   // sorted position of each local site (LDS)
    int k;
    int up = 0;
    int lastup = 0;
    __device__ __forceinline__ void put(int m, int id) {
        const int q = id >= 0 ? lpos[id] : id;
        dst[m * stride] = q;
        const int v = q >= 0 ? sid[q] : q;
        lastup = v > k;
        up += lastup;
    }
    __device__ __forceinline__ void drop_last() { up -= lastup; }
};

// Leaf ranges of a region: first sorted position (bitwise complemented when every site of the
// leaf lies in the region: no per-site test) and the prefix of the range lengths, appended in
// parallel.  One 64-bit LDS counter holds (sites so far << 32 | ranges so far), so a range's
// slot and its prefix come from the same atomic and the prefixes grow with the slots.
struct RangeList {
    int *lo, *ofs;              // LOC_RCAP each (LDS)
    unsigned long long *rc;     // the counter (LDS)
    int *fail;                  // set on overflow (LDS)
    __device__ __forceinline__ void add(int a, int b, bool full) const {
        if (a >= b) return;
        const unsigned long long old = atomicAdd(rc, ((unsigned long long)(b - a) << 32) | 1ull);
        const int slot = (int)(old & 0xffffffffull);
        if (slot >= LOC_RCAP) {
            *fail = 1;
            return;
        }
        lo[slot] = full ? ~a : a;
        ofs[slot] = (int)(old >> 32);
    }
};

// The leaves of the refinement tree that meet region RW, breadth first over the whole
// workgroup: the grid buckets that meet RW, then level by level the sub-buckets of the refined
// ones (one round of loads per level instead of a depth-first walk of dependent loads).  The
// leaves go to `R`; `*fail` is set when a level holds more than LOC_NF refined nodes or the
// region more than LOC_GBMAX grid buckets.  Every thread calls it (barriers); the LDS scratch
// `nodeinfo` holds 2 LOC_NF frontier ids and 9 LOC_NF node fields (nodes 2t and 2t + 1 are
// thread t's).
__device__ __forceinline__ void gather_leaves(const SetDesc &S, const Tree &T, const Rect &RW,
                                              const RangeList &R, int *nodeinfo, int *nfront,
                                              int *wsum) {
    const int tid = threadIdx.x;
    int *front[2] = {nodeinfo, nodeinfo + LOC_NF};
    int *ntab = nodeinfo + 2 * LOC_NF, *nm = ntab + LOC_NF, *nox = nm + LOC_NF;
    int *noy = nox + LOC_NF, *nss = noy + LOC_NF, *ni0 = nss + LOC_NF, *nj0 = ni0 + LOC_NF;
    int *nni = nj0 + LOC_NF, *nofs = nni + LOC_NF;
    const int bx0 = RW.x0 / S.s, bx1 = min(RW.x1 / S.s, S.gx - 1);
    const int by0 = RW.y0 / S.s, by1 = min(RW.y1 / S.s, S.gy - 1);
    const int nbx = bx1 - bx0 + 1, nbb = nbx * (by1 - by0 + 1);
    if (nbb > LOC_GBMAX) {
        if (tid == 0) *R.fail = 1;
        return;   // (uniform: every thread computed the same nbb)
    }
    for (int i = tid; i < nbb; i += LOC_BLOCK) {
        const int bx = bx0 + i % nbx, by = by0 + i / nbx;
        const int k = S.bucket_off + by * S.gx + bx;
        const int c = T.tchild[k];
        if (c < 0) {
            const Rect cr{bx * S.s, bx * S.s + S.s - 1, by * S.s, by * S.s + S.s - 1};
            R.add(T.tstart[k], T.tstart[k + 1], rect_inside(cr, RW));
        } else {
            const int slot = atomicAdd(&nfront[0], 1);
            if (slot < LOC_NF) front[0][slot] = c;
            else *R.fail = 1;
        }
    }
    __syncthreads();
    for (int lv = 0; lv < TREE_LEVELS; ++lv) {
        const int cur = lv & 1;
        const int nf = nfront[cur];
        if (nf == 0 || *R.fail) return;   // uniform: read after a barrier
        int cnt[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int a = 2 * tid + h;
            if (a >= nf) continue;
            const TNode t = T.nodes[front[cur][a]];
            // the children that meet RW (the sites' square is m ss wide from (ox, oy))
            const int i0 = max(RW.x0 - t.ox, 0) / t.ss, j0 = max(RW.y0 - t.oy, 0) / t.ss;
            const int i1 = RW.x1 < t.ox ? -1 : min((RW.x1 - t.ox) / t.ss, t.m - 1);
            const int j1 = RW.y1 < t.oy ? -1 : min((RW.y1 - t.oy) / t.ss, t.m - 1);
            const int ni = i1 - i0 + 1, nj = j1 - j0 + 1;
            cnt[h] = ni > 0 && nj > 0 ? ni * nj : 0;
            ntab[a] = t.tab;
            nm[a] = t.m;
            nox[a] = t.ox;
            noy[a] = t.oy;
            nss[a] = t.ss;
            ni0[a] = i0;
            nj0[a] = j0;
            nni[a] = max(ni, 1);
        }
        if (tid == 0) nfront[cur ^ 1] = 0;
        int tot;
        const int o = block_exscan<LOC_BLOCK>(cnt[0] + cnt[1], wsum, tot);
        if (2 * tid < nf) nofs[2 * tid] = o;
        if (2 * tid + 1 < nf) nofs[2 * tid + 1] = o + cnt[0];
        __syncthreads();
        for (int idx = tid; idx < tot; idx += LOC_BLOCK) {
            int a = 0, b = nf - 1;   // the node holding child idx
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (nofs[mid] <= idx) a = mid; else b = mid - 1;
            }
            const int loc = idx - nofs[a];
            const int i = ni0[a] + loc % nni[a], j = nj0[a] + loc / nni[a];
            const int k = ntab[a] + j * nm[a] + i;
            const int c = T.tchild[k];
            if (c < 0) {
                const int cx = nox[a] + i * nss[a], cy = noy[a] + j * nss[a];
                const Rect cr{cx, cx + nss[a] - 1, cy, cy + nss[a] - 1};
                R.add(T.tstart[k], T.tstart[k + 1], rect_inside(cr, RW));
            } else {
                const int slot = atomicAdd(&nfront[cur ^ 1], 1);
                if (slot < LOC_NF) front[cur ^ 1][slot] = c;
                else *R.fail = 1;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && nfront[TREE_LEVELS & 1] != 0) *R.fail = 1;   // deeper than the tree can be
}

}  // namespace vor
