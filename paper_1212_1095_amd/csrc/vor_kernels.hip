// vor_kernels.hip -- the device pipeline of one call (one point set or a batch of sets):
//
//   prep      validate, relative coordinates, bucket of every site (Method 11.5)
//   scan      bucket counts -> bucket starts (counting sort)
//   scatter   sites into bucket order (structure of arrays, FP32 coordinates)
//   refine    buckets with many sites become grids of sub-buckets, recursively (adaptive
//             bucketing for clustered sets; the sites of every sub-bucket stay contiguous)
//   dups      equal sites share a leaf bucket: compare inside leaves (lexicographic check of
//             the distinctness remark in Appendix 2, done per leaf)
//   cells     the projector algorithm per cell, FP32 filtered; undecided cells are queued,
//             cells whose scans meet a crowded bucket are handed to the adaptive pass
//   adaptive  those cells again: on local grids of their own density (chunks of consecutive
//             cells), then the rest by scanning the refined buckets by coordinate rectangles
//   exact     queued cells again with exact fallback (or every cell, exact-only precision)
//   deep      cells deeper than the exact pass's per-worker capacity
//   scans     line counts -> CSR offsets, Delaunay counts (from the cell passes) -> offsets
//   emit      canonical rotation, neighbour ids, pair-form vertices (Section 6) and Delaunay
//             edges (i, j), i < j, sorted (Section 7), one block per 256 consecutive cells
//
// Every kernel reads the device status word first and returns when an input error is set, so
// the whole sequence can be launched (or replayed as a HIP graph) without host round trips.
#include <algorithm>

#include "vor_cell.hpp"
#include "vor_internal.h"
#include "vor_local.hpp"
#include "vor_tree.hpp"

namespace vor {

__device__ __forceinline__ int find_set(const int *__restrict__ set_off, int nsets, int pos) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (set_off[mid] <= pos) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous range of cells so
// that neighbouring cells (which read the same buckets) share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = nb >> 3;   // nb is a multiple of 8
    return (b & 7) * per + (b >> 3);
}

constexpr int KEY_BOUNDARY = 1 << 30;   // bucket key flag: the site lies on the boundary of X

__global__ void k_clear(int *__restrict__ p, long long n, int *__restrict__ small, int nsmall,
                        unsigned long long *__restrict__ stats, unsigned *__restrict__ flags,
                        long long nflags) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
    if (i < nflags) flags[i] = 0u;
    if (i < nsmall) small[i] = 0;
    if (i < SL_COUNT) stats[i] = 0;
}

__global__ void k_prep(const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
                       const SideRel *__restrict__ sides, const int *__restrict__ in_x,
                       const int *__restrict__ in_y, int total, int2 *__restrict__ xyid,
                       int *__restrict__ key, int *__restrict__ bcnt, int *__restrict__ rank,
                       int *__restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const SetDesc S = sets[find_set(set_off, nsets, i)];
    long long rx = (long long)in_x[i] - S.x0, ry = (long long)in_y[i] - S.y0;
    // in the closed X; on its boundary when on a side (the cell of such a site is computed in
    // an enlarged box and clipped to X, see k_cells_bnd)
    bool inside = rx >= 0 && rx <= S.W && ry >= 0 && ry <= S.H;
    bool onb = S.ns == 0 && (rx == 0 || rx == S.W || ry == 0 || ry == S.H);
    for (int e = 0; e < S.ns && inside; ++e) {   // inside or on every side of a polygon X
        const SideRel s = sides[S.side_off + e];
        const int64_t v = (int64_t)s.nx * rx + (int64_t)s.ny * ry;
        inside = v <= s.c;
        onb |= v == s.c;
    }
    if (!inside) {
        atomicOr(status, ST_DOMAIN);
        rx = rx < 0 ? 0 : (rx > S.W ? S.W : rx);
        ry = ry < 0 ? 0 : (ry > S.H ? S.H : ry);
        onb = false;
    }
    xyid[i] = make_int2((int)rx, (int)ry);
    const int bx = min((int)rx / S.s, S.gx - 1), by = min((int)ry / S.s, S.gy - 1);
    const int b = S.bucket_off + by * S.gx + bx;
    key[i] = b | (onb ? KEY_BOUNDARY : 0);   // bucket ids stay below 2^30
    rank[i] = atomicAdd(&bcnt[b], 1);          // the site's slot among its bucket's sites
}

// Counting-sort scatter: a site goes to its bucket's start plus the slot its count gave it (no
// atomics here).  Sites on the boundary of X are flagged by sorted position and listed for the
// boundary pass.
__global__ void k_scatter(const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
                          int total, const int2 *__restrict__ xyid, const int *__restrict__ key,
                          const int *__restrict__ bstart, const int *__restrict__ rank,
                          float2 *__restrict__ sxy, int *__restrict__ sid,
                          unsigned char *__restrict__ bflag, int *__restrict__ queue5,
                          int *__restrict__ qcount5) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int kb = key[i];
    const int b = kb & ~KEY_BOUNDARY;
    const int pos = bstart[b] + rank[i];
    const int2 r = xyid[i];
    sxy[pos] = make_float2((float)r.x, (float)r.y);
    sid[pos] = i - set_off[find_set(set_off, nsets, i)];
    if (kb & KEY_BOUNDARY) {   // the flags were cleared with the counters
        bflag[pos] = 1;
        queue5[atomicAdd(qcount5, 1)] = pos;
    }
}

// Leaf bucket of the site at sorted position pos: its first sorted position.
__device__ __forceinline__ int leaf_start(const SetDesc &S, float2 a, const int *__restrict__ tstart,
                                          const int *__restrict__ tchild,
                                          const TNode *__restrict__ nodes) {
    const int x = (int)a.x, y = (int)a.y;
    int k = S.bucket_off + min(y / S.s, S.gy - 1) * S.gx + min(x / S.s, S.gx - 1);
    int c = tchild[k];
    for (int lv = 0; c >= 0 && lv < TREE_LEVELS; ++lv) {
        const TNode nd = nodes[c];
        const int i = min((x - nd.ox) / nd.ss, nd.m - 1), j = min((y - nd.oy) / nd.ss, nd.m - 1);
        k = nd.tab + j * nd.m + i;
        c = tchild[k];
    }
    return tstart[k];
}

// Runs after the refinement; the refinement kernels return at once when an input error is
// already flagged, so their slots and nodes are not written in that call and must not be
// walked: with the status word set this kernel does nothing (the call fails anyway).
__global__ void k_dups(const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
                       int total, const float2 *__restrict__ sxy, const int *__restrict__ tstart,
                       const int *__restrict__ tchild, const TNode *__restrict__ nodes,
                       int *__restrict__ status) {
    if (*status) return;
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= total) return;
    const SetDesc S = sets[find_set(set_off, nsets, pos)];
    const float2 a = sxy[pos];
    const int lo = leaf_start(S, a, tstart, tchild, nodes);
    for (int j = lo; j < pos; ++j) {
        const float2 b = sxy[j];
        if (b.x == a.x && b.y == a.y) {
            atomicOr(status, ST_DUP);
            break;
        }
    }
}

// ------------------------------------------------------------------------------ refinement
// Set of global bucket b (sets are stored in bucket order too).
__device__ __forceinline__ int find_set_bucket(const SetDesc *__restrict__ sets, int nsets, long long b) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sets[mid].bucket_off <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Every grid bucket with more than TREE_C0 sites gets a refinement node.
__global__ void k_tree_mark0(const SetDesc *__restrict__ sets, int nsets, long long gtot,
                             const int *__restrict__ bstart, int *__restrict__ tchild,
                             int *__restrict__ refined, TNode *__restrict__ nodes, int ncap,
                             int *__restrict__ nodecnt, const int *__restrict__ status) {
    if (*status) return;
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > gtot) return;
    if (b == gtot) {
        tchild[b] = -1;
        return;
    }
    const int cnt = bstart[b + 1] - bstart[b];
    int id = -1;
    if (cnt > TREE_C0) {
        const SetDesc S = sets[find_set_bucket(sets, nsets, b)];
        const int local = (int)(b - S.bucket_off);
        id = atomicAdd(nodecnt, 1);
        if (id < ncap) {
            TNode t;
            t.ox = (local % S.gx) * S.s;
            t.oy = (local / S.gx) * S.s;
            t.size = S.s;
            t.a = bstart[b];
            t.cnt = cnt;
            t.pk = (int)b;
            t.ss = t.m = t.tab = 0;
            t.lv = 1;
            nodes[id] = t;
        } else {
            id = -1;
        }
    }
    tchild[b] = id;
    refined[b] = id >= 0 ? 1 : 0;
}

// One refinement level per launch, one block per node: a counting sort of the node's sites into
// an m x m grid of sub-buckets over their bounding square (through the scratch arrays), the
// node's sub-bucket starts, and nodes for crowded sub-buckets, listed for the next level.
// Level 1 refines the grid buckets marked by k_tree_mark0 (node ids 0..roots-1); level l > 1
// takes its node ids from list l, filled by the launch of level l - 1.
constexpr int REFINE_BLOCK = 256;
constexpr int REFINE_MAXSUB = TREE_MMAX * TREE_MMAX;

__global__ __launch_bounds__(REFINE_BLOCK) void k_tree_refine(
    TNode *__restrict__ nodes, int level, const int *__restrict__ rootcnt,
    int *__restrict__ childcnt, int *__restrict__ lvcnt, int *__restrict__ nlist, int lcap,
    int ncap, int *__restrict__ tstart, int *__restrict__ tchild, int *__restrict__ tabcnt,
    long long tab0, long long tabcap, float2 *__restrict__ sxy, int *__restrict__ sid,
    float2 *__restrict__ txy, int *__restrict__ tid, int *__restrict__ status) {
    __shared__ int cnt[REFINE_MAXSUB];
    __shared__ int pre[REFINE_MAXSUB + 1];
    __shared__ int sh_tab;
    __shared__ int sh_box[4];
    if (*status) return;
    const int nroot = min(*rootcnt, ncap);
    const int nlevel = level == 1 ? nroot : min(lvcnt[level], lcap);
    const int *mine = nlist + (size_t)max(level - 2, 0) * lcap;
    int *next = nlist + (size_t)(level - 1) * lcap;
    for (int i = blockIdx.x; i < nlevel; i += gridDim.x) {
        const int id = level == 1 ? i : mine[i];
        if (id < 0) continue;   // uniform across the block
        TNode t = nodes[id];
        // bounding square of the node's sites
        if (threadIdx.x == 0) {
            sh_box[0] = INT32_MAX; sh_box[1] = INT32_MIN; sh_box[2] = INT32_MAX;
            sh_box[3] = INT32_MIN;
        }
        __syncthreads();
        {
            int x0 = INT32_MAX, x1 = INT32_MIN, y0 = INT32_MAX, y1 = INT32_MIN;
            for (int p = t.a + threadIdx.x; p < t.a + t.cnt; p += REFINE_BLOCK) {
                const float2 q = sxy[p];
                x0 = min(x0, (int)q.x); x1 = max(x1, (int)q.x);
                y0 = min(y0, (int)q.y); y1 = max(y1, (int)q.y);
            }
            atomicMin(&sh_box[0], x0); atomicMax(&sh_box[1], x1);
            atomicMin(&sh_box[2], y0); atomicMax(&sh_box[3], y1);
        }
        __syncthreads();
        t.ox = sh_box[0];
        t.oy = sh_box[2];
        t.size = max(sh_box[1] - sh_box[0], sh_box[3] - sh_box[2]) + 1;
        // sub-buckets per axis: a power of two near sqrt(cnt), at most TREE_MMAX and the side
        int m = 2;
        while (m < TREE_MMAX && 2 * m * m <= t.cnt) m *= 2;
        m = min(m, t.size);
        const int ss = (t.size + m - 1) / m;
        const int mm = m * m;
        if (threadIdx.x == 0) {
            const int tb = atomicAdd(tabcnt, mm + 1);
            sh_tab = ((long long)tb + mm + 1 > tabcap || t.size < 2) ? -1 : tb;
            if (t.size < 2) atomicOr(status, ST_DUP);   // many sites on one lattice point
        }
        for (int k = threadIdx.x; k < mm; k += REFINE_BLOCK) cnt[k] = 0;
        __syncthreads();
        const int tb = sh_tab;
        if (tb < 0) {
            if (threadIdx.x == 0) tchild[t.pk] = -1;   // stays a leaf
            __syncthreads();
            continue;
        }
        for (int p = t.a + threadIdx.x; p < t.a + t.cnt; p += REFINE_BLOCK) {
            const float2 q = sxy[p];
            const int i2 = min(((int)q.x - t.ox) / ss, m - 1);
            const int j2 = min(((int)q.y - t.oy) / ss, m - 1);
            atomicAdd(&cnt[j2 * m + i2], 1);
        }
        __syncthreads();
        // exclusive scan of cnt[0..mm) into pre (mm <= 64): one wavefront, lane k holds cnt[k]
        static_assert(REFINE_MAXSUB <= 64, "the sub-bucket scan uses one wavefront");
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const int v = lane < mm ? cnt[lane] : 0;
            int x = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (lane < mm) pre[lane] = x - v;
            if (lane == 0) pre[mm] = t.cnt;
        }
        __syncthreads();
        const long long base = tab0 + tb;
        for (int k = threadIdx.x; k <= mm; k += REFINE_BLOCK) tstart[base + k] = t.a + pre[k];
        // scatter into the scratch arrays, then back (the range is the node's own)
        for (int k = threadIdx.x; k < mm; k += REFINE_BLOCK) cnt[k] = pre[k];
        __syncthreads();
        for (int p = t.a + threadIdx.x; p < t.a + t.cnt; p += REFINE_BLOCK) {
            const float2 q = sxy[p];
            const int i2 = min(((int)q.x - t.ox) / ss, m - 1);
            const int j2 = min(((int)q.y - t.oy) / ss, m - 1);
            const int dst = t.a + atomicAdd(&cnt[j2 * m + i2], 1);
            txy[dst] = q;
            tid[dst] = sid[p];
        }
        __syncthreads();
        for (int p = t.a + threadIdx.x; p < t.a + t.cnt; p += REFINE_BLOCK) {
            sxy[p] = txy[p];
            sid[p] = tid[p];
        }
        // children: crowded sub-buckets below the last level become nodes of the next list
        for (int k = threadIdx.x; k < mm; k += REFINE_BLOCK) {
            const int c = pre[k + 1] - pre[k];
            int cid = -1;
            if (c > TREE_C1 && level < TREE_LEVELS) {
                const int slot = atomicAdd(&lvcnt[level + 1], 1);
                if (slot < lcap) {
                    cid = nroot + atomicAdd(childcnt, 1);
                    if (cid < ncap) {
                        TNode u;
                        u.ox = t.ox + (k % m) * ss;
                        u.oy = t.oy + (k / m) * ss;
                        u.size = ss;
                        u.a = t.a + pre[k];
                        u.cnt = c;
                        u.pk = (int)(base + k);
                        u.ss = u.m = u.tab = 0;
                        u.lv = level + 1;
                        nodes[cid] = u;
                    } else {
                        cid = -1;
                    }
                    next[slot] = cid;   // -1: skipped by the next level
                }
            }
            tchild[base + k] = cid;
        }
        if (threadIdx.x == 0) {
            nodes[id].ox = t.ox;
            nodes[id].oy = t.oy;
            nodes[id].size = t.size;
            nodes[id].ss = ss;
            nodes[id].m = m;
            nodes[id].tab = (int)base;
        }
        __syncthreads();
    }
}

// POLY = false: every set of the launch has the box as X (the side code folds to the box's).
template <bool POLY = true>
__device__ __forceinline__ Cell make_cell(const SetDesc &S, float2 p,
                                          const SideRel *__restrict__ sides) {
    Cell C;
    C.gx = S.gx;
    C.gy = S.gy;
    C.s = S.s;
    C.boff = S.bucket_off;
    C.h = S.h;
    C.ht = S.ht;
    C.pxf = p.x;
    C.pyf = p.y;
    C.px = (int)p.x;
    C.py = (int)p.y;
    C.bx = min(C.px / S.s, S.gx - 1);
    C.by = min(C.py / S.s, S.gy - 1);
    C.W = S.W;
    C.H = S.H;
    C.ns = POLY ? S.ns : 0;
    C.sides = POLY ? sides + S.side_off : nullptr;
    C.grow = 0;
    return C;
}

// tree: cells taken by the adaptive pass; adaptive: the evaluations are the adaptive pass's.
__device__ __forceinline__ void reduce_stats(const Counters &K, uint32_t edges, uint32_t deferred,
                                             uint32_t tree, unsigned long long *sh,
                                             unsigned long long *stats, bool adaptive = false) {
    atomicAdd(&sh[SL_RAYS], (unsigned long long)K.rays);
    atomicAdd(&sh[SL_NODES], (unsigned long long)K.nodes);
    atomicAdd(&sh[SL_EVALS], (unsigned long long)K.evals);
    atomicAdd(&sh[SL_EXACT], (unsigned long long)K.exact);
    atomicAdd(&sh[SL_SHELLS], (unsigned long long)K.shells);
    atomicAdd(&sh[SL_EDGES], (unsigned long long)edges);
    atomicAdd(&sh[SL_DEFERRED], (unsigned long long)deferred);
    atomicAdd(&sh[SL_VTESTS], (unsigned long long)(K.vt & 0xFFFFu));
    atomicAdd(&sh[SL_XINC], (unsigned long long)K.xinc);
    atomicAdd(&sh[SL_VRAYS], (unsigned long long)(K.vt >> 16));
    if (tree) atomicAdd(&sh[SL_TREE], (unsigned long long)tree);
    if (adaptive) atomicAdd(&sh[SL_TEVALS], (unsigned long long)K.evals);
    __syncthreads();
    if (threadIdx.x < SL_COUNT && sh[threadIdx.x]) atomicAdd(&stats[threadIdx.x], sh[threadIdx.x]);
}

// Filtered pass: one thread per cell, cells in bucket order, stack in LDS.  Cells whose scans
// meet a crowded bucket go to the adaptive pass (queue3), undecided cells to the exact pass.
// Five waves per SIMD (the register budget that this asks for beats the few spills it costs).
template <int BLOCK, bool POLY>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_cells_fast(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const SideRel *__restrict__ sides,
    const float2 *__restrict__ sxy, const int *__restrict__ sid, const int *__restrict__ bstart,
    int total, int *__restrict__ ocnt, int *__restrict__ olines, int *__restrict__ ovf,
    int *__restrict__ dcnt, int *__restrict__ queue, int *__restrict__ qcount,
    int *__restrict__ queue3, int *__restrict__ qcount3, unsigned long long *__restrict__ stats,
    const unsigned char *__restrict__ bflag, unsigned char *__restrict__ hand,
    const int *__restrict__ status) {
    __shared__ int stk[SCAP][BLOCK];
    __shared__ int rlo[MAXROWS][BLOCK], rhi[MAXROWS][BLOCK];
    __shared__ unsigned long long sh[SL_COUNT];
    if (*status) return;
    if (threadIdx.x < SL_COUNT) sh[threadIdx.x] = 0;
    __syncthreads();
    const int pos = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    Counters K{};
    uint32_t edges = 0, deferred = 0;
    bool handed = false;
    if (pos < total && !bflag[pos]) {   // sites on the boundary of X: the boundary pass
        const SetDesc S = sets[find_set(set_off, nsets, pos)];
        const Cell C = make_cell<POLY>(S, sxy[pos], sides);
        const int k = sid[pos];
        const int g = S.site_off + k;
        LdsStack<BLOCK> st{stk, 0};
        // the corner rays' summaries in the stack's top nine rows (empty in the corner phase)
        static_assert(SCAP >= 9, "the stack holds the corner summaries");
        GridScan<Solo, LdsRows<BLOCK>, true, LdsCorners<BLOCK>> sc{
            LdsRows<BLOCK>{rlo, rhi, 0}, bstart, false, LdsCorners<BLOCK>{&stk[SCAP - 9]}};
        Sink sink{olines + pos, total, sid, k};
        const int r = run_cell<0, Solo>(C, sxy, sc, st, SCAP, sink, KOUT, K);
        ovf[pos] = -1;
        if (r >= 0) {
            ocnt[g] = r;
            dcnt[g] = sink.up;
            edges = (uint32_t)r;
        } else {
            ocnt[g] = -1;
            if (r == -4) {
                queue3[atomicAdd(qcount3, 1)] = pos;
                handed = true;
            } else {
                queue[atomicAdd(qcount, 1)] = pos;
                deferred = 1;
            }
        }
    }
    if (pos < total) hand[pos] = handed;   // every position written: no clearing needed
    reduce_stats(K, edges, deferred, 0, sh, stats);
}

// Adaptive pass, first part: the handed-over cells (hand[pos], or every cell with `all`) in
// chunks of LOC_BLOCK consecutive sorted positions, one workgroup per chunk and one thread per
// cell, on local grids (vor_local.hpp).  A group of the chunk's cells (at first all of them)
// takes as its region RW the bounding box of its cells widened by LOC_MARGIN local spacings;
// the workgroup gathers the leaves that meet RW level by level, copies the sites inside RW to
// LDS and buckets them at LOC_SPB sites per bucket; then every thread of the group walks its
// cell (FP32 decisions).  A region with more than LOC_CAP sites (a group that spans distant
// parts of the tree order) splits the group in halves, down to LOC_MINGROUP cells.  Cells whose
// rays leave RW or meet an uncertified decision go to queue4 (the tree scans), as do the cells
// of a group that cannot be split further and cells of a second set in the chunk; cells over the
// stack / line capacity go to the exact pass.
__global__ __launch_bounds__(LOC_BLOCK) void k_cells_local(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const SideRel *__restrict__ sides, const float2 *__restrict__ sxy,
    const int *__restrict__ sid, const int *__restrict__ tstart, const int *__restrict__ tchild,
    const TNode *__restrict__ nodes, const int *__restrict__ tref, int total,
    const unsigned char *__restrict__ hand, int all, const int *__restrict__ qcount3,
    int *__restrict__ ocnt, int *__restrict__ olines, int *__restrict__ ovf,
    int *__restrict__ dcnt, int *__restrict__ queue, int *__restrict__ qcount,
    int *__restrict__ queue4, int *__restrict__ qcount4,
    unsigned long long *__restrict__ stats, const unsigned char *__restrict__ bflag,
    const int *__restrict__ status) {
    __shared__ float2 lxy[LOC_CAP];
    __shared__ int lpos[LOC_CAP];
    __shared__ int lstart[LOC_BCAP + 1];
    // leaf ranges of the gather (first position or its complement, prefix); then the sort's
    // fill counters
    __shared__ int raux[2 * LOC_RCAP];
    // the gather's frontier and node fields; then the gathered sites, unsorted; then the
    // walks' stacks and block rows
    __shared__ int work[(SCAP + 2 * MAXROWS) * LOC_BLOCK];
    __shared__ unsigned long long sh[SL_COUNT];
    __shared__ unsigned long long s_rc;
    __shared__ int s_set, s_ncell, s_bb[4], s_cnt, s_fail, s_nf[2], s_wsum[LOC_BLOCK / 64];
    __shared__ int s_gsp, s_glo[8], s_ghi[8], s_lo, s_hi;
    static_assert(3 * LOC_CAP <= (SCAP + 2 * MAXROWS) * LOC_BLOCK, "gather staging fits");
    static_assert(11 * LOC_NF <= (SCAP + 2 * MAXROWS) * LOC_BLOCK, "gather frontier fits");
    if (*status) return;
    if (*qcount3 == 0) return;   // nothing handed over
    const int tid = threadIdx.x;
    if (tid < SL_COUNT) sh[tid] = 0;
    float2 *const txy = reinterpret_cast<float2 *>(work);
    int *const tpos = work + 2 * LOC_CAP;
    const RangeList RL{raux, raux + LOC_RCAP, &s_rc, &s_fail};
    const Tree T{tstart, tchild, nodes, tref};
    Counters K{};
    uint32_t edges = 0, deferred = 0, handled = 0;
    const int nchunks = (total + LOC_BLOCK - 1) / LOC_BLOCK;
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int pos = c * LOC_BLOCK + tid;
        const bool cand = pos < total && (all || hand[pos]) && !bflag[pos];
        // every thread is past the previous chunk here, and takes the same branch
        if (!__syncthreads_or(cand)) continue;
        const int set = cand ? find_set(set_off, nsets, pos) : nsets;
        handled += cand;
        if (tid == 0) {
            s_set = nsets;
            s_gsp = 1;
            s_glo[0] = 0;
            s_ghi[0] = LOC_BLOCK;
        }
        __syncthreads();
        if (cand) atomicMin(&s_set, set);
        __syncthreads();
        const int cs = s_set;   // the chunk's set: the smallest among its cells
        if (cand && set != cs) queue4[atomicAdd(qcount4, 1)] = pos;
        const SetDesc S = sets[cs];
        for (;;) {
            if (s_gsp == 0) break;   // uniform: the stack changes only before a barrier
            __syncthreads();         // every thread has read it
            if (tid == 0) {
                --s_gsp;
                s_lo = s_glo[s_gsp];
                s_hi = s_ghi[s_gsp];
                s_ncell = 0;
                s_bb[0] = s_bb[2] = INT32_MAX;
                s_bb[1] = s_bb[3] = INT32_MIN;
                s_fail = 0;
                s_cnt = 0;
                s_rc = 0;
                s_nf[0] = 0;
            }
            __syncthreads();
            const int glo = s_lo, ghi = s_hi;
            const bool mine = cand && set == cs && tid >= glo && tid < ghi;
            const float2 p = mine ? sxy[pos] : make_float2(0.0f, 0.0f);
            if (mine) {
                atomicAdd(&s_ncell, 1);
                atomicMin(&s_bb[0], (int)p.x);
                atomicMax(&s_bb[1], (int)p.x);
                atomicMin(&s_bb[2], (int)p.y);
                atomicMax(&s_bb[3], (int)p.y);
            }
            __syncthreads();
            if (s_ncell == 0) continue;   // uniform
            // the region: the cells' box widened by LOC_MARGIN spacings of their own density
            const float bw = (float)(s_bb[1] - s_bb[0] + 1), bh = (float)(s_bb[3] - s_bb[2] + 1);
            const int mg = (int)ceilf(LOC_MARGIN * sqrtf(bw * bh / (float)s_ncell)) + 2;
            const Rect RW{max(s_bb[0] - mg, 0), min(s_bb[1] + mg, S.W), max(s_bb[2] - mg, 0),
                          min(s_bb[3] + mg, S.H)};
            gather_leaves(S, T, RW, RL, work, s_nf, s_wsum);
            __syncthreads();
            const int nr = min((int)(s_rc & 0xffffffffull), LOC_RCAP);
            const long long ntot = (long long)(s_rc >> 32);
            bool fail = s_fail || ntot > 4 * LOC_CAP;
            if (!fail) {
                // copy the sites inside RW (unsorted) to the staging arrays
                for (int i = tid; i < (int)ntot; i += LOC_BLOCK) {
                    int lo = 0, hi = nr - 1;   // the range holding flat index i
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (RL.ofs[mid] <= i) lo = mid; else hi = mid - 1;
                    }
                    const int l0 = RL.lo[lo];
                    const int q = (l0 < 0 ? ~l0 : l0) + (i - RL.ofs[lo]);
                    const float2 a = sxy[q];
                    if (l0 < 0 || in_rect(RW, a.x, a.y)) {
                        const int slot = atomicAdd(&s_cnt, 1);
                        if (slot < LOC_CAP) {
                            txy[slot] = a;
                            tpos[slot] = q;
                        }
                    }
                }
            }
            __syncthreads();
            const int nl = s_cnt;
            fail = fail || nl > LOC_CAP;
            if (fail) {
                // split the group, or hand its cells on
                const bool split = ghi - glo > LOC_MINGROUP;
                if (split && tid == 0) {
                    const int mid = (glo + ghi) >> 1;
                    s_glo[s_gsp] = mid;
                    s_ghi[s_gsp] = ghi;
                    s_glo[s_gsp + 1] = glo;
                    s_ghi[s_gsp + 1] = mid;
                    s_gsp += 2;
                }
                if (!split && mine) queue4[atomicAdd(qcount4, 1)] = pos;
                __syncthreads();
                continue;
            }
            // local buckets at about LOC_SPB sites each, at most LOC_BCAP of them
            const int rw = RW.x1 - RW.x0 + 1, rh = RW.y1 - RW.y0 + 1;
            int sb = max(1, (int)ceilf(sqrtf((float)rw * (float)rh * LOC_SPB / (float)nl)));
            int gx = (rw + sb - 1) / sb, gy = (rh + sb - 1) / sb;
            while ((long long)gx * gy > LOC_BCAP) {
                sb += sb / 4 + 1;
                gx = (rw + sb - 1) / sb;
                gy = (rh + sb - 1) / sb;
            }
            const int nb = gx * gy, ox = RW.x0, oy = RW.y0;
            // counting sort of the staged sites by local bucket
            for (int b2 = tid; b2 <= nb; b2 += LOC_BLOCK) lstart[b2] = 0;
            for (int b2 = tid; b2 < nb; b2 += LOC_BLOCK) raux[b2] = 0;   // fill counters
            __syncthreads();
            for (int i = tid; i < nl; i += LOC_BLOCK) {
                const int bx = ((int)txy[i].x - ox) / sb, by = ((int)txy[i].y - oy) / sb;
                atomicAdd(&lstart[by * gx + bx], 1);
            }
            __syncthreads();
            {
                // exclusive scan of the nb <= 4 LOC_BLOCK counts, four per thread
                int v[4], sum = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int b2 = 4 * tid + k;
                    v[k] = b2 < nb ? lstart[b2] : 0;
                    sum += v[k];
                }
                int tot;
                int before = block_exscan<LOC_BLOCK>(sum, s_wsum, tot);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int b2 = 4 * tid + k;
                    if (b2 < nb) lstart[b2] = before;
                    before += v[k];
                }
                if (tid == 0) lstart[nb] = tot;   // = nl
            }
            __syncthreads();
            for (int i = tid; i < nl; i += LOC_BLOCK) {
                const float2 a = txy[i];
                const int bk = (((int)a.y - oy) / sb) * gx + ((int)a.x - ox) / sb;
                const int slot = lstart[bk] + atomicAdd(&raux[bk], 1);
                lxy[slot] = a;
                lpos[slot] = tpos[i];
            }
            __syncthreads();
            if (mine) {
                const Cell C = make_cell(S, p, sides);
                const LocalGrid G{lxy, lstart, RW, ox, oy, sb, gx, gy};
                const Cell CL = local_cell(C, G);
                const int k = sid[pos];
                const int g = S.site_off + k;
                int(*stk)[LOC_BLOCK] = reinterpret_cast<int(*)[LOC_BLOCK]>(work);
                int(*rlo)[LOC_BLOCK] = reinterpret_cast<int(*)[LOC_BLOCK]>(work + SCAP * LOC_BLOCK);
                int(*rhi)[LOC_BLOCK] =
                    reinterpret_cast<int(*)[LOC_BLOCK]>(work + (SCAP + MAXROWS) * LOC_BLOCK);
                LdsStack<LOC_BLOCK> st{stk, 0};
                LocalScan<LOC_BLOCK> sc{G, LdsRows<LOC_BLOCK>{rlo, rhi, 0}, false,
                                        LdsCorners<LOC_BLOCK>{stk + SCAP - 9}};
                LocalSink sink{olines + pos, total, sid, lpos, k};
                const int r = run_cell<0, Solo>(CL, lxy, sc, st, SCAP, sink, KOUT, K);
                if (r >= 0) {
                    ovf[pos] = -1;
                    ocnt[g] = r;
                    dcnt[g] = sink.up;
                    edges += (uint32_t)r;
                } else if (r == -4 || r == -1) {
                    queue4[atomicAdd(qcount4, 1)] = pos;
                } else {
                    queue[atomicAdd(qcount, 1)] = pos;
                    ++deferred;
                }
            }
            __syncthreads();   // the next group reuses the LDS
        }
    }
    __syncthreads();
    reduce_stats(K, edges, deferred, handled, sh, stats, true);
}

// Adaptive pass, second part: the cells the local grids handed on (queue4), one thread per
// cell over a persistent grid, scanning the refined buckets (TreeScan) with a per-cell candidate
// list and exact decisions in the lane.  Cells over the work budget or the stack / line capacity
// go to the exact pass.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK, 3) void k_cells_tree(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const SideRel *__restrict__ sides,
    const float2 *__restrict__ sxy, const int *__restrict__ sid, const int *__restrict__ tstart,
    const int *__restrict__ tchild, const TNode *__restrict__ nodes, const int *__restrict__ tref,
    int total, int *__restrict__ ocnt,
    int *__restrict__ olines, int *__restrict__ ovf, int *__restrict__ dcnt,
    int *__restrict__ queue, int *__restrict__ qcount, const int *__restrict__ queue4,
    const int *__restrict__ qcount4, int *__restrict__ tlist,
    unsigned long long *__restrict__ stats, const unsigned char *__restrict__ bflag,
    int *__restrict__ done, const int *__restrict__ status) {
    __shared__ int stk[SCAP][BLOCK];
    __shared__ int fr[TFRAMES][3][BLOCK];
    __shared__ unsigned long long sh[SL_COUNT];
    if (*status) return;
    const int nq = *qcount4;
    const int *const qin = queue4;
    if ((int)(blockIdx.x * BLOCK) >= nq) return;
    if (threadIdx.x < SL_COUNT) sh[threadIdx.x] = 0;
    __syncthreads();
    // the tail: all but an eighth of the workgroups that have cells are done
    const int busy = min((int)gridDim.x, (nq + BLOCK - 1) / BLOCK);
    const int tail = busy - max(1, busy / 8);
    Counters K{};
    uint32_t edges = 0, deferred = 0;
    for (int qi = blockIdx.x * BLOCK + threadIdx.x; qi < nq; qi += gridDim.x * BLOCK) {
        const int pos = qin[qi];
        if (bflag[pos]) continue;   // the boundary pass takes it
        const SetDesc S = sets[find_set(set_off, nsets, pos)];
        const Cell C = make_cell(S, sxy[pos], sides);
        const int k = sid[pos];
        const int g = S.site_off + k;
        LdsStack<BLOCK> st{stk, 0};
        TreeScan<Solo, LdsFrames<BLOCK>, GlobalList<TREE_LIST>> sc{
            Tree{tstart, tchild, nodes, tref}, LdsFrames<BLOCK>{fr},
            GlobalList<TREE_LIST>{tlist + blockIdx.x * BLOCK + threadIdx.x,
                                  (int)(gridDim.x * BLOCK)},
            Rect{}, false, Rect{}, 0, false};
        sc.done = done;
        sc.tail = tail;
        Sink sink{olines + pos, total, sid, k};
        const int r = run_cell<1, Solo>(C, sxy, sc, st, SCAP, sink, KOUT, K);
        if (r >= 0) {
            ovf[pos] = -1;
            ocnt[g] = r;
            dcnt[g] = sink.up;
            edges += (uint32_t)r;
        } else {
            queue[atomicAdd(qcount, 1)] = pos;
            ++deferred;
        }
    }
    reduce_stats(K, edges, deferred, 0, sh, stats, true);   // ends with a barrier
    if (threadIdx.x == 0) atomicAdd(done, 1);
}

// Every cell into a queue, in bucket order.
__global__ void k_queue_all(int total, int *__restrict__ queue, int *__restrict__ qcount,
                            const int *__restrict__ status) {
    if (*status) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) queue[i] = i;
    if (i == 0) *qcount = total;
}

// One cell by one wave (the Coop policy) with scanner Sc; the cell's stack and output live in
// `area` (dcap entries each).
template <int MODE, class Sc>
__device__ __forceinline__ int coop_cell(const Cell &C, const float2 *__restrict__ sxy,
                                         const int *__restrict__ sid, int k, Sc &sc, int *area,
                                         int dcap, Counters &K, int &up) {
    GStack st{area, 0};
    Sink sink{area + dcap, 1, sid, k};
    const int r = run_cell<MODE, Coop>(C, sxy, sc, st, dcap, sink, dcap, K);
    up = sink.up;
    return r;
}

// Exact pass over a queue of cells: one wave per cell (the Coop policy), a persistent grid of
// one-wave blocks.  The scans run over the uniform grid even where buckets were refined: with
// 64 lanes a crowded bucket is read in coalesced rows, which beats walking its sub-buckets.
// LCAP > 0: the stack and output of a cell live in LDS (LCAP entries each, the usual pass);
// LCAP == 0: in the block's area of wbuf (dcap entries each, the deep pass).
template <int MODE, int LCAP>
__global__ __launch_bounds__(64) void k_cells_exact(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const SideRel *__restrict__ sides,
    const float2 *__restrict__ sxy, const int *__restrict__ sid, const int *__restrict__ bstart,
    int total, int *__restrict__ ocnt, int *__restrict__ olines, int *__restrict__ dcnt,
    int *__restrict__ ovf, int *__restrict__ pool, int *__restrict__ poolcnt, long long poolcap,
    const int *__restrict__ queue, const int *__restrict__ qcount, int *__restrict__ queue2,
    int *__restrict__ qcount2, int *__restrict__ wbuf, int dcap,
    unsigned long long *__restrict__ stats, const unsigned char *__restrict__ bflag,
    int *__restrict__ status, int skip_upto) {
    __shared__ unsigned long long sh[SL_COUNT];
    __shared__ int larea[LCAP > 0 ? 2 * LCAP : 1];
    if (*status & (ST_DOMAIN | ST_DUP)) return;
    const int nq = *qcount;
    if ((int)blockIdx.x >= nq) return;   // no cell for this worker
    if (nq <= skip_upto) return;         // the workgroup-per-cell pass took them
    if (threadIdx.x < SL_COUNT) sh[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x;
    int *area = LCAP > 0 ? larea : wbuf + (size_t)blockIdx.x * 2 * dcap;
    if (LCAP > 0) dcap = LCAP;
    Counters K{};
    uint32_t edges = 0;
    for (int qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const int pos = queue[qi];
        if (bflag[pos]) continue;   // the boundary pass takes it
        const SetDesc S = sets[find_set(set_off, nsets, pos)];
        const Cell C = make_cell(S, sxy[pos], sides);
        const int k = sid[pos];
        const int g = S.site_off + k;
        GridScan<Coop, GlobalRows, false> sc{GlobalRows{0}, bstart, false};
        int up = 0;
        const int r = coop_cell<MODE>(C, sxy, sid, k, sc, area, dcap, K, up);
        if (r == -2) {
            if (lane == 0) {
                if (queue2) queue2[atomicAdd(qcount2, 1)] = pos;
                else atomicOr(status, ST_CAPACITY);
            }
            continue;
        }
        if (r < 0) {
            if (lane == 0) atomicOr(status, ST_INTERNAL);
            continue;
        }
        edges += (uint32_t)r;
        const int *src = area + dcap;
        int off = -1;
        if (r > KOUT) {
            if (lane == 0) off = atomicAdd(poolcnt, r);
            off = __shfl(off, 0, 64);
            if ((long long)off + r > poolcap) {
                if (lane == 0) atomicOr(status, ST_CAPACITY);
                continue;
            }
        }
        int *dst = off >= 0 ? pool + off : olines + pos;
        const long long stride = off >= 0 ? 1 : total;
        for (int t = lane; t < r; t += 64) dst[t * stride] = src[t];
        if (lane == 0) {
            ovf[pos] = off;
            ocnt[g] = r;
            dcnt[g] = up;
        }
    }
    // every lane ran the same control flow: count it once; evaluations are split across lanes
    if (lane != 0) {
        K.rays = K.nodes = K.exact = K.shells = K.vt = K.xinc = 0;
        edges = 0;
    }
    reduce_stats(K, edges, 0, 0, sh, stats);
}

// Cells with the subwedges of one cell spread over the waves of a workgroup (the parallel case
// of Appendix 2: several processing units share one cell's projector).  The cell's corners form
// a counter-clockwise linked list (line of each corner, next corner); a subedge is a corner and
// its successor.  Rounds: every pending subedge is resolved by one wave (its 64 lanes split the
// candidate scans), a new corner is spliced in between its two corners and both halves become
// pending in the next round; a barrier ends the round.  Two waves never touch the same corner's
// successor link, since each owns the subedge that starts there.  After the last round one lane
// walks the list and writes the corners' lines with repeats removed: the same cyclic list the
// depth-first walk yields (the set of prime subedges does not depend on the order they are
// resolved in).  A cell then takes a few rounds instead of one ray after another, which is what
// bounds a pass over few cells.
// CAP > 0: the deferred cells of the filtered passes (queue), lists in LDS (CAP corners each);
// a cell with more corners goes to queue2.  CAP == 0: the deep cells (queue2), lists in the
// block's area of wbuf (WIDE_CAP corners each: corner lines, successor links, two frontiers).
// The deferred-cell pass runs only when it has at most WIDE_QMAX cells (a pass over few cells
// is bound by the slowest cell); the one-wave-per-cell pass takes larger queues, where the
// waves that idle in the early rounds would cost more than the shorter chain of rays saves.
constexpr int WIDE_QMAX = 16384;    // deferred cells up to which the workgroup-per-cell pass runs
constexpr int WIDE_LCAP = 256;      // corners of a deferred cell in that pass (LDS lists)
constexpr int WIDE_LWAVES = 4;      // waves of its workgroups
constexpr int WIDE_LBLOCKS = 2048;  // its workgroups
constexpr int ERR_SPILL = 1 << 30;  // a deferred cell with more corners than the LDS lists hold

// Four waves per SIMD: the register budget this asks for (128) costs the deferred-cell pass no
// spill (the deep pass a few), and a pass over thousands of deferred cells keeps a third more
// of them in flight than at three.
template <int MODE, int CAP, int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_cells_wide(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const SideRel *__restrict__ sides,
    const float2 *__restrict__ sxy, const int *__restrict__ sid, const int *__restrict__ bstart,
    int total, int *__restrict__ ocnt, int *__restrict__ olines, int *__restrict__ dcnt,
    int *__restrict__ ovf, int *__restrict__ pool, int *__restrict__ poolcnt, long long poolcap,
    const int *__restrict__ queue, const int *__restrict__ qcount, int *__restrict__ wbuf,
    int *__restrict__ queue2, int *__restrict__ qcount2, const unsigned char *__restrict__ bflag,
    unsigned long long *__restrict__ stats, int *__restrict__ status) {
    constexpr int WCAP = CAP > 0 ? CAP : WIDE_CAP;
    __shared__ unsigned long long sh[SL_COUNT];
    __shared__ int fcount[2], ncorner, err, s_m, s_up, s_off;
    __shared__ int lists[CAP > 0 ? 4 * CAP : 1];
    if (*status & (ST_DOMAIN | ST_DUP)) return;
    const int nq = *qcount;
    if ((int)blockIdx.x >= nq) return;   // no cell for this worker
    if (CAP > 0 && nq > WIDE_QMAX) return;   // the one-wave-per-cell pass takes them
    if (threadIdx.x < SL_COUNT) sh[threadIdx.x] = 0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int *cline = CAP > 0 ? lists : wbuf + (size_t)blockIdx.x * 4 * WIDE_CAP;
    int *nxt = cline + WCAP;
    int *F[2] = {nxt + WCAP, nxt + 2 * WCAP};
    Counters K{};
    uint32_t edges = 0;
    for (int qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const int pos = queue[qi];
        if (CAP > 0 && bflag[pos]) continue;   // the boundary pass takes it (uniform: one pos)
        const SetDesc S = sets[find_set(set_off, nsets, pos)];
        const Cell C = make_cell(S, sxy[pos], sides);
        const int k = sid[pos];
        const int g = S.site_off + k;
        GridScan<Coop, GlobalRows, false> sc{GlobalRows{0}, bstart, false};
        sc.load(C, sxy);
        __syncthreads();   // the previous cell's list is no longer read
        if (threadIdx.x == 0) {
            ncorner = 3;
            err = 0;
            fcount[0] = 3;
            fcount[1] = 0;
        }
        // round 0: the projector's three corner rays, one wave each
        if (wave < 3) {
            Line L{};
            ray<MODE, Coop>(C, sc, sxy, corner_dir(wave), 0, INT32_MIN, INT32_MIN, L, K);
            K.rays++;
            if (lane == 0) {
                cline[wave] = L.id;
                nxt[wave] = wave == 2 ? 0 : wave + 1;
                F[0][wave] = wave;
            }
        }
        __threadfence_block();   // the lists are shared by this workgroup's waves only
        __syncthreads();
        int cur = 0;
        while (fcount[cur] > 0 && !err) {
            const int nf = fcount[cur];
            for (int f = wave; f < nf; f += WAVES) {
                const int i = F[cur][f];
                const int j = nxt[i];
                const Line L1 = make_line(C, sxy, cline[i]), L2 = make_line(C, sxy, cline[j]);
                K.nodes++;
                if (L1.id == L2.id) continue;   // SameLines
                Dir d;
                int64_t Den;
                int ex1 = INT32_MIN, ex2 = INT32_MIN;
                split_dir(L1, L2, d, Den, ex1, ex2);
                Line L3{};
                const int r = ray<MODE, Coop>(C, sc, sxy, d, Den, ex1, ex2, L3, K);
                K.vt += Den > 0 ? VT_VRAY : 0u;
                if (r == 1) {   // u is a vertex of the cell: the subedge is prime
                    K.vt++;
                    continue;
                }
                K.rays++;
                int nk = 0;
                if (lane == 0) nk = atomicAdd(&ncorner, 1);
                nk = __shfl(nk, 0, 64);
                if (nk >= WCAP || r < 0) {
                    if (lane == 0)
                        atomicOr(&err, r < 0 ? ST_INTERNAL : CAP > 0 ? ERR_SPILL : ST_CAPACITY);
                    continue;
                }
                if (lane == 0) {
                    cline[nk] = L3.id;
                    nxt[nk] = j;
                    nxt[i] = nk;
                    const int at = atomicAdd(&fcount[cur ^ 1], 2);
                    F[cur ^ 1][at] = i;
                    F[cur ^ 1][at + 1] = nk;
                }
            }
            __threadfence_block();
            __syncthreads();
            if (threadIdx.x == 0) fcount[cur] = 0;
            cur ^= 1;
            __syncthreads();
        }
        if (err) {
            if (threadIdx.x == 0) {
                if (err & ~ERR_SPILL) atomicOr(status, err & ~ERR_SPILL);
                else queue2[atomicAdd(qcount2, 1)] = pos;   // to the deep pass
            }
            continue;   // uniform across the block (err is read after the last barrier)
        }
        // the cyclic list of distinct lines, counter-clockwise from corner 0 (into F[0])
        if (threadIdx.x == 0) {
            int m = 0, up = 0, last = INT32_MIN, c = 0;
            const int first = cline[0];
            do {
                const int id = cline[c];   // sorted position or side code
                if (id != last) {
                    F[0][m++] = id;
                    up += (id >= 0 ? sid[id] : id) > k;
                    last = id;
                }
                c = nxt[c];
            } while (c != 0);
            if (m > 1 && last == first) {
                --m;
                up -= (last >= 0 ? sid[last] : last) > k;
            }
            int off = -1;
            if (m > KOUT) {
                off = atomicAdd(poolcnt, m);
                if ((long long)off + m > poolcap) {
                    atomicOr(status, ST_CAPACITY);
                    m = -1;
                }
            }
            s_m = m;
            s_up = up;
            s_off = off;
        }
        __threadfence_block();
        __syncthreads();
        const int m = s_m, off = s_off;
        if (m < 0) continue;
        int *dst = off >= 0 ? pool + off : olines + pos;
        const long long stride = off >= 0 ? 1 : total;
        for (int t = threadIdx.x; t < m; t += blockDim.x) dst[t * stride] = F[0][t];
        if (threadIdx.x == 0) {
            ovf[pos] = off;
            ocnt[g] = m;
            dcnt[g] = s_up;
            edges += (uint32_t)m;
        }
    }
    // every lane of a wave ran the same control flow: count it once; evaluations are split
    // across the lanes
    if (lane != 0) {
        K.rays = K.nodes = K.exact = K.shells = K.vt = K.xinc = 0;
        edges = 0;
    }
    reduce_stats(K, edges, 0, 0, sh, stats);
}

// ------------------------------------------------------------------------------ boundary sites
// Cells of sites on the boundary of X (the definition of a cell extends to them unchanged; the
// problem statement of Section 2 notes it).  The projector needs a ray origin strictly inside
// the region, so such a cell is computed in the box grown by one unit on every side, which holds
// every site strictly inside (the embedding in a larger region of the paper's remark on a
// non-polygonal X, Section 10: the cells in the larger region intersected with X are the cells
// in X); the sites all lie in X's grid, so the scans and their certificates are unchanged.  The
// cell is then intersected with X one side at a time, exactly: for the vertices of consecutive
// lines the sign of side - vertex in 128-bit integers; an edge is kept when one of its ends is
// strictly inside; the side's line goes in once where the part outside begins.
constexpr int BND_BLOCKS = 64;     // one-wave workers of the boundary pass
constexpr int BND_CAP = DCAP1;     // lines of such a cell in the grown box (more: capacity error)
constexpr int BND_LIST = BND_CAP + 256 + 8;   // lines after the intersection, at most (a polygon
                                                 // X has at most 256 sides)
constexpr int BND_XCODE = 1024;    // an inserted side e of X is named -(e+1) - BND_XCODE until
                                   // the output (grown-box sides keep -1..-4)

__device__ __forceinline__ Line bnd_line(const Cell &Cg, const Cell &Cx,
                                         const float2 *__restrict__ sxy, int id) {
    if (id >= 0) return site_line(Cg, sxy, id);
    if (id < -BND_XCODE) {
        Line L = side_line(Cx, id + BND_XCODE);
        L.id = id;
        return L;
    }
    return side_line(Cg, id);
}

// Sign of line L at the vertex of the consecutive lines A, B (p's doubled frame): with
// Den = cross(N_A, N_B) > 0 and the vertex Z / Den, sign(c_L Den - N_L . Z): +1 inside, 0 on,
// -1 outside.  |c Den| < 2^103 and |N . Z| < 2^101.
__device__ __forceinline__ int vertex_side(const Line &A, const Line &B, const Line &L) {
    const int64_t Den = (int64_t)A.nx * B.ny - (int64_t)A.ny * B.nx;
    const i128 Zx = (i128)A.c * B.ny - (i128)B.c * A.ny;
    const i128 Zy = (i128)A.nx * B.c - (i128)B.nx * A.c;
    const i128 v = (i128)L.c * Den - ((i128)L.nx * Zx + (i128)L.ny * Zy);
    return v > 0 ? 1 : (v < 0 ? -1 : 0);
}

// The cyclic list lin[0..m) intersected with the half-plane of line `xs` into lout; sgn is
// scratch for m vertex signs.  Returns the new count.
__device__ int clip_side(const Cell &Cg, const Cell &Cx, const float2 *__restrict__ sxy,
                         const int *lin, int m, int xs, int *lout, int *sgn) {
    const Line H = bnd_line(Cg, Cx, sxy, xs);
    bool out = false;
    Line A = bnd_line(Cg, Cx, sxy, lin[0]);
    const Line L0 = A;
    for (int i = 0; i < m; ++i) {   // vertex i between lines i and i + 1
        const Line B = i + 1 < m ? bnd_line(Cg, Cx, sxy, lin[i + 1]) : L0;
        sgn[i] = vertex_side(A, B, H);
        out |= sgn[i] < 0;
        A = B;
    }
    if (!out) {
        for (int i = 0; i < m; ++i) lout[i] = lin[i];
        return m;
    }
    // edge t lies on line t, from vertex t - 1 to vertex t; start at a kept edge (one exists:
    // a convex cell that meets the open half-plane has a vertex strictly inside it)
    int t0 = 0;
    while (t0 < m && max(sgn[(t0 + m - 1) % m], sgn[t0]) <= 0) ++t0;
    if (t0 == m) return -1;
    int k = 0;
    bool put = false;
    lout[k++] = lin[t0];
    for (int j = 1; j < m; ++j) {
        const int t = (t0 + j) % m, v = (t + m - 1) % m;
        if (!put && sgn[v] < 0) {
            lout[k++] = xs;
            put = true;
        }
        if (max(sgn[v], sgn[t]) > 0) lout[k++] = lin[t];
    }
    if (!put) lout[k++] = xs;   // the part outside is at the vertex before edge t0
    return k;
}

template <int MODE>
__global__ __launch_bounds__(64) void k_cells_bnd(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const SideRel *__restrict__ sides,
    const float2 *__restrict__ sxy, const int *__restrict__ sid, const int *__restrict__ bstart,
    int total, int *__restrict__ ocnt, int *__restrict__ olines, int *__restrict__ dcnt,
    int *__restrict__ ovf, int *__restrict__ pool, int *__restrict__ poolcnt, long long poolcap,
    const int *__restrict__ queue, const int *__restrict__ qcount,
    unsigned long long *__restrict__ stats, int *__restrict__ status) {
    __shared__ unsigned long long sh[SL_COUNT];
    __shared__ int area[2 * BND_CAP];
    __shared__ int la[BND_LIST], lb[BND_LIST], sg[BND_LIST];
    if (*status & (ST_DOMAIN | ST_DUP)) return;
    const int nq = *qcount;
    if ((int)blockIdx.x >= nq) return;
    if (threadIdx.x < SL_COUNT) sh[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x;
    Counters K{};
    uint32_t edges = 0;
    for (int qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const int pos = queue[qi];
        const SetDesc S = sets[find_set(set_off, nsets, pos)];
        const Cell Cx = make_cell(S, sxy[pos], sides);   // X itself
        Cell Cg = Cx;                                     // the grown box
        Cg.ns = 0;
        Cg.sides = nullptr;
        Cg.grow = 1;
        const int k = sid[pos];
        const int g = S.site_off + k;
        GridScan<Coop, GlobalRows, false> sc{GlobalRows{0}, bstart, false};
        GStack st{area, 0};
        PosSink sink{area + BND_CAP};
        const int r = run_cell<MODE, Coop>(Cg, sxy, sc, st, BND_CAP, sink, BND_CAP, K);
        if (r < 0) {
            if (lane == 0) atomicOr(status, r == -2 ? ST_CAPACITY : ST_INTERNAL);
            continue;
        }
        // the grown-box cell intersected with X (lane 0; a few lines and sides)
        int m = 0, up = 0, off = -1;
        if (lane == 0) {
            m = r;
            for (int t = 0; t < m; ++t) la[t] = area[BND_CAP + t];
            int *cur = la, *nxt = lb;
            const int ns = Cx.ns > 0 ? Cx.ns : 4;
            for (int e = 0; e < ns && m > 0; ++e) {
                if (m + 1 > BND_LIST) {
                    m = -2;
                    break;
                }
                m = clip_side(Cg, Cx, sxy, cur, m, -(e + 1) - BND_XCODE, nxt, sg);
                int *t = cur;
                cur = nxt;
                nxt = t;
            }
            // names -> output: sorted positions, sides of X; no grown-box side may remain
            for (int t = 0; t < m; ++t) {
                const int id = cur[t];
                int v;
                if (id >= 0) v = id;
                else if (id < -BND_XCODE) v = id + BND_XCODE;
                else {
                    m = -1;
                    break;
                }
                la[t] = v;
                up += (v >= 0 ? sid[v] : v) > k;
            }
            if (m > KOUT) {
                off = atomicAdd(poolcnt, m);
                if ((long long)off + m > poolcap) m = -2;
            }
            if (m < 0) atomicOr(status, m == -2 ? ST_CAPACITY : ST_INTERNAL);
        }
        m = __shfl(m, 0, 64);
        off = __shfl(off, 0, 64);
        if (m < 0) continue;
        int *dst = off >= 0 ? pool + off : olines + pos;
        const long long stride = off >= 0 ? 1 : total;
        for (int t = lane; t < m; t += 64) dst[t * stride] = la[t];
        if (lane == 0) {
            ovf[pos] = off;
            ocnt[g] = m;
            dcnt[g] = up;
            edges += (uint32_t)m;
        }
    }
    if (lane != 0) {
        K.rays = K.nodes = K.exact = K.shells = K.vt = K.xinc = 0;
        edges = 0;
    }
    reduce_stats(K, edges, 0, 0, sh, stats);
}

// ------------------------------------------------------------------------------ scan
// Exclusive scan of n int32 values (>= 0) into out[0..n], out[n] = total.  Three launches:
// block sums, a single-block scan of the sums, per-block scan plus offset.


__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const int *__restrict__ in, long long n,
                                                            int *__restrict__ bsum,
                                                            const int *__restrict__ status,
                                                            int gate) {
    __shared__ int sh[SCAN_BLOCK / 64 + 1];
    if (gate && *status) return;
    const long long base = (long long)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int v = 0;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t)
        if (base + t < n) v += in[base + t];
    int total;
    (void)block_exscan<SCAN_BLOCK>(v, sh, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_top(int *__restrict__ bsum, int nb,
                                                         const int *__restrict__ status, int gate) {
    __shared__ int sh[SCAN_BLOCK / 64 + 1];
    if (gate && *status) return;
    int carry = 0;
    for (int base = 0; base < nb; base += SCAN_BLOCK) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int total;
        const int e = block_exscan<SCAN_BLOCK>(v, sh, total);
        if (i < nb) bsum[i] = e + carry;
        carry += total;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const int *__restrict__ in, long long n,
                                                           const int *__restrict__ bsum,
                                                           int *__restrict__ out,
                                                           const int *__restrict__ status,
                                                           int gate, int *__restrict__ tot) {
    __shared__ int sh[SCAN_BLOCK / 64 + 1];
    if (gate && *status) return;
    const long long base = (long long)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        v[t] = base + t < n ? in[base + t] : 0;
        s += v[t];
    }
    int total;
    int e = block_exscan<SCAN_BLOCK>(s, sh, total) + bsum[blockIdx.x];
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        if (base + t < n) out[base + t] = e;
        e += v[t];
        if (base + t == n - 1) {
            out[n] = e;
            if (tot) *tot = e;
        }
    }
}

// ------------------------------------------------------------------------------ output
// Absolute line N.x <= c of neighbour j of the cell whose site is at relative p (site lines:
// N = 2 (q - p), c = |q|^2 - |p|^2 with q the neighbour's site; sides: primitive outward normal,
// unit for the box).
__device__ __forceinline__ void abs_line(const SetDesc &S, const SideRel *__restrict__ sides,
                                         int2 p, int j, int2 q, long long &nx, long long &ny,
                                         long long &c) {
    const long long px = (long long)p.x + S.x0, py = (long long)p.y + S.y0;
    if (j < 0 && S.ns > 0) {
        const SideRel s = sides[S.side_off - j - 1];
        nx = s.nx;
        ny = s.ny;
        c = s.c + (long long)s.nx * S.x0 + (long long)s.ny * S.y0;
    } else if (j >= 0) {
        const long long qx = (long long)q.x + S.x0, qy = (long long)q.y + S.y0;
        nx = 2 * (qx - px);
        ny = 2 * (qy - py);
        c = (qx * qx + qy * qy) - (px * px + py * py);
    } else if (j == -1) {
        nx = 0; ny = -1; c = -(long long)S.y0;
    } else if (j == -2) {
        nx = 1; ny = 0; c = (long long)S.x0 + S.W;
    } else if (j == -3) {
        nx = 0; ny = 1; c = (long long)S.y0 + S.H;
    } else {
        nx = -1; ny = 0; c = -(long long)S.x0;
    }
}

struct Rat {
    uint64_t x_lo;
    int64_t x_hi;
    uint64_t y_lo;
    int64_t y_hi;
    int64_t d;
};

// Vertex of lines 1 and 2 in pair form (X/D, Y/D), Cramer's rule.
__device__ __forceinline__ Rat pair_vertex(const SetDesc &S, const SideRel *__restrict__ sides,
                                           int2 p, int a, int2 qa, int b, int2 qb) {
    long long n1x, n1y, c1, n2x, n2y, c2;
    abs_line(S, sides, p, a, qa, n1x, n1y, c1);
    abs_line(S, sides, p, b, qb, n2x, n2y, c2);
    const i128 X = (i128)c1 * n2y - (i128)c2 * n1y;
    const i128 Y = (i128)n1x * c2 - (i128)n2x * c1;
    Rat v;
    v.x_lo = (uint64_t)X;
    v.x_hi = (int64_t)(X >> 64);
    v.y_lo = (uint64_t)Y;
    v.y_hi = (int64_t)(Y >> 64);
    v.d = n1x * n2y - n1y * n2x;
    return v;
}

constexpr int EMIT_BLOCK = 256;   // cells per block (consecutive sorted positions)
constexpr int EMIT_ECAP = 2048;   // CSR entries staged per block (mean about 6 per cell)
static_assert(EMIT_BLOCK <= 256, "a byte names a block's cell");

// Line t of the cell at sorted position pos: sorted position of the neighbour's site, or side code
// (the cell passes store entry-major by position; cells with more than KOUT lines in the pool).
__device__ __forceinline__ int cell_line(const int *__restrict__ olines,
                                         const int *__restrict__ pool, long long total, int pos,
                                         int of, int t) {
    return of >= 0 ? pool[of + t] : olines[(long long)t * total + pos];
}

// Cell by cell (blocks whose entries exceed the LDS capacity: cells with very many edges).
// Returns false, writing nothing, when the neighbours > k are not the dn the cell pass counted.
template <bool VERT>
__device__ bool emit_cell(const SetDesc &S, const SideRel *__restrict__ sides, int k, int2 p,
                          const int *__restrict__ olines, const int *__restrict__ pool,
                          long long total, int pos, int of, int m, int dn, long long base,
                          long long dbase, const int *__restrict__ sid,
                          const float2 *__restrict__ sxy, int *__restrict__ nbr,
                          Rat *__restrict__ vtx, unsigned *__restrict__ del) {
    auto id = [&](int t) {
        const int q = cell_line(olines, pool, total, pos, of, t);
        return q >= 0 ? sid[q] : q;
    };
    auto xy = [&](int t) {
        const int q = cell_line(olines, pool, total, pos, of, t);
        return q >= 0 ? make_int2((int)sxy[q].x, (int)sxy[q].y) : make_int2(0, 0);
    };
    int r = 0, up = 0, rid = id(0);
    for (int t = 0; t < m; ++t) {
        const int j = id(t);
        if ((uint32_t)j < (uint32_t)rid) {
            r = t;
            rid = j;
        }
        up += j > k;
    }
    if (up != dn) return false;
    for (int t = 0; t < m; ++t) nbr[base + t] = id((r + t) % m);
    if (VERT)
        for (int t = 0; t < m; ++t) {
            const int ta = (r + t) % m, tb = (r + t + 1) % m;
            vtx[base + t] = pair_vertex(S, sides, p, id(ta), xy(ta), id(tb), xy(tb));
        }
    for (int t = 0; t < m; ++t) {   // Delaunay pairs: rank of each neighbour > k
        const int j = id(t);
        if (j <= k) continue;
        int rank = 0;
        for (int u = 0; u < m; ++u) {
            const int v = id(u);
            rank += v > k && v < j;
        }
        del[2 * (dbase + rank)] = (unsigned)k;
        del[2 * (dbase + rank) + 1] = (unsigned)j;
    }
    return true;
}

// Output of 256 consecutive cells in sorted order: the canonical rotation of each cell's lines
// (the entry smallest as uint32 first), the neighbour ids, the pair-form vertices (Section 6)
// and the Delaunay pairs (k, j), k < j, ascending (Section 7).  Taking the cells in sorted order
// keeps the neighbours' sites of a block within a few rows of buckets, so their ids and
// coordinates come from cache; the block's lines are read entry by entry into LDS, the rotation
// and the Delaunay order are found there, and each entry then writes its CSR slot (at the cell's
// offset by id), its vertex and its Delaunay pair.  A block whose entries exceed the LDS
// capacity works cell by cell instead.
template <bool VERT>
__global__ __launch_bounds__(EMIT_BLOCK) void k_emit(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const SideRel *__restrict__ sides, int total, const int *__restrict__ sid,
    const float2 *__restrict__ sxy, const int *__restrict__ olines, const int *__restrict__ ovf,
    const int *__restrict__ pool, const int *__restrict__ cell_off, long long cap,
    const int *__restrict__ del_off, long long del_cap, int *__restrict__ nbr,
    Rat *__restrict__ vtx, unsigned *__restrict__ del, int *__restrict__ status) {
    __shared__ int lin[EMIT_ECAP];
    __shared__ unsigned char own[EMIT_ECAP];
    __shared__ int2 qc[VERT ? EMIT_ECAP : 1];
    __shared__ int clo[EMIT_BLOCK + 1];
    __shared__ long long cbase[EMIT_BLOCK], cdel[EMIT_BLOCK];
    __shared__ int ck[EMIT_BLOCK], cof[EMIT_BLOCK], crot[EMIT_BLOCK], cset[EMIT_BLOCK];
    __shared__ int2 pc[EMIT_BLOCK];
    __shared__ int bad, stop, s_wsum[EMIT_BLOCK / 64];
    const int tid = threadIdx.x;
    const int pos0 = blockIdx.x * EMIT_BLOCK;
    const int nc = min(EMIT_BLOCK, total - pos0);
    const int pos = pos0 + tid;
    if (tid == 0) {
        stop = *status;   // one read, so that every wave of the block takes the same branch
        bad = 0;
        // more entries or Delaunay pairs in the run than the buffers hold (the sizes follow
        // from Euler's formula, so this is a capacity error, never an internal one)
        if (!stop && ((long long)cell_off[total] > cap || (long long)del_off[total] > del_cap)) {
            atomicOr(status, ST_CAPACITY);
            stop = ST_CAPACITY;
        }
    }
    __syncthreads();
    if (stop) return;
    // per cell: its id, offsets and line source
    int s = 0, k = 0, m = 0, dn = 0, of = -1;
    long long base = 0, dbase = 0;
    int2 p = make_int2(0, 0);
    if (tid < nc) {
        s = find_set(set_off, nsets, pos);
        k = sid[pos];
        const int g = set_off[s] + k;
        base = cell_off[g];
        m = cell_off[g + 1] - (int)base;
        dbase = del_off[g];
        dn = del_off[g + 1] - (int)dbase;
        of = ovf[pos];
        const float2 a = sxy[pos];
        p = make_int2((int)a.x, (int)a.y);
        if (m < 3 || base + m > cap || dn < 0 || dbase + dn > del_cap || (of < 0 && m > KOUT)) {
            bad = 1;
            m = 0;
        }
    }
    int ne;
    const int lo = block_exscan<EMIT_BLOCK>(m, s_wsum, ne);
    const bool staged = ne <= EMIT_ECAP;   // uniform
    if (bad) {
        if (tid == 0) atomicOr(status, ST_INTERNAL);
        return;
    }
    if (!staged) {
        if (tid < nc &&
            !emit_cell<VERT>(sets[s], sides, k, p, olines, pool, total, pos, of, m, dn, base,
                             dbase, sid, sxy, nbr, vtx, del))
            atomicOr(status, ST_INTERNAL);
        return;
    }
    if (tid < nc) {
        clo[tid] = lo;
        cbase[tid] = base;
        cdel[tid] = dbase;
        ck[tid] = k;
        cof[tid] = of;
        cset[tid] = s;
        pc[tid] = p;
        for (int t = 0; t < m; ++t) own[lo + t] = (unsigned char)tid;
    }
    if (tid == 0) clo[nc] = ne;
    __syncthreads();
    // per entry: the line's site id and coordinates
    for (int e = tid; e < ne; e += EMIT_BLOCK) {
        const int o = own[e];
        const int q = cell_line(olines, pool, total, pos0 + o, cof[o], e - clo[o]);
        lin[e] = q >= 0 ? sid[q] : q;
        if (VERT) {
            const float2 a = q >= 0 ? sxy[q] : make_float2(0.0f, 0.0f);
            qc[e] = make_int2((int)a.x, (int)a.y);
        }
    }
    __syncthreads();
    // per cell: rotation, and the count of neighbours > k against the cell pass's count
    if (tid < nc) {
        int r = 0, up = 0;
        for (int t = 0; t < m; ++t) {
            const int a = lin[lo + t];
            r = (uint32_t)a < (uint32_t)lin[lo + r] ? t : r;
            up += a > k;
        }
        crot[tid] = r;
        if (up != dn) bad = 1;
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) atomicOr(status, ST_INTERNAL);
        return;
    }
    // per entry (found order u): CSR slot (u - r) mod m, the vertex with the next line, and the
    // Delaunay pair at the rank of j among the cell's neighbours > k
    uint2 *__restrict__ del2 = reinterpret_cast<uint2 *>(del);
    for (int e = tid; e < ne; e += EMIT_BLOCK) {
        const int o = own[e];
        const int lo2 = clo[o], mo = clo[o + 1] - lo2, u = e - lo2;
        int t = u - crot[o];
        t += t < 0 ? mo : 0;
        const int j = lin[e];
        const long long b0 = cbase[o];
        nbr[b0 + t] = j;
        if (VERT) {
            const int e2 = u + 1 == mo ? lo2 : e + 1;
            vtx[b0 + t] = pair_vertex(sets[cset[o]], sides, pc[o], j, qc[e], lin[e2], qc[e2]);
        }
        const int ko = ck[o];
        if (j > ko) {
            int rank = 0;
            for (int v = lo2; v < lo2 + mo; ++v) rank += lin[v] > ko && lin[v] < j;
            del2[cdel[o] + rank] = make_uint2((unsigned)ko, (unsigned)j);
        }
    }
}

__global__ void k_symmetry(const SetDesc *__restrict__ sets, int nsets,
                           const int *__restrict__ set_off, int total,
                           const int *__restrict__ cell_off, const int *__restrict__ nbr,
                           unsigned long long *__restrict__ stats, const int *__restrict__ status) {
    if (*status) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int so = set_off[find_set(set_off, nsets, g)];
    const int k = g - so;
    unsigned long long bad = 0;
    for (int t = cell_off[g]; t < cell_off[g + 1]; ++t) {
        const int j = nbr[t];
        if (j < 0) continue;
        bool found = false;
        for (int u = cell_off[so + j]; u < cell_off[so + j + 1]; ++u) found |= (nbr[u] == k);
        bad += !found;
    }
    if (bad) atomicAdd(&stats[SL_ASYM], bad);
}

// ------------------------------------------------------------------------------ launchers
static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Exclusive prefix sums of in[0..n) into out[0..n], the total also into *tot when given.
void launch_scan(const int *in, long long n, int *out, int *tmp, const int *status, int gate,
                 hipStream_t st, int *tot = nullptr) {
    const unsigned nb = nblk(n, SCAN_TILE);
    k_scan_reduce<<<nb, SCAN_BLOCK, 0, st>>>(in, n, tmp, status, gate);
    k_scan_top<<<1, SCAN_BLOCK, 0, st>>>(tmp, (int)nb, status, gate);
    k_scan_apply<<<nb, SCAN_BLOCK, 0, st>>>(in, n, tmp, out, status, gate, tot);
}


template <int BLOCK>
static void launch_fast(const PipeArgs &a, hipStream_t st) {
    const unsigned nb = (nblk(a.total, BLOCK) + 7) & ~7u;
    if (a.any_poly)
        k_cells_fast<BLOCK, true><<<nb, BLOCK, 0, st>>>(
            a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.total, a.ocnt,
            a.olines, a.ovf, a.dcnt, a.queue, a.qcount(), a.queue3, a.qcount3(), a.stats,
            a.bflag, a.hand, a.status());
    else
        k_cells_fast<BLOCK, false><<<nb, BLOCK, 0, st>>>(
            a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.total, a.ocnt,
            a.olines, a.ovf, a.dcnt, a.queue, a.qcount(), a.queue3, a.qcount3(), a.stats,
            a.bflag, a.hand, a.status());
}

template <int MODE>
static void launch_exact(const PipeArgs &a, hipStream_t st) {
    // cells of sites on the boundary of X
    k_cells_bnd<MODE><<<BND_BLOCKS, 64, 0, st>>>(
        a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.total, a.ocnt, a.olines,
        a.dcnt, a.ovf, a.pool, a.poolcnt(), a.poolcap, a.queue5, a.qcount5(), a.stats, a.status_rw());
    // the deferred cells: few of them (the usual case after the filtered passes) a workgroup
    // each, the subwedges of a cell spread over its waves; else one wave each
    if (!(a.exact_only || a.coop_all))
        k_cells_wide<MODE, WIDE_LCAP, WIDE_LWAVES><<<WIDE_LBLOCKS, 64 * WIDE_LWAVES, 0, st>>>(
            a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.total, a.ocnt,
            a.olines, a.dcnt, a.ovf, a.pool, a.poolcnt(), a.poolcap, a.queue, a.qcount(), nullptr,
            a.queue2, a.qcount2(), a.bflag, a.stats, a.status_rw());
    k_cells_exact<MODE, DCAP1><<<a.exact_blocks, 64, 0, st>>>(
        a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.total, a.ocnt, a.olines,
        a.dcnt, a.ovf, a.pool, a.poolcnt(), a.poolcap, a.queue, a.qcount(), a.queue2,
        a.qcount2(), a.wbuf, DCAP1, a.stats, a.bflag, a.status_rw(),
        a.exact_only || a.coop_all ? 0 : WIDE_QMAX);
    // deep cells: few workgroups, the subwedges of each cell spread over their waves
    k_cells_wide<MODE, 0, WIDE_WAVES><<<DEEP_BLOCKS, 64 * WIDE_WAVES, 0, st>>>(
        a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.total, a.ocnt, a.olines,
        a.dcnt, a.ovf, a.pool, a.poolcnt(), a.poolcap, a.queue2, a.qcount2(), a.wbuf2, nullptr,
        nullptr, nullptr, a.stats, a.status_rw());
}

void launch_stage(const PipeArgs &a, hipStream_t st, int stage) {
    const int T = a.total;
    if (stage == 0) {
        // clear counters (no memset nodes: the sequence is captured as a graph)
        const long long n = a.gtot;
        const long long nf = ((long long)a.total + 3) / 4;   // boundary flags as 32-bit words
        const long long big = std::max(std::max(n, nf), 64LL);
        k_clear<<<nblk(big, 256), 256, 0, st>>>(a.bcnt, n, a.small, SMALL_INTS, a.stats,
                                                (unsigned *)a.bflag, nf);
        // grid build (Method 11.5), then adaptive refinement of crowded buckets
        // the slots of the counting sort are kept by input index in the per-cell line counts,
        // which the cell passes write later
        k_prep<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, a.sides, a.in_x,
                                              a.in_y, T, a.xyid, a.key, a.bcnt, a.ocnt,
                                              a.status());
        launch_scan(a.bcnt, a.gtot, a.bstart, a.scan_tmp, a.status(), 0, st);
        k_scatter<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.xyid, a.key,
                                                 a.bstart, a.ocnt, a.sxy, a.sid, a.bflag,
                                                 a.queue5, a.qcount5());
        k_tree_mark0<<<nblk(a.gtot + 1, 256), 256, 0, st>>>(a.sets, a.nsets, a.gtot, a.bstart,
                                                            a.tchild, a.bcnt, a.nodes, a.ncap,
                                                            a.rootcnt(), a.status());
        launch_scan(a.bcnt, a.gtot, a.tref, a.scan_tmp, a.status(), 1, st);
        const unsigned rb = (unsigned)std::max(1, std::min(2048, a.ncap));
        for (int lv = 1; lv <= TREE_LEVELS; ++lv)
            k_tree_refine<<<rb, REFINE_BLOCK, 0, st>>>(
                a.nodes, lv, a.rootcnt(), a.nodecnt(), a.small + LVCNT0, a.nlist, a.ncap, a.ncap,
                a.bstart, a.tchild, a.tabcnt(), a.gtot + 1, a.tabcap, a.sxy, a.sid, a.txy, a.tid,
                a.status_rw());
        k_dups<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.sxy, a.bstart,
                                              a.tchild, a.nodes, a.status_rw());
    } else if (stage == 1) {
        // filtered cell pass
        if (a.exact_only || a.coop_all)
            k_queue_all<<<nblk(T, 256), 256, 0, st>>>(T, a.queue, a.qcount(), a.status());
        else if (a.tree_all)
            k_queue_all<<<nblk(T, 256), 256, 0, st>>>(T, a.queue3, a.qcount3(), a.status());
        else if (a.block == 64)
            launch_fast<64>(a, st);
        else if (a.block == 128)
            launch_fast<128>(a, st);
        else
            launch_fast<256>(a, st);
    } else if (stage == 2) {
        // adaptive pass over the cells that met crowded buckets
        if (!(a.exact_only || a.coop_all)) {
            // local grids over chunks of consecutive cells (every cell with tree_all, else the
            // handed-over ones), then the tree scans for what they hand on
            const long long nch = ((long long)T + LOC_BLOCK - 1) / LOC_BLOCK;
            const unsigned lb = (unsigned)std::max(1LL, std::min(nch, (long long)LOC_GRID_MAX));
            k_cells_local<<<lb, LOC_BLOCK, 0, st>>>(
                a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.tchild, a.nodes,
                a.tref, T, a.hand, a.tree_all ? 1 : 0, a.qcount3(), a.ocnt, a.olines, a.ovf,
                a.dcnt, a.queue, a.qcount(), a.queue4, a.qcount4(), a.stats, a.bflag, a.status());
            // the list buffer holds TREE_LIST entries for each thread of this grid
            const unsigned nb = (unsigned)tree_pass_blocks(T);
            k_cells_tree<TREE_PASS_BLOCK><<<nb, TREE_PASS_BLOCK, 0, st>>>(
                a.sets, a.nsets, a.set_off, a.sides, a.sxy, a.sid, a.bstart, a.tchild, a.nodes, a.tref,
                T, a.ocnt, a.olines, a.ovf, a.dcnt, a.queue, a.qcount(), a.queue4, a.qcount4(),
                a.tlist, a.stats, a.bflag, a.tree_done(), a.status());
        }
    } else if (stage == 3) {
        if (a.exact_only) launch_exact<2>(a, st);
        else launch_exact<1>(a, st);
    } else {
        // CSR offsets and Delaunay offsets, then neighbours, vertices and Delaunay pairs
        launch_scan(a.ocnt, T, a.cell_off, a.scan_tmp, a.status(), 1, st, a.tot_entries());
        launch_scan(a.dcnt, T, a.del_off, a.scan_tmp, a.status(), 1, st, a.tot_dels());
        if (a.with_vertices)
            k_emit<true><<<nblk(T, EMIT_BLOCK), EMIT_BLOCK, 0, st>>>(
                a.sets, a.nsets, a.set_off, a.sides, T, a.sid, a.sxy, a.olines, a.ovf, a.pool,
                a.cell_off, a.nbr_cap, a.del_off, a.del_cap, a.nbr, (Rat *)a.vtx, a.del,
                a.status_rw());
        else
            k_emit<false><<<nblk(T, EMIT_BLOCK), EMIT_BLOCK, 0, st>>>(
                a.sets, a.nsets, a.set_off, a.sides, T, a.sid, a.sxy, a.olines, a.ovf, a.pool,
                a.cell_off, a.nbr_cap, a.del_off, a.del_cap, a.nbr, nullptr, a.del, a.status_rw());
        if (a.check_symmetry)
            k_symmetry<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.cell_off,
                                                      a.nbr, a.stats, a.status());
    }
}

void launch_pipeline(const PipeArgs &a, hipStream_t st) {
    for (int s = 0; s < NSTAGES; ++s) launch_stage(a, st, s);
}

}  // namespace vor
