// vor_kernels.hip -- the device pipeline of one call (one point set or a batch of sets):
//
//   prep      validate, relative coordinates, bucket of every site (Method 11.5)
//   scan      bucket counts -> bucket starts (counting sort)
//   scatter   sites into bucket order (structure of arrays, FP32 coordinates)
//   dups      equal sites share a bucket: compare inside buckets (lexicographic check of the
//             distinctness remark in Appendix 2, done per bucket)
//   cells     the projector algorithm per cell, FP32 filtered; undecided cells are queued
//   exact     queued cells again with exact fallback (or every cell, exact-only precision)
//   deep      cells deeper than the exact pass's per-worker capacity
//   scan      line counts -> CSR offsets
//   fill      canonical rotation, neighbour ids, pair-form vertices (Section 6)
//   scan/del  Delaunay edges (i, j), i < j, sorted (Section 7)
//
// Every kernel reads the device status word first and returns when an input error is set, so
// the whole sequence can be launched (or replayed as a HIP graph) without host round trips.
#include <algorithm>

#include "vor_cell.hpp"
#include "vor_internal.h"

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

__global__ void k_clear(int *__restrict__ p, long long n, int *__restrict__ small, int nsmall,
                        unsigned long long *__restrict__ stats) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
    if (i < nsmall) small[i] = 0;
    if (i < SL_COUNT) stats[i] = 0;
}

__global__ void k_prep(const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
                       const int *__restrict__ in_x, const int *__restrict__ in_y, int total,
                       int2 *__restrict__ xyid, int *__restrict__ key, int *__restrict__ bcnt,
                       int *__restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const SetDesc S = sets[find_set(set_off, nsets, i)];
    long long rx = (long long)in_x[i] - S.x0, ry = (long long)in_y[i] - S.y0;
    if (!(rx > 0 && rx < S.W && ry > 0 && ry < S.H)) {
        atomicOr(status, ST_DOMAIN);
        rx = rx < 1 ? 1 : (rx > S.W - 1 ? S.W - 1 : rx);
        ry = ry < 1 ? 1 : (ry > S.H - 1 ? S.H - 1 : ry);
    }
    xyid[i] = make_int2((int)rx, (int)ry);
    const int bx = min((int)rx / S.s, S.gx - 1), by = min((int)ry / S.s, S.gy - 1);
    const int b = S.bucket_off + by * S.gx + bx;
    key[i] = b;
    atomicAdd(&bcnt[b], 1);
}

// Counting-sort scatter.  bcnt counts down to zero again, ready for the next call.
__global__ void k_scatter(const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
                          int total, const int2 *__restrict__ xyid, const int *__restrict__ key,
                          const int *__restrict__ bstart, int *__restrict__ bcnt,
                          float2 *__restrict__ sxy, int *__restrict__ sid) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = key[i];
    const int pos = bstart[b] + atomicSub(&bcnt[b], 1) - 1;
    const int2 r = xyid[i];
    sxy[pos] = make_float2((float)r.x, (float)r.y);
    sid[pos] = i - set_off[find_set(set_off, nsets, i)];
}

__global__ void k_dups(const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
                       int total, const float2 *__restrict__ sxy, const int *__restrict__ bstart,
                       int *__restrict__ status) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= total) return;
    const SetDesc S = sets[find_set(set_off, nsets, pos)];
    const float2 a = sxy[pos];
    const int bx = min((int)a.x / S.s, S.gx - 1), by = min((int)a.y / S.s, S.gy - 1);
    const int lo = bstart[S.bucket_off + by * S.gx + bx];
    for (int j = lo; j < pos; ++j) {
        const float2 b = sxy[j];
        if (b.x == a.x && b.y == a.y) {
            atomicOr(status, ST_DUP);
            break;
        }
    }
}

__device__ __forceinline__ Cell make_cell(const SetDesc &S, float2 p) {
    Cell C;
    C.gx = S.gx;
    C.gy = S.gy;
    C.s = S.s;
    C.boff = S.bucket_off;
    C.h = S.h;
    C.pxf = p.x;
    C.pyf = p.y;
    C.px = (int)p.x;
    C.py = (int)p.y;
    C.bx = min(C.px / S.s, S.gx - 1);
    C.by = min(C.py / S.s, S.gy - 1);
    C.W = S.W;
    C.H = S.H;
    return C;
}

__device__ __forceinline__ void reduce_stats(const Counters &K, uint32_t edges, uint32_t deferred,
                                             unsigned long long *sh, unsigned long long *stats) {
    atomicAdd(&sh[SL_RAYS], (unsigned long long)K.rays);
    atomicAdd(&sh[SL_NODES], (unsigned long long)K.nodes);
    atomicAdd(&sh[SL_EVALS], (unsigned long long)K.evals);
    atomicAdd(&sh[SL_EXACT], (unsigned long long)K.exact);
    atomicAdd(&sh[SL_SHELLS], (unsigned long long)K.shells);
    atomicAdd(&sh[SL_EDGES], (unsigned long long)edges);
    atomicAdd(&sh[SL_DEFERRED], (unsigned long long)deferred);
    atomicAdd(&sh[SL_VTESTS], (unsigned long long)K.vtests);
    __syncthreads();
    if (threadIdx.x < SL_COUNT && sh[threadIdx.x]) atomicAdd(&stats[threadIdx.x], sh[threadIdx.x]);
}

// Filtered pass: one thread per cell, cells in bucket order, stack in LDS.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_cells_fast(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const float2 *__restrict__ sxy, const int *__restrict__ sid, const int *__restrict__ bstart,
    int total, int *__restrict__ ocnt, int *__restrict__ olines, int *__restrict__ ovf,
    int *__restrict__ queue, int *__restrict__ qcount, unsigned long long *__restrict__ stats,
    const int *__restrict__ status) {
    __shared__ int stk[SCAP][BLOCK];
    __shared__ int rlo[MAXROWS][BLOCK], rhi[MAXROWS][BLOCK];
    __shared__ unsigned long long sh[SL_COUNT];
    if (*status) return;
    if (threadIdx.x < SL_COUNT) sh[threadIdx.x] = 0;
    __syncthreads();
    const int pos = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    Counters K{0, 0, 0, 0, 0, 0};
    uint32_t edges = 0, deferred = 0;
    if (pos < total) {
        const SetDesc S = sets[find_set(set_off, nsets, pos)];
        const Cell C = make_cell(S, sxy[pos]);
        const int g = S.site_off + sid[pos];
        LdsStack<BLOCK> st{stk, 0};
        LdsRows<BLOCK> rows{rlo, rhi, 0};
        Sink sink{olines + (size_t)g * KOUT, sid};
        const int r = run_cell<0, Solo>(C, sxy, bstart, st, SCAP, rows, sink, KOUT, K);
        ovf[g] = -1;
        if (r >= 0) {
            ocnt[g] = r;
            edges = (uint32_t)r;
        } else {
            ocnt[g] = -1;
            queue[atomicAdd(qcount, 1)] = pos;
            deferred = 1;
        }
    }
    reduce_stats(K, edges, deferred, sh, stats);
}

__global__ void k_queue_all(int total, int *__restrict__ queue, int *__restrict__ qcount,
                            const int *__restrict__ status) {
    if (*status) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) queue[i] = i;
    if (i == 0) *qcount = total;
}

// Exact pass over a queue of cells: one wave per cell (the Coop policy), a persistent grid of
// one-wave blocks; the cell's stack and output live in the block's area of dcap entries each.
template <int MODE>
__global__ __launch_bounds__(64) void k_cells_exact(
    const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
    const float2 *__restrict__ sxy, const int *__restrict__ sid, const int *__restrict__ bstart,
    int *__restrict__ ocnt, int *__restrict__ olines, int *__restrict__ ovf,
    int *__restrict__ pool, int *__restrict__ poolcnt, long long poolcap,
    const int *__restrict__ queue, const int *__restrict__ qcount, int *__restrict__ queue2,
    int *__restrict__ qcount2, int *__restrict__ wbuf, int dcap,
    unsigned long long *__restrict__ stats, int *__restrict__ status) {
    __shared__ unsigned long long sh[SL_COUNT];
    if (*status & (ST_DOMAIN | ST_DUP)) return;
    if (threadIdx.x < SL_COUNT) sh[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x;
    const int nq = *qcount;
    int *area = wbuf + (size_t)blockIdx.x * 2 * dcap;
    Counters K{0, 0, 0, 0, 0, 0};
    uint32_t edges = 0;
    for (int qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const int pos = queue[qi];
        const SetDesc S = sets[find_set(set_off, nsets, pos)];
        const Cell C = make_cell(S, sxy[pos]);
        const int g = S.site_off + sid[pos];
        GStack st{area, 0};
        GlobalRows rows{0};
        Sink sink{area + dcap, sid};
        const int r = run_cell<MODE, Coop>(C, sxy, bstart, st, dcap, rows, sink, dcap, K);
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
        int *dst = off >= 0 ? pool + off : olines + (size_t)g * KOUT;
        for (int t = lane; t < r; t += 64) dst[t] = src[t];
        if (lane == 0) {
            ovf[g] = off;
            ocnt[g] = r;
        }
    }
    // every lane ran the same control flow: count it once; evaluations are split across lanes
    if (lane != 0) {
        K.rays = K.nodes = K.exact = K.shells = K.vtests = 0;
        edges = 0;
    }
    reduce_stats(K, edges, 0, sh, stats);
}

// ------------------------------------------------------------------------------ scan
// Exclusive scan of n int32 values (>= 0) into out[0..n], out[n] = total.  Three launches:
// block sums, a single-block scan of the sums, per-block scan plus offset.
constexpr int SCAN_BLOCK = 256, SCAN_ITEMS = 4, SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int block_excl_scan(int v, int *sh, int &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < SCAN_BLOCK / 64; ++i) {
            const int t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[SCAN_BLOCK / 64] = acc;
    }
    __syncthreads();
    total = sh[SCAN_BLOCK / 64];
    const int r = x - v + sh[wid];
    __syncthreads();
    return r;
}

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
    (void)block_excl_scan(v, sh, total);
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
        const int e = block_excl_scan(v, sh, total);
        if (i < nb) bsum[i] = e + carry;
        carry += total;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const int *__restrict__ in, long long n,
                                                           const int *__restrict__ bsum,
                                                           int *__restrict__ out,
                                                           const int *__restrict__ status,
                                                           int gate) {
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
    int e = block_excl_scan(s, sh, total) + bsum[blockIdx.x];
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        if (base + t < n) out[base + t] = e;
        e += v[t];
        if (base + t == n - 1) out[n] = e;
    }
}

// ------------------------------------------------------------------------------ CSR fill
__device__ __forceinline__ void abs_line(const SetDesc &S, const int2 *__restrict__ xyid, int k,
                                         int j, long long &nx, long long &ny, long long &c) {
    // absolute coordinates: x = rel + x0
    const long long px = (long long)xyid[S.site_off + k].x + S.x0;
    const long long py = (long long)xyid[S.site_off + k].y + S.y0;
    if (j >= 0) {
        const long long qx = (long long)xyid[S.site_off + j].x + S.x0;
        const long long qy = (long long)xyid[S.site_off + j].y + S.y0;
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

// Per cell: canonical rotation, neighbour ids, the owner of every CSR entry, Delaunay count.
__global__ void k_fill(const SetDesc *__restrict__ sets, int nsets, const int *__restrict__ set_off,
                       int total, const int *__restrict__ ocnt, const int *__restrict__ olines,
                       const int *__restrict__ ovf, const int *__restrict__ pool,
                       const int *__restrict__ cell_off, long long cap, int *__restrict__ nbr,
                       int *__restrict__ ecell, int *__restrict__ dcnt, int *__restrict__ status) {
    if (*status) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int k = g - set_off[find_set(set_off, nsets, g)];
    const int m = ocnt[g];
    const long long base = cell_off[g];
    if (m < 3 || base + m > cap) {
        atomicOr(status, ST_INTERNAL);
        return;
    }
    const int *src = ovf[g] >= 0 ? pool + ovf[g] : olines + (size_t)g * KOUT;
    int r = 0;
    for (int t = 1; t < m; ++t)
        if ((uint32_t)src[t] < (uint32_t)src[r]) r = t;
    int up = 0;
    for (int t = 0; t < m; ++t) {
        const int a = src[(r + t) % m];
        nbr[base + t] = a;
        ecell[base + t] = g;
        up += a > k;
    }
    dcnt[g] = up;
}

// Per CSR entry (consecutive threads write consecutive 40-byte vertices): vertex i of cell k is
// line(nbr[i]) ∩ line(nbr[i+1 cyclic]) in pair form, Cramer's rule on the absolute lines.
__global__ void k_vertices(const SetDesc *__restrict__ sets, int nsets,
                           const int *__restrict__ set_off, int total,
                           const int *__restrict__ cell_off, const int *__restrict__ nbr,
                           const int *__restrict__ ecell, const int2 *__restrict__ xyid,
                           Rat *__restrict__ vtx, const int *__restrict__ status) {
    if (*status) return;
    const long long E = cell_off[total];
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += stride) {
        const int g = ecell[e];
        const SetDesc S = sets[find_set(set_off, nsets, g)];
        const int k = g - S.site_off;
        const int lo = cell_off[g], hi = cell_off[g + 1];
        const int a = nbr[e];
        const int b = nbr[e + 1 == hi ? lo : e + 1];
        long long n1x, n1y, c1, n2x, n2y, c2;
        abs_line(S, xyid, k, a, n1x, n1y, c1);
        abs_line(S, xyid, k, b, n2x, n2y, c2);
        const long long D = n1x * n2y - n1y * n2x;
        const i128 X = (i128)c1 * n2y - (i128)c2 * n1y;
        const i128 Y = (i128)n1x * c2 - (i128)n2x * c1;
        Rat v;
        v.x_lo = (uint64_t)X;
        v.x_hi = (int64_t)(X >> 64);
        v.y_lo = (uint64_t)Y;
        v.y_hi = (int64_t)(Y >> 64);
        v.d = D;
        vtx[e] = v;
    }
}

__global__ void k_delaunay(const SetDesc *__restrict__ sets, int nsets,
                           const int *__restrict__ set_off, int total,
                           const int *__restrict__ cell_off, const int *__restrict__ nbr,
                           const int *__restrict__ del_off, unsigned *__restrict__ del,
                           long long del_cap, int *__restrict__ status) {
    if (*status) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    if ((long long)del_off[g + 1] > del_cap) {
        atomicOr(status, ST_INTERNAL);
        return;
    }
    const int k = g - set_off[find_set(set_off, nsets, g)];
    const int lo = cell_off[g], hi = cell_off[g + 1];
    long long o = del_off[g];
    int prev = k;
    for (;;) {   // ascending neighbours > k (selection; cells are small)
        int nxt = INT32_MAX;
        for (int t = lo; t < hi; ++t) {
            const int a = nbr[t];
            if (a > prev && a < nxt) nxt = a;
        }
        if (nxt == INT32_MAX) break;
        del[2 * o] = (unsigned)k;
        del[2 * o + 1] = (unsigned)nxt;
        ++o;
        prev = nxt;
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

void launch_scan(const int *in, long long n, int *out, int *tmp, const int *status, int gate,
                 hipStream_t st) {
    const unsigned nb = nblk(n, SCAN_TILE);
    k_scan_reduce<<<nb, SCAN_BLOCK, 0, st>>>(in, n, tmp, status, gate);
    k_scan_top<<<1, SCAN_BLOCK, 0, st>>>(tmp, (int)nb, status, gate);
    k_scan_apply<<<nb, SCAN_BLOCK, 0, st>>>(in, n, tmp, out, status, gate);
}

long long scan_tmp_ints(long long n) { return (long long)nblk(n, SCAN_TILE) + 1; }

void launch_stage(const PipeArgs &a, hipStream_t st, int stage) {
    const int T = a.total;
    if (stage == 0) {
    // 1. clear counters (no memset nodes: the sequence is captured as a graph)
    {
        const long long n = a.gtot;
        const long long big = n > 64 ? n : 64;
        k_clear<<<nblk(big, 256), 256, 0, st>>>(a.bcnt, n, a.small, SMALL_INTS, a.stats);
    }
    // 2. grid build
    k_prep<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, a.in_x, a.in_y, T, a.xyid,
                                          a.key, a.bcnt, a.status());
    launch_scan(a.bcnt, a.gtot, a.bstart, a.scan_tmp, a.status(), 0, st);
    k_scatter<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.xyid, a.key, a.bstart,
                                             a.bcnt, a.sxy, a.sid);
    k_dups<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.sxy, a.bstart,
                                          a.status());
    } else if (stage == 1) {
    // 3. cells
    if (a.exact_only || a.coop_all) {
        k_queue_all<<<nblk(T, 256), 256, 0, st>>>(T, a.queue, a.qcount(), a.status());
    } else {
        const int B = a.block;
        const unsigned nb = (nblk(T, B) + 7) & ~7u;
        if (B == 64)
            k_cells_fast<64><<<nb, 64, 0, st>>>(a.sets, a.nsets, a.set_off, a.sxy, a.sid, a.bstart,
                                               T, a.ocnt, a.olines, a.ovf, a.queue, a.qcount(),
                                               a.stats, a.status());
        else if (B == 128)
            k_cells_fast<128><<<nb, 128, 0, st>>>(a.sets, a.nsets, a.set_off, a.sxy, a.sid,
                                                 a.bstart, T, a.ocnt, a.olines, a.ovf, a.queue,
                                                 a.qcount(), a.stats, a.status());
        else
            k_cells_fast<256><<<nb, 256, 0, st>>>(a.sets, a.nsets, a.set_off, a.sxy, a.sid,
                                                 a.bstart, T, a.ocnt, a.olines, a.ovf, a.queue,
                                                 a.qcount(), a.stats, a.status());
    }
    } else if (stage == 2) {
    if (a.exact_only)
        k_cells_exact<2><<<a.exact_blocks, 64, 0, st>>>(
            a.sets, a.nsets, a.set_off, a.sxy, a.sid, a.bstart, a.ocnt, a.olines, a.ovf, a.pool,
            a.poolcnt(), a.poolcap, a.queue, a.qcount(), a.queue2, a.qcount2(), a.wbuf, DCAP1,
            a.stats, a.status_rw());
    else
        k_cells_exact<1><<<a.exact_blocks, 64, 0, st>>>(
            a.sets, a.nsets, a.set_off, a.sxy, a.sid, a.bstart, a.ocnt, a.olines, a.ovf, a.pool,
            a.poolcnt(), a.poolcap, a.queue, a.qcount(), a.queue2, a.qcount2(), a.wbuf, DCAP1,
            a.stats, a.status_rw());
    // deep cells: few workers with a large area each
    if (a.exact_only)
        k_cells_exact<2><<<DEEP_BLOCKS, 64, 0, st>>>(
            a.sets, a.nsets, a.set_off, a.sxy, a.sid, a.bstart, a.ocnt, a.olines, a.ovf, a.pool,
            a.poolcnt(), a.poolcap, a.queue2, a.qcount2(), nullptr, nullptr, a.wbuf2, DCAP2,
            a.stats, a.status_rw());
    else
        k_cells_exact<1><<<DEEP_BLOCKS, 64, 0, st>>>(
            a.sets, a.nsets, a.set_off, a.sxy, a.sid, a.bstart, a.ocnt, a.olines, a.ovf, a.pool,
            a.poolcnt(), a.poolcap, a.queue2, a.qcount2(), nullptr, nullptr, a.wbuf2, DCAP2,
            a.stats, a.status_rw());
    } else {
    // 4. CSR
    launch_scan(a.ocnt, T, a.cell_off, a.scan_tmp, a.status(), 1, st);
    k_fill<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.ocnt, a.olines, a.ovf,
                                          a.pool, a.cell_off, a.nbr_cap, a.nbr, a.ecell, a.dcnt,
                                          a.status_rw());
    if (a.with_vertices) {
        const long long cap = a.nbr_cap;
        const unsigned nb = (unsigned)std::min<long long>(nblk(cap, 256), 8192);
        k_vertices<<<nb, 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.cell_off, a.nbr, a.ecell,
                                       a.xyid, (Rat *)a.vtx, a.status());
    }
    launch_scan(a.dcnt, T, a.del_off, a.scan_tmp, a.status(), 1, st);
    k_delaunay<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.cell_off, a.nbr,
                                              a.del_off, a.del, a.del_cap, a.status_rw());
    if (a.check_symmetry)
        k_symmetry<<<nblk(T, 256), 256, 0, st>>>(a.sets, a.nsets, a.set_off, T, a.cell_off, a.nbr,
                                                  a.stats, a.status());
    }
}

void launch_pipeline(const PipeArgs &a, hipStream_t st) {
    for (int s = 0; s < NSTAGES; ++s) launch_stage(a, st, s);
}

}  // namespace vor
