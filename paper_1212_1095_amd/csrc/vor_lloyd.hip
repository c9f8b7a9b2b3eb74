// vor_lloyd.hip -- Lloyd iterations on the integer grid: each step computes the diagram with the
// pipeline, then moves every site to the rounded centroid of its cell.  The paper motivates a
// fast diagram by algorithms that recompute it many times (centroidal Voronoi relaxation among
// them); the rounding and the collision rule below are this library's definition of a step.
//
//   propose   per cell: vertices relative to the site in IEEE double (the exact integer
//             X - p D converted once, correctly rounded, then divided by D), the shoelace sums
//             in the stored vertex order (contraction off: every product and sum rounds once),
//             offset = S / (3 A2), proposal = p + rint(offset); a proposal not strictly inside X
//             keeps p.
//   resolve   while a position is proposed by more than one site, every such site whose
//             proposal is not its current position keeps its current position (sites at their
//             current positions never collide, so the rounds end); a hash table of proposals
//             with per-slot counts, one round per launch pair.
#include "vor.h"
#include "vor_device.hpp"
#include "vor_internal.h"

namespace vor {

#pragma clang fp contract(off)
__device__ __forceinline__ void rel_vertex(const vor_rat &v, long long px, long long py,
                                           double &ux, double &uy) {
    const i128 X = ((i128)v.x_hi << 64) | (i128)v.x_lo;
    const i128 Y = ((i128)v.y_hi << 64) | (i128)v.y_lo;
    const double d = (double)v.d;
    ux = (double)(X - (i128)px * v.d) / d;
    uy = (double)(Y - (i128)py * v.d) / d;
}

__global__ void k_lloyd_propose(const SetDesc *__restrict__ sets,
                                const SideRel *__restrict__ sides, int n,
                                const int *__restrict__ cell_off, const vor_rat *__restrict__ vtx,
                                const int *__restrict__ cx, const int *__restrict__ cy,
                                int *__restrict__ qx, int *__restrict__ qy,
                                const int *__restrict__ status) {
    if (*status) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const SetDesc S = sets[0];
    const long long px = cx[g], py = cy[g];
    const int lo = cell_off[g], m = cell_off[g + 1] - lo;
    double ux0, uy0;
    rel_vertex(vtx[lo], px, py, ux0, uy0);
    double ux = ux0, uy = uy0, a2 = 0.0, sx = 0.0, sy = 0.0;
    for (int t = 0; t < m; ++t) {
        double vx, vy;
        if (t + 1 < m) {
            rel_vertex(vtx[lo + t + 1], px, py, vx, vy);
        } else {
            vx = ux0;
            vy = uy0;
        }
        const double c = ux * vy - vx * uy;
        a2 += c;
        sx += (ux + vx) * c;
        sy += (uy + vy) * c;
        ux = vx;
        uy = vy;
    }
    const double ox = sx / (3.0 * a2), oy = sy / (3.0 * a2);
    const long long nx = px + (long long)rint(ox), ny = py + (long long)rint(oy);
    // strictly inside X (relative to the box origin)
    const long long rx = nx - S.x0, ry = ny - S.y0;
    bool inside = rx > 0 && rx < S.W && ry > 0 && ry < S.H;
    for (int e = 0; e < S.ns && inside; ++e) {
        const SideRel s = sides[S.side_off + e];
        inside = (long long)s.nx * rx + (long long)s.ny * ry < s.c;
    }
    qx[g] = inside ? (int)nx : (int)px;
    qy[g] = inside ? (int)ny : (int)py;
}
#pragma clang fp contract(fast)

// |coordinate| <= 2^30, so the offset halves lie in [2^30, 3 2^30]: never the empty key.
constexpr unsigned long long HASH_EMPTY = ~0ull;
__device__ __forceinline__ unsigned long long pos_key(int x, int y) {
    return ((unsigned long long)((long long)x + (1LL << 31)) << 32) |
           (unsigned long long)((long long)y + (1LL << 31));
}
__device__ __forceinline__ unsigned hash_slot(unsigned long long k, unsigned mask) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    return (unsigned)k & mask;
}

__global__ void k_hash_clear(unsigned long long *__restrict__ keys, int *__restrict__ cnt,
                             unsigned cap, int *__restrict__ flag) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cap) {
        keys[i] = HASH_EMPTY;
        cnt[i] = 0;
    }
    if (i == 0) *flag = 0;
}

__global__ void k_hash_count(const int *__restrict__ qx, const int *__restrict__ qy, int n,
                             unsigned long long *__restrict__ keys, int *__restrict__ cnt,
                             unsigned mask) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const unsigned long long k = pos_key(qx[g], qy[g]);
    unsigned h = hash_slot(k, mask);
    for (unsigned probe = 0; probe <= mask; ++probe) {   // the table has 2n slots or more
        const unsigned long long prev = atomicCAS(&keys[h], HASH_EMPTY, k);
        if (prev == HASH_EMPTY || prev == k) {
            atomicAdd(&cnt[h], 1);
            return;
        }
        h = (h + 1) & mask;
    }
}

__global__ void k_hash_revert(int *__restrict__ qx, int *__restrict__ qy,
                              const int *__restrict__ cx, const int *__restrict__ cy, int n,
                              const unsigned long long *__restrict__ keys,
                              const int *__restrict__ cnt, unsigned mask, int *__restrict__ flag) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int x = qx[g], y = qy[g];
    const unsigned long long k = pos_key(x, y);
    unsigned h = hash_slot(k, mask);
    for (unsigned probe = 0; probe <= mask; ++probe) {
        if (keys[h] == k) break;
        h = (h + 1) & mask;
    }
    if (cnt[h] > 1 && (x != cx[g] || y != cy[g])) {
        qx[g] = cx[g];
        qy[g] = cy[g];
        atomicOr(flag, 1);
    }
}

__global__ void k_count_moved(const int *__restrict__ qx, const int *__restrict__ qy,
                              const int *__restrict__ cx, const int *__restrict__ cy, int n,
                              int *__restrict__ moved) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int mv = g < n && (qx[g] != cx[g] || qy[g] != cy[g]);
    const unsigned long long bal = __ballot(mv);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(moved, __popcll(bal));
}

static unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }

void lloyd_propose(const PipeArgs &a, const int *cx, const int *cy, int *qx, int *qy,
                   hipStream_t st) {
    k_lloyd_propose<<<blocks(a.total), 256, 0, st>>>(a.sets, a.sides, a.total, a.cell_off,
                                                     (const vor_rat *)a.vtx, cx, cy, qx, qy,
                                                     a.status());
}

void lloyd_round(int n, int *qx, int *qy, const int *cx, const int *cy,
                 unsigned long long *keys, int *cnt, unsigned cap, int *flag, hipStream_t st) {
    k_hash_clear<<<blocks(cap), 256, 0, st>>>(keys, cnt, cap, flag);
    k_hash_count<<<blocks(n), 256, 0, st>>>(qx, qy, n, keys, cnt, cap - 1);
    k_hash_revert<<<blocks(n), 256, 0, st>>>(qx, qy, cx, cy, n, keys, cnt, cap - 1, flag);
}

__global__ void k_zero(int *__restrict__ p) { *p = 0; }

void lloyd_moved(int n, const int *qx, const int *qy, const int *cx, const int *cy, int *moved,
                 hipStream_t st) {
    k_zero<<<1, 1, 0, st>>>(moved);
    k_count_moved<<<blocks(n), 256, 0, st>>>(qx, qy, cx, cy, n, moved);
}

}  // namespace vor
