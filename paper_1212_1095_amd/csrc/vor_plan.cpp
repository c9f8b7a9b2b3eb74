// vor_plan.cpp -- host-side planning of a pipeline run: validation of sets and polygon regions,
// the bucket grid of Method 11.5, buffer sizes and launch arguments.
#include "vor_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "vor_tree.hpp"

namespace vor {

double region_area(uint32_t K, const int32_t *vx, const int32_t *vy) {
    __int128 s = 0;
    for (uint32_t e = 0; e < K; ++e) {
        const uint32_t f = (e + 1) % K;
        s += (__int128)vx[e] * vy[f] - (__int128)vy[e] * vx[f];
    }
    return (double)s / 2.0;
}

// Convex polygon X (Remark 11.1): 3..VOR_MAX_SIDES vertices, counter-clockwise, every turn
// strictly left and the edge directions going round once (they switch between the upper and
// the lower half-plane exactly twice).  Writes its bounding box.
int check_region(uint32_t K, const int32_t *vx, const int32_t *vy, vor_box &bb) {
    if (K < 3 || K > VOR_MAX_SIDES || !vx || !vy) return VOR_E_INVAL;
    const long long lim = 1LL << 30;
    long long mnx = vx[0], mxx = vx[0], mny = vy[0], mxy = vy[0];
    for (uint32_t e = 0; e < K; ++e) {
        if (vx[e] < -lim || vx[e] > lim || vy[e] < -lim || vy[e] > lim) return VOR_E_DOMAIN;
        mnx = std::min<long long>(mnx, vx[e]);
        mxx = std::max<long long>(mxx, vx[e]);
        mny = std::min<long long>(mny, vy[e]);
        mxy = std::max<long long>(mxy, vy[e]);
    }
    if (mxx - mnx > (1LL << 24) || mxy - mny > (1LL << 24)) return VOR_E_DOMAIN;
    int changes = 0;
    for (uint32_t e = 0; e < K; ++e) {
        const uint32_t f = (e + 1) % K, g = (e + 2) % K;
        const long long ax = (long long)vx[f] - vx[e], ay = (long long)vy[f] - vy[e];
        const long long bx = (long long)vx[g] - vx[f], by = (long long)vy[g] - vy[f];
        if (ax * by - ay * bx <= 0) return VOR_E_INVAL;
        const bool ua = ay > 0 || (ay == 0 && ax > 0), ub = by > 0 || (by == 0 && bx > 0);
        changes += ua != ub;
    }
    if (changes != 2) return VOR_E_INVAL;
    bb = vor_box{(int32_t)mnx, (int32_t)mny, (int32_t)mxx, (int32_t)mxy};
    return VOR_OK;
}

// Side lines of a checked polygon, relative to its bounding-box origin (x0, y0): side e is
// N.x <= c with the primitive outward normal N = (dy, -dx) / gcd.
void region_sides(uint32_t K, const int32_t *vx, const int32_t *vy, int32_t x0, int32_t y0,
                  SideRel *out) {
    for (uint32_t e = 0; e < K; ++e) {
        const long long ax = (long long)vx[e] - x0, ay = (long long)vy[e] - y0;
        const long long bx = (long long)vx[(e + 1) % K] - x0, by = (long long)vy[(e + 1) % K] - y0;
        long long dx = bx - ax, dy = by - ay, g = std::gcd(dx < 0 ? -dx : dx, dy < 0 ? -dy : dy);
        SideRel s;
        s.nx = (int32_t)(dy / g);
        s.ny = (int32_t)(-dx / g);
        s.c = (int64_t)s.nx * ax + (int64_t)s.ny * ay;
        s.vx = (int32_t)ax;
        s.vy = (int32_t)ay;
        out[e] = s;
    }
}



// Validates a set and returns the HostSet the pipeline runs (device: inputs in HBM).
int check_set(const vor_set *s, HostSet &h) {
    if (!s || s->n == 0 || !s->x || !s->y) return VOR_E_INVAL;
    h = HostSet{s->n, s->x, s->y, s->box, (s->flags & VOR_SET_DEVICE) != 0};
    if (s->nregion) {
        const int rc = check_region(s->nregion, s->region_x, s->region_y, h.box);
        if (rc != VOR_OK) return rc;
        h.nreg = s->nregion;
        h.rx = s->region_x;
        h.ry = s->region_y;
        h.area = region_area(h.nreg, h.rx, h.ry);
    }
    const vor_box &b = h.box;
    if (!(b.x0 < b.x1 && b.y0 < b.y1)) return VOR_E_INVAL;
    const long long lim = 1LL << 30;
    if (b.x0 < -lim || b.y0 < -lim || b.x1 > lim || b.y1 > lim) return VOR_E_DOMAIN;
    if ((long long)b.x1 - b.x0 > (1LL << 24) || (long long)b.y1 - b.y0 > (1LL << 24))
        return VOR_E_DOMAIN;
    if ((long long)s->n > MAX_RUN_SITES) return VOR_E_INVAL;
    return VOR_OK;
}

// Uniform grid of Method 11.5 with about `rho` sites per square bucket.
// `area`: the area of X (W H for the box; less for a polygon X, whose sites crowd a part of
// the bounding box: the buckets are sized for the sites' density in X).
void choose_grid(const vor_box &b, uint32_t n, float rho, int hw, SetDesc &d, double area) {
    const double W = (double)b.x1 - b.x0, H = (double)b.y1 - b.y0;
    if (!(area > 0) || area > W * H) area = W * H;
    double s = std::sqrt(area * (double)rho / (double)n);
    long long si = (long long)std::ceil(s);
    if (si < 1) si = 1;
    long long gx = (long long)std::ceil(W / (double)si), gy = (long long)std::ceil(H / (double)si);
    // keep the grid at most ~4 buckets per site of X's area (16 at most in all)
    const long long per = (long long)std::min(16.0, std::ceil(4.0 * W * H / area));
    while (gx * gy > per * (long long)n + 16) {
        si *= 2;
        gx = (long long)std::ceil(W / (double)si);
        gy = (long long)std::ceil(H / (double)si);
    }
    d.s = (int32_t)si;
    d.gx = (int32_t)std::max(1LL, gx);
    d.gy = (int32_t)std::max(1LL, gy);
    // block of shells 0..h scanned first: about two site spacings in each direction
    const double h = hw > 0 ? (double)hw : std::round(2.0 / std::sqrt((double)rho));
    d.h = (int32_t)std::max(1.0, std::min(h, 16.0));
}

int map_status(int st) {
    if (st & ST_DUP) return VOR_E_DUPLICATE;
    if (st & ST_DOMAIN) return VOR_E_DOMAIN;
    if (st & ST_CAPACITY) return VOR_E_CAPACITY;
    if (st & ST_INTERNAL) return VOR_E_DEVICE;
    return VOR_OK;
}

size_t footprint_bytes(uint64_t total, uint64_t gtot, bool vertices, uint64_t sides) {
    const uint64_t E = (uint64_t)entry_cap((long long)total, (long long)sides);
    size_t b = 0;
    b += total * (4 + 4 + 8 + 4 + 8 + 4 + 4 + 4 + 4 + 4 + 4 + 4);   // inputs, grid, queues, counts
    b += total * 4ull * KOUT;                                       // filtered-pass lines
    b += E * 4 * 2;                                                 // pool, nbr
    if (vertices) b += E * sizeof(vor_rat);
    b += (3 * total + 8) * 8;                                       // delaunay
    b += gtot * 16;                                                 // counts, starts, tree slots
    b += total * (8 + 4 + 4 + 4);                                   // refinement scratch, queues
    b += (3 * total + 1024) * 8;                                    // sub-bucket tables
    b += 4ull * TREE_LIST * TREE_PASS_BLOCK * tree_pass_blocks((long long)total);   // lists
    b += (TREE_LEVELS * (total / (TREE_C1 + 1)) + 64) * (sizeof(TNode) + 4 * (TREE_LEVELS - 1));
    b += 2 * (total + 4);                                           // boundary, hand-over flags
    return b;
}

// Descriptor of one set placed at global site `site_off`, bucket `bucket_off` and side-table
// entry `side_off` of a run; its polygon sides (if any) go to side_tab[side_off..].
void plan_set(const vor_tuning &tune, const HostSet &s, long long site_off, long long bucket_off,
              int side_off, SetDesc &d, SideRel *side_tab) {
    d.W = s.box.x1 - s.box.x0;
    d.H = s.box.y1 - s.box.y0;
    d.x0 = s.box.x0;
    d.y0 = s.box.y0;
    d.n = (int32_t)s.n;
    d.site_off = (int32_t)site_off;
    choose_grid(s.box, s.n, tune.sites_per_bucket, tune.block_halfwidth, d, s.area);
    d.ht = tune.leaf_halfwidth;
    d.bucket_off = (int32_t)bucket_off;
    d.ns = (int32_t)s.nreg;
    d.side_off = side_off;
    if (s.nreg) region_sides(s.nreg, s.rx, s.ry, s.box.x0, s.box.y0, side_tab + side_off);
}


int run_sizes(long long T, long long gtot, long long sides, int K, size_t nsides, bool vertices,
              bool exact_only, long long coop_below, RunSizes &z, int max_exact_blocks) {
    if (T >= (1LL << 30) || gtot >= (1LL << 30)) return VOR_E_NOMEM;
    for (size_t &x : z.b) x = 0;
    z.T = T;
    z.gtot = gtot;
    z.K = K;
    z.E = entry_cap(T, sides);
    if (z.E >= (1LL << 31)) return VOR_E_NOMEM;   // 32-bit entry offsets
    z.D = 3 * T + 8;
    z.coop_all = !exact_only && T <= coop_below;
    // one-wave workers of the exact pass: enough to fill the GPU when every cell goes through
    // it, fewer when it only takes the cells the filtered pass deferred
    z.exact_blocks = (int)std::max<long long>(
        1, std::min<long long>(std::min(exact_only || z.coop_all ? 8192 : 2048, max_exact_blocks), T));
    const long long stmp = scan_tmp_ints(std::max(T, gtot)) + 8;
    // refinement: every node holds > TREE_C1 sites and the nodes of one level are disjoint;
    // a node's table has m*m + 1 <= 2 cnt + 1 entries; a table or node overflow leaves the
    // bucket unrefined (slower, still exact)
    z.ncap = std::max<long long>(64, TREE_LEVELS * (T / (TREE_C1 + 1)) + 64);
    z.tabcap = 3 * T + 1024;
    const long long E = z.E, D = z.D, ncap = z.ncap, tabcap = z.tabcap;
    size_t *b = z.b;
    b[B_SETS] = sizeof(SetDesc) * K;
    b[B_SETOFF] = 4ull * (K + 1);
    b[B_INX] = b[B_INY] = 4ull * T;
    b[B_XYID] = 8ull * T;
    b[B_KEY] = 4ull * T;
    b[B_BCNT] = 4ull * gtot;
    b[B_BSTART] = b[B_TCHILD] = 4ull * (gtot + 1 + tabcap);
    b[B_NODES] = sizeof(TNode) * ncap;
    b[B_TXY] = 8ull * T;
    b[B_TID] = b[B_QUEUE3] = b[B_QUEUE4] = b[B_QUEUE5] = 4ull * T;
    b[B_BFLAG] = 4ull * ((T + 3) / 4);   // cleared as 32-bit words
    b[B_HAND] = 4ull * ((T + 3) / 4);
    b[B_TREF] = 4ull * (gtot + 1);
    b[B_NLIST] = 4ull * (TREE_LEVELS - 1) * ncap;
    b[B_SXY] = 8ull * T;
    b[B_SID] = b[B_OCNT] = b[B_OVF] = b[B_QUEUE] = b[B_QUEUE2] = b[B_DCNT] = 4ull * T;
    b[B_OLINES] = 4ull * KOUT * T;
    b[B_POOL] = b[B_NBR] = 4ull * E;
    b[B_WBUF] = 4ull * 2 * DCAP1 * z.exact_blocks;
    b[B_WBUF2] = 4ull * 4 * WIDE_CAP * DEEP_BLOCKS;
    b[B_CELLOFF] = b[B_DELOFF] = 4ull * (T + 1);
    b[B_VTX] = vertices ? sizeof(vor_rat) * E : 16;
    b[B_DEL] = 8ull * D;
    b[B_SCANTMP] = 4ull * stmp;
    b[B_SMALL] = SUMMARY_BYTES;   // the small words and the counters together
    b[B_STATS] = 8;
    b[B_SIDES] = sizeof(SideRel) * std::max<size_t>(1, nsides);
    b[B_TLIST] = 4ull * TREE_LIST * TREE_PASS_BLOCK * tree_pass_blocks(T);
    return VOR_OK;
}

// Launch arguments of a run whose buffers are at p[B_*] (device memory laid out as run_sizes).
void fill_args(PipeArgs &a, void *const p[B_COUNT], const RunSizes &z, bool any_poly,
               const int *in_x, const int *in_y, const vor_tuning &tune, bool exact_only,
               bool vertices, bool symmetry, bool time_stages) {
    std::memset(&a, 0, sizeof(a));
    a.sets = (const SetDesc *)p[B_SETS];
    a.nsets = z.K;
    a.sides = (const SideRel *)p[B_SIDES];
    a.any_poly = any_poly;
    a.set_off = (const int *)p[B_SETOFF];
    a.total = (int)z.T;
    a.gtot = z.gtot;
    a.in_x = in_x;
    a.in_y = in_y;
    a.xyid = (int2 *)p[B_XYID];
    a.key = (int *)p[B_KEY];
    a.bcnt = (int *)p[B_BCNT];
    a.bstart = (int *)p[B_BSTART];
    a.tchild = (int *)p[B_TCHILD];
    a.nodes = (TNode *)p[B_NODES];
    a.ncap = (int)z.ncap;
    a.tabcap = z.tabcap;
    a.txy = (float2 *)p[B_TXY];
    a.tid = (int *)p[B_TID];
    a.queue3 = (int *)p[B_QUEUE3];
    a.queue4 = (int *)p[B_QUEUE4];
    a.tref = (int *)p[B_TREF];
    a.nlist = (int *)p[B_NLIST];
    a.bflag = (unsigned char *)p[B_BFLAG];
    a.queue5 = (int *)p[B_QUEUE5];
    a.hand = (unsigned char *)p[B_HAND];
    a.sxy = (float2 *)p[B_SXY];
    a.sid = (int *)p[B_SID];
    a.ocnt = (int *)p[B_OCNT];
    a.olines = (int *)p[B_OLINES];
    a.ovf = (int *)p[B_OVF];
    a.pool = (int *)p[B_POOL];
    a.poolcap = z.E;
    a.queue = (int *)p[B_QUEUE];
    a.queue2 = (int *)p[B_QUEUE2];
    a.wbuf = (int *)p[B_WBUF];
    a.wbuf2 = (int *)p[B_WBUF2];
    a.exact_blocks = z.exact_blocks;
    a.cell_off = (int *)p[B_CELLOFF];
    a.nbr = (int *)p[B_NBR];
    a.nbr_cap = z.E;
    a.vtx = p[B_VTX];
    a.dcnt = (int *)p[B_DCNT];
    a.tlist = (int *)p[B_TLIST];
    a.del_off = (int *)p[B_DELOFF];
    a.del = (unsigned *)p[B_DEL];
    a.del_cap = z.D;
    a.scan_tmp = (int *)p[B_SCANTMP];
    a.small = (int *)p[B_SMALL];
    a.stats = (unsigned long long *)((char *)p[B_SMALL] + 4 * SMALL_INTS);
    a.block = tune.block;
    a.tree_all = tune.scan_path == VOR_PATH_TREE;
    a.exact_only = exact_only;
    a.with_vertices = vertices;
    a.check_symmetry = symmetry;
    a.coop_all = z.coop_all;
    a.time_stages = time_stages;
}

void fill_stats(vor_stats &st, const unsigned long long *sl) {
    st.rays = sl[SL_RAYS];
    st.nodes = sl[SL_NODES];
    st.evals = sl[SL_EVALS];
    st.exact_decisions = sl[SL_EXACT];
    st.deferred_cells = sl[SL_DEFERRED];
    st.asym_pairs = sl[SL_ASYM];
    st.shells = sl[SL_SHELLS];
    st.edges = sl[SL_EDGES];
    st.vertex_tests = sl[SL_VTESTS];
    st.adaptive_cells = sl[SL_TREE];
    st.adaptive_evals = sl[SL_TEVALS];
    st.fallback_incircle = sl[SL_XINC];
    st.fallback_cmp = sl[SL_EXACT] - sl[SL_XINC];
    st.vertex_rays = sl[SL_VRAYS];
}

}  // namespace vor
