// vor_internal.h -- interface between the host runtime (vor_api.cpp) and the device pipeline.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vor {

struct SetDesc;
struct SideRel;
struct TNode;
constexpr int SMALL_INTS = 20;   // status, queue counters, pool / tree counters, totals, spare
constexpr int DEEP_BLOCKS = 4;   // workgroups of the deep-cell pass (one cell each at a time)
constexpr int WIDE_WAVES = 8;    // waves of such a workgroup (subwedges resolved in parallel)
constexpr int WIDE_CAP = 65536 + 64;   // corners of one deep cell (a cell has at most 65536
                                       // lines; rays <= lines + 1, Lemma on shot rays)
constexpr int LVCNT0 = 8;        // small[LVCNT0 + l]: nodes listed for refinement level l (2..6)
constexpr int TREE_PASS_BLOCK = 128;       // threads per block of the adaptive pass
constexpr int TREE_PASS_MAXBLOCKS = 2048;  // its persistent grid at most
// Blocks of the adaptive pass for `total` sites: one thread per cell up to the persistent size.
inline long long tree_pass_blocks(long long total) {
    const long long b = (total + TREE_PASS_BLOCK - 1) / TREE_PASS_BLOCK;
    return b < 1 ? 1 : (b > TREE_PASS_MAXBLOCKS ? TREE_PASS_MAXBLOCKS : b);
}

// Device pointers and sizes of one pipeline launch.
struct PipeArgs {
    const SetDesc *sets;
    int nsets;
    const SideRel *sides;   // sides of the polygon regions (at least one entry)
    bool any_poly;          // some set of the launch has a polygon X
    const int *set_off;     // [nsets + 1] first global site of each set
    int total;              // sites in all sets
    long long gtot;         // buckets in all sets
    const int *in_x, *in_y; // absolute input coordinates [total]
    int2 *xyid;             // relative coordinates by site [total]
    int *key;               // bucket of each site [total]
    int *bcnt;              // [gtot]
    int *bstart;            // [gtot + 1 + tabcap]: bucket starts, then sub-bucket starts
    int *tchild;            // [gtot + 1 + tabcap]: refining node of each slot, or -1
    TNode *nodes;           // [ncap] refinement nodes
    int ncap;
    long long tabcap;       // sub-bucket table entries after the grid's
    float2 *txy;            // [total] refinement scratch
    int *tid;               // [total]
    int *queue3;            // cells handed to the adaptive pass [total]
    int *queue4;            // cells of the adaptive pass that need the full scanner [total]
    int *tref;              // [gtot + 1] refined grid buckets before each bucket
    float2 *sxy;            // sorted coordinates [total]
    int *sid;               // local id of each sorted site [total]
    int *ocnt;              // [total] lines of each cell, by site id (-1: not done); before the
                            // cell passes, the counting sort's slot of each site
    int *olines;            // [KOUT * total] line t of the cell at sorted position pos at
                            // t * total + pos: the neighbour's sorted position or a side code
    int *ovf;               // [total] by sorted position: pool offset of a cell with more than
                            // KOUT lines, else -1
    int *pool;
    long long poolcap;
    int *queue, *queue2;
    int *wbuf, *wbuf2;
    int exact_blocks;
    int *cell_off;          // [total + 1]
    int *nbr;
    long long nbr_cap;
    void *vtx;              // vor_rat [nbr_cap]
    int *dcnt, *del_off;    // [total], [total + 1]
    int *tlist;             // adaptive pass candidate lists: TREE_LIST entries per thread of the
                            // pass, entry i of thread t at i * threads + t
    unsigned *del;          // [2 * del_cap]
    long long del_cap;
    int *scan_tmp;
    int *small;             // SMALL_INTS
    unsigned long long *stats;
    int block;
    bool exact_only, with_vertices, check_symmetry;
    bool coop_all;              // every cell through the one-wave-per-cell pass (small sets)
    bool tree_all;              // every cell through the coordinate-rectangle pass
    bool time_stages;           // HIP events between the stages (one graph per stage)

    int *status() const { return small; }
    int *status_rw() const { return small; }
    int *qcount() const { return small + 1; }
    int *qcount2() const { return small + 2; }
    int *poolcnt() const { return small + 3; }
    int *nodecnt() const { return small + 4; }   // nodes below the roots
    int *tabcnt() const { return small + 5; }
    int *rootcnt() const { return small + 6; }   // refined grid buckets (tree roots)
    int *qcount4() const { return small + 7; }   // cells the local grids hand to the tree scans
    int *qcount3() const { return small + 8; }
    int *tree_done() const { return small + 9; }   // workgroups of the tree scans done
    int *nlist;             // [TREE_LEVELS - 1][ncap] node ids of refinement levels 2..
    unsigned char *bflag;   // [total] by sorted position: the site lies on the boundary of X
    unsigned char *hand;    // [total] by sorted position: the filtered pass handed the cell on
    int *queue5;            // sorted positions of such sites (the boundary pass) [total]
    int *qcount5() const { return small + 15; }
    // the run's totals (entries, Delaunay pairs) beside the counters, so that one copy brings
    // back status, counters and totals; the device counters follow the SMALL_INTS words
    int *tot_entries() const { return small + 16; }
    int *tot_dels() const { return small + 17; }
};

// stages: 0 grid build and refinement, 1 filtered cell pass, 2 adaptive pass, 3 exact / deep
// passes, 4 CSR, vertices and Delaunay edges
constexpr int NSTAGES = 5;
void launch_stage(const PipeArgs &a, hipStream_t st, int stage);
void launch_pipeline(const PipeArgs &a, hipStream_t st);
// Lloyd steps (vor_lloyd.hip): proposals from the cells of the last pipeline run, one
// collision round (flag set when a site went back), the count of sites that moved.
void lloyd_propose(const PipeArgs &a, const int *cx, const int *cy, int *qx, int *qy,
                   hipStream_t st);
void lloyd_round(int n, int *qx, int *qy, const int *cx, const int *cy,
                 unsigned long long *keys, int *cnt, unsigned cap, int *flag, hipStream_t st);
void lloyd_moved(int n, const int *qx, const int *qy, const int *cx, const int *cy, int *moved,
                 hipStream_t st);
// Prefix sums: SCAN_ITEMS values per thread of a SCAN_BLOCK-thread block; the per-tile partial
// sums (one int per tile, plus one) live in scan_tmp.
constexpr int SCAN_BLOCK = 256, SCAN_ITEMS = 4, SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;
inline long long scan_tmp_ints(long long n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

}  // namespace vor
