// vor_plan.h -- host-side planning of a pipeline run (validation, bucket grid, buffer sizes,
// launch arguments), shared by the context-based entry points and the no-allocation one.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "vor.h"
#include "vor_device.hpp"
#include "vor_internal.h"

namespace vor {

enum BufId {
    B_SETS, B_SETOFF, B_INX, B_INY, B_XYID, B_KEY, B_BCNT, B_BSTART, B_SXY, B_SID, B_OCNT,
    B_OLINES, B_OVF, B_POOL, B_QUEUE, B_QUEUE2, B_WBUF, B_WBUF2, B_CELLOFF, B_NBR, B_VTX,
    B_DCNT, B_DELOFF, B_DEL, B_SCANTMP, B_SMALL, B_STATS, B_TCHILD, B_NODES, B_TXY,
    B_TID, B_QUEUE3, B_TREF, B_NLIST, B_SIDES, B_TLIST, B_QUEUE4, B_BFLAG, B_QUEUE5, B_HAND, B_COUNT
};

struct HostSet {   // validated description of one input set
    uint32_t n;
    const int32_t *x, *y;
    vor_box box;           // X, or the bounding box of a polygon X
    bool device;
    uint32_t nreg = 0;     // vertices of a convex polygon X (0: X is the box)
    const int32_t *rx = nullptr, *ry = nullptr;
    double area = 0;       // area of X
};

// Convex polygon X (Remark 11.1): checks and bounding box; side lines; area.
double region_area(uint32_t K, const int32_t *vx, const int32_t *vy);
int check_region(uint32_t K, const int32_t *vx, const int32_t *vy, vor_box &bb);
void region_sides(uint32_t K, const int32_t *vx, const int32_t *vy, int32_t x0, int32_t y0,
                  SideRel *out);

// Sites in one pipeline run (a set, a batch, or the requests admitted together).  Entry
// offsets and the overflow pool are 32-bit; with the entry bound below, 2^27 sites keep every
// offset below 2^31 unless the sets bring very many polygon sides (run_sizes checks the sum).
constexpr long long MAX_RUN_SITES = 1LL << 27;

// Entries (neighbour-list lines) of a run: a set of n sites in a convex X with K sides has
// sum e_k <= 6n + K - 6.  Euler's formula for the subdivision of X by the restricted diagram
// (n cells and the outer face) gives E = V + n - 1 edges; every vertex has degree >= 3 except
// corners of X without a Voronoi edge (degree 2), so 2E >= 3V - K and E <= 3n - 3 + K; each
// interior edge borders two cells and each of the >= K boundary edges one, so
// sum e_k = 2E - E_boundary <= 6n + K - 6 (the box: 6n - 2, inside the paper's 10n for a
// rectangle).  The Delaunay pairs are the interior edges, E - E_boundary <= 3n - 3.
inline long long entry_cap(long long sites, long long sides) { return 6 * sites + sides + 16; }

// Validates a set and returns the HostSet the pipeline runs (device: inputs in HBM).
int check_set(const vor_set *s, HostSet &h);

// Uniform grid of Method 11.5 with about `rho` sites per square bucket (area: of X).
void choose_grid(const vor_box &b, uint32_t n, float rho, int hw, SetDesc &d, double area = 0);

// The words read back after a run, one copy: SMALL_INTS status / counter / total words, then
// the device counters (stats) right after them in the same buffer.
constexpr size_t SUMMARY_BYTES = 4 * SMALL_INTS + 8 * SL_COUNT;
static_assert((4 * SMALL_INTS) % 8 == 0, "the counters follow the small words 8-byte aligned");

// Device status word -> VOR status.
int map_status(int st);

// HBM footprint of one run (admission of the request loop).
size_t footprint_bytes(uint64_t total, uint64_t gtot, bool vertices, uint64_t sides);

// Descriptor of one set placed at global site `site_off`, bucket `bucket_off` and side-table
// entry `side_off` of a run; its polygon sides (if any) go to side_tab[side_off..].
void plan_set(const vor_tuning &tune, const HostSet &s, long long site_off, long long bucket_off,
              int side_off, SetDesc &d, SideRel *side_tab);

// Buffer sizes of one run.
struct RunSizes {
    size_t b[B_COUNT];
    long long T, gtot, E, D, ncap, tabcap;
    int K, exact_blocks;
    bool coop_all;
};
// Sizes for T sites in K sets with gtot buckets, `sides` sides in all (4 per box) of which
// `nsides` polygon sides in the side table; at most max_exact_blocks one-wave exact workers.
int run_sizes(long long T, long long gtot, long long sides, int K, size_t nsides, bool vertices,
              bool exact_only, long long coop_below, RunSizes &z, int max_exact_blocks = 8192);

// Launch arguments of a run whose buffers are at p[B_*] (device memory laid out as run_sizes).
void fill_args(PipeArgs &a, void *const p[B_COUNT], const RunSizes &z, bool any_poly,
               const int *in_x, const int *in_y, const vor_tuning &tune, bool exact_only,
               bool vertices, bool symmetry, bool time_stages);

// Device counters (SL_* slots) -> vor_stats.
void fill_stats(vor_stats &st, const unsigned long long *sl);

}  // namespace vor
