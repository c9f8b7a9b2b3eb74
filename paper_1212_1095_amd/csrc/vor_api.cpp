// vor_api.cpp -- host runtime behind include/vor.h: contexts, device workspaces, the
// graph-captured pipeline, batched sets and the continuous-batching request loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "vor.h"
#include "vor_device.hpp"
#include "vor_internal.h"
#include "vor_plan.h"
#include "vor_tree.hpp"

using namespace vor;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = bytes < 256 ? 256 : bytes;
        want += want / 8;   // headroom so slightly larger calls reuse the buffer
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <class T> T *as() const { return (T *)p; }
};

struct HostBuf {   // pinned staging
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap && p) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = bytes < 256 ? 256 : bytes + bytes / 8;
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};


// Pinned host memory for results, kept for reuse: a block that its results no longer need goes
// back to the free list (up to PINNED_CACHE bytes, or twice the largest block asked for, stay
// cached: a caller that holds one run's results while the next runs needs two such blocks), so
// that once the pool has grown to what the caller holds at a time, runs neither pin new memory
// nor wait on its release.
constexpr size_t PINNED_CACHE = 8ull << 30;
constexpr size_t PINNED_GRAIN = 2ull << 20;
struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, void *> free;   // size -> block
    size_t cached = 0;
    size_t biggest = 0;
    ~PinnedPool() {
        for (auto &kv : free) (void)hipHostFree(kv.second);
    }
    // A block of at least `bytes` (its size in `got`): a cached one at most half as large again,
    // else a new one; nullptr when pinned memory runs short.
    void *get(size_t bytes, size_t &got) {
        const size_t want = (std::max<size_t>(bytes, 1) + PINNED_GRAIN - 1) / PINNED_GRAIN * PINNED_GRAIN;
        {
            std::lock_guard<std::mutex> lk(mu);
            biggest = std::max(biggest, want);
            auto it = free.lower_bound(want);
            if (it != free.end() && it->first <= want + want / 2) {
                void *p = it->second;
                got = it->first;
                cached -= got;
                free.erase(it);
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        got = want;
        return p;
    }
    void put(void *p, size_t size) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (cached + size <= std::max(PINNED_CACHE, 2 * biggest)) {
                free.emplace(size, p);
                cached += size;
                return;
            }
        }
        (void)hipHostFree(p);
    }
};

// Host memory that results point into: a pool block (pinned) or, when pinned memory runs
// short, a pageable one.  Every result of the block holds a reference.
struct OutBlock {
    void *p = nullptr;
    size_t cap = 0;
    std::shared_ptr<PinnedPool> pool;   // null: malloc'd
    ~OutBlock() {
        if (!p) return;
        if (pool)
            pool->put(p, cap);
        else
            std::free(p);
    }
};

struct Workspace {
    DevBuf b[B_COUNT];
    HostBuf h_in, h_small;          // pinned staging: inputs, summary
    std::vector<SideRel> sides_h;   // side table of the sets being launched
    std::vector<char> up_cache;     // set descriptors, side table, set offsets last uploaded
    DevBuf lcx, lcy, lqx, lqy, lkeys, lcnt, lflag;   // Lloyd iterations
    HostBuf h_lloyd;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ek[NSTAGES + 1] = {};
    hipGraphExec_t gexec[NSTAGES] = {};
    hipGraph_t graph[NSTAGES] = {};
    PipeArgs gkey{};
    PipeArgs last{};          // the arguments of the last run launched kernel by kernel
    bool have_last = false;
    bool have_graph = false;
    bool graph_broken = false;
    bool last_timed = false;
    bool used_graph = false;

    hipError_t init() {
        hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        if ((e = hipEventCreate(&ev0)) != hipSuccess) return e;
        for (auto &x : ek)
            if ((e = hipEventCreate(&x)) != hipSuccess) return e;
        return hipEventCreate(&ev1);
    }
    void drop_graph() {
        for (int s = 0; s < NSTAGES; ++s) {
            if (gexec[s]) (void)hipGraphExecDestroy(gexec[s]);
            if (graph[s]) (void)hipGraphDestroy(graph[s]);
            gexec[s] = nullptr;
            graph[s] = nullptr;
        }
        have_graph = false;
    }
    // device and pinned buffers back to the runtime (the stream must be idle); the next launch
    // allocates what it needs again
    void release_buffers() {
        drop_graph();
        for (auto &x : b) x.release();
        h_in.release();
        up_cache.clear();
    }
    void destroy() {
        if (stream) (void)hipStreamSynchronize(stream);
        drop_graph();
        for (auto &x : b) x.release();
        for (DevBuf *x : {&lcx, &lcy, &lqx, &lqy, &lkeys, &lcnt, &lflag}) x->release();
        h_in.release();
        h_small.release();
        h_lloyd.release();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        for (auto &x : ek)
            if (x) (void)hipEventDestroy(x);
        if (stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
};




struct ResultBox {   // vor_result plus the storage it points to
    vor_result r;
    std::vector<uint32_t> off;
    std::vector<int32_t> nbr;
    std::vector<vor_rat> vtx;
    std::vector<uint32_t> del;
    std::shared_ptr<OutBlock> block;   // a run's host block (instead of the vectors)
};

vor_result *new_result(ResultBox *&box) {
    box = new (std::nothrow) ResultBox();
    if (!box) return nullptr;
    std::memset(&box->r, 0, sizeof(box->r));
    return &box->r;
}

// vor_result is the first member of ResultBox: vor_result_free converts the pointer back.

}  // namespace

struct Request {
    uint64_t ticket;
    std::vector<int32_t> x, y;
    vor_box box;
    std::vector<int32_t> rx, ry;   // polygon X (empty: the box)
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = VOR_PENDING;
    vor_result *result = nullptr;
    size_t footprint = 0;
    bool alone = false;   // re-run by itself (an input error in its batch)
    // the request is finished: its copied inputs are no longer needed
    void release_inputs() {
        std::vector<int32_t>().swap(x);
        std::vector<int32_t>().swap(y);
        std::vector<int32_t>().swap(rx);
        std::vector<int32_t>().swap(ry);
    }
};

// Batches of the request loop on the GPU at once (one workspace and stream each); three or four
// gave no better latency on the mixed request stream.
constexpr int REQ_WORKSPACES = 4;
struct vor_ctx {
    int device = 0;
    vor_opts opts{};
    // the autotuned setting for uniform 2^20 sites, also the fastest measured for batches of
    // 32..65536-site sets and of 1000-site sets
    vor_tuning tune{1.5f, 256, 2, 0, VOR_PATH_GRID_FIRST};
    // per-set grid parameters by size class (vor_set_size_tuning); empty: `tune` for every set
    std::vector<vor_size_tuning> size_tune;
    Workspace ws;            // vor_compute / vor_compute_batch
    std::shared_ptr<PinnedPool> pool = std::make_shared<PinnedPool>();   // host result memory
    std::mutex mu;           // serialises vor_compute*
    bool use_graph = true;
    long long coop_below = 4096;   // sets up to this size: one wave per cell
    // sites per admitted batch of the request loop (a request larger than this runs alone):
    // bounds how long a request that arrives just after an admission waits for the batch ahead
    long long serve_batch_sites = 1 << 18;
    // request loop
    Workspace rws[REQ_WORKSPACES];
    std::mutex qmu;
    std::condition_variable qcv;
    std::deque<std::shared_ptr<Request>> pending;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool loop_started = false;
    std::thread loop;
    uint64_t budget = 0;
};

namespace {


// The tuning a set of n sites runs with: the context's, with the grid parameters of the size
// class nearest to log2 n when a size table is set.
vor_tuning set_tuning(const vor_ctx *ctx, uint32_t n) {
    vor_tuning t = ctx->tune;
    if (ctx->size_tune.empty()) return t;
    const double l = std::log2((double)std::max<uint32_t>(n, 1));
    const vor_size_tuning *best = &ctx->size_tune[0];
    for (const vor_size_tuning &e : ctx->size_tune)
        if (std::fabs(e.log2n - l) < std::fabs(best->log2n - l)) best = &e;
    t.sites_per_bucket = best->sites_per_bucket;
    t.block_halfwidth = best->block_halfwidth;
    t.leaf_halfwidth = best->leaf_halfwidth;
    return t;
}

// Prepare descriptors, size the workspace and launch the pipeline on ws.stream.  Inputs are
// either device pointers (single set, VOR_SET_DEVICE) or gathered into pinned staging and
// copied.  Returns a VOR status; on success the launch is in flight.
int launch(vor_ctx *ctx, Workspace &ws, const std::vector<HostSet> &sets, bool vertices,
           bool exact_only, bool symmetry, bool use_graph, PipeArgs &a,
           std::vector<SetDesc> &descs, std::vector<int> &set_off) {
    const int K = (int)sets.size();
    descs.resize(K);
    set_off.assign(K + 1, 0);
    size_t nsides = 0;
    for (const HostSet &s : sets) nsides += s.nreg;
    ws.sides_h.resize(nsides);
    long long total = 0, gtot = 0, sides = 0;
    int side_off = 0;
    for (int i = 0; i < K; ++i) {
        const HostSet &s = sets[i];
        sides += s.nreg ? s.nreg : 4;
        plan_set(set_tuning(ctx, s.n), s, total, gtot, side_off, descs[i], ws.sides_h.data());
        side_off += (int)s.nreg;
        set_off[i] = (int)total;
        total += s.n;
        gtot += (long long)descs[i].gx * descs[i].gy;
    }
    set_off[K] = (int)total;
    RunSizes z;
    int rc = run_sizes(total, gtot, sides, K, nsides, vertices, exact_only, ctx->coop_below, z);
    if (rc != VOR_OK) return rc;
    const long long T = total;
    bool grew = false;
    for (int id = 0; id < B_COUNT; ++id) {
        const size_t before = ws.b[id].cap;
        const void *pb = ws.b[id].p;
        if (ws.b[id].ensure(z.b[id]) != hipSuccess) {
            (void)hipGetLastError();
            return VOR_E_NOMEM;
        }
        grew |= (ws.b[id].cap != before) || (ws.b[id].p != pb);
    }
    if (grew) ws.drop_graph();
    // inputs
    const bool dev_in = (K == 1 && sets[0].device);
    const int *in_x, *in_y;
    hipError_t e;
    if (dev_in) {
        in_x = sets[0].x;
        in_y = sets[0].y;
    } else {
        if (ws.h_in.ensure(8ull * T) != hipSuccess) return VOR_E_NOMEM;
        int32_t *hx = (int32_t *)ws.h_in.p, *hy = hx + T;
        for (int i = 0; i < K; ++i) {
            std::memcpy(hx + set_off[i], sets[i].x, 4ull * sets[i].n);
            std::memcpy(hy + set_off[i], sets[i].y, 4ull * sets[i].n);
        }
        e = hipMemcpyAsync(ws.b[B_INX].p, hx, 4ull * T, hipMemcpyHostToDevice, ws.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws.b[B_INY].p, hy, 4ull * T, hipMemcpyHostToDevice, ws.stream);
        if (e != hipSuccess) return VOR_E_DEVICE;
        in_x = ws.b[B_INX].as<int>();
        in_y = ws.b[B_INY].as<int>();
    }
    // set descriptors, side table and set offsets: uploaded when they differ from what these
    // buffers last received (repeated calls on one shape skip the copies)
    const size_t nd = sizeof(SetDesc) * K, ns = sizeof(SideRel) * ws.sides_h.size();
    std::vector<char> up(nd + ns + 4ull * (K + 1));
    std::memcpy(up.data(), descs.data(), nd);
    if (ns) std::memcpy(up.data() + nd, ws.sides_h.data(), ns);
    std::memcpy(up.data() + nd + ns, set_off.data(), 4ull * (K + 1));
    if (grew || up != ws.up_cache) {
        ws.up_cache.clear();   // valid again only once every copy was issued
        e = hipMemcpyAsync(ws.b[B_SETS].p, descs.data(), nd, hipMemcpyHostToDevice, ws.stream);
        if (e == hipSuccess && ns)
            e = hipMemcpyAsync(ws.b[B_SIDES].p, ws.sides_h.data(), ns, hipMemcpyHostToDevice,
                               ws.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws.b[B_SETOFF].p, set_off.data(), 4ull * (K + 1),
                               hipMemcpyHostToDevice, ws.stream);
        if (e != hipSuccess) return VOR_E_DEVICE;
        ws.up_cache.swap(up);
    }

    void *ptrs[B_COUNT];
    for (int id = 0; id < B_COUNT; ++id) ptrs[id] = ws.b[id].p;
    fill_args(a, ptrs, z, !ws.sides_h.empty(), in_x, in_y, ctx->tune, exact_only, vertices,
              symmetry, (ctx->opts.flags & VOR_TIME_KERNELS) != 0);

    ws.last_timed = a.time_stages;
    if ((e = hipEventRecord(ws.ev0, ws.stream)) != hipSuccess) return VOR_E_DEVICE;
    // one graph for the whole pipeline, or one per stage with events between the stages
    const int ngraphs = a.time_stages ? NSTAGES : 1;
    bool launched = false;
    // a graph pays when it is replayed: the first run of a new shape launches kernel by kernel,
    // and the graph is captured when the same shape comes again (the request loop's batches
    // rarely repeat one)
    const bool same_graph = ws.have_graph && std::memcmp(&ws.gkey, &a, sizeof(a)) == 0;
    const bool repeat = ws.have_last && std::memcmp(&ws.last, &a, sizeof(a)) == 0;
    if (use_graph && !ws.graph_broken && (same_graph || repeat)) {
        if (!same_graph) {
            ws.drop_graph();
            bool ok = true;
            for (int g = 0; g < ngraphs && ok; ++g) {
                ok = hipStreamBeginCapture(ws.stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (!ok) break;
                if (ngraphs == 1) launch_pipeline(a, ws.stream);
                else launch_stage(a, ws.stream, g);
                ok = hipStreamEndCapture(ws.stream, &ws.graph[g]) == hipSuccess;
                if (ok)
                    ok = hipGraphInstantiate(&ws.gexec[g], ws.graph[g], nullptr, nullptr, 0) ==
                         hipSuccess;
            }
            if (ok) {
                ws.gkey = a;
                ws.have_graph = true;
            } else {
                // capture not available for this sequence: launch the kernels directly from now on
                (void)hipGetLastError();
                ws.drop_graph();
                ws.graph_broken = true;
            }
        }
        if (ws.have_graph) {
            for (int g = 0; g < ngraphs; ++g) {
                if (a.time_stages && (e = hipEventRecord(ws.ek[g], ws.stream)) != hipSuccess)
                    return VOR_E_DEVICE;
                if ((e = hipGraphLaunch(ws.gexec[g], ws.stream)) != hipSuccess) return VOR_E_DEVICE;
            }
            if (a.time_stages && (e = hipEventRecord(ws.ek[NSTAGES], ws.stream)) != hipSuccess)
                return VOR_E_DEVICE;
            launched = true;
        }
    }
    if (!launched) {
        for (int g = 0; g < NSTAGES; ++g) {
            if (a.time_stages && (e = hipEventRecord(ws.ek[g], ws.stream)) != hipSuccess)
                return VOR_E_DEVICE;
            launch_stage(a, ws.stream, g);
        }
        if (a.time_stages && (e = hipEventRecord(ws.ek[NSTAGES], ws.stream)) != hipSuccess)
            return VOR_E_DEVICE;
        if ((e = hipGetLastError()) != hipSuccess) return VOR_E_DEVICE;
        ws.last = a;
        ws.have_last = true;
    }
    ws.used_graph = launched;
    if ((e = hipEventRecord(ws.ev1, ws.stream)) != hipSuccess) return VOR_E_DEVICE;
    // small summary in one copy: status words, totals, counters
    if (ws.h_small.ensure(SUMMARY_BYTES) != hipSuccess) return VOR_E_NOMEM;
    e = hipMemcpyAsync(ws.h_small.p, a.small, SUMMARY_BYTES, hipMemcpyDeviceToHost, ws.stream);
    return e == hipSuccess ? VOR_OK : VOR_E_DEVICE;
}

struct Summary {
    int status;
    unsigned long long stats[SL_COUNT];
    long long edges, dels;
    float ms, cells_ms, exact_ms, stage_ms[NSTAGES];
    bool graph;
};

Summary read_summary(Workspace &ws) {
    Summary s;
    const char *hs = (const char *)ws.h_small.p;
    const int *sm = (const int *)hs;
    s.status = sm[0];
    std::memcpy(s.stats, hs + 4 * SMALL_INTS, 8 * SL_COUNT);
    s.edges = sm[16];   // PipeArgs::tot_entries
    s.dels = sm[17];    // PipeArgs::tot_dels
    s.ms = s.cells_ms = s.exact_ms = 0.0f;
    for (auto &x : s.stage_ms) x = 0.0f;
    (void)hipEventElapsedTime(&s.ms, ws.ev0, ws.ev1);
    if (ws.last_timed) {
        for (int g = 0; g < NSTAGES; ++g)
            if (hipEventElapsedTime(&s.stage_ms[g], ws.ek[g], ws.ek[g + 1]) != hipSuccess)
                s.stage_ms[g] = -1.0f;
        s.cells_ms = s.stage_ms[1];
        s.exact_ms = s.stage_ms[3];
    }
    s.graph = ws.used_graph;
    return s;
}


// A host block of at least `bytes` for results: from the pinned pool, else pageable.
std::shared_ptr<OutBlock> take_out_block(const std::shared_ptr<PinnedPool> &pool, size_t bytes) {
    try {
        auto nb = std::make_shared<OutBlock>();
        nb->p = pool->get(bytes, nb->cap);
        if (nb->p) {
            nb->pool = pool;
            return nb;
        }
        nb->p = std::malloc(bytes);
        if (!nb->p) return nullptr;
        nb->cap = bytes;
        return nb;
    } catch (...) {
        return nullptr;
    }
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// Fills a set's result (arrays at the given host addresses) with the run's figures.
void fill_result(vor_result *r, const Summary &sm, uint32_t n, const uint32_t *off,
                 const int32_t *nbr, const vor_rat *vtx, uint64_t m, const uint32_t *del) {
    r->n = n;
    r->cell_off = off;
    r->nbr = nbr;
    r->vtx = vtx;
    r->m = m;
    r->del = del;
    fill_stats(r->stats, sm.stats);
    r->device_ms = sm.ms;
    r->cells_ms = sm.cells_ms;
    r->exact_ms = sm.exact_ms;
    r->grid_ms = sm.stage_ms[0];
    r->adaptive_ms = sm.stage_ms[2];
    r->emit_ms = sm.stage_ms[4];
    r->graph_replayed = sm.graph ? 1 : 0;
    r->status = VOR_OK;
}

// The host copy of a run's output arrays: enqueued on the workspace's stream right behind the
// pipeline, so that the copy engine starts as soon as the kernels end, without a round trip
// through the host.  The totals are not known yet, so the arrays go over at their capacity
// (sized by the Euler bound, a little above the totals: the cells at X's boundary have fewer
// lines); one pool block holds them and the rebased offsets of every set.
struct HostCopy {
    std::shared_ptr<OutBlock> blk;
    size_t o_doff = 0, o_nbr = 0, o_vtx = 0, o_del = 0, o_rel = 0;
};

int enqueue_host_copy(Workspace &ws, const std::shared_ptr<PinnedPool> &pool, const PipeArgs &a,
                      int K, bool vertices, HostCopy &hc) {
    const long long T = a.total;
    const size_t b_off = 4ull * (T + 1), b_nbr = 4ull * a.nbr_cap;
    const size_t b_vtx = vertices ? sizeof(vor_rat) * a.nbr_cap : 0, b_del = 8ull * a.del_cap;
    hc.o_doff = up256(b_off);
    hc.o_nbr = hc.o_doff + up256(b_off);
    hc.o_vtx = hc.o_nbr + up256(b_nbr);
    hc.o_del = hc.o_vtx + up256(b_vtx);
    hc.o_rel = hc.o_del + up256(b_del);
    hc.blk = take_out_block(pool, hc.o_rel + 4ull * (T + K));
    if (!hc.blk) return VOR_E_NOMEM;
    char *hp = (char *)hc.blk->p;
    hipError_t e = hipMemcpyAsync(hp, a.cell_off, b_off, hipMemcpyDeviceToHost, ws.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp + hc.o_doff, a.del_off, b_off, hipMemcpyDeviceToHost, ws.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp + hc.o_nbr, a.nbr, b_nbr, hipMemcpyDeviceToHost, ws.stream);
    if (e == hipSuccess && b_vtx)
        e = hipMemcpyAsync(hp + hc.o_vtx, a.vtx, b_vtx, hipMemcpyDeviceToHost, ws.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp + hc.o_del, a.del, b_del, hipMemcpyDeviceToHost, ws.stream);
    return e == hipSuccess ? VOR_OK : VOR_E_DEVICE;
}

// The results of every set from a finished host copy (the stream is idle): each set's offsets
// rebased to its first entry inside the block, every set's result pointing at its slices and
// holding a reference to the block.
int finish_host(const HostCopy &hc, const PipeArgs &a, const std::vector<SetDesc> &descs,
                const Summary &sm, bool vertices, std::vector<vor_result *> &outs) {
    const long long T = a.total;
    const int K = (int)descs.size();
    char *hp = (char *)hc.blk->p;
    const int *off = (const int *)hp;
    const int *doff = (const int *)(hp + hc.o_doff);
    const int32_t *nbr = (const int32_t *)(hp + hc.o_nbr);
    const vor_rat *vtx = (const vor_rat *)(hp + hc.o_vtx);
    const uint32_t *del = (const uint32_t *)(hp + hc.o_del);
    uint32_t *rel = (uint32_t *)(hp + hc.o_rel);   // set i's n+1 offsets at site_off + i
    // rebasing: pieces of at most 2^20 offsets, spread over a few threads for large runs
    constexpr int PIECE = 1 << 20;
    std::vector<std::pair<int, int>> pieces;   // (set, first offset)
    for (int i = 0; i < K; ++i)
        for (int t = 0; t <= descs[i].n; t += PIECE) pieces.emplace_back(i, t);
    std::atomic<size_t> next{0};
    auto rebase = [&] {
        for (size_t j; (j = next.fetch_add(1)) < pieces.size();) {
            const int i = pieces[j].first, t0 = pieces[j].second;
            const int so = descs[i].site_off, n = descs[i].n, e0 = off[so];
            const int t1 = std::min(n + 1, t0 + PIECE);
            uint32_t *d = rel + so + i;
            for (int t = t0; t < t1; ++t) d[t] = (uint32_t)(off[so + t] - e0);
        }
    };
    const int nt = T + K > (4ll << 20)
                       ? (int)std::min(8u, std::max(1u, std::thread::hardware_concurrency())) : 1;
    std::vector<std::thread> th;
    try {
        for (int k = 1; k < nt; ++k) th.emplace_back(rebase);
    } catch (...) {
    }
    rebase();
    for (auto &x : th) x.join();
    outs.assign(K, nullptr);
    for (int i = 0; i < K; ++i) {
        ResultBox *box;
        vor_result *r = new_result(box);
        if (!r) {
            for (auto &o : outs) vor_result_free(o);
            outs.clear();
            return VOR_E_NOMEM;
        }
        outs[i] = r;
        box->block = hc.blk;
        const int so = descs[i].site_off, n = descs[i].n;
        const int e0 = off[so];
        const int d0 = doff[so], d1 = doff[so + n];
        fill_result(r, sm, (uint32_t)n, rel + so + i, nbr + e0, vertices ? vtx + e0 : nullptr,
                    (uint64_t)(d1 - d0), del + 2ll * d0);
    }
    return VOR_OK;
}

int run_sync(vor_ctx *ctx, Workspace &ws, const std::vector<HostSet> &sets,
             std::vector<vor_result *> &outs, bool device_result) {
    const bool vertices = !(ctx->opts.flags & VOR_NO_VERTICES);
    const bool exact_only = ctx->opts.precision == VOR_EXACT_ONLY;
    const bool sym = (ctx->opts.flags & VOR_CHECK_SYMMETRY) != 0;
    PipeArgs a;
    std::vector<SetDesc> descs;
    std::vector<int> set_off;
    int rc = launch(ctx, ws, sets, vertices, exact_only, sym, ctx->use_graph, a, descs, set_off);
    HostCopy hc;
    if (rc == VOR_OK && !device_result)
        rc = enqueue_host_copy(ws, ctx->pool, a, (int)descs.size(), vertices, hc);
    if (rc != VOR_OK) {
        (void)hipStreamSynchronize(ws.stream);
        return rc;
    }
    if (hipStreamSynchronize(ws.stream) != hipSuccess) return VOR_E_DEVICE;
    Summary sm = read_summary(ws);
    rc = map_status(sm.status);
    if (rc != VOR_OK) return rc;
    if (device_result) {
        ResultBox *box;
        vor_result *r = new_result(box);
        if (!r) return VOR_E_NOMEM;
        r->n = sets[0].n;
        r->cell_off = (const uint32_t *)a.cell_off;
        r->nbr = a.nbr;
        r->vtx = vertices ? (const vor_rat *)a.vtx : nullptr;
        r->m = (uint64_t)sm.dels;
        r->del = a.del;
        fill_stats(r->stats, sm.stats);
        r->device_ms = sm.ms;
        r->cells_ms = sm.cells_ms;
        r->exact_ms = sm.exact_ms;
        r->grid_ms = sm.stage_ms[0];
        r->adaptive_ms = sm.stage_ms[2];
        r->emit_ms = sm.stage_ms[4];
        r->graph_replayed = sm.graph ? 1 : 0;
        r->status = VOR_OK;
        outs.assign(1, r);
        return VOR_OK;
    }
    return finish_host(hc, a, descs, sm, vertices, outs);
}

// ------------------------------------------------------------------------------ request loop
void request_loop(vor_ctx *ctx) {
    (void)hipSetDevice(ctx->device);
    struct InFlight {
        std::vector<std::shared_ptr<Request>> reqs;
        PipeArgs a;
        std::vector<SetDesc> descs;
        std::vector<int> set_off;
        HostCopy hc;     // the outputs' host copy, enqueued behind the pipeline
        bool busy = false;
        size_t fp = 0;   // admitted footprint
    } fl[REQ_WORKSPACES];
    // footprint of the batches on the GPU: admission keeps it within the budget
    size_t in_flight = 0;
    auto any_busy = [&] {
        for (const auto &f : fl)
            if (f.busy) return true;
        return false;
    };
    const bool vertices = !(ctx->opts.flags & VOR_NO_VERTICES);
    const bool exact_only = ctx->opts.precision == VOR_EXACT_ONLY;
    for (;;) {
        bool did = false;
        // completions
        for (int w = 0; w < REQ_WORKSPACES; ++w) {
            if (!fl[w].busy) continue;
            const hipError_t q = hipStreamQuery(ctx->rws[w].stream);
            if (q == hipErrorNotReady) continue;
            did = true;
            fl[w].busy = false;
            in_flight -= fl[w].fp;
            std::vector<vor_result *> outs;
            int rc = q == hipSuccess ? VOR_OK : VOR_E_DEVICE;
            Summary sm{};
            if (rc == VOR_OK) {
                sm = read_summary(ctx->rws[w]);
                rc = map_status(sm.status);
            }
            if (rc == VOR_OK) rc = finish_host(fl[w].hc, fl[w].a, fl[w].descs, sm, vertices, outs);
            fl[w].hc.blk.reset();   // the results hold the block now (or nobody does)
            if (rc != VOR_OK && rc != VOR_E_DEVICE && fl[w].reqs.size() > 1) {
                // an input error of one request: re-run each alone so the others succeed
                std::lock_guard<std::mutex> lk(ctx->qmu);
                for (auto it = fl[w].reqs.rbegin(); it != fl[w].reqs.rend(); ++it) {
                    (*it)->alone = true;
                    ctx->pending.push_front(*it);
                }
                continue;
            }
            // a batch above its share of the budget leaves its buffers sized for it: release
            // them so that the workspaces together keep within the budget
            if (fl[w].fp > ctx->budget / REQ_WORKSPACES) ctx->rws[w].release_buffers();
            const double t = now_s();
            std::lock_guard<std::mutex> lk(ctx->qmu);
            for (size_t i = 0; i < fl[w].reqs.size(); ++i) {
                Request &r = *fl[w].reqs[i];
                r.t_done = t;
                if (rc == VOR_OK) {
                    r.result = outs[i];
                    r.result->t_submit = r.t_submit;
                    r.result->t_admit = r.t_admit;
                    r.result->t_done = r.t_done;
                    r.status = VOR_OK;
                } else {
                    r.status = rc;
                }
                r.release_inputs();
            }
        }
        // admissions
        for (int w = 0; w < REQ_WORKSPACES; ++w) {
            if (fl[w].busy) continue;
            std::vector<std::shared_ptr<Request>> take;
            {
                std::lock_guard<std::mutex> lk(ctx->qmu);
                if (ctx->stop) break;
                size_t used = 0;
                long long sites = 0;
                // what the batches already on the GPU leave of the budget
                const size_t avail = ctx->budget > in_flight ? ctx->budget - in_flight : 0;
                while (!ctx->pending.empty()) {
                    auto &r = ctx->pending.front();
                    const bool alone = r->alone;
                    const size_t fp = r->footprint;
                    const long long ns = (long long)r->x.size();
                    if (take.empty() && fp > ctx->budget) {   // never fits, even alone
                        r->status = VOR_E_NOMEM;
                        r->t_done = now_s();
                        r->release_inputs();
                        ctx->pending.pop_front();
                        continue;
                    }
                    // waits (in order) until the batches in flight leave room for it
                    if (used + fp > avail) break;
                    if (!take.empty() && (alone || sites + ns > ctx->serve_batch_sites)) break;
                    take.push_back(r);
                    used += fp;
                    sites += ns;
                    ctx->pending.pop_front();
                    if (alone) break;
                }
            }
            if (take.empty()) continue;
            did = true;
            std::vector<HostSet> sets;
            const double t = now_s();
            for (auto &r : take) {
                r->t_admit = t;
                HostSet h{(uint32_t)r->x.size(), r->x.data(), r->y.data(), r->box, false};
                if (!r->rx.empty()) {
                    h.nreg = (uint32_t)r->rx.size();
                    h.rx = r->rx.data();
                    h.ry = r->ry.data();
                    h.area = region_area(h.nreg, h.rx, h.ry);
                }
                sets.push_back(h);
            }
            fl[w].reqs = take;
            fl[w].fp = 0;
            for (auto &r : take) fl[w].fp += r->footprint;
            int rc = launch(ctx, ctx->rws[w], sets, vertices, exact_only, false, ctx->use_graph,
                            fl[w].a, fl[w].descs, fl[w].set_off);
            if (rc == VOR_OK)
                rc = enqueue_host_copy(ctx->rws[w], ctx->pool, fl[w].a, (int)fl[w].descs.size(),
                                       vertices, fl[w].hc);
            if (rc != VOR_OK) {
                (void)hipStreamSynchronize(ctx->rws[w].stream);
                fl[w].hc.blk.reset();   // after the stream: no copy still going into it
                std::lock_guard<std::mutex> lk(ctx->qmu);
                for (auto &r : take) {
                    r->status = rc;
                    r->t_done = now_s();
                    r->release_inputs();
                }
                continue;
            }
            fl[w].busy = true;
            in_flight += fl[w].fp;
        }
        {
            std::unique_lock<std::mutex> lk(ctx->qmu);
            if (ctx->stop && !any_busy()) break;
            if (!did) {
                if (any_busy())
                    ctx->qcv.wait_for(lk, std::chrono::microseconds(100));
                else
                    ctx->qcv.wait_for(lk, std::chrono::milliseconds(20),
                                      [&] { return ctx->stop || !ctx->pending.empty(); });
            }
        }
    }
}

}  // namespace

// ------------------------------------------------------------------------------ C ABI
extern "C" {

const char *vor_version(void) { return "vor-mi355x 0.1 (gfx950)"; }

const char *vor_strerror(int s) {
    switch (s) {
    case VOR_OK: return "ok";
    case VOR_PENDING: return "pending";
    case VOR_E_INVAL: return "invalid argument";
    case VOR_E_DOMAIN: return "site not strictly inside the box, or box out of range";
    case VOR_E_DUPLICATE: return "duplicate sites";
    case VOR_E_NOMEM: return "out of device memory / HBM budget";
    case VOR_E_DEVICE: return "HIP device error";
    case VOR_E_TICKET: return "unknown or consumed ticket";
    case VOR_E_CAPACITY: return "cell deeper than the supported capacity";
    default: return "unknown status";
    }
}

int vor_create(const vor_opts *opts, vor_ctx **out) {
    if (!out) return VOR_E_INVAL;
    *out = nullptr;
    vor_ctx *c = new (std::nothrow) vor_ctx();
    if (!c) return VOR_E_NOMEM;
    if (opts) c->opts = *opts;
    else c->opts.precision = VOR_FP32_FILTERED;
    c->device = c->opts.device;
    if (c->opts.precision != VOR_EXACT_ONLY && c->opts.precision != VOR_FP32_FILTERED) {
        delete c;
        return VOR_E_INVAL;
    }
    // exact-only: every cell in the wave-per-cell pass, which prefers a finer grid (36.6 against
    // 38.9 ms for uniform 2^20 sites)
    if (c->opts.precision == VOR_EXACT_ONLY) c->tune = vor_tuning{1.0f, 256, 1, 0, VOR_PATH_GRID_FIRST};
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c->device < 0 || c->device >= ndev) {
        (void)hipGetLastError();
        delete c;
        return VOR_E_DEVICE;
    }
    if (hipSetDevice(c->device) != hipSuccess || c->ws.init() != hipSuccess) {
        delete c;
        return VOR_E_DEVICE;
    }
    const char *g = std::getenv("VOR_NO_GRAPH");
    c->use_graph = !(g && g[0] == '1');
    if (const char *cb = std::getenv("VOR_COOP_BELOW")) c->coop_below = std::atoll(cb);
    if (const char *sb = std::getenv("VOR_SERVE_BATCH_SITES"))
        c->serve_batch_sites = std::min(std::max(std::atoll(sb), 1LL), MAX_RUN_SITES);
    size_t fr = 0, tot = 0;
    (void)hipMemGetInfo(&fr, &tot);
    c->budget = c->opts.hbm_budget_bytes ? c->opts.hbm_budget_bytes : (uint64_t)(tot / 4 * 3);
    *out = c;
    return VOR_OK;
}

int vor_destroy(vor_ctx *ctx) {
    if (!ctx) return VOR_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(ctx->qmu);
        ctx->stop = true;
        ctx->pending.clear();
    }
    ctx->qcv.notify_all();
    if (ctx->loop.joinable()) ctx->loop.join();
    (void)hipSetDevice(ctx->device);
    for (auto &kv : ctx->all)
        if (kv.second->result) vor_result_free(kv.second->result);
    ctx->all.clear();
    ctx->ws.destroy();
    if (ctx->loop_started)
        for (auto &w : ctx->rws) w.destroy();
    delete ctx;
    return VOR_OK;
}

int vor_set_tuning(vor_ctx *ctx, const vor_tuning *t) {
    if (!ctx || !t) return VOR_E_INVAL;
    if (!(t->sites_per_bucket >= 0.0625f && t->sites_per_bucket <= 64.0f)) return VOR_E_INVAL;
    if (t->block != 64 && t->block != 128 && t->block != 256) return VOR_E_INVAL;
    if (t->block_halfwidth < 0 || t->block_halfwidth > 16) return VOR_E_INVAL;
    if (t->leaf_halfwidth < 0 || t->leaf_halfwidth > 4) return VOR_E_INVAL;
    if (t->scan_path != VOR_PATH_GRID_FIRST && t->scan_path != VOR_PATH_TREE) return VOR_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tune = *t;
    return VOR_OK;
}

int vor_get_tuning(vor_ctx *ctx, vor_tuning *t) {
    if (!ctx || !t) return VOR_E_INVAL;
    *t = ctx->tune;
    return VOR_OK;
}

int vor_set_size_tuning(vor_ctx *ctx, const vor_size_tuning *t, uint32_t count) {
    if (!ctx || (count && !t) || count > 64) return VOR_E_INVAL;
    for (uint32_t i = 0; i < count; ++i) {
        const vor_size_tuning &e = t[i];
        if (e.log2n < 0 || e.log2n > 30) return VOR_E_INVAL;
        if (!(e.sites_per_bucket >= 0.0625f && e.sites_per_bucket <= 64.0f)) return VOR_E_INVAL;
        if (e.block_halfwidth < 0 || e.block_halfwidth > 16) return VOR_E_INVAL;
        if (e.leaf_halfwidth < 0 || e.leaf_halfwidth > 4) return VOR_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::lock_guard<std::mutex> lq(ctx->qmu);
    ctx->size_tune.assign(t, t + count);
    return VOR_OK;
}

int vor_compute(vor_ctx *ctx, const vor_set *set, vor_result **out) {
    if (!ctx || !out) return VOR_E_INVAL;
    *out = nullptr;
    HostSet h;
    int rc = check_set(set, h);
    if (rc != VOR_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return VOR_E_DEVICE;
    std::vector<HostSet> sets{h};
    std::vector<vor_result *> outs;
    rc = run_sync(ctx, ctx->ws, sets, outs, (ctx->opts.flags & VOR_RESULT_DEVICE) != 0);
    if (rc == VOR_OK) *out = outs[0];
    return rc;
}

int vor_compute_batch(vor_ctx *ctx, const vor_set *sets, uint32_t k, vor_result **outs) {
    if (!ctx || !sets || !outs || k == 0) return VOR_E_INVAL;
    for (uint32_t i = 0; i < k; ++i) outs[i] = nullptr;
    std::vector<HostSet> hs;
    long long total = 0;
    for (uint32_t i = 0; i < k; ++i) {
        HostSet h;
        int rc = check_set(&sets[i], h);
        if (rc != VOR_OK) return rc;
        if (sets[i].flags & VOR_SET_DEVICE) return VOR_E_INVAL;   // batches take host inputs
        hs.push_back(h);
        total += sets[i].n;
    }
    if (total > MAX_RUN_SITES) return VOR_E_NOMEM;   // more than one run holds
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return VOR_E_DEVICE;
    std::vector<vor_result *> res;
    int rc = run_sync(ctx, ctx->ws, hs, res, false);
    if (rc != VOR_OK) {
        // an input error inside the batch: find the offending sets, run the rest
        if (rc == VOR_E_DEVICE || rc == VOR_E_NOMEM) return rc;
        int first_err = rc;
        for (uint32_t i = 0; i < k; ++i) {
            std::vector<HostSet> one{hs[i]};
            std::vector<vor_result *> r1;
            int r = run_sync(ctx, ctx->ws, one, r1, false);
            if (r == VOR_OK) {
                outs[i] = r1[0];
            } else {
                ResultBox *box;
                vor_result *er = new_result(box);
                if (er) er->status = r;
                outs[i] = er;
                if (r == VOR_E_DEVICE) return r;
            }
        }
        return first_err;
    }
    for (uint32_t i = 0; i < k; ++i) outs[i] = res[i];
    return VOR_OK;
}

int vor_lloyd(vor_ctx *ctx, const vor_set *set, uint32_t iters, int32_t *out_x, int32_t *out_y,
              uint32_t *moved) {
    if (!ctx || !out_x || !out_y) return VOR_E_INVAL;
    HostSet h;
    int rc = check_set(set, h);
    if (rc != VOR_OK) return rc;
    if (h.device) return VOR_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return VOR_E_DEVICE;
    Workspace &ws = ctx->ws;
    const int n = (int)h.n;
    unsigned cap = 1024;
    while (cap < 2u * (unsigned)n) cap <<= 1;
    if (ws.lcx.ensure(4ull * n) != hipSuccess || ws.lcy.ensure(4ull * n) != hipSuccess ||
        ws.lqx.ensure(4ull * n) != hipSuccess || ws.lqy.ensure(4ull * n) != hipSuccess ||
        ws.lkeys.ensure(8ull * cap) != hipSuccess || ws.lcnt.ensure(4ull * cap) != hipSuccess ||
        ws.lflag.ensure(16) != hipSuccess || ws.h_lloyd.ensure(16) != hipSuccess) {
        (void)hipGetLastError();
        return VOR_E_NOMEM;
    }
    int *cx = ws.lcx.as<int>(), *cy = ws.lcy.as<int>(), *qx = ws.lqx.as<int>(),
        *qy = ws.lqy.as<int>(), *flag = ws.lflag.as<int>(), *hf = (int *)ws.h_lloyd.p;
    hipStream_t st = ws.stream;
    if (hipMemcpyAsync(cx, h.x, 4ull * n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(cy, h.y, 4ull * n, hipMemcpyHostToDevice, st) != hipSuccess)
        return VOR_E_DEVICE;
    HostSet hd = h;
    hd.x = cx;
    hd.y = cy;
    hd.device = true;
    const std::vector<HostSet> sets{hd};
    const bool exact_only = ctx->opts.precision == VOR_EXACT_ONLY;
    for (uint32_t it = 0; it < iters; ++it) {
        PipeArgs a;
        std::vector<SetDesc> descs;
        std::vector<int> set_off;
        rc = launch(ctx, ws, sets, true, exact_only, false, ctx->use_graph, a, descs, set_off);
        if (rc != VOR_OK) {
            (void)hipStreamSynchronize(st);
            return rc;
        }
        if (hipStreamSynchronize(st) != hipSuccess) return VOR_E_DEVICE;
        rc = map_status(read_summary(ws).status);
        if (rc != VOR_OK) return rc;
        lloyd_propose(a, cx, cy, qx, qy, st);
        for (int round = 0; round <= n; ++round) {
            lloyd_round(n, qx, qy, cx, cy, ws.lkeys.as<unsigned long long>(), ws.lcnt.as<int>(),
                        cap, flag, st);
            if (hipMemcpyAsync(hf, flag, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return VOR_E_DEVICE;
            if (!*hf) break;
        }
        lloyd_moved(n, qx, qy, cx, cy, flag + 1, st);
        if (hipMemcpyAsync(hf + 1, flag + 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(cx, qx, 4ull * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(cy, qy, 4ull * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return VOR_E_DEVICE;
        if (moved) moved[it] = (uint32_t)hf[1];
    }
    if (hipMemcpyAsync(out_x, cx, 4ull * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(out_y, cy, 4ull * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return VOR_E_DEVICE;
    return VOR_OK;
}

int vor_submit(vor_ctx *ctx, const vor_set *set, uint64_t *ticket) {
    if (!ctx || !ticket) return VOR_E_INVAL;
    HostSet h;
    int rc = check_set(set, h);
    if (rc != VOR_OK) return rc;
    if (set->flags & VOR_SET_DEVICE) return VOR_E_INVAL;
    auto r = std::make_shared<Request>();
    r->x.assign(set->x, set->x + set->n);
    r->y.assign(set->y, set->y + set->n);
    r->box = h.box;
    if (h.nreg) {
        r->rx.assign(h.rx, h.rx + h.nreg);
        r->ry.assign(h.ry, h.ry + h.nreg);
    }
    r->t_submit = now_s();
    SetDesc d{};
    const vor_tuning st = set_tuning(ctx, set->n);
    choose_grid(h.box, set->n, st.sites_per_bucket, st.block_halfwidth, d, h.area);
    r->footprint = footprint_bytes(set->n, (uint64_t)d.gx * d.gy,
                                   !(ctx->opts.flags & VOR_NO_VERTICES), h.nreg ? h.nreg : 4);
    {
        std::lock_guard<std::mutex> lk(ctx->qmu);
        if (ctx->stop) return VOR_E_INVAL;
        if (!ctx->loop_started) {
            for (auto &w : ctx->rws)
                if (w.init() != hipSuccess) return VOR_E_DEVICE;
            ctx->loop_started = true;
            ctx->loop = std::thread(request_loop, ctx);
        }
        r->ticket = ctx->next_ticket++;
        *ticket = r->ticket;
        ctx->all[r->ticket] = r;
        ctx->pending.push_back(r);
    }
    ctx->qcv.notify_all();
    return VOR_OK;
}

int vor_poll(vor_ctx *ctx, uint64_t ticket, vor_result **out) {
    if (!ctx || !out) return VOR_E_INVAL;
    *out = nullptr;
    std::lock_guard<std::mutex> lk(ctx->qmu);
    auto it = ctx->all.find(ticket);
    if (it == ctx->all.end()) return VOR_E_TICKET;
    Request &r = *it->second;
    if (r.status == VOR_PENDING) return VOR_PENDING;
    const int st = r.status;
    if (st == VOR_OK) {
        *out = r.result;   // carries the request's latency stamps
        r.result = nullptr;
    }
    ctx->all.erase(it);    // consumed: the context keeps nothing of it
    return st;
}

int vor_ticket_count(vor_ctx *ctx, uint64_t *held) {
    if (!ctx || !held) return VOR_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->qmu);
    *held = ctx->all.size();
    return VOR_OK;
}

int vor_footprint(vor_ctx *ctx, const vor_set *set, uint64_t *bytes) {
    if (!ctx || !bytes) return VOR_E_INVAL;
    HostSet h;
    const int rc = check_set(set, h);
    if (rc != VOR_OK) return rc;
    SetDesc d{};
    const vor_tuning st = set_tuning(ctx, set->n);
    choose_grid(h.box, set->n, st.sites_per_bucket, st.block_halfwidth, d, h.area);
    *bytes = footprint_bytes(set->n, (uint64_t)d.gx * d.gy, !(ctx->opts.flags & VOR_NO_VERTICES),
                             h.nreg ? h.nreg : 4);
    return VOR_OK;
}

int vor_ticket_times(vor_ctx *ctx, uint64_t ticket, double *ts, double *ta, double *td) {
    if (!ctx) return VOR_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->qmu);
    auto it = ctx->all.find(ticket);
    if (it == ctx->all.end()) return VOR_E_TICKET;
    if (ts) *ts = it->second->t_submit;
    if (ta) *ta = it->second->t_admit;
    if (td) *td = it->second->t_done;
    return VOR_OK;
}

void vor_result_free(vor_result *r) {
    if (!r) return;
    delete reinterpret_cast<ResultBox *>(r);
}

int vor_result_layout(const vor_result *const *results, uint32_t k, uint64_t *table) {
    if (!results || !table) return VOR_E_INVAL;
    for (uint32_t i = 0; i < k; ++i) {
        uint64_t *t = table + 8ull * i;
        std::memset(t, 0, 8 * sizeof(uint64_t));
        const vor_result *r = results[i];
        if (!r) continue;
        t[0] = r->n;
        t[1] = r->m;
        t[2] = (uint64_t)(uintptr_t)r->cell_off;
        t[3] = (uint64_t)(uintptr_t)r->nbr;
        t[4] = (uint64_t)(uintptr_t)r->vtx;
        t[5] = (uint64_t)(uintptr_t)r->del;
        // vor_result is the first member of ResultBox
        const ResultBox *box = reinterpret_cast<const ResultBox *>(r);
        if (box->block && r->status == VOR_OK) {
            t[6] = (uint64_t)(uintptr_t)box->block->p;
            t[7] = box->block->cap;
        }
    }
    return VOR_OK;
}

int vor_result_to_host(vor_ctx *ctx, const vor_result *dev, vor_result **out) {
    if (!ctx || !dev || !out) return VOR_E_INVAL;
    *out = nullptr;
    if (!dev->cell_off || (dev->m && !dev->del)) return VOR_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return VOR_E_DEVICE;
    ResultBox *box;
    vor_result *r = new_result(box);
    if (!r) return VOR_E_NOMEM;
    const size_t n = dev->n;
    box->off.resize(n + 1);
    hipError_t e = hipMemcpy(box->off.data(), dev->cell_off, 4 * (n + 1), hipMemcpyDeviceToHost);
    const size_t E = e == hipSuccess ? box->off[n] : 0;
    if (e == hipSuccess && E && !dev->nbr) e = hipErrorInvalidValue;
    if (e == hipSuccess) {
        box->nbr.resize(E);
        if (E) e = hipMemcpy(box->nbr.data(), dev->nbr, 4 * E, hipMemcpyDeviceToHost);
    }
    if (e == hipSuccess && dev->vtx) {
        box->vtx.resize(E);
        if (E) e = hipMemcpy(box->vtx.data(), dev->vtx, sizeof(vor_rat) * E, hipMemcpyDeviceToHost);
    }
    if (e == hipSuccess) {
        box->del.resize(2 * dev->m);
        if (dev->m) e = hipMemcpy(box->del.data(), dev->del, 8 * dev->m, hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete box;
        return e == hipErrorInvalidValue ? VOR_E_INVAL : VOR_E_DEVICE;
    }
    *r = *dev;
    r->cell_off = box->off.data();
    r->nbr = box->nbr.data();
    r->vtx = dev->vtx ? box->vtx.data() : nullptr;
    r->del = box->del.data();
    *out = r;
    return VOR_OK;
}

}  // extern "C"
