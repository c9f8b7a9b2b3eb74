// vor_noalloc.cpp -- vor_compute for callers that cannot allocate device memory: every
// working buffer of one pipeline run is carved out of a fixed device array of this file.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "vor.h"
#include "vor_internal.h"
#include "vor_plan.h"

using namespace vor;

namespace {

// Working memory of vor_compute_noalloc: one array per GPU, held until the process ends.  Host
// code never passes this name to a kernel or a copy: it stands for a host-side shadow; the
// device address comes from hipGetSymbolAddress, once per device, and only that is used.
static __device__ __align__(256) unsigned char scratch[VOR_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
struct NoallocDevice {
    std::mutex mu;           // serialises the calls of this process on the device
    void *ptr = nullptr;     // device address of `scratch` on it
    bool ready = false;
};
NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];

}  // namespace

extern "C" int vor_compute_noalloc(int32_t device, void *stream, const vor_set *set, int32_t precision,
                        uint32_t *cell_off, int32_t *nbr, vor_rat *vtx, uint64_t nbr_cap,
                        uint32_t *del, uint64_t del_cap, uint64_t *entries, uint64_t *m,
                        vor_stats *stats) {
    if (!cell_off || !nbr || !del || !entries || !m) return VOR_E_INVAL;
    if (precision != VOR_EXACT_ONLY && precision != VOR_FP32_FILTERED) return VOR_E_INVAL;
    HostSet h;
    int rc = check_set(set, h);
    if (rc != VOR_OK) return rc;
    if (h.n > VOR_NOALLOC_MAX_SITES) return VOR_E_INVAL;
    const long long n = h.n, sides = h.nreg ? h.nreg : 4;
    if ((long long)nbr_cap < entry_cap(n, sides) || (long long)del_cap < 3 * n + 8)
        return VOR_E_INVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
        device >= NOALLOC_MAX_DEVICES) {
        (void)hipGetLastError();
        return VOR_E_DEVICE;
    }
    NoallocDevice &D = g_noalloc[device];
    std::lock_guard<std::mutex> lk(D.mu);
    if (hipSetDevice(device) != hipSuccess) return VOR_E_DEVICE;
    if (!D.ready) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return VOR_E_DEVICE;
        }
        D.ptr = p;
        D.ready = true;
    }
    // the run's descriptors, on the stack (copied to the device below; the call waits for its
    // work, so they outlive every copy)
    const vor_tuning tune = precision == VOR_EXACT_ONLY
                                ? vor_tuning{1.0f, 256, 1, 0, VOR_PATH_GRID_FIRST}
                                : vor_tuning{1.5f, 256, 2, 0, VOR_PATH_GRID_FIRST};
    SetDesc desc;
    SideRel side_tab[VOR_MAX_SIDES];
    plan_set(tune, h, 0, 0, 0, desc, side_tab);
    const int set_off[2] = {0, (int)n};
    RunSizes z;
    rc = run_sizes(n, (long long)desc.gx * desc.gy, sides, 1, h.nreg, vtx != nullptr,
                   precision == VOR_EXACT_ONLY, 4096, z, 2048);
    if (rc != VOR_OK) return rc;
    // carve the buffers out of the array; the outputs are the caller's
    void *p[B_COUNT];
    size_t off = 0;
    for (int id = 0; id < B_COUNT; ++id) {
        const bool caller = id == B_CELLOFF || id == B_NBR || id == B_VTX || id == B_DEL ||
                            ((id == B_INX || id == B_INY) && h.device);
        p[id] = nullptr;
        if (caller) continue;
        p[id] = (char *)D.ptr + off;
        off += (z.b[id] + 255) & ~(size_t)255;
    }
    if (off > VOR_NOALLOC_SCRATCH_BYTES) return VOR_E_INVAL;   // beyond the array (not expected
                                                                // for n <= the maximum)
    hipStream_t st = (hipStream_t)stream;
    const int *in_x = h.device ? h.x : (const int *)p[B_INX];
    const int *in_y = h.device ? h.y : (const int *)p[B_INY];
    hipError_t e = hipSuccess;
    if (!h.device) {
        e = hipMemcpyAsync(p[B_INX], h.x, 4ull * n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(p[B_INY], h.y, 4ull * n, hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(p[B_SETS], &desc, sizeof(desc), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p[B_SETOFF], set_off, sizeof(set_off), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && h.nreg)
        e = hipMemcpyAsync(p[B_SIDES], side_tab, sizeof(SideRel) * h.nreg, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return VOR_E_DEVICE;
    }
    PipeArgs a;
    fill_args(a, p, z, h.nreg > 0, in_x, in_y, tune, precision == VOR_EXACT_ONLY, vtx != nullptr,
              false, false);
    a.cell_off = (int *)cell_off;
    a.nbr = nbr;
    a.vtx = vtx;
    a.del = del;
    launch_pipeline(a, st);
    // status, totals and counters back to the host, one copy
    alignas(8) unsigned char sum[SUMMARY_BYTES];
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(sum, a.small, SUMMARY_BYTES, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return VOR_E_DEVICE;
    }
    const int *small = (const int *)sum;
    unsigned long long sl[SL_COUNT];
    std::memcpy(sl, sum + 4 * SMALL_INTS, sizeof(sl));
    rc = map_status(small[0]);
    if (rc != VOR_OK) return rc;
    *entries = (uint64_t)small[16];   // PipeArgs::tot_entries
    *m = (uint64_t)small[17];         // PipeArgs::tot_dels
    if (stats) fill_stats(*stats, sl);
    return VOR_OK;
}
