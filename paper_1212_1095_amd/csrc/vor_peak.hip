// vor_peak.hip -- measured peaks of the GPU the library runs on, for the roofline figures beside
// the published ones: an FP32 FMA loop (the vector rate the cell kernels can use, built like
// them without packed FP32) and a plain device-to-device copy (the HBM rate).  Not on the hot
// path.
#include <hip/hip_runtime.h>

#include "vor.h"

namespace vor {

constexpr int PEAK_BLOCK = 256;
constexpr int PEAK_CHAINS = 8;   // independent FMA chains per thread

// Every thread runs PEAK_CHAINS dependent FMA chains of `iters` steps and writes one sum, so
// that nothing is removed.  x -> a x + b with |a| < 1 keeps the values bounded.
__global__ __launch_bounds__(PEAK_BLOCK) void k_peak_fma(float *__restrict__ out, int iters,
                                                         float a, float b) {
    const int t = blockIdx.x * PEAK_BLOCK + threadIdx.x;
    float x[PEAK_CHAINS];
#pragma unroll
    for (int c = 0; c < PEAK_CHAINS; ++c) x[c] = (float)(threadIdx.x + c) * 1.0e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PEAK_CHAINS; ++c) x[c] = fmaf(x[c], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < PEAK_CHAINS; ++c) s += x[c];
    out[t] = s;
}

// Grid-stride copy of n 16-byte words.
__global__ __launch_bounds__(PEAK_BLOCK) void k_peak_copy(const float4 *__restrict__ src,
                                                          float4 *__restrict__ dst, long long n) {
    const long long stride = (long long)gridDim.x * PEAK_BLOCK;
    for (long long i = (long long)blockIdx.x * PEAK_BLOCK + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace vor

namespace {

// Mean time of `reps` launches after one warm-up, from events on a stream of the call's own.
template <class F>
hipError_t time_launches(F launch, int reps, hipStream_t st, float *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    *ms = t / (float)reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

extern "C" int vor_peak_fp32(int32_t device, double *tflops) {
    using namespace vor;
    if (!tflops) return VOR_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return VOR_E_DEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        return VOR_E_DEVICE;
    const int blocks = cus * 16;   // 16 blocks of 4 waves per CU: every SIMD full
    const int iters = 4096;
    float *out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * PEAK_BLOCK) != hipSuccess) {
        (void)hipGetLastError();
        return VOR_E_NOMEM;
    }
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = time_launches(
            [&] {
                k_peak_fma<<<blocks, PEAK_BLOCK, 0, st>>>(out, iters, 0.999999f, 1.0e-7f);
            },
            10, st, &ms);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(out);
    if (e != hipSuccess || !(ms > 0.0f)) return VOR_E_DEVICE;
    const double flops = 2.0 * PEAK_CHAINS * (double)iters * blocks * PEAK_BLOCK;
    *tflops = flops / (ms * 1.0e-3) / 1.0e12;
    return VOR_OK;
}

extern "C" int vor_peak_copy(int32_t device, uint64_t bytes, double *gbps) {
    using namespace vor;
    if (!gbps || bytes < 16) return VOR_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return VOR_E_DEVICE;
    const long long n = (long long)(bytes / 16);
    float4 *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, 16ull * n) != hipSuccess || hipMalloc(&dst, 16ull * n) != hipSuccess) {
        (void)hipGetLastError();
        if (src) (void)hipFree(src);
        return VOR_E_NOMEM;
    }
    hipStream_t st = nullptr;
    hipError_t e = hipMemsetAsync(src, 0, 16ull * n, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    int cus = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    float ms = 0.0f;
    if (e == hipSuccess && cus > 0)
        e = time_launches(
            [&] { k_peak_copy<<<cus * 8, PEAK_BLOCK, 0, st>>>(src, dst, n); }, 10, st, &ms);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (e != hipSuccess || cus <= 0 || !(ms > 0.0f)) return VOR_E_DEVICE;
    *gbps = 2.0 * 16.0 * (double)n / (ms * 1.0e-3) / 1.0e9;
    return VOR_OK;
}
