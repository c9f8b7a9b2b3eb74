// vor_diag.hip -- diagnostic entry point: the FP32 filter keys of single (line, ray) instances,
// computed by the same device functions that the cell passes use (Method 11.5 filter in
// front of the exact comparisons of eq. Tdef).  Not on the hot path: it exists so that the
// bounds the filter relies on can be checked against exact rational arithmetic on the host.
#include "vor.h"
#include "vor_cell.hpp"

namespace vor {

__global__ void k_filter_keys(int64_t n, const int32_t *__restrict__ kind,
                              const int32_t *__restrict__ nx, const int32_t *__restrict__ ny,
                              const int64_t *__restrict__ c, const int64_t *__restrict__ dir,
                              float *__restrict__ out, int32_t *__restrict__ sigma) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const i128 x = ((i128)dir[4 * i] << 64) | (i128)(uint64_t)dir[4 * i + 1];
    const i128 y = ((i128)dir[4 * i + 2] << 64) | (i128)(uint64_t)dir[4 * i + 3];
    const Dir d = make_dir(x, y);
    const int a = nx[i], b = ny[i];
    const float fa = (float)a, fb = (float)b;
    uint64_t cc;
    float klo, khi;
    if (kind[i] == 0) {   // site: delta = (a, b), q = |delta|^2 rounded in FP32 (site_q)
        cc = (uint64_t)((int64_t)a * a + (int64_t)b * b);
        const float q = site_q(fa, fb);
        klo = key_lo_line(q, fa, fb, d.fx, d.fy);
        khi = key_hi_line(q, fa, fb, d.fx, d.fy);
    } else {              // general line (N, c): c converted to FP32 as for the box sides
        cc = (uint64_t)c[i];
        klo = key_lo_line((float)c[i], fa, fb, d.fx, d.fy);
        khi = key_hi_line((float)c[i], fa, fb, d.fx, d.fy);
    }
    const i128 den = (i128)a * d.x + (i128)b * d.y;
    XBest xb;
    xb.id = 0;
    xb.nx = a;
    xb.ny = b;
    xb.c = cc;
    xb.den = den > 0 ? (u128)den : (u128)0;
    xb.have = den > 0;
    float *o = out + 8 * i;
    o[0] = klo;
    o[1] = khi;
    o[2] = klo * CERT_DN;
    o[3] = khi * CERT_UP;
    o[4] = x_upper(xb, d);
    o[5] = d.fx;
    o[6] = d.fy;
    o[7] = 0.0f;
    sigma[i] = d.sigma;
}

}  // namespace vor

extern "C" int vor_filter_keys(int32_t device, int64_t n, const int32_t *kind, const int32_t *nx,
                               const int32_t *ny, const int64_t *c, const int64_t *dir,
                               float *out, int32_t *sigma) {
    using namespace vor;
    if (n < 0) return VOR_E_INVAL;
    if (n == 0) return VOR_OK;
    if (!kind || !nx || !ny || !c || !dir || !out || !sigma) return VOR_E_INVAL;
    const int64_t LIM = (int64_t)1 << 24;
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != 0 && kind[i] != 1) return VOR_E_INVAL;
        if (nx[i] < -LIM || nx[i] > LIM || ny[i] < -LIM || ny[i] > LIM) return VOR_E_INVAL;
        if (nx[i] == 0 && ny[i] == 0) return VOR_E_INVAL;
        if (kind[i] == 1 && (c[i] <= 0 || c[i] > ((int64_t)1 << 50))) return VOR_E_INVAL;
        const int64_t xh = dir[4 * i], yh = dir[4 * i + 2];
        // |component| < 2^100 keeps N.d inside 128 bits (vertex directions of the walk stay
        // below 2^77: products of a right-hand side < 2^50 and a normal < 2^25, twice)
        if (xh >= ((int64_t)1 << 36) || xh < -((int64_t)1 << 36) || yh >= ((int64_t)1 << 36) ||
            yh < -((int64_t)1 << 36))
            return VOR_E_INVAL;
        if ((xh | dir[4 * i + 1] | yh | dir[4 * i + 3]) == 0) return VOR_E_INVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return VOR_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return VOR_E_DEVICE;
    const size_t b4 = (size_t)n * 4, b8 = (size_t)n * 8;
    const size_t sizes[7] = {b4, b4, b4, b8, 4 * b8, 8 * b4, b4};
    size_t total = 0, offs[7];
    for (int k = 0; k < 7; ++k) {
        offs[k] = total;
        total += (sizes[k] + 255) & ~(size_t)255;
    }
    char *buf = nullptr;
    if (hipMalloc(&buf, total) != hipSuccess) return VOR_E_NOMEM;
    const void *src[5] = {kind, nx, ny, c, dir};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 5 && e == hipSuccess; ++k)
        e = hipMemcpy(buf + offs[k], src[k], sizes[k], hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const int T = 256;
        const unsigned blocks = (unsigned)((n + T - 1) / T);
        hipLaunchKernelGGL(k_filter_keys, dim3(blocks), dim3(T), 0, 0, n,
                           (const int32_t *)(buf + offs[0]), (const int32_t *)(buf + offs[1]),
                           (const int32_t *)(buf + offs[2]), (const int64_t *)(buf + offs[3]),
                           (const int64_t *)(buf + offs[4]), (float *)(buf + offs[5]),
                           (int32_t *)(buf + offs[6]));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, buf + offs[5], sizes[5], hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(sigma, buf + offs[6], sizes[6], hipMemcpyDeviceToHost);
    const hipError_t ef = hipFree(buf);
    return (e == hipSuccess && ef == hipSuccess) ? VOR_OK : VOR_E_DEVICE;
}
