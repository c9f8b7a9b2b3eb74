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

// ------------------------------------------------------------------------------ regions
namespace vor {

// The candidate regions of one ray bound (Method 11.6 with the lemma on sites in the large
// square), computed by the same device functions the scans use: need_rect (bucket rectangle of
// the uniform grid), need_crect (coordinate rectangle of the adaptive scan) and need_disk (the
// disk the adaptive scan prunes with), plus the disk test of one given point.
__global__ void k_region_diag(int64_t n, const int32_t *__restrict__ geom,
                              const int64_t *__restrict__ dir, const float *__restrict__ T,
                              const int32_t *__restrict__ z, int32_t *__restrict__ rects,
                              float *__restrict__ disk, int32_t *__restrict__ inside,
                              int32_t *__restrict__ sigma, float *__restrict__ ds) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t *g = geom + 7 * i;
    Cell C{};
    C.px = g[0];
    C.py = g[1];
    C.pxf = (float)g[0];
    C.pyf = (float)g[1];
    C.W = g[2];
    C.H = g[3];
    C.s = g[4];
    C.gx = g[5];
    C.gy = g[6];
    C.bx = min(C.px / C.s, C.gx - 1);
    C.by = min(C.py / C.s, C.gy - 1);
    const i128 x = ((i128)dir[4 * i] << 64) | (i128)(uint64_t)dir[4 * i + 1];
    const i128 y = ((i128)dir[4 * i + 2] << 64) | (i128)(uint64_t)dir[4 * i + 3];
    const Dir d = make_dir(x, y);
    const Rect R = need_rect(C, T[i], d.fx, d.fy);
    const Rect Q = need_crect(C, T[i], d.fx, d.fy);
    const Disk D = need_disk(C, T[i], d.fx, d.fy);
    int32_t *r = rects + 8 * i;
    r[0] = R.x0; r[1] = R.x1; r[2] = R.y0; r[3] = R.y1;
    r[4] = Q.x0; r[5] = Q.x1; r[6] = Q.y0; r[7] = Q.y1;
    disk[3 * i] = D.cx;
    disk[3 * i + 1] = D.cy;
    disk[3 * i + 2] = D.r2;
    inside[i] = in_disk(D, (float)(z[2 * i] - C.px), (float)(z[2 * i + 1] - C.py)) ? 1 : 0;
    sigma[i] = d.sigma;
    ds[2 * i] = d.fx;
    ds[2 * i + 1] = d.fy;
}

}  // namespace vor

extern "C" int vor_region_diag(int32_t device, int64_t n, const int32_t *geom,
                               const int64_t *dir, const float *T, const int32_t *z,
                               int32_t *rects, float *disk, int32_t *inside, int32_t *sigma,
                               float *ds) {
    using namespace vor;
    if (n < 0) return VOR_E_INVAL;
    if (n == 0) return VOR_OK;
    if (!geom || !dir || !T || !z || !rects || !disk || !inside || !sigma || !ds)
        return VOR_E_INVAL;
    const int64_t LIM = (int64_t)1 << 24;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *g = geom + 7 * i;
        const int32_t px = g[0], py = g[1], W = g[2], H = g[3], s = g[4], gx = g[5], gy = g[6];
        if (W < 1 || H < 1 || W > LIM || H > LIM || s < 1 || gx < 1 || gy < 1) return VOR_E_INVAL;
        if ((int64_t)gx * s < W || (int64_t)gy * s < H) return VOR_E_INVAL;   // grid covers X
        if (px < 0 || px > W || py < 0 || py > H) return VOR_E_INVAL;
        if (z[2 * i] < -LIM || z[2 * i] > 2 * LIM || z[2 * i + 1] < -LIM || z[2 * i + 1] > 2 * LIM)
            return VOR_E_INVAL;
        if (!(T[i] >= 0.0f)) return VOR_E_INVAL;   // +inf allowed, NaN not
        const int64_t xh = dir[4 * i], yh = dir[4 * i + 2];
        if (xh >= ((int64_t)1 << 36) || xh < -((int64_t)1 << 36) || yh >= ((int64_t)1 << 36) ||
            yh < -((int64_t)1 << 36))
            return VOR_E_INVAL;
        if ((xh | dir[4 * i + 1] | yh | dir[4 * i + 3]) == 0) return VOR_E_INVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return VOR_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return VOR_E_DEVICE;
    // inputs geom, dir, T, z; outputs rects, disk, inside, sigma, ds
    const size_t sizes[9] = {(size_t)n * 28, (size_t)n * 32, (size_t)n * 4, (size_t)n * 8,
                             (size_t)n * 32, (size_t)n * 12, (size_t)n * 4, (size_t)n * 4,
                             (size_t)n * 8};
    size_t total = 0, offs[9];
    for (int k = 0; k < 9; ++k) {
        offs[k] = total;
        total += (sizes[k] + 255) & ~(size_t)255;
    }
    char *buf = nullptr;
    if (hipMalloc(&buf, total) != hipSuccess) return VOR_E_NOMEM;
    const void *src[4] = {geom, dir, T, z};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        e = hipMemcpy(buf + offs[k], src[k], sizes[k], hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const int TB = 256;
        const unsigned blocks = (unsigned)((n + TB - 1) / TB);
        hipLaunchKernelGGL(k_region_diag, dim3(blocks), dim3(TB), 0, 0, n,
                           (const int32_t *)(buf + offs[0]), (const int64_t *)(buf + offs[1]),
                           (const float *)(buf + offs[2]), (const int32_t *)(buf + offs[3]),
                           (int32_t *)(buf + offs[4]), (float *)(buf + offs[5]),
                           (int32_t *)(buf + offs[6]), (int32_t *)(buf + offs[7]),
                           (float *)(buf + offs[8]));
        e = hipGetLastError();
    }
    void *dst[5] = {rects, disk, inside, sigma, ds};
    for (int k = 0; k < 5 && e == hipSuccess; ++k)
        e = hipMemcpy(dst[k], buf + offs[4 + k], sizes[4 + k], hipMemcpyDeviceToHost);
    const hipError_t ef = hipFree(buf);
    return (e == hipSuccess && ef == hipSuccess) ? VOR_OK : VOR_E_DEVICE;
}
