// hbm_probe.hip -- streaming copy and reads of a known size (bandwidth
// ceiling, counter calibration, and whether a re-read is served faster than a
// first read; see include/hbm_probe.h).
#include <hip/hip_runtime.h>

#include "../../include/hbm_probe.h"

namespace {

__global__ void __launch_bounds__(256) k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(256) k_read(const double2 *__restrict__ src, size_t n, double *__restrict__ sink)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 v = src[i];
        acc += v.x + v.y;
    }
    if (acc != 0.0) sink[blockIdx.x] = acc; // the buffer is zero: never taken, but keeps the loads
}

} // namespace

extern "C" int hbm_read_probe(size_t bytes, int reps, double *ms)
{
    if (!ms || reps < 1 || bytes == 0 || bytes % 64) return -1;
    void *a = nullptr;
    double *sink = nullptr;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    const dim3 grid((unsigned)cus * 8), block(256);
    if (hipMalloc(&a, bytes) != hipSuccess) return -2;
    if (hipMalloc((void **)&sink, grid.x * sizeof(double)) != hipSuccess) {
        (void)hipFree(a);
        return -2;
    }
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float t = 0.f;
    const size_t n = bytes / sizeof(double2);
    if (hipMemset(a, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = -3;
    } else {
        hipLaunchKernelGGL(k_read, grid, block, 0, 0, (const double2 *)a, n, sink);
        (void)hipEventRecord(e0, 0);
        for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_read, grid, block, 0, 0, (const double2 *)a, n, sink);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -3;
        *ms = (double)t / reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(sink);
    return rc;
}

extern "C" int hbm_reread_probe(size_t bytes, size_t flush_bytes, int reps, double *ms_hot, double *ms_cold)
{
    if (!ms_hot || !ms_cold || reps < 1 || bytes == 0 || bytes % 64 || flush_bytes == 0 || flush_bytes % 64)
        return -1;
    void *a = nullptr, *f = nullptr;
    double *sink = nullptr;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    const dim3 grid((unsigned)cus * 8), block(256);
    if (hipMalloc(&a, bytes) != hipSuccess) return -2;
    if (hipMalloc(&f, flush_bytes) != hipSuccess) {
        (void)hipFree(a);
        return -2;
    }
    if (hipMalloc((void **)&sink, grid.x * sizeof(double)) != hipSuccess) {
        (void)hipFree(a);
        (void)hipFree(f);
        return -2;
    }
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t n = bytes / sizeof(double2), nf = flush_bytes / sizeof(double2);
    float best_hot = 1e30f, best_cold = 1e30f;
    if (hipMemset(a, 0, bytes) != hipSuccess || hipMemset(f, 0, flush_bytes) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = -3;
    } else {
        for (int r = 0; r < reps && rc == 0; ++r) {
            for (int cold = 0; cold < 2 && rc == 0; ++cold) {
                // a first read of the buffer, then (cold) a read of the flush buffer, then the timed read
                hipLaunchKernelGGL(k_read, grid, block, 0, 0, (const double2 *)a, n, sink);
                if (cold) hipLaunchKernelGGL(k_read, grid, block, 0, 0, (const double2 *)f, nf, sink);
                (void)hipEventRecord(e0, 0);
                hipLaunchKernelGGL(k_read, grid, block, 0, 0, (const double2 *)a, n, sink);
                (void)hipEventRecord(e1, 0);
                float t = 0.f;
                if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -3;
                float &best = cold ? best_cold : best_hot;
                if (t < best) best = t;
            }
        }
        *ms_hot = best_hot;
        *ms_cold = best_cold;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(f);
    (void)hipFree(sink);
    return rc;
}

extern "C" int hbm_copy_probe(size_t bytes, int reps, double *ms)
{
    if (!ms || reps < 1 || bytes == 0 || bytes % 64) return -1;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return -2;
    if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipFree(a);
        return -2;
    }
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t n = bytes / sizeof(double2);
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    const dim3 grid((unsigned)cus * 8), block(256);
    float t = 0.f;
    if (hipMemset(a, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = -3;
        goto done;
    }
    hipLaunchKernelGGL(k_copy, grid, block, 0, 0, (const double2 *)a, (double2 *)b, n);
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_copy, grid, block, 0, 0, (const double2 *)a, (double2 *)b, n);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -3;
    *ms = (double)t / reps;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}
