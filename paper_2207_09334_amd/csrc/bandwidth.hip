// Streaming reference kernels: the HBM bandwidth a plain HIP kernel reaches on this device,
// the yardstick for the step's measured traffic.  A copy (read and write every byte once) and a
// read-only sum, both with 16-byte accesses, four in flight per lane, and a grid of eight
// 256-thread workgroups per compute unit walking the buffer in grid-sized strides.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace {

constexpr int kUnroll = 4;

__global__ void __launch_bounds__(256) stream_copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                          long n) {
    const long stride = (long)gridDim.x * blockDim.x;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        float4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(256) stream_read_kernel(const float4* __restrict__ src, long n, float* out) {
    const long stride = (long)gridDim.x * blockDim.x;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.0f;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        float4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    for (; i < n; i += stride) s += src[i].x;
    // one value per thread keeps the loads live; the sum itself is not used
    out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void fill_kernel(float4* p, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
}

}  // namespace

using cronos::fail;

extern "C" cronos_status cronos_stream_bandwidth(int32_t device, int64_t bytes, int32_t reps, double* copy_gbs,
                                                 double* read_gbs) {
    cronos::clear_error();
    if (bytes < (1 << 20) || reps < 1) return fail(CRONOS_EINVAL, "stream_bandwidth: bytes >= 1 MiB and reps >= 1");
    if (hipSetDevice(device) != hipSuccess) return fail(CRONOS_EDEVICE, "stream_bandwidth: no device %d", device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(CRONOS_EDEVICE, "stream_bandwidth: properties");
    const long n = (long)(bytes / 16);
    const int grid = prop.multiProcessorCount * 8;
    float4 *src = nullptr, *dst = nullptr;
    float* out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    cronos_status status = CRONOS_OK;
    auto run = [&]() -> cronos_status {
        if (hipMalloc((void**)&src, n * sizeof(float4)) != hipSuccess ||
            hipMalloc((void**)&dst, n * sizeof(float4)) != hipSuccess ||
            hipMalloc((void**)&out, (size_t)grid * 256 * sizeof(float)) != hipSuccess)
            return fail(CRONOS_ENOMEM, "stream_bandwidth: device allocation of 2 x %lld bytes failed", (long long)bytes);
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess)
            return fail(CRONOS_EDEVICE, "stream_bandwidth: stream or event creation failed");
        hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, st, src, n);
        hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, st, dst, n);
        double best_copy = 1e300, best_read = 1e300;
        for (int r = 0; r <= reps; ++r) {   // the first round warms up
            float ms = 0.0f;
            hipEventRecord(e0, st);
            hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(256), 0, st, src, dst, n);
            hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return fail(CRONOS_EDEVICE, "stream_bandwidth: copy timing failed");
            if (r) best_copy = std::min(best_copy, (double)ms);
            hipEventRecord(e0, st);
            hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, st, src, n, out);
            hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return fail(CRONOS_EDEVICE, "stream_bandwidth: read timing failed");
            if (r) best_read = std::min(best_read, (double)ms);
        }
        if (hipGetLastError() != hipSuccess) return fail(CRONOS_EDEVICE, "stream_bandwidth: kernel launch failed");
        if (copy_gbs) *copy_gbs = 2.0 * (double)n * 16.0 / (best_copy * 1e-3) / 1e9;
        if (read_gbs) *read_gbs = (double)n * 16.0 / (best_read * 1e-3) / 1e9;
        return CRONOS_OK;
    };
    status = run();
    if (st) (void)hipStreamSynchronize(st);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    return status;
}
