// lgf_util.hip -- measurement utility: the bandwidth of a plain device copy,
// the practical ceiling against which the streaming sweep kernels are measured
// (one 16-byte vector per lane, non-temporal loads and stores, one pass).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lgf.h"
#include "lgf_device.hpp"
#include "lgf_host.hpp"

namespace lgf {

__global__ void __launch_bounds__(256) copy_kernel(const v4f *__restrict__ src, v4f *__restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

__global__ void __launch_bounds__(256) fill_kernel(v4f *__restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = v4f{1.f, 2.f, 3.f, (float)(i & 1023u)};
}

}  // namespace lgf

extern "C" lgf_status lgf_copy_bandwidth(size_t bytes, int reps, void *hip_stream, double *GBs)
{
    using lgf::fail;
    if (!GBs) return fail(LGF_EINVAL, "GBs is NULL");
    if (reps < 1) return fail(LGF_EINVAL, "reps must be >= 1");
    if (bytes < 16 || bytes % 16 != 0 || bytes / 16 / 256 >= 0x7fffffffull)
        return fail(LGF_EINVAL, "bytes must be a positive multiple of 16 below 8 TiB");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t n = bytes / 16;
    const dim3 grid((unsigned)((n + 255) / 256));
    lgf::v4f *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lgf_status st = LGF_OK;
    float ms = 0.f;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(LGF_ENOMEM, "cannot allocate 2 x %zu bytes for the copy", bytes);
    }
    hipError_t e = hipSuccess;
    if (st == LGF_OK) {
        hipLaunchKernelGGL(lgf::fill_kernel, grid, dim3(256), 0, s, a, n);
        hipLaunchKernelGGL(lgf::copy_kernel, grid, dim3(256), 0, s, a, b, n);  // warm-up
        if ((e = hipGetLastError()) == hipSuccess && (e = hipEventCreate(&e0)) == hipSuccess &&
            (e = hipEventCreate(&e1)) == hipSuccess && (e = hipEventRecord(e0, s)) == hipSuccess) {
            for (int r = 0; r < reps; ++r)
                hipLaunchKernelGGL(lgf::copy_kernel, grid, dim3(256), 0, s, (r & 1) ? b : a, (r & 1) ? a : b, n);
            if ((e = hipGetLastError()) == hipSuccess && (e = hipEventRecord(e1, s)) == hipSuccess &&
                (e = hipEventSynchronize(e1)) == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
        }
        if (e != hipSuccess) st = fail(LGF_EHIP, "copy bandwidth: %s", hipGetErrorString(e));
    }
    if (a) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (st != LGF_OK) return st;
    *GBs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return LGF_OK;
}
