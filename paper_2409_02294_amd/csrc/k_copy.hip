// Plain streaming device copy: the achievable-bandwidth reference against
// which the pass kernels' HBM rates are read.  Each thread copies COPY_U
// 16-byte items of a workgroup's contiguous chunk (lanes adjacent).  On
// MI355X one item per thread in 256-thread workgroups measured fastest at
// 1-4 GiB (about 6.2 TB/s read + write), ahead of 4 to 16 items per thread
// (5.2-5.9 TB/s) and of grid-stride loops (4.6-5.3 TB/s).
#include <hip/hip_runtime.h>

#include "ps_internal.hpp"

namespace ps {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int COPY_NT = 256;
constexpr int COPY_U = 1;

// Whole chunks of COPY_NT * COPY_U items, no bounds checks (a conditional
// load into an array element makes the compiler spill the whole array).
__global__ __launch_bounds__(COPY_NT) void k_stream_copy(const f4* __restrict__ src, f4* __restrict__ dst)
{
    const size_t base = (size_t)blockIdx.x * (COPY_NT * COPY_U) + threadIdx.x;
    f4 t[COPY_U];
#pragma unroll
    for (int u = 0; u < COPY_U; ++u) t[u] = src[base + (size_t)u * COPY_NT];
#pragma unroll
    for (int u = 0; u < COPY_U; ++u) dst[base + (size_t)u * COPY_NT] = t[u];
}

// The last partial chunk, one item per thread.
__global__ __launch_bounds__(COPY_NT) void k_stream_copy_tail(const f4* __restrict__ src, f4* __restrict__ dst,
                                                              size_t begin, size_t n)
{
    const size_t i = begin + (size_t)blockIdx.x * COPY_NT + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

hipError_t stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream)
{
    const size_t n = bytes / 16;
    const size_t per = (size_t)COPY_NT * COPY_U;
    const size_t full = n / per;
    if (full > 0x7fffffff) return hipErrorInvalidValue;
    const f4* a = static_cast<const f4*>(src);
    f4* b = static_cast<f4*>(dst);
    if (full) hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)full), dim3(COPY_NT), 0, stream, a, b);
    const size_t rest = n - full * per;
    if (rest)
        hipLaunchKernelGGL(k_stream_copy_tail, dim3((unsigned)((rest + COPY_NT - 1) / COPY_NT)), dim3(COPY_NT), 0,
                           stream, a, b, full * per, n);
    return hipGetLastError();
}

}  // namespace ps
