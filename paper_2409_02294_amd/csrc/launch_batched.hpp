// Launch of the persistent batched kernel: counter reset, then one launch
// sized to the resident workgroup count.
#pragma once
#include "k_batched.hpp"
#include "ps_internal.hpp"

namespace ps {

template <typename T, int PMAX, int NT, int MT> hipError_t batched_launch(const BatchArgs& a)
{
    static int grid_cap = 0;  // resident workgroups for this instantiation
    if (grid_cap == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched<T, PMAX, NT, MT>, NT, 0);
        if (e != hipSuccess) return e;
        grid_cap = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    }
    const int nd = a.nsolves * 5;
    hipLaunchKernelGGL(k_batch_reset, dim3((nd + 255) / 256), dim3(256), 0, a.stream, a.ctl, a.done, nd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = a.total < grid_cap ? a.total : grid_cap;
    hipLaunchKernelGGL((k_batched<T, PMAX, NT, MT>), dim3(grid), dim3(NT), 0, a.stream, a.ctl, a.sol, a.prefix, a.done,
                       a.stab, a.spin_limit);
    return hipGetLastError();
}

}  // namespace ps
