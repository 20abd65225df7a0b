// Device-resident work-list records of a persistent batched launch, shared by
// the host (which builds and uploads them) and the kernel.
#pragma once
#include <hip/hip_runtime.h>

namespace ps {

struct BatchSolve {
    const void* rho;
    void* phi;
    void* t1;
    void* t2;
    void* t3;
    const void* ghat;
    const void* twf;
    const void* twi;
    int P;
    int ntile[5];
};

struct BatchCtl {
    unsigned next;    // work-item dispenser
    unsigned error;   // set when a dependency wait reached the spin limit
    int nsolves;
    int total;        // number of items
    int pass_begin[6];
    int pad[6];
};

// Tile grid of each pass for a padded length P (used by host and device).
__host__ __device__ constexpr int batch_zt(int real_bytes) { return real_bytes == 4 ? 16 : 8; }
__host__ __device__ inline void batch_tiles(int P, int real_bytes, int out[5])
{
    const int N = P / 2, H = N + 1, ZT = batch_zt(real_bytes);
    out[0] = ((N + 15) / 16) * N;
    out[1] = ((N + ZT - 1) / ZT) * H;
    out[2] = (P / ZT) * H;
    out[3] = ((H + ZT - 1) / ZT) * N;
    out[4] = ((N + 15) / 16) * N;
}

}  // namespace ps
