// The device buffers of one pruned solve, as the pass kernels read them from
// a device array indexed by grid z: a plan's own record for single solves, or
// the records of a group of equal-length solves (a batch).
#pragma once
#include <hip/hip_runtime.h>

// In device code the fields point into global memory; typing them so lets the
// compiler use global (not flat) loads and stores with scalar base addresses.
#if defined(__HIP_DEVICE_COMPILE__)
#define PS_GLOBAL __attribute__((address_space(1)))
#else
#define PS_GLOBAL
#endif

namespace ps {

struct SolveRec {
    const PS_GLOBAL void* rho;   // N^3 real
    PS_GLOBAL void* phi;         // N^3 real
    PS_GLOBAL void* t1;          // T1 [H][N][N] complex; later T4 [N][N][HP]
    PS_GLOBAL void* t2;          // T2 [H][P][N] complex
    PS_GLOBAL void* t3;          // T3 [H][N][P] complex
    const PS_GLOBAL void* ghat;  // [H][H][H] real octant, scaled
    const PS_GLOBAL void* twf;   // forward-plan twiddles, radix-16-based family
    const PS_GLOBAL void* twi;   // inverse-plan twiddles, radix-16-based family
    const PS_GLOBAL void* twf1;  // forward-plan twiddles, radix-32-based family (where it exists)
    const PS_GLOBAL void* twi1;  // inverse-plan twiddles, radix-32-based family
};

}  // namespace ps
