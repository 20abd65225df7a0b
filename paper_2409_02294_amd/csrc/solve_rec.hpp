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

// Twiddle tables are per axis (x, y, z: index 0, 1, 2); a cubic solve points
// all three at one set.  nx, ny, nz are the box's cell counts, read by the
// kernels built for boxes (a cubic kernel uses its compile-time length).
struct SolveRec {
    const PS_GLOBAL void* rho;      // nz x ny x nx real
    PS_GLOBAL void* phi;            // nz x ny x nx real
    PS_GLOBAL void* t1;             // T1 [Hx][nz][ny] complex; later T4 [nz][ny][HPx]
    PS_GLOBAL void* t2;             // T2 [Hx][Py][nz] complex
    PS_GLOBAL void* t3;             // T3 [Hx][nz][Py] complex
    const PS_GLOBAL void* ghat;     // [Hx][Hy][Hz] real octant, scaled
    const PS_GLOBAL void* twf[3];   // forward-plan twiddles per axis, radix-16-based family
    const PS_GLOBAL void* twi[3];   // inverse-plan twiddles per axis, radix-16-based family
    const PS_GLOBAL void* twf1[3];  // forward-plan twiddles per axis, radix-32-based family (where it exists)
    const PS_GLOBAL void* twi1[3];  // inverse-plan twiddles per axis, radix-32-based family
    int nx, ny, nz, pad_;
};

}  // namespace ps
