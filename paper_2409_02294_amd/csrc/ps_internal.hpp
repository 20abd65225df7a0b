// Host-side internals shared by the ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ps.h"
#include "solve_rec.hpp"

namespace ps {

// Kernel variants of the pruned pipeline (chosen per plan, e.g. by the
// autotuner).  fam: radix-plan family (0: radix-16 based, 1: radix-32 based
// where P allows it, else 0); for the y passes bit 1 (value 2, 3) selects
// the persistent form with a one-tile prefetch.  zmode: 0 workgroup-synchronised z pass,
// 1 wave-owned pencils (family 0), 2 wave-owned pencils (family 1),
// 3 persistent wave-owned pencils with a one-tile prefetch (family 1 where
// it exists, else family 0; split plans: family 0), 4 the same on family 0
// with fewer pencils per wavefront (one at P = 1024).  Boxes take the
// one-tile-per-workgroup variants only (y: 0, 1; z: 0, 1, 2).  ztile: pencils
// per z-pass workgroup, 0 the full tile (16 float, 8 double: 128-byte output
// rows), 1 half of it (64-byte rows, half the LDS, twice the workgroups).
struct PrunedVariant {
    int x_fam = 0, y_fam = 0, zmode = 0, yi_fam = 0, xc_fam = 0;
    int mterms = 0;  // 0: vector-ALU DFTs; 3 or 6: split-bf16 matrix-core radix-16 DFTs (float only)
    int ztile = 0;
};
constexpr int NUM_ZMODES = 6;

// Launch arguments of the pruned pipeline: `count` equal-length solves whose
// records are the device array `list` (grid z indexes it).  in[k] / out[k],
// when not NULL, replace pass k's input / output array of the record (a
// single solve's rho and phi, or the arrays of a debug pass).  Complex arrays
// are interleaved (re, im) of the plan's real type.
struct PrunedBufs {
    const SolveRec* list = nullptr;
    int count = 1;
    // padded length of each axis (x, y, z); box = false: a cube, every axis
    // of length px, run by the kernels built for cubes; box = true: the
    // kernels built for boxes, with the extents nx, ny, nz
    int px = 0, py = 0, pz = 0;
    bool box = false;
    int nx = 0, ny = 0, nz = 0;
    const void* in[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    void* out[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    const unsigned short* stab = nullptr;  // split-bf16 DFT-16 matrix pieces (mterms > 0)
    PrunedVariant var;
    hipStream_t stream = nullptr;
};

// Runs passes [lo, hi) of the pruned pipeline (0 x_r2c, 1 y_fwd, 2 z_conv,
// 3 y_inv, 4 x_c2r), each on its axis's padded length.  Returns
// hipErrorInvalidValue for an unsupported length or a variant boxes lack.
// Each arithmetic is compiled as two units, one per half of the lengths
// (is_short_p); pruned_run sends every pass to the half of its length.
constexpr bool is_short_p(int P) { return P <= 480; }
using PrunedRunFn = hipError_t (*)(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_f32_short(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_f32_long(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_f64_short(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_f64_long(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_split6_short(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_split6_long(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_split3_short(int lo, int hi, const PrunedBufs& b);
hipError_t pruned_run_split3_long(int lo, int hi, const PrunedBufs& b);
inline hipError_t pruned_run(PrunedRunFn fshort, PrunedRunFn flong, int lo, int hi, const PrunedBufs& b)
{
    if (!b.box) return (is_short_p(b.px) ? fshort : flong)(lo, hi, b);
    for (int pass = lo; pass < hi; ++pass) {
        const int P = pass == 2 ? b.pz : (pass == 1 || pass == 3) ? b.py : b.px;
        const hipError_t e = (is_short_p(P) ? fshort : flong)(pass, pass + 1, b);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
inline hipError_t pruned_run_f32(int lo, int hi, const PrunedBufs& b)
{
    return pruned_run(pruned_run_f32_short, pruned_run_f32_long, lo, hi, b);
}
inline hipError_t pruned_run_f64(int lo, int hi, const PrunedBufs& b)
{
    return pruned_run(pruned_run_f64_short, pruned_run_f64_long, lo, hi, b);
}
inline hipError_t pruned_run_split6(int lo, int hi, const PrunedBufs& b)
{
    return pruned_run(pruned_run_split6_short, pruned_run_split6_long, lo, hi, b);
}
inline hipError_t pruned_run_split3(int lo, int hi, const PrunedBufs& b)
{
    return pruned_run(pruned_run_split3_short, pruned_run_split3_long, lo, hi, b);
}

// Transformed-kernel build (double precision throughout), on a box of
// nx x ny x nz cells (a cube when all three are equal).
struct GreenBufs {
    int nx, ny, nz;      // cells per axis; padded lengths 2 nx, 2 ny, 2 nz
    double* g1;          // [Hx][Hz][Hy] scratch
    void* ghat;          // output, float or double
    const void* twf64[3];  // forward-plan twiddles in double, per axis
    double dx;           // x spacing
    double sy, sz;       // y and z spacings over dx (1 for cubic cells)
    double self_value;   // K(0)
    double scale;        // G dV / P^3
    bool out_f32;
    bool plain_layout;   // [kz][ky][kx] instead of [kx][ky][kz]
    hipStream_t stream;
};
hipError_t green_run(const GreenBufs& b);

// The plain method: materialised padded grid and full half spectrum.
struct PlainBufs {
    const void* rho;   // N^3 real
    void* phi;         // N^3 real
    void* pad;         // P^3 real (padded density, later the padded potential)
    void* spec;        // [P][P][H] complex (kx fastest)
    const void* ghat;  // [H][H][H] real octant in [kz][ky][kx] layout
    const void* twf;
    const void* twi;
    hipStream_t stream;
};
hipError_t plain_run_f32(int P, const PlainBufs& b);
hipError_t plain_run_f64(int P, const PlainBufs& b);

// Device scratch of solves that allocate nothing (ps_solve_static): a
// file-scope device array of this many bytes per GPU, held until the process
// ends.  static_scratch() returns its device address on the current device
// (looked up once per device).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)128 << 20;
hipError_t static_scratch(void** out);

// Plain device copy of `bytes` (a multiple of 16; 16-byte aligned arrays).
hipError_t stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

// Radix plans (forward; the inverse is the reverse) for a supported P and
// plan family; family 1 falls back to family 0 where it does not exist.
bool host_radices(int P, std::vector<int>& fwd, int fam = 0);
bool has_family1(int P);

}  // namespace ps
