// Transformed free-space kernel (the Green's-function spectrum), built once
// per plan in double precision on the GPU.
//
// The padded kernel K_pad[z][y][x] = K(min(x,P-x), min(y,P-y), min(z,P-z)),
// with K(d) = -1/(dx |(dx sx, dy sy, dz sz)|) for cells of spacings dx,
// dx sy, dx sz (sx = 1; all ratios 1 for cubes) and K(0) = the self value
// (-self_coeff/dx for cubes), is real and even along
// every axis, so its 3D DFT is real and even and one octant [0,Hx) x [0,Hy)
// x [0,Hz) (H = n + 1 per axis) holds all of it.  Evenness also means that
// only the rows with y < Hy, z < Hz need a transform along x, and so on per
// axis.  Three passes:
//
//   green_x  K generated on the fly for rows (z, y) in [0,Hz) x [0,Hy),
//            length-Px forward FFT along x, kx in [0,Hx) kept
//                                                    -> G1[kx][z][y]
//   green_y  pencils along y, even extension y -> min(y, P-y), in place
//                                                    -> G1[kx][z][ky]
//   green_z  pencils along z, even extension, scaled by G dV / P^3 and
//            rounded once to the plan's type        -> Ghat[kx][ky][kz]
//            (or Ghat[kz][ky][kx] for the plain method's layout)
//
// Two real, even pencils are packed as the real and imaginary parts of one
// complex FFT; the transform of each is real, so the real and imaginary parts
// of the output are the two results.
#pragma once
#include "plans.hpp"

namespace ps {

// Each kernel transforms one axis, of padded length P (template); the other
// axes' half lengths hx, hy, hz (n + 1 per axis) are arguments, so a box of
// nx x ny x nz cells builds with one kernel per axis length.
template <int P, int NT, int MAP_MID>
__global__ __launch_bounds__(NT) void k_green_x(double* __restrict__ g1, const double2* __restrict__ tw, int hy,
                                                int hz, double dx, double sy, double sz, double self_value)
{
    using V = double2;
    using E = Engine<double, typename PlanFor<P>::Fwd, 8, NT>;
    constexpr int N = P / 2, H = N + 1;
    __shared__ V lds[E::LDS_ELEMS];
    const int y0 = blockIdx.x * 16;
    const int z = blockIdx.y;
    auto kv = [&](int x, int y) -> double {
        if (y >= hy) return 0.0;
        const int ax = x <= N ? x : P - x;
        const double ry = double(y) * sy, rz = double(z) * sz;
        const double r2 = double(ax) * ax + ry * ry + rz * rz;
        return r2 == 0.0 ? self_value : -1.0 / (dx * sqrt(r2));
    };
    auto ld = [&](int p, int idx) -> V {
        const int ya = y0 + 2 * p;
        return V{kv(idx, ya), kv(idx, ya + 1)};
    };
    auto st = [&](int p, int idx, V v) {
        const int ya = y0 + 2 * p;
        double* row = g1 + ((size_t)idx * hz + z) * hy;  // G1[kx][z][y]
        if (ya < hy) row[ya] = v.x;
        if (ya + 1 < hy) row[ya + 1] = v.y;
    };
    E::template run<-1, MAP_EF, MAP_MID, MAP_PF, P, H>(lds, tw, ld, st);
}

template <int P, int NT, int MAP_MID>
__global__ __launch_bounds__(NT) void k_green_y(double* __restrict__ g1, const double2* __restrict__ tw, int hz)
{
    using V = double2;
    using E = Engine<double, typename PlanFor<P>::Fwd, 8, NT>;
    constexpr int N = P / 2, H = N + 1;
    __shared__ V lds[E::LDS_ELEMS];
    const int z0 = blockIdx.x * 16;
    const int kx = blockIdx.y;
    double* plane = g1 + (size_t)kx * hz * H;  // G1[kx][z][y], y < H
    auto ld = [&](int p, int idx) -> V {
        const int za = z0 + 2 * p;
        const int y = idx <= N ? idx : P - idx;
        const double a = za < hz ? plane[(size_t)za * H + y] : 0.0;
        const double b = za + 1 < hz ? plane[(size_t)(za + 1) * H + y] : 0.0;
        return V{a, b};
    };
    auto st = [&](int p, int idx, V v) {
        const int za = z0 + 2 * p;
        if (za < hz) plane[(size_t)za * H + idx] = v.x;
        if (za + 1 < hz) plane[(size_t)(za + 1) * H + idx] = v.y;
    };
    E::template run<-1, MAP_EF, MAP_MID, MAP_EF, P, H>(lds, tw, ld, st);
}

// PLAIN_LAYOUT: write Ghat[kz][ky][kx] instead of Ghat[kx][ky][kz].
template <typename TOUT, int P, int NT, int MAP_MID, bool PLAIN_LAYOUT>
__global__ __launch_bounds__(NT) void k_green_z(const double* __restrict__ g1, TOUT* __restrict__ ghat,
                                                const double2* __restrict__ tw, int hx, int hy, double scale)
{
    using V = double2;
    using E = Engine<double, typename PlanFor<P>::Fwd, 8, NT>;
    constexpr int N = P / 2, H = N + 1;
    __shared__ V lds[E::LDS_ELEMS];
    const int ky0 = blockIdx.x * 16;
    const int kx = blockIdx.y;
    const double* plane = g1 + (size_t)kx * H * hy;  // G1[kx][z][ky], z < H
    auto ld = [&](int p, int idx) -> V {
        const int ka = ky0 + 2 * p;
        const int z = idx <= N ? idx : P - idx;
        const double a = ka < hy ? plane[(size_t)z * hy + ka] : 0.0;
        const double b = ka + 1 < hy ? plane[(size_t)z * hy + ka + 1] : 0.0;
        return V{a, b};
    };
    auto st = [&](int p, int idx, V v) {
        const int ka = ky0 + 2 * p;
        if constexpr (PLAIN_LAYOUT) {
            if (ka < hy) ghat[((size_t)idx * hy + ka) * hx + kx] = TOUT(scale * v.x);
            if (ka + 1 < hy) ghat[((size_t)idx * hy + ka + 1) * hx + kx] = TOUT(scale * v.y);
        } else {
            if (ka < hy) ghat[((size_t)kx * hy + ka) * H + idx] = TOUT(scale * v.x);
            if (ka + 1 < hy) ghat[((size_t)kx * hy + ka + 1) * H + idx] = TOUT(scale * v.y);
        }
    };
    E::template run<-1, MAP_PF, MAP_MID, MAP_EF, P, H>(lds, tw, ld, st);
}

}  // namespace ps
