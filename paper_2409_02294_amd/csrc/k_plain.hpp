// The plain FFT-convolution method: every step materialised, nothing pruned.
//
//   pad     rho (N^3) -> R[z][y][x] (P^3 real, zeros outside [0,N)^3)
//   x_r2c   R rows -> S[z][y][kx]        (P x P x H complex, kx fastest, pitch H)
//   y fwd   S in place along y           (all P inputs, all P outputs)
//   z fwd   S in place along z
//   mul     S[kz][ky][kx] *= Ghat[min(kz,P-kz)][min(ky,P-ky)][kx]
//   z inv, y inv in place
//   x_c2r   S rows -> R[z][y][x]         (all P outputs)
//   crop    R -> phi (N^3)
//
// This is the textbook method with a standard half-spectrum layout; it uses
// the same LDS-staged, coalesced pencil engine as the pruned pipeline, so the
// difference between the two measures the pruning and fusion alone.
#pragma once
#include "plans.hpp"

namespace ps {

template <typename T> __global__ void k_plain_pad(const T* __restrict__ rho, T* __restrict__ pad, int N, int P)
{
    const size_t total = (size_t)P * P * P;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % P);
        const size_t r = i / P;
        const int y = (int)(r % P), z = (int)(r / P);
        pad[i] = (x < N && y < N && z < N) ? rho[((size_t)z * N + y) * N + x] : T(0);
    }
}

template <typename T> __global__ void k_plain_crop(const T* __restrict__ pad, T* __restrict__ phi, int N, int P)
{
    const size_t total = (size_t)N * N * N;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % N);
        const size_t r = i / N;
        const int y = (int)(r % N), z = (int)(r / N);
        phi[i] = pad[((size_t)z * P + y) * P + x];
    }
}

// S[kz][ky][kx] *= Ghat[kz'][ky'][kx], Ghat in [kz][ky][kx] layout (H^3).
template <typename T> __global__ void k_plain_mul(cx<T>* __restrict__ spec, const T* __restrict__ ghat, int P)
{
    const int H = P / 2 + 1;
    const size_t total = (size_t)P * P * H;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int kx = (int)(i % H);
        const size_t r = i / H;
        int ky = (int)(r % P), kz = (int)(r / P);
        ky = ky <= P / 2 ? ky : P - ky;
        kz = kz <= P / 2 ? kz : P - kz;
        const T g = ghat[((size_t)kz * H + ky) * H + kx];
        const cx<T> v = spec[i];
        spec[i] = cx<T>{v.x * g, v.y * g};
    }
}

// 16 rows (8 packed pairs) of one z-plane: real P-point FFT of each row.
template <typename T, int P, int NT>
__global__ __launch_bounds__(NT) void k_plain_x_r2c(const T* __restrict__ pad, cx<T>* __restrict__ spec,
                                                    const cx<T>* __restrict__ tw)
{
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P>::Fwd, 8, NT>;
    constexpr int H = P / 2 + 1;
    __shared__ V lds[E::LDS_ELEMS];
    const int y0 = blockIdx.x * 16;
    const int z = blockIdx.y;
    const T* plane = pad + (size_t)z * P * P;
    auto ld = [&](int p, int idx) -> V {
        const int ya = y0 + 2 * p;
        return V{plane[(size_t)ya * P + idx], plane[(size_t)(ya + 1) * P + idx]};
    };
    auto st = [&](int p, int idx, V v) { lds[E::lidx(p, idx)] = v; };
    E::template run<-1, MAP_EF, MAP_EF, MAP_EF, P, P, true>(lds, tw, ld, st);
    __syncthreads();
    V* out = spec + ((size_t)z * P + y0) * H;  // 16 consecutive rows of H
    for (int e = threadIdx.x; e < 16 * H; e += NT) {
        const int row = e / H, k = e - row * H;
        const int p = row >> 1;
        const V z1 = lds[E::lidx(p, k)];
        const V z2 = lds[E::lidx(p, k == 0 ? 0 : P - k)];
        V x;
        if (row & 1) x = V{T(0.5) * (z1.y + z2.y), T(-0.5) * (z1.x - z2.x)};
        else x = V{T(0.5) * (z1.x + z2.x), T(0.5) * (z1.y - z2.y)};
        out[e] = x;
    }
}

// W interleaved pencils (consecutive kx) along y (AXIS 1) or z (AXIS 2), in place.
template <typename T, int P, int W, int NT, int DIR, int AXIS>
__global__ __launch_bounds__(NT) void k_plain_yz(cx<T>* __restrict__ spec, const cx<T>* __restrict__ tw)
{
    using V = cx<T>;
    using RP = std::conditional_t<(DIR < 0), typename PlanFor<P>::Fwd, typename PlanFor<P>::Inv>;
    using E = Engine<T, RP, W, NT>;
    constexpr int H = P / 2 + 1;
    __shared__ V lds[E::LDS_ELEMS];
    const int kx0 = blockIdx.x * W;
    const int other = blockIdx.y;  // z for AXIS 1, y for AXIS 2
    const size_t stride = AXIS == 1 ? (size_t)H : (size_t)P * H;
    V* base = spec + (AXIS == 1 ? (size_t)other * P * H : (size_t)other * H) + kx0;
    auto ld = [&](int p, int idx) -> V { return kx0 + p < H ? base[idx * stride + p] : V{T(0), T(0)}; };
    auto st = [&](int p, int idx, V v) {
        if (kx0 + p < H) base[idx * stride + p] = v;
    };
    E::template run<DIR, MAP_PF, MAP_EF, MAP_PF, P, P>(lds, tw, ld, st);
}

// 16 rows (8 packed pairs) of one z-plane: inverse real FFT (all P outputs).
template <typename T, int P, int NT>
__global__ __launch_bounds__(NT) void k_plain_x_c2r(const cx<T>* __restrict__ spec, T* __restrict__ pad,
                                                    const cx<T>* __restrict__ tw)
{
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P>::Inv, 8, NT>;
    constexpr int N = P / 2, H = N + 1;
    constexpr int XP = H + 1;
    constexpr int LDS = E::LDS_ELEMS > 16 * XP ? E::LDS_ELEMS : 16 * XP;
    __shared__ V lds[LDS];
    const int y0 = blockIdx.x * 16;
    const int z = blockIdx.y;
    const V* in = spec + ((size_t)z * P + y0) * H;
    for (int e = threadIdx.x; e < 16 * H; e += NT) {
        const int row = e / H, k = e - row * H;
        lds[row * XP + k] = in[e];
    }
    __syncthreads();
    auto ld = [&](int p, int idx) -> V {
        const V* xa = lds + (2 * p) * XP;
        const V* xb = xa + XP;
        V a, b;
        if (idx <= N) {
            a = xa[idx];
            b = xb[idx];
            if (idx == 0 || idx == N) {
                a.y = T(0);
                b.y = T(0);
            }
        } else {
            a = cconj(xa[P - idx]);
            b = cconj(xb[P - idx]);
        }
        return V{a.x - b.y, a.y + b.x};
    };
    T* plane = pad + (size_t)z * P * P;
    auto st = [&](int p, int idx, V v) {
        const int ya = y0 + 2 * p;
        plane[(size_t)ya * P + idx] = v.x;
        plane[(size_t)(ya + 1) * P + idx] = v.y;
    };
    E::template run<+1, MAP_EF, MAP_EF, MAP_EF, P, P>(lds, tw, ld, st);
}

}  // namespace ps
