// The pruned, fused FFT-convolution pipeline for one N^3 solve (P = 2N,
// H = N + 1), in five passes:
//
//   x_r2c   rho[z][y][x]  (N^3 real)      -> T1[kx][z][y]  (H x N x N complex)
//   y_fwd   T1[kx][z][y]                  -> T2[kx][ky][z] (H x P x N complex)
//   z_conv  T2[kx][ky][z] -> forward z FFT -> * Ghat -> inverse z FFT -> T2 (in place)
//   y_inv   T2[kx][ky][z]                 -> T1[kx][z][y]  (inverse along y, y < N kept)
//   x_c2r   T1[kx][z][y]                  -> phi[z][y][x]  (inverse real FFT, x < N kept)
//
// The zero padding to P is never stored: the first stage of every forward
// transform treats inputs >= N as zeros, and the last stage of every inverse
// transform produces only outputs < N (the crop).  Each intermediate is laid
// out so that one pass reads whole contiguous pencils and the next reads
// 16-pencil tiles (128 bytes per row in FP32) of interleaved pencils.
//
// Real transforms along x pack two density rows into one complex pencil
// (row a + i row b); the two half spectra separate by Hermitian symmetry,
// A[k] = (Z[k] + conj Z[-k]) / 2 and B[k] = (Z[k] - conj Z[-k]) / (2i).  The
// inverse packs A + i B with the Hermitian extension X[P-k] = conj X[k] and
// reads the two real rows off the real and imaginary parts.
//
// Ghat is the real octant [kx][ky'][kz'] (H^3, ky' = min(ky, P-ky),
// kz' = min(kz, P-kz)) of the transformed kernel, already scaled by
// G dx^3 / P^3, so the pipeline itself applies no normalisation.
#pragma once
#include "plans.hpp"

namespace ps {

// Ordering of the P ky pencils for the z pass: ky 0 and N first, then the
// pairs (i, P - i) next to each other so that a workgroup holding both reads
// their shared Ghat row once.
__device__ __forceinline__ int z_pencil_ky(int q, int N)
{
    if (q < 2) return q == 0 ? 0 : N;
    const int i = q >> 1;
    return (q & 1) ? 2 * N - i : i;
}

// ---------------------------------------------------------------------------
// x_r2c: 16 rows (8 packed pairs) of one z-plane per workgroup.
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int NT, int MAP_MID>
__global__ __launch_bounds__(NT) void k_x_r2c(const T* __restrict__ rho, cx<T>* __restrict__ t1,
                                              const cx<T>* __restrict__ tw)
{
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P, FAM>::Fwd, 8, NT>;
    constexpr int N = P / 2, H = N + 1;
    __shared__ V lds[E::LDS_ELEMS];
    const int y0 = blockIdx.x * 16;
    const int z = blockIdx.y;
    const T* plane = rho + (size_t)z * N * N;
    auto ld = [&](int p, int idx) -> V {
        const int ya = y0 + 2 * p;
        const T a = ya < N ? plane[(size_t)ya * N + idx] : T(0);
        const T b = ya + 1 < N ? plane[(size_t)(ya + 1) * N + idx] : T(0);
        return V{a, b};
    };
    auto st = [&](int p, int idx, V v) { lds[E::lidx(p, idx)] = v; };
    E::template run<-1, MAP_EF, MAP_MID, MAP_EF, N, P, true>(lds, tw, ld, st);
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * H; e += NT) {
        const int row = e & 15, k = e >> 4;
        const int y = y0 + row;
        if (y >= N) continue;
        const int p = row >> 1;
        const V z1 = lds[E::lidx(p, k)];
        const V z2 = lds[E::lidx(p, k == 0 ? 0 : P - k)];
        V x;
        if (row & 1) {
            x = V{T(0.5) * (z1.y + z2.y), T(-0.5) * (z1.x - z2.x)};
        } else {
            x = V{T(0.5) * (z1.x + z2.x), T(0.5) * (z1.y - z2.y)};
        }
        t1[((size_t)k * N + z) * N + y] = x;
    }
}

// ---------------------------------------------------------------------------
// y_fwd: ZT z-pencils of one kx per workgroup.
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int ZT, int NT, int MAP_MID>
__global__ __launch_bounds__(NT) void k_y_fwd(const cx<T>* __restrict__ t1, cx<T>* __restrict__ t2,
                                              const cx<T>* __restrict__ tw)
{
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P, FAM>::Fwd, ZT, NT>;
    constexpr int N = P / 2;
    __shared__ V lds[E::LDS_ELEMS];
    const int z0 = blockIdx.x * ZT;
    const int kx = blockIdx.y;
    const V* in = t1 + (size_t)kx * N * N;
    V* out = t2 + (size_t)kx * P * N;
    auto ld = [&](int p, int idx) -> V {
        return z0 + p < N ? in[(size_t)(z0 + p) * N + idx] : V{T(0), T(0)};
    };
    auto st = [&](int p, int idx, V v) {
        if (z0 + p < N) out[(size_t)idx * N + z0 + p] = v;
    };
    E::template run<-1, MAP_EF, MAP_MID, MAP_PF, N, P>(lds, tw, ld, st);
}

// ---------------------------------------------------------------------------
// z_conv: B z-pencils (ky pencils of one kx) per workgroup, in place.
// WAVE: each wavefront owns its pencils for the whole transform and the stage
// exchanges synchronise the wavefront only.
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int B, int NT, bool WAVE>
__global__ __launch_bounds__(NT) void k_z_conv(cx<T>* __restrict__ t2, const T* __restrict__ ghat,
                                               const cx<T>* __restrict__ twf, const cx<T>* __restrict__ twi)
{
    using V = cx<T>;
    using EF = Engine<T, typename PlanFor<P, FAM>::Fwd, B, NT, WAVE>;
    using EI = Engine<T, typename PlanFor<P, FAM>::Inv, B, NT, WAVE>;
    constexpr int MAP_IO = WAVE ? MAP_WV : MAP_EF;
    constexpr int MAP_MID = MAP_IO, MAP_Z = MAP_IO;
    static_assert(EF::LDS_ELEMS == EI::LDS_ELEMS, "plans share one LDS buffer");
    constexpr int N = P / 2, H = N + 1;
    constexpr int SL = EF::S - 1;
    __shared__ V lds[EF::LDS_ELEMS];
    const int q0 = blockIdx.x * B;
    const int kx = blockIdx.y;
    V* base = t2 + (size_t)kx * P * N;
    auto ld = [&](int p, int idx) -> V { return base[(size_t)z_pencil_ky(q0 + p, N) * N + idx]; };
    typename EF::template Regs<SL> g;
    EF::template run_to_regs<-1, MAP_IO, MAP_MID, MAP_Z, N>(lds, twf, ld, g);
    // multiply by the real, even transformed kernel at (kz, ky, kx)
    {
        constexpr int R = EF::template R<SL>;
        constexpr int Q = P / R;
        const T* grow = ghat + (size_t)kx * H * H;
#pragma unroll
        for (int i = 0; i < EF::template NB<SL>; ++i) {
            const int b = threadIdx.x + i * NT;
            if (!EF::template valid<SL, MAP_Z>(b)) continue;
            int p, j;
            EF::template pj<SL, MAP_Z>(b, p, j);
            const int ky = z_pencil_ky(q0 + p, N);
            const int kyf = ky <= N ? ky : P - ky;
            const T* gr = grow + (size_t)kyf * H;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int kz = j + r * Q;
                const T gv = gr[kz <= N ? kz : P - kz];
                g.v[i][r] = V{g.v[i][r].x * gv, g.v[i][r].y * gv};
            }
        }
    }
    auto st = [&](int p, int idx, V v) { base[(size_t)z_pencil_ky(q0 + p, N) * N + idx] = v; };
    EI::template run_from_regs<+1, MAP_Z, MAP_MID, MAP_IO, N>(lds, twi, g, st);
}

// ---------------------------------------------------------------------------
// y_inv: ZT z-pencils of one kx per workgroup.
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int ZT, int NT, int MAP_MID>
__global__ __launch_bounds__(NT) void k_y_inv(const cx<T>* __restrict__ t2, cx<T>* __restrict__ t1,
                                              const cx<T>* __restrict__ tw)
{
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P, FAM>::Inv, ZT, NT>;
    constexpr int N = P / 2;
    __shared__ V lds[E::LDS_ELEMS];
    const int z0 = blockIdx.x * ZT;
    const int kx = blockIdx.y;
    const V* in = t2 + (size_t)kx * P * N;
    V* out = t1 + (size_t)kx * N * N;
    auto ld = [&](int p, int idx) -> V {
        return z0 + p < N ? in[(size_t)idx * N + z0 + p] : V{T(0), T(0)};
    };
    auto st = [&](int p, int idx, V v) {
        if (z0 + p < N) out[(size_t)(z0 + p) * N + idx] = v;
    };
    E::template run<+1, MAP_PF, MAP_MID, MAP_EF, P, N>(lds, tw, ld, st);
}

// ---------------------------------------------------------------------------
// x_c2r: 16 rows (8 packed pairs) of one z-plane per workgroup.
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int NT, int MAP_MID>
__global__ __launch_bounds__(NT) void k_x_c2r(const cx<T>* __restrict__ t1, T* __restrict__ phi,
                                              const cx<T>* __restrict__ tw)
{
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P, FAM>::Inv, 8, NT>;
    constexpr int N = P / 2, H = N + 1;
    constexpr int XP = H + 1;  // pitch of the staged half spectra
    constexpr int LDS = E::LDS_ELEMS > 16 * XP ? E::LDS_ELEMS : 16 * XP;
    __shared__ V lds[LDS];
    const int y0 = blockIdx.x * 16;
    const int z = blockIdx.y;
    for (int e = threadIdx.x; e < 16 * H; e += NT) {
        const int row = e & 15, k = e >> 4;
        const int y = y0 + row;
        lds[row * XP + k] = y < N ? t1[((size_t)k * N + z) * N + y] : V{T(0), T(0)};
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
    T* plane = phi + (size_t)z * N * N;
    auto st = [&](int p, int idx, V v) {
        const int ya = y0 + 2 * p;
        if (ya < N) plane[(size_t)ya * N + idx] = v.x;
        if (ya + 1 < N) plane[(size_t)(ya + 1) * N + idx] = v.y;
    };
    E::template run<+1, MAP_EF, MAP_MID, MAP_EF, P, N>(lds, tw, ld, st);
}

}  // namespace ps
