// The pruned, fused FFT-convolution pipeline for one N^3 solve (P = 2N,
// H = N + 1), in five passes:
//
//   x_r2c   rho[z][y][x]  (N^3 real)      -> T1[kx][z][y]  (H x N x N complex)
//   y_fwd   T1[kx][z][y]                  -> T2[kx][ky][z] (H x P x N complex)
//   z_conv  T2[kx][ky][z] -> forward z FFT -> * Ghat -> inverse z FFT
//                                         -> T3[kx][z][ky] (H x N x P complex)
//   y_inv   T3[kx][z][ky]                 -> T4[z][y][kx]  (N x N x HP complex, inverse
//                                            along y, y < N kept; row pitch HP = H rounded
//                                            up to 16)
//   x_c2r   T4[z][y][kx]                  -> phi[z][y][x]  (inverse real FFT, x < N kept)
//
// The zero padding to P is never stored: the first stage of every forward
// transform treats inputs >= N as zeros, and the last stage of every inverse
// transform produces only outputs < N (the crop).  Every pass reads whole
// contiguous pencils (x_c2r: whole rows of T4) and writes its output as rows
// of 16 interleaved pencils (128 bytes in FP32, 8 pencils in FP64), the
// access pattern HBM serves best in both directions on MI355X; x_c2r writes
// the cropped real rows of phi directly.
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
#include <type_traits>

#include "plans.hpp"
#include "solve_rec.hpp"

namespace ps {

// Row pitch (complex elements) of T4: H rounded up to 16 so that the rows of
// interleaved pencils written by y_inv start 128-byte aligned.
__host__ __device__ constexpr int t4_pitch(int H) { return (H + 15) / 16 * 16; }

// Each pass is a tile function (one workgroup's share, addressed by tile
// coordinates, using a caller-provided LDS buffer of at least LDS elements),
// wrapped below as a one-tile-per-workgroup kernel; the y and z passes also
// have persistent kernels that walk the tiles with a one-tile prefetch.
//
// Boxes.  A pass transforms one axis, whose length is the template P; with
// BOX the extents of the other two axes come from the solve record (nx, ny,
// nz cells; H = n + 1 and padded lengths 2n per axis), so one kernel per
// axis length serves every box shape.  Without BOX all three axes have
// length P / 2 at compile time.
template <bool BOX> __device__ __forceinline__ int ext(int box_value, int cubic_value)
{
    if constexpr (BOX) return box_value;
    else return cubic_value;
}

// Element-wise copy of COUNT items src(e) -> dst(e, v) by the NT threads of a
// workgroup, each thread issuing all its loads before its stores, so a tile
// waits one memory latency rather than one per element it stages.
template <typename V, int NT, int COUNT, class SRC, class DST>
__device__ __forceinline__ void block_copy(SRC&& src, DST&& dst)
{
    constexpr int K = (COUNT + NT - 1) / NT;
    V tmp[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = (int)threadIdx.x + i * NT;
        if (COUNT % NT == 0 || e < COUNT) tmp[i] = src(e);
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = (int)threadIdx.x + i * NT;
        if (COUNT % NT == 0 || e < COUNT) dst(e, tmp[i]);
    }
}

// ---------------------------------------------------------------------------
// x_r2c: ROWS rows (ROWS/2 packed pairs) of one z-plane; tile (y-tile bx, z by).
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int NT, int MAP_MID, int MT, bool BOX = false, int ROWS = 16> struct TileXR2C {
    using V = cx<T>;
    static_assert(ROWS == 8 || ROWS == 16 || ROWS == 32, "rows per x tile");
    using E = Engine<T, typename PlanFor<P, FAM>::Fwd, ROWS / 2, NT, false, MT>;
    static constexpr int N = P / 2, H = N + 1;  // x length, half spectrum
    static constexpr int LDS = E::LDS_ELEMS;
    __device__ __forceinline__ static void run(int bx, int by, const T* __restrict__ rho, V* __restrict__ t1,
                                               const V* __restrict__ tw, V* lds, const typename E::SA& sa,
                                               int ny_box = 0, int nz_box = 0)
    {
        const int Ny = ext<BOX>(ny_box, N), Nz = ext<BOX>(nz_box, N);
        const int y0 = bx * ROWS;
        const int z = by;
        const T* plane = rho + ((size_t)z * Ny + y0) * N;  // block-uniform base, 32-bit offsets below
        auto ld = [&](int p, int idx) -> V {
            const int ya = y0 + 2 * p;
            const T a = ya < Ny ? plane[(unsigned)(2 * p * N + idx)] : T(0);
            const T b = ya + 1 < Ny ? plane[(unsigned)((2 * p + 1) * N + idx)] : T(0);
            return V{a, b};
        };
        auto st = [&](int p, int idx, V v) { lds[E::lidx(p, idx)] = v; };
        E::template run<-1, MAP_EF, MAP_MID, MAP_EF, N, P, true>(lds, tw, ld, st, sa);
        __syncthreads();
        V* t1z = t1 + (size_t)z * Ny;
        // separate the two half spectra of each packed pair: element e is
        // (row e % ROWS, k = e / ROWS), written to T1[k][z][y0 + row]
        auto sep = [&](int e) -> V {
            const int row = (int)((unsigned)e % ROWS), k = (int)((unsigned)e / ROWS);
            const int p = row >> 1;
            const V z1 = lds[E::lidx(p, k)];
            const V z2 = lds[E::lidx(p, k == 0 ? 0 : P - k)];
            if (row & 1) return V{T(0.5) * (z1.y + z2.y), T(-0.5) * (z1.x - z2.x)};
            return V{T(0.5) * (z1.x + z2.x), T(0.5) * (z1.y - z2.y)};
        };
        auto put = [&](int e, V x) {
            const int row = (int)((unsigned)e % ROWS), k = (int)((unsigned)e / ROWS);
            if (y0 + row < Ny) t1z[(unsigned)(k * Nz * Ny + y0 + row)] = x;
        };
        block_copy<V, NT, ROWS * H>(sep, put);
    }
};

// Wavefronts per SIMD for two resident workgroups of NT threads: the register
// budget the half-LDS forms are compiled to, so that the halved LDS rows do
// let a second workgroup onto the compute unit.
constexpr int half_waves_per_simd(int NT) { return NT / 128 > 1 ? NT / 128 : 1; }

// ---------------------------------------------------------------------------
// y_fwd: ZT z-pencils of one kx; tile (z-tile bx, kx by).
// ---------------------------------------------------------------------------
// HALF: stage exchanges through half the LDS in two rounds (twice the
// workgroups resident per compute unit, the same 128-byte output rows).
template <typename T, int P, int FAM, int ZT, int NT, int MAP_MID, int MT, bool BOX = false, bool HALF = false>
struct TileYFwd {
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P, FAM>::Fwd, ZT, NT, false, MT>;
    static constexpr int N = P / 2;  // y length
    static constexpr int LDS = HALF ? ZT * E::half_pitch() : E::LDS_ELEMS;
    __device__ __forceinline__ static void run(int bx, int by, const V* __restrict__ t1, V* __restrict__ t2,
                                               const V* __restrict__ tw, V* lds, const typename E::SA& sa,
                                               int nz_box = 0)
    {
        const int Nz = ext<BOX>(nz_box, N);
        const int z0 = bx * ZT;
        const int kx = by;
        const V* in = t1 + ((size_t)kx * Nz + z0) * N;
        V* out = t2 + (size_t)kx * P * Nz + z0;
        auto ld = [&](int p, int idx) -> V {
            return z0 + p < Nz ? in[(unsigned)(p * N + idx)] : V{T(0), T(0)};
        };
        auto st = [&](int p, int idx, V v) {
            if (z0 + p < Nz) out[(unsigned)(idx * Nz + p)] = v;
        };
        if constexpr (HALF) E::template run_half<-1, MAP_EF, MAP_PF, N, P, E::half_pitch()>(lds, tw, ld, st, sa);
        else E::template run<-1, MAP_EF, MAP_MID, MAP_PF, N, P>(lds, tw, ld, st, sa);
    }
};

// ---------------------------------------------------------------------------
// z_conv: B consecutive ky pencils of one kx; tile (ky-tile bx, kx by).
// WAVE: each wavefront owns its pencils through every stage but the last,
// and those stage exchanges synchronise the wavefront only; the last stage
// spans the workgroup so its stores form rows of B interleaved pencils.
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int B, int NT, bool WAVE, int MT, bool BOX = false> struct TileZConv {
    using V = cx<T>;
    // the two plans share one LDS buffer with one row pitch (their pad
    // granularities may differ), so a wavefront's pencils sit in the same rows
    static constexpr int LPF = pad_pitch(P, 1 << pad_shift(PlanFor<P, FAM>::Fwd::r[0]), (int)sizeof(V));
    static constexpr int LPI = pad_pitch(P, 1 << pad_shift(PlanFor<P, FAM>::Inv::r[0]), (int)sizeof(V));
    static constexpr int LPZ = LPF > LPI ? LPF : LPI;
    using EF = Engine<T, typename PlanFor<P, FAM>::Fwd, B, NT, WAVE, MT, LPZ>;
    using EI = Engine<T, typename PlanFor<P, FAM>::Inv, B, NT, WAVE, MT, LPZ>;
    static constexpr int N = P / 2, H = N + 1;  // z length, z half spectrum
    static constexpr int LDS = EF::LDS_ELEMS;
    static_assert(EF::LDS_ELEMS == EI::LDS_ELEMS, "plans share one LDS buffer");
    __device__ __forceinline__ static void run(int bx, int by, const V* __restrict__ t2, V* __restrict__ t3,
                                               const T* __restrict__ ghat, const V* __restrict__ twf,
                                               const V* __restrict__ twi, V* lds, const typename EF::SA& sa,
                                               int ny_box = 0)
    {
        constexpr int MAP_IO = WAVE ? MAP_WV : MAP_EF;
        constexpr int SL = EF::S - 1;
        const int Ny = ext<BOX>(ny_box, N), Py = 2 * Ny, Hy = Ny + 1;
        const int ky0 = bx * B;
        const int kx = by;
        const V* in = t2 + ((size_t)kx * Py + ky0) * N;  // pencil p at in + p N
        V* out = t3 + (size_t)kx * N * Py + ky0;         // element (z, p) at out[z Py + p]
        const T* grow = ghat + (size_t)kx * Hy * H;
        auto ld = [&](int p, int idx) -> V { return in[(unsigned)(p * N + idx)]; };
        typename EF::template Regs<SL> g;
        EF::template run_to_regs<-1, MAP_IO, MAP_IO, MAP_IO, N>(lds, twf, ld, g, sa);
        // multiply by the real, even transformed kernel at (kz, ky, kx)
        auto mul = [&](int p, int kz, V& v) {
            const int ky = ky0 + p;
            const T* gr = grow + (unsigned)((ky <= Ny ? ky : Py - ky) * H);
            const T gv = gr[kz <= N ? kz : P - kz];
            v = V{v.x * gv, v.y * gv};
        };
        EF::template for_each_out<SL, MAP_IO>(g, mul);
        auto st = [&](int p, int idx, V v) { out[(unsigned)(idx * Py + p)] = v; };
        EI::template run_from_regs<+1, MAP_IO, MAP_IO, MAP_PF, N>(lds, twi, g, st, sa);
    }
};

// ---------------------------------------------------------------------------
// y_inv: ZT consecutive kx pencils of one z; tile (kx-tile bx, z by).
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int ZT, int NT, int MAP_MID, int MT, bool BOX = false, bool HALF = false>
struct TileYInv {
    using V = cx<T>;
    using E = Engine<T, typename PlanFor<P, FAM>::Inv, ZT, NT, false, MT>;
    static constexpr int N = P / 2;  // y length
    static constexpr int LDS = HALF ? ZT * E::half_pitch() : E::LDS_ELEMS;
    __device__ __forceinline__ static void run(int bx, int by, const V* __restrict__ t3, V* __restrict__ t4,
                                               const V* __restrict__ tw, V* lds, const typename E::SA& sa,
                                               int nx_box = 0, int nz_box = 0)
    {
        const int Nz = ext<BOX>(nz_box, N), Hx = ext<BOX>(nx_box, N) + 1, HP = t4_pitch(Hx);
        const int kx0 = bx * ZT;
        const int z = by;
        const V* in = t3 + ((size_t)kx0 * Nz + z) * P;  // pencil p (kx0 + p) at in + p Nz P
        V* out = t4 + (size_t)z * N * HP + kx0;         // element (y, p) at out[y HP + p]
        auto ld = [&](int p, int idx) -> V {
            return kx0 + p < Hx ? in[(unsigned)(p * Nz * P + idx)] : V{T(0), T(0)};
        };
        auto st = [&](int p, int idx, V v) {
            if (kx0 + p < Hx) out[(unsigned)(idx * HP + p)] = v;
        };
        if constexpr (HALF) E::template run_half<+1, MAP_EF, MAP_PF, P, N, E::half_pitch()>(lds, tw, ld, st, sa);
        else E::template run<+1, MAP_EF, MAP_MID, MAP_PF, P, N>(lds, tw, ld, st, sa);
    }
};

// ---------------------------------------------------------------------------
// x_c2r: 16 rows (8 packed pairs) of one z-plane; tile (y-tile bx, z by).
// ---------------------------------------------------------------------------
template <typename T, int P, int FAM, int NT, int MAP_MID, int MT, bool BOX = false, int ROWS = 16> struct TileXC2R {
    using V = cx<T>;
    static_assert(ROWS == 8 || ROWS == 16 || ROWS == 32, "rows per x tile");
    using E = Engine<T, typename PlanFor<P, FAM>::Inv, ROWS / 2, NT, false, MT>;
    static constexpr int N = P / 2, H = N + 1, HP = t4_pitch(H);  // x length, half spectrum, T4 pitch
    static constexpr int XP = H + 1;  // pitch of the staged half spectra
    static constexpr int LDS = E::LDS_ELEMS > ROWS * XP ? E::LDS_ELEMS : ROWS * XP;
    __device__ __forceinline__ static void run(int bx, int by, const V* __restrict__ t4, T* __restrict__ phi,
                                               const V* __restrict__ tw, V* lds, const typename E::SA& sa,
                                               int ny_box = 0)
    {
        const int Ny = ext<BOX>(ny_box, N);
        const int y0 = bx * ROWS;
        const int z = by;
        const V* rows = t4 + ((size_t)z * Ny + y0) * HP;  // ROWS consecutive rows of H (pitch HP)
        block_copy<V, NT, ROWS * H>(
            [&](int e) -> V {
                const int row = e / H, k = e - row * H;
                return y0 + row < Ny ? rows[(unsigned)(row * HP + k)] : V{T(0), T(0)};
            },
            [&](int e, V v) {
                const int row = e / H, k = e - row * H;
                lds[row * XP + k] = v;
            });
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
        T* plane = phi + ((size_t)z * Ny + y0) * N;
        auto st = [&](int p, int idx, V v) {
            const int ya = y0 + 2 * p;
            if (ya < Ny) plane[(unsigned)(2 * p * N + idx)] = v.x;
            if (ya + 1 < Ny) plane[(unsigned)((2 * p + 1) * N + idx)] = v.y;
        };
        E::template run<+1, MAP_EF, MAP_MID, MAP_EF, P, N>(lds, tw, ld, st, sa);
    }
};

// ---------------------------------------------------------------------------
// One-tile-per-workgroup kernels.  Grid (x, y) are tile coordinates; grid z
// selects the solve's record in `list`.  A non-NULL `in` or `out` replaces the
// pass's input or output array of the record (a single solve's rho and phi).
// ---------------------------------------------------------------------------
template <typename X> __device__ __forceinline__ X* gp(const PS_GLOBAL void* p)
{
    return (X*)(const PS_GLOBAL X*)p;
}
template <typename X> __device__ __forceinline__ X* gp(PS_GLOBAL void* p)
{
    return (X*)(PS_GLOBAL X*)p;
}
// twiddle tables of axis AX (0 x, 1 y, 2 z) for plan family FAM
template <typename V, int FAM, int AX> __device__ __forceinline__ const V* tw_fwd(const SolveRec& s)
{
    return gp<const V>(FAM == 1 ? s.twf1[AX] : s.twf[AX]);
}
template <typename V, int FAM, int AX> __device__ __forceinline__ const V* tw_inv(const SolveRec& s)
{
    return gp<const V>(FAM == 1 ? s.twi1[AX] : s.twi[AX]);
}

template <typename T, int P, int FAM, int NT, int MAP_MID, int MT, bool BOX = false, int ROWS = 16>
__global__ __launch_bounds__(NT) void k_x_r2c(const T* in, cx<T>* out, const SolveRec* __restrict__ list,
                                              const unsigned short* __restrict__ stab)
{
    using TL = TileXR2C<T, P, FAM, NT, MAP_MID, MT, BOX, ROWS>;
    using V = cx<T>;
    __shared__ V lds[TL::LDS];
    typename TL::E::SA sa;
    sa.load(stab);
    const SolveRec& s = list[blockIdx.z];
    TL::run(blockIdx.x, blockIdx.y, in ? in : gp<const T>(s.rho), out ? out : gp<V>(s.t1), tw_fwd<V, FAM, 0>(s),
            lds, sa, ext<BOX>(s.ny, 0), ext<BOX>(s.nz, 0));
}

template <typename T, int P, int FAM, int ZT, int NT, int MAP_MID, int MT, bool BOX = false, bool HALF = false>
__global__ __launch_bounds__(NT, HALF ? half_waves_per_simd(NT) : 1) void k_y_fwd(const cx<T>* in, cx<T>* out, const SolveRec* __restrict__ list,
                                              const unsigned short* __restrict__ stab)
{
    using TL = TileYFwd<T, P, FAM, ZT, NT, MAP_MID, MT, BOX, HALF>;
    using V = cx<T>;
    __shared__ V lds[TL::LDS];
    typename TL::E::SA sa;
    sa.load(stab);
    const SolveRec& s = list[blockIdx.z];
    TL::run(blockIdx.x, blockIdx.y, in ? in : gp<const V>(s.t1), out ? out : gp<V>(s.t2), tw_fwd<V, FAM, 1>(s),
            lds, sa, ext<BOX>(s.nz, 0));
}

// z-pass tile order.  Pencils ky and P - ky multiply by the same Ghat rows,
// so tile t of a kx (NTILE tiles of B pencils) shares all but one of its
// rows with tile NTILE - 1 - t.  Workgroups go to the XCDs round-robin by
// linear index (here blockIdx.x mod 8, NTILE being a multiple of 8), so in
// launch order a tile and its mirror land on different XCDs and fetch the
// rows into two L2s.  Remapped, linear indices 16 g + x and 16 g + 8 + x
// (the same XCD, consecutive there) hold pair q = 8 g + x and its mirror.
template <int NTILE> __device__ __forceinline__ int z_tile(int l)
{
    if constexpr (NTILE % 16 != 0) {
        return l;
    } else {
        const int q = (l & 7) + 8 * (l >> 4);
        return (l & 8) ? NTILE - 1 - q : q;
    }
}

// (a box's tiles run in launch order: its ky extent is not known at compile time)
template <typename T, int P, int FAM, int B, int NT, bool WAVE, int MT, bool BOX = false>
__global__ __launch_bounds__(NT) void k_z_conv(const cx<T>* in, cx<T>* out, const SolveRec* __restrict__ list,
                                               const unsigned short* __restrict__ stab)
{
    using TL = TileZConv<T, P, FAM, B, NT, WAVE, MT, BOX>;
    using V = cx<T>;
    __shared__ V lds[TL::LDS];
    typename TL::EF::SA sa;
    sa.load(stab);
    const SolveRec& s = list[blockIdx.z];
    const int bx = BOX ? (int)blockIdx.x : z_tile<P / B>(blockIdx.x);
    TL::run(bx, blockIdx.y, in ? in : gp<const V>(s.t2), out ? out : gp<V>(s.t3), gp<const T>(s.ghat),
            tw_fwd<V, FAM, 2>(s), tw_inv<V, FAM, 2>(s), lds, sa, ext<BOX>(s.ny, 0));
}

// Fused z pass whose exchanges go through half the LDS in two rounds
// (wave-owned pencils, one tile per workgroup): a pencil holds a row of P/2
// instead of P, so twice as many pencils stay resident on a compute unit.
// On the two-stage plans (two or more pencils per wavefront) the rows of two
// workgroups fit where one did: FP64 holds 16 instead of 8 1024-point
// pencils per compute unit, FP32 32 instead of 16 (four wavefronts per SIMD
// instead of two).  The last inverse stage reads
// pencil-fastest, so the stores of the cropped output stay coalesced.
template <typename T, int P, int FAM, int B, int NT>
__global__ __launch_bounds__(NT) void k_z_conv_half(const cx<T>* in, cx<T>* out, const SolveRec* __restrict__ list,
                                                    const unsigned short* __restrict__ stab)
{
    using V = cx<T>;
    using EF = Engine<T, typename PlanFor<P, FAM>::Fwd, B, NT, true>;
    using EI = Engine<T, typename PlanFor<P, FAM>::Inv, B, NT, true>;
    constexpr int LPH = EF::half_pitch() > EI::half_pitch() ? EF::half_pitch() : EI::half_pitch();
    constexpr int N = P / 2, H = N + 1, SL = EF::S - 1;
    static_assert(EF::S > 1 && EI::S > 1, "two or more stages");
    __shared__ V lds[B * LPH];
    typename EF::SA sa;
    sa.load(stab);
    const SolveRec& s = list[blockIdx.z];
    const int ky0 = z_tile<P / B>(blockIdx.x) * B;
    const int kx = blockIdx.y;
    const V* pin = (in ? in : gp<const V>(s.t2)) + ((size_t)kx * P + ky0) * N;  // pencil p at pin + p N
    V* pout = (out ? out : gp<V>(s.t3)) + (size_t)kx * N * P + ky0;             // element (z, p) at pout[z P + p]
    const T* grow = gp<const T>(s.ghat) + (size_t)kx * H * H;
    auto ld = [&](int p, int idx) -> V { return pin[(unsigned)(p * N + idx)]; };
    typename EF::template Regs<0> g0;
    EF::template load_first<MAP_WV, N>(g0, ld);
    typename EF::template Regs<SL> g;
    EF::template stages_half<0, -1, MAP_WV, MAP_WV, MAP_WV, LPH>(g0, g, lds, typename EF::TW(tw_fwd<V, FAM, 2>(s)),
                                                                  sa);
    // multiply by the real, even transformed kernel at (kz, ky, kx)
    auto mul = [&](int p, int kz, V& v) {
        const int ky = ky0 + p;
        const T gv = grow[(unsigned)((ky <= N ? ky : P - ky) * H + (kz <= N ? kz : P - kz))];
        v = V{v.x * gv, v.y * gv};
    };
    EF::template for_each_out<SL, MAP_WV>(g, mul);
    typename EI::template Regs<EI::S - 1> h;
    EI::template stages_half<0, +1, MAP_WV, MAP_PF, MAP_WV, LPH>(g, h, lds, typename EI::TW(tw_inv<V, FAM, 2>(s)), sa);
    auto st = [&](int p, int idx, V v) { pout[(unsigned)(idx * P + p)] = v; };
    EI::template store_last<MAP_PF, N>(h, st);
}

// Persistent y passes with a one-tile prefetch: workgroups walk the tiles
// (same order as the one-tile-per-workgroup grid) and load the next tile's
// pencils before transforming the current ones.  Column twiddles (every
// stage but the last) are read from an LDS copy, since a global twiddle
// load would also wait for the prefetch.
template <typename V, class RP, int NT> __device__ __forceinline__ void copy_columns(const V* tab, V* dst)
{
    constexpr int C = RP::tw_size();
    const V* col = tab + C;  // columns follow the rows
    for (int e = threadIdx.x; e < C; e += NT) dst[e] = col[e];
}

template <typename T, int P, int FAM, int ZT, int NT, int MT>
__global__ __launch_bounds__(NT) void k_y_fwd_pf(const cx<T>* in, cx<T>* out, const SolveRec* __restrict__ list,
                                                 const unsigned short* __restrict__ stab, int count)
{
    using RP = typename PlanFor<P, FAM>::Fwd;
    using E = Engine<T, RP, ZT, NT, false, MT>;
    using V = cx<T>;
    constexpr int N = P / 2, H = N + 1, NZ = (N + ZT - 1) / ZT, C = RP::tw_size() > 0 ? RP::tw_size() : 1;
    __shared__ V lds[E::LDS_ELEMS];
    __shared__ V lcol[C];
    typename E::SA sa;
    sa.load(stab);
    const int total = NZ * H * count;
    int t = blockIdx.x;
    if (t >= total) return;
    copy_columns<V, RP, NT>(tw_fwd<V, FAM, 1>(list[0]), lcol);  // made visible by the first stage's barrier
    auto tile = [&](int u, int& zs, int& kx, int& z0) {
        zs = u / (NZ * H);
        const int r = u - zs * (NZ * H);
        kx = r / NZ;
        z0 = (r - kx * NZ) * ZT;
    };
    auto load = [&](int u, typename E::template Regs<0>& g) {
        int zs, kx, z0;
        tile(u, zs, kx, z0);
        const V* pin = (in ? in : gp<const V>(list[zs].t1)) + ((size_t)kx * N + z0) * N;
        auto ld = [&](int p, int idx) -> V { return z0 + p < N ? pin[(unsigned)(p * N + idx)] : V{T(0), T(0)}; };
        E::template load_first<MAP_EF, N>(g, ld);
    };
    typename E::template Regs<0> cur;
    load(t, cur);
    for (; t < total; t += gridDim.x) {
        typename E::template Regs<0> nxt;
        if (t + (int)gridDim.x < total) load(t + gridDim.x, nxt);
        int zs, kx, z0;
        tile(t, zs, kx, z0);
        const SolveRec& s = list[zs];
        V* pout = (out ? out : gp<V>(s.t2)) + (size_t)kx * P * N + z0;
        auto st = [&](int p, int idx, V v) {
            if (z0 + p < N) pout[(unsigned)(idx * N + p)] = v;
        };
        E::template run_from_regs<-1, MAP_EF, MAP_EF, MAP_PF, P>(lds, typename E::TW(tw_fwd<V, FAM, 1>(s), lcol), cur,
                                                                  st, sa);
        cur = nxt;
    }
}

template <typename T, int P, int FAM, int ZT, int NT, int MT>
__global__ __launch_bounds__(NT) void k_y_inv_pf(const cx<T>* in, cx<T>* out, const SolveRec* __restrict__ list,
                                                 const unsigned short* __restrict__ stab, int count)
{
    using RP = typename PlanFor<P, FAM>::Inv;
    using E = Engine<T, RP, ZT, NT, false, MT>;
    using V = cx<T>;
    constexpr int N = P / 2, H = N + 1, HP = t4_pitch(H), NK = (H + ZT - 1) / ZT;
    constexpr int C = RP::tw_size() > 0 ? RP::tw_size() : 1;
    __shared__ V lds[E::LDS_ELEMS];
    __shared__ V lcol[C];
    typename E::SA sa;
    sa.load(stab);
    const int total = NK * N * count;
    int t = blockIdx.x;
    if (t >= total) return;
    copy_columns<V, RP, NT>(tw_inv<V, FAM, 1>(list[0]), lcol);  // made visible by the first stage's barrier
    // z fastest: consecutive tiles read neighbouring rows of the same 16 kx planes
    auto tile = [&](int u, int& zs, int& kx0, int& z) {
        zs = u / (NK * N);
        const int r = u - zs * (NK * N);
        kx0 = (r / N) * ZT;
        z = r - (r / N) * N;
    };
    auto load = [&](int u, typename E::template Regs<0>& g) {
        int zs, kx0, z;
        tile(u, zs, kx0, z);
        const V* pin = (in ? in : gp<const V>(list[zs].t3)) + ((size_t)kx0 * N + z) * P;
        auto ld = [&](int p, int idx) -> V {
            return kx0 + p < H ? pin[(unsigned)(p * N * P + idx)] : V{T(0), T(0)};
        };
        E::template load_first<MAP_EF, P>(g, ld);
    };
    typename E::template Regs<0> cur;
    load(t, cur);
    for (; t < total; t += gridDim.x) {
        typename E::template Regs<0> nxt;
        if (t + (int)gridDim.x < total) load(t + gridDim.x, nxt);
        int zs, kx0, z;
        tile(t, zs, kx0, z);
        const SolveRec& s = list[zs];
        V* pout = (out ? out : gp<V>(s.t1)) + (size_t)z * N * HP + kx0;
        auto st = [&](int p, int idx, V v) {
            if (kx0 + p < H) pout[(unsigned)(idx * HP + p)] = v;
        };
        E::template run_from_regs<+1, MAP_EF, MAP_EF, MAP_PF, N>(lds, typename E::TW(tw_inv<V, FAM, 1>(s), lcol), cur,
                                                                  st, sa);
        cur = nxt;
    }
}

// z_conv, persistent, with a one-tile prefetch (wave-owned pencils).  Each
// workgroup walks tiles blockIdx.x, + gridDim.x, ... of all `count` solves
// (the grid is a multiple of 8, so the XCD pairing of z_tile holds).  Per
// tile it first issues the loads of the tile's kernel values, then those of
// the next tile's pencils, and only then transforms the current pencils, so
// memory latency overlaps arithmetic instead of stalling each tile's start.
// Vector loads complete in issue order, so a global twiddle load inside the
// transforms would also wait for the prefetch: the column twiddles (every
// stage but the last inverse one) are copied to LDS once per workgroup; the
// last inverse stage reads its row twiddles from global memory after the
// tile's arithmetic.
template <typename T, int P, int FAM, int B, int NT, int MT>
__global__ __launch_bounds__(NT) void k_z_conv_pf(const cx<T>* in, cx<T>* out, const SolveRec* __restrict__ list,
                                                  const unsigned short* __restrict__ stab, int count)
{
    using TL = TileZConv<T, P, FAM, B, NT, true, MT>;
    using EF = typename TL::EF;
    using EI = typename TL::EI;
    using V = cx<T>;
    using RF = typename PlanFor<P, FAM>::Fwd;
    using RI = typename PlanFor<P, FAM>::Inv;
    constexpr int N = P / 2, H = N + 1, NTILE = P / B, SL = EF::S - 1;
    constexpr bool SAME = std::is_same<RF, RI>::value;  // palindromic plan: one table serves both directions
    constexpr int CF = RF::tw_size(), CI = SAME ? 0 : RI::tw_size();
    __shared__ V lds[TL::LDS];
    __shared__ V lcol[CF + CI];
    typename EF::SA sa;
    sa.load(stab);
    const int total = NTILE * H * count;
    int t = blockIdx.x;
    if (t >= total) return;
    {
        // columns follow the rows in each table; one plan serves every record of a launch
        const V* cf = tw_fwd<V, FAM, 2>(list[0]) + CF;
        for (int e = threadIdx.x; e < CF; e += NT) lcol[e] = cf[e];
        if constexpr (!SAME) {
            const V* ci = tw_inv<V, FAM, 2>(list[0]) + RI::tw_size();
            for (int e = threadIdx.x; e < CI; e += NT) lcol[CF + e] = ci[e];
        }
        __syncthreads();
    }
    auto tile = [&](int u, int& zs, int& kx, int& ky0) {
        zs = u / (NTILE * H);
        const int r = u - zs * (NTILE * H);
        kx = r / NTILE;
        ky0 = z_tile<NTILE>(r - kx * NTILE) * B;
    };
    auto load = [&](int u, typename EF::template Regs<0>& g) {
        int zs, kx, ky0;
        tile(u, zs, kx, ky0);
        const V* pin = (in ? in : gp<const V>(list[zs].t2)) + ((size_t)kx * P + ky0) * N;
        auto ld = [&](int p, int idx) -> V { return pin[(unsigned)(p * N + idx)]; };
        EF::template load_first<MAP_WV, N>(g, ld);
    };
    typename EF::template Regs<0> cur;
    load(t, cur);
    for (; t < total; t += gridDim.x) {
        int zs, kx, ky0;
        tile(t, zs, kx, ky0);
        const SolveRec& s = list[zs];
        const T* grow = gp<const T>(s.ghat) + (size_t)kx * H * H;
        auto gk = [&](int p, int kz) -> T {
            const int ky = ky0 + p;
            return grow[(unsigned)((ky <= N ? ky : P - ky) * H + (kz <= N ? kz : P - kz))];
        };
        T gv[EF::template NB<SL>][EF::template RS<SL>];
        EF::template gather<SL, MAP_WV>(gv, gk);
        typename EF::template Regs<0> nxt;
        if (t + (int)gridDim.x < total) load(t + gridDim.x, nxt);
        typename EF::template Regs<SL> g;
        EF::template run_to_regs_loaded<-1, MAP_WV, MAP_WV, MAP_WV>(
            lds, typename EF::TW(tw_fwd<V, FAM, 2>(s), lcol), cur, g, sa);
        EF::template scale<SL>(g, gv);
        V* pout = (out ? out : gp<V>(s.t3)) + (size_t)kx * N * P + ky0;
        auto st = [&](int p, int idx, V v) { pout[(unsigned)(idx * P + p)] = v; };
        EI::template run_from_regs<+1, MAP_WV, MAP_WV, MAP_PF, N>(
            lds, typename EI::TW(tw_inv<V, FAM, 2>(s), SAME ? lcol : lcol + CF), g, st, sa);
        __syncthreads();  // the last stage read every pencil's rows; the next tile rewrites them
        cur = nxt;
    }
}

template <typename T, int P, int FAM, int ZT, int NT, int MAP_MID, int MT, bool BOX = false, bool HALF = false>
__global__ __launch_bounds__(NT, HALF ? half_waves_per_simd(NT) : 1) void k_y_inv(const cx<T>* in, cx<T>* out, const SolveRec* __restrict__ list,
                                              const unsigned short* __restrict__ stab)
{
    using TL = TileYInv<T, P, FAM, ZT, NT, MAP_MID, MT, BOX, HALF>;
    using V = cx<T>;
    __shared__ V lds[TL::LDS];
    typename TL::E::SA sa;
    sa.load(stab);
    const SolveRec& s = list[blockIdx.z];
    TL::run(blockIdx.x, blockIdx.y, in ? in : gp<const V>(s.t3), out ? out : gp<V>(s.t1), tw_inv<V, FAM, 1>(s),
            lds, sa, ext<BOX>(s.nx, 0), ext<BOX>(s.nz, 0));
}

template <typename T, int P, int FAM, int NT, int MAP_MID, int MT, bool BOX = false, int ROWS = 16>
__global__ __launch_bounds__(NT) void k_x_c2r(const cx<T>* in, T* out, const SolveRec* __restrict__ list,
                                              const unsigned short* __restrict__ stab)
{
    using TL = TileXC2R<T, P, FAM, NT, MAP_MID, MT, BOX, ROWS>;
    using V = cx<T>;
    __shared__ V lds[TL::LDS];
    typename TL::E::SA sa;
    sa.load(stab);
    const SolveRec& s = list[blockIdx.z];
    TL::run(blockIdx.x, blockIdx.y, in ? in : gp<const V>(s.t1), out ? out : gp<T>(s.phi), tw_inv<V, FAM, 0>(s),
            lds, sa, ext<BOX>(s.ny, 0));
}

}  // namespace ps
