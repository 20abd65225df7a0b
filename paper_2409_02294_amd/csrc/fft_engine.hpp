// Block-level pencil FFT engine for gfx950.
//
// A workgroup of NT threads transforms B pencils of length P = product of the
// radices in RP.  The algorithm is a self-sorting (Stockham) mixed-radix FFT:
// stage s with radix R and span NS = R_0 ... R_{s-1} takes, for every
// butterfly j in [0, P/R), the inputs at j + r P/R, multiplies input r by
// w^(r (j mod NS)) with w = exp(DIR 2 pi i / (NS R)), applies a length-R DFT in
// registers and writes output r to (j / NS) NS R + (j mod NS) + r NS.  After
// the last stage the data is in natural order.
//
// Stage 0 reads straight from a caller "loader" (global memory or LDS) and the
// last stage writes straight to a caller "storer", so the first and last
// passes over each pencil need no LDS round trip.  Inputs at index >= LIN are
// zero and outputs at index >= LOUT are not produced; with an even first
// radix and LIN = P/2 (zero padding) half of the first-stage inputs are
// compile-time zeros, and with an even last radix and LOUT = P/2 (cropping)
// half of the last-stage outputs are skipped.
//
// Between stages the pencils live in LDS, pencil p at row p with pitch LP and
// one pad slot every 16 elements (k -> k + k/16), which keeps both the
// stride-1 and the stride-R access patterns of the Stockham exchange free of
// systematic bank conflicts.
//
// Butterfly-to-thread mapping per stage: MAP_PF puts the pencil index in the
// fastest-varying position (lane-contiguous across pencils: coalesced access
// to arrays whose pencils are interleaved element by element), MAP_EF puts
// the butterfly index fastest (coalesced access to contiguous pencils), and
// MAP_WV gives each wavefront its own B / (NT/64) pencils with the butterfly
// index fastest across the wave's lanes.  When every stage of a transform uses
// MAP_WV no pencil is shared between wavefronts, and with WSYNC the stage
// exchanges synchronise the wavefront only, not the workgroup.
//
// Twiddles come from a per-plan table computed in double precision on the
// host and rounded once to T: for stage s >= 1 a row of R entries per
// residue m = j mod NS, entry r = exp(-2 pi i r m / (NS R)); the inverse
// direction uses the conjugate.
#pragma once
#include <type_traits>

#include "ps_complex.hpp"

namespace ps {

enum { MAP_PF = 0, MAP_EF = 1, MAP_WV = 2 };

template <int... Rs> struct Radices {
    static constexpr int S = sizeof...(Rs);
    static constexpr int r[S] = {Rs...};
    static constexpr int P = (1 * ... * Rs);
    static constexpr int ns(int s)
    {
        int v = 1;
        for (int i = 0; i < s; ++i) v *= r[i];
        return v;
    }
    // offset (complex entries) of stage s's twiddle rows
    static constexpr int tw_off(int s)
    {
        int o = 0;
        for (int i = 1; i < s; ++i) o += ns(i) * r[i];
        return o;
    }
    static constexpr int tw_size() { return tw_off(S); }
};

// Register block of NB butterflies of radix R; shared by engines whose stages
// have the same shape, so registers can pass from one plan to another.
template <typename V, int NB, int R> struct RegBlock {
    V v[NB][R];
};

template <int I, int N, class F> __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

template <typename T, class RP, int B, int NT, bool WSYNC = false> struct Engine {
    using V = cx<T>;
    static constexpr int NW = NT / 64;
    static constexpr int PPW = B / NW;  // pencils per wavefront under MAP_WV
    static_assert(!WSYNC || (NT % 64 == 0 && B % NW == 0 && PPW >= 1), "wave-owned pencils need B divisible by waves");

    __device__ __forceinline__ static void sync()
    {
        if constexpr (WSYNC) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    }
    static constexpr int P = RP::P;
    static constexpr int S = RP::S;
    static constexpr int LP = P + P / 16 + 1;
    static constexpr int LDS_ELEMS = B * LP;

    template <int s> static constexpr int R = RP::r[s];
    template <int s> static constexpr int Q = P / RP::r[s];
    template <int s> static constexpr int BF = B * (P / RP::r[s]);
    template <int s> static constexpr int NB = (BF<s> + NT - 1) / NT;
    template <int s> static constexpr bool FULL = (BF<s> % NT) == 0;

    template <int s> using Regs = RegBlock<V, NB<s>, R<s>>;

    __device__ __forceinline__ static int lidx(int p, int k) { return p * LP + k + (k >> 4); }

    template <int s, int MAP> __device__ __forceinline__ static void pj(int b, int& p, int& j)
    {
        if constexpr (MAP == MAP_PF) {
            p = b % B;
            j = b / B;
        } else if constexpr (MAP == MAP_EF) {
            j = b % Q<s>;
            p = b / Q<s>;
        } else {
            const int i = b / NT, t = b % NT;
            const int wb = (t & 63) + 64 * i;
            p = (t >> 6) * PPW + wb / Q<s>;
            j = wb % Q<s>;
        }
    }
    template <int s, int MAP> __device__ __forceinline__ static bool valid(int b)
    {
        if constexpr (MAP == MAP_WV) {
            if constexpr ((PPW * Q<s>) % 64 == 0) return true;
            else return ((b % NT) & 63) + 64 * (b / NT) < PPW * Q<s>;
        } else {
            return FULL<s> || b < BF<s>;
        }
    }

    // Stage-s twiddles and DFT on the registers of every butterfly this thread owns.
    template <int s, int DIR, int MAP> __device__ __forceinline__ static void compute(Regs<s>& g, const V* __restrict__ tw)
    {
        constexpr int Rs = R<s>;
        constexpr int NSs = RP::ns(s);
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = tid + i * NT;
            if constexpr (NSs > 1) {
                int p, j;
                pj<s, MAP>(b, p, j);
                if (valid<s, MAP>(b)) {
                    const V* row = tw + RP::tw_off(s) + (j % NSs) * Rs;
#pragma unroll
                    for (int r = 1; r < Rs; ++r) g.v[i][r] = ctw<DIR>(g.v[i][r], row[r]);
                }
            }
            dft<Rs, DIR>(g.v[i]);
        }
    }

    template <int s, int MAP> __device__ __forceinline__ static void store_lds(const Regs<s>& g, V* lds)
    {
        constexpr int Rs = R<s>;
        constexpr int NSs = RP::ns(s);
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = tid + i * NT;
            if (!valid<s, MAP>(b)) continue;
            int p, j;
            pj<s, MAP>(b, p, j);
            const int k0 = (j / NSs) * NSs * Rs + (j % NSs);
#pragma unroll
            for (int r = 0; r < Rs; ++r) lds[lidx(p, k0 + r * NSs)] = g.v[i][r];
        }
    }

    template <int s, int MAP> __device__ __forceinline__ static void load_lds(Regs<s>& g, const V* lds)
    {
        constexpr int Rs = R<s>;
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = tid + i * NT;
            if (!valid<s, MAP>(b)) {
#pragma unroll
                for (int r = 0; r < Rs; ++r) g.v[i][r] = V{T(0), T(0)};
                continue;
            }
            int p, j;
            pj<s, MAP>(b, p, j);
#pragma unroll
            for (int r = 0; r < Rs; ++r) g.v[i][r] = lds[lidx(p, j + r * Q<s>)];
        }
    }

    // Stage-0 inputs from ld(p, idx); idx >= LIN reads as zero.
    template <int MAP, int LIN, class LD> __device__ __forceinline__ static void load_first(Regs<0>& g, LD& ld)
    {
        constexpr int Rs = R<0>;
        constexpr int Qs = Q<0>;
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NB<0>; ++i) {
            const int b = tid + i * NT;
            int p, j;
            pj<0, MAP>(b, p, j);
            const bool ok = valid<0, MAP>(b);
            static_for<0, Rs>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                const int idx = j + r * Qs;
                if constexpr ((r + 1) * Qs <= LIN) {
                    g.v[i][r] = ok ? ld(p, idx) : V{T(0), T(0)};
                } else if constexpr (r * Qs >= LIN) {
                    g.v[i][r] = V{T(0), T(0)};
                } else {
                    g.v[i][r] = (ok && idx < LIN) ? ld(p, idx) : V{T(0), T(0)};
                }
            });
        }
    }

    // Last-stage outputs (natural order) to st(p, idx, v) for idx < LOUT.
    template <int MAP, int LOUT, class ST> __device__ __forceinline__ static void store_last(const Regs<S - 1>& g, ST& st)
    {
        constexpr int s = S - 1;
        constexpr int Rs = R<s>;
        constexpr int Qs = Q<s>;
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = tid + i * NT;
            if (!valid<s, MAP>(b)) continue;
            int p, j;
            pj<s, MAP>(b, p, j);
            static_for<0, Rs>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                const int idx = j + r * Qs;
                if constexpr ((r + 1) * Qs <= LOUT) {
                    st(p, idx, g.v[i][r]);
                } else if constexpr (r * Qs >= LOUT) {
                } else {
                    if (idx < LOUT) st(p, idx, g.v[i][r]);
                }
            });
        }
    }

    // Middle stages [S0, S1) through LDS with mapping MAP.
    template <int s, int S1, int DIR, int MAP> __device__ __forceinline__ static void middle(V* lds, const V* tw)
    {
        if constexpr (s < S1) {
            Regs<s> g;
            sync();
            load_lds<s, MAP>(g, lds);
            compute<s, DIR, MAP>(g, tw);
            sync();
            store_lds<s, MAP>(g, lds);
            middle<s + 1, S1, DIR, MAP>(lds, tw);
        }
    }

    // Full transform: loader -> stages -> storer.  DST_LDS: the storer writes
    // into the same LDS buffer, so a barrier separates the last reads from
    // those writes.
    template <int DIR, int MAP_IN, int MAP_MID, int MAP_OUT, int LIN, int LOUT, bool DST_LDS = false, class LD, class ST>
    __device__ __forceinline__ static void run(V* lds, const V* __restrict__ tw, LD& ld, ST& st)
    {
        if constexpr (S == 1) {
            Regs<0> g;
            load_first<MAP_IN, LIN>(g, ld);
            compute<0, DIR, MAP_IN>(g, tw);
            if constexpr (MAP_IN == MAP_OUT) {
                if constexpr (DST_LDS) sync();
                store_last<MAP_OUT, LOUT>(g, st);
            } else {
                // one stage but different access patterns on the two sides:
                // go through LDS in natural order
                static_assert(!DST_LDS, "LDS destination needs matching mappings");
                sync();
                store_lds<0, MAP_IN>(g, lds);
                sync();
                for (int e = threadIdx.x; e < B * LOUT; e += NT) {
                    int p, idx;
                    if constexpr (MAP_OUT == MAP_PF) {
                        p = e % B;
                        idx = e / B;
                    } else {
                        idx = e % LOUT;
                        p = e / LOUT;
                    }
                    st(p, idx, lds[lidx(p, idx)]);
                }
            }
        } else {
            {
                Regs<0> g;
                load_first<MAP_IN, LIN>(g, ld);
                compute<0, DIR, MAP_IN>(g, tw);
                sync();
                store_lds<0, MAP_IN>(g, lds);
            }
            middle<1, S - 1, DIR, MAP_MID>(lds, tw);
            {
                Regs<S - 1> g;
                sync();
                load_lds<S - 1, MAP_OUT>(g, lds);
                compute<S - 1, DIR, MAP_OUT>(g, tw);
                if constexpr (DST_LDS) sync();
                store_last<MAP_OUT, LOUT>(g, st);
            }
        }
    }

    // Forward stages ending in registers: the last stage's outputs for each
    // owned butterfly (p, j) sit in g.v[i][r] at natural index j + r P/R.
    template <int DIR, int MAP_IN, int MAP_MID, int MAP_OUT, int LIN, class LD>
    __device__ __forceinline__ static void run_to_regs(V* lds, const V* __restrict__ tw, LD& ld, Regs<S - 1>& out)
    {
        if constexpr (S == 1) {
            static_assert(MAP_IN == MAP_OUT, "single-stage plans need one mapping");
            load_first<MAP_IN, LIN>(out, ld);
            compute<0, DIR, MAP_IN>(out, tw);
        } else {
            {
                Regs<0> g;
                load_first<MAP_IN, LIN>(g, ld);
                compute<0, DIR, MAP_IN>(g, tw);
                sync();
                store_lds<0, MAP_IN>(g, lds);
            }
            middle<1, S - 1, DIR, MAP_MID>(lds, tw);
            sync();
            load_lds<S - 1, MAP_OUT>(out, lds);
            compute<S - 1, DIR, MAP_OUT>(out, tw);
        }
    }

    // Stages starting from registers that already hold the stage-0 inputs
    // (index j + r P/R for each owned butterfly (p, j) under MAP_IN).
    template <int DIR, int MAP_IN, int MAP_MID, int MAP_OUT, int LOUT, class ST>
    __device__ __forceinline__ static void run_from_regs(V* lds, const V* __restrict__ tw, Regs<0>& g, ST& st)
    {
        if constexpr (S == 1) {
            static_assert(MAP_IN == MAP_OUT, "single-stage plans need one mapping");
            compute<0, DIR, MAP_IN>(g, tw);
            store_last<MAP_OUT, LOUT>(g, st);
        } else {
            compute<0, DIR, MAP_IN>(g, tw);
            sync();
            store_lds<0, MAP_IN>(g, lds);
            middle<1, S - 1, DIR, MAP_MID>(lds, tw);
            {
                Regs<S - 1> h;
                sync();
                load_lds<S - 1, MAP_OUT>(h, lds);
                compute<S - 1, DIR, MAP_OUT>(h, tw);
                store_last<MAP_OUT, LOUT>(h, st);
            }
        }
    }
};

}  // namespace ps
