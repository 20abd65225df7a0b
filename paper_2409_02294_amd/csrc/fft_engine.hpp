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
// one pad slot every G elements (k -> k + k/G), G = 32 when the first radix
// is 32 and 16 otherwise.  The first stage's stores run over butterflies j
// at stride R (element j R + r), which the pad turns into an odd stride of
// R + 1 slots for R = G, so the 8-byte stores of a wavefront spread over all
// banks; every later stage reads and writes consecutive elements across
// lanes, which the pad does not disturb.
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
// host and rounded once to T: for stage s >= 1 and residue m = j mod NS,
// entry r is exp(-2 pi i r m / (NS R)) (the inverse direction uses the
// conjugate).  The table holds every stage twice: by rows (m major, R
// entries per residue) and by columns (r major, NS entries per r).  A stage
// whose lanes run over consecutive butterflies (MAP_EF, MAP_WV) reads
// columns, one contiguous span per wavefront load; a stage whose lanes run
// over pencils first (MAP_PF, where groups of B lanes share a residue) reads
// rows, a few wide loads per lane.
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
    // offset (complex entries) of stage s's twiddle rows; its columns follow
    // all the rows, at tw_size() + tw_off(s)
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

// ---------------------------------------------------------------------------
// Radix-16 DFTs on the bf16 matrix cores with split operands.
//
// A length-16 DFT of 32 pencils at once is the real product
//   [Re y; Im y] = [[Wr, -Wi], [Wi, Wr]] [Re x; Im x]
// of a 32 x 32 matrix and a 32 x 32 block (one column per pencil), done as
// two v_mfma_f32_32x32x16_bf16 per product term (K = 16 real parts, then 16
// imaginary parts).  Every operand is split into bf16 pieces, x = x0 + x1 + x2
// with x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1) (each
// difference is exact in fp32), and the product is summed over the piece
// pairs of order <= 2 (six terms, MT = 6) or <= 1 with two pieces (three
// terms, MT = 3), accumulating in fp32.  The matrix pieces are split in double
// on the host and loaded once per workgroup.
//
// Lane layout (wavefront of 64): lane l works on pencil column c = l % 32 and
// holds elements 8h .. 8h+7 (h = l / 32) of that column's 16 inputs, and
// after the product the same element indices of the 16 outputs: the matrix
// rows are permuted so that the accumulator layout of the instruction (lane l
// holds rows 8j + 4h + i, j, i < 4) lands on outputs 8h + 4(j % 2) + i, real
// part for j < 2 and imaginary part for j >= 2.  The inverse transform uses
// conj(DFT(conj x)).
// ---------------------------------------------------------------------------
typedef __bf16 ps_bf16x8 __attribute__((ext_vector_type(8)));
typedef float ps_f32x16 __attribute__((ext_vector_type(16)));

template <int MT> struct SplitA {
    ps_bf16x8 a[3][2];  // [piece][K chunk: 0 real parts, 1 imaginary parts]
    // tab: [piece][chunk][lane][8] bf16 bit patterns
    __device__ __forceinline__ void load(const unsigned short* __restrict__ tab)
    {
        const int l = threadIdx.x & 63;
#pragma unroll
        for (int pc = 0; pc < 3; ++pc)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                a[pc][c] = *reinterpret_cast<const ps_bf16x8*>(tab + ((pc * 2 + c) * 64 + l) * 8);
    }
};
template <> struct SplitA<0> {
    __device__ __forceinline__ void load(const unsigned short*) {}
};

typedef float ps_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 ps_bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned ps_u32x4 __attribute__((ext_vector_type(4)));

// The NP bf16 pieces of x[0..7], two elements per 32-bit register as the
// matrix instruction's operand holds them: each pair is rounded by one
// packed conversion (round to nearest even), and its residual is formed
// from the two halves of the packed result (a bf16 value is the top half of
// the float it rounds to, so shifting or masking recovers it exactly).
template <int NP> __device__ __forceinline__ void split_pieces(const float* x, ps_bf16x8* out)
{
    ps_u32x4 w[NP];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ps_f32x2 r = {x[2 * i], x[2 * i + 1]};
#pragma unroll
        for (int pc = 0; pc < NP; ++pc) {
            const unsigned u = __builtin_bit_cast(unsigned, __builtin_convertvector(r, ps_bf16x2));
            w[pc][i] = u;
            if (pc + 1 < NP)
                r = ps_f32x2{r[0] - __builtin_bit_cast(float, u << 16), r[1] - __builtin_bit_cast(float, u & 0xffff0000u)};
        }
    }
#pragma unroll
    for (int pc = 0; pc < NP; ++pc) out[pc] = __builtin_bit_cast(ps_bf16x8, w[pc]);
}

// In-place forward (DIR -1) or inverse (DIR +1) DFT-16 of the lane's 8 elements.
template <int MT, int DIR> __device__ __forceinline__ void dft16_split(float2* v, const SplitA<MT>& sa)
{
    static_assert(MT == 3 || MT == 6, "3 or 6 product terms");
    constexpr int NP = MT == 6 ? 3 : 2;
    float re[8], im[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        re[q] = v[q].x;
        im[q] = DIR < 0 ? v[q].y : -v[q].y;
    }
    ps_bf16x8 br[NP], bi[NP];
    split_pieces<NP>(re, br);
    split_pieces<NP>(im, bi);
    ps_f32x16 acc = {};
    // smallest terms first
    if constexpr (MT == 6) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[2][0], br[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[2][1], bi[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[1][0], br[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[1][1], bi[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[0][0], br[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[0][1], bi[2], acc, 0, 0, 0);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[1][0], br[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[1][1], bi[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[0][0], br[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[0][1], bi[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[0][0], br[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa.a[0][1], bi[0], acc, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = float2{acc[q], DIR < 0 ? acc[8 + q] : -acc[8 + q]};
}

// LDS row pitch (complex elements) of a length-P pencil with one pad slot
// every G elements, for elements of EB bytes.  8-byte elements take
// P + P/G + 1.  16-byte elements take the next pitch that is 4 mod 8: with
// the pencil-fastest mapping (8 pencils by 2 offsets in 16 lanes), 16-byte
// accesses measured free of bank conflicts on gfx950 only at such pitches
// (8 extra cycles per instruction at 1 mod 16, 4 at 2 mod 16).
constexpr int pad_pitch(int P, int G, int EB = 8)
{
    const int lp = P + P / G + 1;
    return EB == 16 ? lp + (12 - lp % 8) % 8 : lp;
}
constexpr int pad_shift(int r0) { return r0 == 32 ? 5 : 4; }

// MT: 0 = every stage on the vector ALUs; 3 or 6 = radix-16 stages on the
// matrix cores with that many split product terms (T = float only).
// PITCH: LDS row pitch of a pencil, when it must exceed the plan's own (two
// plans sharing one buffer under wavefront-level synchronisation need equal
// rows, so that each wavefront's pencils occupy the same LDS in both).
template <typename T, class RP, int B, int NT, bool WSYNC = false, int MT = 0, int PITCH = 0> struct Engine {
    using V = cx<T>;
    using SA = SplitA<MT>;
    static_assert(MT == 0 || std::is_same<T, float>::value, "split matrix-core DFTs are single precision");
    static constexpr int NW = NT / 64;
    static constexpr int PPW = B / NW;  // pencils per wavefront under MAP_WV
    static_assert(!WSYNC || (NT % 64 == 0 && B % NW == 0 && PPW >= 1), "wave-owned pencils need B divisible by waves");
    static_assert(MT == 0 || NT % 64 == 0, "matrix-core stages need whole wavefronts");

    // Barrier between an LDS phase with mapping MA and one with mapping MB:
    // wavefront-level only when both keep every pencil inside one wavefront.
    template <int MA, int MB> __device__ __forceinline__ static void sync2()
    {
        if constexpr (WSYNC && MA == MAP_WV && MB == MAP_WV) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    }
    static constexpr int P = RP::P;
    static constexpr int S = RP::S;
    static constexpr int GS = pad_shift(RP::r[0]);  // log2 of the pad granularity G
    static constexpr int G = 1 << GS;
    static_assert(PITCH == 0 || PITCH >= pad_pitch(P, G), "row pitch below the padded pencil");
    static constexpr int LP = PITCH > 0 ? PITCH : pad_pitch(P, G, (int)sizeof(V));
    static constexpr int LDS_ELEMS = B * LP;

    // Twiddle source: the row and column layouts of the plan's table.  A
    // plain table pointer holds both (columns after all the rows); a kernel
    // may instead point the columns at a copy in LDS.
    struct TW {
        const V* rows;
        const V* cols;
        __device__ __forceinline__ TW(const V* t) : rows(t), cols(t + RP::tw_size()) {}
        __device__ __forceinline__ TW(const V* r, const V* c) : rows(r), cols(c) {}
    };

    template <int s> static constexpr int R = RP::r[s];
    template <int s> static constexpr int Q = P / RP::r[s];
    template <int s> static constexpr int BF = B * (P / RP::r[s]);
    // Slots: a thread holds NB slots of RS elements per stage.  A slot is a
    // whole butterfly on the vector ALUs, or half of one (8 of 16 elements)
    // on a matrix-core stage, where a wavefront spans 32 butterflies.
    template <int s> static constexpr bool MF = (MT > 0) && (RP::r[s] == 16);
    template <int s> static constexpr int RS = MF<s> ? 8 : RP::r[s];
    template <int s> static constexpr int NTV = MF<s> ? NT / 2 : NT;
    template <int s> static constexpr int WVW = MF<s> ? 32 : 64;
    template <int s> static constexpr int NB = (BF<s> + NTV<s> - 1) / NTV<s>;
    template <int s> static constexpr bool FULL = (BF<s> % NTV<s>) == 0;

    template <int s> using Regs = RegBlock<V, NB<s>, RS<s>>;

    __device__ __forceinline__ static int lidx(int p, int k) { return p * LP + k + (k >> GS); }

    // virtual thread index and element offset of this thread for stage s
    template <int s> __device__ __forceinline__ static int vthread()
    {
        const int tid = threadIdx.x;
        if constexpr (MF<s>) return (tid >> 6) * 32 + (tid & 31);
        else return tid;
    }
    template <int s> __device__ __forceinline__ static int roff()
    {
        if constexpr (MF<s>) return 8 * ((threadIdx.x & 63) >> 5);
        else return 0;
    }

    template <int s, int MAP> __device__ __forceinline__ static void pj(int b, int& p, int& j)
    {
        if constexpr (MAP == MAP_PF) {
            p = b % B;
            j = b / B;
        } else if constexpr (MAP == MAP_EF) {
            j = b % Q<s>;
            p = b / Q<s>;
        } else {
            const int i = b / NTV<s>, t = b % NTV<s>;
            const int wb = (t % WVW<s>) + WVW<s> * i;
            p = (t / WVW<s>) * PPW + wb / Q<s>;
            j = wb % Q<s>;
        }
    }
    template <int s, int MAP> __device__ __forceinline__ static bool valid(int b)
    {
        if constexpr (MAP == MAP_WV) {
            if constexpr ((PPW * Q<s>) % WVW<s> == 0) return true;
            else return (b % NTV<s>) % WVW<s> + WVW<s> * (b / NTV<s>) < PPW * Q<s>;
        } else {
            return FULL<s> || b < BF<s>;
        }
    }

    // Stage-s twiddles and DFT on every slot this thread owns.
    template <int s, int DIR, int MAP>
    __device__ __forceinline__ static void compute(Regs<s>& g, const TW& tw, const SA& sa)
    {
        constexpr int Rs = R<s>;
        constexpr int NSs = RP::ns(s);
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            if constexpr (NSs > 1) {
                int p, j;
                pj<s, MAP>(b, p, j);
                if (valid<s, MAP>(b)) {
                    if constexpr (MAP == MAP_PF) {
                        const V* row = tw.rows + RP::tw_off(s) + (j % NSs) * Rs + ro;
#pragma unroll
                        for (int q = 0; q < RS<s>; ++q)
                            if (MF<s> || q > 0) g.v[i][q] = ctw<DIR>(g.v[i][q], row[q]);
                    } else {
                        const V* col = tw.cols + RP::tw_off(s) + ro * NSs + (j % NSs);
#pragma unroll
                        for (int q = 0; q < RS<s>; ++q)
                            if (MF<s> || q > 0) g.v[i][q] = ctw<DIR>(g.v[i][q], col[q * NSs]);
                    }
                }
            }
            if constexpr (MF<s>) dft16_split<MT, DIR>(g.v[i], sa);
            else dft<Rs, DIR>(g.v[i]);
        }
    }

    template <int s, int MAP> __device__ __forceinline__ static void store_lds(const Regs<s>& g, V* lds)
    {
        constexpr int Rs = R<s>;
        constexpr int NSs = RP::ns(s);
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            if (!valid<s, MAP>(b)) continue;
            int p, j;
            pj<s, MAP>(b, p, j);
            const int k0 = (j / NSs) * NSs * Rs + (j % NSs);
            // LDS addresses as one base plus compile-time offsets where the
            // pad-every-G layout allows it
            if constexpr (NSs % G == 0) {
                V* base = lds + lidx(p, k0) + (ro * NSs) * (G + 1) / G;
#pragma unroll
                for (int q = 0; q < RS<s>; ++q) base[(q * NSs) * (G + 1) / G] = g.v[i][q];
            } else if constexpr (NSs == 1 && Rs % G == 0) {
                V* base = lds + lidx(p, k0) + ro;  // k0 = j R is a multiple of G, ro + q < G or ro = 0
#pragma unroll
                for (int q = 0; q < RS<s>; ++q) base[q + (q >> GS)] = g.v[i][q];
            } else {
#pragma unroll
                for (int q = 0; q < RS<s>; ++q) lds[lidx(p, k0 + (ro + q) * NSs)] = g.v[i][q];
            }
        }
    }

    template <int s, int MAP> __device__ __forceinline__ static void load_lds(Regs<s>& g, const V* lds)
    {
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            if (!valid<s, MAP>(b)) {
#pragma unroll
                for (int q = 0; q < RS<s>; ++q) g.v[i][q] = V{T(0), T(0)};
                continue;
            }
            int p, j;
            pj<s, MAP>(b, p, j);
            if constexpr (Q<s> % G == 0) {
                const V* base = lds + lidx(p, j) + (ro * Q<s>) * (G + 1) / G;
#pragma unroll
                for (int q = 0; q < RS<s>; ++q) g.v[i][q] = base[(q * Q<s>) * (G + 1) / G];
            } else {
#pragma unroll
                for (int q = 0; q < RS<s>; ++q) g.v[i][q] = lds[lidx(p, j + (ro + q) * Q<s>)];
            }
        }
    }

    // Two-round exchange through half the LDS: round RND moves the positions
    // [RND P/2, (RND + 1) P/2) of every pencil, so a pencil needs a row of
    // P/2 (padded as a full row is) instead of P.  LPH: that row's pitch,
    // shared by the plans that use one buffer.
    static constexpr int half_pitch() { return pad_pitch(P / 2, G, (int)sizeof(V)); }
    template <int LPH> __device__ __forceinline__ static int lidxh(int p, int k) { return p * LPH + k + (k >> GS); }

    template <int s, int MAP, int RND, int LPH> __device__ __forceinline__ static void store_lds_half(const Regs<s>& g, V* lds)
    {
        constexpr int Rs = R<s>;
        constexpr int NSs = RP::ns(s);
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            if (!valid<s, MAP>(b)) continue;
            int p, j;
            pj<s, MAP>(b, p, j);
            const int k0 = (j / NSs) * NSs * Rs + (j % NSs);
#pragma unroll
            for (int q = 0; q < RS<s>; ++q) {
                const int k = k0 + (ro + q) * NSs;
                if ((k >= P / 2) == (RND == 1)) lds[lidxh<LPH>(p, k - RND * (P / 2))] = g.v[i][q];
            }
        }
    }

    template <int s, int MAP, int RND, int LPH> __device__ __forceinline__ static void load_lds_half(Regs<s>& g, const V* lds)
    {
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            if (!valid<s, MAP>(b)) {
                if constexpr (RND == 0) {
#pragma unroll
                    for (int q = 0; q < RS<s>; ++q) g.v[i][q] = V{T(0), T(0)};
                }
                continue;
            }
            int p, j;
            pj<s, MAP>(b, p, j);
#pragma unroll
            for (int q = 0; q < RS<s>; ++q) {
                const int k = j + (ro + q) * Q<s>;
                if ((k >= P / 2) == (RND == 1)) g.v[i][q] = lds[lidxh<LPH>(p, k - RND * (P / 2))];
            }
        }
    }

    // Stage s's outputs (mapping MW) to stage s + 1's inputs (mapping MR) in
    // two rounds; MPREV is the mapping of the last LDS reads before it.
    template <int s, int MW, int MR, int MPREV, int LPH>
    __device__ __forceinline__ static void exchange_half(const Regs<s>& g, Regs<s + 1>& g2, V* lds)
    {
        sync2<MPREV, MW>();
        store_lds_half<s, MW, 0, LPH>(g, lds);
        sync2<MW, MR>();
        load_lds_half<s + 1, MR, 0, LPH>(g2, lds);
        sync2<MR, MW>();
        store_lds_half<s, MW, 1, LPH>(g, lds);
        sync2<MW, MR>();
        load_lds_half<s + 1, MR, 1, LPH>(g2, lds);
    }

    // Stages s .. S - 1 on g (stage s's inputs), exchanging through half the
    // LDS; stages before the last use mapping MAP, the last MLAST.  out: the
    // last stage's outputs.
    template <int s, int DIR, int MAP, int MLAST, int MPREV, int LPH>
    __device__ __forceinline__ static void stages_half(Regs<s>& g, Regs<S - 1>& out, V* lds, const TW& tw, const SA& sa)
    {
        constexpr int M = s == S - 1 ? MLAST : MAP;
        compute<s, DIR, M>(g, tw, sa);
        if constexpr (s == S - 1) {
            out = g;
        } else {
            constexpr int MN = s + 1 == S - 1 ? MLAST : MAP;
            Regs<s + 1> g2;
            exchange_half<s, M, MN, MPREV, LPH>(g, g2, lds);
            stages_half<s + 1, DIR, MAP, MLAST, MN, LPH>(g2, out, lds, tw, sa);
        }
    }

    // Full transform as run(), every stage exchange through half the LDS
    // (LPH: its row pitch); stage 0 and the middle stages use MAP_IN.
    template <int DIR, int MAP_IN, int MAP_OUT, int LIN, int LOUT, int LPH, class LD, class ST>
    __device__ __forceinline__ static void run_half(V* lds, const TW& tw, LD& ld, ST& st, const SA& sa = SA{})
    {
        static_assert(S > 1, "two or more stages");
        Regs<0> g;
        load_first<MAP_IN, LIN>(g, ld);
        Regs<S - 1> h;
        stages_half<0, DIR, MAP_IN, MAP_OUT, MAP_IN, LPH>(g, h, lds, tw, sa);
        store_last<MAP_OUT, LOUT>(h, st);
    }

    // Stage-0 inputs from ld(p, idx); idx >= LIN reads as zero.
    template <int MAP, int LIN, class LD> __device__ __forceinline__ static void load_first(Regs<0>& g, LD& ld)
    {
        constexpr int Qs = Q<0>;
        const int vt = vthread<0>(), ro = roff<0>();
#pragma unroll
        for (int i = 0; i < NB<0>; ++i) {
            const int b = vt + i * NTV<0>;
            int p, j;
            pj<0, MAP>(b, p, j);
            const bool ok = valid<0, MAP>(b);
            if constexpr (MF<0>) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int idx = j + (ro + q) * Qs;
                    g.v[i][q] = (ok && idx < LIN) ? ld(p, idx) : V{T(0), T(0)};
                }
            } else {
                static_for<0, RS<0>>([&](auto rc) {
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
    }

    // Last-stage outputs (natural order) to st(p, idx, v) for idx < LOUT.
    template <int MAP, int LOUT, class ST> __device__ __forceinline__ static void store_last(const Regs<S - 1>& g, ST& st)
    {
        constexpr int s = S - 1;
        constexpr int Qs = Q<s>;
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            if (!valid<s, MAP>(b)) continue;
            int p, j;
            pj<s, MAP>(b, p, j);
            if constexpr (MF<s>) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int idx = j + (ro + q) * Qs;
                    if (idx < LOUT) st(p, idx, g.v[i][q]);
                }
            } else {
                static_for<0, RS<s>>([&](auto rc) {
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
    }

    // f(p, idx, v&) on every element held after stage s (index in natural
    // order of that stage's outputs when s is the last stage).
    template <int s, int MAP, class F> __device__ __forceinline__ static void for_each_out(Regs<s>& g, F& f)
    {
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            if (!valid<s, MAP>(b)) continue;
            int p, j;
            pj<s, MAP>(b, p, j);
#pragma unroll
            for (int q = 0; q < RS<s>; ++q) f(p, j + (ro + q) * Q<s>, g.v[i][q]);
        }
    }

    // out[i][q] = f(p, idx) for every element held after stage s, in the
    // layout of Regs<s> (slots this thread does not own are zero).
    template <int s, int MAP, class F>
    __device__ __forceinline__ static void gather(T (&out)[NB<s>][RS<s>], F& f)
    {
        const int vt = vthread<s>(), ro = roff<s>();
#pragma unroll
        for (int i = 0; i < NB<s>; ++i) {
            const int b = vt + i * NTV<s>;
            const bool ok = valid<s, MAP>(b);
            int p, j;
            pj<s, MAP>(b, p, j);
#pragma unroll
            for (int q = 0; q < RS<s>; ++q) out[i][q] = ok ? f(p, j + (ro + q) * Q<s>) : T(0);
        }
    }
    // g *= w element by element (w real, laid out like Regs<s>).
    template <int s> __device__ __forceinline__ static void scale(Regs<s>& g, const T (&w)[NB<s>][RS<s>])
    {
#pragma unroll
        for (int i = 0; i < NB<s>; ++i)
#pragma unroll
            for (int q = 0; q < RS<s>; ++q) g.v[i][q] = V{g.v[i][q].x * w[i][q], g.v[i][q].y * w[i][q]};
    }

    // Middle stages [S0, S1) through LDS with mapping MAP; MPREV is the
    // mapping of the stage that wrote the LDS before stage S0.
    template <int s, int S1, int DIR, int MAP, int MPREV>
    __device__ __forceinline__ static void middle(V* lds, const TW& tw, const SA& sa)
    {
        if constexpr (s < S1) {
            Regs<s> g;
            sync2<MPREV, MAP>();
            load_lds<s, MAP>(g, lds);
            compute<s, DIR, MAP>(g, tw, sa);
            sync2<MAP, MAP>();
            store_lds<s, MAP>(g, lds);
            middle<s + 1, S1, DIR, MAP, MAP>(lds, tw, sa);
        }
    }
    // mapping of the stage that writes the LDS read by the last stage
    template <int MAP_IN, int MAP_MID> static constexpr int map_before_last = S > 2 ? MAP_MID : MAP_IN;

    // Full transform: loader -> stages -> storer.  DST_LDS: the storer writes
    // into the same LDS buffer, so a barrier separates the last reads from
    // those writes.
    template <int DIR, int MAP_IN, int MAP_MID, int MAP_OUT, int LIN, int LOUT, bool DST_LDS = false, class LD, class ST>
    __device__ __forceinline__ static void run(V* lds, const TW& tw, LD& ld, ST& st, const SA& sa = SA{})
    {
        if constexpr (S == 1) {
            Regs<0> g;
            load_first<MAP_IN, LIN>(g, ld);
            compute<0, DIR, MAP_IN>(g, tw, sa);
            if constexpr (MAP_IN == MAP_OUT) {
                if constexpr (DST_LDS) __syncthreads();
                store_last<MAP_OUT, LOUT>(g, st);
            } else {
                // one stage but different access patterns on the two sides:
                // go through LDS in natural order
                static_assert(!DST_LDS, "LDS destination needs matching mappings");
                __syncthreads();
                store_lds<0, MAP_IN>(g, lds);
                __syncthreads();
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
                compute<0, DIR, MAP_IN>(g, tw, sa);
                sync2<MAP_IN, MAP_IN>();
                store_lds<0, MAP_IN>(g, lds);
            }
            middle<1, S - 1, DIR, MAP_MID, MAP_IN>(lds, tw, sa);
            {
                Regs<S - 1> g;
                sync2<map_before_last<MAP_IN, MAP_MID>, MAP_OUT>();
                load_lds<S - 1, MAP_OUT>(g, lds);
                compute<S - 1, DIR, MAP_OUT>(g, tw, sa);
                if constexpr (DST_LDS) __syncthreads();
                store_last<MAP_OUT, LOUT>(g, st);
            }
        }
    }

    // Forward stages ending in registers: the last stage's outputs for each
    // owned butterfly (p, j) sit in g.v[i][r] at natural index j + r P/R.
    template <int DIR, int MAP_IN, int MAP_MID, int MAP_OUT, int LIN, class LD>
    __device__ __forceinline__ static void run_to_regs(V* lds, const TW& tw, LD& ld, Regs<S - 1>& out,
                                                       const SA& sa = SA{})
    {
        if constexpr (S == 1) {
            static_assert(MAP_IN == MAP_OUT, "single-stage plans need one mapping");
            load_first<MAP_IN, LIN>(out, ld);
            compute<0, DIR, MAP_IN>(out, tw, sa);
        } else {
            {
                Regs<0> g;
                load_first<MAP_IN, LIN>(g, ld);
                compute<0, DIR, MAP_IN>(g, tw, sa);
                sync2<MAP_IN, MAP_IN>();
                store_lds<0, MAP_IN>(g, lds);
            }
            middle<1, S - 1, DIR, MAP_MID, MAP_IN>(lds, tw, sa);
            sync2<map_before_last<MAP_IN, MAP_MID>, MAP_OUT>();
            load_lds<S - 1, MAP_OUT>(out, lds);
            compute<S - 1, DIR, MAP_OUT>(out, tw, sa);
        }
    }

    // As run_to_regs, with the stage-0 inputs already in registers (loaded
    // by load_first earlier, e.g. one tile ahead).  The first LDS exchange
    // synchronises only as MAP_IN requires: a caller reusing the LDS across
    // tiles separates the tiles with a workgroup barrier.
    template <int DIR, int MAP_IN, int MAP_MID, int MAP_OUT>
    __device__ __forceinline__ static void run_to_regs_loaded(V* lds, const TW& tw, Regs<0>& g, Regs<S - 1>& out,
                                                              const SA& sa = SA{})
    {
        static_assert(S > 1, "single-stage plans load and compute in one step");
        compute<0, DIR, MAP_IN>(g, tw, sa);
        sync2<MAP_IN, MAP_IN>();
        store_lds<0, MAP_IN>(g, lds);
        middle<1, S - 1, DIR, MAP_MID, MAP_IN>(lds, tw, sa);
        sync2<map_before_last<MAP_IN, MAP_MID>, MAP_OUT>();
        load_lds<S - 1, MAP_OUT>(out, lds);
        compute<S - 1, DIR, MAP_OUT>(out, tw, sa);
    }

    // Stages starting from registers that already hold the stage-0 inputs
    // (index j + r P/R for each owned butterfly (p, j) under MAP_IN).
    template <int DIR, int MAP_IN, int MAP_MID, int MAP_OUT, int LOUT, class ST>
    __device__ __forceinline__ static void run_from_regs(V* lds, const TW& tw, Regs<0>& g, ST& st,
                                                         const SA& sa = SA{})
    {
        if constexpr (S == 1) {
            compute<0, DIR, MAP_IN>(g, tw, sa);
            if constexpr (MAP_IN == MAP_OUT) {
                store_last<MAP_OUT, LOUT>(g, st);
            } else {
                // one stage, different output pattern: through LDS in natural order
                __syncthreads();
                store_lds<0, MAP_IN>(g, lds);
                __syncthreads();
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
            compute<0, DIR, MAP_IN>(g, tw, sa);
            sync2<MAP_IN, MAP_IN>();
            store_lds<0, MAP_IN>(g, lds);
            middle<1, S - 1, DIR, MAP_MID, MAP_IN>(lds, tw, sa);
            {
                Regs<S - 1> h;
                sync2<map_before_last<MAP_IN, MAP_MID>, MAP_OUT>();
                load_lds<S - 1, MAP_OUT>(h, lds);
                compute<S - 1, DIR, MAP_OUT>(h, tw, sa);
                store_last<MAP_OUT, LOUT>(h, st);
            }
        }
    }
};

}  // namespace ps
