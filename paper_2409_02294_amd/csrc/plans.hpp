// Radix factorisations for the supported padded lengths P = 2N.
//
// Every supported P is 16 m, P <= 1024, with m free of prime factors above 5
// (P = 2^a 3^b 5^c, a >= 4).  The forward plan
// starts with radix 16 (so zero padding of half the pencil removes half of
// the first stage's inputs at compile time) and the inverse plan is the
// forward plan reversed (so it ends with radix 16 and cropping removes half
// of the last stage's outputs, and the fused z pass can hand the forward's
// last-stage registers straight to the inverse's first stage).
#pragma once
#include "fft_engine.hpp"

namespace ps {

// Family 0: radix 16 first, the remaining factors, the inverse reversed.
template <int P, int FAM = 0> struct PlanFor;
template <> struct PlanFor<16, 0> { using Fwd = Radices<16>; using Inv = Radices<16>; };
template <> struct PlanFor<32, 0> { using Fwd = Radices<16, 2>; using Inv = Radices<2, 16>; };
template <> struct PlanFor<48, 0> { using Fwd = Radices<16, 3>; using Inv = Radices<3, 16>; };
template <> struct PlanFor<64, 0> { using Fwd = Radices<16, 4>; using Inv = Radices<4, 16>; };
template <> struct PlanFor<96, 0> { using Fwd = Radices<16, 6>; using Inv = Radices<6, 16>; };
template <> struct PlanFor<128, 0> { using Fwd = Radices<16, 8>; using Inv = Radices<8, 16>; };
template <> struct PlanFor<192, 0> { using Fwd = Radices<16, 12>; using Inv = Radices<12, 16>; };
template <> struct PlanFor<256, 0> { using Fwd = Radices<16, 16>; using Inv = Radices<16, 16>; };
template <> struct PlanFor<384, 0> { using Fwd = Radices<16, 3, 8>; using Inv = Radices<8, 3, 16>; };
template <> struct PlanFor<512, 0> { using Fwd = Radices<16, 2, 16>; using Inv = Radices<16, 2, 16>; };
template <> struct PlanFor<768, 0> { using Fwd = Radices<16, 3, 16>; using Inv = Radices<16, 3, 16>; };
template <> struct PlanFor<1024, 0> { using Fwd = Radices<16, 4, 16>; using Inv = Radices<16, 4, 16>; };
// lengths with factors 3^2 or 5; radices 6, 10, 12, 15, 20 are prime-factor
// DFTs in registers (no inner twiddles), which saves a stage and its LDS
// exchange against splitting them into their factors
template <> struct PlanFor<80, 0> { using Fwd = Radices<16, 5>; using Inv = Radices<5, 16>; };
template <> struct PlanFor<144, 0> { using Fwd = Radices<16, 3, 3>; using Inv = Radices<3, 3, 16>; };
template <> struct PlanFor<160, 0> { using Fwd = Radices<16, 10>; using Inv = Radices<10, 16>; };
template <> struct PlanFor<240, 0> { using Fwd = Radices<16, 15>; using Inv = Radices<15, 16>; };
template <> struct PlanFor<288, 0> { using Fwd = Radices<16, 6, 3>; using Inv = Radices<3, 6, 16>; };
template <> struct PlanFor<320, 0> { using Fwd = Radices<16, 20>; using Inv = Radices<20, 16>; };
template <> struct PlanFor<400, 0> { using Fwd = Radices<16, 5, 5>; using Inv = Radices<5, 5, 16>; };
template <> struct PlanFor<432, 0> { using Fwd = Radices<16, 3, 3, 3>; using Inv = Radices<3, 3, 3, 16>; };
template <> struct PlanFor<480, 0> { using Fwd = Radices<16, 15, 2>; using Inv = Radices<2, 15, 16>; };
template <> struct PlanFor<576, 0> { using Fwd = Radices<16, 12, 3>; using Inv = Radices<3, 12, 16>; };
template <> struct PlanFor<640, 0> { using Fwd = Radices<16, 5, 8>; using Inv = Radices<8, 5, 16>; };
template <> struct PlanFor<720, 0> { using Fwd = Radices<16, 15, 3>; using Inv = Radices<3, 15, 16>; };
template <> struct PlanFor<800, 0> { using Fwd = Radices<16, 10, 5>; using Inv = Radices<5, 10, 16>; };
template <> struct PlanFor<864, 0> { using Fwd = Radices<16, 6, 3, 3>; using Inv = Radices<3, 3, 6, 16>; };
template <> struct PlanFor<960, 0> { using Fwd = Radices<16, 15, 4>; using Inv = Radices<4, 15, 16>; };

// Every supported P, for the launchers' switch statements.
#define PS_FOR_EACH_P(X)                                                                                      \
    X(16) X(32) X(48) X(64) X(80) X(96) X(128) X(144) X(160) X(192) X(240) X(256) X(288) X(320) X(384)    \
    X(400) X(432) X(480) X(512) X(576) X(640) X(720) X(768) X(800) X(864) X(960) X(1024)

// Family 1: two stages in all (one LDS exchange fewer per transform than
// family 0 where that has three or more), radix 32 first where P allows it,
// else radix 24 or 16; 10, 12, 15, 20, 24 and 30 are prime-factor DFTs in
// registers, 9, 25 and 27 Cooley-Tukey ones (3 x 3, 5 x 5, 3 x 9).
template <int P> constexpr bool has_fam1()
{
    return P == 144 || P == 288 || P == 320 || P == 384 || P == 400 || P == 432 || P == 480 || P == 512 ||
           P == 576 || P == 640 || P == 720 || P == 768 || P == 800 || P == 864 || P == 960 || P == 1024;
}
template <> struct PlanFor<144, 1> { using Fwd = Radices<16, 9>; using Inv = Radices<9, 16>; };
template <> struct PlanFor<288, 1> { using Fwd = Radices<24, 12>; using Inv = Radices<12, 24>; };
template <> struct PlanFor<320, 1> { using Fwd = Radices<32, 10>; using Inv = Radices<10, 32>; };
template <> struct PlanFor<384, 1> { using Fwd = Radices<32, 12>; using Inv = Radices<12, 32>; };
template <> struct PlanFor<400, 1> { using Fwd = Radices<16, 25>; using Inv = Radices<25, 16>; };
template <> struct PlanFor<432, 1> { using Fwd = Radices<16, 27>; using Inv = Radices<27, 16>; };
template <> struct PlanFor<480, 1> { using Fwd = Radices<32, 15>; using Inv = Radices<15, 32>; };
template <> struct PlanFor<512, 1> { using Fwd = Radices<32, 16>; using Inv = Radices<16, 32>; };
template <> struct PlanFor<576, 1> { using Fwd = Radices<24, 24>; using Inv = Radices<24, 24>; };
template <> struct PlanFor<640, 1> { using Fwd = Radices<32, 20>; using Inv = Radices<20, 32>; };
template <> struct PlanFor<720, 1> { using Fwd = Radices<24, 30>; using Inv = Radices<30, 24>; };
template <> struct PlanFor<768, 1> { using Fwd = Radices<32, 24>; using Inv = Radices<24, 32>; };
template <> struct PlanFor<800, 1> { using Fwd = Radices<32, 25>; using Inv = Radices<25, 32>; };
template <> struct PlanFor<864, 1> { using Fwd = Radices<32, 27>; using Inv = Radices<27, 32>; };
template <> struct PlanFor<960, 1> { using Fwd = Radices<32, 30>; using Inv = Radices<30, 32>; };
template <> struct PlanFor<1024, 1> { using Fwd = Radices<32, 32>; using Inv = Radices<32, 32>; };
// Elements per thread of a family-1 pass: 32 where both radices are powers
// of two (a thread may hold two radix-16 butterflies), else the smaller
// radix, so that the stage with the most butterflies gives each thread one.
template <int P> constexpr int fam1_elems()
{
    if constexpr (!has_fam1<P>() || P == 512 || P == 1024) {
        return 32;
    } else {
        using R = typename PlanFor<P, 1>::Fwd;
        return R::r[0] < R::r[1] ? R::r[0] : R::r[1];
    }
}

// Threads for B pencils of length P at ~E elements per thread, whole waves.
constexpr int threads_for(int B, int P, int E = 16)
{
    int t = B * P / E;
    t = (t + 63) / 64 * 64;
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return t;
}

}  // namespace ps
