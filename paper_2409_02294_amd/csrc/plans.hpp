// Radix factorisations for the supported padded lengths P = 2N.
//
// Every supported P is 2^a or 3 * 2^a with 16 <= P <= 1024.  The forward plan
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
template <> struct PlanFor<96, 0> { using Fwd = Radices<16, 3, 2>; using Inv = Radices<2, 3, 16>; };
template <> struct PlanFor<128, 0> { using Fwd = Radices<16, 8>; using Inv = Radices<8, 16>; };
template <> struct PlanFor<192, 0> { using Fwd = Radices<16, 3, 4>; using Inv = Radices<4, 3, 16>; };
template <> struct PlanFor<256, 0> { using Fwd = Radices<16, 16>; using Inv = Radices<16, 16>; };
template <> struct PlanFor<384, 0> { using Fwd = Radices<16, 3, 8>; using Inv = Radices<8, 3, 16>; };
template <> struct PlanFor<512, 0> { using Fwd = Radices<16, 2, 16>; using Inv = Radices<16, 2, 16>; };
template <> struct PlanFor<768, 0> { using Fwd = Radices<16, 3, 16>; using Inv = Radices<16, 3, 16>; };
template <> struct PlanFor<1024, 0> { using Fwd = Radices<16, 4, 16>; using Inv = Radices<16, 4, 16>; };

// Family 1: radix 32 first, one stage fewer (one LDS exchange fewer per
// transform) where P allows it.
template <int P> constexpr bool has_fam1() { return P == 512 || P == 1024; }
template <> struct PlanFor<512, 1> { using Fwd = Radices<32, 16>; using Inv = Radices<16, 32>; };
template <> struct PlanFor<1024, 1> { using Fwd = Radices<32, 32>; using Inv = Radices<32, 32>; };

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
