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

template <int P> struct PlanFor;
template <> struct PlanFor<16> { using Fwd = Radices<16>; using Inv = Radices<16>; };
template <> struct PlanFor<32> { using Fwd = Radices<16, 2>; using Inv = Radices<2, 16>; };
template <> struct PlanFor<48> { using Fwd = Radices<16, 3>; using Inv = Radices<3, 16>; };
template <> struct PlanFor<64> { using Fwd = Radices<16, 4>; using Inv = Radices<4, 16>; };
template <> struct PlanFor<96> { using Fwd = Radices<16, 3, 2>; using Inv = Radices<2, 3, 16>; };
template <> struct PlanFor<128> { using Fwd = Radices<16, 8>; using Inv = Radices<8, 16>; };
template <> struct PlanFor<192> { using Fwd = Radices<16, 3, 4>; using Inv = Radices<4, 3, 16>; };
template <> struct PlanFor<256> { using Fwd = Radices<16, 16>; using Inv = Radices<16, 16>; };
template <> struct PlanFor<384> { using Fwd = Radices<16, 3, 8>; using Inv = Radices<8, 3, 16>; };
template <> struct PlanFor<512> { using Fwd = Radices<16, 2, 16>; using Inv = Radices<16, 2, 16>; };
template <> struct PlanFor<768> { using Fwd = Radices<16, 3, 16>; using Inv = Radices<16, 3, 16>; };
template <> struct PlanFor<1024> { using Fwd = Radices<16, 4, 16>; using Inv = Radices<16, 4, 16>; };

// Threads for B pencils of length P at ~16 elements per thread, whole waves.
constexpr int threads_for(int B, int P)
{
    int t = B * P / 16;
    t = (t + 63) / 64 * 64;
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return t;
}

// Apply F<P>() for the runtime P; returns false if P is not supported.
template <template <int> class F, class... A> bool dispatch_p(int P, A&&... a)
{
    switch (P) {
    case 16: F<16>::run(a...); return true;
    case 32: F<32>::run(a...); return true;
    case 48: F<48>::run(a...); return true;
    case 64: F<64>::run(a...); return true;
    case 96: F<96>::run(a...); return true;
    case 128: F<128>::run(a...); return true;
    case 192: F<192>::run(a...); return true;
    case 256: F<256>::run(a...); return true;
    case 384: F<384>::run(a...); return true;
    case 512: F<512>::run(a...); return true;
    case 768: F<768>::run(a...); return true;
    case 1024: F<1024>::run(a...); return true;
    default: return false;
    }
}

}  // namespace ps
