// Launchers of the transformed-kernel build, every supported P.
#include <vector>

#include "k_green.hpp"
#include "ps_internal.hpp"

namespace ps {

template <int P> static hipError_t green_passes(const GreenBufs& b)
{
    constexpr int N = P / 2, H = N + 1;
    constexpr int NT = threads_for(8, P);
    const double2* tw = static_cast<const double2*>(b.twf64);
    const dim3 grid((H + 15) / 16, H);
    hipLaunchKernelGGL((k_green_x<P, NT, MAP_EF>), grid, dim3(NT), 0, b.stream, b.g1, tw, b.dx, b.sy, b.sz,
                       b.self_value);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_green_y<P, NT, MAP_EF>), grid, dim3(NT), 0, b.stream, b.g1, tw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.out_f32) {
        if (b.plain_layout)
            hipLaunchKernelGGL((k_green_z<float, P, NT, MAP_EF, true>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<float*>(b.ghat), tw, b.scale);
        else
            hipLaunchKernelGGL((k_green_z<float, P, NT, MAP_EF, false>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<float*>(b.ghat), tw, b.scale);
    } else {
        if (b.plain_layout)
            hipLaunchKernelGGL((k_green_z<double, P, NT, MAP_EF, true>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<double*>(b.ghat), tw, b.scale);
        else
            hipLaunchKernelGGL((k_green_z<double, P, NT, MAP_EF, false>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<double*>(b.ghat), tw, b.scale);
    }
    return hipGetLastError();
}

hipError_t green_run(int P, const GreenBufs& b)
{
    switch (P) {
#define PS_CASE(PP) \
    case PP: return green_passes<PP>(b);
        PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
    default: return hipErrorInvalidValue;
    }
}

template <class RP> static void rlist(std::vector<int>& v) { v.assign(RP::r, RP::r + RP::S); }

bool has_family1(int P) { return P == 512 || P == 1024; }

bool host_radices(int P, std::vector<int>& fwd, int fam)
{
    if (fam == 1 && has_family1(P)) {
        if (P == 512) rlist<PlanFor<512, 1>::Fwd>(fwd);
        else rlist<PlanFor<1024, 1>::Fwd>(fwd);
        return true;
    }
    switch (P) {
#define PS_CASE(PP) \
    case PP: rlist<PlanFor<PP>::Fwd>(fwd); return true;
        PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
    default: return false;
    }
}

}  // namespace ps
