// Launchers of the transformed-kernel build, every supported P.
#include <vector>

#include "k_green.hpp"
#include "ps_internal.hpp"

namespace ps {

template <int P> static void green_x(const GreenBufs& b)
{
    constexpr int NT = threads_for(8, P);
    const int hy = b.ny + 1, hz = b.nz + 1;
    hipLaunchKernelGGL((k_green_x<P, NT, MAP_EF>), dim3((hy + 15) / 16, hz), dim3(NT), 0, b.stream, b.g1,
                       static_cast<const double2*>(b.twf64[0]), hy, hz, b.dx, b.sy, b.sz, b.self_value);
}

template <int P> static void green_y(const GreenBufs& b)
{
    constexpr int NT = threads_for(8, P);
    const int hx = b.nx + 1, hz = b.nz + 1;
    hipLaunchKernelGGL((k_green_y<P, NT, MAP_EF>), dim3((hz + 15) / 16, hx), dim3(NT), 0, b.stream, b.g1,
                       static_cast<const double2*>(b.twf64[1]), hz);
}

template <int P> static void green_z(const GreenBufs& b)
{
    constexpr int NT = threads_for(8, P);
    const int hx = b.nx + 1, hy = b.ny + 1;
    const dim3 grid((hy + 15) / 16, hx);
    const double2* tw = static_cast<const double2*>(b.twf64[2]);
    if (b.out_f32) {
        if (b.plain_layout)
            hipLaunchKernelGGL((k_green_z<float, P, NT, MAP_EF, true>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<float*>(b.ghat), tw, hx, hy, b.scale);
        else
            hipLaunchKernelGGL((k_green_z<float, P, NT, MAP_EF, false>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<float*>(b.ghat), tw, hx, hy, b.scale);
    } else {
        if (b.plain_layout)
            hipLaunchKernelGGL((k_green_z<double, P, NT, MAP_EF, true>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<double*>(b.ghat), tw, hx, hy, b.scale);
        else
            hipLaunchKernelGGL((k_green_z<double, P, NT, MAP_EF, false>), grid, dim3(NT), 0, b.stream, b.g1,
                               static_cast<double*>(b.ghat), tw, hx, hy, b.scale);
    }
}

// The three passes, each on its axis's padded length.
hipError_t green_run(const GreenBufs& b)
{
    for (int axis = 0; axis < 3; ++axis) {
        const int P = 2 * (axis == 0 ? b.nx : axis == 1 ? b.ny : b.nz);
        switch (P) {
#define PS_CASE(PP)                      \
    case PP:                             \
        if (axis == 0) green_x<PP>(b);   \
        else if (axis == 1) green_y<PP>(b); \
        else green_z<PP>(b);             \
        break;
            PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
        default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class RP> static void rlist(std::vector<int>& v) { v.assign(RP::r, RP::r + RP::S); }

bool has_family1(int P)
{
    switch (P) {
#define PS_CASE(PP) \
    case PP: return has_fam1<PP>();
        PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
    default: return false;
    }
}

template <int P> static void rlist1(std::vector<int>& fwd)
{
    if constexpr (has_fam1<P>()) rlist<typename PlanFor<P, 1>::Fwd>(fwd);
}

bool host_radices(int P, std::vector<int>& fwd, int fam)
{
    if (fam == 1 && has_family1(P)) {
        switch (P) {
#define PS_CASE(PP) \
    case PP: rlist1<PP>(fwd); break;
            PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
        default: break;
        }
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
