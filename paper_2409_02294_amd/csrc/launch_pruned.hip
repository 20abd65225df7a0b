// Launchers of the pruned pipeline for float and double, every supported P.
#include "k_pruned.hpp"
#include "ps_internal.hpp"

namespace ps {

template <typename T> struct PrunedShape {
    static constexpr int ZT = sizeof(T) == 4 ? 16 : 8;  // y-pass tile: 128-byte rows of interleaved pencils
    static constexpr int ZB = 4;                        // pencils per z-pass workgroup
};

template <typename T, int P> static hipError_t pruned_passes(int lo, int hi, const PrunedBufs& b)
{
    using V = cx<T>;
    constexpr int N = P / 2, H = N + 1;
    constexpr int ZT = PrunedShape<T>::ZT, ZB = PrunedShape<T>::ZB;
    constexpr int NTX = threads_for(8, P);
    constexpr int NTY = threads_for(ZT, P);
    constexpr int NTZ = threads_for(ZB, P);
    const V* twf = static_cast<const V*>(b.twf);
    const V* twi = static_cast<const V*>(b.twi);
    for (int pass = lo; pass < hi; ++pass) {
        switch (pass) {
        case 0:
            hipLaunchKernelGGL((k_x_r2c<T, P, NTX, MAP_EF>), dim3((N + 15) / 16, N), dim3(NTX), 0, b.stream,
                               static_cast<const T*>(b.rho), static_cast<V*>(b.t1), twf);
            break;
        case 1:
            hipLaunchKernelGGL((k_y_fwd<T, P, ZT, NTY, MAP_EF>), dim3((N + ZT - 1) / ZT, H), dim3(NTY), 0, b.stream,
                               static_cast<const V*>(b.t1), static_cast<V*>(b.t2), twf);
            break;
        case 2:
            hipLaunchKernelGGL((k_z_conv<T, P, ZB, NTZ, MAP_EF, MAP_EF>), dim3(P / ZB, H), dim3(NTZ), 0, b.stream,
                               static_cast<V*>(b.t2), static_cast<const T*>(b.ghat), twf, twi);
            break;
        case 3:
            hipLaunchKernelGGL((k_y_inv<T, P, ZT, NTY, MAP_EF>), dim3((N + ZT - 1) / ZT, H), dim3(NTY), 0, b.stream,
                               static_cast<const V*>(b.t2), static_cast<V*>(b.t1), twi);
            break;
        case 4:
            hipLaunchKernelGGL((k_x_c2r<T, P, NTX, MAP_EF>), dim3((N + 15) / 16, N), dim3(NTX), 0, b.stream,
                               static_cast<const V*>(b.t1), static_cast<T*>(b.phi), twi);
            break;
        default:
            return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T> static hipError_t pruned_dispatch(int P, int lo, int hi, const PrunedBufs& b)
{
    switch (P) {
#define PS_CASE(PP) \
    case PP: return pruned_passes<T, PP>(lo, hi, b);
        PS_CASE(16) PS_CASE(32) PS_CASE(48) PS_CASE(64) PS_CASE(96) PS_CASE(128)
        PS_CASE(192) PS_CASE(256) PS_CASE(384) PS_CASE(512) PS_CASE(768) PS_CASE(1024)
#undef PS_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t pruned_run_f32(int P, int lo, int hi, const PrunedBufs& b) { return pruned_dispatch<float>(P, lo, hi, b); }
hipError_t pruned_run_f64(int P, int lo, int hi, const PrunedBufs& b) { return pruned_dispatch<double>(P, lo, hi, b); }

}  // namespace ps
