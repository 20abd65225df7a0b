// Launchers of the plain method for float and double, every supported P.
#include "k_plain.hpp"
#include "ps_internal.hpp"

namespace ps {

template <typename T, int P> static hipError_t plain_passes(const PlainBufs& b)
{
    using V = cx<T>;
    constexpr int N = P / 2, H = N + 1;
    constexpr int W = sizeof(T) == 4 ? 16 : 8;  // 128-byte rows of interleaved pencils
    constexpr int NTX = threads_for(8, P);
    constexpr int NTW = threads_for(W, P);
    const V* twf = static_cast<const V*>(b.twf);
    const V* twi = static_cast<const V*>(b.twi);
    T* pad = static_cast<T*>(b.pad);
    V* spec = static_cast<V*>(b.spec);
    const dim3 rows(P / 16, P), cols((H + W - 1) / W, P);
    const int eb = 256, eg = 256 * 8 * 4;  // elementwise kernels: grid-stride over the array
    hipError_t e;
#define PS_CHECK() \
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_plain_pad<T>), dim3(eg), dim3(eb), 0, b.stream, static_cast<const T*>(b.rho), pad, N, P);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_x_r2c<T, P, NTX>), rows, dim3(NTX), 0, b.stream, pad, spec, twf);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_yz<T, P, W, NTW, -1, 1>), cols, dim3(NTW), 0, b.stream, spec, twf);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_yz<T, P, W, NTW, -1, 2>), cols, dim3(NTW), 0, b.stream, spec, twf);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_mul<T>), dim3(eg), dim3(eb), 0, b.stream, spec, static_cast<const T*>(b.ghat), P);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_yz<T, P, W, NTW, +1, 2>), cols, dim3(NTW), 0, b.stream, spec, twi);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_yz<T, P, W, NTW, +1, 1>), cols, dim3(NTW), 0, b.stream, spec, twi);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_x_c2r<T, P, NTX>), rows, dim3(NTX), 0, b.stream, spec, pad, twi);
    PS_CHECK();
    hipLaunchKernelGGL((k_plain_crop<T>), dim3(eg), dim3(eb), 0, b.stream, pad, static_cast<T*>(b.phi), N, P);
    PS_CHECK();
#undef PS_CHECK
    return hipSuccess;
}

template <typename T> static hipError_t plain_dispatch(int P, const PlainBufs& b)
{
    switch (P) {
#define PS_CASE(PP) \
    case PP: return plain_passes<T, PP>(b);
        PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t plain_run_f32(int P, const PlainBufs& b) { return plain_dispatch<float>(P, b); }
hipError_t plain_run_f64(int P, const PlainBufs& b) { return plain_dispatch<double>(P, b); }

}  // namespace ps
