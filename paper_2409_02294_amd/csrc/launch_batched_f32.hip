// Persistent batched launches, single precision.
#include "k_batched.hpp"
#include "launch_batched.hpp"

namespace ps {
hipError_t batched_run_f32(const BatchArgs& a)
{
    return a.pmax > 256 ? batched_launch<float, 1024, 1024, 0>(a) : batched_launch<float, 256, 256, 0>(a);
}
}  // namespace ps
