// Persistent batched launches, single precision with split-bf16 matrix-core DFT-16.
#include "k_batched.hpp"
#include "launch_batched.hpp"

namespace ps {
hipError_t batched_run_split(const BatchArgs& a)
{
    return a.pmax > 256 ? batched_launch<float, 1024, 1024, 6>(a) : batched_launch<float, 256, 256, 6>(a);
}
}  // namespace ps
