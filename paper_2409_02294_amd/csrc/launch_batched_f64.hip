// Persistent batched launches, double precision.
#include "k_batched.hpp"
#include "launch_batched.hpp"

namespace ps {
hipError_t batched_run_f64(const BatchArgs& a)
{
    return a.pmax > 256 ? batched_launch<double, 1024, 512, 0>(a) : batched_launch<double, 256, 256, 0>(a);
}
}  // namespace ps
