// Pruned pipeline, single precision with the radix-16 DFTs on the bf16 matrix cores, six product
// terms: the lengths P <= 480.
#include "launch_pruned.hpp"
namespace ps {
hipError_t pruned_run_split6_short(int lo, int hi, const PrunedBufs& b)
{
    return pruned_dispatch<float, 6, true>(lo, hi, b);
}
}  // namespace ps
