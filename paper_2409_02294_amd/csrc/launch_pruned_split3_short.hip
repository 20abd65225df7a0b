// Pruned pipeline, single precision with the radix-16 DFTs on the bf16 matrix cores, three product
// terms (the less accurate form): the lengths P <= 480.
#include "launch_pruned.hpp"
namespace ps {
hipError_t pruned_run_split3_short(int lo, int hi, const PrunedBufs& b)
{
    return pruned_dispatch<float, 3, true>(lo, hi, b);
}
}  // namespace ps
