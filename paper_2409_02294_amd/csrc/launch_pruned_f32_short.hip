// Pruned pipeline, single precision on the vector ALUs: the lengths P <= 480.
#include "launch_pruned.hpp"
namespace ps {
hipError_t pruned_run_f32_short(int lo, int hi, const PrunedBufs& b)
{
    return pruned_dispatch<float, 0, true>(lo, hi, b);
}
}  // namespace ps
