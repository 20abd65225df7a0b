// Pruned pipeline, double precision on the vector ALUs: the lengths P > 480.
#include "launch_pruned.hpp"
namespace ps {
hipError_t pruned_run_f64_long(int lo, int hi, const PrunedBufs& b)
{
    return pruned_dispatch<double, 0, false>(lo, hi, b);
}
}  // namespace ps
