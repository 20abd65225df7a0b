// Pruned pipeline, double precision.
#include "launch_pruned.hpp"
namespace ps {
hipError_t pruned_run_f64(int lo, int hi, const PrunedBufs& b) { return pruned_dispatch<double, 0>(lo, hi, b); }
}  // namespace ps
