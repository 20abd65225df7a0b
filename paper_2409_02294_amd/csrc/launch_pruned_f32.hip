// Pruned pipeline, single precision on the vector ALUs.
#include "launch_pruned.hpp"
namespace ps {
hipError_t pruned_run_f32(int lo, int hi, const PrunedBufs& b) { return pruned_dispatch<float, 0>(lo, hi, b); }
}  // namespace ps
