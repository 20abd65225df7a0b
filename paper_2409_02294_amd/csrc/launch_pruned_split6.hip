// Pruned pipeline, single precision with the radix-16 DFTs on the bf16 matrix
// cores: split operands, six product terms.
#include "launch_pruned.hpp"
namespace ps {
hipError_t pruned_run_split6(int lo, int hi, const PrunedBufs& b) { return pruned_dispatch<float, 6>(lo, hi, b); }
}  // namespace ps
