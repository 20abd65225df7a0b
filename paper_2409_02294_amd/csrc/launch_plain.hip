// Launchers of the plain method (filled in by the plain-method kernels).
#include "ps_internal.hpp"

namespace ps {

hipError_t plain_run_f32(int, const PlainBufs&) { return hipErrorNotSupported; }
hipError_t plain_run_f64(int, const PlainBufs&) { return hipErrorNotSupported; }

}  // namespace ps
