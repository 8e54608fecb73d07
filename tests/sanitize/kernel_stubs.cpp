// Host-only stand-ins for the kernel launch functions of the library, so that
// the planner and the C ABI can be built with the host compiler alone (under
// AddressSanitizer and UndefinedBehaviorSanitizer).  A host-only context never
// launches: each stand-in reports an error if it is ever reached.
#include "../../paper_2106_15740_amd/csrc/kernels.hpp"

namespace qtn {

hipError_t launch_op(bool, const OpDesc*, const OpDesc&, int, const Env&, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_batch(bool, bool, int, const OpDesc*, int, int, const Env&, hipStream_t, int32_t*, const int32_t*, int) {
  return hipErrorNotSupported;
}
hipError_t launch_small_copy(const void*, void*, size_t, hipStream_t, int32_t*, const int32_t*, int) {
  return hipErrorNotSupported;
}
hipError_t launch_copy(const void*, void*, size_t, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reset(int32_t*, const int32_t*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_persistent(bool, bool, int, const OpDesc*, const QItem*, int, const int32_t*, int32_t*, const Env&,
                             int, int, size_t, long long, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_small(bool, const SmallOp*, const int32_t*, int, const Env&, int, size_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t scratch_address(int, void**) { return hipErrorNotSupported; }
hipError_t launch_final(bool, const double*, int, int, int, int, void*, double*, double*, const int32_t*, int32_t*,
                        hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace qtn
