// Strip kernel placeholder: replaced by the r-marching register-ring kernel.
#include "common.h"
#include "launch.h"

namespace pclb {

template <class R>
bool strip_supported(const Tables&) { return false; }

template <class R>
hipError_t launch_step_strip(const Tables&, const void*, void*, const void*, int, hipStream_t) {
  return hipErrorNotSupported;
}

template bool strip_supported<float>(const Tables&);
template bool strip_supported<double>(const Tables&);
template hipError_t launch_step_strip<float>(const Tables&, const void*, void*, const void*, int, hipStream_t);
template hipError_t launch_step_strip<double>(const Tables&, const void*, void*, const void*, int, hipStream_t);

}  // namespace pclb
