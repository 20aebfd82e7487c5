// bsw_lanev_s.hip -- instantiations of the register-row lane kernel for
// query caps 32, 64, 96, 128.
#include "bsw_lanev_impl.h"

namespace bsw {

template <> LaneVFn lanev_kernel<32>(bool sym) {
  return sym ? k_lanev<32, true> : k_lanev<32, false>;
}

template <> LaneVFn lanev_kernel<64>(bool sym) {
  return sym ? k_lanev<64, true> : k_lanev<64, false>;
}

template <> LaneVFn lanev_kernel<96>(bool sym) {
  return sym ? k_lanev<96, true> : k_lanev<96, false>;
}

template <> LaneVFn lanev_kernel<128>(bool sym) {
  return sym ? k_lanev<128, true> : k_lanev<128, false>;
}

}  // namespace bsw
