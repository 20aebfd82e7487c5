// bsw_lanev_m.hip -- instantiations of the register-row lane kernel for
// query caps 160, 192.
#include "bsw_lanev_impl.h"

namespace bsw {

template <> LaneVFn lanev_kernel<160>(bool sym) {
  return sym ? k_lanev<160, true> : k_lanev<160, false>;
}

template <> LaneVFn lanev_kernel<192>(bool sym) {
  return sym ? k_lanev<192, true> : k_lanev<192, false>;
}

}  // namespace bsw
