// bsw_lanev_x.hip -- instantiations of the register-row lane kernel for
// query caps 256.
#include "bsw_lanev_impl.h"

namespace bsw {

template <> LaneVFn lanev_kernel<256>(bool sym) {
  return sym ? k_lanev<256, true> : k_lanev<256, false>;
}

}  // namespace bsw
