// bsw_lanev_l.hip -- instantiations of the register-row lane kernel for
// query caps 224.
#include "bsw_lanev_impl.h"

namespace bsw {

template <> LaneVFn lanev_kernel<224>(bool sym) {
  return sym ? k_lanev<224, true> : k_lanev<224, false>;
}

}  // namespace bsw
