// bsw_lanev.h -- the register-row lane kernel (8-bit records, queries up
// to 256 columns): one instantiation per class, built in the translation
// units bsw_lanev_*.hip so that they compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/bsw.h"
#include "bsw_internal.h"

namespace bsw {

typedef void (*LaneVFn)(const PairDesc*, const long long*, const uint8_t*,
                        const uint8_t*, const KParams*, bsw_result*, bsw_diag*,
                        uint32_t*, const Status*, PairDesc*, long long*, int,
                        unsigned long long*, unsigned long long*);

// The kernel of the class with query cap CAP, symmetric gap costs or not.
template <int CAP> LaneVFn lanev_kernel(bool sym);
template <> LaneVFn lanev_kernel<32>(bool sym);
template <> LaneVFn lanev_kernel<64>(bool sym);
template <> LaneVFn lanev_kernel<96>(bool sym);
template <> LaneVFn lanev_kernel<128>(bool sym);
template <> LaneVFn lanev_kernel<160>(bool sym);
template <> LaneVFn lanev_kernel<192>(bool sym);
template <> LaneVFn lanev_kernel<224>(bool sym);
template <> LaneVFn lanev_kernel<256>(bool sym);

}  // namespace bsw
