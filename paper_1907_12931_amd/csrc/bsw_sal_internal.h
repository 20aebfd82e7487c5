// bsw_sal_internal.h -- types shared by the suffix-array lookup's host code
// (bsw_sal.cpp) and its kernels (bsw_sal_kernels.hip).  Not exported.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bsw.h"

namespace bsw {

// Status of one lookup call.
struct SalStatus {
  uint32_t bad;       // some interval leaves the suffix array
  uint32_t too_big;   // the total exceeds the caller's capacity
  unsigned long long first_bad_inv;  // ~(first bad interval); 0 = none
  unsigned long long total;          // coordinates the call produces
};

constexpr int SCAN_TILE = 2048;  // intervals per block of the offset scan
constexpr int SAL_TILE = 256;    // output slots per tile of the gather (one block)

void launch_iv_check(const bsw_sa_interval* iv, int64_t n, uint64_t sa_len, uint64_t* cnt,
                     SalStatus* st, hipStream_t s);
// exclusive scan of cnt[0..n) into off[0..n], off[n] = total; part holds
// one entry per SCAN_TILE elements
void launch_offset_scan(const uint64_t* cnt, int64_t n, uint64_t* part, uint64_t* off,
                        hipStream_t s);
void launch_sal_total(const uint64_t* off, int64_t n, uint64_t cap, SalStatus* st,
                      hipStream_t s);
// tile_start holds ceil(cap / SAL_TILE) entries
void launch_tile_map(const uint64_t* off, int64_t n, const SalStatus* st, int64_t* tile_start,
                     hipStream_t s);
void launch_sal_gather(const int64_t* sa, const bsw_sa_interval* iv, const uint64_t* off,
                       int64_t n, const int64_t* tile_start, const SalStatus* st,
                       uint64_t* out_off, int64_t* out_pos, unsigned blocks, hipStream_t s);

}  // namespace bsw
