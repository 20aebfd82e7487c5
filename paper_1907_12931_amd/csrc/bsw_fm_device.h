// bsw_fm_device.h -- device-side FM-index steps shared by the kernels of
// bsw_fm_kernels.hip: the occurrence counts of one entry (Algorithm 1) and
// the bi-interval extensions (Algorithms 2 and 3).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/bsw.h"

namespace bsw {

// The two counts one extension by base c needs, from one entry: O(c, t),
// and the occurrences in B[0 .. t] of the bases after c (c < d <= 3).
// Symbols are bytes 0..5; a byte equals c exactly when x = byte ^ c is zero
// (the test above), and exceeds c exactly when byte + 0x7f - c has its top
// bit set (no sum passes 0xff, so no carry crosses bytes); bytes above 3
// ($ and past the end) are taken out with the same test for 3.
__device__ __forceinline__ void occ_eq_gt(const bsw_fm_entry* __restrict__ E, int64_t t,
                                          uint32_t c, uint32_t& eq, uint32_t& gt) {
  if (t < 0) {
    eq = gt = 0;
    return;
  }
  const uint4* p = (const uint4*)(E + (t >> 5));
  const uint4 cnt = p[0], b0 = p[1], b1 = p[2];
  const uint32_t w[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
  const int y = (int)(t & 31);
  const uint32_t rep_c = 0x01010101u * c;
  const uint32_t add_c = 0x01010101u * (0x7fu - c);
  uint32_t ne = 0, ng = 0;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int r = y - 4 * d;  // last byte of this dword that is counted
    const uint32_t keep = r < 0 ? 0u : (r >= 3 ? 0x80808080u : 0x80808080u >> (8 * (3 - r)));
    const uint32_t x = w[d] ^ rep_c;
    const uint32_t nonzero = (((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
    ne += (uint32_t)__popc(~nonzero & keep);
    const uint32_t above_c = (w[d] + add_c) & 0x80808080u;
    const uint32_t above_3 = (w[d] + 0x7c7c7c7cu) & 0x80808080u;
    ng += (uint32_t)__popc(above_c & ~above_3 & keep);
  }
  eq = (c == 0 ? cnt.x : c == 1 ? cnt.y : c == 2 ? cnt.z : cnt.w) + ne;
  gt = (c < 1 ? cnt.y : 0u) + (c < 2 ? cnt.z : 0u) + (c < 3 ? cnt.w : 0u) + ng;
}

// Backward extension (Algorithm 2): the bi-interval of cX from that of X.
// The reverse complement's rows: after the row ending in $ (when X's rows
// hold the whole text's row) come the extensions of revcomp(X) by A, C, G,
// T, i.e. of X by T, G, C, A on the left; so base c's l skips the sizes of
// the bases after c.
__device__ __forceinline__ void back_ext(const bsw_fm_entry* __restrict__ E,
                                         const bsw_fm_meta& meta, uint64_t k, uint64_t l,
                                         uint64_t s, uint32_t c, uint64_t& k2, uint64_t& l2,
                                         uint64_t& s2) {
  uint32_t lo_eq, lo_gt, hi_eq, hi_gt;
  occ_eq_gt(E, (int64_t)k - 1, c, lo_eq, lo_gt);
  occ_eq_gt(E, (int64_t)(k + s) - 1, c, hi_eq, hi_gt);
  const uint64_t Cc = c == 0 ? meta.C[0] : c == 1 ? meta.C[1] : c == 2 ? meta.C[2] : meta.C[3];
  k2 = Cc + lo_eq;
  l2 = l + (k <= meta.primary && meta.primary < k + s ? 1 : 0) + (hi_gt - lo_gt);
  s2 = hi_eq - lo_eq;
}

// Forward extension (Algorithm 3): Xc from X, by extending revcomp(X) on
// the left with the complement of c and swapping the two strands.
__device__ __forceinline__ void fwd_ext(const bsw_fm_entry* __restrict__ E,
                                        const bsw_fm_meta& meta, uint64_t k, uint64_t l,
                                        uint64_t s, uint32_t c, uint64_t& k2, uint64_t& l2,
                                        uint64_t& s2) {
  back_ext(E, meta, l, k, s, 3 - c, l2, k2, s2);
}

// The same steps with 32-bit rows (an index built by bsw_fm_build has fewer
// than 2^32 rows, so k + s never wraps): fewer registers per lane.
struct FmRows32 {
  uint32_t C0, C1, C2, C3, primary, rows;
};

__device__ __forceinline__ void back_ext32(const bsw_fm_entry* __restrict__ E,
                                           const FmRows32& m, uint32_t k, uint32_t l,
                                           uint32_t s, uint32_t c, uint32_t& k2, uint32_t& l2,
                                           uint32_t& s2) {
  uint32_t lo_eq, lo_gt, hi_eq, hi_gt;
  occ_eq_gt(E, (int64_t)k - 1, c, lo_eq, lo_gt);
  occ_eq_gt(E, (int64_t)(k + s) - 1, c, hi_eq, hi_gt);
  const uint32_t Cc = c == 0 ? m.C0 : c == 1 ? m.C1 : c == 2 ? m.C2 : m.C3;
  k2 = Cc + lo_eq;
  l2 = l + (k <= m.primary && m.primary < k + s ? 1u : 0u) + (hi_gt - lo_gt);
  s2 = hi_eq - lo_eq;
}

__device__ __forceinline__ void fwd_ext32(const bsw_fm_entry* __restrict__ E,
                                          const FmRows32& m, uint32_t k, uint32_t l,
                                          uint32_t s, uint32_t c, uint32_t& k2, uint32_t& l2,
                                          uint32_t& s2) {
  back_ext32(E, m, l, k, s, 3 - c, l2, k2, s2);
}

}  // namespace bsw
