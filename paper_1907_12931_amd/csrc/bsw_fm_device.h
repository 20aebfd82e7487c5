// bsw_fm_device.h -- device-side FM-index steps shared by the kernels of
// bsw_fm_kernels.hip: O(c, t) (Algorithm 1) and the bi-interval extensions
// (Algorithms 2 and 3).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/bsw.h"

namespace bsw {

// O(c, t) for the four bases at once (Algorithm 1): the entry's counts plus
// the occurrences among its first t % 32 + 1 symbols.  A byte of x is zero
// exactly when ((x & 0x7f) + 0x7f) | x has its top bit clear (no carry
// crosses bytes), so each dword yields exact per-byte matches.
__device__ __forceinline__ void occ4(const bsw_fm_entry* __restrict__ E, int64_t t,
                                     uint32_t o[4]) {
  if (t < 0) {
    o[0] = o[1] = o[2] = o[3] = 0;
    return;
  }
  const uint4* p = (const uint4*)(E + (t >> 5));
  const uint4 cnt = p[0], b0 = p[1], b1 = p[2];
  const uint32_t w[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
  const int y = (int)(t & 31);
  uint32_t n[4] = {0, 0, 0, 0};
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int r = y - 4 * d;  // last byte of this dword that is counted
    const uint32_t keep = r < 0 ? 0u : (r >= 3 ? 0x80808080u : 0x80808080u >> (8 * (3 - r)));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t x = w[d] ^ (0x01010101u * (uint32_t)c);
      const uint32_t nonzero = (((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
      n[c] += (uint32_t)__popc(~nonzero & keep);
    }
  }
  o[0] = cnt.x + n[0];
  o[1] = cnt.y + n[1];
  o[2] = cnt.z + n[2];
  o[3] = cnt.w + n[3];
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
  uint32_t lo[4], hi[4];
  occ4(E, (int64_t)k - 1, lo);
  occ4(E, (int64_t)(k + s) - 1, hi);
  // constant indices only (a runtime index would put the arrays in memory)
  const uint32_t s0 = hi[0] - lo[0], s1 = hi[1] - lo[1], s2_ = hi[2] - lo[2],
                 s3 = hi[3] - lo[3];
  uint64_t nl = l + (k <= meta.primary && meta.primary < k + s ? 1 : 0);
  nl += (c < 3 ? s3 : 0u) + (c < 2 ? s2_ : 0u) + (c < 1 ? s1 : 0u);
  const uint32_t loc = c == 0 ? lo[0] : c == 1 ? lo[1] : c == 2 ? lo[2] : lo[3];
  const uint64_t Cc = c == 0 ? meta.C[0] : c == 1 ? meta.C[1] : c == 2 ? meta.C[2] : meta.C[3];
  k2 = Cc + loc;
  l2 = nl;
  s2 = c == 0 ? s0 : c == 1 ? s1 : c == 2 ? s2_ : s3;
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
// than 2^32 rows, so k + s never wraps): fewer registers per lane.  tp1 is
// t + 1 (0 for t = -1).
__device__ __forceinline__ void occ4_32(const bsw_fm_entry* __restrict__ E, uint32_t tp1,
                                        uint32_t o[4]) {
  if (tp1 == 0) {
    o[0] = o[1] = o[2] = o[3] = 0;
    return;
  }
  occ4(E, (int64_t)(tp1 - 1), o);
}

struct FmRows32 {
  uint32_t C0, C1, C2, C3, primary, rows;
};

__device__ __forceinline__ void back_ext32(const bsw_fm_entry* __restrict__ E,
                                           const FmRows32& m, uint32_t k, uint32_t l,
                                           uint32_t s, uint32_t c, uint32_t& k2, uint32_t& l2,
                                           uint32_t& s2) {
  uint32_t lo[4], hi[4];
  occ4_32(E, k, lo);
  occ4_32(E, k + s, hi);
  const uint32_t s0 = hi[0] - lo[0], s1 = hi[1] - lo[1], s2_ = hi[2] - lo[2],
                 s3 = hi[3] - lo[3];
  uint32_t nl = l + (k <= m.primary && m.primary < k + s ? 1u : 0u);
  nl += (c < 3 ? s3 : 0u) + (c < 2 ? s2_ : 0u) + (c < 1 ? s1 : 0u);
  const uint32_t loc = c == 0 ? lo[0] : c == 1 ? lo[1] : c == 2 ? lo[2] : lo[3];
  const uint32_t Cc = c == 0 ? m.C0 : c == 1 ? m.C1 : c == 2 ? m.C2 : m.C3;
  k2 = Cc + loc;
  l2 = nl;
  s2 = c == 0 ? s0 : c == 1 ? s1 : c == 2 ? s2_ : s3;
}

__device__ __forceinline__ void fwd_ext32(const bsw_fm_entry* __restrict__ E,
                                          const FmRows32& m, uint32_t k, uint32_t l,
                                          uint32_t s, uint32_t c, uint32_t& k2, uint32_t& l2,
                                          uint32_t& s2) {
  back_ext32(E, m, l, k, s, 3 - c, l2, k2, s2);
}

}  // namespace bsw
