// bsw_fm_kernels.hip -- FM-index backward search (Sec. 4.1-4.2): every
// pattern is extended from its last base to its first by the bi-interval
// update (Algorithm 2), reading O(c, t) from 64-byte bucket entries
// (Algorithm 1, the layout of Sec. 4.4).  One pattern per lane: the steps of
// a pattern depend on each other, and the lanes of a wave, with many waves
// per CU, keep enough entry reads in flight to hide their latency (the
// many-queries-at-once form that Sec. 4.3 tried on the CPU).
//   k_fm_check   per pattern: its offsets are ordered
//   k_fm_search  the search, one pattern per lane
#include <hip/hip_runtime.h>

#include "../../include/bsw.h"
#include "bsw_internal.h"

namespace bsw {

namespace {

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

}  // namespace

__global__ void __launch_bounds__(256)
k_fm_check(const uint64_t* __restrict__ off, int64_t n, Status* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += stride)
    if (off[m + 1] < off[m]) {
      atomicMax(&st->first_bad_inv, ~(unsigned long long)m);
      atomicOr(&st->bad, 1u);
    }
}

__global__ void __launch_bounds__(256)
k_fm_search(const bsw_fm_entry* __restrict__ E, bsw_fm_meta meta,
            const uint8_t* __restrict__ pat, const uint64_t* __restrict__ off, int64_t n,
            const Status* st, bsw_bi_interval* __restrict__ out) {
  if (st->bad) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += stride) {
    const uint64_t q0 = off[m], q1 = off[m + 1];
    uint64_t k = 0, l = 0, s = meta.rows;  // the empty string: every row
    int32_t matched = 0;
    for (uint64_t i = q1; i > q0; --i) {
      const uint32_t c = pat[i - 1];
      if (c > 3) break;
      uint32_t lo[4], hi[4];
      occ4(E, (int64_t)k - 1, lo);
      occ4(E, (int64_t)(k + s) - 1, hi);
      uint64_t sz[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) sz[d] = hi[d] - lo[d];
      if (sz[c] == 0) break;
      // the reverse complement's rows: after the row ending in $ (when the
      // interval holds the whole text's row) come the extensions by T, G,
      // C, A of X's complement, i.e. by A, C, G, T of the reverse
      uint64_t nl = l + (k <= meta.primary && meta.primary < k + s ? 1 : 0);
      for (int d = 3; d > (int)c; --d) nl += sz[d];
      k = meta.C[c] + lo[c];
      l = nl;
      s = sz[c];
      ++matched;
    }
    bsw_bi_interval r;
    const bool all = (uint64_t)matched == q1 - q0;
    r.k = all ? k : 0;
    r.l = all ? l : 0;
    r.s = all ? s : 0;
    r.matched = matched;
    r.pad_ = 0;
    out[m] = r;
  }
}

void launch_fm_check(const uint64_t* off, int64_t n, Status* st, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_fm_check, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, off, n, st);
}

void launch_fm_search(const bsw_fm_entry* E, const bsw_fm_meta& meta, const uint8_t* pat,
                      const uint64_t* off, int64_t n, const Status* st, bsw_bi_interval* out,
                      hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(k_fm_search, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, E, meta,
                     pat, off, n, st, out);
}

}  // namespace bsw
