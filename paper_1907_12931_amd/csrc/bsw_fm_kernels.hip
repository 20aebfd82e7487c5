// bsw_fm_kernels.hip -- FM-index backward search (Sec. 4.1-4.2): every
// pattern is extended from its last base to its first by the bi-interval
// update (Algorithm 2), reading O(c, t) from 64-byte bucket entries
// (Algorithm 1, the layout of Sec. 4.4).  One pattern per lane: the steps of
// a pattern depend on each other, and the lanes of a wave, with many waves
// per CU, keep enough entry reads in flight to hide their latency (the
// many-queries-at-once form that Sec. 4.3 tried on the CPU).
//   k_fm_check   per pattern: its offsets are ordered
//   k_fm_search  the search, one pattern per lane
//   k_smem_check per read: offsets ordered, length within the list capacity
//   k_fm_smem    the SMEMs of every read (Algorithms 3 and 4 around each
//                pivot, the pivot moving to the end of the longest forward
//                match), one read per lane, the interval lists of the lanes
//                interleaved in scratch memory
#include <hip/hip_runtime.h>

#include "../../include/bsw.h"
#include "bsw_fm_device.h"
#include "bsw_internal.h"

namespace bsw {

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
      uint64_t k2, l2, s2;
      back_ext(E, meta, k, l, s, c, k2, l2, s2);
      if (s2 == 0) break;
      k = k2;
      l = l2;
      s = s2;
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

__global__ void __launch_bounds__(256)
k_smem_check(const uint64_t* __restrict__ off, int64_t n, uint32_t cap, Status* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += stride)
    if (off[m + 1] < off[m] || off[m + 1] - off[m] > cap) {
      atomicMax(&st->first_bad_inv, ~(unsigned long long)m);
      atomicOr(&st->bad, 1u);
    }
}

namespace {
struct ListEnt {  // a bi-interval (32-bit rows) and the read end of its match
  uint32_t k, l, s, end;
};
}  // namespace

// Per read: pivot x = 0; the SMEMs through x are found by extending X[x]
// forward while it occurs, keeping the bi-interval each time its size
// changes (the matches X[x, e) for every e where the occurrences change),
// then extending those matches backward base by base, longest first: a match
// that cannot grow to the left is a maximal match starting at the current
// position, super-maximal when no longer match failed at the same position
// and no match already kept starts there; among matches whose extensions
// have equal sizes only the longest is kept.  The next pivot is the end of
// the longest forward match.  Output: the read's SMEMs in order of start at
// out[off[r] - off[0] ...], their number in counts[r]; steps counts the
// extension steps (two index entries read each).
__global__ void __launch_bounds__(256)
k_fm_smem(const bsw_fm_entry* __restrict__ E, bsw_fm_meta meta,
          const uint8_t* __restrict__ reads, const uint64_t* __restrict__ off, int64_t n,
          uint32_t cap, ListEnt* __restrict__ scratch, Status* st, bsw_smem* __restrict__ out,
          int32_t* __restrict__ counts) {
  if (st->bad) return;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t G = (int64_t)gridDim.x * blockDim.x;
  // entry j of list b of this lane: the lanes' entries sit side by side, so
  // the lanes of a wave that touch their entry j at once share lines
#define LIST(b, j) scratch[((size_t)(b) * cap + (size_t)(j)) * (size_t)G + (size_t)g]
  const uint64_t base = off[0];
  const FmRows32 m32 = {(uint32_t)meta.C[0], (uint32_t)meta.C[1], (uint32_t)meta.C[2],
                        (uint32_t)meta.C[3], (uint32_t)meta.primary, (uint32_t)meta.rows};
  unsigned long long steps = 0;  // this lane's extension steps
  for (int64_t r = g; r < n; r += G) {
    const uint8_t* X = reads + off[r];
    const int L = (int)(off[r + 1] - off[r]);
    bsw_smem* o = out + (off[r] - base);
    int cnt = 0;
    int x = 0;
    while (x < L) {
      uint32_t c = X[x];
      if (c > 3) {
        ++x;
        continue;
      }
      // forward (Algorithm 3) from the single base at x
      uint32_t k = c == 0 ? m32.C0 : c == 1 ? m32.C1 : c == 2 ? m32.C2 : m32.C3;
      uint32_t l = c == 0 ? m32.C3 : c == 1 ? m32.C2 : c == 2 ? m32.C1 : m32.C0;
      uint32_t s = (c == 0 ? m32.C1 : c == 1 ? m32.C2 : c == 2 ? m32.C3 : m32.rows) - k;
      uint32_t end = (uint32_t)x + 1;
      int cur = 0;  // list ids: 0 and 1
      int ncur = 0;
      int i = x + 1;
      for (; i < L; ++i) {
        c = X[i];
        if (c > 3) {
          LIST(cur, ncur++) = {k, l, s, end};
          break;
        }
        uint32_t k2, l2, s2;
        fwd_ext32(E, m32, k, l, s, c, k2, l2, s2);
        ++steps;
        if (s2 != s) LIST(cur, ncur++) = {k, l, s, end};
        if (s2 == 0) break;
        k = k2;
        l = l2;
        s = s2;
        end = (uint32_t)i + 1;
      }
      if (i == L) LIST(cur, ncur++) = {k, l, s, end};
      const int next = (int)LIST(cur, ncur - 1).end;
      // backward (Algorithm 4), longest forward match first
      int prev = 1;
      int nprev = ncur;
      for (int j = 0; j < ncur; ++j) LIST(prev, j) = LIST(0, ncur - 1 - j);
      cur = 0;
      const int first = cnt;
      for (int ii = x - 1;; --ii) {
        const int cc = ii >= 0 && X[ii] < 4 ? (int)X[ii] : -1;
        ncur = 0;
        for (int j = 0; j < nprev; ++j) {
          const ListEnt p = LIST(prev, j);
          uint32_t k2 = 0, l2 = 0, s2 = 0;
          if (cc >= 0) {
            back_ext32(E, m32, p.k, p.l, p.s, (uint32_t)cc, k2, l2, s2);
            ++steps;
          }
          if (cc < 0 || s2 == 0) {
            if (ncur == 0 && (cnt == first || ii + 1 < (int)o[cnt - 1].start) && cnt < L)
              o[cnt++] = {(uint32_t)(ii + 1), p.end, (uint64_t)p.k, (uint64_t)p.l, (uint64_t)p.s};
          } else if (ncur == 0 || s2 != LIST(cur, ncur - 1).s) {
            LIST(cur, ncur++) = {k2, l2, s2, p.end};
          }
        }
        if (ncur == 0) break;
        const int t = prev;
        prev = cur;
        cur = t;
        nprev = ncur;
      }
      // this pivot's SMEMs came out longest first, i.e. by decreasing start
      for (int a = first, b = cnt - 1; a < b; ++a, --b) {
        const bsw_smem t = o[a];
        o[a] = o[b];
        o[b] = t;
      }
      x = next;
    }
    counts[r] = cnt;
  }
  // one atomic per wave (every lane of the wave gets here)
  for (int d = 32; d > 0; d >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)steps, d, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(steps >> 32), d, 64);
    steps += ((unsigned long long)hi << 32) | lo;
  }
  if ((threadIdx.x & 63) == 0) atomicAdd(&st->cls_cells[0], steps);
#undef LIST
}

void launch_smem_check(const uint64_t* off, int64_t n, uint32_t cap, Status* st,
                       hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_smem_check, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, off, n,
                     cap, st);
}

size_t smem_list_entry_bytes() { return sizeof(ListEnt); }

int fm_smem_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_fm_smem, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    b = 1;
  }
  return b < 1 ? 1 : b;
}

void launch_fm_smem(const bsw_fm_entry* E, const bsw_fm_meta& meta, const uint8_t* reads,
                    const uint64_t* off, int64_t n, uint32_t cap, void* scratch,
                    unsigned blocks, Status* st, bsw_smem* out, int32_t* counts,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_fm_smem, dim3(blocks), dim3(256), 0, s, E, meta, reads, off, n, cap,
                     (ListEnt*)scratch, st, out, counts);
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
