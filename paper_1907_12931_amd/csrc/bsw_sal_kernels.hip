// bsw_sal_kernels.hip -- suffix-array lookup (Sec. 4.5, Eq. (1)): every row
// i of every SA interval becomes the coordinate S[i], the coordinates of
// all intervals packed back to back.
//   k_iv_check   per interval: inside the suffix array?  its row count
//   k_scan_up    per tile of 2,048 intervals: the sum of their row counts
//   k_scan_mid   one block: exclusive scan of the tile sums
//   k_scan_down  per tile: exclusive scan of the row counts -> offsets
//   k_sal_total  the total against the caller's capacity
//   k_tile_map   per tile of 256 output slots: the interval that holds its
//                first slot (each interval marks the tiles starting in it)
//   k_sal_gather load-balanced gather: a block takes a tile of 256
//                consecutive output slots; the offsets and starts of the
//                intervals between the tile's first interval and the next
//                tile's are staged in LDS (one coalesced load), each thread
//                finds its slot's interval there by binary search and copies
//                S[k + slot - off]; reads of one interval are contiguous,
//                writes are coalesced.
// The work is HBM-bound: 8 bytes read from S and 8 written per coordinate,
// plus the intervals and offsets.
#include <hip/hip_runtime.h>

#include "bsw_sal_internal.h"

namespace bsw {

__global__ void __launch_bounds__(256)
k_iv_check(const bsw_sa_interval* __restrict__ iv, int64_t n, uint64_t sa_len,
           uint64_t* __restrict__ cnt, SalStatus* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += stride) {
    const bsw_sa_interval v = iv[m];
    // at most 2^32 rows each, so that 2^31 intervals cannot wrap the sum
    const bool ok = v.k <= sa_len && v.s <= sa_len - v.k && v.s <= (1ull << 32);
    cnt[m] = ok ? v.s : 0;
    if (!ok) {
      atomicMax(&st->first_bad_inv, ~(unsigned long long)m);
      atomicOr(&st->bad, 1u);
    }
  }
}

namespace {

// Inclusive scan of one value per thread over a block of 256 (LDS).
__device__ __forceinline__ uint64_t block_incl_scan(uint64_t v, uint64_t* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const uint64_t a = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const uint64_t r = sh[t];
  __syncthreads();
  return r;
}

constexpr int PER = SCAN_TILE / 256;  // elements per thread

}  // namespace

__global__ void __launch_bounds__(256)
k_scan_up(const uint64_t* __restrict__ cnt, int64_t n, uint64_t* __restrict__ part) {
  __shared__ uint64_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  uint64_t v = 0;
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + threadIdx.x + 256 * j;
    if (i < n) v += cnt[i];
  }
  const uint64_t tot = block_incl_scan(v, sh);
  if (threadIdx.x == 255) part[blockIdx.x] = tot;
}

// One block: exclusive scan of nb tile sums, in place, 1,024 at a time.
__global__ void __launch_bounds__(1024) k_scan_mid(uint64_t* part, int64_t nb) {
  __shared__ uint64_t sh[1024];
  const int t = threadIdx.x;
  uint64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const uint64_t v = c0 + t < nb ? part[c0 + t] : 0;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const uint64_t a = t >= d ? sh[t - d] : 0;
      __syncthreads();
      sh[t] += a;
      __syncthreads();
    }
    if (c0 + t < nb) part[c0 + t] = carry + sh[t] - v;
    carry += sh[1023];
    __syncthreads();
  }
}

// cnt and off may be the same array: the tile is staged in LDS first.
__global__ void __launch_bounds__(256)
k_scan_down(const uint64_t* cnt, int64_t n, const uint64_t* __restrict__ part,
            uint64_t* off) {
  __shared__ uint64_t tile[SCAN_TILE];
  __shared__ uint64_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + threadIdx.x + 256 * j;
    tile[threadIdx.x + 256 * j] = i < n ? cnt[i] : 0;
  }
  __syncthreads();
  // each thread scans its PER consecutive elements
  uint64_t v = 0;
  for (int j = 0; j < PER; ++j) v += tile[threadIdx.x * PER + j];
  uint64_t run = part[blockIdx.x] + block_incl_scan(v, sh) - v;
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + threadIdx.x * PER + j;
    const uint64_t c = tile[threadIdx.x * PER + j];
    if (i < n) off[i] = run;
    if (i == n - 1) off[n] = run + c;
    run += c;
  }
}

__global__ void k_sal_total(const uint64_t* off, int64_t n, uint64_t cap, SalStatus* st) {
  const uint64_t tot = off[n];
  st->total = tot;
  if (tot > cap) st->too_big = 1u;
}

namespace {

// Last interval m in [a, b] with off[m] <= t (it holds slot t: off[m] <= t
// < off[m + 1], empty intervals before it share its offset).
__device__ __forceinline__ int64_t find_iv(const uint64_t* __restrict__ off, int64_t a,
                                           int64_t b, uint64_t t) {
  while (a < b) {
    const int64_t m = (a + b + 1) >> 1;
    if (off[m] <= t) a = m;
    else b = m - 1;
  }
  return a;
}

}  // namespace

// tile_start[T] = the interval holding slot 256 T, for every T below
// ceil(total / 256) (at most the capacity the map was sized for).
__global__ void __launch_bounds__(256)
k_tile_map(const uint64_t* __restrict__ off, int64_t n, const SalStatus* st,
           int64_t* __restrict__ tile_start) {
  if (st->bad || st->too_big) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += stride) {
    const uint64_t lo = off[m], hi = off[m + 1];
    if (hi <= lo) continue;
    for (uint64_t T = (lo + SAL_TILE - 1) / SAL_TILE; T <= (hi - 1) / SAL_TILE; ++T)
      tile_start[T] = m;
  }
}

constexpr int LDS_IV = 512;  // intervals of a tile staged in LDS

__global__ void __launch_bounds__(256)
k_sal_gather(const int64_t* __restrict__ sa, const bsw_sa_interval* __restrict__ iv,
             const uint64_t* __restrict__ off, int64_t n, const int64_t* __restrict__ tile_start,
             const SalStatus* st, uint64_t* __restrict__ out_off,
             int64_t* __restrict__ out_pos) {
  if (st->bad || st->too_big) return;
  __shared__ uint64_t s_off[LDS_IV];
  __shared__ uint64_t s_k[LDS_IV];
  const uint64_t total = off[n];
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t m = tid; m <= n; m += stride) out_off[m] = off[m];
  const uint64_t ntiles = (total + SAL_TILE - 1) / SAL_TILE;
  // the loop bound and the tile's interval range are uniform per block:
  // every thread reaches both barriers
  for (uint64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
    const int64_t a = tile_start[T];
    const int64_t b = T + 1 < ntiles ? tile_start[T + 1] : n - 1;
    const int64_t cnt = b - a + 1;
    const bool staged = cnt <= LDS_IV;
    if (staged)
      for (int64_t i = threadIdx.x; i < cnt; i += SAL_TILE) {
        s_off[i] = off[a + i];
        s_k[i] = iv[a + i].k;
      }
    __syncthreads();
    const uint64_t t = T * SAL_TILE + threadIdx.x;
    if (t < total) {
      if (staged) {
        int64_t lo = 0, hi = cnt - 1;  // last staged interval with offset <= t
        while (lo < hi) {
          const int64_t mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= t) lo = mid;
          else hi = mid - 1;
        }
        out_pos[t] = sa[s_k[lo] + (t - s_off[lo])];
      } else {
        const int64_t m = find_iv(off, a, b, t);
        out_pos[t] = sa[iv[m].k + (t - off[m])];
      }
    }
    __syncthreads();
  }
}

namespace {
unsigned grid_for(int64_t n, int64_t per_block, int64_t cap) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}
}  // namespace

void launch_iv_check(const bsw_sa_interval* iv, int64_t n, uint64_t sa_len, uint64_t* cnt,
                     SalStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_iv_check, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, iv, n,
                     sa_len, cnt, st);
}

void launch_offset_scan(const uint64_t* cnt, int64_t n, uint64_t* part, uint64_t* off,
                        hipStream_t s) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(k_scan_up, dim3((unsigned)nb), dim3(256), 0, s, cnt, n, part);
  hipLaunchKernelGGL(k_scan_mid, dim3(1), dim3(1024), 0, s, part, nb);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(256), 0, s, cnt, n, part, off);
}

void launch_sal_total(const uint64_t* off, int64_t n, uint64_t cap, SalStatus* st,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_sal_total, dim3(1), dim3(1), 0, s, off, n, cap, st);
}

void launch_tile_map(const uint64_t* off, int64_t n, const SalStatus* st, int64_t* tile_start,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_tile_map, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, off, n, st,
                     tile_start);
}

void launch_sal_gather(const int64_t* sa, const bsw_sa_interval* iv, const uint64_t* off,
                       int64_t n, const int64_t* tile_start, const SalStatus* st,
                       uint64_t* out_off, int64_t* out_pos, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_sal_gather, dim3(blocks), dim3(SAL_TILE), 0, s, sa, iv, off, n,
                     tile_start, st, out_off, out_pos);
}

}  // namespace bsw
