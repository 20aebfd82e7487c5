// bsw_kernels.hip -- HIP kernels for banded Smith-Waterman seed extension on
// gfx950 (MI355X).
//
// Pipeline of one batch (paper Sec. 5.3: sort tasks by length, then
// convert to a vector-friendly layout, then run many pairs side by side):
//   k_fill      zero the status block, histogram and tile counters
//   k_prep      per pair: check lengths/h0/scoring id, pick the value width
//               from the score bound (Sec. 5.4.1) and a kernel class from
//               the query length, build a longest-first bin key, histogram
//   k_codes     check that every sequence byte is a code 0..4
//   k_scan      exclusive scan of the histogram -> bin starts, class ranges
//   k_scatter   counting-sort scatter of pair descriptors into bins
//   k_lane      the DP, one pair per lane (inter-task, Sec. 5.3), row
//               buffer of H and E in LDS; results are written straight to
//               the caller's position (no separate un-permute pass)
//   k_long      the DP for queries longer than 256 (outside the paper's
//               read lengths), one pair per wave, row buffer in HBM
//
// The cell update follows Sec. 5.1 Eq. (2) with the boundary of Eq. (3):
// M = H(i-1,j-1) + S(t_i, q_j) taken only from a positive diagonal cell;
// H = max(M, E, F); E(i+1,j) = max(E - e_del, M - o_del - e_del, 0);
// F(i,j+1) = max(F - e_ins, M - o_ins - e_ins, 0).  Rows are target
// positions, columns query positions; the one-row buffer holds H shifted
// by one column (index j has H(i-1,j-1) when row i reaches it) and E.
#include <hip/hip_runtime.h>

#include "../../include/bsw.h"
#include "bsw_device.h"
#include "bsw_internal.h"
#include "bsw_lanev.h"
#include "bsw_runtime.h"

namespace bsw {

// ---------------------------------------------------------------------------
// small helpers

// ---------------------------------------------------------------------------
// preparation kernels

__global__ void k_fill(uint32_t* p, int64_t nwords) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}


// Estimated rows of a pair for the sort key (only the order of the pairs
// depends on it).  The whole wave walks one pair, 64 positions per step:
// along a diagonal without gaps from h0, the running score is followed
// until it falls to zero or more than z-drop below its running maximum
// (the stops of Sec. 5.1 (b)).
//  - a stop at zero says little (the band still holds other diagonals, and
//    the extension seldom ends there): the estimate is `cap`;
//  - a z-drop is often an indel rather than the end of the alignment: the
//    sequences are compared again after the best position on the diagonals
//    +-1 .. +-ESTIMATE_SHIFT (32 positions, at least 5 in 8 equal); where
//    they agree the walk goes on there from the best score less the gap's
//    cost, otherwise the stop row is the estimate;
//  - a walk that reaches the end of either sequence gives `cap`.
// qs/ts hold Lq/Lt codes; cap = the last row any cell can have + 1.  best
// receives the walk's best score: a path the extension scores as well.
constexpr int ESTIMATE_SHIFT = 8;
constexpr int ESTIMATE_HOPS = 8;

__device__ int estimate_rows(const uint8_t* qs, const uint8_t* ts, int Lq, int Lt, int h0,
                             const KParams& P, int cap, int& best) {
  const int lane = threadIdx.x & 63;
  int pq = 0, pt = 0;      // start of the diagonal being walked
  int base = h0, mx = h0;  // score entering it, best score so far
  for (int hop = 0; hop < ESTIMATE_HOPS; ++hop) {
    const int L = imin(Lq - pq, Lt - pt);
    int bpos = -1;  // position of the best score on this diagonal (-1: its start)
    int stop = -1;  // position of the z-drop
    for (int j0 = 0; j0 < L; j0 += 64) {
      const int j = j0 + lane;
      int sc = 0;
      if (j < L) {
        const int a = ts[pt + j], bq = qs[pq + j];
        sc = (int)(int8_t)(__builtin_amdgcn_perm(P.prow[a < 5 ? a : 0][1],
                                                 P.prow[a < 5 ? a : 0][0], bq) & 0xffu);
      }
      const int run = base + wave_prefix_sum(sc);
      const int rmx = imax(mx, wave_prefix_max(run));
      const bool zs = j < L && P.zdrop > 0 && rmx - run > P.zdrop;
      const unsigned long long m = __ballot(j < L && (run <= 0 || zs));
      const int last = m ? __builtin_ctzll(m) : 63;  // lanes up to the stop count
      const int rlast = __shfl(rmx, last, 64);
      if (rlast > mx) {
        const unsigned long long at = __ballot(lane <= last && j < L && run == rlast);
        bpos = j0 + __builtin_ctzll(at);
        mx = rlast;
      }
      if (m) {
        if (!__shfl((int)zs, last, 64)) {
          best = mx;
          return cap;
        }
        stop = j0 + last;
        break;
      }
      base = __shfl(run, 63, 64);
    }
    if (stop < 0) {
      best = mx;
      return cap;
    }
    // look for the sequences to agree again after the best position: lanes
    // 0-31 try the shift +d (extra target bases: target read d further on),
    // lanes 32-63 the shift -d (extra query bases); every byte is loaded
    // before the first comparison
    const int aq = pq + bpos + 1, at = pt + bpos + 1, x = lane & 31;
    const bool up = lane < 32;
    const uint8_t* fs = up ? qs + aq : ts + at;  // the side read unshifted
    const uint8_t* ss = up ? ts + at : qs + aq;  // the side read at +d
    const int flen = up ? Lq - aq : Lt - at, slen = up ? Lt - at : Lq - aq;
    const uint32_t f = x < flen ? fs[x] : 4u;
    uint32_t sv[ESTIMATE_SHIFT];
#pragma unroll
    for (int d = 1; d <= ESTIMATE_SHIFT; ++d) sv[d - 1] = x + d < slen ? ss[x + d] : 5u;
    int nq = -1, nt = -1, dd = 0;
#pragma unroll
    for (int d = 1; d <= ESTIMATE_SHIFT; ++d) {
      const int n = imin(32, imin(flen, slen - d));
      const unsigned long long e = __ballot(x < n && f < 4 && f == sv[d - 1]);
      const int n_lo = __shfl(n, 0, 64), n_hi = __shfl(n, 32, 64);
      const int c_lo = __builtin_popcount((uint32_t)e);
      const int c_hi = __builtin_popcount((uint32_t)(e >> 32));
      if (nq < 0 && n_lo >= 8 && 8 * c_lo >= 5 * n_lo) {
        nq = aq;
        nt = at + d;
        dd = d;
      } else if (nq < 0 && n_hi >= 8 && 8 * c_hi >= 5 * n_hi) {
        nq = aq + d;
        nt = at;
        dd = d;
      }
    }
    if (nq < 0) {
      best = mx;
      return imin(pt + stop + 1, cap);
    }
    base = mx - P.o_del - dd * P.e_del;
    if (base <= 0) {
      best = mx;
      return cap;
    }
    pq = nq;
    pt = nt;
  }
  best = mx;
  return cap;
}

// Add one to cnt[key] for every lane with active set, with one atomic per
// distinct key in the wave (pairs that share a bin, as short or empty
// queries of one length do, would otherwise serialise on its counter).
// The lanes are grouped by key first (ALU only); then the first lane of
// each group adds the group's size, all groups in one atomic instruction.
// Returns the lane's slot: the counter's old value plus the lane's rank in
// its group.  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_count_add(uint32_t* cnt, uint32_t key,
                                                   bool active) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned long long todo = __ballot(active);
  int leader = lane;
  uint32_t rank = 0, size = 0;
  while (todo) {
    const int l = __builtin_ctzll(todo);
    const uint32_t kl = (uint32_t)__builtin_amdgcn_readlane((int)key, l);
    const unsigned long long same = __ballot(active && key == kl);
    todo &= ~same;
    if ((same >> lane) & 1ull) {
      leader = l;
      rank = (uint32_t)__popcll(same & below);
      size = (uint32_t)__popcll(same);
    }
  }
  uint32_t base = 0;
  if (active && leader == lane) base = atomicAdd(&cnt[key], size);
  return (uint32_t)__shfl((int)base, leader, 64) + rank;
}

// Pair k's sequences are q[q_off[k] .. q_end[k]) and t[t_off[k] .. t_end[k]);
// for an ordinary batch q_end = q_off + 1 and t_end = t_off + 1.  Each wave
// takes 64 consecutive pairs, one per lane.
__global__ void __launch_bounds__(256)
k_prep(int64_t n, const uint8_t* __restrict__ q, const uint8_t* __restrict__ t,
       const uint64_t* __restrict__ q_off, const uint64_t* __restrict__ q_end,
       const uint64_t* __restrict__ t_off, const uint64_t* __restrict__ t_end,
       const int32_t* __restrict__ h0, const uint8_t* __restrict__ pid, int n_params,
       const KParams* __restrict__ kp, int min_bits, int spec16,
       uint32_t* __restrict__ keys, uint32_t* __restrict__ hist, Status* st) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t g = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
       g * 64 < n; g += nwaves) {
    const int64_t k = g * 64 + lane;
    bool ok = k < n;
    uint64_t qo = 0, qe = 0, to = 0, te = 0;
    int p = 0, hh = 1;
    if (ok) {
      qo = q_off[k];
      qe = q_end[k];
      to = t_off[k];
      te = t_end[k];
      p = pid ? pid[k] : 0;
      hh = h0[k];
      ok = qe >= qo && te >= to && qe - qo <= BSW_MAX_LEN && te - to <= BSW_MAX_LEN &&
           hh >= 1 && hh <= BSW_MAX_H0 && p < n_params;
      if (!ok) {
        atomicMax(&st->first_bad_inv, ~(unsigned long long)k);
        atomicOr(&st->bad, 1u);
        keys[k] = 0xffffffffu;
      }
    }
    const int ql = ok ? (int)(qe - qo) : 0, tl = ok ? (int)(te - to) : 0;
    const KParams& P = kp[ok ? p : 0];
    // longest first inside a class: larger query first, then more rows.
    // For wide queries the rows are estimated by the diagonal walk, capped
    // by the band (no row past qlen + w + 1 has a cell): pairs that end
    // early then share tiles, so the lanes of a tile finish together.
    int rows_est = imin(tl, ql + band_cap(P, ql) + 1);
    int walk_best = 0;  // best score of the walk (a path the DP also scores)
    unsigned long long walk = __ballot(ok && ql > 192 && ql <= 256);
    while (walk) {
      const int l = __builtin_ctzll(walk);
      walk &= walk - 1;
      const uint64_t wq = __shfl(qo, l, 64), wt = __shfl(to, l, 64);
      const int wlq = __shfl(ql, l, 64), wlt = __shfl(tl, l, 64);
      const int wh = __shfl(hh, l, 64), wp = __shfl(p, l, 64);
      const int wcap = __shfl(rows_est, l, 64);
      int wbest = 0;
      const int r = estimate_rows(q + wq, t + wt, wlq, wlt, wh, kp[wp], wcap, wbest);
      if (lane == l) {
        rows_est = r;
        walk_best = wbest;
      }
    }
    uint32_t key = 0;
    if (ok) {
      // bound on every stored H and E of the pair (Sec. 5.4.1 precision)
      const int64_t U = (int64_t)hh + (int64_t)P.amax * (ql < tl ? ql : tl);
      int wd = U <= 255 ? W8 : (U <= 65535 ? W16 : W32);
      if (min_bits >= 16 && wd < W16) wd = W16;
      if (min_bits >= 32) wd = W32;
      // 16-bit pairs start at 8 bits when the seed itself leaves room
      const int slack = P.amax - P.oe_del > 0 ? P.amax - P.oe_del : 0;
      // (not when the walk already scored past what 8-bit records hold:
      // the pair would only be rerun)
      const bool spec8 = wd == W8 || (spec16 && wd == W16 && min_bits < 16 &&
                                      hh + slack <= 255 && walk_best + slack < 255);
      int cls, cap;
      if (ql > 256) {
        cls = CLS_LONG;
        cap = BSW_MAX_LEN;
        atomicMax(&st->long_max, (unsigned long long)ql);
      } else if (spec8) {
        int c = 0;
        while (L8_CAP[c] < ql) ++c;
        cls = CLS_L8 + c;
        cap = L8_CAP[c];
      } else {
        int c = 0;
        while (LW_CAP[c] < ql) ++c;
        cls = (wd == W16 ? CLS_W16 : CLS_W32) + c;
        cap = LW_CAP[c];
      }
      int qq = (int)((int64_t)ql * 64 / (cap + 1));
      int tq = rows_est >> 3;
      qq = qq > 63 ? 63 : qq;
      tq = tq > 63 ? 63 : (tq < 0 ? 0 : tq);
      const uint32_t sub = ((uint32_t)(63 - qq) << 6) | (uint32_t)(63 - tq);
      key = ((uint32_t)cls << KEY_SUB_BITS) | sub;
      keys[k] = key;
    }
    (void)wave_count_add(hist, key, ok);
  }
}

// Every byte of q[off[0] .. off[n]) must be a code 0..4; a bad byte names
// the pair that holds it (binary search over the offsets).
__device__ __forceinline__ uint64_t imin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__global__ void k_codes(const uint8_t* __restrict__ s,
                        const uint64_t* __restrict__ off, int64_t n,
                        Status* st) {
  const uint64_t lo = off[0], hi = off[n];
  if (hi <= lo) return;
  const uint64_t len = hi - lo;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // 16 bytes per step; the leading bytes up to a 16-byte boundary and the
  // tail are checked one by one
  const uint64_t head = (16 - ((uintptr_t)(s + lo) & 15)) & 15;
  const uint64_t h = head < len ? head : len;
  const uint64_t nv = (len - h) >> 4;
  const uint4* w = (const uint4*)(s + lo + h);
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t badpos = ~0ull;
  for (uint64_t i = tid; i < nv; i += stride) {
    const uint4 v4 = w[i];
    const uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
    // a byte is > 4 iff (byte + 0x7b) has bit 7 set, for bytes <= 0x84;
    // bytes >= 0x80 are caught by their own top bit
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) t |= ((v[k] & 0x7f7f7f7fu) + 0x7b7b7b7bu) | v[k];
    if (t & 0x80808080u) {
#pragma unroll
      for (int b = 15; b >= 0; --b)
        if (((v[b >> 2] >> (8 * (b & 3))) & 0xffu) > 4) badpos = imin64(badpos, lo + h + i * 16 + b);
    }
  }
  if (tid < h && s[lo + tid] > 4) badpos = imin64(badpos, lo + tid);
  const uint64_t tail = h + nv * 16;
  if (tid < len - tail && s[lo + tail + tid] > 4) badpos = imin64(badpos, lo + tail + tid);
  if (badpos != ~0ull) {
    int64_t a = 0, b = n - 1;  // largest k with off[k] <= badpos
    while (a < b) {
      const int64_t m = (a + b + 1) >> 1;
      if (off[m] <= badpos) a = m; else b = m - 1;
    }
    // skip empty pairs that share the offset
    while (a + 1 < n && off[a + 1] <= badpos) ++a;
    atomicMax(&st->first_bad_inv, ~(unsigned long long)a);
    atomicOr(&st->bad, 1u);
  }
}

// One block: exclusive scan of hist into cursor, class ranges.
__global__ void __launch_bounds__(1024)
k_scan(const uint32_t* __restrict__ hist, uint32_t* __restrict__ cursor,
       long long* __restrict__ cls_range) {
  __shared__ uint32_t part[1024];
  constexpr int PER = (NBINS + 1023) / 1024;
  const int tid = threadIdx.x;
  const int b0 = tid * PER;
  uint32_t s = 0;
  for (int i = 0; i < PER; ++i)
    if (b0 + i < NBINS) s += hist[b0 + i];
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = tid ? part[tid - 1] : 0;
  for (int i = 0; i < PER; ++i) {
    const int b = b0 + i;
    if (b < NBINS) {
      cursor[b] = run;
      if ((b & ((1 << KEY_SUB_BITS) - 1)) == 0) cls_range[2 * (b >> KEY_SUB_BITS)] = run;
      run += hist[b];
    }
  }
  __syncthreads();
  if (tid < NCLS) {
    // count of class tid = start of the next class - own start
    const long long beg = cls_range[2 * tid];
    const long long end = tid + 1 < NCLS ? cls_range[2 * (tid + 1)] : (long long)part[1023];
    cls_range[2 * tid + 1] = end - beg;
  }
}

__global__ void k_scatter(int64_t n, const uint64_t* __restrict__ q_off,
                          const uint64_t* __restrict__ q_end,
                          const uint64_t* __restrict__ t_off,
                          const uint64_t* __restrict__ t_end,
                          const int32_t* __restrict__ h0,
                          const uint8_t* __restrict__ pid,
                          const uint32_t* __restrict__ keys,
                          uint32_t* __restrict__ cursor,
                          PairDesc* __restrict__ desc, const Status* st) {
  if (st->bad) return;
  // the loop bound is uniform per block, so every lane of a wave takes part
  // in each slot grab
  for (int64_t k0 = blockIdx.x * (int64_t)blockDim.x; k0 < n;
       k0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = k0 + threadIdx.x;
    const bool active = k < n;
    const uint32_t key = active ? keys[k] : 0u;
    const uint32_t pos = wave_count_add(cursor, key, active);
    if (!active) continue;
    PairDesc d;
    d.qo = q_off[k];
    d.to = t_off[k];
    d.ql = (uint16_t)(q_end[k] - d.qo);
    d.tl = (uint16_t)(t_end[k] - d.to);
    d.h0 = h0[k];
    d.idx = (uint32_t)k;
    d.pid = pid ? pid[k] : 0;
    d.cls = (uint8_t)(key >> KEY_SUB_BITS);
    d.pad_[0] = d.pad_[1] = 0;
    desc[pos] = d;
  }
}

// Serving: gather the pairs of several resident requests into one batch.
// Request r covers batch pairs [tab[r].base, tab[r].base + tab[r].n); its
// sequence bytes sit at byte offsets q_at / t_at from the common base and
// its offset arrays are the caller's, taken relative to their first entry.
// Copy of byte ranges from mapped host memory into device memory, one 4 KiB
// chunk per workgroup step: every thread writes whole destination dwords
// (destinations are 4-byte aligned, with at least 3 bytes of slack after
// each range), each composed from the two aligned source dwords that
// cover it; a source dword is read only if it holds a byte of the range,
// so no read leaves the range's pages.
__global__ void __launch_bounds__(256) k_gather(const CopySeg* __restrict__ segs, int ns,
                                                unsigned long long nchunks) {
  for (unsigned long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
    int a = 0, b = ns - 1;
    while (a < b) {
      const int m = (a + b + 1) >> 1;
      if (segs[m].chunk0 <= c) a = m; else b = m - 1;
    }
    const CopySeg sg = segs[a];
    const unsigned long long off = (c - sg.chunk0) * 4096ull;
    const uintptr_t s0 = (uintptr_t)sg.src;
    const uintptr_t sal = s0 & ~(uintptr_t)3;
    const uint32_t sh = (uint32_t)(s0 & 3);
    const uintptr_t slim = s0 + sg.bytes;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned long long o = off + ((unsigned long long)k * 256 + threadIdx.x) * 4;
      if (o >= sg.bytes) break;
      const uintptr_t p0 = sal + o, p1 = p0 + 4;
      const uint32_t w0 = *(const uint32_t*)p0;
      const uint32_t w1 = p1 < slim ? *(const uint32_t*)p1 : 0u;
      *(uint32_t*)(sg.dst + o) = __builtin_amdgcn_alignbyte(w1, w0, sh);
    }
  }
}

// The request of batch pair g: the last table entry whose base is <= g.
__device__ __forceinline__ int req_of(const ReqSlice* __restrict__ tab, int m, int64_t g) {
  int a = 0, b = m - 1;
  while (a < b) {
    const int c = (a + b + 1) >> 1;
    if (tab[c].base <= g) a = c; else b = c - 1;
  }
  return a;
}

// Code check of a serving batch, one pair per thread: a request with a
// byte > 4 in any of its pairs gets bad[a] = ~(its smallest such pair).
__global__ void k_req_codes(const ReqSlice* __restrict__ tab, int m, int64_t n,
                            const uint8_t* __restrict__ base,
                            unsigned long long* __restrict__ bad) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int a = req_of(tab, m, g);
    const ReqSlice& r = tab[a];
    const int64_t i = g - r.base;
    const uint8_t* qs = base + r.q_at + (r.q_off[i] - r.q_off[0]);
    const uint8_t* ts = base + r.t_at + (r.t_off[i] - r.t_off[0]);
    const uint64_t ql = r.q_off[i + 1] - r.q_off[i], tl = r.t_off[i + 1] - r.t_off[i];
    bool ok = true;
    for (uint64_t k = 0; k < ql && ok; ++k) ok = qs[k] <= 4;
    for (uint64_t k = 0; k < tl && ok; ++k) ok = ts[k] <= 4;
    if (!ok) atomicMax(&bad[a], ~(unsigned long long)i);
  }
}

__global__ void k_assemble(const ReqSlice* __restrict__ tab, int m, int64_t n,
                           uint64_t* __restrict__ qb, uint64_t* __restrict__ qe,
                           uint64_t* __restrict__ tb, uint64_t* __restrict__ te,
                           int32_t* __restrict__ h0, uint8_t* __restrict__ pid,
                           const unsigned long long* __restrict__ bad) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int a = req_of(tab, m, g);
    const ReqSlice& r = tab[a];
    const int64_t i = g - r.base;
    if (bad[a]) {  // a rejected request: empty pairs that read no byte
      qb[g] = qe[g] = r.q_at;
      tb[g] = te[g] = r.t_at;
      h0[g] = 1;
      pid[g] = 0;
      continue;
    }
    const uint64_t q0 = r.q_off[0], t0 = r.t_off[0];
    qb[g] = r.q_at + (r.q_off[i] - q0);
    qe[g] = r.q_at + (r.q_off[i + 1] - q0);
    tb[g] = r.t_at + (r.t_off[i] - t0);
    te[g] = r.t_at + (r.t_off[i + 1] - t0);
    h0[g] = r.h0[i];
    pid[g] = r.pid ? r.pid[i] : 0;
  }
}

// ---------------------------------------------------------------------------
// the DP for one pair in one lane; the row buffer entry of column j lives at
// hb[j * S] and the query code at qb[j * S] (S = 64 in LDS, so that the 64
// lanes of a wave hit distinct banks; S = 1 for a private buffer)

template <int W, int S>
__device__ __forceinline__ long long extend_pair(const PairDesc& pd, const KParams& P,
                                            const uint8_t* __restrict__ q,
                                            const uint8_t* __restrict__ t,
                                            typename Rec<W>::T* hb, uint8_t* qb,
                                            bsw_result* __restrict__ out,
                                            bsw_diag* __restrict__ diag) {
  using R = Rec<W>;
  const int Lq = pd.ql, Lt = pd.tl, h0 = pd.h0;
  const int oD = P.o_del, eD = P.e_del, eI = P.e_ins;
  const int oeD = P.oe_del, oeI = P.oe_ins, oI = P.o_ins;
  const int zd = P.zdrop;
  const int wb = band_cap(P, Lq);
  uint32_t pl[5], ph[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    pl[a] = P.prow[a][0];
    ph[a] = P.prow[a][1];
  }

  // first row of Eq. (3): H(-1, j-1) = max(0, h0 - o_ins - e_ins*j), E = 0
  hb[0] = R::pack(h0, 0);
  for (int j = 1; j <= Lq; ++j) hb[j * S] = R::pack(imax(0, h0 - oI - eI * j), 0);
  const uint8_t* qs = q + pd.qo;
  for (int j = 0; j < Lq; ++j) qb[j * S] = qs[j];

  int best = h0, bi = -1, bj = -1, gbest = -1, gi = -1, moff = 0;
  int beg = 0, end = Lq, rows = 0, stop = 0;
  int64_t cells = 0;
  const uint8_t* ts = t + pd.to;
  for (int i = 0; i < Lt; ++i) {
    ++rows;
    // band (Sec. 5.1 (a))
    beg = imax(beg, i - wb);
    end = imin(imin(end, i + wb + 1), Lq);
    if (end > beg) cells += end - beg;
    // score row of this target base
    const int tb = ts[i];
    uint32_t lo = pl[0], hi = ph[0];
#pragma unroll
    for (int a = 1; a < 5; ++a) {
      lo = tb == a ? pl[a] : lo;
      hi = tb == a ? ph[a] : hi;
    }
    // first column of Eq. (3) while the band starts at column 0
    int hl = beg == 0 ? imax(0, h0 - oD - eD * (i + 1)) : 0;
    int f = 0, m = 0, mj = -1;
    for (int j = beg; j < end; ++j) {
      const typename R::T r = hb[j * S];
      const int d = R::h(r), e = R::e(r);
      const int s = score_of(lo, hi, qb[j * S]);
      const int M = d > 0 ? d + s : 0;
      const int h = imax(imax(M, e), f);
      const int en = imax(imax(e - eD, M - oeD), 0);
      hb[j * S] = R::pack(hl, en);
      hl = h;
      mj = h >= m ? j : mj;
      m = imax(m, h);
      f = imax(imax(f - eI, M - oeI), 0);
    }
    hb[end * S] = R::pack(hl, 0);
    // best score touching the end of the query (Sec. 5.4 (b))
    if (imax(beg, end) == Lq) {
      gi = hl >= gbest ? i : gi;
      gbest = imax(gbest, hl);
    }
    // all-zero row (Sec. 5.1 (b))
    if (m == 0) {
      stop = 1;
      break;
    }
    if (m > best) {
      best = m;
      bi = i;
      bj = mj;
      moff = imax(moff, mj > i ? mj - i : i - mj);
    } else if (zd > 0) {
      // drop from the best, net of the gap the drift between the two
      // cells would cost (Sec. 5.1 (b))
      const int drift = (i - bi) - (mj - bj);
      const int drop = best - m - (drift > 0 ? drift * eD : -drift * eI);
      if (drop > zd) {
        stop = 2;
        break;
      }
    }
    // shrink the band by its empty ends (Sec. 5.1 (c))
    while (beg < end && R::empty(hb[beg * S])) ++beg;
    int k = end;
    while (k >= beg && R::empty(hb[k * S])) --k;
    end = imin(k + 2, Lq);
  }
  bsw_result res;
  res.score = best;
  res.qle = bj + 1;
  res.tle = bi + 1;
  res.gtle = gi + 1;
  res.gscore = gbest;
  res.max_off = moff;
  out[pd.idx] = res;
  if (diag) {
    bsw_diag dg;
    dg.rows = rows;
    dg.stop = stop;
    dg.cells = cells;
    diag[pd.idx] = dg;
  }
  return cells;
}

// Lane mode with wide records: one wave runs a tile of 64 pairs of one
// class; range = {first pair, pair count} in desc.  PERSIST: waves pull
// tiles from a counter until the class is done (tiles are in longest-first
// order); otherwise wave w of the grid runs tile w.
template <int W, int LQCAP, bool PERSIST>
__global__ void __launch_bounds__(256)
k_lane(const PairDesc* __restrict__ desc, const long long* __restrict__ range,
       const uint8_t* __restrict__ q, const uint8_t* __restrict__ t,
       const KParams* __restrict__ kp, bsw_result* __restrict__ out,
       bsw_diag* __restrict__ diag, uint32_t* tile_ctr, const Status* st,
       unsigned long long* __restrict__ cls_cells) {
  if (st->bad) return;
  using T = typename Rec<W>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr size_t HB_BYTES = (size_t)(LQCAP + 1) * 64 * sizeof(T);
  constexpr size_t PER_WAVE = HB_BYTES + (size_t)LQCAP * 64;
  T* hb = (T*)(smem + wv * PER_WAVE) + lane;
  uint8_t* qb = smem + wv * PER_WAVE + HB_BYTES + lane;
  const long long begin = range[0], count = range[1];
  const uint32_t ntiles = (uint32_t)((count + 63) >> 6);
  if (ntiles == 0) return;  // an empty class: no atomics
  uint32_t tile = blockIdx.x * (blockDim.x >> 6) + wv;
  unsigned long long acc = 0;
  for (;;) {
    if (PERSIST) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(tile_ctr, 1u);
      tile = wave_first(__shfl(v, 0));
    }
    if (tile >= ntiles) break;
    const long long k = (long long)tile * 64 + lane;
    if (k < count) {
      const PairDesc pd = desc[begin + k];
      acc += (unsigned long long)extend_pair<W, 64>(pd, kp[pd.pid], q, t, hb, qb, out,
                                                    diag);
    }
    if (!PERSIST) break;
  }
  acc = wave_sum64(acc);
  if (lane == 0 && acc) atomicAdd(cls_cells, acc);
}

// ---------------------------------------------------------------------------
// Lane mode with 8-bit records (the main kernel).
//
// Every lane of the wave owns one pair; the wave walks rows in lock step
// and, inside a row, walks the same column j in every lane (each lane masks
// columns at or past its band end; columns left of its band start compute
// zeros because the buffer there is kept at zero), so the row buffer can be
// laid out column-major: chunk c of four columns for lane l is one 8-byte
// LDS word at [c][l], bytes (H0,E0,H1,E1,H2,E2,H3,E3), and the four query
// codes of a chunk are one dword at [c][l] of a per-wave tile in HBM.  One
// LDS read, one LDS write, one global read and one v_perm (four scores)
// serve four cells.  Column CAP is the right-edge slot.
//
// Values are stored as bytes.  A pair that may exceed 8 bits is detected
// from its final best score (all stored H are <= best; stored E are
// <= best + max(0, A - o_del - e_del)); it is then not written but queued
// for a 16-bit rerun.

// Chunk records of the chunked lane kernels: four consecutive columns of
// one lane.  8-bit: an 8-byte word, bytes (H0,E0,H1,E1,H2,E2,H3,E3).
// 16-bit: a 16-byte word, one 32-bit (H | E << 16) per column.
template <int WB> struct Chunk;
template <> struct Chunk<8> {
  using T = uint2;
  static constexpr int BYTES = 8;    // per lane per chunk
  static constexpr int REC = 2;      // bytes per column record
  static constexpr int MAXV = 255;
  typedef unsigned short R;          // one column record
};
template <> struct Chunk<16> {
  using T = uint4;
  static constexpr int BYTES = 16;
  static constexpr int REC = 4;
  static constexpr int MAXV = 65535;
  typedef uint32_t R;
};

// One band cell (Sec. 5.1 Eq. (2)): d = stored H(i-1, j-1), e = stored
// E(i, j), s = S(t_i, q_j).  Updates hl (H(i, j-1) -> H(i, j)), f, mkey and
// returns the new record (H(i, j-1), E(i+1, j)) unshifted (H in the low
// field).  Values beyond the record width only occur in pairs that are
// rerun wider, so the record is not masked.
struct CellParams {
  int eD, oeD, eI, oeI;
};
template <int WB>
__device__ __forceinline__ uint32_t cell(int d, int e, int s, int j, int& hl, int& f,
                                         int& key, const CellParams& cp) {
  const int M = d ? d + s : 0;
  const int h = imax(imax(M, e), f);
  const int en = imax(imax(e - cp.eD, M - cp.oeD), 0);
  const uint32_t r = (uint32_t)hl | ((uint32_t)en << WB);
  hl = h;
  key = (int)(((uint32_t)h << 9) | (uint32_t)j);
  f = imax(imax(f - cp.eI, M - cp.oeI), 0);
  return r;
}
__device__ __forceinline__ int imax3(int a, int b, int c) { return imax(imax(a, b), c); }

// the four cells of a whole chunk (no masking)
__device__ __forceinline__ uint2 chunk_cells(const uint2 ch, uint32_t sc, int j0, int& hl,
                                             int& f, int& mkey, const CellParams& cp) {
  int k0, k1, k2, k3;
  const uint32_t r0 = cell<8>(ch.x & 0xff, (ch.x >> 8) & 0xff, (int)(int8_t)sc, j0, hl, f,
                              k0, cp);
  const uint32_t r1 = cell<8>((ch.x >> 16) & 0xff, ch.x >> 24, (int)(int8_t)(sc >> 8),
                              j0 + 1, hl, f, k1, cp);
  const uint32_t r2 = cell<8>(ch.y & 0xff, (ch.y >> 8) & 0xff, (int)(int8_t)(sc >> 16),
                              j0 + 2, hl, f, k2, cp);
  const uint32_t r3 = cell<8>((ch.y >> 16) & 0xff, ch.y >> 24, (int)(int8_t)(sc >> 24),
                              j0 + 3, hl, f, k3, cp);
  mkey = imax3(imax3(mkey, k0, k1), k2, k3);
  return make_uint2(r0 | (r1 << 16), r2 | (r3 << 16));
}
__device__ __forceinline__ uint4 chunk_cells(const uint4 ch, uint32_t sc, int j0, int& hl,
                                             int& f, int& mkey, const CellParams& cp) {
  uint4 r;
  int k0, k1, k2, k3;
  r.x = cell<16>(ch.x & 0xffff, ch.x >> 16, (int)(int8_t)sc, j0, hl, f, k0, cp);
  r.y = cell<16>(ch.y & 0xffff, ch.y >> 16, (int)(int8_t)(sc >> 8), j0 + 1, hl, f, k1, cp);
  r.z = cell<16>(ch.z & 0xffff, ch.z >> 16, (int)(int8_t)(sc >> 16), j0 + 2, hl, f, k2, cp);
  r.w = cell<16>(ch.w & 0xffff, ch.w >> 16, (int)(int8_t)(sc >> 24), j0 + 3, hl, f, k3, cp);
  mkey = imax3(imax3(mkey, k0, k1), k2, k3);
  return r;
}
// Packed 16-bit form of the four cells of an 8-bit chunk: the diagonal,
// E and H terms of two columns at a time (v_pk_* on gfx950); only the F
// recurrence along the row is sequential, and it is unrolled two columns
// per step: F(j+1) = max(F(j) - e_ins, A(j)) with A(j) = max(M(j) - o_ins -
// e_ins, 0), so F(j+2) = max(F(j) - 2 e_ins, A(j) - e_ins, A(j+1)).  Every
// value fits 16 bits: stored values are bytes, scores are bytes, gap costs
// are at most 2000.  The diagonal gate M = d ? d + s : 0 becomes
// min(d + s, 128 d): for d >= 1 that is d + s, for d = 0 it is at most 0,
// which gives the same H, E and F as M = 0 because E and F are >= 0.
// The four cells of an unmasked 8-bit chunk.  hl and f carry H(i, j0-1) and
// F(i, j0) in and H(i, j0+3), F(i, j0+4) out; the chunk's largest H goes to
// m4 (its column is found after the row from the stored values).
template <bool SYM>
__device__ __forceinline__ uint2 chunk_cells_pk(const uint2 ch, uint32_t sc, int& hl, int& f,
                                                int& m4, const PkParams& pp) {
  const s16x2 D01 = pk(__builtin_amdgcn_perm(0u, ch.x, 0x0c020c00u));
  const s16x2 E01 = pk(__builtin_amdgcn_perm(0u, ch.x, 0x0c030c01u));
  const s16x2 D23 = pk(__builtin_amdgcn_perm(0u, ch.y, 0x0c020c00u));
  const s16x2 E23 = pk(__builtin_amdgcn_perm(0u, ch.y, 0x0c030c01u));
  // scores, sign-extended in pairs: the sign of byte b is bit 15 of a word
  // holding that byte at position 1
  const uint32_t sc8 = sc << 8;
  const s16x2 S01 = pk(__builtin_amdgcn_perm(sc8, sc, 0x08010a00u));
  const s16x2 S23 = pk(__builtin_amdgcn_perm(sc8, sc, 0x09030b02u));
  const s16x2 G01 = pmin(D01 + S01, D01 << 7), G23 = pmin(D23 + S23, D23 << 7);
  const s16x2 TD01 = G01 - pp.oeD, TD23 = G23 - pp.oeD;
  const s16x2 EN01 = pmax(psubsat(E01, pp.eD), TD01);
  const s16x2 EN23 = pmax(psubsat(E23, pp.eD), TD23);
  const s16x2 z = bcast(0);
  const s16x2 A01 = pmax(SYM ? TD01 : G01 - pp.oeI, z);
  const s16x2 A23 = pmax(SYM ? TD23 : G23 - pp.oeI, z);
  const s16x2 F12 = pmax(pmax(A01, bcast(A01[0]) - pp.eI), bcast(f) - pp.eI12);
  const s16x2 F34 = pmax(pmax(A23, bcast(A23[0]) - pp.eI), bcast(F12[1]) - pp.eI12);
  const s16x2 F01 = (s16x2){(short)f, F12[0]}, F23 = (s16x2){F12[1], F34[0]};
  const s16x2 H01 = pmax(pmax(G01, E01), F01), H23 = pmax(pmax(G23, E23), F23);
  // records (H(i, j-1), E(i+1, j)): x = (hl, en0, h0, en1), y = (h1, en2, h2, en3)
  const uint32_t hx = __builtin_amdgcn_perm(unpk(H01), (uint32_t)hl, 0x05040100u);
  const uint32_t x = __builtin_amdgcn_perm(unpk(EN01), hx, 0x06020400u);
  const uint32_t hy = __builtin_amdgcn_perm(unpk(H23), unpk(H01), 0x0c040c02u);
  const uint32_t y = __builtin_amdgcn_perm(unpk(EN23), hy, 0x06020400u);
  const s16x2 m2 = pmax(H01, H23);
  m4 = imax(m2[0], m2[1]);
  hl = H23[1];
  f = F34[1];
  return make_uint2(x, y);
}

// The low `bits` bits of a dword (0..32): ~(~0 << bits) taken from a 64-bit
// shift, so that bits = 32 gives all ones.
__device__ __forceinline__ uint32_t low_bits(int bits) { return ~(uint32_t)(~0ull << bits); }

// The same for a chunk that holds the band end of some lane (k = end - j0
// for this lane).  Columns at or past end read as zero, so M <= 0 there and
// their H is below H(i, end-1) (or zero): the chunk maximum is unchanged.
// They keep their stored values, except that column end takes H(i, end-1)
// in its H byte (the right edge of the band, R8) and keeps its E (zero).
template <bool SYM>
__device__ __forceinline__ uint2 chunk_cells_pk_masked(const uint2 ch, uint32_t sc, int k,
                                                       int& hl, int& f, int& m4,
                                                       const PkParams& pp) {
  const int n = imin(imax(k, 0), 4);             // columns read
  const int nb = imin(imax(2 * k + 1, 0), 8);    // bytes written
  const uint2 in = make_uint2(ch.x & low_bits(16 * imin(n, 2)),
                              ch.y & low_bits(16 * imax(n - 2, 0)));
  const uint2 r = chunk_cells_pk<SYM>(in, sc, hl, f, m4, pp);
  const uint32_t mx = low_bits(8 * imin(nb, 4)), my = low_bits(8 * imax(nb - 4, 0));
  return make_uint2((r.x & mx) | (ch.x & ~mx), (r.y & my) | (ch.y & ~my));
}

// column cc of a chunk, read and written as a record
__device__ __forceinline__ uint32_t rec_get(const uint2& c, int cc) {
  return ((cc < 2 ? c.x : c.y) >> (16 * (cc & 1))) & 0xffffu;
}
__device__ __forceinline__ void rec_set(uint2& c, int cc, uint32_t r) {
  uint32_t& w = cc < 2 ? c.x : c.y;
  const int sh = 16 * (cc & 1);
  w = (w & ~(0xffffu << sh)) | ((r & 0xffffu) << sh);
}
__device__ __forceinline__ uint32_t rec_get(const uint4& c, int cc) {
  return cc == 0 ? c.x : (cc == 1 ? c.y : (cc == 2 ? c.z : c.w));
}
__device__ __forceinline__ void rec_set(uint4& c, int cc, uint32_t r) {
  if (cc == 0) c.x = r; else if (cc == 1) c.y = r; else if (cc == 2) c.z = r; else c.w = r;
}

// Row buffer in a ring of RC chunks: the band of row i lies in
// [i - w', i + w' + 1] and nothing outside [beg, highest index written]
// is ever read again, so with 4*RC > 2w' + 4 no live column shares a
// slot with another live column.  Columns are initialised lazily (first-
// row value of Eq. (3)) the first time the band end reaches them.  With
// RC = CAP/4 + 1 the ring never wraps.  The host keeps 2*RC > CAP/4, so
// a chunk index (at most CAP/4) needs at most one subtraction.
__device__ __forceinline__ int ring_slot(int chunk, int rc) {
  return chunk >= rc ? chunk - rc : chunk;
}

// Lane mode with chunk records (the main kernel, 8- or 16-bit records).
//
// Every lane of the wave owns one pair; the wave walks rows in lock step
// and, inside a row, walks the same column j in every lane (each lane masks
// columns at or past its band end; columns left of its band start compute
// zeros because the buffer there is kept at zero), so the row buffer can be
// laid out column-major: chunk c of four columns for lane l is one record
// word at [c][l], and the four query codes of a chunk are one dword at
// [c][l] of a per-wave tile in HBM.  One LDS read, one LDS write, one
// global read and one v_perm (four scores) serve four cells.
//
// A pair that may exceed the record width is detected from its final best
// score (all stored H are <= best; stored E are <= best + max(0, A - o_del
// - e_del)); it is then not written but queued (ovf) for a wider rerun.
template <int CAP, bool SYM, int WB>
__global__ void __launch_bounds__(64)
k_lanec(const PairDesc* __restrict__ desc, const long long* __restrict__ range,
        const uint8_t* __restrict__ q, const uint8_t* __restrict__ t,
        const KParams* __restrict__ kp, bsw_result* __restrict__ out,
        bsw_diag* __restrict__ diag, uint32_t* tile_ctr, const Status* st,
        uint32_t* __restrict__ qtiles, PairDesc* __restrict__ ovf,
        long long* __restrict__ ovf_count, int persist, int RC,
        unsigned long long* __restrict__ cls_cells,
        unsigned long long* __restrict__ work_cells) {
  if (st->bad) return;
  using CK = Chunk<WB>;
  using T = typename CK::T;
  using R = typename CK::R;
  extern __shared__ __align__(16) unsigned char smem[];  // [RC][64] chunk words
  const int lane = threadIdx.x;
  uint32_t* qt = qtiles + (size_t)blockIdx.x * (CAP / 4 + 6) * 64 + lane;
  T* my = (T*)smem + lane;
  unsigned char* myb = smem + lane * CK::BYTES;
  // column x's (H, E) record in this lane's ring
#define COL(x) (*(R*)(myb + ring_slot((x) >> 2, RC) * (64 * CK::BYTES) + ((x) & 3) * CK::REC))
  const long long begin = range[0], count = range[1];
  const uint32_t ntiles = (uint32_t)((count + 63) >> 6);
  if (ntiles == 0) return;  // an empty class: no atomics
  uint32_t tile = blockIdx.x;
  unsigned long long tile_cells_acc = 0;
  unsigned long long span_chunks = 0;  // chunks stepped, summed over rows
  for (;;) {
    if (persist) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(tile_ctr, 1u);
      tile = wave_first(__shfl(v, 0));
    }
    if (tile >= ntiles) break;
    const long long k = (long long)tile * 64 + lane;
    const bool valid = k < count;
    PairDesc pd;
    if (valid) {
      pd = desc[begin + k];
    } else {
      pd.qo = pd.to = 0;
      pd.ql = pd.tl = 0;
      pd.h0 = 1;
      pd.idx = 0;
      pd.pid = 0;
    }
    const KParams& P = kp[pd.pid];
    const int Lq = pd.ql, Lt = valid ? pd.tl : 0, h0 = pd.h0;
    const int oD = P.o_del, eD = P.e_del, oI = P.o_ins, eI = P.e_ins;
    const CellParams cp = {eD, P.oe_del, eI, SYM ? P.oe_del : P.oe_ins};
    const PkParams pp = {bcast(eD), bcast(P.oe_del), bcast(SYM ? P.oe_del : P.oe_ins),
                         bcast(eI), (s16x2){(short)eI, (short)(2 * eI)}};
    const int zd = P.zdrop;
    const int wb = band_cap(P, Lq);
    uint32_t pl[5], ph[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      pl[a] = P.prow[a][0];
      ph[a] = P.prow[a][1];
    }
    // first row of Eq. (3): H(-1, j-1) = max(0, h0 - o_ins - e_ins*j), E = 0,
    // for the columns the ring holds at the start; the rest come lazily
    int hw = imin(Lq, 4 * RC - 1);  // highest initialised column
    for (int c = 0; c < RC; ++c) {
      T w;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int j = 4 * c + cc;
        const int h = j == 0 ? h0 : imax(0, h0 - oI - eI * j);
        rec_set(w, cc, j <= hw ? (uint32_t)imin(h, CK::MAXV) : 0u);
      }
      my[c * 64] = w;
    }
    // query codes, four per dword, column-major tile
    {
      const uint8_t* qs = q + pd.qo;
      const int nq = (Lq + 3) >> 2;
      for (int c = 0; c < CAP / 4; ++c) {
        uint32_t w = 0;
        if (c < nq) {
          const int j = 4 * c;
          w = (uint32_t)qs[j];
          if (j + 1 < Lq) w |= (uint32_t)qs[j + 1] << 8;
          if (j + 2 < Lq) w |= (uint32_t)qs[j + 2] << 16;
          if (j + 3 < Lq) w |= (uint32_t)qs[j + 3] << 24;
        }
        qt[c * 64] = w;
      }
    }

    int best = h0, bi = -1, bj = -1, gbest = -1, gi = -1, moff = 0;
    int beg = 0, end = Lq, rows = 0, stop = 0;
    long long cells = 0;
    bool live = valid && Lt > 0;
    const uint8_t* ts = t + pd.to;
    // target codes of rows i..i+3 packed in tq; b0..b3 hold rows i+4..i+7,
    // loaded four rows before they are packed
    uint32_t tq = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    if (live) {
      b0 = ts[0];
      if (1 < Lt) b1 = ts[1];
      if (2 < Lt) b2 = ts[2];
      if (3 < Lt) b3 = ts[3];
    }
    for (int i = 0;; ++i) {
      live = live && i < Lt;
      if (__ballot(live) == 0) break;
      if ((i & 3) == 0) {
        tq = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
        if (live) {
          if (i + 4 < Lt) b0 = ts[i + 4];
          if (i + 5 < Lt) b1 = ts[i + 5];
          if (i + 6 < Lt) b2 = ts[i + 6];
          if (i + 7 < Lt) b3 = ts[i + 7];
        }
      }
      int hl = 0, f = 0;
      uint32_t lo = 0, hi = 0;
      if (live) {
        ++rows;
        // band (Sec. 5.1 (a)); the column leaving on the left is zeroed so
        // that everything left of beg stays zero
        if (beg < i - wb) {
          COL(beg) = 0;
          beg = i - wb;
        }
        end = imin(imin(end, i + wb + 1), Lq);
        if (end > beg) cells += end - beg;
        // columns entering the ring for the first time get their first-row
        // value
        while (hw < end) {
          ++hw;
          COL(hw) = (R)imax(0, h0 - oI - eI * hw);
        }
        const int tb = (tq >> (8 * (i & 3))) & 0xff;
        lo = pl[0];
        hi = ph[0];
#pragma unroll
        for (int a = 1; a < 5; ++a) {
          lo = tb == a ? pl[a] : lo;
          hi = tb == a ? ph[a] : hi;
        }
        hl = beg == 0 ? imax(0, h0 - oD - eD * (i + 1)) : 0;
      }
      const int rend = live ? end : 0;  // columns >= rend are masked
      // chunks [c0, cf) are inside the band end of every live lane and run
      // unmasked (dead lanes compute on their own private buffer, unused);
      // chunks [cf, c1) mask columns at or past each lane's end
      const int c0 = wave_min(live ? (beg >> 2) : 0x7fffffff);
      const int cf = wave_min(live ? (rend >> 2) : 0x7fffffff);
      const int c1 = wave_max(live ? ((rend + 3) >> 2) : 0);
      if (c1 > c0) span_chunks += (unsigned)(c1 - c0);
      int mkey = 0;
      // 8-bit unmasked chunks keep the row maximum per chunk: the largest
      // chunk maximum and the last chunk that reached it
      int mrun = -1, mch = 0;
      int c = c0;
      if (c < cf) {
        // two chunks per step, A = chunk c and B = chunk c+1; each load is
        // issued right after its register is last used and consumed in the
        // next step, so LDS and L2 latency overlap a whole step of work
        int sa = ring_slot(c, RC);
        int sb = sa + 1 == RC ? 0 : sa + 1;
        T chA = my[sa * 64], chB = my[sb * 64];
        // query dwords of this step (qA, qB) and of the next (qC, qD): the
        // tile may sit in L2 or beyond, so its loads get two steps
        uint32_t qA = qt[c * 64], qB = qt[(c + 1) * 64];
        uint32_t qC = qt[(c + 2) * 64], qD = qt[(c + 3) * 64];
        for (; c + 2 <= cf; c += 2) {
          const int sa2 = sb + 1 == RC ? 0 : sb + 1;
          const int sb2 = sa2 + 1 == RC ? 0 : sa2 + 1;
          {
            const uint32_t sc = __builtin_amdgcn_perm(hi, lo, qA);
            qA = qC;
            qC = qt[(c + 4) * 64];
            if constexpr (WB == 8) {
              int m4;
              my[sa * 64] = chunk_cells_pk<SYM>(chA, sc, hl, f, m4, pp);
              mch = m4 >= mrun ? c : mch;
              mrun = imax(mrun, m4);
            } else {
              my[sa * 64] = chunk_cells(chA, sc, 4 * c, hl, f, mkey, cp);
            }
            chA = my[sa2 * 64];
          }
          {
            const uint32_t sc = __builtin_amdgcn_perm(hi, lo, qB);
            qB = qD;
            qD = qt[(c + 5) * 64];
            if constexpr (WB == 8) {
              int m4;
              my[sb * 64] = chunk_cells_pk<SYM>(chB, sc, hl, f, m4, pp);
              mch = m4 >= mrun ? c + 1 : mch;
              mrun = imax(mrun, m4);
            } else {
              my[sb * 64] = chunk_cells(chB, sc, 4 * c + 4, hl, f, mkey, cp);
            }
            chB = my[sb2 * 64];
          }
          sa = sa2;
          sb = sb2;
        }
        if (c < cf) {
          const uint32_t sc = __builtin_amdgcn_perm(hi, lo, qA);
          if constexpr (WB == 8) {
            int m4;
            my[sa * 64] = chunk_cells_pk<SYM>(chA, sc, hl, f, m4, pp);
            mch = m4 >= mrun ? c : mch;
            mrun = imax(mrun, m4);
          } else {
            my[sa * 64] = chunk_cells(chA, sc, 4 * c, hl, f, mkey, cp);
          }
          ++c;
        }
      }
      if constexpr (WB == 8) {
        for (; c < c1; ++c) {
          const int sl = ring_slot(c, RC);
          const uint32_t sc = __builtin_amdgcn_perm(hi, lo, qt[c * 64]);
          int m4;
          my[sl * 64] = chunk_cells_pk_masked<SYM>(my[sl * 64], sc, rend - 4 * c, hl, f, m4, pp);
          mch = m4 >= mrun ? c : mch;
          mrun = imax(mrun, m4);
        }
      }
      for (; c < c1; ++c) {
        const int j0 = 4 * c;
        if (j0 < rend) {
          const int sl = ring_slot(c, RC);
          T ch = my[sl * 64];
          const uint32_t sc = __builtin_amdgcn_perm(hi, lo, qt[c * 64]);
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const int j = j0 + cc;
            if (j < rend) {
              const uint32_t r = rec_get(ch, cc);
              constexpr uint32_t M = (1u << WB) - 1;
              int key;
              rec_set(ch, cc,
                      cell<WB>(r & M, r >> WB, (int)(int8_t)(sc >> (8 * cc)), j, hl, f,
                               key, cp));
              mkey = imax(mkey, key);
            }
          }
          my[sl * 64] = ch;
        }
      }
      if (live) {
        // right edge (R8): H(i, end-1) at index end; E there is already 0.
        // With 8-bit records the masked chunk holding column end wrote it;
        // when end is a chunk boundary no chunk held it, and the last chunk
        // was fully inside the band, so hl is H(i, end-1)
        if (WB != 8 || end == 4 * c1) COL(end) = (R)(hl & CK::MAXV);
        // best score touching the end of the query (Sec. 5.4 (b))
        if (imax(beg, end) == Lq) {
          const int hend = WB == 8 ? (int)(COL(end) & 0xff) : hl;
          gi = hend >= gbest ? i : gi;
          gbest = imax(gbest, hend);
        }
        // row maximum (ties to the larger column): for 8-bit records the
        // chunks keep the largest chunk maximum and the last chunk that
        // reached it; the column is the last of that chunk's cells inside
        // the band holding the maximum, whose H(i, j) now sit at j + 1
        int m = mkey >> 9, mj = mkey & 511;
        if (WB == 8) {
          m = imax(mrun, 0);  // no chunk at all: an empty band
          const int j0 = 4 * mch;
          mj = imin(j0 + 3, end - 1);
          while (mj > j0 && (int)(COL(mj + 1) & 0xff) != m) --mj;
        }
        if (m == 0) {
          stop = 1;
          live = false;
        } else if (m > best) {
          best = m;
          bi = i;
          bj = mj;
          moff = imax(moff, mj > i ? mj - i : i - mj);
        } else if (zd > 0) {
          const int drift = (i - bi) - (mj - bj);
          const int drop = best - m - (drift > 0 ? drift * eD : -drift * eI);
          if (drop > zd) {
            stop = 2;
            live = false;
          }
        }
        if (live) {
          // shrink the band by its empty ends (Sec. 5.1 (c))
          while (beg < end && COL(beg) == 0) ++beg;
          int x = end;
          while (x >= beg && COL(x) == 0) --x;
          end = imin(x + 2, Lq);
        }
      }
    }
    unsigned long long my_cells = 0;
    if (valid) {
      const int slack = P.amax - P.oe_del > 0 ? P.amax - P.oe_del : 0;
      if (best + slack > CK::MAXV) {
        // some stored value may have needed a wider record: rerun wider
        const unsigned long long pos =
            atomicAdd((unsigned long long*)ovf_count, 1ull);
        ovf[pos] = pd;
      } else {
        my_cells = (unsigned long long)cells;
        bsw_result res;
        res.score = best;
        res.qle = bj + 1;
        res.tle = bi + 1;
        res.gtle = gi + 1;
        res.gscore = gbest;
        res.max_off = moff;
        out[pd.idx] = res;
        if (diag) {
          bsw_diag dg;
          dg.rows = rows;
          dg.stop = stop;
          dg.cells = cells;
          diag[pd.idx] = dg;
        }
      }
    }
    tile_cells_acc += my_cells;
    if (!persist) break;
  }
  tile_cells_acc = wave_sum64(tile_cells_acc);
  if (lane == 0 && tile_cells_acc) atomicAdd(cls_cells, tile_cells_acc);
  if (lane == 0 && span_chunks) atomicAdd(work_cells, span_chunks * 4ull * 64ull);
#undef COL
}

// One pair per wave (the reruns of pairs whose values need more than their
// class's record width): the 64 lanes take 64 consecutive columns of a row
// at a time, with 32-bit values, so a pair's rows take a few wave steps
// each instead of one lane's sequential walk.  Along the row only F is
// sequential; unrolled over a block of columns it is a max-plus prefix:
// F(jb + l) = max(0, F(jb) - l e, max over l' < l of (M(jb + l') - o - e +
// l' e) - (l - 1) e) with the insertion costs o, e, taken with a wave scan.
// The row buffer (H shifted by one column, and E, Sec. 5.1) holds every
// column of the query in LDS and is never reset, as in the one-lane form.
constexpr int WAVE_CAP = 256;  // longest query of the wave kernel
constexpr int NEG = -(1 << 30);

__device__ __forceinline__ int wave_prefix_max_excl(int x) {
  // shift the inclusive scan one lane up across the whole wave; lane 0 and
  // lanes after NEG-only prefixes read NEG
  return imax(__builtin_amdgcn_update_dpp((int)0x80000000u, wave_scan<true>(x), 0x138, 0xf,
                                          0xf, false),
              NEG);
}

__global__ void __launch_bounds__(64)
k_wave(const PairDesc* __restrict__ desc, const long long* __restrict__ range,
       const uint8_t* __restrict__ q, const uint8_t* __restrict__ t,
       const KParams* __restrict__ kp, bsw_result* __restrict__ out,
       bsw_diag* __restrict__ diag, uint32_t* ctr, const Status* st,
       unsigned long long* __restrict__ cls_cells) {
  if (st->bad) return;
  __shared__ int2 hb[WAVE_CAP + 1];
  const int lane = threadIdx.x;
  const long long begin = range[0], count = range[1];
  if (count <= 0) return;  // an empty list: no atomics
  unsigned long long acc = 0;
  for (;;) {
    uint32_t v0 = 0;
    if (lane == 0) v0 = atomicAdd(ctr, 1u);
    const uint32_t k = wave_first(__shfl(v0, 0));
    if (k >= count) break;
    const PairDesc pd = desc[begin + k];
    const KParams& P = kp[pd.pid];
    const int Lq = pd.ql, Lt = pd.tl, h0 = pd.h0;
    const int oD = P.o_del, eD = P.e_del, oI = P.o_ins, eI = P.e_ins;
    const int oeD = P.oe_del, oeI = P.oe_ins, zd = P.zdrop;
    const int wb = band_cap(P, Lq);
    const uint8_t* qs = q + pd.qo;
    const uint8_t* ts = t + pd.to;
    // first row of Eq. (3)
    for (int j = lane; j <= Lq; j += 64)
      hb[j] = make_int2(j == 0 ? h0 : imax(0, h0 - oI - eI * j), 0);
    __syncthreads();
    int best = h0, bi = -1, bj = -1, gbest = -1, gi = -1, moff = 0;
    int beg = 0, end = Lq, rows = 0, stop = 0;
    long long cells = 0;
    for (int i = 0; i < Lt; ++i) {
      ++rows;
      beg = imax(beg, i - wb);
      end = imin(imin(end, i + wb + 1), Lq);
      if (end > beg) cells += end - beg;
      const int tb = ts[i];
      uint32_t lo = P.prow[0][0], hi = P.prow[0][1];
#pragma unroll
      for (int a = 1; a < 5; ++a) {
        lo = tb == a ? P.prow[a][0] : lo;
        hi = tb == a ? P.prow[a][1] : hi;
      }
      int hl = beg == 0 ? imax(0, h0 - oD - eD * (i + 1)) : 0;  // H(i, jb - 1)
      int fin = 0;                                                 // F(i, jb)
      int m = 0, mj = -1;
      for (int jb = beg; jb < end; jb += 64) {
        const int j = jb + lane;
        const bool in = j < end;
        const int2 r = in ? hb[j] : make_int2(0, 0);
        const int s = in ? score_of(lo, hi, qs[j]) : 0;
        const int M = r.x > 0 ? r.x + s : 0;
        const int en = imax(imax(r.y - eD, M - oeD), 0);
        const int X = wave_prefix_max_excl(in ? M - oeI + lane * eI : NEG);
        const int F = imax(imax(fin - lane * eI, X - (lane - 1) * eI), 0);
        const int h = imax(imax(M, r.y), F);
        const int Fn = imax(imax(F - eI, M - oeI), 0);
        const int hprev = __shfl_up(h, 1, 64);
        if (in) hb[j] = make_int2(lane ? hprev : hl, en);
        const int hv = in ? h : -1;
        const int bm = wave_max(hv);
        if (bm >= m) {
          m = bm;
          mj = jb + 63 - __builtin_clzll(__ballot(hv == bm));
        }
        const int last = imin(63, end - 1 - jb);
        hl = __builtin_amdgcn_readlane(h, last);
        fin = __builtin_amdgcn_readlane(Fn, last);
      }
      // right edge (R8): H(i, end-1), E = 0 at index end
      if (lane == 0) hb[end] = make_int2(hl, 0);
      __syncthreads();
      if (imax(beg, end) == Lq) {
        gi = hl >= gbest ? i : gi;
        gbest = imax(gbest, hl);
      }
      if (m == 0) {
        stop = 1;
        break;
      }
      if (m > best) {
        best = m;
        bi = i;
        bj = mj;
        moff = imax(moff, mj > i ? mj - i : i - mj);
      } else if (zd > 0) {
        const int drift = (i - bi) - (mj - bj);
        const int drop = best - m - (drift > 0 ? drift * eD : -drift * eI);
        if (drop > zd) {
          stop = 2;
          break;
        }
      }
      // shrink the band by its empty ends (Sec. 5.1 (c))
      int nb = end;
      for (int jb = beg; jb < end; jb += 64) {
        const int j = jb + lane;
        const unsigned long long mk =
            __ballot(j < end && (hb[j].x != 0 || hb[j].y != 0));
        if (mk) {
          nb = jb + __builtin_ctzll(mk);
          break;
        }
      }
      beg = nb;
      int x = beg - 1;
      for (int jt = end; jt >= beg; jt -= 64) {
        const int j = jt - lane;
        const unsigned long long mk =
            __ballot(j >= beg && (hb[j].x != 0 || hb[j].y != 0));
        if (mk) {
          x = jt - __builtin_ctzll(mk);
          break;
        }
      }
      end = imin(x + 2, Lq);
    }
    if (lane == 0) {
      bsw_result res;
      res.score = best;
      res.qle = bj + 1;
      res.tle = bi + 1;
      res.gtle = gi + 1;
      res.gscore = gbest;
      res.max_off = moff;
      out[pd.idx] = res;
      if (diag) {
        bsw_diag dg;
        dg.rows = rows;
        dg.stop = stop;
        dg.cells = cells;
        diag[pd.idx] = dg;
      }
      acc += (unsigned long long)cells;
    }
    __syncthreads();  // the next pair rewrites the row buffer
  }
  if (lane == 0 && acc) atomicAdd(cls_cells, acc);
}

// ---------------------------------------------------------------------------
// Wave mode with the row in registers (32-bit values, queries up to
// 64 * NSEG).  The intra-task form of Sec. 5.2.1 for pairs whose values or
// bands are wide: one pair per wave, lane l holding columns l, l + 64, ...
// of the row buffer (H shifted by one column, and E) in registers, so a
// row is NSEG wave steps of 64 columns.  Only F runs along the row; within
// a step it is a max-plus prefix over the lanes (a DPP scan),
//   F(jb + l) = max(0, F(jb) - l e, max_{l' < l} (M(jb + l') - o - e + l' e)
//                   - (l - 1) e)      (insertion costs o, e),
// and the step's last F and H carry into the next step.  All per-pair state
// is wave-uniform.  The right-edge column 64 * NSEG (only reached when the
// query fills the class) is a wave-uniform scalar: it is never inside a
// band, so only its H (the query-end score) is ever read.

__device__ __forceinline__ int wave_max_i(int v) { return wave_max(v); }

template <int NSEG>
__global__ void __launch_bounds__(64)
k_wavev(const PairDesc* __restrict__ desc, const long long* __restrict__ range,
        const uint8_t* __restrict__ q, const uint8_t* __restrict__ t,
        const KParams* __restrict__ kp, bsw_result* __restrict__ out,
        bsw_diag* __restrict__ diag, uint32_t* ctr, const Status* st,
        unsigned long long* __restrict__ cls_cells,
        unsigned long long* __restrict__ work_cells) {
  if (st->bad) return;
  constexpr int CAPW = 64 * NSEG;
  const int lane = threadIdx.x;
  const long long begin = range[0], count = range[1];
  if (count <= 0) return;  // an empty list: no atomics
  unsigned long long acc = 0, span = 0;
  for (;;) {
    uint32_t v0 = 0;
    if (lane == 0) v0 = atomicAdd(ctr, 1u);
    const uint32_t k = wave_first(__shfl(v0, 0));
    if (k >= count) break;
    const PairDesc pd = desc[begin + k];
    const KParams& P = kp[pd.pid];
    const int Lq = pd.ql, Lt = pd.tl, h0 = pd.h0;
    const int oD = P.o_del, eD = P.e_del, oI = P.o_ins, eI = P.e_ins;
    const int oeD = P.oe_del, oeI = P.oe_ins, zd = P.zdrop;
    const int wb = band_cap(P, Lq);
    const uint8_t* qs = q + pd.qo;
    const uint8_t* ts = t + pd.to;
    // row buffer: first row of Eq. (3), E = 0; query codes
    int hd[NSEG], ev[NSEG];
    uint32_t qc[NSEG];
#pragma unroll
    for (int sg = 0; sg < NSEG; ++sg) {
      const int j = lane + 64 * sg;
      hd[sg] = j == 0 ? h0 : (j <= Lq ? imax(0, h0 - oI - eI * j) : 0);
      ev[sg] = 0;
      qc[sg] = j < Lq ? qs[j] : 0u;
    }
    int hcap = Lq == CAPW ? imax(0, h0 - oI - eI * CAPW) : 0;  // column CAPW
    int best = h0, bi = -1, bj = -1, gbest = -1, gi = -1, moff = 0;
    int beg = 0, end = Lq, rows = 0, stop = 0;
    long long cells = 0;
    uint32_t tnext = Lt > 0 ? ts[0] : 0u;
    for (int i = 0; i < Lt; ++i) {
      ++rows;
      const uint32_t tb = tnext;
      if (i + 1 < Lt) tnext = ts[i + 1];
      beg = imax(beg, i - wb);
      end = imin(imin(end, i + wb + 1), Lq);
      if (end > beg) cells += end - beg;
      const uint32_t lo = P.prow[tb][0], hi = P.prow[tb][1];
      const int hl = beg == 0 ? imax(0, h0 - oD - eD * (i + 1)) : 0;  // H(i, beg - 1)
      int hin = hl;   // H(i, jb - 1) entering a step
      int fin = 0;    // F(i, jb) entering a step
      int lh = -1, lj = -1;  // this lane's row maximum and its column
      // steps holding the band and its right-edge column (just the right
      // edge when the band is empty)
      const int s0 = imin(beg, end) >> 6, s1 = end >> 6;
      span += (unsigned)(imin(s1, NSEG - 1) + 1 - imin(s0, NSEG));
      // the steps s0 .. s1 as a bit mask (one scalar test per step)
      const uint32_t steps = (s1 >= 31 ? ~0u : ((2u << s1) - 1u)) & (~0u << imin(s0, 31));
      // j in [beg, end) as one unsigned compare
      const uint32_t blen = (uint32_t)imax(end - beg, 0);
#pragma unroll
      for (int sg = 0; sg < NSEG; ++sg) {
        if (!(steps & (1u << sg))) continue;
        const int jb = 64 * sg, j = jb + lane;
        const bool in = (uint32_t)(j - beg) < blen;
        const int d = hd[sg], e = ev[sg];
        const int sc = score_of(lo, hi, qc[sg]);
        const int M = d > 0 ? d + sc : 0;
        const int X = wave_prefix_max_excl(in ? M - oeI + lane * eI : NEG);
        const int F = imax(imax(fin - lane * eI, X - (lane - 1) * eI), 0);
        const int h = imax(imax(M, e), F);
        const int Fn = imax(imax(F - eI, M - oeI), 0);
        // H(i, j - 1) for this lane's column: the lane below, or the value
        // carried in from the previous step
        int hp = __builtin_amdgcn_update_dpp(0, h, 0x138, 0xf, 0xf, false);  // wave_shr:1
        hp = lane == 0 ? hin : hp;
        // the band's first column and the right edge of an empty band take
        // the row's left boundary H(i, beg - 1)
        if (j == (beg < end ? beg : end)) hp = hl;
        // stored: the band's columns and the right edge, by selects (the
        // empty asm keeps the new E from being sunk into a branch, whose
        // exec-mask bookkeeping would load the scalar unit)
        int en = imax(imax(e - eD, M - oeD), 0);
        asm volatile("" : "+v"(en));
        const bool st_col = in || j == end;
        hd[sg] = st_col ? hp : d;
        ev[sg] = st_col ? (in ? en : 0) : e;
        if (in && h >= lh) {
          lh = h;
          lj = j;
        }
        hin = __builtin_amdgcn_readlane(h, 63);
        fin = __builtin_amdgcn_readlane(Fn, 63);
      }
      // right edge in the scalar column CAPW (R8)
      if (end == CAPW) hcap = hin;
      // row maximum, ties to the larger column (R15)
      const int m = imax(wave_max_i(lh), 0);
      const int mj = wave_max_i(lh == m && m > 0 ? lj : -1);
      // best score touching the end of the query (Sec. 5.4 (b)): the stored
      // H(i, end - 1) at column end
      if (imax(beg, end) == Lq) {
        int hend;
        if (end == CAPW) {
          hend = hcap;
        } else {
          hend = 0;
#pragma unroll
          for (int sg = 0; sg < NSEG; ++sg)
            if ((end >> 6) == sg) hend = __builtin_amdgcn_readlane(hd[sg], end & 63);
        }
        gi = hend >= gbest ? i : gi;
        gbest = imax(gbest, hend);
      }
      if (m == 0) {
        stop = 1;
        break;
      }
      if (m > best) {
        best = m;
        bi = i;
        bj = mj;
        moff = imax(moff, mj > i ? mj - i : i - mj);
      } else if (zd > 0) {
        const int drift = (i - bi) - (mj - bj);
        const int drop = best - m - (drift > 0 ? drift * eD : -drift * eI);
        if (drop > zd) {
          stop = 2;
          break;
        }
      }
      // shrink the band by its empty ends (Sec. 5.1 (c)): the first
      // non-empty index in [beg, end) (else end), the last one in [beg,
      // end] (else beg - 1); each lane takes its own columns first, then
      // one wave reduction (vector work rather than a chain of scalar
      // tests, which the scalar unit of a busy CU cannot keep up with)
      int jlo = 0x7fffffff;
#pragma unroll
      for (int sg = NSEG - 1; sg >= 0; --sg) {
        const int j = lane + 64 * sg;
        if ((uint32_t)(j - beg) < blen && (hd[sg] | ev[sg]) != 0) jlo = j;
      }
      const int nb = imin(wave_min(jlo), end);
      int jhi = -1;
#pragma unroll
      for (int sg = 0; sg < NSEG; ++sg) {
        const int j = lane + 64 * sg;
        if ((uint32_t)(j - nb) <= (uint32_t)(end - nb) && (hd[sg] | ev[sg]) != 0) jhi = j;
      }
      int x = imax(wave_max(jhi), nb - 1);
      if (end == CAPW && hcap != 0) x = CAPW;
      beg = nb;
      end = imin(x + 2, Lq);
    }
    if (lane == 0) {
      bsw_result res;
      res.score = best;
      res.qle = bj + 1;
      res.tle = bi + 1;
      res.gtle = gi + 1;
      res.gscore = gbest;
      res.max_off = moff;
      out[pd.idx] = res;
      if (diag) {
        bsw_diag dg;
        dg.rows = rows;
        dg.stop = stop;
        dg.cells = cells;
        diag[pd.idx] = dg;
      }
    }
    acc += (unsigned long long)cells;
  }
  if (lane == 0 && acc) atomicAdd(cls_cells, acc);
  if (lane == 0 && span) atomicAdd(work_cells, span * 64ull);
}

// Queries longer than 256: one pair per wave, lane 0 runs it with a
// 32-bit row buffer in HBM (slot per wave); waves pull pairs from a counter.
__global__ void __launch_bounds__(64)
k_long(const PairDesc* __restrict__ desc, const long long* __restrict__ range,
       const uint8_t* __restrict__ q, const uint8_t* __restrict__ t,
       const KParams* __restrict__ kp, bsw_result* __restrict__ out,
       bsw_diag* __restrict__ diag, uint32_t* ctr, int2* __restrict__ gbuf,
       uint8_t* __restrict__ gq, const Status* st,
       unsigned long long* __restrict__ cls_cells) {
  if (st->bad) return;
  const long long begin = range[0], count = range[1];
  if (count <= 0) return;  // an empty list: no atomics
  int2* hb = gbuf + (size_t)blockIdx.x * LONG_SLOT_COLS;
  uint8_t* qb = gq + (size_t)blockIdx.x * LONG_SLOT_COLS;
  for (;;) {
    uint32_t v = 0;
    if (threadIdx.x == 0) v = atomicAdd(ctr, 1u);
    const uint32_t k = wave_first(__shfl(v, 0));
    if (k >= count) break;
    if (threadIdx.x == 0) {
      const PairDesc pd = desc[begin + k];
      const long long c = extend_pair<W32, 1>(pd, kp[pd.pid], q, t, hb, qb, out, diag);
      atomicAdd(cls_cells, (unsigned long long)c);
    }
  }
}

}  // namespace bsw

// ---------------------------------------------------------------------------
// host-side launchers (called by the runtime in bsw_host.cpp)

namespace bsw {

static int cls_cap(int cls) {
  if (cls < CLS_W16) return L8_CAP[cls - CLS_L8];
  if (cls < CLS_W32) return LW_CAP[cls - CLS_W16];
  return LW_CAP[cls - CLS_W32];
}

// register-row classes (8-bit records), chunked classes with an LDS ring
// (16-bit records) and the 32-bit kernel with a private LDS row
static bool regrow(int cls) { return cls < CLS_W16; }
static bool chunked(int cls) { return cls >= CLS_W16 && cls < CLS_W32; }
static int rec_bytes(int cls) { return cls < CLS_W16 ? 8 : 16; }

// LDS bytes per wave of a class (register-row classes: the nonzero-byte
// mirror; chunked classes: without a ring)
size_t lane_lds_per_wave(int cls) {
  const int cap = cls_cap(cls);
  if (regrow(cls)) return (size_t)(cap / 4 + 1) * 64 * 4;
  if (chunked(cls)) return (size_t)(cap / 4 + 1) * 64 * rec_bytes(cls);
  return (size_t)(cap + 1) * 64 * 8 + (size_t)cap * 64;
}

// LDS bytes per 64-lane chunk row of a chunked class
size_t lane_chunk_row_bytes(int cls) { return (size_t)64 * rec_bytes(cls); }

// waves per workgroup: register-row and chunked classes run one wave per
// group; the 32-bit kernel as many as fit in 64 KiB of LDS (1..4)
int lane_waves_per_block(int cls) {
  if (regrow(cls) || chunked(cls)) return 1;
  const size_t b = lane_lds_per_wave(cls);
  int w = (int)(65536 / b);
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

typedef void (*LaneFn)(const PairDesc*, const long long*, const uint8_t*,
                       const uint8_t*, const KParams*, bsw_result*, bsw_diag*,
                       uint32_t*, const Status*, unsigned long long*);
typedef void (*LaneCFn)(const PairDesc*, const long long*, const uint8_t*,
                        const uint8_t*, const KParams*, bsw_result*, bsw_diag*,
                        uint32_t*, const Status*, uint32_t*, PairDesc*, long long*, int,
                        int, unsigned long long*, unsigned long long*);

static LaneVFn lanev_fn(int cls, bool sym) {
  switch (L8_CAP[cls - CLS_L8]) {
    case 32: return lanev_kernel<32>(sym);
    case 64: return lanev_kernel<64>(sym);
    case 96: return lanev_kernel<96>(sym);
    case 128: return lanev_kernel<128>(sym);
    case 160: return lanev_kernel<160>(sym);
    case 192: return lanev_kernel<192>(sym);
    case 224: return lanev_kernel<224>(sym);
    default: return lanev_kernel<256>(sym);
  }
}

static LaneCFn lanec_fn(int cls, bool sym) {
  static const LaneCFn tab16[2][NLW] = {
      {k_lanec<32, false, 16>, k_lanec<64, false, 16>, k_lanec<128, false, 16>,
       k_lanec<256, false, 16>},
      {k_lanec<32, true, 16>, k_lanec<64, true, 16>, k_lanec<128, true, 16>,
       k_lanec<256, true, 16>}};
  return tab16[sym ? 1 : 0][cls - CLS_W16];
}

static LaneFn lanew_fn(int cls, bool persist) {
  static const LaneFn tab[2][NLW] = {
      {k_lane<W32, 32, false>, k_lane<W32, 64, false>, k_lane<W32, 128, false>,
       k_lane<W32, 256, false>},
      {k_lane<W32, 32, true>, k_lane<W32, 64, true>, k_lane<W32, 128, true>,
       k_lane<W32, 256, true>}};
  return tab[persist ? 1 : 0][cls - CLS_W32];
}

// kernel symbol of a class (for chunked classes "flag" selects the
// symmetric-gap variant, for the 32-bit kernel the persistent one)
static const void* lane_sym(int cls, bool flag) {
  if (regrow(cls)) return (const void*)lanev_fn(cls, flag);
  return chunked(cls) ? (const void*)lanec_fn(cls, flag) : (const void*)lanew_fn(cls, flag);
}

hipError_t lane_setup(int cls, bool flag) {
  const size_t lds = lane_lds_per_wave(cls) * lane_waves_per_block(cls);
  return hipFuncSetAttribute(lane_sym(cls, flag),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// resident workgroups per CU for a lane-mode class, given the LDS bytes
// per workgroup (0 = the class's full row buffer)
int lane_blocks_per_cu(int cls, bool flag, size_t lds) {
  int nb = 0;
  const int wpb = lane_waves_per_block(cls);
  if (!lds) lds = lane_lds_per_wave(cls) * wpb;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lane_sym(cls, flag), wpb * 64,
                                                   lds) != hipSuccess)
    return 1;
  return nb < 1 ? 1 : nb;
}

// ring chunks of a chunked class for band half-widths up to wmax: enough
// for the live band (4*RC > 2w' + 4, plus a spare chunk), and at least half
// of the chunks a query of the class can touch, so that one conditional
// subtraction maps every chunk index (at most full - 1) into the ring
int lane8_ring_chunks(int cls, int wmax) {
  const int full = cls_cap(cls) / 4 + 1;
  long long need = (2LL * wmax + 5 + 3) / 4 + 1;
  if (need < (full + 1) / 2) need = (full + 1) / 2;
  return need >= full ? full : (int)need;
}

// HBM words of query tile per workgroup of a chunked class: the chunks of
// the longest query plus the ones the loads run ahead by
size_t lane8_qtile_words(int cls) { return ((size_t)cls_cap(cls) / 4 + 6) * 64; }

void launch_fill(uint32_t* p, int64_t nwords, hipStream_t s) {
  int64_t blocks = (nwords + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, nwords);
}

void launch_prep(int64_t n, const uint8_t* q, const uint8_t* t, const uint64_t* q_off,
                 const uint64_t* q_end, const uint64_t* t_off, const uint64_t* t_end,
                 const int32_t* h0, const uint8_t* pid, int n_params, const KParams* kp,
                 int min_bits, int spec16, uint32_t* keys, uint32_t* hist, Status* st,
                 hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)blocks), dim3(256), 0, s, n, q, t, q_off,
                     q_end, t_off, t_end, h0, pid, n_params, kp, min_bits, spec16, keys,
                     hist, st);
}

// bytes = the sequence bytes when the host knows them (sizes the grid at
// 4 KiB per group), or 0 for the full grid
void launch_codes(const uint8_t* seq, const uint64_t* off, int64_t n, Status* st,
                  uint64_t bytes, hipStream_t s) {
  uint64_t blocks = bytes ? (bytes + 4095) / 4096 : 4096;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_codes, dim3((unsigned)blocks), dim3(256), 0, s, seq, off, n, st);
}

void launch_scan(const uint32_t* hist, uint32_t* cursor, long long* cls_range,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, hist, cursor, cls_range);
}

void launch_scatter(int64_t n, const uint64_t* q_off, const uint64_t* q_end,
                    const uint64_t* t_off, const uint64_t* t_end, const int32_t* h0,
                    const uint8_t* pid, const uint32_t* keys, uint32_t* cursor,
                    PairDesc* desc, const Status* st, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, n, q_off, q_end,
                     t_off, t_end, h0, pid, keys, cursor, desc, st);
}

void launch_gather(const CopySeg* segs, int ns, unsigned long long nchunks, hipStream_t s) {
  if (!nchunks) return;
  const unsigned blocks = (unsigned)(nchunks < 1024 ? nchunks : 1024);
  hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, s, segs, ns, nchunks);
}

void launch_req_codes(const ReqSlice* tab, int m, int64_t n, const uint8_t* base,
                      unsigned long long* bad, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_req_codes, dim3((unsigned)blocks), dim3(256), 0, s, tab, m, n, base, bad);
}

void launch_assemble(const ReqSlice* tab, int m, int64_t n, uint64_t* qb, uint64_t* qe,
                     uint64_t* tb, uint64_t* te, int32_t* h0, uint8_t* pid,
                     const unsigned long long* bad, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(256), 0, s, tab, m, n, qb, qe,
                     tb, te, h0, pid, bad);
}

void launch_lane(int cls, bool persist, unsigned blocks, const PairDesc* desc,
                 const long long* range, const uint8_t* q, const uint8_t* t,
                 const KParams* kp, bsw_result* out, bsw_diag* diag,
                 uint32_t* tile_ctr, const Status* st, uint32_t* qtiles,
                 PairDesc* ovf, long long* ovf_count, int ring, bool sym,
                 unsigned long long* cls_cells, unsigned long long* work_cells,
                 hipStream_t s) {
  const int wpb = lane_waves_per_block(cls);
  if (regrow(cls))
    hipLaunchKernelGGL(lanev_fn(cls, sym), dim3(blocks), dim3(64), lane_lds_per_wave(cls), s,
                       desc, range, q, t, kp, out, diag, tile_ctr, st, ovf, ovf_count,
                       persist ? 1 : 0, cls_cells, work_cells);
  else if (chunked(cls))
    hipLaunchKernelGGL(lanec_fn(cls, sym), dim3(blocks), dim3(64),
                       (size_t)ring * lane_chunk_row_bytes(cls), s, desc, range, q, t, kp,
                       out, diag, tile_ctr, st, qtiles, ovf, ovf_count, persist ? 1 : 0,
                       ring, cls_cells, work_cells);
  else
    hipLaunchKernelGGL(lanew_fn(cls, persist), dim3(blocks), dim3(wpb * 64),
                       lane_lds_per_wave(cls) * wpb, s, desc, range, q, t, kp, out, diag,
                       tile_ctr, st, cls_cells);
}

void launch_wave(unsigned blocks, const PairDesc* desc, const long long* range,
                 const uint8_t* q, const uint8_t* t, const KParams* kp, bsw_result* out,
                 bsw_diag* diag, uint32_t* ctr, const Status* st,
                 unsigned long long* cls_cells, hipStream_t s) {
  hipLaunchKernelGGL(k_wave, dim3(blocks), dim3(64), 0, s, desc, range, q, t, kp, out, diag,
                     ctr, st, cls_cells);
}

typedef void (*WaveVFn)(const PairDesc*, const long long*, const uint8_t*, const uint8_t*,
                        const KParams*, bsw_result*, bsw_diag*, uint32_t*, const Status*,
                        unsigned long long*, unsigned long long*);

// wave-mode kernel of a 32-bit class: steps of 64 columns covering its cap
static WaveVFn wavev_fn(int cls) {
  const int cap = cls_cap(cls);
  if (cap <= 64) return k_wavev<1>;
  if (cap <= 128) return k_wavev<2>;
  return k_wavev<4>;
}

int wavev_blocks_per_cu(int cls) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wavev_fn(cls), 64, 0) != hipSuccess)
    return 1;
  return nb < 1 ? 1 : nb;
}

void launch_wavev(int cls, unsigned blocks, const PairDesc* desc, const long long* range,
                  const uint8_t* q, const uint8_t* t, const KParams* kp, bsw_result* out,
                  bsw_diag* diag, uint32_t* ctr, const Status* st,
                  unsigned long long* cls_cells, unsigned long long* work_cells,
                  hipStream_t s) {
  hipLaunchKernelGGL(wavev_fn(cls), dim3(blocks), dim3(64), 0, s, desc, range, q, t, kp, out,
                     diag, ctr, st, cls_cells, work_cells);
}

int wave_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_wave, 64, 0) != hipSuccess) return 1;
  return nb < 1 ? 1 : nb;
}

// slots waves, wave w using row-buffer slot w of gbuf / gq
void launch_long(int slots, const PairDesc* desc, const long long* range, const uint8_t* q,
                 const uint8_t* t, const KParams* kp, bsw_result* out,
                 bsw_diag* diag, uint32_t* ctr, int2* gbuf, uint8_t* gq,
                 const Status* st, unsigned long long* cls_cells, hipStream_t s) {
  hipLaunchKernelGGL(k_long, dim3(slots), dim3(64), 0, s, desc, range, q, t,
                     kp, out, diag, ctr, gbuf, gq, st, cls_cells);
}

}  // namespace bsw
