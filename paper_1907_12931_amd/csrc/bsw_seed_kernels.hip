// bsw_seed_kernels.hip -- kernels of the read-level seed driver (the step
// around BSW: each seed is extended to the left, then to the right, Sec. 2
// and Sec. 5.3.2).  The DP itself runs in the BSW pipeline; these kernels
// only build its pair tables and read its results:
//   k_seed_offsets the {0, length} offset pairs of the code checks
//   k_seed_setup   check each seed and write the pair tables of both sides
//   k_reverse      reversed copy of a sequence buffer (the left side runs
//                  forward over reversed reads and reference, so its pairs
//                  are plain slices of the reversed buffers)
//   k_seed_mid     the end kept after the left side and the right side's h0
//   k_seed_finish  the end kept after the right side, and the output records
//   k_seed_filter  after extension: the seeds an alignment of their chain
//                  already covers (Sec. 5.3.2 extends every seed first)
// One thread per seed in every per-seed kernel; grid-stride loops.
#include <hip/hip_runtime.h>

#include "../../include/bsw.h"
#include "bsw_internal.h"
#include "bsw_seed_internal.h"

namespace bsw {

namespace {

__device__ __forceinline__ void flag_bad(Status* st, int64_t k) {
  atomicMax(&st->first_bad_inv, ~(unsigned long long)k);
  atomicOr(&st->bad, 1u);
}

// The end kept after one side: the read end when its score is positive and
// higher than the best score less the end bonus, else the best cell.
struct Kept {
  int32_t score, qlen, how;
  int32_t tlen;
};

__device__ __forceinline__ Kept keep_end(const bsw_result& r, int32_t bonus, int32_t qlen) {
  Kept k;
  if (r.gscore <= 0 || r.gscore <= r.score - bonus) {
    k.score = r.score;
    k.qlen = r.qle;
    k.tlen = r.tle;
    k.how = BSW_END_LOCAL;
  } else {
    k.score = r.gscore;
    k.qlen = qlen;
    k.tlen = r.gtle;
    k.how = BSW_END_READ;
  }
  return k;
}

}  // namespace

__global__ void k_seed_offsets(uint64_t* offs, uint64_t reads_len, uint64_t ref_len) {
  offs[0] = 0;
  offs[1] = reads_len;
  offs[2] = 0;
  offs[3] = ref_len;
}

// Every seed with a bad field, and every seed of a call whose reads or
// reference hold a code > 4, gets empty pairs on both sides: the pipeline
// then reads no sequence byte for it, and the call fails when it completes.
__global__ void __launch_bounds__(256)
k_seed_setup(const bsw_seed* __restrict__ seeds, int64_t n,
             const uint64_t* __restrict__ read_off, int64_t n_reads, uint64_t reads_len,
             uint64_t ref_len, int32_t w, SeedTables T, Status* sts) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool codes_bad = sts[ST_READS].bad || sts[ST_REF].bad;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = tid; k < n; k += stride) {
    const bsw_seed sd = seeds[k];
    bool ok = sd.read >= 0 && sd.read < n_reads;
    uint64_t r0 = 0, r1 = 0;
    if (ok) {
      r0 = read_off[sd.read];
      r1 = read_off[sd.read + 1];
      ok = r0 <= r1 && r1 <= reads_len && r1 - r0 <= (uint64_t)BSW_MAX_LEN;
    }
    const int64_t len = ok ? (int64_t)(r1 - r0) : 0;
    ok = ok && sd.qb >= 0 && sd.qb <= sd.qe && sd.qe <= len && sd.h0 >= 1 &&
         sd.h0 <= BSW_MAX_H0 && sd.rb >= 0 && (uint64_t)sd.rb <= ref_len &&
         (uint64_t)(sd.qe - sd.qb) <= ref_len - (uint64_t)sd.rb;
    int64_t lt_beg = 0, re = 0, rt_end = 0;
    if (ok) {
      lt_beg = sd.rb - sd.qb - (int64_t)w;
      if (lt_beg < 0) lt_beg = 0;
      re = sd.rb + (sd.qe - sd.qb);
      const uint64_t want = (uint64_t)re + (uint64_t)(len - sd.qe) + (uint64_t)w;
      rt_end = (int64_t)(want < ref_len ? want : ref_len);
      ok = sd.rb - lt_beg <= BSW_MAX_LEN && rt_end - re <= BSW_MAX_LEN;
    }
    if (!ok) flag_bad(&sts[ST_SEED], k);
    if (!ok || codes_bad) {
      T.lq0[k] = T.lq1[k] = T.lt0[k] = T.lt1[k] = 0;
      T.rq0[k] = T.rq1[k] = T.rt0[k] = T.rt1[k] = 0;
      T.lh0[k] = 1;
      continue;
    }
    // left: read[r0, r0 + qb) and ref[lt_beg, rb), both reversed, are the
    // slices [M - r0 - qb, M - r0) and [N - rb, N - lt_beg) of the
    // reversed buffers
    T.lq0[k] = reads_len - r0 - (uint64_t)sd.qb;
    T.lq1[k] = reads_len - r0;
    T.lt0[k] = ref_len - (uint64_t)sd.rb;
    T.lt1[k] = ref_len - (uint64_t)lt_beg;
    T.lh0[k] = sd.h0;
    T.rq0[k] = r0 + (uint64_t)sd.qe;
    T.rq1[k] = r1;
    T.rt0[k] = (uint64_t)re;
    T.rt1[k] = (uint64_t)rt_end;
  }
}

// dst[i] = src[len - 1 - i]; dst is 16-byte aligned.  Each thread writes 16
// bytes with one store; the source bytes are read one by one (their
// alignment is arbitrary).
__global__ void __launch_bounds__(256)
k_reverse(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, uint64_t len) {
  const uint64_t nchunk = len >> 4;
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t c = tid; c < nchunk; c += stride) {
    const uint8_t* p = src + (len - 16 * c - 16);  // forward order
    uint32_t v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      v[i] = (uint32_t)p[15 - 4 * i] | (uint32_t)p[14 - 4 * i] << 8 |
             (uint32_t)p[13 - 4 * i] << 16 | (uint32_t)p[12 - 4 * i] << 24;
    *(uint4*)(dst + 16 * c) = make_uint4(v[0], v[1], v[2], v[3]);
  }
  const uint64_t t0 = nchunk << 4;
  if (tid < len - t0) dst[t0 + tid] = src[len - 1 - t0 - tid];
}

// After the left side: keep its end, record it, and set the right side's
// h0 to the kept score.  The left pipeline's status is copied aside first
// (the right call reuses its workspace).  When any seed failed its checks
// or the left call rejected a pair, every right h0 is 1: the call fails
// anyway and the right pipeline must only see valid pairs.
__global__ void __launch_bounds__(256)
k_seed_mid(const bsw_seed* __restrict__ seeds, int64_t n, const bsw_result* __restrict__ lres,
           const Status* __restrict__ lst, Status* lst_copy, int32_t bonus,
           SeedTables T, SeedPart* __restrict__ part, Status* sts) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tid < (int64_t)(sizeof(Status) / 8))
    ((unsigned long long*)lst_copy)[tid] = ((const unsigned long long*)lst)[tid];
  const bool skip = sts[ST_SEED].bad || sts[ST_READS].bad || sts[ST_REF].bad || lst->bad;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = tid; k < n; k += stride) {
    if (skip) {
      T.rh0[k] = 1;
      continue;
    }
    const bsw_seed sd = seeds[k];
    SeedPart p;
    p.qe = sd.qe;
    if (sd.qb == 0) {
      p.h1 = sd.h0;
      p.qbeg = 0;
      p.rbeg = sd.rb;
      p.how = BSW_END_NONE;
    } else {
      const Kept e = keep_end(lres[k], bonus, sd.qb);
      p.h1 = e.score;
      p.qbeg = sd.qb - e.qlen;
      p.rbeg = sd.rb - e.tlen;
      p.how = e.how;
    }
    p.len = (int32_t)(T.rq1[k] - T.rq0[k]) + sd.qe;
    p.re = (int64_t)T.rt0[k];
    part[k] = p;
    if (p.h1 > BSW_MAX_H0) {
      flag_bad(&sts[ST_H1], k);
      T.rh0[k] = 1;
    } else {
      T.rh0[k] = p.h1;
    }
  }
}

// After the right side: keep its end and write the records, unless some
// check of the call failed (then nothing is written).
__global__ void __launch_bounds__(256)
k_seed_finish(int64_t n, const SeedPart* __restrict__ part, const bsw_result* __restrict__ rres,
              const Status* __restrict__ sts, const Status* __restrict__ rst, int32_t bonus,
              bsw_seed_result* __restrict__ out) {
  bool bad = rst->bad;
  for (int i = 0; i < ST_COUNT; ++i) bad = bad || sts[i].bad;
  if (bad) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += stride) {
    const SeedPart p = part[k];
    bsw_seed_result o;
    o.qbeg = p.qbeg;
    o.rbeg = p.rbeg;
    if (p.qe == p.len) {
      o.score = p.h1;
      o.qend = p.len;
      o.rend = p.re;
      o.how = p.how | BSW_END_NONE << 2;
    } else {
      const Kept e = keep_end(rres[k], bonus, p.len - p.qe);
      o.score = e.score;
      o.qend = p.qe + e.qlen;
      o.rend = p.re + e.tlen;
      o.how = p.how | e.how << 2;
    }
    out[k] = o;
  }
}

namespace {
unsigned grid_for(int64_t n, int64_t per_thread, int64_t cap) {
  int64_t b = (n + per_thread * 256 - 1) / (per_thread * 256);
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}
}  // namespace

void launch_seed_offsets(uint64_t* offs, uint64_t reads_len, uint64_t ref_len,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_seed_offsets, dim3(1), dim3(1), 0, s, offs, reads_len, ref_len);
}

void launch_seed_setup(const bsw_seed* seeds, int64_t n, const uint64_t* read_off,
                       int64_t n_reads, uint64_t reads_len, uint64_t ref_len, int32_t w,
                       const SeedTables& T, Status* sts, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_setup, dim3(grid_for(n, 1, 8192)), dim3(256), 0, s, seeds, n,
                     read_off, n_reads, reads_len, ref_len, w, T, sts);
}

void launch_reverse(const uint8_t* src, uint8_t* dst, uint64_t len, hipStream_t s) {
  if (!len) return;
  hipLaunchKernelGGL(k_reverse, dim3(grid_for((int64_t)(len / 16) + 1, 1, 16384)),
                     dim3(256), 0, s, src, dst, len);
}

void launch_seed_mid(const bsw_seed* seeds, int64_t n, const bsw_result* lres,
                     const Status* lst, Status* lst_copy, int32_t bonus, const SeedTables& T,
                     SeedPart* part, Status* sts, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_mid, dim3(grid_for(n, 1, 8192)), dim3(256), 0, s, seeds, n, lres,
                     lst, lst_copy, bonus, T, part, sts);
}

void launch_seed_finish(int64_t n, const SeedPart* part, const bsw_result* rres,
                        const Status* sts, const Status* rst, int32_t bonus,
                        bsw_seed_result* out, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_finish, dim3(grid_for(n, 1, 8192)), dim3(256), 0, s, n, part,
                     rres, sts, rst, bonus, out);
}

// The filter after extending every seed (Sec. 5.3.2).  A chain is a run of
// consecutive seeds of one read; the thread at a chain's first seed walks
// it in order and drops a seed when an earlier kept seed's extension
// contains it in the read ([qbeg, qend) holds [qb, qe)) and in the
// reference ([rbeg, rend) holds [rb, rb + qe - qb)); the first is kept.
__global__ void k_seed_filter(const bsw_seed* __restrict__ seeds, int64_t n,
                              const bsw_seed_result* __restrict__ res,
                              uint8_t* __restrict__ keep) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t read = seeds[k].read;
    if (k > 0 && seeds[k - 1].read == read) continue;  // not a chain start
    for (int64_t j = k; j < n && seeds[j].read == read; ++j) {
      const bsw_seed sj = seeds[j];
      const int64_t re = sj.rb + (sj.qe - sj.qb);
      bool covered = false;
      for (int64_t i = k; i < j && !covered; ++i) {
        if (!keep[i]) continue;
        const bsw_seed_result& r = res[i];
        covered = r.qbeg <= sj.qb && sj.qe <= r.qend && r.rbeg <= sj.rb && re <= r.rend;
      }
      keep[j] = covered ? 0 : 1;
    }
  }
}

void launch_seed_filter(const bsw_seed* seeds, int64_t n, const bsw_seed_result* res,
                        uint8_t* keep, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_seed_filter, dim3((unsigned)blocks), dim3(256), 0, s, seeds, n, res, keep);
}

}  // namespace bsw
