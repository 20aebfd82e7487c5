// bsw_seed_internal.h -- types shared by the seed driver's host code
// (bsw_seeds.cpp) and its kernels (bsw_seed_kernels.hip).  Not exported.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bsw.h"
#include "bsw_internal.h"

namespace bsw {

// Pair tables of the two BSW calls (device arrays of n entries): pair k of
// a side has query q[q0[k], q1[k]) and target t[t0[k], t1[k]); the left
// side indexes the reversed reads and reference.
struct SeedTables {
  uint64_t *lq0, *lq1, *lt0, *lt1;
  uint64_t *rq0, *rq1, *rt0, *rt1;
  int32_t *lh0, *rh0;
};

// What the left side kept, for the right side's records (40 bytes).
struct SeedPart {
  int32_t h1;    // score kept after the left side (the right side's h0)
  int32_t qbeg;  // read start kept
  int32_t how;   // BSW_END_* of the left side
  int32_t qe;    // seed end in the read
  int32_t len;   // read length
  int32_t pad_;
  int64_t rbeg;  // reference start kept
  int64_t re;    // reference end of the seed
};
static_assert(sizeof(SeedPart) == 40, "SeedPart layout");

// Status blocks of one seed call (first_bad_inv = ~index of the first bad
// seed, or read for ST_READS).
enum { ST_SEED = 0, ST_READS, ST_REF, ST_LEFT, ST_H1, ST_COUNT };

void launch_seed_offsets(uint64_t* offs, uint64_t reads_len, uint64_t ref_len,
                         hipStream_t s);
void launch_seed_setup(const bsw_seed* seeds, int64_t n, const uint64_t* read_off,
                       int64_t n_reads, uint64_t reads_len, uint64_t ref_len, int32_t w,
                       const SeedTables& T, Status* sts, hipStream_t s);
void launch_reverse(const uint8_t* src, uint8_t* dst, uint64_t len, hipStream_t s);
void launch_seed_mid(const bsw_seed* seeds, int64_t n, const bsw_result* lres,
                     const Status* lst, Status* lst_copy, int32_t bonus, const SeedTables& T,
                     SeedPart* part, Status* sts, hipStream_t s);
void launch_seed_finish(int64_t n, const SeedPart* part, const bsw_result* rres,
                        const Status* sts, const Status* rst, int32_t bonus,
                        bsw_seed_result* out, hipStream_t s);

void launch_seed_filter(const bsw_seed* seeds, int64_t n, const bsw_seed_result* res,
                        uint8_t* keep, hipStream_t s);

}  // namespace bsw
