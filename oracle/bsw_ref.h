/*
 * bsw_ref.h -- CPU oracle for banded Smith-Waterman seed extension (BSW).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and libbsw_ref.so are used by the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark to
 * decide what the GPU library must return.  Product code never links,
 * loads or calls it.  It shares no header, helper or table with the GPU
 * library: the struct layouts below are declared here independently and
 * happen to match the GPU library's byte for byte, because both follow the
 * same statement of the problem.
 *
 * What is computed (paper Sec. 5.1, Eq. (2) and (3); abort and band rules
 * (a)-(c) in Sec. 5.1; outputs in Sec. 5.4 (a)-(b)): for every pair
 * (query q, target t, seed score h0) the banded affine-gap extension of
 * the seed, rows = target positions, columns = query positions, returning
 * the best score and where it was reached, the best score that reaches the
 * end of the query and the target row where that happened, and the largest
 * distance from the diagonal of any improving cell.
 */
#ifndef BSW_REF_H
#define BSW_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One scoring set.  mat[a*5+b] is the score of target code a against query
 * code b (codes 0..3 = A,C,G,T, 4 = N).  A gap of length k >= 1 costs
 * o + k*e.  Deletions consume target only (vertical moves), insertions
 * consume query only (horizontal moves). */
typedef struct bsw_ref_params {
  int8_t  mat[25];
  int8_t  pad_[3];
  int32_t o_del, e_del, o_ins, e_ins;
  int32_t w;          /* band half-width, >= 0                           */
  int32_t zdrop;      /* <= 0 disables the drop-from-best abort          */
  int32_t end_bonus;  /* >= 0; only narrows the band (see the .c file)   */
} bsw_ref_params;

typedef struct bsw_ref_result {
  int32_t score;   /* best score (h0 if nothing beat the seed)             */
  int32_t qle;     /* query end of the best cell, 1-based; 0 = none        */
  int32_t tle;     /* target end of the best cell, 1-based; 0 = none       */
  int32_t gtle;    /* target end where gscore was reached; 0 = never       */
  int32_t gscore;  /* best score touching the query end; -1 = never        */
  int32_t max_off; /* max |column - row| over improving cells              */
} bsw_ref_result;

typedef struct bsw_ref_diag {
  int32_t rows;    /* rows entered (the stopping row included)             */
  int32_t stop;    /* 0 = ran out of target, 1 = all-zero row, 2 = z-drop  */
  int64_t cells;   /* band cells computed, summed over the rows entered    */
} bsw_ref_diag;

enum { BSW_REF_OK = 0, BSW_REF_EINVAL = -1, BSW_REF_ENOMEM = -2 };
enum { BSW_REF_STOP_END = 0, BSW_REF_STOP_ZERO = 1, BSW_REF_STOP_ZDROP = 2 };

/* Validation limits (shared by meaning, not by code, with the GPU side). */
#define BSW_REF_MAX_LEN     65535   /* max query or target length        */
#define BSW_REF_MAX_H0      (1 << 24)
#define BSW_REF_MAX_GAP     1000    /* max o and e                       */
#define BSW_REF_MAX_BONUS   (1 << 24)

/* Extend one pair.  Inputs are host arrays of codes 0..4.  Returns
 * BSW_REF_OK or BSW_REF_EINVAL (bad codes/params/h0); diag may be NULL. */
int bsw_ref_extend_one(int32_t qlen, const uint8_t* q, int32_t tlen,
                       const uint8_t* t, int32_t h0, const bsw_ref_params* p,
                       bsw_ref_result* out, bsw_ref_diag* diag);

/* The same in lanes of `bits` bits (8, 16 or 32) with saturating
 * arithmetic (Sec. 5.4.1 runs the extension in 8- or 16-bit SIMD lanes);
 * bits = 32 is bsw_ref_extend_one.  h0 must fit the lane. */
int bsw_ref_extend_one_bits(int32_t qlen, const uint8_t* q, int32_t tlen,
                            const uint8_t* t, int32_t h0, const bsw_ref_params* p,
                            bsw_ref_result* out, bsw_ref_diag* diag, int32_t bits);

/* Extend n pairs.  Pair k uses q[q_off[k] .. q_off[k+1]) and
 * t[t_off[k] .. t_off[k+1]), seed score h0[k] and scoring set
 * params[param_id[k]] (param_id may be NULL: set 0 for all).  out[k] and,
 * if diag is non-NULL, diag[k] receive the results in caller order.
 * n_threads <= 0 means one thread per online CPU.  Pairs are dealt out in
 * dynamic chunks of 1024 (the batch-to-thread distribution of Sec. 3.1).
 * All arguments are validated before any pair is computed; on error
 * nothing is written and the index of the first bad pair is stored in
 * *bad_index (if non-NULL). */
int bsw_ref_extend_batch(int64_t n, const uint8_t* q, const uint64_t* q_off,
                         const uint8_t* t, const uint64_t* t_off,
                         const int32_t* h0, const uint8_t* param_id,
                         const bsw_ref_params* params, int32_t n_params,
                         bsw_ref_result* out, bsw_ref_diag* diag,
                         int32_t n_threads, int64_t* bad_index);

#ifdef __cplusplus
}
#endif
#endif
