/*
 * bsw_ref.c -- plain scalar CPU oracle for banded Smith-Waterman seed
 * extension (BSW).  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke
 * check and the benchmark's CPU-baseline leg; the product never loads it.
 *
 * The method (paper Sec. 5.1) computes, row by row, the affine-gap DP of
 * Eq. (2) from the boundary of Eq. (3), restricted to a band around the
 * diagonal, stopping early when a row is all zero or has dropped too far
 * below the best score, and shrinking the band after each row by the zero
 * cells at both of its ends.  It keeps a single row of H and E (Sec. 5.1,
 * last paragraph).  The paper requires output identical to BWA-MEM's BSW
 * (Sec. 6.1.3), so where its summary is silent or inconsistent this file
 * takes the readings listed below; every step is written out in the order
 * the method performs it.  Integer arithmetic only; no vectorisation, no
 * reordering.
 *
 * Readings (paper silent, ambiguous or inconsistent):
 *  R1  rows are target positions i, columns are query positions j.
 *  R2  a gap of length k costs o + k*e; opening therefore subtracts o+e
 *      (Eq. (3) charges g_o + g_e*k, Eq. (2) only g_o; we follow Eq. (3)).
 *  R3  gaps open from the diagonal term M = H(i-1,j-1) + S, not from H, so
 *      an insertion never directly follows a deletion.
 *  R4  the diagonal step is only taken from a positive cell: if the stored
 *      H(i-1,j-1) is 0 then M = 0.  The zero-row abort and the zero-based
 *      band shrink of Sec. 5.1 (b),(c) presuppose that a zero cell is dead.
 *  R5  E and F are floored at 0 (Eq. (2)); H >= 0 follows.
 *  R6  first row: H(-1,j) = max(0, h0 - o_ins - e_ins*(j+1)) (insertions
 *      from the seed); first column, used while the band starts at column
 *      0: H(i,-1) = max(0, h0 - o_del - e_del*(i+1)); E starts at 0; F
 *      restarts at 0 at the band start of every row.
 *  R7  left of the band H = 0 and F = 0.
 *  R8  after a row, (H(i,end-1), E = 0) is stored at buffer index end.
 *  R9  the one-row buffer is never reset: an index that re-enters the band
 *      holds whatever was last written there (first-row value if never).
 *  R10 row i covers columns [max(beg, i-w'), min(end, i+w'+1, qlen)).
 *  R11 end bonus and the maximum score narrow the band:
 *      w' = min(w, cap_ins, cap_del), cap_X = floor((qlen*A + B - o_X)/e_X)
 *      + 1 when the numerator is >= 0, else 1, where A = max(0, max score).
 *  R12 a buffer index is empty iff its stored H and E are both 0; after a
 *      row beg moves to the first non-empty index and end to the last
 *      non-empty index + 2, capped at qlen.
 *  R13 z-drop compares best - m against zdrop after charging the diagonal
 *      drift between the two cells as a gap; only rows that did not raise
 *      the best are tested, and only if zdrop > 0.
 *  R14 row epilogue order: query-end (global) update, zero-row abort,
 *      best / z-drop, band shrink.
 *  R15 ties: within a row the larger column wins; across rows the first
 *      strict improvement wins; the global score takes the latest row with
 *      an equal or larger value; max_off only moves on strict improvement.
 *  R16 qle/tle are 1-based ends (0 = the seed was never beaten); gtle = 0
 *      and gscore = -1 if the query end was never reached.
 *  R20 h0 >= 1 is required; an empty target returns (h0,0,0,0,-1,0).
 */
#include "bsw_ref.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

static int params_ok(const bsw_ref_params* p) {
  if (p->o_del < 0 || p->o_ins < 0 || p->o_del > BSW_REF_MAX_GAP ||
      p->o_ins > BSW_REF_MAX_GAP)
    return 0;
  if (p->e_del < 1 || p->e_ins < 1 || p->e_del > BSW_REF_MAX_GAP ||
      p->e_ins > BSW_REF_MAX_GAP)
    return 0;
  if (p->w < 0) return 0;
  if (p->end_bonus < 0 || p->end_bonus > BSW_REF_MAX_BONUS) return 0;
  return 1;
}

/* Band half-width after the end-bonus / maximum-score cap (R11). */
static int band_cap(int qlen, const bsw_ref_params* p) {
  int a = 0, k, num, cap_ins, cap_del, w = p->w;
  for (k = 0; k < 25; ++k) a = imax(a, p->mat[k]);
  num = qlen * a + p->end_bonus - p->o_ins;
  cap_ins = num >= 0 ? num / p->e_ins + 1 : 1;
  num = qlen * a + p->end_bonus - p->o_del;
  cap_del = num >= 0 ? num / p->e_del + 1 : 1;
  w = imin(w, cap_ins);
  w = imin(w, cap_del);
  return w;
}

/* The method with every cell value held in a lane of `bits` bits (8, 16,
 * or 32 = plain int): Sec. 5.4.1 runs the extension in 8- or 16-bit SIMD
 * lanes.  Such a lane holds 0 .. 2^bits - 1 and its additions saturate;
 * the only value that can grow past what the row buffer already holds is
 * the diagonal term d + S, so that is where the lane clamps (a negative
 * diagonal term needs no clamp: E, F >= 0 dominate it).  With bits = 32
 * this is the method exactly. */
static int extend_bits(int32_t qlen, const uint8_t* q, int32_t tlen,
                       const uint8_t* t, int32_t h0, const bsw_ref_params* p,
                       bsw_ref_result* out, bsw_ref_diag* diag, int32_t bits) {
  int *hbuf, *ebuf; /* one row of H (shifted by one column) and of E */
  int i, j, wb, beg, end, best, bi, bj, gbest, gi, moff, rows, stop;
  const int vmax = bits < 32 ? (1 << bits) - 1 : 0;
  int64_t cells = 0;

  if (h0 < 1 || h0 > BSW_REF_MAX_H0 || qlen < 0 || tlen < 0 ||
      qlen > BSW_REF_MAX_LEN || tlen > BSW_REF_MAX_LEN || !params_ok(p))
    return BSW_REF_EINVAL;
  for (j = 0; j < qlen; ++j)
    if (q[j] > 4) return BSW_REF_EINVAL;
  for (i = 0; i < tlen; ++i)
    if (t[i] > 4) return BSW_REF_EINVAL;

  hbuf = (int*)malloc(sizeof(int) * (size_t)(qlen + 1));
  ebuf = (int*)malloc(sizeof(int) * (size_t)(qlen + 1));
  if (!hbuf || !ebuf) {
    free(hbuf);
    free(ebuf);
    return BSW_REF_ENOMEM;
  }

  /* Step 0: band cap (R11). */
  wb = band_cap(qlen, p);

  /* Step 1: the single row buffer (Eq. (3), first row; R6, R9).
   * hbuf[j] holds H(i-1, j-1) at the start of row i, ebuf[j] holds E(i,j). */
  hbuf[0] = h0;
  for (j = 1; j <= qlen; ++j)
    hbuf[j] = imax(0, h0 - p->o_ins - p->e_ins * j);
  for (j = 0; j <= qlen; ++j) ebuf[j] = 0;

  /* Step 2: running state. */
  best = h0;
  bi = bj = -1;
  gbest = -1;
  gi = -1;
  moff = 0;
  beg = 0;
  end = qlen;
  rows = 0;
  stop = BSW_REF_STOP_END;

  /* Step 3: rows. */
  for (i = 0; i < tlen; ++i) {
    int hl, f, m, mj;
    const int8_t* srow = &p->mat[t[i] * 5];

    ++rows;
    /* 3.1 band (Sec. 5.1 (a), R10) */
    beg = imax(beg, i - wb);
    end = imin(end, i + wb + 1);
    end = imin(end, qlen);
    if (end > beg) cells += end - beg;

    /* 3.2 left boundary: H(i,-1) from Eq. (3) while the band touches
     * column 0, else 0 (R6, R7) */
    hl = 0;
    if (beg == 0) hl = imax(0, h0 - p->o_del - p->e_del * (i + 1));
    f = 0;
    m = 0;
    mj = -1;

    /* 3.3 cells, left to right (Eq. (2) with R2-R5) */
    for (j = beg; j < end; ++j) {
      int d = hbuf[j];   /* H(i-1, j-1) */
      int e = ebuf[j];   /* E(i, j)     */
      int mdiag, h;
      hbuf[j] = hl;      /* keep H(i, j-1) for row i+1 */
      mdiag = d > 0 ? d + srow[q[j]] : 0;
      if (bits < 32 && mdiag > vmax) mdiag = vmax; /* saturating lane */
      h = imax(mdiag, imax(e, f));
      hl = h;
      if (h >= m) mj = j; /* ties: larger column (R15) */
      m = imax(m, h);
      ebuf[j] = imax(imax(e - p->e_del, mdiag - p->o_del - p->e_del), 0);
      f = imax(imax(f - p->e_ins, mdiag - p->o_ins - p->e_ins), 0);
    }

    /* 3.4 right boundary (R8) */
    hbuf[end] = hl;
    ebuf[end] = 0;

    /* 3.5 best score touching the end of the query (Sec. 5.4 (b)) */
    if (imax(beg, end) == qlen) {
      if (hl >= gbest) gi = i;
      gbest = imax(gbest, hl);
    }

    /* 3.6 all-zero row (Sec. 5.1 (b)) */
    if (m == 0) {
      stop = BSW_REF_STOP_ZERO;
      break;
    }

    /* 3.7 best so far, or drop from the best (Sec. 5.1 (b), R13) */
    if (m > best) {
      best = m;
      bi = i;
      bj = mj;
      moff = imax(moff, abs(mj - i));
    } else if (p->zdrop > 0) {
      int drift = (i - bi) - (mj - bj);
      int drop;
      if (drift > 0)
        drop = best - m - drift * p->e_del;
      else
        drop = best - m - (-drift) * p->e_ins;
      if (drop > p->zdrop) {
        stop = BSW_REF_STOP_ZDROP;
        break;
      }
    }

    /* 3.8 shrink the band by the empty indices at both ends (Sec. 5.1 (c),
     * R12) */
    while (beg < end && hbuf[beg] == 0 && ebuf[beg] == 0) ++beg;
    j = end;
    while (j >= beg && hbuf[j] == 0 && ebuf[j] == 0) --j;
    end = imin(j + 2, qlen);
  }

  /* Step 4: outputs (R16). */
  out->score = best;
  out->qle = bj + 1;
  out->tle = bi + 1;
  out->gtle = gi + 1;
  out->gscore = gbest;
  out->max_off = moff;
  if (diag) {
    diag->rows = rows;
    diag->stop = stop;
    diag->cells = cells;
  }
  free(hbuf);
  free(ebuf);
  return BSW_REF_OK;
}

int bsw_ref_extend_one(int32_t qlen, const uint8_t* q, int32_t tlen,
                       const uint8_t* t, int32_t h0, const bsw_ref_params* p,
                       bsw_ref_result* out, bsw_ref_diag* diag) {
  return extend_bits(qlen, q, tlen, t, h0, p, out, diag, 32);
}

int bsw_ref_extend_one_bits(int32_t qlen, const uint8_t* q, int32_t tlen,
                            const uint8_t* t, int32_t h0, const bsw_ref_params* p,
                            bsw_ref_result* out, bsw_ref_diag* diag, int32_t bits) {
  if (bits != 8 && bits != 16 && bits != 32) return BSW_REF_EINVAL;
  if (bits < 32 && h0 > (1 << bits) - 1) return BSW_REF_EINVAL;
  return extend_bits(qlen, q, tlen, t, h0, p, out, diag, bits);
}

/* ---------------------------------------------------------------------- */
/* Batch driver: validation first, then a small pthread pool handing out
 * chunks of 1024 pairs from a shared counter. */

typedef struct job {
  int64_t n;
  const uint8_t *q, *t;
  const uint64_t *q_off, *t_off;
  const int32_t* h0;
  const uint8_t* param_id;
  const bsw_ref_params* params;
  bsw_ref_result* out;
  bsw_ref_diag* diag;
  int64_t next; /* guarded by lock */
  int err;
  pthread_mutex_t lock;
} job;

enum { CHUNK = 1024 };

static void* worker(void* arg) {
  job* jb = (job*)arg;
  for (;;) {
    int64_t b, e, k;
    pthread_mutex_lock(&jb->lock);
    b = jb->next;
    jb->next += CHUNK;
    pthread_mutex_unlock(&jb->lock);
    if (b >= jb->n) break;
    e = b + CHUNK < jb->n ? b + CHUNK : jb->n;
    for (k = b; k < e; ++k) {
      const bsw_ref_params* p = &jb->params[jb->param_id ? jb->param_id[k] : 0];
      int rc = bsw_ref_extend_one(
          (int32_t)(jb->q_off[k + 1] - jb->q_off[k]), jb->q + jb->q_off[k],
          (int32_t)(jb->t_off[k + 1] - jb->t_off[k]), jb->t + jb->t_off[k],
          jb->h0[k], p, &jb->out[k], jb->diag ? &jb->diag[k] : NULL);
      if (rc != BSW_REF_OK) {
        pthread_mutex_lock(&jb->lock);
        jb->err = rc;
        pthread_mutex_unlock(&jb->lock);
      }
    }
  }
  return NULL;
}

int bsw_ref_extend_batch(int64_t n, const uint8_t* q, const uint64_t* q_off,
                         const uint8_t* t, const uint64_t* t_off,
                         const int32_t* h0, const uint8_t* param_id,
                         const bsw_ref_params* params, int32_t n_params,
                         bsw_ref_result* out, bsw_ref_diag* diag,
                         int32_t n_threads, int64_t* bad_index) {
  int64_t k;
  int nt, i;
  job jb;
  pthread_t* th;

  if (bad_index) *bad_index = -1;
  if (n < 0) return BSW_REF_EINVAL;
  if (n == 0) return BSW_REF_OK;
  if (!q_off || !t_off || !h0 || !params || !out || n_params < 1 ||
      n_params > 256)
    return BSW_REF_EINVAL;
  for (i = 0; i < n_params; ++i)
    if (!params_ok(&params[i])) return BSW_REF_EINVAL;
  for (k = 0; k < n; ++k) {
    uint64_t ql, tl, x;
    if (q_off[k + 1] < q_off[k] || t_off[k + 1] < t_off[k]) goto bad;
    ql = q_off[k + 1] - q_off[k];
    tl = t_off[k + 1] - t_off[k];
    if (ql > BSW_REF_MAX_LEN || tl > BSW_REF_MAX_LEN) goto bad;
    if (h0[k] < 1 || h0[k] > BSW_REF_MAX_H0) goto bad;
    if (param_id && param_id[k] >= n_params) goto bad;
    for (x = q_off[k]; x < q_off[k + 1]; ++x)
      if (q[x] > 4) goto bad;
    for (x = t_off[k]; x < t_off[k + 1]; ++x)
      if (t[x] > 4) goto bad;
    continue;
  bad:
    if (bad_index) *bad_index = k;
    return BSW_REF_EINVAL;
  }

  nt = n_threads > 0 ? n_threads : (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (nt < 1) nt = 1;
  if (nt > 256) nt = 256;
  memset(&jb, 0, sizeof jb);
  jb.n = n;
  jb.q = q;
  jb.t = t;
  jb.q_off = q_off;
  jb.t_off = t_off;
  jb.h0 = h0;
  jb.param_id = param_id;
  jb.params = params;
  jb.out = out;
  jb.diag = diag;
  pthread_mutex_init(&jb.lock, NULL);
  if (nt == 1) {
    worker(&jb);
  } else {
    th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nt);
    if (!th) {
      pthread_mutex_destroy(&jb.lock);
      return BSW_REF_ENOMEM;
    }
    for (i = 0; i < nt; ++i) pthread_create(&th[i], NULL, worker, &jb);
    for (i = 0; i < nt; ++i) pthread_join(th[i], NULL);
    free(th);
  }
  pthread_mutex_destroy(&jb.lock);
  return jb.err;
}
