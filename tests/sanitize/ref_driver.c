/* ref_driver.c -- runs the CPU oracle (oracle/bsw_ref.c) from a batch file,
 * for the address/undefined-behaviour sanitizer build of the oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Input file (little-endian):
 *   int64 n, int32 n_params, bsw_ref_params params[n_params],
 *   uint64 q_off[n+1], uint64 t_off[n+1], int32 h0[n], uint8 pid[n],
 *   uint64 q_len, uint8 q[q_len], uint64 t_len, uint8 t[t_len]
 * Every array is copied into a heap block of exactly its size, so that a
 * read one past an end is caught.  Output file: the batch call's rc and bad
 * index, its results and diagnostics, then for each pair the results of
 * the 16-bit and 8-bit lane forms (rc, result) where h0 fits the lane. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bsw_ref.h"

static void* take(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p || (bytes && fread(p, 1, bytes, f) != bytes)) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: ref_driver IN OUT THREADS\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t n;
  int32_t np;
  if (fread(&n, 8, 1, f) != 1 || fread(&np, 4, 1, f) != 1 || n < 0 || np < 0) return 2;
  bsw_ref_params* params = take(f, sizeof(bsw_ref_params) * (size_t)np);
  uint64_t* q_off = take(f, 8 * (size_t)(n + 1));
  uint64_t* t_off = take(f, 8 * (size_t)(n + 1));
  int32_t* h0 = take(f, 4 * (size_t)n);
  uint8_t* pid = take(f, (size_t)n);
  uint64_t ql, tl;
  if (fread(&ql, 8, 1, f) != 1) return 2;
  uint8_t* q = take(f, ql);
  if (fread(&tl, 8, 1, f) != 1) return 2;
  uint8_t* t = take(f, tl);
  fclose(f);

  bsw_ref_result* out = calloc((size_t)n + 1, sizeof *out);
  bsw_ref_diag* diag = calloc((size_t)n + 1, sizeof *diag);
  int64_t bad = -1;
  const int rc = bsw_ref_extend_batch(n, q, q_off, t, t_off, h0, pid, params, np, out, diag,
                                      atoi(argv[3]), &bad);
  FILE* g = fopen(argv[2], "wb");
  if (!g) return 2;
  const int32_t rc32 = rc;
  fwrite(&rc32, 4, 1, g);
  fwrite(&bad, 8, 1, g);
  fwrite(out, sizeof *out, (size_t)n, g);
  fwrite(diag, sizeof *diag, (size_t)n, g);
  for (int64_t k = 0; rc == BSW_REF_OK && k < n; ++k) {
    const int32_t lq = (int32_t)(q_off[k + 1] - q_off[k]);
    const int32_t lt = (int32_t)(t_off[k + 1] - t_off[k]);
    for (int bits = 16; bits >= 8; bits -= 8) {
      bsw_ref_result r;
      memset(&r, 0, sizeof r);
      int32_t rcb = -100;
      if (h0[k] <= (1 << bits) - 1)
        rcb = bsw_ref_extend_one_bits(lq, q + q_off[k], lt, t + t_off[k], h0[k],
                                      &params[pid[k]], &r, NULL, bits);
      fwrite(&rcb, 4, 1, g);
      fwrite(&r, sizeof r, 1, g);
    }
  }
  fclose(g);
  free(params); free(q_off); free(t_off); free(h0); free(pid); free(q); free(t);
  free(out); free(diag);
  return 0;
}
