// bsw_internal.h -- types shared by the host runtime and the HIP kernels of
// libbsw.so (never exported).
#pragma once
#include <stdint.h>

namespace bsw {

// Per-pair descriptor in sorted (binned) order, 32 bytes.
struct PairDesc {
  uint64_t qo, to;   // offsets of the query and target in the input arrays
  uint16_t ql, tl;   // lengths
  int32_t h0;        // seed score
  uint32_t idx;      // position in the caller's order (results go there)
  uint8_t pid;       // scoring set
  uint8_t cls;       // kernel class
  uint8_t pad_[2];
};
static_assert(sizeof(PairDesc) == 32, "PairDesc layout");

// Scoring set as the kernels read it.
struct KParams {
  uint32_t prow[5][2];  // bytes of mat[a][0..3] | mat[a][4], per target code a
  int32_t o_del, e_del, o_ins, e_ins;
  int32_t oe_del, oe_ins;
  int32_t w, zdrop, end_bonus;
  int32_t amax;         // max(0, max mat)
  int32_t pad_[2];
};

// Kernel classes.  Lane mode: one pair per lane, the row buffer of H and E
// in LDS, sized by the class's query-length cap.  Value width: stored H and
// E of a pair never exceed U = h0 + A * min(qlen, tlen), so 8-bit records
// are exact when U <= 255 and 16-bit records when U <= 65535.
enum { W8 = 0, W16 = 1, W32 = 2, NWIDTH = 3 };
enum { NLQ = 4 };                        // query caps 32, 64, 128, 256
constexpr int LQ_CAP[NLQ] = {32, 64, 128, 256};
enum { CLS_LANE_END = NLQ * NWIDTH,      // 12 lane classes
       CLS_LONG = CLS_LANE_END,          // query longer than 256
       NCLS = CLS_LANE_END + 1 };

constexpr int KEY_SUB_BITS = 12;         // sub-key inside a class
constexpr int NBINS = NCLS << KEY_SUB_BITS;

// Device-side status block.
struct Status {
  uint32_t bad;          // nonzero: some pair failed validation
  uint32_t pad_;
  unsigned long long first_bad_inv;  // ~(smallest bad pair index); 0 = none
  unsigned long long long_max;   // largest query length in the long class
};

constexpr int LONG_SLOTS = 256;          // waves running the long class
constexpr int LONG_SLOT_COLS = 65536;    // row-buffer entries per slot

}  // namespace bsw
