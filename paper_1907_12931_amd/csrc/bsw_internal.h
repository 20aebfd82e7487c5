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

// Kernel classes (all lane mode: one pair per lane of a wave).
//  * L8 classes: 8-bit row-buffer records (H and E bytes), used for every
//    pair whose query fits the class cap, unless a wider width is forced.
//    A pair whose bound U = h0 + A*min(qlen,tlen) exceeds 255 runs here
//    speculatively: its final best score tells whether any stored value can
//    have exceeded 8 bits (best + max(0, A - o_del - e_del) > 255), and
//    such pairs are run again with 16-bit records.
//  * W16 classes: 16-bit records, same chunked kernel, for pairs whose
//    bound (or a forced minimum width) needs them; the 8-bit overflow
//    reruns use the widest of them.
//  * W32 classes: 32-bit records (one-lane-per-pair kernel with a private
//    row buffer in LDS) for bounds over 16 bits, a forced 32-bit width and
//    the (rare) 16-bit overflow reruns.
//  * LONG: queries longer than 256.
enum { W8 = 0, W16 = 1, W32 = 2 };
enum { NL8 = 8, NLW = 4 };
constexpr int L8_CAP[NL8] = {32, 64, 96, 128, 160, 192, 224, 256};
constexpr int LW_CAP[NLW] = {32, 64, 128, 256};
enum {
  CLS_L8 = 0,                      // 8 classes
  CLS_W16 = CLS_L8 + NL8,          // 4 classes
  CLS_W32 = CLS_W16 + NLW,         // 4 classes
  CLS_LONG = CLS_W32 + NLW,        // queries longer than 256
  NCLS = CLS_LONG + 1
};

constexpr int KEY_SUB_BITS = 12;         // sub-key inside a class
constexpr int NBINS = NCLS << KEY_SUB_BITS;

// Device-side status block.
struct Status {
  uint32_t bad;          // nonzero: some pair failed validation
  uint32_t pad_;
  unsigned long long first_bad_inv;  // ~(smallest bad pair index); 0 = none
  unsigned long long long_max;   // largest query length in the long class
  long long ovf_range[2];        // {0, number of pairs queued for the rerun}
  unsigned long long cls_cells[32];  // band cells per class (+ rerun slot)
  // lane-cells a class's kernel stepped through (every lane of a wave over
  // the wave's column span of each row, padding and finished lanes
  // included): the work behind cls_cells
  unsigned long long work_cells[32];
};

// One request of a serving batch (see k_assemble).
struct ReqSlice {
  long long base;            // first batch pair of the request
  long long n;               // its pairs
  unsigned long long q_at;   // byte offset of its query bytes from the base
  unsigned long long t_at;   // byte offset of its target bytes from the base
  const uint64_t* q_off;     // its n + 1 query offsets (device)
  const uint64_t* t_off;     // its n + 1 target offsets (device)
  const int32_t* h0;         // its n seed scores (device)
  const uint8_t* pid;        // its n scoring-set indices (device) or null
};

// Launch records name a wave-mode launch of a 32-bit class as the class
// plus WAVE_TAG (its cells are counted under the class).
constexpr int WAVE_TAG = 32;

constexpr int LONG_SLOTS = 256;          // waves running the long class
constexpr int LONG_SLOT_COLS = 65536;    // row-buffer entries per slot

}  // namespace bsw
