// bsw_lanev_impl.h -- body of the register-row lane kernel, included by
// the translation units that instantiate it (bsw_lanev_*.hip).
#pragma once
#include "bsw_device.h"
#include "bsw_lanev.h"

namespace bsw {

// ---------------------------------------------------------------------------
// Lane mode with the row buffer in registers (the main kernel: 8-bit
// records, queries up to CAP).
//
// The inter-task scheme of Sec. 5.3: every lane owns one pair and the wave
// walks rows in lock step, the same four-column chunk in every lane.  The
// row buffer of byte records lives in the lane's vector registers, two
// dwords per chunk of four columns: the H bytes of records 4k .. 4k+3
// (record j holds H(i-1, j-1), the diagonal input of column j) and their E
// bytes (E(i, j)).  The pair's query codes sit in registers too, so the
// cell loop touches no memory.  The loop over chunks is unrolled (chunk k
// always lives in the same registers); a row enters it at the wave's first
// chunk c0 through a switch and leaves after its last chunk c1 - 1.
//
// A chunk where no lane's band starts or ends runs its cells alone and
// updates its records in place.  In the others every lane reads the columns
// outside its band as zero (R7: H = F = 0 left of the band; past the end the
// stored values are not part of the row) and keeps its stored records past
// its band end, while column end takes H(i, end - 1) (R8; its E stays zero,
// as every stored E past the band end is).  Neither kind of masked column
// can raise the row maximum: left of the band every H is 0, and past the
// end H = F < H(i, end - 1).  Columns left of the band are written with the
// zeros computed there; the band start never moves left, so they are not
// read again.
//
// The record of column CAP (the band end of a query of exactly CAP
// columns) is never the input of a cell: it only feeds the band shrink and
// the query-end score, so it is kept in LDS alone.
//
// The row maximum and its column come from 16-bit keys H * 256 + j (the
// larger column wins ties, R15), formed by a saturating multiply-add: a key
// saturates at 0xffff exactly when H >= 256, so best >= 255 flags every pair
// whose values may not fit a byte; those pairs are queued for the 32-bit
// rerun (best + max(0, A - o_del - e_del) >= 255).
//
// The band shrink needs each lane's records at its own band edges, which
// registers cannot be indexed by; a one-byte mirror per column in LDS
// (H | E of the stored record: zero iff the record is empty) serves those
// reads, a word of four columns at a time, and the query-end score, whose
// column-end byte is H(i, end - 1).  Every row rewrites the mirror over the
// wave's chunk span, which holds every column a live lane reads.

// key = H * 256 + j of two columns, saturated at 0xffff (v_pk_mad_u16 with
// clamp); k256 holds 256 in both halves
__device__ __forceinline__ uint32_t row_keys(uint32_t h2, uint32_t k256, uint32_t jj) {
  uint32_t k;
  asm("v_pk_mad_u16 %0, %1, %2, %3 clamp" : "=v"(k) : "v"(h2), "v"(k256), "s"(jj));
  return k;
}

__device__ __forceinline__ uint32_t usubsat16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(
                                          __builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t uaddsat16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(
                                          __builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t umax16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}

// The low 32 - t bits of a dword set, t in 0..32 (clamped): with t = 32 -
// 8n, the bytes c < n.
__device__ __forceinline__ uint32_t low_bits_but(int t) {
  return (uint32_t)(0xffffffffull >> imin(imax(t, 0), 32));
}

// The four cells of a chunk (columns 4k .. 4k+3) in packed 16-bit
// arithmetic, from its records x (H bytes) and y (E bytes) into the new
// ones.  hp carries H(i, 4k-1) in its high half in and [H(i, 4k+2),
// H(i, 4k+3)] out; fp carries F(i, 4k) in its high half in and [F(i, 4k+3),
// F(i, 4k+4)] out.  The row-maximum keys of the four columns (column
// numbers j01, j23) are folded into mkey.
template <bool SYM>
__device__ __forceinline__ void cells4(uint32_t& x, uint32_t& y, uint32_t sc, uint32_t& hp,
                                       uint32_t& fp, uint32_t& mkey, uint32_t j01, uint32_t j23,
                                       const PkParams& pp) {
  const s16x2 D01 = pk(__builtin_amdgcn_perm(0u, x, 0x0c010c00u));
  const s16x2 D23 = pk(__builtin_amdgcn_perm(0u, x, 0x0c030c02u));
  const s16x2 E01 = pk(__builtin_amdgcn_perm(0u, y, 0x0c010c00u));
  const s16x2 E23 = pk(__builtin_amdgcn_perm(0u, y, 0x0c030c02u));
  // the signed score bytes, sign-extended to 16 bits
  const uint32_t sc8 = sc << 8;
  const s16x2 S01 = pk(__builtin_amdgcn_perm(sc8, sc, 0x08010a00u));
  const s16x2 S23 = pk(__builtin_amdgcn_perm(sc8, sc, 0x09030b02u));
  // M = D > 0 ? D + S : 0 as min(D + S, 128 D): equal where D > 0, and <= 0
  // where D = 0, which changes none of E, F and H (maxima with values >= 0)
  const s16x2 G01 = pmin(D01 + S01, D01 << 7), G23 = pmin(D23 + S23, D23 << 7);
  const s16x2 TD01 = G01 - pp.oeD, TD23 = G23 - pp.oeD;
  const s16x2 EN01 = pmax(psubsat(E01, pp.eD), TD01);
  const s16x2 EN23 = pmax(psubsat(E23, pp.eD), TD23);
  const s16x2 z = bcast(0);
  const s16x2 A01 = pmax(SYM ? TD01 : G01 - pp.oeI, z);
  const s16x2 A23 = pmax(SYM ? TD23 : G23 - pp.oeI, z);
  const s16x2 fc = pk(fp);
  const s16x2 F12 = pmax(pmax(A01, bcast(A01[0]) - pp.eI), bcast(fc[1]) - pp.eI12);
  const s16x2 F34 = pmax(pmax(A23, bcast(A23[0]) - pp.eI), bcast(F12[1]) - pp.eI12);
  const s16x2 F01 = (s16x2){fc[1], F12[0]}, F23 = (s16x2){F12[1], F34[0]};
  const uint32_t h01 = unpk(pmax(pmax(G01, E01), F01));
  const uint32_t h23 = unpk(pmax(pmax(G23, E23), F23));
  mkey = umax16x2(mkey, umax16x2(row_keys(h01, 0x01000100u, j01),
                                 row_keys(h23, 0x01000100u, j23)));
  // H bytes [H(4k-1), H(4k), H(4k+1), H(4k+2)], E bytes [E(4k) .. E(4k+3)]
  const uint32_t t3 = __builtin_amdgcn_perm(h01, hp, 0x0c060402u);
  x = __builtin_amdgcn_perm(h23, t3, 0x04020100u);
  y = __builtin_amdgcn_perm(unpk(EN23), unpk(EN01), 0x06040200u);
  hp = h23;
  fp = unpk(F34);
}

// Per-row state of the chunk sweep.
struct RowSweep {
  int mlo, mn, c1;     // wave-uniform: chunks mlo .. mlo + mn - 1 hold no
                       // lane's band start or end (none lies left of any
                       // band start or right of any band end); c1 is one
                       // past the last chunk visited
  int bb, be;          // 8 beg and 8 end of the lane
  uint32_t lo, hi;     // score row of the row's target base
  uint32_t hp, fp;     // carries (see cells4)
  uint32_t mkey;       // packed row-maximum keys
};

// Chunk K of a row (K < NQ), or the record of column CAP (K == NQ).
template <int K, int NQ, int NQW, bool QNIB, bool SYM>
__device__ __forceinline__ void sweep_chunk(uint2 (&r)[NQ], const uint32_t (&qv)[NQW],
                                            uint32_t* mir, const PkParams& pp, RowSweep& w) {
  if constexpr (K < NQ) {
    uint32_t qc;
    if constexpr (QNIB)
      qc = ((K & 1) ? qv[K / 2] >> 4 : qv[K / 2]) & 0x0f0f0f0fu;
    else
      qc = qv[K];
    const uint32_t sc = __builtin_amdgcn_perm(w.hi, w.lo, qc);
    constexpr uint32_t J01 = (uint32_t)(4 * K) | ((uint32_t)(4 * K + 1) << 16);
    constexpr uint32_t J23 = (uint32_t)(4 * K + 2) | ((uint32_t)(4 * K + 3) << 16);
    uint32_t x = r[K].x, y = r[K].y;
    if (__builtin_expect((uint32_t)(K - w.mlo) < (uint32_t)w.mn, 1)) {
      cells4<SYM>(x, y, sc, w.hp, w.fp, w.mkey, J01, J23, pp);
    } else {
      // inputs outside [beg, end) read as zero; records past column end keep
      // their stored bytes
      const uint32_t in =
          ~low_bits_but(32 * (K + 1) - w.bb) & low_bits_but(32 * (K + 1) - w.be);
      const uint32_t nw = low_bits_but(32 * K + 24 - w.be);
      const uint32_t kx = x & ~nw, ky = y & ~nw;
      x &= in;
      y &= in;
      cells4<SYM>(x, y, sc, w.hp, w.fp, w.mkey, J01, J23, pp);
      x = (x & nw) | kx;
      y = (y & nw) | ky;
    }
    r[K] = make_uint2(x, y);
    mir[K * 64] = x | y;
  } else if constexpr (K == NQ) {
    // column CAP: the H byte H(i, CAP - 1), E zero
    mir[NQ * 64] = (w.hp >> 16) & 0xffu;
  }
}

#define BSW_SWEEP_CASE(K)                                          \
  case K:                                                          \
    sweep_chunk<K, NQ, NQW, QNIB, SYM>(r, qv, mir, pp, w);         \
    if (K + 1 >= w.c1) break;                                      \
    [[fallthrough]];
#define BSW_SWEEP_CASES8(K)                                                             \
  BSW_SWEEP_CASE(K) BSW_SWEEP_CASE(K + 1) BSW_SWEEP_CASE(K + 2) BSW_SWEEP_CASE(K + 3) \
  BSW_SWEEP_CASE(K + 4) BSW_SWEEP_CASE(K + 5) BSW_SWEEP_CASE(K + 6) BSW_SWEEP_CASE(K + 7)

// One row over chunks c0 .. c1 - 1 (c0 <= NQ <= 64).
template <int NQ, int NQW, bool QNIB, bool SYM>
__device__ __forceinline__ void sweep_row(int c0, uint2 (&r)[NQ], const uint32_t (&qv)[NQW],
                                          uint32_t* mir, const PkParams& pp, RowSweep& w) {
  static_assert(NQ <= 64, "register row of at most 256 columns");
  switch (c0) {
    BSW_SWEEP_CASES8(0) BSW_SWEEP_CASES8(8) BSW_SWEEP_CASES8(16) BSW_SWEEP_CASES8(24)
    BSW_SWEEP_CASES8(32) BSW_SWEEP_CASES8(40) BSW_SWEEP_CASES8(48) BSW_SWEEP_CASES8(56)
    BSW_SWEEP_CASE(64)
    default:
      break;
  }
}
#undef BSW_SWEEP_CASES8
#undef BSW_SWEEP_CASE

// Waves per SIMD the register budget is set for (512 registers per lane
// of a SIMD): four up to 96 columns, three up to 160, two above.
template <int CAP> struct LaneVRegs {
  static constexpr int WAVES = CAP <= 96 ? 4 : (CAP <= 160 ? 3 : 2);
};

template <int CAP, bool SYM>
__global__ void __launch_bounds__(64, LaneVRegs<CAP>::WAVES)
k_lanev(const PairDesc* __restrict__ desc, const long long* __restrict__ range,
        const uint8_t* __restrict__ q, const uint8_t* __restrict__ t,
        const KParams* __restrict__ kp, bsw_result* __restrict__ out,
        bsw_diag* __restrict__ diag, uint32_t* tile_ctr, const Status* st,
        PairDesc* __restrict__ ovf, long long* __restrict__ ovf_count, int persist,
        unsigned long long* __restrict__ cls_cells,
        unsigned long long* __restrict__ work_cells) {
  if (st->bad) return;
  constexpr int NQ = CAP / 4;   // chunks of query columns (in registers)
  constexpr bool QNIB = CAP > 64;             // query codes as nibbles
  constexpr int NQW = QNIB ? NQ / 2 : NQ;     // words of query codes
  extern __shared__ __align__(16) uint32_t mirror[];  // [NQ + 1][64] mirror words
  const int lane = threadIdx.x;
  uint32_t* mir = mirror + lane;
#define MIRW(x) mir[((x) >> 2) * 64]
  const long long begin = range[0], count = range[1];
  const uint32_t ntiles = (uint32_t)((count + 63) >> 6);
  if (ntiles == 0) return;  // an empty class: no atomics
  uint32_t tile = blockIdx.x;
  // settled cells and lane-cells stepped through, summed over the wave's
  // tiles (wave-uniform, so that they take no vector registers)
  unsigned long long tile_cells_acc = 0, span_chunks = 0;
  uint2 r[NQ];
  uint32_t qv[NQW];
  for (;;) {
    if (persist) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(tile_ctr, 1u);
      tile = wave_first(__shfl(v, 0));
    }
    if (tile >= ntiles) break;
    const long long kk = (long long)tile * 64 + lane;
    const bool valid = kk < count;
    // only what the rows need stays live: the descriptor is read again for
    // a pair that goes to the rerun
    PairDesc pd;
    if (valid) {
      pd = desc[begin + kk];
    } else {
      pd.qo = pd.to = 0;
      pd.ql = pd.tl = 0;
      pd.h0 = 1;
      pd.idx = 0;
      pd.pid = 0;
    }
    const uint32_t pidx = pd.idx;
    const KParams& P = kp[pd.pid];
    const int Lq = pd.ql, Lt = valid ? pd.tl : 0, h0 = pd.h0;
    const int oI = P.o_ins, eI = P.e_ins;
    const PkParams pp = {bcast(P.e_del), bcast(P.oe_del), bcast(SYM ? P.oe_del : P.oe_ins),
                         bcast(eI), (s16x2){(short)eI, (short)(2 * eI)}};
    const int zd = P.zdrop;
    const int wb = band_cap(P, Lq);
    // best + slack >= 255: some stored value may have needed more than a byte
    const int ovf_at = 255 - imax(P.amax - P.oe_del, 0);
    // H(i, -1) = h0 - o_del - e_del (i + 1) of Eq. (3), one row at a time
    int hcol = h0 - P.o_del;
    const uint2* srow = (const uint2*)P.prow;  // score row of each target code
    // query codes: aligned words that hold at least one query byte (never
    // past the word of the last byte), byte-aligned to the query start;
    // chunk c's four codes are byte-aligned word c, kept whole for short
    // classes and as nibbles of a shared word (chunks 2m and 2m+1) otherwise
    {
      const uintptr_t qa = (uintptr_t)(q + pd.qo);
      const uint32_t* qw = (const uint32_t*)(qa & ~(uintptr_t)3);
      const uint32_t sh = (uint32_t)(qa & 3);
      const int nw = Lq > 0 ? ((int)sh + Lq + 3) >> 2 : 0;
      uint32_t w0 = nw > 0 ? qw[0] : 0u;
#pragma unroll
      for (int m = 0; m < NQW; ++m) {
        if constexpr (QNIB) {
          const uint32_t w1 = 2 * m + 1 < nw ? qw[2 * m + 1] : 0u;
          const uint32_t w2 = 2 * m + 2 < nw ? qw[2 * m + 2] : 0u;
          qv[m] = __builtin_amdgcn_alignbyte(w1, w0, sh) |
                  (__builtin_amdgcn_alignbyte(w2, w1, sh) << 4);
          w0 = w2;
        } else {
          const uint32_t w1 = m + 1 < nw ? qw[m + 1] : 0u;
          qv[m] = __builtin_amdgcn_alignbyte(w1, w0, sh);
          w0 = w1;
        }
      }
    }
    // first row of Eq. (3) in every column: H(-1, j-1) = max(0, h0 - o_ins -
    // e_ins*j) (h0 itself at column 0), E = 0, in packed 16-bit pairs: the
    // cost o_ins + e_ins*j saturates at 0xffff, above every 8-bit h0, so the
    // saturating difference is exact.  Columns past the query end are never
    // read (they lie past every band end) and need no clearing.
    {
      const uint32_t hh = (uint32_t)h0 | ((uint32_t)h0 << 16);
      const uint32_t e4 = (uint32_t)(4 * eI) | ((uint32_t)(4 * eI) << 16);
      uint32_t c01 = (uint32_t)imin(oI, 65535) | ((uint32_t)imin(oI + eI, 65535) << 16);
      uint32_t c23 = (uint32_t)imin(oI + 2 * eI, 65535) |
                     ((uint32_t)imin(oI + 3 * eI, 65535) << 16);
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        uint32_t a = usubsat16x2(hh, c01);
        const uint32_t b = usubsat16x2(hh, c23);
        if (c == 0) a = (a & 0xffff0000u) | (uint32_t)h0;
        r[c] = make_uint2(__builtin_amdgcn_perm(b, a, 0x06040200u), 0u);
        c01 = uaddsat16x2(c01, e4);
        c23 = uaddsat16x2(c23, e4);
      }
    }

    // bi + 1 and bj + 1 (row and column of the best cell, -1 before one)
    // share a word, as do the stop reason and the rows entered (set at the
    // stop)
    int best = h0, gbest = -1, gi = -1, moff = 0;
    uint32_t bij = 0;
    int beg = 0, end = Lq, stoprows = 0, cells = 0;
    bool live = valid && Lt > 0;
    const uint8_t* ts = t + pd.to;
    // the score row of the next row and the target code of the one after,
    // loaded a row ahead of their use
    uint2 sr = srow[live ? ts[0] : 0];
    uint32_t tn = live && Lt > 1 ? ts[1] : 0u;
    for (int i = 0;; ++i) {
      live = live && i < Lt;
      if (__ballot(live) == 0) break;
      // the packed query codes are unpacked anew in every row: hoisted out of
      // the row loop, the unpacked codes would take twice the registers
#pragma unroll
      for (int m = 0; m < NQW; ++m) asm volatile("" : "+v"(qv[m]));
      const int eD = pp.eD[0];
      int hl = 0;
      if (live) {
        // band (Sec. 5.1 (a)); columns left of beg are read as zero below
        beg = imax(beg, i - wb);
        end = imin(imin(end, i + wb + 1), Lq);
        if (end > beg) cells += end - beg;
        hcol -= eD;
        hl = beg == 0 ? imax(0, hcol) : 0;
      }
      // chunk span of the live lanes: [c0, c1) is visited; chunks <= cb hold
      // some lane's band start (or lie left of it), chunks >= cf some lane's
      // band end (column end itself included)
      const int c0 = wave_min(live ? (beg >> 2) : 0x7fffffff);
      const int cb = wave_max(live ? (beg >> 2) : -1);
      const int cf = wave_min(live ? (end >> 2) : 0x7fffffff);
      const int c1 = wave_max(live ? (end >> 2) + 1 : 0);
      span_chunks += (unsigned)(c1 - c0);
      RowSweep sw;
      sw.mlo = cb + 1;
      sw.mn = imax(cf - cb - 1, 0);
      sw.c1 = c1;
      sw.bb = 8 * beg;
      sw.be = 8 * end;
      sw.lo = sr.x;
      sw.hi = sr.y;
      sw.hp = (uint32_t)hl << 16;
      sw.fp = 0;
      sw.mkey = 0;
      sweep_row<NQ, NQW, QNIB, SYM>(c0, r, qv, mir, pp, sw);
      const uint32_t mkey = sw.mkey;
      // the next row's score row, and the target code of the row after
      if (live && i + 1 < Lt) {
        sr = srow[tn];
        tn = i + 2 < Lt ? ts[i + 2] : 0u;
      }
      if (live) {
        // best score touching the end of the query (Sec. 5.4 (b)): the
        // stored H(i, end - 1) at column end
        if (imax(beg, end) == Lq) {
          const int hend = (int)((MIRW(end) >> (8 * (end & 3))) & 0xffu);
          gi = hend >= gbest ? i : gi;
          gbest = imax(gbest, hend);
        }
        const uint32_t mk = imax((int)(mkey & 0xffffu), (int)(mkey >> 16));
        const int m = (int)(mk >> 8), mj = (int)(mk & 0xffu);
        if (m == 0) {
          stoprows = (1 << 16) | (i + 1);
          live = false;
        } else if (m > best) {
          best = m;
          bij = ((uint32_t)(i + 1) << 16) | (uint32_t)(mj + 1);
          moff = imax(moff, mj > i ? mj - i : i - mj);
        } else if (zd > 0) {
          const int drift = (i - (int)(bij >> 16)) - (mj - (int)(bij & 0xffffu));
          const int drop = best - m - (drift > 0 ? drift * eD : -drift * pp.eI[0]);
          if (drop > zd) {
            stoprows = (2 << 16) | (i + 1);
            live = false;
          }
        }
        if (live) {
          // shrink the band by its empty ends (Sec. 5.1 (c)), a mirror word
          // at a time: the first nonempty column at or after beg (at most
          // end), and the last at or before end (beg - 1 if none)
          while (beg < end) {
            const uint32_t wv = MIRW(beg) >> (8 * (beg & 3));
            if (wv) {
              beg += __builtin_ctz(wv) >> 3;
              break;
            }
            beg = (beg | 3) + 1;
          }
          beg = imin(beg, end);
          int x = end;
          while (x >= beg) {
            const uint32_t wv = MIRW(x) << (8 * (3 - (x & 3)));
            if (wv) {
              x -= __builtin_clz(wv) >> 3;
              break;
            }
            x = (x | 3) - 4;
          }
          x = imax(x, beg - 1);
          end = imin(x + 2, Lq);
        }
      }
    }
    unsigned long long my_cells = 0;
    if (valid) {
      if (best >= ovf_at) {
        // some value may have needed more than a byte: rerun wider
        const unsigned long long pos = atomicAdd((unsigned long long*)ovf_count, 1ull);
        ovf[pos] = desc[begin + kk];
      } else {
        my_cells = (unsigned long long)cells;
        bsw_result res;
        res.score = best;
        res.qle = (int)(bij & 0xffffu);
        res.tle = (int)(bij >> 16);
        res.gtle = gi + 1;
        res.gscore = gbest;
        res.max_off = moff;
        out[pidx] = res;
        if (diag) {
          bsw_diag dg;
          // a pair that never stopped entered every target row
          dg.rows = stoprows ? (stoprows & 0xffff) : Lt;
          dg.stop = stoprows >> 16;
          dg.cells = cells;
          diag[pidx] = dg;
        }
      }
    }
    {
      const unsigned long long ws = wave_sum64(my_cells);
      tile_cells_acc += ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(ws >> 32))
                         << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)ws);
    }
    if (!persist) break;
  }
  if (lane == 0 && tile_cells_acc) atomicAdd(cls_cells, tile_cells_acc);
  if (lane == 0 && span_chunks) atomicAdd(work_cells, span_chunks * 4ull * 64ull);
#undef MIRW
}

}  // namespace bsw
