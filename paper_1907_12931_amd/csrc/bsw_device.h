// bsw_device.h -- device-side helpers shared by the kernel translation
// units of libbsw.so (never exported).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "bsw_internal.h"

namespace bsw {

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// Score of target code tb against query code qj: byte qj of the 8-byte
// score row {hi, lo} of tb, sign-extended (v_perm picks the byte).
__device__ __forceinline__ int score_of(uint32_t lo, uint32_t hi, uint32_t qj) {
  return (int)(int8_t)(__builtin_amdgcn_perm(hi, lo, qj) & 0xffu);
}

// Band half-width after the end-bonus cap: a gap longer than
// (qlen*A + bonus - o)/e + 1 can never pay for itself.
__device__ __forceinline__ int band_cap(const KParams& P, int Lq) {
  int w = P.w;
  int num = Lq * P.amax + P.end_bonus - P.o_ins;
  w = imin(w, num >= 0 ? num / P.e_ins + 1 : 1);
  num = Lq * P.amax + P.end_bonus - P.o_del;
  w = imin(w, num >= 0 ? num / P.e_del + 1 : 1);
  return w;
}

// Row-buffer records: (H, E) of one column.
template <int W> struct Rec;
template <> struct Rec<W8> {
  using T = uint16_t;
  static __device__ __forceinline__ T pack(int h, int e) { return (T)(h | (e << 8)); }
  static __device__ __forceinline__ int h(T r) { return r & 0xff; }
  static __device__ __forceinline__ int e(T r) { return r >> 8; }
  static __device__ __forceinline__ bool empty(T r) { return r == 0; }
};
template <> struct Rec<W16> {
  using T = uint32_t;
  static __device__ __forceinline__ T pack(int h, int e) { return (T)h | ((T)e << 16); }
  static __device__ __forceinline__ int h(T r) { return (int)(r & 0xffffu); }
  static __device__ __forceinline__ int e(T r) { return (int)(r >> 16); }
  static __device__ __forceinline__ bool empty(T r) { return r == 0; }
};
template <> struct Rec<W32> {
  using T = int2;
  static __device__ __forceinline__ T pack(int h, int e) { return make_int2(h, e); }
  static __device__ __forceinline__ int h(T r) { return r.x; }
  static __device__ __forceinline__ int e(T r) { return r.y; }
  static __device__ __forceinline__ bool empty(T r) { return (r.x | r.y) == 0; }
};

__device__ __forceinline__ uint32_t wave_first(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// 64-bit wave sum (per-class cell counters).
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Wave-wide inclusive prefix sum and prefix maximum (lane l gets the
// result over lanes 0..l), with DPP: shifts by 1, 2, 4 and 8 lanes inside
// each row of 16 (lanes without a source take the identity), then the last
// lane of row 0 and of row 2 is broadcast into rows 1 and 3, and lane 31
// into rows 2 and 3.  Every lane must be active.
template <bool MAX>
__device__ __forceinline__ int wave_scan(int x) {
  // the identity of the operation, so that the compiler folds each DPP
  // move into its max or add
  constexpr int ID = MAX ? (int)0x80000000u : 0;
  auto op = [](int a, int b) { return MAX ? (a > b ? a : b) : a + b; };
  x = op(x, __builtin_amdgcn_update_dpp(ID, x, 0x111, 0xf, 0xf, false));  // row_shr:1
  x = op(x, __builtin_amdgcn_update_dpp(ID, x, 0x112, 0xf, 0xf, false));  // row_shr:2
  x = op(x, __builtin_amdgcn_update_dpp(ID, x, 0x114, 0xf, 0xf, false));  // row_shr:4
  x = op(x, __builtin_amdgcn_update_dpp(ID, x, 0x118, 0xf, 0xf, false));  // row_shr:8
  x = op(x, __builtin_amdgcn_update_dpp(ID, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
  x = op(x, __builtin_amdgcn_update_dpp(ID, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return x;
}
__device__ __forceinline__ int wave_prefix_sum(int x) { return wave_scan<false>(x); }
__device__ __forceinline__ int wave_prefix_max(int x) { return wave_scan<true>(x); }

// Wave-wide min / max of a per-lane value, returned as a wave-uniform
// scalar: four DPP steps reduce each row of 16 lanes (swap neighbours, swap
// pairs, half-row mirror, row mirror), then the four row results are read
// out and combined on the scalar unit.  Every lane must be active.
__device__ __forceinline__ int wave_min(int v) {
  // every lane has a source in these patterns; the identity as the old
  // value lets the compiler fold each DPP move into its min
  constexpr int ID = 0x7fffffff;
  v = imin(v, __builtin_amdgcn_update_dpp(ID, v, 0xb1, 0xf, 0xf, false));
  v = imin(v, __builtin_amdgcn_update_dpp(ID, v, 0x4e, 0xf, 0xf, false));
  v = imin(v, __builtin_amdgcn_update_dpp(ID, v, 0x141, 0xf, 0xf, false));
  v = imin(v, __builtin_amdgcn_update_dpp(ID, v, 0x140, 0xf, 0xf, false));
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return imin(imin(a, b), imin(c, d));
}
__device__ __forceinline__ int wave_max(int v) {
  constexpr int ID = (int)0x80000000u;
  v = imax(v, __builtin_amdgcn_update_dpp(ID, v, 0xb1, 0xf, 0xf, false));
  v = imax(v, __builtin_amdgcn_update_dpp(ID, v, 0x4e, 0xf, 0xf, false));
  v = imax(v, __builtin_amdgcn_update_dpp(ID, v, 0x141, 0xf, 0xf, false));
  v = imax(v, __builtin_amdgcn_update_dpp(ID, v, 0x140, 0xf, 0xf, false));
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return imax(imax(a, b), imax(c, d));
}

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ s16x2 pk(uint32_t x) { return __builtin_bit_cast(s16x2, x); }
__device__ __forceinline__ uint32_t unpk(s16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ s16x2 pmax(s16x2 a, s16x2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s16x2 pmin(s16x2 a, s16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ s16x2 psubsat(s16x2 a, s16x2 b) {  // unsigned, floored at 0
  return __builtin_bit_cast(
      s16x2, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                           __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ s16x2 bcast(int v) { return (s16x2){(short)v, (short)v}; }

struct PkParams {
  s16x2 eD, oeD, oeI, eI, eI12;  // (e_del, e_del), ..., (e_ins, 2 e_ins)
};

}  // namespace bsw
