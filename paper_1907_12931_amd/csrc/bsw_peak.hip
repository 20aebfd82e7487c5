// bsw_peak.hip -- measured integer-VALU peak of the device (the roofline
// that the extension kernels are reported against).
//
// Every lane runs eight independent dependency chains of one instruction
// kind (written in inline asm so that the compiler cannot fold them), on a
// grid of many waves per SIMD over every CU.  The rate is lane-instructions
// per second; a packed 16-bit instruction counts as two operations.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/bsw.h"

namespace bsw {

namespace {

constexpr int PEAK_UNROLL = 16;  // instructions per chain per loop trip
constexpr int PEAK_CHAINS = 8;

template <int KIND>
__device__ __forceinline__ void step(uint32_t& a, uint32_t b, uint32_t c) {
  if constexpr (KIND == BSW_PEAK_ADD_U32)
    asm volatile("v_add_u32 %0, %0, %1" : "+v"(a) : "v"(b));
  else if constexpr (KIND == BSW_PEAK_MAX3_I32)
    asm volatile("v_max3_i32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
  else if constexpr (KIND == BSW_PEAK_PK_ADD_U16)
    asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a) : "v"(b));
  else
    asm volatile("v_pk_max_i16 %0, %0, %1" : "+v"(a) : "v"(b));
}

template <int KIND>
__global__ void __launch_bounds__(256) k_valu_peak(uint32_t* __restrict__ sink, int iters,
                                                   uint32_t seed) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[PEAK_CHAINS];
#pragma unroll
  for (int k = 0; k < PEAK_CHAINS; ++k) a[k] = seed + tid * (k + 1);
  const uint32_t b = seed ^ (tid << 3), c = seed + 7u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < PEAK_UNROLL; ++u) {
#pragma unroll
      for (int k = 0; k < PEAK_CHAINS; ++k) step<KIND>(a[k], b, c);
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < PEAK_CHAINS; ++k) x ^= a[k];
  if (x == 0x9e3779b9u) sink[tid] = x;  // keeps the chains live
}

}  // namespace

}  // namespace bsw

extern "C" int bsw_valu_peak(int32_t device, int32_t kind, double* instr_per_s,
                             double* ops_per_s) {
  using namespace bsw;
  if (kind < BSW_PEAK_ADD_U32 || kind > BSW_PEAK_PK_MAX_I16 || !instr_per_s)
    return BSW_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return BSW_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return BSW_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BSW_EDEVICE;
  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
  const unsigned blocks = (unsigned)prop.multiProcessorCount * 8u;
  const int iters = 4096;
  uint32_t* sink = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BSW_OK;
  if (hipMalloc((void**)&sink, (size_t)blocks * 256 * 4) != hipSuccess) return BSW_ENOMEM;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = BSW_EDEVICE;
  double best = 0.0;
  for (int rep = 0; rep < 4 && rc == BSW_OK; ++rep) {
    (void)hipEventRecord(e0, s);
    switch (kind) {
      case BSW_PEAK_ADD_U32:
        hipLaunchKernelGGL(k_valu_peak<BSW_PEAK_ADD_U32>, dim3(blocks), dim3(256), 0, s, sink,
                           iters, 12345u);
        break;
      case BSW_PEAK_MAX3_I32:
        hipLaunchKernelGGL(k_valu_peak<BSW_PEAK_MAX3_I32>, dim3(blocks), dim3(256), 0, s,
                           sink, iters, 12345u);
        break;
      case BSW_PEAK_PK_ADD_U16:
        hipLaunchKernelGGL(k_valu_peak<BSW_PEAK_PK_ADD_U16>, dim3(blocks), dim3(256), 0, s,
                           sink, iters, 12345u);
        break;
      default:
        hipLaunchKernelGGL(k_valu_peak<BSW_PEAK_PK_MAX_I16>, dim3(blocks), dim3(256), 0, s,
                           sink, iters, 12345u);
        break;
    }
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f) {
      rc = BSW_EDEVICE;
      break;
    }
    const double lane_instr =
        (double)blocks * 256.0 * iters * PEAK_UNROLL * PEAK_CHAINS;
    const double r = lane_instr / (ms * 1e-3);
    if (rep > 0 && r > best) best = r;  // the first run warms the clocks
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(sink);
  if (rc != BSW_OK) return rc;
  *instr_per_s = best;
  if (ops_per_s)
    *ops_per_s = best * (kind == BSW_PEAK_PK_ADD_U16 || kind == BSW_PEAK_PK_MAX_I16 ? 2 : 1);
  return BSW_OK;
}
