// Measured integer VALU peak for the depth-first kernels' instruction pair.
//
// The depth-first stage is rated against the datasheet figure (256 CUs x 4
// SIMDs x 16 lanes x 2.4 GHz).  This probe measures what the device
// sustains for the exact pair of instructions a candidate test issues per
// 32-bit word -- v_and_b32 with a wave-uniform (SGPR) row word, then
// v_bcnt_u32_b32 accumulating -- with eight independent chains per lane and
// eight waves per SIMD, so that neither dependency latency nor occupancy
// limits it.
#include <hip/hip_runtime.h>

#include "../../include/pdfs.h"

namespace {

__global__ __launch_bounds__(256) void k_valu_probe(uint32_t* out, int iters, uint32_t seed) {
  uint32_t y[8], acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    y[k] = (threadIdx.x + 1u) * (2654435761u + 97u * k) ^ seed;
    acc[k] = 0u;
  }
  for (int i = 0; i < iters; ++i) {
    const uint32_t row = __builtin_amdgcn_readfirstlane(seed + (uint32_t)i);   // wave-uniform
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uint32_t t;
      asm volatile("v_and_b32 %0, %1, %2" : "=v"(t) : "s"(row), "v"(y[k]));
      asm volatile("v_bcnt_u32_b32 %0, %1, %2" : "=v"(acc[k]) : "v"(t), "v"(acc[k]));
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += acc[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int32_t pdfs_measure_int_peak(int32_t device, double* lane_ops_per_s) {
  if (!lane_ops_per_s) return PDFS_ERR_INVALID_ARG;
  *lane_ops_per_s = 0.0;
  if (hipSetDevice(device) != hipSuccess) return PDFS_ERR_DEVICE;
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      n_cu < 1)
    return PDFS_ERR_DEVICE;
  const int blocks = n_cu * 8;   // 8 waves per SIMD
  const int iters = 1 << 15;
  uint32_t* out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t rc = PDFS_ERR_DEVICE;
  float ms = 0.f;
  if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) return PDFS_ERR_OUT_OF_MEMORY;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) goto done;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  k_valu_probe<<<blocks, 256, 0, s>>>(out, iters / 8, 1u);   // warm-up (clocks, code)
  if (hipEventRecord(e0, s) != hipSuccess) goto done;
  k_valu_probe<<<blocks, 256, 0, s>>>(out, iters, 12345u);
  if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess) goto done;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) goto done;
  if (ms > 0.f) {
    // two lane-ops (and, popcount-accumulate) per chain per iteration
    const double ops = (double)blocks * 256.0 * (double)iters * 8.0 * 2.0;
    *lane_ops_per_s = ops / (ms * 1e-3);
    rc = PDFS_OK;
  }
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(out);
  return rc;
}
