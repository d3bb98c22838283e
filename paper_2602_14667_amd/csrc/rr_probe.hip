// rr_probe.hip -- plain device copy used as the measured bandwidth reference
// (and to calibrate memory-traffic counters against a known byte count), and
// the stochastically rounding FP16 encode of the storage codec on arrays.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rrmhd.h"
#include "rr_node.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(const v4f *__restrict__ src,
                                                v4f *__restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(src[i], dst + i);
}

__global__ __launch_bounds__(256) void k_sr_encode(const float *__restrict__ x,
                                                   const uint32_t *__restrict__ r,
                                                   uint16_t *__restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = rr::CodecF16SR::enc_sr(x[i], 1.0f, r[i]);
}

}  // namespace

extern "C" int rrmhd_sr_encode(const float *x, const uint32_t *r, uint16_t *out, int64_t n,
                               void *hip_stream) {
  if (!x || !r || !out || n < 0) return RRMHD_EINVAL;
  if (n == 0) return RRMHD_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  hipLaunchKernelGGL(k_sr_encode, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     x, r, out, n);
  return hipGetLastError() == hipSuccess ? RRMHD_OK : RRMHD_EDEVICE;
}

extern "C" int rrmhd_bandwidth_probe(void *dst, const void *src, int64_t bytes,
                                     void *hip_stream) {
  if (!dst || !src || bytes <= 0 || (bytes & 15) || ((uintptr_t)dst & 15) ||
      ((uintptr_t)src & 15))
    return RRMHD_EINVAL;
  const int64_t n16 = bytes / 16;
  int64_t blocks = (n16 + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0,
                     (hipStream_t)hip_stream, (const v4f *)src, (v4f *)dst, n16);
  return hipGetLastError() == hipSuccess ? RRMHD_OK : RRMHD_EDEVICE;
}
