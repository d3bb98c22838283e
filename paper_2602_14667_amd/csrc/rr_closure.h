// rr_closure.h -- launch interfaces of the closure kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rr_kernels.h"

namespace rr {

struct MlpDev;

hipError_t launch_mlp_prepare(const float *params, const float *norm, MlpDev *out,
                              hipStream_t st);
hipError_t launch_mlp_eval(const MlpDev *mlp, const float *x, float *y, int64_t n,
                           hipStream_t st);
hipError_t launch_step_closure(int storage, const Domain &D, const MlpDev *mlp,
                               const void *src, void *dst, int grid_blocks, hipStream_t st);
size_t mlp_dev_bytes();
// The closure's GELU table (65,536 BF16 bit patterns) written to out.
hipError_t launch_gelu_table(uint16_t *out, hipStream_t st);

}  // namespace rr
