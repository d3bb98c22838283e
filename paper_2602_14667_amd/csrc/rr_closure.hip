// rr_closure.hip -- the learned closure on the GPU: parameter preparation,
// standalone BF16-MFMA inference, and the fused step with the network
// correcting a_1^(2) inside the collision (periodic domains).
#include <hip/hip_runtime.h>

#include "rr_closure.h"
#include "rr_mlp.h"
#include "rr_node.h"
#include "rr_pull.h"

namespace rr {

// Convert the FP32 parameter and normalisation vectors into the kernel
// layout (BF16 weights in MFMA operand order, FP32 biases, reciprocal
// sigmas) and fill the GELU table: entry v is the tanh-form GELU, evaluated
// in FP64, of the BF16 value with bit pattern v, rounded to the nearest BF16.
// Every block fills a share of the table; block 0 also writes the weights.
// The tanh form z/2 (1 + tanh v), v = sqrt(2/pi) (z + 0.044715 z^3), written
// as z / (1 + e^(-2 v)): the same function without the cancellation of
// 1 + tanh v at large negative z, so every entry is accurate to FP64
// rounding before it is rounded to BF16.
__device__ __forceinline__ uint16_t gelu_entry(int v) {
  const double z = (double)bf2f((uint16_t)v);
  const double k = 0.79788456080286535588;  // sqrt(2 / pi)
  return d2bf(z / (1.0 + exp(-2.0 * k * (z + 0.044715 * z * z * z))));
}

__global__ void k_gelu_table(uint16_t *__restrict__ out) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < kGeluTable; v += gridDim.x * blockDim.x)
    out[v] = gelu_entry(v);
}

__global__ void k_mlp_prepare(const float *__restrict__ p, const float *__restrict__ norm,
                              MlpDev *__restrict__ out) {
  const int t = threadIdx.x;
  for (int v = blockIdx.x * blockDim.x + t; v < kGeluTable; v += gridDim.x * blockDim.x)
    out->gelu[v] = gelu_entry(v);
  if (blockIdx.x != 0) return;
  for (int k = t; k < kNH * kNIN; k += blockDim.x) out->w1[k] = f2bf(p[kOffW1 + k]);
  // layer 2, A operand of lane (m, s) in K block kb of output block mb:
  // W2[32 mb + m][hid_of(kb, s, j)], j = 0..7
  for (int k = t; k < 2 * 4 * 2 * 32 * 8; k += blockDim.x) {
    const int j = k & 7, m = (k >> 3) & 31, sh = (k >> 8) & 1, kb = (k >> 9) & 3, mb = k >> 11;
    out->w2p[k] = f2bf(p[kOffW2 + (32 * mb + m) * kNH + hid_of(kb, sh, j)]);
  }
  for (int k = t; k < 4 * 2 * kNOUT * 8; k += blockDim.x) {
    const int j = k & 7, o = (k >> 3) % kNOUT, r = (k >> 3) / kNOUT, sh = r & 1, kb = r >> 1;
    out->w3p[k] = f2bf(p[kOffW3 + o * kNH + hid_of(kb, sh, j)]);
  }
  for (int k = t; k < kNH; k += blockDim.x) {
    out->b1[k] = p[kOffB1 + k];
    out->b2[k] = p[kOffB2 + k];
  }
  if (t < kNOUT) {
    out->b3[t] = p[kOffB3 + t];
    out->sigma_out[t] = norm[2 * kNIN + t];
  }
  if (t < kNIN) {
    out->mu[t] = norm[t];
    out->inv_sigma[t] = 1.0f / norm[kNIN + t];
  }
  if (t == 0) {
    out->zero = 0;
    out->pad_ = 0;
  }
}

struct ClosureHook {
  const MlpDev *W;
  __device__ __forceinline__ void operator()(float rho, float ux, float uy, float bx, float by,
                                             float &axx, float &axy, float &ayy) const {
    const float x[kNIN] = {rho, ux, uy, bx, by, axx, axy, ayy};
    float xh[kNIN], y[kNOUT];
#pragma unroll
    for (int k = 0; k < kNIN; ++k) xh[k] = (x[k] - W->mu[k]) * W->inv_sigma[k];
    mlp_wave(W, xh, y);
    axx = fmaf(W->sigma_out[0], y[0], axx);
    axy = fmaf(W->sigma_out[1], y[1], axy);
    ayy = fmaf(W->sigma_out[2], y[2], ayy);
  }
};

// Standalone inference: y[n][3] (normalised outputs) for raw features
// x[n][8].  One wave per 64 samples, 16 waves per block (the parameters and
// the GELU table fill most of a CU's LDS, so one block per CU carries four
// waves per SIMD); lanes past n evaluate a copy of sample 0 and discard it.
__global__ __launch_bounds__(1024) void k_mlp_eval(const MlpDev *__restrict__ g,
                                                    const float *__restrict__ x,
                                                    float *__restrict__ y, int64_t n) {
  __shared__ MlpDev W;
  mlp_to_lds(g, &W);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nw = (n + 63) / 64;
  for (int64_t w = (int64_t)blockIdx.x * 16 + wave; w < nw; w += (int64_t)gridDim.x * 16) {
    asm volatile("" ::: "memory");  // weights stay in LDS (see k_step_closure)
    const int64_t s = w * 64 + lane;
    const int64_t sc = s < n ? s : 0;
    float xh[kNIN], out[kNOUT];
#pragma unroll
    for (int k = 0; k < kNIN; ++k) xh[k] = (x[sc * kNIN + k] - W.mu[k]) * W.inv_sigma[k];
    mlp_wave(&W, xh, out);
    if (s < n) {
#pragma unroll
      for (int o = 0; o < kNOUT; ++o) y[s * kNOUT + o] = out[o];
    }
  }
}

// Fused step with the closure, periodic domain.  A tile is 64 x 16 nodes:
// wave w of the block takes row 16 ty + w, lanes take 64 consecutive x.  The
// grid is persistent (one 1024-thread block per CU, the LDS holding the
// parameters and the GELU table) so the parameters are staged once per block.
template <class C, bool NT, int RM>
__global__ __launch_bounds__(1024) void k_step_closure(PlaneGeom G, CollideParams P,
                                                       const MlpDev *__restrict__ g,
                                                       int tiles_x, int ntiles,
                                                       const typename C::T *__restrict__ src,
                                                       typename C::T *__restrict__ dst) {
  __shared__ MlpDev W;
  mlp_to_lds(g, &W);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const ClosureHook hook{&W};
  // one band of tiles per XCD (tile_band)
  const TileBand B = tile_band(ntiles);
  for (int t = B.first; t < B.end; t += B.stride) {
    // keep the weights in LDS: without this the compiler hoists their loads
    // out of the tile loop and the register file overflows
    asm volatile("" ::: "memory");
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int y = ty * 16 + wave;  // one row per wavefront
    if (y >= G.ny) continue;  // whole wave idle (wave-uniform)
    const int xr = tx * 64 + lane;
    const bool active = xr < G.nx;
    const int x = active ? xr : G.nx - 1;  // idle lanes still join the MLP
    float d[kQ], gg[2 * kQm];
    pull_node_per<C, false>(G, row_addr<RM>(G, src, y), x, d, gg);
    collide<false>(d, gg, P, hook);
    if (active) store_node<C, NT, RM>(G, dst, x, y, d, gg);
  }
}

size_t mlp_dev_bytes() { return sizeof(MlpDev); }

hipError_t launch_gelu_table(uint16_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_gelu_table, dim3(64), dim3(256), 0, st, out);
  return hipGetLastError();
}

hipError_t launch_mlp_prepare(const float *params, const float *norm, MlpDev *out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_prepare, dim3(64), dim3(256), 0, st, params, norm, out);
  return hipGetLastError();
}

hipError_t launch_mlp_eval(const MlpDev *mlp, const float *x, float *y, int64_t n,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t waves = (n + 63) / 64, blocks = (waves + 15) / 16;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_mlp_eval, dim3((unsigned)blocks), dim3(1024), 0, st, mlp, x, y, n);
  return hipGetLastError();
}

template <int RM>
static void closure_t(int storage, const Domain &D, const PlaneGeom &G, const CollideParams &P,
                      const MlpDev *mlp, int tiles_x, int ntiles, int grid, const void *src,
                      void *dst, hipStream_t st) {
  if (storage == kF16 && D.s == 1.0f)
    hipLaunchKernelGGL((k_step_closure<CodecF16U, true, RM>), dim3(grid), dim3(1024), 0, st, G, P,
                       mlp, tiles_x, ntiles, (const uint16_t *)src, (uint16_t *)dst);
  else if (storage == kF16)
    hipLaunchKernelGGL((k_step_closure<CodecF16, true, RM>), dim3(grid), dim3(1024), 0, st, G, P,
                       mlp, tiles_x, ntiles, (const uint16_t *)src, (uint16_t *)dst);
  else
    hipLaunchKernelGGL((k_step_closure<CodecF32, true, RM>), dim3(grid), dim3(1024), 0, st, G, P,
                       mlp, tiles_x, ntiles, (const float *)src, (float *)dst);
}

hipError_t launch_step_closure(int storage, const Domain &D, const MlpDev *mlp,
                               const void *src, void *dst, int grid_blocks, hipStream_t st) {
  const int tiles_x = (D.nx + 63) / 64, tiles_y = (D.ny + 15) / 16;
  const int ntiles = tiles_x * tiles_y;
  int grid = grid_blocks < ntiles ? grid_blocks : ntiles;
  if (grid < 1) grid = 1;
  CollideParams P;
  P.om_c = D.om_c;
  P.omm_c = D.omm_c;
  P.Gx = 0.0f;
  P.Gy = 0.0f;
  P.src_c = 0.0f;
  const PlaneGeom G{D.plane, D.nx, D.ny, D.s, D.inv_s, 0u, D.row};
  if (D.row == D.nx)
    closure_t<RM_OFFSET>(storage, D, G, P, mlp, tiles_x, ntiles, grid, src, dst, st);
  else
    closure_t<RM_UNIFORM>(storage, D, G, P, mlp, tiles_x, ntiles, grid, src, dst, st);
  return hipGetLastError();
}

}  // namespace rr
