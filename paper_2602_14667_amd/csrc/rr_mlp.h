// rr_mlp.h -- the per-node closure network on matrix cores.
//
// Network (a project addition; the paper has no closure): features
// x = (rho, u_x, u_y, b_x, b_y, a_xx, a_xy, a_yy) of a node, x_hat =
// (x - mu) / sigma, h1 = GELU(W1 x_hat + b1) (64), h2 = GELU(W2 h1 + b2) (64),
// y = W3 h2 + b3 (3); the correction sigma_out * y is added to the second-order
// non-equilibrium coefficients before the recursion of algorithm task 3.
// GELU is the tanh form (Hendrycks & Gimpel 2016).
//
// One wavefront evaluates 64 nodes (one per lane).  Layers 1 and 2 run as
// BF16 MFMA 32x32x8 with FP32 accumulation, written transposed
// (Z^T = W X^T): the accumulator layout of layer 1 (lane = node column,
// registers = hidden rows) is exactly the B-operand layout layer 2 needs, so
// activations never leave registers.  Layer 3 (3 outputs) is 32 FMAs per
// lane plus one cross-half exchange.  x_hat, weights and h1/h2 are BF16
// (round to nearest even); biases, GELU and accumulation are FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {

constexpr int kNH = 64, kNIN = 8, kNOUT = 3;
// Flat FP32 parameter vector: W1[64][8], b1[64], W2[64][64], b2[64],
// W3[3][64], b3[3]; normalisation vector: mu[8], sigma[8], sigma_out[3].
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kNH * kNIN, kOffW2 = kOffB1 + kNH,
              kOffB2 = kOffW2 + kNH * kNH, kOffW3 = kOffB2 + kNH,
              kOffB3 = kOffW3 + kNOUT * kNH, kNParam = kOffB3 + kNOUT;
constexpr int kNNorm = 2 * kNIN + kNOUT;

// Prepared parameters (global memory and the LDS copy share this layout).
struct MlpDev {
  uint16_t w1[kNH * kNIN];  // BF16 bits
  uint16_t w2[kNH * kNH];   // BF16 bits
  float b1[kNH], b2[kNH];
  float w3[kNOUT * kNH];  // BF16-rounded values
  float b3[kNOUT];
  float mu[kNIN], inv_sigma[kNIN], sigma_out[kNOUT];
  int zero;  // 1: all weights and biases zero (correction is exactly 0)
};

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__host__ __device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Two FP32 values -> two BF16 (round to nearest even) packed low/high, one
// v_cvt_pk_bf16_f32 on gfx950; same results as f2bf for finite values.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const floatx2 f = {lo, hi};
  const bf16x2_t v = __builtin_convertvector(f, bf16x2_t);
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  return u;
}

__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

__device__ __forceinline__ float bf2f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// GELU in its tanh form, evaluated through the identity
// z/2 (1 + tanh(v)) = z / (1 + exp(-2 v)), v = sqrt(2/pi) (z + 0.044715 z^3):
// one hardware exp2 and one reciprocal instead of a tanh.  Large |v| give
// exp2 -> inf (result -0 or 0) or -> 0 (result z), as the tanh form does.
__device__ __forceinline__ float gelu_f(float z) {
  const float k2 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;  // -2 sqrt(2/pi) / ln 2
  const float v = fmaf(0.044715f * z, z * z, z);
  const float e = __builtin_amdgcn_exp2f(k2 * v);
  return z * __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ shortx4 ld4(const uint16_t *p) {
  shortx4 v;
  __builtin_memcpy(&v, p, 8);
  return v;
}

// Evaluate the network for the 64 nodes of the calling wavefront.  All 64
// lanes must call it together.  xh: this lane's normalised features;
// W: parameters (LDS); xs: 64 x 8 BF16 scratch of this wave (LDS).
// Returns y[3] (normalised output) of this lane's node.
__device__ __forceinline__ void mlp_wave(const MlpDev *__restrict__ W,
                                         uint16_t *__restrict__ xs,
                                         const float (&xh)[kNIN], float (&y)[kNOUT]) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, col = lane & 31;
  // stage this node's features as row `lane` of X (64 x 8)
  uint32_t *xrow = reinterpret_cast<uint32_t *>(xs + lane * kNIN);
#pragma unroll
  for (int k = 0; k < kNIN / 2; ++k) xrow[k] = pack_bf16x2(xh[2 * k], xh[2 * k + 1]);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  float own[kNOUT] = {0.0f, 0.0f, 0.0f};
#pragma unroll 1
  for (int nb = 0; nb < 2; ++nb) {
    // weights are re-read from LDS in each pass: hoisting them out of this
    // loop would hold ~200 loop-invariant values in registers
    asm volatile("" ::: "memory");
    // layer 1, transposed: Z1^T (64 hidden x 32 nodes) = W1 (64 x 8) X^T
    const shortx4 bx = ld4(xs + (32 * nb + col) * kNIN + 4 * half);
    shortx4 b2op[8];  // layer-2 B operands: h1 rows 8 kk + 4 half + q
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const shortx4 aw = ld4(W->w1 + (32 * mb + col) * kNIN + 4 * half);
      floatx16 acc = {0};
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(aw, bx, acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int h = 32 * mb + 8 * r + 4 * half;
        uint32_t w[2];
#pragma unroll
        for (int q = 0; q < 4; q += 2)
          w[q / 2] = pack_bf16x2(gelu_f(acc[4 * r + q] + W->b1[h + q]),
                                 gelu_f(acc[4 * r + q + 1] + W->b1[h + q + 1]));
        __builtin_memcpy(&b2op[4 * mb + r], w, 8);
      }
    }
    // layer 2, transposed: Z2^T (64 x 32 nodes) = W2 (64 x 64) H1^T
    float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f;
#pragma unroll
    for (int mb2 = 0; mb2 < 2; ++mb2) {
      floatx16 acc = {0};
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const shortx4 aw = ld4(W->w2 + (32 * mb2 + col) * kNH + 8 * kk + 4 * half);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(aw, b2op[kk], acc, 0, 0, 0);
      }
      // layer 3 partial sums over this lane's 16 rows of h2 (h2 rounded to
      // BF16 like the layer inputs)
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        const int h = 32 * mb2 + 8 * (i >> 2) + 4 * half + (i & 3);
        const uint32_t u = pack_bf16x2(gelu_f(acc[i] + W->b2[h]), gelu_f(acc[i + 1] + W->b2[h + 1]));
        const float ha = bf16_lo(u), hb = bf16_hi(u);
        p0 = fmaf(W->w3[0 * kNH + h], ha, p0);
        p1 = fmaf(W->w3[1 * kNH + h], ha, p1);
        p2 = fmaf(W->w3[2 * kNH + h], ha, p2);
        p0 = fmaf(W->w3[0 * kNH + h + 1], hb, p0);
        p1 = fmaf(W->w3[1 * kNH + h + 1], hb, p1);
        p2 = fmaf(W->w3[2 * kNH + h + 1], hb, p2);
      }
    }
    // the other half of the wave holds the other 32 rows of the same nodes
    const float s0 = p0 + __shfl_xor(p0, 32, 64);
    const float s1 = p1 + __shfl_xor(p1, 32, 64);
    const float s2 = p2 + __shfl_xor(p2, 32, 64);
    // lane l's node is node 32 * (l / 32) + l % 32 = l: keep block nb = l / 32
    if (nb == half) {
      own[0] = s0;
      own[1] = s1;
      own[2] = s2;
    }
  }
#pragma unroll
  for (int o = 0; o < kNOUT; ++o) y[o] = own[o] + W->b3[o];
}

// Copy the prepared parameters into LDS (all threads of the block).
__device__ __forceinline__ void mlp_to_lds(const MlpDev *__restrict__ g, MlpDev *s) {
  const uint32_t *src = (const uint32_t *)g;
  uint32_t *dst = (uint32_t *)s;
  constexpr int n = sizeof(MlpDev) / 4;
  for (int k = threadIdx.x + threadIdx.y * blockDim.x; k < n; k += blockDim.x * blockDim.y)
    dst[k] = src[k];
  __syncthreads();
}

}  // namespace rr
