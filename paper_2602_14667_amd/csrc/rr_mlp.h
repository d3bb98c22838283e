// rr_mlp.h -- the per-node closure network on matrix cores.
//
// Network (a project addition; the paper has no closure): features
// x = (rho, u_x, u_y, b_x, b_y, a_xx, a_xy, a_yy) of a node, x_hat =
// (x - mu) / sigma, h1 = GELU(W1 x_hat + b1) (64), h2 = GELU(W2 h1 + b2) (64),
// y = W3 h2 + b3 (3); the correction sigma_out * y is added to the second-order
// non-equilibrium coefficients before the recursion of algorithm task 3.
// GELU is the tanh form (Hendrycks & Gimpel 2016).
//
// One wavefront evaluates 64 nodes (one per lane) in two passes of 32 nodes.
// All three layers run on the matrix cores, written transposed (Z^T = W X^T)
// so that nodes are the MFMA columns: layer 1 as BF16 MFMA 32x32x8 (K = the 8
// features), layers 2 and 3 as gfx950's BF16 MFMA 32x32x16 with FP32
// accumulation.  The accumulator of a 32x32 MFMA holds, in lane (column c,
// half s) and register r, row 8 (r / 4) + 4 s + r % 4; a layer's
// activations are handed to the next layer as its B operand in exactly that
// register order, and the next layer's weights are stored permuted to match
// (the contraction does not depend on the order of its K index as long as A
// and B agree), so activations never leave registers.  Biases enter as the
// accumulators' initial values.
//
// GELU is a table lookup: the pre-activation is rounded to BF16 (as the next
// layer's operands are), and the table, held in LDS, gives the correctly
// rounded BF16 value of the tanh-form GELU for every one of the 65,536 BF16
// bit patterns (computed once in FP64 when the parameters are prepared).  Two
// VALU instructions and one LDS read per activation replace an exponential
// and a reciprocal, which made the GELUs the kernel's largest cost.
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
constexpr int kGeluTable = 65536;

// Hidden unit held in slot j (0..7) of the 16-wide K block kb (0..3) by a
// lane of half s: the accumulator rows of block kb / 2, registers
// 8 (kb % 2) + j.
__host__ __device__ constexpr int hid_of(int kb, int s, int j) {
  return 32 * (kb >> 1) + 16 * (kb & 1) + 8 * (j >> 2) + 4 * s + (j & 3);
}

// Prepared parameters (global memory and the LDS copy share this layout;
// every array used by 16-byte LDS reads starts on a 16-byte boundary).
struct alignas(16) MlpDev {
  uint16_t gelu[kGeluTable];          // BF16 bits: GELU of each BF16 value
  uint16_t w1[kNH * kNIN];            // BF16 W1, row-major (layer-1 A operand)
  uint16_t w2p[2 * 4 * 2 * 32 * 8];   // BF16 W2 in A-operand order [mb][kb][s][m][j]
  uint16_t w3p[4 * 2 * kNOUT * 8];    // BF16 W3 in A-operand order [kb][s][o][j]
  float b1[kNH], b2[kNH];
  float b3[kNOUT];
  float mu[kNIN], inv_sigma[kNIN], sigma_out[kNOUT];
  int zero;  // 1: all weights and biases zero (correction is exactly 0)
  int pad_;
};

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__host__ __device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// FP64 -> BF16, correctly rounded to nearest even.  The FP32 rounding of v
// can only create a BF16 tie that v itself does not sit on; that case is
// decided by which side of the FP32 value v lies.
__host__ __device__ __forceinline__ uint16_t d2bf(double v) {
  const float f = (float)v;
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  if ((u & 0xffffu) == 0x8000u && (double)f != v) {
    const bool away = (v > (double)f) == (f > 0.0f);
    return (uint16_t)((u >> 16) + (away ? 1u : 0u));
  }
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

__host__ __device__ __forceinline__ float bf2f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

__device__ __forceinline__ shortx4 ld4(const uint16_t *p) {
  shortx4 v;
  __builtin_memcpy(&v, p, 8);
  return v;
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
  bf16x8 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

__device__ __forceinline__ bf16x8 words8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const uint32_t w[4] = {a, b, c, d};
  bf16x8 v;
  __builtin_memcpy(&v, w, 16);
  return v;
}

// Accumulator initialised with the bias of its rows (32 mb + 8 q + 4 s + i).
__device__ __forceinline__ floatx16 bias_acc(const float *b, int mb, int s) {
  floatx16 acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    floatx4 v;
    __builtin_memcpy(&v, b + 32 * mb + 8 * q + 4 * s, 16);
    acc[4 * q + 0] = v[0];
    acc[4 * q + 1] = v[1];
    acc[4 * q + 2] = v[2];
    acc[4 * q + 3] = v[3];
  }
  return acc;
}

// GELU of an accumulator block through the LDS table: eight words of two
// BF16 activations each, in register order.
__device__ __forceinline__ void gelu_block(const uint16_t *__restrict__ tab, const floatx16 &acc,
                                           uint32_t (&w)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t p = pack_bf16x2(acc[2 * k], acc[2 * k + 1]);
    w[k] = (uint32_t)tab[p & 0xffffu] | ((uint32_t)tab[p >> 16] << 16);
  }
}

// Evaluate the network for the 64 nodes of the calling wavefront.  All 64
// lanes must call it together.  xh: this lane's normalised features;
// W: parameters (LDS).  Returns y[3] (normalised output) of this lane's node.
__device__ __forceinline__ void mlp_wave(const MlpDev *__restrict__ W, const float (&xh)[kNIN],
                                         float (&y)[kNOUT]) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, col = lane & 31;
  // this node's features as four words of two BF16; a pass over the nodes of
  // half nb needs, in lane (c, s), features 4 s .. 4 s + 3 of node 32 nb + c:
  // its own words when s == nb, else those of lane (c, 1 - s)
  uint32_t fw[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) fw[k] = pack_bf16x2(xh[2 * k], xh[2 * k + 1]);
  const uint32_t send0 = half ? fw[0] : fw[2], send1 = half ? fw[1] : fw[3];
  const uint32_t recv0 = __shfl_xor(send0, 32, 64), recv1 = __shfl_xor(send1, 32, 64);
  const uint32_t own0 = half ? fw[2] : fw[0], own1 = half ? fw[3] : fw[1];
  float own[kNOUT] = {0.0f, 0.0f, 0.0f};
#pragma unroll 1
  for (int nb = 0; nb < 2; ++nb) {
    // weights are re-read from LDS in each pass: hoisted out of this loop
    // they would hold several hundred values in registers
    asm volatile("" ::: "memory");
    const bool mine = nb == half;
    uint32_t xw[2] = {mine ? own0 : recv0, mine ? own1 : recv1};
    shortx4 bx;
    __builtin_memcpy(&bx, xw, 8);
    // layer 1: Z1^T (64 hidden x 32 nodes) = W1 (64 x 8) X^T
    uint32_t h1[2][8];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      floatx16 acc = bias_acc(W->b1, mb, half);
      const shortx4 aw = ld4(W->w1 + (32 * mb + col) * kNIN + 4 * half);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(aw, bx, acc, 0, 0, 0);
      gelu_block(W->gelu, acc, h1[mb]);
    }
    // layer 2: Z2^T (64 x 32 nodes) = W2 (64 x 64) H1^T, four 16-wide K blocks
    uint32_t h2[2][8];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      floatx16 acc = bias_acc(W->b2, mb, half);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 aw = ld8(W->w2p + (((mb * 4 + kb) * 2 + half) * 32 + col) * 8);
        const uint32_t *hw = h1[kb >> 1] + 4 * (kb & 1);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, words8(hw[0], hw[1], hw[2], hw[3]),
                                                       acc, 0, 0, 0);
      }
      gelu_block(W->gelu, acc, h2[mb]);
    }
    // layer 3: rows 0..2 of a 32-row product carry the three outputs (the
    // other rows' weights are zero)
    floatx16 acc3 = {0};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      bf16x8 aw = {};
      if (col < kNOUT) aw = ld8(W->w3p + ((kb * 2 + half) * kNOUT + col) * 8);
      const uint32_t *hw = h2[kb >> 1] + 4 * (kb & 1);
      acc3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, words8(hw[0], hw[1], hw[2], hw[3]),
                                                      acc3, 0, 0, 0);
    }
    // output o of node 32 nb + c sits in lane c (half 0), register o; its
    // owner is lane 32 nb + c
#pragma unroll
    for (int o = 0; o < kNOUT; ++o) {
      const float v = __shfl(acc3[o], col, 64);
      if (mine) own[o] = v;
    }
  }
#pragma unroll
  for (int o = 0; o < kNOUT; ++o) y[o] = own[o] + W->b3[o];
}

// Copy the prepared parameters into LDS (all threads of the block).
__device__ __forceinline__ void mlp_to_lds(const MlpDev *__restrict__ g, MlpDev *s) {
  const uint4 *src = (const uint4 *)g;
  uint4 *dst = (uint4 *)s;
  constexpr int n = sizeof(MlpDev) / 16;
  static_assert(sizeof(MlpDev) % 16 == 0, "MlpDev is copied in 16-byte words");
  for (int k = threadIdx.x + threadIdx.y * blockDim.x; k < n; k += blockDim.x * blockDim.y)
    dst[k] = src[k];
  __syncthreads();
}

}  // namespace rr
