// rr_train.hip -- training kernels of the closure network (FP32): data
// preparation from filtered fine-grid moments, forward and backward passes,
// deterministic gradient reduction, Adam.
//
// Training data (a-priori regression): the fine moments are box-filtered
// over factor x factor blocks; the coarse node's features are
// (rho_bar, u_bar, b_bar, a_CE) with u_bar = (rho u)_bar / rho_bar and the
// Chapman-Enskog estimate a_CE = -rho_bar c_s^2 tau_c (grad u_bar + grad
// u_bar^T) from the isotropic lattice gradient of the coarse grid; the target
// is tau_sgs / (tau_c - 1) with tau_sgs = (rho u u)_bar - rho_bar u_bar
// u_bar + M(b)_bar - M(b_bar), M = |b|^2 I / 2 - b b.  A constant correction
// D added to a_1^(2) every step settles at a = (tau - 1) D, so this target
// makes the added momentum flux equal the subgrid stress.
//
// One-step solver-in-the-loop objective: the coarse grid is restarted from
// the filtered fine fields at t (f = f_eq(rho_bar, u_bar, b_bar) +
// f_neq,reg(u_bar, a_CE), g = g_eq) and advanced one coarse step with the
// network's correction D(Y) added to a_1^(2) at every node Y; the loss is
// L = sum_X |j_c(X) - j_bar(X, t + fac)|^2 / sum_X |j_bar(t + fac) - j_bar(t)|^2.
// The post-collision populations of a node are affine in its own D:
// f*_i(Y) = f*_i(Y)|_{D=0} + (1 - 1/tau_c) w_i R_i(u(Y)) . D(Y), with
// R_i . D the regularised expansion (second order 9/2, recursive third order
// 27/2, fourth order 81/4) of the coefficient D, so after the pull
// j_c(X) = j_c(X)|_{D=0} + sum_i c_i (1 - 1/tau_c) w_i R_i(u(X - c_i)) . D(X - c_i),
// and dL/dD(Y) is the transpose stencil: (2/den) (1 - 1/tau_c) sum_i
// (c_i . r(Y + c_i)) w_i R_i(u(Y)).  The D = 0 part is prepared once per
// snapshot in FP64; the network-dependent part runs in FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <new>

#include "../../include/rrmhd.h"
#include "rr_internal.h"
#include "rr_kernels.h"
#include "rr_mlp.h"
#include "rr_node.h"
#include "rr_pull.h"

namespace rr {

constexpr int kTB = 256;

__device__ __forceinline__ float gelu32(float z) {
  const float k = 0.7978845608028654f;
  return 0.5f * z * (1.0f + tanhf(k * fmaf(0.044715f, z * z * z, z)));
}

__device__ __forceinline__ float gelu32_grad(float z) {
  const float k = 0.7978845608028654f;
  const float t = tanhf(k * fmaf(0.044715f, z * z * z, z));
  return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * k * fmaf(3.0f * 0.044715f, z * z, 1.0f);
}

// ---- data preparation -------------------------------------------------------
// Coarse box-filtered fields, FP64: out[c][Nc] with c = rho, (rho u)x,
// (rho u)y, bx, by, (rho u u)xx, xy, yy, M(b)xx, M(b)xy.
constexpr int kFilt = 10;

__global__ void k_box_filter(const double *__restrict__ rho, const double *__restrict__ u,
                             const double *__restrict__ b, int nf, int fac,
                             double *__restrict__ out) {
  const int nc = nf / fac;
  const int64_t Nc = (int64_t)nc * nc, Nf = (int64_t)nf * nf;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int cy = (int)(c / nc), cx = (int)(c - (int64_t)cy * nc);
  double acc[kFilt] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = 0; j < fac; ++j)
    for (int i = 0; i < fac; ++i) {
      const int64_t f = (int64_t)(cy * fac + j) * nf + (cx * fac + i);
      const double r = rho[f], ux = u[f], uy = u[Nf + f], bx = b[f], by = b[Nf + f];
      acc[0] += r;
      acc[1] += r * ux;
      acc[2] += r * uy;
      acc[3] += bx;
      acc[4] += by;
      acc[5] += r * ux * ux;
      acc[6] += r * ux * uy;
      acc[7] += r * uy * uy;
      acc[8] += 0.5 * (by * by - bx * bx);  // M_xx = -M_yy
      acc[9] += -bx * by;                   // M_xy
    }
  const double inv = 1.0 / (fac * fac);
  for (int k = 0; k < kFilt; ++k) out[(int64_t)k * Nc + c] = acc[k] * inv;
}

// Coarse features (rho_bar, u_bar, b_bar, a_CE) of node (cx, cy), FP64, from
// the filtered fields.
__device__ void features_at(const double *__restrict__ flt, int nc, double tau_c, int cx,
                            int cy, double out[8]) {
  const int64_t Nc = (int64_t)nc * nc;
  auto F = [&](int k, int xx, int yy) {
    xx = (xx + nc) % nc;
    yy = (yy + nc) % nc;
    return flt[(int64_t)k * Nc + (int64_t)yy * nc + xx];
  };
  auto ubar = [&](int comp, int xx, int yy) { return F(1 + comp, xx, yy) / F(0, xx, yy); };
  // isotropic gradient d_a phi = 3 sum_i w_i phi(x + c_i) c_ia on D2Q9
  double g[2][2] = {{0, 0}, {0, 0}};  // g[a][b] = d_a u_b
  for (int i = 1; i < 9; ++i) {
    const double w = 1.0 / (double)wdiv(i);
    for (int comp = 0; comp < 2; ++comp) {
      const double v = ubar(comp, cx + rr::cx(i), cy + rr::cy(i));
      g[0][comp] += 3.0 * w * v * rr::cx(i);
      g[1][comp] += 3.0 * w * v * rr::cy(i);
    }
  }
  const double r = F(0, cx, cy);
  const double k = -r * tau_c / 3.0;
  out[0] = r;
  out[1] = ubar(0, cx, cy);
  out[2] = ubar(1, cx, cy);
  out[3] = F(3, cx, cy);
  out[4] = F(4, cx, cy);
  out[5] = k * 2.0 * g[0][0];
  out[6] = k * (g[0][1] + g[1][0]);
  out[7] = k * 2.0 * g[1][1];
}

// Features x[Nc][8] and raw targets t[Nc][3] (FP32) from the filtered fields.
__global__ void k_samples(const double *__restrict__ flt, int nc, double tau_c,
                          float *__restrict__ x, float *__restrict__ t) {
  const int64_t Nc = (int64_t)nc * nc;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int cy = (int)(c / nc), cx = (int)(c - (int64_t)cy * nc);
  double ft[8];
  features_at(flt, nc, tau_c, cx, cy, ft);
  for (int k = 0; k < 8; ++k) x[c * 8 + k] = (float)ft[k];
  const double r = ft[0], ux = ft[1], uy = ft[2], bx = ft[3], by = ft[4];
  auto F = [&](int k) { return flt[(int64_t)k * Nc + c]; };
  const double mbxx = 0.5 * (by * by - bx * bx), mbxy = -bx * by;
  const double sxx = F(5) - r * ux * ux + F(8) - mbxx;
  const double sxy = F(6) - r * ux * uy + F(9) - mbxy;
  const double syy = F(7) - r * uy * uy - F(8) + mbxx;
  const double inv = 1.0 / (tau_c - 1.0);
  t[c * 3 + 0] = (float)(sxx * inv);
  t[c * 3 + 1] = (float)(sxy * inv);
  t[c * 3 + 2] = (float)(syy * inv);
}

// ---- one-step objective: data preparation (FP64) ----------------------------
// Regularised expansion R_i . a of a second-order coefficient (axx, axy,
// ayy) at velocity u, without the weight: 9/2 H2:a + 27/2 (H_xxy a_xxy +
// H_xyy a_xyy) + 81/4 H_xxyy a_xxyy with the recursive a_xxy = 2 u_x a_xy +
// u_y a_xx, a_xyy = 2 u_y a_xy + u_x a_yy, a_xxyy = u_x^2 a_yy + u_y^2 a_xx +
// 4 u_x u_y a_xy; written with X2 = 3 c_x^2 - 1 = 3 H_xx, Y2 = 3 c_y^2 - 1.
template <typename R>
__device__ __forceinline__ R reg_expand(int i, R ux, R uy, R axx, R axy, R ayy) {
  const R X2 = (R)(3 * rr::cx(i) * rr::cx(i) - 1), Y2 = (R)(3 * rr::cy(i) * rr::cy(i) - 1);
  const R CX = (R)rr::cx(i), CY = (R)rr::cy(i);
  const R a3x = 2 * ux * axy + uy * axx, a3y = 2 * uy * axy + ux * ayy;
  const R a4 = ux * ux * ayy + uy * uy * axx + 4 * ux * uy * axy;
  return (R)1.5 * (X2 * axx + Y2 * ayy) + (R)9 * CX * CY * axy +
         (R)4.5 * (CY * X2 * a3x + CX * Y2 * a3y) + (R)2.25 * X2 * Y2 * a4;
}

// Equilibrium population i (fourth-order Hermite with the Maxwell stress at
// second order), FP64.
__device__ __forceinline__ double feq64(int i, double rho, double ux, double uy, double bx,
                                        double by) {
  const double X2 = 3 * rr::cx(i) * rr::cx(i) - 1, Y2 = 3 * rr::cy(i) * rr::cy(i) - 1;
  const double CX = rr::cx(i), CY = rr::cy(i);
  const double Axx = rho * ux * ux + 0.5 * (by * by - bx * bx);
  const double Axy = rho * ux * uy - bx * by;
  const double Ayy = rho * uy * uy + 0.5 * (bx * bx - by * by);
  const double t2 = 1.5 * (X2 * Axx + Y2 * Ayy) + 9.0 * CX * CY * Axy;
  const double t3 = 4.5 * rho * (CY * X2 * ux * ux * uy + CX * Y2 * ux * uy * uy);
  const double t4 = 2.25 * rho * X2 * Y2 * ux * ux * uy * uy;
  return (rho + 3.0 * rho * (CX * ux + CY * uy) + t2 + t3 + t4) / (double)wdiv(i);
}

// FP64 features of every coarse node: feat[8][Nc].
__global__ void k_features64(const double *__restrict__ flt, int nc, double tau_c,
                             double *__restrict__ feat) {
  const int64_t Nc = (int64_t)nc * nc;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int cy = (int)(c / nc), cx = (int)(c - (int64_t)cy * nc);
  double ft[8];
  features_at(flt, nc, tau_c, cx, cy, ft);
  for (int k = 0; k < 8; ++k) feat[(int64_t)k * Nc + c] = ft[k];
}

// x[Nc][8] (FP32 features), r0[Nc][2] = j_c(X)|_{D=0} - j_bar(X, t + fac)
// (FP32 of FP64) and dm[Nc] = |j_bar(t + fac) - j_bar(t)|^2 (FP64).
__global__ void k_onestep_prep(const double *__restrict__ flt0, const double *__restrict__ flt1,
                               const double *__restrict__ feat, int nc, double omega,
                               float *__restrict__ x, float *__restrict__ r0,
                               double *__restrict__ dm) {
  const int64_t Nc = (int64_t)nc * nc;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int cy = (int)(c / nc), cx = (int)(c - (int64_t)cy * nc);
  for (int k = 0; k < 8; ++k) x[c * 8 + k] = (float)feat[(int64_t)k * Nc + c];
  double jx = 0.0, jy = 0.0;
  for (int i = 1; i < 9; ++i) {
    // f*_i of the upstream node Y = X - c_i arrives at X
    const int yx = (cx - rr::cx(i) + nc) % nc, yy = (cy - rr::cy(i) + nc) % nc;
    const int64_t q = (int64_t)yy * nc + yx;
    double v[8];
    for (int k = 0; k < 8; ++k) v[k] = feat[(int64_t)k * Nc + q];
    const double fs = feq64(i, v[0], v[1], v[2], v[3], v[4]) +
                      (1.0 - omega) * reg_expand<double>(i, v[1], v[2], v[5], v[6], v[7]) /
                          (double)wdiv(i);
    jx += rr::cx(i) * fs;
    jy += rr::cy(i) * fs;
  }
  const double j1x = flt1[1 * Nc + c], j1y = flt1[2 * Nc + c];
  const double dx = j1x - flt0[1 * Nc + c], dy = j1y - flt0[2 * Nc + c];
  r0[2 * c + 0] = (float)(jx - j1x);
  r0[2 * c + 1] = (float)(jy - j1y);
  dm[c] = dx * dx + dy * dy;
}

// out[0] = sum of v[0..n) in a fixed order (one workgroup of 256).
__global__ __launch_bounds__(256) void k_sum64(const double *__restrict__ v, int64_t n,
                                               double *__restrict__ out) {
  __shared__ double red[256];
  double a = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) a += v[k];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---- forward / backward -----------------------------------------------------
// Per-sample activations are kept in SoA scratch arrays [feature][n] so the
// gradient reduction can stream them.
struct Acts {
  float *xh, *h1, *g1, *h2, *g2, *dy, *dz1, *dz2;  // [8|64|3][n]
};

// tg = nullptr: no a-priori loss; A.dy receives the outputs y instead.
__global__ __launch_bounds__(kTB) void k_forward(const float *__restrict__ p,
                                                 const float *__restrict__ norm,
                                                 const float *__restrict__ x,
                                                 const float *__restrict__ tg, int n, Acts A,
                                                 float *__restrict__ loss_part) {
  __shared__ float P[kNParam];
  __shared__ float red[kTB / 64];
  for (int k = threadIdx.x; k < kNParam; k += kTB) P[k] = p[k];
  __syncthreads();
  const int s = blockIdx.x * kTB + threadIdx.x;
  float l = 0.0f;
  if (s < n) {
    float xh[kNIN], h1[kNH];
#pragma unroll
    for (int k = 0; k < kNIN; ++k) {
      xh[k] = (x[(int64_t)s * kNIN + k] - norm[k]) / norm[kNIN + k];
      A.xh[(int64_t)k * n + s] = xh[k];
    }
#pragma unroll
    for (int i = 0; i < kNH; ++i) {
      float z = P[kOffB1 + i];
#pragma unroll
      for (int k = 0; k < kNIN; ++k) z = fmaf(P[kOffW1 + i * kNIN + k], xh[k], z);
      h1[i] = gelu32(z);
      A.h1[(int64_t)i * n + s] = h1[i];
      A.g1[(int64_t)i * n + s] = gelu32_grad(z);
    }
    float y[kNOUT] = {P[kOffB3 + 0], P[kOffB3 + 1], P[kOffB3 + 2]};
    for (int i = 0; i < kNH; ++i) {
      float z = P[kOffB2 + i];
#pragma unroll
      for (int k = 0; k < kNH; ++k) z = fmaf(P[kOffW2 + i * kNH + k], h1[k], z);
      const float h2 = gelu32(z);
      A.h2[(int64_t)i * n + s] = h2;
      A.g2[(int64_t)i * n + s] = gelu32_grad(z);
#pragma unroll
      for (int o = 0; o < kNOUT; ++o) y[o] = fmaf(P[kOffW3 + o * kNH + i], h2, y[o]);
    }
    if (tg) {
#pragma unroll
      for (int o = 0; o < kNOUT; ++o) {
        const float r = y[o] - tg[(int64_t)s * kNOUT + o] / norm[2 * kNIN + o];
        l = fmaf(r, r, l);
        A.dy[(int64_t)o * n + s] = 2.0f * r / (float)n;
      }
    } else {
      // no target: keep the output for the one-step objective
#pragma unroll
      for (int o = 0; o < kNOUT; ++o) A.dy[(int64_t)o * n + s] = y[o];
    }
  }
  // block sum of the squared residuals (fixed order)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) l += __shfl_xor(l, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(kTB) void k_backward(const float *__restrict__ p, int n, Acts A) {
  __shared__ float P[kNParam];
  for (int k = threadIdx.x; k < kNParam; k += kTB) P[k] = p[k];
  __syncthreads();
  const int s = blockIdx.x * kTB + threadIdx.x;
  if (s >= n) return;
  float dy[kNOUT], dz2[kNH];
#pragma unroll
  for (int o = 0; o < kNOUT; ++o) dy[o] = A.dy[(int64_t)o * n + s];
#pragma unroll
  for (int k = 0; k < kNH; ++k) {
    float d = 0.0f;
#pragma unroll
    for (int o = 0; o < kNOUT; ++o) d = fmaf(P[kOffW3 + o * kNH + k], dy[o], d);
    dz2[k] = d * A.g2[(int64_t)k * n + s];
    A.dz2[(int64_t)k * n + s] = dz2[k];
  }
  for (int k = 0; k < kNH; ++k) {
    float d = 0.0f;
#pragma unroll
    for (int i = 0; i < kNH; ++i) d = fmaf(P[kOffW2 + i * kNH + k], dz2[i], d);
    A.dz1[(int64_t)k * n + s] = d * A.g1[(int64_t)k * n + s];
  }
}

// One-step objective, network-dependent part (FP32).  Node s of the batch is
// node s % Nc of snapshot s / Nc (periodic nc x nc).  D = sigma_out * y with
// y = A.dy from k_forward.  res[2][n] = r0 + sum_i c_i (1 - omega) w_i
// R_i(u(X - c_i)) . D(X - c_i); loss_part = per-workgroup sums of |res|^2.
// q (SoA [3][n], may be null) is added to D (feedback form: the restart's
// extra non-equilibrium relaxes with the correction).
__global__ __launch_bounds__(kTB) void k_onestep_fwd(const float *__restrict__ x,
                                                     const float *__restrict__ r0,
                                                     const float *__restrict__ norm, int nsnap,
                                                     int nc, float om1, Acts A,
                                                     const float *__restrict__ q,
                                                     float *__restrict__ res,
                                                     float *__restrict__ loss_part) {
  __shared__ float red[kTB / 64];
  const int Nc = nc * nc, n = nsnap * Nc;
  const int s = blockIdx.x * kTB + threadIdx.x;
  float l = 0.0f;
  if (s < n) {
    const int sn = s / Nc, c = s - sn * Nc;
    const int cy = c / nc, cx = c - cy * nc;
    const float so0 = norm[2 * kNIN + 0], so1 = norm[2 * kNIN + 1], so2 = norm[2 * kNIN + 2];
    float jx = r0[2 * (int64_t)s], jy = r0[2 * (int64_t)s + 1];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int yx = (cx - rr::cx(i) + nc) % nc, yy = (cy - rr::cy(i) + nc) % nc;
      const int qn = sn * Nc + yy * nc + yx;
      const float ux = x[(int64_t)qn * kNIN + 1], uy = x[(int64_t)qn * kNIN + 2];
      float dxx = so0 * A.dy[qn], dxy = so1 * A.dy[(int64_t)n + qn],
            dyy = so2 * A.dy[2 * (int64_t)n + qn];
      if (q) {
        dxx += q[qn];
        dxy += q[(int64_t)n + qn];
        dyy += q[2 * (int64_t)n + qn];
      }
      const float d = om1 * reg_expand<float>(i, ux, uy, dxx, dxy, dyy) / wdiv(i);
      if (rr::cx(i)) jx = fmaf((float)rr::cx(i), d, jx);
      if (rr::cy(i)) jy = fmaf((float)rr::cy(i), d, jy);
    }
    res[s] = jx;
    res[(int64_t)n + s] = jy;
    l = fmaf(jx, jx, jy * jy);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) l += __shfl_xor(l, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Transpose stencil: dL/dy_k(Y) = sigma_out_k scale om1 sum_i (c_i . res(Y +
// c_i)) w_i dR_i/dD_k(u(Y)), scale = 2 / den; written to A.dy (the outputs
// it overwrites are no longer needed).
// gE (SoA [3][n], may be null) receives dL/dD itself (before sigma_out).
__global__ __launch_bounds__(kTB) void k_onestep_adj(const float *__restrict__ x,
                                                     const float *__restrict__ norm, int nsnap,
                                                     int nc, float om1, float scale, Acts A,
                                                     const float *__restrict__ res,
                                                     float *__restrict__ gE) {
  const int Nc = nc * nc, n = nsnap * Nc;
  const int s = blockIdx.x * kTB + threadIdx.x;
  if (s >= n) return;
  const int sn = s / Nc, c = s - sn * Nc;
  const int cy = c / nc, cx = c - cy * nc;
  const float ux = x[(int64_t)s * kNIN + 1], uy = x[(int64_t)s * kNIN + 2];
  float gxx = 0.0f, gxy = 0.0f, gyy = 0.0f;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int xx = (cx + rr::cx(i) + nc) % nc, xy = (cy + rr::cy(i) + nc) % nc;
    const int q = sn * Nc + xy * nc + xx;
    const float m = ((float)rr::cx(i) * res[q] + (float)rr::cy(i) * res[(int64_t)n + q]) / wdiv(i);
    // columns of the linear map D -> R_i . D
    gxx = fmaf(m, reg_expand<float>(i, ux, uy, 1.0f, 0.0f, 0.0f), gxx);
    gxy = fmaf(m, reg_expand<float>(i, ux, uy, 0.0f, 1.0f, 0.0f), gxy);
    gyy = fmaf(m, reg_expand<float>(i, ux, uy, 0.0f, 0.0f, 1.0f), gyy);
  }
  const float k = scale * om1;
  A.dy[s] = norm[2 * kNIN + 0] * k * gxx;
  A.dy[(int64_t)n + s] = norm[2 * kNIN + 1] * k * gxy;
  A.dy[2 * (int64_t)n + s] = norm[2 * kNIN + 2] * k * gyy;
  if (gE) {
    gE[s] = k * gxx;
    gE[(int64_t)n + s] = k * gxy;
    gE[2 * (int64_t)n + s] = k * gyy;
  }
}

// Feedback form, first network pass done (outputs y0 in A0.dy): the
// restart's extra non-equilibrium q = (tau_c - 1) sigma_out y0 (SoA), and
// the features x1 of that restart (a_1^(2) entries shifted by q).
__global__ __launch_bounds__(kTB) void k_feedback_x1(const float *__restrict__ x,
                                                     const float *__restrict__ norm, int n,
                                                     float tm1, Acts A0, float *__restrict__ q,
                                                     float *__restrict__ x1) {
  const int s = blockIdx.x * kTB + threadIdx.x;
  if (s >= n) return;
#pragma unroll
  for (int k = 0; k < 5; ++k) x1[(int64_t)s * kNIN + k] = x[(int64_t)s * kNIN + k];
#pragma unroll
  for (int o = 0; o < kNOUT; ++o) {
    const float v = tm1 * (norm[2 * kNIN + o] * A0.dy[(int64_t)o * n + s]);
    q[(int64_t)o * n + s] = v;
    x1[(int64_t)s * kNIN + 5 + o] = x[(int64_t)s * kNIN + 5 + o] + v;
  }
}

// Feedback form, after reverse mode through the second pass (dz1 in A1):
// dL/dq = gE + dL/dx1 (a_1^(2) entries, through the second pass's input),
// and the first pass's output gradient dL/dy0 = sigma_out (tau_c - 1) dL/dq.
__global__ __launch_bounds__(kTB) void k_feedback_back(const float *__restrict__ p,
                                                       const float *__restrict__ norm, int n,
                                                       float tm1, Acts A1,
                                                       const float *__restrict__ gE, Acts A0) {
  __shared__ float W1[kNH * kNIN];
  for (int k = threadIdx.x; k < kNH * kNIN; k += kTB) W1[k] = p[kOffW1 + k];
  __syncthreads();
  const int s = blockIdx.x * kTB + threadIdx.x;
  if (s >= n) return;
  float g[kNOUT] = {0.0f, 0.0f, 0.0f};
  for (int i = 0; i < kNH; ++i) {
    const float d = A1.dz1[(int64_t)i * n + s];
#pragma unroll
    for (int o = 0; o < kNOUT; ++o) g[o] = fmaf(W1[i * kNIN + 5 + o], d, g[o]);
  }
#pragma unroll
  for (int o = 0; o < kNOUT; ++o) {
    const float gq = gE[(int64_t)o * n + s] + g[o] / norm[kNIN + 5 + o];
    A0.dy[(int64_t)o * n + s] = norm[2 * kNIN + o] * (tm1 * gq);
  }
}

// Gradient reduction: out[chunk][param] = sum over the chunk's samples of
// the per-sample contribution, in a fixed order.  Parameter p of a weight
// matrix is (row i, column k): dW = sum_s delta_i(s) act_k(s); biases use
// act = 1.  Each block handles one chunk of kChunk samples and 256
// parameters.
constexpr int kChunk = 1024;

__device__ __forceinline__ void param_operands(int q, const Acts &A, const float *&dl,
                                               const float *&ac) {
  // returns the delta row and activation row (nullptr = bias) of parameter q
  if (q < kOffB1) {
    dl = A.dz1 + 0;
    ac = A.xh;
  } else if (q < kOffW2) {
    dl = A.dz1;
    ac = nullptr;
  } else if (q < kOffB2) {
    dl = A.dz2;
    ac = A.h1;
  } else if (q < kOffW3) {
    dl = A.dz2;
    ac = nullptr;
  } else if (q < kOffB3) {
    dl = A.dy;
    ac = A.h2;
  } else {
    dl = A.dy;
    ac = nullptr;
  }
}

__global__ __launch_bounds__(kTB) void k_grad_chunks(int n, Acts A, float *__restrict__ part) {
  const int q = blockIdx.y * kTB + threadIdx.x;
  if (q >= kNParam) return;
  int row, col, ncol;
  const float *dl, *ac;
  param_operands(q, A, dl, ac);
  if (q < kOffB1) {
    row = q / kNIN;
    col = q % kNIN;
    ncol = kNIN;
  } else if (q < kOffW2) {
    row = q - kOffB1;
    col = 0;
    ncol = 0;
  } else if (q < kOffB2) {
    row = (q - kOffW2) / kNH;
    col = (q - kOffW2) % kNH;
    ncol = kNH;
  } else if (q < kOffW3) {
    row = q - kOffB2;
    col = 0;
    ncol = 0;
  } else if (q < kOffB3) {
    row = (q - kOffW3) / kNH;
    col = (q - kOffW3) % kNH;
    ncol = kNH;
  } else {
    row = q - kOffB3;
    col = 0;
    ncol = 0;
  }
  (void)ncol;
  const int64_t s0 = (int64_t)blockIdx.x * kChunk;
  const int64_t s1 = s0 + kChunk < n ? s0 + kChunk : n;
  const float *drow = dl + (int64_t)row * n;
  float acc = 0.0f;
  if (ac) {
    const float *arow = ac + (int64_t)col * n;
    for (int64_t s = s0; s < s1; ++s) acc = fmaf(drow[s], arow[s], acc);
  } else {
    for (int64_t s = s0; s < s1; ++s) acc += drow[s];
  }
  part[(int64_t)blockIdx.x * kNParam + q] = acc;
}

__global__ void k_grad_final(const float *__restrict__ part, int nchunks,
                             const float *__restrict__ loss_part, int nlb, double loss_scale,
                             float *__restrict__ grad, float *__restrict__ loss) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < kNParam) {
    float s = 0.0f;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * kNParam + q];
    grad[q] = s;
  }
  if (q == 0 && loss) {
    double l = 0.0;
    for (int b = 0; b < nlb; ++b) l += loss_part[b];
    *loss = (float)(l * loss_scale);
  }
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = fmaf(b1, m[k], (1.0f - b1) * gk);
  const float vk = fmaf(b2, v[k], (1.0f - b2) * gk * gk);
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ---- imposed fluid state (best-velocity bound of the closure protocol) ----
// Writes the fluid planes of a periodic two-buffer state so that the pulled
// populations of node X are f_eq(rho(X), j(X) / rho(X), b(X)), FP64
// evaluated, stored in the handle's codec: the slot of population i at node
// Y is pulled by Y + c_i, so it receives that node's equilibrium.  The
// magnetic planes are not touched.
template <class C>
__global__ void k_impose_fluid(PlaneGeom G, const double *__restrict__ rho,
                               const double *__restrict__ j, const double *__restrict__ b,
                               typename C::T *__restrict__ dst) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= G.nx) return;
  const int64_t N = (int64_t)G.nx * G.ny;
  const int64_t o = (int64_t)y * G.row + x;  // stored state
  for (int i = 0; i < 9; ++i) {
    int tx = x + rr::cx(i), ty = y + rr::cy(i);
    tx = tx < 0 ? tx + G.nx : (tx >= G.nx ? tx - G.nx : tx);
    ty = ty < 0 ? ty + G.ny : (ty >= G.ny ? ty - G.ny : ty);
    const int64_t q = (int64_t)ty * G.nx + tx;
    const double r = rho[q];
    const double f = feq64(i, r, j[q] / r, j[N + q] / r, b[q], b[N + q]);
    dst[(int64_t)i * G.plane + o] = C::enc((float)(f - 1.0 / (double)wdiv(i)), G.s);
  }
}

}  // namespace rr

// Launcher used by rrmhd_train_impose_fluid (rr_api.hip).
extern "C" RR_HIDDEN int rr_launch_impose_fluid(int storage, const rr::Domain *D, void *dst,
                                                const double *rho, const double *j,
                                                const double *b, hipStream_t st) {
  const dim3 block(64), grid((D->nx + 63) / 64, D->ny);
  const rr::PlaneGeom G{D->plane, D->nx, D->ny, D->s, D->inv_s, 0u, D->row};
  if (storage == rr::kF16)
    hipLaunchKernelGGL(rr::k_impose_fluid<rr::CodecF16>, grid, block, 0, st, G, rho, j, b,
                       (uint16_t *)dst);
  else
    hipLaunchKernelGGL(rr::k_impose_fluid<rr::CodecF32>, grid, block, 0, st, G, rho, j, b,
                       (float *)dst);
  return hipGetLastError() == hipSuccess ? RRMHD_OK : RRMHD_EDEVICE;
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
struct rrmhd_trainer {
  int64_t cap = 0;
  hipStream_t st = nullptr;
  float *acts = nullptr;  // SoA activations
  float *part = nullptr;  // [chunks][4931]
  float *loss_part = nullptr;
  float *res = nullptr;  // one-step residuals [2][cap]
  float *acts2 = nullptr;  // second activation set (feedback form)
  float *fb = nullptr;     // feedback form: x1 [cap][8], q [3][cap], gE [3][cap]
  rr::Acts A{};
};

namespace {
thread_local char g_tdetail[256] = "";
int terr(hipError_t e, const char *w) {
  std::snprintf(g_tdetail, sizeof g_tdetail, "%s: %s", w, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? RRMHD_ENOMEM : RRMHD_EDEVICE;
}
#define THIP(expr)                                  \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return terr(e_, #expr);   \
  } while (0)
}  // namespace

extern "C" {

int rrmhd_train_destroy(rrmhd_trainer *t) {
  if (!t) return RRMHD_OK;
  (void)hipStreamSynchronize(t->st);
  if (t->acts) (void)hipFree(t->acts);
  if (t->part) (void)hipFree(t->part);
  if (t->loss_part) (void)hipFree(t->loss_part);
  if (t->res) (void)hipFree(t->res);
  if (t->acts2) (void)hipFree(t->acts2);
  if (t->fb) (void)hipFree(t->fb);
  delete t;
  return RRMHD_OK;
}

int rrmhd_train_create(int64_t max_batch, void *hip_stream, rrmhd_trainer **out) {
  if (!out) return RRMHD_EINVAL;
  *out = nullptr;
  if (max_batch < 1 || max_batch > (int64_t)1 << 26) return RRMHD_EINVAL;
  rrmhd_trainer *t = new (std::nothrow) rrmhd_trainer();
  if (!t) return RRMHD_ENOMEM;
  t->cap = max_batch;
  t->st = (hipStream_t)hip_stream;
  const int64_t per = rr::kNIN + 4 * rr::kNH + rr::kNOUT + 2 * rr::kNH;
  const int64_t chunks = (max_batch + rr::kChunk - 1) / rr::kChunk;
  const int64_t lblocks = (max_batch + rr::kTB - 1) / rr::kTB;
  hipError_t e = hipMalloc((void **)&t->acts, sizeof(float) * per * max_batch);
  // two chunk sets: the feedback form reduces two activation sets
  if (e == hipSuccess) e = hipMalloc((void **)&t->part, sizeof(float) * 2 * chunks * rr::kNParam);
  if (e == hipSuccess) e = hipMalloc((void **)&t->loss_part, sizeof(float) * lblocks);
  if (e == hipSuccess) e = hipMalloc((void **)&t->res, sizeof(float) * 2 * max_batch);
  if (e == hipSuccess) e = hipMalloc((void **)&t->acts2, sizeof(float) * per * max_batch);
  if (e == hipSuccess) e = hipMalloc((void **)&t->fb, sizeof(float) * 14 * max_batch);
  if (e != hipSuccess) {
    int rc = terr(e, "hipMalloc(trainer)");
    rrmhd_train_destroy(t);
    return rc;
  }
  *out = t;
  return RRMHD_OK;
}

}  // extern "C"

// SoA activation arrays of a batch of n samples inside the trainer's buffer.
static rr::Acts acts_of(const rrmhd_trainer *t, int64_t N, bool second = false) {
  float *a = second ? t->acts2 : t->acts;
  rr::Acts A;
  A.xh = a;
  a += rr::kNIN * N;
  A.h1 = a;
  a += rr::kNH * N;
  A.g1 = a;
  a += rr::kNH * N;
  A.h2 = a;
  a += rr::kNH * N;
  A.g2 = a;
  a += rr::kNH * N;
  A.dy = a;
  a += rr::kNOUT * N;
  A.dz1 = a;
  a += rr::kNH * N;
  A.dz2 = a;
  return A;
}

// Reverse mode from dL/dy in A.dy to the parameter gradient, and the loss
// from the per-workgroup partial sums.
static int backward_and_reduce(rrmhd_trainer *t, const float *params, const rr::Acts &A,
                               int64_t n, int nlb, double loss_scale, float *grad,
                               float *loss) {
  const int nb = (int)((n + rr::kTB - 1) / rr::kTB);
  const int nch = (int)((n + rr::kChunk - 1) / rr::kChunk);
  hipLaunchKernelGGL(rr::k_backward, dim3(nb), dim3(rr::kTB), 0, t->st, params, (int)n, A);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_grad_chunks, dim3(nch, (rr::kNParam + rr::kTB - 1) / rr::kTB),
                     dim3(rr::kTB), 0, t->st, (int)n, A, t->part);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_grad_final, dim3((rr::kNParam + 255) / 256), dim3(256), 0, t->st,
                     t->part, nch, t->loss_part, nlb, loss_scale, grad, loss);
  THIP(hipGetLastError());
  return RRMHD_OK;
}

extern "C" {

int rrmhd_train_loss_grad(rrmhd_trainer *t, const float *params, const float *norm,
                          const float *x, const float *target, int64_t n, float *grad,
                          float *loss) {
  if (!t || !params || !norm || !x || !target || !grad || n < 1 || n > t->cap)
    return RRMHD_EINVAL;
  const rr::Acts A = acts_of(t, n);
  const int nb = (int)((n + rr::kTB - 1) / rr::kTB);
  hipLaunchKernelGGL(rr::k_forward, dim3(nb), dim3(rr::kTB), 0, t->st, params, norm, x, target,
                     (int)n, A, t->loss_part);
  THIP(hipGetLastError());
  return backward_and_reduce(t, params, A, n, nb, 1.0 / (double)n, grad, loss);
}

int rrmhd_train_onestep_loss_grad(rrmhd_trainer *t, const float *params, const float *norm,
                                  const float *x, const float *r0, int nsnap, int nc,
                                  double tau_c, double den, int feedback, float *grad,
                                  float *loss) {
  if (!t || !params || !norm || !x || !r0 || !grad || nsnap < 1 || nc < 1 ||
      !(tau_c > 0.5) || !(den > 0.0) || !std::isfinite(den) || (feedback != 0 && feedback != 1))
    return RRMHD_EINVAL;
  const int64_t n = (int64_t)nsnap * nc * nc;
  if (n > t->cap || n > INT32_MAX) return RRMHD_EINVAL;
  const int nb = (int)((n + rr::kTB - 1) / rr::kTB);
  const float om1 = (float)(1.0 - 1.0 / tau_c);
  const rr::Acts A = acts_of(t, n);
  hipLaunchKernelGGL(rr::k_forward, dim3(nb), dim3(rr::kTB), 0, t->st, params, norm, x,
                     (const float *)nullptr, (int)n, A, t->loss_part);
  THIP(hipGetLastError());
  if (!feedback) {
    hipLaunchKernelGGL(rr::k_onestep_fwd, dim3(nb), dim3(rr::kTB), 0, t->st, x, r0, norm,
                       nsnap, nc, om1, A, (const float *)nullptr, t->res, t->loss_part);
    THIP(hipGetLastError());
    hipLaunchKernelGGL(rr::k_onestep_adj, dim3(nb), dim3(rr::kTB), 0, t->st, x, norm, nsnap,
                       nc, om1, (float)(2.0 / den), A, (const float *)t->res, (float *)nullptr);
    THIP(hipGetLastError());
    return backward_and_reduce(t, params, A, n, nb, 1.0 / den, grad, loss);
  }
  // feedback form: pass 0 on the Chapman-Enskog features (A), pass 1 on the
  // features of the restart carrying q = (tau_c - 1) D0 (A1)
  const float tm1 = (float)(tau_c - 1.0);
  const rr::Acts A1 = acts_of(t, n, true);
  float *x1 = t->fb, *q = t->fb + 8 * n, *gE = t->fb + 11 * n;
  hipLaunchKernelGGL(rr::k_feedback_x1, dim3(nb), dim3(rr::kTB), 0, t->st, x, norm, (int)n, tm1,
                     A, q, x1);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_forward, dim3(nb), dim3(rr::kTB), 0, t->st, params, norm,
                     (const float *)x1, (const float *)nullptr, (int)n, A1, t->loss_part);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_onestep_fwd, dim3(nb), dim3(rr::kTB), 0, t->st, (const float *)x1, r0,
                     norm, nsnap, nc, om1, A1, (const float *)q, t->res, t->loss_part);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_onestep_adj, dim3(nb), dim3(rr::kTB), 0, t->st, (const float *)x1,
                     norm, nsnap, nc, om1, (float)(2.0 / den), A1, (const float *)t->res, gE);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_backward, dim3(nb), dim3(rr::kTB), 0, t->st, params, (int)n, A1);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_feedback_back, dim3(nb), dim3(rr::kTB), 0, t->st, params, norm, (int)n,
                     tm1, A1, (const float *)gE, A);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_backward, dim3(nb), dim3(rr::kTB), 0, t->st, params, (int)n, A);
  THIP(hipGetLastError());
  const int nch = (int)((n + rr::kChunk - 1) / rr::kChunk);
  const dim3 gq(nch, (rr::kNParam + rr::kTB - 1) / rr::kTB);
  hipLaunchKernelGGL(rr::k_grad_chunks, gq, dim3(rr::kTB), 0, t->st, (int)n, A, t->part);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_grad_chunks, gq, dim3(rr::kTB), 0, t->st, (int)n, A1,
                     t->part + (int64_t)nch * rr::kNParam);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_grad_final, dim3((rr::kNParam + 255) / 256), dim3(256), 0, t->st,
                     t->part, 2 * nch, t->loss_part, nb, 1.0 / den, grad, loss);
  THIP(hipGetLastError());
  return RRMHD_OK;
}

int rrmhd_train_adam(rrmhd_trainer *t, float *params, float *m, float *v, const float *grad,
                     float lr, float beta1, float beta2, float eps, int step) {
  if (!t || !params || !m || !v || !grad || step < 1) return RRMHD_EINVAL;
  const float c1 = (float)(1.0 - std::pow((double)beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, step));
  hipLaunchKernelGGL(rr::k_adam, dim3((rr::kNParam + 255) / 256), dim3(256), 0, t->st, params, m,
                     v, grad, rr::kNParam, lr, beta1, beta2, eps, c1, c2);
  THIP(hipGetLastError());
  return RRMHD_OK;
}

int rrmhd_train_samples(const double *rho, const double *u, const double *b, int nf,
                        int factor, double tau_c, double *work, float *x, float *target,
                        void *hip_stream) {
  if (!rho || !u || !b || !work || !x || !target || factor < 1 || nf < factor ||
      nf % factor != 0 || !(tau_c > 0.5))
    return RRMHD_EINVAL;
  const hipStream_t st = (hipStream_t)hip_stream;
  const int nc = nf / factor;
  const int64_t Nc = (int64_t)nc * nc;
  const int blocks = (int)((Nc + 255) / 256);
  hipLaunchKernelGGL(rr::k_box_filter, dim3(blocks), dim3(256), 0, st, rho, u, b, nf, factor,
                     work);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_samples, dim3(blocks), dim3(256), 0, st, work, nc, tau_c, x, target);
  THIP(hipGetLastError());
  return RRMHD_OK;
}

int rrmhd_train_box_filter(const double *rho, const double *u, const double *b, int nf,
                           int factor, double *out, void *hip_stream) {
  if (!rho || !u || !b || !out || factor < 1 || nf < factor || nf % factor != 0)
    return RRMHD_EINVAL;
  const int nc = nf / factor;
  const int64_t Nc = (int64_t)nc * nc;
  hipLaunchKernelGGL(rr::k_box_filter, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0,
                     (hipStream_t)hip_stream, rho, u, b, nf, factor, out);
  THIP(hipGetLastError());
  return RRMHD_OK;
}

int rrmhd_train_onestep_samples(const double *rho0, const double *u0, const double *b0,
                                const double *rho1, const double *u1, const double *b1,
                                int nf, int factor, double tau_c, double *work, float *x,
                                float *r0, double *den, void *hip_stream) {
  if (!rho0 || !u0 || !b0 || !rho1 || !u1 || !b1 || !work || !x || !r0 || !den ||
      factor < 1 || nf < factor || nf % factor != 0 || !(tau_c > 0.5))
    return RRMHD_EINVAL;
  const hipStream_t st = (hipStream_t)hip_stream;
  const int nc = nf / factor;
  const int64_t Nc = (int64_t)nc * nc;
  const int blocks = (int)((Nc + 255) / 256);
  // work: filtered fields at t [10][Nc] and t + factor [10][Nc], FP64
  // features [8][Nc], per-node |j_bar(t + factor) - j_bar(t)|^2 [Nc]: 29 Nc
  double *flt0 = work, *flt1 = work + rr::kFilt * Nc, *feat = work + 2 * rr::kFilt * Nc;
  double *dm = feat + 8 * Nc;
  hipLaunchKernelGGL(rr::k_box_filter, dim3(blocks), dim3(256), 0, st, rho0, u0, b0, nf, factor,
                     flt0);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_box_filter, dim3(blocks), dim3(256), 0, st, rho1, u1, b1, nf, factor,
                     flt1);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_features64, dim3(blocks), dim3(256), 0, st, (const double *)flt0, nc,
                     tau_c, feat);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_onestep_prep, dim3(blocks), dim3(256), 0, st, (const double *)flt0,
                     (const double *)flt1, (const double *)feat, nc, 1.0 / tau_c, x, r0, dm);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_sum64, dim3(1), dim3(256), 0, st, (const double *)dm, Nc, den);
  THIP(hipGetLastError());
  return RRMHD_OK;
}

const char *rrmhd_train_last_error_detail(void) { return g_tdetail; }

}  // extern "C"
