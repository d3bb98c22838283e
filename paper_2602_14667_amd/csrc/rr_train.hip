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
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <new>

#include "../../include/rrmhd.h"
#include "rr_mlp.h"

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

// Features x[Nc][8] and raw targets t[Nc][3] (FP32) from the filtered fields.
__global__ void k_samples(const double *__restrict__ flt, int nc, double tau_c,
                          float *__restrict__ x, float *__restrict__ t) {
  const int64_t Nc = (int64_t)nc * nc;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int cy = (int)(c / nc), cx = (int)(c - (int64_t)cy * nc);
  auto F = [&](int k, int xx, int yy) {
    xx = (xx + nc) % nc;
    yy = (yy + nc) % nc;
    return flt[(int64_t)k * Nc + (int64_t)yy * nc + xx];
  };
  auto ubar = [&](int comp, int xx, int yy) { return F(1 + comp, xx, yy) / F(0, xx, yy); };
  // isotropic gradient d_a phi = 3 sum_i w_i phi(x + c_i) c_ia on D2Q9
  const int CXs[9] = {0, -1, -1, -1, 0, 1, 1, 1, 0};
  const int CYs[9] = {0, 1, 0, -1, -1, -1, 0, 1, 1};
  double g[2][2] = {{0, 0}, {0, 0}};  // g[a][b] = d_a u_b
  for (int i = 1; i < 9; ++i) {
    const double w = (i & 1) ? 1.0 / 36.0 : 1.0 / 9.0;
    for (int comp = 0; comp < 2; ++comp) {
      const double v = ubar(comp, cx + CXs[i], cy + CYs[i]);
      g[0][comp] += 3.0 * w * v * CXs[i];
      g[1][comp] += 3.0 * w * v * CYs[i];
    }
  }
  const double r = F(0, cx, cy), ux = ubar(0, cx, cy), uy = ubar(1, cx, cy);
  const double bx = F(3, cx, cy), by = F(4, cx, cy);
  const double k = -r * tau_c / 3.0;
  x[c * 8 + 0] = (float)r;
  x[c * 8 + 1] = (float)ux;
  x[c * 8 + 2] = (float)uy;
  x[c * 8 + 3] = (float)bx;
  x[c * 8 + 4] = (float)by;
  x[c * 8 + 5] = (float)(k * 2.0 * g[0][0]);
  x[c * 8 + 6] = (float)(k * (g[0][1] + g[1][0]));
  x[c * 8 + 7] = (float)(k * 2.0 * g[1][1]);
  const double mbxx = 0.5 * (by * by - bx * bx), mbxy = -bx * by;
  const double sxx = F(5, cx, cy) - r * ux * ux + F(8, cx, cy) - mbxx;
  const double sxy = F(6, cx, cy) - r * ux * uy + F(9, cx, cy) - mbxy;
  const double syy = F(7, cx, cy) - r * uy * uy - F(8, cx, cy) + mbxx;
  const double inv = 1.0 / (tau_c - 1.0);
  t[c * 3 + 0] = (float)(sxx * inv);
  t[c * 3 + 1] = (float)(sxy * inv);
  t[c * 3 + 2] = (float)(syy * inv);
}

// ---- forward / backward -----------------------------------------------------
// Per-sample activations are kept in SoA scratch arrays [feature][n] so the
// gradient reduction can stream them.
struct Acts {
  float *xh, *h1, *g1, *h2, *g2, *dy, *dz1, *dz2;  // [8|64|3][n]
};

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
#pragma unroll
    for (int o = 0; o < kNOUT; ++o) {
      const float r = y[o] - tg[(int64_t)s * kNOUT + o] / norm[2 * kNIN + o];
      l = fmaf(r, r, l);
      A.dy[(int64_t)o * n + s] = 2.0f * r / (float)n;
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
                             const float *__restrict__ loss_part, int nlb, int n,
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
    *loss = (float)(l / n);
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

}  // namespace rr

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
struct rrmhd_trainer {
  int64_t cap = 0;
  hipStream_t st = nullptr;
  float *acts = nullptr;  // SoA activations
  float *part = nullptr;  // [chunks][4931]
  float *loss_part = nullptr;
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
  if (e == hipSuccess) e = hipMalloc((void **)&t->part, sizeof(float) * chunks * rr::kNParam);
  if (e == hipSuccess) e = hipMalloc((void **)&t->loss_part, sizeof(float) * lblocks);
  if (e != hipSuccess) {
    int rc = terr(e, "hipMalloc(trainer)");
    rrmhd_train_destroy(t);
    return rc;
  }
  *out = t;
  return RRMHD_OK;
}

int rrmhd_train_loss_grad(rrmhd_trainer *t, const float *params, const float *norm,
                          const float *x, const float *target, int64_t n, float *grad,
                          float *loss) {
  if (!t || !params || !norm || !x || !target || !grad || n < 1 || n > t->cap)
    return RRMHD_EINVAL;
  float *a = t->acts;
  const int64_t N = n;
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
  const int nb = (int)((n + rr::kTB - 1) / rr::kTB);
  const int nch = (int)((n + rr::kChunk - 1) / rr::kChunk);
  hipLaunchKernelGGL(rr::k_forward, dim3(nb), dim3(rr::kTB), 0, t->st, params, norm, x, target,
                     (int)n, A, t->loss_part);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_backward, dim3(nb), dim3(rr::kTB), 0, t->st, params, (int)n, A);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_grad_chunks, dim3(nch, (rr::kNParam + rr::kTB - 1) / rr::kTB),
                     dim3(rr::kTB), 0, t->st, (int)n, A, t->part);
  THIP(hipGetLastError());
  hipLaunchKernelGGL(rr::k_grad_final, dim3((rr::kNParam + 255) / 256), dim3(256), 0, t->st,
                     t->part, nch, t->loss_part, nb, (int)n, grad, loss);
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

const char *rrmhd_train_last_error_detail(void) { return g_tdetail; }

}  // extern "C"
