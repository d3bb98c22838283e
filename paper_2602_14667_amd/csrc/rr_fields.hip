// rr_fields.hip -- derived diagnostic fields of a periodic grid (FP64):
// the local current density j_z of Eq. current, evaluated from g - g_eq
// (no finite differences), and the vorticity w_z = d_x u_y - d_y u_x with
// the isotropic lattice gradient of Sec. III.  Used to compare with the
// peak current and vorticity the paper tabulates.
#include <hip/hip_runtime.h>

#include "rr_internal.h"
#include "rr_kernels.h"
#include "rr_node.h"
#include "rr_pull.h"

namespace rr {

// SWAPPED: the layout a single-buffer handle holds after an odd number of
// steps, f_i(x) in slot opp(i) of x itself.
// One row per workgroup (blockIdx.y), so RM_UNIFORM applies to any layout.
template <class C, bool SWAPPED, int RM>
__global__ void k_current(PlaneGeom G, const typename C::T *__restrict__ src, double omega_m,
                          double Gx, double Gy, double *__restrict__ jz,
                          double *__restrict__ upl) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= G.nx) return;
  using T = typename C::T;
  constexpr uint32_t E = sizeof(T);
  const RowAddr<T> A = row_addr<RM>(G, src, y);
  float d[kQ], g[2 * kQm];
  if constexpr (SWAPPED) {
    const uint32_t o = A.oz + x * E;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      d[i] = C::dec(ld_at<T, false>(plane_ptr(A.z, opp_f(i), G.plane), o), G.inv_s);
#pragma unroll
    for (int j = 0; j < kQm; ++j)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        g[2 * j + c] =
            C::dec(ld_at<T, false>(plane_ptr(A.z, gplane(opp_g(j), c), G.plane), o), G.inv_s);
  } else {
    pull_node_per<C, false>(G, A, x, d, g);
  }
  double dr = 0.0, jx = 0.0, jy = 0.0, bx = 0.0, by = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    dr += (double)d[i];
    jx += (double)cx(i) * d[i];
    jy += (double)cy(i) * d[i];
  }
#pragma unroll
  for (int j = 0; j < kQm; ++j) {
    bx += (double)g[2 * j];
    by += (double)g[2 * j + 1];
  }
  const double rho = 1.0 + dr;
  const double ux = (jx + 0.5 * rho * Gx) / rho, uy = (jy + 0.5 * rho * Gy) / rho;
  // eps_ab sum_j e_ja (g_jb - g_eq,jb) = sum_j [e_jx (g_jy - geq_jy) - e_jy (g_jx - geq_jx)]
  const double Ez = ux * by - uy * bx;
  double s = 0.0;
#pragma unroll
  for (int j = 1; j < kQm; ++j) {
    const double psi = 1.0 / 6.0;
    const double gxe = psi * (bx - 3.0 * ey(j) * Ez), gye = psi * (by + 3.0 * ex(j) * Ez);
    s += ex(j) * ((double)g[2 * j + 1] - gye) - ey(j) * ((double)g[2 * j] - gxe);
  }
  const int64_t N = (int64_t)G.nx * G.ny, o = (int64_t)y * G.nx + x;
  if (jz) jz[o] = -omega_m * 3.0 * s;
  upl[o] = ux;
  upl[N + o] = uy;
}

__global__ void k_vorticity(int nx, int ny, const double *__restrict__ upl,
                            double *__restrict__ wz) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= nx) return;
  const int64_t N = (int64_t)nx * ny;
  double dxuy = 0.0, dyux = 0.0;
#pragma unroll
  for (int i = 1; i < kQ; ++i) {
    int xx = x + cx(i), yy = y + cy(i);
    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    const int64_t o = (int64_t)yy * nx + xx;
    const double w = (i & 1) ? 1.0 / 36.0 : 1.0 / 9.0;
    dxuy += w * upl[N + o] * cx(i);
    dyux += w * upl[o] * cy(i);
  }
  wz[(int64_t)y * nx + x] = 3.0 * (dxuy - dyux);
}

}  // namespace rr

// Launcher used by rrmhd_current_vorticity (rr_api.hip).
extern "C" RR_HIDDEN int rr_launch_current_vorticity(int storage, const rr::Domain *D, const void *src,
                                           double omega_m, double *jz, double *wz,
                                           double *upl, hipStream_t st, int swapped) {
  const dim3 block(64), grid((D->nx + 63) / 64, D->ny);
  const rr::PlaneGeom G{D->plane, D->nx, D->ny, D->s, D->inv_s, 0u, D->row};
  const double gx = D->Gx, gy = D->Gy;
  auto s16 = (const uint16_t *)src;
  auto s32 = (const float *)src;
  const bool rows = D->row != D->nx;
  if (storage == rr::kF16) {
    if (swapped && rows)
      hipLaunchKernelGGL((rr::k_current<rr::CodecF16, true, rr::RM_UNIFORM>), grid, block, 0, st, G, s16, omega_m, gx, gy, jz, upl);
    else if (swapped)
      hipLaunchKernelGGL((rr::k_current<rr::CodecF16, true, rr::RM_OFFSET>), grid, block, 0, st, G, s16, omega_m, gx, gy, jz, upl);
    else if (rows)
      hipLaunchKernelGGL((rr::k_current<rr::CodecF16, false, rr::RM_UNIFORM>), grid, block, 0, st, G, s16, omega_m, gx, gy, jz, upl);
    else
      hipLaunchKernelGGL((rr::k_current<rr::CodecF16, false, rr::RM_OFFSET>), grid, block, 0, st, G, s16, omega_m, gx, gy, jz, upl);
  } else {
    if (swapped && rows)
      hipLaunchKernelGGL((rr::k_current<rr::CodecF32, true, rr::RM_UNIFORM>), grid, block, 0, st, G, s32, omega_m, gx, gy, jz, upl);
    else if (swapped)
      hipLaunchKernelGGL((rr::k_current<rr::CodecF32, true, rr::RM_OFFSET>), grid, block, 0, st, G, s32, omega_m, gx, gy, jz, upl);
    else if (rows)
      hipLaunchKernelGGL((rr::k_current<rr::CodecF32, false, rr::RM_UNIFORM>), grid, block, 0, st, G, s32, omega_m, gx, gy, jz, upl);
    else
      hipLaunchKernelGGL((rr::k_current<rr::CodecF32, false, rr::RM_OFFSET>), grid, block, 0, st, G, s32, omega_m, gx, gy, jz, upl);
  }
  if (hipGetLastError() != hipSuccess) return RRMHD_EDEVICE;
  if (wz) {
    hipLaunchKernelGGL(rr::k_vorticity, grid, block, 0, st, D->nx, D->ny, upl, wz);
    if (hipGetLastError() != hipSuccess) return RRMHD_EDEVICE;
  }
  return RRMHD_OK;
}
