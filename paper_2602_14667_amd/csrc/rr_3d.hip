// rr_3d.hip -- the three-dimensional extension of the recursive regularised
// LB-MHD step on gfx950: D3Q27 fluid populations with the recursive
// regularisation, D3Q7 vector populations with BGK for the magnetic field.
//
// The paper is two-dimensional and names three-dimensional lattices as the
// next step (Conclusions).  This is the direct generalisation of the
// algorithm of Sec. II.B:
//  - equilibrium: the D3Q27 Hermite series up to sixth order, which is the
//    product of three D1Q3 factors, rho prod_a (1 + e_a) with e(0) = -1.5 u^2
//    and e(+-1) = +-3u + 3u^2, plus the Maxwell stress M = |b|^2/2 I - b b
//    at second order, w_i (9/2) M:H^(2)_i;
//  - a1^(2) by projection, P - (drho/3) I - rho u u - M with P = sum c c d;
//  - the recursion of task 3 in general form, which gives every higher
//    coefficient as a sum over index pairs (p, q) of a1^(2)_pq times the
//    velocities of the other indices, on the 17 D3Q27-supported components
//    of orders 3 to 6 (no direction more than twice);
//  - reconstruction w_i sum_k A_k prod_a F_{n_a}(c_a), F_0 = 1, F_1 = 3c,
//    F_2 = 1.5 (3c^2 - 1) (the Hermite weights 1/(n! c_s^2n) per direction);
//  - collision f* = f_eq + (1 - omega) f_neq,reg;
//  - D3Q7 magnetic lattice, psi = 1/4 (rest) and 1/8, c_m^2 = 1/4:
//    g_eq,j = psi_j [b + 4 e_j.(u b - b u)], BGK with omega_m, the rest
//    population taken from the conserved b as in two dimensions.
// Storage and arithmetic follow the two-dimensional kernels: f_i - w_i and
// g_j stored in FP32 or FP16 (round to nearest even), FP32 arithmetic with
// exactly representable constants and w_i applied as a correctly rounded
// quotient by 1/w_i in {3.375, 13.5, 54, 216}.  Periodic in x, y and z.
// Pull streaming with two buffers, or one buffer with alternating steps: a
// pull whose results go to the opposite-direction slots at x + c_i, then a
// read of the node's own (swapped) slots with local stores.
//
// Velocity order (this library): i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1);
// magnetic j = 0 rest, 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z.  Planes: f_0..f_26,
// then g_0x, g_0y, g_0z, ..., g_6z (48 planes), each [nz][ny][nx].
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <cmath>
#include <new>
#include <utility>

#include "../../include/rrmhd.h"
#include "rr_internal.h"
#include "rr_node.h"
#include "rr_pull.h"

namespace rr3 {

using rr::CodecF16U;
using rr::CodecF32;
using rr::qdiv;
using rr::rdiv;

constexpr int kQ = 27, kQm = 7, kPlanes = kQ + 3 * kQm;

__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int ecomp(int j, int a) {
  return (j == 0 || (j - 1) / 2 != a) ? 0 : ((j & 1) ? 1 : -1);
}
// 1 / w_i: the product of 1.5 (c = 0) and 6 (c = +-1) per direction
__host__ __device__ constexpr float wdiv(int i) {
  return (cx(i) ? 6.0f : 1.5f) * (cy(i) ? 6.0f : 1.5f) * (cz(i) ? 6.0f : 1.5f);
}
__host__ __device__ constexpr double wgt(int i) {
  return (cx(i) ? 1.0 / 6.0 : 2.0 / 3.0) * (cy(i) ? 1.0 / 6.0 : 2.0 / 3.0) *
         (cz(i) ? 1.0 / 6.0 : 2.0 / 3.0);
}

// per-direction Hermite factor F_n(c)
__host__ __device__ constexpr float Fh(int n, int c) {
  return n == 0 ? 1.0f : (n == 1 ? 3.0f * c : 1.5f * (3.0f * c * c - 1.0f));
}

// the 23 regularised components (orders 2..6): counts per direction
struct Comp {
  int nx, ny, nz;
};
__host__ __device__ constexpr Comp comp(int k) {
  constexpr Comp t[23] = {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                          {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2},
                          {1, 1, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1}, {1, 2, 1},
                          {1, 1, 2}, {2, 2, 1}, {2, 1, 2}, {1, 2, 2}, {2, 2, 2}};
  return t[k];
}
template <int I, int K>
__host__ __device__ constexpr float kcoef() {
  return Fh(comp(K).nx, cx(I)) * Fh(comp(K).ny, cy(I)) * Fh(comp(K).nz, cz(I));
}

template <int I, int K>
__device__ __forceinline__ void reg_term(float &r, const float *A) {
  constexpr float k = kcoef<I, K>();
  if constexpr (k != 0.0f) r = fmaf(k, A[K], r);
}
template <int I, int... K>
__device__ __forceinline__ float reg_sum(const float *A, std::integer_sequence<int, K...>) {
  float r = 0.0f;
  (reg_term<I, K>(r, A), ...);
  return r;
}

struct Eq3 {
  float dr, rho;
  float e[3][3];  // e[a][c + 1]: D1Q3 factor minus one, direction a, speed c
  float mdiag[3];  // 1.5 M_aa
  float moff[3];   // 9 M_xy, 9 M_xz, 9 M_yz
};

template <int I>
__device__ __forceinline__ float post_f(const Eq3 &E, const float *A) {
  constexpr int X = cx(I), Y = cy(I), Z = cz(I);
  const float ex = E.e[0][X + 1], ey = E.e[1][Y + 1], ez = E.e[2][Z + 1];
  const float sxy = fmaf(ex, ey, ex + ey);
  const float s = fmaf(sxy, ez, sxy + ez);  // (1 + ex)(1 + ey)(1 + ez) - 1
  float B = fmaf(E.rho, s, E.dr);
  // Maxwell stress: sum_a 1.5 M_aa (3 c_a^2 - 1) + 9 sum_{a<b} M_ab c_a c_b
  float m = E.mdiag[0] * (X ? 2.0f : -1.0f);
  m = fmaf(E.mdiag[1], Y ? 2.0f : -1.0f, m);
  m = fmaf(E.mdiag[2], Z ? 2.0f : -1.0f, m);
  if constexpr (X * Y != 0) m = fmaf((float)(X * Y), E.moff[0], m);
  if constexpr (X * Z != 0) m = fmaf((float)(X * Z), E.moff[1], m);
  if constexpr (Y * Z != 0) m = fmaf((float)(Y * Z), E.moff[2], m);
  const float v = (B + m) + reg_sum<I>(A, std::make_integer_sequence<int, 23>{});
  return qdiv(v, wdiv(I), 1.0f / wdiv(I));
}

template <int... I>
__device__ __forceinline__ void post_all(float *d, const Eq3 &E, const float *A,
                                         std::integer_sequence<int, I...>) {
  ((d[I] = post_f<I>(E, A)), ...);
}

// One collision in place: d[i] = f_i - w_i, g[3j + a] = g_j,a.
__device__ __forceinline__ void collide3(float (&d)[kQ], float (&g)[3 * kQm], float om_c,
                                         float omm_c) {
  float dr = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
  float pxx = 0.0f, pyy = 0.0f, pzz = 0.0f, pxy = 0.0f, pxz = 0.0f, pyz = 0.0f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    dr += d[i];
    if (cx(i)) jx += cx(i) * d[i];
    if (cy(i)) jy += cy(i) * d[i];
    if (cz(i)) jz += cz(i) * d[i];
    if (cx(i)) pxx += d[i];
    if (cy(i)) pyy += d[i];
    if (cz(i)) pzz += d[i];
    if (cx(i) * cy(i)) pxy += (float)(cx(i) * cy(i)) * d[i];
    if (cx(i) * cz(i)) pxz += (float)(cx(i) * cz(i)) * d[i];
    if (cy(i) * cz(i)) pyz += (float)(cy(i) * cz(i)) * d[i];
  }
  const float rho = 1.0f + dr;
  const float rr = __builtin_amdgcn_rcpf(rho);
  const float ux = rdiv(jx, rho, rr), uy = rdiv(jy, rho, rr), uz = rdiv(jz, rho, rr);
  float bx = 0.0f, by = 0.0f, bz = 0.0f;
#pragma unroll
  for (int j = 0; j < kQm; ++j) {
    bx += g[3 * j];
    by += g[3 * j + 1];
    bz += g[3 * j + 2];
  }
  // Maxwell stress M = |b|^2/2 I - b b
  const float bxx = bx * bx, byy = by * by, bzz = bz * bz;
  const float bh = 0.5f * ((bxx + byy) + bzz);
  const float mxx = bh - bxx, myy = bh - byy, mzz = bh - bzz;
  const float mxy = -(bx * by), mxz = -(bx * bz), myz = -(by * bz);
  // a1^(2) = P - (drho / 3) I - rho u u - M
  const float dr3 = qdiv(dr, 3.0f, 1.0f / 3.0f);
  const float rux = rho * ux, ruy = rho * uy, ruz = rho * uz;
  const float axx = fmaf(-rux, ux, pxx - dr3) - mxx;
  const float ayy = fmaf(-ruy, uy, pyy - dr3) - myy;
  const float azz = fmaf(-ruz, uz, pzz - dr3) - mzz;
  const float axy = fmaf(-rux, uy, pxy) - mxy;
  const float axz = fmaf(-rux, uz, pxz) - mxz;
  const float ayz = fmaf(-ruy, uz, pyz) - myz;
  // higher orders: sums over index pairs
  const float x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
  const float xy = ux * uy, xz = ux * uz, yz = uy * uz, xyz_ = xy * uz;
  float A[23];
  A[0] = axx;
  A[1] = ayy;
  A[2] = azz;
  A[3] = axy;
  A[4] = axz;
  A[5] = ayz;
  A[6] = fmaf(uy, axx, 2.0f * ux * axy);                               // xxy
  A[7] = fmaf(uz, axx, 2.0f * ux * axz);                               // xxz
  A[8] = fmaf(ux, ayy, 2.0f * uy * axy);                               // xyy
  A[9] = fmaf(uz, ayy, 2.0f * uy * ayz);                               // yyz
  A[10] = fmaf(ux, azz, 2.0f * uz * axz);                              // xzz
  A[11] = fmaf(uy, azz, 2.0f * uz * ayz);                              // yzz
  A[12] = fmaf(uz, axy, fmaf(uy, axz, ux * ayz));                      // xyz
  A[13] = fmaf(y2, axx, fmaf(x2, ayy, 4.0f * xy * axy));               // xxyy
  A[14] = fmaf(z2, axx, fmaf(x2, azz, 4.0f * xz * axz));               // xxzz
  A[15] = fmaf(z2, ayy, fmaf(y2, azz, 4.0f * yz * ayz));               // yyzz
  A[16] = fmaf(yz, axx, fmaf(2.0f * xz, axy, fmaf(2.0f * xy, axz, x2 * ayz)));  // xxyz
  A[17] = fmaf(xz, ayy, fmaf(2.0f * yz, axy, fmaf(2.0f * xy, ayz, y2 * axz)));  // xyyz
  A[18] = fmaf(xy, azz, fmaf(2.0f * yz, axz, fmaf(2.0f * xz, ayz, z2 * axy)));  // xyzz
  A[19] = fmaf(y2 * uz, axx, fmaf(x2 * uz, ayy, fmaf(4.0f * xyz_, axy,
               fmaf(2.0f * ux * y2, axz, 2.0f * x2 * uy * ayz))));        // xxyyz
  A[20] = fmaf(uy * z2, axx, fmaf(x2 * uy, azz, fmaf(2.0f * ux * z2, axy,
               fmaf(4.0f * xyz_, axz, 2.0f * x2 * uz * ayz))));           // xxyzz
  A[21] = fmaf(ux * z2, ayy, fmaf(ux * y2, azz, fmaf(2.0f * uy * z2, axy,
               fmaf(2.0f * y2 * uz, axz, 4.0f * xyz_ * ayz))));           // xyyzz
  A[22] = fmaf(y2 * z2, axx, fmaf(x2 * z2, ayy, fmaf(x2 * y2, azz,
               4.0f * xyz_ * fmaf(uz, axy, fmaf(uy, axz, ux * ayz)))));   // xxyyzz
#pragma unroll
  for (int k = 0; k < 23; ++k) A[k] = om_c * A[k];

  Eq3 E;
  E.dr = dr;
  E.rho = rho;
  const float u3[3] = {ux, uy, uz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float v = u3[a], v2 = v * v;
    E.e[a][0] = fmaf(-3.0f, v, 3.0f * v2);
    E.e[a][1] = -1.5f * v2;
    E.e[a][2] = fmaf(3.0f, v, 3.0f * v2);
  }
  E.mdiag[0] = 1.5f * mxx;
  E.mdiag[1] = 1.5f * myy;
  E.mdiag[2] = 1.5f * mzz;
  E.moff[0] = 9.0f * mxy;
  E.moff[1] = 9.0f * mxz;
  E.moff[2] = 9.0f * myz;
  post_all(d, E, A, std::make_integer_sequence<int, kQ>{});

  // magnetic: g_eq,j = psi_j (b + 4 e_j.(u b - b u)); E_ab = u_a b_b - u_b b_a
  const float Exy = 4.0f * fmaf(ux, by, -uy * bx);
  const float Exz = 4.0f * fmaf(ux, bz, -uz * bx);
  const float Eyz = 4.0f * fmaf(uy, bz, -uz * by);
  // j = +-x: (b_x, b_y +- Exy, b_z +- Exz); j = +-y: (b_x -+ Exy, b_y, b_z +- Eyz);
  // j = +-z: (b_x -+ Exz, b_y -+ Eyz, b_z); times 1/8 (exact)
  const float geq[3 * kQm] = {
      0.25f * bx, 0.25f * by, 0.25f * bz,
      0.125f * bx, 0.125f * (by + Exy), 0.125f * (bz + Exz),
      0.125f * bx, 0.125f * (by - Exy), 0.125f * (bz - Exz),
      0.125f * (bx - Exy), 0.125f * by, 0.125f * (bz + Eyz),
      0.125f * (bx + Exy), 0.125f * by, 0.125f * (bz - Eyz),
      0.125f * (bx - Exz), 0.125f * (by - Eyz), 0.125f * bz,
      0.125f * (bx + Exz), 0.125f * (by + Eyz), 0.125f * bz};
#pragma unroll
  for (int k = 3; k < 3 * kQm; ++k) g[k] = fmaf(omm_c, g[k] - geq[k], geq[k]);
  // the collision conserves b: the rest population from sum_j g*_j = b
  g[0] = bx - (((g[3] + g[6]) + (g[9] + g[12])) + (g[15] + g[18]));
  g[1] = by - (((g[4] + g[7]) + (g[10] + g[13])) + (g[16] + g[19]));
  g[2] = bz - (((g[5] + g[8]) + (g[11] + g[14])) + (g[17] + g[20]));
}

struct Dom3 {
  int nx, ny, nz;
  int64_t plane;  // elements between plane starts
  float om_c, omm_c;
};

// byte offsets of the source (x - c) along one axis, indexed by c + 1
struct Src3 {
  uint32_t col[3], row[3], slab[3];
};

template <class C, int P>
__device__ __forceinline__ float ld_plane(const typename C::T *__restrict__ s, const Dom3 &D,
                                          const Src3 &S) {
  int a, b, c;
  if constexpr (P < kQ) {
    a = cx(P);
    b = cy(P);
    c = cz(P);
  } else {
    constexpr int j = (P - kQ) / 3;
    a = ecomp(j, 0);
    b = ecomp(j, 1);
    c = ecomp(j, 2);
  }
  const uint32_t off = S.slab[c + 1] + S.row[b + 1] + S.col[a + 1];
  return C::dec(rr::ld_at<typename C::T, false>(s + (int64_t)P * D.plane, off), 1.0f);
}

template <class C, int... P>
__device__ __forceinline__ void load_all(const typename C::T *__restrict__ s, const Dom3 &D,
                                         const Src3 &S, float *v,
                                         std::integer_sequence<int, P...>) {
  ((v[P] = ld_plane<C, P>(s, D, S)), ...);
}

template <class C, int... P>
__device__ __forceinline__ void store_all(typename C::T *__restrict__ dst, const Dom3 &D,
                                          uint32_t o, const float *v,
                                          std::integer_sequence<int, P...>) {
  ((rr::st_at<typename C::T, true>(dst + (int64_t)P * D.plane, o, C::enc(v[P], 1.0f))), ...);
}

__device__ __forceinline__ Src3 sources(const Dom3 &D, int x, int y, int z, uint32_t E) {
  Src3 S;
  const uint32_t pitch = D.nx * E, slab = (uint32_t)D.ny * pitch;
  // source x - c for c = -1, 0, +1
  S.col[0] = (x == D.nx - 1 ? 0 : x + 1) * E;
  S.col[1] = x * E;
  S.col[2] = (x == 0 ? D.nx - 1 : x - 1) * E;
  S.row[0] = (y == D.ny - 1 ? 0 : y + 1) * pitch;
  S.row[1] = y * pitch;
  S.row[2] = (y == 0 ? D.ny - 1 : y - 1) * pitch;
  S.slab[0] = (z == D.nz - 1 ? 0 : z + 1) * slab;
  S.slab[1] = z * slab;
  S.slab[2] = (z == 0 ? D.nz - 1 : z - 1) * slab;
  return S;
}

// Tile of a workgroup: the grid is (row tiles of a z plane, nz) and the
// hardware deals workgroups to the eight XCDs in turn in linear order.  With
// xcd set, within each run of 64 consecutive workgroups XCD k takes tiles
// 8k .. 8k + 7 of the run (neighbouring rows), so their y halos meet in one
// L2.
struct Tile3 {
  int t, z;
};
__device__ __forceinline__ Tile3 tile3(int xcd) {
  const int n = gridDim.x * gridDim.y;
  int L = blockIdx.x + gridDim.x * blockIdx.y;
  if (xcd) {
    const int g = L >> 6, j = L & 63;
    if ((g + 1) * 64 <= n) L = (g << 6) + ((j & 7) << 3) + (j >> 3);
  }
  return Tile3{L % (int)gridDim.x, L / (int)gridDim.x};
}

template <class C>
__global__ __launch_bounds__(256) void k_step3(Dom3 D, int tiles_x, int xcd,
                                               const typename C::T *__restrict__ src,
                                               typename C::T *__restrict__ dst) {
  const Tile3 T = tile3(xcd);
  const int tx = T.t % tiles_x, ty = T.t / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  const int y = ty * blockDim.y + threadIdx.y;
  const int z = T.z;
  if (x >= D.nx || y >= D.ny) return;
  constexpr uint32_t E = sizeof(typename C::T);
  const Src3 S = sources(D, x, y, z, E);
  float v[kPlanes];
  load_all<C>(src, D, S, v, std::make_integer_sequence<int, kPlanes>{});
  float(&d)[kQ] = *reinterpret_cast<float(*)[kQ]>(v);
  float(&g)[3 * kQm] = *reinterpret_cast<float(*)[3 * kQm]>(v + kQ);
  collide3(d, g, D.om_c, D.omm_c);
  store_all<C>(dst, D, S.slab[1] + S.row[1] + S.col[1], v,
               std::make_integer_sequence<int, kPlanes>{});
}

// ---- single-buffer (in-place) streaming ---------------------------------------
// Steps alternate between two forms that each write only the locations their
// own thread has just read: phase 0 pulls as k_step3 does and writes f*_i(x)
// into the slot just read for the opposite direction, buf[opp(i)][x + c_i];
// phase 1 reads the node's own swapped slots (buf[opp(i)][x] = f_i(x)) and
// stores locally, which restores the pull layout.  Slot (p, x) is read and
// written only by node x + c_p, for any box.
__host__ __device__ constexpr int opp_plane(int P) {
  if (P < kQ) return kQ - 1 - P;
  const int j = (P - kQ) / 3, a = (P - kQ) % 3;
  const int oj = j == 0 ? 0 : ((j & 1) ? j + 1 : j - 1);
  return kQ + 3 * oj + a;
}

template <class C, int P>
__device__ __forceinline__ void st_push(typename C::T *buf, const Dom3 &D, const Src3 &S,
                                        const float *v) {
  int a, b, c;
  if constexpr (P < kQ) {
    a = cx(P);
    b = cy(P);
    c = cz(P);
  } else {
    constexpr int j = (P - kQ) / 3;
    a = ecomp(j, 0);
    b = ecomp(j, 1);
    c = ecomp(j, 2);
  }
  // the source entry of -c is the node x + c
  const uint32_t off = S.slab[1 - c] + S.row[1 - b] + S.col[1 - a];
  rr::st_at<typename C::T, true>(buf + (int64_t)opp_plane(P) * D.plane, off, C::enc(v[P], 1.0f));
}
template <class C, int... P>
__device__ __forceinline__ void push_all(typename C::T *buf, const Dom3 &D, const Src3 &S,
                                         const float *v, std::integer_sequence<int, P...>) {
  (st_push<C, P>(buf, D, S, v), ...);
}

template <class C, int... P>
__device__ __forceinline__ void load_own(const typename C::T *buf, const Dom3 &D, uint32_t o,
                                         float *v, std::integer_sequence<int, P...>) {
  ((v[P] = C::dec(rr::ld_at<typename C::T, false>(buf + (int64_t)opp_plane(P) * D.plane, o),
                  1.0f)),
   ...);
}

template <class C, int PHASE>
__global__ __launch_bounds__(256) void k_step3_inplace(Dom3 D, int tiles_x, int xcd,
                                                       typename C::T *buf) {
  const Tile3 T = tile3(xcd);
  const int tx = T.t % tiles_x, ty = T.t / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  const int y = ty * blockDim.y + threadIdx.y;
  const int z = T.z;
  if (x >= D.nx || y >= D.ny) return;
  constexpr uint32_t E = sizeof(typename C::T);
  const Src3 S = sources(D, x, y, z, E);
  const uint32_t own = S.slab[1] + S.row[1] + S.col[1];
  float v[kPlanes];
  if constexpr (PHASE == 0)
    load_all<C>(buf, D, S, v, std::make_integer_sequence<int, kPlanes>{});
  else
    load_own<C>(buf, D, own, v, std::make_integer_sequence<int, kPlanes>{});
  float(&d)[kQ] = *reinterpret_cast<float(*)[kQ]>(v);
  float(&g)[3 * kQm] = *reinterpret_cast<float(*)[3 * kQm]>(v + kQ);
  collide3(d, g, D.om_c, D.omm_c);
  if constexpr (PHASE == 0)
    push_all<C>(buf, D, S, v, std::make_integer_sequence<int, kPlanes>{});
  else
    store_all<C>(buf, D, own, v, std::make_integer_sequence<int, kPlanes>{});
}

// Debug fill of a population buffer with a NaN pattern (32-bit words).
__global__ void k_poison3(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// The pull layout of a single-buffer state held in its swapped form:
// plane p at x is the node x + c_p's own slot of the opposite direction,
// dst[p][x] = buf[opp(p)][x + c_p], copied bit for bit into dense planes.
template <class T>
__global__ void k_swapped_to_pull3(Dom3 D, const T *__restrict__ buf, T *__restrict__ dst) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= D.nx) return;
  const int64_t N = (int64_t)D.nx * D.ny * D.nz;
  const int64_t o = ((int64_t)z * D.ny + y) * D.nx + x;
  auto wrap = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
#pragma unroll 4
  for (int p = 0; p < kPlanes; ++p) {
    int a, b, c;
    if (p < kQ) {
      a = cx(p);
      b = cy(p);
      c = cz(p);
    } else {
      const int j = (p - kQ) / 3;
      a = ecomp(j, 0);
      b = ecomp(j, 1);
      c = ecomp(j, 2);
    }
    const int64_t src = ((int64_t)wrap(z + c, D.nz) * D.ny + wrap(y + b, D.ny)) * D.nx +
                        wrap(x + a, D.nx);
    dst[(int64_t)p * N + o] = buf[(int64_t)opp_plane(p) * D.plane + src];
  }
}

// ---- initialisation at equilibrium (FP64), pull layout ----------------------
__device__ double feq3_d(int i, const double u[3], const double b[3]) {
  const int c[3] = {cx(i), cy(i), cz(i)};
  double prod = 1.0;
  for (int a = 0; a < 3; ++a) {
    const double e = c[a] == 0 ? -1.5 * u[a] * u[a] : 3.0 * c[a] * u[a] + 3.0 * u[a] * u[a];
    prod *= 1.0 + e;
  }
  const double bh = 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  double m = 0.0;
  for (int a = 0; a < 3; ++a) m += 1.5 * (bh - b[a] * b[a]) * (3.0 * c[a] * c[a] - 1.0);
  m += 9.0 * (-b[0] * b[1] * c[0] * c[1] - b[0] * b[2] * c[0] * c[2] - b[1] * b[2] * c[1] * c[2]);
  return wgt(i) * (prod - 1.0 + m);
}

__device__ double geq3_d(int j, int a, const double u[3], const double b[3]) {
  const double psi = j == 0 ? 0.25 : 0.125;
  double s = b[a];
  for (int c = 0; c < 3; ++c) s += 4.0 * ecomp(j, c) * (u[c] * b[a] - u[a] * b[c]);
  return psi * s;
}

template <class C>
__global__ void k_init3(Dom3 D, const double *__restrict__ u, const double *__restrict__ b,
                        typename C::T *__restrict__ dst) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= D.nx) return;
  const int64_t N = (int64_t)D.nx * D.ny * D.nz;
  const int64_t o = ((int64_t)z * D.ny + y) * D.nx + x;
  auto at = [&](int dx, int dy, int dz) {
    int xx = x + dx, yy = y + dy, zz = z + dz;
    xx = xx < 0 ? xx + D.nx : (xx >= D.nx ? xx - D.nx : xx);
    yy = yy < 0 ? yy + D.ny : (yy >= D.ny ? yy - D.ny : yy);
    zz = zz < 0 ? zz + D.nz : (zz >= D.nz ? zz - D.nz : zz);
    return ((int64_t)zz * D.ny + yy) * D.nx + xx;
  };
  for (int i = 0; i < kQ; ++i) {
    const int64_t p = at(cx(i), cy(i), cz(i));
    const double uu[3] = {u[p], u[N + p], u[2 * N + p]}, bb[3] = {b[p], b[N + p], b[2 * N + p]};
    dst[(int64_t)i * D.plane + o] = C::enc((float)feq3_d(i, uu, bb), 1.0f);
  }
  for (int j = 0; j < kQm; ++j) {
    const int64_t p = at(ecomp(j, 0), ecomp(j, 1), ecomp(j, 2));
    const double uu[3] = {u[p], u[N + p], u[2 * N + p]}, bb[3] = {b[p], b[N + p], b[2 * N + p]};
    for (int a = 0; a < 3; ++a)
      dst[(int64_t)(kQ + 3 * j + a) * D.plane + o] = C::enc((float)geq3_d(j, a, uu, bb), 1.0f);
  }
}

// ---- moments and diagnostics (FP64) ----------------------------------------
struct Mom3 {
  double rho, j[3], u[3], b[3];
};

template <class C, bool SW>
__device__ Mom3 moments3(const Dom3 &D, const typename C::T *__restrict__ s, int x, int y,
                         int z) {
  constexpr uint32_t E = sizeof(typename C::T);
  const Src3 S = sources(D, x, y, z, E);
  float v[kPlanes];
  if constexpr (SW)
    load_own<C>(s, D, S.slab[1] + S.row[1] + S.col[1], v,
                std::make_integer_sequence<int, kPlanes>{});
  else
    load_all<C>(s, D, S, v, std::make_integer_sequence<int, kPlanes>{});
  Mom3 m;
  double dr = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    dr += (double)v[i];
    j[0] += (double)cx(i) * v[i];
    j[1] += (double)cy(i) * v[i];
    j[2] += (double)cz(i) * v[i];
  }
  m.rho = 1.0 + dr;
  for (int a = 0; a < 3; ++a) {
    m.j[a] = j[a];
    m.u[a] = j[a] / m.rho;
    double bs = 0.0;
    for (int q = 0; q < kQm; ++q) bs += (double)v[kQ + 3 * q + a];
    m.b[a] = bs;
  }
  return m;
}

template <class C, bool SW>
__global__ void k_moments3(Dom3 D, const typename C::T *__restrict__ src, double *rho, double *u,
                           double *b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= D.nx) return;
  const Mom3 m = moments3<C, SW>(D, src, x, y, z);
  const int64_t N = (int64_t)D.nx * D.ny * D.nz;
  const int64_t o = ((int64_t)z * D.ny + y) * D.nx + x;
  if (rho) rho[o] = m.rho;
  for (int a = 0; a < 3; ++a) {
    if (u) u[a * N + o] = m.u[a];
    if (b) b[a * N + o] = m.b[a];
  }
}

constexpr int kDB = 256, kDG = 1024, kS3 = 9;  // |u|^2, |b|^2, rho, j (3), b (3)

__device__ __forceinline__ double nanmax3(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

template <bool MAX>
__device__ double block_red(double v, double *lds) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = MAX ? nanmax3(v, o) : v + o;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    r = lds[0];
    for (int w = 1; w < kDB / 64; ++w) r = MAX ? nanmax3(r, lds[w]) : r + lds[w];
  }
  return r;
}

template <class C, bool SW>
__global__ __launch_bounds__(kDB) void k_diag3_sums(Dom3 D, const typename C::T *__restrict__ src,
                                                    double *__restrict__ bpl,
                                                    double *__restrict__ part) {
  __shared__ double lds[kDB / 64];
  const int64_t N = (int64_t)D.nx * D.ny * D.nz;
  double acc[kS3] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t n = (int64_t)blockIdx.x * kDB + threadIdx.x; n < N; n += (int64_t)gridDim.x * kDB) {
    const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny),
              z = (int)(n / ((int64_t)D.nx * D.ny));
    const Mom3 m = moments3<C, SW>(D, src, x, y, z);
    acc[0] += m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
    acc[1] += m.b[0] * m.b[0] + m.b[1] * m.b[1] + m.b[2] * m.b[2];
    acc[2] += m.rho;
    for (int a = 0; a < 3; ++a) {
      acc[3 + a] += m.j[a];
      acc[6 + a] += m.b[a];
      bpl[a * N + n] = m.b[a];
    }
  }
  for (int k = 0; k < kS3; ++k) {
    const double r = block_red<false>(acc[k], lds);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kS3 + k] = r;
  }
}

// max |div b| with the isotropic gradient d_a phi = 3 sum_i w_i c_ia phi(x + c_i)
__global__ __launch_bounds__(kDB) void k_diag3_divb(Dom3 D, const double *__restrict__ bpl,
                                                    double *__restrict__ part) {
  __shared__ double lds[kDB / 64];
  const int64_t N = (int64_t)D.nx * D.ny * D.nz;
  double mx = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kDB + threadIdx.x; n < N; n += (int64_t)gridDim.x * kDB) {
    const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny),
              z = (int)(n / ((int64_t)D.nx * D.ny));
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      if (cx(i) == 0 && cy(i) == 0 && cz(i) == 0) continue;
      int xx = x + cx(i), yy = y + cy(i), zz = z + cz(i);
      xx = xx < 0 ? xx + D.nx : (xx >= D.nx ? xx - D.nx : xx);
      yy = yy < 0 ? yy + D.ny : (yy >= D.ny ? yy - D.ny : yy);
      zz = zz < 0 ? zz + D.nz : (zz >= D.nz ? zz - D.nz : zz);
      const int64_t o = ((int64_t)zz * D.ny + yy) * D.nx + xx;
      s += wgt(i) * (cx(i) * bpl[o] + cy(i) * bpl[N + o] + cz(i) * bpl[2 * N + o]);
    }
    mx = nanmax3(mx, fabs(3.0 * s));
  }
  const double r = block_red<true>(mx, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(kDB) void k_diag3_final(const double *__restrict__ ps,
                                                     const double *__restrict__ pm, int nb,
                                                     double inv_2n, double *__restrict__ out) {
  __shared__ double lds[kDB / 64];
  for (int k = 0; k < kS3; ++k) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kDB) v += ps[(int64_t)i * kS3 + k];
    const double r = block_red<false>(v, lds);
    if (threadIdx.x == 0) {
      if (k < 2) out[k] = r * inv_2n;
      else out[k + 1] = r;
    }
  }
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += kDB) m = nanmax3(m, pm[i]);
  const double r = block_red<true>(m, lds);
  if (threadIdx.x == 0) out[2] = r;
}

}  // namespace rr3

// ---- C-ABI ---------------------------------------------------------------------
struct rrmhd3d {
  rr3::Dom3 D{};
  double tau_f = 0, tau_m = 0;
  int storage = 0;
  int64_t elem = 4;
  hipStream_t stream = nullptr;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t steps = 0;
  bool ready = false;
  bool inplace = false;  // one buffer, alternating phases
  int phase = 0;         // in-place: 0 pull layout, 1 swapped layout
  bool poison = false;   // debug: NaN-fill the destination buffer before each step
  int bx = 64, by = 4;
  int xcd = 0;  // XCD-local tile order
  double *diag_work = nullptr;
  double *diag_out = nullptr;
  double *diag_host = nullptr;
};

#define HIP3(x)                                         \
  do {                                                  \
    hipError_t e_ = (x);                                \
    if (e_ != hipSuccess) return rr_device_error(e_, #x); \
  } while (0)

template <class C>
static void launch_inplace3(rrmhd3d *h, dim3 grid, dim3 block, int tiles_x) {
  auto b = (typename C::T *)h->buf[0];
  if (h->phase == 0)
    hipLaunchKernelGGL((rr3::k_step3_inplace<C, 0>), grid, block, 0, h->stream, h->D, tiles_x, h->xcd, b);
  else
    hipLaunchKernelGGL((rr3::k_step3_inplace<C, 1>), grid, block, 0, h->stream, h->D, tiles_x, h->xcd, b);
}

template <class C>
static void launch_moments3(rrmhd3d *h, bool sw, dim3 grid, dim3 block, double *rho, double *u,
                            double *b) {
  auto s = (const typename C::T *)h->buf[h->cur];
  if (sw)
    hipLaunchKernelGGL((rr3::k_moments3<C, true>), grid, block, 0, h->stream, h->D, s, rho, u, b);
  else
    hipLaunchKernelGGL((rr3::k_moments3<C, false>), grid, block, 0, h->stream, h->D, s, rho, u, b);
}

template <class C>
static void launch_diag3(rrmhd3d *h, bool sw, int nb, double *bpl, double *ps) {
  auto s = (const typename C::T *)h->buf[h->cur];
  if (sw)
    hipLaunchKernelGGL((rr3::k_diag3_sums<C, true>), dim3(nb), dim3(rr3::kDB), 0, h->stream, h->D,
                       s, bpl, ps);
  else
    hipLaunchKernelGGL((rr3::k_diag3_sums<C, false>), dim3(nb), dim3(rr3::kDB), 0, h->stream, h->D,
                       s, bpl, ps);
}

extern "C" {

int rrmhd3d_destroy(rrmhd3d *h) {
  if (!h) return RRMHD_OK;
  int rc = RRMHD_OK;
  if (h->buf[0] && hipStreamSynchronize(h->stream) != hipSuccess) rc = RRMHD_EDEVICE;
  for (void *&p : h->buf)
    if (p) (void)hipFree(p), p = nullptr;
  if (h->diag_work) (void)hipFree(h->diag_work);
  if (h->diag_out) (void)hipFree(h->diag_out);
  if (h->diag_host) (void)hipHostFree(h->diag_host);
  delete h;
  return rc;
}

int rrmhd3d_create(int32_t nx, int32_t ny, int32_t nz, int32_t storage, double tau_f,
                   double tau_m, void *hip_stream, rrmhd3d **out) {
  if (!out) return RRMHD_EINVAL;
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1) return RRMHD_EINVAL;
  if (ny > 65535 || nz > 65535) return RRMHD_EINVAL;  // grid dimensions of the launches
  const int kind = storage & 0xff, flags = storage & ~0xff;
  if (kind != RRMHD_STORE_F32 && kind != RRMHD_STORE_F16) return RRMHD_EINVAL;
  if (flags != 0 && flags != RRMHD_STORE_INPLACE) return RRMHD_EINVAL;
  if (!(std::isfinite(tau_f) && std::isfinite(tau_m)) || tau_f <= 0.5 || tau_m <= 0.5)
    return RRMHD_EINVAL;
  const int64_t elem = kind == RRMHD_STORE_F16 ? 2 : 4;
  const int64_t N = (int64_t)nx * ny * nz;
  if (N * elem >= ((int64_t)1 << 32)) return RRMHD_EINVAL;  // 32-bit in-plane byte offsets
  rrmhd3d *h = new (std::nothrow) rrmhd3d();
  if (!h) return RRMHD_ENOMEM;
  h->storage = kind;
  h->inplace = flags == RRMHD_STORE_INPLACE;
  h->elem = elem;
  h->stream = (hipStream_t)hip_stream;
  h->D.nx = nx;
  h->D.ny = ny;
  h->D.nz = nz;
  const int64_t align = 256 / elem;
  h->D.plane = (N + align - 1) / align * align + align;
  h->tau_f = tau_f;
  h->tau_m = tau_m;
  h->D.om_c = (float)(1.0 - 1.0 / tau_f);
  h->D.omm_c = (float)(1.0 - 1.0 / tau_m);
  // measured at 256^3: one row of 128 threads is the best or within 1 % of
  // it (FP16 +6 % over 64 x 4); narrow boxes stack rows to fill 128 threads
  h->bx = nx >= 128 ? 128 : ((nx + 15) / 16) * 16;
  h->by = 128 / h->bx;
  if (h->inplace && nx >= 256) {
    // the alternating single-buffer steps: one row of 256 threads measured
    // best at 256^3 (FP32 61 %, FP16 64 % of 8 TB/s against 56 %, 60 % at 128)
    h->bx = 256;
    h->by = 1;
  }
  // measured at 256^3: the XCD-local order gains about one point of 8 TB/s
  // for FP16 storage (67.6 % against 66.7 %) and for one buffer (FP32 61.5 %
  // against 60.5 %, FP16 65.2 % against 64.2 %); FP32 with two buffers is the
  // same either way and keeps the plain order
  h->xcd = (h->storage == RRMHD_STORE_F16 || h->inplace) ? 1 : 0;
  const size_t bytes = (size_t)h->D.plane * rr3::kPlanes * elem;
  int rc = RRMHD_OK;
  for (int k = 0; k < (h->inplace ? 1 : 2) && rc == RRMHD_OK; ++k)
    if (hipMalloc(&h->buf[k], bytes) != hipSuccess) rc = RRMHD_ENOMEM;
  if (rc == RRMHD_OK && hipMalloc((void **)&h->diag_out, 10 * sizeof(double)) != hipSuccess)
    rc = RRMHD_ENOMEM;
  if (rc == RRMHD_OK &&
      hipHostMalloc((void **)&h->diag_host, 10 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    rc = RRMHD_ENOMEM;
  if (rc != RRMHD_OK) {
    rrmhd3d_destroy(h);
    return rc;
  }
  *out = h;
  return RRMHD_OK;
}

int rrmhd3d_set_launch(rrmhd3d *h, int bx, int by, int xcd) {
  if (!h || bx < 1 || by < 1 || bx * by > 256 || xcd < -1 || xcd > 1) return RRMHD_EINVAL;
  h->bx = bx;
  h->by = by;
  if (xcd >= 0) h->xcd = xcd;
  return RRMHD_OK;
}

int rrmhd3d_init(rrmhd3d *h, const double *u, const double *b) {
  if (!h || !u || !b) return RRMHD_EINVAL;
  const dim3 block(64), grid((h->D.nx + 63) / 64, h->D.ny, h->D.nz);
  if (h->storage == RRMHD_STORE_F16)
    hipLaunchKernelGGL(rr3::k_init3<rr3::CodecF16U>, grid, block, 0, h->stream, h->D, u, b,
                       (uint16_t *)h->buf[0]);
  else
    hipLaunchKernelGGL(rr3::k_init3<rr3::CodecF32>, grid, block, 0, h->stream, h->D, u, b,
                       (float *)h->buf[0]);
  HIP3(hipGetLastError());
  h->cur = 0;
  h->phase = 0;
  h->steps = 0;
  h->ready = true;
  return RRMHD_OK;
}

int rrmhd3d_step(rrmhd3d *h, int64_t n) {
  if (!h || n < 0) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  const int tiles_x = (h->D.nx + h->bx - 1) / h->bx, tiles_y = (h->D.ny + h->by - 1) / h->by;
  const dim3 grid(tiles_x * tiles_y, h->D.nz), block(h->bx, h->by);
  for (int64_t k = 0; k < n && h->inplace; ++k) {
    if (h->storage == RRMHD_STORE_F16)
      launch_inplace3<rr3::CodecF16U>(h, grid, block, tiles_x);
    else
      launch_inplace3<rr3::CodecF32>(h, grid, block, tiles_x);
    HIP3(hipGetLastError());
    h->phase ^= 1;
    h->steps++;
  }
  if (h->inplace) return RRMHD_OK;
  for (int64_t k = 0; k < n; ++k) {
    const void *s = h->buf[h->cur];
    void *d = h->buf[h->cur ^ 1];
    if (h->poison) {
      const int64_t words = h->D.plane * rr3::kPlanes * h->elem / 4;
      hipLaunchKernelGGL(rr3::k_poison3, dim3(2048), dim3(256), 0, h->stream, (uint32_t *)d, words,
                         h->elem == 4 ? 0x7fc00000u : 0x7e007e00u);
    }
    if (h->storage == RRMHD_STORE_F16)
      hipLaunchKernelGGL(rr3::k_step3<rr3::CodecF16U>, grid, block, 0, h->stream, h->D, tiles_x,
                         h->xcd, (const uint16_t *)s, (uint16_t *)d);
    else
      hipLaunchKernelGGL(rr3::k_step3<rr3::CodecF32>, grid, block, 0, h->stream, h->D, tiles_x,
                         h->xcd, (const float *)s, (float *)d);
    HIP3(hipGetLastError());
    h->cur ^= 1;
    h->steps++;
  }
  return RRMHD_OK;
}

int rrmhd3d_set_debug_poison(rrmhd3d *h, int on) {
  if (!h || (on && h->inplace)) return RRMHD_EINVAL;
  h->poison = on != 0;
  return RRMHD_OK;
}

int rrmhd3d_step_count(const rrmhd3d *h, int64_t *out) {
  if (!h || !out) return RRMHD_EINVAL;
  *out = h->steps;
  return RRMHD_OK;
}

int rrmhd3d_moments(rrmhd3d *h, double *rho, double *u, double *b) {
  if (!h) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  if (!rho && !u && !b) return RRMHD_OK;
  const dim3 block(64), grid((h->D.nx + 63) / 64, h->D.ny, h->D.nz);
  const bool sw = h->inplace && h->phase;
  if (h->storage == RRMHD_STORE_F16)
    launch_moments3<rr3::CodecF16U>(h, sw, grid, block, rho, u, b);
  else
    launch_moments3<rr3::CodecF32>(h, sw, grid, block, rho, u, b);
  HIP3(hipGetLastError());
  return RRMHD_OK;
}

static int run_diag3(rrmhd3d *h) {
  const int64_t N = (int64_t)h->D.nx * h->D.ny * h->D.nz;
  if (!h->diag_work)
    HIP3(hipMalloc((void **)&h->diag_work,
                   sizeof(double) * (size_t)(3 * N + rr3::kDG * rr3::kS3 + rr3::kDG)));
  double *bpl = h->diag_work, *ps = bpl + 3 * N, *pm = ps + rr3::kDG * rr3::kS3;
  const int64_t need = (N + rr3::kDB - 1) / rr3::kDB;
  const int nb = (int)(need < rr3::kDG ? need : rr3::kDG);
  const bool sw = h->inplace && h->phase;
  if (h->storage == RRMHD_STORE_F16)
    launch_diag3<rr3::CodecF16U>(h, sw, nb, bpl, ps);
  else
    launch_diag3<rr3::CodecF32>(h, sw, nb, bpl, ps);
  hipLaunchKernelGGL(rr3::k_diag3_divb, dim3(nb), dim3(rr3::kDB), 0, h->stream, h->D, bpl, pm);
  hipLaunchKernelGGL(rr3::k_diag3_final, dim3(1), dim3(rr3::kDB), 0, h->stream, ps, pm, nb,
                     1.0 / (2.0 * (double)N), h->diag_out);
  HIP3(hipGetLastError());
  HIP3(hipMemcpyAsync(h->diag_host, h->diag_out, 10 * sizeof(double), hipMemcpyDeviceToHost,
                      h->stream));
  HIP3(hipStreamSynchronize(h->stream));
  return RRMHD_OK;
}

int rrmhd3d_diagnostics(rrmhd3d *h, double *E_kin, double *E_mag, double *max_div_b) {
  if (!h) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  int rc = run_diag3(h);
  if (rc != RRMHD_OK) return rc;
  const double *r = h->diag_host;
  const bool bad = !(std::isfinite(r[0]) && std::isfinite(r[1]) && std::isfinite(r[2]));
  const double nan = std::nan("");
  if (E_kin) *E_kin = bad ? nan : r[0];
  if (E_mag) *E_mag = bad ? nan : r[1];
  if (max_div_b) *max_div_b = bad ? nan : r[2];
  return bad ? RRMHD_ENONFINITE : RRMHD_OK;
}

int rrmhd3d_invariants(rrmhd3d *h, double out[7]) {
  if (!h || !out) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  int rc = run_diag3(h);
  if (rc != RRMHD_OK) return rc;
  for (int k = 0; k < 7; ++k) out[k] = h->diag_host[3 + k];
  return RRMHD_OK;
}

}  // extern "C"

namespace {

// Checkpoint file header of the three-dimensional handle (little-endian).
struct Ck3Header {
  char magic[8];
  int32_t version, nx, ny, nz, storage, zero;
  double tau_f, tau_m;
  int64_t steps, payload;
};
static_assert(sizeof(Ck3Header) == 64, "checkpoint header layout");
constexpr char kCk3Magic[8] = {'R', 'R', 'M', 'H', 'D', '3', 'C', '1'};

Ck3Header ck3_header(const rrmhd3d *h) {
  Ck3Header c{};
  for (int k = 0; k < 8; ++k) c.magic[k] = kCk3Magic[k];
  c.version = 1;
  c.nx = h->D.nx;
  c.ny = h->D.ny;
  c.nz = h->D.nz;
  c.storage = h->storage;
  c.tau_f = h->tau_f;
  c.tau_m = h->tau_m;
  c.steps = h->steps;
  c.payload = (int64_t)h->D.nx * h->D.ny * h->D.nz * h->elem * rr3::kPlanes;
  return c;
}

bool same_bits(double a, double b) { return __builtin_memcmp(&a, &b, sizeof a) == 0; }

}  // namespace

extern "C" {

int rrmhd3d_save(rrmhd3d *h, const char *path) {
  if (!h || !path) return RRMHD_EINVAL;
  if (!h->ready) return RRMHD_ESTATE;
  const Ck3Header hd = ck3_header(h);
  const size_t row = (size_t)h->D.nx * h->D.ny * h->D.nz * h->elem;
  void *tmp = nullptr;
  const char *base = (const char *)h->buf[h->cur];
  size_t pitch = (size_t)h->D.plane * h->elem;
  if (h->inplace && h->phase) {
    // between the two step forms: gather the swapped layout first
    HIP3(hipMalloc(&tmp, row * rr3::kPlanes));
    const dim3 grid((h->D.nx + 255) / 256, h->D.ny, h->D.nz), block(256);
    if (h->storage == RRMHD_STORE_F16)
      hipLaunchKernelGGL(rr3::k_swapped_to_pull3<uint16_t>, grid, block, 0, h->stream, h->D,
                         (const uint16_t *)h->buf[0], (uint16_t *)tmp);
    else
      hipLaunchKernelGGL(rr3::k_swapped_to_pull3<float>, grid, block, 0, h->stream, h->D,
                         (const float *)h->buf[0], (float *)tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      (void)hipFree(tmp);
      return rr_device_error(e, "k_swapped_to_pull3");
    }
    base = (const char *)tmp;
    pitch = row;
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  int rc = e != hipSuccess ? rr_device_error(e, "hipStreamSynchronize")
                           : rr_ck_write(path, &hd, sizeof hd, base, pitch, row, rr3::kPlanes);
  if (tmp) (void)hipFree(tmp);
  return rc;
}

int rrmhd3d_load(rrmhd3d *h, const char *path) {
  if (!h || !path) return RRMHD_EINVAL;
  Ck3Header hd{};
  FILE *f = nullptr;
  int rc = rr_ck_open(path, &hd, sizeof hd, &f);
  if (rc != RRMHD_OK) return rc;
  const Ck3Header me = ck3_header(h);
  if (__builtin_memcmp(hd.magic, kCk3Magic, 8) != 0 || hd.version != 1)
    rc = rr_ck_mismatch("magic/version");
  else if (hd.nx != me.nx || hd.ny != me.ny || hd.nz != me.nz) rc = rr_ck_mismatch("grid size");
  else if (hd.storage != me.storage) rc = rr_ck_mismatch("storage");
  else if (!same_bits(hd.tau_f, me.tau_f) || !same_bits(hd.tau_m, me.tau_m)) rc = rr_ck_mismatch("tau");
  else if (hd.payload != me.payload || hd.steps < 0) rc = rr_ck_mismatch("payload size / step count");
  if (rc == RRMHD_OK) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = rr_device_error(e, "hipStreamSynchronize");
  }
  bool touched = false;
  if (rc == RRMHD_OK)
    rc = rr_ck_read_planes(f, path, sizeof hd, (char *)h->buf[0], (size_t)h->D.plane * h->elem,
                           (size_t)h->D.nx * h->D.ny * h->D.nz * h->elem, rr3::kPlanes, &touched);
  fclose(f);
  if (rc != RRMHD_OK) {
    if (touched) h->ready = false;  // part of the state was overwritten
    return rc;
  }
  h->cur = 0;
  h->phase = 0;
  h->steps = hd.steps;
  h->ready = true;
  return RRMHD_OK;
}

}  // extern "C"
