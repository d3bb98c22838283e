// rr_kernels.hip -- single-domain kernels: the fused stream-and-collide step,
// equilibrium initialisation, moments and FP64 diagnostics.
//
// Layout in HBM: 19 planes per buffer (f_0..f_8, then g_0x, g_0y, ...,
// g_4x, g_4y), x fastest; element (p, y, x) at p * plane + y * row + x.
// Planes of [ny][nx] (row = nx, `plane` elements between plane starts) or
// row-interleaved (the 19 plane rows of one grid row side by side: plane =
// the row's width, row = 19 plane).  Two buffers (A/B) alternate: a step
// pulls from one and writes the other.  A stored value is the
// post-collision population of the previous step at its source node, so the
// pull f_i(x) = f*_i(x - c_i) is task 6 of the algorithm fused into the
// loads of the next step.
#include "rr_kernels.h"
#include "rr_node.h"
#include "rr_pull.h"

namespace rr {

// ---------------------------------------------------------------------------
// Pull addressing (task 6).  For a node (x, y) the population i comes from
// (x - c_ix, y - c_iy), periodic in x, periodic or walled in y.  With walls,
// a population whose source lies beyond a wall is the node's own
// post-collision population in the opposite direction (half-way
// bounce-back); for the magnetic populations the anti-bounce-back adds the
// wall term: g_j = -g*_opp(j) + 2 psi_j b_wall.
// ---------------------------------------------------------------------------
struct Rows {
  int xm, xp;                // x - 1, x + 1 (periodic)
  int64_t rm, r0, rp;        // element offsets of the rows y - 1, y, y + 1
  bool lo, hi;       // wall below (y == 0) / above (y == ny - 1)
};

template <bool WALLS>
__device__ __forceinline__ Rows rows_of(const Domain &D, int x, int y) {
  Rows R;
  R.xm = x == 0 ? D.nx - 1 : x - 1;
  R.xp = x == D.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? D.ny - 1 : y - 1;
  const int yp = y == D.ny - 1 ? 0 : y + 1;
  R.rm = (int64_t)ym * D.row;
  R.r0 = (int64_t)y * D.row;
  R.rp = (int64_t)yp * D.row;
  R.lo = WALLS && y == 0;
  R.hi = WALLS && y == D.ny - 1;
  return R;
}

// Load population i (decoded, f - w) of node x through the pull.
template <class C, bool WALLS, int I>
__device__ __forceinline__ float pull_f(const Domain &D,
                                        const typename C::T *__restrict__ s,
                                        const Rows &R, int x) {
  constexpr int CX = cx(I), CY = cy(I);
  const int sx = CX == 0 ? x : (CX > 0 ? R.xm : R.xp);
  int64_t off = (CY == 0 ? R.r0 : (CY > 0 ? R.rm : R.rp)) + sx;
  int plane = I;
  if constexpr (WALLS && CY != 0) {
    const bool wall = CY > 0 ? R.lo : R.hi;
    if (wall) {
      plane = opp_f(I);
      off = R.r0 + x;
    }
  }
  return C::dec(s[(int64_t)plane * D.plane + off], D.inv_s);
}

template <class C, bool WALLS, int J>
__device__ __forceinline__ void pull_g(const Domain &D,
                                       const typename C::T *__restrict__ s,
                                       const Rows &R, int x, float &gx,
                                       float &gy) {
  constexpr int EX = ex(J), EY = ey(J);
  const int sx = EX == 0 ? x : (EX > 0 ? R.xm : R.xp);
  int64_t off = (EY == 0 ? R.r0 : (EY > 0 ? R.rm : R.rp)) + sx;
  int j = J;
  bool wall = false;
  if constexpr (WALLS && EY != 0) {
    wall = EY > 0 ? R.lo : R.hi;
    if (wall) {
      j = opp_g(J);
      off = R.r0 + x;
    }
  }
  gx = C::dec(s[(int64_t)gplane(j, 0) * D.plane + off], D.inv_s);
  gy = C::dec(s[(int64_t)gplane(j, 1) * D.plane + off], D.inv_s);
  if constexpr (WALLS && EY != 0) {
    if (wall) {
      gx = D.bw2x - gx;
      gy = D.bw2y - gy;
    }
  }
}

template <class C, bool WALLS>
__device__ __forceinline__ void pull_node(const Domain &D,
                                          const typename C::T *__restrict__ s,
                                          int x, int y, float (&d)[kQ],
                                          float (&g)[2 * kQm]) {
  const Rows R = rows_of<WALLS>(D, x, y);
  d[0] = pull_f<C, WALLS, 0>(D, s, R, x);
  d[1] = pull_f<C, WALLS, 1>(D, s, R, x);
  d[2] = pull_f<C, WALLS, 2>(D, s, R, x);
  d[3] = pull_f<C, WALLS, 3>(D, s, R, x);
  d[4] = pull_f<C, WALLS, 4>(D, s, R, x);
  d[5] = pull_f<C, WALLS, 5>(D, s, R, x);
  d[6] = pull_f<C, WALLS, 6>(D, s, R, x);
  d[7] = pull_f<C, WALLS, 7>(D, s, R, x);
  d[8] = pull_f<C, WALLS, 8>(D, s, R, x);
  pull_g<C, WALLS, 0>(D, s, R, x, g[0], g[1]);
  pull_g<C, WALLS, 1>(D, s, R, x, g[2], g[3]);
  pull_g<C, WALLS, 2>(D, s, R, x, g[4], g[5]);
  pull_g<C, WALLS, 3>(D, s, R, x, g[6], g[7]);
  pull_g<C, WALLS, 4>(D, s, R, x, g[8], g[9]);
}

// Block order: hardware hands consecutive workgroups to the eight XCDs in
// turn.  Renumbering so that each XCD receives a contiguous run of tiles
// keeps the cache lines shared by neighbouring tiles (the +-1 pull offsets)
// inside one L2.
__device__ __forceinline__ int xcd_remap(int L, int n) {
  const int q = n >> 3, r = n & 7, k = L & 7, m = L >> 3;
  return k < r ? k * (q + 1) + m : r * (q + 1) + (k - r) * q + m;
}

// Local variant: within each run of 64 consecutive workgroups, XCD k
// (workgroups L with L % 8 == k) takes 8 neighbouring tiles, so 7 of every 8
// tile boundaries stay inside one L2 while all XCDs still sweep the same
// region of memory together.
__device__ __forceinline__ int xcd_local(int L, int n) {
  const int g = L >> 6, j = L & 63;
  if ((g + 1) * 64 > n) return L;
  return (g << 6) + ((j & 7) << 3) + (j >> 3);
}

// ---------------------------------------------------------------------------
// Fused step: pull (task 6 of the previous step), tasks 1-5, local store.
// 1-D grid of tiles; a tile is blockDim.x nodes of ry consecutive rows,
// blockDim.y tiles high.
// ---------------------------------------------------------------------------
template <class C, bool WALLS, bool FORCED, bool NT, bool NTL, bool FULLM = false,
          int RM = RM_OFFSET>
__global__ __launch_bounds__(256) void k_step(Domain D, int tiles_x, int ry,
                                              int xcd,
                                              const typename C::T *__restrict__ src,
                                              typename C::T *__restrict__ dst) {
  const int ntiles = gridDim.x;
  const int L = xcd == 1 ? xcd_remap(blockIdx.x, ntiles)
                         : (xcd == 2 ? xcd_local(blockIdx.x, ntiles) : (int)blockIdx.x);
  const int tx = L % tiles_x, ty = L / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  const int y0 = (ty * blockDim.y + threadIdx.y) * ry;
  if (x >= D.nx) return;
  CollideParams P;
  P.om_c = D.om_c;
  P.omm_c = D.omm_c;
  P.Gx = D.Gx;
  P.Gy = D.Gy;
  P.src_c = D.src_c;
  for (int r = 0; r < ry; ++r) {
    const int y = y0 + r;
    if (y >= D.ny) return;
    if constexpr (WALLS) {
      float d[kQ], g[2 * kQm];
      pull_node<C, true>(D, src, x, y, d, g);
      collide<FORCED, NoCorrection, FULLM>(d, g, P);
      const int64_t o = (int64_t)y * D.row + x;
      uint32_t seed = 0;
      if constexpr (codec_sr<C>::value)
        seed = sr_seed(D.sr_key, (uint32_t)(y * D.nx + x) * (uint32_t)sizeof(typename C::T));
      auto enc = [&](float v, int p) {
        if constexpr (codec_sr<C>::value)
          return C::enc_sr(v, D.s, sr_plane(seed, p));
        else
          return C::enc(v, D.s);
      };
#pragma unroll
      for (int i = 0; i < kQ; ++i) dst[(int64_t)i * D.plane + o] = enc(d[i], i);
#pragma unroll
      for (int k = 0; k < 2 * kQm; ++k) dst[(int64_t)(kQ + k) * D.plane + o] = enc(g[k], kQ + k);
    } else {
      const PlaneGeom G{D.plane, D.nx, D.ny, D.s, D.inv_s, D.sr_key, D.row};
      update_periodic<C, FORCED, NT, NTL, FULLM, RM>(G, src, dst, x, y, P);
    }
  }
}

// ---------------------------------------------------------------------------
// Single-buffer (in-place) step: the two phases of the alternating update
// (see rr_pull.h).  With walls, a population whose push target lies beyond
// a wall stays in the node's own slot of the same direction (the slot its
// bounce-back read came from), and the swapped read of phase 1 applies the
// magnetic anti-bounce-back to the populations that arrive through a wall.
// ---------------------------------------------------------------------------
template <class T, bool NT>
__device__ __forceinline__ void st_el(T *p, T v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <class C, bool FORCED, bool NT>
__device__ __forceinline__ void update_walled_push(const Domain &D, typename C::T *buf, int x,
                                                   int y, const CollideParams &P) {
  float d[kQ], g[2 * kQm];
  pull_node<C, true>(D, buf, x, y, d, g);
  collide<FORCED>(d, g, P);
  const Rows R = rows_of<true>(D, x, y);
  const int64_t own = R.r0 + x;
  // stochastic rounding: the bits of this node and of the population's own
  // plane, as in the two-buffer step
  uint32_t seed = 0;
  if constexpr (codec_sr<C>::value)
    seed = sr_seed(D.sr_key, (uint32_t)(y * D.nx + x) * (uint32_t)sizeof(typename C::T));
  auto enc = [&](float v, int p) {
    if constexpr (codec_sr<C>::value)
      return C::enc_sr(v, D.s, sr_plane(seed, p));
    else
      return C::enc(v, D.s);
  };
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const bool out = (cy(i) > 0 && R.hi) || (cy(i) < 0 && R.lo);
    const int tx = cx(i) == 0 ? x : (cx(i) > 0 ? R.xp : R.xm);
    const int64_t trow = cy(i) == 0 ? R.r0 : (cy(i) > 0 ? R.rp : R.rm);
    const int plane = out ? i : opp_f(i);
    const int64_t off = out ? own : trow + tx;
    st_el<typename C::T, NT>(&buf[(int64_t)plane * D.plane + off], enc(d[i], i));
  }
#pragma unroll
  for (int j = 0; j < kQm; ++j) {
    const bool out = (ey(j) > 0 && R.hi) || (ey(j) < 0 && R.lo);
    const int tx = ex(j) == 0 ? x : (ex(j) > 0 ? R.xp : R.xm);
    const int64_t trow = ey(j) == 0 ? R.r0 : (ey(j) > 0 ? R.rp : R.rm);
    const int jj = out ? j : opp_g(j);
    const int64_t off = out ? own : trow + tx;
    st_el<typename C::T, NT>(&buf[(int64_t)gplane(jj, 0) * D.plane + off],
                             enc(g[2 * j], gplane(j, 0)));
    st_el<typename C::T, NT>(&buf[(int64_t)gplane(jj, 1) * D.plane + off],
                             enc(g[2 * j + 1], gplane(j, 1)));
  }
}

// Pre-collision populations of node (x, y) from the swapped layout of phase
// 1: f_i(x) = buf[opp(i)][x]; with walls, a magnetic population arriving
// through a wall is the anti-bounce-back of the value stored there.
template <class C, bool WALLS>
__device__ __forceinline__ void own_node(const Domain &D, const typename C::T *buf, int x, int y,
                                         float (&d)[kQ], float (&g)[2 * kQm]) {
  const int64_t o = (int64_t)y * D.row + x;
#pragma unroll
  for (int i = 0; i < kQ; ++i) d[i] = C::dec(buf[(int64_t)opp_f(i) * D.plane + o], D.inv_s);
#pragma unroll
  for (int j = 0; j < kQm; ++j) {
    float gx = C::dec(buf[(int64_t)gplane(opp_g(j), 0) * D.plane + o], D.inv_s);
    float gy = C::dec(buf[(int64_t)gplane(opp_g(j), 1) * D.plane + o], D.inv_s);
    if constexpr (WALLS) {
      const bool in = (ey(j) > 0 && y == 0) || (ey(j) < 0 && y == D.ny - 1);
      if (in) {
        gx = D.bw2x - gx;
        gy = D.bw2y - gy;
      }
    }
    g[2 * j] = gx;
    g[2 * j + 1] = gy;
  }
}

template <class C, bool WALLS, bool FORCED, int PHASE, bool NT, int RM = RM_OFFSET>
__global__ __launch_bounds__(256) void k_step_inplace(Domain D, int tiles_x, int ry, int xcd,
                                                      typename C::T *buf) {
  const int ntiles = gridDim.x;
  const int L = xcd == 1 ? xcd_remap(blockIdx.x, ntiles)
                         : (xcd == 2 ? xcd_local(blockIdx.x, ntiles) : (int)blockIdx.x);
  const int tx = L % tiles_x, ty = L / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  const int y0 = (ty * blockDim.y + threadIdx.y) * ry;
  if (x >= D.nx) return;
  CollideParams P;
  P.om_c = D.om_c;
  P.omm_c = D.omm_c;
  P.Gx = D.Gx;
  P.Gy = D.Gy;
  P.src_c = D.src_c;
  const PlaneGeom G{D.plane, D.nx, D.ny, D.s, D.inv_s, D.sr_key, D.row};
  for (int r = 0; r < ry; ++r) {
    const int y = y0 + r;
    if (y >= D.ny) return;
    if constexpr (PHASE == 0) {
      if constexpr (WALLS)
        update_walled_push<C, FORCED, NT>(D, buf, x, y, P);
      else
        update_periodic_push<C, FORCED, NT, RM>(G, buf, x, y, P);
    } else {
      if constexpr (WALLS) {
        float d[kQ], g[2 * kQm];
        own_node<C, true>(D, buf, x, y, d, g);
        collide<FORCED>(d, g, P);
        const int64_t o = (int64_t)y * D.row + x;
        uint32_t seed = 0;
        if constexpr (codec_sr<C>::value)
          seed = sr_seed(D.sr_key, (uint32_t)(y * D.nx + x) * (uint32_t)sizeof(typename C::T));
        auto enc = [&](float v, int p) {
          if constexpr (codec_sr<C>::value)
            return C::enc_sr(v, D.s, sr_plane(seed, p));
          else
            return C::enc(v, D.s);
        };
#pragma unroll
        for (int i = 0; i < kQ; ++i)
          st_el<typename C::T, NT>(&buf[(int64_t)i * D.plane + o], enc(d[i], i));
#pragma unroll
        for (int k = 0; k < 2 * kQm; ++k)
          st_el<typename C::T, NT>(&buf[(int64_t)(kQ + k) * D.plane + o], enc(g[k], kQ + k));
      } else {
        update_periodic_own<C, FORCED, NT, RM>(G, buf, x, y, P);
      }
    }
  }
}

// Swapped layout -> pull layout, into a dense copy (planes of nx * ny):
// dst[i][x] = f*_i(x), found at buf[opp(i)][x + c_i], or in the node's own
// slot i when x + c_i lies beyond a wall.
template <class T>
__global__ void k_swapped_to_pull(Domain D, const T *__restrict__ buf, T *__restrict__ dst) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= D.nx) return;
  const int64_t N = (int64_t)D.nx * D.ny, o = (int64_t)y * D.nx + x;
  const int64_t ob = (int64_t)y * D.row + x;
  auto src_of = [&](int p, int op, int cxv, int cyv) -> T {
    int tx = x + cxv, ty = y + cyv;
    tx = tx < 0 ? tx + D.nx : (tx >= D.nx ? tx - D.nx : tx);
    if (D.walls && (ty < 0 || ty >= D.ny)) return buf[(int64_t)p * D.plane + ob];
    ty = ty < 0 ? ty + D.ny : (ty >= D.ny ? ty - D.ny : ty);
    return buf[(int64_t)op * D.plane + (int64_t)ty * D.row + tx];
  };
  for (int i = 0; i < kQ; ++i) dst[(int64_t)i * N + o] = src_of(i, opp_f(i), cx(i), cy(i));
  for (int j = 0; j < kQm; ++j)
    for (int c = 0; c < 2; ++c)
      dst[(int64_t)gplane(j, c) * N + o] = src_of(gplane(j, c), gplane(opp_g(j), c), ex(j), ey(j));
}

// ---------------------------------------------------------------------------
// Initialisation at equilibrium (rho = 1), written for the pull layout: the
// value stored in plane p at node n is read by node n + c_p as population p,
// or, beyond a wall, by n itself as the opposite population.  It is set so
// that the first pull yields exactly f_eq(1, u, b), g_eq(u, b) everywhere.
// FP64 arithmetic, rounded once to the storage type.
// ---------------------------------------------------------------------------
__device__ double feq_dev_d(int i, double ux, double uy, double bx, double by,
                           int full) {
  // D1Q3 factors minus one, times the weight split w_i = wx * wy
  const int cxi = cx(i), cyi = cy(i);
  const double ax = cxi == 0 ? -1.5 * ux * ux : 3.0 * cxi * ux + 3.0 * ux * ux;
  const double ay = cyi == 0 ? -1.5 * uy * uy : 3.0 * cyi * uy + 3.0 * uy * uy;
  const double c2 = (double)(cxi * cxi + cyi * cyi);
  const double cb = cxi * bx + cyi * by;
  const double q = 0.5 * (bx * bx + by * by) * c2 - cb * cb;
  const double w = (i == 0) ? 16.0 / 36.0 : ((i & 1) ? 1.0 / 36.0 : 4.0 / 36.0);
  double B = ax + ay + ax * ay + 4.5 * q;
  if (full) {
    // u.M cross terms of a0^(3), a0^(4) (Eq. eq:a0_4) with h = 3 c^2 - 1
    const double mxx = 0.5 * (by * by - bx * bx), mxy = -bx * by;
    const double hx = 3.0 * cxi * cxi - 1.0, hy = 3.0 * cyi * cyi - 1.0;
    const double m3xxy = 2.0 * ux * mxy + uy * mxx;
    const double m3xyy = -ux * mxx + 2.0 * uy * mxy;
    const double m4 = -ux * ux * mxx + uy * uy * mxx + 4.0 * ux * uy * mxy;
    B += 4.5 * (cyi * hx * m3xxy + cxi * hy * m3xyy) + 2.25 * hx * hy * m4;
  }
  return w * B;
}

__device__ void geq_d(int j, double ux, double uy, double bx, double by,
                      double &gx, double &gy) {
  const double E = ux * by - uy * bx;
  const double psi = j == 0 ? 1.0 / 3.0 : 1.0 / 6.0;
  gx = psi * (bx - 3.0 * ey(j) * E);
  gy = psi * (by + 3.0 * ex(j) * E);
}

template <class C>
__global__ void k_init(Domain D, const double *__restrict__ u,
                       const double *__restrict__ b, double bwx, double bwy,
                       typename C::T *__restrict__ dst) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= D.nx) return;
  const int64_t N = (int64_t)D.nx * D.ny;
  const int64_t o = (int64_t)y * D.row + x;  // stored state
  auto fld = [&](const double *a, int comp, int xx, int yy) {
    return a[comp * N + (int64_t)yy * D.nx + xx];
  };
  for (int i = 0; i < kQ; ++i) {
    int tx = x + cx(i), ty = y + cy(i);
    tx = tx < 0 ? tx + D.nx : (tx >= D.nx ? tx - D.nx : tx);
    double v;
    if (D.walls && (ty < 0 || ty >= D.ny)) {
      v = feq_dev_d(opp_f(i), fld(u, 0, x, y), fld(u, 1, x, y), fld(b, 0, x, y),
                    fld(b, 1, x, y), D.feq);
    } else {
      ty = ty < 0 ? ty + D.ny : (ty >= D.ny ? ty - D.ny : ty);
      v = feq_dev_d(i, fld(u, 0, tx, ty), fld(u, 1, tx, ty), fld(b, 0, tx, ty),
                    fld(b, 1, tx, ty), D.feq);
    }
    dst[(int64_t)i * D.plane + o] = C::enc((float)v, D.s);
  }
  for (int j = 0; j < kQm; ++j) {
    int tx = x + ex(j), ty = y + ey(j);
    tx = tx < 0 ? tx + D.nx : (tx >= D.nx ? tx - D.nx : tx);
    double gx, gy;
    if (D.walls && (ty < 0 || ty >= D.ny)) {
      const int o2 = opp_g(j);
      geq_d(o2, fld(u, 0, x, y), fld(u, 1, x, y), fld(b, 0, x, y),
            fld(b, 1, x, y), gx, gy);
      // stored so that -stored + 2 psi b_wall = g_eq
      gx = bwx / 3.0 - gx;
      gy = bwy / 3.0 - gy;
    } else {
      ty = ty < 0 ? ty + D.ny : (ty >= D.ny ? ty - D.ny : ty);
      geq_d(j, fld(u, 0, tx, ty), fld(u, 1, tx, ty), fld(b, 0, tx, ty),
            fld(b, 1, tx, ty), gx, gy);
    }
    dst[(int64_t)gplane(j, 0) * D.plane + o] = C::enc((float)gx, D.s);
    dst[(int64_t)gplane(j, 1) * D.plane + o] = C::enc((float)gy, D.s);
  }
}

// ---------------------------------------------------------------------------
// Moments (task 1) of the current state in FP64.
// ---------------------------------------------------------------------------
struct MomD {
  double rho, jx, jy, ux, uy, bx, by;
};

// The populations of node (x, y): pulled, or read from the node's own slots
// in the swapped layout.
template <class C, bool WALLS, bool SWAPPED>
__device__ __forceinline__ void load_node(const Domain &D, const typename C::T *__restrict__ s,
                                          int x, int y, float (&d)[kQ], float (&g)[2 * kQm]) {
  if constexpr (SWAPPED)
    own_node<C, WALLS>(D, s, x, y, d, g);
  else
    pull_node<C, WALLS>(D, s, x, y, d, g);
}

// b = sum_j g_j in FP64.
__device__ __forceinline__ double2 b_of(const float (&g)[2 * kQm]) {
  double bx = 0.0, by = 0.0;
#pragma unroll
  for (int j = 0; j < kQm; ++j) {
    bx += (double)g[2 * j];
    by += (double)g[2 * j + 1];
  }
  return make_double2(bx, by);
}

// The moments of one node's populations in FP64.
__device__ __forceinline__ MomD moments_of(const Domain &D, const float (&d)[kQ],
                                           const float (&g)[2 * kQm]) {
  MomD m;
  double dr = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    dr += (double)d[i];
    jx += (double)cx(i) * d[i];
    jy += (double)cy(i) * d[i];
  }
  m.rho = 1.0 + dr;
  m.jx = jx;
  m.jy = jy;
  m.ux = (jx + 0.5 * m.rho * (double)D.Gx) / m.rho;
  m.uy = (jy + 0.5 * m.rho * (double)D.Gy) / m.rho;
  const double2 b = b_of(g);
  m.bx = b.x;
  m.by = b.y;
  return m;
}

template <class C, bool WALLS, bool SWAPPED = false>
__device__ __forceinline__ MomD moments_d(const Domain &D,
                                          const typename C::T *__restrict__ s,
                                          int x, int y) {
  float d[kQ], g[2 * kQm];
  load_node<C, WALLS, SWAPPED>(D, s, x, y, d, g);
  return moments_of(D, d, g);
}

template <class C, bool WALLS, bool SWAPPED>
__global__ void k_moments(Domain D, const typename C::T *__restrict__ src,
                          double *__restrict__ rho, double *__restrict__ u,
                          double *__restrict__ b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= D.nx) return;
  const MomD m = moments_d<C, WALLS, SWAPPED>(D, src, x, y);
  const int64_t N = (int64_t)D.nx * D.ny, o = (int64_t)y * D.nx + x;
  if (rho) rho[o] = m.rho;
  if (u) {
    u[o] = m.ux;
    u[N + o] = m.uy;
  }
  if (b) {
    b[o] = m.bx;
    b[N + o] = m.by;
  }
}

// ---------------------------------------------------------------------------
// Diagnostics: FP64 sums with a fixed reduction tree (deterministic for a
// given grid), max |div b| with the isotropic gradient
// d_a phi = 3 sum_i w_i phi(x + c_i) c_ia.
// ---------------------------------------------------------------------------
constexpr int kDiagBlock = 256;
// persistent workgroups of the diagnostics: every one resident at once on
// MI355X (256 CUs x 3 workgroups of 4 waves at the kernel's 146-156 VGPRs)
constexpr int kDiagGrid = 768;
constexpr int kSums = 7;  // |u|^2, |b|^2, rho, j_x, j_y, b_x, b_y

__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

// Sum (or NaN-propagating max) over a 256-thread block; result in thread 0.
template <bool MAX>
__device__ double block_reduce(double v, double *lds) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = MAX ? nanmax(v, o) : v + o;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    r = lds[0];
    for (int w = 1; w < kDiagBlock / 64; ++w) r = MAX ? nanmax(r, lds[w]) : r + lds[w];
  }
  return r;
}

// The magnetic populations of node (x, y) (b = b_of(g), summed as
// moments_of sums it).
template <class C, bool WALLS, bool SWAPPED>
__device__ __forceinline__ void g_at(const Domain &D, const typename C::T *__restrict__ s, int x,
                                     int y, float (&g)[2 * kQm]) {
  if constexpr (SWAPPED) {
    float d[kQ];
    own_node<C, WALLS>(D, s, x, y, d, g);  // the fluid loads are dead code
  } else {
    const Rows R = rows_of<WALLS>(D, x, y);
    pull_g<C, WALLS, 0>(D, s, R, x, g[0], g[1]);
    pull_g<C, WALLS, 1>(D, s, R, x, g[2], g[3]);
    pull_g<C, WALLS, 2>(D, s, R, x, g[4], g[5]);
    pull_g<C, WALLS, 3>(D, s, R, x, g[6], g[7]);
    pull_g<C, WALLS, 4>(D, s, R, x, g[8], g[9]);
  }
}

// One pass over the state: per-node moments and their FP64 sums, and
// max |div b| from b staged in LDS.  Persistent workgroups of 4 waves take
// tiles of kDTX x kDTY nodes; each tile's b, plus a one-node ring around it
// (periodic wrap; zero beyond a wall, where div b is not evaluated), goes
// to LDS, so every node's populations are read once for its moments and
// only the ring's magnetic planes are read again.  Tile cells that lie past
// a ragged edge hold the b of the node they wrap to.
constexpr int kDTX = 64, kDTY = 16;
template <class C, bool WALLS, bool SWAPPED>
__global__ __launch_bounds__(kDiagBlock) void k_diag_tile(Domain D,
                                                          const typename C::T *__restrict__ src,
                                                          double *__restrict__ part_s,
                                                          double *__restrict__ part_m) {
  __shared__ double2 bt[kDTY + 2][kDTX + 2];
  __shared__ double lds[kDiagBlock / 64];
  const int tiles_x = (D.nx + kDTX - 1) / kDTX, tiles_y = (D.ny + kDTY - 1) / kDTY;
  const int ntiles = tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int kRing = 2 * (kDTX + 2) + 2 * kDTY;
  auto wrap = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };
  double acc[kSums] = {0, 0, 0, 0, 0, 0, 0};
  double mx = 0.0;
  constexpr int kWaves = kDiagBlock / 64, kRows = kDTY / kWaves;
  static_assert(kDTY % kWaves == 0 && kRing <= kDiagBlock, "one ring cell per thread");
  const TileBand B = tile_band(ntiles);  // one band of tiles per XCD
  for (int t = B.first; t < B.end; t += B.stride) {
    const int x0 = (t % tiles_x) * kDTX, y0 = (t / tiles_x) * kDTY;
    const int x = x0 + lane;
    // Every load of the tile is issued before any arithmetic: the wave's
    // rows (all populations of the real nodes, g of the cells past a ragged
    // edge), then one cell of the ring per thread (its g).
    float d[kRows][kQ], g[kRows][2 * kQm];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int y = y0 + wave + kWaves * k;
      if (x < D.nx && y < D.ny)
        load_node<C, WALLS, SWAPPED>(D, src, x, y, d[k], g[k]);
      else if (!(WALLS && y >= D.ny))
        g_at<C, WALLS, SWAPPED>(D, src, wrap(x, D.nx), wrap(y, D.ny), g[k]);
    }
    int lx = 0, ly = 0;
    bool ring_live = false;
    float gr[2 * kQm];
    if (threadIdx.x < kRing) {
      const int h = threadIdx.x;
      if (h < kDTX + 2) {
        lx = h - 1;
        ly = -1;
      } else if (h < 2 * (kDTX + 2)) {
        lx = h - (kDTX + 2) - 1;
        ly = kDTY;
      } else {
        const int k = h - 2 * (kDTX + 2);
        lx = k < kDTY ? -1 : kDTX;
        ly = k % kDTY;
      }
      const int y = y0 + ly;
      ring_live = !(WALLS && (y < 0 || y >= D.ny));
      if (ring_live) g_at<C, WALLS, SWAPPED>(D, src, wrap(x0 + lx, D.nx), wrap(y, D.ny), gr);
    }
    // tile cells: moments of the real nodes, b of every cell
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int r = wave + kWaves * k, y = y0 + r;
      double2 bv = make_double2(0.0, 0.0);
      if (x < D.nx && y < D.ny) {
        const MomD m = moments_of(D, d[k], g[k]);
        acc[0] += m.ux * m.ux + m.uy * m.uy;
        acc[1] += m.bx * m.bx + m.by * m.by;
        acc[2] += m.rho;
        acc[3] += m.jx;
        acc[4] += m.jy;
        acc[5] += m.bx;
        acc[6] += m.by;
        bv = make_double2(m.bx, m.by);
      } else if (!(WALLS && y >= D.ny)) {
        bv = b_of(g[k]);
      }
      bt[r + 1][lane + 1] = bv;
    }
    // the ring (zero beyond a wall)
    if (threadIdx.x < kRing) bt[ly + 1][lx + 1] = ring_live ? b_of(gr) : make_double2(0.0, 0.0);
    __syncthreads();
    for (int r = wave; r < kDTY; r += kWaves) {
      const int y = y0 + r;
      if (x >= D.nx || y >= D.ny) continue;
      if (WALLS && (y < 1 || y > D.ny - 2)) continue;
      double sum = 0.0;
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const double2 v = bt[r + 1 + cy(i)][lane + 1 + cx(i)];
        const double w = (i & 1) ? 1.0 / 36.0 : 1.0 / 9.0;
        sum += w * (cx(i) * v.x + cy(i) * v.y);
      }
      mx = nanmax(mx, fabs(3.0 * sum));
    }
    __syncthreads();
  }
  for (int k = 0; k < kSums; ++k) {
    const double r = block_reduce<false>(acc[k], lds);
    if (threadIdx.x == 0) part_s[(int64_t)blockIdx.x * kSums + k] = r;
  }
  const double r = block_reduce<true>(mx, lds);
  if (threadIdx.x == 0) part_m[blockIdx.x] = r;
}

__global__ __launch_bounds__(kDiagBlock) void k_diag_final(
    const double *__restrict__ part_s, int nb_s, const double *__restrict__ part_m,
    int nb_m, double inv_n2, double *__restrict__ out) {
  __shared__ double lds[kDiagBlock / 64];
  for (int k = 0; k < kSums; ++k) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb_s; i += kDiagBlock) v += part_s[(int64_t)i * kSums + k];
    const double r = block_reduce<false>(v, lds);
    if (threadIdx.x == 0) {
      if (k == 0) out[0] = r * inv_n2;
      else if (k == 1) out[1] = r * inv_n2;
      else out[k + 1] = r;
    }
  }
  double m = 0.0;
  for (int i = threadIdx.x; i < nb_m; i += kDiagBlock) m = nanmax(m, part_m[i]);
  const double r = block_reduce<true>(m, lds);
  if (threadIdx.x == 0) out[2] = r;
}

// Periodic grid with nx a multiple of K: each thread updates the nodes x ..
// x + K - 1 with one word per plane (update_periodic_multi); a workgroup of
// bx x by threads covers K bx x by ry nodes.
template <class C, int K, bool FORCED, bool NT, bool NTL, int RM>
__global__ __launch_bounds__(256) void k_step_multi(Domain D, int tiles_x, int ry, int xcd,
                                                   const typename C::T *__restrict__ src,
                                                   typename C::T *__restrict__ dst) {
  const int ntiles = gridDim.x;
  const int L = xcd == 1 ? xcd_remap(blockIdx.x, ntiles)
                         : (xcd == 2 ? xcd_local(blockIdx.x, ntiles) : (int)blockIdx.x);
  const int tx = L % tiles_x, ty = L / tiles_x;
  const int x = K * (tx * blockDim.x + threadIdx.x);
  const int y0 = (ty * blockDim.y + threadIdx.y) * ry;
  if (x >= D.nx) return;
  CollideParams P;
  P.om_c = D.om_c;
  P.omm_c = D.omm_c;
  P.Gx = D.Gx;
  P.Gy = D.Gy;
  P.src_c = D.src_c;
  const PlaneGeom G{D.plane, D.nx, D.ny, D.s, D.inv_s, D.sr_key, D.row};
  for (int r = 0; r < ry; ++r) {
    const int y = y0 + r;
    if (y >= D.ny) return;
    update_periodic_multi<C, K, FORCED, NT, NTL, RM>(G, src, dst, x, y, P);
  }
}

// Single-buffer step on a periodic grid with nx a multiple of K: each thread
// takes the nodes x .. x + K - 1 with one word per plane in either phase
// (update_periodic_push_multi / update_periodic_own_multi).
template <class C, int K, bool FORCED, int PHASE, int RM>
__global__ __launch_bounds__(256) void k_step_inplace_multi(Domain D, int tiles_x, int ry, int xcd,
                                                            typename C::T *buf) {
  const int ntiles = gridDim.x;
  const int L = xcd == 1 ? xcd_remap(blockIdx.x, ntiles)
                         : (xcd == 2 ? xcd_local(blockIdx.x, ntiles) : (int)blockIdx.x);
  const int tx = L % tiles_x, ty = L / tiles_x;
  const int x = K * (tx * blockDim.x + threadIdx.x);
  const int y0 = (ty * blockDim.y + threadIdx.y) * ry;
  if (x >= D.nx) return;
  CollideParams P;
  P.om_c = D.om_c;
  P.omm_c = D.omm_c;
  P.Gx = D.Gx;
  P.Gy = D.Gy;
  P.src_c = D.src_c;
  const PlaneGeom G{D.plane, D.nx, D.ny, D.s, D.inv_s, D.sr_key, D.row};
  for (int r = 0; r < ry; ++r) {
    const int y = y0 + r;
    if (y >= D.ny) return;
    if constexpr (PHASE == 0)
      update_periodic_push_multi<C, K, FORCED, true, RM>(G, buf, x, y, P);
    else
      update_periodic_own_multi<C, K, FORCED, true, RM>(G, buf, x, y, P);
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
LaunchShape default_shape(const Domain &D) {
  // Measured on MI355X at 8192^2.  Row-interleaved planes: FP32 storage two
  // nodes per thread (64-bit words), 128 x 2 threads; FP16 storage four nodes
  // per thread (64-bit words), 128 x 1; both with eight neighbouring tiles
  // per XCD (xcd = 2).  Planes of [ny][nx] (planes 256 B apart beyond
  // alignment): 128 x 2 for FP32; for FP16 128 x 1 threads with two nodes per
  // thread on periodic grids of even width (2-4 % faster than one node per
  // thread in the same run), else 256 x 1; plain block order.  Non-temporal
  // stores throughout.
  LaunchShape L;
  L.ry = 1;
  L.xcd = 0;
  L.nt = 1;
  const bool rows = D.row != D.nx && !D.walls && D.nx >= 512;
  if (D.sr && !D.walls && D.nx >= 512) {
    // stochastic rounding is ALU-bound (a hash per value): more nodes per
    // thread measured no faster (two 67.8 %, four 64-66 %, one 67.1 %)
    L.bx = 128;
    L.by = 1;
    L.xcd = rows ? 2 : 0;
  } else if (rows && D.elem == 2 && D.nx % 4 == 0) {
    L.bx = 128;
    L.by = 1;
    L.xcd = 2;
    L.nt = 9;
  } else if (rows && D.elem == 4 && D.nx % 2 == 0) {
    L.bx = 128;
    L.by = 2;
    L.xcd = 2;
    L.nt = 5;
  } else if (D.elem == 2 && !D.walls && D.nx % 2 == 0 && D.nx >= 512) {
    L.bx = 128;
    L.by = 1;
    L.nt = 5;
  } else if (D.nx >= 256) {
    L.bx = D.elem == 2 ? 256 : 128;
    L.by = 256 / L.bx;
  } else {
    L.bx = ((D.nx + 63) / 64) * 64;
    if (L.bx > 256) L.bx = 256;
    L.by = 256 / L.bx;
  }
  return L;
}

// Every lane of a wavefront updates the same row when the workgroup's rows
// are whole wavefronts wide or the workgroup is one row.
static bool uniform_rows(const LaunchShape &L) { return L.bx % 64 == 0 || L.by == 1; }

// Row addressing of a periodic launch: 32-bit row offsets for planes of
// [ny][nx]; row base pointers for the row-interleaved layout, scalar when
// every wavefront updates one row.
static int row_mode(const Domain &D, const LaunchShape &L) {
  if (D.row == D.nx) return RM_OFFSET;
  return uniform_rows(L) ? RM_UNIFORM : RM_LANE;
}

template <class C, bool FORCED, bool NT, bool NTL, bool FULLM>
static void launch_periodic(const Domain &D, const typename C::T *s, typename C::T *d,
                            const LaunchShape &L, dim3 grid, dim3 block, int tiles_x,
                            hipStream_t st) {
  switch (row_mode(D, L)) {
    case RM_OFFSET:
      hipLaunchKernelGGL((k_step<C, false, FORCED, NT, NTL, FULLM, RM_OFFSET>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
      break;
    case RM_UNIFORM:
      hipLaunchKernelGGL((k_step<C, false, FORCED, NT, NTL, FULLM, RM_UNIFORM>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
      break;
    default:
      hipLaunchKernelGGL((k_step<C, false, FORCED, NT, NTL, FULLM, RM_LANE>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
  }
}

template <class C, bool NT, bool NTL>
static void step_nt(const Domain &D, const void *src, void *dst, const LaunchShape &L,
                    hipStream_t st) {
  const int tiles_x = (D.nx + L.bx - 1) / L.bx;
  const int rows_per_tile = L.by * L.ry;
  const int tiles_y = (D.ny + rows_per_tile - 1) / rows_per_tile;
  const dim3 grid(tiles_x * tiles_y), block(L.bx, L.by);
  const bool forced = D.Gx != 0.0f || D.Gy != 0.0f;
  auto s = (const typename C::T *)src;
  auto d = (typename C::T *)dst;
  if (D.walls) {
    if (forced)
      hipLaunchKernelGGL((k_step<C, true, true, NT, false>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
    else
      hipLaunchKernelGGL((k_step<C, true, false, NT, false>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
  } else {
    if (forced)
      launch_periodic<C, true, NT, NTL, false>(D, s, d, L, grid, block, tiles_x, st);
    else
      launch_periodic<C, false, NT, NTL, false>(D, s, d, L, grid, block, tiles_x, st);
  }
}

// The equilibrium ablation (Domain::feq = 1): single-node update with
// non-temporal stores whatever the launch shape's flags say.
template <class C>
static void step_fullm(const Domain &D, const void *src, void *dst, const LaunchShape &L,
                       hipStream_t st) {
  const int tiles_x = (D.nx + L.bx - 1) / L.bx;
  const int rows_per_tile = L.by * L.ry;
  const int tiles_y = (D.ny + rows_per_tile - 1) / rows_per_tile;
  const dim3 grid(tiles_x * tiles_y), block(L.bx, L.by);
  const bool forced = D.Gx != 0.0f || D.Gy != 0.0f;
  auto s = (const typename C::T *)src;
  auto d = (typename C::T *)dst;
  if (D.walls) {
    if (forced)
      hipLaunchKernelGGL((k_step<C, true, true, true, false, true>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
    else
      hipLaunchKernelGGL((k_step<C, true, false, true, false, true>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
  } else {
    if (forced)
      launch_periodic<C, true, true, false, true>(D, s, d, L, grid, block, tiles_x, st);
    else
      launch_periodic<C, false, true, false, true>(D, s, d, L, grid, block, tiles_x, st);
  }
}

template <class C, int K, bool NT, bool NTL>
static void step_multi_nt(const Domain &D, const void *src, void *dst, const LaunchShape &L,
                          hipStream_t st) {
  const int tiles_x = (D.nx / K + L.bx - 1) / L.bx;
  const int rows_per_tile = L.by * L.ry;
  const int tiles_y = (D.ny + rows_per_tile - 1) / rows_per_tile;
  const dim3 grid(tiles_x * tiles_y), block(L.bx, L.by);
  auto s = (const typename C::T *)src;
  auto d = (typename C::T *)dst;
  const bool forced = D.Gx != 0.0f || D.Gy != 0.0f;
  // multi-node launches on row-interleaved planes require whole-row
  // wavefronts (multi_nodes), so the modes here are RM_OFFSET and RM_UNIFORM
  if (D.row == D.nx) {
    if (forced)
      hipLaunchKernelGGL((k_step_multi<C, K, true, NT, NTL, RM_OFFSET>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
    else
      hipLaunchKernelGGL((k_step_multi<C, K, false, NT, NTL, RM_OFFSET>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
  } else {
    if (forced)
      hipLaunchKernelGGL((k_step_multi<C, K, true, NT, NTL, RM_UNIFORM>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
    else
      hipLaunchKernelGGL((k_step_multi<C, K, false, NT, NTL, RM_UNIFORM>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, s, d);
  }
}

template <class C, int K>
static void step_multi(const Domain &D, const void *src, void *dst, const LaunchShape &L,
                       hipStream_t st) {
  const bool nts = L.nt & 1, ntl = (L.nt & 2) != 0;
  if (nts && ntl)
    step_multi_nt<C, K, true, true>(D, src, dst, L, st);
  else if (nts)
    step_multi_nt<C, K, true, false>(D, src, dst, L, st);
  else if (ntl)
    step_multi_nt<C, K, false, true>(D, src, dst, L, st);
  else
    step_multi_nt<C, K, false, false>(D, src, dst, L, st);
}

// Nodes per thread of a periodic launch (1 when no multi-node form applies).
// nt bit 2: two nodes (FP16 storage on either layout; FP32 storage on
// row-interleaved planes: on planes of [ny][nx] its 64-bit words measured
// slower than one node per thread); nt bit 3: four nodes (FP16 storage, 64-bit
// words).  nx a multiple of the count, and on row-interleaved planes
// whole-row wavefronts.
template <class C>
static int multi_nodes(const Domain &D, const LaunchShape &L) {
  if (!(L.nt & 12) || D.walls) return 1;
  const bool rows = D.row != D.nx;
  if (rows && !uniform_rows(L)) return 1;
  if (sizeof(typename C::T) == 2 && (L.nt & 8) && D.nx % 4 == 0) return 4;
  if ((L.nt & 4) && D.nx % 2 == 0 && (sizeof(typename C::T) == 2 || rows)) return 2;
  return 1;
}

template <class C>
static hipError_t step_t(const Domain &D, const void *src, void *dst,
                         const LaunchShape &L, hipStream_t st) {
  const bool nts = L.nt & 1, ntl = (L.nt & 2) != 0;
  if (D.feq) {
    step_fullm<C>(D, src, dst, L, st);
    return hipGetLastError();
  }
  {
    const int k = multi_nodes<C>(D, L);
    if (k == 2) {
      step_multi<C, 2>(D, src, dst, L, st);
      return hipGetLastError();
    }
    if constexpr (sizeof(typename C::T) == 2) {
      if (k == 4) {
        step_multi<C, 4>(D, src, dst, L, st);
        return hipGetLastError();
      }
    }
  }
  if (nts && ntl)
    step_nt<C, true, true>(D, src, dst, L, st);
  else if (nts)
    step_nt<C, true, false>(D, src, dst, L, st);
  else if (ntl)
    step_nt<C, false, true>(D, src, dst, L, st);
  else
    step_nt<C, false, false>(D, src, dst, L, st);
  return hipGetLastError();
}

hipError_t launch_step(int storage, const Domain &D, const void *src, void *dst,
                       const LaunchShape &L, hipStream_t st) {
  if (L.bx <= 0 || L.by <= 0 || L.bx * L.by > 256 || L.ry <= 0) return hipErrorInvalidValue;
  // planes of [ny][nx]: byte offsets inside one plane are 32-bit (the
  // row-interleaved layout addresses rows through 64-bit bases)
  if (D.row == D.nx && (int64_t)D.nx * D.ny * (storage == kF16 ? 2 : 4) >= ((int64_t)1 << 32))
    return hipErrorInvalidValue;
  if (storage == kF16 && D.sr) return step_t<CodecF16SR>(D, src, dst, L, st);
  if (storage == kF16)  // S = 1 (the default) needs no scaling of the stored values
    return D.s == 1.0f ? step_t<CodecF16U>(D, src, dst, L, st) : step_t<CodecF16>(D, src, dst, L, st);
  return step_t<CodecF32>(D, src, dst, L, st);
}

hipError_t launch_init(int storage, const Domain &D, const double *u,
                       const double *b, double bwx, double bwy, void *dst,
                       hipStream_t st) {
  const dim3 block(64), grid((D.nx + 63) / 64, D.ny);
  if (storage == kF16 && D.s == 1.0f)
    hipLaunchKernelGGL(k_init<CodecF16U>, grid, block, 0, st, D, u, b, bwx, bwy,
                       (uint16_t *)dst);
  else if (storage == kF16)
    hipLaunchKernelGGL(k_init<CodecF16>, grid, block, 0, st, D, u, b, bwx, bwy,
                       (uint16_t *)dst);
  else
    hipLaunchKernelGGL(k_init<CodecF32>, grid, block, 0, st, D, u, b, bwx, bwy,
                       (float *)dst);
  return hipGetLastError();
}

template <class C, bool SW>
static void moments_t(const Domain &D, const void *src, double *rho, double *u,
                      double *b, hipStream_t st) {
  const dim3 block(64), grid((D.nx + 63) / 64, D.ny);
  auto s = (const typename C::T *)src;
  if (D.walls)
    hipLaunchKernelGGL((k_moments<C, true, SW>), grid, block, 0, st, D, s, rho, u, b);
  else
    hipLaunchKernelGGL((k_moments<C, false, SW>), grid, block, 0, st, D, s, rho, u, b);
}

hipError_t launch_moments(int storage, const Domain &D, const void *src,
                          double *rho, double *u, double *b, hipStream_t st, int swapped) {
  if (storage == kF16)
    swapped ? moments_t<CodecF16, true>(D, src, rho, u, b, st)
            : moments_t<CodecF16, false>(D, src, rho, u, b, st);
  else
    swapped ? moments_t<CodecF32, true>(D, src, rho, u, b, st)
            : moments_t<CodecF32, false>(D, src, rho, u, b, st);
  return hipGetLastError();
}

template <class C, bool FORCED, int PHASE, bool NT>
static void inplace_periodic(const Domain &D, typename C::T *b, const LaunchShape &L, dim3 grid,
                             dim3 block, int tiles_x, hipStream_t st) {
  switch (row_mode(D, L)) {
    case RM_OFFSET:
      hipLaunchKernelGGL((k_step_inplace<C, false, FORCED, PHASE, NT, RM_OFFSET>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
      break;
    case RM_UNIFORM:
      hipLaunchKernelGGL((k_step_inplace<C, false, FORCED, PHASE, NT, RM_UNIFORM>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
      break;
    default:
      hipLaunchKernelGGL((k_step_inplace<C, false, FORCED, PHASE, NT, RM_LANE>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
  }
}

template <class C, int PHASE, bool NT>
static void inplace_t(const Domain &D, void *buf, const LaunchShape &L, hipStream_t st) {
  const int tiles_x = (D.nx + L.bx - 1) / L.bx;
  const int rows_per_tile = L.by * L.ry;
  const int tiles_y = (D.ny + rows_per_tile - 1) / rows_per_tile;
  const dim3 grid(tiles_x * tiles_y), block(L.bx, L.by);
  const bool forced = D.Gx != 0.0f || D.Gy != 0.0f;
  auto b = (typename C::T *)buf;
  if (D.walls) {
    if (forced)
      hipLaunchKernelGGL((k_step_inplace<C, true, true, PHASE, NT>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
    else
      hipLaunchKernelGGL((k_step_inplace<C, true, false, PHASE, NT>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
  } else {
    if (forced)
      inplace_periodic<C, true, PHASE, NT>(D, b, L, grid, block, tiles_x, st);
    else
      inplace_periodic<C, false, PHASE, NT>(D, b, L, grid, block, tiles_x, st);
  }
}

// K nodes per thread, non-temporal stores; as for the two-buffer multi-node
// update, row-interleaved planes come with whole-row wavefronts (RM_UNIFORM).
template <class C, int K, int PHASE>
static void inplace_multi_t(const Domain &D, void *buf, const LaunchShape &L, hipStream_t st) {
  const int tiles_x = (D.nx / K + L.bx - 1) / L.bx;
  const int rows_per_tile = L.by * L.ry;
  const int tiles_y = (D.ny + rows_per_tile - 1) / rows_per_tile;
  const dim3 grid(tiles_x * tiles_y), block(L.bx, L.by);
  const bool forced = D.Gx != 0.0f || D.Gy != 0.0f;
  auto b = (typename C::T *)buf;
  if (D.row == D.nx) {
    if (forced)
      hipLaunchKernelGGL((k_step_inplace_multi<C, K, true, PHASE, RM_OFFSET>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
    else
      hipLaunchKernelGGL((k_step_inplace_multi<C, K, false, PHASE, RM_OFFSET>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
  } else {
    if (forced)
      hipLaunchKernelGGL((k_step_inplace_multi<C, K, true, PHASE, RM_UNIFORM>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
    else
      hipLaunchKernelGGL((k_step_inplace_multi<C, K, false, PHASE, RM_UNIFORM>), grid, block, 0, st, D, tiles_x, L.ry, L.xcd, b);
  }
}

// The multi-node forms take the nodes-per-thread rule of the two-buffer
// step (multi_nodes) and need non-temporal stores (nt bit 0).
template <class C>
static void inplace_phase(const Domain &D, void *buf, int phase, const LaunchShape &L,
                          hipStream_t st) {
  const bool nt = L.nt & 1;
  {
    const int k = nt ? multi_nodes<C>(D, L) : 1;
    if (k == 2) {
      phase ? inplace_multi_t<C, 2, 1>(D, buf, L, st) : inplace_multi_t<C, 2, 0>(D, buf, L, st);
      return;
    }
    if constexpr (sizeof(typename C::T) == 2) {
      if (k == 4) {
        phase ? inplace_multi_t<C, 4, 1>(D, buf, L, st) : inplace_multi_t<C, 4, 0>(D, buf, L, st);
        return;
      }
    }
  }
  if (phase)
    nt ? inplace_t<C, 1, true>(D, buf, L, st) : inplace_t<C, 1, false>(D, buf, L, st);
  else
    nt ? inplace_t<C, 0, true>(D, buf, L, st) : inplace_t<C, 0, false>(D, buf, L, st);
}

hipError_t launch_step_inplace(int storage, const Domain &D, void *buf, int phase,
                               const LaunchShape &L, hipStream_t st) {
  if (L.bx <= 0 || L.by <= 0 || L.bx * L.by > 256 || L.ry <= 0) return hipErrorInvalidValue;
  // as for the two-buffer step: 32-bit offsets inside planes of [ny][nx]
  if (D.row == D.nx && (int64_t)D.nx * D.ny * (storage == kF16 ? 2 : 4) >= ((int64_t)1 << 32))
    return hipErrorInvalidValue;
  if (storage == kF16 && D.sr)
    inplace_phase<CodecF16SR>(D, buf, phase, L, st);
  else if (storage == kF16)
    D.s == 1.0f ? inplace_phase<CodecF16U>(D, buf, phase, L, st)
                : inplace_phase<CodecF16>(D, buf, phase, L, st);
  else
    inplace_phase<CodecF32>(D, buf, phase, L, st);
  return hipGetLastError();
}

hipError_t launch_swapped_to_pull(int storage, const Domain &D, const void *buf, void *dst,
                                  hipStream_t st) {
  const dim3 block(64), grid((D.nx + 63) / 64, D.ny);
  if (storage == kF16)
    hipLaunchKernelGGL(k_swapped_to_pull<uint16_t>, grid, block, 0, st, D,
                       (const uint16_t *)buf, (uint16_t *)dst);
  else
    hipLaunchKernelGGL(k_swapped_to_pull<float>, grid, block, 0, st, D, (const float *)buf,
                       (float *)dst);
  return hipGetLastError();
}

// Workgroups of a diagnostics launch: a fixed count, so the order of the
// FP64 sums depends on the grid size only (not on a kernel's register
// allocation); at most one per tile.
static int diag_grid(const Domain &D) {
  const int64_t tiles = (int64_t)((D.nx + kDTX - 1) / kDTX) * ((D.ny + kDTY - 1) / kDTY);
  return (int)(tiles < kDiagGrid ? tiles : kDiagGrid);
}

size_t diag_work_bytes(const Domain &) {
  return sizeof(double) * (size_t)(kDiagGrid * kSums + kDiagGrid);
}

template <class C, bool SW>
static int diag_t(const Domain &D, const void *src, double *ps, double *pm, hipStream_t st) {
  auto s = (const typename C::T *)src;
  const int nb = diag_grid(D);
  if (D.walls)
    hipLaunchKernelGGL((k_diag_tile<C, true, SW>), dim3(nb), dim3(kDiagBlock), 0, st, D, s, ps, pm);
  else
    hipLaunchKernelGGL((k_diag_tile<C, false, SW>), dim3(nb), dim3(kDiagBlock), 0, st, D, s, ps, pm);
  return nb;
}

hipError_t launch_diagnostics(int storage, const Domain &D, const void *src,
                              void *work, double *out_dev, hipStream_t st, int swapped) {
  const int64_t N = (int64_t)D.nx * D.ny;
  double *ps = (double *)work;
  double *pm = ps + kDiagGrid * kSums;
  int nb;
  if (storage == kF16)
    nb = swapped ? diag_t<CodecF16, true>(D, src, ps, pm, st)
                 : diag_t<CodecF16, false>(D, src, ps, pm, st);
  else
    nb = swapped ? diag_t<CodecF32, true>(D, src, ps, pm, st)
                 : diag_t<CodecF32, false>(D, src, ps, pm, st);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagBlock), 0, st, ps, nb, pm, nb,
                     1.0 / (2.0 * (double)N), out_dev);
  return hipGetLastError();
}

}  // namespace rr
