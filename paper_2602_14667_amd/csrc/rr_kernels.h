// rr_kernels.h -- launch interfaces of the single-domain kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {

enum Storage { kF32 = 0, kF16 = 1 };
constexpr int kStatePlanes = 19;  // 9 fluid + 5 x 2 magnetic planes

// Geometry and physics of one domain, as the kernels see it.
struct Domain {
  int nx, ny;
  int64_t plane;  // elements between consecutive planes of one buffer (of one row)
  int64_t row;    // elements between consecutive rows of one plane: nx for
                  // planes of [ny][nx]; kStatePlanes * plane for the
                  // row-interleaved layout, [ny][plane][x]
  int walls;      // 0 periodic, 1 walls in y
  float om_c, omm_c, src_c;
  float Gx, Gy;
  float bw2x, bw2y;  // 2 psi_j b_wall for j = 1..4 (psi = 1/6): b_wall / 3
  float s, inv_s;    // storage scale (F16)
  int elem;          // bytes per stored value (4 or 2)
  int feq;           // 0: the algorithm's equilibrium; 1: with the u.M
                     // cross terms of the third and fourth orders (ablation)
  int sr = 0;             // FP16 storage written with stochastic rounding
  uint32_t sr_key = 0;    // its per-step key (set before each step)
};

struct LaunchShape {
  int bx, by;  // threads per block in x and y
  int ry;      // rows per thread (block covers by * ry rows)
  int xcd;     // 1: XCD-aware block order
  int nt;      // bit 0: non-temporal stores, bit 1: non-temporal loads,
               // bit 2: two nodes per thread, bit 3: four (periodic grids;
               // see multi_nodes)
};

hipError_t launch_step(int storage, const Domain &D, const void *src, void *dst,
                       const LaunchShape &L, hipStream_t st);
hipError_t launch_init(int storage, const Domain &D, const double *u,
                       const double *b, double bwx, double bwy, void *dst,
                       hipStream_t st);
// swapped = 1 reads the layout a single-buffer handle holds after an odd
// number of its steps (f_i(x) in slot opp(i) of x itself).
hipError_t launch_moments(int storage, const Domain &D, const void *src,
                          double *rho, double *u, double *b, hipStream_t st,
                          int swapped = 0);
// Diagnostics: out_dev[8] = {E_kin, E_mag, max|div b|, mass, j_x, j_y, b_x,
// b_y}.  work must hold diag_work_bytes(D) bytes.
size_t diag_work_bytes(const Domain &D);
hipError_t launch_diagnostics(int storage, const Domain &D, const void *src,
                              void *work, double *out_dev, hipStream_t st, int swapped = 0);

// Single-buffer streaming: one step of the given phase (0: pull read, push
// into the opposite slots; 1: read own swapped slots, store locally) on buf.
hipError_t launch_step_inplace(int storage, const Domain &D, void *buf, int phase,
                               const LaunchShape &L, hipStream_t st);
// The swapped layout of buf rewritten in the pull layout into dst (dense
// planes of nx * ny elements).
hipError_t launch_swapped_to_pull(int storage, const Domain &D, const void *buf, void *dst,
                                  hipStream_t st);

LaunchShape default_shape(const Domain &D);

}  // namespace rr
