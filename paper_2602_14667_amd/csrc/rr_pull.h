// rr_pull.h -- the periodic node update shared by the single-domain and the
// batched kernels: pull the 19 populations of node (x, y) from their
// upstream neighbours (streaming, algorithm task 6), collide (tasks 1-5) and
// store the post-collision values at (x, y).  Every plane base is
// wave-uniform (scalar registers) and the in-plane position is a 32-bit byte
// offset, so each access is one global load/store with a scalar base.
#pragma once
#include <utility>

#include "rr_node.h"

namespace rr {

struct PlaneGeom {
  int64_t plane;  // elements between plane starts
  int nx, ny;
  float s, inv_s;  // storage scale
  uint32_t sr_key = 0;  // per-step key of the stochastic-rounding codec
};

template <class T>
__device__ __forceinline__ const T *plane_ptr(const T *__restrict__ s, int p,
                                              int64_t plane) {
  return s + (int64_t)p * plane;
}

template <class T, bool NT = false>
__device__ __forceinline__ T ld_at(const T *__restrict__ base, uint32_t byte_off) {
  const T *p = (const T *)((const char *)base + byte_off);
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <class T, bool NT>
__device__ __forceinline__ void st_at(T *__restrict__ base, uint32_t byte_off, T v) {
  T *p = (T *)((char *)base + byte_off);
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Population I of node (x, y) comes from (x - c_Ix, y - c_Iy).
template <class C, int I, bool NTL>
__device__ __forceinline__ float pull_f_per(const PlaneGeom &G,
                                            const typename C::T *__restrict__ s,
                                            uint32_t bm, uint32_t b0, uint32_t bp,
                                            uint32_t xm, uint32_t x0, uint32_t xp) {
  constexpr int CX = cx(I), CY = cy(I);
  const uint32_t row = CY == 0 ? b0 : (CY > 0 ? bm : bp);
  const uint32_t col = CX == 0 ? x0 : (CX > 0 ? xm : xp);
  return C::dec(ld_at<typename C::T, NTL>(plane_ptr(s, I, G.plane), row + col), G.inv_s);
}

template <class C, int J, int COMP, bool NTL>
__device__ __forceinline__ float pull_g_per(const PlaneGeom &G,
                                            const typename C::T *__restrict__ s,
                                            uint32_t bm, uint32_t b0, uint32_t bp,
                                            uint32_t xm, uint32_t x0, uint32_t xp) {
  constexpr int EX = ex(J), EY = ey(J);
  const uint32_t row = EY == 0 ? b0 : (EY > 0 ? bm : bp);
  const uint32_t col = EX == 0 ? x0 : (EX > 0 ? xm : xp);
  return C::dec(ld_at<typename C::T, NTL>(plane_ptr(s, gplane(J, COMP), G.plane), row + col),
                G.inv_s);
}

// Store the post-collision populations of one node at byte offset o of
// every plane.  Written plane by plane (not as a loop over a running
// pointer) so each store keeps a scalar plane base and the 32-bit offset.
template <class C, bool NT, int P>
__device__ __forceinline__ void store_plane(const PlaneGeom &G, typename C::T *__restrict__ dst,
                                            uint32_t o, uint32_t seed, const float *d,
                                            const float *g) {
  const float v = P < kQ ? d[P] : g[P - kQ];
  if constexpr (codec_sr<C>::value)
    st_at<typename C::T, NT>(dst + (int64_t)P * G.plane, o, C::enc_sr(v, G.s, sr_plane(seed, P)));
  else
    st_at<typename C::T, NT>(dst + (int64_t)P * G.plane, o, C::enc(v, G.s));
}
template <class C, bool NT, int... P>
__device__ __forceinline__ void store_planes_seq(const PlaneGeom &G,
                                                 typename C::T *__restrict__ dst, uint32_t o,
                                                 uint32_t seed, const float *d, const float *g,
                                                 std::integer_sequence<int, P...>) {
  (store_plane<C, NT, P>(G, dst, o, seed, d, g), ...);
}
template <class C, bool NT>
__device__ __forceinline__ void store_planes(const PlaneGeom &G, typename C::T *__restrict__ dst,
                                             uint32_t o, const float *d, const float *g) {
  uint32_t seed = 0;
  if constexpr (codec_sr<C>::value) seed = sr_seed(G.sr_key, o);
  store_planes_seq<C, NT>(G, dst, o, seed, d, g, std::make_integer_sequence<int, kPlanes>{});
}

// Pull, collide and store one node of a doubly periodic domain.  src/dst
// point at plane 0 of the domain's two buffers.
template <class C, bool FORCED, bool NT, bool NTL, bool FULLM = false>
__device__ __forceinline__ void update_periodic(const PlaneGeom &G,
                                                const typename C::T *__restrict__ src,
                                                typename C::T *__restrict__ dst, int x,
                                                int y, const CollideParams &P) {
  using T = typename C::T;
  constexpr uint32_t E = sizeof(T);
  const uint32_t pitch = G.nx * E;
  const uint32_t x0 = x * E;
  const uint32_t xm = (x == 0 ? G.nx - 1 : x - 1) * E;
  const uint32_t xp = (x == G.nx - 1 ? 0 : x + 1) * E;
  const uint32_t b0 = y * pitch;
  const uint32_t bm = (y == 0 ? G.ny - 1 : y - 1) * pitch;
  const uint32_t bp = (y == G.ny - 1 ? 0 : y + 1) * pitch;
  float d[kQ], g[2 * kQm];
  d[0] = pull_f_per<C, 0, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[1] = pull_f_per<C, 1, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[2] = pull_f_per<C, 2, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[3] = pull_f_per<C, 3, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[4] = pull_f_per<C, 4, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[5] = pull_f_per<C, 5, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[6] = pull_f_per<C, 6, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[7] = pull_f_per<C, 7, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  d[8] = pull_f_per<C, 8, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[0] = pull_g_per<C, 0, 0, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[1] = pull_g_per<C, 0, 1, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[2] = pull_g_per<C, 1, 0, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[3] = pull_g_per<C, 1, 1, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[4] = pull_g_per<C, 2, 0, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[5] = pull_g_per<C, 2, 1, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[6] = pull_g_per<C, 3, 0, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[7] = pull_g_per<C, 3, 1, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[8] = pull_g_per<C, 4, 0, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  g[9] = pull_g_per<C, 4, 1, NTL>(G, src, bm, b0, bp, xm, x0, xp);
  collide<FORCED, NoCorrection, FULLM>(d, g, P);
  store_planes<C, NT>(G, dst, b0 + x0, d, g);
}

// ---- single-buffer (in-place) streaming --------------------------------------
// One buffer instead of two.  Steps alternate between two forms, each of
// which writes only the locations its own thread has just read, so one
// buffer suffices without races:
//  * phase 0 (buffer in the pull layout, stored value of plane i at node y is
//    f*_i(y)): pull f_i(x) = buf[i][x - c_i] as the two-buffer step does,
//    collide, and write f*_i(x) into the slot just read for the opposite
//    direction, buf[opp(i)][x + c_i];
//  * phase 1 (swapped layout, buf[opp(i)][x] = f_i(x), the pre-collision
//    population of x itself): read the node's own slots, collide, and store
//    f*_i(x) at buf[i][x], which restores the pull layout.
// The arithmetic per node is the two-buffer step's, so both give the same
// bits.  buf points at plane 0 and is read and written through one pointer.
template <class C, int P, bool NT>
__device__ __forceinline__ void store_plane_at(const PlaneGeom &G, typename C::T *buf,
                                               uint32_t o, float v, uint32_t seed, int src_plane) {
  // stochastic rounding draws the bits of the computing node and of the
  // population's own plane, whichever slot receives it, so the result is
  // the two-buffer step's bit for bit
  if constexpr (codec_sr<C>::value)
    st_at<typename C::T, NT>(buf + (int64_t)P * G.plane, o,
                             C::enc_sr(v, G.s, sr_plane(seed, src_plane)));
  else
    st_at<typename C::T, NT>(buf + (int64_t)P * G.plane, o, C::enc(v, G.s));
}

template <class C, bool FORCED, bool NT>
__device__ __forceinline__ void update_periodic_push(const PlaneGeom &G, typename C::T *buf,
                                                     int x, int y, const CollideParams &P) {
  using T = typename C::T;
  constexpr uint32_t E = sizeof(T);
  const uint32_t pitch = G.nx * E;
  const uint32_t x0 = x * E;
  const uint32_t xm = (x == 0 ? G.nx - 1 : x - 1) * E;
  const uint32_t xp = (x == G.nx - 1 ? 0 : x + 1) * E;
  const uint32_t b0 = y * pitch;
  const uint32_t bm = (y == 0 ? G.ny - 1 : y - 1) * pitch;
  const uint32_t bp = (y == G.ny - 1 ? 0 : y + 1) * pitch;
  const T *src = buf;
  float d[kQ], g[2 * kQm];
  d[0] = pull_f_per<C, 0, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[1] = pull_f_per<C, 1, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[2] = pull_f_per<C, 2, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[3] = pull_f_per<C, 3, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[4] = pull_f_per<C, 4, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[5] = pull_f_per<C, 5, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[6] = pull_f_per<C, 6, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[7] = pull_f_per<C, 7, false>(G, src, bm, b0, bp, xm, x0, xp);
  d[8] = pull_f_per<C, 8, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[0] = pull_g_per<C, 0, 0, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[1] = pull_g_per<C, 0, 1, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[2] = pull_g_per<C, 1, 0, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[3] = pull_g_per<C, 1, 1, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[4] = pull_g_per<C, 2, 0, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[5] = pull_g_per<C, 2, 1, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[6] = pull_g_per<C, 3, 0, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[7] = pull_g_per<C, 3, 1, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[8] = pull_g_per<C, 4, 0, false>(G, src, bm, b0, bp, xm, x0, xp);
  g[9] = pull_g_per<C, 4, 1, false>(G, src, bm, b0, bp, xm, x0, xp);
  collide<FORCED>(d, g, P);
  // f*_i(x) -> buf[opp(i)][x + c_i]: the slot read for direction opp(i)
  auto at = [&](int cxv, int cyv) {
    return (cyv == 0 ? b0 : (cyv > 0 ? bp : bm)) + (cxv == 0 ? x0 : (cxv > 0 ? xp : xm));
  };
  uint32_t seed = 0;
  if constexpr (codec_sr<C>::value) seed = sr_seed(G.sr_key, b0 + x0);
  store_plane_at<C, opp_f(0), NT>(G, buf, at(cx(0), cy(0)), d[0], seed, 0);
  store_plane_at<C, opp_f(1), NT>(G, buf, at(cx(1), cy(1)), d[1], seed, 1);
  store_plane_at<C, opp_f(2), NT>(G, buf, at(cx(2), cy(2)), d[2], seed, 2);
  store_plane_at<C, opp_f(3), NT>(G, buf, at(cx(3), cy(3)), d[3], seed, 3);
  store_plane_at<C, opp_f(4), NT>(G, buf, at(cx(4), cy(4)), d[4], seed, 4);
  store_plane_at<C, opp_f(5), NT>(G, buf, at(cx(5), cy(5)), d[5], seed, 5);
  store_plane_at<C, opp_f(6), NT>(G, buf, at(cx(6), cy(6)), d[6], seed, 6);
  store_plane_at<C, opp_f(7), NT>(G, buf, at(cx(7), cy(7)), d[7], seed, 7);
  store_plane_at<C, opp_f(8), NT>(G, buf, at(cx(8), cy(8)), d[8], seed, 8);
  store_plane_at<C, gplane(opp_g(0), 0), NT>(G, buf, at(ex(0), ey(0)), g[0], seed,
                                             gplane(0, 0));
  store_plane_at<C, gplane(opp_g(0), 1), NT>(G, buf, at(ex(0), ey(0)), g[1], seed,
                                             gplane(0, 1));
  store_plane_at<C, gplane(opp_g(1), 0), NT>(G, buf, at(ex(1), ey(1)), g[2], seed,
                                             gplane(1, 0));
  store_plane_at<C, gplane(opp_g(1), 1), NT>(G, buf, at(ex(1), ey(1)), g[3], seed,
                                             gplane(1, 1));
  store_plane_at<C, gplane(opp_g(2), 0), NT>(G, buf, at(ex(2), ey(2)), g[4], seed,
                                             gplane(2, 0));
  store_plane_at<C, gplane(opp_g(2), 1), NT>(G, buf, at(ex(2), ey(2)), g[5], seed,
                                             gplane(2, 1));
  store_plane_at<C, gplane(opp_g(3), 0), NT>(G, buf, at(ex(3), ey(3)), g[6], seed,
                                             gplane(3, 0));
  store_plane_at<C, gplane(opp_g(3), 1), NT>(G, buf, at(ex(3), ey(3)), g[7], seed,
                                             gplane(3, 1));
  store_plane_at<C, gplane(opp_g(4), 0), NT>(G, buf, at(ex(4), ey(4)), g[8], seed,
                                             gplane(4, 0));
  store_plane_at<C, gplane(opp_g(4), 1), NT>(G, buf, at(ex(4), ey(4)), g[9], seed,
                                             gplane(4, 1));
}

template <class C, int P>
__device__ __forceinline__ float ld_own(const PlaneGeom &G, const typename C::T *buf,
                                        uint32_t o) {
  return C::dec(ld_at<typename C::T, false>(plane_ptr(buf, P, G.plane), o), G.inv_s);
}

template <class C, bool FORCED, bool NT>
__device__ __forceinline__ void update_periodic_own(const PlaneGeom &G, typename C::T *buf,
                                                    int x, int y, const CollideParams &P) {
  constexpr uint32_t E = sizeof(typename C::T);
  const uint32_t o = y * (G.nx * E) + x * E;
  const typename C::T *src = buf;
  float d[kQ], g[2 * kQm];
  d[0] = ld_own<C, opp_f(0)>(G, src, o);
  d[1] = ld_own<C, opp_f(1)>(G, src, o);
  d[2] = ld_own<C, opp_f(2)>(G, src, o);
  d[3] = ld_own<C, opp_f(3)>(G, src, o);
  d[4] = ld_own<C, opp_f(4)>(G, src, o);
  d[5] = ld_own<C, opp_f(5)>(G, src, o);
  d[6] = ld_own<C, opp_f(6)>(G, src, o);
  d[7] = ld_own<C, opp_f(7)>(G, src, o);
  d[8] = ld_own<C, opp_f(8)>(G, src, o);
  g[0] = ld_own<C, gplane(opp_g(0), 0)>(G, src, o);
  g[1] = ld_own<C, gplane(opp_g(0), 1)>(G, src, o);
  g[2] = ld_own<C, gplane(opp_g(1), 0)>(G, src, o);
  g[3] = ld_own<C, gplane(opp_g(1), 1)>(G, src, o);
  g[4] = ld_own<C, gplane(opp_g(2), 0)>(G, src, o);
  g[5] = ld_own<C, gplane(opp_g(2), 1)>(G, src, o);
  g[6] = ld_own<C, gplane(opp_g(3), 0)>(G, src, o);
  g[7] = ld_own<C, gplane(opp_g(3), 1)>(G, src, o);
  g[8] = ld_own<C, gplane(opp_g(4), 0)>(G, src, o);
  g[9] = ld_own<C, gplane(opp_g(4), 1)>(G, src, o);
  collide<FORCED>(d, g, P);
  store_planes<C, NT>(G, buf, o, d, g);
}

// ---- 16-bit storage, two neighbouring nodes per thread -----------------------
// Nodes (x, x + 1), x even, nx even: every plane moves as one 32-bit word per
// thread (low half node x, high half node x + 1), which halves the memory
// instructions per byte of the 2-byte codec.  The planes shifted by +-1 in x
// read the word at an odd 16-bit position (gfx950 loads unaligned global
// words natively); at the periodic seam (x = 0 for c_x = +1, x = nx - 2 for
// c_x = -1) the two halves come from opposite ends of the row and are read
// separately.
template <int CX, bool NTL>
__device__ __forceinline__ uint32_t ld_pair(const uint16_t *__restrict__ plane, uint32_t row,
                                            int x, int nx) {
  if (CX == 0) return ld_at<uint32_t, NTL>((const uint32_t *)plane, row + 2u * x);
  // first source node, kept inside the row so the word is always in bounds
  const int xs = CX > 0 ? (x > 0 ? x - 1 : 0) : (x + 1 < nx - 1 ? x + 1 : nx - 2);
  uint32_t w = ld_at<uint32_t, NTL>((const uint32_t *)plane, row + 2u * xs);
  if (CX > 0 ? x == 0 : x == nx - 2) {
    // the pair straddles the seam: (nx - 1, 0) in both cases
    const uint32_t lo = ld_at<uint16_t, NTL>(plane, row + 2u * (nx - 1));
    const uint32_t hi = ld_at<uint16_t, NTL>(plane, row);
    w = lo | (hi << 16);
  }
  return w;
}

// Store plane P's word: node x's value (the low half already encoded in
// lo[P]) and node x + 1's from its post-collision arrays.
template <class C, bool NT, int P>
__device__ __forceinline__ void store_pair_plane(const PlaneGeom &G, uint16_t *__restrict__ dst,
                                                 uint32_t o, const uint16_t *lo, const float *d,
                                                 const float *g) {
  const float v = P < kQ ? d[P] : g[P - kQ];
  st_at<uint32_t, NT>((uint32_t *)(dst + (int64_t)P * G.plane), o,
                      (uint32_t)lo[P] | ((uint32_t)C::enc(v, G.s) << 16));
}
template <class C, bool NT, int... P>
__device__ __forceinline__ void store_pair_planes(const PlaneGeom &G, uint16_t *__restrict__ dst,
                                                  uint32_t o, const uint16_t *lo, const float *d,
                                                  const float *g,
                                                  std::integer_sequence<int, P...>) {
  (store_pair_plane<C, NT, P>(G, dst, o, lo, d, g), ...);
}

// C: a 16-bit codec (CodecF16 or CodecF16U).
template <class C, bool FORCED, bool NT, bool NTL>
__device__ __forceinline__ void update_periodic_pair(const PlaneGeom &G,
                                                     const uint16_t *__restrict__ src,
                                                     uint16_t *__restrict__ dst, int x, int y,
                                                     const CollideParams &P) {
  const uint32_t pitch = G.nx * 2u;
  const uint32_t b0 = y * pitch;
  const uint32_t bm = (y == 0 ? G.ny - 1 : y - 1) * pitch;
  const uint32_t bp = (y == G.ny - 1 ? 0 : y + 1) * pitch;
  uint32_t w[kPlanes];
  auto rowf = [&](int cyv) { return cyv == 0 ? b0 : (cyv > 0 ? bm : bp); };
#define RR_LDF(I) w[I] = ld_pair<cx(I), NTL>(plane_ptr(src, I, G.plane), rowf(cy(I)), x, G.nx)
#define RR_LDG(J, K) \
  w[gplane(J, K)] = ld_pair<ex(J), NTL>(plane_ptr(src, gplane(J, K), G.plane), rowf(ey(J)), x, G.nx)
  RR_LDF(0); RR_LDF(1); RR_LDF(2); RR_LDF(3); RR_LDF(4); RR_LDF(5); RR_LDF(6); RR_LDF(7); RR_LDF(8);
  RR_LDG(0, 0); RR_LDG(0, 1); RR_LDG(1, 0); RR_LDG(1, 1); RR_LDG(2, 0); RR_LDG(2, 1);
  RR_LDG(3, 0); RR_LDG(3, 1); RR_LDG(4, 0); RR_LDG(4, 1);
#undef RR_LDF
#undef RR_LDG
  // node x (low halves), then node x + 1 (high halves)
  float d[kQ], g[2 * kQm];
  uint16_t lo[kPlanes];
#pragma unroll
  for (int i = 0; i < kQ; ++i) d[i] = C::dec((uint16_t)(w[i] & 0xffffu), G.inv_s);
#pragma unroll
  for (int k = 0; k < 2 * kQm; ++k) g[k] = C::dec((uint16_t)(w[kQ + k] & 0xffffu), G.inv_s);
  collide<FORCED>(d, g, P);
#pragma unroll
  for (int i = 0; i < kQ; ++i) lo[i] = C::enc(d[i], G.s);
#pragma unroll
  for (int k = 0; k < 2 * kQm; ++k) lo[kQ + k] = C::enc(g[k], G.s);
#pragma unroll
  for (int i = 0; i < kQ; ++i) d[i] = C::dec((uint16_t)(w[i] >> 16), G.inv_s);
#pragma unroll
  for (int k = 0; k < 2 * kQm; ++k) g[k] = C::dec((uint16_t)(w[kQ + k] >> 16), G.inv_s);
  collide<FORCED>(d, g, P);
  store_pair_planes<C, NT>(G, dst, b0 + 2u * x, lo, d, g,
                           std::make_integer_sequence<int, kPlanes>{});
}

}  // namespace rr
