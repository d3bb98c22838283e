// rr_pull.h -- the periodic node update shared by the single-domain and the
// batched kernels: pull the 19 populations of node (x, y) from their
// upstream neighbours (streaming, algorithm task 6), collide (tasks 1-5) and
// store the post-collision values at (x, y).  Every plane base is
// wave-uniform (scalar registers) and the in-plane position is a 32-bit byte
// offset, so each access is one global load/store with a scalar base.
#pragma once
#include <type_traits>
#include <utility>

#include "rr_node.h"

namespace rr {

struct PlaneGeom {
  int64_t plane;  // elements between plane starts (within one row)
  int nx, ny;
  float s, inv_s;  // storage scale
  uint32_t sr_key = 0;  // per-step key of the stochastic-rounding codec
  int64_t row = 0;      // elements between row starts of one plane
};

// Tile order of a persistent grid: the hardware deals workgroups to the
// eight XCDs in turn, so with a grid that is a multiple of 8 (and no larger
// than the tile count) each XCD takes one contiguous band of tiles, its
// workgroups side by side.  Neighbouring tiles, which share the cache lines
// of their halos, then meet in one L2.  Workgroup b visits tiles first,
// first + stride, ... below end.
struct TileBand {
  int first, end, stride;
};
__device__ __forceinline__ TileBand tile_band(int ntiles) {
  TileBand B{(int)blockIdx.x, ntiles, (int)gridDim.x};
  if ((gridDim.x & 7) == 0 && ntiles >= (int)gridDim.x) {
    const int band = (ntiles + 7) >> 3, xcd = blockIdx.x & 7;
    B.first = xcd * band + (blockIdx.x >> 3);
    B.end = min(ntiles, (xcd + 1) * band);
    B.stride = gridDim.x >> 3;
  }
  return B;
}

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

// Row addressing of a node update (rows y - 1, y, y + 1 of a periodic grid).
//  RM_OFFSET: one base per plane, the row as a 32-bit byte offset; for
//    layouts whose rows all lie within 4 GiB of a plane's start (planes of
//    [ny][nx] below 4 GiB).
//  RM_UNIFORM: a base pointer per row with the row index wave-uniform (the
//    caller guarantees that every lane of a wavefront updates the same row),
//    so the bases stay in scalar registers; any layout and size.
//  RM_LANE: a base pointer per row and lane; any layout, size and tile.
// In every mode the in-row position is a 32-bit byte offset.
enum { RM_OFFSET = 0, RM_UNIFORM = 1, RM_LANE = 2 };

template <class T>
struct RowAddr {
  const T *m, *z, *p;   // plane-0 bases for the rows y - 1, y, y + 1
  uint32_t om, oz, op;  // byte offsets added to them
};

template <int RM, class T>
__device__ __forceinline__ RowAddr<T> row_addr(const PlaneGeom &G, const T *s, int y) {
  if constexpr (RM == RM_UNIFORM) y = __builtin_amdgcn_readfirstlane(y);
  const int ym = y == 0 ? G.ny - 1 : y - 1, yp = y == G.ny - 1 ? 0 : y + 1;
  RowAddr<T> A;
  if constexpr (RM == RM_OFFSET) {
    const uint32_t pitch = (uint32_t)G.row * (uint32_t)sizeof(T);
    A.m = A.z = A.p = s;
    A.om = ym * pitch;
    A.oz = y * pitch;
    A.op = yp * pitch;
  } else {
    A.m = s + (int64_t)ym * G.row;
    A.z = s + (int64_t)y * G.row;
    A.p = s + (int64_t)yp * G.row;
    A.om = A.oz = A.op = 0;
  }
  return A;
}

// Where a store to row y goes: base pointer and byte offset of the row.
template <int RM, class T>
__device__ __forceinline__ T *row_dst(const PlaneGeom &G, T *d, int y, uint32_t &off) {
  if constexpr (RM == RM_UNIFORM) y = __builtin_amdgcn_readfirstlane(y);
  if constexpr (RM == RM_OFFSET) {
    off = (uint32_t)y * (uint32_t)G.row * (uint32_t)sizeof(T);
    return d;
  } else {
    off = 0;
    return d + (int64_t)y * G.row;
  }
}

// Population I of node (x, y) comes from (x - c_Ix, y - c_Iy).
template <class C, int I, bool NTL>
__device__ __forceinline__ float pull_f_per(const PlaneGeom &G, const RowAddr<typename C::T> &A,
                                            uint32_t xm, uint32_t x0, uint32_t xp) {
  constexpr int CX = cx(I), CY = cy(I);
  const typename C::T *base = CY == 0 ? A.z : (CY > 0 ? A.m : A.p);
  const uint32_t row = CY == 0 ? A.oz : (CY > 0 ? A.om : A.op);
  const uint32_t col = CX == 0 ? x0 : (CX > 0 ? xm : xp);
  return C::dec(ld_at<typename C::T, NTL>(plane_ptr(base, I, G.plane), row + col), G.inv_s);
}

template <class C, int J, int COMP, bool NTL>
__device__ __forceinline__ float pull_g_per(const PlaneGeom &G, const RowAddr<typename C::T> &A,
                                            uint32_t xm, uint32_t x0, uint32_t xp) {
  constexpr int EX = ex(J), EY = ey(J);
  const typename C::T *base = EY == 0 ? A.z : (EY > 0 ? A.m : A.p);
  const uint32_t row = EY == 0 ? A.oz : (EY > 0 ? A.om : A.op);
  const uint32_t col = EX == 0 ? x0 : (EX > 0 ? xm : xp);
  return C::dec(ld_at<typename C::T, NTL>(plane_ptr(base, gplane(J, COMP), G.plane), row + col),
                G.inv_s);
}

// The 19 populations of node (x, y) through the pull (periodic).
template <class C, bool NTL>
__device__ __forceinline__ void pull_node_per(const PlaneGeom &G, const RowAddr<typename C::T> &A,
                                              int x, float (&d)[kQ], float (&g)[2 * kQm]) {
  constexpr uint32_t E = sizeof(typename C::T);
  const uint32_t x0 = x * E;
  const uint32_t xm = (x == 0 ? G.nx - 1 : x - 1) * E;
  const uint32_t xp = (x == G.nx - 1 ? 0 : x + 1) * E;
  d[0] = pull_f_per<C, 0, NTL>(G, A, xm, x0, xp);
  d[1] = pull_f_per<C, 1, NTL>(G, A, xm, x0, xp);
  d[2] = pull_f_per<C, 2, NTL>(G, A, xm, x0, xp);
  d[3] = pull_f_per<C, 3, NTL>(G, A, xm, x0, xp);
  d[4] = pull_f_per<C, 4, NTL>(G, A, xm, x0, xp);
  d[5] = pull_f_per<C, 5, NTL>(G, A, xm, x0, xp);
  d[6] = pull_f_per<C, 6, NTL>(G, A, xm, x0, xp);
  d[7] = pull_f_per<C, 7, NTL>(G, A, xm, x0, xp);
  d[8] = pull_f_per<C, 8, NTL>(G, A, xm, x0, xp);
  g[0] = pull_g_per<C, 0, 0, NTL>(G, A, xm, x0, xp);
  g[1] = pull_g_per<C, 0, 1, NTL>(G, A, xm, x0, xp);
  g[2] = pull_g_per<C, 1, 0, NTL>(G, A, xm, x0, xp);
  g[3] = pull_g_per<C, 1, 1, NTL>(G, A, xm, x0, xp);
  g[4] = pull_g_per<C, 2, 0, NTL>(G, A, xm, x0, xp);
  g[5] = pull_g_per<C, 2, 1, NTL>(G, A, xm, x0, xp);
  g[6] = pull_g_per<C, 3, 0, NTL>(G, A, xm, x0, xp);
  g[7] = pull_g_per<C, 3, 1, NTL>(G, A, xm, x0, xp);
  g[8] = pull_g_per<C, 4, 0, NTL>(G, A, xm, x0, xp);
  g[9] = pull_g_per<C, 4, 1, NTL>(G, A, xm, x0, xp);
}

// Store the post-collision populations of one node at byte offset o of
// every plane.  Written plane by plane (not as a loop over a running
// pointer) so each store keeps a scalar plane base and the 32-bit offset.
// seed: the stochastic-rounding bits of the node (unused otherwise).
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
// The random bits of the stochastic-rounding codec are keyed by the node's
// position (y nx + x) in bytes of the stored type, whatever the layout.
template <class C>
__device__ __forceinline__ uint32_t node_seed(const PlaneGeom &G, int x, int y) {
  if constexpr (codec_sr<C>::value)
    return sr_seed(G.sr_key, ((uint32_t)y * (uint32_t)G.nx + (uint32_t)x) *
                                 (uint32_t)sizeof(typename C::T));
  else
    return 0;
}
// The stored value of population plane p computed by the node with random
// bits `seed` (stochastic rounding), or the codec's plain encode.
template <class C>
__device__ __forceinline__ typename C::T enc_node(const PlaneGeom &G, float v, uint32_t seed,
                                                  int p) {
  if constexpr (codec_sr<C>::value)
    return C::enc_sr(v, G.s, sr_plane(seed, p));
  else
    return C::enc(v, G.s);
}

template <class C, bool NT, int RM>
__device__ __forceinline__ void store_node(const PlaneGeom &G, typename C::T *__restrict__ dst,
                                           int x, int y, const float *d, const float *g) {
  uint32_t off;
  typename C::T *base = row_dst<RM>(G, dst, y, off);
  store_planes_seq<C, NT>(G, base, off + (uint32_t)x * (uint32_t)sizeof(typename C::T),
                          node_seed<C>(G, x, y), d, g,
                          std::make_integer_sequence<int, kPlanes>{});
}

// Pull, collide and store one node of a doubly periodic domain.  src/dst
// point at plane 0 of the domain's two buffers.
template <class C, bool FORCED, bool NT, bool NTL, bool FULLM = false, int RM = RM_OFFSET>
__device__ __forceinline__ void update_periodic(const PlaneGeom &G,
                                                const typename C::T *__restrict__ src,
                                                typename C::T *__restrict__ dst, int x,
                                                int y, const CollideParams &P) {
  float d[kQ], g[2 * kQm];
  pull_node_per<C, NTL>(G, row_addr<RM>(G, src, y), x, d, g);
  collide<FORCED, NoCorrection, FULLM>(d, g, P);
  store_node<C, NT, RM>(G, dst, x, y, d, g);
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

template <class C, bool FORCED, bool NT, int RM = RM_OFFSET>
__device__ __forceinline__ void update_periodic_push(const PlaneGeom &G, typename C::T *buf,
                                                     int x, int y, const CollideParams &P) {
  using T = typename C::T;
  constexpr uint32_t E = sizeof(T);
  const RowAddr<T> A = row_addr<RM>(G, (const T *)buf, y);
  const uint32_t x0 = x * E;
  const uint32_t xm = (x == 0 ? G.nx - 1 : x - 1) * E;
  const uint32_t xp = (x == G.nx - 1 ? 0 : x + 1) * E;
  float d[kQ], g[2 * kQm];
  pull_node_per<C, false>(G, A, x, d, g);
  collide<FORCED>(d, g, P);
  // f*_i(x) -> buf[opp(i)][x + c_i]: the slot read for direction opp(i)
  auto base = [&](int cyv) { return (T *)(cyv == 0 ? A.z : (cyv > 0 ? A.p : A.m)); };
  auto at = [&](int cxv, int cyv) {
    return (cyv == 0 ? A.oz : (cyv > 0 ? A.op : A.om)) + (cxv == 0 ? x0 : (cxv > 0 ? xp : xm));
  };
  const uint32_t seed = node_seed<C>(G, x, y);
#define RR_PUSHF(I) \
  store_plane_at<C, opp_f(I), NT>(G, base(cy(I)), at(cx(I), cy(I)), d[I], seed, I)
#define RR_PUSHG(J, K2)                                                                  \
  store_plane_at<C, gplane(opp_g(J), K2), NT>(G, base(ey(J)), at(ex(J), ey(J)), g[2 * J + K2], \
                                              seed, gplane(J, K2))
  RR_PUSHF(0); RR_PUSHF(1); RR_PUSHF(2); RR_PUSHF(3); RR_PUSHF(4); RR_PUSHF(5); RR_PUSHF(6);
  RR_PUSHF(7); RR_PUSHF(8);
  RR_PUSHG(0, 0); RR_PUSHG(0, 1); RR_PUSHG(1, 0); RR_PUSHG(1, 1); RR_PUSHG(2, 0);
  RR_PUSHG(2, 1); RR_PUSHG(3, 0); RR_PUSHG(3, 1); RR_PUSHG(4, 0); RR_PUSHG(4, 1);
#undef RR_PUSHF
#undef RR_PUSHG
}

template <class C, int P>
__device__ __forceinline__ float ld_own(const PlaneGeom &G, const typename C::T *buf,
                                        uint32_t o) {
  return C::dec(ld_at<typename C::T, false>(plane_ptr(buf, P, G.plane), o), G.inv_s);
}

template <class C, bool FORCED, bool NT, int RM = RM_OFFSET>
__device__ __forceinline__ void update_periodic_own(const PlaneGeom &G, typename C::T *buf,
                                                    int x, int y, const CollideParams &P) {
  constexpr uint32_t E = sizeof(typename C::T);
  uint32_t off;
  const typename C::T *src = row_dst<RM>(G, buf, y, off);
  const uint32_t o = off + x * E;
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
  store_node<C, NT, RM>(G, buf, x, y, d, g);
}

// ---- K neighbouring nodes per thread -------------------------------------------
// Nodes x .. x + K - 1 (x a multiple of K, nx a multiple of K): every plane
// moves as one word of K stored values per thread (element k: node x + k) --
// two 16-bit values in a 32-bit word or four in a 64-bit word for FP16
// storage, two FP32 values in a 64-bit word -- which divides the memory
// instructions per byte by K.  The planes shifted by +-1 in x read the word
// at an odd element position (gfx950 loads unaligned global words natively);
// at the periodic seam (x = 0 for c_x = +1, x = nx - K for c_x = -1) the
// word's elements come from both ends of the row and are read one by one.
// Each node's post-collision values replace its own elements of the loaded
// words, so the per-node arithmetic and results are those of one node per
// thread.
template <class T, int K>
struct NodeWord {
  static_assert(K * sizeof(T) == 4 || K * sizeof(T) == 8, "32- or 64-bit words");
  using W = std::conditional_t<K * sizeof(T) == 4, uint32_t, uint64_t>;
  using U = std::conditional_t<sizeof(T) == 2, uint16_t, uint32_t>;
  static constexpr int kBits = 8 * sizeof(T);
  __device__ __forceinline__ static T get(W w, int k) { return bits((U)(w >> (k * kBits))); }
  __device__ __forceinline__ static W put(W w, int k, T t) {
    const W m = (W)(U)~(U)0 << (k * kBits);
    return (w & ~m) | ((W)ubits(t) << (k * kBits));
  }
  __device__ __forceinline__ static T bits(U u) {
    T t;
    __builtin_memcpy(&t, &u, sizeof(T));
    return t;
  }
  __device__ __forceinline__ static U ubits(T t) {
    U u;
    __builtin_memcpy(&u, &t, sizeof(T));
    return u;
  }
};

template <int CX, bool NTL, int K, class T>
__device__ __forceinline__ typename NodeWord<T, K>::W ld_word(const T *__restrict__ plane,
                                                              uint32_t row, int x, int nx) {
  using NW = NodeWord<T, K>;
  using W = typename NW::W;
  constexpr uint32_t E = sizeof(T);
  if (CX == 0) return ld_at<W, NTL>((const W *)plane, row + E * x);
  const bool seam = CX > 0 ? x == 0 : x == nx - K;
  // first source node, kept inside the row so the word is always in bounds
  const int xs = CX > 0 ? (seam ? 0 : x - 1) : (seam ? nx - K : x + 1);
  W w = ld_at<W, NTL>((const W *)plane, row + E * xs);
  if (seam) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      int xx = x - CX + k;
      xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
      w = NW::put(w, k, ld_at<T, NTL>(plane, row + E * xx));
    }
  }
  return w;
}

template <class C, bool NT, int K, int P>
__device__ __forceinline__ void store_word(const PlaneGeom &G, typename C::T *__restrict__ dst,
                                           uint32_t o, const typename NodeWord<typename C::T, K>::W *w) {
  using W = typename NodeWord<typename C::T, K>::W;
  st_at<W, NT>((W *)(dst + (int64_t)P * G.plane), o, w[P]);
}
template <class C, bool NT, int K, int... P>
__device__ __forceinline__ void store_words(const PlaneGeom &G, typename C::T *__restrict__ dst,
                                            uint32_t o,
                                            const typename NodeWord<typename C::T, K>::W *w,
                                            std::integer_sequence<int, P...>) {
  (store_word<C, NT, K, P>(G, dst, o, w), ...);
}

// With stochastic rounding each element draws the bits of its own node, as
// one node per thread does.
template <class C, int K, bool FORCED, bool NT, bool NTL, int RM = RM_OFFSET>
__device__ __forceinline__ void update_periodic_multi(const PlaneGeom &G,
                                                      const typename C::T *__restrict__ src,
                                                      typename C::T *__restrict__ dst, int x,
                                                      int y, const CollideParams &P) {
  using T = typename C::T;
  using NW = NodeWord<T, K>;
  const RowAddr<T> A = row_addr<RM>(G, src, y);
  typename NW::W w[kPlanes];
  auto base = [&](int cyv) { return cyv == 0 ? A.z : (cyv > 0 ? A.m : A.p); };
  auto rowf = [&](int cyv) { return cyv == 0 ? A.oz : (cyv > 0 ? A.om : A.op); };
#define RR_LDF(I) \
  w[I] = ld_word<cx(I), NTL, K>(plane_ptr(base(cy(I)), I, G.plane), rowf(cy(I)), x, G.nx)
#define RR_LDG(J, K2)                                                                    \
  w[gplane(J, K2)] = ld_word<ex(J), NTL, K>(plane_ptr(base(ey(J)), gplane(J, K2), G.plane), \
                                            rowf(ey(J)), x, G.nx)
  RR_LDF(0); RR_LDF(1); RR_LDF(2); RR_LDF(3); RR_LDF(4); RR_LDF(5); RR_LDF(6); RR_LDF(7); RR_LDF(8);
  RR_LDG(0, 0); RR_LDG(0, 1); RR_LDG(1, 0); RR_LDG(1, 1); RR_LDG(2, 0); RR_LDG(2, 1);
  RR_LDG(3, 0); RR_LDG(3, 1); RR_LDG(4, 0); RR_LDG(4, 1);
#undef RR_LDF
#undef RR_LDG
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float d[kQ], g[2 * kQm];
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] = C::dec(NW::get(w[i], k), G.inv_s);
#pragma unroll
    for (int m = 0; m < 2 * kQm; ++m) g[m] = C::dec(NW::get(w[kQ + m], k), G.inv_s);
    collide<FORCED>(d, g, P);
    const uint32_t seed = node_seed<C>(G, x + k, y);
#pragma unroll
    for (int i = 0; i < kQ; ++i) w[i] = NW::put(w[i], k, enc_node<C>(G, d[i], seed, i));
#pragma unroll
    for (int m = 0; m < 2 * kQm; ++m)
      w[kQ + m] = NW::put(w[kQ + m], k, enc_node<C>(G, g[m], seed, kQ + m));
  }
  uint32_t off;
  T *out = row_dst<RM>(G, dst, y, off);
  store_words<C, NT, K>(G, out, off + (uint32_t)sizeof(T) * x, w,
                        std::make_integer_sequence<int, kPlanes>{});
}


// ---- single-buffer streaming with K nodes per thread ---------------------------
// The two phases of the alternating update with one word per plane.  Phase 0
// writes each updated word back over the K slots that its own load read
// (element by element at the periodic seam, where the load was assembled
// element by element), phase 1 reads and writes the node's own aligned
// words, so every slot is still read and written by one thread only.
template <int CX, bool NT, int K, class T>
__device__ __forceinline__ void st_word(T *__restrict__ plane, uint32_t row, int x, int nx,
                                        typename NodeWord<T, K>::W w) {
  using NW = NodeWord<T, K>;
  using W = typename NW::W;
  constexpr uint32_t E = sizeof(T);
  if (CX == 0) {
    st_at<W, NT>((W *)plane, row + E * x, w);
    return;
  }
  const bool seam = CX > 0 ? x == 0 : x == nx - K;
  if (!seam) {
    st_at<W, NT>((W *)plane, row + E * (x - CX), w);
    return;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int xx = x - CX + k;
    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
    st_at<T, NT>(plane, row + E * xx, NW::get(w, k));
  }
}

// Phase 0: pull as update_periodic_multi does, collide, and put f*_i of node
// x + k into element k of the word just read for the opposite direction
// (the slot buf[opp(i)][x + k + c_i]); every word returns to where it came
// from.  Stochastic rounding draws the bits of node x + k and of the
// population's own plane, as store_plane_at does.
template <class C, int K, bool FORCED, bool NT, int RM>
__device__ __forceinline__ void update_periodic_push_multi(const PlaneGeom &G,
                                                           typename C::T *buf, int x, int y,
                                                           const CollideParams &P) {
  using T = typename C::T;
  using NW = NodeWord<T, K>;
  const RowAddr<T> A = row_addr<RM>(G, (const T *)buf, y);
  typename NW::W w[kPlanes];
  auto base = [&](int cyv) { return (T *)(cyv == 0 ? A.z : (cyv > 0 ? A.m : A.p)); };
  auto rowf = [&](int cyv) { return cyv == 0 ? A.oz : (cyv > 0 ? A.om : A.op); };
#define RR_LDF(I) \
  w[I] = ld_word<cx(I), false, K>(plane_ptr((const T *)base(cy(I)), I, G.plane), rowf(cy(I)), x, G.nx)
#define RR_LDG(J, K2)                                                                      \
  w[gplane(J, K2)] = ld_word<ex(J), false, K>(                                            \
      plane_ptr((const T *)base(ey(J)), gplane(J, K2), G.plane), rowf(ey(J)), x, G.nx)
  RR_LDF(0); RR_LDF(1); RR_LDF(2); RR_LDF(3); RR_LDF(4); RR_LDF(5); RR_LDF(6); RR_LDF(7); RR_LDF(8);
  RR_LDG(0, 0); RR_LDG(0, 1); RR_LDG(1, 0); RR_LDG(1, 1); RR_LDG(2, 0); RR_LDG(2, 1);
  RR_LDG(3, 0); RR_LDG(3, 1); RR_LDG(4, 0); RR_LDG(4, 1);
#undef RR_LDF
#undef RR_LDG
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float d[kQ], g[2 * kQm];
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] = C::dec(NW::get(w[i], k), G.inv_s);
#pragma unroll
    for (int m = 0; m < 2 * kQm; ++m) g[m] = C::dec(NW::get(w[kQ + m], k), G.inv_s);
    collide<FORCED>(d, g, P);
    const uint32_t seed = node_seed<C>(G, x + k, y);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      w[opp_f(i)] = NW::put(w[opp_f(i)], k, enc_node<C>(G, d[i], seed, i));
#pragma unroll
    for (int j = 0; j < kQm; ++j) {
      w[gplane(opp_g(j), 0)] =
          NW::put(w[gplane(opp_g(j), 0)], k, enc_node<C>(G, g[2 * j], seed, gplane(j, 0)));
      w[gplane(opp_g(j), 1)] =
          NW::put(w[gplane(opp_g(j), 1)], k, enc_node<C>(G, g[2 * j + 1], seed, gplane(j, 1)));
    }
  }
#define RR_STF(I) \
  st_word<cx(I), NT, K>(base(cy(I)) + (int64_t)(I) * G.plane, rowf(cy(I)), x, G.nx, w[I])
#define RR_STG(J, K2)                                                                     \
  st_word<ex(J), NT, K>(base(ey(J)) + (int64_t)gplane(J, K2) * G.plane, rowf(ey(J)), x, G.nx, \
                        w[gplane(J, K2)])
  RR_STF(0); RR_STF(1); RR_STF(2); RR_STF(3); RR_STF(4); RR_STF(5); RR_STF(6); RR_STF(7); RR_STF(8);
  RR_STG(0, 0); RR_STG(0, 1); RR_STG(1, 0); RR_STG(1, 1); RR_STG(2, 0); RR_STG(2, 1);
  RR_STG(3, 0); RR_STG(3, 1); RR_STG(4, 0); RR_STG(4, 1);
#undef RR_STF
#undef RR_STG
}

// Phase 1: the node's own aligned words in the swapped layout (population i
// of node x + k is element k of plane opp(i)), collide, store in the pull
// layout at the same words.
template <class C, int K, bool FORCED, bool NT, int RM>
__device__ __forceinline__ void update_periodic_own_multi(const PlaneGeom &G,
                                                          typename C::T *buf, int x, int y,
                                                          const CollideParams &P) {
  using T = typename C::T;
  using NW = NodeWord<T, K>;
  using W = typename NW::W;
  uint32_t off;
  T *row = row_dst<RM>(G, buf, y, off);
  const uint32_t o = off + (uint32_t)sizeof(T) * x;
  W w[kPlanes];
#pragma unroll
  for (int p = 0; p < kPlanes; ++p) w[p] = ld_at<W, false>((const W *)(row + (int64_t)p * G.plane), o);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float d[kQ], g[2 * kQm];
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] = C::dec(NW::get(w[opp_f(i)], k), G.inv_s);
#pragma unroll
    for (int j = 0; j < kQm; ++j) {
      g[2 * j] = C::dec(NW::get(w[gplane(opp_g(j), 0)], k), G.inv_s);
      g[2 * j + 1] = C::dec(NW::get(w[gplane(opp_g(j), 1)], k), G.inv_s);
    }
    collide<FORCED>(d, g, P);
    const uint32_t seed = node_seed<C>(G, x + k, y);
#pragma unroll
    for (int i = 0; i < kQ; ++i) w[i] = NW::put(w[i], k, enc_node<C>(G, d[i], seed, i));
#pragma unroll
    for (int m = 0; m < 2 * kQm; ++m)
      w[kQ + m] = NW::put(w[kQ + m], k, enc_node<C>(G, g[m], seed, kQ + m));
  }
  store_words<C, NT, K>(G, row, o, w, std::make_integer_sequence<int, kPlanes>{});
}

}  // namespace rr
