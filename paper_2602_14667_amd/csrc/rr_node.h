// rr_node.h -- per-node arithmetic of the recursive regularised LB-MHD step
// on gfx950: the collision of one node (algorithm tasks 1-5 of Sec. II.B),
// the storage codecs and the pull addressing of task 6.  Every kernel that
// advances populations (single domain, batched ensemble) goes through these
// functions, so all variants round identically.
//
// Floating-point contract: the library is compiled with -ffp-contract=off;
// every fused multiply-add below is written as fmaf() on purpose, so the
// rounding does not depend on the surrounding code.
//
// Arithmetic is FP32 on deviations d_i = f_i - w_i.  Constants that are not
// exactly representable (w_i, 1/3, 1/6) never enter as rounded multipliers:
// the equilibrium and regularised parts are formed as w_i * [bracket] where
// the bracket uses only exact constants (3, 4.5, 1.5, 2.25, 9), and w_i is
// applied as a quotient by 36/W_i in {2.25, 9, 36} with one Newton/FMA
// correction, so a rounding error never repeats with the same sign every
// step.  The forced step (a body force, the project's reading for the
// Hartmann channel) is the exception: it runs tasks 1-5 in FP64 and rounds
// only on storage (collide_forced64 below says why).
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rr {

// ---- Sec. II.A lattices -------------------------------------------------
// D2Q9 velocities in Latt's ordering: c_x = [0,-1,-1,-1,0,1,1,1,0],
// c_y = [0,1,0,-1,-1,-1,0,1,1]; weights 4/9 (rest), 1/36 (diagonals,
// odd i), 1/9 (axes, even i > 0).  D2Q5: e_x = [0,-1,0,1,0],
// e_y = [0,0,-1,0,1], weights 1/3 and 1/6.
constexpr int kQ = 9;
constexpr int kQm = 5;
constexpr int kPlanes = kQ + 2 * kQm;  // f_0..f_8, then g_jx, g_jy pairs

__host__ __device__ constexpr int cx(int i) {
  return (i >= 1 && i <= 3) ? -1 : ((i >= 5 && i <= 7) ? 1 : 0);
}
__host__ __device__ constexpr int cy(int i) {
  return (i == 1 || i == 7 || i == 8) ? 1 : ((i >= 3 && i <= 5) ? -1 : 0);
}
__host__ __device__ constexpr int ex(int j) {
  return j == 1 ? -1 : (j == 3 ? 1 : 0);
}
__host__ __device__ constexpr int ey(int j) {
  return j == 2 ? -1 : (j == 4 ? 1 : 0);
}
// 36 / W_i: the divisor that applies w_i = W_i / 36.
__host__ __device__ constexpr float wdiv(int i) {
  return i == 0 ? 2.25f : ((i & 1) ? 36.0f : 9.0f);
}
__host__ __device__ constexpr int opp_f(int i) { return i == 0 ? 0 : ((i + 3) & 7) + 1; }
__host__ __device__ constexpr int opp_g(int j) { return j == 0 ? 0 : ((j + 1) & 3) + 1; }
__host__ __device__ constexpr int gplane(int j, int comp) { return kQ + 2 * j + comp; }

// a / d for an exactly representable constant d with rd = RN(1/d): the
// product a*rd is corrected by one FMA residual step (Markstein), which
// returns the correctly rounded quotient for normal operands.
__device__ __forceinline__ float qdiv(float a, float d, float rd) {
  float q = a * rd;
  float e = fmaf(-q, d, a);
  return fmaf(e, rd, q);
}

// a / b for a runtime divisor b near 1 (the density): hardware reciprocal
// estimate refined by the same residual step.
__device__ __forceinline__ float rdiv(float a, float b, float rb) {
  float q = a * rb;
  float e = fmaf(-q, b, a);
  return fmaf(e, rb, q);
}

// ---- storage codecs ------------------------------------------------------
// Stored value for the fluid plane i: S (f_i - w_i); for a magnetic plane:
// S g.  F32 keeps S = 1.  F16 converts with round-to-nearest-even.
//
// The FP16 encodes round the FP32 value as computed.  Left to itself the
// compiler may fold the last FMA of the collision and the conversion into one
// mixed-precision instruction that rounds the exact result once, and it
// makes that choice kernel by kernel, so two kernels would then differ by one
// FP16 unit where the FP32 value sits on a rounding tie.  An empty asm
// statement hides where the value came from, which keeps every kernel's
// stores identical.
__device__ __forceinline__ float f32_as_computed(float v) {
  asm("" : "+v"(v));
  return v;
}
struct CodecF32 {
  using T = float;
  __device__ __forceinline__ static float dec(T v, float) { return v; }
  __device__ __forceinline__ static T enc(float v, float) { return v; }
};
struct CodecF16 {
  using T = uint16_t;  // IEEE binary16 bit pattern
  __device__ __forceinline__ static float dec(T v, float inv_s) {
    return __half2float(__ushort_as_half(v)) * inv_s;
  }
  __device__ __forceinline__ static T enc(float v, float s) {
    return __half_as_ushort(__float2half_rn(f32_as_computed(v * s)));
  }
};
// The F16 codec at S = 1 (the default), used by every kernel that writes
// populations when S = 1: the same stored bits as CodecF16 at S = 1 without
// the multiplies by 1 on decode and encode.
struct CodecF16U {
  using T = uint16_t;
  __device__ __forceinline__ static float dec(T v, float) {
    return __half2float(__ushort_as_half(v));
  }
  __device__ __forceinline__ static T enc(float v, float) {
    return __half_as_ushort(__float2half_rn(f32_as_computed(v)));
  }
};

// FP16 storage with stochastic rounding (an optional variant of the codec):
// a value is rounded to one of its two FP16 neighbours, away from zero with
// probability equal to its distance from the one toward zero in units of the
// gap, so the stored value is unbiased.  The random bits come from the caller
// (a counter-based hash of step, node and plane).  Decoding and the plain
// encode (used at initialisation) are those of CodecF16.
//
// With e the biased FP32 exponent of x = v s and m its significand with the
// leading one (24 bits), the FP16 grid below |x| has spacing 2^(e-150+d)
// where d = max(126 - e, 13) bits of m are dropped (13 in FP16's normal
// range, more below 2^-14 where the grid is 2^-24).  The dropped fraction is
// kept to 13 bits, t = floor(m 2^(13-d)), and the kept integer is
// k = floor((t + r_13) 2^-13) with r_13 the top 13 of the 32 random bits: the
// carry happens with probability equal to the dropped fraction -- exactly in
// FP16's normal range, to 2^-13 of the 2^-24 grid below (toward zero), and
// magnitudes below 2^-37 store zero.  k is the FP16 pattern less the
// exponent field ((e - 113) << 10 for normal values, nothing for
// subnormals).  Results past the largest finite value store infinity; NaN
// stores a quiet NaN of the same sign and the top ten payload bits.  gfx950
// performs this conversion in one instruction (v_cvt_sr_f16_f32); a GPU test
// compares the library's encode with this rule written out value by value.
struct CodecF16SR {
  using T = uint16_t;
  static constexpr bool kSR = true;
  __device__ __forceinline__ static float dec(T v, float inv_s) {
    return __half2float(__ushort_as_half(v)) * inv_s;
  }
  __device__ __forceinline__ static T enc(float v, float s) {
    return __half_as_ushort(__float2half_rn(v * s));
  }
  __device__ __forceinline__ static T enc_sr(float v, float s, uint32_t r) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 z = {0, 0};
    z = __builtin_amdgcn_cvt_sr_f16_f32(z, v * s, r, false);
    const _Float16 lo = z[0];
    T u;
    __builtin_memcpy(&u, &lo, sizeof u);
    return u;
  }
};

// Whether a codec rounds stochastically.
template <class C, class = void>
struct codec_sr : std::false_type {};
template <class C>
struct codec_sr<C, std::void_t<decltype(C::kSR)>> : std::bool_constant<C::kSR> {};

// 32-bit mixer (the MurmurHash3 finaliser) for counter-based random bits.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
// Random bits for the plane p of a node: a node seed from the step key k and
// the node's in-plane byte offset o (computed once per node), then one
// multiply-xorshift round over a Weyl sequence in the plane number.
__device__ __forceinline__ uint32_t sr_seed(uint32_t k, uint32_t o) {
  return mix32(k ^ (o * 0x9e3779b1u));
}
__device__ __forceinline__ uint32_t sr_plane(uint32_t seed, int p) {
  uint32_t h = seed + (uint32_t)(p + 1) * 0x9e3779b9u;
  h ^= h >> 16;
  h *= 0x21f0aaadu;
  return h ^ (h >> 15);
}

// ---- parameters of the collision ------------------------------------------
struct CollideParams {
  float om_c;   // 1 - omega,   omega   = 1 / tau_f
  float omm_c;  // 1 - omega_m, omega_m = 1 / tau_m
  float Gx, Gy;  // body force per unit mass (zero in the paper's method)
  float src_c;   // 1 - omega / 2 (forcing source factor)
};

struct Acoef {
  float xx, xy, yy, xxy, xyy, xxyy;
};

// Regularised non-equilibrium bracket for velocity (CX, CY), times (1-omega)
// already folded into A (Eq. fineq_reg restricted to the D2Q9-supported
// components): with h = 3 c^2 - 1,
//   R = 1.5 (hx Axx + hy Ayy) + 9 cx cy Axy
//     + 4.5 (cy hx Axxy + cx hy Axyy) + 2.25 hx hy Axxyy,
// so that f_neq,reg,i = w_i R.
template <int CX, int CY>
__device__ __forceinline__ float reg_bracket(const Acoef &A) {
  constexpr float hx = CX ? 2.0f : -1.0f;
  constexpr float hy = CY ? 2.0f : -1.0f;
  float r = 1.5f * fmaf(hx, A.xx, hy * A.yy);
  if constexpr (CX != 0 && CY != 0) r = fmaf(9.0f * CX * CY, A.xy, r);
  if constexpr (CY != 0) r = fmaf(4.5f * CY * hx, A.xxy, r);
  if constexpr (CX != 0) r = fmaf(4.5f * CX * hy, A.xyy, r);
  return fmaf(2.25f * hx * hy, A.xxyy, r);
}

struct EqTerms {
  float dr, rho;
  float ex0, exp, exm, ey0, eyp, eym;  // D1Q3 factors minus one
  float mq;                            // 4.5 M_xx
  float mxy;                           // 9 b_x b_y
};

// Equilibrium bracket: f_eq,i - w_i = w_i B with
//   B = rho (1 + e_x)(1 + e_y) - 1 + 4.5 [|b|^2 |c|^2 / 2 - (c.b)^2],
// where (1 + e) is the D1Q3 factor 1 - 1.5 u^2 (c = 0) or 1 +- 3u + 3u^2
// (c = +-1).  The product equals the fourth-order Hermite equilibrium of
// algorithm task 2 at b = 0 term by term, including its u_x^2 u_y^2 term
// with the coefficient 1/(4 c_s^8).
template <int CX, int CY>
__device__ __forceinline__ float eq_bracket(const EqTerms &E) {
  const float exv = CX == 0 ? E.ex0 : (CX > 0 ? E.exp : E.exm);
  const float eyv = CY == 0 ? E.ey0 : (CY > 0 ? E.eyp : E.eym);
  float s = fmaf(exv, eyv, exv + eyv);
  float B = fmaf(E.rho, s, E.dr);
  if constexpr (CX != 0 && CY == 0) B = B + E.mq;
  if constexpr (CX == 0 && CY != 0) B = B - E.mq;
  if constexpr (CX != 0 && CY != 0) B = fmaf(-(float)(CX * CY), E.mxy, B);
  return B;
}

template <int I>
__device__ __forceinline__ float post_f(const EqTerms &E, const Acoef &A) {
  constexpr int CX = cx(I), CY = cy(I);
  const float v = eq_bracket<CX, CY>(E) + reg_bracket<CX, CY>(A);
  return qdiv(v, wdiv(I), 1.0f / wdiv(I));
}

// Hook applied to the second-order non-equilibrium coefficients between
// their projection and the recursion (task 3).  The plain method uses none.
struct NoCorrection {
  __device__ __forceinline__ void operator()(float, float, float, float, float, float &,
                                             float &, float &) const {}
};

// ---- the forced collision, in FP64 ------------------------------------------
// A body force adds the same small impulse to every node at every step (G =
// 1e-6 against velocities of 1e-2 in the Hartmann channel: a few hundred
// units in the last place of an FP32 velocity).  In FP32 arithmetic that
// increment is added to values that sit on the FP32 grid, so its rounding
// has the same sign at every node and every step: a coherent bias (about
// -0.2 % of the force in a uniform box) that the storage rounding alone does
// not have, since the stored values are pseudo-random in their low bits.
// The forced step therefore evaluates tasks 1-5 in FP64 and rounds only when
// it stores; the unforced method keeps FP32 arithmetic.  Constants enter as
// FP64 products with correctly rounded FP64 reciprocals (their rounding is
// far below the FP32 storage's).
template <int CX, int CY>
__device__ __forceinline__ double reg_bracket64(const double (&A)[6]) {
  constexpr double hx = CX ? 2.0 : -1.0;
  constexpr double hy = CY ? 2.0 : -1.0;
  double r = 1.5 * fma(hx, A[0], hy * A[2]);
  if constexpr (CX != 0 && CY != 0) r = fma(9.0 * CX * CY, A[1], r);
  if constexpr (CY != 0) r = fma(4.5 * CY * hx, A[3], r);
  if constexpr (CX != 0) r = fma(4.5 * CX * hy, A[4], r);
  return fma(2.25 * hx * hy, A[5], r);
}

template <int I, bool FULLM>
__device__ __forceinline__ float post_f64(double rho, double dr, const double (&ex)[3],
                                          const double (&ey)[3], double mq, double mxy,
                                          const double (&A)[6], double a1c, double a1x,
                                          double a1y, double sc, double Fx, double Fy,
                                          double ux, double uy) {
  constexpr int CX = cx(I), CY = cy(I);
  constexpr double hx = CX ? 2.0 : -1.0;
  constexpr double hy = CY ? 2.0 : -1.0;
  // equilibrium bracket (D1Q3 product, Maxwell stress at second order)
  const double exv = ex[CX + 1], eyv = ey[CY + 1];
  double B = fma(rho, fma(exv, eyv, exv + eyv), dr);
  if constexpr (CX != 0 && CY == 0) B = B + mq;
  if constexpr (CX == 0 && CY != 0) B = B - mq;
  if constexpr (CX != 0 && CY != 0) B = fma(-(double)(CX * CY), mxy, B);
  // forcing: (1 - omega) 3 c.a1 + (1 - omega/2)[3 c.F + 3 (hx ux Fx + hy uy Fy)
  // + 9 cx cy (ux Fy + uy Fx)]
  double ca1 = 0.0, cF = 0.0;
  if constexpr (CX != 0) { ca1 = CX * a1x; cF = CX * Fx; }
  if constexpr (CY != 0) { ca1 = ca1 + CY * a1y; cF = cF + CY * Fy; }
  double fs = 3.0 * fma(hx * ux, Fx, hy * uy * Fy) + 3.0 * cF;
  if constexpr (CX != 0 && CY != 0) fs = fma(9.0 * CX * CY, fma(ux, Fy, uy * Fx), fs);
  const double v = B + reg_bracket64<CX, CY>(A) + fma(a1c, ca1, sc * fs);
  return (float)(v * (1.0 / (double)wdiv(I)));
}

template <bool FULLM>
__device__ __forceinline__ void collide_forced64(float (&d)[kQ], float (&g)[2 * kQm],
                                                 const CollideParams &P) {
  double f[kQ], m[2 * kQm];
#pragma unroll
  for (int i = 0; i < kQ; ++i) f[i] = d[i];
#pragma unroll
  for (int k = 0; k < 2 * kQm; ++k) m[k] = g[k];
  // task 1, with the velocity carrying half the force impulse
  const double dr = ((f[0] + f[2]) + (f[4] + f[6])) + (((f[1] + f[3]) + (f[5] + f[7])) + f[8]);
  const double rho = 1.0 + dr;
  const double jx = ((f[5] + f[6]) + f[7]) - ((f[1] + f[2]) + f[3]);
  const double jy = ((f[1] + f[7]) + f[8]) - ((f[3] + f[4]) + f[5]);
  const double Gx = P.Gx, Gy = P.Gy;
  const double Fx = rho * Gx, Fy = rho * Gy;
  const double ux = fma(0.5, Fx, jx) / rho;
  const double uy = fma(0.5, Fy, jy) / rho;
  const double bx = ((m[0] + m[2]) + (m[4] + m[6])) + m[8];
  const double by = ((m[1] + m[3]) + (m[5] + m[7])) + m[9];
  // task 3: exact Hermite moments of f_eq, projection, recursion
  const double pxx = ((f[1] + f[2]) + f[3]) + ((f[5] + f[6]) + f[7]);
  const double pyy = ((f[1] + f[3]) + (f[5] + f[7])) + (f[4] + f[8]);
  const double pxy = (f[3] + f[7]) - (f[1] + f[5]);
  const double dr3 = dr * (1.0 / 3.0);
  const double bxy = bx * by;
  const double mxx = 0.5 * (by * by - bx * bx);
  const double rux = rho * ux, ruy = rho * uy;
  const double axx = fma(-rux, ux, pxx - dr3) - mxx;
  const double ayy = fma(-ruy, uy, pyy - dr3) + mxx;
  const double axy = fma(-rux, uy, pxy) + bxy;
  const double om = P.om_c;
  double A[6];
  A[0] = om * axx;
  A[1] = om * axy;
  A[2] = om * ayy;
  A[3] = om * fma(2.0 * ux, axy, uy * axx);
  A[4] = om * fma(2.0 * uy, axy, ux * ayy);
  A[5] = om * fma(ux * ux, ayy, fma(uy * uy, axx, (4.0 * ux) * (uy * axy)));
  if constexpr (FULLM) {
    // u.M cross terms of the third- and fourth-order equilibrium (ablation)
    A[3] += fma(uy, mxx, -2.0 * (ux * bxy));
    A[4] += fma(-ux, mxx, -2.0 * (uy * bxy));
    A[5] += fma(fma(uy, uy, -ux * ux), mxx, -4.0 * (ux * (uy * bxy)));
  }
  // task 2: D1Q3 factors minus one, indexed by c + 1
  const double ux2 = ux * ux, uy2 = uy * uy;
  const double ex[3] = {fma(-3.0, ux, 3.0 * ux2), -1.5 * ux2, fma(3.0, ux, 3.0 * ux2)};
  const double ey[3] = {fma(-3.0, uy, 3.0 * uy2), -1.5 * uy2, fma(3.0, uy, 3.0 * uy2)};
  const double mq = 4.5 * mxx, mxy = 9.0 * bxy;
  const double a1c = 3.0 * om, a1x = -0.5 * Fx, a1y = -0.5 * Fy;
  const double sc = P.src_c;
  // tasks 4-5 per velocity, rounded once to FP32
  d[0] = post_f64<0, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[1] = post_f64<1, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[2] = post_f64<2, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[3] = post_f64<3, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[4] = post_f64<4, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[5] = post_f64<5, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[6] = post_f64<6, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[7] = post_f64<7, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  d[8] = post_f64<8, FULLM>(rho, dr, ex, ey, mq, mxy, A, a1c, a1x, a1y, sc, Fx, Fy, ux, uy);
  // magnetic BGK with E = u_x b_y - u_y b_x; the rest population from the
  // conservation of b, as in the FP32 collision
  const double E3 = 3.0 * fma(ux, by, -uy * bx);
  const double r3 = 1.0 / 3.0, r6 = 1.0 / 6.0;
  const double bx3 = bx * r3, by3 = by * r3, bx6 = bx * r6, by6 = by * r6;
  const double geq[2 * kQm] = {bx3, by3, bx6, (by - E3) * r6, (bx + E3) * r6, by6,
                               bx6, (by + E3) * r6, (bx - E3) * r6, by6};
  const double omm = P.omm_c;
  double gs[2 * kQm];
#pragma unroll
  for (int k = 2; k < 2 * kQm; ++k) gs[k] = fma(omm, m[k] - geq[k], geq[k]);
  gs[0] = bx - ((gs[2] + gs[4]) + (gs[6] + gs[8]));
  gs[1] = by - ((gs[3] + gs[5]) + (gs[7] + gs[9]));
#pragma unroll
  for (int k = 0; k < 2 * kQm; ++k) g[k] = (float)gs[k];
}

// One collision (algorithm tasks 1-5) in place.  d[i] = f_i - w_i on entry,
// f*_i - w_i on exit; g[2j + c] = g_j,c before and after.  corr(rho, u_x,
// u_y, b_x, b_y, a_xx, a_xy, a_yy) may adjust the three a_1^(2) components.
// FULLM selects the equilibrium variant that keeps the u.M cross terms of
// the third- and fourth-order equilibrium coefficients (Eq. eq:a0_4), which
// the algorithm's equilibrium (Eq. feq_4th, task 2) leaves out; it exists
// for the ablation of that reading only.
template <bool FORCED, class Corr = NoCorrection, bool FULLM = false>
__device__ __forceinline__ void collide(float (&d)[kQ], float (&g)[2 * kQm],
                                        const CollideParams &P,
                                        const Corr &corr = Corr()) {
  if constexpr (FORCED) {
    static_assert(std::is_same_v<Corr, NoCorrection>, "the closure runs unforced");
    collide_forced64<FULLM>(d, g, P);
    return;
  }
  // task 1: macroscopic variables
  const float dr = ((d[0] + d[2]) + (d[4] + d[6])) +
                   (((d[1] + d[3]) + (d[5] + d[7])) + d[8]);
  const float rho = 1.0f + dr;
  const float jx = ((d[5] + d[6]) + d[7]) - ((d[1] + d[2]) + d[3]);
  const float jy = ((d[1] + d[7]) + d[8]) - ((d[3] + d[4]) + d[5]);
  const float rr = __builtin_amdgcn_rcpf(rho);
  const float ux = rdiv(jx, rho, rr);
  const float uy = rdiv(jy, rho, rr);
  const float bx = ((g[0] + g[2]) + (g[4] + g[6])) + g[8];
  const float by = ((g[1] + g[3]) + (g[5] + g[7])) + g[9];

  // task 3 (needs only the Hermite moments of f_eq, which are exact):
  // a_ab = sum_i H_ab,i (f_i - f_eq,i) = P_ab - c_s^2 dr delta_ab
  //        - rho u_a u_b - M_ab, with P_ab = sum_i c_a c_b d_i.
  const float pxx = ((d[1] + d[2]) + d[3]) + ((d[5] + d[6]) + d[7]);
  const float pyy = ((d[1] + d[3]) + (d[5] + d[7])) + (d[4] + d[8]);
  const float pxy = (d[3] + d[7]) - (d[1] + d[5]);
  const float dr3 = qdiv(dr, 3.0f, 1.0f / 3.0f);
  const float bxx = bx * bx, byy = by * by, bxy = bx * by;
  const float mxx = 0.5f * (byy - bxx);  // M_xx = -M_yy; M_xy = -b_x b_y
  const float rux = rho * ux, ruy = rho * uy;
  Acoef A;
  float axx = fmaf(-rux, ux, pxx - dr3) - mxx;
  float ayy = fmaf(-ruy, uy, pyy - dr3) + mxx;
  float axy = fmaf(-rux, uy, pxy) + bxy;
  corr(rho, ux, uy, bx, by, axx, axy, ayy);
  // recursion for the third and fourth orders (D2Q9-supported components)
  const float axxy = fmaf(2.0f * ux, axy, uy * axx);
  const float axyy = fmaf(2.0f * uy, axy, ux * ayy);
  const float axxyy =
      fmaf(ux * ux, ayy, fmaf(uy * uy, axx, (4.0f * ux) * (uy * axy)));
  A.xx = P.om_c * axx;
  A.yy = P.om_c * ayy;
  A.xy = P.om_c * axy;
  A.xxy = P.om_c * axxy;
  A.xyy = P.om_c * axyy;
  A.xxyy = P.om_c * axxyy;
  if constexpr (FULLM) {
    // The cross terms of a0^(3) and a0^(4) on the supported components,
    // with M_yy = -M_xx and M_xy = -b_x b_y:
    //   xxy: 2 u_x M_xy + u_y M_xx,  xyy: u_x M_yy + 2 u_y M_xy,
    //   xxyy: u_x^2 M_yy + u_y^2 M_xx + 4 u_x u_y M_xy.
    // Their Hermite weights in the equilibrium series equal those of the
    // regularised bracket (4.5 c_y h_x, 4.5 c_x h_y, 2.25 h_x h_y), so they
    // enter as additions to the third- and fourth-order coefficients.
    const float m3xxy = fmaf(uy, mxx, -2.0f * (ux * bxy));
    const float m3xyy = fmaf(-ux, mxx, -2.0f * (uy * bxy));
    const float m4 = fmaf(fmaf(uy, uy, -ux * ux), mxx, -4.0f * (ux * (uy * bxy)));
    A.xxy = A.xxy + m3xxy;
    A.xyy = A.xyy + m3xyy;
    A.xxyy = A.xxyy + m4;
  }

  // task 2: equilibrium factors
  EqTerms E;
  E.dr = dr;
  E.rho = rho;
  const float ux2 = ux * ux, uy2 = uy * uy;
  E.ex0 = -1.5f * ux2;
  E.exp = fmaf(3.0f, ux, 3.0f * ux2);
  E.exm = fmaf(-3.0f, ux, 3.0f * ux2);
  E.ey0 = -1.5f * uy2;
  E.eyp = fmaf(3.0f, uy, 3.0f * uy2);
  E.eym = fmaf(-3.0f, uy, 3.0f * uy2);
  E.mq = 4.5f * mxx;
  E.mxy = 9.0f * bxy;

  // tasks 4-5: regularised reconstruction and collision, per velocity
  d[0] = post_f<0>(E, A);
  d[1] = post_f<1>(E, A);
  d[2] = post_f<2>(E, A);
  d[3] = post_f<3>(E, A);
  d[4] = post_f<4>(E, A);
  d[5] = post_f<5>(E, A);
  d[6] = post_f<6>(E, A);
  d[7] = post_f<7>(E, A);
  d[8] = post_f<8>(E, A);

  // magnetic BGK: g_eq,j = psi_j [b + e_j.(u b - b u) / c_s^2], i.e. with
  // E = u_x b_y - u_y b_x: g_eq,j = psi_j (b_x - 3 e_jy E, b_y + 3 e_jx E).
  const float Ez3 = 3.0f * fmaf(ux, by, -uy * bx);
  const float bx3 = qdiv(bx, 3.0f, 1.0f / 3.0f);
  const float by3 = qdiv(by, 3.0f, 1.0f / 3.0f);
  const float bx6 = 0.5f * bx3, by6 = 0.5f * by3;  // exact halving
  const float q1y = qdiv(by - Ez3, 6.0f, 1.0f / 6.0f);
  const float q2x = qdiv(bx + Ez3, 6.0f, 1.0f / 6.0f);
  const float q3y = qdiv(by + Ez3, 6.0f, 1.0f / 6.0f);
  const float q4x = qdiv(bx - Ez3, 6.0f, 1.0f / 6.0f);
  const float geq[2 * kQm] = {bx3, by3, bx6, q1y, q2x, by6, bx6, q3y, q4x, by6};
#pragma unroll
  for (int k = 2; k < 2 * kQm; ++k) g[k] = fmaf(P.omm_c, g[k] - geq[k], geq[k]);
  // The collision leaves b = sum_j g_j unchanged (sum_j g_eq,j = b), so the
  // rest population is taken from that identity: g*_0 = b - sum_{j>0} g*_j.
  // Each node then conserves its field exactly up to one rounding per step
  // instead of accumulating the roundings of five relaxations.
  g[0] = bx - ((g[2] + g[4]) + (g[6] + g[8]));
  g[1] = by - ((g[3] + g[5]) + (g[7] + g[9]));
}

}  // namespace rr
