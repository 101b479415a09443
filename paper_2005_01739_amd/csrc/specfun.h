// Device special functions for the pair weights of the periodic-box
// power-spectrum and bispectrum estimators (Philcox 2020, arXiv:2005.01739).
//
// The bin-averaged spherical Bessel function (Sec. 3, eq. jla-def) is
//   jbar^a_l(r) = 3 [D_l(k_{a+1} r) - D_l(k_a r)] / (r^3 (k_{a+1}^3 - k_a^3)),
// with D_l(u) = int u^2 j_l(u) du (Appendix C).  The kernels accumulate, per
// bin edge e, G_l(k_e r) = Dt_l(k_e r) / (k_e r)^3 where Dt_l(u) = D_l(u) -
// D_l(0) = int_0^u t^2 j_l(t) dt, so that
//   jbar^a_l(r) = 3 [k_{a+1}^3 G_l(k_{a+1} r) - k_a^3 G_l(k_a r)] / (k_{a+1}^3 - k_a^3).
// G_l is bounded (G_0(0) = 1/3, G_{l>0}(0) = 0) and smooth, so pairs at r -> 0
// need no special case.
//
// Running the Appendix C recursion (I_0 = Si, I_1 = -j_0) symbolically gives
// D_l(u) = c_l Si(u) + a_l(u) sin u + b_l(u) cos u with Laurent polynomials
// a_l, b_l and c_l = 0, 3, 15/2, 105/8 for even l = 0, 2, 4, 6 (c_l = 0 for
// odd l); D_l(0) = 0, -2, 0, -8, 0, -16, 0 for l = 0..6.  For large u the sine
// integral is written through its auxiliary functions,
//   Si(u) = pi/2 - f(u) cos u - g(u) sin u,
// so every term is a smooth amplitude times sin u or cos u.  Below U_BIG the
// closed form cancels badly (the Laurent terms grow like u^-l), and G_l is
// summed from its Taylor series instead.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coeffs.h"

namespace hipster {

constexpr int kLMax = 6;

// a * b + c rounded once, written as the three-operand v_fma_f64.  For a
// Horner step whose addend is a constant held in a register, the compiler
// otherwise emits the two-operand v_fmac_f64 (which overwrites its addend)
// plus a copy of the constant, two instructions per step.  The result is the
// same correctly rounded fused multiply-add either way.  A translation unit
// that defines HIPSTER_PLAIN_FMA gets the plain fma instead: the asm operands
// must be VGPRs, so every coefficient then occupies a VGPR pair for the
// whole loop, which a register-bound kernel cannot afford.
#ifdef HIPSTER_PLAIN_FMA
static __device__ inline double fma3(double a, double b, double c) { return fma(a, b, c); }
#else
static __device__ inline double fma3(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
#endif
constexpr double kPi = 3.14159265358979323846;
constexpr double kHalfPi = 1.57079632679489661923;
// Below this argument the Taylor series needs only 14 terms, and the mixed
// form switches from the Taylor series to the closed form.
constexpr double kUSmall = 2.0;

// Smooth truncation window W(x), x = r / R0 (Sec. 2, eq. window_defn).
template <typename T>
__host__ __device__ inline T window(T x) {
  if (x < T(0.5)) return T(1);
  if (x < T(0.75)) {
    T t = T(2) * x - T(1);
    T t3 = t * t * t;
    return T(1) - T(8) * t3 + T(8) * t3 * t;
  }
  if (x < T(1)) {
    T t = x - T(1);
    T t3 = t * t * t;
    return T(-64) * t3 - T(128) * t3 * t;
  }
  return T(0);
}

// Legendre polynomials of even order, L_0 .. L_{2(NE-1)}.
template <typename T, int NE>
__host__ __device__ inline void legendre_even(T mu, T (&L)[NE]) {
  T m2 = mu * mu;
  L[0] = T(1);
  if (NE > 1) L[1] = T(1.5) * m2 - T(0.5);
  if (NE > 2) L[2] = (T(35) * m2 * m2 - T(30) * m2 + T(3)) * T(0.125);
  if (NE > 3) L[3] = ((T(231) * m2 - T(315)) * m2 * m2 + T(105) * m2 - T(5)) * T(0.0625);
}

// --------------------------------------------------------------- Taylor form
// G_l(u) = u^l sum_s TAYLOR_G[l][s] (u^2)^s, double precision, NT terms.
template <int NT>
__device__ inline double taylor_G64(int l, double v, double ul) {
  double p = TAYLOR_G[l][NT - 1];
#pragma unroll
  for (int s = NT - 2; s >= 0; --s) p = fma3(p, v, TAYLOR_G[l][s]);
  return p * ul;
}

// ------------------------------------------------------ closed-form pieces
// Dt_l(u) from sin u, cos u, Si(u) and w = 1/u (closed forms of the Appendix C
// recursion, minus D_l(0)).
template <typename T>
__device__ inline T Dt_closed(int l, T u, T w, T s, T c, T si) {
  switch (l) {
    case 0: return s - u * c;
    case 1: return T(2) - u * s - T(2) * c;
    case 2: return T(3) * si - T(4) * s + u * c;
    case 3: return T(8) + (u - T(15) * w) * s + T(7) * c;
    case 4: {
      T w2 = w * w;
      return T(7.5) * si + (T(11) - T(52.5) * w2) * s + (T(52.5) * w - u) * c;
    }
    case 5: {
      T w2 = w * w;
      return T(16) + ((T(105) - T(315) * w2) * w - u) * s + (T(315) * w2 - T(16)) * c;
    }
    default: {
      T w2 = w * w;
      return T(13.125) * si + ((T(-2598.75) * w2 + T(1063.125)) * w2 - T(22)) * s +
             (u + (T(2598.75) * w2 - T(196.875)) * w) * c;
    }
  }
}

// Horner sum of a polynomial with double coefficients.
template <int N>
__device__ inline double horner64(const double (&p)[N], double t) {
  double r = p[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) r = fma3(r, t, p[k]);
  return r;
}

// Values G_l(u) for l = 0, LSTEP, 2 LSTEP, ... (NL of them), returned in
// registers.
template <typename T, int NL>
struct Gv {
  T v[NL];
};

// Taylor branch in double precision (u < U_BIG).  INL selects where it is
// compiled: inline in the caller (the power-spectrum kernels, measured
// faster), or out of line (the bispectrum kernel, whose registers the inline
// form would overflow into the accumulation registers).
template <int NL, int LSTEP>
__device__ __forceinline__ Gv<double, NL> G_taylor64_inl(double u) {
  Gv<double, NL> G;
  double v = u * u, ul = 1.0;
  // 14 terms reach 1e-17 relative for u < 2; 32 terms for u < U_BIG.
  const bool few = u < kUSmall;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    if (i > 0) {
#pragma unroll
      for (int q = 0; q < LSTEP; ++q) ul *= u;
    }
    G.v[i] = few ? taylor_G64<14>(i * LSTEP, v, ul) : taylor_G64<HIPSTER_N_TAYLOR>(i * LSTEP, v, ul);
  }
  return G;
}

template <int NL, int LSTEP>
__device__ __noinline__ Gv<double, NL> G_taylor64_call(double u) {
  return G_taylor64_inl<NL, LSTEP>(u);
}

template <int NL, int LSTEP, bool INL>
__device__ inline Gv<double, NL> G_taylor64(double u) {
  if constexpr (INL) return G_taylor64_inl<NL, LSTEP>(u);
  else return G_taylor64_call<NL, LSTEP>(u);
}

// The same below kUSmall only (14 terms), for callers that branch there.
template <int NL, int LSTEP>
__device__ __forceinline__ Gv<double, NL> G_taylor_small_inl(double u) {
  Gv<double, NL> G;
  double v = u * u, ul = 1.0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    if (i > 0) {
#pragma unroll
      for (int q = 0; q < LSTEP; ++q) ul *= u;
    }
    G.v[i] = taylor_G64<14>(i * LSTEP, v, ul);
  }
  return G;
}

template <int NL, int LSTEP>
__device__ __noinline__ Gv<double, NL> G_taylor_small_call(double u) {
  return G_taylor_small_inl<NL, LSTEP>(u);
}

// ----------------------------------------------------------- FP64 form
template <int NL, int LSTEP, bool INL = false>
__device__ __noinline__ Gv<double, NL> G_fp64(double u) {
  if (u < HIPSTER_U_BIG) return G_taylor64<NL, LSTEP, INL>(u);
  Gv<double, NL> G;
  double s, c;
  sincos(u, &s, &c);
  double w = 1.0 / u;
  double t = HIPSTER_U_BIG * w;
  double f = horner64(POLY_F64, t) * w;
  double g = horner64(POLY_G64, t) * w * w;
  double si = kHalfPi - f * c - g * s;
  double w3 = w * w * w;
#pragma unroll
  for (int i = 0; i < NL; ++i) G.v[i] = Dt_closed<double>(i * LSTEP, u, w, s, c, si) * w3;
  return G;
}

// ---------------------------------------------------------- mixed form
// G_l(u) with the phase reduced in double precision, sin and cos from a
// table in double, and the sine integral's auxiliaries in single precision.
// Below kUSmall the Taylor series is summed in double precision.
// sin and cos of u >= 0 from a table of sin, cos at n 2 pi / N (N = 256: the
// generated SINCOS_TAB; N = 64: its every fourth entry), staged in LDS by the
// caller as tab[n] = {sin, cos} (stage_sincos_tab), and short polynomials in
// the remainder x = u - n 2 pi / N, |x| <= pi / N:
//   sin u = S_n cos x + C_n sin x,  cos u = C_n cos x - S_n sin x.
// N = 256: sin x through x^5 (truncation < 1e-17), cos x through x^4 (< 5e-15);
// N = 64: sin x through x^7 (< 5e-18), cos x through x^6 (< 1e-15).  The
// reduction (pi/128 split in 27 + 53 bits, scaled by 256/N) is exact for
// u < 2^26 pi/128 ~ 1.6e6.  n = round(u N / (2 pi)) comes from adding
// 1.5 * 2^52: the fused sum rounds to an integer whose low mantissa bits are
// n, so the table index is read from the low word of the sum.
constexpr int kSinCosTab = 256;
template <int N>
__device__ inline void stage_sincos_tab(double2 *tab) {
  static_assert(N == 256 || N == 64, "table sizes 256 and 64");
  for (int i = threadIdx.x; i < N; i += blockDim.x)
    tab[i] = make_double2(SINCOS_TAB[i * (256 / N)][0], SINCOS_TAB[i * (256 / N)][1]);
}
template <int N = kSinCosTab, bool FULL = false>
__device__ inline void sincos_tab(double u, const double2 *__restrict__ tab, double &s, double &c) {
  constexpr double kScale = 256.0 / N;  // a power of two: the scalings are exact
  constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52
  const double big = fma(u, INV_PIO128 / kScale, kRound);
  const double n = big - kRound;
  double x = fma(-n, PIO128_HI * kScale, u);
  x = fma(-n, PIO128_LO * kScale, x);
  const double2 sc = tab[__double2loint(big) & (N - 1)];
  const double x2 = x * x;
  double sx, cx;
  if constexpr (N == 256 && FULL) {
    // the FP64 form: sin x through x^7, cos x through x^6 (truncation < 1e-20)
    sx = fma(x * x2, fma3(x2, fma3(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), x);
    cx = fma3(x2, fma3(x2, fma3(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  } else if constexpr (N == 256) {
    sx = fma(x * x2, fma3(x2, 1.0 / 120.0, -1.0 / 6.0), x);
    cx = fma3(x2, fma3(x2, 1.0 / 24.0, -0.5), 1.0);
  } else {
    sx = fma(x * x2, fma3(x2, fma3(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), x);
    cx = fma3(x2, fma3(x2, fma3(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  }
  s = fma(sc.x, cx, sc.y * sx);
  c = fma(sc.y, cx, -(sc.x * sx));
}

template <int N>
__device__ inline float horner32(const float (&p)[N], float t) {
  float r = p[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) r = fmaf(r, t, p[k]);
  return r;
}

// Closed form in the mixed form: sin and cos in double precision from the
// table (sincos_tab; NTAB entries staged in LDS by the caller) and the Laurent
// amplitudes a_l, b_l in double -- bin averages difference neighbouring edges,
// and single-precision amplitudes leave per-pair errors of ~5e-7 after that
// differencing.  The form is used
// from u = kUSmall = 2 up: there its worst cancellation (l = 6 at u = 2, a
// factor ~4e5) still leaves ~4e-11 relative error.  Si comes from its power
// series below U_BIG (at most a factor ~40 of cancellation at u = 8) and
// through its auxiliary functions f and g above; f and g are evaluated in
// single precision, since they enter multiplied by c_l / u and need only
// ~1e-8 relative accuracy.  Below u = 2 G_l is summed from its Taylor series.
// wd = 1/u, supplied by the caller (from per-pair 1/r and per-edge 1/k).
template <int NL, int LSTEP, int NTAB = kSinCosTab, bool INL = false>
__device__ inline Gv<double, NL> G_mixed_w(double u, double wd, const double2 *__restrict__ tab) {
  constexpr bool kNeedSi = (NL - 1) * LSTEP >= 2;  // some even l >= 2 is requested
  if (u < kUSmall) {
    if constexpr (INL) return G_taylor_small_inl<NL, LSTEP>(u);
    else return G_taylor_small_call<NL, LSTEP>(u);
  }
  Gv<double, NL> G;
  double s, c;
  sincos_tab<NTAB>(u, tab, s, c);
  double si = 0.0;
  if constexpr (kNeedSi) {
    if (u < HIPSTER_U_BIG) {
      const double v = u * u;
      double p = SI_TAYLOR[HIPSTER_N_SI_TAYLOR - 1];
#pragma unroll
      for (int n = HIPSTER_N_SI_TAYLOR - 2; n >= 0; --n) p = fma3(p, v, SI_TAYLOR[n]);
      si = p * u;
    } else {
      const float w = float(wd);
      const float t = float(HIPSTER_U_BIG) * w;
      const float f = horner32(POLY_F32, t) * w;
      const float g = horner32(POLY_G32, t) * w * w;
      si = kHalfPi - double(f) * c - double(g) * s;
    }
  }
  const double w3 = wd * wd * wd;
#pragma unroll
  for (int i = 0; i < NL; ++i) G.v[i] = Dt_closed<double>(i * LSTEP, u, wd, s, c, si) * w3;
  return G;
}

// Dt_l(u) = u^3 G_l(u) on the large-argument side (u >= U_BIG) in the mixed
// form: sin and cos from the table, the sine-integral auxiliaries f and g in
// single precision as in G_mixed_w (single-precision FMAs issue at twice the
// double rate on this hardware), written in w = 1/u (wd; wf its
// single-precision rounding) rather than t = U_BIG w: f = w P(t) = w P''(w),
// g = w^2 Q(t) = w^2 Q''(w) with P''_k = P_k U_BIG^k, Q''_k = Q_k U_BIG^k
// (exact scalings by powers of two for U_BIG = 8).
// FP64 = true gives the FP64 form of the same path: sin and cos from the table
// with longer remainder polynomials, f and g from their 22-term double
// fits (as G_fp64).  NTAB: entries of the sine/cosine table (256 or 64).
template <int NL, int LSTEP, bool FP64 = false, int NTAB = kSinCosTab>
__device__ inline Gv<double, NL> Dt_far(double u, double wd, const double2 *__restrict__ tab) {
  constexpr bool kNeedSi = (NL - 1) * LSTEP >= 2;
  static_assert(HIPSTER_U_BIG == 8.0, "the coefficient scalings assume U_BIG = 8");
  Gv<double, NL> D;
  double s, c;
  sincos_tab<NTAB, FP64>(u, tab, s, c);
  double si = 0.0;
  if constexpr (kNeedSi && FP64) {
    const double t = HIPSTER_U_BIG * wd;
    const double f = horner64(POLY_F64, t) * wd;
    const double g = horner64(POLY_G64, t) * wd * wd;
    si = kHalfPi - f * c - g * s;
  } else if constexpr (kNeedSi) {
    const float wf = float(wd);
    float pf = POLY_F32[HIPSTER_N_POLY32 - 1] * float(1 << (3 * (HIPSTER_N_POLY32 - 1)));
    float pg = POLY_G32[HIPSTER_N_POLY32 - 1] * float(1 << (3 * (HIPSTER_N_POLY32 - 1)));
#pragma unroll
    for (int k = HIPSTER_N_POLY32 - 2; k >= 0; --k) {
      pf = fmaf(pf, wf, POLY_F32[k] * float(1 << (3 * k)));
      pg = fmaf(pg, wf, POLY_G32[k] * float(1 << (3 * k)));
    }
    const float f = pf * wf, g = pg * wf * wf;
    si = fma(-double(g), s, fma(-double(f), c, kHalfPi));
  }
  // l = 0, 2, 4 rewritten through Dt_0 = s - u c (the same closed forms):
  //   Dt_2 = 3 (Si - s) - Dt_0,  Dt_4 = 7.5 Si + 10 s + Dt_0 - 52.5 w (w s - c)
  const double d0 = fma(-u, c, s);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int l = i * LSTEP;
    if (l == 0) D.v[i] = d0;
    else if (l == 2) D.v[i] = fma(3.0, si - s, -d0);
    else if (l == 4) D.v[i] = fma(-52.5, wd * fma(wd, s, -c), fma(7.5, si, fma(10.0, s, d0)));
    else D.v[i] = Dt_closed<double>(l, u, wd, s, c, si);
  }
  return D;
}

template <int NL, int LSTEP, bool INL = false>
__device__ inline Gv<double, NL> G_mixed(double u, const double2 *__restrict__ tab) {
  // 1/u from the single-precision reciprocal and two Newton steps (~1e-16)
  double wd = double(__builtin_amdgcn_rcpf(float(u)));
  wd = wd * fma(-u, wd, 2.0);
  wd = wd * fma(-u, wd, 2.0);
  return G_mixed_w<NL, LSTEP, kSinCosTab, INL>(u, wd, tab);
}

}  // namespace hipster
